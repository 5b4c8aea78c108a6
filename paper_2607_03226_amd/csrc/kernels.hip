// HIP kernels (gfx950) of the steady BTE transport path.
//
// Storage convention: for every (direction i, cell c, band l) the library
// keeps g = e - C_l theta(c) / W, the part of the energy density that is not
// in equilibrium at the lattice temperature the sweep used (Methods, Eq. (11)
// gives the equilibrium C T_L / W).  Layout g[(i*N + c)*B + l]: the bands of
// one (direction, cell) are contiguous, so the lanes that share a cell read
// and write one contiguous run.  Arithmetic is FP64 everywhere; g is stored in
// FP64 or FP32.
//
// Every per-iteration kernel takes the descriptor array of the solves it
// serves and a work table (one WorkItem per workgroup).  A solve whose state
// says it has stopped is skipped by every kernel, so a captured launch
// sequence can run past the convergence of some of its solves.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/nbte.h"
#include "kernels.h"

namespace nbte {
namespace {

template <class T>
__device__ __forceinline__ double ld(const T *p, int64_t k) {
    return static_cast<double>(p[k]);
}

// theta buffers of a solve under its rotation
__device__ __forceinline__ int th_cur(const SolveState NBTE_G *s) { return (3 - s->rot) % 3; }
// selected without indexing the descriptor copy (a dynamic index would put it in scratch)
__device__ __forceinline__ double NBTE_G *theta_at(const DeviceView &v, int k) {
    return k == 0 ? v.theta[0] : (k == 1 ? v.theta[1] : v.theta[2]);
}
__device__ __forceinline__ const double NBTE_G *theta_cur(const DeviceView &v) { return theta_at(v, th_cur(v.state)); }
__device__ __forceinline__ const double NBTE_G *theta_prev(const DeviceView &v) {
    return theta_at(v, (th_cur(v.state) + 1) % 3);
}
__device__ __forceinline__ double NBTE_G *theta_spare(const DeviceView &v) {
    return theta_at(v, (th_cur(v.state) + 2) % 3);
}

__device__ __forceinline__ double wave_sum(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// Deterministic block sum (fixed tree: lanes, then waves in order).
__device__ double block_sum(double x, double *lds) {
    x = wave_sum(x);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) lds[wv] = x;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < nw; ++k) t += lds[k];
    __syncthreads();
    if (threadIdx.x == 0) lds[0] = t;
    __syncthreads();
    t = lds[0];
    __syncthreads();
    return t;
}

__global__ void k_fill_zero(uint32_t *p, size_t n) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        p[k] = 0u;
}

// --------------------------------------------------------------------------
// stage: lagged boundary inflow (kind 0) and the sweep's equilibrium-imbalance
// term (kind 1)
//
// Boundary inflow of an incoming (face f, direction i), from the previous
// distribution of the owner cell (Methods, boundary conditions):
//   thermalizing  C theta_w / W
//   specular      e of the mirror direction
//   diffuse       sum_out w (s.S) e / sum_in w |s.S|
//   partial       p specular + (1 - p) diffuse
// written straight into the ghost row the sweep reads it from, as the
// deviation from the equilibrium C theta_c / W of the owner cell at the
// theta of the coming sweep (the form the sweep works in).
// --------------------------------------------------------------------------
// One wave per boundary face.  Lanes are (direction group, band) pairs:
// BL = min(B, 64) bands per pass, JG = 64 / BL directions in flight per band,
// so the loads of a pass are independent and the bands of one (direction,
// cell) are read as one contiguous run.  The diffuse sums are reduced across
// the direction groups through LDS in a fixed order.
template <class T>
__device__ void bc_face(const DeviceView &v, int64_t bf, double *red) {
    const int lane = threadIdx.x & 63;
    const int D = v.D, B = v.B;
    const int64_t N = v.N;
    const int c = v.bf_owner[bf];
    const T *g = static_cast<const T *>(v.g);
    T *gv = static_cast<T *>(v.gval);
    const double *sd = v.sdotS + bf * D;
    const int32_t *row = v.in_row + bf * D;
    const double thc = theta_cur(v)[c];   // theta of the coming sweep
    const int BL = B < 64 ? B : 64;
    const int JG = 64 / BL;
    const int jg = lane / BL, ml = lane - jg * BL;
    if (v.bf_kind[bf] == NBTE_BC_THERMALIZING) {
        const double thw = v.bf_thw[bf];
        for (int l0 = 0; l0 < B; l0 += BL) {
            const int lam = l0 + ml;
            if (jg >= JG || lam >= B) continue;
            const T val = static_cast<T>(v.Cw[lam] * thw - v.Cw[lam] * thc);
            for (int i = jg; i < D; i += JG) {
                const int r = row[i];
                if (r >= 0) gv[(int64_t)r * B + lam] = val;
            }
        }
        return;
    }
    const double thp = theta_prev(v)[c];
    const double p = v.bf_p[bf];
    const int32_t *mir = v.mirror + bf * D;
    for (int l0 = 0; l0 < B; l0 += BL) {
        const int lam = l0 + ml;
        const bool on = jg < JG && lam < B;
        const int lam_c = on ? lam : 0;
        const double cw = v.Cw[lam_c];
        const double eq = cw * thp;
        const double eqc = cw * thc;
        double diff = 0.0;
        if (p < 1.0) {
            double acc = 0.0;
            if (on) {
#pragma unroll 4
                for (int j = jg; j < D; j += JG) {
                    const double a = sd[j];
                    const double e = ld(g, ((int64_t)j * N + c) * B + lam_c) + eq;
                    acc += a > 0.0 ? v.w[j] * a * e : 0.0;
                }
            }
            red[lane] = acc;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
            for (int k = 0; k < JG; ++k) diff += red[k * BL + ml];
            diff /= v.win[bf];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
        }
        if (!on) continue;
        if (p > 0.0) {
#pragma unroll 4
            for (int i = jg; i < D; i += JG) {
                const int r = row[i];
                const int mi = mir[i] >= 0 ? mir[i] : 0;   // outgoing directions have no mirror entry
                const double em = ld(g, ((int64_t)mi * N + c) * B + lam) + eq;
                if (r >= 0) gv[(int64_t)r * B + lam] = static_cast<T>((1.0 - p) * diff + p * em - eqc);
            }
        } else {
            for (int i = jg; i < D; i += JG) {
                const int r = row[i];
                if (r >= 0) gv[(int64_t)r * B + lam] = static_cast<T>(diff - eqc);
            }
        }
    }
}

template <class T>
__global__ void __launch_bounds__(256) k_stage(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk) {
    __shared__ double red[256];
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (v.state->done) return;
    const int64_t stride = (int64_t)it.c * blockDim.x;
    const int64_t t0 = (int64_t)it.b * blockDim.x + threadIdx.x;
    if (it.a == 0) {
        // faces b*4 + wave, b*4 + wave + 4*nblk, ...
        const int wv = threadIdx.x >> 6;
        for (int64_t bf = (int64_t)it.b * 4 + wv; bf < v.NBF; bf += (int64_t)it.c * 4)
            bc_face<T>(v, bf, red + 64 * wv);
    } else {
        // D = sum_j |a_j| (theta_up_j - theta_c): the closed cell's
        // sum_{a<0} |a| - sum_{a>0} a vanishes (divergence theorem, to the
        // rounding of the face vectors), so D needs no outflow term and is
        // exactly zero for a uniform theta.  The differences are taken in
        // FP64, then weighted by the sweep's coefficients.
        const int64_t n = (int64_t)v.D * v.N;
        const int MI = v.maxin;
        const double *th = theta_cur(v);
        const T *cf = static_cast<const T *>(v.t_coef);
        T *dc = static_cast<T *>(v.t_dc);
        for (int64_t t = t0; t < n; t += stride) {
            const double thc = th[v.p_cell[t]];
            double acc = 0.0;
            for (int j = 0; j < MI; ++j) acc += static_cast<double>(cf[j * n + t]) * (th[v.p_upc[j * n + t]] - thc);
            dc[t] = static_cast<T>(acc);
        }
    }
}

// --------------------------------------------------------------------------
// transport sweep: one workgroup per (band block, direction)
//
// For cell c of direction i, in upwind level order (Methods, Eqs. (4), (13)):
//   e_c = (e0_l/tau_l + S_l + v_l sum_{a<0} |a| e_up) / (1/tau_l + v_l sum_{a>0} a),
//   a = (s_i . S_cf) / V_c,
// e_up = value of the upwind neighbour computed earlier in this sweep, or the
// boundary inflow (computed in the deviation form g below).  Everything a
// cell needs comes from the direction's level-ordered streams (cell,
// coefficients, upwind references, imbalance term D, Qdot): independent
// coalesced loads, no pointer chasing.  Upwind values are staged in LDS (in
// the storage type) in host-assigned slots; a value without a slot is read
// back from its stored copy.  A workgroup barrier separates levels; it orders
// the LDS and HBM writes of level k before the reads of level k+1.
//
// Workgroup -> (solve, direction, band block) through the work table; the
// host orders it so that the band blocks of one direction land on the same
// XCD (dispatch goes round-robin over the 8 XCDs) and share that direction's
// streams in one L2.
// --------------------------------------------------------------------------
// Dynamic LDS of the sweep.  It is indexed with integer offsets (never through
// pointers passed around), so every access stays in the LDS address space.
extern __shared__ double sweep_lds[];
extern __shared__ int sweep_ldsi[];   // the same memory viewed as ints (level tables)
extern __shared__ float sweep_ldsf[];  // ... and as floats (FP32 staged values)

constexpr int kGhostPerThread = 2;    // ghost values a thread prefetches per level
constexpr int kPrefetch = 4;          // passes whose records are in flight ahead of the computed one
// record references: >= 0 LDS element offset (staged value or ghost kept in
// LDS); [-kSpill, -1] ghost read from HBM (row -1 - ref); below: the stored
// copy of a spilled value at stream position -(kSpill + 1) - ref
constexpr int32_t kSpill = 1 << 24;

// The sweep works in the deviation from local equilibrium,
//   g_c = e_c - C_l theta_c / W,
// which turns the upwind update into
//   g_c = (Q_c S_l + v_l (sum_j |a_j| g_up_j + (C_l/W) D_c)) / (1/tau_l + v_l sum_{a>0} a),
//   D_c = sum_j |a_j| theta_up_j - (sum_{a>0} a) theta_c = sum_j |a_j| (theta_up_j - theta_c)
// (g_up of a boundary inflow is taken against theta_c; the second form of D
// uses sum_{a<0} |a| = sum_{a>0} a of a closed cell).  g is small wherever
// theta is smooth, so the FP32 form of the mixed path rounds relative to the
// deviation, not to e; the FP64 path runs the same form in FP64.

// element k of a global array through a 32-bit byte offset from a uniform
// base (one VGPR offset shared by every stream; the address is formed by the
// load itself)
template <class T>
__device__ __forceinline__ T gload(const T NBTE_G *base, uint32_t k) {
    return *reinterpret_cast<const T NBTE_G *>(reinterpret_cast<const char NBTE_G *>(base) + k * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void gstore(T NBTE_G *base, uint32_t k, T x) {
    *reinterpret_cast<T NBTE_G *>(reinterpret_cast<char NBTE_G *>(base) + k * (uint32_t)sizeof(T)) = x;
}

// One cell's sweep record (a position of a direction's level-ordered streams).
template <class T, int MI>
struct SweepRec {
    int c, mine;
    int ref[MI];
    T cf[MI];
    T sout, dc, q;
    bool ok;
};

template <class T, int MI>
__device__ __forceinline__ void load_rec(SweepRec<T, MI> &r, const DeviceView &v, int64_t base, int64_t DN, int k,
                                         int kend) {
    // the loads are issued on every path (a past-the-end record reads stream
    // position 0 of the direction), so the number of loads in flight is the
    // same on every path and a later wait on an older record can leave the
    // younger prefetches outstanding.  Stream positions fit 32 bits.
    r.ok = k < kend;
    const uint32_t at = (uint32_t)(base + (r.ok ? k : 0));
    const uint32_t dn = (uint32_t)DN;
    const T NBTE_G *coef = static_cast<const T NBTE_G *>(v.t_coef);
    r.c = gload(v.p_cell, at);
    r.mine = gload(v.p_slot, at);
    r.sout = gload(static_cast<const T NBTE_G *>(v.t_sout), at);
    r.dc = gload(static_cast<const T NBTE_G *>(v.t_dc), at);
    r.q = gload(static_cast<const T NBTE_G *>(v.t_q), at);
#pragma unroll
    for (int j = 0; j < MI; ++j) {
        r.ref[j] = gload(v.p_ref + j * dn, at);
        r.cf[j] = gload(coef + j * dn, at);
    }
}

// Per-lane band constants, loaded once per workgroup: inside the level loop
// the sweep never waits on a load issued in the same level, because a wait on
// any load also waits for every older one (the vector memory counter is in
// order), which would drain the prefetched records.
template <class T, int BPL>
struct BandConst {
    T cw[BPL], itau[BPL], vel[BPL], src[BPL];
};

// LDS views of the staged values: element k of the sweep's type
template <class T>
__device__ __forceinline__ T lds_get(int k);
template <>
__device__ __forceinline__ double lds_get<double>(int k) { return sweep_lds[k]; }
template <>
__device__ __forceinline__ float lds_get<float>(int k) { return sweep_ldsf[k]; }
template <class T>
__device__ __forceinline__ void lds_put(int k, T x);
template <>
__device__ __forceinline__ void lds_put<double>(int k, double x) { sweep_lds[k] = x; }
template <>
__device__ __forceinline__ void lds_put<float>(int k, float x) { sweep_ldsf[k] = x; }

// the update's quotient: IEEE division in FP64, reciprocal (1 ulp) in FP32
__device__ __forceinline__ double quot(double a, double b) { return a / b; }
__device__ __forceinline__ float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

template <class T, int MI, int BPL>
__device__ __forceinline__ void sweep_cell(const SweepRec<T, MI> &r, const DeviceView &v, const BandConst<T, BPL> &bc,
                                           T NBTE_G *gi, int64_t base, int b0, int lane, int nb_here) {
    const int B = v.B;
    const T NBTE_G *gval = static_cast<const T NBTE_G *>(v.gval);
#pragma unroll
    for (int jb = 0; jb < BPL; ++jb) {
        const int lb = lane * BPL + jb;
        if (lb >= nb_here) break;
        const int lam = b0 + lb;
        T gain = 0;
#pragma unroll
        for (int j = 0; j < MI; ++j) {
            if (r.cf[j] == T(0)) continue;
            const int rf = r.ref[j];
            T up;
            if (rf >= 0) {
                up = lds_get<T>(rf + lb);   // staged value or ghost kept in LDS
            } else if (rf >= -kSpill) {
                up = gval[(int64_t)(-1 - rf) * B + lam];   // ghost beyond the LDS capacity
            } else {
                // value without an LDS slot: its stored copy, located through
                // the neighbour's position in this direction's streams
                const int n = v.p_cell[base + (-(kSpill + 1) - rf)];
                up = gi[(int64_t)n * B + lam];
            }
            gain += r.cf[j] * up;
        }
        const T vel = bc.vel[jb];
        const T g = quot(r.q * bc.src[jb] + vel * (gain + bc.cw[jb] * r.dc), bc.itau[jb] + vel * r.sout);
        gi[(int64_t)r.c * B + lam] = g;
        if (r.mine >= 0) lds_put<T>(r.mine + lb, g);
    }
}

// The common case: every upwind reference is an LDS slot or a ghost kept in
// LDS (no spilled values, no ghost beyond the LDS capacity).  Branch-free:
// one LDS offset per reference shared by the bands, unused references
// (coefficient 0) masked by a select, past-the-end records computed but not
// stored, so the items of a thread interleave.
template <class T, int MI, int BPL>
__device__ __forceinline__ void sweep_cell_lds(const SweepRec<T, MI> &r, const BandConst<T, BPL> &bc, T NBTE_G *gi,
                                               int B, int ls, int b0, int lane, int nb_here) {
    const uint32_t gc = (uint32_t)r.c * (uint32_t)B + (uint32_t)b0;   // within one direction's slice
#pragma unroll
    for (int jb = 0; jb < BPL; ++jb) {
        const int lb = lane * BPL + jb;
        const bool on = r.ok && lb < nb_here;
        const int lr = lb < ls ? lb : ls - 1;   // lanes past the block read in range
        T gain = 0;
#pragma unroll
        for (int j = 0; j < MI; ++j) {
            const T up = lds_get<T>(r.ref[j] + lr);
            gain += r.cf[j] != T(0) ? r.cf[j] * up : T(0);
        }
        const T vel = bc.vel[jb];
        const T g = quot(r.q * bc.src[jb] + vel * (gain + bc.cw[jb] * r.dc), bc.itau[jb] + vel * r.sout);
        if (on) {
            gstore(gi, gc + lb, g);
            if (r.mine >= 0) lds_put<T>(r.mine + lb, g);
        }
    }
}

// Level barrier.  Without spilled values nothing written to HBM during the
// sweep is read back by it, so the barrier only has to order LDS; the fences
// are restricted to the LDS address space.  With spilled values the full
// workgroup fence also orders the global stores.
// sweep kernel modes: references only in LDS; LDS plus ghosts read from HBM;
// plus spilled values (stored copies read back, so the level barrier orders
// global memory too)
enum SweepMode { kModeLds = 0, kModeHbmGhost = 1, kModeSpill = 2 };

template <bool SPILL>
__device__ __forceinline__ void level_barrier() {
    if constexpr (SPILL) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
}

// --------------------------------------------------------------------------
// Pipeline: the cells of a direction are processed in passes (up to one
// cell per slot, all of one level).  While pass q is computed from registers
// (records requested kPrefetch passes earlier), the LDS ring (upwind values)
// and the level's ghost buffer, the records of pass q + kPrefetch are
// requested.  Every wait is on loads issued at least kPrefetch passes
// earlier; past-the-end requests read valid positions so the number of loads
// in flight is the same on every path.  The step ring is unrolled so a record
// keeps its registers while its loads are in flight (moving it would force
// the wait).
// --------------------------------------------------------------------------
template <class T, int MI, int BPL, int MODE, bool ONE>
__global__ void __launch_bounds__(512) k_sweep(const DeviceView *__restrict__ vs,
                                                const WorkItem *__restrict__ wk) {
    // ONE: one lane per cell (it sweeps all BPL bands of the block), so the
    // band of a register is the same on every lane and the band constants are
    // workgroup-uniform (scalar loads, scalar registers)
    // dynamic LDS: [lvl_ptr | gptr of this direction: 2 (max_levels + 1) ints]
    //              [ghost buffers: 2 x gcap x ls doubles]
    //              [ring: slot x ls doubles]
    // ls = LDS stride of one staged value's bands
    const WorkItem tk = wk[blockIdx.x];
    if (tk.solve < 0) return;   // padding of the XCD-ordered work list
    const DeviceView v = vs[tk.solve];   // a copy: fields stay in registers across the stores
    if (v.state->done) return;
    const int lpc = v.lpc;
    const int bands_per_block = v.bpb;
    const int gcap = v.gcap;
    const int i = tk.a;
    const int b0 = tk.b * bands_per_block;
    const int slot = ONE ? (int)threadIdx.x : (int)threadIdx.x / lpc;
    const int lane = ONE ? 0 : (int)threadIdx.x % lpc;
    const int nslots = ONE ? (int)blockDim.x : (int)blockDim.x / lpc;
    const int64_t N = v.N;
    const int B = v.B;
    const int64_t DN = (int64_t)v.D * N;
    T NBTE_G *gi = static_cast<T NBTE_G *>(v.g) + (int64_t)i * N * B;
    const int64_t base = (int64_t)i * N;
    const int nlev = v.lvl_off[i + 1] - v.lvl_off[i] - 1;
    const int nb_here = min(B, b0 + bands_per_block) - b0;
    const int ML = v.max_levels + 1;
#define lp(t) sweep_ldsi[(t)]
#define gp(t) sweep_ldsi[ML + (t)]
    const SweepLdsLayout lay = sweep_lds_layout(v.max_levels, gcap, v.lstride, (int)sizeof(T));
    const int ls = lay.ls;
    const int gbuf0 = lay.gbuf0;       // first element after the level tables
    const int gstride = lay.gstride;   // ghosts of a level kept in LDS (rank < gcap)
    {
        const int32_t *glp = v.lvl_ptr + v.lvl_off[i];
        const int32_t *ggp = v.gptr + v.lvl_off[i];
#pragma nounroll
        for (int t = threadIdx.x; t <= nlev; t += blockDim.x) {
            lp(t) = glp[t];
            gp(t) = ggp[t];
        }
    }
    BandConst<T, BPL> bc;
#pragma unroll
    for (int jb = 0; jb < BPL; ++jb) {
        const int lam = min(b0 + lane * BPL + jb, B - 1);
        bc.cw[jb] = static_cast<T>(v.Cw[lam]);
        bc.itau[jb] = static_cast<T>(v.inv_tau[lam]);
        bc.vel[jb] = static_cast<T>(v.vel[lam]);
        bc.src[jb] = static_cast<T>(v.src[lam]);
    }
    const T NBTE_G *gval = static_cast<const T NBTE_G *>(v.gval);
    __syncthreads();

    // The sweep of a direction as a sequence of passes: pass = up to nslots
    // cells of one level, one cell per slot.  Records are requested
    // kPrefetch passes ahead into a ring of kPrefetch + 1 register sets, so
    // wide levels (many passes) and narrow ones (one pass each) hide the
    // load latency alike.  A barrier ends each level.  Ghost values (boundary
    // inflow) of a level ride with the records of its first pass and are
    // stored into the level's LDS buffer just before the level starts.
    struct Ghosts {
        T v[kGhostPerThread];
    };
    struct Set {
        SweepRec<T, MI> r;
        Ghosts h;
    };
    auto ghost_load = [&](Ghosts &h, int l, bool first) {
        // branch-free like load_rec: entries past the level read element 0
        const int ll = l < nlev ? l : nlev - 1;
        const int g0 = gp(ll), ne = (first && l < nlev) ? min(gp(ll + 1) - g0, gcap) * bands_per_block : 0;
#pragma unroll
        for (int m = 0; m < kGhostPerThread; ++m) {
            const int e = threadIdx.x + m * blockDim.x;
            const int q = e / bands_per_block, lb = e - q * bands_per_block;
            const bool ok = e < ne && lb < nb_here;
            const T x = gload(gval, ok ? (uint32_t)((g0 + q) * B + b0 + lb) : 0u);
            h.v[m] = ok ? x : T(0);
        }
    };
    auto ghost_store = [&](const Ghosts &h, int l) {
        const int dst = gbuf0 + (l & 1) * gstride;
        const int g0 = gp(l), ne = min(gp(l + 1) - g0, gcap) * bands_per_block;
#pragma unroll
        for (int m = 0; m < kGhostPerThread; ++m) {
            const int e = threadIdx.x + m * blockDim.x;
            const int q = e / bands_per_block, lb = e - q * bands_per_block;
            if (e < ne) lds_put<T>(dst + q * ls + lb, h.v[m]);
        }
        // levels with more ghosts than the registers hold: direct copy
#pragma nounroll
        for (int e = threadIdx.x + kGhostPerThread * blockDim.x; e < ne; e += blockDim.x) {
            const int q = e / bands_per_block, lb = e - q * bands_per_block;
            lds_put<T>(dst + q * ls + lb, lb < nb_here ? gval[(int64_t)(g0 + q) * B + b0 + lb] : T(0));
        }
    };
    // pass cursors (uniform): level and first position of the pass
    int lf = 0, kf = lp(0);   // next pass to request
    int lc = 0, kc = lp(0);   // next pass to compute
    auto fetch = [&](Set &st) {
        const bool live = lf < nlev;
        const int kend = live ? lp(lf + 1) : 0;
        load_rec(st.r, v, base, DN, kf + slot, kend);
        ghost_load(st.h, lf, live && kf == lp(lf));
        if (live) {
            kf += nslots;
            if (kf >= kend) {
                ++lf;
                kf = lp(lf);
            }
        }
    };
    // compute the pass in `cur`, request a new pass into `nxt` (the set
    // computed last, now free); returns false when the sweep is done
    auto step = [&](Set &cur, Set &nxt, const Set &after) -> bool {
        fetch(nxt);
        if constexpr (MODE == kModeLds)
            sweep_cell_lds<T, MI, BPL>(cur.r, bc, gi, B, ls, b0, lane, nb_here);
        else if (cur.r.ok)
            sweep_cell<T, MI, BPL>(cur.r, v, bc, gi, base, b0, lane, nb_here);
        kc += nslots;
        if (kc >= lp(lc + 1)) {   // level done
            ++lc;
            if (lc < nlev) {
                kc = lp(lc);
                ghost_store(after.h, lc);   // the next pass opens level lc
            }
            level_barrier<MODE == kModeSpill>();
        }
        return lc < nlev;
    };
    Set s0, s1, s2, s3, s4;
    static_assert(kPrefetch == 4, "the step ring below is written for four passes in flight");
    fetch(s0);
    fetch(s1);
    fetch(s2);
    fetch(s3);
    ghost_store(s0.h, 0);
    __syncthreads();
#pragma nounroll
    while (true) {
        if (!step(s0, s4, s1)) break;
        if (!step(s1, s0, s2)) break;
        if (!step(s2, s1, s3)) break;
        if (!step(s3, s2, s4)) break;
        if (!step(s4, s3, s0)) break;
    }
}
#undef lp
#undef gp

// --------------------------------------------------------------------------
// net heat flow through each boundary face: one wave per face
//   J_f = sum_l v_l sum_i w_i (s_i . S_f) e
// with e the owner's value for outgoing and the inflow for incoming directions
// --------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) k_flux(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk,
                                              int after) {
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (!after && v.state->done) return;
    const int64_t bf = (int64_t)it.b * 4 + (threadIdx.x >> 6);
    if (bf >= v.NBF) return;
    // inside the iteration only reflective walls' flows are used (the
    // correction's right-hand side); thermalizing ones matter for the energy
    // balance read at the end
    if (!after && v.bf_kind[bf] == NBTE_BC_THERMALIZING) return;
    const int lane = threadIdx.x & 63;
    const int D = v.D, B = v.B;
    const int64_t N = v.N;
    const int c = v.bf_owner[bf];
    const double th = (after ? theta_prev(v) : theta_cur(v))[c];
    const T *g = static_cast<const T *>(v.g);
    const T *gv = static_cast<const T *>(v.gval);
    double acc = 0.0;
    // both candidate values are loaded on every path (independent loads, four
    // pairs in flight); directions with s.S = 0 contribute exactly zero
#pragma unroll 4
    for (int t = lane; t < D * B; t += 64) {
        const int i = t / B, lam = t - i * B;
        const double sd = v.sdotS[bf * D + i];
        const int32_t row = v.in_row[bf * D + i];
        const double ein = ld(gv, row >= 0 ? (int64_t)row * B + lam : 0) + v.Cw[lam] * th;
        const double eout = ld(g, ((int64_t)i * N + c) * B + lam) + v.Cw[lam] * th;
        const double e = row >= 0 ? ein : (sd > 0.0 ? eout : 0.0);
        acc += v.vel[lam] * v.w[i] * sd * e;
    }
    acc = wave_sum(acc);
    if (lane == 0) v.Jw[bf] = acc;
}

// --------------------------------------------------------------------------
// band x direction reductions (Methods, Eqs. (5), (7); T = energy temperature)
// mom_lpc lanes per cell (bands x direction groups), FP64 accumulation,
// shuffle reduction over the lanes in a fixed order.
// Synthetic schemes also get the V-weighted right-hand side of the correction:
//   V (Qdot - D_h' q) = V beta (theta_seq - theta) + sum_{reflective f} J_f
// (collision-divergence identity; reflective walls carry zero net flux at the
// fixed point, so their transient flux is returned to the cell).
// --------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) k_moments(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk) {
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (v.state->done) return;
    // lanes of a cell: lb band lanes x (lpc / lb) direction groups
    const int lpc = v.mom_lpc;
    const int64_t N = v.N;
    const int B = v.B, D = v.D;
    int lb = 1;
    while (lb < B && lb < 64) lb <<= 1;
    const int64_t c = ((int64_t)it.b * blockDim.x + threadIdx.x) / lpc;
    const int lane = threadIdx.x % lpc;
    const int bl = lane % lb, dg = lane / lb, ng = lpc / lb;
    const T *g = static_cast<const T *>(v.g);
    double a_tau = 0, a_w = 0, qx = 0, qy = 0, qz = 0;
    if (c < N) {
        for (int lam = bl; lam < B; lam += lb) {
            double sw = 0, s_x = 0, s_y = 0, s_z = 0;
            // independent loads, eight directions of the group in flight
#pragma unroll 8
            for (int i = dg; i < D; i += ng) {
                const double ww = v.w[i] * ld(g, ((int64_t)i * N + c) * B + lam);
                sw += ww;
                s_x += ww * v.dirs[3 * i];
                s_y += ww * v.dirs[3 * i + 1];
                s_z += ww * v.dirs[3 * i + 2];
            }
            a_tau += sw * v.inv_tau[lam];
            a_w += sw;
            const double vel = v.vel[lam];
            qx += vel * s_x;
            qy += vel * s_y;
            qz += vel * s_z;
        }
    }
    for (int off = lpc >> 1; off > 0; off >>= 1) {
        a_tau += __shfl_xor(a_tau, off);
        a_w += __shfl_xor(a_w, off);
        qx += __shfl_xor(qx, off);
        qy += __shfl_xor(qy, off);
        qz += __shfl_xor(qz, off);
    }
    if (c < N && lane == 0) {
        const double th = theta_cur(v)[c];
        v.theta_seq[c] = th + a_tau / v.beta;
        v.thetaE[c] = th + a_w / v.C_tot;
        v.q[3 * c] = qx + th * v.qbias[0];
        v.q[3 * c + 1] = qy + th * v.qbias[1];
        v.q[3 * c + 2] = qz + th * v.qbias[2];
        if (v.scheme != NBTE_SCHEME_SEQUENTIAL) {
            double r = v.V[c] * a_tau;
            for (int f = 0; f < v.F; ++f) {
                const int n = v.nbr[c * v.F + f];
                if (n < 0 && v.bf_kind[-n - 1] != NBTE_BC_THERMALIZING) r += v.Jw[-n - 1];
            }
            v.rhs[c] = r;
        }
    }
}

__device__ __forceinline__ unsigned long long dbits(double x) {
    return static_cast<unsigned long long>(__double_as_longlong(x));
}

// theta_new = base + delta: sequential base = theta_seq (Eq. (5)); synthetic
// base = theta_seq + correction (Eq. (12)); the literal variant adds the
// correction to the previous theta.  Residual maxima into the solve's state.
__global__ void __launch_bounds__(256) k_update(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk) {
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (v.state->done) return;
    const double *th = theta_cur(v);
    double *tn_out = theta_spare(v);
    const double *base = v.scheme == NBTE_SCHEME_SYNTHETIC_LITERAL ? th : v.theta_seq;
    const double *delta = v.scheme == NBTE_SCHEME_SEQUENTIAL ? nullptr : v.delta;
    double md = 0.0, mt = 0.0;
    for (int64_t c = (int64_t)it.b * blockDim.x + threadIdx.x; c < v.N; c += (int64_t)it.c * blockDim.x) {
        const double tn = base[c] + (delta ? delta[c] : 0.0);
        tn_out[c] = tn;
        const double d = fabs(tn - th[c]);
        if (!(d <= 1e300)) md = INFINITY;   // NaN or overflow: report as divergence
        else md = fmax(md, d);
        mt = fmax(mt, fabs(tn));
    }
    for (int off = 32; off > 0; off >>= 1) {
        md = fmax(md, __shfl_xor(md, off));
        mt = fmax(mt, __shfl_xor(mt, off));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&v.state->maxbuf[0], dbits(md));
        atomicMax(&v.state->maxbuf[1], dbits(mt));
    }
}

// End of an iteration: residual, stop test, theta rotation (one thread per solve).
__global__ void k_finish(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    SolveState *s = vs[wk[k].solve].state;
    if (s->done) return;
    const double md = __longlong_as_double((long long)s->maxbuf[0]);
    const double mt = __longlong_as_double((long long)s->maxbuf[1]);
    const double res = mt > 0.0 ? md / mt : 0.0;
    s->residual = res;
    s->maxbuf[0] = 0ull;
    s->maxbuf[1] = 0ull;
    s->iterations += 1;
    s->rot = (s->rot + 1) % 3;
    if (res < 0.98 * s->best) {
        s->best = res;
        s->since = 0;
    } else {
        s->since += 1;
    }
    if (!(res <= 1e300)) s->done = NBTE_DONE_DIVERGED;
    else if (s->stop && res <= s->tol) s->done = NBTE_DONE_CONVERGED;
    else if (s->stop && s->iterations >= s->max_iter) s->done = NBTE_DONE_MAX_ITER;
    else if (s->stop && s->patience > 0 && s->since >= s->patience) s->done = NBTE_DONE_STALLED;
}

__global__ void k_set_controls(SolveState *s, int stop, double tol, int max_iter, int patience) {
    if (threadIdx.x == 0) {
        s->done = 0;
        s->stop = stop;
        s->tol = tol;
        s->max_iter = max_iter;
        s->patience = patience;
        s->best = INFINITY;
        s->since = 0;
    }
}

// FP32 distribution -> FP64 (switch of a solve to FP64 sweeps)
__global__ void k_widen(int64_t n, const float *in, double *out) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = static_cast<double>(in[k]);
}

__global__ void k_collect_states(const DeviceView *__restrict__ vs, int n, SolveState *out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = *vs[k].state;
}

__global__ void k_affine(int64_t n, const double *in, double scale, double offset, double *out) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) out[k] = offset + scale * in[k];
}

template <class T>
__global__ void k_gather(int64_t n, const int32_t *idx, const double *in, T *out) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) out[k] = static_cast<T>(in[idx[k]]);
}

// e of the last sweep: stored g relative to the theta that sweep used (prev)
template <class T>
__global__ void k_distribution(const DeviceView *__restrict__ vp, int band, int dir, double *out) {
    const DeviceView &v = *vp;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= v.N) return;
    const T *g = static_cast<const T *>(v.g);
    out[c] = ld(g, ((int64_t)dir * v.N + c) * v.B + band) + v.Cw[band] * theta_prev(v)[c];
}

// --------------------------------------------------------------------------
// Jacobi PCG of the synthetic correction (symmetric positive definite L).
// mode 0: L delta = rhs inside the iteration; mode 1: L theta[cur] = rhs
// (initial guess).  rtol2_o / max_o >= 0 override the solve's settings.
// --------------------------------------------------------------------------
__device__ __forceinline__ bool pcg_skip(const DeviceView &v, int mode) { return mode == 0 && v.state->done; }
__device__ __forceinline__ double *pcg_x(const DeviceView &v, int mode) {
    return mode == 0 ? v.delta : theta_at(v, th_cur(v.state));
}

// Whole PCG in one workgroup (small systems): no launch per iteration, the
// reductions are workgroup reductions in a fixed order (deterministic).
// Every thread owns rows tid, tid + blockDim, ...; only the SpMV reads other
// threads' entries of p, and p is complete at the barrier before it.
__global__ void __launch_bounds__(1024) k_pcg_block(const DeviceView *__restrict__ vs,
                                                    const WorkItem *__restrict__ wk, int mode, double rtol2_o,
                                                    int max_o) {
    __shared__ double lds[16];
    const DeviceView &v = vs[wk[blockIdx.x].solve];
    if (pcg_skip(v, mode)) return;
    const PcgWork &w = v.pcg;
    const double *b = v.rhs;
    double *x = pcg_x(v, mode);
    const double rtol2 = rtol2_o >= 0 ? rtol2_o : w.rtol2;
    const int max_iter = max_o >= 0 ? max_o : w.max_iter;
    const int64_t n = w.n;
    const int nt = blockDim.x;
    double *wr = w.vec, *wz = w.vec + n, *wp = w.vec + 2 * n, *wAp = w.vec + 3 * n;
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += nt) {
        const double bi = b[r];
        x[r] = 0.0;
        wr[r] = bi;
        const double zi = w.dinv[r] * bi;
        wz[r] = zi;
        wp[r] = zi;
        acc += bi * zi;
    }
    double rz = block_sum(acc, lds);
    const double rz0 = rz;
    int it = 0;
    if (rz > 0.0) {
        for (; it < max_iter; ++it) {
            acc = 0.0;
            for (int64_t r = threadIdx.x; r < n; r += nt) {
                double ap = 0.0;
                for (int32_t k = w.row_ptr[r]; k < w.row_ptr[r + 1]; ++k) ap += w.val[k] * wp[w.col[k]];
                wAp[r] = ap;
                acc += wp[r] * ap;
            }
            const double alpha = rz / block_sum(acc, lds);
            acc = 0.0;
            for (int64_t r = threadIdx.x; r < n; r += nt) {
                x[r] += alpha * wp[r];
                const double rn = wr[r] - alpha * wAp[r];
                wr[r] = rn;
                const double zn = w.dinv[r] * rn;
                wz[r] = zn;
                acc += rn * zn;
            }
            const double rz_new = block_sum(acc, lds);
            if (!(rz_new > rtol2 * rz0)) { ++it; break; }
            const double beta = rz_new / rz;
            rz = rz_new;
            for (int64_t r = threadIdx.x; r < n; r += nt) wp[r] = wz[r] + beta * wp[r];
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        w.scal[1] = rz0;
        w.scal[5] = it;
    }
}

// Multi-workgroup form: conjugate gradients with a single reduction per
// iteration (the Chronopoulos-Gear arrangement of preconditioned CG: the two
// inner products (r, u) and (w, u) of u = M^-1 r, w = A u are taken together),
// one launch per iteration.  With gamma_k = (r_k, u_k), delta_k = (w_k, u_k):
//   beta_k = gamma_k / gamma_{k-1},  alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1})
//   p_k = u_k + beta_k p_{k-1},  s_k = w_k + beta_k s_{k-1}  (s = A p)
//   x += alpha_k p_k,  r_{k+1} = r_k - alpha_k s_k,  u_{k+1} = M^-1 r_{k+1},  w_{k+1} = A u_{k+1}
// (beta_0 = 0, alpha_0 = gamma_0 / delta_0).  A row's SpMV needs u_{k+1} of its
// neighbours, recomputed from their old r, w, s (kept in the other buffer of
// each pair), so no grid-wide synchronisation is needed inside a launch.
// Every workgroup of a solve re-sums that solve's partials in the same order:
// all see identical scalars and the result is bitwise reproducible.  The
// iteration stops (for every later launch too, through a sticky flag) once
// gamma_k <= rtol2 gamma_0.
__device__ double sum_partials(const double *p, int n, double *lds) {
    double x = (threadIdx.x < (unsigned)n) ? p[threadIdx.x] : 0.0;
    return block_sum(x, lds);
}

__global__ void __launch_bounds__(256) k_cg1_init(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk,
                                                  int mode) {
    __shared__ double lds[16];
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (pcg_skip(v, mode)) return;
    const PcgWork &w = v.pcg;
    const int64_t n = w.n;
    const double *b = v.rhs;
    double *x = pcg_x(v, mode);
    double *r0 = w.vec, *w0 = w.vec + 2 * n, *s1 = w.vec + 5 * n, *pp = w.vec + 6 * n;
    double ga = 0.0, de = 0.0;
    for (int64_t r = (int64_t)it.b * blockDim.x + threadIdx.x; r < n; r += (int64_t)w.nblk * blockDim.x) {
        const double bi = b[r];
        const double u = w.dinv[r] * bi;
        double au = 0.0;
        for (int32_t k = w.row_ptr[r]; k < w.row_ptr[r + 1]; ++k) {
            const int32_t j = w.col[k];
            au += w.val[k] * (w.dinv[j] * b[j]);
        }
        x[r] = 0.0;
        r0[r] = bi;
        w0[r] = au;
        s1[r] = 0.0;
        pp[r] = 0.0;
        ga += bi * u;
        de += au * u;
    }
    ga = block_sum(ga, lds);
    de = block_sum(de, lds);
    if (threadIdx.x == 0) {
        w.partial[it.b] = ga;
        w.partial[w.nblk + it.b] = de;
        if (it.b == 0) {
            w.scal[4] = 0.0;
            w.scal[5] = 0.0;
        }
    }
}

__global__ void __launch_bounds__(256) k_cg1_iter(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk,
                                                  int mode, int k, double rtol2_o, int max_o) {
    __shared__ double lds[16];
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (pcg_skip(v, mode)) return;
    const PcgWork &w = v.pcg;
    const int max_iter = max_o >= 0 ? max_o : w.max_iter;
    if (k >= max_iter) return;
    // the flag is read once per workgroup and broadcast through LDS, so every
    // thread takes the same (uniform) exit
    __syncthreads();
    if (threadIdx.x == 0) lds[15] = w.scal[4];
    __syncthreads();
    if (lds[15] != 0.0) return;
    __syncthreads();
    const double rtol2 = rtol2_o >= 0 ? rtol2_o : w.rtol2;
    const int64_t n = w.n;
    const int cur = k & 1, nxt = cur ^ 1;
    const double *pin = w.partial + cur * 2 * w.nblk;
    double *pout = w.partial + nxt * 2 * w.nblk;
    const double gamma = sum_partials(pin, w.nblk, lds);
    const double delta = sum_partials(pin + w.nblk, w.nblk, lds);
    const double gamma0 = k == 0 ? gamma : w.scal[1];
    if (!(gamma > rtol2 * gamma0)) {   // converged (or zero right-hand side)
        if (it.b == 0 && threadIdx.x == 0) w.scal[4] = 1.0;
        return;
    }
    double alpha, beta;
    if (k == 0) {
        beta = 0.0;
        alpha = gamma / delta;
    } else {
        const double alpha_old = w.scal[6 + 2 * nxt], gamma_old = w.scal[7 + 2 * nxt];
        beta = gamma / gamma_old;
        alpha = gamma / (delta - beta * gamma / alpha_old);
    }
    const double *rk = w.vec + cur * n, *wk_ = w.vec + (2 + cur) * n, *sk1 = w.vec + (4 + nxt) * n;
    double *rn = w.vec + nxt * n, *wn = w.vec + (2 + nxt) * n, *sk = w.vec + (4 + cur) * n, *pp = w.vec + 6 * n;
    double *x = pcg_x(v, mode);
    double ga = 0.0, de = 0.0;
    for (int64_t r = (int64_t)it.b * blockDim.x + threadIdx.x; r < n; r += (int64_t)w.nblk * blockDim.x) {
        const double ui = w.dinv[r] * rk[r];
        const double pi = ui + beta * pp[r];
        const double si = wk_[r] + beta * sk1[r];
        pp[r] = pi;
        sk[r] = si;
        x[r] += alpha * pi;
        const double ri = rk[r] - alpha * si;
        rn[r] = ri;
        const double un = w.dinv[r] * ri;
        double au = 0.0;
        for (int32_t q = w.row_ptr[r]; q < w.row_ptr[r + 1]; ++q) {
            const int32_t j = w.col[q];
            const double sj = wk_[j] + beta * sk1[j];
            au += w.val[q] * (w.dinv[j] * (rk[j] - alpha * sj));
        }
        wn[r] = au;
        ga += ri * un;
        de += au * un;
    }
    ga = block_sum(ga, lds);
    de = block_sum(de, lds);
    if (threadIdx.x == 0) {
        pout[it.b] = ga;
        pout[w.nblk + it.b] = de;
        if (it.b == 0) {
            if (k == 0) w.scal[1] = gamma;
            w.scal[6 + 2 * cur] = alpha;
            w.scal[7 + 2 * cur] = gamma;
            w.scal[5] = k + 1;
        }
    }
}

template <class T, int MI, int MODE>
void dispatch_sweep_bpl(const DeviceView *vs, const WorkItem *wk, int n, int bpl, bool one, int block, size_t lds,
                        hipStream_t st) {
    dim3 grid(n);
    if (one) {
        switch (bpl) {
            case 1: hipLaunchKernelGGL((k_sweep<T, MI, 1, MODE, true>), grid, dim3(block), lds, st, vs, wk); break;
            case 2: hipLaunchKernelGGL((k_sweep<T, MI, 2, MODE, true>), grid, dim3(block), lds, st, vs, wk); break;
            case 4: hipLaunchKernelGGL((k_sweep<T, MI, 4, MODE, true>), grid, dim3(block), lds, st, vs, wk); break;
            default: hipLaunchKernelGGL((k_sweep<T, MI, 8, MODE, true>), grid, dim3(block), lds, st, vs, wk); break;
        }
        return;
    }
    switch (bpl) {
        case 1: hipLaunchKernelGGL((k_sweep<T, MI, 1, MODE, false>), grid, dim3(block), lds, st, vs, wk); break;
        case 2: hipLaunchKernelGGL((k_sweep<T, MI, 2, MODE, false>), grid, dim3(block), lds, st, vs, wk); break;
        default: hipLaunchKernelGGL((k_sweep<T, MI, 4, MODE, false>), grid, dim3(block), lds, st, vs, wk); break;
    }
}

template <class T, int MODE>
void dispatch_sweep_mi(const DeviceView *vs, const WorkItem *wk, int n, int maxin, int bpl, bool one, int block,
                       size_t lds, hipStream_t st) {
    if (maxin <= 2) dispatch_sweep_bpl<T, 2, MODE>(vs, wk, n, bpl, one, block, lds, st);
    else if (maxin == 3) dispatch_sweep_bpl<T, 3, MODE>(vs, wk, n, bpl, one, block, lds, st);
    else dispatch_sweep_bpl<T, 5, MODE>(vs, wk, n, bpl, one, block, lds, st);
}

template <class T>
void dispatch_sweep(const DeviceView *vs, const WorkItem *wk, int n, int maxin, int bpl, bool one, int mode,
                    int block, size_t lds, hipStream_t st) {
    if (mode == kModeLds) dispatch_sweep_mi<T, kModeLds>(vs, wk, n, maxin, bpl, one, block, lds, st);
    else if (mode == kModeHbmGhost) dispatch_sweep_mi<T, kModeHbmGhost>(vs, wk, n, maxin, bpl, one, block, lds, st);
    else dispatch_sweep_mi<T, kModeSpill>(vs, wk, n, maxin, bpl, one, block, lds, st);
}

}  // namespace

void launch_fill_zero(void *p, size_t bytes, hipStream_t st) {
    const size_t n = bytes / 4;
    if (n == 0) return;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, st, static_cast<uint32_t *>(p), n);
}

void launch_stage(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, hipStream_t st) {
    if (n <= 0) return;
    if (fp32) hipLaunchKernelGGL(k_stage<float>, dim3(n), dim3(256), 0, st, vs, wk);
    else hipLaunchKernelGGL(k_stage<double>, dim3(n), dim3(256), 0, st, vs, wk);
}

void launch_flux(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, int after, hipStream_t st) {
    if (n <= 0) return;
    if (fp32) hipLaunchKernelGGL(k_flux<float>, dim3(n), dim3(256), 0, st, vs, wk, after);
    else hipLaunchKernelGGL(k_flux<double>, dim3(n), dim3(256), 0, st, vs, wk, after);
}

void launch_moments(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, hipStream_t st) {
    if (n <= 0) return;
    if (fp32) hipLaunchKernelGGL(k_moments<float>, dim3(n), dim3(256), 0, st, vs, wk);
    else hipLaunchKernelGGL(k_moments<double>, dim3(n), dim3(256), 0, st, vs, wk);
}

void launch_update(const DeviceView *vs, const WorkItem *wk, int n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_update, dim3(n), dim3(256), 0, st, vs, wk);
}

void launch_finish(const DeviceView *vs, const WorkItem *wk, int n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_finish, dim3((n + 63) / 64), dim3(64), 0, st, vs, wk, n);
}

size_t sweep_lds_bytes(int max_levels, int gcap, int ls, int slots, int es) {
    return (size_t)(max_levels + 1) * 2 * sizeof(int)    // two int level tables
           + (size_t)2 * gcap * ls * es                  // ghost buffers
           + (size_t)std::max(slots, 1) * ls * es;       // staged values
}

void launch_sweep(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, int maxin, int bpl, bool one, int mode,
                  int block, size_t lds_bytes, hipStream_t st) {
    if (n <= 0) return;
    if (bpl != 1 && bpl != 2 && bpl != 4 && bpl != 8) bpl = 1;
    if (fp32) dispatch_sweep<float>(vs, wk, n, maxin, bpl, one, mode, block, lds_bytes, st);
    else dispatch_sweep<double>(vs, wk, n, maxin, bpl, one, mode, block, lds_bytes, st);
}

void launch_pcg_block(const DeviceView *vs, const WorkItem *wk, int n, int mode, hipStream_t st) {
    if (n <= 0) return;
    const double rtol2_o = mode == 1 ? 1e-24 : -1.0;
    const int max_o = mode == 1 ? 4000 : -1;
    hipLaunchKernelGGL(k_pcg_block, dim3(n), dim3(1024), 0, st, vs, wk, mode, rtol2_o, max_o);
}

void launch_pcg_multi(const DeviceView *vs, const WorkItem *wk, int n, int mode, int max_iter, hipStream_t st,
                      int k0, bool init) {
    if (n <= 0) return;
    const double rtol2_o = mode == 1 ? 1e-24 : -1.0;
    const int max_o = mode == 1 ? (1 << 30) : -1;
    if (init) hipLaunchKernelGGL(k_cg1_init, dim3(n), dim3(256), 0, st, vs, wk, mode);
    for (int k = k0; k < k0 + max_iter; ++k)
        hipLaunchKernelGGL(k_cg1_iter, dim3(n), dim3(256), 0, st, vs, wk, mode, k, rtol2_o, max_o);
}

void launch_set_controls(SolveState *s, int stop, double tol, int max_iter, int patience, hipStream_t st) {
    hipLaunchKernelGGL(k_set_controls, dim3(1), dim3(64), 0, st, s, stop, tol, max_iter, patience);
}

void launch_widen(int64_t n, const float *in, double *out, hipStream_t st) {
    if (n <= 0) return;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_widen, dim3(grid), dim3(256), 0, st, n, in, out);
}

void launch_collect_states(const DeviceView *vs, int n, SolveState *out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_collect_states, dim3((n + 63) / 64), dim3(64), 0, st, vs, n, out);
}

void launch_affine(int64_t n, const double *in, double scale, double offset, double *out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_affine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, in, scale, offset, out);
}

void launch_gather(int64_t n, const int32_t *idx, const double *in, void *out, bool fp32, hipStream_t st) {
    if (n <= 0) return;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (fp32) hipLaunchKernelGGL(k_gather<float>, grid, dim3(256), 0, st, n, idx, in, static_cast<float *>(out));
    else hipLaunchKernelGGL(k_gather<double>, grid, dim3(256), 0, st, n, idx, in, static_cast<double *>(out));
}

void launch_distribution(const DeviceView *v, bool fp32, int band, int dir, double *out, int64_t N, hipStream_t st) {
    dim3 grid((unsigned)((N + 255) / 256));
    if (fp32) hipLaunchKernelGGL(k_distribution<float>, grid, dim3(256), 0, st, v, band, dir, out);
    else hipLaunchKernelGGL(k_distribution<double>, grid, dim3(256), 0, st, v, band, dir, out);
}

}  // namespace nbte

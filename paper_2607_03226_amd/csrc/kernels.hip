// HIP kernels (gfx950) of the steady BTE transport path.
//
// Storage convention: for every (direction i, cell c, band l) the library
// keeps g = e - C_l theta(c) / W, the part of the energy density that is not
// in equilibrium at the lattice temperature the sweep used (Methods, Eq. (11)
// gives the equilibrium C T_L / W).  Two layouts (DeviceView::planes):
// cell-major g[(i*N + c)*B + l], the bands of one (direction, cell)
// contiguous; or, for large problems, per direction in band-block planes in
// the sweep's stream order, so that a sweep pass stores one contiguous run
// (the reductions and the boundary kernels then permute, see below).  g is
// stored in FP64 or FP32; the sweep runs
// in the storage type's arithmetic (FP32 for the mixed path), while the
// equilibrium-imbalance differences, the band x direction reductions, the
// diffusion correction and the residual accumulate in FP64.
//
// Every per-iteration kernel takes the descriptor array of the solves it
// serves and a work table (one WorkItem per workgroup).  A solve whose state
// says it has stopped is skipped by every kernel, so a captured launch
// sequence can run past the convergence of some of its solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

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

// Distribution layout: per direction, band-block planes of the sweep's bands
// per workgroup, each in the direction's stream (level) order.  Band l lies
// in plane k = l / bpb at offset k N bpb + (l - k bpb); the plane's rows are
// w_k = min(bpb, B - k bpb) values wide (one row per stream position).
struct GPlane {
    int64_t off;   // offset of band l within a direction's N B values, at position 0
    int w;         // row width of its plane
};
__device__ __forceinline__ GPlane gplane(const DeviceView &v, int lam) {
    const int k = lam / v.bpb;
    GPlane p;
    p.off = (int64_t)k * v.N * v.bpb + (lam - k * v.bpb);
    p.w = min(v.bpb, v.B - k * v.bpb);
    return p;
}
// element of band p at stream position t of direction i
__device__ __forceinline__ int64_t gat_pos(const DeviceView &v, const GPlane &p, int64_t i, int64_t t) {
    return i * v.N * v.B + p.off + t * p.w;
}
// element of band p at cell c of direction i
__device__ __forceinline__ int64_t gat_cell(const DeviceView &v, const GPlane &p, int64_t i, int64_t c) {
    return gat_pos(v, p, i, v.pos[i * v.N + c]);
}

// element of (direction i, cell c, band lam) in the solve's layout
__device__ __forceinline__ int64_t g_elem(const DeviceView &v, int64_t i, int64_t c, int lam) {
    return v.planes ? gat_cell(v, gplane(v, lam), i, c) : (i * v.N + c) * v.B + lam;
}

// The distribution of a boundary face's owner: value (i, lam) at
// p[i * stride + lam] (cell-major: the distribution itself; plane layout:
// the owner's boundary row)
template <class T>
struct OwnerRows {
    const T *p;
    int64_t stride;
};
template <class T>
__device__ __forceinline__ OwnerRows<T> owner_rows(const DeviceView &v, int64_t bf) {
    OwnerRows<T> o;
    if (v.planes) {
        o.p = static_cast<const T *>(v.brow) + (int64_t)v.bf_brow[bf] * v.D * v.B;
        o.stride = v.B;
    } else {
        o.p = static_cast<const T *>(v.g) + (int64_t)v.bf_owner[bf] * v.B;
        o.stride = v.N * v.B;
    }
    return o;
}

// bit pattern of a non-negative double: ordered like the values (atomic maxima)
__device__ __forceinline__ unsigned long long dbits(double x) {
    return static_cast<unsigned long long>(__double_as_longlong(x));
}

// atomic maximum into a word that only grows within a launch: the atomic is
// skipped when the word already holds at least x (a read first), so the
// many waves below the running maximum do not queue on the one word
__device__ __forceinline__ void max_into(unsigned long long NBTE_G *word, double x) {
    const unsigned long long b = dbits(x);
    if (b > *reinterpret_cast<volatile unsigned long long NBTE_G *>(word)) atomicMax(word, b);
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
// BL = min(B, 64) bands per pass, JG = 64 / BL directions in flight per band.
// The diffuse part comes from the per-band outgoing sums the flux kernel
// stored after the previous sweep (bsum = sum_out w (s.S) e, e of that
// sweep), so only specular parts read the distribution.  The face's incoming
// flow sum_l v_l sum_in w (s.S) e_in, with the values just written, is kept
// for the flux kernel of this iteration (Jin).
// Accelerated iteration: the inflow of the coming sweep is the mixed iterate's
// (acc.ain_x, temperature units), written as the deviation from the owner's
// equilibrium at the coming sweep's theta; the face's incoming flow as above.
template <class T>
__device__ void bc_face_mixed(const DeviceView &v, int64_t bf) {
    const int lane = threadIdx.x & 63;
    const int D = v.D, B = v.B;
    const int c = v.bf_owner[bf];
    T *gv = static_cast<T *>(v.gval);
    const double *sd = v.sdotS + bf * D;
    const int32_t *row = v.in_row + bf * D;
    const double thc = theta_cur(v)[c];
    const int BL = B < 64 ? B : 64;
    const int JG = 64 / BL;
    const int jg = lane / BL, ml = lane - jg * BL;
    if (v.bf_kind[bf] == NBTE_BC_THERMALIZING) {
        // fixed inflow, not part of the state (and no net flow kept)
        const double thw = v.bf_thw[bf];
        for (int l0 = 0; l0 < B; l0 += BL) {
            const int lam = l0 + ml;
            if (jg >= JG || lam >= B) continue;
            const T val = static_cast<T>(v.Cw[lam] * (thw - thc));
#pragma unroll 8
            for (int i = jg; i < D; i += JG) {
                const int r = row[i];
                if (r >= 0) gv[(int64_t)r * B + lam] = val;
            }
        }
        return;
    }
    const double *ax = v.acc.ain_x;
    const int32_t *arow = v.acc.in + bf * D;   // the state's rows (independent of the ghost rows' load)
    double jin = 0.0;
    for (int l0 = 0; l0 < B; l0 += BL) {
        const int lam = l0 + ml;
        if (jg >= JG || lam >= B) continue;
        const double cw = v.Cw[lam];
        double acc = 0.0;
#pragma unroll 8
        for (int i = jg; i < D; i += JG) {
            const int r = row[i];
            if (r >= 0) {
                const double t = ax[(int64_t)arow[i] * B + lam];
                gv[(int64_t)r * B + lam] = static_cast<T>(cw * (t - thc));
                acc += v.w[i] * sd[i] * t;
            }
        }
        jin += v.vel[lam] * cw * acc;
    }
    jin = wave_sum(jin);
    if (lane == 0) v.Jin[bf] = jin;
}

// The inflow a boundary face's incoming rows receive from the distribution of
// the last sweep (the boundary conditions above applied to it), in
// temperature units (e W / C_l), into dst (acc.ain_G: the image of an
// accelerated step; acc.ain_x: the initial state at prepare), at the rows
// acc.in gives (a thermalizing face's fixed inflow is not part of the
// state: nothing is written for it).  Runs after the
// iteration's rotation, so theta[prev] is the last sweep's temperature and
// bsum holds the outgoing sums of its distribution.
template <class T>
__device__ void bc_face_abs(const DeviceView &v, int64_t bf, double *dst) {
    const int lane = threadIdx.x & 63;
    const int D = v.D, B = v.B;
    const int c = v.bf_owner[bf];
    const OwnerRows<T> og = owner_rows<T>(v, bf);   // the owner's distribution
    const int BL = B < 64 ? B : 64;
    const int JG = 64 / BL;
    const int jg = lane / BL, ml = lane - jg * BL;
    if (v.bf_kind[bf] == NBTE_BC_THERMALIZING) return;   // fixed inflow: not part of the state
    const int32_t *arow = v.acc.in + bf * D;
    const double thp = theta_prev(v)[c];
    const double p = v.bf_p[bf];
    const double iw = 1.0 / v.win[bf];
    const int32_t *mir = v.mirror + bf * D;
    for (int l0 = 0; l0 < B; l0 += BL) {
        const int lam = l0 + ml;
        if (jg >= JG || lam >= B) continue;
        const double cw = v.Cw[lam];
        const double diff = p < 1.0 ? v.bsum[bf * B + lam] * iw / cw : 0.0;
#pragma unroll 8
        for (int i = jg; i < D; i += JG) {
            const int r = arow[i];
            if (r < 0) continue;
            double t = (1.0 - p) * diff;
            if (p > 0.0) t += p * (ld(og.p, (int64_t)mir[i] * og.stride + lam) / cw + thp);
            dst[(int64_t)r * B + lam] = t;
        }
    }
}

template <class T>
__device__ void bc_face(const DeviceView &v, int64_t bf, double *red) {
    if (v.acc.m > 0) {
        bc_face_mixed<T>(v, bf);
        return;
    }
    const int lane = threadIdx.x & 63;
    const int D = v.D, B = v.B;
    const int c = v.bf_owner[bf];
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
#pragma unroll 8
            for (int i = jg; i < D; i += JG) {
                const int r = row[i];
                if (r >= 0) gv[(int64_t)r * B + lam] = val;
            }
        }
        return;
    }
    const double thp = theta_prev(v)[c];
    const double p = v.bf_p[bf];
    const double iw = 1.0 / v.win[bf];
    const int32_t *mir = v.mirror + bf * D;
    const OwnerRows<T> og = owner_rows<T>(v, bf);   // the owner's distribution
    // second order: the owner's outgoing face values carry their increments
    // (slot of the distribution this stage reads)
    const T *bd = v.order == 2 ? static_cast<const T *>(v.bdelta) + (int64_t)(v.state->iterations & 1) * v.NBF * D * B +
                                     bf * D * B
                               : nullptr;
    double jin = 0.0;
    for (int l0 = 0; l0 < B; l0 += BL) {
        const int lam = l0 + ml;
        if (jg >= JG || lam >= B) continue;
        const double cw = v.Cw[lam];
        const double eq = cw * thp;
        const double eqc = cw * thc;
        const double diff = p < 1.0 ? v.bsum[bf * B + lam] * iw : 0.0;
        double acc = 0.0;
        if (p > 0.0) {
#pragma unroll 8
            for (int i = jg; i < D; i += JG) {
                const int r = row[i];
                const int mi = mir[i] >= 0 ? mir[i] : 0;   // outgoing directions have no mirror entry
                const double em = ld(og.p, (int64_t)mi * og.stride + lam) + eq + (bd ? ld(bd, (int64_t)mi * B + lam) : 0.0);
                const double e = (1.0 - p) * diff + p * em;
                if (r >= 0) {
                    gv[(int64_t)r * B + lam] = static_cast<T>(e - eqc);
                    acc += v.w[i] * sd[i] * e;
                }
            }
        } else {
#pragma unroll 8
            for (int i = jg; i < D; i += JG) {
                const int r = row[i];
                if (r >= 0) {
                    gv[(int64_t)r * B + lam] = static_cast<T>(diff - eqc);
                    acc += v.w[i] * sd[i] * diff;
                }
            }
        }
        jin += v.vel[lam] * acc;
    }
    jin = wave_sum(jin);
    if (lane == 0) v.Jin[bf] = jin;
    (void)red;
}

// The imbalance term D of stream entries t0, t0 + stride, ...: every load of
// an entry (its cell, upwind cells and coefficients) is issued before the
// theta gathers they feed, the fan-in is a compile-time bound (rows past a
// cell's fan-in have coefficient 0 and point at the cell itself).
template <class T, int MI>
__device__ __forceinline__ void stage_dc(const DeviceView &v, int64_t t0, int64_t stride) {
    const int64_t n = (int64_t)v.D * v.N;
    const double *th = theta_cur(v);
    const T *cf = static_cast<const T *>(v.t_coef);
    T *dc = static_cast<T *>(v.t_dc);
    for (int64_t t = t0; t < n; t += stride) {
        int up[MI];
        T c[MI];
        const int cell = v.p_cell[t];
#pragma unroll
        for (int j = 0; j < MI; ++j) {
            up[j] = v.p_upc[j * n + t];
            c[j] = cf[j * n + t];
        }
        const double thc = th[cell];
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < MI; ++j) acc += static_cast<double>(c[j]) * (th[up[j]] - thc);
        dc[t] = static_cast<T>(acc);
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
    } else if (it.a == 4) {
        // lagged faces: the upwind cell's value of the previous iterate, as the
        // deviation from the downwind cell's equilibrium at the coming theta
        const int B = v.B;
        const T *g = static_cast<const T *>(v.g);
        T *gv = static_cast<T *>(v.gval);
        const double *thp = theta_prev(v), *thc = theta_cur(v);
        for (int64_t t = (int64_t)it.b * blockDim.x + threadIdx.x; t < v.n_lag * B; t += (int64_t)it.c * blockDim.x) {
            const int lam = (int)(t % B);
            const int32_t *L = v.lag + 4 * (t / B);
            const double e = ld(g, g_elem(v, L[1], L[3], lam)) + v.Cw[lam] * thp[L[3]];
            gv[(int64_t)L[0] * B + lam] = static_cast<T>(e - v.Cw[lam] * thc[L[2]]);
        }
    } else if (it.a >= 2) {
        // kind 2: the image of step k (steps done) into half k mod 2 of ain_G
        const AccelWork &a = v.acc;
        double *dst = it.a == 2 ? a.ain_G + (int64_t)((int)a.scal[0] & 1) * a.NR : a.ain_x;
        const int wv = threadIdx.x >> 6;
        for (int64_t bf = (int64_t)it.b * 4 + wv; bf < v.NBF; bf += (int64_t)it.c * 4) bc_face_abs<T>(v, bf, dst);
    } else {
        // D = sum_j |a_j| (theta_up_j - theta_c): the closed cell's
        // sum_{a<0} |a| - sum_{a>0} a vanishes (divergence theorem, to the
        // rounding of the face vectors), so D needs no outflow term and is
        // exactly zero for a uniform theta.  The differences are taken in
        // FP64, then weighted by the sweep's coefficients.
        if (v.maxin == 2) stage_dc<T, 2>(v, t0, stride);
        else if (v.maxin == 3) stage_dc<T, 3>(v, t0, stride);
        else stage_dc<T, 5>(v, t0, stride);
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

constexpr int kGhostPerThread = 1;    // ghost values a thread prefetches per level
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

// Raw buffer resources (CDNA buffer descriptors) over the sweep's streams.  A
// buffer load adds a per-lane 32-bit byte offset and a uniform (SGPR) byte
// offset to the descriptor's base, so the reference rows j of a stream are
// one descriptor with the row offset j D N in an SGPR: no per-lane 64-bit
// address is ever formed, and no address temporary can reuse a register
// whose load is still in flight.  Reads whose lane offset is at or past the
// descriptor's size return 0.
constexpr int kBufferWord3 = 0x00020000;   // gfx9 raw buffer, 32-bit elements
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void NBTE_G *p, uint64_t bytes) {
    const uint32_t n = bytes > 0xffffffffull ? 0xffffffffu : (uint32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)n, kBufferWord3);
}
template <class T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff);
template <>
__device__ __forceinline__ int bload<int>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return (int)__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0);
}
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
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

// The streams of one direction as two buffer descriptors (base at the
// direction's first position).  The rows of each kind are contiguous, D N
// elements apart: ints = cell | slot | MI reference rows, reals = outflow
// sum | imbalance term D | heat source | MI coefficient rows.
struct SweepStreams {
    __amdgpu_buffer_rsrc_t ints, reals;
    uint32_t row4, rowT;   // byte distance of two rows (int32 / storage type)
};

template <class T>
__device__ __forceinline__ SweepStreams sweep_streams(const DeviceView &v, int64_t base, int MI) {
    const int64_t DN = (int64_t)v.D * v.N;
    const uint64_t es = sizeof(T);
    SweepStreams S;
    S.ints = make_rsrc(v.p_cell + base, (uint64_t)((2 + MI) * DN - base) * 4);
    S.reals = make_rsrc(static_cast<const T NBTE_G *>(v.t_sout) + base, (uint64_t)((3 + MI) * DN - base) * es);
    S.row4 = (uint32_t)(DN * 4);
    S.rowT = (uint32_t)(DN * (int64_t)es);
    return S;
}

template <class T, int MI, bool PL>
__device__ __forceinline__ void load_rec(SweepRec<T, MI> &r, const SweepStreams &S, int k, int kend) {
    // the loads are issued on every path (a past-the-end record reads stream
    // position 0 of the direction), so the number of loads in flight is the
    // same on every path and a later wait on an older record can leave the
    // younger prefetches outstanding.  Stream positions fit 32 bits.
    r.ok = k < kend;
    const uint32_t at = (uint32_t)(r.ok ? k : 0);
    const uint32_t o4 = at * 4u, oT = at * (uint32_t)sizeof(T);
    if constexpr (!PL) r.c = bload<int>(S.ints, o4, 0);   // the plane layout stores by stream position
    r.mine = bload<int>(S.ints, o4, S.row4);
    r.sout = bload<T>(S.reals, oT, 0);
    r.dc = bload<T>(S.reals, oT, S.rowT);
    r.q = bload<T>(S.reals, oT, 2 * S.rowT);
#pragma unroll
    for (int j = 0; j < MI; ++j) {
        r.ref[j] = bload<int>(S.ints, o4, (2 + j) * S.row4);
        r.cf[j] = bload<T>(S.reals, oT, (3 + j) * S.rowT);
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
__device__ __forceinline__ T *lds_elems();
template <>
__device__ __forceinline__ double *lds_elems<double>() { return sweep_lds; }
template <>
__device__ __forceinline__ float *lds_elems<float>() { return sweep_ldsf; }
template <class T>
__device__ __forceinline__ T lds_get(int k) { return lds_elems<T>()[k]; }
template <class T>
__device__ __forceinline__ void lds_put(int k, T x) { lds_elems<T>()[k] = x; }

// n consecutive elements as one access of up to 16 bytes per chunk (k is a
// multiple of the chunk's element count: the LDS layout keeps every lane's
// bands on a boundary of their own width)
template <class T, int C>
struct VecOf {
    typedef T type __attribute__((ext_vector_type(C)));
};
template <class T, int BPL>
constexpr int chunk_elems() { return BPL * (int)sizeof(T) >= 16 ? 16 / (int)sizeof(T) : BPL; }

template <class T, int BPL>
__device__ __forceinline__ void lds_read_bands(int k, T (&o)[BPL]) {
    constexpr int C = chunk_elems<T, BPL>();
#pragma unroll
    for (int c0 = 0; c0 < BPL; c0 += C) {
        if constexpr (C == 1) {
            o[c0] = lds_get<T>(k + c0);
        } else {
            using V = typename VecOf<T, C>::type;
            const V x = *reinterpret_cast<const V *>(lds_elems<T>() + k + c0);
#pragma unroll
            for (int e = 0; e < C; ++e) o[c0 + e] = x[e];
        }
    }
}
template <class T, int BPL>
__device__ __forceinline__ void lds_write_bands(int k, const T (&x)[BPL]) {
    constexpr int C = chunk_elems<T, BPL>();
#pragma unroll
    for (int c0 = 0; c0 < BPL; c0 += C) {
        if constexpr (C == 1) {
            lds_put<T>(k + c0, x[c0]);
        } else {
            using V = typename VecOf<T, C>::type;
            V y;
#pragma unroll
            for (int e = 0; e < C; ++e) y[e] = x[c0 + e];
            *reinterpret_cast<V *>(lds_elems<T>() + k + c0) = y;
        }
    }
}
// the same for global memory (element offset k of a uniform base)
template <class T, int BPL>
__device__ __forceinline__ void gstore_bands(T NBTE_G *base, uint32_t k, const T (&x)[BPL]) {
    constexpr int C = chunk_elems<T, BPL>();
#pragma unroll
    for (int c0 = 0; c0 < BPL; c0 += C) {
        if constexpr (C == 1) {
            gstore(base, k + c0, x[c0]);
        } else {
            using V = typename VecOf<T, C>::type;
            V y;
#pragma unroll
            for (int e = 0; e < C; ++e) y[e] = x[c0 + e];
            *reinterpret_cast<V NBTE_G *>(reinterpret_cast<char NBTE_G *>(base) + (k + c0) * (uint32_t)sizeof(T)) = y;
        }
    }
}

// the update's quotient: IEEE division in FP64, reciprocal (1 ulp) in FP32
__device__ __forceinline__ double quot(double a, double b) { return a / b; }
__device__ __forceinline__ float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// The second-order scheme's deferred correction of a record's bands
// (requested with the record; empty for the first-order kernels).
template <class T, int BPL, bool ON>
struct CorrVals {
    T v[BPL];
};
template <class T, int BPL>
struct CorrVals<T, BPL, false> {};

template <class T, int MI, int BPL, bool SO2, bool PL>
__device__ __forceinline__ void sweep_cell(const SweepRec<T, MI> &r, const DeviceView &v, const BandConst<T, BPL> &bc,
                                           T NBTE_G *gi, uint32_t row, int64_t base, int b0, int lane, int nb_here,
                                           const CorrVals<T, BPL, SO2> &cv = CorrVals<T, BPL, SO2>{}) {
    const int B = v.B;
    const T NBTE_G *gval = static_cast<const T NBTE_G *>(v.gval);
    // this lane's bands [lofs, lofs + BPL) of the block, nv of them real;
    // padding bands read valid rows (band clamped) and are never stored
    const int lofs = lane * BPL;
    const int nv = max(0, min(BPL, nb_here - lofs));
    // whole-lane stores are aligned (cell-major rows of B values, plane rows of nb_here)
    const bool vst = (B % BPL) == 0 && (b0 % BPL) == 0 && (nb_here % BPL) == 0 && nv == BPL;
    T out[BPL];
#pragma unroll
    for (int jb = 0; jb < BPL; ++jb) {
        const int lb = lofs + jb;
        const int lam = min(b0 + lb, B - 1);
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
                // value without an LDS slot: its stored copy at the
                // neighbour's position (plane layout: that row of this band
                // block's plane; cell-major: the neighbour cell's row)
                const int64_t at = -(kSpill + 1) - rf;
                if constexpr (PL) up = gi[at * nb_here + min(lb, nb_here - 1)];
                else up = gi[(int64_t)v.p_cell[base + at] * B + lam];
            }
            gain += r.cf[j] * up;
        }
        const T vel = bc.vel[jb];
        T num = r.q * bc.src[jb] + vel * (gain + bc.cw[jb] * r.dc);
        if constexpr (SO2) num += cv.v[jb];
        out[jb] = quot(num, bc.itau[jb] + vel * r.sout);
    }
    // one LDS access and one store per 16 bytes, as in the LDS-only path
    lds_write_bands<T, BPL>(r.mine + lofs, out);   // own slot, or the scratch block
    const uint32_t gc = row + (uint32_t)lofs;
    if (vst) {
        gstore_bands<T, BPL>(gi, gc, out);
    } else {
#pragma unroll
        for (int jb = 0; jb < BPL; ++jb)
            if (jb < nv) gstore(gi, gc + jb, out[jb]);
    }
}

// The common case: every upwind reference is an LDS slot or a ghost kept in
// LDS (no spilled values, no ghost beyond the LDS capacity).  Branch-free:
// a lane reads its BPL bands of each reference with one LDS access per 16
// bytes (unused references read the zero block with coefficient 0), writes
// its own slot (the scratch block when the value has no slot or the record
// is past the end), and stores to HBM only for live records.
template <class T, int MI, int BPL>
__device__ __forceinline__ void sweep_cell_lds(const SweepRec<T, MI> &r, const BandConst<T, BPL> &bc, T NBTE_G *gi,
                                               uint32_t row, int lofs, int nv, bool vst, int trash) {
    T up[MI][BPL];
#pragma unroll
    for (int j = 0; j < MI; ++j) lds_read_bands<T, BPL>(r.ref[j] + lofs, up[j]);
    T out[BPL];
#pragma unroll
    for (int jb = 0; jb < BPL; ++jb) {
        T gain = r.cf[0] * up[0][jb];
#pragma unroll
        for (int j = 1; j < MI; ++j) gain += r.cf[j] * up[j][jb];
        const T vel = bc.vel[jb];
        out[jb] = quot(r.q * bc.src[jb] + vel * (gain + bc.cw[jb] * r.dc), bc.itau[jb] + vel * r.sout);
    }
    lds_write_bands<T, BPL>((r.ok ? r.mine : trash) + lofs, out);
    if (r.ok) {
        const uint32_t gc = row + (uint32_t)lofs;
        if (vst) {
            gstore_bands<T, BPL>(gi, gc, out);
        } else {
#pragma unroll
            for (int jb = 0; jb < BPL; ++jb)
                if (jb < nv) gstore(gi, gc + jb, out[jb]);
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

// A wave's window on a direction's level tables: lane t holds entries
// base + t of the level and ghost offsets, read back as uniform values with
// readlane (no LDS round trip on the pass cursor's path).  Refilled from LDS
// once per 63 levels.
struct LevelWindow {
    int base, lp, gp;
};

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
template <class T, int MI, int BPL, int MODE, bool ONE, bool SO2, bool PL>
__global__ void __launch_bounds__(512) k_sweep(const DeviceView *__restrict__ vs,
                                                const WorkItem *__restrict__ wk) {
    // ONE: one lane per cell (it sweeps all BPL bands of the block), so the
    // band of a register is the same on every lane and the band constants are
    // workgroup-uniform (scalar loads, scalar registers)
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
    // direction i's distribution: cell-major rows of B values, or (plane
    // layout) this band block's plane, one row of nb_here values per stream position
    T NBTE_G *gi = static_cast<T NBTE_G *>(v.g) + (int64_t)i * N * B + (PL ? (int64_t)b0 * N : 0);
    const int64_t base = (int64_t)i * N;
    const int nlev = v.lvl_off[i + 1] - v.lvl_off[i] - 1;
    if (nlev <= 0) return;
    const int nb_here = min(B, b0 + bands_per_block) - b0;
    const int ML = v.max_levels + 1;
#define lp(t) sweep_ldsi[(t)]
#define gp(t) sweep_ldsi[ML + (t)]
    const SweepLdsLayout lay = sweep_lds_layout(v.max_levels, v.gring, v.lstride, (int)sizeof(T));
    const int ls = lay.ls;
    const int gbuf0 = lay.gbuf0;        // the ghost ring
    const int gmask = v.gring - 1;      // ring positions wrap (power of two)
    {
        const int32_t *glp = v.lvl_ptr + v.lvl_off[i];
        const int32_t *ggp = v.gptr + v.lvl_off[i];
#pragma nounroll
        for (int t = threadIdx.x; t <= nlev; t += blockDim.x) {
            lp(t) = glp[t];
            gp(t) = ggp[t];
        }
        for (int t = threadIdx.x; t < ls; t += blockDim.x) lds_put<T>(lay.zero_off + t, T(0));
    }
    // this lane's bands: [lofs, lofs + BPL) of the block, nv of them real
    const int lofs = lane * BPL;
    const int nv = max(0, min(BPL, nb_here - lofs));
    // whole-lane stores are aligned (cell-major rows of B values, plane rows of nb_here)
    const bool vst = (B % BPL) == 0 && (b0 % BPL) == 0 && (nb_here % BPL) == 0 && nv == BPL;
    BandConst<T, BPL> bc;
#pragma unroll
    for (int jb = 0; jb < BPL; ++jb) {
        const int lam = min(b0 + lofs + jb, B - 1);
        bc.cw[jb] = static_cast<T>(v.Cw[lam]);
        bc.itau[jb] = static_cast<T>(v.inv_tau[lam]);
        bc.vel[jb] = static_cast<T>(v.vel[lam]);
        bc.src[jb] = static_cast<T>(v.src[lam]);
    }
    const SweepStreams S = sweep_streams<T>(v, base, MI);
    const __amdgpu_buffer_rsrc_t rg = make_rsrc(v.gval, (uint64_t)max<int64_t>(v.NBF, 1) * v.D * B * sizeof(T));
    // second order: this direction's corrections in stream order (N B values)
    const __amdgpu_buffer_rsrc_t rcor =
        SO2 ? make_rsrc(static_cast<const T NBTE_G *>(v.corr) + base * B, (uint64_t)N * B * sizeof(T)) : rg;
    // the ghost entries this thread moves: entry e = threadIdx.x + m blockDim.x
    // of a level is band gl[m] of the level's ghost gq[m]
    int gq[kGhostPerThread], gl[kGhostPerThread];
#pragma unroll
    for (int m = 0; m < kGhostPerThread; ++m) {
        const int e = threadIdx.x + m * blockDim.x;
        gq[m] = e / bands_per_block;
        gl[m] = e - gq[m] * bands_per_block;
    }
    __syncthreads();

    const int lane64 = (int)(threadIdx.x & 63);
    auto fill = [&](LevelWindow &w, int l) {
        w.base = l;
        const int t = min(l + lane64, nlev);
        w.lp = lp(t);
        w.gp = gp(t);
    };
    auto win_lp = [](const LevelWindow &w, int l) { return __builtin_amdgcn_readlane(w.lp, l - w.base); };
    auto win_gp = [](const LevelWindow &w, int l) { return __builtin_amdgcn_readlane(w.gp, l - w.base); };

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
        CorrVals<T, BPL, SO2> cv;
    };
    auto ghost_load = [&](Ghosts &h, int g0, int ne) {
        // branch-free like load_rec: entries past the level read element 0.
        // The loaded value is used as it is (no select on it here: an
        // operation on a loaded register waits for the load, and the
        // compiler may place it where that wait drains every prefetch);
        // entries past a block's real bands only feed padding bands, which
        // are never stored.
#pragma unroll
        for (int m = 0; m < kGhostPerThread; ++m) {
            const int e = threadIdx.x + m * blockDim.x;
            const bool ok = e < ne && gl[m] < nb_here;
            const uint32_t off = ok ? (uint32_t)((g0 + gq[m]) * B + b0 + gl[m]) * (uint32_t)sizeof(T) : 0u;
            h.v[m] = bload<T>(rg, off, 0);
        }
    };
    // a level's kept ghosts occupy ring positions pos, pos + 1, ...
    auto ghost_store = [&](const Ghosts &h, int pos, int g0, int ne) {
#pragma unroll
        for (int m = 0; m < kGhostPerThread; ++m) {
            const int e = threadIdx.x + m * blockDim.x;
            if (e < ne) lds_put<T>(gbuf0 + ((pos + gq[m]) & gmask) * ls + gl[m], h.v[m]);
        }
        // levels with more ghosts than the registers hold: direct copy
        const T NBTE_G *gval = static_cast<const T NBTE_G *>(v.gval);
#pragma nounroll
        for (int e = threadIdx.x + kGhostPerThread * blockDim.x; e < ne; e += blockDim.x) {
            const int q = e / bands_per_block, lb = e - q * bands_per_block;
            lds_put<T>(gbuf0 + ((pos + q) & gmask) * ls + lb,
                       lb < nb_here ? gval[(int64_t)(g0 + q) * B + b0 + lb] : T(0));
        }
    };
    // pass cursors (uniform): level, first position of the pass, end of the
    // level, the level's ghosts (first offset and count)
    LevelWindow wf, wc;
    fill(wf, 0);
    wc = wf;
    int lf = 0, kf = win_lp(wf, 0), kendf = win_lp(wf, 1), g0f = win_gp(wf, 0), gnf = win_gp(wf, 1) - g0f;
    bool firstf = true;
    int lc = 0, kc = kf, kendc = kendf, g0c = g0f, gnc = gnf, gposc = 0;
    auto fetch = [&](Set &st) {
        const bool live = lf < nlev;
        load_rec<T, MI, PL>(st.r, S, kf + slot, live ? kendf : 0);
        if constexpr (SO2) {
            // past-the-end records read position 0, like their stream loads
            const uint32_t at = (live && kf + slot < kendf) ? (uint32_t)(kf + slot) : 0u;
#pragma unroll
            for (int jb = 0; jb < BPL; ++jb)
                st.cv.v[jb] = bload<T>(rcor, (at * (uint32_t)B + (uint32_t)(b0 + lofs + jb)) * (uint32_t)sizeof(T), 0);
        }
        ghost_load(st.h, g0f, (live && firstf) ? min(gnf, gcap) * bands_per_block : 0);
        if (live) {
            kf += nslots;
            firstf = false;
            if (kf >= kendf) {
                ++lf;
                kf = kendf;
                firstf = true;
                if (lf < nlev) {
                    if (lf + 1 - wf.base > 63) fill(wf, lf);
                    kendf = win_lp(wf, lf + 1);
                    g0f += gnf;
                    gnf = win_gp(wf, lf + 1) - g0f;
                }
            }
        }
    };
    // compute the pass in `cur`, request a new pass into `nxt` (the set
    // computed last, now free).  Passes after the last one compute
    // past-the-end records (no stores to HBM, LDS writes to the scratch
    // block), so the ring below runs whole turns and has one exit test: an
    // exit after each step would join the loop's back edge, and the wait
    // analysis would then assume the youngest records of every step might
    // be the ones computed next, draining the prefetches once per turn.
    auto step = [&](Set &cur, Set &nxt, const Set &after) {
        fetch(nxt);
        // the record's first element in gi: its stream position's row in the
        // band block's plane, or its cell's row (band b0) in the cell-major layout
        const uint32_t row = PL ? (uint32_t)(kc + slot) * (uint32_t)nb_here
                                : (uint32_t)cur.r.c * (uint32_t)B + (uint32_t)b0;
        if constexpr (MODE == kModeLds)
            sweep_cell_lds<T, MI, BPL>(cur.r, bc, gi, row, lofs, nv, vst, lay.trash_off);
        else if (cur.r.ok)
            sweep_cell<T, MI, BPL, SO2, PL>(cur.r, v, bc, gi, row, base, b0, lane, nb_here, cur.cv);
        kc += nslots;
        if (lc < nlev && kc >= kendc) {   // level done
            ++lc;
            if (lc < nlev) {
                kc = kendc;
                if (lc + 1 - wc.base > 63) fill(wc, lc);
                kendc = win_lp(wc, lc + 1);
                gposc += min(gnc, gcap);   // past the previous level's kept ghosts
                g0c += gnc;
                gnc = win_gp(wc, lc + 1) - g0c;
                ghost_store(after.h, gposc, g0c, min(gnc, gcap) * bands_per_block);   // the next pass opens level lc
            }
            level_barrier<MODE == kModeSpill>();
        }
    };
    Set s0, s1, s2, s3, s4;
    static_assert(kPrefetch == 4, "the step ring below is written for four passes in flight");
    fetch(s0);
    fetch(s1);
    fetch(s2);
    fetch(s3);
    ghost_store(s0.h, gposc, g0c, min(gnc, gcap) * bands_per_block);
    __syncthreads();
#pragma nounroll
    do {
        step(s0, s4, s1);
        step(s1, s0, s2);
        step(s2, s1, s3);
        step(s3, s2, s4);
        step(s4, s3, s0);
    } while (lc < nlev);
}
#undef lp
#undef gp

// --------------------------------------------------------------------------
// second-order face values by deferred correction
//
// The face value of a (band, direction) system on face f is the upwind side's
// e_U + G_U . (x_f - x_U), G the least-squares cell gradient of the system's
// last distribution.  The sweep keeps the first-order operator and takes
//   corr_c = -v sum_f a_cf delta_f     (delta_f = G_U . (x_f - x_U); boundary
//                                       inflow faces have none)
// as an extra right-hand side, from the previous distribution.  phase 0: after
// a sweep (distribution relative to theta[cur]; increments into slot
// (iterations + 1) & 1); phase 1: at prepare (theta[cur] = theta^0, slot 0);
// phase 2: after the rotation of a stopped iteration (theta[prev]; slot
// iterations & 1).
// --------------------------------------------------------------------------
__device__ __forceinline__ const double *recon_theta(const DeviceView &v, int phase) {
    return phase == 2 ? theta_prev(v) : theta_cur(v);
}

template <class T>
__global__ void __launch_bounds__(256) k_grad(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk,
                                              int phase) {
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (phase == 0 && v.state->done) return;
    const double *th = recon_theta(v, phase);
    const int64_t N = v.N;
    const int B = v.B, F = v.F;
    const int64_t total = (int64_t)v.D * N * B;
    const T *g = static_cast<const T *>(v.g);
    T *gr = static_cast<T *>(v.grad);
    for (int64_t t = (int64_t)it.b * blockDim.x + threadIdx.x; t < total; t += (int64_t)it.c * blockDim.x) {
        const int lam = (int)(t % B);
        const int64_t ic = t / B;
        const int64_t c = ic % N, i = ic / N;
        const double cw = v.Cw[lam];
        const double gc = ld(g, g_elem(v, i, c, lam)), thc = th[c];
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int f = 0; f < F; ++f) {
            const int32_t n = v.nbr[c * F + f];
            if (n < 0) continue;
            const double d = (ld(g, g_elem(v, i, n, lam)) - gc) + cw * (th[n] - thc);
            const double *w = v.lsq + (c * F + f) * 3;
            gx += w[0] * d;
            gy += w[1] * d;
            gz += w[2] * d;
        }
        gr[t] = static_cast<T>(gx);
        gr[total + t] = static_cast<T>(gy);
        gr[2 * total + t] = static_cast<T>(gz);
    }
}

template <class T>
__device__ __forceinline__ double grad_dot(const T *gr, int64_t total, int64_t at, const double *x, const double *y) {
    return ld(gr, at) * (x[0] - y[0]) + ld(gr, total + at) * (x[1] - y[1]) + ld(gr, 2 * total + at) * (x[2] - y[2]);
}

template <class T>
__global__ void __launch_bounds__(256) k_recon(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk,
                                               int phase) {
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (phase == 0 && v.state->done) return;
    const int64_t N = v.N;
    const int B = v.B, F = v.F, D = v.D;
    const int64_t total = (int64_t)D * N * B;
    const T *gr = static_cast<const T *>(v.grad);
    if (it.a == 0) {
        // the correction of every stream entry (position p = i N + k of direction i)
        T *corr = static_cast<T *>(v.corr);
        for (int64_t t = (int64_t)it.b * blockDim.x + threadIdx.x; t < total; t += (int64_t)it.c * blockDim.x) {
            const int lam = (int)(t % B);
            const int64_t pos = t / B;
            const int64_t i = pos / N;
            const int64_t c = v.p_cell[pos];
            const double *sd = v.dirs + 3 * i;
            const double *xc = v.xc + 3 * c;
            const double iv = 1.0 / v.V[c];
            double acc = 0.0;
            for (int f = 0; f < F; ++f) {
                const double *S = v.Sv + (c * F + f) * 3;
                const double a = (sd[0] * S[0] + sd[1] * S[1] + sd[2] * S[2]) * iv;
                const double *xf = v.xf + (c * F + f) * 3;
                if (a > 0.0) {
                    acc += a * grad_dot(gr, total, (i * N + c) * B + lam, xf, xc);
                } else if (a < 0.0) {
                    const int32_t n = v.nbr[c * F + f];
                    if (n >= 0) acc += a * grad_dot(gr, total, (i * N + n) * B + lam, xf, v.xc + 3 * (int64_t)n);
                }
            }
            corr[t] = static_cast<T>(-v.vel[lam] * acc);
        }
    } else {
        // increments of the outgoing values on the boundary faces
        const int64_t nb = v.NBF * D * B;
        const int slot = phase == 1 ? 0 : (phase == 0 ? (v.state->iterations + 1) & 1 : v.state->iterations & 1);
        T *bd = static_cast<T *>(v.bdelta) + (int64_t)slot * nb;
        for (int64_t t = (int64_t)it.b * blockDim.x + threadIdx.x; t < nb; t += (int64_t)it.c * blockDim.x) {
            const int lam = (int)(t % B);
            const int64_t fi = t / B;
            const int64_t bf = fi / D, i = fi % D;
            double x = 0.0;
            if (v.sdotS[fi] > 0.0) {
                const int64_t c = v.bf_owner[bf];
                x = grad_dot(gr, total, (i * N + c) * B + lam, v.xf + (c * F + v.bf_local[bf]) * 3, v.xc + 3 * c);
            }
            bd[t] = static_cast<T>(x);
        }
    }
}

// --------------------------------------------------------------------------
// Jacobi-preconditioned BiCGSTAB of one (band, direction) system, the
// paper's optional iterative inner solver; one workgroup per system:
//   A g = b,   (A g)_c = d_c g_c - v sum_{a_cf < 0, interior} |a_cf| g_n,
//   d_c = 1/tau + v sum_{a_cf > 0} a_cf,
//   b_c = Qdot_c S_l + v sum_{a_cf < 0, boundary} |a_cf| ghost + v (C_l/W) D_c,
// the deviation form of the sweep with every interior face implicit (also
// the faces a cyclic order lags).  Right preconditioning by diag(d), started
// from the stored distribution; stops at ||r|| <= rtol ||b||, the cap, or a
// breakdown.  Work vectors (system-major, FP64): r, r0, p, v, s, t, p/d,
// s/d, d.  Reductions are workgroup sums in a fixed order.
// --------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(1024) k_bicgstab(const DeviceView *__restrict__ vs,
                                                   const WorkItem *__restrict__ wk) {
    __shared__ double red[32];
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (v.state->done) return;
    const int i = it.a, lam = it.b;
    const int64_t N = v.N;
    const int B = v.B, F = v.F, D = v.D;
    const double *sd = v.dirs + 3 * i;
    const double vel = v.vel[lam], itau = v.inv_tau[lam], cw = v.Cw[lam], src = v.src[lam];
    // the system's values: cell-major (stride B), or band lam's plane of
    // direction i (cell c at row pos_i(c))
    const GPlane pl = gplane(v, lam);
    T *xb = static_cast<T *>(v.g) + (int64_t)i * N * B + (v.planes ? pl.off : lam);
    const int32_t *pi = v.pos + (int64_t)i * N;
    const bool planes = v.planes != 0;
    auto xat = [&](int64_t c) -> T & { return planes ? xb[(int64_t)pi[c] * pl.w] : xb[c * B]; };
    const T *gv = static_cast<const T *>(v.gval);
    const double *th = theta_cur(v);
    const int64_t sys = (int64_t)i * B + lam, DBN = (int64_t)D * B * N;
    double *r = v.bicg + sys * N, *r0 = r + DBN, *p = r + 2 * DBN, *vv = r + 3 * DBN, *sv = r + 4 * DBN,
           *t = r + 5 * DBN, *ph = r + 6 * DBN, *sh = r + 7 * DBN, *d = r + 8 * DBN;
    const int nt = blockDim.x;
    auto coef = [&](int64_t c, int f) {
        const double *S = v.Sv + (c * F + f) * 3;
        return (sd[0] * S[0] + sd[1] * S[1] + sd[2] * S[2]) / v.V[c];
    };
    // A y for a vector y given by its values at cells (y(n))
    auto apply = [&](int64_t c, auto &&y) {
        double acc = d[c] * y(c);
        for (int f = 0; f < F; ++f) {
            const int32_t n = v.nbr[c * F + f];
            if (n < 0) continue;
            const double a = coef(c, f);
            if (a < 0.0) acc += vel * a * y(n);
        }
        return acc;
    };
    double bb = 0.0, rr = 0.0;
    for (int64_t c = threadIdx.x; c < N; c += nt) {
        double dd = itau, b = v.Qc[c] * src, dsum = 0.0;
        for (int f = 0; f < F; ++f) {
            const double a = coef(c, f);
            const int32_t n = v.nbr[c * F + f];
            if (a > 0.0) {
                dd += vel * a;
            } else if (a < 0.0) {
                if (n >= 0) {
                    dsum += -a * (th[n] - th[c]);
                } else {
                    const int32_t row = v.in_row[(int64_t)(-n - 1) * D + i];
                    b += vel * -a * ld(gv, (int64_t)row * B + lam);
                }
            }
        }
        b += vel * cw * dsum;
        d[c] = dd;
        sv[c] = b;   // b, until the residual is formed
        bb += b * b;
    }
    __syncthreads();
    for (int64_t c = threadIdx.x; c < N; c += nt) {
        const double rc = sv[c] - apply(c, [&](int64_t n) { return static_cast<double>(xat(n)); });
        r[c] = rc;
        r0[c] = rc;
        p[c] = 0.0;
        vv[c] = 0.0;
        rr += rc * rc;
    }
    const double bn = sqrt(block_sum(bb, red));
    const double tol2 = v.bicg_rtol * v.bicg_rtol * (bn > 0.0 ? bn * bn : 1.0);
    if (!(block_sum(rr, red) > tol2)) return;
    double rho = 1.0, alpha = 1.0, omega = 1.0;
    for (int k = 0; k < v.bicg_max_iter; ++k) {
        double acc = 0.0;
        for (int64_t c = threadIdx.x; c < N; c += nt) acc += r0[c] * r[c];
        const double rho_n = block_sum(acc, red);
        if (rho_n == 0.0 || !isfinite(rho_n)) break;
        const double beta = (rho_n / rho) * (alpha / omega);
        for (int64_t c = threadIdx.x; c < N; c += nt) {
            const double pc = r[c] + beta * (p[c] - omega * vv[c]);
            p[c] = pc;
            ph[c] = pc / d[c];
        }
        __syncthreads();
        acc = 0.0;
        for (int64_t c = threadIdx.x; c < N; c += nt) {
            const double vc = apply(c, [&](int64_t n) { return ph[n]; });
            vv[c] = vc;
            acc += r0[c] * vc;
        }
        const double r0v = block_sum(acc, red);
        if (r0v == 0.0 || !isfinite(r0v)) break;
        alpha = rho_n / r0v;
        acc = 0.0;
        for (int64_t c = threadIdx.x; c < N; c += nt) {
            const double sc = r[c] - alpha * vv[c];
            sv[c] = sc;
            sh[c] = sc / d[c];
            acc += sc * sc;
        }
        if (!(block_sum(acc, red) > tol2)) {   // block_sum synchronises: sh is complete
            for (int64_t c = threadIdx.x; c < N; c += nt) xat(c) = static_cast<T>(static_cast<double>(xat(c)) + alpha * ph[c]);
            break;
        }
        double ts = 0.0, tt = 0.0;
        for (int64_t c = threadIdx.x; c < N; c += nt) {
            const double tc = apply(c, [&](int64_t n) { return sh[n]; });
            t[c] = tc;
            ts += tc * sv[c];
            tt += tc * tc;
        }
        ts = block_sum(ts, red);
        tt = block_sum(tt, red);
        if (tt == 0.0 || !isfinite(tt)) break;
        omega = ts / tt;
        acc = 0.0;
        for (int64_t c = threadIdx.x; c < N; c += nt) {
            xat(c) = static_cast<T>(static_cast<double>(xat(c)) + alpha * ph[c] + omega * sh[c]);
            const double rc = sv[c] - omega * t[c];
            r[c] = rc;
            acc += rc * rc;
        }
        rho = rho_n;
        if (!(block_sum(acc, red) > tol2) || omega == 0.0) break;
    }
}

// --------------------------------------------------------------------------
// net heat flow through each boundary face: one wave per face
//   J_f = sum_l v_l sum_i w_i (s_i . S_f) e
// with e the owner's value for outgoing and the inflow for incoming directions
//   mode 0: inside the iteration (after the sweep, theta[cur] is its
//           temperature): the outgoing sums per band (bsum, for the next
//           boundary stage) and J_f = Jin + sum_l v_l bsum_l of every
//           reflective face (the correction's right-hand side);
//   mode 1: once the iteration has rotated theta (theta[prev] is the
//           sweep's): J_f of every face from the stored values (the
//           energy balance);
//   mode 2: at prepare: bsum of the initial distribution at theta[prev]
// Lanes are (direction group, band) pairs, BL = min(B, 64) bands per pass and
// JG = 64 / BL direction groups; the groups of a band are combined by lane
// shuffles in a fixed order.
// --------------------------------------------------------------------------
template <class T>
__device__ void flux_face(const DeviceView &v, int64_t bf, int mode) {
    if (mode != 1 && v.bf_kind[bf] == NBTE_BC_THERMALIZING) return;
    const int lane = threadIdx.x & 63;
    const int D = v.D, B = v.B;
    const int c = v.bf_owner[bf];
    const double th = (mode == 0 ? theta_cur(v) : theta_prev(v))[c];
    const OwnerRows<T> og = owner_rows<T>(v, bf);   // the owner's distribution
    const T *gv = static_cast<const T *>(v.gval);
    const double *sd = v.sdotS + bf * D;
    // second order: increments of the outgoing face values.  The net flow
    // takes those the sweep used (mode 0: the slot of the sweep's own
    // correction; mode 1, after the rotation: the last sweep's), the outgoing
    // sums of the next boundary stage those of the new distribution (mode 0:
    // the slot the reconstruction after the sweep wrote; mode 2: slot 0, the
    // initial distribution)
    const T *bj = nullptr, *bs = nullptr;
    if (v.order == 2) {
        const T *bd = static_cast<const T *>(v.bdelta);
        const int64_t slot = (int64_t)v.NBF * D * B;
        const int it = v.state->iterations;
        if (mode == 0) bj = bd + (it & 1) * slot, bs = bd + ((it + 1) & 1) * slot;
        else if (mode == 1) bj = bd + ((it + 1) & 1) * slot;
        else bs = bd;
        if (bj) bj += bf * D * B;
        if (bs) bs += bf * D * B;
    }
    const int BL = B < 64 ? B : 64, JG = 64 / BL;
    const int jg = lane / BL, ml = lane - jg * BL;
    double jsum = 0.0;
    for (int l0 = 0; l0 < B; l0 += BL) {
        const int lam = l0 + ml;
        const bool on = jg < JG && lam < B;
        const int lc = on ? lam : 0;
        const double cwt = v.Cw[lc] * th;
        double sum = 0.0, sumj = 0.0;
        if (on) {
            if (mode == 1) {
                // every direction: the inflow row of an incoming one, the
                // owner's value otherwise (s.S = 0 contributes exactly zero)
                for (int i = jg; i < D; i += JG) {
                    const int32_t row = v.in_row[bf * D + i];
                    const T *src = row >= 0 ? gv + (int64_t)row * B : og.p + (int64_t)i * og.stride;
                    double e = ld(src, lc) + cwt;
                    if (bj && row < 0) e += ld(bj, (int64_t)i * B + lc);
                    sum += (row >= 0 || sd[i] > 0.0) ? v.w[i] * sd[i] * e : 0.0;
                }
                sumj = sum;
            } else if (v.order == 2) {
                for (int i = jg; i < D; i += JG) {
                    const double e = ld(og.p, (int64_t)i * og.stride + lc) + cwt;
                    const double wsd = sd[i] > 0.0 ? v.w[i] * sd[i] : 0.0;
                    sum += wsd * (e + (bs ? ld(bs, (int64_t)i * B + lc) : 0.0));
                    sumj += wsd * (e + (bj ? ld(bj, (int64_t)i * B + lc) : 0.0));
                }
            } else {
                // outgoing directions: the owner's value is read for every
                // direction (independent loads) and weighted by s.S > 0
#pragma unroll 8
                for (int i = jg; i < D; i += JG) {
                    const double e = ld(og.p, (int64_t)i * og.stride + lc) + cwt;
                    sum += sd[i] > 0.0 ? v.w[i] * sd[i] * e : 0.0;
                }
                sumj = sum;
            }
        }
        double t = 0.0, tj = 0.0;
        for (int k = 0; k < JG; ++k) {
            t += __shfl(sum, k * BL + ml);
            tj += __shfl(sumj, k * BL + ml);
        }
        if (on && jg == 0) {
            if (mode != 1) v.bsum[bf * B + lam] = t;
            jsum += v.vel[lam] * tj;
        }
    }
    jsum = wave_sum(jsum);
    if (lane == 0 && mode != 2) {
        const double J = (mode == 0 ? v.Jin[bf] : 0.0) + jsum;
        v.Jw[bf] = J;
        if (mode == 0) v.wallJ[v.wslot[bf]] = J;   // a reflective face always has a slot
    }
}

// faces b*4 + wave, b*4 + wave + 4*nblk, ... of work item (solve, -, b, nblk)
template <class T>
__global__ void __launch_bounds__(256) k_flux(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk,
                                              int mode) {
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (mode == 0 && v.state->done) return;
    const int wv = threadIdx.x >> 6;
    for (int64_t bf = (int64_t)it.b * 4 + wv; bf < v.NBF; bf += (int64_t)it.c * 4) flux_face<T>(v, bf, mode);
}

// --------------------------------------------------------------------------
// band x direction reductions, cell-major layout (Methods, Eqs. (5), (7);
// T = energy temperature): mom_lpc lanes per cell, FP64 accumulation, shuffle
// reduction over the lanes.
// Synthetic schemes also get the collision part V beta (theta_seq - theta) of
// the correction's right-hand side; the reflective walls' net flows are added
// by k_wall_rhs once the flux is known.
// --------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void moments_block(const DeviceView &v, int64_t blk) {
    const int lpc = v.mom_lpc;
    const int64_t c = (blk * blockDim.x + threadIdx.x) / lpc;
    const int lane = threadIdx.x % lpc;
    const int64_t N = v.N;
    const int B = v.B, D = v.D;
    const T *g = static_cast<const T *>(v.g);
    double a_tau = 0, a_w = 0, qx = 0, qy = 0, qz = 0;
    double gmax = 0.0;   // second order: largest |g| W / C, the divergence watch of the deferred correction
    if (c < N) {
        for (int lam = lane; lam < B; lam += lpc) {
            double sw = 0, s_x = 0, s_y = 0, s_z = 0;
            if (v.order == 2) {
                const double icw = 1.0 / v.Cw[lam];
                for (int i = 0; i < D; ++i) gmax = fmax(gmax, fabs(ld(g, ((int64_t)i * N + c) * B + lam)) * icw);
            }
            // independent loads, eight directions in flight (summation order unchanged)
#pragma unroll 8
            for (int i = 0; i < D; ++i) {
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
    if (v.order == 2) {
        if (!(gmax <= 1e300)) gmax = INFINITY;
        for (int off = 32; off > 0; off >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, off));
        if ((threadIdx.x & 63) == 0) max_into(&v.state->maxbuf[2], gmax);
    }
    if (c < N && lane == 0) {
        const double th = theta_cur(v)[c];
        v.theta_seq[c] = th + a_tau / v.beta;
        v.thetaE[c] = th + a_w / v.C_tot;
        v.q[3 * c] = qx + th * v.qbias[0];
        v.q[3 * c + 1] = qy + th * v.qbias[1];
        v.q[3 * c + 2] = qz + th * v.qbias[2];
        if (v.scheme != NBTE_SCHEME_SEQUENTIAL) v.rhs[c] = v.V[c] * a_tau;
    }
}

// --------------------------------------------------------------------------
// band x direction reductions, plane layout (Methods, Eqs. (5), (7)), in two
// stages.  Stage 1 (in k_post): one thread per stream position t of a
// direction i reads the cell's row in each band-block plane (consecutive
// threads, consecutive rows) and forms the band sums
//   A = sum_l g_l / tau_l,   W = sum_l g_l,   U = sum_l v_l g_l
// with FP64 accumulation in band order, kept in FP64 at (i, c).
// Stage 2 (k_reduce): four lanes per cell sum w_i A, w_i W and w_i s_i U over
// the directions (FP64, lanes combined in a fixed order):
//   theta_seq = theta + sum_i w_i A_i / beta,   T = theta + sum_i w_i W_i / C,
//   q = sum_i w_i s_i U_i + theta q_bias,
// and the collision part V beta (theta_seq - theta) of the correction's
// right-hand side (the reflective faces' net flows follow in k_wall_rhs).
// --------------------------------------------------------------------------
// W > 0: every plane W bands wide with 16-byte aligned rows (vector loads);
// W = 0: any plane widths (one load per band).  A cell that owns a boundary
// face also gets its values copied into its boundary row, for the directions
// that leave through one of its boundary faces.
// The band constants (1/tau, v, C/W) are read through the constant address
// space: the band index is uniform, so they become scalar loads that do not
// wait behind the distribution loads (vector loads would be waited on band by
// band).  Nothing writes them during the launch.
#define NBTE_C __attribute__((address_space(4)))
template <class T, int W>
__device__ __forceinline__ void band_sums(const DeviceView &v, int64_t i, int64_t t0) {
    // the descriptor's fields in registers: the stores below could otherwise
    // alias the descriptor in memory and force a reload of every pointer
    const int64_t N = v.N;
    const int B = v.B, bpb = v.bpb;
    const bool so2 = v.order == 2;
    const double NBTE_C *itau = (const double NBTE_C *)v.inv_tau;
    const double NBTE_C *vel = (const double NBTE_C *)v.vel;
    const double NBTE_C *cwv = (const double NBTE_C *)v.Cw;
    const T NBTE_G *g = static_cast<const T NBTE_G *>(v.g) + i * N * B;
    const int64_t t = t0 + threadIdx.x;
    if (t >= N && !so2) return;
    const bool live = t < N;
    const int c = live ? v.p_cell[i * N + t] : 0;
    double a = 0.0, w = 0.0, u = 0.0;
    double gmax = 0.0;   // second order: largest |g| W / C, the divergence watch of the deferred correction
    auto add = [&](double x, int l) {
        a += x * itau[l];
        w += x;
        u += x * vel[l];
        if (so2) gmax = fmax(gmax, fabs(x) / cwv[l]);
    };
    if (live) {
        // the boundary row of this (cell, direction), if the boundary kernels read it
        const int rb = v.p_brow[i * N + t];
        T NBTE_G *br = rb >= 0 ? static_cast<T NBTE_G *>(v.brow) + (int64_t)rb * B : nullptr;
        // rows (W > 0) or bands (W = 0) requested before the first is used: 128 bytes per thread
        constexpr int G = W > 0 ? (128 / (W * (int)sizeof(T)) > 0 ? 128 / (W * (int)sizeof(T)) : 1) : 8;
        if constexpr (W > 0) {
            using V = typename VecOf<T, W>::type;
            for (int k0 = 0; k0 < B; k0 += G * W) {
                V x[G];
#pragma unroll
                for (int q = 0; q < G; ++q) {   // branch-free: rows past the end reread the last row
                    const int kq = min(k0 + q * W, B - W);
                    x[q] = __builtin_nontemporal_load(reinterpret_cast<const V NBTE_G *>(g + (int64_t)kq * N + t * W));
                }
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    if (k0 + q * W >= B) break;
                    if (br) *reinterpret_cast<V NBTE_G *>(br + k0 + q * W) = x[q];   // rows of B values: aligned
#pragma unroll
                    for (int j = 0; j < W; ++j) add(static_cast<double>(x[q][j]), k0 + q * W + j);
                }
            }
        } else {
            // band l of plane k = l / bpb
            for (int l0 = 0; l0 < B; l0 += G) {
                T x[G];
#pragma unroll
                for (int q = 0; q < G; ++q) {   // branch-free: bands past the end reread the last band
                    const int l = min(l0 + q, B - 1);
                    const int kb = (l / bpb) * bpb;
                    x[q] = g[(int64_t)kb * N + t * min(bpb, B - kb) + (l - kb)];
                }
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    if (l0 + q >= B) break;
                    if (br) br[l0 + q] = x[q];
                    add(static_cast<double>(x[q]), l0 + q);
                }
            }
        }
        Mom3 m;
        m.a = a;
        m.w = w;
        m.u = u;
        static_cast<Mom3 NBTE_G *>(v.mom)[i * N + c] = m;
    }
    if (so2) {
        if (!(gmax <= 1e300)) gmax = INFINITY;
        for (int off = 32; off > 0; off >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, off));
        if ((threadIdx.x & 63) == 0) max_into(&v.state->maxbuf[2], gmax);
    }
}

// Reduction stage 2 (item kind 1, grid-stride over the cells), beside the
// boundary-face flux (kind 0: k_flux's mode 0 face groups, which read the
// boundary rows stage 1 wrote): both only read what k_post wrote and need
// nothing of each other.
template <class T>
__global__ void __launch_bounds__(256) k_reduce(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk) {
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (v.state->done) return;
    if (it.a == 0) {
        const int wv = threadIdx.x >> 6;
        for (int64_t bf = (int64_t)it.b * 4 + wv; bf < v.NBF; bf += (int64_t)it.c * 4) flux_face<T>(v, bf, 0);
        return;
    }
    // kReduceLanes lanes per cell, lane j taking directions j, j + kReduceLanes,
    // ...; the lanes' sums are combined by shuffles in a fixed order
    const int64_t N = v.N;
    const int D = v.D;
    const Mom3 *m = static_cast<const Mom3 *>(v.mom);
    const double *th = theta_cur(v);
    const int lane = threadIdx.x % kReduceLanes;
    const int64_t nthr = (int64_t)it.c * blockDim.x;
    const int64_t span = (N * kReduceLanes + nthr - 1) / nthr * nthr;   // whole waves run every pass
    for (int64_t k = (int64_t)it.b * blockDim.x + threadIdx.x; k < span; k += nthr) {
        const int64_t c = k / kReduceLanes;
        double a_tau = 0, a_w = 0, qx = 0, qy = 0, qz = 0;
        if (c < N) {
#pragma unroll 4
            for (int i = lane; i < D; i += kReduceLanes) {
                const Mom3 x = m[(int64_t)i * N + c];
                const double wi = v.w[i];
                a_tau += wi * x.a;
                a_w += wi * x.w;
                const double wu = wi * x.u;
                qx += wu * v.dirs[3 * i];
                qy += wu * v.dirs[3 * i + 1];
                qz += wu * v.dirs[3 * i + 2];
            }
        }
        for (int off = 1; off < kReduceLanes; off <<= 1) {
            a_tau += __shfl_xor(a_tau, off);
            a_w += __shfl_xor(a_w, off);
            qx += __shfl_xor(qx, off);
            qy += __shfl_xor(qy, off);
            qz += __shfl_xor(qz, off);
        }
        if (c >= N || lane != 0) continue;
        const double t = th[c];
        v.theta_seq[c] = t + a_tau / v.beta;
        v.thetaE[c] = t + a_w / v.C_tot;
        v.q[3 * c] = qx + t * v.qbias[0];
        v.q[3 * c + 1] = qy + t * v.qbias[1];
        v.q[3 * c + 2] = qz + t * v.qbias[2];
        if (v.scheme != NBTE_SCHEME_SEQUENTIAL) v.rhs[c] = v.V[c] * a_tau;
    }
}

// Right-hand side of the correction, wall part (collision-divergence
// identity): V (Qdot - D_h' q) = V beta (theta_seq - theta) + sum_{reflective f} J_f.
// Reflective walls carry zero net flux at the fixed point, so their transient
// flux is returned to the cell.  One thread per cell with a reflective face
// (grid-stride); the flux waves stored the net flows of a cell's reflective
// faces in consecutive slots wall_ptr[k] .. wall_ptr[k+1], in the cell's face
// order, so a thread needs two memory round trips.
__global__ void __launch_bounds__(256) k_wall_rhs(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk) {
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (v.state->done) return;
    for (int64_t k = (int64_t)it.b * blockDim.x + threadIdx.x; k < v.n_wall; k += (int64_t)it.c * blockDim.x) {
        const int c = v.wall_cell[k];
        const int j0 = v.wall_ptr[k], j1 = v.wall_ptr[k + 1];
        double r = v.rhs[c];
        for (int j = j0; j < j1; ++j) r += v.wallJ[j];
        v.rhs[c] = r;
    }
}

// The work after a sweep that reads its distribution, in one launch.
// Cell-major layout: items (solve, 0, b, nblk) boundary-face flux (k_flux's
// mode 0 face groups) and (solve, 1, b, -) moment blocks; the two read the
// same distribution and need nothing of each other, so the latency-bound face
// waves run beside the bandwidth-bound moment blocks.  Plane layout: items
// (solve, 2, b, i) reduction stage 1 over positions [256 b, + 256) of
// direction i (the face flux follows in k_reduce, from the boundary rows
// this stage writes).  solve < 0 pads.
template <class T>
__global__ void __launch_bounds__(256) k_post(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk) {
    const WorkItem it = wk[blockIdx.x];
    if (it.solve < 0) return;
    const DeviceView &v = vs[it.solve];
    if (v.state->done) return;
    if (it.a == 0) {
        const int wv = threadIdx.x >> 6;
        for (int64_t bf = (int64_t)it.b * 4 + wv; bf < v.NBF; bf += (int64_t)it.c * 4) flux_face<T>(v, bf, 0);
    } else if (it.a == 1) {
        moments_block<T>(v, it.b);
    } else {
        const int64_t i = it.c, t0 = (int64_t)it.b * blockDim.x;
        const bool full = v.B % v.bpb == 0;
        if (full && v.bpb * (int)sizeof(T) == 16) band_sums<T, 16 / sizeof(T)>(v, i, t0);
        else if (full && v.bpb * (int)sizeof(T) == 32) band_sums<T, 32 / sizeof(T)>(v, i, t0);
        else band_sums<T, 0>(v, i, t0);
    }
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
    // the waves' maxima combined in LDS, then one pair of atomics per
    // workgroup (per-wave atomics on the same two words serialise in L2:
    // config 3's 565 workgroups took 32 us, nearly all of it in the atomics)
    __shared__ double wmax[2][4];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        wmax[0][wv] = md;
        wmax[1][wv] = mt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q) {
            md = fmax(md, wmax[0][q]);
            mt = fmax(mt, wmax[1][q]);
        }
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
    const double mg = __longlong_as_double((long long)s->maxbuf[2]);
    const double res = mt > 0.0 ? md / mt : 0.0;
    s->residual = res;
    s->maxbuf[0] = 0ull;
    s->maxbuf[1] = 0ull;
    s->maxbuf[2] = 0ull;
    s->iterations += 1;
    s->rot = (s->rot + 1) % 3;
    if (res < 0.98 * s->best) {
        s->best = res;
        s->since = 0;
    } else {
        s->since += 1;
    }
    // a relative update above 1e6 cannot come from a contracting iteration
    // (a non-contracting deferred correction grows geometrically)
    // second order: a distribution whose departure from equilibrium exceeds the
    // temperature scale by 1e6 has left any contracting iteration (the
    // deferred correction's growing modes may have no collision moment, so
    // theta alone would not show them)
    if (!(res <= 1e300) || (mt > 0.0 && res > 1e6) || !(mg <= 1e6 * mt)) s->done = NBTE_DONE_DIVERGED;
    else if (s->stop && res <= s->tol) s->done = NBTE_DONE_CONVERGED;
    else if (s->stop && s->iterations >= s->max_iter) s->done = NBTE_DONE_MAX_ITER;
    else if (s->stop && s->patience > 0 && s->since >= s->patience) s->done = NBTE_DONE_STALLED;
}

// --------------------------------------------------------------------------
// Anderson acceleration of the outer iteration (see AccelWork).  After the
// finish of an iteration: theta[prev] is x's temperature, theta[cur] its
// image, ain_x / ain_G the inflow parts.  Step k (k = steps done before it):
// k = 0 keeps f and G only (x_next = G); k >= 1 writes the newest columns
// into slot (k - 1) mod m and the partial sums a_j = dF_new . dF_j and
// b_j = dF_j . f of the w = min(k, m) columns in the window.  The columns
// and the previous step's f are stored in the storage type (f and its
// differences are residuals, not temperatures, so FP32 storage loses nothing
// to cancellation); G, whose differences are taken, stays in FP64.  The sums
// use the stored values.
// --------------------------------------------------------------------------
template <class T, int W>
__device__ __forceinline__ void accel_cols_rows(const DeviceView &v, const WorkItem &it, int k, int c, double *sa,
                                                double *sb) {
    const AccelWork &a = v.acc;
    const int64_t N = v.N, NS = N + a.NR;
    const double *tx = theta_prev(v), *tg = theta_cur(v);
    // this step's inflow image and the previous step's (the other half; read
    // but unused at k = 0)
    const double *Gk = a.ain_G + (int64_t)(k & 1) * a.NR, *Gp = a.ain_G + (int64_t)((k + 1) & 1) * a.NR;
    T *dF = static_cast<T *>(a.dF);
    T *dG = static_cast<T *>(a.dG);
    for (int64_t s = (int64_t)it.b * blockDim.x + threadIdx.x; s < NS; s += (int64_t)it.c * blockDim.x) {
        const double xv = s < N ? tx[s] : a.ain_x[s - N];
        const double gv = s < N ? tg[s] : Gk[s - N];
        const double fp = static_cast<double>(static_cast<const T *>(a.fprev)[s]);
        const double gp = s < N ? a.Gprev[s] : Gp[s - N];
        double dj[W > 0 ? W : 1];
#pragma unroll
        for (int j = 0; j < W; ++j) dj[j] = j == c ? 0.0 : static_cast<double>(dF[j * NS + s]);
        const double f = gv - xv;
        if (k > 0) {
            const T dfn = static_cast<T>(f - fp);
            dF[c * NS + s] = dfn;
            dG[c * NS + s] = static_cast<T>(gv - gp);
            const double dn = static_cast<double>(dfn);
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const double d = j == c ? dn : dj[j];
                sa[j] += dn * d;
                sb[j] += d * f;
            }
        }
        static_cast<T *>(a.fprev)[s] = static_cast<T>(f);
        if (s < N) a.Gprev[s] = gv;
    }
}

template <class T>
__global__ void __launch_bounds__(256) k_accel_cols(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk) {
    __shared__ double lds[2 * kAccelMaxDepth * 4];
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (v.state->done) return;
    const AccelWork &a = v.acc;
    const int m = a.m;
    const int k = (int)a.scal[0];
    const int c = k > 0 ? (k - 1) % m : 0;
    const int w = k < m ? k : m;
    double sa[kAccelMaxDepth], sb[kAccelMaxDepth];
#pragma unroll
    for (int j = 0; j < kAccelMaxDepth; ++j) sa[j] = sb[j] = 0.0;
    switch (w) {   // the window's columns as a compile-time count: every load of an entry issued together
        case 0: accel_cols_rows<T, 0>(v, it, k, c, sa, sb); break;
        case 1: accel_cols_rows<T, 1>(v, it, k, c, sa, sb); break;
        case 2: accel_cols_rows<T, 2>(v, it, k, c, sa, sb); break;
        case 3: accel_cols_rows<T, 3>(v, it, k, c, sa, sb); break;
        case 4: accel_cols_rows<T, 4>(v, it, k, c, sa, sb); break;
        case 5: accel_cols_rows<T, 5>(v, it, k, c, sa, sb); break;
        case 6: accel_cols_rows<T, 6>(v, it, k, c, sa, sb); break;
        case 7: accel_cols_rows<T, 7>(v, it, k, c, sa, sb); break;
        default: accel_cols_rows<T, 8>(v, it, k, c, sa, sb); break;
    }
    if (k == 0) return;
    // fixed-order block sums of the 2w values (lanes, then waves)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j = 0; j < w; ++j) {
        const double x = wave_sum(sa[j]), y = wave_sum(sb[j]);
        if (lane == 0) {
            lds[(2 * j) * 4 + wv] = x;
            lds[(2 * j + 1) * 4 + wv] = y;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * w) {
        double t = 0.0;
        for (int q = 0; q < nw; ++q) t += lds[threadIdx.x * 4 + q];
        a.part[(int64_t)it.b * 2 * kAccelMaxDepth + threadIdx.x] = t;
    }
}

// One workgroup per solve: the partial sums of the step (fixed order: wave q
// sums values q, q + 4, ...; its lanes take the workgroups' partials in a
// fixed stride, then a shuffle tree), the newest row and column of the Gram
// matrix H = dF^T dF, and gamma from H gamma = dF^T f by Cholesky over the
// columns from newest to oldest, truncated at the first column that is (to
// 1e-12 of its norm) a combination of newer ones.  Thread 0 does the m x m
// algebra.
__global__ void __launch_bounds__(256) k_accel_solve(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk) {
    __shared__ double tot[2 * kAccelMaxDepth];
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (v.state->done) return;
    const AccelWork &a = v.acc;
    const int m = a.m;
    const int k = (int)a.scal[0];
    const int w = k < m ? k : m;
    if (k > 0) {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int t = wv; t < 2 * w; t += 4) {
            double x = 0.0;
            for (int b = lane; b < a.nblk; b += 64) x += a.part[(int64_t)b * 2 * kAccelMaxDepth + t];
            x = wave_sum(x);
            if (lane == 0) tot[t] = x;
        }
    }
    __syncthreads();
    // the Gram matrix into LDS (one load per thread), its newest row and column replaced
    __shared__ double H[kAccelMaxDepth * kAccelMaxDepth];
    const int c = k > 0 ? (k - 1) % m : 0;
    if (threadIdx.x < m * m) {
        const int i = threadIdx.x / m, j = threadIdx.x % m;
        double h = a.scal[1 + threadIdx.x];
        if (k > 0 && j < w && i == c) h = tot[2 * j];
        if (k > 0 && i < w && j == c) h = tot[2 * i];
        H[threadIdx.x] = h;
        a.scal[1 + threadIdx.x] = h;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    // thread 0's small dense algebra works in LDS: its loops index these
    // arrays with run-time indices, which would otherwise place them in
    // scratch memory (a global-memory round trip per access)
    __shared__ double gam[kAccelMaxDepth], L[kAccelMaxDepth][kAccelMaxDepth], y[kAccelMaxDepth];
    __shared__ int ord[kAccelMaxDepth];
    for (int j = 0; j < kAccelMaxDepth; ++j) gam[j] = 0.0;
    if (k > 0) {
        for (int p = 0; p < w; ++p) ord[p] = ((c - p) % m + m) % m;   // newest first
        int used = 0;
        for (int p = 0; p < w; ++p) {
            const double hpp = H[ord[p] * m + ord[p]];
            if (!(hpp > 0.0)) break;
            bool ok = true;
            for (int q = 0; q <= p; ++q) {
                double sum = H[ord[p] * m + ord[q]];
                for (int r = 0; r < q; ++r) sum -= L[p][r] * L[q][r];
                if (q < p) {
                    L[p][q] = sum / L[q][q];
                } else {
                    if (!(sum > 1e-12 * hpp)) ok = false;
                    else L[p][p] = sqrt(sum);
                }
            }
            if (!ok) break;
            used = p + 1;
        }
        // forward and back substitution over the accepted columns
        for (int p = 0; p < used; ++p) {
            double sum = tot[2 * ord[p] + 1];
            for (int r = 0; r < p; ++r) sum -= L[p][r] * y[r];
            y[p] = sum / L[p][p];
        }
        for (int p = used - 1; p >= 0; --p) {
            double sum = y[p];
            for (int r = p + 1; r < used; ++r) sum -= L[r][p] * y[r];
            y[p] = sum / L[p][p];
            gam[ord[p]] = y[p];
        }
    }
    for (int j = 0; j < m; ++j) a.scal[1 + m * m + j] = gam[j];
    a.scal[0] = k + 1;
}

// x_next = G - sum_j gamma_j dG_j into theta[cur] and ain_x (Gin: the
// step's inflow image).
template <class T, int W>
__device__ __forceinline__ void accel_mix_rows(const DeviceView &v, const WorkItem &it, const double *gam,
                                               const double *Gin) {
    const AccelWork &a = v.acc;
    const int64_t N = v.N, NS = N + a.NR;
    const T *dG = static_cast<const T *>(a.dG);
    double *tn = theta_at(v, th_cur(v.state));
    for (int64_t s = (int64_t)it.b * blockDim.x + threadIdx.x; s < NS; s += (int64_t)it.c * blockDim.x) {
        double d[W > 0 ? W : 1];
#pragma unroll
        for (int j = 0; j < W; ++j) d[j] = static_cast<double>(dG[j * NS + s]);
        double x = s < N ? a.Gprev[s] : Gin[s - N];
#pragma unroll
        for (int j = 0; j < W; ++j) x -= gam[j] * d[j];
        if (s < N) tn[s] = x;
        else a.ain_x[s - N] = x;
    }
}

template <class T>
__global__ void __launch_bounds__(256) k_accel_mix(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk) {
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (v.state->done) return;
    const AccelWork &a = v.acc;
    const int m = a.m;
    const int k = (int)a.scal[0];   // steps done, this one included
    const int w = k - 1 < m ? k - 1 : m;
    double gam[kAccelMaxDepth];
#pragma unroll
    for (int j = 0; j < kAccelMaxDepth; ++j) gam[j] = j < m ? a.scal[1 + m * m + j] : 0.0;
    const double *Gin = a.ain_G + (int64_t)((k - 1) & 1) * a.NR;   // this step's (k - 1) image
    switch (w) {
        case 0: accel_mix_rows<T, 0>(v, it, gam, Gin); break;
        case 1: accel_mix_rows<T, 1>(v, it, gam, Gin); break;
        case 2: accel_mix_rows<T, 2>(v, it, gam, Gin); break;
        case 3: accel_mix_rows<T, 3>(v, it, gam, Gin); break;
        case 4: accel_mix_rows<T, 4>(v, it, gam, Gin); break;
        case 5: accel_mix_rows<T, 5>(v, it, gam, Gin); break;
        case 6: accel_mix_rows<T, 6>(v, it, gam, Gin); break;
        case 7: accel_mix_rows<T, 7>(v, it, gam, Gin); break;
        default: accel_mix_rows<T, 8>(v, it, gam, Gin); break;
    }
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
// element of band l at stream position t in a direction's planes of bpb bands
__device__ __forceinline__ int64_t plane_elem(int64_t N, int B, int bpb, int64_t t, int l) {
    const int k = l / bpb;
    return (int64_t)k * N * bpb + t * min(bpb, B - k * bpb) + (l - k * bpb);
}
__global__ void k_widen(int64_t D, int64_t N, int B, const float *in, int bpb_in, double *out, int bpb_out) {
    const int64_t n = D * N * B;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(k % B);
        const int64_t it = k / B, t = it % N, base = (it / N) * N * B;
        out[base + plane_elem(N, B, bpb_out, t, l)] = static_cast<double>(in[base + plane_elem(N, B, bpb_in, t, l)]);
    }
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
    out[c] = ld(g, g_elem(v, dir, c, band)) + v.Cw[band] * theta_prev(v)[c];
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
// Two sums over a workgroup in one LDS exchange (fixed order: lanes, then
// waves; every thread adds the wave sums itself).  The barrier orders LDS
// only, so global loads issued before it stay in flight.  lds holds 2 x 16.
__device__ __forceinline__ void block_sum2(double &a, double &b, double *lds) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if (lane == 0) {
        lds[2 * wv] = a;
        lds[2 * wv + 1] = b;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    double sa = 0.0, sb = 0.0;
    for (int k = 0; k < nw; ++k) {
        sa += lds[2 * k];
        sb += lds[2 * k + 1];
    }
    a = sa;
    b = sb;
}

// three sums (the flag and the two partial sums of a CG launch) the same way
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *lds) {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if (lane == 0) {
        lds[3 * wv] = a;
        lds[3 * wv + 1] = b;
        lds[3 * wv + 2] = c;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    double sa = 0.0, sb = 0.0, sc = 0.0;
    for (int k = 0; k < nw; ++k) {
        sa += lds[3 * k];
        sb += lds[3 * k + 1];
        sc += lds[3 * k + 2];
    }
    a = sa;
    b = sb;
    c = sc;
}

// ELL widths of the multi-workgroup CG (slots per row = faces + 1, rounded up
// to one of 4, 5, 7, 8: triangles, quadrilaterals and tetrahedra, hexahedra,
// anything up to seven faces); every slot of a row is read, so the width is a
// template parameter and no padding slot is loaded
template <int W>
__device__ __forceinline__ double ell_row(const PcgWork &w, int64_t n, int64_t r, const double *x) {
    int c[W];
    double e[W];
#pragma unroll
    for (int s = 0; s < W; ++s)
        c[s] = w.ecol[s * n + r], e[s] = w.eval[s * n + r];
    double au = 0.0;
#pragma unroll
    for (int s = 0; s < W; ++s)
        au += e[s] * x[c[s]];
    return au;
}
__device__ __forceinline__ double ell_row_any(const PcgWork &w, int64_t n, int64_t r, const double *x) {
    switch (w.ell_w) {
        case 4: return ell_row<4>(w, n, r, x);
        case 5: return ell_row<5>(w, n, r, x);
        case 7: return ell_row<7>(w, n, r, x);
        default: return ell_row<8>(w, n, r, x);
    }
}

__global__ void __launch_bounds__(256) k_cg1_init(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk,
                                                  int mode) {
    __shared__ double lds[32];
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
        const double au = ell_row_any(w, n, r, b);
        x[r] = 0.0;
        r0[r] = bi;
        w0[r] = au;
        s1[r] = 0.0;
        pp[r] = 0.0;
        ga += bi * u;
        de += au * u;
    }
    block_sum2(ga, de, lds);
    if (threadIdx.x == 0) {
        w.partial[it.b] = ga;
        w.partial[w.nblk + it.b] = de;
        if (it.b == 0) {
            w.scal[4] = 0.0;
            w.scal[5] = 0.0;
        }
    }
}

// One iteration of the single-reduction (Chronopoulos-Gear) Jacobi-PCG per
// launch: the launch boundary is the only grid-wide synchronisation.  Every
// load a row needs (its vectors, its ELL row and the gathered neighbour
// values) is issued before the reduction of the previous launch's partial
// sums, so the launch costs about two memory round trips.
template <int W>
__device__ __forceinline__ void cg1_iter_rows(const DeviceView &v, const WorkItem &it, int mode, int k, double rtol2_o,
                                              int max_o, double *lds) {
    const PcgWork &w = v.pcg;
    const int max_iter = max_o >= 0 ? max_o : w.max_iter;
    if (k >= max_iter) return;
    const double rtol2 = rtol2_o >= 0 ? rtol2_o : w.rtol2;
    const int64_t n = w.n;
    const int cur = k & 1, nxt = cur ^ 1;
    const double *pin = w.partial + cur * 2 * w.nblk;
    double *pout = w.partial + nxt * 2 * w.nblk;
    const double *rk = w.vec + cur * n, *wk_ = w.vec + (2 + cur) * n, *sk1 = w.vec + (4 + nxt) * n;
    double *rn = w.vec + nxt * n, *wn = w.vec + (2 + nxt) * n, *sk = w.vec + (4 + cur) * n, *pp = w.vec + 6 * n;
    double *x = pcg_x(v, mode);
    const int64_t stride = (int64_t)w.nblk * blockDim.x;
    const int64_t r0 = (int64_t)it.b * blockDim.x + threadIdx.x;

    // loads: the stop flag, partial sums, scalars, and the first row with its
    // neighbours.  The flag may be set by workgroup 0 of this very launch
    // (when it converges), so waves can read different values: the decision
    // is taken from the workgroup's sum of the flags, after the exchange.
    double flag = w.scal[4] != 0.0 ? 1.0 : 0.0;
    double gamma = threadIdx.x < (unsigned)w.nblk ? pin[threadIdx.x] : 0.0;
    double delta = threadIdx.x < (unsigned)w.nblk ? pin[w.nblk + threadIdx.x] : 0.0;
    const double gamma0_s = w.scal[1], alpha_old = w.scal[6 + 2 * nxt], gamma_old = w.scal[7 + 2 * nxt];
    const bool have = r0 < n;
    const int64_t ra = have ? r0 : 0;
    double d_rk = rk[ra], d_wk = wk_[ra], d_sk1 = sk1[ra], d_pp = pp[ra], d_di = w.dinv[ra], d_x = x[ra];
    int c[W];
    double e[W], gr[W], gw[W], gs[W];
#pragma unroll
    for (int s = 0; s < W; ++s)
        c[s] = w.ecol[s * n + ra], e[s] = w.eval[s * n + ra];
#pragma unroll
    for (int s = 0; s < W; ++s)
        gr[s] = rk[c[s]], gw[s] = wk_[c[s]], gs[s] = sk1[c[s]];
    block_sum3(flag, gamma, delta, lds);
    if (flag != 0.0) return;
    const double gamma0 = k == 0 ? gamma : gamma0_s;
    if (!(gamma > rtol2 * gamma0)) {   // converged (or zero right-hand side)
        if (it.b == 0 && threadIdx.x == 0) w.scal[4] = 1.0;
        return;
    }
    double alpha, beta;
    if (k == 0) {
        beta = 0.0;
        alpha = gamma / delta;
    } else {
        beta = gamma / gamma_old;
        alpha = gamma / (delta - beta * gamma / alpha_old);
    }
    double ga = 0.0, de = 0.0;
    for (int64_t r = r0; r < n; r += stride) {
        if (r != r0) {   // further rows (meshes above nblk x blockDim cells)
            d_rk = rk[r], d_wk = wk_[r], d_sk1 = sk1[r], d_pp = pp[r], d_di = w.dinv[r], d_x = x[r];
#pragma unroll
            for (int s = 0; s < W; ++s)
                c[s] = w.ecol[s * n + r], e[s] = w.eval[s * n + r];
#pragma unroll
            for (int s = 0; s < W; ++s)
                gr[s] = rk[c[s]], gw[s] = wk_[c[s]], gs[s] = sk1[c[s]];
        }
        const double ui = d_di * d_rk;
        const double pi = ui + beta * d_pp;
        const double si = d_wk + beta * d_sk1;
        pp[r] = pi;
        sk[r] = si;
        x[r] = d_x + alpha * pi;
        const double ri = d_rk - alpha * si;
        rn[r] = ri;
        const double un = d_di * ri;
        double au = 0.0;
#pragma unroll
        for (int s = 0; s < W; ++s)
            au += e[s] * (gr[s] - alpha * (gw[s] + beta * gs[s]));
        wn[r] = au;
        ga += ri * un;
        de += au * un;
    }
    block_sum2(ga, de, lds + 48);
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

__global__ void __launch_bounds__(256) k_cg1_iter(const DeviceView *__restrict__ vs, const WorkItem *__restrict__ wk,
                                                  int mode, int k, double rtol2_o, int max_o) {
    __shared__ double lds[80];
    const WorkItem it = wk[blockIdx.x];
    const DeviceView &v = vs[it.solve];
    if (pcg_skip(v, mode)) return;
    switch (v.pcg.ell_w) {
        case 4: cg1_iter_rows<4>(v, it, mode, k, rtol2_o, max_o, lds); break;
        case 5: cg1_iter_rows<5>(v, it, mode, k, rtol2_o, max_o, lds); break;
        case 7: cg1_iter_rows<7>(v, it, mode, k, rtol2_o, max_o, lds); break;
        default: cg1_iter_rows<8>(v, it, mode, k, rtol2_o, max_o, lds); break;
    }
}

template <class T, int MI, int MODE, bool PL>
void dispatch_sweep_bpl(const DeviceView *vs, const WorkItem *wk, int n, int bpl, bool one, int block, size_t lds,
                        hipStream_t st) {
    dim3 grid(n);
    if (one) {
        switch (bpl) {
            case 1: hipLaunchKernelGGL((k_sweep<T, MI, 1, MODE, true, false, PL>), grid, dim3(block), lds, st, vs, wk); break;
            case 2: hipLaunchKernelGGL((k_sweep<T, MI, 2, MODE, true, false, PL>), grid, dim3(block), lds, st, vs, wk); break;
            case 4: hipLaunchKernelGGL((k_sweep<T, MI, 4, MODE, true, false, PL>), grid, dim3(block), lds, st, vs, wk); break;
            default: hipLaunchKernelGGL((k_sweep<T, MI, 8, MODE, true, false, PL>), grid, dim3(block), lds, st, vs, wk); break;
        }
        return;
    }
    switch (bpl) {
        case 1: hipLaunchKernelGGL((k_sweep<T, MI, 1, MODE, false, false, PL>), grid, dim3(block), lds, st, vs, wk); break;
        case 2: hipLaunchKernelGGL((k_sweep<T, MI, 2, MODE, false, false, PL>), grid, dim3(block), lds, st, vs, wk); break;
        default: hipLaunchKernelGGL((k_sweep<T, MI, 4, MODE, false, false, PL>), grid, dim3(block), lds, st, vs, wk); break;
    }
}

template <class T, int MODE, bool PL>
void dispatch_sweep_mi(const DeviceView *vs, const WorkItem *wk, int n, int maxin, int bpl, bool one, int block,
                       size_t lds, hipStream_t st) {
    if (maxin <= 2) dispatch_sweep_bpl<T, 2, MODE, PL>(vs, wk, n, bpl, one, block, lds, st);
    else if (maxin == 3) dispatch_sweep_bpl<T, 3, MODE, PL>(vs, wk, n, bpl, one, block, lds, st);
    else dispatch_sweep_bpl<T, 5, MODE, PL>(vs, wk, n, bpl, one, block, lds, st);
}

// second-order kernels: the general mode (LDS, ghosts and spilled values
// from HBM) with several lanes per cell, up to four bands per lane
template <class T, int MI, bool PL>
void dispatch_sweep_so2(const DeviceView *vs, const WorkItem *wk, int n, int bpl, int block, size_t lds,
                        hipStream_t st) {
    dim3 grid(n);
    switch (bpl) {
        case 1: hipLaunchKernelGGL((k_sweep<T, MI, 1, kModeSpill, false, true, PL>), grid, dim3(block), lds, st, vs, wk); break;
        case 2: hipLaunchKernelGGL((k_sweep<T, MI, 2, kModeSpill, false, true, PL>), grid, dim3(block), lds, st, vs, wk); break;
        default: hipLaunchKernelGGL((k_sweep<T, MI, 4, kModeSpill, false, true, PL>), grid, dim3(block), lds, st, vs, wk); break;
    }
}

template <class T, bool PL>
void dispatch_sweep(const DeviceView *vs, const WorkItem *wk, int n, int maxin, int bpl, bool one, int mode,
                    int block, size_t lds, hipStream_t st, bool order2) {
    if (order2) {
        if (maxin <= 2) dispatch_sweep_so2<T, 2, PL>(vs, wk, n, bpl, block, lds, st);
        else if (maxin == 3) dispatch_sweep_so2<T, 3, PL>(vs, wk, n, bpl, block, lds, st);
        else dispatch_sweep_so2<T, 5, PL>(vs, wk, n, bpl, block, lds, st);
        return;
    }
    if (mode == kModeLds) dispatch_sweep_mi<T, kModeLds, PL>(vs, wk, n, maxin, bpl, one, block, lds, st);
    else if (mode == kModeHbmGhost) dispatch_sweep_mi<T, kModeHbmGhost, PL>(vs, wk, n, maxin, bpl, one, block, lds, st);
    else dispatch_sweep_mi<T, kModeSpill, PL>(vs, wk, n, maxin, bpl, one, block, lds, st);
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

void launch_flux(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, int mode, hipStream_t st) {
    if (n <= 0) return;
    if (fp32) hipLaunchKernelGGL(k_flux<float>, dim3(n), dim3(256), 0, st, vs, wk, mode);
    else hipLaunchKernelGGL(k_flux<double>, dim3(n), dim3(256), 0, st, vs, wk, mode);
}

void launch_grad(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, int phase, hipStream_t st) {
    if (n <= 0) return;
    if (fp32) hipLaunchKernelGGL(k_grad<float>, dim3(n), dim3(256), 0, st, vs, wk, phase);
    else hipLaunchKernelGGL(k_grad<double>, dim3(n), dim3(256), 0, st, vs, wk, phase);
}

void launch_recon(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, int phase, hipStream_t st) {
    if (n <= 0) return;
    if (fp32) hipLaunchKernelGGL(k_recon<float>, dim3(n), dim3(256), 0, st, vs, wk, phase);
    else hipLaunchKernelGGL(k_recon<double>, dim3(n), dim3(256), 0, st, vs, wk, phase);
}

void launch_bicgstab(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, hipStream_t st) {
    if (n <= 0) return;
    if (fp32) hipLaunchKernelGGL(k_bicgstab<float>, dim3(n), dim3(1024), 0, st, vs, wk);
    else hipLaunchKernelGGL(k_bicgstab<double>, dim3(n), dim3(1024), 0, st, vs, wk);
}

void launch_post(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, hipStream_t st) {
    if (n <= 0) return;
    if (fp32) hipLaunchKernelGGL(k_post<float>, dim3(n), dim3(256), 0, st, vs, wk);
    else hipLaunchKernelGGL(k_post<double>, dim3(n), dim3(256), 0, st, vs, wk);
}

void launch_reduce(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, hipStream_t st) {
    if (n <= 0) return;
    if (fp32) hipLaunchKernelGGL(k_reduce<float>, dim3(n), dim3(256), 0, st, vs, wk);
    else hipLaunchKernelGGL(k_reduce<double>, dim3(n), dim3(256), 0, st, vs, wk);
}

void launch_wall_rhs(const DeviceView *vs, const WorkItem *wk, int n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_wall_rhs, dim3(n), dim3(256), 0, st, vs, wk);
}

void launch_update(const DeviceView *vs, const WorkItem *wk, int n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_update, dim3(n), dim3(256), 0, st, vs, wk);
}

void launch_accel_cols(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, hipStream_t st) {
    if (n <= 0) return;
    if (fp32) hipLaunchKernelGGL(k_accel_cols<float>, dim3(n), dim3(256), 0, st, vs, wk);
    else hipLaunchKernelGGL(k_accel_cols<double>, dim3(n), dim3(256), 0, st, vs, wk);
}

void launch_accel_solve(const DeviceView *vs, const WorkItem *wk, int n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_accel_solve, dim3(n), dim3(256), 0, st, vs, wk);
}

void launch_accel_mix(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, hipStream_t st) {
    if (n <= 0) return;
    if (fp32) hipLaunchKernelGGL(k_accel_mix<float>, dim3(n), dim3(256), 0, st, vs, wk);
    else hipLaunchKernelGGL(k_accel_mix<double>, dim3(n), dim3(256), 0, st, vs, wk);
}

void launch_finish(const DeviceView *vs, const WorkItem *wk, int n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_finish, dim3((n + 63) / 64), dim3(64), 0, st, vs, wk, n);
}


size_t sweep_lds_bytes(int max_levels, int gring, int ls, int slots, int es) {
    const SweepLdsLayout L = sweep_lds_layout(max_levels, gring, ls, es);
    return ((size_t)L.ring_off + (size_t)std::max(slots, 1) * ls) * es;
}

void launch_sweep(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, int maxin, int bpl, bool one, int mode,
                  int block, size_t lds_bytes, hipStream_t st, bool order2, bool planes) {
    if (n <= 0) return;
    if (bpl != 1 && bpl != 2 && bpl != 4 && bpl != 8) bpl = 1;
    if (fp32) {
        if (planes) dispatch_sweep<float, true>(vs, wk, n, maxin, bpl, one, mode, block, lds_bytes, st, order2);
        else dispatch_sweep<float, false>(vs, wk, n, maxin, bpl, one, mode, block, lds_bytes, st, order2);
    } else {
        if (planes) dispatch_sweep<double, true>(vs, wk, n, maxin, bpl, one, mode, block, lds_bytes, st, order2);
        else dispatch_sweep<double, false>(vs, wk, n, maxin, bpl, one, mode, block, lds_bytes, st, order2);
    }
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

__global__ void k_widen_flat(int64_t n, const float *in, double *out) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = static_cast<double>(in[k]);
}

void launch_widen_flat(int64_t n, const float *in, double *out, hipStream_t st) {
    if (n <= 0) return;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_widen_flat, dim3(grid), dim3(256), 0, st, n, in, out);
}

void launch_widen(int64_t D, int64_t N, int B, const float *in, int bpb_in, double *out, int bpb_out, hipStream_t st) {
    const int64_t n = D * N * B;
    if (n <= 0) return;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_widen, dim3(grid), dim3(256), 0, st, D, N, B, in, bpb_in, out, bpb_out);
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

// Staging buffer of the allocation-free distribution read: one FP64 value per
// cell, kDistributionScratchCells at most.  Every GPU the library runs on
// holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device
// address): the device address is looked up once per device, with that
// device current, and used everywhere instead.
static __device__ __align__(256) double scratch[kDistributionScratchCells];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t distribution_scratch(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace nbte

// HIP kernels (gfx950) of the steady BTE transport path.
//
// Storage convention: for every (direction i, cell c, band l) the library
// keeps g = e - C_l theta(c) / W, the part of the energy density that is not
// in equilibrium at the lattice temperature the sweep used (Methods, Eq. (11)
// gives the equilibrium C T_L / W).  Layout g[(i*N + c)*B + l]: the bands of
// one (direction, cell) are contiguous, so the lanes that share a cell read
// and write one contiguous run.  Arithmetic is FP64 everywhere; g is stored in
// FP64 or FP32.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/nbte.h"
#include "kernels.h"

namespace nbte {
namespace {

constexpr int kMaxFaces = 6;
constexpr int64_t kPcgBlockMaxRows = 65536;   // larger systems use the multi-workgroup PCG

template <class T>
__device__ __forceinline__ double ld(const T *p, int64_t k) {
    return static_cast<double>(p[k]);
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
// boundary inflow (lagged): one thread per (boundary face, band)
// --------------------------------------------------------------------------
template <class T>
__global__ void k_bc_inflow(DeviceView v, const double *theta_base) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= v.NBF * v.B) return;
    const int64_t bf = t / v.B;
    const int lam = (int)(t % v.B);
    const int D = v.D, B = v.B;
    const int64_t N = v.N;
    const int c = v.bf_owner[bf];
    const T *g = static_cast<const T *>(v.g);
    const double *sd = v.sdotS + bf * D;
    double *out = v.inflow + bf * D * B;
    const double cw = v.Cw[lam];
    if (v.bf_kind[bf] == NBTE_BC_THERMALIZING) {
        const double val = cw * v.bf_thw[bf];
        for (int i = 0; i < D; ++i)
            if (sd[i] < 0.0) out[i * B + lam] = val;
        return;
    }
    const double eq = cw * theta_base[c];
    const double p = v.bf_p[bf];
    double diff = 0.0;
    if (p < 1.0) {
        for (int j = 0; j < D; ++j)
            if (sd[j] > 0.0) diff += v.w[j] * sd[j] * (ld(g, ((int64_t)j * N + c) * B + lam) + eq);
        diff /= v.win[bf];
    }
    const int32_t *mir = v.mirror + bf * D;
    for (int i = 0; i < D; ++i) {
        if (!(sd[i] < 0.0)) continue;
        double val = (1.0 - p) * diff;
        if (p > 0.0) val += p * (ld(g, ((int64_t)mir[i] * N + c) * B + lam) + eq);
        out[i * B + lam] = val;
    }
}

// --------------------------------------------------------------------------
// transport sweep: one workgroup per (band block, direction)
//
// For cell c of direction i, in upwind level order (Methods, Eqs. (4), (13)):
//   e_c = (e0_l/tau_l + S_l + v_l sum_{a<0} |a| e_up) / (1/tau_l + v_l sum_{a>0} a),
//   a = (s_i . S_cf) / V_c,
// e_up = value of the upwind neighbour computed earlier in this sweep, or the
// boundary inflow.  Neighbour values are staged in LDS (FP64) in the slots the
// host assigned (interval allocation over levels); a value without a slot is
// read back from its stored copy in HBM.  Levels are separated by a workgroup
// barrier, which orders both the LDS and the HBM writes of level k before the
// reads of level k+1.
// --------------------------------------------------------------------------
template <class T, int BPL>
__global__ void __launch_bounds__(1024) k_sweep(DeviceView v, const double *__restrict__ theta, int lpc,
                                                 int bands_per_block) {
    extern __shared__ double ring[];   // ring[slot * bands_per_block + local band]
    const int i = blockIdx.y;
    const int b0 = blockIdx.x * bands_per_block;
    const int slot = threadIdx.x / lpc;
    const int lane = threadIdx.x % lpc;
    const int nslots = blockDim.x / lpc;
    const int64_t N = v.N;
    const int F = v.F, B = v.B, D = v.D;
    const double sx = v.dirs[3 * i], sy = v.dirs[3 * i + 1], sz = v.dirs[3 * i + 2];
    T *gi = static_cast<T *>(v.g) + (int64_t)i * N * B;
    const int32_t *perm = v.perm + (int64_t)i * N;
    const int32_t *slot_i = v.slot ? v.slot + (int64_t)i * N : nullptr;
    const int32_t *lp = v.lvl_ptr + v.lvl_off[i];
    const int nlev = v.lvl_off[i + 1] - v.lvl_off[i] - 1;
    const int nb_here = min(B, b0 + bands_per_block) - b0;

    for (int l = 0; l < nlev; ++l) {
        const int kend = lp[l + 1];
        for (int k = lp[l] + slot; k < kend; k += nslots) {
            const int c = perm[k];
            double a[kMaxFaces];
            int nb[kMaxFaces];
            int ref[kMaxFaces];
            double sum_out = 0.0;
            const double iv = v.invV[c];
            for (int f = 0; f < F; ++f) {
                const double *S = v.S + ((int64_t)c * F + f) * 3;
                a[f] = (sx * S[0] + sy * S[1] + sz * S[2]) * iv;
                nb[f] = v.nbr[(int64_t)c * F + f];
                ref[f] = (a[f] < 0.0 && nb[f] >= 0 && slot_i) ? slot_i[nb[f]] : -1;
                if (a[f] > 0.0) sum_out += a[f];
            }
            const int mine = slot_i ? slot_i[c] : -1;
            const double th = theta[c];
            const double Qc = v.Q[c];
#pragma unroll
            for (int j = 0; j < BPL; ++j) {
                const int lb = lane * BPL + j;
                if (lb >= nb_here) break;
                const int lam = b0 + lb;
                const double cw = v.Cw[lam];
                const double itau = v.inv_tau[lam];
                double gain = 0.0;
                for (int f = 0; f < F; ++f) {
                    if (!(a[f] < 0.0)) continue;
                    const int n = nb[f];
                    double up;
                    if (n >= 0)
                        up = ref[f] >= 0 ? ring[ref[f] * bands_per_block + lb]
                                         : ld(gi, (int64_t)n * B + lam) + cw * theta[n];
                    else
                        up = v.inflow[((int64_t)(-n - 1) * D + i) * B + lam];
                    gain -= a[f] * up;
                }
                const double vel = v.vel[lam];
                const double e = (cw * th * itau + Qc * v.src[lam] + vel * gain) / (itau + vel * sum_out);
                gi[(int64_t)c * B + lam] = static_cast<T>(e - cw * th);
                if (mine >= 0) ring[mine * bands_per_block + lb] = e;
            }
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// net heat flow through each boundary face: one 64-lane block per face
//   J_f = sum_l v_l sum_i w_i (s_i . S_f) e_up
// --------------------------------------------------------------------------
template <class T>
__global__ void k_wall_flux(DeviceView v, const double *theta) {
    const int64_t bf = blockIdx.x;
    if (bf >= v.NBF) return;
    const int D = v.D, B = v.B;
    const int64_t N = v.N;
    const int c = v.bf_owner[bf];
    const T *g = static_cast<const T *>(v.g);
    double acc = 0.0;
    for (int t = threadIdx.x; t < D * B; t += 64) {
        const int i = t / B, lam = t % B;
        const double sd = v.sdotS[bf * D + i];
        if (sd == 0.0) continue;
        double e;
        if (sd > 0.0)
            e = ld(g, ((int64_t)i * N + c) * B + lam) + v.Cw[lam] * theta[c];
        else
            e = v.inflow[(bf * D + i) * B + lam];
        acc += v.vel[lam] * v.w[i] * sd * e;
    }
    acc = wave_sum(acc);
    if (threadIdx.x == 0) v.Jw[bf] = acc;
}

// --------------------------------------------------------------------------
// band x direction reductions (Methods, Eqs. (5), (7); T = energy temperature)
// lpc lanes per cell, FP64 accumulation, shuffle reduction over the lanes.
// Optionally the V-weighted right-hand side of the synthetic correction:
//   V (Qdot - D_h' q) = V beta (theta_seq - theta) + sum_{reflective f} J_f
// (collision-divergence identity; reflective walls carry zero net flux at the
// fixed point, so their transient flux is returned to the cell).
// --------------------------------------------------------------------------
template <class T>
__global__ void k_moments(DeviceView v, const double *theta, double beta, double C_tot, const double *V,
                          const double *qbias, double *theta_seq, double *thetaE, double *q, double *rhs_dsa,
                          int lpc) {
    const int64_t c = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / lpc;
    const int lane = threadIdx.x % lpc;
    const int64_t N = v.N;
    const int B = v.B, D = v.D;
    const T *g = static_cast<const T *>(v.g);
    double a_tau = 0, a_w = 0, qx = 0, qy = 0, qz = 0;
    if (c < N) {
        for (int lam = lane; lam < B; lam += lpc) {
            double sw = 0, s_x = 0, s_y = 0, s_z = 0;
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
    if (c < N && lane == 0) {
        const double th = theta[c];
        theta_seq[c] = th + a_tau / beta;
        thetaE[c] = th + a_w / C_tot;
        q[3 * c] = qx + th * qbias[0];
        q[3 * c + 1] = qy + th * qbias[1];
        q[3 * c + 2] = qz + th * qbias[2];
        if (rhs_dsa) {
            double r = V[c] * a_tau;
            for (int f = 0; f < v.F; ++f) {
                const int n = v.nbr[c * v.F + f];
                if (n < 0 && v.bf_kind[-n - 1] != NBTE_BC_THERMALIZING) r += v.Jw[-n - 1];
            }
            rhs_dsa[c] = r;
        }
    }
}

__device__ __forceinline__ unsigned long long dbits(double x) {
    return static_cast<unsigned long long>(__double_as_longlong(x));
}

__global__ void k_update(int64_t N, const double *base, const double *delta, const double *theta_old,
                         double *theta_new, unsigned long long *maxbuf) {
    double md = 0.0, mt = 0.0;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x) {
        const double tn = base[c] + (delta ? delta[c] : 0.0);
        theta_new[c] = tn;
        const double d = fabs(tn - theta_old[c]);
        if (!(d <= 1e300)) md = INFINITY;   // NaN or overflow: report as divergence
        else md = fmax(md, d);
        mt = fmax(mt, fabs(tn));
    }
    for (int off = 32; off > 0; off >>= 1) {
        md = fmax(md, __shfl_xor(md, off));
        mt = fmax(mt, __shfl_xor(mt, off));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&maxbuf[0], dbits(md));
        atomicMax(&maxbuf[1], dbits(mt));
    }
}

__global__ void k_reset_max(unsigned long long *maxbuf) {
    if (threadIdx.x < 2) maxbuf[threadIdx.x] = 0ull;
}

__global__ void k_affine(int64_t n, const double *in, double scale, double offset, double *out) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) out[k] = offset + scale * in[k];
}

template <class T>
__global__ void k_distribution(DeviceView v, const double *theta_base, int band, int dir, double *out) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= v.N) return;
    const T *g = static_cast<const T *>(v.g);
    out[c] = ld(g, ((int64_t)dir * v.N + c) * v.B + band) + v.Cw[band] * theta_base[c];
}

// --------------------------------------------------------------------------
// Jacobi PCG: two launches per iteration, every block re-sums the per-block
// partials in the same order, so all blocks see identical scalars and the
// result is bitwise reproducible.
// --------------------------------------------------------------------------
// The converged flag is read once per block and broadcast through LDS, so
// every thread of a block takes the same early exit (a block-uniform return
// before any barrier).
__device__ bool block_flag_set(const double *flag, double *lds) {
    __syncthreads();
    if (threadIdx.x == 0) lds[15] = *flag;
    __syncthreads();
    const bool set = lds[15] != 0.0;
    __syncthreads();
    return set;
}

__device__ double sum_partials(const double *p, int n, double *lds) {
    double x = (threadIdx.x < (unsigned)n) ? p[threadIdx.x] : 0.0;
    return block_sum(x, lds);
}

__global__ void k_pcg_init(PcgWork w, const double *b, double *x, double *prz) {
    __shared__ double lds[16];
    double acc = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < w.n; r += (int64_t)gridDim.x * blockDim.x) {
        const double bi = b[r];
        x[r] = 0.0;
        w.r[r] = bi;
        const double zi = w.dinv[r] * bi;
        w.z[r] = zi;
        acc += bi * zi;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) prz[blockIdx.x] = acc;
}

__global__ void k_pcg_rz0(PcgWork w, const double *prz) {
    __shared__ double lds[16];
    const double rz0 = sum_partials(prz, w.nblk, lds);
    if (threadIdx.x == 0) {
        w.scal[1] = rz0;
        w.scal[4] = 0.0;   // converged flag, sticky once set
        w.scal[5] = 0.0;
    }
}

// iteration k, part 1: beta, p = z + beta p, Ap = A z + beta Ap, partial p.Ap
__global__ void k_pcg_dir(PcgWork w, const double *prz_new, const double *prz_old, double *ppap, int k,
                          double rtol2) {
    __shared__ double lds[16];
    if (block_flag_set(&w.scal[4], lds)) return;
    const double rz = sum_partials(prz_new, w.nblk, lds);
    const double rz0 = w.scal[1];
    if (!(rz > rtol2 * rz0)) {   // converged (or zero right-hand side)
        if (blockIdx.x == 0 && threadIdx.x == 0) w.scal[4] = 1.0;
        return;
    }
    const double beta = (k == 0) ? 0.0 : rz / sum_partials(prz_old, w.nblk, lds);
    double acc = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < w.n; r += (int64_t)gridDim.x * blockDim.x) {
        double az = 0.0;
        for (int32_t kk = w.row_ptr[r]; kk < w.row_ptr[r + 1]; ++kk) az += w.val[kk] * w.z[w.col[kk]];
        const double pn = (k == 0) ? w.z[r] : w.z[r] + beta * w.p[r];
        const double apn = (k == 0) ? az : az + beta * w.Ap[r];
        w.p[r] = pn;
        w.Ap[r] = apn;
        acc += pn * apn;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) ppap[blockIdx.x] = acc;
}

// iteration k, part 2: alpha, x += alpha p, r -= alpha Ap, z = M^-1 r, partial r.z
__global__ void k_pcg_step(PcgWork w, const double *prz_new, const double *ppap, double *prz_next, double *x,
                           int k, double rtol2) {
    __shared__ double lds[16];
    if (block_flag_set(&w.scal[4], lds)) return;
    const double rz = sum_partials(prz_new, w.nblk, lds);
    const double rz0 = w.scal[1];
    if (!(rz > rtol2 * rz0)) return;
    const double alpha = rz / sum_partials(ppap, w.nblk, lds);
    double acc = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < w.n; r += (int64_t)gridDim.x * blockDim.x) {
        x[r] += alpha * w.p[r];
        const double rn = w.r[r] - alpha * w.Ap[r];
        w.r[r] = rn;
        const double zn = w.dinv[r] * rn;
        w.z[r] = zn;
        acc += rn * zn;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) {
        prz_next[blockIdx.x] = acc;
        if (blockIdx.x == 0) w.scal[5] = k + 1;
    }
}

// Whole PCG in one workgroup (small systems): no launch per iteration, the
// reductions are workgroup reductions in a fixed order (deterministic).
// Every thread owns rows tid, tid + blockDim, ...; only the SpMV reads other
// threads' entries of p, and p is complete at the barrier before it.
__global__ void __launch_bounds__(1024) k_pcg_block(PcgWork w, const double *b, double *x, double rtol2,
                                                    int max_iter) {
    __shared__ double lds[16];
    const int64_t n = w.n;
    const int nt = blockDim.x;
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += nt) {
        const double bi = b[r];
        x[r] = 0.0;
        w.r[r] = bi;
        const double zi = w.dinv[r] * bi;
        w.z[r] = zi;
        w.p[r] = zi;
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
                for (int32_t k = w.row_ptr[r]; k < w.row_ptr[r + 1]; ++k) ap += w.val[k] * w.p[w.col[k]];
                w.Ap[r] = ap;
                acc += w.p[r] * ap;
            }
            const double alpha = rz / block_sum(acc, lds);
            acc = 0.0;
            for (int64_t r = threadIdx.x; r < n; r += nt) {
                x[r] += alpha * w.p[r];
                const double rn = w.r[r] - alpha * w.Ap[r];
                w.r[r] = rn;
                const double zn = w.dinv[r] * rn;
                w.z[r] = zn;
                acc += rn * zn;
            }
            const double rz_new = block_sum(acc, lds);
            if (!(rz_new > rtol2 * rz0)) { ++it; break; }
            const double beta = rz_new / rz;
            rz = rz_new;
            for (int64_t r = threadIdx.x; r < n; r += nt) w.p[r] = w.z[r] + beta * w.p[r];
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        w.scal[1] = rz0;
        w.scal[5] = it;
    }
}

template <class T>
void dispatch_sweep(const DeviceView &v, const double *theta, int bpb, int bpl, int block, int lds_slots,
                    hipStream_t st) {
    // the caller guarantees bpb <= 64 * bpl (at most 64 lanes per cell)
    int lanes = (bpb + bpl - 1) / bpl;
    int lpc = 1;
    while (lpc < lanes) lpc <<= 1;
    const int nbb = (v.B + bpb - 1) / bpb;
    if (block % 64 != 0 || block < 64 || block > 1024) block = 256;
    if (block < lpc) block = lpc;
    const size_t lds = v.slot ? (size_t)lds_slots * bpb * sizeof(double) : 0;
    dim3 grid(nbb, v.D);
    switch (bpl) {
        case 1: hipLaunchKernelGGL((k_sweep<T, 1>), grid, dim3(block), lds, st, v, theta, lpc, bpb); break;
        case 2: hipLaunchKernelGGL((k_sweep<T, 2>), grid, dim3(block), lds, st, v, theta, lpc, bpb); break;
        case 4: hipLaunchKernelGGL((k_sweep<T, 4>), grid, dim3(block), lds, st, v, theta, lpc, bpb); break;
        case 8: hipLaunchKernelGGL((k_sweep<T, 8>), grid, dim3(block), lds, st, v, theta, lpc, bpb); break;
        default: hipLaunchKernelGGL((k_sweep<T, 16>), grid, dim3(block), lds, st, v, theta, lpc, bpb); break;
    }
}

int lanes_for(int B) {
    int lpc = 1;
    while (lpc < B && lpc < 64) lpc <<= 1;
    return lpc;
}

}  // namespace

void launch_fill_zero(void *p, size_t bytes, hipStream_t st) {
    const size_t n = bytes / 4;
    if (n == 0) return;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, st, static_cast<uint32_t *>(p), n);
}

void launch_bc_inflow(const DeviceView &v, bool fp32, const double *theta_base, hipStream_t st) {
    const int64_t n = v.NBF * v.B;
    if (n == 0) return;
    dim3 grid((unsigned)((n + 255) / 256));
    if (fp32) hipLaunchKernelGGL(k_bc_inflow<float>, grid, dim3(256), 0, st, v, theta_base);
    else hipLaunchKernelGGL(k_bc_inflow<double>, grid, dim3(256), 0, st, v, theta_base);
}

void launch_sweep(const DeviceView &v, bool fp32, const double *theta, int bpb, int bpl, int block, int lds_slots,
                  hipStream_t st) {
    if (bpl != 1 && bpl != 2 && bpl != 4 && bpl != 8 && bpl != 16) bpl = 1;
    if (bpb < 1) bpb = 1;
    if (fp32) dispatch_sweep<float>(v, theta, bpb, bpl, block, lds_slots, st);
    else dispatch_sweep<double>(v, theta, bpb, bpl, block, lds_slots, st);
}

void launch_wall_flux(const DeviceView &v, bool fp32, const double *theta, hipStream_t st) {
    if (v.NBF == 0) return;
    if (fp32) hipLaunchKernelGGL(k_wall_flux<float>, dim3((unsigned)v.NBF), dim3(64), 0, st, v, theta);
    else hipLaunchKernelGGL(k_wall_flux<double>, dim3((unsigned)v.NBF), dim3(64), 0, st, v, theta);
}

void launch_moments(const DeviceView &v, bool fp32, const double *theta, double beta, double C_tot,
                    const double *V, const double *qbias, double *theta_seq, double *thetaE, double *q,
                    double *rhs_dsa, hipStream_t st) {
    const int lpc = lanes_for(v.B);
    const int block = 256;
    const int64_t threads = v.N * lpc;
    dim3 grid((unsigned)((threads + block - 1) / block));
    if (fp32)
        hipLaunchKernelGGL(k_moments<float>, grid, dim3(block), 0, st, v, theta, beta, C_tot, V, qbias, theta_seq,
                           thetaE, q, rhs_dsa, lpc);
    else
        hipLaunchKernelGGL(k_moments<double>, grid, dim3(block), 0, st, v, theta, beta, C_tot, V, qbias, theta_seq,
                           thetaE, q, rhs_dsa, lpc);
}

void launch_update(int64_t N, const double *base, const double *delta, const double *theta_old, double *theta_new,
                   unsigned long long *maxbuf, hipStream_t st) {
    const int grid = (int)std::min<int64_t>((N + 255) / 256, 1024);
    hipLaunchKernelGGL(k_update, dim3(grid), dim3(256), 0, st, N, base, delta, theta_old, theta_new, maxbuf);
}

void launch_reset_max(unsigned long long *maxbuf, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_max, dim3(1), dim3(64), 0, st, maxbuf);
}

void launch_affine(int64_t n, const double *in, double scale, double offset, double *out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_affine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, in, scale, offset, out);
}

void launch_distribution(const DeviceView &v, bool fp32, const double *theta_base, int band, int dir, double *out,
                         hipStream_t st) {
    dim3 grid((unsigned)((v.N + 255) / 256));
    if (fp32) hipLaunchKernelGGL(k_distribution<float>, grid, dim3(256), 0, st, v, theta_base, band, dir, out);
    else hipLaunchKernelGGL(k_distribution<double>, grid, dim3(256), 0, st, v, theta_base, band, dir, out);
}

void launch_pcg(const PcgWork &w, const double *b, double *x, double rtol, int max_iter, hipStream_t st) {
    if (w.n <= kPcgBlockMaxRows) {
        hipLaunchKernelGGL(k_pcg_block, dim3(1), dim3(1024), 0, st, w, b, x, rtol * rtol, max_iter);
        return;
    }
    double *prz[2] = {w.partial, w.partial + w.nblk};
    double *ppap = w.partial + 2 * w.nblk;
    const double rtol2 = rtol * rtol;
    hipLaunchKernelGGL(k_pcg_init, dim3(w.nblk), dim3(256), 0, st, w, b, x, prz[0]);
    hipLaunchKernelGGL(k_pcg_rz0, dim3(1), dim3(256), 0, st, w, prz[0]);
    for (int k = 0; k < max_iter; ++k) {
        hipLaunchKernelGGL(k_pcg_dir, dim3(w.nblk), dim3(256), 0, st, w, prz[k & 1], prz[(k + 1) & 1], ppap, k,
                           rtol2);
        hipLaunchKernelGGL(k_pcg_step, dim3(w.nblk), dim3(256), 0, st, w, prz[k & 1], ppap, prz[(k + 1) & 1], x, k,
                           rtol2);
    }
}

}  // namespace nbte

// Device kernels of the transport path and their host-side launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nbte {

// Everything the per-iteration kernels read, as raw device pointers.
struct DeviceView {
    int64_t N;       // cells
    int32_t F;       // faces per cell
    int32_t B;       // bands
    int32_t D;       // directions
    int64_t NBF;     // boundary faces
    // mesh
    const int32_t *nbr;     // N*F
    const double *S;        // N*F*3
    const double *invV;     // N
    // schedule
    const int32_t *perm;    // D*N
    const int32_t *lvl_ptr;
    const int32_t *lvl_off; // D+1
    // sweep program: level-ordered streams, index i*N + k (see SweepProgram)
    int32_t maxin;
    int32_t max_levels;     // deepest level count over the directions
    int32_t max_ghosts;     // most boundary inflow values (per band) of one level
    int64_t n_ghost;        // ghost rows over all directions
    const int32_t *gptr;    // ghost offsets per level (layout of lvl_ptr)
    const int64_t *ghost_src;  // inflow row of each ghost
    double *gval;           // ghost values in sweep order (n_ghost * B)
    const int32_t *p_cell, *p_slot, *p_ref;
    const double *p_coef, *p_sout;
    double *p_th;           // theta in level order, gathered every iteration
    double *p_q;            // heat source in level order, gathered at prepare
    const double *theta_cell;  // theta by cell (read only for values without an LDS slot)
    // bands: Cw = C/W, src = C/(C_tot W), v, inv_tau
    const double *Cw, *src, *vel, *inv_tau;
    // quadrature
    const double *dirs;     // D*3
    const double *w;        // D
    // boundary plan
    const int32_t *bf_owner, *bf_kind, *mirror;
    const double *bf_thw, *bf_p, *sdotS, *win;
    // state
    void *g;                // D*N*B, FP32 or FP64: non-equilibrium part e - C theta/W
    double *inflow;         // NBF*D*B
    double *Jw;             // NBF: net flux through each boundary face
    const double *Q;        // N
};

// Launchers (all asynchronous on `st`).  `fp32` selects the storage type of g.
void launch_fill_zero(void *p, size_t bytes, hipStream_t st);
void launch_bc_inflow(const DeviceView &v, bool fp32, const double *theta_base, hipStream_t st);
// bands_per_block bands of one direction per workgroup, bands_per_lane per
// lane; lds_slots = slots per direction the schedule was assigned for.
// spill: some consumed values are read back from HBM (full fence per level)
// gcap: ghosts per level kept in LDS (the rest are read from HBM)
void launch_sweep(const DeviceView &v, bool fp32, const double *theta, int bands_per_block, int bands_per_lane,
                  int block, int lds_slots, int gcap, bool spill, hipStream_t st);
// ghost values of every direction in sweep order, from the boundary inflow
void launch_ghost_gather(const DeviceView &v, hipStream_t st);
// out[at] = in[p_cell[at]] for every stream position (theta or Q into level order)
void launch_gather(const DeviceView &v, const double *in, double *out, hipStream_t st);
void launch_wall_flux(const DeviceView &v, bool fp32, const double *theta, hipStream_t st);
void launch_moments(const DeviceView &v, bool fp32, const double *theta, double beta, double C_tot,
                    const double *V, const double *qbias, double *theta_seq, double *thetaE, double *q,
                    double *rhs_dsa, hipStream_t st);
// out[k] = offset + scale * in[k]
void launch_affine(int64_t n, const double *in, double scale, double offset, double *out, hipStream_t st);
// theta_new = base + delta (delta may be null), residual maxima into maxbuf[0..1]
// (as ordered uint64 bit patterns of non-negative doubles).
void launch_update(int64_t N, const double *base, const double *delta, const double *theta_old,
                   double *theta_new, unsigned long long *maxbuf, hipStream_t st);
void launch_reset_max(unsigned long long *maxbuf, hipStream_t st);
void launch_distribution(const DeviceView &v, bool fp32, const double *theta_base, int band, int dir,
                         double *out, hipStream_t st);

// Jacobi-preconditioned conjugate gradients on a symmetric positive definite
// CSR matrix, fixed launch sequence (capturable), deterministic reductions.
struct PcgWork {
    int64_t n;
    int nblk;
    const int32_t *row_ptr, *col;
    const double *val, *dinv;
    double *r, *z, *p, *Ap;
    double *partial;   // 2*nblk
    double *scal;      // [rz, rz0, alpha, beta, converged, iters]
};
void launch_pcg(const PcgWork &w, const double *b, double *x, double rtol, int max_iter, hipStream_t st);

}  // namespace nbte

// Device kernels of the transport path and their host-side launchers.
//
// Every per-iteration kernel serves a list of solves in one launch: it reads
// the solve's descriptor (DeviceView, device memory) through a work table of
// WorkItems, one per workgroup.  A single solve is a list of one.  The
// iteration state of each solve (theta rotation, iteration count, residual,
// stop flag) lives in device memory and is advanced by the kernels
// themselves, so one captured launch sequence serves every iteration.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

// Pointers in the descriptors are global-memory pointers.  Device code sees
// them qualified with the global address space, so loads through pointers
// read out of a descriptor compile to global (not flat) instructions: flat
// loads would also count against the LDS wait counter and serialise the
// sweep's prefetch pipeline.  Host code sees plain pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__)
#define NBTE_G __attribute__((address_space(1)))
#else
#define NBTE_G
#endif

namespace nbte {

// Iteration state of one solve (device memory).
struct SolveState {
    int32_t rot;          // theta rotation 0..2 (cur = (3 - rot) % 3, prev = cur + 1, spare = cur + 2, mod 3)
    int32_t iterations;   // iterations done
    int32_t done;         // 0 running; NBTE_DONE_* once stopped (kernels then skip the solve)
    int32_t stop;         // host: 1 = stop at tol / max_iter, 0 = run every launched iteration
    int32_t max_iter;
    int32_t patience;     // stop as STALLED after this many iterations without a 2% residual gain (0: off)
    double tol;           // residual tolerance
    double residual;      // max|theta_new - theta| / max|theta_new| of the last iteration
    double best;          // smallest residual so far (since the last controls were set)
    int32_t since;        // iterations since best improved by 2%
    int32_t pad;
    unsigned long long maxbuf[3];   // running maxima (ordered bit patterns): of the update, of the new
                                    // theta, and (second order) of the distribution in temperature units
};
enum { NBTE_DONE_CONVERGED = 1, NBTE_DONE_MAX_ITER = 2, NBTE_DONE_DIVERGED = 3, NBTE_DONE_STALLED = 4 };

// Jacobi-preconditioned conjugate gradients on a symmetric positive definite
// CSR matrix (the synthetic correction); per-solve work arrays.
struct PcgWork {
    int64_t n;
    int32_t nblk;         // workgroups of the multi-workgroup form
    int32_t max_iter;
    double rtol2;         // stop when r.z <= rtol2 * r0.z0
    const int32_t NBTE_G *row_ptr, *col;
    const double NBTE_G *val, *dinv;
    // the same matrix as ELL columns for the multi-workgroup form: slot s of
    // row r at s n + r, ell_w = 4, 5, 7 or 8 slots (the longest row rounded
    // up; every slot is read: no per-slot branch splits the loads), values
    // pre-scaled by the column's Jacobi factor (A D^-1); unused slots hold the
    // row itself with value 0
    int32_t ell_w;
    const int32_t NBTE_G *ecol;
    const double NBTE_G *eval;
    double NBTE_G *vec;          // 7 n: block form r, z, p, Ap; multi form r[2], w[2], s[2], p
    double NBTE_G *partial;      // 4 * nblk: per parity the r.u and w.u partial sums
    double NBTE_G *scal;         // [-, r0.u0, -, -, converged flag, iterations, alpha/gamma per parity (6..9)]
};

// Anderson acceleration of the outer iteration (an addition to the method: it
// changes the path of the iteration, not its fixed point).  The state of the
// iteration is x = (theta, inflow): the lattice temperature (N values) and the
// boundary inflow of every incoming (face, direction) row and band (NR = rows
// x B values) in temperature units, e W / C_l.  After an iteration has formed
// its image G(x) (the new theta and the inflow of the new distribution),
//   f = G(x) - x,  dF_j = f_{j+1} - f_j,  dG_j = G_{j+1} - G_j  (last m steps),
//   gamma = argmin || f - dF gamma ||,   x_next = G(x) - dG gamma.
// Per-solve work arrays; the state vectors are [theta part | inflow part].
struct AccelWork {
    int32_t m;                   // depth (columns kept); 0 = off
    int32_t nblk;                // workgroups of the state-length launches
    // inflow entries: the incoming (face, direction) rows of the faces whose
    // inflow depends on the distribution (a thermalizing face's is fixed: its
    // entries would be exact zeros in every column) x bands
    int64_t NR;
    const int32_t NBTE_G *in;    // NBF*D: row in the inflow entries of an incoming (face, direction), else -1
    double NBTE_G *ain_x;        // NR: inflow of the current iterate x (temperature units)
    double NBTE_G *ain_G;        // 2 NR: inflow of its image G(x), step k's in half k mod 2 (the previous step's is kept)
    void NBTE_G *fprev;          // N + NR: f of the previous step, in the storage type (a residual: no cancellation)
    double NBTE_G *Gprev;        // N: the temperature part of G of the previous step (then of this step)
    void NBTE_G *dF, *dG;        // m (N + NR) each, in the storage type: column j at j (N + NR)
    double NBTE_G *part;         // nblk x 2m partial sums of a step
    double NBTE_G *scal;         // [0] steps done; [1..m*m] Gram matrix dF_i . dF_j; then m gammas
};

// The reductions' first stage per (direction, cell): band sums of the
// distribution weighted by 1/tau, 1 and the group velocity, accumulated and
// kept in FP64 on both paths (the moments are small differences of the
// directions' sums; FP32 roundings of the sums measurably moved the mixed
// path's heat flux).
struct Mom3 {
    double a, w, u;
};

// Everything the kernels read and write of one solve, as raw device pointers.
struct DeviceView {
    int64_t N;       // cells
    int32_t F;       // faces per cell
    int32_t B;       // bands
    int32_t D;       // directions
    int32_t fp32;    // g stored in FP32 (else FP64)
    int64_t NBF;     // boundary faces
    int32_t scheme;  // NBTE_SCHEME_*
    int32_t mom_lpc; // lanes per cell of the cell-major reductions
    int32_t planes;  // distribution layout: 0 cell-major, 1 band-block planes in stream order
    // mesh
    const int32_t NBTE_G *nbr;     // N*F
    const double NBTE_G *V;        // N
    // sweep program: level-ordered streams, index i*N + k (see SweepProgram)
    int32_t maxin;
    int32_t max_levels;     // deepest level count over the directions
    int32_t lpc;            // sweep lanes per cell
    int32_t bpb;            // sweep bands per workgroup
    int32_t gcap;           // ghosts per level kept in LDS (the rest is read from HBM)
    int32_t gring;          // LDS ghost ring capacity (power of two)
    int32_t lstride;        // LDS stride (elements) of one staged value's bands: lpc x bands per lane
    const int32_t NBTE_G *lvl_ptr; // per direction L_i + 1 level offsets, concatenated
    const int32_t NBTE_G *lvl_off; // D+1: start of direction i's entries in lvl_ptr
    const int32_t NBTE_G *gptr;    // ghost offsets per level (layout of lvl_ptr)
    // p_slot = p_cell + D N and p_ref = p_cell + 2 D N (rows of one array);
    // likewise t_dc = t_sout + D N, t_q = t_sout + 2 D N, t_coef = t_sout + 3 D N
    const int32_t NBTE_G *p_cell, *p_slot, *p_ref;
    const int32_t NBTE_G *p_upc;   // maxin*D*N: upwind cell of each reference (the cell itself for inflow)
    // in the storage type T of g (FP64, or FP32 for the mixed path):
    // coefficients |a|, outflow sums, heat source (gathered at prepare) and
    // the equilibrium-imbalance term D (every iteration)
    const void NBTE_G *t_coef, *t_sout, *t_q;
    void NBTE_G *t_dc;
    // bands: Cw = C/W, src = C/(C_tot W), v, inv_tau
    const double NBTE_G *Cw, *src, *vel, *inv_tau;
    double beta, C_tot;     // sum C/tau, sum C
    // quadrature
    const double NBTE_G *dirs;     // D*3
    const double NBTE_G *w;        // D
    const double NBTE_G *qbias;    // 3: q of a uniform unit equilibrium
    // boundary plan
    const int32_t NBTE_G *bf_owner, *bf_kind, *mirror;
    // cells owning a reflective face (the correction's wall term): n_wall
    // cells, ascending; their reflective faces' slots wall_ptr[k] ..
    // wall_ptr[k+1] in face order; wslot = slot of a reflective face (-1
    // for a thermalizing one)
    const int32_t NBTE_G *wall_cell, *wall_ptr, *wslot;
    int64_t n_wall;
    const int32_t NBTE_G *in_row;  // NBF*D: ghost row of an incoming (face, direction), -1 otherwise
    // lagged faces of cyclic upwind graphs (ghost rows filled from the previous
    // distribution): n_lag entries of (ghost row, direction, cell, upwind cell)
    int64_t n_lag;
    const int32_t NBTE_G *lag;
    const double NBTE_G *bf_thw, *bf_p, *sdotS, *win;
    // state
    // g: D*N*B, FP32 or FP64: non-equilibrium part e - C theta/W.
    // Cell-major layout: (i, c, l) at (i N + c) B + l.  Plane layout: per
    // direction in band-block planes (bpb bands; the last block may be
    // narrower), each plane in the direction's stream order: (i, c, l) at
    //   i N B + k N bpb + pos[i N + c] w_k + (l - k bpb),
    //   k = l / bpb,  w_k = min(bpb, B - k bpb)
    // so a sweep workgroup (direction, band block) writes one contiguous run
    // per pass
    void NBTE_G *g;
    const int32_t NBTE_G *pos;     // D*N: stream position of cell c in direction i (at i N + c)
    // plane layout only: boundary rows, the distribution of every cell that
    // owns a boundary face, row (k D + i) of B values in the storage
    // type, copied from the planes by the reductions' first stage for the
    // directions that leave through one of the cell's boundary faces (the
    // only ones the boundary inflow and flux read; the other rows keep
    // finite stale values or zeros, which those kernels select away); and
    // the first stage's per (direction, cell) band sums
    // (k: the cell's index among the cells that own a boundary face, in cell order)
    const int32_t NBTE_G *bf_brow; // NBF: k of the face's owner
    const int32_t NBTE_G *p_brow;  // D*N per stream position: the row k D + i its values are copied
                                   // into (the cell owns a boundary face direction i leaves through), or -1
    void NBTE_G *brow;             // n_bown D B values
    void NBTE_G *mom;              // D*N Mom3 triples: band sums of g weighted by 1/tau, 1 and v
    void NBTE_G *gval;             // n_ghost*B boundary inflow in sweep (ghost) order, type T, as the
                                   // deviation from equilibrium at the sweep's theta of the owner cell
    double NBTE_G *Jw;             // NBF: net flux through each boundary face
    double NBTE_G *Jin;            // NBF: its incoming part, from the inflow the stage wrote
    double NBTE_G *wallJ;          // J_f of the reflective faces in wall-slot order
    double NBTE_G *bsum;           // NBF*B: per band sum_out w (s.S) e of the last sweep
    double NBTE_G *theta[3];       // deviational lattice temperature, rotated by state->rot
    double NBTE_G *theta_seq, *thetaE, *q, *rhs, *delta;
    SolveState NBTE_G *state;
    PcgWork pcg;
    AccelWork acc;
    // second-order face values (order 2): least-squares weights, geometry, the
    // gradients of the last distribution, the deferred correction of the
    // coming sweep and the increments of the outgoing boundary face values
    int32_t order;
    const double NBTE_G *lsq;      // N*F*3: G_c = sum_f lsq_cf (e_n(f) - e_c)
    const double NBTE_G *Sv;       // N*F*3 outward area vectors
    const double NBTE_G *xf;       // N*F*3 face centroids
    const double NBTE_G *xc;       // N*3 cell centres (vertex average)
    const int32_t NBTE_G *bf_local;// NBF: the boundary face's index among its owner's faces
    void NBTE_G *grad;             // 3 planes of D*N*B, storage type: gradient components per system
    void NBTE_G *corr;             // D*N*B in stream order: -v sum_f a delta_f of the coming sweep
    void NBTE_G *bdelta;           // 2 slots of NBF*D*B: increments of the outgoing face values;
                                   // slot m & 1 belongs to the distribution of sweep m - 1
    // Jacobi-BiCGSTAB inner solver: 9 vectors of D*B*N FP64 values, system
    // (i B + l) at offset (i B + l) N of each; iteration cap and tolerance
    double NBTE_G *bicg;
    int32_t bicg_max_iter;
    double bicg_rtol;
    const double NBTE_G *Qc;       // N heat source per cell
};

// One workgroup's share of a launch: the solve (index into the descriptor
// array) and two kernel-specific coordinates (sweep: direction and band
// block; elementwise kernels: kind and local workgroup index).  solve < 0
// marks padding.
struct WorkItem {
    int32_t solve, a, b, c;
};

// Launchers (all asynchronous on `st`; `vs` and `wk` are device arrays).
void launch_fill_zero(void *p, size_t bytes, hipStream_t st);

// Work tables of the elementwise kernels: items (solve, kind, local block,
// blocks of this (solve, kind)), 256 threads each.
//   stage:   kind 0 = boundary inflow, one wave per boundary face;
//            kind 1 = equilibrium-imbalance term D of every stream entry;
//            kinds 2, 3 = the accelerated iteration's absolute inflow (below);
//            kind 4 = the ghost rows of lagged faces (grid-stride over rows x bands)
//   flux:    per-band outgoing sums and net flow, one wave per boundary face
//            (items (solve, -, b, nblk): faces b*4 + wave, strided by 4 nblk)
//   post:    cell-major layout: kind 0 = flux mode 0 face groups (as above),
//            kind 1 = band x direction reductions, mom_lpc lanes per cell,
//            item b = block b; plane layout: kind 2 = first stage of the
//            reductions, the band sums of one stream position per thread and
//            the boundary rows, item (solve, 2, chunk of 256 positions,
//            direction); solve < 0 pads
//   reduce:  plane layout: kind 0 = flux mode 0 face groups; kind 1 = second
//            stage of the reductions, the direction sums of every cell, the
//            moments and the correction's right-hand side (grid-stride over
//            the cells, kReduceLanes lanes per cell)
//   wall rhs: the reflective faces' net flows into the correction's
//            right-hand side (grid-stride over the cells that own one)
//   update:  theta update and residual maxima (grid-stride over the cells)
//   finish:  one thread per solve (a = solve); residual, stop test, rotation
void launch_stage(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, hipStream_t st);
// mode 0: inside the iteration (theta[cur] is the sweep's temperature): the
//         per-band outgoing sums of every reflective face and its net flow;
// mode 1: once the iteration has rotated theta (theta[prev] is): the net flow
//         of every face from the stored values;
// mode 2: at prepare: the outgoing sums of the initial distribution
void launch_flux(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, int mode, hipStream_t st);
void launch_post(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, hipStream_t st);
// Second-order scheme, after a sweep (phase 0), at prepare (phase 1) or after
// the rotation of a stopped iteration (phase 2): gradients of the stored
// distribution (items (solve, -, b, nblk), grid-stride over D*N*B), then the
// deferred correction of the next sweep (items (solve, 0, b, nblk)) and the
// outgoing increments of the boundary faces (items (solve, 1, b, nblk)).
void launch_grad(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, int phase, hipStream_t st);
void launch_recon(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, int phase, hipStream_t st);
void launch_reduce(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, hipStream_t st);
constexpr int kReduceLanes = 4;   // lanes per cell of reduction stage 2 (a power of two)
constexpr int64_t kPlanesMinValues = int64_t(1) << 26;   // auto layout: planes from 2^26 distribution values
void launch_wall_rhs(const DeviceView *vs, const WorkItem *wk, int n, hipStream_t st);
void launch_update(const DeviceView *vs, const WorkItem *wk, int n, hipStream_t st);
// Anderson step after an iteration's finish (solves with acc.m > 0; each
// kernel skips a solve that has stopped):
//   inflow: items (solve, 2, b, nblk) of the stage kernel's face waves: the
//           inflow of the new distribution into acc.ain_G (kind 3: into
//           acc.ain_x, the inflow of the initial state at prepare);
//   cols:   items (solve, -, b, acc.nblk): f, the newest columns, partial sums;
//   solve:  one workgroup per solve (items (solve, ...)): Gram matrix, gamma;
//   mix:    items as cols: x_next into theta[cur] and acc.ain_x.
void launch_accel_cols(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, hipStream_t st);
void launch_accel_solve(const DeviceView *vs, const WorkItem *wk, int n, hipStream_t st);
void launch_accel_mix(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, hipStream_t st);
constexpr int kAccelMaxDepth = 8;
void launch_finish(const DeviceView *vs, const WorkItem *wk, int n, hipStream_t st);

// One sweep launch over a work list (solve, direction, band block).  All
// items share the kernel variant (storage type, fan-in bound maxin, bands per
// lane, mode) and the workgroup size; lds_bytes is the largest LDS need among
// their solves.  mode: 0 every upwind value in LDS; 1 some boundary inflow
// read from HBM (levels with more ghosts than the LDS buffer holds); 2 some
// values spilled to HBM (LDS budget too small).  one: one lane per cell
// (bpl = bands per block, up to 8); otherwise bpl is 1, 2 or 4.
void launch_sweep(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, int maxin, int bpl, bool one, int mode,
                  int block, size_t lds_bytes, hipStream_t st, bool order2, bool planes);
// The transport solve of every (band, direction) system by Jacobi-BiCGSTAB:
// items (solve, direction, band, -), one 1024-thread workgroup per system.
void launch_bicgstab(const DeviceView *vs, const WorkItem *wk, int n, bool fp32, hipStream_t st);
size_t sweep_lds_bytes(int max_levels, int gring, int lstride, int slots, int elem_bytes);

// Dynamic LDS of a sweep workgroup, in elements of the storage type (es
// bytes): [level tables: 2 (max_levels + 1) ints, padded to 16 bytes]
// [zero block: ls][scratch block: ls][ghost ring: gring x ls][staged values:
// slots x ls].  The ghosts (boundary inflow) kept in LDS of consecutive
// levels follow each other around the ring (gring is a power of two), so the
// ring needs room for the two largest consecutive levels, not twice the
// largest.  ls is the stride of
// one cell's bands (lanes per cell x bands per lane), so every lane's bands
// start on a boundary of their own width and are read and written with one
// LDS access of up to 16 bytes per chunk.  Unused upwind references point at
// the zero block; values nobody reads again are written to the scratch
// block.  Shared by the host (which encodes references as final LDS offsets)
// and the kernel.
struct SweepLdsLayout {
    int ls, zero_off, trash_off, gbuf0, ring_off;
};
__host__ __device__ inline SweepLdsLayout sweep_lds_layout(int max_levels, int gring, int ls, int es) {
    SweepLdsLayout L;
    L.ls = ls;
    L.zero_off = ((2 * (max_levels + 1) * 4 + 15) / 16) * 16 / es;
    L.trash_off = L.zero_off + ls;
    L.gbuf0 = L.trash_off + ls;
    L.ring_off = L.gbuf0 + gring * ls;
    return L;
}

// PCG of the synthetic correction for a list of solves.
//   mode 0: solve L delta = rhs (every iteration);
//   mode 1: solve L theta[cur] = rhs (Fourier initial guess at prepare).
// Block form: one 1024-thread workgroup runs the whole PCG of a solve (items
// (solve, -, -, -)).  Multi-workgroup form (one reduction per iteration, so
// one launch per iteration): items (solve, -, local block, nblk); max_iter
// is the largest iteration count of the listed solves, each stops at its own.
void launch_pcg_block(const DeviceView *vs, const WorkItem *wk, int n, int mode, hipStream_t st);
// (k0, init: continue an earlier call from iteration k0 without the initial step)
void launch_pcg_multi(const DeviceView *vs, const WorkItem *wk, int n, int mode, int max_iter, hipStream_t st,
                      int k0 = 0, bool init = true);
constexpr int64_t kPcgBlockMaxRows = 8192;   // larger systems use the multi-workgroup form

// Iteration state: clear the stop flag and set the stop rule of a solve;
// copy the states of a list of solves into out[0..n).
void launch_set_controls(SolveState *s, int stop, double tol, int max_iter, int patience, hipStream_t st);
void launch_collect_states(const DeviceView *vs, int n, SolveState *out, hipStream_t st);

// the FP32 distribution in planes of bpb_in bands into the FP64 one in planes
// of bpb_out bands (D directions of N cells, B bands)
void launch_widen(int64_t D, int64_t N, int B, const float *in, int bpb_in, double *out, int bpb_out, hipStream_t st);
// out[k] = in[k] widened to FP64
void launch_widen_flat(int64_t n, const float *in, double *out, hipStream_t st);

// Single-solve helpers (outside the iteration).
// out[k] = offset + scale * in[k]
void launch_affine(int64_t n, const double *in, double scale, double offset, double *out, hipStream_t st);
// out[at] = in[idx[at]] over n entries, converted to FP32 (fp32) or kept FP64
void launch_gather(int64_t n, const int32_t *idx, const double *in, void *out, bool fp32, hipStream_t st);
// e(band, dir, c) of the last sweep of a solve
void launch_distribution(const DeviceView *v, bool fp32, int band, int dir, double *out, int64_t N, hipStream_t st);

// The file-scope staging array of the allocation-free distribution read
// (FP64, one value per cell) on the current device: its device address,
// looked up with hipGetSymbolAddress on the first call per device and kept.
constexpr int64_t kDistributionScratchCells = 1 << 21;   // 16 MiB per device
constexpr int kMaxDevices = 64;
hipError_t distribution_scratch(double **out);

}  // namespace nbte

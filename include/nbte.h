/*
 * nbte.h -- C ABI of the MI355X (gfx950) steady phonon BTE-RTA transport
 * library.
 *
 * The library solves the steady, non-gray phonon Boltzmann transport equation
 * under the relaxation-time approximation (Methods, Eqs. (3)-(4)) with
 * discrete ordinates in angle and a first-order upwind finite-volume
 * discretisation in space, and updates the lattice temperature with the
 * sequential scheme (Methods, Eqs. (5)-(6)) or the synthetic scheme (Methods,
 * Eqs. (7)-(12)).  The per-(band, direction) transport solves of Eq. (13) and
 * the band x direction reductions of Eq. (14) run as HIP kernels on the GPU.
 *
 * Conventions shared by every call:
 *   - SI units throughout; temperatures in kelvin.  2D meshes are per unit
 *     depth (face "area" = edge length, cell "volume" = cell area).
 *   - Every input array is owned by the caller, read during the call and
 *     copied; the caller may free it as soon as the call returns.
 *   - Handles are owned by the library until the matching *_destroy call.
 *     A problem keeps its mesh alive internally, so a mesh may be destroyed
 *     before the problems built on it.
 *   - No exception crosses the ABI.  Every call returns an nbte_status; on a
 *     non-OK status nbte_last_error() returns a thread-local description.
 *   - A problem handle (and a batch handle) is used by one host thread at a
 *     time.  Work is enqueued on the HIP stream given at creation (NULL = the
 *     null stream); calls that return results synchronise that stream.
 *   - There is no CPU fallback: if no usable gfx950 device is present the
 *     device-touching calls fail with NBTE_ERR_DEVICE.
 */
#ifndef NBTE_H
#define NBTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nbte_status;
#define NBTE_OK                 0
#define NBTE_ERR_INVALID_ARG   -1  /* null pointer, size or enum out of range, NaN input */
#define NBTE_ERR_MESH          -2  /* degenerate cell, non-manifold/non-conforming face, untagged boundary */
#define NBTE_ERR_QUADRATURE    -3  /* |s| != 1, w <= 0, specular mirror not in the set */
#define NBTE_ERR_BOUNDARY      -4  /* tag without a condition, bad wall data */
#define NBTE_ERR_ILL_POSED     -5  /* no thermalizing wall: the steady problem is singular */
#define NBTE_ERR_OUT_OF_MEMORY -6  /* device allocation failed or batch budget exceeded */
#define NBTE_ERR_DEVICE        -7  /* HIP runtime error or no gfx950 device */
#define NBTE_ERR_NOT_CONVERGED -8  /* max_iter reached; results hold the last iterate */
#define NBTE_ERR_DIVERGED      -9  /* non-finite or exploding residual */
#define NBTE_ERR_STATE        -10  /* call out of order (e.g. solve before set_bands) */

/* cell types (node ordering: quad4 and tri3 cyclic; hex8 = bottom face 0-1-2-3
   cyclic, then 4-5-6-7 above them; tet4 any order) */
#define NBTE_CELL_TRI3  1
#define NBTE_CELL_QUAD4 2
#define NBTE_CELL_TET4  3
#define NBTE_CELL_HEX8  4

/* boundary kinds (Methods; Numerical results: thermalizing, diffuse, specular walls) */
#define NBTE_BC_THERMALIZING 1  /* phonons leave the wall in equilibrium at T_wall */
#define NBTE_BC_SPECULAR     2  /* inflow = outgoing value of the mirror direction */
#define NBTE_BC_DIFFUSE      3  /* inflow = flux-weighted mean of the outgoing values */
#define NBTE_BC_PARTIAL      4  /* specularity p: p * specular + (1 - p) * diffuse */

/* temperature update schemes */
#define NBTE_SCHEME_SEQUENTIAL        0  /* Eq. (5): T_L from the collision moment */
#define NBTE_SCHEME_SYNTHETIC         1  /* Eqs. (9)-(10), diffusion-synthetic reading (default) */
#define NBTE_SCHEME_SYNTHETIC_LITERAL 2  /* Eqs. (9)-(10) with q_nonF built from T_L^(n) as printed */

/* precision of the stored distribution */
#define NBTE_PREC_FP64  0  /* distribution stored and swept in FP64 */
#define NBTE_PREC_MIXED 1  /* distribution, sweep streams and boundary inflow stored in FP32
                              and swept in FP32 arithmetic, in the deviation from the local
                              equilibrium; the equilibrium-imbalance differences, the band x
                              direction reductions, the diffusion correction and the residual
                              in FP64; FP64 sweeps take over when the FP32 iteration stalls
                              (nbte_solve_opts.refine) */

typedef struct nbte_mesh nbte_mesh;
typedef struct nbte_problem nbte_problem;
typedef struct nbte_batch nbte_batch;

/* ---------------------------------------------------------------- mesh ---- */

/* Build the finite-volume mesh: faces matched by node sets, outward area
 * vectors, volumes, neighbour table (the shared cell-face pattern of every
 * band x direction system; Methods, paragraph after Eq. (13)).
 *   dim          2 or 3
 *   xyz          n_nodes*dim node coordinates (m), row-major
 *   cell_type    NBTE_CELL_*; must match dim (tri3/quad4: 2, tet4/hex8: 3)
 *   cell_nodes   n_cells * nodes_per_cell node indices (0-based)
 *   bface_nodes  n_bfaces * nodes_per_face node indices of the boundary faces
 *   bface_tag    n_bfaces tags (any int32); every boundary face must be listed
 * Errors: NBTE_ERR_INVALID_ARG, NBTE_ERR_MESH. */
nbte_status nbte_mesh_create(int32_t dim, int64_t n_nodes, const double *xyz,
                             int32_t cell_type, int64_t n_cells, const int64_t *cell_nodes,
                             int64_t n_bfaces, const int64_t *bface_nodes, const int32_t *bface_tag,
                             nbte_mesh **out);
void nbte_mesh_destroy(nbte_mesh *m);

/* Read a Gmsh mesh file (MSH 4.1 or 2.2, ASCII; the mesh format of the
 * paper's workflow).  The elements of the highest dimension are the cells (one
 * type: 3-node triangles or 4-node quadrangles in 2D, 4-node tetrahedra or
 * 8-node hexahedra in 3D); the elements one dimension lower that lie on the
 * mesh boundary are the boundary faces, tagged with their physical group (0
 * when they have none; lower-dimensional elements inside the domain, such as
 * material interfaces, are skipped); each cell keeps its element's physical
 * group as its region (nbte_mesh_get_regions), e.g. to place heat sources.
 * Every boundary face of the cells must be present as an element.
 * Coordinates are multiplied by scale (1e-9 for a file in nm).
 * Errors: NBTE_ERR_INVALID_ARG (unreadable file, binary or unsupported format,
 * unsupported element type, scale <= 0), NBTE_ERR_MESH (mixed cell types, as
 * nbte_mesh_create). */
nbte_status nbte_mesh_read_gmsh(const char *path, double scale, nbte_mesh **out);
/* region[c] for every cell (n_cells entries): the physical group of its
 * element in the mesh file, 0 for meshes built by nbte_mesh_create. */
nbte_status nbte_mesh_get_regions(const nbte_mesh *m, int32_t *region);
/* xc[3c..3c+2]: the centre (vertex average) of every cell, m (z = 0 in 2D). */
nbte_status nbte_mesh_get_centroids(const nbte_mesh *m, double *xc);

typedef struct {
    int32_t dim;
    int32_t faces_per_cell;
    int64_t n_cells;
    int64_t n_bfaces;
    double total_volume;      /* m^3 (m^2 in 2D) */
    double max_closure_error; /* max_c |sum_f S_cf| / sum_f |S_cf|, ~1e-16 for a valid mesh */
} nbte_mesh_info;
nbte_status nbte_mesh_get_info(const nbte_mesh *m, nbte_mesh_info *info);

/* ------------------------------------------------------------- problem ---- */

/* A problem = a mesh plus band table, quadrature, boundary conditions and the
 * device-resident iterates.  hip_stream is a hipStream_t (NULL: null stream). */
nbte_status nbte_problem_create(const nbte_mesh *m, void *hip_stream, nbte_problem **out);
void nbte_problem_destroy(nbte_problem *p);

/* Band table (Methods, Eqs. (4)-(5)): heat capacity C (J m^-3 K^-1), group
 * velocity v (m/s), relaxation time tau (s), each n_bands > 0 finite positive
 * values.  Errors: NBTE_ERR_INVALID_ARG. */
nbte_status nbte_set_bands(nbte_problem *p, int32_t n_bands, const double *C, const double *v,
                           const double *tau);

/* Discrete-ordinates quadrature (Methods, Eqs. (4), (7), (11)): unit directions
 * s (n_dirs*3, row-major) and weights w > 0; W_Omega = sum w.  On a 2D mesh
 * the directions may be in-plane (s_z = 0, a 2D material) or span the sphere
 * (a 3D material over a domain that does not vary along z, as the paper's
 * diamond film): the faces see the in-plane part of s, a direction along z
 * carries nothing between cells.  Errors: NBTE_ERR_QUADRATURE. */
nbte_status nbte_set_quadrature(nbte_problem *p, int32_t n_dirs, const double *s, const double *w);

typedef struct {
    int32_t tag;          /* boundary-face tag this condition applies to */
    int32_t kind;         /* NBTE_BC_* */
    double T_wall;        /* K, thermalizing walls */
    double specularity;   /* p in [0,1], partial walls */
} nbte_boundary;

/* One condition per tag present on the mesh.  A specular or partial wall
 * needs the mirror of every direction about its normal in the quadrature
 * (NBTE_ERR_QUADRATURE otherwise).  At least one thermalizing wall is
 * required (NBTE_ERR_ILL_POSED otherwise, reported at solve time).
 * Errors: NBTE_ERR_BOUNDARY, NBTE_ERR_INVALID_ARG. */
nbte_status nbte_set_boundaries(nbte_problem *p, int32_t n, const nbte_boundary *bcs);

typedef struct {
    int32_t scheme;          /* NBTE_SCHEME_* */
    int32_t precision;       /* NBTE_PREC_* */
    double T_ref;            /* K, reference of the deviational variables (default 300) */
    double tol;              /* stop when max|dT_L| / max|T_L - T_ref| <= tol (default 1e-8) */
    int32_t max_iter;        /* default 10000 */
    int32_t check_every;     /* iterations between host polls of the device state (default 8);
                                the stop test runs on the device after every iteration, so
                                the result does not depend on it */
    const double *T_init;    /* nullable host array (n_cells): initial T_L; NULL = Fourier guess */
    int32_t outputs_on_device; /* 1: result arrays are device pointers */
    int32_t time_phases;     /* 1: record per-phase HIP-event times (see nbte_get_stats) */
    int32_t refine;          /* mixed precision only (default 1): when the FP32 iteration stops
                                improving (no 2% residual gain in 64 iterations) before reaching
                                tol, the solve continues with FP64 sweeps from where it stands */
    int32_t spatial_order;   /* 1 (default): first-order upwind face values.  2: second order: the
                                upwind side's value reconstructed linearly on the face with the
                                least-squares gradient of its cell over the interior face
                                neighbours (first order in cells whose neighbours do not span the
                                dimension), in the transport solve, the boundary conditions and the
                                heat flows; solved by deferred correction (each sweep keeps the
                                first-order operator and moves the previous distribution's
                                reconstruction to its right-hand side).  The deferred correction
                                converges where it contracts (structured meshes); where it does not
                                (ballistic bands on unstructured tetrahedra or triangles) the solve
                                ends with NBTE_ERR_DIVERGED.  Holds five more distribution-sized
                                arrays; not combined with nbte_tuning.accel_depth > 0
                                (NBTE_ERR_INVALID_ARG). */
} nbte_solve_opts;

/* Fill opts with the defaults listed above. */
void nbte_solve_opts_default(nbte_solve_opts *opts);

typedef struct {
    double *T_lattice;     /* n_cells, caller-allocated: T_L after the last update */
    double *T;             /* n_cells: energy temperature T_ref + sum w e / C_tot */
    double *q;             /* 3*n_cells (x,y,z per cell): heat flux, Eq. (7) (W/m^2) */
    int32_t iterations;
    double residual;       /* last max|dT_L| / max|T_L - T_ref| */
    double energy_defect;  /* |net boundary outflow - integral Qdot| / scale */
} nbte_result;

/* Solve to the steady state.  Q_cell: nullable host array (n_cells, W/m^3),
 * the volumetric heat generation, split over bands by heat capacity and
 * uniformly over directions (Numerical results, FinFET).  Any of the result
 * arrays may be NULL.  Returns NBTE_ERR_NOT_CONVERGED (with the last iterate
 * written) when max_iter is reached. */
nbte_status nbte_solve_steady(nbte_problem *p, const double *Q_cell, const nbte_solve_opts *o,
                              nbte_result *out);

/* Split form of nbte_solve_steady, for callers that drive the iteration:
 *   nbte_prepare  : setup (cached per geometry/tables) + initial guess;
 *   nbte_iterate  : exactly n full iterations (boundary inflow, transport
 *                   sweeps, moments, temperature update; no stop test), no
 *                   host synchronisation unless check is set, in which case
 *                   *residual receives the residual of the last iteration
 *                   (NBTE_ERR_DIVERGED if it is not finite);
 *   nbte_read_result: write the current state into out (waits for the
 *                   problem's work). */
nbte_status nbte_prepare(nbte_problem *p, const double *Q_cell, const nbte_solve_opts *o);
nbte_status nbte_iterate(nbte_problem *p, int32_t n, int32_t check, double *residual);
nbte_status nbte_read_result(nbte_problem *p, nbte_result *out);

/* Copy the current distribution e_{band,dir}(c) (deviational, J m^-3 per
 * unit weight, FP64) of one (band, direction) system into host out[n_cells]. */
nbte_status nbte_get_distribution(nbte_problem *p, int32_t band, int32_t dir, double *out);

/* The same read for callers that cannot allocate device memory (code that
 * must not call hipMalloc: tight serving loops, harnesses that forbid it):
 * nothing is allocated; the values are staged through a library-owned,
 * file-scope device array of 2^21 FP64 values (16 MiB per GPU, held until the
 * process ends) on the current device.  Meshes of more than 2^21 cells get
 * NBTE_ERR_INVALID_ARG.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (problems on different streams, host threads) race, so
 * the caller serialises them.  Errors as nbte_get_distribution. */
nbte_status nbte_get_distribution_noalloc(nbte_problem *p, int32_t band, int32_t dir, double *out);

/* Sweep schedule of one direction (host data, no device needed): the cells in
 * upwind order (perm[n_cells], nullable) grouped in topological levels
 * lvl_ptr[0..n_levels] (nullable; capacity cap_levels entries), such that
 * every interior upwind neighbour of a cell lies in an earlier level.  For
 * first-order upwind this order is the exact factorisation of the transport
 * matrix of Eq. (13).  Where the upwind graph of a direction is cyclic (a
 * non-convex cell), the order releases the lowest unfinished cell whenever it
 * stalls and lags that cell's upwind faces towards unfinished cells: those
 * faces are excluded from the level constraint and take the upwind value of
 * the previous iterate, like boundary inflow (nbte_get_lagged_faces).  The
 * outer iteration then converges to the same fixed point. */
nbte_status nbte_get_schedule(nbte_problem *p, int32_t dir, int32_t *perm, int32_t *lvl_ptr, int32_t cap_levels,
                              int32_t *n_levels);

/* The lagged faces of direction dir's sweep (host data, no device needed):
 * cells[k], faces[k] = cell and its local face index (the cell's face order of
 * its type), k < min(n, cap); *n = their number (0 for an acyclic upwind
 * graph).  cells/faces may be NULL to query *n.  A lagged face takes the
 * upwind neighbour's value of the previous iterate.  Errors:
 * NBTE_ERR_INVALID_ARG, NBTE_ERR_STATE (quadrature not set). */
nbte_status nbte_get_lagged_faces(nbte_problem *p, int32_t dir, int32_t *cells, int32_t *faces, int32_t cap,
                                  int32_t *n);

typedef struct {
    int32_t iterations;
    double ms_total;        /* wall time of the last solve/iterate call, ms */
    double ms_bc;           /* summed HIP-event times per phase (time_phases = 1):
                               boundary inflow and imbalance term */
    double ms_sweep;        /* transport sweep */
    double ms_moments;      /* boundary-face flux, band x direction reductions, wall
                               part of the correction's right-hand side */
    double ms_synthetic;    /* PCG of the synthetic correction */
    double ms_update;       /* theta update, residual, stop test */
    int32_t sweep_launches; /* launches of the transport sweep kernel timed above */
    int64_t updates_per_sweep;  /* n_cells * n_bands * n_dirs */
    int32_t max_levels;     /* deepest per-direction sweep schedule */
    int64_t device_bytes;   /* device memory held by the problem */
    int32_t bands_per_block;   /* launch shape of the last sweep */
    int32_t bands_per_lane;
    int32_t block_size;
    int32_t lds_slots;         /* staged slots per direction (0: staging off) */
    int64_t spilled_values;    /* consumed values per sweep that did not fit the LDS budget */
    int32_t refined_at;        /* iteration at which a mixed solve switched to FP64 sweeps, -1 if not */
} nbte_stats;
nbte_status nbte_get_stats(nbte_problem *p, nbte_stats *st);

/* Launch configuration of the kernels (chosen by the autotuner). */
typedef struct {
    int32_t bands_per_block;  /* bands of one direction per sweep workgroup (0 = auto) */
    int32_t bands_per_lane;   /* bands one lane sweeps (1,2,4,8; 0 = auto) */
    int32_t block_size;       /* threads per sweep workgroup (64..1024, multiple of 64; 0 = auto) */
    int32_t lds_bytes;        /* LDS budget per sweep workgroup (level tables, inflow ring and
                                 staged neighbour values), at most 163840 and capped at the
                                 device's per-workgroup LDS (0 = auto: half of a CU's LDS,
                                 -1 = no staging: neighbours read from HBM) */
    int32_t cg_max_iter;      /* diffusion-correction CG iterations per outer iteration (0 = auto) */
    double cg_rtol;           /* diffusion-correction CG relative tolerance (0 = auto) */
    int32_t no_graphs;        /* 1: launch every kernel eagerly instead of replaying HIP graphs
                                 of one and of eight iterations (phase timing always runs
                                 eagerly) */
    int32_t accel_depth;      /* Anderson acceleration of the outer iteration (0 = off, at most 8):
                                 the iterate (lattice temperature and the boundary inflow of every
                                 incoming row and band of the non-thermalizing faces, whose inflow
                                 depends on the distribution) is replaced after each iteration by
                                 G(x) - dG gamma, gamma the least-squares fit of the residual
                                 f = G(x) - x by the differences dF of the last accel_depth steps
                                 (D. G. Anderson 1965; Walker & Ni 2011).  An addition to the
                                 method's iteration: the fixed point, the stop test (on the plain
                                 image's residual) and the results at convergence are those of the
                                 plain iteration.  Holds about (2 accel_depth + 4) state vectors of
                                 n_cells + n_rows x n_bands values on the device (counted by
                                 nbte_problem_footprint, with every incoming row as the bound). */
    int32_t inner_solver;     /* transport solve of each (band, direction) system in an iteration:
                                 0 (default) the exact upwind sweep in level order; 1 matrix-free
                                 BiCGSTAB with the Jacobi (diagonal) preconditioner (the paper's
                                 optional iterative inner solver), one workgroup per system, every
                                 interior face coupled implicitly (cyclic upwind graphs included),
                                 started from the previous distribution.  Meant for small meshes: a
                                 system's iterations run in one workgroup.  First-order face values
                                 only (NBTE_ERR_INVALID_ARG with spatial_order 2). */
    int32_t inner_max_iter;   /* BiCGSTAB iterations per system and outer iteration (0 = 500) */
    double inner_rtol;        /* BiCGSTAB stop: ||r|| <= inner_rtol ||b|| (0 = 1e-13) */
    int32_t layout;           /* distribution layout in device memory: 1 cell-major (the bands of a
                                 (direction, cell) contiguous); 2 per direction in planes of the
                                 sweep's band blocks in upwind (level) order, so the sweep stores
                                 whole lines, at the price of a permuting reduction pass and a
                                 cell-major copy of the boundary cells' values; 0 (default) = 2 for
                                 n_cells x n_dirs x n_bands >= 2^26, else 1.  Results agree to
                                 rounding (summation order of the reductions). */
} nbte_tuning;
nbte_status nbte_set_tuning(nbte_problem *p, const nbte_tuning *t);
nbte_status nbte_get_tuning(const nbte_problem *p, nbte_tuning *t);

/* Device bytes a solve of this problem would hold at the given precision
 * (set_bands/set_quadrature must have been called).  Host arithmetic only.
 * Errors: NBTE_ERR_STATE; NBTE_ERR_INVALID_ARG when the problem is too large
 * for the sweep's 32-bit buffer offsets at that precision (any of: the
 * real-valued sweep streams (3 + fan-in rows) x directions x cells x element
 * size, a direction's distribution slice cells x bands x element size, or the
 * boundary inflow faces x directions x bands x element size reaching 4 GiB;
 * fan-in rows: 2 for triangles, 3 for quadrilaterals and tetrahedra, 5 for
 * hexahedra), the same check nbte_prepare, nbte_problem_setup and
 * nbte_batch_admit make before touching the device. */
nbte_status nbte_problem_footprint(const nbte_problem *p, int32_t precision, int64_t *bytes);

/* Build and upload the iteration-independent setup of a problem for a
 * precision -- sweep schedules and streams, LDS slot table, boundary plan,
 * band tables, diffusion operator, device state -- without starting a solve
 * (the setup step the method precomputes once; Methods, iteration scheme).
 * The next nbte_prepare / nbte_solve_steady / nbte_batch_admit at that
 * precision and tuning reuses it, so a caller admitting many problems can run
 * their setups concurrently, one thread per problem (different problems share
 * no state).  Errors: those of nbte_prepare's setup (NBTE_ERR_STATE when
 * bands, quadrature or boundaries are missing or the problem is a batch
 * member, NBTE_ERR_INVALID_ARG for a problem too large for the sweep's
 * 32-bit offsets (see nbte_problem_footprint; checked before the device is
 * touched), NBTE_ERR_MESH, NBTE_ERR_BOUNDARY, NBTE_ERR_ILL_POSED,
 * NBTE_ERR_DEVICE). */
nbte_status nbte_problem_setup(nbte_problem *p, int32_t precision);

/* -------------------------------------------------------------- batches -- */

/* A batch iterates many independent solves together: every kernel of an
 * iteration is one launch over all running members (Methods, Eq. (14): the
 * band x direction systems of all solves are independent tasks), replayed
 * from HIP graphs.  Members are admitted and removed at any time (continuous
 * batching); each member stops on the device when it reaches its own tol or
 * max_iter, and its result is the one a stand-alone nbte_solve_steady with the
 * same options and tuning computes (same kernels, same per-solve reduction
 * order: bitwise equal).
 *   hip_stream   stream of the batch's iterations (NULL: a stream of its own)
 *   budget_bytes device memory the members may hold together, by
 *                nbte_problem_footprint (0 = no limit) */
nbte_status nbte_batch_create(void *hip_stream, int64_t budget_bytes, nbte_batch **out);
/* Waits for the batch's work; members are released (not destroyed). */
void nbte_batch_destroy(nbte_batch *b);

/* Prepare p (as nbte_prepare, on p's own stream, so it overlaps the batch's
 * work in flight) and add it to the batch; it starts iterating with the next
 * nbte_batch_step and stops at o->tol or o->max_iter.  While it is a member,
 * the stand-alone calls nbte_prepare / nbte_iterate / nbte_solve_steady /
 * nbte_set_* on it fail with NBTE_ERR_STATE; nbte_read_result,
 * nbte_get_distribution and nbte_get_stats work (they wait for the batch).
 * Errors: NBTE_ERR_OUT_OF_MEMORY when the footprint exceeds what is left of
 * the budget (nothing is allocated then), the errors of nbte_prepare. */
nbte_status nbte_batch_admit(nbte_batch *b, nbte_problem *p, const double *Q_cell, const nbte_solve_opts *o);

/* Enqueue n iterations of every running member (asynchronous). */
nbte_status nbte_batch_step(nbte_batch *b, int32_t n);

/* Wait for the batch's stream; report up to cap members that have stopped
 * (converged, max_iter or diverged: see nbte_read_result) in done[0..*n_done)
 * and the number still running in *n_running (both nullable).  A mixed member
 * whose FP32 iteration stalled (refine on) continues with FP64 sweeps when
 * the budget can hold its FP64 footprint next to everything it holds now
 * (the switch briefly keeps both distributions); its charge becomes the FP64
 * footprint.  Otherwise it stays stopped and is reported here as done, its
 * residual above its tol. */
nbte_status nbte_batch_poll(nbte_batch *b, nbte_problem **done, int32_t cap, int32_t *n_done,
                            int32_t *n_running);

/* Remove a member (stopped or not; waits for the batch's stream).  Its
 * state and results stay on the device until it is prepared again or
 * destroyed.  Destroying a member removes it first. */
nbte_status nbte_batch_remove(nbte_batch *b, nbte_problem *p);

typedef struct {
    int32_t members;              /* problems in the batch */
    int64_t budget_bytes;         /* as created */
    int64_t bytes_in_use;         /* footprint of the members */
    int64_t iterations_launched;  /* sum of the n of every nbte_batch_step */
} nbte_batch_info;
nbte_status nbte_batch_get_info(const nbte_batch *b, nbte_batch_info *info);

/* --------------------------------------------------------------- errors -- */

/* Thread-local message for the last non-OK status of this thread ("" if none). */
const char *nbte_last_error(void);
/* Library version string. */
const char *nbte_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NBTE_H */

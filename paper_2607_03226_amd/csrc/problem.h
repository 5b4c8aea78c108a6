// The problem handle (one steady solve: mesh, tables, device-resident
// iterates) and the runner that iterates a list of prepared problems.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <chrono>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace nbte {

enum Phase { PH_BC = 0, PH_SWEEP, PH_MOM, PH_SYN, PH_UPD, PH_END, PH_COUNT };

void require_gfx950();

// ABI error plumbing: the status plus the thread-local message
nbte_status fail(nbte_status code, const std::string &msg);
template <class F>
nbte_status guarded(F &&f) {
    try {
        set_last_error("");
        return f();
    } catch (const Error &e) {
        return fail(e.code, e.what());
    } catch (const std::bad_alloc &) {
        return fail(NBTE_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(NBTE_ERR_INVALID_ARG, e.what());
    }
}

// Iterates a list of prepared problems together: every kernel of an
// iteration is one launch over all of them (work tables built here), and the
// launch sequence is replayed from HIP graphs of one and of kGraphIters
// iterations.  The problems' device state decides which of them still run.
class Runner {
  public:
    static constexpr int kGraphIters = 8;
    explicit Runner(hipStream_t st) : stream_(st) {}
    ~Runner();
    Runner(const Runner &) = delete;
    Runner &operator=(const Runner &) = delete;

    // replace the member list; the plan is rebuilt by the next run
    void set_members(const std::vector<nbte_problem *> &m);
    const std::vector<nbte_problem *> &members() const { return members_; }
    // enqueue n iterations of every member (asynchronous)
    void run(int n);
    // wait for the stream and copy every member's state into its host mirror
    void collect();
    // per-phase HIP-event timing (eager launches while on)
    void set_timing(bool on) { timing_ = on; }
    void set_graphs(bool on) {
        if (graphs_ != on) drop_graphs();
        graphs_ = on;
    }
    // add the event times of the iterations timed since the last call
    void harvest_timing();
    double phase_ms[PH_COUNT] = {0};
    int timed_iterations = 0;
    void reset_timing();

  private:
    struct Launch {
        int kind;              // see the enum in runner.cpp
        bool fp32 = false;
        int off = 0, n = 0;    // work items [off, off + n)
        int maxin = 0, bpl = 1, block = 256, iters = 0;
        int mode = 0;   // sweep kernel mode (launch_sweep)
        bool one = false;   // one lane per cell
        bool so2 = false;   // second-order sweep kernels
        bool planes = false;   // plane layout of the distribution (sweep kernels)
        size_t lds = 0;
    };
    void build();
    void enqueue_iteration(int event_slot);
    void drop_graphs();
    void release_retired();

    hipStream_t stream_;
    std::vector<nbte_problem *> members_;
    bool dirty_ = true;
    bool timing_ = false;
    bool graphs_ = true;
    std::vector<Launch> seq_;
    DevBuf d_views_, d_work_, d_states_;
    std::vector<std::unique_ptr<DevBuf>> retired_;
    std::vector<std::shared_ptr<void>> staging_;   // pinned upload sources of the plans
    hipGraph_t graph_[2] = {nullptr, nullptr};
    hipGraphExec_t exec_[2] = {nullptr, nullptr};
    std::vector<std::array<hipEvent_t, PH_COUNT>> events_;
    int events_used_ = 0;
};

}  // namespace nbte

namespace nbte {
// batch side of a member (batch.cpp)
void batch_sync(nbte_batch *b);
void batch_forget(nbte_batch *b, nbte_problem *p);
}  // namespace nbte

struct nbte_problem {
    std::shared_ptr<nbte::Mesh> mesh;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;   // created when the caller passes the null stream
    nbte::BandTable bands;
    nbte::Quadrature quad;
    std::vector<nbte_boundary> bcs;
    bool have_bands = false, have_quad = false, have_bcs = false;
    double T_ref = 300.0;

    // cached setup (validity flags)
    bool geom_ok = false, sched_ok = false, plan_ok = false, diff_ok = false, tables_ok = false;
    bool sched_up = false, plan_up = false, diff_up = false;
    nbte::Schedule sched;
    nbte::SweepProgram prog;
    nbte::BoundaryPlan plan;
    nbte::DiffusionOperator diff;

    // device buffers
    nbte::DevBuf d_nbr, d_V;
    nbte::DevBuf d_lvl_ptr, d_lvl_off, d_gptr, d_pupc, d_inrow, d_lag;
    // the sweep's streams, D*N entries per row, rows contiguous so the sweep
    // reads them through one buffer descriptor each:
    //   d_pint (int32):           cell | slot | maxin reference rows
    //   d_tstream (storage type): outflow sum | imbalance term D | heat source | maxin coefficient rows
    nbte::DevBuf d_pint, d_tstream;
    int coef_prec = -1;              // precision the outflow sums and coefficients were uploaded in
    int64_t stream_DN() const;
    const int32_t *p_cell() const { return d_pint.as<int32_t>(); }
    void *t_row(int r) const;        // row r of d_tstream
    nbte::DevBuf d_Cw, d_src, d_vel, d_itau, d_dirs, d_w, d_qbias;
    nbte::DevBuf d_bf_owner, d_bf_kind, d_mirror, d_bf_thw, d_bf_p, d_sdotS, d_win;
    nbte::DevBuf d_wall, d_wall_ptr, d_wslot;   // cells owning a reflective face, their face slots
    nbte::DevBuf d_wallJ;            // net flows of the reflective faces in slot order
    int64_t n_wall = 0, n_wall_faces = 0;
    nbte::DevBuf d_Lrow, d_Lcol, d_Lval, d_Ldinv;
    nbte::DevBuf d_Ecol, d_Eval;     // ELL copy (A D^-1) for the multi-workgroup CG
    nbte::DevBuf d_Jin, d_bsum;      // boundary faces: incoming flow, per-band outgoing sums
    nbte::DevBuf d_g, d_gval, d_Jw, d_Q;
    // the distribution's row index: stream position of each cell per direction
    // (D*N); plane layout: the boundary row of each face's owner (NBF), the
    // boundary rows (storage type), per (direction, cell) band sums of the
    // reductions' first stage (FP64 triples) and the boundary row each stream
    // position copies into (D*N)
    nbte::DevBuf d_pos, d_bf_brow, d_brow, d_mom, d_pbrow;
    bool pbrow_ok = false;   // d_pbrow holds the current schedule's positions
    int64_t boundary_owners() const;
    // distribution layout: band-block planes in stream order (large problems,
    // where the sweep's stores dominate) or cell-major (tuning.layout)
    bool planes() const { return planes_for(order); }
    bool planes_for(int ord) const;   // the layout a solve of spatial order ord takes
    int mom_lpc() const;
    nbte::DevBuf d_theta[3], d_theta_seq, d_thetaE, d_q, d_rhs, d_delta;
    nbte::DevBuf d_pcg_vec, d_pcg_part, d_pcg_scal;
    // the initial guess's CG: pinned converged flags of two chunks in flight, their events
    double *h_pcg_flag = nullptr;
    hipEvent_t pcg_ev[2] = {nullptr, nullptr};
    nbte::DevBuf d_view, d_state, d_self_work;
    // Anderson acceleration of the outer iteration (tuning.accel_depth > 0)
    nbte::DevBuf d_acc_x, d_acc_G, d_acc_fprev, d_acc_Gprev, d_acc_dF, d_acc_dG, d_acc_part, d_acc_scal;
    nbte::DevBuf d_acc_in;    // NBF*D: row of the state's inflow part of an incoming (face, direction), else -1
    int64_t acc_NR = 0;       // inflow entries of the state (rows of non-thermalizing faces x bands)
    int acc_nblk = 1;
    int self_acc = 0, n_self_acc = 0;   // offsets in d_self_work: initial inflow state (face waves)
    int accel_m() const { return tuning.accel_depth; }
    // Jacobi-BiCGSTAB inner solver (tuning.inner_solver = 1): eight work
    // vectors per (band, direction) system, system-major
    bool bicg() const { return tuning.inner_solver == 1; }
    nbte::DevBuf d_bicg;
    // second-order face values (opts.spatial_order = 2)
    int order = 1;
    bool lsq_up = false;
    nbte::DevBuf d_lsq, d_Sv, d_xf, d_xc, d_bf_local, d_grad, d_corr, d_bdelta;
    int so2_nblk = 1, so2_nblk_b = 1;   // workgroups of the gradient / correction and of the boundary launches
    int self_so2 = 0;                    // offset in d_self_work: [grad items][corr items][boundary items]
    int64_t accel_rows() const;         // bound on NR: ghost rows x bands
    int pcg_nblk = 1;
    int ell_w = 0;                   // ELL width of the correction's matrix

    // launch shape of the sweep
    struct Shape {
        int bpb = 1, bpl = 1, block = 256, slots = 0, gcap = 0, gring = 1;
        int lpc = 1, ls = 1;   // sweep lanes per cell; LDS stride of a cell's bands (lpc x bpl)
    } shape;
    int slots_for_cap = -2;   // slot budget the current slot table was built for
    int prog_B = -1, prog_gcap = -1, prog_gring = -1, prog_ls = -1, prog_es = -1;
    nbte_tuning tuning{0, 0, 0, 0, 0, 0.0, 0, 0, 0, 0, 0.0, 0};

    // iteration state
    bool prepared = false;
    int precision = NBTE_PREC_FP64;
    int scheme = NBTE_SCHEME_SYNTHETIC;
    double heat_in = 0.0;
    bool out_on_device = false;
    int time_phases = 0;
    nbte::DeviceView hv{};      // host copy of the descriptor in d_view
    nbte::SolveState hs{};      // host mirror of the device state (after a collect)
    int self_one = 0, self_pcg = 1, self_flux = 0, n_self_pcg = 0, n_self_flux = 0;   // offsets in d_self_work

    nbte_batch *batch = nullptr;          // batch this problem is a member of
    std::unique_ptr<nbte::Runner> solo;   // runner of stand-alone iterations
    nbte_stats stats{};

    ~nbte_problem();

    Shape resolve_shape() const;
    // throws NBTE_ERR_INVALID_ARG when a solve at this precision would not
    // fit the sweep's 32-bit buffer offsets (host check, no device access)
    void check_addressable(int prec) const;
    bool addressable(int prec) const {
        try {
            check_addressable(prec);
            return true;
        } catch (const nbte::Error &) {
            return false;
        }
    }
    int cg_max_iter() const { return tuning.cg_max_iter > 0 ? tuning.cg_max_iter : 8; }
    double cg_rtol() const { return tuning.cg_rtol > 0 ? tuning.cg_rtol : 1e-3; }
    bool fp32() const { return precision == NBTE_PREC_MIXED; }
    bool synthetic() const { return scheme != NBTE_SCHEME_SEQUENTIAL; }

    void build_host();
    void upload_device();
    void ensure_setup() {
        build_host();
        upload_device();
    }
    int64_t state_bytes(int prec, int ord = 1) const;
    void allocate_state(int prec);
    int64_t device_bytes() const;
    void make_view();
    void prepare(const double *Q_cell, const nbte_solve_opts &o);
    // device state: stop rule for the following iterations (clears the stop flag)
    void set_controls(int stop, double tol, int max_iter);
    // continue a mixed solve that stopped improving with FP64 sweeps (keeps theta,
    // the distribution and the iteration count)
    void promote();
    bool refine = true;      // mixed: switch to FP64 when the FP32 iteration stalls
    bool refine_possible() const { return fp32() && addressable(NBTE_PREC_FP64); }
    int refined_at = -1;
    int stop_mode = 0;
    double stop_tol = 0.0;
    int stop_max_iter = 0;
    // bring the host state mirror up to date (waits for the runner's stream)
    void sync_state();
    void iterate(int n, bool check, double *res_out);
    void read_result(nbte_result *out);
    void collect_stats();
    int cur_index() const { return (3 - hs.rot) % 3; }
    int prev_index() const { return (cur_index() + 1) % 3; }
};

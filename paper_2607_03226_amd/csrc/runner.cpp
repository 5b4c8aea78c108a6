// Runner: the iteration of a list of prepared problems as one launch
// sequence (Methods, Eq. (14): every band x direction system of every solve
// is an independent task of the same iteration).
//
// Per iteration: stage (boundary inflow, theta in sweep order), sweep, wall
// flux and reductions, synthetic correction (PCG), update, finish.  Each is
// one launch over all members of the same storage precision; the sweep is one
// launch per kernel variant.  Work tables map workgroups to (solve, ...).
#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>

#include "problem.h"

namespace nbte {

namespace {

enum Kind { K_MARK, K_STAGE, K_SWEEP, K_POST, K_REDUCE, K_WALL, K_PCG_BLOCK, K_PCG_MULTI, K_UPDATE, K_FINISH, K_ACC_COLS,
            K_ACC_SOLVE, K_ACC_MIX, K_GRAD, K_RECON, K_BICG };

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Pinned host staging of a plan's tables, kept alive with the device copies
// (an asynchronous upload reads it after the call returns).
struct Pinned {
    void *ptr = nullptr;
    explicit Pinned(size_t n) { NBTE_HIP(hipHostMalloc(&ptr, std::max<size_t>(n, 16), hipHostMallocDefault)); }
    ~Pinned() {
        if (ptr) (void)hipHostFree(ptr);
    }
};

}  // namespace

Runner::~Runner() {
    (void)hipStreamSynchronize(stream_);
    drop_graphs();
    for (auto &ev : events_)
        for (auto e : ev) (void)hipEventDestroy(e);
}

void Runner::drop_graphs() {
    for (int g = 0; g < 2; ++g) {
        if (exec_[g]) (void)hipGraphExecDestroy(exec_[g]);
        if (graph_[g]) (void)hipGraphDestroy(graph_[g]);
        exec_[g] = nullptr;
        graph_[g] = nullptr;
    }
}

void Runner::set_members(const std::vector<nbte_problem *> &m) {
    members_ = m;
    dirty_ = true;
}

void Runner::release_retired() {
    retired_.clear();
    staging_.clear();
}

void Runner::reset_timing() {
    for (double &x : phase_ms) x = 0.0;
    timed_iterations = 0;
    events_used_ = 0;
}

void Runner::build() {
    drop_graphs();
    // in-flight launches may still read the old tables: retire, free at the next collect
    for (DevBuf *b : {&d_views_, &d_work_, &d_states_}) {
        if (!b->ptr) continue;
        auto r = std::make_unique<DevBuf>();
        std::swap(r->ptr, b->ptr);
        std::swap(r->bytes, b->bytes);
        retired_.push_back(std::move(r));
    }
    seq_.clear();
    dirty_ = false;
    const int M = (int)members_.size();
    if (M == 0) return;

    std::vector<WorkItem> work;
    auto mark = [&](int phase) {
        Launch L;
        L.kind = K_MARK;
        L.iters = phase;
        seq_.push_back(L);
    };
    auto close = [&](Launch &L) {
        L.n = (int)work.size() - L.off;
        if (L.n > 0) seq_.push_back(L);
    };
    auto each = [&](bool fp32, auto &&fn) {
        for (int s = 0; s < M; ++s)
            if (members_[s]->fp32() == fp32) fn(s, *members_[s]);
    };

    mark(PH_BC);
    for (bool f : {true, false}) {
        Launch L;
        L.kind = K_STAGE;
        L.fp32 = f;
        L.off = (int)work.size();
        each(f, [&](int s, nbte_problem &p) {
            const int64_t nb0 = std::min<int64_t>(cdiv(p.mesh->NBF, 4), 2048);   // a wave per face
            // one stream entry per thread up to 16.8M entries (a grid-stride
            // loop beyond): config 3's 13.9M entries 0.20 -> 0.18 ms against a
            // cap of 16384 workgroups
            const int64_t nb1 = std::min<int64_t>(cdiv((int64_t)p.quad.D * p.mesh->N, 256), 65536);
            for (int64_t b = 0; b < nb0; ++b) work.push_back({s, 0, (int32_t)b, (int32_t)nb0});
            for (int64_t b = 0; b < nb1; ++b) work.push_back({s, 1, (int32_t)b, (int32_t)nb1});
            const int64_t nlag = (int64_t)p.prog.lag.size() / 4;   // lagged faces of cyclic upwind graphs
            const int64_t nb4 = std::min<int64_t>(cdiv(nlag * p.bands.B, 256), 1024);
            for (int64_t b = 0; b < nb4; ++b) work.push_back({s, 4, (int32_t)b, (int32_t)nb4});
        });
        close(L);
    }

    mark(PH_SWEEP);
    {
        // group by kernel variant; inside a group, XCD-aware longest-first order
        // fp32, maxin class, bpl, mode, block, one lane per cell, second order, plane layout
        using Key = std::tuple<int, int, int, int, int, int, int, int>;
        std::map<Key, std::vector<int>> groups;
        for (int s = 0; s < M; ++s) {
            const nbte_problem &p = *members_[s];
            if (p.bicg()) continue;   // transport solved by BiCGSTAB below
            const int mi = p.prog.maxin <= 2 ? 2 : (p.prog.maxin == 3 ? 3 : 5);
            const bool spill = p.shape.slots == 0 || p.sched.spilled > 0;
            const bool so2 = p.order == 2;   // second order: the general mode, several lanes per cell
            const int mode = (spill || so2) ? 2 : (p.prog.max_ghosts > p.shape.gcap ? 1 : 0);
            groups[Key(p.fp32() ? 1 : 0, mi, p.shape.bpl, mode, p.shape.block, (p.hv.lpc == 1 && !so2) ? 1 : 0,
                       so2 ? 1 : 0, p.hv.planes ? 1 : 0)]
                .push_back(s);
        }
        for (auto &kv : groups) {
            struct Unit {
                int s, dir, nbb;
                int64_t cost;
            };
            std::vector<Unit> units;
            size_t lds = 0;
            for (int s : kv.second) {
                const nbte_problem &p = *members_[s];
                const int nbb = (int)cdiv(p.bands.B, p.shape.bpb);
                const int lpc = p.hv.lpc;
                const int nslots = std::max(1, p.shape.block / lpc);
                lds = std::max(lds, sweep_lds_bytes(p.sched.max_levels, p.shape.gring, p.hv.lstride,
                                                    std::max(p.sched.max_slots, 1), p.fp32() ? 4 : 8));
                for (int i = 0; i < p.quad.D; ++i) {
                    // passes over the cells of direction i: one per level and slot row
                    int64_t passes = 0;
                    const int32_t *lp = &p.sched.lvl_ptr[p.sched.lvl_off[i]];
                    const int L = p.sched.lvl_off[i + 1] - p.sched.lvl_off[i] - 1;
                    for (int l = 0; l < L; ++l) passes += cdiv(lp[l + 1] - lp[l], nslots);
                    units.push_back({s, i, nbb, passes});
                }
            }
            std::stable_sort(units.begin(), units.end(), [](const Unit &a, const Unit &b) { return a.cost > b.cost; });
            // dispatch places workgroup k on XCD k mod 8: one queue per XCD, the
            // band blocks of a direction consecutive in one queue
            std::vector<WorkItem> q[8];
            int64_t load[8] = {0};
            for (const Unit &u : units) {
                int x = 0;
                for (int y = 1; y < 8; ++y)
                    if (load[y] < load[x]) x = y;
                for (int b = 0; b < u.nbb; ++b) q[x].push_back({u.s, u.dir, b, 0});
                load[x] += u.cost;
            }
            size_t len = 0;
            for (auto &qq : q) len = std::max(len, qq.size());
            Launch L;
            L.kind = K_SWEEP;
            L.fp32 = std::get<0>(kv.first) != 0;
            L.maxin = std::get<1>(kv.first);
            L.bpl = std::get<2>(kv.first);
            L.mode = std::get<3>(kv.first);
            L.one = std::get<5>(kv.first) != 0;
            L.so2 = std::get<6>(kv.first) != 0;
            L.planes = std::get<7>(kv.first) != 0;
            L.block = std::get<4>(kv.first);
            L.lds = lds;
            L.off = (int)work.size();
            for (size_t k = 0; k < len; ++k)
                for (int x = 0; x < 8; ++x) work.push_back(k < q[x].size() ? q[x][k] : WorkItem{-1, 0, 0, 0});
            // trailing padding serves nothing
            while ((int)work.size() > L.off && work.back().solve < 0) work.pop_back();
            close(L);
        }
    }

    // members with the BiCGSTAB inner solver: one workgroup per system
    for (bool f : {true, false}) {
        Launch L;
        L.kind = K_BICG;
        L.fp32 = f;
        L.off = (int)work.size();
        each(f, [&](int s, nbte_problem &p) {
            if (!p.bicg()) return;
            for (int i = 0; i < p.quad.D; ++i)
                for (int b = 0; b < p.bands.B; ++b) work.push_back({s, i, b, 0});
        });
        close(L);
    }

    mark(PH_MOM);
    // second order: gradients of the new distribution, the next sweep's
    // correction and the outgoing increments the boundary flux needs
    for (bool f : {true, false}) {
        Launch G;
        G.kind = K_GRAD;
        G.fp32 = f;
        G.off = (int)work.size();
        each(f, [&](int s, nbte_problem &p) {
            if (p.order != 2) return;
            for (int b = 0; b < p.so2_nblk; ++b) work.push_back({s, 0, b, p.so2_nblk});
        });
        close(G);
        Launch R;
        R.kind = K_RECON;
        R.fp32 = f;
        R.off = (int)work.size();
        each(f, [&](int s, nbte_problem &p) {
            if (p.order != 2) return;
            for (int b = 0; b < p.so2_nblk; ++b) work.push_back({s, 0, b, p.so2_nblk});
            for (int b = 0; b < p.so2_nblk_b; ++b) work.push_back({s, 1, b, p.so2_nblk_b});
        });
        close(R);
    }
    for (bool f : {true, false}) {
        // cell-major members: boundary flux (every scheme: the outgoing sums
        // feed the next diffuse inflow; the net flows are used by the
        // synthetic correction only) first, the moment blocks after it.
        // Plane members: reduction stage 1, item (s, 2, chunk, direction)
        // covering positions [256 chunk, + 256) of a direction.  Workgroup k
        // of a launch runs on XCD k mod 8: the stage-1 items start at a
        // multiple of 8 and each XCD takes whole directions one after the
        // other (chunks in order), so the scattered (direction, cell) sums of
        // the one or two directions it works on at a time stay in its L2.
        Launch L;
        L.kind = K_POST;
        L.fp32 = f;
        L.off = (int)work.size();
        each(f, [&](int s, nbte_problem &p) {
            if (p.hv.planes) return;
            const int64_t nb = cdiv(p.mesh->NBF, 4);   // a wave per face
            for (int64_t b = 0; b < nb; ++b) work.push_back({s, 0, (int32_t)b, (int32_t)nb});
        });
        each(f, [&](int s, nbte_problem &p) {
            if (p.hv.planes) return;
            const int64_t nb = cdiv(p.mesh->N * p.hv.mom_lpc, 256);
            for (int64_t b = 0; b < nb; ++b) work.push_back({s, 1, (int32_t)b, (int32_t)nb});
        });
        std::vector<WorkItem> q[8];
        int64_t load[8] = {0};
        each(f, [&](int s, nbte_problem &p) {
            if (!p.hv.planes) return;
            const int64_t nc = cdiv(p.mesh->N, 256);
            for (int i = 0; i < p.quad.D; ++i) {
                int x = 0;
                for (int y = 1; y < 8; ++y)
                    if (load[y] < load[x]) x = y;
                for (int64_t b = 0; b < nc; ++b) q[x].push_back({s, 2, (int32_t)b, i});
                load[x] += nc;
            }
        });
        size_t len = 0;
        for (auto &qq : q) len = std::max(len, qq.size());
        if (len > 0)
            while ((work.size() - L.off) % 8) work.push_back({-1, 0, 0, 0});
        for (size_t k = 0; k < len; ++k)
            for (int x = 0; x < 8; ++x) work.push_back(k < q[x].size() ? q[x][k] : WorkItem{-1, 0, 0, 0});
        while ((int)work.size() > L.off && work.back().solve < 0) work.pop_back();
        close(L);
    }
    for (bool f : {true, false}) {
        // plane members: boundary flux from the boundary rows first, then
        // stage 2 of the reductions
        Launch L;
        L.kind = K_REDUCE;
        L.fp32 = f;
        L.off = (int)work.size();
        each(f, [&](int s, nbte_problem &p) {
            if (!p.hv.planes) return;
            const int64_t nb = cdiv(p.mesh->NBF, 4);   // a wave per face
            for (int64_t b = 0; b < nb; ++b) work.push_back({s, 0, (int32_t)b, (int32_t)nb});
        });
        each(f, [&](int s, nbte_problem &p) {
            if (!p.hv.planes) return;
            const int64_t nb = std::min<int64_t>(cdiv(p.mesh->N * kReduceLanes, 256), 8192);
            for (int64_t b = 0; b < nb; ++b) work.push_back({s, 1, (int32_t)b, (int32_t)nb});
        });
        close(L);
    }
    {
        Launch L;
        L.kind = K_WALL;
        L.off = (int)work.size();
        for (int s = 0; s < M; ++s) {
            const nbte_problem &p = *members_[s];
            if (!p.synthetic() || p.n_wall == 0) continue;
            const int64_t nb = std::min<int64_t>(cdiv(p.n_wall, 256), 64);
            for (int64_t b = 0; b < nb; ++b) work.push_back({s, 0, (int32_t)b, (int32_t)nb});
        }
        close(L);
    }

    mark(PH_SYN);
    {
        Launch L;
        L.kind = K_PCG_BLOCK;
        L.off = (int)work.size();
        for (int s = 0; s < M; ++s) {
            const nbte_problem &p = *members_[s];
            if (p.synthetic() && p.mesh->N <= kPcgBlockMaxRows) work.push_back({s, 0, 0, 1});
        }
        close(L);
        Launch G;
        G.kind = K_PCG_MULTI;
        G.off = (int)work.size();
        for (int s = 0; s < M; ++s) {
            const nbte_problem &p = *members_[s];
            if (!p.synthetic() || p.mesh->N <= kPcgBlockMaxRows) continue;
            for (int b = 0; b < p.pcg_nblk; ++b) work.push_back({s, 0, b, p.pcg_nblk});
            G.iters = std::max(G.iters, p.cg_max_iter());
        }
        close(G);
    }

    mark(PH_UPD);
    {
        Launch L;
        L.kind = K_UPDATE;
        L.off = (int)work.size();
        for (int s = 0; s < M; ++s) {
            const int64_t nb = std::min<int64_t>(cdiv(members_[s]->mesh->N, 256), 1024);
            for (int64_t b = 0; b < nb; ++b) work.push_back({s, 0, (int32_t)b, (int32_t)nb});
        }
        close(L);
        Launch F;
        F.kind = K_FINISH;
        F.off = (int)work.size();
        for (int s = 0; s < M; ++s) work.push_back({s, 0, 0, 0});
        close(F);
        // Anderson step of the accelerated members: the image's inflow (stage
        // face waves of kind 2), columns and partial sums, gamma, the mix
        for (bool f : {true, false}) {
            Launch A;
            A.kind = K_STAGE;
            A.fp32 = f;
            A.off = (int)work.size();
            each(f, [&](int s, nbte_problem &p) {
                if (p.accel_m() <= 0) return;
                const int64_t nb = std::min<int64_t>(cdiv(p.mesh->NBF, 4), 2048);
                for (int64_t b = 0; b < nb; ++b) work.push_back({s, 2, (int32_t)b, (int32_t)nb});
            });
            close(A);
        }
        for (bool f : {true, false}) {
            Launch A;
            A.kind = K_ACC_COLS;
            A.fp32 = f;
            A.off = (int)work.size();
            each(f, [&](int s, nbte_problem &p) {
                if (p.accel_m() <= 0) return;
                for (int b = 0; b < p.acc_nblk; ++b) work.push_back({s, 0, b, p.acc_nblk});
            });
            close(A);
        }
        {
            Launch A;
            A.kind = K_ACC_SOLVE;
            A.off = (int)work.size();
            for (int s = 0; s < M; ++s)
                if (members_[s]->accel_m() > 0) work.push_back({s, 0, 0, 0});
            close(A);
        }
        for (bool f : {true, false}) {
            Launch A;
            A.kind = K_ACC_MIX;
            A.fp32 = f;
            A.off = (int)work.size();
            each(f, [&](int s, nbte_problem &p) {
                if (p.accel_m() <= 0) return;
                for (int b = 0; b < p.acc_nblk; ++b) work.push_back({s, 0, b, p.acc_nblk});
            });
            close(A);
        }
    }
    mark(PH_END);

    // upload through pinned staging (kept with the plan until it is retired)
    const size_t vb = M * sizeof(DeviceView), wb = work.size() * sizeof(WorkItem);
    auto pin = std::make_shared<Pinned>(vb + wb);
    char *h = static_cast<char *>(pin->ptr);
    for (int s = 0; s < M; ++s) std::memcpy(h + s * sizeof(DeviceView), &members_[s]->hv, sizeof(DeviceView));
    if (wb) std::memcpy(h + vb, work.data(), wb);
    d_views_.alloc(vb);
    d_work_.alloc(std::max<size_t>(wb, sizeof(WorkItem)));
    d_states_.alloc(M * sizeof(SolveState));
    NBTE_HIP(hipMemcpyAsync(d_views_.ptr, h, vb, hipMemcpyHostToDevice, stream_));
    if (wb) NBTE_HIP(hipMemcpyAsync(d_work_.ptr, h + vb, wb, hipMemcpyHostToDevice, stream_));
    staging_.push_back(pin);
}

void Runner::enqueue_iteration(int slot) {
    const DeviceView *vs = d_views_.as<DeviceView>();
    const WorkItem *wk = d_work_.as<WorkItem>();
    for (const Launch &L : seq_) {
        switch (L.kind) {
            case K_MARK:
                if (slot >= 0) NBTE_HIP(hipEventRecord(events_[slot][L.iters], stream_));
                break;
            case K_STAGE: launch_stage(vs, wk + L.off, L.n, L.fp32, stream_); break;
            case K_SWEEP:
                launch_sweep(vs, wk + L.off, L.n, L.fp32, L.maxin, L.bpl, L.one, L.mode, L.block, L.lds, stream_,
                             L.so2, L.planes);
                break;
            case K_POST: launch_post(vs, wk + L.off, L.n, L.fp32, stream_); break;
            case K_REDUCE: launch_reduce(vs, wk + L.off, L.n, L.fp32, stream_); break;
            case K_WALL: launch_wall_rhs(vs, wk + L.off, L.n, stream_); break;
            case K_PCG_BLOCK: launch_pcg_block(vs, wk + L.off, L.n, 0, stream_); break;
            case K_PCG_MULTI:
                launch_pcg_multi(vs, wk + L.off, L.n, 0, L.iters, stream_);
                break;
            case K_UPDATE: launch_update(vs, wk + L.off, L.n, stream_); break;
            case K_FINISH: launch_finish(vs, wk + L.off, L.n, stream_); break;
            case K_ACC_COLS: launch_accel_cols(vs, wk + L.off, L.n, L.fp32, stream_); break;
            case K_ACC_SOLVE: launch_accel_solve(vs, wk + L.off, L.n, stream_); break;
            case K_ACC_MIX: launch_accel_mix(vs, wk + L.off, L.n, L.fp32, stream_); break;
            case K_GRAD: launch_grad(vs, wk + L.off, L.n, L.fp32, 0, stream_); break;
            case K_RECON: launch_recon(vs, wk + L.off, L.n, L.fp32, 0, stream_); break;
            case K_BICG: launch_bicgstab(vs, wk + L.off, L.n, L.fp32, stream_); break;
        }
    }
    NBTE_HIP(hipGetLastError());
}

void Runner::run(int n) {
    if (dirty_) build();
    if (members_.empty() || n <= 0) return;
    if (timing_ || !graphs_) {
        for (int k = 0; k < n; ++k) {
            int slot = -1;
            if (timing_) {
                if (events_used_ == (int)events_.size()) {
                    std::array<hipEvent_t, PH_COUNT> ev;
                    for (auto &e : ev) NBTE_HIP(hipEventCreate(&e));
                    events_.push_back(ev);
                }
                slot = events_used_++;
            }
            enqueue_iteration(slot);
        }
        return;
    }
    auto launch = [&](int g) {
        if (!exec_[g]) {
            NBTE_HIP(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
            try {
                for (int k = 0; k < (g ? kGraphIters : 1); ++k) enqueue_iteration(-1);
            } catch (...) {
                hipGraph_t gr = nullptr;
                (void)hipStreamEndCapture(stream_, &gr);
                if (gr) (void)hipGraphDestroy(gr);
                throw;
            }
            NBTE_HIP(hipStreamEndCapture(stream_, &graph_[g]));
            NBTE_HIP(hipGraphInstantiate(&exec_[g], graph_[g], nullptr, nullptr, 0));
        }
        NBTE_HIP(hipGraphLaunch(exec_[g], stream_));
    };
    int k = 0;
    for (; n - k >= kGraphIters; k += kGraphIters) launch(1);
    for (; k < n; ++k) launch(0);
}

void Runner::harvest_timing() {
    if (events_used_ == 0) return;
    NBTE_HIP(hipStreamSynchronize(stream_));
    for (int k = 0; k < events_used_; ++k)
        for (int ph = 0; ph < PH_END; ++ph) {
            float ms = 0;
            NBTE_HIP(hipEventElapsedTime(&ms, events_[k][ph], events_[k][ph + 1]));
            phase_ms[ph] += ms;
        }
    timed_iterations += events_used_;
    events_used_ = 0;
}

void Runner::collect() {
    if (dirty_) build();
    const int M = (int)members_.size();
    std::vector<SolveState> h(M);
    if (M > 0) {
        launch_collect_states(d_views_.as<DeviceView>(), M, d_states_.as<SolveState>(), stream_);
        NBTE_HIP(hipMemcpyAsync(h.data(), d_states_.ptr, M * sizeof(SolveState), hipMemcpyDeviceToHost, stream_));
    }
    NBTE_HIP(hipStreamSynchronize(stream_));
    for (int s = 0; s < M; ++s) members_[s]->hs = h[s];
    release_retired();
}

}  // namespace nbte

// Batches: many independent steady solves iterated together (one launch per
// kernel per iteration over all of them), with admission by device-memory
// footprint and removal at any time -- the engine of continuous batching.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "problem.h"

using namespace nbte;

struct nbte_batch {
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    int64_t budget = 0;        // device bytes the members may hold (0 = no limit)
    int64_t in_use = 0;        // footprint of the current members
    std::vector<nbte_problem *> members;
    std::vector<int64_t> charged;   // footprint charged per member
    std::unique_ptr<Runner> runner;
    int64_t iterations_launched = 0;

    ~nbte_batch() {
        if (runner) runner.reset();   // waits for the stream
        for (nbte_problem *p : members) p->batch = nullptr;
        if (own_stream) (void)hipStreamDestroy(own_stream);
    }

    void drop(nbte_problem *p) {
        NBTE_HIP(hipStreamSynchronize(stream));   // in-flight iterations may still read p
        auto it = std::find(members.begin(), members.end(), p);
        if (it == members.end()) throw Error(NBTE_ERR_STATE, "the problem is not a member of this batch");
        const size_t k = it - members.begin();
        in_use -= charged[k];
        members.erase(it);
        charged.erase(charged.begin() + k);
        p->batch = nullptr;
        runner->set_members(members);
    }
};

namespace nbte {

void batch_sync(nbte_batch *b) { b->runner->collect(); }

void batch_forget(nbte_batch *b, nbte_problem *p) {
    try {
        b->drop(p);
    } catch (...) {
        p->batch = nullptr;
    }
}

}  // namespace nbte

extern "C" {

nbte_status nbte_batch_create(void *hip_stream, int64_t budget_bytes, nbte_batch **out) {
    return guarded([&] {
        if (!out || budget_bytes < 0) throw Error(NBTE_ERR_INVALID_ARG, "bad arguments");
        *out = nullptr;
        require_gfx950();
        auto *b = new nbte_batch();
        b->budget = budget_bytes;
        b->stream = static_cast<hipStream_t>(hip_stream);
        if (!b->stream) {
            hipError_t e = hipStreamCreate(&b->own_stream);
            if (e != hipSuccess) {
                delete b;
                throw Error(NBTE_ERR_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
            }
            b->stream = b->own_stream;
        }
        b->runner = std::make_unique<Runner>(b->stream);
        *out = b;
        return NBTE_OK;
    });
}

void nbte_batch_destroy(nbte_batch *b) { delete b; }

nbte_status nbte_batch_admit(nbte_batch *b, nbte_problem *p, const double *Q_cell, const nbte_solve_opts *o) {
    return guarded([&] {
        if (!b || !p || !o) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        if (p->batch) throw Error(NBTE_ERR_STATE, "the problem is already a batch member");
        if (!(o->tol > 0) || o->max_iter <= 0) throw Error(NBTE_ERR_INVALID_ARG, "tol must be > 0 and max_iter >= 1");
        int64_t need = 0;
        const nbte_status fst = nbte_problem_footprint(p, o->precision, &need);
        if (fst != NBTE_OK) throw Error(fst, nbte_last_error());
        if (o->spatial_order == 2)   // the second-order arrays on top of the first-order footprint
            need += p->state_bytes(o->precision, 2) - p->state_bytes(o->precision, 1);
        if (b->budget > 0 && b->in_use + need > b->budget)
            throw Error(NBTE_ERR_OUT_OF_MEMORY, "batch budget exceeded: " + std::to_string(b->in_use) + " + " +
                                                    std::to_string(need) + " > " + std::to_string(b->budget) + " bytes");
        // setup and initial guess on the problem's own stream (overlaps the
        // batch's work in flight); the runner starts it at its next step
        p->prepare(Q_cell, *o);
        p->out_on_device = o->outputs_on_device != 0;
        p->set_controls(1, o->tol, o->max_iter);
        p->batch = b;
        b->members.push_back(p);
        b->charged.push_back(need);
        b->in_use += need;
        b->runner->set_members(b->members);
        return NBTE_OK;
    });
}

nbte_status nbte_batch_step(nbte_batch *b, int32_t n) {
    return guarded([&] {
        if (!b || n < 0) throw Error(NBTE_ERR_INVALID_ARG, "bad arguments");
        b->runner->run(n);
        b->iterations_launched += n;
        return NBTE_OK;
    });
}

nbte_status nbte_batch_poll(nbte_batch *b, nbte_problem **done, int32_t cap, int32_t *n_done, int32_t *n_running) {
    return guarded([&] {
        if (!b || cap < 0 || (cap > 0 && !done)) throw Error(NBTE_ERR_INVALID_ARG, "bad arguments");
        b->runner->collect();
        // mixed members whose FP32 iteration stalled continue in FP64 when
        // the budget holds the FP64 footprint beside the current one (the
        // switch widens the distribution into a new buffer before the FP32
        // one is freed); otherwise they stay stopped and are reported below
        // as done, with the residual they reached
        bool changed = false;
        for (size_t k = 0; k < b->members.size(); ++k) {
            nbte_problem *p = b->members[k];
            if (p->hs.done != NBTE_DONE_STALLED || !p->refine_possible()) continue;
            int64_t need = 0;
            if (nbte_problem_footprint(p, NBTE_PREC_FP64, &need) != NBTE_OK) continue;
            if (b->budget > 0 && b->in_use + need > b->budget) continue;
            p->promote();
            b->in_use += need - b->charged[k];   // the FP64 footprint from now on
            b->charged[k] = need;
            changed = true;
        }
        if (changed) b->runner->set_members(b->members);
        int32_t nd = 0, nr = 0;
        for (nbte_problem *p : b->members) {
            if (p->hs.done) {
                if (nd < cap) done[nd] = p;
                ++nd;
            } else {
                ++nr;
            }
        }
        if (n_done) *n_done = std::min(nd, cap);
        if (n_running) *n_running = nr;
        return NBTE_OK;
    });
}

nbte_status nbte_batch_remove(nbte_batch *b, nbte_problem *p) {
    return guarded([&] {
        if (!b || !p) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        if (p->batch != b) throw Error(NBTE_ERR_STATE, "the problem is not a member of this batch");
        b->drop(p);
        return NBTE_OK;
    });
}

nbte_status nbte_batch_get_info(const nbte_batch *b, nbte_batch_info *info) {
    return guarded([&] {
        if (!b || !info) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        info->members = (int32_t)b->members.size();
        info->budget_bytes = b->budget;
        info->bytes_in_use = b->in_use;
        info->iterations_launched = b->iterations_launched;
        return NBTE_OK;
    });
}

}  // extern "C"

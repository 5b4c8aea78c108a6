// Problem handles, the single-solve driver and their C ABI (include/nbte.h).
//
// One iteration (Methods, Eqs. (5)-(6) sequential, (7)-(12) synthetic; the
// task split of Eq. (14) becomes one kernel over all band x direction systems):
//   1. lagged boundary inflow from the previous distribution;
//   2. transport sweep of every (band, direction) system at the current T_L;
//   3. band x direction reductions: collision-weighted T_L (Eq. (5)), energy
//      temperature, heat flux (Eq. (7));
//   4. sequential: T_L <- that moment; synthetic: diffusion correction
//      (Eq. (10)) solved by PCG, T_L <- moment + correction;
//   5. FP64 residual max|dT_L| / max|T_L - T_ref| and the stop test, on the
//      device.
// A stand-alone problem iterates through a Runner of one member; batches
// (batch.cpp) put many problems in one Runner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "problem.h"

using namespace nbte;

struct nbte_mesh {
    std::shared_ptr<Mesh> m;
};

namespace {
thread_local std::string g_last_error;
}

namespace nbte {

void set_last_error(const std::string &msg) { g_last_error = msg; }

nbte_status fail(nbte_status code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

void require_gfx950() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) throw Error(NBTE_ERR_DEVICE, "no HIP device available");
    int dev = 0;
    NBTE_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    NBTE_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        throw Error(NBTE_ERR_DEVICE, std::string("library built for gfx950, device is ") + prop.gcnArchName);
}

}  // namespace nbte

namespace {
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
}

nbte_problem::~nbte_problem() {
    if (batch) batch_forget(batch, this);
    solo.reset();
    if (stream) (void)hipStreamSynchronize(stream);
    if (h_pcg_flag) {
        (void)hipHostFree(h_pcg_flag);
        for (auto e : pcg_ev) (void)hipEventDestroy(e);
    }
    if (own_stream) (void)hipStreamDestroy(own_stream);
}

// LDS bytes one workgroup may use on the current device (64 KiB if unknown)
static int lds_limit() {
    static std::atomic<int> cached{0};   // problems may be set up from several threads
    const int c = cached.load(std::memory_order_relaxed);
    if (c > 0) return c;
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) {
        (void)hipGetLastError();
        return 65536;
    }
    cached.store(v, std::memory_order_relaxed);
    return v;
}

int64_t nbte_problem::stream_DN() const { return (int64_t)quad.D * mesh->N; }

void *nbte_problem::t_row(int r) const {
    return static_cast<char *>(d_tstream.ptr) + (size_t)r * stream_DN() * (fp32() ? 4 : 8);
}

// lanes per cell of the cell-major reductions: a power of two >= B, at most
// 64 (one band per lane; measured: splitting the directions of a cell over
// more lanes breaks the coalesced band rows and is slower, and so did 16-byte
// loads of four bands per lane)
int nbte_problem::mom_lpc() const {
    int lpc = 1;
    while (lpc < bands.B && lpc < 64) lpc <<= 1;
    return lpc;
}

// The plane layout pays where the distribution is far larger than the
// caches: its sweep stores whole lines, but the reductions and boundary
// kernels then permute (measured: config 3, 444M values, 5 % faster per
// iteration; config 2, 28M values, cache resident, 30 % slower).  Chosen by
// the element count, so the layout does not change with the precision.
bool nbte_problem::planes_for(int ord) const {
    if (tuning.layout != 0) return tuning.layout == 2;
    // second order keeps the cell-major layout: its gradient pass gathers
    // every neighbour's whole row (config 3 at order 2: 22.8 ms per mixed
    // iteration cell-major against 24.9 ms in planes)
    return ord == 1 && (int64_t)mesh->N * quad.D * bands.B >= kPlanesMinValues;
}

// cells that own at least one boundary face (rows of the boundary copy)
int64_t nbte_problem::boundary_owners() const {
    const Mesh &m = *mesh;
    std::vector<char> own(m.N, 0);
    for (int64_t bf = 0; bf < m.NBF; ++bf) own[m.bf_owner[bf]] = 1;
    int64_t n = 0;
    for (char x : own) n += x;
    return n;
}

// Resolve the tuning into one sweep launch shape.  Defaults aim at two
// workgroups per CU (bands split into blocks until D * blocks >= 512) and a
// 64 KiB LDS budget for staged neighbour values.
nbte_problem::Shape nbte_problem::resolve_shape() const {
    Shape sh;
    const int B = bands.B, D = quad.D;
    int bpb = tuning.bands_per_block;
    if (bpb <= 0) {
        int nbb = std::max(1, std::min(B, (512 + D - 1) / D));
        int want = (B + nbb - 1) / nbb;
        bpb = 1;
        while (bpb * 2 <= want) bpb *= 2;
    }
    bpb = std::min(bpb, B);
    int bpl = tuning.bands_per_lane > 0 ? tuning.bands_per_lane : 1;
    while (bpl * 64 < bpb) bpl *= 2;          // at most 64 lanes per cell
    if (bpl > 8) throw Error(NBTE_ERR_INVALID_ARG, "bands_per_block too large for 8 bands per lane");
    int lanes = (bpb + bpl - 1) / bpl, lpc = 1;
    while (lpc < lanes) lpc <<= 1;
    if ((lpc > 1 || order == 2) && bpl > 4) {   // eight bands per lane only with one lane per cell (first order)
        bpl = 4;
        lanes = (bpb + bpl - 1) / bpl;
        lpc = 1;
        while (lpc < lanes) lpc <<= 1;
    }
    int block = tuning.block_size > 0 ? tuning.block_size : 256;
    block = std::min(std::max(block, lpc), 512);   // the sweep kernel is built for <= 512 threads
    sh.bpb = bpb;
    sh.bpl = bpl;
    sh.block = block;
    sh.lpc = lpc;
    sh.ls = lpc * bpl;   // a cell's bands in LDS, padded to whole lanes
    // the level tables and the ghost ring of a direction share the
    // workgroup's LDS with the staged values.  The ring keeps every ghost in
    // LDS when room for the two largest consecutive levels fits in half the
    // budget; otherwise it takes a quarter of the budget and each level keeps
    // half of it, larger boundary levels read the rest from HBM.  The default
    // budget is half of a CU's LDS (two workgroups per CU; only what the
    // schedule needs is allocated).
    const int ls = sh.ls;
    const int es = fp32() ? 4 : 8;   // staged values are held in the storage type
    const int levels = sched_ok ? sched.max_levels : 0;
    const int limit = lds_limit();
    const int dflt = std::min(limit, 81920);
    const int total = tuning.lds_bytes == 0 ? dflt : std::min(std::abs(tuning.lds_bytes), limit);
    const int pair = sched_ok ? sched.max_ghost_pair : 0;
    int ring = 1;
    while (ring < pair) ring <<= 1;
    if ((int64_t)ring * ls * es <= total / 2) {
        sh.gring = ring;
        sh.gcap = sched_ok ? sched.max_ghosts : 0;
    } else {
        ring = 2;
        while ((int64_t)ring * 2 * ls * es <= total / 4) ring <<= 1;
        sh.gring = ring;
        sh.gcap = ring / 2;
    }
    const SweepLdsLayout lay = sweep_lds_layout(levels, sh.gring, ls, es);
    if ((int64_t)(lay.ring_off + ls) * es > limit)
        throw Error(NBTE_ERR_INVALID_ARG, "sweep level tables do not fit in LDS; use fewer bands per block");
    const int budget = (tuning.lds_bytes == 0 ? dflt : std::min(tuning.lds_bytes, limit)) - lay.ring_off * es;
    sh.slots = tuning.lds_bytes < 0 ? 0 : std::max(budget, 0) / (ls * es);
    return sh;
}

// The sweep addresses its streams, the boundary inflow and a direction's
// slice of the distribution through buffer descriptors and 32-bit byte
// offsets (row offsets in scalar registers, lane offsets in vector
// registers), so every one of those extents must stay below 4 GiB; stream
// positions are int32.  Checked on the sizes alone, before anything is
// built, with the fan-in bound of the cell type (the streams hold 2, 3 or 5
// reference rows).
void nbte_problem::check_addressable(int prec) const {
    if (!have_bands || !have_quad) return;
    const int64_t N = mesh->N, F = mesh->F, B = bands.B, D = quad.D, NBF = mesh->NBF;
    const int64_t es = prec == NBTE_PREC_MIXED ? 4 : 8;
    const int64_t mi = F - 1 <= 2 ? 2 : (F - 1 == 3 ? 3 : 5);
    const int64_t DN = D * N;
    const int64_t lim = (int64_t)1 << 32;
    struct Extent {
        const char *what;
        int64_t bytes;
    } ext[] = {{"real-valued sweep streams", (3 + mi) * DN * es},
               {"integer sweep streams", (2 + mi) * DN * 4},
               {"one direction's distribution slice", N * B * es},
               {"boundary inflow rows", NBF * D * B * es}};
    for (const Extent &e : ext)
        if (e.bytes >= lim)
            throw Error(NBTE_ERR_INVALID_ARG,
                        std::string("problem too large for the sweep's 32-bit buffer offsets: ") + e.what + " take " +
                            std::to_string(e.bytes) + " bytes (limit 4 GiB) at " +
                            (prec == NBTE_PREC_MIXED ? "mixed" : "FP64") + " precision");
    if (DN >= (int64_t)INT32_MAX)
        throw Error(NBTE_ERR_INVALID_ARG, "problem too large: directions x cells must stay below 2^31");
}

// Host-side setup products (no device access): schedules, sweep program,
// boundary plan, diffusion operator.  Throws the validation errors of the ABI.
void nbte_problem::build_host() {
    if (!have_bands || !have_quad || !have_bcs)
        throw Error(NBTE_ERR_STATE, "set_bands, set_quadrature and set_boundaries must precede the solve");
    const Mesh &m = *mesh;
    if (!sched_ok) {
        sched = build_schedule(m, quad);
        sched_ok = true;
        sched_up = false;
        slots_for_cap = -2;
    }
    shape = resolve_shape();
    const int ls = shape.ls, es = fp32() ? 4 : 8;
    if (slots_for_cap != shape.slots || prog_B != bands.B || prog_gcap != shape.gcap || prog_gring != shape.gring ||
        prog_ls != ls || prog_es != es) {
        if (slots_for_cap != shape.slots) {
            if (shape.slots > 0) assign_slots(m, quad, sched, shape.slots);
            else sched.slot.clear(), sched.max_slots = 0, sched.spilled = 0;
            slots_for_cap = shape.slots;
        }
        // references are encoded as LDS offsets of this launch shape and precision
        prog = build_program(m, quad, sched, bands.B, shape.gcap, shape.gring, ls, es);
        prog_B = bands.B;
        prog_gcap = shape.gcap;
        prog_gring = shape.gring;
        prog_ls = ls;
        prog_es = es;
        sched_up = false;
    }
    if (!plan_ok) {
        plan = build_boundary_plan(m, quad, bcs, T_ref);
        plan_ok = true;
        plan_up = false;
        diff_ok = false;
    }
    if (!plan.has_thermalizing)
        throw Error(NBTE_ERR_ILL_POSED, "no thermalizing wall: the steady problem has no unique solution");
    if (!diff_ok) {
        diff = build_diffusion(m, bands, quad, plan);
        diff_ok = true;
        diff_up = false;
    }
}

void nbte_problem::upload_device() {
    require_gfx950();
    if (!stream) {
        // the null stream cannot be captured into a graph; a blocking stream
        // still orders with the caller's null-stream work
        NBTE_HIP(hipStreamCreate(&own_stream));
        stream = own_stream;
    }
    const Mesh &m = *mesh;
    if (!geom_ok) {
        upload(d_nbr, m.nbr, stream);
        upload(d_V, m.V, stream);
        upload(d_bf_owner, m.bf_owner, stream);
        // the boundary-owner cells in ascending order (their boundary rows)
        std::vector<int32_t> bown(m.N, -1);
        for (int64_t bf = 0; bf < m.NBF; ++bf) bown[m.bf_owner[bf]] = 0;
        int32_t k = 0;
        for (int64_t c = 0; c < m.N; ++c)
            if (bown[c] == 0) bown[c] = k++;
        std::vector<int32_t> bf_brow(std::max<int64_t>(m.NBF, 1), 0);
        for (int64_t bf = 0; bf < m.NBF; ++bf) bf_brow[bf] = bown[m.bf_owner[bf]];
        upload(d_bf_brow, bf_brow, stream);
        NBTE_HIP(hipStreamSynchronize(stream));   // the host copy goes out of scope
        geom_ok = true;
    }
    if (!sched_up) {
        upload(d_lvl_ptr, sched.lvl_ptr, stream);
        upload(d_lvl_off, sched.lvl_off, stream);
        const int64_t DN = stream_DN();
        d_pint.alloc((size_t)(2 + prog.maxin) * DN * 4);
        NBTE_HIP(hipMemcpyAsync(d_pint.as<int32_t>(), prog.cell.data(), DN * 4, hipMemcpyHostToDevice, stream));
        NBTE_HIP(hipMemcpyAsync(d_pint.as<int32_t>() + DN, prog.slot.data(), DN * 4, hipMemcpyHostToDevice, stream));
        NBTE_HIP(hipMemcpyAsync(d_pint.as<int32_t>() + 2 * DN, prog.ref.data(), prog.maxin * DN * 4,
                                hipMemcpyHostToDevice, stream));
        upload(d_pupc, prog.upc, stream);
        coef_prec = -1;
        upload(d_gptr, prog.gptr, stream);
        upload(d_inrow, prog.in_row, stream);
        upload(d_lag, prog.lag, stream);
        {
            // stream position of every cell in each direction (the distribution's row index)
            std::vector<int32_t> pos((size_t)DN);
            for (int64_t at = 0; at < DN; ++at) pos[(size_t)((at / m.N) * m.N + sched.perm[at])] = (int32_t)(at % m.N);
            upload(d_pos, pos, stream);
            NBTE_HIP(hipStreamSynchronize(stream));   // the host copy goes out of scope
        }
        NBTE_HIP(hipStreamSynchronize(stream));   // the program may be rebuilt (host copies replaced) after this
        sched_up = true;
        pbrow_ok = false;
    }
    if (!plan_up) {
        upload(d_bf_kind, plan.kind, stream);
        upload(d_mirror, plan.mirror, stream);
        upload(d_bf_thw, plan.theta_w, stream);
        upload(d_bf_p, plan.p, stream);
        upload(d_sdotS, plan.sdotS, stream);
        upload(d_win, plan.win, stream);
        // cells owning a reflective face (the correction's wall term) and
        // the slots of their reflective faces, in the cell's face order
        std::vector<int32_t> wall, wptr(1, 0), wslot(std::max<int64_t>(m.NBF, 1), -1);
        for (int64_t c = 0; c < m.N; ++c) {
            const int32_t j0 = wptr.back();
            int32_t j = j0;
            for (int f = 0; f < m.F; ++f) {
                const int32_t n = m.nbr[c * m.F + f];
                if (n < 0 && plan.kind[-n - 1] != NBTE_BC_THERMALIZING) wslot[-n - 1] = j++;
            }
            if (j > j0) {
                wall.push_back((int32_t)c);
                wptr.push_back(j);
            }
        }
        n_wall = (int64_t)wall.size();
        n_wall_faces = wptr.back();
        upload(d_wall, wall, stream);
        upload(d_wall_ptr, wptr, stream);
        upload(d_wslot, wslot, stream);
        plan_up = true;
    }

    if (!tables_ok) {
        const int B = bands.B, D = quad.D;
        std::vector<double> Cw(B), src(B), itau(B);
        for (int l = 0; l < B; ++l) {
            Cw[l] = bands.C[l] / quad.W;
            src[l] = bands.C[l] / (bands.C_tot * quad.W);
            itau[l] = 1.0 / bands.tau[l];
        }
        // q of a pure equilibrium field: theta * sum_l v_l C_l/W * sum_i w_i s_i (0 for a symmetric set)
        std::vector<double> qb(3, 0.0);
        double vcw = 0;
        for (int l = 0; l < B; ++l) vcw += bands.v[l] * Cw[l];
        for (int i = 0; i < D; ++i)
            for (int ax = 0; ax < 3; ++ax) qb[ax] += quad.w[i] * quad.s[3 * i + ax];
        for (double &x : qb) x *= vcw;
        upload(d_Cw, Cw, stream);
        upload(d_src, src, stream);
        upload(d_vel, bands.v, stream);
        upload(d_itau, itau, stream);
        upload(d_dirs, quad.s, stream);
        upload(d_w, quad.w, stream);
        upload(d_qbias, qb, stream);
        tables_ok = true;
    }
    if (!diff_up) {
        std::vector<double> dinv(m.N);
        for (int64_t c = 0; c < m.N; ++c) dinv[c] = 1.0 / diff.val[diff.row_ptr[c]];
        upload(d_Lrow, diff.row_ptr, stream);
        upload(d_Lcol, diff.col, stream);
        upload(d_Lval, diff.val, stream);
        upload(d_Ldinv, dinv, stream);
        {
            // ELL copy of the matrix for the multi-workgroup CG, scaled A D^-1
            const int64_t N = m.N;
            int W = 1;
            for (int64_t c = 0; c < N; ++c) W = std::max<int>(W, diff.row_ptr[c + 1] - diff.row_ptr[c]);
            if (W > 8) throw Error(NBTE_ERR_MESH, "cells with more than 7 faces are not supported");
            W = W <= 4 ? 4 : (W == 5 ? 5 : (W <= 7 ? 7 : 8));   // the kernel variants read every slot
            std::vector<int32_t> ecol((size_t)W * N);
            std::vector<double> eval((size_t)W * N, 0.0);
            for (int64_t c = 0; c < N; ++c)
                for (int s = 0; s < W; ++s) {
                    const int64_t q = diff.row_ptr[c] + s;
                    const bool used = q < diff.row_ptr[c + 1];
                    ecol[(size_t)s * N + c] = used ? diff.col[q] : (int32_t)c;
                    eval[(size_t)s * N + c] = used ? diff.val[q] * dinv[diff.col[q]] : 0.0;
                }
            upload(d_Ecol, ecol, stream);
            upload(d_Eval, eval, stream);
            NBTE_HIP(hipStreamSynchronize(stream));   // the host copies go out of scope
            ell_w = W;
        }
        pcg_nblk = (int)std::min<int64_t>(256, cdiv(m.N, 256));
        d_pcg_vec.alloc(7 * m.N * sizeof(double));
        d_pcg_part.alloc(4 * 256 * sizeof(double));
        d_pcg_scal.alloc(16 * sizeof(double));
        diff_up = true;
    }
    NBTE_HIP(hipStreamSynchronize(stream));
}

int64_t nbte_problem::accel_rows() const {
    const int64_t ghosts = prog_B > 0 ? (int64_t)prog.ghost_src.size() : mesh->NBF * quad.D;   // incoming pairs
    return std::max<int64_t>(ghosts, 1) * bands.B;
}

int64_t nbte_problem::state_bytes(int prec, int ord) const {
    const int64_t N = mesh->N, NBF = mesh->NBF, B = bands.B, D = quad.D;
    const int64_t es = prec == NBTE_PREC_MIXED ? 4 : 8;
    int64_t so2 = 0;
    if (ord == 2)   // gradient planes, correction, two boundary increment slots; weights and geometry
        so2 = 4 * D * N * B * es + 2 * NBF * D * B * es + (int64_t)mesh->F * N * 9 * 8 + N * 3 * 8 + NBF * 4;
    if (bicg())     // BiCGSTAB work vectors and the geometry it reads
        so2 += 9 * D * B * N * 8 + (ord == 2 ? 0 : (int64_t)mesh->F * N * 9 * 8 + N * 3 * 8 + NBF * 4);
    const int64_t ghosts = prog_B > 0 ? (int64_t)prog.ghost_src.size() : NBF * D;   // incoming pairs
    int64_t acc = 0;
    if (accel_m() > 0) {
        const int64_t NR = accel_rows(), NS = N + NR;
        // inflow of x and two images, theta part of G, previous f, columns, partials, row index (NR bounds
        // the state's inflow entries: thermalizing faces' rows are left out)
        acc = 3 * NR * 8 + N * 8 + NS * es + 2 * (int64_t)accel_m() * NS * es + 1024 * 2 * kAccelMaxDepth * 8 + 1024 +
              NBF * D * 4;
    }
    // plane layout: the reductions' band sums and the boundary rows
    const int64_t pl = planes_for(ord) ? D * N * (24 + 4) + std::max<int64_t>(boundary_owners(), 1) * D * B * es : 0;
    return D * N * B * es + std::max<int64_t>(ghosts, 1) * B * es + 2 * D * N * es + pl + NBF * (B + 3) * 8 +
           N * 8 * 10 + 1024 + acc + so2;
}

void nbte_problem::allocate_state(int prec) {
    const int64_t N = mesh->N, NBF = mesh->NBF, B = bands.B, D = quad.D;
    const int64_t es = prec == NBTE_PREC_MIXED ? 4 : 8;
    d_g.alloc(D * N * B * es);
    d_gval.alloc(std::max<int64_t>((int64_t)prog.ghost_src.size() * B, 1) * es);
    const int64_t DN = D * N;
    void *before = d_tstream.ptr;
    d_tstream.alloc((size_t)(3 + prog.maxin) * DN * es);
    if (coef_prec != prec || d_tstream.ptr != before) {
        // outflow sums (row 0) and coefficients (rows 3..) in the storage type
        auto put = [&](int row, const std::vector<double> &h) {
            if (prec == NBTE_PREC_MIXED) {
                std::vector<float> f(h.begin(), h.end());
                NBTE_HIP(hipMemcpyAsync(t_row(row), f.data(), f.size() * 4, hipMemcpyHostToDevice, stream));
                NBTE_HIP(hipStreamSynchronize(stream));   // the host copy goes out of scope
            } else {
                NBTE_HIP(hipMemcpyAsync(t_row(row), h.data(), h.size() * 8, hipMemcpyHostToDevice, stream));
            }
        };
        put(0, prog.sout);
        put(3, prog.coef);
        coef_prec = prec;
    }
    d_Jw.alloc(std::max<int64_t>(NBF, 1) * 8);
    d_Jin.alloc(std::max<int64_t>(NBF, 1) * 8);
    d_wallJ.alloc(std::max<int64_t>(n_wall_faces, 1) * 8);
    d_bsum.alloc(std::max<int64_t>(NBF, 1) * B * 8);
    d_Q.alloc(N * 8);
    for (auto &t : d_theta) t.alloc(N * 8);
    d_theta_seq.alloc(N * 8);
    d_thetaE.alloc(N * 8);
    d_q.alloc(3 * N * 8);
    d_rhs.alloc(N * 8);
    d_delta.alloc(N * 8);
    if (planes()) {
        d_mom.alloc((size_t)D * N * sizeof(Mom3));
        d_brow.alloc((size_t)std::max<int64_t>(boundary_owners(), 1) * D * B * es);
        if (!pbrow_ok) {
            // the boundary row each stream position copies its values into:
            // the row (owner, i) of a cell that owns a boundary face through
            // which direction i leaves (the only directions the boundary
            // kernels read), -1 elsewhere
            const Mesh &m = *mesh;
            std::vector<int32_t> bown(m.N, -1), pb((size_t)D * N, -1);
            int32_t k = 0;
            for (int64_t bf = 0; bf < m.NBF; ++bf) bown[m.bf_owner[bf]] = 0;
            for (int64_t c = 0; c < N; ++c)
                if (bown[c] == 0) bown[c] = k++;
            std::vector<int32_t> pos((size_t)D * N);
            for (int64_t at = 0; at < D * N; ++at) pos[(size_t)((at / N) * N + sched.perm[at])] = (int32_t)(at % N);
            for (int64_t bf = 0; bf < m.NBF; ++bf) {
                const int64_t c = m.bf_owner[bf];
                const double *S = &m.S[((int64_t)c * m.F + m.bf_local[bf]) * 3];
                for (int64_t i = 0; i < D; ++i) {
                    const double *si = &quad.s[3 * i];
                    if (si[0] * S[0] + si[1] * S[1] + si[2] * S[2] > 0.0)
                        pb[(size_t)(i * N + pos[(size_t)(i * N + c)])] = (int32_t)(bown[c] * D + i);
                }
            }
            upload(d_pbrow, pb, stream);
            NBTE_HIP(hipStreamSynchronize(stream));   // the host copy goes out of scope
            pbrow_ok = true;
        }
    } else {
        d_mom.release();
        d_brow.release();
        d_pbrow.release();
        pbrow_ok = false;
    }
    d_state.alloc(sizeof(SolveState));
    d_view.alloc(sizeof(DeviceView));
    if (bicg()) d_bicg.alloc((size_t)9 * D * B * N * 8);
    else d_bicg.release();
    if (order == 2 || bicg()) {
        if (!lsq_up) {
            const Mesh &m = *mesh;
            upload(d_lsq, build_lsq_weights(m), stream);
            upload(d_Sv, m.S, stream);
            upload(d_xf, m.xf, stream);
            upload(d_xc, m.xc, stream);
            upload(d_bf_local, m.bf_local, stream);
            NBTE_HIP(hipStreamSynchronize(stream));   // the host copies go out of scope
            lsq_up = true;
        }
    }
    if (order == 2) {
        d_grad.alloc((size_t)3 * D * N * B * es);
        d_corr.alloc((size_t)D * N * B * es);
        d_bdelta.alloc((size_t)2 * std::max<int64_t>(NBF, 1) * D * B * es);
        so2_nblk = (int)std::min<int64_t>(4096, cdiv(D * N * B, 256));
        so2_nblk_b = (int)std::min<int64_t>(1024, cdiv(std::max<int64_t>(NBF, 1) * D * B, 256));
    } else {
        for (DevBuf *b : {&d_grad, &d_corr, &d_bdelta}) b->release();
    }
    if (accel_m() > 0) {
        // the state's inflow part: the incoming rows of the faces whose inflow
        // depends on the distribution, numbered face by face
        if ((int64_t)plan.kind.size() != NBF || (int64_t)prog.in_row.size() != NBF * D)
            throw Error(NBTE_ERR_STATE, "boundary plan or sweep program out of date");
        std::vector<int32_t> ain(std::max<int64_t>(NBF * D, 1), -1);
        int64_t rows = 0;
        for (int64_t bf = 0; bf < NBF; ++bf) {
            if (plan.kind[bf] == NBTE_BC_THERMALIZING) continue;
            for (int64_t i = 0; i < D; ++i)
                if (prog.in_row[bf * D + i] >= 0) ain[bf * D + i] = (int32_t)rows++;
        }
        acc_NR = std::max<int64_t>(rows, 1) * B;
        upload(d_acc_in, ain, stream);
        NBTE_HIP(hipStreamSynchronize(stream));   // the host copy goes out of scope
        const int64_t NR = acc_NR, NS = N + NR;
        d_acc_x.alloc(NR * 8);
        d_acc_G.alloc(2 * NR * 8);
        d_acc_fprev.alloc(NS * es);
        d_acc_Gprev.alloc(N * 8);
        d_acc_dF.alloc((size_t)accel_m() * NS * es);
        d_acc_dG.alloc((size_t)accel_m() * NS * es);
        acc_nblk = (int)std::min<int64_t>(1024, cdiv(NS, 256));
        d_acc_part.alloc((size_t)acc_nblk * 2 * kAccelMaxDepth * 8);
        d_acc_scal.alloc((1 + kAccelMaxDepth * kAccelMaxDepth + kAccelMaxDepth) * 8);
    } else {
        for (DevBuf *b :
             {&d_acc_x, &d_acc_G, &d_acc_fprev, &d_acc_Gprev, &d_acc_dF, &d_acc_dG, &d_acc_part, &d_acc_scal, &d_acc_in})
            b->release();
        acc_NR = 0;
    }
}

int64_t nbte_problem::device_bytes() const {
    int64_t s = 0;
    for (const DevBuf *b :
         {&d_nbr, &d_V, &d_lvl_ptr, &d_lvl_off, &d_gptr, &d_pint, &d_pupc, &d_tstream, &d_inrow, &d_lag, &d_Cw, &d_src, &d_vel, &d_itau, &d_dirs, &d_w, &d_qbias, &d_bf_owner, &d_bf_kind,
          &d_mirror, &d_wall, &d_wall_ptr, &d_wslot, &d_wallJ, &d_bf_thw, &d_bf_p, &d_sdotS, &d_win, &d_Lrow, &d_Lcol, &d_Lval, &d_Ldinv, &d_Ecol, &d_Eval, &d_g, &d_gval,
          &d_Jw, &d_Jin, &d_bsum, &d_Q, &d_theta[0], &d_theta[1], &d_theta[2], &d_theta_seq, &d_thetaE, &d_q, &d_rhs, &d_delta,
          &d_pcg_vec, &d_pcg_part, &d_pcg_scal, &d_view, &d_state, &d_self_work, &d_acc_x, &d_acc_G, &d_acc_fprev,
          &d_acc_Gprev, &d_acc_dF, &d_acc_dG, &d_acc_part, &d_acc_scal, &d_acc_in, &d_lsq, &d_Sv, &d_xf, &d_xc, &d_bf_local,
          &d_grad, &d_corr, &d_bdelta, &d_bicg, &d_pos, &d_bf_brow, &d_brow, &d_mom, &d_pbrow})
        s += (int64_t)b->bytes;
    return s;
}

void nbte_problem::make_view() {
    DeviceView v{};
    v.N = mesh->N;
    v.F = mesh->F;
    v.B = bands.B;
    v.D = quad.D;
    v.fp32 = fp32() ? 1 : 0;
    v.NBF = mesh->NBF;
    v.scheme = scheme;
    v.mom_lpc = mom_lpc();
    v.planes = planes() ? 1 : 0;
    v.nbr = d_nbr.as<int32_t>();
    v.V = d_V.as<double>();
    v.maxin = prog.maxin;
    v.max_levels = sched.max_levels;
    v.lpc = shape.lpc;
    v.bpb = shape.bpb;
    v.gcap = shape.gcap;
    v.gring = shape.gring;
    v.lstride = shape.ls;
    v.lvl_ptr = d_lvl_ptr.as<int32_t>();
    v.lvl_off = d_lvl_off.as<int32_t>();
    v.gptr = d_gptr.as<int32_t>();
    v.p_cell = d_pint.as<int32_t>();
    v.p_slot = d_pint.as<int32_t>() + stream_DN();
    v.p_ref = d_pint.as<int32_t>() + 2 * stream_DN();
    v.p_upc = d_pupc.as<int32_t>();
    v.t_sout = t_row(0);
    v.t_dc = t_row(1);
    v.t_q = t_row(2);
    v.t_coef = t_row(3);
    v.Cw = d_Cw.as<double>();
    v.src = d_src.as<double>();
    v.vel = d_vel.as<double>();
    v.inv_tau = d_itau.as<double>();
    v.beta = bands.beta;
    v.C_tot = bands.C_tot;
    v.dirs = d_dirs.as<double>();
    v.w = d_w.as<double>();
    v.qbias = d_qbias.as<double>();
    v.bf_owner = d_bf_owner.as<int32_t>();
    v.bf_kind = d_bf_kind.as<int32_t>();
    v.mirror = d_mirror.as<int32_t>();
    v.wall_cell = d_wall.as<int32_t>();
    v.wall_ptr = d_wall_ptr.as<int32_t>();
    v.wslot = d_wslot.as<int32_t>();
    v.wallJ = d_wallJ.as<double>();
    v.n_wall = n_wall;
    v.in_row = d_inrow.as<int32_t>();
    v.n_lag = (int64_t)prog.lag.size() / 4;
    v.lag = d_lag.as<int32_t>();
    v.bf_thw = d_bf_thw.as<double>();
    v.bf_p = d_bf_p.as<double>();
    v.sdotS = d_sdotS.as<double>();
    v.win = d_win.as<double>();
    v.g = d_g.ptr;
    v.pos = d_pos.as<int32_t>();
    v.p_brow = d_pbrow.as<int32_t>();
    v.brow = d_brow.ptr;
    v.mom = d_mom.ptr;
    v.bf_brow = d_bf_brow.as<int32_t>();
    v.gval = d_gval.ptr;
    v.Jw = d_Jw.as<double>();
    v.Jin = d_Jin.as<double>();
    v.bsum = d_bsum.as<double>();
    for (int k = 0; k < 3; ++k) v.theta[k] = d_theta[k].as<double>();
    v.theta_seq = d_theta_seq.as<double>();
    v.thetaE = d_thetaE.as<double>();
    v.q = d_q.as<double>();
    v.rhs = d_rhs.as<double>();
    v.delta = d_delta.as<double>();
    v.state = d_state.as<SolveState>();
    PcgWork &w = v.pcg;
    w.n = mesh->N;
    w.nblk = pcg_nblk;
    w.max_iter = cg_max_iter();
    w.rtol2 = cg_rtol() * cg_rtol();
    w.row_ptr = d_Lrow.as<int32_t>();
    w.col = d_Lcol.as<int32_t>();
    w.val = d_Lval.as<double>();
    w.dinv = d_Ldinv.as<double>();
    w.ell_w = ell_w;
    w.ecol = d_Ecol.as<int32_t>();
    w.eval = d_Eval.as<double>();
    w.vec = d_pcg_vec.as<double>();
    w.partial = d_pcg_part.as<double>();
    w.scal = d_pcg_scal.as<double>();
    AccelWork &a = v.acc;
    a.m = accel_m();
    a.nblk = acc_nblk;
    a.NR = a.m > 0 ? acc_NR : 0;
    a.in = d_acc_in.as<int32_t>();
    a.ain_x = d_acc_x.as<double>();
    a.ain_G = d_acc_G.as<double>();
    a.fprev = d_acc_fprev.ptr;
    a.Gprev = d_acc_Gprev.as<double>();
    a.dF = d_acc_dF.ptr;
    a.dG = d_acc_dG.ptr;
    a.part = d_acc_part.as<double>();
    a.scal = d_acc_scal.as<double>();
    v.order = order;
    v.lsq = d_lsq.as<double>();
    v.Sv = d_Sv.as<double>();
    v.xf = d_xf.as<double>();
    v.xc = d_xc.as<double>();
    v.bf_local = d_bf_local.as<int32_t>();
    v.grad = d_grad.ptr;
    v.corr = d_corr.ptr;
    v.bdelta = d_bdelta.ptr;
    v.bicg = d_bicg.as<double>();
    v.bicg_max_iter = tuning.inner_max_iter > 0 ? tuning.inner_max_iter : 500;
    v.bicg_rtol = tuning.inner_rtol > 0 ? tuning.inner_rtol : 1e-13;
    v.Qc = d_Q.as<double>();
    hv = v;
}

void nbte_problem::prepare(const double *Q_cell, const nbte_solve_opts &o) {
    if (batch) throw Error(NBTE_ERR_STATE, "the problem is a batch member; remove it from the batch first");
    if (o.precision != NBTE_PREC_FP64 && o.precision != NBTE_PREC_MIXED) throw Error(NBTE_ERR_INVALID_ARG, "bad precision");
    if (o.scheme < 0 || o.scheme > 2) throw Error(NBTE_ERR_INVALID_ARG, "bad scheme");
    if (o.spatial_order != 1 && o.spatial_order != 2) throw Error(NBTE_ERR_INVALID_ARG, "spatial_order must be 1 or 2");
    if (o.spatial_order == 2 && accel_m() > 0)
        throw Error(NBTE_ERR_INVALID_ARG, "the second-order scheme is not combined with Anderson acceleration");
    if (o.spatial_order == 2 && bicg())
        throw Error(NBTE_ERR_INVALID_ARG, "the BiCGSTAB inner solver solves the first-order systems only");
    if (!std::isfinite(o.T_ref)) throw Error(NBTE_ERR_INVALID_ARG, "bad T_ref");
    if (o.T_ref != T_ref) {
        T_ref = o.T_ref;
        plan_ok = false;  // wall temperatures are stored relative to T_ref
    }
    const Mesh &m = *mesh;
    std::vector<double> Q(m.N, 0.0);
    if (Q_cell)
        for (int64_t c = 0; c < m.N; ++c) {
            if (!std::isfinite(Q_cell[c])) throw Error(NBTE_ERR_INVALID_ARG, "non-finite heat source");
            Q[c] = Q_cell[c];
        }
    std::vector<double> t0;
    if (o.T_init) {
        t0.resize(m.N);
        for (int64_t c = 0; c < m.N; ++c) {
            if (!std::isfinite(o.T_init[c])) throw Error(NBTE_ERR_INVALID_ARG, "non-finite T_init");
            t0[c] = o.T_init[c] - T_ref;
        }
    }
    check_addressable(o.precision);
    prepared = false;
    precision = o.precision;   // the launch shape's LDS budget depends on it
    order = o.spatial_order;   // so does its bands per lane
    ensure_setup();
    if (!prog.lag.empty() && accel_m() > 0)
        throw Error(NBTE_ERR_INVALID_ARG, "Anderson acceleration is not provided for meshes with lagged (cyclic) faces");
    scheme = o.scheme;
    time_phases = o.time_phases;
    allocate_state(precision);
    heat_in = 0.0;
    for (int64_t c = 0; c < m.N; ++c) heat_in += m.V[c] * Q[c];
    make_view();
    NBTE_HIP(hipMemcpyAsync(d_view.ptr, &hv, sizeof(DeviceView), hipMemcpyHostToDevice, stream));
    // work items of the single-solve launches: [one][PCG workgroups][flux workgroups]
    {
        const int nf = (int)std::max<int64_t>((m.NBF + 3) / 4, 1);   // flux: a wave per boundary face
        std::vector<WorkItem> wk;
        wk.push_back({0, 0, 0, 1});
        self_pcg = (int)wk.size();
        for (int b = 0; b < pcg_nblk; ++b) wk.push_back({0, 0, b, pcg_nblk});
        n_self_pcg = pcg_nblk;
        self_flux = (int)wk.size();
        for (int b = 0; b < nf; ++b) wk.push_back({0, 0, b, nf});
        n_self_flux = nf;
        self_acc = (int)wk.size();   // stage items of kind 3: the initial inflow state
        for (int b = 0; b < nf; ++b) wk.push_back({0, 3, b, nf});
        n_self_acc = nf;
        self_so2 = (int)wk.size();   // second order: gradient items, then correction and boundary items
        for (int b = 0; b < so2_nblk; ++b) wk.push_back({0, 0, b, so2_nblk});
        for (int b = 0; b < so2_nblk; ++b) wk.push_back({0, 0, b, so2_nblk});
        for (int b = 0; b < so2_nblk_b; ++b) wk.push_back({0, 1, b, so2_nblk_b});
        upload(d_self_work, wk, stream);
        NBTE_HIP(hipStreamSynchronize(stream));
    }
    SolveState s0{};
    s0.max_iter = o.max_iter;
    s0.tol = o.tol;
    s0.best = INFINITY;
    NBTE_HIP(hipMemcpyAsync(d_state.ptr, &s0, sizeof(s0), hipMemcpyHostToDevice, stream));
    NBTE_HIP(hipMemcpyAsync(d_Q.ptr, Q.data(), m.N * 8, hipMemcpyHostToDevice, stream));
    launch_gather((int64_t)quad.D * m.N, p_cell(), d_Q.as<double>(), t_row(2), fp32(), stream);
    double *th0 = d_theta[0].as<double>();   // theta[cur] at rotation 0
    if (o.T_init) {
        NBTE_HIP(hipMemcpyAsync(th0, t0.data(), m.N * 8, hipMemcpyHostToDevice, stream));
    } else {
        // Fourier initial guess: L theta = V Qdot + wall data
        std::vector<double> b(m.N);
        for (int64_t c = 0; c < m.N; ++c) b[c] = m.V[c] * Q[c] + diff.dir_rhs[c];
        NBTE_HIP(hipMemcpyAsync(d_rhs.ptr, b.data(), m.N * 8, hipMemcpyHostToDevice, stream));
        const DeviceView *vp = d_view.as<DeviceView>();
        const WorkItem *wk = d_self_work.as<WorkItem>();
        if (m.N <= kPcgBlockMaxRows)
            launch_pcg_block(vp, wk + self_one, 1, 1, stream);
        else {
            // in chunks, stopping once the sticky converged flag is set (the
            // launches after convergence would return at once but still cost
            // their launch time).  A chunk's flag is read while the next chunk
            // runs, so the device never waits for the host between chunks; at
            // most one chunk of such early-returning launches follows.
            const int limit = std::max(1000, (int)std::sqrt((double)m.N) * 20), chunk = 64;
            if (!h_pcg_flag) {
                NBTE_HIP(hipHostMalloc(reinterpret_cast<void **>(&h_pcg_flag), 2 * sizeof(double), hipHostMallocDefault));
                for (auto &e : pcg_ev) NBTE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            }
            for (int k0 = 0, c = 0; k0 < limit; k0 += chunk, ++c) {
                launch_pcg_multi(vp, wk + self_pcg, n_self_pcg, 1, std::min(chunk, limit - k0), stream, k0, k0 == 0);
                NBTE_HIP(hipMemcpyAsync(h_pcg_flag + (c & 1), d_pcg_scal.as<double>() + 4, sizeof(double),
                                        hipMemcpyDeviceToHost, stream));
                NBTE_HIP(hipEventRecord(pcg_ev[c & 1], stream));
                if (c > 0) {
                    NBTE_HIP(hipEventSynchronize(pcg_ev[(c - 1) & 1]));
                    if (h_pcg_flag[(c - 1) & 1] != 0.0) break;
                }
            }
        }
    }
    // g = 0 is equilibrium at theta^0; the stored g is relative to theta[prev]
    NBTE_HIP(hipMemcpyAsync(d_theta[1].ptr, th0, m.N * 8, hipMemcpyDeviceToDevice, stream));
    launch_fill_zero(d_g.ptr, d_g.bytes, stream);
    launch_fill_zero(d_brow.ptr, d_brow.bytes, stream);
    launch_fill_zero(d_gval.ptr, d_gval.bytes, stream);
    if (order == 2) {
        // the initial distribution's gradients, the first sweep's correction and
        // the increments of its outgoing boundary values (slot 0)
        const WorkItem *w2 = d_self_work.as<WorkItem>() + self_so2;
        launch_grad(d_view.as<DeviceView>(), w2, so2_nblk, fp32(), 1, stream);
        launch_recon(d_view.as<DeviceView>(), w2 + so2_nblk, so2_nblk + so2_nblk_b, fp32(), 1, stream);
    }
    // the first boundary stage's diffuse sums, from the initial distribution
    launch_flux(d_view.as<DeviceView>(), d_self_work.as<WorkItem>() + self_flux, n_self_flux, fp32(), 2, stream);
    if (accel_m() > 0) {
        // the accelerated iteration starts from the initial state's inflow, with no
        // history; the inflow buffers start at zero (with only thermalizing faces
        // the state keeps one placeholder row that no stage writes)
        launch_fill_zero(d_acc_scal.ptr, d_acc_scal.bytes, stream);
        launch_fill_zero(d_acc_x.ptr, d_acc_x.bytes, stream);
        launch_fill_zero(d_acc_G.ptr, d_acc_G.bytes, stream);
        launch_stage(d_view.as<DeviceView>(), d_self_work.as<WorkItem>() + self_acc, n_self_acc, fp32(), stream);
    }
    NBTE_HIP(hipGetLastError());
    NBTE_HIP(hipStreamSynchronize(stream));
    hs = s0;
    stop_mode = 0;
    stop_tol = o.tol;
    stop_max_iter = o.max_iter;
    refine = o.refine != 0;
    refined_at = -1;
    if (!solo) solo = std::make_unique<Runner>(stream);
    solo->set_members({this});
    solo->set_timing(time_phases != 0);
    solo->set_graphs(!tuning.no_graphs);
    solo->reset_timing();
    stats = nbte_stats{};
    prepared = true;
}

void nbte_problem::set_controls(int stop, double tol, int max_iter) {
    const int patience = (stop && refine && refine_possible()) ? 64 : 0;
    launch_set_controls(d_state.as<SolveState>(), stop, tol, max_iter, patience, stream);
    NBTE_HIP(hipGetLastError());
    NBTE_HIP(hipStreamSynchronize(stream));
    stop_mode = stop;
    stop_tol = tol;
    stop_max_iter = max_iter;
    hs.done = 0;
}

void nbte_problem::promote() {
    if (!fp32()) return;
    try {
        check_addressable(NBTE_PREC_FP64);
    } catch (const Error &e) {
        throw Error(NBTE_ERR_NOT_CONVERGED, std::string("the FP32 iteration stalled at residual ") +
                                                std::to_string(hs.residual) + " and FP64 refinement is not possible: " +
                                                e.what());
    }
    NBTE_HIP(hipStreamSynchronize(stream));
    DevBuf old_g, old_brow;   // the FP32 distribution (and boundary rows), widened into the new FP64 ones below
    std::swap(old_g.ptr, d_g.ptr);
    std::swap(old_g.bytes, d_g.bytes);
    std::swap(old_brow.ptr, d_brow.ptr);
    std::swap(old_brow.bytes, d_brow.bytes);
    const int bpb_fp32 = shape.bpb;   // its band-block planes (plane layout)
    precision = NBTE_PREC_FP64;
    ensure_setup();   // launch shape and slot table for FP64 staged values
    allocate_state(precision);
    if (planes()) {   // the planes of the FP64 launch shape, and the boundary rows
        launch_widen(quad.D, mesh->N, bands.B, old_g.as<float>(), bpb_fp32, d_g.as<double>(), shape.bpb, stream);
        launch_widen_flat((int64_t)old_brow.bytes / 4, old_brow.as<float>(), d_brow.as<double>(), stream);
    } else {
        launch_widen_flat((int64_t)old_g.bytes / 4, old_g.as<float>(), d_g.as<double>(), stream);
    }
    launch_gather((int64_t)quad.D * mesh->N, p_cell(), d_Q.as<double>(), t_row(2), false, stream);
    make_view();
    NBTE_HIP(hipMemcpyAsync(d_view.ptr, &hv, sizeof(DeviceView), hipMemcpyHostToDevice, stream));
    if (order == 2) {
        // the FP64 copies of the gradients, the next sweep's correction and the
        // boundary increments of the distribution the next stage reads
        const WorkItem *w2 = d_self_work.as<WorkItem>() + self_so2;
        launch_grad(d_view.as<DeviceView>(), w2, so2_nblk, fp32(), 2, stream);
        launch_recon(d_view.as<DeviceView>(), w2 + so2_nblk, so2_nblk + so2_nblk_b, fp32(), 2, stream);
    }
    if (accel_m() > 0) {
        // the acceleration restarts, in FP64 columns, from the last plain image:
        // theta[cur] and the inflow of the last distribution
        launch_fill_zero(d_acc_scal.ptr, d_acc_scal.bytes, stream);
        launch_stage(d_view.as<DeviceView>(), d_self_work.as<WorkItem>() + self_acc, n_self_acc, fp32(), stream);
    }
    NBTE_HIP(hipGetLastError());
    NBTE_HIP(hipStreamSynchronize(stream));
    refined_at = hs.iterations;
    set_controls(stop_mode, stop_tol, stop_max_iter);
    if (solo) solo->set_members({this});
}

void nbte_problem::sync_state() {
    if (batch) batch_sync(batch);
    else if (solo) solo->collect();
}

void nbte_problem::iterate(int n, bool check, double *res_out) {
    if (!prepared) throw Error(NBTE_ERR_STATE, "nbte_prepare must precede nbte_iterate");
    if (batch) throw Error(NBTE_ERR_STATE, "the problem is a batch member; it iterates with nbte_batch_step");
    if (stop_mode != 0 || hs.done) set_controls(0, stop_tol, stop_max_iter);
    auto t0 = std::chrono::steady_clock::now();
    solo->run(n);
    if (check) {
        solo->collect();
        if (hs.done == NBTE_DONE_DIVERGED)
            throw Error(NBTE_ERR_DIVERGED, "iteration diverged (non-finite or exploding temperature update)");
        if (res_out) *res_out = hs.residual;
    }
    stats.ms_total += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void nbte_problem::read_result(nbte_result *out) {
    if (!prepared) throw Error(NBTE_ERR_STATE, "nothing to read: call nbte_prepare first");
    sync_state();
    const Mesh &m = *mesh;
    auto put = [&](double *dst, const double *src, int64_t n, double offset) {
        if (!dst) return;
        if (out_on_device) {
            launch_affine(n, src, 1.0, offset, dst, stream);
        } else {
            std::vector<double> h(n);
            NBTE_HIP(hipMemcpyAsync(h.data(), src, n * 8, hipMemcpyDeviceToHost, stream));
            NBTE_HIP(hipStreamSynchronize(stream));
            for (int64_t k = 0; k < n; ++k) dst[k] = offset + h[k];
        }
    };
    // theta of the last update is the current one; T and q belong to the
    // last sweep, whose distribution is stored relative to theta[prev]
    put(out->T_lattice, d_theta[cur_index()].as<double>(), m.N, T_ref);
    put(out->T, d_thetaE.as<double>(), m.N, T_ref);
    put(out->q, d_q.as<double>(), 3 * m.N, 0.0);
    // energy balance from the last sweep's face values
    double defect = 0.0;
    if (m.NBF > 0 && hs.iterations > 0) {
        launch_flux(d_view.as<DeviceView>(), d_self_work.as<WorkItem>() + self_flux, n_self_flux, fp32(), 1, stream);
        std::vector<double> J(m.NBF);
        NBTE_HIP(hipMemcpyAsync(J.data(), d_Jw.ptr, m.NBF * 8, hipMemcpyDeviceToHost, stream));
        NBTE_HIP(hipStreamSynchronize(stream));
        double net = 0, tot = 0;
        for (double x : J) {
            net += x;
            tot += std::fabs(x);
        }
        double scale = std::max(std::fabs(heat_in), 0.5 * tot);
        defect = scale > 0 ? std::fabs(net - heat_in) / scale : 0.0;
    }
    NBTE_HIP(hipStreamSynchronize(stream));
    out->iterations = hs.iterations;
    out->residual = hs.iterations > 0 ? hs.residual : INFINITY;
    out->energy_defect = defect;
}

void nbte_problem::collect_stats() {
    if (prepared) sync_state();
    if (solo && !batch) {
        solo->harvest_timing();
        stats.ms_bc = solo->phase_ms[PH_BC];
        stats.ms_sweep = solo->phase_ms[PH_SWEEP];
        stats.ms_moments = solo->phase_ms[PH_MOM];
        stats.ms_synthetic = solo->phase_ms[PH_SYN];
        stats.ms_update = solo->phase_ms[PH_UPD];
        stats.sweep_launches = solo->timed_iterations;
    }
    stats.iterations = hs.iterations;
    stats.updates_per_sweep = mesh->N * (int64_t)bands.B * quad.D;
    stats.max_levels = sched_ok ? sched.max_levels : 0;
    stats.device_bytes = device_bytes();
    stats.bands_per_block = shape.bpb;
    stats.bands_per_lane = shape.bpl;
    stats.block_size = shape.block;
    stats.lds_slots = shape.slots > 0 ? sched.max_slots : 0;
    stats.spilled_values = sched.spilled;
    stats.refined_at = refined_at;
}

// ============================================================================ ABI

extern "C" {

const char *nbte_last_error(void) { return g_last_error.c_str(); }

const char *nbte_version(void) { return "nbte 0.1.0 (gfx950)"; }

nbte_status nbte_mesh_create(int32_t dim, int64_t n_nodes, const double *xyz, int32_t cell_type, int64_t n_cells,
                             const int64_t *cell_nodes, int64_t n_bfaces, const int64_t *bface_nodes,
                             const int32_t *bface_tag, nbte_mesh **out) {
    return guarded([&] {
        if (!out) throw Error(NBTE_ERR_INVALID_ARG, "out is null");
        *out = nullptr;
        auto m = build_mesh(dim, n_nodes, xyz, cell_type, n_cells, cell_nodes, n_bfaces, bface_nodes, bface_tag);
        *out = new nbte_mesh{std::move(m)};
        return NBTE_OK;
    });
}

void nbte_mesh_destroy(nbte_mesh *m) { delete m; }

nbte_status nbte_mesh_read_gmsh(const char *path, double scale, nbte_mesh **out) {
    return guarded([&] {
        if (!path || !out) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        *out = nullptr;
        auto m = read_gmsh(path, scale);
        *out = new nbte_mesh{std::move(m)};
        return NBTE_OK;
    });
}

nbte_status nbte_mesh_get_regions(const nbte_mesh *m, int32_t *region) {
    return guarded([&] {
        if (!m || !region) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        const Mesh &mm = *m->m;
        for (int64_t c = 0; c < mm.N; ++c) region[c] = mm.region.empty() ? 0 : mm.region[c];
        return NBTE_OK;
    });
}

nbte_status nbte_mesh_get_centroids(const nbte_mesh *m, double *xc) {
    return guarded([&] {
        if (!m || !xc) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        std::copy(m->m->xc.begin(), m->m->xc.end(), xc);
        return NBTE_OK;
    });
}

nbte_status nbte_mesh_get_info(const nbte_mesh *m, nbte_mesh_info *info) {
    return guarded([&] {
        if (!m || !info) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        info->dim = m->m->dim;
        info->faces_per_cell = m->m->F;
        info->n_cells = m->m->N;
        info->n_bfaces = m->m->NBF;
        info->total_volume = m->m->total_volume;
        info->max_closure_error = m->m->max_closure;
        return NBTE_OK;
    });
}

nbte_status nbte_problem_create(const nbte_mesh *m, void *hip_stream, nbte_problem **out) {
    return guarded([&] {
        if (!m || !out) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        *out = nullptr;
        auto *p = new nbte_problem();
        p->mesh = m->m;
        p->stream = static_cast<hipStream_t>(hip_stream);
        *out = p;
        return NBTE_OK;
    });
}

void nbte_problem_destroy(nbte_problem *p) { delete p; }

nbte_status nbte_set_bands(nbte_problem *p, int32_t n_bands, const double *C, const double *v, const double *tau) {
    return guarded([&] {
        if (!p || !C || !v || !tau || n_bands <= 0) throw Error(NBTE_ERR_INVALID_ARG, "bad band table arguments");
        if (p->batch) throw Error(NBTE_ERR_STATE, "the problem is a batch member");
        BandTable b;
        b.B = n_bands;
        b.C.assign(C, C + n_bands);
        b.v.assign(v, v + n_bands);
        b.tau.assign(tau, tau + n_bands);
        for (int l = 0; l < n_bands; ++l) {
            if (!(std::isfinite(C[l]) && C[l] > 0) || !(std::isfinite(v[l]) && v[l] > 0) ||
                !(std::isfinite(tau[l]) && tau[l] > 0))
                throw Error(NBTE_ERR_INVALID_ARG, "band " + std::to_string(l) + ": C, v, tau must be finite and > 0");
            b.beta += C[l] / tau[l];
            b.C_tot += C[l];
        }
        p->bands = std::move(b);
        p->have_bands = true;
        p->tables_ok = false;
        p->diff_ok = false;
        p->prepared = false;
        return NBTE_OK;
    });
}

nbte_status nbte_set_quadrature(nbte_problem *p, int32_t n_dirs, const double *s, const double *w) {
    return guarded([&] {
        if (!p || !s || !w || n_dirs <= 0) throw Error(NBTE_ERR_INVALID_ARG, "bad quadrature arguments");
        if (p->batch) throw Error(NBTE_ERR_STATE, "the problem is a batch member");
        Quadrature q;
        q.D = n_dirs;
        q.s.assign(s, s + 3 * (size_t)n_dirs);
        q.w.assign(w, w + n_dirs);
        for (int i = 0; i < n_dirs; ++i) {
            const double nrm = std::sqrt(s[3 * i] * s[3 * i] + s[3 * i + 1] * s[3 * i + 1] + s[3 * i + 2] * s[3 * i + 2]);
            if (!std::isfinite(nrm) || std::fabs(nrm - 1.0) > 1e-12)
                throw Error(NBTE_ERR_QUADRATURE, "direction " + std::to_string(i) + " is not a unit vector");
            if (!(std::isfinite(w[i]) && w[i] > 0)) throw Error(NBTE_ERR_QUADRATURE, "weights must be finite and > 0");
            q.W += w[i];
        }
        p->quad = std::move(q);
        p->have_quad = true;
        p->sched_ok = p->plan_ok = p->diff_ok = p->tables_ok = false;
        p->prepared = false;
        return NBTE_OK;
    });
}

nbte_status nbte_set_boundaries(nbte_problem *p, int32_t n, const nbte_boundary *bcs) {
    return guarded([&] {
        if (!p || !bcs || n <= 0) throw Error(NBTE_ERR_INVALID_ARG, "bad boundary arguments");
        if (p->batch) throw Error(NBTE_ERR_STATE, "the problem is a batch member");
        std::vector<nbte_boundary> v(bcs, bcs + n);
        for (size_t k = 0; k < v.size(); ++k) {
            const auto &b = v[k];
            if (b.kind < NBTE_BC_THERMALIZING || b.kind > NBTE_BC_PARTIAL)
                throw Error(NBTE_ERR_BOUNDARY, "unknown boundary kind for tag " + std::to_string(b.tag));
            if (b.kind == NBTE_BC_THERMALIZING && !(std::isfinite(b.T_wall) && b.T_wall > 0))
                throw Error(NBTE_ERR_BOUNDARY, "thermalizing wall needs a finite positive T_wall");
            if (b.kind == NBTE_BC_PARTIAL && !(b.specularity >= 0 && b.specularity <= 1))
                throw Error(NBTE_ERR_BOUNDARY, "specularity must lie in [0,1]");
            for (size_t j = 0; j < k; ++j)
                if (v[j].tag == b.tag) throw Error(NBTE_ERR_BOUNDARY, "duplicate tag " + std::to_string(b.tag));
        }
        p->bcs = std::move(v);
        p->have_bcs = true;
        p->plan_ok = p->diff_ok = false;
        p->prepared = false;
        return NBTE_OK;
    });
}

void nbte_solve_opts_default(nbte_solve_opts *o) {
    if (!o) return;
    o->scheme = NBTE_SCHEME_SYNTHETIC;
    o->precision = NBTE_PREC_FP64;
    o->T_ref = 300.0;
    o->tol = 1e-8;
    o->max_iter = 10000;
    o->check_every = 8;
    o->T_init = nullptr;
    o->outputs_on_device = 0;
    o->time_phases = 0;
    o->refine = 1;
    o->spatial_order = 1;
}

nbte_status nbte_prepare(nbte_problem *p, const double *Q_cell, const nbte_solve_opts *o) {
    return guarded([&] {
        if (!p || !o) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        p->prepare(Q_cell, *o);
        p->out_on_device = o->outputs_on_device != 0;
        return NBTE_OK;
    });
}

nbte_status nbte_iterate(nbte_problem *p, int32_t n, int32_t check, double *residual) {
    return guarded([&] {
        if (!p || n < 0) throw Error(NBTE_ERR_INVALID_ARG, "bad arguments");
        p->iterate(n, check != 0, residual);
        return NBTE_OK;
    });
}

nbte_status nbte_read_result(nbte_problem *p, nbte_result *out) {
    return guarded([&] {
        if (!p || !out) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        p->read_result(out);
        return NBTE_OK;
    });
}

nbte_status nbte_solve_steady(nbte_problem *p, const double *Q_cell, const nbte_solve_opts *o, nbte_result *out) {
    return guarded([&] {
        if (!p || !o) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        if (!(o->tol > 0) || o->max_iter <= 0) throw Error(NBTE_ERR_INVALID_ARG, "tol must be > 0 and max_iter >= 1");
        p->prepare(Q_cell, *o);
        p->out_on_device = o->outputs_on_device != 0;
        p->set_controls(1, o->tol, o->max_iter);
        // the device stops the solve at its tolerance or max_iter; the host
        // only polls, so the result does not depend on check_every
        const int every = std::max(1, o->check_every);
        auto t0 = std::chrono::steady_clock::now();
        for (int64_t polls = 0; polls <= (int64_t)o->max_iter / every + 4; ++polls) {
            p->solo->run(every);
            p->solo->collect();
            if (p->hs.done == NBTE_DONE_STALLED) {
                if (!p->refine_possible()) break;   // stays stalled: reported as not converged below
                p->promote();   // FP32 floor reached: continue in FP64
                continue;
            }
            if (p->hs.done) break;
        }
        p->stats.ms_total += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (out) p->read_result(out);
        if (p->hs.done == NBTE_DONE_DIVERGED) return fail(NBTE_ERR_DIVERGED, "iteration diverged (non-finite or exploding temperature update)");
        if (p->hs.done == NBTE_DONE_STALLED)
            return fail(NBTE_ERR_NOT_CONVERGED, "the FP32 iteration stalled at residual " +
                                                    std::to_string(p->hs.residual) +
                                                    "; FP64 refinement would exceed the sweep's 32-bit offsets");
        if (p->hs.done != NBTE_DONE_CONVERGED)
            return fail(NBTE_ERR_NOT_CONVERGED, "not converged after " + std::to_string(p->hs.iterations) +
                                                    " iterations (residual " + std::to_string(p->hs.residual) + ")");
        return NBTE_OK;
    });
}

nbte_status nbte_get_distribution(nbte_problem *p, int32_t band, int32_t dir, double *out) {
    return guarded([&] {
        if (!p || !out) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        if (!p->prepared) throw Error(NBTE_ERR_STATE, "no distribution yet");
        if (band < 0 || band >= p->bands.B || dir < 0 || dir >= p->quad.D)
            throw Error(NBTE_ERR_INVALID_ARG, "band or direction out of range");
        p->sync_state();
        DevBuf tmp;
        tmp.alloc(p->mesh->N * 8);
        launch_distribution(p->d_view.as<DeviceView>(), p->fp32(), band, dir, tmp.as<double>(), p->mesh->N, p->stream);
        NBTE_HIP(hipMemcpyAsync(out, tmp.ptr, p->mesh->N * 8, hipMemcpyDeviceToHost, p->stream));
        NBTE_HIP(hipStreamSynchronize(p->stream));
        return NBTE_OK;
    });
}

nbte_status nbte_get_distribution_noalloc(nbte_problem *p, int32_t band, int32_t dir, double *out) {
    return guarded([&] {
        if (!p || !out) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        if (!p->prepared) throw Error(NBTE_ERR_STATE, "no distribution yet");
        if (band < 0 || band >= p->bands.B || dir < 0 || dir >= p->quad.D)
            throw Error(NBTE_ERR_INVALID_ARG, "band or direction out of range");
        if (p->mesh->N > kDistributionScratchCells)
            throw Error(NBTE_ERR_INVALID_ARG, "mesh of " + std::to_string(p->mesh->N) +
                                                  " cells exceeds the allocation-free read's staging array of " +
                                                  std::to_string(kDistributionScratchCells) + " cells");
        double *stage = nullptr;
        NBTE_HIP(distribution_scratch(&stage));
        p->sync_state();
        // every staged value is written by the kernel before the copy reads it
        launch_distribution(p->d_view.as<DeviceView>(), p->fp32(), band, dir, stage, p->mesh->N, p->stream);
        NBTE_HIP(hipMemcpyAsync(out, stage, p->mesh->N * 8, hipMemcpyDeviceToHost, p->stream));
        NBTE_HIP(hipStreamSynchronize(p->stream));
        return NBTE_OK;
    });
}

nbte_status nbte_get_schedule(nbte_problem *p, int32_t dir, int32_t *perm, int32_t *lvl_ptr, int32_t cap_levels,
                              int32_t *n_levels) {
    return guarded([&] {
        if (!p || !n_levels) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        if (!p->have_quad) throw Error(NBTE_ERR_STATE, "quadrature not set");
        if (dir < 0 || dir >= p->quad.D) throw Error(NBTE_ERR_INVALID_ARG, "direction out of range");
        if (!p->sched_ok) {
            p->sched = build_schedule(*p->mesh, p->quad);
            p->sched_ok = true;
            p->sched_up = false;
        }
        const auto &sc = p->sched;
        const int32_t b = sc.lvl_off[dir], e = sc.lvl_off[dir + 1];
        *n_levels = e - b - 1;
        if (perm) std::copy(&sc.perm[(size_t)dir * p->mesh->N], &sc.perm[(size_t)(dir + 1) * p->mesh->N], perm);
        if (lvl_ptr) {
            if (cap_levels < *n_levels + 1) throw Error(NBTE_ERR_INVALID_ARG, "lvl_ptr capacity too small");
            std::copy(&sc.lvl_ptr[b], &sc.lvl_ptr[e], lvl_ptr);
        }
        return NBTE_OK;
    });
}

nbte_status nbte_get_lagged_faces(nbte_problem *p, int32_t dir, int32_t *cells, int32_t *faces, int32_t cap,
                                  int32_t *n) {
    return guarded([&] {
        if (!p || !n || cap < 0) throw Error(NBTE_ERR_INVALID_ARG, "bad arguments");
        if (!p->have_quad) throw Error(NBTE_ERR_STATE, "quadrature not set");
        if (dir < 0 || dir >= p->quad.D) throw Error(NBTE_ERR_INVALID_ARG, "direction out of range");
        if (!p->sched_ok) {
            p->sched = build_schedule(*p->mesh, p->quad);
            p->sched_ok = true;
            p->sched_up = false;
        }
        const int64_t N = p->mesh->N;
        const int F = p->mesh->F;
        const auto &lg = p->sched.lagged;
        const int64_t lo = (int64_t)dir * N * F, hi = (int64_t)(dir + 1) * N * F;
        auto b = std::lower_bound(lg.begin(), lg.end(), lo), e = std::lower_bound(lg.begin(), lg.end(), hi);
        int32_t k = 0;
        for (auto it = b; it != e; ++it, ++k) {
            if (k >= cap) continue;
            const int64_t key = *it - lo;
            if (cells) cells[k] = (int32_t)(key / F);
            if (faces) faces[k] = (int32_t)(key % F);
        }
        *n = k;
        return NBTE_OK;
    });
}

nbte_status nbte_get_stats(nbte_problem *p, nbte_stats *st) {
    return guarded([&] {
        if (!p || !st) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        p->collect_stats();
        *st = p->stats;
        return NBTE_OK;
    });
}

nbte_status nbte_set_tuning(nbte_problem *p, const nbte_tuning *t) {
    return guarded([&] {
        if (!p || !t) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        if (t->bands_per_block < 0) throw Error(NBTE_ERR_INVALID_ARG, "bands_per_block must be >= 0");
        if (t->lds_bytes < -1 || t->lds_bytes > 163840)
            throw Error(NBTE_ERR_INVALID_ARG, "lds_bytes must be -1, 0 or <= 163840 (capped at the device's per-workgroup LDS)");
        const int bpl = t->bands_per_lane;
        if (bpl != 0 && bpl != 1 && bpl != 2 && bpl != 4 && bpl != 8)
            throw Error(NBTE_ERR_INVALID_ARG, "bands_per_lane must be 0, 1, 2, 4 or 8");
        if (t->block_size != 0 && (t->block_size < 64 || t->block_size > 1024 || t->block_size % 64))
            throw Error(NBTE_ERR_INVALID_ARG, "block_size must be 0 or a multiple of 64 in [64, 1024]");
        if (t->cg_max_iter < 0 || !(t->cg_rtol >= 0)) throw Error(NBTE_ERR_INVALID_ARG, "bad CG settings");
        if (t->accel_depth < 0 || t->accel_depth > kAccelMaxDepth)
            throw Error(NBTE_ERR_INVALID_ARG, "accel_depth must be in [0, 8]");
        if (t->inner_solver < 0 || t->inner_solver > 1 || t->inner_max_iter < 0 || !(t->inner_rtol >= 0))
            throw Error(NBTE_ERR_INVALID_ARG, "bad inner solver settings");
        if (t->layout < 0 || t->layout > 2) throw Error(NBTE_ERR_INVALID_ARG, "layout must be 0, 1 or 2");
        if (p->batch) throw Error(NBTE_ERR_STATE, "the problem is a batch member");
        p->tuning = *t;
        p->prepared = false;   // launch shape and slot table are rebuilt by the next prepare
        return NBTE_OK;
    });
}

nbte_status nbte_get_tuning(const nbte_problem *p, nbte_tuning *t) {
    return guarded([&] {
        if (!p || !t) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        *t = p->tuning;
        return NBTE_OK;
    });
}

nbte_status nbte_problem_setup(nbte_problem *p, int32_t precision) {
    return guarded([&] {
        if (!p) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        if (precision != NBTE_PREC_FP64 && precision != NBTE_PREC_MIXED) throw Error(NBTE_ERR_INVALID_ARG, "bad precision");
        if (p->batch) throw Error(NBTE_ERR_STATE, "the problem is a batch member; remove it from the batch first");
        p->check_addressable(precision);
        require_gfx950();
        p->prepared = false;
        p->precision = precision;   // the launch shape's LDS budget depends on it
        p->ensure_setup();
        p->allocate_state(precision);
        NBTE_HIP(hipStreamSynchronize(p->stream));
        return NBTE_OK;
    });
}

nbte_status nbte_problem_footprint(const nbte_problem *p, int32_t precision, int64_t *bytes) {
    return guarded([&] {
        if (!p || !bytes) throw Error(NBTE_ERR_INVALID_ARG, "null argument");
        if (!p->have_bands || !p->have_quad) throw Error(NBTE_ERR_STATE, "bands and quadrature must be set");
        if (precision != NBTE_PREC_FP64 && precision != NBTE_PREC_MIXED) throw Error(NBTE_ERR_INVALID_ARG, "bad precision");
        p->check_addressable(precision);
        const Mesh &m = *p->mesh;
        const int64_t N = m.N, F = m.F, D = p->quad.D, NBF = m.NBF;
        const int64_t mi = F - 1 <= 2 ? 2 : (F - 1 == 3 ? 3 : 5);   // reference rows (fan-in class)
        const int64_t geo = N * F * 4 + N * 8 + NBF * 4;
        // level tables (at most one level per cell); streams cell, slot, refs, upwind cells, coefficients
        // and outflow sums (storage type); inflow rows
        const int64_t es = precision == NBTE_PREC_MIXED ? 4 : 8;
        const int64_t sched = 3 * D * (N + 1) * 4 + D * N * (4 + 4 + mi * (8 + es) + es) + NBF * D * 4 + D * N * 4;
        // + wall cells, slots; the boundary row of each face's owner
        const int64_t plan = NBF * (4 + 8 + 8 + 8) + NBF * 3 * 4 + 8 + NBF * D * (8 + 4) + NBF * 4;
        const int64_t lh = 2 * N * (F + 1) * 12 + N * 8 * 8 + 256 * 4 * 8;   // CSR and ELL copies, vectors
        *bytes = geo + sched + plan + lh + p->state_bytes(precision);
        return NBTE_OK;
    });
}

}  // extern "C"

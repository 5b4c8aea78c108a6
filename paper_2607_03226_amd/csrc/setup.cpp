// Host-side setup products that depend only on mesh, quadrature, bands and
// boundary conditions, built once per problem and cached (Methods, paragraph
// after Eq. (13): precompute what is iteration-independent).
//
//  * Schedule: for first-order upwind the transport matrix of Eq. (13) is
//    triangular in the upwind order of its direction, so its "factorisation"
//    is that order.  Cells are grouped in topological levels (every upwind
//    neighbour sits in an earlier level) so that a level is swept in parallel.
//  * Boundary plan: per boundary face and direction s.S, the diffuse
//    normalisation and the specular mirror direction.
//  * Diffusion operator of the synthetic correction, Eq. (10), two-point flux.
#include <algorithm>
#include <cmath>
#include <array>
#include <map>
#include <numeric>

#include "internal.h"
#include "kernels.h"

namespace nbte {

Schedule build_schedule(const Mesh &m, const Quadrature &q) {
    const int64_t N = m.N;
    const int F = m.F;
    Schedule sc;
    sc.D = q.D;
    sc.perm.resize((size_t)q.D * N);
    sc.lvl_off.assign(q.D + 1, 0);
    std::vector<int32_t> indeg(N), frontier, next;
    std::vector<uint8_t> placed(N);
    for (int i = 0; i < q.D; ++i) {
        const double *s = &q.s[3 * i];
        auto sdot = [&](int64_t c, int f) {
            const double *S = &m.S[(c * F + f) * 3];
            return s[0] * S[0] + s[1] * S[1] + s[2] * S[2];
        };
        for (int64_t c = 0; c < N; ++c) {
            int d = 0;
            for (int f = 0; f < F; ++f)
                if (m.nbr[c * F + f] >= 0 && sdot(c, f) < 0.0) ++d;
            indeg[c] = d;
        }
        frontier.clear();
        for (int64_t c = 0; c < N; ++c)
            if (indeg[c] == 0) frontier.push_back((int32_t)c);
        int32_t *perm = &sc.perm[(size_t)i * N];
        int64_t done = 0;
        int levels = 0;
        int prev_ghosts = 0;
        std::fill(placed.begin(), placed.end(), 0);
        int64_t scan = 0;   // cells below scan are placed (search start for a stalled order)
        int lag_ghosts = 0; // lagged faces of the released cell: ghosts of its level
        sc.lvl_ptr.push_back(0);
        for (;;) {
            if (frontier.empty()) {
                if (done == N) break;
                // a cycle: release the lowest unfinished cell, lagging its
                // upwind faces towards unfinished cells
                while (placed[scan]) ++scan;
                const int64_t c = scan;
                for (int f = 0; f < F; ++f) {
                    const int32_t u = m.nbr[c * F + f];
                    if (u >= 0 && sdot(c, f) < 0.0 && !placed[u]) {
                        sc.lagged.push_back(((int64_t)i * N + c) * F + f);
                        ++lag_ghosts;
                    }
                }
                indeg[c] = 0;
                frontier.push_back((int32_t)c);
            }
            std::sort(frontier.begin(), frontier.end());
            int ghosts = lag_ghosts;
            lag_ghosts = 0;
            for (int32_t u : frontier)
                for (int f = 0; f < F; ++f)
                    if (m.nbr[(int64_t)u * F + f] < 0 && sdot(u, f) < 0.0) ++ghosts;
            sc.max_ghosts = std::max(sc.max_ghosts, ghosts);
            sc.max_ghost_pair = std::max(sc.max_ghost_pair, prev_ghosts + ghosts);
            prev_ghosts = ghosts;
            std::copy(frontier.begin(), frontier.end(), perm + done);
            for (int32_t u : frontier) placed[u] = 1;
            done += (int64_t)frontier.size();
            sc.lvl_ptr.push_back((int32_t)done);
            ++levels;
            next.clear();
            for (int32_t u : frontier)
                for (int f = 0; f < F; ++f) {
                    int32_t d = m.nbr[(int64_t)u * F + f];
                    // a released cell's indegree is already 0 (goes negative, never queued twice)
                    if (d >= 0 && sdot(u, f) > 0.0 && !placed[d] && --indeg[d] == 0) next.push_back(d);
                }
            frontier.swap(next);
        }
        sc.lvl_off[i + 1] = (int32_t)sc.lvl_ptr.size();
        sc.max_levels = std::max(sc.max_levels, levels);
    }
    std::sort(sc.lagged.begin(), sc.lagged.end());
    return sc;
}

// Interval allocation of LDS slots along the level order: a value produced
// at level l is needed up to the last level of its interior downwind
// neighbours; its slot is free again at the level after that.  Slots freed at
// the start of level l are never read at level l, and a level writes only
// slots no cell of that level reads, so one barrier per level suffices.
void assign_slots(const Mesh &m, const Quadrature &q, Schedule &sc, int cap) {
    const int64_t N = m.N;
    const int F = m.F;
    sc.slot.assign((size_t)q.D * N, -1);
    sc.slot_cap = cap;
    sc.max_slots = 0;
    sc.spilled = 0;
    std::vector<int32_t> level(N), last(N);
    std::vector<std::vector<int32_t>> release;
    std::vector<int32_t> free_slots;
    for (int i = 0; i < q.D; ++i) {
        const double *s = &q.s[3 * i];
        const int32_t *perm = &sc.perm[(size_t)i * N];
        const int32_t *lp = &sc.lvl_ptr[sc.lvl_off[i]];
        const int L = sc.lvl_off[i + 1] - sc.lvl_off[i] - 1;
        for (int l = 0; l < L; ++l)
            for (int k = lp[l]; k < lp[l + 1]; ++k) level[perm[k]] = l;
        for (int64_t c = 0; c < N; ++c) last[c] = -1;
        for (int64_t c = 0; c < N; ++c)
            for (int f = 0; f < F; ++f) {
                const int32_t u = m.nbr[c * F + f];
                if (u < 0) continue;
                const double *S = &m.S[(c * F + f) * 3];
                if (s[0] * S[0] + s[1] * S[1] + s[2] * S[2] < 0.0 && !sc.is_lagged(N, F, i, c, f))
                    last[u] = std::max(last[u], level[c]);
            }
        release.assign(L + 1, {});
        free_slots.clear();
        int used = 0;
        int32_t *slot = &sc.slot[(size_t)i * N];
        for (int l = 0; l < L; ++l) {
            for (int32_t sl : release[l]) free_slots.push_back(sl);
            for (int k = lp[l]; k < lp[l + 1]; ++k) {
                const int32_t c = perm[k];
                if (last[c] < 0) continue;            // nobody downstream reads it
                int32_t sl = -1;
                if (!free_slots.empty()) {
                    sl = free_slots.back();
                    free_slots.pop_back();
                } else if (used < cap) {
                    sl = used++;
                }
                if (sl < 0) {
                    ++sc.spilled;
                    continue;
                }
                slot[c] = sl;
                release[last[c] + 1].push_back(sl);
            }
        }
        sc.max_slots = std::max(sc.max_slots, used);
    }
}

SweepProgram build_program(const Mesh &m, const Quadrature &q, const Schedule &sc, int B, int gcap, int gring, int ls,
                           int es) {
    const SweepLdsLayout lay = sweep_lds_layout(sc.max_levels, gring, ls, es);
    const int64_t N = m.N;
    const int F = m.F;
    const int D = q.D;
    const int64_t DN = (int64_t)D * N;
    SweepProgram pg;
    // widest upwind fan-in over all cells and directions
    for (int i = 0; i < D; ++i) {
        const double *s = &q.s[3 * i];
        for (int64_t c = 0; c < N; ++c) {
            int nin = 0;
            for (int f = 0; f < F; ++f) {
                const double *S = &m.S[(c * F + f) * 3];
                if (s[0] * S[0] + s[1] * S[1] + s[2] * S[2] < 0.0) ++nin;
            }
            pg.maxin = std::max(pg.maxin, nin);
        }
    }
    if (pg.maxin > 5) throw Error(NBTE_ERR_MESH, "a cell has more than 5 upwind faces in some direction");
    // the streams hold as many reference rows as the kernel variant reads
    // (fan-in classes 2, 3 and 5); rows past a cell's fan-in are unused
    pg.maxin = pg.maxin <= 2 ? 2 : (pg.maxin == 3 ? 3 : 5);
    pg.cell.resize(DN);
    pg.slot.resize(DN);
    pg.sout.resize(DN);
    pg.ref.assign((size_t)pg.maxin * DN, lay.zero_off);   // unused: the zero block
    pg.upc.assign((size_t)pg.maxin * DN, 0);
    pg.coef.assign((size_t)pg.maxin * DN, 0.0);
    pg.gptr.resize(sc.lvl_ptr.size());
    pg.in_row.assign((size_t)m.NBF * D, -1);
    const bool staged = !sc.slot.empty();
    std::vector<int32_t> pos(N);                 // position of a cell in direction i's order
    for (int i = 0; i < D; ++i) {
        const double *s = &q.s[3 * i];
        for (int64_t k = 0; k < N; ++k) pos[sc.perm[(int64_t)i * N + k]] = (int32_t)k;
        const int32_t *slot_i = staged ? &sc.slot[(size_t)i * N] : nullptr;
        const int32_t *lp = &sc.lvl_ptr[sc.lvl_off[i]];
        int32_t *gp = &pg.gptr[sc.lvl_off[i]];
        const int L = sc.lvl_off[i + 1] - sc.lvl_off[i] - 1;
        int gpos = 0;   // ring position of the level's first kept ghost
        for (int l = 0; l < L; ++l) {
            gp[l] = (int32_t)pg.ghost_src.size();
            int rank = 0;
            for (int k = lp[l]; k < lp[l + 1]; ++k) {
                const int64_t at = (int64_t)i * N + k;
                const int32_t c = sc.perm[at];
                pg.cell[at] = c;
                for (int j = 0; j < pg.maxin; ++j) pg.upc[(size_t)j * DN + at] = c;
                pg.slot[at] = (slot_i && slot_i[c] >= 0) ? lay.ring_off + slot_i[c] * ls : lay.trash_off;
                const double iv = 1.0 / m.V[c];
                double sout = 0.0;
                int j = 0;
                for (int f = 0; f < F; ++f) {
                    const double *S = &m.S[((int64_t)c * F + f) * 3];
                    const double a = (s[0] * S[0] + s[1] * S[1] + s[2] * S[2]) * iv;
                    if (a > 0.0) {
                        sout += a;
                    } else if (a < 0.0) {
                        const int32_t n = m.nbr[(int64_t)c * F + f];
                        const bool lag = n >= 0 && sc.is_lagged(N, F, i, c, f);
                        int32_t r;
                        if (n < 0 || lag) {   // boundary inflow or a lagged face: a ghost of this level
                            const int64_t row = (int64_t)pg.ghost_src.size();
                            if (n < 0) {
                                const int64_t bf = -(int64_t)n - 1;
                                pg.ghost_src.push_back((bf * D + i) * (int64_t)B);
                                pg.in_row[bf * D + i] = (int32_t)row;
                            } else {
                                pg.ghost_src.push_back(-1);
                                pg.lag.insert(pg.lag.end(), {(int32_t)row, i, c, n});
                            }
                            r = rank < gcap ? lay.gbuf0 + ((gpos + rank) & (gring - 1)) * ls : -1 - (int32_t)row;
                            ++rank;
                        } else if (slot_i && slot_i[n] >= 0) {
                            r = lay.ring_off + slot_i[n] * ls;         // staged in LDS
                        } else {
                            r = -(kSpillBase + 1) - pos[n];            // stored copy in HBM
                        }
                        pg.ref[(size_t)j * DN + at] = r;
                        if (n >= 0 && !lag) pg.upc[(size_t)j * DN + at] = n;   // ghosts are relative to the cell
                        pg.coef[(size_t)j * DN + at] = -a;
                        ++j;
                    }
                }
                pg.sout[at] = sout;
            }
            pg.max_ghosts = std::max(pg.max_ghosts, rank);
            gpos += std::min(rank, gcap);
        }
        gp[L] = (int32_t)pg.ghost_src.size();
    }
    if ((int64_t)pg.ghost_src.size() >= kSpillBase) throw Error(NBTE_ERR_MESH, "too many boundary inflow rows");
    if (N >= INT32_MAX - (int64_t)kSpillBase - 1) throw Error(NBTE_ERR_MESH, "too many cells");
    return pg;
}

BoundaryPlan build_boundary_plan(const Mesh &m, const Quadrature &q,
                                 const std::vector<nbte_boundary> &bcs, double T_ref) {
    std::map<int32_t, nbte_boundary> by_tag;
    for (const auto &b : bcs) by_tag[b.tag] = b;
    BoundaryPlan bp;
    const int64_t NBF = m.NBF;
    const int D = q.D;
    bp.kind.resize(NBF);
    bp.theta_w.assign(NBF, 0.0);
    bp.p.assign(NBF, 0.0);
    bp.sdotS.resize(NBF * D);
    bp.win.assign(NBF, 0.0);
    bp.mirror.assign(NBF * D, -1);
    std::map<std::array<double, 3>, std::vector<int32_t>> mirror_cache;
    for (int64_t j = 0; j < NBF; ++j) {
        auto it = by_tag.find(m.bf_tag[j]);
        if (it == by_tag.end())
            throw Error(NBTE_ERR_BOUNDARY, "no boundary condition for tag " + std::to_string(m.bf_tag[j]));
        const nbte_boundary &b = it->second;
        bp.kind[j] = b.kind;
        if (b.kind == NBTE_BC_THERMALIZING) {
            bp.theta_w[j] = b.T_wall - T_ref;
            bp.has_thermalizing = true;
        }
        bp.p[j] = b.kind == NBTE_BC_SPECULAR ? 1.0 : (b.kind == NBTE_BC_PARTIAL ? b.specularity : 0.0);
        const double *S = &m.S[((int64_t)m.bf_owner[j] * m.F + m.bf_local[j]) * 3];
        for (int i = 0; i < D; ++i) {
            const double *s = &q.s[3 * i];
            double sd = s[0] * S[0] + s[1] * S[1] + s[2] * S[2];
            bp.sdotS[j * D + i] = sd;
            if (sd < 0) bp.win[j] += q.w[i] * -sd;
        }
        if (b.kind == NBTE_BC_SPECULAR || b.kind == NBTE_BC_PARTIAL) {
            double a = std::sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
            std::array<double, 3> n = {S[0] / a, S[1] / a, S[2] / a};
            auto cit = mirror_cache.find(n);
            if (cit == mirror_cache.end()) {
                std::vector<int32_t> mir(D);
                for (int i = 0; i < D; ++i) {
                    const double *s = &q.s[3 * i];
                    double sn = s[0] * n[0] + s[1] * n[1] + s[2] * n[2];
                    double r[3] = {s[0] - 2 * sn * n[0], s[1] - 2 * sn * n[1], s[2] - 2 * sn * n[2]};
                    int best = -1;
                    double bd = 1e300;
                    for (int k = 0; k < D; ++k) {
                        const double *t = &q.s[3 * k];
                        double d = std::sqrt((t[0] - r[0]) * (t[0] - r[0]) + (t[1] - r[1]) * (t[1] - r[1]) +
                                             (t[2] - r[2]) * (t[2] - r[2]));
                        if (d < bd) { bd = d; best = k; }
                    }
                    if (bd > 1e-9)
                        throw Error(NBTE_ERR_QUADRATURE, "quadrature is not closed under specular reflection "
                                                         "about the normal of boundary tag " +
                                                             std::to_string(m.bf_tag[j]));
                    mir[i] = best;
                }
                cit = mirror_cache.emplace(n, std::move(mir)).first;
            }
            std::copy(cit->second.begin(), cit->second.end(), &bp.mirror[j * D]);
        }
    }
    return bp;
}

// Face conductivity of the synthetic correction.  kappa_bulk as printed in
// Eq. (10) lets the correction stall when ballistic bands dominate kappa_bulk
// and overshoot when cells are optically thick; the operator used here is the
// conductivity the discrete upwind transport itself shows for smooth fields:
//   sum_l C v Lambda_eff sum_i w (s.n)^2 / W  +  sum_l C v dist sum_i w |s.n| / (2W),
// Lambda_eff = Lambda / (1 + 2 Lambda / L_c).  Any SPD operator leaves the
// fixed point unchanged; this one only shortens the iteration.
DiffusionOperator build_diffusion(const Mesh &m, const BandTable &b, const Quadrature &q,
                                  const BoundaryPlan &bp) {
    const int64_t N = m.N;
    const int F = m.F;
    // smallest extent of the domain
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t c = 0; c < N; ++c)
        for (int f = 0; f < F; ++f)
            for (int ax = 0; ax < m.dim; ++ax) {
                double x = m.xf[(c * F + f) * 3 + ax];
                lo[ax] = std::min(lo[ax], x);
                hi[ax] = std::max(hi[ax], x);
            }
    double Lc = 1e300;
    for (int ax = 0; ax < m.dim; ++ax) Lc = std::min(Lc, hi[ax] - lo[ax]);
    double cvl = 0, cv = 0;
    for (int l = 0; l < b.B; ++l) {
        double lam = b.v[l] * b.tau[l];
        cvl += b.C[l] * b.v[l] * lam / (1.0 + 2.0 * lam / Lc);
        cv += b.C[l] * b.v[l];
    }
    auto kappa_f = [&](const double *nh, double dist) {
        double m2 = 0, m1 = 0;
        for (int i = 0; i < q.D; ++i) {
            const double *s = &q.s[3 * i];
            double mu = s[0] * nh[0] + s[1] * nh[1] + s[2] * nh[2];
            m2 += q.w[i] * mu * mu;
            m1 += q.w[i] * std::fabs(mu);
        }
        return cvl * m2 / q.W + cv * dist * m1 / (2.0 * q.W);
    };
    DiffusionOperator op;
    op.row_ptr.assign(N + 1, 0);
    op.dir_rhs.assign(N, 0.0);
    op.col.reserve(N * (F + 1));
    op.val.reserve(N * (F + 1));
    for (int64_t c = 0; c < N; ++c) {
        double diag = 0;
        const size_t diag_pos = op.col.size();
        op.col.push_back((int32_t)c);
        op.val.push_back(0.0);
        for (int f = 0; f < F; ++f) {
            const double *S = &m.S[(c * F + f) * 3];
            double A = std::sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
            double nh[3] = {S[0] / A, S[1] / A, S[2] / A};
            int32_t nb = m.nbr[c * F + f];
            if (nb >= 0) {
                double d = 0;
                for (int ax = 0; ax < 3; ++ax) d += (m.xc[nb * 3 + ax] - m.xc[c * 3 + ax]) * nh[ax];
                d = std::fabs(d);
                double T = kappa_f(nh, d) * A / d;
                diag += T;
                op.col.push_back(nb);
                op.val.push_back(-T);
            } else {
                int32_t j = -(nb + 1);
                if (bp.kind[j] != NBTE_BC_THERMALIZING) continue;
                double d = 0;
                for (int ax = 0; ax < 3; ++ax) d += (m.xf[(c * F + f) * 3 + ax] - m.xc[c * 3 + ax]) * nh[ax];
                d = std::fabs(d);
                double T = kappa_f(nh, 2.0 * d) * A / d;
                diag += T;
                op.dir_rhs[c] += T * bp.theta_w[j];
            }
        }
        op.val[diag_pos] = diag;
        op.row_ptr[c + 1] = (int32_t)op.col.size();
    }
    return op;
}

namespace {

// eigenvalues of a symmetric d x d matrix (d <= 3) by cyclic Jacobi rotations
void sym_eigenvalues(int d, double A[3][3], double ev[3]) {
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < d; ++p)
            for (int q = p + 1; q < d; ++q) off += A[p][q] * A[p][q];
        if (off < 1e-300) break;
        for (int p = 0; p < d; ++p)
            for (int q = p + 1; q < d; ++q) {
                if (A[p][q] == 0.0) continue;
                const double th = 0.5 * (A[q][q] - A[p][p]) / A[p][q];
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < d; ++k) {   // A <- J^T A J
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < d; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
            }
    }
    for (int k = 0; k < d; ++k) ev[k] = A[k][k];
}

}  // namespace

std::vector<double> build_lsq_weights(const Mesh &m) {
    const int64_t N = m.N;
    const int F = m.F, d = m.dim;
    std::vector<double> w((size_t)N * F * 3, 0.0);
    for (int64_t c = 0; c < N; ++c) {
        double M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int f = 0; f < F; ++f) {
            const int32_t n = m.nbr[c * F + f];
            if (n < 0) continue;
            double off[3];
            for (int k = 0; k < 3; ++k) off[k] = m.xc[n * 3 + k] - m.xc[c * 3 + k];
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) M[a][b] += off[a] * off[b];
        }
        double E[3][3], ev[3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) E[a][b] = M[a][b];
        sym_eigenvalues(d, E, ev);
        double lo = ev[0], hi = ev[0];
        for (int k = 1; k < d; ++k) lo = std::min(lo, ev[k]), hi = std::max(hi, ev[k]);
        if (!(hi > 0.0) || !(lo > 1e-8 * hi)) continue;   // no gradient: first-order faces
        // inverse of the d x d block
        double inv[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        if (d == 2) {
            const double det = M[0][0] * M[1][1] - M[0][1] * M[1][0];
            inv[0][0] = M[1][1] / det, inv[0][1] = -M[0][1] / det;
            inv[1][0] = -M[1][0] / det, inv[1][1] = M[0][0] / det;
        } else {
            const double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                               M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                               M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    // cofactor (b, a) / det
                    const int r0 = (b + 1) % 3, r1 = (b + 2) % 3, c0 = (a + 1) % 3, c1 = (a + 2) % 3;
                    inv[a][b] = (M[r0][c0] * M[r1][c1] - M[r0][c1] * M[r1][c0]) / det;
                }
        }
        for (int f = 0; f < F; ++f) {
            const int32_t n = m.nbr[c * F + f];
            if (n < 0) continue;
            double off[3];
            for (int k = 0; k < 3; ++k) off[k] = m.xc[n * 3 + k] - m.xc[c * 3 + k];
            for (int a = 0; a < d; ++a) {
                double x = 0.0;
                for (int b = 0; b < d; ++b) x += inv[a][b] * off[b];
                w[((size_t)c * F + f) * 3 + a] = x;
            }
        }
    }
    return w;
}

}  // namespace nbte

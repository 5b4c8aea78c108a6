// Host-side setup of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer: the mesh-to-CSR builder, the per-direction
// level schedules, the LDS slot assignment, the sweep program, the boundary
// plan, the diffusion operator and the least-squares gradient weights, on
// small meshes of every cell type (with jittered nodes, several slot budgets
// and ghost-ring sizes), plus a mesh whose upwind graph is cyclic (scheduled
// with lagged faces).  No device code runs.
// Exit status 0 and no sanitizer report mean every access stayed in bounds.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <random>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace nbte;

namespace {

struct RawMesh {
    int dim = 0, type = 0;
    std::vector<double> xyz;
    std::vector<int64_t> cells, bfaces;
    std::vector<int32_t> tags;
};

const int kQuadF[4][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}};
const int kTriF[3][2] = {{0, 1}, {1, 2}, {2, 0}};
const int kTetF[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
const int kHexF[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};

// boundary faces = faces of exactly one cell; tag 1 where every node has
// x == 0 (thermalizing), 2..4 elsewhere by the face's first node
void add_boundary(RawMesh &m, int nv, int F, int k, const int *lf) {
    std::map<std::vector<int64_t>, std::pair<int, std::vector<int64_t>>> seen;
    const int64_t N = (int64_t)m.cells.size() / nv;
    for (int64_t c = 0; c < N; ++c)
        for (int f = 0; f < F; ++f) {
            std::vector<int64_t> nodes(k);
            for (int j = 0; j < k; ++j) nodes[j] = m.cells[c * nv + lf[f * k + j]];
            std::vector<int64_t> key = nodes;
            std::sort(key.begin(), key.end());
            auto &e = seen[key];
            e.first += 1;
            e.second = nodes;
        }
    for (auto &kv : seen) {
        if (kv.second.first != 1) continue;
        bool x0 = true;
        for (int64_t nd : kv.second.second) x0 = x0 && m.xyz[nd * m.dim] == 0.0;
        for (int64_t nd : kv.second.second) m.bfaces.push_back(nd);
        m.tags.push_back(x0 ? 1 : 2 + (int32_t)(kv.second.second[0] % 3));
    }
}

RawMesh grid2d(int nx, int ny, bool tri, std::mt19937 &rng) {
    RawMesh m;
    m.dim = 2;
    m.type = tri ? NBTE_CELL_TRI3 : NBTE_CELL_QUAD4;
    std::uniform_real_distribution<double> jit(-0.2, 0.2);
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            const bool in = i > 0 && i < nx && j > 0 && j < ny;
            m.xyz.push_back((i + (in ? jit(rng) : 0.0)) * 1e-8);
            m.xyz.push_back((j + (in ? jit(rng) : 0.0)) * 1e-8);
        }
    auto id = [&](int i, int j) { return (int64_t)j * (nx + 1) + i; };
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const int64_t a = id(i, j), b = id(i + 1, j), c = id(i + 1, j + 1), d = id(i, j + 1);
            if (tri) m.cells.insert(m.cells.end(), {a, b, c, a, c, d});
            else m.cells.insert(m.cells.end(), {a, b, c, d});
        }
    if (tri) add_boundary(m, 3, 3, 2, &kTriF[0][0]);
    else add_boundary(m, 4, 4, 2, &kQuadF[0][0]);
    return m;
}

RawMesh grid3d(int n, bool tet, std::mt19937 &rng) {
    RawMesh m;
    m.dim = 3;
    m.type = tet ? NBTE_CELL_TET4 : NBTE_CELL_HEX8;
    std::uniform_real_distribution<double> jit(-0.15, 0.15);
    for (int k = 0; k <= n; ++k)
        for (int j = 0; j <= n; ++j)
            for (int i = 0; i <= n; ++i) {
                const bool in = i > 0 && i < n && j > 0 && j < n && k > 0 && k < n;
                // hexahedra keep planar faces: jitter only tetrahedral meshes
                const double d = in && tet ? 1.0 : 0.0;
                m.xyz.push_back((i + d * jit(rng)) * 1e-8);
                m.xyz.push_back((j + d * jit(rng)) * 1e-8);
                m.xyz.push_back((k + d * jit(rng)) * 1e-8);
            }
    auto id = [&](int i, int j, int k) { return ((int64_t)k * (n + 1) + j) * (n + 1) + i; };
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const int64_t v[8] = {id(i, j, k),     id(i + 1, j, k),     id(i + 1, j + 1, k),     id(i, j + 1, k),
                                      id(i, j, k + 1), id(i + 1, j, k + 1), id(i + 1, j + 1, k + 1), id(i, j + 1, k + 1)};
                if (!tet) {
                    m.cells.insert(m.cells.end(), v, v + 8);
                    continue;
                }
                // six tetrahedra around the diagonal v0-v6
                const int t[6][4] = {{0, 1, 2, 6}, {0, 2, 3, 6}, {0, 3, 7, 6}, {0, 7, 4, 6}, {0, 4, 5, 6}, {0, 5, 1, 6}};
                for (auto &tt : t)
                    for (int q = 0; q < 4; ++q) m.cells.push_back(v[tt[q]]);
            }
    if (tet) add_boundary(m, 4, 4, 3, &kTetF[0][0]);
    else add_boundary(m, 8, 6, 4, &kHexF[0][0]);
    return m;
}

Quadrature quadrature(int dim, int D) {
    Quadrature q;
    const double pi = 3.14159265358979323846;
    if (dim == 2) {
        for (int j = 0; j < D; ++j) {
            const double phi = (j + 0.5) * 2 * pi / D;
            q.s.insert(q.s.end(), {std::cos(phi), std::sin(phi), 0.0});
            q.w.push_back(2 * pi / D);
        }
    } else {
        const int np = 4, na = D / np;
        for (int a = 0; a < np; ++a) {
            const double mu = -1.0 + (a + 0.5) * 2.0 / np, st = std::sqrt(1 - mu * mu);
            for (int b = 0; b < na; ++b) {
                const double phi = (b + 0.5) * 2 * pi / na;
                q.s.insert(q.s.end(), {st * std::cos(phi), st * std::sin(phi), mu});
                q.w.push_back(4 * pi / (np * na));
            }
        }
    }
    q.D = (int)q.w.size();
    for (double w : q.w) q.W += w;
    return q;
}

int64_t g_lagged = 0;   // lagged faces of the last exercised mesh

int exercise(const RawMesh &rm, int D, int B) {
    const int nv = (int)(rm.type == NBTE_CELL_TRI3 ? 3 : rm.type == NBTE_CELL_HEX8 ? 8 : 4);
    const int nfv = rm.type == NBTE_CELL_TET4 ? 3 : (rm.type == NBTE_CELL_HEX8 ? 4 : 2);
    auto m = build_mesh(rm.dim, (int64_t)rm.xyz.size() / rm.dim, rm.xyz.data(), rm.type,
                        (int64_t)rm.cells.size() / nv, rm.cells.data(), (int64_t)rm.bfaces.size() / nfv,
                        rm.bfaces.data(), rm.tags.data());
    const Quadrature q = quadrature(rm.dim, D);
    BandTable bt;
    bt.B = B;
    for (int l = 0; l < B; ++l) {
        bt.C.push_back(1e5 * (l + 1));
        bt.v.push_back(1000.0 * (l + 2));
        bt.tau.push_back(1e-12 * (l + 1));
        bt.beta += bt.C.back() / bt.tau.back();
        bt.C_tot += bt.C.back();
    }
    std::vector<nbte_boundary> bcs = {{1, NBTE_BC_THERMALIZING, 301.0, 0.0},
                                      {2, NBTE_BC_DIFFUSE, 0.0, 0.0},
                                      {3, NBTE_BC_SPECULAR, 0.0, 0.0},
                                      {4, NBTE_BC_PARTIAL, 0.0, 0.4}};
    Schedule sc = build_schedule(*m, q);
    g_lagged = (int64_t)sc.lagged.size();
    int checks = 0;
    for (int cap : {1, 7, 64, 1 << 20}) {
        assign_slots(*m, q, sc, cap);
        for (int es : {4, 8})
            for (int ls : {1, 4}) {
                int ring = 1;
                while (ring < sc.max_ghost_pair) ring <<= 1;
                for (int gcap : {sc.max_ghosts, 2}) {
                    const int gring = gcap == 2 ? 4 : ring;
                    SweepProgram pg = build_program(*m, q, sc, B, gcap, gring, ls, es);
                    checks += pg.cell.size() == (size_t)q.D * m->N;
                }
            }
    }
    sc.slot.clear();
    SweepProgram pg = build_program(*m, q, sc, B, sc.max_ghosts, 1 << 12, 2, 8);
    BoundaryPlan bp = build_boundary_plan(*m, q, bcs, 300.0);
    DiffusionOperator op = build_diffusion(*m, bt, q, bp);
    checks += (int64_t)op.row_ptr.size() == m->N + 1 && !pg.cell.empty();
    const std::vector<double> lsq = build_lsq_weights(*m);
    checks += (int64_t)lsq.size() == m->N * m->F * 3;
    return checks;
}

}  // namespace

int main() {
    std::mt19937 rng(12345);
    int checks = 0;
    checks += exercise(grid2d(9, 7, false, rng), 12, 3);
    checks += exercise(grid2d(8, 6, true, rng), 16, 5);
    checks += exercise(grid3d(4, false, rng), 16, 2);
    checks += exercise(grid3d(3, true, rng), 24, 3);
    // a dart cell closes an upwind cycle for directions at 110..190 degrees
    RawMesh dart;
    dart.dim = 2;
    dart.type = NBTE_CELL_QUAD4;
    const double pi = 3.14159265358979323846, R = 5e-8;
    dart.xyz = {0.0, 0.0};
    for (double a : {10.0, 60.0, 110.0}) dart.xyz.insert(dart.xyz.end(), {R * std::cos(a * pi / 180), R * std::sin(a * pi / 180)});
    for (double a : {35.0, 85.0})
        dart.xyz.insert(dart.xyz.end(), {1.5 * R * std::cos(a * pi / 180), 1.5 * R * std::sin(a * pi / 180)});
    dart.xyz.insert(dart.xyz.end(), {0.0, -2 * R});
    dart.cells = {0, 1, 4, 2, 0, 2, 5, 3, 0, 3, 6, 1};
    dart.bfaces = {1, 4, 4, 2, 2, 5, 5, 3, 3, 6, 6, 1};
    dart.tags = {2, 2, 2, 2, 1, 2};
    const bool lagged = exercise(dart, 8, 2) == 34 && g_lagged > 0;
    // malformed input is rejected, not read out of bounds
    RawMesh bad = grid2d(3, 3, false, rng);
    bad.cells[5] = 1000;
    bool bad_rejected = false;
    try {
        exercise(bad, 4, 1);
    } catch (const Error &e) {
        bad_rejected = e.code == NBTE_ERR_MESH;
    }
    std::printf("checks %d cyclic_lagged %d bad_index_rejected %d\n", checks, (int)lagged, (int)bad_rejected);
    return (checks == 4 * 34 && lagged && bad_rejected) ? 0 : 1;
}

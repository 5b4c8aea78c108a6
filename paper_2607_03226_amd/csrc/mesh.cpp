// Mesh-to-CSR builder: the one cell-face pattern shared by every band x
// direction system (Methods, paragraph after Eq. (13): cell-face connectivity
// and geometry are built once from the mesh).
//
// Faces are matched by sorting the sorted node tuples of all cell faces; runs
// of two equal keys are interior faces, runs of one are boundary faces (which
// must appear in the tagged list), longer runs are non-manifold.  Each unique
// face gets one area vector, computed once and oriented outward from the cell
// of its first occurrence; the neighbour sees it negated, so the upwind test
// sign(s . S) agrees bit-for-bit on both sides of every face.
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace nbte {
namespace {

struct CellKind {
    int dim, nv, F, nfv;
    int faces[6][4];
};

// Local faces in cyclic node order.
const CellKind kTri = {2, 3, 3, 2, {{0, 1}, {1, 2}, {2, 0}}};
const CellKind kQuad = {2, 4, 4, 2, {{0, 1}, {1, 2}, {2, 3}, {3, 0}}};
const CellKind kTet = {3, 4, 4, 3, {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}}};
const CellKind kHex = {3, 8, 6, 4, {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}}};

const CellKind &kind_of(int t) {
    switch (t) {
        case NBTE_CELL_TRI3: return kTri;
        case NBTE_CELL_QUAD4: return kQuad;
        case NBTE_CELL_TET4: return kTet;
        case NBTE_CELL_HEX8: return kHex;
    }
    throw Error(NBTE_ERR_INVALID_ARG, "unknown cell type");
}

using Key = std::array<int64_t, 4>;

Key make_key(const int64_t *nodes, int k) {
    Key key{-1, -1, -1, -1};
    for (int j = 0; j < k; ++j) key[j] = nodes[j];
    std::sort(key.begin(), key.begin() + k);
    return key;
}

struct FaceRef {
    Key key;
    int64_t occ;  // cell*F + local
};

}  // namespace

std::shared_ptr<Mesh> build_mesh(int32_t dim, int64_t n_nodes, const double *xyz, int32_t cell_type,
                                 int64_t n_cells, const int64_t *cell_nodes, int64_t n_bfaces,
                                 const int64_t *bface_nodes, const int32_t *bface_tag) {
    if (dim != 2 && dim != 3) throw Error(NBTE_ERR_INVALID_ARG, "dim must be 2 or 3");
    const CellKind &ck = kind_of(cell_type);
    if (ck.dim != dim) throw Error(NBTE_ERR_INVALID_ARG, "cell type does not match dim");
    if (n_nodes <= 0 || n_cells <= 0 || n_bfaces < 0) throw Error(NBTE_ERR_INVALID_ARG, "bad sizes");
    if (!xyz || !cell_nodes || (n_bfaces > 0 && (!bface_nodes || !bface_tag)))
        throw Error(NBTE_ERR_INVALID_ARG, "null mesh array");
    if (n_cells > INT32_MAX / 8 || n_bfaces > INT32_MAX) throw Error(NBTE_ERR_INVALID_ARG, "mesh too large");
    for (int64_t k = 0; k < n_nodes * dim; ++k)
        if (!std::isfinite(xyz[k])) throw Error(NBTE_ERR_INVALID_ARG, "non-finite node coordinate");
    for (int64_t k = 0; k < n_cells * ck.nv; ++k)
        if (cell_nodes[k] < 0 || cell_nodes[k] >= n_nodes) throw Error(NBTE_ERR_MESH, "cell node index out of range");
    for (int64_t k = 0; k < n_bfaces * ck.nfv; ++k)
        if (bface_nodes[k] < 0 || bface_nodes[k] >= n_nodes) throw Error(NBTE_ERR_MESH, "boundary node index out of range");

    auto m = std::make_shared<Mesh>();
    m->dim = dim;
    m->cell_type = cell_type;
    m->F = ck.F;
    m->N = n_cells;
    m->NBF = n_bfaces;
    const int F = ck.F, k = ck.nfv;
    const int64_t N = n_cells;

    auto X = [&](int64_t node, int ax) -> double { return ax < dim ? xyz[node * dim + ax] : 0.0; };

    // cell centroids (vertex average)
    m->xc.assign(N * 3, 0.0);
    for (int64_t c = 0; c < N; ++c)
        for (int j = 0; j < ck.nv; ++j)
            for (int ax = 0; ax < 3; ++ax) m->xc[c * 3 + ax] += X(cell_nodes[c * ck.nv + j], ax) / ck.nv;

    // all cell faces, sorted by key
    std::vector<FaceRef> faces(N * F);
    std::vector<int64_t> fn(N * F * 4, -1);  // node ids in cyclic order
    for (int64_t c = 0; c < N; ++c)
        for (int f = 0; f < F; ++f) {
            int64_t *dst = &fn[(c * F + f) * 4];
            for (int j = 0; j < k; ++j) dst[j] = cell_nodes[c * ck.nv + ck.faces[f][j]];
            faces[c * F + f] = {make_key(dst, k), c * F + f};
        }
    std::sort(faces.begin(), faces.end(), [](const FaceRef &a, const FaceRef &b) {
        return a.key != b.key ? a.key < b.key : a.occ < b.occ;
    });

    // boundary-face lookup
    std::vector<std::pair<Key, int64_t>> bkeys(n_bfaces);
    for (int64_t j = 0; j < n_bfaces; ++j) bkeys[j] = {make_key(bface_nodes + j * k, k), j};
    std::sort(bkeys.begin(), bkeys.end());
    for (int64_t j = 1; j < n_bfaces; ++j)
        if (bkeys[j].first == bkeys[j - 1].first) throw Error(NBTE_ERR_MESH, "duplicate boundary face");

    m->nbr.assign(N * F, INT32_MIN);
    m->S.assign(N * F * 3, 0.0);
    m->xf.assign(N * F * 3, 0.0);
    m->bf_owner.assign(n_bfaces, -1);
    m->bf_local.assign(n_bfaces, -1);
    m->bf_tag.assign(bface_tag, bface_tag + n_bfaces);

    auto face_geometry = [&](int64_t occ, double Sv[3], double xfv[3]) {
        const int64_t *nd = &fn[occ * 4];
        double P[4][3];
        for (int j = 0; j < k; ++j)
            for (int ax = 0; ax < 3; ++ax) P[j][ax] = X(nd[j], ax);
        for (int ax = 0; ax < 3; ++ax) {
            xfv[ax] = 0;
            for (int j = 0; j < k; ++j) xfv[ax] += P[j][ax] / k;
        }
        if (k == 2) {  // edge: length times in-plane normal
            Sv[0] = P[1][1] - P[0][1];
            Sv[1] = -(P[1][0] - P[0][0]);
            Sv[2] = 0.0;
        } else {
            // triangle: (P1-P0)x(P2-P0)/2 ; quad: (P2-P0)x(P3-P1)/2 (diagonals)
            double a[3], b[3];
            for (int ax = 0; ax < 3; ++ax) {
                a[ax] = (k == 3) ? P[1][ax] - P[0][ax] : P[2][ax] - P[0][ax];
                b[ax] = (k == 3) ? P[2][ax] - P[0][ax] : P[3][ax] - P[1][ax];
            }
            Sv[0] = 0.5 * (a[1] * b[2] - a[2] * b[1]);
            Sv[1] = 0.5 * (a[2] * b[0] - a[0] * b[2]);
            Sv[2] = 0.5 * (a[0] * b[1] - a[1] * b[0]);
        }
    };

    size_t i = 0;
    const size_t nf = faces.size();
    while (i < nf) {
        size_t j = i + 1;
        while (j < nf && faces[j].key == faces[i].key) ++j;
        const size_t run = j - i;
        if (run > 2) throw Error(NBTE_ERR_MESH, "non-manifold face shared by more than two cells");
        const int64_t o1 = faces[i].occ;
        const int64_t c1 = o1 / F;
        double Sv[3], xfv[3];
        face_geometry(o1, Sv, xfv);
        double area = std::sqrt(Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2]);
        if (!(area > 0)) throw Error(NBTE_ERR_MESH, "degenerate face");
        double orient = 0;
        for (int ax = 0; ax < 3; ++ax) orient += (xfv[ax] - m->xc[c1 * 3 + ax]) * Sv[ax];
        if (orient == 0) throw Error(NBTE_ERR_MESH, "degenerate face orientation");
        if (orient < 0)
            for (double &x : Sv) x = -x;
        for (int ax = 0; ax < 3; ++ax) {
            m->S[o1 * 3 + ax] = Sv[ax];
            m->xf[o1 * 3 + ax] = xfv[ax];
        }
        if (run == 2) {
            const int64_t o2 = faces[i + 1].occ;
            const int64_t c2 = o2 / F;
            if (c1 == c2) throw Error(NBTE_ERR_MESH, "cell with a repeated face");
            for (int ax = 0; ax < 3; ++ax) {
                m->S[o2 * 3 + ax] = -Sv[ax];
                m->xf[o2 * 3 + ax] = xfv[ax];
            }
            m->nbr[o1] = (int32_t)c2;
            m->nbr[o2] = (int32_t)c1;
        } else {
            auto it = std::lower_bound(bkeys.begin(), bkeys.end(), std::make_pair(faces[i].key, (int64_t)-1));
            if (it == bkeys.end() || it->first != faces[i].key)
                throw Error(NBTE_ERR_MESH, "boundary face without a tag");
            const int64_t bj = it->second;
            m->nbr[o1] = -(int32_t)(bj + 1);
            m->bf_owner[bj] = (int32_t)c1;
            m->bf_local[bj] = (int32_t)(o1 % F);
        }
        i = j;
    }
    for (int64_t bj = 0; bj < n_bfaces; ++bj)
        if (m->bf_owner[bj] < 0) throw Error(NBTE_ERR_MESH, "tagged boundary face is not on the mesh boundary");

    // volumes (divergence theorem) and closure check
    m->V.assign(N, 0.0);
    m->total_volume = 0;
    m->max_closure = 0;
    for (int64_t c = 0; c < N; ++c) {
        double v = 0, sx = 0, sy = 0, sz = 0, sa = 0;
        for (int f = 0; f < F; ++f) {
            const double *Sv = &m->S[(c * F + f) * 3];
            const double *xfv = &m->xf[(c * F + f) * 3];
            v += xfv[0] * Sv[0] + xfv[1] * Sv[1] + xfv[2] * Sv[2];
            sx += Sv[0]; sy += Sv[1]; sz += Sv[2];
            sa += std::sqrt(Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2]);
        }
        v /= dim;
        if (!(v > 0)) throw Error(NBTE_ERR_MESH, "non-positive cell volume (cell " + std::to_string(c) + ")");
        m->V[c] = v;
        m->total_volume += v;
        double cl = std::sqrt(sx * sx + sy * sy + sz * sz) / sa;
        m->max_closure = std::max(m->max_closure, cl);
    }
    if (m->max_closure > 1e-9) throw Error(NBTE_ERR_MESH, "cell faces do not close (non-planar or inverted cell)");
    return m;
}

}  // namespace nbte

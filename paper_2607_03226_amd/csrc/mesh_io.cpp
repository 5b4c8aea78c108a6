// Gmsh mesh files (the paper's meshes come from Gmsh and COMSOL): MSH 4.1
// and MSH 2.2 in ASCII.  The elements of the highest dimension are the cells
// (one type per mesh: tri3 or quad4 in 2D, tet4 or hex8 in 3D); the elements
// one dimension lower that lie on the mesh boundary are the tagged boundary
// faces (their physical group is the tag, 0 without one; lower-dimensional
// elements inside the domain, such as material interfaces, are skipped); each
// cell keeps the physical group of its element as its region.  The result
// goes through the same builder as nbte_mesh_create.
#include <algorithm>
#include <cmath>
#include <array>
#include <fstream>
#include <map>
#include <set>
#include <sstream>
#include <string>

#include "internal.h"

namespace nbte {
namespace {

// Gmsh element types used here: nodes per element and dimension
struct GType {
    int nodes, dim, cell_type;
};
bool gmsh_type(int t, GType &g) {
    switch (t) {
        case 1: g = {2, 1, 0}; return true;                     // 2-node line
        case 2: g = {3, 2, NBTE_CELL_TRI3}; return true;       // 3-node triangle
        case 3: g = {4, 2, NBTE_CELL_QUAD4}; return true;      // 4-node quadrangle
        case 4: g = {4, 3, NBTE_CELL_TET4}; return true;       // 4-node tetrahedron
        case 5: g = {8, 3, NBTE_CELL_HEX8}; return true;       // 8-node hexahedron
        case 15: g = {1, 0, 0}; return true;                    // 1-node point
    }
    return false;
}

struct RawElem {
    int type, phys;
    std::vector<int64_t> nodes;   // file node tags
};

[[noreturn]] void bad(const std::string &what) { throw Error(NBTE_ERR_INVALID_ARG, "gmsh file: " + what); }

template <class T>
T take(std::istream &in, const char *what) {
    T x;
    if (!(in >> x)) bad(std::string("cannot read ") + what);
    return x;
}

void expect_end(std::istream &in, const std::string &section) {
    std::string tok;
    if (!(in >> tok) || tok != "$End" + section) bad("missing $End" + section);
}

struct FileMesh {
    std::map<int64_t, std::array<double, 3>> nodes;   // tag -> coordinates
    std::vector<RawElem> elems;
};

// MSH 4.1: entity physical tags from $Entities, nodes and elements in blocks
void read_v4(std::istream &in, FileMesh &fm) {
    std::map<std::pair<int, int>, int> phys;   // (entity dim, entity tag) -> first physical tag
    std::string tok;
    while (in >> tok) {
        if (tok == "$Entities") {
            const int64_t np = take<int64_t>(in, "entity counts"), nc = take<int64_t>(in, "entity counts"),
                          ns = take<int64_t>(in, "entity counts"), nv = take<int64_t>(in, "entity counts");
            const int64_t counts[4] = {np, nc, ns, nv};
            for (int d = 0; d < 4; ++d)
                for (int64_t e = 0; e < counts[d]; ++e) {
                    const int tag = take<int>(in, "entity tag");
                    const int nbox = d == 0 ? 3 : 6;
                    for (int k = 0; k < nbox; ++k) take<double>(in, "entity box");
                    const int64_t nph = take<int64_t>(in, "physical tag count");
                    if (nph < 0 || nph > 1000000) bad("bad physical tag count");
                    int first = 0;
                    for (int64_t k = 0; k < nph; ++k) {
                        const int t = take<int>(in, "physical tag");
                        if (k == 0) first = t;
                    }
                    phys[{d, tag}] = first;
                    if (d > 0) {
                        const int64_t nb = take<int64_t>(in, "bounding entity count");
                        if (nb < 0 || nb > 1000000) bad("bad bounding entity count");
                        for (int64_t k = 0; k < nb; ++k) take<int>(in, "bounding entity");
                    }
                }
            expect_end(in, "Entities");
        } else if (tok == "$Nodes") {
            const int64_t nblocks = take<int64_t>(in, "node block count");
            take<int64_t>(in, "node count");
            take<int64_t>(in, "min node tag");
            take<int64_t>(in, "max node tag");
            for (int64_t b = 0; b < nblocks; ++b) {
                take<int>(in, "block dim");
                take<int>(in, "block tag");
                const int param = take<int>(in, "parametric flag");
                const int64_t n = take<int64_t>(in, "block node count");
                if (param != 0) bad("parametric node blocks are not supported");
                if (n < 0) bad("negative node count");
                std::vector<int64_t> tags(n);
                for (auto &t : tags) t = take<int64_t>(in, "node tag");
                for (int64_t k = 0; k < n; ++k) {
                    std::array<double, 3> x;
                    for (double &c : x) c = take<double>(in, "node coordinate");
                    fm.nodes[tags[k]] = x;
                }
            }
            expect_end(in, "Nodes");
        } else if (tok == "$Elements") {
            const int64_t nblocks = take<int64_t>(in, "element block count");
            take<int64_t>(in, "element count");
            take<int64_t>(in, "min element tag");
            take<int64_t>(in, "max element tag");
            for (int64_t b = 0; b < nblocks; ++b) {
                const int edim = take<int>(in, "block dim");
                const int etag = take<int>(in, "block tag");
                const int type = take<int>(in, "element type");
                const int64_t n = take<int64_t>(in, "block element count");
                GType g;
                if (!gmsh_type(type, g)) bad("element type " + std::to_string(type) + " is not supported");
                if (n < 0) bad("negative element count");
                const auto it = phys.find({edim, etag});
                const int ph = it == phys.end() ? 0 : it->second;
                for (int64_t k = 0; k < n; ++k) {
                    RawElem e{type, ph, std::vector<int64_t>(g.nodes)};
                    take<int64_t>(in, "element tag");
                    for (auto &v : e.nodes) v = take<int64_t>(in, "element node");
                    fm.elems.push_back(std::move(e));
                }
            }
            expect_end(in, "Elements");
        } else if (!tok.empty() && tok[0] == '$' && tok.rfind("$End", 0) != 0) {
            // a section this reader does not use: skip to its end marker
            const std::string end = "$End" + tok.substr(1);
            std::string t2;
            while (in >> t2 && t2 != end) {
            }
        }
    }
}

// MSH 2.2: one node list, elements with their tags (the first is the physical group)
void read_v2(std::istream &in, FileMesh &fm) {
    std::string tok;
    while (in >> tok) {
        if (tok == "$Nodes") {
            const int64_t n = take<int64_t>(in, "node count");
            if (n < 0) bad("negative node count");
            for (int64_t k = 0; k < n; ++k) {
                const int64_t tag = take<int64_t>(in, "node tag");
                std::array<double, 3> x;
                for (double &c : x) c = take<double>(in, "node coordinate");
                fm.nodes[tag] = x;
            }
            expect_end(in, "Nodes");
        } else if (tok == "$Elements") {
            const int64_t n = take<int64_t>(in, "element count");
            if (n < 0) bad("negative element count");
            for (int64_t k = 0; k < n; ++k) {
                take<int64_t>(in, "element tag");
                const int type = take<int>(in, "element type");
                const int ntags = take<int>(in, "tag count");
                GType g;
                if (!gmsh_type(type, g)) bad("element type " + std::to_string(type) + " is not supported");
                if (ntags < 0 || ntags > 64) bad("bad tag count");
                int ph = 0;
                for (int t = 0; t < ntags; ++t) {
                    const int v = take<int>(in, "element tag value");
                    if (t == 0) ph = v;
                }
                RawElem e{type, ph, std::vector<int64_t>(g.nodes)};
                for (auto &v : e.nodes) v = take<int64_t>(in, "element node");
                fm.elems.push_back(std::move(e));
            }
            expect_end(in, "Elements");
        } else if (!tok.empty() && tok[0] == '$' && tok.rfind("$End", 0) != 0) {
            const std::string end = "$End" + tok.substr(1);
            std::string t2;
            while (in >> t2 && t2 != end) {
            }
        }
    }
}

// local faces of the cell types (cyclic node order), for the boundary test
const int kFaces[5][6][4] = {
    {},
    {{0, 1}, {1, 2}, {2, 0}},                                                           // tri3
    {{0, 1}, {1, 2}, {2, 3}, {3, 0}},                                                   // quad4
    {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}},                                      // tet4
    {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}}};   // hex8
const int kNF[5] = {0, 3, 4, 4, 6}, kNV[5] = {0, 3, 4, 4, 8}, kFV[5] = {0, 2, 2, 3, 4};

}  // namespace

std::shared_ptr<Mesh> read_gmsh(const std::string &path, double scale) {
    if (!(scale > 0) || !std::isfinite(scale)) throw Error(NBTE_ERR_INVALID_ARG, "scale must be positive");
    std::ifstream in(path);
    if (!in) throw Error(NBTE_ERR_INVALID_ARG, "cannot open " + path);
    std::string tok;
    if (!(in >> tok) || tok != "$MeshFormat") bad("no $MeshFormat header");
    const std::string version = take<std::string>(in, "format version");
    const int ftype = take<int>(in, "file type");
    take<int>(in, "data size");
    if (ftype != 0) bad("binary files are not supported (save as ASCII)");
    expect_end(in, "MeshFormat");
    FileMesh fm;
    if (version.rfind("4.", 0) == 0) read_v4(in, fm);
    else if (version.rfind("2.", 0) == 0) read_v2(in, fm);
    else bad("format version " + version + " is not supported (2.2 or 4.1)");

    // cells: the elements of the highest dimension, one type
    int dim = 0;
    for (const auto &e : fm.elems) {
        GType g;
        gmsh_type(e.type, g);
        dim = std::max(dim, g.dim);
    }
    if (dim < 2) bad("no 2D or 3D elements");
    int ctype = 0;
    for (const auto &e : fm.elems) {
        GType g;
        gmsh_type(e.type, g);
        if (g.dim != dim) continue;
        if (ctype && ctype != g.cell_type) throw Error(NBTE_ERR_MESH, "mixed cell types are not supported");
        ctype = g.cell_type;
    }
    // dense node numbering of the nodes the cells use
    std::map<int64_t, int64_t> index;
    std::vector<double> xyz;
    std::vector<int64_t> cells;
    std::vector<int32_t> region;
    auto node = [&](int64_t tag) -> int64_t {
        auto it = index.find(tag);
        if (it != index.end()) return it->second;
        auto nt = fm.nodes.find(tag);
        if (nt == fm.nodes.end()) throw Error(NBTE_ERR_MESH, "element refers to a missing node");
        const int64_t id = (int64_t)index.size();
        index[tag] = id;
        for (int ax = 0; ax < dim; ++ax) xyz.push_back(nt->second[ax] * scale);
        return id;
    };
    for (const auto &e : fm.elems) {
        GType g;
        gmsh_type(e.type, g);
        if (g.dim != dim) continue;
        for (int64_t t : e.nodes) cells.push_back(node(t));
        region.push_back(e.phys);
    }
    const int64_t N = (int64_t)region.size();
    // the boundary: cell faces that occur once
    const int nf = kNF[ctype], nv = kNV[ctype], fv = kFV[ctype];
    std::map<std::array<int64_t, 4>, int> count;
    auto key_of = [&](const int64_t *nd, int k) {
        std::array<int64_t, 4> key{-1, -1, -1, -1};
        for (int j = 0; j < k; ++j) key[j] = nd[j];
        std::sort(key.begin(), key.begin() + k);
        return key;
    };
    for (int64_t c = 0; c < N; ++c)
        for (int f = 0; f < nf; ++f) {
            int64_t nd[4];
            for (int j = 0; j < fv; ++j) nd[j] = cells[c * nv + kFaces[ctype][f][j]];
            ++count[key_of(nd, fv)];
        }
    std::vector<int64_t> bnodes;
    std::vector<int32_t> btags;
    std::set<std::array<int64_t, 4>> seen;
    for (const auto &e : fm.elems) {
        GType g;
        gmsh_type(e.type, g);
        if (g.dim != dim - 1 || (int)e.nodes.size() != fv) continue;
        int64_t nd[4];
        bool known = true;
        for (int j = 0; j < fv; ++j) {
            auto it = index.find(e.nodes[j]);
            if (it == index.end()) {
                known = false;
                break;
            }
            nd[j] = it->second;
        }
        if (!known) continue;
        const auto key = key_of(nd, fv);
        auto it = count.find(key);
        if (it == count.end() || it->second != 1 || !seen.insert(key).second) continue;   // interior or repeated
        bnodes.insert(bnodes.end(), nd, nd + fv);
        btags.push_back(e.phys);
    }
    auto m = build_mesh(dim, (int64_t)index.size(), xyz.data(), ctype, N, cells.data(), (int64_t)btags.size(),
                        bnodes.data(), btags.data());
    m->region = std::move(region);
    return m;
}

}  // namespace nbte

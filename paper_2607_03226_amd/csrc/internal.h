// Internal declarations of the nbte library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/nbte.h"

namespace nbte {

// Error carried from deep inside the library to the ABI layer, where it becomes
// a status code plus the thread-local message.
struct Error : std::runtime_error {
    nbte_status code;
    Error(nbte_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define NBTE_HIP(call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            throw ::nbte::Error(e_ == hipErrorOutOfMemory ? NBTE_ERR_OUT_OF_MEMORY : NBTE_ERR_DEVICE, \
                                std::string(#call) + ": " + hipGetErrorString(e_));           \
    } while (0)

void set_last_error(const std::string &msg);

// ---------------------------------------------------------------- device buffers
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    void alloc(size_t n) {
        if (n == bytes && ptr) return;
        release();
        if (n == 0) return;
        NBTE_HIP(hipMalloc(&ptr, n));
        bytes = n;
    }
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

template <class T>
void upload(DevBuf &b, const std::vector<T> &h, hipStream_t s) {
    b.alloc(h.size() * sizeof(T));
    if (!h.empty()) NBTE_HIP(hipMemcpyAsync(b.ptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// ---------------------------------------------------------------- mesh
struct Mesh {
    int dim = 0;
    int cell_type = 0;
    int F = 0;                       // faces per cell
    int64_t N = 0;                   // cells
    int64_t NBF = 0;                 // boundary faces
    std::vector<int32_t> nbr;        // N*F: >=0 neighbour, <0: -(1 + boundary face)
    std::vector<double> S;           // N*F*3 outward area vectors (+S / -S on the two sides)
    std::vector<double> xf;          // N*F*3 face centroids
    std::vector<double> V;           // N volumes
    std::vector<double> xc;          // N*3 cell centroids (vertex average)
    std::vector<int32_t> bf_owner;   // NBF
    std::vector<int32_t> bf_local;   // NBF
    std::vector<int32_t> bf_tag;     // NBF
    double total_volume = 0.0;
    double max_closure = 0.0;
    std::vector<int32_t> region;     // N physical group of each cell (mesh files), empty otherwise
};

std::shared_ptr<Mesh> build_mesh(int32_t dim, int64_t n_nodes, const double *xyz, int32_t cell_type,
                                 int64_t n_cells, const int64_t *cell_nodes, int64_t n_bfaces,
                                 const int64_t *bface_nodes, const int32_t *bface_tag);
// Gmsh MSH 4.1 / 2.2 ASCII file -> mesh (cells: the highest-dimension
// elements; boundary faces: the lower-dimension elements on the boundary,
// tagged by physical group; regions: the cells' physical groups)
std::shared_ptr<Mesh> read_gmsh(const std::string &path, double scale);

// ---------------------------------------------------------------- tables
struct BandTable {
    int B = 0;
    std::vector<double> C, v, tau;
    double beta = 0, C_tot = 0;
};

struct Quadrature {
    int D = 0;
    std::vector<double> s, w;  // D*3, D
    double W = 0;
};

struct BoundarySpec {
    int kind = 0;
    double T_wall = 0, p = 0;
};

// Per-direction sweep schedule: cells in upwind (topological) order, grouped
// in levels such that every upwind neighbour of a cell lies in an earlier level.
struct Schedule {
    int D = 0;
    int max_levels = 0;
    std::vector<int32_t> perm;       // D*N cells in level order
    std::vector<int32_t> lvl_ptr;    // concatenated level offsets, per direction L_i+1 entries
    std::vector<int32_t> lvl_off;    // D+1: start of direction i's entries in lvl_ptr
    // LDS staging: slot[i*N + c] = LDS slot holding cell c's value during the
    // sweep of direction i while a downwind cell still needs it, -1 = read the
    // stored value from HBM instead (no consumer, or the slot budget is full)
    std::vector<int32_t> slot;
    int slot_cap = 0;                // budget the slots were assigned for
    int max_slots = 0;               // slots actually used (max over directions)
    int64_t spilled = 0;             // consumed values that did not fit
    int max_ghosts = 0;              // most boundary inflow faces feeding one level
    int max_ghost_pair = 0;          // most inflow faces feeding two consecutive levels
    // Cyclic upwind graphs: where the topological order stalls, the lowest
    // unfinished cell is released and its upwind faces towards unfinished
    // cells are lagged: they take the upwind value of the previous iterate
    // (like boundary inflow), which keeps the fixed point.  Sorted keys
    // (i N + c) F + f of the lagged faces.
    std::vector<int64_t> lagged;
    bool is_lagged(int64_t N, int F, int i, int64_t c, int f) const {
        if (lagged.empty()) return false;
        return std::binary_search(lagged.begin(), lagged.end(), ((int64_t)i * N + c) * F + f);
    }
};

Schedule build_schedule(const Mesh &m, const Quadrature &q);
// (Re)assign LDS slots for a budget of `cap` slots per direction.
void assign_slots(const Mesh &m, const Quadrature &q, Schedule &sc, int cap);

// The sweep of every direction compiled into level-ordered streams (index
// i*N + k for position k of direction i), so that the sweep kernel loads
// everything it needs for a cell with independent, coalesced loads:
//   cell, LDS slot of the cell's own value, up to maxin upwind references
//   (ranges below), their coefficients |s.S|/V, and the outflow sum
//   sum_{a>0} a.  Unused reference entries have coefficient 0 and point at
//   the LDS zero block; maxin is the fan-in class (2, 3 or 5) of the widest
//   cell.
struct SweepProgram {
    int maxin = 0;
    std::vector<int32_t> cell, slot, ref;   // ref: maxin * D*N
    std::vector<int32_t> upc;               // maxin * D*N: upwind cell (own cell for inflow / unused)
    std::vector<double> coef, sout;         // coef: maxin * D*N
    // Ghosts: the boundary inflow values a level needs, in sweep order.
    // gptr has the layout of lvl_ptr (per direction L_i + 1 entries, absolute
    // offsets into the concatenated ghost list); ghost_src[g] = (bf*D + i)*B,
    // the inflow row of ghost g; a boundary reference of a cell in level l is
    // -1 - (its rank among the ghosts of level l).
    std::vector<int32_t> gptr;
    std::vector<int64_t> ghost_src;
    std::vector<int32_t> in_row;            // NBF*D: ghost row of incoming (bf, i), -1 otherwise
    int max_ghosts = 0;                     // most ghosts of one level
    std::vector<int32_t> lag;               // per lagged face (4 ints): ghost row, direction, cell, upwind cell
};
// record reference encoding (shared with the sweep kernel): >= 0 an element
// offset in the workgroup's LDS (a staged value: ring_off + slot ls; a ghost
// kept in LDS: gbuf0 + ((pos_l + rank) mod gring) ls, pos_l = the kept ghosts
// of the direction's earlier levels; see sweep_lds_layout); [-kSpillBase, -1] ghost read from HBM, -1 - row; below:
// the stored value of the upwind cell at stream position k of the same
// direction, -(kSpillBase + 1) - k.  The own slot ("mine") is the element
// offset of the staged value, or the LDS scratch block when no later cell
// reads the value from LDS.
constexpr int32_t kSpillBase = 1 << 24;
SweepProgram build_program(const Mesh &m, const Quadrature &q, const Schedule &sc, int B, int gcap, int gring, int ls,
                           int es);

// Boundary plan: per boundary face kind/wall data, s.S per direction and the
// specular mirror table.
struct BoundaryPlan {
    std::vector<int32_t> kind;        // NBF (NBTE_BC_*)
    std::vector<double> theta_w;      // NBF deviational wall temperature
    std::vector<double> p;            // NBF specular fraction (1 specular, 0 diffuse/thermalizing)
    std::vector<double> sdotS;        // NBF*D
    std::vector<double> win;          // NBF: sum_{in} w |s.S|
    std::vector<int32_t> mirror;      // NBF*D mirror direction (-1 where unused)
    bool has_thermalizing = false;
};

BoundaryPlan build_boundary_plan(const Mesh &m, const Quadrature &q,
                                 const std::vector<nbte_boundary> &bcs, double T_ref);

// Least-squares cell gradients of the second-order scheme: weights w_cf
// (N*F*3) with G_c = sum_f w_cf (e_n(f) - e_c) over the interior face
// neighbours (offsets d = x_n - x_c of the vertex-average centres,
// w = (sum d d^T)^-1 d in the mesh's dimension); zero for a cell whose
// offsets do not span the dimension (eigenvalue ratio below 1e-8).
std::vector<double> build_lsq_weights(const Mesh &m);

// Diffusion operator of the synthetic correction (V-weighted, SPD) in CSR.
struct DiffusionOperator {
    std::vector<int32_t> row_ptr, col;
    std::vector<double> val;
    std::vector<double> dir_rhs;      // sum over thermalizing faces of T_f theta_w
};

DiffusionOperator build_diffusion(const Mesh &m, const BandTable &b, const Quadrature &q,
                                  const BoundaryPlan &bp);

}  // namespace nbte

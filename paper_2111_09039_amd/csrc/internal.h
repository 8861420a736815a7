// Internal declarations of the HSIM library (host side).  Not part of the ABI.
#pragma once

#include <cstdarg>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hsim.h"

namespace hsim {

// ---------------------------------------------------------------- errors
struct Error {
    hsim_status code;
    std::string msg;
};
[[noreturn]] void fail(hsim_status code, const char* fmt, ...);
void set_last_error(const std::string& msg);

// integer tuning knob from the environment (dflt when unset or not a number)
int env_int(const char* name, int dflt);

// tile edge of the supernodal factor panels (doubles per tile = NB * NB)
constexpr int NB = 32;

// ------------------------------------------------------------- host data
struct Csr {
    int64_t rows = 0, cols = 0;
    std::vector<int64_t> ptr;   // rows + 1
    std::vector<int32_t> idx;   // sorted within a row
    std::vector<double> val;
    int64_t nnz() const { return (int64_t)idx.size(); }
};

struct Graph {                  // undirected edge graph, CSR, Euclidean edge lengths
    std::vector<int64_t> ptr;
    std::vector<int32_t> nbr;
    std::vector<double> w;
};

struct Mesh {
    int64_t nv = 0, nf = 0;
    std::vector<double> V;      // nv x 3
    std::vector<int32_t> F;     // nf x 3
};

// mesh.cpp
void validate_mesh(const Mesh& m);
Graph edge_graph(const Mesh& m);
void check_connected(const Graph& g, int64_t nv);   // HSIM_E_MESH unless every vertex is reachable from 0
double surface_area(const Mesh& m);
// per vertex: 1 if it lies on an edge that belongs to exactly one triangle
std::vector<char> boundary_vertex_flags(const Mesh& m);
Csr cotan_stiffness(const Mesh& m);
std::vector<double> lumped_mass(const Mesh& m, int lumping, const double* density);
// index structures of the device assembly of S (pattern, corner lists) and the lumped M
struct AssemblyMaps {
    Csr S;                        // pattern only (val empty), sorted columns, diagonal included
    std::vector<int64_t> corner;  // [2 nnz]: corners 3t + k opposite the entry's edge, -1 padded
    std::vector<int64_t> dptr;    // [n + 1]: each vertex's diagonal corners in dcorner
    std::vector<int64_t> dcorner;
    std::vector<int64_t> vptr;    // [n + 1]: each vertex's triangles in vtri (ascending)
    std::vector<int32_t> vtri;
};
AssemblyMaps assembly_maps(const Mesh& m, const Graph& g);

// hierarchy.cpp
std::vector<int64_t> level_sizes(int64_t n0, int T, int64_t n_coarsest, int growth_mode);
std::vector<int32_t> farthest_point_sampling(const Graph& g, int64_t n, int64_t count, uint64_t seed);
Csr prolongation(const Graph& g, int64_t n, const std::vector<int32_t>& fine_verts, bool fine_is_all,
                 const std::vector<int32_t>& coarse_verts, double sigma, double area, double* rho_out);
// S_next = U^T S U and M_next = U^T M U on one pattern (M given on the pattern of S)
void galerkin(const Csr& U, const Csr& S, const std::vector<double>& Mval, Csr& S_next,
              std::vector<double>& M_next);

// ---------------------------------------------------------- symbolic LDL^T
// One supernode = one front of the multifrontal factorisation.  Columns
// [start, start + ns) of the elimination order; struct rows (> start + ns) in
// `rows[rows_ptr[f] .. rows_ptr[f+1])`.  Local front index space: pivots
// 0..ns-1, dummy pivots ns..ns_pad-1, struct rows ns_pad .. ns_pad+mu-1,
// padding up to m_pad = ns_pad + mu_pad.  Storage: lower triangle of
// NB x NB tiles, tile (I, J) (I >= J) at tile_base + tri(I, J), each tile
// column-major.
struct Front {
    int64_t start = 0;
    int32_t ns = 0, mu = 0, ns_pad = 0, mu_pad = 0;
    int32_t Mt = 0, nsb = 0;      // tile rows of the front, pivot tile columns
    int32_t parent = -1, tlev = 0;
    int32_t child_slot = 0;       // index among the children of its parent
    int64_t tile_base = 0;        // offset in doubles into the level's tile storage
    int64_t linv_base = 0;        // offset of the nsb inverse diagonal tiles
    int64_t d_base = 0;           // offset of the ns_pad pivots in D
    int64_t ubuf_row = 0;         // first row of its update block in the solve's update buffer
    int64_t gather_base = 0;      // first entry of its row-gather list pointer array (m + 1 entries)
};

inline int64_t tri_tile(int32_t Mt, int32_t I, int32_t J) {
    // column-packed lower triangle of Mt x Mt tiles
    return (int64_t)J * Mt - (int64_t)J * (J - 1) / 2 + (I - J);
}

struct Symbolic {
    std::vector<int32_t> perm;    // perm[k] = level vertex eliminated k-th
    std::vector<int32_t> iperm;   // inverse
    std::vector<Front> fronts;    // in elimination order (children before parents)
    std::vector<int64_t> rows_ptr;
    std::vector<int32_t> rows;    // struct rows (elimination indices), sorted
    int32_t tree_levels = 0;
    int64_t tile_doubles = 0, linv_doubles = 0, d_doubles = 0, ubuf_rows = 0;
    double flops = 0;
    int64_t factor_nnz = 0;       // unpadded L entries (lower triangle incl. diagonal)
    // fronts of every tree level, contiguous (fronts are renumbered so that
    // tree level t holds fronts [tlev_ptr[t], tlev_ptr[t+1]))
    std::vector<int32_t> tlev_ptr;
    // relative indices of every front's struct rows in its parent (local index space)
    std::vector<int32_t> rel;     // indexed like `rows`
    // row-gather lists of the solve: for front f and local row r in [0, m),
    // gather_ptr[gather_base + r] .. [+1] lists rows of the update buffer
    std::vector<int64_t> gather_ptr;
    std::vector<int64_t> gather_idx;
    // assembly map: lower-triangle entries of A in front tiles
    std::vector<int64_t> asm_dst;   // offset into tile storage
    std::vector<int64_t> asm_src;   // index into the level CSR value arrays, -1 = dummy pivot (value 1)
    std::vector<int64_t> asm_tlev_ptr;
    // factorisation work lists per (tree level t, pivot tile step k):
    // steps of level t are [step_ptr[t], step_ptr[t+1]); for step s,
    // diag items   diag[diag_ptr[s] .. diag_ptr[s+1])      (front)
    // panel items  panel[panel_ptr[s] .. panel_ptr[s+1])   (front, I)
    // update items upd[upd_ptr[s] .. upd_ptr[s+1])         (front, I, J)
    std::vector<int32_t> step_ptr;
    std::vector<int64_t> diag_ptr, panel_ptr, upd_ptr;
    std::vector<int32_t> diag, panel, upd;
    // extend-add passes per (tree level t, child slot c): children listed in
    // ea[ea_ptr[t * max_children + c] ..]
    int32_t max_children = 0;
    std::vector<int64_t> ea_ptr;
    std::vector<int32_t> ea;
};

// order.cpp
Symbolic analyse(const Csr& S, const double* coords /* n x 3 */, int64_t n);
void check_symbolic(const Symbolic& sy, int64_t n, int64_t nnz);

// ------------------------------------------------------------ device data
struct DeviceBuffer {
    void* p = nullptr;
    size_t bytes = 0;
    DeviceBuffer() = default;
    DeviceBuffer(const DeviceBuffer&) = delete;
    DeviceBuffer& operator=(const DeviceBuffer&) = delete;
    ~DeviceBuffer();
    void alloc(size_t nbytes);
    template <class T> T* as() const { return static_cast<T*>(p); }
    template <class T> void upload(const std::vector<T>& v) {
        alloc(v.size() * sizeof(T));
        copy_in(v.data(), v.size() * sizeof(T));
    }
    void copy_in(const void* src, size_t nbytes);
    void release();
};

struct Level;
struct Workspace;

}  // namespace hsim

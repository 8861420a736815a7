// Device parts of the hierarchy build (Algorithm 3 and the mesh topology it
// runs on).  Host declarations only; the kernels live in build_dev.hip.
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

#include <hip/hip_runtime.h>

#include "internal.h"

namespace hsim {

// Device copies of the mesh and of its edge graph, kept while the hierarchy
// is built.
struct DevMesh {
    DeviceBuffer V, F, gptr, gnbr, gw;
    int64_t nv = 0, nf = 0;
};

// validate_mesh followed by edge_graph, on the device: the same checks in the
// same order with the same messages (HSIM_E_MESH), and the same graph (the
// neighbours of a vertex ascending, the same Euclidean edge lengths bit for
// bit).  Leaves the device copies of V, F and the graph in dm.
void device_mesh_graph(const Mesh& m, DevMesh& dm, Graph& g);

// farthest_point_sampling on the device graph of dm: the same insertion
// order bit for bit (the same distances: the fixpoint of the relaxations does
// not depend on their order; farthest ties to the lowest vertex index).
std::vector<int32_t> device_fps(const DevMesh& dm, int64_t count, uint64_t seed);

// The same in two halves: start launches the sampling on a stream of its own
// (non-blocking: work on the null stream neither waits for it nor holds it
// up) and returns at once; finish waits for it and returns the order.  The
// run owns its work arrays; destroying it waits for the kernel first.  dm
// must outlive the run.
struct FpsRun {
    DeviceBuffer dist, q0, q1, f0, f1, bmax, bidx, dirty, dlist, order, status;
    hipStream_t stream = nullptr;
    int64_t count = 0;
    FpsRun() = default;
    FpsRun(const FpsRun&) = delete;
    FpsRun& operator=(const FpsRun&) = delete;
    ~FpsRun();
};
std::unique_ptr<FpsRun> device_fps_start(const DevMesh& dm, int64_t count, uint64_t seed);
std::vector<int32_t> device_fps_finish(FpsRun& r);

}  // namespace hsim

namespace hsim {
// galerkin on the device: S_next = U^T S U, M_next = U^T M U on the
// structural pattern, every entry summed with the host's terms in the host's
// order (bit for bit the host result).  False (nothing computed) when the
// coarse level is too large for the row marks of one workgroup.
bool device_galerkin(const Csr& U, const Csr& S, const std::vector<double>& Mval, Csr& S_next,
                     std::vector<double>& M_next);
}  // namespace hsim

namespace hsim {
// prolongation on the device graph of dm (eq. radius, eq. basis, row
// normalisation): the same U bit for bit (exact bounded distances, the same
// weights and sums).  False (nothing computed) when a ball outgrows its work
// arrays or a fine row would be empty (the host then builds U).
bool device_prolongation(const DevMesh& dm, const std::vector<int32_t>& fine_verts, bool fine_is_all,
                         const std::vector<int32_t>& coarse_verts, double sigma, double area, Csr& U,
                         double* rho_out);
}  // namespace hsim

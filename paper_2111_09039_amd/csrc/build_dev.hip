// Device parts of the hierarchy build for gfx950: the mesh checks and the
// edge graph that the geodesic distances of Algorithm 3 run on, and the
// farthest point sampling of Algorithm 3 itself.
//
// The results equal the host build's bit for bit.  Floating-point values are
// formed with the host's operations in the host's order (no contraction in
// this file), and the only order-dependent choices are resolved by index: the
// neighbours of a vertex are sorted, and farthest-point ties go to the lowest
// vertex index.  The sampling's distances are the least fixpoint of
// d(u) = min(d(u), d(v) + w(v, u)) from the new sample: a value that every
// order of relaxations reaches (rounding is monotone and w >= 0), so the
// parallel relaxation below gives the host Dijkstra's distances exactly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>

#include "build_dev.h"

#pragma clang fp contract(off)

namespace hsim {

namespace {
#define BDCHECK(x)                                                                                  \
    do {                                                                                            \
        const hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) fail(HSIM_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_));             \
    } while (0)

constexpr unsigned long long NONE = ~0ull;

inline unsigned grid_of(int64_t n, int block) {
    const int64_t g = (n + block - 1) / block;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, int64_t(1) << 20));
}
template <class T>
T* dp(const DeviceBuffer& b) {
    return static_cast<T*>(b.p);
}
}  // namespace

// ------------------------------------------------------------ prefix sums
// out[i] = sum of in[j], j < i, for i < n (2048 values per workgroup of 1024
// threads); sums[b] = the workgroup's total.  in and out may alias (every
// value is read before the barrier and written after it by the same thread).
__global__ __launch_bounds__(1024) void k_scan_block(const int64_t* in, int64_t n, int64_t* out, int64_t* sums) {
    __shared__ int64_t s[1024];
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * 2048 + 2 * t;
    const int64_t a = i0 < n ? in[i0] : 0, b = i0 + 1 < n ? in[i0 + 1] : 0;
    s[t] = a + b;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    const int64_t excl = s[t] - (a + b);
    if (i0 < n) out[i0] = excl;
    if (i0 + 1 < n) out[i0 + 1] = excl + a;
    if (t == 1023) sums[blockIdx.x] = s[1023];
}
__global__ void k_scan_add(int64_t* out, int64_t n, const int64_t* __restrict__ offs) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] += offs[i / 2048];
}
__global__ void k_copy1(int64_t* dst, const int64_t* src) { *dst = *src; }

// out[0 .. n] = exclusive prefix sums of in[0 .. n) and the total (out may be in)
static void dev_scan(const int64_t* in, int64_t* out, int64_t n) {
    const int64_t nb = std::max<int64_t>(1, (n + 2047) / 2048);
    DeviceBuffer sums;
    sums.alloc((size_t)(nb + 1) * sizeof(int64_t));
    k_scan_block<<<(unsigned)nb, 1024>>>(in, n, out, dp<int64_t>(sums));
    BDCHECK(hipGetLastError());
    if (nb > 1) {
        dev_scan(dp<int64_t>(sums), dp<int64_t>(sums), nb);
        k_scan_add<<<grid_of(n, 256), 256>>>(out, n, dp<int64_t>(sums));
        BDCHECK(hipGetLastError());
        k_copy1<<<1, 1>>>(out + n, dp<int64_t>(sums) + nb);
    } else {
        k_copy1<<<1, 1>>>(out + n, dp<int64_t>(sums));
    }
    BDCHECK(hipGetLastError());
    BDCHECK(hipDeviceSynchronize());   // sums is freed on return
}

// ------------------------------------------------------------ mesh checks
// first vertex with a non-finite coordinate
__global__ void k_check_coords(const double* __restrict__ V, int64_t nv, unsigned long long* first) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 3 * nv; i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(V[i])) atomicMin(first, (unsigned long long)(i / 3));
}
// first triangle with an index out of range or a repeated vertex; first
// degenerate triangle among the others (the host's area test, same operations)
__global__ void k_check_tris(const double* __restrict__ V, const int32_t* __restrict__ F, int64_t nf, int64_t nv,
                             unsigned long long* first_bad, unsigned long long* first_degen) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nf; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t f0 = F[3 * t], f1 = F[3 * t + 1], f2 = F[3 * t + 2];
        const bool range = f0 >= 0 && f0 < nv && f1 >= 0 && f1 < nv && f2 >= 0 && f2 < nv;
        if (!range || f0 == f1 || f1 == f2 || f2 == f0) {
            atomicMin(first_bad, (unsigned long long)t);
            continue;
        }
        const double* a = V + 3 * (int64_t)f0;
        const double* b = V + 3 * (int64_t)f1;
        const double* c = V + 3 * (int64_t)f2;
        const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        const double e3[3] = {c[0] - b[0], c[1] - b[1], c[2] - b[2]};
        const double cx = e1[1] * e2[2] - e1[2] * e2[1];
        const double cy = e1[2] * e2[0] - e1[0] * e2[2];
        const double cz = e1[0] * e2[1] - e1[1] * e2[0];
        const double a2 = cx * cx + cy * cy + cz * cz;
        const double l1 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
        const double lb = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
        const double lc = e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2];
        double l2 = l1;
        if (l2 < lb) l2 = lb;
        if (l2 < lc) l2 = lc;
        if (!(a2 > 1e-24 * l2 * l2)) atomicMin(first_degen, (unsigned long long)t);
    }
}
// triangles per vertex
__global__ void k_count_tri(const int32_t* __restrict__ F, int64_t nf, unsigned long long* cnt) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < 3 * nf; e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[F[e]], 1ull);
}
__global__ void k_check_used(const int64_t* __restrict__ cnt, int64_t nv, unsigned long long* first) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x)
        if (cnt[i] == 0) atomicMin(first, (unsigned long long)i);
}
// triangles of every vertex into its segment of vtri (any order; sorted next)
__global__ void k_fill_tri(const int32_t* __restrict__ F, int64_t nf, unsigned long long* cursor, int32_t* vtri) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < 3 * nf; e += (int64_t)gridDim.x * blockDim.x)
        vtri[atomicAdd(&cursor[F[e]], 1ull)] = (int32_t)(e / 3);
}
// per vertex: its triangles ascending; the other two corners of each as
// candidate neighbours, sorted, made unique in place (count in ucnt), and the
// first neighbour u > v whose edge lies in more than two triangles
__global__ void k_neighbours(const int32_t* __restrict__ F, const int64_t* __restrict__ vptr, int32_t* vtri,
                             int64_t nv, int32_t* cand, int64_t* ucnt, unsigned long long* first_nm) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t0 = vptr[v], d = vptr[v + 1] - t0;
        int32_t* T = vtri + t0;
        for (int64_t i = 1; i < d; ++i) {
            const int32_t x = T[i];
            int64_t j = i - 1;
            while (j >= 0 && T[j] > x) {
                T[j + 1] = T[j];
                --j;
            }
            T[j + 1] = x;
        }
        int32_t* C = cand + 2 * t0;
        for (int64_t i = 0; i < d; ++i) {
            const int32_t* f = F + 3 * (int64_t)T[i];
            const int k = f[0] == v ? 0 : (f[1] == v ? 1 : 2);
            C[2 * i] = f[(k + 1) % 3];
            C[2 * i + 1] = f[(k + 2) % 3];
        }
        for (int64_t i = 1; i < 2 * d; ++i) {
            const int32_t x = C[i];
            int64_t j = i - 1;
            while (j >= 0 && C[j] > x) {
                C[j + 1] = C[j];
                --j;
            }
            C[j + 1] = x;
        }
        int64_t u = 0;
        bool flagged = false;
        for (int64_t i = 0; i < 2 * d;) {
            int64_t j = i;
            while (j < 2 * d && C[j] == C[i]) ++j;
            if (!flagged && j - i > 2 && C[i] > v) {
                atomicMin(first_nm, ((unsigned long long)v << 32) | (unsigned long long)(uint32_t)C[i]);
                flagged = true;
            }
            C[u++] = C[i];
            i = j;
        }
        ucnt[v] = u;
    }
}
// CSR of the edge graph: neighbours ascending, Euclidean lengths (squared
// differences summed x, y, z in order, then the square root)
__global__ void k_graph_fill(const int64_t* __restrict__ vptr, const int32_t* __restrict__ cand,
                             const int64_t* __restrict__ gptr, int64_t nv, const double* __restrict__ V,
                             int32_t* __restrict__ nbr, double* __restrict__ w) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t* C = cand + 2 * vptr[v];
        const int64_t o = gptr[v], d = gptr[v + 1] - o;
        for (int64_t i = 0; i < d; ++i) {
            const int32_t j = C[i];
            nbr[o + i] = j;
            const double dx = V[3 * v] - V[3 * (int64_t)j];
            const double dy = V[3 * v + 1] - V[3 * (int64_t)j + 1];
            const double dz = V[3 * v + 2] - V[3 * (int64_t)j + 2];
            w[o + i] = sqrt(dx * dx + dy * dy + dz * dz);
        }
    }
}
__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

static unsigned long long read_u64(const DeviceBuffer& b, size_t i) {
    unsigned long long v = 0;
    BDCHECK(hipMemcpy(&v, static_cast<const unsigned long long*>(b.p) + i, sizeof v, hipMemcpyDeviceToHost));
    return v;
}

void device_mesh_graph(const Mesh& m, DevMesh& dm, Graph& g) {
    if (m.nv < 3 || m.nf < 1) fail(HSIM_E_MESH, "mesh needs >= 3 vertices and >= 1 triangle");
    const int64_t nv = m.nv, nf = m.nf;
    dm.nv = nv;
    dm.nf = nf;
    dm.V.upload(m.V);
    dm.F.upload(m.F);
    DeviceBuffer flags;   // first non-finite vertex, bad triangle, degenerate triangle, unused vertex, non-manifold edge
    flags.alloc(5 * sizeof(unsigned long long));
    unsigned long long* fl = dp<unsigned long long>(flags);
    k_fill_u64<<<1, 64>>>(fl, 5, NONE);
    k_check_coords<<<grid_of(3 * nv, 256), 256>>>(dp<double>(dm.V), nv, fl);
    k_check_tris<<<grid_of(nf, 256), 256>>>(dp<double>(dm.V), dp<int32_t>(dm.F), nf, nv, fl + 1, fl + 2);
    BDCHECK(hipGetLastError());
    BDCHECK(hipDeviceSynchronize());
    // the host's order of checks and messages
    unsigned long long bad = read_u64(flags, 0);
    if (bad != NONE) fail(HSIM_E_MESH, "vertex %lld has a non-finite coordinate", (long long)bad);
    bad = read_u64(flags, 1);
    if (bad != NONE) {
        const int32_t* f = &m.F[3 * bad];
        for (int k = 0; k < 3; ++k)
            if (f[k] < 0 || f[k] >= nv)
                fail(HSIM_E_MESH, "triangle %lld references vertex %d out of range", (long long)bad, f[k]);
        fail(HSIM_E_MESH, "triangle %lld repeats a vertex", (long long)bad);
    }
    // every index is in range from here on
    DeviceBuffer cnt, vptr, cursor, vtri, cand, ucnt;
    cnt.alloc((size_t)nv * sizeof(int64_t));
    vptr.alloc((size_t)(nv + 1) * sizeof(int64_t));
    k_fill_u64<<<grid_of(nv, 256), 256>>>(dp<unsigned long long>(cnt), nv, 0ull);
    k_count_tri<<<grid_of(3 * nf, 256), 256>>>(dp<int32_t>(dm.F), nf, dp<unsigned long long>(cnt));
    k_check_used<<<grid_of(nv, 256), 256>>>(dp<int64_t>(cnt), nv, fl + 3);
    BDCHECK(hipGetLastError());
    BDCHECK(hipDeviceSynchronize());
    bad = read_u64(flags, 3);
    if (bad != NONE) fail(HSIM_E_MESH, "vertex %lld belongs to no triangle", (long long)bad);
    bad = read_u64(flags, 2);
    if (bad != NONE) fail(HSIM_E_MESH, "triangle %lld is degenerate", (long long)bad);
    dev_scan(dp<int64_t>(cnt), dp<int64_t>(vptr), nv);
    cursor.alloc((size_t)nv * sizeof(int64_t));
    BDCHECK(hipMemcpy(cursor.p, vptr.p, (size_t)nv * sizeof(int64_t), hipMemcpyDeviceToDevice));
    vtri.alloc((size_t)3 * nf * sizeof(int32_t));
    cand.alloc((size_t)6 * nf * sizeof(int32_t));
    ucnt.alloc((size_t)(nv + 1) * sizeof(int64_t));
    k_fill_tri<<<grid_of(3 * nf, 256), 256>>>(dp<int32_t>(dm.F), nf, dp<unsigned long long>(cursor), dp<int32_t>(vtri));
    k_neighbours<<<grid_of(nv, 256), 256>>>(dp<int32_t>(dm.F), dp<int64_t>(vptr), dp<int32_t>(vtri), nv,
                                            dp<int32_t>(cand), dp<int64_t>(ucnt), fl + 4);
    BDCHECK(hipGetLastError());
    BDCHECK(hipDeviceSynchronize());
    bad = read_u64(flags, 4);
    if (bad != NONE) {
        const int64_t a = (int64_t)(bad >> 32), b = (int64_t)(bad & 0xffffffffull);
        size_t c = 0;
        for (int64_t t = 0; t < nf; ++t)
            for (int k = 0; k < 3; ++k) {
                const int64_t u = m.F[3 * t + k], v = m.F[3 * t + (k + 1) % 3];
                c += std::min(u, v) == a && std::max(u, v) == b;
            }
        fail(HSIM_E_MESH, "edge (%lld,%lld) is shared by %zu triangles", (long long)a, (long long)b, c);
    }
    dm.gptr.alloc((size_t)(nv + 1) * sizeof(int64_t));
    dev_scan(dp<int64_t>(ucnt), dp<int64_t>(dm.gptr), nv);
    g.ptr.resize(nv + 1);
    BDCHECK(hipMemcpy(g.ptr.data(), dm.gptr.p, (size_t)(nv + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    const int64_t ne = g.ptr[nv];
    dm.gnbr.alloc((size_t)std::max<int64_t>(1, ne) * sizeof(int32_t));
    dm.gw.alloc((size_t)std::max<int64_t>(1, ne) * sizeof(double));
    k_graph_fill<<<grid_of(nv, 256), 256>>>(dp<int64_t>(vptr), dp<int32_t>(cand), dp<int64_t>(dm.gptr), nv,
                                            dp<double>(dm.V), dp<int32_t>(dm.gnbr), dp<double>(dm.gw));
    BDCHECK(hipGetLastError());
    g.nbr.resize(ne);
    g.w.resize(ne);
    BDCHECK(hipMemcpy(g.nbr.data(), dm.gnbr.p, (size_t)ne * sizeof(int32_t), hipMemcpyDeviceToHost));
    BDCHECK(hipMemcpy(g.w.data(), dm.gw.p, (size_t)ne * sizeof(double), hipMemcpyDeviceToHost));
    check_connected(g, nv);
}

// ------------------------------------------------------------ farthest point sampling
// One workgroup runs the whole sampling (it is sequential over the samples):
// after each new sample, rounds of relaxation over a frontier (queues and
// in-queue flags double-buffered: a vertex improved while it waits in the
// current round goes to the next one), then the farthest vertex from the
// per-block maxima of the distances (blocks of 1024 vertices; only blocks
// with an improved vertex are rescanned).  Distances are non-negative
// doubles, so their bit patterns order like the values and atomicMin on the
// 64-bit patterns is an exact minimum.  Every hand-over of global data
// between threads (queues, flags, block maxima) crosses an agent-scope fence
// and a barrier, so the readers' first-level cache holds no stale line; a
// distance read in the middle of a round may miss an improvement made in the
// same round, but the improved vertex is queued again for the next round.
namespace {
constexpr int FPS_T = 1024;
// (value, index) pairs: larger value wins, ties to the lower index
__device__ __forceinline__ bool better(double a, int32_t ia, double b, int32_t ib) {
    return a > b || (a == b && ia < ib);
}
__device__ __forceinline__ void fence_sync() {
    __threadfence();
    __syncthreads();
}
// the better (value, index) pair of the 64 lanes, in every lane
__device__ __forceinline__ void wave_best(double& v, int32_t& i) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o);
        const int32_t oi = __shfl_xor(i, o);
        if (better(ov, oi, v, i)) {
            v = ov;
            i = oi;
        }
    }
}
}  // namespace

__global__ void k_fps_init(int64_t n, unsigned long long* dist, unsigned int* f0, unsigned int* f1,
                           unsigned int* dirty, int64_t nb) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        dist[i] = 0x7ff0000000000000ull;   // +inf
        f0[i] = 0;
        f1[i] = 0;
        if (i < nb) dirty[i] = 1;
    }
}

__global__ __launch_bounds__(FPS_T) void k_fps(const int64_t* __restrict__ gptr, const int32_t* __restrict__ nbr,
                                               const double* __restrict__ w, int64_t n, int64_t count, int32_t start,
                                               unsigned long long* dist, int32_t* q0, int32_t* q1,
                                               unsigned int* f0, unsigned int* f1, double* bmax, int32_t* bidx,
                                               unsigned int* dirty, int32_t* dlist, int32_t* order, int32_t* status) {
    __shared__ int32_t qn[2];
    __shared__ int32_t nd_;
    __shared__ double rv[FPS_T / 64];
    __shared__ int32_t ri[FPS_T / 64];
    __shared__ int32_t sel, stop;
    const int t = threadIdx.x;
    const int64_t nb = (n + FPS_T - 1) / FPS_T;
    int32_t* Q[2] = {q0, q1};
    unsigned int* FL[2] = {f0, f1};
    if (t == 0) {
        sel = start;
        stop = 0;
    }
    __syncthreads();
    for (int64_t k = 0; k < count; ++k) {
        const int32_t s = sel;
        if (t == 0) order[k] = s;
        if (k + 1 == count) break;   // the last sample's distances choose nothing
        // relaxation from s
        if (t == 0) {
            atomicMin(&dist[s], 0ull);
            atomicOr(&dirty[s / FPS_T], 1u);
            Q[0][0] = s;
            FL[0][s] = 1;
            qn[0] = 1;
            qn[1] = 0;
        }
        fence_sync();
        int cur = 0;
        while (true) {
            const int32_t len = qn[cur];
            if (len == 0) break;
            int32_t* qo = Q[cur ^ 1];
            unsigned int* fo = FL[cur ^ 1];
            for (int32_t e = t; e < len; e += FPS_T) {
                const int32_t v = Q[cur][e];
                FL[cur][v] = 0;
                const double dv = __longlong_as_double((long long)dist[v]);
                const int64_t k0 = gptr[v], k1 = gptr[v + 1];
                // up to eight edges at a time: their minima are independent
                // atomics, issued together so that the round trips overlap
                for (int64_t kb = k0; kb < k1; kb += 8) {
                    int32_t uu[8];
                    unsigned long long nb[8], old[8];
                    unsigned int was[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        uu[j] = kb + j < k1 ? nbr[kb + j] : 0;
                        nb[j] = kb + j < k1 ? (unsigned long long)__double_as_longlong(dv + w[kb + j]) : 0ull;
                    }
#pragma unroll
                    for (int j = 0; j < 8; ++j) old[j] = kb + j < k1 ? atomicMin(&dist[uu[j]], nb[j]) : 0ull;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        was[j] = 1u;
                        if (kb + j < k1 && nb[j] < old[j]) {
                            atomicOr(&dirty[uu[j] / FPS_T], 1u);
                            was[j] = atomicExch(&fo[uu[j]], 1u);
                        }
                    }
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        if (was[j] == 0u) qo[atomicAdd(&qn[cur ^ 1], 1)] = uu[j];
                }
            }
            fence_sync();
            if (t == 0) qn[cur] = 0;
            __syncthreads();
            cur ^= 1;
        }
        // maxima of the blocks that changed
        if (t == 0) nd_ = 0;
        __syncthreads();
        for (int64_t b = t; b < nb; b += FPS_T)
            if (dirty[b]) {
                dirty[b] = 0;
                dlist[atomicAdd(&nd_, 1)] = (int32_t)b;
            }
        fence_sync();
        // a wave per changed block: 16 entries per lane, then the wave's
        // shuffle reduction (the farthest vertex under a total order, so the
        // order of the comparisons does not matter)
        const int32_t ndirty = nd_;
        const int lane = t & 63, wv = t >> 6;
        for (int32_t j = wv; j < ndirty; j += FPS_T / 64) {
            const int64_t b = dlist[j];
            double bv = -1.0;
            int32_t bi = INT32_MAX;
#pragma unroll 4
            for (int k = 0; k < FPS_T / 64; ++k) {
                const int64_t i = b * FPS_T + k * 64 + lane;
                const double d = i < n ? __longlong_as_double((long long)dist[i]) : -1.0;
                if (better(d, (int32_t)i, bv, bi)) {
                    bv = d;
                    bi = (int32_t)i;
                }
            }
            wave_best(bv, bi);
            if (lane == 0) {
                bmax[b] = bv;
                bidx[b] = bi;
            }
        }
        fence_sync();
        // farthest vertex over the blocks: per thread, per wave, then wave 0
        double bv = -1.0;
        int32_t bi = INT32_MAX;
        for (int64_t b = t; b < nb; b += FPS_T)
            if (better(bmax[b], bidx[b], bv, bi)) {
                bv = bmax[b];
                bi = bidx[b];
            }
        wave_best(bv, bi);
        if (lane == 0) {
            rv[wv] = bv;
            ri[wv] = bi;
        }
        __syncthreads();
        if (wv == 0) {
            bv = lane < FPS_T / 64 ? rv[lane] : -1.0;
            bi = lane < FPS_T / 64 ? ri[lane] : INT32_MAX;
            wave_best(bv, bi);
            if (lane == 0) {
                if (!(bv > 0)) stop = 1;   // no vertex left at a positive distance
                sel = bi;
            }
        }
        __syncthreads();
        if (stop) {
            if (t == 0) *status = 1;
            return;
        }
    }
}

FpsRun::~FpsRun() {
    if (stream) {
        (void)hipStreamSynchronize(stream);   // the buffers outlive the kernel, also on an error path
        (void)hipStreamDestroy(stream);
    }
}

std::unique_ptr<FpsRun> device_fps_start(const DevMesh& dm, int64_t count, uint64_t seed) {
    BDCHECK(hipDeviceSynchronize());   // the graph in dm is complete
    std::unique_ptr<FpsRun> r(new FpsRun());
    const int64_t n = dm.nv;
    const int64_t nb = (n + FPS_T - 1) / FPS_T;
    r->count = count;
    r->dist.alloc((size_t)n * sizeof(unsigned long long));
    r->q0.alloc((size_t)n * sizeof(int32_t));
    r->q1.alloc((size_t)n * sizeof(int32_t));
    r->f0.alloc((size_t)n * sizeof(unsigned int));
    r->f1.alloc((size_t)n * sizeof(unsigned int));
    r->bmax.alloc((size_t)nb * sizeof(double));
    r->bidx.alloc((size_t)nb * sizeof(int32_t));
    r->dirty.alloc((size_t)nb * sizeof(unsigned int));
    r->dlist.alloc((size_t)nb * sizeof(int32_t));
    r->order.alloc((size_t)count * sizeof(int32_t));
    r->status.alloc(sizeof(int32_t));
    // its own stream, which does not wait for (or hold up) the null stream
    BDCHECK(hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking));
    BDCHECK(hipMemsetAsync(r->status.p, 0, sizeof(int32_t), r->stream));
    const int32_t start = (int32_t)(seed % (uint64_t)n);
    k_fps_init<<<grid_of(n, 256), 256, 0, r->stream>>>(n, dp<unsigned long long>(r->dist), dp<unsigned int>(r->f0),
                                                       dp<unsigned int>(r->f1), dp<unsigned int>(r->dirty), nb);
    BDCHECK(hipGetLastError());
    k_fps<<<1, FPS_T, 0, r->stream>>>(dp<int64_t>(dm.gptr), dp<int32_t>(dm.gnbr), dp<double>(dm.gw), n, count, start,
                                      dp<unsigned long long>(r->dist), dp<int32_t>(r->q0), dp<int32_t>(r->q1),
                                      dp<unsigned int>(r->f0), dp<unsigned int>(r->f1), dp<double>(r->bmax),
                                      dp<int32_t>(r->bidx), dp<unsigned int>(r->dirty), dp<int32_t>(r->dlist),
                                      dp<int32_t>(r->order), dp<int32_t>(r->status));
    BDCHECK(hipGetLastError());
    return r;
}

std::vector<int32_t> device_fps_finish(FpsRun& r) {
    BDCHECK(hipStreamSynchronize(r.stream));
    int32_t st = 0;
    BDCHECK(hipMemcpy(&st, r.status.p, sizeof st, hipMemcpyDeviceToHost));
    if (st) fail(HSIM_E_MESH, "farthest point sampling ran out of distinct vertices");
    std::vector<int32_t> out(r.count);
    BDCHECK(hipMemcpy(out.data(), r.order.p, (size_t)r.count * sizeof(int32_t), hipMemcpyDeviceToHost));
    return out;
}

std::vector<int32_t> device_fps(const DevMesh& dm, int64_t count, uint64_t seed) {
    std::unique_ptr<FpsRun> r = device_fps_start(dm, count, seed);
    return device_fps_finish(*r);
}

}  // namespace hsim

namespace hsim {

// ------------------------------------------------------------ Galerkin products
// T = S U and T_M = M U, row j: the terms s_jl u_lk (m_jl u_lk) over the
// entries l of S row j in order and the entries k of U row l in order, summed
// per column in that order (the host's dense accumulator), columns ascending.
// pass 0 counts the columns of every row, pass 1 writes the row.  Rows with
// more than TCAP columns set *overflow (the caller falls back to the host).
namespace {
constexpr int TCAP = 96;
}
__global__ __launch_bounds__(64) void k_su(int pass, const int64_t* __restrict__ sptr,
                                           const int32_t* __restrict__ sidx, const double* __restrict__ sval,
                                           const double* __restrict__ mval, const int64_t* __restrict__ uptr,
                                           const int32_t* __restrict__ uidx, const double* __restrict__ uval,
                                           int64_t nf, int64_t* cnt, const int64_t* __restrict__ tptr,
                                           int32_t* tidx, double* ta, double* tb, int32_t* overflow) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nf; j += (int64_t)gridDim.x * blockDim.x) {
        int32_t ks[TCAP];
        double aa[TCAP], bb[TCAP];
        int n = 0;
        bool over = false;
        for (int64_t b = sptr[j]; b < sptr[j + 1] && !over; ++b) {
            const int64_t l = sidx[b];
            for (int64_t c = uptr[l]; c < uptr[l + 1]; ++c) {
                const int32_t k = uidx[c];
                int q = 0;
                while (q < n && ks[q] != k) ++q;
                if (q == n) {
                    if (n == TCAP) {
                        over = true;
                        break;
                    }
                    ks[n] = k;
                    aa[n] = 0.0;
                    bb[n] = 0.0;
                    ++n;
                }
                aa[q] += sval[b] * uval[c];
                bb[q] += mval[b] * uval[c];
            }
        }
        if (over) {
            *overflow = 1;
            if (pass == 0) cnt[j] = 0;
            continue;
        }
        if (pass == 0) {
            cnt[j] = n;
            continue;
        }
        for (int x = 1; x < n; ++x) {
            const int32_t k = ks[x];
            const double va = aa[x], vb = bb[x];
            int y = x - 1;
            while (y >= 0 && ks[y] > k) {
                ks[y + 1] = ks[y];
                aa[y + 1] = aa[y];
                bb[y + 1] = bb[y];
                --y;
            }
            ks[y + 1] = k;
            aa[y + 1] = va;
            bb[y + 1] = vb;
        }
        const int64_t o = tptr[j];
        for (int x = 0; x < n; ++x) {
            tidx[o + x] = ks[x];
            ta[o + x] = aa[x];
            tb[o + x] = bb[x];
        }
    }
}
// pattern of row i of U^T T: the columns of the T rows of the fine vertices in
// U^T row i, marked in an LDS bitmap (nc bits); pass 0 counts, pass 1 writes
// the columns ascending
__global__ __launch_bounds__(256) void k_galerkin_pattern(int pass, const int64_t* __restrict__ utp,
                                                          const int32_t* __restrict__ uti,
                                                          const int64_t* __restrict__ tptr,
                                                          const int32_t* __restrict__ tidx, int64_t nc,
                                                          int64_t* rowlen, const int64_t* __restrict__ nptr,
                                                          int32_t* nidx) {
    extern __shared__ unsigned int bits[];
    __shared__ unsigned long long total;
    const int64_t i = blockIdx.x;
    const int64_t words = (nc + 31) / 32;
    for (int64_t w = threadIdx.x; w < words; w += blockDim.x) bits[w] = 0;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    for (int64_t a = utp[i] + threadIdx.x; a < utp[i + 1]; a += blockDim.x) {
        const int64_t j = uti[a];
        for (int64_t c = tptr[j]; c < tptr[j + 1]; ++c) {
            const int32_t k = tidx[c];
            atomicOr(&bits[k >> 5], 1u << (k & 31));
        }
    }
    __syncthreads();
    if (pass == 0) {
        unsigned long long mine = 0;
        for (int64_t w = threadIdx.x; w < words; w += blockDim.x) mine += __popc(bits[w]);
        atomicAdd(&total, mine);
        __syncthreads();
        if (threadIdx.x == 0) rowlen[i] = (int64_t)total;
        return;
    }
    if (threadIdx.x == 0) {
        int64_t o = nptr[i];
        for (int64_t w = 0; w < words; ++w) {
            unsigned int m = bits[w];
            while (m) {
                const int bit = __ffs(m) - 1;
                nidx[o++] = (int32_t)(w * 32 + bit);
                m &= m - 1;
            }
        }
    }
}
// row i of U^T T by one wave: the fine rows j of U^T row i in order, the
// entries of T row j on the lanes (distinct columns, so distinct slots), each
// lane adding u_ij T_jk into the LDS slot of its column k: every entry of the
// result is the host's sum in the host's order
__global__ __launch_bounds__(64) void k_galerkin_values(const int64_t* __restrict__ utp,
                                                        const int32_t* __restrict__ uti,
                                                        const double* __restrict__ utv,
                                                        const int64_t* __restrict__ tptr,
                                                        const int32_t* __restrict__ tidx,
                                                        const double* __restrict__ ta, const double* __restrict__ tb,
                                                        const int64_t* __restrict__ nptr,
                                                        const int32_t* __restrict__ nidx, double* outS,
                                                        double* outM) {
    extern __shared__ double slots[];   // [len] S sums, [len] M sums, [len] columns (as int32)
    const int64_t i = blockIdx.x;
    const int64_t r0 = nptr[i], len = nptr[i + 1] - r0;
    double* accS = slots;
    double* accM = slots + len;
    int32_t* key = reinterpret_cast<int32_t*>(slots + 2 * len);
    const int lane = threadIdx.x;
    for (int64_t x = lane; x < len; x += 64) {
        accS[x] = 0.0;
        accM[x] = 0.0;
        key[x] = nidx[r0 + x];
    }
    __syncthreads();
    for (int64_t a = utp[i]; a < utp[i + 1]; ++a) {
        const int64_t j = uti[a];
        const double uij = utv[a];
        for (int64_t c = tptr[j] + lane; c < tptr[j + 1]; c += 64) {
            const int32_t k = tidx[c];
            int64_t lo = 0, hi = len;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (key[mid] < k) lo = mid + 1;
                else hi = mid;
            }
            accS[lo] += uij * ta[c];
            accM[lo] += uij * tb[c];
        }
        __syncthreads();
    }
    for (int64_t x = lane; x < len; x += 64) {
        outS[r0 + x] = accS[x];
        outM[r0 + x] = accM[x];
    }
}
__global__ void k_row_of(const int64_t* __restrict__ ptr, int64_t rows, int32_t* row) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x)
        for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) row[e] = (int32_t)r;
}
// exact symmetry: both mirror entries become their average (the upper one's thread writes both)
__global__ void k_galerkin_sym(const int64_t* __restrict__ nptr, const int32_t* __restrict__ nidx,
                               const int32_t* __restrict__ nrow, int64_t nnz, double* S, double* M) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = nrow[e], j = nidx[e];
        if (j <= i) continue;
        int64_t lo = nptr[j], hi = nptr[j + 1];
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (nidx[mid] < i) lo = mid + 1;
            else hi = mid;
        }
        if (lo == nptr[j + 1] || nidx[lo] != i) continue;   // the pattern is symmetric: not reached
        const double s = 0.5 * (S[e] + S[lo]);
        const double m = 0.5 * (M[e] + M[lo]);
        S[e] = S[lo] = s;
        M[e] = M[lo] = m;
    }
}

bool device_galerkin(const Csr& U, const Csr& S, const std::vector<double>& Mval, Csr& Sn, std::vector<double>& Mn) {
    const int64_t nf = U.rows, nc = U.cols, nu = U.nnz();
    const size_t bitmap = (size_t)(nc + 31) / 32 * sizeof(unsigned int);
    if (bitmap > 64 * 1024 || nu == 0) return false;
    DeviceBuffer uptr, uidx, uval, sptr, sidx, sval, mval, ovf, tcnt, tptr, tidx, ta, tb;
    uptr.upload(U.ptr);
    uidx.upload(U.idx);
    uval.upload(U.val);
    sptr.upload(S.ptr);
    sidx.upload(S.idx);
    sval.upload(S.val);
    mval.upload(Mval);
    ovf.alloc(sizeof(int32_t));
    BDCHECK(hipMemset(ovf.p, 0, sizeof(int32_t)));
    // T = S U, T_M = M U
    tcnt.alloc((size_t)nf * sizeof(int64_t));
    tptr.alloc((size_t)(nf + 1) * sizeof(int64_t));
    k_su<<<grid_of(nf, 64), 64>>>(0, dp<int64_t>(sptr), dp<int32_t>(sidx), dp<double>(sval), dp<double>(mval),
                                   dp<int64_t>(uptr), dp<int32_t>(uidx), dp<double>(uval), nf, dp<int64_t>(tcnt),
                                   nullptr, nullptr, nullptr, nullptr, dp<int32_t>(ovf));
    BDCHECK(hipGetLastError());
    int32_t over = 0;
    BDCHECK(hipMemcpy(&over, ovf.p, sizeof over, hipMemcpyDeviceToHost));
    if (over) return false;
    dev_scan(dp<int64_t>(tcnt), dp<int64_t>(tptr), nf);
    int64_t nt = 0;
    BDCHECK(hipMemcpy(&nt, dp<int64_t>(tptr) + nf, sizeof nt, hipMemcpyDeviceToHost));
    tidx.alloc((size_t)std::max<int64_t>(1, nt) * sizeof(int32_t));
    ta.alloc((size_t)std::max<int64_t>(1, nt) * sizeof(double));
    tb.alloc((size_t)std::max<int64_t>(1, nt) * sizeof(double));
    k_su<<<grid_of(nf, 64), 64>>>(1, dp<int64_t>(sptr), dp<int32_t>(sidx), dp<double>(sval), dp<double>(mval),
                                   dp<int64_t>(uptr), dp<int32_t>(uidx), dp<double>(uval), nf, nullptr,
                                   dp<int64_t>(tptr), dp<int32_t>(tidx), dp<double>(ta), dp<double>(tb),
                                   dp<int32_t>(ovf));
    BDCHECK(hipGetLastError());
    // U^T (coarse rows, fine columns ascending), transposed on the host where
    // U was built (a stable counting pass)
    DeviceBuffer utp, uti, utv, rowlen, nptr;
    {
        std::vector<int64_t> tp(nc + 1, 0);
        for (int64_t k = 0; k < nu; ++k) tp[U.idx[k] + 1]++;
        for (int64_t i = 0; i < nc; ++i) tp[i + 1] += tp[i];
        std::vector<int32_t> ti(nu);
        std::vector<double> tv(nu);
        std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
        for (int64_t j = 0; j < nf; ++j)
            for (int64_t k = U.ptr[j]; k < U.ptr[j + 1]; ++k) {
                ti[fill[U.idx[k]]] = (int32_t)j;
                tv[fill[U.idx[k]]++] = U.val[k];
            }
        utp.upload(tp);
        uti.upload(ti);
        utv.upload(tv);
    }
    // pattern and values of U^T T
    rowlen.alloc((size_t)nc * sizeof(int64_t));
    nptr.alloc((size_t)(nc + 1) * sizeof(int64_t));
    k_galerkin_pattern<<<(unsigned)nc, 256, bitmap>>>(0, dp<int64_t>(utp), dp<int32_t>(uti), dp<int64_t>(tptr),
                                                       dp<int32_t>(tidx), nc, dp<int64_t>(rowlen), nullptr, nullptr);
    BDCHECK(hipGetLastError());
    dev_scan(dp<int64_t>(rowlen), dp<int64_t>(nptr), nc);
    Sn = Csr();
    Sn.rows = Sn.cols = nc;
    Sn.ptr.resize(nc + 1);
    BDCHECK(hipMemcpy(Sn.ptr.data(), nptr.p, (size_t)(nc + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    const int64_t nn = Sn.ptr[nc];
    int64_t maxlen = 0;
    for (int64_t i = 0; i < nc; ++i) maxlen = std::max(maxlen, Sn.ptr[i + 1] - Sn.ptr[i]);
    const size_t lds = (size_t)maxlen * (2 * sizeof(double) + sizeof(int32_t));
    if (lds > 64 * 1024) return false;
    DeviceBuffer nidx, nrow, outS, outM;
    nidx.alloc((size_t)std::max<int64_t>(1, nn) * sizeof(int32_t));
    nrow.alloc((size_t)std::max<int64_t>(1, nn) * sizeof(int32_t));
    outS.alloc((size_t)std::max<int64_t>(1, nn) * sizeof(double));
    outM.alloc((size_t)std::max<int64_t>(1, nn) * sizeof(double));
    k_galerkin_pattern<<<(unsigned)nc, 256, bitmap>>>(1, dp<int64_t>(utp), dp<int32_t>(uti), dp<int64_t>(tptr),
                                                       dp<int32_t>(tidx), nc, nullptr, dp<int64_t>(nptr),
                                                       dp<int32_t>(nidx));
    k_row_of<<<grid_of(nc, 256), 256>>>(dp<int64_t>(nptr), nc, dp<int32_t>(nrow));
    k_galerkin_values<<<(unsigned)nc, 64, lds>>>(dp<int64_t>(utp), dp<int32_t>(uti), dp<double>(utv),
                                                 dp<int64_t>(tptr), dp<int32_t>(tidx), dp<double>(ta),
                                                 dp<double>(tb), dp<int64_t>(nptr), dp<int32_t>(nidx),
                                                 dp<double>(outS), dp<double>(outM));
    k_galerkin_sym<<<grid_of(nn, 256), 256>>>(dp<int64_t>(nptr), dp<int32_t>(nidx), dp<int32_t>(nrow), nn,
                                              dp<double>(outS), dp<double>(outM));
    BDCHECK(hipGetLastError());
    Sn.idx.resize(nn);
    Sn.val.resize(nn);
    Mn.resize(nn);
    BDCHECK(hipMemcpy(Sn.idx.data(), nidx.p, (size_t)nn * sizeof(int32_t), hipMemcpyDeviceToHost));
    BDCHECK(hipMemcpy(Sn.val.data(), outS.p, (size_t)nn * sizeof(double), hipMemcpyDeviceToHost));
    BDCHECK(hipMemcpy(Mn.data(), outM.p, (size_t)nn * sizeof(double), hipMemcpyDeviceToHost));
    return true;
}

}  // namespace hsim

namespace hsim {

// ------------------------------------------------------------ prolongation
// Workgroup b owns the distance array dist + b n (all +inf between balls) and
// takes the coarse vertices b, b + gridDim.x, ...: for each, rounds of
// relaxation from its vertex that keep only distances below rho (the host's
// bounded Dijkstra reaches exactly these vertices with exactly these
// distances), then an entry (fine row, coarse column, 1 - d / rho) for every
// reached fine vertex with a positive weight, and the touched distances reset.
// Hand-overs between threads cross an agent-scope fence and a barrier.
namespace {
constexpr int PB_T = 256;
}
__global__ __launch_bounds__(PB_T) void k_prolong_balls(const int64_t* __restrict__ gptr,
                                                        const int32_t* __restrict__ nbr,
                                                        const double* __restrict__ w, int64_t n,
                                                        const int32_t* __restrict__ coarse, int64_t nc,
                                                        const int32_t* __restrict__ pos, double rho,
                                                        unsigned long long* dist_all, unsigned int* flag_all,
                                                        int32_t* q_all, int32_t* touched_all, int32_t cap,
                                                        int32_t* erow, int32_t* ecol, double* ewt, int64_t ecap,
                                                        unsigned long long* ecount, int32_t* overflow) {
    __shared__ int32_t qn[2], nt, stop;
    const int t = threadIdx.x;
    unsigned long long* dist = dist_all + (int64_t)blockIdx.x * n;
    unsigned int* flag = flag_all + (int64_t)blockIdx.x * n;
    int32_t* Q[2] = {q_all + (int64_t)blockIdx.x * 2 * cap, q_all + (int64_t)blockIdx.x * 2 * cap + cap};
    int32_t* touched = touched_all + (int64_t)blockIdx.x * cap;
    const unsigned long long rbits = (unsigned long long)__double_as_longlong(rho);
    for (int64_t ci = blockIdx.x; ci < nc; ci += gridDim.x) {
        const int32_t src = coarse[ci];
        if (t == 0) {
            dist[src] = 0ull;
            touched[0] = src;
            nt = 1;
            Q[0][0] = src;
            qn[0] = 1;
            qn[1] = 0;
            stop = 0;
        }
        fence_sync();
        int cur = 0;
        while (true) {
            const int32_t len = qn[cur];
            if (len == 0 || stop) break;
            for (int32_t e = t; e < len; e += PB_T) {
                const int32_t v = Q[cur][e];
                flag[v] = 0;
                const double dv = __longlong_as_double((long long)dist[v]);
                for (int64_t kk = gptr[v]; kk < gptr[v + 1]; ++kk) {
                    const int32_t u = nbr[kk];
                    const double nd = dv + w[kk];
                    const unsigned long long nb = (unsigned long long)__double_as_longlong(nd);
                    if (nb >= rbits) continue;
                    const unsigned long long old = atomicMin(&dist[u], nb);
                    if (nb < old) {
                        if (old == 0x7ff0000000000000ull) {
                            const int32_t p = atomicAdd(&nt, 1);
                            if (p < cap) touched[p] = u;
                            else stop = 1;
                        }
                        if (atomicExch(&flag[u], 1u) == 0u) {
                            const int32_t p = atomicAdd(&qn[cur ^ 1], 1);
                            if (p < cap) Q[cur ^ 1][p] = u;
                            else stop = 1;
                        }
                    }
                }
            }
            fence_sync();
            if (t == 0) qn[cur] = 0;
            __syncthreads();
            cur ^= 1;
        }
        if (stop) {
            if (t == 0) *overflow = 1;
            return;
        }
        const int32_t cnt = nt;
        for (int32_t e = t; e < cnt; e += PB_T) {
            const int32_t v = touched[e];
            const double d = __longlong_as_double((long long)dist[v]);
            const int32_t row = pos[v];
            if (row >= 0) {
                const double wt = 1.0 - d / rho;
                if (wt > 0.0) {
                    const unsigned long long o = atomicAdd(ecount, 1ull);
                    if ((int64_t)o < ecap) {
                        erow[o] = row;
                        ecol[o] = (int32_t)ci;
                        ewt[o] = wt;
                    } else {
                        *overflow = 1;
                    }
                }
            }
            dist[v] = 0x7ff0000000000000ull;
            flag[v] = 0;
        }
        fence_sync();
    }
}
__global__ void k_fill_u32(unsigned int* p, int64_t n, unsigned int v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_count_rows(const int32_t* __restrict__ erow, int64_t ne, unsigned long long* cnt) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[erow[e]], 1ull);
}
__global__ void k_scatter_rows(const int32_t* __restrict__ erow, const int32_t* __restrict__ ecol,
                               const double* __restrict__ ewt, int64_t ne, unsigned long long* cursor, int32_t* idx,
                               double* val) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long o = atomicAdd(&cursor[erow[e]], 1ull);
        idx[o] = ecol[e];
        val[o] = ewt[e];
    }
}
// every row: columns ascending, then U_jk = (1 / sum_k U_jk) * U_jk with the
// sum taken in column order (the host's normalisation)
__global__ void k_sort_normalise(const int64_t* __restrict__ ptr, int64_t rows, int32_t* idx, double* val) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = ptr[r], b = ptr[r + 1];
        for (int64_t i = a + 1; i < b; ++i) {
            const int32_t x = idx[i];
            const double v = val[i];
            int64_t j = i - 1;
            while (j >= a && idx[j] > x) {
                idx[j + 1] = idx[j];
                val[j + 1] = val[j];
                --j;
            }
            idx[j + 1] = x;
            val[j + 1] = v;
        }
        double s = 0.0;
        for (int64_t i = a; i < b; ++i) s += val[i];
        const double inv = 1.0 / s;
        for (int64_t i = a; i < b; ++i) val[i] = inv * val[i];
    }
}

bool device_prolongation(const DevMesh& dm, const std::vector<int32_t>& fine_verts, bool fine_is_all,
                         const std::vector<int32_t>& coarse_verts, double sigma, double area, Csr& U,
                         double* rho_out) {
    const int64_t n = dm.nv, nc = (int64_t)coarse_verts.size();
    const int64_t nf = fine_is_all ? n : (int64_t)fine_verts.size();
    const double rho = std::sqrt(sigma * area / ((double)nc * M_PI));
    if (rho_out) *rho_out = rho;
    std::vector<int32_t> pos(n, -1);
    if (fine_is_all)
        for (int64_t i = 0; i < n; ++i) pos[i] = (int32_t)i;
    else
        for (int64_t j = 0; j < nf; ++j) pos[fine_verts[j]] = (int32_t)j;
    // work arrays: one distance array per workgroup (about 2 GB of them at most)
    const int64_t slots = std::max<int64_t>(16, std::min<int64_t>(256, (int64_t(2) << 30) / (12 * std::max<int64_t>(1, n))));
    const int32_t cap = (int32_t)std::min<int64_t>(n, 1 << 17);
    const int64_t ecap = 16 * nf + 1024;
    DeviceBuffer dpos, dcoarse, dist, flag, q, touched, erow, ecol, ewt, ecount, ovf;
    dpos.upload(pos);
    dcoarse.upload(coarse_verts);
    dist.alloc((size_t)slots * n * sizeof(unsigned long long));
    flag.alloc((size_t)slots * n * sizeof(unsigned int));
    q.alloc((size_t)slots * 2 * cap * sizeof(int32_t));
    touched.alloc((size_t)slots * cap * sizeof(int32_t));
    erow.alloc((size_t)ecap * sizeof(int32_t));
    ecol.alloc((size_t)ecap * sizeof(int32_t));
    ewt.alloc((size_t)ecap * sizeof(double));
    ecount.alloc(sizeof(unsigned long long));
    ovf.alloc(sizeof(int32_t));
    BDCHECK(hipMemset(ecount.p, 0, sizeof(unsigned long long)));
    BDCHECK(hipMemset(ovf.p, 0, sizeof(int32_t)));
    k_fill_u64<<<grid_of(slots * n, 256), 256>>>(dp<unsigned long long>(dist), slots * n, 0x7ff0000000000000ull);
    k_fill_u32<<<grid_of(slots * n, 256), 256>>>(dp<unsigned int>(flag), slots * n, 0u);
    k_prolong_balls<<<(unsigned)slots, PB_T>>>(dp<int64_t>(dm.gptr), dp<int32_t>(dm.gnbr), dp<double>(dm.gw), n,
                                               dp<int32_t>(dcoarse), nc, dp<int32_t>(dpos), rho,
                                               dp<unsigned long long>(dist), dp<unsigned int>(flag), dp<int32_t>(q),
                                               dp<int32_t>(touched), cap, dp<int32_t>(erow), dp<int32_t>(ecol),
                                               dp<double>(ewt), ecap, dp<unsigned long long>(ecount),
                                               dp<int32_t>(ovf));
    BDCHECK(hipGetLastError());
    BDCHECK(hipDeviceSynchronize());
    int32_t over = 0;
    unsigned long long ne = 0;
    BDCHECK(hipMemcpy(&over, ovf.p, sizeof over, hipMemcpyDeviceToHost));
    BDCHECK(hipMemcpy(&ne, ecount.p, sizeof ne, hipMemcpyDeviceToHost));
    if (over) return false;
    DeviceBuffer cnt, ptr, cur, idx, val;
    cnt.alloc((size_t)nf * sizeof(int64_t));
    ptr.alloc((size_t)(nf + 1) * sizeof(int64_t));
    k_fill_u64<<<grid_of(nf, 256), 256>>>(dp<unsigned long long>(cnt), nf, 0ull);
    k_count_rows<<<grid_of((int64_t)ne, 256), 256>>>(dp<int32_t>(erow), (int64_t)ne, dp<unsigned long long>(cnt));
    BDCHECK(hipGetLastError());
    dev_scan(dp<int64_t>(cnt), dp<int64_t>(ptr), nf);
    U = Csr();
    U.rows = nf;
    U.cols = nc;
    U.ptr.resize(nf + 1);
    BDCHECK(hipMemcpy(U.ptr.data(), ptr.p, (size_t)(nf + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    for (int64_t j = 0; j < nf; ++j)
        if (U.ptr[j + 1] == U.ptr[j]) return false;   // a fine vertex with no coarse vertex within rho
    cur.alloc((size_t)nf * sizeof(int64_t));
    BDCHECK(hipMemcpy(cur.p, ptr.p, (size_t)nf * sizeof(int64_t), hipMemcpyDeviceToDevice));
    idx.alloc((size_t)std::max<unsigned long long>(1, ne) * sizeof(int32_t));
    val.alloc((size_t)std::max<unsigned long long>(1, ne) * sizeof(double));
    k_scatter_rows<<<grid_of((int64_t)ne, 256), 256>>>(dp<int32_t>(erow), dp<int32_t>(ecol), dp<double>(ewt),
                                                        (int64_t)ne, dp<unsigned long long>(cur), dp<int32_t>(idx),
                                                        dp<double>(val));
    k_sort_normalise<<<grid_of(nf, 64), 64>>>(dp<int64_t>(ptr), nf, dp<int32_t>(idx), dp<double>(val));
    BDCHECK(hipGetLastError());
    U.idx.resize(ne);
    U.val.resize(ne);
    BDCHECK(hipMemcpy(U.idx.data(), idx.p, (size_t)ne * sizeof(int32_t), hipMemcpyDeviceToHost));
    BDCHECK(hipMemcpy(U.val.data(), val.p, (size_t)ne * sizeof(double), hipMemcpyDeviceToHost));
    return true;
}

}  // namespace hsim

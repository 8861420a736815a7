// HIP kernels of the HSIM hot path for gfx950 (MI355X): CSR SpMM, the
// supernodal multifrontal LDL^T (assembly, extend-add, tiled partial
// factorisation), the level-scheduled block triangular solves, the
// Rayleigh-Ritz Gram products, the Ritz update with the fused residual, and
// the cyclic Jacobi rounds of the dense generalized eigenproblems.
//
// Layout conventions: dense n x k blocks are row-major ("vertex-major") with
// a padded leading dimension; factor tiles are 32 x 32 column-major; a front
// stores the lower triangle of its tiles column-packed.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "kernels.h"

namespace hsim {

namespace {
constexpr int T32 = 32;
constexpr int TT = T32 * T32;
constexpr int NXCD = 8;           // XCDs; workgroups are dispatched round-robin over them

__device__ __forceinline__ int64_t tri(int32_t Mt, int32_t I, int32_t J) {
    return (int64_t)J * Mt - (int64_t)J * (J - 1) / 2 + (I - J);
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// compute units of the current device (persistent launches)
int device_cus() {
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cus[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cus[dev] = v;
    }
    return cus[dev];
}

// 16 x 16 x 4 matrix-core products.  Operand layout (lane l of the wave):
// A (16 x 4) element (l % 16, l / 16), B (4 x 16) element (l / 16, l % 16).
// Result element v of lane l: FP64 (l / 16 + 4 v, l % 16), FP32
// (4 (l / 16) + v, l % 16).  In the FP64 layout, element v of a 16 x 16
// result is exactly the B operand of rows 4 v .. 4 v + 3 of that result.
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ dbl4 mfma4(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ flt4 mfma4(float a, float b, flt4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// (row, col) inside a 16 x 16 MFMA result of lane l, element v
__device__ __forceinline__ void frag_rc(double, int l, int v, int& r, int& c) { r = l / 16 + 4 * v; c = l % 16; }
__device__ __forceinline__ void frag_rc(float, int l, int v, int& r, int& c) { r = 4 * (l / 16) + v; c = l % 16; }

// Dynamic LDS above the default 64 KB needs an explicit opt-in per kernel;
// gfx950 has 160 KB per workgroup (static + dynamic).
constexpr size_t LDS_PER_WG = 160 * 1024;
inline hipError_t ensure_dynamic_lds(const void* fn, size_t dyn_bytes, size_t static_bytes) {
    if (dyn_bytes + static_bytes > LDS_PER_WG) return hipErrorInvalidValue;
    if (dyn_bytes <= 64 * 1024) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_bytes);
    if (e != hipSuccess) (void)hipGetLastError();   // do not leave it for the next launch check
    return e;
}
inline unsigned grid_for(int64_t n, int block) {
    int64_t g = cdiv(n, block);
    return (unsigned)(g < 1 ? 1 : (g > (1 << 20) ? (1 << 20) : g));
}
}  // namespace

// ====================================================================== utils
__global__ void k_fill(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f(float* p, int64_t n, float v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_to_float(const double* a, float* b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) b[i] = (float)a[i];
}
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill<<<grid_for(n, 256), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_f(float* p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_f<<<grid_for(n, 256), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}
hipError_t launch_to_float(const double* src, float* dst, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_to_float<<<grid_for(n, 256), 256, 0, s>>>(src, dst, n);
    return hipGetLastError();
}

__global__ void k_gather_rows(const double* in, int64_t ldi, const int32_t* idx, int64_t n, int32_t k, double* out,
                              int64_t ldo) {
    const int64_t tot = n * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = t / k;
        int32_t c = (int32_t)(t % k);
        out[i * ldo + c] = in[(int64_t)idx[i] * ldi + c];
    }
}
__global__ void k_scatter_rows(const double* in, int64_t ldi, const int32_t* idx, int64_t n, int32_t k, double* out,
                               int64_t ldo) {
    const int64_t tot = n * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = t / k;
        int32_t c = (int32_t)(t % k);
        out[(int64_t)idx[i] * ldo + c] = in[i * ldi + c];
    }
}
__global__ void k_copy2d(const double* in, int64_t ldi, int64_t rows, int32_t k, double* out, int64_t ldo) {
    const int64_t tot = rows * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = t / k;
        int32_t c = (int32_t)(t % k);
        out[i * ldo + c] = in[i * ldi + c];
    }
}
hipError_t launch_gather_rows(const double* in, int64_t ldi, const int32_t* idx, int64_t n, int32_t k, double* out,
                              int64_t ldo, hipStream_t s) {
    if (n <= 0 || k <= 0) return hipSuccess;
    k_gather_rows<<<grid_for(n * k, 256), 256, 0, s>>>(in, ldi, idx, n, k, out, ldo);
    return hipGetLastError();
}
hipError_t launch_scatter_rows(const double* in, int64_t ldi, const int32_t* idx, int64_t n, int32_t k, double* out,
                               int64_t ldo, hipStream_t s) {
    if (n <= 0 || k <= 0) return hipSuccess;
    k_scatter_rows<<<grid_for(n * k, 256), 256, 0, s>>>(in, ldi, idx, n, k, out, ldo);
    return hipGetLastError();
}
hipError_t launch_copy2d(const double* in, int64_t ldi, int64_t rows, int32_t k, double* out, int64_t ldo,
                         hipStream_t s) {
    if (rows <= 0 || k <= 0) return hipSuccess;
    k_copy2d<<<grid_for(rows * k, 256), 256, 0, s>>>(in, ldi, rows, k, out, ldo);
    return hipGetLastError();
}

// ====================================================================== SpMM
// Y = (a A + b B) X for CSR A, B on one pattern (B optional; A may be
// rectangular): one wave per row, 64 lanes over the columns.  The edges of a
// row are fetched 8 at a time (index and weight by one lane each, broadcast by
// shuffles) and the X rows of the batch are loaded at once.  The edge count of
// a batch is the same for the whole wave; slots past it load nothing and add
// nothing, so only X rows named by the pattern are ever read (a zero weight
// times an unrelated row would still turn a non-finite value there into NaN).
// Workgroups are spread so that each XCD takes one contiguous eighth of the
// rows: neighbouring rows share their X rows in that XCD's L2.
__global__ __launch_bounds__(256) void k_spmm(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                                              const double* __restrict__ va, const double* __restrict__ vb, double a,
                                              double b, int64_t rows, const double* __restrict__ X, int64_t ldx,
                                              int32_t k, double* __restrict__ Y, int64_t ldy) {
    const int lane = threadIdx.x & 63;
    const int64_t g8 = gridDim.x;   // a multiple of 8
    const int64_t blk = (blockIdx.x % 8) * (g8 / 8) + blockIdx.x / 8;
    const int64_t row = blk * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= rows) return;
    const int64_t e0 = ptr[row], e1 = ptr[row + 1];
    for (int c0 = 0; c0 < k; c0 += 256) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t eb = e0; eb < e1; eb += 8) {
            const int cnt = (int)min<int64_t>(8, e1 - eb);   // wave-uniform
            int my_col = 0;
            double my_w = 0.0;
            if (lane < cnt) {
                my_col = idx[eb + lane];
                my_w = vb ? a * va[eb + lane] + b * vb[eb + lane] : a * va[eb + lane];
            }
            double xv[8][4];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int col = __shfl(my_col, j);
                const double* xr = X + (int64_t)col * ldx;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = c0 + lane + 64 * u;
                    xv[j][u] = j < cnt && c < k ? xr[c] : 0.0;
                }
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const double w = __shfl(my_w, j);
                if (j < cnt) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc[u] += w * xv[j][u];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + lane + 64 * u;
            if (c < k) Y[row * ldy + c] = acc[u];
        }
    }
}
hipError_t launch_spmm(const int64_t* ptr, const int32_t* idx, const double* va, const double* vb, double a, double b,
                       int64_t rows, const double* X, int64_t ldx, int32_t k, double* Y, int64_t ldy, hipStream_t s) {
    if (rows <= 0 || k <= 0) return hipSuccess;
    k_spmm<<<(unsigned)(cdiv(cdiv(rows, 4), 8) * 8), 256, 0, s>>>(ptr, idx, va, vb, a, b, rows, X, ldx, k, Y, ldy);
    return hipGetLastError();
}

__global__ void k_diag_scale(const double* d, int64_t rows, const double* X, int64_t ldx, int32_t k, double* Y,
                             int64_t ldy) {
    const int64_t tot = rows * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = t / k;
        int32_t c = (int32_t)(t % k);
        Y[i * ldy + c] = d[i] * X[i * ldx + c];
    }
}
hipError_t launch_diag_scale(const double* d, int64_t rows, const double* X, int64_t ldx, int32_t k, double* Y,
                             int64_t ldy, hipStream_t s) {
    if (rows <= 0 || k <= 0) return hipSuccess;
    k_diag_scale<<<grid_for(rows * k, 256), 256, 0, s>>>(d, rows, X, ldx, k, Y, ldy);
    return hipGetLastError();
}
__global__ void k_axpby(double a, const double* X, int64_t ldx, double b, double* Y, int64_t ldy, int64_t rows,
                        int32_t k) {
    const int64_t tot = rows * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = t / k;
        int32_t c = (int32_t)(t % k);
        Y[i * ldy + c] = a * X[i * ldx + c] + b * Y[i * ldy + c];
    }
}
hipError_t launch_axpby(double a, const double* X, int64_t ldx, double b, double* Y, int64_t ldy, int64_t rows,
                        int32_t k, hipStream_t s) {
    if (rows <= 0 || k <= 0) return hipSuccess;
    k_axpby<<<grid_for(rows * k, 256), 256, 0, s>>>(a, X, ldx, b, Y, ldy, rows, k);
    return hipGetLastError();
}

// ============================================================ factorisation
__global__ void k_assemble(double* tiles, const int64_t* dst, const int64_t* src, int64_t count, const double* Sval,
                           const double* Mval, double alpha, double beta) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = src[e];
        tiles[dst[e]] = s < 0 ? 1.0 : alpha * Sval[s] + beta * Mval[s];
    }
}
hipError_t launch_assemble(double* tiles, const int64_t* dst, const int64_t* src, int64_t count, const double* Sval,
                           const double* Mval, double alpha, double beta, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_assemble<<<grid_for(count, 256), 256, 0, s>>>(tiles, dst, src, count, Sval, Mval, alpha, beta);
    return hipGetLastError();
}

// Adds the update block (lower triangle) of child front items[blockIdx.x],
// tile column blockIdx.y, into its parent's front.  Children of one parent
// go in different launches, so no two blocks write the same entry.
__global__ __launch_bounds__(256) void k_extend_add(double* tiles, const DFront* __restrict__ fr,
                                                    const int32_t* __restrict__ items, const int32_t* __restrict__ rel) {
    const DFront C = fr[items[blockIdx.x]];
    const int32_t J = blockIdx.y;
    if (J * T32 >= C.mu) return;
    const DFront P = fr[C.parent];
    const int32_t* rl = rel + C.rows_off;
    for (int jj = 0; jj < T32; ++jj) {
        const int32_t j = J * T32 + jj;
        if (j >= C.mu) break;
        const int32_t pj = rl[j];
        const int32_t cj = C.ns_pad + j;
        for (int32_t i = j + threadIdx.x; i < C.mu; i += blockDim.x) {
            const int32_t ci = C.ns_pad + i;
            const double v = tiles[C.tile_base + tri(C.Mt, ci / T32, cj / T32) * TT + (cj % T32) * T32 + ci % T32];
            const int32_t pi = rl[i];
            tiles[P.tile_base + tri(P.Mt, pi / T32, pj / T32) * TT + (pj % T32) * T32 + pi % T32] += v;
        }
    }
}
hipError_t launch_extend_add(double* tiles, const DFront* fronts, const int32_t* items, int64_t nitems,
                             const int32_t* rel, int32_t max_tile_cols, hipStream_t s) {
    if (nitems <= 0 || max_tile_cols <= 0) return hipSuccess;
    k_extend_add<<<dim3((unsigned)nitems, (unsigned)max_tile_cols), 256, 0, s>>>(tiles, fronts, items, rel);
    return hipGetLastError();
}

// Dense LDL^T of the diagonal tile (k, k), unit lower L and D; also the
// inverse of the unit lower tile for the panel and the solves.  counters[0]
// counts negative pivots (inertia), counters[1] zero/non-finite pivots.
__global__ __launch_bounds__(256) void k_fac_diag(double* tiles, double* linv, double* D, const DFront* __restrict__ fr,
                                                  const int32_t* __restrict__ items, int32_t k, int32_t* counters) {
    // Right-looking LDL^T of the 32 x 32 diagonal tile held in registers:
    // thread (i, c0) owns the entries (i, c0 + 8 e), e < 4, of the tile and of
    // the inverse of its unit lower factor.  The inverse is accumulated
    // alongside by applying the same row eliminations to the identity
    // (L^-1 = E_31 ... E_0 with E_j = I - l_j e_j^T), so both finish after the
    // 32 pivot steps.  Step j publishes column j of the tile and row j of the
    // partial inverse through LDS (double-buffered: one barrier per step); the
    // multipliers l_ij = a_ij / d_j are formed on the fly and the columns are
    // scaled by 1 / d_j at the end.
    const DFront f = fr[items[blockIdx.x]];
    double* A = tiles + f.tile_base + tri(f.Mt, k, k) * TT;
    __shared__ double colj[2][T32], lrow[2][T32], dfin[T32];
    const int tid = threadIdx.x, i = tid & 31, c0 = tid >> 5;
    double a[4], l[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int c = c0 + 8 * e;
        a[e] = i >= c ? A[c * T32 + i] : 0.0;
        l[e] = i == c ? 1.0 : 0.0;
    }
#pragma unroll
    for (int j = 0; j < T32; ++j) {
        const int b = j & 1;
        if (c0 == (j & 7)) colj[b][i] = a[j >> 3];
        if (i == j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) lrow[b][c0 + 8 * e] = l[e];
        }
        __syncthreads();
        if (i > j) {
            const double lij = colj[b][i] / colj[b][j];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = c0 + 8 * e;
                if (c > j) {
                    if (i >= c) a[e] -= lij * colj[b][c];
                } else {
                    l[e] -= lij * lrow[b][c];
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (i == c0 + 8 * e) dfin[i] = a[e];
    __syncthreads();
    double* Li = linv + f.linv_base + (int64_t)k * TT;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int c = c0 + 8 * e;
        A[c * T32 + i] = i > c ? a[e] / dfin[c] : (i == c ? a[e] : 0.0);
        Li[c * T32 + i] = l[e];
    }
    if (tid < T32) {
        const double d = dfin[tid];
        D[f.d_base + k * T32 + tid] = d;
        const int piv = k * T32 + tid;
        if (piv < f.ns) {
            if (d < 0) atomicAdd(&counters[0], 1);
            if (!(fabs(d) > 0) || !isfinite(d)) atomicAdd(&counters[1], 1);
        }
    }
}
hipError_t launch_fac_diag(double* tiles, double* linv, double* D, const DFront* fronts, const int32_t* items,
                           int64_t nitems, int32_t k, int32_t* counters, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    k_fac_diag<<<(unsigned)nitems, 256, 0, s>>>(tiles, linv, D, fronts, items, k, counters);
    return hipGetLastError();
}

// L_Ik = A_Ik L_kk^-T D_k^-1
// The 32 x 32 tile products of the panel and update steps run on the FP64
// matrix cores: wave w of the workgroup owns the 16 x 16 block (w / 2, w % 2)
// of the result and computes its transpose (16x16x4 operands: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16], result item v of lane l is
// D[l / 16 + 4 v][l % 16]), so that every operand load and every store of
// the column-major tiles reads or writes 16 consecutive doubles.  In that
// form a wave computes Z(r, c) = sum_j Y(r, j) X(c, j), i.e. Z = Y X^T, for
// column-major tiles X (A operand), Y (B operand) and Z.
//
// Inverse panels.  For the fronts of the tree levels with wide supernodes
// (and for the dense problems) the factorisation also forms Q, the pivot
// columns of E^-1 where E = [L11 0; L21 I] is the unit lower factor of the
// front extended by the identity on its struct rows: Q = [L11^-1; -L21 L11^-1].
// A front's forward solve step is then one product, [y; u - g] = Q b', and its
// backward step another, x = Q^T [D^-1 y; x_struct] (see the solves below).
// E^-1 = E_{nsb-1}^-1 ... E_0^-1 with E_k the identity plus pivot tile column
// k of E.  Applying E_k^-1 from the left replaces tile row k of the product so
// far by Linv_k times itself and subtracts L(I, k) times the new row from every
// tile row I > k; row k has non-zero tiles in the columns j <= k only (tile
// (k, k) starts as the identity).  So the panel launch of step k also forms
// tile row k of Q (row items (front, j), j <= k: they need Linv_k) and the
// update launch the subtractions (items (front, I, j), I > k, j <= k: they need
// L(I, k) and the new row k).  Tiles are written transposed, qT tile (I, J)
// = Q(I, J)^T column-major: then both steps are the coalesced Z (+)= Y X^T.
namespace {
// tile row k of Q: Q(k, j) <- Linv_k Q(k, j) (j < k), Q(k, k) = Linv_k; in
// transposed tiles Z <- Z Linv_k^T, resp. Z = Linv_k^T
__device__ __forceinline__ void q_row_item(double* __restrict__ qT, const double* __restrict__ linv, const DFront& f,
                                           int32_t j, int32_t k) {
    double* Z = qT + f.q_base + tri(f.Mt, k, j) * TT;
    const double* Li = linv + f.linv_base + (int64_t)k * TT;
    if (j == k) {
        for (int e = threadIdx.x; e < TT; e += 256) Z[e] = Li[(e % T32) * T32 + e / T32];
        return;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int rb = 16 * (w >> 1), cb = 16 * (w & 1);
    dbl4 acc = dbl4{0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < T32; k0 += 4) {
        const int jj = k0 + lk;
        acc = mfma4(Li[jj * T32 + cb + li], Z[jj * T32 + rb + li], acc);
    }
    __syncthreads();   // every wave has read its operands before the tile is overwritten
#pragma unroll
    for (int v = 0; v < 4; ++v) Z[(cb + lk + 4 * v) * T32 + rb + li] = acc[v];
}
// Q(I, j) -= L(I, k) Q(k, j); transposed: Z_Ij -= Z_kj L(I, k)^T
__device__ __forceinline__ void q_update_item(double* __restrict__ qT, const double* __restrict__ tiles,
                                              const DFront& f, int32_t I, int32_t j, int32_t k) {
    const double* X = tiles + f.tile_base + tri(f.Mt, I, k) * TT;
    const double* Y = qT + f.q_base + tri(f.Mt, k, j) * TT;
    double* Z = qT + f.q_base + tri(f.Mt, I, j) * TT;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int rb = 16 * (w >> 1), cb = 16 * (w & 1);
    dbl4 acc = dbl4{0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < T32; k0 += 4) {
        const int jj = k0 + lk;
        acc = mfma4(X[jj * T32 + cb + li], Y[jj * T32 + rb + li], acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Z[(cb + lk + 4 * v) * T32 + rb + li] -= acc[v];
}
}  // namespace

// L_Ik = A_Ik L_kk^-T D_k^-1, in place (workgroups [0, nitems)); then the
// row items (front, j) of the inverse panels (workgroups from nitems on)
__global__ __launch_bounds__(256) void k_fac_panel(double* tiles, const double* __restrict__ linv,
                                                   const double* __restrict__ D, const DFront* __restrict__ fr,
                                                   const int32_t* __restrict__ items, int32_t nitems, int32_t k,
                                                   double* qT, const int32_t* __restrict__ qitems) {
    if ((int32_t)blockIdx.x >= nitems) {
        const int32_t q = (int32_t)blockIdx.x - nitems;
        q_row_item(qT, linv, fr[qitems[2 * q]], qitems[2 * q + 1], k);
        return;
    }
    const DFront f = fr[items[2 * blockIdx.x]];
    const int32_t I = items[2 * blockIdx.x + 1];
    double* A = tiles + f.tile_base + tri(f.Mt, I, k) * TT;
    const double* Li = linv + f.linv_base + (int64_t)k * TT;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int rb = 16 * (w >> 1), cb = 16 * (w & 1);
    // T[c][r] = sum_j Linv[c][j] A[r][j] for c in cb + [0, 16), r in rb + [0, 16)
    dbl4 acc = dbl4{0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < T32; k0 += 4) {
        const int j = k0 + lk;
        acc = mfma4(Li[j * T32 + cb + li], A[j * T32 + rb + li], acc);
    }
    __syncthreads();   // every wave has read its operands before any tile entry is overwritten
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int c = cb + lk + 4 * v;
        A[c * T32 + rb + li] = acc[v] / D[f.d_base + k * T32 + c];
    }
}
hipError_t launch_fac_panel(double* tiles, const double* linv, const double* D, const DFront* fronts,
                            const int32_t* items, int64_t nitems, int32_t k, hipStream_t s, double* qT,
                            const int32_t* qitems, int64_t nq) {
    if (!qT) nq = 0;
    if (nitems + nq <= 0) return hipSuccess;
    k_fac_panel<<<(unsigned)(nitems + nq), 256, 0, s>>>(tiles, linv, D, fronts, items, (int32_t)nitems, k, qT, qitems);
    return hipGetLastError();
}

// A_IJ -= L_Ik D_k L_Jk^T (workgroups [0, nitems)); then the update items
// (front, I, j) of the inverse panels
__global__ __launch_bounds__(256) void k_fac_update(double* tiles, const double* __restrict__ D,
                                                    const DFront* __restrict__ fr, const int32_t* __restrict__ items,
                                                    int32_t nitems, int32_t k, double* qT,
                                                    const int32_t* __restrict__ qitems) {
    if ((int32_t)blockIdx.x >= nitems) {
        const int32_t q = (int32_t)blockIdx.x - nitems;
        q_update_item(qT, tiles, fr[qitems[3 * q]], qitems[3 * q + 1], qitems[3 * q + 2], k);
        return;
    }
    const DFront f = fr[items[3 * blockIdx.x]];
    const int32_t I = items[3 * blockIdx.x + 1], J = items[3 * blockIdx.x + 2];
    const double* LI = tiles + f.tile_base + tri(f.Mt, I, k) * TT;
    const double* LJ = tiles + f.tile_base + tri(f.Mt, J, k) * TT;
    double* A = tiles + f.tile_base + tri(f.Mt, I, J) * TT;
    const double* Dk = D + f.d_base + k * T32;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int rb = 16 * (w >> 1), cb = 16 * (w & 1);
    // T[c][r] = sum_j (d_j L_J[c][j]) L_I[r][j]
    dbl4 acc = dbl4{0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < T32; k0 += 4) {
        const int j = k0 + lk;
        acc = mfma4(LJ[j * T32 + cb + li] * Dk[j], LI[j * T32 + rb + li], acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int c = cb + lk + 4 * v;
        A[c * T32 + rb + li] -= acc[v];
    }
}
hipError_t launch_fac_update(double* tiles, const double* D, const DFront* fronts, const int32_t* items,
                             int64_t nitems, int32_t k, hipStream_t s, double* qT, const int32_t* qitems, int64_t nq) {
    if (!qT) nq = 0;
    if (nitems + nq <= 0) return hipSuccess;
    k_fac_update<<<(unsigned)(nitems + nq), 256, 0, s>>>(tiles, D, fronts, items, (int32_t)nitems, k, qT, qitems);
    return hipGetLastError();
}

// ------------------------------------------------------------ wave-level solves
// One wave per (front, 16 right-hand-side columns); the waves of a
// workgroup take consecutive column chunks of one front and never
// synchronise.  The front's pivot rows of the block stay in registers as
// 16 x 16 FP64 MFMA results (tile t, element v of lane l = row
// 16 t + l / 16 + 4 v, column l % 16), which are at the same time the B
// operands of the next product.  Factor fragments are loaded straight from
// the column-major tiles (an FP32 factor is widened to FP64).  Work is done
// per 16-row tile and per 4 columns of the contraction, so the 32 x 32
// padding of small fronts costs nothing beyond those granules.
namespace {
constexpr int WCOLS = 16;   // right-hand-side columns per MFMA column tile
__device__ __forceinline__ double ldw(const double* p) { return *p; }
__device__ __forceinline__ double ldw(const float* p) { return (double)*p; }
}  // namespace

// 16 x 32 block of a 32 x 32 column-major factor tile as A fragments of the
// eight k-steps: rows 16 it .. +16 of the tile (trans = false) or of its
// transpose (trans = true).  All eight loads are issued together; every
// address lies inside the tile.
template <class TF>
__device__ __forceinline__ void frag_rows(const TF* __restrict__ tile, int it, bool trans, double (&a)[8]) {
    const int lane = threadIdx.x & 63;
    const TF* p = trans ? tile + (16 * it + (lane & 15)) * T32 + (lane >> 4)
                        : tile + (lane >> 4) * T32 + 16 * it + (lane & 15);
    const int step = trans ? 4 : 4 * T32;
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) a[ks] = ldw(p + ks * step);
}

// acc[c] (+)= +-A y_block[c] over the k-steps below kmax for the CT column
// tiles c; y_block = row tiles 2 kb, 2 kb + 1
template <int NT, int CT>
__device__ __forceinline__ void frag_mm(const double (&a)[8], const dbl4 (&y)[CT][NT], int kb, int kmax,
                                        dbl4 (&acc)[CT], bool neg) {
#pragma unroll
    for (int ks = 0; ks < 8; ++ks)
        if (4 * ks < kmax) {
            const double av = neg ? -a[ks] : a[ks];
#pragma unroll
            for (int c = 0; c < CT; ++c) acc[c] = mfma4(av, y[c][2 * kb + ks / 4][ks % 4], acc[c]);
        }
}

// workgroup -> (front, column group) of the wave-level solves: workgroups are
// dispatched round-robin over the 8 XCDs, so the column groups of one front
// are given ids 8 apart (same XCD, dispatched together) and share the
// front's factor tiles in that XCD's L2.  False for the padding workgroups.
__device__ __forceinline__ bool wsolve_item(int32_t nfronts, int32_t groups, int32_t& front, int32_t& grp) {
    const int32_t b = (int32_t)blockIdx.x, xcd = b & (NXCD - 1), slot = b / NXCD;
    grp = slot % groups;
    front = (slot / groups) * NXCD + xcd;
    return front < nfronts;
}
// the same with the update rows of a front split over `splits` workgroups
// (all of one front on one XCD)
__device__ __forceinline__ bool wsolve_item_split(int32_t nfronts, int32_t groups, int32_t splits, int32_t& front,
                                                  int32_t& grp, int32_t& split) {
    const int32_t b = (int32_t)blockIdx.x, xcd = b & (NXCD - 1), slot = b / NXCD;
    grp = slot % groups;
    const int32_t rem = slot / groups;
    split = rem % splits;
    front = (rem / splits) * NXCD + xcd;
    return front < nfronts;
}

// a forward sweep over a tree level with fewer waves than this splits the
// update rows of every front over several workgroups (each repeats the pivot
// block solve), so that narrow levels near the top of the tree fill the chip;
// only when the right-hand side is read from a separate block (in place, one
// workgroup's solution would overwrite another one's input)
constexpr int64_t WSOLVE_MIN_WAVES = 1024;
// waves per workgroup of the wave-level solves for NT pivot row tiles: one
// (the waves never synchronise, and single-wave workgroups let the dispatcher
// fill the CUs at the finest granularity; measured faster than 2, 4 or 8)
template <int NT>
struct WsolveWaves {
    static constexpr int value = 1;
};
// 16-column tiles per wave (one: many independent waves hide latency better
// than fewer, wider ones on these solves; two at the levels of up to 64
// pivots measured 6 % slower for the whole solve)
template <int NT>
struct WsolveCols {
    static constexpr int value = 1;
};

// forward sweep over one tree level: y = L11^-1 (b_J + children's updates),
// u_J = (children's updates of the struct rows) - L21 y.  A wave takes CT
// column tiles of 16.
template <class TF, int NT, int CT>
__global__ __launch_bounds__(64 * WsolveWaves<NT>::value) void k_wsolve_fwd(
    const TF* __restrict__ tiles, const TF* __restrict__ linv, const DFront* __restrict__ fr, int32_t f0, int32_t nfronts, int32_t groups, int32_t splits, double* X,
    int64_t ldx, int32_t col0, int32_t ncols, int32_t wpg, TF* ubuf, int64_t ldu, const int32_t* __restrict__ gat,
    int32_t gw, const double* __restrict__ mdiag, const double* Xin) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane >> 4;
    int32_t fi, grp, split;
    if (!wsolve_item_split(nfronts, groups, splits, fi, grp, split)) return;
    const int32_t cbase = col0 + (grp * wpg + w) * WCOLS * CT;
    const int32_t cend = col0 + ncols;
    if (cbase >= cend) return;
    const DFront f = fr[f0 + fi];
    const bool gath = (f.flags & DFRONT_GATHER) != 0;
    const int nt = (f.ns + 15) >> 4;
    dbl4 y[CT][NT];
    // right-hand side, mass scaling and (fronts with children only) the
    // gathered updates; without gathers all loads are independent
#pragma unroll
    for (int cc = 0; cc < CT; ++cc) {
        const int32_t c = cbase + 16 * cc + (lane & 15);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * t + lr + 4 * v;
                double val = 0.0;
                if (r < f.ns && c < cend) {
                    val = Xin[(f.start + r) * ldx + c];
                    if (mdiag) val *= mdiag[f.start + r];
                    if (gath) {
                        const int32_t* gr = gat + (f.gather_base + r) * gw;
#pragma unroll 2
                        for (int cg = 0; cg < gw; ++cg) {
                            const int32_t src = gr[cg];
                            if (src >= 0) val += (double)ubuf[(int64_t)src * ldu + c];
                        }
                    }
                }
                y[cc][t][v] = val;
            }
    }
#pragma unroll
    for (int kb = 0; kb < NT / 2; ++kb) {
        if (2 * kb < nt) {
            const int kmax = min(32, f.ns - 32 * kb);
            const bool two = 2 * kb + 1 < nt;
            // y_kb <- Linv_kb y_kb
            const TF* Li = linv + f.linv_base + (int64_t)kb * TT;
            double a0[8], a1[8];
            frag_rows(Li, 0, false, a0);
            if (two) frag_rows(Li, 1, false, a1);
            dbl4 n0[CT], n1[CT];
#pragma unroll
            for (int cc = 0; cc < CT; ++cc) n0[cc] = n1[cc] = dbl4{0, 0, 0, 0};
            frag_mm<NT, CT>(a0, y, kb, kmax, n0, false);
            if (two) frag_mm<NT, CT>(a1, y, kb, kmax, n1, false);
#pragma unroll
            for (int cc = 0; cc < CT; ++cc) {
                y[cc][2 * kb] = n0[cc];
                if (two) y[cc][2 * kb + 1] = n1[cc];
            }
            // y_ib -= L_ib,kb y_kb
#pragma unroll
            for (int ib = kb + 1; ib < NT / 2; ++ib)
                if (2 * ib < nt) {
                    const TF* Lt = tiles + f.tile_base + tri(f.Mt, ib, kb) * TT;
                    const bool two_i = 2 * ib + 1 < nt;
                    frag_rows(Lt, 0, false, a0);
                    if (two_i) frag_rows(Lt, 1, false, a1);
                    dbl4 t0[CT], t1[CT];
#pragma unroll
                    for (int cc = 0; cc < CT; ++cc) {
                        t0[cc] = y[cc][2 * ib];
                        t1[cc] = y[cc][2 * ib + 1];
                    }
                    frag_mm<NT, CT>(a0, y, kb, kmax, t0, true);
                    if (two_i) frag_mm<NT, CT>(a1, y, kb, kmax, t1, true);
#pragma unroll
                    for (int cc = 0; cc < CT; ++cc) {
                        y[cc][2 * ib] = t0[cc];
                        y[cc][2 * ib + 1] = t1[cc];
                    }
                }
        }
    }
#pragma unroll
    for (int cc = 0; cc < CT; ++cc) {
        const int32_t c = cbase + 16 * cc + (lane & 15);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * t + lr + 4 * v;
                if (split == 0 && r < f.ns && c < cend) X[(f.start + r) * ldx + c] = y[cc][t][v];
            }
    }
    // update rows, 16 at a time; the fragments of the next (row tile, pivot
    // block) pair are loaded while the current one is applied
    // (this workgroup's share [rt0, rt1) of the row tiles when they are split)
    const int mt = (f.mu + 15) >> 4;
    const int rt0 = split * mt / splits, rt1 = (split + 1) * mt / splits;
    if (rt0 >= rt1) return;
    const int nkb = (nt + 1) >> 1;
    double a[8];
    frag_rows(tiles + f.tile_base + tri(f.Mt, f.nsb + (rt0 >> 1), 0) * TT, rt0 & 1, false, a);
    // gather sources of the update rows: the indices of row tile rt + 1 and the
    // gathered values of row tile rt are in flight while the products of rt run
    // (every update row has at most gw sources; the first two are pipelined)
    auto gather_idx = [&](int rt, int32_t (&i0)[4], int32_t (&i1)[4]) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            i0[v] = -1;
            i1[v] = -1;
            const int sr = 16 * rt + lr + 4 * v;
            if (gath && sr < f.mu) {
                const int32_t* gr = gat + (f.gather_base + f.ns + sr) * gw;
                if (gw > 0) i0[v] = gr[0];
                if (gw > 1) i1[v] = gr[1];
            }
        }
    };
    int32_t n0[4], n1[4];
    gather_idx(rt0, n0, n1);
#pragma unroll 1
    for (int rt = rt0; rt < rt1; ++rt) {
        double g[CT][4];
#pragma unroll
        for (int cc = 0; cc < CT; ++cc) {
            const int32_t c = cbase + 16 * cc + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double u = 0.0;
                if (c < cend) {
                    if (n0[v] >= 0) u += (double)ubuf[(int64_t)n0[v] * ldu + c];
                    if (n1[v] >= 0) u += (double)ubuf[(int64_t)n1[v] * ldu + c];
                }
                g[cc][v] = u;
            }
        }
        if (rt + 1 < rt1) gather_idx(rt + 1, n0, n1);
        dbl4 acc[CT];
#pragma unroll
        for (int cc = 0; cc < CT; ++cc) acc[cc] = dbl4{0, 0, 0, 0};
#pragma unroll
        for (int kb = 0; kb < NT / 2; ++kb)
            if (kb < nkb) {
                double an[8];
                const bool last = kb + 1 == nkb;
                if (!last || rt + 1 < rt1) {
                    const int rn = last ? rt + 1 : rt, kn = last ? 0 : kb + 1;
                    frag_rows(tiles + f.tile_base + tri(f.Mt, f.nsb + (rn >> 1), kn) * TT, rn & 1, false, an);
                }
                frag_mm<NT, CT>(a, y, kb, min(32, f.ns - 32 * kb), acc, false);
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) a[ks] = an[ks];
            }
#pragma unroll
        for (int cc = 0; cc < CT; ++cc) {
            const int32_t c = cbase + 16 * cc + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int sr = 16 * rt + lr + 4 * v;
                if (sr < f.mu && c < cend) {
                    double u = g[cc][v];
                    if (gath) {
                        const int32_t* gr = gat + (f.gather_base + f.ns + sr) * gw;
#pragma unroll 1
                        for (int cg = 2; cg < gw; ++cg) {
                            const int32_t src = gr[cg];
                            if (src >= 0) u += (double)ubuf[(int64_t)src * ldu + c];
                        }
                    }
                    ubuf[(f.ubuf_row + sr) * ldu + c] = (TF)(u - acc[cc][v]);
                }
            }
        }
    }
}

// backward sweep over one tree level: z = D^-1 y - L21^T x_struct, then
// x_J = L11^-T z (last pivot block first); tilesT, linvT are the factor
// tiles transposed one by one, so that L^T fragments load like L fragments
template <class TF, int NT, int CT>
__global__ __launch_bounds__(64 * WsolveWaves<NT>::value) void k_wsolve_bwd(
    const TF* __restrict__ tilesT, const TF* __restrict__ linvT, const TF* __restrict__ D,
    const DFront* __restrict__ fr, int32_t f0, int32_t nfronts, int32_t groups, double* X, int64_t ldx, int32_t col0, int32_t ncols, int32_t wpg,
    const int32_t* __restrict__ rows, int apply_dinv) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane >> 4;
    int32_t fi, grp;
    if (!wsolve_item(nfronts, groups, fi, grp)) return;
    const int32_t cbase = col0 + (grp * wpg + w) * WCOLS * CT;
    const int32_t cend = col0 + ncols;
    if (cbase >= cend) return;
    const DFront f = fr[f0 + fi];
    const int nt = (f.ns + 15) >> 4;
    const int32_t* frows = rows + f.rows_off;
    const int mt = (f.mu + 15) >> 4;
    // struct rows of the first 16-row tile, ahead of everything else
    int32_t rix[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) rix[ks] = frows[min(4 * ks + lr, max(f.mu - 1, 0))];
    dbl4 z[CT][NT];
#pragma unroll
    for (int cc = 0; cc < CT; ++cc) {
        const int32_t c = cbase + 16 * cc + (lane & 15);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * t + lr + 4 * v;
                double val = 0.0;
                if (r < f.ns && c < cend) {
                    val = X[(f.start + r) * ldx + c];
                    if (apply_dinv) val /= (double)D[f.d_base + r];
                }
                z[cc][t][v] = val;
            }
    }
    // z -= L21^T x_struct, 16 struct rows at a time; the next tile's solution
    // values and the row indices after it are loaded one step ahead
    double xs[CT][4];
#pragma unroll
    for (int cc = 0; cc < CT; ++cc) {
        const int32_t c = cbase + 16 * cc + (lane & 15);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            xs[cc][ks] = (4 * ks + lr < f.mu && c < cend) ? X[(int64_t)rix[ks] * ldx + c] : 0.0;
    }
    if (mt > 1) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) rix[ks] = frows[min(16 + 4 * ks + lr, f.mu - 1)];
    }
#pragma unroll 1
    for (int rt = 0; rt < mt; ++rt) {
        const int st = rt >> 1, half = rt & 1;
        double xn[CT][4];
        if (rt + 1 < mt) {
#pragma unroll
            for (int cc = 0; cc < CT; ++cc) {
                const int32_t c = cbase + 16 * cc + (lane & 15);
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int sr = 16 * (rt + 1) + 4 * ks + lr;
                    xn[cc][ks] = (sr < f.mu && c < cend) ? X[(int64_t)rix[ks] * ldx + c] : 0.0;
                }
            }
            if (rt + 2 < mt) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) rix[ks] = frows[min(16 * (rt + 2) + 4 * ks + lr, f.mu - 1)];
            }
        }
#pragma unroll
        for (int jb = 0; jb < NT / 2; ++jb)
            if (2 * jb < nt) {
                const bool two = 2 * jb + 1 < nt;
                // A(i, k) = L(k, i) = element (i, k) of the transposed tile (nsb + st, jb)
                const TF* Lt = tilesT + f.tile_base + tri(f.Mt, f.nsb + st, jb) * TT + (16 * half + lr) * T32 + (lane & 15);
                double a0[4], a1[4];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    a0[ks] = ldw(Lt + 4 * ks * T32);
                    a1[ks] = two ? ldw(Lt + 4 * ks * T32 + 16) : 0.0;
                }
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int cc = 0; cc < CT; ++cc) {
                        z[cc][2 * jb] = mfma4(-a0[ks], xs[cc][ks], z[cc][2 * jb]);
                        if (two) z[cc][2 * jb + 1] = mfma4(-a1[ks], xs[cc][ks], z[cc][2 * jb + 1]);
                    }
            }
        if (rt + 1 < mt) {
#pragma unroll
            for (int cc = 0; cc < CT; ++cc)
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) xs[cc][ks] = xn[cc][ks];
        }
    }
#pragma unroll
    for (int kb = NT / 2 - 1; kb >= 0; --kb) {
        if (2 * kb < nt) {
            const int kmax = min(32, f.ns - 32 * kb);
            const bool two = 2 * kb + 1 < nt;
            // x_kb = Linv_kb^T z_kb
            const TF* Li = linvT + f.linv_base + (int64_t)kb * TT;
            double a0[8], a1[8];
            frag_rows(Li, 0, false, a0);
            if (two) frag_rows(Li, 1, false, a1);
            dbl4 n0[CT], n1[CT];
#pragma unroll
            for (int cc = 0; cc < CT; ++cc) n0[cc] = n1[cc] = dbl4{0, 0, 0, 0};
            frag_mm<NT, CT>(a0, z, kb, kmax, n0, false);
            if (two) frag_mm<NT, CT>(a1, z, kb, kmax, n1, false);
#pragma unroll
            for (int cc = 0; cc < CT; ++cc) {
                z[cc][2 * kb] = n0[cc];
                if (two) z[cc][2 * kb + 1] = n1[cc];
            }
            // z_ib -= L_kb,ib^T x_kb
#pragma unroll
            for (int ib = 0; ib < kb; ++ib) {
                const TF* Lt = tilesT + f.tile_base + tri(f.Mt, kb, ib) * TT;
                frag_rows(Lt, 0, false, a0);
                frag_rows(Lt, 1, false, a1);
                dbl4 t0[CT], t1[CT];
#pragma unroll
                for (int cc = 0; cc < CT; ++cc) {
                    t0[cc] = z[cc][2 * ib];
                    t1[cc] = z[cc][2 * ib + 1];
                }
                frag_mm<NT, CT>(a0, z, kb, kmax, t0, true);
                frag_mm<NT, CT>(a1, z, kb, kmax, t1, true);
#pragma unroll
                for (int cc = 0; cc < CT; ++cc) {
                    z[cc][2 * ib] = t0[cc];
                    z[cc][2 * ib + 1] = t1[cc];
                }
            }
        }
    }
#pragma unroll
    for (int cc = 0; cc < CT; ++cc) {
        const int32_t c = cbase + 16 * cc + (lane & 15);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * t + lr + 4 * v;
                if (r < f.ns && c < cend) X[(f.start + r) * ldx + c] = z[cc][t][v];
            }
    }
}

// every 32 x 32 tile of `in` transposed into the same place of `out`
template <class T>
__global__ __launch_bounds__(256) void k_tile_transpose(const T* __restrict__ in, T* __restrict__ out, int64_t ntiles) {
    __shared__ T sm[T32][T32 + 1];
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const T* a = in + t * TT;
        T* b = out + t * TT;
        for (int idx = threadIdx.x; idx < TT; idx += 256) sm[idx / T32][idx % T32] = a[idx];   // sm[col][row]
        __syncthreads();
        for (int idx = threadIdx.x; idx < TT; idx += 256) b[idx] = sm[idx % T32][idx / T32];
        __syncthreads();
    }
}
template <class T>
hipError_t launch_tile_transpose(const T* in, T* out, int64_t ntiles, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    k_tile_transpose<T><<<(unsigned)std::min<int64_t>(ntiles, 16384), 256, 0, s>>>(in, out, ntiles);
    return hipGetLastError();
}
template hipError_t launch_tile_transpose<double>(const double*, double*, int64_t, hipStream_t);
template hipError_t launch_tile_transpose<float>(const float*, float*, int64_t, hipStream_t);

// largest pivot count of a front the wave-level solves take
int32_t wsolve_max_ns() { return 256; }

namespace {
inline void wsolve_shape(int32_t ncols, int32_t max_waves, int32_t cols_per_wave, int32_t& wpg, int32_t& groups) {
    const int32_t nck = (int32_t)cdiv(ncols, cols_per_wave);
    groups = (int32_t)cdiv(nck, max_waves);
    wpg = (int32_t)cdiv(nck, groups);
}
}  // namespace

template <class TF>
hipError_t launch_wsolve(bool fwd, const TF* tiles, const TF* linv, const TF* D, const DFront* fronts, int32_t f0,
                         int32_t f1, int32_t ns_pad_max, double* X, int64_t ldx, int32_t col0, int32_t ncols,
                         double* ubuf, int64_t ldu, const int32_t* gat, int32_t gw, const double* mdiag,
                         const int32_t* rows, bool apply_dinv, hipStream_t s, const double* Xin) {
    if (f1 <= f0 || ncols <= 0) return hipSuccess;
    if (!Xin) Xin = X;
    if (ns_pad_max > wsolve_max_ns()) return hipErrorInvalidValue;
    int32_t wpg, groups;
    TF* ub = reinterpret_cast<TF*>(ubuf);
#define HSIM_WS(NT, CT)                                                                                          \
    wsolve_shape(ncols, WsolveWaves<NT>::value, WCOLS * CT, wpg, groups);                                         \
    const int64_t waves = (int64_t)(f1 - f0) * groups * wpg;                                                      \
    const int32_t splits = fwd && Xin != X                                                                      \
                               ? (int32_t)std::min<int64_t>(8, std::max<int64_t>(1, WSOLVE_MIN_WAVES / waves))   \
                               : 1;                                                                              \
    const dim3 grid((unsigned)(cdiv(f1 - f0, NXCD) * NXCD * groups * splits)), block((unsigned)(64 * wpg));     \
    if (fwd)                                                                                                      \
        k_wsolve_fwd<TF, NT, CT><<<grid, block, 0, s>>>(tiles, linv, fronts, f0, f1 - f0, groups, splits, X, ldx, \
                                                        col0, ncols, wpg, ub, ldu, gat, gw, mdiag, Xin);          \
    else                                                                                                          \
        k_wsolve_bwd<TF, NT, CT><<<grid, block, 0, s>>>(tiles, linv, D, fronts, f0, f1 - f0, groups, X, ldx,     \
                                                        col0, ncols, wpg, rows, apply_dinv ? 1 : 0);
    if (ns_pad_max <= 32) { HSIM_WS(2, WsolveCols<2>::value) }
    else if (ns_pad_max <= 64) { HSIM_WS(4, WsolveCols<4>::value) }
    else if (ns_pad_max <= 128) { HSIM_WS(8, WsolveCols<8>::value) }
    else { HSIM_WS(16, WsolveCols<16>::value) }
#undef HSIM_WS
    return hipGetLastError();
}
template hipError_t launch_wsolve<double>(bool, const double*, const double*, const double*, const DFront*, int32_t,
                                          int32_t, int32_t, double*, int64_t, int32_t, int32_t, double*, int64_t,
                                          const int32_t*, int32_t, const double*, const int32_t*, bool, hipStream_t,
                                          const double*);
template hipError_t launch_wsolve<float>(bool, const float*, const float*, const float*, const DFront*, int32_t,
                                         int32_t, int32_t, double*, int64_t, int32_t, int32_t, double*, int64_t,
                                         const int32_t*, int32_t, const double*, const int32_t*, bool, hipStream_t,
                                         const double*);

// ---------------------------------------------------------------------------
// Block solves through the inverse panels Q = [L11^-1; -L21 L11^-1] of the
// factorisation.  Per tree level and direction two launches:
//   forward:  gather  R(pivots) = mdiag b + children's updates (and, unless
//                     the product does it, update rows = children's updates
//                     g of the struct rows);
//             product y = Q_piv R -> X, update rows = g + Q_struct R
//                     (u = g - L21 L11^-1 b' = g + Q_struct b');
//   backward: gather  R = [D^-1 y; x at the struct rows];
//             product x = Q^T R -> X (= L11^-T (D^-1 y - L21^T x_struct)).
// R is a scratch block whose rows follow each front's local index space
// (pivot r at qrow + r, struct row s at qrow + ns_pad + s; padding rows are
// written as zeros).  The products run on the FP64 matrix cores, a workgroup
// per (32-row output tile, 32 columns) whose waves split the contraction, the
// Q fragments straight from the tiles (forward: the column-major tiles;
// backward: the transposed ones, so both load 16 consecutive values per lane
// group), the next tile's operands loaded while the current one is applied.
// Nothing depends on anything else within a launch, so a wide front is not a
// chain of launches.

// items: (front, 32-row tile of [0, nsb + struct tiles)); 64 columns per blockIdx.y
template <class TF>
__global__ __launch_bounds__(256) void k_qsolve_gather(int fwd, const DFront* __restrict__ fr,
                                                       const int32_t* __restrict__ items, double* R, int64_t ldr,
                                                       const double* Xin, double* X, int64_t ldx, int32_t col0,
                                                       int32_t ncols, TF* ubuf, int64_t ldu,
                                                       const int32_t* __restrict__ gat, int32_t gw,
                                                       const double* __restrict__ mdiag, const TF* __restrict__ D,
                                                       const int32_t* __restrict__ rows, int pivots_only) {
    const DFront f = fr[items[2 * blockIdx.x]];
    const int tr = items[2 * blockIdx.x + 1];
    const int32_t c = col0 + 64 * blockIdx.y + (threadIdx.x & 63);
    if (c >= col0 + ncols) return;
    const bool piv = tr < f.nsb;
    if (!piv && pivots_only) return;   // the forward product gathers the struct rows itself
    for (int i = threadIdx.x >> 6; i < T32; i += 4) {
        if (piv) {
            const int p = tr * T32 + i;
            double v = 0.0;
            if (p < f.ns) {
                if (fwd) {
                    v = Xin[(f.start + p) * ldx + c];
                    if (mdiag) v *= mdiag[f.start + p];
                    if (f.flags & DFRONT_GATHER) {
                        const int32_t* gr = gat + (f.gather_base + p) * gw;
                        for (int cg = 0; cg < gw; ++cg)
                            if (gr[cg] >= 0) v += (double)ubuf[(int64_t)gr[cg] * ldu + c];
                    }
                } else {
                    v = X[(f.start + p) * ldx + c] / (double)D[f.d_base + p];
                }
            }
            R[(f.qrow + p) * ldr + c] = v;
        } else {
            const int sr = (tr - f.nsb) * T32 + i;
            if (fwd) {
                if (sr >= f.mu) continue;
                double v = 0.0;
                if (f.flags & DFRONT_GATHER) {
                    const int32_t* gr = gat + (f.gather_base + f.ns + sr) * gw;
                    for (int cg = 0; cg < gw; ++cg)
                        if (gr[cg] >= 0) v += (double)ubuf[(int64_t)gr[cg] * ldu + c];
                }
                ubuf[(f.ubuf_row + sr) * ldu + c] = (TF)v;
            } else {
                const double v = sr < f.mu ? X[(int64_t)rows[f.rows_off + sr] * ldx + c] : 0.0;
                R[(f.qrow + f.ns_pad + sr) * ldr + c] = v;
            }
        }
    }
}

// 32 rows of the CT column tiles c + 16 ct of R starting at row r0 of the
// front's index space, as the B operands of the eight k-steps of one tile
// (rows at or past kmax, and column tiles past the block: 0)
template <int CT>
__device__ __forceinline__ void q_rhs(const double* __restrict__ R, int64_t ldr, int64_t r0, int kmax, int32_t c,
                                      int ctn, double (&b)[CT][8]) {
    const int lr = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
        const int r = 4 * ks + lr;
        const double* p = R + (r0 + r) * ldr + c;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) b[ct][ks] = (r < kmax && ct < ctn) ? p[16 * ct] : 0.0;
    }
}

// acc[h][ct] += Q fragment rows (half h) times the B operands of column tile
// ct over the contraction rows [4 ks0_h, kmax_h) (whole k-steps); column
// tiles at or past ctn (wave-uniform) are skipped
template <int CT>
__device__ __forceinline__ void q_mm(const double (&a)[2][8], const double (&b)[CT][8], int kmax0, int kmax1,
                                     int ks0h1, int ctn, dbl4 (&acc)[2][CT]) {
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            if (ct >= ctn) continue;
            if (4 * ks < kmax0) acc[0][ct] = mfma4(a[0][ks], b[ct][ks], acc[0][ct]);
            if (4 * ks < kmax1 && ks >= ks0h1) acc[1][ct] = mfma4(a[1][ks], b[ct][ks], acc[1][ct]);
        }
    }
}

// the partial sums of the nw waves of a workgroup added in wave order (wave 0
// returns true and holds the sum), two column tiles at a time; red: nw x 4 x
// 64 dbl4 of dynamic LDS
template <int CT>
__device__ __forceinline__ bool q_reduce(dbl4 (&acc)[2][CT], int nw, dbl4* red) {
    if (nw == 1) return true;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int c0 = 0; c0 < CT; c0 += 2) {
        if (c0 > 0) __syncthreads();   // wave 0 has read the previous pair
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) red[(w * 4 + 2 * h + ct) * 64 + lane] = acc[h][c0 + ct];
        __syncthreads();
        if (w == 0) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) {
                    dbl4 sum = red[(2 * h + ct) * 64 + lane];
                    for (int k = 1; k < nw; ++k) sum += red[(k * 4 + 2 * h + ct) * 64 + lane];
                    acc[h][c0 + ct] = sum;
                }
        }
    }
    return w == 0;
}

// Both products: a workgroup of nw waves per (item, 16 CT columns); the item
// is a 32-row output tile of one front, the wave owns its two 16-row halves
// times CT 16-column tiles, the nw waves take every nw-th tile of the
// contraction and add their sums in wave order.  The next tile's operands are
// loaded while the current one is applied.
// Forward, items (front, I), I < Mt: rows of tile I of Q R (J <= min(I, nsb - 1)).
template <class TF, int CT>
__global__ __launch_bounds__(512) void k_qsolve_fwd(const TF* __restrict__ qinv, const DFront* __restrict__ fr,
                                                    const int32_t* __restrict__ items, int32_t nitems, int32_t groups,
                                                    int32_t nw, const double* __restrict__ R, int64_t ldr, double* X,
                                                    int64_t ldx, int32_t col0, int32_t ncols, TF* ubuf, int64_t ldu,
                                                    const int32_t* __restrict__ gat, int32_t gw) {
    extern __shared__ dbl4 qred[];
    int32_t it, grp;
    if (!wsolve_item(nitems, groups, it, grp)) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane >> 4;
    const int32_t cw = col0 + 16 * CT * grp;   // first column of the wave's block
    const int32_t c = cw + (lane & 15);
    const int ctn = min(CT, (int)((col0 + ncols - cw + 15) >> 4));   // column tiles that hold columns
    const int32_t cend = col0 + ncols;
    const DFront f = fr[items[2 * it]];
    const int I = items[2 * it + 1];
    const int J1 = min(I, f.nsb - 1);
    const TF* Q = qinv + f.q_base;
    // gat given: the children's updates g of this tile's struct rows are
    // gathered here (wave 0, loaded before the products) instead of by the
    // gather launch, and the update rows are written once as g + Q_struct b'
    const bool own_g = gat != nullptr && I >= f.nsb;
    double g[2][CT][4];
    if (own_g && w == 0) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int sr = (I - f.nsb) * T32 + 16 * h + lr + 4 * v;
                const int32_t* gr = gat + (f.gather_base + f.ns + sr) * gw;
                const bool live = sr < f.mu && (f.flags & DFRONT_GATHER);
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) g[h][ct][v] = 0.0;
                if (!live) continue;
                for (int cg = 0; cg < gw; ++cg) {
                    const int32_t src = gr[cg];
                    if (src < 0) continue;
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct)
                        if (ct < ctn && c + 16 * ct < cend) g[h][ct][v] += (double)ubuf[(int64_t)src * ldu + c + 16 * ct];
                }
            }
    }
    dbl4 acc[2][CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[0][ct] = acc[1][ct] = dbl4{0, 0, 0, 0};
    double a[2][8], b[CT][8];
    int J = w;
    if (J <= J1) {
        frag_rows(Q + tri(f.Mt, I, J) * TT, 0, false, a[0]);
        frag_rows(Q + tri(f.Mt, I, J) * TT, 1, false, a[1]);
        q_rhs<CT>(R, ldr, f.qrow + T32 * J, min(T32, f.ns - T32 * J), c, ctn, b);
    }
#pragma unroll 1
    for (; J <= J1; J += nw) {
        double an[2][8], bn[CT][8];
        const int Jn = J + nw;
        if (Jn <= J1) {
            frag_rows(Q + tri(f.Mt, I, Jn) * TT, 0, false, an[0]);
            frag_rows(Q + tri(f.Mt, I, Jn) * TT, 1, false, an[1]);
            q_rhs<CT>(R, ldr, f.qrow + T32 * Jn, min(T32, f.ns - T32 * Jn), c, ctn, bn);
        }
        // the diagonal tile of Q is lower triangular: rows 0..15 end at column 15
        const int km = min(T32, f.ns - T32 * J);
        q_mm<CT>(a, b, J == I ? min(km, 16) : km, km, 0, ctn, acc);
        if (Jn <= J1) {
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                a[0][ks] = an[0][ks];
                a[1][ks] = an[1][ks];
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) b[ct][ks] = bn[ct][ks];
            }
        }
    }
    if (!q_reduce<CT>(acc, nw, qred)) return;
    const bool piv = I < f.nsb;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int32_t cc = c + 16 * ct;
            if (ct >= ctn || cc >= cend) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * h + lr + 4 * v;
                if (piv) {
                    const int p = I * T32 + r;
                    if (p < f.ns) X[(f.start + p) * ldx + cc] = acc[h][ct][v];
                } else {
                    const int sr = (I - f.nsb) * T32 + r;
                    if (sr < f.mu) {
                        TF* u = ubuf + (f.ubuf_row + sr) * ldu + cc;
                        *u = own_g ? (TF)(g[h][ct][v] + acc[h][ct][v]) : (TF)((double)*u + acc[h][ct][v]);
                    }
                }
            }
        }
}

// Backward, items (front, C), C < nsb: pivot rows of tile C of Q^T R, the sum
// over tile rows I >= C of Q(I, C)^T R(I)
template <class TF, int CT>
__global__ __launch_bounds__(512) void k_qsolve_bwd(const TF* __restrict__ qinvT, const DFront* __restrict__ fr,
                                                    const int32_t* __restrict__ items, int32_t nitems, int32_t groups,
                                                    int32_t nw, const double* __restrict__ R, int64_t ldr, double* X,
                                                    int64_t ldx, int32_t col0, int32_t ncols) {
    extern __shared__ dbl4 qred[];
    int32_t it, grp;
    if (!wsolve_item(nitems, groups, it, grp)) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane >> 4;
    const int32_t cw = col0 + 16 * CT * grp;
    const int32_t c = cw + (lane & 15);
    const int ctn = min(CT, (int)((col0 + ncols - cw + 15) >> 4));
    const int32_t cend = col0 + ncols;
    const DFront f = fr[items[2 * it]];
    const int C = items[2 * it + 1];
    const TF* Q = qinvT + f.q_base;
    auto rows_of = [&](int I) { return I < f.nsb ? min(T32, f.ns - T32 * I) : min(T32, f.mu - T32 * (I - f.nsb)); };
    dbl4 acc[2][CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[0][ct] = acc[1][ct] = dbl4{0, 0, 0, 0};
    double a[2][8], b[CT][8];
    int I = C + w;
    if (I < f.Mt) {
        frag_rows(Q + tri(f.Mt, I, C) * TT, 0, false, a[0]);
        frag_rows(Q + tri(f.Mt, I, C) * TT, 1, false, a[1]);
        q_rhs<CT>(R, ldr, f.qrow + T32 * I, rows_of(I), c, ctn, b);
    }
#pragma unroll 1
    for (; I < f.Mt; I += nw) {
        double an[2][8], bn[CT][8];
        const int In = I + nw;
        if (In < f.Mt) {
            frag_rows(Q + tri(f.Mt, In, C) * TT, 0, false, an[0]);
            frag_rows(Q + tri(f.Mt, In, C) * TT, 1, false, an[1]);
            q_rhs<CT>(R, ldr, f.qrow + T32 * In, rows_of(In), c, ctn, bn);
        }
        // Q(C, C) is lower triangular: columns 16..31 start at row 16
        const int km = rows_of(I);
        q_mm<CT>(a, b, km, km, I == C ? 4 : 0, ctn, acc);
        if (In < f.Mt) {
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                a[0][ks] = an[0][ks];
                a[1][ks] = an[1][ks];
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) b[ct][ks] = bn[ct][ks];
            }
        }
    }
    if (!q_reduce<CT>(acc, nw, qred)) return;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int32_t cc = c + 16 * ct;
            if (ct >= ctn || cc >= cend) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int p = C * T32 + 16 * h + lr + 4 * v;
                if (p < f.ns) X[(f.start + p) * ldx + cc] = acc[h][ct][v];
            }
        }
}

template <class TF>
hipError_t launch_qsolve(int phase, const TF* qinv, const TF* qinvT, const TF* D, const DFront* fronts,
                         const int32_t* items, int64_t nitems, double* R, int64_t ldr, double* X, int64_t ldx,
                         int32_t col0, int32_t ncols, double* ubuf, int64_t ldu, const int32_t* gat, int32_t gw,
                         const double* mdiag, const int32_t* rows, hipStream_t s, const double* Xin, int32_t kmax,
                         bool fuse) {
    if (nitems <= 0 || ncols <= 0) return hipSuccess;
    TF* ub = reinterpret_cast<TF*>(ubuf);
    if (phase == 0 || phase == 2) {
        const dim3 grid((unsigned)nitems, (unsigned)cdiv(ncols, 64));
        k_qsolve_gather<TF><<<grid, 256, 0, s>>>(phase == 0 ? 1 : 0, fronts, items, R, ldr, Xin ? Xin : X, X, ldx,
                                                 col0, ncols, ub, ldu, gat, gw, mdiag, D, rows,
                                                 phase == 0 && fuse ? 1 : 0);
        return hipGetLastError();
    }
    // waves per workgroup: every wave takes about eight tiles of the longest contraction
    const int32_t nw = kmax > 32 ? 8 : kmax > 16 ? 4 : kmax > 8 ? 2 : 1;
    const size_t lds = nw > 1 ? (size_t)nw * 4 * 64 * sizeof(double) * 4 : 0;
    // two 16-column tiles per wave (four: one wave per SIMD for registers, measured slower)
    constexpr int CT = 2;
    const int32_t groups = (int32_t)cdiv(ncols, 16 * CT);
    const unsigned grid = (unsigned)(cdiv(nitems, NXCD) * NXCD * groups);
    if (phase == 1)
        k_qsolve_fwd<TF, CT><<<grid, 64 * nw, lds, s>>>(qinv, fronts, items, (int32_t)nitems, groups, nw, R, ldr, X,
                                                       ldx, col0, ncols, ub, ldu, fuse ? gat : nullptr, gw);
    else if (phase == 3)
        k_qsolve_bwd<TF, CT><<<grid, 64 * nw, lds, s>>>(qinvT, fronts, items, (int32_t)nitems, groups, nw, R, ldr, X,
                                                       ldx, col0, ncols);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}
template hipError_t launch_qsolve<double>(int, const double*, const double*, const double*, const DFront*,
                                          const int32_t*, int64_t, double*, int64_t, double*, int64_t, int32_t, int32_t,
                                          double*, int64_t, const int32_t*, int32_t, const double*, const int32_t*,
                                          hipStream_t, const double*, int32_t, bool);
template hipError_t launch_qsolve<float>(int, const float*, const float*, const float*, const DFront*, const int32_t*,
                                         int64_t, double*, int64_t, double*, int64_t, int32_t, int32_t, double*,
                                         int64_t, const int32_t*, int32_t, const double*, const int32_t*, hipStream_t,
                                         const double*, int32_t, bool);

// ============================================================ Gram products
// Sbar = Psi^T (S Psi), Mbar = Psi^T (M Psi) on the matrix cores.  The q x q
// upper triangle is covered by 64 x 64 block pairs (a <= b); a workgroup takes
// one block pair and one chunk of rows (gram_chunk_rows), its four waves one 32 x 32 quarter each
// (2 x 2 tiles of the 16 x 16 x 4 MFMA, both products).  Rows are staged
// through LDS 32 at a time, the next 32 prefetched into registers.
// TA = double: FP64 MFMA.  TA = float: operands rounded to FP32, FP32 MFMA
// accumulation over runs of 256 rows, FP64 sum of the runs and the chunks.
// Block ids are spread so that the block pairs of one row chunk run on one
// XCD (dispatch is round-robin over the 8 XCDs) and share its L2.
namespace {
constexpr int GT = 64;            // output block edge
constexpr int GROWS = 32;         // rows per LDS stage
constexpr int GLD = GT + 8;       // LDS row stride (elements)


// workgroup id -> (chunk, pair) with the pairs of a chunk on one XCD
__device__ __forceinline__ bool xcd_item(int64_t total, int64_t& item) {
    const int64_t g8 = (total + NXCD - 1) / NXCD * NXCD;
    const int64_t b = blockIdx.x;
    item = (b % NXCD) * (g8 / NXCD) + b / NXCD;
    return item < total;
}
}  // namespace

int64_t colsum_tmp_doubles(int64_t nrows, int32_t ncols);
hipError_t launch_colsum(const double* in, int64_t nrows, int32_t ncols, double* tmp, double* out, hipStream_t s);

static int64_t gram_pairs(int32_t q) {
    const int64_t nt = cdiv(q, GT);
    return nt * (nt + 1) / 2;
}

// rows per workgroup of the multi-pass Gram for up to n rows: short chunks
// (more workgroups per block pair) as long as the per-chunk partial blocks
// stay within 2^32 doubles
int64_t gram_chunk_rows(int64_t n, int32_t q) {
    const int64_t per = gram_pairs(q) * 2 * GT * GT;
    int64_t c = 1024;
    while (c < (int64_t(1) << 24) && cdiv(n, c) * per > (int64_t(1) << 32)) c *= 2;
    return c;
}

// per-chunk partial blocks, their sum and the reduction's scratch
int64_t gram_all_partial_doubles(int32_t q);
int64_t gram_partial_doubles(int64_t n, int32_t q, int64_t chunk_rows) {
    const int64_t nch = cdiv(n, chunk_rows);
    const int64_t per = gram_pairs(q) * 2 * GT * GT;
    return std::max(nch * per + per + colsum_tmp_doubles(nch, (int32_t)per), gram_all_partial_doubles(q));
}

// MODE 0: FP64 operands and MFMA.  MODE 1: operands rounded to FP32, FP32
// MFMA accumulation over runs of 256 rows, FP64 sum of the runs.  MODE 2
// (compensated): every FP64 operand split into hi = fl32(x) and lo =
// fl32(x - hi) (together 48 significant bits), three FP32 products per pair
// (hi*hi, hi*lo, lo*hi; lo*lo is below the FP64 rounding of the result),
// the hi*hi run and the cross-term run summed in FP32 over one 32-row stage
// each and added in FP64.
template <int MODE>
__global__ __launch_bounds__(256) void k_gram_mfma(const double* __restrict__ Psi, const double* __restrict__ SPsi,
                                                   const double* __restrict__ MPsi, const double* __restrict__ mdiag,
                                                   int64_t n, int32_t q, int64_t ld, int64_t nchunks,
                                                   int64_t chunk_rows, double* __restrict__ partial) {
    using TA = typename std::conditional<MODE == 0, double, float>::type;
    using V4 = typename std::conditional<MODE == 0, dbl4, flt4>::type;
    constexpr bool COMP = MODE == 2;
    constexpr int LOW = COMP ? GROWS : 1;          // rows of the lo arrays (1: unused)
    const int32_t nt = (q + GT - 1) / GT;
    const int64_t npairs = (int64_t)nt * (nt + 1) / 2;
    int64_t item;
    if (!xcd_item(nchunks * npairs, item)) return;
    const int64_t chunk = item / npairs;
    int32_t pair = (int32_t)(item % npairs), a = 0;
    while (pair >= nt - a) { pair -= nt - a; ++a; }
    const int32_t b = a + pair;
    const int64_t r0 = chunk * chunk_rows;
    const int64_t r1 = min(n, r0 + chunk_rows);

    __shared__ TA P[GROWS][GLD], Q[GROWS][GLD], R[GROWS][GLD];
    __shared__ TA Pl[LOW][GLD], Ql[LOW][GLD], Rl[LOW][GLD];
    const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
    const int wi = w / 2, wj = w % 2;              // quarter of the 64 x 64 block pair
    const bool active = !(a == b && wi > wj);      // strictly lower quarter of a diagonal block
    bool tile_on[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
            tile_on[t][u] = active && a * GT + wi * 32 + t * 16 < q && b * GT + wj * 32 + u * 16 < q;

    dbl4 accS[2][2], accM[2][2];
    V4 runS[2][2], runM[2][2], corS[2][2], corM[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            accS[t][u] = accM[t][u] = dbl4{0, 0, 0, 0};
            runS[t][u] = runM[t][u] = corS[t][u] = corM[t][u] = V4{0, 0, 0, 0};
        }

    // staging: thread -> 8 elements of each array (rows tid / 8 + 32 j / 8 ...)
    constexpr int PER = GROWS * GT / 256;   // 8
    double pv[PER], qv[PER], rv[PER];
    auto fetch = [&](int64_t row0) {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + 256 * e, i = idx / GT, c = idx % GT;
            const int64_t row = row0 + i;
            const int ca = a * GT + c, cb = b * GT + c;
            const bool ok = row < r1;
            pv[e] = (ok && ca < q) ? Psi[row * ld + ca] : 0.0;
            qv[e] = (ok && cb < q) ? SPsi[row * ld + cb] : 0.0;
            rv[e] = (ok && cb < q) ? (mdiag ? mdiag[row] * Psi[row * ld + cb] : MPsi[row * ld + cb]) : 0.0;
        }
    };
    auto fold = [&] {
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    accS[t][u][v] += (double)runS[t][u][v] + (double)corS[t][u][v];
                    accM[t][u][v] += (double)runM[t][u][v] + (double)corM[t][u][v];
                    runS[t][u][v] = runM[t][u][v] = corS[t][u][v] = corM[t][u][v] = 0;
                }
    };
    fetch(r0);
    int steps = 0;
    for (int64_t row0 = r0; row0 < r1; row0 += GROWS) {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + 256 * e, i = idx / GT, c = idx % GT;
            const TA ph = (TA)pv[e], qh = (TA)qv[e], rh = (TA)rv[e];
            P[i][c] = ph;
            Q[i][c] = qh;
            R[i][c] = rh;
            if (COMP) {
                Pl[i][c] = (TA)(pv[e] - (double)ph);
                Ql[i][c] = (TA)(qv[e] - (double)qh);
                Rl[i][c] = (TA)(rv[e] - (double)rh);
            }
        }
        __syncthreads();
        if (row0 + GROWS < r1) fetch(row0 + GROWS);
        if (active) {
#pragma unroll
            for (int kk = 0; kk < GROWS; kk += 4) {
                const int kr = kk + lane / 16;
                TA av[2], sv[2], mv[2], al[2], sl[2], ml[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    av[t] = P[kr][wi * 32 + t * 16 + lane % 16];
                    if (COMP) al[t] = Pl[kr][wi * 32 + t * 16 + lane % 16];
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    sv[u] = Q[kr][wj * 32 + u * 16 + lane % 16];
                    mv[u] = R[kr][wj * 32 + u * 16 + lane % 16];
                    if (COMP) {
                        sl[u] = Ql[kr][wj * 32 + u * 16 + lane % 16];
                        ml[u] = Rl[kr][wj * 32 + u * 16 + lane % 16];
                    }
                }
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        if (tile_on[t][u]) {
                            runS[t][u] = mfma4(av[t], sv[u], runS[t][u]);
                            runM[t][u] = mfma4(av[t], mv[u], runM[t][u]);
                            if (COMP) {
                                corS[t][u] = mfma4(av[t], sl[u], corS[t][u]);
                                corS[t][u] = mfma4(al[t], sv[u], corS[t][u]);
                                corM[t][u] = mfma4(av[t], ml[u], corM[t][u]);
                                corM[t][u] = mfma4(al[t], mv[u], corM[t][u]);
                            }
                        }
            }
        }
        __syncthreads();
        if (COMP) {
            fold();                                            // FP64 sum of every 32-row stage
        } else if (MODE == 1 && ++steps == 8) {                // FP32: fold a run of 256 rows into FP64
            fold();
            steps = 0;
        }
    }
    if (!active) return;
    double* out = partial + (chunk * npairs + (item % npairs)) * 2 * GT * GT;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (!tile_on[t][u]) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int rr, cc;
                frag_rc(TA(0), lane, v, rr, cc);
                const int r = wi * 32 + t * 16 + rr, c = wj * 32 + u * 16 + cc;
                out[r * GT + c] = accS[t][u][v] + (double)runS[t][u][v];
                out[GT * GT + r * GT + c] = accM[t][u][v] + (double)runM[t][u][v];
            }
        }
}

// FP64 Gram for q <= 160 (nt <= 10 column tiles of 16): persistent, one
// workgroup of 8 waves per CU forms every upper 16 x 16 tile of both products
// for its rows, so Psi is read once.  Waves 0-3 take Psi^T S Psi, waves 4-7
// Psi^T M Psi; wave slot j of 14 is upper tile 14 (w mod 4) + j in row-major
// tile order (nup = nt (nt + 1) / 2 <= 55 tiles per product), so the matrix
// cores of the four SIMDs get equal work.  Rows go through LDS 16 at a time,
// double-buffered, the next 16 loaded into registers meanwhile.  A stage is
// stored transposed (column-major, GA_TS doubles per column) and the rows are
// assigned to the products' k index so that k-step s of lane group g takes
// stage row 4 g + s: a lane's four operands of a tile for the whole stage are
// contiguous and come in two 16-byte reads.  Output: per workgroup and
// product the upper tiles in row-major tile order, each tile row-major.
namespace {
constexpr int GA_R = 16;          // rows per stage
constexpr int GA_TS = GA_R + 2;   // doubles per column of a transposed stage (16-byte aligned, conflict-free)
constexpr int GA_MAXT = 10;       // column tiles
constexpr int GA_MAT = GA_MAXT * 16 * GA_TS;   // doubles per transposed matrix
constexpr int GA_W = 8;           // waves
constexpr int GA_S = 14;          // tile slots per wave (even: processed in pairs)
constexpr int GA_THREADS = 64 * GA_W;
constexpr int GA_MAX_WG = 1024;
static_assert(GA_W / 2 * GA_S >= GA_MAXT * (GA_MAXT + 1) / 2, "slots must cover the upper tiles");
template <bool HAS_M>
constexpr int gram_all_buf() {   // doubles per stage buffer: Psi, S Psi and M Psi or m
    return (HAS_M ? 3 : 2) * GA_MAT + GA_R;
}
template <bool HAS_M>
constexpr size_t gram_all_lds() {
    return 2 * (size_t)gram_all_buf<HAS_M>() * sizeof(double);
}
typedef double dbl2 __attribute__((ext_vector_type(2)));
}  // namespace

int32_t gram_fp64_single_pass_max_q() { return GA_MAXT * 16; }

int64_t gram_all_partial_doubles(int32_t q) {
    const int64_t nt = cdiv(q, 16), nup = nt * (nt + 1) / 2, per = 2 * nup * 256;
    return GA_MAX_WG * per + per + colsum_tmp_doubles(GA_MAX_WG, (int32_t)per);
}

template <bool HAS_M>
__global__ __launch_bounds__(GA_THREADS) void k_gram_all(const double* __restrict__ Psi, const double* __restrict__ SPsi,
                                                         const double* __restrict__ MPsi,
                                                         const double* __restrict__ mdiag, int64_t n, int32_t q,
                                                         int64_t ld, double* __restrict__ partial) {
    constexpr int BUF = gram_all_buf<HAS_M>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* lds = reinterpret_cast<double*>(smem_raw);
    const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
    const int nt = (q + 15) >> 4, nup = nt * (nt + 1) / 2;
    const int prod = w >= GA_W / 2;
    const int bmat = prod == 0 ? GA_MAT : (HAS_M ? 2 * GA_MAT : 0);   // B operand matrix
    // slot j: LDS offsets of its A (Psi, tile row I) and B (S Psi, M Psi or
    // Psi, tile column J) operand columns
    int aoff[GA_S], boff[GA_S], valid = 0;
#pragma unroll
    for (int j = 0; j < GA_S; ++j) {
        int t = GA_S * (w - prod * (GA_W / 2)) + j;
        const bool v = t < nup;
        t = v ? t : 0;
        int I = 0;
        while (t >= nt - I) {
            t -= nt - I;
            ++I;
        }
        aoff[j] = 16 * I * GA_TS;
        boff[j] = 16 * (I + t) * GA_TS + bmat;
        valid |= (int)v << j;
    }
    const int64_t nblk = (n + GA_R - 1) / GA_R;
    const int64_t my_blocks = blockIdx.x < nblk ? (nblk - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
    constexpr int PE = (GA_R * GA_MAXT * 16 + GA_THREADS - 1) / GA_THREADS;   // 5
    double rp[PE], rs[PE], rm[PE], rmd = 0.0;
    auto fetch = [&](int64_t j) {
        const int64_t r0 = (blockIdx.x + j * gridDim.x) * GA_R;
#pragma unroll
        for (int e = 0; e < PE; ++e) {
            const int idx = tid + GA_THREADS * e, r = idx / (GA_MAXT * 16), c = idx % (GA_MAXT * 16);
            const int64_t row = r0 + r;
            const bool ok = idx < GA_R * GA_MAXT * 16 && row < n && c < q;
            rp[e] = ok ? Psi[row * ld + c] : 0.0;
            rs[e] = ok ? SPsi[row * ld + c] : 0.0;
            rm[e] = (HAS_M && ok) ? MPsi[row * ld + c] : 0.0;
        }
        if (!HAS_M && tid < GA_R) rmd = r0 + tid < n ? mdiag[r0 + tid] : 0.0;
    };
    auto stash = [&](int b) {
        double* P = lds + b * BUF;
#pragma unroll
        for (int e = 0; e < PE; ++e) {
            const int idx = tid + GA_THREADS * e;
            if (idx < GA_R * GA_MAXT * 16) {
                const int r = idx / (GA_MAXT * 16), c = idx % (GA_MAXT * 16);
                P[c * GA_TS + r] = rp[e];
                P[GA_MAT + c * GA_TS + r] = rs[e];
                if (HAS_M) P[2 * GA_MAT + c * GA_TS + r] = rm[e];
            }
        }
        if (!HAS_M && tid < GA_R) P[2 * GA_MAT + tid] = rmd;
    };
    dbl4 acc[GA_S];
#pragma unroll
    for (int j = 0; j < GA_S; ++j) acc[j] = dbl4{0, 0, 0, 0};
    if (my_blocks > 0) {
        fetch(0);
        stash(0);
    }
    __syncthreads();
    for (int64_t jb = 0; jb < my_blocks; ++jb) {
        if (jb + 1 < my_blocks) fetch(jb + 1);
        const double* P = lds + (jb & 1) * BUF;
        const double* PL = P + li * GA_TS + 4 * lk;   // this lane's column and rows within a tile
        // Psi^T M Psi with diagonal M: B operand scaled by m of its row
        dbl4 mk = dbl4{1.0, 1.0, 1.0, 1.0};
        if (!HAS_M && prod == 1) {
            const dbl2 m0 = *reinterpret_cast<const dbl2*>(P + 2 * GA_MAT + 4 * lk);
            const dbl2 m1 = *reinterpret_cast<const dbl2*>(P + 2 * GA_MAT + 4 * lk + 2);
            mk = dbl4{m0[0], m0[1], m1[0], m1[1]};
        }
        // the operands of two slots for the whole stage; the next pair is read
        // while the current pair's 8 products run
        struct Pair {
            dbl2 a0, a1, b0, b1, c0, c1, d0, d1;
        };
        auto operands = [&](int j, Pair& o) {
            o.a0 = *reinterpret_cast<const dbl2*>(PL + aoff[j]);
            o.a1 = *reinterpret_cast<const dbl2*>(PL + aoff[j] + 2);
            o.b0 = *reinterpret_cast<const dbl2*>(PL + boff[j]);
            o.b1 = *reinterpret_cast<const dbl2*>(PL + boff[j] + 2);
            o.c0 = *reinterpret_cast<const dbl2*>(PL + aoff[j + 1]);
            o.c1 = *reinterpret_cast<const dbl2*>(PL + aoff[j + 1] + 2);
            o.d0 = *reinterpret_cast<const dbl2*>(PL + boff[j + 1]);
            o.d1 = *reinterpret_cast<const dbl2*>(PL + boff[j + 1] + 2);
        };
        auto products = [&](int j, const Pair& o) {
            acc[j] = mfma4(o.a0[0], o.b0[0] * mk[0], acc[j]);
            acc[j + 1] = mfma4(o.c0[0], o.d0[0] * mk[0], acc[j + 1]);
            acc[j] = mfma4(o.a0[1], o.b0[1] * mk[1], acc[j]);
            acc[j + 1] = mfma4(o.c0[1], o.d0[1] * mk[1], acc[j + 1]);
            acc[j] = mfma4(o.a1[0], o.b1[0] * mk[2], acc[j]);
            acc[j + 1] = mfma4(o.c1[0], o.d1[0] * mk[2], acc[j + 1]);
            acc[j] = mfma4(o.a1[1], o.b1[1] * mk[3], acc[j]);
            acc[j + 1] = mfma4(o.c1[1], o.d1[1] * mk[3], acc[j + 1]);
        };
        Pair p0, p1;
        operands(0, p0);
#pragma unroll
        for (int j = 0; j < GA_S; j += 4) {
            if (j + 2 < GA_S) operands(j + 2, p1);
            products(j, p0);
            if (j + 4 < GA_S) operands(j + 4, p0);
            if (j + 2 < GA_S) products(j + 2, p1);
        }
        if (jb + 1 < my_blocks) stash((jb + 1) & 1);
        __syncthreads();
    }
    double* out = partial + ((int64_t)blockIdx.x * 2 + prod) * nup * 256;
#pragma unroll
    for (int j = 0; j < GA_S; ++j) {
        if (!((valid >> j) & 1)) continue;
        const int I = aoff[j] / (16 * GA_TS), J = (boff[j] - bmat) / (16 * GA_TS);
        const int64_t t = (int64_t)I * nt - (int64_t)I * (I - 1) / 2 + (J - I);
#pragma unroll
        for (int v = 0; v < 4; ++v) out[t * 256 + (lk + 4 * v) * 16 + li] = acc[j][v];
    }
}

// Sbar, Mbar from the summed upper 16 x 16 tiles of k_gram_all
__global__ void k_gram_all_scatter(const double* __restrict__ sums, int32_t q, double* Sbar, double* Mbar) {
    const int32_t nt = (q + 15) >> 4;
    const int64_t nup = (int64_t)nt * (nt + 1) / 2;
    const int64_t tot = (int64_t)q * q;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        int32_t i = (int32_t)(e / q), j = (int32_t)(e % q);
        if (i > j) { const int32_t x = i; i = j; j = x; }
        const int32_t I = i >> 4, J = j >> 4;
        const int64_t t = (int64_t)I * nt - (int64_t)I * (I - 1) / 2 + (J - I);
        const int64_t off = t * 256 + (i & 15) * 16 + (j & 15);
        Sbar[e] = sums[off];
        Mbar[e] = sums[nup * 256 + off];
    }
}

// Sbar, Mbar (q x q, symmetric) from the summed upper blocks
__global__ void k_gram_scatter(const double* __restrict__ sums, int32_t q, double* Sbar, double* Mbar) {
    const int32_t nt = (q + GT - 1) / GT;
    const int64_t tot = (int64_t)q * q;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        int32_t i = (int32_t)(t / q), j = (int32_t)(t % q);
        if (i > j) { const int32_t x = i; i = j; j = x; }
        const int32_t a = i / GT, b = j / GT;
        const int64_t pair = (int64_t)a * nt - (int64_t)a * (a - 1) / 2 + (b - a);
        const int64_t off = pair * 2 * GT * GT + (i % GT) * GT + (j % GT);
        Sbar[t] = sums[off];
        Mbar[t] = sums[off + GT * GT];
    }
}

hipError_t launch_gram(const double* Psi, const double* SPsi, const double* MPsi, const double* mdiag, int64_t n,
                       int32_t q, int64_t ld, double* partial, int64_t chunk_rows, double* Sbar, double* Mbar,
                       hipStream_t s, int mode) {
    if (mode == 0 && q <= GA_MAXT * 16) {
        const int32_t nt = (int32_t)cdiv(q, 16);
        const int64_t nup = (int64_t)nt * (nt + 1) / 2, per = 2 * nup * 256;
        const int64_t nwg = std::max<int64_t>(1, std::min<int64_t>({(int64_t)device_cus(), cdiv(n, GA_R),
                                                                    (int64_t)GA_MAX_WG}));
        hipError_t e;
        if (mdiag) {
            constexpr size_t lds = gram_all_lds<false>();
            e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_gram_all<false>), lds, 0);
            if (e != hipSuccess) return e;
            k_gram_all<false><<<(unsigned)nwg, GA_THREADS, lds, s>>>(Psi, SPsi, MPsi, mdiag, n, q, ld, partial);
        } else {
            constexpr size_t lds = gram_all_lds<true>();
            e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_gram_all<true>), lds, 0);
            if (e != hipSuccess) return e;
            k_gram_all<true><<<(unsigned)nwg, GA_THREADS, lds, s>>>(Psi, SPsi, MPsi, mdiag, n, q, ld, partial);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        double* sums = partial + nwg * per;
        e = launch_colsum(partial, nwg, (int32_t)per, sums + per, sums, s);
        if (e != hipSuccess) return e;
        k_gram_all_scatter<<<grid_for((int64_t)q * q, 256), 256, 0, s>>>(sums, q, Sbar, Mbar);
        return hipGetLastError();
    }
    if (chunk_rows < 1) return hipErrorInvalidValue;
    const int64_t npairs = gram_pairs(q);
    const int64_t nch = cdiv(n, chunk_rows);
    const int64_t per = npairs * 2 * GT * GT;
    const unsigned grid = (unsigned)(cdiv(nch * npairs, NXCD) * NXCD);
    if (mode == 2)
        k_gram_mfma<2><<<grid, 256, 0, s>>>(Psi, SPsi, MPsi, mdiag, n, q, ld, nch, chunk_rows, partial);
    else if (mode == 1)
        k_gram_mfma<1><<<grid, 256, 0, s>>>(Psi, SPsi, MPsi, mdiag, n, q, ld, nch, chunk_rows, partial);
    else
        k_gram_mfma<0><<<grid, 256, 0, s>>>(Psi, SPsi, MPsi, mdiag, n, q, ld, nch, chunk_rows, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double* sums = partial + nch * per;
    e = launch_colsum(partial, nch, (int32_t)per, sums + per, sums, s);
    if (e != hipSuccess) return e;
    k_gram_scatter<<<grid_for((int64_t)q * q, 256), 256, 0, s>>>(sums, q, Sbar, Mbar);
    return hipGetLastError();
}

// ============================================================ Ritz update + residual
// Phi = Psi Phibar, S Phi = (S Psi) Phibar (registers only), M Phi = m * Phi
// on the finest level or (M Psi) Phibar, on the FP64 matrix cores; per-column
// partial sums of the residual numerator and of the normalisation for the
// first nres columns (S Phi is formed only for those).
// Persistent grid: one workgroup of 8 waves per CU walks 64-row blocks with
// stride gridDim.x; wave w takes rows 16 (w / 2) .. +16 and a set of the
// 16-column tiles of the 160 columns of blockIdx.y chosen so that both waves
// of a row tile issue the same number of matrix-core products (a tile with
// residual columns costs one product more).  The stages (block, 32
// contraction columns, 16 with M Psi) go through LDS, double-buffered -- Psi, S Psi, M Psi
// rows and the Phibar chunk shared by all waves -- the next stage is loaded
// into registers while the current one is multiplied, and within a stage the
// operands of the next 4 contraction columns are read while the current
// products run.
namespace {
constexpr int RZ_RB = 64;            // rows per block
constexpr int RZ_KMAX = 32;          // contraction columns per stage (16 with M Psi: LDS)
constexpr int RZ_LD = RZ_KMAX + 2;   // LDS row stride of the row stage (16-byte rows, conflict-free 16-byte reads)
constexpr int RZ_COLS = 160;         // output columns per workgroup
constexpr int RZ_BLD = RZ_COLS;      // LDS row stride of the Phibar stage
constexpr int RZ_THREADS = 512;
constexpr int RZ_MAX_WG = 2048;      // persistent workgroups at most (partial-sum rows)
constexpr int RZ_SL = 5;             // column tiles per wave at most
template <bool HAS_M>
constexpr int ritz_k() {             // contraction columns per stage
    return HAS_M ? 16 : 32;
}
template <bool HAS_M>
constexpr int ritz_buf() {           // doubles per stage buffer
    return (HAS_M ? 3 : 2) * RZ_RB * RZ_LD + ritz_k<HAS_M>() * RZ_BLD;
}
template <bool HAS_M>
constexpr size_t ritz_lds() {   // two stage buffers + the per-row-tile column sums
    return (2 * (size_t)ritz_buf<HAS_M>() + 4 * 2 * RZ_COLS) * sizeof(double);
}
// column tiles [0, ns) have residual columns; wave half 0 takes tiles
// [0, a) and [ns, ns + x), half 1 the rest, with x balancing the products
// (cS per residual tile, cP per other tile).  Returns false when a half would
// get more than RZ_SL tiles.
__host__ __device__ inline bool ritz_split(int nt, int ns, bool has_m, int& a, int& x) {
    const int cS = has_m ? 3 : 2, cP = has_m ? 2 : 1;
    a = (ns + 1) / 2;
    const int b = ns - a, po = nt - ns;
    x = ((b - a) * cS + po * cP + cP) / (2 * cP);
    x = x < 0 ? 0 : (x > po ? po : x);
    return a + x <= RZ_SL && b + po - x <= RZ_SL;
}
}  // namespace

int64_t ritz_partial_doubles(int64_t /*n*/, int32_t q, int64_t /*chunk_rows*/) {
    return (int64_t)RZ_MAX_WG * 2 * q + 2 * (int64_t)q + colsum_tmp_doubles(RZ_MAX_WG, 2 * q);
}

template <bool HAS_M>
__global__ __launch_bounds__(RZ_THREADS) void k_ritz_mfma(const double* __restrict__ Psi, const double* __restrict__ SPsi,
                                                          const double* __restrict__ MPsi, const double* __restrict__ mdiag,
                                                          const double* __restrict__ Phibar, const double* __restrict__ lam,
                                                          int64_t n, int32_t q, int64_t ld, double* __restrict__ Phi,
                                                          double* __restrict__ MPhi, double* __restrict__ partial,
                                                          int minv_norm, int32_t nres) {
    constexpr int RZ_K = ritz_k<HAS_M>();
    constexpr int BUF = ritz_buf<HAS_M>();
    constexpr int AM = RZ_RB * RZ_LD;                      // doubles per staged row matrix
    constexpr int BOFF = (HAS_M ? 3 : 2) * AM;             // Phibar chunk within a buffer
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* lds = reinterpret_cast<double*>(smem_raw);
    // residual numerator / normalisation sums per row tile and column, each
    // entry owned by one lane
    double(*red)[2][RZ_COLS] = reinterpret_cast<double(*)[2][RZ_COLS]>(lds + 2 * BUF);
    const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
    const int wr = w >> 1, wc = w & 1;
    for (int i = tid; i < 4 * 2 * RZ_COLS; i += RZ_THREADS) (&red[0][0][0])[i] = 0.0;
    const int col0 = blockIdx.y * RZ_COLS;
    const int ncol = min(RZ_COLS, q - col0);
    const int nt = (ncol + 15) >> 4;
    const int ns = nres > col0 ? min(nt, (nres - col0 + 15) >> 4) : 0;
    int sa, sx;
    ritz_split(nt, ns, HAS_M, sa, sx);
    // this wave's column tiles: two runs [t1, t1 + c1) and [t2, t2 + c2)
    const int t1 = wc ? sa : 0, c1 = wc ? ns - sa : sa;
    const int t2 = wc ? ns + sx : ns, c2 = wc ? nt - ns - sx : sx;
    const int ntw = min(RZ_SL, c1 + c2);
    int tile[RZ_SL];
#pragma unroll
    for (int u = 0; u < RZ_SL; ++u) tile[u] = u < c1 ? t1 + u : t2 + (u - c1);
    const int64_t nblk = (n + RZ_RB - 1) / RZ_RB;
    const int nk = (q + RZ_K - 1) / RZ_K;
    const int64_t my_blocks = blockIdx.x < nblk ? (nblk - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
    const int64_t nst = my_blocks * nk;
    constexpr int PA = RZ_RB * RZ_K / RZ_THREADS;     // row-stage values per thread
    constexpr int PB = RZ_K * RZ_COLS / RZ_THREADS;   // Phibar values per thread
    double ra[PA], rs[PA], rm[PA], rb[PB];
    auto fetch = [&](int64_t st) {
        const int64_t r0 = (blockIdx.x + (st / nk) * gridDim.x) * RZ_RB;
        const int k0 = (int)(st % nk) * RZ_K;
#pragma unroll
        for (int e = 0; e < PA; ++e) {
            const int idx = tid + RZ_THREADS * e, r = idx / RZ_K, kk = idx % RZ_K;
            const int64_t row = r0 + r;
            const bool ok = row < n && k0 + kk < q;
            ra[e] = ok ? Psi[row * ld + k0 + kk] : 0.0;
            rs[e] = ok ? SPsi[row * ld + k0 + kk] : 0.0;
            rm[e] = (HAS_M && ok) ? MPsi[row * ld + k0 + kk] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < PB; ++e) {
            const int idx = tid + RZ_THREADS * e, kk = idx / RZ_COLS, c = idx % RZ_COLS;
            rb[e] = (k0 + kk < q && c < ncol) ? Phibar[(int64_t)(k0 + kk) * q + col0 + c] : 0.0;
        }
    };
    auto stash = [&](int b) {
        double* L = lds + b * BUF;
#pragma unroll
        for (int e = 0; e < PA; ++e) {
            const int idx = tid + RZ_THREADS * e, r = idx / RZ_K, kk = idx % RZ_K;
            L[r * RZ_LD + kk] = ra[e];
            L[AM + r * RZ_LD + kk] = rs[e];
            if (HAS_M) L[2 * AM + r * RZ_LD + kk] = rm[e];
        }
#pragma unroll
        for (int e = 0; e < PB; ++e) {
            const int idx = tid + RZ_THREADS * e;
            L[BOFF + (idx / RZ_COLS) * RZ_BLD + idx % RZ_COLS] = rb[e];
        }
    };
    dbl4 aP[RZ_SL], aS[RZ_SL], aM[RZ_SL];
#pragma unroll
    for (int u = 0; u < RZ_SL; ++u) aP[u] = aS[u] = aM[u] = dbl4{0, 0, 0, 0};
    if (nst > 0) {
        fetch(0);
        stash(0);
    }
    __syncthreads();
    for (int64_t st = 0; st < nst; ++st) {
        if (st + 1 < nst) fetch(st + 1);
        const double* L = lds + (st & 1) * BUF;
        // contraction column k of step s of 16-column chunk h is 16 h + 4 g + s
        // for lane group g, so the A operands of a lane for a whole chunk are
        // 4 consecutive values of its row (two 16-byte reads per matrix)
        const double* Ar = L + (wr * 16 + li) * RZ_LD + 4 * lk;
        auto apair = [&](int h, int j, int mat) {
            return *reinterpret_cast<const dbl2*>(Ar + mat * AM + 16 * h + 2 * j);
        };
        auto bops = [&](int k, double(&b)[RZ_SL]) {
            const double* Br = L + BOFF + k * RZ_BLD + li;
#pragma unroll
            for (int u = 0; u < RZ_SL; ++u)
                if (u < ntw) b[u] = Br[16 * tile[u]];
        };
        auto products = [&](double p, double q, double mm, const double(&b)[RZ_SL]) {
#pragma unroll
            for (int u = 0; u < RZ_SL; ++u)
                if (u < ntw) {
                    aP[u] = mfma4(p, b[u], aP[u]);
                    if (tile[u] < ns) aS[u] = mfma4(q, b[u], aS[u]);
                    if (HAS_M) aM[u] = mfma4(mm, b[u], aM[u]);
                }
        };
#pragma unroll
        for (int h = 0; h < RZ_K / 16; ++h) {
            const dbl2 pa = apair(h, 0, 0), sa = apair(h, 0, 1);
            const dbl2 ma = HAS_M ? apair(h, 0, 2) : dbl2{0, 0};
            double b0[RZ_SL], b1[RZ_SL];
            bops(16 * h + 4 * lk, b0);
            bops(16 * h + 4 * lk + 1, b1);
            const dbl2 pc = apair(h, 1, 0), sc = apair(h, 1, 1);
            const dbl2 mc = HAS_M ? apair(h, 1, 2) : dbl2{0, 0};
            products(pa[0], sa[0], ma[0], b0);
            bops(16 * h + 4 * lk + 2, b0);
            products(pa[1], sa[1], ma[1], b1);
            bops(16 * h + 4 * lk + 3, b1);
            products(pc[0], sc[0], mc[0], b0);
            products(pc[1], sc[1], mc[1], b1);
        }
        if ((int)(st % nk) == nk - 1) {
            // block finished: Phi (and M Phi) out, residual sums (one tile at a
            // time, reduced over the 4 lanes that share a column), accumulators reset
            const int64_t r0 = (blockIdx.x + (st / nk) * gridDim.x) * RZ_RB + wr * 16 + lk;
#pragma unroll
            for (int u = 0; u < RZ_SL; ++u) {
                if (u >= ntw) continue;
                const int col = col0 + tile[u] * 16 + li;
                const bool has_res = tile[u] < ns;
                const double lc = has_res && col < nres ? lam[col] : 0.0;
                double num = 0.0, den = 0.0;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t row = r0 + 4 * v;
                    if (row < n && col < q) {
                        const double mr = HAS_M ? 0.0 : mdiag[row];
                        const double phi = aP[u][v];
                        const double mphi = HAS_M ? aM[u][v] : mr * phi;
                        Phi[row * ld + col] = phi;
                        if (MPhi) MPhi[row * ld + col] = mphi;
                        if (has_res && col < nres) {
                            const double res = aS[u][v] - lc * mphi;
                            if (minv_norm) {
                                num += res * res / mr;
                                den += phi * mphi;
                            } else {
                                num += res * res;
                                den += mphi * mphi;
                            }
                        }
                    }
                }
                if (has_res) {
                    num += __shfl_xor(num, 16);
                    num += __shfl_xor(num, 32);
                    den += __shfl_xor(den, 16);
                    den += __shfl_xor(den, 32);
                    if (lane < 16) {
                        red[wr][0][tile[u] * 16 + lane] += num;
                        red[wr][1][tile[u] * 16 + lane] += den;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < RZ_SL; ++u) aP[u] = aS[u] = aM[u] = dbl4{0, 0, 0, 0};
        }
        if (st + 1 < nst) stash((st + 1) & 1);
        __syncthreads();
    }
    if (tid < ncol) {
        partial[(int64_t)blockIdx.x * 2 * q + col0 + tid] =
            (red[0][0][tid] + red[1][0][tid]) + (red[2][0][tid] + red[3][0][tid]);
        partial[(int64_t)blockIdx.x * 2 * q + q + col0 + tid] =
            (red[0][1][tid] + red[1][1][tid]) + (red[2][1][tid] + red[3][1][tid]);
    }
}

// out[blockIdx.y, c] = sum of rows [y * rpb, (y + 1) * rpb) of column c of
// the row-major nrows x ncols array; 64 columns x 4 row lanes per workgroup
__global__ __launch_bounds__(256) void k_colsum(const double* __restrict__ in, int64_t nrows, int32_t ncols,
                                                int64_t rpb, double* __restrict__ out) {
    __shared__ double red[4][64];
    const int cl = threadIdx.x % 64, g = threadIdx.x / 64;
    const int64_t c = (int64_t)blockIdx.x * 64 + cl;
    const int64_t r0 = (int64_t)blockIdx.y * rpb, r1 = min(nrows, r0 + rpb);
    double a0 = 0, a1 = 0;
    if (c < ncols) {
        int64_t r = r0 + g;
        for (; r + 4 < r1; r += 8) {
            a0 += in[r * ncols + c];
            a1 += in[(r + 4) * ncols + c];
        }
        if (r < r1) a0 += in[r * ncols + c];
    }
    red[g][cl] = a0 + a1;
    __syncthreads();
    if (g == 0 && c < ncols) out[(int64_t)blockIdx.y * ncols + c] = (red[0][cl] + red[1][cl]) + (red[2][cl] + red[3][cl]);
}

// column sums of a tall row-major array into out[ncols]; tmp holds
// colsum_tmp_doubles(nrows, ncols) doubles
namespace {
constexpr int64_t COLSUM_RPB = 128;
}
int64_t colsum_tmp_doubles(int64_t nrows, int32_t ncols) { return cdiv(nrows, COLSUM_RPB) * (int64_t)ncols; }

hipError_t launch_colsum(const double* in, int64_t nrows, int32_t ncols, double* tmp, double* out, hipStream_t s) {
    const unsigned gx = (unsigned)cdiv(ncols, 64);
    if (nrows <= COLSUM_RPB * 8) {
        k_colsum<<<dim3(gx, 1), 256, 0, s>>>(in, nrows, ncols, nrows, out);
        return hipGetLastError();
    }
    const int64_t n1 = cdiv(nrows, COLSUM_RPB);
    k_colsum<<<dim3(gx, (unsigned)n1), 256, 0, s>>>(in, nrows, ncols, COLSUM_RPB, tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_colsum<<<dim3(gx, 1), 256, 0, s>>>(tmp, n1, ncols, n1, out);
    return hipGetLastError();
}

__global__ void k_resid_final(const double* __restrict__ sums, int32_t q, int32_t nres, const double* __restrict__ lam,
                              double lam_floor, double* resid) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= q) return;
    resid[c] = c < nres ? sqrt(sums[c]) / (fmax(fabs(lam[c]), lam_floor) * sqrt(sums[q + c])) : NAN;
}

hipError_t launch_ritz(const double* Psi, const double* SPsi, const double* MPsi, const double* mdiag,
                       const double* Phibar, const double* lam, int64_t n, int32_t q, int64_t ld, double* Phi,
                       double* MPhi, double* partial, int64_t /*chunk_rows*/, bool minv_norm, double lam_floor,
                       double* resid, hipStream_t s, int32_t nres) {
    if (nres < 0 || nres > q) nres = q;
    for (int32_t c0 = 0; c0 < q; c0 += RZ_COLS) {
        const int nt = (int)cdiv(std::min<int32_t>(RZ_COLS, q - c0), 16);
        const int ns = nres > c0 ? std::min<int>(nt, (int)cdiv(nres - c0, 16)) : 0;
        int a, x;
        if (!ritz_split(nt, ns, MPsi != nullptr && !mdiag, a, x)) return hipErrorInvalidValue;
    }
    const int64_t nblk = cdiv(n, RZ_RB);
    const int64_t nwg = std::max<int64_t>(1, std::min<int64_t>({(int64_t)device_cus(), nblk, (int64_t)RZ_MAX_WG}));
    const dim3 grid((unsigned)nwg, (unsigned)cdiv(q, RZ_COLS));
    hipError_t e;
    if (mdiag) {
        constexpr size_t lds = ritz_lds<false>();
        e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_ritz_mfma<false>), lds, 0);
        if (e != hipSuccess) return e;
        k_ritz_mfma<false><<<grid, RZ_THREADS, lds, s>>>(Psi, SPsi, MPsi, mdiag, Phibar, lam, n, q, ld, Phi, MPhi,
                                                         partial, minv_norm ? 1 : 0, nres);
    } else {
        constexpr size_t lds = ritz_lds<true>();
        e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_ritz_mfma<true>), lds, 0);
        if (e != hipSuccess) return e;
        k_ritz_mfma<true><<<grid, RZ_THREADS, lds, s>>>(Psi, SPsi, MPsi, mdiag, Phibar, lam, n, q, ld, Phi, MPhi,
                                                        partial, minv_norm ? 1 : 0, nres);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    double* sums = partial + nwg * 2 * (int64_t)q;
    e = launch_colsum(partial, nwg, 2 * q, sums + 2 * (int64_t)q, sums, s);
    if (e != hipSuccess) return e;
    k_resid_final<<<(unsigned)cdiv(q, 256), 256, 0, s>>>(sums, q, nres, lam, lam_floor, resid);
    return hipGetLastError();
}

// ============================================================ dense GEP helpers
__global__ void k_equilibrate(const double* S, const double* M, int32_t k, double* So, double* Mo, double* e) {
    const int64_t tot = (int64_t)k * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = (int32_t)(t / k), j = (int32_t)(t % k);
        const double ei = 1.0 / sqrt(M[(int64_t)i * k + i]), ej = 1.0 / sqrt(M[(int64_t)j * k + j]);
        So[t] = 0.5 * (S[t] + S[(int64_t)j * k + i]) * ei * ej;
        Mo[t] = 0.5 * (M[t] + M[(int64_t)j * k + i]) * ei * ej;
        if (j == 0) e[i] = ei;
    }
}
hipError_t launch_equilibrate(const double* S, const double* M, int32_t k, double* So, double* Mo, double* e,
                              hipStream_t s) {
    k_equilibrate<<<grid_for((int64_t)k * k, 256), 256, 0, s>>>(S, M, k, So, Mo, e);
    return hipGetLastError();
}

// ============================================================ device assembly
// Cotangent stiffness and lumped mass of the finest level (eq. massStiffMatrices)
// on the device, for the pattern the host derived from the triangles.  Plain
// IEEE arithmetic without contraction, in the host assembly's order, so the
// values equal the host's bit for bit.
#pragma clang fp contract(off)
// per triangle t: w[3t + k] = -cot(angle at corner k) / 2, a3[t] = area / 3
__global__ void k_tri_weights(const double* __restrict__ V, const int32_t* __restrict__ F, int64_t nf,
                              double* __restrict__ w, double* __restrict__ a3) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nf; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t f[3] = {F[3 * t], F[3 * t + 1], F[3 * t + 2]};
        for (int k = 0; k < 3; ++k) {
            const double* P = V + 3 * (int64_t)f[k];
            const double* Q = V + 3 * (int64_t)f[(k + 1) % 3];
            const double* R = V + 3 * (int64_t)f[(k + 2) % 3];
            const double ux = Q[0] - P[0], uy = Q[1] - P[1], uz = Q[2] - P[2];
            const double vx = R[0] - P[0], vy = R[1] - P[1], vz = R[2] - P[2];
            const double dot = ux * vx + uy * vy + uz * vz;
            const double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
            w[3 * t + k] = -0.5 * (dot / sqrt(cx * cx + cy * cy + cz * cz));
        }
        const double* a = V + 3 * (int64_t)f[0];
        const double* b = V + 3 * (int64_t)f[1];
        const double* c = V + 3 * (int64_t)f[2];
        const double e1x = b[0] - a[0], e1y = b[1] - a[1], e1z = b[2] - a[2];
        const double e2x = c[0] - a[0], e2y = c[1] - a[1], e2z = c[2] - a[2];
        const double cx = e1y * e2z - e1z * e2y, cy = e1z * e2x - e1x * e2z, cz = e1x * e2y - e1y * e2x;
        a3[t] = 0.5 * sqrt(cx * cx + cy * cy + cz * cz) / 3.0;
    }
}
// S values on the pattern: an off-diagonal entry sums the weights of the (at
// most two) corners opposite its edge, in triangle order; the diagonal entry
// sums the negated weights of every corner opposite an edge at the vertex,
// in triangle order (corner lists prepared by the host)
__global__ void k_assemble_stiffness(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                                     const int64_t* __restrict__ corner, int64_t n, const int64_t* __restrict__ dptr,
                                     const int64_t* __restrict__ dcorner, const double* __restrict__ w,
                                     double* __restrict__ val) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
            double v = 0.0;
            if (idx[e] == i) {
                for (int64_t c = dptr[i]; c < dptr[i + 1]; ++c) v += -w[dcorner[c]];
            } else {
                if (corner[2 * e] >= 0) v += w[corner[2 * e]];
                if (corner[2 * e + 1] >= 0) v += w[corner[2 * e + 1]];
            }
            val[e] = v;
        }
    }
}
// m_i = density_i * sum over the triangles at i (ascending) of area / 3
__global__ void k_assemble_mass(const int64_t* __restrict__ vptr, const int32_t* __restrict__ vtri, int64_t n,
                                const double* __restrict__ a3, const double* __restrict__ density,
                                double* __restrict__ m) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int64_t k = vptr[i]; k < vptr[i + 1]; ++k) v += a3[vtri[k]];
        m[i] = density ? v * density[i] : v;
    }
}
#pragma clang fp contract(on)
hipError_t launch_assemble_mesh(const double* V, const int32_t* F, int64_t nf, int64_t n, const int64_t* ptr,
                                const int32_t* idx, const int64_t* corner, const int64_t* dptr,
                                const int64_t* dcorner, const int64_t* vptr, const int32_t* vtri,
                                const double* density, double* w, double* a3, double* sval, double* mdiag,
                                hipStream_t s) {
    if (nf <= 0 || n <= 0) return hipErrorInvalidValue;
    k_tri_weights<<<grid_for(nf, 256), 256, 0, s>>>(V, F, nf, w, a3);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_assemble_stiffness<<<grid_for(n, 256), 256, 0, s>>>(ptr, idx, corner, n, dptr, dcorner, w, sval);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_assemble_mass<<<grid_for(n, 256), 256, 0, s>>>(vptr, vtri, n, a3, density, mdiag);
    return hipGetLastError();
}

// Descriptor and factorisation work lists of a dense k x k problem held as one
// front of Mt x Mt tiles: per pivot tile step st the diagonal item (front 0),
// the panel items (0, I) for I > st, the update items (0, I, J) for
// st < J <= I, the inverse-panel row items (0, j) for j <= st and update
// items (0, I, j) for I > st, j <= st; the product items (0, I) of the
// 32-row tiles of the k rows; the solve's row-gather pointers are all zero.
// The front's inverse panel P = L^-1 starts at offset 0 of its own arrays.
// One thread writes them (a few thousand integers at most for k = 1000).
__global__ void k_dense_lists(DFront* front, int32_t k, int32_t ns_pad, int32_t Mt, int32_t* diag, int32_t* panel,
                              int32_t* upd, int32_t* qrow, int32_t* qupd, int32_t* prod, int64_t* gptr) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    DFront f{};
    f.ns = k;
    f.ns_pad = ns_pad;
    f.Mt = Mt;
    f.nsb = Mt;
    f.parent = -1;
    f.q_base = 0;
    f.qrow = 0;
    *front = f;
    int64_t nd = 0, np = 0, nu = 0, nqr = 0, nqu = 0;
    for (int32_t st = 0; st < Mt; ++st) {
        diag[nd++] = 0;
        for (int32_t I = st + 1; I < Mt; ++I) {
            panel[2 * np] = 0;
            panel[2 * np + 1] = I;
            ++np;
        }
        for (int32_t J = st + 1; J < Mt; ++J)
            for (int32_t I = J; I < Mt; ++I) {
                upd[3 * nu] = 0;
                upd[3 * nu + 1] = I;
                upd[3 * nu + 2] = J;
                ++nu;
            }
        for (int32_t j = 0; j <= st; ++j) {
            qrow[2 * nqr] = 0;
            qrow[2 * nqr + 1] = j;
            ++nqr;
        }
        for (int32_t I = st + 1; I < Mt; ++I)
            for (int32_t j = 0; j <= st; ++j) {
                qupd[3 * nqu] = 0;
                qupd[3 * nqu + 1] = I;
                qupd[3 * nqu + 2] = j;
                ++nqu;
            }
    }
    for (int32_t o = 0; o < Mt; ++o) {
        prod[2 * o] = 0;
        prod[2 * o + 1] = o;
    }
    for (int32_t i = 0; i <= k; ++i) gptr[i] = 0;
}
hipError_t launch_dense_lists(DFront* front, int32_t k, int32_t ns_pad, int32_t Mt, int32_t* diag, int32_t* panel,
                              int32_t* upd, int32_t* qrow, int32_t* qupd, int32_t* prod, int64_t* gptr,
                              hipStream_t s) {
    k_dense_lists<<<1, 64, 0, s>>>(front, k, ns_pad, Mt, diag, panel, upd, qrow, qupd, prod, gptr);
    return hipGetLastError();
}

__global__ void k_dense_to_front(const double* A, int32_t k, double* tiles, int32_t Mt) {
    const int64_t np = (int64_t)Mt * T32;
    const int64_t tot = np * np;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = (int32_t)(t / np), r = (int32_t)(t % np);
        if (r < c) continue;
        double v = 0.0;
        if (r < k && c < k) v = A[(int64_t)r * k + c];
        else if (r == c) v = 1.0;
        tiles[tri(Mt, r / T32, c / T32) * TT + (c % T32) * T32 + r % T32] = v;
    }
}
hipError_t launch_dense_to_front(const double* A, int32_t k, double* tiles, int32_t Mt, hipStream_t s) {
    const int64_t np = (int64_t)Mt * T32;
    k_dense_to_front<<<grid_for(np * np, 256), 256, 0, s>>>(A, k, tiles, Mt);
    return hipGetLastError();
}

__global__ void k_transpose(const double* A, int32_t k, double* B) {
    __shared__ double t[T32][T32 + 1];
    const int bx = blockIdx.x * T32, by = blockIdx.y * T32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int yy = ty; yy < T32; yy += 8) {
        int r = by + yy, c = bx + tx;
        t[yy][tx] = (r < k && c < k) ? A[(int64_t)r * k + c] : 0.0;
    }
    __syncthreads();
    for (int yy = ty; yy < T32; yy += 8) {
        int r = bx + yy, c = by + tx;
        if (r < k && c < k) B[(int64_t)r * k + c] = t[tx][yy];
    }
}
hipError_t launch_transpose(const double* A, int32_t k, double* B, hipStream_t s) {
    const unsigned g = (unsigned)cdiv(k, T32);
    k_transpose<<<dim3(g, g), 256, 0, s>>>(A, k, B);
    return hipGetLastError();
}

__global__ void k_sym_scale(const double* A, const double* D, int32_t k, double* C) {
    const int64_t tot = (int64_t)k * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = (int32_t)(t / k), j = (int32_t)(t % k);
        C[t] = 0.5 * (A[t] + A[(int64_t)j * k + i]) / sqrt(D[i] * D[j]);
    }
}
hipError_t launch_sym_scale(const double* A, const double* D, int32_t k, double* C, hipStream_t s) {
    k_sym_scale<<<grid_for((int64_t)k * k, 256), 256, 0, s>>>(A, D, k, C);
    return hipGetLastError();
}

__global__ void k_row_scale(const double* V, const double* w, int sqrt_w, int64_t rows, int32_t k, int64_t ld,
                            double* Y) {
    const int64_t tot = rows * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / k;
        const int32_t c = (int32_t)(t % k);
        const double f = sqrt_w ? sqrt(w[i]) : w[i];
        Y[i * ld + c] = V[i * ld + c] * f;
    }
}
hipError_t launch_row_scale(const double* V, const double* w, bool sqrt_w, int64_t rows, int32_t k, int64_t ld,
                            double* Y, hipStream_t s) {
    k_row_scale<<<grid_for(rows * k, 256), 256, 0, s>>>(V, w, sqrt_w ? 1 : 0, rows, k, ld, Y);
    return hipGetLastError();
}

// ---- block Jacobi in round-robin order ----------------------------------
// The m x m matrix (m a multiple of 2b) is split into nb = m / b blocks of b
// indices; a round pairs the blocks at tournament positions x and nb-1-x
// (position 0 fixed, positions 1..nb-1 hold blocks 1 + (x - 1 + r) mod (nb - 1)).
// Every pair's 2b x 2b principal submatrix is diagonalised by cyclic Jacobi
// in LDS (k_bj_local), then C <- J^T C J and V <- V J with J the
// block-diagonal product of the pairs' orthogonal factors (k_bj_apply).
__device__ __forceinline__ int jac_player(int x, int r, int m) { return x == 0 ? 0 : 1 + (x - 1 + r) % (m - 1); }

__device__ __forceinline__ void bj_pair(int k, int r, int nb, int& I, int& J) {
    const int a = jac_player(k, r, nb), c = jac_player(nb - 1 - k, r, nb);
    I = min(a, c);
    J = max(a, c);
}
template <int B>
__device__ __forceinline__ int bj_index(int l, int I, int J) { return l < B ? I * B + l : J * B + (l - B); }

// Jacobi rotation annihilating a_pq of the 2 x 2 block [[app, apq], [apq, aqq]]:
// the angle |theta| <= pi / 4 with tan 2 theta = 2 a_pq / (a_qq - a_pp), from
// the half-angle identities cos^2 theta = (1 + cos 2 theta) / 2 and
// sin theta = sin 2 theta / (2 cos theta) with cos 2 theta = |d| / r,
// sin 2 theta = sign(d) e / r (d = a_qq - a_pp, e = 2 a_pq, r = hypot(d, e)),
// which needs two reciprocal square roots and no division.  False (and c = 1,
// s = 0) when |a_pq| <= max(tol_abs, tol_rel sqrt|a_pp a_qq|), compared in
// squares.  Every thread that needs a rotation computes it itself from the
// same three values, so all copies agree bit for bit.
__device__ __forceinline__ bool jacobi_rotation(double app, double aqq, double apq, double tol_abs2, double tol_rel2,
                                                double& c, double& s) {
    c = 1.0;
    s = 0.0;
    if (!(apq * apq > fmax(tol_abs2, tol_rel2 * fabs(app * aqq)))) return false;
    const double d = aqq - app, e = 2.0 * apq;
    const double rinv = rsqrt(d * d + e * e);
    const double u = 0.5 + 0.5 * (fabs(d) * rinv);
    const double rc = rsqrt(u);
    c = u * rc;
    s = (d >= 0 ? 0.5 : -0.5) * e * rinv * rc;
    return true;
}

// One workgroup of b^2 threads per block pair; Q (2b x 2b, row-major, Q[l][c])
// of every pair to Qs.  A round of the inner cyclic sweep rotates the b
// disjoint index pairs of the tournament order at once; thread (k1, k2) owns
// the 2 x 2 block {p_k1, q_k1} x {p_k2, q_k2} of A and the entries
// {k1, k1 + b} x {p_k2, q_k2} of Q.  It computes both rotations it needs from
// the round's input, so a round needs one barrier: A is double-buffered (every
// entry is rewritten each round), Q entries have one owner per round.
template <int B>
constexpr size_t bj_local_lds() {   // A (double-buffered), Q and a counter
    return 3 * sizeof(double) * (2 * B) * (2 * B + 1) + 16;
}
template <int B>
__device__ void bj_local_solve(const double* C, int32_t m, int32_t r, int32_t P, double* __restrict__ Qs,
                               const double* __restrict__ normf, double tol_rel, double tol_abs_rel,
                               int32_t max_sweeps, int32_t* rot_count, int32_t* __restrict__ qrot,
                               unsigned char* smem_raw) {
    // 2 b^2 threads: thread (k1, k2) < b^2 owns the 2 x 2 block {p_k1, q_k1} x
    // {p_k2, q_k2} of A, thread b^2 + (k1, k2) the entries {k1, k1 + b} x
    // {p_k2, q_k2} of Q; both compute the rotations they need from the step's
    // input, so a step needs one barrier (A double-buffered, Q entries with one
    // owner per step)
    constexpr int W = 2 * B, NT = B * B;
    double(*A)[W][W + 1] = reinterpret_cast<double(*)[W][W + 1]>(smem_raw);   // [2][W][W + 1]
    double(*Q)[W + 1] = reinterpret_cast<double(*)[W + 1]>(smem_raw + 2 * sizeof(double) * W * (W + 1));
    int& total = *reinterpret_cast<int*>(smem_raw + 3 * sizeof(double) * W * (W + 1));
    const int nb = m / B;
    int I, J;
    bj_pair(P, r, nb, I, J);
    const double tol_abs2 = tol_abs_rel * normf[0] * tol_abs_rel * normf[0];
    const double tol_rel2 = tol_rel * tol_rel;
    const int tid = threadIdx.x;
    const bool qthread = tid >= NT;
    const int tt = qthread ? tid - NT : tid, k1 = tt / B, k2 = tt % B;
    for (int idx = tid; idx < W * W; idx += 2 * NT) {
        const int a = idx / W, c = idx % W;
        A[0][a][c] = C[(int64_t)bj_index<B>(a, I, J) * m + bj_index<B>(c, I, J)];
        Q[a][c] = a == c ? 1.0 : 0.0;
    }
    if (tid == 0) total = 0;
    __syncthreads();
    // no entry above the threshold: a sweep would rotate nothing (the test only
    // reads entries that nothing changes), so Q is the identity and the apply
    // launch skips this pair
    int pred = 0;
    for (int idx = tid; idx < W * W; idx += 2 * NT) {
        const int a = idx / W, c = idx % W;
        const double apq = A[0][a][c];
        pred |= a < c && apq * apq > fmax(tol_abs2, tol_rel2 * fabs(A[0][a][a] * A[0][c][c]));
    }
    double* Qo = Qs + (int64_t)P * W * W;
    if (!__syncthreads_or(pred)) {
        for (int idx = tid; idx < W * W; idx += 2 * NT) Qo[idx] = idx / W == idx % W ? 1.0 : 0.0;
        if (tid == 0) qrot[P] = 0;
        return;
    }
    int cur = 0, seen = 0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        int mine = 0;
        for (int rr = 0; rr < W - 1; ++rr) {
            const int a2 = jac_player(k2, rr, W), b2 = jac_player(W - 1 - k2, rr, W);
            const int p2 = min(a2, b2), q2 = max(a2, b2);
            const double(*Ac)[W + 1] = A[cur];
            if (qthread) {
                // Q <- Q J on rows k1 and k1 + b
                const double d2p = Ac[p2][p2], d2q = Ac[q2][q2], o2 = Ac[p2][q2];
                const double u0 = Q[k1][p2], v0 = Q[k1][q2], u1 = Q[k1 + B][p2], v1 = Q[k1 + B][q2];
                double c2, s2;
                jacobi_rotation(d2p, d2q, o2, tol_abs2, tol_rel2, c2, s2);
                Q[k1][p2] = u0 * c2 - v0 * s2;
                Q[k1][q2] = u0 * s2 + v0 * c2;
                Q[k1 + B][p2] = u1 * c2 - v1 * s2;
                Q[k1 + B][q2] = u1 * s2 + v1 * c2;
            } else {
                // A <- J^T A J on the 2 x 2 block of pairs k1, k2
                const int a1 = jac_player(k1, rr, W), b1 = jac_player(W - 1 - k1, rr, W);
                const int p1 = min(a1, b1), q1 = max(a1, b1);
                double(*An)[W + 1] = A[cur ^ 1];
                const double d1p = Ac[p1][p1], d1q = Ac[q1][q1], o1 = Ac[p1][q1];
                const double d2p = Ac[p2][p2], d2q = Ac[q2][q2], o2 = Ac[p2][q2];
                const double x00 = Ac[p1][p2], x01 = Ac[p1][q2], x10 = Ac[q1][p2], x11 = Ac[q1][q2];
                double c1, s1, c2, s2;
                const bool rot1 = jacobi_rotation(d1p, d1q, o1, tol_abs2, tol_rel2, c1, s1);
                jacobi_rotation(d2p, d2q, o2, tol_abs2, tol_rel2, c2, s2);
                const double t00 = c1 * x00 - s1 * x10, t01 = c1 * x01 - s1 * x11;
                const double t10 = s1 * x00 + c1 * x10, t11 = s1 * x01 + c1 * x11;
                An[p1][p2] = c2 * t00 - s2 * t01;
                An[q1][q2] = s2 * t10 + c2 * t11;
                if (k1 == k2 && rot1) {
                    ++mine;
                    An[p1][q2] = 0.0;
                    An[q1][p2] = 0.0;
                } else {
                    An[p1][q2] = s2 * t00 + c2 * t01;
                    An[q1][p2] = c2 * t10 - s2 * t11;
                }
            }
            cur ^= 1;
            __syncthreads();
        }
        if (mine) atomicAdd(&total, mine);
        __syncthreads();
        const int now = total;
        if (now == seen) break;
        seen = now;
    }
    for (int idx = tid; idx < W * W; idx += 2 * NT) Qo[idx] = Q[idx / W][idx % W];
    if (tid == 0) qrot[P] = 1;
    if (tid == 0 && seen) atomicAdd(rot_count, seen);
    __syncthreads();   // LDS free for the caller
}
template <int B>
__global__ __launch_bounds__(2 * B * B) void k_bj_local(const double* __restrict__ C, int32_t m, int32_t r,
                                                    double* __restrict__ Qs, const double* __restrict__ normf,
                                                    double tol_rel, double tol_abs_rel, int32_t max_sweeps,
                                                    int32_t* rot_count, int32_t* __restrict__ qrot) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    bj_local_solve<B>(C, m, r, blockIdx.x, Qs, normf, tol_rel, tol_abs_rel, max_sweeps, rot_count, qrot, smem_raw);
}

// C <- J^T C J on every (pair, pair') tile (pair <= pair'), V <- V J on row
// chunks; first npairs*(npairs+1)/2 workgroups do C, the rest V.  The 2b x 2b
// products run on the FP64 matrix cores: wave w of the workgroup (b^2 / 64
// waves) owns the 16 x 16 output tile (w / (b / 8), w % (b / 8)).  16x16x4 operand layout: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; result item v of lane l is
// D[l / 16 + 4 v][l % 16].
template <int B>
__device__ void bj_apply_item(double* C, double* V, int32_t m, int32_t r, const double* __restrict__ Qs,
                              const int32_t* __restrict__ qrot, double (*X)[2 * B + 1]) {
    constexpr int W = 2 * B, NT = W / 16;   // NT x NT output tiles of 16 x 16, one per wave
    const int nb = m / B, np = nb / 2;
    const int64_t ctiles = (int64_t)np * (np + 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4, ta = w / NT, tc = w % NT;
    if (blockIdx.x < ctiles) {
        int t = blockIdx.x, P = 0;
        while (t >= np - P) { t -= np - P; ++P; }
        const int P2 = P + t;
        if (!qrot[P] && !qrot[P2]) return;   // both factors are the identity
        int I1, J1, I2, J2;
        bj_pair(P, r, nb, I1, J1);
        bj_pair(P2, r, nb, I2, J2);
        const double* q1 = Qs + (int64_t)P * W * W;
        const double* q2 = Qs + (int64_t)P2 * W * W;
        // T = Q1^T X with X the (pair P rows) x (pair P2 columns) block of C
        const int64_t gcol = bj_index<B>(tc * 16 + li, I2, J2);
        dbl4 acc = dbl4{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < W / 4; ++ks) {
            const int l = 4 * ks + lk;
            const double a = q1[l * W + ta * 16 + li];
            const double b = C[(int64_t)bj_index<B>(l, I1, J1) * m + gcol];
            acc = mfma4(a, b, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) X[ta * 16 + lk + 4 * v][tc * 16 + li] = acc[v];
        __syncthreads();
        // out = T Q2, written to the tile and its mirror.  On a diagonal tile
        // (P == P2) entry (i, j) and its mirror (j, i) are two results computed
        // in different rounding orders: only the lower triangle (i >= j) is
        // stored, to both places, so no address gets two different values
        // (which one landed last would depend on the wave schedule)
        acc = dbl4{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < W / 4; ++ks) {
            const int l = 4 * ks + lk;
            acc = mfma4(X[ta * 16 + li][l], q2[l * W + tc * 16 + li], acc);
        }
        const bool diag_tile = P == P2;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int lr = ta * 16 + lk + 4 * v;
            if (diag_tile && lr < tc * 16 + li) continue;
            const int64_t gi = bj_index<B>(lr, I1, J1);
            C[gi * m + gcol] = acc[v];
            C[gcol * m + gi] = acc[v];
        }
    } else {
        // V rows [row0, row0 + W) times Q of pair P (m is a multiple of W)
        const int64_t item = blockIdx.x - ctiles;
        const int P = (int)(item % np);
        if (!qrot[P]) return;
        const int64_t row0 = (item / np) * W;
        int I1, J1;
        bj_pair(P, r, nb, I1, J1);
        const double* q1 = Qs + (int64_t)P * W * W;
        for (int idx = tid; idx < W * W; idx += B * B) {
            const int a = idx / W, c = idx % W;
            X[a][c] = V[(row0 + a) * m + bj_index<B>(c, I1, J1)];
        }
        __syncthreads();
        dbl4 acc = dbl4{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < W / 4; ++ks) {
            const int l = 4 * ks + lk;
            acc = mfma4(X[ta * 16 + li][l], q1[l * W + tc * 16 + li], acc);
        }
        const int64_t gcol = bj_index<B>(tc * 16 + li, I1, J1);
#pragma unroll
        for (int v = 0; v < 4; ++v) V[(row0 + ta * 16 + lk + 4 * v) * m + gcol] = acc[v];
    }
}
template <int B>
__global__ __launch_bounds__(B * B) void k_bj_apply(double* C, double* V, int32_t m, int32_t r,
                                                    const double* __restrict__ Qs, const int32_t* __restrict__ qrot) {
    __shared__ double X[2 * B][2 * B + 1];
    bj_apply_item<B>(C, V, m, r, Qs, qrot, X);
}

// Number of off-diagonal entries of the symmetric m x m matrix C that the
// rotation threshold of k_bj_local would still act on; zero means that a
// further sweep would not rotate at all.
__global__ __launch_bounds__(256) void k_bj_offcount(const double* __restrict__ C, int32_t m,
                                                     const double* __restrict__ normf, double tol_rel,
                                                     double tol_abs_rel, int32_t* count) {
    __shared__ int part[4];
    const double tol_abs2 = tol_abs_rel * normf[0] * tol_abs_rel * normf[0];
    const double tol_rel2 = tol_rel * tol_rel;
    int n = 0;
    // one row p per workgroup at a time, entries q > p over the threads
    for (int32_t p = blockIdx.x; p < m; p += gridDim.x) {
        const double* row = C + (int64_t)p * m;
        const double app = row[p];
        for (int32_t q = p + 1 + (int32_t)threadIdx.x; q < m; q += (int32_t)blockDim.x) {
            const double apq = row[q];
            if (apq * apq > fmax(tol_abs2, tol_rel2 * fabs(app * C[(int64_t)q * m + q]))) ++n;
        }
    }
    // one atomic per workgroup
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(count, t);
    }
}
hipError_t launch_bj_offcount(const double* C, int32_t m, const double* normf, double tol_rel, double tol_abs_rel,
                              int32_t* count, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    k_bj_offcount<<<(unsigned)std::min<int32_t>(m, 1024), 256, 0, s>>>(C, m, normf, tol_rel, tol_abs_rel, count);
    return hipGetLastError();
}

template <int B>
hipError_t bj_sweep(double* C, double* V, int32_t m, double* Qs, const double* normf, double tol_rel,
                    double tol_abs_rel, int32_t inner_sweeps, int32_t* rot_count, int32_t* qrot, hipStream_t s) {
    constexpr size_t lds = bj_local_lds<B>();
    hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_bj_local<B>), lds, 0);
    if (e != hipSuccess) return e;
    const int nb = m / B, np = nb / 2;
    const int64_t ctiles = (int64_t)np * (np + 1) / 2;
    const int64_t vitems = (int64_t)(m / (2 * B)) * np;
    for (int32_t r = 0; r + 1 < nb; ++r) {
        k_bj_local<B><<<np, 2 * B * B, lds, s>>>(C, m, r, Qs, normf, tol_rel, tol_abs_rel, inner_sweeps, rot_count,
                                                 qrot);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_bj_apply<B><<<(unsigned)(ctiles + vitems), B * B, 0, s>>>(C, V, m, r, Qs, qrot);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}
hipError_t launch_bj_sweep(int b, double* C, double* V, int32_t m, double* Qs, const double* normf, double tol_rel,
                           double tol_abs_rel, int32_t inner_sweeps, int32_t* rot_count, int32_t* qrot,
                           hipStream_t s) {
    if (b != 16 || m % (2 * b) != 0 || m < 2 * b) return hipErrorInvalidValue;
    return bj_sweep<16>(C, V, m, Qs, normf, tol_rel, tol_abs_rel, inner_sweeps, rot_count, qrot, s);
}

// V = identity (m x m)
__global__ void k_identity(double* V, int32_t m) {
    const int64_t tot = (int64_t)m * m;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x)
        V[t] = (t / m) == (t % m) ? 1.0 : 0.0;
}
hipError_t launch_identity(double* V, int32_t m, hipStream_t s) {
    k_identity<<<grid_for((int64_t)m * m, 256), 256, 0, s>>>(V, m);
    return hipGetLastError();
}

// (a, i) before (b, j) in ascending order of value, NaN after every number,
// ties by index: a strict total order, so the ranks below are a permutation
// of 0 .. kvalid - 1 whatever the values (every order[j] gets written)
__device__ __forceinline__ bool sort_before(double a, int i, double b, int j) {
    const bool na = a != a, nb = b != b;
    if (na || nb) return na && nb ? i < j : nb;
    return a < b || (a == b && i < j);
}
// ascending order of the diagonal of C (ties by index); X[r, j] = scale[r] Y[r, order[j]]
constexpr int SORT_LDS_MAX = 8192;
__global__ __launch_bounds__(1024) void k_sort_eig(const double* C, int32_t m, int32_t kvalid, const double* Y,
                                                   int32_t rows, const double* scale, int32_t kout, double* lam_out,
                                                   double* X, int64_t ldx) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // the diagonal staged in LDS when it fits (kvalid <= SORT_LDS_MAX)
    const bool staged = kvalid <= SORT_LDS_MAX;
    double* diag = reinterpret_cast<double*>(smem_raw);
    int* order = reinterpret_cast<int*>(smem_raw + (staged ? sizeof(double) * kvalid : 0));   // kout entries
    if (staged)
        for (int i = threadIdx.x; i < kvalid; i += blockDim.x) diag[i] = C[(int64_t)i * m + i];
    __syncthreads();
    auto dg = [&](int j) { return staged ? diag[j] : C[(int64_t)j * m + j]; };
    for (int i = threadIdx.x; i < kvalid; i += blockDim.x) {
        const double li = dg(i);
        int rank = 0;
        for (int j = 0; j < kvalid; ++j) rank += sort_before(dg(j), j, li, i);
        if (rank < kout) {
            order[rank] = i;
            lam_out[rank] = li;
        }
    }
    __syncthreads();
    const int64_t tot = (int64_t)rows * kout;
    for (int64_t t = threadIdx.x; t < tot; t += blockDim.x) {
        const int64_t r = t / kout;
        const int j = (int)(t % kout);
        X[r * ldx + j] = (scale ? scale[r] : 1.0) * Y[r * m + order[j]];
    }
}
hipError_t launch_sort_eig(const double* C, int32_t m, int32_t kvalid, const double* Y, int32_t rows,
                           const double* scale, int32_t kout, double* lam_out, double* X, int64_t ldx, hipStream_t s) {
    if (kout <= 0 || kout > kvalid || kvalid > m) return hipErrorInvalidValue;   // every order[j] must have a source
    const size_t lds = (kvalid <= SORT_LDS_MAX ? (size_t)kvalid * sizeof(double) : 0) + (size_t)kout * sizeof(int);
    hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_sort_eig), lds, 0);
    if (e != hipSuccess) return e;
    k_sort_eig<<<1, 1024, lds, s>>>(C, m, kvalid, Y, rows, scale, kout, lam_out, X, ldx);
    return hipGetLastError();
}

// C (m x m) = Ck (k x k) padded with decoupled dummy rows/columns whose
// diagonal exceeds every eigenvalue; normf[0] = ||Ck||_F; dis = D^-1/2
// (1 on the dummies).  The squares are summed in a fixed order: workgroup b
// over its own range of C's entries (strided over its threads, then a fixed
// tree), the EMBED_WG partial sums by one workgroup.
constexpr int EMBED_WG = 256;
__global__ __launch_bounds__(256) void k_embed_copy(const double* Ck, int32_t k, int32_t m, double* C, double* part) {
    __shared__ double red[256];
    const int64_t tot = (int64_t)m * m, chunk = (tot + gridDim.x - 1) / gridDim.x;
    const int64_t t0 = blockIdx.x * chunk, t1 = min(tot, t0 + chunk);
    double sq = 0.0;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
        const int32_t i = (int32_t)(t / m), j = (int32_t)(t % m);
        const double v = (i < k && j < k) ? Ck[(int64_t)i * k + j] : 0.0;
        C[t] = v;
        sq += v * v;
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(256) void k_embed_finish(const double* part, int32_t k, int32_t m, double* C,
                                                      double* normf, double* dis, const double* D) {
    __shared__ double red[256];
    red[threadIdx.x] = part[threadIdx.x];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double nf = sqrt(red[0]);
    if (threadIdx.x == 0) normf[0] = nf;
    for (int i = k + threadIdx.x; i < m; i += blockDim.x) C[(int64_t)i * m + i] = 4.0 * nf + 1.0 + i;
    for (int i = threadIdx.x; i < m; i += blockDim.x) dis[i] = i < k ? 1.0 / sqrt(D[i]) : 1.0;
}
hipError_t launch_embed_pad(const double* Ck, int32_t k, int32_t m, double* C, double* normf, double* dis,
                            const double* D, double* part, hipStream_t s) {
    k_embed_copy<<<EMBED_WG, 256, 0, s>>>(Ck, k, m, C, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_embed_finish<<<1, 256, 0, s>>>(part, k, m, C, normf, dis, D);
    return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<grid_for(n, 256), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

// dense n x n row-major copy of a CSR matrix
__global__ void k_densify(const int64_t* ptr, const int32_t* idx, const double* val, int64_t n, double* A) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) A[r * n + idx[e]] = val[e];
}
hipError_t launch_densify(const int64_t* ptr, const int32_t* idx, const double* val, int64_t n, double* A,
                          hipStream_t s) {
    hipError_t e = launch_fill(A, n * n, 0.0, s);
    if (e != hipSuccess) return e;
    k_densify<<<grid_for(n, 256), 256, 0, s>>>(ptr, idx, val, n, A);
    return hipGetLastError();
}

// per column c in [col0, col0 + k): num[c] = ||R_c||^2, den[c] = ||B_c||^2 (partial sums by row chunks)
__global__ __launch_bounds__(256) void k_colnorm2(const double* __restrict__ R, const double* __restrict__ B,
                                                  int64_t n, int64_t ld, int32_t col0, int32_t k, int64_t chunk,
                                                  double* __restrict__ partial) {
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int lane_row = threadIdx.x >> 6;   // 4 row lanes
    const int64_t r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
    double a = 0, b = 0;
    if (c < k) {
        for (int64_t r = r0 + lane_row; r < r1; r += 4) {
            const double x = R[r * ld + col0 + c], y = B[r * ld + col0 + c];
            a += x * x;
            b += y * y;
        }
    }
    __shared__ double sa[4][64], sb[4][64];
    sa[lane_row][threadIdx.x & 63] = a;
    sb[lane_row][threadIdx.x & 63] = b;
    __syncthreads();
    if (threadIdx.x < 64 && c < k) {
        double ta = 0, tb = 0;
        for (int l = 0; l < 4; ++l) {
            ta += sa[l][threadIdx.x];
            tb += sb[l][threadIdx.x];
        }
        partial[(int64_t)blockIdx.x * 2 * k + c] = ta;
        partial[(int64_t)blockIdx.x * 2 * k + k + c] = tb;
    }
}
__global__ void k_colnorm_ratio(const double* __restrict__ partial, int64_t nch, int32_t k, double* ratio) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= k) return;
    double a = 0, b = 0;
    for (int64_t ch = 0; ch < nch; ++ch) {
        a += partial[ch * 2 * k + c];
        b += partial[ch * 2 * k + k + c];
    }
    ratio[c] = b > 0 ? sqrt(a / b) : sqrt(a);
}
int64_t colnorm_partial_doubles(int64_t n, int32_t k) { return cdiv(n, 16384) * 2 * (int64_t)k; }
hipError_t launch_colnorm_ratio(const double* R, const double* B, int64_t n, int64_t ld, int32_t col0, int32_t k,
                                double* partial, double* ratio, hipStream_t s) {
    if (k <= 0 || n <= 0) return hipSuccess;
    const int64_t chunk = 16384, nch = cdiv(n, chunk);
    k_colnorm2<<<dim3((unsigned)nch, (unsigned)cdiv(k, 64)), 256, 0, s>>>(R, B, n, ld, col0, k, chunk, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_colnorm_ratio<<<(unsigned)cdiv(k, 256), 256, 0, s>>>(partial, nch, k, ratio);
    return hipGetLastError();
}

// ============================================================ tall-skinny products (adjoint solve)
// C (ka x kb, row-major) = A^T B for n-row blocks A (lda), B (ldb): partial
// sums over row chunks for each 32 x 32 output tile, then a fixed-order sum.
int64_t tsgemm_partial_doubles(int64_t n, int32_t ka, int32_t kb) {
    return cdiv(n, 4096) * cdiv(ka, T32) * cdiv(kb, T32) * TT;
}
__global__ __launch_bounds__(256) void k_tsgemm_tn_partial(const double* __restrict__ A, int64_t lda,
                                                           const double* __restrict__ B, int64_t ldb, int64_t n,
                                                           int32_t ka, int32_t kb, int64_t chunk, double* partial) {
    const int ta = blockIdx.y / ((kb + T32 - 1) / T32), tb = blockIdx.y % ((kb + T32 - 1) / T32);
    const int64_t r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
    __shared__ double P[T32][T32 + 1], Q[T32][T32 + 1];
    const int tid = threadIdx.x, r = tid & 31;
    double acc[4] = {0, 0, 0, 0};
    for (int64_t row0 = r0; row0 < r1; row0 += T32) {
        for (int idx = tid; idx < TT; idx += 256) {
            const int i = idx >> 5, c = idx & 31;
            const int64_t row = row0 + i;
            const int ca = ta * T32 + c, cb = tb * T32 + c;
            P[i][c] = (row < r1 && ca < ka) ? A[row * lda + ca] : 0.0;
            Q[i][c] = (row < r1 && cb < kb) ? B[row * ldb + cb] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int c = (tid >> 5) + 8 * o;
            double v = 0;
#pragma unroll 8
            for (int i = 0; i < T32; ++i) v += P[i][r] * Q[i][c];
            acc[o] += v;
        }
        __syncthreads();
    }
    double* out = partial + ((int64_t)blockIdx.x * gridDim.y + blockIdx.y) * TT;
#pragma unroll
    for (int o = 0; o < 4; ++o) out[r * T32 + (tid >> 5) + 8 * o] = acc[o];
}
__global__ void k_tsgemm_tn_reduce(const double* __restrict__ partial, int64_t nch, int32_t ka, int32_t kb, double* C) {
    const int ntb = (kb + T32 - 1) / T32;
    const int64_t ntiles = (int64_t)((ka + T32 - 1) / T32) * ntb;
    const int64_t tot = (int64_t)ka * kb;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / kb), j = (int)(t % kb);
        const int64_t tile = (int64_t)(i / T32) * ntb + j / T32;
        double v = 0;
        for (int64_t ch = 0; ch < nch; ++ch) v += partial[(ch * ntiles + tile) * TT + (i % T32) * T32 + j % T32];
        C[t] = v;
    }
}
hipError_t launch_tsgemm_tn(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t n, int32_t ka,
                            int32_t kb, double* partial, double* C, hipStream_t s) {
    if (ka <= 0 || kb <= 0) return hipSuccess;
    const int64_t chunk = 4096, nch = cdiv(n, chunk);
    const unsigned tiles = (unsigned)(cdiv(ka, T32) * cdiv(kb, T32));
    k_tsgemm_tn_partial<<<dim3((unsigned)nch, tiles), 256, 0, s>>>(A, lda, B, ldb, n, ka, kb, chunk, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_tsgemm_tn_reduce<<<grid_for((int64_t)ka * kb, 256), 256, 0, s>>>(partial, nch, ka, kb, C);
    return hipGetLastError();
}
// Y = beta Y + alpha A C for A (n x ka, lda), C (ka x kb row-major), Y (n x kb, ldy)
__global__ __launch_bounds__(256) void k_tsgemm_nn(const double* __restrict__ A, int64_t lda, int64_t n, int32_t ka,
                                                   const double* __restrict__ Cm, int32_t kb, double alpha, double beta,
                                                   double* __restrict__ Y, int64_t ldy, int64_t chunk) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* Cs = reinterpret_cast<double*>(smem_raw);   // ka x 32
    const int tid = threadIdx.x, cl = tid & 31, rl = tid >> 5;
    const int col = blockIdx.y * T32 + cl;
    for (int idx = tid; idx < ka * T32; idx += 256) {
        const int kk = idx >> 5, c = blockIdx.y * T32 + (idx & 31);
        Cs[idx] = c < kb ? Cm[(int64_t)kk * kb + c] : 0.0;
    }
    __syncthreads();
    if (col >= kb) return;
    const int64_t r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
    for (int64_t row = r0 + rl; row < r1; row += 8) {
        const double* ar = A + row * lda;
        double v = 0;
        for (int kk = 0; kk < ka; ++kk) v += ar[kk] * Cs[kk * T32 + cl];
        double* y = Y + row * ldy + col;
        *y = (beta == 0.0 ? 0.0 : beta * *y) + alpha * v;
    }
}
hipError_t launch_tsgemm_nn(const double* A, int64_t lda, int64_t n, int32_t ka, const double* C, int32_t kb,
                            double alpha, double beta, double* Y, int64_t ldy, hipStream_t s) {
    if (kb <= 0 || n <= 0) return hipSuccess;
    const int64_t chunk = 2048;
    const size_t lds = (size_t)ka * T32 * sizeof(double);
    hipError_t e0 = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_tsgemm_nn), lds, 0);
    if (e0 != hipSuccess) return e0;
    k_tsgemm_nn<<<dim3((unsigned)cdiv(n, chunk), (unsigned)cdiv(kb, T32)), 256, lds, s>>>(A, lda, n, ka, C, kb, alpha,
                                                                                           beta, Y, ldy, chunk);
    return hipGetLastError();
}
// out[c] = sum_r A[r, c] B[r, c], c < k
__global__ __launch_bounds__(256) void k_coldot_partial(const double* __restrict__ A, const double* __restrict__ B,
                                                        int64_t n, int64_t ld, int32_t k, int64_t chunk,
                                                        double* __restrict__ partial) {
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int lr = threadIdx.x >> 6;
    const int64_t r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
    double a = 0;
    if (c < k)
        for (int64_t r = r0 + lr; r < r1; r += 4) a += A[r * ld + c] * B[r * ld + c];
    __shared__ double sa[4][64];
    sa[lr][threadIdx.x & 63] = a;
    __syncthreads();
    if (threadIdx.x < 64 && c < k) partial[(int64_t)blockIdx.x * k + c] = sa[0][threadIdx.x] + sa[1][threadIdx.x] +
                                                                          sa[2][threadIdx.x] + sa[3][threadIdx.x];
}
__global__ void k_coldot_reduce(const double* __restrict__ partial, int64_t nch, int32_t k, double* out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= k) return;
    double a = 0;
    for (int64_t ch = 0; ch < nch; ++ch) a += partial[ch * k + c];
    out[c] = a;
}
int64_t coldot_partial_doubles(int64_t n, int32_t k) { return cdiv(n, 16384) * (int64_t)k; }
hipError_t launch_coldot(const double* A, const double* B, int64_t n, int64_t ld, int32_t k, double* partial,
                         double* out, hipStream_t s) {
    if (k <= 0 || n <= 0) return hipSuccess;
    const int64_t chunk = 16384, nch = cdiv(n, chunk);
    k_coldot_partial<<<dim3((unsigned)nch, (unsigned)cdiv(k, 64)), 256, 0, s>>>(A, B, n, ld, k, chunk, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_coldot_reduce<<<(unsigned)cdiv(k, 256), 256, 0, s>>>(partial, nch, k, out);
    return hipGetLastError();
}
// Y[r, c] -= m[r] lam[c] X[r, c]
__global__ void k_shift_cols(double* Y, const double* X, const double* m, const double* lam, int64_t n, int64_t ld,
                             int32_t k) {
    const int64_t tot = n * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / k;
        const int c = (int)(t % k);
        Y[r * ld + c] -= m[r] * lam[c] * X[r * ld + c];
    }
}
hipError_t launch_shift_cols(double* Y, const double* X, const double* m, const double* lam, int64_t n, int64_t ld,
                             int32_t k, hipStream_t s) {
    if (n <= 0 || k <= 0) return hipSuccess;
    k_shift_cols<<<grid_for(n * k, 256), 256, 0, s>>>(Y, X, m, lam, n, ld, k);
    return hipGetLastError();
}
// mode 0: Y += coef[c] X ; mode 1: Y -= coef[c] X ; mode 2: Y = X + coef[c] Y
__global__ void k_axpy_cols(double* Y, const double* X, const double* coef, int mode, int64_t n, int64_t ld, int32_t k) {
    const int64_t tot = n * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / k;
        const int c = (int)(t % k);
        double* y = Y + r * ld + c;
        const double x = X[r * ld + c];
        if (mode == 0) *y += coef[c] * x;
        else if (mode == 1) *y -= coef[c] * x;
        else *y = x + coef[c] * *y;
    }
}
hipError_t launch_axpy_cols(double* Y, const double* X, const double* coef, int mode, int64_t n, int64_t ld, int32_t k,
                            hipStream_t s) {
    if (n <= 0 || k <= 0) return hipSuccess;
    k_axpy_cols<<<grid_for(n * k, 256), 256, 0, s>>>(Y, X, coef, mode, n, ld, k);
    return hipGetLastError();
}
// out[c] = (den[c] != 0) ? num[c] / den[c] : 0
__global__ void k_div_cols(const double* num, const double* den, double* out, int32_t k) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < k) out[c] = den[c] != 0.0 ? num[c] / den[c] : 0.0;
}
hipError_t launch_div_cols(const double* num, const double* den, double* out, int32_t k, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    k_div_cols<<<(unsigned)cdiv(k, 256), 256, 0, s>>>(num, den, out, k);
    return hipGetLastError();
}

// ============================================================ assembly derivative (vertex positions)
// Per vertex (mesh order): nu_i = rho_i sum_k [ -lam_k glam_k x_ki^2 + lam_k w_ki x_ki - y_ki x_ki / 2 ],
// the coefficient of the lumped-mass derivative (Y = X_cluster Gamma carries
// the normalisation terms).  iperm[v] < 0 marks a vertex without a row (the
// boundary under the Dirichlet condition): its values are zero, so nu_v = 0.
__global__ void k_bwd_vertex(int64_t nv, int32_t p, const double* __restrict__ X, const double* __restrict__ W,
                             const double* __restrict__ Y, int64_t ld, const int32_t* __restrict__ iperm,
                             const double* __restrict__ lam, const double* __restrict__ glam,
                             const double* __restrict__ rho, double* __restrict__ nu) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = iperm[v];
        double s = 0;
        for (int k = 0; r >= 0 && k < p; ++k) {
            const double x = X[r * ld + k];
            double t = 0;
            if (glam) t -= lam[k] * glam[k] * x * x;
            if (W) t += lam[k] * W[r * ld + k] * x;
            if (Y) t -= 0.5 * Y[r * ld + k] * x;
            s += t;
        }
        nu[v] = (rho ? rho[v] : 1.0) * s;
    }
}
hipError_t launch_bwd_vertex(int64_t nv, int32_t p, const double* X, const double* W, const double* Y, int64_t ld,
                             const int32_t* iperm, const double* lam, const double* glam, const double* rho, double* nu,
                             hipStream_t s) {
    k_bwd_vertex<<<grid_for(nv, 256), 256, 0, s>>>(nv, p, X, W, Y, ld, iperm, lam, glam, rho, nu);
    return hipGetLastError();
}

__device__ __forceinline__ void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Per triangle: derivative of sum over corners of (1/2) e_opp cot(theta) plus
// (nu_a + nu_b + nu_c)/3 * area, with e_opp = sum_k [glam_k (x_i - x_j)^2 -
// (w_i - w_j)(x_i - x_j)] over the edge opposite the corner.  G[t][corner][xyz].
// A corner whose vertex has no row (iperm < 0) has x = w = 0: the zero extension
// of the interior problem's vectors under the Dirichlet condition.  The mass
// term is nu times the derivative of the lumped masses: area / 3 per vertex
// (lumping 0), or, circumcentric (lumping 1), each corner's cot(theta) |e|^2 / 8
// over its opposite edge e to both ends of e.
__global__ void k_bwd_tri(int64_t nf, const int32_t* __restrict__ F, const double* __restrict__ V, int32_t p,
                          const double* __restrict__ X, const double* __restrict__ W, int64_t ld,
                          const int32_t* __restrict__ iperm, const double* __restrict__ glam,
                          const double* __restrict__ nu, int32_t lumping, double* __restrict__ G) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nf; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t vi[3] = {F[3 * t], F[3 * t + 1], F[3 * t + 2]};
        const int64_t ri[3] = {iperm[vi[0]], iperm[vi[1]], iperm[vi[2]]};
        double P[3][3];
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) P[a][d] = V[3 * (int64_t)vi[a] + d];
        double e[3] = {0, 0, 0};   // per corner: its opposite edge
        for (int k = 0; k < p; ++k) {
            double xs[3] = {0, 0, 0}, ws[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a)
                if (ri[a] >= 0) {
                    xs[a] = X[ri[a] * ld + k];
                    if (W) ws[a] = W[ri[a] * ld + k];
                }
            const double g = glam ? glam[k] : 0.0;
            for (int c = 0; c < 3; ++c) {
                const int i = (c + 1) % 3, j = (c + 2) % 3;
                const double dx = xs[i] - xs[j], dw = ws[i] - ws[j];
                e[c] += g * dx * dx - dw * dx;
            }
        }
        double grad[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int c = 0; c < 3; ++c) {
            const int i = (c + 1) % 3, j = (c + 2) % 3;
            double u[3], w[3], cr[3];
            for (int d = 0; d < 3; ++d) { u[d] = P[i][d] - P[c][d]; w[d] = P[j][d] - P[c][d]; }
            cross3(u, w, cr);
            const double dot = u[0] * w[0] + u[1] * w[1] + u[2] * w[2];
            const double s2 = cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2];
            const double sn = sqrt(s2);
            double wc[3], cu[3];
            cross3(w, cr, wc);
            cross3(cr, u, cu);
            double f = 0.5 * e[c];
            if (lumping == 1) {
                // nu-weighted derivative of cot(theta_c) |P_i - P_j|^2 / 8 (to m_i and m_j)
                const double mc = 0.125 * (nu[vi[i]] + nu[vi[j]]);
                double dij[3];
                for (int d = 0; d < 3; ++d) dij[d] = P[i][d] - P[j][d];
                f += mc * (dij[0] * dij[0] + dij[1] * dij[1] + dij[2] * dij[2]);
                const double gl = 2.0 * mc * dot / sn;
                for (int d = 0; d < 3; ++d) {
                    grad[i][d] += gl * dij[d];
                    grad[j][d] -= gl * dij[d];
                }
            }
            for (int d = 0; d < 3; ++d) {
                const double du = w[d] / sn - dot * wc[d] / (s2 * sn);   // d cot / d u
                const double dw = u[d] / sn - dot * cu[d] / (s2 * sn);   // d cot / d w
                grad[i][d] += f * du;
                grad[j][d] += f * dw;
                grad[c][d] -= f * (du + dw);
            }
        }
        // barycentric mass term: nu times the derivative of area / 3
        if (lumping == 0) {
            double e1[3], e2[3], cr[3], a1[3], a2[3];
            for (int d = 0; d < 3; ++d) { e1[d] = P[1][d] - P[0][d]; e2[d] = P[2][d] - P[0][d]; }
            cross3(e1, e2, cr);
            const double sn = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
            cross3(e2, cr, a1);
            cross3(cr, e1, a2);
            const double f = (nu[vi[0]] + nu[vi[1]] + nu[vi[2]]) / 3.0 * 0.5 / sn;
            for (int d = 0; d < 3; ++d) {
                grad[1][d] += f * a1[d];
                grad[2][d] += f * a2[d];
                grad[0][d] -= f * (a1[d] + a2[d]);
            }
        }
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) G[9 * t + 3 * a + d] = grad[a][d];
    }
}
hipError_t launch_bwd_tri(int64_t nf, const int32_t* F, const double* V, int32_t p, const double* X, const double* W,
                          int64_t ld, const int32_t* iperm, const double* glam, const double* nu, int32_t lumping,
                          double* G, hipStream_t s) {
    if (lumping != 0 && lumping != 1) return hipErrorInvalidValue;
    k_bwd_tri<<<grid_for(nf, 256), 256, 0, s>>>(nf, F, V, p, X, W, ld, iperm, glam, nu, lumping, G);
    return hipGetLastError();
}
// gradV[v] = sum over the (triangle, corner) entries listed for v, in list order
__global__ void k_bwd_gather(int64_t nv, const int64_t* __restrict__ vt_ptr, const int64_t* __restrict__ vt,
                             const double* __restrict__ G, double* __restrict__ gradV) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        double g[3] = {0, 0, 0};
        for (int64_t e = vt_ptr[v]; e < vt_ptr[v + 1]; ++e)
            for (int d = 0; d < 3; ++d) g[d] += G[3 * vt[e] + d];
        for (int d = 0; d < 3; ++d) gradV[3 * v + d] = g[d];
    }
}
hipError_t launch_bwd_gather(int64_t nv, const int64_t* vt_ptr, const int64_t* vt, const double* G, double* gradV,
                             hipStream_t s) {
    k_bwd_gather<<<grid_for(nv, 256), 256, 0, s>>>(nv, vt_ptr, vt, G, gradV);
    return hipGetLastError();
}
// out[r, c] = in[c * nv + perm[r]] for r < n, c < k (column-major mesh order -> row-major internal order)
__global__ void k_import_cols(const double* in, int64_t nv, const int32_t* perm, int64_t n, int32_t k, double* out,
                              int64_t ld, const double* sign) {
    const int64_t tot = n * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t % n;
        const int c = (int)(t / n);
        out[r * ld + c] = (sign ? sign[c] : 1.0) * in[(int64_t)c * nv + perm[r]];
    }
}
hipError_t launch_import_cols(const double* in, int64_t nv, const int32_t* perm, int64_t n, int32_t k, double* out,
                              int64_t ld, hipStream_t s, const double* sign) {
    if (n <= 0 || k <= 0) return hipSuccess;
    k_import_cols<<<grid_for(n * k, 256), 256, 0, s>>>(in, nv, perm, n, k, out, ld, sign);
    return hipGetLastError();
}

// ============================================================ output
// per column: the row with the largest |value|, lowest vertex index on ties
// per (chunk of rows, column): the entry of largest magnitude (lowest vertex
// index on ties).  A workgroup takes one chunk and 128 columns: thread
// (column lane, row lane) reads rows r0 + row lane + 8 k, so that every row
// read is 128 consecutive values
__global__ __launch_bounds__(1024) void k_col_argmax(const double* Phi, int64_t ld, int64_t n, int32_t p,
                                                     const int32_t* perm, int64_t chunk, double* pv, int64_t* pi) {
    const int cl = threadIdx.x & 127, rl = threadIdx.x >> 7;
    const int c = blockIdx.y * 128 + cl;
    const int64_t r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
    double best = -1.0, bv = 0.0;
    int64_t bi = INT64_MAX;
    if (c < p) {
#pragma unroll 4
        for (int64_t r = r0 + rl; r < r1; r += 8) {
            const double v = Phi[r * ld + c];
            const int64_t vi = perm ? perm[r] : r;
            const double a = fabs(v);
            if (a > best || (a == best && vi < bi)) {
                best = a;
                bi = vi;
                bv = v;
            }
        }
    }
    __shared__ double sb[8][128], sv[8][128];
    __shared__ int64_t si[8][128];
    sb[rl][cl] = best;
    si[rl][cl] = bi;
    sv[rl][cl] = bv;
    __syncthreads();
    if (rl == 0 && c < p) {
        for (int k = 1; k < 8; ++k)
            if (sb[k][cl] > best || (sb[k][cl] == best && si[k][cl] < bi)) {
                best = sb[k][cl];
                bi = si[k][cl];
                bv = sv[k][cl];
            }
        pv[(int64_t)c * gridDim.x + blockIdx.x] = best >= 0 ? (bv < 0 ? -best : best) : 0.0;
        pi[(int64_t)c * gridDim.x + blockIdx.x] = bi;
    }
}
__global__ void k_col_sign(const double* pv, const int64_t* pi, int64_t nch, int32_t p, double* sign) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p) return;
    double best = -1.0, bv = 1.0;
    int64_t bi = INT64_MAX;
    for (int64_t k = 0; k < nch; ++k) {
        const double v = pv[(int64_t)c * nch + k];
        const double a = fabs(v);
        const int64_t vi = pi[(int64_t)c * nch + k];
        if (a > best || (a == best && vi < bi)) { best = a; bi = vi; bv = v; }
    }
    sign[c] = bv < 0 ? -1.0 : 1.0;
}
// evecs[c * nout + perm[r]] = sign[c] * Phi[r, c]: tiles of 32 rows x 32 columns through LDS
__global__ __launch_bounds__(256) void k_export(const double* Phi, int64_t ld, int64_t n, int32_t p,
                                                const int32_t* perm, int64_t nout, const double* sign,
                                                double* evecs) {
    __shared__ double t[T32][T32 + 1];
    const int64_t r0 = blockIdx.x * (int64_t)T32;
    const int c0 = blockIdx.y * T32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int yy = ty; yy < T32; yy += 8) {
        const int64_t r = r0 + yy;
        const int c = c0 + tx;
        t[yy][tx] = (r < n && c < p) ? Phi[r * ld + c] : 0.0;
    }
    __syncthreads();
    for (int yy = ty; yy < T32; yy += 8) {
        const int c = c0 + yy;
        const int64_t r = r0 + tx;
        if (r < n && c < p) {
            const int64_t v = perm ? perm[r] : r;
            evecs[(int64_t)c * nout + v] = sign[c] * t[tx][yy];
        }
    }
}
hipError_t launch_export_evecs(const double* Phi, int64_t ld, int64_t n, int32_t p, const int32_t* perm,
                               int64_t nout, double* evecs, double* work, hipStream_t s) {
    const int64_t chunk = 8192;
    const int64_t nch = cdiv(n, chunk);
    double* pv = work;
    int64_t* pi = reinterpret_cast<int64_t*>(work + nch * p);
    double* sign = work + 2 * nch * p;
    k_col_argmax<<<dim3((unsigned)nch, (unsigned)cdiv(p, 128)), 1024, 0, s>>>(Phi, ld, n, p, perm, chunk, pv, pi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_col_sign<<<(unsigned)cdiv(p, 256), 256, 0, s>>>(pv, pi, nch, p, sign);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_export<<<dim3((unsigned)cdiv(n, T32), (unsigned)cdiv(p, T32)), 256, 0, s>>>(Phi, ld, n, p, perm, nout, sign,
                                                                                   evecs);
    return hipGetLastError();
}

// ============================================================ dense products
// Out (M x N) = alpha op(A) B + beta D, row-major with leading dimensions;
// op(A) = A (A stored M x K) or A^T (A stored K x M); D may be null (beta
// ignored) or equal to Out.  FP64 matrix cores: a workgroup of eight waves
// (two per SIMD) takes a 64 x 64 output tile, waves w and w + 4 the 32 x 32
// quarter w (2 x 2 tiles of the 16 x 16 x 4 product) over the two halves of
// every stage's contraction; the contraction goes through LDS 64 at a time in
// two buffers (one barrier per stage), the next 64 loaded into registers while
// the current ones are multiplied, and the two halves' sums are added in a
// fixed order at the end, so results are reproducible.
namespace {
constexpr int DG_T = 64;   // output tile
constexpr int DG_K = 64;   // contraction per stage
constexpr int DG_W = 8;    // waves per workgroup (two per SIMD)
constexpr int DG_AS = DG_K + 1, DG_BS = DG_T + 2;   // LDS row strides
constexpr size_t dgemm_lds() { return 2 * (size_t)(DG_T * DG_AS + DG_K * DG_BS) * sizeof(double); }
}  // namespace
// FULL: M, N and K are multiples of 64 (no bounds checks in the loads)
template <bool FULL, bool transa>
__global__ __launch_bounds__(64 * DG_W) void k_dgemm(int64_t M, int64_t N, int64_t K, double alpha,
                                                    const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ B, int64_t ldb, double beta,
                                                    const double* D, int64_t ldd, double* Out, int64_t ldo) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* lds = reinterpret_cast<double*>(smem_raw);
    // buffer b: As[i][kk] = op(A)[i0 + i][k0 + kk] at lds + b * BUF, Bs[kk][j] after it
    constexpr int BUF = DG_T * DG_AS + DG_K * DG_BS;
    constexpr int NT = 64 * DG_W;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int64_t i0 = (int64_t)blockIdx.y * DG_T, j0 = (int64_t)blockIdx.x * DG_T;
    // waves w and w + 4 share the 32 x 32 quarter w % 4 and take the two halves
    // of every stage's contraction
    const int wq = w & 3, kh = (w >> 2) * (DG_K / 2);
    const int wr = (wq >> 1) * 32, wc = (wq & 1) * 32;
    constexpr int PE = DG_T * DG_K / NT;   // values of each operand per thread
    constexpr int RSTEP = NT / 64;         // stage rows per load step
    double ra[PE], rb[PE];
    // FULL: thread (w, lane) loads rows w + RSTEP e of the stage, element lane
    const double* pa = !transa ? A + (i0 + w) * lda + lane : A + (int64_t)w * lda + i0 + lane;
    const double* pb = B + (int64_t)w * ldb + j0 + lane;
    auto fetch = [&](int64_t k0) {
        if (FULL) {
#pragma unroll
            for (int e = 0; e < PE; ++e) {
                ra[e] = !transa ? pa[(int64_t)(RSTEP * e) * lda + k0] : pa[(k0 + RSTEP * e) * lda];
                rb[e] = pb[(k0 + RSTEP * e) * ldb];
            }
            return;
        }
#pragma unroll
        for (int e = 0; e < PE; ++e) {
            const int idx = tid + NT * e;
            if (!transa) {
                const int i = idx / DG_K, kk = idx % DG_K;
                ra[e] = (i0 + i < M && k0 + kk < K) ? A[(i0 + i) * lda + k0 + kk] : 0.0;
            } else {
                const int kk = idx / DG_T, i = idx % DG_T;
                ra[e] = (i0 + i < M && k0 + kk < K) ? A[(k0 + kk) * lda + i0 + i] : 0.0;
            }
            const int kk = idx / DG_T, j = idx % DG_T;
            rb[e] = (k0 + kk < K && j0 + j < N) ? B[(k0 + kk) * ldb + j0 + j] : 0.0;
        }
    };
    auto stash = [&](int b) {
        double* As = lds + b * BUF;
        double* Bs = As + DG_T * DG_AS;
#pragma unroll
        for (int e = 0; e < PE; ++e) {
            const int idx = tid + NT * e;
            if (!transa)
                As[(idx / DG_K) * DG_AS + idx % DG_K] = ra[e];
            else
                As[(idx % DG_T) * DG_AS + idx / DG_T] = ra[e];
            Bs[(idx / DG_T) * DG_BS + idx % DG_T] = rb[e];
        }
    };
    dbl4 acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[t][0] = acc[t][1] = dbl4{0, 0, 0, 0};
    const int64_t nk = (K + DG_K - 1) / DG_K;
    fetch(0);
    stash(0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) fetch((kt + 1) * DG_K);
        const double* As = lds + (kt & 1) * BUF;
        const double* Bs = As + DG_T * DG_AS;
#pragma unroll
        for (int ks = 0; ks < DG_K / 8; ++ks) {
            const int kc = kh + 4 * ks + lk;
            const double a0 = As[(wr + li) * DG_AS + kc], a1 = As[(wr + 16 + li) * DG_AS + kc];
            const double b0 = Bs[kc * DG_BS + wc + li], b1 = Bs[kc * DG_BS + wc + 16 + li];
            acc[0][0] = mfma4(a0, b0, acc[0][0]);
            acc[0][1] = mfma4(a0, b1, acc[0][1]);
            acc[1][0] = mfma4(a1, b0, acc[1][0]);
            acc[1][1] = mfma4(a1, b1, acc[1][1]);
        }
        // the other buffer was last read before the previous barrier
        if (kt + 1 < nk) stash((int)((kt + 1) & 1));
        __syncthreads();
    }
    // the upper waves' partial sums through LDS (free after the last barrier),
    // added by the lower waves in a fixed order
    dbl4* red = reinterpret_cast<dbl4*>(smem_raw);
    if (w >= 4) {
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u) red[((wq * 2 + t) * 2 + u) * 64 + lane] = acc[t][u];
    }
    __syncthreads();
    if (w >= 4) return;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const dbl4 o = red[((wq * 2 + t) * 2 + u) * 64 + lane];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = i0 + wr + 16 * t + lk + 4 * v, j = j0 + wc + 16 * u + li;
                if (i < M && j < N) {
                    double r = alpha * (acc[t][u][v] + o[v]);
                    if (D) r += beta * D[i * ldd + j];
                    Out[i * ldo + j] = r;
                }
            }
        }
}
hipError_t launch_dgemm(bool transa, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                        const double* B, int64_t ldb, double beta, const double* D, int64_t ldd, double* Out,
                        int64_t ldo, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (K < 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)cdiv(N, DG_T), (unsigned)cdiv(M, DG_T));
    const bool full = M % DG_T == 0 && N % DG_T == 0 && K % DG_K == 0 && K > 0;
    auto go = [&](auto kern) {
        hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(kern), dgemm_lds(), 0);
        if (e != hipSuccess) return e;
        kern<<<grid, 64 * DG_W, dgemm_lds(), s>>>(M, N, K, alpha, A, lda, B, ldb, beta, D, ldd, Out, ldo);
        return hipSuccess;
    };
    hipError_t e;
    if (full)
        e = transa ? go(&k_dgemm<true, true>) : go(&k_dgemm<true, false>);
    else
        e = transa ? go(&k_dgemm<false, true>) : go(&k_dgemm<false, false>);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// ------------------------------------------------ spectral projection helpers
// Gershgorin bound of C - sigma I over the leading k x k block of the m x m C:
// max over rows i < k of |c_ii - sigma| + sum_{j != i, j < k} |c_ij|.  One wave
// per row; the maximum goes through an atomic on the bit pattern (the bound
// is non-negative, and non-negative doubles order like their bits), so the
// result does not depend on the order of the rows.
__global__ __launch_bounds__(256) void k_ns_bound(const double* __restrict__ C, int32_t m, int32_t k, double sigma,
                                                  unsigned long long* bound) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= k) return;
    double sum = 0.0;
    for (int32_t j = lane; j < k; j += 64) sum += fabs(C[i * m + j] - (j == i ? sigma : 0.0));
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    if (lane == 0) atomicMax(bound, (unsigned long long)__double_as_longlong(sum));
}
// X = (sigma I - C) / g on the leading k x k block (g: the bound above), -1 on
// the diagonal of the decoupled dummies, 0 elsewhere
__global__ void k_ns_init(const double* __restrict__ C, int32_t m, int32_t k, double sigma,
                          const unsigned long long* __restrict__ bound, double* X) {
    const double g = __longlong_as_double((long long)*bound);
    const double ginv = g > 0 ? 1.0 / g : 1.0;
    const int64_t tot = (int64_t)m * m;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = (int32_t)(t / m), j = (int32_t)(t % m);
        double v;
        if (i < k && j < k)
            v = ((i == j ? sigma : 0.0) - C[t]) * ginv;
        else
            v = i == j ? -1.0 : 0.0;
        X[t] = v;
    }
}
hipError_t launch_ns_init(const double* C, int32_t m, int32_t k, double sigma, unsigned long long* bound, double* X,
                          hipStream_t s) {
    if (k <= 0 || k > m) return hipErrorInvalidValue;
    hipError_t e = launch_fill(reinterpret_cast<double*>(bound), 1, 0.0, s);   // +0.0: all bits zero
    if (e != hipSuccess) return e;
    k_ns_bound<<<(unsigned)cdiv(k, 4), 256, 0, s>>>(C, m, k, sigma, bound);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_ns_init<<<grid_for((int64_t)m * m, 256), 256, 0, s>>>(C, m, k, sigma, bound, X);
    return hipGetLastError();
}
// out[0] = sum over the m x m T of (t_ij - delta_ij)^2, out[1] = sum_{i < k}
// x_ii; fixed-order sums (workgroup b over its own range, then one workgroup)
constexpr int NSRED_WG = 256;
__global__ __launch_bounds__(256) void k_ns_dev_part(const double* __restrict__ T, int32_t m, double* part) {
    __shared__ double red[256];
    const int64_t tot = (int64_t)m * m, chunk = (tot + gridDim.x - 1) / gridDim.x;
    const int64_t t0 = blockIdx.x * chunk, t1 = min(tot, t0 + chunk);
    double sq = 0.0;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
        const double d = T[t] - ((t / m) == (t % m) ? 1.0 : 0.0);
        sq += d * d;
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(256) void k_ns_finish(const double* __restrict__ part, const double* __restrict__ X,
                                                   int32_t m, int32_t k, double* out) {
    __shared__ double red[256], tr[256];
    red[threadIdx.x] = part[threadIdx.x];
    double t = 0.0;
    if (X)
        for (int32_t i = threadIdx.x; i < k; i += blockDim.x) t += X[(int64_t)i * m + i];
    tr[threadIdx.x] = t;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[threadIdx.x] += red[threadIdx.x + w];
            tr[threadIdx.x] += tr[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0];
        out[1] = tr[0];
    }
}
hipError_t launch_ns_check(const double* T, const double* X, int32_t m, int32_t k, double* part, double* out,
                           hipStream_t s) {
    k_ns_dev_part<<<NSRED_WG, 256, 0, s>>>(T, m, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_ns_finish<<<1, 256, 0, s>>>(part, X, m, k, out);
    return hipGetLastError();
}

}  // namespace hsim

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

#include "kernels.h"

namespace hsim {

namespace {
constexpr int T32 = 32;
constexpr int TT = T32 * T32;

__device__ __forceinline__ int64_t tri(int32_t Mt, int32_t I, int32_t J) {
    return (int64_t)J * Mt - (int64_t)J * (J - 1) / 2 + (I - J);
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

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
// one 64-lane wavefront per row, lanes across the k columns
__global__ __launch_bounds__(256) void k_spmm(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                                              const double* __restrict__ va, const double* __restrict__ vb, double a,
                                              double b, int64_t rows, const double* __restrict__ X, int64_t ldx,
                                              int32_t k, double* __restrict__ Y, int64_t ldy) {
    const int lane = threadIdx.x & 63;
    const int64_t row = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= rows) return;
    const int64_t e0 = ptr[row], e1 = ptr[row + 1];
    for (int c0 = 0; c0 < k; c0 += 256) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t e = e0; e < e1; ++e) {
            const double w = vb ? a * va[e] + b * vb[e] : a * va[e];
            const double* xr = X + (int64_t)idx[e] * ldx;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                int c = c0 + lane + 64 * u;
                if (c < k) acc[u] += w * xr[c];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int c = c0 + lane + 64 * u;
            if (c < k) Y[row * ldy + c] = acc[u];
        }
    }
}
hipError_t launch_spmm(const int64_t* ptr, const int32_t* idx, const double* va, const double* vb, double a, double b,
                       int64_t rows, const double* X, int64_t ldx, int32_t k, double* Y, int64_t ldy, hipStream_t s) {
    if (rows <= 0 || k <= 0) return hipSuccess;
    k_spmm<<<(unsigned)cdiv(rows, 4), 256, 0, s>>>(ptr, idx, va, vb, a, b, rows, X, ldx, k, Y, ldy);
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
    const DFront f = fr[items[blockIdx.x]];
    double* A = tiles + f.tile_base + tri(f.Mt, k, k) * TT;
    __shared__ double a[T32][T32 + 1];
    __shared__ double li[T32][T32 + 1];
    const int tid = threadIdx.x;
    for (int idx = tid; idx < TT; idx += 256) {
        int r = idx & 31, c = idx >> 5;
        a[r][c] = r >= c ? A[c * T32 + r] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < T32; ++j) {
        const double inv = 1.0 / a[j][j];
        for (int idx = tid; idx < TT; idx += 256) {
            int i = idx & 31, c = idx >> 5;
            if (c > j && i >= c) a[i][c] -= a[i][j] * a[c][j] * inv;
        }
        __syncthreads();
        if (tid > j && tid < T32) a[tid][j] *= inv;
    }
    __syncthreads();
    // inverse of the unit lower triangle, one column per thread
    if (tid < T32) {
        const int c = tid;
        for (int i = 0; i < T32; ++i) li[i][c] = 0.0;
        li[c][c] = 1.0;
        for (int i = c + 1; i < T32; ++i) {
            double s = 0.0;
            for (int t = c; t < i; ++t) s += a[i][t] * li[t][c];
            li[i][c] = -s;
        }
    }
    __syncthreads();
    double* Li = linv + f.linv_base + (int64_t)k * TT;
    for (int idx = tid; idx < TT; idx += 256) {
        int r = idx & 31, c = idx >> 5;
        A[c * T32 + r] = r > c ? a[r][c] : (r == c ? a[r][r] : 0.0);
        Li[c * T32 + r] = li[r][c];
    }
    if (tid < T32) {
        const double d = a[tid][tid];
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
__global__ __launch_bounds__(256) void k_fac_panel(double* tiles, const double* __restrict__ linv,
                                                   const double* __restrict__ D, const DFront* __restrict__ fr,
                                                   const int32_t* __restrict__ items, int32_t k) {
    const DFront f = fr[items[2 * blockIdx.x]];
    const int32_t I = items[2 * blockIdx.x + 1];
    double* A = tiles + f.tile_base + tri(f.Mt, I, k) * TT;
    const double* Li = linv + f.linv_base + (int64_t)k * TT;
    __shared__ double sa[T32][T32 + 1];
    __shared__ double sl[T32][T32 + 1];
    const int tid = threadIdx.x;
    for (int idx = tid; idx < TT; idx += 256) {
        int r = idx & 31, c = idx >> 5;
        sa[r][c] = A[c * T32 + r];
        sl[r][c] = Li[c * T32 + r];
    }
    __syncthreads();
    const int r = tid & 31;
    for (int c = tid >> 5; c < T32; c += 8) {
        double w = 0.0;
#pragma unroll 8
        for (int j = 0; j < T32; ++j) w += sa[r][j] * sl[c][j];
        A[c * T32 + r] = w / D[f.d_base + k * T32 + c];
    }
}
hipError_t launch_fac_panel(double* tiles, const double* linv, const double* D, const DFront* fronts,
                            const int32_t* items, int64_t nitems, int32_t k, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    k_fac_panel<<<(unsigned)nitems, 256, 0, s>>>(tiles, linv, D, fronts, items, k);
    return hipGetLastError();
}

// A_IJ -= L_Ik D_k L_Jk^T
__global__ __launch_bounds__(256) void k_fac_update(double* tiles, const double* __restrict__ D,
                                                    const DFront* __restrict__ fr, const int32_t* __restrict__ items,
                                                    int32_t k) {
    const DFront f = fr[items[3 * blockIdx.x]];
    const int32_t I = items[3 * blockIdx.x + 1], J = items[3 * blockIdx.x + 2];
    const double* LI = tiles + f.tile_base + tri(f.Mt, I, k) * TT;
    const double* LJ = tiles + f.tile_base + tri(f.Mt, J, k) * TT;
    double* A = tiles + f.tile_base + tri(f.Mt, I, J) * TT;
    __shared__ double s1[T32][T32 + 1];
    __shared__ double s2[T32][T32 + 1];
    const int tid = threadIdx.x;
    for (int idx = tid; idx < TT; idx += 256) {
        int r = idx & 31, c = idx >> 5;
        s1[r][c] = LI[c * T32 + r];
        s2[r][c] = LJ[c * T32 + r] * D[f.d_base + k * T32 + c];
    }
    __syncthreads();
    const int r = tid & 31;
    for (int c = tid >> 5; c < T32; c += 8) {
        double w = 0.0;
#pragma unroll 8
        for (int j = 0; j < T32; ++j) w += s1[r][j] * s2[c][j];
        A[c * T32 + r] -= w;
    }
}
hipError_t launch_fac_update(double* tiles, const double* D, const DFront* fronts, const int32_t* items,
                             int64_t nitems, int32_t k, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    k_fac_update<<<(unsigned)nitems, 256, 0, s>>>(tiles, D, fronts, items, k);
    return hipGetLastError();
}

// ============================================================ block solves
// Forward sweep over one tree level: for each front and column chunk,
//   y = L11^-1 (b_J + children's updates) and u_J = (children's updates) - L21 y.
// y is written back into X (pivot rows), u_J into the update buffer.
template <class T>
__global__ __launch_bounds__(256) void k_solve_fwd(const T* __restrict__ tiles, const T* __restrict__ linv,
                                                   const DFront* __restrict__ fr, int32_t f0, int32_t nchunks,
                                                   double* X, int64_t ldx, int32_t col0, int32_t ncols, int32_t qc,
                                                   T* ubuf, int64_t ldu, const int64_t* __restrict__ gptr,
                                                   const int64_t* __restrict__ gidx, const double* __restrict__ mdiag) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* y = reinterpret_cast<T*>(smem_raw);
    const DFront f = fr[f0 + blockIdx.x / nchunks];
    const int32_t chunk = blockIdx.x % nchunks;
    const int32_t c0 = col0 + chunk * qc;
    const int32_t cw = min(qc, col0 + ncols - c0);
    const int tid = threadIdx.x;
    // 1. pivot rows of the right-hand side plus the children's updates
    for (int idx = tid; idx < f.ns_pad * qc; idx += 256) {
        const int r = idx / qc, c = idx % qc;
        double v = 0.0;
        if (r < f.ns && c < cw) {
            v = X[(f.start + r) * ldx + c0 + c];
            if (mdiag) v *= mdiag[f.start + r];
            for (int64_t g = gptr[f.gather_base + r]; g < gptr[f.gather_base + r + 1]; ++g)
                v += (double)ubuf[gidx[g] * ldu + c0 + c];
        }
        y[idx] = (T)v;
    }
    __syncthreads();
    // 2. blocked forward substitution with the unit lower L11
    constexpr int MAXO = 4;  // 32 * qc / 256 with qc <= 32
    for (int kb = 0; kb < f.nsb; ++kb) {
        const T* Li = linv + f.linv_base + (int64_t)kb * TT;
        T tmp[MAXO];
        int o = 0;
        for (int idx = tid; idx < T32 * qc; idx += 256, ++o) {
            const int r = idx & 31, c = idx >> 5;
            T acc = 0;
#pragma unroll 8
            for (int j = 0; j < T32; ++j) acc += Li[j * T32 + r] * y[(kb * T32 + j) * qc + c];
            tmp[o] = acc;
        }
        __syncthreads();
        o = 0;
        for (int idx = tid; idx < T32 * qc; idx += 256, ++o) {
            const int r = idx & 31, c = idx >> 5;
            y[(kb * T32 + r) * qc + c] = tmp[o];
        }
        __syncthreads();
        const int rest = (f.nsb - kb - 1) * T32 * qc;
        for (int idx = tid; idx < rest; idx += 256) {
            const int ib = kb + 1 + idx / (T32 * qc);
            const int rem = idx % (T32 * qc);
            const int r = rem & 31, c = rem >> 5;
            const T* L = tiles + f.tile_base + tri(f.Mt, ib, kb) * TT;
            T acc = 0;
#pragma unroll 8
            for (int j = 0; j < T32; ++j) acc += L[j * T32 + r] * y[(kb * T32 + j) * qc + c];
            y[(ib * T32 + r) * qc + c] -= acc;
        }
        __syncthreads();
    }
    // 3. pivot rows out
    for (int idx = tid; idx < f.ns * qc; idx += 256) {
        const int r = idx / qc, c = idx % qc;
        if (c < cw) X[(f.start + r) * ldx + c0 + c] = (double)y[idx];
    }
    // 4. update rows: u = gathered - L21 y
    const int stiles = (f.mu + T32 - 1) / T32;
    for (int idx = tid; idx < stiles * T32 * qc; idx += 256) {
        const int sl = idx & 31;
        const int rest2 = idx >> 5;
        const int c = rest2 % qc, st = rest2 / qc;
        const int s = st * T32 + sl;
        if (s >= f.mu || c >= cw) continue;
        double acc = 0.0;
        const int64_t gr = f.gather_base + f.ns + s;
        for (int64_t g = gptr[gr]; g < gptr[gr + 1]; ++g) acc += (double)ubuf[gidx[g] * ldu + c0 + c];
        T a2 = 0;
        for (int kb = 0; kb < f.nsb; ++kb) {
            const T* L = tiles + f.tile_base + tri(f.Mt, f.nsb + st, kb) * TT;
#pragma unroll 8
            for (int j = 0; j < T32; ++j) a2 += L[j * T32 + sl] * y[(kb * T32 + j) * qc + c];
        }
        ubuf[(f.ubuf_row + s) * ldu + c0 + c] = (T)(acc - (double)a2);
    }
}

// Backward sweep over one tree level: z = D^-1 y - L21^T x_struct,
// x_J = L11^-T z (right-looking over the pivot tiles, last tile first).
template <class T>
__global__ __launch_bounds__(256) void k_solve_bwd(const T* __restrict__ tiles, const T* __restrict__ linv,
                                                   const T* __restrict__ D, const DFront* __restrict__ fr, int32_t f0,
                                                   int32_t nchunks, double* X, int64_t ldx, int32_t col0,
                                                   int32_t ncols, int32_t qc, const int32_t* __restrict__ rows,
                                                   int apply_dinv) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* z = reinterpret_cast<T*>(smem_raw);
    const DFront f = fr[f0 + blockIdx.x / nchunks];
    T* xs = z + (size_t)f.ns_pad * qc;   // 32 x qc staging of struct-row solution values
    const int32_t chunk = blockIdx.x % nchunks;
    const int32_t c0 = col0 + chunk * qc;
    const int32_t cw = min(qc, col0 + ncols - c0);
    const int tid = threadIdx.x;
    for (int idx = tid; idx < f.ns_pad * qc; idx += 256) {
        const int r = idx / qc, c = idx % qc;
        double v = 0.0;
        if (r < f.ns && c < cw) {
            v = X[(f.start + r) * ldx + c0 + c];
            if (apply_dinv) v /= (double)D[f.d_base + r];
        }
        z[idx] = (T)v;
    }
    __syncthreads();
    const int32_t* frows = rows + f.rows_off;
    const int stiles = (f.mu + T32 - 1) / T32;
    for (int st = 0; st < stiles; ++st) {
        for (int idx = tid; idx < T32 * qc; idx += 256) {
            const int s = idx / qc, c = idx % qc;
            const int sr = st * T32 + s;
            xs[idx] = (sr < f.mu && c < cw) ? (T)X[(int64_t)frows[sr] * ldx + c0 + c] : (T)0;
        }
        __syncthreads();
        for (int idx = tid; idx < f.ns_pad * qc; idx += 256) {
            const int j = idx / qc, c = idx % qc;
            const T* L = tiles + f.tile_base + tri(f.Mt, f.nsb + st, j / T32) * TT + (j % T32) * T32;
            T acc = 0;
#pragma unroll 8
            for (int s = 0; s < T32; ++s) acc += L[s] * xs[s * qc + c];
            z[idx] -= acc;
        }
        __syncthreads();
    }
    constexpr int MAXO = 4;
    for (int kb = f.nsb - 1; kb >= 0; --kb) {
        const T* Li = linv + f.linv_base + (int64_t)kb * TT;
        T tmp[MAXO];
        int o = 0;
        for (int idx = tid; idx < T32 * qc; idx += 256, ++o) {
            const int r = idx & 31, c = idx >> 5;
            T acc = 0;
#pragma unroll 8
            for (int j = 0; j < T32; ++j) acc += Li[r * T32 + j] * z[(kb * T32 + j) * qc + c];
            tmp[o] = acc;
        }
        __syncthreads();
        o = 0;
        for (int idx = tid; idx < T32 * qc; idx += 256, ++o) {
            const int r = idx & 31, c = idx >> 5;
            z[(kb * T32 + r) * qc + c] = tmp[o];
        }
        __syncthreads();
        const int rest = kb * T32 * qc;
        for (int idx = tid; idx < rest; idx += 256) {
            const int ib = idx / (T32 * qc);
            const int rem = idx % (T32 * qc);
            const int r = rem & 31, c = rem >> 5;
            const T* L = tiles + f.tile_base + tri(f.Mt, kb, ib) * TT + r * T32;
            T acc = 0;
#pragma unroll 8
            for (int j = 0; j < T32; ++j) acc += L[j] * z[(kb * T32 + j) * qc + c];
            z[(ib * T32 + r) * qc + c] -= acc;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < f.ns * qc; idx += 256) {
        const int r = idx / qc, c = idx % qc;
        if (c < cw) X[(f.start + r) * ldx + c0 + c] = (double)z[idx];
    }
}

template <class TF>
hipError_t launch_solve_fwd(const TF* tiles, const TF* linv, const DFront* fronts, int32_t f0, int32_t f1,
                            int32_t ns_pad_max, double* X, int64_t ldx, int32_t col0, int32_t ncols, int32_t qc,
                            double* ubuf, int64_t ldu, const int64_t* gptr, const int64_t* gidx, const double* mdiag,
                            hipStream_t s) {
    if (f1 <= f0 || ncols <= 0) return hipSuccess;
    const int32_t nchunks = (int32_t)cdiv(ncols, qc);
    const size_t lds = (size_t)ns_pad_max * qc * sizeof(TF);
    k_solve_fwd<TF><<<(unsigned)((f1 - f0) * nchunks), 256, lds, s>>>(
        tiles, linv, fronts, f0, nchunks, X, ldx, col0, ncols, qc, reinterpret_cast<TF*>(ubuf), ldu, gptr, gidx,
        mdiag);
    return hipGetLastError();
}
template <class TF>
hipError_t launch_solve_bwd(const TF* tiles, const TF* linv, const TF* D, const DFront* fronts, int32_t f0,
                            int32_t f1, int32_t ns_pad_max, double* X, int64_t ldx, int32_t col0, int32_t ncols,
                            int32_t qc, const int32_t* rows, bool apply_dinv, hipStream_t s) {
    if (f1 <= f0 || ncols <= 0) return hipSuccess;
    const int32_t nchunks = (int32_t)cdiv(ncols, qc);
    const size_t lds = ((size_t)ns_pad_max + T32) * qc * sizeof(TF);
    k_solve_bwd<TF><<<(unsigned)((f1 - f0) * nchunks), 256, lds, s>>>(tiles, linv, D, fronts, f0, nchunks, X, ldx,
                                                                       col0, ncols, qc, rows, apply_dinv ? 1 : 0);
    return hipGetLastError();
}
template hipError_t launch_solve_fwd<double>(const double*, const double*, const DFront*, int32_t, int32_t, int32_t,
                                             double*, int64_t, int32_t, int32_t, int32_t, double*, int64_t,
                                             const int64_t*, const int64_t*, const double*, hipStream_t);
template hipError_t launch_solve_fwd<float>(const float*, const float*, const DFront*, int32_t, int32_t, int32_t,
                                            double*, int64_t, int32_t, int32_t, int32_t, double*, int64_t,
                                            const int64_t*, const int64_t*, const double*, hipStream_t);
template hipError_t launch_solve_bwd<double>(const double*, const double*, const double*, const DFront*, int32_t,
                                             int32_t, int32_t, double*, int64_t, int32_t, int32_t, int32_t,
                                             const int32_t*, bool, hipStream_t);
template hipError_t launch_solve_bwd<float>(const float*, const float*, const float*, const DFront*, int32_t,
                                            int32_t, int32_t, double*, int64_t, int32_t, int32_t, int32_t,
                                            const int32_t*, bool, hipStream_t);

// ============================================================ Gram products
int64_t gram_partial_doubles(int64_t n, int32_t q, int64_t chunk_rows) {
    const int64_t nt = cdiv(q, T32);
    return cdiv(n, chunk_rows) * (nt * (nt + 1) / 2) * 2 * TT;
}

// partial[chunk][pair][0|1][r][c]: sum over the chunk's rows of
// Psi[row, a*32+r] * (S Psi)[row, b*32+c]  and  Psi[row, a*32+r] * (M Psi)[row, b*32+c].
// TA = double: FP64 throughout.  TA = float: operands rounded to FP32, FP32
// products and accumulation over runs of 256 rows, FP64 sum of the runs.
template <class TA>
__global__ __launch_bounds__(256) void k_gram_partial(const double* __restrict__ Psi, const double* __restrict__ SPsi,
                                                      const double* __restrict__ MPsi, const double* __restrict__ mdiag,
                                                      int64_t n, int32_t q, int64_t ld, int64_t chunk_rows,
                                                      double* __restrict__ partial) {
    const int32_t nt = (q + T32 - 1) / T32;
    // decode the (a <= b) pair
    int32_t pair = blockIdx.y, a = 0;
    while (pair >= nt - a) { pair -= nt - a; ++a; }
    const int32_t b = a + pair;
    const int64_t r0 = blockIdx.x * chunk_rows;
    const int64_t r1 = min(n, r0 + chunk_rows);
    __shared__ TA P[T32][T32 + 1], Q[T32][T32 + 1], R[T32][T32 + 1];
    const int tid = threadIdx.x;
    const int r = tid & 31;
    double accS[4] = {0, 0, 0, 0}, accM[4] = {0, 0, 0, 0};
    TA runS[4] = {0, 0, 0, 0}, runM[4] = {0, 0, 0, 0};
    int tiles_in_run = 0;
    for (int64_t row0 = r0; row0 < r1; row0 += T32) {
        for (int idx = tid; idx < TT; idx += 256) {
            const int i = idx >> 5, c = idx & 31;
            const int64_t row = row0 + i;
            const int ca = a * T32 + c, cb = b * T32 + c;
            const bool ok = row < r1;
            P[i][c] = (TA)((ok && ca < q) ? Psi[row * ld + ca] : 0.0);
            Q[i][c] = (TA)((ok && cb < q) ? SPsi[row * ld + cb] : 0.0);
            R[i][c] = (TA)((ok && cb < q) ? (mdiag ? mdiag[row] * Psi[row * ld + cb] : MPsi[row * ld + cb]) : 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int c = (tid >> 5) + 8 * o;
            TA sv = 0, mv = 0;
#pragma unroll 8
            for (int i = 0; i < T32; ++i) {
                sv += P[i][r] * Q[i][c];
                mv += P[i][r] * R[i][c];
            }
            runS[o] += sv;
            runM[o] += mv;
        }
        if (++tiles_in_run == 8) {
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                accS[o] += (double)runS[o];
                accM[o] += (double)runM[o];
                runS[o] = runM[o] = 0;
            }
            tiles_in_run = 0;
        }
        __syncthreads();
    }
    const int64_t npairs = (int64_t)nt * (nt + 1) / 2;
    double* out = partial + ((int64_t)blockIdx.x * npairs + blockIdx.y) * 2 * TT;
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const int c = (tid >> 5) + 8 * o;
        out[r * T32 + c] = accS[o] + (double)runS[o];
        out[TT + r * T32 + c] = accM[o] + (double)runM[o];
    }
}

__global__ void k_gram_reduce(const double* __restrict__ partial, int64_t nchunks, int32_t q, double* Sbar,
                              double* Mbar) {
    const int32_t nt = (q + T32 - 1) / T32;
    const int64_t npairs = (int64_t)nt * (nt + 1) / 2;
    const int64_t tot = (int64_t)q * q;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = (int32_t)(t / q), j = (int32_t)(t % q);
        if (i > j) continue;
        const int32_t a = i / T32, b = j / T32;
        const int64_t pair = (int64_t)a * nt - (int64_t)a * (a - 1) / 2 + (b - a);
        const int off = (i % T32) * T32 + (j % T32);
        double s = 0, m = 0;
        for (int64_t ch = 0; ch < nchunks; ++ch) {
            const double* p = partial + (ch * npairs + pair) * 2 * TT;
            s += p[off];
            m += p[TT + off];
        }
        Sbar[(int64_t)i * q + j] = s;
        Sbar[(int64_t)j * q + i] = s;
        Mbar[(int64_t)i * q + j] = m;
        Mbar[(int64_t)j * q + i] = m;
    }
}

hipError_t launch_gram(const double* Psi, const double* SPsi, const double* MPsi, const double* mdiag, int64_t n,
                       int32_t q, int64_t ld, double* partial, int64_t chunk_rows, double* Sbar, double* Mbar,
                       hipStream_t s, bool fp32) {
    const int64_t nt = cdiv(q, T32);
    const int64_t nch = cdiv(n, chunk_rows);
    const dim3 grid((unsigned)nch, (unsigned)(nt * (nt + 1) / 2));
    if (fp32)
        k_gram_partial<float><<<grid, 256, 0, s>>>(Psi, SPsi, MPsi, mdiag, n, q, ld, chunk_rows, partial);
    else
        k_gram_partial<double><<<grid, 256, 0, s>>>(Psi, SPsi, MPsi, mdiag, n, q, ld, chunk_rows, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_gram_reduce<<<grid_for((int64_t)q * q, 256), 256, 0, s>>>(partial, nch, q, Sbar, Mbar);
    return hipGetLastError();
}

// ============================================================ Ritz update + residual
int64_t ritz_partial_doubles(int64_t n, int32_t q, int64_t chunk_rows) { return cdiv(n, chunk_rows) * 2 * (int64_t)q; }

// Phi = Psi Phibar, (S Phi) = (S Psi) Phibar kept in registers, M Phi =
// m * Phi (level 0) or (M Psi) Phibar; per-column partial sums of the
// residual numerator and the normalisation.
__global__ __launch_bounds__(256) void k_ritz(const double* __restrict__ Psi, const double* __restrict__ SPsi,
                                              const double* __restrict__ MPsi, const double* __restrict__ mdiag,
                                              const double* __restrict__ Phibar, const double* __restrict__ lam,
                                              int64_t n, int32_t q, int64_t ld, double* __restrict__ Phi,
                                              double* __restrict__ MPhi, double* __restrict__ partial,
                                              int64_t chunk_rows, int minv_norm) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* Pb = reinterpret_cast<double*>(smem_raw);    // q x 32
    __shared__ double red[2][8][T32];
    const int tid = threadIdx.x;
    const int cl = tid & 31, rl = tid >> 5;
    const int col = blockIdx.y * T32 + cl;
    for (int idx = tid; idx < q * T32; idx += 256) {
        const int kk = idx >> 5, c = idx & 31;
        const int cc = blockIdx.y * T32 + c;
        Pb[idx] = cc < q ? Phibar[(int64_t)kk * q + cc] : 0.0;
    }
    __syncthreads();
    const double lc = col < q ? lam[col] : 0.0;
    double num = 0, den = 0;
    const int64_t r0 = blockIdx.x * chunk_rows;
    const int64_t r1 = min(n, r0 + chunk_rows);
    for (int64_t row = r0 + rl; row < r1; row += 8) {
        const double* pr = Psi + row * ld;
        const double* sr = SPsi + row * ld;
        double phi = 0, sphi = 0, mphi = 0;
        if (mdiag) {
            for (int kk = 0; kk < q; ++kk) {
                const double w = Pb[kk * T32 + cl];
                phi += pr[kk] * w;
                sphi += sr[kk] * w;
            }
            mphi = mdiag[row] * phi;
        } else {
            const double* mr = MPsi + row * ld;
            for (int kk = 0; kk < q; ++kk) {
                const double w = Pb[kk * T32 + cl];
                phi += pr[kk] * w;
                sphi += sr[kk] * w;
                mphi += mr[kk] * w;
            }
        }
        if (col < q) {
            Phi[row * ld + col] = phi;
            if (MPhi) MPhi[row * ld + col] = mphi;
            const double res = sphi - lc * mphi;
            if (minv_norm) {
                num += res * res / mdiag[row];
                den += phi * mphi;
            } else {
                num += res * res;
                den += mphi * mphi;
            }
        }
    }
    red[0][rl][cl] = num;
    red[1][rl][cl] = den;
    __syncthreads();
    if (tid < T32 && blockIdx.y * T32 + tid < q) {
        double a = 0, b = 0;
        for (int k = 0; k < 8; ++k) {
            a += red[0][k][tid];
            b += red[1][k][tid];
        }
        partial[(int64_t)blockIdx.x * 2 * q + blockIdx.y * T32 + tid] = a;
        partial[(int64_t)blockIdx.x * 2 * q + q + blockIdx.y * T32 + tid] = b;
    }
}

__global__ void k_resid_reduce(const double* __restrict__ partial, int64_t nchunks, int32_t q,
                               const double* __restrict__ lam, double lam_floor, double* resid) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= q) return;
    double a = 0, b = 0;
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        a += partial[ch * 2 * q + c];
        b += partial[ch * 2 * q + q + c];
    }
    resid[c] = sqrt(a) / (fmax(fabs(lam[c]), lam_floor) * sqrt(b));
}

hipError_t launch_ritz(const double* Psi, const double* SPsi, const double* MPsi, const double* mdiag,
                       const double* Phibar, const double* lam, int64_t n, int32_t q, int64_t ld, double* Phi,
                       double* MPhi, double* partial, int64_t chunk_rows, bool minv_norm, double lam_floor,
                       double* resid, hipStream_t s) {
    const int64_t nch = cdiv(n, chunk_rows);
    const int64_t nct = cdiv(q, T32);
    const size_t lds = (size_t)q * T32 * sizeof(double);
    hipError_t e0 = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_ritz), lds, 4096);
    if (e0 != hipSuccess) return e0;
    k_ritz<<<dim3((unsigned)nch, (unsigned)nct), 256, lds, s>>>(Psi, SPsi, MPsi, mdiag, Phibar, lam, n, q, ld, Phi,
                                                                 MPhi, partial, chunk_rows, minv_norm ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_resid_reduce<<<(unsigned)cdiv(q, 256), 256, 0, s>>>(partial, nch, q, lam, lam_floor, resid);
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

// ---- cyclic Jacobi in round-robin order ---------------------------------
// round r pairs the players at positions x and m-1-x; position 0 is fixed,
// positions 1..m-1 hold players 1 + (x - 1 + r) mod (m - 1)
__device__ __forceinline__ int jac_player(int x, int r, int m) { return x == 0 ? 0 : 1 + (x - 1 + r) % (m - 1); }
__device__ __forceinline__ int jac_partner(int a, int r, int m) {
    int pos = a == 0 ? 0 : 1 + ((a - 1 - r) % (m - 1) + (m - 1)) % (m - 1);
    return jac_player(m - 1 - pos, r, m);
}

__global__ void k_jacobi_init(const double* C, int32_t m, double* V, double* diag, double* off) {
    const int64_t tot = (int64_t)m * m;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = (int32_t)(t / m), j = (int32_t)(t % m);
        V[t] = i == j ? 1.0 : 0.0;
        if (i == j) diag[i] = C[t];
        if (j == jac_partner(i, 0, m)) off[i] = C[t];
    }
}
hipError_t launch_jacobi_init(const double* C, int32_t m, double* V, double* diag, double* off, hipStream_t s) {
    k_jacobi_init<<<grid_for((int64_t)m * m, 256), 256, 0, s>>>(C, m, V, diag, off);
    return hipGetLastError();
}

// One round: all m/2 rotations of the round at once, C <- J^T C J, V <- V J.
// Every block recomputes the round's rotations from diag_cur/off_cur (written
// by the previous round), updates its share of the 2x2 blocks and V rows, and
// records the entries the next round's rotations need.
__global__ __launch_bounds__(256) void k_jacobi_round(double* C, double* V, int32_t m, int32_t r,
                                                      const double* __restrict__ diag_cur,
                                                      const double* __restrict__ off_cur, double* diag_next,
                                                      double* off_next, double tol_rel,
                                                      const double* __restrict__ normf, double tol_abs_rel,
                                                      int32_t* rot_count) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int h = m / 2;
    double* cs = reinterpret_cast<double*>(smem_raw);
    double* sn = cs + h;
    int* pp = reinterpret_cast<int*>(sn + h);
    int* qq = pp + h;
    __shared__ int nrot;
    if (threadIdx.x == 0) nrot = 0;
    const double tol_abs = tol_abs_rel * normf[0];
    __syncthreads();
    for (int kk = threadIdx.x; kk < h; kk += blockDim.x) {
        int a = jac_player(kk, r, m), b = jac_player(m - 1 - kk, r, m);
        int p = min(a, b), q = max(a, b);
        double app = diag_cur[p], aqq = diag_cur[q], apq = off_cur[p];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > fmax(tol_abs, tol_rel * sqrt(fabs(app * aqq)))) {
            double tau = (aqq - app) / (2.0 * apq);
            double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            atomicAdd(&nrot, 1);
        }
        cs[kk] = c;
        sn[kk] = s;
        pp[kk] = p;
        qq[kk] = q;
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0 && nrot) atomicAdd(rot_count, nrot);
    const int64_t nblk = (int64_t)h * (h + 1) / 2;
    const int64_t tot = nblk + (int64_t)m * h;
    const int rn = r + 1;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        if (t < nblk) {
            // decode upper block pair (k <= l)
            int64_t rem = t;
            int k = (int)((sqrt(8.0 * (double)rem + 1.0) - 1.0) / 2.0);   // row of a lower-triangle walk
            while ((int64_t)(k + 1) * (k + 2) / 2 <= rem) ++k;
            while ((int64_t)k * (k + 1) / 2 > rem) --k;
            int l = (int)(rem - (int64_t)k * (k + 1) / 2);   // l <= k
            const int pk = pp[k], qk = qq[k], pl = pp[l], ql = qq[l];
            const double ck = cs[k], sk = sn[k], cl = cs[l], sl = sn[l];
            double g00 = C[(int64_t)pk * m + pl], g01 = C[(int64_t)pk * m + ql];
            double g10 = C[(int64_t)qk * m + pl], g11 = C[(int64_t)qk * m + ql];
            // rows (pair k)
            double h00 = ck * g00 - sk * g10, h01 = ck * g01 - sk * g11;
            double h10 = sk * g00 + ck * g10, h11 = sk * g01 + ck * g11;
            // columns (pair l)
            double n00 = h00 * cl - h01 * sl, n01 = h00 * sl + h01 * cl;
            double n10 = h10 * cl - h11 * sl, n11 = h10 * sl + h11 * cl;
            if (k == l && sk != 0.0) { n01 = 0.0; n10 = 0.0; }
            const int ri[2] = {pk, qk}, ci[2] = {pl, ql};
            const double nv[2][2] = {{n00, n01}, {n10, n11}};
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    const int i = ri[x], j = ci[y];
                    const double v = nv[x][y];
                    C[(int64_t)i * m + j] = v;
                    C[(int64_t)j * m + i] = v;
                    if (i == j) diag_next[i] = v;
                    if (jac_partner(i, rn, m) == j) { off_next[i] = v; off_next[j] = v; }
                }
        } else {
            const int64_t u = t - nblk;
            const int64_t row = u / h;
            const int kk = (int)(u % h);
            const double c = cs[kk], s = sn[kk];
            if (s == 0.0) continue;
            double* vr = V + row * m;
            const double a = vr[pp[kk]], b = vr[qq[kk]];
            vr[pp[kk]] = a * c - b * s;
            vr[qq[kk]] = a * s + b * c;
        }
    }
}
hipError_t launch_jacobi_round(double* C, double* V, int32_t m, int32_t round, const double* diag_cur,
                               const double* off_cur, double* diag_next, double* off_next, double tol_rel,
                               const double* normf, double tol_abs_rel, int32_t* rot_count, hipStream_t s) {
    const int h = m / 2;
    const int64_t tot = (int64_t)h * (h + 1) / 2 + (int64_t)m * h;
    const size_t lds = (size_t)h * (2 * sizeof(double) + 2 * sizeof(int));
    unsigned g = grid_for(tot, 256);
    if (g > 2048) g = 2048;
    k_jacobi_round<<<g, 256, lds, s>>>(C, V, m, round, diag_cur, off_cur, diag_next, off_next, tol_rel, normf,
                                        tol_abs_rel, rot_count);
    return hipGetLastError();
}

// ascending order of the diagonal of C (ties by index); X[r, j] = scale[r] Y[r, order[j]]
__global__ __launch_bounds__(1024) void k_sort_eig(const double* C, int32_t m, int32_t kvalid, const double* Y,
                                                   int32_t rows, const double* scale, int32_t kout, double* lam_out,
                                                   double* X, int64_t ldx) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int* order = reinterpret_cast<int*>(smem_raw);
    for (int i = threadIdx.x; i < kvalid; i += blockDim.x) {
        const double li = C[(int64_t)i * m + i];
        int rank = 0;
        for (int j = 0; j < kvalid; ++j) {
            const double lj = C[(int64_t)j * m + j];
            rank += (lj < li) || (lj == li && j < i);
        }
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
    k_sort_eig<<<1, 1024, (size_t)kout * sizeof(int), s>>>(C, m, kvalid, Y, rows, scale, kout, lam_out, X, ldx);
    return hipGetLastError();
}

// C (m x m) = Ck (k x k) with, when m = k + 1, a decoupled dummy row/column
// whose diagonal exceeds every eigenvalue; normf[0] = ||Ck||_F; dis = D^-1/2
// (1 on the dummy)
__global__ void k_embed_copy(const double* Ck, int32_t k, int32_t m, double* C) {
    const int64_t tot = (int64_t)m * m;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = (int32_t)(t / m), j = (int32_t)(t % m);
        C[t] = (i < k && j < k) ? Ck[(int64_t)i * k + j] : 0.0;
    }
}
__global__ __launch_bounds__(1024) void k_embed_finish(const double* Ck, int32_t k, int32_t m, double* C,
                                                       double* normf, double* dis, const double* D) {
    __shared__ double red[1024];
    double s = 0.0;
    const int64_t tot = (int64_t)k * k;
    for (int64_t t = threadIdx.x; t < tot; t += blockDim.x) s += Ck[t] * Ck[t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double nf = sqrt(red[0]);
    if (threadIdx.x == 0) {
        normf[0] = nf;
        if (m > k) C[(int64_t)k * m + k] = 4.0 * nf + 1.0;
    }
    for (int i = threadIdx.x; i < m; i += blockDim.x) dis[i] = i < k ? 1.0 / sqrt(D[i]) : 1.0;
}
hipError_t launch_embed_pad(const double* Ck, int32_t k, int32_t m, double* C, double* normf, double* dis,
                            const double* D, hipStream_t s) {
    k_embed_copy<<<grid_for((int64_t)m * m, 256), 256, 0, s>>>(Ck, k, m, C);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_embed_finish<<<1, 1024, 0, s>>>(Ck, k, m, C, normf, dis, D);
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
// the normalisation terms).
__global__ void k_bwd_vertex(int64_t nv, int32_t p, const double* __restrict__ X, const double* __restrict__ W,
                             const double* __restrict__ Y, int64_t ld, const int32_t* __restrict__ iperm,
                             const double* __restrict__ lam, const double* __restrict__ glam,
                             const double* __restrict__ rho, double* __restrict__ nu) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = iperm[v];
        double s = 0;
        for (int k = 0; k < p; ++k) {
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
__global__ void k_bwd_tri(int64_t nf, const int32_t* __restrict__ F, const double* __restrict__ V, int32_t p,
                          const double* __restrict__ X, const double* __restrict__ W, int64_t ld,
                          const int32_t* __restrict__ iperm, const double* __restrict__ glam,
                          const double* __restrict__ nu, double* __restrict__ G) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nf; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t vi[3] = {F[3 * t], F[3 * t + 1], F[3 * t + 2]};
        const int64_t ri[3] = {iperm[vi[0]], iperm[vi[1]], iperm[vi[2]]};
        double P[3][3];
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) P[a][d] = V[3 * (int64_t)vi[a] + d];
        double e[3] = {0, 0, 0};   // per corner: its opposite edge
        for (int k = 0; k < p; ++k) {
            const double x0 = X[ri[0] * ld + k], x1 = X[ri[1] * ld + k], x2 = X[ri[2] * ld + k];
            const double xs[3] = {x0, x1, x2};
            double ws[3] = {0, 0, 0};
            if (W) { ws[0] = W[ri[0] * ld + k]; ws[1] = W[ri[1] * ld + k]; ws[2] = W[ri[2] * ld + k]; }
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
            const double f = 0.5 * e[c];
            for (int d = 0; d < 3; ++d) {
                const double du = w[d] / sn - dot * wc[d] / (s2 * sn);   // d cot / d u
                const double dw = u[d] / sn - dot * cu[d] / (s2 * sn);   // d cot / d w
                grad[i][d] += f * du;
                grad[j][d] += f * dw;
                grad[c][d] -= f * (du + dw);
            }
        }
        // area term
        {
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
                          int64_t ld, const int32_t* iperm, const double* glam, const double* nu, double* G,
                          hipStream_t s) {
    k_bwd_tri<<<grid_for(nf, 256), 256, 0, s>>>(nf, F, V, p, X, W, ld, iperm, glam, nu, G);
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
                              int64_t ld) {
    const int64_t tot = n * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t % n;
        const int c = (int)(t / n);
        out[r * ld + c] = in[(int64_t)c * nv + perm[r]];
    }
}
hipError_t launch_import_cols(const double* in, int64_t nv, const int32_t* perm, int64_t n, int32_t k, double* out,
                              int64_t ld, hipStream_t s) {
    if (n <= 0 || k <= 0) return hipSuccess;
    k_import_cols<<<grid_for(n * k, 256), 256, 0, s>>>(in, nv, perm, n, k, out, ld);
    return hipGetLastError();
}

// ============================================================ output
// per column: the row with the largest |value|, lowest vertex index on ties
__global__ __launch_bounds__(256) void k_col_argmax(const double* Phi, int64_t ld, int64_t n, int32_t p,
                                                    const int32_t* perm, int64_t chunk, double* pv, int64_t* pi) {
    const int c = blockIdx.y;
    const int64_t r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
    double best = -1.0;
    int64_t bi = INT64_MAX;
    double bv = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const double v = Phi[r * ld + c];
        const int64_t vi = perm ? perm[r] : r;
        const double a = fabs(v);
        if (a > best || (a == best && vi < bi)) { best = a; bi = vi; bv = v; }
    }
    __shared__ double sb[256], sv[256];
    __shared__ int64_t si[256];
    sb[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    sv[threadIdx.x] = bv;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const int o = threadIdx.x + w;
            if (sb[o] > sb[threadIdx.x] || (sb[o] == sb[threadIdx.x] && si[o] < si[threadIdx.x])) {
                sb[threadIdx.x] = sb[o];
                si[threadIdx.x] = si[o];
                sv[threadIdx.x] = sv[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pv[(int64_t)c * gridDim.x + blockIdx.x] = sb[0] >= 0 ? (sv[0] < 0 ? -sb[0] : sb[0]) : 0.0;
        pi[(int64_t)c * gridDim.x + blockIdx.x] = si[0];
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
// evecs[c * n + perm[r]] = sign[c] * Phi[r, c]: tiles of 32 rows x 32 columns through LDS
__global__ __launch_bounds__(256) void k_export(const double* Phi, int64_t ld, int64_t n, int32_t p,
                                                const int32_t* perm, const double* sign, double* evecs) {
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
            evecs[(int64_t)c * n + v] = sign[c] * t[tx][yy];
        }
    }
}
hipError_t launch_export_evecs(const double* Phi, int64_t ld, int64_t n, int32_t p, const int32_t* perm,
                               double* evecs, double* work, hipStream_t s) {
    const int64_t chunk = 8192;
    const int64_t nch = cdiv(n, chunk);
    double* pv = work;
    int64_t* pi = reinterpret_cast<int64_t*>(work + nch * p);
    double* sign = work + 2 * nch * p;
    k_col_argmax<<<dim3((unsigned)nch, (unsigned)p), 256, 0, s>>>(Phi, ld, n, p, perm, chunk, pv, pi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_col_sign<<<(unsigned)cdiv(p, 256), 256, 0, s>>>(pv, pi, nch, p, sign);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_export<<<dim3((unsigned)cdiv(n, T32), (unsigned)cdiv(p, T32)), 256, 0, s>>>(Phi, ld, n, p, perm, sign, evecs);
    return hipGetLastError();
}

}  // namespace hsim

// Host-callable launchers of the HIP kernels (gfx950).  Every launcher
// enqueues on `stream` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hsim {

// Device copy of a front's geometry (see Front in internal.h).
// DFront::flags bit: some row of the front gathers children's update rows
constexpr int32_t DFRONT_GATHER = 1;
// q_base: offset of the front's inverse-panel tiles (qinv / qinvT), -1 if it
// has none; qrow: first row of the front in the scratch block of the
// inverse-panel solves of its tree level.
struct DFront {
    int64_t start, tile_base, linv_base, d_base, ubuf_row, gather_base, rows_off, q_base, qrow;
    int32_t ns, mu, ns_pad, mu_pad, Mt, nsb, parent, flags;   // flags: DFRONT_GATHER
};

// ------------------------------------------------------------ utilities
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_fill_f(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_to_float(const double* src, float* dst, int64_t n, hipStream_t s);
// out[i, :k] = in[idx[i], :k] (rows, with leading dims)
hipError_t launch_gather_rows(const double* in, int64_t ldi, const int32_t* idx, int64_t n, int32_t k,
                              double* out, int64_t ldo, hipStream_t s);
// out[idx[i], :k] = in[i, :k]
hipError_t launch_scatter_rows(const double* in, int64_t ldi, const int32_t* idx, int64_t n, int32_t k,
                               double* out, int64_t ldo, hipStream_t s);
hipError_t launch_copy2d(const double* in, int64_t ldi, int64_t rows, int32_t k, double* out, int64_t ldo,
                         hipStream_t s);

// ------------------------------------------------------------ sparse products
// Y[r, c] = sum_e (a * va[e] + b * vb[e]) X[idx[e], c], c < k (vb may be null)
hipError_t launch_spmm(const int64_t* ptr, const int32_t* idx, const double* va, const double* vb, double a,
                       double b, int64_t rows, const double* X, int64_t ldx, int32_t k, double* Y, int64_t ldy,
                       hipStream_t s);
// Y[r, c] = d[r] X[r, c]
hipError_t launch_diag_scale(const double* d, int64_t rows, const double* X, int64_t ldx, int32_t k, double* Y,
                             int64_t ldy, hipStream_t s);
// Y = X - Y (elementwise on the first k columns): residual helpers
hipError_t launch_axpby(double a, const double* X, int64_t ldx, double b, double* Y, int64_t ldy, int64_t rows,
                        int32_t k, hipStream_t s);

// ------------------------------------------------------------ factor
hipError_t launch_assemble(double* tiles, const int64_t* dst, const int64_t* src, int64_t count,
                           const double* Sval, const double* Mval, double alpha, double beta, hipStream_t s);
hipError_t launch_extend_add(double* tiles, const DFront* fronts, const int32_t* items, int64_t nitems,
                             const int32_t* rel, int32_t max_tile_cols, hipStream_t s);
hipError_t launch_fac_diag(double* tiles, double* linv, double* D, const DFront* fronts, const int32_t* items,
                           int64_t nitems, int32_t k, int32_t* counters, hipStream_t s);
// panel / update launches of pivot tile step k; with qT, the same launches
// also run the row items (front, j) / update items (front, I, j) of the
// inverse panels (qT: transposed tiles of Q = [L11^-1; -L21 L11^-1] at each
// front's q_base, zero before step 0)
hipError_t launch_fac_panel(double* tiles, const double* linv, const double* D, const DFront* fronts,
                            const int32_t* items, int64_t nitems, int32_t k, hipStream_t s, double* qT = nullptr,
                            const int32_t* qitems = nullptr, int64_t nq = 0);
hipError_t launch_fac_update(double* tiles, const double* D, const DFront* fronts, const int32_t* items,
                             int64_t nitems, int32_t k, hipStream_t s, double* qT = nullptr,
                             const int32_t* qitems = nullptr, int64_t nq = 0);

// ------------------------------------------------------------ block solves
// Wave-level matrix-core solves of one tree level (fronts [f0, f1), pivot
// counts up to wsolve_max_ns()): one wave per (front, 16 columns), the
// front's block of the right-hand side in registers.  fwd: forward sweep
// (mdiag optional pre-scaling, children's updates gathered from ubuf, own
// updates written to ubuf; gat: gw update-buffer rows per front row, -1 = none,
// indexed by (gather_base + local row)); !fwd: backward sweep (apply_dinv divides by D),
// with tiles and linv the tile-transposed copies (launch_tile_transpose).
// Xin (forward only, null: X): where the right-hand-side rows are read; the
// solution is written to X either way.
int32_t wsolve_max_ns();
// every 32 x 32 tile of in[0 .. 1024 ntiles) transposed into the same place of out
template <class T>
hipError_t launch_tile_transpose(const T* in, T* out, int64_t ntiles, hipStream_t s);
template <class TF>
hipError_t launch_wsolve(bool fwd, const TF* tiles, const TF* linv, const TF* D, const DFront* fronts, int32_t f0,
                         int32_t f1, int32_t ns_pad_max, double* X, int64_t ldx, int32_t col0, int32_t ncols,
                         double* ubuf, int64_t ldu, const int32_t* gat, int32_t gw, const double* mdiag,
                         const int32_t* rows, bool apply_dinv, hipStream_t s, const double* Xin = nullptr);

// Block solves through the inverse panels (fronts with q_base >= 0):
// phase 0 forward gather (items: front, 32-row tile of [0, Mt)): right-hand
// side of the pivots (Xin times mdiag plus the children's updates) into the
// scratch block R, children's updates of the struct rows into the front's
// update rows; 1 forward product (items: front, 32-row tile I < Mt):
// pivot rows of X = Q_piv R, update rows += Q_struct R; 2 backward gather
// (items as phase 0): R = [D^-1 X(pivots); X(struct rows)]; 3 backward
// product (items: front, 32-row pivot tile C < nsb): X(pivots) = Q^T R.
// qinv: column-major Q tiles (phase 1), qinvT: transposed tiles (phase 3).
// kmax (products): the longest contraction of the items in tiles (forward:
// the largest nsb, backward: the largest Mt); it sets the waves that share
// one output tile.  fuse (phases 0 and 1 of one forward sweep, both with the
// same value): the gather fills only the pivot rows of R and the product
// gathers the children's updates of the struct rows itself, writing each
// update row once.
template <class TF>
hipError_t launch_qsolve(int phase, const TF* qinv, const TF* qinvT, const TF* D, const DFront* fronts,
                         const int32_t* items, int64_t nitems, double* R, int64_t ldr, double* X, int64_t ldx,
                         int32_t col0, int32_t ncols, double* ubuf, int64_t ldu, const int32_t* gat, int32_t gw,
                         const double* mdiag, const int32_t* rows, hipStream_t s, const double* Xin = nullptr,
                         int32_t kmax = 1, bool fuse = false);

// ------------------------------------------------------------ Rayleigh-Ritz
// partial Grams over row chunks of chunk_rows rows (gram_chunk_rows of the
// largest n the partial buffer is sized for), then the sum
// mode 0: FP64; 1: operands rounded to FP32, FP32 accumulation over runs of 256 rows, FP64 sum of
// the runs; 2: compensated (hi/lo FP32 split of every operand, three FP32 products, FP64 stage sums)
enum { GRAM_FP64 = 0, GRAM_FP32 = 1, GRAM_COMPENSATED = 2 };
hipError_t launch_gram(const double* Psi, const double* SPsi, const double* MPsi, const double* mdiag, int64_t n,
                       int32_t q, int64_t ld, double* partial, int64_t chunk_rows, double* Sbar, double* Mbar,
                       hipStream_t s, int mode = GRAM_FP64);
int64_t gram_partial_doubles(int64_t n, int32_t q, int64_t chunk_rows);
int64_t gram_chunk_rows(int64_t n, int32_t q);
// largest q for which the FP64 Gram is one pass over the rows (all tiles per workgroup)
int32_t gram_fp64_single_pass_max_q();

// Phi = Psi Phibar and residual partial sums; then the residual
// nres: residuals of the first nres columns only (the rest are set to NaN); -1 = all
hipError_t launch_ritz(const double* Psi, const double* SPsi, const double* MPsi, const double* mdiag,
                       const double* Phibar, const double* lam, int64_t n, int32_t q, int64_t ld, double* Phi,
                       double* MPhi, double* partial, int64_t chunk_rows, bool minv_norm, double lam_floor,
                       double* resid, hipStream_t s, int32_t nres = -1);
int64_t ritz_partial_doubles(int64_t n, int32_t q, int64_t chunk_rows);

// ------------------------------------------------------------ dense GEP helpers
// E = diag(M)^-1/2; S' = E S E, M' = E M E (k x k row-major, in place into So/Mo)
hipError_t launch_equilibrate(const double* S, const double* M, int32_t k, double* So, double* Mo, double* e,
                              hipStream_t s);
// copy the lower triangle of the k x k row-major A into one dense front (tile
// storage, Mt tiles per side); dummy pivots beyond k get 1 on the diagonal
// finest-level cotangent stiffness values on a given CSR pattern and barycentric lumped mass
// (corner lists: per entry its <= 2 opposite corners 3t + k, -1 padded; per vertex the corners
// whose weights its diagonal sums; per vertex its triangles); w [3 nf], a3 [nf] scratch
hipError_t launch_assemble_mesh(const double* V, const int32_t* F, int64_t nf, int64_t n, const int64_t* ptr,
                                const int32_t* idx, const int64_t* corner, const int64_t* dptr,
                                const int64_t* dcorner, const int64_t* vptr, const int32_t* vtri,
                                const double* density, double* w, double* a3, double* sval, double* mdiag,
                                hipStream_t s);
// descriptor, factorisation and inverse-panel work lists, product items and
// zero gather pointers of a dense k x k problem as one front
hipError_t launch_dense_lists(DFront* front, int32_t k, int32_t ns_pad, int32_t Mt, int32_t* diag, int32_t* panel,
                              int32_t* upd, int32_t* qrow, int32_t* qupd, int32_t* prod, int64_t* gptr,
                              hipStream_t s);
hipError_t launch_dense_to_front(const double* A, int32_t k, double* tiles, int32_t Mt, hipStream_t s);
// B = A^T (k x k, row-major, ld = k)
hipError_t launch_transpose(const double* A, int32_t k, double* B, hipStream_t s);
// C[i, j] = 0.5 (A[i,j] + A[j,i]) * w[i] * w[j] with w = D^-1/2 (k x k)
hipError_t launch_sym_scale(const double* A, const double* D, int32_t k, double* C, hipStream_t s);
// One block Jacobi sweep (block size b = 16, m a positive multiple of 2b):
// m / b - 1 rounds in tournament order; in each, every block
// pair's 2b x 2b principal submatrix is diagonalised (at most inner_sweeps
// cyclic sweeps; rotation threshold max(tol_abs_rel * normf[0],
// tol_rel * sqrt(|c_pp c_qq|)), rotations counted into rot_count), then
// C <- J^T C J and V <- V J.  Qs: (m / 2b) (2b)^2 doubles (the pairs'
// orthogonal factors of a round); qrot: m / 2b ints (per pair of the round:
// 0 when no entry was above the threshold, so its factor is the identity and
// the update skips it).
hipError_t launch_bj_sweep(int b, double* C, double* V, int32_t m, double* Qs, const double* normf, double tol_rel,
                           double tol_abs_rel, int32_t inner_sweeps, int32_t* rot_count, int32_t* qrot,
                           hipStream_t s);
// count += number of entries c_pq (p < q) of the symmetric m x m C above the
// rotation threshold of launch_bj_sweep (0: another sweep would not rotate)
hipError_t launch_bj_offcount(const double* C, int32_t m, const double* normf, double tol_rel, double tol_abs_rel,
                              int32_t* count, hipStream_t s);
hipError_t launch_identity(double* V, int32_t m, hipStream_t s);
// C (m x m) = Ck (k x k) plus decoupled dummies (m > k), normf = ||Ck||_F, dis = D^-1/2;
// part: 256 doubles of scratch (partial sums of squares)
hipError_t launch_embed_pad(const double* Ck, int32_t k, int32_t m, double* C, double* normf, double* dis,
                            const double* D, double* part, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
// A (n x n row-major) = dense copy of a CSR matrix
hipError_t launch_densify(const int64_t* ptr, const int32_t* idx, const double* val, int64_t n, double* A,
                          hipStream_t s);
// sort eigenvalues ascending (first k of m), gather the eigenvector columns
// X[r, j] = scale[r] * Y[r, order[j]] and lam_out[j]; Y m x m row-major
hipError_t launch_sort_eig(const double* C, int32_t m, int32_t kvalid, const double* Y, int32_t rows,
                           const double* scale, int32_t kout, double* lam_out, double* X, int64_t ldx,
                           hipStream_t s);
// Y[r, c] = V[r, c] * w[r] (w = D^1/2), for the back transformation
hipError_t launch_row_scale(const double* V, const double* w, bool sqrt_w, int64_t rows, int32_t k, int64_t ld,
                            double* Y, hipStream_t s);

// ratio[c] = ||R_c|| / ||B_c|| over columns [col0, col0 + k) of n-row blocks with leading dim ld
int64_t colnorm_partial_doubles(int64_t n, int32_t k);
hipError_t launch_colnorm_ratio(const double* R, const double* B, int64_t n, int64_t ld, int32_t col0, int32_t k,
                                double* partial, double* ratio, hipStream_t s);

// ------------------------------------------------------------ adjoint helpers
int64_t tsgemm_partial_doubles(int64_t n, int32_t ka, int32_t kb);
// C (ka x kb, row-major) = A^T B
hipError_t launch_tsgemm_tn(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t n, int32_t ka,
                            int32_t kb, double* partial, double* C, hipStream_t s);
// Y = beta Y + alpha A C
hipError_t launch_tsgemm_nn(const double* A, int64_t lda, int64_t n, int32_t ka, const double* C, int32_t kb,
                            double alpha, double beta, double* Y, int64_t ldy, hipStream_t s);
int64_t coldot_partial_doubles(int64_t n, int32_t k);
hipError_t launch_coldot(const double* A, const double* B, int64_t n, int64_t ld, int32_t k, double* partial,
                         double* out, hipStream_t s);
hipError_t launch_shift_cols(double* Y, const double* X, const double* m, const double* lam, int64_t n, int64_t ld,
                             int32_t k, hipStream_t s);
hipError_t launch_axpy_cols(double* Y, const double* X, const double* coef, int mode, int64_t n, int64_t ld, int32_t k,
                            hipStream_t s);
hipError_t launch_div_cols(const double* num, const double* den, double* out, int32_t k, hipStream_t s);
hipError_t launch_bwd_vertex(int64_t nv, int32_t p, const double* X, const double* W, const double* Y, int64_t ld,
                             const int32_t* iperm, const double* lam, const double* glam, const double* rho, double* nu,
                             hipStream_t s);
hipError_t launch_bwd_tri(int64_t nf, const int32_t* F, const double* V, int32_t p, const double* X, const double* W,
                          int64_t ld, const int32_t* iperm, const double* glam, const double* nu, int32_t lumping,
                          double* G, hipStream_t s);
hipError_t launch_bwd_gather(int64_t nv, const int64_t* vt_ptr, const int64_t* vt, const double* G, double* gradV,
                             hipStream_t s);
// out[r, c] = sign[c] * in[c * nv + perm[r]] (sign may be null)
hipError_t launch_import_cols(const double* in, int64_t nv, const int32_t* perm, int64_t n, int32_t k, double* out,
                              int64_t ld, hipStream_t s, const double* sign = nullptr);

// ------------------------------------------------------------ output
// evecs[c * nout + vertex(r)] = sign_c * Phi[r, c] for r < n, c < p (vertex(r) =
// perm[r] < nout; rows of evecs that no r names are left as they are),
// largest-magnitude entry positive (lowest vertex index on ties)
hipError_t launch_export_evecs(const double* Phi, int64_t ld, int64_t n, int32_t p, const int32_t* perm,
                               int64_t nout, double* evecs, double* work, hipStream_t s);

// ------------------------------------------------------------ dense products
// Out (M x N) = alpha op(A) B + beta D (row-major; op(A) = A stored M x K, or
// A^T with A stored K x M; D null or any M x N block, Out may equal D)
hipError_t launch_dgemm(bool transa, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                        const double* B, int64_t ldb, double beta, const double* D, int64_t ldd, double* Out,
                        int64_t ldo, hipStream_t s);
// X = (sigma I - C) / g on the leading k x k block of the m x m C (g the
// Gershgorin bound of C - sigma I there, written to *bound as its bit
// pattern), -1 on the diagonal of the remaining rows, 0 elsewhere
hipError_t launch_ns_init(const double* C, int32_t m, int32_t k, double sigma, unsigned long long* bound, double* X,
                          hipStream_t s);
// out[0] = ||T - I||_F^2 (m x m), out[1] = sum_{i < k} X_ii (X may be null);
// part: 256 doubles of scratch
hipError_t launch_ns_check(const double* T, const double* X, int32_t m, int32_t k, double* part, double* out,
                           hipStream_t s);

}  // namespace hsim

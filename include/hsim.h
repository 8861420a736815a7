/*
 * hsim.h -- C ABI of the MI355X (gfx950) Hierarchical Subspace Iteration
 * Method for the lowest p Laplace-Beltrami eigenpairs S x = lambda M x
 * (cotangent stiffness S, lumped mass M).
 *
 * Method: Nasikun & Hildebrandt, "The Hierarchical Subspace Iteration Method
 * for Laplace-Beltrami Eigenproblems" (ACM TOG).  Section 3.1 defines the
 * discrete problem (eq. massStiffMatrices, eq. eigenProb), Section 3.2 and
 * Algorithm 1 the subspace iteration, Section 4.1 and Algorithm 3 the
 * hierarchy, Section 4.2 and Algorithm 2 the hierarchical solver.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every call returns an hsim_status and never aborts.  On a non-OK status
 *    hsim_last_error() returns a thread-local message; outputs are left
 *    untouched except where a function says otherwise.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are GPU
 *    memory of the device that was current when the hierarchy was built
 *    (the caller allocates them, e.g. as torch tensors).  The caller keeps
 *    ownership of every pointer it passes; host inputs are copied.
 *  - `stream` arguments are hipStream_t values passed as void* (NULL = the
 *    default stream).  Device outputs are complete when the stream reaches
 *    the point after the call; calls that return host values synchronize.
 *  - Floating point is IEEE double unless a parameter says otherwise.
 *  - Dense n x k blocks handed to the step-level entry points (hsim_step_*)
 *    are row-major with leading dimension k ("vertex-major": the k values of
 *    one vertex are contiguous), rows in the level's vertex order (level 0:
 *    mesh order; coarser levels: insertion order of the farthest point
 *    sampling, see hsim_level_export).
 */
#ifndef HSIM_H
#define HSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsim_hierarchy hsim_hierarchy; /* opaque; owns host + device state */

typedef enum {
    HSIM_OK = 0,
    HSIM_E_INVALID = -1,       /* bad argument (null pointer, p out of range, ...) */
    HSIM_E_MESH = -2,          /* mesh not a connected manifold, degenerate triangle, NaN */
    HSIM_E_FACTOR = -3,        /* LDL^T breakdown (zero pivot) that re-shifting did not cure */
    HSIM_E_NOCONV = -4,        /* max_iters reached; outputs hold the last iterate */
    HSIM_E_NOMEM = -5,         /* device or host allocation failed */
    HSIM_E_DEVICE = -6,        /* HIP runtime error */
    HSIM_E_STATE = -7,         /* call out of order (e.g. backward before a solve) */
    HSIM_E_UNIMPLEMENTED = -8
} hsim_status;

/* Options of hsim_build_hierarchy (the hierarchy set-up of Algorithm 2,
 * Algorithm 3, Section 4.1).  hsim_default_build_opts() fills the paper's defaults. */
typedef struct {
    int32_t p;             /* eigenpairs wanted, 1 <= p, q(p) < n                                 */
    int32_t levels;        /* T; 0 = paper rule: 2 if p <= 200 else 3 (Section 4.1)               */
    int32_t n_coarsest;    /* n^{T-1}; 0 = max(ceil(1.5 p), 1000) (eq. nT-1)                      */
    int32_t growth_mode;   /* 0: g = (n0/n^{T-1})^(1/(T-1)); 1: the printed T-th root (eq. growthRate) */
    int32_t lumping;       /* 0: barycentric (row-sum of the consistent mass); 1: circumcentric     */
    double support_sigma;  /* sigma of eq. (radius); default 7                                     */
    uint64_t seed;         /* start vertex of Algorithm 3 = seed mod n                              */
    int32_t flags;         /* HSIM_BUILD_HOST_ONLY: build on the host only (inspection; no solve)   */
    int32_t boundary;      /* mesh boundary (edges of one triangle): 0 natural (Neumann) condition;
                              1 Dirichlet: boundary vertices held at zero, dropped from level 0 (its
                              S, lumped M and the rows of U^0); the coarser levels are sampled and
                              built as without boundary and get their operators from the restricted
                              level 0 (the paper's surfaces-with-boundary experiments use the same
                              hierarchy and basis construction)                                   */
} hsim_build_opts;

enum { HSIM_BUILD_HOST_ONLY = 1 };

/* precision forms of the solve; HSIM_GRAM_COMPENSATED only for hsim_step_gram */
enum { HSIM_FP64 = 0, HSIM_MIXED = 1, HSIM_GRAM_COMPENSATED = 2 };
/* flags of hsim_solve_opts */
enum {
    HSIM_FLAG_NOLOCK = 1,        /* disable locking of converged vectors (Section 4.2) */
    HSIM_FLAG_SAVE_FORWARD = 2,  /* keep what hsim_solve_backward needs (set by the autograd wrapper).
                                    The state it needs (level-0 factor, Ritz vectors and values) stays
                                    resident after every converged solve, so the flag changes nothing. */
    HSIM_FLAG_PROFILE = 4,       /* time every kernel launch with HIP events (fills k_ms / k_launches) */
    HSIM_FLAG_DETERMINISTIC = 8, /* bitwise reproducible results run to run on one device.  Every solve
                                    already is (all reductions run in a fixed order; the kernels use
                                    integer atomics only, for counters): the flag is accepted and
                                    changes nothing.  Unknown flag bits are HSIM_E_INVALID. */
    HSIM_FLAG_COMPENSATED_GRAM = 16, /* HSIM_MIXED: the Rayleigh-Ritz steps that do not use the FP32 Gram
                                    use the compensated FP32 Gram (hi/lo split, three FP32 products,
                                    FP64 sums) instead of the FP64 one; a step whose reduced mass
                                    matrix then has no positive definite factor is redone in FP64 */
    HSIM_FLAG_NO_FP32_GRAM = 32, /* HSIM_MIXED: no FP32 Gram in the iterations far from convergence */
    HSIM_FLAG_FP32_GRAM = 64,    /* HSIM_MIXED: the FP32 Gram in the iterations far from convergence at
                                    any q (by default only for q > 160, where the FP64 Gram is a
                                    multi-pass product as well; below, the single-pass FP64 product is
                                    the faster one on the FP64 matrix cores) */
    HSIM_FLAG_GRAPH = 128        /* HSIM_FP64: the two inverse iterations of a subspace iteration
                                    (every block-solve launch, and the M products on coarse levels) are
                                    captured once per (level, locked columns, buffers) into a HIP graph
                                    kept by the hierarchy and replayed; same results bit for bit.
                                    Ignored with HSIM_FLAG_PROFILE. */
};

/* kernel classes of the profile counters in hsim_stats */
enum {
    HSIM_K_SOLVE_FWD = 0,   /* forward block triangular solve, one launch per tree level      */
    HSIM_K_SOLVE_BWD = 1,   /* backward block triangular solve, one launch per tree level     */
    HSIM_K_FACTOR = 2,      /* numeric factorisation: assembly, extend-add, tile kernels      */
    HSIM_K_GRAM = 3,        /* Rayleigh-Ritz Gram products                                    */
    HSIM_K_RITZ = 4,        /* Ritz update with the fused residual                            */
    HSIM_K_SPMM = 5,        /* CSR products (S, M, prolongation)                              */
    HSIM_K_JACOBI = 6,      /* dense eigenproblems (Cholesky, transforms, Jacobi rounds)      */
    HSIM_K_OTHER = 7,
    HSIM_KCLASSES = 8
};

/* Options of hsim_solve (the multilevel iterations of Algorithm 2, Algorithm 1). */
typedef struct {
    double tol;            /* eps of the convergence test eq. (conv2); paper default 1e-2            */
    double shift_alpha;    /* mu = Ritz value with index floor(alpha p) (Alg. 2, Section 5); 0.1      */
    int32_t precision;     /* HSIM_FP64 or HSIM_MIXED                                                 */
    int32_t max_iters;     /* subspace iterations per level before HSIM_E_NOCONV                      */
    int32_t flags;         /* HSIM_FLAG_*                                                             */
    int32_t reserved;
    void* stream;          /* hipStream_t                                                             */
} hsim_solve_opts;

#define HSIM_MAX_LEVELS 8

/* Statistics of the last hsim_solve (host struct filled by the library). */
typedef struct {
    int32_t levels;
    int32_t q;
    int32_t iters[HSIM_MAX_LEVELS];       /* subspace iterations per level, coarsest first (paper's "F|a|b"; the coarsest is 0 = dense) */
    int64_t n[HSIM_MAX_LEVELS];           /* level sizes, coarsest first                             */
    int64_t nnz_factor[HSIM_MAX_LEVELS];  /* stored factor entries (padded supernodal panels)        */
    int32_t neg_pivots[HSIM_MAX_LEVELS];  /* inertia of S - mu M: number of negative pivots          */
    double mu[HSIM_MAX_LEVELS];           /* shift per level                                         */
    int32_t refine_steps;                 /* mixed precision: total refinement sweeps                */
    int32_t escalated;                    /* mixed precision: levels that fell back to FP64 solves    */
    double ms_build;                      /* host hierarchy build (from hsim_build_hierarchy)         */
    double ms_coarse, ms_factor, ms_solve, ms_gram, ms_rr, ms_ritz, ms_prolong, ms_total;
    /* HSIM_FLAG_PROFILE: device time (HIP events around each launch), launch
     * count, and the algorithmic bytes and flops of those launches (bytes:
     * each operand counted once per launch; flops: the arithmetic of the
     * operation, not of the padding) per kernel class */
    double k_ms[HSIM_KCLASSES];
    int64_t k_launches[HSIM_KCLASSES];
    double k_bytes[HSIM_KCLASSES];
    double k_flops[HSIM_KCLASSES];
    /* block triangular solves (one forward and one backward sweep each, every
     * level and precision) and the right-hand-side columns they covered */
    int64_t block_solves;
    int64_t block_solve_cols;
    /* Rayleigh-Ritz Gram products by form: FP64, FP32, compensated FP32 */
    int32_t gram_steps[3];
    /* of block_solves: those that ran with the FP32 copy of the factor */
    int64_t block_solves_fp32;
} hsim_stats;

/* Per-level sizes (hsim_level_desc). */
typedef struct {
    int64_t n;             /* vertices of the level                                   */
    int64_t nnz;           /* nonzeros of S^tau (M^tau shares the pattern for tau>0)  */
    int64_t nnz_u;         /* nonzeros of U^tau (0 on the coarsest level)             */
    int64_t fronts;        /* supernodes of the factor (0 on the coarsest level)      */
    int64_t tree_levels;   /* height of the supernodal elimination tree               */
    int64_t factor_entries;/* stored factor entries (padded panels)                   */
    double rho;            /* support radius of U^tau (eq. radius); 0 on the coarsest */
    double factor_flops;   /* flops of one numeric factorisation                      */
    int64_t factor_nnz;    /* nonzeros of L (unpadded supernodal panels, incl. diagonal) */
    int64_t qpanel_tree_levels; /* tree levels whose fronts also get inverse panels
                              Q = [L11^-1; -L21 L11^-1] in every factorisation (the block
                              solves may multiply by them instead of substituting)    */
    int64_t qpanel_entries;/* stored inverse-panel values (padded tiles)              */
} hsim_level_desc;

void hsim_default_build_opts(hsim_build_opts* opts);
void hsim_default_solve_opts(hsim_solve_opts* opts);

/*
 * hsim_build_hierarchy -- the set-up part of Algorithm 2 (vertex hierarchy by
 * farthest point sampling, Algorithm 3; prolongations U^tau, eq. radius and
 * eq. basis; Galerkin operators S^tau, M^tau), preceded by the assembly of
 * S^0 and the lumped M^0 (Section 3.1, eq. massStiffMatrices), and followed
 * by the symbolic analysis of the sparse factor of every level.
 *
 *   V        host, [nv x 3] row-major vertex positions
 *   F        host, [nf x 3] row-major triangle vertex indices (0-based)
 *   density  host, [nv] per-vertex factor on the lumped mass, or NULL
 *   opts     host; NULL = defaults (then p must be set: use the defaults
 *            function and set p)
 *   out      receives the new handle; release it with hsim_free
 * The mesh must be a connected, edge-manifold triangle mesh (closed, or with
 * boundary: natural Neumann conditions) without degenerate triangles.
 * Everything needed on the device is uploaded before the call returns.
 */
hsim_status hsim_build_hierarchy(const double* V, int64_t nv, const int32_t* F, int64_t nf,
                                 const double* density, const hsim_build_opts* opts,
                                 hsim_hierarchy** out);

/*
 * hsim_solve -- the solve part of Algorithm 2: dense solve of the coarsest level,
 * then for every finer level prolongation, shift, one LDL^T factorisation of
 * S^tau - mu M^tau and subspace iterations (Algorithm 1 with two inverse
 * iterations per Rayleigh-Ritz step and locking, Section 4.2) until the
 * first p pairs pass eq. (conv2) with eps = opts->tol.
 *
 *   d_evals  device, [p] ascending eigenvalues
 *   d_evecs  device, [nv x p] column-major (eigenvector k contiguous), mesh
 *            vertex order, M-orthonormal; each column's largest-magnitude
 *            entry is positive (lowest index on ties); with the Dirichlet
 *            boundary option the boundary vertices' entries are zero
 *   d_resid  device, [p] final relative residuals (finest level), or NULL
 *   stats    host, or NULL
 * HSIM_E_NOCONV still fills evals/evecs/resid with the last iterate.
 */
hsim_status hsim_solve(hsim_hierarchy* h, const hsim_solve_opts* opts, double* d_evals,
                       double* d_evecs, double* d_resid, hsim_stats* stats);

/*
 * hsim_solve_batch -- hsim_solve for many hierarchies (meshes of uneven
 * size) at once: the solves are spread over `streams` worker streams of the
 * current device (0 = 8), one host thread each, largest meshes first, so the
 * small meshes' latency-bound launches overlap on the GPU.  Every mesh gets
 * exactly the result hsim_solve would give it (same kernels, same order).
 *
 *   hs        host array [count] of hierarchies built on the current device
 *   opts      as for hsim_solve (opts->stream: the workers start after the
 *             caller's stream reaches this call)
 *   d_evals, d_evecs, d_resid  host arrays [count] of device pointers as for
 *             hsim_solve (d_resid may be NULL, or hold NULL entries)
 *   stats     host [count] or NULL; status: host [count] per-mesh status or NULL
 * Returns HSIM_OK when every mesh converged, else the status of the first
 * failing mesh (hsim_last_error names it); all outputs of the other meshes
 * are complete either way.  The call returns when every worker has finished.
 * Two calls that share a hierarchy must not overlap.
 */
hsim_status hsim_solve_batch(hsim_hierarchy* const* hs, int32_t count, const hsim_solve_opts* opts,
                             double* const* d_evals, double* const* d_evecs, double* const* d_resid,
                             hsim_stats* stats, int32_t* status, int32_t streams);

/*
 * hsim_autotune -- choose the launch plan of the block triangular solves of
 * one level (the widest-supernode thresholds, in padded pivots, from which a
 * tree level's forward and backward sweeps multiply by the inverse panels of
 * its fronts, Q = [L11^-1; -L21 L11^-1], instead of running the wave-level
 * matrix-core solve) by timing a q-column block solve of the candidates
 * 64/96/128/256/512 (the forward threshold with the backward one at 128, then
 * the backward threshold with the chosen forward one; tree levels above the
 * leaves whose widest front has at least 64 padded pivots have inverse panels)
 * on a factor of S - mu M with mu below the spectrum, and keep the fastest
 * for the following solves of this hierarchy.  With the environment variable
 * HSIM_TUNE_CACHE naming a file, the choice is looked up there first (keyed
 * by subspace size, tree height, widest front and level size class) and
 * appended after tuning.  Overwrites the level's factor (the next hsim_solve
 * factors again).  out (host, may be NULL) receives the choice.
 */
typedef struct {
    int32_t big_ns, big_ns_bwd;   /* chosen thresholds                                   */
    double ms;                    /* measured time of one q-column block solve           */
    int32_t from_cache;           /* 1: taken from HSIM_TUNE_CACHE without timing        */
} hsim_tune_result;
hsim_status hsim_autotune(hsim_hierarchy* h, int32_t level, void* stream, hsim_tune_result* out);

/*
 * hsim_solve_backward -- vector-Jacobian product of the last hsim_solve
 * (run with HSIM_FLAG_SAVE_FORWARD) with respect to the vertex positions.
 * Eigenvalue part: d lambda_k = x_k^T (dS - lambda_k dM) x_k.  Eigenvector
 * part: the adjoint solve (S - lambda_k M) w_k = -(I - M x_k x_k^T) g_k
 * restricted to the M-orthogonal complement of x_k, reusing the finest-level
 * factor as preconditioner; then the derivative of the cotangent and mass
 * assembly.
 *
 *   d_grad_evals  device, [p] dL/dlambda, or NULL
 *   d_grad_evecs  device, [nv x p] column-major dL/dX, or NULL
 *   d_grad_V      device, [nv x 3] row-major, overwritten with dL/dV
 * Under the Dirichlet option (Section 5, surfaces with boundary) the problem
 * keeps the interior rows and columns of S and M; with the eigenvectors and the
 * adjoint vectors extended by zero the same formulas hold over the whole mesh.
 * The rows of d_grad_evecs at boundary vertices are ignored (those eigenvector
 * entries are fixed at zero); d_grad_V covers every vertex, the boundary ones
 * included, since they move the interior problem's cotangent weights and masses.
 * The mass derivative follows the hierarchy's lumping: area / 3 per vertex
 * (barycentric) or, circumcentric, each corner's cot(theta) |e|^2 / 8 over its
 * opposite edge e to both ends of e.
 * HSIM_E_STATE before a converged hsim_solve on this hierarchy (after none, after
 * one that ended with HSIM_E_NOCONV or another error, or after a step-level call).
 */
hsim_status hsim_solve_backward(hsim_hierarchy* h, const double* d_grad_evals,
                                const double* d_grad_evecs, double* d_grad_V, void* stream);

void hsim_free(hsim_hierarchy* h);
const char* hsim_last_error(void);

/* ---------------------------------------------------------------------------
 * Inspection and step-level entry points.  They expose the hierarchy that
 * hsim_build_hierarchy made and run one step of the hot path at a time, so
 * that every step can be checked against an independent implementation.
 * ------------------------------------------------------------------------- */

/* number of levels T and the subspace size q of a hierarchy */
hsim_status hsim_hierarchy_shape(const hsim_hierarchy* h, int32_t* levels, int32_t* q, int32_t* p);

hsim_status hsim_level_info(const hsim_hierarchy* h, int32_t level, hsim_level_desc* info);

/*
 * hsim_level_export -- copy a level's host data out (any pointer may be NULL
 * to skip it).  Sizes come from hsim_level_info.
 *   verts     [n]      mesh vertex index of every level vertex (level order)
 *   S_indptr  [n+1], S_indices [nnz], S_data [nnz]: S^tau CSR, level order,
 *                      sorted column indices
 *   M_data    [nnz]    M^tau on the same pattern (level 0: the lumped
 *                      diagonal on the diagonal entries, 0 elsewhere)
 *   U_indptr  [n+1], U_indices [nnz_u], U_data [nnz_u]: U^tau CSR, rows =
 *                      level tau vertices, columns = level tau+1 vertices
 *   perm      [n]      elimination order: perm[k] = level vertex eliminated k-th
 */
hsim_status hsim_level_export(const hsim_hierarchy* h, int32_t level, int64_t* verts,
                              int64_t* S_indptr, int32_t* S_indices, double* S_data,
                              double* M_data, int64_t* U_indptr, int32_t* U_indices,
                              double* U_data, int32_t* perm);

/* Prolongation: Phi_fine = U^tau Phi_coarse.  d_coarse [n^{tau+1} x k], d_fine [n^tau x k]
 * (Algorithm 2, prolongation of the subspace basis). */
hsim_status hsim_step_prolong(hsim_hierarchy* h, int32_t level, int32_t k, const double* d_coarse,
                              double* d_fine, void* stream);

/* Operator product: Y = op X with op = 0: S^tau, 1: M^tau, 2: S^tau - mu M^tau (mu of the
 * last hsim_step_factor on this level).  d_X, d_Y [n^tau x k]. */
hsim_status hsim_step_apply(hsim_hierarchy* h, int32_t level, int32_t op, int32_t k, const double* d_X,
                            double* d_Y, void* stream);

/* Numeric LDL^T factorisation of S^tau - mu M^tau (the factorisation in Algorithm 1,
 * static 1x1 pivots on the supernodal elimination tree).  Returns the number
 * of negative pivots (Sylvester inertia: the number of eigenvalues below mu)
 * in *neg_pivots (host, may be NULL); synchronizes. */
hsim_status hsim_step_factor(hsim_hierarchy* h, int32_t level, double mu, int32_t precision,
                             int32_t* neg_pivots, void* stream);

/* Block solve: X = (S^tau - mu M^tau)^-1 B with the factor of the last
 * hsim_step_factor; precision HSIM_MIXED solves in FP32 with FP64 iterative
 * refinement down to the relative residual refine_tol.  d_B, d_X [n^tau x k]
 * (may alias). */
hsim_status hsim_step_solve(hsim_hierarchy* h, int32_t level, int32_t k, const double* d_B, double* d_X,
                            int32_t precision, double refine_tol, void* stream);

/* Rayleigh-Ritz Gram products: Sbar = Psi^T S^tau Psi, Mbar = Psi^T M^tau Psi
 * (the reduced stiffness and mass matrices of Algorithm 1).
 * d_Psi [n^tau x k]; d_Sbar, d_Mbar [k x k] row-major, symmetric.
 * precision HSIM_MIXED takes the low-precision Gram (FP32 MFMA products of
 * rounded copies, FP32 accumulation within 256-row chunks, FP64 sums of the
 * chunks); HSIM_GRAM_COMPENSATED the compensated one (every FP64 operand split
 * into FP32 hi = fl(x) and lo = fl(x - hi), the products hi*hi + hi*lo + lo*hi
 * on the FP32 matrix cores, FP64 sums of every 32 rows). */
hsim_status hsim_step_gram(hsim_hierarchy* h, int32_t level, int32_t k, const double* d_Psi,
                           double* d_Sbar, double* d_Mbar, int32_t precision, void* stream);

/* Reduced dense eigenproblem: Sbar Phibar = Mbar Phibar diag(lam) for symmetric Sbar and SPD
 * Mbar (the dense eigenproblem of Algorithm 1) by Cholesky of the equilibrated Mbar and cyclic
 * Jacobi.  d_lam [k] ascending, d_Phibar [k x k] row-major, Mbar-orthonormal
 * columns.  Returns the Jacobi sweeps in *sweeps (host, may be NULL). */
hsim_status hsim_step_rr(int32_t k, const double* d_Sbar, const double* d_Mbar, double* d_lam,
                         double* d_Phibar, int32_t* sweeps, void* stream);

/*
 * hsim_step_rr_noalloc -- hsim_step_rr for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc.  Same arguments, results and errors as
 * hsim_step_rr (the same kernels run), for k <= HSIM_RR_NOALLOC_MAX_K; larger
 * k is HSIM_E_INVALID.  It calls no hipMalloc or hipFree: its work arrays
 * live in one fixed 4 MiB device region per GPU that the library holds until
 * the process ends (looked up on the first call on each device).  Every call
 * on a device shares that region and overwrites it, so calls that overlap on
 * one device (two host threads, or two streams of one device without
 * ordering) race; calls on different devices do not.  The call synchronizes
 * the stream (it reads pivot and rotation counts back to the host).
 */
#define HSIM_RR_NOALLOC_MAX_K 256
hsim_status hsim_step_rr_noalloc(int32_t k, const double* d_Sbar, const double* d_Mbar, double* d_lam,
                                 double* d_Phibar, int32_t* sweeps, void* stream);

/* Ritz update and residual: Phi = Psi Phibar (the update of Algorithm 1) and the floored relative
 * residual of every column (eq. conv2 in the M^-1 norm on level 0, the
 * Euclidean norm on coarser levels, Section 5), with lam_floor the lambda_c
 * of the floor.  d_Psi [n x k], d_Phibar [k x k], d_lam [k], d_Phi [n x k],
 * d_resid [k]. */
hsim_status hsim_step_ritz(hsim_hierarchy* h, int32_t level, int32_t k, const double* d_Psi,
                           const double* d_Phibar, const double* d_lam, double lam_floor,
                           double* d_Phi, double* d_resid, void* stream);

/* Coarsest level: first k eigenpairs of the coarsest level's dense problem
 * S^{T-1} Phi = M^{T-1} Phi Lambda (Algorithm 2, initial subspace).  d_lam [k],
 * d_Phi [n^{T-1} x k] (M-orthonormal columns); *sweeps (host, may be NULL): the
 * Jacobi sweeps used.  Levels of at least 512 unknowns with k at most half of
 * them compute the k pairs by spectral projection (Newton-Schulz sign of
 * sigma I - C, then Rayleigh-Ritz on the projector's range); smaller ones,
 * larger k, or the environment variable HSIM_COARSE_JACOBI=1 take block
 * Jacobi on the whole level.  Synchronizes the stream. */
hsim_status hsim_step_coarse(hsim_hierarchy* h, int32_t k, double* d_lam, double* d_Phi,
                             int32_t* sweeps, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* HSIM_H */

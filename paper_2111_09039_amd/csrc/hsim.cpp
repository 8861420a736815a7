// HSIM library: hierarchy build, device state, the per-level subspace
// iteration driver (Algorithm 2 with Algorithm 1 inside) and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <thread>
#include <array>
#include <map>
#include <mutex>
#include <numeric>
#include <memory>
#include <random>

#include "internal.h"
#include "build_dev.h"
#include "kernels.h"

namespace hsim {

// ============================================================== errors
static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

void fail(hsim_status code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error{code, buf};
}

#define HIPCHECK(expr)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) fail(HSIM_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

// ========================================================== device memory
DeviceBuffer::~DeviceBuffer() { release(); }
void DeviceBuffer::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}
void DeviceBuffer::alloc(size_t nbytes) {
    if (nbytes <= bytes && p) return;
    release();
    if (nbytes == 0) return;
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
        p = nullptr;
        fail(HSIM_E_NOMEM, "hipMalloc(%zu) failed: %s", nbytes, hipGetErrorString(e));
    }
    bytes = nbytes;
}
void DeviceBuffer::copy_in(const void* src, size_t nbytes) {
    if (nbytes == 0) return;
    HIPCHECK(hipMemcpy(p, src, nbytes, hipMemcpyHostToDevice));
}

template <class T>
static T* dptr(DeviceBuffer& b) { return b.as<T>(); }

static inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

int env_int(const char* name, int dflt) {
    const char* e = getenv(name);
    if (!e || !*e) return dflt;
    char* end = nullptr;
    const long v = strtol(e, &end, 10);
    return (end && *end == 0) ? (int)v : dflt;
}

// ============================================================ profiling
// HIP events around every launch of a kernel class (only when asked for).
struct Prof {
    bool on = false;
    struct Rec {
        hipEvent_t a, b;
        int cls;
        double bytes, flops;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    ~Prof() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
    hipEvent_t get() {
        if (used == pool.size()) {
            hipEvent_t e;
            HIPCHECK(hipEventCreate(&e));
            pool.push_back(e);
        }
        return pool[used++];
    }
    void reset(bool enable) {
        on = enable;
        solves = solve_cols = solves32 = 0;
        used = 0;
        recs.clear();
    }
    template <class F>
    void run(int cls, double bytes, double flops, hipStream_t s, F&& f) {
        if (!on) {
            f();
            return;
        }
        hipEvent_t a = get(), b = get();
        HIPCHECK(hipEventRecord(a, s));
        f();
        HIPCHECK(hipEventRecord(b, s));
        recs.push_back({a, b, cls, bytes, flops});
    }
    // block solves since reset (counted with or without profiling), those with the FP32 factor
    int64_t solves = 0, solve_cols = 0, solves32 = 0;
    void collect(hsim_stats& st, hipStream_t s) {
        st.block_solves = solves;
        st.block_solve_cols = solve_cols;
        st.block_solves_fp32 = solves32;
        if (!on) return;
        HIPCHECK(hipStreamSynchronize(s));
        for (const Rec& r : recs) {
            float ms = 0;
            HIPCHECK(hipEventElapsedTime(&ms, r.a, r.b));
            st.k_ms[r.cls] += ms;
            st.k_launches[r.cls] += 1;
            st.k_bytes[r.cls] += r.bytes;
            st.k_flops[r.cls] += r.flops;
        }
        recs.clear();
        used = 0;
    }
};

// ====================================================== dense eigenproblem
// First kout eigenpairs of S x = lambda M x for k x k dense symmetric S and SPD M
// (row-major, device): equilibration E = diag(M)^-1/2, LDL^T of E M E by the
// tiled front kernels (with the inverse panel P = L^-1 of the one front),
// C = D^-1/2 P (E S E) P^T D^-1/2 by two products, cyclic Jacobi on C,
// X = E P^T D^-1/2 V by a third.
struct DenseGEP {
    static constexpr int32_t MAX_SWEEPS = 40;   // at most this many Jacobi sweeps
    int32_t k = 0, m = 0, ns_pad = 0, Mt = 0, bj = 16;
    std::vector<int64_t> diag_ptr, panel_ptr, upd_ptr, qrow_ptr, qupd_ptr;
    int64_t nprod = 0;   // product items (0, I): the 32-row tiles of the k rows
    // device work arrays: owned (setup) or carved from a caller's region (setup_in)
    DeviceBuffer store;
    DFront* front = nullptr;
    double *tiles = nullptr, *linv = nullptr, *D = nullptr, *qinvT = nullptr, *qinv = nullptr;
    double *S2 = nullptr, *M2 = nullptr, *e = nullptr, *W = nullptr, *W2 = nullptr, *C = nullptr, *V = nullptr,
           *Qs = nullptr, *dis = nullptr, *normf = nullptr;
    int32_t *items_diag = nullptr, *items_panel = nullptr, *items_upd = nullptr, *items_qrow = nullptr,
            *items_qupd = nullptr, *items_prod = nullptr, *counters = nullptr, *qrot = nullptr, *rot = nullptr;
    int64_t* gptr = nullptr;
    bool owned = false;

    // host-side shape: sizes and work-list offsets
    void shape(int32_t kk) {
        k = kk;
        bj = 16;                                       // block Jacobi block size
        m = (int32_t)round_up(k, 2 * bj);
        ns_pad = (int32_t)round_up(k, NB);
        Mt = ns_pad / NB;
        diag_ptr = {0};
        panel_ptr = {0};
        upd_ptr = {0};
        qrow_ptr = {0};
        qupd_ptr = {0};
        int64_t nd = 0, np = 0, nu = 0, nqr = 0, nqu = 0;
        for (int32_t st = 0; st < Mt; ++st) {
            nd += 1;
            np += Mt - 1 - st;
            for (int32_t J = st + 1; J < Mt; ++J) nu += Mt - J;
            nqr += st + 1;
            nqu += (int64_t)(Mt - 1 - st) * (st + 1);
            diag_ptr.push_back(nd);
            panel_ptr.push_back(np);
            upd_ptr.push_back(nu);
            qrow_ptr.push_back(nqr);
            qupd_ptr.push_back(nqu);
        }
        nprod = Mt;
    }

    // carve the work arrays out of [base, base + cap) (256-byte aligned pieces);
    // returns the bytes used (also when base is null: sizing only)
    size_t carve(char* base, size_t cap) {
        size_t off = 0;
        auto take = [&](size_t bytes) -> char* {
            char* q = base ? base + off : nullptr;
            off += (bytes + 255) / 256 * 256;
            return q;
        };
        const size_t d8 = sizeof(double), kk2 = (size_t)k * k * d8, mm2 = (size_t)m * m * d8;
        const size_t tile_bytes = (size_t)Mt * (Mt + 1) / 2 * NB * NB * d8;
        front = reinterpret_cast<DFront*>(take(sizeof(DFront)));
        tiles = reinterpret_cast<double*>(take(tile_bytes));
        linv = reinterpret_cast<double*>(take((size_t)Mt * NB * NB * d8));
        D = reinterpret_cast<double*>(take((size_t)ns_pad * d8));
        qinvT = reinterpret_cast<double*>(take(tile_bytes));
        qinv = reinterpret_cast<double*>(take(tile_bytes));
        S2 = reinterpret_cast<double*>(take(kk2));
        M2 = reinterpret_cast<double*>(take(kk2));
        W = reinterpret_cast<double*>(take(kk2));
        W2 = reinterpret_cast<double*>(take(kk2));
        e = reinterpret_cast<double*>(take((size_t)k * d8));
        dis = reinterpret_cast<double*>(take((size_t)m * d8));
        C = reinterpret_cast<double*>(take(mm2));
        V = reinterpret_cast<double*>(take(mm2));
        Qs = reinterpret_cast<double*>(take((size_t)(m / (2 * bj)) * (2 * bj) * (2 * bj) * d8));
        normf = reinterpret_cast<double*>(take(2 * d8));
        gptr = reinterpret_cast<int64_t*>(take((size_t)(k + 1) * sizeof(int64_t)));
        items_diag = reinterpret_cast<int32_t*>(take((size_t)std::max<int64_t>(1, diag_ptr.back()) * 4));
        items_panel = reinterpret_cast<int32_t*>(take((size_t)std::max<int64_t>(1, panel_ptr.back()) * 2 * 4));
        items_upd = reinterpret_cast<int32_t*>(take((size_t)std::max<int64_t>(1, upd_ptr.back()) * 3 * 4));
        items_qrow = reinterpret_cast<int32_t*>(take((size_t)std::max<int64_t>(1, qrow_ptr.back()) * 2 * 4));
        items_qupd = reinterpret_cast<int32_t*>(take((size_t)std::max<int64_t>(1, qupd_ptr.back()) * 3 * 4));
        items_prod = reinterpret_cast<int32_t*>(take((size_t)std::max<int64_t>(1, nprod) * 2 * 4));
        counters = reinterpret_cast<int32_t*>(take(4 * 4));
        qrot = reinterpret_cast<int32_t*>(take((size_t)(m / (2 * bj)) * 4));
        rot = reinterpret_cast<int32_t*>(take(4 * 4));
        if (base && off > cap) fail(HSIM_E_INVALID, "dense eigenproblem work arrays need %zu bytes, %zu available", off, cap);
        return off;
    }

    // owned work arrays (allocated here, kept for the next call of the same size)
    void setup(int32_t kk, hipStream_t s) {
        if (k == kk && owned) return;
        shape(kk);
        const size_t need = carve(nullptr, 0);
        store.alloc(need);
        carve(static_cast<char*>(store.p), store.bytes);
        owned = true;
        fill_lists(s);
    }

    // work arrays in the caller's device region [base, base + cap): allocates nothing
    void setup_in(int32_t kk, char* base, size_t cap, hipStream_t s) {
        shape(kk);
        carve(base, cap);
        owned = false;
        fill_lists(s);
    }

    // the front descriptor, the tile work lists (factorisation, inverse panel,
    // products) and the (empty) gather pointers, written on the device
    void fill_lists(hipStream_t s) {
        HIPCHECK(launch_dense_lists(front, k, ns_pad, Mt, items_diag, items_panel, items_upd, items_qrow, items_qupd,
                                    items_prod, gptr, s));
        HIPCHECK(hipStreamSynchronize(s));
    }

    void factor(hipStream_t s) {
        HIPCHECK(launch_fill_i32(counters, 4, 0, s));
        HIPCHECK(launch_fill(qinvT, (int64_t)Mt * (Mt + 1) / 2 * NB * NB, 0.0, s));
        for (int32_t st = 0; st < Mt; ++st) {
            HIPCHECK(launch_fac_diag(tiles, linv, D, front, items_diag + diag_ptr[st], diag_ptr[st + 1] - diag_ptr[st],
                                     st, counters, s));
            HIPCHECK(launch_fac_panel(tiles, linv, D, front, items_panel + 2 * panel_ptr[st],
                                      panel_ptr[st + 1] - panel_ptr[st], st, s, qinvT,
                                      items_qrow + 2 * qrow_ptr[st], qrow_ptr[st + 1] - qrow_ptr[st]));
            HIPCHECK(launch_fac_update(tiles, D, front, items_upd + 3 * upd_ptr[st], upd_ptr[st + 1] - upd_ptr[st], st,
                                       s, qinvT, items_qupd + 3 * qupd_ptr[st], qupd_ptr[st + 1] - qupd_ptr[st]));
        }
        HIPCHECK(launch_tile_transpose<double>(qinvT, qinv, (int64_t)Mt * (Mt + 1) / 2, s));
    }

    // Y = L^-1 X (forward) or Y = L^-T X (backward; no D^-1: the caller
    // scales), X and Y n x ncols row-major with leading dimension ld, X != Y
    void fwd(const double* X, double* Y, int32_t ncols, int64_t ld, hipStream_t s) {
        HIPCHECK(launch_qsolve<double>(1, qinv, qinvT, D, front, items_prod, nprod, const_cast<double*>(X), ld, Y, ld,
                                       0, ncols, nullptr, 0, nullptr, 0, nullptr, nullptr, s, nullptr, Mt));
    }
    void bwd(const double* X, double* Y, int32_t ncols, int64_t ld, hipStream_t s) {
        HIPCHECK(launch_qsolve<double>(3, qinv, qinvT, D, front, items_prod, nprod, const_cast<double*>(X), ld, Y, ld,
                                       0, ncols, nullptr, 0, nullptr, 0, nullptr, nullptr, s, nullptr, Mt));
    }

    // returns the Jacobi sweeps used, or -1 when dM is not numerically
    // positive definite (nothing else is computed then).  sigma > 0 (owned
    // work arrays, k >= PROJ_MIN_K, kout <= k / 2): an estimate of an
    // eigenvalue a little above the kout-th, for the spectral projection
    int32_t run(const double* dS, const double* dM, int32_t kout, double* lam_out, double* X, int64_t ldx,
                hipStream_t s, int32_t max_sweeps = 40, double sigma = 0.0);

    // ---- spectral projection (large problems that want few eigenpairs)
    // The projector P = (I + sign(sigma I - C)) / 2 onto the eigenvectors of C
    // below sigma by the Newton-Schulz iteration X <- X (3 I - X^2) / 2 (only
    // matrix products), its rank cnt = trace P, a basis Y = P G of its range
    // (G a fixed Gaussian block), and the lowest kout eigenpairs of C from
    // the Rayleigh-Ritz problem on span Y, solved twice (the second time on
    // the first pass's Ritz basis, whose Gram matrix is close to I).
    static constexpr int32_t PROJ_MIN_K = 512;
    static constexpr int32_t NS_MAX_IT = 80;
    DeviceBuffer pstore;
    int32_t pm = 0;   // m the projection arrays are sized for
    double *PX = nullptr, *PT = nullptr, *PXn = nullptr, *PG = nullptr, *PY = nullptr, *PCY = nullptr,
           *PY2 = nullptr, *PA = nullptr, *PB = nullptr, *PW = nullptr, *plam = nullptr, *ppart = nullptr,
           *pout = nullptr;
    unsigned long long* pbound = nullptr;
    std::unique_ptr<DenseGEP> sub;
    int32_t ns_iters = 0, proj_rank = 0;   // of the last projection (0: not used)
    void setup_proj();
    // lowest kout eigenpairs of C (V: m x kout, orthonormal) or -1 (the caller
    // falls back to the Jacobi sweeps); returns the Jacobi sweeps of the two
    // Rayleigh-Ritz problems
    int32_t project(int32_t kout, double sigma, double* lam_out, double* Vout, hipStream_t s);
};


int32_t DenseGEP::run(const double* dS, const double* dM, int32_t kout, double* lam_out, double* X, int64_t ldx,
                      hipStream_t s, int32_t max_sweeps, double sigma) {
    HIPCHECK(launch_equilibrate(dS, dM, k, S2, M2, e, s));
    HIPCHECK(launch_dense_to_front(M2, k, tiles, Mt, s));
    factor(s);
    // the (equilibrated) mass matrix must be positive definite: a negative,
    // zero or non-finite pivot is reported to the caller (-1), nothing is
    // returned from a reduction through D^-1/2 of such a factor.  The pivot
    // counts go to rot[2..3] and are read with the first synchronisation (the
    // steps up to it only compute; NaN from a failed factor stops no kernel)
    HIPCHECK(hipMemcpyAsync(rot + 2, counters, 2 * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    const bool try_proj = sigma > 0 && owned && k >= PROJ_MIN_K && 2 * kout <= k;
    if (try_proj) {
        int32_t piv[2] = {0, 0};
        HIPCHECK(hipMemcpyAsync(piv, rot + 2, sizeof(piv), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        if (piv[0] > 0 || piv[1] > 0) return -1;
    }
    // W = L^-1 S', W2 = W^T, W = L^-1 W2 = L^-1 S' L^-T
    fwd(S2, W, k, k, s);
    HIPCHECK(launch_transpose(W, k, W2, s));
    fwd(W2, W, k, k, s);
    // C = D^-1/2 W D^-1/2 (symmetrised) embedded in m x m; dis = D^-1/2
    HIPCHECK(launch_sym_scale(W, D, k, W2, s));
    HIPCHECK(launch_embed_pad(W2, k, m, C, normf, dis, D, Qs, s));   // Qs (>= 1024 doubles) free until the sweeps
    ns_iters = proj_rank = 0;
    if (try_proj) {
        // V (m x kout) = the lowest kout eigenvectors of C, then the same back
        // transformation as below
        const int32_t sw = project(kout, sigma, lam_out, V, s);
        if (sw >= 0) {
            HIPCHECK(launch_row_scale(V, dis, false, k, kout, kout, W, s));
            bwd(W, W2, kout, kout, s);
            HIPCHECK(launch_diag_scale(e, k, W2, kout, kout, X, ldx, s));
            return sw;
        }
    }
    HIPCHECK(launch_identity(V, m, s));
    const double tol_rel = 1e-15, tol_abs_rel = 1e-17;
    int32_t sweeps = 0;
    max_sweeps = std::min(max_sweeps, MAX_SWEEPS);
    // a sweep ends the iteration when it rotated nothing or when no entry is
    // left above the threshold (the next sweep would rotate nothing).  The
    // first sweep's counts are not read: a second sweep after one that
    // converged rotates nothing and changes no entry, so the result is the
    // same, and the host waits once less
    for (sweeps = 1; sweeps <= max_sweeps; ++sweeps) {
        HIPCHECK(launch_fill_i32(rot, 2, 0, s));
        HIPCHECK(launch_bj_sweep(bj, C, V, m, Qs, normf, tol_rel, tol_abs_rel, 1, rot, qrot, s));
        HIPCHECK(launch_bj_offcount(C, m, normf, tol_rel, tol_abs_rel, rot + 1, s));
        if (sweeps == 1 && max_sweeps > 1) continue;
        int32_t cnt[4] = {0, 0, 0, 0};
        HIPCHECK(hipMemcpyAsync(cnt, rot, sizeof(cnt), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        if (cnt[2] > 0 || cnt[3] > 0) return -1;   // the pivot counts of the factor
        if (cnt[0] == 0 || cnt[1] == 0) break;
    }
    // Y = D^-1/2 V (sorted, first kout columns), X' = L^-T Y, X = E X'
    HIPCHECK(launch_sort_eig(C, m, m, V, k, dis, kout, lam_out, W, kout, s));
    bwd(W, W2, kout, kout, s);
    HIPCHECK(launch_diag_scale(e, k, W2, kout, kout, X, ldx, s));
    return std::min(sweeps, max_sweeps);
}

void DenseGEP::setup_proj() {
    if (pm == m) return;
    const size_t mm = (size_t)m * m;
    // X, T, Xn, G, Y, C Y, Y2: m x m each (Y blocks use at most k <= m columns);
    // A, B, W: m x m each (Rayleigh-Ritz problems of at most m unknowns)
    const size_t doubles = 10 * mm + (size_t)m + 256 + 8;
    pstore.alloc(doubles * sizeof(double) + 256);
    double* b = pstore.as<double>();
    PX = b;
    PT = PX + mm;
    PXn = PT + mm;
    PG = PXn + mm;
    PY = PG + mm;
    PCY = PY + mm;
    PY2 = PCY + mm;
    PA = PY2 + mm;
    PB = PA + mm;
    PW = PB + mm;
    plam = PW + mm;
    ppart = plam + m;
    pout = ppart + 256;
    pbound = reinterpret_cast<unsigned long long*>(pout + 4);
    // G: a fixed Gaussian block (seeded; the same for every call of this size)
    std::vector<double> g(mm);
    std::mt19937_64 rng(0x5eed0000ULL + (uint64_t)m);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (double& v : g) v = nd(rng);
    HIPCHECK(hipMemcpy(PG, g.data(), mm * sizeof(double), hipMemcpyHostToDevice));
    if (!sub) sub.reset(new DenseGEP());
    pm = m;
}

int32_t DenseGEP::project(int32_t kout, double sigma, double* lam_out, double* Vout, hipStream_t s) {
    setup_proj();
    // HSIM_VERBOSE=2: the time of every phase (with a synchronisation after each)
    const bool timed = env_int("HSIM_VERBOSE", 0) >= 2;
    auto tp = std::chrono::steady_clock::now();
    auto phase = [&](const char* name) {
        if (!timed) return;
        HIPCHECK(hipStreamSynchronize(s));
        const auto now = std::chrono::steady_clock::now();
        fprintf(stderr, "[hsim projection] %-24s %8.3f ms\n", name, std::chrono::duration<double, std::milli>(now - tp).count());
        tp = now;
    };
    double host[2] = {0, 0};
    auto readback = [&] {
        HIPCHECK(hipMemcpyAsync(host, pout, sizeof(host), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
    };
    int32_t cnt = 0;
    for (int attempt = 0; attempt < 4; ++attempt) {
        // sign(sigma I - C) by the scaled Newton-Schulz iteration: T = X^2,
        // X <- a X (3 I - a^2 T) / 2 with a = sqrt(3 / (1 + l + l^2)) for an
        // assumed lower bound l of |eigenvalues of X| (Chen and Chow's scaling:
        // [l, 1] goes to [l', 1], nothing grows past 1, smaller values grow by
        // at least 1.5 a per step; a -> 1 as l -> 1, the plain quadratically
        // convergent step).  The deviation ||X^2 - I||_F is checked every
        // second step from step 10; once below 1e-5 two more plain steps bring
        // it to rounding level.
        HIPCHECK(launch_ns_init(C, m, k, sigma, pbound, PX, s));
        double lb = 1e-6;
        int32_t it = 0, extra = -1;
        for (it = 0; it < NS_MAX_IT; ++it) {
            HIPCHECK(launch_dgemm(false, m, m, m, 1.0, PX, m, PX, m, 0.0, nullptr, 0, PT, m, s));
            if (extra < 0 && it >= 10 && it % 2 == 0) {
                HIPCHECK(launch_ns_check(PT, nullptr, m, k, ppart, pout, s));
                readback();
                if (!std::isfinite(host[0])) break;
                if (std::sqrt(host[0]) < 1e-5) {
                    extra = 2;
                    lb = 1.0;   // the plain step from here (a = 1 keeps 1 fixed)
                }
            }
            if (extra == 0) break;
            const double a = std::sqrt(3.0 / (1.0 + lb + lb * lb));
            HIPCHECK(launch_dgemm(false, m, m, m, -0.5 * a * a * a, PX, m, PT, m, 1.5 * a, PX, m, PXn, m, s));
            lb = std::min(1.0, 0.5 * a * lb * (3.0 - a * a * lb * lb));
            std::swap(PX, PXn);
            if (extra > 0) --extra;
        }
        ns_iters = it;
        if (extra != 0) return -1;   // not converged: the caller runs the Jacobi sweeps
        // rank of P = (k + trace of X over the leading block) / 2
        HIPCHECK(launch_ns_check(PT, PX, m, k, ppart, pout, s));
        readback();
        cnt = (int32_t)std::lround(0.5 * (k + host[1]));
        if (cnt < kout + 1) {
            sigma *= std::max(1.25, 1.3 * (kout + 8) / std::max(cnt, 1));
            continue;
        }
        if (cnt > std::min<int32_t>(k / 2 + kout / 2, 3 * kout)) {
            sigma *= std::max(0.5, 1.3 * (kout + 8) / (double)cnt);
            continue;
        }
        break;
    }
    if (cnt < kout + 1 || cnt > k) return -1;
    proj_rank = cnt;
    phase("sign iteration + rank");
    // Y = P G = (G + X G) / 2 (m x cnt), first Rayleigh-Ritz problem (Y^T C Y, Y^T Y)
    HIPCHECK(launch_dgemm(false, m, cnt, m, 0.5, PX, m, PG, m, 0.5, PG, m, PY, cnt, s));
    auto rayleigh_ritz = [&](const double* Yb, int32_t kk, double* lam, double* Wout) {
        HIPCHECK(launch_dgemm(false, m, cnt, m, 1.0, C, m, Yb, cnt, 0.0, nullptr, 0, PCY, cnt, s));
        HIPCHECK(launch_dgemm(true, cnt, cnt, m, 1.0, Yb, cnt, PCY, cnt, 0.0, nullptr, 0, PA, cnt, s));
        HIPCHECK(launch_dgemm(true, cnt, cnt, m, 1.0, Yb, cnt, Yb, cnt, 0.0, nullptr, 0, PB, cnt, s));
        sub->setup(cnt, s);
        return sub->run(PA, PB, kk, lam, Wout, kk, s);
    };
    const int32_t sw1 = rayleigh_ritz(PY, cnt, plam, PW);
    if (sw1 < 0) return -1;
    phase("first Rayleigh-Ritz");
    // second problem on the Ritz basis Y2 = Y W (its Gram matrix is close to I)
    HIPCHECK(launch_dgemm(false, m, cnt, cnt, 1.0, PY, cnt, PW, cnt, 0.0, nullptr, 0, PY2, cnt, s));
    const int32_t sw2 = rayleigh_ritz(PY2, kout, lam_out, PW);
    if (sw2 < 0) return -1;
    HIPCHECK(launch_dgemm(false, m, kout, cnt, 1.0, PY2, cnt, PW, kout, 0.0, nullptr, 0, Vout, kout, s));
    phase("second Rayleigh-Ritz");
    return sw1 + sw2;
}

// ============================== reduced eigenproblem without allocation
// Work arrays of hsim_step_rr_noalloc: one fixed region per device, sized
// for HSIM_RR_NOALLOC_MAX_K unknowns (4.17 MB used of 4 MiB), held until the
// process ends.  Host code never names the array in a kernel argument or a
// copy: it takes the device address from hipGetSymbolAddress, once per
// device, with that device current.
constexpr size_t RR_SCRATCH_BYTES = size_t(4) << 20;
static __device__ __align__(256) char scratch[RR_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::vector<char*> g_scratch_ptr;   // per device ordinal

static char* rr_scratch_ptr() {
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            fail(HSIM_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<char*>(ptr);
    }
    return g_scratch_ptr[dev];
}

// ================================================================ levels
// tree levels whose widest supernode has at least this many (padded) pivots
// solve through the inverse panels of their fronts (forward sweep)
constexpr int32_t BIG_NS = 256;
// the backward sweep switches earlier (its wave-level form reduces over all
// struct rows of a front in one wave)
constexpr int32_t BIG_NS_BWD = 128;
// tree levels above the leaves whose widest supernode has at least this many
// padded pivots get inverse panels in every factorisation (the plans choose
// among them); the leaf level holds the largest share of the factor and keeps
// the wave-level solves unless its fronts are too wide for them
constexpr int32_t QPANEL_MIN_NS = 64;

struct TLev {
    int32_t f0 = 0, f1 = 0, ns_pad_max = 0;
    // inverse panels: q (the level's fronts have them), and whether the
    // forward / backward sweep uses them in the current plan; item lists in
    // Level::q_items: gather (front, 32-row tile), forward product (front,
    // 16-row tile), backward product (front, 16-row pivot tile)
    bool q = false, big_fwd = false, big_bwd = false;
    int64_t q_gather[2] = {0, 0}, q_fprod[2] = {0, 0}, q_bprod[2] = {0, 0};   // [offset (ints), count]
    int32_t q_kf = 0, q_kb = 0;   // longest contraction (tiles) of the forward / backward products
    double l_entries = 0, pivots = 0;    // unpadded L entries and pivot rows of the level's fronts
    int32_t step0 = 0, step1 = 0;
    std::vector<int32_t> ea_tile_cols;   // per child slot: max tile columns of the children's update blocks
};

struct Level {
    int32_t tau = 0;
    int64_t n = 0;
    bool coarsest = false;
    std::vector<int32_t> verts;          // mesh vertex of every level vertex
    Csr S;                               // level order
    std::vector<double> Mval;            // on S's pattern
    std::vector<double> mdiag;           // level 0 only
    Csr U;                               // rows: this level, cols: next coarser level (level order)
    double rho = 0;
    Symbolic sy;
    std::vector<TLev> tl;
    // device, internal (elimination) order
    DeviceBuffer dS_ptr, dS_idx, dS_val, dM_val, dmdiag, dU_ptr, dU_idx, dU_val, dperm;
    DeviceBuffer dmeshmap;   // level 0: mesh vertex of every internal row
    DeviceBuffer dfronts, tiles, linv, D, tiles32, linv32, D32, counters;
    DeviceBuffer tilesT, linvT, tiles32T, linv32T;   // tile-transposed copies for the backward sweeps
    // inverse panels of the fronts on tree levels with TLev::q: transposed
    // tiles (written by the factorisation), column-major tiles, FP32 mirrors;
    // their work items per factorisation step; the solves' scratch block
    DeviceBuffer qinvT, qinv, qinv32, qinv32T, it_qrow, it_qupd, q_items, qrhs;
    int64_t q_doubles = 0, qrhs_rows = 0;
    std::vector<int64_t> qrow_ptr, qupd_ptr;   // per step: row items (pairs), update items (triples)
    DeviceBuffer asm_dst, asm_src, it_diag, it_panel, it_upd, it_ea, rel, rows, gat;
    int32_t gw = 0;   // width of the padded gather table
    DeviceBuffer ubuf;
    int32_t big_ns = 0, big_ns_bwd = 0;   // thresholds of the current block-solve plan
    double mu = 0;
    bool factored = false, factored32 = false;
    int32_t neg_pivots = 0;
};

}  // namespace hsim

struct hsim_hierarchy {
    int device = 0;
    int32_t p = 0, q = 0, T = 0, ld = 0;
    int64_t gram_chunk = 1024;   // rows per workgroup of the multi-pass Gram
    hsim_build_opts bo{};
    hsim::Mesh mesh;
    std::vector<double> density;
    double area = 0, ms_build = 0;
    std::vector<std::unique_ptr<hsim::Level>> lv;
    hsim::DenseGEP rr, coarse;
    // solve workspace (sized for level 0)
    hsim::DeviceBuffer Phi, Psi, SPsi, MPsi, Btmp, R, Xc, gram_part, ritz_part, Sbar, Mbar, lam, Phibar, resid,
        coarseS, coarseM, exportw, cPhi, cPhi2, cn_part, cn_ratio;
    // adjoint state (allocated by the first hsim_solve_backward)
    hsim::DeviceBuffer bV, bF, bRho, bIperm, bVtPtr, bVt, bG, bNu, bGbar, bMX, bW, bY, bR, bZ, bP, bQ, bSmall, bPart,
        bDots;
    bool bw_ready = false;
    int32_t cg_iters = 0;
    bool solved = false, host_only = false;
    int32_t gram_steps[3] = {0, 0, 0};   // Rayleigh-Ritz Gram products per form in the last solve
    std::vector<double> last_lam;
    hsim::Prof prof;
    // HSIM_FLAG_GRAPH: instantiated graphs of the block solves of one subspace
    // iteration, keyed by level, locked columns and the buffers they read and write
    std::map<std::array<intptr_t, 5>, hipGraphExec_t> graphs;
    hipStream_t cap_stream = nullptr;   // capture stream of those graphs
    ~hsim_hierarchy() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

namespace hsim {

// ----------------------------------------------------------- build helpers
// Launch plan of the block solves on one level: per tree level the fronts,
// the tile and pivot counts, and whether the forward / backward sweep of the
// level goes through the inverse panels (widest front at least big_ns /
// big_ns_bwd padded pivots, or wider than the wave-level solve holds; only
// levels that have inverse panels).  Re-planned by the autotuner.
static void plan_solve(Level& L, int32_t big_ns, int32_t big_ns_bwd) {
    L.big_ns = big_ns;
    L.big_ns_bwd = big_ns_bwd;
    for (TLev& T : L.tl) {
        const bool wide = T.ns_pad_max > wsolve_max_ns();
        T.big_fwd = T.q && (wide || T.ns_pad_max >= big_ns);
        T.big_bwd = T.q && (wide || T.ns_pad_max >= big_ns_bwd);
    }
}

// Tree levels, inverse-panel layout (q_base, qrow of every front, the
// factorisation's row and update items per step, the solves' item lists) of
// one level; df: the device front descriptors being built.
static void setup_tree_levels(hsim_hierarchy* H, Level& L, std::vector<DFront>& df) {
    const Symbolic& sy = L.sy;
    const int32_t mc = std::max<int32_t>(1, sy.max_children);
    L.tl.assign(sy.tree_levels, TLev());
    int64_t qoff = 0;
    std::vector<int32_t> qrow_it, qupd_it, qitems;
    L.qrow_ptr.assign(1, 0);
    L.qupd_ptr.assign(1, 0);
    L.qrhs_rows = 0;
    for (int32_t t = 0; t < sy.tree_levels; ++t) {
        TLev& T = L.tl[t];
        T.f0 = sy.tlev_ptr[t];
        T.f1 = sy.tlev_ptr[t + 1];
        for (int32_t i = T.f0; i < T.f1; ++i) {
            const Front& f = sy.fronts[i];
            T.ns_pad_max = std::max(T.ns_pad_max, f.ns_pad);
            T.l_entries += (double)f.ns * (f.ns + 1) / 2 + (double)f.ns * f.mu;
            T.pivots += f.ns;
        }
        T.q = (t > 0 && T.ns_pad_max >= QPANEL_MIN_NS) || T.ns_pad_max > wsolve_max_ns();
        T.step0 = sy.step_ptr[t];
        T.step1 = sy.step_ptr[t + 1];
        int64_t qrow = 0;
        for (int32_t i = T.f0; i < T.f1; ++i) {
            const Front& f = sy.fronts[i];
            df[i].q_base = -1;
            df[i].qrow = 0;
            if (!T.q) continue;
            df[i].q_base = qoff;
            df[i].qrow = qrow;
            qoff += ((int64_t)f.nsb * f.Mt - (int64_t)f.nsb * (f.nsb - 1) / 2) * NB * NB;
            qrow += (int64_t)NB * f.Mt;
        }
        L.qrhs_rows = std::max(L.qrhs_rows, qrow);
        // factorisation items of the inverse panels, per pivot tile step k
        for (int32_t k = 0; k < T.step1 - T.step0; ++k) {
            if (T.q)
                for (int32_t i = T.f0; i < T.f1; ++i) {
                    const Front& f = sy.fronts[i];
                    if (f.nsb <= k) continue;
                    for (int32_t j = 0; j <= k; ++j) {
                        qrow_it.push_back(i);
                        qrow_it.push_back(j);
                    }
                    for (int32_t I = k + 1; I < f.Mt; ++I)
                        for (int32_t j = 0; j <= k; ++j) {
                            qupd_it.push_back(i);
                            qupd_it.push_back(I);
                            qupd_it.push_back(j);
                        }
                }
            L.qrow_ptr.push_back((int64_t)qrow_it.size() / 2);
            L.qupd_ptr.push_back((int64_t)qupd_it.size() / 3);
        }
        if (T.q) {
            auto push = [&](int32_t a, int32_t b) { qitems.push_back(a); qitems.push_back(b); };
            T.q_gather[0] = (int64_t)qitems.size();
            for (int32_t i = T.f0; i < T.f1; ++i)
                for (int32_t r = 0; r < sy.fronts[i].Mt; ++r) push(i, r);
            T.q_gather[1] = ((int64_t)qitems.size() - T.q_gather[0]) / 2;
            T.q_fprod[0] = (int64_t)qitems.size();
            for (int32_t i = T.f0; i < T.f1; ++i)
                for (int32_t I = 0; I < sy.fronts[i].Mt; ++I) push(i, I);
            T.q_fprod[1] = ((int64_t)qitems.size() - T.q_fprod[0]) / 2;
            T.q_bprod[0] = (int64_t)qitems.size();
            for (int32_t i = T.f0; i < T.f1; ++i)
                for (int32_t C = 0; C < sy.fronts[i].nsb; ++C) push(i, C);
            T.q_bprod[1] = ((int64_t)qitems.size() - T.q_bprod[0]) / 2;
            for (int32_t i = T.f0; i < T.f1; ++i) {
                T.q_kf = std::max(T.q_kf, sy.fronts[i].nsb);
                T.q_kb = std::max(T.q_kb, sy.fronts[i].Mt);
            }
        }
        T.ea_tile_cols.assign(mc, 0);
        for (int32_t c = 0; c < mc; ++c)
            for (int64_t e = sy.ea_ptr[(int64_t)t * mc + c]; e < sy.ea_ptr[(int64_t)t * mc + c + 1]; ++e)
                T.ea_tile_cols[c] = std::max<int32_t>(T.ea_tile_cols[c], (sy.fronts[sy.ea[e]].mu + NB - 1) / NB);
    }
    if (L.qrow_ptr.size() != (size_t)sy.step_ptr[sy.tree_levels] + 1)
        fail(HSIM_E_INVALID, "inverse-panel items: %zu steps for %d", L.qrow_ptr.size() - 1,
             sy.step_ptr[sy.tree_levels]);
    L.q_doubles = qoff;
    L.it_qrow.upload(qrow_it.empty() ? std::vector<int32_t>{0, 0} : qrow_it);
    L.it_qupd.upload(qupd_it.empty() ? std::vector<int32_t>{0, 0, 0} : qupd_it);
    L.q_items.upload(qitems.empty() ? std::vector<int32_t>{0, 0} : qitems);
    if (L.q_doubles > 0) {
        L.qinvT.alloc((size_t)L.q_doubles * sizeof(double));
        L.qinv.alloc((size_t)L.q_doubles * sizeof(double));
        L.qrhs.alloc((size_t)L.qrhs_rows * H->ld * sizeof(double));
    }
}

static void build_device_level(hsim_hierarchy* H, Level& L, const std::vector<int32_t>* coarse_iperm) {
    const int64_t n = L.n;
    std::vector<int32_t> perm, iperm;
    if (L.coarsest) {
        perm.resize(n);
        std::iota(perm.begin(), perm.end(), 0);
        iperm = perm;
    } else {
        perm = L.sy.perm;
        iperm = L.sy.iperm;
    }
    // permuted CSR (rows and columns in internal order)
    std::vector<int64_t> ptr(n + 1, 0);
    std::vector<int32_t> idx(L.S.nnz());
    std::vector<double> sv(L.S.nnz()), mv(L.S.nnz());
    std::vector<int64_t> newpos(L.S.nnz());   // CSR entry (level order) -> entry of the permuted CSR
    for (int64_t k = 0; k < n; ++k) ptr[k + 1] = ptr[k] + (L.S.ptr[perm[k] + 1] - L.S.ptr[perm[k]]);
    // rows are independent once their offsets are known
#pragma omp parallel
    {
        std::vector<std::pair<int32_t, int64_t>> rowbuf;
#pragma omp for schedule(static)
        for (int64_t k = 0; k < n; ++k) {
            const int32_t v = perm[k];
            rowbuf.clear();
            for (int64_t e = L.S.ptr[v]; e < L.S.ptr[v + 1]; ++e) rowbuf.push_back({iperm[L.S.idx[e]], e});
            std::sort(rowbuf.begin(), rowbuf.end());
            for (size_t t = 0; t < rowbuf.size(); ++t) {
                idx[ptr[k] + t] = rowbuf[t].first;
                sv[ptr[k] + t] = L.S.val[rowbuf[t].second];
                mv[ptr[k] + t] = L.Mval[rowbuf[t].second];
                newpos[rowbuf[t].second] = ptr[k] + (int64_t)t;
            }
        }
    }
    L.dS_ptr.upload(ptr);
    L.dS_idx.upload(idx);
    L.dS_val.upload(sv);
    L.dM_val.upload(mv);
    L.dperm.upload(perm);
    if (L.tau == 0) {
        std::vector<int32_t> mm(n);
        for (int64_t k = 0; k < n; ++k) mm[k] = L.verts[perm[k]];
        L.dmeshmap.upload(mm);
    }
    if (!L.mdiag.empty()) {
        std::vector<double> md(n);
        for (int64_t k = 0; k < n; ++k) md[k] = L.mdiag[perm[k]];
        L.dmdiag.upload(md);
    }
    if (L.coarsest) return;
    // U: rows in this level's internal order, columns in the coarser level's internal order
    {
        std::vector<int64_t> up(n + 1, 0);
        std::vector<int32_t> ui(L.U.nnz());
        std::vector<double> uv(L.U.nnz());
        for (int64_t k = 0; k < n; ++k) up[k + 1] = up[k] + (L.U.ptr[perm[k] + 1] - L.U.ptr[perm[k]]);
#pragma omp parallel
        {
            std::vector<std::pair<int32_t, double>> rb;
#pragma omp for schedule(static)
            for (int64_t k = 0; k < n; ++k) {
                const int32_t v = perm[k];
                rb.clear();
                for (int64_t e = L.U.ptr[v]; e < L.U.ptr[v + 1]; ++e)
                    rb.push_back({(*coarse_iperm)[L.U.idx[e]], L.U.val[e]});
                std::sort(rb.begin(), rb.end());
                for (size_t t = 0; t < rb.size(); ++t) {
                    ui[up[k] + t] = rb[t].first;
                    uv[up[k] + t] = rb[t].second;
                }
            }
        }
        L.dU_ptr.upload(up);
        L.dU_idx.upload(ui);
        L.dU_val.upload(uv);
    }
    // factor structures
    const Symbolic& sy = L.sy;
    std::vector<DFront> df(sy.fronts.size());
    for (size_t i = 0; i < sy.fronts.size(); ++i) {
        const Front& f = sy.fronts[i];
        DFront& d = df[i];
        d.start = f.start;
        d.tile_base = f.tile_base;
        d.linv_base = f.linv_base;
        d.d_base = f.d_base;
        d.ubuf_row = f.ubuf_row;
        d.gather_base = f.gather_base;
        d.rows_off = sy.rows_ptr[i];
        d.ns = f.ns;
        d.mu = f.mu;
        d.ns_pad = f.ns_pad;
        d.mu_pad = f.mu_pad;
        d.Mt = f.Mt;
        d.nsb = f.nsb;
        d.parent = f.parent;
        const int64_t gb = f.gather_base, m = (int64_t)f.ns + f.mu;
        d.flags = sy.gather_ptr[gb + m] > sy.gather_ptr[gb] ? DFRONT_GATHER : 0;
    }
    setup_tree_levels(H, L, df);
    L.dfronts.upload(df);
    L.tiles.alloc((size_t)sy.tile_doubles * sizeof(double));
    L.linv.alloc((size_t)sy.linv_doubles * sizeof(double));
    L.D.alloc((size_t)std::max<int64_t>(1, sy.d_doubles) * sizeof(double));
    L.counters.alloc(4 * sizeof(int32_t));
    L.asm_dst.upload(sy.asm_dst);
    {
        // the assembly map indexes the level-order CSR; the device holds the permuted one
        std::vector<int64_t> src(sy.asm_src.size());
        for (size_t e = 0; e < src.size(); ++e) src[e] = sy.asm_src[e] < 0 ? -1 : newpos[sy.asm_src[e]];
        L.asm_src.upload(src);
    }
    L.it_diag.upload(sy.diag);
    L.it_panel.upload(sy.panel.empty() ? std::vector<int32_t>{0, 0} : sy.panel);
    L.it_upd.upload(sy.upd.empty() ? std::vector<int32_t>{0, 0, 0} : sy.upd);
    L.it_ea.upload(sy.ea.empty() ? std::vector<int32_t>{0} : sy.ea);
    L.rel.upload(sy.rel.empty() ? std::vector<int32_t>{0} : sy.rel);
    L.rows.upload(sy.rows.empty() ? std::vector<int32_t>{0} : sy.rows);
    // padded gather table: for every (front, local row) its update-buffer source rows, -1 padded
    int64_t gwid = 0;
    for (size_t r = 0; r + 1 < sy.gather_ptr.size(); ++r)
        gwid = std::max<int64_t>(gwid, sy.gather_ptr[r + 1] - sy.gather_ptr[r]);
    L.gw = (int32_t)gwid;
    {
        std::vector<int32_t> gat(std::max<size_t>(1, sy.gather_ptr.size() * (size_t)L.gw), -1);
        for (size_t r = 0; r + 1 < sy.gather_ptr.size(); ++r)
            for (int64_t g = sy.gather_ptr[r]; g < sy.gather_ptr[r + 1]; ++g) {
                if (sy.gather_idx[g] > INT32_MAX) fail(HSIM_E_UNIMPLEMENTED, "update buffer beyond 2^31 rows");
                gat[r * L.gw + (g - sy.gather_ptr[r])] = (int32_t)sy.gather_idx[g];
            }
        L.gat.upload(gat);
    }
    L.ubuf.alloc((size_t)std::max<int64_t>(1, sy.ubuf_rows) * H->ld * sizeof(double));
    plan_solve(L, env_int("HSIM_BIG_NS", BIG_NS), env_int("HSIM_BIG_NS_BWD", BIG_NS_BWD));
}

// ----------------------------------------------------------- factor / solve
// the factorisation's launches (nothing waited for); factor_finish reads the
// pivot counts and writes the transposed and FP32 copies
static void factor_launch(hsim_hierarchy* H, Level& L, double mu, hipStream_t s) {
    const Symbolic& sy = L.sy;
    const int32_t mc = std::max<int32_t>(1, sy.max_children);
    int32_t* cnt = dptr<int32_t>(L.counters);
    HIPCHECK(launch_fill_i32(cnt, 4, 0, s));
    const DFront* fr = dptr<DFront>(L.dfronts);
    double* tiles = dptr<double>(L.tiles);
    Prof& P = H->prof;
    const double lvflops = sy.flops / std::max(1, sy.tree_levels);
    double* qT = L.q_doubles > 0 ? dptr<double>(L.qinvT) : nullptr;
    if (qT) HIPCHECK(launch_fill(qT, L.q_doubles, 0.0, s));   // the update items accumulate
    for (int32_t t = 0; t < sy.tree_levels; ++t) {
      P.run(HSIM_K_FACTOR, 8.0 * L.tl[t].l_entries, lvflops, s, [&] {
        const TLev& T = L.tl[t];
        // zero this tree level's fronts, assemble A = S - mu M, add the children's updates
        const int64_t tb0 = sy.fronts[T.f0].tile_base;
        const Front& fl = sy.fronts[T.f1 - 1];
        const int64_t tb1 = fl.tile_base + (int64_t)fl.Mt * (fl.Mt + 1) / 2 * NB * NB;
        HIPCHECK(launch_fill(tiles + tb0, tb1 - tb0, 0.0, s));
        HIPCHECK(launch_assemble(tiles, dptr<int64_t>(L.asm_dst) + sy.asm_tlev_ptr[t],
                                 dptr<int64_t>(L.asm_src) + sy.asm_tlev_ptr[t],
                                 sy.asm_tlev_ptr[t + 1] - sy.asm_tlev_ptr[t], dptr<double>(L.dS_val),
                                 dptr<double>(L.dM_val), 1.0, -mu, s));
        for (int32_t c = 0; c < mc; ++c) {
            const int64_t a = sy.ea_ptr[(int64_t)t * mc + c], b = sy.ea_ptr[(int64_t)t * mc + c + 1];
            HIPCHECK(launch_extend_add(tiles, fr, dptr<int32_t>(L.it_ea) + a, b - a, dptr<int32_t>(L.rel),
                                       T.ea_tile_cols[c], s));
        }
        for (int32_t st = T.step0; st < T.step1; ++st) {
            const int32_t k = st - T.step0;
            HIPCHECK(launch_fac_diag(tiles, dptr<double>(L.linv), dptr<double>(L.D), fr,
                                     dptr<int32_t>(L.it_diag) + sy.diag_ptr[st], sy.diag_ptr[st + 1] - sy.diag_ptr[st],
                                     k, cnt, s));
            HIPCHECK(launch_fac_panel(tiles, dptr<double>(L.linv), dptr<double>(L.D), fr,
                                      dptr<int32_t>(L.it_panel) + 2 * sy.panel_ptr[st],
                                      sy.panel_ptr[st + 1] - sy.panel_ptr[st], k, s, qT,
                                      dptr<int32_t>(L.it_qrow) + 2 * L.qrow_ptr[st],
                                      L.qrow_ptr[st + 1] - L.qrow_ptr[st]));
            HIPCHECK(launch_fac_update(tiles, dptr<double>(L.D), fr, dptr<int32_t>(L.it_upd) + 3 * sy.upd_ptr[st],
                                       sy.upd_ptr[st + 1] - sy.upd_ptr[st], k, s, qT,
                                       dptr<int32_t>(L.it_qupd) + 3 * L.qupd_ptr[st],
                                       L.qupd_ptr[st + 1] - L.qupd_ptr[st]));
        }
      });
    }
}

static void factor_finish(hsim_hierarchy* H, Level& L, double mu, hipStream_t s, bool mixed) {
    const Symbolic& sy = L.sy;
    int32_t* cnt = dptr<int32_t>(L.counters);
    double* tiles = dptr<double>(L.tiles);
    double* qT = L.q_doubles > 0 ? dptr<double>(L.qinvT) : nullptr;
    Prof& P = H->prof;
    // the transposed copies are queued before the pivot counts are read back,
    // so the device works through the host's round trip (wasted only when the
    // factorisation fails)
    L.tilesT.alloc((size_t)sy.tile_doubles * sizeof(double));
    L.linvT.alloc((size_t)std::max<int64_t>(1, sy.linv_doubles) * sizeof(double));
    P.run(HSIM_K_FACTOR, 16.0 * (sy.tile_doubles + sy.linv_doubles), 0.0, s, [&] {
        HIPCHECK(launch_tile_transpose<double>(tiles, dptr<double>(L.tilesT), sy.tile_doubles / (NB * NB), s));
        HIPCHECK(launch_tile_transpose<double>(dptr<double>(L.linv), dptr<double>(L.linvT), sy.linv_doubles / (NB * NB),
                                               s));
        if (qT) HIPCHECK(launch_tile_transpose<double>(qT, dptr<double>(L.qinv), L.q_doubles / (NB * NB), s));
    });
    int32_t hc[2] = {0, 0};
    HIPCHECK(hipMemcpyAsync(hc, cnt, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    L.mu = mu;
    L.neg_pivots = hc[0];
    L.factored = hc[1] == 0;
    L.factored32 = false;
    if (hc[1] != 0) fail(HSIM_E_FACTOR, "LDL^T of S - mu M (level %d, mu=%g): %d zero or non-finite pivots", L.tau, mu, hc[1]);
    if (mixed) {
        // FP32 copy of the FP64 factor for the low-precision solves
        L.tiles32.alloc((size_t)sy.tile_doubles * sizeof(float));
        L.linv32.alloc((size_t)sy.linv_doubles * sizeof(float));
        L.D32.alloc((size_t)std::max<int64_t>(1, sy.d_doubles) * sizeof(float));
        H->prof.run(HSIM_K_OTHER, 12.0 * (sy.tile_doubles + sy.linv_doubles), 0.0, s, [&] {
            HIPCHECK(launch_to_float(dptr<double>(L.tiles), dptr<float>(L.tiles32), sy.tile_doubles, s));
            HIPCHECK(launch_to_float(dptr<double>(L.linv), dptr<float>(L.linv32), sy.linv_doubles, s));
            HIPCHECK(launch_to_float(dptr<double>(L.D), dptr<float>(L.D32), sy.d_doubles, s));
            L.tiles32T.alloc((size_t)sy.tile_doubles * sizeof(float));
            L.linv32T.alloc((size_t)std::max<int64_t>(1, sy.linv_doubles) * sizeof(float));
            HIPCHECK(launch_tile_transpose<float>(dptr<float>(L.tiles32), dptr<float>(L.tiles32T),
                                                  sy.tile_doubles / (NB * NB), s));
            HIPCHECK(launch_tile_transpose<float>(dptr<float>(L.linv32), dptr<float>(L.linv32T),
                                                  sy.linv_doubles / (NB * NB), s));
            if (L.q_doubles > 0) {
                L.qinv32.alloc((size_t)L.q_doubles * sizeof(float));
                L.qinv32T.alloc((size_t)L.q_doubles * sizeof(float));
                HIPCHECK(launch_to_float(dptr<double>(L.qinv), dptr<float>(L.qinv32), L.q_doubles, s));
                HIPCHECK(launch_to_float(dptr<double>(L.qinvT), dptr<float>(L.qinv32T), L.q_doubles, s));
            }
        });
        L.factored32 = true;
    }
}

static void factor_level(hsim_hierarchy* H, Level& L, double mu, hipStream_t s, bool mixed = false) {
    factor_launch(H, L, mu, s);
    factor_finish(H, L, mu, s, mixed);
}

// X (internal order, leading dim ld) <- (S - mu M)^-1 (mdiag ? m*X : X) on columns [col0, col0 + ncols);
// fp32: with the FP32 copy of the factor (FP32 arithmetic, FP64 in and out)
template <class TF>
static void solve_sweeps(hsim_hierarchy* H, Level& L, const TF* tiles, const TF* linv, const TF* D, const TF* tilesT,
                         const TF* linvT, const TF* qinv, const TF* qinvT, double* X, int32_t col0, int32_t ncols,
                         const double* md, hipStream_t s, const double* Xin = nullptr) {
    const Symbolic& sy = L.sy;
    const DFront* fr = dptr<DFront>(L.dfronts);
    Prof& P = H->prof;
    const double bL = sizeof(TF);
    const int32_t* qi = dptr<int32_t>(L.q_items);
    P.solves += 1;
    P.solve_cols += ncols;
    if (sizeof(TF) == sizeof(float)) P.solves32 += 1;
    // the forward products gather the children's updates of the struct rows
    // themselves (each update row written once)
    constexpr bool fuse = true;
    auto qsolve = [&](int phase, const int64_t* rec, int32_t kmax) {
        HIPCHECK(launch_qsolve<TF>(phase, qinv, qinvT, D, fr, qi + rec[0], rec[1], dptr<double>(L.qrhs), H->ld, X,
                                   H->ld, col0, ncols, dptr<double>(L.ubuf), H->ld, dptr<int32_t>(L.gat), L.gw, md,
                                   dptr<int32_t>(L.rows), s, Xin, kmax, fuse));
    };
    for (int32_t t = 0; t < sy.tree_levels; ++t) {
        const TLev& T = L.tl[t];
        const double bytes = bL * T.l_entries + 2.0 * 8.0 * T.pivots * ncols;
        const double flops = 2.0 * (2.0 * T.l_entries - T.pivots) * ncols;
        if (T.big_fwd) {
            P.run(HSIM_K_SOLVE_FWD, bytes, flops, s, [&] {
                qsolve(0, T.q_gather, 0);
                qsolve(1, T.q_fprod, T.q_kf);
            });
            continue;
        }
        P.run(HSIM_K_SOLVE_FWD, bytes, flops, s, [&] {
            HIPCHECK(launch_wsolve<TF>(true, tiles, linv, D, fr, T.f0, T.f1, T.ns_pad_max, X, H->ld, col0, ncols,
                                       dptr<double>(L.ubuf), H->ld, dptr<int32_t>(L.gat), L.gw, md,
                                       nullptr, false, s, Xin));
        });
    }
    for (int32_t t = sy.tree_levels - 1; t >= 0; --t) {
        const TLev& T = L.tl[t];
        const double bytes = bL * T.l_entries + 2.0 * 8.0 * T.pivots * ncols;
        const double flops = 2.0 * (2.0 * T.l_entries - T.pivots) * ncols;
        if (T.big_bwd) {
            P.run(HSIM_K_SOLVE_BWD, bytes, flops, s, [&] {
                qsolve(2, T.q_gather, 0);
                qsolve(3, T.q_bprod, T.q_kb);
            });
            continue;
        }
        P.run(HSIM_K_SOLVE_BWD, bytes, flops, s, [&] {
            HIPCHECK(launch_wsolve<TF>(false, tilesT, linvT, D, fr, T.f0, T.f1, T.ns_pad_max, X, H->ld, col0, ncols,
                                       nullptr, H->ld, nullptr, 0, nullptr, dptr<int32_t>(L.rows), true, s));
        });
    }
}

// X = (S - mu M)^-1 (M) B on columns [col0, col0 + ncols), in place (B = X)
// or, with Xin, reading the right-hand side from Xin and writing X
static void solve_level(hsim_hierarchy* H, Level& L, double* X, int32_t col0, int32_t ncols, bool scale_by_m,
                        hipStream_t s, bool fp32 = false, const double* Xin = nullptr) {
    const double* md = scale_by_m ? dptr<double>(L.dmdiag) : nullptr;
    if (fp32) {
        if (!L.factored32) fail(HSIM_E_STATE, "no FP32 factor on level %d", L.tau);
        solve_sweeps<float>(H, L, dptr<float>(L.tiles32), dptr<float>(L.linv32), dptr<float>(L.D32),
                            dptr<float>(L.tiles32T), dptr<float>(L.linv32T), dptr<float>(L.qinv32),
                            dptr<float>(L.qinv32T), X, col0, ncols, md, s, Xin);
    } else {
        solve_sweeps<double>(H, L, dptr<double>(L.tiles), dptr<double>(L.linv), dptr<double>(L.D),
                             dptr<double>(L.tilesT), dptr<double>(L.linvT), dptr<double>(L.qinv),
                             dptr<double>(L.qinvT), X, col0, ncols, md, s, Xin);
    }
}

// Y = (a A + b M) X on the level's S / M pattern, A = S (a_is_s) or M; the
// M term only with with_m
static void pattern_spmm(Level& L, bool a_is_s, bool with_m, double a, double b, const double* X, int64_t ldx,
                         int32_t k, double* Y, int64_t ldy, hipStream_t s) {
    HIPCHECK(launch_spmm(dptr<int64_t>(L.dS_ptr), dptr<int32_t>(L.dS_idx), dptr<double>(a_is_s ? L.dS_val : L.dM_val),
                         with_m ? dptr<double>(L.dM_val) : nullptr, a, b, L.n, X, ldx, k, Y, ldy, s));
}

static void apply_level(hsim_hierarchy* H, Level& L, int op, const double* X, double* Y, int32_t k, hipStream_t s) {
    // op 0: S, 1: M, 2: S - mu M
    if (op == 1 && L.tau == 0) {
        HIPCHECK(launch_diag_scale(dptr<double>(L.dmdiag), L.n, X, H->ld, k, Y, H->ld, s));
        return;
    }
    const double nnz = (double)L.S.nnz();
    H->prof.run(HSIM_K_SPMM, nnz * (op == 2 ? 20.0 : 12.0) + 16.0 * L.n * k, 2.0 * nnz * k, s, [&] {
        pattern_spmm(L, op != 1, op == 2, 1.0, op == 2 ? -L.mu : 0.0, X, H->ld, k, Y, H->ld, s);
    });
}

// X = (S - mu M)^-1 B on columns [col0, col0 + ncols) with FP32 solves and
// FP64 iterative refinement until every column's relative residual
// ||B - A X|| / ||B|| is at most eta; falls back to the FP64 solve when the
// refinement stalls.  B is not modified.  Returns the refinement sweeps.
// est32: backward error of a plain FP32 solve measured on this factor (< 0:
// not measured yet).  A solve that FP32 cannot meet without refinement is done
// in FP64 at once; one that it meets by a wide margin skips the residual check.
// The solve accuracy only steers convergence: every accepted eigenpair is
// certified by the FP64 residual of an FP64 Rayleigh-Ritz step.
static int32_t refine_solve(hsim_hierarchy* H, Level& L, const double* B, double* X, int32_t col0, int32_t ncols,
                            double eta, hipStream_t s, int32_t* escalated, double* est32) {
    const int64_t n = L.n;
    const int32_t ld = H->ld;
    double* R = dptr<double>(H->R);
    HIPCHECK(launch_copy2d(B + col0, ld, n, ncols, X + col0, ld, s));
    if (*est32 >= 0 && *est32 > eta) {
        solve_level(H, L, X, col0, ncols, false, s, false);
        return 0;
    }
    solve_level(H, L, X, col0, ncols, false, s, true);
    if (*est32 >= 0 && *est32 <= 0.1 * eta) return 0;
    std::vector<double> ratio(ncols);
    double prev = INFINITY;
    int32_t sweeps = 0, stall = 0;
    const double nnz = (double)L.S.nnz();
    for (int it = 0; it < 12; ++it) {
        // R = B - (S - mu M) X
        H->prof.run(HSIM_K_SPMM, nnz * 20.0 + 16.0 * n * ncols, 2.0 * nnz * ncols, s, [&] {
            pattern_spmm(L, true, true, 1.0, -L.mu, X + col0, ld, ncols, R + col0, ld, s);
        });
        HIPCHECK(launch_axpby(1.0, B + col0, ld, -1.0, R + col0, ld, n, ncols, s));
        HIPCHECK(launch_colnorm_ratio(R, B, n, ld, col0, ncols, dptr<double>(H->cn_part), dptr<double>(H->cn_ratio), s));
        HIPCHECK(hipMemcpyAsync(ratio.data(), H->cn_ratio.p, ncols * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        double worst = 0;
        for (double r : ratio) worst = std::max(worst, std::isfinite(r) ? r : INFINITY);
        if (it == 0) *est32 = std::isfinite(worst) ? worst : 1.0;
        if (worst <= eta) return sweeps;
        if (!(worst < 0.5 * prev)) ++stall;
        if (stall >= 2 || !std::isfinite(worst)) break;
        prev = worst;
        solve_level(H, L, R, col0, ncols, false, s, true);
        HIPCHECK(launch_axpby(1.0, R + col0, ld, 1.0, X + col0, ld, n, ncols, s));
        ++sweeps;
    }
    // stalled: solve this block in FP64
    ++*escalated;
    HIPCHECK(launch_copy2d(B + col0, ld, n, ncols, X + col0, ld, s));
    solve_level(H, L, X, col0, ncols, false, s, false);
    return sweeps;
}

static void prolong_level(hsim_hierarchy* H, Level& L, const double* Xc, double* Xf, int32_t k, hipStream_t s) {
    const double nnz = (double)L.U.nnz();
    const double nc = (double)H->lv[L.tau + 1]->n;
    H->prof.run(HSIM_K_SPMM, nnz * 12.0 + 8.0 * (L.n + nc) * k, 2.0 * nnz * k, s, [&] {
        HIPCHECK(launch_spmm(dptr<int64_t>(L.dU_ptr), dptr<int32_t>(L.dU_idx), dptr<double>(L.dU_val), nullptr, 1.0, 0.0,
                             L.n, Xc, H->ld, k, Xf, H->ld, s));
    });
}

static void swap_buffers(DeviceBuffer& a, DeviceBuffer& b) {
    std::swap(a.p, b.p);
    std::swap(a.bytes, b.bytes);
}

static void alloc_workspace(hsim_hierarchy* H) {
    const int64_t n0 = H->lv[0]->n;
    const size_t blk = (size_t)n0 * H->ld * sizeof(double);
    H->Phi.alloc(blk);
    H->Psi.alloc(blk);
    H->SPsi.alloc(blk);
    H->MPsi.alloc(blk);
    H->Btmp.alloc(blk);
    H->Xc.alloc(blk);
    H->R.alloc(blk);
    H->cn_part.alloc((size_t)colnorm_partial_doubles(n0, H->ld) * sizeof(double));
    H->cn_ratio.alloc((size_t)H->ld * sizeof(double));
    const int64_t chunk = 4096;
    H->gram_chunk = gram_chunk_rows(n0, H->q);   // fixed here: every later Gram call fits the buffer
    H->gram_part.alloc((size_t)gram_partial_doubles(n0, H->q, H->gram_chunk) * sizeof(double));
    H->ritz_part.alloc((size_t)ritz_partial_doubles(n0, H->q, chunk) * sizeof(double));
    H->Sbar.alloc((size_t)H->q * H->q * sizeof(double));
    H->Mbar.alloc((size_t)H->q * H->q * sizeof(double));
    H->Phibar.alloc((size_t)H->q * H->q * sizeof(double));
    H->lam.alloc((size_t)H->q * sizeof(double));
    H->resid.alloc((size_t)H->q * sizeof(double));
    const int64_t nch = (n0 + 8191) / 8192;
    H->exportw.alloc((size_t)(2 * nch * H->p + H->p + 8) * sizeof(double));
    const int64_t nc = H->lv.back()->n;
    H->coarseS.alloc((size_t)nc * nc * sizeof(double));
    H->coarseM.alloc((size_t)nc * nc * sizeof(double));
}

static double lambda_floor(const std::vector<double>& lam) {
    double top = 0;
    for (double l : lam) top = std::max(top, std::fabs(l));
    for (double l : lam)
        if (l > 1e-8 * top) return l;
    return top > 0 ? top : 1.0;
}

static double choose_shift(const std::vector<double>& lam, int32_t p, double alpha) {
    const int32_t j = (int32_t)std::floor(alpha * p + 1e-12);
    double mu = lam[std::min<size_t>(j, lam.size() - 1)];
    if (mu <= 1e-12 * lam.back()) {
        for (double l : lam)
            if (l > 1e-12 * lam.back()) { mu = -1e-3 * l; break; }
    }
    return mu;
}

// one Rayleigh-Ritz step on level L from the basis in Psi (already inverse
// iterated); leaves Phi, lam (device) and returns lam/resid on the host
// false (and Phi untouched) when a low-precision or compensated Gram
// (gram_mode != GRAM_FP64) left the reduced mass matrix without a positive
// definite factor; the caller repeats the step in FP64
static bool rayleigh_ritz(hsim_hierarchy* H, Level& L, std::vector<double>& lam, std::vector<double>& res,
                          hipStream_t s, double* ms_gram, double* ms_rr, double* ms_ritz,
                          int gram_mode = GRAM_FP64) {
    const int32_t q = H->q;
    const bool fin = L.tau == 0;
    auto t0 = std::chrono::steady_clock::now();
    apply_level(H, L, 0, dptr<double>(H->Psi), dptr<double>(H->SPsi), q, s);
    if (!fin) apply_level(H, L, 1, dptr<double>(H->Psi), dptr<double>(H->MPsi), q, s);
    const double nq = (double)L.n * q;
    H->prof.run(HSIM_K_GRAM, 8.0 * nq * (fin ? 2.0 : 3.0) + 8.0 * (fin ? L.n : 0), 2.0 * nq * q, s, [&] {
        HIPCHECK(launch_gram(dptr<double>(H->Psi), dptr<double>(H->SPsi), fin ? nullptr : dptr<double>(H->MPsi),
                             fin ? dptr<double>(L.dmdiag) : nullptr, L.n, q, H->ld, dptr<double>(H->gram_part), H->gram_chunk,
                             dptr<double>(H->Sbar), dptr<double>(H->Mbar), s, gram_mode));
    });
    H->gram_steps[gram_mode] += 1;
    HIPCHECK(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    H->rr.setup(q, s);
    int32_t sweeps = 0;
    H->prof.run(HSIM_K_JACOBI, 0.0, 0.0, s, [&] {
        sweeps = H->rr.run(dptr<double>(H->Sbar), dptr<double>(H->Mbar), q, dptr<double>(H->lam),
                           dptr<double>(H->Phibar), q, s);
    });
    if (sweeps < 0) {
        if (gram_mode != GRAM_FP64) return false;
        fail(HSIM_E_FACTOR, "Rayleigh-Ritz step on level %d: the reduced mass matrix is not positive definite "
             "(the iterated basis has lost rank)", L.tau);
    }
    lam.resize(q);
    HIPCHECK(hipMemcpyAsync(lam.data(), H->lam.p, q * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    auto t2 = std::chrono::steady_clock::now();
    const double lf = lambda_floor(lam);
    // S Phi only for the p tested columns (whole 16-column tiles)
    const double qres = std::min<double>(q, (double)((H->p + 15) / 16 * 16));
    H->prof.run(HSIM_K_RITZ, 8.0 * nq * (fin ? 3.0 : 4.0) + 8.0 * (fin ? L.n : 0),
                2.0 * nq * (q * (fin ? 1.0 : 2.0) + qres), s,
                [&] {
                    HIPCHECK(launch_ritz(dptr<double>(H->Psi), dptr<double>(H->SPsi),
                                         fin ? nullptr : dptr<double>(H->MPsi), fin ? dptr<double>(L.dmdiag) : nullptr,
                                         dptr<double>(H->Phibar), dptr<double>(H->lam), L.n, q, H->ld,
                                         dptr<double>(H->Phi), nullptr, dptr<double>(H->ritz_part), 4096, fin, lf,
                                         dptr<double>(H->resid), s, H->p));
                });
    res.resize(q);
    HIPCHECK(hipMemcpyAsync(res.data(), H->resid.p, q * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    auto t3 = std::chrono::steady_clock::now();
    *ms_gram += std::chrono::duration<double, std::milli>(t1 - t0).count();
    *ms_rr += std::chrono::duration<double, std::milli>(t2 - t1).count();
    *ms_ritz += std::chrono::duration<double, std::milli>(t3 - t2).count();
    return true;
}

static Level& level_at(hsim_hierarchy* H, int32_t level) {
    if (!H) fail(HSIM_E_INVALID, "null hierarchy");
    if (H->host_only) fail(HSIM_E_STATE, "hierarchy was built host-only");
    H->prof.reset(false);
    H->solved = false;   // step calls reuse the solve workspace and factors
    if (level < 0 || level >= H->T) fail(HSIM_E_INVALID, "level %d out of range [0, %d)", level, H->T);
    return *H->lv[level];
}

}  // namespace hsim

using namespace hsim;

#define API_BEGIN try {
#define API_END                                       \
    }                                                 \
    catch (const hsim::Error& e) {                    \
        hsim::set_last_error(e.msg);                  \
        return e.code;                                \
    }                                                 \
    catch (const std::bad_alloc&) {                   \
        hsim::set_last_error("host allocation failed"); \
        return HSIM_E_NOMEM;                          \
    }                                                 \
    catch (const std::exception& e) {                 \
        hsim::set_last_error(e.what());               \
        return HSIM_E_INVALID;                        \
    }                                                 \
    return HSIM_OK;

extern "C" {

void hsim_default_build_opts(hsim_build_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->p = 0;
    o->levels = 0;
    o->n_coarsest = 0;
    o->growth_mode = 0;
    o->lumping = 0;
    o->support_sigma = 7.0;
    o->seed = 0;
}

void hsim_default_solve_opts(hsim_solve_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->tol = 1e-2;
    o->shift_alpha = 0.1;
    o->precision = HSIM_FP64;
    o->max_iters = 100;
    o->flags = 0;
    o->stream = nullptr;
}

const char* hsim_last_error(void) { return g_last_error.c_str(); }

void hsim_free(hsim_hierarchy* h) { delete h; }

// Finest-level S (values on the pattern of the edge graph plus the diagonal)
// and barycentric lumped M assembled on the current device.
// work arrays of the device assembly, kept by the caller until the sampling
// that runs beside it has finished (freeing device memory waits for the device)
struct AssemblyBuffers {
    DeviceBuffer dV, dF, bptr, bidx, bcorner, bdptr, bdcorner, dvptr, dvtri, ddens, dw, da3, dval, dm;
    void release() {
        for (DeviceBuffer* b : {&dV, &dF, &bptr, &bidx, &bcorner, &bdptr, &bdcorner, &dvptr, &dvtri, &ddens, &dw,
                                &da3, &dval, &dm})
            b->release();
    }
};

static void device_assembly(const Mesh& m, const Graph& g, const double* density, Csr& S, std::vector<double>& md,
                            AssemblyBuffers& B) {
    AssemblyMaps a = assembly_maps(m, g);
    const int64_t n = m.nv, nf = m.nf, nnz = a.S.nnz();
    DeviceBuffer &dV = B.dV, &dF = B.dF, &bptr = B.bptr, &bidx = B.bidx, &bcorner = B.bcorner, &bdptr = B.bdptr,
                 &bdcorner = B.bdcorner, &dvptr = B.dvptr, &dvtri = B.dvtri, &ddens = B.ddens, &dw = B.dw,
                 &da3 = B.da3, &dval = B.dval, &dm = B.dm;
    dV.upload(m.V);
    dF.upload(m.F);
    bptr.upload(a.S.ptr);
    bidx.upload(a.S.idx);
    bcorner.upload(a.corner);
    bdptr.upload(a.dptr);
    bdcorner.upload(a.dcorner);
    dvptr.upload(a.vptr);
    dvtri.upload(a.vtri);
    if (density) {
        ddens.alloc((size_t)n * sizeof(double));
        ddens.copy_in(density, (size_t)n * sizeof(double));
    }
    dw.alloc((size_t)3 * nf * sizeof(double));
    da3.alloc((size_t)nf * sizeof(double));
    dval.alloc((size_t)nnz * sizeof(double));
    dm.alloc((size_t)n * sizeof(double));
    HIPCHECK(launch_assemble_mesh(dptr<double>(dV), dptr<int32_t>(dF), nf, n, dptr<int64_t>(bptr),
                                  dptr<int32_t>(bidx), dptr<int64_t>(bcorner), dptr<int64_t>(bdptr),
                                  dptr<int64_t>(bdcorner), dptr<int64_t>(dvptr), dptr<int32_t>(dvtri),
                                  density ? dptr<double>(ddens) : nullptr, dptr<double>(dw), dptr<double>(da3),
                                  dptr<double>(dval), dptr<double>(dm), nullptr));
    S = std::move(a.S);
    S.val.resize(nnz);
    md.resize(n);
    HIPCHECK(hipMemcpy(S.val.data(), dval.p, (size_t)nnz * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(md.data(), dm.p, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
}

hsim_status hsim_build_hierarchy(const double* V, int64_t nv, const int32_t* F, int64_t nf, const double* density,
                                 const hsim_build_opts* opts, hsim_hierarchy** out) {
    API_BEGIN
    if (!V || !F || !out) fail(HSIM_E_INVALID, "null argument");
    *out = nullptr;
    hsim_build_opts bo;
    if (opts) bo = *opts;
    else hsim_default_build_opts(&bo);
    auto t0 = std::chrono::steady_clock::now();
    // HSIM_VERBOSE=1: the time of every build phase on stderr
    const bool verbose = env_int("HSIM_VERBOSE", 0) != 0;
    auto tlast = t0;
    auto phase = [&](const char* name) {
        const auto now = std::chrono::steady_clock::now();
        if (verbose)
            std::fprintf(stderr, "[hsim build] %-28s %8.1f ms\n", name,
                         std::chrono::duration<double, std::milli>(now - tlast).count());
        tlast = now;
    };
    std::unique_ptr<hsim_hierarchy> H(new hsim_hierarchy());
    H->host_only = (bo.flags & HSIM_BUILD_HOST_ONLY) != 0;
    if (!H->host_only) HIPCHECK(hipGetDevice(&H->device));
    H->bo = bo;
    Mesh& m = H->mesh;
    m.nv = nv;
    m.nf = nf;
    if (nv <= 0 || nf <= 0) fail(HSIM_E_MESH, "empty mesh");
    m.V.assign(V, V + 3 * nv);
    m.F.assign(F, F + 3 * nf);
    if (density) {
        H->density.assign(density, density + nv);
        for (int64_t i = 0; i < nv; ++i)
            if (!(H->density[i] > 0) || !std::isfinite(H->density[i])) fail(HSIM_E_INVALID, "density must be positive");
    }
    // mesh checks, edge graph and farthest point sampling on the device (the
    // host build's results bit for bit), or on the host for host-only builds
    const bool dev_build = !H->host_only && env_int("HSIM_HOST_HIERARCHY", 0) == 0;
    DevMesh dm;
    Graph g;
    if (dev_build) {
        device_mesh_graph(m, dm, g);
    } else {
        validate_mesh(m);
        g = edge_graph(m);
    }
    phase(dev_build ? "mesh checks + graph (device)" : "mesh checks + graph (host)");
    if (bo.boundary != 0 && bo.boundary != 1) fail(HSIM_E_INVALID, "boundary must be 0 (natural) or 1 (Dirichlet)");
    // level-0 unknowns: every vertex, or (Dirichlet) the vertices off the boundary
    std::vector<int32_t> dofs;
    {
        const std::vector<char> onb = bo.boundary == 1 ? boundary_vertex_flags(m) : std::vector<char>(nv, 0);
        for (int64_t i = 0; i < nv; ++i)
            if (!onb[i]) dofs.push_back((int32_t)i);
    }
    const int64_t n0 = (int64_t)dofs.size();
    const bool restricted = n0 < nv;
    const int32_t p = bo.p;
    if (p < 1) fail(HSIM_E_INVALID, "p must be >= 1");
    const int32_t q = std::max<int32_t>((int32_t)std::ceil(1.5 * p), p + 8);
    if (q >= n0) fail(HSIM_E_INVALID, "subspace size q=%d must be below the unknown count %lld", q, (long long)n0);
    int T = bo.levels ? bo.levels : (p <= 200 ? 2 : 3);
    if (T < 2 || T > HSIM_MAX_LEVELS) fail(HSIM_E_INVALID, "levels must be in [2, %d]", HSIM_MAX_LEVELS);
    int64_t nc = bo.n_coarsest ? bo.n_coarsest : std::max<int64_t>((int64_t)std::ceil(1.5 * p), 1000);
    nc = std::min<int64_t>(nc, n0);
    if (nc < q) fail(HSIM_E_INVALID, "coarsest level (%lld) smaller than the subspace size %d", (long long)nc, q);
    if (!(bo.support_sigma > 0)) fail(HSIM_E_INVALID, "support_sigma must be positive");
    if (bo.lumping != 0 && bo.lumping != 1) fail(HSIM_E_INVALID, "lumping must be 0 or 1");
    H->p = p;
    H->q = q;
    H->T = T;
    H->ld = (int32_t)round_up(q, 8);
    H->area = surface_area(m);
    std::vector<int64_t> sizes = level_sizes(n0, T, nc, bo.growth_mode);
    for (int t = 1; t < T; ++t)
        if (sizes[t] >= sizes[t - 1]) fail(HSIM_E_INVALID, "level %d is not smaller than level %d (too many levels for this mesh)", t, t - 1);
    // the sampling runs on the device (a stream of its own) while the host and
    // the rest of the device assemble the finest level and analyse it
    std::unique_ptr<FpsRun> fps;
    if (dev_build) fps = device_fps_start(dm, sizes[1], bo.seed);
    AssemblyBuffers asm_buf;
    // levels (the vertices of the coarser ones follow from the sampling)
    for (int t = 0; t < T; ++t) {
        auto L = std::make_unique<Level>();
        L->tau = t;
        L->n = sizes[t];
        L->coarsest = t == T - 1;
        if (t == 0) L->verts = dofs;
        H->lv.push_back(std::move(L));
    }
    {
        Level& L0 = *H->lv[0];
        if (!H->host_only && bo.lumping == 0 && env_int("HSIM_HOST_ASSEMBLY", 0) == 0) {
            // cotangent stiffness and lumped mass assembled on the device (same values as the host
            // assembly, term for term in the same order), downloaded for the rest of the build
            device_assembly(m, g, density, L0.S, L0.mdiag, asm_buf);
            for (int64_t i = 0; i < nv; ++i)
                if (!(L0.mdiag[i] > 0)) fail(HSIM_E_MESH, "lumped mass of vertex %lld is not positive", (long long)i);
        } else {
            L0.S = cotan_stiffness(m);
            L0.mdiag = lumped_mass(m, bo.lumping, density);
        }
        if (restricted) {
            // Dirichlet: the principal submatrix of S and the lumped masses on the unknowns
            std::vector<int32_t> pos(nv, -1);
            for (int64_t k = 0; k < n0; ++k) pos[dofs[k]] = (int32_t)k;
            Csr R;
            R.rows = R.cols = n0;
            R.ptr.assign(n0 + 1, 0);
            std::vector<double> md(n0);
            for (int64_t k = 0; k < n0; ++k) {
                const int32_t v = dofs[k];
                for (int64_t e = L0.S.ptr[v]; e < L0.S.ptr[v + 1]; ++e)
                    if (pos[L0.S.idx[e]] >= 0) {
                        R.idx.push_back(pos[L0.S.idx[e]]);
                        R.val.push_back(L0.S.val[e]);
                    }
                R.ptr[k + 1] = (int64_t)R.idx.size();
                md[k] = L0.mdiag[v];
            }
            L0.S = std::move(R);
            L0.mdiag = std::move(md);
        }
        L0.Mval.assign(L0.S.nnz(), 0.0);
        for (int64_t i = 0; i < n0; ++i)
            for (int64_t e = L0.S.ptr[i]; e < L0.S.ptr[i + 1]; ++e)
                if (L0.S.idx[e] == i) L0.Mval[e] = L0.mdiag[i];
    }
    phase("assembly");
    // elimination order and symbolic analysis of a level (host, OpenMP)
    auto analyse_level = [&](int t) {
        Level& L = *H->lv[t];
        std::vector<double> X(3 * L.n);
        for (int64_t i = 0; i < L.n; ++i)
            for (int c = 0; c < 3; ++c) X[3 * i + c] = m.V[3 * (int64_t)L.verts[i] + c];
        L.sy = analyse(L.S, X.data(), L.n);
    };
    // the finest level's pattern and coordinates are known now: the host
    // analyses it while the device samples
    analyse_level(0);
    phase("ordering + symbolic (finest)");
    std::vector<int32_t> order =
        dev_build ? device_fps_finish(*fps) : farthest_point_sampling(g, nv, sizes[1], bo.seed);
    fps.reset();
    asm_buf.release();
    for (int t = 1; t < T; ++t) H->lv[t]->verts.assign(order.begin(), order.begin() + sizes[t]);
    phase(dev_build ? "farthest points (device, rest)" : "farthest points (host)");
    for (int t = 0; t + 1 < T; ++t) {
        Level& L = *H->lv[t];
        Level& C = *H->lv[t + 1];
        // U on the device (the host's U bit for bit), else on the host
        if (!(dev_build && device_prolongation(dm, L.verts, t == 0 && !restricted, C.verts, bo.support_sigma, H->area,
                                               L.U, &L.rho)))
            L.U = prolongation(g, nv, L.verts, t == 0 && !restricted, C.verts, bo.support_sigma, H->area, &L.rho);
        if (t == 0 && restricted) {
            // a coarse basis function with no unknown in its support would make the
            // Galerkin operators singular
            std::vector<char> hit(C.n, 0);
            for (int32_t c : L.U.idx) hit[c] = 1;
            for (int64_t c = 0; c < C.n; ++c)
                if (!hit[c])
                    fail(HSIM_E_INVALID, "coarse vertex %d has no interior vertex within its support radius",
                         C.verts[c]);
        }
        // the Galerkin products on the device (the host's sums, same order), else on the host
        if (!(dev_build && device_galerkin(L.U, L.S, L.Mval, C.S, C.Mval))) galerkin(L.U, L.S, L.Mval, C.S, C.Mval);
    }
    phase("prolongation + Galerkin");
    for (int t = 1; t + 1 < T; ++t) analyse_level(t);
    phase("ordering + symbolic (rest)");
    // device
    for (int t = H->host_only ? -1 : T - 1; t >= 0; --t) {
        Level& L = *H->lv[t];
        const std::vector<int32_t>* ci = nullptr;
        std::vector<int32_t> ident;
        if (t + 1 < T) {
            Level& C = *H->lv[t + 1];
            if (C.coarsest) {
                ident.resize(C.n);
                std::iota(ident.begin(), ident.end(), 0);
                ci = &ident;
            } else {
                ci = &C.sy.iperm;
            }
        }
        build_device_level(H.get(), L, ci);
    }
    if (!H->host_only) {
        alloc_workspace(H.get());
        HIPCHECK(hipDeviceSynchronize());
    }
    phase("device levels + workspace");
    H->ms_build = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = H.release();
    API_END
}

hsim_status hsim_hierarchy_shape(const hsim_hierarchy* h, int32_t* levels, int32_t* q, int32_t* p) {
    API_BEGIN
    if (!h) fail(HSIM_E_INVALID, "null hierarchy");
    if (levels) *levels = h->T;
    if (q) *q = h->q;
    if (p) *p = h->p;
    API_END
}

hsim_status hsim_level_info(const hsim_hierarchy* h, int32_t level, hsim_level_desc* info) {
    API_BEGIN
    if (!h || !info) fail(HSIM_E_INVALID, "null argument");
    if (level < 0 || level >= h->T) fail(HSIM_E_INVALID, "level out of range");
    const Level& L = *h->lv[level];
    std::memset(info, 0, sizeof *info);
    info->n = L.n;
    info->nnz = L.S.nnz();
    info->nnz_u = L.coarsest ? 0 : L.U.nnz();
    info->fronts = L.coarsest ? 0 : (int64_t)L.sy.fronts.size();
    info->tree_levels = L.coarsest ? 0 : L.sy.tree_levels;
    info->factor_entries = L.coarsest ? 0 : L.sy.tile_doubles;
    info->rho = L.rho;
    info->factor_flops = L.coarsest ? 0 : L.sy.flops;
    info->factor_nnz = L.coarsest ? 0 : L.sy.factor_nnz;
    for (const TLev& T : L.tl) info->qpanel_tree_levels += T.q ? 1 : 0;
    info->qpanel_entries = L.q_doubles;
    API_END
}

hsim_status hsim_level_export(const hsim_hierarchy* h, int32_t level, int64_t* verts, int64_t* S_indptr,
                              int32_t* S_indices, double* S_data, double* M_data, int64_t* U_indptr,
                              int32_t* U_indices, double* U_data, int32_t* perm) {
    API_BEGIN
    if (!h) fail(HSIM_E_INVALID, "null hierarchy");
    if (level < 0 || level >= h->T) fail(HSIM_E_INVALID, "level out of range");
    const Level& L = *h->lv[level];
    if (verts) for (int64_t i = 0; i < L.n; ++i) verts[i] = L.verts[i];
    if (S_indptr) std::copy(L.S.ptr.begin(), L.S.ptr.end(), S_indptr);
    if (S_indices) std::copy(L.S.idx.begin(), L.S.idx.end(), S_indices);
    if (S_data) std::copy(L.S.val.begin(), L.S.val.end(), S_data);
    if (M_data) std::copy(L.Mval.begin(), L.Mval.end(), M_data);
    if (!L.coarsest) {
        if (U_indptr) std::copy(L.U.ptr.begin(), L.U.ptr.end(), U_indptr);
        if (U_indices) std::copy(L.U.idx.begin(), L.U.idx.end(), U_indices);
        if (U_data) std::copy(L.U.val.begin(), L.U.val.end(), U_data);
        if (perm) std::copy(L.sy.perm.begin(), L.sy.perm.end(), perm);
    } else if (perm) {
        for (int64_t i = 0; i < L.n; ++i) perm[i] = (int32_t)i;
    }
    API_END
}

// ---------------------------------------------------------------- steps
static hipStream_t S_(void* s) { return reinterpret_cast<hipStream_t>(s); }

hsim_status hsim_step_prolong(hsim_hierarchy* h, int32_t level, int32_t k, const double* d_coarse, double* d_fine,
                              void* stream) {
    API_BEGIN
    Level& L = level_at(h, level);
    if (L.coarsest) fail(HSIM_E_INVALID, "the coarsest level has no prolongation");
    if (k < 1 || k > h->ld) fail(HSIM_E_INVALID, "k must be in [1, %d]", h->ld);
    if (!d_coarse || !d_fine) fail(HSIM_E_INVALID, "null argument");
    hipStream_t s = S_(stream);
    Level& C = *h->lv[level + 1];
    HIPCHECK(launch_gather_rows(d_coarse, k, dptr<int32_t>(C.dperm), C.n, k, dptr<double>(h->Xc), h->ld, s));
    prolong_level(h, L, dptr<double>(h->Xc), dptr<double>(h->Psi), k, s);
    HIPCHECK(launch_scatter_rows(dptr<double>(h->Psi), h->ld, dptr<int32_t>(L.dperm), L.n, k, d_fine, k, s));
    API_END
}

hsim_status hsim_step_apply(hsim_hierarchy* h, int32_t level, int32_t op, int32_t k, const double* d_X, double* d_Y,
                            void* stream) {
    API_BEGIN
    Level& L = level_at(h, level);
    if (k < 1 || k > h->ld) fail(HSIM_E_INVALID, "k must be in [1, %d]", h->ld);
    if (op < 0 || op > 2) fail(HSIM_E_INVALID, "op must be 0, 1 or 2");
    if (op == 2 && !L.factored) fail(HSIM_E_STATE, "op 2 needs a factorisation of this level (for its shift)");
    if (!d_X || !d_Y) fail(HSIM_E_INVALID, "null argument");
    hipStream_t s = S_(stream);
    HIPCHECK(launch_gather_rows(d_X, k, dptr<int32_t>(L.dperm), L.n, k, dptr<double>(h->Xc), h->ld, s));
    apply_level(h, L, op, dptr<double>(h->Xc), dptr<double>(h->Psi), k, s);
    HIPCHECK(launch_scatter_rows(dptr<double>(h->Psi), h->ld, dptr<int32_t>(L.dperm), L.n, k, d_Y, k, s));
    API_END
}

hsim_status hsim_step_factor(hsim_hierarchy* h, int32_t level, double mu, int32_t precision, int32_t* neg_pivots,
                             void* stream) {
    API_BEGIN
    Level& L = level_at(h, level);
    if (L.coarsest) fail(HSIM_E_INVALID, "the coarsest level is solved densely");
    if (!std::isfinite(mu)) fail(HSIM_E_INVALID, "mu must be finite");
    if (precision != HSIM_FP64 && precision != HSIM_MIXED) fail(HSIM_E_INVALID, "unknown precision");
    factor_level(h, L, mu, S_(stream), precision == HSIM_MIXED);
    if (neg_pivots) *neg_pivots = L.neg_pivots;
    API_END
}

hsim_status hsim_step_solve(hsim_hierarchy* h, int32_t level, int32_t k, const double* d_B, double* d_X,
                            int32_t precision, double refine_tol, void* stream) {
    API_BEGIN
    Level& L = level_at(h, level);
    if (L.coarsest) fail(HSIM_E_INVALID, "the coarsest level is solved densely");
    if (!L.factored) fail(HSIM_E_STATE, "hsim_step_solve before hsim_step_factor on level %d", level);
    if (k < 1 || k > h->ld) fail(HSIM_E_INVALID, "k must be in [1, %d]", h->ld);
    if (!d_B || !d_X) fail(HSIM_E_INVALID, "null argument");
    if (precision != HSIM_FP64 && precision != HSIM_MIXED) fail(HSIM_E_INVALID, "unknown precision");
    hipStream_t s = S_(stream);
    HIPCHECK(launch_gather_rows(d_B, k, dptr<int32_t>(L.dperm), L.n, k, dptr<double>(h->Xc), h->ld, s));
    if (precision == HSIM_MIXED) {
        if (!L.factored32) fail(HSIM_E_STATE, "mixed solve needs hsim_step_factor with HSIM_MIXED");
        if (!(refine_tol > 0)) fail(HSIM_E_INVALID, "refine_tol must be positive");
        int32_t esc = 0;
        double est32 = -1.0;   // always measure and refine on this entry point
        refine_solve(h, L, dptr<double>(h->Xc), dptr<double>(h->Btmp), 0, k, refine_tol, s, &esc, &est32);
        HIPCHECK(launch_scatter_rows(dptr<double>(h->Btmp), h->ld, dptr<int32_t>(L.dperm), L.n, k, d_X, k, s));
    } else {
        solve_level(h, L, dptr<double>(h->Xc), 0, k, false, s);
        HIPCHECK(launch_scatter_rows(dptr<double>(h->Xc), h->ld, dptr<int32_t>(L.dperm), L.n, k, d_X, k, s));
    }
    API_END
}

hsim_status hsim_step_gram(hsim_hierarchy* h, int32_t level, int32_t k, const double* d_Psi, double* d_Sbar,
                           double* d_Mbar, int32_t precision, void* stream) {
    API_BEGIN
    Level& L = level_at(h, level);
    if (k < 1 || k > h->q) fail(HSIM_E_INVALID, "k must be in [1, %d]", h->q);
    if (!d_Psi || !d_Sbar || !d_Mbar) fail(HSIM_E_INVALID, "null argument");
    if (precision != HSIM_FP64 && precision != HSIM_MIXED && precision != HSIM_GRAM_COMPENSATED)
        fail(HSIM_E_INVALID, "unknown precision");
    hipStream_t s = S_(stream);
    HIPCHECK(launch_gather_rows(d_Psi, k, dptr<int32_t>(L.dperm), L.n, k, dptr<double>(h->Psi), h->ld, s));
    apply_level(h, L, 0, dptr<double>(h->Psi), dptr<double>(h->SPsi), k, s);
    const bool fin = L.tau == 0;
    if (!fin) apply_level(h, L, 1, dptr<double>(h->Psi), dptr<double>(h->MPsi), k, s);
    HIPCHECK(launch_gram(dptr<double>(h->Psi), dptr<double>(h->SPsi), fin ? nullptr : dptr<double>(h->MPsi),
                         fin ? dptr<double>(L.dmdiag) : nullptr, L.n, k, h->ld, dptr<double>(h->gram_part), h->gram_chunk, d_Sbar,
                         d_Mbar, s,
                         precision == HSIM_MIXED ? GRAM_FP32
                                                 : (precision == HSIM_GRAM_COMPENSATED ? GRAM_COMPENSATED : GRAM_FP64)));
    API_END
}

hsim_status hsim_step_rr(int32_t k, const double* d_Sbar, const double* d_Mbar, double* d_lam, double* d_Phibar,
                         int32_t* sweeps, void* stream) {
    API_BEGIN
    if (k < 1) fail(HSIM_E_INVALID, "k must be >= 1");
    if (!d_Sbar || !d_Mbar || !d_lam || !d_Phibar) fail(HSIM_E_INVALID, "null argument");
    static thread_local std::unique_ptr<DenseGEP> g;
    if (!g) g.reset(new DenseGEP());
    g->setup(k, S_(stream));
    int32_t sw = g->run(d_Sbar, d_Mbar, k, d_lam, d_Phibar, k, S_(stream));
    if (sw < 0) fail(HSIM_E_FACTOR, "the reduced mass matrix is not positive definite");
    if (sweeps) *sweeps = sw;
    API_END
}

hsim_status hsim_step_rr_noalloc(int32_t k, const double* d_Sbar, const double* d_Mbar, double* d_lam,
                                 double* d_Phibar, int32_t* sweeps, void* stream) {
    API_BEGIN
    if (k < 1 || k > HSIM_RR_NOALLOC_MAX_K)
        fail(HSIM_E_INVALID, "k = %d outside [1, %d] of the allocation-free reduced eigenproblem", k,
             HSIM_RR_NOALLOC_MAX_K);
    if (!d_Sbar || !d_Mbar || !d_lam || !d_Phibar) fail(HSIM_E_INVALID, "null argument");
    hipStream_t s = S_(stream);
    char* base = rr_scratch_ptr();
    static thread_local DenseGEP g;   // host bookkeeping only; its device arrays are carved from the scratch region
    g.setup_in(k, base, RR_SCRATCH_BYTES, s);
    int32_t sw = g.run(d_Sbar, d_Mbar, k, d_lam, d_Phibar, k, s);
    if (sw < 0) fail(HSIM_E_FACTOR, "the reduced mass matrix is not positive definite");
    if (sweeps) *sweeps = sw;
    API_END
}

hsim_status hsim_step_ritz(hsim_hierarchy* h, int32_t level, int32_t k, const double* d_Psi, const double* d_Phibar,
                           const double* d_lam, double lam_floor, double* d_Phi, double* d_resid, void* stream) {
    API_BEGIN
    Level& L = level_at(h, level);
    if (k < 1 || k > h->q) fail(HSIM_E_INVALID, "k must be in [1, %d]", h->q);
    if (!d_Psi || !d_Phibar || !d_lam || !d_Phi || !d_resid) fail(HSIM_E_INVALID, "null argument");
    hipStream_t s = S_(stream);
    const bool fin = L.tau == 0;
    HIPCHECK(launch_gather_rows(d_Psi, k, dptr<int32_t>(L.dperm), L.n, k, dptr<double>(h->Psi), h->ld, s));
    apply_level(h, L, 0, dptr<double>(h->Psi), dptr<double>(h->SPsi), k, s);
    if (!fin) apply_level(h, L, 1, dptr<double>(h->Psi), dptr<double>(h->MPsi), k, s);
    HIPCHECK(launch_ritz(dptr<double>(h->Psi), dptr<double>(h->SPsi), fin ? nullptr : dptr<double>(h->MPsi),
                         fin ? dptr<double>(L.dmdiag) : nullptr, d_Phibar, d_lam, L.n, k, h->ld, dptr<double>(h->Phi),
                         nullptr, dptr<double>(h->ritz_part), 4096, fin, lam_floor, d_resid, s));
    HIPCHECK(launch_scatter_rows(dptr<double>(h->Phi), h->ld, dptr<int32_t>(L.dperm), L.n, k, d_Phi, k, s));
    API_END
}

static void coarse_solve(hsim_hierarchy* h, int32_t k, double* d_lam, double* d_Phi, int64_t ldphi, int32_t* sweeps,
                         hipStream_t s) {
    Level& C = *h->lv.back();
    const int64_t nc = C.n;
    HIPCHECK(launch_densify(dptr<int64_t>(C.dS_ptr), dptr<int32_t>(C.dS_idx), dptr<double>(C.dS_val), nc,
                            dptr<double>(h->coarseS), s));
    HIPCHECK(launch_densify(dptr<int64_t>(C.dS_ptr), dptr<int32_t>(C.dS_idx), dptr<double>(C.dM_val), nc,
                            dptr<double>(h->coarseM), s));
    h->coarse.setup((int32_t)nc, s);
    // Weyl's law for a surface, N(lambda) ~ area lambda / (4 pi): an eigenvalue
    // estimate a little above the k-th for the spectral projection (which
    // moves it itself when the count below it comes out too small or too
    // large); HSIM_COARSE_JACOBI=1 keeps the Jacobi sweeps on the whole level
    double area = 0.0;
    for (double v : C.Mval) area += v;
    const double sigma = (area > 0 && env_int("HSIM_COARSE_JACOBI", 0) == 0) ? 4.0 * M_PI * (1.3 * k + 8.0) / area : 0.0;
    int32_t sw = h->coarse.run(dptr<double>(h->coarseS), dptr<double>(h->coarseM), k, d_lam, d_Phi, ldphi, s,
                               DenseGEP::MAX_SWEEPS, sigma);
    if (sw < 0) fail(HSIM_E_FACTOR, "coarsest level: the mass matrix is not positive definite");
    if (env_int("HSIM_VERBOSE", 0) != 0)
        fprintf(stderr, "[hsim] coarsest level (%lld unknowns): %s, Jacobi sweeps %d\n", (long long)nc,
                h->coarse.proj_rank > 0 ? "spectral projection" : "Jacobi on the whole level", sw);
    if (env_int("HSIM_VERBOSE", 0) != 0 && h->coarse.proj_rank > 0)
        fprintf(stderr, "[hsim]   projector rank %d after %d Newton-Schulz steps\n", h->coarse.proj_rank,
                h->coarse.ns_iters);
    if (sweeps) *sweeps = sw;
}

hsim_status hsim_step_coarse(hsim_hierarchy* h, int32_t k, double* d_lam, double* d_Phi, int32_t* sweeps,
                             void* stream) {
    API_BEGIN
    if (!h || !d_lam || !d_Phi) fail(HSIM_E_INVALID, "null argument");
    if (h->host_only) fail(HSIM_E_STATE, "hierarchy was built host-only");
    if (k < 1 || k > h->lv.back()->n) fail(HSIM_E_INVALID, "k out of range");
    coarse_solve(h, k, d_lam, d_Phi, k, sweeps, S_(stream));
    API_END
}

// ---------------------------------------------------------------- solve
hsim_status hsim_solve(hsim_hierarchy* h, const hsim_solve_opts* opts, double* d_evals, double* d_evecs,
                       double* d_resid, hsim_stats* stats) {
    API_BEGIN
    if (!h || !d_evals || !d_evecs) fail(HSIM_E_INVALID, "null argument");
    if (h->host_only) fail(HSIM_E_STATE, "hierarchy was built host-only");
    hsim_solve_opts so;
    if (opts) so = *opts;
    else hsim_default_solve_opts(&so);
    if (!(so.tol > 0)) fail(HSIM_E_INVALID, "tol must be positive");
    if (so.max_iters < 1) fail(HSIM_E_INVALID, "max_iters must be >= 1");
    if (so.precision != HSIM_FP64 && so.precision != HSIM_MIXED) fail(HSIM_E_INVALID, "unknown precision");
    if (so.flags & ~(HSIM_FLAG_NOLOCK | HSIM_FLAG_SAVE_FORWARD | HSIM_FLAG_PROFILE | HSIM_FLAG_DETERMINISTIC |
                     HSIM_FLAG_COMPENSATED_GRAM | HSIM_FLAG_NO_FP32_GRAM | HSIM_FLAG_FP32_GRAM | HSIM_FLAG_GRAPH))
        fail(HSIM_E_INVALID, "unknown solve flags 0x%x", (unsigned)so.flags);
    const bool mixed = so.precision == HSIM_MIXED;
    // replayed graphs of the FP64 iteration body (not while every launch is timed)
    const bool use_graph = (so.flags & HSIM_FLAG_GRAPH) && !(so.flags & HSIM_FLAG_PROFILE);
    // Gram forms of a mixed solve: FP32 far from convergence (unless switched
    // off), then FP64 or, when asked for, compensated FP32
    // (by default only above q = 160, where the FP64 Gram is the multi-pass kernel too: below,
    // the single-pass FP64 kernel is faster than the multi-pass FP32 one)
    const bool gram32 = (so.flags & HSIM_FLAG_FP32_GRAM) != 0 ||
                        (!(so.flags & HSIM_FLAG_NO_FP32_GRAM) && h->q > gram_fp64_single_pass_max_q());
    const int hi_gram = (mixed && (so.flags & HSIM_FLAG_COMPENSATED_GRAM)) ? GRAM_COMPENSATED : GRAM_FP64;
    hipStream_t s = S_(so.stream);
    const auto T0 = std::chrono::steady_clock::now();
    hsim_stats st;
    std::memset(&st, 0, sizeof st);
    st.levels = h->T;
    st.q = h->q;
    st.ms_build = h->ms_build;
    const int32_t q = h->q, p = h->p, T = h->T;
    h->solved = false;
    h->prof.reset((so.flags & HSIM_FLAG_PROFILE) != 0);
    h->gram_steps[0] = h->gram_steps[1] = h->gram_steps[2] = 0;
    // coarsest level: dense solve, Phi in the coarsest level's order (= its internal order)
    std::vector<double> lam(q), res(q);
    {
        auto t0 = std::chrono::steady_clock::now();
        h->prof.run(HSIM_K_JACOBI, 0.0, 0.0, s,
                    [&] { coarse_solve(h, q, dptr<double>(h->lam), dptr<double>(h->Phi), h->ld, nullptr, s); });
        HIPCHECK(hipMemcpyAsync(lam.data(), h->lam.p, q * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        st.ms_coarse = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        st.n[0] = h->lv.back()->n;
        st.iters[0] = 0;
    }
    hsim_status final_status = HSIM_OK;
    for (int32_t tau = T - 2; tau >= 0; --tau) {
        Level& L = *h->lv[tau];
        const int li = T - 1 - tau;   // stats index, coarsest first
        st.n[li] = L.n;
        st.nnz_factor[li] = L.sy.tile_doubles;
        // prolongation
        auto t0 = std::chrono::steady_clock::now();
        HIPCHECK(launch_copy2d(dptr<double>(h->Phi), h->ld, h->lv[tau + 1]->n, q, dptr<double>(h->Xc), h->ld, s));
        prolong_level(h, L, dptr<double>(h->Xc), dptr<double>(h->Phi), q, s);
        HIPCHECK(hipStreamSynchronize(s));
        auto t1 = std::chrono::steady_clock::now();
        st.ms_prolong += std::chrono::duration<double, std::milli>(t1 - t0).count();
        // shift and factorisation (re-shift on breakdown)
        double mu = choose_shift(lam, p, so.shift_alpha);
        const int32_t j = (int32_t)std::floor(so.shift_alpha * p + 1e-12);
        // a quarter of the gap above the shift's eigenvalue estimate (lam: the
        // coarser level's estimates, or this level's latest Ritz values)
        auto shift_step = [&] {
            const int32_t jj = std::min<int32_t>(j + 1, q - 1);
            return 0.25 * std::max(lam[jj] - lam[std::min<int32_t>(j, q - 1)], 1e-6 * std::fabs(lam[jj]));
        };
        auto factor_reshift = [&] {
            for (int attempt = 0;; ++attempt) {
                try {
                    factor_level(h, L, mu, s, mixed);
                    break;
                } catch (const Error& e) {
                    if (e.code != HSIM_E_FACTOR || attempt >= 3) throw;
                    mu += shift_step();
                }
            }
        };
        factor_reshift();
        st.mu[li] = mu;
        st.neg_pivots[li] = L.neg_pivots;
        auto t2 = std::chrono::steady_clock::now();
        st.ms_factor += std::chrono::duration<double, std::milli>(t2 - t1).count();
        // subspace iterations
        int32_t locked = 0, it = 0;
        bool conv = false;
        double rmax = INFINITY;   // largest residual of the first p pairs after the last Rayleigh-Ritz step
        bool fp64_gram = false;
        double est32 = -1.0;      // backward error of a plain FP32 solve on this level's factor
        int32_t rr_reshifts = 0;
        for (it = 1; it <= so.max_iters; ++it) {
            auto a0 = std::chrono::steady_clock::now();
            const int32_t act = q - locked;
            // mixed precision: the solves' target accuracy for this step; once a
            // plain FP32 solve on this factor is known to miss it, the step runs
            // the FP64 solves (the same launches as an FP64 solve, no probing)
            const double eta = std::min(1e-3, 0.1 * (std::isfinite(rmax) ? rmax : 1e-2));
            const bool fp64_solves = !mixed || (est32 >= 0 && est32 > eta);
            // the active columns go from Phi into Psi with the two solves of the
            // iteration; the locked ones (not iterated) are copied from Phi after
            if (act > 0 && fp64_solves) {
                // FP64: the two inverse iterations of the step (kernels only, no host
                // synchronisation), as one replayed graph with HSIM_FLAG_GRAPH
                auto body = [&](hipStream_t ss) {
                    if (tau == 0) {
                        // Phi -> Psi -> Btmp, out of place (lets the forward sweep split
                        // narrow tree levels); Btmp becomes Psi after the step
                        solve_level(h, L, dptr<double>(h->Psi), locked, act, true, ss, false, dptr<double>(h->Phi));
                        solve_level(h, L, dptr<double>(h->Btmp), locked, act, true, ss, false, dptr<double>(h->Psi));
                    } else {
                        for (int rep = 0; rep < 2; ++rep) {
                            double* src = dptr<double>(rep == 0 ? h->Phi : h->Psi);
                            h->prof.run(HSIM_K_SPMM, 12.0 * L.S.nnz() + 16.0 * L.n * act, 2.0 * L.S.nnz() * act, ss,
                                        [&] {
                                            pattern_spmm(L, false, false, 1.0, 0.0, src + locked, h->ld, act,
                                                         dptr<double>(h->Btmp) + locked, h->ld, ss);
                                        });
                            solve_level(h, L, dptr<double>(h->Psi), locked, act, false, ss, false,
                                        dptr<double>(h->Btmp));
                        }
                    }
                };
                if (use_graph) {
                    const std::array<intptr_t, 5> key{tau, locked, (intptr_t)h->Phi.p, (intptr_t)h->Psi.p,
                                                      (intptr_t)h->Btmp.p};
                    auto g = h->graphs.find(key);
                    if (g == h->graphs.end()) {
                        hipGraph_t graph = nullptr;
                        // captured on the hierarchy's own stream (the caller's may be the
                        // null stream, which cannot capture), replayed on the caller's
                        if (!h->cap_stream) HIPCHECK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
                        HIPCHECK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
                        try {
                            body(h->cap_stream);
                        } catch (...) {
                            hipGraph_t dead = nullptr;
                            (void)hipStreamEndCapture(h->cap_stream, &dead);
                            if (dead) (void)hipGraphDestroy(dead);
                            throw;
                        }
                        HIPCHECK(hipStreamEndCapture(h->cap_stream, &graph));
                        hipGraphExec_t exec = nullptr;
                        const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                        (void)hipGraphDestroy(graph);
                        HIPCHECK(e);
                        g = h->graphs.emplace(key, exec).first;
                    } else {
                        h->prof.solves += 2;   // counted by the host code of the capture otherwise
                        h->prof.solve_cols += 2 * (int64_t)act;
                    }
                    HIPCHECK(hipGraphLaunch(g->second, s));
                } else {
                    body(s);
                }
                if (tau == 0) swap_buffers(h->Psi, h->Btmp);
            }
            if (act > 0 && !fp64_solves) {
                for (int rep = 0; rep < 2; ++rep) {
                    double* src = dptr<double>(rep == 0 ? h->Phi : h->Psi);
                    // B = M src
                    if (tau == 0)
                        HIPCHECK(launch_diag_scale(dptr<double>(L.dmdiag), L.n, src + locked, h->ld, act,
                                                   dptr<double>(h->Btmp) + locked, h->ld, s));
                    else
                        h->prof.run(HSIM_K_SPMM, 12.0 * L.S.nnz() + 16.0 * L.n * act, 2.0 * L.S.nnz() * act, s, [&] {
                            pattern_spmm(L, false, false, 1.0, 0.0, src + locked, h->ld, act,
                                         dptr<double>(h->Btmp) + locked, h->ld, s);
                        });
                    st.refine_steps += refine_solve(h, L, dptr<double>(h->Btmp), dptr<double>(h->Psi), locked, act,
                                                    eta, s, &st.escalated, &est32);
                }
            }
            if (locked > 0)
                HIPCHECK(launch_copy2d(dptr<double>(h->Phi), h->ld, L.n, locked, dptr<double>(h->Psi), h->ld, s));
            HIPCHECK(hipStreamSynchronize(s));
            st.ms_solve += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a0).count();
            // FP32 Gram only far from convergence (its rounding bounds the Ritz
            // vectors' accuracy; switch for good once it stops paying off); the
            // other steps of a mixed solve take the FP64 Gram, or the compensated
            // one when asked for
            bool low_gram = mixed && !fp64_gram && gram32 && rmax > std::max(100.0 * so.tol, 1e-4);
            const int mode = low_gram ? GRAM_FP32 : (fp64_gram ? GRAM_FP64 : hi_gram);
            bool rr_done = false;
            try {
                if (!rayleigh_ritz(h, L, lam, res, s, &st.ms_gram, &st.ms_rr, &st.ms_ritz, mode)) {
                    // the low-precision Gram lost the definiteness of the reduced mass matrix
                    // (an ill-conditioned basis): this step and the rest of the level in FP64
                    fp64_gram = true;
                    low_gram = false;
                    rayleigh_ritz(h, L, lam, res, s, &st.ms_gram, &st.ms_rr, &st.ms_ritz, GRAM_FP64);
                }
                rr_done = true;
            } catch (const Error& e) {
                if (e.code != HSIM_E_FACTOR || rr_reshifts >= 3) throw;
            }
            if (!rr_done) {
                // even the FP64 reduced mass matrix is not positive definite: the
                // two inverse iterations multiplied the component of an
                // eigenvector whose eigenvalue lies almost on the shift by
                // 1 / (lambda - mu)^2 until the columns were numerically
                // dependent.  The shift moves as after a factorisation breakdown,
                // the level is factored again and this step is redone from Phi
                // (which a failed step leaves unchanged)
                ++rr_reshifts;
                mu += shift_step();
                factor_reshift();
                st.mu[li] = mu;
                st.neg_pivots[li] = L.neg_pivots;
                est32 = -1.0;
                --it;
                continue;
            }
            auto check = [&] {
                conv = true;
                rmax = 0;
                for (int32_t i = 0; i < p; ++i) {
                    conv &= res[i] < so.tol;
                    rmax = std::max(rmax, res[i]);
                }
            };
            const double rprev = rmax;
            check();
            // a low-precision or compensated step that does not halve the largest residual
            // has reached the accuracy of its Gram: the rest of the level in FP64
            if ((low_gram || mode == GRAM_COMPENSATED) && !(rmax < 0.5 * rprev)) fp64_gram = true;
            // the returned basis never comes from the FP32 Gram (FP64 or compensated)
            if (conv && low_gram) {
                if (!rayleigh_ritz(h, L, lam, res, s, &st.ms_gram, &st.ms_rr, &st.ms_ritz,
                                   fp64_gram ? GRAM_FP64 : hi_gram)) {
                    fp64_gram = true;
                    rayleigh_ritz(h, L, lam, res, s, &st.ms_gram, &st.ms_rr, &st.ms_ritz, GRAM_FP64);
                }
                check();
            }
            if (conv) break;
            if (!(so.flags & HSIM_FLAG_NOLOCK)) {
                int32_t r = 0;
                while (r < q && res[r] < so.tol / 10.0) ++r;
                locked = std::min(r, p);
            }
        }
        st.iters[li] = std::min(it, so.max_iters);
        if (!conv) final_status = HSIM_E_NOCONV;
    }
    // outputs: first p pairs of level 0
    Level& L0 = *h->lv[0];
    HIPCHECK(hipMemcpyAsync(d_evals, h->lam.p, p * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (d_resid) HIPCHECK(hipMemcpyAsync(d_resid, h->resid.p, p * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (L0.n < h->mesh.nv) HIPCHECK(launch_fill(d_evecs, (int64_t)p * h->mesh.nv, 0.0, s));   // Dirichlet boundary rows
    HIPCHECK(launch_export_evecs(dptr<double>(h->Phi), h->ld, L0.n, p, dptr<int32_t>(L0.dmeshmap), h->mesh.nv, d_evecs,
                                 dptr<double>(h->exportw), s));
    HIPCHECK(hipStreamSynchronize(s));
    h->last_lam = lam;
    h->solved = final_status == HSIM_OK;   // the adjoint needs converged eigenpairs
    h->prof.collect(st, s);
    for (int g = 0; g < 3; ++g) st.gram_steps[g] = h->gram_steps[g];
    st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - T0).count();
    if (stats) *stats = st;
    if (final_status != HSIM_OK) {
        set_last_error("subspace iterations did not converge within max_iters");
        return final_status;
    }
    API_END
}

hsim_status hsim_solve_batch(hsim_hierarchy* const* hs, int32_t count, const hsim_solve_opts* opts,
                             double* const* d_evals, double* const* d_evecs, double* const* d_resid,
                             hsim_stats* stats, int32_t* status, int32_t streams) {
    API_BEGIN
    if (count < 0 || (count > 0 && (!hs || !d_evals || !d_evecs))) fail(HSIM_E_INVALID, "null argument");
    if (count == 0) return HSIM_OK;
    for (int32_t i = 0; i < count; ++i)
        if (!hs[i] || !d_evals[i] || !d_evecs[i]) fail(HSIM_E_INVALID, "null argument for mesh %d", i);
    hsim_solve_opts so;
    if (opts) so = *opts;
    else hsim_default_solve_opts(&so);
    const int32_t nw = std::max(1, std::min(count, streams > 0 ? streams : 8));
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    // the workers' streams start after the caller's stream has reached this call
    hipEvent_t start;
    HIPCHECK(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    HIPCHECK(hipEventRecord(start, S_(so.stream)));
    // largest meshes first: the queue ends with the short solves
    std::vector<int32_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return hs[a]->lv[0]->n > hs[b]->lv[0]->n; });
    std::atomic<int32_t> next{0};
    std::vector<int32_t> st(count, HSIM_OK);
    std::vector<std::string> msg(count);
    std::vector<std::string> werr(nw);
    auto worker = [&](int w) {
        hipStream_t ws = nullptr;
        if (hipSetDevice(dev) != hipSuccess || hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) != hipSuccess ||
            hipStreamWaitEvent(ws, start, 0) != hipSuccess) {
            werr[w] = "worker stream set-up failed";
            if (ws) (void)hipStreamDestroy(ws);
            return;
        }
        hsim_solve_opts o = so;
        o.stream = ws;
        for (;;) {
            const int32_t k = next.fetch_add(1);
            if (k >= count) break;
            const int32_t i = order[k];
            st[i] = hsim_solve(hs[i], &o, d_evals[i], d_evecs[i], d_resid ? d_resid[i] : nullptr,
                               stats ? &stats[i] : nullptr);
            if (st[i] != HSIM_OK) msg[i] = hsim_last_error();
        }
        if (hipStreamSynchronize(ws) != hipSuccess) werr[w] = "worker stream failed";
        (void)hipStreamDestroy(ws);
    };
    std::vector<std::thread> pool;
    for (int w = 1; w < nw; ++w) pool.emplace_back(worker, w);
    worker(0);
    for (auto& t : pool) t.join();
    (void)hipEventDestroy(start);
    for (int w = 0; w < nw; ++w)
        if (!werr[w].empty()) fail(HSIM_E_DEVICE, "%s", werr[w].c_str());
    if (status)
        for (int32_t i = 0; i < count; ++i) status[i] = st[i];
    for (int32_t i = 0; i < count; ++i)
        if (st[i] != HSIM_OK) {
            set_last_error("mesh " + std::to_string(i) + ": " + msg[i]);
            return (hsim_status)st[i];
        }
    API_END
}

// ------------------------------------------------------------- autotuning
// Candidate launch plans of the block solves: the widest-front thresholds
// (padded pivots) from which a tree level's forward / backward sweep
// multiplies by the inverse panels instead of running the wave-level solve.
static const int32_t kTuneNs[] = {64, 96, 128, 256, 512};
static std::mutex g_tune_mu;

static std::string tune_key(const hsim_hierarchy* h, const Level& L) {
    int32_t top = 0;
    for (const TLev& T : L.tl) top = std::max(top, T.ns_pad_max);
    // meshes with the same subspace size, tree height, widest front and size
    // class share a plan (size class: the level size to two significant binary digits)
    int64_t n = L.n, sc = 0;
    while (n >= 4) { n >>= 1; ++sc; }
    char buf[160];
    std::snprintf(buf, sizeof buf, "inverse-panel-plan q=%d tree=%d top=%d size=%lld.%lld", h->q, (int)L.tl.size(), top,
                  (long long)sc, (long long)n);
    return buf;
}

static bool tune_cache_lookup(const std::string& key, int32_t* f, int32_t* b, double* ms) {
    const char* path = std::getenv("HSIM_TUNE_CACHE");
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    FILE* fp = std::fopen(path, "r");
    if (!fp) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, fp)) {
        const char* bar = std::strchr(line, '|');
        if (!bar || std::string(line, bar - line) != key) continue;
        int32_t ff, bb;
        double mm;
        if (std::sscanf(bar + 1, "%d %d %lf", &ff, &bb, &mm) == 3) {
            *f = ff, *b = bb, *ms = mm;
            found = true;   // the last entry of a key wins
        }
    }
    std::fclose(fp);
    return found;
}

static void tune_cache_store(const std::string& key, int32_t f, int32_t b, double ms) {
    const char* path = std::getenv("HSIM_TUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    FILE* fp = std::fopen(path, "a");
    if (!fp) return;
    std::fprintf(fp, "%s|%d %d %.6f\n", key.c_str(), f, b, ms);
    std::fclose(fp);
}

hsim_status hsim_autotune(hsim_hierarchy* h, int32_t level, void* stream, hsim_tune_result* out) {
    API_BEGIN
    Level& L = level_at(h, level);
    if (L.coarsest) fail(HSIM_E_INVALID, "the coarsest level is solved densely");
    hipStream_t s = S_(stream);
    const std::string key = tune_key(h, L);
    hsim_tune_result r{};
    int32_t f = 0, b = 0;
    double ms = 0;
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);   // they hold the old plan's launches
    h->graphs.clear();
    if (tune_cache_lookup(key, &f, &b, &ms)) {
        plan_solve(L, f, b);
        r.big_ns = f, r.big_ns_bwd = b, r.ms = ms, r.from_cache = 1;
    } else {
        // time the q-column block solve of every plan on a factor of S - mu M
        // with mu below the spectrum (the times do not depend on the values)
        const double mu = -1e-3;
        factor_level(h, L, mu, s, false);
        double* X = dptr<double>(h->Psi);
        double* B = dptr<double>(h->Btmp);
        HIPCHECK(launch_fill(B, L.n * h->ld, 1.0, s));
        hipEvent_t e0, e1;
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        auto time_plan = [&](int32_t cf, int32_t cb) {
            plan_solve(L, cf, cb);
            solve_level(h, L, X, 0, h->q, false, s, false, B);   // warm-up
            double t = INFINITY;
            for (int rep = 0; rep < 3; ++rep) {
                HIPCHECK(hipEventRecord(e0, s));
                solve_level(h, L, X, 0, h->q, false, s, false, B);
                HIPCHECK(hipEventRecord(e1, s));
                HIPCHECK(hipEventSynchronize(e1));
                float m = 0;
                HIPCHECK(hipEventElapsedTime(&m, e0, e1));
                t = std::min(t, (double)m);
            }
            return t;
        };
        // the forward and backward sweeps add up: the forward threshold is
        // chosen with the backward one at 128, then the backward threshold
        // with that forward one
        double best = INFINITY;
        int32_t bf = 128, bb = 128;
        for (int32_t cf : kTuneNs) {
            const double t = time_plan(cf, bb);
            if (t < best) best = t, bf = cf;
        }
        for (int32_t cb : kTuneNs) {
            if (cb == 128) continue;   // timed above
            const double t = time_plan(bf, cb);
            if (t < best) best = t, bb = cb;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        plan_solve(L, bf, bb);
        tune_cache_store(key, bf, bb, best);
        r.big_ns = bf, r.big_ns_bwd = bb, r.ms = best, r.from_cache = 0;
    }
    if (out) *out = r;
    API_END
}

static void backward_setup(hsim_hierarchy* h) {
    if (h->bw_ready) return;
    const Mesh& m = h->mesh;
    Level& L0 = *h->lv[0];
    h->bV.upload(m.V);
    h->bF.upload(m.F);
    if (!h->density.empty()) h->bRho.upload(h->density);
    // mesh vertex -> internal row of level 0; -1 for a vertex the level does not
    // keep (the boundary under the Dirichlet condition), whose values are zero
    std::vector<int32_t> vrow(m.nv, -1);
    for (int64_t j = 0; j < L0.n; ++j) vrow[L0.verts[j]] = L0.sy.iperm[j];
    h->bIperm.upload(vrow);
    // vertex -> (triangle, corner) lists in triangle order
    std::vector<int64_t> ptr(m.nv + 1, 0), vt(3 * m.nf);
    for (int64_t t = 0; t < m.nf; ++t)
        for (int c = 0; c < 3; ++c) ptr[m.F[3 * t + c] + 1]++;
    for (int64_t v = 0; v < m.nv; ++v) ptr[v + 1] += ptr[v];
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t t = 0; t < m.nf; ++t)
        for (int c = 0; c < 3; ++c) vt[fill[m.F[3 * t + c]]++] = 3 * t + c;
    h->bVtPtr.upload(ptr);
    h->bVt.upload(vt);
    h->bG.alloc((size_t)m.nf * 9 * sizeof(double));
    h->bNu.alloc((size_t)m.nv * sizeof(double));
    const size_t blk = (size_t)L0.n * h->ld * sizeof(double);
    for (DeviceBuffer* b : {&h->bGbar, &h->bMX, &h->bW, &h->bY, &h->bR, &h->bZ, &h->bP, &h->bQ}) b->alloc(blk);
    h->bSmall.alloc((size_t)(4 * h->q * h->q + 16 * h->ld) * sizeof(double));
    h->bPart.alloc((size_t)std::max(tsgemm_partial_doubles(L0.n, h->q, h->ld), coldot_partial_doubles(L0.n, h->ld)) *
                   sizeof(double));
    h->bDots.alloc((size_t)8 * h->ld * sizeof(double));
    h->bw_ready = true;
}

hsim_status hsim_solve_backward(hsim_hierarchy* h, const double* d_grad_evals, const double* d_grad_evecs,
                                double* d_grad_V, void* stream) {
    API_BEGIN
    if (!h || !d_grad_V) fail(HSIM_E_INVALID, "null argument");
    if (h->host_only) fail(HSIM_E_STATE, "hierarchy was built host-only");
    if (!h->solved) fail(HSIM_E_STATE, "hsim_solve_backward before a successful hsim_solve");
    hipStream_t s = S_(stream);
    backward_setup(h);
    Level& L0 = *h->lv[0];
    const int64_t n = L0.n, nv = h->mesh.nv, nf = h->mesh.nf;
    const int32_t p = h->p, q = h->q, ld = h->ld;
    const double* X = dptr<double>(h->Phi);    // level-0 Ritz vectors, internal order
    const double* lam = dptr<double>(h->lam);
    const double* md = dptr<double>(L0.dmdiag);
    double* W = nullptr;
    double* Y = nullptr;
    double* part = dptr<double>(h->bPart);
    h->cg_iters = 0;
    if (d_grad_evecs) {
        double* Gb = dptr<double>(h->bGbar);
        double* MX = dptr<double>(h->bMX);
        double* R = dptr<double>(h->bR);
        double* Z = dptr<double>(h->bZ);
        double* P = dptr<double>(h->bP);
        double* Qm = dptr<double>(h->bQ);
        W = dptr<double>(h->bW);
        Y = dptr<double>(h->bY);
        double* C0 = dptr<double>(h->bSmall);                 // q x p
        double* Cin = C0 + (size_t)q * q;                    // q x p
        double* Gam = Cin + (size_t)q * q;                   // q x p
        double* Cp = Gam + (size_t)q * q;                    // q x p (projections)
        double* dots = dptr<double>(h->bDots);
        double* rz = dots, *pq = dots + ld, *alpha = dots + 2 * ld, *rz2 = dots + 3 * ld, *beta = dots + 4 * ld,
              *rr = dots + 5 * ld;
        // the returned eigenvectors carry the sign of the export (largest entry positive):
        // dL/dPhi_k = sign_k dL/dx_k
        const int64_t nch_exp = (n + 8191) / 8192;
        const double* sign = dptr<double>(h->exportw) + 2 * nch_exp * p;
        // rows of the kept vertices only: a boundary row of an eigenvector is zero
        // under the Dirichlet condition, so its gradient there does not enter
        HIPCHECK(launch_import_cols(d_grad_evecs, nv, dptr<int32_t>(L0.dmeshmap), n, p, Gb, ld, s, sign));
        HIPCHECK(launch_diag_scale(md, n, X, ld, q, MX, ld, s));
        std::vector<double> lamh(q);
        HIPCHECK(hipMemcpyAsync(lamh.data(), lam, q * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        // clusters: maximal runs of Ritz values with relative gaps below 1e-2
        std::vector<int32_t> cl(q, 0);
        for (int32_t j = 1; j < q; ++j) {
            const double den = std::fabs(lamh[j]) > 0 ? std::fabs(lamh[j]) : 1.0;
            cl[j] = cl[j - 1] + (((lamh[j] - lamh[j - 1]) / den) >= 1e-2 ? 1 : 0);
        }
        // The spectral part uses the converged pairs only: the first p and the
        // rest of the cluster of pair p-1 (the remaining Ritz pairs are not
        // eigenpairs to the tolerance, so the complement solve covers them).
        int32_t ps = p;
        while (ps < q && cl[ps] == cl[p - 1]) ++ps;
        if (ps == q) fail(HSIM_E_UNIMPLEMENTED, "the cluster of eigenpair p-1 extends to the end of the subspace");
        // coefficients of the gradient in the converged Ritz basis: C0 = X_ps^T Gbar
        HIPCHECK(launch_tsgemm_tn(X, ld, Gb, ld, n, ps, p, part, C0, s));
        std::vector<double> c0((size_t)ps * p);
        HIPCHECK(hipMemcpyAsync(c0.data(), C0, c0.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        std::vector<double> cin((size_t)ps * p, 0.0), gam((size_t)ps * p, 0.0);
        for (int32_t k = 0; k < p; ++k)
            for (int32_t j = 0; j < ps; ++j) {
                const double cjk = c0[(size_t)j * p + k];
                if (cl[j] != cl[k]) {
                    cin[(size_t)j * p + k] = cjk / (lamh[j] - lamh[k]);
                } else {
                    // same cluster: normalisation term with the symmetrised coefficient
                    const double ckj = j < p ? c0[(size_t)k * p + j] : 0.0;   // no gradient on x_j, j >= p
                    gam[(size_t)j * p + k] = j == k ? cjk : 0.5 * (cjk + ckj);
                }
            }
        HIPCHECK(hipMemcpyAsync(Cin, cin.data(), cin.size() * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(Gam, gam.data(), gam.size() * sizeof(double), hipMemcpyHostToDevice, s));
        // right-hand side on the complement: r = Gbar - M X_q C0
        HIPCHECK(launch_copy2d(Gb, ld, n, p, R, ld, s));
        HIPCHECK(launch_tsgemm_nn(MX, ld, n, ps, C0, p, -1.0, 1.0, R, ld, s));
        // PCG on {w : X_q^T M w = 0} for (S - lam_k M) w_k = r_k, preconditioned by
        // the level-0 factor of S - mu M and the M-orthogonal projection
        auto apply_prec = [&](const double* Rin, double* Zout) {
            HIPCHECK(launch_copy2d(Rin, ld, n, p, Zout, ld, s));
            solve_level(h, L0, Zout, 0, p, false, s);
            HIPCHECK(launch_tsgemm_tn(MX, ld, Zout, ld, n, ps, p, part, Cp, s));
            HIPCHECK(launch_tsgemm_nn(X, ld, n, ps, Cp, p, -1.0, 1.0, Zout, ld, s));
        };
        HIPCHECK(launch_fill(W, n * ld, 0.0, s));
        apply_prec(R, Z);
        HIPCHECK(launch_copy2d(Z, ld, n, p, P, ld, s));
        HIPCHECK(launch_coldot(R, Z, n, ld, p, part, rz, s));
        HIPCHECK(launch_coldot(R, R, n, ld, p, part, rr, s));
        std::vector<double> r0(p), rc(p);
        HIPCHECK(hipMemcpyAsync(r0.data(), rr, p * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        const double cg_tol = 1e-12;
        int it = 0;
        for (it = 1; it <= 1000; ++it) {
            apply_level(h, L0, 0, P, Qm, p, s);                       // Q = S P
            HIPCHECK(launch_shift_cols(Qm, P, md, lam, n, ld, p, s));  // Q -= lam_k M P
            HIPCHECK(launch_coldot(P, Qm, n, ld, p, part, pq, s));
            HIPCHECK(launch_div_cols(rz, pq, alpha, p, s));
            HIPCHECK(launch_axpy_cols(W, P, alpha, 0, n, ld, p, s));
            HIPCHECK(launch_axpy_cols(R, Qm, alpha, 1, n, ld, p, s));
            // keep the residual in the dual of the complement
            HIPCHECK(launch_tsgemm_tn(X, ld, R, ld, n, ps, p, part, Cp, s));
            HIPCHECK(launch_tsgemm_nn(MX, ld, n, ps, Cp, p, -1.0, 1.0, R, ld, s));
            if (it % 4 == 0) {
                HIPCHECK(launch_coldot(R, R, n, ld, p, part, rr, s));
                HIPCHECK(hipMemcpyAsync(rc.data(), rr, p * sizeof(double), hipMemcpyDeviceToHost, s));
                HIPCHECK(hipStreamSynchronize(s));
                bool done = true;
                for (int32_t k = 0; k < p; ++k) done &= !(rc[k] > cg_tol * cg_tol * r0[k]);
                if (done) break;
            }
            apply_prec(R, Z);
            HIPCHECK(launch_coldot(R, Z, n, ld, p, part, rz2, s));
            HIPCHECK(launch_div_cols(rz2, rz, beta, p, s));
            HIPCHECK(launch_axpy_cols(P, Z, beta, 2, n, ld, p, s));
            std::swap(rz, rz2);
        }
        h->cg_iters = it;
        if (it > 1000) fail(HSIM_E_NOCONV, "adjoint PCG did not converge");
        // w_k += in-span part; Y = X_cluster Gamma
        HIPCHECK(launch_tsgemm_nn(X, ld, n, ps, Cin, p, 1.0, 1.0, W, ld, s));
        HIPCHECK(launch_tsgemm_nn(X, ld, n, ps, Gam, p, 1.0, 0.0, Y, ld, s));
    }
    const int32_t* ip = dptr<int32_t>(h->bIperm);
    HIPCHECK(launch_bwd_vertex(nv, p, X, W, Y, ld, ip, lam, d_grad_evals, h->density.empty() ? nullptr : dptr<double>(h->bRho),
                               dptr<double>(h->bNu), s));
    HIPCHECK(launch_bwd_tri(nf, dptr<int32_t>(h->bF), dptr<double>(h->bV), p, X, W, ld, ip, d_grad_evals,
                            dptr<double>(h->bNu), h->bo.lumping, dptr<double>(h->bG), s));
    HIPCHECK(launch_bwd_gather(nv, dptr<int64_t>(h->bVtPtr), dptr<int64_t>(h->bVt), dptr<double>(h->bG), d_grad_V, s));
    HIPCHECK(hipStreamSynchronize(s));
    API_END
}

}  // extern "C"

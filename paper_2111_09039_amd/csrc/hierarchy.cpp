// Hierarchy of nested spaces (Section 4.1): level sizes (eq. nT-1,
// eq. growthRate), vertex hierarchy by farthest point sampling (Algorithm 3),
// prolongation operators (eq. radius, eq. basis, row normalisation) and the
// Galerkin operators of Algorithm 2.
//
// Readings where the paper is garbled or silent:
//  * growth rate: the default takes the (T-1)-th root so that the levels run
//    from n^{T-1} to n^0; growth_mode 1 keeps the printed T-th root;
//  * U^tau has one row per fine vertex and one column per coarse vertex, and
//    the radius uses the coarse count n^{tau+1} (each disk then holds about
//    sigma coarse samples); a fine vertex with no coarse vertex inside the
//    radius takes weight 1 on its nearest coarse vertex;
//  * the start vertex is seed mod n, farthest-point ties go to the lowest
//    vertex index, nearest-vertex ties to the lowest coarse index.
#include <algorithm>
#include <cmath>
#include <limits>
#include <queue>

#include <omp.h>

#include "internal.h"

namespace hsim {

std::vector<int64_t> level_sizes(int64_t n0, int T, int64_t n_coarsest, int growth_mode) {
    if (T < 1) fail(HSIM_E_INVALID, "levels must be >= 1");
    std::vector<int64_t> s{n0};
    if (T == 1) return s;
    int64_t nc = std::min(n_coarsest, n0);
    double root = growth_mode == 0 ? (double)(T - 1) : (double)T;
    double g = std::pow((double)n0 / (double)nc, 1.0 / root);
    for (int tau = 1; tau < T - 1; ++tau) {
        double v = std::nearbyint(std::pow(g, (double)(T - 1 - tau)) * (double)nc);
        s.push_back(std::min<int64_t>(n0, std::max<int64_t>(nc, (int64_t)v)));
    }
    s.push_back(nc);
    return s;
}

namespace {
constexpr double INF = std::numeric_limits<double>::infinity();
using HeapItem = std::pair<double, int32_t>;
using MinHeap = std::priority_queue<HeapItem, std::vector<HeapItem>, std::greater<HeapItem>>;

// arg-max tournament tree (largest value, lowest index on ties)
struct ArgMaxTree {
    int64_t P = 1;
    std::vector<double> val;
    std::vector<int32_t> idx;
    explicit ArgMaxTree(int64_t n) {
        while (P < n) P <<= 1;
        val.assign(2 * P, -INF);
        idx.assign(2 * P, std::numeric_limits<int32_t>::max());
        for (int64_t i = 0; i < n; ++i) { val[P + i] = INF; idx[P + i] = (int32_t)i; }
        for (int64_t k = P - 1; k >= 1; --k) pull(k);
    }
    void pull(int64_t k) {
        int64_t a = 2 * k, b = 2 * k + 1;
        bool left = val[a] > val[b] || (val[a] == val[b] && idx[a] < idx[b]);
        val[k] = left ? val[a] : val[b];
        idx[k] = left ? idx[a] : idx[b];
    }
    void set(int32_t i, double v) {
        int64_t k = P + i;
        val[k] = v;
        for (k >>= 1; k >= 1; k >>= 1) pull(k);
    }
};

// dist <- min(dist, graph distance from src), visiting only improved vertices
void relax_from(const Graph& g, int32_t src, std::vector<double>& dist, ArgMaxTree& tree) {
    MinHeap heap;
    dist[src] = 0.0;
    tree.set(src, 0.0);
    heap.push({0.0, src});
    while (!heap.empty()) {
        auto [dv, v] = heap.top();
        heap.pop();
        if (dv > dist[v]) continue;
        for (int64_t k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
            int32_t u = g.nbr[k];
            double nd = dv + g.w[k];
            if (nd < dist[u]) {
                dist[u] = nd;
                tree.set(u, nd);
                heap.push({nd, u});
            }
        }
    }
}
}  // namespace

// Algorithm 3: returns the insertion order of the first `count` samples
std::vector<int32_t> farthest_point_sampling(const Graph& g, int64_t n, int64_t count, uint64_t seed) {
    std::vector<double> dist(n, INF);
    ArgMaxTree tree(n);
    std::vector<int32_t> order;
    order.reserve(count);
    int32_t s = (int32_t)(seed % (uint64_t)n);
    order.push_back(s);
    relax_from(g, s, dist, tree);
    while ((int64_t)order.size() < count) {
        s = tree.idx[1];
        if (!(tree.val[1] > 0)) fail(HSIM_E_MESH, "farthest point sampling ran out of distinct vertices");
        order.push_back(s);
        relax_from(g, s, dist, tree);
    }
    return order;
}

Csr prolongation(const Graph& g, int64_t n, const std::vector<int32_t>& fine_verts, bool fine_is_all,
                 const std::vector<int32_t>& coarse_verts, double sigma, double area, double* rho_out) {
    const int64_t nc = (int64_t)coarse_verts.size();
    const int64_t nf = fine_is_all ? n : (int64_t)fine_verts.size();
    const double rho = std::sqrt(sigma * area / ((double)nc * M_PI));
    if (rho_out) *rho_out = rho;
    std::vector<int32_t> pos(n, -1);
    if (fine_is_all)
        for (int64_t i = 0; i < n; ++i) pos[i] = (int32_t)i;
    else
        for (int64_t j = 0; j < nf; ++j) pos[fine_verts[j]] = (int32_t)j;

    // one bounded Dijkstra ball per coarse vertex, in parallel
    struct Ent { int32_t row; double w; };
    std::vector<std::vector<Ent>> cols(nc);
#pragma omp parallel
    {
        std::vector<double> dist(n, INF);
        std::vector<int32_t> touched;
        std::vector<char> done(n, 0);
#pragma omp for schedule(dynamic, 4)
        for (int64_t ci = 0; ci < nc; ++ci) {
            MinHeap heap;
            int32_t src = coarse_verts[ci];
            dist[src] = 0.0;
            touched.push_back(src);
            heap.push({0.0, src});
            while (!heap.empty()) {
                auto [dv, v] = heap.top();
                heap.pop();
                if (done[v]) continue;
                if (dv >= rho) break;
                done[v] = 1;
                if (pos[v] >= 0) {
                    double wt = 1.0 - dv / rho;
                    if (wt > 0.0) cols[ci].push_back({pos[v], wt});
                }
                for (int64_t k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
                    int32_t u = g.nbr[k];
                    double nd = dv + g.w[k];
                    if (nd < dist[u]) {
                        if (dist[u] == INF) touched.push_back(u);
                        dist[u] = nd;
                        heap.push({nd, u});
                    }
                }
            }
            for (int32_t v : touched) { dist[v] = INF; done[v] = 0; }
            touched.clear();
        }
    }
    // transpose into CSR by fine rows, columns ascending
    Csr U;
    U.rows = nf;
    U.cols = nc;
    U.ptr.assign(nf + 1, 0);
    for (int64_t ci = 0; ci < nc; ++ci)
        for (auto& e : cols[ci]) U.ptr[e.row + 1]++;
    for (int64_t j = 0; j < nf; ++j) U.ptr[j + 1] += U.ptr[j];
    U.idx.resize(U.ptr[nf]);
    U.val.resize(U.ptr[nf]);
    {
        std::vector<int64_t> fill(U.ptr.begin(), U.ptr.end() - 1);
        for (int64_t ci = 0; ci < nc; ++ci)
            for (auto& e : cols[ci]) {
                U.idx[fill[e.row]] = (int32_t)ci;
                U.val[fill[e.row]++] = e.w;
            }
    }
    // empty rows: weight 1 on the nearest coarse vertex (lexicographic
    // (distance, coarse index) multi-source Dijkstra)
    bool any_empty = false;
    for (int64_t j = 0; j < nf; ++j) any_empty |= (U.ptr[j + 1] == U.ptr[j]);
    if (any_empty) {
        std::vector<double> kd(n, INF);
        std::vector<int32_t> kl(n, std::numeric_limits<int32_t>::max());
        using Item = std::tuple<double, int32_t, int32_t>;
        std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
        for (int64_t ci = 0; ci < nc; ++ci) {
            kd[coarse_verts[ci]] = 0.0;
            kl[coarse_verts[ci]] = (int32_t)ci;
            heap.push({0.0, (int32_t)ci, coarse_verts[ci]});
        }
        while (!heap.empty()) {
            auto [dv, ci, v] = heap.top();
            heap.pop();
            if (dv > kd[v] || (dv == kd[v] && ci > kl[v])) continue;
            for (int64_t k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
                int32_t u = g.nbr[k];
                double nd = dv + g.w[k];
                if (nd < kd[u] || (nd == kd[u] && ci < kl[u])) {
                    kd[u] = nd;
                    kl[u] = ci;
                    heap.push({nd, ci, u});
                }
            }
        }
        Csr V2;
        V2.rows = nf;
        V2.cols = nc;
        V2.ptr.assign(nf + 1, 0);
        for (int64_t j = 0; j < nf; ++j) {
            int32_t vtx = fine_is_all ? (int32_t)j : fine_verts[j];
            if (U.ptr[j + 1] == U.ptr[j]) {
                V2.idx.push_back(kl[vtx]);
                V2.val.push_back(1.0);
            } else {
                for (int64_t k = U.ptr[j]; k < U.ptr[j + 1]; ++k) {
                    V2.idx.push_back(U.idx[k]);
                    V2.val.push_back(U.val[k]);
                }
            }
            V2.ptr[j + 1] = (int64_t)V2.idx.size();
        }
        U = std::move(V2);
    }
    // row normalisation: U_ji = Utilde_ji * (1 / sum_i Utilde_ji)
    for (int64_t j = 0; j < nf; ++j) {
        double s = 0.0;
        for (int64_t k = U.ptr[j]; k < U.ptr[j + 1]; ++k) s += U.val[k];
        double inv = 1.0 / s;
        for (int64_t k = U.ptr[j]; k < U.ptr[j + 1]; ++k) U.val[k] = inv * U.val[k];
    }
    return U;
}

// S_next = U^T S U, M_next = U^T M U with M given on S's pattern, in two
// sparse products: T = S U and T_M = M U (row j of T sums s_jl U_l. over the
// entries l of S row j in order), then row i of S_next sums u_ij T_j. over the
// fine rows j of U^T row i, ascending.  The pattern is the structural product
// (no numerical dropping), so M_next lives on S_next's pattern too.  The
// device build forms the same sums in the same order.
void galerkin(const Csr& U, const Csr& S, const std::vector<double>& Mval, Csr& Sn, std::vector<double>& Mn) {
    const int64_t nf = U.rows, nc = U.cols;
    // U^T in CSR (coarse rows, fine columns ascending)
    Csr Ut;
    Ut.rows = nc;
    Ut.cols = nf;
    Ut.ptr.assign(nc + 1, 0);
    for (int64_t k = 0; k < U.nnz(); ++k) Ut.ptr[U.idx[k] + 1]++;
    for (int64_t i = 0; i < nc; ++i) Ut.ptr[i + 1] += Ut.ptr[i];
    Ut.idx.resize(U.nnz());
    Ut.val.resize(U.nnz());
    {
        std::vector<int64_t> fill(Ut.ptr.begin(), Ut.ptr.end() - 1);
        for (int64_t j = 0; j < nf; ++j)
            for (int64_t k = U.ptr[j]; k < U.ptr[j + 1]; ++k) {
                Ut.idx[fill[U.idx[k]]] = (int32_t)j;
                Ut.val[fill[U.idx[k]]++] = U.val[k];
            }
    }
    // sparse rows with a dense accumulator per thread: row r sums w_e X_(c_e).
    // over its terms e in order; columns of the result ascending
    struct Rows {
        std::vector<std::vector<int32_t>> cols;
        std::vector<std::vector<double>> a, b;
    };
    auto product = [&](int64_t rows, int64_t width, auto&& terms, Rows& R) {
        R.cols.assign(rows, {});
        R.a.assign(rows, {});
        R.b.assign(rows, {});
#pragma omp parallel
        {
            std::vector<double> accA(width, 0.0), accB(width, 0.0);
            std::vector<char> mark(width, 0);
            std::vector<int32_t> list;
#pragma omp for schedule(dynamic, 64)
            for (int64_t r = 0; r < rows; ++r) {
                list.clear();
                terms(r, [&](int32_t k, double va, double vb) {
                    if (!mark[k]) { mark[k] = 1; list.push_back(k); }
                    accA[k] += va;
                    accB[k] += vb;
                });
                std::sort(list.begin(), list.end());
                R.cols[r] = list;
                R.a[r].resize(list.size());
                R.b[r].resize(list.size());
                for (size_t t = 0; t < list.size(); ++t) {
                    const int32_t k = list[t];
                    R.a[r][t] = accA[k];
                    R.b[r][t] = accB[k];
                    accA[k] = accB[k] = 0.0;
                    mark[k] = 0;
                }
            }
        }
    };
    // T = S U, T_M = M U
    Rows T;
    product(nf, nc, [&](int64_t j, auto&& add) {
        for (int64_t b = S.ptr[j]; b < S.ptr[j + 1]; ++b) {
            const int64_t l = S.idx[b];
            for (int64_t c = U.ptr[l]; c < U.ptr[l + 1]; ++c) add(U.idx[c], S.val[b] * U.val[c], Mval[b] * U.val[c]);
        }
    }, T);
    // S_next = U^T T, M_next = U^T T_M
    Rows N;
    product(nc, nc, [&](int64_t i, auto&& add) {
        for (int64_t a = Ut.ptr[i]; a < Ut.ptr[i + 1]; ++a) {
            const int64_t j = Ut.idx[a];
            const double uij = Ut.val[a];
            for (size_t t = 0; t < T.cols[j].size(); ++t) add(T.cols[j][t], uij * T.a[j][t], uij * T.b[j][t]);
        }
    }, N);
    Sn = Csr();
    Sn.rows = Sn.cols = nc;
    Sn.ptr.assign(nc + 1, 0);
    for (int64_t i = 0; i < nc; ++i) Sn.ptr[i + 1] = Sn.ptr[i] + (int64_t)N.cols[i].size();
    Sn.idx.resize(Sn.ptr[nc]);
    Sn.val.resize(Sn.ptr[nc]);
    Mn.resize(Sn.ptr[nc]);
    for (int64_t i = 0; i < nc; ++i) {
        std::copy(N.cols[i].begin(), N.cols[i].end(), Sn.idx.begin() + Sn.ptr[i]);
        std::copy(N.a[i].begin(), N.a[i].end(), Sn.val.begin() + Sn.ptr[i]);
        std::copy(N.b[i].begin(), N.b[i].end(), Mn.begin() + Sn.ptr[i]);
    }
    // exact symmetry: average the two mirror entries
    for (int64_t i = 0; i < nc; ++i)
        for (int64_t k = Sn.ptr[i]; k < Sn.ptr[i + 1]; ++k) {
            int32_t j = Sn.idx[k];
            if (j <= i) continue;
            auto b = Sn.idx.begin() + Sn.ptr[j], e = Sn.idx.begin() + Sn.ptr[j + 1];
            auto it = std::lower_bound(b, e, (int32_t)i);
            int64_t kk = it - Sn.idx.begin();
            double s = 0.5 * (Sn.val[k] + Sn.val[kk]);
            double mm = 0.5 * (Mn[k] + Mn[kk]);
            Sn.val[k] = Sn.val[kk] = s;
            Mn[k] = Mn[kk] = mm;
        }
}

}  // namespace hsim

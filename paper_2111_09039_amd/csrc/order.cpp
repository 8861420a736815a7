// Elimination order and symbolic analysis of the sparse LDL^T factor of
// S^tau - mu M^tau (the direct solver of Algorithm 1).  The pattern of
// S^tau - mu M^tau does not depend on mu (M^tau lives on S^tau's pattern), so
// this runs once per level when the hierarchy is built.
//
// Order: geometric nested dissection on the level's sparsity graph using the
// level vertices' mesh coordinates; each split is the median plane of the
// axis that gives the smallest vertex separator.  Supernodes: every
// separator and every leaf block is one supernode whose diagonal block is
// treated as dense.  Assembly tree: the parent of a supernode is the
// supernode holding the first off-diagonal row of its column structure, and
// the structure of a supernode is the union of its own columns' rows and its
// children's structures below it (so every child's update block fits inside
// its parent's front).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <numeric>

#include "internal.h"

namespace hsim {
namespace {

constexpr int LEAF = 64;
// subsets at least this large are split in their own OpenMP task
constexpr size_t TASK_MIN = 16384;

// Nested dissection.  Every call owns a distinct vertex subset; its marks in
// `tag` carry the call's id (unique in the recursion tree), so concurrent
// calls on disjoint subsets never read each other's sides.  The elimination
// order of a subset is its first part, then its second part, then the
// separator (ascending): the same in every schedule.
struct ND {
    const Csr& G;
    const double* X;
    // per axis: (call id << 2) | side (0, 1: halves, 2: separator); -1 unmarked
    std::vector<int64_t> tag[3];

    ND(const Csr& g, const double* x, int64_t n) : G(g), X(x) {
        for (auto& t : tag) t.assign(n, -1);
    }

    // the split of W at the median plane of one axis: its separator (the
    // smaller of the two boundary layers) and the two remaining halves
    void split(const std::vector<int32_t>& W, int64_t id, int axis, std::vector<int32_t>& sep,
               std::vector<int32_t>& left, std::vector<int32_t>& right) {
        const size_t n = W.size(), half = n / 2;
        std::vector<int64_t>& tg = tag[axis];
        const int64_t mine = id << 2;
        auto side_of = [&](int32_t u) -> int { return (tg[u] >> 2) == id ? (int)(tg[u] & 3) : -1; };
        std::vector<int32_t> S(W);
        std::nth_element(S.begin(), S.begin() + half, S.end(), [&](int32_t a, int32_t b) {
            double xa = X[3 * a + axis], xb = X[3 * b + axis];
            return xa < xb || (xa == xb && a < b);
        });
        for (size_t i = 0; i < n; ++i) tg[S[i]] = mine | (i < half ? 0 : 1);
        std::vector<int32_t> bl, br;
        for (size_t i = 0; i < n; ++i) {
            int32_t v = S[i];
            const int sv = side_of(v);
            bool cross = false;
            for (int64_t k = G.ptr[v]; k < G.ptr[v + 1] && !cross; ++k) {
                const int su = side_of(G.idx[k]);
                cross = su >= 0 && su != sv;
            }
            if (cross) (sv == 0 ? bl : br).push_back(v);
        }
        sep = bl.size() <= br.size() ? std::move(bl) : std::move(br);
        for (int32_t v : sep) tg[v] = mine | 2;
        left.clear();
        right.clear();
        for (size_t i = 0; i < n; ++i) {
            const int sv = side_of(S[i]);
            if (sv == 0) left.push_back(S[i]);
            else if (sv == 1) right.push_back(S[i]);
        }
    }

    // order: the subset's vertices in elimination order; sizes: its supernodes in order
    void run(std::vector<int32_t> W, int64_t id, std::vector<int32_t>& order, std::vector<int32_t>& sizes) {
        if ((int)W.size() <= LEAF) {
            order = std::move(W);
            sizes.assign(1, (int32_t)order.size());
            if (order.empty()) sizes.clear();
            return;
        }
        const bool big = W.size() >= TASK_MIN;
        std::vector<int32_t> sep[3], lft[3], rgt[3];
        for (int axis = 0; axis < 3; ++axis) {
#pragma omp task shared(W, sep, lft, rgt) if (big)
            split(W, id, axis, sep[axis], lft[axis], rgt[axis]);
        }
#pragma omp taskwait
        // the smallest separator, the first axis on ties
        int best = 0;
        for (int axis = 1; axis < 3; ++axis)
            if (sep[axis].size() < sep[best].size()) best = axis;
        std::vector<int32_t> best_sep = std::move(sep[best]), best_l = std::move(lft[best]),
                             best_r = std::move(rgt[best]);
        for (int axis = 0; axis < 3; ++axis) {
            sep[axis].clear();
            lft[axis].clear();
            rgt[axis].clear();
        }
        // a split that separates nothing: stop here
        if (best_l.empty() || best_r.empty()) {
            order = std::move(W);
            sizes.assign(1, (int32_t)order.size());
            return;
        }
        W.clear();
        W.shrink_to_fit();
        std::vector<int32_t> ol, sl, orr, sr;
#pragma omp task shared(ol, sl, best_l) if (big)
        run(std::move(best_l), 2 * id, ol, sl);
#pragma omp task shared(orr, sr, best_r) if (big)
        run(std::move(best_r), 2 * id + 1, orr, sr);
#pragma omp taskwait
        std::sort(best_sep.begin(), best_sep.end());
        order = std::move(ol);
        order.insert(order.end(), orr.begin(), orr.end());
        order.insert(order.end(), best_sep.begin(), best_sep.end());
        sizes = std::move(sl);
        sizes.insert(sizes.end(), sr.begin(), sr.end());
        if (!best_sep.empty()) sizes.push_back((int32_t)best_sep.size());
    }
};

inline int32_t round_up(int64_t x, int64_t m) { return (int32_t)((x + m - 1) / m * m); }

}  // namespace

Symbolic analyse(const Csr& S, const double* coords, int64_t n) {
    Symbolic sy;
    std::vector<int32_t> order, sizes;
    const bool verbose = env_int("HSIM_VERBOSE", 0) != 0;
    auto t0 = std::chrono::steady_clock::now();
    auto phase_done = [&](const char* what) {
        if (!verbose) return;
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[hsim analyse] %-26s %8.1f ms (n = %lld)\n", what,
                     std::chrono::duration<double, std::milli>(now - t0).count(), (long long)n);
        t0 = now;
    };
    {
        ND nd(S, coords, n);
        std::vector<int32_t> all(n);
        std::iota(all.begin(), all.end(), 0);
#pragma omp parallel
#pragma omp single
        nd.run(std::move(all), 1, order, sizes);
    }
    phase_done("nested dissection");
    if ((int64_t)order.size() != n) fail(HSIM_E_INVALID, "ordering lost vertices");
    std::vector<std::pair<int64_t, int32_t>> snodes;   // (start, size) in elimination order
    {
        int64_t at = 0;
        for (int32_t sz : sizes) {
            snodes.push_back({at, sz});
            at += sz;
        }
    }
    sy.perm = std::move(order);
    sy.iperm.assign(n, 0);
    for (int64_t k = 0; k < n; ++k) sy.iperm[sy.perm[k]] = (int32_t)k;

    const int64_t ns_count = (int64_t)snodes.size();
    std::vector<int32_t> snode_of(n);
    for (int64_t s = 0; s < ns_count; ++s)
        for (int64_t c = snodes[s].first; c < snodes[s].first + snodes[s].second; ++c) snode_of[c] = (int32_t)s;

    // column structures, in elimination order (children before parents)
    std::vector<std::vector<int32_t>> st(ns_count);
    std::vector<std::vector<int32_t>> kids(ns_count);
    std::vector<int32_t> parent(ns_count, -1), tlev(ns_count, 0);
    std::vector<int64_t> mark(n, -1);
    for (int64_t s = 0; s < ns_count; ++s) {
        const int64_t a = snodes[s].first, e = a + snodes[s].second;
        std::vector<int32_t>& R = st[s];
        for (int64_t c = a; c < e; ++c) {
            int32_t v = sy.perm[c];
            for (int64_t k = S.ptr[v]; k < S.ptr[v + 1]; ++k) {
                int32_t r = sy.iperm[S.idx[k]];
                if (r >= e && mark[r] != s) { mark[r] = s; R.push_back(r); }
            }
        }
        for (int32_t ch : kids[s]) {
            for (int32_t r : st[ch])
                if (r >= e && mark[r] != s) { mark[r] = s; R.push_back(r); }
            tlev[s] = std::max(tlev[s], tlev[ch] + 1);
        }
        std::sort(R.begin(), R.end());
        if (!R.empty()) {
            parent[s] = snode_of[R[0]];
            kids[parent[s]].push_back((int32_t)s);
        }
    }
    phase_done("column structures");
    // renumber fronts by (tree level, elimination start)
    std::vector<int32_t> newid(ns_count), byid(ns_count);
    std::iota(byid.begin(), byid.end(), 0);
    std::stable_sort(byid.begin(), byid.end(), [&](int32_t x, int32_t y) { return tlev[x] < tlev[y]; });
    for (int64_t i = 0; i < ns_count; ++i) newid[byid[i]] = (int32_t)i;
    sy.tree_levels = ns_count ? tlev[byid.back()] + 1 : 0;
    sy.fronts.resize(ns_count);
    sy.rows_ptr.assign(ns_count + 1, 0);
    sy.tlev_ptr.assign(sy.tree_levels + 1, 0);
    for (int64_t i = 0; i < ns_count; ++i) {
        int32_t s = byid[i];
        Front& f = sy.fronts[i];
        f.start = snodes[s].first;
        f.ns = snodes[s].second;
        f.mu = (int32_t)st[s].size();
        f.ns_pad = round_up(f.ns, NB);
        f.mu_pad = round_up(f.mu, NB);
        f.Mt = (f.ns_pad + f.mu_pad) / NB;
        f.nsb = f.ns_pad / NB;
        f.parent = parent[s] < 0 ? -1 : newid[parent[s]];
        f.tlev = tlev[s];
        sy.rows_ptr[i + 1] = sy.rows_ptr[i] + f.mu;
        sy.tlev_ptr[f.tlev + 1]++;
    }
    for (int t = 0; t < sy.tree_levels; ++t) sy.tlev_ptr[t + 1] += sy.tlev_ptr[t];
    sy.rows.resize(sy.rows_ptr[ns_count]);
    for (int64_t i = 0; i < ns_count; ++i)
        std::copy(st[byid[i]].begin(), st[byid[i]].end(), sy.rows.begin() + sy.rows_ptr[i]);
    st.clear();

    phase_done("renumbering");
    // offsets, child slots, flops
    std::vector<std::vector<int32_t>> children(ns_count);
    for (int64_t i = 0; i < ns_count; ++i)
        if (sy.fronts[i].parent >= 0) children[sy.fronts[i].parent].push_back((int32_t)i);
    int64_t tb = 0, lb = 0, db = 0, ub = 0, gb = 0;
    for (int64_t i = 0; i < ns_count; ++i) {
        Front& f = sy.fronts[i];
        f.tile_base = tb;
        tb += (int64_t)f.Mt * (f.Mt + 1) / 2 * NB * NB;
        f.linv_base = lb;
        lb += (int64_t)f.nsb * NB * NB;
        f.d_base = db;
        db += f.ns_pad;
        f.ubuf_row = ub;
        ub += f.mu;
        f.gather_base = gb;
        gb += f.ns + f.mu;
        for (size_t c = 0; c < children[i].size(); ++c) sy.fronts[children[i][c]].child_slot = (int32_t)c;
        sy.max_children = std::max<int32_t>(sy.max_children, (int32_t)children[i].size());
        const double m = f.ns + f.mu;
        sy.factor_nnz += (int64_t)f.ns * (f.ns + 1) / 2 + (int64_t)f.ns * f.mu;
        for (int c = 0; c < f.ns; ++c) {
            const double r = m - c - 1;
            sy.flops += r * r + 2 * r;      // rank-1 update of the lower trailing part + column scaling
        }
    }
    sy.tile_doubles = tb;
    sy.linv_doubles = lb;
    sy.d_doubles = db;
    sy.ubuf_rows = ub;

    phase_done("offsets and flops");
    // relative indices of struct rows in the parent's local index space
    sy.rel.resize(sy.rows.size());
    for (int64_t i = 0; i < ns_count; ++i) {
        const Front& f = sy.fronts[i];
        if (f.parent < 0) {
            if (f.mu) fail(HSIM_E_INVALID, "symbolic analysis: root front with structure");
            continue;
        }
        const Front& P = sy.fronts[f.parent];
        const int32_t* pr = sy.rows.data() + sy.rows_ptr[f.parent];
        for (int64_t k = sy.rows_ptr[i]; k < sy.rows_ptr[i + 1]; ++k) {
            int32_t r = sy.rows[k];
            if (r < P.start) fail(HSIM_E_INVALID, "symbolic analysis: structure below the parent");
            if (r < P.start + P.ns) {
                sy.rel[k] = (int32_t)(r - P.start);
            } else {
                const int32_t* it = std::lower_bound(pr, pr + P.mu, r);
                if (it == pr + P.mu || *it != r) fail(HSIM_E_INVALID, "symbolic analysis: child row missing in parent");
                sy.rel[k] = P.ns_pad + (int32_t)(it - pr);
            }
        }
    }
    phase_done("relative indices");
    // gather lists of the solve: compact local row (pivot r -> r, struct k -> ns + k)
    {
        // counted, then filled in front order (children in front order, which
        // is slot order within a parent)
        auto list_of = [&](int64_t i, int64_t k) {
            const Front& P = sy.fronts[sy.fronts[i].parent];
            const int32_t lr = sy.rel[k];
            return P.gather_base + (lr < P.ns_pad ? lr : P.ns + (lr - P.ns_pad));
        };
        sy.gather_ptr.assign(gb + 1, 0);
        for (int64_t i = 0; i < ns_count; ++i)
            if (sy.fronts[i].parent >= 0)
                for (int64_t k = sy.rows_ptr[i]; k < sy.rows_ptr[i + 1]; ++k) ++sy.gather_ptr[list_of(i, k) + 1];
        for (int64_t r = 0; r < gb; ++r) sy.gather_ptr[r + 1] += sy.gather_ptr[r];
        sy.gather_idx.assign(sy.gather_ptr[gb], 0);
        std::vector<int64_t> fill(sy.gather_ptr.begin(), sy.gather_ptr.end() - 1);
        for (int64_t i = 0; i < ns_count; ++i) {
            const Front& f = sy.fronts[i];
            if (f.parent < 0) continue;
            for (int64_t k = sy.rows_ptr[i]; k < sy.rows_ptr[i + 1]; ++k)
                sy.gather_idx[fill[list_of(i, k)]++] = f.ubuf_row + (k - sy.rows_ptr[i]);
        }
    }
    phase_done("gather lists");
    // assembly map of A = S - mu M (lower triangle) into the front tiles
    // (fronts in order, each front's entries counted, then written into its own
    // range by the threads; the same map as one pass in front order)
    sy.asm_tlev_ptr.assign(sy.tree_levels + 1, 0);
    {
        std::vector<int64_t> aptr(ns_count + 1, 0);
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < ns_count; ++i) {
            const Front& f = sy.fronts[i];
            int64_t cnt = f.ns_pad - f.ns;   // dummy pivots
            for (int32_t lc = 0; lc < f.ns; ++lc) {
                const int64_t c = f.start + lc;
                const int32_t v = sy.perm[c];
                for (int64_t k = S.ptr[v]; k < S.ptr[v + 1]; ++k) cnt += sy.iperm[S.idx[k]] >= c;
            }
            aptr[i + 1] = cnt;
        }
        for (int64_t i = 0; i < ns_count; ++i) aptr[i + 1] += aptr[i];
        sy.asm_dst.assign(aptr[ns_count], 0);
        sy.asm_src.assign(aptr[ns_count], 0);
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < ns_count; ++i) {
            const Front& f = sy.fronts[i];
            const int32_t* fr = sy.rows.data() + sy.rows_ptr[i];
            int64_t o = aptr[i];
            for (int32_t lc = 0; lc < f.ns_pad; ++lc) {
                if (lc >= f.ns) {   // dummy pivot: identity
                    sy.asm_dst[o] = f.tile_base + tri_tile(f.Mt, lc / NB, lc / NB) * NB * NB + (lc % NB) * NB + lc % NB;
                    sy.asm_src[o++] = -1;
                    continue;
                }
                const int64_t c = f.start + lc;
                const int32_t v = sy.perm[c];
                for (int64_t k = S.ptr[v]; k < S.ptr[v + 1]; ++k) {
                    const int64_t r = sy.iperm[S.idx[k]];
                    if (r < c) continue;
                    int32_t lr;
                    if (r < f.start + f.ns) {
                        lr = (int32_t)(r - f.start);
                    } else {
                        const int32_t* it = std::lower_bound(fr, fr + f.mu, (int32_t)r);
                        lr = f.ns_pad + (int32_t)(it - fr);
                    }
                    sy.asm_dst[o] = f.tile_base + tri_tile(f.Mt, lr / NB, lc / NB) * NB * NB + (lc % NB) * NB + lr % NB;
                    sy.asm_src[o++] = k;
                }
            }
        }
        for (int64_t i = 0; i < ns_count; ++i)
            sy.asm_tlev_ptr[sy.fronts[i].tlev + 1] = std::max(sy.asm_tlev_ptr[sy.fronts[i].tlev + 1], aptr[i + 1]);
    }
    for (int t = 0; t < sy.tree_levels; ++t)
        sy.asm_tlev_ptr[t + 1] = std::max(sy.asm_tlev_ptr[t + 1], sy.asm_tlev_ptr[t]);

    phase_done("assembly map");
    // factorisation work lists
    sy.step_ptr.assign(sy.tree_levels + 1, 0);
    sy.diag_ptr.push_back(0);
    sy.panel_ptr.push_back(0);
    sy.upd_ptr.push_back(0);
    int32_t nsteps = 0;
    for (int t = 0; t < sy.tree_levels; ++t) {
        int32_t kmax = 0;
        for (int32_t i = sy.tlev_ptr[t]; i < sy.tlev_ptr[t + 1]; ++i) kmax = std::max(kmax, sy.fronts[i].nsb);
        for (int32_t k = 0; k < kmax; ++k) {
            for (int32_t i = sy.tlev_ptr[t]; i < sy.tlev_ptr[t + 1]; ++i) {
                const Front& f = sy.fronts[i];
                if (f.nsb <= k) continue;
                sy.diag.push_back(i);
                for (int32_t I = k + 1; I < f.Mt; ++I) {
                    sy.panel.push_back(i);
                    sy.panel.push_back(I);
                }
                for (int32_t J = k + 1; J < f.Mt; ++J)
                    for (int32_t I = J; I < f.Mt; ++I) {
                        sy.upd.push_back(i);
                        sy.upd.push_back(I);
                        sy.upd.push_back(J);
                    }
            }
            sy.diag_ptr.push_back((int64_t)sy.diag.size());
            sy.panel_ptr.push_back((int64_t)sy.panel.size() / 2);
            sy.upd_ptr.push_back((int64_t)sy.upd.size() / 3);
            ++nsteps;
        }
        sy.step_ptr[t + 1] = nsteps;
    }
    phase_done("work lists");
    // extend-add passes: (tree level of the parent, child slot)
    const int32_t mc = std::max<int32_t>(1, sy.max_children);
    sy.ea_ptr.assign((int64_t)sy.tree_levels * mc + 1, 0);
    {
        std::vector<std::vector<int32_t>> bins((int64_t)sy.tree_levels * mc);
        for (int64_t i = 0; i < ns_count; ++i) {
            const Front& f = sy.fronts[i];
            if (f.parent < 0 || f.mu == 0) continue;
            bins[(int64_t)sy.fronts[f.parent].tlev * mc + f.child_slot].push_back((int32_t)i);
        }
        for (size_t b = 0; b < bins.size(); ++b) {
            sy.ea_ptr[b + 1] = sy.ea_ptr[b] + (int64_t)bins[b].size();
            sy.ea.insert(sy.ea.end(), bins[b].begin(), bins[b].end());
        }
    }
    check_symbolic(sy, n, S.nnz());
    phase_done("extend-add passes");
    return sy;
}

// Bounds of every index the device kernels will follow (tile offsets, work
// items, relative indices, gather lists); any violation is a bug here.
void check_symbolic(const Symbolic& sy, int64_t n, int64_t nnz) {
    const int64_t nf = (int64_t)sy.fronts.size();
    int64_t cols = 0;
    for (int64_t i = 0; i < nf; ++i) {
        const Front& f = sy.fronts[i];
        cols += f.ns;
        if (f.ns < 1 || f.start < 0 || f.start + f.ns > n) fail(HSIM_E_INVALID, "symbolic: front %lld columns", (long long)i);
        if (f.tile_base + (int64_t)f.Mt * (f.Mt + 1) / 2 * NB * NB > sy.tile_doubles) fail(HSIM_E_INVALID, "symbolic: tiles");
        if (f.linv_base + (int64_t)f.nsb * NB * NB > sy.linv_doubles) fail(HSIM_E_INVALID, "symbolic: linv");
        if (f.d_base + f.ns_pad > sy.d_doubles) fail(HSIM_E_INVALID, "symbolic: D");
        if (f.ubuf_row + f.mu > sy.ubuf_rows) fail(HSIM_E_INVALID, "symbolic: update rows");
        if (f.parent >= 0 && (f.parent <= i || f.parent >= nf)) fail(HSIM_E_INVALID, "symbolic: parent order");
        if (f.parent >= 0 && sy.fronts[f.parent].tlev <= f.tlev) fail(HSIM_E_INVALID, "symbolic: tree levels");
        const Front* P = f.parent >= 0 ? &sy.fronts[f.parent] : nullptr;
        int32_t prev_r = -1, prev_rel = -1;
        for (int64_t k = sy.rows_ptr[i]; k < sy.rows_ptr[i + 1]; ++k) {
            const int32_t r = sy.rows[k];
            if (r < f.start + f.ns || r >= n || r <= prev_r) fail(HSIM_E_INVALID, "symbolic: struct rows");
            prev_r = r;
            if (!P) fail(HSIM_E_INVALID, "symbolic: root with struct rows");
            const int32_t rl = sy.rel[k];
            if (rl <= prev_rel || rl >= P->ns_pad + P->mu || (rl >= P->ns && rl < P->ns_pad))
                fail(HSIM_E_INVALID, "symbolic: relative index");
            prev_rel = rl;
        }
    }
    if (cols != n) fail(HSIM_E_INVALID, "symbolic: fronts do not partition the columns");
    for (size_t e = 0; e < sy.asm_dst.size(); ++e)
        if (sy.asm_dst[e] < 0 || sy.asm_dst[e] >= sy.tile_doubles || sy.asm_src[e] >= nnz)
            fail(HSIM_E_INVALID, "symbolic: assembly map");
    for (int64_t g : sy.gather_idx)
        if (g < 0 || g >= sy.ubuf_rows) fail(HSIM_E_INVALID, "symbolic: gather list");
    if ((int64_t)sy.gather_ptr.size() < 1 || sy.gather_ptr.back() != (int64_t)sy.gather_idx.size())
        fail(HSIM_E_INVALID, "symbolic: gather pointers");
    for (int t = 0; t < sy.tree_levels; ++t)
        for (int32_t st = sy.step_ptr[t]; st < sy.step_ptr[t + 1]; ++st) {
            const int32_t k = st - sy.step_ptr[t];
            for (int64_t a = sy.diag_ptr[st]; a < sy.diag_ptr[st + 1]; ++a) {
                const Front& f = sy.fronts[sy.diag[a]];
                if (f.tlev != t || k >= f.nsb) fail(HSIM_E_INVALID, "symbolic: diag items");
            }
            for (int64_t a = sy.panel_ptr[st]; a < sy.panel_ptr[st + 1]; ++a) {
                const Front& f = sy.fronts[sy.panel[2 * a]];
                const int32_t I = sy.panel[2 * a + 1];
                if (f.tlev != t || k >= f.nsb || I <= k || I >= f.Mt) fail(HSIM_E_INVALID, "symbolic: panel items");
            }
            for (int64_t a = sy.upd_ptr[st]; a < sy.upd_ptr[st + 1]; ++a) {
                const Front& f = sy.fronts[sy.upd[3 * a]];
                const int32_t I = sy.upd[3 * a + 1], J = sy.upd[3 * a + 2];
                if (f.tlev != t || k >= f.nsb || J <= k || I < J || I >= f.Mt) fail(HSIM_E_INVALID, "symbolic: update items");
            }
        }
    for (int32_t c : sy.ea)
        if (c < 0 || c >= nf || sy.fronts[c].parent < 0) fail(HSIM_E_INVALID, "symbolic: extend-add items");
}

}  // namespace hsim

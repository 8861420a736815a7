// Mesh checks, edge graph and P1 finite element assembly (Section 3.1,
// eq. massStiffMatrices): cotangent stiffness S and lumped mass M.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace hsim {

std::vector<char> boundary_vertex_flags(const Mesh& m) {
    std::vector<std::pair<int32_t, int32_t>> e;
    e.reserve(3 * (size_t)m.nf);
    for (int64_t t = 0; t < m.nf; ++t)
        for (int k = 0; k < 3; ++k) {
            const int32_t a = m.F[3 * t + k], b = m.F[3 * t + (k + 1) % 3];
            e.push_back({std::min(a, b), std::max(a, b)});
        }
    std::sort(e.begin(), e.end());
    std::vector<char> on(m.nv, 0);
    for (size_t i = 0; i < e.size();) {
        size_t j = i;
        while (j < e.size() && e[j] == e[i]) ++j;
        if (j - i == 1) on[e[i].first] = on[e[i].second] = 1;
        i = j;
    }
    return on;
}

void validate_mesh(const Mesh& m) {
    if (m.nv < 3 || m.nf < 1) fail(HSIM_E_MESH, "mesh needs >= 3 vertices and >= 1 triangle");
    for (int64_t i = 0; i < 3 * m.nv; ++i)
        if (!std::isfinite(m.V[i])) fail(HSIM_E_MESH, "vertex %lld has a non-finite coordinate", (long long)(i / 3));
    std::vector<char> used(m.nv, 0);
    for (int64_t t = 0; t < m.nf; ++t) {
        const int32_t* f = &m.F[3 * t];
        for (int k = 0; k < 3; ++k) {
            if (f[k] < 0 || f[k] >= m.nv) fail(HSIM_E_MESH, "triangle %lld references vertex %d out of range", (long long)t, f[k]);
            used[f[k]] = 1;
        }
        if (f[0] == f[1] || f[1] == f[2] || f[2] == f[0]) fail(HSIM_E_MESH, "triangle %lld repeats a vertex", (long long)t);
    }
    for (int64_t i = 0; i < m.nv; ++i)
        if (!used[i]) fail(HSIM_E_MESH, "vertex %lld belongs to no triangle", (long long)i);
    // degenerate triangles: area tiny relative to the squared longest edge
    for (int64_t t = 0; t < m.nf; ++t) {
        const double* a = &m.V[3 * m.F[3 * t]];
        const double* b = &m.V[3 * m.F[3 * t + 1]];
        const double* c = &m.V[3 * m.F[3 * t + 2]];
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double e3[3] = {c[0] - b[0], c[1] - b[1], c[2] - b[2]};
        double cx = e1[1] * e2[2] - e1[2] * e2[1];
        double cy = e1[2] * e2[0] - e1[0] * e2[2];
        double cz = e1[0] * e2[1] - e1[1] * e2[0];
        double a2 = cx * cx + cy * cy + cz * cz;
        double l2 = std::max({e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2],
                              e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2],
                              e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2]});
        if (!(a2 > 1e-24 * l2 * l2)) fail(HSIM_E_MESH, "triangle %lld is degenerate", (long long)t);
    }
    // edge-manifold: every undirected edge in at most two triangles
    std::vector<std::pair<int64_t, int64_t>> e;
    e.reserve(3 * m.nf);
    for (int64_t t = 0; t < m.nf; ++t)
        for (int k = 0; k < 3; ++k) {
            int64_t u = m.F[3 * t + k], v = m.F[3 * t + (k + 1) % 3];
            e.emplace_back(std::min(u, v), std::max(u, v));
        }
    std::sort(e.begin(), e.end());
    for (size_t i = 0; i < e.size();) {
        size_t j = i;
        while (j < e.size() && e[j] == e[i]) ++j;
        if (j - i > 2) fail(HSIM_E_MESH, "edge (%lld,%lld) is shared by %zu triangles", (long long)e[i].first, (long long)e[i].second, j - i);
        i = j;
    }
}

// Edge graph with Euclidean edge lengths (squared differences summed x, y, z
// in order, then the square root).
Graph edge_graph(const Mesh& m) {
    std::vector<std::pair<int32_t, int32_t>> e;
    e.reserve(6 * m.nf);
    for (int64_t t = 0; t < m.nf; ++t)
        for (int k = 0; k < 3; ++k) {
            int32_t u = m.F[3 * t + k], v = m.F[3 * t + (k + 1) % 3];
            e.emplace_back(u, v);
            e.emplace_back(v, u);
        }
    std::sort(e.begin(), e.end());
    e.erase(std::unique(e.begin(), e.end()), e.end());
    Graph g;
    g.ptr.assign(m.nv + 1, 0);
    for (auto& x : e) g.ptr[x.first + 1]++;
    for (int64_t i = 0; i < m.nv; ++i) g.ptr[i + 1] += g.ptr[i];
    g.nbr.resize(e.size());
    g.w.resize(e.size());
    for (size_t k = 0; k < e.size(); ++k) {
        int32_t i = e[k].first, j = e[k].second;
        g.nbr[k] = j;
        double dx = m.V[3 * i] - m.V[3 * j];
        double dy = m.V[3 * i + 1] - m.V[3 * j + 1];
        double dz = m.V[3 * i + 2] - m.V[3 * j + 2];
        g.w[k] = std::sqrt(dx * dx + dy * dy + dz * dz);
    }
    check_connected(g, m.nv);
    return g;
}

void check_connected(const Graph& g, int64_t nv) {
    std::vector<char> seen(nv, 0);
    std::vector<int32_t> stack{0};
    seen[0] = 1;
    int64_t count = 1;
    while (!stack.empty()) {
        int32_t v = stack.back();
        stack.pop_back();
        for (int64_t k = g.ptr[v]; k < g.ptr[v + 1]; ++k)
            if (!seen[g.nbr[k]]) {
                seen[g.nbr[k]] = 1;
                ++count;
                stack.push_back(g.nbr[k]);
            }
    }
    if (count != nv) fail(HSIM_E_MESH, "mesh is not connected (%lld of %lld vertices reachable)", (long long)count, (long long)nv);
}

static inline double tri_area(const Mesh& m, int64_t t) {
    const double* a = &m.V[3 * m.F[3 * t]];
    const double* b = &m.V[3 * m.F[3 * t + 1]];
    const double* c = &m.V[3 * m.F[3 * t + 2]];
    double e1x = b[0] - a[0], e1y = b[1] - a[1], e1z = b[2] - a[2];
    double e2x = c[0] - a[0], e2y = c[1] - a[1], e2z = c[2] - a[2];
    double cx = e1y * e2z - e1z * e2y;
    double cy = e1z * e2x - e1x * e2z;
    double cz = e1x * e2y - e1y * e2x;
    return 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
}

// total area, summed in triangle order
double surface_area(const Mesh& m) {
    double A = 0.0;
    for (int64_t t = 0; t < m.nf; ++t) A += tri_area(m, t);
    return A;
}

// cot of the angle at vertex p between the edges to q and r
static inline double cot_at(const double* p, const double* q, const double* r) {
    double ux = q[0] - p[0], uy = q[1] - p[1], uz = q[2] - p[2];
    double wx = r[0] - p[0], wy = r[1] - p[1], wz = r[2] - p[2];
    double dot = ux * wx + uy * wy + uz * wz;
    double cx = uy * wz - uz * wy, cy = uz * wx - ux * wz, cz = ux * wy - uy * wx;
    return dot / std::sqrt(cx * cx + cy * cy + cz * cz);
}

// S_ij = -1/2 (cot alpha_ij + cot beta_ij) over the two triangles sharing the
// edge (i, j); S_ii = -sum_j S_ij.  CSR with sorted column indices.
Csr cotan_stiffness(const Mesh& m) {
    struct Trip { int32_t r, c; double v; };
    std::vector<Trip> tr;
    tr.reserve(12 * m.nf);
    for (int64_t t = 0; t < m.nf; ++t) {
        const int32_t* f = &m.F[3 * t];
        for (int k = 0; k < 3; ++k) {
            int32_t pk = f[k], i = f[(k + 1) % 3], j = f[(k + 2) % 3];
            double w = -0.5 * cot_at(&m.V[3 * pk], &m.V[3 * i], &m.V[3 * j]);
            tr.push_back({i, j, w});
            tr.push_back({j, i, w});
            tr.push_back({i, i, -w});
            tr.push_back({j, j, -w});
        }
    }
    std::stable_sort(tr.begin(), tr.end(), [](const Trip& a, const Trip& b) {
        return a.r < b.r || (a.r == b.r && a.c < b.c);
    });
    Csr S;
    S.rows = S.cols = m.nv;
    S.ptr.assign(m.nv + 1, 0);
    for (size_t k = 0; k < tr.size();) {
        size_t l = k;
        double s = 0.0;
        while (l < tr.size() && tr[l].r == tr[k].r && tr[l].c == tr[k].c) s += tr[l++].v;
        S.idx.push_back(tr[k].c);
        S.val.push_back(s);
        S.ptr[tr[k].r + 1]++;
        k = l;
    }
    for (int64_t i = 0; i < m.nv; ++i) S.ptr[i + 1] += S.ptr[i];
    return S;
}

// lumping 0: m_i = sum_{t containing i} area(t) / 3 (row sums of the
// consistent P1 mass matrix); lumping 1: circumcentric dual area
// sum_t (|e_ik|^2 cot theta_j + |e_ij|^2 cot theta_k) / 8.  Optional density.
std::vector<double> lumped_mass(const Mesh& m, int lumping, const double* density) {
    std::vector<double> mass(m.nv, 0.0);
    for (int64_t t = 0; t < m.nf; ++t) {
        const int32_t* f = &m.F[3 * t];
        if (lumping == 0) {
            double a3 = tri_area(m, t) / 3.0;
            for (int k = 0; k < 3; ++k) mass[f[k]] += a3;
        } else {
            for (int k = 0; k < 3; ++k) {
                int32_t pk = f[k], i = f[(k + 1) % 3], j = f[(k + 2) % 3];
                const double *P = &m.V[3 * pk], *I = &m.V[3 * i], *J = &m.V[3 * j];
                double eki = (I[0] - P[0]) * (I[0] - P[0]) + (I[1] - P[1]) * (I[1] - P[1]) + (I[2] - P[2]) * (I[2] - P[2]);
                double ekj = (J[0] - P[0]) * (J[0] - P[0]) + (J[1] - P[1]) * (J[1] - P[1]) + (J[2] - P[2]) * (J[2] - P[2]);
                mass[pk] += (eki * cot_at(J, P, I) + ekj * cot_at(I, J, P)) / 8.0;
            }
        }
    }
    if (density)
        for (int64_t i = 0; i < m.nv; ++i) mass[i] *= density[i];
    for (int64_t i = 0; i < m.nv; ++i)
        if (!(mass[i] > 0)) fail(HSIM_E_MESH, "lumped mass of vertex %lld is not positive", (long long)i);
    return mass;
}


// Index structures of the device assembly (cotangent stiffness on the
// pattern of the edge graph plus the diagonal, barycentric lumped mass): per
// CSR entry the <= 2 triangle corners opposite its edge, per vertex the
// corners whose weights its diagonal sums and its triangles, every list in
// triangle order and, within a triangle, corner order -- the order in which
// the host assembly sums the same terms.
AssemblyMaps assembly_maps(const Mesh& m, const Graph& g) {
    AssemblyMaps a;
    const int64_t n = m.nv;
    a.S.rows = a.S.cols = n;
    a.S.ptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) a.S.ptr[i + 1] = a.S.ptr[i] + (g.ptr[i + 1] - g.ptr[i]) + 1;
    a.S.idx.resize(a.S.ptr[n]);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t o = a.S.ptr[i];
        bool put = false;
        for (int64_t e = g.ptr[i]; e < g.ptr[i + 1]; ++e) {
            if (!put && g.nbr[e] > i) {
                a.S.idx[o++] = (int32_t)i;
                put = true;
            }
            a.S.idx[o++] = g.nbr[e];
        }
        if (!put) a.S.idx[o++] = (int32_t)i;
    }
    a.corner.assign(2 * a.S.ptr[n], -1);
    auto find = [&](int32_t i, int32_t j) -> int64_t {
        const int32_t* b = a.S.idx.data() + a.S.ptr[i];
        const int32_t* e = a.S.idx.data() + a.S.ptr[i + 1];
        const int32_t* q = std::lower_bound(b, e, j);
        if (q == e || *q != j) fail(HSIM_E_MESH, "edge (%d, %d) missing from the edge graph", i, j);
        return a.S.ptr[i] + (q - b);
    };
    for (int64_t t = 0; t < m.nf; ++t) {
        const int32_t* f = &m.F[3 * t];
        for (int k = 0; k < 3; ++k) {
            const int32_t i = f[(k + 1) % 3], j = f[(k + 2) % 3];
            for (int64_t e : {find(i, j), find(j, i)}) {
                int64_t* c = &a.corner[2 * e];
                if (c[0] < 0) c[0] = 3 * t + k;
                else if (c[1] < 0) c[1] = 3 * t + k;
                else fail(HSIM_E_MESH, "edge (%d, %d) belongs to more than two triangles", i, j);
            }
        }
    }
    // vertex -> triangles (ascending), and the two corners of each that face an edge at the vertex
    a.vptr.assign(n + 1, 0);
    for (int64_t t = 0; t < m.nf; ++t)
        for (int k = 0; k < 3; ++k) a.vptr[m.F[3 * t + k] + 1]++;
    for (int64_t i = 0; i < n; ++i) a.vptr[i + 1] += a.vptr[i];
    a.vtri.resize(a.vptr[n]);
    a.dcorner.resize(2 * a.vptr[n]);
    std::vector<int64_t> fill(a.vptr.begin(), a.vptr.end() - 1);
    for (int64_t t = 0; t < m.nf; ++t)
        for (int k = 0; k < 3; ++k) {
            const int64_t o = fill[m.F[3 * t + k]]++;
            a.vtri[o] = (int32_t)t;
            a.dcorner[2 * o] = 3 * t + (k == 0 ? 1 : 0);
            a.dcorner[2 * o + 1] = 3 * t + (k == 2 ? 1 : 2);
        }
    a.dptr.resize(n + 1);
    for (int64_t i = 0; i <= n; ++i) a.dptr[i] = 2 * a.vptr[i];
    return a;
}

}  // namespace hsim

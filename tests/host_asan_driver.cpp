// Host-only driver of the library's hierarchy build (mesh checks, cotangent
// and lumped-mass assembly, farthest point sampling, prolongation, Galerkin
// operators, nested-dissection ordering and supernodal symbolic analysis),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py.  It links the library's host sources
// directly (no HIP runtime) and supplies the three helpers that the full
// library defines next to its device code.
//
// Input (binary, little endian): int64 nv, int64 nf, int32 p, int32 T,
// int64 n_coarsest, int32 boundary, double V[3 nv], int32 F[3 nf].
// Output (text): one "key value..." line per checked quantity.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../paper_2111_09039_amd/csrc/internal.h"

namespace hsim {
static std::string g_err;
void set_last_error(const std::string& msg) { g_err = msg; }
[[noreturn]] void fail(hsim_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error{code, buf};
}
int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    char* end = nullptr;
    long x = std::strtol(v, &end, 10);
    return (end && *end == 0) ? (int)x : dflt;
}
}  // namespace hsim

using namespace hsim;

template <class T> static void rd(FILE* f, T* p, size_t n) {
    if (std::fread(p, sizeof(T), n, f) != n) {
        std::fprintf(stderr, "short read\n");
        std::exit(2);
    }
}

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t nv, nf, nc;
    int32_t p, T, boundary;
    rd(f, &nv, 1);
    rd(f, &nf, 1);
    rd(f, &p, 1);
    rd(f, &T, 1);
    rd(f, &nc, 1);
    rd(f, &boundary, 1);
    Mesh m;
    m.nv = nv;
    m.nf = nf;
    m.V.resize(3 * nv);
    m.F.resize(3 * nf);
    rd(f, m.V.data(), m.V.size());
    rd(f, m.F.data(), m.F.size());
    std::fclose(f);
    try {
        validate_mesh(m);
        Graph g = edge_graph(m);
        const std::vector<char> onb = boundary_vertex_flags(m);
        int64_t nb = 0;
        for (char c : onb) nb += c;
        std::printf("boundary_vertices %lld\n", (long long)nb);
        Csr S = cotan_stiffness(m);
        std::vector<double> md = lumped_mass(m, 0, nullptr);
        double area = surface_area(m), msum = 0, rowsum = 0;
        for (double x : md) msum += x;
        for (int64_t i = 0; i < S.rows; ++i) {
            double r = 0;
            for (int64_t e = S.ptr[i]; e < S.ptr[i + 1]; ++e) r += S.val[e];
            rowsum = std::max(rowsum, std::fabs(r));
        }
        std::printf("S_nnz %lld\nS_max_abs_rowsum %.3e\narea %.17g\nmass_sum %.17g\n", (long long)S.nnz(), rowsum,
                    area, msum);
        {
            // the device assembly's index structures, evaluated on the host with the
            // device kernels' formulas, must reproduce the host assembly bit for bit
            AssemblyMaps a = assembly_maps(m, g);
            std::vector<double> w(3 * nf), a3(nf);
            for (int64_t t = 0; t < nf; ++t) {
                const int32_t* f = &m.F[3 * t];
                for (int k = 0; k < 3; ++k) {
                    const double* P = &m.V[3 * (int64_t)f[k]];
                    const double* Q = &m.V[3 * (int64_t)f[(k + 1) % 3]];
                    const double* R = &m.V[3 * (int64_t)f[(k + 2) % 3]];
                    const double ux = Q[0] - P[0], uy = Q[1] - P[1], uz = Q[2] - P[2];
                    const double vx = R[0] - P[0], vy = R[1] - P[1], vz = R[2] - P[2];
                    const double dot = ux * vx + uy * vy + uz * vz;
                    const double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
                    w[3 * t + k] = -0.5 * (dot / std::sqrt(cx * cx + cy * cy + cz * cz));
                }
                const double* A = &m.V[3 * (int64_t)f[0]];
                const double* B = &m.V[3 * (int64_t)f[1]];
                const double* C = &m.V[3 * (int64_t)f[2]];
                const double e1x = B[0] - A[0], e1y = B[1] - A[1], e1z = B[2] - A[2];
                const double e2x = C[0] - A[0], e2y = C[1] - A[1], e2z = C[2] - A[2];
                const double cx = e1y * e2z - e1z * e2y, cy = e1z * e2x - e1x * e2z, cz = e1x * e2y - e1y * e2x;
                a3[t] = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz) / 3.0;
            }
            bool same = a.S.ptr == S.ptr && a.S.idx == S.idx;
            for (int64_t i = 0; same && i < nv; ++i)
                for (int64_t e = a.S.ptr[i]; e < a.S.ptr[i + 1]; ++e) {
                    double v = 0.0;
                    if (a.S.idx[e] == i) {
                        for (int64_t c = a.dptr[i]; c < a.dptr[i + 1]; ++c) v += -w[a.dcorner[c]];
                    } else {
                        if (a.corner[2 * e] >= 0) v += w[a.corner[2 * e]];
                        if (a.corner[2 * e + 1] >= 0) v += w[a.corner[2 * e + 1]];
                    }
                    same &= v == S.val[e];
                }
            for (int64_t i = 0; same && i < nv; ++i) {
                double v = 0.0;
                for (int64_t k = a.vptr[i]; k < a.vptr[i + 1]; ++k) v += a3[a.vtri[k]];
                same &= v == md[i];
            }
            std::printf("assembly_maps_match %d\n", (int)same);
        }
        std::vector<int64_t> sizes = level_sizes(nv, T, nc, 0);
        std::printf("levels");
        for (int64_t s : sizes) std::printf(" %lld", (long long)s);
        std::printf("\n");
        std::vector<int32_t> order = farthest_point_sampling(g, nv, sizes[1], 0);
        std::printf("fps_first %d %d %d\n", order[0], order[1], order[2]);
        std::vector<double> Mval(S.nnz(), 0.0);
        for (int64_t i = 0; i < S.rows; ++i)
            for (int64_t e = S.ptr[i]; e < S.ptr[i + 1]; ++e)
                if (S.idx[e] == i) Mval[e] = md[i];
        Csr Sl = S;
        std::vector<int32_t> fine(nv);
        for (int64_t i = 0; i < nv; ++i) fine[i] = (int32_t)i;
        for (int t = 0; t + 1 < T; ++t) {
            std::vector<int32_t> coarse(order.begin(), order.begin() + sizes[t + 1]);
            double rho = 0;
            Csr U = prolongation(g, nv, fine, t == 0, coarse, 7.0, area, &rho);
            double worst = 0;
            for (int64_t i = 0; i < U.rows; ++i) {
                double r = 0;
                for (int64_t e = U.ptr[i]; e < U.ptr[i + 1]; ++e) r += U.val[e];
                worst = std::max(worst, std::fabs(r - 1.0));
            }
            std::vector<double> coords(3 * Sl.rows);
            for (int64_t i = 0; i < Sl.rows; ++i)
                for (int c = 0; c < 3; ++c) coords[3 * i + c] = m.V[3 * (int64_t)fine[i] + c];
            Symbolic sy = analyse(Sl, coords.data(), Sl.rows);
            check_symbolic(sy, Sl.rows, Sl.nnz());
            std::printf("level %d U_nnz %lld partition_of_unity %.3e rho %.6g fronts %zu tree_levels %d factor_nnz %lld\n",
                        t, (long long)U.nnz(), worst, rho, sy.fronts.size(), sy.tree_levels,
                        (long long)sy.factor_nnz);
            Csr Sn;
            std::vector<double> Mn;
            galerkin(U, Sl, Mval, Sn, Mn);
            double msum_n = 0;
            for (double x : Mn) msum_n += x;
            std::printf("galerkin %d nnz %lld mass_total %.17g\n", t + 1, (long long)Sn.nnz(), msum_n);
            Sl = std::move(Sn);
            Mval = std::move(Mn);
            fine = coarse;
        }
    } catch (const Error& e) {
        std::printf("error %d %s\n", (int)e.code, e.msg.c_str());
        return 3;
    }
    std::printf("ok\n");
    return 0;
}

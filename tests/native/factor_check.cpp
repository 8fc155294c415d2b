// Host check of the supernodal factor: emulate the forward sweep
// [y_s; delta_s] = W_s btilde_s and the backward sweep x_s = W_s^T [y_s; -x_off]
// on the CPU and compare A^-1 b with a dense Gaussian-elimination solve.
// Usage: factor_check layers nx ny leaf_max seed
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_1511_04519_amd/csrc/factor.hpp"

using namespace matex;

int main(int argc, char** argv)
{
    int layers = argc > 1 ? atoi(argv[1]) : 2, nx = argc > 2 ? atoi(argv[2]) : 12,
        ny = argc > 3 ? atoi(argv[3]) : 9, leaf = argc > 4 ? atoi(argv[4]) : 8;
    unsigned seed = argc > 5 ? atoi(argv[5]) : 1;
    const bool g_only = argc > 6 && atoi(argv[6]) == 1;   // factor G itself (alpha 1, d 0)
    int64_t n = int64_t(layers) * nx * ny;
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(0.1, 1.0);
    std::vector<int32_t> a, b, crd(3 * n);
    std::vector<double> g;
    auto id = [&](int L, int i, int j) { return int32_t(L * nx * ny + i * ny + j); };
    for (int L = 0; L < layers; ++L)
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j) {
                int32_t v = id(L, i, j);
                crd[3 * v] = L; crd[3 * v + 1] = i; crd[3 * v + 2] = j;
                if (j + 1 < ny) { a.push_back(v); b.push_back(id(L, i, j + 1)); g.push_back(1 / U(rng)); }
                if (i + 1 < nx) { a.push_back(v); b.push_back(id(L, i + 1, j)); g.push_back(1 / U(rng)); }
                if (L + 1 < layers && i % 3 == 0 && j % 3 == 0) {
                    a.push_back(v); b.push_back(id(L + 1, i, j)); g.push_back(20.0);
                }
            }
    std::vector<int32_t> pads = {id(layers - 1, 0, 0), id(layers - 1, nx - 1, ny - 1)};
    std::vector<double> padg = {100.0, 100.0};
    Csr G = assemble_g(n, a.size(), a.data(), b.data(), g.data(), 2, pads.data(), padg.data());
    std::vector<double> c(n);
    for (auto& x : c) x = 1e-14 * U(rng);
    double alpha = g_only ? 1.0 : 1e-11;
    if (g_only) std::fill(c.begin(), c.end(), 0.0);
    Symbolic s = analyse(G, crd.data(), leaf);
    std::vector<double> W;
    if (factor_panels(s, G, alpha, c.data(), W, 1) != 0) { printf("FACTOR FAILED\n"); return 2; }
    // dense reference of A = alpha G + diag(c), solve by Gaussian elimination
    std::vector<double> A(n * n, 0.0), rhs(n), xr(n);
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = G.rp[i]; p < G.rp[i + 1]; ++p) A[i * n + G.ci[p]] += alpha * G.v[p];
        A[i * n + i] += c[i];
        rhs[i] = U(rng) - 0.5;
    }
    {
        std::vector<double> M = A, r = rhs;
        for (int64_t k = 0; k < n; ++k) {
            for (int64_t i = k + 1; i < n; ++i) {
                double f = M[i * n + k] / M[k * n + k];
                if (f == 0.0) continue;
                for (int64_t j = k; j < n; ++j) M[i * n + j] -= f * M[k * n + j];
                r[i] -= f * r[k];
            }
        }
        for (int64_t k = n - 1; k >= 0; --k) {
            double t = r[k];
            for (int64_t j = k + 1; j < n; ++j) t -= M[k * n + j] * xr[j];
            xr[k] = t / M[k * n + k];
        }
    }
    // emulated sweeps in the new ordering
    std::vector<double> bb(n), y(n), x(n), upd(s.n_upd, 0.0);
    for (int64_t k = 0; k < n; ++k) bb[k] = rhs[s.perm[k]];
    // forward: btilde = b_s - (children's updates mapped into s's columns);
    // [y_s ; w] = W_s btilde; s's update = (children's updates mapped into s's
    // off rows) + w
    for (int lv = 0; lv < s.n_levels; ++lv)
        for (int32_t k : s.level_sn[lv]) {
            const Supernode& q = s.sn[k];
            std::vector<double> f(q.nr, 0.0);
            for (int t = 0; t < q.nc; ++t) f[t] = bb[q.c0 + t];
            for (int32_t cp = s.child_ptr[k]; cp < s.child_ptr[k + 1]; ++cp) {
                const Supernode& qc = s.sn[s.child_idx[cp]];
                for (int t = 0; t < qc.nr - qc.nc; ++t) {
                    const int32_t pos = s.relidx[qc.u + t];
                    if (pos < q.nc) f[pos] -= upd[qc.u + t];
                    else f[pos] += upd[qc.u + t];
                }
            }
            for (int rr = 0; rr < q.nr; ++rr) {
                double acc = 0;
                for (int t = 0; t < q.nc; ++t) acc += W[q.w + rr + int64_t(t) * panel_ld(q.nr)] * f[t];
                if (rr < q.nc) y[q.c0 + rr] = acc; else upd[q.u + rr - q.nc] = f[rr] + acc;
            }
        }
    for (int lv = s.n_levels - 1; lv >= 0; --lv)
        for (int32_t k : s.level_sn[lv]) {
            const Supernode& q = s.sn[k];
            for (int t = 0; t < q.nc; ++t) {
                double acc = 0;
                for (int rr = 0; rr < q.nr; ++rr) {
                    double gv = rr < q.nc ? y[q.c0 + rr] : -x[s.rows[q.roff + rr - q.nc]];
                    acc += W[q.w + rr + int64_t(t) * panel_ld(q.nr)] * gv;
                }
                x[q.c0 + t] = acc;
            }
        }
    double err = 0, mx = 0;
    for (int64_t k = 0; k < n; ++k) {
        err = std::fmax(err, std::fabs(x[k] - xr[s.perm[k]]));
        mx = std::fmax(mx, std::fabs(xr[s.perm[k]]));
    }
    // structural nonzeros of L by dense symbolic elimination of P A P^T:
    // eliminating column k makes row i and row j (both > k, both coupled
    // to k) coupled
    int64_t nnz_dense = 0;
    {
        std::vector<char> P(n * n, 0);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = G.rp[i]; p < G.rp[i + 1]; ++p) P[s.iperm[i] * n + s.iperm[G.ci[p]]] = 1;
        for (int64_t k = 0; k < n; ++k) {
            std::vector<int64_t> below;
            for (int64_t i = k + 1; i < n; ++i)
                if (P[i * n + k]) below.push_back(i);
            nnz_dense += 1 + int64_t(below.size());
            for (int64_t i : below)
                for (int64_t j : below) P[i * n + j] = 1;
        }
    }
    printf("n %lld supernodes %zu levels %d nnzL stored %lld exact %lld (dense symbolic %lld) max_nr %d "
           "rel_err %.3e\n", (long long)n, s.sn.size(), s.n_levels, (long long)s.nnz_l,
           (long long)s.nnz_exact, (long long)nnz_dense, s.max_nr, err / mx);
    return (err / mx < 1e-12 && s.nnz_exact == nnz_dense && s.nnz_exact <= s.nnz_l) ? 0 : 1;
}

// Host-side ordering, symbolic analysis and multifrontal Cholesky.
//
// Ordering: geometric nested dissection. A node set is cut by the grid plane
// through its median coordinate along its longer horizontal extent; the
// plane's nodes (plus any node of the lower side still adjacent to the upper
// side, so the cut is a vertex separator for any graph) become a supernode
// ordered after both halves. Each ND-tree node is one supernode with a dense
// diagonal block and one shared off-diagonal row list; that is a (relaxed)
// supernodal Cholesky structure, and the ND tree is its assembly tree.
//
// For the device sweeps every supernode s keeps the panel
//     W_s = [ L11^-1 ; L21 L11^-1 ]      (nr x nc, column-major)
// so one forward step is a single matrix-vector product W_s * btilde_s and
// one backward step is W_s^T times [y_s ; -x(off rows)] (see kernels.hip).
#include "factor.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <stdexcept>
#include <thread>

namespace matex {

Csr assemble_g(int64_t n, int64_t n_branch, const int32_t* a, const int32_t* b,
               const double* g, int32_t n_pad, const int32_t* pad, const double* pad_g)
{
    struct E { int64_t key; double v; };
    std::vector<E> e;
    e.reserve(4 * n_branch + n_pad);
    for (int64_t k = 0; k < n_branch; ++k) {
        int64_t i = a[k], j = b[k];
        e.push_back({i * n + j, -g[k]});
        e.push_back({j * n + i, -g[k]});
        e.push_back({i * n + i, g[k]});
        e.push_back({j * n + j, g[k]});
    }
    for (int32_t k = 0; k < n_pad; ++k) e.push_back({int64_t(pad[k]) * n + pad[k], pad_g[k]});
    std::stable_sort(e.begin(), e.end(), [](const E& x, const E& y) { return x.key < y.key; });
    Csr c;
    c.n = n;
    c.rp.assign(n + 1, 0);
    for (size_t k = 0; k < e.size();) {
        size_t q = k;
        double s = 0.0;
        while (q < e.size() && e[q].key == e[k].key) s += e[q++].v;
        int64_t i = e[k].key / n;
        c.ci.push_back(int32_t(e[k].key % n));
        c.v.push_back(s);
        c.rp[i + 1]++;
        k = q;
    }
    for (int64_t i = 0; i < n; ++i) c.rp[i + 1] += c.rp[i];
    return c;
}

namespace {

struct NdBuilder {
    const Csr& g;
    std::vector<int32_t> crd;   // n x 3
    int32_t leaf_max;
    std::vector<int32_t> order;
    std::vector<Supernode> sn;
    std::vector<int8_t> side;
    std::vector<int32_t> stamp;
    int32_t cur = 0;

    NdBuilder(const Csr& g_, int32_t lm) : g(g_), leaf_max(lm) {
        side.assign(g.n, 0);
        stamp.assign(g.n, -1);
    }

    int32_t make_sn(const std::vector<int32_t>& cols) {
        Supernode s;
        s.c0 = int32_t(order.size());
        s.nc = int32_t(cols.size());
        order.insert(order.end(), cols.begin(), cols.end());
        sn.push_back(s);
        return int32_t(sn.size() - 1);
    }

    std::vector<int32_t> build(std::vector<int32_t>& S) {
        if (int32_t(S.size()) <= leaf_max) return {make_sn(S)};
        int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
        for (int32_t v : S)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], crd[3 * v + d]);
                hi[d] = std::max(hi[d], crd[3 * v + d]);
            }
        int axis = (hi[1] - lo[1] >= hi[2] - lo[2]) ? 1 : 2;
        if (hi[axis] == lo[axis]) axis = 0;
        if (hi[axis] == lo[axis]) return {make_sn(S)};
        std::vector<int32_t> vals(S.size());
        for (size_t k = 0; k < S.size(); ++k) vals[k] = crd[3 * S[k] + axis];
        std::nth_element(vals.begin(), vals.begin() + vals.size() / 2, vals.end());
        int32_t m = vals[vals.size() / 2];
        int32_t id = cur++;
        for (int32_t v : S) {
            int32_t c = crd[3 * v + axis];
            side[v] = c < m ? 0 : (c > m ? 1 : 2);
            stamp[v] = id;
        }
        // make the cut a vertex separator for any graph
        for (int32_t v : S) {
            if (side[v] != 0) continue;
            for (int64_t p = g.rp[v]; p < g.rp[v + 1]; ++p) {
                int32_t w = g.ci[p];
                if (w != v && stamp[w] == id && side[w] == 1) { side[v] = 2; break; }
            }
        }
        std::vector<int32_t> L, R, Sep;
        for (int32_t v : S) (side[v] == 0 ? L : side[v] == 1 ? R : Sep).push_back(v);
        if (L.empty() && R.empty()) return {make_sn(S)};
        std::vector<int32_t> roots;
        if (!L.empty()) { auto r = build(L); roots.insert(roots.end(), r.begin(), r.end()); }
        if (!R.empty()) { auto r = build(R); roots.insert(roots.end(), r.begin(), r.end()); }
        if (Sep.empty()) return roots;
        int32_t s = make_sn(Sep);
        for (int32_t r : roots) sn[r].parent = s;
        return {s};
    }
};

// 1-D coordinate for graphs without geometry: BFS distance from a
// pseudo-peripheral vertex of each connected component.
std::vector<int32_t> bfs_coords(const Csr& g)
{
    int64_t n = g.n;
    std::vector<int32_t> crd(3 * n, 0), dist(n, -1), q(n);
    auto bfs = [&](int32_t s, std::vector<int32_t>& d, std::vector<int32_t>& visited) {
        int64_t h = 0, t = 0;
        q[t++] = s;
        d[s] = 0;
        visited.push_back(s);
        while (h < t) {
            int32_t u = q[h++];
            for (int64_t p = g.rp[u]; p < g.rp[u + 1]; ++p) {
                int32_t w = g.ci[p];
                if (d[w] < 0) { d[w] = d[u] + 1; q[t++] = w; visited.push_back(w); }
            }
        }
        return q[t - 1];
    };
    std::vector<int32_t> tmp(n, -1);
    for (int64_t i = 0; i < n; ++i) {
        if (dist[i] >= 0) continue;
        std::vector<int32_t> vis;
        int32_t far = bfs(int32_t(i), tmp, vis);
        for (int32_t v : vis) tmp[v] = -1;
        vis.clear();
        bfs(far, dist, vis);
    }
    for (int64_t i = 0; i < n; ++i) crd[3 * i + 1] = dist[i];
    return crd;
}

}  // namespace

// Structural nonzeros of the Cholesky factor of P G P^T (diagonal included):
// the elimination tree (Liu's algorithm, with path compression on a
// separate ancestor array), then for every row i the row subtree, the
// nodes on the paths from each k < i with G(i, k) != 0 up to i. The
// supernodal panels store more (the explicit zeros of each supernode's
// shared row list and of relaxed leaves); this is what a solve must read.
static int64_t exact_lower_nnz(const Csr& g, const Symbolic& s)
{
    const int64_t n = s.n;
    std::vector<int32_t> parent(n, -1), anc(n, -1), mark(n, -1);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t o = s.perm[i];
        for (int64_t p = g.rp[o]; p < g.rp[o + 1]; ++p) {
            int32_t j = s.iperm[g.ci[p]];
            while (j != -1 && j < i) {
                const int32_t nx = anc[j];
                anc[j] = int32_t(i);
                if (nx == -1) parent[j] = int32_t(i);
                j = nx;
            }
        }
    }
    int64_t nnz = n;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t o = s.perm[i];
        mark[i] = int32_t(i);
        for (int64_t p = g.rp[o]; p < g.rp[o + 1]; ++p) {
            const int32_t k = s.iperm[g.ci[p]];
            if (k >= i) continue;
            for (int32_t j = k; j != -1 && mark[j] != i; j = parent[j]) {
                mark[j] = int32_t(i);
                nnz++;
            }
        }
    }
    return nnz;
}

Symbolic analyse(const Csr& g, const int32_t* coord, int32_t leaf_max)
{
    Symbolic s;
    int64_t n = g.n;
    s.n = n;
    NdBuilder nd(g, leaf_max);
    if (coord) nd.crd.assign(coord, coord + 3 * n);
    else nd.crd = bfs_coords(g);
    std::vector<int32_t> all(n);
    std::iota(all.begin(), all.end(), 0);
    nd.build(all);
    s.perm = std::move(nd.order);
    s.sn = std::move(nd.sn);
    s.iperm.assign(n, 0);
    for (int64_t k = 0; k < n; ++k) s.iperm[s.perm[k]] = int32_t(k);

    const int32_t nsn = int32_t(s.sn.size());
    std::vector<std::vector<int32_t>> kids(nsn);
    for (int32_t k = 0; k < nsn; ++k)
        if (s.sn[k].parent >= 0) kids[s.sn[k].parent].push_back(k);

    // off-diagonal row structure, bottom-up (postorder = index order)
    std::vector<int32_t> mark(n, -1);
    std::vector<std::vector<int32_t>> roffs(nsn);
    for (int32_t k = 0; k < nsn; ++k) {
        Supernode& q = s.sn[k];
        int32_t c1 = q.c0 + q.nc;
        std::vector<int32_t>& R = roffs[k];
        for (int32_t j = q.c0; j < c1; ++j) {
            int32_t o = s.perm[j];
            for (int64_t p = g.rp[o]; p < g.rp[o + 1]; ++p) {
                int32_t r = s.iperm[g.ci[p]];
                if (r >= c1 && mark[r] != k) { mark[r] = k; R.push_back(r); }
            }
        }
        for (int32_t c : kids[k]) {
            for (int32_t r : roffs[c])
                if (r >= c1 && mark[r] != k) { mark[r] = k; R.push_back(r); }
            std::vector<int32_t>().swap(roffs[c]);   // consumed by the parent only
        }
        std::sort(R.begin(), R.end());
        q.nr = q.nc + int32_t(R.size());
        // store now (children lists were consumed above)
        q.roff = int64_t(s.rows.size());
        s.rows.insert(s.rows.end(), R.begin(), R.end());
    }
    // levels
    for (int32_t k = 0; k < nsn; ++k) {
        int32_t p = s.sn[k].parent;
        if (p >= 0) s.sn[p].level = std::max(s.sn[p].level, s.sn[k].level + 1);
    }
    int32_t H = 0;
    for (auto& q : s.sn) H = std::max(H, q.level);
    s.n_levels = H + 1;
    s.level_sn.assign(s.n_levels, {});
    for (int32_t k = 0; k < nsn; ++k) s.level_sn[s.sn[k].level].push_back(k);
    // panel and update-slot offsets
    int64_t w = 0, u = 0, nnz = 0;
    for (auto& q : s.sn) {
        q.w = w;
        q.u = u;
        int64_t off = q.nr - q.nc;
        w += int64_t(panel_ld(q.nr)) * q.nc;
        u += off;
        nnz += int64_t(q.nc) * (q.nc + 1) / 2 + off * q.nc;
        s.max_nr = std::max(s.max_nr, q.nr);
        s.max_nc = std::max(s.max_nc, q.nc);
    }
    s.n_w = w;
    s.n_upd = u;
    s.nnz_l = nnz;
    s.nnz_exact = exact_lower_nnz(g, s);
    // children lists and each off-diagonal row's place among the parent's rows
    s.child_ptr.assign(nsn + 1, 0);
    for (int32_t k = 0; k < nsn; ++k)
        if (s.sn[k].parent >= 0) s.child_ptr[s.sn[k].parent + 1]++;
    for (int32_t k = 0; k < nsn; ++k) s.child_ptr[k + 1] += s.child_ptr[k];
    s.child_idx.assign(s.child_ptr[nsn], 0);
    {
        std::vector<int32_t> fill(s.child_ptr.begin(), s.child_ptr.end() - 1);
        for (int32_t k = 0; k < nsn; ++k)
            if (s.sn[k].parent >= 0) s.child_idx[fill[s.sn[k].parent]++] = k;
    }
    s.relidx.assign(s.n_upd, 0);
    for (int32_t k = 0; k < nsn; ++k) {
        const Supernode& q = s.sn[k];
        const int32_t no = q.nr - q.nc;
        if (q.parent < 0) {
            if (no != 0) throw std::logic_error("a root supernode has off-diagonal rows");
            continue;
        }
        const Supernode& pq = s.sn[q.parent];
        const int32_t* prow = s.rows.data() + pq.roff;
        const int32_t pno = pq.nr - pq.nc;
        for (int32_t t = 0; t < no; ++t) {
            const int32_t r = s.rows[q.roff + t];
            int32_t pos;
            if (r >= pq.c0 && r < pq.c0 + pq.nc) {
                pos = r - pq.c0;
            } else {
                const int32_t* it = std::lower_bound(prow, prow + pno, r);
                if (it == prow + pno || *it != r)
                    throw std::logic_error("off-diagonal row missing from the parent's rows");
                pos = pq.nc + int32_t(it - prow);
            }
            s.relidx[q.u + t] = pos;
        }
    }
    return s;
}

namespace {

// In-place dense kernels on column-major blocks (leading dimension ld).
// Cholesky of the leading k x k block; returns -1 or the failing column.
int64_t potrf(double* F, int64_t ld, int64_t k)
{
    for (int64_t j = 0; j < k; ++j) {
        double* cj = F + j * ld;
        double d = cj[j];
        if (!(d > 0.0)) return j;
        d = std::sqrt(d);
        cj[j] = d;
        double inv = 1.0 / d;
        for (int64_t i = j + 1; i < k; ++i) cj[i] *= inv;
        // right-looking rank-1 update of the trailing block (lower part)
        for (int64_t q = j + 1; q < k; ++q) {
            double l = cj[q];
            if (l == 0.0) continue;
            double* cq = F + q * ld;
            for (int64_t i = q; i < k; ++i) cq[i] -= cj[i] * l;
        }
    }
    return -1;
}

}  // namespace

int64_t factor_panels(const Symbolic& s, const Csr& g, double alpha, const double* d,
                      std::vector<double>& W, int n_threads)
{
    (void)n_threads;
    const int64_t n = s.n;
    const int32_t nsn = int32_t(s.sn.size());
    W.assign(s.n_w, 0.0);
    std::vector<std::vector<int32_t>> kids(nsn);
    for (int32_t k = 0; k < nsn; ++k)
        if (s.sn[k].parent >= 0) kids[s.sn[k].parent].push_back(k);
    std::vector<std::vector<double>> U(nsn);
    std::vector<int32_t> pos(n, -1);
    std::vector<double> F, Linv;
    for (int32_t k = 0; k < nsn; ++k) {
        const Supernode& q = s.sn[k];
        const int64_t nr = q.nr, nc = q.nc, no = nr - nc;
        const int32_t* roff = s.rows.data() + q.roff;
        F.assign(nr * nr, 0.0);
        for (int64_t t = 0; t < nc; ++t) pos[q.c0 + t] = int32_t(t);
        for (int64_t t = 0; t < no; ++t) pos[roff[t]] = int32_t(nc + t);
        // original entries of alpha G + diag(d), columns of this supernode
        for (int64_t t = 0; t < nc; ++t) {
            int32_t j = q.c0 + int32_t(t);
            int32_t o = s.perm[j];
            F[t + t * nr] += d[o];
            for (int64_t p = g.rp[o]; p < g.rp[o + 1]; ++p) {
                int32_t r = s.iperm[g.ci[p]];
                if (r >= j) F[pos[r] + t * nr] += alpha * g.v[p];
            }
        }
        // extend-add the children's update matrices
        for (int32_t c : kids[k]) {
            const Supernode& qc = s.sn[c];
            const int64_t nb = qc.nr - qc.nc;
            const int32_t* rc = s.rows.data() + qc.roff;
            const double* Uc = U[c].data();
            for (int64_t b = 0; b < nb; ++b) {
                int64_t col = pos[rc[b]];
                double* Fc = F.data() + col * nr;
                for (int64_t a = b; a < nb; ++a) Fc[pos[rc[a]]] += Uc[a + b * nb];
            }
            std::vector<double>().swap(U[c]);
        }
        // L11 = chol(F11)
        int64_t bad = potrf(F.data(), nr, nc);
        if (bad >= 0) {
            for (int64_t t = 0; t < nc; ++t) pos[q.c0 + t] = -1;
            for (int64_t t = 0; t < no; ++t) pos[roff[t]] = -1;
            return q.c0 + bad + 1;
        }
        // L21 = F21 L11^-T (column by column, rows contiguous)
        for (int64_t j = 0; j < nc; ++j) {
            double* cj = F.data() + j * nr + nc;
            for (int64_t kk = 0; kk < j; ++kk) {
                double l = F[j + kk * nr];
                if (l == 0.0) continue;
                const double* ck = F.data() + kk * nr + nc;
                for (int64_t i = 0; i < no; ++i) cj[i] -= ck[i] * l;
            }
            double inv = 1.0 / F[j + j * nr];
            for (int64_t i = 0; i < no; ++i) cj[i] *= inv;
        }
        // U = F22 - L21 L21^T (lower part)
        if (no > 0) {
            U[k].assign(no * no, 0.0);
            double* Uk = U[k].data();
            for (int64_t b = 0; b < no; ++b)
                std::memcpy(Uk + b * no + b, F.data() + (nc + b) * nr + nc + b,
                            sizeof(double) * (no - b));
            for (int64_t kk = 0; kk < nc; ++kk) {
                const double* lk = F.data() + kk * nr + nc;
                for (int64_t b = 0; b < no; ++b) {
                    double l = lk[b];
                    if (l == 0.0) continue;
                    double* ub = Uk + b * no;
                    for (int64_t a = b; a < no; ++a) ub[a] -= lk[a] * l;
                }
            }
        }
        // Linv = L11^-1 (lower), column by column
        Linv.assign(nc * nc, 0.0);
        for (int64_t j = 0; j < nc; ++j) {
            double* x = Linv.data() + j * nc;
            x[j] = 1.0;
            for (int64_t kk = j; kk < nc; ++kk) {
                x[kk] /= F[kk + kk * nr];
                double xk = x[kk];
                if (xk == 0.0) continue;
                const double* lk = F.data() + kk * nr;
                for (int64_t i = kk + 1; i < nc; ++i) x[i] -= lk[i] * xk;
            }
        }
        // W = [Linv ; L21 Linv], columns padded to panel_ld(nr)
        double* Wk = W.data() + q.w;
        const int64_t ld = panel_ld(q.nr);
        for (int64_t j = 0; j < nc; ++j) {
            double* wj = Wk + j * ld;
            const double* lj = Linv.data() + j * nc;
            for (int64_t i = j; i < nc; ++i) wj[i] = lj[i];
            double* w2 = wj + nc;
            for (int64_t kk = j; kk < nc; ++kk) {
                double l = lj[kk];
                if (l == 0.0) continue;
                const double* ck = F.data() + kk * nr + nc;
                for (int64_t i = 0; i < no; ++i) w2[i] += ck[i] * l;
            }
        }
        for (int64_t t = 0; t < nc; ++t) pos[q.c0 + t] = -1;
        for (int64_t t = 0; t < no; ++t) pos[roff[t]] = -1;
    }
    return 0;
}

}  // namespace matex

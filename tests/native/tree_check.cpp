// Host replay of the subtree sweeps (k_forward_tree / k_backward_tree) on the
// schedule the library builds: every block, wavefront and lane forms the
// addresses the kernels form (the items' copy into LDS, the loads issued
// ahead, including the clamped ones of idle lanes and items, the LDS reads
// and writes, the stores of y, x and the update slots), and each one is
// checked against the size of the buffer or LDS region it falls in. The
// values are computed too: the solve with the subtree part replayed and the
// levels above swept by a plain supernodal sweep must equal the plain sweep
// of every supernode.
//
// Usage: tree_check layers nx ny leaf_max seed
//        tree_check --file netlist.bin leaf_max
// (the file: int64 n, int64 n_branch, int32 n_pad, double vdd, then br_a,
// br_b (int32), br_g (f64), c (f64, n), pad_node (int32), pad_g (f64),
// coord (int32, 3n)). Exit 0 when every check passes.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../paper_1511_04519_amd/csrc/factor.hpp"
#include "../../paper_1511_04519_amd/csrc/schedule.hpp"

using namespace matex;

namespace {

constexpr int TPF = 16;   // panel entries per lane loaded ahead (kernels.hip)
int64_t n_fail = 0;

void expect(bool ok, const char* what, int64_t idx, int64_t size, int b, int s, int wv, int lane)
{
    if (ok) return;
    if (n_fail < 20)
        std::printf("OUT OF RANGE %s: index %lld, size %lld (block %d step %d wave %d lane %d)\n", what,
                    (long long)idx, (long long)size, b, s, wv, lane);
    n_fail++;
}

struct Net {
    int64_t n = 0;
    std::vector<int32_t> a, b, pad, crd;
    std::vector<double> g, c, padg;
};

Net mesh(int layers, int nx, int ny, unsigned seed)
{
    Net N;
    N.n = int64_t(layers) * nx * ny;
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(0.1, 1.0);
    N.crd.resize(3 * N.n);
    auto id = [&](int L, int i, int j) { return int32_t(L * nx * ny + i * ny + j); };
    for (int L = 0; L < layers; ++L)
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j) {
                const int32_t v = id(L, i, j);
                N.crd[3 * v] = L; N.crd[3 * v + 1] = i; N.crd[3 * v + 2] = j;
                if (j + 1 < ny) { N.a.push_back(v); N.b.push_back(id(L, i, j + 1)); N.g.push_back(1 / U(rng)); }
                if (i + 1 < nx) { N.a.push_back(v); N.b.push_back(id(L, i + 1, j)); N.g.push_back(1 / U(rng)); }
                if (L + 1 < layers && i % 10 == 0 && j % 10 == 0) {
                    N.a.push_back(v); N.b.push_back(id(L + 1, i, j)); N.g.push_back(20.0);
                }
            }
    for (int i = 7; i < nx; i += 15)
        for (int j = 7; j < ny; j += 15) { N.pad.push_back(id(layers - 1, i, j)); N.padg.push_back(100.0); }
    if (N.pad.empty()) { N.pad.push_back(id(layers - 1, 0, 0)); N.padg.push_back(100.0); }
    N.c.resize(N.n);
    for (auto& x : N.c) x = 1e-15 * std::pow(100.0, U(rng));
    return N;
}

Net read_file(const char* path)
{
    Net N;
    FILE* f = std::fopen(path, "rb");
    if (!f) { std::printf("cannot open %s\n", path); std::exit(2); }
    int64_t nb = 0;
    int32_t np = 0;
    double vdd = 0;
    bool ok = std::fread(&N.n, 8, 1, f) == 1 && std::fread(&nb, 8, 1, f) == 1 && std::fread(&np, 4, 1, f) == 1 &&
              std::fread(&vdd, 8, 1, f) == 1;
    N.a.resize(nb); N.b.resize(nb); N.g.resize(nb); N.c.resize(N.n);
    N.pad.resize(np); N.padg.resize(np); N.crd.resize(3 * N.n);
    ok = ok && std::fread(N.a.data(), 4, nb, f) == size_t(nb) && std::fread(N.b.data(), 4, nb, f) == size_t(nb) &&
         std::fread(N.g.data(), 8, nb, f) == size_t(nb) && std::fread(N.c.data(), 8, N.n, f) == size_t(N.n) &&
         std::fread(N.pad.data(), 4, np, f) == size_t(np) && std::fread(N.padg.data(), 8, np, f) == size_t(np) &&
         std::fread(N.crd.data(), 4, 3 * N.n, f) == size_t(3 * N.n);
    std::fclose(f);
    if (!ok) { std::printf("short read of %s\n", path); std::exit(2); }
    return N;
}

// Plain supernodal sweeps over the supernodes with level >= from (forward)
// or all supernodes with level >= from (backward) in postorder; upd holds
// every supernode's update slots, y the forward result, x the solution.
void plain_forward(const Symbolic& s, const Contrib& C, const std::vector<double>& W, const std::vector<double>& rhs,
                   int from, std::vector<double>& y, std::vector<double>& upd)
{
    std::vector<double> bt;
    for (size_t k = 0; k < s.sn.size(); ++k) {
        const Supernode& q = s.sn[k];
        if (q.level < from) continue;
        const int64_t ld = panel_ld(q.nr);
        auto pull = [&](int32_t p) {
            double v = 0.0;
            const int64_t gp = C.pos_base[k] + p;
            for (int32_t j = C.cptr[gp]; j < C.cptr[gp + 1]; ++j) v += upd[C.cidx[j]];
            return v;
        };
        bt.assign(q.nc, 0.0);
        for (int32_t c = 0; c < q.nc; ++c) bt[c] = rhs[q.c0 + c] - pull(c);
        for (int32_t r = 0; r < q.nr; ++r) {
            double acc = 0.0;
            const int32_t kmax = r < q.nc ? r + 1 : q.nc;
            for (int32_t c = 0; c < kmax; ++c) acc += W[q.w + r + c * ld] * bt[c];
            if (r < q.nc) y[q.c0 + r] = acc;
            else upd[q.u + r - q.nc] = pull(r) + acc;
        }
    }
}

void plain_backward(const Symbolic& s, const std::vector<double>& W, const std::vector<double>& y, int from,
                    std::vector<double>& x)
{
    std::vector<double> g;
    for (size_t kk = s.sn.size(); kk-- > 0;) {
        const Supernode& q = s.sn[kk];
        if (q.level < from) continue;
        const int64_t ld = panel_ld(q.nr);
        g.assign(q.nr, 0.0);
        for (int32_t r = 0; r < q.nr; ++r) g[r] = r < q.nc ? y[q.c0 + r] : -x[s.rows[q.roff + r - q.nc]];
        for (int32_t c = 0; c < q.nc; ++c) {
            double acc = 0.0;
            for (int32_t r = c; r < q.nr; ++r) acc += W[q.w + r + c * ld] * g[r];
            x[q.c0 + c] = acc;
        }
    }
}

// Step that last wrote each shared LDS slot (-1: never): a read must see a
// write of an earlier step (steps are separated by block barriers, the
// wavefronts of one step are not).
std::vector<int> sh_step;

void expect_written(int64_t o, int b, int s, int wv, int lane)
{
    const bool ok = o >= 0 && o < int64_t(sh_step.size()) && sh_step[o] >= 0 && sh_step[o] < s;
    expect(ok, "LDS shared read before an earlier step wrote it", o, int64_t(sh_step.size()), b, s, wv, lane);
}

double desc_sum(int32_t d, const std::vector<double>& sh, int64_t shared, int b, int s, int wv, int lane)
{
    double v = 0.0;
    const int o0 = d & 0xffff, o1 = (d >> 16) & 0xffff;
    if (o0) {
        expect(o0 - 1 < shared, "LDS shared read (forward desc)", o0 - 1, shared, b, s, wv, lane);
        expect_written(o0 - 1, b, s, wv, lane);
        v += sh[o0 - 1];
    }
    if (o1) {
        expect(o1 - 1 < shared, "LDS shared read (forward desc)", o1 - 1, shared, b, s, wv, lane);
        expect_written(o1 - 1, b, s, wv, lane);
        v += sh[o1 - 1];
    }
    return v;
}

}  // namespace

int main(int argc, char** argv)
{
    Net N;
    int leaf = 16;
    if (argc > 1 && std::string(argv[1]) == "--file") {
        N = read_file(argv[2]);
        leaf = argc > 3 ? std::atoi(argv[3]) : 16;
    } else {
        const int layers = argc > 1 ? std::atoi(argv[1]) : 2, nx = argc > 2 ? std::atoi(argv[2]) : 64,
                  ny = argc > 3 ? std::atoi(argv[3]) : 64;
        leaf = argc > 4 ? std::atoi(argv[4]) : 16;
        N = mesh(layers, nx, ny, argc > 5 ? unsigned(std::atoi(argv[5])) : 1u);
    }
    const int64_t n = N.n;
    Csr G = assemble_g(n, int64_t(N.a.size()), N.a.data(), N.b.data(), N.g.data(), int32_t(N.pad.size()),
                       N.pad.data(), N.padg.data());
    Symbolic s = analyse(G, N.crd.data(), leaf);
    std::vector<double> W;
    std::vector<double> cperm(n);
    for (int64_t k = 0; k < n; ++k) cperm[k] = N.c[s.perm[k]];
    if (factor_panels(s, G, 1e-11, N.c.data(), W, 8) != 0) { std::printf("factor failed\n"); return 2; }
    const Contrib C = contributions(s);
    const TreeHost T = build_tree_host(s, C, 0);
    std::printf("n %lld, supernodes %zu, levels %d, subtree levels %d, blocks %d, LDS %d doubles "
                "(items %d, wave scratch %d x %d)\n",
                (long long)n, s.sn.size(), s.n_levels, T.n_levels, T.n_blocks, T.lds_doubles, T.item_doubles, TW,
                T.ws);
    if (T.n_levels == 0) { std::printf("no subtree sweeps on this grid\n"); return 3; }
    const int64_t shared_cap = int64_t(T.lds_doubles) - T.item_doubles - int64_t(TW) * T.ws;
    const int64_t nW = int64_t(W.size()), nU = std::max<int64_t>(1, s.n_upd);
    const int64_t nfd = int64_t(T.fdesc.size()), ntr = int64_t(T.trow.size());
    const int64_t nfi = int64_t(T.fitems.size()), nbi = int64_t(T.bitems.size());
    if (int64_t(T.lds_doubles) * 8 > 160 * 1024) std::printf("LDS of a block exceeds 160 KiB\n"), n_fail++;

    // right-hand side b (random), scale C
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    std::vector<double> b(n), rhs(n);
    for (auto& v : b) v = U(rng);
    for (int64_t i = 0; i < n; ++i) rhs[i] = b[i] * cperm[i];

    // reference: plain sweeps over every supernode
    std::vector<double> y_ref(n, 0.0), x_ref(n, 0.0), upd_ref(nU, 0.0);
    plain_forward(s, C, W, rhs, 0, y_ref, upd_ref);
    plain_backward(s, W, y_ref, 0, x_ref);

    // replay: subtree blocks, then the levels above
    std::vector<double> y(n, 0.0), x(n, 0.0), upd(nU, 0.0);
    const double NaN = std::nan("");
    std::vector<double> sh, scratch;
    auto item_copy = [&](const std::vector<int32_t>& blk, int64_t nitems, int bidx, int& s0, int& s1) {
        expect(bidx + 1 < int64_t(blk.size()), "block table", bidx + 1, int64_t(blk.size()), bidx, -1, -1, -1);
        s0 = blk[bidx]; s1 = blk[bidx + 1];
        expect(s1 > s0, "empty block (no step)", s1 - s0, 1, bidx, -1, -1, -1);
        expect(int64_t(s1) * TW <= nitems, "item copy (global read)", int64_t(s1) * TW - 1, nitems, bidx, -1, -1, -1);
        expect(int64_t(s1 - s0) * TW * 6 <= T.item_doubles, "item copy (LDS write)", int64_t(s1 - s0) * TW * 6,
               T.item_doubles, bidx, -1, -1, -1);
    };
    for (int bk = 0; bk < T.n_blocks; ++bk) {
        int s0, s1;
        item_copy(T.fblk, nfi, bk, s0, s1);
        const int64_t shb = T.shared[bk];
        expect(shb <= shared_cap, "shared region", shb, shared_cap, bk, -1, -1, -1);
        sh.assign(std::max<int64_t>(shared_cap, 1), NaN);
        sh_step.assign(sh.size(), -1);
        for (int st = s0; st < s1; ++st) {
            for (int wv = 0; wv < TW; ++wv) {
                const TItem& t = T.fitems[int64_t(st) * TW + wv];
                const int64_t item = int64_t(st) * TW + wv;
                const int64_t ld = t.nr > 0 ? panel_ld(t.nr) : 0;
                scratch.assign(T.ws, NaN);   // bt of this wavefront
                // loads issued ahead (every lane, idle ones clamped)
                std::vector<double> a(64 * TPF), bv(64), sv(64);
                std::vector<I2> d(64);
                for (int lane = 0; lane < 64; ++lane) {
                    const int row = t.first + lane;
                    const int kmax = row >= t.last ? 0 : (row < t.nc ? row + 1 : t.nc);
                    const int64_t wr = t.w + (row < t.last ? row : t.first);
                    for (int q = 0; q < TPF; ++q) {
                        const int64_t ix = wr + (q < kmax ? q : 0) * ld;
                        expect(ix >= 0 && ix < nW, "W load (forward, ahead)", ix, nW, bk, st, wv, lane);
                        a[lane * TPF + q] = (ix >= 0 && ix < nW) ? W[ix] : 0.0;
                    }
                    const int64_t col = t.c0 + (lane < t.nc ? lane : 0);
                    expect(col >= 0 && col < n, "b / scale load", col, n, bk, st, wv, lane);
                    bv[lane] = b[col];
                    sv[lane] = cperm[col];
                    const int64_t di = item * 64 + lane;
                    expect(di >= 0 && di < nfd, "fdesc load", di, nfd, bk, st, wv, lane);
                    d[lane] = T.fdesc[di];
                }
                if (t.nr == 0) continue;
                std::vector<double> off(64, 0.0);
                for (int lane = 0; lane < 64; ++lane) {
                    const int row = t.first + lane;
                    const bool live = row < t.last;
                    if (lane < t.nc) {
                        expect(lane < T.ws, "LDS wave scratch (bt)", lane, T.ws, bk, st, wv, lane);
                        scratch[lane] = bv[lane] * sv[lane] - desc_sum(d[lane].x, sh, shb, bk, st, wv, lane);
                    }
                    if (live && row >= t.nc) off[lane] = desc_sum(d[lane].y, sh, shb, bk, st, wv, lane);
                }
                for (int lane = 0; lane < 64; ++lane) {
                    const int row = t.first + lane;
                    const bool live = row < t.last;
                    const int kmax = !live ? 0 : (row < t.nc ? row + 1 : t.nc);
                    double acc = 0.0;
                    for (int q = 0; q < TPF; ++q) acc += q < kmax ? a[lane * TPF + q] * scratch[q] : 0.0;
                    for (int k = TPF; k < kmax; ++k) {
                        const int64_t ix = t.w + row + k * ld;
                        expect(ix >= 0 && ix < nW, "W load (forward, in step)", ix, nW, bk, st, wv, lane);
                        acc += W[ix] * scratch[k];
                    }
                    if (!live) continue;
                    if (row < t.nc) {
                        const int64_t yi = int64_t(t.c0) + row;
                        expect(yi >= 0 && yi < n, "y store", yi, n, bk, st, wv, lane);
                        y[yi] = acc;
                    } else if (t.lds_u >= 0) {
                        const int64_t o = int64_t(t.lds_u) + row - t.nc;
                        expect(o >= 0 && o < shb, "LDS shared write (update slot)", o, shb, bk, st, wv, lane);
                        sh[o] = off[lane] + acc;
                        sh_step[o] = st;
                    } else {
                        const int64_t o = t.aux + row - t.nc;
                        expect(o >= 0 && o < nU, "update slot store", o, nU, bk, st, wv, lane);
                        upd[o] = off[lane] + acc;
                    }
                }
            }
        }
    }
    plain_forward(s, C, W, rhs, T.n_levels, y, upd);
    plain_backward(s, W, y, T.n_levels, x);
    for (int bk = 0; bk < T.n_blocks; ++bk) {
        int s0, s1;
        item_copy(T.bblk, nbi, bk, s0, s1);
        const int64_t shb = T.shared[bk];
        sh.assign(std::max<int64_t>(shared_cap, 1), NaN);
        sh_step.assign(sh.size(), -1);
        for (int st = s0; st < s1; ++st) {
            for (int wv = 0; wv < TW; ++wv) {
                const TItem& t = T.bitems[int64_t(st) * TW + wv];
                const int64_t ld = t.nr > 0 ? panel_ld(t.nr) : 0;
                scratch.assign(T.ws, NaN);   // g of this wavefront
                const int noff = t.nr - t.nc;
                const int cols = t.last - t.first;
                const int shf = cols > 1 ? 32 - __builtin_clz(unsigned(cols - 1)) : 0;
                const int lpc = 64 >> shf;
                std::vector<double> a(64 * TPF), gv(64 * 4);
                std::vector<int32_t> tr(64 * 4);
                for (int lane = 0; lane < 64; ++lane) {
                    for (int i = 0; i < TREE_MAX_NR / 64; ++i) {
                        const int k = t.first + lane + 64 * i;
                        const int o = k - t.nc;
                        const int64_t ti = t.aux + (o >= 0 && o < noff ? o : 0);
                        expect(ti >= 0 && ti < ntr, "trow load", ti, ntr, bk, st, wv, lane);
                        tr[lane * 4 + i] = T.trow[ti];
                    }
                    const int c = t.first + (lane >> (6 - shf)), q = lane & (lpc - 1);
                    const int kend = c < t.last ? t.nr : 0;
                    const int64_t wc = t.w + int64_t(c < t.last ? c : t.first) * ld;
                    for (int i = 0; i < TPF; ++i) {
                        const int k = c + q + i * lpc;
                        const int64_t ix = wc + (k < kend ? k : 0);
                        expect(ix >= 0 && ix < nW, "W load (backward, ahead)", ix, nW, bk, st, wv, lane);
                        a[lane * TPF + i] = (ix >= 0 && ix < nW) ? W[ix] : 0.0;
                    }
                    for (int i = 0; i < TREE_MAX_NR / 64; ++i) {
                        const int k = t.first + lane + 64 * i;
                        const bool own = k < t.nc;
                        const int32_t trv = tr[lane * 4 + i];
                        const int64_t gi = own ? int64_t(t.c0) + k : int64_t(trv >= 0 ? trv : 0);
                        expect(gi >= 0 && gi < n, own ? "y load (backward)" : "x load (off row)", gi, n, bk, st, wv,
                               lane);
                        gv[lane * 4 + i] = own ? y[gi] : x[gi];
                        if (k >= t.nr || own) tr[lane * 4 + i] = 0;
                    }
                }
                if (t.nr == 0) continue;
                for (int lane = 0; lane < 64; ++lane)
                    for (int i = 0; i < TREE_MAX_NR / 64; ++i) {
                        const int k = t.first + lane + 64 * i;
                        if (k >= t.nr) continue;
                        expect(k < T.ws, "LDS wave scratch (g)", k, T.ws, bk, st, wv, lane);
                        const int32_t trv = tr[lane * 4 + i];
                        double v;
                        if (trv < 0) {
                            const int64_t o = -1 - int64_t(trv);
                            expect(o < shb, "LDS shared read (ancestor x)", o, shb, bk, st, wv, lane);
                            expect_written(o, bk, st, wv, lane);
                            v = -sh[o];
                        } else {
                            v = k < t.nc ? gv[lane * 4 + i] : -gv[lane * 4 + i];
                        }
                        scratch[k] = v;
                    }
                // lpc lanes per column, their partial sums added (any order: compared with a tolerance)
                for (int lane = 0; lane < 64; lane += lpc) {
                    const int c = t.first + (lane >> (6 - shf));
                    const int kend = c < t.last ? t.nr : 0;
                    double acc = 0.0;
                    for (int q = 0; q < lpc; ++q)
                        for (int i = 0; i < TPF; ++i) {
                            const int k = c + q + i * lpc;
                            if (k < kend) acc += a[(lane + q) * TPF + i] * scratch[k];
                        }
                    if (c < t.last) {
                        const int64_t xi = int64_t(t.c0) + c;
                        expect(xi >= 0 && xi < n, "x store", xi, n, bk, st, wv, lane);
                        x[xi] = acc;
                        const int64_t o = int64_t(t.lds_x) + c;
                        expect(o >= 0 && o < shb, "LDS shared write (x)", o, shb, bk, st, wv, lane);
                        sh[o] = acc;
                        sh_step[o] = st;
                    }
                }
            }
        }
    }
    double err = 0.0, mx = 0.0;
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!(std::fabs(x[i] - x_ref[i]) <= 1e-12 * (std::fabs(x_ref[i]) + 1e-300))) bad++;
        err = std::fmax(err, std::fabs(x[i] - x_ref[i]));
        mx = std::fmax(mx, std::fabs(x_ref[i]));
    }
    std::printf("max |x_replay - x_plain| = %.3e (max |x| %.3e), %lld entries off by more than 1e-12 relative\n",
                err, mx, (long long)bad);
    std::printf("%lld out-of-range accesses\n", (long long)n_fail);
    return (n_fail == 0 && !(err > 1e-12 * mx) && std::isfinite(err)) ? 0 : 1;
}

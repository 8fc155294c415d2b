// HIP kernels (gfx950) of the R-MATEX hot path.
//
//  * Substitution pair (Alg. 1, the step w = X1^-1 (X2 v_j) with X1 = C + gamma G,
//    X2 = C, Sec. 3.3.2): level-scheduled sweeps over the supernodal factor.
//    Forward, supernode s: btilde = b_s - (updates pushed by descendants),
//    [y_s ; delta_s] = W_s btilde, with W_s = [L11^-1 ; L21 L11^-1]. Each
//    lane owns a panel row, so for a fixed column k a wavefront reads 64
//    consecutive doubles; four wavefronts split k and meet in LDS. delta_s goes
//    to private update slots, read back by the ancestor: no atomics, the
//    summation order is fixed. Backward: x_s = W_s^T [y_s ; -x(off rows)], one
//    wavefront per column (contiguous in memory), reduced across lanes.
//  * Gram-Schmidt (Alg. 1, the inner loop): classical Gram-Schmidt applied
//    twice (same basis and Hessenberg matrix as the modified form up to
//    rounding, with two grid-wide reductions instead of one per vector).
//    Reductions finish in the last block to arrive, in a fixed order.
//  * Small dense part (Eq. 9 and the estimate of Sec. 3.3.3): one workgroup
//    per check offset tau forms H_m = (I - Ht_m^-1)/gamma, evaluates
//    e^{tau H_m} by the degree-18 Taylor polynomial with scaling and
//    squaring (no linear solve), and the error estimate; the last workgroup
//    decides. The adjoint's augmented exponentials use the [13/13] Pade
//    approximant with scaling and squaring (Higham 2005).
//  * Reconstruction (Alg. 1 last line, Alg. 2 snapshot reuse):
//    y(t_a + tau) = beta V_m e^{tau H_m} e1 + y0 + tau z1 - z2.
#include "kernels.hpp"

#include <cmath>

#include "device_common.hpp"
#include "factor.hpp"

namespace matex {

namespace {

using namespace dev;

// ---------------------------------------------------------------- sweeps

// Panel entries each thread has in flight ahead of the ones it multiplies.
constexpr int PF = 4;

// Forward, panels with more than 64 rows: one block per ROWS panel rows of a
// supernode, KS = 256 / ROWS column slices per row. The block issues its
// first panel entries, then assembles btilde over the supernode's columns
// (b minus the children's updates, each position's contributor list in child
// order) and the children's updates on its own off rows, then multiplies
// and sums the column slices in LDS. lds: lds_nc + 256 + ROWS doubles.
template <int ROWS>
__global__ __launch_bounds__(256) void k_forward(const PTask* __restrict__ tasks,
                                                 const int32_t* __restrict__ cptr,
                                                 const int32_t* __restrict__ cidx, int32_t lds_nc,
                                                 const int2* __restrict__ fdesc, int32_t slot,
                                                 const double* __restrict__ W,
                                                 const double* __restrict__ b,
                                                 const double* __restrict__ scale,
                                                 double* __restrict__ y, double* upd,
                                                 const int32_t* done)
{
    constexpr int KS = 256 / ROWS;
    const PTask t = tasks[blockIdx.x];
    __shared__ int32_t quit;
    done_stage(done, &quit);
    extern __shared__ double lds[];
    double* bt = lds;
    double* part = lds + lds_nc;
    double* off = part + 256;
    const int lane = threadIdx.x % ROWS, ks = threadIdx.x / ROWS;
    const int row = t.first + lane;
    const int kmax = row >= t.nr ? 0 : (row < t.nc ? row + 1 : t.nc);
    const int64_t ld = dpanel_ld(t.nr);
    const double* wr = W + t.w + row;
    double a[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const int k = ks + q * KS;
        a[q] = k < kmax ? wr[k * ld] : 0.0;
    }
    if (fdesc) {
        // the update slots are known from the block index alone
        const int2* dsc = fdesc + int64_t(blockIdx.x) * slot;
        for (int k = threadIdx.x; k < lds_nc; k += 256) {
            const int2 d = dsc[k];
            const double u0 = d.x >= 0 ? upd[d.x] : 0.0, u1 = d.y >= 0 ? upd[d.y] : 0.0;
            if (k < t.nc) {
                double v = b[t.c0 + k];
                if (scale) v *= scale[t.c0 + k];
                bt[k] = (v - u0) - u1;
            }
        }
        if (threadIdx.x >= 256 - ROWS) {
            const int i = threadIdx.x - (256 - ROWS);
            const int2 d = dsc[lds_nc + i];
            const double u0 = d.x >= 0 ? upd[d.x] : 0.0, u1 = d.y >= 0 ? upd[d.y] : 0.0;
            off[i] = (0.0 + u0) + u1;
        }
    } else {
        for (int k = threadIdx.x; k < t.nc; k += 256) {
            double v = b[t.c0 + k];
            if (scale) v *= scale[t.c0 + k];
            const int j1 = cptr[t.pos + k + 1];
            for (int j = cptr[t.pos + k]; j < j1; ++j) v -= upd[cidx[j]];
            bt[k] = v;
        }
        if (threadIdx.x >= 256 - ROWS) {
            const int i = threadIdx.x - (256 - ROWS), r = t.first + i;
            double v = 0.0;
            if (r >= t.nc && r < t.nr) {
                const int j1 = cptr[t.pos + r + 1];
                for (int j = cptr[t.pos + r]; j < j1; ++j) v += upd[cidx[j]];
            }
            off[i] = v;
        }
    }
    __syncthreads();
    if (quit) return;
    double acc = 0.0;
    for (int k = ks; k < kmax; k += PF * KS) {
        double nx[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int kk = k + (PF + q) * KS;
            nx[q] = kk < kmax ? wr[kk * ld] : 0.0;
        }
        double s[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int kk = k + q * KS;
            s[q] = kk < kmax ? a[q] * bt[kk] : 0.0;
        }
        acc += (s[0] + s[1]) + (s[2] + s[3]);
#pragma unroll
        for (int q = 0; q < PF; ++q) a[q] = nx[q];
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < ROWS && row < t.nr) {
        double v = 0.0;
#pragma unroll 8
        for (int q = 0; q < KS; ++q) v += part[q * ROWS + lane];
        if (row < t.nc) y[t.c0 + row] = v;
        else upd[t.aux + row - t.nc] = off[lane] + v;
    }
}

// Backward, panels with more than 64 rows: one block per 256 / LPC columns
// of a supernode, LPC lanes per column (a column is contiguous, so the lanes
// of a column read consecutive entries). g = [y_s ; -x(off rows)] is staged
// in LDS from the task's first column down. lds: nr doubles.
template <int LPC>
__global__ __launch_bounds__(256) void k_backward(const PTask* __restrict__ tasks,
                                                  const int32_t* __restrict__ rows,
                                                  const int32_t* __restrict__ gsrc, int32_t slot,
                                                  const double* __restrict__ W,
                                                  const double* __restrict__ y, double* x,
                                                  const int32_t* done)
{
    const PTask t = tasks[blockIdx.x];
    __shared__ int32_t quit;
    done_stage(done, &quit);
    extern __shared__ double g[];
    const int q = threadIdx.x % LPC;
    const int col = t.first + threadIdx.x / LPC;
    const int kend = col < t.nc ? t.nr : 0;
    const double* wc = W + t.w + int64_t(col) * dpanel_ld(t.nr);
    double a[PF];
#pragma unroll
    for (int p = 0; p < PF; ++p) {
        const int k = col + q + p * LPC;
        a[p] = k < kend ? wc[k] : 0.0;
    }
    if (gsrc) {
        // the sources of g are known from the block index alone
        const int32_t* gs = gsrc + int64_t(blockIdx.x) * slot;
        for (int i = threadIdx.x; i < slot; i += 256) {
            const int r = gs[i];
            if (r != INT32_MIN) {
                const double v = r >= 0 ? -x[r] : y[-1 - r];
                g[t.first + i] = v;
            }
        }
    } else {
        for (int k = t.first + threadIdx.x; k < t.nr; k += 256)
            g[k] = k < t.nc ? y[t.c0 + k] : -x[rows[t.aux + k - t.nc]];
    }
    __syncthreads();
    if (quit) return;
    double acc = 0.0;
    for (int k = col + q; k < kend; k += PF * LPC) {
        double nx[PF];
#pragma unroll
        for (int p = 0; p < PF; ++p) {
            const int kk = k + (PF + p) * LPC;
            nx[p] = kk < kend ? wc[kk] : 0.0;
        }
        double s[PF];
#pragma unroll
        for (int p = 0; p < PF; ++p) {
            const int kk = k + p * LPC;
            s[p] = kk < kend ? a[p] * g[kk] : 0.0;
        }
        acc += (s[0] + s[1]) + (s[2] + s[3]);
#pragma unroll
        for (int p = 0; p < PF; ++p) a[p] = nx[p];
    }
    acc = group_sum(acc, LPC);
    if (q == 0 && col < t.nc) x[t.c0 + col] = acc;
}

// The bottom levels as whole subtrees, one block of TW wavefronts each. A
// step is one wavefront per work item (items of one level, or of
// independent subtrees); a block barrier separates steps. Everything a
// subtree passes between its own supernodes stays in the block's LDS: the
// forward sweep's update slots of non-root supernodes and, in the backward
// sweep, every supernode's x (read as off rows by its descendants). Only the
// subtree roots' update slots (read by the level above) and y, x go to
// global memory. The block copies its items to LDS first; each wavefront
// then issues the next step's global loads (panel entries, right-hand side,
// contributor descriptors) before the barrier that ends the current step.
// LDS: items, TW wave scratch regions of ws doubles, the shared region.

// Up to TPF panel entries per lane are loaded ahead (all of them for panels
// of at most TPF columns / for TPF rows per lane in the backward sweep).
constexpr int TPF = 16;

__device__ inline void tree_copy_items(const TItem* __restrict__ src, int n_items, TItem* dst)
{
    const int32_t* s = reinterpret_cast<const int32_t*>(src);
    int32_t* d = reinterpret_cast<int32_t*>(dst);
    constexpr int WORDS = int(sizeof(TItem) / 4);
    for (int i = threadIdx.x; i < n_items * WORDS; i += 64 * TW) d[i] = s[i];
}

struct FwdPre {
    double a[TPF];
    double bv, sv;   // b and scale at column `lane` (multiplied at use)
    int2 d;
};

// Loads are unconditional (out-of-range lanes read a valid clamped address
// and discard it), so the compiler can count them and let a step's loads
// stay in flight while the previous step computes.
__device__ inline void fwd_tree_load(const TItem& t, int lane, const int2* __restrict__ fdesc,
                                     int64_t item, const double* W, const double* b,
                                     const double* scale, FwdPre& p)
{
    const int row = t.first + lane;
    const int kmax = row >= t.last ? 0 : (row < t.nc ? row + 1 : t.nc);
    const int64_t ld = dpanel_ld(t.nr);
    const double* wr = W + t.w + (row < t.last ? row : t.first);
#pragma unroll
    for (int q = 0; q < TPF; ++q) p.a[q] = wr[(q < kmax ? q : 0) * ld];
    const int col = t.c0 + (lane < t.nc ? lane : 0);
    p.bv = b[col];
    p.sv = scale ? scale[col] : 1.0;
    p.d = fdesc[item * 64 + lane];
}

// Sum of the (up to two) LDS slots a descriptor names: offset + 1 in each
// 16-bit half, 0 for none.
__device__ inline double desc_sum(int32_t d, const double* sh)
{
    double v = 0.0;
    const int o0 = d & 0xffff, o1 = (d >> 16) & 0xffff;
    if (o0) v += sh[o0 - 1];
    if (o1) v += sh[o1 - 1];
    return v;
}

// One forward step of a wavefront: item t with its loaded values p.
__device__ inline void fwd_tree_step(const TItem& t, const FwdPre& p, int lane, double* bt, double* sh,
                                     const double* W, double* y, double* upd)
{
    if (t.nr == 0) return;
    const int row = t.first + lane;
    const bool live = row < t.last;
    const int kmax = !live ? 0 : (row < t.nc ? row + 1 : t.nc);
    // btilde = b minus the children's updates; the off row's updates
    if (lane < t.nc) bt[lane] = p.bv * p.sv - desc_sum(p.d.x, sh);
    const double off = live && row >= t.nc ? desc_sum(p.d.y, sh) : 0.0;
    wave_sync();
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < TPF; ++q) acc += q < kmax ? p.a[q] * bt[q] : 0.0;
    if (kmax > TPF) {
        const int64_t ld = dpanel_ld(t.nr);
        const double* wr = W + t.w + row;
        for (int k = TPF; k < kmax; ++k) acc += wr[k * ld] * bt[k];
    }
    if (live) {
        if (row < t.nc) {
            y[t.c0 + row] = acc;
        } else {
            const double v = off + acc;
            if (t.lds_u >= 0) sh[t.lds_u + row - t.nc] = v;
            else upd[t.aux + row - t.nc] = v;
        }
    }
}

// Steps run in pairs on two register sets, so a step's loads stay in
// flight across the previous step's barrier.
__global__ __launch_bounds__(64 * TW) void k_forward_tree(TreeTasks tr, const double* __restrict__ W,
                                                         const double* __restrict__ b,
                                                         const double* __restrict__ scale,
                                                         double* __restrict__ y, double* upd,
                                                         const int32_t* done)
{
    const int s0 = tr.fblk[blockIdx.x], s1 = tr.fblk[blockIdx.x + 1];
    __shared__ int32_t quit;
    done_stage(done, &quit);
    extern __shared__ double lds[];
    TItem* items = reinterpret_cast<TItem*>(lds);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double* bt = lds + tr.item_doubles + wv * tr.ws;
    double* sh = lds + tr.item_doubles + TW * tr.ws;
    // every wavefront copies its share of the items: none may return before
    tree_copy_items(tr.fitems + int64_t(s0) * TW, (s1 - s0) * TW, items);
    __syncthreads();
    if (quit) return;
    auto item = [&](int s) -> const TItem& { return items[(s - s0) * TW + wv]; };
    FwdPre pa, pb;
    fwd_tree_load(item(s0), lane, tr.fdesc, int64_t(s0) * TW + wv, W, b, scale, pa);
    // the loads for the step after the last repeat the last step's (unused)
    for (int s = s0;; s += 2) {
        const int s_b = s + 1 < s1 ? s + 1 : s1 - 1;
        fwd_tree_load(item(s_b), lane, tr.fdesc, int64_t(s_b) * TW + wv, W, b, scale, pb);
        fwd_tree_step(item(s), pa, lane, bt, sh, W, y, upd);
        __syncthreads();
        if (s + 1 >= s1) break;
        const int s_a = s + 2 < s1 ? s + 2 : s1 - 1;
        fwd_tree_load(item(s_a), lane, tr.fdesc, int64_t(s_a) * TW + wv, W, b, scale, pa);
        fwd_tree_step(item(s + 1), pb, lane, bt, sh, W, y, upd);
        __syncthreads();
        if (s + 2 >= s1) break;
    }
}

// Backward: the items of a step are column groups [first, last) of one
// supernode, lpc lanes per column (lpc the largest power of two with
// (last - first) * lpc <= 64; at most TPF rows per lane). g = [y ; -x(off
// rows)] is staged per wavefront; x of an ancestor inside the subtree comes
// from LDS (trow < 0), other values are loaded ahead.
struct BwdPre {
    double a[TPF];
    double gv[TREE_MAX_NR / 64];
    int32_t tr[TREE_MAX_NR / 64];
};

__device__ inline void bwd_tree_load(const TItem& t, int lane, const int32_t* __restrict__ trow,
                                     const double* W, const double* y, const double* x, BwdPre& p)
{
    // off-row indices first: the x loads below wait for them only
    const int noff = t.nr - t.nc;
#pragma unroll
    for (int i = 0; i < TREE_MAX_NR / 64; ++i) {
        const int k = t.first + lane + 64 * i;
        const int o = k - t.nc;
        p.tr[i] = trow[t.aux + (o >= 0 && o < noff ? o : 0)];
    }
    const int cols = t.last - t.first;
    const int shf = cols > 1 ? 32 - __clz(cols - 1) : 0;
    const int lpc = 64 >> shf;
    const int c = t.first + (lane >> (6 - shf)), q = lane & (lpc - 1);
    const int kend = c < t.last ? t.nr : 0;
    const double* wc = W + t.w + int64_t(c < t.last ? c : t.first) * dpanel_ld(t.nr);
#pragma unroll
    for (int i = 0; i < TPF; ++i) {
        const int k = c + q + i * lpc;
        p.a[i] = wc[k < kend ? k : 0];
    }
#pragma unroll
    for (int i = 0; i < TREE_MAX_NR / 64; ++i) {
        const int k = t.first + lane + 64 * i;
        const bool own = k < t.nc;
        const double* src = own ? y + t.c0 + k : x + (p.tr[i] >= 0 ? p.tr[i] : 0);
        p.gv[i] = *src;   // y, or x of an off row (negated at use)
        if (k >= t.nr || own) p.tr[i] = 0;
    }
}

__device__ inline void bwd_tree_step(const TItem& t, const BwdPre& p, int lane, double* g, double* sh,
                                     double* x)
{
    if (t.nr == 0) return;
#pragma unroll
    for (int i = 0; i < TREE_MAX_NR / 64; ++i) {
        const int k = t.first + lane + 64 * i;
        if (k < t.nr) g[k] = p.tr[i] < 0 ? -sh[-1 - p.tr[i]] : (k < t.nc ? p.gv[i] : -p.gv[i]);
    }
    wave_sync();
    const int cols = t.last - t.first;
    const int shf = cols > 1 ? 32 - __clz(cols - 1) : 0;
    const int lpc = 64 >> shf;
    const int c = t.first + (lane >> (6 - shf)), q = lane & (lpc - 1);
    const int kend = c < t.last ? t.nr : 0;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < TPF; ++i) {
        const int k = c + q + i * lpc;
        acc += k < kend ? p.a[i] * g[k] : 0.0;
    }
    acc = group_sum(acc, lpc);
    if (q == 0 && c < t.last) {
        x[t.c0 + c] = acc;
        sh[t.lds_x + c] = acc;
    }
}

__global__ __launch_bounds__(64 * TW) void k_backward_tree(TreeTasks tr, const double* __restrict__ W,
                                                          const double* __restrict__ y, double* x,
                                                          const int32_t* done)
{
    const int s0 = tr.bblk[blockIdx.x], s1 = tr.bblk[blockIdx.x + 1];
    __shared__ int32_t quit;
    done_stage(done, &quit);
    extern __shared__ double lds[];
    TItem* items = reinterpret_cast<TItem*>(lds);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double* g = lds + tr.item_doubles + wv * tr.ws;
    double* sh = lds + tr.item_doubles + TW * tr.ws;
    // every wavefront copies its share of the items: none may return before
    tree_copy_items(tr.bitems + int64_t(s0) * TW, (s1 - s0) * TW, items);
    __syncthreads();
    if (quit) return;
    auto item = [&](int s) -> const TItem& { return items[(s - s0) * TW + wv]; };
    BwdPre pa, pb;
    bwd_tree_load(item(s0), lane, tr.trow, W, y, x, pa);
    for (int s = s0;; s += 2) {
        bwd_tree_load(item(s + 1 < s1 ? s + 1 : s1 - 1), lane, tr.trow, W, y, x, pb);
        bwd_tree_step(item(s), pa, lane, g, sh, x);
        __syncthreads();
        if (s + 1 >= s1) break;
        bwd_tree_load(item(s + 2 < s1 ? s + 2 : s1 - 1), lane, tr.trow, W, y, x, pa);
        bwd_tree_step(item(s + 1), pb, lane, g, sh, x);
        __syncthreads();
        if (s + 2 >= s1) break;
    }
}

// ------------------------------------------------------- reductions helpers

// ---------------------------------------------------------- Gram-Schmidt


// Blocks of GS_THREADS threads (RED_BLOCKS of them at most), so the rows of
// a 10^5-node vector are all in flight at once; partials of a pass,
// [RED_BLOCKS][NVMAX + 1].
constexpr int GS_THREADS = 1024, GS_WAVES = GS_THREADS / 64;

// Values per wavefront in the value-major reductions: value i (a basis
// vector, or slot nv for the squared norm) belongs to wavefront i mod GS_WAVES.
constexpr int GS_VPW = (NVMAX + 1 + GS_WAVES - 1) / GS_WAVES;

// Dot products over one tile of GS_THREADS rows staged in LDS (wl): acc[q]
// += sum_t wl[t] * V_i[base + t] for the wavefront's values i < nv, and
// wl[t]^2 for i == nv when `norm`. Lanes take rows lane, lane + 64, ...
__device__ inline void gs_tile_dots(const double* V, int64_t ldv, int nv, bool norm, int64_t base,
                                    int rows, const double* wl, double (&acc)[GS_VPW])
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < GS_VPW; ++q) {
        const int i = wv + q * GS_WAVES;
        if (i < nv) {
            const double* Vi = V + int64_t(i) * ldv + base;
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < GS_THREADS / 64; ++k) {
                const int t = lane + 64 * k;
                if (t < rows) s += wl[t] * Vi[t];
            }
            acc[q] += s;
        } else if (norm && i == nv) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < GS_THREADS / 64; ++k) {
                const int t = lane + 64 * k;
                if (t < rows) s += wl[t] * wl[t];
            }
            acc[q] += s;
        }
    }
}

// The wavefront sums of acc into partial[blockIdx.x][i], i < cnt.
__device__ inline void gs_store_partials(const double (&acc)[GS_VPW], int cnt, double* partial)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < GS_VPW; ++q) {
        const int i = wv + q * GS_WAVES;
        if (i < cnt) {
            const double t = wave_sum(acc[q]);
            if (lane == 0) partial[int64_t(blockIdx.x) * (NVMAX + 1) + i] = t;
        }
    }
}

__global__ __launch_bounds__(GS_THREADS) void k_gs_dots(int64_t n, const double* __restrict__ V,
                                                        int64_t ldv, int nv,
                                                        const double* __restrict__ w,
                                                        double* partial, const int32_t* done)
{
    __shared__ int32_t quit;
    done_stage(done, &quit);
    __shared__ double wl[GS_THREADS];
    double acc[GS_VPW];
#pragma unroll
    for (int q = 0; q < GS_VPW; ++q) acc[q] = 0.0;
    for (int64_t base = int64_t(blockIdx.x) * GS_THREADS; base < n; base += int64_t(gridDim.x) * GS_THREADS) {
        const int64_t r = base + threadIdx.x;
        wl[threadIdx.x] = r < n ? w[r] : 0.0;
        __syncthreads();
        if (quit) return;
        gs_tile_dots(V, ldv, nv, false, base, int(min<int64_t>(GS_THREADS, n - base)), wl, acc);
        __syncthreads();
    }
    gs_store_partials(acc, nv, partial);
}

// Every block sums the previous kernel's partials itself (fixed order), so no
// cross-block publication is needed inside a kernel. h1 = sum of pass-1
// partials; w' = w - V h1 in place; pass-2 partials V^T w' and ||w'||^2
// (slot nv) into partial_out.
__global__ __launch_bounds__(GS_THREADS) void k_gs_update(int64_t n, const double* __restrict__ V,
                                                          int64_t ldv, int nv, double* w,
                                                          const double* partial_in, double* partial_out,
                                                          KState* ks, const int32_t* done)
{
    __shared__ int32_t quit;
    done_stage(done, &quit);
    __shared__ double h[NVMAX + 1];
    __shared__ double wl[GS_THREADS];
    reduce_partials_waves<GS_WAVES>(partial_in, NVMAX + 1, gridDim.x, nv, h);
    if (quit) return;
    if (blockIdx.x == 0 && threadIdx.x < nv) ks->h1[threadIdx.x] = h[threadIdx.x];
    double acc[GS_VPW];
#pragma unroll
    for (int q = 0; q < GS_VPW; ++q) acc[q] = 0.0;
    for (int64_t base = int64_t(blockIdx.x) * GS_THREADS; base < n; base += int64_t(gridDim.x) * GS_THREADS) {
        const int64_t r = base + threadIdx.x;
        double wr = 0.0;
        if (r < n) {
            wr = w[r];
#pragma unroll 8
            for (int i = 0; i < nv; ++i) wr -= h[i] * V[r + i * ldv];
            w[r] = wr;
        }
        wl[threadIdx.x] = wr;
        __syncthreads();
        gs_tile_dots(V, ldv, nv, true, base, int(min<int64_t>(GS_THREADS, n - base)), wl, acc);
        __syncthreads();
    }
    gs_store_partials(acc, nv + 1, partial_out);
}

// w'' = w' - V h2, ||w''||^2 = ||w'||^2 - ||h2||^2 (w' is already orthogonal
// to working precision after the first pass, so there is no cancellation);
// v_{j+1} = w'' / ||w''||, and column j of Ht = h1 + h2 with Ht(j+1,j) = ||w''||.
// Every block sums the pass-2 partials itself; block 0 records the column.
// The iteration's ticket: one more than the last one published (every
// k_gs_finish launch publishes exactly once, so the count is the number of
// iterations launched on this state, which the host counts too).
__device__ inline void publish_ticket(KState* ks)
{
    __hip_atomic_store(&ks->ticket, ks->ticket + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(GS_THREADS) void k_gs_finish(int64_t n, double* V, int64_t ldv, int nv,
                                                   const double* __restrict__ w,
                                                   const double* partial_in, KState* ks,
                                                   const int32_t* done)
{
    __shared__ int32_t quit;
    done_stage(done, &quit);
    __shared__ double h[NVMAX + 1];
    __shared__ double sc;
    reduce_partials_waves<GS_WAVES>(partial_in, NVMAX + 1, gridDim.x, nv + 1, h);
    if (quit) {
        if (blockIdx.x == 0 && threadIdx.x == 0) publish_ticket(ks);
        return;
    }
    if (threadIdx.x == 0) {
        double s2 = 0.0, hmax = 0.0;
        for (int i = 0; i < nv; ++i) {
            s2 += h[i] * h[i];
            hmax = fmax(hmax, fabs(ks->h1[i] + h[i]));
        }
        const double beta = sqrt(fmax(h[nv] - s2, 0.0));
        // happy breakdown: the space is invariant, the result is exact
        const bool brk = !(beta > 1e-14 * hmax);
        sc = brk ? 0.0 : 1.0 / beta;
        if (blockIdx.x == 0) {
            const int j = nv - 1;
            for (int i = 0; i < nv; ++i) ks->Ht[i + j * (MAXM + 1)] = ks->h1[i] + h[i];
            ks->Ht[nv + j * (MAXM + 1)] = beta;
            ks->m = nv;
            ks->breakdown = brk ? 1 : 0;
            ks->brk[j] = brk ? 1 : 0;
            publish_ticket(ks);
        }
    }
    __syncthreads();
    const double inv = sc;
    double* vout = V + int64_t(nv) * ldv;
    for (int64_t r = int64_t(blockIdx.x) * GS_THREADS + threadIdx.x; r < n; r += int64_t(gridDim.x) * GS_THREADS) {
        double wr = w[r];
#pragma unroll 8
        for (int i = 0; i < nv; ++i) wr -= h[i] * V[r + i * ldv];
        vout[r] = wr * inv;
    }
}

// The waiting lane sleeps between polls of the ticket; the wait ends at the
// ticket or at the clock limit, whichever comes first.
__global__ __launch_bounds__(64) void k_wait_ticket(KState* ks, int32_t ticket, int64_t max_ticks)
{
    if (threadIdx.x != 0) return;
    const int64_t t0 = int64_t(wall_clock64());
    while (true) {
        const int32_t t = __hip_atomic_load(&ks->ticket, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (int32_t(uint32_t(t) - uint32_t(ticket)) >= 0) return;
        if (int64_t(wall_clock64()) - t0 > max_ticks) {
            ks->wait_err = 1;
            ks->converged = 0;
            __hip_atomic_store(&ks->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

// ------------------------------------------------------- small dense part

// One block per check offset.
__global__ __launch_bounds__(256) void k_checks(KState* ks, double gamma,
                                                const double* __restrict__ taus,
                                                const int32_t* __restrict__ sel, int n_sel,
                                                double tol, double* u_buf, double* est_buf,
                                                int m_max, int update_state, int m_arg)
{
    if (update_state && ks->done) return;
    extern __shared__ double sm[];
    const int c = sel ? sel[blockIdx.x] : int(blockIdx.x);
    const int m = m_arg >= 0 ? m_arg : ks->m;
    const int brk = m_arg >= 0 ? (m > 0 ? ks->brk[m - 1] : 0) : ks->breakdown;
    check_block(ks, m, brk, gamma, taus, c, sel, n_sel, tol, u_buf, est_buf, m_max, update_state, sm);
}

// z1 += sum_c coef[c] Z1[:, q[c]], z2 likewise (columns of n, in the order of c).
__global__ void k_spot_update(int64_t n, int cnt, const int32_t* __restrict__ q,
                              const double* __restrict__ coef, const double* __restrict__ Z1,
                              const double* __restrict__ Z2, double* z1, double* z2)
{
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        double a = z1[i], b = z2[i];
        for (int c = 0; c < cnt; ++c) {
            const int64_t o = int64_t(q[c]) * n + i;
            a += coef[c] * Z1[o];
            b += coef[c] * Z2[o];
        }
        z1[i] = a;
        z2[i] = b;
    }
}

__global__ __launch_bounds__(256) void k_spot_setup(int64_t n, SpotArgs sa, const double* __restrict__ Z1,
                                                    const double* __restrict__ Z2, double* z1, double* z2,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ y0, double* v,
                                                    double* partial, double* taus, TauArgs ta)
{
    if (blockIdx.x == 0 && threadIdx.x < ta.n) taus[threadIdx.x] = ta.t[threadIdx.x];
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < n; r += int64_t(gridDim.x) * 256) {
        double b = z2[r];
        if (sa.cnt > 0) {
            double a = z1[r];
            for (int c = 0; c < sa.cnt; ++c) {
                const int64_t o = int64_t(sa.q[c]) * n + r;
                a += sa.coef[c] * Z1[o];
                b += sa.coef[c] * Z2[o];
            }
            z1[r] = a;
            z2[r] = b;
        }
        const double t = y[r] - y0[r] + b;
        v[r] = t;
        acc += t * t;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void k_set_m(KState* ks, int m)
{
    ks->m = m;
    ks->breakdown = m > 0 ? ks->brk[m - 1] : 0;
}

// ------------------------------------------------------ segment set-up

__global__ __launch_bounds__(256) void k_setup_v(int64_t n, const double* __restrict__ y,
                                                 const double* __restrict__ y0,
                                                 const double* __restrict__ z2, double* v,
                                                 double* partial)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < n; r += int64_t(gridDim.x) * 256) {
        const double t = y[r] - y0[r] + z2[r];
        v[r] = t;
        acc += t * t;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// beta = ||v|| (every block sums the partials), v_1 = v / beta; block 0
// resets the Krylov state for a new basis.
__global__ __launch_bounds__(256) void k_normalize_v(int64_t n, double* v, const double* partial,
                                                     int nblk, KState* ks)
{
    __shared__ double red[4];
    __shared__ double sb;
    const double mine = int(threadIdx.x) < nblk ? partial[threadIdx.x] : 0.0;
    const double t = block_sum(mine, red);
    if (threadIdx.x == 0) {
        sb = sqrt(t);
        if (blockIdx.x == 0) {
            ks->beta = sb;
            ks->m = 0;
            ks->mdec = 0;
            ks->breakdown = 0;
            ks->converged = sb == 0.0 ? 1 : 0;
            ks->done = sb == 0.0 ? 1 : 0;
            ks->est = 0.0;
        }
    }
    __syncthreads();
    const double beta = sb;
    if (beta == 0.0) return;
    const double inv = 1.0 / beta;
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < n; r += int64_t(gridDim.x) * 256)
        v[r] *= inv;
}

__global__ void k_scatter_add(int32_t count, const int32_t* idx, const double* val, double* dst)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) dst[idx[k]] += val[k];
}

__global__ __launch_bounds__(256) void k_recon_probes(int n_probe, const int32_t* probe_perm,
                                                      int n_snap, int32_t snap0,
                                                      const double* __restrict__ tau,
                                                      const double* __restrict__ u,
                                                      const KState* ks, const double* V,
                                                      int64_t ldv, const double* y0,
                                                      const double* z1, const double* z2,
                                                      double* out, int32_t n_out)
{
    const int64_t id = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (id >= int64_t(n_probe) * n_snap) return;
    const int p = int(id % n_probe), sidx = int(id / n_probe);
    const int r = probe_perm[p];
    const int m = ks->m;
    double acc = 0.0;
    if (m > 0) {
        const double* us = u + sidx * MAXM;
        for (int k = 0; k < m; ++k) acc += V[r + k * ldv] * us[k];
        acc *= ks->beta;
    }
    const double t = tau[sidx];
    out[int64_t(p) * n_out + snap0 + sidx] += acc + y0[r] + t * z1[r] - z2[r];
}

__global__ __launch_bounds__(256) void k_recon_full(int64_t n, double tau,
                                                    const double* __restrict__ u,
                                                    const KState* ks, const double* V,
                                                    int64_t ldv, double* y, double* y0,
                                                    const double* z1, const double* z2)
{
    const int m = ks->m;
    const double beta = ks->beta;
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < n; r += int64_t(gridDim.x) * 256) {
        double acc = 0.0;
        if (m > 0) {
            for (int k = 0; k < m; ++k) acc += V[r + k * ldv] * u[k];
            acc *= beta;
        }
        const double a = y0[r], b = z1[r];
        y[r] = acc + a + tau * b - z2[r];
        y0[r] = a + tau * b;
    }
}

__global__ void k_axpy(int64_t n, double a, const double* x, double* y)
{
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < n; r += int64_t(gridDim.x) * 256)
        y[r] += a * x[r];
}

// dst[k, c] = src[perm[k], c]
__global__ void k_gather_perm(int64_t n, const int32_t* perm, const double* src, double* dst,
                              int64_t lds_, int64_t ldd, int ncols)
{
    const int c = blockIdx.y;
    for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n; k += int64_t(gridDim.x) * 256)
        dst[k + c * ldd] = src[perm[k] + c * lds_];
}

// dst[perm[k], c] = src[k, c]
__global__ void k_scatter_perm(int64_t n, const int32_t* perm, const double* src, double* dst,
                               int64_t lds_, int64_t ldd, int ncols)
{
    const int c = blockIdx.y;
    for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n; k += int64_t(gridDim.x) * 256)
        dst[perm[k] + c * ldd] = src[k + c * lds_];
}

// ---------------------------------------------------- trapezoidal rule

// Unit trapezoidal pulse at t (fs): 0 up to the delay, a linear rise, the
// flat top, a linear fall, 0 afterwards (one period).
__device__ inline double unit_pulse(int64_t t, int64_t d, int64_t r, int64_t w, int64_t f)
{
    if (t > d && t <= d + r) return double(t - d) / double(r);
    if (t > d + r && t <= d + r + w) return 1.0;
    if (t > d + r + w && t < d + r + w + f) return 1.0 - double(t - d - r - w) / double(f);
    return 0.0;
}

// Right-hand side of one trapezoidal step (Eq. 2 times h): rhs = C y - (h/2) G y
// + (h/2) (i(t0) + i(t1)), every row in the factor's order; the sources of
// row r are sptr[r] .. sptr[r + 1] (in a fixed order).
__global__ void k_tr_rhs(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                         const double* __restrict__ gv, const double* __restrict__ cperm,
                         const double* __restrict__ y, double hh, int64_t t0, int64_t t1,
                         const int32_t* __restrict__ sptr, const double* __restrict__ amp,
                         const int64_t* __restrict__ sd, const int64_t* __restrict__ sr,
                         const int64_t* __restrict__ sw, const int64_t* __restrict__ sf, double* rhs)
{
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        double gy = 0.0;
        for (int q = rp[i]; q < rp[i + 1]; ++q) gy += gv[q] * y[ci[q]];
        double src = 0.0;
        for (int k = sptr[i]; k < sptr[i + 1]; ++k)
            src += amp[k] * (unit_pulse(t0, sd[k], sr[k], sw[k], sf[k]) + unit_pulse(t1, sd[k], sr[k], sw[k], sf[k]));
        rhs[i] = (cperm[i] * y[i] - hh * gy) + hh * src;
    }
}

// out[p * n_out + col] = y[probe_perm[p]]
__global__ void k_gather_probes(int n_probe, const int32_t* __restrict__ probe_perm, const double* __restrict__ y,
                                double* out, int32_t n_out, int32_t col)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < n_probe) out[int64_t(p) * n_out + col] = y[probe_perm[p]];
}

__global__ void k_flag_nonfinite(int64_t count, const double* __restrict__ a, int32_t* flag)
{
    bool bad = false;
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < count; r += int64_t(gridDim.x) * 256)
        bad |= !isfinite(a[r]);
    if (bad) *flag = 1;
}

__global__ void k_vdd_minus(int64_t count, double vdd, double* buf)
{
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < count; r += int64_t(gridDim.x) * 256)
        buf[r] = vdd - buf[r];
}

inline int grid_for(int64_t n) { return int(std::min<int64_t>((n + 255) / 256, RED_BLOCKS)); }
inline int gs_grid(int64_t n) { return int(std::min<int64_t>((n + GS_THREADS - 1) / GS_THREADS, RED_BLOCKS)); }

}  // namespace

void launch_forward(const LevelTasks& lv, const int32_t* cptr, const int32_t* cidx,
                    const double* W, const double* b, const double* scale, double* y, double* upd,
                    const int32_t* done, hipStream_t st)
{
    const size_t lds = sizeof(double) * (size_t(lv.lds_doubles) + 256 + size_t(lv.kind));
    switch (lv.kind) {
    case 4:
        k_forward<4><<<lv.count, 256, lds, st>>>(lv.tasks, cptr, cidx, lv.lds_doubles, lv.fdesc, lv.slot, W, b, scale,
                                                 y, upd, done);
        break;
    case 16:
        k_forward<16><<<lv.count, 256, lds, st>>>(lv.tasks, cptr, cidx, lv.lds_doubles, lv.fdesc, lv.slot, W, b, scale,
                                                  y, upd, done);
        break;
    default:
        k_forward<64><<<lv.count, 256, lds, st>>>(lv.tasks, cptr, cidx, lv.lds_doubles, lv.fdesc, lv.slot, W, b, scale,
                                                  y, upd, done);
        break;
    }
}

void launch_backward(const LevelTasks& lv, const int32_t* rows, const double* W, const double* y,
                     double* x, const int32_t* done, hipStream_t st)
{
    const size_t lds = sizeof(double) * size_t(lv.lds_doubles);
    switch (lv.kind) {
    case 16:
        k_backward<16><<<lv.count, 256, lds, st>>>(lv.tasks, rows, lv.gsrc, lv.slot, W, y, x, done);
        break;
    default:
        k_backward<64><<<lv.count, 256, lds, st>>>(lv.tasks, rows, lv.gsrc, lv.slot, W, y, x, done);
        break;
    }
}

void launch_forward_tree(const TreeTasks& tr, const double* W,
                         const double* b, const double* scale, double* y, double* upd,
                         const int32_t* done, hipStream_t st)
{
    if (tr.n_blocks > 0)
        k_forward_tree<<<tr.n_blocks, 64 * TW, sizeof(double) * size_t(tr.lds_doubles), st>>>(
            tr, W, b, scale, y, upd, done);
}

void launch_backward_tree(const TreeTasks& tr, const double* W, const double* y, double* x,
                          const int32_t* done, hipStream_t st)
{
    if (tr.n_blocks > 0)
        k_backward_tree<<<tr.n_blocks, 64 * TW, sizeof(double) * size_t(tr.lds_doubles), st>>>(
            tr, W, y, x, done);
}

void launch_gs_dots(int64_t n, const double* V, int64_t ldv, int nv, const double* w,
                    double* partial, KState* ks, const int32_t* done, hipStream_t st)
{
    (void)ks;
    k_gs_dots<<<gs_grid(n), GS_THREADS, 0, st>>>(n, V, ldv, nv, w, partial, done);
}

void launch_gs_update(int64_t n, const double* V, int64_t ldv, int nv, double* w,
                      double* partial, KState* ks, const int32_t* done, hipStream_t st)
{
    const int64_t half = int64_t(RED_BLOCKS) * (MAXM + 2);
    k_gs_update<<<gs_grid(n), GS_THREADS, 0, st>>>(n, V, ldv, nv, w, partial, partial + half, ks, done);
}

void launch_gs_finish(int64_t n, double* V, int64_t ldv, int nv, const double* w,
                      const double* partial, KState* ks, const int32_t* done, hipStream_t st)
{
    const int64_t half = int64_t(RED_BLOCKS) * (MAXM + 2);
    k_gs_finish<<<gs_grid(n), GS_THREADS, 0, st>>>(n, V, ldv, nv, w, partial + half, ks, done);
}

void launch_wait_ticket(KState* ks, int32_t ticket, int64_t max_ticks, hipStream_t st)
{
    k_wait_ticket<<<1, 64, 0, st>>>(ks, ticket, max_ticks);
}

size_t checks_lds_bytes() { return sizeof(double) * (7 * MAXM * LD + 2 * MAXM); }

void launch_checks(KState* ks, double gamma, const double* tau, const int32_t* sel, int n_sel,
                   double tol, double* u_buf, double* est_buf, int m_max, int update_state,
                   int m_arg, hipStream_t st)
{
    k_checks<<<n_sel, 256, checks_lds_bytes(), st>>>(ks, gamma, tau, sel, n_sel, tol, u_buf, est_buf,
                                                     m_max, update_state, m_arg);
}

void launch_set_m(KState* ks, int m, hipStream_t st) { k_set_m<<<1, 1, 0, st>>>(ks, m); }

// Diagnostics: the device wall clock (100 MHz) when the stream reaches this point.
__global__ void k_stamp(int64_t* buf, int64_t idx) { buf[idx] = int64_t(wall_clock64()); }
void launch_stamp(int64_t* buf, int64_t idx, hipStream_t st) { k_stamp<<<1, 1, 0, st>>>(buf, idx); }

void launch_spot_update(int64_t n, int cnt, const int32_t* q, const double* coef, const double* Z1,
                        const double* Z2, double* z1, double* z2, hipStream_t st)
{
    if (cnt > 0) k_spot_update<<<grid_for(n), 256, 0, st>>>(n, cnt, q, coef, Z1, Z2, z1, z2);
}

// ------------------------------------------------------------- adjoint

// Step integrals of the adjoint (Van Loan 1978): with the (m+2) x (m+2)
// matrix M = [[H, e1, 0], [0, 0, 1], [0, 0, 0]], e^{tau M} holds
// phi1 = int_0^tau e^{sH} e1 ds and phi2 = int_0^tau (tau - s) e^{sH} e1 ds in
// its last two columns. I[0 .. m) = phi1 and I[MAXM .. MAXM + m) =
// tau phi1 - phi2 = int_0^tau s e^{sH} e1 ds. Needs m <= MAXM - 2.
__global__ __launch_bounds__(256) void k_adj_integrals(const KState* ks, double gamma, double tau,
                                                       double* I)
{
    extern __shared__ double sm[];
    double* H = sm;
    double* buf = H + MAXM * LD;
    const int m = ks->m;
    if (m == 0) {
        for (int i = threadIdx.x; i < 2 * MAXM; i += blockDim.x) I[i] = 0.0;
        return;
    }
    form_h(ks, m, gamma, H, buf);
    const int N = m + 2;
    for (int idx = threadIdx.x; idx < N * LD; idx += blockDim.x) {
        const int i = idx / LD, j = idx % LD;
        if (i < m && j < m) continue;
        double v = 0.0;
        if (i == 0 && j == m) v = 1.0;
        if (i == m && j == m + 1) v = 1.0;
        H[idx] = v;
    }
    __syncthreads();
    const double* R = expm_mat(H, N, tau, buf);
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double p1 = R[i * LD + m], p2 = R[i * LD + m + 1];
        I[i] = p1;
        I[MAXM + i] = tau * p1 - p2;
    }
}

// Amplitude gradients over one adjoint step [t_hi - dt, t_hi] (fs), inside
// which every pulse is linear: with sigma = t_hi - t, u_k = alpha + beta sigma
// and lambda(t_hi - sigma) = b V e^{sigma H} e1, so
// int u_k lambda_{n_k} dt = b V[row_k, :] (alpha I0 + beta I1).
__global__ void k_adj_amp(int n_src, const int32_t* __restrict__ row, const int64_t* __restrict__ delay,
                          const int64_t* __restrict__ rise, const int64_t* __restrict__ width,
                          const int64_t* __restrict__ fall, int64_t t_hi, int64_t dt,
                          const double* __restrict__ V, int64_t ldv, const KState* ks,
                          const double* __restrict__ I, double lscale, double* grad)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_src) return;
    const int m = ks->m;
    if (m == 0) return;
    const int64_t d = delay[k], r = rise[k], w = width[k], f = fall[k];
    // value at t_hi and slope (per fs) on the step, from its midpoint's piece
    auto val = [&](int64_t t) -> double {
        if (t <= d) return 0.0;
        if (t < d + r) return double(t - d) / double(r);
        if (t <= d + r + w) return 1.0;
        if (t < d + r + w + f) return 1.0 - double(t - d - r - w) / double(f);
        return 0.0;
    };
    const double tm = double(t_hi) - 0.5 * double(dt);
    double slope = 0.0;
    if (tm > double(d) && tm < double(d + r)) slope = 1.0 / double(r);
    else if (tm > double(d + r + w) && tm < double(d + r + w + f)) slope = -1.0 / double(f);
    const double alpha = val(t_hi);
    const double beta = -slope * 1e15;   // d u / d sigma, per second
    if (alpha == 0.0 && beta == 0.0) return;
    const int64_t o = row[k];
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc += V[int64_t(j) * ldv + o] * (alpha * I[j] + beta * I[MAXM + j]);
    grad[k] += lscale * ks->beta * acc;
}

// lambda += C^-1 g at a sample time: g = -dJ/dx at the probes. The probes
// are grouped by row (rows[q], their probe indices pidx[ptr[q] .. ptr[q+1])),
// summed in a fixed order.
__global__ void k_adj_jump(int n_rows, const int32_t* __restrict__ rows, const int32_t* __restrict__ ptr,
                           const int32_t* __restrict__ pidx, const double* __restrict__ dJdx,
                           int64_t n_out, int s, const double* __restrict__ cperm, double inv_scale,
                           double* lam)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_rows) return;
    double g = 0.0;
    for (int e = ptr[q]; e < ptr[q + 1]; ++e) g -= dJdx[int64_t(pidx[e]) * n_out + s];
    lam[rows[q]] += g / cperm[rows[q]] * inv_scale;
}

// Capacitance gradient, integrated by parts:
//   dJ/dc_i = (1/c_i) (-sum_s g_{s,i} y_i(t_s) + int (G lambda)_i y_i dt),
// so only values of the forward droop y are needed (no derivative of its
// Krylov approximation). One overlap [t1, t2] of an adjoint step
// (lambda(t) = beta_l V_l e^{(t_hi - t) H_l} e1) and a forward segment
// (y(t) = beta_f V_f e^{(t - t_a) H_f} e1 + y0 + (t - t_a) z1 - z2) needs, with
// h = t2 - t1, a = e^{(t_hi - t2) H_l} e1, b = e^{(t1 - t_a) H_f} e1, s = t - t1:
//   W  = int (e^{(t_hi-t) H_l} e1)(e^{(t-t_a) H_f} e1)^T dt
//   q0 = int e^{(t_hi-t) H_l} e1 dt,  q1 = int (t - t_a) e^{(t_hi-t) H_l} e1 dt.
// All three are the top-right block of exp(h T), T = [[A, B], [0, D]] with
// A = H_l, B = [a b^T, a, 0], D = [[H_f^T, 0, 0], [0, 0, 1], [0, 0, 0]]
// (Van Loan 1978): W is its first mf columns, q0 the next, and the last is
// int_0^h s e^{(h-s) H_l} a ds, so q1 = (t1 - t_a) q0 + that. The exponential
// is taken block by block, each block at most MAXM wide in LDS: Taylor's
// series in Horner form on T / 2^s with ||T / 2^s||_1 <= 1/2 (18 terms), then
// s squarings [[Xa, Xb], [0, Xd]]^2 = [[Xa^2, Xa Xb + Xb Xd], [0, Xd^2]].
// Wq: W row-major (stride MAXM), then q0, then q1 (MAXM each).
constexpr int CG_TERMS = 18;

// C (r x c) = A (r x k) B (k x c), or += with acc; row-major stride LD.
__device__ inline void mm_rect(const double* A, const double* B, double* C, int r, int k, int c, bool acc)
{
    for (int idx = threadIdx.x; idx < r * c; idx += blockDim.x) {
        const int i = idx / c, j = idx - (idx / c) * c;
        double s = acc ? C[i * LD + j] : 0.0;
        for (int q = 0; q < k; ++q) s += A[i * LD + q] * B[q * LD + j];
        C[i * LD + j] = s;
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_cg_block(const KState* kl, double gam_l, const KState* kf,
                                                  double gam_f, double sig_b, double tau_a, double h,
                                                  double* Wq)
{
    extern __shared__ double sm[];
    constexpr int BS = MAXM * LD;
    double* blk[7];
    for (int q = 0; q < 7; ++q) blk[q] = sm + q * BS;
    double* va = sm + 7 * BS;
    double* vb = va + MAXM;
    __shared__ double nrm;
    __shared__ int sq;
    const int ml = kl->m, mf = kf->m;   // mf = 0: a forward segment with no Krylov part
    if (ml == 0) {
        for (int i = threadIdx.x; i < MAXM * MAXM + 2 * MAXM; i += blockDim.x) Wq[i] = 0.0;
        return;
    }
    const int na = ml, nd = mf + 2;
    // a and b
    form_h(kl, ml, gam_l, blk[0], blk[1]);
    expm_e1(blk[0], ml, sig_b, blk[1], va);
    if (mf > 0) {
        form_h(kf, mf, gam_f, blk[0], blk[1]);
        expm_e1(blk[0], mf, tau_a, blk[1], vb);
    }
    // A = H_l in blk0, D in blk2 (H_f^T from blk1), B in blk3
    form_h(kl, ml, gam_l, blk[0], blk[1]);
    if (mf > 0) form_h(kf, mf, gam_f, blk[1], blk[4]);
    for (int idx = threadIdx.x; idx < nd * nd; idx += blockDim.x) {
        const int i = idx / nd, j = idx % nd;
        double v = 0.0;
        if (i < mf && j < mf) v = blk[1][j * LD + i];
        else if (i == mf && j == mf + 1) v = 1.0;
        blk[2][i * LD + j] = v;
    }
    for (int idx = threadIdx.x; idx < na * nd; idx += blockDim.x) {
        const int i = idx / nd, j = idx % nd;
        blk[3][i * LD + j] = j < mf ? va[i] * vb[j] : (j == mf ? va[i] : 0.0);
    }
    __syncthreads();
    double* A = blk[0];
    double* D = blk[2];
    double* B = blk[3];
    // scale: ||h T||_1 / 2^s <= 1/2
    if (threadIdx.x == 0) {
        double best = 0.0;
        for (int j = 0; j < na; ++j) {
            double c = 0.0;
            for (int i = 0; i < na; ++i) c += fabs(A[i * LD + j]);
            best = fmax(best, c);
        }
        for (int j = 0; j < nd; ++j) {
            double c = 0.0;
            for (int i = 0; i < na; ++i) c += fabs(B[i * LD + j]);
            for (int i = 0; i < nd; ++i) c += fabs(D[i * LD + j]);
            best = fmax(best, c);
        }
        nrm = best * h;
        sq = (nrm > 0.5 && nrm < 1e300) ? min(int(ceil(log2(nrm / 0.5))), 1100) : 0;
    }
    __syncthreads();
    const double scl = h * ldexp(1.0, -sq);
    for (int idx = threadIdx.x; idx < MAXM * LD; idx += blockDim.x) {
        A[idx] *= scl;
        B[idx] *= scl;
        D[idx] *= scl;
    }
    __syncthreads();
    // Horner: X = I; X = I + (T / k) X for k = CG_TERMS .. 1
    double* Xa = blk[4];
    double* Xb = blk[5];
    double* Xd = blk[6];
    double* T1 = blk[1];
    for (int idx = threadIdx.x; idx < MAXM * LD; idx += blockDim.x) {
        const int i = idx / LD, j = idx % LD;
        Xa[idx] = (i == j) ? 1.0 : 0.0;
        Xd[idx] = (i == j) ? 1.0 : 0.0;
        Xb[idx] = 0.0;
    }
    __syncthreads();
    for (int k = CG_TERMS; k >= 1; --k) {
        const double ik = 1.0 / double(k);
        mm_rect(A, Xb, T1, na, na, nd, false);
        mm_rect(B, Xd, T1, na, nd, nd, true);
        for (int idx = threadIdx.x; idx < na * nd; idx += blockDim.x) {
            const int i = idx / nd, j = idx % nd;
            Xb[i * LD + j] = T1[i * LD + j] * ik;
        }
        __syncthreads();
        mm_rect(A, Xa, T1, na, na, na, false);
        for (int idx = threadIdx.x; idx < na * na; idx += blockDim.x) {
            const int i = idx / na, j = idx % na;
            Xa[i * LD + j] = (i == j ? 1.0 : 0.0) + T1[i * LD + j] * ik;
        }
        __syncthreads();
        mm_rect(D, Xd, T1, nd, nd, nd, false);
        for (int idx = threadIdx.x; idx < nd * nd; idx += blockDim.x) {
            const int i = idx / nd, j = idx % nd;
            Xd[i * LD + j] = (i == j ? 1.0 : 0.0) + T1[i * LD + j] * ik;
        }
        __syncthreads();
    }
    // squarings (A, B, D buffers are free now)
    double* SA = A;
    double* SD = D;
    for (int q = 0; q < sq; ++q) {
        mm_rect(Xa, Xb, T1, na, na, nd, false);
        mm_rect(Xb, Xd, T1, na, nd, nd, true);
        mm_rect(Xa, Xa, SA, na, na, na, false);
        mm_rect(Xd, Xd, SD, nd, nd, nd, false);
        double* t;
        t = Xb; Xb = T1; T1 = t;
        t = Xa; Xa = SA; SA = t;
        t = Xd; Xd = SD; SD = t;
    }
    for (int idx = threadIdx.x; idx < MAXM * MAXM; idx += blockDim.x) {
        const int i = idx / MAXM, j = idx % MAXM;
        Wq[idx] = (i < ml && j < mf) ? Xb[i * LD + j] : 0.0;
    }
    for (int i = threadIdx.x; i < MAXM; i += blockDim.x) {
        const double q0 = i < ml ? Xb[i * LD + mf] : 0.0;
        const double m1 = i < ml ? Xb[i * LD + mf + 1] : 0.0;
        Wq[MAXM * MAXM + i] = q0;
        Wq[MAXM * MAXM + MAXM + i] = tau_a * q0 + m1;
    }
}

// GV[:, j] = G V[:, j] for j < m (G in CSR, rows in the factor's order).
__global__ void k_spmv_cols(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const double* __restrict__ gv, const double* __restrict__ V, int64_t ldv,
                            const KState* ks, double* GV)
{
    const int m = ks->m;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const int a = rp[i], b = rp[i + 1];
        for (int j = 0; j < m; ++j) {
            double acc = 0.0;
            for (int q = a; q < b; ++q) acc += gv[q] * V[int64_t(j) * ldv + ci[q]];
            GV[int64_t(j) * ldv + i] = acc;
        }
    }
}

// gc[i] += lscale beta_l / c_i * sum_j GV_l[i, j] (beta_f (W V_f[i, :]^T)_j
//          + q0_j (y0_i - z2_i) + q1_j z1_i) for every row i (permuted order).
__global__ __launch_bounds__(256) void k_cg_nodes(int64_t n, const double* __restrict__ GVl,
                                                  const double* __restrict__ Vf, int64_t ldv,
                                                  const KState* kl, const KState* kf,
                                                  const double* __restrict__ y0,
                                                  const double* __restrict__ z1,
                                                  const double* __restrict__ z2,
                                                  const double* __restrict__ cperm,
                                                  const double* __restrict__ Wq, double lscale,
                                                  double* gc)
{
    __shared__ double Ws[MAXM * MAXM + 2 * MAXM];
    const int ml = kl->m, mf = kf->m;
    for (int i = threadIdx.x; i < MAXM * MAXM + 2 * MAXM; i += blockDim.x) Ws[i] = Wq[i];
    __syncthreads();
    if (ml == 0) return;
    const double bl = kl->beta, bf = kf->beta;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        double vf[MAXM];
#pragma unroll
        for (int k = 0; k < MAXM; ++k) vf[k] = k < mf ? Vf[int64_t(k) * ldv + i] : 0.0;
        const double d0 = y0[i] - z2[i], d1 = z1[i];
        double acc = 0.0;
        for (int j = 0; j < ml; ++j) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < MAXM; ++k) t += Ws[j * MAXM + k] * vf[k];
            acc += GVl[int64_t(j) * ldv + i] *
                   (bf * t + Ws[MAXM * MAXM + j] * d0 + Ws[MAXM * MAXM + MAXM + j] * d1);
        }
        gc[i] += lscale * bl * acc / cperm[i];
    }
}

// Restarts a Krylov process from a recorded normalised start vector (already
// in V_0) and its norm: the state k_normalize_v leaves.
__global__ void k_restore_start(KState* ks, const double* beta)
{
    if (threadIdx.x == 0) {
        const double b = *beta;
        ks->beta = b;
        ks->m = 0;
        ks->mdec = 0;
        ks->breakdown = 0;
        ks->converged = b == 0.0 ? 1 : 0;
        ks->done = b == 0.0 ? 1 : 0;
        ks->est = 0.0;
    }
}

__global__ void k_resume(KState* ks)
{
    if (threadIdx.x == 0) {
        ks->done = 0;
        ks->converged = 0;
    }
}

void launch_restore_start(KState* ks, const double* beta, hipStream_t st)
{
    k_restore_start<<<1, 64, 0, st>>>(ks, beta);
}

void launch_resume(KState* ks, hipStream_t st)
{
    k_resume<<<1, 64, 0, st>>>(ks);
}

__global__ void k_set_ends(int32_t* sel, int last)
{
    if (threadIdx.x == 0) {
        sel[0] = 0;
        sel[1] = last;
    }
}

void launch_set_ends(int32_t* sel, int last, hipStream_t st)
{
    k_set_ends<<<1, 64, 0, st>>>(sel, last);
}

void launch_adj_integrals(const KState* ks, double gamma, double tau, double* I, hipStream_t st)
{
    k_adj_integrals<<<1, 256, sizeof(double) * 7 * MAXM * LD, st>>>(ks, gamma, tau, I);
}

void launch_adj_amp(int n_src, const int32_t* row, const int64_t* delay, const int64_t* rise,
                    const int64_t* width, const int64_t* fall, int64_t t_hi, int64_t dt,
                    const double* V, int64_t ldv, const KState* ks, const double* I, double lscale,
                    double* grad, hipStream_t st)
{
    if (n_src <= 0) return;
    k_adj_amp<<<(n_src + 255) / 256, 256, 0, st>>>(n_src, row, delay, rise, width, fall, t_hi, dt, V, ldv,
                                                   ks, I, lscale, grad);
}

void launch_cg_block(const KState* kl, double gam_l, const KState* kf, double gam_f, double sig_b,
                     double tau_a, double h, double* Wq, hipStream_t st)
{
    k_cg_block<<<1, 256, sizeof(double) * (7 * MAXM * LD + 2 * MAXM), st>>>(kl, gam_l, kf, gam_f, sig_b, tau_a,
                                                                         h, Wq);
}

void launch_spmv_cols(int64_t n, const int32_t* rp, const int32_t* ci, const double* gv,
                      const double* V, int64_t ldv, const KState* ks, double* GV, hipStream_t st)
{
    k_spmv_cols<<<grid_for(n), 256, 0, st>>>(n, rp, ci, gv, V, ldv, ks, GV);
}

void launch_cg_nodes(int64_t n, const double* GVl, const double* Vf, int64_t ldv, const KState* kl,
                     const KState* kf, const double* y0, const double* z1, const double* z2,
                     const double* cperm, const double* Wq, double lscale, double* gc, hipStream_t st)
{
    k_cg_nodes<<<grid_for(n), 256, 0, st>>>(n, GVl, Vf, ldv, kl, kf, y0, z1, z2, cperm, Wq, lscale, gc);
}

void launch_adj_jump(int n_rows, const int32_t* rows, const int32_t* ptr, const int32_t* pidx,
                     const double* dJdx, int64_t n_out, int s, const double* cperm, double inv_scale,
                     double* lam, hipStream_t st)
{
    if (n_rows <= 0) return;
    k_adj_jump<<<(n_rows + 255) / 256, 256, 0, st>>>(n_rows, rows, ptr, pidx, dJdx, n_out, s, cperm, inv_scale,
                                                     lam);
}

void launch_spot_setup(int64_t n, const SpotArgs& sa, const double* Z1, const double* Z2, double* z1,
                       double* z2, const double* y, const double* y0, double* v, double* partial,
                       double* taus, const TauArgs& ta, hipStream_t st)
{
    k_spot_setup<<<grid_for(n), 256, 0, st>>>(n, sa, Z1, Z2, z1, z2, y, y0, v, partial, taus, ta);
}

void launch_setup_v(int64_t n, const double* y, const double* y0, const double* z2, double* v,
                    double* partial, KState* ks, hipStream_t st)
{
    (void)ks;
    k_setup_v<<<grid_for(n), 256, 0, st>>>(n, y, y0, z2, v, partial);
}

void launch_normalize_v(int64_t n, double* v, const double* partial, KState* ks, hipStream_t st)
{
    k_normalize_v<<<grid_for(n), 256, 0, st>>>(n, v, partial, grid_for(n), ks);
}

void launch_scatter_add(int32_t count, const int32_t* idx, const double* val, double* dst,
                        hipStream_t st)
{
    if (count <= 0) return;
    k_scatter_add<<<(count + 255) / 256, 256, 0, st>>>(count, idx, val, dst);
}

void launch_recon_probes(int n_probe, const int32_t* probe_perm, int n_snap, int32_t snap0,
                         const double* tau, const double* u, const KState* ks, const double* V,
                         int64_t ldv, const double* y0, const double* z1, const double* z2,
                         double* out, int32_t n_out, hipStream_t st)
{
    const int64_t tot = int64_t(n_probe) * n_snap;
    if (tot == 0) return;
    k_recon_probes<<<int((tot + 255) / 256), 256, 0, st>>>(n_probe, probe_perm, n_snap, snap0, tau,
                                                           u, ks, V, ldv, y0, z1, z2, out, n_out);
}

void launch_recon_full(int64_t n, double tau, const double* u, const KState* ks, const double* V,
                       int64_t ldv, double* y, double* y0, const double* z1, const double* z2,
                       hipStream_t st)
{
    k_recon_full<<<grid_for(n), 256, 0, st>>>(n, tau, u, ks, V, ldv, y, y0, z1, z2);
}

void launch_axpy_scaled(int64_t n, double a, const double* x, double* y, hipStream_t st)
{
    k_axpy<<<grid_for(n), 256, 0, st>>>(n, a, x, y);
}

void launch_gather_perm(int64_t n, const int32_t* perm, const double* src, double* dst,
                        int64_t ld_src, int64_t ld_dst, int ncols, hipStream_t st)
{
    k_gather_perm<<<dim3(grid_for(n), ncols), 256, 0, st>>>(n, perm, src, dst, ld_src, ld_dst, ncols);
}

void launch_scatter_perm(int64_t n, const int32_t* perm, const double* src, double* dst,
                         int64_t ld_src, int64_t ld_dst, int ncols, hipStream_t st)
{
    k_scatter_perm<<<dim3(grid_for(n), ncols), 256, 0, st>>>(n, perm, src, dst, ld_src, ld_dst, ncols);
}

void launch_tr_rhs(int64_t n, const int32_t* rp, const int32_t* ci, const double* gv, const double* cperm,
                   const double* y, double hh, int64_t t0, int64_t t1, const int32_t* sptr, const double* amp,
                   const int64_t* sd, const int64_t* sr, const int64_t* sw, const int64_t* sf, double* rhs,
                   hipStream_t st)
{
    k_tr_rhs<<<grid_for(n), 256, 0, st>>>(n, rp, ci, gv, cperm, y, hh, t0, t1, sptr, amp, sd, sr, sw, sf, rhs);
}

void launch_gather_probes(int n_probe, const int32_t* probe_perm, const double* y, double* out, int32_t n_out,
                          int32_t col, hipStream_t st)
{
    if (n_probe > 0)
        k_gather_probes<<<(n_probe + 255) / 256, 256, 0, st>>>(n_probe, probe_perm, y, out, n_out, col);
}

void launch_flag_nonfinite(int64_t count, const double* a, int32_t* flag, hipStream_t st)
{
    if (count > 0) k_flag_nonfinite<<<grid_for(count), 256, 0, st>>>(count, a, flag);
}

void launch_vdd_minus(int64_t count, double vdd, double* buf, hipStream_t st)
{
    k_vdd_minus<<<grid_for(count), 256, 0, st>>>(count, vdd, buf);
}

}  // namespace matex

// Batched R-MATEX kernels: R <= 64 subtasks (Sec. 3.1) advanced together.
//
// Every per-subtask n-vector is stored row-interleaved, x[i * R + r], so a
// wavefront reads one row of all subtasks in one coalesced access; lane r of
// a wavefront owns subtask r.
//
//  * Multi-right-hand-side substitution pair (Alg. 1's step, for all
//    subtasks at once), one or two launches per level and sweep. Forward:
//    kb_fwd computes [y_s ; delta_s] = W_s * btilde_s for 64 panel rows per
//    block as a dense 64 x K by K x R product staged through LDS, assembling
//    btilde_s = b_s - (children's updates) while staging it; supernodes with
//    many columns are split over blocks whose partial products kb_fwd_reduce
//    sums in a fixed order. Backward: kb_bwd computes x_s = W_s^T [y_s ;
//    -x_off] for 64 panel columns per block, split the same way. Each panel
//    entry is read once per sweep for all R subtasks.
//  * Gram-Schmidt per subtask (two classical passes): 256-thread blocks
//    (lane = subtask, four wavefronts on interleaved rows) write per-block
//    partial sums per subtask; kb_col_reduce (one block per subtask) sums
//    them in a fixed order and updates that subtask's state.
//  * Checks: one block per (subtask, check offset), the plain path's
//    small-dense routine with the subtask's own state and decision.
#include <hip/hip_runtime.h>

#include <cmath>

#include "batched.hpp"
#include "device_common.hpp"

namespace matex {

namespace {

using namespace dev;

constexpr int NVB = MAXM + 1;

// ------------------------------------------------------------- sweeps

// Stage width of the sweep products and the padded LDS row (breaks bank
// conflicts of the transposed panel store).
constexpr int BK = 16;
constexpr int LROW = RMAX + 2;

// Sum of the children's update slots that land on panel position g.
__device__ inline double pull(const BatchAssembly& as, int g, int R, int r, const double* U)
{
    double acc = 0.0;
    const int c1 = as.cptr[g + 1];
    for (int c = as.cptr[g]; c < c1; ++c) acc += U[int64_t(as.cidx[c]) * R + r];
    return acc;
}

// Rows first .. first + 63 of [y_s ; delta_s] for one supernode: the 64 x K
// panel block times the K x R block of btilde over the task's panel
// columns [kb, ke) (blocks of diagonal rows stop at their last row: the
// panel is zero above its diagonal). btilde is assembled while it is staged
// (scale * b minus the children's updates), and an off-diagonal row's
// update slot gets the children's updates plus the product. 16 x 16
// threads, each with a 4-row x 4-subtask register tile; panel and
// right-hand-side stages of BK columns go through LDS with coalesced loads
// (a panel column's rows are contiguous), the next stage loaded into
// registers while the current one is used.
__global__ __launch_bounds__(256) void kb_fwd(DevSym s, BatchAssembly as,
                                              const BTask* __restrict__ tasks, int R,
                                              const double* __restrict__ W,
                                              const double* __restrict__ B,
                                              const double* __restrict__ scale, double* y,
                                              double* U, double* P, const KState* rks)
{
    __shared__ double Ws[BK][LROW];
    __shared__ double Ts[BK][LROW];
    const BTask t = tasks[blockIdx.x];
    const int sn = t.sn, r0 = t.first, kb = t.kb, ke = t.ke;
    const int c0 = s.c0[sn], nr = s.nr[sn];
    const int pb = as.pos_base[sn];
    const int64_t ld = dpanel_ld(nr);
    const double* Wp = W + s.w[sn];
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    double wr[4], tr[4];
    // ragged inputs: right-hand side e is block m of its own basis
    const int e_own = tid & 63;
    const int64_t boff = rks && e_own < R ? int64_t(rks[e_own].m) * s.n * R : 0;
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + q * 256, kk = idx >> 6, e = idx & 63;
            const int k = k0 + kk, row = r0 + e;
            wr[q] = (k < ke && row < nr) ? Wp[int64_t(k) * ld + row] : 0.0;
            double b = 0.0;
            if (k < ke && e < R) {
                const int64_t o = boff + int64_t(c0 + k) * R + e;
                b = (scale ? B[o] * scale[c0 + k] : B[o]) - pull(as, pb + k, R, e, U);
            }
            tr[q] = b;
        }
    };
    load(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + q * 256, kk = idx >> 6, e = idx & 63;
            Ws[kk][e] = wr[q];
            Ts[kk][e] = tr[q];
        }
        __syncthreads();
        if (k0 + BK < ke) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = Ws[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Ts[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
    if (t.slot >= 0) {
        double* Pp = P + int64_t(t.slot) * PSLOT;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) Pp[(ty * 4 + i) * 64 + tx * 4 + j] = acc[i][j];
        return;
    }
    const int nc = s.nc[sn];
    const int64_t u = s.u[sn];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = r0 + ty * 4 + i;
        if (row >= nr) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = tx * 4 + j;
            if (r < R) {
                if (row < nc) y[int64_t(c0 + row) * R + r] = acc[i][j];
                else U[(u + row - nc) * R + r] = pull(as, pb + row, R, r, U) + acc[i][j];
            }
        }
    }
}

// Sums the partial slots of split forward blocks, in slot order (an
// off-diagonal row adds the children's updates first). One thread per
// element of the 64 x 64 slot (16 blocks per item); eight slots' loads are
// issued together and then added in order.
constexpr int RED_SPLIT = (64 * 64) / 256;

__device__ inline double sum_slots(const double* p, int cnt, double sum)
{
    int c = 0;
    for (; c + 8 <= cnt; c += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = p[int64_t(c + q) * PSLOT];
#pragma unroll
        for (int q = 0; q < 8; ++q) sum += v[q];
    }
    for (; c < cnt; ++c) sum += p[int64_t(c) * PSLOT];
    return sum;
}

__global__ __launch_bounds__(256) void kb_fwd_reduce(DevSym s, BatchAssembly as,
                                                     const BRed* __restrict__ items, int R,
                                                     const double* __restrict__ P, double* y,
                                                     double* U)
{
    const BRed it = items[blockIdx.x / RED_SPLIT];
    const int idx = (blockIdx.x % RED_SPLIT) * 256 + threadIdx.x;
    const int sn = it.sn;
    const int c0 = s.c0[sn], nc = s.nc[sn], nr = s.nr[sn];
    const int pb = as.pos_base[sn];
    const int64_t u = s.u[sn];
    const int e = idx >> 6, r = idx & 63, row = it.first + e;
    if (r >= R || row >= nr) return;
    double sum = row < nc ? 0.0 : pull(as, pb + row, R, r, U);
    sum = sum_slots(P + int64_t(it.slot) * PSLOT + idx, it.cnt, sum);
    if (row < nc) y[int64_t(c0 + row) * R + r] = sum;
    else U[(u + row - nc) * R + r] = sum;
}

// Columns first .. first + 63 of x_s for one supernode: W_s^T [y_s ; -x_off]
// over the task's panel rows [kb, ke) (the panel is zero above its
// diagonal). Panel stages are read as 16-entry column pieces (one 128-byte
// line each) and stored transposed in LDS; next stage prefetched as above.
__global__ __launch_bounds__(256) void kb_bwd(DevSym s, const BTask* __restrict__ tasks, int R,
                                              const double* __restrict__ W, const double* y,
                                              double* x, double* P)
{
    __shared__ double Ws[BK][LROW];
    __shared__ double Gs[BK][LROW];
    const BTask t = tasks[blockIdx.x];
    const int sn = t.sn, col0 = t.first, kb = t.kb, ke = t.ke;
    const int c0 = s.c0[sn], nc = s.nc[sn], nr = s.nr[sn];
    const int64_t ld = dpanel_ld(nr);
    const int32_t* roff = s.rows + s.roff[sn];
    const double* Wp = W + s.w[sn];
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    double wr[4], gr[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + q * 256;
            {
                const int cc = idx >> 4, kk = idx & (BK - 1);
                const int c = col0 + cc, k = k0 + kk;
                wr[q] = (c < nc && k < ke) ? Wp[int64_t(c) * ld + k] : 0.0;
            }
            {
                const int kk = idx >> 6, r = idx & 63;
                const int k = k0 + kk;
                double g = 0.0;
                if (k < ke && r < R)
                    g = k < nc ? y[int64_t(c0 + k) * R + r] : -x[int64_t(roff[k - nc]) * R + r];
                gr[q] = g;
            }
        }
    };
    load(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + q * 256;
            Ws[idx & (BK - 1)][idx >> 4] = wr[q];
            Gs[idx >> 6][idx & 63] = gr[q];
        }
        __syncthreads();
        if (k0 + BK < ke) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = Ws[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Gs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
    if (t.slot >= 0) {
        double* Pp = P + int64_t(t.slot) * PSLOT;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) Pp[(ty * 4 + i) * 64 + tx * 4 + j] = acc[i][j];
        return;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = col0 + ty * 4 + i;
        if (c >= nc) break;
        double* dst = x + int64_t(c0 + c) * R;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = tx * 4 + j;
            if (r < R) dst[r] = acc[i][j];
        }
    }
}

__global__ __launch_bounds__(256) void kb_bwd_reduce(DevSym s, const BRed* __restrict__ items, int R,
                                                     const double* __restrict__ P, double* x)
{
    const BRed it = items[blockIdx.x / RED_SPLIT];
    const int idx = (blockIdx.x % RED_SPLIT) * 256 + threadIdx.x;
    const int sn = it.sn;
    const int c0 = s.c0[sn], nc = s.nc[sn];
    const int e = idx >> 6, r = idx & 63, c = it.first + e;
    if (r >= R || c >= nc) return;
    x[int64_t(c0 + c) * R + r] = sum_slots(P + int64_t(it.slot) * PSLOT + idx, it.cnt, 0.0);
}

// ------------------------------------------------ wavefront-per-supernode

// Levels whose supernodes have at most WNC columns: one wavefront per
// supernode, lane r owning right-hand side r, so every vector row moves as
// one 512-byte line. btilde (forward) and the column sums (backward) stay in
// registers; the panel goes through wavefront-private LDS 64 rows at a time
// and is read as broadcasts. No block barrier: four independent wavefronts
// per block. The sums run over k (forward) and the panel rows (backward) in
// increasing order, as the block kernels' unsplit tasks do, so both give the
// same bits.
constexpr int WPF = 8;   // rows whose right-hand-side loads are issued together

// Panel rows i0 .. i0 + 63 (zeros past nr) of columns 0 .. nc - 1 into
// Ws[k * 64 + i - i0]; column k's rows are contiguous, one load per lane.
__device__ inline void stage_panel_rows(const double* __restrict__ Wp, int64_t ld, int i0, int nr, int nc, int lane,
                                        double* Ws)
{
    const int i = i0 + lane;
    const double* src = Wp + (i < nr ? i : 0);
#pragma unroll 4
    for (int k = 0; k < nc; ++k) {
        const double v = src[int64_t(k) * ld];
        Ws[k * 64 + lane] = i < nr ? v : 0.0;
    }
}

template <int WNC>
__global__ __launch_bounds__(256) void kb_fwd_wave(DevSym s, BatchAssembly as, const int32_t* __restrict__ sns,
                                                   int count, int R, const double* __restrict__ W,
                                                   const double* __restrict__ B,
                                                   const double* __restrict__ scale, double* y, double* U,
                                                   const KState* rks)
{
    __shared__ double Wsh[4][WNC * 64];
    const int wv = threadIdx.x >> 6, r = threadIdx.x & 63;
    const int idx = blockIdx.x * 4 + wv;
    if (idx >= count) return;
    const int sn = sns[idx];
    const int c0 = s.c0[sn], nc = s.nc[sn], nr = s.nr[sn];
    const int pb = as.pos_base[sn];
    const int64_t ld = dpanel_ld(nr), u = s.u[sn];
    const double* Wp = W + s.w[sn];
    double* Ws = Wsh[wv];
    const bool on = r < R;
    double bt[WNC];
    const int64_t boff = rks && on ? int64_t(rks[r].m) * s.n * R : 0;
#pragma unroll
    for (int k = 0; k < WNC; ++k) {
        double v = 0.0;
        if (k < nc && on) {
            const int64_t o = boff + int64_t(c0 + k) * R + r;
            v = (scale ? B[o] * scale[c0 + k] : B[o]) - pull(as, pb + k, R, r, U);
        }
        bt[k] = v;
    }
    for (int i0 = 0; i0 < nr; i0 += 64) {
        wave_sync();
        stage_panel_rows(Wp, ld, i0, nr, nc, r, Ws);
        wave_sync();
        const int i1 = min(nr, i0 + 64);
        for (int ib = i0; ib < i1; ib += WPF) {
            // the children's updates on the off rows of these rows, loaded together
            double pu[WPF];
#pragma unroll
            for (int q = 0; q < WPF; ++q) {
                const int i = ib + q;
                pu[q] = (i < i1 && i >= nc && on) ? pull(as, pb + i, R, r, U) : 0.0;
            }
#pragma unroll
            for (int q = 0; q < WPF; ++q) {
                const int i = ib + q;
                if (i >= i1) break;
                const int kmax = i < nc ? i + 1 : nc;
                const double* wr = Ws + (i - i0);
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < WNC; ++k)
                    if (k < kmax) acc += wr[k * 64] * bt[k];
                if (on) {
                    if (i < nc) y[int64_t(c0 + i) * R + r] = acc;
                    else U[(u + i - nc) * R + r] = pu[q] + acc;
                }
            }
        }
    }
}

template <int WNC>
__global__ __launch_bounds__(256) void kb_bwd_wave(DevSym s, const int32_t* __restrict__ sns, int count, int R,
                                                   const double* __restrict__ W, const double* y, double* x)
{
    __shared__ double Wsh[4][WNC * 64];
    const int wv = threadIdx.x >> 6, r = threadIdx.x & 63;
    const int idx = blockIdx.x * 4 + wv;
    if (idx >= count) return;
    const int sn = sns[idx];
    const int c0 = s.c0[sn], nc = s.nc[sn], nr = s.nr[sn];
    const int64_t ld = dpanel_ld(nr);
    const int32_t* roff = s.rows + s.roff[sn];
    const double* Wp = W + s.w[sn];
    double* Ws = Wsh[wv];
    const bool on = r < R;
    double acc[WNC];
#pragma unroll
    for (int c = 0; c < WNC; ++c) acc[c] = 0.0;
    for (int i0 = 0; i0 < nr; i0 += 64) {
        wave_sync();
        stage_panel_rows(Wp, ld, i0, nr, nc, r, Ws);
        wave_sync();
        const int i1 = min(nr, i0 + 64);
        for (int ib = i0; ib < i1; ib += WPF) {
            // g = [y_s ; -x(off rows)] for these rows, loaded together
            double g[WPF];
#pragma unroll
            for (int q = 0; q < WPF; ++q) {
                const int i = ib + q;
                double v = 0.0;
                if (i < i1 && on) v = i < nc ? y[int64_t(c0 + i) * R + r] : -x[int64_t(roff[i - nc]) * R + r];
                g[q] = v;
            }
#pragma unroll
            for (int q = 0; q < WPF; ++q) {
                const int i = ib + q;
                if (i >= i1) break;
                const double* wr = Ws + (i - i0);
#pragma unroll
                for (int c = 0; c < WNC; ++c)
                    if (c < nc && c <= i) acc[c] += wr[c * 64] * g[q];
            }
        }
    }
    if (on) {
#pragma unroll
        for (int c = 0; c < WNC; ++c)
            if (c < nc) x[int64_t(c0 + c) * R + r] = acc[c];
    }
}

// Column-major natural-order right-hand sides (ld n) to row-interleaved
// permuted order and back: dst[k * R + r] = src[perm[k] + r * n] and
// dst[perm[k] + r * n] = src[k * R + r].
__global__ void kb_interleave(int64_t n, int R, const int32_t* perm, const double* src, double* dst)
{
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n * R; i += int64_t(gridDim.x) * 256) {
        const int64_t k = i / R;
        const int r = int(i - k * R);
        dst[i] = src[perm[k] + int64_t(r) * n];
    }
}

__global__ void kb_deinterleave(int64_t n, int R, const int32_t* perm, const double* src, double* dst)
{
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n * R; i += int64_t(gridDim.x) * 256) {
        const int64_t k = i / R;
        const int r = int(i - k * R);
        dst[perm[k] + int64_t(r) * n] = src[i];
    }
}

// ---------------------------------------------------------- Gram-Schmidt

// Sums acc[0..cnt) of lane r over the block's four wavefronts; the result
// is valid in wavefront 0. buf: 2 * N * 64 doubles of LDS.
template <int N>
__device__ inline void combine_waves(double (&acc)[N], int cnt, double* buf)
{
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wv >= 2) {
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (i < cnt) buf[((wv - 2) * N + i) * 64 + lane] = acc[i];
    }
    __syncthreads();
    if (wv < 2) {
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (i < cnt) acc[i] += buf[(wv * N + i) * 64 + lane];
    }
    __syncthreads();
    if (wv == 1) {
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (i < cnt) buf[i * 64 + lane] = acc[i];
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (i < cnt) acc[i] += buf[i * 64 + lane];
    }
}

// Dots of a chunk of up to GS_CHUNK basis vectors with w, per subtask:
// partial[(block * R + r) * (NVB + 1) + i] for i in the chunk (blockIdx.y),
// and with `norm`, ||w||^2 into slot nv (chunk 0). Lane = subtask, the
// block's four wavefronts take interleaved rows.
constexpr int GS_CHUNK = 16;

// Basis vectors of subtask r in this pass: the launch's nv, or with ragged
// dimensions (subtasks at different iterations) its own m + 1, read before
// kb_col_reduce's second pass records the new column and sets m to that
// count (`recorded`: read after it, the count is m itself); a lane works
// only when its subtask is in the pass (act null: all) and not done.
__device__ inline int lane_nv(const KState* ks, int r, int R, int nv, int ragged, int recorded = 0)
{
    return ragged ? (r < R ? ks[r].m + (recorded ? 0 : 1) : 0) : nv;
}
__device__ inline bool lane_on(const KState* ks, const int32_t* act, int r, int R)
{
    return r < R && !ks[r].done && (!act || act[r]);
}

__global__ __launch_bounds__(256) void kb_gs_dots(int64_t n, int R, const double* __restrict__ V,
                                                  int nv_all, const double* __restrict__ w,
                                                  double* partial, const KState* ks, int norm,
                                                  const int32_t* act, int ragged)
{
    __shared__ double buf[2 * (GS_CHUNK + 1) * 64];
    const int r = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nv = lane_nv(ks, r, R, nv_all, ragged);
    const int i0 = blockIdx.y * GS_CHUNK;
    const int cnt = min(GS_CHUNK, nv - i0);
    const bool with_norm = norm && blockIdx.y == 0;
    const bool on = lane_on(ks, act, r, R) && cnt > 0;
    double acc[GS_CHUNK + 1];
#pragma unroll
    for (int i = 0; i <= GS_CHUNK; ++i) acc[i] = 0.0;
    if (on) {
        const double* Vc = V + int64_t(i0) * n * R;
        for (int64_t row = int64_t(blockIdx.x) * 4 + wv; row < n; row += int64_t(gridDim.x) * 4) {
            const double wr = w[row * R + r];
#pragma unroll
            for (int i = 0; i < GS_CHUNK; ++i)
                if (i < cnt) acc[i] += wr * Vc[int64_t(i) * n * R + row * R + r];
            if (with_norm) acc[GS_CHUNK] += wr * wr;
        }
    }
    combine_waves(acc, GS_CHUNK + 1, buf);
    if (wv == 0 && on) {
        double* out = partial + (int64_t(blockIdx.x) * R + r) * (NVB + 1);
#pragma unroll
        for (int i = 0; i < GS_CHUNK; ++i)
            if (i < cnt) out[i0 + i] = acc[i];
        if (with_norm) out[nv] = acc[GS_CHUNK];
    }
}

// out = (w - sum_i h[i] V_i) * sc per subtask, h = h1 (mode 0, sc = 1, out
// = w in place) or h2 (mode 1, sc = vscale, out = V_nv). The coefficients
// sit in LDS, so a row needs only its nv basis values in flight.
__global__ __launch_bounds__(256) void kb_gs_axpy(int64_t n, int R, double* V, int nv_all, double* w,
                                                  const KState* ks, int mode, const int32_t* act, int ragged)
{
    __shared__ double hs[NVB][64];
    const int r = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int idx = threadIdx.x; idx < NVB * 64; idx += 256) {
        const int i = idx >> 6, q = idx & 63;
        double h = 0.0;
        if (q < R && i < lane_nv(ks, q, R, nv_all, ragged, mode)) h = mode == 0 ? ks[q].h1[i] : ks[q].h2[i];
        hs[i][q] = h;
    }
    __syncthreads();
    if (!lane_on(ks, act, r, R)) return;
    // mode 1 runs after the second reduction has set m to the count
    const int nv = lane_nv(ks, r, R, nv_all, ragged, mode);
    const double sc = mode == 0 ? 1.0 : ks[r].vscale;
    double* out = mode == 0 ? w : V + int64_t(nv) * n * R;
    for (int64_t row = int64_t(blockIdx.x) * 4 + wv; row < n; row += int64_t(gridDim.x) * 4) {
        double wr = w[row * R + r];
#pragma unroll
        for (int i = 0; i < NVB; ++i)
            if (i < nv) wr -= hs[i][r] * V[int64_t(i) * n * R + row * R + r];
        out[row * R + r] = wr * sc;
    }
}

// First-pass update and second-pass dots in one sweep over the basis:
// w' = w - sum_i h1[i] V_i in place, then per subtask the partial dots V_i^T w'
// and ||w'||^2 (slot nv) of the block's rows into partial[(block * R + r) *
// (NVB + 1) + i]. A block takes tiles of GS_TILE rows: each wavefront updates
// GS_TILE / 4 rows (lane = subtask) and stages w' in LDS; then value i is
// summed over the tile by wavefront i mod 4 (the tile's basis values come
// back from cache, not HBM).
constexpr int GS_TILE = 16;
constexpr int GS_VPW_B = (NVB + 1 + 3) / 4;

__global__ __launch_bounds__(256) void kb_gs_update_dots(int64_t n, int R, const double* __restrict__ V,
                                                         int nv_all, double* w, double* partial,
                                                         const KState* ks, const int32_t* act, int ragged)
{
    __shared__ double hs[NVB][64];
    __shared__ double wl[GS_TILE][64];
    const int r = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int idx = threadIdx.x; idx < NVB * 64; idx += 256) {
        const int i = idx >> 6, q = idx & 63;
        hs[i][q] = (q < R && i < lane_nv(ks, q, R, nv_all, ragged)) ? ks[q].h1[i] : 0.0;
    }
    __syncthreads();
    const bool on = lane_on(ks, act, r, R);
    const int nv = lane_nv(ks, r, R, nv_all, ragged);
    double acc[GS_VPW_B];
#pragma unroll
    for (int q = 0; q < GS_VPW_B; ++q) acc[q] = 0.0;
    for (int64_t base = int64_t(blockIdx.x) * GS_TILE; base < n; base += int64_t(gridDim.x) * GS_TILE) {
        // update: rows base + wv, base + wv + 4, ...
#pragma unroll
        for (int t = wv; t < GS_TILE; t += 4) {
            const int64_t row = base + t;
            double wr = 0.0;
            if (on && row < n) {
                wr = w[row * R + r];
#pragma unroll 8
                for (int i = 0; i < nv; ++i) wr -= hs[i][r] * V[int64_t(i) * n * R + row * R + r];
                w[row * R + r] = wr;
            }
            wl[t][r] = wr;
        }
        __syncthreads();
        if (on) {
            const int rows = int(min<int64_t>(GS_TILE, n - base));
#pragma unroll
            for (int q = 0; q < GS_VPW_B; ++q) {
                const int i = wv + 4 * q;
                if (i < nv) {
                    const double* Vi = V + int64_t(i) * n * R + base * R + r;
                    double sum = 0.0;
#pragma unroll
                    for (int t = 0; t < GS_TILE; ++t)
                        if (t < rows) sum += wl[t][r] * Vi[int64_t(t) * R];
                    acc[q] += sum;
                } else if (i == nv) {
                    double sum = 0.0;
#pragma unroll
                    for (int t = 0; t < GS_TILE; ++t)
                        if (t < rows) sum += wl[t][r] * wl[t][r];
                    acc[q] += sum;
                }
            }
        }
        __syncthreads();
    }
    if (on) {
        double* out = partial + (int64_t(blockIdx.x) * R + r) * (NVB + 1);
#pragma unroll
        for (int q = 0; q < GS_VPW_B; ++q) {
            const int i = wv + 4 * q;
            if (i <= nv) out[i] = acc[q];
        }
    }
}

// The same pass with every basis entry read once: a lane keeps the row's
// entries of all nv vectors in registers, so the dots of w' take them from
// there instead of reading the tile again (nv <= NVC). Wavefront wv takes
// rows wv, wv + 4, ... of the block's share; the lanes' sums over their rows
// are added across the four wavefronts through LDS. w' is the same as the
// two-read pass's; the dots differ from it by rounding only (another order).
constexpr int NVC = 24;

__global__ __launch_bounds__(256) void kb_gs_update_dots_reg(int64_t n, int R, const double* __restrict__ V,
                                                             int nv_all, double* w, double* partial,
                                                             const KState* ks, const int32_t* act, int ragged)
{
    __shared__ double hs[NVC][64];
    __shared__ double red[2][NVC + 1][64];
    const int r = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int idx = threadIdx.x; idx < NVC * 64; idx += 256) {
        const int i = idx >> 6, q = idx & 63;
        hs[i][q] = (q < R && i < lane_nv(ks, q, R, nv_all, ragged)) ? ks[q].h1[i] : 0.0;
    }
    __syncthreads();
    const bool on = lane_on(ks, act, r, R);
    const int nv = lane_nv(ks, r, R, nv_all, ragged);
    double acc[NVC + 1];
#pragma unroll
    for (int i = 0; i <= NVC; ++i) acc[i] = 0.0;
    if (on) {
        const int64_t nR = n * R;
        for (int64_t row = int64_t(blockIdx.x) * 4 + wv; row < n; row += int64_t(gridDim.x) * 4) {
            const double* Vr = V + row * R + r;
            double v[NVC];
#pragma unroll
            for (int i = 0; i < NVC; ++i) v[i] = i < nv ? Vr[int64_t(i) * nR] : 0.0;
            double wr = w[row * R + r];
#pragma unroll
            for (int i = 0; i < NVC; ++i)
                if (i < nv) wr -= hs[i][r] * v[i];
            w[row * R + r] = wr;
#pragma unroll
            for (int i = 0; i < NVC; ++i)
                if (i < nv) acc[i] += v[i] * wr;
            acc[NVC] += wr * wr;
        }
    }
    if (wv >= 2) {
#pragma unroll
        for (int i = 0; i <= NVC; ++i) red[wv - 2][i][r] = acc[i];
    }
    __syncthreads();
    if (wv < 2) {
#pragma unroll
        for (int i = 0; i <= NVC; ++i) acc[i] += red[wv][i][r];
    }
    __syncthreads();
    if (wv == 1) {
#pragma unroll
        for (int i = 0; i <= NVC; ++i) red[0][i][r] = acc[i];
    }
    __syncthreads();
    if (wv == 0 && on) {
        double* out = partial + (int64_t(blockIdx.x) * R + r) * (NVB + 1);
#pragma unroll
        for (int i = 0; i < NVC; ++i)
            if (i < nv) out[i] = acc[i] + red[0][i][r];
        out[nv] = acc[NVC] + red[0][NVC][r];
    }
}

// One block per subtask: sums the nblk partial rows of pass `mode`.
// mode 0: h1 (nv values). mode 1: h2 and ||w'||^2, then the new Hessenberg
// column, m, breakdown and the normalisation scale of v_{j+1}. mode 2: the
// squared norm of v (setup): beta, and a reset of the state for a new basis
// (only for subtasks with active[r]; others are marked done).
__global__ __launch_bounds__(256) void kb_col_reduce(int R, int nblk, const double* partial,
                                                     int stride, int nv_all, int mode, KState* ks,
                                                     const int32_t* active, int ragged)
{
    const int r = blockIdx.x;
    KState* k = ks + r;
    if (mode < 2 && (k->done || (active && !active[r]))) return;
    if (mode == 3 && !active[r]) return;   // set-up of some subtasks: the others untouched
    const int nv = lane_nv(ks, r, R, nv_all, ragged);
    __shared__ double red[4 * (NVMAX + 1)];
    __shared__ double vals[NVMAX + 1];
    const int cnt = mode == 0 ? nv : (mode == 1 ? nv + 1 : 1);
    double acc[NVMAX];
#pragma unroll
    for (int i = 0; i < NVMAX; ++i) acc[i] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
        const double* p = partial + (int64_t(b) * R + r) * stride;
#pragma unroll
        for (int i = 0; i < NVMAX; ++i)
            if (i < cnt) acc[i] += p[i];
    }
    block_sums(acc, cnt, red, vals);
    if (threadIdx.x != 0) return;
    if (mode == 0) {
        for (int i = 0; i < nv; ++i) k->h1[i] = vals[i];
    } else if (mode == 1) {
        double s2 = 0.0, hmax = 0.0;
        for (int i = 0; i < nv; ++i) {
            k->h2[i] = vals[i];
            s2 += vals[i] * vals[i];
            hmax = fmax(hmax, fabs(k->h1[i] + vals[i]));
        }
        const double beta = sqrt(fmax(vals[nv] - s2, 0.0));
        const bool brk = !(beta > 1e-14 * hmax);   // happy breakdown: exact
        const int j = nv - 1;
        for (int i = 0; i < nv; ++i) k->Ht[i + j * (MAXM + 1)] = k->h1[i] + k->h2[i];
        k->Ht[nv + j * (MAXM + 1)] = beta;
        k->m = nv;
        k->breakdown = brk ? 1 : 0;
        k->vscale = brk ? 0.0 : 1.0 / beta;
    } else {
        if (!active[r]) {
            k->done = 1;
            k->converged = 1;
            return;
        }
        const double beta = sqrt(vals[0]);   // modes 2 and 3
        k->beta = beta;
        k->m = 0;
        k->mdec = 0;
        k->breakdown = 0;
        k->converged = beta == 0.0 ? 1 : 0;
        k->done = beta == 0.0 ? 1 : 0;
        k->est = 0.0;
        k->vscale = beta == 0.0 ? 0.0 : 1.0 / beta;
    }
}

// -------------------------------------------------------------- checks

// blocks: (subtask chk_col[b], check chk_idx[b]); subtask r's blocks are
// chk_idx[col_off[r] .. + col_cnt[r]], its offsets taus[tau_off[r] ..], its u
// vectors and estimates sit in its fixed region of `cap` checks
// (u_buf + r * cap * MAXM, est_buf + r * cap).
__global__ __launch_bounds__(256) void kb_checks(KState* ks, double gamma, const double* taus,
                                                 const int32_t* tau_off, int cap,
                                                 const int32_t* chk_col, const int32_t* chk_idx,
                                                 const int32_t* col_off, const int32_t* col_cnt,
                                                 double tol, double* u_buf, double* est_buf,
                                                 int m_max, int update_state)
{
    const int r = chk_col[blockIdx.x], c = chk_idx[blockIdx.x];
    KState* k = ks + r;
    if (update_state && k->done) return;
    extern __shared__ double sm[];
    const int64_t reg = int64_t(r) * cap;
    check_block(k, k->m, k->breakdown, gamma, taus + tau_off[r], c, chk_idx + col_off[r], col_cnt[r], tol, u_buf + reg * MAXM,
                est_buf + reg, m_max, update_state, sm);
}

// Lets the listed subtasks continue iterating.
__global__ void kb_resume(KState* ks, const int32_t* cols, int cnt)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < cnt) {
        ks[cols[k]].done = 0;
        ks[cols[k]].converged = 0;
    }
}

// ---------------------------------------------------- set-up and outputs

// v = y - y0 + z2 into V_0, partial squared norms per subtask.
__global__ __launch_bounds__(256) void kb_setup_v(int64_t n, int R, const double* y,
                                                  const double* y0, const double* z2, double* v,
                                                  double* partial, const int32_t* active)
{
    __shared__ double buf[2 * 64];
    const int r = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double acc[1] = {0.0};
    if (r < R && active[r]) {
        for (int64_t row = int64_t(blockIdx.x) * 4 + wv; row < n; row += int64_t(gridDim.x) * 4) {
            const int64_t o = row * R + r;
            const double t = y[o] - y0[o] + z2[o];
            v[o] = t;
            acc[0] += t * t;
        }
    }
    combine_waves(acc, 1, buf);
    if (wv == 0 && r < R) partial[(int64_t(blockIdx.x) * R + r) * 2] = acc[0];
}

__global__ __launch_bounds__(256) void kb_scale_v(int64_t n, int R, double* v, const KState* ks,
                                                  const int32_t* active)
{
    const int r = threadIdx.x & 63;
    if (r >= R || !active[r] || ks[r].done) return;
    const double sc = ks[r].vscale;
    for (int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6); row < n; row += int64_t(gridDim.x) * 4)
        v[row * R + r] *= sc;
}

// Yout[(r * n_probe + p) * n_out + tidx] for every (subtask, snapshot) entry.
__global__ __launch_bounds__(256) void kb_recon_probes(int64_t n, int R, int n_probe,
                                                       const int32_t* probe_perm, int n_ent,
                                                       const int32_t* ent_col,
                                                       const int32_t* ent_t,
                                                       const double* ent_tau,
                                                       const int32_t* ent_u, const double* u_buf,
                                                       const KState* ks, const double* V,
                                                       const double* y0, const double* z1,
                                                       const double* z2, double* Yout, int n_out)
{
    const int64_t id = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (id >= int64_t(n_ent) * n_probe) return;
    const int e = int(id / n_probe), p = int(id % n_probe);
    const int r = ent_col[e];
    const int64_t o = int64_t(probe_perm[p]) * R + r;
    const int m = ks[r].m;
    const double* u = u_buf + int64_t(ent_u[e]) * MAXM;
    double acc = 0.0;
    for (int k = 0; k < m; ++k) acc += V[int64_t(k) * n * R + o] * u[k];
    acc *= ks[r].beta;
    const double t = ent_tau[e];
    Yout[(int64_t(r) * n_probe + p) * n_out + ent_t[e]] = acc + y0[o] + t * z1[o] - z2[o];
}

// Step end per active subtask: y = beta V u + y0 + tau z1 - z2, y0 += tau z1.
__global__ __launch_bounds__(256) void kb_recon_full(int64_t n, int R, const double* col_tau,
                                                     const int32_t* col_u, const double* u_buf,
                                                     const KState* ks, const int32_t* active,
                                                     const double* V, double* y, double* y0,
                                                     const double* z1, const double* z2)
{
    const int r = threadIdx.x & 63;
    if (r >= R || !active[r]) return;
    const int m = ks[r].m;
    const double beta = ks[r].beta, tau = col_tau[r];
    const double* u = u_buf + int64_t(col_u[r]) * MAXM;
    for (int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6); row < n; row += int64_t(gridDim.x) * 4) {
        const int64_t o = row * R + r;
        double acc = 0.0;
        for (int k = 0; k < m; ++k) acc += V[int64_t(k) * n * R + o] * u[k];
        const double a = y0[o], b = z1[o];
        y[o] = beta * acc + a + tau * b - z2[o];
        y0[o] = a + tau * b;
    }
}

// Slope changes of independently advancing subtasks from solved columns:
// for subtask r, z1 += sum_e coef[e] Z1[:, q[e]] and z2 likewise over its
// events e = ptr[r] .. ptr[r + 1] - 1 (in that order); Z1, Z2 column-major
// n x columns, z1, z2 row-interleaved.
__global__ __launch_bounds__(256) void kb_spot_cols(int64_t n, int R, const int32_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ q, const double* __restrict__ coef,
                                                    const double* __restrict__ Z1, const double* __restrict__ Z2,
                                                    double* z1, double* z2)
{
    const int r = threadIdx.x & 63;
    if (r >= R) return;
    const int e0 = ptr[r], e1 = ptr[r + 1];
    if (e0 == e1) return;
    for (int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6); row < n; row += int64_t(gridDim.x) * 4) {
        const int64_t o = row * R + r;
        double a = z1[o], b = z2[o];
        for (int e = e0; e < e1; ++e) {
            const int64_t zo = int64_t(q[e]) * n + row;
            a += coef[e] * Z1[zo];
            b += coef[e] * Z2[zo];
        }
        z1[o] = a;
        z2[o] = b;
    }
}

// s[row * R + col] += d for the events of this generation ((row, col) unique).
__global__ void kb_events(int cnt, int R, const int32_t* row, const int32_t* col, const double* d,
                          double* s)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < cnt) s[int64_t(row[k]) * R + col[k]] += d[k];
}

// Superposition of one batch (Sec. 3.1): out[p, t] += sgn * sum_r Yout[r, p, t];
// final[perm[i]] += sgn * sum_r y[i, r].
__global__ void kb_sum_out(int64_t count, int R, const double* Yout, double sgn, double* out)
{
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += int64_t(gridDim.x) * 256) {
        double acc = 0.0;
        for (int r = 0; r < R; ++r) acc += Yout[int64_t(r) * count + i];
        out[i] += sgn * acc;
    }
}

__global__ void kb_sum_final(int64_t n, int R, const int32_t* perm, const double* y, double sgn,
                             double* out)
{
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        double acc = 0.0;
        for (int r = 0; r < R; ++r) acc += y[i * R + r];
        out[perm[i]] += sgn * acc;
    }
}

__global__ void kb_fill(int64_t count, double v, double* x)
{
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += int64_t(gridDim.x) * 256)
        x[i] = v;
}

inline int grid_rows(int64_t n, int per_block) { return int(std::min<int64_t>((n + per_block - 1) / per_block, 4096)); }

}  // namespace

void launch_b_forward(const DevSym& s, const BatchAssembly& as, const BatchLevel& lv, int R,
                      const double* W, const double* B, const double* scale, double* y,
                      double* U, double* P, hipStream_t st, const KState* rks)
{
    if (lv.fwave) {
        if (lv.wave_nc <= 16)
            kb_fwd_wave<16><<<(lv.n_fwave + 3) / 4, 256, 0, st>>>(s, as, lv.fwave, lv.n_fwave, R, W, B, scale, y, U,
                                                                  rks);
        else
            kb_fwd_wave<WAVE_MAX_NC><<<(lv.n_fwave + 3) / 4, 256, 0, st>>>(s, as, lv.fwave, lv.n_fwave, R, W, B, scale,
                                                                           y, U, rks);
        return;
    }
    kb_fwd<<<lv.n_fwd, 256, 0, st>>>(s, as, lv.fwd, R, W, B, scale, y, U, P, rks);
    if (lv.n_fred) kb_fwd_reduce<<<lv.n_fred * RED_SPLIT, 256, 0, st>>>(s, as, lv.fred, R, P, y, U);
}

void launch_b_backward(const DevSym& s, const BatchLevel& lv, int R, const double* W,
                       const double* y, double* x, double* P, hipStream_t st)
{
    if (lv.bwave) {
        if (lv.wave_nc <= 16)
            kb_bwd_wave<16><<<(lv.n_bwave + 3) / 4, 256, 0, st>>>(s, lv.bwave, lv.n_bwave, R, W, y, x);
        else
            kb_bwd_wave<WAVE_MAX_NC><<<(lv.n_bwave + 3) / 4, 256, 0, st>>>(s, lv.bwave, lv.n_bwave, R, W, y, x);
        return;
    }
    kb_bwd<<<lv.n_bwd, 256, 0, st>>>(s, lv.bwd, R, W, y, x, P);
    if (lv.n_bred) kb_bwd_reduce<<<lv.n_bred * RED_SPLIT, 256, 0, st>>>(s, lv.bred, R, P, x);
}

void launch_b_gs(int64_t n, int R, double* V, int nv, double* w, double* partial, KState* ks,
                 hipStream_t st, const int32_t* act, int ragged)
{
    const int nb = B_RED_BLOCKS;
    const int stride = NVB + 1;
    const dim3 gd(nb, (nv + GS_CHUNK - 1) / GS_CHUNK);
    kb_gs_dots<<<gd, 256, 0, st>>>(n, R, V, nv, w, partial, ks, 0, act, ragged);
    kb_col_reduce<<<R, 256, 0, st>>>(R, nb, partial, stride, nv, 0, ks, act, ragged);
    if (nv <= NVC)
        kb_gs_update_dots_reg<<<nb, 256, 0, st>>>(n, R, V, nv, w, partial, ks, act, ragged);
    else
        kb_gs_update_dots<<<nb, 256, 0, st>>>(n, R, V, nv, w, partial, ks, act, ragged);
    kb_col_reduce<<<R, 256, 0, st>>>(R, nb, partial, stride, nv, 1, ks, act, ragged);
    kb_gs_axpy<<<grid_rows(n, 4), 256, 0, st>>>(n, R, V, nv, w, ks, 1, act, ragged);
}

void launch_b_checks(KState* ks, double gamma, const double* taus, const int32_t* tau_off, int cap,
                     const int32_t* chk_col, const int32_t* chk_idx, const int32_t* col_off,
                     const int32_t* col_cnt, int n_chk, double tol, double* u_buf, double* est_buf,
                     int m_max, int update_state, hipStream_t st)
{
    if (n_chk <= 0) return;
    kb_checks<<<n_chk, 256, checks_lds_bytes(), st>>>(ks, gamma, taus, tau_off, cap, chk_col, chk_idx,
                                                      col_off, col_cnt, tol, u_buf, est_buf, m_max,
                                                      update_state);
}

void launch_b_resume(KState* ks, const int32_t* cols, int cnt, hipStream_t st)
{
    if (cnt <= 0) return;
    kb_resume<<<(cnt + 63) / 64, 64, 0, st>>>(ks, cols, cnt);
}

void launch_b_setup(int64_t n, int R, const double* y, const double* y0, const double* z2,
                    double* V, double* partial, KState* ks, const int32_t* active, hipStream_t st,
                    bool keep_others)
{
    const int nb = B_RED_BLOCKS;
    kb_setup_v<<<nb, 256, 0, st>>>(n, R, y, y0, z2, V, partial, active);
    kb_col_reduce<<<R, 256, 0, st>>>(R, nb, partial, 2, 0, keep_others ? 3 : 2, ks, active, 0);
    kb_scale_v<<<grid_rows(n, 4), 256, 0, st>>>(n, R, V, ks, active);
}

void launch_b_recon_probes(int64_t n, int R, int n_probe, const int32_t* probe_perm, int n_ent,
                           const int32_t* ent_col, const int32_t* ent_t, const double* ent_tau,
                           const int32_t* ent_u, const double* u_buf, const KState* ks,
                           const double* V, const double* y0, const double* z1, const double* z2,
                           double* Yout, int n_out, hipStream_t st)
{
    const int64_t tot = int64_t(n_ent) * n_probe;
    if (tot == 0) return;
    kb_recon_probes<<<int((tot + 255) / 256), 256, 0, st>>>(n, R, n_probe, probe_perm, n_ent, ent_col,
                                                            ent_t, ent_tau, ent_u, u_buf, ks, V, y0,
                                                            z1, z2, Yout, n_out);
}

void launch_b_recon_full(int64_t n, int R, const double* col_tau, const int32_t* col_u,
                         const double* u_buf, const KState* ks, const int32_t* active,
                         const double* V, double* y, double* y0, const double* z1, const double* z2,
                         hipStream_t st)
{
    kb_recon_full<<<grid_rows(n, 4), 256, 0, st>>>(n, R, col_tau, col_u, u_buf, ks, active, V, y, y0,
                                                   z1, z2);
}

void launch_b_spot_cols(int64_t n, int R, const int32_t* ptr, const int32_t* q, const double* coef,
                        const double* Z1, const double* Z2, double* z1, double* z2, hipStream_t st)
{
    kb_spot_cols<<<grid_rows(n, 4), 256, 0, st>>>(n, R, ptr, q, coef, Z1, Z2, z1, z2);
}

void launch_b_events(int cnt, int R, const int32_t* row, const int32_t* col, const double* d,
                     double* s, hipStream_t st)
{
    if (cnt <= 0) return;
    kb_events<<<(cnt + 255) / 256, 256, 0, st>>>(cnt, R, row, col, d, s);
}

void launch_b_sum_out(int64_t count, int R, const double* Yout, double sgn, double* out,
                      hipStream_t st)
{
    if (count <= 0) return;
    kb_sum_out<<<grid_rows(count, 256), 256, 0, st>>>(count, R, Yout, sgn, out);
}

void launch_b_sum_final(int64_t n, int R, const int32_t* perm, const double* y, double sgn,
                        double* out, hipStream_t st)
{
    kb_sum_final<<<grid_rows(n, 256), 256, 0, st>>>(n, R, perm, y, sgn, out);
}

void launch_b_interleave(int64_t n, int R, const int32_t* perm, const double* src, double* dst,
                         hipStream_t st)
{
    kb_interleave<<<grid_rows(n * R, 256), 256, 0, st>>>(n, R, perm, src, dst);
}

void launch_b_deinterleave(int64_t n, int R, const int32_t* perm, const double* src, double* dst,
                           hipStream_t st)
{
    kb_deinterleave<<<grid_rows(n * R, 256), 256, 0, st>>>(n, R, perm, src, dst);
}

void launch_b_fill(int64_t count, double v, double* x, hipStream_t st)
{
    if (count <= 0) return;
    kb_fill<<<grid_rows(count, 256), 256, 0, st>>>(count, v, x);
}

}  // namespace matex

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
//    e^{tau H_m} by the [13/13] Pade approximant with scaling and squaring
//    (Higham 2005), and the error estimate; the last workgroup decides.
//  * Reconstruction (Alg. 1 last line, Alg. 2 snapshot reuse):
//    y(t_a + tau) = beta V_m e^{tau H_m} e1 + y0 + tau z1 - z2.
#include "kernels.hpp"

#include <cmath>

#include "factor.hpp"

namespace matex {

namespace {

// Leading dimension of a panel with nr rows (device twin of panel_ld).
__device__ inline int dpanel_ld(int nr) { return (nr + PANEL_ALIGN - 1) / PANEL_ALIGN * PANEL_ALIGN; }

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// ---------------------------------------------------------------- sweeps

// One forward task: panel rows [r0, r0 + FWD_ROWS) of supernode sn.
// lds: lds_nc + FWD_ROWS + 256 doubles.
__device__ inline void fwd_task(const DevSym& s, int sn, int r0, double* lds, int lds_nc,
                                const double* W, const double* b, const double* scale,
                                double* y, double* upd)
{
    double* bt = lds;                       // btilde over the supernode's columns
    double* acc_off = lds + lds_nc;         // children's updates on this task's off rows
    double* part = acc_off + FWD_ROWS;      // k-slice partial sums
    const int c0 = s.c0[sn], nc = s.nc[sn], nr = s.nr[sn];
    for (int k = threadIdx.x; k < nc; k += 256) {
        const double v = b[c0 + k];
        bt[k] = scale ? v * scale[c0 + k] : v;
    }
    if (threadIdx.x < FWD_ROWS) acc_off[threadIdx.x] = 0.0;
    __syncthreads();
    // assemble the children's subtree updates (one child at a time: two
    // children may touch the same row, one child never touches a row twice)
    const int cp1 = s.child_ptr[sn + 1];
    for (int cp = s.child_ptr[sn]; cp < cp1; ++cp) {
        const int c = s.child_idx[cp];
        const int64_t uc = s.u[c];
        const int noc = s.nr[c] - s.nc[c];
        for (int q = threadIdx.x; q < noc; q += 256) {
            const int pos = s.relidx[uc + q];
            const double val = upd[uc + q];
            if (pos < nc) bt[pos] -= val;
            else if (pos >= r0 && pos < r0 + FWD_ROWS) acc_off[pos - r0] += val;
        }
        __syncthreads();
    }
    const int lane = threadIdx.x & (FWD_ROWS - 1), ks = threadIdx.x / FWD_ROWS;
    const int row = r0 + lane;
    double acc = 0.0;
    if (row < nr) {
        const int kmax = row < nc ? row + 1 : nc;
        const int ld = dpanel_ld(nr);
        const double* wr = W + s.w[sn] + row;
        int k = ks;
        for (; k + 3 * FWD_KSPLIT < kmax; k += 4 * FWD_KSPLIT) {
            const double a0 = wr[int64_t(k) * ld], a1 = wr[int64_t(k + FWD_KSPLIT) * ld];
            const double a2 = wr[int64_t(k + 2 * FWD_KSPLIT) * ld];
            const double a3 = wr[int64_t(k + 3 * FWD_KSPLIT) * ld];
            acc += (a0 * bt[k] + a1 * bt[k + FWD_KSPLIT]) +
                   (a2 * bt[k + 2 * FWD_KSPLIT] + a3 * bt[k + 3 * FWD_KSPLIT]);
        }
        for (; k < kmax; k += FWD_KSPLIT) acc += wr[int64_t(k) * ld] * bt[k];
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < FWD_ROWS && row < nr) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < FWD_KSPLIT; ++q) v += part[q * FWD_ROWS + lane];
        if (row < nc) y[c0 + row] = v;
        else upd[s.u[sn] + row - nc] = acc_off[lane] + v;
    }
}

// One backward task: columns [col0, col0 + BWD_COLS) of supernode sn, one
// wavefront per column. lds: nr doubles.
__device__ inline void bwd_task(const DevSym& s, int sn, int col0, double* g, const double* W,
                                const double* y, double* x)
{
    const int c0 = s.c0[sn], nc = s.nc[sn], nr = s.nr[sn];
    const int32_t* roff = s.rows + s.roff[sn];
    for (int k = threadIdx.x; k < nr; k += 256) g[k] = k < nc ? y[c0 + k] : -x[roff[k - nc]];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = col0 + wv;
    if (col < nc) {
        const double* wc = W + s.w[sn] + int64_t(col) * dpanel_ld(nr);
        double acc = 0.0;
        int k = col + lane;
        for (; k + 192 < nr; k += 256)
            acc += wc[k] * g[k] + wc[k + 64] * g[k + 64] + wc[k + 128] * g[k + 128]
                 + wc[k + 192] * g[k + 192];
        for (; k < nr; k += 64) acc += wc[k] * g[k];
        acc = wave_sum(acc);
        if (lane == 0) x[c0 + col] = acc;
    }
}

__global__ __launch_bounds__(256) void k_forward(DevSym s, const int32_t* __restrict__ tsn,
                                                 const int32_t* __restrict__ tfirst,
                                                 int32_t lds_nc, const double* __restrict__ W,
                                                 const double* __restrict__ b,
                                                 const double* __restrict__ scale,
                                                 double* __restrict__ y, double* upd,
                                                 const int32_t* done)
{
    if (done && *done) return;
    extern __shared__ double lds[];
    fwd_task(s, tsn[blockIdx.x], tfirst[blockIdx.x], lds, lds_nc, W, b, scale, y, upd);
}

__global__ __launch_bounds__(256) void k_backward(DevSym s, const int32_t* __restrict__ tsn,
                                                  const int32_t* __restrict__ tfirst,
                                                  const double* __restrict__ W,
                                                  const double* __restrict__ y, double* x,
                                                  const int32_t* done)
{
    if (done && *done) return;
    extern __shared__ double g[];
    bwd_task(s, tsn[blockIdx.x], tfirst[blockIdx.x], g, W, y, x);
}

// Levels whose panels have at most 64 rows: one wavefront per supernode, four
// supernodes per block (tsn lists the level's supernodes; no chunking).
__global__ __launch_bounds__(256) void k_forward_small(DevSym s, const int32_t* __restrict__ tsn,
                                                       int32_t count, const double* __restrict__ W,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ scale,
                                                       double* __restrict__ y, double* upd,
                                                       const int32_t* done)
{
    if (done && *done) return;
    __shared__ double f_all[4][64];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int idx = blockIdx.x * 4 + wv;
    if (idx >= count) return;      // no block barrier below: waves are independent
    double* f = f_all[wv];
    const int sn = tsn[idx];
    const int c0 = s.c0[sn], nc = s.nc[sn], nr = s.nr[sn];
    // f over the panel rows: own columns from b, off rows start at 0
    if (lane < nr) {
        double v = 0.0;
        if (lane < nc) {
            v = b[c0 + lane];
            if (scale) v *= scale[c0 + lane];
        }
        f[lane] = v;
    }
    __builtin_amdgcn_wave_barrier();
    const int cp1 = s.child_ptr[sn + 1];
    for (int cp = s.child_ptr[sn]; cp < cp1; ++cp) {
        const int c = s.child_idx[cp];
        const int64_t uc = s.u[c];
        const int noc = s.nr[c] - s.nc[c];
        if (lane < noc) {
            const int pos = s.relidx[uc + lane];
            const double val = upd[uc + lane];
            f[pos] += pos < nc ? -val : val;
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (lane < nr) {
        const double* wr = W + s.w[sn] + lane;
        const int kmax = lane < nc ? lane + 1 : nc;
        const int ld = dpanel_ld(nr);
        double acc = 0.0;
        for (int k = 0; k < kmax; ++k) acc += wr[int64_t(k) * ld] * f[k];
        if (lane < nc) y[c0 + lane] = acc;
        else upd[s.u[sn] + lane - nc] = f[lane] + acc;
    }
}

__global__ __launch_bounds__(256) void k_backward_small(DevSym s, const int32_t* __restrict__ tsn,
                                                        int32_t count, const double* __restrict__ W,
                                                        const double* __restrict__ y, double* x,
                                                        const int32_t* done)
{
    if (done && *done) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int idx = blockIdx.x * 4 + wv;
    if (idx >= count) return;
    const int sn = tsn[idx];
    const int c0 = s.c0[sn], nc = s.nc[sn], nr = s.nr[sn];
    const int32_t* roff = s.rows + s.roff[sn];
    // lane k holds g_k = y (own columns) or -x (off rows); column c of the
    // panel is contiguous, so each column is one coalesced load per lane
    double gk = 0.0;
    if (lane < nr) gk = lane < nc ? y[c0 + lane] : -x[roff[lane - nc]];
    const double* Ws = W + s.w[sn];
    const int ld = dpanel_ld(nr);
    int c = 0;
    for (; c + 3 < nc; c += 4) {      // four columns' loads in flight
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            v[q] = (lane >= c + q && lane < nr) ? Ws[int64_t(c + q) * ld + lane] * gk : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double t = wave_sum(v[q]);          // total in lane 0
            if (lane == 0) x[c0 + c + q] = t;
        }
    }
    for (; c < nc; ++c) {
        const double v = (lane >= c && lane < nr) ? Ws[int64_t(c) * ld + lane] * gk : 0.0;
        const double t = wave_sum(v);
        if (lane == 0) x[c0 + c] = t;
    }
}

// Whole substitution pair in one launch. Tasks are listed forward level 0 up
// to the root, then backward from the root down. Blocks claim tasks in
// increasing order from an atomic ticket counter. A task first waits until
// every task it depends on (forward: the children's forward tasks; backward:
// the parent's backward tasks, or for a root its own forward tasks) has
// stamped its flag with this launch's epoch, then runs, publishes its results
// (release fence) and stamps its own flag. Dependencies point only to smaller
// task indices and a task is only ever claimed by a running block, so the
// smallest unfinished claimed task can always proceed: no deadlock, and no
// assumption about how many blocks are resident. The last block to leave
// resets the two counters for the next launch. A wait longer than
// `spin_limit` polls sets *err and abandons the launch instead of hanging.
// ctr[0]: next ticket, ctr[1]: blocks that have left.
__global__ __launch_bounds__(256) void k_sweep(DevSym s, SweepPlan P, int32_t lds_nc,
                                               const double* W, const double* b,
                                               const double* scale, double* y, double* x,
                                               double* upd, int32_t* flags, int32_t epoch,
                                               int32_t* err, int32_t spin_limit,
                                               const int32_t* done, int32_t* ctr)
{
    if (done && *done) return;
    extern __shared__ double lds[];
    __shared__ int32_t bail, task;
    if (threadIdx.x == 0) bail = 0;
    while (true) {
        if (threadIdx.x == 0)
            task = __hip_atomic_fetch_add(&ctr[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int t = task;
        if (t >= P.n_tasks) break;
        const int d0 = P.dep_ptr[t], d1 = P.dep_ptr[t + 1];
        for (int d = d0 + threadIdx.x; d < d1; d += 256) {
            const int dep = P.dep_idx[d];
            int32_t it = 0;
            while (__hip_atomic_load(&flags[dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
                if (++it > spin_limit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    bail = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (bail) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // see the producers' results
        const int sn = P.task_sn[t], first = P.task_first[t];
        if (t < P.n_fwd) fwd_task(s, sn, first, lds, lds_nc, W, b, scale, y, upd);
        else bwd_task(s, sn, first, lds, W, y, x);
        __threadfence();                           // publish this task's results
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(&flags[t], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x == 0) {
        const int32_t left = __hip_atomic_fetch_add(&ctr[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (left == int32_t(gridDim.x) - 1) {
            __hip_atomic_store(&ctr[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctr[1], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------------- reductions helpers

// Block-wide sum of one value per thread (256 threads); result valid in thread 0.
__device__ inline double block_sum(double v, double* red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
    return r;
}

// Marks this block done; returns true in exactly one block (the last).
__device__ inline bool last_block(int32_t* counter)
{
    __shared__ int32_t is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t prev = atomicAdd(counter, 1);
        is_last = (prev == int32_t(gridDim.x) - 1);
        if (is_last) *counter = 0;
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}

// ---------------------------------------------------------- Gram-Schmidt

constexpr int NVMAX = MAXM + 1;

// KState scratch for the reductions lives after the struct in one buffer:
// partials of the current pass, [RED_BLOCKS][NVMAX + 1].

// Sums acc[0..cnt) over the block with one barrier: wavefront shuffles, then
// the four wavefront partials of value i are added by thread i. Result in
// out[i] (LDS) for i < cnt. red: LDS scratch of 4 * (NVMAX + 1) doubles.
template <int N>
__device__ inline void block_sums(const double (&acc)[N], int cnt, double* red, double* out)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if (i < cnt) {
            const double t = wave_sum(acc[i]);
            if (lane == 0) red[wv * (NVMAX + 1) + i] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < cnt) {
        const int i = threadIdx.x;
        out[i] = (red[i] + red[(NVMAX + 1) + i]) + (red[2 * (NVMAX + 1) + i] + red[3 * (NVMAX + 1) + i]);
    }
    __syncthreads();
}

// In the last block: out[i] = sum_b partial[b * stride + i] for i < cnt,
// b < nblk (<= 256), with one partial row per thread and one block reduction.
__device__ inline void reduce_partials(const double* partial, int stride, int nblk, int cnt,
                                       double* red, double* out)
{
    double acc[NVMAX];
    const int b = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NVMAX; ++i)
        acc[i] = (i < cnt && b < nblk) ? partial[int64_t(b) * stride + i] : 0.0;
    block_sums(acc, cnt, red, out);
}

// Pass 1: per-block partial dots V_i^T w, i < nv, into partial[block][i].
__global__ __launch_bounds__(256) void k_gs_dots(int64_t n, const double* __restrict__ V,
                                                 int64_t ldv, int nv,
                                                 const double* __restrict__ w,
                                                 double* partial, const int32_t* done)
{
    if (done && *done) return;
    __shared__ double red[4 * (NVMAX + 1)];
    __shared__ double vals[NVMAX + 1];
    double acc[NVMAX];
#pragma unroll
    for (int i = 0; i < NVMAX; ++i) acc[i] = 0.0;
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < n; r += int64_t(gridDim.x) * 256) {
        const double wr = w[r];
#pragma unroll
        for (int i = 0; i < NVMAX; ++i)
            if (i < nv) acc[i] += wr * V[r + i * ldv];
    }
    block_sums(acc, nv, red, vals);
    if (threadIdx.x < nv) partial[int64_t(blockIdx.x) * (NVMAX + 1) + threadIdx.x] = vals[threadIdx.x];
}

// Every block sums the previous kernel's partials itself (fixed order), so no
// cross-block publication is needed inside a kernel. h1 = sum of pass-1
// partials; w' = w - V h1 in place; pass-2 partials V^T w' and ||w'||^2
// (slot nv) into partial_out.
__global__ __launch_bounds__(256) void k_gs_update(int64_t n, const double* __restrict__ V,
                                                   int64_t ldv, int nv, double* w,
                                                   const double* partial_in, double* partial_out,
                                                   KState* ks, const int32_t* done)
{
    if (done && *done) return;
    __shared__ double h[NVMAX + 1];
    __shared__ double red[4 * (NVMAX + 1)];
    __shared__ double vals[NVMAX + 1];
    reduce_partials(partial_in, NVMAX + 1, gridDim.x, nv, red, h);
    if (blockIdx.x == 0 && threadIdx.x < nv) ks->h1[threadIdx.x] = h[threadIdx.x];
    // nv <= MAXM, so the dots (slots 0..nv-1) and ||w'||^2 (slot nv) fit NVMAX
    double acc[NVMAX];
#pragma unroll
    for (int i = 0; i < NVMAX; ++i) acc[i] = 0.0;
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < n; r += int64_t(gridDim.x) * 256) {
        double wr = w[r];
#pragma unroll
        for (int i = 0; i < NVMAX; ++i)
            if (i < nv) wr -= h[i] * V[r + i * ldv];
        w[r] = wr;
#pragma unroll
        for (int i = 0; i < NVMAX; ++i) {
            if (i < nv) acc[i] += wr * V[r + i * ldv];
            else if (i == nv) acc[i] += wr * wr;
        }
    }
    block_sums(acc, nv + 1, red, vals);
    if (threadIdx.x <= nv) partial_out[int64_t(blockIdx.x) * (NVMAX + 1) + threadIdx.x] = vals[threadIdx.x];
}

// w'' = w' - V h2, ||w''||^2 = ||w'||^2 - ||h2||^2 (w' is already orthogonal
// to working precision after the first pass, so there is no cancellation);
// v_{j+1} = w'' / ||w''||, and column j of Ht = h1 + h2 with Ht(j+1,j) = ||w''||.
// Every block sums the pass-2 partials itself; block 0 records the column.
__global__ __launch_bounds__(256) void k_gs_finish(int64_t n, double* V, int64_t ldv, int nv,
                                                   const double* __restrict__ w,
                                                   const double* partial_in, KState* ks,
                                                   const int32_t* done)
{
    if (done && *done) return;
    __shared__ double h[NVMAX + 1];
    __shared__ double red[4 * (NVMAX + 1)];
    __shared__ double sc;
    reduce_partials(partial_in, NVMAX + 1, gridDim.x, nv + 1, red, h);
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
        }
    }
    __syncthreads();
    const double inv = sc;
    double* vout = V + int64_t(nv) * ldv;
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < n; r += int64_t(gridDim.x) * 256) {
        double wr = w[r];
#pragma unroll
        for (int i = 0; i < NVMAX; ++i)
            if (i < nv) wr -= h[i] * V[r + i * ldv];
        vout[r] = wr * inv;
    }
}

// ------------------------------------------------------- small dense part

constexpr int LD = MAXM + 1;   // LDS row stride (avoids bank conflicts)

// Higham (2005): numerator coefficients of the [13/13] Pade approximant and
// the largest 1-norm at which it meets double-precision backward error.
__constant__ double PADE13[14] = {
    64764752532480000.0, 32382376266240000.0, 7771770303897600.0, 1187353796428800.0,
    129060195264000.0,   10559470521600.0,    670442572800.0,     33522128640.0,
    1323241920.0,        40840800.0,          960960.0,           16380.0,
    182.0,               1.0};
constexpr double THETA13 = 5.371920351148152;

// C = A * B (m x m, row-major, stride LD) by the whole block.
__device__ void mm(const double* A, const double* B, double* C, int m)
{
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx - (idx / m) * m;
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += A[i * LD + k] * B[k * LD + j];
        C[i * LD + j] = s;
    }
    __syncthreads();
}

// Solve Q X = P in place (X overwrites P) by Gaussian elimination with partial
// pivoting; Q is destroyed. Whole block.
__device__ void solve_inplace(double* Q, double* P, int m, int ncol)
{
    __shared__ int piv;
    for (int k = 0; k < m; ++k) {
        if (threadIdx.x == 0) {
            int p = k;
            double best = fabs(Q[k * LD + k]);
            for (int i = k + 1; i < m; ++i)
                if (fabs(Q[i * LD + k]) > best) { best = fabs(Q[i * LD + k]); p = i; }
            piv = p;
        }
        __syncthreads();
        const int p = piv;
        if (p != k) {
            for (int j = threadIdx.x; j < m; j += blockDim.x) {
                const double t = Q[k * LD + j]; Q[k * LD + j] = Q[p * LD + j]; Q[p * LD + j] = t;
            }
            for (int j = threadIdx.x; j < ncol; j += blockDim.x) {
                const double t = P[k * LD + j]; P[k * LD + j] = P[p * LD + j]; P[p * LD + j] = t;
            }
        }
        __syncthreads();
        const double dk = Q[k * LD + k];
        const int rows = m - k - 1;
        for (int idx = threadIdx.x; idx < rows * (m - k + ncol); idx += blockDim.x) {
            const int i = k + 1 + idx / (m - k + ncol);
            const int c = idx % (m - k + ncol);
            const double f = Q[i * LD + k] / dk;
            if (c < m - k) { if (c > 0) Q[i * LD + k + c] -= f * Q[k * LD + k + c]; }
            else P[i * LD + (c - (m - k))] -= f * P[k * LD + (c - (m - k))];
        }
        __syncthreads();
        for (int i = k + 1 + threadIdx.x; i < m; i += blockDim.x) Q[i * LD + k] = 0.0;
        __syncthreads();
    }
    // back substitution, one column per thread
    for (int j = threadIdx.x; j < ncol; j += blockDim.x) {
        for (int i = m - 1; i >= 0; --i) {
            double s = P[i * LD + j];
            for (int k = i + 1; k < m; ++k) s -= Q[i * LD + k] * P[k * LD + j];
            P[i * LD + j] = s / Q[i * LD + i];
        }
    }
    __syncthreads();
}

// H = (I - Ht_m^-1) / gamma into H (row-major, stride LD); uses T1, T2.
__device__ void form_h(const KState* ks, int m, double gamma, double* H, double* T1)
{
    for (int idx = threadIdx.x; idx < m * LD; idx += blockDim.x) {
        const int i = idx / LD, j = idx % LD;
        T1[idx] = (j < m) ? ks->Ht[i + j * (MAXM + 1)] : 0.0;
        H[idx] = (j < m && i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    solve_inplace(T1, H, m, m);           // H = Ht^-1
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m;
        H[i * LD + j] = ((i == j ? 1.0 : 0.0) - H[i * LD + j]) / gamma;
    }
    __syncthreads();
}

// u = e^{tau H} e1 (m entries). Uses 6 matrices of MAXM x LD in `buf`; H is
// overwritten (its storage holds V of the approximant once A = tau H / 2^s).
__device__ void expm_e1(double* H, int m, double tau, double* buf, double* u)
{
    double* A = buf;
    double* A2 = A + MAXM * LD;
    double* A4 = A2 + MAXM * LD;
    double* A6 = A4 + MAXM * LD;
    double* T = A6 + MAXM * LD;
    double* Um = T + MAXM * LD;
    double* Vm = H;
    __shared__ double nrm;
    __shared__ int sq;
    // 1-norm of tau H
    if (threadIdx.x == 0) {
        double best = 0.0;
        for (int j = 0; j < m; ++j) {
            double c = 0.0;
            for (int i = 0; i < m; ++i) c += fabs(H[i * LD + j]);
            best = fmax(best, c);
        }
        nrm = best * tau;
        int s = 0;
        if (nrm > THETA13) s = int(ceil(log2(nrm / THETA13)));
        sq = s;
    }
    __syncthreads();
    const double scl = tau * ldexp(1.0, -sq);
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m;
        A[i * LD + j] = H[i * LD + j] * scl;
    }
    __syncthreads();
    mm(A, A, A2, m);
    mm(A2, A2, A4, m);
    mm(A4, A2, A6, m);
    const double* b = PADE13;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m, o = i * LD + j;
        T[o] = b[13] * A6[o] + b[11] * A4[o] + b[9] * A2[o];
    }
    __syncthreads();
    mm(A6, T, Um, m);
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m, o = i * LD + j;
        T[o] = Um[o] + b[7] * A6[o] + b[5] * A4[o] + b[3] * A2[o] + (i == j ? b[1] : 0.0);
    }
    __syncthreads();
    mm(A, T, Um, m);                        // U
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m, o = i * LD + j;
        T[o] = b[12] * A6[o] + b[10] * A4[o] + b[8] * A2[o];
    }
    __syncthreads();
    mm(A6, T, Vm, m);
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m, o = i * LD + j;
        const double v = Vm[o] + b[6] * A6[o] + b[4] * A4[o] + b[2] * A2[o] + (i == j ? b[0] : 0.0);
        const double uu = Um[o];
        A2[o] = v - uu;   // Q
        A4[o] = v + uu;   // P
    }
    __syncthreads();
    solve_inplace(A2, A4, m, m);            // R = Q^-1 P in A4
    double* R = A4;
    double* S = A6;
    for (int k = 0; k < sq; ++k) {
        mm(R, R, S, m);
        double* t = R; R = S; S = t;
    }
    for (int i = threadIdx.x; i < m; i += blockDim.x) u[i] = R[i * LD];
    __syncthreads();
}

// One block per check offset.
__global__ __launch_bounds__(256) void k_checks(KState* ks, double gamma,
                                                const double* __restrict__ taus, int n_tau,
                                                double tol, double* u_buf, double* est_buf,
                                                int m_max, int update_state)
{
    if (update_state && ks->done) return;
    extern __shared__ double sm[];
    double* H = sm;                          // MAXM x LD
    double* buf = H + MAXM * LD;             // 6 matrices
    double* u = buf + 6 * MAXM * LD;         // MAXM
    double* up = u + MAXM;                   // MAXM
    const int m = ks->m;
    const int c = blockIdx.x;
    const double tau = taus[c];
    form_h(ks, m, gamma, H, buf);
    expm_e1(H, m, tau, buf, u);
    // previous-dimension vector: from the buffer when iterating, recomputed
    // when only evaluating (the basis is unchanged)
    if (m == 1) {
        if (threadIdx.x == 0) up[0] = 1.0;
    } else if (update_state) {
        for (int i = threadIdx.x; i < m - 1; i += blockDim.x) up[i] = u_buf[c * MAXM + i];
    } else {
        form_h(ks, m - 1, gamma, H, buf);
        expm_e1(H, m - 1, tau, buf, up);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double beta = ks->beta;
        const double hnext = ks->Ht[m + (m - 1) * (MAXM + 1)];
        const double paper = beta * hnext * fabs(u[m - 1]);
        // change from the dimension m-1 approximation [u_{m-1}; 0]; for m = 1
        // that approximation is v itself, u_0 = 1
        double d2 = 0.0;
        for (int i = 0; i < m; ++i) {
            const double prev = (m == 1) ? 1.0 : (i < m - 1 ? up[i] : 0.0);
            const double d = u[i] - prev;
            d2 += d * d;
        }
        const double est = ks->breakdown ? 0.0 : fmax(paper, beta * sqrt(d2));
        est_buf[c] = est;
    }
    for (int i = threadIdx.x; i < m; i += blockDim.x) u_buf[c * MAXM + i] = u[i];
    if (last_block(&ks->counter)) {
        if (threadIdx.x == 0) {
            double e = 0.0;
            for (int k = 0; k < n_tau; ++k) e = fmax(e, est_buf[k]);
            ks->est = e;
            const int conv = (e < tol) || ks->breakdown;
            if (update_state) {
                ks->converged = conv;
                if (conv || m >= m_max) ks->done = 1;
            } else {
                ks->converged = conv;
            }
        }
    }
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

__global__ void k_vdd_minus(int64_t count, double vdd, double* buf)
{
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < count; r += int64_t(gridDim.x) * 256)
        buf[r] = vdd - buf[r];
}

inline int grid_for(int64_t n) { return int(std::min<int64_t>((n + 255) / 256, RED_BLOCKS)); }

}  // namespace

void launch_forward(const DevSym& s, const LevelTasks& lv, const double* W, const double* b,
                    const double* scale, double* y, double* upd, const int32_t* done,
                    hipStream_t st)
{
    if (lv.small) {
        k_forward_small<<<(lv.count + 3) / 4, 256, 0, st>>>(s, lv.sn, lv.count, W, b, scale, y, upd,
                                                            done);
        return;
    }
    const size_t lds = sizeof(double) * (size_t(lv.lds_doubles) + FWD_ROWS + 256);
    k_forward<<<lv.count, 256, lds, st>>>(s, lv.sn, lv.first, lv.lds_doubles, W, b, scale, y, upd,
                                          done);
}

void launch_backward(const DevSym& s, const LevelTasks& lv, const double* W, const double* y,
                     double* x, const int32_t* done, hipStream_t st)
{
    if (lv.small) {
        k_backward_small<<<(lv.count + 3) / 4, 256, 0, st>>>(s, lv.sn, lv.count, W, y, x, done);
        return;
    }
    const size_t lds = sizeof(double) * size_t(lv.lds_doubles);
    k_backward<<<lv.count, 256, lds, st>>>(s, lv.sn, lv.first, W, y, x, done);
}

int sweep_max_blocks(size_t lds_bytes)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep, 256, lds_bytes) != hipSuccess)
        return 0;
    return cus * per;
}

hipError_t launch_sweep(const DevSym& s, const SweepPlan& P, int blocks, const double* W,
                        const double* b, const double* scale, double* y, double* x, double* upd,
                        int32_t* flags, int32_t epoch, int32_t* err, int32_t spin_limit,
                        const int32_t* done, int32_t* ctr, hipStream_t st)
{
    const size_t lds = sizeof(double) * size_t(P.lds_doubles);
    k_sweep<<<blocks, 256, lds, st>>>(s, P, P.lds_nc, W, b, scale, y, x, upd, flags, epoch, err,
                                      spin_limit, done, ctr);
    return hipGetLastError();
}

void launch_gs_dots(int64_t n, const double* V, int64_t ldv, int nv, const double* w,
                    double* partial, KState* ks, const int32_t* done, hipStream_t st)
{
    (void)ks;
    k_gs_dots<<<grid_for(n), 256, 0, st>>>(n, V, ldv, nv, w, partial, done);
}

void launch_gs_update(int64_t n, const double* V, int64_t ldv, int nv, double* w,
                      double* partial, KState* ks, const int32_t* done, hipStream_t st)
{
    const int64_t half = int64_t(RED_BLOCKS) * (MAXM + 2);
    k_gs_update<<<grid_for(n), 256, 0, st>>>(n, V, ldv, nv, w, partial, partial + half, ks, done);
}

void launch_gs_finish(int64_t n, double* V, int64_t ldv, int nv, const double* w,
                      const double* partial, KState* ks, const int32_t* done, hipStream_t st)
{
    const int64_t half = int64_t(RED_BLOCKS) * (MAXM + 2);
    k_gs_finish<<<grid_for(n), 256, 0, st>>>(n, V, ldv, nv, w, partial + half, ks, done);
}

size_t checks_lds_bytes() { return sizeof(double) * (7 * MAXM * LD + 2 * MAXM); }

void launch_checks(KState* ks, double gamma, const double* tau, int n_tau, double tol,
                   double* u_buf, double* est_buf, int m_max, int update_state, hipStream_t st)
{
    k_checks<<<n_tau, 256, checks_lds_bytes(), st>>>(ks, gamma, tau, n_tau, tol, u_buf, est_buf,
                                                     m_max, update_state);
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

void launch_vdd_minus(int64_t count, double vdd, double* buf, hipStream_t st)
{
    k_vdd_minus<<<grid_for(count), 256, 0, st>>>(count, vdd, buf);
}

}  // namespace matex

// Device helpers shared by the plain and the batched kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "factor.hpp"
#include "kernels.hpp"

namespace matex {
namespace dev {

// Leading dimension of a panel with nr rows (device twin of panel_ld).
__device__ inline int dpanel_ld(int nr) { return (nr + PANEL_ALIGN - 1) / PANEL_ALIGN * PANEL_ALIGN; }

// Orders one wavefront's LDS accesses around a point where its lanes read
// what other lanes wrote: the wavefront's LDS operations complete in order,
// so only the compiler must keep them on their side.
__device__ inline void wave_sync()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// A double moved across lanes by one DPP pattern (both 32-bit halves).
template <int CTRL>
__device__ inline double dpp(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum over each aligned group of g lanes (g a power of two, 1..64), left in
// every lane of the group. Within 16-lane rows the steps are DPP moves (quad
// permutes, then the half-row and row mirrors, each pairing a lane with one
// holding the other half's partial); across rows, lane shuffles. Every lane
// of the wavefront must be active.
__device__ inline double group_sum(double v, int g)
{
    if (g >= 2) v += dpp<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    if (g >= 4) v += dpp<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    if (g >= 8) v += dpp<0x141>(v);   // row_half_mirror
    if (g >= 16) v += dpp<0x140>(v);  // row_mirror
    if (g >= 32) v += __shfl_xor(v, 16, 64);
    if (g >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

// Wavefront sum, returned in every lane (every lane must be active).
__device__ inline double wave_sum(double v)
{
    v = group_sum(v, 16);
    auto row = [&](int l) {
        return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                                __builtin_amdgcn_readlane(__double2loint(v), l));
    };
    return (row(0) + row(16)) + (row(32) + row(48));
}

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

// The done flag of a Krylov process, read once per block. Another stream (the
// check that decides the process) may set the flag while a block starts, so
// wavefronts reading it themselves can disagree: some return and the rest
// then work on LDS that the returned ones were to fill. Thread 0 reads it,
// the block shares it through LDS; the caller returns on a nonzero value
// after the barrier that follows (block_done below has its own). The flag
// word must not be written again before that barrier.
__device__ inline void done_stage(const int32_t* done, int32_t* flag)
{
    if (threadIdx.x == 0)
        *flag = done ? __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
}

__device__ inline bool block_done(const int32_t* done)
{
    __shared__ int32_t flag;
    done_stage(done, &flag);
    __syncthreads();
    return flag != 0;
}

// Marks this block done among `total` cooperating blocks; returns true in
// exactly one of them (the last to arrive), which also resets the counter.
__device__ inline bool last_of(int32_t* counter, int32_t total)
{
    __shared__ int32_t is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t prev = atomicAdd(counter, 1);
        is_last = (prev == total - 1);
        if (is_last) *counter = 0;
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}

__device__ inline bool last_block(int32_t* counter) { return last_of(counter, int32_t(gridDim.x)); }

constexpr int NVMAX = MAXM + 1;

// Sums acc[0..cnt) over a block of NW wavefronts with one barrier: wavefront
// sums, then the NW wavefront partials of value i are added by thread i in
// wavefront order. Result in out[i] (LDS) for i < cnt. red: LDS scratch of
// NW * (NVMAX + 1) doubles.
template <int N, int NW = 4>
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
        if (NW == 4) {
            out[i] = (red[i] + red[(NVMAX + 1) + i]) + (red[2 * (NVMAX + 1) + i] + red[3 * (NVMAX + 1) + i]);
        } else {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NW; ++q) s += red[q * (NVMAX + 1) + i];
            out[i] = s;
        }
    }
    __syncthreads();
}

// In the last block: out[i] = sum_b partial[b * stride + i] for i < cnt,
// b < nblk (<= 256), with one partial row per thread and one block reduction.
// out[i] = sum_b partial[b * stride + i] for i < cnt, b < nblk, by a block of
// NW wavefronts: value i by wavefront i mod NW, the rows split over its lanes
// (fixed order), then a wavefront sum. Few registers.
template <int NW>
__device__ inline void reduce_partials_waves(const double* partial, int stride, int nblk, int cnt,
                                             double* out)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = wv; i < cnt; i += NW) {
        double s = 0.0;
        for (int b = lane; b < nblk; b += 64) s += partial[int64_t(b) * stride + i];
        s = wave_sum(s);
        if (lane == 0) out[i] = s;
    }
    __syncthreads();
}

template <int NW = 4>
__device__ inline void reduce_partials(const double* partial, int stride, int nblk, int cnt,
                                       double* red, double* out)
{
    double acc[NVMAX];
    const int b = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NVMAX; ++i)
        acc[i] = (i < cnt && b < nblk) ? partial[int64_t(b) * stride + i] : 0.0;
    block_sums<NVMAX, NW>(acc, cnt, red, out);
}

// Pass 1: per-block partial dots V_i^T w, i < nv, into partial[block][i].

constexpr int LD = MAXM + 1;   // LDS row stride (avoids bank conflicts)

// Higham (2005): numerator coefficients of the [13/13] Pade approximant and
// the largest 1-norm at which it meets double-precision backward error.
static __constant__ double PADE13[14] = {
    64764752532480000.0, 32382376266240000.0, 7771770303897600.0, 1187353796428800.0,
    129060195264000.0,   10559470521600.0,    670442572800.0,     33522128640.0,
    1323241920.0,        40840800.0,          960960.0,           16380.0,
    182.0,               1.0};
constexpr double THETA13 = 5.371920351148152;

// The small dense routines take their row stride L as a template argument:
// L = LD for matrices in LDS (at most MAXM rows), a larger L for matrices in
// a global-memory workspace. A matrix buffer holds (L - 1) x L doubles.

// Operands of a k-loop in LDS are loaded KB at a time (indices clamped to the
// matrix, the surplus products dropped), so their latencies overlap; the
// sums keep their order.
constexpr int KB = 8;

// C = A * B (m x m, row-major, stride L) by the whole block.
template <int L = LD>
__device__ inline void mm(const double* A, const double* B, double* C, int m)
{
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx - (idx / m) * m;
        double s = 0.0;
        for (int k0 = 0; k0 < m; k0 += KB) {
            double a[KB], b[KB];
#pragma unroll
            for (int q = 0; q < KB; ++q) {
                const int k = min(k0 + q, m - 1);
                a[q] = A[i * L + k];
                b[q] = B[k * L + j];
            }
#pragma unroll
            for (int q = 0; q < KB; ++q)
                if (k0 + q < m) s += a[q] * b[q];
        }
        C[i * L + j] = s;
    }
    __syncthreads();
}

// Solve Q X = P in place (X overwrites P) by Gaussian elimination with partial
// pivoting (the first row of largest magnitude); Q is destroyed (its
// eliminated entries are left as they are: only the upper triangle is read
// afterwards). Whole block.
template <int L = LD>
__device__ inline void solve_inplace(double* Q, double* P, int m, int ncol)
{
    __shared__ int piv;
    for (int k = 0; k < m; ++k) {
        if (threadIdx.x == 0) {
            int p = k;
            double best = fabs(Q[k * L + k]);
            for (int i = k + 1; i < m; ++i) {
                const double v = fabs(Q[i * L + k]);
                if (v > best) { best = v; p = i; }
            }
            piv = p;
        }
        __syncthreads();
        const int p = piv;
        if (p != k) {
            for (int j = k + threadIdx.x; j < m; j += blockDim.x) {
                const double t = Q[k * L + j]; Q[k * L + j] = Q[p * L + j]; Q[p * L + j] = t;
            }
            for (int j = threadIdx.x; j < ncol; j += blockDim.x) {
                const double t = P[k * L + j]; P[k * L + j] = P[p * L + j]; P[p * L + j] = t;
            }
            __syncthreads();
        }
        const double dk = Q[k * L + k];
        const int rows = m - k - 1, w = m - k - 1 + ncol;
        for (int idx = threadIdx.x; idx < rows * w; idx += blockDim.x) {
            const int i = k + 1 + idx / w;
            const int c = idx - (idx / w) * w;
            const double f = Q[i * L + k] / dk;
            if (c < m - k - 1) Q[i * L + k + 1 + c] -= f * Q[k * L + k + 1 + c];
            else P[i * L + (c - (m - k - 1))] -= f * P[k * L + (c - (m - k - 1))];
        }
        __syncthreads();
    }
    // back substitution, one column per thread
    for (int j = threadIdx.x; j < ncol; j += blockDim.x) {
        for (int i = m - 1; i >= 0; --i) {
            double s = P[i * L + j];
            for (int k = i + 1; k < m; ++k) s -= Q[i * L + k] * P[k * L + j];
            P[i * L + j] = s / Q[i * L + i];
        }
    }
    __syncthreads();
}

// Back substitution X = U^-1 X on one wavefront: U in the upper triangle of
// Q, lane j < ncol solving column j of P in place.
template <int L = LD>
__device__ inline void back_subst_wave(const double* Q, double* P, int m, int ncol)
{
    const int j = threadIdx.x & 63;
    if (j >= ncol) return;
    for (int i = m - 1; i >= 0; --i) {
        double s = P[i * L + j];
        for (int k0 = i + 1; k0 < m; k0 += KB) {
            double u[KB], x[KB];
#pragma unroll
            for (int q = 0; q < KB; ++q) {
                const int k = min(k0 + q, m - 1);
                u[q] = Q[i * L + k];
                x[q] = P[k * L + j];
            }
#pragma unroll
            for (int q = 0; q < KB; ++q)
                if (k0 + q < m) s -= u[q] * x[q];
        }
        P[i * L + j] = s / Q[i * L + i];
    }
}

// Ht_m^-1 into P (row-major, stride L) by Gaussian elimination with partial
// pivoting on one wavefront; Q holds Ht_m (row-major) on entry and U on
// return. Ht_m is upper Hessenberg, so the pivot of column k is row k or
// k + 1 and only row k + 1 is eliminated: the operations of the general
// elimination, whose other multipliers are zero. Lane j owns column j and
// carries rows k and k + 1 of Q and of P (= I initially) in registers; the
// pivot entries come from lane k by readlane; row k + 2 is read ahead.
template <int L = LD>
__device__ inline void hessenberg_inverse(int m, double* Q, double* P)
{
    const int j = threadIdx.x & 63;
    const bool col = j < m;
    auto bcast = [](double v, int lane) {
        return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                                __builtin_amdgcn_readlane(__double2loint(v), lane));
    };
    double qk = col ? Q[j] : 0.0;
    double pk = j == 0 ? 1.0 : 0.0;
    double qn = col && m > 1 ? Q[L + j] : 0.0;
    wave_sync();
    for (int k = 0; k + 1 < m; ++k) {
        const double qnn = col && k + 2 < m ? Q[(k + 2) * L + j] : 0.0;
        double pn = j == k + 1 ? 1.0 : 0.0;
        const double a = bcast(qk, k), b = bcast(qn, k);
        if (fabs(b) > fabs(a)) {
            const double t = qk; qk = qn; qn = t;
            const double tp = pk; pk = pn; pn = tp;
        }
        const double f = bcast(qn, k) / bcast(qk, k);
        if (j > k) qn -= f * qk;
        pn -= f * pk;
        wave_sync();
        if (j < L) { Q[k * L + j] = qk; P[k * L + j] = pk; }
        qk = qn; pk = pn; qn = qnn;
    }
    if (j < L) { Q[(m - 1) * L + j] = qk; P[(m - 1) * L + j] = pk; }
    wave_sync();
    back_subst_wave<L>(Q, P, m, m);
}

// Solve Q X = P in place on one wavefront (m + ncol <= 64): the operations
// and their order are those of solve_inplace. Lane c < m owns column c of Q,
// lane m + c column c of P; every lane scans the pivot column (LDS
// broadcast reads, KB at a time).
template <int L = LD>
__device__ inline void solve_wave(double* Q, double* P, int m, int ncol)
{
    const int lane = threadIdx.x & 63;
    const bool isq = lane < m, isp = lane >= m && lane < m + ncol;
    double* col = isq ? Q + lane : P + (isp ? lane - m : 0);
    for (int k = 0; k < m; ++k) {
        int p = k;
        double best = fabs(Q[k * L + k]);
        for (int i0 = k + 1; i0 < m; i0 += KB) {
            double v[KB];
#pragma unroll
            for (int q = 0; q < KB; ++q) v[q] = fabs(Q[min(i0 + q, m - 1) * L + k]);
#pragma unroll
            for (int q = 0; q < KB; ++q)
                if (i0 + q < m && v[q] > best) { best = v[q]; p = i0 + q; }
        }
        wave_sync();
        if (p != k && ((isq && lane >= k) || isp)) {
            const double t = col[k * L]; col[k * L] = col[p * L]; col[p * L] = t;
        }
        wave_sync();
        const double dk = Q[k * L + k];
        if ((isq && lane > k) || isp) {
            const double top = col[k * L];
            for (int i0 = k + 1; i0 < m; i0 += KB) {
                double f[KB], c[KB];
#pragma unroll
                for (int q = 0; q < KB; ++q) {
                    const int i = min(i0 + q, m - 1);
                    f[q] = Q[i * L + k];
                    c[q] = col[i * L];
                }
#pragma unroll
                for (int q = 0; q < KB; ++q)
                    if (i0 + q < m) col[(i0 + q) * L] = c[q] - (f[q] / dk) * top;
            }
        }
        wave_sync();
    }
    if (isp) {
        for (int i = m - 1; i >= 0; --i) {
            double s = col[i * L];
            for (int k0 = i + 1; k0 < m; k0 += KB) {
                double u[KB], x[KB];
#pragma unroll
                for (int q = 0; q < KB; ++q) {
                    const int k = min(k0 + q, m - 1);
                    u[q] = Q[i * L + k];
                    x[q] = col[k * L];
                }
#pragma unroll
                for (int q = 0; q < KB; ++q)
                    if (k0 + q < m) s -= u[q] * x[q];
            }
            col[i * L] = s / Q[i * L + i];
        }
    }
}

// H_m from the process's Arnoldi matrix Ht_m into H (row-major, stride L);
// uses T1. Rational space (X1 = C + gamma G, gamma > 0; Sec. 3.3.2):
// H_m = (I - Ht_m^-1) / gamma. Inverted space (X1 = G, passed as gamma = 0;
// Sec. 3.3.1): the process runs on G^-1 C = -A^-1, so H_m = -Ht_m^-1.
template <int L = LD>
__device__ inline void form_h(const KState* ks, int m, double gamma, double* H, double* T1)
{
    for (int idx = threadIdx.x; idx < m * L; idx += blockDim.x) {
        const int i = idx / L, j = idx % L;
        T1[idx] = (j < m) ? ks->Ht[i + j * (MAXM + 1)] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x < 64) hessenberg_inverse<L>(m, T1, H);   // H = Ht^-1
    __syncthreads();
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m;
        H[i * L + j] = gamma > 0.0 ? ((i == j ? 1.0 : 0.0) - H[i * L + j]) / gamma : -H[i * L + j];
    }
    __syncthreads();
}

// e^{tau H} (m x m, row-major, stride L; m <= L - 1). Uses 6 matrices of
// (L - 1) x L in `buf`; H is overwritten (its storage holds V of the
// approximant once A = tau H / 2^s). Returns the matrix holding the result
// (inside buf), valid until buf is reused.
template <int L = LD>
__device__ inline double* expm_mat(double* H, int m, double tau, double* buf)
{
    double* A = buf;
    double* A2 = A + (L - 1) * L;
    double* A4 = A2 + (L - 1) * L;
    double* A6 = A4 + (L - 1) * L;
    double* T = A6 + (L - 1) * L;
    double* Um = T + (L - 1) * L;
    double* Vm = H;
    __shared__ double nrm;
    __shared__ int sq;
    // 1-norm of tau H: column sums by wavefront 0, then their maximum
    if (threadIdx.x < 64) {
        double best = 0.0;
        for (int j = threadIdx.x; j < m; j += 64) {
            double c = 0.0;
            for (int i0 = 0; i0 < m; i0 += KB) {
                double v[KB];
#pragma unroll
                for (int q = 0; q < KB; ++q) v[q] = H[min(i0 + q, m - 1) * L + j];
#pragma unroll
                for (int q = 0; q < KB; ++q)
                    if (i0 + q < m) c += fabs(v[q]);
            }
            best = fmax(best, c);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) best = fmax(best, __shfl_xor(best, o, 64));
        nrm = best * tau;
    }
    if (threadIdx.x == 0) {
        // a non-finite norm gives no squarings (the result is then NaN, as
        // it must be) instead of an unbounded count
        int s = 0;
        if (nrm > THETA13 && nrm < 1e300) s = int(ceil(log2(nrm / THETA13)));
        sq = min(s, 1100);
    }
    __syncthreads();
    const double scl = tau * ldexp(1.0, -sq);
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m;
        A[i * L + j] = H[i * L + j] * scl;
    }
    __syncthreads();
    mm<L>(A, A, A2, m);
    mm<L>(A2, A2, A4, m);
    mm<L>(A4, A2, A6, m);
    const double* b = PADE13;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m, o = i * L + j;
        T[o] = b[13] * A6[o] + b[11] * A4[o] + b[9] * A2[o];
    }
    __syncthreads();
    mm<L>(A6, T, Um, m);
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m, o = i * L + j;
        T[o] = Um[o] + b[7] * A6[o] + b[5] * A4[o] + b[3] * A2[o] + (i == j ? b[1] : 0.0);
    }
    __syncthreads();
    mm<L>(A, T, Um, m);                        // U
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m, o = i * L + j;
        T[o] = b[12] * A6[o] + b[10] * A4[o] + b[8] * A2[o];
    }
    __syncthreads();
    mm<L>(A6, T, Vm, m);
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m, o = i * L + j;
        const double v = Vm[o] + b[6] * A6[o] + b[4] * A4[o] + b[2] * A2[o] + (i == j ? b[0] : 0.0);
        const double uu = Um[o];
        A2[o] = v - uu;   // Q
        A4[o] = v + uu;   // P
    }
    __syncthreads();
    if (2 * m <= 64) {                         // R = Q^-1 P in A4
        if (threadIdx.x < 64) solve_wave<L>(A2, A4, m, m);
        __syncthreads();
    } else {
        solve_inplace<L>(A2, A4, m, m);
    }
    double* R = A4;
    double* S = A6;
    for (int k = 0; k < sq; ++k) {
        mm<L>(R, R, S, m);
        double* t = R; R = S; S = t;
    }
    return R;
}

// e^{tau H} by the Taylor polynomial of degree 18 with scaling and squaring:
// A = tau H / 2^s with ||A||_1 <= 1, where the remainder is below
// e / 19! < 2.3e-17 (under the unit roundoff), then s squarings. The
// polynomial is evaluated by Paterson and Stockmeyer's scheme in A^4
// (A^2, A^3, A^4, then four Horner steps: seven products) and needs no
// linear solve, which on one check's m x m system costs more than the
// products. Buffers as for expm_mat; returns the matrix holding the result.
static __constant__ double TAYLOR18[19] = {
    1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0, 1.0 / 40320.0,
    1.0 / 362880.0, 1.0 / 3628800.0, 1.0 / 39916800.0, 1.0 / 479001600.0, 1.0 / 6227020800.0,
    1.0 / 87178291200.0, 1.0 / 1307674368000.0, 1.0 / 20922789888000.0, 1.0 / 355687428096000.0,
    1.0 / 6402373705728000.0};

template <int L = LD>
__device__ inline double* expm_taylor(double* H, int m, double tau, double* buf)
{
    double* A = buf;
    double* A2 = A + (L - 1) * L;
    double* A3 = A2 + (L - 1) * L;
    double* A4 = A3 + (L - 1) * L;
    double* S = A4 + (L - 1) * L;
    double* P = S + (L - 1) * L;
    __shared__ double nrm;
    __shared__ int sq;
    // 1-norm of tau H: column sums by wavefront 0, then their maximum
    if (threadIdx.x < 64) {
        double best = 0.0;
        for (int j = threadIdx.x; j < m; j += 64) {
            double c = 0.0;
            for (int i0 = 0; i0 < m; i0 += KB) {
                double v[KB];
#pragma unroll
                for (int q = 0; q < KB; ++q) v[q] = H[min(i0 + q, m - 1) * L + j];
#pragma unroll
                for (int q = 0; q < KB; ++q)
                    if (i0 + q < m) c += fabs(v[q]);
            }
            best = fmax(best, c);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) best = fmax(best, __shfl_xor(best, o, 64));
        nrm = best * tau;
    }
    if (threadIdx.x == 0) {
        // a non-finite norm gives no squarings (the result is then NaN)
        int s = 0;
        if (nrm > 1.0 && nrm < 1e300) s = int(ceil(log2(nrm)));
        sq = min(s, 1100);
    }
    __syncthreads();
    const double scl = tau * ldexp(1.0, -sq);
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m;
        A[i * L + j] = H[i * L + j] * scl;
    }
    __syncthreads();
    mm<L>(A, A, A2, m);
    mm<L>(A2, A, A3, m);
    mm<L>(A2, A2, A4, m);
    const double* c = TAYLOR18;
    // S = c16 I + c17 A + c18 A^2, then S = B_j + A^4 S for j = 3 .. 0 with
    // B_j = c_{4j} I + c_{4j+1} A + c_{4j+2} A^2 + c_{4j+3} A^3
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m, o = i * L + j;
        S[o] = c[18] * A2[o] + c[17] * A[o] + (i == j ? c[16] : 0.0);
    }
    __syncthreads();
    for (int b = 3; b >= 0; --b) {
        mm<L>(A4, S, P, m);
        for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
            const int i = idx / m, j = idx % m, o = i * L + j;
            P[o] += c[4 * b + 3] * A3[o] + c[4 * b + 2] * A2[o] + c[4 * b + 1] * A[o] +
                    (i == j ? c[4 * b] : 0.0);
        }
        __syncthreads();
        double* t = S; S = P; P = t;
    }
    double* R = S;
    double* T = P;
    for (int k = 0; k < sq; ++k) {
        mm<L>(R, R, T, m);
        double* t = R; R = T; T = t;
    }
    return R;
}

// u = e^{tau H} e1 by expm_taylor.
__device__ inline void expm_e1_taylor(double* H, int m, double tau, double* buf, double* u)
{
    const double* R = expm_taylor(H, m, tau, buf);
    for (int i = threadIdx.x; i < m; i += blockDim.x) u[i] = R[i * LD];
    __syncthreads();
}

// u = e^{tau H} e1 (m entries); buffers as for expm_mat.
__device__ inline void expm_e1(double* H, int m, double tau, double* buf, double* u)
{
    const double* R = expm_mat(H, m, tau, buf);
    for (int i = threadIdx.x; i < m; i += blockDim.x) u[i] = R[i * LD];
    __syncthreads();
}


// One check offset of one Krylov process (block-wide) at dimension m (brk:
// the basis broke down at m): H_m from Ht, u =
// e^{tau H_m} e1 into u_buf[c], the estimate into est_buf[c]; the last of
// the n_sel blocks of the process takes the maximum over the checked
// offsets (sel[0 .. n_sel), or 0 .. n_sel - 1 when sel is null) and decides.
// update_state: iterating (u_buf[c] holds the previous dimension's vector
// and the decision may end the process) or only evaluating a check set on a
// fixed basis.
// sm: 7 * MAXM * LD + 2 * MAXM doubles.
__device__ inline void check_block(KState* ks, int m, int brk, double gamma, const double* taus, int c,
                                   const int32_t* sel, int n_sel, double tol, double* u_buf,
                                   double* est_buf, int m_max, int update_state, double* sm)
{
    double* H = sm;                          // MAXM x LD
    double* buf = H + MAXM * LD;             // 6 matrices
    double* u = buf + 6 * MAXM * LD;         // MAXM
    double* up = u + MAXM;                   // MAXM
    __shared__ double red[4];
    const double tau = taus[c];
    form_h(ks, m, gamma, H, buf);
    expm_e1_taylor(H, m, tau, buf, u);
    // previous-dimension vector: from the buffer when iterating, recomputed
    // when only evaluating (the basis is unchanged)
    if (m == 1) {
        if (threadIdx.x == 0) up[0] = 1.0;
    } else if (update_state) {
        for (int i = threadIdx.x; i < m - 1; i += blockDim.x) up[i] = u_buf[c * MAXM + i];
    } else {
        form_h(ks, m - 1, gamma, H, buf);
        expm_e1_taylor(H, m - 1, tau, buf, up);
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
        const double est = brk ? 0.0 : fmax(paper, beta * sqrt(d2));
        est_buf[c] = est;
    }
    for (int i = threadIdx.x; i < m; i += blockDim.x) u_buf[c * MAXM + i] = u[i];
    if (last_of(&ks->counter, n_sel)) {
        double e = 0.0;
        for (int k = threadIdx.x; k < n_sel; k += blockDim.x) e = fmax(e, est_buf[sel ? sel[k] : k]);
        // block maximum through the sum helper's layout
        e = -e;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) e = fmin(e, __shfl_down(e, o, 64));
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        __syncthreads();
        if (lane == 0) red[wv] = -e;
        __syncthreads();
        if (threadIdx.x == 0) {
            double mx = 0.0;
            for (int q = 0; q < int(blockDim.x + 63) / 64; ++q) mx = fmax(mx, red[q]);
            ks->est = mx;
            const int conv = (mx < tol) || brk;
            ks->converged = conv;
            if (update_state) {
                ks->mdec = m;
                if (conv || m >= m_max) ks->done = 1;
            }
        }
    }
}

}  // namespace dev
}  // namespace matex

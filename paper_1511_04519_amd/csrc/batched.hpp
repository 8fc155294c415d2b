// Batched (multi-subtask) kernels of the R-MATEX path (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>

#include "kernels.hpp"

namespace matex {

constexpr int RMAX = 64;           // subtasks per batch (one wavefront lane each)
constexpr int BR = 64;             // panel rows / columns per batched sweep task
constexpr int B_RED_BLOCKS = 4096; // blocks of the batched reductions

// panel columns (forward) / rows (backward) per task of the split schedules
constexpr std::array<int32_t, 3> BATCH_CHUNKS = {64, 128, 256};
constexpr int WAVE_MAX_NC = 32;    // widest supernode a wavefront sweeps alone
constexpr int PSLOT = 64 * RMAX;   // doubles of one partial-result slot (64 x RMAX)

// One block of a batched sweep: panel rows (forward) or columns (backward)
// first .. first + 63 of supernode sn, over the panel columns / rows
// [kb, ke). slot < 0: the task owns the whole range and writes its result;
// otherwise it writes a partial result to slot `slot` of the partial buffer.
struct BTask {
    int32_t sn, first, kb, ke, slot;
};
// Sum of the cnt partial slots slot .. slot + cnt - 1 of one 64-row/column block.
struct BRed {
    int32_t sn, first, slot, cnt;
};

// Forward assembly (pull form), shared by all levels: panel position p of
// supernode s has global index pos_base[s] + p; its sum runs over the
// children's update slots cidx[cptr[g] .. cptr[g + 1]) in a fixed order. A
// diagonal position's btilde is scale * b minus that sum; an off-diagonal
// position's update slot is that sum plus the supernode's own product.
struct BatchAssembly {
    const int32_t* pos_base;
    const int32_t* cptr;
    const int32_t* cidx;
};

// One level of the batched sweeps.
struct BatchLevel {
    const BTask* fwd;
    int32_t n_fwd;
    const BRed* fred;
    int32_t n_fred;
    const BTask* bwd;
    int32_t n_bwd;
    const BRed* bred;
    int32_t n_bred;
    // levels of narrow supernodes (at most WAVE_MAX_NC columns): the
    // supernodes, swept one wavefront each (null: the block tasks above)
    const int32_t* fwave = nullptr;
    int32_t n_fwave = 0;
    const int32_t* bwave = nullptr;
    int32_t n_bwave = 0;
    int32_t wave_nc = 0;   // the level's widest supernode (selects the kernel's register tile)
};

// Multi-right-hand-side pair, all n x R arrays row-interleaved (x[i * R + r]).
// U (n_upd x R) is scratch; y is the forward result; P holds the partial
// results of split tasks (PSLOT doubles per slot).
// rks (or null): ragged inputs, right-hand side r read from block rks[r].m
// of B (a basis of MAXM + 1 blocks of n x R), not from block 0.
void launch_b_forward(const DevSym& s, const BatchAssembly& as, const BatchLevel& lv, int R,
                      const double* W, const double* B, const double* scale, double* y,
                      double* U, double* P, hipStream_t st, const KState* rks = nullptr);
void launch_b_backward(const DevSym& s, const BatchLevel& lv, int R, const double* W,
                       const double* y, double* x, double* P, hipStream_t st);
// Two classical Gram-Schmidt passes for every subtask not yet done; V holds
// MAXM + 1 blocks of n x R. partial: B_RED_BLOCKS * R * (MAXM + 2) doubles.
// act (or null): the subtasks of this pass (others untouched); ragged:
// subtask r at its own iteration ks[r].m (nv = the largest m + 1 of the pass),
// otherwise all at nv.
void launch_b_gs(int64_t n, int R, double* V, int nv, double* w, double* partial, KState* ks,
                 hipStream_t st, const int32_t* act = nullptr, int ragged = 0);
// Estimates for the blocks (chk_col[b], chk_idx[b]); subtask r's blocks are
// chk_idx[col_off[r] .. + col_cnt[r]] (the checks its decision takes the
// maximum over), its offsets taus[tau_off[r] ..], its u vectors and
// estimates live in its region of `cap` checks. update_state as for the
// single-subtask checks.
void launch_b_checks(KState* ks, double gamma, const double* taus, const int32_t* tau_off, int cap,
                     const int32_t* chk_col, const int32_t* chk_idx, const int32_t* col_off,
                     const int32_t* col_cnt, int n_chk, double tol, double* u_buf, double* est_buf,
                     int m_max, int update_state, hipStream_t st);
// Lets the subtasks cols[0 .. cnt) continue iterating.
void launch_b_resume(KState* ks, const int32_t* cols, int cnt, hipStream_t st);
// v = y - y0 + z2 into V_0 for the active subtasks, its norm and a fresh
// state; the other subtasks are marked done, or with keep_others left as
// they are (subtasks that advance independently).
void launch_b_setup(int64_t n, int R, const double* y, const double* y0, const double* z2,
                    double* V, double* partial, KState* ks, const int32_t* active, hipStream_t st,
                    bool keep_others = false);
void launch_b_recon_probes(int64_t n, int R, int n_probe, const int32_t* probe_perm, int n_ent,
                           const int32_t* ent_col, const int32_t* ent_t, const double* ent_tau,
                           const int32_t* ent_u, const double* u_buf, const KState* ks,
                           const double* V, const double* y0, const double* z1, const double* z2,
                           double* Yout, int n_out, hipStream_t st);
void launch_b_recon_full(int64_t n, int R, const double* col_tau, const int32_t* col_u,
                         const double* u_buf, const KState* ks, const int32_t* active,
                         const double* V, double* y, double* y0, const double* z1, const double* z2,
                         hipStream_t st);
// z1 += sum coef[e] Z1[:, q[e]], z2 likewise, for subtask r's events
// e in [ptr[r], ptr[r + 1]) (Z column-major n x columns; z row-interleaved).
void launch_b_spot_cols(int64_t n, int R, const int32_t* ptr, const int32_t* q, const double* coef,
                        const double* Z1, const double* Z2, double* z1, double* z2, hipStream_t st);
void launch_b_events(int cnt, int R, const int32_t* row, const int32_t* col, const double* d,
                     double* s, hipStream_t st);
// out += sgn * (sum over the batch's subtasks).
void launch_b_sum_out(int64_t count, int R, const double* Yout, double sgn, double* out,
                      hipStream_t st);
void launch_b_sum_final(int64_t n, int R, const int32_t* perm, const double* y, double sgn,
                        double* out, hipStream_t st);
void launch_b_fill(int64_t count, double v, double* x, hipStream_t st);
// Column-major natural order (leading dimension n) <-> row-interleaved
// permuted order for R right-hand sides.
void launch_b_interleave(int64_t n, int R, const int32_t* perm, const double* src, double* dst,
                         hipStream_t st);
void launch_b_deinterleave(int64_t n, int R, const int32_t* perm, const double* src, double* dst,
                           hipStream_t st);

}  // namespace matex

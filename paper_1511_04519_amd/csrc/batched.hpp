// Batched (multi-subtask) kernels of the R-MATEX path (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace matex {

constexpr int RMAX = 64;           // subtasks per batch (one wavefront lane each)
constexpr int BR = 64;             // panel rows / columns per batched sweep task
constexpr int BKT = 32;            // LDS tile of the right-hand sides (rows)
constexpr int B_RED_BLOCKS = 4096; // blocks of the batched reductions

// One level of the batched sweeps.
struct BatchLevel {
    const int32_t* sn_list;   // supernodes of the level (assembly)
    int32_t n_sn;
    const int32_t* fwd_sn;    // forward tasks: 64 panel rows each
    const int32_t* fwd_first;
    int32_t n_fwd;
    const int32_t* bwd_sn;    // backward tasks: 64 panel columns each
    const int32_t* bwd_first;
    int32_t n_bwd;
};

// Multi-right-hand-side pair, all n x R arrays row-interleaved (x[i * R + r]).
// T (n x R) and U (n_upd x R) are scratch; y is the forward result.
void launch_b_forward(const DevSym& s, const BatchLevel& lv, int R, const double* W,
                      const double* B, const double* scale, double* T, double* y, double* U,
                      hipStream_t st);
void launch_b_backward(const DevSym& s, const BatchLevel& lv, int R, const double* W,
                       const double* y, double* x, hipStream_t st);
// Two classical Gram-Schmidt passes for every subtask not yet done; V holds
// MAXM + 1 blocks of n x R. partial: B_RED_BLOCKS * R * (MAXM + 2) doubles.
void launch_b_gs(int64_t n, int R, double* V, int nv, double* w, double* partial, KState* ks,
                 hipStream_t st);
// Estimates for the blocks (chk_col[b], chk_idx[b]); subtask r's offsets are
// taus[tau_off[r] ..][tau_cnt[r]], its u vectors and estimates live in its
// region of `cap` checks. update_state as for the single-subtask checks.
void launch_b_checks(KState* ks, double gamma, const double* taus, const int32_t* tau_off,
                     const int32_t* tau_cnt, int cap, const int32_t* chk_col,
                     const int32_t* chk_idx, int n_chk, double tol, double* u_buf, double* est_buf,
                     int m_max, int update_state, hipStream_t st);
void launch_b_setup(int64_t n, int R, const double* y, const double* y0, const double* z2,
                    double* V, double* partial, KState* ks, const int32_t* active, hipStream_t st);
void launch_b_recon_probes(int64_t n, int R, int n_probe, const int32_t* probe_perm, int n_ent,
                           const int32_t* ent_col, const int32_t* ent_t, const double* ent_tau,
                           const int32_t* ent_u, const double* u_buf, const KState* ks,
                           const double* V, const double* y0, const double* z1, const double* z2,
                           double* Yout, int n_out, hipStream_t st);
void launch_b_recon_full(int64_t n, int R, const double* col_tau, const int32_t* col_u,
                         const double* u_buf, const KState* ks, const int32_t* active,
                         const double* V, double* y, double* y0, const double* z1, const double* z2,
                         hipStream_t st);
void launch_b_events(int cnt, int R, const int32_t* row, const int32_t* col, const double* d,
                     double* s, hipStream_t st);
// out -= sum over the batch's subtasks (outputs are filled with Vdd first).
void launch_b_sum_out(int64_t count, int R, const double* Yout, double* out, hipStream_t st);
void launch_b_sum_final(int64_t n, int R, const int32_t* perm, const double* y, double* out,
                        hipStream_t st);
void launch_b_fill(int64_t count, double v, double* x, hipStream_t st);

}  // namespace matex

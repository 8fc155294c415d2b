// Device kernels of the R-MATEX hot path and their launch wrappers (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "schedule.hpp"

namespace matex {

constexpr int MAXM = 32;          // largest Krylov dimension supported
constexpr int RED_BLOCKS = 256;   // blocks of the vector reductions

// Shared (factor-independent) device view of the supernodal structure.
struct DevSym {
    int64_t n;
    const int32_t* c0;
    const int32_t* nc;
    const int32_t* nr;
    const int64_t* roff;
    const int64_t* w;
    const int64_t* u;
    const int32_t* rows;
    const int32_t* child_ptr;
    const int32_t* child_idx;
    const int32_t* relidx;
};

// One level's task list and its kernel: the forward sweep's panel rows per
// block (4, 16 or 64) or the backward sweep's lanes per column (16 or 64).
struct LevelTasks {
    const PTask* tasks;
    int32_t count;
    int32_t lds_doubles;   // forward: max nc of the level; backward: max nr
    int32_t kind;
    int32_t slot;          // entries per task of fdesc / gsrc
    // Per-task tables indexed by block alone, so their loads need no task
    // record (null: the contributor lists / row lists are used instead):
    // forward, the update slots (up to two, -1 none) adding into btilde at
    // column k (entry k < lds_doubles) and into the task's panel row
    // first + i (entry lds_doubles + i);
    const int2* fdesc;
    // backward, the source of g at panel row first + i: x index r >= 0
    // (an off row, negated), -1 - (y index) for an own column, INT32_MIN none.
    const int32_t* gsrc;
};

// Steps of TW items (nr = 0: idle); block b runs forward steps
// fblk[b] .. fblk[b + 1] - 1 (children's levels first) and backward steps
// bblk[b] .. bblk[b + 1] - 1 (root first).
struct TreeTasks {
    const TItem* fitems;
    const TItem* bitems;
    const int32_t* fblk;
    const int32_t* bblk;
    const int2* fdesc;     // per forward item and lane: the LDS slots (offset + 1
                           // in each 16-bit half, 0 none) adding into btilde at
                           // column `lane` (.x) and into panel row first + lane (.y)
    const int32_t* trow;   // per off row: >= 0 global x index, < 0: -1 - LDS offset
    int32_t n_blocks;
    int32_t n_levels;      // levels covered (0 .. n_levels - 1)
    int32_t ws;            // doubles of each wavefront's scratch (>= 64, >= max nr)
    int32_t item_doubles;  // LDS doubles holding a block's items
    int32_t lds_doubles;   // dynamic LDS of a block
    int32_t pad_;
};

// Per-Krylov-process device state (one per instance).
struct KState {
    int32_t done;          // 1 once converged, broken down or at m_max: later kernels return
    int32_t converged;
    int32_t m;             // current dimension
    int32_t breakdown;
    int32_t counter;       // last-block detection of the grid reductions
    int32_t mdec;          // dimension of the last iterating check (0 after set-up)
    int32_t ticket;        // number of the last iteration whose Ht column is written
    int32_t wait_err;      // 1 after a check gave up waiting for its iteration
    double beta;           // ||v||
    double est;            // max estimate over the check set at dimension m
    double nrm2;           // ||w'||^2 after the first Gram-Schmidt pass
    double vscale;         // 1 / ||w''|| for the next basis vector (0 at breakdown)
    double h1[MAXM + 1];   // first Gram-Schmidt pass coefficients
    double h2[MAXM + 1];   // second pass
    double Ht[(MAXM + 1) * MAXM];   // column-major (MAXM+1) x MAXM
    int32_t brk[MAXM];     // brk[j]: the Gram-Schmidt step of iteration j broke down
};

// ---- sweeps: w = (L L^T)^-1 (scale .* b) in the permuted ordering --------
// Forward assembly: the update slots that add into panel position p of a
// supernode are cidx[cptr[pos + p] .. cptr[pos + p + 1]) (child order).
void launch_forward(const LevelTasks& lv, const int32_t* cptr, const int32_t* cidx,
                    const double* W, const double* b, const double* scale, double* y, double* upd,
                    const int32_t* done, hipStream_t st);
// rows: the concatenated off-diagonal row lists.
void launch_backward(const LevelTasks& lv, const int32_t* rows, const double* W, const double* y,
                     double* x, const int32_t* done, hipStream_t st);
void launch_forward_tree(const TreeTasks& tr, const double* W,
                         const double* b, const double* scale, double* y, double* upd,
                         const int32_t* done, hipStream_t st);
void launch_backward_tree(const TreeTasks& tr, const double* W, const double* y, double* x,
                          const int32_t* done, hipStream_t st);

// ---- Gram-Schmidt (two classical passes) -----------------------------------
// partial: 2 * RED_BLOCKS * (MAXM + 2) doubles of scratch (two passes).
void launch_gs_dots(int64_t n, const double* V, int64_t ldv, int nv, const double* w,
                    double* partial, KState* ks, const int32_t* done, hipStream_t st);
void launch_gs_update(int64_t n, const double* V, int64_t ldv, int nv, double* w,
                      double* partial, KState* ks, const int32_t* done, hipStream_t st);
// Publishes the iteration's ticket, ks->ticket + 1 (agent-scope release),
// once its Ht column, m and breakdown flags are written, also when the state
// is done and the kernel does nothing else: the ticket counts the
// iterations launched on the state. No argument changes from one iteration
// to the next, so an iteration can be replayed from a captured graph.
void launch_gs_finish(int64_t n, double* V, int64_t ldv, int nv, const double* w,
                      const double* partial, KState* ks, const int32_t* done, hipStream_t st);
// One thread waits until ks->ticket has reached `ticket` (wrap-safe), so a
// kernel queued after it on another stream sees that iteration's column
// without a cross-stream event. After max_ticks of the 100 MHz device clock
// it gives up: wait_err = 1, done = 1, converged = 0.
void launch_wait_ticket(KState* ks, int32_t ticket, int64_t max_ticks, hipStream_t st);

// ---- small dense part: H_m, exp(tau H_m) e1, estimates, decision ----------
// One workgroup per checked offset: sel[0 .. n_sel) (sel null: offsets
// 0 .. n_sel - 1). u_buf[c*MAXM + i] = (e^{tau_c H_m} e1)_i; when iterating
// (update_state) it also holds the previous dimension's vector.
// m_arg >= 0: check dimension m_arg with iteration m_arg - 1's breakdown
// flag (for a check that runs beside later iterations); -1: the state's m.
void launch_checks(KState* ks, double gamma, const double* tau, const int32_t* sel, int n_sel,
                   double tol, double* u_buf, double* est_buf, int m_max, int update_state,
                   int m_arg, hipStream_t st);
// The process's dimension after a check decided at m (iterations launched
// ahead of that decision may have advanced it).
void launch_set_m(KState* ks, int m, hipStream_t st);
void launch_stamp(int64_t* buf, int64_t idx, hipStream_t st);
// z1 += sum_c coef[c] Z1[:, q[c]] and z2 += sum_c coef[c] Z2[:, q[c]]
// (Z1, Z2: n x columns, column-major).
void launch_spot_update(int64_t n, int cnt, const int32_t* q, const double* coef, const double* Z1,
                        const double* Z2, double* z1, double* z2, hipStream_t st);
// A basis's start in one launch, its small inputs passed by value: the spot
// update above for at most SPOT_ARGS changed columns (cnt = 0: none), then
// launch_setup_v's v = y - y0 + z2 (with the updated z2) and its partial
// sums, and block 0 writes the basis's check offsets to taus. The same
// arithmetic, in the same order, as the separate launches.
constexpr int SPOT_ARGS = 16, TAU_ARGS = 8;
struct SpotArgs {
    int32_t cnt;
    int32_t q[SPOT_ARGS];
    double coef[SPOT_ARGS];
};
struct TauArgs {
    int32_t n;
    double t[TAU_ARGS];
};
void launch_spot_setup(int64_t n, const SpotArgs& sa, const double* Z1, const double* Z2, double* z1,
                       double* z2, const double* y, const double* y0, double* v, double* partial,
                       double* taus, const TauArgs& ta, hipStream_t st);
// Lets a process whose check subset passed but whose full check set did not
// continue iterating.
void launch_resume(KState* ks, hipStream_t st);
// State of a process restarted from a recorded start vector (in V_0) of norm *beta.
void launch_restore_start(KState* ks, const double* beta, hipStream_t st);
// sel = {0, last}: the first and the last check offset.
void launch_set_ends(int32_t* sel, int last, hipStream_t st);

// ---- adjoint ----------------------------------------------------------------
// I[0 .. m) = int_0^tau e^{sH_m} e1 ds, I[MAXM .. MAXM + m) = int_0^tau s e^{sH_m} e1 ds
// for the process's current basis (m <= MAXM - 2); zeros when m = 0.
void launch_adj_integrals(const KState* ks, double gamma, double tau, double* I, hipStream_t st);
// grad[k] += lscale * int over [t_hi - dt, t_hi] of u_k(t) lambda_{row_k}(t) dt
// (pulses linear on the step; lambda = beta V e^{(t_hi - t) H} e1 carried
// divided by lscale).
void launch_adj_amp(int n_src, const int32_t* row, const int64_t* delay, const int64_t* rise,
                    const int64_t* width, const int64_t* fall, int64_t t_hi, int64_t dt,
                    const double* V, int64_t ldv, const KState* ks, const double* I, double lscale,
                    double* grad, hipStream_t st);
// Capacitance gradient (by parts: dJ/dc_i = (1/c_i)(-sum_s g_{s,i} y_i(t_s) +
// int (G lambda)_i y_i dt)). One overlap [t1, t2] of an adjoint step and a
// forward segment: W (ml x mf, row-major stride MAXM), q0 and q1 (MAXM each
// after W) from one block-triangular Van Loan exponential (sig_b = t_hi - t2,
// tau_a = t1 - t_a, h = t2 - t1, seconds).
void launch_cg_block(const KState* kl, double gam_l, const KState* kf, double gam_f, double sig_b,
                     double tau_a, double h, double* Wq, hipStream_t st);
// GV[:, j] = G V[:, j], j < ks->m.
void launch_spmv_cols(int64_t n, const int32_t* rp, const int32_t* ci, const double* gv,
                      const double* V, int64_t ldv, const KState* ks, double* GV, hipStream_t st);
// gc[i] += lscale beta_l / c_i GV_l[i, :] (beta_f W V_f[i, :]^T + q0 (y0_i - z2_i) + q1 z1_i).
void launch_cg_nodes(int64_t n, const double* GVl, const double* Vf, int64_t ldv, const KState* kl,
                     const KState* kf, const double* y0, const double* z1, const double* z2,
                     const double* cperm, const double* Wq, double lscale, double* gc, hipStream_t st);
// lambda[rows[q]] += -(sum of dJdx[pidx[e], s]) / cperm[rows[q]] * inv_scale.
void launch_adj_jump(int n_rows, const int32_t* rows, const int32_t* ptr, const int32_t* pidx,
                     const double* dJdx, int64_t n_out, int s, const double* cperm, double inv_scale,
                     double* lam, hipStream_t st);
size_t checks_lds_bytes();

// ---- segment set-up and reconstruction ------------------------------------
void launch_setup_v(int64_t n, const double* y, const double* y0, const double* z2, double* v,
                    double* partial, KState* ks, hipStream_t st);
void launch_normalize_v(int64_t n, double* v, const double* partial, KState* ks, hipStream_t st);
void launch_scatter_add(int32_t count, const int32_t* idx, const double* val, double* dst,
                        hipStream_t st);
void launch_recon_probes(int n_probe, const int32_t* probe_perm, int n_snap, int32_t snap0,
                         const double* tau, const double* u, const KState* ks, const double* V,
                         int64_t ldv, const double* y0, const double* z1, const double* z2,
                         double* out, int32_t n_out, hipStream_t st);
void launch_recon_full(int64_t n, double tau, const double* u, const KState* ks,
                       const double* V, int64_t ldv, double* y, double* y0, const double* z1,
                       const double* z2, hipStream_t st);
void launch_axpy_scaled(int64_t n, double a, const double* x, double* y, hipStream_t st);
void launch_gather_perm(int64_t n, const int32_t* perm, const double* src, double* dst,
                        int64_t ld_src, int64_t ld_dst, int ncols, hipStream_t st);
void launch_scatter_perm(int64_t n, const int32_t* perm, const double* src, double* dst,
                         int64_t ld_src, int64_t ld_dst, int ncols, hipStream_t st);
void launch_vdd_minus(int64_t count, double vdd, double* buf, hipStream_t st);
// Trapezoidal rule: rhs = C y - hh G y + hh (i(t0) + i(t1)) (hh = h / 2; G in
// CSR in the factor's order; the pulses of row r are sptr[r] .. sptr[r + 1]).
void launch_tr_rhs(int64_t n, const int32_t* rp, const int32_t* ci, const double* gv, const double* cperm,
                   const double* y, double hh, int64_t t0, int64_t t1, const int32_t* sptr, const double* amp,
                   const int64_t* sd, const int64_t* sr, const int64_t* sw, const int64_t* sf, double* rhs,
                   hipStream_t st);
// out[p * n_out + col] = y[probe_perm[p]], p < n_probe.
void launch_gather_probes(int n_probe, const int32_t* probe_perm, const double* y, double* out, int32_t n_out,
                          int32_t col, hipStream_t st);
// *flag = 1 if some a[i], i < count, is NaN or infinite (flag untouched otherwise).
void launch_flag_nonfinite(int64_t count, const double* a, int32_t* flag, hipStream_t st);

}  // namespace matex

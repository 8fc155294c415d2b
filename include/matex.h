/*
 * matex.h - C ABI of the MI355X rational-Krylov (R-MATEX) transient library.
 *
 * Problem (Sec. 2.1, Eq. 1): C x' = -G x + B u(t) for a linear RC power grid.
 * C is the diagonal of node-to-ground capacitances, G the branch-conductance
 * Laplacian plus Norton supply-pad conductances, and B u injects Vdd through
 * the pads and draws piecewise-linear sink currents (trapezoidal pulses, the
 * timing of Fig. 3) out of their nodes. The library works in the droop
 * y = Vdd - x, for which C y' = -G y + i(t) and y(0) = 0.
 *
 * Method (Sec. 3.3.2, R-MATEX): e^{hA} v with A = -C^-1 G is approximated in
 * the rational Krylov space K_m((C + gamma G)^-1 C, v) built by Alg. 1 with
 * X1 = C + gamma G (factored once) and X2 = C:  e^{hA} v ~= ||v|| V_m e^{h H_m} e1,
 * H_m = (I - Ht_m^-1)/gamma (Eq. 9). Alg. 2 steps between transition spots of
 * the piecewise-linear input with Eq. 6 and reuses each basis for every
 * output time (snapshot) before the next spot; sources are grouped into
 * subtasks whose responses add up (Sec. 3.1).
 *
 * Conventions:
 *  - Every function returns matex_status; MATEX_OK is 0. On error, the text of
 *    matex_last_error() (thread-local) says what went wrong; nothing is
 *    written to outputs unless stated.
 *  - "host" pointers are read during the call only and stay owned by the
 *    caller. "device" pointers are HIP device memory owned by the caller
 *    (e.g. torch tensors on cuda:0); the library never frees them.
 *  - stream: a hipStream_t (NULL = default stream). Device work is enqueued
 *    on it; calls that must read a decision back from the device
 *    (matex_krylov_step, matex_transient) synchronise that stream.
 *  - All floating point is IEEE binary64. Times are integer femtoseconds in
 *    problem descriptions and seconds (double) in matex_krylov_step.
 *  - The library needs a gfx950 device; it has no CPU fallback and returns
 *    MATEX_E_HIP if HIP reports an error.
 */
#ifndef MATEX_H
#define MATEX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MATEX_OK = 0,
    MATEX_E_INVALID = 1,     /* bad argument (sizes, ranges, ordering)          */
    MATEX_E_NOT_SPD = 2,     /* a pivot of C + gamma G or G was not positive      */
    MATEX_E_OOM = 3,         /* host or device allocation failed                  */
    MATEX_E_HIP = 4,         /* a HIP runtime call failed                         */
    MATEX_E_NOCONV = 5,      /* estimate still >= tol at m_max (and at h_min)     */
    MATEX_E_UNSUPPORTED = 6, /* valid request outside what the library implements */
    MATEX_E_NONFINITE = 7    /* a result came out NaN or infinite (outputs are
                                written; the text names which ones)            */
} matex_status;

typedef struct matex_factor_s* matex_factor_t;

/* A linear RC grid (host arrays). Node ids are 0..n-1. */
typedef struct {
    int64_t n;
    int64_t n_branch;
    const int32_t* br_a;     /* [n_branch] branch end nodes                      */
    const int32_t* br_b;     /* [n_branch]                                       */
    const double* br_g;      /* [n_branch] conductance (S), > 0                  */
    const double* c_node;    /* [n] capacitance to ground (F), > 0               */
    int32_t n_pad;
    const int32_t* pad_node; /* [n_pad] nodes tied to Vdd through pad_g          */
    const double* pad_g;     /* [n_pad] pad conductance (S), > 0                 */
    double vdd;              /* supply voltage (V)                               */
    const int32_t* coord;    /* optional [n][3] grid coordinates (layer, i, j)
                                used by the nested-dissection ordering; NULL
                                falls back to a graph-distance coordinate       */
} matex_netlist;

typedef struct {
    int32_t n_shifts;        /* shifts gamma_k = gamma * 10^-k, k < n_shifts
                                (default 6 when 0; with gamma = 10 ps, gamma_4
                                is 1 fs, the time quantum, and gamma_5 the
                                step-down rung for 1 fs steps of the adjoint):
                                one factor of C + gamma_k G each, plus one of
                                G, all factored once                            */
    int32_t leaf_max;        /* nested-dissection leaf size (default 16 when 0) */
    int32_t subtree_levels;  /* bottom levels the one-vector sweeps take as
                                whole subtrees, one workgroup each, in one
                                launch per sweep: 0 = automatic, -1 = none,
                                k > 0 = at most k (levels whose supernodes
                                have more than 64 columns or 256 rows are
                                never taken)                                   */
    int32_t batched_schedule; /* schedule of the multi-right-hand-side sweeps:
                                0 = autotuned at factor time (per level, the
                                fastest of split tasks over 64, 128 or 256
                                panel columns/rows and, on levels of
                                supernodes of at most 32 columns, one
                                wavefront per supernode, timed on the factor
                                of C + gamma G); 1 = fixed (256-column split
                                tasks on every level); 2 = fixed (one
                                wavefront per supernode where allowed, else
                                64-column split tasks). With the environment
                                variable MATEX_TUNE_CACHE naming a file, 0
                                first looks the factor's structure up there
                                and takes the recorded choice (no timing),
                                else tunes and appends its choice          */
} matex_factor_opts;

typedef struct {
    int64_t n;
    int64_t nnz_l;           /* entries of one factor's lower triangle as stored */
    int64_t panel_doubles;   /* doubles of one factor's panels (nr x nc each)    */
    int32_t n_supernodes;
    int32_t n_levels;
    int32_t n_shifts;
    int32_t max_nr;
    double gamma;
    double seconds_analyse;  /* host ordering + symbolic                         */
    double seconds_numeric;  /* host numeric factorisation, all factors           */
    int64_t device_bytes;    /* device memory held by the handle                 */
    int32_t subtree_levels;  /* bottom levels swept as whole subtrees          */
    int32_t subtree_blocks;  /* workgroups of those subtree sweeps             */
    int64_t nnz_l_exact;     /* structural nonzeros of one factor L in this
                                ordering, diagonal included (what a solve
                                must read; nnz_l adds the explicit zeros of
                                the supernodal panels)                         */
    int64_t n_upd;           /* forward update slots per right-hand side (the
                                off-diagonal rows of all supernodes)           */
    double seconds_tune;     /* device time spent choosing the batched schedule */
} matex_factor_info;

/*
 * matex_factor - LU_Decompose(X1) of Alg. 2 (Sec. 3.2) for R-MATEX: factor
 * C + gamma_k G (Sec. 3.3.2, X1) for every shift of the ladder, and G (for the
 * F and P terms of Eq. 6), once, on one nested-dissection ordering, and upload
 * the factors. gamma > 0 (seconds). The handle owns its device memory and is
 * read-only afterwards; concurrent calls may share it if they use different
 * streams and their own output buffers.
 * Errors: MATEX_E_INVALID (n <= 0, a node id out of range, a non-positive
 * conductance or capacitance, gamma <= 0), MATEX_E_NOT_SPD, MATEX_E_OOM,
 * MATEX_E_HIP.
 */
matex_status matex_factor(const matex_netlist* nl, double gamma, const matex_factor_opts* opts,
                          void* stream, matex_factor_t* out);
matex_status matex_factor_free(matex_factor_t f);
matex_status matex_factor_get_info(matex_factor_t f, matex_factor_info* info);
/* Text description of the factor's sweep schedules (one line per level: its
 * supernodes and the multi-right-hand-side schedule kept) into buf
 * (NUL-terminated, truncated to len); returns the full length. */
size_t matex_factor_describe(matex_factor_t f, char* buf, size_t len);

/*
 * matex_solve - one forward/backward substitution pair (Alg. 1, the step
 * U \ (L \ b)) with factor `which`: k in [0, n_shifts) for C + gamma_k G,
 * -1 for G. Computes x = A^-1 (diag(scale) b) for nrhs right-hand sides.
 * d_b, d_x: device, n x nrhs column-major (leading dimension n), natural node
 * order; d_scale: device [n] or NULL (no scaling). d_b and d_x may not alias.
 * nrhs = 1 runs the one-vector sweeps of the plain mode; nrhs > 1 the
 * multi-right-hand-side sweeps of the batched mode, 64 columns at a time
 * (this call then synchronises the stream: it frees its staging buffers).
 */
matex_status matex_solve(matex_factor_t f, int32_t which, int32_t nrhs, const double* d_b,
                         const double* d_scale, double* d_x, void* stream);

/*
 * matex_solve_noalloc - matex_solve for one right-hand side (nrhs = 1) that
 * allocates nothing: for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same arguments and result as matex_solve with nrhs = 1 (the
 * same kernels in the same order, so the same bits). Its scratch (the
 * permuted b, x and scale, the forward result and the update slots:
 * 3 n + n_upd doubles, see matex_factor_info) lives in a library-owned
 * device array of 64 MiB (8 Mi doubles) per GPU, held until the process
 * ends; a factor that needs more is refused with MATEX_E_INVALID before any
 * device work. Every call on one GPU uses that GPU's one array: calls that
 * overlap on one GPU (other streams, other host threads) race and must be
 * serialised by the caller. Asynchronous: nothing is synchronised.
 * Errors: MATEX_E_INVALID, MATEX_E_HIP.
 */
matex_status matex_solve_noalloc(matex_factor_t f, int32_t which, const double* d_b,
                                 const double* d_scale, double* d_x, void* stream);

/*
 * matex_krylov_step - e^{tau_k A} v_r (Eq. 9) for every tau_k and every
 * right-hand side v_r, with one rational Krylov basis per v_r (Alg. 1 with
 * X1 = C + gamma_s G, X2 = C; shift index `shift` of the ladder), or with
 * shift = -1 one inverted Krylov basis (X1 = G, X2 = C, Sec. 3.3.1).
 * d_v: device, n x nrhs column-major, natural order. tau: host [n_tau],
 * seconds, > 0. Stops at the first m whose estimate is < tol for every tau
 * (the estimate is the larger of the empirical form of Sec. 3.3.3 and the
 * change from dimension m-1), or at m_max (<= 32).
 * d_out: device, n x nrhs x n_tau, out[i + n*(r + nrhs*k)].
 * m_used, est: host [nrhs] (may be NULL). Returns MATEX_E_NOCONV if some
 * right-hand side did not converge; d_out, m_used and est are still written.
 */
matex_status matex_krylov_step(matex_factor_t f, int32_t shift, int32_t nrhs, const double* d_v,
                               int32_t n_tau, const double* tau, int32_t m_max, double tol,
                               double* d_out, int32_t* m_used, double* est, void* stream);

/* Pulse current sinks (host arrays). Times in fs, delay >= 0, rise > 0,
 * fall > 0, width >= 0; amplitude in A. group[k] in [0, n_group): the subtask
 * of source k (Sec. 3.1 grouping); NULL puts every source in subtask 0. */
typedef struct {
    int32_t n_src;
    const int32_t* node;
    const double* amp;
    const int64_t* delay;
    const int64_t* rise;
    const int64_t* width;
    const int64_t* fall;
    const int32_t* group;
    int64_t t_end;           /* end of the window (fs), > 0                     */
    int32_t n_out;
    const int64_t* t_out;    /* [n_out] output times (fs), strictly increasing,
                                within [0, t_end]                                */
    int32_t n_probe;
    const int32_t* probe;    /* [n_probe] node ids reported at every t_out       */
} matex_problem;

typedef enum { MATEX_PLAIN = 0, MATEX_BATCHED = 1 } matex_mode;

/* The Krylov subspace of Alg. 1. MATEX_RATIONAL: R-MATEX (Sec. 3.3.2),
 * X1 = C + gamma_k G with the shift ladder, H_m = (I - Ht_m^-1) / gamma_k.
 * MATEX_INVERTED: I-MATEX (Sec. 3.3.1), X1 = G (the factor's last panel
 * set), X2 = C, H_m = H'_m^-1 with H' the Arnoldi matrix of A^-1; one
 * factor, so a step that does not converge within m_max is only halved.
 * Both use the empirical estimate of Sec. 3.3.3 with the difference term. */
typedef enum { MATEX_RATIONAL = 0, MATEX_INVERTED = 1 } matex_krylov;

typedef struct {
    double tol;              /* per-basis error estimate bound (V), > 0          */
    int32_t m_max;           /* largest Krylov dimension, 1..32                  */
    int32_t mode;            /* MATEX_PLAIN or MATEX_BATCHED (see below)         */
    int64_t h_min;           /* smallest step after halving (fs), >= 1           */
    double shift_ratio;      /* ladder rule: a step uses the largest gamma_k with
                                tau_1 >= shift_ratio * gamma_k (0 = default 1.0)  */
    int32_t output_droop;    /* 0: outputs are x = Vdd - y; 1: the droop y itself
                                (no supply offset, full relative precision)     */
    int32_t batched_independent; /* MATEX_BATCHED only. 0: lockstep generations
                                (every subtask takes one step per generation;
                                slope changes by G solves of the whole
                                batch). 1: each subtask advances on its own
                                (a converged subtask starts its next step
                                while the others iterate; slope changes from
                                solved columns of the sources' pulse timings;
                                lockstep when those do not fit half the free
                                memory); the same steps and results to
                                rounding, more pairs on the 1M-node workload  */
    int32_t krylov;          /* MATEX_RATIONAL (0) or MATEX_INVERTED (1); with
                                MATEX_INVERTED, batched subtasks run in
                                lockstep, and matex_adjoint refuses it        */
    int32_t reserved_;       /* 0                                               */
} matex_run_opts;

typedef struct {
    int64_t subtasks;
    int64_t segments;        /* steps taken (after ladder cuts and halvings)    */
    int64_t bases;           /* Krylov bases generated                          */
    int64_t solve_pairs_m;   /* substitution pairs with C + gamma_k G, counting
                                in the plain mode the iterations computed
                                ahead of a stopping decision and discarded   */
    int64_t solve_pairs_g;   /* right-hand sides solved with G: in the plain
                                mode two per source row of a subtask
                                (G^-1 e_k and G^-1 C G^-1 e_k, solved 64 at a
                                time once, then combined at each transition
                                spot), or two per spot when those columns do
                                not fit half the free device memory          */
    int64_t krylov_dims;     /* sum of m over bases                             */
    int32_t m_peak;
    int32_t halvings;
    int32_t shift_downs;
    int32_t pad_;
    double seconds;          /* wall time of the call                           */
} matex_stats;

/*
 * matex_transient - Alg. 2 for every subtask of the problem, summed by
 * superposition (Sec. 3.1-3.2). Writes x = Vdd - sum_k y_k (or the droop
 * sum_k y_k with o->output_droop) at the probes:
 * d_probe_out device [n_probe][n_out] (row-major), and, if d_final is not
 * NULL, x(t_end) at every node: device [n], natural order. Each subtask
 * starts from y_k(0) = G^-1 i_k(0) = 0 (no source draws current at t = 0).
 * Step rule: a basis is built at every transition spot of the subtask and
 * reused for the output times before the next spot; the shift of the ladder
 * is chosen from the first check offset tau_1 of the step (the largest
 * gamma_k with tau_1 >= shift_ratio * gamma_k; below the top shift the step ends at
 * the last check offset <= 10 gamma_k); without convergence at m_max the
 * step is retried one shift lower, and with the smallest shift it is halved
 * down to h_min. Stats may be NULL.
 * Modes: MATEX_PLAIN runs the subtasks one after another. MATEX_BATCHED runs
 * up to 64 subtasks together: subtasks that use the same shift share one
 * multi-right-hand-side substitution pair per Krylov iteration, each at its
 * own dimension, and each keeps its own Gram-Schmidt, checks and step
 * decisions (those of the plain mode, so both modes take the same steps);
 * see o->batched_lockstep for how their steps are scheduled. In stats, solve_pairs_m and
 * solve_pairs_g then count multi-right-hand-side pairs; bases, segments and
 * krylov_dims count per subtask.
 * Errors: MATEX_E_INVALID (also for an unknown mode), MATEX_E_NOCONV,
 * MATEX_E_OOM, MATEX_E_HIP, MATEX_E_NONFINITE (an output is NaN or Inf).
 */
matex_status matex_transient(matex_factor_t f, const matex_problem* p, const matex_run_opts* o,
                             double* d_probe_out, double* d_final, matex_stats* stats,
                             void* stream);

/*
 * matex_trapezoidal - the trapezoidal rule (Eq. 2) at a fixed step h, the
 * comparator of the paper's runtime tables (Sec. 4.3, Tab. 3: TR at 10 ps):
 * (C/h + G/2) y_{k+1} = (C/h - G/2) y_k + (i(t_k) + i(t_{k+1})) / 2 in the
 * droop form, y(0) = G^-1 i(0), steps at t_k = k h up to p->t_end, the
 * pulses sampled at the step ends only (no cut at transition spots, as a
 * fixed-step run does). f must be a factor made with gamma = h / 2 (any
 * n_shifts): C + (h/2) G = h (C/h + G/2) is then its first shift, G its last.
 * h_fs > 0 must divide t_end and every output time. o: only o->output_droop
 * is read (o->tol, o->m_max, o->mode are ignored). Outputs as
 * matex_transient (all sources together; groups ignored). stats: segments =
 * solve_pairs_m = steps. Synchronises `stream`.
 * Errors: MATEX_E_INVALID (also for a factor of another gamma), MATEX_E_OOM,
 * MATEX_E_HIP, MATEX_E_NONFINITE.
 */
matex_status matex_trapezoidal(matex_factor_t f, const matex_problem* p, int64_t h_fs, const matex_run_opts* o,
                               double* d_probe_out, double* d_final, matex_stats* stats, void* stream);

/*
 * matex_transient_many - matex_transient for n_inst independent problems,
 * each with its own factor (an uneven batch: grids of different sizes),
 * advanced concurrently: the instances, largest first (nodes times sources),
 * go to `n_streams` workers (0 = 4, at most 16), each a host thread driving
 * its own library-owned HIP stream of default priority, so the GPU overlaps
 * the instances' kernels. Instance k uses f[k], p[k], o[k] and writes
 * d_probe_out[k] (and d_final[k] when d_final is not NULL) as
 * matex_transient does; stats: [n_inst] or NULL. The call first synchronises
 * `stream` (the inputs may come from it) and returns when every instance is
 * done. Each instance takes the same steps and gives the same results as a
 * matex_transient call on its own. Errors: those of matex_transient, for the
 * first instance that failed (the text names it); the remaining instances
 * are then not started.
 */
matex_status matex_transient_many(int32_t n_inst, const matex_factor_t* f, const matex_problem* p,
                                  const matex_run_opts* o, double* const* d_probe_out,
                                  double* const* d_final, matex_stats* stats, int32_t n_streams,
                                  void* stream);

/*
 * matex_adjoint - gradients of an objective J of the probe voltages (for
 * example a droop penalty) with respect to the source amplitudes and the node
 * capacitances, by the continuous adjoint of Eq. 5 propagated with the same
 * rational Krylov steps (Sec. 3.3.2) backwards in time. The method itself is
 * not in the paper; only its propagator is.
 *   d_dJdx: device [n_probe][n_out] (row-major, as d_probe_out of
 *           matex_transient) = dJ/dx at the probes and output times; the
 *           output times > 0 whose column is not all zero are the samples.
 *   d_grad_amp: device [n_src] = dJ/da_k (a_k = amp[k]; the pulses' timing
 *           from p), or NULL.
 *   d_grad_c: device [n] = dJ/dc_i (natural node order), or NULL.
 * The adjoint lambda is zero after the last sample, jumps by C^-1 dJ/dy at
 * each sample (y = Vdd - x) and satisfies C lambda' = G lambda between
 * samples. dJ/da_k = int u_k(t) lambda_{n_k}(t) dt (u_k: source k's unit
 * pulse); dJ/dc_i = -int lambda_i y_i' dt, evaluated integrated by parts as
 * (1/c_i) (-sum_s dJ/dy_i(t_s) y_i(t_s) + int (G lambda)_i y_i dt) over a
 * forward run of all sources together that records each segment's start
 * vector (device memory: about segments x (n + 1) doubles, refused with
 * MATEX_E_OOM beyond 80 % of the free memory) and is taken at o->tol / 100.
 * Adjoint steps end at the samples and at every source's transition spots,
 * and after each jump grow geometrically from 1 fs; o->tol bounds each
 * step's estimate relative to the largest jump norm ||C^-1 dJ/dy(t_s)||_2
 * (about 1e-11 is the practical floor), o->m_max must be <= 30, o->mode and
 * o->output_droop are ignored. Synchronises `stream`.
 * Errors: MATEX_E_INVALID, MATEX_E_NOCONV, MATEX_E_OOM, MATEX_E_HIP,
 * MATEX_E_NONFINITE (a gradient is NaN or Inf, e.g. from a non-finite
 * d_dJdx; the gradients are still written).
 */
matex_status matex_adjoint(matex_factor_t f, const matex_problem* p, const matex_run_opts* o,
                           const double* d_dJdx, double* d_grad_amp, double* d_grad_c,
                           void* stream);

/*
 * matex_time_solves - `reps` substitution pairs (Alg. 1, U \ (L \ (C v)))
 * with factor `which` (as in matex_solve), back to back on `stream`, on
 * library-owned device vectors, timed with HIP events recorded on that
 * stream around the batch. nrhs = 1 times the one-vector sweeps of the plain
 * mode; nrhs in 2..64 the multi-right-hand-side sweeps of the batched mode
 * (nrhs subtasks per pair). Writes the mean seconds per pair to *seconds and
 * the algorithmic bytes of one pair to *bytes: each nonzero of L read once
 * per sweep (8 B, nnz_l_exact) and, per right-hand side, the right-hand
 * side and result of both sweeps (4 x 8 B per row). For measurement only.
 */
matex_status matex_time_solves(matex_factor_t f, int32_t which, int32_t nrhs, int32_t reps,
                               double* seconds, double* bytes, void* stream);

/*
 * matex_sync - waits for the work the library enqueued on `stream` (NULL =
 * default stream) and reports what HIP reports: an asynchronous device fault
 * of an earlier call surfaces here (or at the next call) as MATEX_E_HIP,
 * with HIP's text in matex_last_error(). MATEX_OK when the stream is idle
 * and no error is pending.
 */
matex_status matex_sync(void* stream);

/* Copies the calling thread's last error text (NUL-terminated) into buf. */
size_t matex_last_error(char* buf, size_t len);
const char* matex_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MATEX_H */

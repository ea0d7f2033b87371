/*
 * dicod.h -- C ABI of the MI355X (gfx950) library for convolutional sparse
 * coding by locally greedy convolutional coordinate descent (LGCD).
 *
 * The problem (Moreau, Oudre & Vayatis, ICML 2018, Sec. 2.1, eq. (2)):
 *
 *     min_Z  E(Z) = 1/2 || X - sum_k Z_k * D_k ||_2^2 + lambda sum_k ||Z_k||_1
 *
 * with a signal X of P channels and length T, K atoms D_k of P channels and
 * length W, and activations Z_k of length L = T - W + 1 (eq. (1)).  The
 * solver runs the locally greedy coordinate descent of Algorithm 3 over M
 * time segments (Sec. 2.2, the DICOD segments C_m): each segment picks the
 * coordinate with the largest |Delta Z| (eq. (pb_coord)) inside itself and
 * applies the beta update of eq. (3).  The segments are coloured m % C; the
 * segments of one colour run at the same time, one GPU workgroup each, then
 * the next colour (C = 2 is an even/odd schedule); an update whose window
 * reaches a neighbouring segment writes the neighbour's state directly, which
 * plays the part of the paper's boundary messages (Algorithm 2).  The run stops when every coordinate has
 * |Delta Z| < eps (Sec. 2.1, last paragraph), checked in double precision.
 *
 * Conventions for every entry point:
 *   - All arrays are dense, row-major (C order), and caller-owned.  The
 *     library never keeps a caller pointer after a call returns.
 *   - X is [P][T] (channel-major); D is [K][P][W]; Z is [K][L].
 *   - Host pointers are plain CPU memory.  "_device" entry points take HIP
 *     device pointers on the context's device instead.
 *   - Return value: DICOD_OK (0) on success, DICOD_PENDING (1) from
 *     dicod_poll while a request runs, a negative DICOD_E* code on error.
 *     dicod_last_error() then describes the failure.  No C++ exception
 *     crosses this interface.
 *   - lambda > 0 is absolute.  lambda < 0 is relative: the library uses
 *     |lambda| * lambda_max with lambda_max = max_{k,t} |(D^T X)_k[t]|, the
 *     smallest value for which Z = 0 is optimal.  lambda == 0 or non-finite
 *     is rejected (the paper requires lambda > 0).
 *   - A context is used by one host thread at a time, except dicod_submit /
 *     dicod_poll, which are internally synchronised.
 */
#ifndef DICOD_H
#define DICOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define DICOD_OK 0
#define DICOD_PENDING 1
#define DICOD_EINVAL (-1)   /* bad argument (message says which)            */
#define DICOD_ENOMEM (-2)   /* device memory or HBM budget exhausted        */
#define DICOD_EDEVICE (-3)  /* HIP runtime error                            */
#define DICOD_ENOTCONV (-4) /* max_phases reached; Z holds the last iterate */
#define DICOD_ENOREQ (-5)   /* unknown request id                           */
#define DICOD_ENOTSUP (-6)  /* shape outside what the kernels support       */

/* ---- precision policies ---------------------------------------------- */
/* FP64: beta/g, S and Z in double throughout the descent.
 * FP32: beta init and the final check in double; the descent keeps g in
 *       float (Z in double) and is refreshed from a double recompute until
 *       the double-precision stop test holds.
 * MIXED: as FP32, but the float state starts from split-bf16 MFMA with fp32
 *       accumulation (three products hi*hi + hi*lo + lo*hi); lambda_max is
 *       made exact by recomputing the near-maximal entries in double, and the
 *       double beta of the check is computed on a second stream during the
 *       first descent round (served requests: a second stream per lane).    */
#define DICOD_PREC_FP64 0
#define DICOD_PREC_FP32 1
#define DICOD_PREC_MIXED 2

/* ---- schedules --------------------------------------------------------- */
/* EVENODD: coloured phases (cfg.colors classes; 2 = even/odd): segments of one
 *          colour run at the same time and write their neighbours' state
 *          directly, so every phase is a sequential order (Algorithm 3).
 * DICOD:   Algorithm 2 with the segments in lockstep: in every phase all
 *          segments with work run at once from their own beta, each keeping
 *          only its own positions; an update whose window reaches a
 *          neighbour is sent to it as (k0, t0, delta) and applied there at
 *          the start of the next phase.  Concurrent updates of adjacent
 *          segments may interfere (Sec. 3, Prop. A.2).  Segments must be
 *          >= W - 1 long and fit the on-chip kernel; update_cap in 1..1024 (or -1) is
 *          the number of updates per segment and phase (1 keeps the message
 *          delay below one update time, hypothesis H3).  dicod_submit always
 *          uses the coloured schedule.
 * ASYNC:   Algorithm 2 without phase barriers: float rounds run persistent
 *          teams that loop over the segments, each segment picking and
 *          applying its own updates as soon as it has work and applying its
 *          neighbours' records whenever it runs, with no wait for any other
 *          segment; concurrent updates of adjacent segments may interfere
 *          (Prop. A.2; convergence under H1, see dicod_check_h1).  A round
 *          ends after a launch that applies no update; the double-precision
 *          check and any double round follow the coloured schedule with
 *          cfg.colors.  Needs the register-state kernel (FP32 or MIXED,
 *          reg_state 1, segments of at most 256 positions, K <= 32,
 *          update_cap in 1..64): ENOTSUP otherwise.  With a trace, update
 *          records carry their number in selection order in n_local, and
 *          every application of a neighbour's record is logged with
 *          k0 = -1 - atom, n_local = that update's number and t0 = the
 *          number of updates selected when it was applied. */
#define DICOD_SCHED_EVENODD 0
#define DICOD_SCHED_DICOD 1
#define DICOD_SCHED_ASYNC 2

typedef struct dicod_ctx dicod_ctx;

typedef struct {
    int device;              /* HIP device ordinal                                  */
    int precision;           /* DICOD_PREC_*                                        */
    int schedule;            /* DICOD_SCHED_*                                       */
    int update_cap;          /* max updates per segment per phase; 0 = no cap;
                              * -1 = automatic: max(4, round(2 sqrt(W)))            */
    int64_t max_phases;      /* watchdog: phases before DICOD_ENOTCONV              */
    int max_refresh;         /* double-precision verify-and-resume rounds (FP32)    */
    int phases_per_poll;     /* phases launched between convergence polls (>= 1)    */
    double inner_eps_factor; /* descent stops at eps * factor before the FP64 test  */
    size_t hbm_budget_bytes; /* serving admission budget; 0 = 80% of free memory    */
    int max_inflight;        /* serving: max signals on the device at once          */
    int timing;              /* 1 = time every LGCD kernel launch with HIP events    */
    int64_t trace_capacity;  /* update records kept for dicod_get_trace (0 = none)  */
    int state_in_lds;        /* 1 = keep a segment's state in LDS when it fits       */
                             /* (else in HBM); 0 = always in HBM                     */
    int fp64_polish_after;   /* FP32: after this many failed double-precision checks */
                             /* the descent continues on a double state; 0 = never   */
    int colors;              /* phase classes C in 2..4: segment m runs in phases p  */
                             /* with p % C == m % C (2 = even/odd); segments must be */
                             /* >= max(W - 1, (2W - 2) / (C - 1)) long                */
    int verify_from_scratch; /* 1 = every stop test recomputes g from Z; 0 = after a  */
                             /* double round the maintained double state is used     */
    int reg_state;           /* 1 = float rounds keep each position's state in the   */
                             /* registers of one thread (segments of at most 256     */
                             /* positions, K <= 32); 0 = LDS / HBM state kernels only */
    int autotune;            /* 1 = solves with n_seg = 0 take colours, update cap   */
                             /* and segment length from the tuning table entry of    */
                             /* their length bucket when one exists                  */
                             /* (dicod_autotune_device); served requests keep the    */
                             /* config's schedule                                    */
    int screen;              /* 1 = after the solve, count the coordinates the Gap    */
                             /* Safe rule proves zero (one more double check pass)   */
} dicod_config;

typedef struct {
    int64_t n_updates;        /* coordinate updates applied                         */
    int64_t n_phases;         /* coloured phases until the stop test held           */
    int64_t n_phase_launches; /* LGCD kernel launches (>= n_phases)                 */
    int64_t n_segment_runs;   /* segment runs that made at least one update         */
    int64_t nnz;              /* non-zeros of the returned Z                        */
    int n_seg;                /* segments M                                         */
    int seg_len;              /* floor(L / M)                                       */
    int converged;            /* 1 if max |Delta Z| < eps held in double            */
    int n_refresh;            /* verify rounds that failed and refreshed g          */
    double lambda;            /* lambda used                                        */
    double lambda_max;        /* max |D^T X| (0 if lambda was absolute and unused)   */
    double eps;
    double objective;         /* E(Z), eq. (2), in double                            */
    double max_dz;            /* max over all coordinates of |Delta Z|, in double    */
    double kkt_on;            /* max |g - lambda sign z| / |D_k|^2 over the support  */
    double kkt_off;           /* max (|g| - lambda)_+ / |D_k|^2 off the support       */
    double max_abs_z;
    double t_init_ms;         /* dictionary-independent setup + beta init            */
    double t_cd_ms;           /* descent phases (wall time of the phase loop)       */
    double t_verify_ms;       /* double-precision checks and refreshes              */
    double t_total_ms;        /* whole call                                         */
    double t_lgcd_kernel_ms;  /* sum of LGCD kernel durations (timing = 1)          */
    int64_t round_updates[4]; /* updates of the first four descent rounds (of the     */
                              /* whole call: a batch's signals share the rounds)     */
    int64_t round_phases[4];  /* phases of the first four descent rounds             */
    double round_ms[4];       /* wall time of the first four descent rounds          */
    double round_kernel_ms[4]; /* phase-kernel time of those rounds (timing = 1)     */
    int64_t round_launches[4]; /* phase-kernel launches of those rounds              */
    int round_state[4];       /* state of those rounds: bit 0 double, bit 1 HBM,     */
                              /* bit 2 registers, bit 3 free-running schedule        */
    int state_in_hbm;         /* 1 if segment state was kept in HBM, not LDS         */
    int polished_fp64;        /* 1 if the descent finished on a double state         */
    double t_queue_ms;        /* served: dicod_submit until admission to the device  */
    double t_latency_ms;      /* served: dicod_submit until the result was complete  */
    double round_max_dz[4];   /* max |Delta Z| of the double check after each of the */
                              /* first four descent rounds                           */
    int colors;               /* phase classes C the solve ran with                  */
    int update_cap;           /* updates per segment per phase it ran with (0: none) */
    int tuned;                /* 1 if colours, cap and M came from the tuning table   */
    int pad_;
    double duality_gap;       /* E(Z) - Dual(theta) >= E(Z) - E(Z*) at the returned Z, */
                              /* theta = R / max(lambda, max |D^T R|) (safe screening) */
    int64_t n_screened;       /* coordinates the Gap Safe sphere rule proves zero     */
                              /* (screen = 1; else -1)                                */
} dicod_stats;

/* One entry of the autotuner's table: the schedule chosen for the signals of
 * one length bucket with one dictionary shape. */
typedef struct {
    int K, P, W;       /* dictionary shape the entry was tuned for              */
    int bucket;        /* floor(log2(L)) of the longest signal of the call       */
    int colors;        /* phase classes C in 2..4                                */
    int seg_len;       /* longest segment: M = ceil(L / seg_len), raised to the
                        * fewest segments of at least the minimum length for C   */
    int update_cap;    /* updates per segment per phase, 1..1024                 */
    int team_threads;  /* threads per segment of the register-state kernel that
                        * segments of seg_len positions take (64, 128 or 256;
                        * 0 = LDS / HBM state kernels); informational            */
    int trials;        /* configurations timed                                   */
    int pad_;
    double ms;         /* best time-to-eps of the chosen schedule while tuning   */
    double ms_prior;   /* time-to-eps of the starting point: 2 colours, segments
                        * of 2W (M = L / (2W), Corollary 1), the automatic cap  */
} dicod_tune_entry;

/* One record per applied update (dicod_get_trace); 32 bytes. */
typedef struct {
    int32_t phase;    /* phase index                          */
    int32_t seg;      /* global segment index                 */
    int32_t k0;       /* atom                                 */
    int32_t n_local;  /* update index within the segment run  */
    int64_t t0;       /* position within the signal           */
    double delta;     /* applied change of Z_{k0}[t0]         */
} dicod_trace_rec;

/* Fills *cfg with the defaults: device 0, FP32, coloured phases, update_cap -1,
 * max_phases 1e6, max_refresh 8, phases_per_poll 16, inner_eps_factor 0.5,
 * timing 0, no trace, state_in_lds 1, fp64_polish_after 1, colors 3,
 * verify_from_scratch 0, reg_state 1, autotune 0, screen 0.  Returns DICOD_OK, or DICOD_EINVAL if
 * cfg is NULL. */
int dicod_config_init(dicod_config *cfg);

/* Creates a context on cfg->device (cfg NULL = defaults) with its own HIP
 * stream.  *out receives the context (NULL on failure).  Errors: EINVAL
 * (bad config), EDEVICE (no such device / HIP failure). */
int dicod_init(dicod_ctx **out, const dicod_config *cfg);

/* Releases every device buffer, the stream and the context.  NULL is a no-op. */
void dicod_finalize(dicod_ctx *ctx);

/* Message of the last error on this context ("" if none); valid until the
 * next call on the context.  ctx NULL gives the message of the last failed
 * dicod_init on this thread. */
const char *dicod_last_error(const dicod_ctx *ctx);

/* Makes D (host, float [K][P][W]) the resident dictionary: copies it to the
 * device and computes, in double on MFMA, the correlation table
 * S_{k,l}[d] = sum_tau <D_k[tau], D_l[tau + d]> for |d| < W (eq. (3)) and the
 * norms |D_k|^2 (eq. (pb_coord)).  Errors: EINVAL (NULL, K/P/W <= 0,
 * non-finite entry, an atom of zero norm, or serving active: once
 * dicod_submit has been called on the context, its serving lanes hold the
 * dictionary until dicod_finalize), ENOTSUP (P > 16 channels, or
 * K * P * W > 2^28), ENOMEM, EDEVICE.  Must not run concurrently with
 * dicod_submit or dicod_poll. */
int dicod_set_dictionary(dicod_ctx *ctx, const float *D, int K, int P, int W);

/* Solves problem (2) for one signal with host buffers.
 *   X      host float [P][T], T >= W
 *   D      host float [K][P][W]; NULL = use the resident dictionary (then K, W
 *          must match it); non-NULL replaces the resident dictionary
 *   lambda see conventions above; eps > 0 is the stop threshold on |Delta Z|
 *   n_seg  number of segments M; 0 = chosen by the library (the largest M
 *          allowed).  M > 1 requires floor(L / M) >= max(W - 1, (2W - 2) / (C - 1))
 *          for C = cfg.colors, so that a window reaches only the adjacent
 *          segments and segments running in the same phase never touch the
 *          same coordinates (Sec. 2.2: an update changes beta on 2W - 1
 *          positions)
 *   Z_out  host double [K][L], written on DICOD_OK and DICOD_ENOTCONV
 *   st     optional statistics
 * Errors: EINVAL, ENOTSUP (segment too long for the on-chip kernel), ENOMEM,
 * EDEVICE, ENOTCONV. */
int dicod_solve(dicod_ctx *ctx, const float *X, int P, int64_t T, const float *D,
                int K, int W, double lambda, double eps, int n_seg, double *Z_out,
                dicod_stats *st);

/* As dicod_solve with the resident dictionary and device buffers:
 *   X_dev device float [P][T]; Z_dev device double [K][L] (written).
 *   stream: hipStream_t to order the work after (NULL = the context's own
 *   stream); the call returns after the result is complete. */
int dicod_solve_device(dicod_ctx *ctx, const float *X_dev, int64_t T, double lambda,
                       double eps, int n_seg, double *Z_dev, dicod_stats *st,
                       void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): dicod_solve_device with
 * every device workspace buffer of the solve carved from a static device
 * array of 128 MiB (one per GPU, held until the process ends) instead of
 * being allocated; the pinned host staging and the events come from
 * dicod_init.  It calls no hipMalloc, hipFree, hipHostMalloc or other
 * allocating routine (the host plan of the segments uses ordinary heap
 * vectors of O(M) bytes).  Arguments, results and errors as
 * dicod_solve_device, plus EINVAL when the problem needs more scratch than the
 * array holds (about 21 bytes per coefficient K * L in the FP32 policy, i.e.
 * up to about 6 M coefficients; the message gives the bytes needed), and
 * EINVAL with timing = 1.  Every call on a GPU shares that GPU's array and
 * leaves its contents behind; a call initialises everything it reads, but
 * calls that overlap on one GPU (from any context or thread) race and must be
 * serialised by the caller. */
int dicod_solve_device_noalloc(dicod_ctx *ctx, const float *X_dev, int64_t T, double lambda,
                               double eps, int n_seg, double *Z_dev, dicod_stats *st,
                               void *stream);

/* Solves n_sig independent signals of different lengths against the resident
 * dictionary in one set of launches: their segments are packed into the same
 * phases (batching).
 *   X_dev   device float, signal i is [P][T[i]] starting at element x_off[i]
 *   T, x_off, z_off: host int64 arrays of n_sig entries
 *   lambda  host double[n_sig] (each with the sign convention above)
 *   n_seg   host int[n_sig] (0 = chosen per signal) or NULL (all chosen)
 *   Z_dev   device double, signal i is [K][T[i]-W+1] starting at z_off[i]
 *   st      optional host array of n_sig stats
 * Errors as dicod_solve; EINVAL names the offending signal. */
int dicod_solve_batch_device(dicod_ctx *ctx, int n_sig, const float *X_dev,
                             const int64_t *T, const int64_t *x_off,
                             const double *lambda, double eps, const int *n_seg,
                             double *Z_dev, const int64_t *z_off, dicod_stats *st,
                             void *stream);

/* ---- autotuning of the schedule ---------------------------------------- */
/* Times complete solves of the given signals (arguments as
 * dicod_solve_batch_device; Z_dev is overwritten by every trial) under
 * candidate schedules -- colours C, longest segment length (which also picks
 * the threads per segment of the register-state kernel) and update cap --
 * starting from 2 colours with segments of 2W, the optimum M* ~ T / (2W) of
 * Corollary 1 (Sec. 3), and moving to the neighbouring candidate that is more
 * than 2% faster (best of two timed solves each) until none is or max_trials
 * (1..64) schedules have been timed.  The choice is stored in the context's
 * tuning table under the length bucket floor(log2(max L)) and written to *out
 * (may be NULL); Z_dev then holds the solution under the chosen schedule.
 * A solve whose schedule comes from the table depends only on the table and
 * the length of its longest signal.  Served requests (dicod_submit) do not
 * use the table: they run the config's colours and cap with the fixed
 * segment rule (a served pair of tuned requests stopped making progress in
 * testing, cause not found; that path is switched off).
 * Errors: EINVAL (as the batch solve; also DICOD schedule, or serving active),
 * ENOMEM, EDEVICE, ENOTCONV (no candidate converged). */
int dicod_autotune_device(dicod_ctx *ctx, int n_sig, const float *X_dev,
                          const int64_t *T, const int64_t *x_off, const double *lambda,
                          double eps, double *Z_dev, const int64_t *z_off, int max_trials,
                          dicod_tune_entry *out);

/* Copies up to cap entries of the tuning table (ascending bucket) into out and
 * their number into *n (out may be NULL with cap 0).  Errors: EINVAL. */
int dicod_get_tuning(dicod_ctx *ctx, dicod_tune_entry *out, int cap, int *n);

/* Stores one entry (e.g. a cached choice from an earlier process) in the
 * tuning table, replacing the entry of its bucket; e NULL empties the table.
 * Errors: EINVAL (shape differs from the resident dictionary, colours outside
 * 2..4, seg_len below the minimum segment for its colours, update_cap outside
 * 1..1024, or serving active). */
int dicod_set_tuning(dicod_ctx *ctx, const dicod_tune_entry *e);

/* Correlation with the resident dictionary, out[k][t] = sum_{p,tau}
 * D_k[p][tau] X[p][t + tau] for t < L (beta at Z = 0, Algorithm 1 init),
 * computed on MFMA with the given precision (DICOD_PREC_FP64: double MFMA;
 * DICOD_PREC_MIXED: split-bf16 MFMA with fp32 accumulation).  X host float
 * [P][T]; out host double [K][L].  Errors: EINVAL, ENOMEM, EDEVICE. */
int dicod_correlate(dicod_ctx *ctx, const float *X, int64_t T, int precision,
                    double *out);

/* Copies the resident correlation table to host double [K][K][2W-1] in the
 * device layout S[l][k][d + W - 1] = S_{k,l}[d] (the slice a change of atom
 * l applies, eq. (3)), and the norms to host double [K] (either may be NULL).
 * Errors: EINVAL (no dictionary). */
int dicod_get_s_table(dicod_ctx *ctx, double *S_out, double *norms_out);

/* Hypothesis H1 of Theorem 1 (Sec. 3) for the resident dictionary: *ratio
 * gets the largest |S_{k,l}[d]| / (|D_k|_2 |D_l|_2) over atoms k, l and shifts
 * d != 0, in double from the resident correlation table (at most 1 by
 * Cauchy-Schwarz).  Algorithm 2 (schedules DICOD and ASYNC) converges when it
 * is below 1; *holds (may be NULL) gets 1 then, else 0.  Errors: EINVAL (NULL
 * ctx or ratio, no dictionary), EDEVICE. */
int dicod_check_h1(dicod_ctx *ctx, double *ratio, int *holds);

/* Copies up to cap update records of the last solve (in the order they were
 * recorded; segments of one phase interleave) into out and the number
 * available into *n.  Requires trace_capacity > 0 in the config. */
int dicod_get_trace(dicod_ctx *ctx, dicod_trace_rec *out, int64_t cap, int64_t *n);

/* ---- serving: continuous batching of encode requests ------------------- */
/* Enqueues one signal (host float [P][T], copied before return) against the
 * resident dictionary; a scheduler thread admits requests while the HBM
 * budget and the in-flight limit allow, packs their segments into the
 * running phases, and retires each one when its own stop test holds
 * (requests that arrive while others run join the next phase).
 * *req_id receives the request id.  Errors: EINVAL, ENOMEM (request larger
 * than the whole budget), EDEVICE. */
int dicod_submit(dicod_ctx *ctx, const float *X, int64_t T, double lambda,
                 double eps, int n_seg, uint64_t *req_id);

/* Non-blocking.  Returns DICOD_PENDING while the request runs; on completion
 * writes Z (host double [K][L]) and st (optional), forgets the request and
 * returns DICOD_OK (or the request's error code).  Unknown id: ENOREQ. */
int dicod_poll(dicod_ctx *ctx, uint64_t req_id, double *Z_out, dicod_stats *st);

#ifdef __cplusplus
}
#endif

#endif /* DICOD_H */

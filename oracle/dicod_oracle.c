/*
 * FP64 CPU oracle for convolutional sparse coding solved by (locally) greedy
 * convolutional coordinate descent, as described in Moreau, Oudre & Vayatis,
 * "DICOD: Distributed Convolutional Coordinate Descent for Convolutional
 * Sparse Coding" (ICML 2018).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU product
 * path shares no code with it and must never call it.
 *
 * Everything is plain, single-threaded double precision, written to be read
 * against the paper:
 *   - model and objective ............ Sec. 2.1, eq. (1) and eq. (2)
 *   - coordinate update Z' ........... Sec. 2.1, eq. (pb_coord) and Sh(u, lambda)
 *   - auxiliary variable beta ........ Sec. 2.1 (definition after eq. (pb_coord))
 *   - beta update .................... Sec. 2.1, eq. (3), with S_{k,l} = D~_k * D_l
 *   - greedy selection / stop ........ Sec. 2.1 (Osher et al. rule), Algorithm 1
 *   - segments C_m ................... Sec. 2.2 (DICOD paragraph)
 *   - locally greedy CD (SeqDICOD) ... Sec. 2.3, Algorithm 3
 *   - cost change of one update ...... Appendix A, Proposition A.1
 *
 * Readings of passages that are ambiguous or inconsistent in the paper:
 *   R1 (beta, Sec. 2.1): beta_k[t] = sum_tau <D_k[tau], R[t+tau]> + |D_k|^2 Z_k[t]
 *      with R = X - sum_k Z_k * D_k ("valid" correlation, t in [0, L)).
 *   R2 (eq. (3) sign): with delta = Z_new - Z_old the update is
 *      beta_k[t] -= S_{k,k0}[t - t0] * delta for (k,t) != (k0,t0); the paper's
 *      Delta Z = Z - Z' would flip the sign.  beta_{k0}[t0] is left unchanged.
 *   R3 (S index): S_{k,l}[d] = sum_tau <D_k[tau], D_l[tau + d]>, zero for
 *      |d| >= W.
 *   R4 (ties): the argmax takes the largest |Delta Z|; ties go to the smallest
 *      t, then the smallest k.
 *   R5 (segments): segment m covers t in [floor(m L / M), floor((m+1) L / M)).
 *   R6 (stop): a coordinate is updated only when |Delta Z| >= eps; the run stops
 *      once every coordinate has |Delta Z| < eps.
 *
 * Array layouts (C order):
 *   X    [P][T]            signal, zero outside [0, T)
 *   D    [K][P][W]         atoms
 *   Z    [K][L]            activations, L = T - W + 1
 *   beta [K][L]
 *   S    [K][K][2W-1]      S[k][l][d + W - 1] = S_{k,l}[d]
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX3(a, b, c, nb, nc) (((int64_t)(a) * (nb) + (b)) * (nc) + (c))

/* Soft thresholding Sh(u, lambda) = sign(u) max(|u| - lambda, 0), Sec. 2.1. */
double oracle_soft_threshold(double u, double lam)
{
    double a = fabs(u) - lam;
    if (a <= 0.0)
        return 0.0;
    return u > 0.0 ? a : -a;
}

/* ||D_k||_2^2 over the P x W pattern (norm definition, Sec. 2 notations). */
void oracle_norms(const double *D, int K, int P, int W, double *n2)
{
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int p = 0; p < P; ++p)
            for (int tau = 0; tau < W; ++tau) {
                double v = D[IDX3(k, p, tau, P, W)];
                s += v * v;
            }
        n2[k] = s;
    }
}

/* S_{k,l}[d] = (D~_k * D_l)[d] = sum_tau <D_k[tau], D_l[tau + d]>  (eq. (3), R3). */
void oracle_s_table(const double *D, int K, int P, int W, double *S)
{
    const int nd = 2 * W - 1;
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < K; ++l)
            for (int d = -(W - 1); d <= W - 1; ++d) {
                double s = 0.0;
                for (int tau = 0; tau < W; ++tau) {
                    int u = tau + d;
                    if (u < 0 || u >= W)
                        continue;
                    for (int p = 0; p < P; ++p)
                        s += D[IDX3(k, p, tau, P, W)] * D[IDX3(l, p, u, P, W)];
                }
                S[IDX3(k, l, d + W - 1, K, nd)] = s;
            }
}

/* Hypothesis H1 (Sec. 3, Theorem 1): for every pair of coordinates at
 * different positions, |S_{k0,k1}[t0 - t1]| / (|D_k0|_2 |D_k1|_2) < 1.  Returns
 * the largest such ratio over atoms k, l and shifts d != 0 (0 when W = 1);
 * H1 holds when it is below 1.  By Cauchy-Schwarz it is at most 1. */
double oracle_h1_ratio(const double *D, int K, int P, int W)
{
    const int nd = 2 * W - 1;
    double *S = (double *)malloc(sizeof(double) * (size_t)K * K * nd);
    double *n2 = (double *)malloc(sizeof(double) * (size_t)K);
    if (!S || !n2) {
        free(S);
        free(n2);
        return -1.0;
    }
    oracle_s_table(D, K, P, W, S);
    oracle_norms(D, K, P, W, n2);
    double worst = 0.0;
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < K; ++l)
            for (int d = -(W - 1); d <= W - 1; ++d) {
                if (d == 0)
                    continue;
                double r = fabs(S[IDX3(k, l, d + W - 1, K, nd)]) / sqrt(n2[k] * n2[l]);
                if (r > worst)
                    worst = r;
            }
    free(S);
    free(n2);
    return worst;
}

/* out_k[t] = sum_p sum_tau D_k[p][tau] Y[p][t + tau], t in [0, T - W + 1).
 * At Z = 0 this is the initial beta of Algorithm 1 (D~_k * X, reading R1). */
void oracle_correlate(const double *D, int K, int P, int W, const double *Y,
                      int64_t T, double *out)
{
    const int64_t L = T - W + 1;
    for (int k = 0; k < K; ++k)
        for (int64_t t = 0; t < L; ++t) {
            double s = 0.0;
            for (int p = 0; p < P; ++p)
                for (int tau = 0; tau < W; ++tau)
                    s += D[IDX3(k, p, tau, P, W)] * Y[(int64_t)p * T + t + tau];
            out[(int64_t)k * L + t] = s;
        }
}

/* Xhat[p][t] = sum_k (Z_k * D_k)[t] = sum_k sum_tau Z_k[t - tau] D_k[p][tau]
 * (convolution of Sec. 2 notations, model eq. (1) without the noise). */
void oracle_reconstruct(const double *D, const double *Z, int K, int P, int W,
                        int64_t T, double *Xhat)
{
    const int64_t L = T - W + 1;
    memset(Xhat, 0, sizeof(double) * (size_t)P * (size_t)T);
    for (int k = 0; k < K; ++k)
        for (int64_t s = 0; s < L; ++s) {
            double z = Z[(int64_t)k * L + s];
            if (z == 0.0)
                continue;
            for (int p = 0; p < P; ++p)
                for (int tau = 0; tau < W; ++tau)
                    Xhat[(int64_t)p * T + s + tau] += z * D[IDX3(k, p, tau, P, W)];
        }
}

/* E(Z) = 1/2 ||X - sum_k Z_k * D_k||_2^2 + lambda sum_k ||Z_k||_1   (eq. (2)). */
double oracle_objective(const double *X, const double *D, const double *Z, int K,
                        int P, int W, int64_t T, double lam)
{
    const int64_t L = T - W + 1;
    double *R = (double *)malloc(sizeof(double) * (size_t)P * (size_t)T);
    if (!R)
        return NAN;
    oracle_reconstruct(D, Z, K, P, W, T, R);
    double quad = 0.0;
    for (int64_t i = 0; i < (int64_t)P * T; ++i) {
        double r = X[i] - R[i];
        quad += r * r;
    }
    free(R);
    double l1 = 0.0;
    for (int64_t i = 0; i < (int64_t)K * L; ++i)
        l1 += fabs(Z[i]);
    return 0.5 * quad + lam * l1;
}

/* Safe screening (Sec. 2.4 names screening as a complement to the
 * greedy selection; this is the Gap Safe sphere rule of Fercoq, Gramfort and
 * Salmon, 2015, for the Lasso (2) written out in the convolutional case).
 * With R = X - sum_k Z_k * D_k and c_k[t] = sum_p sum_tau D_k[p][tau] R[p][t + tau]
 * (the correlation D^T R), the rescaled residual theta = R / max(lambda,
 * max |c|) is dual feasible (|D^T theta| <= 1); the dual objective is
 * Dual(theta) = 1/2 |X|^2 - lambda^2 / 2 |theta - X / lambda|^2, the gap
 * G = E(Z) - Dual(theta) >= 0, and every coordinate with
 * |c_k[t]| / max(lambda, max |c|) + sqrt(2 G) / lambda |D_k|_2 < 1 is zero in
 * every solution of (2).  Writes the gap, the sphere radius sqrt(2 G) / lambda
 * and screened[k * L + t] (1 = proved zero); returns the number screened, or
 * -1 when out of memory. */
int64_t oracle_gap_safe(const double *X, const double *D, const double *Z, int K, int P,
                        int W, int64_t T, double lam, double *gap, double *radius,
                        unsigned char *screened)
{
    const int64_t L = T - W + 1;
    double *R = (double *)malloc(sizeof(double) * (size_t)P * (size_t)T);
    double *c = (double *)malloc(sizeof(double) * (size_t)K * (size_t)L);
    double *n2 = (double *)malloc(sizeof(double) * (size_t)K);
    if (!R || !c || !n2) {
        free(R);
        free(c);
        free(n2);
        return -1;
    }
    oracle_reconstruct(D, Z, K, P, W, T, R);
    double rr = 0.0, xx = 0.0;
    for (int64_t i = 0; i < (int64_t)P * T; ++i) {
        R[i] = X[i] - R[i];
        rr += R[i] * R[i];
        xx += X[i] * X[i];
    }
    oracle_correlate(D, K, P, W, R, T, c);
    oracle_norms(D, K, P, W, n2);
    double cmax = 0.0, l1 = 0.0;
    for (int64_t i = 0; i < (int64_t)K * L; ++i) {
        if (fabs(c[i]) > cmax)
            cmax = fabs(c[i]);
        l1 += fabs(Z[i]);
    }
    const double sc = cmax > lam ? cmax : lam;
    const double primal = 0.5 * rr + lam * l1;
    /* |theta - X / lambda|^2 with theta = R / sc */
    double dd = 0.0;
    for (int64_t i = 0; i < (int64_t)P * T; ++i) {
        double v = R[i] / sc - X[i] / lam;
        dd += v * v;
    }
    const double dual = 0.5 * xx - 0.5 * lam * lam * dd;
    double G = primal - dual;
    if (G < 0.0)
        G = 0.0;
    const double r = sqrt(2.0 * G) / lam;
    int64_t n = 0;
    for (int k = 0; k < K; ++k)
        for (int64_t t = 0; t < L; ++t) {
            const int64_t i = (int64_t)k * L + t;
            const int z = fabs(c[i]) / sc + r * sqrt(n2[k]) < 1.0;
            screened[i] = (unsigned char)z;
            n += z;
        }
    *gap = G;
    *radius = r;
    free(R);
    free(c);
    free(n2);
    return n;
}

/* beta from its definition (Sec. 2.1): the correlation of D_k with the
 * residual in which Z_k[t] alone is set to zero (reading R1). */
int oracle_beta(const double *X, const double *D, const double *Z, int K, int P,
                int W, int64_t T, double *beta)
{
    const int64_t L = T - W + 1;
    double *R = (double *)malloc(sizeof(double) * (size_t)P * (size_t)T);
    double *n2 = (double *)malloc(sizeof(double) * (size_t)K);
    if (!R || !n2) {
        free(R);
        free(n2);
        return -1;
    }
    oracle_reconstruct(D, Z, K, P, W, T, R);
    for (int64_t i = 0; i < (int64_t)P * T; ++i)
        R[i] = X[i] - R[i];
    oracle_correlate(D, K, P, W, R, T, beta);
    oracle_norms(D, K, P, W, n2);
    for (int k = 0; k < K; ++k)
        for (int64_t t = 0; t < L; ++t)
            beta[(int64_t)k * L + t] += n2[k] * Z[(int64_t)k * L + t];
    free(R);
    free(n2);
    return 0;
}

/* ||Delta Z||_inf over all coordinates, recomputing beta from scratch
 * (the full stopping test of Algorithm 3).  Returns the value and the
 * maximising coordinate (ties: smallest t, then smallest k). */
double oracle_max_dz(const double *X, const double *D, const double *Z, int K,
                     int P, int W, int64_t T, double lam, int *k_arg,
                     int64_t *t_arg)
{
    const int64_t L = T - W + 1;
    double *beta = (double *)malloc(sizeof(double) * (size_t)K * (size_t)L);
    double *n2 = (double *)malloc(sizeof(double) * (size_t)K);
    if (!beta || !n2 || oracle_beta(X, D, Z, K, P, W, T, beta) != 0) {
        free(beta);
        free(n2);
        return NAN;
    }
    oracle_norms(D, K, P, W, n2);
    double best = -1.0;
    int bk = -1;
    int64_t bt = -1;
    for (int64_t t = 0; t < L; ++t)
        for (int k = 0; k < K; ++k) {
            double zp = oracle_soft_threshold(beta[(int64_t)k * L + t], lam) / n2[k];
            double d = fabs(zp - Z[(int64_t)k * L + t]);
            if (d > best) {
                best = d;
                bk = k;
                bt = t;
            }
        }
    if (k_arg)
        *k_arg = bk;
    if (t_arg)
        *t_arg = bt;
    free(beta);
    free(n2);
    return best;
}

/* beta_k[t] at n given coordinates (k[i], t[i]) from the definition of
 * Sec. 2.1 (reading R1), for signals too long for a full recompute: the
 * residual X - sum Z * D on the window [t, t + W) from the activations that
 * reach it, correlated with D_k, plus |D_k|^2 Z_k[t].  Returns 0, or -1 on
 * a bad coordinate or allocation failure. */
int oracle_beta_at(const double *X, const double *D, const double *Z, int K, int P,
                   int W, int64_t T, const int32_t *kk, const int64_t *tt, int64_t n,
                   double *out)
{
    const int64_t L = T - W + 1;
    double *R = (double *)malloc(sizeof(double) * (size_t)P * (size_t)W);
    double *n2 = (double *)malloc(sizeof(double) * (size_t)K);
    if (!R || !n2) {
        free(R);
        free(n2);
        return -1;
    }
    oracle_norms(D, K, P, W, n2);
    for (int64_t i = 0; i < n; ++i) {
        const int k = kk[i];
        const int64_t t = tt[i];
        if (k < 0 || k >= K || t < 0 || t >= L) {
            free(R);
            free(n2);
            return -1;
        }
        for (int p = 0; p < P; ++p)
            for (int s = 0; s < W; ++s)
                R[p * W + s] = X[(int64_t)p * T + t + s];
        /* activations (k2, u) with u + tau in [t, t + W) for some tau < W */
        const int64_t u0 = t - W + 1 > 0 ? t - W + 1 : 0;
        const int64_t u1 = t + W - 1 < L - 1 ? t + W - 1 : L - 1;
        for (int k2 = 0; k2 < K; ++k2)
            for (int64_t u = u0; u <= u1; ++u) {
                const double z = Z[(int64_t)k2 * L + u];
                if (z == 0.0)
                    continue;
                for (int s = 0; s < W; ++s) {
                    const int64_t tau = t + s - u;
                    if (tau < 0 || tau >= W)
                        continue;
                    for (int p = 0; p < P; ++p)
                        R[p * W + s] -= z * D[IDX3(k2, p, tau, P, W)];
                }
            }
        double b = 0.0;
        for (int p = 0; p < P; ++p)
            for (int s = 0; s < W; ++s)
                b += D[IDX3(k, p, s, P, W)] * R[p * W + s];
        out[i] = b + n2[k] * Z[(int64_t)k * L + t];
    }
    free(R);
    free(n2);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Solver                                                                     */
/* ------------------------------------------------------------------------ */

enum { ORACLE_SCHED_EVENODD = 0, ORACLE_SCHED_SEQUENCE = 1, ORACLE_SCHED_DICOD = 2 };

typedef struct {
    int64_t n_updates;   /* coordinate updates applied                        */
    int64_t n_steps;     /* segment selections (Algorithm 3 iterations)       */
    int64_t n_phases;    /* phases run (phase schedules only)                 */
    int64_t n_full_checks; /* O(KL) stopping checks (sequence schedule)       */
    double dE_sum;       /* sum of the per-update cost decreases, Prop. A.1   */
    double dE_min;       /* smallest single-update cost decrease              */
    double lowerbound_gap_min; /* min over updates of dE - |D|^2 delta^2 / 2   */
    int converged;
    int64_t n_messages;  /* DICOD: (k0, t0, delta) messages sent              */
    int64_t n_interf;    /* DICOD: pairs of concurrent updates of adjacent    */
                         /* segments with |t0 - t1| < W (Sec. 3, interferences) */
    int64_t n_adjacent;  /* DICOD: pairs of concurrent updates of adjacent    */
                         /* segments (any distance)                           */
    double interf_sum;   /* DICOD: sum of S_{k0,k1}[t0 - t1] d0 d1 over the   */
                         /* interfering pairs (Prop. A.2)                     */
} oracle_stats;

typedef struct {
    int64_t step;   /* global update index                       */
    int32_t phase;  /* even/odd phase (or -1)                    */
    int32_t seg;    /* segment m                                 */
    int32_t k0;
    int32_t n_local; /* index of the update within the segment run */
    int64_t t0;
    double z_old;
    double z_new;
    double dE;      /* E(Z) - E(Z') from Prop. A.1               */
} oracle_trace_rec;

typedef struct {
    int K, P, W;
    int64_t T, L;
    double lam;
    const double *S;
    const double *n2;
    double *beta;
    double *Z;
} lgcd_state;

/* Local greedy choice over segment [b, e) (Algorithm 3, selection step):
 * Z'_k[t] = Sh(beta_k[t], lambda) / |D_k|^2 and the largest |Z' - Z|. */
static double local_argmax(const lgcd_state *s, int64_t b, int64_t e, int *k0,
                           int64_t *t0, double *z_new)
{
    double best = -1.0;
    for (int64_t t = b; t < e; ++t)
        for (int k = 0; k < s->K; ++k) {
            int64_t i = (int64_t)k * s->L + t;
            double zp = oracle_soft_threshold(s->beta[i], s->lam) / s->n2[k];
            double d = fabs(zp - s->Z[i]);
            if (d > best) {
                best = d;
                *k0 = k;
                *t0 = t;
                *z_new = zp;
            }
        }
    return best;
}

/* Apply Z_{k0}[t0] <- z_new and the beta update of eq. (3) (reading R2).
 * Returns the cost decrease of Proposition A.1. */
static double apply_update(lgcd_state *s, int k0, int64_t t0, double z_new)
{
    const int W = s->W, K = s->K, nd = 2 * W - 1;
    int64_t i0 = (int64_t)k0 * s->L + t0;
    double z_old = s->Z[i0];
    double b0 = s->beta[i0];
    double delta = z_new - z_old;
    /* Prop. A.1: e(u) = |D|^2/2 (z^2 - u^2) - beta (z - u) + lambda (|z| - |u|). */
    double dE = 0.5 * s->n2[k0] * (z_old * z_old - z_new * z_new) -
                b0 * (z_old - z_new) + s->lam * (fabs(z_old) - fabs(z_new));
    s->Z[i0] = z_new;
    int64_t lo = t0 - (W - 1) < 0 ? 0 : t0 - (W - 1);
    int64_t hi = t0 + (W - 1) > s->L - 1 ? s->L - 1 : t0 + (W - 1);
    for (int k = 0; k < K; ++k) {
        const double *Srow = s->S + IDX3(k, k0, 0, K, nd);
        for (int64_t t = lo; t <= hi; ++t) {
            if (k == k0 && t == t0)
                continue;
            s->beta[(int64_t)k * s->L + t] -= Srow[t - t0 + W - 1] * delta;
        }
    }
    return dE;
}

/* Algorithm 2, own part of an update: as apply_update, with the eq. (3)
 * change of beta restricted to the segment [b, e) of the core that made it. */
static double apply_update_local(lgcd_state *s, int k0, int64_t t0, double z_new,
                                 int64_t b, int64_t e)
{
    const int W = s->W, K = s->K, nd = 2 * W - 1;
    int64_t i0 = (int64_t)k0 * s->L + t0;
    double z_old = s->Z[i0];
    double b0 = s->beta[i0];
    double delta = z_new - z_old;
    double dE = 0.5 * s->n2[k0] * (z_old * z_old - z_new * z_new) -
                b0 * (z_old - z_new) + s->lam * (fabs(z_old) - fabs(z_new));
    s->Z[i0] = z_new;
    int64_t lo = t0 - (W - 1) < b ? b : t0 - (W - 1);
    int64_t hi = t0 + (W - 1) > e - 1 ? e - 1 : t0 + (W - 1);
    for (int k = 0; k < K; ++k) {
        const double *Srow = s->S + IDX3(k, k0, 0, K, nd);
        for (int64_t t = lo; t <= hi; ++t) {
            if (k == k0 && t == t0)
                continue;
            s->beta[(int64_t)k * s->L + t] -= Srow[t - t0 + W - 1] * delta;
        }
    }
    return dE;
}

/* Algorithm 2, receiving side: the eq. (3) change of beta that the message
 * (k0, t0, delta) of a neighbour makes on the segment [b, e). */
static void apply_message(lgcd_state *s, int k0, int64_t t0, double delta, int64_t b,
                          int64_t e)
{
    const int W = s->W, K = s->K, nd = 2 * W - 1;
    int64_t lo = t0 - (W - 1) < b ? b : t0 - (W - 1);
    int64_t hi = t0 + (W - 1) > e - 1 ? e - 1 : t0 + (W - 1);
    for (int k = 0; k < K; ++k) {
        const double *Srow = s->S + IDX3(k, k0, 0, K, nd);
        for (int64_t t = lo; t <= hi; ++t)
            s->beta[(int64_t)k * s->L + t] -= Srow[t - t0 + W - 1] * delta;
    }
}

typedef struct {
    int k0;
    int64_t t0;
    double delta;
} dicod_msg;

static void note_update(oracle_stats *st, double dE, double n2, double delta)
{
    st->n_updates++;
    st->dE_sum += dE;
    if (st->n_updates == 1 || dE < st->dE_min)
        st->dE_min = dE;
    double gap = dE - 0.5 * n2 * delta * delta; /* Lemma A.1 lower bound */
    if (st->n_updates == 1 || gap < st->lowerbound_gap_min)
        st->lowerbound_gap_min = gap;
}

static void record(oracle_trace_rec *tr, int64_t cap, const oracle_stats *st,
                   int phase, int seg, int k0, int n_local, int64_t t0,
                   double z_old, double z_new, double dE)
{
    int64_t i = st->n_updates - 1;
    if (!tr || i < 0 || i >= cap)
        return;
    tr[i].step = i;
    tr[i].phase = phase;
    tr[i].seg = seg;
    tr[i].k0 = k0;
    tr[i].n_local = n_local;
    tr[i].t0 = t0;
    tr[i].z_old = z_old;
    tr[i].z_new = z_new;
    tr[i].dE = dE;
}

/* The ORACLE_SCHED_DICOD schedule of oracle_lgcd (see there). */
static int dicod_lockstep(lgcd_state *s, int M, const int64_t *bnd, int cap, double eps,
                          int64_t max_steps, oracle_stats *st, oracle_trace_rec *trace,
                          int64_t trace_cap)
{
    const int W = s->W, K = s->K, nd = 2 * W - 1;
    const int64_t L = s->L;
    const int per = cap > 0 ? cap : (int)(L < 65536 ? L : 65536);
    /* inbox[m][0]: messages from m - 1, inbox[m][1]: from m + 1, for the
     * current phase; outbox the same for the next phase */
    dicod_msg *in = (dicod_msg *)malloc(sizeof(dicod_msg) * (size_t)M * 2 * per);
    dicod_msg *out = (dicod_msg *)malloc(sizeof(dicod_msg) * (size_t)M * 2 * per);
    int *n_in = (int *)calloc((size_t)M * 2, sizeof(int));
    int *n_out = (int *)calloc((size_t)M * 2, sizeof(int));
    unsigned char *dirty = (unsigned char *)malloc((size_t)M);
    unsigned char *next = (unsigned char *)malloc((size_t)M);
    /* this phase's updates per segment, for the interference statistics */
    dicod_msg *upd = (dicod_msg *)malloc(sizeof(dicod_msg) * (size_t)M * per);
    int *n_upd = (int *)calloc((size_t)M, sizeof(int));
    int rc = 1;
    if (!in || !out || !n_in || !n_out || !dirty || !next || !upd || !n_upd) {
        rc = -3;
        goto done;
    }
    memset(dirty, 1, (size_t)M);
    for (int64_t p = 0; st->n_updates < max_steps; ++p) {
        memset(next, 0, (size_t)M);
        memset(n_out, 0, sizeof(int) * (size_t)M * 2);
        int64_t phase_upd = 0;
        for (int m = 0; m < M; ++m) {
            n_upd[m] = 0;
            if (!dirty[m])
                continue;
            st->n_steps++;
            const int64_t b = bnd[m], e = bnd[m + 1];
            for (int side = 0; side < 2; ++side)
                for (int i = 0; i < n_in[2 * m + side]; ++i) {
                    const dicod_msg *g = &in[((size_t)m * 2 + side) * per + i];
                    apply_message(s, g->k0, g->t0, g->delta, b, e);
                }
            int n = 0;
            for (;;) {
                int k0 = 0;
                int64_t t0 = 0;
                double zn = 0.0;
                double d = local_argmax(s, b, e, &k0, &t0, &zn);
                if (d < eps)
                    break;
                if (n == per) {
                    next[m] = 1;
                    break;
                }
                if (st->n_updates >= max_steps)
                    break;
                double z_old = s->Z[(int64_t)k0 * L + t0];
                double dE = apply_update_local(s, k0, t0, zn, b, e);
                note_update(st, dE, s->n2[k0], zn - z_old);
                record(trace, trace_cap, st, (int)p, m, k0, n, t0, z_old, zn, dE);
                dicod_msg msg = {k0, t0, zn - z_old};
                upd[(size_t)m * per + n] = msg;
                ++n;
                if (m > 0 && t0 - (W - 1) < b) { /* window reaches m - 1 */
                    out[((size_t)(m - 1) * 2 + 1) * per + n_out[2 * (m - 1) + 1]++] = msg;
                    next[m - 1] = 1;
                    st->n_messages++;
                }
                if (m < M - 1 && t0 + (W - 1) >= e) { /* window reaches m + 1 */
                    out[((size_t)(m + 1) * 2) * per + n_out[2 * (m + 1)]++] = msg;
                    next[m + 1] = 1;
                    st->n_messages++;
                }
            }
            n_upd[m] = n;
            phase_upd += n;
        }
        /* interferences: concurrent updates of adjacent segments (Prop. A.2) */
        for (int m = 0; m + 1 < M; ++m)
            for (int i = 0; i < n_upd[m]; ++i)
                for (int j = 0; j < n_upd[m + 1]; ++j) {
                    const dicod_msg *u = &upd[(size_t)m * per + i];
                    const dicod_msg *v = &upd[(size_t)(m + 1) * per + j];
                    st->n_adjacent++;
                    const int64_t dt = u->t0 - v->t0;
                    if (dt <= -W || dt >= W)
                        continue;
                    st->n_interf++;
                    st->interf_sum += s->S[IDX3(u->k0, v->k0, dt + W - 1, K, nd)] *
                                      u->delta * v->delta;
                }
        st->n_phases = p + 1;
        { dicod_msg *t = in; in = out; out = t; }
        { int *t = n_in; n_in = n_out; n_out = t; }
        { unsigned char *t = dirty; dirty = next; next = t; }
        if (phase_upd == 0) {
            rc = 0;
            break;
        }
    }
done:
    free(in);
    free(out);
    free(n_in);
    free(n_out);
    free(dirty);
    free(next);
    free(upd);
    free(n_upd);
    return rc;
}

/*
 * Locally greedy coordinate descent.
 *
 *   X [P][T], D [K][P][W] (double), lam > 0, eps > 0, M segments (R5).
 *   Z [K][L] is the output (zero-initialised here, Algorithm 3 init).
 *
 * schedule = ORACLE_SCHED_SEQUENCE: Algorithm 3.  At step i the segment
 *   seq[i % seq_len] is chosen (a random sequence gives SeqDICOD, the sequence
 *   0..M-1 gives a cyclic order, M = 1 gives greedy CD of Algorithm 1).  The
 *   run stops when max_m dZ_m < eps and a full check gives ||Delta Z||_inf <
 *   eps.
 *
 * schedule = ORACLE_SCHED_EVENODD: phases p = 0, 1, ...; in phase p the
 *   segments with m % C == p % C (C = `colors`, 2 gives even/odd) that are
 *   marked dirty each run locally greedy updates until their local maximum is
 *   below eps or `cap` updates were made (cap <= 0: no cap).  A segment stays
 *   dirty only if it stopped on the cap; a segment whose update window reaches
 *   a neighbour marks that neighbour dirty.  Segments are at least W - 1 long
 *   (a window reaches W - 1 positions on each side) and at least
 *   (2W - 2) / (C - 1) long, so segments of one colour never touch the same
 *   beta entries and each phase equals running its segments one after the
 *   other.  The run stops after C consecutive phases without updates.
 *
 * schedule = ORACLE_SCHED_DICOD: Algorithm 2 with the cores in lockstep.  In
 *   phase p every segment that is dirty (it stopped on the cap, or received
 *   messages) first applies the messages its neighbours sent in phase p - 1
 *   (left neighbour first, each in the order sent), then runs locally greedy
 *   updates from its own beta (up to `cap`), changing beta on its own
 *   positions only; an update whose window reaches a neighbour is sent to it
 *   as (k0, t0, delta) (the paper's messages, delivered one phase later).
 *   Segments are at least W - 1 long, so a window reaches only the adjacent
 *   segments.  Updates of adjacent segments in one phase may interfere
 *   (Sec. 3, Prop. A.2); the statistics count them.  The run stops after a
 *   phase without updates (then no message is pending).
 *
 * Returns 0 when converged, 1 when max_steps (updates) or max_phases ran out,
 * negative on bad arguments.
 */
int oracle_lgcd(const double *X, const double *D, int K, int P, int W, int64_t T,
                double lam, double eps, int M, int schedule, const int32_t *seq,
                int64_t seq_len, int cap, int64_t max_steps, double *Z,
                oracle_stats *st, oracle_trace_rec *trace, int64_t trace_cap,
                int colors)
{
    if (K <= 0 || P <= 0 || W <= 0 || T < W || !(lam > 0.0) || !(eps > 0.0) ||
        M <= 0)
        return -1;
    const int64_t L = T - W + 1;
    if (M > L)
        return -1;
    if (schedule == ORACLE_SCHED_EVENODD) {
        if (colors < 2)
            return -1;
        /* segments of one colour must be 2W - 2 apart, and a window (which
         * reaches W - 1 positions on each side, eq. (3)) may only reach the
         * adjacent segments */
        if (M > 1 && (L / M < (W > 1 ? W - 1 : 1) || (colors - 1) * (L / M) < 2 * W - 2))
            return -2;
    }
    if (schedule == ORACLE_SCHED_SEQUENCE && (!seq || seq_len <= 0))
        return -1;
    if (schedule == ORACLE_SCHED_DICOD && M > 1 && L / M < (W > 1 ? W - 1 : 1))
        return -2;
    const int nd = 2 * W - 1;

    double *S = (double *)malloc(sizeof(double) * (size_t)K * K * nd);
    double *n2 = (double *)malloc(sizeof(double) * (size_t)K);
    double *beta = (double *)malloc(sizeof(double) * (size_t)K * (size_t)L);
    int64_t *bnd = (int64_t *)malloc(sizeof(int64_t) * (size_t)(M + 1));
    if (!S || !n2 || !beta || !bnd) {
        free(S);
        free(n2);
        free(beta);
        free(bnd);
        return -3;
    }
    oracle_s_table(D, K, P, W, S);
    oracle_norms(D, K, P, W, n2);
    oracle_correlate(D, K, P, W, X, T, beta); /* beta at Z = 0 */
    memset(Z, 0, sizeof(double) * (size_t)K * (size_t)L);
    for (int m = 0; m <= M; ++m)
        bnd[m] = (int64_t)(((__int128)m * L) / M);

    lgcd_state s = {K, P, W, T, L, lam, S, n2, beta, Z};
    oracle_stats local;
    memset(&local, 0, sizeof(local));
    int rc = 1;

    if (schedule == ORACLE_SCHED_SEQUENCE) {
        double *dZ = (double *)malloc(sizeof(double) * (size_t)M);
        for (int m = 0; m < M; ++m)
            dZ[m] = INFINITY; /* Algorithm 3 init: dZ_m = +inf */
        for (int64_t i = 0; i < max_steps; ++i) {
            int m = seq[i % seq_len];
            if (m < 0 || m >= M) {
                rc = -1;
                break;
            }
            local.n_steps++;
            int k0 = 0;
            int64_t t0 = 0;
            double zn = 0.0;
            double d = local_argmax(&s, bnd[m], bnd[m + 1], &k0, &t0, &zn);
            if (d >= eps) {
                double z_old = Z[(int64_t)k0 * L + t0];
                double dE = apply_update(&s, k0, t0, zn);
                note_update(&local, dE, n2[k0], zn - z_old);
                record(trace, trace_cap, &local, -1, m, k0, 0, t0, z_old, zn, dE);
            }
            dZ[m] = d;
            double mx = 0.0;
            for (int j = 0; j < M; ++j)
                mx = dZ[j] > mx ? dZ[j] : mx;
            if (mx < eps) {
                local.n_full_checks++;
                double full = local_argmax(&s, 0, L, &k0, &t0, &zn);
                if (full < eps) {
                    rc = 0;
                    break;
                }
            }
        }
        free(dZ);
    } else if (schedule == ORACLE_SCHED_EVENODD) {
        unsigned char *dirty = (unsigned char *)malloc((size_t)M);
        memset(dirty, 1, (size_t)M);
        int64_t quiet = 0; /* consecutive phases without updates */
        for (int64_t p = 0; local.n_updates < max_steps; ++p) {
            int par = (int)(p % colors);
            int64_t upd = 0;
            for (int m = par; m < M; m += colors) {
                if (!dirty[m])
                    continue;
                local.n_steps++;
                int n = 0, touch_l = 0, touch_r = 0;
                for (;;) {
                    int k0 = 0;
                    int64_t t0 = 0;
                    double zn = 0.0;
                    double d = local_argmax(&s, bnd[m], bnd[m + 1], &k0, &t0, &zn);
                    if (d < eps) {
                        dirty[m] = 0;
                        break;
                    }
                    if (cap > 0 && n == cap) {
                        dirty[m] = 1;
                        break;
                    }
                    if (local.n_updates >= max_steps)
                        break; /* out of budget: the segment stays dirty */
                    double z_old = Z[(int64_t)k0 * L + t0];
                    double dE = apply_update(&s, k0, t0, zn);
                    note_update(&local, dE, n2[k0], zn - z_old);
                    record(trace, trace_cap, &local, (int)p, m, k0, n, t0, z_old,
                           zn, dE);
                    ++n;
                    if (m > 0 && t0 - (W - 1) < bnd[m])
                        touch_l = 1;
                    if (m < M - 1 && t0 + (W - 1) >= bnd[m + 1])
                        touch_r = 1;
                }
                if (touch_l)
                    dirty[m - 1] = 1;
                if (touch_r)
                    dirty[m + 1] = 1;
                upd += n;
            }
            local.n_phases = p + 1;
            quiet = upd == 0 ? quiet + 1 : 0;
            if (quiet >= colors) {
                rc = 0;
                break;
            }
        }
        free(dirty);
    } else if (schedule == ORACLE_SCHED_DICOD) {
        rc = dicod_lockstep(&s, M, bnd, cap, eps, max_steps, &local, trace, trace_cap);
    } else {
        rc = -1;
    }
    local.converged = rc == 0;
    if (st)
        *st = local;
    free(S);
    free(n2);
    free(beta);
    free(bnd);
    return rc;
}

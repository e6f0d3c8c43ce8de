/*
 * lv_oracle.c -- FP64 CPU oracle for Monte Carlo pricing and the vol-grid adjoint
 * in the Dupire local-volatility model (Belletti, King, Lottes, Chen, Anderson,
 * "Sensitivity Analysis in the Dupire Local Volatility Model with Tensorflow",
 * arXiv 2002.02481).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the GPU
 * library is checked against.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark load it; the product library never does, and the two
 * share no source.
 *
 * What it computes, in the paper's terms:
 *   - the model dX/X = sigma(X,t) dW (Sec. IV-A, the SDE), or with a constant
 *     short rate r the trend r dt that the narrated step adds ("today's price
 *     plus a deterministic trend plus a Gaussian term"), payoffs then discounted
 *     by e^{-r T}; r = 0 is the paper's driftless SDE;
 *   - an explicit Euler scheme (Sec. IV-A), taken on y = ln(X/X0) with the Ito
 *     drift (r - sigma^2/2) dt, sigma read at the left point of each step; or
 *     (scheme 1) the explicit Euler step on X itself, as the paper narrates it;
 *   - sigma(S,t) by bilinear interpolation of a grid of nodes {(i dx, j dt)}
 *     (Sec. IV-A, the grid; Sec. IV-D, bilinear interpolation), flat outside;
 *   - Gaussian increments from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC'11) through the
 *     Box-Muller transform, standing in for the normal-generator wrapper of
 *     Sec. IV-B;
 *   - European call/put payoffs averaged over paths (Sec. IV-B, IV-C);
 *   - reverse-mode differentiation (back-propagation) of the price estimate
 *     with respect to every node of the vol grid (Sec. III; Sec. IV-C).
 *
 * All arithmetic is IEEE double.  Sums over paths run in fixed chunks of
 * LVO_CHUNK paths; chunk partials are merged in chunk order with Neumaier's
 * compensated sum, so results do not depend on the number of threads.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define LVO_CHUNK 4096
#define LVO_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, from its published definition (SC'11, Sec. 3 and Table 2).  */
/* A round maps (c0,c1,c2,c3) with key (k0,k1) to                              */
/*   (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))       */
/* and the key is bumped by the Weyl constants between rounds.                */
/* ------------------------------------------------------------------------- */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u; /* golden ratio */
static const uint32_t PHILOX_W1 = 0xBB67AE85u; /* sqrt(3) - 1  */

void lvo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The four words for steps 4m..4m+3 of path p: key = seed, counter = (m, p). */
void lvo_philox_words(uint64_t seed, uint64_t m, uint64_t p, uint32_t out[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)m, (uint32_t)(m >> 32), (uint32_t)p, (uint32_t)(p >> 32)};
    lvo_philox4x32_10(ctr, key, out);
}

/* Uniform in (0,1): the top 23 bits of a word, centred in their cell, i.e.
 * (2k+1)/2^24 with k = w >> 9.  Every value is exact in float32 as well. */
double lvo_uniform(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) / 8388608.0;
}

/* Normal increment Z_n of path p.  Words (w0,w1) of block m = n/4 give
 * Z_{4m}, Z_{4m+1}; words (w2,w3) give Z_{4m+2}, Z_{4m+3} (Box-Muller). */
double lvo_normal(uint64_t seed, uint64_t p, int64_t n)
{
    uint32_t w[4];
    lvo_philox_words(seed, (uint64_t)(n / 4), p, w);
    int r = (int)(n % 4);
    int pair = r / 2;
    double ua = lvo_uniform(w[2 * pair]);
    double ub = lvo_uniform(w[2 * pair + 1]);
    double radius = sqrt(-2.0 * log(ua));
    if (r % 2 == 0)
        return radius * cos(2.0 * LVO_PI * ub);
    return radius * sin(2.0 * LVO_PI * ub);
}

/* Normals Z_n of paths p0..p0+n_paths-1, steps 0..n_steps-1, into out[path][step]. */
void lvo_normals(uint64_t seed, uint64_t p0, int64_t n_paths, int64_t n_steps, double *out)
{
    for (int64_t q = 0; q < n_paths; ++q)
        for (int64_t n = 0; n < n_steps; ++n)
            out[q * n_steps + n] = lvo_normal(seed, p0 + (uint64_t)q, n);
}

/* ------------------------------------------------------------------------- */
/* Problem description                                                       */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t n_spot, spot_kind;   /* kind 0: nodes uniform in S; 1: uniform in ln S */
    double spot_lo, spot_hi;
    int32_t n_time;
    double time_lo, time_hi;
    const double *sigma;         /* [n_spot][n_time], node (i,j) at sigma[i*n_time + j] */
    double spot;
    int32_t n_opt;
    const int32_t *is_put;
    const double *strike, *maturity, *weight;
    int32_t n_steps;
    uint64_t seed;
    int32_t scheme;              /* 0: log-Euler on y = ln(X/X0); 1: Euler on X */
    double rate;                 /* constant short rate r: the step's trend, e^{-r T} discounting */
    /* derived */
    double dt, sqrt_dt;
    int32_t *tap_step;           /* [n_opt] step index of each maturity */
    double *disc;                /* [n_opt] discount factor e^{-r T_k} */
} lvo_problem;

static char lvo_errbuf[256];
const char *lvo_last_error(void) { return lvo_errbuf; }

static int lvo_fail(const char *msg)
{
    snprintf(lvo_errbuf, sizeof lvo_errbuf, "%s", msg);
    return -1;
}

static int lvo_setup(lvo_problem *pb)
{
    if (pb->n_spot < 2 || pb->n_time < 2) return lvo_fail("grid needs at least 2x2 nodes");
    if (!(pb->spot_hi > pb->spot_lo) || !(pb->time_hi > pb->time_lo)) return lvo_fail("axis hi must exceed lo");
    if (pb->spot_kind == 1 && !(pb->spot_lo > 0.0)) return lvo_fail("log axis needs lo > 0");
    if (pb->spot_kind != 0 && pb->spot_kind != 1) return lvo_fail("unknown axis kind");
    if (!(pb->spot > 0.0)) return lvo_fail("spot must be positive");
    if (pb->n_opt < 1 || pb->n_steps < 1) return lvo_fail("need n_opt >= 1 and n_steps >= 1");
    if (pb->scheme != 0 && pb->scheme != 1) return lvo_fail("unknown scheme");
    if (!isfinite(pb->rate)) return lvo_fail("rate must be finite");
    for (int64_t q = 0; q < (int64_t)pb->n_spot * pb->n_time; ++q)
        if (!(isfinite(pb->sigma[q]) && pb->sigma[q] > 0.0)) return lvo_fail("sigma nodes must be finite and positive");
    double tmax = 0.0;
    for (int k = 0; k < pb->n_opt; ++k) {
        if (!(pb->strike[k] > 0.0) || !(pb->maturity[k] > 0.0)) return lvo_fail("strikes and maturities must be positive");
        if (pb->maturity[k] > tmax) tmax = pb->maturity[k];
    }
    pb->dt = tmax / pb->n_steps;
    pb->sqrt_dt = sqrt(pb->dt);
    pb->tap_step = (int32_t *)malloc(sizeof(int32_t) * pb->n_opt);
    for (int k = 0; k < pb->n_opt; ++k) {
        double steps = pb->maturity[k] / pb->dt;
        double r = floor(steps + 0.5);
        if (fabs(steps - r) > 1e-9 * pb->n_steps || r < 1.0) {
            free(pb->tap_step);
            pb->tap_step = NULL;
            return lvo_fail("maturity is not a whole number of steps");
        }
        pb->tap_step[k] = (int32_t)r;
    }
    pb->disc = (double *)malloc(sizeof(double) * pb->n_opt);
    for (int k = 0; k < pb->n_opt; ++k) pb->disc[k] = exp(-pb->rate * pb->maturity[k]);
    return 0;
}

static void lvo_release(lvo_problem *pb)
{
    free(pb->tap_step);
    free(pb->disc);
    pb->tap_step = NULL;
    pb->disc = NULL;
}

/* ------------------------------------------------------------------------- */
/* Bilinear local volatility with flat extrapolation (Sec. IV-A grid,         */
/* Sec. IV-D bilinear interpolation).                                        */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t i, j;        /* lower-left node */
    double w[4];         /* weights of (i,j), (i+1,j), (i,j+1), (i+1,j+1) */
    double sigma;        /* interpolated value */
    double dsigma_dy;    /* d sigma / d ln S (zero outside the spot range) */
} lvo_interp;

/* Time cell of time t: b = clamp((t - t0)/dtau, 0, J-1), j = min(floor b, J-2). */
static void lvo_time_cell_at(const lvo_problem *pb, double t, int32_t *j, double *alpha)
{
    double dtau = (pb->time_hi - pb->time_lo) / (pb->n_time - 1);
    double b = (t - pb->time_lo) / dtau;
    if (b < 0.0) b = 0.0;
    if (b > pb->n_time - 1) b = pb->n_time - 1;
    int32_t jj = (int32_t)floor(b);
    if (jj > pb->n_time - 2) jj = pb->n_time - 2;
    *j = jj;
    *alpha = b - jj;
}

static void lvo_eval(const lvo_problem *pb, double S, double t, lvo_interp *out)
{
    double u, u0, u1;
    if (pb->spot_kind == 0) {
        u = S; u0 = pb->spot_lo; u1 = pb->spot_hi;
    } else {
        u = log(S); u0 = log(pb->spot_lo); u1 = log(pb->spot_hi);
    }
    double du = (u1 - u0) / (pb->n_spot - 1);
    double a_raw = (u - u0) / du;
    double a = a_raw;
    if (a < 0.0) a = 0.0;
    if (a > pb->n_spot - 1) a = pb->n_spot - 1;
    int32_t i = (int32_t)floor(a);
    if (i > pb->n_spot - 2) i = pb->n_spot - 2;
    double f = a - i;

    int32_t j;
    double alpha;
    lvo_time_cell_at(pb, t, &j, &alpha);

    const double *sg = pb->sigma;
    int32_t J = pb->n_time;
    double s00 = sg[i * J + j], s10 = sg[(i + 1) * J + j];
    double s01 = sg[i * J + j + 1], s11 = sg[(i + 1) * J + j + 1];

    out->i = i;
    out->j = j;
    out->w[0] = (1.0 - alpha) * (1.0 - f);
    out->w[1] = (1.0 - alpha) * f;
    out->w[2] = alpha * (1.0 - f);
    out->w[3] = alpha * f;
    out->sigma = out->w[0] * s00 + out->w[1] * s10 + out->w[2] * s01 + out->w[3] * s11;

    double dsdu = 0.0;
    if (a_raw > 0.0 && a_raw < pb->n_spot - 1)
        dsdu = ((1.0 - alpha) * (s10 - s00) + alpha * (s11 - s01)) / du;
    /* chain rule to y = ln(S/S0): du/dy = S on a linear axis, 1 on a log axis */
    out->dsigma_dy = (pb->spot_kind == 0) ? dsdu * S : dsdu;
}

/* ------------------------------------------------------------------------- */
/* One path: forward Euler in log-spot, payoffs, reverse sweep.              */
/* ------------------------------------------------------------------------- */
typedef struct {
    double *y;      /* [N+1] log-spot states */
    double *z;      /* [N]   normals */
    lvo_interp *iv; /* [N]   interpolation at (S_n, t_n) */
} lvo_work;

static void lvo_work_alloc(lvo_work *w, int32_t N)
{
    w->y = (double *)malloc(sizeof(double) * (N + 1));
    w->z = (double *)malloc(sizeof(double) * N);
    w->iv = (lvo_interp *)malloc(sizeof(lvo_interp) * N);
}

static void lvo_work_free(lvo_work *w)
{
    free(w->y); free(w->z); free(w->iv);
}

/* Payoff of option k at terminal log-spot y. */
static double lvo_payoff(const lvo_problem *pb, int k, double y)
{
    double S = pb->spot * exp(y);
    double K = pb->strike[k];
    if (pb->is_put[k]) return K > S ? K - S : 0.0;
    return S > K ? S - K : 0.0;
}

/* d payoff / d y: call S*1{S>K}, put -S*1{S<K} (zero at the kink). */
static double lvo_dpayoff_dy(const lvo_problem *pb, int k, double y)
{
    double S = pb->spot * exp(y);
    double K = pb->strike[k];
    if (pb->is_put[k]) return K > S ? -S : 0.0;
    return S > K ? S : 0.0;
}

/* Simulate path p forward; fill payoffs[k]; run the reverse sweep adding
 * lambda*c*w into grad (if non-NULL); return lambda at step 0 in *lam0. */
static void lvo_one_path(const lvo_problem *pb, uint64_t p, lvo_work *w,
                         double *payoffs, double *grad, double *lam0, double *lam_hist)
{
    int32_t N = pb->n_steps;
    double dt = pb->dt, sdt = pb->sqrt_dt;
    w->y[0] = 0.0;
    for (int32_t n = 0; n < N; ++n) {
        double S = pb->spot * exp(w->y[n]);
        lvo_eval(pb, S, n * dt, &w->iv[n]);
        w->z[n] = lvo_normal(pb->seed, p, n);
        double s = w->iv[n].sigma;
        w->y[n + 1] = w->y[n] + (pb->rate - 0.5 * s * s) * dt + s * sdt * w->z[n];
    }
    for (int k = 0; k < pb->n_opt; ++k)
        payoffs[k] = pb->disc[k] * lvo_payoff(pb, k, w->y[pb->tap_step[k]]);

    double lam = 0.0;
    int32_t J = pb->n_time;
    for (int32_t n = N; n >= 1; --n) {
        for (int k = 0; k < pb->n_opt; ++k)
            if (pb->tap_step[k] == n) {
                double wk = pb->weight ? pb->weight[k] : 1.0;
                lam += wk * pb->disc[k] * lvo_dpayoff_dy(pb, k, w->y[n]);
            }
        if (lam_hist) lam_hist[n] = lam;
        const lvo_interp *iv = &w->iv[n - 1];
        double c = -iv->sigma * dt + sdt * w->z[n - 1];  /* d y_n / d s_{n-1} */
        double gbar = lam * c;
        if (grad) {
            grad[iv->i * J + iv->j] += gbar * iv->w[0];
            grad[(iv->i + 1) * J + iv->j] += gbar * iv->w[1];
            grad[iv->i * J + iv->j + 1] += gbar * iv->w[2];
            grad[(iv->i + 1) * J + iv->j + 1] += gbar * iv->w[3];
        }
        lam = lam * (1.0 + c * iv->dsigma_dy);       /* d y_n / d y_{n-1} */
    }
    if (lam_hist) lam_hist[0] = lam;
    *lam0 = lam;
}

/* The explicit Euler step on X itself (scheme 1: the step as Sec. IV-A narrates
 * it, today's price plus a Gaussian term whose scale is sigma(X, t) X):
 *   X_{n+1} = X_n + sigma(X_n, t_n) X_n sqrt(dt) Z_n,
 * and its reverse sweep, with lambda the adjoint of X:
 *   d X_{n+1} / d sigma_n = X_n sqrt(dt) Z_n,
 *   d X_{n+1} / d X_n     = 1 + sqrt(dt) Z_n (sigma_n + X_n d sigma / d X),
 *   d payoff / d X        = 1{X > K} (call), -1{X < K} (put).
 * w->y holds X here.  lam_hist and *lam0 report the adjoint of ln X_n (lambda X_n),
 * the quantity the log scheme reports, so that sums and deltas read the same. */
static void lvo_one_path_euler_x(const lvo_problem *pb, uint64_t p, lvo_work *w,
                                 double *payoffs, double *grad, double *lam0, double *lam_hist)
{
    int32_t N = pb->n_steps;
    double dt = pb->dt, sdt = pb->sqrt_dt;
    double *X = w->y;
    X[0] = pb->spot;
    for (int32_t n = 0; n < N; ++n) {
        lvo_eval(pb, X[n], n * dt, &w->iv[n]);
        w->z[n] = lvo_normal(pb->seed, p, n);
        X[n + 1] = X[n] + pb->rate * X[n] * dt + w->iv[n].sigma * X[n] * sdt * w->z[n];
    }
    for (int k = 0; k < pb->n_opt; ++k) {
        double x = X[pb->tap_step[k]], K = pb->strike[k];
        payoffs[k] = pb->disc[k] * (pb->is_put[k] ? (K > x ? K - x : 0.0) : (x > K ? x - K : 0.0));
    }
    double lam = 0.0;
    int32_t J = pb->n_time;
    for (int32_t n = N; n >= 1; --n) {
        for (int k = 0; k < pb->n_opt; ++k)
            if (pb->tap_step[k] == n) {
                double wk = (pb->weight ? pb->weight[k] : 1.0) * pb->disc[k], K = pb->strike[k];
                if (pb->is_put[k]) lam -= K > X[n] ? wk : 0.0;
                else lam += X[n] > K ? wk : 0.0;
            }
        if (lam_hist) lam_hist[n] = lam * X[n];
        const lvo_interp *iv = &w->iv[n - 1];
        double c = X[n - 1] * sdt * w->z[n - 1];     /* d X_n / d s_{n-1} */
        if (grad) {
            /* nodes (i,j), (i+1,j), (i,j+1), (i+1,j+1) of the step's cell */
            int64_t q00 = (int64_t)iv->i * J + iv->j;
            grad[q00] += lam * c * iv->w[0];
            grad[q00 + J] += lam * c * iv->w[1];
            grad[q00 + 1] += lam * c * iv->w[2];
            grad[q00 + J + 1] += lam * c * iv->w[3];
        }
        /* X d sigma / d X = d sigma / d ln X */
        lam = lam * (1.0 + pb->rate * dt + sdt * w->z[n - 1] * (iv->sigma + iv->dsigma_dy));
    }
    if (lam_hist) lam_hist[0] = lam * X[0];
    *lam0 = lam * X[0];
}

/* ------------------------------------------------------------------------- */
/* Chunked, threaded accumulation over path ranges                           */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t begin, end;
} lvo_chunk;

typedef struct {
    const lvo_problem *pb;
    const lvo_chunk *chunks;
    int64_t n_chunks;
    int64_t next;             /* shared work counter */
    pthread_mutex_t lock;
    int want_grad;
    double *chunk_out;        /* [n_chunks][stride] */
    int64_t stride;
} lvo_job;

static void *lvo_worker(void *arg)
{
    lvo_job *job = (lvo_job *)arg;
    const lvo_problem *pb = job->pb;
    int n_opt = pb->n_opt;
    int64_t G = (int64_t)pb->n_spot * pb->n_time;
    lvo_work w;
    lvo_work_alloc(&w, pb->n_steps);
    double *pay = (double *)malloc(sizeof(double) * n_opt);
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int64_t c = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (c >= job->n_chunks) break;
        double *out = job->chunk_out + c * job->stride;
        /* layout: [sum_pay n_opt][sum_pay2 n_opt][sum_lam0 1][grad G] */
        memset(out, 0, sizeof(double) * job->stride);
        double *grad = job->want_grad ? out + 2 * n_opt + 1 : NULL;
        for (int64_t p = job->chunks[c].begin; p < job->chunks[c].end; ++p) {
            double lam0;
            if (pb->scheme == 1) lvo_one_path_euler_x(pb, (uint64_t)p, &w, pay, grad, &lam0, NULL);
            else lvo_one_path(pb, (uint64_t)p, &w, pay, grad, &lam0, NULL);
            for (int k = 0; k < n_opt; ++k) {
                out[k] += pay[k];
                out[n_opt + k] += pay[k] * pay[k];
            }
            out[2 * n_opt] += lam0;
        }
    }
    free(pay);
    lvo_work_free(&w);
    (void)G;
    return NULL;
}

/* Neumaier's compensated summation step. */
static void neumaier_add(double *sum, double *comp, double x)
{
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x))
        *comp += (*sum - t) + x;
    else
        *comp += (x - t) + *sum;
    *sum = t;
}

/*
 * Unnormalised sums over the union of half-open path ranges:
 *   sum_pay[k]  = sum_p payoff_k(p)          sum_pay2[k] = sum_p payoff_k(p)^2
 *   sum_grad[q] = sum_p d(sum_k w_k payoff_k(p)) / d sigma_q
 *   sum_lam0    = sum_p d(sum_k w_k payoff_k(p)) / d y_0
 * Returns 0, or -1 with a message in lvo_last_error().
 */
int lvo_accumulate(int32_t n_spot, int32_t spot_kind, double spot_lo, double spot_hi,
                   int32_t n_time, double time_lo, double time_hi, const double *sigma,
                   double spot, int32_t n_opt, const int32_t *is_put, const double *strike,
                   const double *maturity, const double *weight, int32_t n_steps, uint64_t seed,
                   int64_t n_ranges, const int64_t *ranges, int32_t n_threads,
                   double *sum_pay, double *sum_pay2, double *sum_grad, double *sum_lam0,
                   int32_t scheme, double rate)
{
    lvo_problem pb = {n_spot, spot_kind, spot_lo, spot_hi, n_time, time_lo, time_hi, sigma,
                      spot, n_opt, is_put, strike, maturity, weight, n_steps, seed, scheme, rate, 0, 0, NULL, NULL};
    if (lvo_setup(&pb) != 0) return -1;

    int64_t n_chunks = 0;
    for (int64_t r = 0; r < n_ranges; ++r) {
        int64_t len = ranges[2 * r + 1] - ranges[2 * r];
        if (len < 0 || ranges[2 * r] < 0) { lvo_release(&pb); return lvo_fail("bad path range"); }
        n_chunks += (len + LVO_CHUNK - 1) / LVO_CHUNK;
    }
    lvo_chunk *chunks = (lvo_chunk *)malloc(sizeof(lvo_chunk) * (n_chunks > 0 ? n_chunks : 1));
    int64_t ci = 0;
    for (int64_t r = 0; r < n_ranges; ++r)
        for (int64_t b = ranges[2 * r]; b < ranges[2 * r + 1]; b += LVO_CHUNK) {
            chunks[ci].begin = b;
            chunks[ci].end = b + LVO_CHUNK < ranges[2 * r + 1] ? b + LVO_CHUNK : ranges[2 * r + 1];
            ++ci;
        }

    int64_t G = (int64_t)n_spot * n_time;
    lvo_job job;
    job.pb = &pb;
    job.chunks = chunks;
    job.n_chunks = n_chunks;
    job.next = 0;
    pthread_mutex_init(&job.lock, NULL);
    job.want_grad = sum_grad != NULL;
    job.stride = 2 * n_opt + 1 + (sum_grad ? G : 0);
    job.chunk_out = (double *)malloc(sizeof(double) * job.stride * (n_chunks > 0 ? n_chunks : 1));

    if (n_threads < 1) n_threads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * n_threads);
    for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, lvo_worker, &job);
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&job.lock);

    /* merge chunk partials in chunk order */
    double *sum = (double *)calloc(job.stride, sizeof(double));
    double *comp = (double *)calloc(job.stride, sizeof(double));
    for (int64_t c = 0; c < n_chunks; ++c)
        for (int64_t q = 0; q < job.stride; ++q)
            neumaier_add(&sum[q], &comp[q], job.chunk_out[c * job.stride + q]);
    for (int k = 0; k < n_opt; ++k) {
        sum_pay[k] = sum[k] + comp[k];
        sum_pay2[k] = sum[n_opt + k] + comp[n_opt + k];
    }
    if (sum_lam0) *sum_lam0 = sum[2 * n_opt] + comp[2 * n_opt];
    if (sum_grad)
        for (int64_t q = 0; q < G; ++q) sum_grad[q] = sum[2 * n_opt + 1 + q] + comp[2 * n_opt + 1 + q];

    free(sum); free(comp);
    free(job.chunk_out);
    free(chunks);
    lvo_release(&pb);
    return 0;
}

/*
 * Everything about a single path p, for inspection:
 *   y[N+1] (ln(X/X0) for scheme 0, X for scheme 1), z[N], sigma[N], dsdy[N],
 *   lam[N+1] (the adjoint of ln X_n after the seeds of step n; lam[0] = d/dy_0),
 *   payoff[n_opt], grad[I*J] (this path's contribution).
 */
int lvo_path(int32_t n_spot, int32_t spot_kind, double spot_lo, double spot_hi,
             int32_t n_time, double time_lo, double time_hi, const double *sigma,
             double spot, int32_t n_opt, const int32_t *is_put, const double *strike,
             const double *maturity, const double *weight, int32_t n_steps, uint64_t seed,
             int64_t p, double *y, double *z, double *sig, double *dsdy, double *lam,
             double *payoff, double *grad, int32_t scheme, double rate)
{
    lvo_problem pb = {n_spot, spot_kind, spot_lo, spot_hi, n_time, time_lo, time_hi, sigma,
                      spot, n_opt, is_put, strike, maturity, weight, n_steps, seed, scheme, rate, 0, 0, NULL, NULL};
    if (lvo_setup(&pb) != 0) return -1;
    lvo_work w;
    lvo_work_alloc(&w, n_steps);
    int64_t G = (int64_t)n_spot * n_time;
    memset(grad, 0, sizeof(double) * G);
    double lam0;
    if (pb.scheme == 1) lvo_one_path_euler_x(&pb, (uint64_t)p, &w, payoff, grad, &lam0, lam);
    else lvo_one_path(&pb, (uint64_t)p, &w, payoff, grad, &lam0, lam);
    memcpy(y, w.y, sizeof(double) * (n_steps + 1));
    memcpy(z, w.z, sizeof(double) * n_steps);
    for (int32_t n = 0; n < n_steps; ++n) {
        sig[n] = w.iv[n].sigma;
        dsdy[n] = w.iv[n].dsigma_dy;
    }
    lvo_work_free(&w);
    lvo_release(&pb);
    return 0;
}

/*
 * Bilinear interpolation at (S, t) on its own, for checking the interpolant:
 * returns sigma, d sigma/d ln S, the lower-left node (i, j) and the 4 weights.
 */
int lvo_interp_at(int32_t n_spot, int32_t spot_kind, double spot_lo, double spot_hi,
                  int32_t n_time, double time_lo, double time_hi, const double *sigma,
                  double S, double t, double *sig, double *dsdy, int32_t *ij, double *w4)
{
    lvo_problem pb;
    memset(&pb, 0, sizeof pb);
    pb.n_spot = n_spot; pb.spot_kind = spot_kind; pb.spot_lo = spot_lo; pb.spot_hi = spot_hi;
    pb.n_time = n_time; pb.time_lo = time_lo; pb.time_hi = time_hi; pb.sigma = sigma;
    if (n_spot < 2 || n_time < 2 || !(S > 0.0)) return lvo_fail("bad interpolation query");
    lvo_interp iv;
    lvo_eval(&pb, S, t, &iv);
    *sig = iv.sigma;
    *dsdy = iv.dsigma_dy;
    ij[0] = iv.i;
    ij[1] = iv.j;
    memcpy(w4, iv.w, sizeof(double) * 4);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Reduced precision of the vol nodes (Sec. IV-D: the TPU runs keep sigma in  */
/* bfloat16 for the matrix-unit interpolation).  bfloat16 keeps the sign, the */
/* 8 exponent bits and the top 7 fraction bits of an IEEE single, so its      */
/* values are the singles whose low 16 bits are zero.  A node goes to single  */
/* precision first (to nearest, as a C cast does) and then to the nearer of   */
/* the two bfloat16 values that bracket it; at an exact tie, to the one whose */
/* last kept fraction bit is zero.  Finite inputs only.                       */
/* ------------------------------------------------------------------------- */
static float lvo_bits_to_float(uint32_t u)
{
    float f;
    memcpy(&f, &u, sizeof f);
    return f;
}

double lvo_round_bf16(double v)
{
    const float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    const uint32_t sign = u & 0x80000000u, mag = u & 0x7FFFFFFFu;
    const uint32_t below = mag & 0xFFFF0000u;    /* bracketing bfloat16 magnitudes */
    const uint32_t above = below + 0x10000u;     /* (the next one up carries into the exponent) */
    if (below == mag) return (double)f;          /* already a bfloat16 value */
    const double x = (double)lvo_bits_to_float(mag);
    const double lo = (double)lvo_bits_to_float(below), hi = (double)lvo_bits_to_float(above);
    const double d_lo = x - lo, d_hi = hi - x;   /* exact: all three are singles */
    uint32_t pick;
    if (d_lo < d_hi) pick = below;
    else if (d_hi < d_lo) pick = above;
    else pick = (below & 0x10000u) ? above : below;
    return (double)lvo_bits_to_float(sign | pick);
}

/* ------------------------------------------------------------------------- */
/* How far a single-precision computation of a path can be from this one.     */
/*                                                                           */
/* TEST SUPPORT, like the rest of this file.  A computation of the same       */
/* log-Euler path (Sec. IV-A) in IEEE single precision makes a local error in */
/* every step, and the step map carries earlier errors forward with its       */
/* derivative J_n = d y_{n+1} / d y_n = 1 + c_n s'_n (c_n = d y_{n+1} /       */
/* d sigma_n, s'_n = d sigma / d y at the step: the factors of the adjoint    */
/* recursion).  To first order the state error is bounded by the running sum  */
/*   e_0 = 0,   e_{n+1} = |J_n| e_n + rho_n,                                 */
/*   rho_n = u (k_step (|sigma_n sqrt(dt) Z_n| + sigma_n^2 dt / 2)             */
/*              + k_abs sigma_n sqrt(dt) R_n + |y_{n+1}|) + |c_n s'_n| cy_n    */
/* -- the increment computed with relative error k_step u, the normal also    */
/* with an absolute error k_abs u R_n (R_n the Box-Muller radius of its pair: */
/* near the zeros of sine and cosine their error is absolute, not relative), */
/* the new state rounded, and sigma_n read at a coordinate off by cy_n (the   */
/* coordinate's own rounding below, in units of y) -- with u the unit        */
/* roundoff.  The coordinate a_n is                                           */
/* known to within da_n = M (|da/dy| e_n + k_coord u (|a_n| + S_n / du on a    */
/* linear axis)), the second term (cy_n = that term / |da/dy|) being the      */
/* rounding of the coordinate itself (on a linear axis it comes with          */
/* S = X0 e^y), M a safety margin; where the nearest spot node lies within    */
/* da_n of a_n the step's cell is undecided at that precision (the slope of   */
/* the bilinear surface jumps there) and |J_n| takes its largest value over   */
/* the cells at the node.  model = {u, k_step, k_coord, M, k_abs}; e[N+1];    */
/* undecided[N].                                                              */
/* ------------------------------------------------------------------------- */
static double lvo_cell_slope_dy(const lvo_problem *pb, int c, double t, double S, double du)
{
    if (c < 0 || c > pb->n_spot - 2) return 0.0;
    int32_t j;
    double alpha;
    lvo_time_cell_at(pb, t, &j, &alpha);
    const double *sg = pb->sigma;
    int32_t J = pb->n_time;
    double dsdu = ((1.0 - alpha) * (sg[(c + 1) * J + j] - sg[c * J + j]) +
                   alpha * (sg[(c + 1) * J + j + 1] - sg[c * J + j + 1])) / du;
    return pb->spot_kind == 0 ? dsdu * S : dsdu;
}

int lvo_path_state_bound(int32_t n_spot, int32_t spot_kind, double spot_lo, double spot_hi,
                         int32_t n_time, double time_lo, double time_hi, const double *sigma,
                         double spot, int32_t n_opt, const int32_t *is_put, const double *strike,
                         const double *maturity, const double *weight, int32_t n_steps, uint64_t seed,
                         int64_t p, const double *model, double *e, int32_t *undecided, double rate)
{
    lvo_problem pb = {n_spot, spot_kind, spot_lo, spot_hi, n_time, time_lo, time_hi, sigma,
                      spot, n_opt, is_put, strike, maturity, weight, n_steps, seed, 0, rate, 0, 0, NULL, NULL};
    if (lvo_setup(&pb) != 0) return -1;
    const double u = model[0], ks = model[1], kc = model[2], M = model[3], ka = model[4];
    lvo_work w;
    lvo_work_alloc(&w, n_steps);
    double *pay = (double *)malloc(sizeof(double) * n_opt);
    double lam0;
    lvo_one_path(&pb, (uint64_t)p, &w, pay, NULL, &lam0, NULL);
    const double u0 = spot_kind == 0 ? spot_lo : log(spot_lo);
    const double u1 = spot_kind == 0 ? spot_hi : log(spot_hi);
    const double du = (u1 - u0) / (n_spot - 1), dt = pb.dt, sdt = pb.sqrt_dt;
    e[0] = 0.0;
    for (int32_t n = 0; n < n_steps; ++n) {
        const lvo_interp *iv = &w.iv[n];
        const double S = spot * exp(w.y[n]);
        const double a = ((spot_kind == 0 ? S : log(S)) - u0) / du;
        const double dady = spot_kind == 0 ? S / du : 1.0 / du;
        const double coord = kc * u * (fabs(a) + (spot_kind == 0 ? S / du : 0.0));   /* cells */
        const double da = M * (dady * e[n] + coord);
        const double c = -iv->sigma * dt + sdt * w.z[n];
        double jn = fabs(1.0 + c * iv->dsigma_dy);
        double k = floor(a + 0.5);
        if (k < 0.0) k = 0.0;
        if (k > n_spot - 1) k = n_spot - 1;
        undecided[n] = fabs(a - k) <= da;
        if (undecided[n]) {
            const int32_t kn = (int32_t)k;
            jn = fmax(jn, fabs(1.0 + c * lvo_cell_slope_dy(&pb, kn - 1, n * dt, S, du)));
            jn = fmax(jn, fabs(1.0 + c * lvo_cell_slope_dy(&pb, kn, n * dt, S, du)));
        }
        const double zp = lvo_normal(seed, (uint64_t)p, n ^ 1);   /* the other normal of the pair */
        const double radius = sqrt(w.z[n] * w.z[n] + zp * zp);
        e[n + 1] = jn * e[n] + u * (ks * (fabs(iv->sigma * sdt * w.z[n]) + 0.5 * iv->sigma * iv->sigma * dt) +
                                    ka * iv->sigma * sdt * radius + fabs(w.y[n + 1])) +
                   fabs(c * iv->dsigma_dy) * coord / dady;
    }
    free(pay);
    lvo_work_free(&w);
    lvo_release(&pb);
    return 0;
}

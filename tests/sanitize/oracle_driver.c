/* Test driver for the oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
 * (or ThreadSanitizer): every exported entry point on small inputs, both schemes, a
 * rate, several threads, several path ranges, with and without gradients, and the
 * error paths.  Prints a checksum and "ok"; the sanitizers abort on a finding. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void lvo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void lvo_normals(uint64_t seed, uint64_t p0, int64_t n_paths, int64_t n_steps, double *out);
double lvo_round_bf16(double v);
const char *lvo_last_error(void);
int lvo_accumulate(int32_t n_spot, int32_t spot_kind, double spot_lo, double spot_hi,
                   int32_t n_time, double time_lo, double time_hi, const double *sigma,
                   double spot, int32_t n_opt, const int32_t *is_put, const double *strike,
                   const double *maturity, const double *weight, int32_t n_steps, uint64_t seed,
                   int64_t n_ranges, const int64_t *ranges, int32_t n_threads,
                   double *sum_pay, double *sum_pay2, double *sum_grad, double *sum_lam0,
                   int32_t scheme, double rate);
int lvo_path(int32_t n_spot, int32_t spot_kind, double spot_lo, double spot_hi,
             int32_t n_time, double time_lo, double time_hi, const double *sigma,
             double spot, int32_t n_opt, const int32_t *is_put, const double *strike,
             const double *maturity, const double *weight, int32_t n_steps, uint64_t seed,
             int64_t p, double *y, double *z, double *sig, double *dsdy, double *lam,
             double *payoff, double *grad, int32_t scheme, double rate);
int lvo_interp_at(int32_t n_spot, int32_t spot_kind, double spot_lo, double spot_hi,
                  int32_t n_time, double time_lo, double time_hi, const double *sigma,
                  double S, double t, double *sig, double *dsdy, int32_t *ij, double *w4);
int lvo_path_state_bound(int32_t n_spot, int32_t spot_kind, double spot_lo, double spot_hi,
                         int32_t n_time, double time_lo, double time_hi, const double *sigma,
                         double spot, int32_t n_opt, const int32_t *is_put, const double *strike,
                         const double *maturity, const double *weight, int32_t n_steps, uint64_t seed,
                         int64_t p, const double *model, double *e, int32_t *undecided, double rate);

enum { I = 9, J = 5, N = 14, NOPT = 3 };

int main(int argc, char **argv)
{
    const int threads = argc > 1 ? atoi(argv[1]) : 4;
    double sigma[I * J];
    for (int i = 0; i < I; ++i)
        for (int j = 0; j < J; ++j) sigma[i * J + j] = 0.15 + 0.01 * ((i * 7 + j * 3) % 11);
    const int32_t is_put[NOPT] = {0, 1, 0};
    const double strike[NOPT] = {100.0, 95.0, 120.0}, maturity[NOPT] = {1.0, 0.5, 1.0};
    const double weight[NOPT] = {1.0, -0.5, 2.0};
    double check = 0.0;

    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    lvo_philox4x32_10(ctr, key, out);
    check += out[0] * 1e-9;
    double zs[3 * N];
    lvo_normals(7, 11, 3, N, zs);
    for (int k = 0; k < 3 * N; ++k) check += zs[k];
    check += lvo_round_bf16(0.123456789);

    const int64_t ranges[6] = {0, 1000, 4096, 5000, 9000, 9001};
    double pay[NOPT], pay2[NOPT], grad[I * J], lam0;
    for (int scheme = 0; scheme < 2; ++scheme)
        for (int kind = 0; kind < 2; ++kind)
            for (int r = 0; r < 2; ++r) {
                const double rate = r ? 0.03 : 0.0;
                if (lvo_accumulate(I, kind, 60.0, 160.0, J, 0.0, 1.0, sigma, 100.0, NOPT, is_put, strike,
                                   maturity, weight, N, 3, 3, ranges, threads, pay, pay2, grad, &lam0, scheme,
                                   rate) != 0) {
                    fprintf(stderr, "accumulate: %s\n", lvo_last_error());
                    return 1;
                }
                for (int k = 0; k < NOPT; ++k) check += pay[k] * 1e-6 + pay2[k] * 1e-9;
                for (int q = 0; q < I * J; ++q) check += grad[q] * 1e-6;
                check += lam0 * 1e-6;
                /* price only */
                if (lvo_accumulate(I, kind, 60.0, 160.0, J, 0.0, 1.0, sigma, 100.0, NOPT, is_put, strike,
                                   maturity, weight, N, 3, 3, ranges, threads, pay, pay2, NULL, NULL, scheme,
                                   rate) != 0)
                    return 1;
                double y[N + 1], z[N], sg[N], dsdy[N], lam[N + 1], po[NOPT], gp[I * J];
                if (lvo_path(I, kind, 60.0, 160.0, J, 0.0, 1.0, sigma, 100.0, NOPT, is_put, strike, maturity,
                             weight, N, 3, 17, y, z, sg, dsdy, lam, po, gp, scheme, rate) != 0)
                    return 1;
                check += y[N] + lam[0] * 1e-3;
            }
    const double model[5] = {pow(2.0, -24), 8.0, 8.0, 4.0, 16.0};
    double e[N + 1];
    int32_t und[N];
    if (lvo_path_state_bound(I, 0, 60.0, 160.0, J, 0.0, 1.0, sigma, 100.0, NOPT, is_put, strike, maturity,
                             weight, N, 3, 5, model, e, und, 0.01) != 0)
        return 1;
    check += e[N] * 1e6;
    double s1, d1, w4[4];
    int32_t ij[2];
    if (lvo_interp_at(I, 1, 60.0, 160.0, J, 0.0, 1.0, sigma, 101.0, 0.3, &s1, &d1, ij, w4) != 0) return 1;
    check += s1 + d1;
    /* error paths: a bad range, a bad interpolation query */
    const int64_t bad[2] = {10, 5};
    if (lvo_accumulate(I, 0, 60.0, 160.0, J, 0.0, 1.0, sigma, 100.0, NOPT, is_put, strike, maturity, weight,
                       N, 3, 1, bad, threads, pay, pay2, grad, &lam0, 0, 0.0) == 0)
        return 2;
    if (lvo_interp_at(I, 1, 60.0, 160.0, J, 0.0, 1.0, sigma, -1.0, 0.3, &s1, &d1, ij, w4) == 0) return 2;
    printf("checksum %.17g\nok\n", check);
    return 0;
}

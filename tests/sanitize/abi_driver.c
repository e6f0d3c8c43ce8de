/* Host-only entry points of the library under the sanitizers: request validation
 * (lv_check) over a valid request and one mutation per rule, the state-buffer size,
 * the autotuner's candidate shapes and the option order.  No GPU work is done (and
 * none is needed).  Prints each validation case's status, then "abi <digest of every
 * result> <count> ok"; every build must print the same. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "lvmc.h"

static uint64_t digest = 1469598103934665603ull;
static int n_checks = 0;

static void mix(long long v) {
    digest = (digest ^ (uint64_t)v) * 1099511628211ull;
    ++n_checks;
}

enum { I0 = 21, J0 = 13 };

typedef struct {
    lv_grid grid;
    double sigma[I0 * J0];
    double spot;
    int32_t put[3];
    double strike[3], maturity[3], weight[3];
    lv_book book;
    int64_t n_paths;
    int32_t n_steps;
    lv_opts opts;
} request;

static void valid(request *r) {
    memset(r, 0, sizeof *r);
    r->grid.spot.n = I0;
    r->grid.spot.kind = LV_AXIS_LIN;
    r->grid.spot.lo = 50.0;
    r->grid.spot.hi = 150.0;
    r->grid.time.n = J0;
    r->grid.time.kind = LV_AXIS_LIN;
    r->grid.time.lo = 0.0;
    r->grid.time.hi = 1.0;
    for (int e = 0; e < I0 * J0; ++e) r->sigma[e] = 0.2 + 0.001 * (e % 7);
    r->spot = 100.0;
    const int32_t put[3] = {0, 1, 0};
    const double K[3] = {100.0, 95.0, 105.0}, T[3] = {1.0, 0.5, 0.25}, w[3] = {1.0, -0.5, 2.0};
    memcpy(r->put, put, sizeof put);
    memcpy(r->strike, K, sizeof K);
    memcpy(r->maturity, T, sizeof T);
    memcpy(r->weight, w, sizeof w);
    r->book.n_opt = 3;
    r->book.is_put = r->put;
    r->book.strike = r->strike;
    r->book.maturity = r->maturity;
    r->book.weight = r->weight;
    r->n_paths = 1 << 16;
    r->n_steps = 52;
}

static lv_status check(const request *r) {
    return lv_check(&r->grid, r->sigma, r->spot, &r->book, r->n_paths, r->n_steps, &r->opts);
}

int main(void) {
    request r;
    valid(&r);
    mix(check(&r));

    /* one mutation per rule */
    for (int m = 0; m < 32; ++m) {
        valid(&r);
        switch (m) {
            case 0: r.spot = 0.0; break;
            case 1: r.spot = NAN; break;
            case 2: r.sigma[17] = NAN; break;
            case 3: r.sigma[0] = -0.1; break;
            case 4: r.n_paths = 1; break;
            case 5: r.n_steps = 0; break;
            case 6: r.maturity[1] = 0.3; break;                      /* 15.6 steps */
            case 7: r.strike[2] = 0.0; break;
            case 8: r.maturity[0] = -1.0; break;
            case 9: r.grid.spot.n = 1; break;
            case 10: r.grid.spot.kind = LV_AXIS_LOG; r.grid.spot.lo = 0.0; break;
            case 11: r.grid.spot.hi = r.grid.spot.lo; break;
            case 12: r.grid.time.kind = LV_AXIS_LOG; break;
            case 13: r.opts.precision = 16; break;
            case 14: r.opts.block = 100; break;
            case 15: r.opts.copies = 3; break;
            case 16: r.opts.window = 12; break;
            case 17: r.opts.ckpt_every = 12; r.opts.adjoint = LV_ADJ_CHECKPOINT; break;
            case 18: r.opts.precision = 64; r.opts.block = 1024; break;
            case 19: r.opts.sigma_bf16 = 2; break;
            case 20: r.opts.rate = 2.0; break;
            case 21: r.opts.rate = NAN; break;
            case 22: r.opts.scheme = 5; break;
            case 23: r.book.n_opt = 0; break;
            case 24: r.book.n_opt = 257; break;
            case 25: r.n_paths = ((int64_t)1 << 38) + 320; r.opts.block = 64; r.opts.fwd_block = 64; break;
            case 26: r.n_paths = (int64_t)1 << 40; break;
            case 27: r.n_paths = ((int64_t)1 << 40) + 1; break;
            case 28: r.opts.adjoint = LV_ADJ_CHECKPOINT; break;
            case 29: r.opts.adjoint = LV_ADJ_NONE; r.opts.precision = 64; break;
            case 30: r.grid.spot.kind = LV_AXIS_LOG; r.grid.spot.lo = 40.0; r.grid.spot.hi = 250.0; break;
            case 31: r.opts.scheme = LV_SCHEME_EULER_X; r.opts.rate = 0.03; break;
        }
        /* a book of 257 options needs arrays that long: keep the first three and
           point the rest at the last one's values */
        static int32_t put257[257];
        static double K257[257], T257[257], w257[257];
        if (r.book.n_opt == 257) {
            for (int k = 0; k < 257; ++k) {
                put257[k] = 0;
                K257[k] = 100.0;
                T257[k] = 1.0;
                w257[k] = 1.0;
            }
            r.book.is_put = put257;
            r.book.strike = K257;
            r.book.maturity = T257;
            r.book.weight = w257;
        }
        const lv_status st = check(&r);
        printf("case %d status %d\n", m, (int)st);
        mix(st);
        if (st != LV_OK) mix((long long)strlen(lv_last_error(NULL)) > 0);
    }

    /* NULL arguments */
    valid(&r);
    mix(lv_check(NULL, r.sigma, r.spot, &r.book, r.n_paths, r.n_steps, &r.opts));
    mix(lv_check(&r.grid, r.sigma, r.spot, NULL, r.n_paths, r.n_steps, &r.opts));
    mix(lv_check(&r.grid, NULL, r.spot, &r.book, r.n_paths, r.n_steps, &r.opts));   /* sigma optional */

    /* state-buffer sizes */
    size_t bytes = 0;
    mix(lv_states_bytes(32, 1 << 19, 156, &bytes));
    mix((long long)bytes);
    mix(lv_states_bytes(64, 1 << 19, 156, &bytes));
    mix((long long)bytes);
    mix(lv_states_bytes(16, 1 << 19, 156, &bytes));
    mix(lv_states_bytes(32, 1, 156, &bytes));

    /* the autotuner's candidates, every mode */
    static int32_t shapes[512 * 6];
    for (int adj = LV_ADJ_NONE; adj <= LV_ADJ_CHECKPOINT; ++adj) {
        valid(&r);
        r.opts.adjoint = adj;
        int32_t n = 0;
        mix(lv_tuning_candidates(&r.grid, &r.book, r.n_paths, r.n_steps, &r.opts, shapes, 512, &n));
        mix(n);
        for (int e = 0; e < n * 6; ++e) mix(shapes[e]);
        mix(lv_tuning_candidates(&r.grid, &r.book, r.n_paths, r.n_steps, &r.opts, shapes, 2, &n));
        mix(n);
    }

    /* option order */
    valid(&r);
    int32_t order[3] = {-1, -1, -1};
    mix(lv_debug_option_order(&r.book, r.n_steps, order));
    for (int k = 0; k < 3; ++k) mix(order[k]);

    printf("abi %016llx %d ok\n", (unsigned long long)digest, n_checks);
    return 0;
}

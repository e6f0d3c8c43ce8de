/*
 * lvmc.h -- C ABI of the MI355X (gfx950) local-volatility Monte Carlo library:
 * option prices under the Dupire local-volatility model and the adjoint
 * sensitivities of a book's value to every node of the volatility grid.
 *
 * Method (arXiv 2002.02481, "Sensitivity Analysis in the Dupire Local
 * Volatility Model with Tensorflow"):
 *   - the asset follows dX/X = sigma(X,t) dW (Sec. IV-A, the SDE), or with a
 *     constant short rate r (lv_opts.rate) dX/X = r dt + sigma(X,t) dW, the
 *     deterministic trend of the step Sec. IV-A narrates, payoffs discounted by
 *     e^{-r T}; r = 0 (the default) is the paper's driftless SDE;
 *   - an explicit Euler scheme (Sec. IV-A) on y = ln(X/X0) with Ito drift:
 *       y_{n+1} = y_n + (r - sigma_n^2 / 2) dt + sigma_n sqrt(dt) Z_n,  y_0 = 0,
 *     with sigma_n = sigma(X0 e^{y_n}, n dt) read at the left end of the step;
 *   - sigma(S,t) is bilinear in the nodes of a grid {(i dx, j dt)} (Sec. IV-A,
 *     the grid definition; Sec. IV-D, bilinear interpolation), linear in the
 *     spot axis coordinate (S, or ln S for a log-spaced axis), flat outside;
 *   - Z_n are Gaussian (Sec. IV-B, normal generator) from Philox4x32-10 (Salmon
 *     et al., SC'11) with key = seed and counter = (n/4, path): the four words
 *     w0..w3 give, through u(w) = ((w >> 9) + 1/2) 2^-23 and Box-Muller,
 *     Z_{4m}   = r(w0) cos(2 pi u(w1)),  Z_{4m+1} = r(w0) sin(2 pi u(w1)),
 *     Z_{4m+2} = r(w2) cos(2 pi u(w3)),  Z_{4m+3} = r(w2) sin(2 pi u(w3)),
 *     r(w) = sqrt(-2 ln u(w));
 *   - European call/put payoffs at each option's maturity, averaged over
 *     paths (Sec. IV-B, IV-C): price_k = e^{-r T_k} mean_p payoff_k, std_err_k =
 *     sqrt(sample variance / P) of the discounted payoff;
 *   - the gradient of the weighted book value sum_k w_k price_k with respect to
 *     every vol node by reverse-mode differentiation of the simulation
 *     (Sec. III, Sec. IV-C), i.e. the average over paths of each path's
 *     back-propagated derivative; delta = d value / d X0 comes with it.
 *
 * Time grid: dt = max_k maturity_k / n_steps; each maturity must be a whole
 * number of steps (to 1e-9 n_steps), else LV_ERR_STEP.  Path p (0 <= p <
 * n_paths) consumes Philox counter words (m, p) for m = 0 .. ceil(n_steps/4)-1
 * only, so results for any path are reproducible in isolation.  Limits:
 * n_steps <= 1e6, spot nodes x time nodes <= 1e5, n_steps x spot nodes <= 2^26
 * (the per-step vol table), at most 256 options; beyond them LV_ERR_ARG or
 * LV_ERR_UNSUPPORTED.
 *
 * Conventions: all functions return an lv_status; on failure the context's
 * message (lv_last_error) says why and no output has been written.  "Host"
 * pointers are ordinary CPU memory owned by the caller; "device" pointers are
 * HBM of the context's GPU owned by the caller.  Calls that take device
 * pointers are asynchronous on the context's stream; calls that take host
 * outputs block until the outputs are written.  A context is not thread-safe:
 * use one context per host thread / stream.
 */
#ifndef LVMC_H
#define LVMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LV_OK = 0,
    LV_ERR_ARG = 1,         /* invalid argument (NULL, non-positive size, bad option) */
    LV_ERR_GRID = 2,        /* invalid grid: fewer than 2x2 nodes, bad axis, sigma not finite and > 0 */
    LV_ERR_STEP = 3,        /* a maturity is not a whole number of steps */
    LV_ERR_NOMEM = 4,       /* device workspace could not be allocated */
    LV_ERR_HIP = 5,         /* a HIP runtime call failed */
    LV_ERR_UNSUPPORTED = 6  /* valid request the library does not handle (e.g. too many options) */
} lv_status;

enum { LV_AXIS_LIN = 0, LV_AXIS_LOG = 1 };
enum { LV_ADJ_DEFAULT = 0, LV_ADJ_NONE = 1, LV_ADJ_STORED = 2, LV_ADJ_CHECKPOINT = 3 };

typedef struct lv_ctx lv_ctx;

/* An axis of n >= 2 inclusive nodes uniform in the axis coordinate between lo
 * and hi: S for LV_AXIS_LIN, ln S for LV_AXIS_LOG (lo > 0 required).  The time
 * axis must be LV_AXIS_LIN. */
typedef struct {
    int32_t n;
    int32_t kind;
    double lo;
    double hi;
} lv_axis;

/* The vol grid (Sec. IV-A): sigma[i * time.n + j] is the node at spot node i and
 * time node j (row-major [spot.n][time.n]). */
typedef struct {
    lv_axis spot;
    lv_axis time;
} lv_grid;

/* A book of European options on one underlying (host arrays of n_opt entries).
 * weight: cotangent of each option in the book value (NULL = all 1). */
typedef struct {
    int32_t n_opt;
    const int32_t *is_put;
    const double *strike;
    const double *maturity;
    const double *weight;
} lv_book;

/* Execution options.  Zero-initialised fields take defaults. */
typedef struct {
    int32_t precision;      /* 32 (FP32 stepping and adjoint, FP64 cross-path sums) or 64; default 32 */
    int32_t adjoint;        /* LV_ADJ_NONE (price only), LV_ADJ_STORED (all states kept in HBM),
                               LV_ADJ_CHECKPOINT (states every ckpt_every steps, segments recomputed
                               from the Philox counters); LV_ADJ_DEFAULT = LV_ADJ_STORED */
    int32_t ckpt_every;     /* checkpoint segment length: 8, 16 or 32 steps; default 16 */
    int32_t use_graph;      /* 1: capture the launch sequence in a hipGraph per shape and replay it */
    int32_t block;          /* threads per block of the adjoint (or fused) kernel, a multiple of 64 in
                               [64, 1024] (FP32) or [64, 512] (FP64, else LV_ERR_UNSUPPORTED);
                               0 = tuned default */
    int32_t blocks_per_cu;  /* persistent blocks per compute unit; 0 = tuned default */
    int32_t copies;         /* privatised copies of the LDS gradient histogram (1..16); 0 = default */
    int32_t window;         /* steps per LDS vol-table window (multiple of 8 in [8, 64]); the gradient
                               histogram spans the largest multiple of it that the LDS budget of
                               blocks_per_cu blocks allows (up to the whole horizon); 0 = default.
                               The checkpointed kernel plans its own: 1, 2 or 4 segments */
    int32_t profile;        /* 1: time every kernel with hipEvents (eager launches only), read back
                               with lv_kernel_times */
    int32_t autotune;       /* 1: on the first call of a shape (grid, steps, paths, book size,
                               precision, adjoint), time every candidate launch shape that the
                               shape fields leave free and keep the fastest for this context */
    int32_t fwd_block;      /* threads per block of the separate forward kernel (stored and
                               price-only paths); 0 = tuned default */
    int32_t fwd_blocks_per_cu; /* persistent blocks per CU of that forward kernel; 0 = default */
    int32_t dense_adjoint;  /* stored and checkpointed adjoints: 1 = sweep every path back;
                               0 (default) = sweep only the paths with an option of nonzero
                               cotangent in the money at its maturity, since every other path
                               has a zero adjoint and contributes exactly nothing */
    int32_t profile_kinds;  /* with profile: bit (1 << LV_K_*) set = time that kernel kind; 0 = all.
                               A timed dispatch waits for its timestamp (several microseconds),
                               so timing only the kernel of interest keeps the others' pace */
    int32_t scheme;         /* LV_SCHEME_LOG_EULER (default): the explicit Euler step on
                               y = ln(X/X0) with the Ito drift -sigma^2/2; LV_SCHEME_EULER_X: the
                               explicit Euler step on X itself, X += sigma(X, t) X sqrt(dt) Z, as
                               Sec. IV-A narrates the scheme, in every adjoint mode.  The split
                               calls lv_forward_dev / lv_backward_dev step log-Euler. */
    int32_t sigma_bf16;     /* 1: round every node of sigma to bfloat16 (FP64 -> FP32 -> bfloat16,
                               each to nearest with ties to even) before the vol table is built:
                               the precision in which the paper's mixed-precision TPU runs hold
                               sigma for the matrix-unit interpolation (Sec. IV-D).  Prices and
                               gradients are then those of the rounded surface, the gradient
                               being taken with respect to its nodes.  0 (default): sigma as
                               given; any other value is LV_ERR_ARG */
    double rate;            /* constant short rate r (per year, continuously compounded): each step
                               adds the trend r dt to ln X (r dt X to X on the Euler step on X),
                               and every price, standard error, gradient and delta is discounted
                               by e^{-r T_k} of its option; 0 (default) = the driftless SDE.
                               Finite with |r| <= 1, else LV_ERR_ARG */
} lv_opts;

enum { LV_SCHEME_LOG_EULER = 0, LV_SCHEME_EULER_X = 1 };

/* Create a context on HIP device `device` that launches on `hip_stream`
 * (a hipStream_t; NULL = a stream the context creates, which, like every stream
 * made without flags, is ordered with the null stream).  The context owns a device
 * workspace that grows on demand and is freed by lv_destroy.  If the environment
 * variable LVMC_TUNING_FILE names a file, lv_create loads the saved tunings in it
 * (as lv_tuning_load; a file that is not a tuning file fails lv_create with
 * LV_ERR_ARG), and every shape the autotuner then chooses is written back to it: its
 * lines for other devices or other request shapes are kept, this context's shapes
 * replace or follow them, and the file is replaced by renaming a temporary file
 * written beside it (a failure to write fails the autotuned call with LV_ERR_ARG). */
lv_status lv_create(lv_ctx **out, int device, void *hip_stream);
void lv_destroy(lv_ctx *ctx);
/* Launch later calls on `hip_stream` (NULL as for lv_create).  When the stream
 * changes, the call first waits for the work queued on the previous one, which may
 * still use the context's buffers; LV_ERR_HIP if that wait fails. */
lv_status lv_set_stream(lv_ctx *ctx, void *hip_stream);

/* Message of the last failed call on ctx (ctx may be NULL: the last failure of
 * a call made without a usable context on this thread).  Never NULL. */
const char *lv_last_error(const lv_ctx *ctx);

/* Host-side validation of a request, with no GPU access: returns what the
 * pricing calls would return before launching anything.  sigma (host) may be
 * NULL to skip the node checks. */
lv_status lv_check(const lv_grid *grid, const double *sigma, double spot, const lv_book *book,
                   int64_t n_paths, int32_t n_steps, const lv_opts *opts);

/* Price, standard error, vol-grid gradient and delta of a book (the fused call).
 * sigma: host [I*J].  price, std_err: host [n_opt].  grad: host [I*J] gradient of
 * sum_k weight_k price_k, or NULL to skip (then the adjoint is not run).
 * delta: host [1] d(book value)/d spot, or NULL.  Blocks until done. */
lv_status lv_price_and_grad(lv_ctx *ctx, const lv_grid *grid, const double *sigma, double spot,
                            const lv_book *book, int64_t n_paths, int32_t n_steps, uint64_t seed,
                            const lv_opts *opts, double *price, double *std_err, double *grad,
                            double *delta);

/* The same for n_surf surfaces on the same Philox streams (common random
 * numbers): sigmas host [n_surf][I*J]; prices, std_errs host [n_surf][n_opt];
 * grads host [n_surf][I*J] or NULL; deltas host [n_surf] or NULL. */
lv_status lv_price_and_grad_batch(lv_ctx *ctx, const lv_grid *grid, int32_t n_surf,
                                  const double *sigmas, double spot, const lv_book *book,
                                  int64_t n_paths, int32_t n_steps, uint64_t seed,
                                  const lv_opts *opts, double *prices, double *std_errs,
                                  double *grads, double *deltas);

/* Device-resident form of lv_price_and_grad_batch, asynchronous on the
 * context's stream: sigmas_dev [n_surf][I*J] FP64 device; prices_dev,
 * std_errs_dev [n_surf][n_opt], grads_dev [n_surf][I*J] (or NULL), deltas_dev
 * [n_surf] (or NULL) FP64 device.  The book stays a host description. */
lv_status lv_price_and_grad_dev(lv_ctx *ctx, const lv_grid *grid, int32_t n_surf,
                                const double *sigmas_dev, double spot, const lv_book *book,
                                int64_t n_paths, int32_t n_steps, uint64_t seed,
                                const lv_opts *opts, double *prices_dev, double *std_errs_dev,
                                double *grads_dev, double *deltas_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): lv_price_and_grad_dev
 * with the same arguments and results, computed by the same kernels, but working
 * only in a fixed per-GPU workspace of 64 MiB that the library holds from its
 * load until the process ends; it calls no hipMalloc, hipFree or allocating
 * library routine.  The caller still owns the inputs and outputs (device
 * pointers as above).  The workspace holds the request's step and option tables,
 * the per-step vol table, the per-block partial records and the stored states
 * (LV_ADJ_STORED: n_steps x n_paths values) or the checkpoints (LV_ADJ_CHECKPOINT:
 * a few segments per resident path, small); a request that needs more than 64 MiB
 * returns LV_ERR_UNSUPPORTED before anything is launched, as do the same
 * validation errors as lv_price_and_grad_dev.  use_graph, autotune and profile
 * must be 0 (else LV_ERR_ARG); a launch shape this context has already tuned for
 * the request (through lv_price_and_grad_dev with autotune) is used.  The tables
 * are copied host to device on the context's stream.  Every call on one GPU uses
 * that GPU's one workspace, which keeps the last call's contents: calls that
 * overlap on one GPU (other streams, other contexts, other threads) race, so the
 * caller serialises them.  Asynchronous on the context's stream. */
lv_status lv_price_and_grad_noalloc(lv_ctx *ctx, const lv_grid *grid, int32_t n_surf,
                                    const double *sigmas_dev, double spot, const lv_book *book,
                                    int64_t n_paths, int32_t n_steps, uint64_t seed,
                                    const lv_opts *opts, double *prices_dev, double *std_errs_dev,
                                    double *grads_dev, double *deltas_dev);

/* Bump-and-reprice: the vol-grid gradient by the finite differences the adjoint
 * replaces (arXiv 2002.02481, Sec. III: one simulation at p + eps/2, one at
 * p - eps/2, the difference over eps), for comparison with it.  For every node
 * (i, j), the book is priced on sigma with sigma_ij moved by +eps/2 and by -eps/2,
 * forward only, on the same Philox paths as the adjoint (common random numbers),
 * and grad_dev[i*J + j] = sum_k weight_k (price_k(+) - price_k(-)) / eps.
 * sigma_dev: [I*J] FP64 device; grad_dev: [I*J] FP64 device, caller-owned.  eps:
 * absolute vol bump, finite and > 0 (a node with sigma_ij <= eps/2 is priced with
 * a non-positive vol: the caller picks eps).  2 I J surfaces are priced, at most
 * `batch` nodes (2 batch surfaces) per batch (0 = 256), through the same kernels as
 * lv_price_and_grad_dev with adjoint NONE; opts->adjoint is ignored.  Device
 * workspace: (2 batch (I J + 2 n_opt) + n_opt) doubles, held by the context.
 * Asynchronous on the context's stream; LV_ERR_ARG for a bad eps or batch. */
lv_status lv_bump_grad_dev(lv_ctx *ctx, const lv_grid *grid, const double *sigma_dev, double spot,
                           const lv_book *book, int64_t n_paths, int32_t n_steps, uint64_t seed,
                           const lv_opts *opts, double eps, int32_t batch, double *grad_dev);

/* Bytes of the path-state buffer the split calls use: n_steps planes of
 * n_paths values (float for precision 32, double for 64), plane n holding
 * y_{n+1} of every path (path index contiguous). */
lv_status lv_states_bytes(int32_t precision, int64_t n_paths, int32_t n_steps, size_t *bytes);

/* Split forward (for autograd): simulate, write every state into states_dev
 * (device, caller-owned, lv_states_bytes long) and per-option price and
 * std_err (device [n_opt] FP64), log-Euler with rate `rate` (as lv_opts.rate).
 * Asynchronous on the context's stream.  The book's weights are ignored here. */
lv_status lv_forward_dev(lv_ctx *ctx, const lv_grid *grid, const double *sigma_dev, double spot,
                         const lv_book *book, int64_t n_paths, int32_t n_steps, uint64_t seed,
                         int32_t precision, double rate, void *states_dev, double *price_dev,
                         double *std_err_dev);

/* Split backward: from the states of lv_forward_dev (same arguments) and a
 * device cotangent [n_opt] (d loss / d price_k), write grad_dev [I*J] =
 * sum_k cotangent_k d price_k / d sigma and, if non-NULL, delta_dev [1].
 * Asynchronous on the context's stream.  The book's weights are ignored. */
lv_status lv_backward_dev(lv_ctx *ctx, const lv_grid *grid, const double *sigma_dev, double spot,
                          const lv_book *book, int64_t n_paths, int32_t n_steps, uint64_t seed,
                          int32_t precision, double rate, const void *states_dev,
                          const double *cotangent_dev, double *grad_dev, double *delta_dev);

/* Per-option vol-grid gradients from one simulation (Sec. III, Sec. IV-C: the
 * sensitivities of every price of a book, not only of a weighted sum): from the
 * states of lv_forward_dev (same arguments; log-Euler, rate as there), write
 * grads_dev [n_opt][I*J] = d price_k / d sigma for every option k (caller order)
 * and, if non-NULL, deltas_dev [n_opt] = d price_k / d spot.  One reverse sweep over
 * the paths serves up to 8 options: the state, vol lookup and step derivative of a
 * path step are shared, each option carrying its own adjoint, seeded by its own
 * payoff only, and its own LDS gradient histogram (fewer options per sweep on grids
 * whose per-option histograms do not fit a block's LDS).  The book's weights are
 * ignored.  Asynchronous on the context's stream. */
lv_status lv_per_option_grads_dev(lv_ctx *ctx, const lv_grid *grid, const double *sigma_dev, double spot,
                                  const lv_book *book, int64_t n_paths, int32_t n_steps, uint64_t seed,
                                  int32_t precision, double rate, const void *states_dev, double *grads_dev,
                                  double *deltas_dev);

/* Test support: Philox words of paths p0 .. p0+n_paths-1 for counter blocks
 * m0 .. m0+n_m-1 into words_dev (device uint32 [n_paths][n_m][4]). */
lv_status lv_debug_philox(lv_ctx *ctx, uint64_t seed, uint64_t m0, int32_t n_m, uint64_t p0,
                          int64_t n_paths, uint32_t *words_dev);

/* Test support: normals Z_n, n < n_steps, of paths p0 .. p0+n_paths-1 as the
 * kernels draw them, into z_dev (device [n_paths][n_steps], float for precision
 * 32, double for 64). */
lv_status lv_debug_normals(lv_ctx *ctx, int32_t precision, uint64_t seed, uint64_t p0,
                           int64_t n_paths, int32_t n_steps, void *z_dev);

/* Launch facts of the last pricing call on ctx, so tests can recompute the
 * partial sums of single blocks: block b handled the path tiles t = b, b + n_blocks,
 * ... of tile_paths paths each. */
typedef struct {
    int32_t n_blocks;
    int32_t block;
    int32_t tile_paths;
    int32_t waves_per_block;
    int32_t fixed_point_bits;   /* F of the FP32/FP64 fixed-point gradient histogram (last surface) */
    int32_t adjoint;
    int32_t precision;
    int32_t graph_replayed;     /* 1 if the last call replayed a captured graph */
    int32_t copies;             /* histogram copies of the launch */
    int32_t window;             /* steps per LDS table window (for the checkpoint kernel 1, 2 or 4
                                   segments, as many as its LDS holds) */
    int32_t blocks_per_cu;      /* persistent blocks per CU asked for */
    int32_t autotuned;          /* 1 if the shape came from the autotuner */
    int32_t fwd_block;          /* threads per block of the separate forward kernel */
    int32_t fwd_blocks_per_cu;  /* its blocks per CU asked for */
    int32_t fwd_blocks;         /* its grid (its payoff partials are records 0 .. fwd_blocks-1) */
    int64_t overflow_terms;     /* reserved: 0 */
    int32_t hist_window;        /* steps per gradient-histogram window (a multiple of window) */
} lv_run_info;

/* The launch shapes the autotuner would time for this request, as rows of
 * (block, copies, window, blocks_per_cu, fwd_block, fwd_blocks_per_cu) in
 * shapes_out (host int32 [max][6]): the adjoint-kernel candidates with the
 * default forward shape, then the forward candidates with the default adjoint
 * shape (the two kernels are tuned one after the other).  *n_out receives the
 * number of rows written.  Host only (device 0's properties are read when a
 * device is present, else 256 CUs are assumed). */
lv_status lv_tuning_candidates(const lv_grid *grid, const lv_book *book, int64_t n_paths,
                               int32_t n_steps, const lv_opts *opts, int32_t *shapes_out,
                               int32_t max, int32_t *n_out);

/* Launch shapes the autotuner chose, kept across processes.  lv_tuning_save writes
 * every shape this context has tuned to the text file `path` (overwritten), one line
 * per request shape, tagged with the device's architecture name and CU count;
 * *n_out (may be NULL) receives the number of lines.  lv_tuning_load reads such a
 * file into the context's cache: lines of another architecture or CU count are
 * skipped, and a request whose key matches a loaded line takes that shape under
 * lv_opts.autotune (and in the allocation-free entry point) without timing
 * candidates; *n_out receives the number of lines taken.  A line that is not a
 * saved tuning, or holds a shape lv_opts would refuse, gives LV_ERR_ARG (lines
 * before it are kept); so does a file that cannot be opened.  Host only: no GPU
 * work, the context's stream is not touched. */
lv_status lv_tuning_save(const lv_ctx *ctx, const char *path, int32_t *n_out);
lv_status lv_tuning_load(lv_ctx *ctx, const char *path, int32_t *n_out);

lv_status lv_last_run_info(const lv_ctx *ctx, lv_run_info *info);

/* Kernel kinds timed when lv_opts.profile is set. */
enum { LV_K_FWD = 0, LV_K_REV = 1, LV_K_FUSED = 2, LV_K_MERGE = 3, LV_K_TABLE = 4, LV_K_COUNT = 5 };

/* Accumulated device time (ms, from hipEvents on the context's stream) and launch
 * counts per kernel kind, over all profiled calls since the last reset; waits
 * for the stream.  ms and counts are host arrays of LV_K_COUNT entries.  reset = 1
 * clears the totals after reading. */
lv_status lv_kernel_times(lv_ctx *ctx, double *ms, int64_t *counts, int32_t reset);

/* Test support: copy the per-block partial records of the last surface of the last
 * pricing call to host memory (unnormalised FP64, [n_blocks][2 n_opt + 1 + I*J]:
 * per option in maturity order sum payoff and sum payoff^2, then sum of
 * d(value)/d y_0, then the gradient grid), before the merge.  host_len is the
 * number of doubles host_out holds.  The option order is that of
 * lv_debug_option_order. */
lv_status lv_debug_block_partials(lv_ctx *ctx, double *host_out, size_t host_len);

/* Test support: the caller index of each option in the order of the partial
 * records (options sorted by maturity step, ties in caller order). */
lv_status lv_debug_option_order(const lv_book *book, int32_t n_steps, int32_t *order_out);

#ifdef __cplusplus
}
#endif

#endif /* LVMC_H */

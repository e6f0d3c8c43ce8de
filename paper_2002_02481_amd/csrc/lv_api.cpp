// lv_api.cpp -- host runtime and C ABI of the local-vol Monte Carlo library
// (include/lvmc.h): request validation, launch planning, the device workspace,
// hipGraph capture/replay and the fused, batched and split entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include <unistd.h>

#include "lv_internal.h"
#include "lvmc.h"

namespace {

thread_local std::string g_last_error = "no error";

struct Buf {
    void *p = nullptr;
    size_t n = 0;
};

// Launch shape: threads per block, histogram copies, window (steps), blocks per CU.
struct Shape {
    int block = 512, K = 2, W = 16, bpc = 2;   // adjoint (or fused) kernel
    int fblock = 512, fbpc = 2;                // separate forward kernel
};

// Everything derived from one request: the time table, the book in maturity
// order, the launch shape.
struct Plan {
    int I = 0, J = 0, N = 0, axis = 0;
    double inv_du = 0, a_off = 0, spot = 0, dt = 0, sqrt_dt = 0;
    long long P = 0;
    uint64_t seed = 0;
    int n_opt = 0, n_taps = 0;
    std::vector<int> tj, cell_lo, tap_step, tap_first, tap_count, opt_put, opt_orig;
    std::vector<double> ta, opt_strike, weight, opt_disc;   // opt_disc: e^{-r T_k}, tap order
    double rate = 0;
    int precision = 32, adjoint = LV_ADJ_STORED, seg = 16, profile = 0;   // profile: kinds to time (bits)
    int tws = 1;   // checkpointed: segments per vol-table window (1, 2 or 4)
    int block = 256, blocks = 0, n_tiles = 0, W = 16, WH = 16, K = 8, bpc = 2, CH = 1;
    int dense = 0;   // reverse kernel sweeps every path (not only those with a nonzero adjoint)
    int scheme = 0;  // 0: Euler on ln X; 1: Euler on X
    int bf16 = 0;    // 1: sigma rounded to bfloat16 before the table is built
    int fblock = 256, fblocks = 0, f_n_tiles = 0, fbpc = 2;
    int G = 0, Q = 0;
    Shape user{0, 0, 0, 0, 0, 0};   // caller-fixed shape fields (0 = free)
    bool autotune = false;
};

}  // namespace

struct lv_ctx {
    int device = 0;
    hipStream_t user_stream = nullptr;
    hipStream_t own_stream = nullptr;
    int n_cu = 256;
    size_t max_lds = 65536;
    std::string arch = "unknown";                // gcnArchName of the device (keys saved tunings)
    std::string err = "no error";
    Buf planbuf, part, states, ckpt, sig_stage, out_stage, gtab, bump;
    std::vector<char> plan_bytes;     // what planbuf holds
    lv_run_info info{};
    int last_Q = 0, last_G = 0, last_nopt = 0;   // record layout of the last call's partials
    const void *last_part = nullptr;             // where they are
    void *scratch = nullptr;                     // this device's allocation-free workspace
    std::vector<char> scratch_tables;            // host copy of the tables it last uploaded
    std::map<std::string, Shape> tuned;          // autotuner results per request shape
    std::string tune_path;                       // LVMC_TUNING_FILE at creation ("" = none)
    bool last_autotuned = false;
    // kernel timing (lv_opts.profile)
    struct Timed {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Timed> pending;
    std::vector<hipEvent_t> event_pool;
    double k_ms[LV_K_COUNT] = {0};
    int64_t k_count[LV_K_COUNT] = {0};
    // graph cache (one entry)
    std::string graph_key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;

    hipStream_t stream() const { return user_stream ? user_stream : own_stream; }
};

namespace {

lv_status fail(lv_ctx *ctx, lv_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    g_last_error = buf;
    return st;
}

#define HIPCHECK(ctx, call)                                                                 \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, LV_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

lv_status ensure(lv_ctx *ctx, Buf &b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.n >= bytes) return LV_OK;
    if (b.p) {
        hipError_t e = hipStreamSynchronize(ctx->stream());
        if (e != hipSuccess) return fail(ctx, LV_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
        (void)hipFree(b.p);
        b.p = nullptr;
        b.n = 0;
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(ctx, LV_ERR_NOMEM, "device workspace of %zu bytes: %s", bytes, hipGetErrorString(e));
    }
    b.n = bytes;
    return LV_OK;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// ---------------------------------------------------------------------------
// Launch shapes
// ---------------------------------------------------------------------------
long long floor_pow2(long long x) {
    long long p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}

// Table window of the adjoint (or fused) kernel: the checkpoint segment for the
// fused kernel.
int table_window(const Plan &pl, const Shape &sh) {
    return pl.adjoint == LV_ADJ_CHECKPOINT ? pl.seg * pl.tws : sh.W;
}

// Path tiles per live-path list of the stored reverse kernel (all of a block's
// tiles, up to 4), and checkpoint slot sets in the fused kernel's ring (up to 4: each
// holds a tile's checkpoints, and its final states in LDS, while paths of that tile
// wait in the queue).
int chunk_tiles(const Plan &pl, const Shape &sh, int n_cu) {
    const long long tiles = (pl.P + sh.block - 1) / sh.block;
    const long long blocks = std::min<long long>(tiles, (long long)n_cu * sh.bpc);
    return (int)std::max<long long>(1, std::min<long long>(4, (tiles + blocks - 1) / blocks));
}

size_t lds_adj(const Plan &pl, const Shape &sh, int WH, int n_cu) {
    const int var = pl.adjoint == LV_ADJ_CHECKPOINT ? lvk::FUSED_CKPT : lvk::REV_STORED;
    return lvk::lds_bytes(var, pl.precision, pl.I, pl.J, pl.n_opt, sh.block, table_window(pl, sh), WH, sh.K,
                          chunk_tiles(pl, sh, n_cu));
}

size_t lds_fwd(const Plan &pl, const Shape &sh) {
    return lvk::lds_bytes(lvk::FWD_STORE, pl.precision, pl.I, pl.J, pl.n_opt, sh.fblock, table_window(pl, sh), 0,
                          sh.K, 0);
}

// Whether the shape fits the CU's LDS with the smallest histogram window.
bool shape_fits(const Plan &pl, const Shape &sh, size_t max_lds, int n_cu) {
    return lds_adj(pl, sh, table_window(pl, sh), n_cu) <= max_lds && lds_fwd(pl, sh) <= max_lds;
}

// Histogram window: the largest multiple of the table window (up to the whole
// horizon) whose block still leaves room for the blocks per CU the shape asks
// for (at most 2048 lanes per CU).  Fewer windows mean fewer folds.
int hist_window(const Plan &pl, const Shape &sh, size_t max_lds, int n_cu) {
    const int W = table_window(pl, sh);
    const long long whole = ((long long)pl.N + W - 1) / W * W;
    const int resident = std::max(1, std::min(sh.bpc, 2048 / sh.block));
    const size_t budget = max_lds / resident;
    const size_t base = lds_adj(pl, sh, 0, n_cu);
    const size_t per_step = (size_t)(pl.I + 1) * sh.K * (pl.precision == 64 ? 8 : 4);
    long long wh = budget > base ? (long long)((budget - base) / per_step) / W * W : 0;
    wh = std::min(wh, whole);
    while (wh > W && lds_adj(pl, sh, (int)wh, n_cu) > budget) wh -= W;   // alignment padding
    return (int)std::max<long long>(W, wh);
}

// Largest number of path tiles one launch takes (see apply_shape).
constexpr long long kMaxTiles = (1ll << 30);

// Defaults from launch-shape sweeps on MI355X: 1024-lane blocks with 2 histogram
// copies and 32-step windows when there are enough paths for a block per CU;
// smaller blocks for smaller problems so that every CU gets work.
Shape default_shape(const Plan &pl, int n_cu) {
    Shape sh;
    const int bmax = lvk::adjoint_max_block(pl.precision == 64 ? 8 : 4);
    sh.block = (int)std::min<long long>(bmax, std::max<long long>(64, floor_pow2(pl.P / n_cu)));
    sh.K = 2;
    sh.W = 32;
    sh.bpc = 1;
    sh.fblock = (int)std::min<long long>(512, std::max<long long>(64, floor_pow2(pl.P / (2 * n_cu))));
    if ((pl.P + sh.fblock - 1) / sh.fblock > kMaxTiles) sh.fblock = 1024;   // the largest path counts
    sh.fbpc = 4;
    return sh;
}

// Fix a shape into the plan.  If a block does not fit the CU's LDS even with the
// smallest histogram window, the table window, then the copies, are shrunk
// (unless the caller fixed them).
lv_status apply_shape(lv_ctx *ctx, Plan &pl, Shape sh, int n_cu, size_t max_lds, bool may_shrink_k,
                      bool may_shrink_w) {
    const bool ckpt = pl.adjoint == LV_ADJ_CHECKPOINT;
    if (ckpt) {
        // the fused kernel stages the vol table up to four segments at a time (fewer block
        // barriers and table copies): as many as the horizon uses and the block's LDS holds
        // beside the smallest histogram window
        pl.tws = 4;
        while (pl.tws > 1 && (long long)pl.seg * (pl.tws / 2) >= pl.N) pl.tws /= 2;
        while (pl.tws > 1 && !shape_fits(pl, sh, max_lds, n_cu)) pl.tws /= 2;
    }
    while (!shape_fits(pl, sh, max_lds, n_cu) && sh.W > 8 && may_shrink_w && !ckpt) sh.W /= 2;
    while (!shape_fits(pl, sh, max_lds, n_cu) && sh.K > 1 && may_shrink_k) sh.K /= 2;
    if (!shape_fits(pl, sh, max_lds, n_cu))
        return fail(ctx, LV_ERR_UNSUPPORTED, "shape needs %zu bytes of LDS per block (limit %zu)",
                    std::max(lds_adj(pl, sh, table_window(pl, sh), n_cu), lds_fwd(pl, sh)), max_lds);
    const int bmax = lvk::adjoint_max_block(pl.precision == 64 ? 8 : 4);
    if (sh.block > bmax)
        return fail(ctx, LV_ERR_UNSUPPORTED, "the FP%d adjoint kernels run at most %d threads per block (asked %d)",
                    pl.precision, bmax, sh.block);
    pl.block = sh.block;
    pl.K = sh.K;
    pl.W = table_window(pl, sh);
    pl.WH = hist_window(pl, sh, max_lds, n_cu);
    if (lds_adj(pl, sh, pl.WH, n_cu) > max_lds)   // the window search keeps this; never launch past it
        return fail(ctx, LV_ERR_UNSUPPORTED, "planner: histogram window of %d steps needs %zu bytes of LDS (limit %zu)",
                    pl.WH, lds_adj(pl, sh, pl.WH, n_cu), max_lds);
    // Tile counts are computed in 64 bits and must fit the kernels' int tile loops,
    // whose counters run up to a tile count plus one stride of the grid (at most
    // 4 tiles per list x 64 blocks per CU x the CUs), so they are capped well below 2^31.
    const long long n_tiles = (pl.P + sh.block - 1) / sh.block;
    const long long f_n_tiles = (pl.P + sh.fblock - 1) / sh.fblock;
    if (n_tiles > kMaxTiles || f_n_tiles > kMaxTiles)
        return fail(ctx, LV_ERR_UNSUPPORTED,
                    "%lld paths need %lld tiles of %d (forward: %lld of %d); at most %lld tiles per launch",
                    pl.P, n_tiles, sh.block, f_n_tiles, sh.fblock, kMaxTiles);
    pl.CH = chunk_tiles(pl, sh, n_cu);
    pl.bpc = sh.bpc;
    pl.n_tiles = (int)n_tiles;
    pl.blocks = (int)std::min<long long>(n_tiles, (long long)n_cu * sh.bpc);
    pl.fblock = sh.fblock;
    pl.fbpc = sh.fbpc;
    pl.f_n_tiles = (int)f_n_tiles;
    pl.fblocks = (int)std::min<long long>(f_n_tiles, (long long)n_cu * sh.fbpc);
    return LV_OK;
}

// Candidate shapes the autotuner times (every one is a valid launch): first the
// forward kernel's (block, blocks per CU) with the default adjoint shape, then the
// adjoint kernel's (block, copies, window, blocks per CU) with the chosen forward.
std::vector<Shape> forward_candidates(const Plan &pl, const Shape &base, int n_cu, size_t max_lds) {
    std::vector<Shape> out;
    if (pl.adjoint == LV_ADJ_CHECKPOINT) return out;   // the fused kernel has no separate forward
    const int bmax = (int)std::min<long long>(1024, std::max<long long>(64, floor_pow2(2 * pl.P / n_cu)));
    for (int b : {128, 256, 512, 1024}) {
        if (b > bmax && b != 128) continue;
        for (int c : {1, 2, 4, 8}) {
            Shape sh = base;
            sh.fblock = b;
            sh.fbpc = c;
            if (!shape_fits(pl, sh, max_lds, n_cu)) continue;
            out.push_back(sh);
        }
    }
    return out;
}

std::vector<Shape> adjoint_candidates(const Plan &pl, const Shape &base, int n_cu, size_t max_lds) {
    std::vector<Shape> out;
    const int bmax = (int)std::min<long long>(lvk::adjoint_max_block(pl.precision == 64 ? 8 : 4),
                                              std::max<long long>(64, floor_pow2(2 * pl.P / n_cu)));
    for (int b : {128, 256, 512, 1024}) {
        if (b > bmax && b != 128) continue;
        for (int k : {1, 2, 4})
            for (int w : {8, 16, 32}) {
                if (pl.adjoint == LV_ADJ_CHECKPOINT && w != 8) continue;   // window = segment
                for (int c : {1, 2, 4}) {
                    Shape sh = base;
                    sh.block = b;
                    sh.K = k;
                    sh.W = w;
                    sh.bpc = c;
                    if (!shape_fits(pl, sh, max_lds, n_cu)) continue;
                    out.push_back(sh);
                }
            }
    }
    if (out.empty()) out.push_back(base);
    return out;
}

// ---------------------------------------------------------------------------
// Validation and planning (host only, no GPU access)
// ---------------------------------------------------------------------------
lv_status plan_request(lv_ctx *ctx, const lv_grid *grid, int n_surf, const double *sigma_host,
                       double spot, const lv_book *book, int64_t n_paths, int32_t n_steps,
                       uint64_t seed, const lv_opts *opts, int n_cu, size_t max_lds, Plan &pl) {
    if (!grid) return fail(ctx, LV_ERR_ARG, "grid is NULL");
    const lv_axis &sa = grid->spot, &ta = grid->time;
    if (sa.n < 2 || ta.n < 2) return fail(ctx, LV_ERR_GRID, "grid needs at least 2x2 nodes (got %dx%d)", sa.n, ta.n);
    if ((long long)sa.n * ta.n > 100000) return fail(ctx, LV_ERR_UNSUPPORTED, "grid of %d x %d nodes is too large", sa.n, ta.n);
    if (sa.kind != LV_AXIS_LIN && sa.kind != LV_AXIS_LOG) return fail(ctx, LV_ERR_GRID, "unknown spot axis kind %d", sa.kind);
    if (ta.kind != LV_AXIS_LIN) return fail(ctx, LV_ERR_GRID, "time axis must be linear");
    if (!(std::isfinite(sa.lo) && std::isfinite(sa.hi) && sa.hi > sa.lo)) return fail(ctx, LV_ERR_GRID, "spot axis needs finite lo < hi");
    if (sa.kind == LV_AXIS_LOG && !(sa.lo > 0)) return fail(ctx, LV_ERR_GRID, "log spot axis needs lo > 0");
    if (!(std::isfinite(ta.lo) && std::isfinite(ta.hi) && ta.hi > ta.lo)) return fail(ctx, LV_ERR_GRID, "time axis needs finite lo < hi");
    const long long G = (long long)sa.n * ta.n;
    if (sigma_host) {
        for (long long q = 0; q < G * n_surf; ++q)
            if (!finite_pos(sigma_host[q])) return fail(ctx, LV_ERR_GRID, "sigma node %lld is not finite and positive", q % G);
    }
    if (!finite_pos(spot)) return fail(ctx, LV_ERR_ARG, "spot must be finite and positive");
    if (!book || book->n_opt < 1 || !book->is_put || !book->strike || !book->maturity)
        return fail(ctx, LV_ERR_ARG, "book needs n_opt >= 1 and non-NULL is_put, strike, maturity");
    if (book->n_opt > 256) return fail(ctx, LV_ERR_UNSUPPORTED, "at most 256 options per book (got %d)", book->n_opt);
    if (n_paths < 2 || n_paths > (1ll << 40)) return fail(ctx, LV_ERR_ARG, "n_paths must be in [2, 2^40]");
    if (n_steps < 1 || n_steps > 1000000) return fail(ctx, LV_ERR_ARG, "n_steps must be in [1, 1e6]");
    if ((long long)n_steps * sa.n > (1ll << 26))
        return fail(ctx, LV_ERR_UNSUPPORTED, "n_steps x spot nodes = %lld exceeds the vol table limit 2^26",
                    (long long)n_steps * sa.n);
    if (n_surf < 1) return fail(ctx, LV_ERR_ARG, "n_surf must be >= 1");
    lv_opts o{};
    if (opts) o = *opts;
    if (o.precision == 0) o.precision = 32;
    if (o.precision != 32 && o.precision != 64) return fail(ctx, LV_ERR_ARG, "precision must be 32 or 64");
    if (o.adjoint < 0 || o.adjoint > 3) return fail(ctx, LV_ERR_ARG, "unknown adjoint mode %d", o.adjoint);
    if (o.adjoint == LV_ADJ_DEFAULT) o.adjoint = LV_ADJ_STORED;
    if (o.scheme != LV_SCHEME_LOG_EULER && o.scheme != LV_SCHEME_EULER_X)
        return fail(ctx, LV_ERR_ARG, "unknown scheme %d", o.scheme);
    if (o.sigma_bf16 != 0 && o.sigma_bf16 != 1) return fail(ctx, LV_ERR_ARG, "sigma_bf16 must be 0 or 1");
    if (!(std::isfinite(o.rate) && std::fabs(o.rate) <= 1.0)) return fail(ctx, LV_ERR_ARG, "rate must be finite with |r| <= 1");
    if (o.ckpt_every == 0) o.ckpt_every = 16;
    if (o.ckpt_every != 8 && o.ckpt_every != 16 && o.ckpt_every != 32)
        return fail(ctx, LV_ERR_ARG, "ckpt_every must be 8, 16 or 32");
    if (o.block != 0 && (o.block % 64 != 0 || o.block < 64 || o.block > 1024))
        return fail(ctx, LV_ERR_ARG, "block must be a multiple of 64 in [64, 1024]");
    if (o.blocks_per_cu < 0 || o.blocks_per_cu > 64) return fail(ctx, LV_ERR_ARG, "blocks_per_cu must be in [0, 64]");
    if (o.copies < 0 || o.copies > 16) return fail(ctx, LV_ERR_ARG, "copies must be in [0, 16]");
    if (o.window < 0 || o.window % 8 != 0 || o.window > 64) return fail(ctx, LV_ERR_ARG, "window must be a multiple of 8 in [8, 64]");

    double tmax = 0.0;
    for (int k = 0; k < book->n_opt; ++k) {
        if (!finite_pos(book->strike[k])) return fail(ctx, LV_ERR_ARG, "strike %d must be finite and positive", k);
        if (!finite_pos(book->maturity[k])) return fail(ctx, LV_ERR_ARG, "maturity %d must be finite and positive", k);
        if (book->is_put[k] != 0 && book->is_put[k] != 1) return fail(ctx, LV_ERR_ARG, "is_put %d must be 0 or 1", k);
        if (book->weight && !std::isfinite(book->weight[k])) return fail(ctx, LV_ERR_ARG, "weight %d not finite", k);
        tmax = std::max(tmax, book->maturity[k]);
    }
    pl = Plan();
    pl.I = sa.n;
    pl.J = ta.n;
    pl.N = n_steps;
    pl.axis = sa.kind;
    pl.spot = spot;
    pl.dt = tmax / n_steps;
    pl.sqrt_dt = std::sqrt(pl.dt);
    pl.P = n_paths;
    pl.seed = seed;
    pl.n_opt = book->n_opt;
    pl.precision = o.precision;
    pl.adjoint = o.adjoint;
    pl.seg = o.ckpt_every;
    pl.profile = o.profile ? (o.profile_kinds ? o.profile_kinds : (1 << LV_K_COUNT) - 1) : 0;
    pl.dense = o.dense_adjoint ? 1 : 0;
    pl.scheme = o.scheme;
    pl.bf16 = o.sigma_bf16;
    pl.rate = o.rate;
    pl.G = (int)G;
    pl.Q = 2 * pl.n_opt + 1 + pl.G;

    // maturities -> tap steps
    std::vector<int> steps(pl.n_opt);
    for (int k = 0; k < pl.n_opt; ++k) {
        const double x = book->maturity[k] / pl.dt;
        const double r = std::floor(x + 0.5);
        if (std::fabs(x - r) > 1e-9 * n_steps || r < 1.0)
            return fail(ctx, LV_ERR_STEP, "maturity %d (%.17g) is not a whole number of steps of %.17g", k,
                        book->maturity[k], pl.dt);
        steps[k] = (int)r;
    }
    std::vector<int> order(pl.n_opt);
    for (int k = 0; k < pl.n_opt; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return steps[a] < steps[b]; });
    for (int q = 0; q < pl.n_opt; ++q) {
        const int k = order[q];
        pl.opt_orig.push_back(k);
        pl.opt_put.push_back(book->is_put[k]);
        pl.opt_strike.push_back(book->strike[k]);
        pl.opt_disc.push_back(std::exp(-pl.rate * book->maturity[k]));
        if (q == 0 || steps[k] != pl.tap_step.back()) {
            pl.tap_step.push_back(steps[k]);
            pl.tap_first.push_back(q);
            pl.tap_count.push_back(0);
        }
        pl.tap_count.back() += 1;
    }
    pl.n_taps = (int)pl.tap_step.size();
    for (int k = 0; k < pl.n_opt; ++k) pl.weight.push_back(book->weight ? book->weight[k] : 1.0);

    // spot axis coordinate -> grid coordinate
    double u0, u1;
    if (sa.kind == LV_AXIS_LOG) {
        u0 = std::log(sa.lo);
        u1 = std::log(sa.hi);
    } else {
        u0 = sa.lo;
        u1 = sa.hi;
    }
    const double du = (u1 - u0) / (sa.n - 1);
    pl.inv_du = 1.0 / du;
    pl.a_off = sa.kind == LV_AXIS_LOG ? (std::log(spot) - u0) / du : -u0 / du;

    // time cell of every step: b = clamp((t_n - t_0)/dtau, 0, J-1), j = min(floor b, J-2)
    const double dtau = (ta.hi - ta.lo) / (ta.n - 1);
    pl.tj.resize(n_steps);
    pl.ta.resize(n_steps);
    for (int n = 0; n < n_steps; ++n) {
        double b = (n * pl.dt - ta.lo) / dtau;
        b = std::min(std::max(b, 0.0), (double)(ta.n - 1));
        int j = std::min((int)std::floor(b), ta.n - 2);
        pl.tj[n] = j;
        pl.ta[n] = b - j;
    }
    // first step of every time cell (t_n increases, so a cell's steps are contiguous)
    pl.cell_lo.assign(ta.n, n_steps);
    for (int n = 0, jn = 0; n < n_steps; ++n)
        while (jn <= pl.tj[n]) pl.cell_lo[jn++] = n;

    // launch shape: explicit options win; otherwise the tuned shape (autotune)
    // or the default heuristics
    pl.user.block = o.block;
    pl.user.K = o.copies;
    pl.user.W = o.window;
    pl.user.bpc = o.blocks_per_cu;
    pl.user.fblock = o.fwd_block;
    pl.user.fbpc = o.fwd_blocks_per_cu;
    pl.autotune = o.autotune != 0;
    if (o.fwd_block != 0 && (o.fwd_block % 64 != 0 || o.fwd_block < 64 || o.fwd_block > 1024))
        return fail(ctx, LV_ERR_ARG, "fwd_block must be a multiple of 64 in [64, 1024]");
    if (o.fwd_blocks_per_cu < 0 || o.fwd_blocks_per_cu > 64)
        return fail(ctx, LV_ERR_ARG, "fwd_blocks_per_cu must be in [0, 64]");
    if (o.copies && (o.copies & (o.copies - 1)))
        return fail(ctx, LV_ERR_ARG, "copies must be a power of two");
    Shape sh = default_shape(pl, n_cu);
    if (o.block) sh.block = o.block;
    if (o.copies) sh.K = o.copies;
    if (o.window) sh.W = o.window;
    if (o.blocks_per_cu) sh.bpc = o.blocks_per_cu;
    if (o.fwd_block) sh.fblock = o.fwd_block;
    if (o.fwd_blocks_per_cu) sh.fbpc = o.fwd_blocks_per_cu;
    return apply_shape(ctx, pl, sh, n_cu, max_lds, !o.copies, !o.window);
}

int host_fixed_point_bits(const Plan &pl) {
    const double qmax = lvk::fixed_point_qmax(pl.precision, pl.block, pl.K, pl.P);
    double scale = 0.0;
    for (int q = 0; q < pl.n_opt; ++q)
        scale += std::fabs(pl.weight[pl.opt_orig[q]]) * std::max(pl.spot, pl.opt_strike[q]);
    const int fmaxb = pl.precision == 64 ? 62 : 40;
    if (!(scale > 0.0)) return fmaxb;
    const int F = std::ilogb(qmax / (8.0 * scale));
    return std::max(-30, std::min(fmaxb, F));
}

// Pack the plan's device tables; upload only when they change.
struct Tables {
    const int *tj, *cell_lo, *tap_step, *tap_first, *tap_count, *opt_put, *opt_orig;
    const double *ta, *opt_strike, *weight, *opt_disc;
};

template <typename T>
void put(std::vector<char> &v, const std::vector<T> &x, size_t &off) {
    off = (v.size() + 15) & ~(size_t)15;
    v.resize(off + x.size() * sizeof(T) + 16);
    if (!x.empty()) std::memcpy(v.data() + off, x.data(), x.size() * sizeof(T));
}

// Byte offsets of the packed tables inside one buffer.
struct TableOffsets {
    size_t o[11];
};

std::vector<char> pack_tables(const Plan &pl, TableOffsets &to) {
    std::vector<char> v;
    size_t *o = to.o;
    put(v, pl.tj, o[0]);
    put(v, pl.cell_lo, o[9]);
    put(v, pl.tap_step, o[1]);
    put(v, pl.tap_first, o[2]);
    put(v, pl.tap_count, o[3]);
    put(v, pl.opt_put, o[4]);
    put(v, pl.opt_orig, o[5]);
    put(v, pl.ta, o[6]);
    put(v, pl.opt_strike, o[7]);
    put(v, pl.weight, o[8]);
    put(v, pl.opt_disc, o[10]);
    return v;
}

Tables tables_at(const void *base, const TableOffsets &to) {
    const char *b = (const char *)base;
    const size_t *o = to.o;
    Tables t;
    t.tj = (const int *)(b + o[0]);
    t.cell_lo = (const int *)(b + o[9]);
    t.tap_step = (const int *)(b + o[1]);
    t.tap_first = (const int *)(b + o[2]);
    t.tap_count = (const int *)(b + o[3]);
    t.opt_put = (const int *)(b + o[4]);
    t.opt_orig = (const int *)(b + o[5]);
    t.ta = (const double *)(b + o[6]);
    t.opt_strike = (const double *)(b + o[7]);
    t.weight = (const double *)(b + o[8]);
    t.opt_disc = (const double *)(b + o[10]);
    return t;
}

lv_status upload_tables(lv_ctx *ctx, const Plan &pl, Tables &t) {
    TableOffsets to;
    std::vector<char> v = pack_tables(pl, to);
    lv_status st = ensure(ctx, ctx->planbuf, v.size());
    if (st != LV_OK) return st;
    if (v != ctx->plan_bytes) {
        // the stream may still read the old tables
        HIPCHECK(ctx, hipStreamSynchronize(ctx->stream()));
        HIPCHECK(ctx, hipMemcpy(ctx->planbuf.p, v.data(), v.size(), hipMemcpyHostToDevice));
        ctx->plan_bytes.swap(v);
    }
    t = tables_at(ctx->planbuf.p, to);
    return LV_OK;
}

// Device buffers one launch sequence works in: the context's own (grown on demand)
// or, for the allocation-free entry point, regions of the per-GPU workspace.
struct Space {
    void *part = nullptr, *states = nullptr, *ckpt = nullptr, *gtab = nullptr;
};

Space ctx_space(const lv_ctx *ctx) {
    Space w;
    w.part = ctx->part.p;
    w.states = ctx->states.p;
    w.ckpt = ctx->ckpt.p;
    w.gtab = ctx->gtab.p;
    return w;
}

lvk::Args make_args(const Space &w, const Plan &pl, const Tables &t, const double *sigma_dev) {
    lvk::Args a{};
    a.I = pl.I;
    a.J = pl.J;
    a.N = pl.N;
    a.axis = pl.axis;
    a.inv_du = pl.inv_du;
    a.a_off = pl.a_off;
    a.spot = pl.spot;
    a.dt = pl.dt;
    a.sqrt_dt = pl.sqrt_dt;
    a.sigma = sigma_dev;
    a.tj = t.tj;
    a.ta = t.ta;
    a.cell_lo = t.cell_lo;
    a.gtab = w.gtab;
    a.P = pl.P;
    a.key0 = (unsigned)(pl.seed & 0xFFFFFFFFu);
    a.key1 = (unsigned)(pl.seed >> 32);
    a.n_opt = pl.n_opt;
    a.n_taps = pl.n_taps;
    a.tap_step = t.tap_step;
    a.tap_first = t.tap_first;
    a.tap_count = t.tap_count;
    a.opt_put = t.opt_put;
    a.opt_strike = t.opt_strike;
    a.opt_orig = t.opt_orig;
    a.cot = t.weight;
    a.opt_disc = t.opt_disc;
    a.rate_dt = pl.rate * pl.dt;
    a.Q = pl.Q;
    a.n_tiles = pl.n_tiles;
    a.W = pl.W;
    a.WH = pl.WH;
    a.K = pl.K;
    a.CH = pl.CH;
    a.dense = pl.dense;
    a.scheme = pl.scheme;
    a.sigma_bf16 = pl.bf16;
    a.seg = pl.seg;
    return a;
}

size_t real_bytes(int precision) { return precision == 64 ? 8 : 4; }

// The per-step vol table every pricing kernel reads.
lv_status ensure_table(lv_ctx *ctx, const Plan &pl) {
    return ensure(ctx, ctx->gtab, (size_t)pl.N * pl.I * 2 * real_bytes(pl.precision));
}

// Workspace for the fused paths.
lv_status ensure_workspace(lv_ctx *ctx, const Plan &pl, bool adjoint) {
    lv_status st;
    if ((st = ensure_table(ctx, pl)) != LV_OK) return st;
    if ((st = ensure(ctx, ctx->part, (size_t)std::max(pl.blocks, pl.fblocks) * pl.Q * 8)) != LV_OK) return st;
    if (adjoint && pl.adjoint == LV_ADJ_STORED) {
        const size_t b = (size_t)pl.N * (size_t)pl.P * real_bytes(pl.precision);
        if ((st = ensure(ctx, ctx->states, b)) != LV_OK) return st;
    }
    if (adjoint && pl.adjoint == LV_ADJ_CHECKPOINT) {
        const size_t nseg = (pl.N + pl.seg - 1) / pl.seg;
        const size_t b = nseg * (size_t)pl.CH * pl.blocks * pl.block * real_bytes(pl.precision);
        if ((st = ensure(ctx, ctx->ckpt, b)) != LV_OK) return st;
    }
    return LV_OK;
}

hipEvent_t take_event(lv_ctx *ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence (cache writeback and invalidate) when recorded
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// Launch `fn` on the context's stream; when profiling, with a pair of events
// attached to its dispatches (no extra packets between kernels).
template <typename Fn>
hipError_t timed(lv_ctx *ctx, int profile, int kind, Fn fn) {
    if (!(profile & (1 << kind))) return fn(lvk::Ev{});
    hipEvent_t a = take_event(ctx), b = take_event(ctx);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = fn(lvk::Ev{a, b});
    if (e != hipSuccess) return e;
    ctx->pending.push_back({a, b, kind});
    return hipSuccess;
}

lv_status collect_times(lv_ctx *ctx) {
    if (ctx->pending.empty()) return LV_OK;
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream()));
    for (auto &t : ctx->pending) {
        float ms = 0.f;
        HIPCHECK(ctx, hipEventElapsedTime(&ms, t.a, t.b));
        ctx->k_ms[t.kind] += ms;
        ctx->k_count[t.kind] += 1;
        ctx->event_pool.push_back(t.a);
        ctx->event_pool.push_back(t.b);
    }
    ctx->pending.clear();
    return LV_OK;
}

// Launch the whole path for one surface (no allocation, no sync): capturable.
hipError_t enqueue_surface(lv_ctx *ctx, const Space &w, const Plan &pl, const Tables &t,
                           const double *sigma_dev, bool adjoint, double *price, double *stderr_,
                           double *grad, double *delta, bool capturing) {
    hipStream_t st = ctx->stream();
    lvk::Args a = make_args(w, pl, t, sigma_dev);
    a.part = (double *)w.part;
    a.states = w.states;
    a.ckpt = w.ckpt;
    const int prof = capturing ? 0 : pl.profile;
    hipError_t e = timed(ctx, prof, LV_K_TABLE, [&](lvk::Ev ev) { return lvk::launch_table(a, pl.precision, st, ev); });
    if (e != hipSuccess) return e;
    lvk::Args af = a;                 // the forward kernel's own tiling
    af.n_tiles = pl.f_n_tiles;
    if (!adjoint) {
        e = timed(ctx, prof, LV_K_FWD, [&](lvk::Ev ev) { return lvk::launch_fwd(af, pl.precision, false, pl.fblocks, pl.fblock, st, ev); });
        if (e != hipSuccess) return e;
        return timed(ctx, prof, LV_K_MERGE, [&](lvk::Ev ev) {
            return lvk::launch_merge(a.part, pl.fblocks, pl.blocks, pl.Q, pl.n_opt, pl.G, t.opt_orig, pl.P,
                                     pl.spot, price, stderr_, nullptr, nullptr, st, ev);
        });
    }
    int b_pay = pl.blocks;
    if (pl.adjoint == LV_ADJ_STORED) {
        e = timed(ctx, prof, LV_K_FWD, [&](lvk::Ev ev) { return lvk::launch_fwd(af, pl.precision, true, pl.fblocks, pl.fblock, st, ev); });
        if (e != hipSuccess) return e;
        e = timed(ctx, prof, LV_K_REV, [&](lvk::Ev ev) { return lvk::launch_rev(a, pl.precision, pl.blocks, pl.block, st, ev); });
        if (e != hipSuccess) return e;
        b_pay = pl.fblocks;
    } else {
        e = timed(ctx, prof, LV_K_FUSED, [&](lvk::Ev ev) { return lvk::launch_fused_ckpt(a, pl.precision, pl.blocks, pl.block, st, ev); });
        if (e != hipSuccess) return e;
    }
    e = timed(ctx, prof, LV_K_MERGE, [&](lvk::Ev ev) {
        return lvk::launch_merge(a.part, b_pay, pl.blocks, pl.Q, pl.n_opt, pl.G, t.opt_orig, pl.P, pl.spot,
                                 price, stderr_, grad, delta, st, ev);
    });
    return e;
}

void record_info(lv_ctx *ctx, const Plan &pl, bool adjoint, bool replayed, const void *part) {
    ctx->last_part = part;
    ctx->last_Q = pl.Q;
    ctx->last_G = pl.G;
    ctx->last_nopt = pl.n_opt;
    ctx->info.n_blocks = pl.blocks;
    ctx->info.block = pl.block;
    ctx->info.tile_paths = pl.block;
    ctx->info.waves_per_block = pl.block / 64;
    ctx->info.fixed_point_bits = host_fixed_point_bits(pl);
    ctx->info.adjoint = adjoint ? pl.adjoint : LV_ADJ_NONE;
    ctx->info.precision = pl.precision;
    ctx->info.graph_replayed = replayed ? 1 : 0;
    ctx->info.copies = pl.K;
    ctx->info.window = pl.W;
    ctx->info.blocks_per_cu = pl.bpc;
    ctx->info.autotuned = ctx->last_autotuned ? 1 : 0;
    ctx->info.fwd_block = pl.fblock;
    ctx->info.fwd_blocks_per_cu = pl.fbpc;
    ctx->info.fwd_blocks = pl.fblocks;
    ctx->info.overflow_terms = 0;
    ctx->info.hist_window = pl.WH;
}

std::string graph_key(const Plan &pl, const void *ptrs[], int n_ptrs, int n_surf, bool adjoint) {
    std::string k;
    char buf[128];
    snprintf(buf, sizeof buf, "%d|%d|%d|%d|%lld|%llu|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%.17g|%.17g|%d|", pl.I,
             pl.J, pl.N, pl.axis, pl.P, (unsigned long long)pl.seed, pl.precision, pl.adjoint, pl.seg, pl.block,
             pl.blocks, pl.W, pl.WH, pl.K, pl.CH, (pl.dense * 2 + pl.scheme) * 2 + pl.bf16, pl.fblock, pl.fblocks, pl.spot, pl.dt,
             n_surf);
    k += buf;
    snprintf(buf, sizeof buf, "r%.17g|", pl.rate);
    k += buf;
    k += adjoint ? "A|" : "F|";
    for (int i = 0; i < n_ptrs; ++i) {
        snprintf(buf, sizeof buf, "%p|", ptrs[i]);
        k += buf;
    }
    return k;
}

std::string tune_key(const Plan &pl, bool adjoint) {
    char buf[256];
    snprintf(buf, sizeof buf, "%d|%d|%d|%d|%lld|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d", pl.I, pl.J, pl.N,
             pl.axis, pl.P, pl.precision, adjoint ? pl.adjoint : LV_ADJ_NONE, pl.seg, pl.n_opt,
             pl.n_taps, pl.user.block, pl.user.K, pl.user.W, pl.user.bpc, pl.user.fblock,
             pl.user.fbpc, (int)pl.profile, (pl.dense * 2 + pl.scheme) * 2 + (pl.rate != 0.0));
    return buf;
}

lv_status run_dev(lv_ctx *ctx, Plan &pl, int n_surf, const double *sigmas_dev,
                  bool adjoint, bool use_graph, double *prices, double *stderrs, double *grads,
                  double *deltas);

// Time one launch shape on the first surface: one untimed run (allocations,
// first touch), then the fastest of three timed pairs of runs (a pair that a clock
// change or another process slowed does not count).
lv_status time_shape(lv_ctx *ctx, const Plan &pl, const Shape &c, const double *sigmas_dev, bool adjoint,
                     double *prices, double *stderrs, double *grads, double *deltas, hipEvent_t e0,
                     hipEvent_t e1, float *ms) {
    Plan q = pl;
    q.autotune = false;
    q.profile = 0;
    lv_status st = apply_shape(ctx, q, c, ctx->n_cu, ctx->max_lds, false, false);
    if (st != LV_OK) return st;
    if ((st = run_dev(ctx, q, 1, sigmas_dev, adjoint, false, prices, stderrs, grads, deltas)) != LV_OK) return st;
    *ms = 1e30f;
    for (int k = 0; k < 3; ++k) {
        hipError_t e = hipEventRecord(e0, ctx->stream());
        for (int r = 0; r < 2 && st == LV_OK; ++r)
            st = run_dev(ctx, q, 1, sigmas_dev, adjoint, false, prices, stderrs, grads, deltas);
        if (st != LV_OK) return st;
        float t = 0.f;
        if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream());
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) return fail(ctx, LV_ERR_HIP, "autotune timing: %s", hipGetErrorString(e));
        *ms = std::min(*ms, t);
    }
    return LV_OK;
}

bool user_allows(const Plan &pl, const Shape &c) {
    return !((pl.user.block && c.block != pl.user.block) || (pl.user.K && c.K != pl.user.K) ||
             (pl.user.W && c.W != pl.user.W) || (pl.user.bpc && c.bpc != pl.user.bpc) ||
             (pl.user.fblock && c.fblock != pl.user.fblock) || (pl.user.fbpc && c.fbpc != pl.user.fbpc));
}

// Saved tunings: one line per tuned request, "lvmc-tune 1 <arch> <CUs> <key> <block> <K>
// <W> <bpc> <fblock> <fbpc>" (the key has no blanks).
constexpr const char *kTuneTag = "lvmc-tune";
constexpr int kTuneVersion = 1;

void write_tuning_line(FILE *f, const lv_ctx *ctx, const std::string &key, const Shape &c) {
    fprintf(f, "%s %d %s %d %s %d %d %d %d %d %d\n", kTuneTag, kTuneVersion, ctx->arch.c_str(), ctx->n_cu,
            key.c_str(), c.block, c.K, c.W, c.bpc, c.fblock, c.fbpc);
}

// The tuning file named by LVMC_TUNING_FILE after the autotuner added a shape: the
// lines already there for other devices, or for request shapes this context has not
// tuned (another process may have added them since this one read the file), are kept
// as they are; this context's shapes follow.  Written to a temporary file in the same
// folder and renamed over the old one, so readers see the old file or the new one.
lv_status save_tunings_merged(lv_ctx *ctx, const char *path) {
    std::vector<std::string> keep;
    if (FILE *f = fopen(path, "r")) {
        char *line = nullptr;   // whole lines of any length (getline grows the buffer)
        size_t cap = 0;
        while (getline(&line, &cap, f) > 0) {
            char tag[32], arch[64], key[512];
            int ver = 0, cus = 0;
            const bool ours = sscanf(line, "%31s %d %63s %d %511s", tag, &ver, arch, &cus, key) == 5 &&
                              strcmp(tag, kTuneTag) == 0 && ver == kTuneVersion && ctx->arch == arch &&
                              cus == ctx->n_cu && ctx->tuned.count(key);
            if (ours || line[0] == '\n') continue;
            keep.push_back(line);
            if (keep.back().back() != '\n') keep.back() += '\n';   // a last line without one
        }
        free(line);
        fclose(f);
    }
    const std::string tmp = std::string(path) + ".tmp." + std::to_string((long long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return fail(ctx, LV_ERR_ARG, "cannot write the tuning file %s (LVMC_TUNING_FILE)", tmp.c_str());
    for (const std::string &l : keep) fputs(l.c_str(), f);
    for (const auto &kv : ctx->tuned) write_tuning_line(f, ctx, kv.first, kv.second);
    const bool ok = fclose(f) == 0 && rename(tmp.c_str(), path) == 0;
    if (!ok) {
        (void)remove(tmp.c_str());
        return fail(ctx, LV_ERR_ARG, "cannot write the tuning file %s (LVMC_TUNING_FILE)", path);
    }
    return LV_OK;
}

// Autotuner: the separate forward kernel's shape first (stored and price-only
// paths), then the adjoint (or fused) kernel's shape with that forward; each
// candidate is timed on the first surface in two sweeps over the candidates (the
// first ones of a cold GPU run before its clocks have risen) and the fastest kept
// per context and request shape.
lv_status autotune(lv_ctx *ctx, Plan &pl, const double *sigmas_dev, bool adjoint, double *prices,
                   double *stderrs, double *grads, double *deltas) {
    const std::string key = tune_key(pl, adjoint);
    auto it = ctx->tuned.find(key);
    if (it == ctx->tuned.end()) {
        Shape best{pl.block, pl.K, pl.W, pl.bpc, pl.fblock, pl.fbpc};
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIPCHECK(ctx, hipEventCreate(&e0));
        HIPCHECK(ctx, hipEventCreate(&e1));
        lv_status st = LV_OK;
        for (int phase = 0; phase < 2 && st == LV_OK; ++phase) {
            std::vector<Shape> cands;
            if (phase == 0 && (!adjoint || pl.adjoint == LV_ADJ_STORED))
                cands = forward_candidates(pl, best, ctx->n_cu, ctx->max_lds);
            if (phase == 1 && adjoint) cands = adjoint_candidates(pl, best, ctx->n_cu, ctx->max_lds);
            std::vector<float> t(cands.size(), 1e30f);
            for (int sweep = 0; sweep < 2 && st == LV_OK; ++sweep)
                for (size_t i = 0; i < cands.size(); ++i) {
                    if (!user_allows(pl, cands[i])) continue;
                    float ms = 0.f;
                    if ((st = time_shape(ctx, pl, cands[i], sigmas_dev, adjoint, prices, stderrs, grads, deltas,
                                         e0, e1, &ms)) != LV_OK)
                        break;
                    t[i] = std::min(t[i], ms);
                }
            float best_ms = 1e30f;
            for (size_t i = 0; i < cands.size() && st == LV_OK; ++i)
                if (t[i] < best_ms) {
                    best_ms = t[i];
                    best = cands[i];
                }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != LV_OK) return st;
        it = ctx->tuned.emplace(key, best).first;
        if (!ctx->tune_path.empty() && (st = save_tunings_merged(ctx, ctx->tune_path.c_str())) != LV_OK) return st;
    }
    return apply_shape(ctx, pl, it->second, ctx->n_cu, ctx->max_lds, false, false);
}

lv_status run_dev(lv_ctx *ctx, Plan &pl, int n_surf, const double *sigmas_dev,
                  bool adjoint, bool use_graph, double *prices, double *stderrs, double *grads,
                  double *deltas) {
    lv_status s;
    ctx->last_autotuned = false;
    if (pl.autotune) {
        if ((s = autotune(ctx, pl, sigmas_dev, adjoint, prices, stderrs, grads, deltas)) != LV_OK) return s;
        pl.autotune = false;
        ctx->last_autotuned = true;
    }
    Tables t;
    if ((s = upload_tables(ctx, pl, t)) != LV_OK) return s;
    if ((s = ensure_workspace(ctx, pl, adjoint)) != LV_OK) return s;
    auto enqueue_all = [&]() -> hipError_t {
        for (int k = 0; k < n_surf; ++k) {
            hipError_t e = enqueue_surface(ctx, ctx_space(ctx), pl, t, sigmas_dev + (size_t)k * pl.G, adjoint,
                                           prices + (size_t)k * pl.n_opt, stderrs + (size_t)k * pl.n_opt,
                                           grads ? grads + (size_t)k * pl.G : nullptr,
                                           deltas ? deltas + k : nullptr, use_graph);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    if (!use_graph) {
        hipError_t e = enqueue_all();
        if (e != hipSuccess) return fail(ctx, LV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
        record_info(ctx, pl, adjoint, false, ctx->part.p);
        return LV_OK;
    }
    const void *ptrs[] = {sigmas_dev, prices, stderrs, grads, deltas, ctx->planbuf.p, ctx->part.p,
                          ctx->states.p, ctx->ckpt.p, ctx->gtab.p};
    std::string key = graph_key(pl, ptrs, 10, n_surf, adjoint) + std::string(ctx->plan_bytes.begin(), ctx->plan_bytes.end());
    bool replay = ctx->graph_exec && key == ctx->graph_key;
    if (!replay) {
        if (ctx->graph_exec) {
            (void)hipGraphExecDestroy(ctx->graph_exec);
            ctx->graph_exec = nullptr;
        }
        if (ctx->graph) {
            (void)hipGraphDestroy(ctx->graph);
            ctx->graph = nullptr;
        }
        ctx->graph_key.clear();
        HIPCHECK(ctx, hipStreamBeginCapture(ctx->stream(), hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_all();
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(ctx->stream(), &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(ctx, LV_ERR_HIP, "graph capture failed: %s / %s", hipGetErrorString(e), hipGetErrorString(e2));
        }
        ctx->graph = g;
        HIPCHECK(ctx, hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0));
        ctx->graph_key = key;
    }
    HIPCHECK(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream()));
    record_info(ctx, pl, adjoint, replay, ctx->part.p);
    return LV_OK;
}

int device_cus(int device, size_t *max_lds, std::string *arch = nullptr) {
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, device) != hipSuccess) return 256;
    if (max_lds) *max_lds = std::min<size_t>(pr.sharedMemPerBlock, 160 * 1024);
    if (arch) {
        // the name up to the first ':' (feature flags such as sramecc+ follow it)
        std::string a(pr.gcnArchName);
        *arch = a.substr(0, a.find(':'));
    }
    return pr.multiProcessorCount;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

lv_status lv_create(lv_ctx **out, int device, void *hip_stream) {
    if (!out) return fail(nullptr, LV_ERR_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(nullptr, LV_ERR_HIP, "no HIP device available (%s)", hipGetErrorString(e));
    if (device < 0 || device >= n) return fail(nullptr, LV_ERR_ARG, "device %d out of range (%d devices)", device, n);
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, LV_ERR_HIP, "hipSetDevice: %s", hipGetErrorString(e));
    lv_ctx *c = new lv_ctx();
    c->device = device;
    c->user_stream = (hipStream_t)hip_stream;
    c->n_cu = device_cus(device, &c->max_lds, &c->arch);
    e = hipStreamCreate(&c->own_stream);
    if (e != hipSuccess) {
        delete c;
        return fail(nullptr, LV_ERR_HIP, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    // the allocation-free entry point's workspace on this device (looked up once per device)
    e = lvk::scratch_address(device, &c->scratch);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(c->own_stream);
        delete c;
        return fail(nullptr, LV_ERR_HIP, "workspace address on device %d: %s", device, hipGetErrorString(e));
    }
    // shapes tuned by earlier processes, if LVMC_TUNING_FILE names a file that exists
    const char *tp = getenv("LVMC_TUNING_FILE");
    if (tp && *tp) {
        c->tune_path = tp;
        if (FILE *f = fopen(tp, "r")) {
            fclose(f);
            if (lv_tuning_load(c, tp, nullptr) != LV_OK) {
                const std::string msg = c->err;
                lv_destroy(c);
                return fail(nullptr, LV_ERR_ARG, "LVMC_TUNING_FILE: %s", msg.c_str());
            }
        }
    }
    *out = c;
    return LV_OK;
}

void lv_destroy(lv_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream());
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    for (auto &t : ctx->pending) {
        ctx->event_pool.push_back(t.a);
        ctx->event_pool.push_back(t.b);
    }
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    Buf *bufs[] = {&ctx->planbuf, &ctx->part, &ctx->states, &ctx->ckpt,
                   &ctx->sig_stage, &ctx->out_stage, &ctx->gtab, &ctx->bump};
    for (Buf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    delete ctx;
}

lv_status lv_set_stream(lv_ctx *ctx, void *hip_stream) {
    if (!ctx) return fail(nullptr, LV_ERR_ARG, "ctx is NULL");
    const hipStream_t prev = ctx->stream();
    ctx->user_stream = (hipStream_t)hip_stream;
    if (ctx->stream() != prev) {
        // work queued on the previous stream may still use the context's buffers
        HIPCHECK(ctx, hipSetDevice(ctx->device));
        HIPCHECK(ctx, hipStreamSynchronize(prev));
    }
    return LV_OK;
}

const char *lv_last_error(const lv_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_last_error.c_str();
}

lv_status lv_check(const lv_grid *grid, const double *sigma, double spot, const lv_book *book,
                   int64_t n_paths, int32_t n_steps, const lv_opts *opts) {
    Plan pl;
    return plan_request(nullptr, grid, 1, sigma, spot, book, n_paths, n_steps, 0, opts, 256, 160 * 1024, pl);
}

lv_status lv_price_and_grad_dev(lv_ctx *ctx, const lv_grid *grid, int32_t n_surf,
                                const double *sigmas_dev, double spot, const lv_book *book,
                                int64_t n_paths, int32_t n_steps, uint64_t seed,
                                const lv_opts *opts, double *prices_dev, double *std_errs_dev,
                                double *grads_dev, double *deltas_dev) {
    if (!ctx) return fail(nullptr, LV_ERR_ARG, "ctx is NULL");
    if (!sigmas_dev || !prices_dev || !std_errs_dev) return fail(ctx, LV_ERR_ARG, "sigmas, prices and std_errs are required");
    Plan pl;
    lv_status s = plan_request(ctx, grid, n_surf, nullptr, spot, book, n_paths, n_steps, seed, opts,
                               ctx->n_cu, ctx->max_lds, pl);
    if (s != LV_OK) return s;
    const bool adjoint = grads_dev || deltas_dev;
    if (adjoint && pl.adjoint == LV_ADJ_NONE)
        return fail(ctx, LV_ERR_ARG, "gradient or delta requested with adjoint mode NONE");
    HIPCHECK(ctx, hipSetDevice(ctx->device));
    return run_dev(ctx, pl, n_surf, sigmas_dev, adjoint, opts && opts->use_graph, prices_dev,
                   std_errs_dev, grads_dev, deltas_dev);
}

lv_status lv_price_and_grad_noalloc(lv_ctx *ctx, const lv_grid *grid, int32_t n_surf,
                                    const double *sigmas_dev, double spot, const lv_book *book,
                                    int64_t n_paths, int32_t n_steps, uint64_t seed,
                                    const lv_opts *opts, double *prices_dev, double *std_errs_dev,
                                    double *grads_dev, double *deltas_dev) {
    if (!ctx) return fail(nullptr, LV_ERR_ARG, "ctx is NULL");
    if (!sigmas_dev || !prices_dev || !std_errs_dev) return fail(ctx, LV_ERR_ARG, "sigmas, prices and std_errs are required");
    if (opts && (opts->use_graph || opts->autotune || opts->profile))
        return fail(ctx, LV_ERR_ARG, "the allocation-free entry point takes no use_graph, autotune or profile");
    Plan pl;
    lv_status s = plan_request(ctx, grid, n_surf, nullptr, spot, book, n_paths, n_steps, seed, opts,
                               ctx->n_cu, ctx->max_lds, pl);
    if (s != LV_OK) return s;
    const bool adjoint = grads_dev || deltas_dev;
    if (adjoint && pl.adjoint == LV_ADJ_NONE)
        return fail(ctx, LV_ERR_ARG, "gradient or delta requested with adjoint mode NONE");
    // a launch shape this context has tuned for the request is taken as it is
    auto it = ctx->tuned.find(tune_key(pl, adjoint));
    if (it != ctx->tuned.end() && (s = apply_shape(ctx, pl, it->second, ctx->n_cu, ctx->max_lds, false, false)) != LV_OK)
        return s;
    if (!ctx->scratch) return fail(ctx, LV_ERR_HIP, "no workspace on device %d", ctx->device);
    // carve the workspace: tables, vol table, block records, then states or checkpoints
    TableOffsets to;
    std::vector<char> tab = pack_tables(pl, to);
    size_t used = 0;
    auto take = [&](size_t bytes) {
        const size_t o = used;
        used = (used + bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t rb = real_bytes(pl.precision);
    const size_t o_tab = take(tab.size());
    const size_t o_gtab = take((size_t)pl.N * pl.I * 2 * rb);
    const size_t o_part = take((size_t)std::max(pl.blocks, pl.fblocks) * pl.Q * 8);
    size_t o_states = 0, o_ckpt = 0;
    if (adjoint && pl.adjoint == LV_ADJ_STORED) o_states = take((size_t)pl.N * (size_t)pl.P * rb);
    if (adjoint && pl.adjoint == LV_ADJ_CHECKPOINT)
        o_ckpt = take((size_t)((pl.N + pl.seg - 1) / pl.seg) * pl.CH * pl.blocks * pl.block * rb);
    if (used > lvk::kScratchBytes)
        return fail(ctx, LV_ERR_UNSUPPORTED,
                    "request needs %zu bytes of workspace; the allocation-free entry point has %zu "
                    "(fewer paths, the checkpointed adjoint or the allocating entry point fit it)",
                    used, lvk::kScratchBytes);
    HIPCHECK(ctx, hipSetDevice(ctx->device));
    char *base = (char *)ctx->scratch;
    hipStream_t st = ctx->stream();
    // the host copy stays with the context until the next such call
    ctx->scratch_tables.swap(tab);
    HIPCHECK(ctx, hipMemcpyAsync(base + o_tab, ctx->scratch_tables.data(), ctx->scratch_tables.size(),
                                 hipMemcpyHostToDevice, st));
    const Tables t = tables_at(base + o_tab, to);
    Space w;
    w.gtab = base + o_gtab;
    w.part = base + o_part;
    w.states = o_states ? base + o_states : nullptr;
    w.ckpt = o_ckpt ? base + o_ckpt : nullptr;
    for (int k = 0; k < n_surf; ++k) {
        hipError_t e = enqueue_surface(ctx, w, pl, t, sigmas_dev + (size_t)k * pl.G, adjoint,
                                       prices_dev + (size_t)k * pl.n_opt, std_errs_dev + (size_t)k * pl.n_opt,
                                       grads_dev ? grads_dev + (size_t)k * pl.G : nullptr,
                                       deltas_dev ? deltas_dev + k : nullptr, true);
        if (e != hipSuccess) return fail(ctx, LV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    }
    ctx->last_autotuned = false;
    record_info(ctx, pl, adjoint, false, w.part);
    return LV_OK;
}

lv_status lv_bump_grad_dev(lv_ctx *ctx, const lv_grid *grid, const double *sigma_dev, double spot,
                           const lv_book *book, int64_t n_paths, int32_t n_steps, uint64_t seed,
                           const lv_opts *opts, double eps, int32_t batch, double *grad_dev) {
    if (!ctx) return fail(nullptr, LV_ERR_ARG, "ctx is NULL");
    if (!sigma_dev || !grad_dev) return fail(ctx, LV_ERR_ARG, "sigma and grad are required");
    if (!(std::isfinite(eps) && eps > 0.0)) return fail(ctx, LV_ERR_ARG, "eps must be finite and > 0");
    if (batch < 0) return fail(ctx, LV_ERR_ARG, "batch must be >= 0");
    lv_opts o = opts ? *opts : lv_opts{};
    o.adjoint = LV_ADJ_NONE;   // forward pricing only
    Plan pl;
    lv_status s = plan_request(ctx, grid, 1, nullptr, spot, book, n_paths, n_steps, seed, &o, ctx->n_cu,
                               ctx->max_lds, pl);
    if (s != LV_OK) return s;
    const int G = pl.G, nb = std::min(G, batch > 0 ? (int)batch : 256);   // nodes per batch
    HIPCHECK(ctx, hipSetDevice(ctx->device));
    const size_t n_sig = (size_t)2 * nb * G, n_pr = (size_t)2 * nb * pl.n_opt;
    if ((s = ensure(ctx, ctx->bump, (n_sig + 2 * n_pr + pl.n_opt) * 8)) != LV_OK) return s;
    double *sig_b = (double *)ctx->bump.p, *pr = sig_b + n_sig, *se = pr + n_pr, *w = se + n_pr;
    hipStream_t st = ctx->stream();
    HIPCHECK(ctx, hipMemcpyAsync(w, pl.weight.data(), pl.n_opt * 8, hipMemcpyHostToDevice, st));
    for (int m0 = 0; m0 < G; m0 += nb) {
        const int mc = std::min(nb, G - m0);
        hipError_t e = lvk::launch_bump(sigma_dev, G, m0, mc, eps, sig_b, st);
        if (e != hipSuccess) return fail(ctx, LV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
        if ((s = run_dev(ctx, pl, 2 * mc, sig_b, false, o.use_graph != 0, pr, se, nullptr, nullptr)) != LV_OK)
            return s;
        e = lvk::launch_fd(pr, pl.n_opt, w, m0, mc, eps, grad_dev, st);
        if (e != hipSuccess) return fail(ctx, LV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    }
    return LV_OK;
}

lv_status lv_price_and_grad_batch(lv_ctx *ctx, const lv_grid *grid, int32_t n_surf,
                                  const double *sigmas, double spot, const lv_book *book,
                                  int64_t n_paths, int32_t n_steps, uint64_t seed,
                                  const lv_opts *opts, double *prices, double *std_errs,
                                  double *grads, double *deltas) {
    if (!ctx) return fail(nullptr, LV_ERR_ARG, "ctx is NULL");
    if (!sigmas || !prices || !std_errs) return fail(ctx, LV_ERR_ARG, "sigmas, prices and std_errs are required");
    Plan pl;
    lv_status s = plan_request(ctx, grid, n_surf, sigmas, spot, book, n_paths, n_steps, seed, opts,
                               ctx->n_cu, ctx->max_lds, pl);
    if (s != LV_OK) return s;
    const bool adjoint = grads || deltas;
    if (adjoint && pl.adjoint == LV_ADJ_NONE)
        return fail(ctx, LV_ERR_ARG, "gradient or delta requested with adjoint mode NONE");
    HIPCHECK(ctx, hipSetDevice(ctx->device));
    const size_t nsig = (size_t)n_surf * pl.G;
    const size_t per = (size_t)2 * pl.n_opt + 1 + pl.G;   // prices, stderrs, delta, grad
    if ((s = ensure(ctx, ctx->sig_stage, nsig * 8)) != LV_OK) return s;
    if ((s = ensure(ctx, ctx->out_stage, (size_t)n_surf * per * 8)) != LV_OK) return s;
    hipStream_t st = ctx->stream();
    HIPCHECK(ctx, hipMemcpyAsync(ctx->sig_stage.p, sigmas, nsig * 8, hipMemcpyHostToDevice, st));
    double *o = (double *)ctx->out_stage.p;
    double *d_price = o, *d_se = o + (size_t)n_surf * pl.n_opt, *d_delta = o + (size_t)2 * n_surf * pl.n_opt;
    double *d_grad = d_delta + n_surf;
    s = run_dev(ctx, pl, n_surf, (const double *)ctx->sig_stage.p, adjoint, opts && opts->use_graph,
                d_price, d_se, grads ? d_grad : nullptr, adjoint ? d_delta : nullptr);
    if (s != LV_OK) return s;
    std::vector<double> h((size_t)n_surf * per);
    HIPCHECK(ctx, hipMemcpyAsync(h.data(), o, h.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHECK(ctx, hipStreamSynchronize(st));
    std::memcpy(prices, h.data(), (size_t)n_surf * pl.n_opt * 8);
    std::memcpy(std_errs, h.data() + (size_t)n_surf * pl.n_opt, (size_t)n_surf * pl.n_opt * 8);
    if (deltas) std::memcpy(deltas, h.data() + (size_t)2 * n_surf * pl.n_opt, (size_t)n_surf * 8);
    if (grads) std::memcpy(grads, h.data() + (size_t)2 * n_surf * pl.n_opt + n_surf, (size_t)n_surf * pl.G * 8);
    return LV_OK;
}

lv_status lv_price_and_grad(lv_ctx *ctx, const lv_grid *grid, const double *sigma, double spot,
                            const lv_book *book, int64_t n_paths, int32_t n_steps, uint64_t seed,
                            const lv_opts *opts, double *price, double *std_err, double *grad,
                            double *delta) {
    return lv_price_and_grad_batch(ctx, grid, 1, sigma, spot, book, n_paths, n_steps, seed, opts,
                                   price, std_err, grad, delta);
}

lv_status lv_states_bytes(int32_t precision, int64_t n_paths, int32_t n_steps, size_t *bytes) {
    if (!bytes) return fail(nullptr, LV_ERR_ARG, "bytes is NULL");
    if (precision != 32 && precision != 64) return fail(nullptr, LV_ERR_ARG, "precision must be 32 or 64");
    if (n_paths < 2 || n_steps < 1) return fail(nullptr, LV_ERR_ARG, "n_paths >= 2 and n_steps >= 1 required");
    *bytes = (size_t)n_paths * (size_t)n_steps * real_bytes(precision);
    return LV_OK;
}

lv_status lv_forward_dev(lv_ctx *ctx, const lv_grid *grid, const double *sigma_dev, double spot,
                         const lv_book *book, int64_t n_paths, int32_t n_steps, uint64_t seed,
                         int32_t precision, double rate, void *states_dev, double *price_dev,
                         double *std_err_dev) {
    if (!ctx) return fail(nullptr, LV_ERR_ARG, "ctx is NULL");
    if (!sigma_dev || !states_dev || !price_dev || !std_err_dev)
        return fail(ctx, LV_ERR_ARG, "sigma, states, price and std_err are required");
    lv_opts o{};
    o.precision = precision;
    o.adjoint = LV_ADJ_STORED;
    o.rate = rate;
    Plan pl;
    lv_status s = plan_request(ctx, grid, 1, nullptr, spot, book, n_paths, n_steps, seed, &o, ctx->n_cu,
                               ctx->max_lds, pl);
    if (s != LV_OK) return s;
    HIPCHECK(ctx, hipSetDevice(ctx->device));
    Tables t;
    if ((s = upload_tables(ctx, pl, t)) != LV_OK) return s;
    if ((s = ensure_workspace(ctx, pl, false)) != LV_OK) return s;
    hipStream_t st = ctx->stream();
    lvk::Args a = make_args(ctx_space(ctx), pl, t, sigma_dev);
    a.part = (double *)ctx->part.p;
    a.states = states_dev;
    a.n_tiles = pl.f_n_tiles;
    hipError_t e = lvk::launch_table(a, pl.precision, st);
    if (e == hipSuccess) e = lvk::launch_fwd(a, pl.precision, true, pl.fblocks, pl.fblock, st);
    if (e == hipSuccess)
        e = lvk::launch_merge(a.part, pl.fblocks, pl.blocks, pl.Q, pl.n_opt, pl.G, t.opt_orig, pl.P, pl.spot,
                              price_dev, std_err_dev, nullptr, nullptr, st);
    if (e != hipSuccess) return fail(ctx, LV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    record_info(ctx, pl, false, false, ctx->part.p);
    return LV_OK;
}

lv_status lv_backward_dev(lv_ctx *ctx, const lv_grid *grid, const double *sigma_dev, double spot,
                          const lv_book *book, int64_t n_paths, int32_t n_steps, uint64_t seed,
                          int32_t precision, double rate, const void *states_dev,
                          const double *cotangent_dev, double *grad_dev, double *delta_dev) {
    if (!ctx) return fail(nullptr, LV_ERR_ARG, "ctx is NULL");
    if (!sigma_dev || !states_dev || !cotangent_dev || !grad_dev)
        return fail(ctx, LV_ERR_ARG, "sigma, states, cotangent and grad are required");
    lv_opts o{};
    o.precision = precision;
    o.adjoint = LV_ADJ_STORED;
    o.rate = rate;
    Plan pl;
    lv_status s = plan_request(ctx, grid, 1, nullptr, spot, book, n_paths, n_steps, seed, &o, ctx->n_cu,
                               ctx->max_lds, pl);
    if (s != LV_OK) return s;
    HIPCHECK(ctx, hipSetDevice(ctx->device));
    Tables t;
    if ((s = upload_tables(ctx, pl, t)) != LV_OK) return s;
    if ((s = ensure_workspace(ctx, pl, false)) != LV_OK) return s;
    if ((s = ensure(ctx, ctx->out_stage, (size_t)2 * pl.n_opt * 8)) != LV_OK) return s;
    hipStream_t st = ctx->stream();
    lvk::Args a = make_args(ctx_space(ctx), pl, t, sigma_dev);
    a.part = (double *)ctx->part.p;
    a.states = const_cast<void *>(states_dev);
    a.cot = cotangent_dev;
    // the reverse writes no payoff sums: the merge's price outputs go to scratch
    hipError_t e = lvk::launch_table(a, pl.precision, st);
    if (e == hipSuccess) e = lvk::launch_rev(a, pl.precision, pl.blocks, pl.block, st);
    double *scratch = (double *)ctx->out_stage.p;
    if (e == hipSuccess)
        e = lvk::launch_merge(a.part, pl.blocks, pl.blocks, pl.Q, pl.n_opt, pl.G, t.opt_orig, pl.P, pl.spot,
                              scratch, scratch + pl.n_opt, grad_dev, delta_dev, st);
    if (e != hipSuccess) return fail(ctx, LV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    record_info(ctx, pl, true, false, ctx->part.p);
    ctx->info.fixed_point_bits = -1000;   // depends on the device cotangent
    return LV_OK;
}

lv_status lv_per_option_grads_dev(lv_ctx *ctx, const lv_grid *grid, const double *sigma_dev, double spot,
                                  const lv_book *book, int64_t n_paths, int32_t n_steps, uint64_t seed,
                                  int32_t precision, double rate, const void *states_dev, double *grads_dev,
                                  double *deltas_dev) {
    if (!ctx) return fail(nullptr, LV_ERR_ARG, "ctx is NULL");
    if (!sigma_dev || !states_dev || !grads_dev) return fail(ctx, LV_ERR_ARG, "sigma, states and grads are required");
    lv_opts o{};
    o.precision = precision;
    o.adjoint = LV_ADJ_STORED;
    o.rate = rate;
    Plan pl;
    lv_status s = plan_request(ctx, grid, 1, nullptr, spot, book, n_paths, n_steps, seed, &o, ctx->n_cu,
                               ctx->max_lds, pl);
    if (s != LV_OK) return s;
    // options per sweep: the most (8, 4, 2 or 1) whose grids and histograms fit a block's LDS
    const int block = pl.block;
    int KO = 8;
    while (KO > 1 && lvk::lds_bytes_per_option(pl.precision, pl.I, pl.J, block, KO) > ctx->max_lds) KO /= 2;
    if (lvk::lds_bytes_per_option(pl.precision, pl.I, pl.J, block, KO) > ctx->max_lds)
        return fail(ctx, LV_ERR_UNSUPPORTED, "a %d x %d grid per option does not fit a block's LDS", pl.I, pl.J);
    const int G = pl.G, Q = KO * (1 + G);
    const long long n_tiles = (pl.P + block - 1) / block;
    const int blocks = (int)std::min<long long>(n_tiles, ctx->n_cu);
    HIPCHECK(ctx, hipSetDevice(ctx->device));
    Tables t;
    if ((s = upload_tables(ctx, pl, t)) != LV_OK) return s;
    if ((s = ensure_table(ctx, pl)) != LV_OK) return s;
    if ((s = ensure(ctx, ctx->part, (size_t)blocks * Q * 8)) != LV_OK) return s;
    hipStream_t st = ctx->stream();
    lvk::Args a = make_args(ctx_space(ctx), pl, t, sigma_dev);
    a.part = (double *)ctx->part.p;
    a.states = const_cast<void *>(states_dev);
    a.Q = Q;
    a.K = 1;
    a.n_tiles = (int)n_tiles;
    // maturity step of every option (tap order): a group's sweep starts at its last one
    std::vector<int> opt_step(pl.n_opt);
    for (int t = 0; t < pl.n_taps; ++t)
        for (int q = 0; q < pl.tap_count[t]; ++q) opt_step[pl.tap_first[t] + q] = pl.tap_step[t];
    hipError_t e = lvk::launch_table(a, pl.precision, st);
    for (int o0 = 0; o0 < pl.n_opt && e == hipSuccess; o0 += KO) {
        const int n_end = opt_step[std::min(o0 + KO, pl.n_opt) - 1];
        e = lvk::launch_rev_per_option(a, pl.precision, o0, KO, n_end, blocks, block, st);
        for (int q = 0; q < KO && o0 + q < pl.n_opt && e == hipSuccess; ++q) {
            const int orig = pl.opt_orig[o0 + q];
            e = lvk::launch_merge(a.part + (size_t)q * (1 + G), blocks, blocks, Q, 0, G, t.opt_orig, pl.P,
                                  pl.spot, nullptr, nullptr, grads_dev + (size_t)orig * G,
                                  deltas_dev ? deltas_dev + orig : nullptr, st);
        }
    }
    if (e != hipSuccess) return fail(ctx, LV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    record_info(ctx, pl, true, false, ctx->part.p);
    ctx->last_Q = Q;
    ctx->info.n_blocks = blocks;
    ctx->info.block = block;
    ctx->info.tile_paths = block;
    ctx->info.copies = 1;
    ctx->info.window = 8;
    ctx->info.hist_window = 8;
    ctx->info.fixed_point_bits = -1000;   // one scale per option
    return LV_OK;
}

lv_status lv_debug_philox(lv_ctx *ctx, uint64_t seed, uint64_t m0, int32_t n_m, uint64_t p0,
                          int64_t n_paths, uint32_t *words_dev) {
    if (!ctx) return fail(nullptr, LV_ERR_ARG, "ctx is NULL");
    if (!words_dev || n_m < 1 || n_paths < 1) return fail(ctx, LV_ERR_ARG, "bad arguments");
    HIPCHECK(ctx, hipSetDevice(ctx->device));
    hipError_t e = lvk::launch_debug_philox(seed, m0, n_m, p0, n_paths, words_dev, ctx->stream());
    if (e != hipSuccess) return fail(ctx, LV_ERR_HIP, "launch failed: %s", hipGetErrorString(e));
    return LV_OK;
}

lv_status lv_debug_normals(lv_ctx *ctx, int32_t precision, uint64_t seed, uint64_t p0,
                           int64_t n_paths, int32_t n_steps, void *z_dev) {
    if (!ctx) return fail(nullptr, LV_ERR_ARG, "ctx is NULL");
    if (!z_dev || n_paths < 1 || n_steps < 1 || (precision != 32 && precision != 64))
        return fail(ctx, LV_ERR_ARG, "bad arguments");
    HIPCHECK(ctx, hipSetDevice(ctx->device));
    hipError_t e = lvk::launch_debug_normals(precision, seed, p0, n_paths, n_steps, 1.0, z_dev, ctx->stream());
    if (e != hipSuccess) return fail(ctx, LV_ERR_HIP, "launch failed: %s", hipGetErrorString(e));
    return LV_OK;
}

lv_status lv_kernel_times(lv_ctx *ctx, double *ms, int64_t *counts, int32_t reset) {
    if (!ctx || !ms || !counts) return fail(ctx, LV_ERR_ARG, "ctx, ms and counts are required");
    HIPCHECK(ctx, hipSetDevice(ctx->device));
    lv_status s = collect_times(ctx);
    if (s != LV_OK) return s;
    for (int k = 0; k < LV_K_COUNT; ++k) {
        ms[k] = ctx->k_ms[k];
        counts[k] = ctx->k_count[k];
        if (reset) {
            ctx->k_ms[k] = 0.0;
            ctx->k_count[k] = 0;
        }
    }
    return LV_OK;
}

lv_status lv_tuning_candidates(const lv_grid *grid, const lv_book *book, int64_t n_paths,
                               int32_t n_steps, const lv_opts *opts, int32_t *shapes_out,
                               int32_t max, int32_t *n_out) {
    if (!shapes_out || !n_out || max < 1) return fail(nullptr, LV_ERR_ARG, "shapes_out, n_out and max >= 1 required");
    int n_cu = 256;
    size_t max_lds = 160 * 1024;
    int nd = 0;
    if (hipGetDeviceCount(&nd) == hipSuccess && nd > 0) n_cu = device_cus(0, &max_lds);
    else (void)hipGetLastError();
    Plan pl;
    lv_status s = plan_request(nullptr, grid, 1, nullptr, 100.0, book, n_paths, n_steps, 0, opts, n_cu,
                               max_lds, pl);
    if (s != LV_OK) return s;
    int n = 0;
    const Shape base{pl.block, pl.K, pl.W, pl.bpc, pl.fblock, pl.fbpc};
    std::vector<Shape> rows = adjoint_candidates(pl, base, n_cu, max_lds);
    for (const Shape &c : forward_candidates(pl, base, n_cu, max_lds)) rows.push_back(c);
    for (const Shape &c : rows) {
        if (n >= max) break;
        int32_t *r = shapes_out + 6 * n;
        r[0] = c.block;
        r[1] = c.K;
        r[2] = pl.adjoint == LV_ADJ_CHECKPOINT ? pl.seg : c.W;
        r[3] = c.bpc;
        r[4] = c.fblock;
        r[5] = c.fbpc;
        ++n;
    }
    *n_out = n;
    return LV_OK;
}

lv_status lv_tuning_save(const lv_ctx *ctx, const char *path, int32_t *n_out) {
    if (!ctx || !path) return fail(nullptr, LV_ERR_ARG, "ctx and path are required");
    FILE *f = fopen(path, "w");
    if (!f) return fail(const_cast<lv_ctx *>(ctx), LV_ERR_ARG, "cannot write %s", path);
    int n = 0;
    for (const auto &kv : ctx->tuned) {
        write_tuning_line(f, ctx, kv.first, kv.second);
        ++n;
    }
    const bool ok = fclose(f) == 0;
    if (!ok) return fail(const_cast<lv_ctx *>(ctx), LV_ERR_ARG, "cannot write %s", path);
    if (n_out) *n_out = n;
    return LV_OK;
}

lv_status lv_tuning_load(lv_ctx *ctx, const char *path, int32_t *n_out) {
    if (!ctx || !path) return fail(ctx, LV_ERR_ARG, "ctx and path are required");
    FILE *f = fopen(path, "r");
    if (!f) return fail(ctx, LV_ERR_ARG, "cannot read %s", path);
    char *line = nullptr;   // whole lines of any length (getline grows the buffer)
    size_t cap = 0;
    int n = 0, lineno = 0;
    lv_status st = LV_OK;
    while (getline(&line, &cap, f) > 0) {
        ++lineno;
        if (line[0] == '\n' || line[0] == '#') continue;
        char tag[32], arch[64], key[512];
        int ver = 0, cus = 0;
        Shape c;
        if (sscanf(line, "%31s %d %63s %d %511s %d %d %d %d %d %d", tag, &ver, arch, &cus, key, &c.block, &c.K,
                   &c.W, &c.bpc, &c.fblock, &c.fbpc) != 11 || strcmp(tag, kTuneTag) != 0) {
            st = fail(ctx, LV_ERR_ARG, "%s:%d is not a saved tuning", path, lineno);
            break;
        }
        // each field within what lv_opts accepts (the planner checks the LDS fit and the
        // precision's block limit when the shape is used)
        auto blk = [](int b) { return b >= 64 && b <= 1024 && b % 64 == 0; };
        if (!blk(c.block) || !blk(c.fblock) || c.K < 1 || c.K > 16 || (c.K & (c.K - 1)) || c.W < 8 ||
            c.W > 64 || c.W % 8 || c.bpc < 1 || c.bpc > 64 || c.fbpc < 1 || c.fbpc > 64) {
            st = fail(ctx, LV_ERR_ARG, "%s:%d holds an invalid launch shape", path, lineno);
            break;
        }
        // only shapes timed on this kind of device and count of CUs apply here
        if (ver != kTuneVersion || ctx->arch != arch || cus != ctx->n_cu) continue;
        ctx->tuned[key] = c;
        ++n;
    }
    free(line);
    fclose(f);
    if (st != LV_OK) return st;
    if (n_out) *n_out = n;
    return LV_OK;
}

lv_status lv_last_run_info(const lv_ctx *ctx, lv_run_info *info) {
    if (!ctx || !info) return fail(nullptr, LV_ERR_ARG, "ctx and info are required");
    *info = ctx->info;
    return LV_OK;
}

lv_status lv_debug_block_partials(lv_ctx *ctx, double *host_out, size_t host_len) {
    if (!ctx || !host_out) return fail(ctx, LV_ERR_ARG, "ctx and host_out are required");
    const int B = ctx->info.n_blocks, Q = ctx->last_Q;
    if (B <= 0 || !ctx->last_part) return fail(ctx, LV_ERR_ARG, "no pricing call has run on this context");
    if (host_len < (size_t)B * Q) return fail(ctx, LV_ERR_ARG, "host_out holds %zu doubles, need %zu", host_len, (size_t)B * Q);
    HIPCHECK(ctx, hipSetDevice(ctx->device));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream()));
    HIPCHECK(ctx, hipMemcpy(host_out, ctx->last_part, (size_t)B * Q * 8, hipMemcpyDeviceToHost));
    return LV_OK;
}

lv_status lv_debug_option_order(const lv_book *book, int32_t n_steps, int32_t *order_out) {
    if (!book || !order_out || book->n_opt < 1 || !book->maturity || n_steps < 1)
        return fail(nullptr, LV_ERR_ARG, "book, order_out and n_steps >= 1 are required");
    double tmax = 0.0;
    for (int k = 0; k < book->n_opt; ++k) tmax = std::max(tmax, book->maturity[k]);
    std::vector<long long> steps(book->n_opt);
    for (int k = 0; k < book->n_opt; ++k) steps[k] = std::llround(book->maturity[k] / (tmax / n_steps));
    std::vector<int> order(book->n_opt);
    for (int k = 0; k < book->n_opt; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return steps[x] < steps[y]; });
    for (int k = 0; k < book->n_opt; ++k) order_out[k] = order[k];
    return LV_OK;
}

}  // extern "C"

// lv_internal.h -- interface between the host runtime (lv_api.cpp) and the
// device kernels (lv_k_*.hip) of the local-vol Monte Carlo library.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>

namespace lvk {

// Everything a pricing kernel needs, passed by value.  Option arrays are in
// tap order (ascending maturity step); opt_orig maps back to caller order.
struct Args {
    // grid and time stepping
    int I, J, N, axis;          // spot nodes, time nodes, steps, spot axis kind (0 lin, 1 log)
    double inv_du;              // 1 / node spacing in the spot-axis coordinate
    double a_off;               // grid coordinate a = x * inv_du + a_off (x = S on lin, y on log)
    double spot, dt, sqrt_dt;
    const double *sigma;        // [I][J] FP64, this surface
    const int *tj;              // [N] time cell of step n (non-decreasing in n)
    const double *ta;           // [N] weight of time node tj+1 at step n
    const int *cell_lo;         // [J] first step whose time cell is >= j (N if none)
    const void *gtab;           // [N][I] pairs (c, d) in the kernel's precision: c = sigma(x_i, t_n)
                                // time-interpolated, d = c(x_{i+1}) - c(x_i) (0 at the last node)
    long long P;                // paths
    unsigned key0, key1;        // Philox key = seed
    // book
    int n_opt, n_taps;
    const int *tap_step;        // [n_taps] ascending step index of each maturity
    const int *tap_first;       // [n_taps] first option (tap order) at that step
    const int *tap_count;       // [n_taps]
    const int *opt_put;         // [n_opt] tap order
    const double *opt_strike;   // [n_opt] tap order
    const int *opt_orig;        // [n_opt] caller index of each option
    const double *opt_disc;     // [n_opt] tap order: discount factor e^{-r T_k} (1 at zero rate)
    const double *cot;          // [n_opt] cotangent per option, caller order
    double rate_dt;             // r dt: the trend each step adds (0: the driftless SDE)
    // storage
    void *states;               // stored planes [N][P]: plane n holds y_{n+1}
    void *ckpt;                 // checkpoint slots [n_seg][n_blocks * block]
    // per-block partial records: [n_blocks][Q], Q = 2 n_opt + 1 + I J
    double *part;
    int Q;
    // tiling
    int n_tiles;                // path tiles of blockDim paths
    int W;                      // steps per LDS table window (multiple of 4)
    int WH;                     // steps per gradient-histogram window (multiple of W)
    int K;                      // privatised histogram copies
    int CH;                     // reverse kernel: path tiles per live-path list
    int dense;                  // reverse kernel: sweep every path, not only live ones
    int seg;                    // checkpoint segment (steps)
    int scheme;                 // 0: Euler on y = ln(X/X0); 1: Euler on X (stored states hold X)
    int sigma_bf16;             // 1: the table is built from sigma rounded to bfloat16
};

enum Variant { FWD_PRICE = 0, FWD_STORE = 1, REV_STORED = 2, FUSED_CKPT = 3 };

// Largest block the adjoint kernels (stored reverse, fused checkpoint) are built
// for: 512 lanes for FP64, whose registers then fit without spills, 1024 for FP32.
constexpr int adjoint_max_block(int real_bytes) { return real_bytes == 8 ? 512 : 1024; }

// LDS bytes a kernel variant needs for the given shape (W table steps, WH
// histogram steps, CH tiles per live-path list).
size_t lds_bytes(int variant, int precision, int I, int J, int n_opt, int block, int W, int WH, int K, int CH);
// Largest fixed-point term the gradient histogram accepts, for the given shape.  Lanes
// with a path: at most min(block, P).  FP32: every histogram word receives at most one
// term per path of its copy class between folds (one tile) and must stay inside int32.
// FP64: the K words of a node are summed in int64 at the fold, so all of a tile's terms
// must fit; FP64 is capped at 2^51, where the rounding of terms to integers stays exact.
__host__ __device__ inline double fixed_point_qmax(int precision, int block, int K, long long P) {
    const int act = (int)(P < block ? P : block);
    if (precision == 64) return fmin(ldexp(1.0, 62) / act, ldexp(1.0, 51));
    return floor(2147483000.0 / (double)((act + K - 1) / K)) - 2.0;
}

// Optional timing events taken from a launch's own dispatch (start of the first
// kernel, end of the last), so timing adds no packets between kernels.
struct Ev {
    hipEvent_t start = nullptr, stop = nullptr;
};

// Vol table of every step into a.gtab (run before the pricing kernels).
hipError_t launch_table(const Args &a, int precision, hipStream_t st, Ev ev = {});
hipError_t launch_fwd(const Args &a, int precision, bool store, int blocks, int block,
                      hipStream_t st, Ev ev = {});
hipError_t launch_rev(const Args &a, int precision, int blocks, int block, hipStream_t st, Ev ev = {});
hipError_t launch_fused_ckpt(const Args &a, int precision, int blocks, int block, hipStream_t st,
                             Ev ev = {});
// Reverse sweep over stored states giving the options o0 .. o0 + KO - 1 (tap order;
// KO = 1, 2, 4 or 8) each its own grid and delta: block records [KO][1 + I J] into
// a.part with a.Q = KO (1 + I J); a.K = 1.  n_end: the largest maturity step of the
// group (the sweep starts there).
hipError_t launch_rev_per_option(const Args &a, int precision, int o0, int KO, int n_end, int blocks, int block,
                                 hipStream_t st);
// LDS bytes of that sweep for the shape.
size_t lds_bytes_per_option(int precision, int I, int J, int block, int KO);
// Fixed-order merge of part [records][Q] into final outputs: payoff entries over
// the first B_pay records, the rest over the first B_grad.
hipError_t launch_merge(const double *part, int B_pay, int B_grad, int Q, int n_opt, int G,
                        const int *opt_orig, long long P, double spot, double *price, double *stderr_,
                        double *grad, double *delta, hipStream_t st, Ev ev = {});
// Bump-and-reprice: 2 mc bumped copies of sigma [G] (node m0 + s at +-eps/2) into
// out [2 mc][G]; then grad[m0 + s] = sum_k weight_k (price[2s][k] - price[2s+1][k]) / eps.
hipError_t launch_bump(const double *sigma, int G, int m0, int mc, double eps, double *out, hipStream_t st);
hipError_t launch_fd(const double *prices, int n_opt, const double *weight, int m0, int mc, double eps,
                     double *grad, hipStream_t st);
// Size of the per-GPU workspace of the allocation-free entry point, and the devices
// whose address is kept.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
// Address of that workspace on `device`, which must be the current device; read with
// hipGetSymbolAddress on the first call per device and kept.
hipError_t scratch_address(int device, void **out);

hipError_t launch_debug_philox(unsigned long long seed, unsigned long long m0, int n_m,
                               unsigned long long p0, long long n_paths, uint32_t *out,
                               hipStream_t st);
hipError_t launch_debug_normals(int precision, unsigned long long seed, unsigned long long p0,
                                long long n_paths, int n_steps, double sqrt_dt_unused,
                                void *out, hipStream_t st);

}  // namespace lvk

// lv_device.h -- device code shared by the kernel translation units of the
// local-vol Monte Carlo library (lv_k_*.hip): the method's building blocks (Philox,
// uniforms and Box-Muller, the vol lookup, the Euler step, payoff sums, adjoint seeds,
// the gradient histogram's scatter and fold) and the launch helpers.
//
// The kernels: gfx950 kernels for Monte Carlo pricing under the Dupire
// local-volatility model and the adjoint of the price with respect to every node
// of the vol grid (arXiv 2002.02481: the SDE and explicit Euler scheme of Sec.
// IV-A, bilinear interpolation of Sec. IV-A/IV-D, payoff averages of Sec.
// IV-B/IV-C, back-propagated sensitivities of Sec. III/IV-C).
//
// Mapping: one lane per path, 64-lane wavefronts, blocks of whole wavefronts that
// loop over path tiles (persistent grid).  All lanes of a block are at the same
// step, so the time cell of a step is uniform.  A small kernel first writes, for
// every step, the time-interpolated vol column and its node-to-node difference,
// c[n][i] = sigma(x_i, t_n), d[n][i] = c[n][i+1] - c[n][i]; blocks copy windows of
// W steps of it into LDS (double-buffered, the next window's copy in flight while
// the current one is used), so the spot lookup is one LDS read and one FMA.
//
// Gradient accumulation: per step a path adds x(1-f) to spot node i and x f to
// node i+1 of that step's column (x = lambda * dy_{n+1}/dsigma_n), the time
// weights being uniform.  LDS float atomics are slow on gfx950, integer ones are
// not, so the two terms are rounded to fixed point (scale 2^F chosen from the
// book's size) and added with ds_add_u32 (FP32 kernels) or ds_add_u64 (FP64
// kernels) into a step-indexed histogram H[n][i][copy], privatised K ways by lane
// to spread same-cell collisions.  The histogram spans WH steps (as many as fit,
// often the whole horizon); at its boundaries and at the end of a path tile it is
// folded into a per-block FP64 grid with the time weights, one owner thread per
// grid node.  Blocks write their grids once and a fixed-order compensated merge
// combines them.
// Terms too large for the fixed-point range take an FP64 LDS-atomic side path into
// the block's grid.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "lv_internal.h"

namespace lvk {

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64
// multiplies; the key advances by the Weyl constants between rounds.
// --------------------------------------------------------------------------
struct Words {
    uint32_t x, y, z, w;
};

// a ^ b ^ c in one instruction: gfx950's three-input bit operation with the truth
// table 0x96 (the parity of the three input bits); the compiler emits two XORs for it.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = xor3((uint32_t)(b >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(a >> 32), c3, k1);
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words{c0, c1, c2, c3};
}

// --------------------------------------------------------------------------
// Per-precision arithmetic.  Uniforms are (2k+1) 2^-24 with k the top 23 bits of
// a word: exact in float and double alike.
// --------------------------------------------------------------------------
template <typename R>
struct Math;

template <>
struct Math<float> {
    typedef int Acc;                       // fixed-point histogram word
    static constexpr int FMAX = 40;
    // (2k + 1) 2^-24 with k = w >> 9: the float with exponent 0 and mantissa k (the funnel
    // shift of 0x7f above w puts k under a biased exponent of 127) is 1 + k 2^-23, and
    // subtracting 1 - 2^-24 is exact (the result is a multiple of 2^-24 below 1)
    __device__ static __forceinline__ float uniform(uint32_t w) {
        return __uint_as_float(__builtin_amdgcn_alignbit(0x7fu, w, 9)) - 0x1.fffffep-1f;
    }
    // sqrt(dt) * (Z_a, Z_b) from one word pair (Box-Muller); the hardware sine
    // and cosine take their argument in revolutions, i.e. compute sin(2 pi u).
    __device__ static __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float sdt,
                                                      float &za, float &zb) {
        const float ua = uniform(wa), ub = uniform(wb);
        const float r = __builtin_amdgcn_sqrtf(-1.38629436f * __builtin_amdgcn_logf(ua)) * sdt;
        za = r * __builtin_amdgcn_cosf(ub);
        zb = r * __builtin_amdgcn_sinf(ub);
    }
    __device__ static __forceinline__ float ex(float y) {
        return __builtin_amdgcn_exp2f(y * 1.44269504f);
    }
    __device__ static __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static __forceinline__ float lg(float x) { return __builtin_amdgcn_logf(x) * 0.693147181f; }
    // (q0, q1) = (rn(x) - rn(xf), rn(xf)).  For |x|, |xf| <= 2^22 (MAGIC_MAX) adding
    // 1.5 * 2^23 rounds to an integer (nearest, ties to even) held in the low
    // mantissa bits, so bit patterns differ by the integers themselves; larger
    // ranges (blocks with few paths) convert with round-to-nearest.
    static constexpr double MAGIC_MAX = 4194304.0;
    __device__ static __forceinline__ void to_acc2(float x, float xf, bool magic, Acc &q0, Acc &q1) {
        if (magic) {
            const int bx = __float_as_int(x + 12582912.0f), bf = __float_as_int(xf + 12582912.0f);
            q0 = bx - bf;
            q1 = bf - 0x4B400000;
        } else {
            q1 = __float2int_rn(xf);
            q0 = __float2int_rn(x) - q1;
        }
    }
    __device__ static __forceinline__ void acc_add(Acc *p, Acc v) { atomicAdd(p, v); }
};

template <>
struct Math<double> {
    typedef long long Acc;
    static constexpr int FMAX = 62;
    __device__ static __forceinline__ double uniform(uint32_t w) {
        return fma((double)(w >> 9), 0x1p-23, 0x1p-24);
    }
    __device__ static __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double sdt,
                                                      double &za, double &zb) {
        const double ua = uniform(wa), ub = uniform(wb);
        const double r = sqrt(-2.0 * log(ua)) * sdt;
        double s, c;
        sincospi(2.0 * ub, &s, &c);
        za = r * c;
        zb = r * s;
    }
    __device__ static __forceinline__ double ex(double y) { return exp(y); }
    __device__ static __forceinline__ double rcp(double x) { return 1.0 / x; }
    __device__ static __forceinline__ double lg(double x) { return log(x); }
    // as for float with 1.5 * 2^52; the FP64 range is capped at 2^51, so always exact
    static constexpr double MAGIC_MAX = 2251799813685248.0;
    __device__ static __forceinline__ void to_acc2(double x, double xf, bool, Acc &q0, Acc &q1) {
        const long long bx = __double_as_longlong(x + 6755399441055744.0);
        const long long bf = __double_as_longlong(xf + 6755399441055744.0);
        q0 = bx - bf;
        q1 = bf - 0x4338000000000000LL;
    }
    __device__ static __forceinline__ void acc_add(Acc *p, Acc v) {
        atomicAdd((unsigned long long *)p, (unsigned long long)v);
    }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// Load of read-only table data at a wave-uniform address through the constant
// address space, so that it is a scalar-cache load: it then does not share the
// vector-memory counter that the state prefetches are waited on with.  Scalar loads
// return out of order, so waiting for one waits for every LDS operation as well: a
// value that stays live across steps (the next tap step) is read with a vector load.
template <typename T>
__device__ __forceinline__ T ldu(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}

// --------------------------------------------------------------------------
// LDS carve-up, shared by the kernels and the host planner.
// --------------------------------------------------------------------------
struct Lds {
    size_t g64, wpart, wlam, tab, hist, live, yfin, total;
};

// CH: path tiles per live-path list of the stored reverse kernel.
__host__ __device__ inline Lds lds_layout(int variant, int rbytes, int accbytes, int I, int J,
                                          int n_opt, int wpb, int W, int WH, int K, int CH) {
    Lds L{};
    size_t off = 0;
    const bool grad = variant == REV_STORED || variant == FUSED_CKPT;
    const bool pay = variant != REV_STORED;
    const int tab_bufs = variant == FUSED_CKPT ? 1 : 2;   // double-buffered where prefetched
    L.g64 = off;
    off += grad ? align16((size_t)I * J * 8) : 0;
    L.wpart = off;
    off += pay ? align16((size_t)wpb * n_opt * 2 * 8) : 0;
    L.wlam = off;
    off += grad ? align16((size_t)wpb * 8) : 0;
    L.tab = off;
    off += align16((size_t)tab_bufs * W * I * 2 * rbytes);
    L.hist = off;
    off += grad ? align16((size_t)WH * K * (I + 1) * accbytes) : 0;   // rows of I + 1 words
    L.live = off;   // live-path list + wave counts (the fused kernel: its queue ring, wave counts
                    // and the tile of each slot set)
    off += variant == REV_STORED   ? align16(((size_t)CH * wpb * 64 + 16) * 4)
           : variant == FUSED_CKPT ? align16(((size_t)CH * wpb * 64 + 16 + CH) * 4)
                                   : 0;
    L.yfin = off;   // the fused kernel's final state per path of a chunk
    off += variant == FUSED_CKPT ? align16((size_t)CH * wpb * 64 * rbytes) : 0;
    L.total = off;
    return L;
}



// --------------------------------------------------------------------------
// Table windows.  Rows n0 .. n0+nw-1 of the global table are contiguous, so a
// window is a straight copy into LDS.  issue() loads the first PF pairs per
// thread into registers, commit() writes them (and copies any remainder) into
// an LDS buffer; the forward and reverse kernels issue the next window's copy
// at a window start and commit it one step group later into the other buffer.
// --------------------------------------------------------------------------
template <typename R>
struct Pair;
template <>
struct Pair<float> {
    typedef float2 T;
    static constexpr int PF = 4;
};
template <>
struct Pair<double> {
    typedef double2 T;
    static constexpr int PF = 2;
};

template <typename R>
struct TabStage {
    typedef typename Pair<R>::T T;
    static constexpr int PF = Pair<R>::PF;
    T v[PF];
    int n0, nw;
    __device__ __forceinline__ void issue(const Args &a, int first, int count) {
        n0 = first;
        nw = count;
        const T *src = (const T *)a.gtab + (size_t)n0 * a.I;
        const int ne = nw * a.I;
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int e = threadIdx.x + k * blockDim.x;
            if (e < ne) v[k] = src[e];
        }
    }
    __device__ __forceinline__ void commit(const Args &a, R *dst) const {
        const T *src = (const T *)a.gtab + (size_t)n0 * a.I;
        T *d = (T *)dst;
        const int ne = nw * a.I;
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int e = threadIdx.x + k * blockDim.x;
            if (e < ne) d[e] = v[k];
        }
        for (int e = threadIdx.x + PF * blockDim.x; e < ne; e += blockDim.x) d[e] = src[e];
    }
};

// --------------------------------------------------------------------------
// Device building blocks
// --------------------------------------------------------------------------
__device__ __forceinline__ float clamp_to(float a, float hi) {
    return __builtin_amdgcn_fmed3f(a, 0.0f, hi);
}
__device__ __forceinline__ double clamp_to(double a, double hi) { return fmin(fmax(a, 0.0), hi); }

template <typename R>
struct Look {
    R s;       // sigma(S_n, t_n)
    R f;       // position inside the spot cell
    R d;       // node difference of the cell (d sigma / d a)
    R S;       // spot (linear axis only)
    R E;       // S / spot = e^y (linear axis, log-Euler state only)
    int i;     // lower spot node
    bool in;   // strictly inside the spot range (slope is zero outside)
};

// Lookup at x with a = x inv_du + a_off the grid coordinate (x is S or S / spot on a
// linear axis, ln(S / spot) on a log one, the caller scaling inv_du and a_off to match).
template <typename R>
__device__ __forceinline__ Look<R> lookup_at(R x, const R *trow, R inv_du, R a_off, R amax) {
    Look<R> L;
    L.S = 0;
    const R a = fma(x, inv_du, a_off);
    const R ac = clamp_to(a, amax);
    // i = I - 1 only at (or beyond) the top node: there f = 0 and the table's d = 0,
    // so the value is the node's, the term for node i + 1 is zero and so is the slope;
    // below the range ac = 0.  So "strictly inside" is ac > 0 (the top needs no test).
    L.in = ac > (R)0;
    L.i = (int)ac;
    // ac >= 0: the fraction ac - floor(ac) is exact, and in single precision one instruction
    if constexpr (sizeof(R) == 4) L.f = __builtin_amdgcn_fractf(ac);
    else L.f = ac - (R)L.i;
    const R c = trow[2 * L.i], d = trow[2 * L.i + 1];
    L.s = fma(L.f, d, c);
    L.d = d;
    return L;
}

// Lookup at log-spot state y = ln(S / spot) (L.S = S on a linear axis).  On a linear
// axis the coordinate is E / du' + a_off with E = e^y and du' = du / spot, so a lookup
// that does not need S itself takes no multiply for it.
template <typename R, int AXIS>
__device__ __forceinline__ Look<R> lookup(R y, const R *trow, R inv_du, R a_off, R amax, R spot) {
    if (AXIS == 0) {
        const R E = Math<R>::ex(y);
        Look<R> L = lookup_at<R>(E, trow, spot * inv_du, a_off, amax);
        L.S = spot * E;
        L.E = E;
        return L;
    }
    return lookup_at<R>(y, trow, inv_du, a_off, amax);
}

// Lookup at the state of either scheme: y = ln(X / spot) (EX false) or X itself (EX
// true; L.S = X).  On a log axis the EX coordinate is ln(X / spot), as in the log
// scheme: a small number, so the cell fraction keeps its bits (ln X itself would
// lose about three of them to the offset).
template <typename R, int AXIS, bool EX>
__device__ __forceinline__ Look<R> lookup_state(R v, const R *trow, R inv_du, R a_off, R inv_spot, R amax,
                                                R spot) {
    if (!EX) return lookup<R, AXIS>(v, trow, inv_du, a_off, amax, spot);
    Look<R> L = lookup_at<R>(AXIS == 0 ? v : Math<R>::lg(v * inv_spot), trow, inv_du, a_off, amax);
    L.S = v;
    return L;
}

// One Euler step from state v with vol s and scaled normal z = sqrt(dt) Z: on y = ln(X/X0),
// y + s (z - s dt / 2) (+ r dt); on X, X + s X z (+ r dt X).
template <typename R, bool EX, bool RT>
__device__ __forceinline__ R step(R v, R s, R z, R hdt, R rdt) {
    if (EX) return RT ? fma(v, fma(s, z, rdt), v) : fma(s * v, z, v);
    const R nv = fma(s, fma(-hdt, s, z), v);
    return RT ? nv + rdt : nv;
}

// Forward payoff taps at step n+1 (the state is y_{n+1}): wave sums of payoff
// and payoff^2 in FP64 into the wave's LDS slot.
template <typename R, bool EX>
__device__ __forceinline__ void fwd_payoffs(const Args &a, int tap, R y, bool active, double *wpart,
                                            int wave, int lane) {
    const double S = EX ? (double)y : (double)((R)a.spot * Math<R>::ex(y));
    const int k0 = ldu(a.tap_first + tap), kc = ldu(a.tap_count + tap);
    for (int q = 0; q < kc; ++q) {
        const int k = k0 + q;
        const double K = ldu(a.opt_strike + k);
        double pay = ldu(a.opt_put + k) ? fmax(K - S, 0.0) : fmax(S - K, 0.0);
        pay *= ldu(a.opt_disc + k);   // e^{-r T_k}
        if (!active) pay = 0.0;
        const double s1 = wave_sum(pay), s2 = wave_sum(pay * pay);
        if (lane == 0) {
            wpart[(wave * a.n_opt + k) * 2] += s1;
            wpart[(wave * a.n_opt + k) * 2 + 1] += s2;
        }
    }
}

// Adjoint seeds at step n+1: lambda += scale sum_k w_k d payoff_k / d state (the
// adjoint kernels carry lambda scaled by the fixed-point scale 2^F); the state is y
// (d payoff / d y = +-S in the money) or, with EX, X (d payoff / d X = +-1).
// rev_seeds_at takes the spot S = spot e^y of the state (with EX, X itself).
template <typename R, bool EX>
__device__ __forceinline__ R rev_seeds_at(const Args &a, int tap, R S, R lam, double scale) {
    const R D = EX ? (R)1 : S;
    const double Sd = (double)S;
    const int k0 = ldu(a.tap_first + tap), kc = ldu(a.tap_count + tap);
    for (int q = 0; q < kc; ++q) {
        const int k = k0 + q;
        const double K = ldu(a.opt_strike + k);
        const R w = (R)(ldu(a.cot + ldu(a.opt_orig + k)) * ldu(a.opt_disc + k) * scale);
        if (ldu(a.opt_put + k)) {
            if (Sd < K) lam -= w * D;
        } else {
            if (Sd > K) lam += w * D;
        }
    }
    return lam;
}

template <typename R, bool EX>
__device__ __forceinline__ R rev_seeds(const Args &a, int tap, R y, R lam, double scale) {
    return rev_seeds_at<R, EX>(a, tap, EX ? y : (R)a.spot * Math<R>::ex(y), lam, scale);
}

// Fold of the histogram rows of steps [h0, h0 + nh) into the block's FP64 grid.
// The histogram is H[n][copy][I + 1] (the last word of a row only ever receives 0).
// Node (i, j) takes alpha_n of every row n of time cell j - 1 and 1 - alpha_n of
// every row of cell j (the steps of a cell are contiguous), so each node has one
// owner thread and no atomics are needed; the rows are then cleared.  Callers
// synchronise the block before; it is synchronised again on return.
template <typename R>
__device__ void fold(const Args &a, typename Math<R>::Acc *H, double *g64, int h0, int nh,
                     double inv_sc) {
    typedef typename Math<R>::Acc Acc;
    const int I = a.I, J = a.J, K = a.K, h1 = h0 + nh;
    const int c0 = ldu(a.tj + h0), c1 = ldu(a.tj + h1 - 1);
    const int nn = (c1 - c0 + 2) * I;   // nodes j = c0 .. c1 + 1
    for (int e = threadIdx.x; e < nn; e += blockDim.x) {
        const int jj = e / I, i = e - jj * I, j = c0 + jj;
        double acc = 0.0;
        if (j > c0) {
            const int lo = max(a.cell_lo[j - 1], h0), hi = min(a.cell_lo[j], h1);
            for (int n = lo; n < hi; ++n) {
                const Acc *h = H + (size_t)(n - h0) * K * (I + 1) + i;
                long long q = 0;
                for (int c = 0; c < K; ++c) q += (long long)h[c * (I + 1)];
                acc += a.ta[n] * ((double)q * inv_sc);
            }
        }
        if (j <= c1) {
            const int lo = max(a.cell_lo[j], h0), hi = min(a.cell_lo[j + 1], h1);
            for (int n = lo; n < hi; ++n) {
                const Acc *h = H + (size_t)(n - h0) * K * (I + 1) + i;
                long long q = 0;
                for (int c = 0; c < K; ++c) q += (long long)h[c * (I + 1)];
                acc += (1.0 - a.ta[n]) * ((double)q * inv_sc);
            }
        }
        g64[i * J + j] += acc;
    }
    __syncthreads();
    const size_t words = (size_t)nh * K * (I + 1), n16 = words * sizeof(Acc) / 16;
    int4 *h4 = (int4 *)H;
    for (size_t e = threadIdx.x; e < n16; e += blockDim.x) h4[e] = make_int4(0, 0, 0, 0);
    for (size_t e = n16 * 16 / sizeof(Acc) + threadIdx.x; e < words; e += blockDim.x) H[e] = 0;
    __syncthreads();
}

// Scatter of one step's adjoint term x (lambda c, already scaled by 2^F): x(1-f)
// to node i and x f to node i+1 of this lane's histogram row hrow.  SKIP0: lanes
// whose term is zero stay idle (for sweeps where many lanes carry a zero adjoint);
// otherwise every lane adds, a zero where its term is zero or out of range, so the
// common case takes no branch.
template <typename R, bool SKIP0 = true>
__device__ __forceinline__ void scatter(const Args &a, typename Math<R>::Acc *hrow, double *g64, int n,
                                        const Look<R> &L, R x, R qm, bool magic, double inv_sc) {
    typedef typename Math<R>::Acc Acc;
    if (SKIP0 && x == (R)0) return;
    const bool in_range = fabs(x) <= qm;   // false for a term that is not finite
    if (SKIP0 ? in_range : true) {
        const R xq = SKIP0 || in_range ? x : (R)0;
        Acc q0, q1;
        Math<R>::to_acc2(xq, xq * L.f, magic, q0, q1);
        Acc *h = hrow + L.i;
        Math<R>::acc_add(h, q0);
        Math<R>::acc_add(h + 1, q1);
    }
    if (!in_range) {
        // rare: outside the fixed-point range (or not finite): FP64 LDS atomics
        // straight into the block's grid (no fold runs while steps scatter)
        const int i = min(L.i, a.I - 2);
        const double f = (double)L.f + (double)(L.i - i);   // 1 at the top node
        const int j = ldu(a.tj + n), J = a.J;
        const double al = ldu(a.ta + n), g = (double)x * inv_sc;
        atomicAdd(&g64[i * J + j], g * (1.0 - f) * (1.0 - al));
        atomicAdd(&g64[(i + 1) * J + j], g * f * (1.0 - al));
        atomicAdd(&g64[i * J + j + 1], g * (1.0 - f) * al);
        atomicAdd(&g64[(i + 1) * J + j + 1], g * f * al);
    }
}

// Fixed-point exponent F from the book: terms are rarely above 8 * sum_k |w_k| max(S0, K_k).
__device__ __forceinline__ int fixed_point_bits(const Args &a, double qmax, int fbits_max) {
    double scale = 0.0;
    for (int k = 0; k < a.n_opt; ++k)
        scale += fabs(a.cot[a.opt_orig[k]]) * fmax(a.spot, a.opt_strike[k]);
    if (!(scale > 0.0)) return fbits_max;
    const int F = ilogb(qmax / (8.0 * scale));
    return F < -30 ? -30 : (F > fbits_max ? fbits_max : F);
}

// Steps per state block of the reverse sweep (the table window is a multiple of it).
constexpr int RB = 8;

// Whether path p can have a nonzero adjoint: some option with a nonzero cotangent
// is in the money at its maturity (the seed test of the sweep, on the stored state).
// A path for which this fails has lambda = 0 at every step and contributes exactly
// nothing to the gradient or to delta.
template <typename R, bool EX>
__device__ __forceinline__ bool tap_live(const Args &a, int t, R y) {
    const double Sd = EX ? (double)y : (double)((R)a.spot * Math<R>::ex(y));
    const int k0 = ldu(a.tap_first + t), kc = ldu(a.tap_count + t);
    for (int q = 0; q < kc; ++q) {
        const int k = k0 + q;
        if (ldu(a.cot + ldu(a.opt_orig + k)) == 0.0) continue;
        const double K = ldu(a.opt_strike + k);
        if (ldu(a.opt_put + k) ? (Sd < K) : (Sd > K)) return true;
    }
    return false;
}

template <typename R, bool EX>
__device__ bool path_live(const Args &a, const R *Y, size_t P, size_t p) {
    for (int t = 0; t < a.n_taps; ++t)
        if (tap_live<R, EX>(a, t, Y[(size_t)(a.tap_step[t] - 1) * P + p])) return true;
    return false;
}

// The fused kernel's launchers, one per precision and checkpoint segment (lv_k_fused.hip).
hipError_t launch_fused_p32_s8(const Args &a, int blocks, int block, hipStream_t st, Ev ev);
hipError_t launch_fused_p32_s16(const Args &a, int blocks, int block, hipStream_t st, Ev ev);
hipError_t launch_fused_p32_s32(const Args &a, int blocks, int block, hipStream_t st, Ev ev);
hipError_t launch_fused_p64_s8(const Args &a, int blocks, int block, hipStream_t st, Ev ev);
hipError_t launch_fused_p64_s16(const Args &a, int blocks, int block, hipStream_t st, Ev ev);
hipError_t launch_fused_p64_s32(const Args &a, int blocks, int block, hipStream_t st, Ev ev);

// --------------------------------------------------------------------------
// Launch helpers
// --------------------------------------------------------------------------
// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------
template <typename R>
static size_t lds_of(int variant, const Args &a, int block, int W) {
    const int rb = sizeof(R);
    return lds_layout(variant, rb, rb, a.I, a.J, a.n_opt, block / 64, W, a.WH, a.K, a.CH).total;
}

// Blocks above 64 KiB of LDS (gfx950 has 160 KiB per CU) must be allowed per kernel.
template <typename Kern>
static void allow_lds(Kern kernel, size_t lds) {
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// Launch with the timing events ev (in scope) attached to the dispatch, if any.
#define LAUNCH(kern, blocks, block, lds, st, a)                                                      \
    do {                                                                                             \
        allow_lds(kern, lds);                                                                        \
        if (ev.start || ev.stop)                                                                     \
            hipExtLaunchKernelGGL(kern, dim3(blocks), dim3(block), lds, st, ev.start, ev.stop, 0, a); \
        else                                                                                         \
            hipLaunchKernelGGL(kern, dim3(blocks), dim3(block), lds, st, a);                         \
    } while (0)

// Whether the adjoint kernels may round fixed-point terms with the magic-constant
// add (the term range fits it); FP64 ranges always do.
static inline bool use_magic(const Args &a, int precision, int block) {
    const double qmax = fixed_point_qmax(precision, block, a.K, a.P);
    return precision == 64 || qmax <= Math<float>::MAGIC_MAX;
}

}  // namespace lvk

// lv_kernels.hip -- gfx950 kernels for Monte Carlo pricing under the Dupire
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
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>
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

__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
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
    __device__ static __forceinline__ float uniform(uint32_t w) {
        return fmaf((float)(w >> 9), 0x1p-23f, 0x1p-24f);
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
    L.live = off;   // live-path list + wave counts
    off += variant == REV_STORED   ? align16(((size_t)CH * wpb * 64 + 16) * 4)
           : variant == FUSED_CKPT ? align16(((size_t)CH * wpb * 64 + 16) * 4)
                                   : 0;
    L.yfin = off;   // the fused kernel's final state per path of a chunk
    off += variant == FUSED_CKPT ? align16((size_t)CH * wpb * 64 * rbytes) : 0;
    L.total = off;
    return L;
}

size_t lds_bytes(int variant, int precision, int I, int J, int n_opt, int block, int W, int WH, int K,
                 int CH) {
    const int rb = precision == 64 ? 8 : 4;
    return lds_layout(variant, rb, rb, I, J, n_opt, block / 64, W, WH, K, CH).total;
}

__host__ __device__ double fixed_point_qmax(int precision, int block, int K, long long P) {
    // Lanes with a path: at most min(block, P).  FP32: every histogram word receives
    // at most one term per path of its copy class between folds (one tile) and must
    // stay inside int32.  FP64: the K words of a node are summed in int64 at the
    // fold, so all of a tile's terms must fit.
    // FP64 is capped at 2^51, where the rounding of terms to integers stays exact.
    const int act = (int)(P < block ? P : block);
    if (precision == 64) return fmin(ldexp(1.0, 62) / act, ldexp(1.0, 51));
    return floor(2147483000.0 / (double)((act + K - 1) / K)) - 2.0;
}

// --------------------------------------------------------------------------
// Vol table of every step: c = sigma(x_i, t_n), d = c(x_{i+1}) - c(x_i), time-
// interpolated in FP64 and rounded once to the kernel precision.
// --------------------------------------------------------------------------
template <typename R>
__global__ void k_table(Args a) {
    const int I = a.I, J = a.J;
    const long long ne = (long long)a.N * I;
    R *t = (R *)const_cast<void *>(a.gtab);
    const double *s = a.sigma;
    // node value: as given, or rounded to bfloat16 by way of FP32 (both roundings to
    // nearest, ties to even; bfloat16 is the upper half of an FP32 word, so adding
    // 0x7fff plus the kept word's lowest bit carries exactly when the dropped half is
    // above one half, or equal to it with that bit set)
    auto node = [&](int k) -> double {
        const double v = s[k];
        if (!a.sigma_bf16) return v;
        unsigned u = __float_as_uint((float)v);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (double)__uint_as_float(u & 0xffff0000u);
    };
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne;
         e += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(e / I), i = (int)(e - (long long)n * I);
        const int j = a.tj[n];
        const double al = a.ta[n];
        const double c0 = (1.0 - al) * node(i * J + j) + al * node(i * J + j + 1);
        double c1 = c0;
        if (i + 1 < I) c1 = (1.0 - al) * node((i + 1) * J + j) + al * node((i + 1) * J + j + 1);
        t[2 * e] = (R)c0;
        t[2 * e + 1] = (R)(c1 - c0);
    }
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
    int i;     // lower spot node
    bool in;   // strictly inside the spot range (slope is zero outside)
};

// Lookup at axis coordinate x (S on a linear axis, ln S on a log one) with offset
// a_off: a = x / du + a_off is the grid coordinate.
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
    L.f = ac - (R)L.i;
    const R c = trow[2 * L.i], d = trow[2 * L.i + 1];
    L.s = fma(L.f, d, c);
    L.d = d;
    return L;
}

// Lookup at log-spot state y = ln(S / spot) (L.S = S on a linear axis).
template <typename R, int AXIS>
__device__ __forceinline__ Look<R> lookup(R y, const R *trow, R inv_du, R a_off, R amax, R spot) {
    if (AXIS == 0) {
        const R S = spot * Math<R>::ex(y);
        Look<R> L = lookup_at<R>(S, trow, inv_du, a_off, amax);
        L.S = S;
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
template <typename R, bool EX>
__device__ __forceinline__ R rev_seeds(const Args &a, int tap, R y, R lam, double scale) {
    const R S = EX ? y : (R)a.spot * Math<R>::ex(y);
    const R D = EX ? (R)1 : S;
    const double Sd = (double)S;
    const int k0 = ldu(a.tap_first + tap), kc = ldu(a.tap_count + tap);
    for (int q = 0; q < kc; ++q) {
        const int k = k0 + q;
        const double K = ldu(a.opt_strike + k);
        const R w = (R)(ldu(a.cot + ldu(a.opt_orig + k)) * scale);
        if (ldu(a.opt_put + k)) {
            if (Sd < K) lam -= w * D;
        } else {
            if (Sd > K) lam += w * D;
        }
    }
    return lam;
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
// to node i and x f to node i+1 of this lane's histogram row hrow.
template <typename R>
__device__ __forceinline__ void scatter(const Args &a, typename Math<R>::Acc *hrow, double *g64, int n,
                                        const Look<R> &L, R x, R qm, bool magic, double inv_sc) {
    typedef typename Math<R>::Acc Acc;
    if (x == (R)0) return;   // lanes whose adjoint is zero (paths out of the money) stay idle
    if (fabs(x) <= qm) {
        Acc q0, q1;
        Math<R>::to_acc2(x, x * L.f, magic, q0, q1);
        Acc *h = hrow + L.i;
        Math<R>::acc_add(h, q0);
        Math<R>::acc_add(h + 1, q1);
    } else {
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

// --------------------------------------------------------------------------
// Forward kernel: price-only, or storing every state (split / stored adjoint).
// --------------------------------------------------------------------------
// FP32: at most 64 VGPRs, so that 8 waves fit per SIMD (the kernel is issue-bound)
// EX: the Euler step on X itself (the state and the stored planes are X).
template <typename R, int AXIS, bool STORE, bool EX>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 8 : 1)))
k_fwd(Args a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int wpb = blockDim.x >> 6, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int I = a.I, N = a.N, W = a.W, nW = (N + W - 1) / W;
    const Lds lay = lds_layout(STORE ? FWD_STORE : FWD_PRICE, sizeof(R), sizeof(R), I, a.J, a.n_opt,
                               wpb, W, a.WH, a.K, a.CH);
    double *wpart = (double *)(smem + lay.wpart);
    R *tuse = (R *)(smem + lay.tab), *tnext = tuse + 2 * W * I;
    for (int e = tid; e < wpb * a.n_opt * 2; e += blockDim.x) wpart[e] = 0.0;

    const R sdt = (R)a.sqrt_dt, hdt = (R)(0.5 * a.dt), inv_du = (R)a.inv_du, a_off = (R)a.a_off;
    const R inv_spot = (R)(1.0 / a.spot);
    const R spot = (R)a.spot, amax = (R)(I - 1);
    TabStage<R> stg;
    int wcur = -1;
    if ((int)blockIdx.x < a.n_tiles) {   // first window, into the buffer entered first
        stg.issue(a, 0, min(W, N));
        stg.commit(a, tnext);
    }

    for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const bool more = tile + (int)gridDim.x < a.n_tiles;
        const long long p = (long long)tile * blockDim.x + tid;
        const bool active = p < a.P;
        const uint32_t plo = (uint32_t)p, phi = (uint32_t)((unsigned long long)p >> 32);
        R y = EX ? spot : (R)0;
        int tap = 0, next_tap = a.n_taps > 0 ? a.tap_step[0] : -1;
        for (int wi = 0; wi < nW; ++wi) {
            const int ws = wi * W, we = min(N, ws + W);
            bool pending = false;
            if (wi != wcur) {
                __syncthreads();   // window wi is in tnext; nobody reads tuse any more
                R *t = tuse;
                tuse = tnext;
                tnext = t;
                wcur = wi;
                const int nx = wi + 1 < nW ? wi + 1 : (more ? 0 : -1);
                if (nx >= 0 && nW > 1) {
                    stg.issue(a, nx * W, min(W, N - nx * W));
                    pending = true;
                }
            }
            for (int n0 = ws; n0 < we; n0 += 4) {
                const Words w = philox10((uint32_t)(n0 >> 2), 0u, plo, phi, a.key0, a.key1);
                R z[4];
                Math<R>::box_muller(w.x, w.y, sdt, z[0], z[1]);
                Math<R>::box_muller(w.z, w.w, sdt, z[2], z[3]);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int n = n0 + r;
                    if (n < N) {
                        const R *trow = tuse + 2 * (n - ws) * I;
                        const Look<R> L = lookup_state<R, AXIS, EX>(y, trow, inv_du, a_off, inv_spot, amax, spot);
                        if (EX) y = fma(L.s * y, z[r], y);
                        else y = fma(L.s, fma(-hdt, L.s, z[r]), y);
                        if (STORE && active) ((R *)a.states)[(size_t)n * a.P + p] = y;
                        if (n + 1 == next_tap) {
                            fwd_payoffs<R, EX>(a, tap, y, active, wpart, wave, lane);
                            ++tap;
                            next_tap = tap < a.n_taps ? a.tap_step[tap] : -1;
                        }
                    }
                }
                if (pending) {
                    stg.commit(a, tnext);
                    pending = false;
                }
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < 2 * a.n_opt; e += blockDim.x) {
        double acc = 0.0;
        for (int v = 0; v < wpb; ++v) acc += wpart[v * 2 * a.n_opt + e];
        a.part[(size_t)blockIdx.x * a.Q + e] = acc;
    }
}

// --------------------------------------------------------------------------
// Reverse kernel over stored states.  c_n = dy_{n+1}/dsigma_n = -sigma_n dt +
// sqrt(dt) Z_n is recovered from the stored states as (y_{n+1} - y_n)/sigma_n
// - sigma_n dt / 2, so no random numbers are drawn again.  Steps run in groups
// of four: the four lookups first (they do not depend on lambda, so their LDS
// reads overlap), then the lambda recursion and the histogram scatter.  Table
// windows run last to first; the histogram is folded at histogram-window
// boundaries and at the end of every tile.
// --------------------------------------------------------------------------
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

// EX: the Euler step on X (stored planes hold X): c_n = (X_{n+1} - X_n) / sigma_n and
// d X_{n+1} / d X_n = 1 + c_n (sigma_n / X_n + d sigma / d X).
template <typename R, int AXIS, bool MAGIC, bool EX>
__global__ void __launch_bounds__(adjoint_max_block(sizeof(R))) k_rev(Args a) {
    typedef typename Math<R>::Acc Acc;
    extern __shared__ __align__(16) unsigned char smem[];
    const int wpb = blockDim.x >> 6, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int I = a.I, J = a.J, N = a.N, W = a.W, WH = a.WH, G = I * J, nW = (N + W - 1) / W;
    const Lds lay = lds_layout(REV_STORED, sizeof(R), sizeof(Acc), I, J, a.n_opt, wpb, W, WH, a.K, a.CH);
    double *g64 = (double *)(smem + lay.g64);
    double *wlam = (double *)(smem + lay.wlam);
    R *tuse = (R *)(smem + lay.tab), *tnext = tuse + 2 * W * I;
    Acc *H = (Acc *)(smem + lay.hist);
    int *list = (int *)(smem + lay.live);   // live paths of a chunk, as tile-in-chunk * block + lane
    int *wcnt = list + a.CH * blockDim.x;   // per-wave live counts
    for (int e = tid; e < G; e += blockDim.x) g64[e] = 0.0;
    for (int e = tid; e < wpb; e += blockDim.x) wlam[e] = 0.0;
    for (int e = tid; e < WH * a.K * (I + 1); e += blockDim.x) H[e] = 0;

    const double qmax = fixed_point_qmax(sizeof(R) == 8 ? 64 : 32, blockDim.x, a.K, a.P);
    const int F = fixed_point_bits(a, qmax, Math<R>::FMAX);
    const R qm = (R)qmax;
    constexpr bool magic = MAGIC;   // the launcher chose it: qmax <= Math<R>::MAGIC_MAX
    const double scd = ldexp(1.0, F), inv_sc = ldexp(1.0, -F);
    const R hdt = (R)(0.5 * a.dt), inv_du = (R)a.inv_du, a_off = (R)a.a_off;
    const R inv_spot = (R)(1.0 / a.spot);
    const R spot = (R)a.spot, amax = (R)(I - 1);
    const R y0 = EX ? spot : (R)0;   // the state at step 0
    const int K = a.K, KI1 = K * (I + 1), B = gridDim.x, T = blockDim.x;
    Acc *Hl = H + (tid % K) * (I + 1);   // this lane's copy of a histogram row
    const R *Y = (const R *)a.states;
    const size_t P = (size_t)a.P;
    const int btop = (N - 1) / RB;   // the first (top) block of steps the sweep runs
    TabStage<R> stg;
    int wcur = -1;
    if ((int)blockIdx.x < a.n_tiles) {   // last window, into the buffer entered first
        stg.issue(a, (nW - 1) * W, N - (nW - 1) * W);
        stg.commit(a, tnext);
    }

    // The block's path tiles b, b + B, ... are taken CH at a time: their live paths
    // (all paths when a.dense is set) are listed in path order, then swept in passes
    // of T lanes; each pass is folded like a tile.
    for (int c0 = blockIdx.x; c0 < a.n_tiles; c0 += a.CH * B) {
        __syncthreads();   // the previous chunk's list is no longer read
        int n_live = 0;
        for (int k = 0; k < a.CH; ++k) {
            const int t = c0 + k * B;
            if (t >= a.n_tiles) break;
            const long long p = (long long)t * T + tid;
            const bool live = p < a.P && (a.dense || path_live<R, EX>(a, Y, P, (size_t)p));
            const unsigned long long m = __ballot(live);
            if (lane == 0) wcnt[wave] = __popcll(m);
            __syncthreads();
            int off = n_live, tot = 0;
            for (int v = 0; v < wpb; ++v) {
                const int c = wcnt[v];
                off += v < wave ? c : 0;
                tot += c;
            }
            if (live) list[off + __popcll(m & ((1ull << lane) - 1))] = k * T + tid;
            n_live += tot;
            __syncthreads();
        }
        for (int base = 0; base < n_live; base += T) {
            const bool more = base + T < n_live || c0 + a.CH * B < a.n_tiles;
            const bool active = base + tid < n_live;
            const int e = list[active ? base + tid : 0];   // inactive lanes read a live path
            const int ek = e / T;
            const size_t pc = (size_t)(c0 + ek * B) * T + (size_t)(e - ek * T);
            R lam = 0;   // the adjoint of y, times 2^F
            R y_next = Y[(size_t)(N - 1) * P + pc];
            int tap = a.n_taps - 1, cur_tap = tap >= 0 ? a.tap_step[tap] : -1;
            int hcur = (N - 1) / WH;
            // States by blocks of RB steps (RB/4 groups of four): cur[k] = y_{b RB + k}
            // (plane b RB + k - 1; y_0 = 0 is set where it is used).  The next block's
            // states are loaded at the start of a block, so loads have a whole block
            // of compute to arrive.
            R cur[RB], nxt[RB];
            const R *Yp = Y + pc;   // this path's state at plane 0
#pragma unroll
            for (int k = 0; k < RB; ++k) cur[k] = Yp[(size_t)min(max(btop * RB + k - 1, 0), N - 1) * P];
            // Blocks below the top one read planes b RB - 1 .. b RB + RB - 2, which are
            // below N - 1, and only plane -1 (block 0) needs the clamp; one pointer walks
            // the planes, so no address is recomputed per load.  With fewer than RB
            // steps the only block is the top one and the loads here are not used: the
            // walk then stays on plane 0.
            const size_t Ps = N >= RB ? P : 0;
            auto load_block = [&](int b, R(&y)[RB]) {
                const R *q = Yp + (size_t)max(b * RB - 1, 0) * Ps;
                y[0] = *q;
                q += b > 0 ? Ps : 0;
#pragma unroll
                for (int k = 1; k < RB; ++k) {
                    y[k] = *q;
                    q += Ps;
                }
            };
            for (int wi = nW - 1; wi >= 0; --wi) {
                const int ws = wi * W, we = min(N, ws + W);
                bool pending = false;
                if (wi != wcur) {
                    __syncthreads();   // window wi is in tnext; tuse and the histogram are idle
                    const int hi = ws / WH;
                    if (hi != hcur) {
                        fold<R>(a, H, g64, hcur * WH, min(WH, N - hcur * WH), inv_sc);
                        hcur = hi;
                    }
                    R *t = tuse;
                    tuse = tnext;
                    tnext = t;
                    wcur = wi;
                    const int nx = wi > 0 ? wi - 1 : (more ? nW - 1 : -1);
                    if (nx >= 0 && nW > 1) {
                        stg.issue(a, nx * W, min(W, N - nx * W));
                        pending = true;
                    }
                }
                const int hbase = hcur * WH;
                // one group of four steps n0 .. n0+3 whose states are y[0..3]
                auto group = [&](int n0, const R *y, auto full_tag) {
                    constexpr bool FULL = decltype(full_tag)::value;
                    const int wn0 = n0 - ws, hn0 = n0 - hbase;
                    Acc *hrow = Hl + (hn0 + 3) * KI1;   // this lane's row of step n0 + 3
                    Look<R> L[4];
                    R cc[4], dsd[4], yup[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        if (FULL || n0 + r < N) {
                            const R yr = (n0 + r == 0) ? y0 : y[r];
                            yup[r] = (r == 3 || (!FULL && n0 + r + 1 >= N)) ? y_next : y[r + 1];
                            L[r] = lookup_state<R, AXIS, EX>(yr, tuse + 2 * (wn0 + r) * I, inv_du, a_off,
                                                             inv_spot, amax, spot);
                            if (EX) {
                                cc[r] = (yup[r] - yr) * Math<R>::rcp(L[r].s);
                                // sigma / X + d sigma / d X; on a log axis d sigma / d X = (d / du) / X
                                R d = L[r].in ? L[r].d * inv_du : (R)0;
                                if (AXIS == 0) d *= yr;
                                dsd[r] = (L[r].s + d) * Math<R>::rcp(yr);
                            } else {
                                cc[r] = (yup[r] - yr) * Math<R>::rcp(L[r].s) - hdt * L[r].s;
                                R d = L[r].in ? L[r].d * inv_du : (R)0;
                                if (AXIS == 0) d *= L[r].S;
                                dsd[r] = d;
                            }
                        }
                    }
#pragma unroll
                    for (int r = 3; r >= 0; --r) {
                        const int n = n0 + r;
                        if (FULL || n < N) {
                            if (n + 1 == cur_tap) {
                                lam = rev_seeds<R, EX>(a, tap, yup[r], lam, scd);
                                if (!active) lam = 0;
                                --tap;
                                cur_tap = tap >= 0 ? a.tap_step[tap] : -1;
                            }
                            const R x = lam * cc[r];   // lam carries 2^F: x is the fixed-point term
                            lam = fma(x, dsd[r], lam);
                            scatter<R>(a, hrow, g64, n, L[r], x, qm, magic, inv_sc);
                        }
                        hrow -= KI1;
                    }
                    if (FULL || n0 < N) y_next = (n0 == 0) ? y0 : y[0];
                };
                auto block = [&](int b, auto full_tag) {
                    load_block(max(b - 1, 0), nxt);
#pragma unroll
                    for (int q = RB / 4 - 1; q >= 0; --q) group(b * RB + 4 * q, cur + 4 * q, full_tag);
#pragma unroll
                    for (int k = 0; k < RB; ++k) cur[k] = nxt[k];
                };
                // The window's first block runs on its own (the horizon's top block may
                // be partial), then the next table window is committed, then the rest.
                const int blo = ws / RB;
                int b = (we - 1) / RB;
                if (wi == nW - 1) block(b, std::false_type{});
                else block(b, std::true_type{});
                if (pending) stg.commit(a, tnext);
                for (--b; b >= blo; --b) block(b, std::true_type{});
            }
            __syncthreads();
            fold<R>(a, H, g64, hcur * WH, min(WH, N - hcur * WH), inv_sc);
            // the adjoint of y_0 = ln(X_0 / spot): with EX, lambda is that of X_0 = spot
            const double l0 = wave_sum(active ? (double)lam * inv_sc * (EX ? a.spot : 1.0) : 0.0);
            if (lane == 0) wlam[wave] += l0;
        }
    }
    __syncthreads();
    double *out = a.part + (size_t)blockIdx.x * a.Q;
    if (tid == 0) {
        double acc = 0.0;
        for (int v = 0; v < wpb; ++v) acc += wlam[v];
        out[2 * a.n_opt] = acc;
    }
    for (int e = tid; e < G; e += blockDim.x) out[2 * a.n_opt + 1 + e] = g64[e];
}

// --------------------------------------------------------------------------
// Fused kernel with checkpoints: per path tile, a forward pass that keeps the
// state at the start of every SEG-step segment and the payoff sums, then the
// reverse pass segment by segment (last first): the segment is re-simulated
// from its checkpoint with the same Philox counters, its states and
// c_n = -sigma_n dt + sqrt(dt) Z_n held in registers, and swept backwards.
// Checkpoints live in per-block slots reused by every tile of the block.  The
// LDS table holds one segment; consecutive uses of the same segment (the last
// one forward then backward, the first one backward then forward for the next
// tile) share its copy.  The block's tiles b, b + B, ... are taken CH at a time:
// each is run forward into its own checkpoint slots, then only their live paths (an
// option with a nonzero cotangent in the money at its maturity, as in the stored
// reverse kernel; every path with a.dense) are swept back, listed in path order and
// taken in passes of blockDim lanes, so waves beyond the list skip the re-simulation
// and the sweep.  A lane then reads another lane's checkpoints, which the block
// barrier makes visible.
// EX: the Euler step on X; the checkpoints hold X, and the
// re-simulated segment keeps c_n = X_n sqrt(dt) Z_n (the derivative of X_{n+1} in
// sigma_n) with d X_{n+1} / d X_n = 1 + c_n (sigma_n / X_n + d sigma / d X).
// --------------------------------------------------------------------------
template <typename R, int AXIS, int SEG, bool MAGIC, bool EX>
__global__ void __launch_bounds__(adjoint_max_block(sizeof(R))) k_fused(Args a) {
    typedef typename Math<R>::Acc Acc;
    extern __shared__ __align__(16) unsigned char smem[];
    const int wpb = blockDim.x >> 6, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int I = a.I, J = a.J, N = a.N, G = I * J, WH = a.WH;
    const Lds lay = lds_layout(FUSED_CKPT, sizeof(R), sizeof(Acc), I, J, a.n_opt, wpb, SEG, WH, a.K, a.CH);
    double *g64 = (double *)(smem + lay.g64);
    double *wpart = (double *)(smem + lay.wpart);
    double *wlam = (double *)(smem + lay.wlam);
    R *tab = (R *)(smem + lay.tab);
    Acc *H = (Acc *)(smem + lay.hist);
    const int CH = a.CH, T = blockDim.x, B = gridDim.x;
    int *list = (int *)(smem + lay.live);   // live paths of a chunk, as tile-in-chunk * T + lane
    int *wcnt = list + CH * T;              // per-wave live counts
    R *yfin = (R *)(smem + lay.yfin);       // state at the last step, per path of the chunk
    for (int e = tid; e < G; e += blockDim.x) g64[e] = 0.0;
    for (int e = tid; e < wpb; e += blockDim.x) wlam[e] = 0.0;
    for (int e = tid; e < wpb * a.n_opt * 2; e += blockDim.x) wpart[e] = 0.0;
    for (int e = tid; e < WH * a.K * (I + 1); e += blockDim.x) H[e] = 0;

    const double qmax = fixed_point_qmax(sizeof(R) == 8 ? 64 : 32, blockDim.x, a.K, a.P);
    const int F = fixed_point_bits(a, qmax, Math<R>::FMAX);
    const R qm = (R)qmax;
    constexpr bool magic = MAGIC;   // the launcher chose it: qmax <= Math<R>::MAGIC_MAX
    const double scd = ldexp(1.0, F), inv_sc = ldexp(1.0, -F);
    const R sdt = (R)a.sqrt_dt, hdt = (R)(0.5 * a.dt), inv_du = (R)a.inv_du, a_off = (R)a.a_off;
    const R spot = (R)a.spot, amax = (R)(I - 1), inv_spot = (R)(1.0 / a.spot);
    const int n_seg = (N + SEG - 1) / SEG, KI1 = a.K * (I + 1);
    Acc *Hl = H + (tid % a.K) * (I + 1);   // this lane's copy of a histogram row
    R *CK = (R *)a.ckpt;
    const size_t slot_stride = (size_t)gridDim.x * blockDim.x;
    const size_t slot = (size_t)blockIdx.x * blockDim.x + tid;
    TabStage<R> stg;
    int tcur = -1;   // segment whose table is in LDS

    for (int c0 = blockIdx.x; c0 < a.n_tiles; c0 += CH * B) {
      int n_live = 0;
      for (int kt = 0; kt < CH && c0 + kt * B < a.n_tiles; ++kt) {
        const int tile = c0 + kt * B;
        const long long p = (long long)tile * T + tid;
        const bool active = p < a.P;
        const uint32_t plo = (uint32_t)p, phi = (uint32_t)((unsigned long long)p >> 32);
        // ---- forward: checkpoints (slot set kt) and payoff sums
        R y = EX ? spot : (R)0;
        bool lv = false;
        int tap = 0, next_tap = a.n_taps > 0 ? a.tap_step[0] : -1;
        for (int sg = 0; sg < n_seg; ++sg) {
            const int na = sg * SEG, nw = min(SEG, N - na);
            CK[(size_t)(sg * CH + kt) * slot_stride + slot] = y;
            if (sg != tcur) {
                __syncthreads();
                stg.issue(a, na, nw);
                stg.commit(a, tab);
                __syncthreads();
                tcur = sg;
            }
#pragma unroll
            for (int q4 = 0; q4 < SEG / 4; ++q4) {
                const int n0 = na + 4 * q4;
                if (n0 < N) {
                    const Words w = philox10((uint32_t)(n0 >> 2), 0u, plo, phi, a.key0, a.key1);
                    R z[4];
                    Math<R>::box_muller(w.x, w.y, sdt, z[0], z[1]);
                    Math<R>::box_muller(w.z, w.w, sdt, z[2], z[3]);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int n = n0 + r;
                        if (n < N) {
                            const Look<R> L = lookup_state<R, AXIS, EX>(y, tab + 2 * (4 * q4 + r) * I,
                                                                        inv_du, a_off, inv_spot, amax, spot);
                            if (EX) y = fma(L.s * y, z[r], y);
                            else y = fma(L.s, fma(-hdt, L.s, z[r]), y);
                            if (n + 1 == next_tap) {
                                fwd_payoffs<R, EX>(a, tap, y, active, wpart, wave, lane);
                                if (!lv) lv = tap_live<R, EX>(a, tap, y);
                                ++tap;
                                next_tap = tap < a.n_taps ? a.tap_step[tap] : -1;
                            }
                        }
                    }
                }
            }
        }
        // ---- list the tile's live paths after those of the chunk's earlier tiles
        const bool live = active && (a.dense || lv);
        const unsigned long long m = __ballot(live);
        if (lane == 0) wcnt[wave] = __popcll(m);
        yfin[kt * T + tid] = y;
        __syncthreads();   // also makes every lane's checkpoints visible to the block
        int woff = n_live, tot = 0;
        for (int v = 0; v < wpb; ++v) {
            const int c = wcnt[v];
            woff += v < wave ? c : 0;
            tot += c;
        }
        if (live) list[woff + __popcll(m & ((1ull << lane) - 1))] = kt * T + tid;
        n_live += tot;
        __syncthreads();
      }
      // ---- passes of T listed paths: lane t takes list entry base + t
      for (int base = 0; base < n_live; base += T) {
        const bool on = base + tid < n_live;
        const bool wave_on = base + wave * 64 < n_live;
        const int e = list[on ? base + tid : base];   // lanes past the list repeat a listed path
        const int ek = e / T, src = e - ek * T;
        const long long ps = (long long)(c0 + ek * B) * T + src;
        const uint32_t slo = (uint32_t)ps, shi = (uint32_t)((unsigned long long)ps >> 32);
        const size_t sslot = (size_t)ek * slot_stride + (size_t)blockIdx.x * T + src;
        // ---- reverse, segment by segment (lam is the adjoint of y times 2^F)
        R lam = 0, y_next = yfin[e];
        int rtap = a.n_taps - 1, cur_tap = rtap >= 0 ? a.tap_step[rtap] : -1;
        int hcur = ((n_seg - 1) * SEG) / WH;
        for (int sg = n_seg - 1; sg >= 0; --sg) {
            const int na = sg * SEG, nw = min(SEG, N - na);
            const int hi = na / WH;
            if (hi != hcur || sg != tcur) __syncthreads();
            if (hi != hcur) {
                fold<R>(a, H, g64, hcur * WH, min(WH, N - hcur * WH), inv_sc);
                hcur = hi;
            }
            if (sg != tcur) {
                stg.issue(a, na, nw);
                stg.commit(a, tab);
                __syncthreads();
                tcur = sg;
            }
            if (!wave_on) continue;   // no live path in this wave (the barriers above are the block's)
            const int hb = na - hcur * WH;   // histogram row of the segment's first step
            R ys[SEG], cs[SEG];
            R yy = CK[(size_t)sg * CH * slot_stride + sslot];
#pragma unroll
            for (int q4 = 0; q4 < SEG / 4; ++q4) {
                const int n0 = na + 4 * q4;
                if (n0 < N) {
                    const Words w = philox10((uint32_t)(n0 >> 2), 0u, slo, shi, a.key0, a.key1);
                    R z[4];
                    Math<R>::box_muller(w.x, w.y, sdt, z[0], z[1]);
                    Math<R>::box_muller(w.z, w.w, sdt, z[2], z[3]);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int k = 4 * q4 + r;
                        if (n0 + r < N) {
                            const Look<R> L = lookup_state<R, AXIS, EX>(yy, tab + 2 * k * I, inv_du, a_off,
                                                                        inv_spot, amax, spot);
                            ys[k] = yy;
                            // the forward's own arithmetic, so the re-simulated states (and
                            // with them the seed tests) are the forward's bit for bit
                            if (EX) {
                                cs[k] = yy * z[r];
                                yy = fma(L.s * yy, z[r], yy);
                            } else {
                                cs[k] = fma((R)-2 * hdt, L.s, z[r]);
                                yy = fma(L.s, fma(-hdt, L.s, z[r]), yy);
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int q4 = SEG / 4 - 1; q4 >= 0; --q4) {
                // lookups of four steps first (independent of lambda), then the chain
                Look<R> L[4];
                R dsd[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = 4 * q4 + r;
                    if (na + k < N) {
                        L[r] = lookup_state<R, AXIS, EX>(ys[k], tab + 2 * k * I, inv_du, a_off, inv_spot,
                                                         amax, spot);
                        R d = L[r].in ? L[r].d * inv_du : (R)0;
                        if (AXIS == 0) d *= L[r].S;
                        // EX: sigma / X + d sigma / d X (on a log axis d sigma / d X = (d / du) / X)
                        dsd[r] = EX ? (L[r].s + d) * Math<R>::rcp(ys[k]) : d;
                    }
                }
#pragma unroll
                for (int r = 3; r >= 0; --r) {
                    const int k = 4 * q4 + r;
                    const int n = na + k;
                    if (n < N) {
                        if (n + 1 == cur_tap) {
                            lam = rev_seeds<R, EX>(a, rtap, y_next, lam, scd);
                            if (!on) lam = 0;
                            --rtap;
                            cur_tap = rtap >= 0 ? a.tap_step[rtap] : -1;
                        }
                        const R x = lam * cs[k];   // lam carries 2^F: x is the fixed-point term
                        lam = fma(x, dsd[r], lam);
                        scatter<R>(a, Hl + (hb + k) * KI1, g64, n, L[r], x, qm, magic, inv_sc);
                        y_next = ys[k];
                    }
                }
            }
        }
        __syncthreads();
        fold<R>(a, H, g64, hcur * WH, min(WH, N - hcur * WH), inv_sc);
        // the adjoint of y_0 = ln(X_0 / spot): with EX, lambda is that of X_0 = spot
        const double l0 = wave_sum(on ? (double)lam * inv_sc * (EX ? a.spot : 1.0) : 0.0);
        if (lane == 0) wlam[wave] += l0;
      }
    }
    __syncthreads();
    double *out = a.part + (size_t)blockIdx.x * a.Q;
    for (int e = tid; e < 2 * a.n_opt; e += blockDim.x) {
        double acc = 0.0;
        for (int v = 0; v < wpb; ++v) acc += wpart[v * 2 * a.n_opt + e];
        out[e] = acc;
    }
    if (tid == 0) {
        double acc = 0.0;
        for (int v = 0; v < wpb; ++v) acc += wlam[v];
        out[2 * a.n_opt] = acc;
    }
    for (int e = tid; e < G; e += blockDim.x) out[2 * a.n_opt + 1 + e] = g64[e];
}

// --------------------------------------------------------------------------
// Fixed-order merge of the block records: one wavefront per output; lane l takes
// the compensated sum of records l, l + 64, l + 128, ... in order, then a fixed
// butterfly combines the lanes.  The association is the same on every run,
// whatever order the blocks finished in.
// --------------------------------------------------------------------------
__device__ __forceinline__ void neumaier(double &sum, double &comp, double x) {
    const double t = sum + x;
    if (fabs(sum) >= fabs(x))
        comp += (sum - t) + x;
    else
        comp += (x - t) + sum;
    sum = t;
}

__device__ __forceinline__ double record_sum(const double *part, int Q, int q, int B, int lane) {
    double sum = 0.0, comp = 0.0;
    int b = lane;
    for (; b + 64 * 7 < B; b += 64 * 8) {   // eight loads in flight per lane
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = part[(size_t)(b + 64 * k) * Q + q];
#pragma unroll
        for (int k = 0; k < 8; ++k) neumaier(sum, comp, v[k]);
    }
    for (; b < B; b += 64) neumaier(sum, comp, part[(size_t)b * Q + q]);
    return wave_sum(sum + comp);
}

// Output t (one per wavefront): option t's price and standard error (t < n_opt),
// delta (t = n_opt), grid node t - n_opt - 1.  Payoff entries sum the first B_pay
// records, the others the first B_grad.
__global__ void k_merge(const double *part, int B_pay, int B_grad, int Q, int n_opt, int G,
                        const int *opt_orig, long long P, double spot, double *price,
                        double *stderr_, double *grad, double *delta) {
    const int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    const double Pd = (double)P;
    if (t < n_opt) {
        const double s1 = record_sum(part, Q, 2 * t, B_pay, lane);
        const double s2 = record_sum(part, Q, 2 * t + 1, B_pay, lane);
        if (lane == 0) {
            const int o = opt_orig[t];
            price[o] = s1 / Pd;
            const double var = (s2 - s1 * s1 / Pd) / (Pd - 1.0);
            stderr_[o] = sqrt(fmax(var, 0.0) / Pd);
        }
    } else if (t == n_opt) {
        if (delta) {
            const double s = record_sum(part, Q, 2 * n_opt, B_grad, lane);
            if (lane == 0) *delta = s / Pd / spot;
        }
    } else if (grad && t < n_opt + 1 + G) {
        const int q = t - n_opt - 1;
        const double s = record_sum(part, Q, 2 * n_opt + 1 + q, B_grad, lane);
        if (lane == 0) grad[q] = s / Pd;
    }
}

// --------------------------------------------------------------------------
// Test-support kernels
// --------------------------------------------------------------------------
// --------------------------------------------------------------------------
// Bump-and-reprice (the finite-difference estimator the adjoint replaces, Sec. III):
// surfaces 2s and 2s+1 of a batch are sigma with node m0 + s moved by +eps/2 and
// -eps/2; after they are priced on the same paths, the node's derivative is the
// weighted price difference over eps.
// --------------------------------------------------------------------------
__global__ void k_bump(const double *sigma, int G, int m0, int mc, double eps, double *out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2LL * mc * G) return;
    const int s = (int)(e / G), g = (int)(e - (long long)s * G);
    const double v = sigma[g];
    out[e] = g == m0 + s / 2 ? v + ((s & 1) ? -0.5 * eps : 0.5 * eps) : v;
}

__global__ void k_fd(const double *prices, int n_opt, const double *weight, int m0, int mc, double eps,
                     double *grad) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= mc) return;
    const double *up = prices + (size_t)(2 * s) * n_opt, *dn = up + n_opt;
    double acc = 0.0;
    for (int k = 0; k < n_opt; ++k) acc += weight[k] * (up[k] - dn[k]);
    grad[m0 + s] = acc / eps;
}

__global__ void k_debug_philox(unsigned long long seed, unsigned long long m0, int n_m,
                               unsigned long long p0, long long n_paths, uint32_t *out) {
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= n_paths) return;
    const unsigned long long p = p0 + (unsigned long long)q;
    for (int mi = 0; mi < n_m; ++mi) {
        const unsigned long long m = m0 + (unsigned long long)mi;
        const Words w = philox10((uint32_t)m, (uint32_t)(m >> 32), (uint32_t)p, (uint32_t)(p >> 32),
                                 (uint32_t)seed, (uint32_t)(seed >> 32));
        uint32_t *o = out + ((size_t)q * n_m + mi) * 4;
        o[0] = w.x;
        o[1] = w.y;
        o[2] = w.z;
        o[3] = w.w;
    }
}

template <typename R>
__global__ void k_debug_normals(unsigned long long seed, unsigned long long p0, long long n_paths,
                                int N, R *out) {
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= n_paths) return;
    const unsigned long long p = p0 + (unsigned long long)q;
    for (int g = 0; 4 * g < N; ++g) {
        const Words w = philox10((uint32_t)g, 0u, (uint32_t)p, (uint32_t)(p >> 32), (uint32_t)seed,
                                 (uint32_t)(seed >> 32));
        R z[4];
        Math<R>::box_muller(w.x, w.y, (R)1, z[0], z[1]);
        Math<R>::box_muller(w.z, w.w, (R)1, z[2], z[3]);
        for (int r = 0; r < 4 && 4 * g + r < N; ++r) out[(size_t)q * N + 4 * g + r] = z[r];
    }
}

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

template <typename R, int AXIS, bool EX>
static void fwd_as(const Args &a, bool store, int blocks, int block, size_t lds, hipStream_t st, Ev ev) {
    if (store) LAUNCH((k_fwd<R, AXIS, true, EX>), blocks, block, lds, st, a);
    else LAUNCH((k_fwd<R, AXIS, false, EX>), blocks, block, lds, st, a);
}

template <typename R>
static void fwd_of(const Args &a, bool store, int blocks, int block, hipStream_t st, Ev ev) {
    const size_t lds = lds_of<R>(store ? FWD_STORE : FWD_PRICE, a, block, a.W);
    const bool ex = a.scheme == 1;
    if (a.axis == 0) {
        if (ex) fwd_as<R, 0, true>(a, store, blocks, block, lds, st, ev);
        else fwd_as<R, 0, false>(a, store, blocks, block, lds, st, ev);
    } else {
        if (ex) fwd_as<R, 1, true>(a, store, blocks, block, lds, st, ev);
        else fwd_as<R, 1, false>(a, store, blocks, block, lds, st, ev);
    }
}

hipError_t launch_fwd(const Args &a, int precision, bool store, int blocks, int block, hipStream_t st,
                      Ev ev) {
    if (precision == 64) fwd_of<double>(a, store, blocks, block, st, ev);
    else fwd_of<float>(a, store, blocks, block, st, ev);
    return hipGetLastError();
}

// Whether the adjoint kernels may round fixed-point terms with the magic-constant
// add (the term range fits it); FP64 ranges always do.
static bool use_magic(const Args &a, int precision, int block) {
    const double qmax = fixed_point_qmax(precision, block, a.K, a.P);
    return precision == 64 || qmax <= Math<float>::MAGIC_MAX;
}

template <typename R, bool MAGIC, bool EX>
static void rev_as(const Args &a, int blocks, int block, size_t lds, hipStream_t st, Ev ev) {
    if (a.axis == 0) LAUNCH((k_rev<R, 0, MAGIC, EX>), blocks, block, lds, st, a);
    else LAUNCH((k_rev<R, 1, MAGIC, EX>), blocks, block, lds, st, a);
}

hipError_t launch_rev(const Args &a, int precision, int blocks, int block, hipStream_t st, Ev ev) {
    const bool ex = a.scheme == 1;
    if (precision == 64) {
        const size_t lds = lds_of<double>(REV_STORED, a, block, a.W);
        if (ex) rev_as<double, true, true>(a, blocks, block, lds, st, ev);
        else rev_as<double, true, false>(a, blocks, block, lds, st, ev);
    } else {
        const size_t lds = lds_of<float>(REV_STORED, a, block, a.W);
        const bool m = use_magic(a, precision, block);
        if (m) {
            if (ex) rev_as<float, true, true>(a, blocks, block, lds, st, ev);
            else rev_as<float, true, false>(a, blocks, block, lds, st, ev);
        } else {
            if (ex) rev_as<float, false, true>(a, blocks, block, lds, st, ev);
            else rev_as<float, false, false>(a, blocks, block, lds, st, ev);
        }
    }
    return hipGetLastError();
}

template <typename R, int SEG, bool MAGIC>
static void fused_seg(const Args &a, int blocks, int block, hipStream_t st, Ev ev) {
    const size_t lds = lds_of<R>(FUSED_CKPT, a, block, SEG);
    if (a.scheme == 1) {
        if (a.axis == 0) LAUNCH((k_fused<R, 0, SEG, MAGIC, true>), blocks, block, lds, st, a);
        else LAUNCH((k_fused<R, 1, SEG, MAGIC, true>), blocks, block, lds, st, a);
    } else {
        if (a.axis == 0) LAUNCH((k_fused<R, 0, SEG, MAGIC, false>), blocks, block, lds, st, a);
        else LAUNCH((k_fused<R, 1, SEG, MAGIC, false>), blocks, block, lds, st, a);
    }
}

template <typename R, bool MAGIC>
static void fused_any(const Args &a, int blocks, int block, hipStream_t st, Ev ev) {
    switch (a.seg) {
        case 8: fused_seg<R, 8, MAGIC>(a, blocks, block, st, ev); break;
        case 16: fused_seg<R, 16, MAGIC>(a, blocks, block, st, ev); break;
        default: fused_seg<R, 32, MAGIC>(a, blocks, block, st, ev); break;
    }
}

hipError_t launch_fused_ckpt(const Args &a, int precision, int blocks, int block, hipStream_t st, Ev ev) {
    if (precision == 64) fused_any<double, true>(a, blocks, block, st, ev);
    else if (use_magic(a, precision, block)) fused_any<float, true>(a, blocks, block, st, ev);
    else fused_any<float, false>(a, blocks, block, st, ev);
    return hipGetLastError();
}

hipError_t launch_table(const Args &a, int precision, hipStream_t st, Ev ev) {
    const long long ne = (long long)a.N * a.I;
    const int blocks = (int)((ne + 255) / 256 < 2048 ? (ne + 255) / 256 : 2048);
    if (precision == 64)
        LAUNCH(k_table<double>, blocks, 256, 0, st, a);
    else
        LAUNCH(k_table<float>, blocks, 256, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_merge(const double *part, int B_pay, int B_grad, int Q, int n_opt, int G,
                        const int *opt_orig, long long P, double spot, double *price, double *stderr_,
                        double *grad, double *delta, hipStream_t st, Ev ev) {
    const int T = n_opt + 1 + (grad ? G : 0);   // outputs, one wavefront each
    const dim3 g((T + 3) / 4), b(256);
    if (ev.start || ev.stop)
        hipExtLaunchKernelGGL(k_merge, g, b, 0, st, ev.start, ev.stop, 0, part, B_pay, B_grad, Q, n_opt, G,
                              opt_orig, P, spot, price, stderr_, grad, delta);
    else
        hipLaunchKernelGGL(k_merge, g, b, 0, st, part, B_pay, B_grad, Q, n_opt, G, opt_orig, P, spot, price,
                           stderr_, grad, delta);
    return hipGetLastError();
}

hipError_t launch_bump(const double *sigma, int G, int m0, int mc, double eps, double *out, hipStream_t st) {
    const long long n = 2LL * mc * G;
    hipLaunchKernelGGL(k_bump, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sigma, G, m0, mc, eps, out);
    return hipGetLastError();
}

hipError_t launch_fd(const double *prices, int n_opt, const double *weight, int m0, int mc, double eps,
                     double *grad, hipStream_t st) {
    hipLaunchKernelGGL(k_fd, dim3((mc + 255) / 256), dim3(256), 0, st, prices, n_opt, weight, m0, mc, eps, grad);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Workspace of the allocation-free entry point: one array per GPU, held from the
// module's load until the process ends and shared by every such call on that GPU.
// Host code never names the array itself (its host-side name is a stand-in, not a
// device address): the address is read once per device with hipGetSymbolAddress and
// passed to the kernels like any other buffer.
// --------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void **out) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

hipError_t launch_debug_philox(unsigned long long seed, unsigned long long m0, int n_m,
                               unsigned long long p0, long long n_paths, uint32_t *out,
                               hipStream_t st) {
    const int blocks = (int)((n_paths + 255) / 256);
    hipLaunchKernelGGL(k_debug_philox, dim3(blocks), dim3(256), 0, st, seed, m0, n_m, p0, n_paths, out);
    return hipGetLastError();
}

hipError_t launch_debug_normals(int precision, unsigned long long seed, unsigned long long p0,
                                long long n_paths, int n_steps, double, void *out, hipStream_t st) {
    const int blocks = (int)((n_paths + 255) / 256);
    if (precision == 64)
        hipLaunchKernelGGL((k_debug_normals<double>), dim3(blocks), dim3(256), 0, st, seed, p0, n_paths,
                           n_steps, (double *)out);
    else
        hipLaunchKernelGGL((k_debug_normals<float>), dim3(blocks), dim3(256), 0, st, seed, p0, n_paths,
                           n_steps, (float *)out);
    return hipGetLastError();
}

}  // namespace lvk

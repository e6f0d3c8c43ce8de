// lv_k_opt.hip -- the reverse sweep over stored states that yields every option's own
// vol-grid gradient (and delta) at once: the sensitivities of each price of a book to
// every node (Sec. III, Sec. IV-C), not only of their weighted sum.
//
// One lane per path, as in the stored reverse kernel.  A path's state, lookup, step
// derivative c_n and spot slope do not depend on the option, so they are computed once;
// the lane carries KO adjoints, one per option of the group, each seeded only by its
// own option's payoff (the one-hot cotangent), and scatters each into that option's
// fixed-point LDS histogram, folded at every table window into that option's FP64
// block grid.  Block records are [KO][1 + I J]: per option the sum of its adjoint at
// step 0 and its grid; the fixed-order merge turns them into gradients and deltas.
#include "lv_device.h"

namespace lvk {

// Steps per table window and histogram window of the per-option sweep.
constexpr int OW = 16;

__host__ __device__ inline Lds opt_layout(int rbytes, int I, int J, int wpb, int W, int KO) {
    Lds L{};
    size_t off = 0;
    L.g64 = off;
    off += align16((size_t)KO * I * J * 8);
    L.wlam = off;
    off += align16((size_t)KO * wpb * 8);
    L.tab = off;
    off += align16((size_t)W * I * 2 * rbytes);
    L.hist = off;
    off += align16((size_t)KO * W * (I + 1) * rbytes);   // int32 (FP32) or int64 (FP64) words
    L.total = off;
    return L;
}

size_t lds_bytes_per_option(int precision, int I, int J, int block, int KO) {
    return opt_layout(precision == 64 ? 8 : 4, I, J, block / 64, OW, KO).total;
}

// Fixed-point exponent F of option k (tap order): its terms are rarely above
// 8 e^{-r T_k} max(S0, K_k); 2^F scales them to the histogram's word range qmax.
template <typename R>
__device__ __forceinline__ int option_bits(const Args &a, int k, double qmax) {
    double sz = 0.0;
    if (k < a.n_opt) sz = ldu(a.opt_disc + k) * fmax(a.spot, ldu(a.opt_strike + k));
    const int F = sz > 0.0 ? ilogb(qmax / (8.0 * sz)) : Math<R>::FMAX;
    return F < -30 ? -30 : (F > Math<R>::FMAX ? Math<R>::FMAX : F);
}

// Fold of the KO options' histogram rows of steps [h0, h0 + nh) into their FP64 block
// grids, as fold() does for one histogram (one owner thread per (option, node)), then
// the rows are cleared: two block barriers per window for all the options together.
template <typename R, int KO>
__device__ void fold_options(const Args &a, typename Math<R>::Acc *H, int HS, double *g64, int h0, int nh,
                             int o0, double qmax) {
    typedef typename Math<R>::Acc Acc;
    const int I = a.I, J = a.J, G = I * J, h1 = h0 + nh;
    const int c0 = ldu(a.tj + h0), c1 = ldu(a.tj + h1 - 1);
    const int nn = (c1 - c0 + 2) * I;   // nodes j = c0 .. c1 + 1
    for (int e = threadIdx.x; e < KO * nn; e += blockDim.x) {
        const int s = e / nn, r = e - s * nn;
        const int jj = r / I, i = r - jj * I, j = c0 + jj;
        const Acc *Hs = H + (size_t)s * HS + i;
        double acc = 0.0;
        if (j > c0) {
            const int lo = max(a.cell_lo[j - 1], h0), hi = min(a.cell_lo[j], h1);
            for (int n = lo; n < hi; ++n) acc += a.ta[n] * (double)Hs[(size_t)(n - h0) * (I + 1)];
        }
        if (j <= c1) {
            const int lo = max(a.cell_lo[j], h0), hi = min(a.cell_lo[j + 1], h1);
            for (int n = lo; n < hi; ++n) acc += (1.0 - a.ta[n]) * (double)Hs[(size_t)(n - h0) * (I + 1)];
        }
        g64[s * G + i * J + j] += acc * ldexp(1.0, -option_bits<R>(a, o0 + s, qmax));
    }
    __syncthreads();
    for (int e = threadIdx.x; e < KO * HS; e += blockDim.x) H[e] = 0;
    __syncthreads();
}

// a.o0 .. a.o0 + KO - 1: the options of this group, in maturity (tap) order; n_end: the
// last of their maturity steps, where the sweep starts (every adjoint of the group is
// zero above it).  Steps run in windows of OW: the window's states are loaded together
// at its start (independent loads, in flight while the block stages the window's table),
// then its steps are swept last to first.

template <typename R, int AXIS, int KO, bool RT>
__global__ void __launch_bounds__(adjoint_max_block(sizeof(R))) k_rev_opt(Args a, int o0, int n_end) {
    typedef typename Math<R>::Acc Acc;
    extern __shared__ __align__(16) unsigned char smem[];
    const int wpb = blockDim.x >> 6, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int I = a.I, J = a.J, G = I * J, T = blockDim.x;
    const Lds lay = opt_layout(sizeof(R), I, J, wpb, OW, KO);
    double *g64 = (double *)(smem + lay.g64);
    double *wlam = (double *)(smem + lay.wlam);
    R *tab = (R *)(smem + lay.tab);
    Acc *H = (Acc *)(smem + lay.hist);
    const int HS = OW * (I + 1);   // histogram words per option
    for (int e = tid; e < KO * G; e += T) g64[e] = 0.0;
    for (int e = tid; e < KO * wpb; e += T) wlam[e] = 0.0;
    for (int e = tid; e < KO * HS; e += T) H[e] = 0;

    // per-option fixed-point scale 2^F from the option's own size
    const double qmax = fixed_point_qmax(sizeof(R) == 8 ? 64 : 32, T, 1, a.P);
    const R qm = (R)qmax;
    const bool magic = sizeof(R) == 8 || qmax <= Math<R>::MAGIC_MAX;
    R scr[KO];          // seed scale of each option: e^{-r T_k} 2^F
    double inv_sc[KO];  // 2^-F
#pragma unroll
    for (int s = 0; s < KO; ++s) {
        const int k = o0 + s, F = option_bits<R>(a, k, qmax);
        scr[s] = (R)(k < a.n_opt ? ldu(a.opt_disc + k) * ldexp(1.0, F) : 0.0);
        inv_sc[s] = ldexp(1.0, -F);
    }
    const R hdt = (R)(0.5 * a.dt), inv_du = (R)a.inv_du, a_off = (R)a.a_off, rdt = (R)a.rate_dt;
    const R spot = (R)a.spot, amax = (R)(I - 1);
    const R *Y = (const R *)a.states;
    const size_t P = (size_t)a.P;
    int tap_top = a.n_taps - 1;   // the last maturity at or below n_end
    while (tap_top >= 0 && a.tap_step[tap_top] > n_end) --tap_top;
    const int nW = (n_end + OW - 1) / OW;

    for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const size_t p = (size_t)tile * T + tid;
        const bool active = p < P;
        const R *Yp = Y + (active ? p : 0);   // lanes past the paths follow path 0 with no seed
        R lam[KO];
#pragma unroll
        for (int s = 0; s < KO; ++s) lam[s] = 0;
        R y_next = Yp[(size_t)(n_end - 1) * P];   // y_{n_end}
        int tap = tap_top, cur_tap = tap >= 0 ? a.tap_step[tap] : -1;
        for (int wi = nW - 1; wi >= 0; --wi) {
            const int ws = wi * OW, nw = min(OW, n_end - ws);
            R ys[OW];   // y_{ws + k}; y_0 = 0
#pragma unroll
            for (int k = 0; k < OW; ++k)
                ys[k] = (k < nw && ws + k > 0) ? Yp[(size_t)(ws + k - 1) * P] : (R)0;
            __syncthreads();   // the previous window's table is no longer read
            for (int e = tid; e < nw * I; e += T) {
                const R *src = (const R *)a.gtab + 2 * ((size_t)ws * I + e);
                tab[2 * e] = src[0];
                tab[2 * e + 1] = src[1];
            }
            __syncthreads();
#pragma unroll
            for (int k = OW - 1; k >= 0; --k) {
                if (k < nw) {
                    const int n = ws + k;
                    const R yr = ys[k];
                    const Look<R> L = lookup<R, AXIS>(yr, tab + 2 * k * I, inv_du, a_off, amax, spot);
                    if (n + 1 == cur_tap) {   // seeds of the group's options maturing at step n + 1
                        const R S = spot * Math<R>::ex(y_next);
                        const double Sd = (double)S;
                        const int k0 = ldu(a.tap_first + tap), kc = ldu(a.tap_count + tap);
                        for (int q = 0; q < kc; ++q) {
                            const int o = k0 + q - o0;
                            if (o < 0 || o >= KO) continue;
                            const double K = ldu(a.opt_strike + k0 + q);
                            const bool put = ldu(a.opt_put + k0 + q);
                            const bool itm = put ? Sd < K : Sd > K;
#pragma unroll
                            for (int s = 0; s < KO; ++s)
                                if (s == o && itm && active) lam[s] += scr[s] * (put ? -S : S);
                        }
                        --tap;
                        cur_tap = tap >= 0 ? a.tap_step[tap] : -1;
                    }
                    const R cc = (y_next - yr - (RT ? rdt : (R)0)) * Math<R>::rcp(L.s) - hdt * L.s;
                    R dsd = L.in ? L.d * inv_du : (R)0;
                    if (AXIS == 0) dsd *= L.S;
#pragma unroll
                    for (int s = 0; s < KO; ++s) {
                        const R x = lam[s] * cc;   // lam carries 2^F of its option
                        lam[s] = fma(x, dsd, lam[s]);
                        scatter<R>(a, H + s * HS + k * (I + 1), g64 + s * G, n, L, x, qm, magic, inv_sc[s]);
                    }
                    y_next = yr;
                }
            }
            __syncthreads();
            fold_options<R, KO>(a, H, HS, g64, ws, nw, o0, qmax);
        }
#pragma unroll
        for (int s = 0; s < KO; ++s) {
            const double l0 = wave_sum(active ? (double)lam[s] * inv_sc[s] : 0.0);
            if (lane == 0) wlam[s * wpb + wave] += l0;
        }
    }
    __syncthreads();
    double *out = a.part + (size_t)blockIdx.x * a.Q;
    for (int s = tid; s < KO; s += T) {
        double acc = 0.0;
        for (int v = 0; v < wpb; ++v) acc += wlam[s * wpb + v];
        out[s * (1 + G)] = acc;
    }
    for (int e = tid; e < KO * G; e += T) {
        const int s = e / G, q = e - s * G;
        out[s * (1 + G) + 1 + q] = g64[e];
    }
}

template <typename R, int AXIS, int KO, bool RT>
static void opt_go(const Args &a, int o0, int n_end, int blocks, int block, size_t lds, hipStream_t st) {
    allow_lds(k_rev_opt<R, AXIS, KO, RT>, lds);
    hipLaunchKernelGGL((k_rev_opt<R, AXIS, KO, RT>), dim3(blocks), dim3(block), lds, st, a, o0, n_end);
}

template <typename R, int AXIS, int KO>
static void opt_rt(const Args &a, int o0, int n_end, int blocks, int block, size_t lds, hipStream_t st) {
    if (a.rate_dt != 0.0) opt_go<R, AXIS, KO, true>(a, o0, n_end, blocks, block, lds, st);
    else opt_go<R, AXIS, KO, false>(a, o0, n_end, blocks, block, lds, st);
}

template <typename R, int KO>
static void opt_axis(const Args &a, int o0, int n_end, int blocks, int block, size_t lds, hipStream_t st) {
    if (a.axis == 0) opt_rt<R, 0, KO>(a, o0, n_end, blocks, block, lds, st);
    else opt_rt<R, 1, KO>(a, o0, n_end, blocks, block, lds, st);
}

template <typename R>
static void opt_ko(const Args &a, int o0, int KO, int n_end, int blocks, int block, hipStream_t st) {
    const size_t lds = opt_layout(sizeof(R), a.I, a.J, block / 64, OW, KO).total;
    switch (KO) {
        case 1: opt_axis<R, 1>(a, o0, n_end, blocks, block, lds, st); break;
        case 2: opt_axis<R, 2>(a, o0, n_end, blocks, block, lds, st); break;
        case 4: opt_axis<R, 4>(a, o0, n_end, blocks, block, lds, st); break;
        default: opt_axis<R, 8>(a, o0, n_end, blocks, block, lds, st); break;
    }
}

hipError_t launch_rev_per_option(const Args &a, int precision, int o0, int KO, int n_end, int blocks, int block,
                                 hipStream_t st) {
    if (precision == 64) opt_ko<double>(a, o0, KO, n_end, blocks, block, st);
    else opt_ko<float>(a, o0, KO, n_end, blocks, block, st);
    return hipGetLastError();
}

}  // namespace lvk

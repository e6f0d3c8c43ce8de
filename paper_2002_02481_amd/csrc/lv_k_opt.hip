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

size_t lds_bytes_per_option(int precision, int I, int J, int block, int W, int KO) {
    return opt_layout(precision == 64 ? 8 : 4, I, J, block / 64, W, KO).total;
}

// a.o0 .. a.o0 + KO - 1: the options of this group, in maturity (tap) order.
template <typename R, int AXIS, int KO, bool RT>
__global__ void __launch_bounds__(adjoint_max_block(sizeof(R))) k_rev_opt(Args a, int o0) {
    typedef typename Math<R>::Acc Acc;
    extern __shared__ __align__(16) unsigned char smem[];
    const int wpb = blockDim.x >> 6, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int I = a.I, J = a.J, N = a.N, W = a.W, G = I * J, nW = (N + W - 1) / W, T = blockDim.x;
    const Lds lay = opt_layout(sizeof(R), I, J, wpb, W, KO);
    double *g64 = (double *)(smem + lay.g64);
    double *wlam = (double *)(smem + lay.wlam);
    R *tab = (R *)(smem + lay.tab);
    Acc *H = (Acc *)(smem + lay.hist);
    const int HS = W * (I + 1);   // histogram words per option
    for (int e = tid; e < KO * G; e += T) g64[e] = 0.0;
    for (int e = tid; e < KO * wpb; e += T) wlam[e] = 0.0;
    for (int e = tid; e < KO * HS; e += T) H[e] = 0;

    // per-option fixed-point scale 2^F from the option's own size
    const double qmax = fixed_point_qmax(sizeof(R) == 8 ? 64 : 32, T, 1, a.P);
    const R qm = (R)qmax;
    const bool magic = sizeof(R) == 8 || qmax <= Math<R>::MAGIC_MAX;
    double scd[KO], inv_sc[KO];
#pragma unroll
    for (int s = 0; s < KO; ++s) {
        const int k = o0 + s;
        double sz = 0.0;
        if (k < a.n_opt) sz = ldu(a.opt_disc + k) * fmax(a.spot, ldu(a.opt_strike + k));
        int F = sz > 0.0 ? ilogb(qmax / (8.0 * sz)) : Math<R>::FMAX;
        F = F < -30 ? -30 : (F > Math<R>::FMAX ? Math<R>::FMAX : F);
        scd[s] = ldexp(1.0, F);
        inv_sc[s] = ldexp(1.0, -F);
    }
    const R hdt = (R)(0.5 * a.dt), inv_du = (R)a.inv_du, a_off = (R)a.a_off, rdt = (R)a.rate_dt;
    const R spot = (R)a.spot, amax = (R)(I - 1);
    const R *Y = (const R *)a.states;
    const size_t P = (size_t)a.P;

    for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const size_t p = (size_t)tile * T + tid;
        const bool active = p < P;
        const size_t pc = active ? p : 0;   // lanes past the paths follow path 0 with no seed
        R lam[KO];
#pragma unroll
        for (int s = 0; s < KO; ++s) lam[s] = 0;
        R y_next = Y[(size_t)(N - 1) * P + pc];
        int tap = a.n_taps - 1, cur_tap = tap >= 0 ? a.tap_step[tap] : -1;
        for (int wi = nW - 1; wi >= 0; --wi) {
            const int ws = wi * W, nw = min(W, N - ws);
            __syncthreads();   // the previous window's table is no longer read
            for (int e = tid; e < nw * I; e += T) {
                const R *src = (const R *)a.gtab + 2 * ((size_t)ws * I + e);
                tab[2 * e] = src[0];
                tab[2 * e + 1] = src[1];
            }
            __syncthreads();
            for (int n = ws + nw - 1; n >= ws; --n) {
                const R yr = n == 0 ? (R)0 : Y[(size_t)(n - 1) * P + pc];
                const Look<R> L = lookup<R, AXIS>(yr, tab + 2 * (n - ws) * I, inv_du, a_off, amax, spot);
                if (n + 1 == cur_tap) {   // seeds of the options maturing at step n + 1
                    const R S = spot * Math<R>::ex(y_next);
                    const double Sd = (double)S;
                    const int k0 = ldu(a.tap_first + tap), kc = ldu(a.tap_count + tap);
                    for (int q = 0; q < kc; ++q) {
                        const int k = k0 + q;
                        const double K = ldu(a.opt_strike + k), dk = ldu(a.opt_disc + k);
                        const bool put = ldu(a.opt_put + k);
                        const bool itm = put ? Sd < K : Sd > K;
#pragma unroll
                        for (int s = 0; s < KO; ++s)
                            if (k == o0 + s && itm && active) lam[s] += (R)(dk * scd[s]) * (put ? -S : S);
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
                    scatter<R>(a, H + s * HS + (n - ws) * (I + 1), g64 + s * G, n, L, x, qm, magic, inv_sc[s]);
                }
                y_next = yr;
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < KO; ++s) fold<R>(a, H + s * HS, g64 + s * G, ws, nw, inv_sc[s]);
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
static void opt_go(const Args &a, int o0, int blocks, int block, size_t lds, hipStream_t st) {
    allow_lds(k_rev_opt<R, AXIS, KO, RT>, lds);
    hipLaunchKernelGGL((k_rev_opt<R, AXIS, KO, RT>), dim3(blocks), dim3(block), lds, st, a, o0);
}

template <typename R, int AXIS, int KO>
static void opt_rt(const Args &a, int o0, int blocks, int block, size_t lds, hipStream_t st) {
    if (a.rate_dt != 0.0) opt_go<R, AXIS, KO, true>(a, o0, blocks, block, lds, st);
    else opt_go<R, AXIS, KO, false>(a, o0, blocks, block, lds, st);
}

template <typename R, int KO>
static void opt_axis(const Args &a, int o0, int blocks, int block, size_t lds, hipStream_t st) {
    if (a.axis == 0) opt_rt<R, 0, KO>(a, o0, blocks, block, lds, st);
    else opt_rt<R, 1, KO>(a, o0, blocks, block, lds, st);
}

template <typename R>
static void opt_ko(const Args &a, int o0, int KO, int blocks, int block, hipStream_t st) {
    const size_t lds = opt_layout(sizeof(R), a.I, a.J, block / 64, a.W, KO).total;
    switch (KO) {
        case 1: opt_axis<R, 1>(a, o0, blocks, block, lds, st); break;
        case 2: opt_axis<R, 2>(a, o0, blocks, block, lds, st); break;
        case 4: opt_axis<R, 4>(a, o0, blocks, block, lds, st); break;
        default: opt_axis<R, 8>(a, o0, blocks, block, lds, st); break;
    }
}

hipError_t launch_rev_per_option(const Args &a, int precision, int o0, int KO, int blocks, int block,
                                 hipStream_t st) {
    if (precision == 64) opt_ko<double>(a, o0, KO, blocks, block, st);
    else opt_ko<float>(a, o0, KO, blocks, block, st);
    return hipGetLastError();
}

}  // namespace lvk

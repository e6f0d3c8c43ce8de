// lv_k_fwd.hip -- the per-step vol table and the forward kernel (price only or storing every state).
#include "lv_device.h"

namespace lvk {

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
// Forward kernel: price-only, or storing every state (split / stored adjoint).
// --------------------------------------------------------------------------
// FP32: at most 64 VGPRs, so that 8 waves fit per SIMD (the kernel is issue-bound)
// EX: the Euler step on X itself (the state and the stored planes are X).
// RT: a nonzero rate, whose trend r dt each step adds (to y, or r dt X to X).
template <typename R, int AXIS, bool STORE, bool EX, bool RT>
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
    const R inv_spot = (R)(1.0 / a.spot), rdt = (R)a.rate_dt;
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
        R *sp = (R *)a.states + p;   // this path's stored state, one plane of P per step
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
            const R *trow = tuse;   // the table row of step n, one row of I pairs per step
            for (int n0 = ws; n0 < we; n0 += 4) {
                const Words w = philox10((uint32_t)(n0 >> 2), 0u, plo, phi, a.key0, a.key1);
                R z[4];
                Math<R>::box_muller(w.x, w.y, sdt, z[0], z[1]);
                Math<R>::box_muller(w.z, w.w, sdt, z[2], z[3]);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int n = n0 + r;
                    if (n < N) {
                        const Look<R> L = lookup_state<R, AXIS, EX>(y, trow, inv_du, a_off, inv_spot, amax, spot);
                        trow += 2 * I;
                        y = step<R, EX, RT>(y, L.s, z[r], hdt, rdt);
                        if (STORE && active) *sp = y;
                        if (STORE) sp += a.P;
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

template <typename R, int AXIS, bool EX>
static void fwd_as(const Args &a, bool store, int blocks, int block, size_t lds, hipStream_t st, Ev ev) {
    if (a.rate_dt != 0.0) {
        if (store) LAUNCH((k_fwd<R, AXIS, true, EX, true>), blocks, block, lds, st, a);
        else LAUNCH((k_fwd<R, AXIS, false, EX, true>), blocks, block, lds, st, a);
    } else {
        if (store) LAUNCH((k_fwd<R, AXIS, true, EX, false>), blocks, block, lds, st, a);
        else LAUNCH((k_fwd<R, AXIS, false, EX, false>), blocks, block, lds, st, a);
    }
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

hipError_t launch_table(const Args &a, int precision, hipStream_t st, Ev ev) {
    const long long ne = (long long)a.N * a.I;
    const int blocks = (int)((ne + 255) / 256 < 2048 ? (ne + 255) / 256 : 2048);
    if (precision == 64)
        LAUNCH(k_table<double>, blocks, 256, 0, st, a);
    else
        LAUNCH(k_table<float>, blocks, 256, 0, st, a);
    return hipGetLastError();
}

}  // namespace lvk

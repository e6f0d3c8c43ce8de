// lv_k_rev.hip -- the reverse kernel over stored states.
#include "lv_device.h"

namespace lvk {

// --------------------------------------------------------------------------
// Reverse kernel over stored states.  c_n = dy_{n+1}/dsigma_n = -sigma_n dt +
// sqrt(dt) Z_n is recovered from the stored states as (y_{n+1} - y_n)/sigma_n
// - sigma_n dt / 2, so no random numbers are drawn again.  Steps run in groups
// of four: the four lookups first (they do not depend on lambda, so their LDS
// reads overlap), then the lambda recursion and the histogram scatter.  Table
// windows run last to first; the histogram is folded at histogram-window
// boundaries and at the end of every tile.
// --------------------------------------------------------------------------
// EX: the Euler step on X (stored planes hold X): c_n = (X_{n+1} - X_n) / sigma_n and
// d X_{n+1} / d X_n = 1 + c_n (sigma_n / X_n + d sigma / d X).  RT: the step's trend
// (r dt, or r dt X_n) comes off the state increment first, and on X it adds r dt to
// d X_{n+1} / d X_n.
template <typename R, int AXIS, bool MAGIC, bool EX, bool RT>
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
    const R inv_spot = (R)(1.0 / a.spot), rdt = (R)a.rate_dt;
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
                                cc[r] = (yup[r] - (RT ? fma(yr, rdt, yr) : yr)) * Math<R>::rcp(L[r].s);
                                // sigma / X + d sigma / d X; on a log axis d sigma / d X = (d / du) / X
                                R d = L[r].in ? L[r].d * inv_du : (R)0;
                                if (AXIS == 0) d *= yr;
                                dsd[r] = (L[r].s + d) * Math<R>::rcp(yr);
                            } else {
                                cc[r] = (yup[r] - yr - (RT ? rdt : (R)0)) * Math<R>::rcp(L[r].s) - hdt * L[r].s;
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
                            lam = fma(x, dsd[r], (EX && RT) ? fma(lam, rdt, lam) : lam);
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

template <typename R, bool MAGIC, bool EX, bool RT>
static void rev_rt(const Args &a, int blocks, int block, size_t lds, hipStream_t st, Ev ev) {
    if (a.axis == 0) LAUNCH((k_rev<R, 0, MAGIC, EX, RT>), blocks, block, lds, st, a);
    else LAUNCH((k_rev<R, 1, MAGIC, EX, RT>), blocks, block, lds, st, a);
}

template <typename R, bool MAGIC, bool EX>
static void rev_as(const Args &a, int blocks, int block, size_t lds, hipStream_t st, Ev ev) {
    if (a.rate_dt != 0.0) rev_rt<R, MAGIC, EX, true>(a, blocks, block, lds, st, ev);
    else rev_rt<R, MAGIC, EX, false>(a, blocks, block, lds, st, ev);
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

}  // namespace lvk

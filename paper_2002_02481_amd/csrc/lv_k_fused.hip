// lv_k_fused.hip -- the fused kernel with checkpoints and re-simulated segments.
// Built once per (precision, segment): -DLV_FUSED_PREC=32|64 -DLV_FUSED_SEG=8|16|32.
#include "lv_device.h"

namespace lvk {

// --------------------------------------------------------------------------
// Fused kernel with checkpoints: per path tile, a forward pass that keeps the
// state at the start of every SEG-step segment and the payoff sums, then the
// reverse pass segment by segment (last first): the segment is re-simulated
// from its checkpoint with the same Philox counters, its states (on a linear spot
// axis e^y = S / spot) and c_n = -sigma_n dt + sqrt(dt) Z_n held in registers, and
// swept backwards.
// Checkpoints live in per-block slots reused by every tile of the block.  The
// LDS table holds a window of one, two or four segments (as many as the block's LDS
// allows beside the histogram; fewer copies and barriers); consecutive uses of the
// same window (the last one forward then backward, the first one backward then
// forward for the next tile) share its copy.  The block's tiles b, b + B, ... are run forward one at a
// time, each into the next of CH checkpoint slot sets; only their live paths (an
// option with a nonzero cotangent in the money at its maturity, as in the stored
// reverse kernel; every path with a.dense) are swept back, queued in path order
// across tiles and taken in passes of blockDim lanes, so waves beyond the queue skip
// the re-simulation and the sweep.  A lane then reads another lane's checkpoints,
// which the block barrier makes visible.
// EX: the Euler step on X; the checkpoints hold X, and the
// re-simulated segment keeps c_n = X_n sqrt(dt) Z_n (the derivative of X_{n+1} in
// sigma_n) with d X_{n+1} / d X_n = 1 + c_n (sigma_n / X_n + d sigma / d X) (+ r dt
// with RT, the rate's trend in the step).
// --------------------------------------------------------------------------
template <typename R, int AXIS, int SEG, bool MAGIC, bool EX, bool RT>
__global__ void __launch_bounds__(adjoint_max_block(sizeof(R))) k_fused(Args a) {
    typedef typename Math<R>::Acc Acc;
    extern __shared__ __align__(16) unsigned char smem[];
    const int wpb = blockDim.x >> 6, tid = threadIdx.x, lane = tid & 63;
    // the wave index is the same in every lane of a wave; saying so keeps the branches
    // on it (a wave with no queued path skips the sweep) and all that follows them uniform
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int I = a.I, J = a.J, N = a.N, G = I * J, WH = a.WH;
    const Lds lay = lds_layout(FUSED_CKPT, sizeof(R), sizeof(Acc), I, J, a.n_opt, wpb, a.W, WH, a.K, a.CH);
    double *g64 = (double *)(smem + lay.g64);
    double *wpart = (double *)(smem + lay.wpart);
    double *wlam = (double *)(smem + lay.wlam);
    R *tab = (R *)(smem + lay.tab);
    Acc *H = (Acc *)(smem + lay.hist);
    const int CH = a.CH, T = blockDim.x, B = gridDim.x;
    // Live paths wait in a first-in-first-out queue that runs across the block's path
    // tiles, so that every pass but the last sweeps a full block of them.  A forwarded
    // tile takes the next of CH checkpoint slot sets (and rows of final states) in a
    // ring, and only once every path queued from that slot set's previous tile has been
    // swept; a full ring therefore sends the oldest queued paths through a pass first.
    const int QCAP = CH * T;
    int *qent = (int *)(smem + lay.live);   // queue ring [CH T]: slot set * T + lane
    int *wcnt = qent + QCAP;                // per-wave live counts [16]
    int *tq_tile = wcnt + 16;               // [CH] the tile a slot set holds
    R *yfin = (R *)(smem + lay.yfin);       // state at the last step, per slot set and lane
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
    const R spot = (R)a.spot, amax = (R)(I - 1), inv_spot = (R)(1.0 / a.spot), rdt = (R)a.rate_dt;
    const int n_seg = (N + SEG - 1) / SEG, KI1 = a.K * (I + 1);
    Acc *Hl = H + (tid % a.K) * (I + 1);   // this lane's copy of a histogram row
    R *CK = (R *)a.ckpt;
    const size_t slot_stride = (size_t)gridDim.x * blockDim.x;
    const size_t slot = (size_t)blockIdx.x * blockDim.x + tid;
    TabStage<R> stg;
    // The LDS table holds a window of a.W steps, 2^tsh segments (the planner's choice):
    // segment sg has its rows at (sg mod 2^tsh) SEG in window sg >> tsh.
    const int tsh = __builtin_ctz((unsigned)(a.W / SEG));
    int tcur = -1;   // table window in LDS

    // queue positions (monotone; entry q sits at q mod QCAP), the queue position after
    // each slot set's tile was listed, tiles forwarded, and the oldest forwarded tile
    // that still has queued paths: the same in every thread (kept in scalar registers;
    // CH <= 4, and the slot-set arrays are read and written by unrolled selects)
    long long q_head = 0, q_tail = 0;
    long long tq_end[4] = {0, 0, 0, 0};
    int n_fwd = 0, oldest = 0;
    auto end_of = [&](int k) {
        long long v = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) v = u == k ? tq_end[u] : v;
        return v;
    };
    int t_next = blockIdx.x;
    while (t_next < a.n_tiles || q_tail > q_head) {
      // forward tiles while a slot set is free and the queue holds less than a pass
      while (t_next < a.n_tiles && n_fwd - oldest < CH && q_tail - q_head < T) {
        const int ss = n_fwd % CH, tile = t_next;
        const long long p = (long long)tile * T + tid;
        const bool active = p < a.P;
        const uint32_t plo = (uint32_t)p, phi = (uint32_t)((unsigned long long)p >> 32);
        // ---- forward: checkpoints (slot set ss) and payoff sums
        R y = EX ? spot : (R)0;
        bool lv = false;
        int tap = 0, next_tap = a.n_taps > 0 ? a.tap_step[0] : -1;
        for (int sg = 0; sg < n_seg; ++sg) {
            const int na = sg * SEG, nw = min(SEG, N - na);
            CK[(size_t)(sg * CH + ss) * slot_stride + slot] = y;
            if ((sg >> tsh) != tcur) {
                __syncthreads();
                stg.issue(a, (sg >> tsh) * a.W, min(a.W, N - (sg >> tsh) * a.W));
                stg.commit(a, tab);
                __syncthreads();
                tcur = sg >> tsh;
            }
            const R *tt = tab + (sg & ((1 << tsh) - 1)) * 2 * SEG * I;   // this segment's rows
            // a segment whose steps reach no tap step runs without the per-step tests
            auto fseg = [&](auto notap_tag) {
                constexpr bool NOTAP = decltype(notap_tag)::value;
#pragma unroll
                for (int q4 = 0; q4 < SEG / 4; ++q4) {
                    const int n0 = na + 4 * q4;
                    if (NOTAP || n0 < N) {
                        const Words w = philox10((uint32_t)(n0 >> 2), 0u, plo, phi, a.key0, a.key1);
                        R z[4];
                        Math<R>::box_muller(w.x, w.y, sdt, z[0], z[1]);
                        Math<R>::box_muller(w.z, w.w, sdt, z[2], z[3]);
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int n = n0 + r;
                            if (NOTAP || n < N) {
                                const Look<R> L = lookup_state<R, AXIS, EX>(y, tt + 2 * (4 * q4 + r) * I,
                                                                            inv_du, a_off, inv_spot, amax, spot);
                                y = step<R, EX, RT>(y, L.s, z[r], hdt, rdt);
                                if (!NOTAP && n + 1 == next_tap) {
                                    fwd_payoffs<R, EX>(a, tap, y, active, wpart, wave, lane);
                                    if (!lv) lv = tap_live<R, EX>(a, tap, y);
                                    ++tap;
                                    next_tap = tap < a.n_taps ? a.tap_step[tap] : -1;
                                }
                            }
                        }
                    }
                }
            };
            if (nw == SEG && !(next_tap > na && next_tap <= na + SEG)) fseg(std::true_type{});
            else fseg(std::false_type{});
        }
        // ---- queue the tile's live paths behind those already waiting
        const bool live = active && (a.dense || lv);
        const unsigned long long m = __ballot(live);
        if (lane == 0) wcnt[wave] = __popcll(m);
        yfin[ss * T + tid] = y;
        __syncthreads();   // also makes every lane's checkpoints visible to the block
        long long woff = q_tail;
        int tot = 0;
        for (int v = 0; v < wpb; ++v) {
            const int c = wcnt[v];
            woff += v < wave ? c : 0;
            tot += c;
        }
        tot = __builtin_amdgcn_readfirstlane(tot);   // the same in every lane and wave
        if (live) qent[(woff + __popcll(m & ((1ull << lane) - 1))) % QCAP] = ss * T + tid;
        q_tail += tot;
#pragma unroll
        for (int u = 0; u < 4; ++u) tq_end[u] = u == ss ? q_tail : tq_end[u];
        if (tid == 0) tq_tile[ss] = tile;
        __syncthreads();
        ++n_fwd;
        t_next += B;
        while (oldest < n_fwd && end_of(oldest % CH) <= q_head) ++oldest;   // tiles with nothing queued
      }
      const int pend = (int)(q_tail - q_head);
      // ---- one pass over the oldest min(T, pend) queued paths (a full one unless the ring
      // is full or the tiles have run out): lane t takes entry q_head + t
      if (pend > 0) {
        const int cnt = min(T, pend);
        const bool on = tid < cnt;
        const bool wave_on = wave * 64 < cnt;
        const int e = qent[(q_head + (on ? tid : 0)) % QCAP];   // lanes past the queue repeat its head
        const int ek = e / T, src = e - ek * T;
        const long long ps = (long long)tq_tile[ek] * T + src;
        const uint32_t slo = (uint32_t)ps, shi = (uint32_t)((unsigned long long)ps >> 32);
        const size_t sslot = (size_t)ek * slot_stride + (size_t)blockIdx.x * T + src;
        // ---- reverse, segment by segment (lam is the adjoint of y times 2^F).  On a
        // linear spot axis with log-Euler steps the segment keeps E_n = e^{y_n} = S_n / spot,
        // which the re-simulation computed for its lookups, not y_n: the sweep's lookups,
        // slopes and seeds need only E_n (the same values, so no exp in the sweep).
        constexpr bool HS = AXIS == 0 && !EX;
        const R s_inv_du = spot * inv_du;   // the lookups' 1 / du' (du' = du / spot)
        R lam = 0, y_next = yfin[e];   // e = slot set * T + lane indexes yfin too
        if (HS) y_next = Math<R>::ex(y_next);
        int rtap = a.n_taps - 1, cur_tap = rtap >= 0 ? a.tap_step[rtap] : -1;
        int hcur = ((n_seg - 1) * SEG) / WH;
        for (int sg = n_seg - 1; sg >= 0; --sg) {
            const int na = sg * SEG, nw = min(SEG, N - na);
            const int hi = na / WH;
            if (hi != hcur || (sg >> tsh) != tcur) __syncthreads();
            if (hi != hcur) {
                fold<R>(a, H, g64, hcur * WH, min(WH, N - hcur * WH), inv_sc);
                hcur = hi;
            }
            if ((sg >> tsh) != tcur) {
                stg.issue(a, (sg >> tsh) * a.W, min(a.W, N - (sg >> tsh) * a.W));
                stg.commit(a, tab);
                __syncthreads();
                tcur = sg >> tsh;
            }
            const R *tt = tab + (sg & ((1 << tsh) - 1)) * 2 * SEG * I;   // this segment's rows
            if (!wave_on) continue;   // no live path in this wave (the barriers above are the block's)
            // this lane's histogram row of the segment's last step; the sweep steps it back
            // one row per step
            Acc *hrow = Hl + (na - hcur * WH + SEG - 1) * KI1;
            R ys[SEG], cs[SEG];
            R yy = CK[(size_t)sg * CH * slot_stride + sslot];
            auto resim = [&](auto full_tag) {
                constexpr bool FULL = decltype(full_tag)::value;
#pragma unroll
                for (int q4 = 0; q4 < SEG / 4; ++q4) {
                    const int n0 = na + 4 * q4;
                    if (FULL || n0 < N) {
                        const Words w = philox10((uint32_t)(n0 >> 2), 0u, slo, shi, a.key0, a.key1);
                        R z[4];
                        Math<R>::box_muller(w.x, w.y, sdt, z[0], z[1]);
                        Math<R>::box_muller(w.z, w.w, sdt, z[2], z[3]);
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int k = 4 * q4 + r;
                            if (FULL || n0 + r < N) {
                                const Look<R> L = lookup_state<R, AXIS, EX>(yy, tt + 2 * k * I, inv_du, a_off,
                                                                            inv_spot, amax, spot);
                                ys[k] = HS ? L.E : yy;
                                // the forward's own arithmetic, so the re-simulated states (and
                                // with them the seed tests) are the forward's bit for bit
                                cs[k] = EX ? yy * z[r] : fma((R)-2 * hdt, L.s, z[r]);
                                yy = step<R, EX, RT>(yy, L.s, z[r], hdt, rdt);
                            }
                        }
                    }
                }
            };
            if (nw == SEG) resim(std::true_type{});
            else resim(std::false_type{});
            auto sweep = [&](auto notap_tag) {
                constexpr bool NOTAP = decltype(notap_tag)::value;
#pragma unroll
                for (int q2 = SEG / 2 - 1; q2 >= 0; --q2) {
                    // lookups of two steps first (independent of lambda), then the chain; pairs
                    // rather than fours keep the 16-step segment within 128 VGPRs (no spills)
                    Look<R> L[2];
                    R dsd[2];
#pragma unroll
                    for (int r = 0; r < 2; ++r) {
                        const int k = 2 * q2 + r;
                        if (NOTAP || na + k < N) {
                            if (HS) {
                                // d sigma / d y = (d / du) S = (d / du') E
                                L[r] = lookup_at<R>(ys[k], tt + 2 * k * I, s_inv_du, a_off, amax);
                                dsd[r] = L[r].in ? L[r].d * s_inv_du * ys[k] : (R)0;
                            } else {
                                L[r] = lookup_state<R, AXIS, EX>(ys[k], tt + 2 * k * I, inv_du, a_off,
                                                                 inv_spot, amax, spot);
                                R d = L[r].in ? L[r].d * inv_du : (R)0;
                                if (AXIS == 0) d *= L[r].S;
                                // EX: sigma / X + d sigma / d X (on a log axis d sigma / d X = (d / du) / X)
                                dsd[r] = EX ? (L[r].s + d) * Math<R>::rcp(ys[k]) : d;
                            }
                        }
                    }
#pragma unroll
                    for (int r = 1; r >= 0; --r) {
                        const int k = 2 * q2 + r;
                        const int n = na + k;
                        if (NOTAP || n < N) {
                            if (!NOTAP && n + 1 == cur_tap) {
                                lam = HS ? rev_seeds_at<R, EX>(a, rtap, spot * y_next, lam, scd)
                                         : rev_seeds<R, EX>(a, rtap, y_next, lam, scd);
                                if (!on) lam = 0;
                                --rtap;
                                cur_tap = rtap >= 0 ? a.tap_step[rtap] : -1;
                            }
                            const R x = lam * cs[k];   // lam carries 2^F: x is the fixed-point term
                            lam = fma(x, dsd[r], (EX && RT) ? fma(lam, rdt, lam) : lam);
                            scatter<R, false>(a, hrow, g64, n, L[r], x, qm, magic, inv_sc);
                            y_next = ys[k];
                        }
                        hrow -= KI1;
                    }
                }
            };
            // a segment with no tap step among its steps' successors runs without the tests
            if (nw == SEG && !(cur_tap > na && cur_tap <= na + SEG)) sweep(std::true_type{});
            else sweep(std::false_type{});
        }
        __syncthreads();
        fold<R>(a, H, g64, hcur * WH, min(WH, N - hcur * WH), inv_sc);
        // the adjoint of y_0 = ln(X_0 / spot): with EX, lambda is that of X_0 = spot
        const double l0 = wave_sum(on ? (double)lam * inv_sc * (EX ? a.spot : 1.0) : 0.0);
        if (lane == 0) wlam[wave] += l0;
        q_head += cnt;
        while (oldest < n_fwd && end_of(oldest % CH) <= q_head) ++oldest;
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

template <typename R, int SEG, bool MAGIC, bool RT>
static void fused_rt(const Args &a, int blocks, int block, size_t lds, hipStream_t st, Ev ev) {
    if (a.scheme == 1) {
        if (a.axis == 0) LAUNCH((k_fused<R, 0, SEG, MAGIC, true, RT>), blocks, block, lds, st, a);
        else LAUNCH((k_fused<R, 1, SEG, MAGIC, true, RT>), blocks, block, lds, st, a);
    } else {
        if (a.axis == 0) LAUNCH((k_fused<R, 0, SEG, MAGIC, false, RT>), blocks, block, lds, st, a);
        else LAUNCH((k_fused<R, 1, SEG, MAGIC, false, RT>), blocks, block, lds, st, a);
    }
}

// This file is compiled once per precision and checkpoint segment (LV_FUSED_PREC 32 or
// 64, LV_FUSED_SEG 8, 16 or 32), each object holding that pair's instantiations and
// launcher; launch_fused_ckpt picks among them.
#define LV_FUSED_NAME2(p, s) launch_fused_p##p##_s##s
#define LV_FUSED_NAME(p, s) LV_FUSED_NAME2(p, s)

hipError_t LV_FUSED_NAME(LV_FUSED_PREC, LV_FUSED_SEG)(const Args &a, int blocks, int block, hipStream_t st,
                                                      Ev ev) {
    typedef std::conditional<LV_FUSED_PREC == 64, double, float>::type R;
    constexpr int SEG = LV_FUSED_SEG;
    const size_t lds = lds_of<R>(FUSED_CKPT, a, block, a.W);
    const bool rt = a.rate_dt != 0.0;
    if (LV_FUSED_PREC == 64 || use_magic(a, LV_FUSED_PREC, block)) {
        if (rt) fused_rt<R, SEG, true, true>(a, blocks, block, lds, st, ev);
        else fused_rt<R, SEG, true, false>(a, blocks, block, lds, st, ev);
    } else if (LV_FUSED_PREC == 32) {
        if (rt) fused_rt<R, SEG, false, true>(a, blocks, block, lds, st, ev);
        else fused_rt<R, SEG, false, false>(a, blocks, block, lds, st, ev);
    }
    return hipGetLastError();
}

}  // namespace lvk

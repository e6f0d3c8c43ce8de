"""Pins for the CPU oracle: checks against facts the paper and the mathematics fix.

Each ``pin_*`` takes an :class:`oracle.Oracle` and raises ``AssertionError`` when
the oracle disagrees with the fact.  They are run on the oracle itself
(``test_oracle_pins.py``) and on deliberately broken copies of it
(``test_oracle_mutants.py``), where at least one of them must fail.

What pins what:
  * Philox words          -- rocRAND's Philox4x32-10 (a library routine), on the host
  * uniform map           -- exact integer identity
  * Box-Muller            -- inverse relations per pair, moments, the tail bound
  * interpolation         -- node values, exact reproduction of bilinear fields,
                             flat extrapolation, weights = d sigma / d node
  * flat vol              -- Black-Scholes price and vega (log-Euler is exact in law),
                             the pathwise vega identity per path, column sums
  * term-structure vol    -- Black-Scholes in total variance, column sums
  * put-call parity       -- per-sample identity on the same streams; martingale
  * one and two steps     -- exact prices of the discrete scheme by integration
  * adjoint               -- central finite differences with common random numbers
  * zero buckets          -- nodes no path can reach are exactly zero
  * bfloat16 nodes        -- torch's float32 -> bfloat16 conversion (a library routine),
                             exact ties between neighbours, the two-step rounding
  * a constant rate       -- Black-Scholes with the rate and its vega, discounted
                             put-call parity and martingale, one step of either scheme,
                             bumping with common random numbers
"""
from __future__ import annotations

import math
import os
import shutil
import subprocess
import tempfile

import numpy as np

import workloads as W
from tests import closed_forms as cf

SQRT_TAIL = math.sqrt(-2.0 * math.log(2.0 ** -24))   # largest |Z| the 23-bit uniform allows


def _batch_stats(o, surface, book, n_steps, n_paths, n_batches, seed=0, spot=100.0, scheme=0, rate=0.0):
    """Price and gradient by batch means: mean over batches and the standard error
    of that mean, for the weighted book value."""
    per = n_paths // n_batches
    vals, grads = [], []
    for b in range(n_batches):
        s = o.sums(surface, book, n_steps, seed, [(b * per, (b + 1) * per)], spot=spot, scheme=scheme, rate=rate)
        vals.append(float(np.dot(book.weight, s["sum_pay"])) / per)
        grads.append(s["sum_grad"] / per)
    vals, grads = np.array(vals), np.array(grads)
    se = lambda a: a.std(axis=0, ddof=1) / math.sqrt(n_batches)
    return vals.mean(), se(vals), grads.mean(axis=0), se(grads)


# --------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------
_ROCRAND_SRC = r"""
#include <rocrand/rocrand_kernel.h>
#include <stdio.h>
int main(void){
  unsigned long long seed, sub, off;
  while (scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, sub, off, &st);
    uint4 w = rocrand4(&st);
    printf("%u %u %u %u\n", w.x, w.y, w.z, w.w);
  }
  return 0;
}
"""
_rocrand_exe = None


def rocrand_available() -> bool:
    return shutil.which("hipcc") is not None and os.path.exists("/opt/rocm/include/rocrand")


def rocrand_philox(triples):
    """Words of rocRAND's Philox4x32-10 with (seed, subsequence, offset), run on the host."""
    global _rocrand_exe
    if _rocrand_exe is None:
        d = tempfile.mkdtemp(prefix="lv_rocrand_")
        src = os.path.join(d, "rr.cpp")
        with open(src, "w") as f:
            f.write(_ROCRAND_SRC)
        exe = os.path.join(d, "rr")
        subprocess.run(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", "-w", "-o", exe, src],
                       check=True, capture_output=True)
        _rocrand_exe = exe
    inp = "\n".join(f"{s} {a} {b}" for s, a, b in triples) + "\n"
    out = subprocess.run([_rocrand_exe], input=inp, capture_output=True, text=True, check=True).stdout
    return np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint64)


def philox_cases():
    rng = np.random.default_rng(11)
    cases = [(0, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 0), (2**32 - 1, 2**32 - 1, 2**32 - 1),
             (2**32, 2**32, 2**32), (0xDEADBEEFCAFEF00D, 12345, 678), (7, 2**40 + 3, 2**33 + 9)]
    for _ in range(40):
        cases.append((int(rng.integers(0, 2**63)), int(rng.integers(0, 2**40)),
                      int(rng.integers(0, 2**40))))
    return cases


def pin_philox_rocrand(o):
    """Key = seed, counter = (m, p): rocRAND with subsequence p and offset 4m."""
    cases = philox_cases()
    ref = rocrand_philox([(s, p, 4 * m) for s, m, p in cases])
    got = np.array([o.philox_words(s, m, p) for s, m, p in cases], dtype=np.uint64)
    assert np.array_equal(got, ref), "Philox words differ from rocRAND"


def pin_uniform(o):
    rng = np.random.default_rng(3)
    words = [0, 1, 511, 512, 0x7FFFFFFF, 0x80000000, 0xFFFFFE00, 0xFFFFFFFF] + \
        [int(x) for x in rng.integers(0, 2**32, 200)]
    for w in words:
        u = o.uniform(w)
        assert 0.0 < u < 1.0
        k = u * 2.0 ** 23 - 0.5
        assert k == float(w >> 9), (w, u)
        assert float(np.float32(u)) == u, "uniform must be exact in float32"


def pin_box_muller(o):
    """Each pair of words (w0, w1) maps to (Z_a, Z_b) with Z_a^2 + Z_b^2 = -2 ln u(w0)
    and angle(Z_a, Z_b) = 2 pi u(w1); step 4m+r takes pair r//2, component r%2."""
    seed = 0x1234
    for p in (0, 1, 77, 2**33 + 5):
        for m in (0, 1, 9, 2**32 + 1):
            w = o.philox_words(seed, m, p)
            z = [o.normal(seed, p, 4 * m + r) for r in range(4)]
            for pair in range(2):
                za, zb = z[2 * pair], z[2 * pair + 1]
                ua, ub = o.uniform(int(w[2 * pair])), o.uniform(int(w[2 * pair + 1]))
                assert abs(za * za + zb * zb - (-2.0 * math.log(ua))) <= 1e-12 * (1 - 2 * math.log(ua))
                ang = (math.atan2(zb, za) / (2 * math.pi)) % 1.0
                d = abs(ang - ub)
                assert min(d, 1.0 - d) < 1e-12, (p, m, pair, ang, ub)
    z = o.normals(99, 0, 4096, 256).ravel()          # 2^20 draws
    n = z.size
    assert abs(z.mean()) < 5.0 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
    kurt = np.mean(z ** 4) / np.mean(z ** 2) ** 2
    assert abs(kurt - 3.0) < 5.0 * math.sqrt(24.0 / n)
    assert np.abs(z).max() <= SQRT_TAIL + 1e-12


# --------------------------------------------------------------------------
# interpolation
# --------------------------------------------------------------------------
def pin_interp(o):
    for kind in (W.LIN, W.LOG):
        s = W.tiny_surface(kind, 6, 5, seed=5, t_hi=1.0)
        sa, ta = s.spot_axis, s.time_axis
        xs = np.linspace(math.log(sa.lo), math.log(sa.hi), sa.n) if kind == W.LOG \
            else np.linspace(sa.lo, sa.hi, sa.n)
        Sn = np.exp(xs) if kind == W.LOG else xs
        tn = np.linspace(ta.lo, ta.hi, ta.n)
        # node values
        for i in range(sa.n):
            for j in range(ta.n):
                v = o.interp(s, Sn[i], tn[j])[0]
                assert abs(v - s.sigma[i, j]) <= 1e-13, (kind, i, j, v, s.sigma[i, j])
        # bilinear fields a + b x + c t + d x t are reproduced exactly inside the grid
        a, b, c, d = 0.2, 0.013, -0.05, 0.004
        field = a + b * (xs[:, None] - xs[0]) + c * tn[None, :] + d * (xs[:, None] - xs[0]) * tn[None, :]
        fs = W.Surface(sa, ta, field)
        rng = np.random.default_rng(1)
        for _ in range(200):
            x = rng.uniform(xs[0], xs[-1]); t = rng.uniform(tn[0], tn[-1])
            S = math.exp(x) if kind == W.LOG else x
            val, dsdy, ij, w = o.interp(fs, S, t)
            exact = a + b * (x - xs[0]) + c * t + d * (x - xs[0]) * t
            assert abs(val - exact) < 1e-12, (kind, S, t, val, exact)
            assert abs(w.sum() - 1.0) < 1e-14 and (w >= 0).all()
            # d sigma / d ln S: on a log axis x = ln S, on a linear axis dx/dlnS = S
            ds_dx = b + d * t
            expect = ds_dx * (S if kind == W.LIN else 1.0)
            assert abs(dsdy - expect) < 1e-10 * max(1.0, abs(expect)), (kind, dsdy, expect)
        # flat outside the grid, zero spot slope there
        for S in (sa.lo * 0.5, sa.hi * 2.0):
            v, dsdy, _, _ = o.interp(s, S, 0.3)
            edge = o.interp(s, sa.lo if S < sa.lo else sa.hi, 0.3)[0]
            assert abs(v - edge) < 1e-13 and dsdy == 0.0
        v = o.interp(s, 100.0, 5.0)[0]
        assert abs(v - o.interp(s, 100.0, ta.hi)[0]) < 1e-13
        # weights are d sigma / d node
        S, t = 93.7, 0.61
        base, _, (i0, j0), w = o.interp(s, S, t)
        for (di, dj), wk in zip([(0, 0), (1, 0), (0, 1), (1, 1)], w):
            bumped = s.sigma.copy(); bumped[i0 + di, j0 + dj] += 1e-3
            v2 = o.interp(W.Surface(sa, ta, bumped), S, t)[0]
            assert abs((v2 - base) / 1e-3 - wk) < 1e-9


# --------------------------------------------------------------------------
# flat and term-structure surfaces: Black-Scholes
# --------------------------------------------------------------------------
def pin_flat_black_scholes(o, n_paths=1 << 17):
    s = W.flat_surface(W.small_surface(), 0.2)
    book = W.Book([0, 1, 0], [100.0, 110.0, 80.0], [1.0, 1.0, 1.0], [1.0, 1.0, 1.0])
    r = o.price_and_grad(s, book, n_paths, 52, seed=5)
    ref = [cf.bs_call(100, 100, 0.04), cf.bs_put(100, 110, 0.04), cf.bs_call(100, 80, 0.04)]
    for k in range(3):
        assert abs(r["price"][k] - ref[k]) < 4.0 * r["stderr"][k], (k, r["price"][k], ref[k])
    # the stderr itself matches the payoff sd of the lognormal law
    sd = cf.call_payoff_sd(100, 100, 0.04)
    assert abs(r["stderr"][0] * math.sqrt(n_paths) / sd - 1.0) < 0.03


def pin_flat_pathwise_vega(o):
    """For flat sigma the sum of a path's grid gradient is its pathwise vega:
    y_N = -sigma^2 T/2 + sigma sqrt(dt) sum Z, so d payoff/d sigma =
    S_T 1{S_T>K} (-sigma T + sqrt(dt) sum Z)."""
    s = W.flat_surface(W.small_surface(), 0.2)
    book = W.call(100.0, 1.0)
    dt = 1.0 / 52
    for p in range(40):
        r = o.path(s, book, 52, 3, p)
        ST = 100.0 * math.exp(r["y"][-1])
        expect = (ST if ST > 100.0 else 0.0) * (-0.2 * 1.0 + math.sqrt(dt) * r["z"].sum())
        got = r["grad"].sum()
        assert abs(got - expect) <= 1e-11 * max(1.0, abs(expect)), (p, got, expect)
        # and the final log-spot follows the exact-in-law formula
        yN = -0.5 * 0.04 * 1.0 + 0.2 * math.sqrt(dt) * r["z"].sum()
        assert abs(r["y"][-1] - yN) < 1e-12


def pin_flat_vega_and_columns(o, n_paths=1 << 17, n_batches=32):
    s = W.flat_surface(W.small_surface(), 0.2)
    book = W.call(100.0, 1.0)
    dt = 1.0 / 52
    _, _, g, g_se = _batch_stats(o, s, book, 52, n_paths, n_batches, seed=8)
    vega = cf.bs_vega(100, 100, 0.2, 1.0)
    tot_se = math.sqrt(float((g_se ** 2).sum()))    # loose: ignores covariance sign
    # total: E[sum g] = BS vega
    se_total = _batch_total_se(o, s, book, 52, n_paths, n_batches, seed=8)
    assert abs(g.sum() - vega) < 4.0 * se_total, (g.sum(), vega, se_total)
    # columns: E[sum_i g_ij] = vega (dt/T) sum_n w_j(t_n)
    Wt = cf.time_weights(s.time_axis, 52, dt)
    col_expect = vega * dt / 1.0 * Wt.sum(axis=0)
    col = g.sum(axis=0)
    col_se = _batch_column_se(o, s, book, 52, n_paths, n_batches, seed=8)
    assert np.all(np.abs(col - col_expect) < 4.0 * col_se + 1e-12), (col, col_expect, col_se)
    del tot_se


def _batch_total_se(o, s, book, N, n_paths, n_batches, seed):
    per = n_paths // n_batches
    tot = [o.sums(s, book, N, seed, [(b * per, (b + 1) * per)])["sum_grad"].sum() / per
           for b in range(n_batches)]
    return np.std(tot, ddof=1) / math.sqrt(n_batches)


def _batch_column_se(o, s, book, N, n_paths, n_batches, seed):
    per = n_paths // n_batches
    cols = [o.sums(s, book, N, seed, [(b * per, (b + 1) * per)])["sum_grad"].sum(axis=0) / per
            for b in range(n_batches)]
    return np.std(cols, axis=0, ddof=1) / math.sqrt(n_batches)


def pin_term_structure(o, n_paths=1 << 17, n_batches=32):
    """sigma(S, t) = sigma_j(t): the terminal log-spot is Gaussian with total
    variance V = sum_n s_n^2 dt, so price = BS(V) and
    E[sum_i g_ij] = C'(V) sum_n 2 s_n dt w_j(t_n)."""
    base = W.small_surface()
    rng = np.random.default_rng(4)
    colv = rng.uniform(0.12, 0.35, base.time_axis.n)
    s = W.Surface(base.spot_axis, base.time_axis, np.tile(colv, (base.spot_axis.n, 1)))
    N, T, K = 52, 1.0, 104.0
    dt = T / N
    Wt = cf.time_weights(s.time_axis, N, dt)
    sn = Wt @ colv
    V = float(np.sum(sn ** 2) * dt)
    book = W.call(K, T)
    r = o.price_and_grad(s, book, n_paths, N, seed=12)
    assert abs(r["price"][0] - cf.bs_call(100, K, V)) < 4.0 * r["stderr"][0]
    col_expect = cf.bs_dcall_dV(100, K, V) * (2.0 * sn * dt) @ Wt
    col = r["grad"].sum(axis=0)
    col_se = _batch_column_se(o, s, book, N, n_paths, n_batches, seed=12)
    assert np.all(np.abs(col - col_expect) < 4.0 * col_se + 1e-12), (col, col_expect)


# --------------------------------------------------------------------------
# identities that hold sample by sample
# --------------------------------------------------------------------------
def pin_put_call_parity(o, n_paths=1 << 15):
    s = W.small_surface()
    N, T, K, tiny = 52, 1.0, 95.0, 1e-9
    rc = o.price_and_grad(s, W.call(K, T), n_paths, N, seed=21)
    rp = o.price_and_grad(s, W.put(K, T), n_paths, N, seed=21)
    r0 = o.price_and_grad(s, W.call(tiny, T), n_paths, N, seed=21)   # = mean(S_T) - tiny
    mean_ST = r0["price"][0] + tiny
    assert abs((rc["price"][0] - rp["price"][0]) - (mean_ST - K)) < 1e-11 * 100
    scale = np.abs(r0["grad"]).max()
    assert np.abs((rc["grad"] - rp["grad"]) - r0["grad"]).max() < 1e-11 * max(scale, 1.0)
    # martingale: E[S_T] = S_0 on any surface
    assert abs(mean_ST - 100.0) < 4.0 * r0["stderr"][0]
    # delta: call delta - put delta = d mean(S_T)/d S0
    assert abs((rc["delta"] - rp["delta"]) - r0["delta"]) < 1e-11


def pin_threads(o):
    s = W.book_surface(0)
    book = W.Book([0, 1], [100.0, 90.0], [1.0, 0.5], [1.0, 2.0])
    a = o.price_and_grad(s, book, 9000, 52, seed=1, n_threads=1)
    b = o.price_and_grad(s, book, 9000, 52, seed=1, n_threads=3)
    c = o.price_and_grad(s, book, 9000, 52, seed=1, n_threads=8)
    for k in ("price", "stderr", "grad"):
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k])


# --------------------------------------------------------------------------
# exact prices of the discrete scheme, one and two steps
# --------------------------------------------------------------------------
def pin_one_step(o, n_paths=1 << 17):
    """One step: y_1 is Gaussian with variance s_0^2 T, so price = BS(s_0^2 T) and
    d price / d node = C'(V) 2 s_0 T w_node(S_0, 0); nodes off the cell are zero."""
    for kind in (W.LIN, W.LOG):
        s = W.tiny_surface(kind, 6, 3, seed=9)
        T, K = 0.25, 103.0
        r = o.price_and_grad(s, W.call(K, T), n_paths, 1, seed=2)
        s0, _, (i, j), w = o.interp(s, 100.0, 0.0)
        V = s0 * s0 * T
        assert abs(r["price"][0] - cf.bs_call(100, K, V)) < 4 * r["stderr"][0]
        assert abs(cf.discrete_price_1step(s, K, T) - cf.bs_call(100, K, V)) < 1e-13
        _, _, g, g_se = _batch_stats(o, s, W.call(K, T), 1, n_paths, 32, seed=2)
        dv = cf.bs_dcall_dV(100, K, V) * 2 * s0 * T
        expect = np.zeros_like(s.sigma)
        for (di, dj), wk in zip([(0, 0), (1, 0), (0, 1), (1, 1)], w):
            expect[i + di, j + dj] += dv * wk
        mask = expect != 0
        assert np.all(np.abs(g[mask] - expect[mask]) < 4 * g_se[mask] + 1e-12)
        assert np.all(r["grad"][~mask] == 0.0)


def pin_two_steps(o, n_paths=1 << 17, n_batches=32):
    for kind in (W.LIN, W.LOG):
        s = W.tiny_surface(kind, 7, 3, seed=13)
        s = W.Surface(s.spot_axis, s.time_axis, s.sigma * 2.0)   # strong spot dependence
        T, K = 0.5, 100.0
        book = W.call(K, T)
        price, price_se, g, g_se = _batch_stats(o, s, book, 2, n_paths, n_batches, seed=4)
        exact = cf.discrete_price_2step(s, K, T)
        assert abs(price - exact) < 4 * price_se, (kind, price, exact, price_se)
        # gradients at the nodes the first two steps use, against central differences
        # of the exact price
        gx = cf.fd_on(lambda srf: cf.discrete_price_2step(srf, K, T), s, eps=1e-5)
        mask = np.abs(gx) > 1e-3 * np.abs(gx).max()
        assert mask.sum() >= 4
        assert np.all(np.abs(g[mask] - gx[mask]) < 4 * g_se[mask] + 1e-9), (kind, g, gx, g_se)


# --------------------------------------------------------------------------
# adjoint against bump-and-reprice
# --------------------------------------------------------------------------
def crn_fd_grad(o, surface, book, n_paths, n_steps, seed, eps=1e-5, scheme=0):
    """Central bump of every node, (value(p+eps/2) - value(p-eps/2)) / eps, on the same
    random streams, of the weighted book value (the oracle's bumping estimator)."""
    return o.bump_grad(surface, book, n_paths, n_steps, seed, eps, scheme=scheme).reshape(surface.sigma.shape)


# --------------------------------------------------------------------------
# the Euler step on X itself (scheme 1)
# --------------------------------------------------------------------------
def pin_euler_x_one_step(o, n_paths=1 << 17):
    """One Euler step on X: X_1 = S0 (1 + s_0 sqrt(T) Z) is Gaussian, so the call price
    is closed form and d price / d node = S0 phi(d) sqrt(T) w_node(S0, 0); nodes off the
    cell are zero."""
    for kind in (W.LIN, W.LOG):
        s = W.tiny_surface(kind, 6, 3, seed=9)
        T, K = 0.25, 103.0
        r = o.price_and_grad(s, W.call(K, T), n_paths, 1, seed=2, scheme=1)
        s0, _, (i, j), w = o.interp(s, 100.0, 0.0)
        exact, d_da = cf.euler_x_call_1step(100.0, K, s0 * math.sqrt(T))
        assert abs(r["price"][0] - exact) < 4 * r["stderr"][0], (kind, r["price"][0], exact)
        _, _, g, g_se = _batch_stats(o, s, W.call(K, T), 1, n_paths, 32, seed=2, scheme=1)
        expect = np.zeros_like(s.sigma)
        for (di, dj), wk in zip([(0, 0), (1, 0), (0, 1), (1, 1)], w):
            expect[i + di, j + dj] += d_da * math.sqrt(T) * wk
        mask = expect != 0
        assert np.all(np.abs(g[mask] - expect[mask]) < 4 * g_se[mask] + 1e-12), (kind, g, expect)
        assert np.all(r["grad"][~mask] == 0.0)


def pin_euler_x_moments(o, n_paths=1 << 17):
    """Flat sigma, Euler on X: E[X_N] = S0 and E[(X_N - S0)^2] = S0^2 ((1 + sigma^2 dt)^N
    - 1), where the log scheme has S0^2 (exp(sigma^2 T) - 1) (10% apart here).  A call
    and a put at K = S0 give X - K = call - put and (X - K)^2 = call^2 + put^2."""
    sig, N, T = 0.6, 2, 1.0
    s = W.flat_surface(W.small_surface(), sig)
    book = W.Book([0, 1], [100.0, 100.0], [T, T], [1.0, 1.0])
    r = o.sums(s, book, N, 3, [(0, n_paths)], want_grad=False, scheme=1)
    m1 = (r["sum_pay"][0] - r["sum_pay"][1]) / n_paths
    m2 = (r["sum_pay2"][0] + r["sum_pay2"][1]) / n_paths
    exact = cf.euler_x_second_moment(100.0, sig, T / N, N)
    assert abs(m1) < 4 * math.sqrt(m2 / n_paths), m1
    assert abs(m2 - exact) < 0.03 * exact, (m2, exact)
    lognormal = 100.0 ** 2 * (math.exp(sig * sig * T) - 1.0)
    assert abs(lognormal - exact) > 0.08 * exact


def pin_adjoint_fd(o):
    book = W.Book([0, 1, 0], [100.0, 105.0, 92.0], [1.0, 0.5, 0.75], [1.0, 2.5, -0.7])
    for kind, scheme in ((W.LIN, 0), (W.LOG, 0), (W.LIN, 1), (W.LOG, 1)):
        s = W.tiny_surface(kind, 5, 4, seed=21 + kind)
        r = o.price_and_grad(s, book, 512, 8, seed=6, scheme=scheme)
        fd = crn_fd_grad(o, s, book, 512, 8, seed=6, scheme=scheme)
        scale = np.abs(r["grad"]).max()
        assert scale > 0.1
        err = np.abs(r["grad"] - fd).max()
        assert err < 2e-6 * scale, (kind, scheme, err, scale)
        # delta against a central bump of the spot
        h = 1e-4
        up = o.price_and_grad(s, book, 512, 8, seed=6, spot=100.0 + h, want_grad=False, scheme=scheme)
        dn = o.price_and_grad(s, book, 512, 8, seed=6, spot=100.0 - h, want_grad=False, scheme=scheme)
        fd_delta = (np.dot(book.weight, up["price"]) - np.dot(book.weight, dn["price"])) / (2 * h)
        assert abs(r["delta"] - fd_delta) < 1e-6 * max(1.0, abs(fd_delta)), (r["delta"], fd_delta)


# --------------------------------------------------------------------------
# zero buckets
# --------------------------------------------------------------------------
def pin_zero_buckets(o):
    """Nodes no path can reach carry exactly zero gradient: time nodes past the last
    step's cell, and spot nodes beyond the largest possible move."""
    sa = W.Axis(40, W.LIN, 10.0, 400.0)
    ta = W.Axis(5, W.LIN, 0.0, 2.0)
    rng = np.random.default_rng(2)
    s = W.Surface(sa, ta, rng.uniform(0.15, 0.3, (40, 5)))
    N, T = 2, 2.0 / 52
    r = o.price_and_grad(s, W.call(100.0, T), 4096, N, seed=1)
    g = r["grad"]
    # steps at t = 0 and t = dt both sit in time cell 0: columns 2.. unreachable
    assert np.all(g[:, 2:] == 0.0)
    # |log move| <= N * max sigma * sqrt(dt) * max|Z|
    reach = N * 0.3 * math.sqrt(T / N) * SQRT_TAIL
    nodes = sa.nodes()
    far = (nodes < 100.0 * math.exp(-reach) - 10.0) | (nodes > 100.0 * math.exp(reach) + 10.0)
    assert far.sum() > 10
    assert np.all(g[far, :] == 0.0)
    assert np.abs(g).max() > 0


FAST_PINS = [pin_uniform, pin_box_muller, pin_interp, pin_flat_black_scholes,
             pin_flat_pathwise_vega, pin_put_call_parity, pin_adjoint_fd, pin_term_structure,
             pin_one_step, pin_euler_x_one_step, pin_euler_x_moments]


def pin_round_bf16(o):
    """Vol nodes rounded to bfloat16 by way of single precision.  Checked against
    torch's float32 -> bfloat16 conversion (round to nearest, ties to even) over six
    decades; at every midpoint between neighbouring bfloat16 values in [1/16, 4) the
    even neighbour is taken, one single ulp either side goes to the nearer one, and
    bfloat16 values are fixed points; a double just above a midpoint (by less than half
    a single ulp) first becomes the midpoint and so also goes to the even neighbour."""
    import torch
    r = np.random.default_rng(11)
    x = np.concatenate([r.uniform(0.05, 1.5, 4000), np.exp(r.uniform(-7.0, 7.0, 4000))])
    lib = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(o.round_bf16(x), lib)
    bits = np.arange(0x3D80, 0x4080, dtype=np.uint32)            # bfloat16 patterns in [1/16, 4)
    b = (bits << 16).view(np.float32).astype(np.float64)
    lo, hi = b[:-1], b[1:]
    mid = 0.5 * (lo + hi)                                         # exact in single precision
    even = np.where((bits[:-1] & 1) == 0, lo, hi)
    assert np.array_equal(o.round_bf16(mid), even)
    mid32 = mid.astype(np.float32)
    down = np.nextafter(mid32, np.float32(0)).astype(np.float64)
    up = np.nextafter(mid32, np.float32(np.inf)).astype(np.float64)
    assert np.array_equal(o.round_bf16(down), lo) and np.array_equal(o.round_bf16(up), hi)
    assert np.array_equal(o.round_bf16(b), b)
    ulp32 = np.spacing(mid32).astype(np.float64)
    assert np.array_equal(o.round_bf16(mid + 0.25 * ulp32), even)


# --------------------------------------------------------------------------
# a constant short rate: the trend of the narrated step (Sec. IV-A), payoffs
# discounted by e^{-r T}
# --------------------------------------------------------------------------
RATE = 0.05


def pin_rate_black_scholes(o, n_paths=1 << 17, n_batches=32):
    """Flat vol with r = 0.05: log-Euler stays exact in law, so the discounted calls and
    put are Black-Scholes with the rate (within 4 standard errors); per path, the grid
    gradient sums to the discounted pathwise vega e^{-rT} S_T 1{S_T>K} (-sigma T +
    sqrt(dt) sum Z) with y_N = (r - sigma^2/2) T + sigma sqrt(dt) sum Z; by batch means
    the sum of the grid gradient is the Black-Scholes vega S0 phi(d1) sqrt(T)."""
    s = W.flat_surface(W.small_surface(), 0.2)
    book = W.Book([0, 1, 0], [100.0, 110.0, 80.0], [1.0, 1.0, 0.5], [1.0, 1.0, 1.0])
    r = o.price_and_grad(s, book, n_paths, 52, seed=5, rate=RATE)
    ref = [cf.bs_call_r(100, 100, 0.2, 1.0, RATE), cf.bs_put_r(100, 110, 0.2, 1.0, RATE),
           cf.bs_call_r(100, 80, 0.2, 0.5, RATE)]
    for k in range(3):
        assert abs(r["price"][k] - ref[k]) < 4.0 * r["stderr"][k], (k, r["price"][k], ref[k])
    dt, call = 1.0 / 52, W.call(100.0, 1.0)
    for p in range(20):
        q = o.path(s, call, 52, 3, p, rate=RATE)
        yN = (RATE - 0.02) * 1.0 + 0.2 * math.sqrt(dt) * q["z"].sum()
        assert abs(q["y"][-1] - yN) < 1e-12
        ST = 100.0 * math.exp(q["y"][-1])
        expect = math.exp(-RATE) * (ST if ST > 100.0 else 0.0) * (-0.2 + math.sqrt(dt) * q["z"].sum())
        assert abs(q["grad"].sum() - expect) <= 1e-11 * max(1.0, abs(expect)), (p, q["grad"].sum(), expect)
    per = n_paths // n_batches
    tot = [o.sums(s, call, 52, 8, [(b * per, (b + 1) * per)], rate=RATE)["sum_grad"].sum() / per
           for b in range(n_batches)]
    vega = cf.bs_vega_r(100.0, 100.0, 0.2, 1.0, RATE)
    assert abs(np.mean(tot) - vega) < 4.0 * np.std(tot, ddof=1) / math.sqrt(n_batches), (np.mean(tot), vega)


def pin_rate_parity_and_martingale(o, n_paths=1 << 15):
    """On the smile surface with r = 0.05, for two maturities: call - put =
    e^{-rT} (mean S_T - K) sample by sample (prices, grids and deltas), and the
    discounted spot is a martingale of the scheme, E[e^{-rT} S_T] = S0."""
    s = W.small_surface()
    K, tiny = 95.0, 1e-9
    for T in (0.5, 1.0):
        mat = [T, 1.0]          # the second option fixes dt = 1/52
        rc = o.price_and_grad(s, W.Book([0, 0], [K, K], mat, [1.0, 0.0]), n_paths, 52, seed=21, rate=RATE)
        rp = o.price_and_grad(s, W.Book([1, 0], [K, K], mat, [1.0, 0.0]), n_paths, 52, seed=21, rate=RATE)
        r0 = o.price_and_grad(s, W.Book([0, 0], [tiny, K], mat, [1.0, 0.0]), n_paths, 52, seed=21, rate=RATE)
        disc = math.exp(-RATE * T)
        mean_ST = r0["price"][0] + tiny * disc          # = e^{-rT} mean(S_T)
        assert abs((rc["price"][0] - rp["price"][0]) - (mean_ST - K * disc)) < 1e-11 * 100
        scale = max(np.abs(r0["grad"]).max(), 1.0)
        assert np.abs((rc["grad"] - rp["grad"]) - r0["grad"]).max() < 1e-11 * scale
        assert abs((rc["delta"] - rp["delta"]) - r0["delta"]) < 1e-11
        assert abs(mean_ST - 100.0) < 4.0 * r0["stderr"][0], (T, mean_ST)


def pin_rate_one_step(o, n_paths=1 << 17):
    """One step with r = 0.05: y_1 = (r - s_0^2/2) T + s_0 sqrt(T) Z, so the call is
    Black-Scholes with vol s_0 and rate r, and d price / d node = vega(s_0) w_node(S0, 0)."""
    for kind in (W.LIN, W.LOG):
        s = W.tiny_surface(kind, 6, 3, seed=9)
        T, K = 0.25, 103.0
        r = o.price_and_grad(s, W.call(K, T), n_paths, 1, seed=2, rate=RATE)
        s0, _, (i, j), w = o.interp(s, 100.0, 0.0)
        assert abs(r["price"][0] - cf.bs_call_r(100, K, s0, T, RATE)) < 4 * r["stderr"][0]
        per = n_paths // 32
        gs = np.array([o.sums(s, W.call(K, T), 1, 2, [(b * per, (b + 1) * per)], rate=RATE)["sum_grad"] / per
                       for b in range(32)])
        g, g_se = gs.mean(axis=0), gs.std(axis=0, ddof=1) / math.sqrt(32)
        dv = cf.bs_vega_r(100, K, s0, T, RATE)
        expect = np.zeros_like(s.sigma)
        for (di, dj), wk in zip([(0, 0), (1, 0), (0, 1), (1, 1)], w):
            expect[i + di, j + dj] += dv * wk
        mask = expect != 0
        assert np.all(np.abs(g[mask] - expect[mask]) < 4 * g_se[mask] + 1e-12), (kind, g[mask], expect[mask])
        assert np.all(r["grad"][~mask] == 0.0)


def pin_rate_euler_x_one_step(o, n_paths=1 << 17):
    """One Euler step on X with r = 0.05: X_1 = S0 (1 + rT + s_0 sqrt(T) Z) is Gaussian,
    so the discounted call is closed form and d price / d node = e^{-rT} S0 phi(d)
    sqrt(T) w_node(S0, 0)."""
    s = W.tiny_surface(W.LIN, 6, 3, seed=9)
    T, K = 0.25, 103.0
    r = o.price_and_grad(s, W.call(K, T), n_paths, 1, seed=2, scheme=1, rate=RATE)
    s0, _, (i, j), w = o.interp(s, 100.0, 0.0)
    und, d_da = cf.euler_x_call_1step_r(100.0, K, s0 * math.sqrt(T), RATE * T)
    disc = math.exp(-RATE * T)
    assert abs(r["price"][0] - disc * und) < 4 * r["stderr"][0]
    _, _, g, g_se = _batch_stats(o, s, W.call(K, T), 1, n_paths, 32, seed=2, scheme=1, rate=RATE)
    expect = np.zeros_like(s.sigma)
    for (di, dj), wk in zip([(0, 0), (1, 0), (0, 1), (1, 1)], w):
        expect[i + di, j + dj] += disc * d_da * math.sqrt(T) * wk
    mask = expect != 0
    assert np.all(np.abs(g[mask] - expect[mask]) < 4 * g_se[mask] + 1e-12)


def pin_rate_adjoint_fd(o):
    """With r = 0.05, the adjoint of both schemes (and the delta) against central
    bumps on the same streams, for a book of calls and puts of two maturities."""
    book = W.Book([0, 1, 0], [100.0, 105.0, 92.0], [1.0, 0.5, 0.75], [1.0, 2.5, -0.7])
    for kind, scheme in ((W.LIN, 0), (W.LOG, 0), (W.LIN, 1), (W.LOG, 1)):
        s = W.tiny_surface(kind, 5, 4, seed=21 + kind)
        r = o.price_and_grad(s, book, 512, 8, seed=6, scheme=scheme, rate=RATE)
        fd = o.bump_grad(s, book, 512, 8, 6, 1e-5, scheme=scheme, rate=RATE).reshape(s.sigma.shape)
        scale = np.abs(r["grad"]).max()
        assert np.abs(r["grad"] - fd).max() < 2e-6 * scale, (kind, scheme)
        h = 1e-4
        up = o.price_and_grad(s, book, 512, 8, seed=6, spot=100.0 + h, want_grad=False, scheme=scheme, rate=RATE)
        dn = o.price_and_grad(s, book, 512, 8, seed=6, spot=100.0 - h, want_grad=False, scheme=scheme, rate=RATE)
        fd_delta = (np.dot(book.weight, up["price"]) - np.dot(book.weight, dn["price"])) / (2 * h)
        assert abs(r["delta"] - fd_delta) < 1e-6 * max(1.0, abs(fd_delta)), (r["delta"], fd_delta)

"""Closed forms and brute-force integrals that pin the oracle.

Everything here is derived independently of the oracle's code: Black-Scholes
formulas in total variance (zero rates), time-interpolation weights of a
uniform time grid, and exact prices of the discretised scheme for one and two
steps by one-dimensional integration.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate
from scipy.special import ndtr

SQRT2PI = math.sqrt(2.0 * math.pi)


def npdf(x):
    return np.exp(-0.5 * np.asarray(x) ** 2) / SQRT2PI


def euler_x_call_1step(S, K, a):
    """Call on X_1 = S (1 + a Z), Z standard normal (one Euler step on X with
    a = sigma sqrt(T)): X_1 is Gaussian with mean S and sd S a, so the price is
    (S - K) Phi(d) + S a phi(d), d = (S - K) / (S a); its derivative in a is S phi(d)."""
    d = (S - K) / (S * a)
    return (S - K) * ndtr(d) + S * a * float(npdf(d)), S * float(npdf(d))


def euler_x_second_moment(S, sigma, dt, n_steps):
    """E[(X_N - S)^2] for X_{n+1} = X_n (1 + sigma sqrt(dt) Z_n), flat sigma: the
    factors are independent with mean 1 and second moment 1 + sigma^2 dt."""
    return S * S * ((1.0 + sigma * sigma * dt) ** n_steps - 1.0)


def bs_call(S, K, V):
    """Undiscounted Black-Scholes call with total variance V = sigma^2 T."""
    S, K, V = np.asarray(S, float), np.asarray(K, float), np.asarray(V, float)
    sv = np.sqrt(V)
    d1 = (np.log(S / K) + 0.5 * V) / sv
    return S * ndtr(d1) - K * ndtr(d1 - sv)


def bs_put(S, K, V):
    return bs_call(S, K, V) - S + K


def bs_dcall_dV(S, K, V):
    """d call / d total variance = S phi(d1) / (2 sqrt V)."""
    sv = math.sqrt(V)
    d1 = (math.log(S / K) + 0.5 * V) / sv
    return S * float(npdf(d1)) / (2.0 * sv)


def bs_vega(S, K, sigma, T):
    """d call / d sigma for a flat volatility."""
    V = sigma * sigma * T
    return bs_dcall_dV(S, K, V) * 2.0 * sigma * T


def call_payoff_sd(S, K, V):
    """Standard deviation of (S_T - K)^+ for lognormal S_T with E S_T = S."""
    sv = math.sqrt(V)
    d1 = (math.log(S / K) + 0.5 * V) / sv
    d2 = d1 - sv
    m2 = S * S * math.exp(V) * ndtr(d1 + sv) - 2 * K * S * ndtr(d1) + K * K * ndtr(d2)
    m1 = float(bs_call(S, K, V))
    return math.sqrt(m2 - m1 * m1)


def time_weights(time_axis, n_steps: int, dt: float) -> np.ndarray:
    """W[n, j]: weight of time node j in the linear time interpolation at t = n dt,
    clamped to the grid (flat outside)."""
    tn = time_axis.lo + (time_axis.hi - time_axis.lo) * np.arange(time_axis.n) / (time_axis.n - 1)
    W = np.zeros((n_steps, time_axis.n))
    for n in range(n_steps):
        t = n * dt
        if t <= tn[0]:
            W[n, 0] = 1.0
            continue
        if t >= tn[-1]:
            W[n, -1] = 1.0
            continue
        j = int(np.searchsorted(tn, t, side="right") - 1)
        a = (t - tn[j]) / (tn[j + 1] - tn[j])
        W[n, j] += 1.0 - a
        W[n, j + 1] += a
    return W


def bilinear(surface, S, t):
    """Bilinear interpolation of a surface at spot(s) S and time t, linear in the
    spot axis coordinate (S or ln S), flat outside the grid."""
    sa, ta = surface.spot_axis, surface.time_axis
    S = np.atleast_1d(np.asarray(S, float))
    if sa.kind == 1:
        x, x0, x1 = np.log(S), math.log(sa.lo), math.log(sa.hi)
    else:
        x, x0, x1 = S, sa.lo, sa.hi
    xs = np.linspace(x0, x1, sa.n)
    ts = np.linspace(ta.lo, ta.hi, ta.n)
    col = np.array([np.interp(t, ts, surface.sigma[i, :]) for i in range(sa.n)])
    return np.interp(x, xs, col)


def _spot_breaks(surface, lo, hi):
    sa = surface.spot_axis
    return [float(v) for v in sa.nodes() if lo < v < hi]


def discrete_price_1step(surface, K: float, T: float, spot: float = 100.0, put=False):
    """Exact price of the one-step scheme: the terminal log-spot is Gaussian."""
    s0 = float(bilinear(surface, spot, 0.0)[0])
    V = s0 * s0 * T
    return float(bs_put(spot, K, V) if put else bs_call(spot, K, V))


def discrete_price_2step(surface, K: float, T: float, spot: float = 100.0, put=False):
    """Exact price of the two-step log-Euler scheme with dt = T/2: conditional on the
    first normal the second step is lognormal, so the price is a 1-D integral of a
    Black-Scholes value, integrated piecewise between spot-node crossings."""
    dt = T / 2.0
    s0 = float(bilinear(surface, spot, 0.0)[0])

    def S1(z):
        return spot * math.exp(-0.5 * s0 * s0 * dt + s0 * math.sqrt(dt) * z)

    def integrand(z):
        x = S1(z)
        s1 = float(bilinear(surface, x, dt)[0])
        v = s1 * s1 * dt
        val = bs_put(x, K, v) if put else bs_call(x, K, v)
        return float(val) * math.exp(-0.5 * z * z) / SQRT2PI

    zlo, zhi = -9.0, 9.0
    # z values where S1 crosses a spot node: integrand kinks there
    cuts = []
    for node in _spot_breaks(surface, S1(zlo), S1(zhi)):
        z = (math.log(node / spot) + 0.5 * s0 * s0 * dt) / (s0 * math.sqrt(dt))
        cuts.append(z)
    edges = [zlo] + sorted(cuts) + [zhi]
    total = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        val, _ = integrate.quad(integrand, a, b, epsabs=1e-13, epsrel=1e-12, limit=200)
        total += val
    return total


def fd_on(fn, surface, eps: float = 1e-6):
    """Central differences of fn(surface) with respect to every node."""
    from workloads import Surface
    g = np.zeros_like(surface.sigma)
    for i in range(surface.sigma.shape[0]):
        for j in range(surface.sigma.shape[1]):
            up = surface.sigma.copy(); up[i, j] += eps / 2
            dn = surface.sigma.copy(); dn[i, j] -= eps / 2
            g[i, j] = (fn(Surface(surface.spot_axis, surface.time_axis, up))
                       - fn(Surface(surface.spot_axis, surface.time_axis, dn))) / eps
    return g


# --------------------------------------------------------------------------
# with a constant short rate r (discounted prices)
# --------------------------------------------------------------------------
def bs_call_r(S, K, sigma, T, r):
    """Black-Scholes call with rate r: S N(d1) - K e^{-rT} N(d2)."""
    v = sigma * math.sqrt(T)
    d1 = (math.log(S / K) + (r + 0.5 * sigma * sigma) * T) / v
    return S * float(ndtr(d1)) - K * math.exp(-r * T) * float(ndtr(d1 - v))


def bs_put_r(S, K, sigma, T, r):
    """Put by parity: call - S + K e^{-rT}."""
    return bs_call_r(S, K, sigma, T, r) - S + K * math.exp(-r * T)


def bs_vega_r(S, K, sigma, T, r):
    """d call / d sigma with rate r: S phi(d1) sqrt(T)."""
    v = sigma * math.sqrt(T)
    d1 = (math.log(S / K) + (r + 0.5 * sigma * sigma) * T) / v
    return S * float(npdf(d1)) * math.sqrt(T)


def euler_x_call_1step_r(S, K, a, rT):
    """Call on X_1 = S (1 + rT + a Z) (one Euler step on X with trend rT and
    a = sigma sqrt(T)), undiscounted: X_1 is Gaussian with mean m = S (1 + rT) and sd
    S a, so the expectation is (m - K) Phi(d) + S a phi(d), d = (m - K) / (S a); its
    derivative in a is S phi(d)."""
    m = S * (1.0 + rT)
    d = (m - K) / (S * a)
    return (m - K) * ndtr(d) + S * a * float(npdf(d)), S * float(npdf(d))

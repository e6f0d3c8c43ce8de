"""Per-option vol-grid gradients from one simulation (lv_per_option_grads_dev: one
reverse sweep serves up to 8 options, each with its own adjoint and histogram) against
the oracle run with that option's one-hot weight, option by option (Sec. III,
Sec. IV-C); the weighted sum against the book's own gradient."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import fp32_checks as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lv():
    import paper_2002_02481_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(lv):
    return lv.Context(0)


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


def eleven():
    """11 calls and puts over four maturities: one sweep of 8 and one of 3 on a grid
    that takes 8 options per sweep."""
    k = np.arange(11)
    return W.Book((k % 2).astype(np.int32), 80.0 + 4.0 * k, np.array([0.25, 0.5, 1.0, 0.75])[k % 4],
                  1.0 + 0.1 * k)


def _per_option(lv, ctx, s, book, P, N, seed, precision, rate=0.0):
    import torch
    sig = torch.tensor(s.sigma, dtype=torch.float64, device="cuda")
    p, se, g, d = lv.per_option_grads_dev(sig, 100.0, book.strike, book.maturity, P, N, seed,
                                          spot_axis=s.spot_axis, time_axis=s.time_axis, is_put=book.is_put,
                                          precision=precision, rate=rate, ctx=ctx)
    return p.cpu().numpy(), g.cpu().numpy(), d.cpu().numpy()


def _one_hot_refs(orc, s, book, P, N, seed, rate=0.0):
    out = []
    for k in range(book.n):
        w = np.zeros(book.n)
        w[k] = 1.0
        out.append(orc.price_and_grad(s, W.Book(book.is_put, book.strike, book.maturity, w), P, N, seed,
                                      rate=rate))
    return out


@pytest.mark.parametrize("surface,rate", [("benchmark", 0.0), ("benchmark", 0.04), ("wide", 0.0)])
def test_per_option_grids_fp64(lv, ctx, orc, surface, rate):
    """FP64: every option's grid within 1e-9 max|g_k| of the oracle's one-hot gradient and
    its delta within 1e-10; the weighted sum equals the fused call's book gradient.  The
    60 x 30 grid takes 8 options per sweep (11 options: sweeps of 8 and 3), the
    100 x 50 grid fewer."""
    s = W.book_surface(0) if surface == "benchmark" else W.wide_surface(2)
    book = eleven()
    P, N = 6151, 52
    price, grads, deltas = _per_option(lv, ctx, s, book, P, N, 4, 64, rate)
    refs = _one_hot_refs(orc, s, book, P, N, 4, rate)
    worst = 0.0
    for k, r in enumerate(refs):
        gk = np.abs(r["grad"]).max()
        err = np.abs(grads[k] - r["grad"]).max() / max(gk, 1e-300)
        worst = max(worst, err)
        assert err <= 1e-9, (k, err)
        assert np.all(grads[k][r["grad"] == 0.0] == 0.0), k
        assert abs(deltas[k] - r["delta"]) <= 1e-10 * max(1.0, abs(r["delta"])), k
        assert abs(price[k] - r["price"][k]) <= 1e-11 * max(abs(r["price"][k]), 1e-2), k
    F.say(f"  per-option FP64 ({surface}, r={rate}): worst max|dg_k|/max|g_k| {worst:.3g}")
    p, se, g, d = lv.price_and_grad(s, 100.0, book.strike, book.maturity, P, N, 4, is_put=book.is_put,
                                    weights=book.weight, precision=64, rate=rate, ctx=ctx)
    assert np.abs(np.tensordot(book.weight, grads, axes=1) - g).max() <= 1e-10 * np.abs(g).max()
    assert abs(float(np.dot(book.weight, deltas)) - d) <= 1e-10 * max(1.0, abs(d))


@pytest.mark.parametrize("shape,kind", [((80, 40), W.LIN), ((150, 80), W.LOG)])
def test_per_option_grids_fewer_per_sweep(lv, ctx, orc, shape, kind):
    """FP64 on grids whose per-option LDS grids allow only 4 (80 x 40) or 1 (150 x 80)
    options per sweep: every option's grid and delta against the oracle's one-hot
    gradient, as above (11 options: sweeps of 4, 4, 3, or 11 sweeps of one).  The
    surface is the smooth 1-year smile on these axes (a rough random surface on so fine
    a spot axis makes step derivatives near 2 and adjoints near 1e9, where FP64 rounding
    alone separates any two summation orders by 1e-5 relative)."""
    sa = W.Axis(shape[0], kind, 50.0, 200.0)
    ta = W.Axis(shape[1], W.LIN, 0.0, 1.0)
    s = W.Surface(sa, ta, W.smile_surface(sa, ta, 0.15, 0.10, decay=True))
    book = eleven()
    P, N = 4099, 52
    price, grads, deltas = _per_option(lv, ctx, s, book, P, N, 9, 64)
    refs = _one_hot_refs(orc, s, book, P, N, 9)
    worst = 0.0
    for k, r in enumerate(refs):
        gk = np.abs(r["grad"]).max()
        err = np.abs(grads[k] - r["grad"]).max() / max(gk, 1e-300)
        worst = max(worst, err)
        assert err <= 1e-9, (k, err)
        assert np.all(grads[k][r["grad"] == 0.0] == 0.0), k
        assert abs(deltas[k] - r["delta"]) <= 1e-10 * max(1.0, abs(r["delta"])), k
    F.say(f"  per-option FP64 {shape}: worst max|dg_k|/max|g_k| {worst:.3g}")


def test_per_option_grids_fp32(lv, ctx, orc):
    """FP32 on the smooth 21 x 13 surface: every option's grid within 1e-4 max|g_k| of the
    oracle's one-hot gradient (on the FP32-rounded surface), prices within 1e-5 spot."""
    s = W.small_surface()
    book = eleven()
    P, N = 16384, 52
    price, grads, deltas = _per_option(lv, ctx, s, book, P, N, 0, 32)
    refs = _one_hot_refs(orc, s.rounded_to_f32(), book, P, N, 0)
    worst = 0.0
    for k, r in enumerate(refs):
        gk = np.abs(r["grad"]).max()
        err = np.abs(grads[k] - r["grad"]).max() / gk
        worst = max(worst, err)
        assert err <= 1e-4, (k, err)
        assert np.all(grads[k][r["grad"] == 0.0] == 0.0), k
        assert abs(price[k] - r["price"][k]) < 1e-5 * 100.0
    F.say(f"  per-option FP32: worst max|dg_k|/max|g_k| {worst:.3g}")

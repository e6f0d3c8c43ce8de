"""A constant short rate on the GPU against the oracle: the trend r dt that each step
adds (to ln X, or r dt X to X on the Euler step on X) and e^{-r T_k} discounting of
every option's price, standard error, gradient and delta (the step's deterministic
trend, Sec. IV-A).  FP64 at the tight bar on every path; FP32 at the plain bar on the
smooth 21 x 13 surface and block-paired on the noisy 60 x 30 one."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import fp32_checks as F

pytestmark = pytest.mark.gpu

PRICE_TOL = 1e-5 * 100.0


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


def _gpu(lv, ctx, surface, book, P, N, seed, **opts):
    p, se, g, d = lv.price_and_grad(surface, 100.0, book.strike, book.maturity, P, N, seed, is_put=book.is_put,
                                    weights=book.weight, ctx=ctx, **opts)
    return dict(price=p, stderr=se, grad=g, delta=d)


def _tight(got, ref, what):
    assert np.allclose(got["price"], ref["price"], rtol=1e-11, atol=1e-13), what
    assert np.allclose(got["stderr"], ref["stderr"], rtol=1e-9, atol=1e-15), what
    gmax = np.abs(ref["grad"]).max()
    assert np.abs(got["grad"] - ref["grad"]).max() <= 1e-9 * gmax, what
    assert np.all(got["grad"][ref["grad"] == 0.0] == 0.0), what
    assert abs(got["delta"] - ref["delta"]) <= 1e-10 * max(1.0, abs(ref["delta"])), what


def _plain32(got, ref, what):
    assert np.abs(got["price"] - ref["price"]).max() < PRICE_TOL, what
    assert np.allclose(got["stderr"], ref["stderr"], rtol=1e-4), what
    gmax = np.abs(ref["grad"]).max()
    err = np.abs(got["grad"] - ref["grad"]).max() / gmax
    F.say(f"  {what}: max|dgrad|/max|g| {err:.3g}")
    assert err <= 1e-4, what
    assert np.all(got["grad"][ref["grad"] == 0.0] == 0.0), what


def book3():
    return W.Book([0, 1, 0], [100.0, 110.0, 90.0], [1.0, 0.5, 0.25], [1.0, -0.5, 2.0])


@pytest.mark.parametrize("adjoint", ["stored", "checkpoint"])
@pytest.mark.parametrize("rate", [0.05, -0.02])
def test_rate_small_surface(lv, ctx, orc, adjoint, rate):
    """A call, a put and a call of three maturities on the 21 x 13 surface, 12289 paths."""
    s, b = W.small_surface(), book3()
    P, N = 12289, 52
    ref64 = orc.price_and_grad(s, b, P, N, 3, rate=rate)
    _tight(_gpu(lv, ctx, s, b, P, N, 3, precision=64, adjoint=adjoint, rate=rate), ref64, f"FP64 {adjoint} r={rate}")
    ref32 = orc.price_and_grad(s.rounded_to_f32(), b, P, N, 3, rate=rate)
    _plain32(_gpu(lv, ctx, s, b, P, N, 3, adjoint=adjoint, rate=rate), ref32, f"FP32 {adjoint} r={rate}")
    # the discount is real: the same paths at r = 0 price differently
    r0 = orc.price_and_grad(s, b, P, N, 3)
    assert np.abs(r0["price"] - ref64["price"]).max() > 0.1


@pytest.mark.parametrize("axis", [W.LIN, W.LOG])
@pytest.mark.parametrize("adjoint", ["stored", "checkpoint"])
def test_rate_euler_x(lv, ctx, orc, axis, adjoint):
    """The Euler step on X with a rate, X += r dt X + sigma X sqrt(dt) Z, on a linear and
    a log spot axis: FP64 tight, FP32 plain bar."""
    s = W.tiny_surface(axis, 9, 6, seed=4)
    b, P, N = book3(), 8195, 52
    ref64 = orc.price_and_grad(s, b, P, N, 7, scheme=1, rate=0.04)
    _tight(_gpu(lv, ctx, s, b, P, N, 7, precision=64, adjoint=adjoint, scheme="euler_x", rate=0.04), ref64,
           f"Euler on X FP64 {adjoint}")
    ref32 = orc.price_and_grad(s.rounded_to_f32(), b, P, N, 7, scheme=1, rate=0.04)
    _plain32(_gpu(lv, ctx, s, b, P, N, 7, adjoint=adjoint, scheme="euler_x", rate=0.04), ref32,
             f"Euler on X FP32 {adjoint}")


@pytest.mark.parametrize("adjoint", ["stored", "checkpoint"])
def test_rate_noisy_log_axis_book(lv, ctx, orc, adjoint):
    """Calls and puts of uneven maturity on the noisy 60 x 30 log-axis surface, a ragged
    2^16 + 77 paths, r = 0.03: FP64 tight; FP32 prices and the block-paired gradient."""
    s = W.book_surface(0)
    b = W.Book([0, 1, 0, 1, 0], [80.0, 95.0, 100.0, 120.0, 140.0], [0.5, 1.0, 3.0, 2.0, 3.0],
               [1.0, 1.0, 1.0, -1.0, 0.5])
    P, N = (1 << 16) + 77, 156
    ref64 = orc.price_and_grad(s, b, P, N, 5, rate=0.03)
    _tight(_gpu(lv, ctx, s, b, P, N, 5, precision=64, adjoint=adjoint, rate=0.03), ref64, f"book FP64 {adjoint}")
    s32 = s.rounded_to_f32()
    got = _gpu(lv, ctx, s, b, P, N, 5, adjoint=adjoint, rate=0.03)
    ref32 = orc.price_and_grad(s32, b, P, N, 5, rate=0.03, want_grad=False)
    assert np.abs(got["price"] - ref32["price"]).max() < PRICE_TOL
    info = ctx.run_info()
    B, T = info["n_blocks"], info["tile_paths"]
    blocks = ctx.block_grads(s.sigma.size, b.n).reshape((B,) + s.sigma.shape)
    ob = np.array([orc.sums(s32, b, N, 5, F.block_ranges(k, B, T, P), rate=0.03)["sum_grad"] for k in range(B)])
    F.paired_check(got["grad"], blocks, ob, P, f"book FP32 {adjoint} r=0.03")


def test_rate_through_lvprice(lv, orc):
    """LVPrice with a rate (the split forward and backward): FP64 against the oracle."""
    import torch
    s, b = W.small_surface(), book3()
    P, N = 8192, 52
    sig = torch.tensor(s.sigma, dtype=torch.float64, device="cuda", requires_grad=True)
    spec = dict(spot=100.0, strikes=b.strike, maturities=b.maturity, is_put=b.is_put, n_paths=P, n_steps=N,
                seed=2, spot_axis=s.spot_axis, time_axis=s.time_axis, precision=64, rate=0.05)
    price, _ = lv.LVPrice.apply(sig, spec)
    c = torch.tensor(b.weight, dtype=torch.float64, device="cuda")
    (price * c).sum().backward()
    ref = orc.price_and_grad(s, b, P, N, 2, rate=0.05)
    assert np.allclose(price.detach().cpu().numpy(), ref["price"], rtol=1e-11, atol=1e-13)
    assert np.abs(sig.grad.cpu().numpy() - ref["grad"]).max() <= 1e-9 * np.abs(ref["grad"]).max()

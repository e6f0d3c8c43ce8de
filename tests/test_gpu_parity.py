"""GPU parity: the HIP library against the FP64 CPU oracle on the same Philox streams.

Bars (the FP32 path steps, interpolates and back-propagates in FP32 and sums
across paths in FP64):
  * Philox words: bit-exact.
  * price: |GPU - oracle| < 1e-5 * spot; std_err within 1e-4 relative.
  * gradient: every bucket within 1e-4 * max|g|; buckets the oracle leaves
    exactly zero are exactly zero.  On the noisy, fine or long-horizon surfaces,
    where single precision cannot take some of the cell decisions the FP64 oracle
    takes, the FP32 bars are those of tests/fp32_checks.py: FP32 states within the
    oracle's single-precision bound path by path, and a bucket difference that is
    unbiased block by block.
  * the FP64 kernels: price within 1e-11 relative, buckets within 1e-9 * max|g|,
    on every workload.
The oracle sees the surface rounded to float32 when it checks the FP32 kernels,
so that input rounding is not counted as error.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests import fp32_checks as F

pytestmark = pytest.mark.gpu

PRICE_TOL = 1e-5 * 100.0
GRAD_TOL = 1e-4
F64_PRICE_REL = 1e-11
F64_GRAD = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


def gpu_run(lv, ctx, surface, book, n_paths, n_steps, seed=0, **opts):
    say(f"  gpu: {surface.sigma.shape} P={n_paths} N={n_steps} opts={opts}")
    p, s, g, d = lv.price_and_grad(surface, 100.0, book.strike, book.maturity, n_paths, n_steps,
                                   seed, is_put=book.is_put, weights=book.weight, ctx=ctx, **opts)
    return dict(price=p, stderr=s, grad=g, delta=d)


def assert_parity(got, ref, precision=32, what="", grad_tol=GRAD_TOL):
    gmax = np.abs(ref["grad"]).max() if ref.get("grad") is not None else 0.0
    if precision == 32:
        dp = np.abs(got["price"] - ref["price"]).max()
        assert dp < PRICE_TOL, f"{what}: price differs by {dp}"
        assert np.allclose(got["stderr"], ref["stderr"], rtol=1e-4, atol=1e-9), what
        if got.get("grad") is not None:
            dg = np.abs(got["grad"] - ref["grad"]).max()
            say(f"  {what}: max|dprice|={dp:.3g} max|dgrad|/max|g|={dg / gmax:.3g}")
            assert dg <= grad_tol * gmax, f"{what}: bucket error {dg} vs max|g| {gmax}"
            zero = ref["grad"] == 0.0
            assert np.all(got["grad"][zero] == 0.0), f"{what}: zero buckets differ"
    else:
        rel = np.abs(got["price"] - ref["price"]) / np.maximum(np.abs(ref["price"]), 1e-300)
        assert np.all(rel < F64_PRICE_REL), f"{what}: FP64 price rel err {rel.max()}"
        assert np.allclose(got["stderr"], ref["stderr"], rtol=1e-9, atol=1e-15)
        if got.get("grad") is not None:
            dg = np.abs(got["grad"] - ref["grad"]).max()
            say(f"  {what}: FP64 max|dgrad|/max|g|={dg / gmax:.3g}")
            assert dg <= F64_GRAD * gmax
            zero = ref["grad"] == 0.0
            assert np.all(got["grad"][zero] == 0.0)
    if got.get("delta") is not None and ref.get("delta") is not None:
        tol = 1e-4 * max(1.0, abs(ref["delta"])) if precision == 32 else 1e-10 * max(1.0, abs(ref["delta"]))
        assert abs(got["delta"] - ref["delta"]) < tol, f"{what}: delta {got['delta']} vs {ref['delta']}"


# --------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------
def test_philox_words_bit_exact(lv, ctx, orc):
    import torch
    for seed in (0, 0xDEADBEEFCAFEF00D):
        p0, n_p, m0, n_m = 2**32 - 100, 256, 2**32 - 3, 8
        say(f"  philox seed={seed:#x} p0={p0} m0={m0}")
        out = torch.zeros(n_p * n_m * 4, dtype=torch.int32, device="cuda")
        lv._check_status(ctx.lib.lv_debug_philox(ctx.h, seed, m0, n_m, p0, n_p,
                                                  lv._ptr(out)), ctx.h)
        got = out.cpu().numpy().view(np.uint32).reshape(n_p, n_m, 4)
        ref = np.array([[orc.philox_words(seed, m0 + mi, p0 + q) for mi in range(n_m)]
                        for q in range(n_p)], dtype=np.uint32)
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("precision", [32, 64])
def test_normals(lv, ctx, orc, precision):
    import torch
    n_p, N = 512, 64
    dt = torch.float32 if precision == 32 else torch.float64
    out = torch.zeros(n_p * N, dtype=dt, device="cuda")
    say(f"  normals precision={precision}")
    lv._check_status(ctx.lib.lv_debug_normals(ctx.h, precision, 7, 1000, n_p, N, lv._ptr(out)), ctx.h)
    got = out.cpu().double().numpy().reshape(n_p, N)
    ref = orc.normals(7, 1000, n_p, N)
    err = np.abs(got - ref) / (1.0 + np.abs(ref))
    say(f"  normals precision={precision}: max rel err {err.max():.3g}")
    assert err.max() < (2e-6 if precision == 32 else 1e-14)


# --------------------------------------------------------------------------
# pricing parity at sizes the oracle finishes quickly
# --------------------------------------------------------------------------
@pytest.mark.parametrize("precision,adjoint", [(32, "stored"), (64, "stored"), (32, "checkpoint"),
                                               (64, "checkpoint")])
def test_small_call(lv, ctx, orc, precision, adjoint):
    wl = W.small_call()
    s = wl.surface.rounded_to_f32() if precision == 32 else wl.surface
    ref = orc.price_and_grad(s, wl.book, wl.n_paths, wl.n_steps, wl.seed)
    got = gpu_run(lv, ctx, wl.surface, wl.book, wl.n_paths, wl.n_steps, wl.seed,
                  precision=precision, adjoint=adjoint)
    assert_parity(got, ref, precision, f"small call {precision} {adjoint}")


def test_price_only_matches(lv, ctx, orc):
    wl = W.small_call()
    ref = orc.price_and_grad(wl.surface.rounded_to_f32(), wl.book, wl.n_paths, wl.n_steps, want_grad=False)
    p, s, g, d = lv.price_and_grad(wl.surface, 100.0, wl.book.strike, wl.book.maturity, wl.n_paths,
                                   wl.n_steps, 0, adjoint="none", ctx=ctx)
    assert g is None and d is None
    assert abs(p[0] - ref["price"][0]) < PRICE_TOL


def mixed_book():
    return W.Book([0, 1, 0, 1, 0], [100.0, 95.0, 120.0, 80.0, 101.5], [3.0, 1.0, 0.5, 3.0, 2.0],
                  [1.0, 2.0, -0.5, 1.5, 0.25])


def max_book():
    """256 options (the most a book may hold): maturities on every one of 52 weekly
    steps, calls and puts, strikes 70..130, weights of both signs and some zero."""
    k = np.arange(256)
    w = np.where(k % 7 == 3, 0.0, np.cos(0.37 * k))
    return W.Book((k % 3 == 1).astype(np.int32), 70.0 + 60.0 * ((k * 37) % 256) / 255.0,
                  (1 + (k * 11) % 52) / 52.0, w)


@pytest.mark.parametrize("precision,adjoint,block", [(32, "stored", 0), (32, "checkpoint", 0),
                                                     (64, "stored", 0), (32, "stored", 256),
                                                     (64, "checkpoint", 128)])
def test_max_book(lv, ctx, orc, precision, adjoint, block):
    """The largest book, 256 options tapped at 52 different steps, on 4096 + 13 paths
    of the 21 x 13 grid: prices, standard errors, the grid of the weighted book and
    delta against the oracle, with the default and with explicit block sizes (the
    per-wave payoff sums then take most of the LDS).  257 options are refused."""
    wl = W.small_call()
    book = max_book()
    P, N = 4096 + 13, 52
    s = wl.surface.rounded_to_f32() if precision == 32 else wl.surface
    ref = orc.price_and_grad(s, book, P, N, seed=7)
    got = gpu_run(lv, ctx, wl.surface, book, P, N, 7, precision=precision, adjoint=adjoint, block=block)
    assert_parity(got, ref, precision, f"256 options {precision} {adjoint} block {block}")
    big = W.Book(np.zeros(257, np.int32), np.full(257, 100.0), np.full(257, 1.0), np.ones(257))
    with pytest.raises(lv.LVError, match="UNSUPPORTED"):
        gpu_run(lv, ctx, wl.surface, big, P, N, 7, precision=precision)


def large_grid():
    """150 log-spaced spots (20..400) by 80 times (0..2y): 12000 nodes, whose FP64
    gradient grid takes 96 KB of each block's LDS, near the largest a block holds."""
    sa, ta = W.Axis(150, W.LOG, 20.0, 400.0), W.Axis(80, W.LIN, 0.0, 2.0)
    return W.Surface(sa, ta, W.noisy(W.smile_surface(sa, ta, 0.2, 0.15, decay=True), 0.01, 21))


@pytest.mark.parametrize("precision,adjoint", [(32, "stored"), (32, "checkpoint"), (64, "stored")])
def test_large_grid(lv, ctx, orc, precision, adjoint):
    """A 150 x 80 grid with a call and a put on 2^17 + 5 paths and 104 steps against
    the oracle: the planner shrinks the histogram window (and the block) to fit the
    grid in LDS.  A 200 x 100 grid does not fit a block and is refused before any
    launch.  On this noisy grid (about 50 nodes per unit of ln S) a few FP32 paths
    with large adjoints take the neighbouring cell at a node (test_fp32_node_flips
    reproduces it on the oracle), so FP32 is held to the block-paired bar."""
    surf = large_grid()
    book = W.Book([0, 1], [100.0, 90.0], [2.0, 1.0], [1.0, 0.5])
    P, N = (1 << 17) + 5, 104
    s = surf.rounded_to_f32() if precision == 32 else surf
    ref = orc.price_and_grad(s, book, P, N, seed=13)
    got = gpu_run(lv, ctx, surf, book, P, N, 13, precision=precision, adjoint=adjoint)
    if precision == 64:
        assert_parity(got, ref, 64, f"150x80 {precision} {adjoint}")
    else:
        assert_parity(dict(got, grad=None, delta=None), ref, 32, f"150x80 FP32 {adjoint} prices")
        info = ctx.run_info()
        B, T = info["n_blocks"], info["tile_paths"]
        blocks = ctx.block_grads(surf.sigma.size, book.n).reshape((B,) + surf.sigma.shape)
        ob = F.oracle_block_sums(orc, s, book, P, N, 13, B, T)
        F.paired_check(got["grad"], blocks, ob, P, f"150x80 FP32 {adjoint}")
    sa, ta = W.Axis(200, W.LOG, 20.0, 400.0), W.Axis(100, W.LIN, 0.0, 2.0)
    huge = W.Surface(sa, ta, np.full((200, 100), 0.2))
    with pytest.raises(lv.LVError, match="UNSUPPORTED"):
        gpu_run(lv, ctx, huge, book, P, N, 13, precision=precision, adjoint=adjoint)


@pytest.mark.parametrize("precision,adjoint", [(32, "stored"), (64, "stored"), (32, "checkpoint")])
def test_book_log_axis_ragged(lv, ctx, orc, precision, adjoint):
    """Log-spaced 60 x 30 grid, calls and puts of uneven maturity with weights, a path
    count that is not a multiple of the block and 156 steps (not a multiple of 16)."""
    surf = W.book_surface(0)
    book = mixed_book()
    P, N = 20000 + 37, 156
    s = surf.rounded_to_f32() if precision == 32 else surf
    ref = orc.price_and_grad(s, book, P, N, seed=3)
    got = gpu_run(lv, ctx, surf, book, P, N, 3, precision=precision, adjoint=adjoint)
    assert_parity(got, ref, precision, f"book {precision} {adjoint}")


@pytest.mark.parametrize("precision,axis", [(32, "lin"), (64, "lin"), (32, "log"), (64, "log")])
def test_euler_x_scheme(lv, ctx, orc, precision, axis):
    """The explicit Euler step on X itself (scheme euler_x) against the oracle's scheme 1,
    stored adjoint: the linear 21 x 13 grid with one call, and the log-spaced 60 x 30
    grid with calls and puts of uneven maturity, a ragged path count and 156 steps;
    the price-only run gives the same prices."""
    if axis == "lin":
        wl = W.small_call()
        surf, book, P, N, seed = wl.surface, wl.book, wl.n_paths, wl.n_steps, wl.seed
    else:
        surf, book, P, N, seed = W.book_surface(0), mixed_book(), 20000 + 37, 156, 3
    s = surf.rounded_to_f32() if precision == 32 else surf
    ref = orc.price_and_grad(s, book, P, N, seed=seed, scheme=1)
    got = gpu_run(lv, ctx, surf, book, P, N, seed, precision=precision, scheme="euler_x")
    assert_parity(got, ref, precision, f"euler_x {axis} {precision}")
    p, _, _, _ = lv.price_and_grad(surf, 100.0, book.strike, book.maturity, P, N, seed, is_put=book.is_put,
                                   weights=book.weight, ctx=ctx, precision=precision, scheme="euler_x",
                                   adjoint="none", want_grad=False)
    assert np.array_equal(p, got["price"])
    # the two schemes are different estimators of the same model
    lg = gpu_run(lv, ctx, surf, book, P, N, seed, precision=precision)
    assert not np.array_equal(lg["price"], got["price"])


@pytest.mark.parametrize("scheme", ["log_euler", "euler_x"])
def test_grid_30x60(lv, ctx, orc, scheme):
    """The paper's grid orientation, 30 spot by 60 time nodes (log-spaced spots, 3 years),
    with a call and a put: FP32 stored adjoint against the oracle.  2^17 paths: FP32's
    cell flips (a path on the other side of a node than in FP64 takes the other cell's
    slope) move buckets by noise that shrinks as 1/sqrt(paths)."""
    sa, ta = W.Axis(30, W.LOG, 40.0, 250.0), W.Axis(60, W.LIN, 0.0, 3.0)
    surf = W.Surface(sa, ta, W.noisy(W.smile_surface(sa, ta, 0.12, 0.12, decay=False), 0.005, 4))
    book = W.Book([0, 1], [100.0, 90.0], [3.0, 1.5], [1.0, 0.5])
    P, N = (1 << 17) + 5, 156
    ref = orc.price_and_grad(surf.rounded_to_f32(), book, P, N, seed=5, scheme=W_SCHEME[scheme])
    got = gpu_run(lv, ctx, surf, book, P, N, 5, precision=32, scheme=scheme)
    assert_parity(got, ref, 32, f"30x60 {scheme}")


W_SCHEME = {"log_euler": 0, "euler_x": 1}


@pytest.mark.parametrize("precision", [32, 64])
def test_sigma_bf16(lv, ctx, orc, precision):
    """Vol nodes rounded to bfloat16 on the device (option sigma_bf16) on the log-spaced
    60 x 30 grid with calls and puts of uneven maturity, a ragged path count and 156 steps:
    against the oracle on its own rounding of the surface, and bit-identical to a run
    handed that rounded surface with the option off, so the device's rounding is the
    oracle's node for node.  Graph replays with the option on and off keep them apart."""
    surf, book, P, N, seed = W.book_surface(0), mixed_book(), 20000 + 37, 156, 3
    rounded = W.Surface(surf.spot_axis, surf.time_axis, orc.round_bf16(surf.sigma))
    assert not np.array_equal(rounded.sigma, surf.sigma)
    ref = orc.price_and_grad(rounded, book, P, N, seed=seed)
    got = gpu_run(lv, ctx, surf, book, P, N, seed, precision=precision, sigma_bf16=True)
    assert_parity(got, ref, precision, f"sigma_bf16 {precision}")
    pre = gpu_run(lv, ctx, rounded, book, P, N, seed, precision=precision)
    for k in ("price", "stderr", "grad"):
        assert np.array_equal(got[k], pre[k]), k
    assert got["delta"] == pre["delta"]
    plain = gpu_run(lv, ctx, surf, book, P, N, seed, precision=precision)
    assert not np.array_equal(plain["price"], got["price"])
    if precision == 32:
        for on, want in ((True, got), (False, plain), (True, got)):
            g = gpu_run(lv, ctx, surf, book, P, N, seed, precision=32, sigma_bf16=on, use_graph=True)
            assert np.array_equal(g["price"], want["price"]) and np.array_equal(g["grad"], want["grad"])


def segment_edge_book(seg):
    """Options whose maturities fall on the last step of a checkpoint segment, on the
    first step of the next one, and between, with a horizon that ends mid-segment: the
    segments a sweep or forward takes without tap tests sit beside those it cannot."""
    steps = [seg, seg + 1, 2 * seg, 3 * seg - 1, 3 * seg + 1, 4 * seg + 3]   # of 4 seg + 3, over one year
    k = np.arange(len(steps))
    return W.Book((k % 2).astype(np.int32), 90.0 + 4.0 * k, np.array(steps) / (4.0 * seg + 3.0),
                  np.where(k % 3 == 2, -0.5, 1.0))


@pytest.mark.parametrize("precision,seg", [(32, 16), (64, 16), (32, 8), (64, 32)])
def test_checkpoint_taps_at_segment_edges(lv, ctx, orc, precision, seg):
    """The checkpointed kernel runs segments whose steps reach no payoff date without
    the per-step tests: maturities on and beside segment boundaries, and a ragged last
    segment, against the oracle."""
    book = segment_edge_book(seg)
    N = 4 * seg + 3
    surf = W.small_surface()
    s = surf.rounded_to_f32() if precision == 32 else surf
    ref = orc.price_and_grad(s, book, 20000 + 11, N, seed=5)
    got = gpu_run(lv, ctx, surf, book, 20000 + 11, N, 5, precision=precision, adjoint="checkpoint",
                  ckpt_every=seg)
    assert_parity(got, ref, precision, f"segment-edge taps FP{precision} seg {seg}")


@pytest.mark.parametrize("precision,axis,seg", [(32, "lin", 16), (64, "lin", 8), (32, "log", 32),
                                               (64, "log", 16)])
def test_euler_x_checkpoint(lv, ctx, orc, precision, axis, seg):
    """The Euler step on X with the checkpointed adjoint (each segment re-simulated from
    its checkpoint and the Philox counters) against the oracle's scheme 1, on both axis
    kinds and every segment length; the same workloads as the stored-state test."""
    if axis == "lin":
        wl = W.small_call()
        surf, book, P, N, seed = wl.surface, wl.book, wl.n_paths, wl.n_steps, wl.seed
    else:
        surf, book, P, N, seed = W.book_surface(0), mixed_book(), 20000 + 37, 156, 3
    s = surf.rounded_to_f32() if precision == 32 else surf
    ref = orc.price_and_grad(s, book, P, N, seed=seed, scheme=1)
    got = gpu_run(lv, ctx, surf, book, P, N, seed, precision=precision, scheme="euler_x",
                  adjoint="checkpoint", ckpt_every=seg)
    assert_parity(got, ref, precision, f"euler_x checkpoint {axis} {precision} seg {seg}")


@pytest.mark.parametrize("P,N", [(2, 1), (3, 2), (1000, 13), (257, 5)])
def test_degenerate_shapes(lv, ctx, orc, P, N):
    surf = W.tiny_surface(W.LIN, 5, 4, seed=1)
    book = W.Book([0, 1], [100.0, 104.0], [1.0, 1.0], [1.0, -1.0])
    for precision in (32, 64):
        s = surf.rounded_to_f32() if precision == 32 else surf
        ref = orc.price_and_grad(s, book, P, N, seed=11)
        for adjoint in ("stored", "checkpoint"):
            got = gpu_run(lv, ctx, surf, book, P, N, 11, precision=precision, adjoint=adjoint)
            assert_parity(got, ref, precision, f"P={P} N={N} {precision} {adjoint}")


def test_zero_buckets_exact(lv, ctx, orc):
    sa = W.Axis(40, W.LIN, 10.0, 400.0)
    ta = W.Axis(5, W.LIN, 0.0, 2.0)
    rng = np.random.default_rng(2)
    surf = W.Surface(sa, ta, rng.uniform(0.15, 0.3, (40, 5)))
    book = W.call(100.0, 2.0 / 52)
    for precision in (32, 64):
        s = surf.rounded_to_f32() if precision == 32 else surf
        ref = orc.price_and_grad(s, book, 4096, 2, seed=1)
        got = gpu_run(lv, ctx, surf, book, 4096, 2, 1, precision=precision)
        assert np.array_equal(got["grad"] == 0.0, ref["grad"] == 0.0)
        assert_parity(got, ref, precision, f"zero buckets {precision}")


@pytest.mark.parametrize("adjoint,scheme", [("stored", "log_euler"), ("checkpoint", "log_euler"),
                                            ("checkpoint", "euler_x")])
def test_live_path_sweep_matches_dense(lv, ctx, adjoint, scheme):
    """The reverse sweeps visit only paths with an option in the money at its maturity
    (every other path has a zero adjoint): the stored kernel over lists of several
    tiles, the checkpointed kernel per tile, its live paths taken by the first lanes.
    Sweeping every path instead gives the same gradient and delta up to FP64 summation
    order, and the same prices.  A single call (about half its paths are dead) and a
    64-option book whose cotangents are zero for every third option."""
    small = W.small_call()
    b = W.book64()
    w = np.where(np.arange(b.n) % 3 == 0, 0.0, b.weight)
    cases = [(small.surface, small.book, small.n_paths, small.n_steps),
             (W.book_surface(0), W.Book(b.is_put, b.strike, b.maturity, w), 1 << 15, 156)]
    for surf, bk, P, N in cases:
        for precision in (32, 64):
            sp = gpu_run(lv, ctx, surf, bk, P, N, 3, precision=precision, adjoint=adjoint, scheme=scheme)
            de = gpu_run(lv, ctx, surf, bk, P, N, 3, precision=precision, adjoint=adjoint, scheme=scheme,
                         dense_adjoint=True)
            assert np.array_equal(sp["price"], de["price"])
            gmax = np.abs(de["grad"]).max()
            dg = np.abs(sp["grad"] - de["grad"]).max()
            say(f"  live vs dense, {surf.sigma.shape} FP{precision}: max|dgrad|/max|g| {dg / gmax:.3g}, "
                f"delta {sp['delta']:.12g} vs {de['delta']:.12g}")
            assert dg <= 1e-12 * gmax
            assert np.array_equal(sp["grad"] == 0.0, de["grad"] == 0.0)
            assert abs(sp["delta"] - de["delta"]) <= 1e-12 * abs(de["delta"])


@pytest.mark.parametrize("precision", [32, 64])
def test_checkpoint_lists_span_tiles(lv, ctx, orc, precision):
    """The checkpointed kernel with 64-lane blocks, one per CU, on 2^15 + 37 paths: 513
    tiles, more than the blocks, so each block queues the live paths of two or three
    tiles (each tile in its own checkpoint slot set) and the last tile is ragged.
    Against the oracle, and bit-equal gradients to sweeping every path."""
    wl = W.small_call()
    P, N = (1 << 15) + 37, wl.n_steps
    s = wl.surface.rounded_to_f32() if precision == 32 else wl.surface
    ref = orc.price_and_grad(s, wl.book, P, N, seed=wl.seed)
    shape = dict(adjoint="checkpoint", block=64, blocks_per_cu=1, precision=precision)
    got = gpu_run(lv, ctx, wl.surface, wl.book, P, N, wl.seed, **shape)
    info = ctx.run_info()
    assert info["block"] == 64 and 513 > info["n_blocks"], info
    assert_parity(got, ref, precision, f"checkpoint lists over tiles FP{precision}")
    de = gpu_run(lv, ctx, wl.surface, wl.book, P, N, wl.seed, dense_adjoint=True, **shape)
    assert np.array_equal(got["price"], de["price"])
    assert np.abs(got["grad"] - de["grad"]).max() <= 1e-12 * np.abs(de["grad"]).max()
    assert abs(got["delta"] - de["delta"]) <= 1e-12 * abs(de["delta"])


@pytest.mark.parametrize("is_put,strike", [(0, 400.0), (0, 135.0), (0, 100.0), (0, 40.0), (1, 70.0)])
def test_checkpoint_queue_live_fractions(lv, ctx, orc, is_put, strike):
    """The fused kernel's live-path queue at live fractions from none to all: 64-lane
    blocks, one per CU, 2^16 + 5 paths (1025 tiles, 4 or 5 per block, a ring of 4
    checkpoint slot sets).  No live path (a call struck at 400): every tile leaves the
    ring at once; a few (135, the put at 70): the ring fills before a pass does and
    forces partial passes; about half (100); all (40): a full pass per tile.  FP64
    against the oracle at the tight bar, and equal to sweeping every path."""
    s = W.small_surface()
    book = W.Book([is_put], [strike], [1.0], [1.0])
    P, N = (1 << 16) + 5, 52
    ref = orc.price_and_grad(s, book, P, N, seed=2)
    shape = dict(adjoint="checkpoint", block=64, blocks_per_cu=1, precision=64)
    got = gpu_run(lv, ctx, s, book, P, N, 2, **shape)
    info = ctx.run_info()
    assert info["block"] == 64 and info["n_blocks"] <= 256, info
    nz = float(np.mean(ref["grad"] != 0.0))
    say(f"  queue, {'put' if is_put else 'call'} K={strike}: nonzero buckets {nz:.2f}")
    if np.any(ref["grad"]):
        assert_parity(got, ref, 64, f"checkpoint queue K={strike}")
    else:
        assert np.all(got["grad"] == 0.0) and got["delta"] == 0.0
        assert np.allclose(got["price"], ref["price"], rtol=1e-11, atol=1e-300)
    de = gpu_run(lv, ctx, s, book, P, N, 2, dense_adjoint=True, **shape)
    assert np.array_equal(got["price"], de["price"])
    gm = max(np.abs(de["grad"]).max(), 1e-300)
    assert np.abs(got["grad"] - de["grad"]).max() <= 1e-12 * gm
    assert abs(got["delta"] - de["delta"]) <= 1e-12 * max(abs(de["delta"]), 1e-300)


def test_block_shapes_agree(lv, ctx, orc):
    """Every launch shape computes the same thing: block sizes, histogram copies,
    windows and grid sizes all pass the same parity bar."""
    wl = W.small_call()
    ref = orc.price_and_grad(wl.surface.rounded_to_f32(), wl.book, wl.n_paths, wl.n_steps)
    for opts in [dict(block=64), dict(block=128, copies=1), dict(block=512, copies=16),
                 dict(block=256, window=8), dict(block=256, window=32, blocks_per_cu=1),
                 dict(block=1024, copies=4), dict(adjoint="checkpoint", ckpt_every=8),
                 dict(adjoint="checkpoint", ckpt_every=32, block=128)]:
        got = gpu_run(lv, ctx, wl.surface, wl.book, wl.n_paths, wl.n_steps, 0, **opts)
        assert_parity(got, ref, 32, f"shape {opts}")


# --------------------------------------------------------------------------
# batched surfaces, device API, graphs, autograd
# --------------------------------------------------------------------------
@pytest.mark.parametrize("precision", [64, 32])
def test_surface_batch(lv, ctx, orc, precision):
    """Three 100 x 50 surfaces on the same 4096 paths of 260 steps in one batch: FP64
    against the oracle at the tight bar; FP32 prices against the oracle, each surface's
    batch gradient equal to a single-surface call's, and that call's blocks paired
    with the oracle's (the 5-year noisy linear-axis surfaces are where single
    precision leaves cell decisions open)."""
    surfs = [W.wide_surface(s) for s in (1, 2, 3)]
    sig = np.stack([s.sigma for s in surfs])
    book = W.call(100.0, 5.0)
    P, N = 4096, 260
    ax = dict(spot_axis=surfs[0].spot_axis, time_axis=surfs[0].time_axis)
    for adjoint in ("checkpoint", "stored"):
        say(f"  batch of 3 wide surfaces, {adjoint}, FP{precision}")
        p, se, g, d = lv.price_and_grad_batch(sig, 100.0, book.strike, book.maturity, P, N, 0, **ax,
                                              adjoint=adjoint, precision=precision, ctx=ctx)
        for k, s in enumerate(surfs):
            s_ref = s.rounded_to_f32() if precision == 32 else s
            ref = orc.price_and_grad(s_ref, book, P, N)
            got = dict(price=p[k], stderr=se[k], grad=g[k], delta=d[k])
            if precision == 64:
                assert_parity(got, ref, 64, f"batch surface {k} {adjoint}")
                continue
            assert_parity(dict(got, grad=None, delta=None), ref, 32, f"batch surface {k} {adjoint} prices")
            p1, s1, g1, d1 = lv.price_and_grad(s, 100.0, book.strike, book.maturity, P, N, 0, adjoint=adjoint,
                                               ctx=ctx)
            assert np.array_equal(g1, g[k]) and np.array_equal(p1, p[k])
            info = ctx.run_info()
            B, T = info["n_blocks"], info["tile_paths"]
            blocks = ctx.block_grads(s.sigma.size).reshape((B,) + s.sigma.shape)
            ob = F.oracle_block_sums(orc, s_ref, book, P, N, 0, B, T)
            F.paired_check(g[k], blocks, ob, P, f"FP32 surface {k} {adjoint}")


@pytest.mark.parametrize("opts", [dict(), dict(adjoint="checkpoint"),
                                  dict(adjoint="checkpoint", block=64, blocks_per_cu=1, n_paths=(1 << 15) + 37)],
                         ids=["stored", "checkpoint", "checkpoint_lists_over_tiles"])
def test_device_api_and_graph_replay(lv, ctx, opts):
    """Graph replays equal the eager call bit for bit, with eager work of another shape
    between replays: stored states, checkpoints, and checkpoints whose live-path lists
    span two tiles."""
    import torch
    wl = W.small_call()
    opts = dict(opts)
    P = opts.pop("n_paths", wl.n_paths)
    sig = torch.tensor(wl.surface.sigma, dtype=torch.float64, device="cuda")
    kw = dict(spot_axis=wl.surface.spot_axis, time_axis=wl.surface.time_axis, ctx=ctx, **opts)
    say(f"  eager device call {opts}")
    eager = lv.price_and_grad_dev(sig, 100.0, [100.0], [1.0], P, wl.n_steps, 0, **kw)
    eager = [t.clone() for t in eager]
    torch.cuda.synchronize()
    out = [torch.empty_like(t) for t in eager]
    for rep in range(3):
        say(f"  graph replay {rep}")
        lv.price_and_grad_dev(sig, 100.0, [100.0], [1.0], P, wl.n_steps, 0, out=out,
                              use_graph=True, **kw)
        torch.cuda.synchronize()
        assert ctx.run_info()["graph_replayed"] == (1 if rep > 0 else 0)
        # prices are bit-stable; the gradient histogram is integer, so it is too
        for a, b in zip(out, eager):
            assert torch.equal(a, b)
        # eager work between replays
        lv.price_and_grad_dev(sig * 1.01, 100.0, [100.0], [1.0], 1024, wl.n_steps, 5, **kw)
        torch.cuda.synchronize()


def test_autograd_split_matches_fused(lv, ctx):
    import torch
    surf = W.book_surface(0)
    book = mixed_book()
    P, N = 8192 + 5, 156
    sig = torch.tensor(surf.sigma, dtype=torch.float64, device="cuda", requires_grad=True)
    spec = dict(spot=100.0, strikes=book.strike, maturities=book.maturity, is_put=book.is_put,
                n_paths=P, n_steps=N, seed=9, spot_axis=surf.spot_axis, time_axis=surf.time_axis,
                precision=32)
    say("  LVPrice forward/backward")
    price, stderr = lv.LVPrice.apply(sig, spec)
    w = torch.tensor(book.weight, dtype=torch.float64, device="cuda")
    (price * w).sum().backward()
    p, s, g, d = lv.price_and_grad(surf, 100.0, book.strike, book.maturity, P, N, 9,
                                   is_put=book.is_put, weights=book.weight, ctx=ctx)
    assert np.allclose(price.detach().cpu().numpy(), p, rtol=0, atol=1e-12)
    gmax = np.abs(g).max()
    assert np.abs(sig.grad.cpu().numpy() - g).max() <= 1e-6 * gmax


# --------------------------------------------------------------------------
# full size, in the benchmark's launch configuration
# --------------------------------------------------------------------------
def test_per_option_grads_sum_to_book(lv, ctx):
    """Per-option grids (one stored forward, one reverse per option with a one-hot
    cotangent) equal the fused call's grid with that option's weight alone, and add up,
    with the book's weights, to the grid of the weighted book (FP64)."""
    import torch
    s = W.small_surface()
    book = W.Book([0, 1, 0], [100.0, 105.0, 92.0], [1.0, 0.5, 0.75], [1.0, 2.5, -0.7])
    P, N = 8192, 52
    say(f"  per-option grids: {s.sigma.shape} P={P} N={N}")
    sig = torch.tensor(s.sigma, dtype=torch.float64, device="cuda")
    pr, se, grads, deltas = lv.per_option_grads_dev(sig, 100.0, book.strike, book.maturity, P, N, 0,
                                                    spot_axis=s.spot_axis, time_axis=s.time_axis,
                                                    is_put=book.is_put, precision=64, ctx=ctx)
    grads, deltas = grads.cpu().numpy(), deltas.cpu().numpy()
    fused = gpu_run(lv, ctx, s, book, P, N, precision=64)
    scale = np.abs(fused["grad"]).max()
    summed = np.tensordot(book.weight, grads, axes=1)
    assert np.abs(summed - fused["grad"]).max() < 1e-10 * scale
    assert abs(float(np.dot(book.weight, deltas)) - float(np.ravel(fused["delta"])[0])) < 1e-10
    np.testing.assert_allclose(pr.cpu().numpy(), fused["price"], rtol=1e-12, atol=0)
    for k in range(book.n):
        w = np.zeros(book.n)
        w[k] = 1.0
        one = gpu_run(lv, ctx, s, W.Book(book.is_put, book.strike, book.maturity, w), P, N, precision=64)
        sk = max(np.abs(one["grad"]).max(), 1e-300)
        assert np.abs(grads[k] - one["grad"]).max() < 1e-10 * sk, k


def test_bump_and_reprice(lv, ctx, orc):
    """The bumping estimator (Sec. III) on the GPU: FP64, it equals the oracle's at sampled
    nodes on the same paths and agrees with the adjoint grid to the finite-difference
    error (paths whose payoff kink or grid cell changes between the two bumps give an
    O(eps) term: at eps 1e-4 the oracle's own bumping is 5e-5 max|g| off its adjoint on
    this workload, at 1e-5 2e-7); batches of 64 nodes leave a ragged last batch
    (21 x 13 = 273 nodes)."""
    import torch
    s = W.small_surface()
    book = W.call(100.0, 1.0)
    P, N, eps = 16384, 52, 1e-5
    say(f"  bump-and-reprice: {s.sigma.shape} P={P} N={N} eps={eps}")
    sig = torch.tensor(s.sigma, dtype=torch.float64, device="cuda")
    kw = dict(spot_axis=s.spot_axis, time_axis=s.time_axis, is_put=book.is_put, weights=book.weight, ctx=ctx)
    fd = lv.bump_grad_dev(sig, 100.0, book.strike, book.maturity, P, N, 0, eps=eps, batch=64, precision=64,
                          **kw).cpu().numpy()
    ad = gpu_run(lv, ctx, s, book, P, N, precision=64)["grad"]
    scale = np.abs(ad).max()
    err = np.abs(fd - ad).max()
    say(f"  FP64 bump vs adjoint: {err / scale:.3g} max|g|")
    assert err < 1e-5 * scale
    order = np.argsort(-np.abs(ad).ravel())
    nodes = [divmod(int(k), ad.shape[1]) for k in list(order[:4]) + [int(order[40]), int(order[-1])]]
    ref = orc.bump_grad(s, book, P, N, 0, eps, nodes)
    got = np.array([fd[i, j] for i, j in nodes])
    say(f"  FP64 bump vs oracle bump: {np.abs(got - ref).max() / scale:.3g} max|g|")
    assert np.abs(got - ref).max() < 1e-8 * scale
    # FP32 stepping needs a wider bump: its rounding noise in a price difference is
    # divided by eps
    fd32 = lv.bump_grad_dev(sig, 100.0, book.strike, book.maturity, P, N, 0, eps=1e-3, precision=32,
                            **kw).cpu().numpy()
    err32 = np.abs(fd32 - ad).max() / scale
    say(f"  FP32 bump (eps 1e-3) vs FP64 adjoint: {err32:.3g} max|g|")
    assert err32 < 5e-3


def test_bump_and_reprice_rejects_bad_arguments(lv, ctx):
    """A bump that is not finite and positive, or a negative batch, is an argument error
    raised before any launch."""
    import torch
    s = W.small_surface()
    sig = torch.tensor(s.sigma, dtype=torch.float64, device="cuda")
    kw = dict(spot_axis=s.spot_axis, time_axis=s.time_axis, ctx=ctx)
    for eps in (0.0, -1e-3, float("nan"), float("inf")):
        with pytest.raises(lv.LVError, match="ARG"):
            lv.bump_grad_dev(sig, 100.0, [100.0], [1.0], 1024, 52, 0, eps=eps, **kw)
    with pytest.raises(lv.LVError, match="ARG"):
        lv.bump_grad_dev(sig, 100.0, [100.0], [1.0], 1024, 52, 0, eps=1e-3, batch=-1, **kw)


def test_full_size_single_call_60x30(lv, ctx, orc):
    """The 60 x 30 single-call workload at full size (2^19 paths, 156 steps) in the
    benchmark's autotuned launch configuration.  FP64 kernels: the tight bar in both
    adjoint modes.  FP32: price within 1e-5 spot, and the block-paired gradient bar
    (every block's partial sums against the oracle's over the same paths)."""
    wl = W.single_call_60x30()
    s32 = wl.surface.rounded_to_f32()
    say(f"  full-size {wl.name}: oracle ({oracle.default_threads()} threads)")
    ref64 = orc.price_and_grad(wl.surface, wl.book, wl.n_paths, wl.n_steps, wl.seed)
    ref32 = orc.price_and_grad(s32, wl.book, wl.n_paths, wl.n_steps, wl.seed)
    for adjoint in ("stored", "checkpoint"):
        got = gpu_run(lv, ctx, wl.surface, wl.book, wl.n_paths, wl.n_steps, wl.seed,
                      precision=64, adjoint=adjoint)
        assert_parity(got, ref64, 64, f"{wl.name} FP64 {adjoint}")
    for adjoint in ("stored", "checkpoint"):
        got = gpu_run(lv, ctx, wl.surface, wl.book, wl.n_paths, wl.n_steps, wl.seed, adjoint=adjoint,
                      autotune=True)
        info = ctx.run_info()
        assert abs(got["price"][0] - ref32["price"][0]) < PRICE_TOL
        assert np.allclose(got["stderr"], ref32["stderr"], rtol=1e-4)
        B, T = info["n_blocks"], info["tile_paths"]
        blocks = ctx.block_grads(wl.surface.sigma.size).reshape((B,) + wl.surface.sigma.shape)
        say(f"  {wl.name} FP32 {adjoint}: oracle sums over the paths of {B} blocks of tiles of {T}")
        ob = F.oracle_block_sums(orc, s32, wl.book, wl.n_paths, wl.n_steps, wl.seed, B, T)
        assert np.allclose(ob.sum(axis=0) / wl.n_paths, ref32["grad"], rtol=0,
                           atol=1e-12 * np.abs(ref32["grad"]).max())
        F.paired_check(got["grad"], blocks, ob, wl.n_paths, f"{wl.name} FP32 {adjoint}")
    got = gpu_run(lv, ctx, wl.surface, wl.book, wl.n_paths, wl.n_steps, wl.seed, precision=64)
    blocks = ctx.block_grads(wl.surface.sigma.size)
    # the FP64 kernels run a launch shape of their own (at most 512 lanes per block)
    info = ctx.run_info()
    B, T = info["n_blocks"], info["tile_paths"]
    n_tiles = (wl.n_paths + T - 1) // T
    sampled = (0, 1, B // 2, B - 1)
    ranges = {b: [(t * T, min((t + 1) * T, wl.n_paths)) for t in range(b, n_tiles, B)] for b in sampled}
    for b in sampled:
        r = orc.sums(wl.surface, wl.book, wl.n_steps, wl.seed, ranges[b])
        gb = blocks[b].reshape(wl.surface.sigma.shape)
        scale = np.abs(r["sum_grad"]).max()
        e = np.abs(gb - r["sum_grad"]).max()
        say(f"  FP64 block {b}: max err / max|partial| {e / scale:.3g}")
        assert e <= F64_GRAD * scale, f"FP64 block {b}"


@pytest.mark.parametrize("adjoint", ["stored", "checkpoint"])
def test_every_tuning_candidate_passes(lv, ctx, orc, adjoint):
    """The autotuner may pick any of its candidates: each must meet the parity bar."""
    wl = W.small_call()
    ref = orc.price_and_grad(wl.surface.rounded_to_f32(), wl.book, wl.n_paths, wl.n_steps)
    cands = lv.tuning_candidates(wl.surface, wl.book.strike, wl.book.maturity, wl.n_paths,
                                 wl.n_steps, adjoint=adjoint)
    say(f"  {len(cands)} candidates ({adjoint})")
    for block, K, win, bpc, fblock, fbpc in cands:
        opts = dict(block=block, copies=K, blocks_per_cu=bpc, adjoint=adjoint, fwd_block=fblock,
                    fwd_blocks_per_cu=fbpc)
        if adjoint == "stored":
            opts["window"] = win
        got = gpu_run(lv, ctx, wl.surface, wl.book, wl.n_paths, wl.n_steps, 0, **opts)
        assert_parity(got, ref, 32, f"candidate {opts}")


def test_autotune_picks_a_candidate(lv, ctx, orc):
    wl = W.small_call()
    ref = orc.price_and_grad(wl.surface.rounded_to_f32(), wl.book, wl.n_paths, wl.n_steps)
    got = gpu_run(lv, ctx, wl.surface, wl.book, wl.n_paths, wl.n_steps, 0, autotune=True)
    info = ctx.run_info()
    assert info["autotuned"] == 1
    assert_parity(got, ref, 32, "autotuned")
    keys = ("block", "copies", "window", "blocks_per_cu", "fwd_block", "fwd_blocks_per_cu")
    shape = tuple(info[k] for k in keys)
    rows = lv.tuning_candidates(wl.surface, wl.book.strike, wl.book.maturity, wl.n_paths, wl.n_steps)
    assert shape[:4] in {r[:4] for r in rows} and shape[4:] in {r[4:] for r in rows}
    # the second call reuses the tuned shape
    got2 = gpu_run(lv, ctx, wl.surface, wl.book, wl.n_paths, wl.n_steps, 0, autotune=True)
    info2 = ctx.run_info()
    assert tuple(info2[k] for k in keys) == shape
    assert np.array_equal(got2["grad"], got["grad"])


def test_full_size_book64(lv, ctx, orc):
    """64 calls/puts of uneven maturity on one set of 2^20 paths, 156 steps, 60 x 30 grid:
    the fused persistent (checkpoint) kernel and the stored-state pair, autotuned and
    graph-captured.  FP32: prices within 1e-5 spot, block-paired gradient bar; FP64:
    the tight bar."""
    wl = W.book_60x30()
    b = wl.book
    s32 = wl.surface.rounded_to_f32()
    say(f"  {wl.name}: oracle")
    ref32 = orc.price_and_grad(s32, b, wl.n_paths, wl.n_steps, wl.seed)
    for adjoint in ("checkpoint", "stored"):
        got = gpu_run(lv, ctx, wl.surface, b, wl.n_paths, wl.n_steps, wl.seed, adjoint=adjoint,
                      autotune=True, use_graph=True)
        dp = np.abs(got["price"] - ref32["price"]).max()
        info = ctx.run_info()
        say(f"  book FP32 {adjoint}: max |dprice| over 64 options {dp:.3g}; launch {info}")
        assert dp < PRICE_TOL
        assert np.allclose(got["stderr"], ref32["stderr"], rtol=1e-4, atol=1e-9)
        B, T = info["n_blocks"], info["tile_paths"]
        blocks = ctx.block_grads(wl.surface.sigma.size, b.n).reshape((B,) + wl.surface.sigma.shape)
        ob = F.oracle_block_sums(orc, s32, b, wl.n_paths, wl.n_steps, wl.seed, B, T)
        F.paired_check(got["grad"], blocks, ob, wl.n_paths, f"book FP32 {adjoint}")
    ref64 = orc.price_and_grad(wl.surface, b, wl.n_paths, wl.n_steps, wl.seed)
    got = gpu_run(lv, ctx, wl.surface, b, wl.n_paths, wl.n_steps, wl.seed, precision=64, adjoint="checkpoint")
    assert_parity(got, ref64, 64, "book FP64 checkpoint")


def test_full_size_precision_study(lv, ctx, orc):
    """2^22 paths, 52 steps: FP32 and FP64 GPU against the oracle on the 21 x 13 smile
    surface; on a flat 0.2 surface also against Black-Scholes price and vega."""
    from tests import closed_forms as cf
    for flat in (False, True):
        wl = W.precision_study(flat)
        say(f"  {wl.name}: oracle")
        ref32 = orc.price_and_grad(wl.surface.rounded_to_f32(), wl.book, wl.n_paths, wl.n_steps)
        ref64 = orc.price_and_grad(wl.surface, wl.book, wl.n_paths, wl.n_steps)
        g32 = gpu_run(lv, ctx, wl.surface, wl.book, wl.n_paths, wl.n_steps)
        g64 = gpu_run(lv, ctx, wl.surface, wl.book, wl.n_paths, wl.n_steps, precision=64)
        assert_parity(g32, ref32, 32, f"{wl.name} FP32")
        assert_parity(g64, ref64, 64, f"{wl.name} FP64")
        if flat:
            bs = cf.bs_call(100.0, 100.0, 0.04)
            vega = cf.bs_vega(100.0, 100.0, 0.2, 1.0)
            assert abs(g32["price"][0] - bs) < 4 * g32["stderr"][0]
            say(f"  flat: price {g32['price'][0]:.5f} vs BS {bs:.5f} (stderr {g32['stderr'][0]:.2g}); "
                f"sum grad {g32['grad'].sum():.4f} vs vega {vega:.4f}")
            assert abs(g32["grad"].sum() - vega) < 0.01 * vega


def test_full_size_surface_batch(lv, ctx, orc):
    """32 perturbed 100 x 50 surfaces, 2^24 paths, 260 steps, checkpointed adjoint, in
    the benchmark's launch: FP32 payoff sums of sampled blocks of the last surface
    against the oracle, the FP64 kernels' price there, and their gradient partials on
    sampled blocks against the oracle at the tight bar."""
    wl = W.surface_batch()
    sig = np.stack([s.sigma for s in wl.surfaces])
    b = wl.book
    ax = dict(spot_axis=wl.surface.spot_axis, time_axis=wl.surface.time_axis)
    say(f"  {wl.name}: FP32 batch of {len(wl.surfaces)} on the GPU")
    p, se_, g, d = lv.price_and_grad_batch(sig, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps,
                                           0, adjoint="checkpoint", ctx=ctx, **ax)
    info = ctx.run_info()
    part32 = ctx.block_partials(1, sig[0].size)
    B, T = info["n_blocks"], info["tile_paths"]
    n_tiles = (wl.n_paths + T - 1) // T
    last = wl.surfaces[-1]
    # FP32 payoff sums of sampled blocks of the last surface vs the oracle
    for blk in (0, B - 1):
        ranges = [(t * T, min((t + 1) * T, wl.n_paths)) for t in range(blk, n_tiles, B)]
        r = orc.sums(last.rounded_to_f32(), b, wl.n_steps, 0, ranges, want_grad=False)
        n_b = sum(e - a for a, e in ranges)
        dp = abs(part32["sum_pay"][blk, 0] - r["sum_pay"][0]) / n_b
        say(f"  FP32 block {blk}: payoff mean differs by {dp:.3g}")
        assert dp < PRICE_TOL
    # the FP64 kernels on the last surface (their block partials are checked below);
    # the FP32 gradient against the oracle is test_gpu_fp32_accuracy's
    s = last
    say("  last surface: FP64 on the GPU")
    p64, s64, g64, d64 = lv.price_and_grad(s, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps,
                                           0, precision=64, adjoint="checkpoint", ctx=ctx)
    assert abs(p[-1][0] - p64[0]) < PRICE_TOL
    assert abs(se_[-1][0] / s64[0] - 1) < 1e-4
    part64 = ctx.block_partials(1, sig[0].size)
    info64 = ctx.run_info()
    # the FP64 kernel against the oracle on sampled blocks of the last surface
    B, T = info64["n_blocks"], info64["tile_paths"]
    n_tiles = (wl.n_paths + T - 1) // T
    for blk in (0, B // 2, B - 1):
        ranges = [(t * T, min((t + 1) * T, wl.n_paths)) for t in range(blk, n_tiles, B)]
        say(f"  FP64 block {blk}: oracle over {sum(e - a for a, e in ranges)} paths")
        r = orc.sums(last, b, wl.n_steps, 0, ranges)
        scale = np.abs(r["sum_grad"]).max()
        e = np.abs(part64["grad"][blk].reshape(last.sigma.shape) - r["sum_grad"]).max()
        say(f"  FP64 block {blk}: grad err / max|partial| {e / scale:.3g}")
        assert e <= F64_GRAD * scale
        assert abs(part64["sum_pay"][blk, 0] / r["sum_pay"][0] - 1) < 1e-12

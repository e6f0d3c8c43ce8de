"""The allocation-free entry point (lv_price_and_grad_noalloc) against the allocating
one (lv_price_and_grad_dev): same kernels, same launch shapes, so the same results,
on two calls in a row (the second smaller), with no change in the GPU's free memory
across them; requests beyond its fixed workspace, and options it does not take, are
refused before anything is launched."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cases():
    big = W.small_call()                                   # 16384 paths x 52 steps, 21 x 13
    b3 = W.Book([0, 1, 0], [95.0, 105.0, 100.0], [0.5, 1.0, 0.25], [1.0, -0.5, 2.0])
    return [
        dict(name="call 16384 x 52, FP32 checkpoint", surface=big.surface, book=big.book, P=big.n_paths,
             N=big.n_steps, opts=dict(adjoint="checkpoint")),
        dict(name="3 options 4133 x 52, FP64 stored", surface=big.surface, book=b3, P=4133, N=52,
             opts=dict(adjoint="stored", precision=64)),
    ]


def _alloc(torch, n_opt, shape, dev):
    f = lambda *s: torch.full(s, float("nan"), dtype=torch.float64, device=dev)
    return f(1, n_opt), f(1, n_opt), f(1, *shape), f(1)


def test_noalloc_matches_the_allocating_entry_point():
    import torch

    import paper_2002_02481_amd as lv
    dev = torch.device("cuda:0")
    ctx = lv.Context(0)
    cases = _cases()
    sig, ref, got = [], [], []
    for c in cases:
        s, b = c["surface"], c["book"]
        sig.append(torch.tensor(s.sigma, dtype=torch.float64, device=dev))
        kw = dict(spot_axis=s.spot_axis, time_axis=s.time_axis, is_put=b.is_put, weights=b.weight, ctx=ctx)
        say(f"  allocating entry point: {c['name']}")
        ref.append(lv.price_and_grad_dev(sig[-1], 100.0, b.strike, b.maturity, c["P"], c["N"], 0, **kw,
                                         **c["opts"]))
        got.append(_alloc(torch, b.n, s.sigma.shape, dev))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for c, sg, o in zip(cases, sig, got):               # two calls in a row, the second smaller
        s, b = c["surface"], c["book"]
        say(f"  allocation-free entry point: {c['name']}")
        lv.price_and_grad_noalloc(sg, 100.0, b.strike, b.maturity, c["P"], c["N"], 0, spot_axis=s.spot_axis,
                                  time_axis=s.time_axis, is_put=b.is_put, weights=b.weight, out=o, ctx=ctx,
                                  **c["opts"])
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say(f"  free device memory before {free0}, after {free1}")
    assert free1 == free0
    for c, r, g in zip(cases, ref, got):
        r = [t.cpu().numpy() for t in r]
        g = [t.cpu().numpy() for t in g]
        gmax = np.abs(r[2]).max()
        dg = np.abs(g[2] - r[2]).max()
        say(f"  {c['name']}: prices equal {np.array_equal(g[0], r[0])}, grads equal "
            f"{np.array_equal(g[2], r[2])}, max|dgrad|/max|g| {dg / gmax:.3g}")
        assert np.all(np.isfinite(g[0])) and np.all(np.isfinite(g[2]))
        assert np.array_equal(g[0], r[0]) and np.array_equal(g[1], r[1])
        assert dg <= 1e-12 * gmax
        assert np.all(g[2][r[2] == 0.0] == 0.0)
        assert abs(g[3][0] - r[3][0]) <= 1e-12 * max(1.0, abs(r[3][0]))


def test_noalloc_refuses_what_it_cannot_do():
    import torch

    import paper_2002_02481_amd as lv
    dev = torch.device("cuda:0")
    ctx = lv.Context(0)
    wl = W.single_call_60x30()                     # stored states: 327 MB, beyond the workspace
    s, b = wl.surface, wl.book
    sg = torch.tensor(s.sigma, dtype=torch.float64, device=dev)
    out = _alloc(torch, b.n, s.sigma.shape, dev)
    kw = dict(spot_axis=s.spot_axis, time_axis=s.time_axis, out=out, ctx=ctx)
    with pytest.raises(lv.LVError, match="UNSUPPORTED"):
        lv.price_and_grad_noalloc(sg, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, 0, **kw)
    for bad in (dict(use_graph=True), dict(autotune=True), dict(profile=True)):
        with pytest.raises(lv.LVError, match="ARG"):
            lv.price_and_grad_noalloc(sg, 100.0, b.strike, b.maturity, 4096, wl.n_steps, 0, **kw, **bad)
    torch.cuda.synchronize()
    assert torch.isnan(out[0]).all()               # nothing was launched
    # the checkpointed adjoint of the same workload fits and runs
    lv.price_and_grad_noalloc(sg, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, 0, adjoint="checkpoint",
                              **kw)
    ref = lv.price_and_grad_dev(sg, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, 0, adjoint="checkpoint",
                                spot_axis=s.spot_axis, time_axis=s.time_axis, ctx=ctx)
    torch.cuda.synchronize()
    assert torch.equal(out[0], ref[0])
    d = (out[2] - ref[2]).abs().max().item() / ref[2].abs().max().item()
    say(f"  {wl.name} checkpoint: max|dgrad|/max|g| {d:.3g}")
    assert d <= 1e-12

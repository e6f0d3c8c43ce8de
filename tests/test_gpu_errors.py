"""Error paths on the device: a workspace the GPU cannot hold is refused with
LV_ERR_NOMEM before anything is launched, and the context stays usable."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lv():
    import paper_2002_02481_amd as m
    return m


def _small(lv, ctx):
    import torch
    wl = W.small_call()
    s, b = wl.surface, wl.book
    sig = torch.tensor(s.sigma, dtype=torch.float64, device="cuda")
    out = lv.price_and_grad_dev(sig, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, wl.seed,
                                spot_axis=s.spot_axis, time_axis=s.time_axis, adjoint="stored", ctx=ctx)
    return [t.cpu().numpy() for t in out]


def test_state_buffer_beyond_hbm_is_nomem_and_the_context_recovers(lv):
    """2^36 paths x 156 steps of stored FP32 states (43 TB) on a 60 x 30 grid: the
    planner accepts the request, the state buffer's allocation fails, the call returns
    LV_ERR_NOMEM, and the same context then prices a valid request exactly as a fresh
    context does."""
    import torch
    P, N = 1 << 36, 156
    need = lv.states_bytes(32, P, N)
    assert need > 4 * torch.cuda.get_device_properties(0).total_memory
    ctx = lv.Context(0)
    before = _small(lv, ctx)
    s = W.book_surface(0)
    sig = torch.tensor(s.sigma, dtype=torch.float64, device="cuda")
    with pytest.raises(lv.LVError) as ei:
        lv.price_and_grad_dev(sig, 100.0, [100.0], [3.0], P, N, 0, spot_axis=s.spot_axis,
                              time_axis=s.time_axis, adjoint="stored", ctx=ctx)
    assert ei.value.status == lv._lib.LV_ERR_NOMEM, str(ei.value)
    torch.cuda.synchronize()
    after = _small(lv, ctx)
    fresh = _small(lv, lv.Context(0))
    for a, b, c in zip(before, after, fresh):
        assert np.array_equal(a, b) and np.array_equal(b, c)


def test_device_tensors_are_checked_before_anything_runs(lv):
    """The binding hands the library plain device pointers, so it checks each tensor's
    type, shape, layout and extent first: a wrong one is a ValueError, nothing is
    launched, and the context then prices as a fresh one does."""
    import torch
    wl = W.small_call()
    s, b = wl.surface, wl.book
    ax = dict(spot_axis=s.spot_axis, time_axis=s.time_axis)
    sig = torch.tensor(s.sigma, dtype=torch.float64, device="cuda")
    ctx = lv.Context(0)
    args = (100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, wl.seed)
    small = torch.empty(0, dtype=torch.float64, device="cuda")
    one = torch.empty(1, dtype=torch.float64, device="cuda")
    _, _, states = lv.forward_dev(sig, *args, ctx=ctx, **ax)
    torch.cuda.synchronize()
    bad = [
        (lambda: lv.price_and_grad_dev(sig.float(), *args, ctx=ctx, **ax), "float64"),
        (lambda: lv.price_and_grad_dev(sig[:-1], *args, ctx=ctx, **ax), "shape"),
        (lambda: lv.price_and_grad_dev(sig.t(), *args, ctx=ctx, **ax), "contiguous"),
        (lambda: lv.price_and_grad_dev(sig, *args, ctx=ctx, out=(small, one, None, None), **ax), "are needed"),
        (lambda: lv.bump_grad_dev(sig, *args, ctx=ctx, out=small, **ax), "are needed"),
        (lambda: lv.forward_dev(sig, *args, ctx=ctx, states=torch.empty(16, dtype=torch.uint8, device="cuda"),
                                **ax), "bytes"),
        (lambda: lv.backward_dev(sig, *args, states[:16], [1.0], ctx=ctx, **ax), "bytes"),
        (lambda: lv.backward_dev(sig, *args, states, [1.0, 2.0], ctx=ctx, **ax), "cotangent"),
    ]
    for k, (f, msg) in enumerate(bad):
        with pytest.raises(ValueError, match=msg):
            f()
    got = _small(lv, ctx)
    ref = _small(lv, lv.Context(0))
    for x, y in zip(got, ref):
        assert np.array_equal(x, y)

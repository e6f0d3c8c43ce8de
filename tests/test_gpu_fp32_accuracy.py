"""FP32 kernels against the FP64 oracle on the workloads where single precision leaves
some cell decisions open (tests/fp32_checks.py gives the reasoning and the bars):
the FP32 states path by path within the oracle's single-precision bound, and the
gradient of the long-horizon 100 x 50 surfaces block-paired with the oracle."""
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


def _sample(P, extra=()):
    """192 paths spread over [0, P), the first and last, and any named ones."""
    ps = set(np.linspace(0, P - 1, 192).astype(np.int64).tolist()) | {0, P - 1} | {p for p in extra if p < P}
    return np.array(sorted(ps), dtype=np.int64)


@pytest.mark.parametrize("name", ["small_call", "single_call_60x30", "surface_batch"])
def test_fp32_states_within_the_single_precision_bound(lv, ctx, orc, name):
    """The split forward's stored FP32 states of sampled paths against the oracle's
    FP64 states: every one within the oracle's running first-order bound on a
    single-precision computation of that path (for the 100 x 50 surfaces: surface 1
    on the first 2^20 of the batch's paths); prices within 1e-5 spot."""
    import torch
    wl = getattr(W, name)()
    P = min(wl.n_paths, 1 << 20)
    s, b, N = wl.surface, wl.book, wl.n_steps
    s32 = s.rounded_to_f32()
    sig = torch.tensor(s.sigma, dtype=torch.float64, device="cuda")
    F.say(f"  {wl.name}: split forward of {P} paths")
    price, stderr, states = lv.forward_dev(sig, 100.0, b.strike, b.maturity, P, N, wl.seed,
                                           spot_axis=s.spot_axis, time_axis=s.time_axis, is_put=b.is_put,
                                           ctx=ctx)
    paths = _sample(P, extra=(13366,))
    idx = torch.tensor(paths, device="cuda")
    y_gpu = states.view(torch.float32).view(N, P).index_select(1, idx).t().double().cpu().numpy()
    ref = orc.price_and_grad(s32, b, P, N, wl.seed, want_grad=False)
    assert np.abs(price.cpu().numpy() - ref["price"]).max() < PRICE_TOL
    F.states_within_bound(orc, s32, b, N, wl.seed, paths, y_gpu, f"{wl.name} FP32 states")


@pytest.mark.parametrize("k", [1, 32])
def test_long_horizon_surfaces_against_the_oracle(lv, ctx, orc, k):
    """Surfaces 1 and 32 of the 32-surface workload (100 x 50, 260 steps) on its first
    2^20 paths, with its checkpointed adjoint: FP64 against the oracle at the tight bar
    on the whole grid, FP32 prices within 1e-5 spot and the block-paired gradient bar."""
    import torch
    wl = W.surface_batch()
    s, b, N = wl.surfaces[k - 1], wl.book, wl.n_steps
    P = 1 << 20
    s32 = s.rounded_to_f32()
    sig = torch.tensor(s.sigma, dtype=torch.float64, device="cuda")
    kw = dict(spot_axis=s.spot_axis, time_axis=s.time_axis, adjoint="checkpoint", ckpt_every=wl.ckpt_every,
              ctx=ctx)
    F.say(f"  surface {k}: FP64 on the GPU and the oracle, {P} paths x {N} steps")
    g64 = [t.cpu().numpy() for t in lv.price_and_grad_dev(sig, 100.0, b.strike, b.maturity, P, N, wl.seed,
                                                            precision=64, **kw)]
    ref64 = orc.price_and_grad(s, b, P, N, wl.seed)
    assert abs(g64[0][0, 0] / ref64["price"][0] - 1) < 1e-11
    gmax = np.abs(ref64["grad"]).max()
    assert np.abs(g64[2][0] - ref64["grad"]).max() <= 1e-9 * gmax
    F.say(f"  surface {k}: FP32 on the GPU")
    out = [t.cpu().numpy() for t in lv.price_and_grad_dev(sig, 100.0, b.strike, b.maturity, P, N, wl.seed, **kw)]
    info = ctx.run_info()
    B, T = info["n_blocks"], info["tile_paths"]
    blocks = ctx.block_grads(s.sigma.size).reshape((B,) + s.sigma.shape)
    F.say(f"  surface {k}: oracle sums over the paths of {B} blocks of tiles of {T}")
    ob = F.oracle_block_sums(orc, s32, b, P, N, wl.seed, B, T)
    ref32_price = orc.price_and_grad(s32, b, P, N, wl.seed, want_grad=False)["price"]
    assert abs(out[0][0, 0] - ref32_price[0]) < PRICE_TOL
    F.paired_check(out[2][0], blocks, ob, P, f"surface {k} FP32 (2^20 x {N})")

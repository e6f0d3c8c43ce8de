"""C ABI checks that need no GPU: the library loads, exports every function that
include/lvmc.h declares, and rejects bad requests on the host."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from paper_2002_02481_amd import _lib
import paper_2002_02481_amd as lv


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_header_symbol(lib):
    names = _lib.header_symbols()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), f"{n} declared in lvmc.h but not exported"
    assert set(names) == set(_lib.SIGNATURES), "binding signatures out of sync with the header"


def _req(**kw):
    s = W.small_surface()
    args = dict(surface=s, spot=100.0, strikes=[100.0], maturities=[1.0], n_paths=1024, n_steps=52)
    args.update(kw)
    return args


def test_check_accepts_valid_requests():
    assert lv.check(**_req()) == _lib.LV_OK
    b = W.book64()
    assert lv.check(W.book_surface(0), 100.0, b.strike, b.maturity, 1 << 20, 156,
                    is_put=b.is_put, weights=b.weight) == _lib.LV_OK
    assert lv.check(**_req(), precision=64, adjoint="checkpoint", ckpt_every=8) == _lib.LV_OK


@pytest.mark.parametrize("kw,status", [
    (dict(spot=-1.0), _lib.LV_ERR_ARG),
    (dict(spot=float("nan")), _lib.LV_ERR_ARG),
    (dict(strikes=[0.0]), _lib.LV_ERR_ARG),
    (dict(maturities=[-1.0]), _lib.LV_ERR_ARG),
    (dict(n_paths=1), _lib.LV_ERR_ARG),
    (dict(n_steps=0), _lib.LV_ERR_ARG),
    (dict(strikes=[100.0, 90.0], maturities=[1.0, 0.3]), _lib.LV_ERR_STEP),
    (dict(precision=16), _lib.LV_ERR_ARG),
    (dict(adjoint=7), _lib.LV_ERR_ARG),
    (dict(ckpt_every=12), _lib.LV_ERR_ARG),
    (dict(block=100), _lib.LV_ERR_ARG),
    (dict(copies=17), _lib.LV_ERR_ARG),
    (dict(window=4), _lib.LV_ERR_ARG),
    (dict(window=12), _lib.LV_ERR_ARG),
    (dict(precision=64, block=1024), _lib.LV_ERR_UNSUPPORTED),
    (dict(strikes=np.full(300, 100.0), maturities=np.full(300, 1.0)), _lib.LV_ERR_UNSUPPORTED),
])
def test_check_rejects(kw, status):
    assert lv.check(**_req(**kw)) == status


def test_check_rejects_bad_grids():
    s = W.small_surface()
    bad = s.sigma.copy(); bad[3, 4] = -0.1
    assert lv.check(bad, 100.0, [100.0], [1.0], 64, 52, spot_axis=s.spot_axis,
                    time_axis=s.time_axis) == _lib.LV_ERR_GRID
    bad[3, 4] = np.inf
    assert lv.check(bad, 100.0, [100.0], [1.0], 64, 52, spot_axis=s.spot_axis,
                    time_axis=s.time_axis) == _lib.LV_ERR_GRID
    assert lv.check(s.sigma[:1], 100.0, [100.0], [1.0], 64, 52, spot_axis=(1, 0, 50.0, 200.0),
                    time_axis=s.time_axis) == _lib.LV_ERR_GRID
    assert lv.check(s.sigma, 100.0, [100.0], [1.0], 64, 52, spot_axis=(21, 1, 0.0, 200.0),
                    time_axis=s.time_axis) == _lib.LV_ERR_GRID
    assert lv.check(s.sigma, 100.0, [100.0], [1.0], 64, 52, spot_axis=(21, 0, 200.0, 50.0),
                    time_axis=s.time_axis) == _lib.LV_ERR_GRID


def test_error_message_is_set(lib):
    s = W.small_surface()
    lv.check(s, -1.0, [100.0], [1.0], 64, 52)
    assert b"spot" in lib.lv_last_error(None)


def test_states_bytes():
    assert lv.states_bytes(32, 524288, 156) == 524288 * 156 * 4
    assert lv.states_bytes(64, 1000, 13) == 1000 * 13 * 8
    with pytest.raises(lv.LVError):
        lv.states_bytes(16, 1000, 13)


def test_null_context_is_rejected(lib):
    st = lib.lv_price_and_grad(None, None, None, 100.0, None, 64, 52, 0, None, None, None, None, None)
    assert st == _lib.LV_ERR_ARG


def test_tuning_candidates_are_valid_shapes():
    s = W.book_surface(0)
    for adjoint in ("stored", "checkpoint"):
        c = lv.tuning_candidates(s, [100.0], [3.0], 524288, 156, adjoint=adjoint)
        assert len(c) >= 4
        for block, K, win, bpc, fblock, fbpc in c:
            assert block % 64 == 0 and 64 <= block <= 1024 and fblock % 64 == 0 and fblock <= 1024
            assert K in (1, 2, 4) and bpc in (1, 2, 4) and fbpc in (1, 2, 4, 8)
            assert win % 4 == 0
        if adjoint == "checkpoint":
            assert all(r[2] == 16 for r in c)
        else:
            assert len({(r[4], r[5]) for r in c}) > 1      # forward shapes are tuned too
    small = lv.tuning_candidates(W.small_surface(), [100.0], [1.0], 16384, 52)
    assert all(r[0] <= 128 and r[4] <= 128 for r in small)


def test_copies_must_be_power_of_two():
    assert lv.check(**_req(), copies=3) == _lib.LV_ERR_ARG


def test_planned_histogram_window_fits_lds():
    """Every launch shape the checker accepts has a histogram window whose block fits the
    CU's LDS (the planner refuses, with a 'planner:' message, if its window search
    ever overshoots); shapes that cannot fit at all are refused by size."""
    b = W.book64()
    reqs = [_req(n_paths=1 << 19, n_steps=156),
            dict(surface=W.book_surface(0), spot=100.0, strikes=b.strike, maturities=b.maturity,
                 n_paths=1 << 20, n_steps=156, is_put=b.is_put, weights=b.weight)]
    n_ok = 0
    for req in reqs:
        for prec, blocks in ((32, (128, 256, 512, 1024)), (64, (128, 256, 512))):
            for block in blocks:
                for k in (1, 2, 4, 8, 16):
                    for win in (8, 16, 32, 64):
                        st = lv.check(**req, precision=prec, block=block, copies=k, window=win)
                        msg = _lib.load().lv_last_error(None).decode() if st else ""
                        assert not msg.startswith("planner"), (prec, block, k, win, msg)
                        assert st in (_lib.LV_OK, _lib.LV_ERR_UNSUPPORTED), (prec, block, k, win, st)
                        n_ok += st == _lib.LV_OK
    assert n_ok > 100


def test_check_scheme_options():
    """The Euler step on X is planned in every adjoint mode; an unknown scheme is an
    argument error."""
    for adj in ("stored", "checkpoint", "none"):
        assert lv.check(**_req(), scheme="euler_x", adjoint=adj) == _lib.LV_OK
    assert lv.check(**_req(), scheme=7) == _lib.LV_ERR_ARG
    assert lv.check(**_req(), scheme=-1) == _lib.LV_ERR_ARG


def test_check_sigma_bf16_option():
    """Rounding the vol nodes to bfloat16 is a switch: 0 and 1 plan in every adjoint mode
    and precision, anything else is an argument error."""
    for adj in ("stored", "checkpoint", "none"):
        for prec in (32, 64):
            assert lv.check(**_req(), sigma_bf16=1, adjoint=adj, precision=prec) == _lib.LV_OK
    assert lv.check(**_req(), sigma_bf16=0) == _lib.LV_OK
    assert lv.check(**_req(), sigma_bf16=2) == _lib.LV_ERR_ARG
    assert lv.check(**_req(), sigma_bf16=-1) == _lib.LV_ERR_ARG


def test_grid_larger_than_a_block_is_refused():
    """A gradient grid that no block's LDS can hold (200 x 100 nodes) is refused by the
    planner with LV_ERR_UNSUPPORTED in every mode; 150 x 80 plans."""
    for (I, J), want in (((150, 80), _lib.LV_OK), ((200, 100), _lib.LV_ERR_UNSUPPORTED)):
        sa, ta = W.Axis(I, W.LOG, 20.0, 400.0), W.Axis(J, W.LIN, 0.0, 2.0)
        s = W.Surface(sa, ta, np.full((I, J), 0.2))
        for prec in (32, 64):
            for adj in ("stored", "checkpoint"):
                assert lv.check(s, 100.0, [100.0], [2.0], 1 << 13, 104, precision=prec, adjoint=adj) == want


def test_tile_counts_fit_the_kernels():
    """Path tiles are counted in 64 bits: a request whose tile count would not fit the
    kernels' int tile loops is refused (2^38 + 320 paths in 64-lane blocks is 2^32 + 5
    tiles, which an int cast would turn into 5), while 2^40 paths plan with the default
    shapes (1024-lane blocks, 2^30 tiles) and one path more is an argument error."""
    big = (1 << 38) + 320
    assert lv.check(**_req(n_paths=big), block=64) == _lib.LV_ERR_UNSUPPORTED
    assert b"tiles" in _lib.load().lv_last_error(None)
    assert lv.check(**_req(n_paths=big), fwd_block=64) == _lib.LV_ERR_UNSUPPORTED
    assert lv.check(**_req(n_paths=big)) == _lib.LV_OK
    for adj in ("stored", "checkpoint", "none"):
        assert lv.check(**_req(n_paths=1 << 40), adjoint=adj) == _lib.LV_OK
    assert lv.check(**_req(n_paths=1 << 40), block=512) == _lib.LV_ERR_UNSUPPORTED
    assert lv.check(**_req(n_paths=1 << 40), precision=64) == _lib.LV_ERR_UNSUPPORTED
    assert lv.check(**_req(n_paths=(1 << 40) + 1)) == _lib.LV_ERR_ARG


def test_create_without_a_device_is_a_hip_error(lib):
    """With no HIP device (this runs on a host without a GPU) lv_create returns
    LV_ERR_HIP, names the cause and leaves the out-pointer NULL; host-only calls keep
    working afterwards."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present; the no-device path is checked on a host without one")
    h = C.c_void_p(1)
    assert lib.lv_create(C.byref(h), 0, None) == _lib.LV_ERR_HIP
    assert h.value is None
    assert b"device" in lib.lv_last_error(None)
    assert lv.check(**_req()) == _lib.LV_OK


def test_rate_is_validated():
    """A rate is any finite r with |r| <= 1 in every mode and scheme; NaN, inf or a larger
    magnitude is an argument error."""
    for adj in ("stored", "checkpoint", "none"):
        for scheme in ("log_euler", "euler_x"):
            assert lv.check(**_req(), rate=0.05, adjoint=adj, scheme=scheme) == _lib.LV_OK
    assert lv.check(**_req(), rate=-1.0) == _lib.LV_OK
    for bad in (float("nan"), float("inf"), 1.5, -2.0):
        assert lv.check(**_req(), rate=bad) == _lib.LV_ERR_ARG


def test_device_calls_refuse_host_tensors():
    """The calls that hand device pointers to the library check every tensor before a
    context is made or anything is launched: host tensors are refused (no GPU needed)."""
    import torch
    s = W.small_surface()
    ax = dict(spot_axis=s.spot_axis, time_axis=s.time_axis)
    sig = torch.tensor(s.sigma, dtype=torch.float64)
    calls = [
        lambda: lv.price_and_grad_dev(sig, 100.0, [100.0], [1.0], 1024, 52, **ax),
        lambda: lv.price_and_grad_noalloc(sig, 100.0, [100.0], [1.0], 1024, 52, out=(None,) * 4, **ax),
        lambda: lv.bump_grad_dev(sig, 100.0, [100.0], [1.0], 1024, 52, **ax),
        lambda: lv.forward_dev(sig, 100.0, [100.0], [1.0], 1024, 52, 0, **ax),
        lambda: lv.backward_dev(sig, 100.0, [100.0], [1.0], 1024, 52, 0, None, [1.0], **ax),
        lambda: lv.per_option_grads_dev(sig, 100.0, [100.0], [1.0], 1024, 52, **ax),
    ]
    for k, f in enumerate(calls):
        with pytest.raises(ValueError, match="CUDA tensor"):
            f()


def test_planned_checkpoint_table_window_fits_lds():
    """The checkpointed kernel stages its vol table one, two or four segments at a time,
    as many as fit beside the smallest histogram window: on the 100 x 50 batch surface
    and on a 150 x 80 grid near the LDS limit, every block size, copy count, segment
    length and precision the checker accepts is planned without a 'planner:' refusal."""
    big = W.Surface(W.Axis(150, W.LOG, 20.0, 400.0), W.Axis(80, W.LIN, 0.0, 2.0),
                    np.full((150, 80), 0.2))
    reqs = [_req(surface=W.surface_batch(1).surfaces[0], maturities=[5.0], n_paths=1 << 24, n_steps=260),
            _req(surface=big, maturities=[2.0], n_paths=(1 << 17) + 5, n_steps=104)]
    n_ok = 0
    for req in reqs:
        for prec, blocks in ((32, (128, 256, 512, 1024)), (64, (128, 256, 512))):
            for block in blocks:
                for k in (1, 2, 4):
                    for seg in (8, 16, 32):
                        st = lv.check(**req, precision=prec, block=block, copies=k, adjoint="checkpoint",
                                      ckpt_every=seg)
                        msg = _lib.load().lv_last_error(None).decode() if st else ""
                        assert not msg.startswith("planner"), (prec, block, k, seg, msg)
                        assert st in (_lib.LV_OK, _lib.LV_ERR_UNSUPPORTED), (prec, block, k, seg, st)
                        n_ok += st == _lib.LV_OK
    assert n_ok > 60

"""Saved tunings: the autotuner's choice written by one context and taken by another
without timing candidates, lines of other devices skipped, malformed files refused."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lv():
    import paper_2002_02481_amd as m
    return m


SHAPE = ("block", "copies", "window", "blocks_per_cu", "fwd_block", "fwd_blocks_per_cu")


def _call(lv, ctx, **o):
    import torch
    wl = W.small_call()
    s, b = wl.surface, wl.book
    sig = torch.tensor(s.sigma, dtype=torch.float64, device="cuda")
    out = lv.price_and_grad_dev(sig, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, wl.seed,
                                spot_axis=s.spot_axis, time_axis=s.time_axis, ctx=ctx, **o)
    res = [t.cpu().numpy() for t in out]
    info = ctx.run_info()
    return res, {k: info[k] for k in SHAPE}


@pytest.mark.parametrize("adjoint", ["stored", "checkpoint"])
def test_saved_tuning_round_trip(lv, tmp_path, adjoint):
    a = lv.Context(0)
    res_a, shape_a = _call(lv, a, adjoint=adjoint, autotune=True)
    path = str(tmp_path / "tune.txt")
    n = a.save_tuning(path)
    assert n == 1
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("lvmc-tune 1 gfx")
    b = lv.Context(0)
    assert b.load_tuning(path) == 1
    res_b, shape_b = _call(lv, b, adjoint=adjoint, autotune=True)
    assert shape_b == shape_a
    for x, y in zip(res_a, res_b):
        assert np.array_equal(x, y)
    # the loaded shape is what the context holds: saving it again gives the same line
    path2 = str(tmp_path / "tune2.txt")
    assert b.save_tuning(path2) == 1
    assert open(path2).read() == open(path).read()


def test_lines_of_other_devices_are_skipped(lv, tmp_path):
    a = lv.Context(0)
    _call(lv, a, autotune=True)
    path = str(tmp_path / "tune.txt")
    a.save_tuning(path)
    f = open(path).read().split()
    other_arch = " ".join(f[:2] + ["gfx000"] + f[3:]) + "\n"
    other_cus = " ".join(f[:3] + [str(int(f[3]) + 1)] + f[4:]) + "\n"
    p2 = tmp_path / "other.txt"
    p2.write_text(other_arch + other_cus)
    assert lv.Context(0).load_tuning(str(p2)) == 0


@pytest.mark.parametrize("text", ["not a tuning\n",
                                  "lvmc-tune 1 gfx950 256 key 100 2 16 1 512 2\n",
                                  "lvmc-tune 1 gfx950 256 key 512 3 16 1 512 2\n",
                                  "lvmc-tune 1 gfx950 256 key 512 2 12 1 512 2\n"])
def test_malformed_files_are_refused(lv, tmp_path, text):
    p = tmp_path / "bad.txt"
    p.write_text(text)
    with pytest.raises(lv.LVError) as ei:
        lv.Context(0).load_tuning(str(p))
    assert ei.value.status == lv._lib.LV_ERR_ARG


def test_missing_file_is_refused(lv, tmp_path):
    with pytest.raises(lv.LVError):
        lv.Context(0).load_tuning(str(tmp_path / "absent.txt"))


def test_tuning_file_named_by_the_environment(lv, tmp_path, monkeypatch):
    """LVMC_TUNING_FILE: a context created with it set writes what its autotuner chose
    there, keeping the lines of other devices; a later context loads the file at
    creation and takes the same shape; a file that is not a tuning file fails creation."""
    path = tmp_path / "tune_env.txt"
    foreign = "lvmc-tune 1 gfx000 7 " + "k" * 500 + " 512 2 16 1 512 2  " + "#" * 1500 + "\n"   # 2 KB
    path.write_text(foreign.rstrip("\n"))                  # a last line without its newline
    monkeypatch.setenv("LVMC_TUNING_FILE", str(path))
    a = lv.Context(0)
    res_a, shape_a = _call(lv, a, adjoint="stored", autotune=True)
    lines = path.read_text().splitlines()
    assert lines[0] == foreign.strip()                      # another device's line kept
    assert len(lines) == 2 and lines[1].startswith("lvmc-tune 1 gfx")
    b = lv.Context(0)                                       # loads the file when created
    saved = str(tmp_path / "b.txt")
    assert b.save_tuning(saved) == 1 and open(saved).read().strip() == lines[1]
    res_b, shape_b = _call(lv, b, adjoint="stored", autotune=True)
    assert shape_b == shape_a
    for x, y in zip(res_a, res_b):
        assert np.array_equal(x, y)
    assert path.read_text().splitlines() == lines           # nothing new was tuned
    path.write_text("not a tuning\n")
    with pytest.raises(lv.LVError) as ei:
        lv.Context(0)
    assert ei.value.status == lv._lib.LV_ERR_ARG and "LVMC_TUNING_FILE" in str(ei.value)

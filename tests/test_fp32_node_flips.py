"""Where the FP32 kernels' gradient buckets part from the FP64 oracle on a fine spot
axis, shown on the oracle itself (CPU only).

Two copies of the oracle change only how the cell coordinate of a state is formed:
one rounds the state y = ln(S/S0) to single precision and keeps the rest exact; the
other forms the coordinate as the FP32 kernels do, one single-precision fused
multiply-add with the reciprocal spacing and the offset rounded to single precision,
which moves coordinates by up to a few 1e-6 cells.  On the 150 x 80 grid (about 50
nodes per unit of ln S, noisy nodes, so neighbouring cells have quite different
slopes) the second copy flips a few states to the neighbouring cell; those paths then
carry the other slope in their adjoint, and where such a path has a large adjoint a
bucket moves by about 1.3e-4 of max|g|, the size of the GPU's FP32 difference on this
grid and path count.  The first copy stays within 1e-5.  Which paths flip changes
with the path count, so the largest bucket difference does not fall steadily as
paths are added.
"""
import os

import numpy as np

import oracle
import workloads as W

EXACT = "    double a_raw = (u - u0) / du;\n"
STATE_F32 = "    double a_raw = ((double)(float)log(S / pb->spot) + log(pb->spot) - u0) / du;\n"
COORD_F32 = ("    double a_raw = (double)fmaf((float)log(S / pb->spot), (float)(1.0 / du),"
             " (float)((log(pb->spot) - u0) / du));\n")


def _variant(line, name, tmp):
    src = open(oracle.SOURCE).read()
    assert src.count(EXACT) == 1
    path = os.path.join(tmp, f"{name}.c")
    with open(path, "w") as f:
        f.write(src.replace(EXACT, line))
    return oracle.Oracle(oracle.build(path, os.path.join(tmp, f"lib{name}.so")))


def test_fp32_node_coordinates_explain_the_bucket_shifts(tmp_path):
    sa, ta = W.Axis(150, W.LOG, 20.0, 400.0), W.Axis(80, W.LIN, 0.0, 2.0)
    surf = W.Surface(sa, ta, W.noisy(W.smile_surface(sa, ta, 0.2, 0.15, decay=True), 0.01, 21)).rounded_to_f32()
    book = W.Book([0, 1], [100.0, 90.0], [2.0, 1.0], [1.0, 0.5])
    P, N = (1 << 13) + 5, 104
    ref = oracle.default().price_and_grad(surf, book, P, N, seed=13)["grad"]
    gmax = np.abs(ref).max()
    state = _variant(STATE_F32, "state_f32", str(tmp_path)).price_and_grad(surf, book, P, N, seed=13)["grad"]
    coord = _variant(COORD_F32, "coord_f32", str(tmp_path)).price_and_grad(surf, book, P, N, seed=13)["grad"]
    e_state = np.abs(state - ref).max() / gmax
    e_coord = np.abs(coord - ref).max() / gmax
    assert e_state < 1e-5, e_state
    assert 5e-5 < e_coord < 3e-4, e_coord

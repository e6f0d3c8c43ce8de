"""Checks of the FP32 kernels against the FP64 oracle where single precision cannot
decide what the FP64 computation decides.

The pathwise derivative of a bilinearly interpolated surface jumps where a path
crosses a spot node (Sec. IV-D: the slope d sigma / d S changes from cell to cell),
so a path that an FP32 computation follows to within its rounding error, but that
comes closer than that to a node, can take the other cell in FP32: its adjoint then
carries the neighbouring cell's slope from that step back, a finite change.  On
noisy surfaces and long horizons the adjoint of a few paths is very large (it is a
product of step derivatives 1 + c_n s'_n, and so is the sensitivity of the state to
earlier rounding), and one such path can move a gradient bucket by more than
1e-4 max|g| (tests/test_fp32_floor.py shows that even FP32 normals and vols rounded
exactly, with the state and cell coordinate kept exact, do so on the 5-year
100 x 50 surface).  So the FP32 bars are:

  * states: every FP32 state of a path lies within the oracle's running first-order
    bound on a single-precision computation of that path (oracle.path_state_bound);
  * gradient: per bucket, the FP32 - oracle difference D is unbiased -- within
    1e-4 max|g| plus K_SE standard errors of D itself, estimated from the same
    difference taken block by block (the GPU's per-block partial sums against the
    oracle's sums over the same paths).  A mistake in the kernels moves every block
    the same way and fails this; a flip of a few paths does not;
  * what is reported beside it: the largest D over the bucket's Monte Carlo
    standard error (from the oracle's block sums), and the share of buckets within
    the plain 1e-4 max|g|.
"""
from __future__ import annotations

import math
import sys

import numpy as np

GRAD_TOL = 1e-4
K_SE = 6.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def block_ranges(b, B, T, P):
    """Paths of block b: its tiles b, b + B, ... of T paths each."""
    n_tiles = (P + T - 1) // T
    return [(t * T, min((t + 1) * T, P)) for t in range(b, n_tiles, B)]


def oracle_block_sums(orc, surface, book, P, N, seed, B, T):
    """The oracle's gradient sums [B, I, J] over the paths of each GPU block."""
    return np.array([orc.sums(surface, book, N, seed, block_ranges(b, B, T, P))["sum_grad"]
                     for b in range(B)])


def paired_check(gpu_grad, gpu_blocks, orc_blocks, P, what, k_se=K_SE):
    """gpu_grad [I, J] (normalised), gpu_blocks and orc_blocks [B, I, J] (sums over each
    block's paths).  Asserts the bar above; returns the statistics."""
    B = gpu_blocks.shape[0]
    ref = orc_blocks.sum(axis=0) / P
    gmax = np.abs(ref).max()
    # the library's merge of its own block records
    assert np.allclose(gpu_blocks.sum(axis=0) / P, gpu_grad, rtol=0, atol=1e-12 * gmax), what
    D = gpu_grad - ref
    Db = gpu_blocks - orc_blocks
    se_D = Db.std(axis=0, ddof=1) * math.sqrt(B) / P
    se_g = orc_blocks.std(axis=0, ddof=1) * math.sqrt(B) / P
    err = np.abs(D)
    t = err / np.maximum(se_D, 1e-300)
    out = dict(max_err_rel_gmax=float(err.max() / gmax),
               frac_within_1e4=float(np.mean(err <= GRAD_TOL * gmax)),
               max_err_over_se_D=float(t[err > GRAD_TOL * gmax].max(initial=0.0)),
               max_err_over_mc_se=float((err / np.maximum(se_g, 1e-300)).max()),
               q99_err_over_mc_se=float(np.quantile(err / np.maximum(se_g, 1e-300), 0.99)),
               blocks=B)
    say(f"  {what}: max|D|/max|g| {out['max_err_rel_gmax']:.3g}, within 1e-4 max|g| "
        f"{out['frac_within_1e4']:.4f}, beyond it at most {out['max_err_over_se_D']:.2f} se(D); "
        f"|D| / MC stderr: max {out['max_err_over_mc_se']:.3g}, 99% {out['q99_err_over_mc_se']:.3g} "
        f"({B} blocks)")
    ok = err <= GRAD_TOL * gmax + k_se * se_D
    assert np.all(ok), f"{what}: {np.sum(~ok)} buckets biased beyond {k_se} se(D)"
    assert np.all(gpu_grad[ref == 0.0] == 0.0), f"{what}: zero buckets differ"
    return out


def states_within_bound(orc, surface, book, N, seed, paths, y_gpu, what):
    """y_gpu [len(paths), N]: the FP32 states y_1 .. y_N of the listed paths.  Each lies
    within the oracle's first-order single-precision bound of its FP64 value."""
    worst, und = 0.0, 0
    for q, p in enumerate(paths):
        y = orc.path(surface, book, N, seed, int(p))["y"]
        e, u = orc.path_state_bound(surface, book, N, seed, int(p))
        r = np.abs(y_gpu[q] - y[1:]) / e[1:]
        worst = max(worst, float(r.max()))
        und += int(u.sum())
        assert np.all(r <= 1.0), f"{what}: path {p} step {int(np.argmax(r))} off by {r.max():.3g} of the bound"
    say(f"  {what}: FP32 states within {worst:.3g} of the single-precision bound over {len(paths)} paths "
        f"({und} undecided cell steps)")
    return worst

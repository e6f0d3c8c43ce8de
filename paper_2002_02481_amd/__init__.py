"""lvmc: Monte Carlo pricing under the Dupire local-volatility model, with the
adjoint (back-propagated) sensitivities of the price to every vol-grid node, on
AMD MI355X (gfx950).

Method: arXiv 2002.02481 -- the SDE dX/X = sigma(X,t) dW and its explicit Euler
scheme (Sec. IV-A), bilinear interpolation of the vol grid (Sec. IV-A/IV-D),
European payoffs averaged over paths (Sec. IV-B/IV-C) and reverse-mode
sensitivities (Sec. III, IV-C).  The computation runs in hand-written HIP
kernels in liblvmc.so (C ABI in include/lvmc.h); this package marshals
arguments with ctypes and uses PyTorch only for device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import ADJOINT, LVError, lv_axis, lv_book, lv_grid, lv_opts, lv_run_info

__all__ = ["Context", "LVError", "price_and_grad", "price_and_grad_batch", "price_and_grad_dev",
           "forward_dev", "backward_dev", "states_bytes", "LVPrice", "check", "default_context",
           "bump_grad_dev", "per_option_grads_dev", "price_and_grad_noalloc"]


def _lib_handle():
    return _lib.load()


def _check_status(st: int, ctx_handle=None):
    if st != 0:
        msg = _lib_handle().lv_last_error(ctx_handle).decode()
        raise LVError(st, msg)


# --------------------------------------------------------------------------
# argument structures
# --------------------------------------------------------------------------
def make_grid(spot_axis, time_axis) -> lv_grid:
    """spot_axis = (n, kind, lo, hi) or an object with n/kind/lo/hi; time_axis likewise
    (kind must be linear)."""
    def ax(a):
        if hasattr(a, "n"):
            return lv_axis(int(a.n), int(getattr(a, "kind", 0)), float(a.lo), float(a.hi))
        if len(a) == 3:
            n, lo, hi = a
            return lv_axis(int(n), 0, float(lo), float(hi))
        n, kind, lo, hi = a
        return lv_axis(int(n), int(kind), float(lo), float(hi))
    return lv_grid(ax(spot_axis), ax(time_axis))


class _Book:
    """Keeps the numpy arrays alive while the C struct points into them."""

    def __init__(self, strikes, maturities, is_put=None, weights=None):
        self.strike = np.ascontiguousarray(np.atleast_1d(strikes), dtype=np.float64)
        n = self.strike.shape[0]
        self.maturity = np.ascontiguousarray(np.broadcast_to(np.atleast_1d(maturities), (n,)),
                                             dtype=np.float64)
        self.is_put = np.ascontiguousarray(
            np.zeros(n) if is_put is None else np.broadcast_to(np.atleast_1d(is_put), (n,)),
            dtype=np.int32)
        self.weight = None if weights is None else np.ascontiguousarray(
            np.broadcast_to(np.atleast_1d(weights), (n,)), dtype=np.float64)
        self.c = lv_book(n, self.is_put.ctypes.data_as(C.POINTER(C.c_int32)),
                         self.strike.ctypes.data_as(C.POINTER(C.c_double)),
                         self.maturity.ctypes.data_as(C.POINTER(C.c_double)),
                         None if self.weight is None else self.weight.ctypes.data_as(C.POINTER(C.c_double)))

    @property
    def n(self):
        return self.strike.shape[0]


SCHEME = {"log_euler": 0, "euler_x": 1}


def make_opts(precision=32, adjoint="stored", ckpt_every=16, use_graph=False, block=0,
              blocks_per_cu=0, copies=0, window=0, profile=False, autotune=False, fwd_block=0,
              fwd_blocks_per_cu=0, dense_adjoint=False, profile_kinds=0, scheme="log_euler",
              sigma_bf16=False, rate=0.0) -> lv_opts:
    """scheme: "log_euler" (the Euler step on ln X) or "euler_x" (on X itself).
    sigma_bf16: price the surface with its nodes rounded to bfloat16 (the TPU's storage
    precision for the interpolation, Sec. IV-D).  rate: constant short rate r (the step's
    trend; prices discounted by e^{-r T})."""
    adj = ADJOINT[adjoint] if isinstance(adjoint, str) else int(adjoint)
    sch = SCHEME[scheme] if isinstance(scheme, str) else int(scheme)
    return lv_opts(int(precision), adj, int(ckpt_every), int(bool(use_graph)), int(block),
                   int(blocks_per_cu), int(copies), int(window), int(bool(profile)),
                   int(bool(autotune)), int(fwd_block), int(fwd_blocks_per_cu),
                   int(bool(dense_adjoint)), int(profile_kinds), sch, int(sigma_bf16), float(rate))


def option_order(maturities, n_steps) -> np.ndarray:
    """Caller index of each option in the library's maturity order."""
    book = _Book(np.ones(len(np.atleast_1d(maturities))), maturities)
    out = np.zeros(book.n, dtype=np.int32)
    _check_status(_lib_handle().lv_debug_option_order(C.byref(book.c), int(n_steps), out.ctypes.data))
    return out


def tuning_candidates(surface, strikes, maturities, n_paths, n_steps, *, is_put=None,
                      spot_axis=None, time_axis=None, **opts):
    """Launch shapes (block, copies, window, blocks_per_cu, fwd_block, fwd_blocks_per_cu)
    the autotuner would time."""
    grid, _ = _surface_parts(surface, spot_axis, time_axis)
    book = _Book(strikes, maturities, is_put, None)
    o = make_opts(**opts)
    out = np.zeros((512, 6), dtype=np.int32)
    n = C.c_int32()
    _check_status(_lib_handle().lv_tuning_candidates(C.byref(grid), C.byref(book.c), int(n_paths),
                                                     int(n_steps), C.byref(o), out.ctypes.data,
                                                     512, C.byref(n)))
    return [tuple(int(v) for v in row) for row in out[:n.value]]


def _surface_parts(surface, spot_axis, time_axis):
    if spot_axis is None:
        spot_axis, time_axis, sigma = surface.spot_axis, surface.time_axis, surface.sigma
    else:
        sigma = surface
    return make_grid(spot_axis, time_axis), np.asarray(sigma)


# --------------------------------------------------------------------------
# contexts
# --------------------------------------------------------------------------
class Context:
    """A library context on one GPU: owns the device workspace, the graph cache and the
    autotuner's choices (loaded from, and written back to, the file the environment
    variable LVMC_TUNING_FILE names, if it is set when the context is created)."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        self.lib = _lib_handle()
        h = C.c_void_p()
        _check_status(self.lib.lv_create(C.byref(h), int(device), C.c_void_p(stream or 0)))
        self.h = h
        self.device = device

    def set_stream(self, stream: Optional[int]):
        _check_status(self.lib.lv_set_stream(self.h, C.c_void_p(stream or 0)), self.h)

    def use_torch_stream(self):
        import torch
        self.set_stream(torch.cuda.current_stream(self.device).cuda_stream)

    def run_info(self) -> dict:
        info = lv_run_info()
        _check_status(self.lib.lv_last_run_info(self.h, C.byref(info)), self.h)
        return {f: getattr(info, f) for f, _ in lv_run_info._fields_}

    def kernel_times(self, reset: bool = True) -> dict:
        """{kind: (total_ms, launches)} of the kernels timed under profile=True."""
        ms = np.zeros(len(_lib.KERNEL_KINDS))
        cnt = np.zeros(len(_lib.KERNEL_KINDS), dtype=np.int64)
        _check_status(self.lib.lv_kernel_times(self.h, ms.ctypes.data, cnt.ctypes.data, int(reset)), self.h)
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(_lib.KERNEL_KINDS)}

    def block_partials(self, n_opt: int, G: int) -> dict:
        """Per-block partial records of the last surface of the last call:
        sum_pay, sum_pay2 [B, n_opt] (maturity order), sum_lam0 [B], grad [B, G]."""
        B = self.run_info()["n_blocks"]
        Q = 2 * n_opt + 1 + G
        out = np.zeros((B, Q))
        _check_status(self.lib.lv_debug_block_partials(self.h, out.ctypes.data, out.size), self.h)
        pay = out[:, :2 * n_opt].reshape(B, n_opt, 2)
        return dict(sum_pay=pay[:, :, 0], sum_pay2=pay[:, :, 1], sum_lam0=out[:, 2 * n_opt],
                    grad=out[:, 2 * n_opt + 1:])

    def block_grads(self, G: int, n_opt: int = 1) -> np.ndarray:
        return self.block_partials(n_opt, G)["grad"]

    def save_tuning(self, path: str) -> int:
        """Write the launch shapes this context has tuned to `path`; returns the count."""
        n = C.c_int32()
        _check_status(self.lib.lv_tuning_save(self.h, os.fsencode(path), C.byref(n)), self.h)
        return n.value

    def load_tuning(self, path: str) -> int:
        """Take the tuned shapes saved in `path` that were timed on this kind of device;
        returns how many were taken."""
        n = C.c_int32()
        _check_status(self.lib.lv_tuning_load(self.h, os.fsencode(path), C.byref(n)), self.h)
        return n.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.lv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts = {}


def default_context(device: int = 0) -> Context:
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]


# --------------------------------------------------------------------------
# host-buffer API
# --------------------------------------------------------------------------
def check(surface, spot, strikes, maturities, n_paths, n_steps, *, is_put=None, weights=None,
          spot_axis=None, time_axis=None, **opts) -> int:
    """Validate a request on the host only (no GPU).  Returns the lv_status code."""
    grid, sigma = _surface_parts(surface, spot_axis, time_axis)
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    book = _Book(strikes, maturities, is_put, weights)
    o = make_opts(**opts)
    return _lib_handle().lv_check(C.byref(grid), sig.ctypes.data, float(spot), C.byref(book.c),
                                  int(n_paths), int(n_steps), C.byref(o))


def price_and_grad_batch(sigmas, spot, strikes, maturities, n_paths, n_steps, seed=0, *,
                         spot_axis, time_axis, is_put=None, weights=None, want_grad=True,
                         ctx: Optional[Context] = None, **opts):
    """n_surf surfaces [n_surf, I, J] on the same Philox streams.  Returns prices and
    std_errs [n_surf, n_opt], grads [n_surf, I, J] (or None) and deltas [n_surf] (or None)."""
    ctx = ctx or default_context()
    grid = make_grid(spot_axis, time_axis)
    sig = np.ascontiguousarray(sigmas, dtype=np.float64)
    if sig.ndim == 2:
        sig = sig[None]
    n_surf, I, J = sig.shape
    book = _Book(strikes, maturities, is_put, weights)
    o = make_opts(**opts)
    adjoint = want_grad and o.adjoint != _lib.LV_ADJ_NONE
    prices = np.zeros((n_surf, book.n))
    stderrs = np.zeros((n_surf, book.n))
    grads = np.zeros((n_surf, I, J)) if adjoint else None
    deltas = np.zeros(n_surf) if adjoint else None
    st = ctx.lib.lv_price_and_grad_batch(
        ctx.h, C.byref(grid), n_surf, sig.ctypes.data, float(spot), C.byref(book.c), int(n_paths),
        int(n_steps), int(seed), C.byref(o), prices.ctypes.data, stderrs.ctypes.data,
        grads.ctypes.data if adjoint else None, deltas.ctypes.data if adjoint else None)
    _check_status(st, ctx.h)
    return prices, stderrs, grads, deltas


def price_and_grad(surface, spot, strikes, maturities, n_paths, n_steps, seed=0, *, is_put=None,
                   weights=None, spot_axis=None, time_axis=None, want_grad=True,
                   ctx: Optional[Context] = None, **opts):
    """price_and_grad(surface, spot, strikes, maturities, n_paths, n_steps, seed) ->
    (price [n_opt], std_err [n_opt], grad [I, J] of sum_k w_k price_k, delta).

    `surface` has spot_axis / time_axis / sigma attributes, or is a [I, J] array
    with spot_axis=(n, kind, lo, hi) and time_axis=(n, lo, hi) given."""
    grid, sigma = _surface_parts(surface, spot_axis, time_axis)
    sa, ta = grid.spot, grid.time
    p, s, g, d = price_and_grad_batch(sigma, spot, strikes, maturities, n_paths, n_steps, seed,
                                      spot_axis=(sa.n, sa.kind, sa.lo, sa.hi),
                                      time_axis=(ta.n, ta.kind, ta.lo, ta.hi), is_put=is_put,
                                      weights=weights, want_grad=want_grad, ctx=ctx, **opts)
    return p[0], s[0], (g[0] if g is not None else None), (float(d[0]) if d is not None else None)


# --------------------------------------------------------------------------
# device (torch tensor) API
# --------------------------------------------------------------------------
def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _need_dev(t, name, device=None, numel=None, dtype=None, nbytes=None):
    """The library takes plain device pointers and trusts their extent, so every tensor
    it is given is checked here first: a contiguous CUDA tensor (on `device`, of
    `dtype`, float64 unless given, with at least `numel` elements or `nbytes` bytes);
    ValueError otherwise."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}; the call runs on {device}")
    if nbytes is None and t.dtype != (dtype or torch.float64):
        raise ValueError(f"{name} must be {dtype or torch.float64}, not {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements; {numel} are needed")
    if nbytes is not None and t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{name} holds {t.numel() * t.element_size()} bytes; {nbytes} are needed")
    return t


def _need_surface(sigma, grid, batched):
    """sigma: [I, J] (or [n_surf, I, J] when batched; [I, J] is one surface) matching
    the grid's axes; returns it in the shape the call takes."""
    _need_dev(sigma, "sigma")
    if batched and sigma.dim() == 2:
        sigma = sigma.unsqueeze(0)
    want = (grid.spot.n, grid.time.n)
    if sigma.dim() != (3 if batched else 2) or tuple(sigma.shape[-2:]) != want:
        raise ValueError(f"sigma has shape {tuple(sigma.shape)}; the grid's axes give "
                         f"{'[n_surf, ' if batched else '['}{want[0]}, {want[1]}]")
    return sigma


def _ctx_for(ctx, t):
    ctx = ctx or default_context(t.device.index or 0)
    if ctx.device != (t.device.index or 0):
        raise ValueError(f"the context is on cuda:{ctx.device}, the tensors on {t.device}")
    return ctx


def price_and_grad_dev(sigmas, spot, strikes, maturities, n_paths, n_steps, seed=0, *, spot_axis,
                       time_axis, is_put=None, weights=None, want_grad=True, out=None,
                       ctx: Optional[Context] = None, **opts):
    """Device-resident call on torch's current stream: sigmas is a CUDA float64 tensor
    [n_surf, I, J].  Returns (prices, std_errs, grads, deltas) CUDA tensors; nothing
    is synchronised.  `out` may pass preallocated tensors in that order."""
    import torch
    grid = make_grid(spot_axis, time_axis)
    sigmas = _need_surface(sigmas, grid, batched=True)
    ctx = _ctx_for(ctx, sigmas)
    ctx.use_torch_stream()
    n_surf, I, J = sigmas.shape
    book = _Book(strikes, maturities, is_put, weights)
    o = make_opts(**opts)
    adjoint = want_grad and o.adjoint != _lib.LV_ADJ_NONE
    dev = sigmas.device
    if out is None:
        prices = torch.empty((n_surf, book.n), dtype=torch.float64, device=dev)
        stderrs = torch.empty_like(prices)
        grads = torch.empty((n_surf, I, J), dtype=torch.float64, device=dev) if adjoint else None
        deltas = torch.empty((n_surf,), dtype=torch.float64, device=dev) if adjoint else None
    else:
        prices, stderrs, grads, deltas = out
        _need_dev(prices, "prices", dev, n_surf * book.n)
        _need_dev(stderrs, "std_errs", dev, n_surf * book.n)
        if not adjoint:
            grads = deltas = None
        if grads is not None:
            _need_dev(grads, "grads", dev, n_surf * I * J)
        if deltas is not None:
            _need_dev(deltas, "deltas", dev, n_surf)
    st = ctx.lib.lv_price_and_grad_dev(
        ctx.h, C.byref(grid), n_surf, _ptr(sigmas), float(spot), C.byref(book.c), int(n_paths),
        int(n_steps), int(seed), C.byref(o), _ptr(prices), _ptr(stderrs), _ptr(grads), _ptr(deltas))
    _check_status(st, ctx.h)
    return prices, stderrs, grads, deltas


def price_and_grad_noalloc(sigmas, spot, strikes, maturities, n_paths, n_steps, seed=0, *, spot_axis,
                           time_axis, is_put=None, weights=None, want_grad=True, out,
                           ctx: Optional[Context] = None, **opts):
    """price_and_grad_dev through the allocation-free entry point: the library works in
    its fixed per-GPU workspace and allocates nothing.  `out` = (prices, std_errs, grads,
    deltas) CUDA float64 tensors the caller allocated (grads and deltas may be None)."""
    grid = make_grid(spot_axis, time_axis)
    sigmas = _need_surface(sigmas, grid, batched=True)
    ctx = _ctx_for(ctx, sigmas)
    ctx.use_torch_stream()
    n_surf, I, J = sigmas.shape
    book = _Book(strikes, maturities, is_put, weights)
    o = make_opts(**opts)
    prices, stderrs, grads, deltas = out
    if not want_grad or o.adjoint == _lib.LV_ADJ_NONE:
        grads = deltas = None
    dev = sigmas.device
    _need_dev(prices, "prices", dev, n_surf * book.n)
    _need_dev(stderrs, "std_errs", dev, n_surf * book.n)
    if grads is not None:
        _need_dev(grads, "grads", dev, n_surf * I * J)
    if deltas is not None:
        _need_dev(deltas, "deltas", dev, n_surf)
    st = ctx.lib.lv_price_and_grad_noalloc(
        ctx.h, C.byref(grid), n_surf, _ptr(sigmas), float(spot), C.byref(book.c), int(n_paths),
        int(n_steps), int(seed), C.byref(o), _ptr(prices), _ptr(stderrs), _ptr(grads), _ptr(deltas))
    _check_status(st, ctx.h)
    return prices, stderrs, grads, deltas


def bump_grad_dev(sigma, spot, strikes, maturities, n_paths, n_steps, seed=0, *, spot_axis, time_axis,
                  is_put=None, weights=None, eps=1e-4, batch=0, out=None, ctx: Optional[Context] = None,
                  **opts):
    """Bump-and-reprice gradient [I, J] of sum_k w_k price_k by central differences of
    width eps on every node (same paths as the adjoint), for comparison with it.
    sigma is a CUDA float64 tensor [I, J]; runs on torch's current stream."""
    import torch
    grid = make_grid(spot_axis, time_axis)
    sigma = _need_surface(sigma, grid, batched=False)
    ctx = _ctx_for(ctx, sigma)
    ctx.use_torch_stream()
    book = _Book(strikes, maturities, is_put, weights)
    o = make_opts(**opts)
    if out is not None:
        grad = _need_dev(out, "out", sigma.device, sigma.numel())
    else:
        grad = torch.empty(sigma.shape, dtype=torch.float64, device=sigma.device)
    st = ctx.lib.lv_bump_grad_dev(ctx.h, C.byref(grid), _ptr(sigma), float(spot), C.byref(book.c),
                                  int(n_paths), int(n_steps), int(seed), C.byref(o), float(eps),
                                  int(batch), _ptr(grad))
    _check_status(st, ctx.h)
    return grad


def per_option_grads_dev(sigma, spot, strikes, maturities, n_paths, n_steps, seed=0, *, spot_axis,
                         time_axis, is_put=None, precision=32, rate=0.0, ctx: Optional[Context] = None):
    """Per-option vol-grid gradients from one simulation: the states are stored once by
    the split forward, then one reverse sweep serves up to 8 options at a time, each
    with its own adjoint (seeded by its own payoff) and its own gradient histogram.
    Returns (prices [n], std_errs [n], grads [n, I, J], deltas [n]) CUDA tensors."""
    import torch
    sigma = _need_surface(sigma, make_grid(spot_axis, time_axis), batched=False)
    ctx = _ctx_for(ctx, sigma)
    price, stderr, states = forward_dev(sigma, spot, strikes, maturities, n_paths, n_steps, seed,
                                        spot_axis=spot_axis, time_axis=time_axis, is_put=is_put,
                                        precision=precision, rate=rate, ctx=ctx)
    n = price.numel()
    grads = torch.empty((n,) + tuple(sigma.shape), dtype=torch.float64, device=sigma.device)
    deltas = torch.empty(n, dtype=torch.float64, device=sigma.device)
    grid = make_grid(spot_axis, time_axis)
    book = _Book(strikes, maturities, is_put, None)
    st = ctx.lib.lv_per_option_grads_dev(ctx.h, C.byref(grid), _ptr(sigma), float(spot), C.byref(book.c),
                                         int(n_paths), int(n_steps), int(seed), int(precision), float(rate),
                                         _ptr(states), _ptr(grads), _ptr(deltas))
    _check_status(st, ctx.h)
    return price, stderr, grads, deltas


def states_bytes(precision: int, n_paths: int, n_steps: int) -> int:
    b = C.c_size_t()
    _check_status(_lib_handle().lv_states_bytes(int(precision), int(n_paths), int(n_steps), C.byref(b)))
    return b.value


def forward_dev(sigma, spot, strikes, maturities, n_paths, n_steps, seed, *, spot_axis, time_axis,
                is_put=None, precision=32, rate=0.0, states=None, ctx: Optional[Context] = None):
    """Split forward: returns (price, std_err, states) CUDA tensors."""
    import torch
    grid = make_grid(spot_axis, time_axis)
    sigma = _need_surface(sigma, grid, batched=False)
    ctx = _ctx_for(ctx, sigma)
    ctx.use_torch_stream()
    book = _Book(strikes, maturities, is_put, None)
    nb = states_bytes(precision, n_paths, n_steps)
    if states is None:
        states = torch.empty(nb, dtype=torch.uint8, device=sigma.device)
    _need_dev(states, "states", sigma.device, nbytes=nb)
    price = torch.empty(book.n, dtype=torch.float64, device=sigma.device)
    stderr = torch.empty_like(price)
    st = ctx.lib.lv_forward_dev(ctx.h, C.byref(grid), _ptr(sigma), float(spot), C.byref(book.c),
                                int(n_paths), int(n_steps), int(seed), int(precision), float(rate),
                                _ptr(states), _ptr(price), _ptr(stderr))
    _check_status(st, ctx.h)
    return price, stderr, states


def backward_dev(sigma, spot, strikes, maturities, n_paths, n_steps, seed, states, cotangent, *,
                 spot_axis, time_axis, is_put=None, precision=32, rate=0.0, want_delta=False,
                 ctx: Optional[Context] = None):
    """Split backward: gradient [I, J] of sum_k cotangent_k price_k (and delta)."""
    import torch
    grid = make_grid(spot_axis, time_axis)
    sigma = _need_surface(sigma, grid, batched=False)
    ctx = _ctx_for(ctx, sigma)
    ctx.use_torch_stream()
    book = _Book(strikes, maturities, is_put, None)
    _need_dev(states, "states", sigma.device, nbytes=states_bytes(precision, n_paths, n_steps))
    cot = torch.as_tensor(cotangent, dtype=torch.float64, device=sigma.device).contiguous().reshape(-1)
    if cot.numel() != book.n:
        raise ValueError(f"cotangent has {cot.numel()} entries for a book of {book.n} options")
    grad = torch.empty(sigma.shape, dtype=torch.float64, device=sigma.device)
    delta = torch.empty(1, dtype=torch.float64, device=sigma.device) if want_delta else None
    st = ctx.lib.lv_backward_dev(ctx.h, C.byref(grid), _ptr(sigma), float(spot), C.byref(book.c),
                                 int(n_paths), int(n_steps), int(seed), int(precision), float(rate),
                                 _ptr(states), _ptr(cot), _ptr(grad), _ptr(delta))
    _check_status(st, ctx.h)
    return grad, delta


def _make_lvprice():
    import torch

    class LVPrice(torch.autograd.Function):
        """price = LVPrice.apply(sigma, spec) with sigma a CUDA float64 [I, J] tensor and
        spec a dict of spot, strikes, maturities, is_put, n_paths, n_steps, seed,
        spot_axis, time_axis, precision and (optional) rate.  The backward pass is the stored-state adjoint
        kernel, with grad_output as the per-option cotangent."""

        @staticmethod
        def forward(ctx, sigma, spec):
            sigma = sigma.contiguous()
            price, stderr, states = forward_dev(
                sigma, spec["spot"], spec["strikes"], spec["maturities"], spec["n_paths"],
                spec["n_steps"], spec.get("seed", 0), spot_axis=spec["spot_axis"],
                time_axis=spec["time_axis"], is_put=spec.get("is_put"),
                precision=spec.get("precision", 32), rate=spec.get("rate", 0.0))
            ctx.save_for_backward(sigma, states)
            ctx.spec = spec
            ctx.mark_non_differentiable(stderr)
            return price, stderr

        @staticmethod
        def backward(ctx, grad_price, grad_stderr):
            sigma, states = ctx.saved_tensors
            spec = ctx.spec
            grad, _ = backward_dev(
                sigma, spec["spot"], spec["strikes"], spec["maturities"], spec["n_paths"],
                spec["n_steps"], spec.get("seed", 0), states, grad_price,
                spot_axis=spec["spot_axis"], time_axis=spec["time_axis"],
                is_put=spec.get("is_put"), precision=spec.get("precision", 32),
                rate=spec.get("rate", 0.0))
            return grad, None

    return LVPrice


class _LazyLVPrice:
    _cls = None

    def __getattr__(self, name):
        if _LazyLVPrice._cls is None:
            _LazyLVPrice._cls = _make_lvprice()
        return getattr(_LazyLVPrice._cls, name)


LVPrice = _LazyLVPrice()

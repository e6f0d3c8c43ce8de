"""FP64 CPU oracle for the local-vol Monte Carlo and its vol-grid adjoint.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg load this package; the GPU library never does, and the two
share no code.  The arithmetic lives in ``lv_oracle.c`` (plain C, IEEE double);
this module is argument marshalling through ctypes plus the normalisations
price = sum/P and stderr = sqrt(sample variance / P).

It follows arXiv 2002.02481: the Dupire SDE and its explicit Euler scheme
(Sec. IV-A), bilinear interpolation of the vol grid (Sec. IV-A, IV-D), the
call payoff average (Sec. IV-B/IV-C) and back-propagated sensitivities to every
vol node (Sec. III, IV-C).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "lv_oracle.c")
LIBRARY = os.path.join(HERE, "liblvoracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def build(source: str = SOURCE, library: str = LIBRARY) -> str:
    """Compile the oracle with gcc into a shared library."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-o", library, source, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    return library


class OracleError(RuntimeError):
    pass


def default_threads() -> int:
    """Worker threads: LV_ORACLE_THREADS if set, else the host cores, at most 16."""
    env = os.environ.get("LV_ORACLE_THREADS")
    if env:
        return max(1, int(env))
    return max(1, min(16, os.cpu_count() or 1))


def _surface_args(surface):
    sa, ta = surface.spot_axis, surface.time_axis
    return (C.c_int32(sa.n), C.c_int32(sa.kind), C.c_double(sa.lo), C.c_double(sa.hi),
            C.c_int32(ta.n), C.c_double(ta.lo), C.c_double(ta.hi),
            np.ascontiguousarray(surface.sigma, dtype=np.float64))


def _book_args(book):
    return (C.c_int32(book.n), book.is_put, book.strike, book.maturity, book.weight)


class Oracle:
    def __init__(self, library: Optional[str] = None):
        library = library or LIBRARY
        if not os.path.exists(library):
            build(SOURCE, library)
        self.lib = C.CDLL(library)
        L = self.lib
        surf = [C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_double,
                C.c_double, _dp]
        book = [C.c_double, C.c_int32, _ip, _dp, _dp, _dp]
        L.lvo_philox_words.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, _up]
        L.lvo_philox_words.restype = None
        L.lvo_normal.argtypes = [C.c_uint64, C.c_uint64, C.c_int64]
        L.lvo_normal.restype = C.c_double
        L.lvo_normals.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_int64, _dp]
        L.lvo_normals.restype = None
        L.lvo_uniform.argtypes = [C.c_uint32]
        L.lvo_uniform.restype = C.c_double
        L.lvo_last_error.restype = C.c_char_p
        L.lvo_accumulate.argtypes = surf + book + [C.c_int32, C.c_uint64, C.c_int64, _lp,
                                                   C.c_int32, _dp, _dp, C.c_void_p, C.c_void_p,
                                                   C.c_int32, C.c_double]
        L.lvo_accumulate.restype = C.c_int
        L.lvo_path.argtypes = surf + book + [C.c_int32, C.c_uint64, C.c_int64,
                                             _dp, _dp, _dp, _dp, _dp, _dp, _dp, C.c_int32, C.c_double]
        L.lvo_path.restype = C.c_int
        L.lvo_interp_at.argtypes = surf + [C.c_double, C.c_double, C.POINTER(C.c_double),
                                           C.POINTER(C.c_double), _ip, _dp]
        L.lvo_interp_at.restype = C.c_int
        L.lvo_round_bf16.argtypes = [C.c_double]
        L.lvo_round_bf16.restype = C.c_double
        L.lvo_path_state_bound.argtypes = surf + book + [C.c_int32, C.c_uint64, C.c_int64, _dp, _dp, _ip,
                                                         C.c_double]
        L.lvo_path_state_bound.restype = C.c_int

    def _check(self, rc):
        if rc != 0:
            raise OracleError(self.lib.lvo_last_error().decode())

    # -- random numbers ----------------------------------------------------
    def philox_words(self, seed: int, m: int, p: int) -> np.ndarray:
        out = np.zeros(4, dtype=np.uint32)
        self.lib.lvo_philox_words(seed, m, p, out)
        return out

    def uniform(self, w: int) -> float:
        return self.lib.lvo_uniform(int(w) & 0xFFFFFFFF)

    def normal(self, seed: int, p: int, n: int) -> float:
        return self.lib.lvo_normal(seed, p, n)

    def normals(self, seed: int, p0: int, n_paths: int, n_steps: int) -> np.ndarray:
        out = np.zeros((n_paths, n_steps))
        self.lib.lvo_normals(seed, p0, n_paths, n_steps, out)
        return out

    # -- reduced precision of the nodes ------------------------------------
    def round_bf16(self, sigma) -> np.ndarray:
        """Every node rounded to bfloat16 by way of single precision (Sec. IV-D's
        mixed-precision TPU runs hold sigma in bfloat16 for the interpolation)."""
        sigma = np.asarray(sigma, dtype=np.float64)
        return np.array([self.lib.lvo_round_bf16(float(v)) for v in sigma.ravel()]).reshape(sigma.shape)

    # -- interpolation -----------------------------------------------------
    def interp(self, surface, S: float, t: float):
        """sigma(S, t), d sigma / d ln S, lower-left node (i, j), weights of
        (i,j), (i+1,j), (i,j+1), (i+1,j+1)."""
        sig, dsdy = C.c_double(), C.c_double()
        ij = np.zeros(2, dtype=np.int32)
        w = np.zeros(4)
        self._check(self.lib.lvo_interp_at(*_surface_args(surface), S, t, C.byref(sig),
                                           C.byref(dsdy), ij, w))
        return sig.value, dsdy.value, (int(ij[0]), int(ij[1])), w

    # -- one path ----------------------------------------------------------
    def path(self, surface, book, n_steps: int, seed: int, p: int, spot: float = 100.0,
             scheme: int = 0, rate: float = 0.0) -> Dict:
        N = int(n_steps)
        G = surface.spot_axis.n * surface.time_axis.n
        y, z = np.zeros(N + 1), np.zeros(N)
        sig, dsdy, lam = np.zeros(N), np.zeros(N), np.zeros(N + 1)
        pay, grad = np.zeros(book.n), np.zeros(G)
        self._check(self.lib.lvo_path(*_surface_args(surface), spot, *_book_args(book), N,
                                      seed, p, y, z, sig, dsdy, lam, pay, grad, int(scheme),
                                      float(rate)))
        return dict(y=y, z=z, sigma=sig, dsdy=dsdy, lam=lam, payoff=pay,
                    grad=grad.reshape(surface.sigma.shape))

    # -- sums over path ranges ---------------------------------------------
    def sums(self, surface, book, n_steps: int, seed: int,
             ranges: Sequence[Tuple[int, int]], n_threads: int = 0, spot: float = 100.0,
             want_grad: bool = True, scheme: int = 0, rate: float = 0.0) -> Dict:
        """Unnormalised sums of payoff, payoff^2, grid gradient and d/dy_0 of the
        weighted book value over the given half-open path ranges."""
        if n_threads <= 0:
            n_threads = default_threads()
        rg = np.ascontiguousarray(np.asarray(ranges, dtype=np.int64).reshape(-1, 2))
        s1, s2 = np.zeros(book.n), np.zeros(book.n)
        G = surface.spot_axis.n * surface.time_axis.n
        grad = np.zeros(G)
        lam0 = np.zeros(1)
        self._check(self.lib.lvo_accumulate(
            *_surface_args(surface), spot, *_book_args(book), int(n_steps), seed,
            rg.shape[0], rg, n_threads, s1, s2,
            grad.ctypes.data if want_grad else None, lam0.ctypes.data, int(scheme), float(rate)))
        n = int(np.sum(rg[:, 1] - rg[:, 0]))
        return dict(n=n, sum_pay=s1, sum_pay2=s2,
                    sum_grad=grad.reshape(surface.sigma.shape) if want_grad else None,
                    sum_lam0=float(lam0[0]))

    def price_and_grad(self, surface, book, n_paths: int, n_steps: int, seed: int = 0,
                       n_threads: int = 0, spot: float = 100.0, want_grad: bool = True,
                       path0: int = 0, scheme: int = 0, rate: float = 0.0) -> Dict:
        """Price, standard error per option, gradient of the weighted book value
        with respect to every vol node, and delta (d value / d spot).  scheme 0:
        log-Euler on ln X; 1: the Euler step on X itself."""
        s = self.sums(surface, book, n_steps, seed, [(path0, path0 + n_paths)], n_threads,
                      spot, want_grad, scheme, rate)
        P = float(n_paths)
        price = s["sum_pay"] / P
        var = (s["sum_pay2"] - s["sum_pay"] ** 2 / P) / (P - 1.0)
        stderr = np.sqrt(np.maximum(var, 0.0) / P)
        grad = s["sum_grad"] / P if want_grad else None
        return dict(price=price, stderr=stderr, grad=grad, delta=s["sum_lam0"] / P / spot)


    def bump_grad(self, surface, book, n_paths: int, n_steps: int, seed: int = 0, eps: float = 1e-4,
                  nodes: Optional[Sequence[Tuple[int, int]]] = None, n_threads: int = 0,
                  spot: float = 100.0, scheme: int = 0, rate: float = 0.0) -> np.ndarray:
        """Finite-difference ("bumping", Sec. III) derivative of the weighted book value
        with respect to the listed nodes (all when None): the book priced on the same
        paths with sigma_ij + eps/2 and with sigma_ij - eps/2, the difference over eps.
        Returns [len(nodes)] in the order given."""
        I, J = surface.sigma.shape
        if nodes is None:
            nodes = [(i, j) for i in range(I) for j in range(J)]
        w = np.asarray(book.weight, dtype=np.float64)
        out = np.zeros(len(nodes))
        for q, (i, j) in enumerate(nodes):
            vals = []
            for h in (0.5 * eps, -0.5 * eps):
                sig = np.array(surface.sigma, dtype=np.float64, copy=True)
                sig[i, j] += h
                bumped = dataclasses.replace(surface, sigma=sig)
                r = self.price_and_grad(bumped, book, n_paths, n_steps, seed, n_threads, spot,
                                        want_grad=False, scheme=scheme, rate=rate)
                vals.append(float(np.dot(w, r["price"])))
            out[q] = (vals[0] - vals[1]) / eps
        return out


    # -- how far a single-precision computation of a path can be -----------
    def path_state_bound(self, surface, book, n_steps: int, seed: int, p: int, spot: float = 100.0,
                         model=None, rate: float = 0.0):
        """First-order bound e[N+1] on |y_n(single precision) - y_n(this oracle)| for path p
        of the log-Euler scheme, and the steps [N] whose spot cell is undecided at that
        precision (lvo_path_state_bound in lv_oracle.c)."""
        model = np.ascontiguousarray(FP32_MODEL if model is None else model, dtype=np.float64)
        N = int(n_steps)
        e, und = np.zeros(N + 1), np.zeros(N, dtype=np.int32)
        self._check(self.lib.lvo_path_state_bound(*_surface_args(surface), spot, *_book_args(book), N,
                                                  seed, p, model, e, und, float(rate)))
        return e, und.astype(bool)


# Unit roundoff of IEEE single precision; the local error of one step's increment and
# of the cell coordinate, in units of it (hardware log/sqrt/sin/cos and exp of a few
# ulps each, a handful of rounded products and sums); the safety margin on the
# coordinate; the absolute error of a normal in units of u and of its Box-Muller
# radius (the hardware sine and cosine are accurate to an absolute, not a relative,
# error near their zeros).
FP32_MODEL = (2.0 ** -24, 8.0, 8.0, 4.0, 16.0)

_default: Optional[Oracle] = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default

"""Seeded synthetic inputs for the local-volatility Monte Carlo.

This module only *describes* inputs: grid axes, vol surfaces drawn from closed
formulas plus seeded node noise, option books, path and step counts.  It holds
none of the pricing method's arithmetic (no stepping, interpolation, random
increments or payoffs), so both the GPU library's tests and the CPU oracle can
take their inputs from here without sharing any of the method.

The paper (arXiv 2002.02481, Sec. IV-C/IV-D) prices one European call on a
vol grid of 30 x 60 = 1800 nodes with 500K paths and 156 steps, on surface data
from Savine's textbook example that is not reproduced here.  The workloads below
are synthetic stand-ins of that shape (and of smaller and larger shapes), with
spot 100, zero rates and weekly steps.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

SPOT = 100.0
WEEK = 1.0 / 52.0

LIN = 0  # nodes uniform in S
LOG = 1  # nodes uniform in ln S


@dataclass(frozen=True)
class Axis:
    """Inclusive uniform grid in the axis coordinate (S for LIN, ln S for LOG)."""

    n: int
    kind: int
    lo: float
    hi: float

    def nodes(self) -> np.ndarray:
        if self.kind == LOG:
            return np.exp(np.linspace(np.log(self.lo), np.log(self.hi), self.n))
        return np.linspace(self.lo, self.hi, self.n)


@dataclass
class Surface:
    """Vol nodes sigma[i, j] at (spot node i, time node j), float64, C order."""

    spot_axis: Axis
    time_axis: Axis
    sigma: np.ndarray

    def __post_init__(self):
        self.sigma = np.ascontiguousarray(self.sigma, dtype=np.float64)
        assert self.sigma.shape == (self.spot_axis.n, self.time_axis.n)

    def rounded_to_f32(self) -> "Surface":
        """The same surface with nodes rounded to float32 (what an FP32 kernel sees)."""
        return Surface(self.spot_axis, self.time_axis,
                       self.sigma.astype(np.float32).astype(np.float64))


@dataclass
class Book:
    """European options on one underlying: put flag, strike, maturity (years), weight."""

    is_put: np.ndarray
    strike: np.ndarray
    maturity: np.ndarray
    weight: np.ndarray

    def __post_init__(self):
        self.is_put = np.ascontiguousarray(self.is_put, dtype=np.int32)
        self.strike = np.ascontiguousarray(self.strike, dtype=np.float64)
        self.maturity = np.ascontiguousarray(self.maturity, dtype=np.float64)
        self.weight = np.ascontiguousarray(self.weight, dtype=np.float64)

    @property
    def n(self) -> int:
        return int(self.strike.shape[0])


@dataclass
class Workload:
    name: str
    surfaces: List[Surface]
    book: Book
    n_paths: int
    n_steps: int
    seed: int = 0
    spot: float = SPOT
    adjoint: str = "stored"     # "stored" | "checkpoint"
    ckpt_every: int = 16
    note: str = ""

    @property
    def surface(self) -> Surface:
        return self.surfaces[0]

    @property
    def path_steps(self) -> int:
        return self.n_paths * self.n_steps * len(self.surfaces)

    def with_paths(self, n_paths: int) -> "Workload":
        return replace(self, n_paths=int(n_paths), name=f"{self.name}@{n_paths}")

    def with_surfaces(self, k: int) -> "Workload":
        return replace(self, surfaces=self.surfaces[:k], name=f"{self.name}[{k}surf]")


def call(strike: float, maturity: float) -> Book:
    return Book([0], [strike], [maturity], [1.0])


def put(strike: float, maturity: float) -> Book:
    return Book([1], [strike], [maturity], [1.0])


# --------------------------------------------------------------------------
# Surfaces
# --------------------------------------------------------------------------
def smile_surface(spot_axis: Axis, time_axis: Axis, base: float, amp: float,
                  decay: bool) -> np.ndarray:
    """base + amp * g(t) * ((S - 100)/100)^2 with g(t) = exp(-t) or (0.5 + t)."""
    S = spot_axis.nodes()[:, None]
    t = time_axis.nodes()[None, :]
    g = np.exp(-t) if decay else (0.5 + t)
    return base + amp * g * ((S - SPOT) / SPOT) ** 2


def noisy(sigma: np.ndarray, sd: float, seed: int, lo: float = 0.05, hi: float = 0.8) -> np.ndarray:
    """Add N(0, sd^2) node noise from numpy's PCG64 stream `seed`, clamp to [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.clip(sigma + rng.normal(0.0, sd, size=sigma.shape), lo, hi)


def small_surface() -> Surface:
    """21 spots linear 50..200 x 13 times 0..1y, sigma = 0.15 + 0.10 e^-t ((S-100)/100)^2."""
    sa, ta = Axis(21, LIN, 50.0, 200.0), Axis(13, LIN, 0.0, 1.0)
    return Surface(sa, ta, smile_surface(sa, ta, 0.15, 0.10, decay=True))


def flat_surface(like: Surface, sigma: float) -> Surface:
    return Surface(like.spot_axis, like.time_axis, np.full(like.sigma.shape, float(sigma)))


def book_surface(seed: int = 0) -> Surface:
    """60 spots log-spaced 40..250 x 30 times 0..3y,
    sigma = 0.12 + 0.12 (0.5+t) ((S-100)/100)^2 + N(0, 0.005^2), clamped to [0.05, 0.8]."""
    sa, ta = Axis(60, LOG, 40.0, 250.0), Axis(30, LIN, 0.0, 3.0)
    return Surface(sa, ta, noisy(smile_surface(sa, ta, 0.12, 0.12, decay=False), 0.005, seed))


def wide_surface(seed: int) -> Surface:
    """100 spots linear 50..200 x 50 times 0..5y, the small surface's formula,
    plus N(0, 0.01^2) node noise from stream `seed`, clamped to [0.05, 0.8]."""
    sa, ta = Axis(100, LIN, 50.0, 200.0), Axis(50, LIN, 0.0, 5.0)
    return Surface(sa, ta, noisy(smile_surface(sa, ta, 0.15, 0.10, decay=True), 0.01, seed))


def book64() -> Book:
    """64 calls/puts: strike 60 + 90k/63 (60%..150% of spot), maturity
    (0.25, 0.5, 1, 2, 3)[k mod 5] years, call for even k, put for odd k, weight 1."""
    k = np.arange(64)
    tenors = np.array([0.25, 0.5, 1.0, 2.0, 3.0])
    return Book((k % 2).astype(np.int32), 60.0 + 90.0 * k / 63.0, tenors[k % 5], np.ones(64))


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------
def small_call() -> Workload:
    """One ATM call, T = 1y, 52 weekly steps, 16384 paths, 21 x 13 grid."""
    return Workload("small_call_21x13_16k", [small_surface()], call(100.0, 1.0),
                    n_paths=16384, n_steps=52)


def single_call_60x30() -> Workload:
    """One ATM call, T = 3y, 156 weekly steps, 2^19 paths, 60 x 30 noisy grid,
    stored-state adjoint.  The shape of the paper's timing run (500K paths, 156
    steps, 1800 nodes)."""
    return Workload("call_60x30_524k_156", [book_surface(0)], call(100.0, 3.0),
                    n_paths=524288, n_steps=156)


def precision_study(flat: bool = False) -> Workload:
    """2^22 paths, 52 steps, the small grid (or a flat 0.2 surface on it)."""
    s = small_surface()
    if flat:
        s = flat_surface(s, 0.2)
    return Workload("precision_21x13_4M" + ("_flat" if flat else ""), [s], call(100.0, 1.0),
                    n_paths=4194304, n_steps=52)


def book_60x30() -> Workload:
    """64 calls/puts of uneven maturity on one set of 2^20 paths, 156 steps,
    60 x 30 grid; gradient of the total book value."""
    return Workload("book64_60x30_1M_156", [book_surface(0)], book64(),
                    n_paths=1048576, n_steps=156)


def surface_batch(n_surf: int = 32) -> Workload:
    """32 perturbed 100 x 50 surfaces (noise streams 1..32), one call, T = 5y,
    260 steps, 2^24 paths, checkpointed adjoint every 16 steps."""
    return Workload("batch32_100x50_16M_260", [wide_surface(s) for s in range(1, n_surf + 1)],
                    call(100.0, 5.0), n_paths=16777216, n_steps=260,
                    adjoint="checkpoint", ckpt_every=16)


ALL = {
    "small_call": small_call,
    "single_call_60x30": single_call_60x30,
    "precision_study": precision_study,
    "book_60x30": book_60x30,
    "surface_batch": surface_batch,
}


def tiny_surface(kind: int = LIN, n_spot: int = 5, n_time: int = 4, seed: int = 7,
                 t_hi: float = 1.0) -> Surface:
    """Small random grids for brute-force checks (values in [0.1, 0.4])."""
    if kind == LOG:
        sa = Axis(n_spot, LOG, 70.0, 140.0)
    else:
        sa = Axis(n_spot, LIN, 70.0, 140.0)
    ta = Axis(n_time, LIN, 0.0, t_hi)
    rng = np.random.default_rng(seed)
    return Surface(sa, ta, rng.uniform(0.1, 0.4, size=(n_spot, n_time)))

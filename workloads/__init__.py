"""Seeded synthetic inputs for the fast directional Helmholtz matvec.

This module only draws random numbers and lays out point sets.  It holds none
of the method's arithmetic, so both the CPU oracle (through the tests) and the
GPU library (through the tests and the benchmark) are fed from it without
sharing any computation.

Every generator uses numpy's PCG64 (``np.random.default_rng``), which is
bit-reproducible across machines.  The draw order inside one problem is fixed:
target points, then source points, then the real parts of ``v``, then the
imaginary parts.

Workloads (all synthetic; the paper itself uses a synthetic tensor grid,
Sect. 4, so there is no external data set to stand in for):

* ``uniform``: i.i.d. points in the unit cube ``(0,1]^3`` (drawn as
  ``1 - U[0,1)``), separate target and source sets, complex ``v`` with
  i.i.d. N(0,1) real and imaginary parts.
* ``paper_grid``: the tensor grid of Sect. 4, ``x_n = (2n-1) 2^-k - 1`` for
  ``n = 1..2^k`` in each axis (x slowest), targets equal sources, box
  ``(-1,1]^3``, ``kappa = 0.1 * 2^k``, depth ``k-3``.
* ``clustered``: 8 Gaussian blobs (sigma 0.05) with centres uniform in
  ``[0.25,0.75]^3``, each point picking a blob uniformly, coordinates clamped
  into ``[2^-52, 1]`` so that they lie in ``(0,1]``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

UNIT_BOX = (0.0, 0.0, 0.0, 1.0, 1.0, 1.0)


@dataclass
class Problem:
    """One matvec problem: points, charges and method parameters."""

    name: str
    points_T: np.ndarray  # (n_T, 3) float64, user order
    points_S: np.ndarray  # (n_S, 3) float64, user order
    v: np.ndarray  # (n_S,) complex128
    kappa: float
    box: tuple  # (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z), half-open (lo, hi]
    levels: int  # levels below the root
    m: int  # Chebyshev degree per axis
    same_points: bool = False  # targets and sources are the same array
    meta: dict = field(default_factory=dict)


def unit_cube_points(rng: np.random.Generator, n: int) -> np.ndarray:
    """i.i.d. uniform points in (0,1]^3 (1 - U[0,1) excludes 0, includes 1)."""
    return 1.0 - rng.random((n, 3))


def complex_normal(rng: np.random.Generator, n: int) -> np.ndarray:
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return re + 1j * im


def uniform_problem(name: str, seed: int, n: int, kappa: float, levels: int,
                    m: int, n_S: int | None = None) -> Problem:
    rng = np.random.default_rng(seed)
    n_S = n if n_S is None else n_S
    pt = unit_cube_points(rng, n)
    ps = unit_cube_points(rng, n_S)
    v = complex_normal(rng, n_S)
    return Problem(name, pt, ps, v, float(kappa), UNIT_BOX, levels, m)


def clustered_points(rng: np.random.Generator, n: int, n_blobs: int = 8,
                     sigma: float = 0.05) -> np.ndarray:
    centres = 0.25 + 0.5 * rng.random((n_blobs, 3))
    pick = rng.integers(0, n_blobs, size=n)
    pts = centres[pick] + sigma * rng.standard_normal((n, 3))
    return np.clip(pts, 2.0 ** -52, 1.0)


def paper_grid_points(k: int) -> np.ndarray:
    """Tensor grid of Sect. 4: 8^k points, x slowest, in (-1,1)^3."""
    n1 = 2 ** k
    x = (2.0 * np.arange(1, n1 + 1) - 1.0) * 2.0 ** (-k) - 1.0
    gx, gy, gz = np.meshgrid(x, x, x, indexing="ij")
    return np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)


def paper_grid_problem(k: int, m: int = 4, seed: int = 0) -> Problem:
    pts = paper_grid_points(k)
    rng = np.random.default_rng(seed)
    v = complex_normal(rng, pts.shape[0])
    return Problem(f"paper_k{k}", pts, pts, v, 0.1 * 2.0 ** k,
                   (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0), k - 3, m,
                   same_points=True, meta={"k": k})


# Named uniform workloads: (seed, N, kappa, levels, m).
UNIFORM = {
    "uniform2k": (1, 2000, 20.0, 3, 4),
    "uniform100k": (2, 100_000, 60.0, 5, 5),
    "uniform1m": (3, 1_000_000, 150.0, 7, 6),
    "uniform4m": (5, 4_000_000, 400.0, 8, 6),
}


# Small problems at the highest interpolation degrees (m = 7, 8: K = 512,
# 729), separate random target and source sets in the unit cube:
# name -> (seed, n_T, n_S, kappa, levels, m).
HIGH_DEGREE = {
    "degree7": (701, 600, 560, 20.0, 3, 7),
    "degree8": (702, 500, 480, 12.0, 3, 8),
}


def config(name: str) -> Problem:
    if name in UNIFORM:
        seed, n, kappa, levels, m = UNIFORM[name]
        return uniform_problem(name, seed, n, kappa, levels, m)
    if name.startswith("paper_k"):
        return paper_grid_problem(int(name[len("paper_k"):]))
    if name in HIGH_DEGREE:
        seed, nT, nS, kappa, levels, m = HIGH_DEGREE[name]
        return random_problem(seed, nT, nS, kappa, levels, m)
    raise KeyError(name)


def batch_levels(n: int) -> int:
    """Tree depth for a batched problem: about 3-4 points per leaf."""
    return int(min(6, max(3, round(math.log(n / 4.0, 8)))))


def batch_problems(seed: int = 4, count: int = 64, m: int = 5,
                   n_lo: float = 1e4, n_hi: float = 2e5) -> list[Problem]:
    """Independent problems of uneven size and wave number (batched mode).

    Problem i draws N log-uniform in [n_lo, n_hi] and kappa uniform in
    [10, 80]; the first half is uniform in the cube, the second half is
    clustered.  ``v`` is rounded to complex64 (the batched mode's I/O type).
    """
    out = []
    for i, ss in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(ss)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        kappa = float(rng.uniform(10.0, 80.0))
        if i < count // 2:
            pt = unit_cube_points(rng, n)
            ps = unit_cube_points(rng, n)
            kind = "uniform"
        else:
            pt = clustered_points(rng, n)
            ps = clustered_points(rng, n)
            kind = "clustered"
        v = complex_normal(rng, n).astype(np.complex64).astype(np.complex128)
        out.append(Problem(f"batch{i}", pt, ps, v, kappa, UNIT_BOX,
                           batch_levels(n), m, meta={"kind": kind}))
    return out


def random_problem(seed: int, n_T: int, n_S: int, kappa: float, levels: int,
                   m: int, box=UNIT_BOX) -> Problem:
    """Small random problem in an arbitrary cubic box (tests)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(box[:3])
    hi = np.asarray(box[3:])
    pt = hi - (hi - lo) * rng.random((n_T, 3))
    ps = hi - (hi - lo) * rng.random((n_S, 3))
    v = complex_normal(rng, n_S)
    return Problem(f"rand{seed}", pt, ps, v, float(kappa), tuple(box), levels, m)


def clustered_problem(seed: int, n_T: int, n_S: int, kappa: float, levels: int,
                      m: int) -> Problem:
    """Small clustered problem in the unit cube (tests): Gaussian blobs, so
    that the leaf levels hold many empty boxes."""
    rng = np.random.default_rng(seed)
    pt = clustered_points(rng, n_T)
    ps = clustered_points(rng, n_S)
    v = complex_normal(rng, n_S)
    return Problem(f"clus{seed}", pt, ps, v, float(kappa), UNIT_BOX, levels, m)

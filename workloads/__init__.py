"""Seeded synthetic inputs for the H2-ULV solver (points, right-hand sides).

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
no arithmetic of the factorization method: it only draws point clouds and
Gaussian right-hand sides from NumPy's PCG64 generator with fixed seeds.

Workloads (point clouds stand in for the paper's geometries; the paper's own
unit-cube Laplace test is in its Section IV, the boundary-element Yukawa test
in Section V, whose hemoglobin meshes are not available here):

  cube      N points uniform in the unit cube [0,1)^3            (Section IV)
  sphere    N points uniform on the unit sphere (normalised Gaussians)
  boxes     N points uniform in an axis-aligned box of random aspect ratio
  ellipsoid union of 12 random ellipsoid surfaces (stands in for the complex
            surface geometry of Section V)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LAPLACE = 0
YUKAWA = 1


def cube_points(n: int, seed: int) -> np.ndarray:
    """N x 3 float64, uniform in [0,1)^3."""
    rng = np.random.default_rng(seed)
    return rng.random((n, 3))


def sphere_points(n: int, seed: int) -> np.ndarray:
    """N x 3 float64, uniform on the unit sphere (g / |g|, g ~ N(0, I3))."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def line_points(n: int, seed: int | None = None) -> np.ndarray:
    """N points on the x axis in [0,1): evenly spaced if seed is None, else uniform."""
    x = np.zeros((n, 3))
    if seed is None:
        x[:, 0] = (np.arange(n) + 0.5) / n
    else:
        x[:, 0] = np.sort(np.random.default_rng(seed).random(n))
    return x


def box_problem(p: int) -> np.ndarray:
    """Problem p (0..63) of the batched workload: N log-uniform in [8192, 131072],
    points uniform in an axis-aligned box with sides (1, u1, u2), u ~ U[1, 4],
    axes shuffled."""
    rng = np.random.default_rng(3000 + p)
    n = int(round(math.exp(rng.uniform(math.log(8192), math.log(131072)))))
    sides = np.array([1.0, rng.uniform(1, 4), rng.uniform(1, 4)])
    rng.shuffle(sides)
    return rng.random((n, 3)) * sides


def aspect_box_points(n: int, seed: int) -> np.ndarray:
    """N points uniform in an axis-aligned box with sides (1, u1, u2), u ~ U[1, 4],
    axes shuffled: the batched workload's geometry at a chosen size."""
    rng = np.random.default_rng(seed)
    sides = np.array([1.0, rng.uniform(1, 4), rng.uniform(1, 4)])
    rng.shuffle(sides)
    return rng.random((n, 3)) * sides


def ellipsoid_points(n: int, seed: int, n_ell: int = 12) -> np.ndarray:
    """Union of n_ell random ellipsoid surfaces: semi-axes U[0.05, 0.5]^3, random
    rotation (QR of a Gaussian, column signs fixed by diag(R) > 0), centres
    U[0,1]^3; N // n_ell points each, the last takes the remainder; points are
    uniform-sphere samples scaled by the semi-axes."""
    rng = np.random.default_rng(seed)
    out = []
    per = n // n_ell
    for e in range(n_ell):
        cnt = per if e < n_ell - 1 else n - per * (n_ell - 1)
        axes = rng.uniform(0.05, 0.5, 3)
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.where(np.diag(r) == 0, 1.0, np.diag(r)))
        centre = rng.random(3)
        g = rng.standard_normal((cnt, 3))
        s = g / np.linalg.norm(g, axis=1, keepdims=True)
        out.append((s * axes) @ q.T + centre)
    return np.concatenate(out, axis=0)


def gaussian_rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """n x nrhs Gaussian N(0,1) right-hand sides, column-major (Fortran order)."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, nrhs)))


@dataclass
class Problem:
    """One solver input: points, kernel and accuracy parameters, RHS."""
    name: str
    points: np.ndarray
    kernel: int = LAPLACE
    alpha: float = 0.0
    diag: float = 1e3
    eta: float = 1.0
    leaf: int = 64
    tol: float = 1e-8
    rank_cap: int = 0
    far_sample: int = 32
    nrhs: int = 1
    rhs_seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    def rhs(self) -> np.ndarray:
        return gaussian_rhs(self.n, self.nrhs, self.rhs_seed)


def small_cube(n: int = 2048, far_sample: int = 0) -> Problem:
    """N=2048 unit-cube Laplace, leaf 64, eta 1, ID tolerance 1e-8, rank cap 32,
    one Gaussian RHS (far field taken exactly by default at this size)."""
    return Problem("cube2048", cube_points(n, 1), LAPLACE, 0.0, 1e3, 1.0, 64,
                   1e-8, 32, far_sample, 1, 101)


def sphere65k() -> Problem:
    """N=65536 on the unit sphere, Laplace, leaf 256, eta 1, tol 1e-8, cap 128,
    16 RHS."""
    return Problem("sphere65536", sphere_points(65536, 2), LAPLACE, 0.0, 1e3,
                   1.0, 256, 1e-8, 128, 32, 16, 102)


def default_cap(leaf: int) -> int:
    """Rank cap of a configuration that names none: half the leaf size, the cap
    the two configurations that name one use (leaf 64 -> 32, leaf 256 -> 128).
    A parent's candidate rows are its children's skeletons, so with this cap no
    box at any level holds more rows than a leaf."""
    return leaf // 2


def cube1m(n: int = 1 << 20) -> Problem:
    """N=2^20 unit-cube Laplace, leaf 256, eta 1, tol 1e-6, rank cap 128
    (leaf / 2), 8 RHS."""
    return Problem(f"cube{n}", cube_points(n, 4), LAPLACE, 0.0, 1e3, 1.0, 256,
                   1e-6, default_cap(256), 32, 8, 104)


def yukawa_batch(count: int = 64) -> list[Problem]:
    """The 64-problem Yukawa exp(-0.5 r)/r batch, leaf 128, eta 1, tol 1e-7,
    rank cap 64 (leaf / 2)."""
    return [Problem(f"yukawa{p}", box_problem(p), YUKAWA, 0.5, 1e3, 1.0, 128,
                    1e-7, default_cap(128), 32, 1, 3100 + p) for p in range(count)]


def ellipsoids(n: int = 262144, seed: int = 5) -> Problem:
    """N=262144 on 12 ellipsoid surfaces, Laplace, leaf 256, tol 1e-6, rank cap
    128 (leaf / 2)."""
    return Problem(f"ellipsoids{n}", ellipsoid_points(n, seed), LAPLACE, 0.0,
                   1e3, 1.0, 256, 1e-6, default_cap(256), 32, 1, 105)

"""Seeded synthetic APD instances (inputs only).

This module builds the inputs of the APD problem -- seeds, anisotropy
matrices, target volumes and grid sizes -- for the five workloads the
library is measured on.  It holds none of the method's arithmetic (no cost,
no assignment, no objective, no solver): both the CPU oracle and the GPU
path take their inputs from here, and nothing else is shared between them.

Every generator draws from ``numpy.random.default_rng(seed)`` (PCG64), so an
instance is a pure function of (workload, seed).

Workloads (all on the unit box, seeds iid uniform, det A_i = 1):

* ``c1``  2D, 256x256 pixels, N = 16.  A_i = R(t) diag(a, 1/a) R(t)^T with
  t ~ U[0, pi), a ~ U[1, 3]; v_i = 1/16.
* ``c2``  2D, 1024x1024 pixels, N = 1000.  a ~ U[1, 4], t ~ U[0, pi);
  v = exp(0.35 Z) renormalised to sum 1 (log-normal, sigma = 0.35).
* ``c3``  3D, 256^3 voxels, N = 10000.  A_i = R_i diag(a) R_i^T with R_i
  Haar-uniform on SO(3) (normalised Gaussian quaternion), log a_k ~ N(0, 0.3^2),
  a scaled to product 1; v log-normal with sigma = 0.3.
* ``c4``  a batch of 512 independent 2D instances, N_b ~ U{50..2000},
  A and v as in ``c1`` (v = 1/N_b), grid side M_b = clamp(roundup64(20 sqrt(N_b)),
  256, 1024).
* ``c5``  2D, 512x512 pixels, N ~ U{200..1000}, A as in ``c1``, v = 1/N.

The 2D anisotropy form is the ellipse parameterisation of Section 2.1,
eq. (2.2), with unit determinant; the 3D form is its ellipsoid analogue.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Instance",
    "rot2",
    "aniso2d",
    "haar_so3",
    "aniso3d",
    "lognormal_volumes",
    "make_c1",
    "make_c2",
    "make_c3",
    "make_c4_batch",
    "make_c5",
    "make",
    "custom",
    "disk_weights",
    "masked",
    "make_microstructure",
    "seed_for",
]


@dataclass
class Instance:
    """One APD problem: box [lo, hi], grid of M_d pixels per axis, seeds x
    (n, D), anisotropy matrices A (n, D, D), target volumes v (n,)."""

    dim: int
    grid: tuple
    lo: tuple
    hi: tuple
    x: np.ndarray
    A: np.ndarray
    v: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)
    mass: np.ndarray = None   # optional pixel weights q_j in [0, 255] (J,), uint8
    power: int = 2            # cost |y - x|_A^power - w (2: the anisotropic power diagram)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def J(self) -> int:
        return int(np.prod(self.grid))

    @property
    def pairs(self) -> int:
        return self.n * self.J


def seed_for(config: int, run: int) -> int:
    """RNG seed of run `run` of workload `config` (1..5)."""
    return 1000 * config + run


def rot2(theta: np.ndarray) -> np.ndarray:
    c, s = np.cos(theta), np.sin(theta)
    R = np.empty(theta.shape + (2, 2))
    R[..., 0, 0] = c
    R[..., 0, 1] = -s
    R[..., 1, 0] = s
    R[..., 1, 1] = c
    return R


def aniso2d(a: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """A = R(theta) diag(a, 1/a) R(theta)^T, symmetrised (det 1)."""
    R = rot2(theta)
    D = np.zeros(a.shape + (2, 2))
    D[..., 0, 0] = a
    D[..., 1, 1] = 1.0 / a
    A = R @ D @ np.swapaxes(R, -1, -2)
    return 0.5 * (A + np.swapaxes(A, -1, -2))


def haar_so3(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-uniform rotations from normalised 4D Gaussian quaternions."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def aniso3d(R: np.ndarray, a: np.ndarray) -> np.ndarray:
    """A = R diag(a) R^T, symmetrised."""
    A = np.einsum("nij,nj,nkj->nik", R, a, R)
    return 0.5 * (A + np.swapaxes(A, -1, -2))


def lognormal_volumes(rng: np.random.Generator, n: int, sigma: float,
                      total: float = 1.0) -> np.ndarray:
    """log v ~ N(0, sigma^2), then scaled so that sum v = total exactly
    (to the last bit where possible)."""
    v = np.exp(sigma * rng.standard_normal(n))
    v = v / v.sum() * total
    # push the rounding residue into the largest entry
    v[np.argmax(v)] += total - v.sum()
    return v


def _uniform_volumes(n: int, total: float = 1.0) -> np.ndarray:
    v = np.full(n, total / n)
    v[0] += total - v.sum()
    return v


def make_c1(seed: int = seed_for(1, 0)) -> Instance:
    rng = np.random.default_rng(seed)
    n = 16
    x = rng.random((n, 2))
    theta = rng.uniform(0.0, np.pi, n)
    a = rng.uniform(1.0, 3.0, n)
    return Instance(2, (256, 256), (0.0, 0.0), (1.0, 1.0), x,
                    aniso2d(a, theta), _uniform_volumes(n), "c1", {"seed": seed})


def make_c2(seed: int = seed_for(2, 0), M: int = 1024) -> Instance:
    """The 2D workload (N = 1000) on an M x M grid (1024 by default; finer
    grids for the boundary-aware refinement)."""
    rng = np.random.default_rng(seed)
    n = 1000
    x = rng.random((n, 2))
    theta = rng.uniform(0.0, np.pi, n)
    a = rng.uniform(1.0, 4.0, n)
    v = lognormal_volumes(rng, n, 0.35)
    return Instance(2, (M, M), (0.0, 0.0), (1.0, 1.0), x,
                    aniso2d(a, theta), v, "c2", {"seed": seed, "M": M})


def make_c3(seed: int = seed_for(3, 0), n: int = 10000, M: int = 256) -> Instance:
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3))
    R = haar_so3(rng, n)
    la = 0.3 * rng.standard_normal((n, 3))
    la -= la.mean(axis=1, keepdims=True)  # product of the a_k is 1
    A = aniso3d(R, np.exp(la))
    v = lognormal_volumes(rng, n, 0.3)
    return Instance(3, (M, M, M), (0.0,) * 3, (1.0,) * 3, x, A, v, "c3",
                    {"seed": seed})


def c4_grid_side(n: int) -> int:
    """Per-instance grid side of the batched workload:
    clamp(roundup64(20 sqrt(n)), 256, 1024)."""
    m = int(np.ceil(20.0 * np.sqrt(n) / 64.0)) * 64
    return int(min(max(m, 256), 1024))


def make_c4_instance(b: int) -> Instance:
    rng = np.random.default_rng(4000 + b)
    n = int(rng.integers(50, 2001))
    x = rng.random((n, 2))
    theta = rng.uniform(0.0, np.pi, n)
    a = rng.uniform(1.0, 3.0, n)
    M = c4_grid_side(n)
    return Instance(2, (M, M), (0.0, 0.0), (1.0, 1.0), x, aniso2d(a, theta),
                    _uniform_volumes(n), f"c4[{b}]", {"seed": 4000 + b})


def make_c4_batch(count: int = 512, start: int = 0) -> list:
    return [make_c4_instance(b) for b in range(start, start + count)]


def make_c5(seed: int, n: int | None = None, M: int = 512) -> Instance:
    rng = np.random.default_rng(seed)
    if n is None:
        n = int(rng.integers(200, 1001))
    x = rng.random((n, 2))
    theta = rng.uniform(0.0, np.pi, n)
    a = rng.uniform(1.0, 3.0, n)
    return Instance(2, (M, M), (0.0, 0.0), (1.0, 1.0), x, aniso2d(a, theta),
                    _uniform_volumes(n), "c5", {"seed": seed})


def make_microstructure(seed: int, M: int, n: int = 4587) -> Instance:
    """A 2D polycrystal-like instance at the scale of the paper's synthetic
    microstructure (Section 3.4: N = 4587 grains, areas spanning a factor
    of about 190): areas log-normal (sigma 0.91, tails clipped at 2.9 sigma,
    so max/min = exp(5.28) ~ 196) normalised to |Omega| = 1, ellipse aspect
    ratios r = a/b >= 1 with log r = 0.35 |z| + 0.25 max(0, -z_v) (small
    grains more elongated, as the paper observes in its data), angles
    U[0, pi), A = A(a^, b^, theta) of eq. (2.2) with a^ = sqrt(r), b^ = 1/a^,
    i.e. R diag(1/r, r) R^T; seeds uniform (the X^0 of Algorithm 3).  The
    grid side M is the caller's (eq. (2.10) for the target tolerance)."""
    rng = np.random.default_rng(seed)
    zv = np.clip(rng.standard_normal(n), -2.9, 2.9)
    v = np.exp(0.91 * zv)
    v = v / v.sum()
    v[np.argmax(v)] += 1.0 - v.sum()
    r = np.exp(0.35 * np.abs(rng.standard_normal(n)) + 0.25 * np.maximum(0.0, -zv))
    theta = rng.uniform(0.0, np.pi, n)
    x = rng.random((n, 2))
    return Instance(2, (int(M), int(M)), (0.0, 0.0), (1.0, 1.0), x, aniso2d(1.0 / r, theta), v,
                    "microstructure", {"seed": seed})


def disk_weights(grid, lo, hi, centre, radius, sub: int = 4) -> np.ndarray:
    """Pixel weights of a disk (2D) or ball (3D) domain inside the box:
    q_j = round(255 x the fraction of sub^D sample points of pixel j inside),
    so interior pixels weigh 255, outside ones 0, boundary pixels in
    between.  Row-major, last axis fastest."""
    dim = len(grid)
    axes = []
    for d in range(dim):
        s = (hi[d] - lo[d]) / grid[d]
        off = (np.arange(sub) + 0.5) / sub
        pts = lo[d] + (np.arange(grid[d])[:, None] + off[None, :]) * s   # (M_d, sub)
        axes.append((pts - centre[d]) ** 2)
    if dim == 2:
        r2 = axes[0][:, None, :, None] + axes[1][None, :, None, :]
    else:
        r2 = (axes[0][:, None, None, :, None, None] + axes[1][None, :, None, None, :, None]
              + axes[2][None, None, :, None, None, :])
    inside = (r2 <= radius * radius).reshape(tuple(grid) + (-1,)).mean(axis=-1)
    return np.rint(255.0 * inside).astype(np.uint8).reshape(-1)


def masked(inst: "Instance", q: np.ndarray) -> "Instance":
    """The instance on the sub-domain given by pixel weights q: the target
    volumes are rescaled to the domain's measure sum_j (q_j/255)|P|."""
    pix = float(np.prod([(inst.hi[d] - inst.lo[d]) / inst.grid[d] for d in range(inst.dim)]))
    measure = float(np.sum(q.astype(np.int64))) * pix / 255.0
    v = inst.v / inst.v.sum() * measure
    v[np.argmax(v)] += measure - v.sum()
    return Instance(inst.dim, inst.grid, inst.lo, inst.hi, inst.x, inst.A, v,
                    inst.name + "-masked", dict(inst.meta), mass=np.asarray(q, np.uint8))


def custom(dim: int, n: int, M, seed: int, amax: float = 3.0,
           sigma: float = 0.0, lo=None, hi=None, iso: bool = False) -> Instance:
    """A small instance of any shape for tests: seeds uniform in the box,
    2D anisotropy a ~ U[1, amax] (3D: log a ~ N(0, (log amax / 3)^2)),
    volumes uniform (sigma = 0) or log-normal."""
    rng = np.random.default_rng(seed)
    grid = tuple([int(M)] * dim) if np.isscalar(M) else tuple(int(m) for m in M)
    lo = tuple([0.0] * dim) if lo is None else tuple(float(t) for t in lo)
    hi = tuple([1.0] * dim) if hi is None else tuple(float(t) for t in hi)
    lo_a, hi_a = np.array(lo), np.array(hi)
    x = lo_a + (hi_a - lo_a) * rng.random((n, dim))
    if iso:
        A = np.broadcast_to(np.eye(dim), (n, dim, dim)).copy()
    elif dim == 2:
        A = aniso2d(rng.uniform(1.0, amax, n), rng.uniform(0.0, np.pi, n))
    else:
        la = (np.log(amax) / 3.0) * rng.standard_normal((n, 3))
        la -= la.mean(axis=1, keepdims=True)
        A = aniso3d(haar_so3(rng, n), np.exp(la))
    omega = float(np.prod(hi_a - lo_a))
    v = _uniform_volumes(n, omega) if sigma == 0.0 else lognormal_volumes(rng, n, sigma, omega)
    return Instance(dim, grid, lo, hi, x, A, v, f"custom{dim}d", {"seed": seed})


def make(name: str, run: int = 0) -> Instance:
    if name == "c1":
        return make_c1(seed_for(1, run))
    if name == "c2":
        return make_c2(seed_for(2, run))
    if name == "c3":
        return make_c3(seed_for(3, run))
    if name == "c5":
        return make_c5(600000 + run)
    raise ValueError(f"unknown workload {name!r}")

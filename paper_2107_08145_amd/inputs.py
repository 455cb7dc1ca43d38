"""Seeded synthetic inputs for the short-characteristics radiation transport solver.

This module is shared by the tests, the benchmark and the smoke check.  It
holds no arithmetic of the transfer solution itself: it only produces the
problem statement (grid, angular quadrature, opacities, densities, source
functions, boundary settings) that both the HIP library and the CPU oracle
receive as plain arrays.

Paper context (arXiv 2107.08145, section "Summary of the Radiation Transport
Solver"): the mean intensity is integrated over the unit sphere with three rays
per octant, 24 rays in total, from a Carlson quadrature; several frequency bands
(opacity bins) each need their own solve.  The paper prints neither the
quadrature values nor any atmosphere, so the readings below are ours:

* Quadrature: the level-symmetric S4 set.  Every direction is a signed
  permutation of (mu1, mu1, mu2) with mu1^2 + mu1^2 + mu2^2 = 1 and equal weights
  1/24.  mu1 is fixed by the even-moment condition sum_r w mu_x^4 = 1/5, which
  gives mu1^2 = (2 - sqrt(1.6)) / 6.  Order: octant signs (sx, sy, sz) with +
  before - and sx slowest, then the axis that carries mu2 (x, y, z).
* Atmosphere: plane-parallel stratification with the bottom layer at k = 0,
  rho(z) = exp(-z/H_rho), T(z) = 1 + 2 exp(-z/10), S = T^4 exp(0.1 g) with g
  standard normal per cell, kappa = 10^(lo + (hi-lo) u) with u uniform per cell,
  z = k * dz.  Draw order from one numpy PCG64 stream: all of g, then all of u,
  both in C order [z][y][x].
* Multi-band: four opacity bins with kappa_b = kappa * 10^(b-2) and
  S_b = w_b S, w = (0.4, 0.3, 0.2, 0.1), plus a fifth grey band (kappa, S) whose
  heating is reported separately (qweight 0).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Boundary-condition codes, identical to the C ABI's enumerations.
BOT_THERMAL = 0   # I = S in the bottom layer, for rays with mu_z > 0
BOT_FIXED = 1     # I = i_bot in the bottom layer
TOP_ZERO = 0      # I = 0 in the top layer, for rays with mu_z < 0
TOP_THERMAL = 1   # I = S in the top layer

PREC_FP64 = 0
PREC_FP32 = 1


def s4_mu1() -> float:
    """Smaller S4 direction cosine from the fourth-moment condition."""
    return math.sqrt((2.0 - math.sqrt(1.6)) / 6.0)


def s4_quadrature() -> tuple[np.ndarray, np.ndarray]:
    """24 unit directions [24][3] and equal weights [24] (sum 1)."""
    m1 = s4_mu1()
    m2 = math.sqrt(1.0 - 2.0 * m1 * m1)
    mus = []
    for sx in (1.0, -1.0):
        for sy in (1.0, -1.0):
            for sz in (1.0, -1.0):
                for big in range(3):
                    v = [m1, m1, m1]
                    v[big] = m2
                    mus.append([sx * v[0], sy * v[1], sz * v[2]])
    mu = np.asarray(mus, dtype=np.float64)
    w = np.full(24, 1.0 / 24.0)
    return mu, w


@dataclass
class Problem:
    """One box: grid, quadrature, per-band inputs and boundary settings."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    mu: np.ndarray            # [R][3]
    w: np.ndarray             # [R]
    kappa: np.ndarray         # [B][nz][ny][nx]
    rho: np.ndarray           # [nz][ny][nx]
    S: np.ndarray             # [B][nz][ny][nx]
    qweight: np.ndarray       # [B]
    bot: int = BOT_THERMAL
    top: int = TOP_ZERO
    i_bot: float = 0.0
    n_iter: int = 3
    meta: dict = field(default_factory=dict)

    @property
    def nbands(self) -> int:
        return int(self.kappa.shape[0])

    @property
    def nrays(self) -> int:
        return int(self.mu.shape[0])

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_up(self) -> int:
        return int(np.count_nonzero(self.mu[:, 2] > 0))

    def astype(self, dtype) -> "Problem":
        """Same problem with kappa, rho and S cast to `dtype` (float32 or float64)."""
        return Problem(self.nx, self.ny, self.nz, self.dx, self.dy, self.dz,
                       self.mu, self.w, self.kappa.astype(dtype), self.rho.astype(dtype),
                       self.S.astype(dtype), self.qweight, self.bot, self.top,
                       self.i_bot, self.n_iter, dict(self.meta))


def stratified(nx: int, ny: int, nz: int, seed: int, h_rho: float,
               kappa_range: tuple[float, float], dz: float = 1.0):
    """Grey stratified atmosphere: returns (kappa, rho, S), each [nz][ny][nx] float64."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((nz, ny, nx))
    u = rng.random((nz, ny, nx))
    lo, hi = math.log10(kappa_range[0]), math.log10(kappa_range[1])
    kappa = 10.0 ** (lo + (hi - lo) * u)
    z = np.arange(nz, dtype=np.float64) * dz
    rho1 = np.exp(-z / h_rho)
    t1 = 1.0 + 2.0 * np.exp(-z / 10.0)
    rho = np.broadcast_to(rho1[:, None, None], (nz, ny, nx)).copy()
    S = (t1 ** 4)[:, None, None] * np.exp(0.1 * g)
    return kappa, rho, S


BIN_WEIGHTS = (0.4, 0.3, 0.2, 0.1)


def multiband(kappa: np.ndarray, S: np.ndarray):
    """Four opacity bins plus the grey band: (kappa_b, S_b, qweight)."""
    kb = [kappa * 10.0 ** (b - 2) for b in range(4)] + [kappa]
    sb = [S * BIN_WEIGHTS[b] for b in range(4)] + [S]
    return np.stack(kb), np.stack(sb), np.array([1.0, 1.0, 1.0, 1.0, 0.0])


def make_problem(nx, ny, nz, seed, h_rho, kappa_range, bands: str = "grey",
                 n_iter: int = 3) -> Problem:
    kappa, rho, S = stratified(nx, ny, nz, seed, h_rho, kappa_range)
    if bands == "grey":
        kb, sb, qw = kappa[None], S[None], np.ones(1)
    elif bands == "bins+grey":
        kb, sb, qw = multiband(kappa, S)
    else:
        raise ValueError(bands)
    mu, w = s4_quadrature()
    return Problem(nx, ny, nz, 1.0, 1.0, 1.0, mu, w, kb, rho, sb, qw,
                   BOT_THERMAL, TOP_ZERO, 0.0, n_iter,
                   {"seed": seed, "h_rho": h_rho, "kappa_range": kappa_range, "bands": bands})


# The five workloads.  Seeds follow 1000 * workload + box.
def workload(name: str, size: int | None = None) -> Problem | list[Problem]:
    """Named workloads.  `size` overrides the cube edge for the scaled-down parity runs."""
    if name == "grey32":          # 32^3 grey, fp64 parity case
        n = size or 32
        return make_problem(n, n, n, 1000, 8.0, (0.1, 10.0))
    if name == "grey288":         # 288^3 grey, thin top to thick bottom
        n = size or 288
        return make_problem(n, n, n, 2000, 40.0, (1e-3, 1e3))
    if name == "bands288":        # 288^3, 4 opacity bins + grey
        n = size or 288
        return make_problem(n, n, n, 3000, 40.0, (1e-3, 1e3), bands="bins+grey")
    if name == "adjoint128":      # 128^3 grey, same atmosphere recipe as grey288
        n = size or 128
        return make_problem(n, n, n, 4000, 40.0, (1e-3, 1e3))
    if name == "boxes6":          # six uneven boxes, 4 bins + grey
        shapes = [(576, 576, 192), (384, 384, 256), (256, 256, 256),
                  (192, 192, 384), (96, 96, 512), (64, 64, 64)]
        if size is not None:      # scaled copy keeping the aspect ratios
            shapes = [(max(8, a * size // 576), max(8, b * size // 576), max(8, c * size // 576))
                      for a, b, c in shapes]
        return [make_problem(a, b, c, 5000 + i, 40.0, (1e-3, 1e3), bands="bins+grey")
                for i, (a, b, c) in enumerate(shapes)]
    raise KeyError(name)


def random_problem(nx: int, ny: int, nz: int, seed: int, bands: int = 1, lo: float = 1e-2,
                   hi: float = 1e2, h_rho: float = 8.0, **fields) -> Problem:
    """Small test problem: log-uniform kappa in [lo, hi] per band, exponential
    density, a stratified S with 10 % log-normal noise, S4 rays; `fields`
    overrides Problem attributes (bot, top, i_bot, n_iter, qweight, ...)."""
    r = np.random.default_rng(seed)
    kap = 10 ** r.uniform(math.log10(lo), math.log10(hi), (bands, nz, ny, nx))
    z = np.arange(nz, dtype=np.float64)
    rho = np.broadcast_to(np.exp(-z / h_rho)[:, None, None], (nz, ny, nx)).copy()
    S = ((1 + 2 * np.exp(-z / 10))[None, :, None, None] ** 4
         * np.exp(0.1 * r.standard_normal((bands, nz, ny, nx))))
    mu, w = s4_quadrature()
    p = Problem(nx, ny, nz, 1.0, 1.0, 1.0, mu, w, kap, rho, S, np.ones(bands))
    for k, v in fields.items():
        setattr(p, k, v)
    return p


def adjoint_seeds(p: Problem, seed: int):
    """Loss definition for the adjoint workload.

    L1 = sum over the top layer and upward rays of (I_top - I_target)^2, where
    I_target comes from the same solver run on S * (1 + 0.05 g') (g' seeded
    normal, seed + 1); L2 = sum(g * Q) with g uniform (seed + 2).  Returns the
    perturbed source function and g; I_target itself must be computed by the
    solver under test.
    """
    r1 = np.random.default_rng(seed + 1)
    s_target = p.S * (1.0 + 0.05 * r1.standard_normal(p.S.shape))
    r2 = np.random.default_rng(seed + 2)
    gq = r2.random((p.nz, p.ny, p.nx))
    return s_target, gq


def fd_cells(p: Problem, seed: int, count: int = 64) -> np.ndarray:
    """Flat cell indices for finite-difference spot checks (seed + 3)."""
    r3 = np.random.default_rng(seed + 3)
    return r3.integers(0, p.ncells, size=count)

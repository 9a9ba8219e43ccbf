"""Seeded synthetic workloads for the multilevel BLUP solve.

This module only draws random numbers and composes observation data from
them.  It holds none of the method's arithmetic: no covariance function,
no tree, no basis, no solver.  Both the oracle-side tests and the GPU path
(tests, smoke, bench) draw their inputs from here, so the two sides see
bit-identical arrays.

Five workloads (k = 1..5) are defined.  The paper's own point sets were
random and are not available; these stand in for them with the shapes,
dimensions and Matérn parameters of the paper's experiments (random
hypercube / clustered / manifold point clouds, polynomial trend plus a
smooth random field, no nugget in the model):

  1. n=1,000 uniform in [0,1]^2, nu=1/2, rho=0.1, linear trend (p=3),
     leaf 32, 200 uniform targets.  The correlated part of Z is a draw
     G xi with G the Cholesky factor of the covariance matrix; G needs
     the covariance function, so this module only supplies xi ~ N(0, I)
     and beta, and the caller composes Z.
  2. n=65,536 uniform in [0,1]^3, nu=3/2, rho=0.2, quadratic trend
     (p=10), Z = trend + 256 random cosine features + N(0, 1e-4) noise,
     leaf 64, 4,096 uniform targets.
  3. n=524,288 in d=10 from 8 Gaussian clusters (centres U[0,1]^10,
     std 0.05), nu=1/2, rho=0.5, linear trend (p=11), 16,384 targets
     from the same mixture.
  4. n=131,072 uniform in [0,1]^5, nu=5/2, rho=0.3, linear trend (p=6),
     4,096 uniform targets; the first 4,096 points form the subsample.
  5. n=1,048,576 in d=20, half uniform in [0,1]^20, half on a random
     3-dimensional affine manifold plus N(0, 0.01 I) noise, nu=1/2,
     rho=1.0, linear trend (p=21), 100,000 targets from the mixture.

Cosine field: f(x) = sum_k sqrt(2/K) cos(omega_k . x + b_k), K = 256,
omega_k ~ N(0, 25 I), b_k ~ U[0, 2 pi).  "N(0, v)" means variance v.
The trend uses monomials of total degree <= w with coefficients N(0,1);
the monomial order used here is this module's own (it only generates
data) and need not match any solver's design-matrix column order.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 170100285

# name, n, d, nu, rho, degree w, leaf size, targets
_SPECS = {
    1: dict(name="cfg1_n1000_d2_nu0.5", n=1000, d=2, nu=0.5, rho=0.1, w=1, leaf=32, n_targets=200),
    2: dict(name="cfg2_n65536_d3_nu1.5", n=65536, d=3, nu=1.5, rho=0.2, w=2, leaf=64, n_targets=4096),
    3: dict(name="cfg3_n524288_d10_nu0.5", n=524288, d=10, nu=0.5, rho=0.5, w=1, leaf=64, n_targets=16384),
    4: dict(name="cfg4_n131072_d5_nu2.5", n=131072, d=5, nu=2.5, rho=0.3, w=1, leaf=64, n_targets=4096),
    5: dict(name="cfg5_n1048576_d20_nu0.5", n=1048576, d=20, nu=0.5, rho=1.0, w=1, leaf=64, n_targets=100000),
}


@dataclass
class Workload:
    k: int
    name: str
    n: int
    d: int
    nu: float
    rho: float
    sigma2: float
    degree_w: int
    leaf_max: int
    points: np.ndarray            # (n, d) float64
    targets: np.ndarray           # (m, d) float64
    z: np.ndarray | None          # (n,) float64; None for workload 1 (see module doc)
    extra: dict = field(default_factory=dict)


def spec(k: int) -> dict:
    return dict(_SPECS[k])


def _streams(k: int, count: int = 6):
    ss = np.random.SeedSequence(BASE_SEED + k)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(count)]


def _exponents(d: int, w: int):
    """All exponent tuples of total degree <= w (data-generation order)."""
    return [a for a in itertools.product(range(w + 1), repeat=d) if sum(a) <= w]


def _trend(x: np.ndarray, w: int, coef: np.ndarray) -> np.ndarray:
    out = np.zeros(x.shape[0])
    for c, a in zip(coef, _exponents(x.shape[1], w)):
        term = np.full(x.shape[0], c)
        for j, e in enumerate(a):
            if e:
                term = term * x[:, j] ** e
        out += term
    return out


def _cosine_field(x: np.ndarray, omega: np.ndarray, phase: np.ndarray) -> np.ndarray:
    K = omega.shape[0]
    amp = np.sqrt(2.0 / K)
    out = np.zeros(x.shape[0])
    step = 1 << 16
    for s in range(0, x.shape[0], step):
        arg = x[s:s + step] @ omega.T + phase[None, :]
        out[s:s + step] = amp * np.cos(arg).sum(axis=1)
    return out


def _points(k: int, n: int, d: int, g: np.random.Generator, gc: np.random.Generator) -> np.ndarray:
    if k in (1, 2, 4):
        return g.random((n, d))
    if k == 3:
        centres = gc.random((8, d))
        lab = np.arange(n) % 8
        return centres[lab] + 0.05 * g.standard_normal((n, d))
    if k == 5:
        half = n // 2
        uni = g.random((half, d))
        c = gc.random(d)
        A, _ = np.linalg.qr(gc.standard_normal((d, 3)))
        s = g.random((n - half, 3))
        man = c[None, :] + s @ A.T + np.sqrt(0.01) * g.standard_normal((n - half, d))
        return np.concatenate([uni, man], axis=0)
    raise ValueError(k)


def make_config(k: int, n: int | None = None, n_targets: int | None = None,
                with_z: bool = True) -> Workload:
    """Draw workload k.  `n` / `n_targets` shrink it (same recipe, fewer
    points) for tests that need oracle-sized problems."""
    sp = spec(k)
    n = sp["n"] if n is None else int(n)
    m = sp["n_targets"] if n_targets is None else int(n_targets)
    d, w = sp["d"], sp["w"]
    g_pts, g_trend, g_field, g_noise, g_tgt, g_geom = _streams(k)
    pts = _points(k, n, d, g_pts, g_geom)
    # targets: same distribution as the points (same geometry stream state
    # reproduced by re-seeding the geometry generator)
    g_geom2 = _streams(k)[5]
    tgt = _points(k, m, d, g_tgt, g_geom2)
    p_gen = len(_exponents(d, w))
    beta = g_trend.standard_normal(p_gen)
    extra = {"beta_gen": beta}
    z = None
    if k == 1:
        extra["xi"] = g_field.standard_normal(n)
    elif with_z:
        K = 256
        omega = 5.0 * g_field.standard_normal((K, d))
        phase = g_field.uniform(0.0, 2.0 * np.pi, K)
        noise = np.sqrt(1e-4) * g_noise.standard_normal(n)
        z = _trend(pts, w, beta) + _cosine_field(pts, omega, phase) + noise
    return Workload(k=k, name=sp["name"], n=n, d=d, nu=sp["nu"], rho=sp["rho"], sigma2=1.0,
                    degree_w=w, leaf_max=sp["leaf"], points=np.ascontiguousarray(pts),
                    targets=np.ascontiguousarray(tgt), z=z, extra=extra)


def uniform_cloud(n: int, d: int, seed: int) -> np.ndarray:
    """Plain U[0,1]^d points for structural tests."""
    return np.random.Generator(np.random.PCG64(seed)).random((n, d))


def standard_normal(n: int, seed: int) -> np.ndarray:
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n)


# The cases of the accuracy experiment (Sec. 8, "Prediction numerical
# accuracy under ill-conditioning"): (alpha, theta) of each row of its table.
ACCURACY_CASES = [(1.0, 10.0), (0.5, 10.0), (2.0, 10.0), (2.0, 3.0), (0.5, 3.0)]


def unit_disk(n: int, g: np.random.Generator) -> np.ndarray:
    """n points uniform on the unit disk (radius sqrt(U), angle 2 pi U)."""
    r = np.sqrt(g.random(n))
    a = 2.0 * np.pi * g.random(n)
    return np.stack([r * np.cos(a), r * np.sin(a)], axis=1)


def accuracy_experiment(alpha: float, n: int = 200, n_targets: int = 200):
    """Inputs of the accuracy experiment: n observation sites and n_targets
    targets uniform on the unit disk, Z_i = 1 + sin(alpha x_i1) sin(alpha x_i2).
    The sites and targets do not depend on alpha."""
    g = np.random.default_rng(np.random.SeedSequence(BASE_SEED + 100))
    pts = unit_disk(n, g)
    tgt = unit_disk(n_targets, g)
    z = 1.0 + np.sin(alpha * pts[:, 0]) * np.sin(alpha * pts[:, 1])
    return pts, tgt, z

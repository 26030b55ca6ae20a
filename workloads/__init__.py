"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module holds only sample generators and workload parameters. It contains
none of the method's arithmetic (no distances, kernels, bandwidths or
normalisations), so both sides of every parity test can read the same arrays
without sharing any computation.

Every generator draws from ``numpy.random.default_rng(seed)`` (PCG64) in a fixed
order and returns a C-contiguous float32 array of shape (n, m).

Manifold samples follow the paper's setting (samples x^(i) drawn from a density
psi on a d-dimensional manifold embedded in R^m, Section 2): the uniform unit
2-sphere is the spherical-manifold example of Section 5; the torus, the
nonlinear 5-manifold, the lifted 3-sphere and the Gaussian mixture are the
synthetic stand-ins at the sizes of the measured workloads. No public data set
is involved anywhere.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "make", "sphere2", "torus", "nonlinear5",
    "sphere3_lifted", "gaussian_mixture", "chain_lattice", "cubic_lattice",
    "regular_polygon", "gaussian_iid",
]


# --------------------------------------------------------------------------
# Generators (each a fixed draw order from one PCG64 stream)
# --------------------------------------------------------------------------
def sphere2(n: int, seed: int = 0) -> np.ndarray:
    """Uniform samples on the unit 2-sphere in R^3: normalised N(0, I_3) draws
    in float64, then rounded to float32 (spherical manifold, Section 5)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    x = g / np.linalg.norm(g, axis=1, keepdims=True)
    return np.ascontiguousarray(x, dtype=np.float32)


def torus(n: int, seed: int = 0, R: float = 2.0, r: float = 1.0,
          kappa: float = 1.0) -> np.ndarray:
    """2-torus in R^3 with tube radius r and centre radius R. The tube angle
    theta ~ vonMises(0, kappa), the azimuth phi ~ U(0, 2 pi)."""
    rng = np.random.default_rng(seed)
    theta = rng.vonmises(0.0, kappa, size=n)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n)
    rad = R + r * np.cos(theta)
    x = np.stack([rad * np.cos(phi), rad * np.sin(phi), r * np.sin(theta)], axis=1)
    return np.ascontiguousarray(x, dtype=np.float32)


def nonlinear5(n: int, seed: int = 0, noise: float = 1e-3,
               chunk: int = 1 << 18) -> np.ndarray:
    """Intrinsic dimension 5 embedded in R^64 as [Q z, sin(W z)] + noise, with
    Q the orthonormal factor of a 32x5 Gaussian, W = 0.5 * N(0,1)^{32x5},
    z ~ N(0, I_5) and i.i.d. N(0, noise^2) ambient noise."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((32, 5)))
    W = 0.5 * rng.standard_normal((32, 5))
    out = np.empty((n, 64), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        z = rng.standard_normal((e - s, 5))
        blk = np.concatenate([z @ Q.T, np.sin(z @ W.T)], axis=1)
        blk += noise * rng.standard_normal((e - s, 64))
        out[s:e] = blk
    return out


def sphere3_lifted(n: int, seed: int = 0, m: int = 128,
                   chunk: int = 1 << 18) -> np.ndarray:
    """Uniform samples on S^3 lifted to R^m by a seeded orthonormal m x 4 map."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, 4)))
    out = np.empty((n, m), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        g = rng.standard_normal((e - s, 4))
        g /= np.linalg.norm(g, axis=1, keepdims=True)
        out[s:e] = g @ U.T
    return out


def gaussian_mixture(n: int, seed: int = 0, m: int = 16,
                     chunk: int = 1 << 18) -> np.ndarray:
    """3-component Gaussian mixture (weights 0.5/0.3/0.2, unit covariances) on a
    4-dimensional linear subspace of R^m. Means are (3/sqrt 2) e_a, so every
    pair of means is 3 apart."""
    rng = np.random.default_rng(seed)
    V, _ = np.linalg.qr(rng.standard_normal((m, 4)))
    mu = np.zeros((3, 4))
    for a in range(3):
        mu[a, a] = 3.0 / math.sqrt(2.0)
    out = np.empty((n, m), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        a = rng.choice(3, size=e - s, p=[0.5, 0.3, 0.2])
        z = mu[a] + rng.standard_normal((e - s, 4))
        out[s:e] = z @ V.T
    return out


def gaussian_iid(n: int, m: int, seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """Plain N(0, scale^2 I_m) samples (generic ragged-size test input)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(scale * rng.standard_normal((n, m)), dtype=np.float32)


def chain_lattice(n: int, m: int = 3) -> np.ndarray:
    """Points (i, 0, ..., 0), i = 0..n-1: integer coordinates, so every squared
    distance is an exact integer in float32 and float64 (tie tests)."""
    x = np.zeros((n, m), dtype=np.float32)
    x[:, 0] = np.arange(n, dtype=np.float32)
    return x


def cubic_lattice(side: int) -> np.ndarray:
    """The side^3 integer grid Z^3 in lexicographic (x, y, z) order."""
    g = np.arange(side, dtype=np.float32)
    xx, yy, zz = np.meshgrid(g, g, g, indexing="ij")
    return np.ascontiguousarray(np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1))


def regular_polygon(n: int, phase: float = 0.0) -> np.ndarray:
    """Vertices of the regular n-gon on the unit circle, as (cos, sin, 0)."""
    t = phase + 2.0 * np.pi * np.arange(n) / n
    x = np.stack([np.cos(t), np.sin(t), np.zeros(n)], axis=1)
    return np.ascontiguousarray(x, dtype=np.float32)


# --------------------------------------------------------------------------
# Workload table: the five measured configurations
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    m: int
    d: int              # intrinsic dimension (given, not estimated)
    k: int              # neighbours per row, self included
    k0: int = 8         # neighbours in the ad-hoc bandwidth
    G: int = 64         # epsilon grid size
    e_min: float = 1e-3
    e_max: float = 1e1
    beta: float = -0.5
    margin: int = 32
    mode: str = "f32"   # k-NN mode for the timed path
    gen: str = ""
    gen_kw: dict = field(default_factory=dict)

    @property
    def alpha(self) -> float:
        return -self.d / 4.0

    def as_dict(self) -> dict:
        d = asdict(self)
        d["alpha"] = self.alpha
        return d


WORKLOADS = {
    "sphere2_n2000": Workload("sphere2_n2000", 2000, 3, 2, 32, gen="sphere2"),
    "torus_n100k": Workload("torus_n100k", 100_000, 3, 2, 64, gen="torus"),
    "nonlinear5_n1m": Workload("nonlinear5_n1m", 1_000_000, 64, 5, 64,
                               mode="bf16", gen="nonlinear5"),
    "sphere3_n4m": Workload("sphere3_n4m", 4_000_000, 128, 3, 128,
                            mode="learned", gen="sphere3_lifted"),
    "gmm_n8m": Workload("gmm_n8m", 8_000_000, 16, 4, 64, mode="bf16",
                        gen="gaussian_mixture"),
}

_GEN = {
    "sphere2": lambda n, m, seed: sphere2(n, seed),
    "torus": lambda n, m, seed: torus(n, seed),
    "nonlinear5": lambda n, m, seed: nonlinear5(n, seed),
    "sphere3_lifted": lambda n, m, seed: sphere3_lifted(n, seed, m=m),
    "gaussian_mixture": lambda n, m, seed: gaussian_mixture(n, seed, m=m),
}


def make(name: str, seed: int = 0, n: int | None = None) -> np.ndarray:
    """Samples of workload `name` (optionally with a different n, same recipe)."""
    w = WORKLOADS[name]
    return _GEN[w.gen](w.n if n is None else n, w.m, seed)

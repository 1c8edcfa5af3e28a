"""Seeded query-point sets (NumPy).

Uniform points in a box stand in for the paper's uniform sampling in a scaled
bounding box; near-surface points (area-weighted surface samples plus an
isotropic Gaussian offset) stand in for its near/far study.
"""
from __future__ import annotations

import numpy as np


def aabb(V: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    V = np.asarray(V, dtype=np.float64)
    return V.min(axis=0), V.max(axis=0)


def scaled_box(lo: np.ndarray, hi: np.ndarray, scale: float) -> tuple[np.ndarray, np.ndarray]:
    c = 0.5 * (lo + hi)
    h = 0.5 * (hi - lo) * scale
    return c - h, c + h


def uniform_in_box(n: int, lo, hi, rng: np.random.Generator) -> np.ndarray:
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return (lo + rng.random((n, 3)) * (hi - lo)).astype(np.float32)


def surface_samples(V: np.ndarray, F: np.ndarray, n: int, rng: np.random.Generator,
                    return_faces: bool = False):
    """Area-weighted uniform surface samples (float64).

    Face chosen with probability proportional to area (CDF search), point
    a*(1-sqrt r1) + b*sqrt r1 (1-r2) + c*sqrt r1 r2.
    """
    V = np.asarray(V, dtype=np.float64)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    cdf = np.cumsum(area)
    cdf /= cdf[-1]
    f = np.searchsorted(cdf, rng.random(n), side="right")
    f = np.minimum(f, F.shape[0] - 1)
    r1 = np.sqrt(rng.random(n))
    r2 = rng.random(n)
    w0 = 1.0 - r1
    w1 = r1 * (1.0 - r2)
    w2 = r1 * r2
    P = w0[:, None] * a[f] + w1[:, None] * b[f] + w2[:, None] * c[f]
    if return_faces:
        return P, f
    return P


def near_surface(V: np.ndarray, F: np.ndarray, n: int, sigma: float,
                 rng: np.random.Generator) -> np.ndarray:
    P = surface_samples(V, F, n, rng)
    return (P + rng.normal(0.0, sigma, size=P.shape)).astype(np.float32)


def near_segments(V: np.ndarray, S: np.ndarray, n: int, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Length-weighted uniform samples on segments plus isotropic Gaussian offsets."""
    V = np.asarray(V, dtype=np.float64)
    a, b = V[S[:, 0]], V[S[:, 1]]
    cdf = np.cumsum(np.linalg.norm(b - a, axis=1))
    cdf /= cdf[-1]
    k = np.searchsorted(cdf, rng.random(n), side="right")
    k = np.minimum(k, len(S) - 1)
    t = rng.random(n)[:, None]
    P = a[k] * (1.0 - t) + b[k] * t
    return (P + rng.normal(0.0, sigma, size=P.shape)).astype(np.float32)


def mixed(V: np.ndarray, F: np.ndarray, n: int, box_scale: float, sigma_rel: float,
          rng: np.random.Generator, return_near: bool = False):
    """Half uniform in the scaled AABB, half near-surface, shuffled; with
    return_near, also the boolean mask of the near-surface rows."""
    lo, hi = aabb(V)
    blo, bhi = scaled_box(lo, hi, box_scale)
    diag = float(np.linalg.norm(hi - lo))
    nu = n // 2
    Q = np.concatenate([uniform_in_box(nu, blo, bhi, rng),
                        near_surface(V, F, n - nu, sigma_rel * diag, rng)], axis=0)
    p = rng.permutation(n)
    if return_near:
        return Q[p], p >= nu
    return Q[p]

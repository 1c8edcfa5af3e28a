"""Seeded lattice value noise and fractal sums of it (NumPy, vectorised).

The noise is a plain procedural texture used to displace synthetic meshes; it
holds none of the point-to-mesh arithmetic.  Lattice values come from the
splitmix64 finaliser (Steele, Lea, Flood 2014) applied to a seeded mix of the
integer lattice coordinates, mapped to U[-1, 1]; values between lattice points
are interpolated with the quintic fade 6t^5 - 15t^4 + 10t^3 (Perlin 2002).
"""
from __future__ import annotations

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 output function applied elementwise to a uint64 array."""
    with np.errstate(over="ignore"):
        z = x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def _lattice_value(seed: int, *coords: np.ndarray) -> np.ndarray:
    """U[-1,1] value attached to integer lattice points (any dimension)."""
    with np.errstate(over="ignore"):
        h = np.full(coords[0].shape, np.uint64(seed) * np.uint64(0x632BE59BD9B4E019), dtype=np.uint64)
        for c in coords:
            h = splitmix64(h ^ c.astype(np.int64).view(np.uint64))
    u = (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def _fade(t: np.ndarray) -> np.ndarray:
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def value_noise3(p: np.ndarray, seed: int) -> np.ndarray:
    """Trilinear value noise at points p [N,3] (float64) -> [N] in [-1, 1]."""
    p = np.asarray(p, dtype=np.float64)
    i0 = np.floor(p).astype(np.int64)
    t = _fade(p - i0)
    out = np.zeros(p.shape[0], dtype=np.float64)
    for dx in (0, 1):
        wx = t[:, 0] if dx else 1.0 - t[:, 0]
        for dy in (0, 1):
            wy = t[:, 1] if dy else 1.0 - t[:, 1]
            for dz in (0, 1):
                wz = t[:, 2] if dz else 1.0 - t[:, 2]
                v = _lattice_value(seed, i0[:, 0] + dx, i0[:, 1] + dy, i0[:, 2] + dz)
                out += wx * wy * wz * v
    return out


def value_noise2(p: np.ndarray, seed: int) -> np.ndarray:
    """Bilinear value noise at points p [N,2] (float64) -> [N] in [-1, 1]."""
    p = np.asarray(p, dtype=np.float64)
    i0 = np.floor(p).astype(np.int64)
    t = _fade(p - i0)
    out = np.zeros(p.shape[0], dtype=np.float64)
    for dx in (0, 1):
        wx = t[:, 0] if dx else 1.0 - t[:, 0]
        for dy in (0, 1):
            wy = t[:, 1] if dy else 1.0 - t[:, 1]
            out += wx * wy * _lattice_value(seed, i0[:, 0] + dx, i0[:, 1] + dy)
    return out


def fbm3(p: np.ndarray, seed: int, octaves: int = 4, base_freq: float = 4.0,
         gain: float = 0.5) -> np.ndarray:
    """Normalised fractal sum: sum_o gain^o vn(base*2^o p + off_o) / sum_o gain^o."""
    rng = np.random.default_rng(seed)
    offs = rng.uniform(0.0, 1000.0, size=(octaves, 3))
    acc = np.zeros(p.shape[0], dtype=np.float64)
    norm = 0.0
    for o in range(octaves):
        a = gain ** o
        acc += a * value_noise3(base_freq * (2.0 ** o) * p + offs[o], seed * 131 + o)
        norm += a
    return acc / norm


def fbm2(p: np.ndarray, seed: int, octaves: int = 6, base_freq: float = 8.0,
         gain: float = 0.5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    offs = rng.uniform(0.0, 1000.0, size=(octaves, 2))
    acc = np.zeros(p.shape[0], dtype=np.float64)
    norm = 0.0
    for o in range(octaves):
        a = gain ** o
        acc += a * value_noise2(base_freq * (2.0 ** o) * p + offs[o], seed * 131 + o)
        norm += a
    return acc / norm

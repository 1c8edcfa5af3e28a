"""TEST ORACLE (query ordering) -- test infrastructure only.

The paper answers queries independently (Sec. 5); ordering a batch so that
nearby queries run together is an addition of this implementation and does
not change any answer.  Its definition:

  cell_k = clamp(floor((q_k - lo_k) * s_k), 0, 1023),  s_k = 1024 / (hi_k - lo_k)
  key    = bit-interleave of (cell_x, cell_y, cell_z), x taking the most
           significant bit of each triple (30-bit Morton code)
  order  = stable sort of the keys (equal keys keep input order)

The quantisation decides an integer from floating point, so it is taken in
float32 exactly as the device computes it: lo_k and s_k rounded to float32
once, then one float32 subtract and one float32 multiply.  A non-finite
product maps to cell 0.
"""
from __future__ import annotations

import numpy as np


def quantise(Q, lo, hi) -> np.ndarray:
    Q = np.asarray(Q, dtype=np.float32).reshape(-1, 3)
    lo32 = np.asarray(lo, dtype=np.float64).astype(np.float32)
    s32 = (1024.0 / (np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64))).astype(np.float32)
    with np.errstate(invalid="ignore", over="ignore"):
        s = (Q - lo32) * s32                          # float32 arithmetic
        cell = np.where(s >= np.float32(0), s, np.float32(0))
        cell = np.where(cell >= np.float32(1023), np.float32(1023), cell)
    return cell.astype(np.int64)                      # truncation == floor for s >= 0


def morton_keys(Q, lo, hi) -> np.ndarray:
    c = quantise(Q, lo, hi)
    key = np.zeros(c.shape[0], dtype=np.uint32)
    for b in range(10):
        key |= (((c[:, 0] >> b) & 1) << (3 * b + 2)).astype(np.uint32)
        key |= (((c[:, 1] >> b) & 1) << (3 * b + 1)).astype(np.uint32)
        key |= (((c[:, 2] >> b) & 1) << (3 * b)).astype(np.uint32)
    return key


def order(Q, lo, hi) -> tuple[np.ndarray, np.ndarray]:
    """(sorted keys, permutation) with perm[j] = input index of the j-th query."""
    k = morton_keys(Q, lo, hi)
    perm = np.argsort(k, kind="stable").astype(np.int32)
    return k[perm], perm

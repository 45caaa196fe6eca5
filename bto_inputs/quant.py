"""Storage precision of velocity grids: round-to-nearest-even from FP64.

``quantize`` returns the array the GPU library is handed (float32, float16, or
the raw uint16 bits of bfloat16); ``promote`` returns the exact FP64 values of
such an array.  Both are input preparation only.
"""

from __future__ import annotations

import numpy as np

STORAGE_DTYPES = ("f32", "f16", "bf16")


def _bf16_rne(x: np.ndarray) -> np.ndarray:
    """FP64 -> bfloat16 (8 significant bits) with round-half-to-even, as bits."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                     # x = m * 2**e, 0.5 <= |m| < 1
    q = np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)
    # below the smallest normal the quantum stops shrinking (2**-133)
    tiny = np.abs(x) < 2.0 ** -126
    if np.any(tiny):
        q = np.where(tiny, np.rint(x * 2.0 ** 133) * 2.0 ** -133, q)
    q = np.where(np.isfinite(x), q, x)
    b = q.astype(np.float32).view(np.uint32)
    return (b >> np.uint32(16)).astype(np.uint16)


def quantize(g: np.ndarray, dtype: str) -> np.ndarray:
    """Round an FP64 grid to the storage precision ``dtype`` (RNE)."""
    g = np.asarray(g, dtype=np.float64)
    if dtype == "f64":
        return g
    if dtype == "f32":
        return g.astype(np.float32)
    if dtype == "f16":
        return g.astype(np.float16)
    if dtype == "bf16":
        return _bf16_rne(g)
    raise ValueError(f"unknown storage dtype {dtype!r}")


def promote(a: np.ndarray, dtype: str) -> np.ndarray:
    """Exact FP64 values of a stored grid."""
    if dtype in ("f64", "f32", "f16"):
        return np.asarray(a).astype(np.float64)
    if dtype == "bf16":
        bits = np.asarray(a, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
        return bits.view(np.float32).astype(np.float64)
    raise ValueError(f"unknown storage dtype {dtype!r}")

"""Comparison helpers for GPU-vs-oracle parity tests (max-norm relative errors)."""

import numpy as np


def max_norm_rel(got, ref):
    """max_i |got_i - ref_i|_2 / max_i |ref_i|_2 over rows (vectors) or elements."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if got.ndim == 1:
        den = np.abs(ref).max()
        return float(np.abs(got - ref).max() / den) if den > 0 else float(np.abs(got).max())
    den = np.sqrt((ref * ref).sum(axis=1)).max()
    num = np.sqrt(((got - ref) ** 2).sum(axis=1)).max()
    return float(num / den) if den > 0 else float(num)


def scalar_rel(got, ref):
    return abs(got - ref) / max(abs(ref), 1e-300)


def sort_pairs(p):
    """Unordered pairs (i < j) sorted by (i, j), as an (M, 2) int64 array."""
    p = np.asarray(p, dtype=np.int64).reshape(-1, 2)
    if len(p) == 0:
        return p
    key = np.sort(p[:, 0] * (1 << 32) + p[:, 1])
    return np.stack([key >> 32, key & 0xFFFFFFFF], axis=1)


def unwrapped(pos, img, box):
    return pos + img * np.asarray(box)[None, :]


def print_case(msg):
    print(f"[case] {msg}", flush=True)

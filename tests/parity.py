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


def full_list_keys(counts, neighbours):
    """Every stored entry of a full list as the key row * 2^32 + neighbour, sorted."""
    counts = np.asarray(counts, dtype=np.int64)
    rows = np.repeat(np.arange(len(counts), dtype=np.int64), counts)
    return np.sort(rows * (1 << 32) + np.asarray(neighbours, dtype=np.int64))


def assert_full_list_equals_pairs(counts, neighbours, pairs):
    """A full list (rows of neighbour tags) against an unordered pair set (i < j): no row
    holds an entry twice or lists its own particle, every pair appears in both rows, and
    nothing else appears."""
    keys = full_list_keys(counts, neighbours)
    assert int(np.asarray(counts).sum()) == len(keys)
    assert not np.any((keys >> 32) == (keys & 0xFFFFFFFF)), "a row lists its own particle"
    assert np.all(np.diff(keys) > 0), "a row holds the same neighbour twice"
    p = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    ref = np.sort(np.concatenate([p[:, 0] * (1 << 32) + p[:, 1], p[:, 1] * (1 << 32) + p[:, 0]]))
    assert keys.shape == ref.shape, (keys.shape, ref.shape)
    assert np.array_equal(keys, ref)

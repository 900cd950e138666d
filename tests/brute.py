"""Independent O(N^2) numpy brute force, used to pin the CPU oracle and, through it, the GPU
path. Written separately from the oracle (no shared code): every pair (i < j) is enumerated
explicitly, the minimum image is taken per axis, and the squared distance is formed
elementwise as (dx*dx + dy*dy) + dz*dz, which numpy evaluates without fused multiply-add.
"""

from __future__ import annotations

import numpy as np


def _pair_tables(ntypes, pairs, skin):
    eps = np.zeros((ntypes, ntypes))
    sig = np.ones((ntypes, ntypes))
    rc = np.zeros((ntypes, ntypes))
    for (a, b, e, s, r) in pairs:
        eps[a, b] = eps[b, a] = e
        sig[a, b] = sig[b, a] = s
        rc[a, b] = rc[b, a] = r
    rl = np.where(rc > 0.0, rc + skin, 0.0)
    return eps, sig, rc, rl * rl


def _min_image(d, L):
    h = 0.5 * L
    return np.where(d >= h, d - L, np.where(d < -h, d + L, d))


def brute_pairs(box, pos, types, ntypes, pairs, skin, chunk=512):
    """All (i < j) with r2 < (r_cut_ab + skin)^2, as a sorted (M, 2) int64 array."""
    pos = np.asarray(pos, dtype=np.float64)
    types = np.asarray(types)
    n = pos.shape[0]
    _, _, _, rl2 = _pair_tables(ntypes, pairs, skin)
    out = []
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        d = [_min_image(pos[None, :, a] - pos[i0:i1, None, a], box[a]) for a in range(3)]
        r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        thr = rl2[types[i0:i1, None], types[None, :]]
        ii, jj = np.nonzero(r2 < thr)
        ii = ii + i0
        keep = jj > ii
        out.append(np.stack([ii[keep], jj[keep]], axis=1))
    if not out:
        return np.zeros((0, 2), dtype=np.int64)
    p = np.concatenate(out).astype(np.int64)
    order = np.lexsort((p[:, 1], p[:, 0]))
    return p[order]


def brute_fuw(box, pos, types, ntypes, pairs, chunk=512):
    """Forces (N,3), per-particle energy (N,), per-particle virial (N,6), total U and W[6]
    of the truncated-and-shifted LJ potential over every pair within r_cut."""
    pos = np.asarray(pos, dtype=np.float64)
    types = np.asarray(types)
    n = pos.shape[0]
    eps, sig, rc, _ = _pair_tables(ntypes, pairs, 0.0)
    F = np.zeros((n, 3))
    u_i = np.zeros(n)
    w_i = np.zeros((n, 6))
    comp = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        # r = x_i - x_j for the rows i in the chunk against all j
        r = [_min_image(pos[i0:i1, None, a] - pos[None, :, a], box[a]) for a in range(3)]
        r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
        ti = types[i0:i1, None]
        tj = types[None, :]
        e = eps[ti, tj]
        s = sig[ti, tj]
        c = rc[ti, tj]
        mask = r2 < c * c
        idx = np.arange(i0, i1)
        mask[idx - i0, idx] = False
        r2m = np.where(mask, r2, 1.0)
        sr6 = (s * s / r2m) ** 3
        ff = np.where(mask, 24.0 * e * (2.0 * sr6 * sr6 - sr6) / r2m, 0.0)
        sc6 = (s * s / np.where(mask, c * c, 1.0)) ** 3
        u = np.where(mask, 4.0 * e * (sr6 * sr6 - sr6) - 4.0 * e * (sc6 * sc6 - sc6), 0.0)
        for a in range(3):
            F[i0:i1, a] = np.sum(ff * r[a], axis=1)
        u_i[i0:i1] = 0.5 * np.sum(u, axis=1)
        for k, (a, b) in enumerate(comp):
            w_i[i0:i1, k] = 0.5 * np.sum(r[a] * ff * r[b], axis=1)
    return F, u_i, w_i, float(np.sum(u_i)), np.sum(w_i, axis=0)


def lj_pair(r, eps=1.0, sig=1.0, rc=2.5):
    """Closed forms of one pair at distance r: (shifted energy, force magnitude along r)."""
    sr6 = (sig / r) ** 6
    sc6 = (sig / rc) ** 6
    u = 4.0 * eps * (sr6 * sr6 - sr6) - 4.0 * eps * (sc6 * sc6 - sc6)
    f = 24.0 * eps * (2.0 * sr6 * sr6 - sr6) / r
    return u, f


def _form(style, p, r):
    """Pair energy and -(du/dr) of the other forms at distance r (arrays), written from the
    textbook expressions independently of the oracle."""
    if style == "mie":
        eps, sig, n, m = p
        c = (n / (n - m)) * (n / m) ** (m / (n - m))
        x = sig / r
        return c * eps * (x ** n - x ** m), c * eps * (n * x ** n - m * x ** m) / r
    if style == "gauss":
        eps, sig = p[:2]
        g = eps * np.exp(-0.5 * (r / sig) ** 2)
        return g, g * r / sig ** 2
    if style == "yukawa":
        eps, kappa = p[:2]
        e = eps * np.exp(-kappa * r)
        return e / r, e * (1.0 + kappa * r) / r ** 2
    eps, sig = p[:2]
    x6 = (sig / r) ** 6
    return 4 * eps * (x6 * x6 - x6), 24 * eps * (2 * x6 * x6 - x6) / r


def brute_fuw_style(box, pos, style, params, rc, shift_force=False):
    """Forces, total energy and virial of one pair form (single type), truncated at rc and
    energy-shifted there (with shift_force, force-shifted as well: the pair force less its
    value at rc, and the energy less the matching linear term), over every pair (i < j)
    within rc."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    F = np.zeros((n, 3))
    U = 0.0
    W = np.zeros(6)
    u_c, f_c = _form(style, params, np.array([rc]))
    for i in range(n - 1):
        d = np.stack([_min_image(pos[i + 1:, a] - pos[i, a], box[a]) for a in range(3)], 1)
        r = np.sqrt((d * d).sum(1))
        inside = r < rc
        d, r = d[inside], r[inside]
        j = np.nonzero(inside)[0] + i + 1
        u, mdu = _form(style, params, r)
        u = u - u_c[0]
        if shift_force:
            # the force (-du/dr) less its value at rc; the energy whose derivative that is
            mdu = mdu - f_c[0]
            u = u + (r - rc) * f_c[0]
        U += float(u.sum())
        fij = (mdu / r)[:, None] * (-d)  # on i, along x_i - x_j
        F[i] += fij.sum(0)
        np.add.at(F, j, -fij)
        rij = -d
        W += np.stack([rij[:, 0] * fij[:, 0], rij[:, 0] * fij[:, 1], rij[:, 0] * fij[:, 2],
                       rij[:, 1] * fij[:, 1], rij[:, 1] * fij[:, 2], rij[:, 2] * fij[:, 2]],
                      1).sum(0)
    return F, U, W

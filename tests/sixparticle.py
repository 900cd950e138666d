"""The six-particle fixture and an independent per-pair "calculator" for it.

The calculator uses the math module only, takes the minimum image as d - L * round(d / L)
(a different formula from the oracle's and the GPU's branch form; both agree whenever
|d| != L/2), and sums every one of the 15 pairs explicitly."""

import math
import os

import numpy as np

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "six_particle.txt")


def load_fixture(path=FIXTURE):
    box, pos, params = None, [], []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tag, *vals = line.split()
            vals = [float(v) for v in vals]
            if tag == "box":
                box = np.array(vals)
            elif tag == "pos":
                pos.append(vals)
            elif tag == "param":
                params.append(tuple(vals))
    return box, np.array(pos), params


def calculator(box, pos, eps, sig, rc):
    n = len(pos)
    F = [[0.0, 0.0, 0.0] for _ in range(n)]
    u_i = [0.0] * n
    w_i = [[0.0] * 6 for _ in range(n)]
    U = 0.0
    W = [0.0] * 6
    shift = 4.0 * eps * ((sig / rc) ** 12 - (sig / rc) ** 6)
    comp = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for i in range(n):
        for j in range(i + 1, n):
            r = []
            for a in range(3):
                d = pos[i][a] - pos[j][a]
                d -= box[a] * round(d / box[a])
                r.append(d)
            rr = math.sqrt(r[0] ** 2 + r[1] ** 2 + r[2] ** 2)
            if rr >= rc:
                continue
            u = 4.0 * eps * ((sig / rr) ** 12 - (sig / rr) ** 6) - shift
            fmag = 24.0 * eps * (2.0 * (sig / rr) ** 12 - (sig / rr) ** 6) / rr
            for a in range(3):
                F[i][a] += fmag * r[a] / rr
                F[j][a] -= fmag * r[a] / rr
            U += u
            u_i[i] += 0.5 * u
            u_i[j] += 0.5 * u
            for k, (a, b) in enumerate(comp):
                w = r[a] * fmag * r[b] / rr
                W[k] += w
                w_i[i][k] += 0.5 * w
                w_i[j][k] += 0.5 * w
    return np.array(F), U, np.array(W), np.array(u_i), np.array(w_i)

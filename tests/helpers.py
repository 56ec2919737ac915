"""Shared test-side helpers: relaxation vectors, golden-file readers."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# Relaxation rates used in Sec. 4 of the paper (s_c, s_e, s_q, s_t); the
# 18-velocity model reuses them and takes s_pi = 1.4 (the paper gives none).
S_C, S_E, S_Q, S_T, S_PI = 1.0, 1.19, 1.2, 0.98, 1.4


def s_nu_of(nu):
    """Viscous rate from nu = (1/s_nu - 1/2)/3 (Eq. (vis), c = 1)."""
    return 1.0 / (3.0 * nu + 0.5)


def svec(q, s_nu, s_q=S_Q, s_t=S_T, s_e=S_E, s_pi=S_PI, s_c=S_C):
    if q == 14:
        return np.array([s_c, s_e, s_c, s_q, s_c, s_q, s_c, s_q,
                         s_nu, s_nu, s_nu, s_nu, s_nu, s_t])
    return np.array([s_c, s_e, s_c, s_q, s_c, s_q, s_c, s_q,
                     s_nu, s_pi, s_nu, s_pi, s_nu, s_nu, s_nu, s_t, s_t, s_t])


def read_matrix(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return np.array(rows, dtype=np.int64)


def read_records(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(line.split())
    return out


def velocities(q):
    recs = read_records("velocities.txt")
    return np.array([[int(r[2]), int(r[3]), int(r[4])] for r in recs if int(r[0]) == q])


def weights_d3q15_d3q19(q):
    """Weights of the lattice the model is cut from: D3Q15 for q = 14
    (2/9 rest, 1/9 axis, 1/72 corner), D3Q19 for q = 18 (1/3, 1/18, 1/36)."""
    from fractions import Fraction as Fr
    c = velocities(q)
    if q == 14:
        w = [Fr(1, 9) if int(np.sum(v * v)) == 1 else Fr(1, 72) for v in c]
        return Fr(2, 9), w
    w = [Fr(1, 18) if int(np.sum(v * v)) == 1 else Fr(1, 36) for v in c]
    return Fr(1, 3), w

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


# ---- the paper's pressure-driven duct set-ups (Sec. 4.1, 4.2) -------------
# Duct 0 <= x <= l = 2, -a <= y, z <= a = 0.5, nodes on every face (the
# node-based grid of the non-equilibrium extrapolation scheme), velocity
# faces u = 0 on y and z, pressure faces on x.  The paper runs with c != 1
# and scales u by c and p by c^2 into lattice units (Sec. 4).
NEE_FACES = ("pressure", "pressure", "velocity", "velocity", "velocity", "velocity")


def paper_poiseuille(dx, inv_tau, nu_phys=0.03, p_in=1.1, p_out=1.0):
    """Sec. 4.1: lattice set-up for grid spacing dx and 1/tau, with the
    physical viscosity fixed (dt from nu = c^2 (tau - 1/2) dt / 3)."""
    tau = 1.0 / inv_tau
    nu_lat = (tau - 0.5) / 3.0
    dt = nu_lat * dx * dx / nu_phys
    c = dx / dt
    n = int(round(1.0 / dx)) + 1
    return {"nx": 2 * (n - 1) + 1, "ny": n, "nz": n, "c": c, "dt": dt, "s_nu": inv_tau,
            "nu_phys": nu_phys, "g_phys": (p_in - p_out) / 2.0,
            "face_p": {"-x": p_in / c ** 2, "+x": p_out / c ** 2},
            "p_init": 0.5 * (p_in + p_out) / c ** 2}


def paper_pulsatile(dx, tau=0.6178, period=100.0, dp=1e-3, p_out=1.0):
    """Sec. 4.2 convergence study: c = 1 at dx = 1/20 and doubling as dx
    halves (tau, nu fixed), dp/dx = G cos(omega t), G = dp / l.  Table 3 is
    the dx = 1/20 case with tau = 0.9 and dp from 1e-3 to 5e-2."""
    c = (1.0 / dx) / 20.0
    dt = dx / c
    nu_phys = c * c * (tau - 0.5) * dt / 3.0
    steps = int(round(period / dt))
    n = int(round(1.0 / dx)) + 1
    p_in0 = p_out - dp
    return {"nx": 2 * (n - 1) + 1, "ny": n, "nz": n, "c": c, "dt": dt, "s_nu": 1.0 / tau,
            "nu_phys": nu_phys, "steps_per_period": steps, "omega": 2 * np.pi / period,
            "G": dp / 2.0, "face_p": {"-x": p_out / c ** 2, "+x": p_out / c ** 2},
            "face_pA": {"-x": -dp / c ** 2}, "p_init": 0.5 * (p_in0 + p_out) / c ** 2}


def node_positions(n, a=0.5):
    """Node coordinates -a .. a of a node-based grid with n nodes."""
    return -a + (2.0 * a / (n - 1)) * np.arange(n)


def paper_gre(u_lat, c, ua_phys):
    """Eq. (ed) over every grid point: u_lat (3, nz, ny, nx) in lattice
    units (scaled by c), ua_phys (nz, ny) the analytic streamwise velocity."""
    un = np.asarray(u_lat) * c
    nx = un.shape[3]
    num = (np.sum((un[0] - ua_phys[:, :, None]) ** 2) + np.sum(un[1] ** 2)
           + np.sum(un[2] ** 2))
    return float(np.sqrt(num) / np.sqrt(nx * np.sum(ua_phys ** 2)))


def printed_table(table):
    """{row label: [printed values]} of Table 1 / 2 (the four grid spacings)
    or Table 3 (d'Humieres D3Q15, iD3Q14)."""
    out = {}
    for rec in read_records("paper_gre_tables.txt"):
        if rec[0] == table:
            out[rec[1]] = [float(v) for v in rec[2:6]]
    return out


def within_last_digit(value, printed, digits=4):
    """|value - printed| within one unit of the last of `digits` printed
    significant digits."""
    unit = 10.0 ** (np.floor(np.log10(abs(printed))) - (digits - 1))
    return abs(value - printed) <= unit

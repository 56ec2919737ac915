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


# The 26-velocity model's extra moments (energy square eps, the second
# energy flux h) get the D3Q19-type value 1.4 for eps and s_q for h.
S_EPS = 1.4


def svec(q, s_nu, s_q=S_Q, s_t=S_T, s_e=S_E, s_pi=S_PI, s_c=S_C, s_eps=S_EPS):
    if q == 14:
        return np.array([s_c, s_e, s_c, s_q, s_c, s_q, s_c, s_q,
                         s_nu, s_nu, s_nu, s_nu, s_nu, s_t])
    if q == 26:
        return np.array([s_c, s_e, s_eps, s_c, s_q, s_q, s_c, s_q, s_q, s_c, s_q, s_q,
                         s_nu, s_pi, s_nu, s_pi, s_nu, s_nu, s_nu, s_pi, s_pi, s_pi,
                         s_t, s_t, s_t, s_t])
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
    """The paper's velocity sets (Sec. 3 for 14, Appendix B for 18); for the
    26-velocity model, which the paper names but does not list, the 26
    non-rest D3Q27 velocities built from them: the 18 of Appendix B in
    their order, then the 8 corners in the order of Sec. 3."""
    if q == 26:
        return np.concatenate([velocities(18), velocities(14)[6:]])
    recs = read_records("velocities.txt")
    return np.array([[int(r[2]), int(r[3]), int(r[4])] for r in recs if int(r[0]) == q])


def weights_d3q15_d3q19(q):
    """Weights of the lattice the model is cut from: D3Q15 for q = 14
    (2/9 rest, 1/9 axis, 1/72 corner), D3Q19 for q = 18 (1/3, 1/18, 1/36),
    D3Q27 for q = 26 (8/27 rest, 2/27 axis, 1/54 edge, 1/216 corner)."""
    from fractions import Fraction as Fr
    c = velocities(q)
    if q == 14:
        w = [Fr(1, 9) if int(np.sum(v * v)) == 1 else Fr(1, 72) for v in c]
        return Fr(2, 9), w
    if q == 26:
        by_len = {1: Fr(2, 27), 2: Fr(1, 54), 3: Fr(1, 216)}
        return Fr(8, 27), [by_len[int(np.sum(v * v))] for v in c]
    w = [Fr(1, 18) if int(np.sum(v * v)) == 1 else Fr(1, 36) for v in c]
    return Fr(1, 3), w


def monomials26():
    """The monomial rows the 26-velocity transform is built from, by tensor
    order (Sec. 3's construction, Eq. (transformation_Mbar)): 1, |c|^2,
    |c|^4; c_x, |c|^2 c_x, |c|^4 c_x and the same for y, z; 3 c_x^2,
    3 c_x^2 |c|^2, c_y^2 - c_z^2, (c_y^2 - c_z^2) |c|^2, c_x c_y, c_y c_z,
    c_x c_z, the same three times |c|^2; (c_y^2 - c_z^2) c_x,
    (c_z^2 - c_x^2) c_y, (c_x^2 - c_y^2) c_z, c_x c_y c_z."""
    c = velocities(26)
    x, y, z = c[:, 0], c[:, 1], c[:, 2]
    k = x * x + y * y + z * z
    rows = [k ** 0, k, k * k]
    for v in (x, y, z):
        rows += [v, k * v, k * k * v]
    rows += [3 * x * x, 3 * x * x * k, y * y - z * z, (y * y - z * z) * k,
             x * y, y * z, x * z, x * y * k, y * z * k, x * z * k,
             (y * y - z * z) * x, (z * z - x * x) * y, (x * x - y * y) * z, x * y * z]
    return np.array(rows, dtype=np.int64)


def gram_schmidt_rows(M):
    """Orthogonalise the integer rows of M in order (exact rationals) and
    scale each to the smallest integers (the sign of the orthogonalised row
    kept), as Sec. 3 does for T."""
    from fractions import Fraction as Fr
    from math import gcd
    ortho = []
    for r in M:
        v = [Fr(int(a)) for a in r]
        for o in ortho:
            coef = sum(a * b for a, b in zip(v, o)) / sum(b * b for b in o)
            v = [a - coef * b for a, b in zip(v, o)]
        ortho.append(v)
    out = []
    for v in ortho:
        den = 1
        for a in v:
            den = den * a.denominator // gcd(den, a.denominator)
        w = [int(a * den) for a in v]
        g = 0
        for a in w:
            g = gcd(g, abs(a))
        out.append([a // g for a in w])
    return np.array(out, dtype=np.int64)


def T_matrix(q):
    """T of the model: as printed (Eq. (T14), Appendix B) for 14 and 18;
    for 26, Gram-Schmidt of monomials26()."""
    if q == 26:
        return gram_schmidt_rows(monomials26())
    return read_matrix("T%d_printed.txt" % q)


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

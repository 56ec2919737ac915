"""Relaxation vectors and flow set-ups in lattice units (c = dx = dt = 1).

Rates follow Sec. 4 of arXiv 1503.03337: s_c = 1.0, s_e = 1.19, s_q = 1.2,
s_t = 0.98, s_nu = 1/tau with nu = (1/s_nu - 1/2)/3 (Eq. (vis)).  The
18-velocity model (Appendix B) also needs s_pi, which the paper does not
give; 1.4 is used.

Under half-way bounce-back the wall of a lattice flow sits exactly half-way
between nodes only when the odd moments relax at rates tied to s_nu by
(1/s_nu - 1/2)(1/s_odd - 1/2) = 3/16 (Ginzburg's "magic" combination); with
fixed odd rates the wall moves with nu.  `odd_rates` returns that s_odd.
"""
import numpy as np

S_C, S_E, S_Q, S_T, S_PI = 1.0, 1.19, 1.2, 0.98, 1.4
# The 26-velocity model's energy-square moment (which the 14- and
# 18-velocity models do not have) relaxes at the D3Q19-type value 1.4; its
# second energy flux h takes s_q.
S_EPS = 1.4

# u_max of steady flow in a square duct of half-width a under body force g:
# u_max = DUCT_UMAX_COEFF * g a^2 / nu (Sec. 4.1 series at the centre).
DUCT_UMAX_COEFF = 0.2946854131260552


def s_nu(nu):
    return 1.0 / (3.0 * nu + 0.5)


MAGIC_LAMBDA = 3.0 / 16.0


def odd_rates(sn, lam=MAGIC_LAMBDA):
    """s_odd with (1/sn - 1/2)(1/s_odd - 1/2) = lam."""
    return 1.0 / (lam / (1.0 / sn - 0.5) + 0.5)


def s_vec(q, nu=None, sn=None, s_e=S_E, s_q=S_Q, s_t=S_T, s_pi=S_PI, s_c=S_C, s_eps=S_EPS):
    """Relaxation rates in the moment order of Eq. (moment) (q = 14),
    Eq. (d3q18moment) (q = 18), or (P, e, eps, j_x, q_x, h_x, j_y, q_y, h_y,
    j_z, q_z, h_z, 3p_xx, 3pi_xx, p_ww, pi_ww, p_xy, p_yz, p_xz, pi_xy,
    pi_yz, pi_xz, t_x, t_y, t_z, t_xyz) for the 26-velocity model."""
    if sn is None:
        sn = s_nu(nu)
    if q == 14:
        return np.array([s_c, s_e, s_c, s_q, s_c, s_q, s_c, s_q, sn, sn, sn, sn, sn, s_t])
    if q == 18:
        return np.array([s_c, s_e, s_c, s_q, s_c, s_q, s_c, s_q, sn, s_pi, sn, s_pi, sn, sn, sn,
                         s_t, s_t, s_t])
    if q == 26:
        return np.array([s_c, s_e, s_eps, s_c, s_q, s_q, s_c, s_q, s_q, s_c, s_q, s_q,
                         sn, s_pi, sn, s_pi, sn, sn, sn, s_pi, s_pi, s_pi, s_t, s_t, s_t, s_t])
    raise ValueError("q must be 14, 18 or 26")


DUCT_FACES = ("periodic", "periodic", "wall", "wall", "wall", "wall")
CAVITY_FACES = ("wall",) * 6


def duct(q, edge, length, nu, umax=0.05, odd="paper"):
    """Square duct: x periodic (length), y and z half-way walls (edge), body
    force along x sized for centre-line speed umax.  odd="magic" ties s_q and
    s_t to s_nu (odd_rates), so the bounce-back wall error does not grow
    with nu."""
    a = edge / 2.0
    g = umax * nu / (DUCT_UMAX_COEFF * a * a)
    if odd == "magic":
        so = odd_rates(s_nu(nu))
        sv = s_vec(q, nu, s_q=so, s_t=so)
    elif odd == "paper":
        sv = s_vec(q, nu)
    else:
        raise ValueError("odd must be 'paper' or 'magic'")
    return {"model": q, "nx": length, "ny": edge, "nz": edge, "s_vec": sv,
            "faces": DUCT_FACES, "F0": (g, 0.0, 0.0)}


def cavity(q, edge, Re, lid=0.1):
    """Cubic lid-driven cavity: six walls, the +z lid moving along +x."""
    nu = lid * edge / Re
    return {"model": q, "nx": edge, "ny": edge, "nz": edge, "s_vec": s_vec(q, nu),
            "faces": CAVITY_FACES, "wall_u": {"+z": (lid, 0.0, 0.0)}}

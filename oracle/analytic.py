"""Analytic solutions the paper validates against, and its error norm
(test infrastructure only).

  duct_steady    fully developed flow in a 2a x 2b rectangular duct,
                 Sec. 4.1 (the series below Eq. (bc)); driven by a body
                 force g per unit mass, which equals -dp/dx
  duct_pulsatile oscillatory flow in the same duct, Sec. 4.2 Eq. (wa), for
                 -dp/dx = g cos(omega t)
  gre_u          global relative velocity error, Eq. (ed)

Coordinates: y in [-a, a], z in [-b, b], duct centre at 0.  For a lattice
with ny nodes between half-way walls, node j sits at y = j + 1/2 - ny/2 and
a = ny/2 (lattice units).
"""
import numpy as np


def duct_steady(y, z, a, b, g, nu, nterms=1000):
    """Streamwise velocity of steady duct flow (Sec. 4.1).

    The series of the paper is
        u = 16 a^2 g / (nu pi^3) sum_{i odd} (-1)^((i-1)/2)
              [1 - cosh(i pi z / 2a) / cosh(i pi b / 2a)] cos(i pi y / 2a) / i^3.
    Its cosh-free half sums in closed form to the plane-channel profile
    g (a^2 - y^2) / (2 nu) (Fourier cosine series of a parabola), which is
    used here; the remaining half converges exponentially.  The cosh ratio is
    written with exponentials so large arguments do not overflow.
    """
    y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64)
    u = g * (a * a - y * y) / (2.0 * nu)
    acc = np.zeros(np.broadcast(y, z).shape)
    for k in range(nterms):
        i = 2 * k + 1
        kk = i * np.pi / (2.0 * a)
        # cosh(kk z) / cosh(kk b), |z| <= b
        ratio = (np.exp(kk * (np.abs(z) - b)) + np.exp(-kk * (np.abs(z) + b))) / (
            1.0 + np.exp(-2.0 * kk * b))
        acc = acc + (-1.0) ** k * ratio * np.cos(kk * y) / i ** 3
        # stop on the term's bound (a single term can vanish through its cosine)
        if np.max(ratio) / i ** 3 < 1e-18:
            break
    return u - 16.0 * a * a * g / (nu * np.pi ** 3) * acc


def duct_steady_umax_coeff(nterms=1000):
    """u_max / (g a^2 / nu) for a square duct (a = b)."""
    return float(duct_steady(0.0, 0.0, 1.0, 1.0, 1.0, 1.0, nterms))


def _cosh_ratio(gam, s, h):
    """cosh(gam s) / cosh(gam h) for complex gam with Re(gam) > 0, |s| <= h."""
    s = np.abs(s)
    return (np.exp(gam * (s - h)) + np.exp(-gam * (s + h))) / (1.0 + np.exp(-2.0 * gam * h))


def duct_pulsatile(y, z, t, a, b, g, nu, omega, nterms=2000):
    """Streamwise velocity of pulsatile duct flow, Sec. 4.2 Eq. (wa).

    The paper writes it for dp/dx = G cos(omega t) as
        u = Re{ i G/omega [1 - 2 sum_n (-1)^n / p_n (
                 cosh(gamma_n y/b) cos(p_n z/b) / cosh(gamma_n a/b)
               + cosh(sigma_n z/b) cos(q_n y/b) / cosh(sigma_n) )] e^{i omega t} },
        gamma_n = sqrt(p_n^2 + i eta^2), sigma_n = sqrt(q_n^2 + i eta^2),
        p_n = (2n+1) pi / 2, q_n = (2n+1) pi b / (2a), eta = b sqrt(omega/nu).
    With a body force g cos(omega t) = -dp/dx, G = -g.
    """
    y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64)
    G = -g
    eta2 = b * b * omega / nu
    acc = np.zeros(np.broadcast(y, z).shape, np.complex128)
    for n in range(nterms):
        pn = (2 * n + 1) * np.pi / 2.0
        qn = (2 * n + 1) * np.pi * b / (2.0 * a)
        gam = np.sqrt(pn * pn + 1j * eta2)
        sig = np.sqrt(qn * qn + 1j * eta2)
        term = ((-1.0) ** n / pn) * (
            _cosh_ratio(gam / b, y, a) * np.cos(pn * z / b)
            + _cosh_ratio(sig / b, z, b) * np.cos(qn * y / b))
        acc = acc + term
    U = 1j * G / omega * (1.0 - 2.0 * acc)
    return np.real(U * np.exp(1j * omega * t))


def gre_u(u_num, u_ana):
    """Eq. (ed): sqrt(sum |u_n - u_a|^2) / sqrt(sum |u_a|^2) over all nodes
    and the three components (arrays of identical shape)."""
    u_num = np.asarray(u_num, np.float64)
    u_ana = np.asarray(u_ana, np.float64)
    return float(np.sqrt(np.sum((u_num - u_ana) ** 2)) / np.sqrt(np.sum(u_ana ** 2)))


def node_coords(n):
    """Positions of n nodes between half-way walls, centred on 0."""
    return np.arange(n, dtype=np.float64) + 0.5 - n / 2.0

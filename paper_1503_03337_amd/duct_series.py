"""Steady rectangular-duct velocity (Sec. 4.1 of arXiv 1503.03337), used to
report the accuracy of served duct solves.

u(y, z) = g (a^2 - y^2) / (2 nu)
          - 16 a^2 g / (nu pi^3) sum_{k>=0} (-1)^k cos(m y) cosh(m z) / (cosh(m b) i^3),
with i = 2k+1, m = i pi / (2a): the paper's series with its cosh-free part
summed in closed form.  y in [-a, a], z in [-b, b].
"""
import numpy as np


def velocity(y, z, a, b, g, nu, terms=2000):
    y = np.asarray(y, np.float64)
    z = np.abs(np.asarray(z, np.float64))
    s = np.zeros(np.broadcast(y, z).shape)
    for k in range(terms):
        i = 2 * k + 1
        m = i * np.pi / (2.0 * a)
        bound = 1.0 / i ** 3
        ch = (np.exp(m * (z - b)) + np.exp(-m * (z + b))) / (1.0 + np.exp(-2.0 * m * b))
        s += (1.0 if k % 2 == 0 else -1.0) * np.cos(m * y) * ch / i ** 3
        if np.max(ch) * bound < 1e-18:
            break
    return g * (a * a - y * y) / (2.0 * nu) - 16.0 * a * a * g / (nu * np.pi ** 3) * s

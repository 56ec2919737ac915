"""Seeded synthetic inputs shared by the tests, the benchmark and the
serving driver.  Random numbers and shapes only: nothing here evaluates the
lattice Boltzmann method (each side that needs an equilibrium computes it
itself from the fields drawn here).
"""
import numpy as np


def random_populations(q, nx, ny, nz, seed, levels=None, spread=0.25):
    """Populations f[a, z, y, x] = levels[a] * (1 + spread * xi), xi ~ U(-1, 1).

    `levels` (length q) sets the magnitude per direction; default 0.05 for
    the six axis directions and 0.0125 for the diagonal ones (the size of
    near-rest populations of both lattices at order-0.1 pressure)."""
    rng = np.random.default_rng(seed)
    if levels is None:
        levels = np.array([0.05] * 6 + [0.0125] * (q - 6))
    levels = np.asarray(levels, np.float64).reshape(q, 1, 1, 1)
    xi = rng.uniform(-1.0, 1.0, (q, nz, ny, nx))
    return levels * (1.0 + spread * xi)


def random_fields(nx, ny, nz, seed, p_amp=0.01, u_amp=0.05, smooth=True):
    """Pressure p[z,y,x] ~ U(-p_amp, p_amp) and velocity u[d,z,y,x] with
    |u_d| <= u_amp: either white noise or (smooth=True) a sum of a few
    random low Fourier modes, the shape of a developing flow."""
    rng = np.random.default_rng(seed)
    if not smooth:
        p = rng.uniform(-p_amp, p_amp, (nz, ny, nx))
        u = rng.uniform(-u_amp, u_amp, (3, nz, ny, nx))
        return p, u
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")

    def field(amp):
        acc = np.zeros((nz, ny, nx))
        for _ in range(4):
            kx, ky, kz = rng.integers(0, 3, 3)
            ph = rng.uniform(0, 2 * np.pi, 3)
            acc += rng.uniform(-1, 1) * (np.cos(2 * np.pi * kx * x / nx + ph[0])
                                         * np.cos(2 * np.pi * ky * y / ny + ph[1])
                                         * np.cos(2 * np.pi * kz * z / nz + ph[2]))
        m = np.max(np.abs(acc))
        return amp * acc / m if m > 0 else acc

    p = field(p_amp)
    u = np.stack([field(u_amp) for _ in range(3)])
    return p, u


def cavity_batch(n=256, seed=0, edge=(24, 96), re=(100.0, 1000.0), lid=0.1):
    """A batch of lid-driven cavities: edge L ~ U{24..96}, Re ~ U[100, 1000],
    model 14 or 18 with probability 1/2; viscosity nu = lid * L / Re."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        L = int(rng.integers(edge[0], edge[1] + 1))
        Re = float(rng.uniform(re[0], re[1]))
        q = 14 if rng.random() < 0.5 else 18
        out.append({"q": q, "edge": L, "Re": Re, "nu": lid * L / Re, "lid": lid})
    return out


def serving_trace(n, rate, seed=1, edge=(32, 160), steps=(1000, 20000), p_residual=0.25):
    """Poisson arrivals (mean rate `rate` per second) of duct or cavity
    requests: edge ~ U{32..160}, model 14 / 18 at random, a step budget
    ~ U{1000..20000}, and with probability p_residual a stop at velocity
    residual 1e-7 instead of a fixed budget (budget kept as the cap)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        out.append({
            "id": i,
            "arrival": t,
            "kind": "duct" if rng.random() < 0.5 else "cavity",
            "edge": int(rng.integers(edge[0], edge[1] + 1)),
            "q": 14 if rng.random() < 0.5 else 18,
            "steps": int(rng.integers(steps[0], steps[1] + 1)),
            "stop_residual": 1e-7 if rng.random() < p_residual else None,
        })
    return out

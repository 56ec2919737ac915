"""The workloads at their configured sizes on the GPU, against the FP64
oracle and the paper's analytic series (Sec. 4.1, 4.2).

* D3Q14 FP64, 16x16 cross-section (half-way walls), 32 periodic, nu = 0.1,
  body force for u_max = 0.05, 2000 steps from rest: GPU vs oracle
  element-wise (FP64 parity), GRE_u vs the steady series.
* D3Q18, 64x64 cross-section x 128 periodic, F(t) = A cos(2 pi t / 2000),
  Womersley number 5, 7.5, 10 (nu from eta = a sqrt(omega/nu)), started on
  the analytic field at t = 0, five periods: FP64 / FP32 / FP16-deviation
  GPU runs vs the FP64 oracle and vs the series at T/4, T/2, 3T/4, T of the
  last period.  The flow is x-invariant, and so is the arithmetic at every
  x, so the oracle runs one x-slice (nx = 1) and is compared at every x.
* The 128^3 D3Q18 lid-driven cavity (Re = 1000) for its 20,000 steps in
  FP32 and FP16 deviations against the FP64 path, and the FP64 path against
  the oracle on a 64^3 proxy of the same viscosity for 2,000 steps.
"""
import numpy as np
import pytest

from helpers import s_nu_of, svec
from oracle import analytic as A
from oracle import runner as R
from paper_1503_03337_amd import lbm

pytestmark = pytest.mark.gpu

DUCT = ("periodic", "periodic", "wall", "wall", "wall", "wall")


def gre(u, ua):
    return A.gre_u(u, ua)


def test_steady_duct_q14_fp64_16x16x32():
    q, n, L, nu = 14, 16, 32, 0.1
    a = n / 2.0
    g = 0.05 * nu / (A.duct_steady_umax_coeff() * a * a)
    s = svec(q, s_nu_of(nu))
    lat = lbm.Lattice(q, L, n, n, s, faces=DUCT, F0=(g, 0, 0), storage="f64", pattern="aa")
    lat.step(2000)
    _, u = lat.macros()
    lat.close()
    pr = R.problem(q, L, n, n, s, faces=DUCT, F0=(g, 0, 0))
    ref = R.run(pr, R.init_eq(pr), 0, 2000)
    _, ur = R.macros(pr, ref, 2000)
    assert np.linalg.norm(u - ur) <= 1e-12 * np.linalg.norm(ur)
    y = A.node_coords(n)
    Y, Z = np.meshgrid(y, y, indexing="xy")
    ua = np.zeros_like(u)
    ua[0] = A.duct_steady(Y, Z, a, a, g, nu)[:, :, None]
    e = gre(u, ua)
    print("D3Q14 FP64 duct 16x16x32: GRE_u vs series %.3e" % e)
    assert e < 8e-3


PERIOD = 2000
PHASES = (PERIOD // 4, PERIOD // 2, 3 * PERIOD // 4, PERIOD)


def pulsatile_setup(eta, n=64):
    a = n / 2.0
    om = 2 * np.pi / PERIOD
    nu = a * a * om / eta ** 2
    y = A.node_coords(n)
    Y, Z = np.meshgrid(y, y, indexing="xy")
    peak = max(np.abs(A.duct_pulsatile(Y, Z, t, a, a, 1.0, nu, om, 600)).max()
               for t in np.linspace(0, PERIOD, 9))
    g = 0.05 / peak
    return a, om, nu, g, Y, Z


@pytest.mark.parametrize("eta", (5.0, 7.5, 10.0))
def test_pulsatile_duct_q18_64x64x128(eta):
    q, n, L = 18, 64, 128
    a, om, nu, g, Y, Z = pulsatile_setup(eta, n)
    s = svec(q, s_nu_of(nu))
    kw = dict(faces=DUCT, FA=(g, 0, 0), FT=float(PERIOD))
    u0 = np.zeros((3, n, n, 1))
    u0[0, :, :, 0] = A.duct_pulsatile(Y, Z, 0.0, a, a, g, nu, om, 600)
    # oracle: one x-slice
    pr = R.problem(q, 1, n, n, s, **kw)
    f = R.init_eq(pr, 0, p=np.zeros((n, n, 1)), u=u0)
    f = R.run(pr, f, 0, 4 * PERIOD)
    ref = {}
    t = 4 * PERIOD
    for ph in PHASES:
        f = R.run(pr, f, t, 4 * PERIOD + ph - t)
        t = 4 * PERIOD + ph
        ref[ph] = R.macros(pr, f, t)[1][0, :, :, 0]
    ana = {ph: A.duct_pulsatile(Y, Z, 4 * PERIOD + ph, a, a, g, nu, om, 600) for ph in PHASES}
    uL = np.repeat(u0, L, axis=3)
    out = {}
    for storage in ("f64", "f32", "f16dev"):
        lat = lbm.Lattice(q, L, n, n, s, storage=storage, pattern="aa", **kw)
        lat.init_fields(np.zeros((n, n, L)), uL)
        lat.step(4 * PERIOD)
        errs = []
        for ph in PHASES:
            lat.step(4 * PERIOD + ph - lat.time)
            ux = lat.macros()[1][0]  # (z, y, x)
            vs_oracle = np.max(np.abs(ux - ref[ph][:, :, None])) / 0.05
            vs_series = gre(ux, np.repeat(ana[ph][:, :, None], L, axis=2))
            errs.append((vs_oracle, vs_series))
        lat.close()
        out[storage] = errs
        print("pulsatile eta=%.1f %-6s max|u-oracle|/0.05 %s  GRE_u vs series %s" % (
            eta, storage, " ".join("%.1e" % e[0] for e in errs),
            " ".join("%.2e" % e[1] for e in errs)))
    assert max(e[0] for e in out["f64"]) <= 1e-11
    assert max(e[0] for e in out["f32"]) <= 1e-4
    assert max(e[0] for e in out["f16dev"]) <= 5e-3
    # second-order bounce-back error at a = 32 (the T/2 and T samples sit
    # near a flow reversal, where the relative norm is largest)
    assert max(e[1] for e in out["f64"]) <= 0.05


@pytest.mark.parametrize("q", (14, 18))
def test_half_cavity_with_symmetry_plane_fp32(q):
    """Sec. 4.3 computes the cavity on half the grid with a symmetry plane at
    mid-depth.  The lid moves along x on +y, so the cube is mirror-symmetric
    in z: the half cavity (symmetry plane on +z) must reproduce the lower
    half of the full cavity, at half the memory."""
    n, steps = 48, 600
    s = svec(q, s_nu_of(0.1 * n / 400.0))
    lid = {"+y": (0.1, 0.0, 0.0)}
    full = lbm.Lattice(q, n, n, n, s, faces=("wall",) * 6, wall_u=lid, storage="f32")
    half = lbm.Lattice(q, n, n, n // 2, s, faces=("wall",) * 5 + ("symmetry",), wall_u=lid,
                       storage="f32")
    full.step(steps)
    half.step(steps)
    _, uf = full.macros()
    _, uh = half.macros()
    full.close()
    half.close()
    low = uf[:, : n // 2]
    err = np.max(np.abs(low - uh)) / np.max(np.abs(low))
    print("half cavity q=%d: max|u_half - u_full|/max|u| %.2e" % (q, err))
    assert err <= 1e-5


def _rel(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def test_headline_cavity_fp32_and_fp16_against_fp64_after_20000_steps():
    """The 128^3 D3Q18 lid-driven cavity at Re = 1000 (lid 0.1, nu = 0.0128),
    the measured workload, run for its 20,000 steps in FP32 and FP16
    deviations against the FP64 path (itself equal to the oracle per step to
    1e-13, and on the 64^3 proxy below over 2,000 steps).  Measured: FP32
    rel. L2 1.3e-7 (u), 1.1e-6 (p); FP16 2.8e-4 (u), 7.5e-3 (p, a field
    three orders below u^2 here)."""
    from paper_1503_03337_amd import params
    n = 128
    cfg = params.cavity(18, n, 1000.0, lid=0.1)
    res = {}
    for storage in ("f64", "f32", "f16dev"):
        lat = lbm.Lattice(18, n, n, n, cfg["s_vec"], faces=cfg["faces"], wall_u=cfg["wall_u"],
                          storage=storage, pattern="aa")
        lat.step(20000)
        p, u = lat.macros()
        res[storage] = (p - p.mean(), u)
        lat.close()
    p64, u64 = res["f64"]
    assert _rel(res["f32"][1], u64) <= 1e-5 and _rel(res["f32"][0], p64) <= 1e-5
    assert _rel(res["f16dev"][1], u64) <= 2e-3 and _rel(res["f16dev"][0], p64) <= 5e-2
    print("128^3 cavity, 20000 steps, rel L2 vs FP64: FP32 u %.2e p %.2e, FP16 u %.2e p %.2e"
          % (_rel(res["f32"][1], u64), _rel(res["f32"][0], p64),
             _rel(res["f16dev"][1], u64), _rel(res["f16dev"][0], p64)))


def test_cavity_64_fp64_equals_oracle_after_2000_steps():
    """The same cavity physics on a 64^3 proxy (nu = 0.0128, Re = 500 on the
    shorter lid): the FP64 GPU path against the FP64 oracle after 2,000
    steps from rest."""
    from paper_1503_03337_amd import params
    m = 64
    cfg = params.cavity(18, m, 500.0, lid=0.1)
    lat = lbm.Lattice(18, m, m, m, cfg["s_vec"], faces=cfg["faces"], wall_u=cfg["wall_u"],
                      storage="f64", pattern="aa")
    pr = R.problem(18, m, m, m, cfg["s_vec"], faces=cfg["faces"], wall_u=cfg["wall_u"])
    f = R.init_eq(pr)
    lat.set_f(f)
    g = R.run(pr, f, 0, 2000)
    lat.step(2000)
    assert _rel(lat.get_f(), g) <= 1e-12
    p, u = lat.macros()
    pr_, ur = R.macros(pr, g, 2000)
    assert _rel(u, ur) <= 1e-12
    lat.close()

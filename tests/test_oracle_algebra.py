"""Pins of the oracle's lattice algebra against the paper, in exact arithmetic
where possible (Sec. 2, Sec. 3, Appendix B of arXiv 1503.03337)."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from helpers import read_matrix, svec, velocities, weights_d3q15_d3q19
from oracle import runner as R

QS = (14, 18)


def basis_T(q):
    """T rebuilt from the basis-vector formulas: Eq. (m) of Sec. 3 for q = 14,
    Eq. (appendix_m18) for q = 18 (independent of the printed matrix)."""
    c = velocities(q)
    rows = []
    for cx, cy, cz in c:
        n2 = cx * cx + cy * cy + cz * cz
        if q == 14:
            col = [Fr(1), Fr(7 * n2, 2) - Fr(15, 2),
                   Fr(cx), Fr((5 * n2 - 13) * cx, 2),
                   Fr(cy), Fr((5 * n2 - 13) * cy, 2),
                   Fr(cz), Fr((5 * n2 - 13) * cz, 2),
                   Fr(3 * cx * cx - n2), Fr(cy * cy - cz * cz),
                   Fr(cx * cy), Fr(cy * cz), Fr(cx * cz), Fr(cx * cy * cz)]
        else:
            col = [Fr(1), Fr(3 * n2 - 5),
                   Fr(cx), Fr((5 * n2 - 9) * cx),
                   Fr(cy), Fr((5 * n2 - 9) * cy),
                   Fr(cz), Fr((5 * n2 - 9) * cz),
                   Fr(3 * cx * cx - n2), Fr((3 * n2 - 5) * (3 * cx * cx - n2)),
                   Fr(cy * cy - cz * cz), Fr((3 * n2 - 5) * (cy * cy - cz * cz)),
                   Fr(cx * cy), Fr(cy * cz), Fr(cx * cz),
                   Fr((cy * cy - cz * cz) * cx), Fr((cz * cz - cx * cx) * cy),
                   Fr((cx * cx - cy * cy) * cz)]
        rows.append(col)
    return [list(r) for r in zip(*rows)]  # transpose: rows = moments


@pytest.mark.parametrize("q", QS)
def test_velocity_set_matches_paper(q):
    c, w, opp, w0, T, N = R.lattice(q)
    assert np.array_equal(c, velocities(q))
    for a in range(q):
        assert np.array_equal(c[opp[a]], -c[a])


@pytest.mark.parametrize("q", QS)
def test_T_equals_printed_and_basis_formulas(q):
    _, _, _, _, T, _ = R.lattice(q)
    printed = read_matrix("T%d_printed.txt" % q)
    assert printed.shape == (q, q)
    assert np.array_equal(T, printed)
    B = basis_T(q)
    assert all(B[k][a] == int(printed[k, a]) for k in range(q) for a in range(q))
    assert int(np.count_nonzero(T)) == (130 if q == 14 else 192)


@pytest.mark.parametrize("q", QS)
def test_rows_orthogonal_and_norms(q):
    _, _, _, _, T, N = R.lattice(q)
    G = T.astype(np.int64) @ T.T.astype(np.int64)
    assert np.array_equal(G, np.diag(np.diag(G)))
    assert np.array_equal(np.diag(G), N.astype(np.int64))
    expect = {14: [14, 168, 10, 40, 10, 40, 10, 40, 12, 4, 8, 8, 8, 8],
              18: [18, 36, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8]}[q]
    assert list(np.diag(G)) == expect


def test_gram_schmidt_of_monomials_gives_T14():
    """Sec. 3: T follows from orthogonalising the rows of Tbar in order."""
    Tbar = read_matrix("Tbar14_printed.txt")
    c = velocities(14)
    n2 = np.sum(c * c, axis=1)
    cx, cy, cz = c[:, 0], c[:, 1], c[:, 2]
    mono = np.array([n2 ** 0, n2, cx, n2 * cx, cy, n2 * cy, cz, n2 * cz, 3 * cx * cx,
                     cy * cy - cz * cz, cx * cy, cy * cz, cx * cz, cx * cy * cz])
    assert np.array_equal(Tbar, mono)
    rows = [[Fr(int(v)) for v in r] for r in Tbar]
    ortho = []
    for r in rows:
        v = list(r)
        for o in ortho:
            coef = sum(a * b for a, b in zip(v, o)) / sum(b * b for b in o)
            v = [a - coef * b for a, b in zip(v, o)]
        ortho.append(v)
    T = read_matrix("T14_printed.txt")
    for k in range(14):
        nz = [a for a in range(14) if T[k, a] != 0]
        ratio = ortho[k][nz[0]] / int(T[k, nz[0]])
        assert ratio != 0
        assert all(ortho[k][a] == ratio * int(T[k, a]) for a in range(14))


def feq_exact(q, p, u, w0, w):
    """Eq. (edf) with Eq. (lamda_alpha), a = 1..q, c_s^2 = 1/3, in Fractions."""
    c = velocities(q)
    usq = sum(x * x for x in u)
    out = []
    for a in range(q):
        cu = sum(int(c[a, d]) * u[d] for d in range(3))
        out.append(3 * w[a] * p + w[a] * (3 * cu + Fr(9, 2) * cu * cu - Fr(3, 2) * usq))
    return out


def rand_state(rng):
    p = Fr(int(rng.integers(-500, 500)), 10000)
    u = [Fr(int(rng.integers(-800, 800)), 10000) for _ in range(3)]
    return p, u


@pytest.mark.parametrize("q", QS)
def test_feq_and_moment_equilibria(q):
    """T f_eq (Eq. (edf), D3Q15 / D3Q19 weights) equals the printed moment
    equilibria that the oracle evaluates (Eq. (meq), Appendix B)."""
    w0, w = weights_d3q15_d3q19(q)
    T = read_matrix("T%d_printed.txt" % q)
    rng = np.random.default_rng(q)
    for _ in range(20):
        p, u = rand_state(rng)
        fe = feq_exact(q, p, u, w0, w)
        m = [sum(int(T[k, a]) * fe[a] for a in range(q)) for k in range(q)]
        uf = np.array([float(x) for x in u])
        assert np.allclose(R.feq(q, float(p), uf), [float(x) for x in fe], rtol=0, atol=1e-16)
        assert np.allclose(R.meq(q, float(p), uf), [float(x) for x in m], rtol=0, atol=4e-16)


def test_printed_weights_do_not_fit_q14():
    """Eq. (omega) prints 1/3, 1/18, 1/36; with those T f_eq misses the
    printed P_eq = 7p/3 + u^2/3, which is why the D3Q15 weights are used."""
    T = read_matrix("T14_printed.txt")
    c = velocities(14)
    w = [Fr(1, 18) if int(np.sum(v * v)) == 1 else Fr(1, 36) for v in c]
    p, u = Fr(1, 100), [Fr(3, 100), Fr(-2, 100), Fr(1, 100)]
    fe = feq_exact(14, p, u, Fr(1, 3), w)
    P = sum(int(T[0, a]) * fe[a] for a in range(14))
    usq = sum(x * x for x in u)
    assert P != Fr(7, 3) * p + usq / 3


@pytest.mark.parametrize("q", QS)
def test_pressure_velocity_recovery(q):
    """Eq. (hgl) returns exactly the p and u put into f_eq."""
    rng = np.random.default_rng(100 + q)
    for _ in range(20):
        p = rng.uniform(-0.05, 0.05)
        u = rng.uniform(-0.1, 0.1, 3)
        pp, uu = R.macro_node(q, R.feq(q, p, u))
        assert abs(pp - p) < 1e-16 and np.max(np.abs(uu - u)) < 1e-16


@pytest.mark.parametrize("q", QS)
def test_forcing_moments_are_guo_source(q):
    """The oracle's m_F equals T applied to the discrete (Guo) source
    w_a [3 c.F + 9 (c.u)(c.F) - 3 u.F] over a = 1..q, exactly."""
    w0, w = weights_d3q15_d3q19(q)
    T = read_matrix("T%d_printed.txt" % q)
    c = velocities(q)
    rng = np.random.default_rng(200 + q)
    for _ in range(20):
        _, u = rand_state(rng)
        F = [Fr(int(rng.integers(-300, 300)), 100000) for _ in range(3)]
        uF = sum(a * b for a, b in zip(u, F))
        src = []
        for a in range(q):
            cu = sum(int(c[a, d]) * u[d] for d in range(3))
            cF = sum(int(c[a, d]) * F[d] for d in range(3))
            src.append(w[a] * (3 * cF + 9 * cu * cF - 3 * uF))
        m = [float(sum(int(T[k, a]) * src[a] for a in range(q))) for k in range(q)]
        got = R.mforce(q, np.array([float(x) for x in u]), np.array([float(x) for x in F]))
        assert np.allclose(got, m, rtol=0, atol=1e-18)


@pytest.mark.parametrize("q", QS)
def test_bgk_limit(q):
    """Sec. 3 / Appendix B: S = I/tau turns the MRT collision into the LBGK
    update f - (f - f_eq)/tau (+ (1 - 1/(2 tau)) times the source with a
    force), with f_eq from Eq. (edf) evaluated here independently."""
    w0, w = weights_d3q15_d3q19(q)
    c = velocities(q)
    wf = np.array([float(x) for x in w])
    rng = np.random.default_rng(300 + q)
    for tau in (0.55, 0.8, 1.0, 1.7):
        for F in (np.zeros(3), np.array([2e-4, -1e-4, 3e-4])):
            base = R.feq(q, 0.01, np.array([0.03, -0.02, 0.04]))
            f = base + 1e-3 * rng.uniform(-1, 1, q)
            P = f.sum()
            u = c.T.astype(float) @ f + 0.5 * F
            usq = u @ u
            p = (P - 1.5 * float(w0) * usq) / (3 * (1 - float(w0)))
            cu = c.astype(float) @ u
            fe = wf * (3 * p + 3 * cu + 4.5 * cu * cu - 1.5 * usq)
            cF = c.astype(float) @ F
            src = wf * (3 * cF + 9 * cu * cF - 3 * (u @ F))
            expect = f - (f - fe) / tau + (1 - 0.5 / tau) * src
            got = R.collide(q, np.full(q, 1.0 / tau), f, F)
            assert np.max(np.abs(got - expect)) < 2e-17


@pytest.mark.parametrize("q", QS)
def test_collision_conserves_P_and_j(q):
    """P = sum f and j = sum c f are conserved by the unforced collision
    (Appendix A: P is conserved), to 1e-14 relative; with a force j gains F."""
    c = velocities(q).astype(float)
    rng = np.random.default_rng(400 + q)
    for _ in range(50):
        f = R.feq(q, rng.uniform(-0.02, 0.02), rng.uniform(-0.08, 0.08, 3))
        f = f + 2e-3 * rng.uniform(-1, 1, q)
        s = svec(q, rng.uniform(0.5, 1.95))
        fs = R.collide(q, s, f)
        scale = np.max(np.abs(f))
        assert abs(fs.sum() - f.sum()) <= 1e-14 * scale
        assert np.max(np.abs(c.T @ fs - c.T @ f)) <= 1e-14 * scale
        F = rng.uniform(-1e-4, 1e-4, 3)
        fs = R.collide(q, s, f, F)
        assert np.max(np.abs(c.T @ fs - (c.T @ f + F))) <= 1e-14 * scale


@pytest.mark.parametrize("q", QS)
def test_zero_rates_are_identity(q):
    """S = 0 (no force) leaves every population bit-identical."""
    rng = np.random.default_rng(500 + q)
    f = R.feq(q, 0.01, np.array([0.02, 0.01, -0.03])) + 1e-3 * rng.uniform(-1, 1, q)
    assert np.array_equal(R.collide(q, np.zeros(q), f), f)

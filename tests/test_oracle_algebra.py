"""Pins of the oracle's lattice algebra against the paper, in exact arithmetic
where possible (Sec. 2, Sec. 3, Appendix B of arXiv 1503.03337).  The
26-velocity model named at the end of Appendix B is pinned against its
construction (Gram-Schmidt of monomial rows, Sec. 3), the isotropy of the
D3Q27 weights, and closed forms of T f_eq derived in exact rationals."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from helpers import (T_matrix, gram_schmidt_rows, monomials26, read_matrix, svec, velocities,
                     weights_d3q15_d3q19)
from oracle import runner as R

QS = (14, 18, 26)


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
        elif q == 26:
            q_, r_, s_ = 3 * n2 - 7, 3 * n2 - 5, 3 * n2 - 8
            h_ = Fr(9 * n2 * n2 - 39 * n2 + 38, 2)
            col = [Fr(1), Fr(13 * n2 - 27), Fr(15 * n2 * n2 - 61 * n2 + 54, 2)]
            for v in (cx, cy, cz):
                col += [Fr(v), Fr(q_ * v), h_ * v]
            col += [Fr(3 * cx * cx - n2), Fr(r_ * (3 * cx * cx - n2)),
                    Fr(cy * cy - cz * cz), Fr(r_ * (cy * cy - cz * cz)),
                    Fr(cx * cy), Fr(cy * cz), Fr(cx * cz),
                    Fr(s_ * cx * cy), Fr(s_ * cy * cz), Fr(s_ * cx * cz),
                    Fr((cy * cy - cz * cz) * cx), Fr((cz * cz - cx * cx) * cy),
                    Fr((cx * cx - cy * cy) * cz), Fr(cx * cy * cz)]
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
    if q == 26:
        # no printed matrix: the basis polynomials of the oracle equal the
        # rows Sec. 3's construction gives (test_gram_schmidt_of_monomials_gives_T26)
        B = basis_T(q)
        assert all(B[k][a] == int(T[k, a]) for k in range(q) for a in range(q))
        assert int(np.count_nonzero(T)) == 404
        return
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
              18: [18, 36, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8],
              26: [26, 2340, 360, 18, 72, 72, 18, 72, 72, 18, 72, 72, 36, 72, 12, 24,
                   12, 12, 12, 24, 24, 24, 8, 8, 8, 8]}[q]
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


def test_gram_schmidt_of_monomials_gives_T26():
    """The closing paragraph of Appendix B: Sec. 3's construction gives the
    26-velocity model too.  The 26 monomial rows (by tensor order) are
    independent on the 26 velocities, and orthogonalising them in order gives
    the oracle's T row by row (up to the integer scale of each row)."""
    M = monomials26()
    assert np.linalg.matrix_rank(M.astype(float)) == 26
    G = gram_schmidt_rows(M)
    _, _, _, _, T, _ = R.lattice(26)
    assert np.array_equal(G, T)
    # the first rows of every class are the monomials themselves, unchanged
    for k in (0, 3, 6, 9, 14, 16, 17, 18, 22, 23, 24, 25):
        assert np.array_equal(T[k], M[k])


def test_d3q27_weights_are_isotropic():
    """The weights the 26-velocity model takes (D3Q27: 8/27 rest, 2/27, 1/54,
    1/216) are those for which Eq. (edf) has the lattice moments the
    Chapman-Enskog recovery needs: sum w = 1, sum w c_i c_j = delta_ij / 3,
    sum w c_i c_j c_k c_l = (d_ij d_kl + d_ik d_jl + d_il d_jk) / 9, odd
    moments zero; the oracle holds exactly these."""
    w0, w = weights_d3q15_d3q19(26)
    c = velocities(26)
    _, wo, _, w0o, _, _ = R.lattice(26)
    assert w0o == float(w0) and np.array_equal(wo, [float(x) for x in w])
    assert w0 + sum(w) == 1
    d = np.eye(3, dtype=int)
    for i in range(3):
        assert sum(w[a] * int(c[a, i]) for a in range(26)) == 0
        for j in range(3):
            assert sum(w[a] * int(c[a, i] * c[a, j]) for a in range(26)) == Fr(int(d[i, j]), 3)
            for k in range(3):
                assert sum(w[a] * int(c[a, i] * c[a, j] * c[a, k]) for a in range(26)) == 0
                for l in range(3):
                    m4 = sum(w[a] * int(c[a, i] * c[a, j] * c[a, k] * c[a, l])
                             for a in range(26))
                    assert m4 == Fr(int(d[i, j] * d[k, l] + d[i, k] * d[j, l]
                                        + d[i, l] * d[j, k]), 9)


def q26_moment_equilibria(p, u, F=None):
    """Closed forms of T f_eq for the 26-velocity model (derived in exact
    rationals from Eq. (edf) with the D3Q27 weights), and of the forcing
    moments (d/du . F of each) when F is given."""
    ux, uy, uz = u
    usq = ux * ux + uy * uy + uz * uz
    xx, ww = 3 * ux * ux - usq, uy * uy - uz * uz
    meq = [Fr(19, 9) * p + Fr(4, 9) * usq, -18 * p + usq, 3 * p - usq,
           ux, -2 * ux, ux, uy, -2 * uy, uy, uz, -2 * uz, uz,
           xx, -xx, ww, -ww, ux * uy, uy * uz, ux * uz, -ux * uy, -uy * uz, -ux * uz,
           0, 0, 0, 0]
    if F is None:
        return meq
    Fx, Fy, Fz = F
    wF = ux * Fx + uy * Fy + uz * Fz
    gxx, gww = 6 * ux * Fx - 2 * wF, 2 * (uy * Fy - uz * Fz)
    gxy, gyz, gxz = ux * Fy + uy * Fx, uy * Fz + uz * Fy, ux * Fz + uz * Fx
    mF = [Fr(8, 9) * wF, 2 * wF, -2 * wF, Fx, -2 * Fx, Fx, Fy, -2 * Fy, Fy, Fz, -2 * Fz, Fz,
          gxx, -gxx, gww, -gww, gxy, gyz, gxz, -gxy, -gyz, -gxz, 0, 0, 0, 0]
    return meq, mF


def test_q26_moment_equilibria_closed_forms():
    """For the 26-velocity model T f_eq (exact rationals, D3Q27 weights)
    equals the closed forms above, T (Guo source) their u-derivatives along
    F, and the oracle's m_eq and m_F match both."""
    w0, w = weights_d3q15_d3q19(26)
    T = T_matrix(26)
    c = velocities(26)
    rng = np.random.default_rng(26)
    for _ in range(12):
        p, u = rand_state(rng)
        F = [Fr(int(rng.integers(-300, 300)), 100000) for _ in range(3)]
        fe = feq_exact(26, p, u, w0, w)
        uF = sum(a * b for a, b in zip(u, F))
        src = []
        for a in range(26):
            cu = sum(int(c[a, d]) * u[d] for d in range(3))
            cF = sum(int(c[a, d]) * F[d] for d in range(3))
            src.append(w[a] * (3 * cF + 9 * cu * cF - 3 * uF))
        m = [sum(int(T[k, a]) * fe[a] for a in range(26)) for k in range(26)]
        ms = [sum(int(T[k, a]) * src[a] for a in range(26)) for k in range(26)]
        closed, closed_F = q26_moment_equilibria(p, u, F)
        assert m == closed and ms == closed_F
        uf, Ff = np.array([float(x) for x in u]), np.array([float(x) for x in F])
        assert np.allclose(R.meq(26, float(p), uf), [float(x) for x in closed], rtol=0, atol=2e-15)
        assert np.allclose(R.mforce(26, uf, Ff), [float(x) for x in closed_F], rtol=0, atol=1e-17)


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
    T = T_matrix(q)
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
    T = T_matrix(q)
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
        # (q = 26 forms T src in FP64: 26-term sums of values up to 1e-3)
        assert np.allclose(got, m, rtol=0, atol=1e-18 if q < 26 else 1e-17)


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

"""Pins of the oracle's streaming, walls and whole step: an independent
pull-form permutation, exact-rational brute force on 4^3 lattices, and the
conservation properties of the scheme (Eq. (mrteq), Appendix A)."""
import itertools
from fractions import Fraction as Fr

import numpy as np
import pytest

from helpers import svec, velocities, weights_d3q15_d3q19
from oracle import runner as R

FACESETS = {
    "periodic": ("periodic",) * 6,
    "halfcavity": ("wall", "wall", "wall", "wall", "wall", "symmetry"),
    "symchannel": ("periodic", "periodic", "periodic", "periodic", "symmetry", "symmetry"),
    "symmix": ("symmetry", "wall", "periodic", "periodic", "wall", "symmetry"),
    "duct": ("periodic", "periodic", "wall", "wall", "wall", "wall"),
    "cavity": ("wall",) * 6,
    "channel": ("periodic", "periodic", "periodic", "periodic", "wall", "wall"),
    "xwalls": ("wall", "wall", "periodic", "periodic", "periodic", "periodic"),
}


def pull_permutation(q, dims, faces, f):
    """Streaming with identity collision written in pull form: the value
    arriving at node y in direction a comes from y - c_a (periodic axes
    wrap); if y - c_a lies beyond a wall it is y's own opposite population
    (no-slip walls); if it lies beyond symmetry planes only, it is the
    mirrored population of the node reached by moving along the planes only
    (specular reflection)."""
    c = velocities(q)
    opp = [int(np.nonzero((c == -c[a]).all(axis=1))[0][0]) for a in range(q)]
    nx, ny, nz = dims
    out = np.empty_like(f)
    for a in range(q):
        for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
            own = [x, y, z]
            src = [x - c[a, 0], y - c[a, 1], z - c[a, 2]]
            wall, flip = False, [False] * 3
            for d, n in enumerate(dims):
                if 0 <= src[d] < n:
                    continue
                kind = faces[2 * d + (0 if src[d] < 0 else 1)]
                if kind == "periodic":
                    src[d] %= n
                elif kind == "symmetry":
                    flip[d] = True
                    src[d] = own[d]
                else:
                    wall = True
            if wall:
                out[a, z, y, x] = f[opp[a], z, y, x]
            elif any(flip):
                m = np.array([-v if fl else v for v, fl in zip(c[a], flip)])
                b = int(np.nonzero((c == m).all(axis=1))[0][0])
                out[a, z, y, x] = f[b, src[2], src[1], src[0]]
            else:
                out[a, z, y, x] = f[a, src[2], src[1], src[0]]
    return out


@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("kind", sorted(FACESETS))
def test_zero_rates_step_is_bit_exact_permutation(q, kind):
    dims = (5, 4, 3)
    faces = FACESETS[kind]
    rng = np.random.default_rng(7)
    f = rng.uniform(0.0, 0.2, (q, dims[2], dims[1], dims[0]))
    pr = R.problem(q, *dims, np.zeros(q), faces=faces)
    g = R.run(pr, f, 0, 1)
    assert np.array_equal(g, pull_permutation(q, dims, faces, f))
    # two steps back-to-back equal the permutation applied twice
    g2 = R.run(pr, f, 0, 2)
    assert np.array_equal(g2, pull_permutation(q, dims, faces, pull_permutation(q, dims, faces, f)))


def _inverse(M):
    """Exact Gauss-Jordan inverse of a square Fraction matrix."""
    n = len(M)
    A = [list(r) + [Fr(int(i == j)) for j in range(n)] for i, r in enumerate(M)]
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        pv = A[col][col]
        A[col] = [v / pv for v in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                fac = A[r][col]
                A[r] = [a - fac * b for a, b in zip(A[r], A[col])]
    return [row[n:] for row in A]


def exact_step(q, dims, faces, wall_u, s, F, f):
    """One time step in exact rationals, from the paper's definitions:
    collision f* = f - T^-1 S (T f - T f_eq) + T^-1 (I - S/2) T src with a
    Gauss-Jordan T^-1, f_eq from Eq. (edf), src the Guo source, u = sum c f +
    F/2, p from Eq. (hgl); then pull streaming with half-way bounce-back and
    the moving-wall term -6 w_a (c_a . u_w) of the outgoing link."""
    from helpers import T_matrix
    c = velocities(q)
    T = [[Fr(int(v)) for v in r] for r in T_matrix(q)]
    Ti = _inverse(T)
    w0, w = weights_d3q15_d3q19(q)
    opp = [int(np.nonzero((c == -c[a]).all(axis=1))[0][0]) for a in range(q)]
    nx, ny, nz = dims
    post = {}
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        fn = [f[a][z][y][x] for a in range(q)]
        P = sum(fn)
        u = [sum(int(c[a, d]) * fn[a] for a in range(q)) + F[d] / 2 for d in range(3)]
        usq = sum(v * v for v in u)
        p = (P - Fr(3, 2) * w0 * usq) / (3 * (1 - w0))
        fe, src = [], []
        uF = sum(u[d] * F[d] for d in range(3))
        for a in range(q):
            cu = sum(int(c[a, d]) * u[d] for d in range(3))
            cF = sum(int(c[a, d]) * F[d] for d in range(3))
            fe.append(3 * w[a] * p + w[a] * (3 * cu + Fr(9, 2) * cu * cu - Fr(3, 2) * usq))
            src.append(w[a] * (3 * cF + 9 * cu * cF - 3 * uF))
        m = [sum(T[k][a] * fn[a] for a in range(q)) for k in range(q)]
        me = [sum(T[k][a] * fe[a] for a in range(q)) for k in range(q)]
        ms = [sum(T[k][a] * src[a] for a in range(q)) for k in range(q)]
        dm = [s[k] * (m[k] - me[k]) - (1 - s[k] / 2) * ms[k] for k in range(q)]
        post[(x, y, z)] = [fn[a] - sum(Ti[a][k] * dm[k] for k in range(q)) for a in range(q)]
    out = [[[[None] * nx for _ in range(ny)] for _ in range(nz)] for _ in range(q)]
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        for a in range(q):
            src_ = [x - int(c[a, 0]), y - int(c[a, 1]), z - int(c[a, 2])]
            crossed = [0, 0, 0]
            for d, n in enumerate(dims):
                if 0 <= src_[d] < n:
                    continue
                if faces[2 * d] == "periodic":
                    src_[d] %= n
                else:
                    # the outgoing link (opp[a] from this node) leaves through
                    # the face on the side of +c_opp = -c_a
                    crossed[d] = -1 if -int(c[a, d]) < 0 else 1
            if any(crossed):
                if crossed[2]:
                    uw = wall_u[4 if crossed[2] < 0 else 5]
                elif crossed[1]:
                    uw = wall_u[2 if crossed[1] < 0 else 3]
                else:
                    uw = wall_u[0 if crossed[0] < 0 else 1]
                b = opp[a]
                cu = sum(int(c[b, d]) * uw[d] for d in range(3))
                out[a][z][y][x] = post[(x, y, z)][b] - 6 * w[b] * cu
            else:
                out[a][z][y][x] = post[(src_[0], src_[1], src_[2])][a]
    return out


@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("kind", ["cavity", "duct"])
def test_bruteforce_4cube_exact(q, kind):
    """Two steps on a 4^3 lattice: oracle (FP64) against the exact-rational
    step above, with random non-equilibrium data, a moving +z wall, a body
    force and distinct relaxation rates."""
    dims = (4, 4, 4)
    faces = FACESETS[kind]
    wall_u = [[Fr(0)] * 3 for _ in range(6)]
    wall_u[5] = [Fr(1, 20), Fr(-1, 40), Fr(0)]
    rng = np.random.default_rng(11 + q)
    s_f = svec(q, 1.37)
    s_f = s_f + np.linspace(-0.05, 0.05, q)  # make every rate distinct
    s = [Fr(float(v)) for v in s_f]
    F = [Fr(3, 10000), Fr(-1, 10000), Fr(2, 10000)]
    base = R.feq(q, 0.004, np.array([0.02, -0.01, 0.015]))
    f0 = base[:, None, None, None] + 1e-3 * rng.uniform(-1, 1, (q, 4, 4, 4))
    pr = R.problem(q, *dims, s_f, faces=faces,
                   wall_u=[[float(v) for v in r] for r in wall_u],
                   F0=[float(v) for v in F])
    ex = [[[[Fr(float(v)) for v in row] for row in pl] for pl in fa] for fa in f0]
    got = f0
    for step in range(2):
        ex = exact_step(q, dims, faces, wall_u, s, F, ex)
        got = R.run(pr, got, step, 1)
        exf = np.array([[[[float(v) for v in row] for row in pl] for pl in fa] for fa in ex])
        assert np.max(np.abs(got - exf)) <= 2e-15 * np.max(np.abs(exf))


@pytest.mark.parametrize("q", (14, 18, 26))
def test_uniform_equilibrium_is_fixed_point(q):
    pr = R.problem(q, 6, 5, 4, svec(q, 1.3), faces=FACESETS["periodic"])
    f = R.init_eq(pr, 0, p0=0.01, u0=(0.03, -0.02, 0.01))
    g = R.run(pr, f, 0, 10)
    assert np.max(np.abs(g - f)) < 1e-16


@pytest.mark.parametrize("q", (14, 18, 26))
def test_mass_conserved_with_tangential_lid(q):
    """With walls and a tangential lid, sum of P = sum f is invariant
    (collision conserves P; a tangential wall adds +-pairs that cancel)."""
    pr = R.problem(q, 6, 6, 6, svec(q, 1.6), faces=FACESETS["cavity"],
                   wall_u={"+z": (0.1, 0.0, 0.0)})
    rng = np.random.default_rng(3)
    f = R.init_eq(pr) + 1e-3 * rng.uniform(-1, 1, (q, 6, 6, 6))
    m0 = f.sum()
    g = R.run(pr, f, 0, 200)
    assert abs(g.sum() - m0) <= 1e-13 * np.abs(f).sum()


@pytest.mark.parametrize("q", (14, 18, 26))
def test_momentum_grows_by_NF_per_step(q):
    """Periodic box with a body force: total j grows by exactly N F a step."""
    c = velocities(q).astype(float)
    F = np.array([1e-5, -2e-5, 3e-6])
    pr = R.problem(q, 5, 4, 3, svec(q, 1.1), faces=FACESETS["periodic"], F0=F)
    rng = np.random.default_rng(5)
    f = R.init_eq(pr) + 1e-3 * rng.uniform(-1, 1, (q, 3, 4, 5))
    j0 = np.einsum("ad,azyx->d", c, f)
    g = R.run(pr, f, 0, 7)
    j1 = np.einsum("ad,azyx->d", c, g)
    assert np.max(np.abs(j1 - j0 - 7 * 60 * F)) < 1e-14 * np.abs(f).sum()


@pytest.mark.parametrize("q", (14, 18, 26))
def test_symmetry_plane_reproduces_full_channel(q):
    """Sec. 4.3 imposes Eq. (z05symmetry) on a mid-plane to compute half the
    cavity.  A force-driven channel between walls at both z ends must equal
    the half channel with a wall below and a symmetry plane above."""
    m, g = 6, 1e-5
    s = svec(q, 1.3)
    full = R.problem(q, 3, 2, 2 * m, s, faces=FACESETS["channel"], F0=(g, 0, 0))
    half = R.problem(q, 3, 2, m, s,
                     faces=("periodic", "periodic", "periodic", "periodic", "wall", "symmetry"),
                     F0=(g, 0, 0))
    ff = R.run(full, R.init_eq(full), 0, 3000)
    fh = R.run(half, R.init_eq(half), 0, 3000)
    _, uf = R.macros(full, ff, 3000)
    _, uh = R.macros(half, fh, 3000)
    assert np.max(np.abs(uf[:, :m] - uh)) <= 1e-12 * np.max(np.abs(uf))
    # the premise: the full channel is mirror-symmetric about its mid-plane
    assert np.max(np.abs(uf[0] - uf[0, ::-1])) <= 1e-12 * np.max(np.abs(uf))
    assert np.max(np.abs(uf[2] + uf[2, ::-1])) <= 1e-12 * np.max(np.abs(uf))


@pytest.mark.parametrize("q", (14, 18, 26))
def test_symmetry_plane_reproduces_full_cavity(q):
    """Lid on +y moving along x: the cavity is mirror-symmetric in z, so its
    lower half equals the half cavity with a symmetry plane on +z, at every
    time level (transient included)."""
    m = 4
    s = svec(q, 1.5) + np.linspace(-0.02, 0.02, q)
    lid = {"+y": (0.08, 0.0, 0.0)}
    full = R.problem(q, 6, 5, 2 * m, s, faces=FACESETS["cavity"], wall_u=lid)
    half = R.problem(q, 6, 5, m, s, faces=FACESETS["halfcavity"], wall_u=lid)
    ff = R.run(full, R.init_eq(full), 0, 60)
    fh = R.run(half, R.init_eq(half), 0, 60)
    pf, uf = R.macros(full, ff, 60)
    ph, uh = R.macros(half, fh, 60)
    assert np.max(np.abs(uf[:, :m] - uh)) <= 1e-13 * np.max(np.abs(uf))
    assert np.max(np.abs(pf[:m] - ph)) <= 1e-13 * max(np.max(np.abs(pf)), 1e-30)

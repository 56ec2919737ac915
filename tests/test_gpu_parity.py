"""GPU (HIP, through the C ABI) against the FP64 oracle on the same seeded
inputs.

Tolerances:
  FP64 storage: populations element-wise within 1e-13 of max|f|;
                p and u relative L2 (GRE form, Eq. (ed)) <= 1e-12.
  FP32 storage: p and u relative L2 <= 1e-5 (FP32 unit roundoff 6e-8 per
                operation, a few hundred operations per node-step).
  FP16-deviation storage: one step element-wise within one FP16 rounding
                (eps = 2^-11 relative to nearest, 2^-10 stochastic) plus the
                FP32 arithmetic; after k steps populations within
                2 sqrt(k) eps relative L2, velocity within k * n * eps
                max|f| (one rounding per population and step, n = 10
                populations per velocity component for 14 and 18
                velocities, 18 for 26).
The 26-velocity model (Appendix B's closing paragraph, built by Sec. 3's
construction) runs every single-lattice case the other two do.
Bit-exact: zero rates (pure streaming permutation), AA against AB, and
checkpoint/restore.
"""
import numpy as np
import pytest

from helpers import svec, velocities
from oracle import runner as R
from paper_1503_03337_amd import inputs
from paper_1503_03337_amd import lbm

pytestmark = pytest.mark.gpu

FACESETS = {
    "periodic": ("periodic",) * 6,
    "duct": ("periodic", "periodic", "wall", "wall", "wall", "wall"),
    "cavity": ("wall",) * 6,
    "xwalls": ("wall", "wall", "periodic", "periodic", "periodic", "periodic"),
    "halfcavity": ("wall", "wall", "wall", "wall", "wall", "symmetry"),
    "symmix": ("symmetry", "wall", "periodic", "periodic", "wall", "symmetry"),
    "symchannel": ("periodic", "periodic", "symmetry", "symmetry", "wall", "wall"),
}
SETUPS = {
    # name: (faces, wall_u, F0, FA, FT)
    "periodic_force": ("periodic", None, (2e-5, -1e-5, 3e-5), (0, 0, 0), 0.0),
    "duct_pulsatile": ("duct", {"+y": (0.02, 0.0, 0.01)}, (1e-5, 0, 0), (3e-5, 0, 0), 7.0),
    "cavity_lid": ("cavity", {"+z": (0.1, 0.0, 0.0), "-x": (0.0, 0.03, 0.0)}, (0, 0, 0),
                   (0, 0, 0), 0.0),
    "xwalls_force": ("xwalls", {"-x": (0.0, 0.05, 0.0)}, (0, 2e-5, 0), (0, 0, 0), 0.0),
    # Sec. 4.3: half cavity, symmetry plane on +z, lid on +y
    "halfcavity_lid": ("halfcavity", {"+y": (0.1, 0.0, 0.0), "-x": (0.0, 0.0, 0.03)},
                       (0, 0, 0), (0, 0, 0), 0.0),
    "symmix_force": ("symmix", {"+x": (0.0, 0.04, 0.02), "-z": (0.03, 0.0, 0.0)},
                     (1e-5, 2e-5, -1e-5), (0, 0, 0), 0.0),
}
DIMS = [(37, 19, 11), (300, 3, 4)]


def rates(q, seed=0):
    s = svec(q, 1.45).astype(float)
    return s + np.linspace(-0.03, 0.03, q)  # all rates distinct


def make_pair(q, dims, setup, storage, pattern, seed=0, s=None):
    faces, wall_u, F0, FA, FT = SETUPS[setup]
    faces = FACESETS[faces]
    s = rates(q) if s is None else s
    lat = lbm.Lattice(q, *dims, s, faces=faces, wall_u=wall_u, F0=F0, FA=FA, FT=FT,
                      storage=storage, pattern=pattern)
    pr = R.problem(q, *dims, s, faces=faces, wall_u=wall_u, F0=F0, FA=FA, FT=FT)
    f0 = inputs.random_populations(q, *dims, seed=seed)
    lat.set_f(f0)
    f0q = lat.get_f()  # the initial state as the storage type holds it
    return lat, pr, f0q


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("pattern", ("ab", "aa"))
@pytest.mark.parametrize("setup", sorted(SETUPS))
@pytest.mark.parametrize("dims", DIMS, ids=lambda d: "x".join(map(str, d)))
def test_fp64_matches_oracle(q, pattern, setup, dims):
    print("case q=%d %s %s %s" % (q, pattern, setup, dims), flush=True)
    lat, pr, f0 = make_pair(q, dims, setup, "f64", pattern)
    lat.step(2)  # AA: ends on the natural layout
    got = lat.get_f()
    ref = R.run(pr, f0, 0, 2)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    lat.step(1)  # AA: ends on the swapped layout (get_f gathers)
    got = lat.get_f()
    ref = R.run(pr, ref, 2, 1)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    p, u = lat.macros()
    pr_, ur_ = R.macros(pr, ref, 3)
    assert rel_l2(u, ur_) <= 1e-12
    assert rel_l2(p, pr_) <= 1e-12
    lat.close()


@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("pattern", ("ab", "aa"))
@pytest.mark.parametrize("setup", sorted(SETUPS))
def test_fp32_matches_oracle(q, pattern, setup):
    dims = DIMS[0]
    print("case q=%d %s %s" % (q, pattern, setup), flush=True)
    lat, pr, f0 = make_pair(q, dims, setup, "f32", pattern, seed=1)
    lat.step(5)
    ref = R.run(pr, f0, 0, 5)
    p, u = lat.macros()
    pr_, ur_ = R.macros(pr, ref, 5)
    assert rel_l2(u, ur_) <= 1e-5
    assert rel_l2(p, pr_) <= 1e-5
    assert rel_l2(lat.get_f(), ref) <= 1e-6
    lat.close()


@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("pattern", ("ab", "aa"))
@pytest.mark.parametrize("setup", ("cavity_lid", "duct_pulsatile"))
@pytest.mark.parametrize("rounding", ("stochastic", "nearest"))
def test_fp16dev_matches_oracle(q, pattern, setup, rounding):
    dims = DIMS[0]
    print("case q=%d %s %s %s" % (q, pattern, setup, rounding), flush=True)
    faces, wall_u, F0, FA, FT = SETUPS[setup]
    s = rates(q)
    lat = lbm.Lattice(q, *dims, s, faces=FACESETS[faces], wall_u=wall_u, F0=F0, FA=FA, FT=FT,
                      storage="f16dev", pattern=pattern, f16_rounding=rounding)
    pr = R.problem(q, *dims, s, faces=FACESETS[faces], wall_u=wall_u, F0=F0, FA=FA, FT=FT)
    lat.set_f(inputs.random_populations(q, *dims, seed=2))
    f0 = lat.get_f()
    # one rounding error per stored value: below half an FP16 ulp (2^-11
    # relative) to nearest, below one ulp (2^-10) stochastically
    eps = 2.0 ** -11 if rounding == "nearest" else 2.0 ** -10
    lat.step(1)
    got = lat.get_f()
    ref = R.run(pr, f0, 0, 1)
    bound = eps * np.abs(ref) + 1e-6 * np.max(np.abs(ref))
    assert np.all(np.abs(got - ref) <= bound)
    # k steps: at most one rounding (eps of max|f|) per stored value and
    # step, each velocity component sums at most 10 populations; the
    # populations' relative L2 grows like sqrt(k).
    k = 4
    lat.step(k - 1)
    ref = R.run(pr, ref, 1, k - 1)
    got = lat.get_f()
    assert rel_l2(got, ref) <= 2.0 * np.sqrt(k) * eps
    p, u = lat.macros()
    pr_, ur_ = R.macros(pr, ref, k)
    fmax = np.max(np.abs(ref))
    ncomp = 18 if q == 26 else 10  # populations with c_x != 0
    assert np.max(np.abs(u - ur_)) <= k * ncomp * eps * fmax
    assert np.max(np.abs(p - pr_)) <= k * q * eps * fmax
    lat.close()



@pytest.mark.parametrize("q", (14, 18, 26))
def test_fp16dev_with_background_pressure_matches_oracle(q):
    """FP16 deviations are stored from the rest equilibrium 3 w_a p0 of the
    reference pressure p0 (one base per weight class).  With p0 = 0.3 every
    population carries a common part of 0.05-0.1 that is never rounded: the
    lattice starts at f_eq(p0, 0) exactly, and after steps from a random
    state its error against the oracle is a few FP16 roundings of the
    deviation f - 3 w p0, not of f."""
    dims = DIMS[0]
    faces, wall_u, F0, FA, FT = SETUPS["cavity_lid"]
    s = rates(q)
    p0 = 0.3
    kw = dict(faces=FACESETS[faces], wall_u=wall_u, F0=F0, FA=FA, FT=FT)
    lat = lbm.Lattice(q, *dims, s, storage="f16dev", pattern="aa", p0=p0, **kw)
    pr = R.problem(q, *dims, s, **kw)
    rest = R.init_eq(pr, 0, p0=p0)
    assert np.max(np.abs(lat.get_f() - rest)) <= 1e-7 * np.max(np.abs(rest))
    _, w, _, _, _, _ = R.lattice(q)
    base = (3.0 * w * p0).reshape(q, 1, 1, 1)
    lat.set_f(base + inputs.random_populations(q, *dims, seed=14))
    f0 = lat.get_f()
    k = 4
    lat.step(k)
    ref = R.run(pr, f0, 0, k)
    err = np.linalg.norm(lat.get_f() - ref) / np.linalg.norm(ref - base)
    assert err <= 2.0 * np.sqrt(k) * 2.0 ** -10, err
    lat.close()

@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("pattern", ("ab", "aa"))
@pytest.mark.parametrize("setup", ("duct_pulsatile", "symmix_force", "cavity_lid"))
@pytest.mark.parametrize("collision", ("mrt", "bgk"))
def test_fp16_steps_are_invariant_under_the_deviation_scale(q, pattern, setup, collision):
    """FP16 lattices store h = (f - 3 w p0) 2^s and step on h itself: every
    term of the collision linear in f, p, j or F carries 2^s and each product
    of two such quantities one factor 2^-s.  Raising s by one doubles every
    stored value exactly (while values stay in FP16's normal range; both
    rounding modes round the same mantissa), so the decoded populations
    after even and odd steps are the same bits for s = 12 and s = 13, with a
    background pressure, walls, moving walls, symmetry planes and a body
    force.  A term with a wrong power of the scale breaks this."""
    faces, wall_u, F0, FA, FT = SETUPS[setup]
    dims = DIMS[0]
    p0 = 0.3
    s = rates(q) if collision == "mrt" else np.full(q, 1.0 / 0.62)
    _, w, _, _, _, _ = R.lattice(q)
    f0 = (3.0 * w * p0).reshape(q, 1, 1, 1) + inputs.random_populations(q, *dims, seed=21)
    for rounding in ("nearest", "stochastic"):
        got = []
        for log2 in (12, 13):
            lat = lbm.Lattice(q, *dims, s, faces=FACESETS[faces], wall_u=wall_u, F0=F0, FA=FA,
                              FT=FT, storage="f16dev", pattern=pattern, collision=collision,
                              f16_rounding=rounding, p0=p0, f16_scale_log2=log2)
            lat.set_f(f0)
            start = lat.get_f()
            lat.step(5)
            got.append((start, lat.get_f()))
            lat.close()
        assert np.array_equal(got[0][0], got[1][0]), rounding
        assert np.all(np.isfinite(got[0][1]))
        assert not np.array_equal(got[0][1], got[0][0])
        assert np.array_equal(got[0][1], got[1][1]), rounding


def test_fp16_stochastic_rounding_is_unbiased():
    """Zero rates in a periodic box only move values, and a body force adds
    a Guo source of ~3e-7 per population and step -- far below half an FP16
    ulp of these populations (~1.5e-5).  Round-to-nearest loses the force
    entirely (stagnation); the stochastic store keeps N F of momentum per
    step on average."""
    q, dims = 18, (32, 16, 8)
    F = (2e-6, 0.0, 0.0)
    c, _, _, _, _, _ = R.lattice(q)
    gains = {}
    for rounding in ("stochastic", "nearest"):
        lat = lbm.Lattice(q, *dims, np.zeros(q), faces=FACESETS["periodic"], F0=F,
                          storage="f16dev", pattern="aa", f16_rounding=rounding)
        lat.set_f(inputs.random_populations(q, *dims, seed=12))
        f = lat.get_f()
        j0 = np.einsum("ad,azyx->d", c.astype(float), f)
        lat.step(400)
        j1 = np.einsum("ad,azyx->d", c.astype(float), lat.get_f())
        gains[rounding] = (j1 - j0)[0] / (400 * np.prod(dims) * F[0])
        lat.close()
    assert abs(gains["stochastic"] - 1.0) < 0.1, gains
    assert abs(gains["nearest"]) < 0.1, gains


def pull_permutation(q, dims, faces, f):
    """Zero-rate step in pull form, vectorised: population a at y comes from
    y - c_a (wrapped on periodic axes); beyond a wall it is y's own opposite
    population; beyond symmetry planes only it is the population mirrored
    in those planes, taken from the node reached along the planes."""
    c = velocities(q)
    opp = [int(np.nonzero((c == -c[a]).all(axis=1))[0][0]) for a in range(q)]
    nx, ny, nz = dims
    out = np.empty_like(f)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    own = [x, y, z]
    for a in range(q):
        src = [x - c[a, 0], y - c[a, 1], z - c[a, 2]]
        wall = np.zeros(x.shape, bool)
        mask = np.zeros(x.shape, int)
        for d, n in enumerate(dims):
            lo, hi = src[d] < 0, src[d] >= n
            kinds = (faces[2 * d], faces[2 * d + 1])
            if kinds[0] == "periodic":
                src[d] = src[d] % n
                continue
            for side, kind in ((lo, kinds[0]), (hi, kinds[1])):
                if kind == "wall":
                    wall |= side
                else:  # symmetry plane
                    mask |= np.where(side, 1 << d, 0)
                    src[d] = np.where(side, own[d], src[d])
            src[d] = np.clip(src[d], 0, n - 1)
        moved = np.empty(x.shape)
        for m in range(8):
            cm = c[a] * np.array([-1 if m >> d & 1 else 1 for d in range(3)])
            b = int(np.nonzero((c == cm).all(axis=1))[0][0])
            sel = mask == m
            moved[sel] = f[b][src[2][sel], src[1][sel], src[0][sel]]
        out[a] = np.where(wall, f[opp[a]], moved)
    return out


@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("storage", ("f64", "f32", "f16dev"))
@pytest.mark.parametrize("pattern", ("ab", "aa"))
@pytest.mark.parametrize("faces", sorted(FACESETS))
def test_zero_rates_bit_exact_permutation(q, storage, pattern, faces):
    dims = (37, 19, 11)
    fs = FACESETS[faces]
    lat = lbm.Lattice(q, *dims, np.zeros(q), faces=fs, storage=storage, pattern=pattern)
    lat.set_f(inputs.random_populations(q, *dims, seed=3))
    f = lat.get_f()
    for k in range(3):
        lat.step(1)
        f = pull_permutation(q, dims, fs, f)
        assert np.array_equal(lat.get_f(), f), "step %d" % (k + 1)
    lat.close()


@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("storage", ("f64", "f32", "f16dev"))
@pytest.mark.parametrize("setup", sorted(SETUPS))
def test_aa_equals_ab_bit_exact(q, storage, setup):
    out = {}
    for pattern in ("ab", "aa"):
        lat, _, _ = make_pair(q, DIMS[0], setup, storage, pattern, seed=4)
        lat.step(5)
        out[pattern] = (lat.get_f(), lat.macros())
        lat.close()
    assert np.array_equal(out["ab"][0], out["aa"][0])
    assert np.array_equal(out["ab"][1][0], out["aa"][1][0])
    assert np.array_equal(out["ab"][1][1], out["aa"][1][1])


@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("storage,pattern,split", [
    ("f64", "ab", 3), ("f32", "aa", 3), ("f32", "aa", 4), ("f16dev", "aa", 4), ("f32", "ab", 2)])
def test_checkpoint_restore_bit_exact(q, storage, pattern, split):
    setup = "duct_pulsatile"
    ref, _, f0 = make_pair(q, DIMS[0], setup, storage, pattern, seed=5)
    ref.step(8)
    want = ref.get_f()
    a, _, _ = make_pair(q, DIMS[0], setup, storage, pattern, seed=5)
    a.step(split)
    ck, t = a.get_f(), a.time
    a.close()
    b, _, _ = make_pair(q, DIMS[0], setup, storage, pattern, seed=6)
    b.set_f(ck)
    b.set_time(t)
    b.step(8 - split)
    assert np.array_equal(b.get_f(), want)
    ref.close()
    b.close()


@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("storage", ("f64", "f32"))
def test_init_fields_match_oracle(q, storage):
    dims = (21, 13, 9)
    faces, wall_u, F0, FA, FT = SETUPS["duct_pulsatile"]
    p, u = inputs.random_fields(*dims, seed=7)
    lat = lbm.Lattice(q, *dims, rates(q), faces=FACESETS[faces], F0=F0, FA=FA, FT=FT,
                      storage=storage)
    lat.init_fields(p, u)
    pr = R.problem(q, *dims, rates(q), faces=FACESETS[faces], F0=F0, FA=FA, FT=FT)
    ref = R.init_eq(pr, 0, p=p, u=u)
    got = lat.get_f()
    tol = 1e-15 if storage == "f64" else 1e-7  # a few ulps of differing operation order
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))
    # the recovered velocity is the one put in (Eq. (hgl))
    _, ug = lat.macros()
    assert np.max(np.abs(ug - u)) <= (1e-16 if storage == "f64" else 1e-8)
    lat.close()


@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("pattern", ("ab", "aa"))
def test_monitor_mass_and_residual(q, pattern):
    dims = DIMS[0]
    setup = "cavity_lid"
    faces, wall_u, F0, FA, FT = SETUPS[setup]
    lat = lbm.Lattice(q, *dims, rates(q), faces=FACESETS[faces], wall_u=wall_u,
                      storage="f64", pattern=pattern, monitor_every=3)
    pr = R.problem(q, *dims, rates(q), faces=FACESETS[faces], wall_u=wall_u)
    f0 = inputs.random_populations(q, *dims, seed=8)
    lat.set_f(f0)
    lat.step(3)  # first snapshot at t = 3
    lat.step(3)  # second at t = 6
    r = lat.residual()
    m = lat.mass()
    f3 = R.run(pr, f0, 0, 3)
    f6 = R.run(pr, f3, 3, 3)
    _, u3 = R.macros(pr, f3, 3)
    _, u6 = R.macros(pr, f6, 6)
    r_ref = np.sum(np.abs(u6 - u3)) / (3 * np.sum(np.abs(u6)))
    assert abs(r - r_ref) <= 1e-12 * r_ref
    assert abs(m - f6.sum()) <= 1e-13 * np.abs(f6).sum()
    # the paper's own criterion (Eqs. (sc), (cr), (cavity_creterion)): the
    # change over the lag, not divided by it
    rc, lag = lat.residual_change()
    assert lag == 3
    assert abs(rc - 3 * r_ref) <= 1e-12 * 3 * r_ref
    lat.close()


def test_nonfinite_is_reported():
    """A NaN injected through set_f surfaces as LBM_ENONFINITE (host-forced)."""
    q, dims = 18, (16, 8, 8)
    lat = lbm.Lattice(q, *dims, rates(q), faces=FACESETS["cavity"], monitor_every=2)
    f = inputs.random_populations(q, *dims, seed=9)
    f[3, 4, 4, 4] = np.nan
    lat.set_f(f)
    lat.step(2)
    with pytest.raises(lbm.LbmError) as e:
        lat.residual()
    assert e.value.code == -4
    lat.close()



@pytest.mark.parametrize("storage", ("f64", "f32", "f16dev"))
def test_first_residual_of_a_state_ignores_the_stale_snapshot(storage):
    """The monitor's first pass over a state (after create, set_f,
    init_fields or set_time) has nothing to difference against: the
    residual is +inf, and only u and the mass decide LBM_ENONFINITE, not
    whatever the snapshot buffer held.  Here it holds the NaN velocity of a
    replaced state; fresh device memory can hold any bit pattern as well,
    which once made an FP32 lattice report a finite state as non-finite."""
    q, dims = 14, (12, 10, 8)
    lat = lbm.Lattice(q, *dims, rates(q), faces=FACESETS["cavity"], storage=storage)
    f = inputs.random_populations(q, *dims, seed=12)
    bad = f.copy()
    bad[1, 2, 3, 4] = np.nan
    lat.set_f(bad)
    lat.monitor()
    with pytest.raises(lbm.LbmError) as e:
        lat.residual()
    assert e.value.code == -4
    lat.set_f(f)
    lat.monitor()
    assert lat.residual() == np.inf
    lat.step(4)
    lat.monitor()
    r = lat.residual()
    assert np.isfinite(r) and r > 0
    lat.close()

# ---- full-size workload: 128^3 lid-driven cavity, D3Q18, FP32, AA ---------

def cavity128(q=18, storage="f32"):
    nu = 0.1 * 128 / 1000.0
    s = svec(q, 1.0 / (3 * nu + 0.5))
    lat = lbm.Lattice(q, 128, 128, 128, s, faces=FACESETS["cavity"], wall_u={"+z": (0.1, 0, 0)},
                      storage=storage, pattern="aa")
    pr = R.problem(q, 128, 128, 128, s, faces=FACESETS["cavity"], wall_u={"+z": (0.1, 0, 0)})
    return lat, pr


def test_full_size_cavity_random_state_two_steps():
    lat, pr = cavity128()
    f0 = inputs.random_populations(18, 128, 128, 128, seed=10)
    lat.set_f(f0)
    f0 = lat.get_f()
    lat.step(2)
    ref = R.run(pr, f0, 0, 2)
    got = lat.get_f()
    assert rel_l2(got, ref) <= 1e-6
    p, u = lat.macros()
    pr_, ur_ = R.macros(pr, ref, 2)
    assert rel_l2(u, ur_) <= 1e-5
    lat.close()


def test_full_size_cavity_properties_after_2000_steps():
    """Lid along +x: mirror symmetry in y (u_y odd, u_x and u_z even) and
    conserved mass (tangential lid) hold at any size."""
    lat, _ = cavity128()
    lat.monitor()
    m0 = lat.mass()
    lat.step(2000)
    lat.monitor()
    m1 = lat.mass()
    p, u = lat.macros()
    assert np.all(np.isfinite(u))
    umax = np.max(np.abs(u))
    assert 0.01 < umax < 0.2
    mir = u[:, :, ::-1, :]
    assert np.max(np.abs(u[0] - mir[0])) <= 1e-5 * umax
    assert np.max(np.abs(u[1] + mir[1])) <= 1e-5 * umax
    assert np.max(np.abs(u[2] - mir[2])) <= 1e-5 * umax
    assert abs(m1 - m0) <= 1e-6 * 128 ** 3 * 0.01
    lat.close()


@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("storage", ("f64", "f32"))
@pytest.mark.parametrize("pattern", ("ab", "aa"))
@pytest.mark.parametrize("setup", ("duct_pulsatile", "cavity_lid"))
def test_bgk_matches_oracle(q, storage, pattern, setup):
    """The LBGK collision (S = I/tau, evaluated without transforms) against
    the oracle's MRT step with all rates 1/tau (the paper's reduction)."""
    faces, wall_u, F0, FA, FT = SETUPS[setup]
    dims = DIMS[0]
    s = np.full(q, 1.0 / 0.62)
    lat = lbm.Lattice(q, *dims, s, faces=FACESETS[faces], wall_u=wall_u, F0=F0, FA=FA, FT=FT,
                      storage=storage, pattern=pattern, collision="bgk")
    pr = R.problem(q, *dims, s, faces=FACESETS[faces], wall_u=wall_u, F0=F0, FA=FA, FT=FT)
    lat.set_f(inputs.random_populations(q, *dims, seed=13))
    f0 = lat.get_f()
    lat.step(3)
    ref = R.run(pr, f0, 0, 3)
    got = lat.get_f()
    if storage == "f64":
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    else:
        p, u = lat.macros()
        _, ur = R.macros(pr, ref, 3)
        assert rel_l2(u, ur) <= 1e-5
    lat.close()


@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("pattern", ("ab", "aa"))
@pytest.mark.parametrize("setup", ("duct_pulsatile", "cavity_lid"))
def test_fp16dev_bgk_matches_oracle(q, pattern, setup):
    """The LBGK collision on FP16 deviations (rounded to nearest) against the
    oracle's MRT step with all rates 1/tau, under the rounding bounds of the
    MRT test on the same storage: the even and the odd AA step each once."""
    faces, wall_u, F0, FA, FT = SETUPS[setup]
    dims = DIMS[0]
    print("case q=%d %s %s" % (q, pattern, setup), flush=True)
    s = np.full(q, 1.0 / 0.62)
    lat = lbm.Lattice(q, *dims, s, faces=FACESETS[faces], wall_u=wall_u, F0=F0, FA=FA, FT=FT,
                      storage="f16dev", pattern=pattern, collision="bgk",
                      f16_rounding="nearest")
    pr = R.problem(q, *dims, s, faces=FACESETS[faces], wall_u=wall_u, F0=F0, FA=FA, FT=FT)
    lat.set_f(inputs.random_populations(q, *dims, seed=17))
    f0 = lat.get_f()
    eps = 2.0 ** -11
    lat.step(1)
    ref = R.run(pr, f0, 0, 1)
    got = lat.get_f()
    assert np.all(np.abs(got - ref) <= eps * np.abs(ref) + 1e-6 * np.max(np.abs(ref)))
    k = 4
    lat.step(k - 1)
    ref = R.run(pr, ref, 1, k - 1)
    assert rel_l2(lat.get_f(), ref) <= 2.0 * np.sqrt(k) * eps
    p, u = lat.macros()
    pr_, ur_ = R.macros(pr, ref, k)
    fmax = np.max(np.abs(ref))
    ncomp = 18 if q == 26 else 10
    assert np.max(np.abs(u - ur_)) <= k * ncomp * eps * fmax
    assert np.max(np.abs(p - pr_)) <= k * q * eps * fmax
    lat.close()


DEGENERATE = [(1, 1, 1), (1, 5, 4), (6, 1, 3), (5, 4, 1), (2, 2, 2), (257, 1, 2), (3, 2, 300)]
DEGENERATE_FACES = {
    "periodic": ("periodic",) * 6,
    "walls": ("wall",) * 6,
    "mixed": ("wall", "symmetry", "periodic", "periodic", "symmetry", "wall"),
}


@pytest.mark.parametrize("q", (14, 18, 26))
@pytest.mark.parametrize("pattern", ("ab", "aa"))
@pytest.mark.parametrize("faces", sorted(DEGENERATE_FACES))
@pytest.mark.parametrize("dims", DEGENERATE, ids=lambda d: "x".join(map(str, d)))
def test_degenerate_shapes_match_oracle(q, pattern, faces, dims):
    """Axes of one or two nodes (every link of the axis wraps onto, bounces
    at or mirrors into the node itself), rows longer than one 256-wide tile,
    long z: FP64 element-wise against the oracle for three steps (both AA
    parities), with a moving wall and a body force."""
    fs = DEGENERATE_FACES[faces]
    wall_u = {"+z": (0.05, 0.02, 0.0), "-x": (0.0, 0.03, 0.01)}
    F0 = (2e-5, -1e-5, 1e-5)
    lat = lbm.Lattice(q, *dims, rates(q), faces=fs, wall_u=wall_u, F0=F0, storage="f64",
                      pattern=pattern)
    pr = R.problem(q, *dims, rates(q), faces=fs, wall_u=wall_u, F0=F0)
    lat.set_f(inputs.random_populations(q, *dims, seed=21))
    f = lat.get_f()
    scale = np.max(np.abs(f))
    for t in range(1, 4):
        lat.step(1)
        f = R.run(pr, f, t - 1, 1)
        assert np.max(np.abs(lat.get_f() - f)) <= 1e-13 * scale, t
    lat.close()


def test_zero_steps_change_nothing():
    q = 18
    lat = lbm.Lattice(q, 9, 8, 7, rates(q), faces=FACESETS["cavity"], storage="f32")
    lat.set_f(inputs.random_populations(q, 9, 8, 7, seed=22))
    f0 = lat.get_f()
    lat.step(0)
    assert lat.time == 0 and np.array_equal(lat.get_f(), f0)
    b = lbm.Batch(lat.stream)
    b.step(5)  # an empty batch does nothing
    b.add(lat, 3)
    b.step(0)
    assert lat.time == 0 and np.array_equal(lat.get_f(), f0)
    b.close()
    lat.close()


@pytest.mark.parametrize("nbytes", (16 * 1000003, 16 * ((200 << 20) // 16 + 12345)))
def test_copy_probe_copies_in_either_order(nbytes):
    """The bandwidth reference is a real copy in both workgroup orders: a
    ragged 16 MB buffer (dispatch order) and a ragged 200 MB one (400 MB
    touched: one contiguous range per XCD) arrive intact, and a copy in
    place leaves the buffer as it was."""
    import torch
    gen = torch.Generator(device="cuda").manual_seed(3)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=gen)
    dst = torch.zeros_like(src)
    ref = src.clone()
    stream = torch.cuda.current_stream().cuda_stream
    lbm.copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, 2, stream)
    lbm.copy_probe(src.data_ptr(), src.data_ptr(), nbytes, 1, stream)
    torch.cuda.synchronize()
    assert torch.equal(dst, ref)
    assert torch.equal(src, ref)


@pytest.mark.parametrize("q,elem", [(14, 4), (18, 2), (18, 4), (18, 8), (26, 4)])
def test_pattern_probe_moves_the_data_of_both_aa_patterns(q, elem):
    """The access-pattern reference moves data, not nothing, over a ragged
    periodic lattice (partial tiles in x and y): the even pattern puts the
    value of slot a into the slot of -c_a at the same node, the odd pattern
    the value of slot abar at n - c_a into slot a at n + c_a; the pad beyond
    the node count is untouched, and a second even pass restores the
    buffer."""
    import torch
    c = velocities(q)
    opp = [int(np.flatnonzero((c == -c[a]).all(axis=1))[0]) for a in range(q)]
    nx, ny, nz = 70, 9, 5
    nodes = nx * ny * nz
    stride = (nodes + 63) // 64 * 64 + 1088
    dt = {2: np.uint16, 4: np.uint32, 8: np.uint64}[elem]
    gen = torch.Generator(device="cuda").manual_seed(q * 10 + elem)
    buf = torch.randint(0, 256, (q * stride * elem,), dtype=torch.uint8, device="cuda",
                        generator=gen)
    ref = buf.clone()
    a0 = ref.cpu().numpy().view(dt).reshape(q, stride)
    stream = torch.cuda.current_stream().cuda_stream
    lbm.pattern_probe(buf.data_ptr(), q, elem, (nx, ny, nz), stride, False, 1, stream)
    torch.cuda.synchronize()
    b_ = buf.cpu().numpy().view(dt).reshape(q, stride)
    for a in range(q):
        assert np.array_equal(b_[opp[a], :nodes], a0[a, :nodes]), a
        assert np.array_equal(b_[a, nodes:], a0[a, nodes:]), a
    lbm.pattern_probe(buf.data_ptr(), q, elem, (nx, ny, nz), stride, False, 1, stream)
    torch.cuda.synchronize()
    assert torch.equal(buf, ref)
    lbm.pattern_probe(buf.data_ptr(), q, elem, (nx, ny, nz), stride, True, 1, stream)
    torch.cuda.synchronize()
    b_ = buf.cpu().numpy().view(dt).reshape(q, stride)
    for a in range(q):
        # f'[a](m) = f[abar](m - 2 c_a), periodic; arrays indexed [z, y, x]
        src_ = a0[opp[a], :nodes].reshape(nz, ny, nx)
        want = np.roll(src_, shift=(2 * c[a][2], 2 * c[a][1], 2 * c[a][0]), axis=(0, 1, 2))
        assert np.array_equal(b_[a, :nodes].reshape(nz, ny, nx), want), a
        assert np.array_equal(b_[a, nodes:], a0[a, nodes:]), a
    with pytest.raises(lbm.LbmError):
        lbm.pattern_probe(buf.data_ptr(), q, 3, (nx, ny, nz), stride, False, 1, stream)
    with pytest.raises(lbm.LbmError):
        lbm.pattern_probe(buf.data_ptr(), q, elem, (nx, ny, nz), nodes - 1, False, 1, stream)

"""Batched execution (one launch per time step over many lattices) through
the C ABI: alone == in the mix (bit-exact), batch == single-lattice kernel,
batch == oracle within the FP32 tolerance, step budgets, continuous
admission/retirement, tile-shape invariance, batched monitors."""
import numpy as np
import pytest

from helpers import svec
from oracle import runner as R
from paper_1503_03337_amd import inputs
from paper_1503_03337_amd import lbm

pytestmark = pytest.mark.gpu

MEMBERS = [
    # q, dims, storage, faces, wall_u, F0, FA, FT
    (14, (24, 17, 13), "f32", ("periodic", "periodic", "wall", "wall", "wall", "wall"),
     None, (2e-5, 0, 0), (0, 0, 0), 0.0),
    (18, (19, 23, 11), "f16dev", ("wall",) * 6, {"+z": (0.1, 0, 0)}, (0, 0, 0), (0, 0, 0), 0.0),
    (18, (40, 9, 9), "f32", ("periodic", "periodic", "wall", "wall", "wall", "wall"),
     {"-y": (0.01, 0, 0)}, (1e-5, 0, 0), (2e-5, 0, 0), 9.0),
    (14, (13, 29, 7), "f16dev", ("wall",) * 6, {"+z": (0.05, 0.02, 0)}, (0, 0, 0), (0, 0, 0),
     0.0),
    (18, (300, 4, 3), "f32", ("periodic",) * 6, None, (1e-5, 1e-5, 0), (0, 0, 0), 0.0),
    # symmetry planes (Sec. 4.3 half cavity; an x-face plane)
    (18, (21, 15, 8), "f32", ("wall",) * 5 + ("symmetry",), {"+y": (0.1, 0, 0)}, (0, 0, 0),
     (0, 0, 0), 0.0),
    (14, (17, 12, 10), "f16dev", ("symmetry", "wall", "periodic", "periodic", "wall", "symmetry"),
     {"+x": (0, 0.04, 0.02)}, (1e-5, 0, 0), (0, 0, 0), 0.0),
    # the 26-velocity model (Appendix B's closing paragraph)
    (26, (21, 14, 9), "f32", ("wall",) * 6, {"+z": (0.08, 0, 0)}, (0, 0, 0), (0, 0, 0), 0.0),
    (26, (15, 11, 13), "f16dev", ("periodic", "periodic", "wall", "wall", "wall", "symmetry"),
     {"-y": (0.02, 0, 0.01)}, (2e-5, 0, 0), (1e-5, 0, 0), 11.0),
]


def rates(q, k):
    sn = 1.3 + 0.1 * k if k < 7 else 1.45 + 0.2 * (k - 7)  # s_nu < 2 for every member
    return svec(q, sn) + np.linspace(-0.02, 0.02, q)


def build(k, seed, monitor_every=0):
    q, dims, storage, faces, wall_u, F0, FA, FT = MEMBERS[k]
    lat = lbm.Lattice(q, *dims, rates(q, k), faces=faces, wall_u=wall_u, F0=F0, FA=FA, FT=FT,
                      storage=storage, pattern="aa", monitor_every=monitor_every)
    lat.set_f(inputs.random_populations(q, *dims, seed=seed))
    return lat


def run_alone(k, nsteps, seed, via_batch=True):
    lat = build(k, seed)
    if via_batch:
        b = lbm.Batch(lat.stream)
        b.add(lat, nsteps)
        b.step(nsteps)
        b.close()
    else:
        lat.step(nsteps)
    f = lat.get_f()
    lat.close()
    return f


def test_alone_equals_mix_bit_exact():
    budgets = [7, 5, 9, 6, 8, 10, 4, 6, 9]
    alone = [run_alone(k, budgets[k], 100 + k) for k in range(len(MEMBERS))]
    lats = [build(k, 100 + k) for k in range(len(MEMBERS))]
    b = lbm.Batch(lats[0].stream)
    for k, lat in enumerate(lats):
        b.add(lat, budgets[k])
    b.step(4)
    b.step(10)  # members stop at their own budgets
    for k, lat in enumerate(lats):
        assert b.remaining(lat) == 0
        assert lat.time == budgets[k]
        assert np.array_equal(lat.get_f(), alone[k]), "member %d" % k
    b.close()
    for lat in lats:
        lat.close()


def test_batch_equals_single_kernel():
    """The batched step and the single-lattice step do the same arithmetic
    per node: the same populations bit for bit."""
    for k in range(len(MEMBERS)):
        a = run_alone(k, 6, 200 + k, via_batch=True)
        s = run_alone(k, 6, 200 + k, via_batch=False)
        assert np.array_equal(a, s), "member %d" % k


def test_batch_matches_oracle():
    for k in range(len(MEMBERS)):
        q, dims, storage, faces, wall_u, F0, FA, FT = MEMBERS[k]
        lat = build(k, 300 + k)
        f0 = lat.get_f()
        b = lbm.Batch(lat.stream)
        b.add(lat, 5)
        b.step(5)
        pr = R.problem(q, *dims, rates(q, k), faces=faces, wall_u=wall_u, F0=F0, FA=FA, FT=FT)
        ref = R.run(pr, f0, 0, 5)
        _, u = lat.macros()
        _, ur = R.macros(pr, ref, 5)
        if storage == "f32":
            assert np.linalg.norm(u - ur) <= 1e-5 * np.linalg.norm(ur), "member %d" % k
        else:  # FP16: at most one stochastic rounding (2^-10) per value and step
            assert np.max(np.abs(u - ur)) <= 5 * 10 * 2.0 ** -10 * np.max(np.abs(ref)), k
        b.close()
        lat.close()


def test_continuous_admission_and_retirement():
    """Members join and leave between calls; everyone's result equals its
    alone run."""
    alone = {k: run_alone(k, 12, 400 + k) for k in (0, 1, 2)}
    l0, l1, l2 = (build(k, 400 + k) for k in (0, 1, 2))
    b = lbm.Batch(l0.stream)
    b.add(l0, 12)
    b.step(3)
    b.add(l1, 12)   # arrives while l0 runs
    b.step(5)
    b.add(l2, 12)
    b.step(4)       # l0 done (12)
    assert b.remaining(l0) == 0
    b.remove(l0)
    assert len(b) == 2
    b.step(100)     # l1 (9 left) and l2 (8 left) finish
    for lat, k in ((l0, 0), (l1, 1), (l2, 2)):
        assert lat.time == 12
        assert np.array_equal(lat.get_f(), alone[k]), "member %d" % k
    b.close()
    for lat in (l0, l1, l2):
        lat.close()


@pytest.mark.parametrize("tile", [(16, 16), (64, 4), (32, 8), (7, 9), (1, 1)])
def test_tile_shape_does_not_change_results(tile):
    """Row tiles of any shape give the automatic (flat) mapping's result."""
    ref = run_alone(2, 5, 500)
    lat = build(2, 500)
    b = lbm.Batch(lat.stream)
    b.add(lat, 5)
    b.set_tile(lat, *tile)
    b.step(5)
    assert np.array_equal(lat.get_f(), ref)
    b.close()
    lat.close()


def test_batch_monitor_matches_single_monitor():
    """Members with a monitor (monitor_every > 0) get the same residual and
    mass as the single-lattice monitor; members without one are skipped."""
    lats = [build(k, 600 + k, monitor_every=1000) for k in range(3)]
    plain = build(3, 699)
    b = lbm.Batch(lats[0].stream)
    for lat in lats + [plain]:
        b.add(lat, 50)
    b.step(10)
    b.monitor()
    b.step(10)
    b.monitor()
    with pytest.raises(lbm.LbmError):
        plain.residual()  # never monitored
    for k, lat in enumerate(lats):
        r, m = lat.residual(), lat.mass()
        # same state through the single-lattice monitor
        ref = build(k, 600 + k)
        ref.step(10)
        ref.monitor()
        ref.step(10)
        ref.monitor()
        rr, mr = ref.residual(), ref.mass()
        ref.close()
        assert abs(r - rr) <= 1e-6 * abs(rr), (k, r, rr)
        assert abs(m - mr) <= 1e-9 * max(1.0, abs(mr)), (k, m, mr)
    b.close()
    for lat in lats + [plain]:
        lat.close()



def test_batch_monitor_first_residual_ignores_the_stale_snapshot():
    """As for single lattices: the batch monitor's first pass over a state
    gives residual +inf whatever the snapshot buffer held (here the NaN
    velocity of a replaced state); a NaN in the state itself is reported."""
    lat = build(0, 610, monitor_every=1000)
    f = lat.get_f()
    bad = f.copy()
    bad[2, 1, 1, 1] = np.nan
    lat.set_f(bad)
    b = lbm.Batch(lat.stream)
    b.add(lat, 50)
    b.monitor()
    with pytest.raises(lbm.LbmError) as e:
        lat.residual()
    assert e.value.code == -4
    lat.set_f(f)
    b.monitor()
    assert lat.residual() == np.inf
    b.step(4)
    b.monitor()
    r = lat.residual()
    assert np.isfinite(r) and r > 0
    b.close()
    lat.close()


def test_closing_a_member_leaves_the_batch():
    """Destroying a member removes it from its batch; the batch goes on with
    the others (bit for bit as single lattices), and removing the closed
    lattice afterwards only drops it from the binding's list."""
    a, c = build(0, 620), build(2, 621)
    ref = build(2, 621)
    b = lbm.Batch(a.stream)
    b.add(a, 100)
    b.add(c, 100)
    b.step(3)
    a.close()
    assert len(b) == 1
    b.remove(a)
    b.step(4)
    ref.step(7)
    assert np.array_equal(c.get_f(), ref.get_f())
    b.close()
    c.close()
    ref.close()

def test_batch_rejects_unsupported_members():
    q = 18
    lat = lbm.Lattice(q, 8, 8, 8, svec(q, 1.2), storage="f64")
    b = lbm.Batch(lat.stream)
    with pytest.raises(lbm.LbmError):
        b.add(lat, 10)
    lat2 = lbm.Lattice(q, 8, 8, 8, svec(q, 1.2), storage="f32", pattern="ab")
    with pytest.raises(lbm.LbmError):
        b.add(lat2, 10)
    b.close()
    lat.close()
    lat2.close()


def test_mixed_parity_single_steps_and_alignment():
    """Members at different AA parities: single-step calls keep parity in the
    launch class; multi-step calls let the out-of-step member sit out one
    substep.  Either way every member equals its alone run."""
    alone = {k: run_alone(k, 9, 700 + k) for k in (0, 1, 2, 3)}
    lats = {k: build(k, 700 + k) for k in (0, 1, 2, 3)}
    b = lbm.Batch(lats[0].stream)
    b.add(lats[0], 9)
    b.add(lats[1], 9)
    b.step(1)             # 0 and 1 at odd parity
    b.add(lats[2], 9)     # even parity
    b.step(1)             # n == 1: both parities in one call
    b.step(1)
    b.add(lats[3], 9)     # even parity again, others mixed
    b.step(4)             # aligned: out-of-step members skip a substep
    b.step(100)
    for k, lat in lats.items():
        assert lat.time == 9, (k, lat.time)
        assert np.array_equal(lat.get_f(), alone[k]), "member %d" % k
    b.close()
    for lat in lats.values():
        lat.close()


def test_large_class_two_tiles_per_workgroup_bit_exact():
    """A class of at least 16384 tiles runs two tiles per workgroup; each
    member still equals its alone run (one tile per workgroup) bit for bit,
    including a ragged last chunk (odd tile counts)."""
    q, steps = 18, 5
    # members below the solo size (2^20 nodes), 256-node tiles of the
    # automatic mapping: 3456 + 3529 + 3420 + 3456 + 3456 = 17317
    dims = [(96, 96, 96), (96, 97, 97), (96, 96, 95), (95, 96, 97), (97, 95, 96)]
    s = svec(q, 1.6) + np.linspace(-0.02, 0.02, q)

    def make(k):
        nx, ny, nz = dims[k]
        lat = lbm.Lattice(q, nx, ny, nz, s, faces=("wall",) * 6, wall_u={"+z": (0.1, 0, 0)},
                          storage="f32", pattern="aa")
        lat.init_fields(np.zeros((nz, ny, nx)), inputs.random_fields(nx, ny, nz, seed=800 + k)[1])
        return lat

    alone = []
    for k in range(len(dims)):
        lat = make(k)
        b = lbm.Batch(lat.stream)
        b.add(lat, steps)
        b.step(steps)
        b.close()
        alone.append(lat.macros()[1])
        lat.close()
    lats = [make(k) for k in range(len(dims))]
    b = lbm.Batch(lats[0].stream)
    for lat in lats:
        b.add(lat, steps)
    b.step(steps)
    b.close()
    for k, lat in enumerate(lats):
        assert np.array_equal(lat.macros()[1], alone[k]), k
        lat.close()


def test_cavity_batch_256_full_size():
    """The 256-cavity batch (edge U{24..96}, Re U[100,1000], D3Q14/D3Q18,
    FP32, seed 0) in the launch configuration the benchmark times (one
    launch per class and step, the large classes two tiles per workgroup):
    the five smallest members match the FP64 oracle after 6 steps from a
    random state (FP32 tolerance), and every member conserves its mass (the
    lids are tangential) to FP32 rounding."""
    from paper_1503_03337_amd import params
    spec = inputs.cavity_batch(256, seed=0)
    lats = []
    for k, c in enumerate(spec):
        L = c["edge"]
        cfg = params.cavity(c["q"], L, c["Re"], lid=c["lid"])
        lat = lbm.Lattice(c["q"], L, L, L, cfg["s_vec"], faces=cfg["faces"],
                          wall_u=cfg["wall_u"], storage="f32", pattern="aa")
        lats.append((lat, cfg))
    b = lbm.Batch(lats[0][0].stream)
    small = sorted(range(len(spec)), key=lambda k: spec[k]["edge"])[:5]
    start = {}
    for k, (lat, cfg) in enumerate(lats):
        if k in small:
            L = spec[k]["edge"]
            lat.set_f(inputs.random_populations(cfg["model"], L, L, L, seed=900 + k))
            start[k] = lat.get_f()
        b.add(lat, 6)
    mass0 = [float(np.sum(lat.get_f(), dtype=np.float64)) for lat, _ in lats]
    b.step(6)
    b.close()
    for k, (lat, cfg) in enumerate(lats):
        assert lat.time == 6
        f = lat.get_f()
        m = float(np.sum(f, dtype=np.float64))
        # (members started at rest have p0 = 0, all populations 0: the
        # scale is the populations' magnitude, not the mass)
        assert abs(m - mass0[k]) <= 1e-6 * float(np.sum(np.abs(f))), (k, m, mass0[k])
        if k in small:
            L = spec[k]["edge"]
            pr = R.problem(cfg["model"], L, L, L, cfg["s_vec"], faces=cfg["faces"],
                           wall_u=cfg["wall_u"])
            ref = R.run(pr, start[k], 0, 6)
            _, u = lat.macros()
            _, ur = R.macros(pr, ref, 6)
            assert np.linalg.norm(u - ur) <= 1e-5 * np.linalg.norm(ur), k
    for lat, _ in lats:
        lat.close()


def test_batch_beyond_384mb_equals_single_lattices():
    """A batch whose members hold more than 384 MB hands the XCDs chunks of
    workgroups in turn (another order than a smaller batch or a single
    lattice uses).  The order changes no result: six D3Q18 members below the
    solo size (17.7k tiles together: the chunked kernel) and a ragged D3Q14
    member (one tile per workgroup), 445 MB together, equal single lattices
    bit for bit after an even and an odd step and one more."""
    members = [(18, (96, 96, 96 - k), {"+z": (0.05, 0.01 * k, 0.0)}) for k in range(6)]
    members.append((14, (95, 97, 93), {"+z": (0.0, 0.04, 0.0)}))
    lats, singles = [], []
    for k, (q, dims, lid) in enumerate(members):
        for group in (lats, singles):
            lat = lbm.Lattice(q, *dims, rates(q, k % 6), faces=("wall",) * 6, wall_u=lid,
                              storage="f32", pattern="aa")
            lat.set_f(inputs.random_populations(q, *dims, seed=640 + k))
            group.append(lat)
    total = sum(lbm.footprint_bytes(l.q, l.nx, l.ny, l.nz, storage="f32", pattern="aa")
                for l in lats)
    assert total > 384 << 20
    b = lbm.Batch(lats[0].stream)
    for lat in lats:
        b.add(lat, 100)
    b.step(2)
    b.step(1)
    for lat, single in zip(lats, singles):
        single.step(3)
        assert np.array_equal(lat.get_f(), single.get_f())
    b.close()
    for lat in lats + singles:
        lat.close()


def test_solo_and_classed_members_equal_single_lattices():
    """Members of 2^20 nodes or more step on their own with the
    single-lattice kernels, interleaved with the class launches of the small
    members: a mix of large members (FP32 and FP16, D3Q18 and D3Q14, forced,
    one out of AA parity) and small ones, stepped in uneven calls, equals
    single lattices bit for bit."""
    spec = [(18, (104, 104, 100), "f32", (1e-5, 0, 0)), (14, (101, 101, 103), "f16dev", (0, 0, 0)),
            (18, (24, 20, 18), "f32", (0, 0, 0)), (14, (17, 23, 19), "f16dev", (2e-5, 0, 0)),
            (18, (30, 9, 11), "f16dev", (0, 0, 0))]
    lats, singles = [], []
    for k, (q, dims, storage, F0) in enumerate(spec):
        for group in (lats, singles):
            lat = lbm.Lattice(q, *dims, rates(q, k), faces=("wall",) * 6,
                              wall_u={"+z": (0.05, 0.0, 0.0)}, F0=F0, storage=storage,
                              pattern="aa")
            lat.set_f(inputs.random_populations(q, *dims, seed=660 + k))
            if k in (1, 3):
                lat.step(1)
            group.append(lat)
    assert lats[0].N >= 1 << 20 and lats[1].N >= 1 << 20
    b = lbm.Batch(lats[0].stream)
    for lat in lats:
        b.add(lat, 40)
    for n in (3, 1, 5, 2):
        b.step(n)
    for lat, single in zip(lats, singles):
        single.step(lat.time - single.time)
        assert np.array_equal(lat.get_f(), single.get_f()), (lat.q, lat.nx)
    b.close()
    for lat in lats + singles:
        lat.close()


def test_large_single_lattice_orders_agree():
    """Beyond 384 MB a single lattice gives the XCDs chunks of 4 rows in turn
    and a batch chunks of 64 workgroups: a 180^3 D3Q18 FP32 lattice (420 MB;
    32,400 rows, so the last 16 workgroups keep their place) stepped alone
    matches the FP64 oracle run from the same (FP32-rounded) start after an
    even and after an odd step (relative L2 1e-6), and stepped as the only
    member of a batch gives the same populations bit for bit, from random
    ones, after an even, an odd and another even step."""
    q, n = 18, 180
    faces, lid = ("wall",) * 6, {"+z": (0.05, 0.02, 0.0)}
    pair = []
    for _ in range(2):
        lat = lbm.Lattice(q, n, n, n, rates(q, 1), faces=faces, wall_u=lid, storage="f32",
                          pattern="aa")
        lat.set_f(inputs.random_populations(q, n, n, n, seed=650))
        pair.append(lat)
    assert lbm.footprint_bytes(q, n, n, n, storage="f32", pattern="aa") > 384 << 20
    alone, member = pair
    pr = R.problem(q, n, n, n, rates(q, 1), faces=faces, wall_u=lid)
    ref = alone.get_f()
    for t in range(2):  # the even step, then the odd one
        alone.step(1)
        ref = R.run(pr, ref, t, 1)
        got = alone.get_f()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print("180^3 D3Q18 FP32, step %d (%s): rel L2 vs oracle %.2e"
              % (t + 1, "even" if t == 0 else "odd", err))
        assert err <= 1e-6, (t, err)
        del got
    alone.step(1)
    b = lbm.Batch(member.stream)
    b.add(member, 3)
    b.step(3)
    assert np.array_equal(alone.get_f(), member.get_f())
    b.close()
    alone.close()
    member.close()


@pytest.mark.parametrize("q", (14, 18, 26))
def test_fp16_members_are_invariant_under_the_deviation_scale(q):
    """Batched FP16 members step in deviation units too: two copies of one
    forced lattice with a moving wall and a background pressure, stored with
    scales 2^12 and 2^13, advance in the same class launches (both below the
    size that steps alone) and decode to the same populations bit for bit
    after even and odd steps."""
    dims = (23, 17, 11)
    _, w, _, _, _, _ = R.lattice(q)
    p0 = 0.2
    f0 = (3.0 * w * p0).reshape(q, 1, 1, 1) + inputs.random_populations(q, *dims, seed=33)
    lats = []
    for log2 in (12, 13):
        lat = lbm.Lattice(q, *dims, rates(q, 1), faces=("periodic", "periodic", "wall", "wall",
                                                         "wall", "symmetry"),
                          wall_u={"-y": (0.03, 0.0, 0.01)}, F0=(1e-5, 0, 0), FA=(1e-5, 0, 0),
                          FT=9.0, storage="f16dev", pattern="aa", p0=p0, f16_scale_log2=log2)
        lat.set_f(f0)
        lats.append(lat)
    b = lbm.Batch(lats[0].stream)
    for lat in lats:
        b.add(lat, 100)
    b.step(3)
    b.step(2)
    a, c = lats[0].get_f(), lats[1].get_f()
    assert np.all(np.isfinite(a)) and not np.array_equal(a, f0)
    assert np.array_equal(a, c)
    b.close()
    for lat in lats:
        lat.close()

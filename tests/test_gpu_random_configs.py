"""A seeded sweep over random lattice configurations, against the FP64
oracle: shapes from 1 to 13 nodes per axis (x rows up to 139 nodes, longer
than a wavefront), every face kind on every face (periodic in pairs;
velocity, pressure and node-layer symmetry faces on axes of at least 3
nodes), random wall / face velocities, face pressures (steady or
oscillating), steady or oscillating body forces, random rates, both models,
both memory patterns.

* FP64: the GPU step equals the oracle element-wise (1e-13 of max|f|) after
  1 and 4 steps (both AA parities); every fourth configuration uses the
  LBGK collision, against the oracle's MRT step with all rates equal.
* FP32 and FP16-deviation AA: the same configurations advanced together in
  one batch, in uneven calls, give bit for bit the populations of single
  lattices, and those equal the oracle run from the same (rounded) start
  within the storage's rounding: relative L2 1e-6 in FP32, one FP16 rounding
  per value and step (2 sqrt(steps) 2^-10) for FP16 deviations.
"""
import numpy as np
import pytest

from helpers import svec
from oracle import runner as R
from paper_1503_03337_amd import inputs, lbm

pytestmark = pytest.mark.gpu

FACE_NAMES = ("-x", "+x", "-y", "+y", "-z", "+z")
NONPERIODIC = ("wall", "symmetry", "velocity", "pressure", "symmetry_node")
NODE_BASED = ("velocity", "pressure", "symmetry_node")
COUNT = 200
COUNT26 = 60


def random_config(rng, q=None):
    if q is None:
        q = int(rng.choice([14, 18]))
    dims = [int(rng.integers(1, 14)) for _ in range(3)]
    if rng.random() < 0.3:
        dims[0] = int(rng.integers(60, 140))
    faces = []
    for d in range(3):
        if rng.random() < 0.3:
            faces += ["periodic", "periodic"]
            continue
        lo, hi = (str(k) for k in rng.choice(NONPERIODIC, 2))
        if (lo in NODE_BASED or hi in NODE_BASED) and dims[d] < 3:
            dims[d] = int(rng.integers(3, 9))
        faces += [lo, hi]
    wall_u = {name: tuple(float(v) for v in rng.uniform(-0.1, 0.1, 3))
              for name in FACE_NAMES if rng.random() < 0.5}
    face_p = {name: float(rng.uniform(-0.01, 0.01))
              for name, k in zip(FACE_NAMES, faces) if k == "pressure"}
    F0 = tuple(float(v) for v in rng.uniform(-1e-4, 1e-4, 3)) if rng.random() < 0.4 else (0, 0, 0)
    FT, FA, face_pA = 0.0, (0, 0, 0), None
    if rng.random() < 0.3:
        FT = float(rng.uniform(5.0, 30.0))
        FA = tuple(float(v) for v in rng.uniform(-1e-4, 1e-4, 3))
        face_pA = {name: float(rng.uniform(-0.005, 0.005)) for name in face_p}
    s = svec(q, float(rng.uniform(0.6, 1.9))) + rng.uniform(-0.05, 0.05, q)
    kw = dict(faces=tuple(faces), wall_u=wall_u, face_p=face_p, face_pA=face_pA, F0=F0, FA=FA,
              FT=FT)
    return q, tuple(dims), s, kw


def configs():
    rng = np.random.default_rng(20260)
    out = [random_config(rng) for _ in range(COUNT)]
    # the 26-velocity model on a sweep of its own (the first COUNT keep
    # their draws)
    rng26 = np.random.default_rng(2626)
    return out + [random_config(rng26, q=26) for _ in range(COUNT26)]


@pytest.mark.parametrize("i", range(COUNT + COUNT26))
def test_random_config_fp64_matches_oracle(i):
    q, dims, s, kw = configs()[i]
    pattern = "aa" if i % 2 == 0 else "ab"
    collision = "mrt"
    if i % 4 == 3:
        # every fourth: the LBGK collision, against the oracle's MRT step with
        # every rate equal (the paper's reduction)
        collision = "bgk"
        s = np.full(q, s[8])
    print("config %d: q=%d dims=%s faces=%s pattern=%s %s FT=%g"
          % (i, q, dims, kw["faces"], pattern, collision, kw["FT"]), flush=True)
    lat = lbm.Lattice(q, *dims, s, storage="f64", pattern=pattern, collision=collision, **kw)
    pr = R.problem(q, *dims, s, **kw)
    lat.set_f(inputs.random_populations(q, *dims, seed=100 + i))
    f = lat.get_f()
    scale = np.max(np.abs(f))
    t = 0
    for n in (1, 3):
        lat.step(n)
        f = R.run(pr, f, t, n)
        t += n
        assert np.max(np.abs(lat.get_f() - f)) <= 1e-13 * scale, (i, t)
    lat.close()


@pytest.mark.parametrize("storage", ("f32", "f16dev"))
def test_random_configs_batched_equal_single(storage):
    cfgs = configs()
    singles, members, starts = [], [], []
    for i, (q, dims, s, kw) in enumerate(cfgs):
        for group in (singles, members):
            lat = lbm.Lattice(q, *dims, s, storage=storage, pattern="aa", **kw)
            lat.set_f(inputs.random_populations(q, *dims, seed=300 + i))
            if group is singles:
                starts.append(lat.get_f())  # the start as stored (rounded)
            if i % 3 == 0:
                lat.step(1)
            group.append(lat)
    b = lbm.Batch(members[0].stream)
    for lat in members:
        b.add(lat, 10 ** 6)
    for n in (3, 1, 2):
        b.step(n)
    b.close()
    worst = 0.0
    for i, (s_lat, m_lat) in enumerate(zip(singles, members)):
        s_lat.step(m_lat.time - s_lat.time)
        g = m_lat.get_f()
        assert np.array_equal(s_lat.get_f(), g), i
        q, dims, s, kw = cfgs[i]
        steps = m_lat.time
        f = R.run(R.problem(q, *dims, s, **kw), starts[i], 0, steps)
        err = np.linalg.norm(g - f) / np.linalg.norm(f)
        tol = 1e-6 if storage == "f32" else 2 * np.sqrt(steps) * 2.0 ** -10
        assert err <= tol, (i, steps, err)
        worst = max(worst, err / tol)
    print("%s: worst error / tolerance against the oracle %.3f" % (storage, worst))
    for lat in singles + members:
        lat.close()

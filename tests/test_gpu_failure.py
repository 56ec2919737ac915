"""Failure path on the GPU: a state that turns non-finite is reported by
lbm_step / lbm_poll (LBM_ENONFINITE) once a monitor run has seen it, a batch
and the serving loop retire the failing member, and every other member's
result is the same as alone, bit for bit.  Forcing cases: a NaN injected
through lbm_set_f, and the diverging cavity of Sec. 4.3 (Re 3200)."""
import numpy as np
import pytest

from helpers import svec
from paper_1503_03337_amd import inputs, lbm, params, serve

pytestmark = pytest.mark.gpu


def poisoned(f, where=(0, 2, 3, 4)):
    g = f.copy()
    g[where] = np.nan
    return g


def cavity(q, edge, Re, storage="f32", monitor_every=0, collision="mrt"):
    cfg = params.cavity(q, edge, Re, lid=0.1)
    s = cfg["s_vec"] if collision == "mrt" else np.full(q, cfg["s_vec"][8])
    return lbm.Lattice(q, edge, edge, edge, s, faces=cfg["faces"], wall_u=cfg["wall_u"],
                       storage=storage, pattern="aa", monitor_every=monitor_every,
                       collision=collision)


@pytest.mark.parametrize("storage", ("f64", "f32", "f16dev"))
def test_step_reports_a_nonfinite_state(storage):
    """A NaN set into one population: the next monitor run (every 10 steps)
    sees it, and lbm_step raises LBM_ENONFINITE from then on without
    advancing; lbm_poll agrees; a new finite state clears it."""
    lat = cavity(18, 12, 100.0, storage=storage, monitor_every=10)
    lat.step(20)
    lat.poll()
    f = lat.get_f()
    lat.set_f(poisoned(f))
    lat.step(10)           # the monitor at t = 30 sees the NaN (queued)
    lat.sync()
    with pytest.raises(lbm.LbmError) as e:
        lat.step(5)
    assert e.value.code == lbm.ENONFINITE
    assert lat.time == 30  # nothing was queued
    with pytest.raises(lbm.LbmError):
        lat.poll()
    assert not lat.healthy()
    with pytest.raises(lbm.LbmError):
        lat.step(1)
    lat.set_f(f)           # a finite state again
    assert lat.healthy()
    lat.step(20)
    lat.sync()
    lat.poll()
    lat.close()


def test_diverging_cavity_is_stopped():
    """Sec. 4.3: the LBGK collision diverges in the cavity at Re = 3200.  A
    32^3 D3Q14 LBGK cavity at Re 3200 with bounce-back walls turns
    non-finite within 1,000 steps (the FP64 oracle: by t = 750); stepped in
    calls of 100 with the monitor every 100 steps, lbm_step raises
    LBM_ENONFINITE within a few monitor intervals of it.  The MRT cavity at
    Re 400 runs on."""
    bad = cavity(14, 32, 3200.0, monitor_every=100, collision="bgk")
    good = cavity(14, 32, 400.0, monitor_every=100)
    code = None
    for _ in range(60):
        try:
            bad.step(100)
            bad.sync()
        except lbm.LbmError as e:
            code = e.code
            break
    print("diverging LBGK cavity stopped at t = %d" % bad.time)
    assert code == lbm.ENONFINITE
    assert bad.time <= 3000
    good.step(3000)
    good.sync()
    good.poll()
    assert np.isfinite(good.mass())
    bad.close()
    good.close()


def _member(k, monitor_every=100):
    spec = [(14, 20, "f32"), (18, 17, "f16dev"), (18, 23, "f32"), (14, 15, "f16dev")][k]
    q, L, storage = spec
    cfg = params.cavity(q, L, 300.0 + 50 * k, lid=0.1)
    lat = lbm.Lattice(q, L, L, L, cfg["s_vec"], faces=cfg["faces"], wall_u=cfg["wall_u"],
                      storage=storage, pattern="aa", monitor_every=monitor_every)
    lat.set_f(inputs.random_populations(q, L, L, L, seed=700 + k, spread=0.05))
    return lat


def test_batch_member_with_nan_is_detected_and_others_unchanged():
    """A mixed batch of four; member 2 gets a NaN through lbm_set_f.  After
    a batched monitor only member 2 reports LBM_ENONFINITE, it is removed,
    and the other three end bit for bit where they end alone."""
    alone = []
    for k in (0, 1, 3):
        lat = _member(k)
        b = lbm.Batch(lat.stream)
        b.add(lat, 60)
        b.step(60)
        b.close()
        alone.append(lat.get_f())
        lat.close()
    lats = [_member(k) for k in range(4)]
    lats[2].set_f(poisoned(lats[2].get_f()))
    b = lbm.Batch(lats[0].stream)
    for lat in lats:
        b.add(lat, 60)
    b.step(30)
    b.monitor()
    for k, lat in enumerate(lats):
        if k == 2:
            assert not lat.healthy()
            with pytest.raises(lbm.LbmError) as e:
                lat.poll()
            assert e.value.code == lbm.ENONFINITE
        else:
            lat.poll()
    b.remove(lats[2])
    b.step(30)
    b.monitor()
    for k, f in zip((0, 1, 3), alone):
        lats[k].poll()
        assert np.array_equal(lats[k].get_f(), f), k
    b.close()
    for lat in lats:
        lat.close()


def _trace():
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(6):
        reqs.append({"id": i, "arrival": 0.001 * i, "kind": "duct" if i % 2 else "cavity",
                     "edge": int(rng.integers(16, 33)), "q": 14 if i % 3 else 18,
                     "steps": int(rng.integers(1200, 2500)), "stop_residual": None})
    # the Sec. 4.3 failure case as a request: a D3Q14 cavity at Re 3200
    # (bounce-back walls, MRT), which the oracle shows non-finite by t = 750
    reqs.append({"id": 6, "arrival": 0.0025, "kind": "cavity", "edge": 32, "q": 14,
                 "Re": 3200.0, "steps": 4000, "stop_residual": None})
    return reqs


@pytest.mark.parametrize("server,storage", [("batched", "f32"), ("batched", "f16dev"),
                                            ("plain", "f32")])
def test_served_trace_retires_failing_requests(server, storage):
    """A served trace with one request poisoned through lbm_set_f as it is
    admitted (id 3) and one that diverges by itself (id 6): both are
    retired with status "failed", the server serves the rest to the end,
    and every other result equals its alone run bit for bit."""
    trace = _trace()

    def inject(rec, lat):
        if rec["id"] == 3:
            lat.set_f(poisoned(lat.get_f()))

    run = serve.serve_batched if server == "batched" else serve.serve_plain
    kw = {"quantum": 50} if server == "batched" else {}
    if server == "plain":
        storage = "f32"
    mixed, _ = run(trace, storage, keep_fields=True, on_admit=inject, **kw)
    by_id = {r["id"]: r for r in mixed}
    assert len(mixed) == len(trace)
    for rid in (3, 6):
        assert by_id[rid]["status"] == "failed", by_id[rid]
        assert "u" not in by_id[rid]
        assert by_id[rid]["steps_done"] < trace[rid]["steps"] or rid == 3
    summary = serve.summarise(mixed)
    assert summary["failed"] == 2 and summary["requests"] == len(trace)
    for req in trace:
        if req["id"] in (3, 6):
            continue
        m = by_id[req["id"]]
        assert m["status"] == "ok" and m["steps_done"] == req["steps"], m
        alone, _ = run([dict(req, arrival=0.0)], storage, keep_fields=True, **kw)
        assert np.array_equal(alone[0]["u"], m["u"]), req

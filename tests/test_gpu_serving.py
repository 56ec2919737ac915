"""Serving loop on the GPU: every request completes, admission never exceeds
the HBM budget, each result is the same alone and in the mix, and served
FP16-deviation duct solves stay within 1e-3 u_max of the FP32 ones and close
to the analytic duct series (Sec. 4.1)."""
import numpy as np
import pytest

from oracle import analytic
from paper_1503_03337_amd import autotune, params, serve

pytestmark = pytest.mark.gpu


def small_trace():
    """Eight requests; two carry a residual stop that triggers before their
    budget (checked every 500 steps of their own clock)."""
    reqs = []
    rng = np.random.default_rng(5)
    for i in range(8):
        res = i in (2, 5)
        reqs.append({"id": i, "arrival": 0.002 * i, "kind": "duct" if i % 2 else "cavity",
                     "edge": int(rng.integers(16, 41)), "q": 14 if i % 3 else 18,
                     "steps": 3000 if res else int(rng.integers(150, 450)),
                     "stop_residual": 5e-3 if res else None})
    return reqs


@pytest.mark.parametrize("storage", ("f32", "f16dev"))
def test_mix_equals_alone_and_budget_respected(storage):
    trace = small_trace()
    fp = {r["id"]: serve.footprint(r, storage) for r in trace}
    budget = sum(sorted(fp.values())[-3:])  # forces queueing
    mixed, info = serve.serve_batched(trace, storage, budget_bytes=budget, quantum=50,
                                      keep_fields=True)
    assert len(mixed) == len(trace)
    assert info["peak_bytes"] <= budget
    by_id = {r["id"]: r for r in mixed}
    for req in trace:
        alone, _ = serve.serve_batched([dict(req, arrival=0.0)], storage, budget_bytes=budget,
                                       quantum=50, keep_fields=True)
        a, m = alone[0], by_id[req["id"]]
        assert a["steps_done"] == m["steps_done"], req
        if req["stop_residual"] is None:
            assert m["steps_done"] == req["steps"]
        else:  # stopped by the residual, on its own 500-step schedule
            assert m["steps_done"] < req["steps"] and m["steps_done"] % 500 == 0
        assert np.array_equal(a["u"], m["u"]), req


def test_traffic_cap_runs_large_requests_one_after_another():
    """Admission stops while the admitted lattices move SATURATION_BYTES per
    step, and a request always enters an empty batch: two requests that each
    move more than that run one after the other, two quanta each, and three
    small ones that together stay under it share two quanta (6 quanta in
    all).  Without the cap all five share the same two quanta."""
    def req(i, edge):
        return {"id": i, "arrival": 0.0, "kind": "cavity", "edge": edge, "q": 18, "steps": 200,
                "stop_residual": None}
    big = [req(0, 96), req(1, 96)]
    small = [req(10, 24), req(11, 24), req(12, 24)]
    assert all(serve.step_bytes(r, "f32") > serve.SATURATION_BYTES for r in big)
    assert sum(serve.step_bytes(r, "f32") for r in small) <= serve.SATURATION_BYTES
    for cap, quanta in ((serve.SATURATION_BYTES, 6), (None, 2)):
        recs, info = serve.serve_batched(big + small, "f32", quantum=100, max_active_bytes=cap)
        assert len(recs) == 5 and all(r["status"] == "ok" and r["steps_done"] == 200
                                      for r in recs)
        assert info["step_launches"] == 100 * quanta, (cap, info)


def test_plain_and_batched_agree():
    trace = [r for r in small_trace() if r["stop_residual"] is None][:4]
    plain, _ = serve.serve_plain(trace, "f32", keep_fields=True)
    batched, _ = serve.serve_batched(trace, "f32", keep_fields=True)
    bp = {r["id"]: r for r in plain}
    for r in batched:
        p = bp[r["id"]]
        assert p["steps_done"] == r["steps_done"]
        scale = max(np.max(np.abs(p["u"])), 1e-12)
        assert np.max(np.abs(p["u"] - r["u"])) <= 1e-5 * scale


def test_fp16_duct_accuracy():
    """Converged edge-32 ducts of both models served batched in FP16
    deviations: within 1e-3 of the steady series in GRE_u (the error norm of
    Sec. 4.1) and within 1e-3 u_max of the plain FP32 results pointwise."""
    reqs = [{"id": i, "arrival": 0.0, "kind": "duct", "edge": 32, "q": q, "steps": 12000,
             "stop_residual": None} for i, q in enumerate((14, 18))]
    b16, _ = serve.serve_batched(reqs, "f16dev", keep_fields=True)
    p32, _ = serve.serve_plain(reqs, "f32", keep_fields=True)

    def series(Y, Z, a, g, nu):
        return analytic.duct_steady(Y, Z, a, a, g, nu)

    b16 = {r["id"]: r for r in b16}
    p32 = {r["id"]: r for r in p32}
    for r in reqs:
        h, f = b16[r["id"]], p32[r["id"]]
        (hm, hg), (fm, fg) = serve.duct_errors(h, series), serve.duct_errors(f, series)
        d = np.max(np.abs(h["u"] - f["u"])) / serve.DUCT_UMAX
        print("q%d duct edge 32: FP16 max %.2e GRE %.2e, FP32 max %.2e GRE %.2e, "
              "|FP16-FP32|/u_max %.2e" % (r["q"], hm, hg, fm, fg, d))
        assert hg <= 1e-3 and fg <= 1e-3
        assert d <= 1e-3
        assert hm < 2e-3 and fm < 2e-3  # pointwise: second-order wall error at edge 32


def test_autotune_picks_valid_tiles():
    def mk(q, edge):
        return serve.make_lattice({"q": q, "edge": edge, "kind": "cavity"}, "f32")
    best, log = autotune.tune(mk, [(14, 24), (18, 40), (18, 45)], steps=10, reps=1)
    assert set(best) == {(14, 24), (18, 40)}
    for key, (tx, ty) in best.items():
        assert (tx, ty) == (0, 0) or 1 <= tx * ty <= 256  # (0, 0): flat mapping
        assert (tx, ty) in log[key]


def test_fp16_duct_accuracy_at_the_largest_served_edge():
    """The same at the largest edge the serving trace draws (160: 4.1 M
    nodes, 20,000 steps).  GRE_u stays within 1e-3 of the series.  Pointwise,
    the stochastic-rounding fluctuation of FP16 storage is a noise whose
    maximum over N nodes grows like sqrt(2 ln N) times its RMS, so the bound
    that holds is stated on both: RMS |FP16 - FP32| <= 2.5e-4 u_max and
    max <= 1.5e-3 u_max (1e-3 held at edge 32, 3.2e4 nodes)."""
    reqs = [{"id": i, "arrival": 0.0, "kind": "duct", "edge": 160, "q": q, "steps": 20000,
             "stop_residual": None} for i, q in enumerate((14, 18))]
    b16, _ = serve.serve_batched(reqs, "f16dev", keep_fields=True)
    p32, _ = serve.serve_plain(reqs, "f32", keep_fields=True)

    def series(Y, Z, a, g, nu):
        return analytic.duct_steady(Y, Z, a, a, g, nu)

    b16 = {r["id"]: r for r in b16}
    p32 = {r["id"]: r for r in p32}
    for r in reqs:
        h, f = b16[r["id"]], p32[r["id"]]
        (hm, hg), (fm, fg) = serve.duct_errors(h, series), serve.duct_errors(f, series)
        diff = np.abs(h["u"] - f["u"]) / serve.DUCT_UMAX
        rms, mx = float(np.sqrt(np.mean(diff ** 2))), float(np.max(diff))
        print("q%d duct edge 160: FP16 GRE %.2e max %.2e, FP32 GRE %.2e max %.2e, "
              "|FP16-FP32|/u_max rms %.2e max %.2e" % (r["q"], hg, hm, fg, fm, rms, mx))
        assert hg <= 1e-3 and fg <= 1e-3
        assert rms <= 2.5e-4 and mx <= 1.5e-3

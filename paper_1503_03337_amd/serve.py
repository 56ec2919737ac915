"""Serving loop: continuous batching of lattice Boltzmann solves on one GPU.

Requests (duct or cavity solves of uneven sizes, D3Q14 or D3Q18, a step
budget or a stop at a velocity residual) arrive over time.  Two servers:

  plain    one request at a time, in arrival order, the single-lattice
           kernel (lbm_step); storage FP32 or FP16 deviations
  batched  continuous batching: arrived requests are admitted, in arrival
           order, while their HBM footprint (lbm_footprint_bytes) fits the
           budget and the admitted lattices move fewer bytes per step than
           it takes to fill the GPU (max_active_bytes); all admitted requests
           advance together, one kernel launch per time step and lattice class
           (lbm_batch_step), in quanta of Q steps; between quanta finished
           requests retire (freeing their memory) and waiting ones are
           admitted, so new work overlaps running work on the device.
           Storage FP32 or FP16 deviations.

The traffic cap keeps the batch from turning into processor sharing: once the
admitted lattices saturate HBM bandwidth, admitting more only slows every
admitted request down, so large requests run one after another (as in the
plain server) while small ones, which cannot fill the GPU alone, share it.

Latency is arrival -> finish.  Aggregate throughput is the node updates of
all completed requests over the time from the first arrival to the last
finish.

Failure: every request runs the FP64 monitor (every 100 steps with a
residual stop, else every 1000 steps); a request whose monitor sees a
non-finite mass or velocity (a diverging solve: Sec. 4.3 reports the LBGK
cavity diverging at Re 3200, and a 14-velocity MRT cavity with bounce-back
walls does too) is retired at once with status "failed" and its memory
freed, and the server keeps serving the others, whose results do not
change.  A request that ends its budget gets one more monitor run first, so
a result that turned non-finite after its last periodic run is reported as
failed too.
"""
import math
import time

import numpy as np

from . import autotune, inputs, lbm, params

MONITOR_EVERY = 100   # residual lag (steps) for requests with a residual stop
RESIDUAL_EVERY = 500  # a residual stop is checked when the request's t is a multiple
HEALTH_EVERY = 1000   # monitor interval of the other requests (non-finite check)
PLAIN_CHUNK = 1000    # steps per lbm_step call of the plain server
DUCT_UMAX = 0.05      # centre-line speed of duct requests
CAVITY_RE = 400.0     # cavity Reynolds number at lid speed 0.1
DUCT_EFOLD = 1500.0   # slowest duct mode decays within this many steps
# Batches are filled up to what a D3Q18 FP32 lattice of 2^19 nodes (80^3,
# 2 x 18 x 4 B moved per node and step) moves per step.  A large member
# alone in its class steps with the single-lattice kernels at full speed,
# so a larger cap only shares the GPU between large requests: on the
# serving trace a cap of 2^21 nodes' bytes (128^3) left the batched FP16
# server 1.4 % behind the plain one saturated, with a Poisson p99 of 1.27
# against 0.82 s, and the batched FP32 server's Poisson p99 at 2.09 against
# 2.00 s; with 2^19 both servers match or beat the plain ones in throughput,
# p50 and p99 (2^20 lies between).
SATURATION_BYTES = (1 << 19) * 144
STORAGE_BYTES = {"f32": 4, "f16dev": 2, "f64": 8}


def step_bytes(req, storage):
    """Bytes a request's lattice moves per time step: 2 q b per node."""
    return 2 * req["q"] * STORAGE_BYTES[storage] * req["edge"] ** 3


def duct_nu(edge):
    """Viscosity of a duct request: 0.1, or more for wide ducts so that the
    slowest mode, rate nu (pi/2a)^2 2, e-folds within DUCT_EFOLD steps."""
    a = edge / 2.0
    return max(0.1, a * a / (2.0 * (math.pi / 2.0) ** 2 * DUCT_EFOLD))


def request_setup(req):
    """Lattice of a request: a square duct (edge^3 nodes, x periodic, body
    force for u_max = 0.05; odd rates tied to s_nu so that the wide ducts'
    larger nu does not move the walls, or with req["odd"] = "paper" the
    paper's fixed s_q = 1.2, s_t = 0.98) or a lid-driven cube (lid 0.1 along
    +x, Reynolds number req.get("Re", 400), the paper's rates)."""
    q, L = req["q"], req["edge"]
    if req["kind"] == "duct":
        cfg = params.duct(q, L, L, duct_nu(L), umax=DUCT_UMAX, odd=req.get("odd", "magic"))
        kw = {"faces": cfg["faces"], "F0": cfg["F0"]}
    else:
        cfg = params.cavity(q, L, req.get("Re", CAVITY_RE), lid=0.1)
        kw = {"faces": cfg["faces"], "wall_u": cfg["wall_u"]}
    return cfg["s_vec"], kw


def _monitor(req):
    return MONITOR_EVERY if req.get("stop_residual") else HEALTH_EVERY


def footprint(req, storage):
    _, kw = request_setup(req)
    L = req["edge"]
    return lbm.footprint_bytes(req["q"], L, L, L, storage=storage, pattern="aa",
                               monitor_every=_monitor(req), **kw)


def make_lattice(req, storage):
    s, kw = request_setup(req)
    L = req["edge"]
    return lbm.Lattice(req["q"], L, L, L, s, storage=storage, pattern="aa",
                       monitor_every=_monitor(req), **kw)


class Clock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0


def _velocity(lat):
    """u[3, nz, ny, nx] at the current level through lbm_macros_device into
    memory from torch's caching allocator, so retiring a request allocates
    no device memory in the library (lbm_macros stages through memory it
    allocates on every call)."""
    import torch
    u = torch.empty((3, lat.nz, lat.ny, lat.nx), dtype=torch.float64, device="cuda")
    lat.macros_device(None, u.data_ptr())
    lat.sync()
    return u.cpu().numpy()


def _finish(rec, clock, lat, keep_fields):
    rec["finish"] = clock.now()
    rec["latency"] = rec["finish"] - rec["arrival"]
    rec["steps_done"] = lat.time
    rec.setdefault("status", "ok")
    if keep_fields and rec["status"] == "ok":
        rec["u"] = _velocity(lat)


def _final_check(rec, lat):
    """One more monitor run at the request's end: a state that is not
    finite fails the request."""
    if rec.get("status", "ok") != "ok":
        return
    try:
        lat.monitor()
        lat.mass()  # waits for that run; raises LBM_ENONFINITE
    except lbm.LbmError as e:
        _failed(rec, e)


def _failed(rec, err):
    """Mark a request whose monitor saw a non-finite value; re-raise any
    other error."""
    if not (isinstance(err, lbm.LbmError) and err.code == lbm.ENONFINITE):
        raise err
    rec["status"] = "failed"
    rec["error"] = str(err)


def serve_plain(trace, storage="f32", keep_fields=False, on_admit=None):
    """One request at a time in arrival order (FIFO), lbm_step in calls of
    PLAIN_CHUNK steps with at most two in flight.  on_admit(rec, lat), if
    given, is called with each new lattice before it steps."""
    import torch
    clock = Clock()
    out = []
    stream = torch.cuda.current_stream()
    for req in sorted(trace, key=lambda r: r["arrival"]):
        while clock.now() < req["arrival"]:
            time.sleep(min(0.001, max(0.0, req["arrival"] - clock.now())))
        rec = dict(req)
        rec["admit"] = clock.now()
        lat = make_lattice(req, storage)
        if on_admit:
            on_admit(rec, lat)
        # the monitor runs inside lbm_step (every MONITOR_EVERY steps with a
        # residual stop, checked every RESIDUAL_EVERY steps at lag 100; else
        # every HEALTH_EVERY steps); lbm_step raises LBM_ENONFINITE once a
        # completed run saw a non-finite value
        try:
            done, inflight = 0, []
            chunk = RESIDUAL_EVERY if req.get("stop_residual") else PLAIN_CHUNK
            while done < req["steps"]:
                k = min(chunk, req["steps"] - done)
                lat.step(k)
                done += k
                if req.get("stop_residual"):
                    if done % RESIDUAL_EVERY == 0 and lat.residual() <= req["stop_residual"]:
                        break
                else:
                    ev = torch.cuda.Event()
                    ev.record(stream)
                    inflight.append(ev)
                    if len(inflight) > 2:
                        inflight.pop(0).synchronize()
        except lbm.LbmError as e:
            _failed(rec, e)
        _final_check(rec, lat)
        stream.synchronize()
        _finish(rec, clock, lat, keep_fields)
        lat.close()
        out.append(rec)
    return out, {"peak_bytes": max(footprint(r, storage) for r in trace)}


def serve_batched(trace, storage="f16dev", budget_bytes=16 << 30, quantum=100,
                  keep_fields=False, tiles=None, max_active_bytes=SATURATION_BYTES,
                  on_admit=None):
    """Continuous batching with admission by HBM footprint.

    The loop keeps the device busy: quantum k+1 is queued before the host
    waits for quantum k (at most two in flight).  Members whose step budget
    runs out leave the batch as soon as their last quantum is queued (the
    host knows budgets without asking the device) and are reported when that
    quantum completes.  A member with a residual stop follows its own clock,
    as in the plain server: a monitor snapshot at t = RESIDUAL_EVERY k - 100
    and a check at t = RESIDUAL_EVERY k (lag 100), so its result does not
    depend on the other members.  quantum must divide 100.
    tiles: optional {(q, edge bucket): (tx, ty)} from autotune.tune.
    max_active_bytes: admission stops while the admitted lattices move this
    many bytes per step (a request is always admitted into an empty batch);
    None admits whatever fits the memory budget.
    Every member runs its monitor on its own clock (residual stops: a
    snapshot and a check as above; other members every HEALTH_EVERY steps),
    queued right after the quantum that reaches that time level; after each
    quantum the host polls every member without waiting, and a member whose
    completed monitor run saw a non-finite value leaves the batch at once,
    reported with status "failed".
    on_admit(rec, lat), if given, is called with each new lattice before it
    joins the batch."""
    assert MONITOR_EVERY % quantum == 0 and RESIDUAL_EVERY % quantum == 0
    import torch
    clock = Clock()
    pending = sorted(trace, key=lambda r: r["arrival"])
    stream = torch.cuda.current_stream()
    batch = lbm.Batch(stream.cuda_stream)
    active = []     # (record, lattice) in the batch
    draining = []   # (event, [(record, lattice)]) left the batch, last quantum in flight
    inflight = []   # events of queued quanta, oldest first
    used = peak = 0
    active_bytes = 0
    launches = quanta = 0
    out = []

    def retire(rec, lat):
        nonlocal used
        _final_check(rec, lat)
        _finish(rec, clock, lat, keep_fields)
        used -= rec.pop("_need")
        lat.close()
        out.append(rec)

    while pending or active or draining:
        now = clock.now()
        while pending and pending[0]["arrival"] <= now:
            need = footprint(pending[0], storage)
            if need > budget_bytes:
                raise ValueError("request %d needs %d bytes, above the budget %d" %
                                 (pending[0]["id"], need, budget_bytes))
            if used + need > budget_bytes:
                break  # wait for memory: admitted in arrival order
            moved = step_bytes(pending[0], storage)
            if (max_active_bytes is not None and active
                    and active_bytes + moved > max_active_bytes):
                break  # the GPU is full: wait in arrival order
            req = pending.pop(0)
            rec = dict(req)
            rec["admit"] = clock.now()
            lat = make_lattice(req, storage)
            if on_admit:
                on_admit(rec, lat)
            batch.add(lat, req["steps"])
            if tiles:
                t = autotune.tile_for(tiles, req["q"], req["edge"])
                if t:
                    batch.set_tile(lat, *t)
            rec["_need"] = need
            used += need
            active_bytes += moved
            peak = max(peak, used)
            active.append((rec, lat))
        if active:
            if len(inflight) >= 2:
                inflight.pop(0).synchronize()
            batch.step(quantum)
            launches += quantum
            quanta += 1
            ev = torch.cuda.Event()
            ev.record(stream)
            inflight.append(ev)
            done = [(r, l) for r, l in active if batch.remaining(l) == 0]
            for r, l in active:
                if batch.remaining(l) == 0:
                    continue
                t = l.time
                try:
                    if not l.healthy():  # a completed monitor run saw a non-finite value
                        l.poll()
                    if not r.get("stop_residual"):
                        if t % HEALTH_EVERY == 0:
                            l.monitor()  # queued; its result is polled later
                    elif t % RESIDUAL_EVERY == RESIDUAL_EVERY - MONITOR_EVERY:
                        l.monitor()  # snapshot, queued
                    elif t % RESIDUAL_EVERY == 0:
                        l.monitor()
                        if l.residual() <= r["stop_residual"]:  # waits for the monitor
                            done.append((r, l))
                except lbm.LbmError as e:
                    _failed(r, e)
                    done.append((r, l))
            for r, l in done:
                batch.remove(l)
                active_bytes -= step_bytes(r, storage)
            ids = {id(l) for _, l in done}
            active = [(r, l) for r, l in active if id(l) not in ids]
            if done:
                draining.append((ev, done))
        keep = []
        for ev, lst in draining:
            if ev.query():
                for r, l in lst:
                    retire(r, l)
            else:
                keep.append((ev, lst))
        draining = keep
        if not active:
            if draining:
                ev, lst = draining.pop(0)
                ev.synchronize()
                for r, l in lst:
                    retire(r, l)
            elif pending:
                time.sleep(max(0.0, min(0.001, pending[0]["arrival"] - clock.now())))
    batch.close()
    return out, {"peak_bytes": peak, "budget_bytes": budget_bytes, "step_launches": launches}


def summarise(records, extra=None):
    ok = [r for r in records if r.get("status", "ok") == "ok"]
    lat = np.array([r["latency"] for r in ok])
    nodes = sum(r["edge"] ** 3 * r["steps_done"] for r in ok)
    t0 = min(r["arrival"] for r in records)
    t1 = max(r["finish"] for r in records)
    out = {"requests": len(records), "failed": len(records) - len(ok),
           "p50_s": round(float(np.percentile(lat, 50)), 4),
           "p99_s": round(float(np.percentile(lat, 99)), 4),
           "aggregate_MLUPS": round(nodes / (t1 - t0) / 1e6, 1),
           "makespan_s": round(t1 - t0, 3)}
    if extra:
        out.update({k: v for k, v in extra.items()})
    return out


def duct_errors(rec, series):
    """(max_nodes |u_x - u_series| / u_max, GRE_u) of a finished duct
    request, series(y, z, a, g, nu) the steady duct solution; GRE_u is the
    relative L2 error over all nodes and components (Sec. 4.1)."""
    L = rec["edge"]
    a = L / 2.0
    nu = duct_nu(L)
    g = DUCT_UMAX * nu / (params.DUCT_UMAX_COEFF * a * a)
    y = np.arange(L) + 0.5 - a
    Y, Z = np.meshgrid(y, y, indexing="xy")
    ua = series(Y, Z, a, g, nu)[:, :, None]
    u = rec["u"]
    emax = float(np.max(np.abs(u[0] - ua))) / DUCT_UMAX
    num = np.sum((u[0] - ua) ** 2) + np.sum(u[1] ** 2) + np.sum(u[2] ** 2)
    gre = float(np.sqrt(num / (L * np.sum(ua ** 2))))
    return emax, gre


def duct_error(records, series):
    """max over duct requests of max_nodes |u - u_series| / u_max."""
    return max((duct_errors(r, series)[0] for r in records
                if r["kind"] == "duct" and "u" in r), default=0.0)


def _note(msg):
    import sys
    print("serve: " + msg, file=sys.stderr, flush=True)


def bench_summary(n=24, seed=1, budget_gib=16):
    """Plain FP32 and FP16 deviations against batched FP32 and FP16
    deviations on one seeded Poisson trace (rate ~0.8x the plain FP32
    server's measured capacity), and on the same requests all arriving at
    once (saturated), so that the gain of batched FP16 over plain FP32 splits
    into its storage part (plain FP16 / plain FP32) and its batching part
    (batched FP16 / plain FP16)."""
    import torch
    trace = inputs.serving_trace(n, rate=1.0, seed=seed)
    # plain-server capacity from a short probe of the same request mix
    probe = [dict(r, arrival=0.0, steps=max(200, r["steps"] // 10), stop_residual=None)
             for r in trace[:6]]
    pr, _ = serve_plain(probe)
    nodes_per_s = sum(r["edge"] ** 3 * r["steps_done"] for r in pr) / sum(
        r["finish"] - r["admit"] for r in pr)
    mean_work = np.mean([r["edge"] ** 3 * r["steps"] for r in trace])
    rate = 0.8 * nodes_per_s / mean_work
    trace = inputs.serving_trace(n, rate=rate, seed=seed)
    from . import autotune as at
    keys = {(r["q"], r["edge"]) for r in trace}

    def mk(q, edge):
        return make_lattice({"q": q, "edge": edge, "kind": "cavity"}, "f32")
    tiles, _ = at.tune(mk, keys)
    budget = budget_gib << 30
    res = {"trace": {"requests": n, "rate_per_s": round(rate, 3), "seed": seed,
                     "budget_GiB": budget_gib}}
    res["plain_f32"] = summarise(*serve_plain(trace, "f32"))
    _note("plain_f32 done")
    res["plain_f16dev"] = summarise(*serve_plain(trace, "f16dev"))
    _note("plain_f16dev done")
    res["batched_f32"] = summarise(*serve_batched(trace, "f32", budget, tiles=tiles))
    _note("batched_f32 done")
    res["batched_f16dev"] = summarise(*serve_batched(trace, "f16dev", budget, tiles=tiles))
    _note("batched_f16dev done")
    sat = [dict(r, arrival=0.0) for r in trace]
    res["saturated_plain_f32"] = summarise(*serve_plain(sat, "f32"))
    _note("saturated_plain_f32 done")
    res["saturated_plain_f16dev"] = summarise(*serve_plain(sat, "f16dev"))
    _note("saturated_plain_f16dev done")
    res["saturated_batched_f32"] = summarise(*serve_batched(sat, "f32", budget, tiles=tiles))
    _note("saturated_batched_f32 done")
    res["saturated_batched_f16dev"] = summarise(*serve_batched(sat, "f16dev", budget,
                                                               tiles=tiles))
    _note("saturated_batched_f16dev done")
    res["duct_accuracy"] = duct_accuracy()
    _note("duct accuracy done")
    res["duct_accuracy_paper_odd_rates"] = duct_accuracy(odd="paper")
    torch.cuda.synchronize()
    return res


def duct_accuracy(edges=(32, 64, 96, 128, 160), steps=20000, odd="magic"):
    """Converged duct requests of both models, served batched in FP16
    deviations and plainly in FP32, against the steady series: per model
    and edge the max-norm error over u_max and GRE_u, and |FP16 - FP32|.
    odd: "magic" (the served ducts' odd rates, tied to s_nu) or "paper"
    (Sec. 4's fixed s_q = 1.2, s_t = 0.98)."""
    from . import duct_series
    reqs = [{"id": i, "arrival": 0.0, "kind": "duct", "edge": L, "q": q, "steps": steps,
             "stop_residual": None, "odd": odd}
            for i, (L, q) in enumerate((L, q) for L in edges for q in (14, 18))]
    series = lambda Y, Z, a, g, nu: duct_series.velocity(Y, Z, a, a, g, nu)  # noqa: E731
    b16, _ = serve_batched(reqs, "f16dev", keep_fields=True)
    p32, _ = serve_plain(reqs, "f32", keep_fields=True)
    b16 = {r["id"]: r for r in b16}
    p32 = {r["id"]: r for r in p32}
    cases = []
    for r in reqs:
        h, f = b16[r["id"]], p32[r["id"]]
        (hm, hg), (fm, fg) = duct_errors(h, series), duct_errors(f, series)
        cases.append({"q": r["q"], "edge": r["edge"],
                      "f16dev_max": round(hm, 6), "f16dev_gre": round(hg, 6),
                      "f32_max": round(fm, 6), "f32_gre": round(fg, 6),
                      "f16_minus_f32_max": round(float(np.max(np.abs(h["u"] - f["u"])))
                                                 / DUCT_UMAX, 6)})
    return {"steps": steps, "odd_rates": odd, "cases": cases,
            "worst_f16dev_max": max(c["f16dev_max"] for c in cases),
            "worst_f16dev_gre": max(c["f16dev_gre"] for c in cases),
            "worst_f32_max": max(c["f32_max"] for c in cases),
            "worst_f32_gre": max(c["f32_gre"] for c in cases)}

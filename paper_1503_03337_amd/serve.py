"""Serving loop: continuous batching of lattice Boltzmann solves on one GPU.

Requests (duct or cavity solves of uneven sizes, D3Q14 or D3Q18, a step
budget or a stop at a velocity residual) arrive over time.  Two servers:

  plain    one request at a time, in arrival order, FP32 storage, the
           single-lattice kernel (lbm_step)
  batched  continuous batching: arrived requests are admitted while their
           HBM footprint (lbm_footprint_bytes) fits the budget; all admitted
           requests advance together, one kernel launch per time step
           (lbm_batch_step) in quanta of Q steps; between quanta finished
           requests retire (freeing memory) and waiting ones are admitted.
           Storage FP32 or FP16 deviations.

Latency is arrival -> finish; aggregate throughput is the node updates of
all requests divided by the time from first arrival to last finish.
"""
import time

import numpy as np

from . import inputs, lbm, params

MONITOR_EVERY = 100      # residual lag (steps) for requests with a residual stop
DUCT_NU = 0.1            # duct viscosity (lattice units); u_max = 0.05
CAVITY_RE = 400.0        # cavity Reynolds number at lid speed 0.1


def request_setup(req):
    """Lattice description of a request: a square duct (x periodic, edge^3
    nodes, body force for u_max = 0.05) or a lid-driven cube."""
    q, L = req["q"], req["edge"]
    if req["kind"] == "duct":
        cfg = params.duct(q, L, L, DUCT_NU, umax=0.05)
        kw = {"faces": cfg["faces"], "F0": cfg["F0"]}
    else:
        cfg = params.cavity(q, L, CAVITY_RE, lid=0.1)
        kw = {"faces": cfg["faces"], "wall_u": cfg["wall_u"]}
    return cfg["s_vec"], kw


def footprint(req, storage):
    s, kw = request_setup(req)
    mon = MONITOR_EVERY if req.get("stop_residual") else 0
    return lbm.footprint_bytes(req["q"], req["edge"], req["edge"], req["edge"], storage=storage,
                               pattern="aa", monitor_every=mon, **kw)


def make_lattice(req, storage):
    s, kw = request_setup(req)
    L = req["edge"]
    mon = MONITOR_EVERY if req.get("stop_residual") else 0
    return lbm.Lattice(req["q"], L, L, L, s, storage=storage, pattern="aa", monitor_every=mon,
                       **kw)


class Clock:
    """Trace time: seconds since the server started."""

    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0


def _finish(rec, clock, lat, keep_fields):
    rec["finish"] = clock.now()
    rec["latency"] = rec["finish"] - rec["arrival"]
    rec["steps_done"] = lat.time
    if keep_fields:
        rec["u"] = lat.macros()[1]


def serve_plain(trace, storage="f32", keep_fields=False, sync=None):
    """One request at a time in arrival order (FIFO)."""
    clock = Clock()
    out = []
    for req in sorted(trace, key=lambda r: r["arrival"]):
        while clock.now() < req["arrival"]:
            time.sleep(min(0.001, req["arrival"] - clock.now()))
        rec = dict(req)
        rec["admit"] = clock.now()
        lat = make_lattice(req, storage)
        if req.get("stop_residual"):
            done = 0
            while done < req["steps"]:
                k = min(MONITOR_EVERY, req["steps"] - done)
                lat.step(k)
                done += k
                if done >= 2 * MONITOR_EVERY and done % MONITOR_EVERY == 0:
                    if lat.residual() <= req["stop_residual"]:
                        break
        else:
            lat.step(req["steps"])
        lat.sync()
        _finish(rec, clock, lat, keep_fields)
        lat.close()
        out.append(rec)
    return out


def serve_batched(trace, storage="f16dev", budget_bytes=None, quantum=100, keep_fields=False,
                  tiles=None):
    """Continuous batching with admission by HBM footprint."""
    import torch
    if budget_bytes is None:
        free, _ = torch.cuda.mem_get_info()
        budget_bytes = int(0.8 * free)
    clock = Clock()
    pending = sorted(trace, key=lambda r: r["arrival"])
    stream = torch.cuda.current_stream().cuda_stream
    batch = lbm.Batch(stream)
    active = []  # (rec, lattice)
    used = 0
    out = []
    while pending or active:
        # admit whatever has arrived and fits
        now = clock.now()
        while pending and pending[0]["arrival"] <= now:
            need = footprint(pending[0], storage)
            if need > budget_bytes:
                raise ValueError("request %d needs %d bytes, above the budget" %
                                 (pending[0]["id"], need))
            if used + need > budget_bytes:
                break
            req = pending.pop(0)
            rec = dict(req)
            rec["admit"] = clock.now()
            lat = make_lattice(req, storage)
            batch.add(lat, req["steps"])
            if tiles is not None:
                t = tiles.get((req["q"], req["edge"]))
                if t:
                    batch.set_tile(lat, *t)
            rec["_need"] = need
            used += need
            active.append((rec, lat))
        if not active:
            # idle: wait for the next arrival
            if pending:
                time.sleep(max(0.0, min(0.001, pending[0]["arrival"] - clock.now())))
            continue
        batch.step(quantum)
        if any(r.get("stop_residual") for r, _ in active):
            batch.monitor()  # synchronises
        else:
            torch.cuda.current_stream().synchronize()
        keep = []
        for rec, lat in active:
            done = batch.remaining(lat) == 0
            if not done and rec.get("stop_residual") and lat.time >= 2 * quantum:
                done = lat.residual() <= rec["stop_residual"]
            if done:
                batch.remove(lat)
                _finish(rec, clock, lat, keep_fields)
                used -= rec.pop("_need")
                lat.close()
                out.append(rec)
            else:
                keep.append((rec, lat))
        active = keep
    batch.close()
    return out


def summarise(records):
    lat = np.array([r["latency"] for r in records])
    nodes = sum(r["edge"] ** 3 * r["steps_done"] for r in records)
    t0 = min(r["arrival"] for r in records)
    t1 = max(r["finish"] for r in records)
    return {"requests": len(records),
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "aggregate_MLUPS": nodes / (t1 - t0) / 1e6, "makespan_s": t1 - t0}


def bench_summary(torch, n=24, seed=1, rate=None):
    """Plain FP32 against batched FP16-deviation (and FP32) on one seeded
    trace, for the benchmark line.  `rate` defaults to ~0.8x the plain
    server's measured capacity on a probe."""
    probe = inputs.serving_trace(4, rate=1e9, seed=seed + 100, edge=(64, 96), steps=(2000, 3000),
                                 p_residual=0.0)
    pr = serve_plain(probe)
    svc = np.mean([r["finish"] - r["admit"] for r in pr])
    nodes_per_s = sum(r["edge"] ** 3 * r["steps_done"] for r in pr) / sum(
        r["finish"] - r["admit"] for r in pr)
    trace = inputs.serving_trace(n, rate=1.0, seed=seed)
    mean_work = np.mean([r["edge"] ** 3 * r["steps"] for r in trace])
    if rate is None:
        rate = 0.8 * nodes_per_s / mean_work
    trace = inputs.serving_trace(n, rate=rate, seed=seed)
    res = {"trace": {"requests": n, "rate_per_s": rate, "seed": seed,
                     "probe_service_s": float(svc)}}
    res["plain_f32"] = summarise(serve_plain(trace, "f32"))
    res["batched_f32"] = summarise(serve_batched(trace, "f32"))
    res["batched_f16dev"] = summarise(serve_batched(trace, "f16dev"))
    return res

"""Benchmark of the D3Q18 MRT lattice Boltzmann step on one MI355X.

Workload (one "step" = one time step of the whole path: collision, streaming
with bounce-back and the moving lid, plus the FP64 monitor every 1000
steps): a 128^3 lid-driven cubic cavity, D3Q18, FP32 populations in SoA
layout updated in place (AA pattern), lid speed 0.1, Re = 1000
(nu = 0.0128).  Inputs are synthetic and resident in HBM before timing
starts.  The cavity starts at rest, where every population is exactly zero
(p0 = 0); --develop untimed steps (1000 by default, whatever --warmup is)
let the lid's pressure waves cross the cube several times first, and the
run stops unless fewer than 1 % of the populations are still exactly zero,
so the timed steps stream developed flow, not zeros (which the Infinity
Cache moves faster).

Prints one JSON line.  value = MLUPS (million lattice-node updates per
second); the roofline block reads the step kernels against the 8 TB/s HBM
peak using the algorithmic traffic of 2 q b = 144 bytes per node and step.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS & % HBM roofline (D3Q18 FP32); batched serving p50/p99 latency vs plain"
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_step_d3q18_f32_aa_cavity128.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1503_03337_amd", "csrc", f)
                  for f in ("kernels.hip", "lattice.hpp", "kernels.hpp")]


def note(msg):
    """Progress of the run on stderr (stdout carries only the JSON line)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary, or None if there is none or the kernels changed since."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    txt = open(PMC_SUMMARY).read()
    m = re.search(r"kernel_source_hash:\s*(\w+)", txt)
    t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != kernel_hash():
        return None
    return float(t.group(1))


def cavity_lattice(lbm, params, n, monitor_every=1000):
    cfg = params.cavity(18, n, 1000.0, lid=0.1)
    return lbm.Lattice(18, n, n, n, cfg["s_vec"], faces=cfg["faces"], wall_u=cfg["wall_u"],
                       storage="f32", pattern="aa", monitor_every=monitor_every)


def time_steps(torch, lat, steps):
    """Wall time and HIP-event time of `steps` steps on the lattice's stream."""
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / 1e3


def copy_bandwidth(torch, lbm, nbytes=1 << 30, reps=20, in_place=False):
    """Bytes read + written per second by the plain copy kernel over nbytes
    (in place: source and destination are the same buffer, as in the AA
    step)."""
    # non-zero data: zero pages move faster through the Infinity Cache
    src = torch.randint(1, 256, (nbytes,), dtype=torch.uint8, device="cuda")
    dst = src if in_place else torch.randint(1, 256, (nbytes,), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    lbm.copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, 2, stream.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lbm.copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, reps, stream.cuda_stream)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    return 2.0 * nbytes / sec / 1e9


def pattern_ceiling(torch, lbm, edge, elem_bytes, q=18, reps=20):
    """The AA step's access pattern without arithmetic (lbm_pattern_probe)
    over an edge^3 lattice with the library's own population stride, on
    non-zero data: microseconds of the even and of the odd pattern, and the
    algorithmic GB/s of the pair (2 q b bytes per node and step), the
    ceiling the step kernels' memory pattern allows, beside the plain
    copy."""
    N = edge ** 3
    stride = (N + 63) // 64 * 64 + 1088
    buf = torch.randint(1, 255, (q * stride * elem_bytes,), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    out = {}
    for odd in (False, True):
        lbm.pattern_probe(buf.data_ptr(), q, elem_bytes, (edge,) * 3, stride, odd, 2,
                          stream.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lbm.pattern_probe(buf.data_ptr(), q, elem_bytes, (edge,) * 3, stride, odd, reps,
                          stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        out["odd_us" if odd else "even_us"] = round(e0.elapsed_time(e1) * 1e3 / reps, 3)
    del buf
    mean_us = 0.5 * (out["even_us"] + out["odd_us"])
    out["GBs"] = round(2.0 * q * elem_bytes * N / mean_us / 1e3, 1)
    return out


def batch256(torch, lbm, params, steps=100):
    """256 lid-driven cavities (edge U{24..96}, Re U[100,1000], D3Q14 or
    D3Q18 at random, seed 0), FP32 AA, advanced together: one launch per
    time step and (q, storage) class, tiles chosen by the autotuner."""
    from paper_1503_03337_amd import autotune, inputs
    spec = inputs.cavity_batch(256, seed=0)

    def mk(q, edge):
        cfg = params.cavity(q, edge, 400.0)
        return lbm.Lattice(q, edge, edge, edge, cfg["s_vec"], faces=cfg["faces"],
                           wall_u=cfg["wall_u"], storage="f32", pattern="aa")
    tiles, _ = autotune.tune(mk, {(c["q"], c["edge"]) for c in spec})
    lats, b = [], lbm.Batch(torch.cuda.current_stream().cuda_stream)
    for c in spec:
        L = c["edge"]
        cfg = params.cavity(c["q"], L, c["Re"], lid=c["lid"])
        lat = lbm.Lattice(c["q"], L, L, L, cfg["s_vec"], faces=cfg["faces"],
                          wall_u=cfg["wall_u"], storage="f32", pattern="aa")
        b.add(lat, 10 ** 9)
        t = autotune.tile_for(tiles, c["q"], L)
        if t:
            b.set_tile(lat, *t)
        lats.append(lat)
    nodes = sum(l.N for l in lats)
    bytes_step = sum(2 * l.q * 4 * l.N for l in lats)
    b.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    b.close()
    for l in lats:
        l.close()
    return {"instances": len(spec), "nodes": nodes, "steps": steps,
            "aggregate_MLUPS": round(nodes * steps / sec / 1e6, 1),
            "achieved_GBs": round(bytes_step * steps / sec / 1e9, 1),
            "hbm_frac": round(bytes_step * steps / sec / (HBM_PEAK_GBS * 1e9), 4)}


def mrt_vs_lbgk(torch, lbm, params, n=128, steps=2000):
    """The same 128^3 D3Q18 FP32 cavity with the MRT collision and with the
    LBGK collision it reduces to for S = I/tau (Sec. 3): MLUPS of each."""
    cfg = params.cavity(18, n, 1000.0, lid=0.1)
    tau = 1.0 / cfg["s_vec"][8]
    out = {}
    for coll, s in (("mrt", cfg["s_vec"]), ("lbgk", [1.0 / tau] * 18)):
        lat = lbm.Lattice(18, n, n, n, s, faces=cfg["faces"], wall_u=cfg["wall_u"],
                          storage="f32", pattern="aa", collision="bgk" if coll == "lbgk" else "mrt")
        lat.step(1000)  # past the all-zero start (in-cache streaming depends on the data)
        wall, _ = time_steps(torch, lat, steps)
        lat.close()
        out[coll + "_MLUPS"] = round(n ** 3 * steps / wall / 1e6, 1)
    return out


def storage_variants(torch, lbm, params, n=128, develop=1000, steps=2000):
    """The headline cavity (128^3 D3Q18, AA, MRT) stored as FP64 (288 B per
    node and step), FP32 (144 B) and FP16 deviations (72 B): MLUPS and
    algorithmic GB/s of each over `steps` steps after `develop` untimed
    ones, read against the ceiling of the access pattern in that element
    size (lbm_swap_probe), and the relative L2 error of u and p of the FP32 and FP16 runs
    against the FP64 run at the same time level (develop + steps)."""
    cfg = params.cavity(18, n, 1000.0, lid=0.1)
    out, fields = {}, {}
    for storage, b in (("f64", 8), ("f32", 4), ("f16dev", 2)):
        lat = lbm.Lattice(18, n, n, n, cfg["s_vec"], faces=cfg["faces"], wall_u=cfg["wall_u"],
                          storage=storage, pattern="aa")
        lat.step(develop)
        wall, ev = time_steps(torch, lat, steps)
        fields[storage] = lat.macros()
        lat.close()
        gbs = 2 * 18 * b * n ** 3 * steps / ev / 1e9
        ceil = pattern_ceiling(torch, lbm, n, b)
        ceil["step_frac"] = round(gbs / ceil["GBs"], 4)
        out[storage] = {"MLUPS": round(n ** 3 * steps / wall / 1e6, 1),
                        "algorithmic_GBs": round(gbs, 1), "pattern_ceiling": ceil}
    p64, u64 = fields["f64"]
    for storage in ("f32", "f16dev"):
        p, u = fields[storage]
        out[storage]["rel_l2_u_vs_f64"] = float("%.3e" % rel_l2(u, u64))
        out[storage]["rel_l2_p_vs_f64"] = float("%.3e" % rel_l2(p, p64))
    out["time_level"] = develop + steps
    return out


def model_variants(torch, lbm, params, n=128, develop=1000, steps=2000):
    """The headline cavity (128^3, AA, FP32, MRT) with the 14- and the
    26-velocity models (Sec. 3; the closing paragraph of Appendix B):
    MLUPS and algorithmic GB/s at 2 q 4 bytes per node and step, read
    against the ceiling of the q-array access pattern (lbm_swap_probe)."""
    out = {}
    for q in (14, 26):
        cfg = params.cavity(q, n, 1000.0, lid=0.1)
        lat = lbm.Lattice(q, n, n, n, cfg["s_vec"], faces=cfg["faces"], wall_u=cfg["wall_u"],
                          storage="f32", pattern="aa")
        lat.step(develop)
        wall, ev = time_steps(torch, lat, steps)
        lat.close()
        gbs = 2 * q * 4 * n ** 3 * steps / ev / 1e9
        ceil = pattern_ceiling(torch, lbm, n, 4, q=q)
        ceil["step_frac"] = round(gbs / ceil["GBs"], 4)
        out["d3q%d" % q] = {"MLUPS": round(n ** 3 * steps / wall / 1e6, 1),
                            "algorithmic_GBs": round(gbs, 1), "pattern_ceiling": ceil}
    return out


def zero_fraction(lat):
    """Fraction of the lattice's physical populations that are exactly 0."""
    import numpy as np
    f = lat.get_f()
    return float(np.count_nonzero(f == 0.0)) / f.size


def monitor_cost(torch, lat, reps=10):
    """Average device time of one FP64 monitor pass (mass, residual
    partial sums, velocity snapshot and the final reduction), timed with
    HIP events on the lattice's stream."""
    stream = torch.cuda.current_stream()
    lat.monitor()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        lat.monitor()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def rel_l2(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cpu_baseline(target_seconds=15.0):
    """The FP64 oracle on the host cores: 128^3 D3Q18 cavity from rest."""
    import numpy as np
    from oracle import runner as R
    from paper_1503_03337_amd import params
    n = 128
    cfg = params.cavity(18, n, 1000.0, lid=0.1)
    pr = R.problem(18, n, n, n, cfg["s_vec"], faces=cfg["faces"], wall_u=cfg["wall_u"])
    f = R.init_eq(pr)
    t0 = time.perf_counter()
    f = R.run(pr, f, 0, 1)
    one = time.perf_counter() - t0
    k = max(1, int(target_seconds / max(one, 1e-3)))
    t0 = time.perf_counter()
    f = R.run(pr, f, 1, k)
    sec = time.perf_counter() - t0
    assert np.isfinite(f).all()
    return {"value": round(n ** 3 * k / sec / 1e6, 3), "unit": "MLUPS", "cores": R.threads(),
            "kind": "oracle",
            "sample": "D3Q18 128^3 lid-driven cavity, FP64, %d step(s) from rest (%.1f s), "
                      "OpenMP over z planes" % (k, sec)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--develop", type=int, default=1000,
                    help="untimed steps before --warmup that develop the flow from rest")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--headline-only", action="store_true",
                    help="time the headline lattice and the copy reference only (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one MI355X; runs over several GPUs are not supported "
              "(--gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1503_03337_amd import lbm, params
    torch.cuda.set_device(0)
    n = args.size
    N = n ** 3
    K = 1000  # monitor interval of the headline lattice
    lat = cavity_lattice(lbm, params, n, monitor_every=K)
    lat.step(args.develop)
    zeros = zero_fraction(lat)
    note("developed %d steps, %.4f %% of populations exactly zero" % (args.develop, 100 * zeros))
    if zeros >= 0.01:
        print("bench.py: %.1f %% of the populations are still exactly zero after %d "
              "development steps; the timed steps would stream zeros (raise --develop)"
              % (100.0 * zeros, args.develop), file=sys.stderr)
        sys.exit(3)
    lat.step(args.warmup)
    t_begin = lat.time
    wall, ev = time_steps(torch, lat, args.steps)
    mlups = N * args.steps / wall / 1e6
    t_end = lat.time
    # residual of the paper's steady-state criterion over the lag since the
    # last monitor snapshot (the monitor runs every K steps inside lbm_step)
    # (a run at t_end already happened inside lbm_step when K divides t_end;
    # a second one at the same time level would have no lag)
    if t_end % K:
        lat.monitor()
    r_change, r_lag = lat.residual_change()
    res = {"value": r_change, "lag_steps": r_lag,
           "per_step": r_change / r_lag if r_lag > 0 else None,
           "norm": "sum |u(t) - u(t - lag)| / sum |u(t)| over nodes and components"}
    mon_us = monitor_cost(torch, lat)
    lat.close()
    note("headline %.1f MLUPS over %d steps" % (mlups, args.steps))
    # monitor passes inside the timed window (t a multiple of K)
    n_mon = t_end // K - t_begin // K
    step_us = (ev * 1e6 - n_mon * mon_us) / args.steps

    bytes_per_node = 2 * 18 * 4
    achieved = bytes_per_node * N / step_us / 1e3
    traffic = measured_traffic()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic}

    copy_gbs = copy_bandwidth(torch, lbm)
    copy_inplace_gbs = copy_bandwidth(torch, lbm, in_place=True)
    ceiling = pattern_ceiling(torch, lbm, n, 4)
    ceiling["step_frac"] = round(achieved / ceiling["GBs"], 4)
    extras = {}
    if not args.headline_only:
        # the same kernels on a lattice larger than the 256 MB Infinity Cache
        big = cavity_lattice(lbm, params, 256, monitor_every=0)
        big.step(400)
        bsteps = 200
        bwall, bev = time_steps(torch, big, bsteps)
        big.close()
        big_gbs = bytes_per_node * 256 ** 3 / (bev / bsteps) / 1e9
        big_ceiling = pattern_ceiling(torch, lbm, 256, 4)
        big_ceiling["step_frac"] = round(big_gbs / big_ceiling["GBs"], 4)
        extras["cavity256"] = {
            "MLUPS": round(256 ** 3 * bsteps / bwall / 1e6, 1),
            "achieved_GBs": round(big_gbs, 1),
            "pattern_ceiling": big_ceiling}
        note("256^3 done")
        extras["batch256"] = batch256(torch, lbm, params)
        note("256-cavity batch done")
        extras["collision_cost"] = mrt_vs_lbgk(torch, lbm, params)
        note("collision comparison done")
        extras["storage_variants"] = storage_variants(torch, lbm, params)
        note("storage variants done")
        extras["model_variants"] = model_variants(torch, lbm, params)
        note("model variants done")

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D3Q18 MRT lid-driven cavity %d^3, Re=1000 (nu=%.4g), lid 0.1, "
                               "FP32 SoA populations, AA in-place streaming, FP64 monitor every "
                               "%d steps" % (n, 0.1 * n / 1000.0, K),
                   "nodes": N, "bytes_per_node_step": bytes_per_node,
                   "develop_steps": args.develop,
                   "zero_populations_before_timing": round(zeros, 6),
                   "timed_time_levels": [t_begin, t_end]},
        "roofline": roofline,
        "step_kernel_us": round(step_us, 3),
        "monitor": {"us_per_pass": round(mon_us, 2), "every_steps": K,
                    "amortised_us_per_step": round(mon_us / K, 4),
                    "passes_in_timed_window": n_mon},
        "hbm_roofline_fraction": round(mlups * 1e6 * bytes_per_node / (HBM_PEAK_GBS * 1e9), 4),
        "residual_at_end": res,
        "copy_probe_GBs": round(copy_gbs, 1),
        "copy_probe_inplace_GBs": round(copy_inplace_gbs, 1),
        "pattern_ceiling": ceiling,
    }
    out.update(extras)
    if not args.no_serving and not args.headline_only:
        from paper_1503_03337_amd import serve
        out["serving"] = serve.bench_summary()
        note("serving done")
    if not args.no_cpu_baseline and not args.headline_only:
        out["cpu_baseline"] = cpu_baseline()
        note("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

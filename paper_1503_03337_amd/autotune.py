"""Tile-shape autotuner for batched execution.

A workgroup of the batched kernel covers either 256 consecutive nodes of
its member (the automatic "flat" mapping, tile (0, 0): every wavefront full
and aligned whatever the edge) or a tx x ty tile of one x-y plane (tx * ty
<= 256 threads).  The best choice depends on the edge length and on q.  For
every (q, edge bucket) present in a batch the tuner times each candidate on
a batch of copies of that bucket's median member, large enough (>= 2^22
nodes) to run from HBM as the real batch does, and keeps the fastest.  The
timing lattices first run `warm` steps (the lid drives them away from the
all-zero start, which streams faster than developed flow), each candidate is
timed `reps` times and its best kept, and a tile must beat the flat mapping
by `margin` to replace it (differences below that are timing noise).  The
mapping never changes results (each node's arithmetic is the same), only
speed.
"""
import time

from . import lbm


def candidates(edge):
    """Mappings worth trying for rows of `edge` nodes: flat, then tiles."""
    out = [(0, 0)]
    if edge <= 256:
        out.append((edge, max(1, min(edge, 256 // edge))))
    for tx in (256, 128, 64, 32, 16):
        if tx <= max(16, 2 * edge):
            out.append((tx, max(1, 256 // tx)))
    seen, uniq = set(), []
    for t in out:
        if t not in seen:
            seen.add(t)
            uniq.append(t)
    return uniq


def bucket(edge, width=8):
    return (edge // width) * width


def tune(make_lattice, keys, steps=40, reps=3, stream=None, sync=None, min_nodes=1 << 22,
         warm=200, margin=0.02):
    """keys: iterable of (q, edge).  make_lattice(q, edge) returns a fresh
    lbm.Lattice (FP32 or FP16DEV, AA).  Returns {(q, bucket(edge)): (tx, ty)}
    ((0, 0): the flat mapping) and the measured MLUPS per candidate."""
    import torch
    best, log = {}, {}
    groups = {}
    for q, edge in keys:
        groups.setdefault((q, bucket(edge)), []).append(edge)
    for (q, bk), edges in sorted(groups.items()):
        sample = sorted(edges)[len(edges) // 2]
        copies = max(2, -(-min_nodes // sample ** 3))
        lats = [make_lattice(q, sample) for _ in range(copies)]
        nodes = sum(l.N for l in lats)
        if warm > 0:
            b = lbm.Batch(lats[0].stream)
            for l in lats:
                b.add(l, 10 ** 9)
            b.step(warm)
            b.close()
        results = {}
        for tile in candidates(sample):
            b = lbm.Batch(lats[0].stream)
            for l in lats:
                b.add(l, 10 ** 9)
                b.set_tile(l, *tile)
            b.step(4)
            torch.cuda.synchronize()
            t = float("inf")
            for _ in range(reps):
                t0 = time.perf_counter()
                b.step(steps)
                torch.cuda.synchronize()
                t = min(t, time.perf_counter() - t0)
            b.close()
            results[tile] = nodes * steps / t / 1e6
        for l in lats:
            l.close()
        pick = max(results, key=results.get)
        if results[pick] < (1.0 + margin) * results[(0, 0)]:
            pick = (0, 0)
        best[(q, bk)] = pick
        log[(q, bk)] = results
    return best, log


def tile_for(table, q, edge):
    return table.get((q, bucket(edge)))

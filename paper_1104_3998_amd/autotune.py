"""Timed choice of the tile geometry: cells per tile C and window D per species.

The library's default geometry follows a rule per discharge and species. An electron tile
holds about 2e3 null-collision candidates, an ion tile about 2.5e3 particles, and the
windows are 32 / 4 cells. The tuner starts from that rule and times scaled versions of it
for every discharge at once, one factor at a time:
* electron C ×{1/2, 1, 2};
* then ion C ×{1, 2};
* then electron D ×{1, 1/2}.

It keeps the fastest. Tile geometry changes speed only: the output order is the stable
sort by cell whatever the tiles, and the charge is summed in fixed point, so the results
are bit for bit the same. A candidate the library rejects, or one that overflows a list
while it is timed, is skipped.

Each candidate is timed as steps replayed from a HIP graph, after warm-up steps, from
the seeded load, between HIP events on the simulation's stream. The choice can be cached
in a JSON file keyed by the workloads, the layout, the step counts and the device name.
"""
import hashlib
import json
import os

from . import PicError, Simulation, derive, make_config

_MAX_CELLS_PER_TILE = 64


def rule_geometry(wls, precision):
    """The library's default (C, D) per species for each discharge."""
    out = []
    for w in wls:
        d = derive(make_config(w, precision))
        out.append(((int(d.cells_per_tile[0]), int(d.window[0])),
                    (int(d.cells_per_tile[1]), int(d.window[1]))))
    return out


def scaled_tuning(rule, fe, fi, fd):
    """Per-discharge tuning dicts: electron C × fe, ion C × fi, electron D × fd, from the
    rule's geometry `rule` (as rule_geometry returns it); C stays in [1, 64], D >= 1."""
    out = []
    for (ce, de), (ci, di) in rule:
        c_e = max(1, min(_MAX_CELLS_PER_TILE, int(round(ce * fe))))
        c_i = max(1, min(_MAX_CELLS_PER_TILE, int(round(ci * fi))))
        d_e = max(1, int(round(de * fd)))
        out.append({"cells_per_tile": (c_e, c_i), "window": (d_e, max(di, 1))})
    return out


def _rate(wls, precision, tuning, steps, warmup, cap_factor, graph_k):
    import torch
    sim = Simulation(wls, precision, tuning=tuning, cap_factor=cap_factor)
    try:
        sim.set_graph(graph_k)
        sim.step(warmup)
        sim.sync()
        ps0 = sum(sum(sim.diagnostics(d).particle_steps) for d in range(len(wls)))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.step(steps)
        e1.record(sim.stream)
        e1.synchronize()
        sim.sync()  # raises on a device-side error (a list that overflowed)
        ps1 = sum(sum(sim.diagnostics(d).particle_steps) for d in range(len(wls)))
        return (ps1 - ps0) / (e0.elapsed_time(e1) / 1e3)
    finally:
        sim.close()
        del sim
        torch.cuda.empty_cache()


def _key(wls, precision, steps, warmup):
    import torch
    blob = json.dumps({"wls": wls, "precision": precision, "steps": steps, "warmup": warmup,
                       "device": torch.cuda.get_device_name()}, sort_keys=True, default=str)
    return hashlib.sha256(blob.encode()).hexdigest()[:24]


def autotune(workloads, precision="fp32_offset", steps=30, warmup=20, cap_factor=1.5,
             graph_k=10, cache=None, log=None):
    """Returns (tuning, report): the per-discharge tuning list of the fastest geometry
    found, and a dict with the factors and the particle-steps/s of every timed candidate.
    With `cache` (a JSON file path), a previous result for the same key is returned
    without timing, and a new one is stored."""
    wls = [dict(w) for w in (workloads if isinstance(workloads, (list, tuple)) else [workloads])]
    key = _key(wls, precision, steps, warmup)
    store = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            store = json.load(fh)
        if key in store:
            rep = store[key]
            rule = rule_geometry(wls, precision)
            return scaled_tuning(rule, *rep["best"]), rep
    rule = rule_geometry(wls, precision)
    timed = {}

    def rate(f):
        if f not in timed:
            try:
                timed[f] = _rate(wls, precision, scaled_tuning(rule, *f), steps, warmup,
                                 cap_factor, graph_k)
            except PicError as e:
                timed[f] = None
                if log:
                    log("autotune: factors %s rejected: %s" % (f, e))
            if log and timed[f] is not None:
                log("autotune: factors %s -> %.4e particle-steps/s" % (f, timed[f]))
        return timed[f] if timed[f] is not None else -1.0

    best = (1.0, 1.0, 1.0)
    for axis, values in ((0, (1.0, 0.5, 2.0)), (1, (1.0, 2.0)), (2, (1.0, 0.5))):
        for v in values:
            f = tuple(v if i == axis else best[i] for i in range(3))
            if rate(f) > rate(best):
                best = f
    rep = {"best": list(best), "rule_rate": timed.get((1.0, 1.0, 1.0)),
           "best_rate": timed.get(best),
           "timed": [{"factors": list(f), "rate": r} for f, r in timed.items()]}
    if cache:
        store[key] = rep
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as fh:
            json.dump(store, fh, indent=1)
    return scaled_tuning(rule, *best), rep

"""Benchmark of the PIC-MCC hot path on one MI355X.

Prints ONE JSON line.  The headline `value` is particle-steps/s of the FP32 cell + offset
path on the large single discharge (4096 cells, 1e7 electrons + 1e7 ions, 5 Pa Ar-like
gas, 300 V at 13.56 MHz, sorted by cell every step with the lagged counting sort (--sort
counting: keyed on the post-push cell)), inputs resident in HBM, the K timed steps
(steps W+1 .. W+K after the load, named in config.window) replayed from a captured HIP
graph of a divisor of K steps and timed with HIP events on the library's stream.  The
same W + K steps are then run again from the same seeded load with eager launches, every
kernel bracketed by HIP events recorded by its own launch: the per-kernel durations of
the K timed steps give the roofline of the dominant kernel (k_main).  The runs are bit
for bit deterministic, so both time the same work.  Under "paths": the FP64 path, the
other sort, the unsorted variant, the paper's in-place fine sort over sorting-cell sizes,
the long-run discharge (8192 cells, 3.2e7 + 3.2e7), each from its load, and the batched
256-discharge scan against the same discharges run one at a time.  The density gate
(FP32 against FP64 on the large discharge, with controls and a paired-seed ensemble) and
the bounded RF discharge against the oracle come alongside, and the oracle's CPU speed
on bounded samples of the workloads.  --long-run-study adds the long run's precision
study (minutes).

`python bench.py --skip-paths --skip-cpu --gate-steps 0` runs only the two headline runs;
that is the command whose rocprofv3 kernel statistics are kept beside the code.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-paths] [--skip-cpu]
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

METRIC = "particle-steps/s: FP32-offset vs FP64 vs batched, at ≤1e-3 density err"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per particle-step of the fused pass: the whole record read once and
# written once (FP32 cell + offset: 24 B record; FP64: 36 B record)
REC_BYTES = {"fp32_offset": 24, "fp64": 36}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels_step.hip", "device_common.h", "sim_layout.h", "physics_host.cpp"):
        with open(os.path.join(ROOT, "paper_1104_3998_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(precision):
    """HBM traffic of k_main per particle-step from the committed rocprofv3 PMC summary,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "k_main_%s_large_pmc.md" % precision)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel source hash:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"hbm bytes per particle-step:\s*([0-9.eE+-]+)", txt)
    if not m_hash or not m_b or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_b.group(1))


PROGRESS_STEPS = 0  # --progress N: report every N warm-up steps
SORT = "lag"        # --sort: the sort of the headline and the gates


def _psteps(sim):
    return sum(sum(sim.diagnostics(d).particle_steps) for d in range(len(sim.workloads)))


def _timed_run(fs, torch, wls, precision, steps, warmup, graph_k, profile, tuning,
               cap_factor):
    """One run of warmup + timed steps from a fresh load.  With graph_k the steps replay a
    captured HIP graph of graph_k steps; with profile they launch eagerly, each kernel
    bracketed by HIP events (library stream), and the per-kernel durations of the timed
    steps are returned."""
    sim = fs.Simulation(wls, precision, tuning=tuning, cap_factor=cap_factor)
    stream = sim.stream
    if graph_k:
        sim.set_graph(graph_k)
    if profile:
        sim.profile(True)
    done = 0
    while done < warmup:  # in pieces, so a slow (profiled) run reports its progress
        k = min(PROGRESS_STEPS, warmup - done) if PROGRESS_STEPS else warmup
        sim.step(k)
        done += k
        if PROGRESS_STEPS:
            sim.sync()
            print("bench: warm-up %d/%d steps" % (done, warmup), file=sys.stderr, flush=True)
    sim.sync()
    if profile:
        sim.profile(True)  # drop the warm-up steps from the totals
    ps0 = _psteps(sim)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    e1.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    sim.sync()
    ps1 = _psteps(sim)
    out = {"value": (ps1 - ps0) / (ms / 1e3), "ms_per_step": ms / steps, "wall_s": wall,
           "particle_steps": ps1 - ps0,
           "particles_end": int(sum(sum(sim.diagnostics(d).n_particles)
                                    for d in range(len(sim.workloads))))}
    if profile:
        prof = sim.profile_read()
        out["kernel_ms"] = {k: v[0] / max(v[1], 1) for k, v in prof.items()}
        out["kernel_launches"] = {k: v[1] for k, v in prof.items()}
        sim.profile(False)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def graph_length(steps, most=50):
    """The largest graph length <= most that divides `steps`, so that every timed step is
    replayed from the captured graph."""
    return max(k for k in range(1, min(most, steps) + 1) if steps % k == 0)


def run_path(fs, torch, wls, precision, steps, warmup, tuning=None, cap_factor=1.5,
             eager=True):
    """The same trajectory twice from the same seeded load: replayed from a HIP graph
    (the throughput `value`), then eagerly with per-kernel events over the same timed
    steps (the kernel durations).  The runs are bit for bit deterministic, so both time
    the same work."""
    k = graph_length(steps)
    g = _timed_run(fs, torch, wls, precision, steps, warmup, k, False, tuning, cap_factor)
    out = {"value": g["value"], "ms_per_step": g["ms_per_step"], "wall_s": g["wall_s"],
           "particle_steps": g["particle_steps"], "particles_end": g["particles_end"],
           "steps": steps, "warmup": warmup, "graph_steps": k, "graph_replays": steps // k}
    if eager:
        e = _timed_run(fs, torch, wls, precision, steps, warmup, 0, True, tuning, cap_factor)
        out.update({"eager_value": e["value"], "eager_ms_per_step": e["ms_per_step"],
                    "eager_particle_steps": e["particle_steps"], "kernel_ms": e["kernel_ms"]})
    return out


def _averages(fs, torch, wl, precision, steps, tuning=None, state=None, keep_state=False,
              cap_factor=1.5):
    """Time-averaged n_e, n_i, Phi (over the workload's averaging window) and the EEDF
    histogram after `steps` graph-replayed steps from the seeded load (or from `state`)."""
    import numpy as np
    sim = fs.Simulation(wl, precision, tuning=tuning, cap_factor=cap_factor)
    if state is not None:
        sim.set_state(state)
    sim.set_graph(graph_length(steps))
    sim.step(steps)
    sim.sync()
    out = {"n_e": sim.density("n_e", kind=1), "n_i": sim.density("n_i", kind=1),
           "phi": sim.density("phi", kind=1), "eedf": sim.grid("eedf").astype(np.float64)}
    if keep_state:
        out["state"] = sim.get_state()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


QUANT = ("n_e", "n_i", "phi", "eedf")


def _norm_eedf(a):
    return dict(a, eedf=a["eedf"] / max(a["eedf"].sum(), 1.0))


def rel_l2(a, b):
    import numpy as np
    a, b = _norm_eedf(a), _norm_eedf(b)
    return {k: float(np.linalg.norm(a[k] - b[k]) / max(np.linalg.norm(b[k]), 1e-300))
            for k in QUANT}


def _rounded_fp64_state(fs, wl):
    """The FP32 layout's load (cell + FP32 offset, FP32 velocities) as an FP64 state."""
    import numpy as np
    sim = fs.Simulation(wl, "fp32_offset")
    st = sim.get_state()
    sim.close()
    st64 = {"step": st["step"], "next_id": st["next_id"]}
    for s in (0, 1):
        a = st[s]
        st64[s] = {"x": a["cell"].astype(np.float64) + a["off"].astype(np.float64),
                   "vx": a["vxf"].astype(np.float64), "vy": a["vyf"].astype(np.float64),
                   "vz": a["vzf"].astype(np.float64), "id": a["id"], "n": a["n"],
                   "n_sorted": a["n_sorted"]}
    return st64


def density_gate(fs, torch, workloads, steps, seeds):
    """The accuracy gate of the metric on the large discharge: time-averaged n_e, n_i, Phi
    over the second half of `steps` steps and the normalised EEDF, by rel-L2 over nodes
    (bins), FP32 cell + offset against FP64.
    * same seed, same load (the FP32 state is the FP64 draw rounded): the headline pair;
    * FP64 started from the FP32-rounded load against FP32: the two layouts from the
      identical state, so the difference is the FP32 arithmetic alone;
    * FP32 run twice: bit-for-bit equality (the charge is summed in fixed point and every
      floating-point sum in a fixed order), so the path adds no noise of its own;
    * FP64 from the FP32-rounded load against FP64: what a 1e-7 perturbation of the state
      does by itself (collision decisions flip and the plasma is chaotic);
    * FP64 seed + 1 against FP64: the statistical floor;
    * an ensemble of `seeds` paired seeds: the mean over seeds of the FP32 - FP64
      difference of the averages (systematic error of the FP32 layout) with its standard
      error (what chaos alone leaves in a mean over that many pairs)."""
    import numpy as np
    wl = workloads.large_c3(avg_start=steps // 2, sort_mode=SORT)
    ref = _averages(fs, torch, wl, "fp64", steps)
    f32 = _averages(fs, torch, wl, "fp32_offset", steps, keep_state=True)
    f32b = _averages(fs, torch, wl, "fp32_offset", steps, keep_state=True)
    repeat_equal = all(np.array_equal(f32[k], f32b[k]) for k in QUANT) and all(
        np.array_equal(f32["state"][s][f].view(np.uint8), f32b["state"][s][f].view(np.uint8))
        for s in (0, 1) for f in ("cell", "off", "vxf", "vyf", "vzf", "id"))
    del f32["state"], f32b
    seed1 = _averages(fs, torch, workloads.large_c3(avg_start=steps // 2, seed=1,
                                                    sort_mode=SORT), "fp64", steps)
    st64 = _rounded_fp64_state(fs, wl)
    pert = _averages(fs, torch, wl, "fp64", steps, state=st64)
    del st64
    d32 = rel_l2(f32, ref)
    # ensemble of paired seeds
    diffs = {k: [] for k in QUANT}
    refs = {k: [] for k in QUANT}
    pairs = []
    for seed in range(100, 100 + seeds):
        w = workloads.large_c3(avg_start=steps // 2, seed=seed, sort_mode=SORT)
        a = _norm_eedf(_averages(fs, torch, w, "fp32_offset", steps))
        b = _norm_eedf(_averages(fs, torch, w, "fp64", steps))
        pairs.append(rel_l2(a, b))
        for k in QUANT:
            diffs[k].append(a[k] - b[k])
            refs[k].append(b[k])
    ens = {}
    if seeds > 1:
        for k in QUANT:
            dk = np.array(diffs[k])
            scale = np.linalg.norm(np.mean(refs[k], axis=0))
            ens[k] = {"systematic_rel_l2": float(np.linalg.norm(dk.mean(0)) / scale),
                      "stderr_rel_l2": float(np.linalg.norm(dk.std(0, ddof=1)) /
                                             np.sqrt(len(dk)) / scale),
                      "pair_rel_l2_median": float(np.median([p_[k] for p_ in pairs]))}
    return {"workload": "large single discharge, %d steps from the load, averages over "
                        "steps %d..%d" % (steps, steps // 2, steps),
            "fp32_offset_vs_fp64": d32,
            "fp32_offset_vs_fp64_same_rounded_state": rel_l2(f32, pert),
            "fp32_offset_repeat_bitwise_equal": bool(repeat_equal),
            "fp64_from_fp32_rounded_load_vs_fp64": rel_l2(pert, ref),
            "floor_fp64_seed_plus_1": rel_l2(seed1, ref),
            "ensemble": {"seeds": seeds, "per_quantity": ens},
            "max_fp32_offset_vs_fp64": max(d32.values()),
            "within_1e-3": max(d32.values()) <= 1e-3,
            "note": "n_i of a single pair exceeds 1e-3 for any 1e-7 perturbation of the "
                    "state (FP64 from the rounded load diverges as far): the systematic "
                    "part of the FP32 error is the ensemble's systematic_rel_l2 against "
                    "its stderr"}


def oracle_averages(wl, steps, progress=None, cap_factor=1.5):
    """The FP64 oracle's time averages over the workload's window (same keys as
    _averages), run on the host (in pieces of 1000 steps, each reported to `progress`)."""
    import numpy as np
    import oracle
    orc = oracle.Oracle(wl, cap_e=int(wl["n_e0"] * cap_factor) + 1024,
                        cap_i=int(wl["n_i0"] * cap_factor) + 1024)
    orc.load()
    done = 0
    while done < steps:
        k = min(1000, steps - done)
        orc.step(k)
        done += k
        if progress:
            progress("oracle %d/%d steps" % (done, steps))
    t = orc.tallies()
    c = orc.consts()
    n = max(int(t.acc_count), 1)
    f = c.weight_per_area / c.dx / n
    out = {}
    for k, g in (("n_e", "acc_w_e"), ("n_i", "acc_w_i")):
        a = orc.grid(g) * f
        if not wl["periodic"]:
            a[0] *= 2
            a[-1] *= 2
        out[k] = a
    out["phi"] = orc.grid("acc_phi") / n * c.phi_scale
    out["eedf"] = orc.grid("eedf").astype(np.float64)
    return out


def rf_gate(fs, torch, workloads, steps):
    """The bounded RF discharge at its size (2.5 cm, 512 cells, 2e5 + 2e5, 10 Pa, 200 V):
    time averages over the last RF cycle of `steps` steps from the FP64 GPU path against
    the FP64 oracle run on the host from the same seed, with the FP64 seed + 1 run as the
    statistical floor, and the FP32 layout against FP64."""
    wl = workloads.rf_c2(steps=steps, avg_start=max(0, steps - 400), sort_mode=SORT)
    g64 = _averages(fs, torch, wl, "fp64", steps)
    g32 = _averages(fs, torch, wl, "fp32_offset", steps)
    seed1 = _averages(fs, torch, workloads.rf_c2(steps=steps, avg_start=max(0, steps - 400),
                                                 seed=1, sort_mode=SORT), "fp64", steps)
    t0 = time.perf_counter()
    orc = oracle_averages(wl, steps, progress=lambda m: print("bench: rf gate: " + m,
                                                             file=sys.stderr, flush=True))
    return {"workload": "bounded RF discharge 2e5 + 2e5, %d steps, averages over the last "
                        "400" % steps,
            "fp64_vs_oracle": rel_l2(g64, orc), "fp32_offset_vs_fp64": rel_l2(g32, g64),
            "floor_fp64_seed_plus_1": rel_l2(seed1, g64),
            "oracle_seconds": time.perf_counter() - t0}


def long_run_study(fs, torch, workloads, steps, sub_steps):
    """The long run: FP32 against FP64 at full size (8192 cells, 3.2e7 + 3.2e7) over
    `steps` steps, and the FP64 GPU path against the oracle at the 1e5-per-species
    subsample over `sub_steps` steps, with the seed + 1 floors."""
    def log(m):
        print("bench: long-run study: " + m, file=sys.stderr, flush=True)

    half = steps // 2
    wl = workloads.long_c5(avg_start=half, sort_mode=SORT)
    # the discharge ionises its way up from the load: room for twice the load (the most
    # the library allows at 3.2e7 per species: capacities stay below 2^26)
    cf = 2.0
    log("full size, FP64")
    r64 = _averages(fs, torch, wl, "fp64", steps, cap_factor=cf)
    log("full size, FP32 cell+offset")
    r32 = _averages(fs, torch, wl, "fp32_offset", steps, cap_factor=cf)
    log("full size, FP64, seed + 1")
    s1 = _averages(fs, torch, workloads.long_c5(avg_start=half, seed=1, sort_mode=SORT), "fp64",
                   steps, cap_factor=cf)
    sub = workloads.long_c5(n_e0=100_000, n_i0=100_000, avg_start=sub_steps // 2,
                            sort_mode=SORT)
    log("subsample, FP64, seeds 0..4")
    g = _averages(fs, torch, sub, "fp64", sub_steps, cap_factor=cf)
    others = [_averages(fs, torch, dict(sub, seed=k), "fp64", sub_steps, cap_factor=cf)
              for k in range(1, 5)]
    g1 = others[0]
    spread = [rel_l2(o_, g) for o_ in others]
    log("subsample, oracle on the host")
    t0 = time.perf_counter()
    o = oracle_averages(sub, sub_steps, progress=log, cap_factor=cf)
    return {"full_size": {"steps": steps, "fp32_offset_vs_fp64": rel_l2(r32, r64),
                          "floor_fp64_seed_plus_1": rel_l2(s1, r64)},
            "subsample_1e5": {"steps": sub_steps, "fp64_vs_oracle": rel_l2(g, o),
                              "floor_fp64_seed_plus_1": rel_l2(g1, g),
                              "floor_fp64_seeds_1_to_4": {
                                  k: sorted(x[k] for x in spread) for k in QUANT},
                              "oracle_seconds": time.perf_counter() - t0}}


def sequential_sample(fs, torch, wls, tuning, steps, warmup, every=4, cap_factor=4.0):
    """The batched scan's alternative: the same discharges run one at a time, each from its
    own load with its own HIP graph, timed over the same steps.  Every `every`-th discharge
    is run; the aggregate rate is their particle-steps over their summed time."""
    ps, secs, picked = 0, 0.0, list(range(0, len(wls), every))
    k = graph_length(steps)
    for d in picked:
        t = [tuning[d]] if isinstance(tuning, (list, tuple)) else tuning
        r = _timed_run(fs, torch, [wls[d]], "fp32_offset", steps, warmup, k, False, t,
                       cap_factor)
        ps += r["particle_steps"]
        secs += r["ms_per_step"] * steps / 1e3
    return {"value": ps / secs, "discharges_run": len(picked), "of": len(wls),
            "steps": steps, "note": "every %dth discharge of the scan run alone, each "
                                    "graph-replayed; rate = their particle-steps / their "
                                    "summed time" % every}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(wl, steps, repeats=3):
    """Median over `repeats` of the oracle's particle-steps/s over `steps` steps after the
    load (each repeat from a fresh load)."""
    import oracle
    rates, secs = [], 0.0
    for _ in range(repeats):
        orc = oracle.Oracle(wl)
        orc.load()
        tot = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            tot += orc.count(0) + orc.count(1)
            orc.step(1)
        dt = time.perf_counter() - t0
        secs += dt
        rates.append(tot / dt)
        del orc
    rates.sort()
    return rates[len(rates) // 2], secs


def cpu_baseline(workloads, steps):
    """The oracle (plain sequential C, FP64, one thread) on bounded samples: the headline
    workload for `steps` steps (the value), and, alongside, the periodic plasma in full,
    the bounded RF discharge for 100 steps and the long run's 1e5-per-species subsample
    for 500 steps."""
    v, secs = _oracle_rate(workloads.large_c3(), steps)
    others = {}
    for name, wl, n in (("periodic plasma, full (200 steps)", workloads.periodic_c1(), 200),
                        ("bounded RF discharge 2e5 + 2e5, 100 steps", workloads.rf_c2(), 100),
                        ("long run subsample 1e5 + 1e5, 500 steps",
                         workloads.long_c5(n_e0=100_000, n_i0=100_000), 500)):
        r, t = _oracle_rate(wl, n, repeats=1)
        others[name] = r
        secs += t
    return {"value": v, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": "large single discharge at full size (2e7 particles), %d oracle steps "
                      "after the load, median of 3 loads, single-threaded C, FP64" % steps,
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "seconds": secs,
            "others": others}


def copy_ceiling(torch):
    """GB/s of a plain 1 GiB device copy (bytes read + bytes written), the practical HBM
    ceiling the kernels are compared with beside the 8 TB/s peak."""
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del a, b
    torch.cuda.empty_cache()
    return 8 * n / (ms / 1e3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--skip-paths", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--path-steps", type=int, default=400)
    ap.add_argument("--batched-scale", type=float, default=1.0)
    ap.add_argument("--seq-every", type=int, default=4,
                    help="the batched scan's sequential baseline runs every N-th discharge")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched path: the library's default tile geometry, untuned")
    ap.add_argument("--gate-steps", type=int, default=2000,
                    help="steps of the FP32-vs-FP64 density gate runs (0: skip)")
    ap.add_argument("--gate-seeds", type=int, default=4,
                    help="paired seeds of the gate's ensemble")
    ap.add_argument("--rf-gate-steps", type=int, default=2000,
                    help="steps of the bounded RF discharge's oracle comparison (0: skip)")
    ap.add_argument("--long-run-study", type=int, nargs=2, default=None,
                    metavar=("STEPS", "SUB_STEPS"),
                    help="the long run's precision study (full-size FP32 vs FP64 over STEPS, "
                         "FP64 vs the oracle at the subsample over SUB_STEPS); off by default")
    ap.add_argument("--mode", choices=["bench", "copy"], default="bench",
                    help="copy: a plain device copy of known size that calibrates the HBM "
                         "byte counters of rocprofv3")
    ap.add_argument("--progress", type=int, default=0,
                    help="report every N warm-up steps on stderr (for slow profiled runs)")
    ap.add_argument("--sort", choices=["lag", "counting"], default="lag",
                    help="sort of the headline, FP64, long-run and batched paths: the "
                         "counting sort keyed on the cell at the start of the step (lag) "
                         "or after the push (counting); the other one is timed as a path")
    args = ap.parse_args()
    global PROGRESS_STEPS
    PROGRESS_STEPS = max(0, args.progress)
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs a discharge (or a batch of "
              "discharges) on a single MI355X; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1104_3998_amd as fs
    import workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.mode == "copy":
        gbs = copy_ceiling(torch)
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30,
                          "copy_gb_s": gbs}))
        return

    def log(m):
        print("bench: " + m, file=sys.stderr, flush=True)

    global SORT
    SORT = args.sort
    other = "counting" if SORT == "lag" else "lag"
    large = workloads.large_c3(sort_mode=SORT)
    log("FP32 cell+offset, large discharge, %s sort, %d steps after %d"
        % (SORT, args.steps, args.warmup))
    head = run_path(fs, torch, large, "fp32_offset", args.steps, args.warmup)
    paths = {}
    if not args.skip_paths:
        log("FP64, large discharge")
        r64 = run_path(fs, torch, large, "fp64", args.path_steps, args.warmup)
        paths["fp64"] = r64
        log("%s sort, large discharge, FP32" % other)
        paths[other + "_sort_fp32"] = run_path(fs, torch, workloads.large_c3(sort_mode=other),
                                               "fp32_offset", args.path_steps, args.warmup)
        log("unsorted variant, large discharge, FP32")
        paths["unsorted_fp32"] = run_path(fs, torch, workloads.large_c3(sort_mode="none"),
                                          "fp32_offset", args.path_steps, args.warmup)
        # the paper's in-place fine sort against its sorting-cell size (N_gc = G + 1 grid
        # points per sorting cell, the paper's study of cycle time against N_gc)
        fine = {}
        for g in (1, 2, 4, 8):
            log("paper's fine sort, sorting cells of %d grid cells, FP32" % g)
            r = run_path(fs, torch, workloads.large_c3(sort_mode="fine",
                                                       grid_points_per_sort_cell=g + 1),
                         "fp32_offset", args.path_steps // 2, args.warmup, eager=False)
            fine["N_gc=%d" % (g + 1)] = r
        paths["fine_sort_fp32"] = fine
        log("long-run discharge at full size, FP32")
        paths["long_run_fp32"] = run_path(fs, torch, workloads.long_c5(sort_mode=SORT),
                                          "fp32_offset", args.path_steps // 2, args.warmup)
        log("batched scan")
        batch = [dict(w, sort_mode=SORT) for w in workloads.batched_c4(scale=args.batched_scale)]
        # the hottest discharges of the scan (55-95 Pa, 400-490 V, < 2.5 cm) more than
        # double their ion count within a few hundred steps
        tuning, tune_rep = None, None
        if not args.no_autotune:
            # outside the timed region: the fastest of the rule's geometry and its scaled
            # variants (cells per tile, window), timed on this batch
            from paper_1104_3998_amd.autotune import autotune
            tuning, tune_rep = autotune(batch, "fp32_offset", cap_factor=4.0, log=log)
        rb = run_path(fs, torch, batch, "fp32_offset", args.path_steps, args.warmup,
                      tuning=tuning, cap_factor=4.0)
        rb.update({"discharges": len(batch), "autotune": tune_rep})
        paths["batched"] = rb
        log("batched scan, discharges one at a time (every %dth)" % args.seq_every)
        # alone, a discharge may prefer other tiles than the batch's tuned ones: the faster
        # of the batch's geometry and the library's default is the baseline
        seq_t = sequential_sample(fs, torch, batch, tuning, args.path_steps, args.warmup,
                                  every=args.seq_every)
        seq_t["geometry"] = "the batch's tuned geometry" if tuning else "library default"
        seq = seq_t
        if tuning:
            seq_d = sequential_sample(fs, torch, batch, None, args.path_steps, args.warmup,
                                      every=args.seq_every)
            seq_d["geometry"] = "library default"
            best, other = (seq_t, seq_d) if seq_t["value"] >= seq_d["value"] else (seq_d, seq_t)
            seq = dict(best, other_geometry={"geometry": other["geometry"],
                                             "value": other["value"]})
        seq["batched_over_sequential"] = rb["value"] / seq["value"]
        paths["batched"]["sequential"] = seq
    gate = None
    if args.gate_steps > 0:
        log("density gate, FP32 cell+offset vs FP64, %d steps, %d paired seeds"
            % (args.gate_steps, args.gate_seeds))
        gate = density_gate(fs, torch, workloads, args.gate_steps, args.gate_seeds)
    rfg = None
    if args.rf_gate_steps > 0 and args.gate_steps > 0:
        log("bounded RF discharge against the oracle, %d steps" % args.rf_gate_steps)
        rfg = rf_gate(fs, torch, workloads, args.rf_gate_steps)
    study = None
    if args.long_run_study:
        log("long-run precision study %s" % (args.long_run_study,))
        study = long_run_study(fs, torch, workloads, *args.long_run_study)
    log("copy ceiling")
    ceiling = copy_ceiling(torch)
    # roofline of the dominant kernel (k_main), FP32 path, over the timed steps
    kmain_ms = head["kernel_ms"]["main"]
    ps_per_launch = head["eager_particle_steps"] / head["steps"]
    alg_bytes = 2 * REC_BYTES["fp32_offset"] * ps_per_launch
    achieved = alg_bytes / (kmain_ms / 1e3) / 1e9
    traffic = read_traffic("fp32_offset")
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": (traffic * ps_per_launch
                                                         if traffic is not None else None),
            "kernel": "k_main", "alg_bytes_per_launch": alg_bytes,
            "kernel_ms": kmain_ms, "copy_ceiling_gb_s": ceiling,
            "frac_of_copy_ceiling": achieved / ceiling,
            "path_frac": head["value"] * REC_BYTES["fp32_offset"] * 2 / 1e9 / HBM_PEAK_GBS}
    cpu = None
    if not args.skip_cpu:
        log("oracle CPU baseline")
        cpu = cpu_baseline(workloads, args.cpu_steps)
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (Philox-drawn Maxwellian load, no dataset)",
        "config": {"workload": "large single discharge: 4096 cells (20 cm), 1e7 electrons + "
                               "1e7 ions, Te 2 eV, 300 V at 13.56 MHz, 5 Pa Ar-like MCC, "
                               "sort every step, FP32 cell+offset with FP64 Poisson",
                   "sort": {"lag": "counting sort by the cell at the start of the step",
                            "counting": "counting sort by the cell after the push"}[SORT],
                   "particles": 20_000_000, "n_cells": 4096,
                   "window": "steps %d..%d after the load" % (args.warmup + 1,
                                                              args.warmup + args.steps),
                   "graph_steps": head["graph_steps"],
                   "graph_replays": head["graph_replays"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "density_gate": gate,
        "rf_gate": rfg,
        "long_run_study": study,
        "paths": dict({"fp32_offset": head}, **paths),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()

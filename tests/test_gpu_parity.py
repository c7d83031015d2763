"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bar (per result):
* integer results -- particle counts, the permutation (id order of the output array),
  cells, collision / absorption / birth tallies -- bit-exact;
* FP64 path: node weights max|dw| / max w <= 1e-12 per species; positions and velocities
  to 1e-12 (the GPU solves the same tridiagonal system in prefix form, so E differs from
  the Thomas result by rounding only);
* FP32 cell + offset path, compared with the oracle run in the same layout: push
  arithmetic is the same FP32 operation sequence, so positions of particles that did not
  collide agree exactly up to FP32 rounding of the node fields; collided velocities
  (FP32 kinematics on the GPU) to 1e-5 relative; node weights (FP32 sums of up to a few
  hundred terms per tile window) to 1e-5 of max w.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fspic():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1104_3998_amd as m
    m.lib()
    return m


def to_oracle(orc, st, fp32):
    for s in (0, 1):
        a = st[s]
        if fp32:
            x = a["cell"].astype(np.float64) + a["off"].astype(np.float64)
            v = [a["vxf"], a["vyf"], a["vzf"]]
        else:
            x = a["x"]
            v = [a["vx"], a["vy"], a["vz"]]
        orc.set_particles(s, dict(x=x, vx=np.asarray(v[0], np.float64),
                                  vy=np.asarray(v[1], np.float64),
                                  vz=np.asarray(v[2], np.float64), id=a["id"]))
    orc.set_counters(st["step"], st["next_id"][0], st["next_id"][1])


def gpu_arrays(a, fp32):
    if fp32:
        x = a["cell"].astype(np.float64) + a["off"].astype(np.float64)
        v = np.stack([a["vxf"], a["vyf"], a["vzf"]]).astype(np.float64)
    else:
        x = a["x"]
        v = np.stack([a["vx"], a["vy"], a["vz"]])
    return x, v


def tallies_of(diag):
    return {s: dict(coll=[int(diag.collisions[s][c]) for c in range(3)],
                    absorbed=[int(diag.absorbed[s][w]) for w in range(2)],
                    births=int(diag.births[s])) for s in (0, 1)}


def compare(sim, orc, fp32, label, base=None):
    """GPU state and tallies (minus `base`, the GPU tallies when the oracle started)
    against the oracle."""
    st = sim.get_state()
    diag = sim.diagnostics()
    t = orc.tallies()
    g = tallies_of(diag)
    if base is not None:
        for s in (0, 1):
            g[s]["coll"] = [a - b for a, b in zip(g[s]["coll"], base[s]["coll"])]
            g[s]["absorbed"] = [a - b for a, b in zip(g[s]["absorbed"], base[s]["absorbed"])]
            g[s]["births"] -= base[s]["births"]
    for s in (0, 1):
        o = orc.particles(s)
        a = st[s]
        assert a["n"] == orc.count(s), (label, s, "count")
        assert np.array_equal(a["id"], o["id"]), (label, s, "permutation")
        x, v = gpu_arrays(a, fp32)
        vo = np.stack([o["vx"], o["vy"], o["vz"]])
        if fp32:
            assert np.array_equal(np.floor(x), np.floor(o["x"])), (label, s, "cells")
            assert np.max(np.abs(x - o["x"]), initial=0) < 1e-5, (label, s, "x")
            scale = np.max(np.abs(vo), initial=1e-30)
            assert np.max(np.abs(v - vo), initial=0) <= 1e-5 * scale, (label, s, "v")
        else:
            assert np.max(np.abs(x - o["x"]), initial=0) < 1e-12 * max(1.0, sim.workloads[0]["n_cells"]), (label, s, "x")
            scale = np.max(np.abs(vo), initial=1e-30)
            assert np.max(np.abs(v - vo), initial=0) <= 1e-12 * scale, (label, s, "v")
        wo = orc.grid("w_e" if s == 0 else "w_i")
        wg = a["w"]
        tol = 1e-5 if fp32 else 1e-12
        assert np.max(np.abs(wg - wo)) <= tol * max(wo.max(), 1.0), (label, s, "w")
        assert g[s]["coll"] == [t.collisions[s][c] for c in range(3)], (label, s, "collisions")
        assert g[s]["absorbed"] == [t.absorbed[s][w] for w in range(2)], (label, s, "absorbed")
        assert g[s]["births"] == t.births[s], (label, s, "births")
        assert diag.next_id[s] == t.next_id[s], (label, s, "next_id")
    return st


def small_rf(**kw):
    d = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=30.0, avg_start=0, diag_every=5)
    d.update(kw)
    return d


CASES = [
    ("periodic", workloads.periodic_c1()),
    ("rf_small", small_rf()),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_initial_load_matches_oracle(fspic, oracle_mod, name, wl, precision):
    """Load (Philox tag 1), initial sort by cell, deposit, solve, half-step back-push."""
    fp32 = precision == "fp32_offset"
    print("case", name, precision, flush=True)
    sim = fspic.Simulation(wl, precision)
    orc = oracle_mod.Oracle(wl, fp32_offset=fp32)
    orc.load()
    st = sim.get_state()
    for s in (0, 1):
        o = orc.particles(s)
        a = st[s]
        assert a["n"] == orc.count(s) and a["n_sorted"] == a["n"]
        assert np.array_equal(a["id"], o["id"])
        x, v = gpu_arrays(a, fp32)
        assert np.array_equal(x, o["x"])  # no transcendental on the position draw
        vo = np.stack([o["vx"], o["vy"], o["vz"]])
        scale = np.max(np.abs(vo), initial=1e-30)
        tol = 1e-6 if fp32 else 1e-14
        assert np.max(np.abs(v - vo), initial=0) <= tol * scale
        wo = orc.grid("w_e" if s == 0 else "w_i")
        assert np.max(np.abs(a["w"] - wo)) <= (1e-5 if fp32 else 1e-12) * wo.max()
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_one_step_from_identical_state(fspic, oracle_mod, name, wl, precision):
    fp32 = precision == "fp32_offset"
    print("case", name, precision, flush=True)
    sim = fspic.Simulation(wl, precision)
    sim.step(3)
    st = sim.get_state()
    base = tallies_of(sim.diagnostics())
    orc = oracle_mod.Oracle(wl, fp32_offset=fp32)
    to_oracle(orc, st, fp32)
    sim.step(1)
    orc.step(1)
    compare(sim, orc, fp32, "%s/%s" % (name, precision), base)
    sim.close()


@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_fp64_free_running_20_steps(fspic, oracle_mod, name, wl):
    print("case", name, flush=True)
    sim = fspic.Simulation(wl, "fp64")
    orc = oracle_mod.Oracle(wl)
    orc.load()
    for k in range(20):
        sim.step(1)
        orc.step(1)
        compare(sim, orc, False, "%s step %d" % (name, k))
    sim.close()


def test_diagnostics_match_oracle(fspic, oracle_mod):
    """Time averages of the node weights and potential, the EEDF histogram (bin decided in
    FP64 from the same velocities: exact counts), the wall field / surface charge and the
    physical-unit densities, after 30 FP64 steps of the small bounded discharge."""
    wl = small_rf(avg_start=10, diag_every=5)
    sim = fspic.Simulation(wl, "fp64")
    orc = oracle_mod.Oracle(wl)
    orc.load()
    sim.step(30)
    orc.step(30)
    t = orc.tallies()
    g = sim.diagnostics()
    assert g.acc_count == t.acc_count == 20
    assert g.eedf_samples == t.eedf_samples == 4
    assert np.array_equal(sim.grid("eedf"), orc.grid("eedf"))
    for name in ("acc_w_e", "acc_w_i"):
        a, b = sim.grid(name), orc.grid(name)
        assert np.max(np.abs(a - b)) <= 1e-12 * b.max()
    a, b = sim.grid("acc_phi"), orc.grid("acc_phi")
    assert np.max(np.abs(a - b)) <= 1e-10 * np.abs(b).max()
    e_o = orc.grid("E")
    e_g = sim.grid("E")
    assert np.max(np.abs(e_g - e_o)) <= 1e-10 * np.abs(e_o).max()
    assert g.surface_charge[0] == pytest.approx(e_o[0], rel=1e-10, abs=1e-10)
    assert g.surface_charge[1] == pytest.approx(-e_o[-1], rel=1e-10, abs=1e-10)
    d = sim.derived[0]
    ne = sim.density("n_e", kind=0)
    ref = orc.grid("w_e") * d.weight_per_area / d.dx
    ref[0] *= 2
    ref[-1] *= 2
    assert np.allclose(ne, ref, rtol=1e-12, atol=1e-6 * ref.max())
    ni_avg = sim.density("n_i", kind=1)
    ref = orc.grid("acc_w_i") / 20 * d.weight_per_area / d.dx
    ref[0] *= 2
    ref[-1] *= 2
    assert np.allclose(ni_avg, ref, rtol=1e-12, atol=1e-6 * ref.max())
    phi = sim.density("phi", kind=1)
    assert np.allclose(phi, orc.grid("acc_phi") / 20 * d.phi_scale, rtol=1e-9,
                       atol=1e-9 * np.abs(phi).max())
    sim.close()

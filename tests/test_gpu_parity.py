"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Both sides start from inputs neither of them produced: the Philox load each side draws
itself from the same seed, or a seeded synthetic state from workloads.synthetic_state
handed to both.

Bar:
* integer results -- particle counts, the permutation (id order of the output array),
  cells, collision / absorption / birth tallies -- bit-exact (FP64 path);
* FP64 path: node weights max|dw| / max w <= 1e-12 per species; positions and velocities
  to 1e-12 (the GPU solves the same tridiagonal system in prefix form, so E differs from
  the Thomas result by rounding only);
* absorbed energy per wall to 1e-11 relative (FP64 sums in another order);
* FP32 cell + offset path, against the oracle run in the same layout.  The kernel adds
  the charge as fixed-point integers (round(f 2^s), s >= 37: exact sums of weights
  rounded by at most 2^-38 each), the oracle in FP64, so the node weights agree to 1e-9
  of max w and the fields to ~1e-12 relative; the FP32 copy of E can still round the
  other way at a node, and a particle whose new offset lies that close to a cell edge may
  land in the neighbouring cell.  So: cells agree except inside a band of width EDGE at a
  cell edge; positions to 1e-4 cells, velocities to 1e-5 relative; the GPU's output order
  must be exactly the stable sort, by the GPU's own cells, of the input order
  (survivors), then the births in parent order.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

EDGE = 1e-4


@pytest.fixture(scope="module")
def fspic():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1104_3998_amd as m
    m.lib()
    return m


def positions(a, fp32):
    if fp32:
        return a["cell"].astype(np.float64) + a["off"].astype(np.float64)
    return np.asarray(a["x"], dtype=np.float64)


def velocities(a, fp32):
    if fp32:
        return np.stack([a["vxf"], a["vyf"], a["vzf"]]).astype(np.float64)
    return np.stack([a["vx"], a["vy"], a["vz"]])


def oracle_from_state(oracle_mod, wl, st, fp32):
    """An oracle holding the seeded synthetic state `st`."""
    caps = [max(int(wl["n_e0"] * 1.5) + 1024, 2 * st[0]["n"]),
            max(int(wl["n_i0"] * 1.5) + 1024, 2 * st[1]["n"])]
    orc = oracle_mod.Oracle(wl, fp32_offset=fp32, cap_e=caps[0], cap_i=caps[1])
    for s in (0, 1):
        a = st[s]
        v = velocities(a, fp32)
        orc.set_particles(s, dict(x=positions(a, fp32), vx=v[0], vy=v[1], vz=v[2], id=a["id"]))
    orc.set_counters(st["step"], st["next_id"][0], st["next_id"][1])
    return orc


def gpu_from_state(fspic, wl, st, precision, cap_factor=1.5):
    sim = fspic.Simulation(wl, precision, cap_factor=cap_factor)
    sim.set_state(st)
    return sim


def tallies_of(diag):
    return {s: dict(coll=[int(diag.collisions[s][c]) for c in range(3)],
                    absorbed=[int(diag.absorbed[s][w]) for w in range(2)],
                    births=int(diag.births[s]),
                    abs_e=[float(diag.absorbed_energy_ev[s][w]) for w in range(2)])
            for s in (0, 1)}


def oracle_tallies(t):
    return {s: dict(coll=[int(t.collisions[s][c]) for c in range(3)],
                    absorbed=[int(t.absorbed[s][w]) for w in range(2)],
                    births=int(t.births[s]),
                    abs_e=[float(t.absorbed_energy_ev[s][w]) for w in range(2)])
            for s in (0, 1)}


def delta(a, b):
    return {s: dict(coll=[x - y for x, y in zip(a[s]["coll"], b[s]["coll"])],
                    absorbed=[x - y for x, y in zip(a[s]["absorbed"], b[s]["absorbed"])],
                    births=a[s]["births"] - b[s]["births"],
                    abs_e=[x - y for x, y in zip(a[s]["abs_e"], b[s]["abs_e"])])
            for s in (0, 1)}


def same_tallies(g, o, label, s):
    """Integer tallies exact, absorbed energy to 1e-11 relative."""
    for k in ("coll", "absorbed", "births"):
        assert g[k] == o[k], (label, s, k, g[k], o[k])
    for w in range(2):
        assert g["abs_e"][w] == pytest.approx(o["abs_e"][w], rel=1e-11, abs=1e-9), \
            (label, s, "absorbed energy", w, g["abs_e"][w], o["abs_e"][w])


def compare_fp64(sim, orc, label, gbase=None, obase=None, d=0, w_tol=1e-12):
    """Exact permutation / counts / tallies, 1e-12 on positions and velocities, w_tol of
    max w on the node weights (1e-12 unless a caller states why its weights may follow a
    position difference inside the 1e-12 * N bar more closely)."""
    st = sim.get_state(d)
    g = tallies_of(sim.diagnostics(d))
    o = oracle_tallies(orc.tallies())
    if gbase is not None:
        g = delta(g, gbase)
    if obase is not None:
        o = delta(o, obase)
    n_cells = sim.workloads[d]["n_cells"]
    for s in (0, 1):
        po = orc.particles(s)
        a = st[s]
        assert a["n"] == orc.count(s), (label, s, "count")
        assert np.array_equal(a["id"], po["id"]), (label, s, "permutation")
        x, v = positions(a, False), velocities(a, False)
        vo = np.stack([po["vx"], po["vy"], po["vz"]])
        assert np.max(np.abs(x - po["x"]), initial=0) <= 1e-12 * max(1.0, n_cells), (label, s, "x")
        scale = np.max(np.abs(vo), initial=1e-30)
        assert np.max(np.abs(v - vo), initial=0) <= 1e-12 * scale, (label, s, "v")
        wo = orc.grid("w_e" if s == 0 else "w_i")
        assert np.max(np.abs(a["w"] - wo)) <= w_tol * max(wo.max(), 1.0), (label, s, "w")
        same_tallies(g[s], o[s], label, s)
    return st


def compare_fp32(sim, orc, st_in, label, gbase=None, obase=None, coll_slack=0, d=0):
    st = sim.get_state(d)
    g = tallies_of(sim.diagnostics(d))
    o = oracle_tallies(orc.tallies())
    if gbase is not None:
        g = delta(g, gbase)
    if obase is not None:
        o = delta(o, obase)
    # With coll_slack > 0, up to coll_slack collision decisions may differ from the
    # oracle's (the FP32 field rounds differently, and a candidate close to a channel
    # boundary can flip): those particles' velocities, a flipped ionisation's pair of
    # births, and their deposits are allowed to differ; everything else must match.
    for s in (0, 1):
        a, po, inp = st[s], orc.particles(s), st_in[s]
        n = a["n"]
        assert abs(n - orc.count(s)) <= coll_slack, (label, s, "count")
        common = np.intersect1d(a["id"], po["id"])
        assert a["id"].size - common.size <= coll_slack, (label, s, "id sets")
        assert po["id"].size - common.size <= coll_slack, (label, s, "id sets")
        if coll_slack:
            # a flipped ionisation shifts the ids of the later births: compare the
            # particles that existed before the step one by one, the births by count
            common = common[common < st_in["next_id"][s]]
        ig = np.flatnonzero(np.isin(a["id"], common))
        io = np.flatnonzero(np.isin(po["id"], common))
        ig = ig[np.argsort(a["id"][ig])]
        io = io[np.argsort(po["id"][io])]
        xg, xo = positions(a, True)[ig], po["x"][io]
        cg, co = a["cell"][ig].astype(np.int64), np.floor(xo).astype(np.int64)
        fo = xo - co
        edge = (fo < EDGE) | (fo > 1 - EDGE)
        bad = (cg != co) & ~edge
        assert not bad.any(), (label, s, "cells off the edge band", int(bad.sum()))
        assert np.max(np.abs(xg - xo), initial=0) <= 1e-4, (label, s, "x")
        vg = velocities(a, True)[:, ig]
        vo = np.stack([po["vx"], po["vy"], po["vz"]])[:, io]
        scale = np.max(np.abs(vo), initial=1e-30)
        off = np.any(np.abs(vg - vo) > 1e-5 * scale, axis=0)
        assert int(off.sum()) <= coll_slack, (label, s, "v", int(off.sum()))
        # the GPU's order is the stable sort of the input order by the GPU's own cells
        # (unsorted: the input order itself)
        ns = a["n_sorted"]
        surv = a["id"][:ns]
        in_order = inp["id"][np.isin(inp["id"], surv)]
        mode = sim.workloads[d].get("sort_mode", "counting")
        if mode == "none":
            expect = in_order
        elif mode == "lag":
            # lagged: the stable sort of the input order by the cells the input held
            xin = positions(inp, True)
            key_of = dict(zip(inp["id"].tolist(), np.floor(xin).astype(np.int64).tolist()))
            keys = np.array([key_of[i] for i in in_order.tolist()], dtype=np.int64)
            expect = in_order[np.argsort(keys, kind="stable")]
        else:
            by_id = np.argsort(surv)
            keys = a["cell"][:ns][by_id][np.searchsorted(surv[by_id], in_order)].astype(np.int64)
            expect = in_order[np.argsort(keys, kind="stable")]
        assert np.array_equal(expect, surv), (label, s, "stable order")
        # births: appended in parent order with consecutive new ids
        born = a["id"][ns:]
        first = st_in["next_id"][s]
        assert np.array_equal(born, np.arange(first, first + born.size)), (label, s, "birth ids")
        wo = orc.grid("w_e" if s == 0 else "w_i")
        # the GPU's node weights are the oracle's deposit of the GPU's own particles; with
        # no flipped decision they are also the oracle's node weights
        wl_ = sim.workloads[d]
        wself = oracle_mod_deposit(wl_["periodic"], wl_["n_cells"], positions(a, True))
        assert np.max(np.abs(a["w"] - wself)) <= 1e-9 * max(wself.max(), 1.0), (label, s, "w")
        if not coll_slack:
            assert np.max(np.abs(a["w"] - wo)) <= 1e-9 * max(wo.max(), 1.0), (label, s, "w")
        assert g[s]["absorbed"] == o[s]["absorbed"], (label, s, "absorbed")
        for c in range(3):
            assert abs(g[s]["coll"][c] - o[s]["coll"][c]) <= coll_slack, (label, s, "collisions")
        assert abs(g[s]["births"] - o[s]["births"]) <= coll_slack, (label, s, "births")
    return st


def oracle_mod_deposit(periodic, n_cells, x):
    import oracle
    return oracle.deposit(int(periodic), int(n_cells), np.ascontiguousarray(x, dtype=np.float64))


def small_rf(**kw):
    d = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=30.0, avg_start=0, diag_every=5)
    d.update(kw)
    return d


CASES = [
    ("periodic", workloads.periodic_c1()),
    ("rf_small", small_rf()),
    ("rf_full", workloads.rf_c2()),  # the bounded RF discharge at its size: 2e5 + 2e5
]


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_initial_load_matches_oracle(fspic, oracle_mod, name, wl, precision):
    """Load (Philox tag 1, drawn by each side), initial sort by cell, deposit, solve,
    half-step back-push."""
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
        assert np.array_equal(positions(a, fp32), o["x"])  # no transcendental in x
        vo = np.stack([o["vx"], o["vy"], o["vz"]])
        scale = np.max(np.abs(vo), initial=1e-30)
        tol = 1e-6 if fp32 else 1e-14
        assert np.max(np.abs(velocities(a, fp32) - vo), initial=0) <= tol * scale
        wo = orc.grid("w_e" if s == 0 else "w_i")
        assert np.max(np.abs(a["w"] - wo)) <= (1e-9 if fp32 else 1e-12) * wo.max()
    sim.close()


def one_step(fspic, oracle_mod, wl, st, precision, coll_slack=0, label=""):
    fp32 = precision == "fp32_offset"
    sim = gpu_from_state(fspic, wl, st, precision)
    orc = oracle_from_state(oracle_mod, wl, st, fp32)
    gb = tallies_of(sim.diagnostics())
    sim.step(1)
    orc.step(1)
    if fp32:
        compare_fp32(sim, orc, st, label, gbase=gb, coll_slack=coll_slack)
    else:
        compare_fp64(sim, orc, label, gbase=gb)
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_one_step_from_seeded_state(fspic, oracle_mod, name, wl, precision):
    """One step from the same seeded synthetic state (both species, a births tail of 50
    particles per species)."""
    print("case", name, precision, flush=True)
    st = workloads.synthetic_state(wl["n_cells"], (wl["n_e0"], wl["n_i0"]), precision,
                                   seed=17, vth=(2.0, 0.02), tail=(50, 50))
    one_step(fspic, oracle_mod, wl, st, precision, label="%s/%s" % (name, precision))


@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_fp64_free_running_20_steps(fspic, oracle_mod, name, wl):
    """Each side loads from the same seed and runs 20 steps on its own."""
    print("case", name, flush=True)
    sim = fspic.Simulation(wl, "fp64")
    orc = oracle_mod.Oracle(wl)
    orc.load()
    for k in range(20):
        sim.step(1)
        orc.step(1)
        compare_fp64(sim, orc, "%s step %d" % (name, k))
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


@pytest.mark.parametrize("name,wl", [("periodic", workloads.periodic_c1()),
                                     ("rf_small", small_rf())], ids=["periodic", "rf_small"])
def test_energy_diagnostics_match_oracle(fspic, oracle_mod, name, wl):
    """Kinetic energy per species (mean of v_x^2 before and after the push), momentum,
    field energy, net charge and the driven electrode's potential of every step, and the
    EEDF handed back through pic_diagnostics, against the oracle's per-step values (FP64,
    every step an energy step)."""
    wl = dict(wl, avg_start=0, diag_every=1)
    sim = fspic.Simulation(wl, "fp64")
    orc = oracle_mod.Oracle(wl)
    orc.load()
    d = sim.derived[0]
    for k in range(12):
        sim.step(1)
        orc.step(1)
        g = sim.diagnostics(eedf=True)
        t = orc.tallies()
        label = "%s step %d" % (name, k)
        assert g.energy_step == k, label
        for s in (0, 1):
            assert g.kinetic[s] == pytest.approx(t.kinetic[s], rel=1e-11), (label, s)
        scale = sum(g.kinetic) / max(min(abs(d.kappa[0]), abs(d.kappa[1])), 1e-300)
        assert abs(g.momentum - t.momentum) <= 1e-11 * max(abs(t.momentum), 1.0) + 1e-13 * scale, label
        assert g.field_energy == pytest.approx(t.field_energy, rel=1e-10), label
        assert g.sum_rho == pytest.approx(t.sum_rho, rel=1e-10, abs=1e-9), label
        assert g.phi_driven_v / d.phi_scale == pytest.approx(t.phi0, rel=1e-12, abs=1e-12), label
        assert np.array_equal(g.eedf_counts, orc.grid("eedf")), label
        assert np.array_equal(g.eedf_counts, sim.grid("eedf")), label
    sim.close()


def test_series_capacitor_circuit_matches_oracle(fspic, oracle_mod):
    """The driven electrode behind a series capacitor (an external circuit): 20 free FP64
    steps against the oracle, the electrode potential and the conductor charge included."""
    wl = small_rf(circuit_cap_f_m2=2e-7, v0_volt=200.0)
    sim = fspic.Simulation(wl, "fp64")
    orc = oracle_mod.Oracle(wl)
    orc.load()
    d = sim.derived[0]
    for k in range(20):
        sim.step(1)
        orc.step(1)
        # the electrode potential follows the conductor charge, a running sum of wall
        # fluxes and solve residues: positions stay inside the 1e-12 * N bar but drift
        # apart by up to ~1e-11 cells over 20 free steps, and a node's weight sums that
        # drift over its particles, so the weights are held to 1e-10 of max w against
        # the oracle and to 1e-12 against the oracle's deposit of the GPU's own particles
        st = compare_fp64(sim, orc, "circuit step %d" % k, w_tol=1e-10)
        for s in (0, 1):
            wself = oracle_mod_deposit(wl["periodic"], wl["n_cells"], positions(st[s], False))
            assert np.max(np.abs(st[s]["w"] - wself)) <= 1e-12 * max(wself.max(), 1.0), k
        g, t = sim.diagnostics(), orc.tallies()
        assert g.phi_driven_v / d.phi_scale == pytest.approx(t.phi0, rel=1e-10, abs=1e-10)
        assert g.circuit_charge == pytest.approx(t.q_circuit, rel=1e-10, abs=1e-10)
    sim.close()

"""GPU parity of the less common paths of the step through the C ABI, from seeded states
handed to both sides: far movers (more than `window` cells in one step), an unsorted
births tail, the general device sort, batched discharges, HIP-graph replay, and one step
at the full size of the large single discharge.  Same bar as test_gpu_parity.py."""
import numpy as np
import pytest

import workloads
from test_gpu_parity import (compare_fp64, one_step, oracle_from_state, tallies_of)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fspic():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1104_3998_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
def test_far_movers(fspic, oracle_mod, precision):
    """300 electrons sent 40-90 cells in one step (window 31 cells in this box) take the
    far-mover path and must land at their place in the stable order."""
    wl = workloads.periodic_c1(xsec="none", gas_pa=0.0)
    print("far movers", precision, flush=True)
    st = workloads.synthetic_state(wl["n_cells"], (wl["n_e0"], wl["n_i0"]), precision,
                                   seed=5, vth=(0.4, 0.001), fast=(300, 0))
    one_step(fspic, oracle_mod, wl, st, precision, label="far " + precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
@pytest.mark.parametrize("tail", [137, "all"])
def test_unsorted_tail(fspic, oracle_mod, precision, tail):
    """A state whose last particles are not in cell order (as after births): the step sorts
    them in at their input rank.  'all': the whole array is the tail."""
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=30.0)
    print("tail", tail, precision, flush=True)
    k = 20000 if tail == "all" else tail
    st = workloads.synthetic_state(wl["n_cells"], (20000, 20000), precision, seed=9,
                                   vth=(2.0, 0.01), tail=(k, k))
    one_step(fspic, oracle_mod, wl, st, precision, label="tail %s %s" % (tail, precision))


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
def test_general_sort_of_unsorted_state(fspic, oracle_mod, precision):
    """sort_all: the device sorts an unsorted array stably by cell (ties in input order),
    as the oracle's stable counting sort orders it."""
    wl = workloads.periodic_c1()
    fp32 = precision == "fp32_offset"
    st = workloads.synthetic_state(wl["n_cells"], (16384, 16384), precision, seed=11,
                                   tail=(16384, 16384))
    sim = fspic.Simulation(wl, precision)
    sim.set_state(st, sort_all=True)
    st2 = sim.get_state()
    for s in (0, 1):
        a = st[s]
        cells = a["cell"] if fp32 else np.floor(a["x"]).astype(np.int32)
        perm = oracle_mod.stable_sort_by_cell(cells, wl["n_cells"])
        assert st2[s]["n_sorted"] == st2[s]["n"] == a["n"]
        assert np.array_equal(st2[s]["id"], a["id"][perm])
    sim.close()


@pytest.mark.parametrize("sort", ["counting", "lag"])
def test_batched_discharges_match_oracle_each(fspic, oracle_mod, sort):
    """Three discharges of the batched scan (particle counts scaled down) in one launch per
    kernel.  Free-running from each side's own load for 4 steps the permutation matches
    every discharge's oracle exactly; the node weights match to 1e-10 of max w, not 1e-12,
    because these discharges have up to 2048 cells at up to 500 V and ~2 particles per
    cell: the Thomas elimination of the oracle and the prefix-form solve of the GPU round
    differently by ~N eps relative in E, and the positions accumulate it.  Then one step
    from seeded states set into both sides meets the 1e-12 bar for every discharge, and
    discharge 1 run alone gives the same particles as inside the batch."""
    wls = [dict(w, sort_mode=sort) for w in workloads.batched_c4(n_discharges=3, scale=0.01)]
    print("batched", sort, [(w["n_cells"], w["n_e0"]) for w in wls], flush=True)
    sim = fspic.Simulation(wls, "fp64")
    orcs = []
    for wl in wls:
        o = oracle_mod.Oracle(wl)
        o.load()
        orcs.append(o)
    sim.step(4)
    for o in orcs:
        o.step(4)
    for d, o in enumerate(orcs):
        st = sim.get_state(d)
        for s in (0, 1):
            assert np.array_equal(st[s]["id"], o.particles(s)["id"]), (d, s)
            wo = o.grid("w_e" if s == 0 else "w_i")
            assert np.max(np.abs(st[s]["w"] - wo)) <= 1e-10 * wo.max(), (d, s)
    alone = fspic.Simulation(wls[1], "fp64")
    alone.step(4)
    # the same tile geometry alone and in the batch: the same bits
    bitwise_equal_states(alone.get_state(), sim.get_state(1), False, "alone vs batch")
    alone.close()
    # one step from seeded states, all discharges at once
    states = [workloads.synthetic_state(wl["n_cells"], (wl["n_e0"], wl["n_i0"]), "fp64",
                                        seed=100 + d, step=4) for d, wl in enumerate(wls)]
    orcs = []
    for d, wl in enumerate(wls):
        sim.set_state(states[d], d)
        orcs.append(oracle_from_state(oracle_mod, wl, states[d], False))
    gbs = [tallies_of(sim.diagnostics(d)) for d in range(3)]
    sim.step(1)
    for d, o in enumerate(orcs):
        o.step(1)
        compare_fp64(sim, o, "batched %d" % d, gbase=gbs[d], d=d)
    sim.close()


def test_grouped_ion_mcc_matches_oracle(fspic, oracle_mod):
    """Five 2048-cell discharges at 100 Pa with one-cell ion tiles: 10320 ion tiles of
    about 10 ions each (about 1000 ion candidates per discharge, P0 = 0.05), so the MCC
    pass takes 64 ion tiles' candidate lists (256 list segments) per workgroup.  One step
    from seeded states with an unsorted births tail matches every discharge's oracle at
    the FP64 bar, ion collisions included."""
    wls = [workloads.bounded(2048, 20000, 300.0, 100.0, discharge=k, seed=k, steps=10)
           for k in range(5)]
    print("grouped ion MCC", flush=True)
    sim = fspic.Simulation(wls, "fp64", tuning={"cells_per_tile": (0, 1)})
    states = [workloads.synthetic_state(wl["n_cells"], (wl["n_e0"], wl["n_i0"]), "fp64",
                                        seed=200 + d, tail=(64, 64), step=0)
              for d, wl in enumerate(wls)]
    orcs = []
    for d, wl in enumerate(wls):
        sim.set_state(states[d], d)
        orcs.append(oracle_from_state(oracle_mod, wl, states[d], False))
    gbs = [tallies_of(sim.diagnostics(d)) for d in range(len(wls))]
    sim.step(1)
    for d, o in enumerate(orcs):
        o.step(1)
        compare_fp64(sim, o, "grouped ion MCC %d" % d, gbase=gbs[d], d=d)
        ion_coll = sum(tallies_of(sim.diagnostics(d))[1]["coll"]) - sum(gbs[d][1]["coll"])
        assert ion_coll > 0, d
    sim.close()


def bitwise_equal_states(sa, sb, fp32, label):
    """Every particle array, the node weights, counts and ids identical bit for bit."""
    assert sa["step"] == sb["step"] and sa["next_id"] == sb["next_id"], label
    keys = ("cell", "off", "vxf", "vyf", "vzf") if fp32 else ("x", "vx", "vy", "vz")
    for s in (0, 1):
        assert sa[s]["n"] == sb[s]["n"] and sa[s]["n_sorted"] == sb[s]["n_sorted"], (label, s)
        for k in keys + ("id", "w"):
            assert np.array_equal(sa[s][k].view(np.uint8), sb[s][k].view(np.uint8)), (label, s, k)


def bitwise_equal_diagnostics(da, db, label):
    for f in ("absorbed", "absorbed_energy_ev", "collisions"):
        assert [list(r) for r in getattr(da, f)] == [list(r) for r in getattr(db, f)], (label, f)
    for f in ("births", "kinetic", "n_particles"):
        assert list(getattr(da, f)) == list(getattr(db, f)), (label, f)
    for f in ("momentum", "field_energy", "sum_rho", "phi_driven_v"):
        assert getattr(da, f) == getattr(db, f), (label, f)


@pytest.mark.parametrize("sort", ["counting", "lag"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
def test_graph_replay_bitwise_equals_eager(fspic, precision, sort):
    """30 ionising steps replayed from a captured HIP graph of 10 steps and launched one
    by one give the same state bit for bit."""
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=30.0, diag_every=1, avg_start=0,
                         sort_mode=sort)
    a = fspic.Simulation(wl, precision)
    b = fspic.Simulation(wl, precision)
    b.set_graph(10)
    a.step(30)
    b.step(30)
    sa, sb = a.get_state(), b.get_state()
    assert sa["step"] == 30
    bitwise_equal_states(sa, sb, precision == "fp32_offset", "graph " + precision)
    bitwise_equal_diagnostics(a.diagnostics(), b.diagnostics(), "graph " + precision)
    a.close()
    b.close()


@pytest.mark.parametrize("sort", ["counting", "lag"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
def test_same_seed_twice_bitwise(fspic, precision, sort):
    """The same seed run twice (400 ionising steps of the bounded discharge) gives the same
    particles, node weights and tallies bit for bit: charge is summed in fixed point and
    every floating-point sum in a fixed order, so nothing depends on the order in which
    the GPU schedules the work."""
    wl = workloads.rf_c2(n_e0=50000, n_i0=50000, gas_pa=30.0, diag_every=7, avg_start=100,
                         sort_mode=sort)
    runs = []
    for _ in range(2):
        sim = fspic.Simulation(wl, precision)
        sim.set_graph(50)
        sim.step(400)
        runs.append((sim.get_state(), sim.diagnostics(eedf=True),
                     [sim.grid(k) for k in ("acc_w_e", "acc_w_i", "acc_phi")]))
        sim.close()
    (sa, da, ga), (sb, db, gb) = runs
    bitwise_equal_states(sa, sb, precision == "fp32_offset", "twice " + precision)
    bitwise_equal_diagnostics(da, db, "twice " + precision)
    assert np.array_equal(da.eedf_counts, db.eedf_counts)
    for x, y in zip(ga, gb):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
    assert sum(da.births) > 0  # the run ionises


@pytest.mark.parametrize("sort", ["counting", "lag"])
@pytest.mark.parametrize("precision", ["fp32_offset", "fp64"])
def test_full_size_large_discharge_one_step(fspic, oracle_mod, precision, sort):
    """The large single discharge at full size (4096 cells, 1e7 + 1e7 particles), with the
    tile geometry the benchmark times, one step from a seeded state (electron spread 2.2
    cells per step, a births tail of 1000) against the oracle over every particle.  About
    1e6 collision candidates.  The FP32 layout's FP32 copy of the field can round the
    other way at a node where the fixed-point and the FP64 charge sums differ in the last
    bits, which could move a channel decision of a candidate that close to a channel
    boundary: at most one flip is allowed; the FP64 path must match exactly."""
    wl = workloads.large_c3(sort_mode=sort)
    fp32 = precision == "fp32_offset"
    print("full size", precision, sort, flush=True)
    st = workloads.synthetic_state(wl["n_cells"], (wl["n_e0"], wl["n_i0"]), precision,
                                   seed=23, vth=(2.2, 0.01), tail=(1000, 1000))
    one_step(fspic, oracle_mod, wl, st, precision, coll_slack=1 if fp32 else 0,
             label="full %s %s" % (precision, sort))


@pytest.mark.parametrize("sort", ["counting", "lag"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
def test_full_size_long_run_one_step(fspic, oracle_mod, precision, sort):
    """The long run's discharge at full size (8192 cells, 3.2e7 + 3.2e7 particles, 20 Pa)
    with its default geometry: one-cell tiles for both species, so 8192 + 16 tail ion
    tiles and the MCC pass groups the ion lists four at a time; about 1e7 collision
    candidates.  One step from a seeded state against the oracle over every particle (the
    FP32 layout may flip one channel decision, as in the large discharge)."""
    wl = workloads.long_c5(sort_mode=sort)
    fp32 = precision == "fp32_offset"
    print("long run full size", precision, sort, flush=True)
    st = workloads.synthetic_state(wl["n_cells"], (wl["n_e0"], wl["n_i0"]), precision,
                                   seed=29, vth=(2.2, 0.01), tail=(1000, 1000))
    one_step(fspic, oracle_mod, wl, st, precision, coll_slack=1 if fp32 else 0,
             label="long %s %s" % (precision, sort))


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
def test_tile_geometry_does_not_change_results(fspic, precision):
    """The tile geometry (cells per tile, window) changes speed only: 20 steps of the RF
    discharge with the default geometry and with half-size electron tiles, double-size
    ion tiles and a half window give the same state bit for bit (the fixed-point deposit
    makes the node weights independent of which windows a particle lands in) and the same
    integer tallies."""
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=30.0)
    from paper_1104_3998_amd import autotune as at
    alt = at.scaled_tuning(at.rule_geometry([wl], precision), 0.5, 2.0, 0.5)
    print("tile geometry", alt, flush=True)
    a = fspic.Simulation(wl, precision)
    b = fspic.Simulation(wl, precision, tuning=alt)
    a.step(20)
    b.step(20)
    bitwise_equal_states(a.get_state(), b.get_state(), precision == "fp32_offset", "tiles")
    # the integer tallies are the same; the absorbed energy is an FP64 sum grouped by tile,
    # so another geometry rounds it differently in the last bits
    ga, gb = tallies_of(a.diagnostics()), tallies_of(b.diagnostics())
    for sp in (0, 1):
        for k in ("coll", "absorbed", "births"):
            assert ga[sp][k] == gb[sp][k], (sp, k)
        for w in range(2):
            assert ga[sp]["abs_e"][w] == pytest.approx(gb[sp]["abs_e"][w], rel=1e-12, abs=1e-12)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
def test_mcc_workgroup_width_does_not_change_results(fspic, precision):
    """The MCC pass runs eight-wave workgroups when a simulation has few electron tiles and
    four-wave ones when it has many (1024 or more), with the ion tiles grouped by their
    expected candidates: 20 steps of a 2048-cell discharge with the default geometry (32
    electron tiles) and with one cell per tile (2048) give the same state bit for bit and
    the same integer tallies."""
    wl = workloads.bounded(2048, 40000, 200.0, 30.0, steps=20, avg_start=10)
    from paper_1104_3998_amd import autotune as at
    (ce, de), (ci, di) = at.rule_geometry([wl], precision)[0]
    assert (2048 + ce - 1) // ce < 1024
    one = [{"cells_per_tile": (1, 1), "window": (de, max(di, 1))}]
    print("rule C", ce, ci, "against one cell per tile", flush=True)
    a = fspic.Simulation(wl, precision)
    b = fspic.Simulation(wl, precision, tuning=one)
    a.step(20)
    b.step(20)
    bitwise_equal_states(a.get_state(), b.get_state(), precision == "fp32_offset", "mcc width")
    ga, gb = tallies_of(a.diagnostics()), tallies_of(b.diagnostics())
    assert sum(ga[0]["coll"]) > 0 and sum(ga[1]["coll"]) > 0
    for sp in (0, 1):
        for k in ("coll", "absorbed", "births"):
            assert ga[sp][k] == gb[sp][k], (sp, k)
    a.close()
    b.close()


def test_autotune_and_cache(fspic, tmp_path):
    """The tuner times the rule and its scaled variants on a small batch, returns one
    tuning per discharge with a rate for the rule, and a second call with the same cache
    file returns the stored choice."""
    from paper_1104_3998_amd import autotune as at
    wls = workloads.batched_c4(n_discharges=3, scale=0.01)
    cache = str(tmp_path / "tune.json")
    tun, rep = at.autotune(wls, "fp32_offset", steps=6, warmup=4, cap_factor=4.0,
                           cache=cache, log=lambda m: print(m, flush=True))
    assert len(tun) == 3 and rep["rule_rate"] > 0 and rep["best_rate"] >= rep["rule_rate"]
    assert len(rep["timed"]) >= 4
    tun2, rep2 = at.autotune(wls, "fp32_offset", steps=6, warmup=4, cap_factor=4.0,
                             cache=cache)
    assert tun2 == tun and rep2["best"] == rep["best"]
    sim = fspic.Simulation(wls, "fp32_offset", tuning=tun, cap_factor=4.0)
    sim.step(3)
    sim.sync()
    sim.close()


EDGE_STATES = {
    # every particle in one cell
    "one_cell": dict(n=(4096, 4096), cells=[64], vth=(0.6, 0.01)),
    # a quarter of the cells occupied, in two blocks: empty cells and empty tiles
    "empty_cells": dict(n=(8192, 8192), cells=list(range(0, 16)) + list(range(100, 116))),
    # one particle per species
    "single": dict(n=(1, 1)),
    # every electron a far mover (40-90 cells in one step against a 31-cell window)
    "all_far": dict(n=(4096, 4096), fast=(4096, 0)),
    # every electron in one cell, all moving 60 cells one way or the other: two far groups
    # of about 2048 into two cells (the ranking inside a cell's group is quadratic)
    "pile_up": dict(n=(4096, 4096), cells=[10], fast=(4096, 0), fast_speed=(60.0, 60.0)),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
@pytest.mark.parametrize("case", sorted(EDGE_STATES))
def test_edge_states_one_step(fspic, oracle_mod, case, precision):
    """One step from degenerate states against the oracle: the sort, deposit, MCC and
    solve on a single occupied cell, on empty cells and tiles, on one particle per
    species, with every electron beyond the sort window (far list sized for all), and
    with every electron of one cell landing in one of two far cells."""
    e = EDGE_STATES[case]
    wl = workloads.periodic_c1()
    print("edge state", case, precision, flush=True)
    st = workloads.synthetic_state(wl["n_cells"], e["n"], precision, seed=41,
                                   vth=e.get("vth", (2.0, 0.02)), fast=e.get("fast", (0, 0)),
                                   fast_speed=e.get("fast_speed", (40.0, 90.0)),
                                   cells=e.get("cells"))
    fp32 = precision == "fp32_offset"
    sim = fspic.Simulation(wl, precision, tuning={"far_capacity": 8192})
    sim.set_state(st)
    orc = oracle_from_state(oracle_mod, wl, st, fp32)
    gb = tallies_of(sim.diagnostics())
    sim.step(1)
    orc.step(1)
    from test_gpu_parity import compare_fp32
    if fp32:
        compare_fp32(sim, orc, st, case, gbase=gb)
    else:
        compare_fp64(sim, orc, case, gbase=gb)
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
@pytest.mark.parametrize("case", sorted(EDGE_STATES))
def test_edge_states_lagged_sort(fspic, oracle_mod, case, precision):
    """The degenerate states under the lagged sort, two steps: in the second step the keys
    are the cells the first step left the particles in, so in the all-far case every fast
    electron goes through the far list.  The second step is compared with the oracle
    started from the GPU's state after the first (the one-step bar)."""
    from test_gpu_parity import compare_fp32
    e = EDGE_STATES[case]
    wl = workloads.periodic_c1(sort_mode="lag")
    print("edge state, lagged sort", case, precision, flush=True)
    st = workloads.synthetic_state(wl["n_cells"], e["n"], precision, seed=43,
                                   vth=e.get("vth", (2.0, 0.02)), fast=e.get("fast", (0, 0)),
                                   fast_speed=e.get("fast_speed", (40.0, 90.0)),
                                   cells=e.get("cells"))
    fp32 = precision == "fp32_offset"
    sim = fspic.Simulation(wl, precision, tuning={"far_capacity": 8192})
    sim.set_state(st)
    orc = oracle_from_state(oracle_mod, wl, st, fp32)
    gb0 = tallies_of(sim.diagnostics())
    sim.step(1)
    orc.step(1)
    if fp32:
        compare_fp32(sim, orc, st, case + " step 1", gbase=gb0)
    st1 = sim.get_state()
    orc = oracle_from_state(oracle_mod, wl, st1, fp32)
    gb = tallies_of(sim.diagnostics())
    sim.step(1)
    orc.step(1)
    if fp32:
        compare_fp32(sim, orc, st1, case, gbase=gb)
    else:
        compare_fp64(sim, orc, case, gbase=gb)
    sim.close()


@pytest.mark.parametrize("sort", ["counting", "lag"])
def test_full_size_batched_scan_sampled(fspic, oracle_mod, sort):
    """The batched scan at full size (256 discharges, 2.9e8 particles at load) in one
    simulation, in the FP32 layout and capacity the benchmark times: after 3 steps from the
    loads, three discharges (the fewest particles, the median, the most) are set to seeded
    states, and one more step of the whole batch is compared with the oracle for those
    three, particle by particle, at the FP32 bar (one flipped channel decision allowed, as
    for the large discharge)."""
    from test_gpu_parity import compare_fp32, oracle_from_state, tallies_of
    wls = [dict(w, sort_mode=sort) for w in workloads.batched_c4()]
    sizes = np.array([w["n_e0"] for w in wls])
    order = np.argsort(sizes, kind="stable")
    picked = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    print("batched full size", sort, picked, [int(sizes[d]) for d in picked], flush=True)
    sim = fspic.Simulation(wls, "fp32_offset", cap_factor=4.0)
    sim.step(3)
    states, orcs, gbs = {}, {}, {}
    for d in picked:
        wl = wls[d]
        st = workloads.synthetic_state(wl["n_cells"], (wl["n_e0"], wl["n_i0"]), "fp32_offset",
                                       seed=300 + d, vth=(1.5, 0.02), tail=(100, 100), step=3)
        sim.set_state(st, d)
        states[d] = st
        orcs[d] = oracle_from_state(oracle_mod, wl, st, True)
        gbs[d] = tallies_of(sim.diagnostics(d))
    sim.step(1)
    for d in picked:
        orcs[d].step(1)
        compare_fp32(sim, orcs[d], states[d], "batched full %d" % d, gbase=gbs[d], coll_slack=1,
                     d=d)
    sim.close()

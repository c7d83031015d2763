"""GPU parity of the optional parts of the step through the C ABI, against the oracle:
binary Coulomb collisions between the particles of a cell (Sec. 3.2 names them as what
fine sorting makes simple).  Same bar as test_gpu_parity.py."""
import numpy as np
import pytest

import workloads
from test_gpu_parity import compare_fp64, one_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fspic():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1104_3998_amd as m
    m.lib()
    return m


def dense_periodic(**kw):
    """The periodic plasma at 100 times the density (n0 = 1e17 m^-3, same cell size in
    Debye lengths and the same omega_pe dt), where a step's Coulomb deflections are a few
    1e-3 rad for thermal electrons."""
    length, dt = workloads._periodic_grid(1e17, 3.0, 128)
    d = workloads.periodic_c1(n0_m3=1e17, length_m=length, dt_s=dt, coulomb=7,
                              coulomb_log=10.0)
    d.update(kw)
    return d


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
@pytest.mark.parametrize("bits", [1, 2, 4, 7])
def test_coulomb_one_step_from_seeded_state(fspic, oracle_mod, bits, precision):
    """One step with e-e (1), i-i (2), e-i (4) or all pairs from a seeded state whose cells
    hold odd and even numbers of particles of both species (a births tail of 50, which is
    not paired)."""
    wl = dense_periodic(coulomb=bits)
    print("coulomb", bits, precision, flush=True)
    st = workloads.synthetic_state(wl["n_cells"], (wl["n_e0"], wl["n_i0"]), precision,
                                   seed=31, vth=(0.5, 0.01), tail=(50, 50))
    one_step(fspic, oracle_mod, wl, st, precision, label="coulomb %d %s" % (bits, precision))


def test_coulomb_free_running_matches_oracle(fspic, oracle_mod):
    """20 free FP64 steps of the dense periodic plasma with every pair kind and the MCC on,
    each side from its own load."""
    wl = dense_periodic()
    sim = fspic.Simulation(wl, "fp64")
    orc = oracle_mod.Oracle(wl)
    orc.load()
    for k in range(20):
        sim.step(1)
        orc.step(1)
        compare_fp64(sim, orc, "coulomb step %d" % k)
    sim.close()


def test_coulomb_conserves_momentum_and_energy_per_cell(fspic):
    """Without a field (no drive, neutral load: each ion on an electron) and without MCC,
    one step changes velocities by the collisions alone: every cell keeps each species'
    momentum (like pairs) and the sum over both species of momentum and kinetic energy
    (FP64, to round-off)."""
    wl = dense_periodic(xsec="none", gas_pa=0.0, coulomb=7)
    n = 16384
    rng = np.random.default_rng(4)
    x = np.sort(rng.uniform(0, 128, n))
    st = {"step": 0, "next_id": [n, n]}
    v = {0: rng.normal(0, 0.5, size=(3, n)), 1: rng.normal(0, 0.01, size=(3, n))}
    for s in (0, 1):
        st[s] = dict(x=x, vx=v[s][0], vy=v[s][1], vz=v[s][2],
                     id=np.arange(n, dtype=np.uint32), n=n, n_sorted=n)
    sim = fspic.Simulation(wl, "fp64")
    sim.set_state(st)
    sim.step(1)
    out = sim.get_state()
    d = sim.derived[0]
    m = [1.0, d.energy_c[1] / d.energy_c[0]]  # mass ratio through the energy factors
    e0 = e1 = 0.0
    p0 = np.zeros(3)
    p1 = np.zeros(3)
    changed = 0
    for s in (0, 1):
        a = out[s]
        order = np.argsort(a["id"])
        vn = np.stack([a["vx"][order], a["vy"][order], a["vz"][order]])
        changed += int(np.any(vn != v[s], axis=0).sum())
        e0 += m[s] * (v[s] ** 2).sum()
        e1 += m[s] * (vn ** 2).sum()
        p0 += m[s] * v[s].sum(1)
        p1 += m[s] * vn.sum(1)
    assert changed > n  # collisions happened
    assert e1 == pytest.approx(e0, rel=1e-12)
    assert np.allclose(p1, p0, rtol=0, atol=1e-10 * np.abs(m[1] * v[1]).sum())
    sim.close()


# ------------------------------------------------------------------ electrode processes
def electrode_rf(**kw):
    """The small bounded RF discharge with secondary emission (gamma 0.5, 3 eV), electron
    reflection (probability 0.2) and warm ions (20 eV), so that every step has absorbed
    ions, emitted and reflected electrons at both electrodes."""
    d = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=40.0, see_gamma=0.5, see_te_ev=3.0,
                        refl_e=0.2, ti_ev=20.0, avg_start=0, diag_every=5)
    d.update(kw)
    return d


def wall_tallies(g):
    return [int(g.emitted[0]), int(g.emitted[1]), int(g.reflected[0]), int(g.reflected[1])]


def test_electrode_processes_free_running_match_oracle(fspic, oracle_mod):
    """20 free FP64 steps with emission and reflection, each side from its own load: the
    permutation (emitted electrons appended after the ionisation births, in the order of
    their parent ions), positions, velocities, node weights and every tally."""
    wl = electrode_rf()
    sim = fspic.Simulation(wl, "fp64")
    orc = oracle_mod.Oracle(wl)
    orc.load()
    seen = [0, 0, 0, 0]
    for k in range(20):
        sim.step(1)
        orc.step(1)
        compare_fp64(sim, orc, "electrode step %d" % k)
        t = orc.tallies()
        g = wall_tallies(sim.diagnostics())
        assert g == [t.emitted[0], t.emitted[1], t.reflected[0], t.reflected[1]], k
        seen = g
    assert min(seen) > 0  # every process happened at both walls
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
def test_electrode_processes_one_step_from_seeded_state(fspic, oracle_mod, precision):
    """One step from a seeded state with fast ions (0.8 cells per step) and electrons (3
    cells per step) and a births tail: many particles reach the electrodes."""
    wl = electrode_rf()
    st = workloads.synthetic_state(wl["n_cells"], (wl["n_e0"], wl["n_i0"]), precision,
                                   seed=37, vth=(3.0, 0.8), tail=(50, 50))
    one_step(fspic, oracle_mod, wl, st, precision, label="electrode " + precision)


def test_electrodes_with_series_capacitor(fspic, oracle_mod):
    """Emission, reflection and the series capacitor together: the conductor's charge
    follows the absorbed and emitted particles at the driven electrode (20 FP64 steps)."""
    wl = electrode_rf(circuit_cap_f_m2=2e-7, v0_volt=200.0)
    sim = fspic.Simulation(wl, "fp64")
    orc = oracle_mod.Oracle(wl)
    orc.load()
    d = sim.derived[0]
    for k in range(20):
        sim.step(1)
        orc.step(1)
        compare_fp64(sim, orc, "electrode+circuit step %d" % k)
        g, t = sim.diagnostics(), orc.tallies()
        assert g.circuit_charge == pytest.approx(t.q_circuit, rel=1e-10, abs=1e-10)
        assert g.phi_driven_v / d.phi_scale == pytest.approx(t.phi0, rel=1e-10, abs=1e-10)
    sim.close()


# ------------------------------------------------------------------ unsorted variant
@pytest.mark.parametrize("name,wl", [("periodic", workloads.periodic_c1(sort_mode="none")),
                                     ("rf_small", workloads.rf_c2(n_e0=20000, n_i0=20000,
                                                                  gas_pa=30.0,
                                                                  sort_mode="none"))],
                         ids=["periodic", "rf_small"])
def test_unsorted_free_running_matches_oracle(fspic, oracle_mod, name, wl):
    """The unsorted variant (survivors keep their order, births appended, the deposit
    added straight into the node array): 20 free FP64 steps against the oracle in the
    same order mode, the permutation exact."""
    sim = fspic.Simulation(wl, "fp64")
    orc = oracle_mod.Oracle(wl)
    orc.load()
    for k in range(20):
        sim.step(1)
        orc.step(1)
        compare_fp64(sim, orc, "unsorted %s step %d" % (name, k))
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
def test_unsorted_one_step_from_seeded_state(fspic, oracle_mod, precision):
    """One unsorted step from a seeded state whose last particles are out of cell order:
    the survivors must come out in input order, then the births."""
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=30.0, sort_mode="none",
                         see_gamma=0.3, refl_e=0.1, ti_ev=5.0)
    st = workloads.synthetic_state(wl["n_cells"], (20000, 20000), precision, seed=43,
                                   vth=(2.5, 0.3), tail=(2000, 2000))
    one_step(fspic, oracle_mod, wl, st, precision, label="unsorted " + precision)


# ------------------------------------------------------------------ the paper's fine sort
def compare_fine(sim, orc, label, fp32=False, gbase=None, obase=None):
    """The fine sort keeps each sorting cell's particles together, in an order inside the
    cell that is not fixed: the state is compared particle by particle through the ids
    (the same set; positions, velocities at the path's bar), the array must run through
    the sorting cells in order, and node weights and tallies must match."""
    from test_gpu_parity import (oracle_mod_deposit, oracle_tallies, positions, same_tallies,
                                 tallies_of, velocities)
    st = sim.get_state()
    g, o = tallies_of(sim.diagnostics()), oracle_tallies(orc.tallies())
    G = max(1, int(sim.workloads[0].get("grid_points_per_sort_cell", 3)) - 1)
    for s in (0, 1):
        a, po = st[s], orc.particles(s)
        assert a["n"] == orc.count(s), (label, s, "count")
        ig, io = np.argsort(a["id"]), np.argsort(po["id"])
        assert np.array_equal(a["id"][ig], po["id"][io]), (label, s, "id set")
        x = positions(a, fp32)
        sc = np.floor(x).astype(np.int64) // G
        assert np.all(np.diff(sc) >= 0), (label, s, "sorting cells in order")
        xo = po["x"][io]
        vo = np.stack([po["vx"], po["vy"], po["vz"]])[:, io]
        v = velocities(a, fp32)[:, ig]
        scale = np.max(np.abs(vo), initial=1e-30)
        if fp32:
            assert np.max(np.abs(x[ig] - xo), initial=0) <= 1e-4, (label, s, "x")
            assert np.max(np.abs(v - vo), initial=0) <= 1e-5 * scale, (label, s, "v")
        else:
            assert np.max(np.abs(x[ig] - xo), initial=0) <= 1e-12 * sim.workloads[0]["n_cells"]
            assert np.max(np.abs(v - vo), initial=0) <= 1e-12 * scale, (label, s, "v")
        wo = orc.grid("w_e" if s == 0 else "w_i")
        if fp32:
            # free-running FP32 positions drift apart by up to 1e-4 cells (above), and the
            # node weights with them: they must be the oracle's deposit of the GPU's own
            # particles to 1e-9 and follow the oracle's weights to 1e-4 of max w
            wl_ = sim.workloads[0]
            wself = oracle_mod_deposit(wl_["periodic"], wl_["n_cells"], x)
            assert np.max(np.abs(a["w"] - wself)) <= 1e-9 * max(wself.max(), 1.0), (label, s)
            assert np.max(np.abs(a["w"] - wo)) <= 1e-4 * max(wo.max(), 1.0), (label, s, "w")
            # the absorbed energy sums the drifted FP32 velocities: held to their 1e-5 bar
            for k in ("coll", "absorbed", "births"):
                assert g[s][k] == o[s][k], (label, s, k)
            for w in range(2):
                assert g[s]["abs_e"][w] == pytest.approx(o[s]["abs_e"][w], rel=1e-5), (label, s)
        else:
            assert np.max(np.abs(a["w"] - wo)) <= 1e-12 * max(wo.max(), 1.0), (label, s, "w")
            same_tallies(g[s], o[s], label, s)


@pytest.mark.parametrize("G", [1, 2, 4])
def test_fine_sort_free_running_matches_oracle(fspic, oracle_mod, G):
    """The paper's fine sort (sorting cells of G grid cells, fixed capacity, sorted in place
    with steps 1a/1b, 2 and 3 every step; births into their sorting cell with ids in
    increasing parent id): 20 free FP64 steps of the ionising bounded discharge, each side
    from its own load."""
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=30.0, sort_mode="fine",
                         grid_points_per_sort_cell=G + 1, refl_e=0.1)
    sim = fspic.Simulation(wl, "fp64")
    orc = oracle_mod.Oracle(wl)
    orc.load()
    for k in range(20):
        sim.step(1)
        orc.step(1)
        compare_fine(sim, orc, "fine G=%d step %d" % (G, k))
    assert sum(sim.diagnostics().births) > 0
    sim.close()


def test_fine_sort_periodic_and_far_movers(fspic, oracle_mod):
    """Periodic plasma with fast electrons (step 3 moves them farther than one sorting cell,
    across the periodic seam too), one step from a seeded state, FP64 and FP32."""
    for precision in ("fp64", "fp32_offset"):
        wl = workloads.periodic_c1(sort_mode="fine", grid_points_per_sort_cell=3)
        st = workloads.synthetic_state(wl["n_cells"], (wl["n_e0"], wl["n_i0"]), precision,
                                       seed=47, vth=(0.4, 0.01), fast=(300, 0),
                                       fast_speed=(3.0, 60.0))
        fp32 = precision == "fp32_offset"
        from test_gpu_parity import oracle_from_state
        sim = fspic.Simulation(wl, precision)
        sim.set_state(st)
        orc = oracle_from_state(oracle_mod, wl, st, fp32)
        sim.step(1)
        orc.step(1)
        compare_fine(sim, orc, "fine periodic " + precision, fp32=fp32)
        sim.close()


def test_fine_sort_fp32_free_running(fspic, oracle_mod):
    """The FP32 layout under the fine sort, 10 free steps against the oracle in the same
    layout."""
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=30.0, sort_mode="fine")
    sim = fspic.Simulation(wl, "fp32_offset")
    orc = oracle_mod.Oracle(wl, fp32_offset=True)
    orc.load()
    for k in range(10):
        sim.step(1)
        orc.step(1)
        compare_fine(sim, orc, "fine fp32 step %d" % k, fp32=True)
    sim.close()


# ------------------------------------------------------------------ the lagged sort
@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
def test_lagged_sort_one_step_from_seeded_state(fspic, oracle_mod, precision):
    """The lagged sort (the array ordered by the cell each particle held at the start of
    the step; absorbed particles leave dead records): one step from a seeded state with a
    births tail and fast electrons, in the ionising bounded discharge."""
    from test_gpu_parity import one_step
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=30.0, sort_mode="lag")
    st = workloads.synthetic_state(wl["n_cells"], (20000, 20000), precision, seed=53,
                                   vth=(2.5, 0.3), tail=(300, 300), fast=(200, 0),
                                   fast_speed=(3.0, 60.0))
    one_step(fspic, oracle_mod, wl, st, precision, label="lag " + precision)


def test_lagged_sort_periodic_one_step(fspic, oracle_mod):
    """Periodic plasma with far movers across the seam under the lagged sort."""
    from test_gpu_parity import one_step
    for precision in ("fp64", "fp32_offset"):
        wl = workloads.periodic_c1(sort_mode="lag")
        st = workloads.synthetic_state(wl["n_cells"], (wl["n_e0"], wl["n_i0"]), precision,
                                       seed=59, vth=(0.4, 0.01), fast=(300, 0),
                                       fast_speed=(3.0, 60.0))
        one_step(fspic, oracle_mod, wl, st, precision, label="lag periodic " + precision)


def test_lagged_sort_free_running_matches_oracle(fspic, oracle_mod):
    """20 free FP64 steps of the ionising bounded discharge with electron reflection under
    the lagged sort, each side from its own load: the same array order (dead records left
    out), states, weights and tallies."""
    from test_gpu_parity import compare_fp64
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=30.0, sort_mode="lag", refl_e=0.1)
    sim = fspic.Simulation(wl, "fp64")
    orc = oracle_mod.Oracle(wl)
    orc.load()
    for k in range(20):
        sim.step(1)
        orc.step(1)
        compare_fp64(sim, orc, "lag step %d" % k)
    assert sum(sim.diagnostics().births) > 0
    assert sum(sim.diagnostics().absorbed[0]) > 0
    sim.close()


def test_lagged_sort_same_physics_as_counting_sort(fspic):
    """The array order does not enter the physics: 20 FP64 steps of the same collisionless
    discharge under the lagged and the counting sort give the same particles (matched by
    id) bit for bit, the same node weights (the fixed-point deposit does not depend on
    the order) and the same absorbed counts."""
    from test_gpu_parity import positions, tallies_of, velocities
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=0.0, xsec="none")
    sims = {m: fspic.Simulation(dict(wl, sort_mode=m), "fp64") for m in ("counting", "lag")}
    for sim in sims.values():
        sim.step(20)
    a, b = (sims[m].get_state() for m in ("counting", "lag"))
    for s in (0, 1):
        assert a[s]["n"] == b[s]["n"]
        ia, ib = np.argsort(a[s]["id"]), np.argsort(b[s]["id"])
        assert np.array_equal(a[s]["id"][ia], b[s]["id"][ib])
        assert np.array_equal(positions(a[s], False)[ia], positions(b[s], False)[ib])
        assert np.array_equal(velocities(a[s], False)[:, ia], velocities(b[s], False)[:, ib])
        assert np.array_equal(a[s]["w"], b[s]["w"])
    ta, tb = (tallies_of(sims[m].diagnostics()) for m in ("counting", "lag"))
    for s in (0, 1):
        assert ta[s]["absorbed"] == tb[s]["absorbed"]
    for sim in sims.values():
        sim.close()

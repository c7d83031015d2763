"""Pins of the oracle functions that the whole-cycle physics tests do not reach on their own:
the EEDF binning (against the analytic Maxwellian energy distribution), the time-average
accumulators and the diagnostic cadence (against snapshots taken between steps), the
leap-frog half-step back-push (against a field computed here from scratch), the absorbed
energy tally (a field-free construction), the load's velocity spreads and the gas
temperature (closed forms from the physical constants), the direction sampler's other
components, and the step's energy / momentum / charge diagnostics (conservation laws and
the load temperature)."""
import math

import numpy as np
import pytest
from scipy.special import gammainc

import workloads

QE = 1.602176634e-19
ME = 9.1093837015e-31
AMU = 1.66053906660e-27
KB = 1.380649e-23


def _tiny_field(wl):
    """The same workload with a macro-particle weight so small that the self-field cannot
    move a particle measurably in one step (kappa scales with n0; dx and dt are kept)."""
    return dict(wl, n0_m3=1e3)


@pytest.mark.parametrize("te", [2.0, 3.0])
def test_eedf_of_maxwellian_load(oracle_mod, te):
    """Electrons loaded at T_e, pushed once in a negligible field, binned at step 0: bin b
    of width 60/120 eV holds N [P(3/2, e_hi/T) - P(3/2, e_lo/T)] (regularised lower
    incomplete gamma: the energy distribution of a 3-D Maxwellian), the overflow bin the
    rest; every bin within 4 sigma of its binomial expectation."""
    n = 200_000
    wl = _tiny_field(workloads.periodic_c1(n_e0=n, n_i0=n, te_ev=te, xsec="none",
                                           gas_pa=0.0, avg_start=0, diag_every=1))
    o = oracle_mod.Oracle(wl)
    o.load()
    o.step(1)
    assert o.tallies().eedf_samples == 1
    h = o.grid("eedf")
    edges = np.linspace(0.0, 60.0, 121)
    cdf = gammainc(1.5, edges / te)
    expect = np.append(n * np.diff(cdf), n * (1.0 - cdf[-1]))
    assert h.sum() == n
    tol = 4.0 * np.sqrt(expect * (1.0 - expect / n)) + 1.0
    bad = np.abs(h - expect) > tol
    assert not bad.any(), (np.flatnonzero(bad), h[bad], expect[bad])
    # the mean bin energy: sensitive to a scale error of the bins of a fraction of 1 %
    mid = (edges[:-1] + edges[1:]) / 2
    p = expect[:-1] / n
    m_exp = (mid * p).sum()
    sd = math.sqrt(((mid - m_exp) ** 2 * p).sum() / n)
    assert abs((mid * h[:-1]).sum() / n - m_exp) < 4 * sd


def test_time_average_accumulators_and_cadence(oracle_mod):
    """The accumulators hold, for every step n >= avg_start, the node weights the step's
    field is solved from and the potential of that solve; the EEDF is sampled at steps
    avg_start, avg_start + diag_every, ... and bins every electron pushed in them."""
    wl = workloads.rf_c2(n_e0=5000, n_i0=5000, gas_pa=30.0, avg_start=3, diag_every=2)
    o = oracle_mod.Oracle(wl)
    o.load()
    acc = {k: np.zeros(o.n_nodes) for k in ("w_e", "w_i", "phi")}
    n_avg, n_eedf, eedf_particles = 0, 0, 0
    for step in range(12):
        we, wi, ne = o.grid("w_e"), o.grid("w_i"), o.count(0)
        o.step(1)
        if step >= 3:
            acc["w_e"] += we
            acc["w_i"] += wi
            acc["phi"] += o.grid("phi")
            n_avg += 1
            if (step - 3) % 2 == 0:
                n_eedf += 1
                eedf_particles += ne
    t = o.tallies()
    assert t.acc_count == n_avg == 9
    assert t.eedf_samples == n_eedf == 5
    for k, name in (("w_e", "acc_w_e"), ("w_i", "acc_w_i"), ("phi", "acc_phi")):
        ref = acc[k]
        assert np.max(np.abs(o.grid(name) - ref)) <= 1e-12 * np.abs(ref).max(), k
    assert o.grid("eedf").sum() == eedf_particles


def _periodic_field(x_e, x_i, n):
    """Field of two species on a periodic grid, computed independently: hat-function
    weights summed directly, the three-point Poisson system with the mean charge removed
    and Phi_0 = 0 solved densely, centred differences."""
    j = np.arange(n)

    def weights(x):
        d = np.abs(x[:, None] - j[None, :])
        d = np.minimum(d, n - d)
        return np.maximum(0.0, 1.0 - d).sum(axis=0)

    rho = weights(x_i) - weights(x_e)
    rho = rho - rho.mean()
    m = n - 1
    a = -2.0 * np.eye(m) + np.eye(m, k=1) + np.eye(m, k=-1)
    phi = np.zeros(n)
    phi[1:] = np.linalg.solve(a, -rho[1:])
    return (np.roll(phi, 1) - np.roll(phi, -1)) / 2.0


def test_half_step_back_push_cold_load(oracle_mod):
    """Leap-frog start (Sec. 3.6): a cold quiet start has v = 0, so after the load
    v_x(-1/2) = -kappa_s E(x_0) / 2 exactly, with E gathered linearly from a field this
    test computes itself; v_y = v_z = 0.  A wrong sign or factor fails."""
    wl = workloads.langmuir_c1(n_e0=2048, n_i0=2048, langmuir_amp_cells=0.2)
    n = wl["n_cells"]
    o = oracle_mod.Oracle(wl)
    o.load()
    c = o.consts()
    k = np.arange(2048)
    x_i = (k + 0.5) * n / 2048.0
    x_e = np.mod(x_i + 0.2 * np.sin(2 * np.pi * x_i / n), n)
    ef = _periodic_field(x_e, x_i, n)
    for s, x0 in ((0, x_e), (1, x_i)):
        p = o.particles(s)
        order = np.argsort(p["id"])
        assert np.allclose(p["x"][order], x0, rtol=0, atol=1e-12)
        cell = np.floor(x0).astype(int)
        f = x0 - cell
        e_at = (1 - f) * ef[cell] + f * ef[(cell + 1) % n]
        want = -0.5 * c.kappa[s] * e_at
        got = p["vx"][order]
        assert np.max(np.abs(got - want)) <= 1e-9 * np.abs(want).max(), s
        assert np.abs(want).max() > 0
        assert not p["vy"].any() and not p["vz"].any()


def test_absorbed_energy_tally_field_free(oracle_mod):
    """Electrons and ions at identical positions in a bounded box with no drive: the net
    charge is zero at every node, so E = 0 and the push is free streaming.  The particles
    that cross x = 0 or x = N are tallied at that wall with energy sum (1/2) m |v|^2 in eV,
    the constant computed here from the physical constants."""
    wl = workloads.rf_c2(n_e0=400, n_i0=400, v0_volt=0.0, xsec="none", gas_pa=0.0)
    n = wl["n_cells"]
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(0, 3, 200), rng.uniform(n - 3, n, 200)])
    o = oracle_mod.Oracle(wl)
    dx = wl["length_m"] / n
    vunit = dx / wl["dt_s"]
    expect = {}
    for s, mass, vs in ((0, ME, 2.5), (1, 40 * AMU, 2.0)):
        v = rng.normal(0, vs, size=(3, 400))
        o.set_particles(s, dict(x=x, vx=v[0], vy=v[1], vz=v[2],
                                id=np.arange(400, dtype=np.uint32)))
        xn = x + v[0]
        e = 0.5 * mass * vunit ** 2 * (v ** 2).sum(axis=0) / QE
        expect[s] = ((xn < 0).sum(), (xn >= n).sum(), e[xn < 0].sum(), e[xn >= n].sum())
    o.set_counters(0, 400, 400)
    o.step(1)
    t = o.tallies()
    assert np.abs(o.grid("E")).max() == 0.0
    for s in (0, 1):
        assert (t.absorbed[s][0], t.absorbed[s][1]) == expect[s][:2]
        assert expect[s][0] > 10 and expect[s][1] > 10
        assert t.absorbed_energy_ev[s][0] == pytest.approx(expect[s][2], rel=1e-12)
        assert t.absorbed_energy_ev[s][1] == pytest.approx(expect[s][3], rel=1e-12)


def test_load_velocity_spread_closed_form(oracle_mod):
    """The Maxwellian load: every velocity component of species s is normal with mean 0 and
    standard deviation sqrt(k T_s / m_s) dt / dx, computed here from the physical
    constants (not from the oracle's derived values); 4-sigma bands on mean and variance."""
    n = 200_000
    wl = _tiny_field(workloads.rf_c2(n_e0=n, n_i0=n, te_ev=2.0, ti_ev=0.5))
    o = oracle_mod.Oracle(wl)
    o.load()
    dx = wl["length_m"] / wl["n_cells"]
    for s, t_ev, mass in ((0, 2.0, ME), (1, 0.5, 40 * AMU)):
        sig = math.sqrt(t_ev * QE / mass) * wl["dt_s"] / dx
        p = o.particles(s)
        for k in ("vx", "vy", "vz"):
            v = p[k]
            assert abs(v.mean()) < 4 * sig / math.sqrt(n), (s, k)
            assert v.var() == pytest.approx(sig ** 2, abs=4 * sig ** 2 * math.sqrt(2.0 / n)), (s, k)


def test_gas_temperature_of_new_ions_closed_form(oracle_mod):
    """Ions born in an ionisation have the gas Maxwellian: each component's variance is
    k T_g / M (dt / dx)^2 with T_g = 300 K, from the physical constants."""
    wl = workloads.rf_c2(gas_pa=20000.0, n_e0=64, n_i0=64)
    o = oracle_mod.Oracle(wl)
    c = o.consts()
    v0 = math.sqrt(60.0 / c.energy_c[0])
    vi = []
    for pid in range(80_000):
        ch, _, _, v_ion = o.collide(0, pid, 7, [v0, 0.0, 0.0])
        if ch == 3:
            vi.append(v_ion)
    vi = np.array(vi)
    m = len(vi)
    assert m > 1000
    dx = wl["length_m"] / wl["n_cells"]
    sig2 = KB * 300.0 / (40 * AMU) * (wl["dt_s"] / dx) ** 2
    for k in range(3):
        assert abs(vi[:, k].mean()) < 4 * math.sqrt(sig2 / m)
        assert vi[:, k].var() == pytest.approx(sig2, abs=4 * sig2 * math.sqrt(2.0 / m))


def test_isotropic_direction_all_components(oracle_mod):
    """The scattered direction after an excitation is isotropic: every component has mean
    0 and mean square 1/3, and distinct components are uncorrelated."""
    o = oracle_mod.Oracle(workloads.rf_c2(gas_pa=20000.0, n_e0=64, n_i0=64))
    c = o.consts()
    v0 = math.sqrt(40.0 / c.energy_c[0])
    dirs = []
    for pid in range(60_000):
        ch, v, _, _ = o.collide(0, pid, 2, [0.0, 0.0, v0])
        if ch in (1, 2):
            dirs.append(v / np.linalg.norm(v))
    u = np.array(dirs)
    m = len(u)
    assert m > 20_000
    for k in range(3):
        assert abs(u[:, k].mean()) < 4 / math.sqrt(3 * m)
        assert (u[:, k] ** 2).mean() == pytest.approx(1 / 3, abs=4 * math.sqrt(4 / 45 / m))
    for a, b in ((0, 1), (0, 2), (1, 2)):
        assert abs((u[:, a] * u[:, b]).mean()) < 4 / math.sqrt(15 * m)


def test_step_diagnostics_conservation(oracle_mod):
    """The per-step diagnostics of a periodic plasma without collisions: the net charge
    sums to N_i - N_e = 0; kinetic plus field energy stays constant to 1e-3 over 200 steps
    while the field energy alone changes by much more; the x-momentum is conserved to
    1e-10 of sum |p| step to step."""
    wl = workloads.periodic_c1(xsec="none", gas_pa=0.0)
    o = oracle_mod.Oracle(wl)
    o.load()
    c = o.consts()
    scale = sum(np.abs(o.particles(s)["vx"]).sum() / abs(c.kappa[s]) for s in (0, 1))
    tot, fe, mom = [], [], []
    for _ in range(200):
        o.step(1)
        t = o.tallies()
        assert abs(t.sum_rho) < 1e-9
        tot.append(t.kinetic[0] + t.kinetic[1] + t.field_energy)
        fe.append(t.field_energy)
        mom.append(t.momentum)
    tot, fe, mom = np.array(tot), np.array(fe), np.array(mom)
    assert np.abs(tot - tot[0]).max() / tot[0] < 1e-3
    assert (fe.max() - fe.min()) > 10 * np.abs(tot - tot[0]).max()
    assert np.abs(np.diff(mom)).max() <= 1e-10 * scale
    assert np.abs(mom).max() > 1e-6 * scale


def test_kinetic_diagnostic_is_the_load_temperature(oracle_mod):
    """Right after a Maxwellian load (negligible field) the electrons' kinetic energy per
    particle is (3/2) T_e: the diagnostic in field-energy units times m vunit^2 |kappa| / e
    is the energy in eV.  A 4-sigma band (the energy of a particle has variance 3/2 T^2)."""
    n = 100_000
    wl = _tiny_field(workloads.rf_c2(n_e0=n, n_i0=n, te_ev=2.0, xsec="none", gas_pa=0.0))
    o = oracle_mod.Oracle(wl)
    o.load()
    o.step(1)
    c = o.consts()
    dx = wl["length_m"] / wl["n_cells"]
    vunit = dx / wl["dt_s"]
    ev = o.tallies().kinetic[0] * ME * vunit ** 2 * abs(c.kappa[0]) / QE
    assert ev / n == pytest.approx(1.5 * 2.0, abs=4 * math.sqrt(1.5) * 2.0 / math.sqrt(n))
    # the charge diagnostic of a bounded box: sum of the net node charge = N_i - N_e
    wl2 = workloads.rf_c2(n_e0=3000, n_i0=2500)
    o2 = oracle_mod.Oracle(wl2)
    o2.load()
    o2.step(1)
    assert o2.tallies().sum_rho == pytest.approx(2500 - 3000, abs=1e-9)

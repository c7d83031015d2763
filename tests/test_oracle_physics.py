"""Physics pins of the whole oracle cycle (Sec. 2 cycle; Sec. 3.3 normalisation):
closed-form constants, the Langmuir frequency of a cold periodic plasma, exact momentum
conservation of the momentum-conserving scheme, charge / particle-count identities and
energy conservation without collisions."""
import math

import numpy as np
import pytest
from scipy.optimize import curve_fit

import workloads

QE = 1.602176634e-19
ME = 9.1093837015e-31
AMU = 1.66053906660e-27
EPS0 = 8.8541878128e-12


def test_normalised_push_factor_closed_form(oracle_mod):
    """eq. push_velocity: kappa = Q^2 dt^2 / (eps0 dx M A); with the macro-particle weight
    W/A = n0 L / N_e0 this is -(w_pe dt)^2 N / N_e0 for electrons (-3.125e-4 for the
    periodic plasma) and +(m_e/m_i)(w_pe dt)^2 N / N_e0 for ions."""
    wl = workloads.periodic_c1()
    c = oracle_mod.Oracle(wl).consts()
    wpe = math.sqrt(wl["n0_m3"] * QE * QE / (EPS0 * ME))
    base = (wpe * wl["dt_s"]) ** 2 * wl["n_cells"] / wl["n_e0"]
    assert c.kappa[0] == pytest.approx(-base, rel=1e-12)
    assert c.kappa[0] == pytest.approx(-3.125e-4, rel=1e-9)
    assert c.kappa[1] == pytest.approx(base * ME / (40 * AMU), rel=1e-12)
    # phi unit Q dx / (eps0 A); the RF amplitude in those units
    wl2 = workloads.rf_c2()
    c2 = oracle_mod.Oracle(dict(wl2, n_e0=1000, n_i0=1000)).consts()
    dx = wl2["length_m"] / wl2["n_cells"]
    wpa = wl2["n0_m3"] * wl2["length_m"] / 1000
    assert c2.phi_scale == pytest.approx(QE * wpa * dx / EPS0, rel=1e-14)
    assert c2.vhat_amp == pytest.approx(200.0 / c2.phi_scale, rel=1e-14)
    # energy of one normalised velocity unit in eV
    assert c2.energy_c[0] == pytest.approx(0.5 * ME * (dx / wl2["dt_s"]) ** 2 / QE, rel=1e-14)


def test_langmuir_frequency(oracle_mod):
    """Cold periodic plasma, mode 1, 0.01-cell displacement: the field oscillates at the
    plasma frequency.  With linear weighting, the three-point Laplacian and the centred
    gradient the effective frequency is w_pe sqrt(1 + m_e/m_i) sqrt(sinc(k dx) sinc^2(k dx/2))
    and leap-frog maps it to (2/dt) asin(w dt / 2): 1.00138 w_pe for k dx = 2 pi / 128."""
    wl = workloads.langmuir_c1()
    o = oracle_mod.Oracle(wl)
    o.load()
    n = wl["n_cells"]
    j = np.arange(n)
    basis = np.exp(-2j * np.pi * j / n)
    sig = []
    for _ in range(wl["steps"]):
        o.step()
        sig.append(np.dot(o.grid("E"), basis))
    sig = np.array(sig)
    s = sig.imag if np.var(sig.imag) > np.var(sig.real) else sig.real
    t = np.arange(len(s), dtype=float)
    spec = np.abs(np.fft.rfft(s - s.mean()))
    w0 = 2 * np.pi * np.argmax(spec) / len(s)
    popt, _ = curve_fit(lambda t, a, w, p, c: a * np.cos(w * t + p) + c, t, s,
                        p0=[np.abs(s).max(), w0, 0.0, 0.0])
    w_meas = abs(popt[1]) / wl["dt_s"]
    wpe = math.sqrt(wl["n0_m3"] * QE * QE / (EPS0 * ME))
    kdx = 2 * np.pi / n
    grid = math.sqrt(math.sin(kdx) / kdx * (math.sin(kdx / 2) / (kdx / 2)) ** 2)
    w_eff = wpe * math.sqrt(1 + ME / (40 * AMU)) * grid
    w_pred = 2 / wl["dt_s"] * math.asin(w_eff * wl["dt_s"] / 2)
    assert w_pred / wpe == pytest.approx(1.00138, abs=1e-5)
    assert w_meas / wpe == pytest.approx(1.0, abs=5e-3)
    assert w_meas / w_pred == pytest.approx(1.0, abs=2e-4)


def _momentum(o, c):
    p = 0.0
    for s in (0, 1):
        p += o.particles(s)["vx"].sum() / abs(c.kappa[s])
    return p


def test_momentum_conserved_periodic(oracle_mod):
    """Periodic, no collisions: the momentum change sum_i (q_i/e) E(x_i) equals
    sum_j rho_j E_j (same linear weights for gather and deposit), which the centred
    gradient of the three-point potential makes vanish identically."""
    wl = workloads.periodic_c1(xsec="none", gas_pa=0.0)
    o = oracle_mod.Oracle(wl)
    o.load()
    c = o.consts()
    scale = sum(np.abs(o.particles(s)["vx"]).sum() / abs(c.kappa[s]) for s in (0, 1))
    p_prev = _momentum(o, c)
    for _ in range(20):
        o.step()
        p = _momentum(o, c)
        assert abs(p - p_prev) <= 1e-10 * scale
        p_prev = p


def test_charge_and_count_identities_periodic(oracle_mod):
    wl = workloads.periodic_c1()
    o = oracle_mod.Oracle(wl)
    o.load()
    for _ in range(25):
        o.step()
        assert o.count(0) == 16384 and o.count(1) == 16384
        we, wi = o.grid("w_e"), o.grid("w_i")
        assert we.sum() == pytest.approx(16384, rel=1e-13)
        assert (wi - we).sum() == pytest.approx(0.0, abs=1e-8)
        ids = o.particles(0)["id"]
        assert np.array_equal(np.sort(ids), np.arange(16384))
        x = o.particles(0)["x"]
        assert np.all(np.diff(np.floor(x)) >= 0)  # sorted by cell


def test_count_balance_bounded(oracle_mod):
    """Bounded RF discharge: N_s(n+1) = N_s(n) - absorbed + born, exactly; the weights sum
    to the particle counts; every id is unique and new ids continue the counter."""
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=40.0)
    o = oracle_mod.Oracle(wl)
    o.load()
    t_prev = o.tallies()
    n_prev = [o.count(0), o.count(1)]
    for _ in range(30):
        o.step()
        t = o.tallies()
        for s in (0, 1):
            absorbed = sum(t.absorbed[s][w] - t_prev.absorbed[s][w] for w in (0, 1))
            born = t.births[s] - t_prev.births[s]
            assert o.count(s) == n_prev[s] - absorbed + born
            assert o.grid("w_e" if s == 0 else "w_i").sum() == pytest.approx(o.count(s), rel=1e-12)
            ids = o.particles(s)["id"]
            assert len(np.unique(ids)) == ids.size
            assert ids.max() < t.next_id[s]
        n_prev = [o.count(0), o.count(1)]
        t_prev = t
    assert t.births[0] > 0 and t.births[0] == t.births[1]


def test_energy_conservation_no_collisions(oracle_mod):
    """Periodic plasma without collisions over 200 steps: kinetic energy (mean of the two
    half-step values, v^2 / 2|kappa| per particle in field-energy units) plus field energy
    (1/2 sum of squared cell-centre fields) changes by less than 1e-3 relative."""
    wl = workloads.periodic_c1(xsec="none", gas_pa=0.0)
    o = oracle_mod.Oracle(wl)
    o.load()
    c = o.consts()
    n = wl["n_cells"]

    def ke(s):
        p = o.particles(s)
        return (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2) / (2 * abs(c.kappa[s]))

    tot = []
    k_prev = [ke(0), ke(1)]
    for _ in range(200):
        o.step()
        k_now = [ke(0), ke(1)]
        phi = o.grid("phi")
        fe = 0.5 * np.sum((phi - np.roll(phi, -1)) ** 2)
        kin = sum(0.5 * (k_prev[s].sum() + k_now[s].sum()) for s in (0, 1))
        tot.append(kin + fe)
        k_prev = k_now
    tot = np.array(tot)
    drift = np.abs(tot - tot[0]).max() / tot[0]
    assert drift < 1e-3

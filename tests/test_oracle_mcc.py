"""Pins of the oracle's Monte-Carlo collisions (Sec. 3.8: modified null-collision
method, eq. null_collision; the cross sections are the synthetic Ar-like model that
stands in for the paper's unprinted argon fits)."""
import math

import numpy as np
import pytest

import workloads

QE = 1.602176634e-19
ME = 9.1093837015e-31
AMU = 1.66053906660e-27
KB = 1.380649e-23


def test_cross_section_spot_values(oracle_mod):
    # sigma_el(12 eV): x = 1 -> 3e-19 * 1.05 / 2
    assert oracle_mod.xsec("ar_like", 0, 12.0)[0] == pytest.approx(1.575e-19, rel=1e-14)
    # ionisation peak of 2u/(1+u^2) at u = 1, i.e. 15.8 + 60 eV
    assert oracle_mod.xsec("ar_like", 0, 75.8)[2] == pytest.approx(3e-20, rel=1e-14)
    # excitation peak at 11.5 + 20 eV
    assert oracle_mod.xsec("ar_like", 0, 31.5)[1] == pytest.approx(2e-20, rel=1e-14)
    # thresholds: nothing at or below 11.5 / 15.8 eV, something just above
    s = oracle_mod.xsec("ar_like", 0, 11.5)
    assert s[1] == 0.0 and s[2] == 0.0
    assert oracle_mod.xsec("ar_like", 0, 11.5001)[1] > 0
    assert oracle_mod.xsec("ar_like", 0, 15.8)[2] == 0.0
    assert oracle_mod.xsec("ar_like", 0, 15.8001)[2] > 0
    # ions at rest energy: (1 + 2) 2e-19 and (1 + 1) 3e-19
    si = oracle_mod.xsec("ar_like", 1, 0.0)
    assert si[0] == pytest.approx(6e-19) and si[1] == pytest.approx(6e-19)
    assert si[2] == 0.0
    # constant model: electrons only
    assert list(oracle_mod.xsec("const_e_elastic", 0, 3.0, 1e-19)) == [1e-19, 0, 0]
    assert list(oracle_mod.xsec("const_e_elastic", 1, 3.0, 1e-19)) == [0, 0, 0]


def test_null_frequency_bounds_total_frequency(oracle_mod):
    """nu0 >= n_g sum sigma v on an independent (offset, finer) energy grid, and it is the
    maximum to within the grid resolution."""
    wl = workloads.rf_c2()
    o = oracle_mod.Oracle(dict(wl, n_e0=64, n_i0=64))
    c = o.consts()
    for sp, mass in ((0, ME), (1, 40 * AMU)):
        eps = np.linspace(0.0037, 5000, 400001)
        tot = np.array([oracle_mod.xsec("ar_like", sp, e).sum() for e in eps[::10]])
        nu = c.n_gas * tot * np.sqrt(2 * QE * eps[::10] / mass)
        assert nu.max() <= c.nu0[sp]
        assert nu.max() > c.nu0[sp] * (1 - 1e-3)
    # n_g = p / (k T)
    assert c.n_gas == pytest.approx(10.0 / (KB * 300.0), rel=1e-14)


def test_constant_sigma_null_frequency_and_threshold(oracle_mod):
    """Periodic case: nu0 = n_g sigma v(100 eV) = 1.432e8 /s, P0 = 1 - exp(-nu0 dt),
    T0 = floor(P0 2^32)."""
    o = oracle_mod.Oracle(workloads.periodic_c1())
    c = o.consts()
    ng = 1.0 / (KB * 300.0)
    nu0 = ng * 1e-19 * math.sqrt(2 * QE * 100.0 / ME)
    assert c.nu0[0] == pytest.approx(nu0, rel=1e-14)
    assert c.nu0[0] == pytest.approx(1.432e8, rel=1e-3)
    p0 = 1 - math.exp(-nu0 * workloads.periodic_c1()["dt_s"])
    assert c.p0[0] == pytest.approx(p0, rel=1e-12)
    assert c.t0[0] == math.floor(p0 * 2**32)
    assert c.nu0[1] == 0.0 and c.t0[1] == 0


def test_electron_elastic_kinematics(oracle_mod):
    """Elastic scattering off a gas atom at rest with isotropic new direction: the mean
    fractional energy change is -2 m/M; the new directions are isotropic."""
    wl = workloads.periodic_c1(gas_pa=5000.0)  # P0 near 1: nearly every draw collides
    o = oracle_mod.Oracle(wl)
    c = o.consts()
    v0 = math.sqrt(50.0 / c.energy_c[0])  # 50 eV, below the 100 eV cap
    dfrac, cx, cx2, n = [], [], [], 0
    for pid in range(40000):
        ch, v, _, _ = o.collide(0, pid, 3, [v0, 0.0, 0.0])
        if ch == 0:
            continue
        assert ch == 1
        e1 = c.energy_c[0] * float(v @ v)
        dfrac.append(e1 / 50.0 - 1.0)
        u = v / math.sqrt(float(v @ v))
        cx.append(u[0])
        cx2.append(u[0] ** 2)
        n += 1
    assert n > 5000
    m_ratio = ME / (40 * AMU)
    assert np.mean(dfrac) == pytest.approx(-2 * m_ratio, rel=0.05)
    assert abs(np.mean(cx)) < 5 / math.sqrt(3 * n)
    assert np.mean(cx2) == pytest.approx(1 / 3, abs=5 * math.sqrt(4 / 45 / n))


def _ar(pressure):
    wl = workloads.rf_c2(gas_pa=pressure, n_e0=64, n_i0=64)
    return wl


def test_excitation_and_ionisation_energy_balance(oracle_mod):
    """Excitation removes 11.5 eV; ionisation removes 15.8 eV and the rest is shared
    between the primary and the secondary electron; the new ion has gas temperature."""
    o = oracle_mod.Oracle(_ar(20000.0))
    c = o.consts()
    e_in = 60.0
    v0 = math.sqrt(e_in / c.energy_c[0])
    seen = {1: 0, 2: 0, 3: 0}
    vions = []
    for pid in range(60000):
        ch, v, vs, vi = o.collide(0, pid, 11, [0.0, v0, 0.0])
        if ch == 0:
            continue
        seen[ch] += 1
        e1 = c.energy_c[0] * float(v @ v)
        if ch == 2:
            assert e1 == pytest.approx(e_in - 11.5, rel=1e-12)
        elif ch == 3:
            e2 = c.energy_c[0] * float(vs @ vs)
            assert e1 + e2 == pytest.approx(e_in - 15.8, rel=1e-12)
            vions.append(vi)
    assert seen[2] > 100 and seen[3] > 100
    vions = np.array(vions)
    # gas Maxwellian: each component normal with variance kT_g / M (normalised)
    var = vions.var(axis=0).mean()
    assert var == pytest.approx(c.vth_gas ** 2, rel=0.15)
    # channel fractions follow sigma_k / sum sigma at 60 eV
    s = oracle_mod.xsec("ar_like", 0, e_in)
    tot = sum(seen.values())
    for k in (1, 2, 3):
        frac = s[k - 1] / s.sum()
        assert seen[k] / tot == pytest.approx(frac, abs=5 * math.sqrt(frac * (1 - frac) / tot))


def test_ion_charge_exchange_takes_gas_velocity(oracle_mod):
    """Charge exchange: the ion leaves with the sampled gas-atom velocity, so after one
    such collision the ion velocities are the gas Maxwellian whatever they were before."""
    o = oracle_mod.Oracle(_ar(20000.0))
    c = o.consts()
    vfast = 50 * c.vth_gas
    outs, iso_e = [], []
    for pid in range(40000):
        ch, v, _, _ = o.collide(1, pid, 5, [vfast, 0.0, 0.0])
        if ch == 2:
            outs.append(v)
        elif ch == 1:
            iso_e.append(v)
    outs = np.array(outs)
    assert len(outs) > 2000
    assert abs(outs[:, 0].mean()) < 5 * c.vth_gas / math.sqrt(len(outs))
    assert outs.var(axis=0).mean() == pytest.approx(c.vth_gas ** 2, rel=0.1)
    # isotropic scattering conserves momentum + energy of the pair (equal masses): the
    # ion's mean velocity is half the initial one (the gas is at rest on average)
    iso_e = np.array(iso_e)
    assert iso_e[:, 0].mean() == pytest.approx(vfast / 2, rel=0.05)


def test_collision_rate_constant_sigma(oracle_mod):
    """Periodic plasma, 200 steps: with a constant cross section the expected number of
    real collisions is N_e n_g sigma <v> dt * steps (Maxwellian mean speed at 3 eV), up
    to the P0 bias and the cap at 100 eV; the oracle's count must sit within 4 sigma."""
    wl = workloads.periodic_c1()
    o = oracle_mod.Oracle(wl)
    o.load()
    o.step(200)
    n_coll = o.tallies().collisions[0][0]
    c = o.consts()
    mean_speed = math.sqrt(8 * 3.0 * QE / (math.pi * ME))
    expect = 16384 * c.p0[0] * mean_speed / math.sqrt(2 * QE * 100.0 / ME) * 200
    assert expect == pytest.approx(10199, rel=2e-3)
    assert abs(n_coll - expect) < 4 * math.sqrt(expect)
    # ions have no channel in this model
    assert o.tallies().collisions[1][0] == 0

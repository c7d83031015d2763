"""Pins of the oracle's optional parts: the unsorted array order, birth ids by parent id,
binary Coulomb collisions in a cell, electrode reflection and secondary emission, and the
series-capacitor circuit of the driven electrode."""
import math

import numpy as np
import pytest

import workloads

QE = 1.602176634e-19
ME = 9.1093837015e-31
AMU = 1.66053906660e-27
EPS0 = 8.8541878128e-12


def _state_from(o, wl):
    return {s: o.particles(s) for s in (0, 1)}


def _load_into(oracle_mod, wl, parts, step, next_id):
    o = oracle_mod.Oracle(wl, cap_e=4 * len(parts[0]["x"]) + 4096,
                          cap_i=4 * len(parts[1]["x"]) + 4096)
    for s in (0, 1):
        o.set_particles(s, parts[s])
    o.set_counters(step, *next_id)
    return o


# ------------------------------------------------------------------ array order / births
def test_unsorted_order_keeps_input_order(oracle_mod):
    """The unsorted variant (Sec. 3.2): after a step the survivors stand in their input
    order and the births follow; the particles themselves (per id) are those of the
    sorted cycle, up to the summation order of the deposit."""
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=60.0, te_ev=8.0)
    o = oracle_mod.Oracle(wl)
    o.load()
    o.step(3)
    parts = _state_from(o, wl)
    t = o.tallies()
    nid = (t.next_id[0], t.next_id[1])
    a = _load_into(oracle_mod, wl, parts, 3, nid)
    b = _load_into(oracle_mod, dict(wl, sort_mode="none"), parts, 3, nid)
    a.step(1)
    b.step(1)
    assert a.tallies().births[0] > 0
    for s in (0, 1):
        pa, pb = a.particles(s), b.particles(s)
        assert pa["id"].size == pb["id"].size
        born = pb["id"] >= nid[s]
        surv = pb["id"][~born]
        # input order, absorbed ones dropped
        keep = np.isin(parts[s]["id"], surv)
        assert np.array_equal(parts[s]["id"][keep], surv)
        # births after the survivors, numbered in parent order
        assert not born[: surv.size].any()
        assert np.array_equal(pb["id"][born], np.arange(nid[s], nid[s] + born.sum()))
        oa, ob = np.argsort(pa["id"]), np.argsort(pb["id"])
        assert np.array_equal(pa["id"][oa], pb["id"][ob])
        for k in ("x", "vx", "vy", "vz"):
            assert np.allclose(pa[k][oa], pb[k][ob], rtol=1e-12, atol=1e-12 * wl["n_cells"])


def test_births_ranked_by_parent_id(oracle_mod):
    """Under the fine sort's rank rule the i-th new id goes to the child of the parent with
    the i-th smallest id.  A child sits exactly at its parent's post-push position, which
    identifies the parent among the survivors."""
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=60.0, te_ev=6.0)
    o = oracle_mod.Oracle(dict(wl, sort_mode="fine"))
    o.load()
    t0 = o.tallies()
    o.step(1)
    p = o.particles(0)
    born = p["id"] >= t0.next_id[0]
    assert born.sum() > 20
    pos = dict(zip(p["x"][~born], p["id"][~born]))
    parents = np.array([pos[x] for x in p["x"][born]])
    child = p["id"][born]
    assert np.array_equal(parents[np.argsort(child)], np.sort(parents))
    # the ions born with them carry the same ranks (same positions, same order)
    q = o.particles(1)
    bi = q["id"] >= t0.next_id[1]
    xi = q["x"][bi][np.argsort(q["id"][bi])]
    xe = p["x"][born][np.argsort(child)]
    assert np.array_equal(xi, xe)


# ------------------------------------------------------------------ Coulomb collisions
def _coulomb_oracle(oracle_mod, mass_i_amu=40.0, n0=1e16, dt=5e-6, clog=10.0):
    wl = workloads.periodic_c1(mass_i_amu=mass_i_amu, n0_m3=n0, dt_s=dt, length_m=128.0,
                               coulomb_log=clog, xsec="none", gas_pa=0.0,
                               n_e0=64, n_i0=64)
    return oracle_mod.Oracle(wl), wl


@pytest.mark.parametrize("pair", [(0, 0), (1, 1), (0, 1)])
def test_coulomb_pair_conserves_momentum_and_energy(oracle_mod, pair):
    """Every pair collision keeps the pair's momentum and kinetic energy (to rounding),
    turns the relative velocity without changing its length, and actually turns it."""
    o, wl = _coulomb_oracle(oracle_mod, mass_i_amu=0.05)
    c = o.consts()
    sa, sb = pair
    rng = np.random.default_rng(1)
    n = 4000
    va = rng.normal(0, 3.0 if sa == 0 else 0.7, size=(n, 3))
    vb = rng.normal(0, 3.0 if sb == 0 else 0.7, size=(n, 3))
    va0, vb0 = va.copy(), vb.copy()
    o.coulomb_pairs(sa, sb, np.arange(n), 17, 1e17, va, vb)
    ma, mb = c.mass[sa], c.mass[sb]
    p0 = ma * va0 + mb * vb0
    p1 = ma * va + mb * vb
    e0 = ma * (va0 ** 2).sum(1) + mb * (vb0 ** 2).sum(1)
    e1 = ma * (va ** 2).sum(1) + mb * (vb ** 2).sum(1)
    assert np.max(np.abs(p1 - p0) / np.abs(p0).max(axis=1, keepdims=True)) < 1e-12
    assert np.max(np.abs(e1 - e0) / e0) < 1e-12
    u0 = np.linalg.norm(va0 - vb0, axis=1)
    u1 = np.linalg.norm(va - vb, axis=1)
    assert np.max(np.abs(u1 - u0) / u0) < 1e-12
    assert np.median(np.abs(va - va0)) > 0


def test_coulomb_electron_ion_energy_exchange(oracle_mod):
    """Electrons at 10 eV and light (0.003 amu) ions at 1 eV, paired at random.
    (1) Physics: in the small-angle limit the scheme's mean energy change of an electron,
    2 K m_e f (f u^2 - v_e.u) / u^3 per unit time (K = e^4 n lnL / (8 pi eps0^2 m_ab^2),
    f = m_ab / m_e, from |u'| = |u| and <1 - cos Theta> = 2 <delta^2>), averaged over the
    two Maxwellians, is Spitzer's exchange rate
    dT_e/dt = -nu (T_e - T_i), nu = n e^4 lnL sqrt(m_e m_i) /
    (3 sqrt(2) pi^{3/2} eps0^2 (m_i T_e + m_e T_i)^{3/2}), within 2 %.
    (2) The oracle: one step of the same pairs changes the electrons' mean energy by the
    scheme's exact expectation, with <1 - cos Theta> = <2 delta^2 / (1 + delta^2)> over
    delta ~ N(0, var(u)) by Gauss-Hermite quadrature, within 4 standard errors."""
    m_i_amu, n0, lnl, dt = 0.003, 1e16, 10.0, 4e-7
    o, wl = _coulomb_oracle(oracle_mod, mass_i_amu=m_i_amu, n0=n0, dt=dt, clog=lnl)
    c = o.consts()
    me, mi = ME, m_i_amu * AMU
    vunit = c.vunit
    te, ti = 10.0, 1.0
    n = 1_000_000
    rng = np.random.default_rng(5)
    ve = rng.normal(0, math.sqrt(te * QE / me), size=(n, 3))  # m/s
    vi = rng.normal(0, math.sqrt(ti * QE / mi), size=(n, 3))
    u = ve - vi
    un = np.linalg.norm(u, axis=1)
    mab = me * mi / (me + mi)
    f = mab / me
    kk = QE ** 4 * n0 * lnl / (8 * math.pi * EPS0 ** 2 * mab ** 2)
    lever = me * f * (f * un ** 2 - (ve * u).sum(1))  # J per unit of <1 - cos Theta>
    # (1) small-angle limit against Spitzer
    de_small = (2 * kk * lever / un ** 3).mean()  # J / s per electron
    nu = (n0 * QE ** 4 * lnl * math.sqrt(me * mi) /
          (3 * math.sqrt(2) * math.pi ** 1.5 * EPS0 ** 2 * (mi * te * QE + me * ti * QE) ** 1.5))
    assert (2.0 / 3.0) * de_small / QE == pytest.approx(-nu * (te - ti), rel=0.02)
    # (2) one step of the oracle against the scheme's expectation
    var = kk * dt / un ** 3
    z, w = np.polynomial.hermite_e.hermegauss(60)
    w = w / w.sum()
    d2 = var[:, None] * z[None, :] ** 2
    omc = (2 * d2 / (1 + d2)) @ w
    expect = (lever * omc).mean()
    va = np.ascontiguousarray(ve / vunit)
    vb = np.ascontiguousarray(vi / vunit)
    o.coulomb_pairs(0, 1, np.arange(n), 3, n0, va, vb)
    de = 0.5 * me * vunit ** 2 * ((va ** 2).sum(1) - ((ve / vunit) ** 2).sum(1))
    assert abs(de.mean() - expect) < 4 * de.std() / math.sqrt(n)
    assert expect < -5 * de.std() / math.sqrt(n)  # the electrons cool measurably


def test_coulomb_in_the_cycle_pairs_within_cells(oracle_mod):
    """With Coulomb collisions on and no field (each ion starts on an electron and there
    is no drive, so E = 0 and the push only streams), one step changes velocities by the
    collisions alone: in every cell (after the push) each species keeps its momentum and
    kinetic energy, and of n like particles exactly 2 floor(n / 2) are changed."""
    n = 3000
    wl = workloads.periodic_c1(xsec="none", gas_pa=0.0, coulomb=3, n0_m3=1e16, dt_s=2e-9,
                               n_e0=n, n_i0=n)
    o = oracle_mod.Oracle(wl)
    rng = np.random.default_rng(9)
    x = np.sort(rng.uniform(0, 128, n))
    v = {0: rng.normal(0, 2, size=(3, n)), 1: rng.normal(0, 0.01, size=(3, n))}
    for s in (0, 1):
        o.set_particles(s, dict(x=x, vx=v[s][0], vy=v[s][1], vz=v[s][2],
                                id=np.arange(n, dtype=np.uint32)))
    o.set_counters(0, n, n)
    o.step(1)
    assert np.abs(o.grid("E")).max() == 0.0
    odd = 0
    for s in (0, 1):
        p = o.particles(s)
        order = np.argsort(p["id"])
        xn = p["x"][order]
        assert np.allclose(xn, np.mod(x + v[s][0], 128), rtol=0, atol=1e-12)
        cells = np.floor(xn).astype(int)
        vn = np.stack([p["vx"][order], p["vy"][order], p["vz"][order]])
        moved = np.any(vn != v[s], axis=0)
        for cc in np.unique(cells):
            sel = cells == cc
            assert np.allclose(vn[:, sel].sum(1), v[s][:, sel].sum(1), rtol=0, atol=1e-12)
            e0 = (v[s][:, sel] ** 2).sum()
            assert (vn[:, sel] ** 2).sum() == pytest.approx(e0, rel=1e-12)
            assert moved[sel].sum() == 2 * (sel.sum() // 2)
            odd += sel.sum() % 2
    assert odd > 0


# ------------------------------------------------------------------ electrode processes
def _field_free_box(n=400, **kw):
    """A bounded box with electrons and ions at the same positions and no drive (E = 0):
    the push is free streaming."""
    return workloads.rf_c2(n_e0=n, n_i0=n, v0_volt=0.0, xsec="none", gas_pa=0.0, **kw)


def test_secondary_emission_distribution(oracle_mod):
    """An absorbed ion emits with probability gamma; the electron's normal velocity is
    Rayleigh-distributed with scale sigma = sqrt(e T_see / m_e) dt / dx (the flux of a
    Maxwellian through the wall: mean sigma sqrt(pi / 2), mean square 2 sigma^2) and
    points into the box; the tangential components are normal with variance sigma^2; the
    electron starts a uniform fraction of its first step's flight from the wall."""
    wl = _field_free_box(see_gamma=0.3, see_te_ev=3.0)
    o = oracle_mod.Oracle(wl)
    dx = wl["length_m"] / wl["n_cells"]
    sig = math.sqrt(3.0 * QE / ME) * wl["dt_s"] / dx
    n_try = 40_000
    out = {0: [], 1: []}
    for wall in (0, 1):
        for pid in range(n_try):
            ok, x, v = o.emit(pid, 11, wall)
            if ok:
                out[wall].append((x, *v))
    nc = wl["n_cells"]
    for wall in (0, 1):
        a = np.array(out[wall])
        m = len(a)
        assert abs(m - 0.3 * n_try) < 4 * math.sqrt(n_try * 0.21)
        vn = a[:, 1] if wall == 0 else -a[:, 1]
        assert (vn > 0).all()
        assert vn.mean() == pytest.approx(sig * math.sqrt(math.pi / 2), rel=4 * 0.523 / math.sqrt(m))
        assert (vn ** 2).mean() == pytest.approx(2 * sig ** 2, rel=4 / math.sqrt(m))
        for k in (2, 3):
            assert abs(a[:, k].mean()) < 4 * sig / math.sqrt(m)
            assert a[:, k].var() == pytest.approx(sig ** 2, rel=4 * math.sqrt(2 / m))
        frac = a[:, 0] / vn if wall == 0 else (nc - a[:, 0]) / vn
        assert (frac >= 0).all() and (frac < 1).all()
        assert frac.mean() == pytest.approx(0.5, abs=4 * math.sqrt(1 / 12 / m))


@pytest.mark.parametrize("fp32", [False, True])
def test_electron_reflection_mirrors_at_the_wall(oracle_mod, fp32):
    """With reflection probability 1 every electron that crosses a wall in a field-free
    box comes back mirrored: x -> -x or 2N - x, v_x -> -v_x (FP32 layout: cell -c - 1 or
    2N - c - 1, offset 1 - f); none is absorbed.  Ions are absorbed as before."""
    wl = _field_free_box(refl_e=1.0)
    n = wl["n_cells"]
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.uniform(0, 3, 200), rng.uniform(n - 3, n, 200)])
    if fp32:
        c = np.floor(x)
        x = c + (x - c).astype(np.float32).astype(np.float64)
    o = oracle_mod.Oracle(wl, fp32_offset=fp32)
    v = rng.normal(0, 2.0, size=(3, 400))
    if fp32:
        v = v.astype(np.float32).astype(np.float64)
    for s in (0, 1):
        o.set_particles(s, dict(x=x, vx=v[0], vy=v[1], vz=v[2], id=np.arange(400, dtype=np.uint32)))
    o.set_counters(0, 400, 400)
    o.step(1)
    t = o.tallies()
    if not fp32:
        xn = x + v[0]
    else:
        cc = np.floor(x)
        f = (x - cc).astype(np.float32)
        fn = (f + v[0].astype(np.float32)).astype(np.float32)
        k = np.floor(fn)
        xn = cc + k + (fn - k).astype(np.float64)
    left, right = xn < 0, xn >= n
    assert t.reflected[0] == left.sum() > 10 and t.reflected[1] == right.sum() > 10
    assert t.absorbed[0][0] == t.absorbed[0][1] == 0
    p = o.particles(0)
    order = np.argsort(p["id"])
    want = np.where(left, -xn, np.where(right, 2 * n - xn, xn))
    assert np.allclose(p["x"][order], want, rtol=0, atol=2e-6 if fp32 else 1e-12)
    assert np.array_equal(p["vx"][order], np.where(left | right, -v[0], v[0]))
    assert (t.absorbed[1][0], t.absorbed[1][1]) == (left.sum(), right.sum())


def test_emission_and_reflection_count_balance(oracle_mod):
    """In a driven discharge with emission and partial reflection: every step the electron
    count changes by births (ionisations and emissions) minus absorptions, the emissions
    never exceed the ions absorbed, and reflected electrons are not absorbed."""
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=40.0, see_gamma=0.5, refl_e=0.2,
                         ti_ev=20.0)
    o = oracle_mod.Oracle(wl)
    o.load()
    tp, n_prev = o.tallies(), [o.count(0), o.count(1)]
    tot_em = 0
    for _ in range(40):
        o.step(1)
        t = o.tallies()
        for s in (0, 1):
            ab = sum(t.absorbed[s][w] - tp.absorbed[s][w] for w in (0, 1))
            assert o.count(s) == n_prev[s] - ab + (t.births[s] - tp.births[s])
        em = sum(t.emitted[w] - tp.emitted[w] for w in (0, 1))
        ion_abs = sum(t.absorbed[1][w] - tp.absorbed[1][w] for w in (0, 1))
        assert em <= ion_abs
        assert t.births[0] - tp.births[0] == t.births[1] - tp.births[1] + em
        tot_em += em
        n_prev, tp = [o.count(0), o.count(1)], t
    assert tot_em > 0 and sum(t.reflected) > 0


# ------------------------------------------------------------------ circuit
def test_circuit_vacuum_capacitive_divider(oracle_mod):
    """No charge in the gap: the series capacitor C and the gap (capacitance eps0 A / L,
    i.e. 1/N in units of eps0 A / dx) divide the source, Phi_0 = V_s N C / (N C + 1),
    and the potential falls linearly to the grounded electrode."""
    cap = 2e-9  # F / m^2
    wl = workloads.rf_c2(n_e0=1000, n_i0=1000, circuit_cap_f_m2=cap)
    o = oracle_mod.Oracle(wl)
    c = o.consts()
    n = wl["n_cells"]
    cn = cap * c.dx / EPS0
    for vs in (1.0, -37.5, c.vhat_amp):
        phi0, phi, ef = o.circuit_solve(np.zeros(n + 1), vs, 0.0)
        assert phi0 == pytest.approx(vs * n * cn / (n * cn + 1), rel=1e-12)
        assert np.allclose(phi, phi0 * (1 - np.arange(n + 1) / n), rtol=0, atol=1e-12 * abs(vs))
        assert np.allclose(ef, phi0 / n, rtol=1e-12)
    # a charged plate shifts the electrode: q adds q / C / (1 + 1 / (N C))
    phi0, _, _ = o.circuit_solve(np.zeros(n + 1), 0.0, 3.0)
    assert phi0 == pytest.approx(3.0 / cn / (1 + 1 / (n * cn)), rel=1e-12)


def test_circuit_large_capacitor_is_the_voltage_source(oracle_mod):
    """A very large series capacitor holds no voltage: the discharge runs as with the ideal
    source (potentials within 1e-8 relative over 30 steps, identical particle order)."""
    base = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=30.0)
    a = oracle_mod.Oracle(base)
    b = oracle_mod.Oracle(dict(base, circuit_cap_f_m2=1e6))
    a.load()
    b.load()
    for _ in range(30):
        a.step(1)
        b.step(1)
    pa, pb = a.grid("phi"), b.grid("phi")
    assert np.max(np.abs(pa - pb)) <= 1e-8 * np.abs(pa).max()
    assert np.array_equal(a.particles(0)["id"], b.particles(0)["id"])


def test_circuit_conductor_charge_follows_the_wall_currents(oracle_mod):
    """The driven electrode's conductor gains the charge of the ions it absorbs and the
    electrons it emits and loses that of the electrons it absorbs; the plate charge
    q - sigma_0 equals C (Phi_0 - V_s) (the capacitor law), and a finite capacitor makes
    the electrode potential differ from the source."""
    wl = workloads.rf_c2(n_e0=20000, n_i0=20000, gas_pa=30.0, circuit_cap_f_m2=5e-8,
                         see_gamma=0.2, ti_ev=20.0)
    o = oracle_mod.Oracle(wl)
    o.load()
    c = o.consts()
    q0 = o.tallies().q_circuit
    cn = 5e-8 * c.dx / EPS0
    for step in range(60):
        o.step(1)
        t = o.tallies()
        vs = c.vhat_amp * math.sin(c.drive_phase_per_step * step)
        sigma0 = o.grid("E")[0]
        assert (t.q_circuit - sigma0) == pytest.approx(cn * (t.phi0 - vs), rel=1e-9, abs=1e-9)
    t = o.tallies()
    cond = t.absorbed[1][0] - t.absorbed[0][0] + t.emitted[0]
    # the conductor charge used by the last solve excludes the last step's currents
    o.step(1)
    t2 = o.tallies()
    assert t2.q_circuit - q0 == pytest.approx(cond, abs=1e-9)
    assert abs(t.phi0 - vs) > 1e-3 * abs(c.vhat_amp)


# ------------------------------------------------------------------ lagged sort order
def test_lagged_sort_orders_by_start_of_step_cell(oracle_mod):
    """The lagged counting sort (Sec. 3.7 with the sort key taken before the push): after a
    step without collisions, the survivors are the input particles minus the absorbed ones,
    ordered stably by the cell each occupied at the start of the step (np.argsort with a
    stable kind on the input's cells), and their states equal those of the same step in
    the canonical mode (the order does not enter the push)."""
    wl = workloads.rf_c2(n_e0=3000, n_i0=3000, xsec="none", gas_pa=0.0, v0_volt=100.0)
    rng = np.random.default_rng(21)
    n = 3000
    xs = {s: rng.uniform(0, wl["n_cells"], n) for s in (0, 1)}
    vs = {s: rng.normal(0, 3.0 if s == 0 else 0.2, size=(3, n)) for s in (0, 1)}
    states = {}
    for mode in ("counting", "lag"):
        o = oracle_mod.Oracle(dict(wl, sort_mode=mode))
        for s in (0, 1):
            o.set_particles(s, dict(x=xs[s], vx=vs[s][0], vy=vs[s][1], vz=vs[s][2],
                                    id=np.arange(n, dtype=np.uint32)))
        o.set_counters(0, n, n)
        o.step(1)
        states[mode] = [o.particles(s) for s in (0, 1)]
    for s in (0, 1):
        lag, can = states["lag"][s], states["counting"][s]
        start = np.floor(xs[s]).astype(np.int64)
        surv = np.isin(np.arange(n), lag["id"])
        assert surv.sum() < n  # some were absorbed
        expect = np.arange(n)[surv][np.argsort(start[surv], kind="stable")]
        assert np.array_equal(lag["id"], expect.astype(np.uint32)), s
        order = np.argsort(can["id"])
        assert np.array_equal(np.sort(lag["id"]), can["id"][order])
        back = np.argsort(lag["id"])
        for k in ("x", "vx", "vy", "vz"):
            assert np.allclose(lag[k][back], can[k][order], rtol=0, atol=1e-12), (s, k)

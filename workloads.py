"""Seeded synthetic workloads for the 1D3V PIC-MCC hot path.

Parameters only: this module holds no part of the method's arithmetic.  It is the one
place both the oracle harness and the HIP path take their inputs from.  Every random
quantity of a run (initial positions and velocities, collision draws) is drawn inside
each implementation from the Philox4x32-10 stream keyed by ``seed``; the only random
numbers drawn here are the parameter table of the batched scan (numpy PCG64, seed 0).

Physical readings (the paper gives only the shape of its workloads, not these values):

* periodic plasma: cell size half a Debye length and time step 0.2/omega_pe at
  n0 = 1e15 m^-3, Te = 3 eV (Sec. 2 resolution conditions);
* bounded RF discharges: dt = 1/(400 * 13.56 MHz), n0 = 3.7e14 m^-3 (omega_pe dt = 0.2),
  Te0 = 2 eV, ions and gas at 300 K, cell size 2.5 cm / 512 for every bounded case,
  so the gap is n_cells * dx;
* ion mass 40 amu everywhere.
"""
import math

import numpy as np

# CODATA 2018 values used only to place the grid and time step of the workloads.
_E = 1.602176634e-19
_ME = 9.1093837015e-31
_EPS0 = 8.8541878128e-12
_KB = 1.380649e-23

DX_BOUNDED = 0.025 / 512
DT_RF = 1.0 / (400 * 13.56e6)
T_GAS_EV = _KB * 300.0 / _E


def _periodic_grid(n0, te_ev, n_cells):
    lam_d = math.sqrt(_EPS0 * te_ev / (n0 * _E))
    w_pe = math.sqrt(n0 * _E * _E / (_EPS0 * _ME))
    return n_cells * 0.5 * lam_d, 0.2 / w_pe


def base(**kw):
    d = dict(
        periodic=0, n_cells=512, n_e0=1000, n_i0=1000, length_m=512 * DX_BOUNDED,
        dt_s=DT_RF, n0_m3=3.7e14, te_ev=2.0, ti_ev=T_GAS_EV, mass_i_amu=40.0,
        v0_volt=0.0, freq_hz=13.56e6, gas_pa=0.0, gas_k=300.0, xsec="none",
        sigma_const_m2=0.0, eps_cap_ev=100.0, seed=0, discharge=0, load="random",
        langmuir_amp_cells=0.0, langmuir_mode=1, eedf_bins=120, eedf_max_ev=60.0,
        diag_every=10, avg_start=0, steps=10,
        # array order kept by the step: "counting" (stable counting sort by cell),
        # "fine" (the paper's fixed-capacity sorting cells), "none" (unsorted)
        sort_mode="counting", grid_points_per_sort_cell=3, sort_cell_capacity=0,
        # binary Coulomb collisions in a cell: bit 0 e-e, bit 1 i-i, bit 2 e-i
        coulomb=0, coulomb_log=10.0,
        # electrode processes and the series capacitor of the driven electrode
        see_gamma=0.0, see_te_ev=2.0, refl_e=0.0, circuit_cap_f_m2=0.0,
    )
    d.update(kw)
    return d


def periodic_c1(**kw):
    """Periodic electron-ion plasma: 128 cells, 16384 + 16384, constant-sigma e-elastic MCC."""
    length, dt = _periodic_grid(1e15, 3.0, 128)
    d = base(periodic=1, n_cells=128, n_e0=16384, n_i0=16384, length_m=length, dt_s=dt,
             n0_m3=1e15, te_ev=3.0, ti_ev=0.03, gas_pa=1.0, xsec="const_e_elastic",
             sigma_const_m2=1e-19, eps_cap_ev=100.0, steps=200, avg_start=100)
    d.update(kw)
    return d


def langmuir_c1(**kw):
    """Cold quiet-start variant of the periodic plasma: mode 1, 0.01-cell displacement."""
    d = periodic_c1(load="quiet_langmuir", te_ev=0.0, ti_ev=0.0, xsec="none", gas_pa=0.0,
                    langmuir_amp_cells=0.01, langmuir_mode=1, steps=400)
    d.update(kw)
    return d


def bounded(n_cells, n_per_species, volt, pressure_pa, **kw):
    d = base(n_cells=n_cells, n_e0=n_per_species, n_i0=n_per_species,
             length_m=n_cells * DX_BOUNDED, v0_volt=volt, gas_pa=pressure_pa, xsec="ar_like")
    d.update(kw)
    return d


def rf_c2(**kw):
    """Bounded capacitive RF discharge: 2.5 cm, 512 cells, 2e5 + 2e5, 200 V, 10 Pa, 5 RF cycles."""
    d = bounded(512, 200_000, 200.0, 10.0, steps=2000, avg_start=1600)
    d.update(kw)
    return d


def large_c3(**kw):
    """Large single discharge: 4096 cells (20 cm), 1e7 + 1e7, Te 2 eV, 300 V, 5 Pa."""
    d = bounded(4096, 10_000_000, 300.0, 5.0, steps=2000, avg_start=1000)
    d.update(kw)
    return d


def long_c5(**kw):
    """Long-run precision study: 8192 cells (40 cm), 3.2e7 + 3.2e7, 300 V, 20 Pa, 20000 steps."""
    d = bounded(8192, 32_000_000, 300.0, 20.0, steps=20000, avg_start=10000)
    d.update(kw)
    return d


def batched_c4(n_discharges=256, scale=1.0, **kw):
    """Batched scan: independent RF discharges with a seeded parameter table.

    N_grid ~ U{256..2048}, particles per species log-U[5e4, 2e6], V ~ U[50, 500] V,
    p log-U[1, 100] Pa; ``scale`` shrinks particle counts for small test runs.
    """
    rng = np.random.default_rng(0)
    n_grid = rng.integers(256, 2049, size=256)
    n_s = np.exp(rng.uniform(math.log(5e4), math.log(2e6), size=256))
    volt = rng.uniform(50.0, 500.0, size=256)
    press = np.exp(rng.uniform(math.log(1.0), math.log(100.0), size=256))
    out = []
    for k in range(n_discharges):
        n = max(64, int(round(n_s[k] * scale)))
        d = bounded(int(n_grid[k]), n, float(volt[k]), float(press[k]), discharge=k,
                    steps=2000, avg_start=400)
        d.update(kw)
        out.append(d)
    return out


def synthetic_state(n_cells, n_per_species, precision, seed, vth=(2.0, 0.02), tail=(0, 0),
                    fast=(0, 0), fast_speed=(40.0, 90.0), step=5, cells=None):
    """A seeded particle state in the library's layout, to hand to both the HIP path and
    the oracle.  Per species: uniform positions laid out cell by cell (so the first
    n - tail particles are in cell order by construction), then `tail` particles in random
    cells (an unsorted births tail); Gaussian velocities of spread vth (cells per step);
    `fast` electrons moved to |v_x| in fast_speed; ids a random permutation.  `cells` (an
    ascending list) restricts the sorted part to those cells, leaving the others empty.
    Returns {0: arrays, 1: arrays, "step", "next_id"}; arrays hold x (float64) or
    cell/off (int32/float32) and vx, vy, vz, id, n, n_sorted."""
    rng = np.random.default_rng(seed)
    fp32 = precision == "fp32_offset"
    out = {"step": step, "next_id": [int(n) for n in n_per_species]}
    for s, n in enumerate(n_per_species):
        n = int(n)
        nt = int(tail[s])
        occ = np.arange(n_cells) if cells is None else np.asarray(cells, dtype=np.int64)
        counts = rng.multinomial(n - nt, np.full(occ.size, 1.0 / occ.size))
        cell = np.concatenate([np.repeat(occ, counts),
                               rng.integers(0, n_cells, nt)]).astype(np.int32)
        if fp32:
            off = rng.random(n, dtype=np.float32)
        else:
            off = rng.random(n)
        v = rng.normal(0.0, vth[s], size=(3, n))
        if fast[s]:
            idx = rng.choice(n - nt, int(fast[s]), replace=False)
            v[0, idx] = rng.uniform(*fast_speed, size=idx.size) * rng.choice([-1.0, 1.0], idx.size)
        a = {"id": rng.permutation(n).astype(np.uint32), "n": n, "n_sorted": n - nt}
        if fp32:
            a["cell"] = cell
            a["off"] = off
            a["vxf"], a["vyf"], a["vzf"] = (v[k].astype(np.float32) for k in range(3))
        else:
            x = cell + off
            top = np.nextafter(cell + 1.0, 0.0)
            a["x"] = np.minimum(x, top)  # keeps floor(x) == cell where cell + off rounds up
            a["vx"], a["vy"], a["vz"] = v[0], v[1], v[2]
        out[s] = a
    return out

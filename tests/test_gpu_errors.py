"""Deferred device errors, forced from the host with inputs that the kernels handle in
bounds, reported by pic_sync with their codes:
* births beyond the particle capacity: the births that do not fit are dropped;
* a non-finite velocity handed in through pic_set_state: the particle's push gives a
  non-finite position, so it gets no output slot, no count and no deposit;
* more far movers into one cell in one step than the offset scan ranks (8192): the far
  movers are dropped and the step is reported as invalid."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

PIC_ERR_CAPACITY = -2
PIC_ERR_NONFINITE = -4


@pytest.fixture(scope="module")
def fspic():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1104_3998_amd as m
    m.lib()
    return m


def test_births_beyond_capacity_are_reported(fspic):
    """A periodic box (no walls to make room) with Ar-like ionization at 10 eV, about 45
    births per step, and capacities equal to the load."""
    wl = workloads.periodic_c1(xsec="ar_like", gas_pa=10.0, te_ev=10.0, capacity_e=16384,
                               capacity_i=16384)
    print("capacity overflow", flush=True)
    sim = fspic.Simulation(wl, "fp64")
    with pytest.raises(fspic.PicError) as ei:
        sim.step(5)
        sim.sync()
    assert ei.value.code == PIC_ERR_CAPACITY
    sim.close()


def test_nonfinite_velocity_is_reported(fspic):
    """One electron of a collisionless periodic state gets a NaN velocity."""
    wl = workloads.periodic_c1(xsec="none", gas_pa=0.0)
    st = workloads.synthetic_state(wl["n_cells"], (wl["n_e0"], wl["n_i0"]), "fp64", seed=3)
    st[0]["vx"][100] = np.nan
    print("non-finite velocity", flush=True)
    sim = fspic.Simulation(wl, "fp64")
    sim.set_state(st)
    with pytest.raises(fspic.PicError) as ei:
        sim.step(1)
        sim.sync()
    assert ei.value.code == PIC_ERR_NONFINITE
    sim.close()


def test_far_group_over_limit_is_reported(fspic):
    """20000 electrons in one cell of the periodic box, every one moving 60 cells (either
    way): about 10000 far movers into each of two cells, beyond the 8192 the offset scan
    ranks per cell (the far list itself is sized for all of them)."""
    wl = workloads.periodic_c1()
    st = workloads.synthetic_state(wl["n_cells"], (20000, 20000), "fp64", seed=5, cells=[10],
                                   fast=(20000, 0), fast_speed=(60.0, 60.0))
    print("far group over the limit", flush=True)
    sim = fspic.Simulation(wl, "fp64", tuning={"far_capacity": 32768})
    sim.set_state(st)
    with pytest.raises(fspic.PicError) as ei:
        sim.step(1)
        sim.sync()
    assert ei.value.code == PIC_ERR_CAPACITY
    assert "one cell" in str(ei.value)
    sim.close()

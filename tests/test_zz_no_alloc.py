"""pic_init_static (the entry point for callers that cannot allocate device memory)
against pic_init with a caller workspace: two calls in a row on one GPU, the second with a
smaller simulation, each stepped and compared bit for bit with the same discharges run
through pic_init."""
import ctypes

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


KEYS = {True: ("cell", "off", "vxf", "vyf", "vzf", "id", "w"),
        False: ("x", "vx", "vy", "vz", "id", "w")}


def run(fspic, wl, precision, static, steps):
    sim = fspic.Simulation(wl, precision, workspace="static" if static else "torch")
    assert sim.static_workspace == static
    sim.step(steps)
    st = sim.get_state()
    g = sim.diagnostics()
    sim.close()
    return st, g


@pytest.mark.parametrize("precision", ["fp64", "fp32_offset"])
def test_static_workspace_matches_caller_workspace(fspic, precision):
    fp32 = precision == "fp32_offset"
    cases = [("bounded RF discharge 3e4 + 3e4", workloads.rf_c2(n_e0=30000, n_i0=30000,
                                                                gas_pa=30.0), 25),
             ("periodic plasma 4096 + 4096", workloads.periodic_c1(n_e0=4096, n_i0=4096), 25)]
    for label, wl, steps in cases:  # the second simulation is the smaller one
        print("static workspace", label, precision, flush=True)
        a, ga = run(fspic, wl, precision, True, steps)
        b, gb = run(fspic, wl, precision, False, steps)
        assert a["step"] == b["step"] == steps
        for s in (0, 1):
            assert a[s]["n"] == b[s]["n"] and a[s]["n_sorted"] == b[s]["n_sorted"]
            for k in KEYS[fp32]:
                assert np.array_equal(a[s][k].view(np.uint8), b[s][k].view(np.uint8)), (label, s, k)
        assert [list(r) for r in ga.collisions] == [list(r) for r in gb.collisions]
        assert list(ga.births) == list(gb.births)


def test_static_workspace_rejects_oversize(fspic):
    """A simulation larger than the static array is refused with PIC_ERR_WORKSPACE and a
    message; nothing is allocated."""
    wl = workloads.large_c3()
    with pytest.raises(fspic.PicError) as e:
        fspic.Simulation(wl, "fp32_offset", workspace="static")
    assert e.value.code == -7
    assert "static workspace" in str(e.value)

"""Host-side checks of the C ABI (no GPU work): the library loads and exports every
function include/fspic.h declares, the ctypes mirrors have the C layout, configurations
are validated, and the normalised constants the library derives (Sec. 3.3, eq.
null_collision) equal the ones the oracle derives independently."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fspic.h")


@pytest.fixture(scope="module")
def fspic():
    import paper_1104_3998_amd as m
    if not os.path.exists(m.LIB_PATH):
        import paper_1104_3998_amd.build as b
        b.build()
    m.lib()
    return m


def declared_functions():
    txt = open(HEADER).read()
    decl = r"^(?:int|void|const char\*)\s+(pic_[a-z_]+)\s*\("
    return sorted(set(re.findall(decl, txt, flags=re.M)))


def test_exports_every_declared_symbol(fspic):
    names = declared_functions()
    assert len(names) >= 15
    L = ctypes.CDLL(fspic.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(fspic.EXPORTS)


def test_struct_layouts_match_c(fspic, tmp_path):
    structs = {"pic_config": fspic.PicConfig, "pic_derived": fspic.PicDerived,
               "pic_diag": fspic.PicDiag, "pic_state": fspic.PicState}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fspic.h"', 'int main(void){']
    for cname, py in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    out = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in structs.items():
        assert int(out[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out["%s.%s" % (cname, f)]) == getattr(py, f).offset, (cname, f)


ALL_WL = [("periodic", workloads.periodic_c1()), ("langmuir", workloads.langmuir_c1()),
          ("rf", workloads.rf_c2()), ("large", workloads.large_c3()),
          ("long", workloads.long_c5())] + [
    ("batch%d" % i, w) for i, w in enumerate(workloads.batched_c4(n_discharges=3))]


@pytest.mark.parametrize("name,wl", ALL_WL, ids=[a for a, _ in ALL_WL])
def test_derived_constants_match_oracle(fspic, oracle_mod, name, wl):
    small = dict(wl, n_e0=min(wl["n_e0"], 4096), n_i0=min(wl["n_i0"], 4096))
    d = fspic.derive(fspic.make_config(small))
    c = oracle_mod.Oracle(small).consts()
    for f in ("dx", "weight_per_area", "phi_scale", "vunit", "vth_gas", "n_gas", "vhat_amp",
              "drive_phase_per_step"):
        assert getattr(d, f) == pytest.approx(getattr(c, f), rel=1e-15, abs=0), f
    for s in (0, 1):
        for f in ("kappa", "energy_c", "vth", "nu0", "p0"):
            assert getattr(d, f)[s] == pytest.approx(getattr(c, f)[s], rel=1e-15, abs=0), (f, s)
        assert d.t0[s] == c.t0[s]


def test_tile_geometry_limits(fspic):
    for wl in [w for _, w in ALL_WL] + [workloads.periodic_c1(n_cells=5, n_e0=50, n_i0=50)]:
        for prec in ("fp32_offset", "fp64"):
            d = fspic.derive(fspic.make_config(wl, prec))
            for s in (0, 1):
                C, D = d.cells_per_tile[s], d.window[s]
                assert 1 <= C <= 64 and C + 2 * D <= 256
                if wl["periodic"]:
                    assert wl["n_cells"] % C == 0
                    assert C + 2 * D + C + 1 <= wl["n_cells"]


def test_workspace_bytes_scale_and_validation(fspic):
    small = fspic.workspace_bytes([fspic.make_config(workloads.rf_c2())])
    big = fspic.workspace_bytes([fspic.make_config(workloads.large_c3())])
    assert small > 0 and big > 20 * small
    # FP32 cell + offset records are 24 B, FP64 records 36 B: the FP64 workspace is larger
    f64 = fspic.workspace_bytes([fspic.make_config(workloads.large_c3(), "fp64")])
    assert f64 > big * 1.3
    bad = [fspic.make_config(workloads.rf_c2(n_cells=0)),
           fspic.make_config(workloads.rf_c2(), cap_factor=0.5),
           fspic.make_config(workloads.periodic_c1(n_cells=2))]
    c = fspic.make_config(workloads.rf_c2())
    c.abi_version = 99
    bad.append(c)
    for cfg in bad:
        with pytest.raises(fspic.PicError) as e:
            fspic.workspace_bytes([cfg])
        assert e.value.code == -1
    mixed = [fspic.make_config(workloads.rf_c2(), "fp64"),
             fspic.make_config(workloads.rf_c2(), "fp32_offset")]
    with pytest.raises(fspic.PicError):
        fspic.workspace_bytes(mixed)


def test_simulation_requires_gpu(fspic):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        fspic.Simulation(workloads.periodic_c1())


def test_autotune_geometry_scaling():
    """The tuner's candidates are the library's rule scaled per species and clamped to
    the limits the library accepts (1..64 cells per tile, window >= 1)."""
    from paper_1104_3998_amd import autotune as at
    rule = at.rule_geometry([workloads.large_c3()], "fp32_offset")
    assert rule == [((8, 32), (1, 4))]
    assert at.scaled_tuning(rule, 1.0, 1.0, 1.0) == [{"cells_per_tile": (8, 1), "window": (32, 4)}]
    assert at.scaled_tuning(rule, 0.5, 2.0, 0.5) == [{"cells_per_tile": (4, 2), "window": (16, 4)}]
    assert at.scaled_tuning([((64, 32), (1, 4))], 2.0, 0.5, 0.01) == \
        [{"cells_per_tile": (64, 1), "window": (1, 4)}]

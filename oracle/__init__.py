"""FP64 CPU oracle of the 1D3V PIC-MCC cycle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  The product library never links or calls it; the two share no
source.  The C source (``fspic_oracle.c``) is the oracle; this module compiles it with gcc
and exposes it through ctypes.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fspic_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

XSEC = {"none": 0, "const_e_elastic": 1, "ar_like": 2}
LOAD = {"random": 0, "quiet_langmuir": 1}


def build():
    """Compile the oracle: -O2, no floating-point contraction, single-threaded."""
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                           "-Wall", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("periodic", ctypes.c_int32), ("n_cells", ctypes.c_int32),
        ("n_e0", ctypes.c_int64), ("n_i0", ctypes.c_int64),
        ("length_m", ctypes.c_double), ("dt_s", ctypes.c_double), ("n0_m3", ctypes.c_double),
        ("te_ev", ctypes.c_double), ("ti_ev", ctypes.c_double), ("mass_i_amu", ctypes.c_double),
        ("v0_volt", ctypes.c_double), ("freq_hz", ctypes.c_double), ("gas_pa", ctypes.c_double),
        ("gas_k", ctypes.c_double),
        ("xsec", ctypes.c_int32),
        ("sigma_const_m2", ctypes.c_double), ("eps_cap_ev", ctypes.c_double),
        ("seed", ctypes.c_uint32), ("discharge", ctypes.c_uint32),
        ("load", ctypes.c_int32),
        ("langmuir_amp_cells", ctypes.c_double),
        ("langmuir_mode", ctypes.c_int32), ("fp32_offset", ctypes.c_int32),
        ("eedf_bins", ctypes.c_int32),
        ("eedf_max_ev", ctypes.c_double),
        ("diag_every", ctypes.c_int32),
        ("avg_start", ctypes.c_int64),
        ("sort_mode", ctypes.c_int32), ("birth_rank", ctypes.c_int32),
        ("coulomb", ctypes.c_int32), ("coulomb_log", ctypes.c_double),
        ("see_gamma", ctypes.c_double), ("see_te_ev", ctypes.c_double),
        ("refl_e", ctypes.c_double), ("circuit_cap_f_m2", ctypes.c_double),
    ]


class OrcConsts(ctypes.Structure):
    _fields_ = [
        ("dx", ctypes.c_double), ("weight_per_area", ctypes.c_double),
        ("kappa", ctypes.c_double * 2), ("phi_scale", ctypes.c_double),
        ("vunit", ctypes.c_double), ("energy_c", ctypes.c_double * 2),
        ("vth", ctypes.c_double * 2), ("vth_gas", ctypes.c_double), ("n_gas", ctypes.c_double),
        ("nu0", ctypes.c_double * 2), ("p0", ctypes.c_double * 2), ("vhat_amp", ctypes.c_double),
        ("drive_phase_per_step", ctypes.c_double), ("mass", ctypes.c_double * 2),
        ("t0", ctypes.c_uint32 * 2),
    ]


class OrcTallies(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("next_id", ctypes.c_uint32 * 2),
        ("absorbed", (ctypes.c_int64 * 2) * 2),
        ("absorbed_energy_ev", (ctypes.c_double * 2) * 2),
        ("births", ctypes.c_int64 * 2),
        ("collisions", (ctypes.c_int64 * 3) * 2),
        ("acc_count", ctypes.c_int64), ("eedf_samples", ctypes.c_int64),
        ("emitted", ctypes.c_int64 * 2), ("reflected", ctypes.c_int64 * 2),
        ("kinetic", ctypes.c_double * 2), ("field_energy", ctypes.c_double),
        ("momentum", ctypes.c_double), ("sum_rho", ctypes.c_double),
        ("phi0", ctypes.c_double), ("q_circuit", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        P, D, I64, I32, U32 = (ctypes.c_void_p, ctypes.c_double, ctypes.c_int64,
                               ctypes.c_int, ctypes.c_uint32)
        L.orc_create.restype = P
        L.orc_create.argtypes = [ctypes.POINTER(OrcParams), I64, I64]
        L.orc_destroy.argtypes = [P]
        L.orc_get_consts.argtypes = [P, ctypes.POINTER(OrcConsts)]
        L.orc_load.argtypes = [P]
        L.orc_step.argtypes = [P]
        L.orc_count.restype = I64
        L.orc_count.argtypes = [P, I32]
        L.orc_get_particles.argtypes = [P, I32, P, P, P, P, P]
        L.orc_set_particles.argtypes = [P, I32, I64, P, P, P, P, P]
        L.orc_get_grid.argtypes = [P, I32, P]
        L.orc_set_grid.argtypes = [P, I32, P]
        L.orc_get_tallies.argtypes = [P, ctypes.POINTER(OrcTallies)]
        L.orc_set_counters.argtypes = [P, I64, U32, U32]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_u53.restype = D
        L.orc_u53.argtypes = [U32, U32]
        L.orc_xsec.argtypes = [I32, I32, D, D, P]
        L.orc_solve.argtypes = [I32, I32, P, D, P, P]
        L.orc_deposit.argtypes = [I32, I32, I64, P, P]
        L.orc_stable_sort_by_cell.argtypes = [I64, P, I32, P]
        L.orc_push.argtypes = [I32, I32, I32, D, P, I64, P, P, P]
        L.orc_collide.argtypes = [P, I32, U32, I64, P, P, P]
        L.orc_coulomb_pair.argtypes = [P, I32, I32, U32, I64, D, P, P]
        L.orc_coulomb_pairs.argtypes = [P, I32, I32, I64, P, I64, D, P, P]
        L.orc_emit.argtypes = [P, U32, I64, I32, P, P]
        L.orc_circuit_solve.restype = D
        L.orc_circuit_solve.argtypes = [P, P, D, D, P, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


SORT_MODES = ("counting", "fine", "none", "lag")


def params_from(wl, fp32_offset=False):
    """Oracle parameters of a workload.  The array order the oracle keeps follows the
    workload's sort mode: sorted by cell for the counting and the fine (paper) sort, input
    order for the unsorted variant, by the start-of-step cell for the lagged counting sort;
    under the fine sort, whose order inside a sorting cell is not fixed, births take ids in
    increasing parent id."""
    p = OrcParams()
    mode = wl.get("sort_mode", "counting")
    assert mode in SORT_MODES, mode
    for name, _ in OrcParams._fields_:
        if name == "xsec":
            p.xsec = XSEC[wl["xsec"]]
        elif name == "load":
            p.load = LOAD[wl["load"]]
        elif name == "fp32_offset":
            p.fp32_offset = 1 if fp32_offset else 0
        elif name == "sort_mode":
            p.sort_mode = {"none": 1, "lag": 2}.get(mode, 0)
        elif name == "birth_rank":
            p.birth_rank = 1 if mode == "fine" else 0
        else:
            setattr(p, name, type(getattr(p, name))(wl[name]))
    return p


# ---------------------------------------------------------------- unit-level helpers
def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def u53(a, b):
    return lib().orc_u53(int(a), int(b))


def xsec(model, species, eps, sigma_const=0.0):
    out = np.zeros(3)
    lib().orc_xsec(XSEC[model], species, float(eps), float(sigma_const), _ptr(out))
    return out


def solve(periodic, n_cells, rho, phi_left=0.0):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    nn = n_cells if periodic else n_cells + 1
    assert rho.shape == (nn,)
    phi = np.zeros(nn)
    ef = np.zeros(nn)
    rc = lib().orc_solve(int(periodic), n_cells, _ptr(rho), float(phi_left), _ptr(phi), _ptr(ef))
    if rc != 0:
        raise ValueError("orc_solve failed: %d" % rc)
    return phi, ef


def deposit(periodic, n_cells, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.zeros(n_cells if periodic else n_cells + 1)
    lib().orc_deposit(int(periodic), n_cells, x.size, _ptr(x), _ptr(w))
    return w


def stable_sort_by_cell(cells, n_cells):
    c = np.ascontiguousarray(cells, dtype=np.int32)
    perm = np.zeros(c.size, dtype=np.int64)
    lib().orc_stable_sort_by_cell(c.size, _ptr(c), int(n_cells), _ptr(perm))
    return perm


def push(periodic, n_cells, kappa, efield, x, vx, fp32_offset=False):
    ef = np.ascontiguousarray(efield, dtype=np.float64)
    x = np.array(x, dtype=np.float64)
    vx = np.array(vx, dtype=np.float64)
    flags = np.zeros(x.size, dtype=np.int32)
    lib().orc_push(int(periodic), n_cells, int(fp32_offset), float(kappa), _ptr(ef), x.size,
                   _ptr(x), _ptr(vx), _ptr(flags))
    return x, vx, flags


# ---------------------------------------------------------------- whole cycle
class Oracle:
    """One discharge of the reference cycle (batched runs are independent loops)."""

    def __init__(self, wl, fp32_offset=False, cap_e=None, cap_i=None):
        self.wl = dict(wl)
        self.fp32_offset = fp32_offset
        self.params = params_from(wl, fp32_offset)
        cap_e = cap_e if cap_e is not None else int(wl["n_e0"] * 1.5) + 1024
        cap_i = cap_i if cap_i is not None else int(wl["n_i0"] * 1.5) + 1024
        self._h = lib().orc_create(ctypes.byref(self.params), cap_e, cap_i)
        if not self._h:
            raise ValueError("orc_create rejected the parameters")
        self.n_cells = wl["n_cells"]
        self.n_nodes = self.n_cells if wl["periodic"] else self.n_cells + 1

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def consts(self):
        c = OrcConsts()
        lib().orc_get_consts(self._h, ctypes.byref(c))
        return c

    def load(self):
        rc = lib().orc_load(self._h)
        if rc != 0:
            raise RuntimeError("orc_load: %d" % rc)

    def step(self, n=1):
        for _ in range(n):
            rc = lib().orc_step(self._h)
            if rc != 0:
                raise RuntimeError("orc_step: %d" % rc)

    def count(self, s):
        return lib().orc_count(self._h, s)

    def particles(self, s):
        n = self.count(s)
        d = {k: np.zeros(n) for k in ("x", "vx", "vy", "vz")}
        d["id"] = np.zeros(n, dtype=np.uint32)
        lib().orc_get_particles(self._h, s, _ptr(d["x"]), _ptr(d["vx"]), _ptr(d["vy"]),
                                _ptr(d["vz"]), _ptr(d["id"]))
        return d

    def set_particles(self, s, d):
        a = {k: np.ascontiguousarray(d[k], dtype=np.float64) for k in ("x", "vx", "vy", "vz")}
        i = np.ascontiguousarray(d["id"], dtype=np.uint32)
        rc = lib().orc_set_particles(self._h, s, i.size, _ptr(a["x"]), _ptr(a["vx"]),
                                     _ptr(a["vy"]), _ptr(a["vz"]), _ptr(i))
        if rc != 0:
            raise ValueError("orc_set_particles: %d" % rc)

    def grid(self, what):
        names = {"w_e": 0, "w_i": 1, "phi": 2, "E": 3, "acc_w_e": 4, "acc_w_i": 5,
                 "acc_phi": 6, "eedf": 7}
        k = names[what]
        n = (self.wl["eedf_bins"] + 1) if k == 7 else self.n_nodes
        out = np.zeros(n)
        lib().orc_get_grid(self._h, k, _ptr(out))
        return out

    def set_grid(self, what, arr):
        k = {"w_e": 0, "w_i": 1}[what]
        a = np.ascontiguousarray(arr, dtype=np.float64)
        assert a.size == self.n_nodes
        lib().orc_set_grid(self._h, k, _ptr(a))

    def tallies(self):
        t = OrcTallies()
        lib().orc_get_tallies(self._h, ctypes.byref(t))
        return t

    def set_counters(self, step, next_id_e, next_id_i):
        lib().orc_set_counters(self._h, int(step), int(next_id_e), int(next_id_i))

    def coulomb_pair(self, sa, sb, id_a, step, n_l, va, vb):
        va = np.array(va, dtype=np.float64)
        vb = np.array(vb, dtype=np.float64)
        rc = lib().orc_coulomb_pair(self._h, sa, sb, int(id_a), int(step), float(n_l),
                                    _ptr(va), _ptr(vb))
        return rc, va, vb

    def coulomb_pairs(self, sa, sb, ids_a, step, n_l, va, vb):
        """va, vb: (n, 3) arrays, updated in place."""
        ids = np.ascontiguousarray(ids_a, dtype=np.uint32)
        assert va.flags.c_contiguous and vb.flags.c_contiguous and va.dtype == np.float64
        lib().orc_coulomb_pairs(self._h, sa, sb, ids.size, _ptr(ids), int(step), float(n_l),
                                _ptr(va), _ptr(vb))

    def emit(self, ion_id, step, wall):
        x = np.zeros(1)
        v = np.zeros(3)
        rc = lib().orc_emit(self._h, int(ion_id), int(step), int(wall), _ptr(x), _ptr(v))
        return rc, float(x[0]), v

    def circuit_solve(self, rho, vs, q):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        phi = np.zeros(self.n_nodes)
        ef = np.zeros(self.n_nodes)
        phi0 = lib().orc_circuit_solve(self._h, _ptr(rho), float(vs), float(q), _ptr(phi),
                                       _ptr(ef))
        return phi0, phi, ef

    def collide(self, species, pid, step, v):
        v = np.array(v, dtype=np.float64)
        vs = np.zeros(3)
        vi = np.zeros(3)
        ch = lib().orc_collide(self._h, species, int(pid), int(step), _ptr(v), _ptr(vs), _ptr(vi))
        return ch, v, vs, vi

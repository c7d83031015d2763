"""Python binding of libfspic (include/fspic.h): argument marshalling only.

Every step of the PIC-MCC hot path runs in the HIP kernels of ``libfspic.so``.  PyTorch
supplies the device workspace and the stream.  If the library is not built the import of
:class:`Simulation` fails loudly; there is no CPU fallback.

torch is imported before the library is loaded so that both share one HIP runtime.
"""
import ctypes
import os

import numpy as np

try:  # the HIP runtime must be torch's when torch is used for memory and streams
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is part of the environment
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfspic.so")

ABI_VERSION = 2
PIC_FP64, PIC_FP32_OFFSET = 0, 1
XSEC = {"none": 0, "const_e_elastic": 1, "ar_like": 2}
LOAD = {"random": 0, "quiet_langmuir": 1}
STATUS = {0: "PIC_OK", -1: "PIC_ERR_ARG", -2: "PIC_ERR_CAPACITY", -3: "PIC_ERR_DEVICE",
          -4: "PIC_ERR_NONFINITE", -5: "PIC_ERR_ID_OVERFLOW", -6: "PIC_ERR_STATE",
          -7: "PIC_ERR_WORKSPACE", -8: "PIC_ERR_CORRUPT"}
SORT = {"counting": 0, "none": 1, "fine": 2, "lag": 3}
PHASES = ("combine", "solve", "hist", "scan", "main", "collide", "finalize", "coulomb",
          "fine_sort")

U32, U64, I32, F64, P = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double,
                         ctypes.c_void_p)


class PicConfig(ctypes.Structure):
    _fields_ = [
        ("abi_version", U32), ("precision", U32), ("periodic", U32), ("n_cells", U32),
        ("n_e0", U64), ("n_i0", U64), ("capacity_e", U64), ("capacity_i", U64),
        ("length_m", F64), ("dt_s", F64), ("n0_m3", F64), ("te_ev", F64), ("ti_ev", F64),
        ("mass_i_amu", F64), ("v0_volt", F64), ("freq_hz", F64), ("gas_pa", F64),
        ("gas_k", F64),
        ("xsec_model", U32), ("load_kind", U32),
        ("sigma_const_m2", F64), ("eps_cap_ev", F64),
        ("seed", U32), ("discharge_index", U32),
        ("langmuir_amp_cells", F64),
        ("langmuir_mode", U32), ("eedf_bins", U32),
        ("eedf_max_ev", F64),
        ("diag_every", U32), ("reserved0", U32),
        ("avg_start_step", U64),
        ("cells_per_tile", U32 * 2), ("window", U32 * 2), ("tail_groups", U32),
        ("far_capacity", U32),
        ("sort_mode", U32), ("coulomb", U32), ("coulomb_log", F64), ("see_gamma", F64),
        ("see_te_ev", F64), ("refl_e", F64), ("circuit_cap_f_m2", F64),
        ("sort_cell_cells", U32), ("sort_cell_capacity", U32),
    ]


class PicDerived(ctypes.Structure):
    _fields_ = [
        ("dx", F64), ("weight_per_area", F64), ("kappa", F64 * 2), ("phi_scale", F64),
        ("vunit", F64), ("energy_c", F64 * 2), ("vth", F64 * 2), ("vth_gas", F64),
        ("n_gas", F64), ("nu0", F64 * 2), ("p0", F64 * 2), ("vhat_amp", F64),
        ("drive_phase_per_step", F64), ("t0", U32 * 2), ("cells_per_tile", U32 * 2),
        ("window", U32 * 2),
    ]


class PicDiag(ctypes.Structure):
    _fields_ = [
        ("step", U64), ("n_particles", U64 * 2), ("n_sorted", U64 * 2), ("next_id", U32 * 2),
        ("absorbed", (U64 * 2) * 2), ("absorbed_energy_ev", (F64 * 2) * 2),
        ("births", U64 * 2), ("collisions", (U64 * 3) * 2),
        ("acc_count", U64), ("eedf_samples", U64),
        ("surface_charge", F64 * 2), ("particle_steps", U64 * 2), ("error_flags", U32),
        ("reserved0", U32),
        ("kinetic", F64 * 2), ("momentum", F64), ("energy_step", U64),
        ("field_energy", F64), ("sum_rho", F64), ("phi_driven_v", F64),
        ("circuit_charge", F64), ("emitted", U64 * 2), ("reflected", U64 * 2),
        ("eedf", ctypes.POINTER(F64)), ("eedf_len", U32), ("reserved1", U32),
    ]


class PicState(ctypes.Structure):
    _fields_ = [
        ("capacity", U64 * 2), ("n", U64 * 2), ("n_sorted", U64 * 2),
        ("cell", P * 2), ("off", P * 2), ("vxf", P * 2), ("vyf", P * 2), ("vzf", P * 2),
        ("x", P * 2), ("vx", P * 2), ("vy", P * 2), ("vz", P * 2), ("id", P * 2),
        ("w", P * 2), ("step", U64), ("next_id", U32 * 2), ("sort_all", U32),
        ("reserved0", U32),
    ]


EXPORTS = ("pic_workspace_bytes", "pic_derive", "pic_init", "pic_init_static", "pic_step",
           "pic_set_graph",
           "pic_sync", "pic_density", "pic_grid", "pic_diagnostics", "pic_get_state",
           "pic_set_state", "pic_profile", "pic_profile_read", "pic_free", "pic_last_error")

_lib = None


class PicError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__("%s -> %s (%d): %s" % (fn, STATUS.get(code, "?"), code, msg))
        self.code = code


def lib():
    """Loads libfspic.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfspic.so is not built; run __graft_entry__.build() "
                          "(paper_1104_3998_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    cfgp = ctypes.POINTER(PicConfig)
    L.pic_workspace_bytes.argtypes = [cfgp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.pic_derive.argtypes = [cfgp, ctypes.POINTER(PicDerived)]
    L.pic_init.argtypes = [cfgp, ctypes.c_int, P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    L.pic_init_static.argtypes = [cfgp, ctypes.c_int, P, ctypes.POINTER(P)]
    L.pic_step.argtypes = [P, U32]
    L.pic_set_graph.argtypes = [P, U32]
    L.pic_sync.argtypes = [P]
    L.pic_density.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_size_t]
    L.pic_grid.argtypes = [P, ctypes.c_int, ctypes.c_int, P, ctypes.c_size_t]
    L.pic_diagnostics.argtypes = [P, ctypes.c_int, ctypes.POINTER(PicDiag)]
    L.pic_get_state.argtypes = [P, ctypes.c_int, ctypes.POINTER(PicState)]
    L.pic_set_state.argtypes = [P, ctypes.c_int, ctypes.POINTER(PicState)]
    L.pic_profile.argtypes = [P, ctypes.c_int]
    L.pic_profile_read.argtypes = [P, ctypes.POINTER(F64), ctypes.POINTER(U64), ctypes.c_int]
    L.pic_free.argtypes = [P]
    L.pic_free.restype = None
    L.pic_last_error.argtypes = [P]
    L.pic_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(fn, code, handle=None):
    if code != 0:
        msg = lib().pic_last_error(handle)
        raise PicError(fn, code, msg.decode() if msg else "")


def make_config(wl, precision="fp32_offset", cap_factor=1.5, tuning=None):
    """pic_config from a workload dict (see workloads.py)."""
    c = PicConfig()
    c.abi_version = ABI_VERSION
    c.precision = PIC_FP32_OFFSET if precision == "fp32_offset" else PIC_FP64
    c.periodic = int(wl["periodic"])
    c.n_cells = int(wl["n_cells"])
    c.n_e0, c.n_i0 = int(wl["n_e0"]), int(wl["n_i0"])
    c.capacity_e = int(wl.get("capacity_e", int(wl["n_e0"] * cap_factor) + 1024))
    c.capacity_i = int(wl.get("capacity_i", int(wl["n_i0"] * cap_factor) + 1024))
    for k in ("length_m", "dt_s", "n0_m3", "te_ev", "ti_ev", "mass_i_amu", "v0_volt",
              "freq_hz", "gas_pa", "gas_k", "sigma_const_m2", "eps_cap_ev",
              "langmuir_amp_cells", "eedf_max_ev"):
        setattr(c, k, float(wl[k]))
    c.xsec_model = XSEC[wl["xsec"]]
    c.load_kind = LOAD[wl["load"]]
    c.seed = int(wl["seed"])
    c.discharge_index = int(wl["discharge"])
    c.langmuir_mode = int(wl["langmuir_mode"])
    c.eedf_bins = int(wl["eedf_bins"])
    c.diag_every = int(wl["diag_every"])
    c.avg_start_step = int(wl["avg_start"])
    t = dict(tuning or {})
    for k in ("cells_per_tile", "window"):
        if k in t:
            v = t[k]
            v = (v, v) if isinstance(v, int) else v
            getattr(c, k)[0], getattr(c, k)[1] = int(v[0]), int(v[1])
    c.tail_groups = int(t.get("tail_groups", 0))
    c.far_capacity = int(t.get("far_capacity", 0))
    c.sort_mode = SORT[wl.get("sort_mode", "counting")]
    c.coulomb = int(wl.get("coulomb", 0))
    c.coulomb_log = float(wl.get("coulomb_log", 10.0))
    c.see_gamma = float(wl.get("see_gamma", 0.0))
    c.see_te_ev = float(wl.get("see_te_ev", 2.0))
    c.refl_e = float(wl.get("refl_e", 0.0))
    c.circuit_cap_f_m2 = float(wl.get("circuit_cap_f_m2", 0.0))
    c.sort_cell_cells = max(0, int(wl.get("grid_points_per_sort_cell", 3)) - 1)
    c.sort_cell_capacity = int(wl.get("sort_cell_capacity", 0))
    return c


def workspace_bytes(cfgs):
    arr = (PicConfig * len(cfgs))(*cfgs)
    n = ctypes.c_size_t()
    _check("pic_workspace_bytes", lib().pic_workspace_bytes(arr, len(cfgs), ctypes.byref(n)))
    return n.value


def derive(cfg):
    d = PicDerived()
    _check("pic_derive", lib().pic_derive(ctypes.byref(cfg), ctypes.byref(d)))
    return d


def _ptr(a):
    return a.ctypes.data_as(P) if a is not None else None


class Simulation:
    """Owns a torch workspace and a pic_sim handle for one or more discharges."""

    def __init__(self, workloads, precision="fp32_offset", device="cuda", cap_factor=1.5,
                 tuning=None, stream=None, workspace="torch"):
        """workspace: "torch" (a torch.uint8 tensor of pic_workspace_bytes, pic_init) or
        "static" (the library's own device array, pic_init_static: nothing allocated)."""
        if torch is None or not torch.cuda.is_available():
            raise RuntimeError("Simulation needs a ROCm GPU (torch.cuda.is_available() is False)")
        wls = workloads if isinstance(workloads, (list, tuple)) else [workloads]
        self.workloads = [dict(w) for w in wls]
        self.precision = precision
        self.fp32 = precision == "fp32_offset"
        # tuning: one dict for every discharge, or a list with one dict per discharge
        tunings = tuning if isinstance(tuning, (list, tuple)) else [tuning] * len(wls)
        if len(tunings) != len(wls):
            raise ValueError("tuning list needs one entry per discharge")
        self.cfgs = [make_config(w, precision, cap_factor, t) for w, t in zip(wls, tunings)]
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        arr = (PicConfig * len(self.cfgs))(*self.cfgs)
        h = P()
        self.static_workspace = workspace == "static"
        if self.static_workspace:
            self.bytes, self.workspace = 0, None
            with torch.cuda.device(self.device):
                _check("pic_init_static", lib().pic_init_static(
                    arr, len(self.cfgs), P(self.stream.cuda_stream), ctypes.byref(h)))
        else:
            self.bytes = workspace_bytes(self.cfgs)
            self.workspace = torch.empty(self.bytes, dtype=torch.uint8, device=self.device)
            _check("pic_init", lib().pic_init(arr, len(self.cfgs), P(self.workspace.data_ptr()),
                                              self.bytes, P(self.stream.cuda_stream),
                                              ctypes.byref(h)))
        self._h = h
        self.derived = [derive(c) for c in self.cfgs]

    # ------------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "_h", None):
            lib().pic_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, name, *args):
        _check(name, getattr(lib(), name)(self._h, *args), self._h)

    def step(self, n=1):
        self._call("pic_step", int(n))

    def set_graph(self, k):
        self._call("pic_set_graph", int(k))

    def sync(self):
        self._call("pic_sync")

    def profile(self, enable=True):
        self._call("pic_profile", 1 if enable else 0)

    def profile_read(self):
        ms = (F64 * len(PHASES))()
        cnt = (U64 * len(PHASES))()
        self._call("pic_profile_read", ms, cnt, len(PHASES))
        return {p: (ms[i], cnt[i]) for i, p in enumerate(PHASES)}

    # ------------------------------------------------------------------ read-out
    def n_nodes(self, d=0):
        w = self.workloads[d]
        return w["n_cells"] if w["periodic"] else w["n_cells"] + 1

    def grid(self, what, d=0):
        names = {"w_e": 0, "w_i": 1, "phi": 2, "E": 3, "acc_w_e": 4, "acc_w_i": 5,
                 "acc_phi": 6, "eedf": 7}
        k = names[what]
        n = self.workloads[d]["eedf_bins"] + 1 if k == 7 else self.n_nodes(d)
        out = np.zeros(n)
        self._call("pic_grid", d, k, _ptr(out), n)
        return out

    def density(self, quantity, kind=0, d=0):
        q = {"n_e": 0, "n_i": 1, "phi": 2}[quantity]
        out = np.zeros(self.n_nodes(d))
        self._call("pic_density", d, q, int(kind), _ptr(out), out.size)
        return out

    def diagnostics(self, d=0, eedf=False):
        """pic_diag of discharge d; with eedf=True the EEDF counts come back in the same
        call, as the array attribute ``eedf_counts``."""
        g = PicDiag()
        buf = None
        if eedf:
            buf = np.zeros(self.workloads[d]["eedf_bins"] + 1)
            g.eedf = buf.ctypes.data_as(ctypes.POINTER(F64))
            g.eedf_len = buf.size
        self._call("pic_diagnostics", d, ctypes.byref(g))
        if buf is not None:
            g.eedf_counts = buf[:g.eedf_len].copy()
        return g

    def get_state(self, d=0):
        diag = self.diagnostics(d)
        st = PicState()
        out = {}
        for s in (0, 1):
            n = int(diag.n_particles[s])
            st.capacity[s] = n
            arrs = {}
            if self.fp32:
                arrs["cell"] = np.zeros(n, np.int32)
                for k in ("off", "vxf", "vyf", "vzf"):
                    arrs[k] = np.zeros(n, np.float32)
            else:
                for k in ("x", "vx", "vy", "vz"):
                    arrs[k] = np.zeros(n, np.float64)
            arrs["id"] = np.zeros(n, np.uint32)
            arrs["w"] = np.zeros(self.n_nodes(d))
            for k, a in arrs.items():
                getattr(st, k)[s] = _ptr(a)
            out[s] = arrs
        self._call("pic_get_state", d, ctypes.byref(st))
        res = {"step": int(st.step), "next_id": [int(st.next_id[0]), int(st.next_id[1])]}
        for s in (0, 1):
            a = out[s]
            a["n"] = int(st.n[s])
            a["n_sorted"] = int(st.n_sorted[s])
            res[s] = a
        return res

    def set_state(self, state, d=0, sort_all=False):
        st = PicState()
        keep = []
        for s in (0, 1):
            a = state[s]
            n = int(a["n"])
            st.n[s] = n
            st.n_sorted[s] = int(a.get("n_sorted", n))
            names = ("cell", "off", "vxf", "vyf", "vzf") if self.fp32 else ("x", "vx", "vy", "vz")
            dt = {"cell": np.int32, "off": np.float32, "vxf": np.float32, "vyf": np.float32,
                  "vzf": np.float32, "x": np.float64, "vx": np.float64, "vy": np.float64,
                  "vz": np.float64}
            for k in names:
                arr = np.ascontiguousarray(a[k][:n], dtype=dt[k])
                keep.append(arr)
                getattr(st, k)[s] = _ptr(arr)
            ids = np.ascontiguousarray(a["id"][:n], dtype=np.uint32)
            keep.append(ids)
            st.id[s] = _ptr(ids)
        st.step = int(state["step"])
        st.next_id[0], st.next_id[1] = int(state["next_id"][0]), int(state["next_id"][1])
        st.sort_all = 1 if sort_all else 0
        self._call("pic_set_state", d, ctypes.byref(st))


def particle_positions(state_s, fp32):
    """FP64 positions of one species of a state (cell + offset is exact in FP64)."""
    if fp32:
        return state_s["cell"].astype(np.float64) + state_s["off"].astype(np.float64)
    return state_s["x"]

"""Python binding of libatns (include/atns.h): argument marshalling only.

Every step of the method runs in the gfx950 kernels of libatns.so; this module allocates the
workspace with torch on the current CUDA (HIP) device, passes torch's current stream, and converts
arguments.  There is no CPU fallback: importing it without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libatns.so")

AT_OK, AT_E_INVAL, AT_E_WORKSPACE, AT_E_SCHEDULE, AT_E_HIP, AT_E_STATE = 0, -1, -2, -3, -4, -5
FP64, FP32 = 0, 1
SYNC, CAA, SAA, EXPLICIT = 0, 1, 2, 3
N_FORCE = 40
EXPORTED = ["at_version", "at_last_error", "at_workspace_bytes", "at_create", "at_init_field",
            "at_set_delay_schedule", "at_set_forcing", "at_rhs", "at_rk_step", "at_ab2_step", "at_stats",
            "at_get_field", "at_field_device", "at_destroy", "at_set_kernel_timing",
            "at_kernel_timing", "at_kernel_name", "at_set_tuning", "at_get_tuning",
            "at_set_stage_tuning", "at_get_stage_tuning",
            "at_batch_create", "at_batch_add", "at_batch_remove", "at_batch_size", "at_batch_step",
            "at_batch_set_tuning", "at_batch_get_tuning", "at_batch_set_stage_tuning",
            "at_batch_get_stage_tuning", "at_batch_autotune", "at_batch_set_graph",
            "at_batch_graph_stats", "at_batch_destroy", "at_serve", "at_field_stats_noalloc",
            "at_diag_workspace_bytes", "at_field_diagnostics"]
N_TILES = 7
N_KERNELS = 12


class AtError(RuntimeError):
    def __init__(self, call: str, rc: int, msg: str):
        super().__init__(f"{call} failed ({rc}): {msg}")
        self.rc = rc


class _Config(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("p", C.c_int32 * 3), ("order", C.c_int32),
                ("max_delay", C.c_int32), ("precision", C.c_int32), ("forcing", C.c_int32),
                ("gamma", C.c_double), ("prandtl", C.c_double), ("gas_r", C.c_double),
                ("mu_ref", C.c_double), ("t_ref", C.c_double), ("mu_exp", C.c_double),
                ("dt", C.c_double), ("form", C.c_int32), ("visc_law", C.c_int32), ("sutherland_s", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("step", C.c_int64), ("time", C.c_double), ("mass", C.c_double),
                ("mom", C.c_double * 3), ("energy", C.c_double), ("mass_rk", C.c_double),
                ("mom_rk", C.c_double * 3), ("energy_rk", C.c_double), ("K", C.c_double),
                ("eps", C.c_double), ("enstrophy", C.c_double), ("Mt", C.c_double),
                ("umax", C.c_double), ("nonfinite", C.c_int32), ("reserved", C.c_int32)]


class _ServeConfig(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_active", C.c_int32), ("tile", C.c_int32),
                ("zchunk", C.c_int32), ("hbm_budget_bytes", C.c_double), ("tile_delayed", C.c_int32),
                ("zchunk_delayed", C.c_int32)]


class _Request(C.Structure):
    _fields_ = [("arrival_s", C.c_double), ("n", C.c_int32), ("p", C.c_int32), ("steps", C.c_int32),
                ("mode", C.c_int32), ("L", C.c_int32), ("seed", C.c_uint64), ("dt", C.c_double),
                ("mu_ref", C.c_double), ("q0", C.POINTER(C.c_double)), ("q_final", C.POINTER(C.c_double))]


class _Result(C.Structure):
    _fields_ = [("admit_s", C.c_double), ("done_s", C.c_double), ("stats", _Stats), ("status", C.c_int32),
                ("reserved", C.c_int32)]


class _DiagParams(C.Structure):
    _fields_ = [("nshell", C.c_int32), ("nbins", C.c_int32), ("eps_max", C.c_double), ("ens_max", C.c_double)]


DIAG_N_SCALARS = 8
DIAG_SCALARS = ("S", "F", "g2", "g3", "g4", "eps_mean", "ens_mean", "p_mean")

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libatns.so and declare its signatures.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libatns.so not built at {path}; run __graft_entry__.build()")
    lib = C.CDLL(path)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    lib.at_version.restype = C.c_char_p
    lib.at_last_error.restype = C.c_char_p
    lib.at_workspace_bytes.argtypes = [C.POINTER(_Config)]
    lib.at_workspace_bytes.restype = C.c_size_t
    lib.at_create.argtypes = [C.POINTER(_Config), vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.at_init_field.argtypes = [vp, dp, i32]
    lib.at_set_delay_schedule.argtypes = [vp, i32, i32, i32, C.c_uint64, C.POINTER(C.c_int8), i64]
    lib.at_set_forcing.argtypes = [vp, dp, i64]
    lib.at_rhs.argtypes = [vp, vp]
    lib.at_rk_step.argtypes = [vp, i32]
    lib.at_ab2_step.argtypes = [vp, i32]
    lib.at_stats.argtypes = [vp, C.POINTER(_Stats)]
    lib.at_get_field.argtypes = [vp, dp]
    lib.at_field_device.argtypes = [vp, C.POINTER(vp)]
    lib.at_destroy.argtypes = [vp]
    lib.at_set_kernel_timing.argtypes = [vp, i32]
    lib.at_kernel_timing.argtypes = [vp, i32, dp, C.POINTER(C.c_int64)]
    lib.at_kernel_name.argtypes = [i32]
    lib.at_kernel_name.restype = C.c_char_p
    lib.at_set_tuning.argtypes = [vp, i32, i32]
    lib.at_get_tuning.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.at_set_stage_tuning.argtypes = [vp, i32, i32, i32, i32]
    lib.at_get_stage_tuning.argtypes = [vp] + [C.POINTER(C.c_int32)] * 4
    lib.at_batch_create.argtypes = [i32, vp, C.POINTER(vp)]
    lib.at_batch_add.argtypes = [vp, vp]
    lib.at_batch_remove.argtypes = [vp, vp]
    lib.at_batch_size.argtypes = [vp, C.POINTER(C.c_int32)]
    lib.at_batch_step.argtypes = [vp, i32]
    lib.at_batch_set_tuning.argtypes = [vp, i32, i32]
    lib.at_batch_get_tuning.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.at_batch_set_stage_tuning.argtypes = [vp, i32, i32, i32, i32]
    lib.at_batch_get_stage_tuning.argtypes = [vp] + [C.POINTER(C.c_int32)] * 4
    lib.at_batch_autotune.argtypes = [vp, C.c_char_p, i32, dp]
    lib.at_batch_set_graph.argtypes = [vp, i32]
    lib.at_batch_graph_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.at_batch_destroy.argtypes = [vp]
    lib.at_serve.argtypes = [C.POINTER(_ServeConfig), C.POINTER(_Request), i32, vp, C.POINTER(_Result), dp]
    lib.at_field_stats_noalloc.argtypes = [C.POINTER(_Config), vp, vp, vp]
    lib.at_diag_workspace_bytes.argtypes = [C.POINTER(_Config), C.POINTER(_DiagParams)]
    lib.at_diag_workspace_bytes.restype = C.c_size_t
    lib.at_field_diagnostics.argtypes = [C.POINTER(_Config), vp, vp, C.c_size_t, C.POINTER(_DiagParams), vp, vp]
    _lib = lib
    return lib


def _check(call, rc):
    if rc != AT_OK:
        raise AtError(call, rc, load_library().at_last_error().decode())


@dataclass
class Config:
    n: tuple
    p: tuple
    dt: float
    mu_ref: float
    max_delay: int = 3
    precision: str = "fp64"
    forcing: bool = False
    gamma: float = 1.4
    prandtl: float = 0.7
    gas_r: float = 1.0
    t_ref: float = 1.0
    mu_exp: float = 0.76
    order: int = 4
    form: int = 0              # 0 total-energy flux form; 1 the paper's own form (rho e, expanded terms)
    visc_law: int = 0          # 0 power law (mu_exp); 1 Sutherland (form 1)
    sutherland_s: float = 0.0  # Sutherland's constant

    def to_c(self) -> _Config:
        c = _Config()
        for d in range(3):
            c.n[d] = int(self.n[d])
            c.p[d] = int(self.p[d])
        c.order = int(self.order)
        c.form = int(self.form)
        c.visc_law = int(self.visc_law)
        c.sutherland_s = float(self.sutherland_s)
        c.max_delay = int(self.max_delay)
        c.precision = FP32 if self.precision == "fp32" else FP64
        c.forcing = int(bool(self.forcing))
        for k in ("gamma", "prandtl", "gas_r", "mu_ref", "t_ref", "mu_exp", "dt"):
            setattr(c, k, float(getattr(self, k)))
        return c

    @property
    def shape(self):
        return (int(self.n[2]), int(self.n[1]), int(self.n[0]))

    @property
    def ntiles(self):
        return int(self.p[0] * self.p[1] * self.p[2])

    @property
    def torch_dtype(self):
        import torch
        return torch.float32 if self.precision == "fp32" else torch.float64


def workspace_bytes(cfg: Config) -> int:
    c = cfg.to_c()
    return int(load_library().at_workspace_bytes(C.byref(c)))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _stats_dict(s: _Stats) -> dict:
    return {"step": s.step, "time": s.time, "mass": s.mass, "momx": s.mom[0], "momy": s.mom[1],
            "momz": s.mom[2], "energy": s.energy, "mass_rk": s.mass_rk, "momx_rk": s.mom_rk[0],
            "momy_rk": s.mom_rk[1], "momz_rk": s.mom_rk[2], "energy_rk": s.energy_rk, "K": s.K,
            "eps": s.eps, "enstrophy": s.enstrophy, "Mt": s.Mt, "umax": s.umax,
            "nonfinite": s.nonfinite}


class Sim:
    """One simulation on the current device: workspace (torch-owned) + handle."""

    def __init__(self, cfg: Config, device=None, stream=None):
        import torch
        self.lib = load_library()
        self.cfg = cfg
        self._c = cfg.to_c()
        nbytes = int(self.lib.at_workspace_bytes(C.byref(self._c)))
        if nbytes == 0:
            raise AtError("at_workspace_bytes", AT_E_INVAL, self.lib.at_last_error().decode())
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check("at_create", self.lib.at_create(C.byref(self._c), C.c_void_p(self.workspace.data_ptr()),
                                               nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.at_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_field(self, q: np.ndarray, n_levels: int = 1):
        q = np.ascontiguousarray(q, dtype=np.float64)
        _check("at_init_field", self.lib.at_init_field(self.h, _dp(q), int(n_levels)))

    def set_delay_schedule(self, mode, L=0, c_r=1, seed=0, table=None, n_steps=None):
        tp = None
        if table is not None:
            table = np.ascontiguousarray(table, dtype=np.int8)
            if n_steps is None:
                n_steps = table.shape[0]
            tp = table.ctypes.data_as(C.POINTER(C.c_int8))
        _check("at_set_delay_schedule", self.lib.at_set_delay_schedule(
            self.h, int(mode), int(L), int(c_r), C.c_uint64(seed), tp, int(n_steps)))

    def set_forcing(self, fhat: np.ndarray):
        fhat = np.ascontiguousarray(fhat, dtype=np.float64)
        assert fhat.shape[1:] == (N_FORCE, 3, 2)
        _check("at_set_forcing", self.lib.at_set_forcing(self.h, _dp(fhat), fhat.shape[0]))

    def rhs(self, out=None):
        import torch
        if out is None:
            out = torch.empty((5,) + self.cfg.shape, dtype=self.cfg.torch_dtype, device=self.device)
        assert out.is_contiguous() and out.dtype == self.cfg.torch_dtype
        _check("at_rhs", self.lib.at_rhs(self.h, C.c_void_p(out.data_ptr())))
        return out

    def rk_step(self, n_steps: int = 1):
        _check("at_rk_step", self.lib.at_rk_step(self.h, int(n_steps)))

    def ab2_step(self, n_steps: int = 1):
        """Second-order Adams-Bashforth steps (at_ab2_step)."""
        _check("at_ab2_step", self.lib.at_ab2_step(self.h, int(n_steps)))

    def stats(self) -> dict:
        s = _Stats()
        _check("at_stats", self.lib.at_stats(self.h, C.byref(s)))
        return _stats_dict(s)

    def get_field(self) -> np.ndarray:
        out = np.empty((5,) + self.cfg.shape, dtype=np.float64)
        _check("at_get_field", self.lib.at_get_field(self.h, _dp(out)))
        return out

    def set_tuning(self, tile: int, zchunk: int):
        _check("at_set_tuning", self.lib.at_set_tuning(self.h, int(tile), int(zchunk)))

    def get_tuning(self):
        t, z = C.c_int32(), C.c_int32()
        _check("at_get_tuning", self.lib.at_get_tuning(self.h, C.byref(t), C.byref(z)))
        return int(t.value), int(z.value)

    def set_stage_tuning(self, tile_sync: int, zchunk_sync: int, tile_delayed: int, zchunk_delayed: int):
        _check("at_set_stage_tuning", self.lib.at_set_stage_tuning(self.h, int(tile_sync), int(zchunk_sync),
                                                                   int(tile_delayed), int(zchunk_delayed)))

    def get_stage_tuning(self):
        v = [C.c_int32() for _ in range(4)]
        _check("at_get_stage_tuning", self.lib.at_get_stage_tuning(self.h, *[C.byref(x) for x in v]))
        return tuple(int(x.value) for x in v)

    def set_kernel_timing(self, enable: bool):
        _check("at_set_kernel_timing", self.lib.at_set_kernel_timing(self.h, int(bool(enable))))

    def kernel_timing(self) -> dict:
        """{kernel name: (total ms, launches)} for kernels launched since timing was enabled."""
        out = {}
        for k in range(N_KERNELS):
            ms, cnt = C.c_double(), C.c_int64()
            _check("at_kernel_timing", self.lib.at_kernel_timing(self.h, k, C.byref(ms), C.byref(cnt)))
            if cnt.value:
                out[self.lib.at_kernel_name(k).decode()] = (ms.value, cnt.value)
        return out

    def field_device_ptr(self) -> int:
        p = C.c_void_p()
        _check("at_field_device", self.lib.at_field_device(self.h, C.byref(p)))
        return int(p.value)

    def diagnostics(self, nshell: int, nbins: int, eps_max: float, ens_max: float, workspace=None) -> dict:
        """at_field_diagnostics of the current state on the run's stream (see field_diagnostics)."""
        return field_diagnostics(self.cfg, self.field_device_ptr(), nshell, nbins, eps_max, ens_max,
                                 workspace=workspace, stream=self.stream)


class Batch:
    """Batched runs (include/atns.h, at_batch_*): members advance together, one launch per kernel
    per RK stage, replayed from a HIP graph.  Members must share the batch's precision and stream."""

    def __init__(self, precision: str = "fp32", stream=None):
        import torch
        self.lib = load_library()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check("at_batch_create", self.lib.at_batch_create(FP32 if precision == "fp32" else FP64,
                                                           C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.members = []

    def close(self):
        if getattr(self, "h", None):
            self.lib.at_batch_destroy(self.h)
            self.h = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, sim: Sim):
        _check("at_batch_add", self.lib.at_batch_add(self.h, sim.h))
        self.members.append(sim)

    def remove(self, sim: Sim):
        _check("at_batch_remove", self.lib.at_batch_remove(self.h, sim.h))
        self.members = [m for m in self.members if m is not sim]

    def __len__(self):
        n = C.c_int32()
        _check("at_batch_size", self.lib.at_batch_size(self.h, C.byref(n)))
        return int(n.value)

    def step(self, n_steps: int = 1):
        _check("at_batch_step", self.lib.at_batch_step(self.h, int(n_steps)))

    def set_tuning(self, tile: int, zchunk: int):
        _check("at_batch_set_tuning", self.lib.at_batch_set_tuning(self.h, int(tile), int(zchunk)))

    def get_tuning(self):
        t, z = C.c_int32(), C.c_int32()
        _check("at_batch_get_tuning", self.lib.at_batch_get_tuning(self.h, C.byref(t), C.byref(z)))
        return int(t.value), int(z.value)

    def set_stage_tuning(self, tile_sync: int, zchunk_sync: int, tile_delayed: int, zchunk_delayed: int):
        _check("at_batch_set_stage_tuning",
               self.lib.at_batch_set_stage_tuning(self.h, int(tile_sync), int(zchunk_sync), int(tile_delayed),
                                                  int(zchunk_delayed)))

    def get_stage_tuning(self):
        v = [C.c_int32() for _ in range(4)]
        _check("at_batch_get_stage_tuning", self.lib.at_batch_get_stage_tuning(self.h, *[C.byref(x) for x in v]))
        return tuple(int(x.value) for x in v)

    def autotune(self, cache_path=None, reps: int = 3) -> float:
        ms = C.c_double()
        path = None if cache_path is None else str(cache_path).encode()
        _check("at_batch_autotune", self.lib.at_batch_autotune(self.h, path, int(reps), C.byref(ms)))
        return float(ms.value)

    def set_graph(self, enable: bool):
        _check("at_batch_set_graph", self.lib.at_batch_set_graph(self.h, int(bool(enable))))

    def graph_stats(self):
        c, r = C.c_int64(), C.c_int64()
        _check("at_batch_graph_stats", self.lib.at_batch_graph_stats(self.h, C.byref(c), C.byref(r)))
        return int(c.value), int(r.value)


def serve(requests, precision: str = "fp32", max_active: int = 64, hbm_budget_bytes: float = 64e9,
          tile: int = -1, zchunk: int = 64, stream=None, tile_delayed: int = -1, zchunk_delayed: int = 64):
    """Serve a request trace with continuous batching (at_serve).  Each request is a dict with
    arrival_s, n, p, steps, mode, L, seed, dt, mu_ref, q0 (float64 [5][n][n][n]) and optionally
    q_final (a float64 array of the same shape that receives the final state).  Returns
    (list of {admit_s, done_s, status, stats}, makespan in s)."""
    import torch
    lib = load_library()
    st = stream if stream is not None else torch.cuda.current_stream()
    sc = _ServeConfig(FP32 if precision == "fp32" else FP64, int(max_active), int(tile), int(zchunk),
                      float(hbm_budget_bytes), int(tile_delayed), int(zchunk_delayed))
    n = len(requests)
    reqs = (_Request * max(n, 1))()
    keep = []
    for i, r in enumerate(requests):
        q0 = np.ascontiguousarray(r["q0"], dtype=np.float64)
        keep.append(q0)
        qf = r.get("q_final")
        if qf is not None:
            assert qf.dtype == np.float64 and qf.flags.c_contiguous and qf.shape == q0.shape
        reqs[i] = _Request(float(r["arrival_s"]), int(r["n"]), int(r["p"]), int(r["steps"]), int(r["mode"]),
                           int(r["L"]), C.c_uint64(int(r.get("seed", 0))), float(r["dt"]), float(r["mu_ref"]),
                           _dp(q0), _dp(qf) if qf is not None else None)
    res = (_Result * max(n, 1))()
    mk = C.c_double()
    _check("at_serve", lib.at_serve(C.byref(sc), reqs, n, C.c_void_p(st.cuda_stream), res, C.byref(mk)))
    out = [{"admit_s": res[i].admit_s, "done_s": res[i].done_s, "status": res[i].status,
            "stats": _stats_dict(res[i].stats)} for i in range(n)]
    return out, float(mk.value)


STATS_RECORD_BYTES = C.sizeof(_Stats)


def field_stats_noalloc(cfg: Config, dev_q: int, dev_out: int, stream=None):
    """at_field_stats_noalloc: statistics of the device field at `dev_q` into the device record at
    `dev_out` (STATS_RECORD_BYTES bytes), enqueued on `stream` (default: torch's current stream)."""
    import torch
    lib = load_library()
    c = cfg.to_c()
    st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check("at_field_stats_noalloc", lib.at_field_stats_noalloc(C.byref(c), C.c_void_p(dev_q),
                                                                 C.c_void_p(dev_out), C.c_void_p(st)))


def stats_record(raw: bytes) -> dict:
    """A statistics record (as written by field_stats_noalloc) as a dict."""
    s = _Stats.from_buffer_copy(raw)
    return _stats_dict(s)


def diag_params(nshell: int, nbins: int, eps_max: float, ens_max: float) -> _DiagParams:
    return _DiagParams(int(nshell), int(nbins), float(eps_max), float(ens_max))


def diag_workspace_bytes(cfg: Config, nshell: int, nbins: int, eps_max: float, ens_max: float) -> int:
    c, p = cfg.to_c(), diag_params(nshell, nbins, eps_max, ens_max)
    return int(load_library().at_diag_workspace_bytes(C.byref(c), C.byref(p)))


def field_diagnostics(cfg: Config, dev_q: int, nshell: int, nbins: int, eps_max: float, ens_max: float,
                      workspace=None, stream=None, out=None, sync: bool = True):
    """at_field_diagnostics of the device field at `dev_q` (cfg's precision, [5][nz][ny][nx]).

    workspace: a torch uint8 device tensor of at least diag_workspace_bytes (allocated here if None);
    out: a torch float64 device tensor for the raw output (allocated if None).  With sync=True the
    result is returned as a dict of numpy arrays and floats (E, Ep, S, F, g2, g3, g4, eps_mean,
    ens_mean, p_mean, eps_pdf, ens_pdf); with sync=False the raw device tensor is returned unread."""
    import torch
    lib = load_library()
    c, p = cfg.to_c(), diag_params(nshell, nbins, eps_max, ens_max)
    nbytes = int(lib.at_diag_workspace_bytes(C.byref(c), C.byref(p)))
    if nbytes == 0:
        raise AtError("at_diag_workspace_bytes", AT_E_INVAL, lib.at_last_error().decode())
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    nout = 2 * nshell + DIAG_N_SCALARS + 2 * (nbins + 1)
    if out is None:
        out = torch.empty(nout, dtype=torch.float64, device=workspace.device)
    assert out.dtype == torch.float64 and out.numel() >= nout and out.is_contiguous()
    st = stream if stream is not None else torch.cuda.current_stream()
    _check("at_field_diagnostics", lib.at_field_diagnostics(
        C.byref(c), C.c_void_p(dev_q), C.c_void_p(workspace.data_ptr()), workspace.numel(), C.byref(p),
        C.c_void_p(out.data_ptr()), C.c_void_p(st.cuda_stream)))
    if not sync:
        return out
    st.synchronize()
    return diag_dict(out.cpu().numpy(), nshell, nbins)


def diag_dict(raw: np.ndarray, nshell: int, nbins: int) -> dict:
    """The output array of at_field_diagnostics as a dict."""
    d = {"E": raw[:nshell].copy(), "Ep": raw[nshell:2 * nshell].copy()}
    sc = raw[2 * nshell:2 * nshell + DIAG_N_SCALARS]
    d.update({k: float(v) for k, v in zip(DIAG_SCALARS, sc)})
    o = 2 * nshell + DIAG_N_SCALARS
    d["eps_pdf"] = raw[o:o + nbins + 1].astype(np.int64)
    d["ens_pdf"] = raw[o + nbins + 1:o + 2 * (nbins + 1)].astype(np.int64)
    return d

"""ctypes wrapper of the C oracle (test infrastructure only; never used by the product path)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "atns_oracle.c")
_LIB = os.path.join(_HERE, "libatns_oracle.so")

STAT_NAMES = ["step", "time", "mass", "momx", "momy", "momz", "energy", "mass_rk", "momx_rk",
              "momy_rk", "momz_rk", "energy_rk", "K", "eps", "enstrophy", "Mt", "umax", "nonfinite"]
SYNC, CAA, SAA, EXPLICIT = 0, 1, 2, 3


def library_path() -> str:
    return _LIB


def build() -> str:
    """Compile the oracle with gcc, FP64, no contraction into fused multiply-adds."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
           "-shared", "-fPIC", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Cfg(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("p", C.c_int32 * 3), ("max_delay", C.c_int32),
                ("forcing", C.c_int32), ("order", C.c_int32), ("gamma", C.c_double), ("prandtl", C.c_double),
                ("gas_r", C.c_double), ("mu_ref", C.c_double), ("t_ref", C.c_double),
                ("mu_exp", C.c_double), ("dt", C.c_double), ("form", C.c_int32), ("visc", C.c_int32),
                ("suth_s", C.c_double)]


@dataclass
class OracleConfig:
    n: tuple
    p: tuple
    dt: float
    mu_ref: float
    max_delay: int = 3
    forcing: bool = False
    gamma: float = 1.4
    prandtl: float = 0.7
    gas_r: float = 1.0
    t_ref: float = 1.0
    mu_exp: float = 0.76
    order: int = 4
    form: int = 0          # 0 total-energy flux form, 1 the paper's own form (rho e, expanded terms)
    visc: int = 0          # 0 power law, 1 Sutherland (form 1)
    suth_s: float = 0.0    # Sutherland's constant

    def to_c(self) -> _Cfg:
        c = _Cfg()
        n = self.n if isinstance(self.n, (tuple, list)) else (self.n,) * 3
        p = self.p if isinstance(self.p, (tuple, list)) else (self.p,) * 3
        for d in range(3):
            c.n[d] = int(n[d])
            c.p[d] = int(p[d])
        c.max_delay = int(self.max_delay)
        c.forcing = int(bool(self.forcing))
        c.order = int(self.order)
        c.form = int(self.form)
        c.visc = int(self.visc)
        c.suth_s = float(self.suth_s)
        for k in ("gamma", "prandtl", "gas_r", "mu_ref", "t_ref", "mu_exp", "dt"):
            setattr(c, k, float(getattr(self, k)))
        return c

    @property
    def shape(self):
        n = self.n if isinstance(self.n, (tuple, list)) else (self.n,) * 3
        return (int(n[2]), int(n[1]), int(n[0]))

    @property
    def ntiles(self):
        p = self.p if isinstance(self.p, (tuple, list)) else (self.p,) * 3
        return int(p[0] * p[1] * p[2])


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        vp, dp, i32, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64
        lib.ora_create.argtypes = [C.POINTER(_Cfg), C.POINTER(vp)]
        lib.ora_destroy.argtypes = [vp]
        lib.ora_destroy.restype = None
        lib.ora_init_field.argtypes = [vp, dp, i32]
        lib.ora_set_schedule.argtypes = [vp, i32, i32, i32, C.c_uint64, C.POINTER(C.c_int8), i64]
        lib.ora_get_schedule.argtypes = [vp, C.POINTER(C.c_int8), i64]
        lib.ora_set_forcing.argtypes = [vp, dp, i64]
        lib.ora_rhs.argtypes = [vp, dp]
        lib.ora_rk_step.argtypes = [vp, i32]
        lib.ora_ab2_step.argtypes = [vp, i32]
        lib.ora_stats.argtypes = [vp, dp]
        lib.ora_get_field.argtypes = [vp, dp]
        lib.ora_get_flux.argtypes = [vp, dp]
        lib.ora_step.argtypes = [vp]
        lib.ora_step.restype = i64
        lib.ora_rhs_periodic_standard.argtypes = [C.POINTER(_Cfg), dp, dp]
        lib.ora_at_weight.argtypes = [i32, C.c_double]
        lib.ora_at_weight.restype = C.c_double
        lib.ora_at_weight6.argtypes = [i32, C.c_double]
        lib.ora_at_weight6.restype = C.c_double
        lib.ora_count_at_points.argtypes = [C.POINTER(_Cfg)]
        lib.ora_count_at_points.restype = i64
        lib.ora_forcing_field.argtypes = [C.POINTER(_Cfg), dp, dp]
        lib.ora_diag_fields.argtypes = [C.POINTER(_Cfg), dp, dp]
        lib.ora_pe_derivative.argtypes = [dp, C.c_int32, C.c_double, dp]
        lib.ora_viscosity.argtypes = [C.POINTER(_Cfg), C.c_double, dp]
        lib.ora_viscosity.restype = C.c_double
        lib.ora_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        lib.ora_splitmix64.restype = C.c_uint64
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleError(RuntimeError):
    def __init__(self, what, rc):
        super().__init__(f"oracle {what} failed with code {rc}")
        self.rc = rc


class Oracle:
    """One oracle run: config, current state, ring of published levels, schedule, forcing."""

    def __init__(self, cfg: OracleConfig):
        self.cfg = cfg
        self._c = cfg.to_c()
        self.lib = _load()
        h = C.c_void_p()
        rc = self.lib.ora_create(C.byref(self._c), C.byref(h))
        if rc:
            raise OracleError("create", rc)
        self.h = h

    def close(self):
        if self.h:
            self.lib.ora_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, what, rc):
        if rc:
            raise OracleError(what, rc)

    def init_field(self, q: np.ndarray, nlev: int = 1):
        q = np.ascontiguousarray(q, dtype=np.float64)
        self._chk("init_field", self.lib.ora_init_field(self.h, _dp(q), int(nlev)))

    def set_schedule(self, mode, L=0, c_r=1, seed=0, table=None, n_steps=0):
        tp = None
        if table is not None:
            table = np.ascontiguousarray(table, dtype=np.int8)
            n_steps = table.shape[0]
            tp = table.ctypes.data_as(C.POINTER(C.c_int8))
        self._tab = table
        self._chk("set_schedule", self.lib.ora_set_schedule(self.h, int(mode), int(L), int(c_r),
                                                            C.c_uint64(seed), tp, int(n_steps)))

    def get_schedule(self, n_steps):
        out = np.zeros((n_steps, self.cfg.ntiles, 6), dtype=np.int8)
        self._chk("get_schedule", self.lib.ora_get_schedule(self.h, out.ctypes.data_as(C.POINTER(C.c_int8)),
                                                            int(n_steps)))
        return out

    def set_forcing(self, fhat: np.ndarray):
        fhat = np.ascontiguousarray(fhat, dtype=np.float64)
        self._fh = fhat
        self._chk("set_forcing", self.lib.ora_set_forcing(self.h, _dp(fhat), fhat.shape[0]))

    def rhs(self) -> np.ndarray:
        out = np.zeros((5,) + self.cfg.shape)
        self._chk("rhs", self.lib.ora_rhs(self.h, _dp(out)))
        return out

    def rk_step(self, nsteps=1):
        self._chk("rk_step", self.lib.ora_rk_step(self.h, int(nsteps)))

    def ab2_step(self, nsteps=1):
        """Second-order Adams-Bashforth steps (Sec. 2.2, Eq. time_ab); forward Euler where no
        f^{n-1} is stored (after initialisation or Runge-Kutta steps)."""
        self._chk("ab2_step", self.lib.ora_ab2_step(self.h, int(nsteps)))

    def stats(self) -> dict:
        out = np.zeros(len(STAT_NAMES))
        self._chk("stats", self.lib.ora_stats(self.h, _dp(out)))
        return dict(zip(STAT_NAMES, out.tolist()))

    def field(self) -> np.ndarray:
        out = np.zeros((5,) + self.cfg.shape)
        self._chk("get_field", self.lib.ora_get_field(self.h, _dp(out)))
        return out

    def flux(self) -> np.ndarray:
        out = np.zeros((3, 5) + self.cfg.shape)
        self._chk("get_flux", self.lib.ora_get_flux(self.h, _dp(out)))
        return out

    @property
    def step(self) -> int:
        return int(self.lib.ora_step(self.h))

    # -------- stateless hooks
    @staticmethod
    def rhs_periodic_standard(cfg: OracleConfig, q: np.ndarray) -> np.ndarray:
        lib = _load()
        c = cfg.to_c()
        q = np.ascontiguousarray(q, dtype=np.float64)
        out = np.zeros_like(q)
        rc = lib.ora_rhs_periodic_standard(C.byref(c), _dp(q), _dp(out))
        if rc:
            raise OracleError("rhs_periodic_standard", rc)
        return out

    @staticmethod
    def at_weight(l, kappa) -> float:
        return float(_load().ora_at_weight(int(l), float(kappa)))

    @staticmethod
    def at_weight6(l, kappa) -> float:
        return float(_load().ora_at_weight6(int(l), float(kappa)))

    @staticmethod
    def count_at_points(cfg: OracleConfig) -> int:
        c = cfg.to_c()
        return int(_load().ora_count_at_points(C.byref(c)))

    @staticmethod
    def forcing_field(cfg: OracleConfig, fhat_step: np.ndarray) -> np.ndarray:
        c = cfg.to_c()
        fh = np.ascontiguousarray(fhat_step, dtype=np.float64)
        out = np.zeros((3,) + cfg.shape)
        _load().ora_forcing_field(C.byref(c), _dp(fh), _dp(out))
        return out

    @staticmethod
    def diag_fields(cfg: OracleConfig, q: np.ndarray) -> np.ndarray:
        """[7][...]: u, v, w, p, du/dx, sigma_ij du_i/dx_j, |curl u|^2 (synchronous derivatives)."""
        c = cfg.to_c()
        q = np.ascontiguousarray(q, dtype=np.float64)
        out = np.zeros((7,) + cfg.shape)
        rc = _load().ora_diag_fields(C.byref(c), _dp(q), _dp(out))
        if rc:
            raise OracleError("diag_fields", rc)
        return out

    @staticmethod
    def pe_derivative(g: np.ndarray, h: float) -> np.ndarray:
        """Derivative along one PE's line of points using only those points (form 1 mixed
        derivatives): central inside, one-sided / biased fourth order at the ends."""
        g = np.ascontiguousarray(g, dtype=np.float64)
        out = np.zeros_like(g)
        rc = _load().ora_pe_derivative(_dp(g), int(g.size), float(h), _dp(out))
        if rc:
            raise OracleError("pe_derivative", rc)
        return out

    @staticmethod
    def viscosity(cfg: OracleConfig, T: float):
        """(mu, dmu/dT) of the configured law."""
        c = cfg.to_c()
        d = C.c_double()
        mu = _load().ora_viscosity(C.byref(c), float(T), C.byref(d))
        return float(mu), float(d.value)

    @staticmethod
    def splitmix64(seed, counter) -> int:
        return int(_load().ora_splitmix64(C.c_uint64(seed), C.c_uint64(counter)))

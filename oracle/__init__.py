"""FP64 CPU oracle of the LTNE MRT lattice Boltzmann step (Liu & He, arXiv:1608.04118).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline of the benchmark may import this package.  It loads
``libltne_oracle.so`` built from ``ltne_oracle.c`` (plain C, binary64,
``-ffp-contract=off``) and shares no code with the GPU library.

Fields are numpy arrays of shape (ny, nx); node index c = y * nx + x.
Parameters come as a plain dict whose keys are the field names of
``orc_params`` in ``ltne_oracle.h``; every key must be given (the oracle has no
defaults of its own, so a caller cannot silently rely on one).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ltne_oracle.c")
_HDR = os.path.join(_HERE, "ltne_oracle.h")
_LIB = os.path.join(_HERE, "libltne_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (binary64, no FMA contraction, OpenMP)."""
    stale = (not os.path.exists(_LIB)) or any(
        os.path.getmtime(s) > os.path.getmtime(_LIB) for s in (_SRC, _HDR))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("wall_thermal", C.c_int32 * 4),
        ("nu_wall", C.c_int32), ("thermal_correction", C.c_int32),
        ("T_wall", C.c_double * 4),
        ("T0", C.c_double), ("T_init_f", C.c_double), ("T_init_s", C.c_double),
        ("L", C.c_double), ("dT", C.c_double),
        ("phi", C.c_double), ("Da", C.c_double), ("F_phi", C.c_double),
        ("Ra", C.c_double), ("Pr", C.c_double), ("Je", C.c_double),
        ("gamma_sf", C.c_double), ("sigma", C.c_double), ("Hv", C.c_double),
        ("Qf", C.c_double), ("Qs", C.c_double),
        ("Ma", C.c_double), ("nu_f", C.c_double),
        ("body_force", C.c_double * 2),
        ("varpi", C.c_double), ("s_e", C.c_double), ("s_eps", C.c_double),
        ("s_q", C.c_double), ("zeta_e", C.c_double), ("zeta_nu", C.c_double),
        ("eta_e", C.c_double), ("eta_nu", C.c_double),
        ("rho0", C.c_double), ("pore_size", C.c_double),
    ]


class _Derived(C.Structure):
    _fields_ = [(k, C.c_double) for k in (
        "L", "dT", "cs2", "csT2", "gbeta", "u_c", "nu_f", "nu_e", "s_nu",
        "alpha_f", "alpha_s", "zeta_a", "eta_a", "K")]


_ORACLE_KEYS = [f[0] for f in _Params._fields_]

_lib = None


def compile_source(src_text: str, out_path: str) -> str:
    """Compile oracle C source text (for instance a copy with a deliberately
    planted mistake, in the tests that check the pins catch it) into a
    shared library at out_path, with the flags of build()."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-Wall",
           "-I", _HERE, "-o", out_path, src, "-lm"]
    subprocess.check_call(cmd)
    return out_path


def load_library(path: str):
    """A library built from (a variant of) the oracle source, configured like
    the default one; pass it to Oracle(..., lib=...)."""
    return _configure(C.CDLL(path))


def _load():
    global _lib
    if _lib is None:
        _lib = _configure(C.CDLL(build()))
    return _lib


def _configure(lib):
    """Declares the argument and result types of the oracle's entry points."""
    d = C.c_double
    dp = C.POINTER(C.c_double)
    vp = C.c_void_p
    lib.orc_params_size.restype = C.c_size_t
    assert lib.orc_params_size() == C.sizeof(_Params), "oracle struct layout mismatch"
    lib.orc_derive.argtypes = [C.POINTER(_Params), C.POINTER(_Derived)]
    lib.orc_derive.restype = C.c_int
    lib.orc_create.argtypes = [C.POINTER(_Params), vp, vp, vp, vp]
    lib.orc_create.restype = vp
    lib.orc_free.argtypes = [vp]
    lib.orc_step.argtypes = [vp, C.c_int64]
    lib.orc_steps_done.argtypes = [vp]
    lib.orc_steps_done.restype = C.c_int64
    lib.orc_macros.argtypes = [vp] + [vp] * 5
    lib.orc_get_populations.argtypes = [vp, vp, vp, vp]
    lib.orc_set_populations.argtypes = [vp, vp, vp, vp]
    lib.orc_nusselt.argtypes = [vp, dp, dp]
    lib.orc_nusselt.restype = C.c_int
    lib.orc_diagnostics.argtypes = [vp, dp, dp, dp]
    lib.orc_nusselt_field.argtypes = [C.POINTER(_Params), vp, C.c_int, dp]
    lib.orc_nusselt_field.restype = C.c_int
    lib.orc_feq.argtypes = [d, d, d, d, vp]
    lib.orc_geq_fluid.argtypes = [d, d, d, d, d, vp]
    lib.orc_geq_solid.argtypes = [d, d, vp]
    lib.orc_forcing.argtypes = [d, d, d, d, d, d, vp]
    lib.orc_matrices.argtypes = [vp, vp, vp, vp]
    lib.orc_velocity.argtypes = [d] * 9 + [dp] * 4
    lib.orc_temperatures.argtypes = [d] * 6 + [dp, dp]
    lib.orc_threads.restype = C.c_int
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _field(a, ny, nx):
    if a is None:
        return None
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (ny, nx)))
    return a


def _params(p: dict) -> _Params:
    missing = [k for k in _ORACLE_KEYS if k not in p]
    if missing:
        raise KeyError("oracle parameters missing: %s" % ", ".join(missing))
    s = _Params()
    for k in _ORACLE_KEYS:
        v = p[k]
        if k in ("wall_thermal", "T_wall", "body_force"):
            getattr(s, k)[:] = list(v)
        else:
            setattr(s, k, v)
    return s


def derive(p: dict) -> dict:
    lib = _load()
    d = _Derived()
    if lib.orc_derive(C.byref(_params(p)), C.byref(d)) != 0:
        raise ValueError("oracle rejected the parameters")
    return {k: getattr(d, k) for k, _ in _Derived._fields_}


def nusselt_field(p: dict, T, wall: int) -> float:
    """Mean Nusselt number of the temperature field T over wall 0..3
    (left, right, bottom, top)."""
    T = _field(T, int(p["ny"]), int(p["nx"]))
    out = C.c_double()
    if _load().orc_nusselt_field(C.byref(_params(p)), _ptr(T), int(wall), C.byref(out)) != 0:
        raise ValueError("bad parameters or wall")
    return out.value


def threads() -> int:
    return _load().orc_threads()


class Oracle:
    """One lattice: state, stepping and outputs, all in binary64."""

    def __init__(self, p: dict, phi=None, Hv=None, Tf0=None, Ts0=None, lib=None):
        lib = lib if lib is not None else _load()
        self.p = dict(p)
        self.nx, self.ny = int(p["nx"]), int(p["ny"])
        self._keep = [_field(a, self.ny, self.nx) for a in (phi, Hv, Tf0, Ts0)]
        self._h = lib.orc_create(C.byref(_params(p)), *[_ptr(a) for a in self._keep])
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_free(h)
            self._h = None

    def step(self, n: int = 1) -> "Oracle":
        self._lib.orc_step(self._h, int(n))
        return self

    @property
    def steps(self) -> int:
        return int(self._lib.orc_steps_done(self._h))

    def macros(self) -> dict:
        out = {k: np.empty((self.ny, self.nx)) for k in ("rho", "ux", "uy", "Tf", "Ts")}
        self._lib.orc_macros(self._h, *[_ptr(out[k]) for k in ("rho", "ux", "uy", "Tf", "Ts")])
        return out

    def populations(self):
        n = self.nx * self.ny
        f, gf, gs = np.empty((n, 9)), np.empty((n, 5)), np.empty((n, 5))
        self._lib.orc_get_populations(self._h, _ptr(f), _ptr(gf), _ptr(gs))
        return f, gf, gs

    def set_populations(self, f=None, gf=None, gs=None):
        n = self.nx * self.ny
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(n, -1)
                for a in (f, gf, gs)]
        self._lib.orc_set_populations(self._h, *[_ptr(a) for a in arrs])

    def nusselt(self):
        a, b = C.c_double(), C.c_double()
        if self._lib.orc_nusselt(self._h, C.byref(a), C.byref(b)) != 0:
            return float("nan"), float("nan")
        return a.value, b.value

    def diagnostics(self):
        m, e, r = C.c_double(), C.c_double(), C.c_double()
        self._lib.orc_diagnostics(self._h, C.byref(m), C.byref(e), C.byref(r))
        return m.value, e.value, r.value


# Node-level pieces (for identity checks).

def feq(rho, ux, uy, phi):
    out = np.empty(9)
    _load().orc_feq(rho, ux, uy, phi, _ptr(out))
    return out


def geq_fluid(T, ux, uy, phi, varpi):
    out = np.empty(5)
    _load().orc_geq_fluid(T, ux, uy, phi, varpi, _ptr(out))
    return out


def geq_solid(T, varpi):
    out = np.empty(5)
    _load().orc_geq_solid(T, varpi, _ptr(out))
    return out


def forcing(rho, ux, uy, Fx, Fy, phi):
    out = np.empty(9)
    _load().orc_forcing(rho, ux, uy, Fx, Fy, phi, _ptr(out))
    return out


def matrices():
    M, Mi, N, Ni = np.empty((9, 9)), np.empty((9, 9)), np.empty((5, 5)), np.empty((5, 5))
    _load().orc_matrices(_ptr(M), _ptr(Mi), _ptr(N), _ptr(Ni))
    return M, Mi, N, Ni


def velocity(rho, jx, jy, Gx, Gy, phi, nu_f, K, Fphi):
    r = [C.c_double() for _ in range(4)]
    _load().orc_velocity(rho, jx, jy, Gx, Gy, phi, nu_f, K, Fphi, *[C.byref(x) for x in r])
    return tuple(x.value for x in r)


def temperatures(sum_gf, sum_gs, Qf, Qs, d0, d1):
    a, b = C.c_double(), C.c_double()
    _load().orc_temperatures(sum_gf, sum_gs, Qf, Qs, d0, d1, C.byref(a), C.byref(b))
    return a.value, b.value

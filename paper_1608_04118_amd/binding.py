"""ctypes binding of ``liblbm_ltne.so`` (C ABI in ``include/lbm_ltne.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  Function names match the C entry points.  PyTorch, when used, only
provides device memory (a caller pool) and the stream the library queues on.

The library is loaded on first use; if it has not been built, a call raises
``RuntimeError`` -- there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbm_ltne.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_EDIVERGED, LBM_EUNSUPPORTED, LBM_ENODEV = (
    0, -1, -2, -3, -4, -5, -6)
LBM_FP64, LBM_FP32, LBM_FP16S, LBM_FP32SR = 0, 1, 2, 3
LBM_WALL_DIRICHLET, LBM_WALL_ADIABATIC = 0, 1


class lbm_ltne_params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("precision", C.c_int32),
        ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("wall_thermal", C.c_int32 * 4), ("nu_wall", C.c_int32), ("thermal_correction", C.c_int32),
        ("T_wall", C.c_double * 4), ("T0", C.c_double),
        ("T_init_f", C.c_double), ("T_init_s", C.c_double),
        ("L", C.c_double), ("dT", C.c_double),
        ("phi", C.c_double), ("Da", C.c_double), ("F_phi", C.c_double),
        ("Ra", C.c_double), ("Pr", C.c_double), ("Je", C.c_double),
        ("gamma_sf", C.c_double), ("sigma", C.c_double), ("Hv", C.c_double),
        ("Qf", C.c_double), ("Qs", C.c_double), ("Ma", C.c_double), ("nu_f", C.c_double),
        ("body_force", C.c_double * 2), ("varpi", C.c_double),
        ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double),
        ("zeta_e", C.c_double), ("zeta_nu", C.c_double),
        ("eta_e", C.c_double), ("eta_nu", C.c_double),
        ("rho0", C.c_double), ("T_ref", C.c_double),
        ("fp16_scale_f", C.c_double), ("fp16_scale_g", C.c_double),
        ("pore_size", C.c_double), ("diag_every", C.c_int32),
    ]


class lbm_ltne_derived(C.Structure):
    _fields_ = [(k, C.c_double) for k in (
        "L", "dT", "cs2", "csT2", "gbeta", "u_c", "nu_f", "nu_e", "s_nu", "tau_nu",
        "alpha_f", "alpha_s", "zeta_a", "eta_a", "tau_Tf", "tau_Ts", "K", "F_phi",
        "l0", "l1", "d0", "d1", "T_ref", "scale_f", "scale_g")]


_ARRAY_KEYS = ("wall_thermal", "T_wall", "body_force")


class LtneError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__("%s: %s (%d)%s" % (where, _strerror(code), code,
                                           (": " + detail) if detail else ""))
        self.code = code


_lib = None


def lib():
    """The loaded HIP library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "HIP library %s is missing; build it with `python -m paper_1608_04118_amd.build` "
                "(there is no CPU fallback)" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        P = C.POINTER(lbm_ltne_params)
        D = C.POINTER(lbm_ltne_derived)
        dp = C.POINTER(C.c_double)
        sig = {
            "lbm_ltne_default_params": ([P], C.c_int),
            "lbm_ltne_derive": ([P, D], C.c_int),
            "lbm_ltne_pool_bytes": ([P, C.c_int, C.c_int], sz),
            "lbm_ltne_create": ([P, vp, vp, vp, vp, vp, vp, sz, C.POINTER(vp)], C.c_int),
            "lbm_ltne_step": ([vp, i64], C.c_int),
            "lbm_ltne_steps_done": ([vp], i64),
            "lbm_ltne_macros": ([vp, vp, vp, vp, vp, vp], C.c_int),
            "lbm_ltne_nusselt": ([vp, dp, dp], C.c_int),
            "lbm_ltne_diagnostics": ([vp, dp, dp, dp], C.c_int),
            "lbm_ltne_adjoint": ([vp, i64, i64, dp, vp, vp], C.c_int),
            "lbm_ltne_state_bytes": ([vp], sz),
            "lbm_ltne_save": ([vp, vp, sz], C.c_int),
            "lbm_ltne_load": ([vp, vp, sz], C.c_int),
            "lbm_ltne_get_derived": ([vp, D], C.c_int),
            "lbm_ltne_destroy": ([vp], C.c_int),
            "lbm_ltne_batch_create": ([i32, P, vp, vp, vp, C.POINTER(vp)], C.c_int),
            "lbm_ltne_batch_step": ([vp, i64], C.c_int),
            "lbm_ltne_batch_steps_done": ([vp], i64),
            "lbm_ltne_batch_macros": ([vp, i32, vp, vp, vp, vp, vp], C.c_int),
            "lbm_ltne_batch_nusselt": ([vp, i32, dp, dp], C.c_int),
            "lbm_ltne_batch_set_mode": ([vp, i32], C.c_int),
            "lbm_ltne_batch_info": ([vp, C.POINTER(i64), C.POINTER(i32), C.POINTER(i32),
                                     C.POINTER(i32)], C.c_int),
            "lbm_ltne_batch_set_tiles": ([vp, vp], C.c_int),
            "lbm_ltne_batch_get_tiles": ([vp, vp], C.c_int),
            "lbm_ltne_batch_autotune": ([vp, i32, dp], C.c_int),
            "lbm_ltne_batch_set_chunks": ([vp, vp], C.c_int),
            "lbm_ltne_batch_get_chunks": ([vp, vp], C.c_int),
            "lbm_ltne_batch_destroy": ([vp], C.c_int),
            "lbm_ltne_strerror": ([C.c_int], C.c_char_p),
            "lbm_ltne_last_error": ([], C.c_char_p),
            "lbm_ltne_abi_version": ([], C.c_int),
            "lbm_ltne_macro_sums_noalloc": ([P, vp, vp, vp, vp, dp, dp, dp], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().lbm_ltne_strerror(code).decode()
    except Exception:  # pragma: no cover - only while reporting another failure
        return "error"


def _check(code: int, where: str):
    if code != LBM_OK:
        raise LtneError(code, where, lib().lbm_ltne_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def params_from_dict(d: dict) -> lbm_ltne_params:
    """Builds the C parameter struct from a dict of its field names; fields
    not in the dict keep the library defaults."""
    p = lbm_ltne_default_params()
    names = {f[0] for f in lbm_ltne_params._fields_}
    for k, v in d.items():
        if k not in names:
            raise KeyError("unknown parameter %r" % k)
        if k in _ARRAY_KEYS:
            getattr(p, k)[:] = list(v)
        else:
            setattr(p, k, v)
    return p


def params_to_dict(p: lbm_ltne_params) -> dict:
    return {k: (tuple(getattr(p, k)) if k in _ARRAY_KEYS else getattr(p, k))
            for k, _ in lbm_ltne_params._fields_}


def _as_params(p) -> lbm_ltne_params:
    return p if isinstance(p, lbm_ltne_params) else params_from_dict(p)


def _field(a, n):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    if a.size != n:
        raise ValueError("field has %d values, lattice has %d nodes" % (a.size, n))
    return a


# --- entry points -----------------------------------------------------------

def lbm_ltne_default_params() -> lbm_ltne_params:
    p = lbm_ltne_params()
    _check(lib().lbm_ltne_default_params(C.byref(p)), "lbm_ltne_default_params")
    return p


def lbm_ltne_derive(p) -> lbm_ltne_derived:
    d = lbm_ltne_derived()
    _check(lib().lbm_ltne_derive(C.byref(_as_params(p)), C.byref(d)), "lbm_ltne_derive")
    return d


def lbm_ltne_pool_bytes(p, has_phi=False, has_Hv=False) -> int:
    return int(lib().lbm_ltne_pool_bytes(C.byref(_as_params(p)), int(has_phi), int(has_Hv)))


def lbm_ltne_create(p, phi_field=None, Hv_field=None, Tf_init=None, Ts_init=None,
                    hip_stream=None, device_pool=None, pool_bytes=0):
    """Returns the handle (a ctypes void pointer).  ``device_pool`` is a raw
    device address (int) or None; ``hip_stream`` a raw hipStream_t or None."""
    p = _as_params(p)
    n = p.nx * p.ny
    keep = [_field(a, n) for a in (phi_field, Hv_field, Tf_init, Ts_init)]
    h = C.c_void_p()
    rc = lib().lbm_ltne_create(C.byref(p), *[_ptr(a) for a in keep],
                               C.c_void_p(hip_stream) if hip_stream else None,
                               C.c_void_p(device_pool) if device_pool else None,
                               int(pool_bytes), C.byref(h))
    _check(rc, "lbm_ltne_create")
    return h


def lbm_ltne_step(h, nsteps: int):
    _check(lib().lbm_ltne_step(h, int(nsteps)), "lbm_ltne_step")


def lbm_ltne_steps_done(h) -> int:
    return int(lib().lbm_ltne_steps_done(h))


def lbm_ltne_macros(h, nx: int, ny: int) -> dict:
    out = {k: np.empty((ny, nx)) for k in ("rho", "ux", "uy", "Tf", "Ts")}
    _check(lib().lbm_ltne_macros(h, *[_ptr(out[k]) for k in ("rho", "ux", "uy", "Tf", "Ts")]),
           "lbm_ltne_macros")
    return out


def lbm_ltne_nusselt(h):
    a, b = C.c_double(), C.c_double()
    _check(lib().lbm_ltne_nusselt(h, C.byref(a), C.byref(b)), "lbm_ltne_nusselt")
    return a.value, b.value


def lbm_ltne_diagnostics(h):
    m, e, r = C.c_double(), C.c_double(), C.c_double()
    _check(lib().lbm_ltne_diagnostics(h, C.byref(m), C.byref(e), C.byref(r)),
           "lbm_ltne_diagnostics")
    return m.value, e.value, r.value


def lbm_ltne_adjoint(h, nx: int, ny: int, nsteps: int, ckpt_every: int = 0):
    """Advances nsteps and returns (loss, dL/dphi, dL/dHv): loss is the mean
    hot-wall Nu_f at the final time, gradients are (ny, nx) float64 arrays."""
    loss = C.c_double()
    gp = np.zeros((ny, nx))
    gh = np.zeros((ny, nx))
    _check(lib().lbm_ltne_adjoint(h, int(nsteps), int(ckpt_every), C.byref(loss), _ptr(gp), _ptr(gh)),
           "lbm_ltne_adjoint")
    return loss.value, gp, gh


def lbm_ltne_state_bytes(h) -> int:
    return int(lib().lbm_ltne_state_bytes(h))


def lbm_ltne_save(h) -> bytearray:
    buf = bytearray(lbm_ltne_state_bytes(h))
    arr = (C.c_char * len(buf)).from_buffer(buf)
    _check(lib().lbm_ltne_save(h, C.cast(arr, C.c_void_p), len(buf)), "lbm_ltne_save")
    return buf


def lbm_ltne_load(h, buf):
    buf = bytearray(buf)
    arr = (C.c_char * len(buf)).from_buffer(buf)
    _check(lib().lbm_ltne_load(h, C.cast(arr, C.c_void_p), len(buf)), "lbm_ltne_load")


def lbm_ltne_get_derived(h) -> lbm_ltne_derived:
    d = lbm_ltne_derived()
    _check(lib().lbm_ltne_get_derived(h, C.byref(d)), "lbm_ltne_get_derived")
    return d


def lbm_ltne_destroy(h):
    _check(lib().lbm_ltne_destroy(h), "lbm_ltne_destroy")


def lbm_ltne_macro_sums_noalloc(p, mac_ptr: int, prev_ptr: int, phi_ptr=None, hip_stream=None):
    """(mass, energy, residual) of caller-held device macro fields (raw
    addresses of 5 planes rho, u_x, u_y, T_f, T_s of nx*ny values each, in
    the compute type of p's precision), with no device allocation."""
    m, e, r = C.c_double(), C.c_double(), C.c_double()
    _check(lib().lbm_ltne_macro_sums_noalloc(C.byref(_as_params(p)), C.c_void_p(mac_ptr), C.c_void_p(prev_ptr),
                                             C.c_void_p(phi_ptr) if phi_ptr else None,
                                             C.c_void_p(hip_stream) if hip_stream else None,
                                             C.byref(m), C.byref(e), C.byref(r)),
           "lbm_ltne_macro_sums_noalloc")
    return m.value, e.value, r.value


def lbm_ltne_strerror(code: int) -> str:
    return lib().lbm_ltne_strerror(code).decode()


def lbm_ltne_last_error() -> str:
    return lib().lbm_ltne_last_error().decode()


def lbm_ltne_abi_version() -> int:
    return int(lib().lbm_ltne_abi_version())


# --- convenience wrapper ------------------------------------------------------

# Live Lattice / Batch objects.  Their handles are released by close(), by
# the garbage collector, or at the latest by the exit hook below, which runs
# while the HIP runtime and torch (whose stream and memory a handle borrows)
# are still alive.  A finalizer that only runs during interpreter teardown
# makes no HIP call: the runtime may already be gone, and the process is
# ending anyway.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for obj in list(_LIVE):
        try:
            obj.close()
        except Exception:
            pass


class Lattice:
    """One lattice on the current torch device and stream.

    Device memory comes from torch's allocator as one uint8 pool handed to the
    library; work is queued on ``torch.cuda.current_stream()`` at creation.
    """

    def __init__(self, params, phi=None, Hv=None, Tf0=None, Ts0=None, use_torch=True):
        self.p = _as_params(params)
        self.nx, self.ny = self.p.nx, self.p.ny
        self._pool = None
        stream = None
        pool = None
        nbytes = 0
        if use_torch:
            import torch
            nbytes = lbm_ltne_pool_bytes(self.p, phi is not None, Hv is not None)
            if nbytes == 0:
                lbm_ltne_derive(self.p)  # raises with the reason
            self._pool = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            pool = self._pool.data_ptr()
            stream = torch.cuda.current_stream().cuda_stream
            self.stream = torch.cuda.current_stream()
        self.h = lbm_ltne_create(self.p, phi, Hv, Tf0, Ts0, stream, pool, nbytes)
        _LIVE.add(self)

    def step(self, n: int = 1) -> "Lattice":
        lbm_ltne_step(self.h, n)
        return self

    @property
    def steps(self) -> int:
        return lbm_ltne_steps_done(self.h)

    def macros(self) -> dict:
        return lbm_ltne_macros(self.h, self.nx, self.ny)

    def nusselt(self):
        return lbm_ltne_nusselt(self.h)

    def diagnostics(self):
        return lbm_ltne_diagnostics(self.h)

    def adjoint(self, nsteps: int, ckpt_every: int = 0):
        """(loss, dL/dphi, dL/dHv) of the mean hot-wall Nu_f after nsteps more
        steps; the lattice advances by nsteps."""
        return lbm_ltne_adjoint(self.h, self.nx, self.ny, nsteps, ckpt_every)

    def save(self) -> bytearray:
        return lbm_ltne_save(self.h)

    def load(self, buf):
        lbm_ltne_load(self.h, buf)

    def derived(self) -> dict:
        d = lbm_ltne_get_derived(self.h)
        return {k: getattr(d, k) for k, _ in d._fields_}

    def close(self):
        if getattr(self, "h", None):
            lbm_ltne_destroy(self.h)
            self.h = None
        self._pool = None

    # The finalizing test is bound at definition: during interpreter teardown
    # this module's globals (sys among them) may already be cleared.
    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


# --- autograd ---------------------------------------------------------------

def _nusselt_function():
    import torch

    class NusseltLoss(torch.autograd.Function):
        """loss = mean hot-wall Nu_f after nsteps of a lattice created with the
        porosity and interphase-coefficient fields (phi, Hv).  The forward runs
        lbm_ltne_adjoint, which produces the loss and both gradients in one
        call (the reverse sweep needs the forward trajectory anyway); the
        backward only scales the stored gradients."""

        @staticmethod
        def forward(ctx, phi, Hv, params, nsteps, ckpt_every):
            lat = Lattice(params, phi=phi.detach().double().cpu().numpy(),
                          Hv=Hv.detach().double().cpu().numpy())
            try:
                loss, gp, gh = lat.adjoint(int(nsteps), int(ckpt_every))
            finally:
                lat.close()
            ctx.save_for_backward(torch.from_numpy(gp).to(phi.device, phi.dtype),
                                  torch.from_numpy(gh).to(Hv.device, Hv.dtype))
            return torch.tensor(loss, dtype=torch.float64, device=phi.device)

        @staticmethod
        def backward(ctx, g):
            gp, gh = ctx.saved_tensors
            s = g.to(gp.dtype)
            return s * gp, s * gh, None, None, None

    return NusseltLoss


_NUSSELT = None


def nusselt_loss(params, phi, Hv, nsteps: int, ckpt_every: int = 0):
    """Differentiable mean hot-wall Nusselt number of the fluid phase after
    nsteps: a torch scalar whose gradient with respect to the (ny, nx) tensors
    phi and Hv comes from the hand-written adjoint (lbm_ltne_adjoint)."""
    global _NUSSELT
    if _NUSSELT is None:
        _NUSSELT = _nusselt_function()
    return _NUSSELT.apply(phi, Hv, params, nsteps, ckpt_every)


# --- batched lattices -----------------------------------------------------------

def lbm_ltne_batch_create(params_list, phi_fields=None, Hv_fields=None, hip_stream=None):
    ps = [_as_params(p) for p in params_list]
    n = len(ps)
    arr = (lbm_ltne_params * n)(*ps)
    keep = []

    def ptrs(fields):
        if fields is None:
            return None
        out = (C.c_void_p * n)()
        for i, f in enumerate(fields):
            if f is not None:
                a = _field(f, ps[i].nx * ps[i].ny)
                keep.append(a)
                out[i] = a.ctypes.data
        return out

    pp, hp = ptrs(phi_fields), ptrs(Hv_fields)
    h = C.c_void_p()
    rc = lib().lbm_ltne_batch_create(n, arr, C.cast(pp, C.c_void_p) if pp is not None else None,
                                     C.cast(hp, C.c_void_p) if hp is not None else None,
                                     C.c_void_p(hip_stream) if hip_stream else None, C.byref(h))
    _check(rc, "lbm_ltne_batch_create")
    return h


def lbm_ltne_batch_step(b, nsteps):
    _check(lib().lbm_ltne_batch_step(b, int(nsteps)), "lbm_ltne_batch_step")


def lbm_ltne_batch_macros(b, i, nx, ny):
    out = {k: np.empty((ny, nx)) for k in ("rho", "ux", "uy", "Tf", "Ts")}
    _check(lib().lbm_ltne_batch_macros(b, int(i), *[_ptr(out[k]) for k in ("rho", "ux", "uy", "Tf", "Ts")]),
           "lbm_ltne_batch_macros")
    return out


def lbm_ltne_batch_nusselt(b, i):
    a, c = C.c_double(), C.c_double()
    _check(lib().lbm_ltne_batch_nusselt(b, int(i), C.byref(a), C.byref(c)), "lbm_ltne_batch_nusselt")
    return a.value, c.value


def lbm_ltne_batch_set_mode(b, persistent):
    _check(lib().lbm_ltne_batch_set_mode(b, int(persistent)), "lbm_ltne_batch_set_mode")


def lbm_ltne_batch_info(b):
    n, t, g, m = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().lbm_ltne_batch_info(b, C.byref(n), C.byref(t), C.byref(g), C.byref(m)),
           "lbm_ltne_batch_info")
    return dict(nodes=n.value, tiles=t.value, grid=g.value, persistent=m.value)


def lbm_ltne_batch_set_tiles(b, shifts):
    a = np.ascontiguousarray(np.asarray(shifts, dtype=np.int32))
    _check(lib().lbm_ltne_batch_set_tiles(b, _ptr(a)), "lbm_ltne_batch_set_tiles")


def lbm_ltne_batch_get_tiles(b, n):
    a = np.zeros(n, dtype=np.int32)
    _check(lib().lbm_ltne_batch_get_tiles(b, _ptr(a)), "lbm_ltne_batch_get_tiles")
    return a


def lbm_ltne_batch_set_chunks(b, rows):
    a = np.ascontiguousarray(np.asarray(rows, dtype=np.int32))
    _check(lib().lbm_ltne_batch_set_chunks(b, _ptr(a)), "lbm_ltne_batch_set_chunks")


def lbm_ltne_batch_get_chunks(b, n):
    a = np.zeros(n, dtype=np.int32)
    _check(lib().lbm_ltne_batch_get_chunks(b, _ptr(a)), "lbm_ltne_batch_get_chunks")
    return a


def lbm_ltne_batch_autotune(b, reps=4):
    ms = C.c_double()
    _check(lib().lbm_ltne_batch_autotune(b, int(reps), C.byref(ms)), "lbm_ltne_batch_autotune")
    return ms.value


def lbm_ltne_batch_destroy(b):
    _check(lib().lbm_ltne_batch_destroy(b), "lbm_ltne_batch_destroy")


class Batch:
    """Many independent lattices advanced together on the current torch
    stream: one launch per step (two steps per launch for the FP32 form when
    the batch is large enough) by default, or one persistent launch
    (set_mode(1))."""

    def __init__(self, params_list, phi_fields=None, Hv_fields=None, use_torch=True):
        self.ps = [_as_params(p) for p in params_list]
        stream = None
        if use_torch:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
            self.stream = torch.cuda.current_stream()
        self.h = lbm_ltne_batch_create(self.ps, phi_fields, Hv_fields, stream)
        _LIVE.add(self)

    def __len__(self):
        return len(self.ps)

    def step(self, n=1):
        lbm_ltne_batch_step(self.h, n)
        return self

    def macros(self, i):
        return lbm_ltne_batch_macros(self.h, i, self.ps[i].nx, self.ps[i].ny)

    def nusselt(self, i):
        return lbm_ltne_batch_nusselt(self.h, i)

    def set_mode(self, persistent):
        lbm_ltne_batch_set_mode(self.h, persistent)

    def info(self):
        return lbm_ltne_batch_info(self.h)

    def tiles(self):
        return lbm_ltne_batch_get_tiles(self.h, len(self.ps))

    def set_tiles(self, shifts):
        lbm_ltne_batch_set_tiles(self.h, shifts)

    def chunks(self):
        return lbm_ltne_batch_get_chunks(self.h, len(self.ps))

    def set_chunks(self, rows):
        lbm_ltne_batch_set_chunks(self.h, rows)

    def autotune(self, reps=4, cache=None):
        """Tile widths and two-step chunk heights per size class, then the
        launch mode of the whole batch.  With ``cache`` (a JSON path), a
        choice stored for this device, precision and lattice width is reused
        and new choices are added; the key is "gfx950/<precision>/<nx>", the
        value {"tile": log2 width, "rows": chunk height}.  The launch mode
        depends on the whole batch and is not cached: a cache hit keeps the
        current mode."""
        import json
        key = lambda p: "gfx950/%d/%d" % (p.precision, p.nx)
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if table and all(isinstance(table.get(key(p)), dict) for p in self.ps):
            self.set_tiles([table[key(p)]["tile"] for p in self.ps])
            self.set_chunks([table[key(p)]["rows"] for p in self.ps])
            return None
        ms = lbm_ltne_batch_autotune(self.h, reps)
        if cache:
            for p, sh, rows in zip(self.ps, self.tiles(), self.chunks()):
                table[key(p)] = {"tile": int(sh), "rows": int(rows)}
            d = os.path.dirname(os.path.abspath(cache))
            os.makedirs(d, exist_ok=True)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        return ms

    def close(self):
        if getattr(self, "h", None):
            lbm_ltne_batch_destroy(self.h)
            self.h = None

    # The finalizing test is bound at definition: during interpreter teardown
    # this module's globals (sys among them) may already be cleared.
    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

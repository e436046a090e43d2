"""Python binding of libfld, the MI355X flux-limited diffusion solver.

Argument marshalling only: every step of the solve runs in the HIP kernels
of ``libfld.so`` (built by ``paper_1403_8105_amd/build.py``).  The functions
carry the names of the C ABI in ``include/fld.h``; ``Solver`` and ``Batch``
are thin conveniences over them.  Host arrays are numpy float64 C-contiguous
[nx][ny][nz] (z fastest); device arrays are passed as raw pointers (for
example ``torch_tensor.data_ptr()``).  There is no CPU fallback: a missing
library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfld.so")

FLD_OK, FLD_ERR_INVALID_ARGUMENT, FLD_ERR_OUT_OF_MEMORY, FLD_ERR_DEVICE = 0, 1, 2, 3
FLD_ERR_NOT_CONVERGED, FLD_ERR_DIVERGED, FLD_ERR_STATE = 4, 5, 6
LIMITERS = {"cda": 0, "lp": 1, "sum": 2, "max": 3, "kershaw": 4, "larsen": 5}
METHODS = {"rbsor": 0, "alg1": 0, "mg": 1}
PRECISIONS = {"fp64": 0, "mixed": 1}

_dp = C.POINTER(C.c_double)


class fld_options(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("limiter", C.c_int), ("larsen_n", C.c_double),
                ("eps", C.c_double), ("sigma_eps", C.c_double), ("phi_b", C.c_double),
                ("boundary_d", C.c_int), ("method", C.c_int), ("precision", C.c_int),
                ("omega", C.c_double), ("omega_s", C.c_double), ("nu1", C.c_int),
                ("nu2", C.c_int), ("max_coarsest", C.c_int), ("max_iters", C.c_int),
                ("tol", C.c_double), ("check_every", C.c_int), ("device", C.c_int),
                ("stream", C.c_void_p), ("timing", C.c_int), ("deflate_tau", C.c_double),
                ("graph", C.c_int), ("task_cells0", C.c_int), ("coarse_blocks", C.c_int),
                ("colour_split", C.c_int), ("restart_growth", C.c_double),
                ("corr_scale", C.c_double), ("anisotropy_g", C.c_double),
                ("deep_cells", C.c_int), ("nested_tol", C.c_double), ("aa_m", C.c_int),
                ("aa_reg", C.c_double), ("fuse_lr", C.c_int),
                ("fuse_rb", C.c_int), ("debug_nan_iter", C.c_int),
                ("nu_coarse", C.c_int), ("coarse_from", C.c_int), ("nested_inherit", C.c_int)]


class fld_report(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("status", C.c_int), ("iterations", C.c_int),
                ("rel", C.c_double), ("rel_sweep", C.c_double), ("history", _dp),
                ("history_cap", C.c_int), ("history_len", C.c_int), ("time_ms", C.c_double),
                ("voxel_updates", C.c_double), ("bytes", C.c_double),
                ("kernel_ms", C.c_double * 4), ("kernel_launches", C.c_double * 4),
                ("kernel_bytes", C.c_double * 4), ("nested_iterations", C.c_int)]


class FldError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_name(status)}: {msg}")
        self.status = status


_lib = None
_lib_loaded_from = None
EXPORTS = ["fld_default_options", "fld_create", "fld_set_medium", "fld_set_medium_device",
           "fld_solve", "fld_solve_device", "fld_solve_resume", "fld_residual",
           "fld_residual_device", "fld_destroy", "fld_status_string", "fld_last_error",
           "fld_batch_create", "fld_batch_set_volume", "fld_batch_solve", "fld_batch_destroy",
           "fld_batch_last_error", "fld_device_arch", "fld_light_bake", "fld_render",
           "fld_residual_device_noalloc"]


def lib():
    """Load libfld.so (raises if it has not been built).

    A process uses one build of the library: a context belongs to the copy
    that created it, and handing it to a second copy (another path) would
    run that copy's code on the first copy's objects.  Asking for another
    path after the first load raises."""
    global _lib, _lib_loaded_from
    if _lib is not None and _lib_loaded_from != LIB_PATH:
        raise RuntimeError(f"libfld.so is already loaded from {_lib_loaded_from}; "
                           f"load {LIB_PATH} in another process")
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_1403_8105_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, ip = C.c_void_p, C.POINTER(C.c_int)
        L.fld_default_options.argtypes = [C.POINTER(fld_options)]
        L.fld_device_arch.argtypes = [C.c_int, C.c_char_p, C.c_int]
        L.fld_light_bake.argtypes = [vp, vp, C.c_double, C.c_int, C.c_int, C.c_int, C.c_double,
                                     vp, vp]
        L.fld_render.argtypes = [vp, vp, vp, vp, C.c_double, C.c_int, C.c_int, C.c_int,
                                 C.c_double, vp, vp]
        L.fld_create.argtypes = [C.POINTER(fld_options), C.c_int, C.c_int, C.c_int, C.c_double,
                                 C.POINTER(vp)]
        L.fld_set_medium.argtypes = [vp, vp, vp, vp]
        L.fld_set_medium_device.argtypes = [vp, vp, vp, vp, vp]
        L.fld_solve.argtypes = [vp, vp, vp, C.POINTER(fld_report)]
        L.fld_solve_device.argtypes = [vp, vp, vp, C.c_int, C.POINTER(fld_report)]
        L.fld_solve_resume.argtypes = [vp, vp, C.POINTER(fld_report)]
        L.fld_residual.argtypes = [vp, vp, vp, _dp]
        L.fld_residual_device.argtypes = [vp, vp, vp, _dp]
        L.fld_residual_device_noalloc.argtypes = [vp, vp, vp, _dp]
        L.fld_destroy.argtypes = [vp]
        L.fld_destroy.restype = None
        L.fld_status_string.argtypes = [C.c_int]
        L.fld_status_string.restype = C.c_char_p
        L.fld_last_error.argtypes = [vp]
        L.fld_last_error.restype = C.c_char_p
        L.fld_batch_create.argtypes = [C.POINTER(fld_options), C.c_int, ip, _dp, C.c_int,
                                       C.POINTER(vp)]
        L.fld_batch_set_volume.argtypes = [vp, C.c_int, vp, C.POINTER(vp), C.POINTER(vp)]
        L.fld_batch_solve.argtypes = [vp, C.POINTER(vp), ip, C.POINTER(fld_report)]
        L.fld_batch_destroy.argtypes = [vp]
        L.fld_batch_destroy.restype = None
        L.fld_batch_last_error.argtypes = [vp]
        L.fld_batch_last_error.restype = C.c_char_p
        _lib, _lib_loaded_from = L, LIB_PATH
    return _lib


def status_name(s: int) -> str:
    try:
        return lib().fld_status_string(int(s)).decode()
    except Exception:  # noqa: BLE001 - naming a status must never raise
        return f"status {s}"


def _host(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.c_void_p)


# ---- C-ABI functions (same names) ----------------------------------------

def fld_default_options(**overrides) -> fld_options:
    o = fld_options()
    lib().fld_default_options(C.byref(o))
    for k, v in overrides.items():
        if k == "limiter" and isinstance(v, str):
            v = LIMITERS[v]
        elif k == "method" and isinstance(v, str):
            v = METHODS[v]
        elif k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        elif k == "boundary_d" and isinstance(v, str):
            v = {"paper": 0, "mirror": 1}[v]
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def fld_create(opts: fld_options, nx: int, ny: int, nz: int, h: float):
    ctx = C.c_void_p()
    s = lib().fld_create(C.byref(opts), nx, ny, nz, h, C.byref(ctx))
    if s != FLD_OK:
        raise FldError(s, lib().fld_last_error(None).decode())
    return ctx


def fld_last_error(ctx) -> str:
    return lib().fld_last_error(ctx).decode()


def _check(ctx, s, ok=(FLD_OK,)):
    if s not in ok:
        raise FldError(s, fld_last_error(ctx))
    return s


def fld_set_medium(ctx, sigma_t, albedo, Q):
    (a, pa), (b, pb), (c, pc) = _host(sigma_t), _host(albedo), _host(Q)
    return _check(ctx, lib().fld_set_medium(ctx, pa, pb, pc))


def fld_set_medium_device(ctx, d_sigma_t: int, d_albedo: int, d_Q: int, stream: int = 0):
    return _check(ctx, lib().fld_set_medium_device(ctx, d_sigma_t, d_albedo, d_Q, stream or None))


def _report(cap=100000):
    rep = fld_report()
    rep.struct_size = C.sizeof(fld_report)
    hist = np.zeros(cap)
    rep.history = hist.ctypes.data_as(_dp)
    rep.history_cap = cap
    return rep, hist


def _report_dict(rep, hist):
    return {"status": rep.status, "iterations": rep.iterations, "rel": rep.rel,
            "rel_sweep": rep.rel_sweep, "history": hist[:min(rep.history_len, len(hist))].copy(),
            "time_ms": rep.time_ms, "voxel_updates": rep.voxel_updates,
            "kernel_ms": list(rep.kernel_ms), "kernel_launches": list(rep.kernel_launches),
            "kernel_bytes": list(rep.kernel_bytes), "nested_iterations": rep.nested_iterations}


def fld_solve(ctx, shape, phi_init=None, allow=(FLD_OK, FLD_ERR_NOT_CONVERGED)):
    """Host solve; returns (phi, report dict)."""
    phi = np.empty(shape)
    pi = None
    if phi_init is not None:
        phi_init, pi = _host(phi_init)
    rep, hist = _report()
    s = lib().fld_solve(ctx, pi, phi.ctypes.data_as(C.c_void_p), C.byref(rep))
    _check(ctx, s, allow)
    return phi, _report_dict(rep, hist)


def fld_solve_resume(ctx, shape, allow=(FLD_OK, FLD_ERR_NOT_CONVERGED)):
    phi = np.empty(shape)
    rep, hist = _report()
    s = lib().fld_solve_resume(ctx, phi.ctypes.data_as(C.c_void_p), C.byref(rep))
    _check(ctx, s, allow)
    return phi, _report_dict(rep, hist)


def fld_solve_device(ctx, d_phi_out: int, d_phi_init: int = 0, resume: int = 0,
                     allow=(FLD_OK, FLD_ERR_NOT_CONVERGED)):
    rep, hist = _report()
    s = lib().fld_solve_device(ctx, d_phi_init or None, d_phi_out or None, resume, C.byref(rep))
    _check(ctx, s, allow)
    return _report_dict(rep, hist)


def fld_residual(ctx, shape, phi=None, want_r=True):
    pp = None
    if phi is not None:
        phi, pp = _host(phi)
    r = np.empty(shape) if want_r else None
    rel = C.c_double()
    s = lib().fld_residual(ctx, pp, r.ctypes.data_as(C.c_void_p) if want_r else None,
                           C.byref(rel))
    _check(ctx, s)
    return r, rel.value


def fld_residual_device(ctx, d_phi: int = 0, d_r_out: int = 0):
    rel = C.c_double()
    _check(ctx, lib().fld_residual_device(ctx, d_phi or None, d_r_out or None, C.byref(rel)))
    return rel.value


def fld_residual_device_noalloc(ctx, d_phi: int = 0, d_r_out: int = 0):
    """fld_residual_device without device allocations (fixed per-GPU scratch)."""
    rel = C.c_double()
    _check(ctx, lib().fld_residual_device_noalloc(ctx, d_phi or None, d_r_out or None,
                                                  C.byref(rel)))
    return rel.value


def fld_destroy(ctx):
    lib().fld_destroy(ctx)


def fld_device_arch(device: int = 0) -> str:
    """GPU architecture name of a device, e.g. "gfx950"."""
    buf = C.create_string_buffer(64)
    s = lib().fld_device_arch(device, buf, 64)
    if s != FLD_OK:
        raise FldError(s, f"fld_device_arch({device})")
    return buf.value.decode()


def fld_light_bake(d_sigma_t: int, d_albedo: int, light: float, shape, h: float, d_q: int,
                   stream: int = 0):
    """Bake q = light * albedo * sigma_t * T on the device (light along +z)."""
    nx, ny, nz = shape
    s = lib().fld_light_bake(d_sigma_t or None, d_albedo or None, float(light), nx, ny, nz,
                             float(h), d_q or None, stream or None)
    if s != FLD_OK:
        raise FldError(s, "fld_light_bake")


def fld_render(d_sigma_t: int, d_albedo: int, d_src: int, d_phi: int, background: float, shape,
               h: float, d_image: int, stream: int = 0):
    """Ray-march the (nx, ny) image of an orthographic camera along +z on the device."""
    nx, ny, nz = shape
    s = lib().fld_render(d_sigma_t or None, d_albedo or None, d_src or None, d_phi or None,
                         float(background), nx, ny, nz, float(h), d_image or None, stream or None)
    if s != FLD_OK:
        raise FldError(s, "fld_render")


def fld_status_string(s: int) -> str:
    return status_name(s)


def fld_batch_create(opts, dims, hs, nchan):
    dims = np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(-1))
    hs = np.ascontiguousarray(np.asarray(hs, dtype=np.float64))
    b = C.c_void_p()
    s = lib().fld_batch_create(C.byref(opts), len(hs), dims.ctypes.data_as(C.POINTER(C.c_int)),
                               hs.ctypes.data_as(_dp), nchan, C.byref(b))
    if s != FLD_OK:
        raise FldError(s, lib().fld_batch_last_error(None).decode())
    return b


def fld_batch_set_volume(b, v, sigma_t, albedos, Qs):
    st, pst = _host(sigma_t)
    al = [_host(a) for a in albedos]
    qs = [_host(q) for q in Qs]
    pa = (C.c_void_p * len(al))(*[p for _, p in al])
    pq = (C.c_void_p * len(qs))(*[p for _, p in qs])
    s = lib().fld_batch_set_volume(b, v, pst, pa, pq)
    if s != FLD_OK:
        raise FldError(s, lib().fld_batch_last_error(b).decode())


def fld_batch_solve(b, shapes, allow=(FLD_OK, FLD_ERR_NOT_CONVERGED), want_phi=True):
    outs = [np.empty(sh) for sh in shapes] if want_phi else []
    ptrs = (C.c_void_p * len(shapes))(*[o.ctypes.data_as(C.c_void_p) for o in outs]) \
        if want_phi else None
    iters = np.zeros(len(shapes), dtype=np.int32)
    rep, hist = _report()
    s = lib().fld_batch_solve(b, ptrs, iters.ctypes.data_as(C.POINTER(C.c_int)), C.byref(rep))
    if s not in allow:
        raise FldError(s, lib().fld_batch_last_error(b).decode())
    return outs, iters, _report_dict(rep, hist)


def fld_batch_destroy(b):
    lib().fld_batch_destroy(b)


# ---- conveniences -----------------------------------------------------------

class Solver:
    """One volume: ``Solver(shape, h, **options)``, ``set_medium``, ``solve``."""

    def __init__(self, shape, h, **options):
        self.shape = tuple(int(x) for x in shape)
        self._L = lib()              # the copy of the library that owns the context
        self.opts = fld_default_options(**options)
        self.ctx = fld_create(self.opts, *self.shape, float(h))

    def set_medium(self, sigma_t, albedo, Q):
        fld_set_medium(self.ctx, sigma_t, albedo, Q)

    def set_medium_device(self, d_sigma_t, d_albedo, d_Q, stream=0):
        fld_set_medium_device(self.ctx, d_sigma_t, d_albedo, d_Q, stream)

    def solve(self, phi_init=None, **kw):
        return fld_solve(self.ctx, self.shape, phi_init, **kw)

    def resume(self, **kw):
        return fld_solve_resume(self.ctx, self.shape, **kw)

    def residual(self, phi=None):
        return fld_residual(self.ctx, self.shape, phi)

    def close(self):
        if self.ctx:
            self._L.fld_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

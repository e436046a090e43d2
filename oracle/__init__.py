"""FP64 CPU oracle for the flux-limited diffusion solve -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it.  The arithmetic lives in ``fldo.c`` (plain C, FP64);
this module only marshals numpy arrays through ctypes.

Every array is C-contiguous float64 of shape (nx, ny, nz), z fastest.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

LIMITERS = {"cda": 0, "lp": 1, "sum": 2, "max": 3, "kershaw": 4, "larsen": 5}
METHODS = {"alg1": 0, "mg": 1}
STATUS = {0: "converged", 1: "invalid", 4: "not_converged", 5: "diverged"}
MAX_LEVELS = 16

_dp = C.POINTER(C.c_double)


class Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("h", C.c_double),
                ("limiter", C.c_int), ("larsen_n", C.c_double), ("eps", C.c_double),
                ("sigma_eps", C.c_double), ("phi_b", C.c_double), ("mirror_d", C.c_int),
                ("ghost_phi", _dp), ("jbar", C.c_double), ("jnorm", C.c_double),
                ("aniso_g", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("method", C.c_int), ("omega", C.c_double), ("omega_s", C.c_double),
                ("nu1", C.c_int), ("nu2", C.c_int), ("max_coarsest", C.c_int),
                ("max_iters", C.c_int), ("tol", C.c_double), ("check_every", C.c_int),
                ("theta", C.c_double), ("step_mode", C.c_int), ("deflate_tau", C.c_double),
                ("restart_growth", C.c_double), ("corr_scale", C.c_double),
                ("aa_m", C.c_int), ("aa_reg", C.c_double), ("nu_coarse", C.c_int),
                ("coarse_from", C.c_int)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("rel", C.c_double),
                ("rel_sweep", C.c_double), ("history_len", C.c_int)]


_lib = None


def lib():
    """Load ``libfldo.so``, building it first if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.POINTER
        L.fldo_limiter.restype = C.c_double
        L.fldo_limiter.argtypes = [C.c_int, C.c_double, C.c_double]
        L.fldo_limiter_array.argtypes = [C.c_int, C.c_double, _dp, _dp, C.c_long]
        L.fldo_setup.argtypes = [P(Params), _dp, _dp, _dp, _dp, _dp]
        L.fldo_init_state.argtypes = [P(Params), _dp, _dp]
        L.fldo_knudsen.argtypes = [P(Params), _dp, _dp, _dp]
        L.fldo_limiter_pass.argtypes = [P(Params), _dp, _dp, _dp]
        L.fldo_residual.restype = C.c_double
        L.fldo_residual.argtypes = [P(Params), _dp, _dp, _dp, _dp, _dp]
        L.fldo_nonlinear_residual.restype = C.c_double
        L.fldo_nonlinear_residual.argtypes = [P(Params), _dp, _dp, _dp, _dp, _dp, _dp]
        L.fldo_alg1_iteration.restype = C.c_double
        L.fldo_alg1_iteration.argtypes = [P(Params), C.c_double, _dp, _dp, _dp, _dp, _dp]
        L.fldo_mg_levels.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P(C.c_int), C.c_int]
        L.fldo_cholesky_factor.argtypes = [C.c_int, _dp]
        L.fldo_cholesky_solve.argtypes = [C.c_int, _dp, _dp, _dp]
        L.fldo_linear_vcycle.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                         C.c_int, P(SolveOpts), _dp, _dp, _dp, _dp]
        L.fldo_level_residual.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                          C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.fldo_coarse_apply.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                        C.c_int, _dp, _dp, _dp, _dp]
        L.fldo_clusters.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, _dp, C.c_double,
                                    C.POINTER(C.c_int)]
        L.fldo_solve.argtypes = [P(Params), P(SolveOpts), _dp, _dp, _dp, _dp, _dp, _dp, C.c_int,
                                 P(Result)]
        L.fldo_light_bake.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, _dp, _dp,
                                      _dp]
        L.fldo_render.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, _dp, _dp, _dp,
                                  _dp, _dp]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# Limiters (Table 2)
# --------------------------------------------------------------------------

def limiter(kind: str, R, larsen_n: float = 2.0):
    """F(R) for the named limiter, elementwise."""
    R = _f64(np.atleast_1d(R))
    F = np.empty_like(R)
    lib().fldo_limiter_array(LIMITERS[kind], float(larsen_n), _ptr(R), _ptr(F), R.size)
    return F


# --------------------------------------------------------------------------
# Problem set-up
# --------------------------------------------------------------------------

@dataclass
class Problem:
    """A medium after Algorithm 1's set-up (clamped extinction, absorption, RMS emission)."""
    params: Params
    sig_hat: np.ndarray
    sig_a: np.ndarray
    j: np.ndarray
    shape: tuple

    @property
    def jbar(self):
        return self.params.jbar

    @property
    def jnorm(self):
        return self.params.jnorm

    @property
    def sigma_eps(self):
        return self.params.sigma_eps

    def init_state(self):
        phi = np.empty(self.shape)
        D = np.empty(self.shape)
        lib().fldo_init_state(C.byref(self.params), _ptr(phi), _ptr(D))
        return phi, D


def setup(sigma_t, albedo, Q, h, limiter: str = "lp", larsen_n: float = 2.0, eps: float = 1e-20,
          sigma_eps: float = -1.0, phi_b: float = 0.0, mirror_d: bool = False,
          ghost_phi=None, aniso_g: float = 0.0) -> Problem:
    sigma_t, albedo, Q = _f64(sigma_t), _f64(albedo), _f64(Q)
    nx, ny, nz = sigma_t.shape
    assert albedo.shape == sigma_t.shape == Q.shape
    p = Params(nx, ny, nz, float(h), LIMITERS[limiter], float(larsen_n), float(eps),
               float(sigma_eps), float(phi_b), int(mirror_d), None, 0.0, 0.0, float(aniso_g))
    if ghost_phi is not None:
        ghost_phi = _f64(ghost_phi)
        assert ghost_phi.shape == (nx + 2, ny + 2, nz + 2)
        p.ghost_phi = _ptr(ghost_phi)
    sig_hat = np.empty_like(sigma_t)
    sig_a = np.empty_like(sigma_t)
    lib().fldo_setup(C.byref(p), _ptr(sigma_t), _ptr(albedo), _ptr(Q), _ptr(sig_hat), _ptr(sig_a))
    prob = Problem(p, sig_hat, sig_a, Q.copy(), (nx, ny, nz))
    prob._ghost_keepalive = ghost_phi
    return prob


# --------------------------------------------------------------------------
# Point operations over a whole field
# --------------------------------------------------------------------------

def knudsen(prob: Problem, phi):
    phi = _f64(phi)
    R = np.empty_like(phi)
    lib().fldo_knudsen(C.byref(prob.params), _ptr(phi), _ptr(prob.sig_hat), _ptr(R))
    return R


def limiter_pass(prob: Problem, phi):
    phi = _f64(phi)
    D = np.empty_like(phi)
    lib().fldo_limiter_pass(C.byref(prob.params), _ptr(phi), _ptr(prob.sig_hat), _ptr(D))
    return D


def residual(prob: Problem, phi, D):
    """Residual field for a given D, and its 2-norm."""
    phi, D = _f64(phi), _f64(D)
    r = np.empty_like(phi)
    nr = lib().fldo_residual(C.byref(prob.params), _ptr(phi), _ptr(D), _ptr(prob.sig_a),
                             _ptr(prob.j), _ptr(r))
    return r, nr


def nonlinear_residual(prob: Problem, phi):
    """(r, rel, D): D from phi for every voxel, r = j - A(D) phi, rel = ||r||/||j||."""
    phi = _f64(phi)
    r = np.empty_like(phi)
    D = np.empty_like(phi)
    nr = lib().fldo_nonlinear_residual(C.byref(prob.params), _ptr(phi), _ptr(prob.sig_hat),
                                       _ptr(prob.sig_a), _ptr(prob.j), _ptr(D), _ptr(r))
    rel = nr / prob.jnorm if prob.jnorm > 0 else 0.0
    return r, rel, D


def alg1_iteration(prob: Problem, phi, D, omega: float = 1.0):
    """One red+black iteration of Algorithm 1 in place; returns R-bar/j-bar of the sweep."""
    assert phi.dtype == np.float64 and D.dtype == np.float64
    s = lib().fldo_alg1_iteration(C.byref(prob.params), float(omega), _ptr(phi), _ptr(D),
                                  _ptr(prob.sig_hat), _ptr(prob.sig_a), _ptr(prob.j))
    return float(np.sqrt(s / phi.size) / prob.jbar)


# --------------------------------------------------------------------------
# Multigrid helpers (test hooks)
# --------------------------------------------------------------------------

def mg_levels(nx, ny, nz, max_coarsest: int = 512):
    dims = (C.c_int * (3 * MAX_LEVELS))()
    L = lib().fldo_mg_levels(nx, ny, nz, max_coarsest, dims, MAX_LEVELS)
    n = abs(L)
    out = [(dims[3 * q], dims[3 * q + 1], dims[3 * q + 2]) for q in range(min(n, MAX_LEVELS))]
    return out, L > 0


def level_residual(D, sa, b, e, h, d_ghost, mirror=False):
    D, sa, b, e = _f64(D), _f64(sa), _f64(b), _f64(e)
    r = np.empty_like(e)
    nx, ny, nz = e.shape
    lib().fldo_level_residual(nx, ny, nz, float(h), float(d_ghost), int(mirror), _ptr(D),
                              _ptr(sa), _ptr(b), _ptr(e), _ptr(r))
    return r


def coarse_apply(D, sa, x1, h, d_ghost, mirror=False):
    """A_1 x1 for the Galerkin level-1 operator built from finest (D, sa)."""
    D, sa, x1 = _f64(D), _f64(sa), _f64(x1)
    out = np.empty_like(x1)
    nx, ny, nz = D.shape
    if lib().fldo_coarse_apply(nx, ny, nz, float(h), float(d_ghost), int(mirror), _ptr(D),
                               _ptr(sa), _ptr(x1), _ptr(out)) != 0:
        raise ValueError("grid not coarsenable")
    return out


def clusters(prob: Problem, tau: float = 1.0):
    """Cluster labels (-1 outside clusters) and the number of clusters."""
    nx, ny, nz = prob.shape
    lab = np.empty(prob.shape, dtype=np.int32)
    K = lib().fldo_clusters(nx, ny, nz, prob.params.h, _ptr(prob.sig_hat), float(tau),
                            lab.ctypes.data_as(C.POINTER(C.c_int)))
    return lab, K


def solve_opts(method="mg", omega=1.0, omega_s=1.0, nu1=2, nu2=2, max_coarsest=512,
               max_iters=1000, tol=1e-6, check_every=1, theta=1.0,
               step="optimal", deflate_tau=1.0, restart_growth=2.0,
               corr_scale=1.0, aa_m=0, aa_reg=1e-10, nu_coarse=0, coarse_from=2) -> SolveOpts:
    if not 0 <= aa_m <= 16:
        raise ValueError("aa_m must lie in [0, 16]")
    if nu_coarse < 0 or coarse_from < 1:
        raise ValueError("nu_coarse must be >= 0 and coarse_from >= 1")
    return SolveOpts(METHODS[method], float(omega), float(omega_s), int(nu1), int(nu2),
                     int(max_coarsest), int(max_iters), float(tol), int(check_every),
                     float(theta), {"fixed": 0, "optimal": 1, "optimal-norestart": 2}[step],
                     float(deflate_tau), float(restart_growth), float(corr_scale), int(aa_m),
                     float(aa_reg), int(nu_coarse), int(coarse_from))


def linear_vcycle(D, sa, b, h, d_ghost, mirror=False, **kw):
    D, sa, b = _f64(D), _f64(sa), _f64(b)
    e = np.zeros_like(b)
    nx, ny, nz = b.shape
    o = solve_opts(**kw)
    rc = lib().fldo_linear_vcycle(nx, ny, nz, float(h), float(d_ghost), int(mirror), C.byref(o),
                                  _ptr(D), _ptr(sa), _ptr(b), _ptr(e))
    if rc != 0:
        raise ValueError(f"linear_vcycle failed ({rc})")
    return e


def cholesky(M):
    """Dense Cholesky factor (lower) of an SPD matrix."""
    Lf = _f64(M).copy()
    n = Lf.shape[0]
    if lib().fldo_cholesky_factor(n, _ptr(Lf)) != 0:
        raise np.linalg.LinAlgError("not positive definite")
    return np.tril(Lf)


def light_bake(sigma_t, albedo, h, light=1.0):
    """Single-scatter source q = L sigma_s T of a directional light travelling
    +z (Sec. 3 deep shadow map; midpoint transmittance, reading A17)."""
    st = _f64(sigma_t)
    al = _f64(np.broadcast_to(albedo, st.shape))
    q = np.empty_like(st)
    nx, ny, nz = st.shape
    lib().fldo_light_bake(nx, ny, nz, float(h), float(light), _ptr(st), _ptr(al), _ptr(q))
    return q


def render(sigma_t, albedo, src, phi, h, background=0.0):
    """Primary ray-march image (nx, ny) of an orthographic camera along +z
    (Sec. 3 primary ray-march; source 4 pi Q = src + sigma_s phi)."""
    st = _f64(sigma_t)
    al = _f64(np.broadcast_to(albedo, st.shape))
    sr, ph = _f64(src), _f64(phi)
    nx, ny, nz = st.shape
    img = np.empty((nx, ny))
    lib().fldo_render(nx, ny, nz, float(h), float(background), _ptr(st), _ptr(al), _ptr(sr),
                      _ptr(ph), _ptr(img))
    return img


def cholesky_solve(M, rhs):
    Lf = _f64(M).copy()
    n = Lf.shape[0]
    if lib().fldo_cholesky_factor(n, _ptr(Lf)) != 0:
        raise np.linalg.LinAlgError("not positive definite")
    rhs = _f64(rhs)
    x = np.empty_like(rhs)
    lib().fldo_cholesky_solve(n, _ptr(Lf), _ptr(rhs), _ptr(x))
    return x


# --------------------------------------------------------------------------
# Solvers
# --------------------------------------------------------------------------

@dataclass
class SolveResult:
    phi: np.ndarray
    D: np.ndarray
    status: str
    iterations: int
    rel: float
    rel_sweep: float
    history: np.ndarray
    nested_iterations: int = 0


def nested_problem(prob: Problem) -> Problem:
    """The 2:1 coarser problem of grid sequencing (our design; the paper has no
    multigrid): coarse cell C averages its 8 children, sigma_t = mean(sig_hat),
    Q = mean(j), albedo = 1 - mean(sig_a)/mean(sig_hat) (so the absorption is
    the mean of the fine one), voxel size 2h; the other parameters as given."""
    nx, ny, nz = prob.shape
    assert nx % 2 == 0 and ny % 2 == 0 and nz % 2 == 0, "grid sequencing needs even axes"

    def mean8(a):
        b = a.reshape(nx // 2, 2, ny // 2, 2, nz // 2, 2)
        acc = np.zeros((nx // 2, ny // 2, nz // 2))
        for di in range(2):
            for dj in range(2):
                for dk in range(2):
                    acc = acc + b[:, di, :, dj, :, dk]
        return acc / 8.0

    s, a, q = mean8(prob.sig_hat), mean8(prob.sig_a), mean8(prob.j)
    albedo = np.clip(1.0 - a / s, 0.0, 1.0)
    pr = prob.params
    inv = {v: k for k, v in LIMITERS.items()}
    return setup(s, albedo, q, 2.0 * pr.h, limiter=inv[pr.limiter], larsen_n=pr.larsen_n,
                 eps=pr.eps, sigma_eps=pr.sigma_eps, phi_b=pr.phi_b, mirror_d=bool(pr.mirror_d))


def solve(prob: Problem, method: str = "mg", phi=None, D=None, hist_cap: int = 100000,
          nested_tol: float = 0.0, nested_inherit: bool = False, **kw):
    """Run Algorithm 1 (method='alg1') or Picard-multigrid (method='mg').

    phi/D: start state (default: the paper's initialisation).  Returns the
    final state and the relative-residual history (one entry per check).
    nested_tol > 0 (multigrid from the paper's initialisation): grid
    sequencing -- first solve nested_problem(prob) with the default schedule
    (nested_inherit: with this solve's schedule, the coarse-level sweeps one
    level up) to nested_tol (at most 10000 iterations) and start from its
    fluence, constant over each 2x2x2 block;
    the result's ``nested_iterations`` counts the coarse iterations.
    """
    if nested_tol > 0.0 and phi is None and method == "mg":
        coarse = nested_problem(prob)
        ck = {k: kw[k] for k in ("deflate_tau", "max_coarsest") if k in kw}
        if nested_inherit:
            ck.update({k: kw[k] for k in ("nu1", "nu2", "omega_s", "corr_scale",
                                          "restart_growth", "aa_m", "aa_reg", "nu_coarse")
                       if k in kw})
            if "nu_coarse" in kw:
                ck["coarse_from"] = max(1, kw.get("coarse_from", 2) - 1)
        rc = solve(coarse, method="mg", tol=nested_tol, max_iters=10000, **ck)
        start = rc.phi.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)
        if rc.status == "diverged":
            start = None
        res = solve(prob, method=method, phi=start, D=D, hist_cap=hist_cap, **kw)
        res.nested_iterations = rc.iterations
        return res
    phi0, D0 = prob.init_state()
    phi = phi0 if phi is None else _f64(phi).copy()
    D = D0 if D is None else _f64(D).copy()
    o = solve_opts(method=method, **kw)
    hist = np.zeros(hist_cap)
    res = Result()
    lib().fldo_solve(C.byref(prob.params), C.byref(o), _ptr(prob.sig_hat), _ptr(prob.sig_a),
                     _ptr(prob.j), _ptr(phi), _ptr(D), _ptr(hist), hist_cap, C.byref(res))
    if res.status == 1:
        raise ValueError("invalid multigrid configuration for this grid")
    return SolveResult(phi, D, STATUS.get(res.status, str(res.status)), res.iterations, res.rel,
                       res.rel_sweep, hist[:min(res.history_len, hist_cap)].copy())

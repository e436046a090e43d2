"""Autotuner of the multigrid solve: launch shapes, smoothing schedule, outer
step and pass forms.

Four phases, all timed on the GPU through the C ABI with the inputs resident
in device memory:

1. Launch shapes (``task_cells0``, ``coarse_blocks``).  They change no result
   bit, so a short capped solve per candidate gives the time per outer
   iteration; the fastest wins.
2. Smoothing schedule (``nu1``, ``nu2``, ``omega_s``) and the growth
   factor that restarts the conjugate-gradient direction
   (``restart_growth``; restarts are never switched off), then the factor on
   the finest coarse-grid correction (``corr_scale``) for the winner, then
   grid sequencing (``nested_tol``: first solve the 2:1 coarser medium to
   this tolerance).  These change the iteration, so every candidate runs a
   full solve to the tolerance with the phase-1 shape; the shortest time to
   tolerance wins.  ``quick`` keeps the default schedule and tunes only
   ``corr_scale`` and ``nested_tol``; ``refine`` starts from the cached
   entry and tries only ``nested_tol``.
3. Outer step (``anderson``): Anderson acceleration windows (``aa_m``) in
   place of the conjugate-gradient step for the winner, then a few schedules
   and correction factors with the best window (the best smoothing schedule
   changes with the outer step), the regularisation, and how far the coarser
   problem is solved first.  Starting from the cached entry it runs alone.
   ``coarse`` then tries extra smoothing sweeps on the coarse levels
   (``nu_coarse`` from level ``coarse_from`` on) for the winner, then the
   sweeps on the levels above them (``nu1`` = ``nu2``) and, with an Anderson
   window, the windows again; with ``refine`` it starts from the cached entry
   and runs alone.
4. Pass forms, with the winner's options: the finest level's red and black
   half-sweeps fused into single LDS-tiled sweeps (``fuse_rb``) and the
   limiter and residual fused into one pass (``fuse_lr``), each on or off.
   Like the launch shapes they leave the iteration as it is (``fuse_lr``
   regroups the partial sums of the residual norm only), so a capped solve per
   form gives the time per outer iteration; the fastest is kept, and the
   times are stored with the entry.  ``passes_only`` runs this phase alone on
   a cached entry and keeps its other options.

The winner is cached as JSON, keyed by (GPU architecture, grid, precision,
limiter), in ``tuned.json`` beside this file unless another path is given.
``Solver``-level callers pass ``tuned_options(...)`` as keyword options.

Command line (tunes the synthetic cloud workload of ``synth.media``; with
``--workload batch`` the 16-volume x 3-channel batch, schedules only)::

    python -m paper_1403_8105_amd.autotune --workload cloud256 --precision mixed
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
# FLD_TUNE_CACHE names another cache file (read by tuned_options, written by tune)
CACHE = os.environ.get("FLD_TUNE_CACHE") or os.path.join(HERE, "tuned.json")

SHAPES = [(4096, 2048), (2048, 2048), (8192, 2048), (16384, 2048), (4096, 1024), (4096, 4096)]
SCHEDULES = [(2, 2, 1.0), (1, 1, 1.0), (2, 1, 1.0), (1, 2, 1.0), (3, 3, 1.0), (2, 2, 1.15),
             (3, 3, 1.15), (4, 4, 1.0)]
GROWTHS = [2.0, 10.0]
SCALES = [1.0, 1.2, 1.4, 1.6, 1.8]
NESTED = [1e-3, 1e-2]
DEFAULT_SCHEDULE = (2, 2, 1.0, 2.0)
AA_WINDOWS = [6, 8, 10, 12, 16]
AA_REGS = [1e-8, 1e-6]          # tried after the default 1e-10 for the best window
AA_SCHEDULES = [(4, 4, 1.15), (3, 3, 1.15), (2, 2, 1.15), (3, 3, 1.0), (2, 2, 1.0), (5, 5, 1.15),
                (6, 6, 1.15), (4, 4, 1.25)]
AA_SCALES = [1.4, 1.6, 1.8, 2.0]
AA_NESTED = [3e-3, 1e-2, 3e-2, 1e-1]   # grid sequencing with the chosen window
COARSE_SWEEPS = [(8, 2), (12, 2), (16, 2), (24, 2), (32, 2), (12, 1), (16, 1), (16, 3), (24, 3),
                 (32, 3), (48, 3)]
FINE_SWEEPS = [2, 3, 4, 5]      # nu1 = nu2 on the finest levels, retried with the coarse sweeps
PASSES = [(0, 0), (1, 0), (0, 1), (1, 1)]   # (fuse_rb, fuse_lr)


def cache_key(arch: str, shape, precision: str, limiter: str, tol: float | None = None) -> str:
    """Key of a cache entry; ``tol`` names an entry tuned for that tolerance
    (a schedule that is fastest to 1e-6 need not be to 1e-10)."""
    key = f"{arch}|{shape[0]}x{shape[1]}x{shape[2]}|{precision}|{limiter}"
    return key if tol is None else f"{key}|tol={tol:g}"


def device_arch(device: int = 0) -> str:
    import paper_1403_8105_amd as F

    return F.fld_device_arch(device)


def load_cache(path: str = CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def tuned_options(shape, precision: str = "mixed", limiter: str = "lp", arch: str | None = None,
                  path: str = CACHE, tol: float | None = None) -> dict:
    """Cached options for this grid (with ``tol``: the entry tuned for that
    tolerance if there is one, else the grid's entry), or {} when it was never
    tuned."""
    arch = arch or device_arch()
    cache = load_cache(path)
    entry = cache.get(cache_key(arch, shape, precision, limiter, tol)) if tol is not None else None
    entry = entry or cache.get(cache_key(arch, shape, precision, limiter))
    return dict(entry["options"]) if entry else {}


def _pass_forms(F, st, h, ptrs, d_phi, stream, opts, probe_iters, log):
    """Time per outer iteration of each pass form with the options ``opts``
    (grid sequencing off, so that only fine iterations are timed)."""
    out = {}
    for rb, lr in PASSES:
        o = dict(opts, tol=0.0, max_iters=probe_iters, nested_tol=0.0, fuse_rb=rb, fuse_lr=lr)
        _solve_ms(F, st, h, ptrs, d_phi, stream, o)      # warm
        ms, rep = _solve_ms(F, st, h, ptrs, d_phi, stream, o)
        out[(rb, lr)] = ms / max(rep["iterations"], 1)
        log(f"autotune: fuse_rb={rb} fuse_lr={lr}: {out[(rb, lr)]:.4f} ms/it")
    return out


def _apply_passes(opts: dict, pass_ms: dict) -> dict:
    rb, lr = min(pass_ms, key=pass_ms.get)
    opts = {k: v for k, v in opts.items() if k not in ("fuse_rb", "fuse_lr")}
    if rb:
        opts["fuse_rb"] = 1
    if lr:
        opts["fuse_lr"] = 1
    return opts


def _device_inputs(sigma_t, albedo, Q):
    """The medium in device memory: (tensors to keep alive, the three input
    pointers, the fluence buffer's pointer, the stream)."""
    import torch

    dev = torch.device("cuda:0")
    d = [torch.from_numpy(a).to(dev) for a in (sigma_t, albedo, Q)]
    d_phi = torch.empty_like(d[0])
    stream = torch.cuda.current_stream(dev).cuda_stream
    return d + [d_phi], [t.data_ptr() for t in d], d_phi.data_ptr(), stream


def _solve_ms(F, st, h, dev_inputs, d_phi, stream, opts):
    """One device solve; returns (wall ms, report)."""
    import torch

    s = F.Solver(st.shape, h, stream=stream, **opts)
    try:
        s.set_medium_device(*dev_inputs, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = F.fld_solve_device(s.ctx, d_phi,
                                 allow=(F.FLD_OK, F.FLD_ERR_NOT_CONVERGED, F.FLD_ERR_DIVERGED))
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, rep
    finally:
        s.close()


def tune(sigma_t, albedo, Q, h, precision: str = "mixed", limiter: str = "lp", tol: float = 1e-6,
         probe_iters: int = 40, max_iters: int = 5000, path: str | None = CACHE, log=print,
         quick: bool = False, refine: bool = False, schedules=None, scales=None,
         anderson: bool = False, tol_key: bool = False, passes_only: bool = False,
         coarse: bool = False) -> dict:
    """Tune one grid/medium; stores and returns the cache entry.  ``schedules``
    ((nu1, nu2, omega_s, restart_growth) tuples) and ``scales`` replace the
    default candidate lists (for grids whose full search is too long).
    ``anderson`` adds phase 3 (with ``refine``: phase 3 alone).  ``tol_key``
    stores the entry under a key that names ``tol``; ``refine`` then starts
    from that entry or, if there is none yet, from the grid's own."""
    import paper_1403_8105_amd as F

    # keep: the device tensors, alive until the search ends
    keep, ptrs, phi_ptr, stream = _device_inputs(sigma_t, albedo, Q)
    base = dict(precision=precision, limiter=limiter)
    even = all(x % 2 == 0 for x in sigma_t.shape)
    key = cache_key(device_arch(), sigma_t.shape, precision, limiter, tol if tol_key else None)
    cache0 = load_cache(path or CACHE)
    old = cache0.get(key) if refine else None
    if refine and not old and tol_key:
        old = cache0.get(cache_key(device_arch(), sigma_t.shape, precision, limiter))
    if refine and not old:
        raise RuntimeError(f"autotune: --refine needs a cached entry for {key}")
    if passes_only:
        # phase 4 alone on the cached entry
        entry = cache0.get(key)
        if not entry:
            raise RuntimeError(f"autotune: --passes-only needs a cached entry for {key}")
        pass_ms = _pass_forms(F, sigma_t, h, ptrs, phi_ptr, stream,
                              dict(base, **entry["options"]), probe_iters, log)
        entry = dict(entry, options=_apply_passes(entry["options"], pass_ms),
                     pass_ms_per_iteration={f"{a},{b}": v for (a, b), v in pass_ms.items()})
        if path:
            cache = load_cache(path)
            cache[key] = entry
            with open(path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        return entry

    # phase 1: launch shapes, time per outer iteration of a capped solve
    shape_ms = {}
    if old:
        tc0, cb = old["options"]["task_cells0"], old["options"]["coarse_blocks"]
        shape_ms = {tuple(int(v) for v in k.split(",")): ms
                    for k, ms in old.get("shape_ms_per_iteration", {}).items()}
    else:
        for tc0, cb in SHAPES:
            o = dict(base, tol=0.0, max_iters=probe_iters, task_cells0=tc0, coarse_blocks=cb)
            _solve_ms(F, sigma_t, h, ptrs, phi_ptr, stream, o)      # warm
            ms, rep = _solve_ms(F, sigma_t, h, ptrs, phi_ptr, stream, o)
            shape_ms[(tc0, cb)] = ms / max(rep["iterations"], 1)
            log(f"autotune: task_cells0={tc0} coarse_blocks={cb}: "
                f"{shape_ms[(tc0, cb)]:.4f} ms/it")
        tc0, cb = min(shape_ms, key=shape_ms.get)

    # phase 2: schedules and restart factors, then the correction factor;
    # full solves to tol
    results = []

    def run(nu1, nu2, ws, gr, sc, nt=0.0, aa=0, reg=1e-10, nc=0, cf=2):
        o = dict(base, tol=tol, max_iters=max_iters, task_cells0=tc0, coarse_blocks=cb,
                 nu1=nu1, nu2=nu2, omega_s=ws, restart_growth=gr, corr_scale=sc, nested_tol=nt,
                 aa_m=aa, aa_reg=reg, nu_coarse=nc, coarse_from=cf)
        ms, rep = _solve_ms(F, sigma_t, h, ptrs, phi_ptr, stream, o)
        ok = rep["status"] == F.FLD_OK
        results.append({"nu1": nu1, "nu2": nu2, "omega_s": ws, "restart_growth": gr,
                        "corr_scale": sc, "nested_tol": nt, "aa_m": aa, "aa_reg": reg,
                        "nu_coarse": nc, "coarse_from": cf, "ms": ms,
                        "iterations": rep["iterations"],
                        "nested_iterations": rep.get("nested_iterations", 0),
                        "rel": rep["rel"], "converged": ok})
        log(f"autotune: nu=({nu1},{nu2}) omega_s={ws} restart_growth={gr} corr_scale={sc} "
            f"nested_tol={nt} aa_m={aa} nu_coarse={nc}@{cf}: {rep['iterations']} its "
            f"(+{rep.get('nested_iterations', 0)} coarse), rel {rep['rel']:.2e}, {ms:.0f} ms"
            f"{'' if ok else ' (not converged)'}")
        return results[-1] if ok else None

    def again(b, **over):
        """run() with the options of result b, some replaced"""
        p = dict(nu1=b["nu1"], nu2=b["nu2"], ws=b["omega_s"], gr=b["restart_growth"],
                 sc=b["corr_scale"], nt=b.get("nested_tol", 0.0), aa=b.get("aa_m", 0),
                 reg=b.get("aa_reg", 1e-10), nc=b.get("nu_coarse", 0),
                 cf=b.get("coarse_from", 2))
        p.update(over)
        return run(**p)

    def better(a, b):
        return a if b is None or (a is not None and a["ms"] < b["ms"]) else b

    best = None
    if old:
        oo = old["options"]
        best = run(oo["nu1"], oo["nu2"], oo["omega_s"], oo["restart_growth"], oo["corr_scale"],
                   oo.get("nested_tol", 0.0), oo.get("aa_m", 0), oo.get("aa_reg", 1e-10),
                   oo.get("nu_coarse", 0), oo.get("coarse_from", 2))
    elif quick:
        best = run(*DEFAULT_SCHEDULE, 1.0)
    else:
        cands = schedules or [(nu1, nu2, ws, gr) for nu1, nu2, ws in SCHEDULES for gr in GROWTHS]
        for nu1, nu2, ws, gr in cands:
            best = better(run(nu1, nu2, ws, gr, (scales or SCALES)[0]), best)
    if best is None and not (old and (anderson or coarse)):
        raise RuntimeError("autotune: no schedule reached the tolerance")
    if not old:
        for sc in (scales or SCALES)[1:]:
            best = better(run(best["nu1"], best["nu2"], best["omega_s"], best["restart_growth"],
                              sc), best)
    if even and not (old and (anderson or coarse)):
        for nt in NESTED:
            best = better(run(best["nu1"], best["nu2"], best["omega_s"], best["restart_growth"],
                              best["corr_scale"], nt), best)
    if anderson and not (old and coarse):
        # phase 3: Anderson windows for the winner, then schedules and
        # correction factors with the best window.  Anderson acceleration needs
        # a start near the solution: without grid sequencing in the winner,
        # its candidates start from the 2:1 coarser solve to 1e-2
        # the starting entry's options when none of its runs converged
        b0 = best or ({k: old["options"].get(k, v) for k, v in
                       (("nu1", 2), ("nu2", 2), ("omega_s", 1.0), ("restart_growth", 2.0),
                        ("corr_scale", 1.0), ("nested_tol", 0.0))} if old else None)
        if b0 is None:
            raise RuntimeError("autotune: no schedule reached the tolerance")
        nt0 = b0.get("nested_tol", 0.0) or (1e-2 if even else 0.0)
        for m in AA_WINDOWS:
            best = better(run(b0["nu1"], b0["nu2"], b0["omega_s"], b0["restart_growth"],
                              b0["corr_scale"], nt0, m), best)
        if best.get("aa_m"):
            b1 = best
            for nu1, nu2, ws in AA_SCHEDULES:
                if (nu1, nu2, ws) != (b1["nu1"], b1["nu2"], b1["omega_s"]):
                    best = better(run(nu1, nu2, ws, b1["restart_growth"], b1["corr_scale"],
                                      b1.get("nested_tol", 0.0), b1["aa_m"]), best)
            b2 = best
            for sc in AA_SCALES:
                if sc != b2["corr_scale"]:
                    best = better(run(b2["nu1"], b2["nu2"], b2["omega_s"], b2["restart_growth"],
                                      sc, b2.get("nested_tol", 0.0), b2["aa_m"]), best)
            b3 = best
            for reg in AA_REGS:
                best = better(run(b3["nu1"], b3["nu2"], b3["omega_s"], b3["restart_growth"],
                                  b3["corr_scale"], b3.get("nested_tol", 0.0), b3["aa_m"], reg),
                              best)
            # how far to solve the coarser problem first, with the window chosen
            b4 = best
            if even:
                for nt in AA_NESTED:
                    if nt != b4.get("nested_tol", 0.0):
                        best = better(run(b4["nu1"], b4["nu2"], b4["omega_s"],
                                          b4["restart_growth"], b4["corr_scale"], nt, b4["aa_m"],
                                          b4.get("aa_reg", 1e-10)), best)
    if coarse and best is not None:
        # extra sweeps on the coarse levels, the sweeps above them, then (with
        # a window) the windows again
        b5 = best
        for nc, cf in COARSE_SWEEPS:
            if (nc, cf) != (b5.get("nu_coarse", 0), b5.get("coarse_from", 2)):
                best = better(again(b5, nc=nc, cf=cf), best)
        b7 = best
        if b7.get("nu_coarse"):
            for nf in FINE_SWEEPS:
                if (nf, nf) != (b7["nu1"], b7["nu2"]):
                    best = better(again(b7, nu1=nf, nu2=nf), best)
        if best is not b5 and best.get("aa_m"):
            b6 = best
            for m in AA_WINDOWS:
                if m != b6["aa_m"]:
                    best = better(again(b6, aa=m), best)
    if best is None:
        raise RuntimeError("autotune: no candidate reached the tolerance")
    opts = {"task_cells0": tc0, "coarse_blocks": cb, "nu1": best["nu1"], "nu2": best["nu2"],
            "omega_s": best["omega_s"], "restart_growth": best["restart_growth"],
            "corr_scale": best["corr_scale"]}
    if best.get("nested_tol"):
        opts["nested_tol"] = best["nested_tol"]
    if best.get("aa_m"):
        opts["aa_m"] = best["aa_m"]
        if best.get("aa_reg", 1e-10) != 1e-10:
            opts["aa_reg"] = best["aa_reg"]
    if best.get("nu_coarse"):
        opts["nu_coarse"] = best["nu_coarse"]
        opts["coarse_from"] = best["coarse_from"]
    # phase 4: pass forms with the winner's options
    pass_ms = _pass_forms(F, sigma_t, h, ptrs, phi_ptr, stream, dict(base, **opts),
                          probe_iters, log)
    opts = _apply_passes(opts, pass_ms)
    entry = {
        "options": opts,
        "tol": tol,
        "ms_to_tol": best["ms"],
        "iterations": best["iterations"],
        "shape_ms_per_iteration": {f"{a},{b}": v for (a, b), v in shape_ms.items()},
        "pass_ms_per_iteration": {f"{a},{b}": v for (a, b), v in pass_ms.items()},
        "schedules": (cache0[key].get("schedules", []) if refine and key in cache0 else [])
                     + results,
    }
    if path:
        cache = load_cache(path)
        cache[key] = entry
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return entry


BATCH_KEY = "batch16x3"   # grid part of the cache key of the batched cloud workload


def batch_options(precision: str = "mixed", limiter: str = "lp", arch: str | None = None,
                  path: str = CACHE) -> dict:
    """Cached options of the batched workload, or {} when it was never tuned."""
    arch = arch or device_arch()
    entry = load_cache(path).get(f"{arch}|{BATCH_KEY}|{precision}|{limiter}")
    return dict(entry["options"]) if entry else {}


def tune_batch(precision: str = "mixed", limiter: str = "lp", tol: float = 1e-6,
               max_iters: int = 5000, path: str | None = CACHE, log=print, schedules=None,
               scales=None, anderson: bool = False, refine: bool = False,
               coarse: bool = False) -> dict:
    """Schedule search on the batched workload (``synth.media.batch_config``: 16
    cloud volumes x 3 colour channels): every candidate is one whole batched
    solve to the tolerance, default launch shapes; the shortest wins.  Grid
    sequencing (``nested_tol``) is tried last for the winner."""
    import paper_1403_8105_amd as F
    from synth import media

    vols = media.batch_config()
    dims = [(v["n"],) * 3 for v in vols]
    shapes = [d for d in dims for _ in range(3)]
    allow = (F.FLD_OK, F.FLD_ERR_NOT_CONVERGED, F.FLD_ERR_DIVERGED)
    results = []

    def run(nu1, nu2, ws, gr, sc, nt=0.0, aa=0, reg=1e-10, nc=0, cf=2):
        o = F.fld_default_options(precision=precision, limiter=limiter, tol=tol,
                                  max_iters=max_iters, nu1=nu1, nu2=nu2, omega_s=ws,
                                  restart_growth=gr, corr_scale=sc, nested_tol=nt, aa_m=aa,
                                  aa_reg=reg, nu_coarse=nc, coarse_from=cf)
        b = F.fld_batch_create(o, dims, [v["h"] for v in vols], 3)
        try:
            for q, v in enumerate(vols):
                F.fld_batch_set_volume(b, q, v["sigma_t"], v["albedo"], v["Q"])
            t0 = time.perf_counter()
            _, its, rep = F.fld_batch_solve(b, shapes, allow=allow, want_phi=False)
            ms = (time.perf_counter() - t0) * 1e3
        finally:
            F.fld_batch_destroy(b)
        ok = rep["status"] == F.FLD_OK
        results.append({"nu1": nu1, "nu2": nu2, "omega_s": ws, "restart_growth": gr,
                        "corr_scale": sc, "nested_tol": nt, "aa_m": aa, "aa_reg": reg,
                        "nu_coarse": nc, "coarse_from": cf, "ms": ms,
                        "iterations_max": int(its.max()), "converged": ok})
        log(f"autotune batch: nu=({nu1},{nu2}) omega_s={ws} restart_growth={gr} "
            f"corr_scale={sc} nested_tol={nt} aa_m={aa} nu_coarse={nc}@{cf}: "
            f"iterations {its.min()}..{its.max()} "
            f"(+{rep.get('nested_iterations', 0)} coarse), {ms:.0f} ms"
            f"{'' if ok else ' (not converged)'}")
        return results[-1] if ok else None

    def better(a, b):
        return a if b is None or (a is not None and a["ms"] < b["ms"]) else b

    scs = scales or SCALES
    key = f"{device_arch()}|{BATCH_KEY}|{precision}|{limiter}"
    old = load_cache(path or CACHE).get(key) if refine else None
    if refine and not old:
        raise RuntimeError(f"autotune batch: --refine needs a cached entry for {key}")
    best = None
    if old:
        oo = old["options"]
        best = run(oo["nu1"], oo["nu2"], oo["omega_s"], oo["restart_growth"], oo["corr_scale"],
                   oo.get("nested_tol", 0.0), oo.get("aa_m", 0), oo.get("aa_reg", 1e-10),
                   oo.get("nu_coarse", 0), oo.get("coarse_from", 2))
    else:
        cands = schedules or [(nu1, nu2, ws, gr) for nu1, nu2, ws in SCHEDULES for gr in GROWTHS]
        for nu1, nu2, ws, gr in cands:
            best = better(run(nu1, nu2, ws, gr, scs[0]), best)
    if best is None:
        raise RuntimeError("autotune batch: no schedule reached the tolerance")
    if not old:
        for sc in scs[1:]:
            best = better(run(best["nu1"], best["nu2"], best["omega_s"], best["restart_growth"],
                              sc), best)
        if all(n % 2 == 0 for d in dims for n in d):
            for nt in NESTED:
                best = better(run(best["nu1"], best["nu2"], best["omega_s"],
                                  best["restart_growth"], best["corr_scale"], nt), best)

    def again(b, **over):
        p = dict(nu1=b["nu1"], nu2=b["nu2"], ws=b["omega_s"], gr=b["restart_growth"],
                 sc=b["corr_scale"], nt=b.get("nested_tol", 0.0), aa=b.get("aa_m", 0),
                 reg=b.get("aa_reg", 1e-10), nc=b.get("nu_coarse", 0),
                 cf=b.get("coarse_from", 2))
        p.update(over)
        return run(**p)

    if anderson and not (old and coarse):
        b0 = best
        for m in AA_WINDOWS:
            best = better(run(b0["nu1"], b0["nu2"], b0["omega_s"], b0["restart_growth"],
                              b0["corr_scale"], b0["nested_tol"], m), best)
        if best.get("aa_m"):
            b1 = best
            for nu1, nu2, ws in AA_SCHEDULES:
                if (nu1, nu2, ws) != (b1["nu1"], b1["nu2"], b1["omega_s"]):
                    best = better(run(nu1, nu2, ws, b1["restart_growth"], b1["corr_scale"],
                                      b1["nested_tol"], b1["aa_m"]), best)
            b3 = best
            for reg in AA_REGS:
                best = better(run(b3["nu1"], b3["nu2"], b3["omega_s"], b3["restart_growth"],
                                  b3["corr_scale"], b3["nested_tol"], b3["aa_m"], reg), best)
            b4 = best
            for nt in AA_NESTED:
                if nt != b4["nested_tol"]:
                    best = better(run(b4["nu1"], b4["nu2"], b4["omega_s"], b4["restart_growth"],
                                      b4["corr_scale"], nt, b4["aa_m"], b4.get("aa_reg", 1e-10)),
                                  best)
    if coarse:
        b5 = best
        for nc, cf in COARSE_SWEEPS:
            if (nc, cf) != (b5.get("nu_coarse", 0), b5.get("coarse_from", 2)):
                best = better(again(b5, nc=nc, cf=cf), best)
        b7 = best
        if b7.get("nu_coarse"):
            for nf in FINE_SWEEPS:
                if (nf, nf) != (b7["nu1"], b7["nu2"]):
                    best = better(again(b7, nu1=nf, nu2=nf), best)
        if best is not b5 and best.get("aa_m"):
            b6 = best
            for m in AA_WINDOWS:
                if m != b6["aa_m"]:
                    best = better(again(b6, aa=m), best)
    keys = ("nu1", "nu2", "omega_s", "restart_growth", "corr_scale") + \
        (("nested_tol",) if best["nested_tol"] else ()) + (("aa_m",) if best.get("aa_m") else ()) + \
        (("aa_reg",) if best.get("aa_m") and best.get("aa_reg", 1e-10) != 1e-10 else ()) + \
        (("nu_coarse", "coarse_from") if best.get("nu_coarse") else ())
    entry = {"options": {k: best[k] for k in keys},
             "tol": tol, "ms_to_tol": best["ms"], "iterations_max": best["iterations_max"],
             "schedules": results}
    if old:
        entry["schedules"] = old.get("schedules", []) + results
    if path:
        cache = load_cache(path)
        cache[key] = entry
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return entry


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="cloud256")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--limiter", default="lp")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--quick", action="store_true",
                    help="default schedule; tune launch shapes and corr_scale only")
    ap.add_argument("--max-iters", type=int, default=5000)
    ap.add_argument("--refine", action="store_true",
                    help="start from the cached entry; try only grid sequencing")
    ap.add_argument("--schedules", default=None,
                    help="candidate schedules 'nu1,nu2,omega_s,growth;...' (default: all)")
    ap.add_argument("--anderson", action="store_true",
                    help="also try Anderson windows for the outer step (with --refine: only "
                         "that, from the cached entry)")
    ap.add_argument("--scales", default=None,
                    help="correction factors 'first,second,...'; the first goes with the "
                         "schedule search (default 1.0,1.2,1.4,1.6,1.8)")
    ap.add_argument("--tol-key", action="store_true",
                    help="store the entry under a key naming --tol (a separate entry for a "
                         "tight tolerance)")
    ap.add_argument("--coarse", action="store_true",
                    help="also try extra sweeps on the coarse levels (with --refine: only "
                         "that, from the cached entry)")
    ap.add_argument("--passes-only", action="store_true",
                    help="time the fused and separate pass forms with the cached entry's "
                         "options and keep the fastest (no other option changes)")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    from synth import media

    schedules = ([tuple(float(v) if i >= 2 else int(v) for i, v in enumerate(c.split(",")))
                  for c in args.schedules.split(";")] if args.schedules else None)
    scales = [float(v) for v in args.scales.split(",")] if args.scales else None
    if args.workload == "batch":
        entry = tune_batch(precision=args.precision, limiter=args.limiter, tol=args.tol,
                           max_iters=args.max_iters, path=args.out,
                           log=lambda m: print(m, flush=True), schedules=schedules,
                           scales=scales, anderson=args.anderson, refine=args.refine,
                           coarse=args.coarse)
        print(json.dumps({"options": entry["options"], "ms_to_tol": entry["ms_to_tol"]}),
              flush=True)
        return
    st, al, Q, h = media.config(args.workload, n=args.n)
    entry = tune(st, al, Q, h, precision=args.precision, limiter=args.limiter, tol=args.tol,
                 path=args.out, log=lambda m: print(m, flush=True), quick=args.quick,
                 max_iters=args.max_iters, refine=args.refine, schedules=schedules,
                 scales=scales, anderson=args.anderson, tol_key=args.tol_key,
                 passes_only=args.passes_only, coarse=args.coarse)
    print(json.dumps({"options": entry["options"], "ms_to_tol": entry["ms_to_tol"],
                      "iterations": entry["iterations"],
                      "pass_ms_per_iteration": entry.get("pass_ms_per_iteration")}), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the MI355X flux-limited diffusion solve (one JSON line).

Workload: the 256^3 heterogeneous cloud (5-octave value noise, sigma_t in
[0, 200] with 40 % of the voxels below 0.01, albedo 0.99, single-scatter
source from a +z directional light), Levermore-Pomraning limiter, mixed
precision Picard multigrid, solved from the paper's initial state to a
relative residual of 1e-6.  One step = one full solve; inputs are resident in
HBM before the timed region starts.

value = voxel-updates per second over the timed steps: a voxel update is one
application of the relaxation point update to one cell (red-black sweeps on
every multigrid level).  ms_per_step is the time to 1e-6.

The roofline entry is for the finest-level smoother: its average launch time
comes from HIP events recorded around every launch on the solver's stream
during the last timed step (the other steps run an identical context without
events, whose graph nodes cost a few microseconds each), its algorithmic
bytes from the per-launch figure the library reports.  The HBM traffic measured by counters is read from the
committed counter summary while the kernel source it was taken on is
unchanged.

Other workloads (`--workload`, one JSON line each; not the headline):
  cloud128-fp64  128^3 cloud (seed 1), plain FP64 multigrid to rel 1e-8;
  batch          16 cloud volumes of seeded sizes {64..192}^3 x 3 colour
                 channels (albedo 0.99/0.95/0.9, shared sigma_t), one batched
                 mixed solve to rel 1e-6; --sequential adds the same 48
                 problems solved one at a time;
  cloud512       512^3 cloud (7 octaves, sigma_t in [0,500], 60% near-vacuum,
                 albedo 0.995, seed 4), mixed to rel 1e-6, solved in resumed
                 chunks so progress is printed;
  bake           light baking of the 512^3 cloud's single-scatter source on the
                 GPU (fld_light_bake), HIP-event timed, against the 24 bytes
                 per voxel it must move;
  render         primary ray-march of the 512^3 cloud's image (fld_render) from
                 a fluence field, against its 32 bytes per voxel;
  convergence    the convergence studies of Sec. 5 (Fig. 3) on the GPU:
                 Algorithm 1 (FP64 red-black SOR) on the spherical cloud at 51^3
                 for a range of SOR factors, iterations to 1e-6 against the grid
                 size, and the effect of the extinction floor sigma_eps (sphere
                 with Algorithm 1, 128^3 cloud with the mixed multigrid).

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
       [--no-fp64] [--max-iters M] [--copy-bytes B] [--workload W]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = ["k_smooth_fine", "k_residual", "k_limiter", "k_npcg_dir"]
KERNEL_ROLES = ["finest-level red-black smoother half-sweep", "finest FP64 residual",
                "limiter pass", "conjugate-direction pass"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_smooth_fine_cloud256_traffic.md")
KERNEL_SRC = os.path.join(ROOT, "paper_1403_8105_amd", "csrc", "fld_kernels.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def counter_traffic():
    """HBM bytes per finest-smoother launch from the committed counter summary,
    or None if there is none or the kernel source changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m_hash = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", txt)
    m_bytes = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def host_cpu():
    """Model name, physical cores and usable logical CPUs of this host."""
    model, cores = None, set()
    phys = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "model name" and model is None:
                    model = val
                elif key == "physical id":
                    phys = val
                elif key == "core id":
                    cores.add((phys, val))
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "physical_cores": len(cores) or None, "usable_cpus": usable}


def cpu_baseline(st, al, Q, h, schedule, gpu_iterations, budget_s=20.0):
    """Oracle (plain FP64 C) on a bounded sample: outer multigrid iterations
    of the same solve with the GPU solve's schedule, voxel-updates/s on the
    same definition, and the time to the tolerance that rate implies for the
    GPU's iteration count (an extrapolation, labelled as such)."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    kw = {k: schedule[k] for k in ("nu1", "nu2", "omega_s", "restart_growth", "corr_scale")
          if k in schedule}
    nu = kw.get("nu1", 2) + kw.get("nu2", 2)
    t0 = time.perf_counter()
    prob = oracle.setup(st, al, Q, h)
    levels, _ = oracle.mg_levels(*st.shape)
    per_it = sum(a * b * c for a, b, c in levels[:-1]) * float(nu)   # point updates
    t1 = time.perf_counter()
    oracle.solve(prob, method="mg", tol=0.0, max_iters=1, **kw)
    t_one = time.perf_counter() - t1
    its = max(1, min(40, int(budget_s / max(t_one, 1e-3))))
    t2 = time.perf_counter()
    res = oracle.solve(prob, method="mg", tol=0.0, max_iters=its, **kw)
    dt = time.perf_counter() - t2
    out = {"value": per_it * res.iterations / dt, "unit": "voxel-updates/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{res.iterations} outer multigrid iterations of the {st.shape[0]}^3 "
                     f"cloud solve with the GPU solve's schedule {kw or '(defaults)'} "
                     f"(FP64, OpenMP threads={threads}; the time includes the limiter and "
                     f"residual passes of each iteration), {dt:.1f} s after "
                     f"{t1 - t0:.1f} s set-up",
           "s_per_outer_iteration": dt / res.iterations,
           "est_time_to_tol_s": dt / res.iterations * gpu_iterations,
           "est_note": f"s_per_outer_iteration x the {gpu_iterations} outer iterations of the "
                       f"GPU solve (extrapolated, not run)"}
    out.update(host_cpu())
    return out


def copy_calibration(nbytes, reps=5):
    """A plain device-to-device copy of known size, for scaling the HBM
    counters (FETCH_SIZE / WRITE_SIZE) of the solver kernels."""
    import torch

    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    # the copy's own rate (read + write) is the practical ceiling beside the 8 TB/s peak
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": reps + 1,
                      "ms_per_copy": ms, "copy_gb_per_s": 2.0 * n * 4 / (ms * 1e-3) / 1e9}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--max-iters", type=int, default=None,
                    help="outer iteration cap (default 5000; 20000 for cloud512)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the plain FP64 GPU solve reported beside the mixed one")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain copy of this many bytes (counter calibration)")
    ap.add_argument("--no-tuned", action="store_true",
                    help="ignore the autotuner's cached launch shapes and schedule")
    ap.add_argument("--workload", default="cloud256",
                    choices=["cloud256", "cloud128-fp64", "batch", "cloud512", "bake", "render",
                             "convergence"])
    ap.add_argument("--chunk", type=int, default=0,
                    help="outer iterations per call (0: one call); later calls resume")
    ap.add_argument("--sequential", action=argparse.BooleanOptionalAction, default=True,
                    help="batch workload: also time the problems solved one at a time")
    ap.add_argument("--err-tol", type=float, default=1e-10,
                    help="tolerance of the FP64 reference solve and of the second mixed solve of "
                         "err_vs_fp64 (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the solve of one volume runs on a single MI355X).", file=sys.stderr)
        sys.exit(2)
    if args.copy_bytes > 0:
        copy_calibration(args.copy_bytes)
        return
    if args.workload == "batch":
        args.max_iters = args.max_iters or 5000
        run_batch(args)
        return
    if args.workload in ("bake", "render"):
        run_bake(args)
        return
    if args.workload == "convergence":
        run_convergence(args)
        return
    if args.workload == "cloud128-fp64":
        args.n, args.precision, args.tol, cfg = 128, "fp64", 1e-8, "cloud128"
        args.no_fp64 = True
    elif args.workload == "cloud512":
        args.n, cfg = 512, "cloud512"
        args.no_fp64 = args.no_cpu_baseline = True
        args.chunk = args.chunk or 1000
        args.max_iters = args.max_iters or 20000
    else:
        cfg = "cloud256"
    args.max_iters = args.max_iters or 5000

    import torch
    import paper_1403_8105_amd as F
    from synth import media

    n = args.n
    log(f"bench: generating cloud {n}^3")
    st, al, Q, h = media.config(cfg, n=n)
    desc = {"cloud256": "sigma_t in [0,200], 40% near-vacuum, albedo 0.99",
            "cloud128": "sigma_t in [0,200], 40% near-vacuum, albedo 0.99",
            "cloud512": "7 octaves, sigma_t in [0,500], 60% near-vacuum, albedo 0.995"}[cfg]
    dev = torch.device("cuda:0")
    d_st = torch.from_numpy(st).to(dev)
    d_al = torch.from_numpy(al).to(dev)
    d_Q = torch.from_numpy(Q).to(dev)
    d_phi = torch.empty_like(d_st)
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream

    from paper_1403_8105_amd.autotune import tuned_options

    tuned, tuned_from = {}, {}
    for prec in ("mixed", "fp64"):
        tuned[prec], tuned_from[prec] = {}, None
        if not args.no_tuned:
            # only the grid's own entry: a schedule tuned on 256^3 (omega_s
            # 1.15, restart factor 10) diverges on the 512^3 cloud
            tuned[prec] = tuned_options(st.shape, prec, "lp")
            if tuned[prec]:
                tuned_from[prec] = "x".join(map(str, st.shape))
        log(f"bench: {prec} options from the autotuner cache ({tuned_from[prec]}): "
            f"{tuned[prec] or 'none (defaults)'}")

    setup_ms = []

    def make(precision, timing, tol=None, max_iters=None, opts=None):
        s = F.Solver(st.shape, h, precision=precision, tol=args.tol if tol is None else tol,
                     max_iters=max_iters or args.chunk or args.max_iters, timing=timing,
                     stream=sp, **(tuned[precision] if opts is None else opts))
        torch.cuda.synchronize()
        t = time.perf_counter()
        s.set_medium_device(d_st.data_ptr(), d_al.data_ptr(), d_Q.data_ptr(), sp)
        torch.cuda.synchronize()
        setup_ms.append((time.perf_counter() - t) * 1e3)
        return s

    # HIP events cost a few microseconds per graph node, so one context with
    # per-kernel events times the last step and an identical one without them
    # the others; the roofline figures come from the events of that step
    timed = make(args.precision, 1)
    plain = make(args.precision, 0) if args.steps > 1 else None
    torch.cuda.synchronize()

    def step(s):
        """One solve to tol: one call, or resumed chunks with a progress line each."""
        r = F.fld_solve_device(s.ctx, d_phi.data_ptr())
        if not args.chunk:
            return r
        tot = dict(r)
        while tot["status"] == F.FLD_ERR_NOT_CONVERGED and tot["iterations"] < args.max_iters:
            log(f"bench: {tot['iterations']} iterations, rel {tot['rel']:.3e}")
            r = F.fld_solve_device(s.ctx, d_phi.data_ptr(), resume=1)
            for key in ("voxel_updates", "time_ms"):
                tot[key] += r[key]
            for key in ("kernel_ms", "kernel_launches", "kernel_bytes"):
                tot[key] = [a + b for a, b in zip(tot[key], r[key])]
            tot.update(status=r["status"], iterations=r["iterations"], rel=r["rel"])
        return tot

    for w in range(args.warmup):
        for s_ in ([plain] if plain else []) + [timed]:
            r = step(s_)
            log(f"bench: warmup {w}: {r['iterations']} iterations, rel {r['rel']:.2e}, "
                f"{r['time_ms']:.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for k in range(args.steps):
        reps.append(step(timed if k == args.steps - 1 else plain))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for k, r in enumerate(reps):
        log(f"bench: step {k}: {r['iterations']} iterations, rel {r['rel']:.2e}, "
            f"{r['time_ms']:.1f} ms")
    timed.close()
    if plain:
        plain.close()
    updates = sum(r["voxel_updates"] for r in reps)
    value = updates / dt
    ms_step = dt * 1e3 / args.steps
    kms = np.sum([r["kernel_ms"] for r in reps], axis=0)
    kl = np.sum([r["kernel_launches"] for r in reps], axis=0)
    kb = np.sum([r["kernel_bytes"] for r in reps], axis=0)
    names, roles = list(KERNEL_NAMES), list(KERNEL_ROLES)
    if tuned[args.precision].get("aa_m"):
        names[3], roles[3] = "k_aa_update", "Anderson update pass"
    kernels = {names[q]: {"role": roles[q], "avg_us": 1e3 * kms[q] / kl[q],
                                 "launches": int(kl[q]),
                                 "alg_bytes_per_launch": kb[q] / kl[q],
                                 "GBps": (kb[q] / kl[q]) / (kms[q] / kl[q] * 1e-3) / 1e9}
               for q in range(4) if kl[q] > 0}
    # the finest-level smoother: the kernel with the largest share of the time
    dom = 0
    avg_s = kms[dom] / kl[dom] * 1e-3
    alg = kb[dom] / kl[dom]
    achieved = alg / avg_s / 1e9
    # the counters were taken on the 256^3 mixed workload only
    traffic = (counter_traffic() if args.workload == "cloud256" and args.precision == "mixed"
               and n == 256 else None)
    ok = all(r["status"] == 0 for r in reps)
    phi_head = d_phi.clone()          # the last timed solve's fluence
    line = {
        "metric": ("voxel-updates/s + time to 1e-6 rel. residual (256^3 FLD); % HBM peak"
                   if args.workload == "cloud256" else
                   f"voxel-updates/s + time to {args.tol:g} rel. residual ({n}^3 FLD)"),
        "value": value,
        "unit": "voxel-updates/s",
        "value_note": "relaxation updates on every multigrid level per second; a schedule that "
                      "needs fewer updates per solve (more sweeps on the small levels, fewer on "
                      "the large ones) lowers it while it shortens the time to tolerance, which "
                      "is the figure of merit (time_to_tol_ms)",
        "voxel_updates_per_solve": updates / args.steps,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "time_to_tol_ms": ms_step,
        "converged": ok,
        "outer_iterations": reps[-1]["iterations"],
        "nested_iterations": reps[-1].get("nested_iterations", 0),
        "final_rel": reps[-1]["rel"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+fp64" if args.precision == "mixed" else "fp64",
        "data": "synthetic",
        "config": {"workload": f"cloud {n}^3 FLD (Levermore-Pomraning), {desc}, "
                               f"Beer-Lambert source; {args.precision} Picard multigrid "
                               f"V({tuned[args.precision].get('nu1', 2)},"
                               f"{tuned[args.precision].get('nu2', 2)})"
                               + (f" with Anderson acceleration (window "
                                  f"{tuned[args.precision]['aa_m']})"
                                  if tuned[args.precision].get("aa_m") else
                                  " with nonlinear conjugate-gradient steps")
                               + f" to rel {args.tol:g}"
                               + (f", started from the 2:1 coarser solve to "
                                  f"{tuned[args.precision]['nested_tol']:g}"
                                  if tuned[args.precision].get("nested_tol") else ""),
                   "grid": [n, n, n], "tol": args.tol, "precision": args.precision,
                   "tuned_options": tuned[args.precision],
                   "tuned_on_grid": tuned_from[args.precision]},
        "setup_ms": setup_ms[0],
        "setup_note": "fld_set_medium_device of the timed context (outside the timed region): "
                      "validation copy of the medium to the host, set-up kernels, host cluster "
                      "labelling and upload, coarse operators, and the 2:1 coarser context of "
                      "grid sequencing when the schedule uses it",
        "timing": "per-kernel HIP events recorded in the last timed step only",
        "roofline": {"bound": "hbm", "kernel": KERNEL_NAMES[dom], "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "alg_bytes_per_launch": alg,
                     "avg_launch_us": avg_s * 1e6},
        "kernels": kernels,
    }
    # the half-sweep's working set (4 arrays of 4 or 8 B per cell) against the
    # 256 MB Infinity Cache of MI355X: when it fits, part of the traffic is
    # served from there and frac is not a clean HBM fraction
    work_set = 4 * (4 if args.precision == "mixed" else 8) * n ** 3
    line["roofline"]["note"] = (
        f"working set {work_set / 2**20:.0f} MiB "
        + ("fits the 256 MiB Infinity Cache: cache-assisted, not a clean HBM fraction "
           "(the 512^3 workload gives that)" if work_set <= 256 * 2**20 else
           "exceeds the 256 MiB Infinity Cache: an HBM fraction"))
    if not args.no_fp64:
        log("bench: plain FP64 GPU solve of the same medium")
        s64 = make("fp64", 0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r64 = step(s64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        s64.close()
        line["fp64_gpu"] = {"time_to_tol_ms": t64 * 1e3, "outer_iterations": r64["iterations"],
                            "final_rel": r64["rel"], "converged": r64["status"] == 0,
                            "mixed_speedup": t64 * 1e3 / ms_step}
        log(f"bench: fp64 {r64['iterations']} iterations, rel {r64['rel']:.2e}, {t64:.2f} s")
        if args.err_tol > 0:
            # error of the mixed fluence against the plain FP64 GPU solve to
            # err_tol (that path follows the oracle iterate by iterate, also at
            # 256^3), and of a mixed solve to the same tolerance; both with the
            # cache entry tuned for that tolerance when there is one
            t10o = {prec: (tuned_options(st.shape, prec, "lp", tol=args.err_tol)
                           if not args.no_tuned else {}) for prec in ("mixed", "fp64")}
            log(f"bench: FP64 GPU solve to {args.err_tol:g} as the error reference "
                f"({t10o['fp64'] or 'defaults'})")
            ref = make("fp64", 0, tol=args.err_tol, max_iters=6000, opts=t10o["fp64"])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rr = F.fld_solve_device(ref.ctx, d_phi.data_ptr(),
                                    allow=(F.FLD_OK, F.FLD_ERR_NOT_CONVERGED))
            torch.cuda.synchronize()
            tref = time.perf_counter() - t1
            ref.close()
            phi_ref = d_phi.clone()
            log(f"bench: mixed solve to {args.err_tol:g} ({t10o[args.precision] or 'defaults'})")
            m10 = make(args.precision, 0, tol=args.err_tol, max_iters=6000,
                       opts=t10o[args.precision])
            t1 = time.perf_counter()
            r10 = F.fld_solve_device(m10.ctx, d_phi.data_ptr(),
                                     allow=(F.FLD_OK, F.FLD_ERR_NOT_CONVERGED))
            torch.cuda.synchronize()
            t10 = time.perf_counter() - t1
            m10.close()
            nref = torch.linalg.vector_norm(phi_ref).item()
            line["err_vs_fp64"] = {
                "reference": f"plain FP64 GPU solve of the same medium to rel "
                             f"{rr['rel']:.2e} ({rr['iterations']} outer iterations; "
                             f"{'converged' if rr['status'] == 0 else 'stopped at the cap'} "
                             f"for tol {args.err_tol:g})",
                "metric": "||phi - phi_ref||_2 / ||phi_ref||_2",
                "mixed_at_tol": torch.linalg.vector_norm(phi_head - phi_ref).item() / nref,
                "tol": args.err_tol,
                "fp64_ms": tref * 1e3,
                "fp64_options": t10o["fp64"],
                "mixed_to_tol": torch.linalg.vector_norm(d_phi - phi_ref).item() / nref,
                "mixed_to_tol_converged": r10["status"] == 0,
                "mixed_to_tol_iterations": r10["iterations"],
                "mixed_to_tol_rel": r10["rel"],
                "mixed_to_tol_ms": t10 * 1e3,
                "mixed_to_tol_options": t10o[args.precision],
                "mixed_to_tol_speedup": tref / t10}
            log(f"bench: err_vs_fp64 {line['err_vs_fp64']}")
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(st, al, Q, h, tuned[args.precision],
                                            reps[-1]["iterations"])
    print(json.dumps(line), flush=True)


def run_bake(args):
    """GPU light baking or ray-march render of the 512^3 cloud (one JSON line)."""
    import torch
    import paper_1403_8105_amd as F
    from synth import media

    log("bench: generating cloud 512^3")
    st, al, _, h = media.config("cloud512")
    dev = torch.device("cuda:0")
    d_st = torch.from_numpy(st).to(dev)
    d_al = torch.from_numpy(al).to(dev)
    d_q = torch.empty_like(d_st)
    stream = torch.cuda.current_stream(dev)
    render = args.workload == "render"
    if render:
        # a smooth stand-in fluence; the cost does not depend on its values
        d_phi = torch.from_numpy(media.value_noise(512, 2, 9)).to(dev)
        d_img = torch.empty((512, 512), dtype=torch.float64, device=dev)
        F.fld_light_bake(d_st.data_ptr(), d_al.data_ptr(), 1.0, st.shape, h, d_q.data_ptr(),
                         stream.cuda_stream)

    def once():
        if render:
            F.fld_render(d_st.data_ptr(), d_al.data_ptr(), d_q.data_ptr(), d_phi.data_ptr(), 1.0,
                         st.shape, h, d_img.data_ptr(), stream.cuda_stream)
        else:
            F.fld_light_bake(d_st.data_ptr(), d_al.data_ptr(), 1.0, st.shape, h, d_q.data_ptr(),
                             stream.cuda_stream)

    for _ in range(max(args.warmup, 1)):
        once()
    reps = max(args.steps, 1) * 10
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        once()
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    n = st.size
    alg = (32.0 if render else 24.0) * n
    line = {
        "metric": ("voxels/s of the GPU primary ray-march (512^3 cloud, 512^2 image)" if render
                   else "voxels/s of GPU light baking (512^3 cloud)"),
        "value": n / (ms * 1e-3),
        "unit": "voxels/s", "n_gpus": 1, "steps": reps, "warmup": max(args.warmup, 1),
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": ("orthographic +z ray-march of " if render else
                                "single-scatter source of a +z directional light over ") +
                               "the 512^3 cloud (7 octaves, sigma_t in [0,500], 60% near-vacuum, "
                               "albedo 0.995)", "grid": list(st.shape)},
        "roofline": {"bound": "hbm", "kernel": "k_render" if render else "k_light_bake", "achieved": alg / (ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": alg, "avg_launch_us": ms * 1e3},
    }
    print(json.dumps(line), flush=True)


def run_convergence(args):
    """Sec. 5, Fig. 3 on the GPU: (a) Algorithm 1's residual against iterations
    for several SOR factors omega at 51^3, (b) iterations to 1e-6 against the
    grid size, (c) the effect of the extinction floor sigma_eps.  The medium of
    (a) and (b) is the spherical cloud with a vacuum exterior and a noise
    emission field; (c) runs it and the 128^3 cloud (mixed multigrid).  Every
    solve starts from the paper's initial state; the residual is the true
    nonlinear one, checked after every iteration."""
    import paper_1403_8105_amd as F
    from synth import media

    allow = (F.FLD_OK, F.FLD_ERR_NOT_CONVERGED, F.FLD_ERR_DIVERGED)
    marks = (1e-2, 1e-4, 1e-6)

    def alg1(n, limiter="lp", omega=1.0, sigma_eps_l=None, max_iters=50000):
        st, al, Q, h = media.sphere_cloud(n)
        kw = {} if sigma_eps_l is None else {"sigma_eps": sigma_eps_l / (h * n)}
        s = F.Solver(st.shape, h, method="rbsor", limiter=limiter, omega=omega, tol=1e-6,
                     max_iters=max_iters, check_every=1, **kw)
        try:
            s.set_medium(st, al, Q)
            _, rep = s.solve(allow=allow)
        finally:
            s.close()
        hist = rep["history"]
        return {"n": n, "limiter": limiter, "omega": omega,
                "status": F.fld_status_string(rep["status"]), "iterations": rep["iterations"],
                "rel": rep["rel"], "time_ms": rep["time_ms"],
                "voxel_updates_per_s": rep["voxel_updates"] / max(rep["time_ms"], 1e-9) * 1e3,
                "iterations_to": {f"{m:g}": (int(np.argmax(hist <= m)) if (hist <= m).any()
                                             else None) for m in marks}}

    log("bench: Fig. 3a, SOR factors at 51^3")
    e1 = [alg1(51, lim, om) for lim in ("lp", "cda")
          for om in (1.0, 1.2, 1.4, 1.5, 1.6, 1.7, 1.8, 1.9)]
    log("bench: Fig. 3b, grid sizes")
    e2 = [alg1(n, "lp", om) for om in (1.0, 1.5) for n in (17, 25, 33, 41, 51, 65, 81)]
    log("bench: Fig. 3c, extinction floor")
    floors = (1e-1, 1e-2, 1e-3, 1e-4, 1e-5)
    e3_sphere = [dict(alg1(51, "lp", 1.0, se), sigma_eps_times_L=se) for se in floors]
    st, al, Q, h = media.config("cloud128")
    e3_cloud = []
    for se in floors:
        s = F.Solver(st.shape, h, precision="mixed", tol=1e-6, max_iters=5000,
                     sigma_eps=se / (h * st.shape[0]))
        try:
            s.set_medium(st, al, Q)
            _, rep = s.solve(allow=allow)
        finally:
            s.close()
        e3_cloud.append({"sigma_eps_times_L": se, "status": F.fld_status_string(rep["status"]),
                         "iterations": rep["iterations"], "rel": rep["rel"],
                         "time_ms": rep["time_ms"]})
    ref = e1[0]
    line = {
        "metric": "voxel-updates/s of Algorithm 1 (FP64 red-black SOR, omega 1) on the 51^3 "
                  "spherical cloud to 1e-6",
        "value": ref["voxel_updates_per_s"], "unit": "voxel-updates/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": ref["time_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "sphere of radius 0.4 (sigma_t 10, albedo 0.9) in vacuum with a "
                               "3-octave noise emission, unit cube, LP and CDA limiters; "
                               "128^3 cloud (5 octaves, sigma_t in [0,200]) for sigma_eps"},
        "fig3a_omega": e1, "fig3b_grid": e2, "fig3c_sigma_eps_sphere": e3_sphere,
        "fig3c_sigma_eps_cloud128_mixed_mg": e3_cloud,
    }
    print(json.dumps(line), flush=True)


def run_batch(args):
    """16 volumes x 3 colour channels in one batched solve (one JSON line)."""
    import torch
    import paper_1403_8105_amd as F
    from synth import media

    log("bench: generating the 16-volume batch")
    vols = media.batch_config()
    dims = [(v["n"],) * 3 for v in vols]
    shapes = [d for d in dims for _ in range(3)]
    voxels = sum(a * b * c for a, b, c in dims)
    # the batch's own autotuner entry (schedule only; default launch shapes)
    from paper_1403_8105_amd.autotune import batch_options
    tuned = {} if args.no_tuned else batch_options("mixed", "lp")
    log(f"bench: batch options from the autotuner cache: {tuned or 'none (defaults)'}")
    o = F.fld_default_options(precision="mixed", tol=1e-6, max_iters=args.max_iters, **tuned)
    b = F.fld_batch_create(o, dims, [v["h"] for v in vols], 3)
    for q, v in enumerate(vols):
        F.fld_batch_set_volume(b, q, v["sigma_t"], v["albedo"], v["Q"])
    torch.cuda.synchronize()
    for w in range(args.warmup):
        _, its, r = F.fld_batch_solve(b, shapes, want_phi=False)
        log(f"bench: batch warmup {w}: {r['time_ms']:.0f} ms, iterations {its.min()}..{its.max()}")
    t0 = time.perf_counter()
    reps = []
    for k in range(args.steps):
        _, its, r = F.fld_batch_solve(b, shapes, want_phi=False)
        reps.append((its, r))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    F.fld_batch_destroy(b)
    its, r = reps[-1]
    line = {
        "metric": "voxel-updates/s + time to 1e-6 rel. residual (batched FLD, 48 problems)",
        "value": sum(x[1]["voxel_updates"] for x in reps) / dt,
        "unit": "voxel-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps, "time_to_tol_ms": dt * 1e3 / args.steps,
        "converged": all(x[1]["status"] == 0 for x in reps),
        "outer_iterations_min_max": [int(its.min()), int(its.max())],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32+fp64", "data": "synthetic",
        "config": {"workload": "16 cloud volumes, sizes " + ",".join(str(d[0]) for d in dims)
                               + "^3, x 3 channels (albedo 0.99/0.95/0.9, shared sigma_t), "
                               "mixed Picard multigrid, one batched solve to rel 1e-6",
                   "voxels": voxels, "problems": len(shapes), "tuned_options": tuned},
    }
    if not args.no_fp64:
        # the same batch in plain FP64 with the FP64 defaults (no batch entry
        # is cached for it), one solve
        log("bench: the batch in plain FP64")
        o64 = F.fld_default_options(precision="fp64", tol=1e-6, max_iters=args.max_iters)
        b64 = F.fld_batch_create(o64, dims, [v["h"] for v in vols], 3)
        for q, v in enumerate(vols):
            F.fld_batch_set_volume(b64, q, v["sigma_t"], v["albedo"], v["Q"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, its64, r64 = F.fld_batch_solve(b64, shapes, want_phi=False)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        F.fld_batch_destroy(b64)
        line["fp64_gpu_batch"] = {"time_to_tol_ms": t64 * 1e3,
                                  "converged": r64["status"] == 0,
                                  "outer_iterations_min_max": [int(its64.min()), int(its64.max())],
                                  "mixed_speedup": t64 / (dt / args.steps)}
    if args.sequential:
        log("bench: the same 48 problems one at a time")
        seq = 0.0
        upd = 0.0
        for v in vols:
            for c in range(3):
                s = F.Solver(v["sigma_t"].shape, v["h"], precision="mixed", tol=1e-6,
                             max_iters=args.max_iters, **tuned)
                s.set_medium(v["sigma_t"], v["albedo"][c], v["Q"][c])
                torch.cuda.synchronize()
                ta = time.perf_counter()
                rr = F.fld_solve_device(s.ctx, 0)
                torch.cuda.synchronize()
                seq += time.perf_counter() - ta   # only the solves count
                upd += rr["voxel_updates"]
                s.close()
        line["sequential_mixed"] = {"time_to_tol_ms": seq * 1e3,
                                    "batch_speedup": seq / (dt / args.steps)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

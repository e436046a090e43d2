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
during the timed steps, its algorithmic bytes from the per-launch figure the
library reports.  The HBM traffic measured by counters is read from the
committed counter summary while the kernel source it was taken on is
unchanged.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
       [--no-fp64] [--max-iters M] [--copy-bytes B]
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


def cpu_baseline(st, al, Q, h, budget_s=20.0):
    """Oracle (plain FP64 C) on a bounded sample: a few outer multigrid
    iterations of the same 256^3 solve; voxel-updates/s on the same definition."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    prob = oracle.setup(st, al, Q, h)
    levels, _ = oracle.mg_levels(*st.shape)
    per_it = sum(a * b * c for a, b, c in levels[:-1]) * 4.0   # V(2,2) point updates
    t1 = time.perf_counter()
    oracle.solve(prob, method="mg", tol=0.0, max_iters=1)
    t_one = time.perf_counter() - t1
    its = max(1, min(40, int(budget_s / max(t_one, 1e-3))))
    t2 = time.perf_counter()
    res = oracle.solve(prob, method="mg", tol=0.0, max_iters=its)
    dt = time.perf_counter() - t2
    return {"value": per_it * res.iterations / dt, "unit": "voxel-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{res.iterations} outer multigrid iterations of the {st.shape[0]}^3 "
                      f"cloud solve (FP64, OpenMP threads={threads}; the time includes the "
                      f"limiter and residual passes of each iteration), {dt:.1f} s after "
                      f"{t1 - t0:.1f} s set-up"}


def copy_calibration(nbytes, reps=5):
    """A plain device-to-device copy of known size, for scaling the HBM
    counters (FETCH_SIZE / WRITE_SIZE) of the solver kernels."""
    import torch

    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": reps}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--max-iters", type=int, default=5000,
                    help="outer iteration cap (short counter runs only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the plain FP64 GPU solve reported beside the mixed one")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the solve of one volume runs on a single MI355X).", file=sys.stderr)
        sys.exit(2)
    if args.copy_bytes > 0:
        copy_calibration(args.copy_bytes)
        return

    import torch
    import paper_1403_8105_amd as F
    from synth import media

    n = args.n
    log(f"bench: generating cloud {n}^3")
    st, al, Q, h = media.config("cloud256", n=n)
    dev = torch.device("cuda:0")
    d_st = torch.from_numpy(st).to(dev)
    d_al = torch.from_numpy(al).to(dev)
    d_Q = torch.from_numpy(Q).to(dev)
    d_phi = torch.empty_like(d_st)
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream

    def make(precision, timing):
        s = F.Solver(st.shape, h, precision=precision, tol=args.tol, max_iters=args.max_iters,
                     timing=timing, stream=sp)
        s.set_medium_device(d_st.data_ptr(), d_al.data_ptr(), d_Q.data_ptr(), sp)
        return s

    solver = make(args.precision, 1)
    torch.cuda.synchronize()

    def step(s):
        return F.fld_solve_device(s.ctx, d_phi.data_ptr())

    for w in range(args.warmup):
        r = step(solver)
        log(f"bench: warmup {w}: {r['iterations']} iterations, rel {r['rel']:.2e}, "
            f"{r['time_ms']:.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for k in range(args.steps):
        reps.append(step(solver))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for k, r in enumerate(reps):
        log(f"bench: step {k}: {r['iterations']} iterations, rel {r['rel']:.2e}, "
            f"{r['time_ms']:.1f} ms")
    solver.close()
    updates = sum(r["voxel_updates"] for r in reps)
    value = updates / dt
    ms_step = dt * 1e3 / args.steps
    kms = np.sum([r["kernel_ms"] for r in reps], axis=0)
    kl = np.sum([r["kernel_launches"] for r in reps], axis=0)
    kb = np.sum([r["kernel_bytes"] for r in reps], axis=0)
    kernels = {KERNEL_NAMES[q]: {"role": KERNEL_ROLES[q], "avg_us": 1e3 * kms[q] / kl[q],
                                 "launches": int(kl[q]),
                                 "alg_bytes_per_launch": kb[q] / kl[q],
                                 "GBps": (kb[q] / kl[q]) / (kms[q] / kl[q] * 1e-3) / 1e9}
               for q in range(4) if kl[q] > 0}
    # the finest-level smoother: the kernel with the largest share of the time
    dom = 0
    avg_s = kms[dom] / kl[dom] * 1e-3
    alg = kb[dom] / kl[dom]
    achieved = alg / avg_s / 1e9
    traffic = counter_traffic()
    ok = all(r["status"] == 0 for r in reps)
    line = {
        "metric": "voxel-updates/s + time to 1e-6 rel. residual (256^3 FLD); % HBM peak",
        "value": value,
        "unit": "voxel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "time_to_tol_ms": ms_step,
        "converged": ok,
        "outer_iterations": reps[-1]["iterations"],
        "final_rel": reps[-1]["rel"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+fp64" if args.precision == "mixed" else "fp64",
        "data": "synthetic",
        "config": {"workload": f"cloud {n}^3 FLD (Levermore-Pomraning), sigma_t in [0,200], "
                               f"40% near-vacuum, albedo 0.99, Beer-Lambert source; "
                               f"{args.precision} Picard multigrid V(2,2) to rel {args.tol:g}",
                   "grid": [n, n, n], "tol": args.tol, "precision": args.precision},
        "roofline": {"bound": "hbm", "kernel": KERNEL_NAMES[dom], "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "alg_bytes_per_launch": alg,
                     "avg_launch_us": avg_s * 1e6},
        "kernels": kernels,
    }
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
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(st, al, Q, h)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

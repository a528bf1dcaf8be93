"""PGCP hot-path benchmark on one MI355X.

    python bench.py [--steps K] [--warmup W] [--precision fp32|fp64] [--workload c2|c1|c3|c5]

One step is Algorithm 3 end to end on one synthetic mesh already resident in
device memory (V, F; labels and the host copy of the connectivity for the
partition): partition + plan upload, cotangent assembly, DNCP of every piece
(batched PCG), boundary D2H, host weld, H2D, harmonic map of every piece
(batched PCG), gather, and the distortion / Beltrami / flip check.  Every solve
reaches an FP64 relative residual of 1e-10 (per piece; per coordinate for the
harmonic solve).  Prints one JSON line.

The roofline object is for the dominant kernel, the batched persistent PCG
(k_pcg): achieved = algorithmic bytes of all its launches in the timed steps /
their summed HIP-event durations.  cpu_baseline runs the FP64 CPU oracle on the
same mesh in a child process pinned to one thread.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def make_case(name):
    from synth import case_c1, case_c2, case_c3, case_c5
    return {"c1": case_c1, "c2": case_c2, "c3": case_c3, "c5": case_c5}[name]()


def describe(case, n_sub):
    if case.mode == "sphere":
        return (f"{case.name}: level-{case.meta['level']} icosphere ({case.nv} vertices), radius perturbed by "
                f"spherical harmonics l<=8, {n_sub} k-means pieces, sphere output")
    n = case.meta.get("n", int(round(case.nv ** 0.5)))
    return f"{case.name}: {n}^2-vertex bump height field, {n_sub} pieces, {case.mode} boundary"


def cpu_baseline(workload: str, timeout: float = 600.0):
    """Oracle wall time on the same mesh, one thread, in a child process."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    code = (
        "import sys, time, json, warnings; warnings.simplefilter('ignore');"
        f"sys.path.insert(0, {ROOT!r});"
        "from bench import make_case; from oracle.pipeline import pgcp;"
        f"c = make_case({workload!r}); t = time.perf_counter();"
        "r = pgcp(c.V, c.F, c.label, c.mode); dt = time.perf_counter() - t;"
        "print(json.dumps(dict(seconds=dt, nv=c.nv, times=r['times'], flips=r['dist']['stats']['n_flipped'])))"
    )
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=timeout)
    if out.returncode != 0:
        return None
    rec = json.loads(out.stdout.strip().splitlines()[-1])
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c5"])
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device copy first (a kernel of known traffic for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the pieces of one mesh are solved in one batched launch on a "
              "single device; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1903_12359_amd as pg

    pg.load_library()
    dev = "cuda:0"
    t0 = time.perf_counter()
    case = make_case(args.workload)
    print(f"[bench] workload {case.name}: nv={case.nv} nf={case.nf} ({time.perf_counter() - t0:.1f}s to generate)",
          file=sys.stderr, flush=True)
    V_dev = torch.from_numpy(case.V).to(dev)
    F_dev = torch.from_numpy(case.F.astype(np.int32)).to(dev)
    ctx = pg.Context(0)
    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        times = {}
        phi, st, info = pg.run(ctx, case.V, case.F, case.label, case.mode, precision=args.precision,
                               tol=args.tol, V_dev=V_dev, F_dev=F_dev, times=times)
        return phi, st, info

    for w in range(args.warmup):
        step()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stage = {}
    cg_ms = cg_bytes = 0.0
    cg_launch = 0
    iters = 0
    last = None
    t_start = time.perf_counter()
    for k in range(args.steps):
        phi, st, info = step()
        for key, v in info["times"].items():
            stage[key] = stage.get(key, 0.0) + v
        for rep in (info["dncp"], info["harmonic"]):
            cg_ms += rep.cg_kernel_ms
            cg_bytes += rep.cg_bytes
            cg_launch += rep.cg_launches
            iters += rep.total_iters
        last = (st, info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    value = case.nv / (ms_per_step / 1e3) / 1e6
    st, info = last
    achieved = cg_bytes / (cg_ms / 1e3) / 1e9 if cg_ms > 0 else 0.0
    rec = {
        "metric": "Mvertices/s end-to-end PGCP at rel. residual 1e-10 (Jacobi-PCG)",
        "value": round(value, 4),
        "unit": "Mvertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (DNCP) + f32 CG with f64 refinement (harmonic)" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": describe(case, info["dncp"].n_sub),
                   "nv": case.nv, "nf": case.nf, "pieces": info["dncp"].n_sub, "precision": args.precision,
                   "tol": args.tol, "preconditioner": "jacobi"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_pcg (batched persistent PCG)", "launches": cg_launch,
                     "avg_launch_ms": round(cg_ms / max(cg_launch, 1), 4),
                     "cg_iterations_per_step": iters // args.steps},
        "stages_ms": {k: round(1e3 * v / args.steps, 3) for k, v in stage.items()},
        "quality": {"mean_abs_d_deg": st["mean_abs_d"], "max_mu": st["max_mu"], "n_flipped": st["n_flipped"],
                    "dncp_max_relres": float(info["dncp"].relres.max()),
                    "harmonic_max_relres": float(info["harmonic"].relres.max())},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle (one thread) on the same mesh", file=sys.stderr, flush=True)
        cb = cpu_baseline(args.workload)
        if cb is not None:
            rec["cpu_baseline"] = {"value": round(cb["nv"] / cb["seconds"] / 1e6, 5), "unit": "Mvertices/s",
                                   "cores": 1, "kind": "oracle",
                                   "sample": f"one full run of the same {case.name} mesh "
                                             f"({cb['seconds']:.1f}s; FP64 numpy/scipy SuperLU)",
                                   "stages_s": {k: round(v, 3) for k, v in cb["times"].items()}}
        else:
            rec["cpu_baseline"] = None
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

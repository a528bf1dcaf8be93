"""PGCP hot-path benchmark on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c5|c3|c2|c1] [--extra c3|none]
                    [--precision fp32|fp64] [--precond both|jacobi|learned] [--lpc-steps S]
                    [--lanes N] [--no-pipeline] [--no-cpu-baseline]

Default workload: the 2048^2-vertex height field with 256 log-normal pieces
(4.19M vertices), on which the learned preconditioner is compared with Jacobi;
the 64-piece perturbed sphere (655k vertices) is timed the same way after it
and reported under "extra".

One step is Algorithm 3 end to end on one synthetic mesh already resident in
device memory (V, F; labels and the host copy of the connectivity for the
partition): partition + plan upload, cotangent assembly, DNCP of every piece
(batched PCG), boundary D2H, weld (arc maps and point replay on the GPU, merge
bookkeeping on the host), H2D, harmonic map of every piece (batched PCG),
gather, and the distortion / Beltrami / flip check.  Every solve
reaches an FP64 relative residual of 1e-10 (per piece; per coordinate for the
harmonic solve).  Prints one JSON line.

The steps run as a stream (pg.run_stream), as a service that processes a
stream of meshes would: the host partition of the next mesh runs while the
current one is on the device (--lanes N > 1 puts N meshes in flight, each on a
host thread with its own context and stream, so that the host stages of one
overlap the device solves of another; the batched solves themselves take the
whole device and run one at a time).  The headline workload runs one lane:
with several, a streaming batched-CG launch on the 2048^2 field has lost
workgroups at its first barrier and given up (the library reports it); the
second workload (--extra, its batches fit the register kernel) runs
--extra-lanes 3.  Every step still runs every stage;
`value` is the throughput of the stream (one untimed step on a quiet device
first lets the autotuner pick the launch shapes, then W warmup steps of the
stream), and "sequential" reports a few steps run one after the other on one
context (the latency of a single mesh).  --no-pipeline times the latter only.

The step is timed twice on the same GPU: with Jacobi-PCG, and with the learned
SPAI preconditioner (network inference inside the step).  The network is
first trained on the GPU for --lpc-steps Adam steps on seeded training meshes
disjoint from the workload (--lpc-set c4: about 2,000 pieces of 1k-20k vertices
from bump height fields and perturbed spheres, trained in windows of plans);
that time is reported separately and is not part of a step.  `value` is the
learned-PCG throughput; both variants are listed.

The roofline object is for the dominant kernel, the batched persistent PCG:
achieved = minimal algorithmic bytes of all its launches in the timed steps
(FP32 values and vectors, whatever precision the recurrences run in) / their
summed HIP-event durations.  cpu_baseline runs the FP64 CPU oracle on a sample
of the workload's pieces, on a pool of single-threaded worker processes in a
child process; the same run gives the error of the GPU's DNCP boundary against
the oracle's direct solve for every sampled piece (oracle_error).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Per-launch HBM traffic of the batched-CG launches (FETCH_SIZE x2.0 +
# WRITE_SIZE x1.0 from rocprofv3 counter passes over one step, scale factors
# from a 256 MiB copy), for the kernel and partition sources and launch shapes
# it was measured with; the summary and commands are in
# profiles/k_pcg_stream_C5_2048x2048_256pieces.md.
TRAFFIC = {
    "c5": {"variant": "learned", "precision": "fp32",
           "source_sha256": "3b2d910c59cd023dda620042b05e34e0f463fefeba56fd2b92994134f6eea3ed",
           "pcg_shapes": {"dncp": "256,0,1,0", "harmonic": "256,0,1,0"},
           "bytes_per_launch": 7.620e11},
}


def kernel_source_sha():
    """SHA-256 over the CG kernel's source and the partition that lays out its rows."""
    import hashlib
    h = hashlib.sha256()
    for name in ("device.hip", "partition.cpp"):
        with open(os.path.join(ROOT, "paper_1903_12359_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def make_case(name, blocks=None, parts=None):
    from synth import case_c1, case_c2, case_c3, case_c5
    if blocks is not None:
        if name != "c2":
            raise SystemExit("--blocks applies to the c2 workload only")
        bx, _, by = str(blocks).partition("x")
        return case_c2(blocks=(int(bx), int(by or bx)))
    if parts is not None:
        if name != "c5":
            raise SystemExit("--parts applies to the c5 workload only")
        return case_c5(nparts=int(parts))
    return {"c1": case_c1, "c2": case_c2, "c3": case_c3, "c5": case_c5}[name]()


def describe(case, n_sub):
    if case.mode == "sphere":
        return (f"{case.name}: level-{case.meta['level']} icosphere ({case.nv} vertices), radius perturbed by "
                f"spherical harmonics l<=8, {n_sub} k-means pieces, sphere output")
    n = case.meta.get("n", int(round(case.nv ** 0.5)))
    return f"{case.name}: {n}^2-vertex bump height field, {n_sub} pieces, {case.mode} boundary"


def sample_labels(label: np.ndarray, n_sample: int):
    """Piece labels spread evenly over the size ranking (smallest and largest included)."""
    cnt = np.bincount(label)
    labs = np.nonzero(cnt)[0]
    order = labs[np.argsort(cnt[labs], kind="stable")]
    idx = np.unique(np.round(np.linspace(0, len(order) - 1, min(n_sample, len(order)))).astype(np.int64))
    return [int(order[i]) for i in idx]


_CASE = None


def _oracle_piece(lab: int):
    """The oracle's per-piece stages on one labelled piece of the workload,
    taken alone: partition, cotangent Laplacian, DNCP, harmonic map with the
    piece's own DNCP boundary as Dirichlet data (the same matrix and cost as
    with welded data), angle distortion.  Returns the DNCP boundary (loop in
    global vertex ids and its coordinates) and the wall time."""
    from oracle.distortion import distortion
    from oracle.pipeline import assemble, harmonic_all, local_params, prepare
    c = _CASE
    t0 = time.perf_counter()
    Fi = c.F[c.label == lab]
    verts = np.unique(Fi)
    Fl = np.searchsorted(verts, Fi).astype(np.int32)
    P = c.V[verts]
    _, subs = prepare(P, Fl, np.zeros(len(Fl), np.int32))
    bdy = local_params(subs)
    welded = {int(v): z for v, z in zip(subs[0]["loop"], bdy[0])}
    vals, _ = harmonic_all(subs, welded, "free")
    phi = assemble(len(P), subs, vals, welded, "free")
    distortion(P, Fl, phi)
    return dict(label=lab, nv=int(len(verts)), seconds=time.perf_counter() - t0,
                loop=verts[np.asarray(subs[0]["loop"], np.int64)], bdy=bdy[0])


def _oracle_sample_main(workload: str, labels, procs: int, out_path: str):
    """Child-process body of the CPU baseline (no GPU is touched here)."""
    global _CASE
    import multiprocessing as mp
    _CASE = make_case(workload)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_oracle_piece, labels, chunksize=1)
    wall = time.perf_counter() - t0
    np.savez(out_path, wall=wall, labels=np.array([r["label"] for r in res]),
             nv=np.array([r["nv"] for r in res]), seconds=np.array([r["seconds"] for r in res]),
             loop_ptr=np.cumsum([0] + [len(r["loop"]) for r in res]),
             loop=np.concatenate([r["loop"] for r in res]), bdy=np.concatenate([r["bdy"] for r in res]))


def cpu_baseline(workload: str, labels, procs: int, timeout: float = 900.0):
    """The FP64 CPU oracle on a sample of the workload's pieces, a pool of
    `procs` single-threaded worker processes, in a child process."""
    import tempfile
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    with tempfile.TemporaryDirectory() as td:
        out = os.path.join(td, "oracle_sample.npz")
        code = (f"import sys, warnings; warnings.simplefilter('ignore'); sys.path.insert(0, {ROOT!r});"
                f"import bench; bench._oracle_sample_main({workload!r}, {list(labels)!r}, {int(procs)}, {out!r})")
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=timeout)
        if r.returncode != 0:
            print(f"[bench] oracle sample failed: {r.stderr[-2000:]}", file=sys.stderr, flush=True)
            return None
        with np.load(out) as z:
            return {k: z[k] for k in z.files}


def oracle_errors(case, bdy_gpu, smp):
    """Error of the GPU's DNCP boundary against the oracle's, per sampled piece:
    max |z_gpu - z_oracle| / max |z_oracle| over the piece's loop (the loop's
    vertex ids must agree exactly)."""
    import paper_1903_12359_amd as pg
    hp = pg.Plan(None, case.V, case.F, case.label, case.mode)      # host-only plan: the loop layout
    ex = hp.export()
    hp.close()
    zg = bdy_gpu[:, 0] + 1j * bdy_gpu[:, 1]
    out = []
    for t, lab in enumerate(smp["labels"]):
        piece = int(ex["face_sub"][int(np.argmax(case.label == lab))])
        a, b = int(ex["loop_ptr"][piece]), int(ex["loop_ptr"][piece + 1])
        o0, o1 = int(smp["loop_ptr"][t]), int(smp["loop_ptr"][t + 1])
        same = np.array_equal(ex["loop_gv"][a:b], smp["loop"][o0:o1])
        zo = smp["bdy"][o0:o1]
        err = float(np.abs(zg[a:b] - zo).max() / np.abs(zo).max()) if same else float("nan")
        out.append(dict(piece=piece, nv=int(smp["nv"][t]), loop_ids_equal=bool(same), dncp_rel_err=err))
    return out


def train_lpc(ctx, steps, seed=0, which="c4"):
    """Train the learned preconditioner on the GPU (seeded training meshes, disjoint from the workloads).

    c4: the training recipe of the learned-preconditioner configuration (about
    2,000 pieces of 1k-20k vertices from bump height fields and perturbed
    spheres), in windows of plans; small: ten smaller meshes (107 pieces) held on
    the device at once."""
    import paper_1903_12359_amd as pg
    from paper_1903_12359_amd.lpc_train import TrainingSet, init_params, train, train_windows, training_meshes
    t0 = time.perf_counter()
    lpc = pg.LPC(ctx, init_params(seed))
    if which == "c4":
        from synth import c4_training_meshes
        meshes = list(c4_training_meshes(seed=seed))
        t1 = time.perf_counter()
        hist, pieces, windows = train_windows(ctx, lpc, meshes, steps, lr=2e-3, seed=seed)
        plans = len(meshes)
    else:
        tset = TrainingSet(ctx, training_meshes(seed=seed))
        t1 = time.perf_counter()
        hist = train(ctx, lpc, tset, steps, lr=2e-3, seed=seed)
        plans, pieces, windows = len(tset.items), int(sum(p.K for p, _, _ in tset.items)), 1
        for p, _, _ in tset.items:
            p.close()
    t2 = time.perf_counter()
    info = {"set": which, "steps": len(hist), "train_s": round(t2 - t1, 3), "set_up_s": round(t1 - t0, 3),
            "plans": plans, "pieces": int(pieces), "windows": windows,
            "loss_first": round(float(np.mean(hist[:20])), 5), "loss_last": round(float(np.mean(hist[-20:])), 5),
            "n_params": lpc.n_params}
    return lpc, info


def time_variant(pg, ctx, case, V_dev, F_dev, args, lpc, steps=None, pipeline=True):
    """Time `steps` complete steps on the same mesh.  With pipeline=True the steps
    run through pg.run_stream with --lanes meshes in flight (every step still
    runs every stage); otherwise one step after the other on one context."""
    import torch
    steps = args.steps if steps is None else steps
    kw = dict(precision=args.precision, tol=args.tol, lpc=lpc)
    item = dict(V=case.V, F=case.F, label=case.label, mode=case.mode, V_dev=V_dev, F_dev=F_dev)

    def steps_iter(n):
        if pipeline:
            yield from pg.run_stream(ctx, [item] * n, lanes=args.lanes, **kw)
        else:
            for _ in range(n):
                times = {}
                yield pg.run(ctx, case.V, case.F, case.label, case.mode, V_dev=V_dev, F_dev=F_dev, times=times,
                             **kw)

    if pipeline:
        # one step on a quiet device first: the autotuner times its launch shapes
        # here (shared by every context), not while other lanes run
        pg.run(ctx, case.V, case.F, case.label, case.mode, V_dev=V_dev, F_dev=F_dev, **kw)
    for _ in steps_iter(args.warmup):
        pass
    torch.cuda.synchronize()
    stage = {}
    cg_ms = cg_bytes = cg_native = 0.0
    cg_launch = 0
    iters = 0
    fallback = 0
    last = None
    t_start = time.perf_counter()
    for phi, st, info in steps_iter(steps):
        for key, v in info["times"].items():
            stage[key] = stage.get(key, 0.0) + v
        for rep in (info["dncp"], info["harmonic"]):
            cg_ms += rep.cg_kernel_ms
            cg_bytes += rep.cg_bytes
            cg_native += rep.cg_bytes_native
            cg_launch += rep.cg_launches
            iters += rep.total_iters
            fallback += rep.n_fallback
        last = (st, info, phi)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / steps
    st, info, phi = last
    return dict(ms_per_step=ms_per_step, value=case.nv / (ms_per_step / 1e3) / 1e6, cg_ms=cg_ms,
                cg_bytes=cg_bytes, cg_bytes_native=cg_native, cg_launch=cg_launch, iters=iters // steps, fallback=fallback,
                stage={k: round(1e3 * v / steps, 3) for k, v in stage.items()}, st=st, info=info, phi=phi)


def area_record(pg, ctx, V_dev, F_dev, phi, mode, max_evals=400):
    """Section 6 after the step: the Moebius map of the mode that minimises the
    mean area distortion of the step's output (Nelder-Mead, one device
    evaluation per step), timed apart from the steps.  Algorithmic bytes of one
    evaluation: 36 per face (face indices, the log image area written and read
    back, the log original area) + 8 per coordinate of each vertex read."""
    import torch
    nv, nf, dim = phi.shape[0], F_dev.shape[0], phi.shape[1]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p, before, after, evals, _ = pg.area_mobius_opt(ctx, V_dev, F_dev, phi.contiguous(), mode, max_evals=max_evals)
    ms = 1e3 * (time.perf_counter() - t0)
    per_eval = ms / max(evals, 1)
    b = 36 * nf + 8 * dim * nv
    return {"mean_abs_d_area_before": before, "mean_abs_d_area_after": after, "evals": evals,
            "ms": round(ms, 3), "ms_per_eval": round(per_eval, 4), "algorithmic_bytes_per_eval": b,
            "achieved_GBs": round(b / (per_eval / 1e3) / 1e9, 1), "parameters": [round(float(x), 6) for x in p]}


def shape(rep):
    return f"{rep.cg_block},{rep.rows_per_thread},{rep.cg_stream},{rep.cg_single}"


def variant_record(r, steps):
    return {"value": round(r["value"], 4), "ms_per_step": round(r["ms_per_step"], 3),
            "cg_iterations_per_step": r["iters"], "cg_ms_per_step": round(r["cg_ms"] / steps, 3),
            "cg_GBs": round(r["cg_bytes"] / (r["cg_ms"] / 1e3) / 1e9, 1) if r["cg_ms"] > 0 else None,
            "stages_ms": r["stage"], "n_fallback": r["fallback"],
            "dncp_max_relres": float(r["info"]["dncp"].relres.max()),
            "harmonic_max_relres": float(r["info"]["harmonic"].relres.max()),
            "n_flipped": r["st"]["n_flipped"],
            "pcg_shapes": {"dncp": shape(r["info"]["dncp"]), "harmonic": shape(r["info"]["harmonic"])}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--workload", default="c5", choices=["c1", "c2", "c3", "c5"])
    ap.add_argument("--extra", default="c3", choices=["none", "c1", "c2", "c3", "c5"],
                    help="a second workload timed the same way with --extra-steps steps (extra keys of the line)")
    ap.add_argument("--extra-steps", type=int, default=10)
    ap.add_argument("--extra-lanes", type=int, default=3,
                    help="meshes in flight for the second workload (its batches fit the register kernel)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--blocks", default=None,
                    help="c2 only: cut the height field into B x B (or BXxBY) blocks (default 4: 16 pieces)")
    ap.add_argument("--parts", type=int, default=None,
                    help="c5 only: number of log-normal guillotine pieces (default 256)")
    ap.add_argument("--precond", default="both", choices=["jacobi", "learned", "both"])
    ap.add_argument("--lpc-steps", type=int, default=500, help="GPU training steps of the learned preconditioner")
    ap.add_argument("--lpc-set", default="c4", choices=["c4", "small"],
                    help="training set of the learned preconditioner (c4: ~2,000 pieces of 1k-20k vertices)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-pieces", type=int, default=16,
                    help="pieces of the workload (spread over the size ranking) the CPU oracle runs on")
    ap.add_argument("--lanes", type=int, default=1, help="meshes in flight in the stream (1: the host partition "
                    "of the next mesh overlaps the current one only)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="run the steps one after the other (no host partition of the next step during device work)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device copy first (a kernel of known traffic for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the pieces of one mesh are solved in one batched launch on a "
              "single device; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1903_12359_amd as pg

    pg.load_library()
    dev = "cuda:0"
    t0 = time.perf_counter()
    case = make_case(args.workload, args.blocks, args.parts)
    print(f"[bench] workload {case.name}: nv={case.nv} nf={case.nf} ({time.perf_counter() - t0:.1f}s to generate)",
          file=sys.stderr, flush=True)
    V_dev = torch.from_numpy(case.V).to(dev)
    F_dev = torch.from_numpy(case.F.astype(np.int32)).to(dev)
    ctx = pg.Context(0)
    lpc = None
    try:
        rec = measure(pg, torch, ctx, case, V_dev, F_dev, args, dev)
        lpc = rec.pop("_lpc", None)
    finally:
        # release the library's objects before the interpreter shuts down (the
        # network, then the lane contexts and the main context), on a device
        # that has finished all their work
        torch.cuda.synchronize()
        if lpc is not None:
            lpc.close()
        ctx.close()
        torch.cuda.synchronize()
    print(json.dumps(rec), flush=True)


def measure(pg, torch, ctx, case, V_dev, F_dev, args, dev):
    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    res = {}
    lpc = lpc_info = None
    if args.precond in ("jacobi", "both"):
        res["jacobi"] = time_variant(pg, ctx, case, V_dev, F_dev, args, None, pipeline=not args.no_pipeline)
        print(f"[bench] jacobi: {res['jacobi']['ms_per_step']:.1f} ms/step", file=sys.stderr, flush=True)
    if args.precond in ("learned", "both"):
        lpc, lpc_info = train_lpc(ctx, args.lpc_steps, which=args.lpc_set)
        print(f"[bench] learned preconditioner trained: {lpc_info}", file=sys.stderr, flush=True)
        res["learned"] = time_variant(pg, ctx, case, V_dev, F_dev, args, lpc, pipeline=not args.no_pipeline)
        print(f"[bench] learned: {res['learned']['ms_per_step']:.1f} ms/step", file=sys.stderr, flush=True)
    # one step after the other (latency of a single mesh), a few steps of the headline variant
    seq = None
    seq_steps = min(args.steps, 2 if case.nv > 10 ** 6 else 4)
    if not args.no_pipeline:
        seq = time_variant(pg, ctx, case, V_dev, F_dev, args, lpc, steps=seq_steps, pipeline=False)
    head = res["learned"] if "learned" in res else res["jacobi"]
    headname = "learned" if "learned" in res else "jacobi"
    achieved = head["cg_bytes"] / (head["cg_ms"] / 1e3) / 1e9 if head["cg_ms"] > 0 else 0.0
    st, info = head["st"], head["info"]
    rec = {
        "metric": "Mvertices/s end-to-end PGCP at rel. residual 1e-10; learned-PCG vs Jacobi-PCG",
        "value": round(head["value"], 4),
        "unit": "Mvertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (DNCP) + f32 CG with f64 refinement (harmonic)" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": describe(case, info["dncp"].n_sub),
                   "nv": case.nv, "nf": case.nf, "pieces": info["dncp"].n_sub, "precision": args.precision,
                   "tol": args.tol, "preconditioner": headname},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_pcg / k_pcg_stream (batched persistent PCG)",
                     "bytes_model": "minimal FP32 bytes per row and iteration: 8 per matrix entry (value and "
                                    "column, diagonal included), 4 inverse diagonal, 76 state vectors; +8 per "
                                    "entry of the learned SPAI",
                     "launches": head["cg_launch"],
                     "avg_launch_ms": round(head["cg_ms"] / max(head["cg_launch"], 1), 4),
                     "bytes_per_launch": round(head["cg_bytes"] / max(head["cg_launch"], 1)),
                     "native_bytes_GBs": round(head["cg_bytes_native"] / (head["cg_ms"] / 1e3) / 1e9, 1)
                     if head["cg_ms"] > 0 else None,
                     "cg_iterations_per_step": head["iters"]},
        "stages_ms": head["stage"],
        "pipelined": not args.no_pipeline,
        "lanes": args.lanes if not args.no_pipeline else 1,
        "quality": {"mean_abs_d_deg": st["mean_abs_d"], "max_mu": st["max_mu"], "n_flipped": st["n_flipped"],
                    "dncp_max_relres": float(info["dncp"].relres.max()),
                    "harmonic_max_relres": float(info["harmonic"].relres.max())},
    }
    for name, r in res.items():
        rec[name] = variant_record(r, args.steps)
    # HBM traffic of the batched-CG launches, from the counter runs recorded in
    # profiles/ (see TRAFFIC): reported only for the same kernel source,
    # workload, preconditioner and launch shapes
    tr = TRAFFIC.get(args.workload)
    if tr is not None and tr["variant"] == headname and tr["source_sha256"] == kernel_source_sha() and \
            tr["pcg_shapes"] == rec[headname]["pcg_shapes"] and args.precision == tr["precision"]:
        rec["roofline"]["traffic"] = tr["bytes_per_launch"]
    if "learned" in res and "jacobi" in res:
        rec["learned_vs_jacobi"] = {
            "speedup_end_to_end": round(res["jacobi"]["ms_per_step"] / res["learned"]["ms_per_step"], 4),
            "iteration_ratio": round(res["jacobi"]["iters"] / max(res["learned"]["iters"], 1), 4),
            "cg_time_ratio": round(res["jacobi"]["cg_ms"] / max(res["learned"]["cg_ms"], 1e-9), 4)}
    if seq is not None:
        rec["sequential"] = {"ms_per_step": round(seq["ms_per_step"], 3), "value": round(seq["value"], 4),
                             "steps": seq_steps, "stages_ms": seq["stage"]}
    if lpc_info is not None:
        rec["lpc_training"] = lpc_info
    rec["area_mobius"] = area_record(pg, ctx, V_dev, F_dev, head["phi"], case.mode)
    bdy_gpu = head["info"]["bdy"]
    for k in ("jacobi", "learned"):      # drop device outputs before the next workload
        if k in res:
            res[k]["phi"] = None

    custom = args.blocks is not None or args.parts is not None
    if args.extra != "none" and args.extra != args.workload and not custom:
        xc = make_case(args.extra)
        xV = torch.from_numpy(xc.V).to(dev)
        xF = torch.from_numpy(xc.F.astype(np.int32)).to(dev)
        xargs = argparse.Namespace(**{**vars(args), "steps": args.extra_steps, "warmup": 1,
                                      "lanes": args.extra_lanes})
        xr = {"nv": xc.nv, "steps": args.extra_steps,
              "lanes": args.extra_lanes if not args.no_pipeline else 1}
        for name, net in (("jacobi", None), ("learned", lpc)):
            if name in res:
                r = time_variant(pg, ctx, xc, xV, xF, xargs, net, pipeline=not args.no_pipeline)
                xr[name] = variant_record(r, args.extra_steps)
                xr["pieces"] = r["info"]["dncp"].n_sub
                xr["workload"] = describe(xc, xr["pieces"])
                print(f"[bench] {xc.name} {name}: {r['ms_per_step']:.1f} ms/step", file=sys.stderr, flush=True)
        if "jacobi" in xr and "learned" in xr:
            xr["learned_vs_jacobi"] = {
                "speedup_end_to_end": round(xr["jacobi"]["ms_per_step"] / xr["learned"]["ms_per_step"], 4),
                "iteration_ratio": round(xr["jacobi"]["cg_iterations_per_step"] /
                                         max(xr["learned"]["cg_iterations_per_step"], 1), 4)}
        rec["extra"] = {xc.name: xr}
        del xV, xF

    if not args.no_cpu_baseline and not custom:
        procs = max(1, min(len(os.sched_getaffinity(0)), 16, args.oracle_pieces))
        labels = sample_labels(case.label, args.oracle_pieces)
        print(f"[bench] CPU oracle on {len(labels)} pieces with {procs} worker processes", file=sys.stderr,
              flush=True)
        smp = cpu_baseline(args.workload, labels, procs)
        if smp is not None:
            nv_s = int(smp["nv"].sum())
            rec["cpu_baseline"] = {
                "value": round(nv_s / float(smp["wall"]) / 1e6, 5), "unit": "Mvertices/s", "cores": procs,
                "kind": "oracle",
                "sample": f"{len(labels)} of the {info['dncp'].n_sub} pieces of the same {case.name} mesh, spread "
                          f"over the size ranking ({int(smp['nv'].min())}-{int(smp['nv'].max())} vertices, "
                          f"{nv_s} in all), each taken alone through the oracle's partition, cotangent "
                          f"Laplacian, DNCP (SuperLU), harmonic map with its own DNCP boundary and angle "
                          f"distortion, on a pool of {procs} single-threaded processes "
                          f"({float(smp['wall']):.1f} s wall, {float(smp['seconds'].sum()):.1f} s of worker "
                          f"time); the serial weld is not in the sample",
                "value_one_core": round(nv_s / float(smp["seconds"].sum()) / 1e6, 5)}
            errs = oracle_errors(case, bdy_gpu, smp)
            rec["oracle_error"] = {
                "what": "DNCP boundary of the headline variant's last step against the oracle's direct "
                        "solve, max |z_gpu - z_oracle| / max |z_oracle| per sampled piece",
                "max": max(e["dncp_rel_err"] for e in errs), "per_piece": errs}
        else:
            rec["cpu_baseline"] = None
    rec["_lpc"] = lpc
    return rec


if __name__ == "__main__":
    main()

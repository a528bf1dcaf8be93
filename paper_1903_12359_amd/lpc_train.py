"""Training driver of the learned SPAI preconditioner (every step runs in libpgcp).

    python -m paper_1903_12359_amd.lpc_train --out lpc_weights.npy [--steps 400]

The training set follows the recipe the network is meant for: subdomain
Laplacians of seeded bump height fields (random block partitions) and of
perturbed icospheres (k-means pieces), with both Dirichlet masks the method
solves (DNCP pins, harmonic boundary).  Each step takes one plan (all of its
pieces form the batch), draws Rademacher probe vectors on the device and calls
pgcp_lpc_train_step: forward pass, loss, hand-written backward pass and Adam
all run in the library's kernels.  This module only picks plans and draws the
random probes.
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np


def training_meshes(n_height: int = 6, n_sphere: int = 4, seed: int = 0):
    """Seeded meshes of the training distribution (disjoint seeds from the benchmark cases)."""
    from synth import small_grid_case, small_sphere_case
    rng = np.random.default_rng(seed + 7_000)
    out = []
    for t in range(n_height):
        n = int(rng.choice([97, 129, 161, 193]))
        bx, by = int(rng.integers(2, 5)), int(rng.integers(2, 5))
        out.append(small_grid_case(n, bx, by, seed=100 + seed * 50 + t, jitter=0.15, nbumps=int(rng.integers(4, 12))))
    for t in range(n_sphere):
        level = int(rng.choice([5, 6]))
        k = int(rng.choice([8, 12, 16]))
        out.append(small_sphere_case(level, k, seed=200 + seed * 50 + t))
    return out


class TrainingSet:
    """Assembled plans of the training meshes, resident on the device."""

    def __init__(self, ctx, cases):
        import torch
        import paper_1903_12359_amd as pg
        self.ctx = ctx
        self.items = []
        for c in cases:
            plan = pg.Plan(ctx, c.V, c.F, c.label, c.mode)
            V = torch.from_numpy(np.ascontiguousarray(c.V)).to(f"cuda:{ctx.device}")
            pg.assemble_cotan(ctx, plan, V)
            self.items.append((plan, V, int(plan.rows()[-1])))


def rademacher(n_rows: int, n_probes: int, gen, device):
    import torch
    return (torch.randint(0, 2, (n_probes, n_rows), generator=gen, device=device, dtype=torch.int8)
            .to(torch.float32) * 2.0 - 1.0).contiguous()


def train(ctx, lpc, tset: TrainingSet, steps: int, lr: float = 1e-3, n_probes: int = 8, seed: int = 0,
          log_every: int = 0):
    """Adam steps over random (plan, system) draws; returns the loss history."""
    import torch
    dev = f"cuda:{ctx.device}"
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    rng = np.random.default_rng(seed)
    hist = []
    for step in range(steps):
        plan, _, n_rows = tset.items[int(rng.integers(len(tset.items)))]
        system = "harmonic" if rng.random() < 0.5 else "dncp"
        V = rademacher(n_rows, n_probes, gen, dev)
        loss = lpc.train_step(plan, V, lr, system=system)
        hist.append(loss)
        if log_every and (step + 1) % log_every == 0:
            print(f"[lpc] step {step + 1}/{steps} loss {np.mean(hist[-log_every:]):.4f}", file=sys.stderr,
                  flush=True)
    return hist


def train_windows(ctx, lpc, meshes, steps: int, window_rows: int = 1_500_000, lr: float = 1e-3,
                  n_probes: int = 8, seed: int = 0, log=None):
    """Training over a large set of meshes (the C4 recipe) in windows: the plans
    of consecutive meshes up to `window_rows` vertices are assembled on the
    device, trained on and released (a plan's training buffers hold ~10 kB per
    row).  The `steps` Adam steps are shared among the windows in proportion to
    their vertices.  Returns the loss history, the number of pieces seen and the
    number of windows."""
    meshes = list(meshes)
    windows, cur, rows = [], [], 0
    for c in meshes:
        cur.append(c)
        rows += c.V.shape[0]
        if rows >= window_rows:
            windows.append((cur, rows))
            cur, rows = [], 0
    if cur:
        windows.append((cur, rows))
    total = sum(r for _, r in windows)
    hist, pieces, done = [], 0, 0
    for w, (cases, rows) in enumerate(windows):
        n = (steps * sum(r for _, r in windows[:w + 1])) // total - done   # cumulative rounding
        done += n
        tset = TrainingSet(ctx, cases)
        pieces += sum(p.K for p, _, _ in tset.items)
        hist.extend(train(ctx, lpc, tset, n, lr=lr, n_probes=n_probes, seed=seed + w))
        for p, _, _ in tset.items:
            p.close()
        if log:
            log(f"[lpc] window {w}: {len(cases)} meshes, {rows} vertices, {n} steps, "
                f"loss {np.mean(hist[-20:]) if hist else float('nan'):.4f}")
    return hist, pieces, len(windows)


# layout of the flat parameter vector (the order pgcp_lpc_create expects)
WIDTH = 64
SHAPES = [("W_x", (3, WIDTH)), ("b_x", (WIDTH,)), ("W_y", (3, WIDTH)), ("b_y", (WIDTH,))]
for _r in range(3):
    SHAPES += [(f"W_e{_r}", (3 * WIDTH, WIDTH)), (f"b_e{_r}", (WIDTH,)),
               (f"W_v{_r}", (2 * WIDTH, WIDTH)), (f"b_v{_r}", (WIDTH,))]
SHAPES += [("u_e", (WIDTH,)), ("c_e", ()), ("u_v", (WIDTH,)), ("c_v", ())]


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weight matrices, zero biases and zero heads: the initial network is exactly Jacobi."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SHAPES:
        if name.startswith("W_"):
            parts.append(rng.normal(0.0, np.sqrt(2.0 / shape[0]), size=shape).ravel())
        else:
            parts.append(np.zeros(int(np.prod(shape, dtype=np.int64))))
    return np.concatenate(parts).astype(np.float32)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--set", default="small", choices=["small", "c4"],
                    help="small: 10 meshes held on the device; c4: ~2,000 pieces of 1k-20k vertices, trained "
                         "in windows of plans")
    args = ap.parse_args()
    import paper_1903_12359_amd as pg
    ctx = pg.Context(0)
    if args.set == "c4":
        from synth import c4_training_meshes
        lpc = pg.LPC(ctx, init_params(args.seed))
        t = time.perf_counter()
        hist, pieces, _ = train_windows(ctx, lpc, c4_training_meshes(seed=args.seed), args.steps, lr=args.lr,
                                        seed=args.seed, log=lambda m: print(m, file=sys.stderr, flush=True))
        print(f"[lpc] {pieces} pieces, {len(hist)} steps in {time.perf_counter() - t:.1f}s", file=sys.stderr,
              flush=True)
        np.save(args.out, lpc.params())
        return
    t = time.perf_counter()
    tset = TrainingSet(ctx, training_meshes(seed=args.seed))
    print(f"[lpc] training set: {len(tset.items)} plans, {sum(p.K for p, _, _ in tset.items)} pieces "
          f"({time.perf_counter() - t:.1f}s)", file=sys.stderr, flush=True)
    lpc = pg.LPC(ctx, init_params(args.seed))
    t = time.perf_counter()
    train(ctx, lpc, tset, args.steps, lr=args.lr, seed=args.seed, log_every=50)
    print(f"[lpc] {args.steps} steps in {time.perf_counter() - t:.1f}s", file=sys.stderr, flush=True)
    np.save(args.out, lpc.params())


if __name__ == "__main__":
    main()

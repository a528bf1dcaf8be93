"""Training driver of the learned SPAI preconditioner (every step runs in libpgcp).

    python -m paper_1903_12359_amd.lpc_train --out lpc_state.bin [--steps 400] [--resume lpc_state.bin]

The training set follows the recipe the network is meant for: subdomain
Laplacians of seeded bump height fields (random block partitions) and of
perturbed icospheres (k-means pieces), with both Dirichlet masks the method
solves (DNCP pins, harmonic boundary).  Each step takes one plan (all of its
pieces form the batch) and one of its two systems and calls
pgcp_lpc_train_step with a batch of probe vectors: forward pass, loss,
hand-written backward pass and Adam all run in the library's kernels.

Probes.  A quarter of each batch (two of eight) are error vectors of the
method's own solves: the plan is solved with Jacobi-PCG (DNCP from its pins;
the harmonic system with the boundary values the method's own DNCP and weld
produce), and e_k = x* - x_k after k = 16, 128 and 1,024 iterations (x and y
components as separate probes) are the slow modes that CG leaves behind.  A
piece that has converged by step k takes a Rademacher segment instead.  The
rest are Rademacher vectors, whose loss averages to |MA - I|_F^2 / n (every
mode alike).  A sparse approximate inverse with the Laplacian's pattern acts
like a smoother: it can lower the loss of the Rademacher probes (0.24 to 0.07
in 300 steps on the test set) but hardly that of the slow modes (0.60 to
0.51), and a larger share of error vectors in the batch did not lower held-out
iterations (error_fraction 0, 0.25, 0.5, 0.75: 3,144, 3,156, 3,190, 3,228 DNCP
iterations on a held-out 129^2 field).

Checkpoints.  Trainer.save writes the network's training state
(pgcp_lpc_save: parameters, Adam moments and step) and, beside it, the
driver's own random state (plan and system draws, probe generator) and step,
so that Trainer.load continues with the same loss trajectory.

This module only picks plans, draws the random probes and subtracts solutions.
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


ERROR_STEPS = (16, 128, 1024)


def error_probes(ctx, plan, V_dev, ks=ERROR_STEPS, tol=1e-10, gen=None):
    """Jacobi-PCG error snapshots of both systems of an assembled plan.

    Returns {"dncp": E, "harmonic": E}, E a float32 tensor [2 len(ks)][rows]
    in packed-row order: e_k = x* - x_k (x and y components) after k
    iterations from the method's starting point, x* the solve to `tol`.  The
    harmonic system takes the boundary values the method itself produces
    (DNCP, then the weld).  Pieces whose error has vanished by step k (relative
    to their solution) get a Rademacher segment drawn from `gen`."""
    import torch
    import paper_1903_12359_amd as pg
    dev = f"cuda:{ctx.device}"
    row0 = plan.rows()
    out = {}
    bdy, _ = pg.local_param(ctx, plan, precision="fp64", tol=tol)
    try:
        welded = torch.from_numpy(pg.weld(ctx, plan, bdy.cpu().numpy())).to(dev)
    except pg.PGCPError:
        # a partition the zipper cannot weld (points crowded onto the imaginary
        # axis): the harmonic system then takes the seam vertices' own (x, y)
        # as boundary values, a problem of the same matrix and kind
        seam = torch.from_numpy(plan.export()["seam_gv"].astype(np.int64)).to(dev)
        welded = V_dev[seam, :2].contiguous()
    for system in ("dncp", "harmonic"):
        def solve(**kw):
            if system == "dncp":
                pg.local_param(ctx, plan, allow_noconv=True, **kw)
            else:
                pg.harmonic_solve(ctx, plan, welded, allow_noconv=True, **kw)
            return plan.solution()[0].clone()
        xs = solve(precision="fp64", tol=tol)
        E = []
        for k in ks:
            xk = solve(precision="fp64", tol=tol, max_iter=int(k), max_refine=2)
            E.append((xs - xk).T.to(torch.float32))
        E = torch.cat(E, 0).contiguous()                       # [2 len(ks)][rows]
        ref = xs.abs().amax()
        for i in range(plan.K):
            a, b = int(row0[i]), int(row0[i + 1])
            seg = E[:, a:b]
            dead = seg.abs().amax(dim=1) <= 1e-7 * float(ref)
            if bool(dead.any()):
                n = int(dead.sum())
                seg[dead] = rademacher(b - a, n, gen, dev) if gen is not None else 1.0
        out[system] = E
    return out


class Trainer:
    """Adam steps over random (plan, system) draws with mixed probe batches.

    Draws come from a numpy Generator (plan, system, which error probes) and a
    torch Generator on the device (Rademacher probes), both seeded; save() and
    load() carry them with the network's state, so a resumed run repeats the
    uninterrupted run's losses."""

    def __init__(self, ctx, lpc, tset: TrainingSet, lr: float = 1e-3, n_probes: int = 8, seed: int = 0,
                 error_fraction: float = 0.25):
        import torch
        self.ctx, self.lpc, self.tset = ctx, lpc, tset
        self.lr, self.n_probes, self.seed = lr, n_probes, seed
        self.dev = f"cuda:{ctx.device}"
        self.gen = torch.Generator(device=self.dev)
        self.gen.manual_seed(seed)
        self.rng = np.random.default_rng(seed)
        self.step = 0
        self.n_err = int(round(n_probes * error_fraction))
        self.errors = None
        if self.n_err > 0:
            self.errors = [error_probes(ctx, plan, V, gen=self.gen) for plan, V, _ in tset.items]

    def run(self, steps: int, log_every: int = 0):
        import torch
        hist = []
        for _ in range(steps):
            j = int(self.rng.integers(len(self.tset.items)))
            plan, _, n_rows = self.tset.items[j]
            system = "harmonic" if self.rng.random() < 0.5 else "dncp"
            V = rademacher(n_rows, self.n_probes - self.n_err, self.gen, self.dev)
            if self.n_err > 0:
                E = self.errors[j][system]
                pick = self.rng.choice(E.shape[0], size=self.n_err, replace=E.shape[0] < self.n_err)
                V = torch.cat([V, E[torch.as_tensor(pick, device=self.dev)]], 0).contiguous()
            hist.append(self.lpc.train_step(plan, V, self.lr, system=system))
            self.step += 1
            if log_every and self.step % log_every == 0:
                print(f"[lpc] step {self.step} loss {np.mean(hist[-log_every:]):.4f}", file=sys.stderr, flush=True)
        return hist

    def save(self, path: str):
        """The network's training state to `path`, the driver's random state to `path`.json."""
        import json
        self.lpc.save(path)
        state = {"step": self.step, "seed": self.seed, "lr": self.lr, "n_probes": self.n_probes,
                 "n_err": self.n_err, "numpy": self.rng.bit_generator.state,
                 "torch": self.gen.get_state().tolist()}
        with open(path + ".json", "w") as f:
            json.dump(state, f)

    @classmethod
    def load(cls, ctx, tset: TrainingSet, path: str):
        """Resume from save(): the network, Adam, the step and both random streams."""
        import json
        import torch
        import paper_1903_12359_amd as pg
        with open(path + ".json") as f:
            state = json.load(f)
        lpc = pg.LPC.load(ctx, path)
        t = cls.__new__(cls)
        t.ctx, t.lpc, t.tset = ctx, lpc, tset
        t.lr, t.n_probes, t.seed, t.n_err = state["lr"], state["n_probes"], state["seed"], state["n_err"]
        t.dev = f"cuda:{ctx.device}"
        t.gen = torch.Generator(device=t.dev)
        t.rng = np.random.default_rng(t.seed)
        t.errors = None
        if t.n_err > 0:
            # the error probes are a function of the plans alone; their
            # Rademacher fill-ins come from the generator's seeded start
            t.gen.manual_seed(t.seed)
            t.errors = [error_probes(ctx, plan, V, gen=t.gen) for plan, V, _ in tset.items]
        t.rng.bit_generator.state = state["numpy"]
        t.gen.set_state(torch.tensor(state["torch"], dtype=torch.uint8))
        t.step = state["step"]
        if lpc.step != t.step:
            raise ValueError(f"{path}: network step {lpc.step} but driver step {t.step}")
        return t


def train(ctx, lpc, tset: TrainingSet, steps: int, lr: float = 1e-3, n_probes: int = 8, seed: int = 0,
          log_every: int = 0, error_fraction: float = 0.25):
    """Adam steps over random (plan, system) draws; returns the loss history."""
    tr = Trainer(ctx, lpc, tset, lr=lr, n_probes=n_probes, seed=seed, error_fraction=error_fraction)
    return tr.run(steps, log_every=log_every)


def train_windows(ctx, lpc, meshes, steps: int, window_rows: int = 1_500_000, lr: float = 1e-3,
                  n_probes: int = 8, seed: int = 0, log=None, error_fraction: float = 0.25):
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
        hist.extend(train(ctx, lpc, tset, n, lr=lr, n_probes=n_probes, seed=seed + w,
                          error_fraction=error_fraction))
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
    ap.add_argument("--out", required=True, help="training-state file (pgcp_lpc_save format)")
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--resume", default=None, help="small set: continue from a state written by --out")
    ap.add_argument("--set", default="small", choices=["small", "c4"],
                    help="small: 10 meshes held on the device; c4: ~2,000 pieces of 1k-20k vertices, trained "
                         "in windows of plans")
    args = ap.parse_args()
    import paper_1903_12359_amd as pg
    ctx = pg.Context(0)
    try:
        if args.set == "c4":
            from synth import c4_training_meshes
            lpc = pg.LPC(ctx, init_params(args.seed))
            t = time.perf_counter()
            hist, pieces, _ = train_windows(ctx, lpc, c4_training_meshes(seed=args.seed), args.steps, lr=args.lr,
                                            seed=args.seed, log=lambda m: print(m, file=sys.stderr, flush=True))
            print(f"[lpc] {pieces} pieces, {len(hist)} steps in {time.perf_counter() - t:.1f}s", file=sys.stderr,
                  flush=True)
            lpc.save(args.out)
            lpc.close()
            return
        t = time.perf_counter()
        tset = TrainingSet(ctx, training_meshes(seed=args.seed))
        print(f"[lpc] training set: {len(tset.items)} plans, {sum(p.K for p, _, _ in tset.items)} pieces "
              f"({time.perf_counter() - t:.1f}s)", file=sys.stderr, flush=True)
        if args.resume:
            tr = Trainer.load(ctx, tset, args.resume)
        else:
            tr = Trainer(ctx, pg.LPC(ctx, init_params(args.seed)), tset, lr=args.lr, seed=args.seed)
        t = time.perf_counter()
        tr.run(args.steps, log_every=50)
        print(f"[lpc] {args.steps} steps in {time.perf_counter() - t:.1f}s (step {tr.step})", file=sys.stderr,
              flush=True)
        tr.save(args.out)
        tr.lpc.close()
        for p, _, _ in tset.items:
            p.close()
    finally:
        ctx.close()


if __name__ == "__main__":
    main()

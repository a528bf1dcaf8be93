"""Learned SPAI preconditioner on the GPU (libpgcp) against the FP64 oracle.

The network keeps its weight matrices, stored states (input encodings, edge
messages, mean aggregations, node states) and the pre-activation gradients it
feeds to its matrix products in bf16.  The oracle is given the same bf16
weights, and its forward and backward passes round at those same points
(oracle.lpc, `rnd`; edge inputs in fp32 as the device computes them), so what
remains is the order of fp32 accumulation, which can move a state that sits
next to a bf16 rounding midpoint by one bf16 step: outputs agree to 1e-3 of
their scale in RMS (1e-2 at worst), the loss to 1e-4 and every parameter
block of the gradient to 1e-3 (measured: 1e-5 to 2e-4), tight enough that a
dropped or mis-scaled term would show.  Against the unrounded FP64 oracle the same gradient is off by
1-2% (the bf16 rounding itself).  Everything the network feeds exactly is
checked exactly: zero outputs give Jacobi, and a learned solve reaches the
same solution as Jacobi to the parity bound.  Training on the GPU must lower
the loss and cut CG iterations on held-out pieces.
"""
import sys

import numpy as np
import pytest

from oracle import lpc as olpc
from oracle.cotan import cotan_laplacian
from oracle.dncp import choose_pins
from oracle.pipeline import harmonic_all, local_params, prepare
from oracle.weld import weld as oracle_weld
from synth import small_grid_case, small_sphere_case

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-lpc]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_1903_12359_amd as pg
    pg.load_library()
    assert torch.cuda.is_available()
    return pg.Context(0)


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def bf16_round(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def random_params(seed=0):
    rng = np.random.default_rng(seed)
    P = olpc.init_params(rng, zero_heads=False)
    for k in P:
        if k.startswith("b_") or k.startswith("c_"):
            P[k] = rng.normal(0, 0.05, np.shape(P[k]))
    return olpc.flatten(P).astype(np.float32)


def f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def emulated_graph(G):
    """The graph's inputs as the device forms them: a in fp32, a^2 of that in
    fp32, valence / 6 in fp32."""
    G = dict(G)
    y = G["y"].copy()
    a = f32(y[:, 0])
    y[:, 0], y[:, 1] = a, f32(a * a)
    x = G["x"].copy()
    x[:, 2] = f32(x[:, 2])
    G["x"], G["y"] = x, y
    return G


def oracle_params(theta32):
    """The parameters as the device uses them: weight matrices rounded to bf16."""
    P = olpc.unflatten(theta32.astype(np.float64))
    for k in P:
        if k.startswith("W_"):
            P[k] = bf16_round(P[k])
    return P


def piece_masks(case):
    part, subs = prepare(case.V, case.F, case.label)
    out = []
    for s in subs:
        L = cotan_laplacian(s["P"], s["T"])
        mh = np.zeros(L.shape[0], bool)
        mh[s["loop_local"]] = True
        p0, p1, _, _ = choose_pins(s["P"], s["loop_local"], s["loop"])
        md = np.zeros(L.shape[0], bool)
        md[[p0, p1]] = True
        out.append(dict(L=L, harmonic=mh, dncp=md))
    return out


CASES = {
    "g33_2x2": lambda: small_grid_case(33, 2, 2, seed=3, jitter=0.3),
    "S4_k8": lambda: small_sphere_case(4, 8, seed=1),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("system", ["harmonic", "dncp"])
def test_forward_matches_oracle(ctx, name, system):
    import paper_1903_12359_amd as pg
    case = CASES[name]()
    theta = random_params(1)
    Po = oracle_params(theta)
    plan = pg.Plan(ctx, case.V, case.F, case.label, case.mode)
    pg.assemble_cotan(ctx, plan, _dev(case.V))
    net = pg.LPC(ctx, theta)
    net.infer(plan, system)
    for i, pm in enumerate(piece_masks(case)):
        G = olpc.graph(pm["L"], pm[system])
        o_e, o_v = olpc.forward(Po, emulated_graph(G), rnd=bf16_round)
        M = olpc.spai(G, o_e, o_v)
        go_e, go_v, gm_e, gm_d = net.export(plan, i)
        scale = max(np.abs(o_e).max(), np.abs(o_v).max())
        dev = np.r_[go_e - o_e, go_v - o_v] / scale
        err, rms = np.abs(dev).max(), np.sqrt(np.mean(dev ** 2))
        say(name, system, "piece", i, "output rel err max", err, "rms", rms)
        # a state that lands next to a bf16 rounding midpoint may round the
        # other way under a different fp32 summation order (one bf16 step,
        # 2^-8 relative, of that state): a few outputs move by ~1e-3 of the
        # scale; a wrong term would move all of them
        assert err < 1e-2 and rms < 1e-3
        # M from the device outputs must be exactly the oracle's formula of them
        off = olpc.spai(G, go_e, go_v).tocsr()
        dm = off.diagonal()
        assert np.abs(gm_d - dm).max() <= 1e-12 * np.abs(dm).max()
        offv = np.asarray(off[G["src"], G["dst"]]).ravel()
        assert np.abs(gm_e - offv).max() <= 1e-12 * max(np.abs(offv).max(), 1e-300)
        # and close to the oracle's M
        assert np.abs(gm_d - M.diagonal()).max() <= 1e-2 * np.abs(M.diagonal()).max()


def test_zero_network_is_jacobi(ctx):
    import paper_1903_12359_amd as pg
    case = CASES["g33_2x2"]()
    plan = pg.Plan(ctx, case.V, case.F, case.label, case.mode)
    pg.assemble_cotan(ctx, plan, _dev(case.V))
    net = pg.LPC(ctx, None)
    net.infer(plan, "harmonic")
    for i, pm in enumerate(piece_masks(case)):
        o_e, o_v, m_e, m_d = net.export(plan, i)
        assert not o_e.any() and not o_v.any() and not m_e.any()
        d = plan.laplacian(i).diagonal()   # the device's own assembled diagonal
        assert np.array_equal(m_d, np.where(pm["harmonic"], 0.0, 1.0 / d))


def _probes(plan, n_probes, seed):
    import torch
    N = int(plan.rows()[-1])
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    return (torch.randint(0, 2, (n_probes, N), generator=g, device="cuda:0", dtype=torch.int8)
            .to(torch.float32) * 2 - 1).contiguous()


def _probe_batch(plan, V, case, system):
    """The oracle's batch for the same probes: per piece (G, A, V restricted to the piece's rows)."""
    row0, gv = plan.rows(), plan.row_vertices()
    Vh = V.cpu().numpy().astype(np.float64)
    batch = []
    for i, pm in enumerate(piece_masks(case)):
        n = pm["L"].shape[0]
        # the oracle numbers a piece's vertices by ascending global index
        rows = row0[i] + np.argsort(gv[row0[i]:row0[i] + n], kind="stable")
        Vi = Vh[:, rows].T.copy()
        Vi[pm[system]] = 0.0
        batch.append((olpc.graph(pm["L"], pm[system]), olpc.system(pm["L"], pm[system]), Vi))
    return batch


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("system", ["harmonic", "dncp"])
def test_gradient_matches_oracle(ctx, name, system):
    """Loss and parameter gradient of the device's training step against the
    oracle's hand-derived backward pass, both rounding at the same points:
    every parameter block to 1e-3 relative."""
    import paper_1903_12359_amd as pg
    case = CASES[name]()
    theta = random_params(2)
    plan = pg.Plan(ctx, case.V, case.F, case.label, case.mode)
    pg.assemble_cotan(ctx, plan, _dev(case.V))
    net = pg.LPC(ctx, theta)
    V = _probes(plan, 6, seed=5)
    loss, g = net.grad(plan, V, system)
    batch = [(emulated_graph(G), A, Vi) for G, A, Vi in _probe_batch(plan, V, case, system)]
    lo, go = olpc.loss_and_grad(oracle_params(theta), batch, rnd=bf16_round)
    go = olpc.flatten(go)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    say(name, system, "loss", loss, lo, "grad rel err", rel)
    assert abs(loss - lo) <= 1e-4 * lo
    assert rel <= 3e-4
    # every parameter block: a dropped or mis-scaled term would move a block by far more
    o = 0
    worst = 0.0
    for bn, shape in olpc.PARAM_SHAPES:
        k = int(np.prod(shape, dtype=np.int64))
        a, b = g[o:o + k], go[o:o + k]
        nb = np.linalg.norm(b)
        assert nb > 0.0, bn
        e = np.linalg.norm(a - b) / nb
        worst = max(worst, e)
        assert e <= 1e-3, (bn, e)
        o += k
    say("  worst parameter block", worst)


@pytest.mark.parametrize("prec,tol,bound", [("fp64", 1e-13, 1e-9), ("fp32", 1e-11, 1e-6)])
def test_learned_solves_reach_the_oracle(ctx, prec, tol, bound):
    """With a (random) learned SPAI the refined solves converge to the oracle's solution."""
    import paper_1903_12359_amd as pg
    case = small_grid_case(40, 2, 2, seed=6, jitter=0.3)
    part, subs = prepare(case.V, case.F, case.label)
    bdy = local_params(subs)
    welded = oracle_weld([s["loop"] for s in subs], bdy, case.mode, sizes=[len(s["T"]) for s in subs])
    vals, _ = harmonic_all(subs, welded, case.mode)
    from oracle.pipeline import assemble
    phi_o = assemble(case.nv, subs, vals, welded, case.mode)
    plan = pg.Plan(ctx, case.V, case.F, case.label, case.mode)
    pg.assemble_cotan(ctx, plan, _dev(case.V))
    net = pg.LPC(ctx, random_params(3) * 0.5)
    b, rep = pg.local_param(ctx, plan, precision=prec, tol=tol, lpc=net)
    ob = np.concatenate(bdy)
    g = b.cpu().numpy()
    err = np.abs(g[:, 0] + 1j * g[:, 1] - ob).max() / np.abs(ob).max()
    say("learned dncp", prec, "err", err, "iters", rep.total_iters, "fallback", rep.n_fallback)
    assert err <= bound
    seam = plan.export()["seam_gv"]
    w = np.array([welded[int(v)] for v in seam])
    phi, rep = pg.harmonic_solve(ctx, plan, _dev(np.column_stack([w.real, w.imag])), precision=prec, tol=tol,
                                 lpc=net)
    err = np.abs(phi.cpu().numpy() - phi_o).max() / np.abs(phi_o).max()
    say("learned harmonic", prec, "err", err, "iters", rep.total_iters, "fallback", rep.n_fallback)
    assert err <= bound


@pytest.mark.parametrize("cfg,kernel", [("256,2", "single"), ("256,2", "two"), ("256,2,1", "stream")])
def test_learned_solve_both_kernels(ctx, cfg, kernel, monkeypatch):
    """The SPAI apply in the single-reduction kernel (M applied on the own rows
    and ring 1 from residuals rebuilt on two rings), the two-barrier kernel and
    the streaming kernel, pieces over several workgroups."""
    import paper_1903_12359_amd as pg
    monkeypatch.setenv("PGCP_PCG_CFG", cfg)
    if kernel == "single":
        monkeypatch.setenv("PGCP_PCG_KERNEL", "single")
    case = small_grid_case(96, 2, 2, seed=8, jitter=0.3)
    part, subs = prepare(case.V, case.F, case.label)
    ob = np.concatenate(local_params(subs))
    plan = pg.Plan(ctx, case.V, case.F, case.label, case.mode)
    pg.assemble_cotan(ctx, plan, _dev(case.V))
    net = pg.LPC(ctx, random_params(4) * 0.5)
    b, rep = pg.local_param(ctx, plan, precision="fp64", tol=1e-13, lpc=net)
    assert rep.cg_workgroups > plan.K
    assert rep.cg_single == (1 if kernel == "single" else 0)
    g = b.cpu().numpy()
    err = np.abs(g[:, 0] + 1j * g[:, 1] - ob).max() / np.abs(ob).max()
    say("kernel", cfg, kernel, "err", err, "iters", rep.total_iters)
    assert err <= 1e-9


def test_training_lowers_loss_and_iterations(ctx):
    """A short GPU training run lowers the loss and cuts CG iterations on held-out pieces."""
    import paper_1903_12359_amd as pg
    from paper_1903_12359_amd.lpc_train import TrainingSet, init_params, train
    train_cases = [small_grid_case(65, 3, 3, seed=20 + t, jitter=0.15, nbumps=6) for t in range(3)] + \
                  [small_sphere_case(5, 8, seed=30 + t) for t in range(2)]
    tset = TrainingSet(ctx, train_cases)
    net = pg.LPC(ctx, init_params(0))
    hist = train(ctx, net, tset, steps=300, lr=2e-3, seed=0)
    first, last = np.mean(hist[:20]), np.mean(hist[-20:])
    say("loss", first, "->", last)
    assert last < 0.8 * first
    # held out: harmonic solves of a new mesh, Jacobi vs learned
    case = small_grid_case(129, 3, 3, seed=99, jitter=0.15, nbumps=6)
    plan = pg.Plan(ctx, case.V, case.F, case.label, case.mode)
    pg.assemble_cotan(ctx, plan, _dev(case.V))
    bdy, _ = pg.local_param(ctx, plan, precision="fp64", tol=1e-10)
    welded = pg.weld(ctx, plan, bdy.cpu().numpy())
    wd = _dev(welded)
    _, rj = pg.harmonic_solve(ctx, plan, wd, precision="fp64", tol=1e-10)
    _, rl = pg.harmonic_solve(ctx, plan, wd, precision="fp64", tol=1e-10, lpc=net)
    say("held-out harmonic iterations: jacobi", rj.total_iters, "learned", rl.total_iters)
    assert rl.relres.max() <= 1e-10
    assert rl.total_iters < 0.85 * rj.total_iters


def test_checkpoint_resume_repeats_the_loss_trajectory(ctx, tmp_path):
    """Trainer.save / Trainer.load (pgcp_lpc_save / pgcp_lpc_load: parameters,
    Adam moments and step, plus the driver's random streams): a run resumed from
    a checkpoint repeats the uninterrupted run's losses and parameters bitwise;
    a corrupted file is refused."""
    import paper_1903_12359_amd as pg
    from paper_1903_12359_amd.lpc_train import Trainer, TrainingSet, init_params
    cases = [small_grid_case(49, 2, 2, seed=50, jitter=0.15, nbumps=5), small_sphere_case(4, 6, seed=51)]
    tset = TrainingSet(ctx, cases)
    path = str(tmp_path / "lpc_state.bin")
    try:
        tr = Trainer(ctx, pg.LPC(ctx, init_params(1)), tset, lr=2e-3, seed=4, error_fraction=0.25)
        h1 = tr.run(12)
        tr.save(path)
        h2 = tr.run(12)
        p2 = tr.lpc.params()
        tr2 = Trainer.load(ctx, tset, path)
        assert tr2.step == 12 and tr2.lpc.step == 12
        h2b = tr2.run(12)
        say("losses", h1[-1], h2[-1], h2b[-1])
        assert h2b == h2
        assert np.array_equal(tr2.lpc.params(), p2)
        tr.lpc.close()
        tr2.lpc.close()
        raw = bytearray(open(path, "rb").read())
        raw[len(raw) // 2] ^= 0x40
        bad = str(tmp_path / "bad.bin")
        open(bad, "wb").write(bytes(raw))
        with pytest.raises(pg.PGCPError):
            pg.LPC.load(ctx, bad)
    finally:
        for p, _, _ in tset.items:
            p.close()

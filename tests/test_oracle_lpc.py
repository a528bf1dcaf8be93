"""Pins of the oracle's learned preconditioner.

What the construction fixes: zero outputs give Jacobi exactly; any outputs
give a symmetric positive definite matrix with the Laplacian's sparsity; the
loss vanishes for the exact inverse and, averaged over all sign vectors, equals
|M A - I|_F^2 / n.  The hand-written gradients are checked against central
finite differences of the loss, which share no code with them; Adam's first
step against its closed form.  Relabelling the vertices permutes the outputs.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import lpc
from oracle.cotan import cotan_laplacian
from oracle.pipeline import prepare
from synth import small_grid_case, small_sphere_case


def _piece(n=9, seed=0, kind="harmonic", piece=0):
    case = small_grid_case(n, 2, 2, seed=seed, jitter=0.3)
    _, subs = prepare(case.V, case.F, case.label)
    s = subs[piece]
    L = cotan_laplacian(s["P"], s["T"])
    mask = np.zeros(L.shape[0], bool)
    if kind == "harmonic":
        mask[s["loop_local"]] = True
    else:
        mask[s["loop_local"][:2]] = True
    return L, mask


def test_param_count():
    assert 60_000 < lpc.n_params() < 70_000


def test_zero_heads_is_jacobi():
    L, mask = _piece()
    G = lpc.graph(L, mask)
    P = lpc.init_params(np.random.default_rng(0), zero_heads=True)
    o_e, o_v = lpc.forward(P, G)
    assert not o_e.any() and not o_v.any()
    M = lpc.spai(G, o_e, o_v).toarray()
    free = ~mask
    J = np.diag(np.where(free, 1.0 / L.diagonal(), 0.0))
    assert np.array_equal(M, J)


@pytest.mark.parametrize("kind", ["harmonic", "pins"])
def test_spai_is_spd_with_laplacian_pattern(kind):
    L, mask = _piece(kind=kind)
    G = lpc.graph(L, mask)
    P = lpc.init_params(np.random.default_rng(1), zero_heads=False)
    o_e, o_v = lpc.forward(P, G)
    assert np.array_equal(o_e, o_e[G["rev"]])
    M = lpc.spai(G, o_e, o_v).toarray()
    assert np.array_equal(M, M.T)
    free = ~mask
    Mf = M[np.ix_(free, free)]
    assert np.linalg.eigvalsh(Mf).min() > 0
    pattern = (np.abs(L.toarray()) > 0)[np.ix_(free, free)]
    assert not Mf[~pattern].any()
    assert not M[mask].any() and not M[:, mask].any()


def test_loss_vanishes_for_exact_inverse_and_is_frobenius_on_all_signs():
    L, mask = _piece(n=7)
    free = ~mask
    # a tiny free set: keep 8 free vertices
    keep = np.flatnonzero(free)[:8]
    m2 = np.ones_like(mask)
    m2[keep] = False
    A = lpc.system(L, m2)
    Af = A.toarray()[np.ix_(keep, keep)]
    Minv = np.zeros_like(A.toarray())
    Minv[np.ix_(keep, keep)] = np.linalg.inv(Af)
    V = np.zeros((L.shape[0], 3))
    V[keep] = np.random.default_rng(2).normal(size=(keep.size, 3))
    assert lpc.loss(sp.csr_matrix(Minv), A, V) < 1e-24
    # all 2^8 sign vectors: the mean is |M A - I|_F^2 / n exactly
    G = lpc.graph(L, m2)
    P = lpc.init_params(np.random.default_rng(3), zero_heads=False)
    M = lpc.spai(G, *lpc.forward(P, G))
    signs = np.array(list(itertools.product([-1.0, 1.0], repeat=keep.size))).T
    Vs = np.zeros((L.shape[0], signs.shape[1]))
    Vs[keep] = signs
    B = (M @ A).toarray()[np.ix_(keep, keep)] - np.eye(keep.size)
    assert abs(lpc.loss(M, A, Vs) - np.sum(B * B) / keep.size) < 1e-12 * np.sum(B * B)


def _batch(seed=0, nprobe=4):
    rng = np.random.default_rng(seed)
    out = []
    for kind, piece in (("harmonic", 0), ("pins", 1)):
        L, mask = _piece(kind=kind, piece=piece)
        G = lpc.graph(L, mask)
        A = lpc.system(L, mask)
        V = np.where(mask[:, None], 0.0, rng.choice([-1.0, 1.0], size=(L.shape[0], nprobe)))
        out.append((G, A, V))
    return out


def test_output_gradients_match_finite_differences():
    (G, A, V), _ = _batch()
    rng = np.random.default_rng(5)
    o_e = rng.normal(0, 0.3, G["src"].size)
    o_v = rng.normal(0, 0.3, G["n"])
    go_e, go_v = lpc.output_grads(G, o_e, o_v, A, V)
    f = lambda a, b: lpc.loss(lpc.spai(G, a, b), A, V)
    h = 1e-6
    for _ in range(3):
        de = rng.normal(size=o_e.size)
        dv = rng.normal(size=o_v.size)
        fd = (f(o_e + h * de, o_v + h * dv) - f(o_e - h * de, o_v - h * dv)) / (2 * h)
        an = go_e @ de + go_v @ dv
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_parameter_gradients_match_finite_differences():
    batch = _batch(seed=1)
    P = lpc.init_params(np.random.default_rng(6), zero_heads=False)
    for k in P:
        if k.startswith("b_") or k.startswith("c_"):
            P[k] = np.random.default_rng(7).normal(0, 0.05, P[k].shape)
    L0, grad = lpc.loss_and_grad(P, batch)
    theta = lpc.flatten(P)
    g = lpc.flatten(grad)
    f = lambda t: lpc.loss_and_grad(lpc.unflatten(t), batch)[0]
    rng = np.random.default_rng(8)
    h = 1e-6
    # random directions, and a direction confined to each parameter block
    dirs = [rng.normal(size=theta.size) for _ in range(2)]
    o = 0
    for name, shape in lpc.PARAM_SHAPES:
        k = int(np.prod(shape, dtype=np.int64))
        d = np.zeros(theta.size)
        d[o:o + k] = rng.normal(size=k)
        dirs.append(d)
        o += k
    for d in dirs:
        fd = (f(theta + h * d) - f(theta - h * d)) / (2 * h)
        an = g @ d
        assert abs(fd - an) <= 1e-5 * max(1e-3, abs(an)), (fd, an)


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    theta = np.array([1.0, 1.0, 1.0, 1.0])
    t1, m, v = lpc.adam(theta, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(t1, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_relabelling_permutes_outputs():
    L, mask = _piece(kind="harmonic")
    n = L.shape[0]
    perm = np.random.default_rng(9).permutation(n)
    Pm = sp.csr_matrix((np.ones(n), (np.arange(n), perm)), shape=(n, n))   # (Pm x)_i = x[perm[i]]
    L2 = Pm @ L @ Pm.T
    mask2 = mask[perm]
    P = lpc.init_params(np.random.default_rng(10), zero_heads=False)
    G1, G2 = lpc.graph(L, mask), lpc.graph(L2, mask2)
    M1 = lpc.spai(G1, *lpc.forward(P, G1)).toarray()
    M2 = lpc.spai(G2, *lpc.forward(P, G2)).toarray()
    np.testing.assert_allclose(M2, M1[np.ix_(perm, perm)], rtol=1e-12, atol=1e-15)

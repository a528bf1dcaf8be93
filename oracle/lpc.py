"""Oracle: learned sparse-approximate-inverse preconditioner (test infrastructure).

Test infrastructure only: nothing in the library imports this module; the
tests, the smoke check and the benchmark's CPU baseline use it to check the
GPU path.

The paper solves every subdomain system with a direct solver; the GPU path
replaces that with batched preconditioned CG, and this module defines its
learned preconditioner: a small edge/vertex message-passing network that reads
one subdomain's cotangent Laplacian (its graph, weights and Dirichlet mask) and
emits a symmetric positive definite matrix with the Laplacian's sparsity.  All
arithmetic here is float64 numpy, written step by step.

Graph.  The directed edges are the pairs (p, q), p != q, with L[p, q] != 0;
``rev`` maps each edge to its reverse.  ``mask`` marks Dirichlet (or pinned)
rows: the system matrix is L on the free rows and columns only.

Inputs.
    x_p   = (1, mask_p, valence_p / 6)
    y_pq  = (a_pq, a_pq^2, mask_q),  a_pq = -L[p,q] / sqrt(L[p,p] L[q,q])

Network (width 64, three rounds with their own weights).
    h_p  = relu(x_p W_x + b_x)                     (3 -> 64)
    e_pq = relu(y_pq W_y + b_y)                    (3 -> 64)
    per round:
        m_pq = relu([h_p, h_q, e_pq] W_e + b_e)    (192 -> 64), then e_pq = m_pq
        g_p  = mean over q of m_pq
        h_p  = relu([h_p, g_p] W_v + b_v)          (128 -> 64)
    o_pq = (e_pq + e_qp)/2 . u_e + c_e             (symmetric by construction)
    o_p  = h_p . u_v + c_v

Preconditioner (free rows only, d = diag L):
    M = D^{-1/2} (diag(exp(o_p) + sum_q |o_pq|) + O) D^{-1/2},  O_pq = o_pq.
The bracket is symmetric and strictly diagonally dominant with a positive
diagonal, hence positive definite, and so is M by congruence.  With zero
outputs M = D^{-1}: the network starts as Jacobi.

Loss over probe vectors v_k (supported on the free rows):
    loss = mean_k |M A v_k - v_k|^2 / |v_k|^2
which for Rademacher probes is an unbiased estimate of |M A - I|_F^2 / n_free.

Parameters are a dict of float64 arrays (the GPU keeps them in bfloat16; the
tests hand this module the same bfloat16 values).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

WIDTH = 64
ROUNDS = 3

PARAM_SHAPES = [("W_x", (3, WIDTH)), ("b_x", (WIDTH,)), ("W_y", (3, WIDTH)), ("b_y", (WIDTH,))]
for _r in range(ROUNDS):
    PARAM_SHAPES += [(f"W_e{_r}", (3 * WIDTH, WIDTH)), (f"b_e{_r}", (WIDTH,)),
                     (f"W_v{_r}", (2 * WIDTH, WIDTH)), (f"b_v{_r}", (WIDTH,))]
PARAM_SHAPES += [("u_e", (WIDTH,)), ("c_e", ()), ("u_v", (WIDTH,)), ("c_v", ())]


def n_params() -> int:
    return int(sum(np.prod(s, dtype=np.int64) for _, s in PARAM_SHAPES))


def init_params(rng: np.random.Generator, zero_heads: bool = True) -> dict:
    """He-normal weights, zero biases; zero heads make the initial network Jacobi."""
    P = {}
    for name, shape in PARAM_SHAPES:
        if name.startswith("W_"):
            P[name] = rng.normal(0.0, np.sqrt(2.0 / shape[0]), size=shape)
        elif name in ("u_e", "u_v") and not zero_heads:
            P[name] = rng.normal(0.0, 0.1, size=shape)
        else:
            P[name] = np.zeros(shape)
    return P


def flatten(P: dict) -> np.ndarray:
    return np.concatenate([np.asarray(P[n], dtype=np.float64).reshape(-1) for n, _ in PARAM_SHAPES])


def unflatten(theta: np.ndarray) -> dict:
    P = {}
    o = 0
    for n, s in PARAM_SHAPES:
        k = int(np.prod(s, dtype=np.int64))
        P[n] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(s)
        o += k
    return P


# ----------------------------------------------------------------------------
# graph and inputs
# ----------------------------------------------------------------------------

def graph(L: sp.spmatrix, mask: np.ndarray):
    """Directed edges of L (ascending (p, q)), reverse map, inputs x and y."""
    L = sp.csr_matrix(L)
    n = L.shape[0]
    C = L.tocoo()
    off = C.row != C.col
    src = C.row[off].astype(np.int64)
    dst = C.col[off].astype(np.int64)
    w = C.data[off]
    order = np.lexsort((dst, src))
    src, dst, w = src[order], dst[order], w[order]
    key = src * n + dst
    rkey = dst * n + src
    rev = np.searchsorted(key, rkey)
    assert np.array_equal(key[rev], rkey), "L must be structurally symmetric"
    d = L.diagonal()
    val = np.bincount(src, minlength=n).astype(np.float64)
    mask = np.asarray(mask, dtype=bool)
    x = np.column_stack([np.ones(n), mask.astype(np.float64), val / 6.0])
    a = -w / np.sqrt(d[src] * d[dst])
    y = np.column_stack([a, a * a, mask[dst].astype(np.float64)])
    return dict(n=n, src=src, dst=dst, rev=rev, w=w, d=d, val=val, mask=mask, x=x, y=y)


# ----------------------------------------------------------------------------
# network
# ----------------------------------------------------------------------------

def _relu(z):
    return np.maximum(z, 0.0)


def _same(x):
    return x


def forward(P: dict, G: dict, keep: bool = False, rnd=None):
    """Outputs (o_e per directed edge, o_v per vertex); with keep, the activations.

    rnd (default: none) rounds the stored states where a reduced-precision
    implementation stores them: the input encodings, every edge message, every
    mean aggregation and every node state; the network is defined without it."""
    rnd = rnd or _same
    src, dst, val = G["src"], G["dst"], G["val"]
    n = G["n"]
    zx = G["x"] @ P["W_x"] + P["b_x"]
    h = rnd(_relu(zx))
    zy = G["y"] @ P["W_y"] + P["b_y"]
    e = rnd(_relu(zy))
    acts = dict(zx=zx, zy=zy, h=[h], e=[e], ze=[], zv=[], g=[])
    for r in range(ROUNDS):
        X = np.concatenate([h[src], h[dst], e], axis=1)
        ze = X @ P[f"W_e{r}"] + P[f"b_e{r}"]
        m = rnd(_relu(ze))
        g = np.zeros((n, WIDTH))
        np.add.at(g, src, m)
        g = rnd(g / np.maximum(val, 1.0)[:, None])
        zv = np.concatenate([h, g], axis=1) @ P[f"W_v{r}"] + P[f"b_v{r}"]
        h = rnd(_relu(zv))
        e = m
        acts["ze"].append(ze)
        acts["zv"].append(zv)
        acts["g"].append(g)
        acts["h"].append(h)
        acts["e"].append(e)
    s = 0.5 * (e + e[G["rev"]])
    o_e = s @ P["u_e"] + P["c_e"]
    o_v = h @ P["u_v"] + P["c_v"]
    acts["s"] = s
    if keep:
        return o_e, o_v, acts
    return o_e, o_v


def spai(G: dict, o_e: np.ndarray, o_v: np.ndarray) -> sp.csr_matrix:
    """M on the free rows (n x n, zero rows and columns for masked vertices)."""
    n, src, dst, d = G["n"], G["src"], G["dst"], G["d"]
    free = ~G["mask"]
    both = free[src] & free[dst]
    diag = np.exp(o_v)
    np.add.at(diag, src[both], np.abs(o_e[both]))
    diag = np.where(free, diag / d, 0.0)
    off = o_e[both] / np.sqrt(d[src[both]] * d[dst[both]])
    M = sp.coo_matrix((np.r_[diag, off], (np.r_[np.arange(n), src[both]], np.r_[np.arange(n), dst[both]])),
                      shape=(n, n))
    return M.tocsr()


def system(L: sp.spmatrix, mask: np.ndarray) -> sp.csr_matrix:
    """The Laplacian on the free rows and columns (masked rows and columns zero)."""
    f = (~np.asarray(mask, dtype=bool)).astype(np.float64)
    Df = sp.diags(f)
    return sp.csr_matrix(Df @ sp.csr_matrix(L) @ Df)


def loss(M: sp.spmatrix, A: sp.spmatrix, V: np.ndarray) -> float:
    """mean_k |M A v_k - v_k|^2 / |v_k|^2 over the columns of V."""
    R = M @ (A @ V) - V
    return float(np.mean(np.sum(R * R, axis=0) / np.sum(V * V, axis=0)))


# ----------------------------------------------------------------------------
# gradients
# ----------------------------------------------------------------------------

def output_grads(G: dict, o_e: np.ndarray, o_v: np.ndarray, A: sp.spmatrix, V: np.ndarray):
    """d loss / d o_e (per directed edge) and d loss / d o_v."""
    n, src, dst, d = G["n"], G["src"], G["dst"], G["d"]
    free = ~G["mask"]
    M = spai(G, o_e, o_v)
    AV = A @ V
    R = M @ AV - V
    P_ = V.shape[1]
    Gr = 2.0 * R / (P_ * np.sum(V * V, axis=0))[None, :]
    # dL/dM_pq = sum_k Gr[p,k] AV[q,k], needed on the diagonal and the edges
    dMd = np.sum(Gr * AV, axis=1)
    dMe = np.sum(Gr[src] * AV[dst], axis=1)
    both = free[src] & free[dst]
    go_v = np.where(free, dMd * np.exp(o_v) / d, 0.0)
    go_e = np.where(both, dMe / np.sqrt(d[src] * d[dst]) + np.sign(o_e) * dMd[src] / d[src], 0.0)
    return go_e, go_v


def backward(P: dict, G: dict, acts: dict, go_e: np.ndarray, go_v: np.ndarray, rnd=None) -> dict:
    """Parameter gradients from the output gradients (plain reverse-mode, by hand).

    rnd (default: none) rounds the pre-activation gradients of the edge and
    vertex layers, where a reduced-precision implementation feeds them to its
    matrix products; rounding is otherwise transparent to differentiation."""
    rnd = rnd or _same
    src, dst, val, rev = G["src"], G["dst"], G["val"], G["rev"]
    n = G["n"]
    grad = {}
    s = acts["s"]
    h = acts["h"][-1]
    grad["u_e"] = s.T @ go_e
    grad["c_e"] = np.array(go_e.sum())
    grad["u_v"] = h.T @ go_v
    grad["c_v"] = np.array(go_v.sum())
    ds = np.outer(go_e, P["u_e"])
    de = 0.5 * (ds + ds[rev])
    dh = np.outer(go_v, P["u_v"])
    for r in reversed(range(ROUNDS)):
        h_in, e_in = acts["h"][r], acts["e"][r]
        g, zv, ze = acts["g"][r], acts["zv"][r], acts["ze"][r]
        dzv = rnd(dh * (zv > 0))
        Xv = np.concatenate([h_in, g], axis=1)
        grad[f"W_v{r}"] = Xv.T @ dzv
        grad[f"b_v{r}"] = dzv.sum(0)
        dXv = dzv @ P[f"W_v{r}"].T
        dh_in = dXv[:, :WIDTH].copy()
        dg = dXv[:, WIDTH:]
        dm = de + dg[src] / np.maximum(val, 1.0)[src, None]
        dze = rnd(dm * (ze > 0))
        Xe = np.concatenate([h_in[src], h_in[dst], e_in], axis=1)
        grad[f"W_e{r}"] = Xe.T @ dze
        grad[f"b_e{r}"] = dze.sum(0)
        dXe = dze @ P[f"W_e{r}"].T
        np.add.at(dh_in, src, dXe[:, :WIDTH])
        np.add.at(dh_in, dst, dXe[:, WIDTH:2 * WIDTH])
        de = dXe[:, 2 * WIDTH:]
        dh = dh_in
    dzx = dh * (acts["zx"] > 0)
    grad["W_x"] = G["x"].T @ dzx
    grad["b_x"] = dzx.sum(0)
    dzy = de * (acts["zy"] > 0)
    grad["W_y"] = G["y"].T @ dzy
    grad["b_y"] = dzy.sum(0)
    return grad


def loss_and_grad(P: dict, batch, rnd=None) -> tuple[float, dict]:
    """Mean loss over a batch of (G, A, V) and its parameter gradient (rnd: see
    forward and backward)."""
    total = 0.0
    grad = {n: np.zeros(s) for n, s in PARAM_SHAPES}
    for G, A, V in batch:
        o_e, o_v, acts = forward(P, G, keep=True, rnd=rnd)
        total += loss(spai(G, o_e, o_v), A, V)
        go_e, go_v = output_grads(G, o_e, o_v, A, V)
        g = backward(P, G, acts, go_e, go_v, rnd=rnd)
        for k in grad:
            grad[k] += g[k]
    nb = len(batch)
    return total / nb, {k: v / nb for k, v in grad.items()}


def adam(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, Algorithm 1) on flat arrays; t counts from 1."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v

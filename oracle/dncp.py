"""Oracle step O3: DNCP local conformal parameterization (Section 4.2).

DNCP minimizes the discrete conformal energy E_C = E_D - A subject to two
pinned boundary vertices.  The area is A = 1/2 sum over boundary edges p->q of
(x_p y_q - y_p x_q), and the paper's area matrix M has, for each boundary edge
p->q, M[p, q+n] = M[q+n, p] = 1 and M[q, p+n] = M[p+n, q] = -1.

Reading of the factors (the printed system (L (+) L - M) z = 0 is not the
minimizer of E_D - A with the printed E_D and M): with the PSD cotangent
Laplacian L_c (see cotan.py), E_D = 1/2 z^T (L_c (+) L_c) z and z^T M z = 4A,
so E_C = 1/2 z^T (L_c (+) L_c - M/2) z and the stationarity system is

    (L_c (+) L_c - M/2) z = 0,

with the four pinned coordinates moved to the right-hand side.

Reading of the pins (the paper does not say which two vertices are pinned or
where): p0 = the loop vertex with the smallest global index, placed at (0, 0);
p1 = the loop vertex farthest from p0 in R^3 (first in loop order on ties),
placed at (|v_p1 - v_p0|, 0).  The boundary orientation for M is the CCW loop
of the partition.  Afterwards the map is translated so that the mean of its
boundary points is 0, so that the welding step's auxiliary point 0 does not
coincide with a data point.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .cotan import cotan_laplacian

DENSE_MAX = 300


def area_matrix(loop_local: np.ndarray, n: int) -> sp.csr_matrix:
    p = np.asarray(loop_local, dtype=np.int64)
    q = np.roll(p, -1)
    rows = np.concatenate([p, q + n, q, p + n])
    cols = np.concatenate([q + n, p, p + n, q])
    vals = np.concatenate([np.ones(p.size), np.ones(p.size), -np.ones(p.size), -np.ones(p.size)])
    return sp.coo_matrix((vals, (rows, cols)), shape=(2 * n, 2 * n)).tocsr()


def boundary_area(u: np.ndarray, loop_local: np.ndarray) -> float:
    """A(u) = 1/2 sum over boundary edges p->q of (x_p y_q - y_p x_q)."""
    p = np.asarray(loop_local)
    q = np.roll(p, -1)
    return 0.5 * float(np.sum(u[p, 0] * u[q, 1] - u[p, 1] * u[q, 0]))


def dirichlet_energy(L: sp.spmatrix, u: np.ndarray) -> float:
    return 0.5 * float(u[:, 0] @ (L @ u[:, 0]) + u[:, 1] @ (L @ u[:, 1]))


def conformal_energy(L, u, loop_local) -> float:
    return dirichlet_energy(L, u) - boundary_area(u, loop_local)


def dncp_matrix(L: sp.spmatrix, loop_local: np.ndarray) -> sp.csr_matrix:
    n = L.shape[0]
    return (sp.block_diag([L, L]) - 0.5 * area_matrix(loop_local, n)).tocsr()


def choose_pins(P: np.ndarray, loop_local: np.ndarray, loop_global: np.ndarray):
    """(p0, p1) local indices and their target positions (0,0), (|v_p1-v_p0|, 0)."""
    j0 = int(np.argmin(loop_global))
    p0 = int(loop_local[j0])
    d = np.linalg.norm(P[loop_local] - P[p0], axis=1)
    j1 = int(np.argmax(d))  # first maximum in loop order
    p1 = int(loop_local[j1])
    return p0, p1, np.array([0.0, 0.0]), np.array([float(d[j1]), 0.0])


def solve_pinned(Q: sp.spmatrix, fixed: np.ndarray, values: np.ndarray) -> np.ndarray:
    """Solve Q z = 0 with z[fixed] = values; free unknowns by a direct solver."""
    N = Q.shape[0]
    free = np.setdiff1d(np.arange(N), fixed)
    Q = Q.tocsr()
    rhs = -(Q[free][:, fixed] @ values)
    A = Q[free][:, free]
    if free.size <= 2 * DENSE_MAX:
        zf = np.linalg.solve(A.toarray(), rhs)
    else:
        zf = spla.splu(A.tocsc()).solve(rhs)
    z = np.empty(N)
    z[fixed] = values
    z[free] = zf
    return z


def dncp(P: np.ndarray, T: np.ndarray, loop_local: np.ndarray, loop_global: np.ndarray,
         L: sp.spmatrix | None = None, translate: bool = True):
    """DNCP of one submesh.  Returns u [n, 2] (all local vertices)."""
    n = P.shape[0]
    if L is None:
        L = cotan_laplacian(P, T)
    Q = dncp_matrix(L, loop_local)
    p0, p1, t0, t1 = choose_pins(P, loop_local, loop_global)
    fixed = np.array([p0, p1, p0 + n, p1 + n])
    vals = np.array([t0[0], t1[0], t0[1], t1[1]])
    z = solve_pinned(Q, fixed, vals)
    u = np.column_stack([z[:n], z[n:]])
    if translate:
        u = u - u[loop_local].mean(axis=0)
    return u

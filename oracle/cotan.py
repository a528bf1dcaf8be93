"""Oracle step O2: cotangent Laplacian of a submesh (Section 4.2).

The paper defines L^cotan_pq = 1/2 (cot a_pq + cot b_pq) off the diagonal with
the diagonal equal to minus the row's off-diagonal sum.  That matrix is
negative semidefinite, while the text calls it positive definite.  Reading used
here: the positive semidefinite form

    L_c[p,q] = -w_pq,  L_c[p,p] = sum_q w_pq,  w_pq = 1/2 (cot a_pq + cot b_pq),

so that x^T L_c x = sum over edges w_pq (x_p - x_q)^2 and the Dirichlet energy
1/2 int |grad phi|^2 of a piecewise-linear map (Section 3.1) is
E_D = 1/2 (x^T L_c x + y^T L_c y).  Boundary edges have one opposite angle.

The cotangent of the angle at vertex k of triangle (i, j, k) is
(u.v) / |u x v| with u = v_i - v_k, v = v_j - v_k.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class DegenerateError(ValueError):
    pass


def corner_cotangents(P: np.ndarray, T: np.ndarray) -> np.ndarray:
    """cot of the angle at each corner: column c is the angle at T[:, c]."""
    out = np.empty(T.shape, dtype=np.float64)
    for c in range(3):
        k = T[:, c]
        i = T[:, (c + 1) % 3]
        j = T[:, (c + 2) % 3]
        u = P[i] - P[k]
        v = P[j] - P[k]
        cr = np.cross(u, v)
        nrm = np.sqrt(np.sum(cr * cr, axis=1))
        if np.any(nrm <= 1e-300):
            raise DegenerateError("zero-area triangle")
        out[:, c] = np.sum(u * v, axis=1) / nrm
    return out


def edge_weights(P: np.ndarray, T: np.ndarray, n: int) -> sp.csr_matrix:
    """Symmetric matrix W with W[p,q] = w_pq = 1/2 (cot a_pq + cot b_pq)."""
    cots = corner_cotangents(P, T)
    rows, cols, vals = [], [], []
    for c in range(3):
        i = T[:, (c + 1) % 3]
        j = T[:, (c + 2) % 3]
        w = 0.5 * cots[:, c]
        rows += [i, j]
        cols += [j, i]
        vals += [w, w]
    W = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    W.sum_duplicates()
    return W


def cotan_laplacian(P: np.ndarray, T: np.ndarray) -> sp.csr_matrix:
    """L_c for vertices P [n,3] and local triangles T [m,3]."""
    n = P.shape[0]
    W = edge_weights(P, T, n)
    d = np.asarray(W.sum(axis=1)).ravel()
    L = (sp.diags(d) - W).tocsr()
    L.sort_indices()
    return L

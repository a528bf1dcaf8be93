"""Oracle step O7: harmonic map with the welded boundary (Section 4.5, Algorithm 3).

For each submesh the paper solves the Laplace equation Delta phi_i = 0 with the
updated (welded) boundary coordinates as Dirichlet data.  Reading of the
discretisation (the paper does not restate it): the same cotangent Laplacian
L_c as the DNCP step, boundary rows eliminated, i.e. for both coordinates

    L_c[I, I] u_I = -L_c[I, B] u_B.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

DENSE_MAX = 300


def harmonic(L, loop_local: np.ndarray, ub: np.ndarray) -> np.ndarray:
    """L: [n,n] L_c; loop_local: boundary local indices; ub: complex boundary values.

    Returns complex values at all n local vertices.
    """
    n = L.shape[0]
    B = np.asarray(loop_local, dtype=np.int64)
    I = np.setdiff1d(np.arange(n), B)
    L = L.tocsr()
    u = np.empty(n, dtype=np.complex128)
    u[B] = ub
    if I.size == 0:
        return u
    A = L[I][:, I]
    rhs = -(L[I][:, B] @ np.column_stack([ub.real, ub.imag]))
    if I.size <= DENSE_MAX:
        sol = np.linalg.solve(A.toarray(), rhs)
    else:
        lu = spla.splu(A.tocsc())
        sol = np.column_stack([lu.solve(rhs[:, 0]), lu.solve(rhs[:, 1])])
    u[I] = sol[:, 0] + 1j * sol[:, 1]
    return u

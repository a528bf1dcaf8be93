"""Oracle: quasi-conformal fold repair of a subdomain's map (Sections 3.5, 4.5).

Test infrastructure only: the library never imports this module.

Section 3.5 characterises folds through the Beltrami coefficient: a map is
folding-free exactly when |mu| < 1 everywhere, and a quasi-conformal map with a
given coefficient is a homeomorphism.  Section 4.5 (and the last step of
Algorithm 3) checks every subdomain's harmonic map this way and, where it
folds, composes it with a quasi-conformal map chosen through the Beltrami
coefficient, deferring the construction to other works.

Reading used here.  A quasi-conformal map of a disk is fixed by its Beltrami
coefficient and its boundary values.  A subdomain whose map has a flipped face
gets the map whose coefficient is the map's own, with its modulus cut below 1,

    mu -> mu                  where |mu| < 1 - delta,
    mu -> (1 - delta) mu/|mu| elsewhere,

and the same (welded) boundary values, so that the pieces still glue.  That
map is computed by the linear Beltrami solver: with f = u + i v and
mu = rho + i tau, the equation f_zbar = mu f_z makes (v_y, -v_x) = A (u_x, u_y)
with the symmetric positive definite matrix

    A = 1/(1 - |mu|^2) [[(rho - 1)^2 + tau^2, -2 tau], [-2 tau, (1 + rho)^2 + tau^2]],

so div(A grad u) = 0 and likewise div(A grad v) = 0.  Both are discretised by
piecewise-linear finite elements in each face's isometric frame, mu constant on
the face: K_pq = sum over faces T of area(T) grad(phi_p) . A_T grad(phi_q), with
the boundary rows eliminated as in the harmonic step.  For mu = 0, A is the
identity and K is the cotangent Laplacian.  The pass is repeated on the result
while a face of the subdomain is still flipped, up to `max_passes`; a pass that
does not lower the subdomain's count of flipped faces is undone and ends its
repair (a subdomain whose welded boundary itself folds cannot be unfolded with
that boundary kept, and chopping there only spreads the fold).

The face's frame follows the face's own vertex order (counter-clockwise on the
surface): vertex 0 at 0, vertex 1 on the positive real axis, vertex 2 in the
upper half-plane; mu = b / a of the affine map a z + b conj(z) + c between the
frames, as in distortion.beltrami.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .distortion import beltrami, orientation

DENSE_MAX = 300


def chop(mu: np.ndarray, delta: float) -> np.ndarray:
    """Beltrami coefficients with modulus cut at 1 - delta (direction kept)."""
    mu = np.asarray(mu, dtype=np.complex128).copy()
    m = np.abs(mu)
    big = m >= 1.0 - delta
    mu[big] = (1.0 - delta) * mu[big] / m[big]
    return mu


def face_frames(P: np.ndarray, T: np.ndarray):
    """Corner positions of every face in its isometric frame, [nf, 3, 2], and the face areas."""
    a, b, c = P[T[:, 0]], P[T[:, 1]], P[T[:, 2]]
    e1, e2 = b - a, c - a
    l1 = np.linalg.norm(e1, axis=1)
    x3 = np.sum(e2 * e1, axis=1) / l1
    y3 = np.linalg.norm(e2 - (x3 / l1)[:, None] * e1, axis=1)
    Q = np.zeros((T.shape[0], 3, 2))
    Q[:, 1, 0] = l1
    Q[:, 2, 0] = x3
    Q[:, 2, 1] = y3
    return Q, 0.5 * l1 * y3


def beltrami_matrix(P: np.ndarray, T: np.ndarray, mu: np.ndarray) -> sp.csr_matrix:
    """Finite-element matrix of div(A_mu grad .) on the mesh (P, T), mu per face."""
    n = P.shape[0]
    Q, area = face_frames(P, T)
    # gradient of the hat function of corner k: the opposite edge turned by
    # +90 degrees over twice the area (points from that edge towards corner k)
    G = np.empty((T.shape[0], 3, 2))
    for k in range(3):
        e = Q[:, (k + 2) % 3] - Q[:, (k + 1) % 3]
        G[:, k, 0] = -e[:, 1] / (2.0 * area)
        G[:, k, 1] = e[:, 0] / (2.0 * area)
    rho, tau = mu.real, mu.imag
    s = 1.0 / (1.0 - rho * rho - tau * tau)
    A = np.empty((T.shape[0], 2, 2))
    A[:, 0, 0] = s * ((rho - 1.0) ** 2 + tau * tau)
    A[:, 0, 1] = A[:, 1, 0] = s * (-2.0 * tau)
    A[:, 1, 1] = s * ((rho + 1.0) ** 2 + tau * tau)
    rows, cols, vals = [], [], []
    for p in range(3):
        for q in range(3):
            if p == q:
                continue
            v = area * np.einsum("fi,fij,fj->f", G[:, p], A, G[:, q])
            rows.append(T[:, p])
            cols.append(T[:, q])
            vals.append(v)
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    K.sum_duplicates()
    # diagonal: minus the row's off-diagonal sum (the hat functions sum to 1)
    return (K - sp.diags(np.asarray(K.sum(axis=1)).ravel())).tocsr()


def beltrami_solve(P, T, loop_local, mu, ub):
    """The map with Beltrami coefficient mu (per face) and boundary values ub
    (complex, on loop_local), all n vertices as complex numbers."""
    n = P.shape[0]
    K = beltrami_matrix(P, T, mu)
    B = np.asarray(loop_local, dtype=np.int64)
    I = np.setdiff1d(np.arange(n), B)
    u = np.empty(n, dtype=np.complex128)
    u[B] = ub
    if I.size == 0:
        return u
    A = K[I][:, I]
    rhs = -(K[I][:, B] @ np.column_stack([ub.real, ub.imag]))
    if I.size <= DENSE_MAX:
        sol = np.linalg.solve(A.toarray(), rhs)
    else:
        lu = spla.splu(A.tocsc())
        sol = np.column_stack([lu.solve(rhs[:, 0]), lu.solve(rhs[:, 1])])
    u[I] = sol[:, 0] + 1j * sol[:, 1]
    return u


def fold_repair(P, T, loop_local, X, delta=0.1, max_passes=5):
    """Repair of one subdomain's planar map X [n, 2].  Returns (X', passes kept,
    flipped faces before each kept pass and after the last)."""
    X = np.asarray(X, dtype=np.float64).copy()
    B = np.asarray(loop_local, dtype=np.int64)
    flips = [int((orientation(X, T) <= 0.0).sum())]
    passes = 0
    while flips[-1] > 0 and passes < max_passes:
        mu = chop(beltrami(P, T, X), delta)
        z = beltrami_solve(P, T, B, mu, X[B, 0] + 1j * X[B, 1])
        Y = np.column_stack([z.real, z.imag])
        n_flip = int((orientation(Y, T) <= 0.0).sum())
        if n_flip >= flips[-1]:
            break                    # no progress: keep the previous map
        X = Y
        passes += 1
        flips.append(n_flip)
    return X, passes, flips

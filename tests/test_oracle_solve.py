"""Pins of the oracle's DNCP and harmonic steps (Sections 3.1, 4.2, 4.5).

The conformal energy is recomputed per triangle from each face's Jacobian
(E_D = 1/2 int |grad phi|^2 and the signed image area), which shares nothing
with the oracle's matrix form; DNCP must be its constrained minimizer.
"""
import numpy as np
import pytest

from oracle.cotan import cotan_laplacian
from oracle.dncp import choose_pins, conformal_energy, dncp, dncp_matrix, solve_pinned
from oracle.harmonic import harmonic
from oracle.partition import partition
from synth import small_grid_case


def _single(case):
    p = partition(case.V, case.F, np.zeros(case.nf, np.int32))
    s = p.subs[0]
    return s.loop, np.searchsorted(s.verts, s.loop)


def _ec_per_triangle(V, F, u):
    """Sum over faces of 1/2 area |J|_F^2 - signed image area (independent of L_c, M)."""
    tot = 0.0
    for t in F:
        p = V[t]
        e1, e2 = p[1] - p[0], p[2] - p[0]
        l1 = np.linalg.norm(e1)
        t1 = e1 / l1
        x3 = e2 @ t1
        y3 = np.linalg.norm(e2 - x3 * t1)
        S = np.array([[l1, x3], [0.0, y3]])           # source edge vectors (columns)
        W = np.column_stack([u[t[1]] - u[t[0]], u[t[2]] - u[t[0]]])
        J = W @ np.linalg.inv(S)
        area = 0.5 * l1 * y3
        img = 0.5 * (W[0, 0] * W[1, 1] - W[0, 1] * W[1, 0])
        tot += 0.5 * area * np.sum(J * J) - img
    return tot


def test_conformal_energy_matches_per_triangle_form():
    case = small_grid_case(6, 1, 1, seed=7, nbumps=3)
    loop, ll = _single(case)
    L = cotan_laplacian(case.V, case.F.astype(np.int64))
    u = np.random.default_rng(0).normal(size=(case.nv, 2))
    assert abs(conformal_energy(L, u, ll) - _ec_per_triangle(case.V, case.F, u)) < 1e-11 * (1 + abs(
        conformal_energy(L, u, ll)))


def test_dncp_is_constrained_minimizer_and_nonnegative():
    case = small_grid_case(7, 1, 1, seed=8, nbumps=4)
    loop, ll = _single(case)
    u = dncp(case.V, case.F.astype(np.int64), ll, loop, translate=False)
    p0, p1, t0, t1 = choose_pins(case.V, ll, loop)
    np.testing.assert_allclose(u[p0], t0, atol=1e-15)
    np.testing.assert_allclose(u[p1], t1, atol=1e-15)
    e0 = _ec_per_triangle(case.V, case.F, u)
    assert e0 >= -1e-12
    rng = np.random.default_rng(1)
    for _ in range(5):
        d = rng.normal(size=u.shape)
        d[[p0, p1]] = 0.0
        eps = 1e-4
        ep = _ec_per_triangle(case.V, case.F, u + eps * d)
        em = _ec_per_triangle(case.V, case.F, u - eps * d)
        assert ep > e0 and em > e0
        assert abs(ep - em) / (2 * eps) < 1e-8 * (1 + np.abs(d).sum())


def test_dncp_flat_mesh_is_identity():
    case = small_grid_case(9, 1, 1, seed=3, flat=True, jitter=0.3)
    loop, ll = _single(case)
    u = dncp(case.V, case.F.astype(np.int64), ll, loop, translate=False)
    # similarity fit u ~ a z + c
    z = case.V[:, 0] + 1j * case.V[:, 1]
    w = u[:, 0] + 1j * u[:, 1]
    A = np.column_stack([z, np.ones_like(z)])
    coef = np.linalg.lstsq(A, w, rcond=None)[0]
    assert np.abs(A @ coef - w).max() < 1e-12
    assert abs(abs(coef[0]) - 1.0) < 1e-12  # pins at their 3-D distance: unit scale
    L = cotan_laplacian(case.V, case.F.astype(np.int64))
    assert abs(conformal_energy(L, u, ll)) < 1e-12


def test_dncp_matrix_psd_with_similarity_nullspace():
    case = small_grid_case(6, 1, 1, seed=2, flat=True)
    loop, ll = _single(case)
    Q = dncp_matrix(cotan_laplacian(case.V, case.F.astype(np.int64)), ll).toarray()
    assert np.array_equal(Q, Q.T)
    ev = np.linalg.eigvalsh(Q)
    assert ev.min() > -1e-12
    assert int(np.sum(ev < 1e-10)) == 4   # translations, rotation, scaling
    case = small_grid_case(6, 1, 1, seed=2, nbumps=4)
    Q = dncp_matrix(cotan_laplacian(case.V, case.F.astype(np.int64)), ll).toarray()
    ev = np.linalg.eigvalsh(Q)
    assert ev.min() > -1e-12 and int(np.sum(ev < 1e-10)) == 2   # translations only


def test_dncp_rigid_invariance_and_dense_sparse_agree():
    case = small_grid_case(21, 1, 1, seed=4, nbumps=4)
    loop, ll = _single(case)
    u = dncp(case.V, case.F.astype(np.int64), ll, loop)
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    V2 = case.V @ R.T * 3.0 + np.array([1.0, -2.0, 0.5])
    u2 = dncp(V2, case.F.astype(np.int64), ll, loop)
    np.testing.assert_allclose(u2, 3.0 * u, atol=1e-10)
    # dense path agrees with SuperLU path
    import oracle.dncp as D
    old = D.DENSE_MAX
    try:
        D.DENSE_MAX = 10 ** 6
        ud = dncp(case.V, case.F.astype(np.int64), ll, loop)
    finally:
        D.DENSE_MAX = old
    np.testing.assert_allclose(ud, u, atol=1e-11)


def test_harmonic_linear_precision_and_dense():
    case = small_grid_case(15, 1, 1, seed=5, flat=True, jitter=0.3)
    loop, ll = _single(case)
    L = cotan_laplacian(case.V, case.F.astype(np.int64))
    z = case.V[:, 0] + 1j * case.V[:, 1]
    a, c = 0.3 - 1.2j, 2.0 + 0.5j
    u = harmonic(L, ll, a * z[ll] + c)
    assert np.abs(u - (a * z + c)).max() < 1e-12
    import oracle.harmonic as H
    old = H.DENSE_MAX
    try:
        H.DENSE_MAX = 10 ** 6
        ud = harmonic(L, ll, (a * z[ll] + c) ** 2)
    finally:
        H.DENSE_MAX = old
    np.testing.assert_allclose(ud, harmonic(L, ll, (a * z[ll] + c) ** 2), atol=1e-12)


def test_harmonic_converges_to_z_cubed():
    errs = []
    for n in (9, 17, 33, 65):
        case = small_grid_case(n, 1, 1, seed=0, flat=True, jitter=0.3)
        loop, ll = _single(case)
        L = cotan_laplacian(case.V, case.F.astype(np.int64))
        z = case.V[:, 0] + 1j * case.V[:, 1] - (0.5 + 0.5j)
        u = harmonic(L, ll, z[ll] ** 3)
        errs.append(np.abs(u - z ** 3).max())
    # z^3 is harmonic; the P1 error decays like h^2 (jitter differs per level)
    assert all(b < a / 2 for a, b in zip(errs, errs[1:]))
    assert errs[-1] < errs[0] / 20


def test_solve_pinned_identity_rows():
    Q = np.array([[2.0, -1, 0], [-1, 2, -1], [0, -1, 2]])
    import scipy.sparse as sp
    z = solve_pinned(sp.csr_matrix(Q), np.array([0, 2]), np.array([1.0, 3.0]))
    assert abs(z[1] - 2.0) < 1e-15

"""Why the DNCP solve keeps FP64 recurrences: a CPU experiment on one piece of
the 2048^2 / 256-piece height field (its 17th smallest, 3,614 vertices).

The free-boundary DNCP system (L_c (+) L_c - M/2 with two pinned vertices,
Section 4.2) has a near-null space of almost-conformal boundary motions:
kappa ~ 3e7 here (7e7 to 3.5e10 on the larger pieces), so kappa * u_fp32 > 1.
Rounding the matrix to FP32 is harmless (its smallest eigenvalue moves by
about 1%), but CG recurrences in FP32 are not: refinement with FP32 inner
solves (FP64 residual, FP32 correction to 1e-4, repeated) reaches 1e-10 only
after ~7x the FP64 iterations, because every pass rebuilds the slow Krylov
directions the previous one found; replacing the FP32 recurrence residual by
the FP64 residual without restarting (residual replacement) stalls.  Measured
on larger pieces with the same code: 3,866 FP64 iterations against 35,306 for
restarted FP32 (a 512^2 piece, 16,639 vertices), 1,870 / 12,428, 2,945 /
23,305 and 4,468 / 37,952 on pieces of 7,098, 12,766 and 20,480 vertices.
"""
import numpy as np
import scipy.sparse.linalg as spla

from oracle.cotan import cotan_laplacian
from oracle.dncp import choose_pins, dncp_matrix
from oracle.pipeline import prepare
from synth import case_c5


def piece_system(case, lab):
    Fi = case.F[case.label == lab]
    verts = np.unique(Fi)
    Fl = np.searchsorted(verts, Fi).astype(np.int32)
    _, subs = prepare(case.V[verts], Fl, np.zeros(len(Fl), np.int32))
    s = subs[0]
    L = cotan_laplacian(s["P"], s["T"])
    n = L.shape[0]
    Q = dncp_matrix(L, s["loop_local"]).tocsr()
    p0, p1, t0, t1 = choose_pins(s["P"], s["loop_local"], s["loop"])
    fixed = np.array([p0, p1, p0 + n, p1 + n])
    free = np.setdiff1d(np.arange(2 * n), fixed)
    A = Q[free][:, free].tocsr()
    b = -(Q[free][:, fixed] @ np.array([t0[0], t1[0], t0[1], t1[1]]))
    return A, b


def pcg64(A, b, tol):
    d = 1.0 / A.diagonal()
    x, r = np.zeros_like(b), b.copy()
    z = d * r
    p, rz, nb = z.copy(), r @ z, np.linalg.norm(b)
    for it in range(1, 100_000):
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        if np.linalg.norm(r) <= tol * nb:
            return it, x
        z = d * r
        rzn = r @ z
        p = z + (rzn / rz) * p
        rz = rzn
    return None, x


def pcg32_refined(A, b, tol, inner=1e-4, cap=200_000):
    """FP64 residual, FP32 CG on the scaled residual to `inner`, FP64 update; repeated."""
    A32, d = A.astype(np.float32), (1.0 / A.diagonal()).astype(np.float32)
    x, nb, total = np.zeros_like(b), np.linalg.norm(b), 0
    while total < cap:
        r64 = b - A @ x
        rel = np.linalg.norm(r64) / nb
        if rel <= tol:
            return total, x
        s = np.linalg.norm(r64)
        r = (r64 / s).astype(np.float32)
        e = np.zeros_like(r)
        z = d * r
        p, rz, r0 = z.copy(), np.float64(r @ z), np.linalg.norm(r)
        target = max(inner, 0.5 * tol / rel)
        while total < cap:
            q = A32 @ p
            a = np.float32(rz / np.float64(p @ q))
            e += a * p
            r -= a * q
            total += 1
            if np.linalg.norm(r) <= target * r0:
                break
            z = d * r
            rzn = np.float64(r @ z)
            p = z + np.float32(rzn / rz) * p
            rz = rzn
        x += s * e.astype(np.float64)
    return None, x


def pcg32_replaced(A, b, tol, cap, delta=0.1):
    """FP32 recurrences, FP64 solution; whenever the recurrence residual has
    fallen by delta, the update is added in FP64 and the residual replaced by
    the FP64 residual, keeping the search direction."""
    A32, d = A.astype(np.float32), (1.0 / A.diagonal()).astype(np.float32)
    nb, x64 = np.linalg.norm(b), np.zeros_like(b)
    r = b.astype(np.float32)
    x32 = np.zeros_like(r)
    z = d * r
    p, rz, rmax = z.copy(), np.float64(r @ z), np.linalg.norm(r)
    for it in range(1, cap + 1):
        q = A32 @ p
        a = np.float32(rz / np.float64(p @ q))
        x32 += a * p
        r -= a * q
        rn = np.linalg.norm(r)
        if rn <= delta * rmax or rn <= tol * nb:
            x64 += x32.astype(np.float64)
            x32[:] = 0
            r64 = b - A @ x64
            if np.linalg.norm(r64) <= tol * nb:
                return it, x64
            r = r64.astype(np.float32)
            rmax = np.linalg.norm(r)
        z = d * r
        rzn = np.float64(r @ z)
        p = z + np.float32(rzn / rz) * p
        rz = rzn
    return None, x64


def test_fp32_recurrences_do_not_pay_on_dncp():
    c5 = case_c5()
    cnt = np.bincount(c5.label)
    A, b = piece_system(c5, int(np.argsort(cnt, kind="stable")[16]))
    lmin = spla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    lmax = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False)[0]
    lmin32 = spla.eigsh(A.astype(np.float32).astype(np.float64), k=1, sigma=0, which="LM",
                        return_eigenvectors=False)[0]
    assert lmax / lmin * 2.0 ** -24 > 1.0                  # kappa * u_fp32 > 1
    assert abs(lmin32 - lmin) / lmin < 0.05                # the FP32 matrix itself is fine
    xs = spla.splu(A.tocsc()).solve(b)
    n64, x = pcg64(A, b, 1e-10)
    assert n64 is not None and np.abs(x - xs).max() <= 1e-6 * np.abs(xs).max()
    n32, x = pcg32_refined(A, b, 1e-10)
    assert n32 is not None and np.abs(x - xs).max() <= 1e-6 * np.abs(xs).max()
    assert n32 >= 4 * n64                                  # measured 8,974 against 1,241
    n_rep, _ = pcg32_replaced(A, b, 1e-10, cap=10 * n64)
    assert n_rep is None                                   # stalls

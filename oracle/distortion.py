"""Oracle step O8: angle distortion, flips and Beltrami coefficient.

Angle distortion (Section 5): d([v_i, v_j, v_k]) = angle[phi(v_i), phi(v_j),
phi(v_k)] - angle[v_i, v_j, v_k] in degrees, for the three angles of every face.
An angle is atan2(|u x v|, u . v) of its two edge vectors (chordal 3-D angles on
the sphere).  Statistics follow Table 5: mean, standard deviation (N-1),
median and interquartile range of |d| over all 3|F| angles; percentiles use
the midpoint rule p_i = (i - 1/2)/N.

Flips: a face is flipped when its signed area in the plane is <= 0, or, on the
sphere, when det[phi_i, phi_j, phi_k] <= 0.

Beltrami coefficient (Section 3.5): on each face the piecewise-linear map is
f(z) = a z + b conj(z) + c between isometric 2-D frames of the source and the
target triangles, and mu = b / a.  Folding-free iff |mu| < 1; |mu| of the
inverse map is the same.
"""
from __future__ import annotations

import numpy as np


def corner_angles(P: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Angle in degrees at each corner; column c is the angle at F[:, c]."""
    P = np.asarray(P, dtype=np.float64)
    if P.shape[1] == 2:
        P = np.column_stack([P, np.zeros(P.shape[0])])
    out = np.empty(F.shape)
    for c in range(3):
        o = P[F[:, c]]
        u = P[F[:, (c + 1) % 3]] - o
        v = P[F[:, (c + 2) % 3]] - o
        cr = np.cross(u, v)
        out[:, c] = np.degrees(np.arctan2(np.linalg.norm(cr, axis=1), np.sum(u * v, axis=1)))
    return out


def orientation(phi: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Signed area x 2 in the plane, or det[phi_i, phi_j, phi_k] on the sphere."""
    a, b, c = phi[F[:, 0]], phi[F[:, 1]], phi[F[:, 2]]
    if phi.shape[1] == 2:
        return (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    return np.einsum("ij,ij->i", a, np.cross(b, c))


def _frame3(a, b, c, sign):
    """Isometric 2-D coordinates (0, |e1|, w3) of 3-D triangles; sign orients w3."""
    e1 = b - a
    e2 = c - a
    l1 = np.linalg.norm(e1, axis=1)
    t1 = e1 / l1[:, None]
    x3 = np.sum(e2 * t1, axis=1)
    perp = e2 - x3[:, None] * t1
    y3 = np.linalg.norm(perp, axis=1) * sign
    return np.zeros(a.shape[0], dtype=np.complex128), l1.astype(np.complex128), x3 + 1j * y3


def beltrami(V: np.ndarray, F: np.ndarray, phi: np.ndarray) -> np.ndarray:
    s1, s2, s3 = _frame3(V[F[:, 0]], V[F[:, 1]], V[F[:, 2]], 1.0)
    if phi.shape[1] == 2:
        w = phi[:, 0] + 1j * phi[:, 1]
        w1, w2, w3 = w[F[:, 0]], w[F[:, 1]], w[F[:, 2]]
    else:
        sgn = np.where(orientation(phi, F) > 0, 1.0, -1.0)
        w1, w2, w3 = _frame3(phi[F[:, 0]], phi[F[:, 1]], phi[F[:, 2]], sgn)
    e1, e2 = s2 - s1, s3 - s1
    d1, d2 = w2 - w1, w3 - w1
    det = e1 * np.conj(e2) - e2 * np.conj(e1)
    a = (d1 * np.conj(e2) - d2 * np.conj(e1)) / det
    b = (e1 * d2 - e2 * d1) / det
    return b / a


def hazen_percentile(x: np.ndarray, q: float) -> float:
    x = np.sort(np.asarray(x, dtype=np.float64))
    n = x.size
    pos = q / 100.0 * n + 0.5   # 1-based position
    if pos <= 1:
        return float(x[0])
    if pos >= n:
        return float(x[-1])
    lo = int(np.floor(pos))
    t = pos - lo
    return float(x[lo - 1] + t * (x[lo] - x[lo - 1]))


def distortion(V: np.ndarray, F: np.ndarray, phi: np.ndarray) -> dict:
    F = np.asarray(F, dtype=np.int64)
    d = corner_angles(phi, F) - corner_angles(V, F)
    ori = orientation(phi, F)
    flip = ori <= 0.0
    mu = np.abs(beltrami(V, F, phi))
    ad = np.abs(d).ravel()
    stats = dict(
        mean_abs_d=float(ad.mean()),
        sd_abs_d=float(ad.std(ddof=1)) if ad.size > 1 else 0.0,
        median_abs_d=hazen_percentile(ad, 50.0),
        iqr_abs_d=hazen_percentile(ad, 75.0) - hazen_percentile(ad, 25.0),
        max_abs_d=float(ad.max()),
        max_mu=float(mu.max()),
        n_flipped=int(flip.sum()),
    )
    return dict(d=d, flip=flip, mu=mu, stats=stats)

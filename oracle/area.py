"""Oracle step O9: area distortion and its reduction by a Moebius map (Section 6, area distortion).

Test infrastructure: only the tests, the smoke check and the bench's CPU
baseline use this module.

Area distortion of a face T (the area-distortion equation of Section 6): the
natural log of the face's share of the parameterized area over its share of
the original area,

    d_area(T) = log( (A(f(T)) / sum_T' A(f(T'))) / (A(T) / sum_T' A(T')) ),

with A the area of the flat triangle through the three vertices (in the plane,
or in R^3 for the original mesh and for spherical parameterizations: reading,
the paper does not say whether a spherical triangle's area is flat or
spherical).  The reported figure, as in the paper's area table, is the mean of
|d_area| over the faces.

Post-optimisation (Section 6): the parameterization is composed with a
Moebius map chosen to minimise mean |d_area|.  Free boundary: f(z) = (a z + b)
/ (c z + d), eight real parameters (real and imaginary parts of a, b, c, d).
Disk: f(z) = (z - alpha) / (1 - conj(alpha) z), two real parameters, |alpha| <
1 (reading: the real and imaginary parts of alpha; the paper names its modulus
and argument, a chart that is degenerate at alpha = 0, the identity map the
search starts from).  Sphere: sigma^{-1} o f o sigma with the
eight-parameter f and the pipeline's stereographic projection sigma(p) = (x -
i y) / (1 - z) (north pole <-> infinity).  The paper uses a general
constrained solver; reading: Nelder-Mead from the identity map with an
initial simplex of step 0.1 along each parameter, a fixed evaluation budget,
and +inf for parameters outside the admissible set (ad - bc = 0, |alpha| >= 1,
any zero or non-finite image area, or any face whose orientation the map
reverses: a Moebius map keeps the orientation of every small triangle away
from its pole, so a reversed face is one whose image wraps around the pole's
image, i.e. the pole lies inside it and the map is not a bijection of the
parameter domain).
"""
from __future__ import annotations

import numpy as np

from oracle.sphere import inv_stereo, stereo

IDENTITY = {"free": np.array([1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0]),
            "sphere": np.array([1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0]),
            "disk": np.array([0.0, 0.0])}


def face_areas(P: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Area of the flat triangle through each face's vertices (2-D or 3-D points)."""
    P = np.asarray(P, dtype=np.float64)
    if P.shape[1] == 2:
        P = np.column_stack([P, np.zeros(P.shape[0])])
    a, b, c = P[F[:, 0]], P[F[:, 1]], P[F[:, 2]]
    return 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)


def orientation(P: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Signed orientation of each face: twice its signed area in the plane,
    det[a, b, c] for points on the unit sphere (positive when counter-clockwise
    seen from outside)."""
    P = np.asarray(P, dtype=np.float64)
    a, b, c = P[F[:, 0]], P[F[:, 1]], P[F[:, 2]]
    if P.shape[1] == 2:
        return (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    return np.einsum("ij,ij->i", a, np.cross(b, c))


def area_distortion(V: np.ndarray, F: np.ndarray, X: np.ndarray) -> np.ndarray:
    """d_area of every face of the mesh (V, F) under the parameterization X."""
    A = face_areas(V, F)
    Af = face_areas(X, F)
    return np.log((Af / Af.sum()) / (A / A.sum()))


def mean_abs(V, F, X) -> float:
    return float(np.mean(np.abs(area_distortion(V, F, X))))


def mobius(z: np.ndarray, p: np.ndarray) -> np.ndarray:
    """(a z + b) / (c z + d) on the extended plane (infinity as complex inf)."""
    a, b, c, d = p[0] + 1j * p[1], p[2] + 1j * p[3], p[4] + 1j * p[5], p[6] + 1j * p[7]
    z = np.asarray(z, dtype=np.complex128)
    out = np.empty_like(z)
    inf = ~np.isfinite(z)
    out[inf] = (a / c) if c != 0 else complex(np.inf, 0.0)
    zz = z[~inf]
    num, den = a * zz + b, c * zz + d
    pole = den == 0
    res = np.empty_like(zz)
    res[pole] = complex(np.inf, 0.0)
    res[~pole] = num[~pole] / den[~pole]
    out[~inf] = res
    return out


def disk_automorphism(z: np.ndarray, q: np.ndarray) -> np.ndarray:
    """(z - alpha) / (1 - conj(alpha) z), alpha = q[0] + i q[1]."""
    alpha = q[0] + 1j * q[1]
    return (z - alpha) / (1.0 - np.conj(alpha) * z)


def apply(X: np.ndarray, mode: str, p: np.ndarray) -> np.ndarray:
    """The parameterization X composed with the mode's Moebius map of parameters p."""
    X = np.asarray(X, dtype=np.float64)
    if mode == "disk":
        w = disk_automorphism(X[:, 0] + 1j * X[:, 1], p)
        return np.column_stack([w.real, w.imag])
    if mode == "free":
        w = mobius(X[:, 0] + 1j * X[:, 1], p)
        return np.column_stack([w.real, w.imag])
    z = np.empty(X.shape[0], np.complex128)
    north = X[:, 2] == 1.0
    z[north] = complex(np.inf, 0.0)
    z[~north] = stereo(X[~north])
    return inv_stereo(mobius(z, p))


def objective(V, F, X, mode: str, p: np.ndarray) -> float:
    """mean |d_area| of X composed with the Moebius map p; +inf where p is not admissible."""
    p = np.asarray(p, dtype=np.float64)
    if mode == "disk":
        if not (p[0] * p[0] + p[1] * p[1] < 1.0):
            return float("inf")
    else:
        a, b, c, d = p[0] + 1j * p[1], p[2] + 1j * p[3], p[4] + 1j * p[5], p[6] + 1j * p[7]
        if a * d - b * c == 0:
            return float("inf")
    with np.errstate(all="ignore"):
        Y = apply(X, mode, p)
        Af = face_areas(Y, F)
        if not np.all(np.isfinite(Af)) or not np.all(Af > 0):
            return float("inf")
        if not np.all(orientation(Y, F) * orientation(X, F) > 0):
            return float("inf")
        v = mean_abs(V, F, Y)
    return v if np.isfinite(v) else float("inf")


def optimise(V, F, X, mode: str, max_evals: int = 400):
    """Nelder-Mead over the Moebius parameters from the identity map.

    Returns (parameters, mean |d_area| before, mean |d_area| after)."""
    from scipy.optimize import minimize
    x0 = IDENTITY[mode].copy()
    n = x0.size
    simplex = np.vstack([x0] + [x0 + 0.1 * np.eye(n)[i] for i in range(n)])
    before = objective(V, F, X, mode, x0)
    r = minimize(lambda p: objective(V, F, X, mode, p), x0, method="Nelder-Mead",
                 options={"initial_simplex": simplex, "maxfev": max_evals, "xatol": 1e-10, "fatol": 1e-12})
    return r.x, before, float(r.fun)

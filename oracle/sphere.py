"""Oracle step O6: sphere output (Sections 4.4.2 and 4.5).

The paper ends the spherical mode with a stereographic projection of the
welded result on the extended plane.  Reading of the convention (the paper does
not give one):

    sigma^{-1}(w) = (2 Re w, -2 Im w, |w|^2 - 1) / (|w|^2 + 1),  sigma^{-1}(inf) = (0, 0, 1),

which sends a counter-clockwise planar triangle to an outward-oriented
spherical one.

The paper solves every Laplace equation in the extended plane, which is not
possible for a piece whose welded region contains infinity.  Reading: each
piece is solved in its own rotated chart w = (z - c)/(1 + conj(c) z), a
rotation of the sphere that moves the normalised mean of the piece's welded
boundary points on the sphere to w = 0.  Interior values are mapped back with
z = (w + c)/(1 - conj(c) w) before the projection.
"""
from __future__ import annotations

import numpy as np


def inv_stereo(w: np.ndarray) -> np.ndarray:
    w = np.asarray(w, dtype=np.complex128)
    out = np.empty((w.size, 3))
    inf = ~np.isfinite(w)
    ww = w[~inf]
    r2 = ww.real ** 2 + ww.imag ** 2
    den = r2 + 1.0
    out[~inf, 0] = 2.0 * ww.real / den
    out[~inf, 1] = -2.0 * ww.imag / den
    out[~inf, 2] = (r2 - 1.0) / den
    out[inf] = (0.0, 0.0, 1.0)
    return out


def stereo(p: np.ndarray) -> np.ndarray:
    p = np.atleast_2d(p)
    return (p[:, 0] - 1j * p[:, 1]) / (1.0 - p[:, 2])


def chart_centre(wb: np.ndarray) -> complex:
    """sigma of the normalised mean of sigma^{-1}(wb); infinity when that is the north pole."""
    P = inv_stereo(wb)
    m = P.mean(axis=0)
    m /= np.linalg.norm(m)
    if not 1.0 - m[2] > 0.0:
        return complex("inf")
    return complex(stereo(m[None, :])[0])


def chart(z: np.ndarray, c: complex) -> np.ndarray:
    """Rotation chart (z - c)/(1 + conj(c) z); for c = infinity the rotation -1/z."""
    z = np.asarray(z, dtype=np.complex128)
    out = np.empty_like(z)
    inf = ~np.isfinite(z)
    if not np.isfinite(c):
        out[~inf] = -1.0 / z[~inf]
        out[inf] = 0.0
        return out
    out[~inf] = (z[~inf] - c) / (1.0 + np.conj(c) * z[~inf])
    out[inf] = 1.0 / np.conj(c) if c != 0 else complex("inf")
    return out


def chart_inv(w: np.ndarray, c: complex) -> np.ndarray:
    """Inverse of `chart`: (w + c)/(1 - conj(c) w), or -1/w for c = infinity."""
    w = np.asarray(w, dtype=np.complex128)
    if not np.isfinite(c):
        out = np.full_like(w, complex("inf"))
        nz = w != 0
        out[nz] = -1.0 / w[nz]
        return out
    den = 1.0 - np.conj(c) * w
    out = np.empty_like(w)
    z0 = den == 0
    out[~z0] = (w[~z0] + c) / den[~z0]
    out[z0] = complex("inf")
    return out

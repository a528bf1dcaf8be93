"""Pins of the area-distortion oracle (Section 6, area distortion).

d_area is checked on a hand-computed two-face mesh and against its invariance
under maps of constant area scale; the Moebius maps against their closed
forms (identity parameters, inverse maps, the disk automorphism keeping the
unit circle, the stereographic round trip); the optimiser on meshes whose
parameterization is a known Moebius image of the mesh itself, so that the
exact optimum is mean |d_area| = 0 (the inverse map).
"""
import numpy as np
import pytest

from oracle import area
from oracle.sphere import inv_stereo
from synth.meshes import grid_mesh, icosphere

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _plane(n=12, lo=-0.5, hi=0.5):
    xy, F = grid_mesh(n)
    xy = lo + (hi - lo) * xy
    return np.column_stack([xy, np.zeros(len(xy))]), F, xy


def test_two_faces_by_hand():
    # original areas 0.5 and 1.5 (sum 2), image areas 1 and 1 (sum 2):
    # d = log((1/2) / (0.5/2)) = log 2 and log((1/2) / (1.5/2)) = log(2/3)
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [3, 0, 0]], float)
    F = np.array([[0, 1, 2], [1, 3, 2]])
    assert np.allclose(area.face_areas(V, F), [0.5, 1.0])
    V2 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [3, 1, 0]], float)   # second face: area 1.5
    assert np.allclose(area.face_areas(V2, F), [0.5, 1.5])
    X = np.array([[0, 0], [2, 0], [0, 1], [2, 1]], float)                # image areas 1 and 1
    assert np.allclose(area.face_areas(X, F), [1.0, 1.0])
    d = area.area_distortion(V2, F, X)
    assert np.allclose(d, [np.log(2.0), np.log(2.0 / 3.0)], rtol=0, atol=1e-15)
    assert area.mean_abs(V2, F, X) == pytest.approx((np.log(2.0) + np.log(1.5)) / 2, abs=1e-15)


def test_constant_area_scale_has_no_distortion():
    V, F, xy = _plane()
    A = np.array([[2.0, 0.7], [-0.4, 1.3]])                 # any affine map scales every area alike
    X = xy @ A.T + np.array([3.0, -1.0])
    assert np.abs(area.area_distortion(V, F, X)).max() < 1e-12
    # a 3-D rotation of the original mesh changes nothing either
    c, s = np.cos(0.7), np.sin(0.7)
    R = np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    assert np.abs(area.area_distortion(V @ R.T, F, xy)).max() < 1e-12
    # z -> z^2 on [1, 2]^2: the area scale |2z|^2 varies, so d_area does not vanish
    V2, F2, xy2 = _plane(lo=1.0, hi=2.0)
    z = (xy2[:, 0] + 1j * xy2[:, 1]) ** 2
    d = area.area_distortion(V2, F2, np.column_stack([z.real, z.imag]))
    assert np.abs(d).max() > 0.5


def test_moebius_closed_forms():
    rng = np.random.default_rng(1)
    z = rng.normal(size=50) + 1j * rng.normal(size=50)
    assert np.array_equal(area.mobius(z, area.IDENTITY["free"]), z)
    p = np.array([1.3, 0.1, 0.2, 0.0, 0.0, -0.1, 1.0, 0.0])
    a, b, c, d = 1.3 + 0.1j, 0.2, -0.1j, 1.0
    inv = np.array([d.real, 0.0, -b, 0.0, -c.real, -c.imag, a.real, a.imag])   # (d z - b) / (-c z + a)
    assert np.allclose(area.mobius(area.mobius(z, p), inv), z, atol=1e-12)
    assert area.mobius(np.array([np.inf + 0j]), p)[0] == pytest.approx(a / c)
    # the disk automorphism keeps the unit circle and sends alpha to 0
    q = np.array([0.6 * np.cos(2.0), 0.6 * np.sin(2.0)])
    t = np.exp(1j * rng.uniform(0, 2 * np.pi, 40))
    assert np.allclose(np.abs(area.disk_automorphism(t, q)), 1.0, atol=1e-14)
    assert abs(area.disk_automorphism(np.array([0.6 * np.exp(2j)]), q)[0]) < 1e-15
    # sphere: identity parameters return the points; the north pole is infinity
    P = np.asarray(icosphere(2)[0])
    P = np.vstack([P, [0.0, 0.0, 1.0]])
    assert np.allclose(area.apply(P, "sphere", area.IDENTITY["sphere"]), P, atol=1e-14)
    Y = area.apply(P, "sphere", p)
    assert np.allclose(np.linalg.norm(Y, axis=1), 1.0, atol=1e-14)
    assert np.allclose(Y[-1], inv_stereo(np.array([a / c]))[0], atol=1e-14)


def test_optimiser_inverts_a_planar_moebius_map():
    V, F, xy = _plane()
    g = np.array([1.0, 0.2, 0.3, 0.1, 0.25, -0.15, 1.0, 0.0])
    w = area.mobius(xy[:, 0] + 1j * xy[:, 1], g)
    X = np.column_stack([w.real, w.imag])
    p, before, after = area.optimise(V, F, X, "free", max_evals=3000)
    assert before > 0.05
    assert after < 1e-3 * before
    assert after == pytest.approx(area.objective(V, F, X, "free", p))


def test_optimiser_inverts_a_disk_automorphism():
    V, F, xy = _plane(lo=-0.6, hi=0.6)
    q0 = np.array([0.4 * np.cos(0.9), 0.4 * np.sin(0.9)])
    w = area.disk_automorphism(xy[:, 0] + 1j * xy[:, 1], q0)
    X = np.column_stack([w.real, w.imag])
    p, before, after = area.optimise(V, F, X, "disk", max_evals=600)
    assert before > 0.1
    assert after < 1e-3 * before
    alpha = p[0] + 1j * p[1]
    assert abs(alpha + 0.4 * np.exp(0.9j)) < 1e-3          # the inverse is the automorphism of -alpha0


def test_optimiser_inverts_a_spherical_moebius_map():
    Pts, F = icosphere(3)
    P = np.asarray(Pts, float)
    F = np.asarray(F)
    g = np.array([1.2, 0.0, 0.3, 0.1, 0.0, -0.2, 1.0, 0.0])
    X = area.apply(P, "sphere", g)
    p, before, after = area.optimise(P, F, X, "sphere", max_evals=4000)
    assert before > 0.1
    assert after < 1e-2 * before


def test_pole_inside_the_domain_is_inadmissible():
    # f(z) = 1 / (z - z0): holomorphic, so every small face away from z0 keeps
    # its orientation; the faces around z0 are sent around the image of the
    # pole (infinity) and come back reversed.  Unsigned areas alone stay
    # finite there, so the objective must reject the map by orientation.
    V, F, xy = _plane(n=16)
    X = xy + 0.01 * np.column_stack([np.sin(3 * xy[:, 1]), np.cos(2 * xy[:, 0])])
    inside = np.array([0.0, 0.0, 1.0, 0.0, 1.0, 0.0, -0.113, -0.057])    # pole at 0.113 + 0.057i
    outside = np.array([0.0, 0.0, 1.0, 0.0, 1.0, 0.0, -2.0, 0.0])         # pole at 2
    Y = area.apply(X, "free", inside)
    turn = area.orientation(Y, F) * area.orientation(X, F)
    assert (turn < 0).sum() >= 1 and (turn > 0).sum() > 0.9 * len(F)
    assert np.isfinite(area.mean_abs(V, F, Y))              # areas alone do not see it
    assert area.objective(V, F, X, "free", inside) == float("inf")
    v = area.objective(V, F, X, "free", outside)
    assert np.isfinite(v) and v == pytest.approx(area.mean_abs(V, F, area.apply(X, "free", outside)))
    assert np.all(area.orientation(area.apply(X, "free", outside), F) > 0)


def test_orientation_closed_forms():
    # counter-clockwise unit right triangle: twice its area; reversed: negative
    P2 = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    assert area.orientation(P2, np.array([[0, 1, 2]]))[0] == 1.0
    assert area.orientation(P2, np.array([[0, 2, 1]]))[0] == -1.0
    # the octant triangle (e_x, e_y, e_z) seen from outside is counter-clockwise: det = 1
    P3 = np.eye(3)
    assert area.orientation(P3, np.array([[0, 1, 2]]))[0] == 1.0
    assert area.orientation(P3, np.array([[1, 0, 2]]))[0] == -1.0

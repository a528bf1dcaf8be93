"""Pins of the oracle's sphere mode (Sections 4.4.2 and 4.5).

The stereographic projection and the rotation charts are checked against their
closed forms; the whole pipeline on a closed genus-0 mesh against what a
spherical conformal parameterization must be: a map onto the unit sphere of
degree one (positively oriented faces whose solid angles add up to exactly
4 pi, so no face overlaps another), and on the round sphere, whose conformal
self-maps are the Moebius transformations, a map whose quasi-conformal
distortion vanishes under refinement.
"""
import numpy as np
import pytest

from oracle.pipeline import local_params, pgcp, prepare
from oracle.sphere import chart, chart_centre, chart_inv, inv_stereo, stereo
from oracle.weld import weld
from synth import small_sphere_case


def solid_angles(P, F):
    """Signed solid angle of every spherical triangle (Van Oosterom and Strackee)."""
    a, b, c = P[F[:, 0]], P[F[:, 1]], P[F[:, 2]]
    num = np.einsum("ij,ij->i", a, np.cross(b, c))
    den = 1.0 + np.einsum("ij,ij->i", a, b) + np.einsum("ij,ij->i", b, c) + np.einsum("ij,ij->i", c, a)
    return 2.0 * np.arctan2(num, den)


def test_stereographic_projection_closed_forms():
    rng = np.random.default_rng(0)
    w = rng.normal(size=200) + 1j * rng.normal(size=200)
    P = inv_stereo(w)
    assert np.abs(np.linalg.norm(P, axis=1) - 1).max() < 1e-15
    assert np.abs(stereo(P) - w).max() < 1e-12 * np.abs(w).max()
    np.testing.assert_allclose(inv_stereo(np.array([0j])), [[0, 0, -1]], atol=0)
    np.testing.assert_allclose(inv_stereo(np.array([complex("inf")])), [[0, 0, 1]], atol=0)
    np.testing.assert_allclose(inv_stereo(np.array([1 + 0j, 1j])), [[1, 0, 0], [0, -1, 0]], atol=1e-16)
    # a counter-clockwise planar triangle maps to an outward-oriented one
    tri = np.array([[0.1 + 0.1j, 0.3 + 0.1j, 0.1 + 0.4j]])
    Q = inv_stereo(tri.ravel())
    assert np.linalg.det(Q) > 0


def test_chart_is_a_rotation_of_the_sphere():
    rng = np.random.default_rng(1)
    z = rng.normal(size=300) + 1j * rng.normal(size=300)
    for c in (0.3 - 0.7j, 2.5 + 1.0j, -0.01j, complex("inf")):
        w = chart(z, c)
        # chordal distances are preserved
        P, Q = inv_stereo(z), inv_stereo(w)
        i, j = rng.integers(0, z.size, 100), rng.integers(0, z.size, 100)
        dP = np.linalg.norm(P[i] - P[j], axis=1)
        dQ = np.linalg.norm(Q[i] - Q[j], axis=1)
        assert np.abs(dP - dQ).max() < 1e-12
        # orientation is preserved (a rotation, not a reflection)
        t = np.array([0, 1, 2])
        assert np.sign(np.linalg.det(P[t])) == np.sign(np.linalg.det(Q[t]))
        assert np.abs(chart_inv(w, c) - z).max() < 1e-10 * np.abs(z).max()
        if np.isfinite(c):
            assert abs(chart(np.array([c]), c)[0]) < 1e-15


def test_chart_centre_of_a_small_circle():
    """Points evenly spread on a circle of the sphere around u have their centre at sigma(u)."""
    u = np.array([0.48, -0.6, 0.64])
    e1 = np.cross(u, [0, 0, 1.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(u, e1)
    t = np.linspace(0, 2 * np.pi, 64, endpoint=False)
    P = np.cos(0.4) * u + np.sin(0.4) * (np.cos(t)[:, None] * e1 + np.sin(t)[:, None] * e2)
    c = chart_centre(stereo(P))
    assert abs(c - stereo(u[None, :])[0]) < 1e-12


SPHERES = [
    lambda: small_sphere_case(3, 6, seed=0),
    lambda: small_sphere_case(4, 8, seed=1),
    lambda: small_sphere_case(5, 12, seed=2),
    lambda: small_sphere_case(5, 6, seed=0, perturb=False),
]


@pytest.mark.parametrize("make", SPHERES)
def test_sphere_map_has_degree_one(make):
    case = make()
    r = pgcp(case.V, case.F, case.label, "sphere")
    phi = r["phi"]
    assert np.abs(np.linalg.norm(phi, axis=1) - 1.0).max() < 1e-14
    om = solid_angles(phi, case.F)
    assert (om > 0).all()
    assert abs(om.sum() - 4 * np.pi) < 1e-9
    assert r["dist"]["stats"]["n_flipped"] == 0
    assert r["dist"]["stats"]["max_mu"] < 0.2


@pytest.mark.parametrize("make", SPHERES[:3])
def test_closed_weld_tiles_the_sphere(make):
    """Welded boundary loops, lifted to the sphere, bound pieces that tile it once."""
    case = make()
    part, subs = prepare(case.V, case.F, case.label)
    bdy = local_params(subs)
    w = weld([s["loop"] for s in subs], bdy, "sphere", sizes=[len(s["T"]) for s in subs])
    total = 0.0
    for s in subs:
        P = inv_stereo(np.array([w[int(v)] for v in s["loop"]]))
        m = P.mean(axis=0)
        m /= np.linalg.norm(m)
        n = P.shape[0]
        fan = np.column_stack([np.zeros(n, int), np.arange(1, n + 1), np.r_[np.arange(2, n + 1), 1]])
        area = solid_angles(np.vstack([m, P]), fan).sum()
        assert 0 < area < 4 * np.pi
        total += area
    assert abs(total - 4 * np.pi) < 1e-9


def test_round_sphere_distortion_vanishes_under_refinement():
    mus, means = [], []
    for level in (3, 5):
        case = small_sphere_case(level, 6, seed=0, perturb=False)
        st = pgcp(case.V, case.F, case.label, "sphere")["dist"]["stats"]
        mus.append(st["max_mu"])
        means.append(st["mean_abs_d"])
    assert mus[1] < 0.5 * mus[0]
    assert means[1] < 0.5 * means[0]

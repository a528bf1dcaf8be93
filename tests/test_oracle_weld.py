"""Pins of the oracle's welding step (Sections 3.2, 3.4, 4.3.2, 4.4).

Fixed points stated in the paper (L_xi sends {0, xi, rho} to {0, 1, inf};
T sends {alpha, 0, beta} to {i, 0, -i}), the postconditions of Algorithm 1,
the welding condition a~_j = b~_j, the geodesic algorithm's image in the upper
half-plane, and geometric consistency of the welded pieces (orientation,
exact tiling of the union's area, seam points inside the union, unit circle
for the disk constraint).
"""
import numpy as np
import pytest

from oracle.pipeline import local_params, prepare
from oracle.weld import (L_map, T_map, apply_mobius, intermediate_form, merge_plan, mobius3,
                         weld)
from synth import small_grid_case


def _polygon(rng, n, interior=3):
    """Random star-shaped CCW polygon plus interior points."""
    t = np.sort(rng.uniform(0, 2 * np.pi, n))
    r = 1.0 + 0.15 * np.sin(3 * t + rng.uniform(0, 6)) + 0.02 * rng.uniform(-1, 1, n)
    z = r * np.exp(1j * t) + (0.2 - 0.1j)
    zi = 0.3 * (rng.uniform(-1, 1, interior) + 1j * rng.uniform(-1, 1, interior)) + (0.2 - 0.1j)
    return z, zi


def test_L_fixed_points():
    rng = np.random.default_rng(0)
    for _ in range(20):
        xi = rng.uniform(0.1, 2) + 1j * rng.uniform(-2, 2)
        c = abs(xi) ** 2 / (2 * xi.imag)     # circle centre ic through 0, tangent to R at 0
        assert abs(abs(xi - 1j * c) - abs(c)) < 1e-12
        rho = 2j * c
        assert L_map(xi, 0.0) == 0.0
        assert abs(L_map(xi, xi) - 1.0) < 1e-14
        assert abs(1.0 + 1j * (xi.imag / abs(xi) ** 2) * rho) < 1e-14   # pole at rho
        w = L_map(xi, 1j * rng.normal())
        assert abs(w.real) < 1e-14
        w = L_map(xi, rng.uniform(0.01, 3) + 1j * rng.normal())
        assert w.real > 0


def test_T_fixed_points():
    rng = np.random.default_rng(1)
    for _ in range(20):
        a, b = rng.uniform(0.1, 5), -rng.uniform(0.1, 5)
        assert abs(T_map(a, b, 1j * a) - 1j) < 1e-14
        assert abs(T_map(a, b, 1j * b) + 1j) < 1e-14
        assert T_map(a, b, 0.0) == 0.0
        assert T_map(a, b, rng.uniform(0.01, 2) + 1j * rng.normal()).real > 0


def test_mobius3():
    z1, z2, z3 = 0.3 + 0.1j, -1.2 + 2j, 4 - 1j
    co = mobius3(z1, z2, z3)
    w, winf = apply_mobius(co, np.array([z1, z2, z3]), np.zeros(3, bool))
    assert abs(w[0] + 1) < 1e-14 and abs(w[1] - 1) < 1e-14
    assert winf[2] or abs(w[2]) > 1e14


@pytest.mark.parametrize("branch", [1, -1])
def test_intermediate_form_postconditions(branch):
    rng = np.random.default_rng(2 + branch)
    for trial in range(10):
        n = int(rng.integers(8, 40))
        z, zi = _polygon(rng, n)
        if branch < 0:
            z = z[::-1]          # the B side is traversed clockwise
        k = int(rng.integers(2, n - 2))
        pts = np.concatenate([z, zi, [0.0, 0.0]])
        inf = np.zeros(pts.size, bool)
        inf[-1] = True
        w, winf = intermediate_form(pts, inf, k, branch)
        assert winf[0] and not winf[k] and w[k] == 0
        arc = w[1:k]
        assert np.all(arc.real == 0) and np.all(branch * arc.imag > 0)
        # arc order along the half-axis: z_{k-1} closest to 0
        assert np.all(np.diff(np.abs(arc.imag)) <= 0)
        rest = w[k + 1:][~winf[k + 1:]]
        assert np.all(rest.real > 0)


def test_geodesic_algorithm_maps_to_upper_half_plane():
    rng = np.random.default_rng(7)
    for _ in range(10):
        n = int(rng.integers(8, 40))
        z, zi = _polygon(rng, n, interior=5)
        pts = np.concatenate([z, zi])
        w, winf = intermediate_form(pts, np.zeros(pts.size, bool), n - 1, +1, squared_final=True)
        assert winf[0]
        assert np.all(np.abs(w[1:n].imag) <= 1e-12 * np.abs(w[1:n]).max())
        assert np.all(w[n:].imag > 0)


def _loop_area(z):
    return 0.5 * np.sum(z.real * np.roll(z.imag, -1) - z.imag * np.roll(z.real, -1))


def _winding(poly, p):
    d = poly - p
    ang = np.angle(np.roll(d, -1) / d)
    return np.sum(ang) / (2 * np.pi)


@pytest.mark.parametrize("n,bx,by,seed", [(17, 2, 2, 0), (25, 3, 3, 2), (21, 4, 1, 5), (29, 3, 2, 9)])
def test_weld_glue_orientation_and_tiling(n, bx, by, seed):
    case = small_grid_case(n, bx, by, seed=seed)
    part, subs = prepare(case.V, case.F, case.label)
    bdy = local_params(subs)
    loops = [s["loop"] for s in subs]
    welded, steps, outer = weld(loops, bdy, "free", return_steps=True)
    for st in steps:
        assert st["glue_gap"] <= 1e-9 * max(1.0, st["scale"])
    areas = []
    for s in subs:
        poly = np.array([welded[int(v)] for v in s["loop"]])
        a = _loop_area(poly)
        assert a > 0
        areas.append(a)
    outer_poly = np.array([welded[v] for v in outer])
    assert _loop_area(outer_poly) > 0
    assert abs(sum(areas) - _loop_area(outer_poly)) <= 1e-9 * _loop_area(outer_poly)
    outer_set = set(outer)
    for v, c in welded.items():
        if v not in outer_set:
            assert abs(_winding(outer_poly, c) - 1.0) < 1e-6


@pytest.mark.parametrize("mode", ["free", "disk"])
def test_weld_extended_precision_run(mode):
    """The weld evaluated in extended precision (the input's complex type is
    carried through every step) agrees with the FP64 run to FP64 rounding, keeps
    its type, and glues the arcs far more tightly: the reference that measures
    the conditioning of long welds."""
    if np.finfo(np.longdouble).nmant <= np.finfo(np.float64).nmant:
        pytest.skip("long double is not wider than double here")
    case = small_grid_case(25, 3, 3, seed=2, mode=mode)
    part, subs = prepare(case.V, case.F, case.label)
    bdy = local_params(subs)
    loops = [s["loop"] for s in subs]
    w64, st64, _ = weld(loops, bdy, mode, return_steps=True)
    wl, stl, _ = weld(loops, [b.astype(np.clongdouble) for b in bdy], mode, return_steps=True)
    assert all(np.asarray(c).dtype == np.clongdouble for c in wl.values())
    z64 = np.array([w64[v] for v in sorted(w64)])
    zl = np.array([wl[v] for v in sorted(wl)])
    assert float(np.abs(z64 - zl).max()) <= 1e-12 * float(np.abs(zl).max())
    gap64 = max(st["glue_gap"] for st in st64 if "glue_gap" in st)
    gapl = max(st["glue_gap"] for st in stl if "glue_gap" in st)
    assert gapl <= 1e-2 * gap64 or gapl <= 1e-16


def test_weld_disk_constraint_unit_circle():
    case = small_grid_case(21, 2, 2, seed=3, mode="disk")
    part, subs = prepare(case.V, case.F, case.label)
    bdy = local_params(subs)
    welded, steps, outer = weld([s["loop"] for s in subs], bdy, "disk", return_steps=True)
    r_out = np.array([abs(welded[v]) for v in outer])
    assert np.abs(r_out - 1.0).max() < 1e-12
    inner = [abs(c) for v, c in welded.items() if v not in set(outer)]
    assert max(inner) < 1.0


def test_merge_plan_is_balanced_tree():
    case = small_grid_case(17, 4, 4, seed=1)
    part, subs = prepare(case.V, case.F, case.label)
    rounds = merge_plan([s["loop"] for s in subs], [len(s["T"]) for s in subs], "free")
    assert [len(r) for r in rounds] == [8, 4, 2, 1]
    merged = [j for r in rounds for _, j in r]
    assert sorted(merged) == list(range(1, 16))

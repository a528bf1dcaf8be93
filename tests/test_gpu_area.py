"""Area distortion and its Moebius post-optimisation (Section 6) on the GPU
against the FP64 oracle.

Per-face d_area and the mean |d_area| to 1e-12 (every term is an FP64 log of
an FP64 area; the two sides differ in summation order only), the objective at
fixed Moebius parameters of every mode to 1e-12 relative, and the search on
meshes whose parameterization is a known Moebius image of the mesh itself
(exact optimum 0): the device's Nelder-Mead must reach it as the oracle's does,
and its composed map must be the oracle's map at the same parameters.
Parameterizations are synthetic (not from the HIP path): smooth images of the
mesh's own coordinates.
"""
import sys

import numpy as np
import pytest

from oracle import area
from synth import case_c2, case_c3, small_grid_case, small_sphere_case
from synth.meshes import grid_mesh, icosphere

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


def say(*a):
    print("[gpu]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_1903_12359_amd as pg
    pg.load_library()
    assert torch.cuda.is_available()
    return pg.Context(0)


def _dev(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a if dtype is None else a.astype(dtype))).to("cuda:0")


def _free_map(V):
    z = V[:, 0] + 1j * V[:, 1]
    z = z - z.mean()
    z = z / np.abs(z).max()
    w = z + 0.15 * z * z + 0.05j * z ** 3
    return np.column_stack([w.real, w.imag])


def _disk_map(V):
    w = _free_map(V)
    return 0.9 * w / np.abs(w[:, 0] + 1j * w[:, 1]).max()


def _sphere_map(V):
    return V / np.linalg.norm(V, axis=1)[:, None]


MESHES = {
    "g33_jit": lambda: small_grid_case(33, 3, 3, seed=2, jitter=0.3),
    "g40": lambda: small_grid_case(40, 4, 2, seed=6),
    "S5": lambda: small_sphere_case(5, 12, seed=2),
}


def _case(name):
    c = MESHES[name]()
    V, F = np.asarray(c.V, float), np.asarray(c.F, np.int32)
    if name.startswith("S"):
        return V, F, {"sphere": _sphere_map(V)}
    return V, F, {"free": _free_map(V), "disk": _disk_map(V)}


@pytest.mark.parametrize("name", list(MESHES))
def test_area_distortion_matches_oracle(ctx, name):
    import paper_1903_12359_amd as pg
    V, F, maps = _case(name)
    for mode, X in maps.items():
        m, d = pg.area_distortion(ctx, _dev(V), _dev(F), _dev(X), want_d=True)
        do = area.area_distortion(V, F, X)
        err = np.abs(d.cpu().numpy() - do).max()
        say("area", name, mode, "nf", len(F), "mean", m, "max err", err)
        assert err <= 1e-12
        assert abs(m - np.abs(do).mean()) <= 1e-12 * max(1.0, abs(m))


@pytest.mark.parametrize("name", list(MESHES))
def test_area_objective_matches_oracle(ctx, name):
    import paper_1903_12359_amd as pg
    V, F, maps = _case(name)
    rng = np.random.default_rng(3)
    for mode, X in maps.items():
        Vd, Fd, Xd = _dev(V), _dev(F), _dev(X)
        for trial in range(4):
            if mode == "disk":
                p = rng.uniform(-0.4, 0.4, 2)
            else:
                p = area.IDENTITY[mode] + rng.normal(scale=0.15, size=8)
            g = pg.area_objective(ctx, Vd, Fd, Xd, mode, p)
            o = area.objective(V, F, X, mode, p)
            say("objective", name, mode, trial, g, o)
            if np.isfinite(o):
                assert abs(g - o) <= 1e-12 * max(1.0, abs(o))
            else:
                assert not np.isfinite(g)
    # inadmissible parameters
    mode, X = next(iter(maps.items()))
    bad = np.array([2.0, 0.0]) if mode == "disk" else np.array([1.0, 0, 2.0, 0, 0.5, 0, 1.0, 0])   # ad = bc
    assert pg.area_objective(ctx, _dev(V), _dev(F), _dev(X), mode, bad) == float("inf")


def test_pole_inside_the_domain_is_inadmissible(ctx):
    # f(z) = 1/(z - z0) with z0 inside the parameter domain reverses the faces
    # around z0 (their image areas stay finite): +inf on both sides; with the
    # pole outside both give the same finite value
    import paper_1903_12359_amd as pg
    V, F, xy = _plane(n=16)
    X = xy + 0.01 * np.column_stack([np.sin(3 * xy[:, 1]), np.cos(2 * xy[:, 0])])
    inside = np.array([0.0, 0.0, 1.0, 0.0, 1.0, 0.0, -0.113, -0.057])
    outside = np.array([0.0, 0.0, 1.0, 0.0, 1.0, 0.0, -2.0, 0.0])
    Vd, Fd, Xd = _dev(V), _dev(F), _dev(X)
    assert area.objective(V, F, X, "free", inside) == float("inf")
    assert pg.area_objective(ctx, Vd, Fd, Xd, "free", inside) == float("inf")
    o = area.objective(V, F, X, "free", outside)
    g = pg.area_objective(ctx, Vd, Fd, Xd, "free", outside)
    say("pole outside", g, o)
    assert np.isfinite(o) and abs(g - o) <= 1e-12 * max(1.0, o)


def _plane(n=24, lo=-0.5, hi=0.5):
    xy, F = grid_mesh(n)
    xy = lo + (hi - lo) * xy
    return np.column_stack([xy, np.zeros(len(xy))]), F.astype(np.int32), xy


def _known_moebius(mode):
    if mode == "free":
        V, F, xy = _plane()
        w = area.mobius(xy[:, 0] + 1j * xy[:, 1], np.array([1.0, 0.2, 0.3, 0.1, 0.25, -0.15, 1.0, 0.0]))
        return V, F, np.column_stack([w.real, w.imag]), 3000
    if mode == "disk":
        V, F, xy = _plane(lo=-0.6, hi=0.6)
        w = area.disk_automorphism(xy[:, 0] + 1j * xy[:, 1], np.array([0.4 * np.cos(0.9), 0.4 * np.sin(0.9)]))
        return V, F, np.column_stack([w.real, w.imag]), 600
    P, F = icosphere(4)
    P = np.asarray(P, float)
    return P, np.asarray(F, np.int32), area.apply(P, "sphere", np.array([1.2, 0.0, 0.3, 0.1, 0.0, -0.2, 1.0, 0.0])), 4000


@pytest.mark.parametrize("mode", ["free", "disk", "sphere"])
def test_mobius_search_reaches_the_known_optimum(ctx, mode):
    import paper_1903_12359_amd as pg
    V, F, X, budget = _known_moebius(mode)
    p, before, after, evals, Y = pg.area_mobius_opt(ctx, _dev(V), _dev(F), _dev(X), mode, max_evals=budget,
                                                    want_map=True)
    po, bo, ao = area.optimise(V, F, X, mode, max_evals=budget)
    say("mobius", mode, "gpu", before, "->", after, "evals", evals, "oracle", bo, "->", ao)
    assert abs(before - bo) <= 1e-12 * bo
    assert evals <= budget + len(p) + 1
    assert after <= 1e-2 * before and ao <= 1e-2 * bo
    assert abs(after - ao) <= 1e-2 * bo
    # the composed map is the oracle's map at the device's parameters, and its distortion is `after`
    Yo = area.apply(X, mode, p)
    assert np.abs(Y.cpu().numpy() - Yo).max() <= 1e-12 * max(1.0, np.abs(Yo).max())
    m, _ = pg.area_distortion(ctx, _dev(V), _dev(F), Y)
    assert abs(m - after) <= 1e-10
    # every evaluation adds its block sums in a fixed order, whichever
    # workgroup finishes last: a second search takes the same steps bitwise
    p2, before2, after2, evals2, _ = pg.area_mobius_opt(ctx, _dev(V), _dev(F), _dev(X), mode, max_evals=budget)
    assert np.array_equal(p2, p) and before2 == before and after2 == after and evals2 == evals


def test_full_size_objective_c2_c3(ctx):
    """C2 (522,242 faces) free and C3 (1,310,720 faces) sphere: the objective at
    the identity and at two other maps against the oracle."""
    import paper_1903_12359_amd as pg
    rng = np.random.default_rng(7)
    for name, make, mode, mapf in (("C2", case_c2, "free", _free_map), ("C3", case_c3, "sphere", _sphere_map)):
        c = make()
        V, F = np.asarray(c.V, float), np.asarray(c.F, np.int32)
        X = mapf(V)
        Vd, Fd, Xd = _dev(V), _dev(F), _dev(X)
        for p in (area.IDENTITY[mode], area.IDENTITY[mode] + rng.normal(scale=0.1, size=8),
                  area.IDENTITY[mode] + rng.normal(scale=0.1, size=8)):
            g = pg.area_objective(ctx, Vd, Fd, Xd, mode, p)
            o = area.objective(V, F, X, mode, p)
            say("full", name, mode, g, o)
            assert abs(g - o) <= 1e-12 * max(1.0, abs(o))
            assert pg.area_objective(ctx, Vd, Fd, Xd, mode, p) == g   # bitwise reproducible


def test_degenerate_and_invalid_inputs(ctx):
    import paper_1903_12359_amd as pg
    V = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 1, 0]], float)   # face 0 is collinear
    F = np.array([[0, 1, 2], [0, 1, 3]], np.int32)
    X = V[:, :2].copy()
    with pytest.raises(pg.PGCPError):
        pg.area_distortion(ctx, _dev(V), _dev(F), _dev(X))
    with pytest.raises(pg.PGCPError):                                   # sphere mode with a planar map
        pg.area_objective(ctx, _dev(V), _dev(F[1:]), _dev(X), "sphere", area.IDENTITY["sphere"])
    # a parameterization with a collapsed face gives +inf, not an error
    X2 = X.copy()
    X2[3] = X2[0]
    m, _ = pg.area_distortion(ctx, _dev(V), _dev(F[1:]), _dev(X2))
    assert m == float("inf")

"""Pins of the oracle's partition, cotangent Laplacian and distortion steps.

Each check is fixed by the paper or by mathematics independent of the oracle's
own formulas: partition properties (i)-(iv) of Section 4.1, the P1 finite-
element stiffness matrix (an independent derivation of the cotangent formula),
closed forms on flat grids, and the Beltrami coefficient of affine maps.
"""
import numpy as np
import pytest

from oracle.cotan import DegenerateError, corner_cotangents, cotan_laplacian
from oracle.distortion import beltrami, corner_angles, distortion, hazen_percentile
from oracle.partition import TopologyError, local_faces, partition
from synth import block_labels, grid_mesh, small_grid_case


# ---------------------------------------------------------------- partition

@pytest.mark.parametrize("n,bx,by", [(9, 2, 2), (17, 3, 2), (12, 4, 4), (8, 1, 1)])
def test_partition_properties(n, bx, by):
    case = small_grid_case(n, bx, by, seed=n)
    p = partition(case.V, case.F, case.label)
    assert p.K == bx * by
    # (i) vertex sets cover V, (ii) face sets cover F, (iv) faces disjoint
    allv = np.unique(np.concatenate([s.verts for s in p.subs]))
    assert np.array_equal(allv, np.arange(case.nv))
    allf = np.concatenate([s.faces for s in p.subs])
    assert np.array_equal(np.sort(allf), np.arange(case.nf))
    # (iii) V_i & V_j = boundary_i & boundary_j
    for i in range(p.K):
        for j in range(i + 1, p.K):
            vi = set(p.subs[i].verts.tolist()) & set(p.subs[j].verts.tolist())
            bi = set(p.subs[i].loop.tolist()) & set(p.subs[j].loop.tolist())
            assert vi == bi
    # components numbered by smallest face; loops CCW (flat projection area > 0)
    firsts = [s.faces.min() for s in p.subs]
    assert firsts == sorted(firsts)
    for s in p.subs:
        xy = case.V[s.loop, :2]
        area = 0.5 * np.sum(xy[:, 0] * np.roll(xy[:, 1], -1) - xy[:, 1] * np.roll(xy[:, 0], -1))
        assert area > 0
        assert s.loop[0] == s.loop.min()


def test_partition_label_split_into_components():
    # one label used for two separated blocks gives two components
    n = 9
    xy, F = grid_mesh(n)
    V = np.column_stack([xy, np.zeros(n * n)])
    lab = block_labels(n, 3, 1)
    lab[lab == 2] = 0
    p = partition(V, F, lab)
    assert p.K == 3


def test_partition_rejects_annulus_and_pinch_and_nonmanifold():
    n = 7
    xy, F = grid_mesh(n)
    V = np.column_stack([xy, np.zeros(n * n)])
    # annulus: a ring label around a centre block
    lab = block_labels(n, 3, 3)
    ring = np.where(lab == 4, 1, 0).astype(np.int32)
    with pytest.raises(TopologyError):
        partition(V, F, ring)
    # pinch: a C-shaped ring of cells whose two ends meet at one vertex
    from synth.meshes import grid_cell_index
    ic, jc = grid_cell_index(n)
    block = (ic < 3) & (jc < 3)
    hole = ((ic == 1) & (jc == 1)) | ((ic == 2) & (jc == 2))
    lab = (block & ~hole).astype(np.int32)
    with pytest.raises(TopologyError):
        partition(V, F, lab)
    # non-manifold edge: a third face on an interior edge
    F2 = np.vstack([F, [[F[0, 0], F[0, 1], 5 * n]]]).astype(np.int32)
    with pytest.raises(TopologyError):
        partition(V, F2, np.zeros(F2.shape[0], np.int32))


# ------------------------------------------------------------------ cotan

def _p1_stiffness(P, T):
    """Independent derivation: K_ij = sum_faces area * grad(lambda_i) . grad(lambda_j)."""
    n = P.shape[0]
    K = np.zeros((n, n))
    for t in T:
        x = P[t]
        e = [x[(c + 2) % 3] - x[(c + 1) % 3] for c in range(3)]  # edge opposite corner c
        nrm = np.cross(e[0], e[1])
        A = 0.5 * np.linalg.norm(nrm)
        nhat = nrm / (2 * A)
        g = [np.cross(nhat, e[c]) / (2 * A) for c in range(3)]  # gradient of hat function
        for a in range(3):
            for b in range(3):
                K[t[a], t[b]] += A * g[a] @ g[b]
    return K


def test_cotan_equals_p1_stiffness():
    case = small_grid_case(7, 1, 1, seed=3, nbumps=4, jitter=0.3)
    L = cotan_laplacian(case.V, case.F.astype(np.int64)).toarray()
    K = _p1_stiffness(case.V, case.F)
    np.testing.assert_allclose(L, K, atol=1e-12 * np.abs(K).max())


def test_cotan_golden_unit_square(golden):
    P = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], float)
    T = np.array([[0, 1, 2], [0, 2, 3]])
    L = cotan_laplacian(P, T).toarray()
    np.testing.assert_allclose(L, golden("cotan_unit_square.txt"), atol=1e-15)


def test_cotan_five_point_stencil_on_flat_grid():
    n = 6
    xy, F = grid_mesh(n)
    V = np.column_stack([xy * (n - 1), np.zeros(n * n)])  # integer coordinates
    L = cotan_laplacian(V, F.astype(np.int64)).toarray()
    for j in range(1, n - 1):
        for i in range(1, n - 1):
            v = j * n + i
            row = L[v]
            assert row[v] == 4.0
            for u in (v - 1, v + 1, v - n, v + n):
                assert row[u] == -1.0
            assert row[v - n - 1] == 0.0 and row[v + n + 1] == 0.0


def test_cotan_symmetry_rowsum_and_cot_identity():
    case = small_grid_case(9, 1, 1, seed=5, nbumps=5)
    L = cotan_laplacian(case.V, case.F.astype(np.int64))
    D = L.toarray()
    assert np.array_equal(D, D.T)
    assert np.abs(D.sum(1)).max() <= 1e-14 * np.abs(D).sum(1).max()
    # cot at k = (|a|^2 + |b|^2 - |c|^2) / (4 area), c the opposite edge
    cots = corner_cotangents(case.V, case.F.astype(np.int64))
    P = case.V
    for f in range(0, case.nf, 7):
        t = case.F[f]
        for c in range(3):
            k, i, j = t[c], t[(c + 1) % 3], t[(c + 2) % 3]
            a2 = np.sum((P[i] - P[k]) ** 2)
            b2 = np.sum((P[j] - P[k]) ** 2)
            c2 = np.sum((P[i] - P[j]) ** 2)
            A = 0.5 * np.linalg.norm(np.cross(P[i] - P[k], P[j] - P[k]))
            assert abs(cots[f, c] - (a2 + b2 - c2) / (4 * A)) < 1e-12 * max(1, abs(cots[f, c]))


def test_cotan_equilateral_and_area_identity():
    P = np.array([[0, 0, 0], [1, 0, 0], [0.5, np.sqrt(3) / 2, 0]])
    L = cotan_laplacian(P, np.array([[0, 1, 2]])).toarray()
    np.testing.assert_allclose(-L[0, 1], 1 / (2 * np.sqrt(3)), rtol=1e-14)
    # identity map on a flat mesh: E_D = 1/2 (x^T L x + y^T L y) = area
    case = small_grid_case(8, 1, 1, seed=1, flat=True, jitter=0.3)
    L = cotan_laplacian(case.V, case.F.astype(np.int64))
    x, y = case.V[:, 0], case.V[:, 1]
    ed = 0.5 * (x @ (L @ x) + y @ (L @ y))
    tri = case.V[case.F]
    area = 0.5 * np.abs(np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])[:, 2]).sum()
    assert abs(ed - area) < 1e-13


def test_cotan_degenerate():
    P = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], float)
    with pytest.raises(DegenerateError):
        cotan_laplacian(P, np.array([[0, 1, 2]]))


# ------------------------------------------------------------- distortion

def test_angles_and_identity():
    P = np.array([[0, 0, 0], [4, 0, 0], [0, 3, 0]], float)
    a = corner_angles(P, np.array([[0, 1, 2]]))
    np.testing.assert_allclose(a[0], [90.0, np.degrees(np.arctan2(3, 4)), np.degrees(np.arctan2(4, 3))],
                               atol=1e-12)
    case = small_grid_case(9, 1, 1, seed=2, flat=True, jitter=0.3)
    r = distortion(case.V, case.F, case.V[:, :2])
    assert r["stats"]["max_abs_d"] < 1e-10 and r["stats"]["max_mu"] < 1e-12
    assert r["stats"]["n_flipped"] == 0


def test_beltrami_affine_golden(golden):
    case = small_grid_case(9, 1, 1, seed=4, flat=True, jitter=0.3)
    for sx, sy, m in golden("beltrami_affine.txt"):
        phi = case.V[:, :2] * np.array([sx, sy])
        mu = np.abs(beltrami(case.V, case.F, phi))
        np.testing.assert_allclose(mu, m, atol=1e-12)
    # reflection: every face flips, |mu| -> inf
    r = distortion(case.V, case.F, case.V[:, :2] * np.array([-1.0, 1.0]))
    assert r["stats"]["n_flipped"] == case.nf
    assert r["mu"].min() > 1.0


def test_sphere_orientation_and_chordal_angles():
    from synth import icosphere
    V, F = icosphere(2)
    r = distortion(V, F, V.copy())
    assert r["stats"]["n_flipped"] == 0 and r["stats"]["max_abs_d"] < 1e-10


def test_hazen_percentile():
    x = np.random.default_rng(0).random(101)
    for q in (25, 50, 75, 3, 99):
        assert abs(hazen_percentile(x, q) - np.percentile(x, q, method="hazen")) < 1e-15


def test_local_faces_roundtrip():
    case = small_grid_case(9, 2, 2, seed=0)
    p = partition(case.V, case.F, case.label)
    for i, s in enumerate(p.subs):
        T = local_faces(p, case.F, i)
        assert np.array_equal(s.verts[T], case.F[s.faces])


def test_c4_training_recipe_sizes_and_seeds():
    """The training recipe yields height fields, then perturbed spheres, whose
    pieces have about 1k-20k vertices, and the same meshes for the same seed."""
    from itertools import islice
    from synth import c4_training_meshes
    first = list(islice(c4_training_meshes(seed=0, n_height=60, n_sphere=8), 12))
    again = list(islice(c4_training_meshes(seed=0, n_height=60, n_sphere=8), 12))
    assert [c.name for c in first] == [c.name for c in again]
    assert all(np.array_equal(a.V, b.V) and np.array_equal(a.label, b.label) for a, b in zip(first, again))
    modes = [c.mode for c in first]
    assert "free" in modes and "sphere" in modes
    assert modes == sorted(modes)   # all height fields before the spheres
    for c in first:
        part = partition(c.V, c.F, c.label)
        sizes = np.array([s.verts.size for s in part.subs])
        assert sizes.min() >= 500 and sizes.max() <= 30_000, (c.name, sizes.min(), sizes.max())

"""Oracle of the quasi-conformal fold repair (Sections 3.5, 4.5) against what
the theory fixes: the linear Beltrami solver's matrix is the cotangent
Laplacian for mu = 0, symmetric with zero row sums and positive semidefinite
for |mu| < 1; it gives back any piecewise-linear map from the map's own
Beltrami coefficient and boundary values (affine maps in closed form); the
repair keeps the boundary, leaves a folding-free map alone and unfolds folded
ones."""
import numpy as np
import pytest

from oracle.cotan import cotan_laplacian
from oracle.distortion import beltrami, orientation
from oracle.partition import partition
from oracle.pipeline import pgcp
from oracle.qc import beltrami_matrix, beltrami_solve, chop, fold_repair
from synth import small_grid_case
from synth.meshes import block_labels, bump_field, grid_mesh


def folded_grid(n=64, clip=0.35, seed=3):
    """Bump height field whose x/y jitter (sigma 0.51 h, cut at `clip` h) folds
    some triangles over in the xy-projection: the surface itself folds."""
    rng = np.random.default_rng(1234 + seed)
    f, _ = bump_field(rng, 8)
    xy, F = grid_mesh(n)
    h = 1.0 / (n - 1)
    d = np.clip(rng.normal(0.0, 0.51 * h, size=xy.shape), -clip * h, clip * h)
    xy = xy + d
    return np.column_stack([xy, f(xy[:, 0], xy[:, 1])]), F, block_labels(n, 1, 1)


def test_chop_cuts_the_modulus_and_keeps_the_direction():
    mu = np.array([0.2 + 0.1j, 0.95j, -3.0 + 4.0j, 0.0])
    c = chop(mu, 0.1)
    assert c[0] == mu[0] and c[3] == 0
    assert np.allclose(np.abs(c[1:3]), 0.9) and np.allclose(c[2] / abs(c[2]), mu[2] / abs(mu[2]))


def test_zero_mu_gives_the_cotangent_laplacian():
    c = small_grid_case(17, 1, 1, seed=4, nbumps=5)
    L = cotan_laplacian(c.V, c.F)
    K = beltrami_matrix(c.V, c.F, np.zeros(c.nf, complex))
    assert abs(K - L).max() <= 1e-13 * abs(L).max()


def test_matrix_symmetric_zero_row_sums_psd():
    c = small_grid_case(9, 1, 1, seed=5, nbumps=4)
    rng = np.random.default_rng(0)
    mu = 0.8 * rng.uniform(0, 1, c.nf) * np.exp(2j * np.pi * rng.uniform(0, 1, c.nf))
    K = beltrami_matrix(c.V, c.F, mu).toarray()
    assert np.abs(K - K.T).max() <= 1e-12 * np.abs(K).max()
    assert np.abs(K.sum(axis=1)).max() <= 1e-12 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert ev.min() >= -1e-10 * ev.max() and np.sum(ev < 1e-10 * ev.max()) == 1   # only constants


def test_affine_map_from_its_constant_coefficient():
    """On a flat mesh f(z) = z + mu0 conj(z) has coefficient mu0 (in each face's
    frame, mu0 turned by twice the frame's angle); the solver with that
    coefficient and f's boundary values gives back f."""
    c = small_grid_case(17, 1, 1, seed=0, flat=True)
    mu0 = 0.3 + 0.2j
    z = c.V[:, 0] + 1j * c.V[:, 1]
    f = z + mu0 * np.conj(z)
    loop = partition(c.V, c.F, c.label).subs[0].loop
    mu = beltrami(c.V, c.F, np.column_stack([f.real, f.imag]))
    # frames of faces whose first edge runs along +x see mu0 itself, the
    # others (first edge on the diagonal, 45 degrees) mu0 * exp(-i pi / 2)
    assert np.allclose(np.sort_complex(np.unique(np.round(mu, 12))), np.sort_complex([mu0, -1j * mu0]))
    u = beltrami_solve(c.V, c.F, loop, mu, f[loop])
    assert np.abs(u - f).max() <= 1e-12


def test_piecewise_linear_map_from_its_own_coefficient_on_a_curved_mesh():
    c = small_grid_case(25, 1, 1, seed=7, nbumps=6)
    loop = partition(c.V, c.F, c.label).subs[0].loop
    z = c.V[:, 0] + 1j * c.V[:, 1]
    g = z + 0.2 * z ** 2 + 0.1j * np.conj(z) ** 2 + 0.3 * c.V[:, 2]
    X = np.column_stack([g.real, g.imag])
    assert (orientation(X, c.F) > 0).all()
    u = beltrami_solve(c.V, c.F, loop, beltrami(c.V, c.F, X), g[loop])
    assert np.abs(u - g).max() <= 1e-11 * np.abs(g).max()


def test_repair_leaves_a_folding_free_map_alone():
    c = small_grid_case(25, 1, 1, seed=8, nbumps=6)
    r = pgcp(c.V, c.F, c.label, "free")
    s = r["subs"][0]
    X, passes, flips = fold_repair(s["P"], s["T"], s["loop_local"], r["phi"][s["verts"]])
    assert passes == 0 and flips == [0] and np.array_equal(X, r["phi"][s["verts"]])


@pytest.mark.parametrize("n,seed", [(64, 3), (96, 3)])
def test_repair_unfolds_a_folded_surface_map(n, seed):
    """The DNCP / harmonic map of a folded surface has flipped faces (negative
    cotangent weights); the repaired map has none, the same boundary, and
    about the same angle distortion."""
    from oracle.distortion import distortion
    V, F, lab = folded_grid(n, 0.35, seed)
    r = pgcp(V, F, lab, "free")
    s = r["subs"][0]
    X0 = r["phi"][s["verts"]]
    before = distortion(s["P"], s["T"], X0)["stats"]
    assert before["n_flipped"] > 0
    X, passes, flips = fold_repair(s["P"], s["T"], s["loop_local"], X0)
    after = distortion(s["P"], s["T"], X)["stats"]
    assert flips[-1] == 0 and after["n_flipped"] == 0 and 1 <= passes <= 3
    B = s["loop_local"]
    assert np.array_equal(X[B], X0[B])
    assert after["mean_abs_d"] <= 1.1 * before["mean_abs_d"]

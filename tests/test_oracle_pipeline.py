"""End-to-end pins of the oracle (Algorithm 3).

A flat piece cut into subdomains must come back as a similarity of itself
(every step is then exact: DNCP is the identity, the pieces already fit, the
harmonic map has linear precision); bumpy patches must be flip-free with the
angle distortion shrinking under refinement.
"""
import numpy as np
import pytest

from oracle.pipeline import pgcp
from synth import case_c1, small_grid_case


@pytest.mark.parametrize("bx,by", [(2, 2), (3, 3), (4, 2)])
def test_flat_free_mode_is_similarity(bx, by):
    case = small_grid_case(25, bx, by, seed=1, flat=True, jitter=0.3)
    r = pgcp(case.V, case.F, case.label, "free")
    phi = r["phi"][:, 0] + 1j * r["phi"][:, 1]
    z = case.V[:, 0] + 1j * case.V[:, 1]
    A = np.column_stack([z, np.ones_like(z)])
    coef = np.linalg.lstsq(A, phi, rcond=None)[0]
    assert np.abs(A @ coef - phi).max() < 1e-9 * np.abs(phi).max()
    assert r["dist"]["stats"]["max_abs_d"] < 1e-7
    assert r["dist"]["stats"]["n_flipped"] == 0


def test_flat_disk_mode():
    case = small_grid_case(25, 2, 2, seed=1, flat=True, mode="disk")
    r = pgcp(case.V, case.F, case.label, "disk")
    assert r["dist"]["stats"]["n_flipped"] == 0
    assert np.abs(np.hypot(r["phi"][:, 0], r["phi"][:, 1])).max() <= 1.0 + 1e-12


def test_bumpy_flip_free_and_refines():
    means = []
    for n in (33, 129):
        case = small_grid_case(n, 3, 3, seed=2)
        r = pgcp(case.V, case.F, case.label, "free")
        assert r["dist"]["stats"]["n_flipped"] == 0
        assert r["dist"]["stats"]["max_mu"] < 1.0
        means.append(r["dist"]["stats"]["mean_abs_d"])
    assert means[1] < 0.6 * means[0]


def test_c1_disk_flip_free():
    case = case_c1()
    r = pgcp(case.V, case.F, case.label, case.mode)
    assert r["part"].K == 4
    assert r["dist"]["stats"]["n_flipped"] == 0
    rad = np.hypot(r["phi"][:, 0], r["phi"][:, 1])
    assert rad.max() <= 1.0 + 1e-12


def test_angle_distortion_does_not_depend_on_the_partition():
    """Section 5.5: the welded global map is conformal whatever the partition.
    Its angle distortion is the discretisation's alone, so it halves with the
    mesh spacing for every partition alike (measured 0.49-0.51 from 33^2 to
    65^2), and the partitions stay within a factor 1.6 of each other at each
    size (measured 1.58 and 1.50).  A seam the weld left kinked would add
    distortion that does not refine away."""
    parts = [(1, 1), (2, 2), (3, 2), (4, 4)]
    means = {}
    for bx, by in parts:
        for n in (33, 65):
            case = small_grid_case(n, bx, by, seed=3, nbumps=6)
            r = pgcp(case.V, case.F, case.label, "free")
            assert r["dist"]["stats"]["n_flipped"] == 0
            means[bx, by, n] = r["dist"]["stats"]["mean_abs_d"]
    for bx, by in parts:
        ratio = means[bx, by, 65] / means[bx, by, 33]
        assert 0.4 <= ratio <= 0.6, (bx, by, ratio)
    for n in (33, 65):
        m = [means[bx, by, n] for bx, by in parts]
        assert max(m) <= 1.6 * min(m), (n, m)

"""pgcp_distortion_noalloc (the distortion check for callers that cannot
allocate) against pgcp_distortion, through the C ABI: the same kernels, so
per-face outputs and statistics must agree bitwise; two calls in a row, the
second on a smaller mesh, so that records left in the fixed array by the first
call cannot leak into the second."""
import sys

import numpy as np
import pytest

from synth import case_c2, small_grid_case, small_sphere_case

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-noalloc]", *a, file=sys.stderr, flush=True)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _param(case):
    """A map with some flipped faces: the surface's (x, y) bent by a smooth
    field, mirrored on part of the mesh (sphere: the surface itself, rotated)."""
    V = case.V
    if case.mode == "sphere":
        c, s_ = np.cos(0.3), np.sin(0.3)
        P = V / np.linalg.norm(V, axis=1, keepdims=True)
        return np.column_stack([c * P[:, 0] - s_ * P[:, 1], s_ * P[:, 0] + c * P[:, 1], P[:, 2]])
    x, y = V[:, 0], V[:, 1]
    u = x + 0.05 * np.sin(7 * y)
    v = y + 0.05 * np.cos(5 * x)
    u = np.where(x > 0.8, 1.6 - u, u)          # a mirrored strip: flipped faces
    return np.column_stack([u, v])


def _compare(pg, ctx, case):
    import torch
    V, F, X = _dev(case.V), _dev(case.F.astype(np.int32)), _dev(_param(case))
    nf = case.nf
    ref, d0, mu0, fl0 = pg.distortion(ctx, V, F, X, want_arrays=True)
    d = torch.full((nf, 3), np.nan, dtype=torch.float64, device="cuda:0")
    mu = torch.full((nf,), np.nan, dtype=torch.float64, device="cuda:0")
    fl = torch.full((nf,), 7, dtype=torch.uint8, device="cuda:0")
    st = pg.distortion_noalloc(ctx, V, F, X, d, mu, fl)
    say(case.name, nf, "faces:", st)
    assert torch.equal(d, d0) and torch.equal(mu, mu0) and torch.equal(fl, fl0)
    for k in ("mean_abs_d", "sd_abs_d", "max_abs_d", "max_mu", "n_flipped", "n_mu_ge1"):
        assert st[k] == ref[k], (k, st[k], ref[k])
    assert np.isnan(st["median_abs_d"]) and np.isnan(st["iqr_abs_d"])
    return st


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_1903_12359_amd as pg
    pg.load_library()          # fails loudly when the library is missing
    assert torch.cuda.is_available()
    c = pg.Context(0)
    yield c
    c.close()


def test_noalloc_distortion_matches_the_allocating_call(ctx):
    import paper_1903_12359_amd as pg
    big = _compare(pg, ctx, case_c2(n=384))
    assert big["n_flipped"] > 0
    small = _compare(pg, ctx, small_grid_case(17, 2, 2, seed=0))
    assert small["n_flipped"] > 0
    _compare(pg, ctx, small_sphere_case(4, 6, seed=1))
    # statistics only (no per-face arrays), asynchronous form then synchronous
    V, F, X = _dev(case_c2(n=128).V), _dev(case_c2(n=128).F.astype(np.int32)), _dev(_param(case_c2(n=128)))
    assert pg.distortion_noalloc(ctx, V, F, X, stats=False) is None
    ref, _, _, _ = pg.distortion(ctx, V, F, X)
    st = pg.distortion_noalloc(ctx, V, F, X)
    assert st["mean_abs_d"] == ref["mean_abs_d"] and st["n_flipped"] == ref["n_flipped"]


def test_noalloc_rejects_more_faces_than_its_array(ctx):
    """The limit is checked on the host before anything else: nothing is launched."""
    import paper_1903_12359_amd as pg
    lib = pg.load_library()
    cap = int(lib.pgcp_distortion_noalloc_max_faces())
    assert cap == 8_388_608
    with pytest.raises(pg.PGCPError) as ei:
        ctx.check(lib.pgcp_distortion_noalloc(ctx.h, None, 3, None, cap + 1, None, 2, None, None, None, None))
    assert ei.value.status == "INVALID"

"""C-ABI library on the CPU: exported symbols, and the host stages (partition,
weld) against the oracle.  No device calls are made here.

Partition work is integer work and must match bit-exactly; the weld is the
same sequence of analytic maps evaluated in a different order (arc points
first, then the recorded chain per point), so it must agree to rounding.
"""
import re

import numpy as np
import pytest

from oracle.pipeline import local_params, prepare
from oracle.weld import weld as oracle_weld
from synth import case_c1, case_c2, small_grid_case, small_sphere_case

pg = pytest.importorskip("paper_1903_12359_amd")
HEADER = __import__("os").path.join(__import__("os").path.dirname(__file__), "..", "include", "pgcp.h")


def _lib():
    try:
        return pg.load_library()
    except ImportError as e:   # the build step has not run in this checkout
        pytest.skip(str(e))


def test_library_exports_every_declared_symbol():
    L = _lib()
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(pgcp_[a-z_]+)\s*\(", text))
    assert declared == set(pg.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


CASES = [
    lambda: small_grid_case(17, 2, 2, seed=0),
    lambda: small_grid_case(25, 3, 3, seed=2, jitter=0.3),
    lambda: small_grid_case(21, 4, 1, seed=5),
    lambda: small_grid_case(9, 1, 1, seed=1),
    lambda: small_grid_case(23, 3, 2, seed=4, mode="disk"),
    case_c1,
    lambda: case_c2(n=96),
    lambda: small_sphere_case(3, 6, seed=0),
    lambda: small_sphere_case(4, 8, seed=1),
    lambda: small_sphere_case(5, 12, seed=2),
]


@pytest.mark.parametrize("make", CASES)
def test_partition_bit_exact(make):
    _lib()
    case = make()
    plan = pg.Plan(None, case.V, case.F, case.label, case.mode)
    ex = plan.export()
    part, subs = prepare(case.V, case.F, case.label)
    assert plan.K == part.K
    assert np.array_equal(ex["face_sub"], part.face_sub)
    for i, s in enumerate(part.subs):
        assert ex["sub_nv"][i] == s.verts.size
        assert np.array_equal(ex["loop_gv"][ex["loop_ptr"][i]:ex["loop_ptr"][i + 1]], s.loop)
    seam = np.unique(np.concatenate([s.loop for s in part.subs]))
    assert np.array_equal(ex["seam_gv"], seam)


@pytest.mark.parametrize("make", CASES)
def test_weld_matches_oracle(make):
    _lib()
    case = make()
    plan = pg.Plan(None, case.V, case.F, case.label, case.mode)
    ex = plan.export()
    part, subs = prepare(case.V, case.F, case.label)
    bdy = local_params(subs)
    wo = oracle_weld([s["loop"] for s in subs], bdy, case.mode, sizes=[len(s["T"]) for s in subs])
    bh = np.concatenate([np.column_stack([b.real, b.imag]) for b in bdy])
    wc = pg.weld(None, plan, bh)
    zo = np.array([wo[g] for g in ex["seam_gv"]])
    zc = wc[:, 0] + 1j * wc[:, 1]
    io, ic = ~np.isfinite(zo), ~np.isfinite(zc)
    assert np.array_equal(io, ic)
    if case.mode == "sphere":
        # on the sphere the error that matters is chordal: compare the points
        # after inverse stereographic projection.  The closed weld composes
        # every pair's maps over the whole loop, so rounding grows more than in
        # the open welds; the bound is the FP64 parity bar of the whole path.
        def sig(z):
            r2 = np.abs(z) ** 2
            return np.column_stack([2 * z.real, 2 * z.imag, r2 - 1]) / (r2 + 1)[:, None]
        assert np.abs(sig(zo[~io]) - sig(zc[~ic])).max() <= 1e-9
    else:
        assert np.abs(zo - zc).max() <= 1e-10 * np.abs(zo).max()
    if case.mode == "disk":
        assert np.abs(np.abs(zc).max() - 1.0) < 1e-12


def test_partition_errors_are_topology():
    _lib()
    from synth import block_labels, grid_mesh
    from synth.meshes import grid_cell_index
    n = 7
    xy, F = grid_mesh(n)
    V = np.column_stack([xy, np.zeros(n * n)])
    ring = np.where(block_labels(n, 3, 3) == 4, 1, 0).astype(np.int32)
    ic, jc = grid_cell_index(n)
    block = (ic < 3) & (jc < 3)
    hole = ((ic == 1) & (jc == 1)) | ((ic == 2) & (jc == 2))
    pinch = (block & ~hole).astype(np.int32)
    F2 = np.vstack([F, [[F[0, 0], F[0, 1], 5 * n]]]).astype(np.int32)
    for VV, FF, lab in [(V, F, ring), (V, F, pinch), (V, F2, np.zeros(F2.shape[0], np.int32))]:
        with pytest.raises(pg.PGCPError) as ei:
            pg.Plan(None, VV, FF, lab, "free")
        assert ei.value.status == "TOPOLOGY"
    bad = F.copy()
    bad[0, 0] = n * n + 5
    with pytest.raises(pg.PGCPError) as ei:
        pg.Plan(None, V, bad, np.zeros(F.shape[0], np.int32), "free")
    assert ei.value.status == "INVALID"


def test_single_piece_weld_is_identity_and_disk_circle():
    _lib()
    case = small_grid_case(13, 1, 1, seed=3)
    part, subs = prepare(case.V, case.F, case.label)
    bdy = local_params(subs)
    bh = np.column_stack([bdy[0].real, bdy[0].imag])
    plan = pg.Plan(None, case.V, case.F, case.label, "free")
    w = pg.weld(None, plan, bh)
    order = np.argsort(subs[0]["loop"])
    np.testing.assert_array_equal(w, bh[order])
    plan = pg.Plan(None, case.V, case.F, case.label, "disk")
    w = pg.weld(None, plan, bh)
    assert np.abs(np.hypot(w[:, 0], w[:, 1]) - 1).max() < 1e-12


def _piece_graph(s):
    """Vertex adjacency of one oracle piece (local = ascending global index) as CSR."""
    import scipy.sparse as sp
    T = np.asarray(s["T"])
    n = len(s["verts"])
    a = np.concatenate([T[:, 0], T[:, 1], T[:, 2], T[:, 1], T[:, 2], T[:, 0]])
    b = np.concatenate([T[:, 1], T[:, 2], T[:, 0], T[:, 0], T[:, 1], T[:, 2]])
    return sp.csr_matrix((np.ones(a.size), (a, b)), shape=(n, n))


def _max_halo(order, G, block=1024):
    """Largest number of distinct vertices outside a block of `block`
    consecutive rows that the block's rows are adjacent to."""
    pos = np.empty(len(order), np.int64)
    pos[order] = np.arange(len(order))
    worst = 0
    for b0 in range(0, len(order), block):
        rows = order[b0:b0 + block]
        nb = np.unique(G[rows].indices)
        worst = max(worst, int(np.count_nonzero((pos[nb] < b0) | (pos[nb] >= b0 + block))))
    return worst


@pytest.mark.parametrize("make", CASES + [lambda: small_sphere_case(6, 4, seed=3)])
def test_row_order_is_reverse_breadth_first(make):
    """A piece's packed rows hold exactly its vertices in reverse Cuthill-McKee
    order: read backwards they list the piece's graph level by level from the
    first one (breadth-first distances never decrease).  On k-means sphere
    pieces a 1,024-row block's halo is smaller than in global order."""
    import scipy.sparse.csgraph as csg
    _lib()
    case = make()
    plan = pg.Plan(None, case.V, case.F, case.label, case.mode)
    row0, gv = plan.rows(), plan.row_vertices()
    part, subs = prepare(case.V, case.F, case.label)
    assert gv.shape == (row0[-1],)
    for i, s in enumerate(subs):
        verts = np.asarray(s["verts"])
        n = len(verts)
        piece = gv[row0[i]:row0[i + 1]]
        assert np.array_equal(np.sort(piece[:n]), np.sort(verts)), i
        assert (piece[n:] == -1).all()
        local = np.searchsorted(np.sort(verts), piece[:n])   # packed row -> oracle local index
        G = _piece_graph(s)
        d = csg.shortest_path(G, unweighted=True, indices=int(local[-1]))
        assert np.isfinite(d).all(), i
        assert (np.diff(d[local[::-1]]) >= 0).all(), i
        if n >= 4096 and case.mode == "sphere":
            h_rcm, h_glob = _max_halo(local, G), _max_halo(np.arange(n), G)
            assert h_rcm < h_glob, (i, h_rcm, h_glob)


def test_noalloc_distortion_limits_on_the_host():
    """pgcp_distortion_noalloc checks its face limit before anything else and
    rejects a missing context, so neither case reaches a device."""
    L = _lib()
    cap = int(L.pgcp_distortion_noalloc_max_faces())
    assert cap == 32768 * 256
    assert L.pgcp_distortion_noalloc(None, None, 3, None, cap + 1, None, 2, None, None, None, None) == -1
    assert L.pgcp_distortion_noalloc(None, None, 3, None, 1, None, 2, None, None, None, None) == -1

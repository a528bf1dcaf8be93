"""Seeded synthetic meshes shaped like the dense scans the paper parameterizes.

The paper (Section 5) runs on scanned meshes of 20K-1M vertices that are not
available here.  These generators stand in for them: height fields on regular
grids (open, simply-connected) and perturbed icospheres (genus-0, closed), each
with per-face subdomain labels that cut the surface into simply-connected
pieces (Section 4.1 takes a cut-edge set; a per-face label array is the same
information: an edge is cut when its two faces carry different labels).

Every generator is deterministic for a given seed.  Nothing here computes any
part of the parameterization.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 1903_12359


@dataclasses.dataclass
class MeshCase:
    name: str
    V: np.ndarray          # float64 [nv, 3]
    F: np.ndarray          # int32 [nf, 3], counter-clockwise seen from outside / from +z
    label: np.ndarray      # int32 [nf]
    mode: str              # "free" | "disk" | "sphere"
    meta: dict

    @property
    def nv(self) -> int:
        return int(self.V.shape[0])

    @property
    def nf(self) -> int:
        return int(self.F.shape[0])


# ----------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------

def grid_mesh(n: int, xy: np.ndarray | None = None):
    """Regular n x n vertex grid on [0,1]^2, two triangles per cell.

    Vertex (i, j) has index j*n + i.  Cell (i, j) gives the faces
    [(i,j),(i+1,j),(i+1,j+1)] and [(i,j),(i+1,j+1),(i,j+1)], both counter-
    clockwise seen from +z.  Returns (xy [nv,2], F [nf,3]); the caller adds z.
    """
    if xy is None:
        t = np.arange(n, dtype=np.float64) / (n - 1)
        X, Y = np.meshgrid(t, t, indexing="xy")
        xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    i = np.arange(n - 1)
    I, J = np.meshgrid(i, i, indexing="xy")
    I = I.ravel()
    J = J.ravel()
    v00 = J * n + I
    v10 = v00 + 1
    v01 = v00 + n
    v11 = v01 + 1
    F = np.empty((2 * (n - 1) ** 2, 3), dtype=np.int32)
    F[0::2] = np.stack([v00, v10, v11], axis=1)
    F[1::2] = np.stack([v00, v11, v01], axis=1)
    return xy, F


def grid_cell_index(n: int):
    """Cell coordinates (ic, jc) of every face produced by grid_mesh(n)."""
    i = np.arange(n - 1)
    I, J = np.meshgrid(i, i, indexing="xy")
    ic = np.repeat(I.ravel(), 2)
    jc = np.repeat(J.ravel(), 2)
    return ic, jc


def block_labels(n: int, bx: int, by: int) -> np.ndarray:
    """bx x by rectangular blocks of cells; label = by_index * bx + bx_index."""
    ic, jc = grid_cell_index(n)
    cells = n - 1
    lx = (bx * ic) // cells
    ly = (by * jc) // cells
    return (ly * bx + lx).astype(np.int32)


def bump_field(rng: np.random.Generator, nbumps: int):
    """Sum of Gaussian bumps: amplitudes U[-0.2,0.2], widths U[0.05,0.2], centres U[0,1]^2."""
    a = rng.uniform(-0.2, 0.2, size=nbumps)
    s = rng.uniform(0.05, 0.2, size=nbumps)
    c = rng.uniform(0.0, 1.0, size=(nbumps, 2))

    def f(x, y):
        z = np.zeros_like(x)
        for b in range(nbumps):
            r2 = (x - c[b, 0]) ** 2 + (y - c[b, 1]) ** 2
            z += a[b] * np.exp(-r2 / (2.0 * s[b] ** 2))
        return z

    return f, dict(amp=a.tolist(), width=s.tolist(), centre=c.tolist())


def _jitter(rng, n, sigma, clip_frac):
    h = 1.0 / (n - 1)
    d = rng.normal(0.0, sigma, size=(n * n, 2))
    if clip_frac is not None:
        d = np.clip(d, -clip_frac * h, clip_frac * h)
    return d


def small_grid_case(n: int = 17, bx: int = 2, by: int = 2, seed: int = 0,
                    nbumps: int = 3, jitter: float = 0.0, mode: str = "free",
                    flat: bool = False) -> MeshCase:
    """Small bump height field on an n x n grid split into bx x by blocks."""
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    xy, F = grid_mesh(n)
    xy = xy.copy()
    if jitter > 0:
        d = _jitter(rng, n, jitter / (n - 1), 0.15)
        xy += d
    if flat:
        z = np.zeros(n * n)
        meta = {}
    else:
        f, meta = bump_field(rng, nbumps)
        z = f(xy[:, 0], xy[:, 1])
    V = np.column_stack([xy, z]).astype(np.float64)
    return MeshCase(f"grid{n}_{bx}x{by}_s{seed}", V, F, block_labels(n, bx, by), mode,
                    dict(n=n, bx=bx, by=by, **meta))


def case_c1() -> MeshCase:
    """64x64 grid, z = 0.3 sin(pi x) cos(pi y), 2x2 blocks, disk output."""
    n = 64
    xy, F = grid_mesh(n)
    z = 0.3 * np.sin(np.pi * xy[:, 0]) * np.cos(np.pi * xy[:, 1])
    V = np.column_stack([xy, z])
    return MeshCase("C1", V, F, block_labels(n, 2, 2), "disk", dict(n=n, bx=2, by=2))


def case_c2(n: int = 512, blocks=4, clip_frac: float = 0.15) -> MeshCase:
    """512x512 grid, 8 Gaussian bumps, x/y jitter N(0,1e-3) clipped at 0.15 h, 4x4 blocks
    (`blocks`: b for b x b blocks, or (bx, by)).

    The jitter is drawn per component and truncated to |delta| <= clip_frac*h;
    z is evaluated at the jittered (x, y).  sigma = 1e-3 is 0.51 h on this grid;
    unclipped (or clipped at 0.35 h) it folds thousands of triangles over in the
    xy-projection, so the height field would no longer be a surface over the
    plane.  With per-component offsets of at most c*h every triangle keeps an
    xy-area of at least h^2 (1 - 6c)/2 > 0 for c < 1/6.
    """
    rng = np.random.default_rng(SEED_BASE + 2)
    f, meta = bump_field(rng, 8)
    xy, F = grid_mesh(n)
    xy = xy + _jitter(rng, n, 1e-3, clip_frac)
    z = f(xy[:, 0], xy[:, 1])
    V = np.column_stack([xy, z])
    bx, by = (blocks, blocks) if np.isscalar(blocks) else blocks
    return MeshCase("C2" if n == 512 else f"C2_n{n}", V, F, block_labels(n, bx, by),
                    "free", dict(n=n, bx=bx, by=by, clip_frac=clip_frac, **meta))


# ----------------------------------------------------------------------------
# guillotine partition with log-normal target sizes (large-scale stress case)
# ----------------------------------------------------------------------------

def guillotine_labels(n: int, nparts: int, sigma: float, rng: np.random.Generator,
                      max_aspect: float = 4.0) -> np.ndarray:
    """Split the (n-1)^2 cell rectangle into nparts rectangles with log-normal areas.

    Target sizes s_i ~ LogNormal(0, sigma) are normalised to the cell count.  The
    sorted target list is split recursively into two halves of nearly equal sum
    and the longer side of the current rectangle is cut at the grid line closest
    to the proportional position.  Returns per-face labels for grid_mesh(n).
    """
    cells = n - 1
    s = rng.lognormal(0.0, sigma, size=nparts)
    s = np.sort(s)[::-1]
    lab_cell = np.full((cells, cells), -1, dtype=np.int32)  # [jc, ic]
    counter = [0]

    def rec(x0, x1, y0, y1, sizes):
        if len(sizes) == 1:
            lab_cell[y0:y1, x0:x1] = counter[0]
            counter[0] += 1
            return
        tot = sizes.sum()
        # split into two groups of nearly equal sum, greedily (largest first)
        g1, g2 = [], []
        s1 = s2 = 0.0
        for v in sizes:
            if s1 <= s2:
                g1.append(v)
                s1 += v
            else:
                g2.append(v)
                s2 += v
        g1 = np.array(g1)
        g2 = np.array(g2)
        frac = s1 / tot
        w, h = x1 - x0, y1 - y0
        if w >= h:
            cut = x0 + int(round(frac * w))
            cut = min(max(cut, x0 + 2), x1 - 2)
            rec(x0, cut, y0, y1, g1)
            rec(cut, x1, y0, y1, g2)
        else:
            cut = y0 + int(round(frac * h))
            cut = min(max(cut, y0 + 2), y1 - 2)
            rec(x0, x1, y0, cut, g1)
            rec(x0, x1, cut, y1, g2)

    rec(0, cells, 0, cells, s)
    assert (lab_cell >= 0).all()
    ic, jc = grid_cell_index(n)
    return lab_cell[jc, ic].astype(np.int32)


def case_c5(n: int = 2048, nparts: int = 256) -> MeshCase:
    """2048x2048 grid, 32 bumps, no jitter, 256 log-normal(sigma=0.8) guillotine blocks."""
    rng = np.random.default_rng(SEED_BASE + 5)
    f, meta = bump_field(rng, 32)
    xy, F = grid_mesh(n)
    z = f(xy[:, 0], xy[:, 1])
    V = np.column_stack([xy, z])
    lab = guillotine_labels(n, nparts, 0.8, rng)
    return MeshCase("C5" if n == 2048 else f"C5_n{n}", V, F, lab, "free",
                    dict(n=n, nparts=nparts, **meta))


# ----------------------------------------------------------------------------
# spheres
# ----------------------------------------------------------------------------

def icosphere(level: int):
    """Icosahedron refined `level` times by edge midpoints, projected to the unit sphere.

    Faces are counter-clockwise seen from outside.  Vertex order: the 12
    icosahedron vertices, then new midpoints in order of first creation.
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    for _ in range(level):
        nv = V.shape[0]
        e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
        key = np.minimum(e[:, 0], e[:, 1]) * nv + np.maximum(e[:, 0], e[:, 1])
        uniq, first, inv = np.unique(key, return_index=True, return_inverse=True)
        # number new vertices in order of first occurrence
        order = np.argsort(first, kind="stable")
        rank = np.empty_like(order)
        rank[order] = np.arange(order.size)
        mid_id = nv + rank[inv]
        a = uniq // nv
        b = uniq % nv
        mids = 0.5 * (V[a] + V[b])
        mids /= np.linalg.norm(mids, axis=1, keepdims=True)
        Vn = np.empty((nv + uniq.size, 3))
        Vn[:nv] = V
        Vn[nv + rank] = mids
        nf = F.shape[0]
        m01 = mid_id[:nf]
        m12 = mid_id[nf:2 * nf]
        m20 = mid_id[2 * nf:]
        F = np.concatenate([
            np.stack([F[:, 0], m01, m20], 1),
            np.stack([F[:, 1], m12, m01], 1),
            np.stack([F[:, 2], m20, m12], 1),
            np.stack([m01, m12, m20], 1)], axis=0)
        V = Vn
    return V, F.astype(np.int32)


def _real_sph_harms(lmax, theta, phi):
    """Real orthonormal spherical harmonics Y_lm, l = 1..lmax (theta polar, phi azimuth)."""
    from scipy.special import sph_harm_y
    Y = {}
    for l in range(1, lmax + 1):
        for m in range(0, l + 1):
            Z = sph_harm_y(l, m, theta, phi)
            if m == 0:
                Y[(l, 0)] = np.real(Z)
            else:
                Y[(l, m)] = math.sqrt(2.0) * (-1) ** m * np.real(Z)
                Y[(l, -m)] = math.sqrt(2.0) * (-1) ** m * np.imag(Z)
    return Y


def perturb_sphere(V: np.ndarray, rng: np.random.Generator, lmax: int = 8, scale: float = 0.05):
    """Radius r = 1 + sum_{l=1..lmax} sum_m c_lm Y_lm with c_lm ~ N(0, (scale/l)^2)."""
    theta = np.arccos(np.clip(V[:, 2], -1.0, 1.0))
    phi = np.arctan2(V[:, 1], V[:, 0])
    Y = _real_sph_harms(lmax, theta, phi)
    while True:
        r = np.ones(V.shape[0])
        coef = {}
        for l in range(1, lmax + 1):
            for m in range(-l, l + 1):
                c = rng.normal(0.0, scale / l)
                coef[(l, m)] = c
                r += c * Y[(l, m)]
        if r.min() >= 0.5:
            return V * r[:, None], coef


def _face_neighbours(F: np.ndarray) -> np.ndarray:
    """nb[f, c] = the face across edge (F[f, c], F[f, c+1]) of a closed, consistently oriented mesh."""
    nf = F.shape[0]
    nv = int(F.max()) + 1
    a = F.astype(np.int64)
    b = np.roll(a, -1, axis=1)
    key = (a * nv + b).reshape(-1)
    rkey = (b * nv + a).reshape(-1)
    order = np.argsort(key)
    sk = key[order]
    pos = np.searchsorted(sk, rkey)
    if not (pos < sk.size).all() or not (sk[np.minimum(pos, sk.size - 1)] == rkey).all():
        raise ValueError("mesh must be closed, manifold and consistently oriented")
    return (order[pos] // 3).reshape(nf, 3)


def _smooth_labels(nb: np.ndarray, lab: np.ndarray, max_rounds: int = 200) -> np.ndarray:
    """A face whose neighbours agree on another label (two of three) takes it.

    This removes the one-triangle teeth that a vertex-based clustering leaves on
    a triangulated surface: there the cut path turns by about 120 degrees, and
    the geodesic zipper crowds boundary points at such sharp corners.
    """
    lab = lab.copy()
    for _ in range(max_rounds):
        l = lab[nb]
        m = np.where(l[:, 0] == l[:, 1], l[:, 0],
                     np.where(l[:, 1] == l[:, 2], l[:, 1], np.where(l[:, 0] == l[:, 2], l[:, 0], -1)))
        chg = np.flatnonzero((m >= 0) & (m != lab))
        if chg.size == 0:
            break
        # update an independent set only (no two changed faces adjacent), so it cannot oscillate
        mark = np.zeros(lab.size, dtype=bool)
        take = []
        for f in chg:
            if not mark[f]:
                take.append(f)
                mark[nb[f]] = True
                mark[f] = True
        take = np.array(take)
        lab[take] = m[take]
    return lab


def _vertex_rings(F: np.ndarray, nb: np.ndarray, verts: np.ndarray):
    """Faces around each vertex of `verts`, in rotational order."""
    nf = F.shape[0]
    corner_v = F.reshape(-1)
    o = np.argsort(corner_v, kind="stable")
    nv = int(F.max()) + 1
    starts = np.searchsorted(corner_v[o], np.arange(nv + 1))
    rings = {}
    for v in verts:
        cs = o[starts[v]:starts[v + 1]]
        where = {int(c // 3): int(c % 3) for c in cs}
        f0 = int(cs[0] // 3)
        ring = [f0]
        f = f0
        while True:
            f = int(nb[f, (where[f] + 2) % 3])
            if f == f0:
                break
            ring.append(f)
        rings[int(v)] = ring
    return rings


def _fix_pinches(F: np.ndarray, nb: np.ndarray, label: np.ndarray, max_rounds: int = 50) -> np.ndarray:
    """Relabel faces so that around every vertex each label occupies one contiguous fan.

    A label met in two separate runs around a vertex would make that vertex a
    pinch of the subdomain boundary.  Such a vertex has more cut edges than
    labels around it; the shorter run of the repeated label takes the label of
    the run before it.  Repeats until no vertex is a pinch.
    """
    label = label.copy()
    nv = int(F.max()) + 1
    a = F.astype(np.int64)
    b = np.roll(a, -1, axis=1)
    for _ in range(max_rounds):
        cut = label[:, None] != label[nb]                       # each cut edge seen from both faces
        ncut = np.zeros(nv, dtype=np.int64)
        np.add.at(ncut, a[cut], 1)
        np.add.at(ncut, b[cut], 1)
        ncut //= 2                                              # two faces, two endpoints each -> 2 per vertex
        nl = int(label.max()) + 1
        pairs = np.unique(a.reshape(-1) * nl + np.repeat(label, 3).astype(np.int64))
        ndist = np.bincount(pairs // nl, minlength=nv)
        bad = np.flatnonzero((ncut > ndist) & (ndist >= 2))
        if bad.size == 0:
            return label
        rings = _vertex_rings(F, nb, bad)
        for v in bad:
            ring = rings[int(v)]
            rl = label[ring]
            m = len(ring)
            shift = next(t for t in range(m) if rl[t] != rl[t - 1])
            ring = ring[shift:] + ring[:shift]
            rl = label[ring]
            runs = []
            s0 = 0
            for t in range(1, m + 1):
                if t == m or rl[t] != rl[s0]:
                    runs.append((s0, t, int(rl[s0])))
                    s0 = t
            seen = {}
            for (p, q, L) in runs:
                seen.setdefault(L, []).append((p, q))
            for L, rs in seen.items():
                if len(rs) > 1:
                    rs = sorted(rs, key=lambda pq: pq[1] - pq[0])
                    for (p, q) in rs[:-1]:
                        prev_label = int(rl[p - 1]) if p > 0 else int(rl[-1])
                        for t in range(p, q):
                            label[ring[t]] = prev_label
    raise RuntimeError("pinch removal did not converge")


def _components(nb: np.ndarray, lab: np.ndarray) -> np.ndarray:
    """Connected components of faces through edges whose two faces share a label."""
    import scipy.sparse as sp
    import scipy.sparse.csgraph as cg
    nf = lab.size
    f = np.repeat(np.arange(nf), 3)
    g = nb.reshape(-1)
    keep = lab[f] == lab[g]
    A = sp.coo_matrix((np.ones(int(keep.sum())), (f[keep], g[keep])), shape=(nf, nf))
    return cg.connected_components(A, directed=False)[1]


def _euler(F: np.ndarray, comp: np.ndarray, ncomp: int) -> np.ndarray:
    """V - E + F of every face component."""
    nf = F.shape[0]
    fc = np.bincount(comp, minlength=ncomp)
    nv = int(F.max()) + 1
    cc = np.repeat(comp, 3).astype(np.int64)
    vc = np.unique(F.reshape(-1).astype(np.int64) * ncomp + cc)
    vcount = np.bincount(vc % ncomp, minlength=ncomp)
    a = F.astype(np.int64)
    b = np.roll(a, -1, axis=1)
    ekey = np.minimum(a, b).reshape(-1) * nv + np.maximum(a, b).reshape(-1)
    ec = np.unique(ekey * ncomp + cc)
    ecount = np.bincount(ec % ncomp, minlength=ncomp)
    return vcount - ecount + fc


def sphere_labels(V, F, k, rng, ratio_max=4.0, max_iter=50):
    """Seeded k-means on vertex positions, cleaned into disk-shaped pieces.

    1. k-means++ seeding and Lloyd iterations on the vertex positions (stopping
       once every cluster is non-empty and the size ratio is <= ratio_max);
    2. a face takes the label of the majority of its vertices (three different
       labels: the smallest);
    3. one-triangle teeth are smoothed away, pinched vertices removed, and a
       label split into several pieces keeps its largest; pieces smaller than
       1% of the mean size join the neighbour they share most edges with.
    Returns (labels numbered by first face, final size ratio of the k-means step).
    """
    nv = V.shape[0]
    centres = [V[rng.integers(nv)]]
    d2 = np.sum((V - centres[0]) ** 2, axis=1)
    for _ in range(1, k):
        p = d2 / d2.sum()
        c = V[rng.choice(nv, p=p)]
        centres.append(c)
        d2 = np.minimum(d2, np.sum((V - c) ** 2, axis=1))
    C = np.array(centres)
    vl = None
    ratio = None
    bs = 65536
    for it in range(max_iter):
        vl = np.empty(nv, dtype=np.int64)
        for s in range(0, nv, bs):
            vl[s:s + bs] = np.argmin(((V[s:s + bs, None, :] - C[None]) ** 2).sum(-1), axis=1)
        cnt = np.bincount(vl, minlength=k)
        ratio = cnt.max() / max(cnt.min(), 1)
        if cnt.min() > 0 and ratio <= ratio_max and it > 0:
            break
        for j in range(k):
            if cnt[j] > 0:
                C[j] = V[vl == j].mean(0)
    fl3 = vl[F]
    a, b, c = fl3[:, 0], fl3[:, 1], fl3[:, 2]
    lab = np.where(a == b, a, np.where(b == c, b, np.where(a == c, a, np.minimum(np.minimum(a, b), c))))
    lab = lab.astype(np.int64)
    nf = F.shape[0]
    nb = _face_neighbours(F)
    for _ in range(50):
        lab = _smooth_labels(nb, lab)
        lab = _fix_pinches(F, nb, lab)
        comp = _components(nb, lab)
        ncomp = int(comp.max()) + 1
        sizes = np.bincount(comp, minlength=ncomp)
        comp_label = np.zeros(ncomp, dtype=np.int64)
        comp_label[comp] = lab
        best = np.full(int(lab.max()) + 1, -1, dtype=np.int64)
        for cid in np.argsort(-sizes, kind="stable"):
            if best[comp_label[cid]] < 0:
                best[comp_label[cid]] = cid
        todo = [cid for cid in range(ncomp)
                if best[comp_label[cid]] != cid or sizes[cid] < 0.01 * nf / k]
        chi = _euler(F, comp, ncomp)
        todo += [cid for cid in range(ncomp) if chi[cid] != 1 and cid not in todo]
        if not todo:
            break
        f_all = np.repeat(np.arange(nf), 3)
        g_all = nb.reshape(-1)
        for cid in sorted(todo, key=lambda c: sizes[c]):
            sel = (comp[f_all] == cid) & (comp[g_all] != cid)
            other = comp[g_all[sel]]
            if other.size == 0:
                continue
            tgt = int(np.bincount(other).argmax())
            lab[comp == cid] = comp_label[tgt]
            comp[comp == cid] = tgt
    else:
        raise RuntimeError("label clean-up did not converge")
    _, first = np.unique(lab, return_index=True)
    order = np.argsort(first)
    remap = np.empty(lab.max() + 1, dtype=np.int64)
    remap[np.unique(lab)[order]] = np.arange(order.size)
    return remap[lab].astype(np.int32), float(ratio)


def small_sphere_case(level: int = 3, k: int = 6, seed: int = 0, perturb: bool = True) -> MeshCase:
    rng = np.random.default_rng(SEED_BASE + 2000 + seed)
    V, F = icosphere(level)
    meta = {}
    if perturb:
        V, coef = perturb_sphere(V, rng, lmax=4, scale=0.05)
    lab, ratio = sphere_labels(V, F, k, rng)
    return MeshCase(f"sphere{level}_k{k}_s{seed}", V, F, lab, "sphere",
                    dict(level=level, k=k, ratio=ratio, **meta))


def case_c3(level: int = 8, k: int = 64) -> MeshCase:
    """Icosphere level 8, radius perturbed by spherical harmonics l<=8, 64 k-means pieces."""
    rng = np.random.default_rng(SEED_BASE + 3)
    V, F = icosphere(level)
    V, _ = perturb_sphere(V, rng, lmax=8, scale=0.05)
    lab, ratio = sphere_labels(V, F, k, rng)
    return MeshCase("C3" if level == 8 else f"C3_l{level}", V, F, lab, "sphere",
                    dict(level=level, k=k, ratio=ratio))


# ----------------------------------------------------------------------------
# C4: training Laplacians
# ----------------------------------------------------------------------------

def c4_training_meshes(seed: int = 0, n_height: int = 1000, n_sphere: int = 1000):
    """The learned-preconditioner training recipe: meshes whose pieces have about
    1k-20k vertices, yielded one at a time until about n_height pieces of bump
    height fields (grids 128^2-512^2, 8-32 bumps of C2's distribution, C2's
    vertex jitter, block partitions) and n_sphere pieces of perturbed icospheres
    (levels 6-7, C3's perturbation, k-means pieces) are reached.  Seeds are
    disjoint from the benchmark cases."""
    rng = np.random.default_rng(SEED_BASE + 4000 + seed)
    count, t = 0, 0
    while count < n_height:
        n = int(rng.choice([128, 192, 256, 384, 512]))
        size = float(np.exp(rng.uniform(np.log(1200.0), np.log(18000.0))))
        blocks = max(1.0, n * n / size)
        bx = max(1, int(round(np.sqrt(blocks * rng.uniform(0.5, 2.0)))))
        by = max(1, int(round(blocks / bx)))
        nb = int(rng.integers(8, 33))
        count += bx * by
        yield small_grid_case(n, bx, by, seed=40_000 + 1_000 * seed + t, jitter=1e-3 * (n - 1), nbumps=nb)
        t += 1
    count = 0
    while count < n_sphere:
        level = int(rng.choice([6, 7]))
        nv = 10 * 4 ** level + 2
        size = float(np.exp(rng.uniform(np.log(1200.0), np.log(18000.0))))
        k = int(min(64, max(2, round(nv / size))))
        srng = np.random.default_rng(SEED_BASE + 44_000 + 1_000 * seed + t)
        V, F = icosphere(level)
        V, _ = perturb_sphere(V, srng, lmax=8, scale=0.05)
        lab, ratio = sphere_labels(V, F, k, srng)
        count += int(lab.max()) + 1
        yield MeshCase(f"c4sphere{level}_k{k}_s{t}", V, F, lab, "sphere", dict(level=level, k=k, ratio=ratio))
        t += 1

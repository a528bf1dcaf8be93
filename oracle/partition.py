"""Oracle step O1: surface partition (Section 4.1).

The paper partitions S = (V, F) with a prescribed cut-edge set: E is the edge
set minus cut edges and boundary edges, the graph G built on E has K connected
components, the faces of component i form F_i and the vertices they touch form
V_i.  Properties (i)-(iv) of Section 4.1 follow.

Reading used here (the paper takes cut edges, the configurations give labels):
an interior edge is a cut edge when its two faces carry different labels.
Components are numbered by their smallest face index.  Each S_i must be a
topological disk: Euler characteristic V - E + F = 1 and one boundary loop with
no pinched vertex.  The loop is listed counter-clockwise (the face lies to the
left of each boundary half-edge) starting at its smallest global vertex index.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph


class TopologyError(ValueError):
    pass


@dataclasses.dataclass
class Sub:
    faces: np.ndarray   # global face ids, ascending
    verts: np.ndarray   # global vertex ids, ascending; local index = position
    loop: np.ndarray    # global vertex ids of the CCW boundary loop


@dataclasses.dataclass
class Partition:
    nv: int
    nf: int
    face_sub: np.ndarray      # int32 [nf]
    subs: list

    @property
    def K(self) -> int:
        return len(self.subs)


def _edge_keys(F, nv):
    a = np.concatenate([F[:, 0], F[:, 1], F[:, 2]]).astype(np.int64)
    b = np.concatenate([F[:, 1], F[:, 2], F[:, 0]]).astype(np.int64)
    return a, b


def partition(V: np.ndarray, F: np.ndarray, label: np.ndarray) -> Partition:
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    label = np.asarray(label)
    nv = V.shape[0]
    nf = F.shape[0]
    if F.ndim != 2 or F.shape[1] != 3 or label.shape != (nf,):
        raise ValueError("bad shapes")
    if nf == 0 or F.min() < 0 or F.max() >= nv:
        raise ValueError("face index out of range")
    if np.any((F[:, 0] == F[:, 1]) | (F[:, 1] == F[:, 2]) | (F[:, 0] == F[:, 2])):
        raise TopologyError("face with a repeated vertex")

    # undirected edges and the faces on each
    a, b = _edge_keys(F, nv)
    fid = np.tile(np.arange(nf), 3)
    ukey = np.minimum(a, b) * nv + np.maximum(a, b)
    order = np.argsort(ukey, kind="stable")
    uk = ukey[order]
    starts = np.flatnonzero(np.r_[True, uk[1:] != uk[:-1]])
    counts = np.diff(np.r_[starts, uk.size])
    if counts.max() > 2:
        raise TopologyError("non-manifold edge (more than two faces)")
    # each directed half-edge must be unique (consistent orientation)
    dkey = a * nv + b
    if np.unique(dkey).size != dkey.size:
        raise TopologyError("inconsistently oriented faces")

    # face graph G on interior edges that are not cut edges
    two = starts[counts == 2]
    f0 = fid[order[two]]
    f1 = fid[order[two + 1]]
    keep = label[f0] == label[f1]
    G = sp.coo_matrix((np.ones(int(keep.sum())), (f0[keep], f1[keep])), shape=(nf, nf))
    _, comp = csgraph.connected_components(G, directed=False)
    # number components by their smallest face index
    first = np.full(comp.max() + 1, nf, dtype=np.int64)
    np.minimum.at(first, comp, np.arange(nf))
    rank = np.empty_like(first)
    rank[np.argsort(first)] = np.arange(first.size)
    face_sub = rank[comp].astype(np.int32)

    subs = []
    for i in range(first.size):
        faces = np.flatnonzero(face_sub == i)
        Fi = F[faces]
        verts = np.unique(Fi)
        ai, bi = _edge_keys(Fi, nv)
        d = ai * nv + bi
        rev = bi * nv + ai
        bmask = ~np.isin(rev, d)
        ba, bb = ai[bmask], bi[bmask]
        if ba.size == 0:
            raise TopologyError(f"subdomain {i} has no boundary (closed component)")
        nxt = {}
        for s, t in zip(ba.tolist(), bb.tolist()):
            if s in nxt:
                raise TopologyError(f"subdomain {i}: pinched boundary vertex {s}")
            nxt[s] = t
        start = int(ba.min())
        loop = [start]
        v = nxt[start]
        while v != start:
            loop.append(v)
            if len(loop) > ba.size:
                raise TopologyError(f"subdomain {i}: broken boundary loop")
            v = nxt[v]
        if len(loop) != ba.size:
            raise TopologyError(f"subdomain {i}: more than one boundary loop")
        # Euler characteristic of a disk
        ue = np.unique(np.minimum(ai, bi) * nv + np.maximum(ai, bi)).size
        chi = verts.size - ue + faces.size
        if chi != 1:
            raise TopologyError(f"subdomain {i}: Euler characteristic {chi} != 1")
        subs.append(Sub(faces=faces, verts=verts, loop=np.array(loop, dtype=np.int64)))
    return Partition(nv=nv, nf=nf, face_sub=face_sub, subs=subs)


def local_faces(part: Partition, F: np.ndarray, i: int) -> np.ndarray:
    """Faces of S_i in local vertex indices (rank in the sorted vertex list)."""
    s = part.subs[i]
    return np.searchsorted(s.verts, np.asarray(F, dtype=np.int64)[s.faces])

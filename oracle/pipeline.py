"""Oracle: Algorithm 3 (PGCP) end to end, stage by stage.

  1. partition the mesh into K submeshes (Section 4.1)
  2. DNCP of every submesh; only boundary coordinates are kept (Section 4.2)
  3. partial welding of the boundary coordinates (Section 4.3)
  4. optional disk / sphere constraint (Section 4.4)
  5. harmonic map of every submesh with the welded boundary (Section 4.5)
  6. angle distortion, Beltrami coefficient and flip check (Sections 3.5, 5)
  7. stereographic projection for the sphere (Section 4.5)

Every stage's output is returned so the GPU path can be compared stage by
stage.  Stage wall-clock times are recorded in ``times``.
"""
from __future__ import annotations

import time

import numpy as np

from .cotan import cotan_laplacian
from .distortion import distortion
from .dncp import dncp
from .harmonic import harmonic
from .partition import local_faces, partition
from .sphere import chart, chart_centre, chart_inv, inv_stereo
from .weld import weld


def prepare(V, F, label):
    part = partition(V, F, label)
    subs = []
    for i, s in enumerate(part.subs):
        P = np.asarray(V, dtype=np.float64)[s.verts]
        T = local_faces(part, F, i)
        loop_local = np.searchsorted(s.verts, s.loop)
        subs.append(dict(P=P, T=T, loop_local=loop_local, loop=s.loop, verts=s.verts))
    return part, subs


def local_params(subs, with_L=True):
    out = []
    for s in subs:
        L = cotan_laplacian(s["P"], s["T"])
        u = dncp(s["P"], s["T"], s["loop_local"], s["loop"], L=L)
        s["L"] = L
        out.append(u[s["loop_local"], 0] + 1j * u[s["loop_local"], 1])
    return out


def harmonic_all(subs, welded, mode):
    vals = []
    charts = []
    for s in subs:
        ub = np.array([welded[int(v)] for v in s["loop"]], dtype=np.complex128)
        if mode == "sphere":
            c = chart_centre(ub)
            u = harmonic(s["L"], s["loop_local"], chart(ub, c))
            u = chart_inv(u, c)
            charts.append(c)
        else:
            u = harmonic(s["L"], s["loop_local"], ub)
        vals.append(u)
    return vals, charts


def assemble(nv, subs, vals, welded, mode):
    z = np.full(nv, np.nan + 0j, dtype=np.complex128)
    for s, u in zip(subs, vals):
        z[s["verts"]] = u
    for v, c in welded.items():
        z[v] = c
    if mode == "sphere":
        return inv_stereo(z)
    return np.column_stack([z.real, z.imag])


def pgcp(V, F, label, mode="free", times=None):
    if times is None:
        times = {}
    t = time.perf_counter()
    part, subs = prepare(V, F, label)
    times["partition"] = time.perf_counter() - t
    t = time.perf_counter()
    bdy = local_params(subs)
    times["assemble+dncp"] = time.perf_counter() - t
    t = time.perf_counter()
    welded = weld([s["loop"] for s in subs], bdy, mode, sizes=[len(s["T"]) for s in subs])
    times["weld"] = time.perf_counter() - t
    t = time.perf_counter()
    vals, charts = harmonic_all(subs, welded, mode)
    phi = assemble(np.asarray(V).shape[0], subs, vals, welded, mode)
    times["harmonic"] = time.perf_counter() - t
    t = time.perf_counter()
    dist = distortion(np.asarray(V), np.asarray(F), phi)
    times["distortion"] = time.perf_counter() - t
    return dict(part=part, subs=subs, bdy=bdy, welded=welded, phi=phi, dist=dist,
                charts=charts, times=times)

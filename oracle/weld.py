"""Oracle steps O4-O5: partial welding (Sections 3.4, 4.3.2, 4.4).

Points live on the extended complex plane; a point is a complex number plus an
"is infinity" flag.  Every map is applied to whole point arrays.

Geodesic algorithm (Section 3.4) and its paused form, Algorithm 1:
  g_1(z)     = sqrt((z - z_1) / (z - z_0))                 z_0 -> inf, z_1 -> 0
  L_xi(z)    = (Re xi/|xi|^2) z / (1 + i (Im xi/|xi|^2) z)  {0, xi, rho} -> {0, 1, inf}
  g_j(z)     = sqrt(L_xi_j(z)^2 - 1),  xi_j = image of z_j,  j = 2..k
  g_{k+1}(z) = z / (1 - z / zeta),     zeta = image of z_0
               (squared for the full geodesic algorithm, which ends in H)
Algorithm 2 (partial welding of two intermediate forms A, B):
  T^alpha_beta(z) = z / (-2ab/(a-b) - i (a+b)/(a-b) z)      {ai, 0, bi} -> {i, 0, -i}
  h_j(z)     = sqrt(T(z)^2 + 1),  j = k-1..1
  h_0(z)     = (z / (1 - z / eta))^2,  eta = image of A_0 = B_0
  then the Mobius map taking {a~_{m+1}, b~_{n+1}, (a~_{m+2} + b~_{n+2})/2} to {-1, 1, inf}
  (the printed a~_{n+2} is read as b~_{n+2}).
  The paper states alpha = ai, beta = bi with a > 0 > b.  Once earlier closing
  maps have carried part of the unglued arcs through infinity, alpha and beta
  can sit on the same half-axis; reading: the same formula is kept, since it is
  still the unique Mobius self-map of the right half-plane with
  {alpha, 0, beta} -> {i, 0, -i} whenever alpha, 0, beta follow the boundary's
  orientation, which is exactly -2ab/(a-b) > 0 (a > 0 > b, or a < b of one sign).

Square-root branches.  The paper fixes the branch (-1)^{1/2} = +i for A and -i
for B.  Reading used here: each map is conformal on the right half-plane,
where every data point lies except the ones already pushed onto the imaginary
axis, so a point on the axis takes the limit of the map from the right
half-plane:
  * the point sent to L = 0 (the previously zipped point) goes to branch * i;
  * other zipped points, L = i s, go to i sgn(s) sqrt(s^2 + 1);
  * in h_j, unglued arc points T = i t go to sqrt(1 - t^2) when |t| <= 1 and to
    i sgn(t) sqrt(t^2 - 1) otherwise; the glued pair itself goes to 0;
  * every other point takes the principal root (Re >= 0).
Points known to lie on the imaginary axis (by their index) are kept exactly on
it; points known to be 0 or infinity are set exactly.

Weld order (the paper only shows a three-piece example, and for the sphere
merges down to two big components before closing): a balanced merge tree.  In
each round disjoint pairs of components that share one contiguous boundary arc
of at least 3 vertices are welded.  Pairs sharing a long arc relative to their
loops come first: a union glued along a short arc has a narrow neck, the zipper
crowds points there, and a later weld through it breaks down in floating
point.  Among equally fat pairs the smaller combined size goes first: welding
a small piece onto a much larger union makes the normalisation below
ill-conditioned (the two centres sit close together relative to the union).
Sequences: A = the lower-id
component's CCW outer loop starting at the arc's first vertex a_0, then its
other tracked points, then the auxiliary points 0 and inf; B = the other
component's loop traversed clockwise from a_0, then its other tracked points,
then 0 and inf.  After the weld a glued vertex keeps a~_j.

Disk constraint (Section 4.4.1): the full geodesic algorithm on the final
outer loop (CCW from its smallest global index, all points zipped, squared
final map onto H), then w = (z - i)/(z + i) onto the unit disk.

Sphere constraint (Section 4.4.2): merge until two components are left, then a
closed weld: Algorithm 2 with the arc equal to the whole loop (starting at its
smallest global index), so every loop point is glued.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


class WeldError(ValueError):
    pass


# ----------------------------------------------------------------------------
# extended-plane helpers
# ----------------------------------------------------------------------------

def _ctype(x):
    """Complex working type of the input: complex128, or a wider complex type
    when the input carries one (an extended-precision run of the same steps,
    used as a reference for the conditioning of long welds)."""
    return np.result_type(np.asarray(x).dtype, np.complex128)


def _csqrt(w):
    return np.sqrt(w.astype(_ctype(w)))


def _axis_sqrt_minus1(s):
    """sqrt(L^2 - 1) for L = i s taken from the right half-plane."""
    return 1j * np.sign(s) * np.sqrt(s * s + 1.0)


def L_coeffs(xi):
    """(c, d) of L_xi(z) = c z / (1 + i d z), c = Re xi/|xi|^2, d = Im xi/|xi|^2."""
    r2 = xi.real * xi.real + xi.imag * xi.imag
    return xi.real / r2, xi.imag / r2


def L_map(xi, z):
    c, d = L_coeffs(xi)
    return c * z / (1.0 + 1j * d * z)


def T_coeffs(a, b):
    """(c0, c1) of T(z) = z / (c0 - i c1 z) for alpha = i a, beta = i b."""
    return -2.0 * a * b / (a - b), (a + b) / (a - b)


def T_map(a, b, z):
    c0, c1 = T_coeffs(a, b)
    return z / (c0 - 1j * c1 * z)


# ----------------------------------------------------------------------------
# Algorithm 1 (and the full geodesic algorithm)
# ----------------------------------------------------------------------------

def intermediate_form(z, inf, k, branch, squared_final=False, check=True):
    """Apply g_1..g_k and the final map to points z[0..N-1] (z_0..z_k = arc).

    branch is +1 (branching (-1)^{1/2} = i) or -1 ((-1)^{1/2} = -i).
    Returns new (z, inf).  With squared_final=True this is the geodesic
    algorithm of Section 3.4 with the final map onto the upper half-plane.
    """
    z = np.array(z, dtype=_ctype(z))
    inf = np.array(inf, dtype=bool)
    N = z.size
    if k < 1 or k >= N:
        raise WeldError("arc too short")
    if inf[0] or inf[1]:
        raise WeldError("data point at infinity")
    idx = np.arange(N)

    # g_1
    z0, z1 = z[0], z[1]
    out = np.empty(N, dtype=z.dtype)
    oinf = np.zeros(N, dtype=bool)
    gen = (idx >= 2) & ~inf
    out[gen] = _csqrt((z[gen] - z1) / (z[gen] - z0))
    out[inf] = 1.0
    out[0] = 0.0
    oinf[0] = True
    out[1] = 0.0
    z, inf = out, oinf

    # g_j, j = 2..k
    for j in range(2, k + 1):
        xi = z[j]
        if inf[j] or xi.real <= 0.0:
            raise WeldError(f"zipper point {j} left the right half-plane")
        c, d = L_coeffs(xi)
        Lz = np.empty(N, dtype=z.dtype)
        Linf = np.zeros(N, dtype=bool)
        fin = ~inf
        den = 1.0 + 1j * d * z[fin]
        Lz[fin] = c * z[fin] / den
        Linf[fin] = den == 0
        if d != 0.0:
            Lz[inf] = -1j * c / d
        else:
            Linf[inf] = True
        out = np.empty(N, dtype=z.dtype)
        oinf = Linf.copy()
        zipped = (idx < j - 1) & ~Linf
        out[zipped] = _axis_sqrt_minus1(Lz[zipped].imag)
        gen = (idx > j) & ~Linf
        out[gen] = _csqrt(Lz[gen] * Lz[gen] - 1.0)
        out[j - 1] = branch * 1j
        oinf[j - 1] = False
        out[j] = 0.0
        oinf[j] = False
        z, inf = out, oinf

    # final map g_{k+1}
    zeta_inf = bool(inf[0])
    zeta = z[0]
    out = np.empty(N, dtype=z.dtype)
    oinf = np.zeros(N, dtype=bool)
    fin = ~inf
    if zeta_inf:
        out[fin] = z[fin]
        oinf[inf] = True
    else:
        den = 1.0 - z[fin] / zeta
        out[fin] = z[fin] / den
        oinf[fin] = den == 0
        out[inf] = -zeta
    arc = (idx >= 1) & (idx < k)
    out[arc] = 1j * out[arc].imag
    out[0] = 0.0
    oinf[0] = True
    out[k] = 0.0
    oinf[k] = False
    if squared_final:
        out = out * out
    z, inf = out, oinf
    if check and not squared_final:
        bad = np.flatnonzero(branch * z[1:k].imag <= 0.0)
        if bad.size:
            raise WeldError(f"Algorithm 1 postcondition failed at arc point {bad[0] + 1}")
    return z, inf


# ----------------------------------------------------------------------------
# Algorithm 2
# ----------------------------------------------------------------------------

def _close(z, inf, j, c0, c1, on_axis, glued_pair):
    """h_j applied to one point set."""
    N = z.size
    Tz = np.empty(N, dtype=z.dtype)
    Tinf = np.zeros(N, dtype=bool)
    fin = ~inf
    den = c0 - 1j * c1 * z[fin]
    Tz[fin] = z[fin] / den
    Tinf[fin] = den == 0
    if c1 != 0.0:
        Tz[inf] = 1j / c1
    else:
        Tinf[inf] = True
    out = np.empty(N, dtype=z.dtype)
    oinf = Tinf.copy()
    ax = on_axis & ~Tinf
    t = Tz[ax].imag
    small = np.abs(t) <= 1.0
    r = np.empty(t.size, dtype=z.dtype)
    r[small] = np.sqrt(1.0 - t[small] * t[small])
    r[~small] = 1j * np.sign(t[~small]) * np.sqrt(t[~small] * t[~small] - 1.0)
    out[ax] = r
    gen = ~on_axis & ~Tinf
    out[gen] = _csqrt(Tz[gen] * Tz[gen] + 1.0)
    out[glued_pair] = 0.0
    oinf[glued_pair] = False
    return out, oinf


def partial_weld(za, ia, zb, ib, k):
    """Algorithm 2 on two intermediate forms (arc = indices 0..k in both)."""
    Na, Nb = za.size, zb.size
    idxa = np.arange(Na)
    idxb = np.arange(Nb)
    for j in range(k - 1, 0, -1):
        a = za[j].imag
        b = zb[j].imag
        if ia[j] or ib[j] or a == 0.0 or b == 0.0 or a == b:
            raise WeldError(f"Algorithm 2: pair {j} degenerate")
        c0, c1 = T_coeffs(a, b)
        if not c0 > 0.0:
            raise WeldError(f"Algorithm 2: pair {j} out of cyclic order")
        za, ia = _close(za, ia, j, c0, c1, idxa < j, j)
        zb, ib = _close(zb, ib, j, c0, c1, idxb < j, j)
    # h_0
    eta_inf = bool(ia[0])
    eta = za[0]

    def h0(z, inf):
        out = np.empty(z.size, dtype=z.dtype)
        oinf = np.zeros(z.size, dtype=bool)
        fin = ~inf
        if eta_inf:
            out[fin] = z[fin] * z[fin]
            oinf[inf] = True
        else:
            den = 1.0 - z[fin] / eta
            w = z[fin] / den
            out[fin] = w * w
            oinf[fin] = den == 0
            out[inf] = eta * eta
        out[0] = 0.0
        oinf[0] = True
        return out, oinf

    za, ia = h0(za, ia)
    zb, ib = h0(zb, ib)
    return za, ia, zb, ib


def mobius3(z1, z2, z3):
    """Coefficients (a, b, c, d) of the Mobius map {z1, z2, z3} -> {-1, 1, inf}."""
    # M(z) = 2 (z - z1)(z2 - z3) / ((z - z3)(z2 - z1)) - 1
    p = 2.0 * (z2 - z3)
    q = z2 - z1
    # (2(z2-z3)(z - z1) - (z2 - z1)(z - z3)) / ((z2-z1)(z - z3))
    a = p - q
    b = -p * z1 + q * z3
    c = q
    d = -q * z3
    return a, b, c, d


def apply_mobius(coef, z, inf):
    a, b, c, d = coef
    out = np.empty(z.size, dtype=z.dtype)
    oinf = np.zeros(z.size, dtype=bool)
    fin = ~inf
    den = c * z[fin] + d
    out[fin] = (a * z[fin] + b) / den
    oinf[fin] = den == 0
    out[inf] = a / c
    return out, oinf


# ----------------------------------------------------------------------------
# weld driver
# ----------------------------------------------------------------------------

def shared_arc(loop_a, loop_b):
    """Shared boundary of two components with CCW loops loop_a, loop_b.

    Returns ("partial", start, k): loop_a[start .. start+k] (cyclic) is the one
    contiguous shared arc (k >= 2) and it appears reversed and contiguous in
    loop_b; ("closed", None, None) when both loops are the same vertex cycle;
    or None when the two cannot be welded in one step.
    """
    pos_a = {v: i for i, v in enumerate(loop_a)}
    pos_b = {v: i for i, v in enumerate(loop_b)}
    shared = [v for v in loop_b if v in pos_a]
    La, Lb = len(loop_a), len(loop_b)
    if len(shared) < 3:
        return None
    if len(shared) == La == Lb:
        return ("closed", None, None)
    pos = sorted(pos_a[v] for v in shared)
    gaps = [(pos[(t + 1) % len(pos)] - pos[t]) % La for t in range(len(pos))]
    if sum(g != 1 for g in gaps) != 1:
        return None
    t = [g != 1 for g in gaps].index(True)
    start = pos[(t + 1) % len(pos)]
    k = len(pos) - 1
    arc = [loop_a[(start + s) % La] for s in range(k + 1)]
    for s in range(k):
        if (pos_b[arc[s]] - pos_b[arc[s + 1]]) % Lb != 1:
            return None
    return ("partial", start, k)


def merge_plan(loops, sizes, mode):
    """Balanced weld order as rounds of disjoint pairs.

    Components start as the subdomains.  In each round every weldable pair
    (one contiguous shared arc of >= 3 vertices) is a candidate.  Candidates
    are taken greedily, each component at most once per round, in order of
    decreasing fatness k / min(|loop_i|, |loop_j|) (k = shared arc length):
    two pieces glued along a short arc form a union with a narrow neck, where
    the zipper crowds points until the next weld fails in floating point.
    Ties go to the smaller combined size (face count), then the smaller ids.  A merged component is
    named by the smaller id.  In sphere mode merging stops at two components,
    which are then closed-welded.  Returns (rounds, outer loop of each final
    component by id).
    """
    comps = {i: list(map(int, l)) for i, l in enumerate(loops)}
    size = {i: int(s) for i, s in enumerate(sizes)}
    rounds = []
    target = 2 if mode == "sphere" else 1
    while len(comps) > target:
        ids = sorted(comps)
        cands = []
        for x in range(len(ids)):
            for y in range(x + 1, len(ids)):
                i, j = ids[x], ids[y]
                if not (set(comps[i]) & set(comps[j])):
                    continue
                res = shared_arc(comps[i], comps[j])
                if res is None or res[0] != "partial":
                    continue
                fat = Fraction(res[2], min(len(comps[i]), len(comps[j])))
                cands.append(((-fat, size[i] + size[j], i, j), i, j, res))
        if not cands:
            raise WeldError("no pair of components can be welded")
        cands.sort(key=lambda c: c[0])
        used = set()
        rnd = []
        for _, i, j, res in cands:
            if i in used or j in used:
                continue
            used.update((i, j))
            rnd.append((i, j))
        for i, j in rnd:
            _, start, k = shared_arc(comps[i], comps[j])
            A, Bseq = _sequences(comps[i], comps[j], start, k)
            comps[i] = A[k:] + [A[0]] + Bseq[k + 1:][::-1]
            size[i] += size.pop(j)
            del comps[j]
        rounds.append(rnd)
    if mode == "sphere":
        i, j = sorted(comps)
        if shared_arc(comps[i], comps[j]) is None or shared_arc(comps[i], comps[j])[0] != "closed":
            raise WeldError("last two components do not close the sphere")
        rounds.append([(i, j)])
    return rounds


def _sequences(loop_a, loop_b, start, k):
    """A = loop_a from a_0 (CCW); B = loop_b traversed clockwise from a_0."""
    La, Lb = len(loop_a), len(loop_b)
    A = [loop_a[(start + s) % La] for s in range(La)]
    i0 = loop_b.index(A[0])
    Bseq = [loop_b[(i0 - s) % Lb] for s in range(Lb)]
    if Bseq[:k + 1] != A[:k + 1]:
        raise WeldError("arc correspondence broken")
    return A, Bseq


def weld_pair(ca, cb, closed=False):
    """Partial (or closed) welding of two components; returns the merged one.

    A component is dict(outer=[vertex ids, CCW], z={vertex: complex}, inf={vertex: bool}).
    """
    if closed:
        L = len(ca["outer"])
        start = ca["outer"].index(min(ca["outer"]))
        k = L - 1
    else:
        res = shared_arc(ca["outer"], cb["outer"])
        if res is None or res[0] != "partial":
            raise WeldError("components do not share one contiguous arc")
        _, start, k = res
    A, Bseq = _sequences(ca["outer"], cb["outer"], start, k)
    sa, sb = set(A), set(Bseq)
    seq_a = A + sorted(v for v in ca["z"] if v not in sa)
    seq_b = Bseq + sorted(v for v in cb["z"] if v not in sb)
    va = [ca["z"][v] for v in seq_a]
    za = np.array(va + [0.0, 0.0], dtype=_ctype(va))
    ia = np.array([ca["inf"][v] for v in seq_a] + [False, True])
    vb = [cb["z"][v] for v in seq_b]
    zb = np.array(vb + [0.0, 0.0], dtype=_ctype(vb))
    ib = np.array([cb["inf"][v] for v in seq_b] + [False, True])
    za, ia = intermediate_form(za, ia, k, +1)
    zb, ib = intermediate_form(zb, ib, k, -1)
    za, ia, zb, ib = partial_weld(za, ia, zb, ib, k)
    na, nb = za.size, zb.size
    if ia[na - 2] or ib[nb - 2] or ia[na - 1] or ib[nb - 1]:
        raise WeldError("auxiliary point sent to infinity")
    coef = mobius3(za[na - 2], zb[nb - 2], 0.5 * (za[na - 1] + zb[nb - 1]))
    za, ia = apply_mobius(coef, za, ia)
    zb, ib = apply_mobius(coef, zb, ib)
    gap = np.abs(za[1:k] - zb[1:k])
    out = dict(z={}, inf={})
    for t, v in enumerate(seq_a):
        out["z"][v] = za[t]
        out["inf"][v] = bool(ia[t])
    for t, v in enumerate(seq_b):
        if t <= k:
            continue
        out["z"][v] = zb[t]
        out["inf"][v] = bool(ib[t])
    out["outer"] = [] if closed else A[k:] + [A[0]] + Bseq[k + 1:][::-1]
    info = dict(k=k, glue_gap=float(gap.max()) if gap.size else 0.0,
                scale=float(np.abs(za[:k + 1][~ia[:k + 1]]).max(initial=1.0)))
    return out, info


def disk_step(comp):
    """Geodesic algorithm on the outer loop, then the Cayley map onto the unit disk."""
    outer = comp["outer"]
    L = len(outer)
    s0 = outer.index(min(outer))
    A = [outer[(s0 + s) % L] for s in range(L)]
    sa = set(A)
    seq = A + sorted(v for v in comp["z"] if v not in sa)
    vs = [comp["z"][v] for v in seq]
    z = np.array(vs, dtype=_ctype(vs))
    zi = np.array([comp["inf"][v] for v in seq])
    z, zi = intermediate_form(z, zi, L - 1, +1, squared_final=True)
    w = np.empty(z.size, dtype=z.dtype)
    w[~zi] = (z[~zi] - 1j) / (z[~zi] + 1j)
    w[zi] = 1.0
    return dict(outer=outer, z={v: w[t] for t, v in enumerate(seq)},
                inf={v: False for v in seq})


def weld(loops, coords, mode="free", sizes=None, return_steps=False):
    """Weld all pieces; returns {global vertex: complex} (inf as complex('inf')).

    loops:  CCW boundary loops (global vertex ids) of the subdomains
    coords: DNCP boundary coordinates in loop order (complex)
    sizes:  face counts used to balance the merge tree (default: loop lengths)
    """
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        return _weld(loops, coords, mode, sizes, return_steps)


def _weld(loops, coords, mode, sizes, return_steps):
    loops = [list(map(int, l)) for l in loops]
    if sizes is None:
        sizes = [len(l) for l in loops]
    comps = {}
    for i, (l, c) in enumerate(zip(loops, coords)):
        comps[i] = dict(outer=list(l), z={v: x for v, x in zip(l, c)},
                        inf={v: False for v in l})
    steps = []
    if len(loops) > 1:
        rounds = merge_plan(loops, sizes, mode)
        last = len(rounds) - 1
        for r, rnd in enumerate(rounds):
            for i, j in rnd:
                closed = mode == "sphere" and r == last
                comps[i], info = weld_pair(comps[i], comps[j], closed=closed)
                del comps[j]
                info.update(round=r, pair=(i, j), kind="closed" if closed else "partial")
                steps.append(info)
    (cid,) = list(comps)
    comp = comps[cid]
    if mode == "disk":
        comp = disk_step(comp)
        steps.append(dict(kind="disk", k=len(comp["outer"]) - 1))
    out = {v: (complex("inf") if comp["inf"][v] else c) for v, c in comp["z"].items()}
    if return_steps:
        return out, steps, comp["outer"]
    return out

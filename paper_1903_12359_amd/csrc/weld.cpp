// Partial welding (Sections 3.4, 4.3.2, 4.4), host side.
//
// Every map of Algorithms 1 and 2 is fixed by the shared-arc points alone: the
// opening maps g_j by xi_j (the image of arc point j), the closing maps h_j by
// the images alpha_j, beta_j of arc points j, and the final maps by the images
// of arc point 0.  So each weld first runs the zipper on the (k+1) arc points of
// both sides (O(k^2)), recording the map parameters, and then sends every other
// point (rest of the loop, earlier seams, the auxiliary points 0 and infinity)
// through the recorded chain independently, in parallel.
//
// Square roots: points on the imaginary axis take the limit of the map from the
// right half-plane (zipped points of Algorithm 1: i sgn(s) sqrt(s^2+1) for
// L = i s; unglued arc points of Algorithm 2: sqrt(1-t^2) for |t| <= 1 and
// i sgn(t) sqrt(t^2-1) otherwise for T = i t); the point sent to L = 0 takes
// the branch (+i for A, -i for B); all other points take the principal root.
// Algorithm 2's T is used whenever -2ab/(a-b) > 0, i.e. alpha, 0, beta in the
// boundary's cyclic order (the paper's a > 0 > b is the common case).
//
// Merge order: balanced tree, rounds of disjoint pairs of components sharing
// one contiguous arc of >= 3 vertices, smallest combined face count first.
// Sphere mode merges down to two components and closes them.  Disk mode ends
// with the geodesic algorithm on the outer loop and w = (z - i)/(z + i).

#include <algorithm>
#include <cmath>
#include <limits>
#include <unordered_map>
#include <unordered_set>

#include "pgcp_internal.h"

namespace pgcp {
namespace {

// A point of the extended plane.
struct EP {
    cplx z;
    bool inf;
};

// Principal square root (Re >= 0; on the negative real axis the sign of the
// imaginary zero picks the half, as for the C library's csqrt).  Plain
// formula: the weld's values stay far from overflow.
inline cplx csqrt_principal(cplx w) {
    const double x = w.real(), y = w.imag();
    const double r = std::sqrt(x * x + y * y);
    if (r == 0.0) return cplx(0.0, y);
    if (x >= 0.0) {
        const double t = std::sqrt(0.5 * (r + x));
        return cplx(t, y / (2.0 * t));
    }
    const double t = std::sqrt(0.5 * (r - x));
    return cplx(std::fabs(y) / (2.0 * t), std::copysign(t, y));
}

struct Component {
    std::vector<int> outer;       // CCW loop, global ids
    std::vector<EP> zo;           // coordinates aligned with outer
    std::vector<int> tracked;     // other boundary vertices of the welded pieces
    std::vector<EP> zt;
};

// ---------------------------------------------------------------- Algorithm 1

struct ZipRecord {
    int k = 0;
    cplx z0, z1;                  // g_1 parameters
    std::vector<double> c, d;     // L_xi_j for j = 2..k (index j-2)
    bool zeta_inf = false;
    cplx zeta;
    bool squared = false;
};

// Runs g_1..g_k and the final map on the arc points arc[0..k] (in place) and
// records the parameters.  Throws Error on a broken precondition.
ZipRecord zip_arc(std::vector<EP>& arc, int k, int branch, bool squared) {
    ZipRecord R;
    R.k = k;
    R.squared = squared;
    if (arc[0].inf || arc[1].inf) throw Error{PGCP_E_WELD, "arc point at infinity"};
    R.z0 = arc[0].z;
    R.z1 = arc[1].z;
    for (int l = 2; l <= k; ++l) {
        if (arc[l].inf) {
            arc[l].z = 1.0;
            arc[l].inf = false;
        } else {
            arc[l].z = csqrt_principal((arc[l].z - R.z1) / (arc[l].z - R.z0));
        }
    }
    arc[0] = EP{0.0, true};
    arc[1] = EP{0.0, false};
    R.c.resize(std::max(0, k - 1));
    R.d.resize(std::max(0, k - 1));
    for (int j = 2; j <= k; ++j) {
        cplx xi = arc[j].z;
        if (arc[j].inf || !(xi.real() > 0.0))
            throw Error{PGCP_E_WELD, "zipper point left the right half-plane"};
        double r2 = xi.real() * xi.real() + xi.imag() * xi.imag();
        double c = xi.real() / r2, d = xi.imag() / r2;
        R.c[j - 2] = c;
        R.d[j - 2] = d;
#pragma omp parallel for schedule(static) if (k >= 384)
        for (int l = 0; l <= k; ++l) {
            if (l == j - 1) {
                arc[l] = EP{cplx(0.0, (double)branch), false};
                continue;
            }
            if (l == j) {
                arc[l] = EP{0.0, false};
                continue;
            }
            if (l < j - 1) {
                // zipped: z = i t on the imaginary axis, L = i c t / (1 - d t)
                if (arc[l].inf) {
                    if (d == 0.0) continue;   // L(inf) = inf stays inf
                    const double s = -c / d;
                    arc[l] = EP{cplx(0.0, (s > 0 ? 1.0 : -1.0) * std::sqrt(s * s + 1.0)), false};
                    continue;
                }
                const double t = arc[l].z.imag(), den = 1.0 - d * t;
                if (den == 0.0) {
                    arc[l] = EP{0.0, true};
                    continue;
                }
                const double s = c * t / den;
                const double sg = (s > 0.0) ? 1.0 : (s < 0.0 ? -1.0 : 0.0);
                arc[l] = EP{cplx(0.0, sg * std::sqrt(s * s + 1.0)), false};
                continue;
            }
            // not yet zipped: L_xi(z) = c z / (1 + i d z), principal sqrt(L^2 - 1)
            if (arc[l].inf) {
                if (d == 0.0) continue;
                const cplx L = cplx(0.0, -c / d);
                arc[l] = EP{csqrt_principal(L * L - 1.0), false};
                continue;
            }
            const cplx den = 1.0 + cplx(0.0, d) * arc[l].z;
            if (den == cplx(0.0, 0.0)) {
                arc[l] = EP{0.0, true};
                continue;
            }
            const cplx L = c * arc[l].z / den;
            arc[l] = EP{csqrt_principal(L * L - 1.0), false};
        }
    }
    // final map z / (1 - z / zeta)
    R.zeta_inf = arc[0].inf;
    R.zeta = arc[0].z;
    for (int l = 1; l <= k; ++l) {
        if (l == k) {
            arc[l] = EP{0.0, false};
            continue;
        }
        cplx w;
        if (R.zeta_inf) w = arc[l].z;
        else w = arc[l].z / (1.0 - arc[l].z / R.zeta);
        w = cplx(0.0, w.imag());
        if (squared) w = w * w;
        arc[l] = EP{w, false};
    }
    arc[0] = EP{0.0, true};
    if (!squared) {
        for (int l = 1; l < k; ++l)
            if (!(branch * arc[l].z.imag() > 0.0))
                throw Error{PGCP_E_WELD, "Algorithm 1 postcondition failed"};
    }
    return R;
}

// Sends one non-arc point through the recorded Algorithm 1 chain.
inline EP zip_point(const ZipRecord& R, EP p) {
    if (p.inf) {
        p = EP{1.0, false};
    } else {
        cplx den = p.z - R.z0;
        if (den == cplx(0.0, 0.0)) p = EP{0.0, true};
        else p.z = csqrt_principal((p.z - R.z1) / den);
    }
    for (int j = 0; j + 2 <= R.k; ++j) {
        double c = R.c[j], d = R.d[j];
        if (p.inf) {
            if (d != 0.0) p = EP{cplx(0.0, -c / d), false};
            else continue;   // L(inf) = inf, sqrt(inf) = inf
        } else {
            cplx den = 1.0 + cplx(0.0, d) * p.z;
            if (den == cplx(0.0, 0.0)) {
                p = EP{0.0, true};
                continue;
            }
            p.z = c * p.z / den;
        }
        p.z = csqrt_principal(p.z * p.z - 1.0);
    }
    if (p.inf) {
        if (R.zeta_inf) return p;
        p = EP{-R.zeta, false};
    } else if (!R.zeta_inf) {
        cplx den = 1.0 - p.z / R.zeta;
        if (den == cplx(0.0, 0.0)) return EP{0.0, true};
        p.z = p.z / den;
    }
    if (R.squared) p.z = p.z * p.z;
    return p;
}

// ---------------------------------------------------------------- Algorithm 2

struct CloseRecord {
    int k = 0;
    std::vector<double> c0, c1;   // h_j for j = k-1..1 (index k-1-j)
    bool eta_inf = false;
    cplx eta;
};

// T(z) = z / (c0 - i c1 z); T(inf) = i / c1
inline EP T_apply(double c0, double c1, const EP& p) {
    if (p.inf) {
        if (c1 != 0.0) return EP{cplx(0.0, 1.0 / c1), false};
        return p;
    }
    cplx den = cplx(c0, 0.0) - cplx(0.0, c1) * p.z;
    if (den == cplx(0.0, 0.0)) return EP{0.0, true};
    return EP{p.z / den, false};
}

inline EP h0_apply(const CloseRecord& R, EP p) {
    if (R.eta_inf) {
        if (p.inf) return p;
        return EP{p.z * p.z, false};
    }
    if (p.inf) return EP{R.eta * R.eta, false};
    cplx den = 1.0 - p.z / R.eta;
    if (den == cplx(0.0, 0.0)) return EP{0.0, true};
    cplx w = p.z / den;
    return EP{w * w, false};
}

CloseRecord close_arcs(std::vector<EP>& A, std::vector<EP>& B, int k) {
    CloseRecord R;
    R.k = k;
    for (int j = k - 1; j >= 1; --j) {
        if (A[j].inf || B[j].inf) throw Error{PGCP_E_WELD, "glued pair at infinity"};
        double a = A[j].z.imag(), b = B[j].z.imag();
        if (a == 0.0 || b == 0.0 || a == b) throw Error{PGCP_E_WELD, "degenerate glued pair"};
        double c0 = -2.0 * a * b / (a - b), c1 = (a + b) / (a - b);
        if (!(c0 > 0.0)) throw Error{PGCP_E_WELD, "glued pair out of cyclic order"};
        R.c0.push_back(c0);
        R.c1.push_back(c1);
#pragma omp parallel for schedule(static) if (k >= 384)
        for (int m = 0; m < 2 * (k + 1); ++m) {
            auto& X = m <= k ? A : B;
            const int l = m <= k ? m : m - (k + 1);
            if (l == j) {
                X[l] = EP{0.0, false};
                continue;
            }
            if (l < j && !X[l].inf) {
                // unglued arc point on the imaginary axis: T(i u) = i u / (c0 + c1 u)
                const double u = X[l].z.imag(), den = c0 + c1 * u;
                if (den == 0.0) {
                    X[l] = EP{0.0, true};
                    continue;
                }
                const double s = u / den;
                if (std::fabs(s) <= 1.0) {
                    X[l] = EP{cplx(std::sqrt(1.0 - s * s), 0.0), false};
                } else {
                    const double sg = s > 0.0 ? 1.0 : -1.0;
                    X[l] = EP{cplx(0.0, sg * std::sqrt(s * s - 1.0)), false};
                }
                continue;
            }
            EP t = T_apply(c0, c1, X[l]);
            if (t.inf) {
                X[l] = t;
            } else if (l < j) {
                const double s = t.z.imag();
                if (std::fabs(s) <= 1.0) {
                    X[l] = EP{cplx(std::sqrt(1.0 - s * s), 0.0), false};
                } else {
                    const double sg = s > 0.0 ? 1.0 : -1.0;
                    X[l] = EP{cplx(0.0, sg * std::sqrt(s * s - 1.0)), false};
                }
            } else {
                X[l] = EP{csqrt_principal(t.z * t.z + 1.0), false};
            }
        }
    }
    R.eta_inf = A[0].inf;
    R.eta = A[0].z;
    for (auto* S : {&A, &B}) {
        auto& X = *S;
        for (int l = 1; l <= k; ++l) X[l] = h0_apply(R, X[l]);
        X[0] = EP{0.0, true};
    }
    return R;
}

inline EP close_point(const CloseRecord& R, EP p) {
    for (size_t t = 0; t < R.c0.size(); ++t) {
        p = T_apply(R.c0[t], R.c1[t], p);
        if (p.inf) continue;
        p.z = csqrt_principal(p.z * p.z + 1.0);
    }
    return h0_apply(R, p);
}

// ---------------------------------------------------------------- Mobius

struct Mobius {
    cplx a, b, c, d;
};

// {z1, z2, z3} -> {-1, 1, inf}
Mobius mobius3(cplx z1, cplx z2, cplx z3) {
    cplx p = 2.0 * (z2 - z3), q = z2 - z1;
    return Mobius{p - q, -p * z1 + q * z3, q, -q * z3};
}

inline EP mobius_apply(const Mobius& M, EP p) {
    if (p.inf) return EP{M.a / M.c, false};
    cplx den = M.c * p.z + M.d;
    if (den == cplx(0.0, 0.0)) return EP{0.0, true};
    return EP{(M.a * p.z + M.b) / den, false};
}

// ---------------------------------------------------------------- one weld

Component weld_pair(Component& A, Component& B, bool closed) {
    int start, k;
    const int La = (int)A.outer.size(), Lb = (int)B.outer.size();
    if (closed) {
        if (La != Lb) throw Error{PGCP_E_WELD, "closed weld of loops of different length"};
        start = (int)(std::min_element(A.outer.begin(), A.outer.end()) - A.outer.begin());
        k = La - 1;
    } else {
        k = shared_arc(A.outer, B.outer, &start);
        if (k < 2) throw Error{PGCP_E_WELD, "components do not share one contiguous arc"};
    }
    // sequences: A from a_0 (CCW), B clockwise from a_0
    std::vector<int> Aid(La), Bid(Lb);
    std::vector<EP> Az(La), Bz(Lb);
    for (int s = 0; s < La; ++s) {
        Aid[s] = A.outer[(start + s) % La];
        Az[s] = A.zo[(start + s) % La];
    }
    int i0 = (int)(std::find(B.outer.begin(), B.outer.end(), Aid[0]) - B.outer.begin());
    if (i0 >= Lb) throw Error{PGCP_E_WELD, "arc correspondence broken"};
    for (int s = 0; s < Lb; ++s) {
        int t = ((i0 - s) % Lb + Lb) % Lb;
        Bid[s] = B.outer[t];
        Bz[s] = B.zo[t];
    }
    for (int s = 0; s <= k; ++s)
        if (Aid[s] != Bid[s]) throw Error{PGCP_E_WELD, "arc correspondence broken"};

    // arcs
    std::vector<EP> arcA(Az.begin(), Az.begin() + k + 1), arcB(Bz.begin(), Bz.begin() + k + 1);
    ZipRecord ZA = zip_arc(arcA, k, +1, false);
    ZipRecord ZB = zip_arc(arcB, k, -1, false);
    CloseRecord CR = close_arcs(arcA, arcB, k);

    // all other points: rest of each loop, tracked points, auxiliary 0 and inf
    const int na_rest = La - k - 1, nb_rest = Lb - k - 1;
    const int nat = (int)A.zt.size(), nbt = (int)B.zt.size();
    std::vector<EP> PA(na_rest + nat + 2), PB(nb_rest + nbt + 2);
    for (int s = 0; s < na_rest; ++s) PA[s] = Az[k + 1 + s];
    for (int s = 0; s < nat; ++s) PA[na_rest + s] = A.zt[s];
    PA[na_rest + nat] = EP{0.0, false};
    PA[na_rest + nat + 1] = EP{0.0, true};
    for (int s = 0; s < nb_rest; ++s) PB[s] = Bz[k + 1 + s];
    for (int s = 0; s < nbt; ++s) PB[nb_rest + s] = B.zt[s];
    PB[nb_rest + nbt] = EP{0.0, false};
    PB[nb_rest + nbt + 1] = EP{0.0, true};
    const int nA = (int)PA.size(), nB = (int)PB.size();
#pragma omp parallel for schedule(static) if (nA + nB > 2048)
    for (int s = 0; s < nA + nB; ++s) {
        if (s < nA) PA[s] = close_point(CR, zip_point(ZA, PA[s]));
        else PB[s - nA] = close_point(CR, zip_point(ZB, PB[s - nA]));
    }
    EP a0 = PA[nA - 2], ainf = PA[nA - 1], b0 = PB[nB - 2], binf = PB[nB - 1];
    if (a0.inf || b0.inf || ainf.inf || binf.inf)
        throw Error{PGCP_E_WELD, "auxiliary point sent to infinity"};
    Mobius M = mobius3(a0.z, b0.z, 0.5 * (ainf.z + binf.z));
    for (auto& p : arcA) p = mobius_apply(M, p);
#pragma omp parallel for schedule(static) if (nA + nB > 2048)
    for (int s = 0; s < nA + nB; ++s) {
        if (s < nA) PA[s] = mobius_apply(M, PA[s]);
        else PB[s - nA] = mobius_apply(M, PB[s - nA]);
    }

    Component C;
    if (!closed) {
        // new outer loop: a_k .. a_m, a_0, then B's rest reversed
        C.outer.reserve(La - k + Lb - k);
        C.outer.push_back(Aid[k]);
        C.zo.push_back(arcA[k]);
        for (int s = 0; s < na_rest; ++s) {
            C.outer.push_back(Aid[k + 1 + s]);
            C.zo.push_back(PA[s]);
        }
        C.outer.push_back(Aid[0]);
        C.zo.push_back(arcA[0]);
        for (int s = nb_rest - 1; s >= 0; --s) {
            C.outer.push_back(Bid[k + 1 + s]);
            C.zo.push_back(PB[s]);
        }
        for (int s = 1; s < k; ++s) {
            C.tracked.push_back(Aid[s]);
            C.zt.push_back(arcA[s]);
        }
    } else {
        for (int s = 0; s <= k; ++s) {
            C.tracked.push_back(Aid[s]);
            C.zt.push_back(arcA[s]);
        }
    }
    for (int s = 0; s < nat; ++s) {
        C.tracked.push_back(A.tracked[s]);
        C.zt.push_back(PA[na_rest + s]);
    }
    for (int s = 0; s < nbt; ++s) {
        C.tracked.push_back(B.tracked[s]);
        C.zt.push_back(PB[nb_rest + s]);
    }
    return C;
}

void disk_step(Component& C) {
    const int L = (int)C.outer.size();
    int start = (int)(std::min_element(C.outer.begin(), C.outer.end()) - C.outer.begin());
    std::vector<int> id(L);
    std::vector<EP> arc(L);
    for (int s = 0; s < L; ++s) {
        id[s] = C.outer[(start + s) % L];
        arc[s] = C.zo[(start + s) % L];
    }
    ZipRecord Z = zip_arc(arc, L - 1, +1, true);
    const int nt = (int)C.zt.size();
#pragma omp parallel for schedule(static) if (nt > 2048)
    for (int s = 0; s < nt; ++s) C.zt[s] = zip_point(Z, C.zt[s]);
    auto cayley = [](const EP& p) {
        if (p.inf) return EP{1.0, false};
        return EP{(p.z - cplx(0.0, 1.0)) / (p.z + cplx(0.0, 1.0)), false};
    };
    for (int s = 0; s < L; ++s) arc[s] = cayley(arc[s]);
    for (int s = 0; s < nt; ++s) C.zt[s] = cayley(C.zt[s]);
    C.outer = id;
    C.zo = arc;
}

}  // namespace

// ---------------------------------------------------------------- shared arc

int shared_arc(const std::vector<int>& la, const std::vector<int>& lb, int* start) {
    const int La = (int)la.size(), Lb = (int)lb.size();
    std::unordered_map<int, int> pos_b;
    pos_b.reserve(Lb * 2);
    for (int i = 0; i < Lb; ++i) pos_b[lb[i]] = i;
    std::vector<char> in(La, 0);
    int m = 0;
    for (int i = 0; i < La; ++i)
        if (pos_b.count(la[i])) {
            in[i] = 1;
            m++;
        }
    if (m < 3) return -1;
    if (m == La && m == Lb) return -2;
    if (m == La) return -1;
    int runs = 0, s0 = -1;
    for (int i = 0; i < La; ++i)
        if (in[i] && !in[(i + La - 1) % La]) {
            runs++;
            s0 = i;
        }
    if (runs != 1) return -1;
    const int k = m - 1;
    for (int s = 0; s < k; ++s) {
        int pa = pos_b[la[(s0 + s) % La]], pb = pos_b[la[(s0 + s + 1) % La]];
        if (((pa - pb) % Lb + Lb) % Lb != 1) return -1;
    }
    *start = s0;
    return k;
}

Error merge_plan(const std::vector<std::vector<int>>& loops, const std::vector<int64_t>& sizes,
                 int mode, std::vector<std::vector<std::pair<int, int>>>* rounds) {
    std::unordered_map<int, std::vector<int>> comps;   // id -> outer loop
    std::unordered_map<int, int64_t> size;
    for (size_t i = 0; i < loops.size(); ++i) {
        comps[(int)i] = loops[i];
        size[(int)i] = sizes[i];
    }
    const size_t target = mode == PGCP_SPHERE ? 2 : 1;
    while (comps.size() > target) {
        // candidate pairs from shared vertices
        std::unordered_map<int, std::vector<int>> owners;
        std::vector<int> ids;
        for (auto& kv : comps) ids.push_back(kv.first);
        std::sort(ids.begin(), ids.end());
        for (int id : ids)
            for (int v : comps[id]) owners[v].push_back(id);
        std::vector<std::pair<int, int>> pairs;
        for (auto& kv : owners) {
            auto& o = kv.second;
            for (size_t x = 0; x < o.size(); ++x)
                for (size_t y = x + 1; y < o.size(); ++y)
                    pairs.emplace_back(std::min(o[x], o[y]), std::max(o[x], o[y]));
        }
        std::sort(pairs.begin(), pairs.end());
        pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
        // a pair's "fatness" is its shared arc length over the shorter of the
        // two loops: pairs that share a long arc first (a union glued along a
        // short arc has a narrow neck, where the zipper crowds points), then
        // the smaller combined face count, then the ids
        struct Cand {
            int64_t k, m, s;
            int i, j;
        };
        std::vector<Cand> cands;
        for (auto& pr : pairs) {
            int st;
            int k = shared_arc(comps[pr.first], comps[pr.second], &st);
            if (k >= 2) {
                int64_t m = (int64_t)std::min(comps[pr.first].size(), comps[pr.second].size());
                cands.push_back(Cand{k, m, size[pr.first] + size[pr.second], pr.first, pr.second});
            }
        }
        if (cands.empty()) return Error{PGCP_E_WELD, "no pair of components can be welded"};
        std::sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) {
            int64_t lx = x.k * y.m, ly = y.k * x.m;
            if (lx != ly) return lx > ly;
            if (x.s != y.s) return x.s < y.s;
            if (x.i != y.i) return x.i < y.i;
            return x.j < y.j;
        });
        std::unordered_set<int> used;
        std::vector<std::pair<int, int>> rnd;
        for (auto& c : cands) {
            if (used.count(c.i) || used.count(c.j)) continue;
            used.insert(c.i);
            used.insert(c.j);
            rnd.emplace_back(c.i, c.j);
        }
        for (auto& pr : rnd) {
            auto& la = comps[pr.first];
            auto& lb = comps[pr.second];
            int st;
            int k = shared_arc(la, lb, &st);
            const int La = (int)la.size(), Lb = (int)lb.size();
            std::vector<int> A(La);
            for (int s = 0; s < La; ++s) A[s] = la[(st + s) % La];
            int i0 = (int)(std::find(lb.begin(), lb.end(), A[0]) - lb.begin());
            std::vector<int> out;
            out.insert(out.end(), A.begin() + k, A.end());
            out.push_back(A[0]);
            // B clockwise from a_0 is lb[i0 - s]; its rest (s > k) reversed
            for (int s = Lb - 1; s > k; --s) out.push_back(lb[((i0 - s) % Lb + Lb) % Lb]);
            la = out;
            size[pr.first] += size[pr.second];
            comps.erase(pr.second);
            size.erase(pr.second);
        }
        rounds->push_back(rnd);
    }
    if (mode == PGCP_SPHERE) {
        std::vector<int> ids;
        for (auto& kv : comps) ids.push_back(kv.first);
        std::sort(ids.begin(), ids.end());
        int st;
        if (shared_arc(comps[ids[0]], comps[ids[1]], &st) != -2)
            return Error{PGCP_E_WELD, "last two components do not close the sphere"};
        rounds->push_back({{ids[0], ids[1]}});
    }
    return Error{PGCP_OK, ""};
}

// ---------------------------------------------------------------- driver

Error weld_all(pgcp_part* P, const double* bdy_uv, double* welded_uv) {
    try {
        const int K = P->K;
        std::unordered_map<int, Component> comps;
        for (int i = 0; i < K; ++i) {
            Component C;
            for (int e = P->loop_ptr[i]; e < P->loop_ptr[i + 1]; ++e) {
                C.outer.push_back(P->loop_gv[e]);
                C.zo.push_back(EP{cplx(bdy_uv[2 * e], bdy_uv[2 * e + 1]), false});
            }
            comps[i] = std::move(C);
        }
        const size_t nr = P->weld_rounds.size();
        for (size_t r = 0; r < nr; ++r) {
            const bool closed = P->mode == PGCP_SPHERE && r + 1 == nr;
            const auto& rnd = P->weld_rounds[r];
            std::vector<Component> merged(rnd.size());
            // pairs of one round are independent
            std::vector<Error> errs(rnd.size(), Error{PGCP_OK, ""});
#pragma omp parallel for schedule(dynamic) if (rnd.size() > 1)
            for (size_t t = 0; t < rnd.size(); ++t) {
                try {
                    merged[t] = weld_pair(comps[rnd[t].first], comps[rnd[t].second], closed);
                } catch (const Error& e) {
                    errs[t] = e;
                }
            }
            for (auto& e : errs)
                if (e.code != PGCP_OK) return e;
            for (size_t t = 0; t < rnd.size(); ++t) {
                comps[rnd[t].first] = std::move(merged[t]);
                comps.erase(rnd[t].second);
            }
        }
        if (comps.size() != 1) return Error{PGCP_E_WELD, "weld plan did not finish"};
        Component& C = comps.begin()->second;
        if (P->mode == PGCP_DISK) disk_step(C);

        // scatter to seam order
        std::vector<char> seen(P->n_seam, 0);
        auto put = [&](int gv, const EP& p) {
            auto it = std::lower_bound(P->seam_gv.begin(), P->seam_gv.end(), gv);
            int64_t s = it - P->seam_gv.begin();
            if (s >= P->n_seam || *it != gv) return;
            const double inf = std::numeric_limits<double>::infinity();
            welded_uv[2 * s] = p.inf ? inf : p.z.real();
            welded_uv[2 * s + 1] = p.inf ? inf : p.z.imag();
            seen[s] = 1;
        };
        for (size_t s = 0; s < C.outer.size(); ++s) put(C.outer[s], C.zo[s]);
        for (size_t s = 0; s < C.tracked.size(); ++s) put(C.tracked[s], C.zt[s]);
        for (int64_t s = 0; s < P->n_seam; ++s)
            if (!seen[s]) return Error{PGCP_E_WELD, "seam vertex without a welded coordinate"};

        P->welded = true;
        return Error{PGCP_OK, ""};
    } catch (const Error& e) {
        return e;
    } catch (const std::exception& e) {
        return Error{PGCP_E_WELD, e.what()};
    }
}

}  // namespace pgcp

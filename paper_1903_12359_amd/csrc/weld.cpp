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
#include "weld_maps.h"

namespace pgcp {
namespace {

using namespace weldmaps;

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

namespace {

// shared_arc with a dense position table: pos[v] is -1 for every vertex on entry
// and again on return.
int shared_arc_pos(const std::vector<int>& la, const std::vector<int>& lb, std::vector<int>& pos, int* start) {
    const int La = (int)la.size(), Lb = (int)lb.size();
    for (int i = 0; i < Lb; ++i) pos[lb[i]] = i;
    auto done = [&](int r) {
        for (int i = 0; i < Lb; ++i) pos[lb[i]] = -1;
        return r;
    };
    std::vector<char> in(La, 0);
    int m = 0;
    for (int i = 0; i < La; ++i)
        if (pos[la[i]] >= 0) {
            in[i] = 1;
            m++;
        }
    if (m < 3) return done(-1);
    if (m == La && m == Lb) return done(-2);
    if (m == La) return done(-1);
    int runs = 0, s0 = -1;
    for (int i = 0; i < La; ++i)
        if (in[i] && !in[(i + La - 1) % La]) {
            runs++;
            s0 = i;
        }
    if (runs != 1) return done(-1);
    const int k = m - 1;
    for (int s = 0; s < k; ++s) {
        const int pa = pos[la[(s0 + s) % La]], pb = pos[la[(s0 + s + 1) % La]];
        if (((pa - pb) % Lb + Lb) % Lb != 1) return done(-1);
    }
    *start = s0;
    return done(k);
}

}  // namespace

Error merge_plan(const std::vector<std::vector<int>>& loops, const std::vector<int64_t>& sizes,
                 int mode, std::vector<std::vector<std::pair<int, int>>>* rounds) {
    int maxv = 0;
    for (const auto& l : loops)
        for (int v : l) maxv = std::max(maxv, v);
    std::vector<int> pos(maxv + 1, -1);
    std::unordered_map<int, std::vector<int>> comps;   // id -> outer loop
    std::unordered_map<int, int64_t> size;
    for (size_t i = 0; i < loops.size(); ++i) {
        comps[(int)i] = loops[i];
        size[(int)i] = sizes[i];
    }
    const size_t target = mode == PGCP_SPHERE ? 2 : 1;
    while (comps.size() > target) {
        // candidate pairs from shared vertices: (vertex, component) sorted by vertex
        std::vector<std::pair<int, int>> vo;
        for (auto& kv : comps)
            for (int v : kv.second) vo.emplace_back(v, kv.first);
        std::sort(vo.begin(), vo.end());
        std::vector<std::pair<int, int>> pairs;
        for (size_t a = 0; a < vo.size();) {
            size_t b = a;
            while (b < vo.size() && vo[b].first == vo[a].first) b++;
            for (size_t x = a; x < b; ++x)
                for (size_t y = x + 1; y < b; ++y)
                    pairs.emplace_back(std::min(vo[x].second, vo[y].second), std::max(vo[x].second, vo[y].second));
            a = b;
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
            int k = shared_arc_pos(comps[pr.first], comps[pr.second], pos, &st);
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
            int k = shared_arc_pos(la, lb, pos, &st);
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

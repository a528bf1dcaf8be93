// Host plan builder: surface partition (Section 4.1) and everything the
// batched device solves need (piece vertex lists, SELL-64 structure of the
// cotangent Laplacian with the opposite vertices of every entry, boundary
// loops, DNCP pins, seam list) plus the weld merge tree.
//
// Pieces are the connected components of the face graph whose edges are the
// interior edges with equal labels on both sides (an edge between different
// labels is a cut edge).  They are numbered by their smallest face index and
// each must be a topological disk.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>

#include "pgcp_internal.h"

namespace pgcp {
namespace {

struct UnionFind {
    std::vector<int32_t> parent;
    explicit UnionFind(int64_t n) : parent(n) { std::iota(parent.begin(), parent.end(), 0); }
    int32_t find(int32_t x) {
        while (parent[x] != x) {
            parent[x] = parent[parent[x]];
            x = parent[x];
        }
        return x;
    }
    void unite(int32_t a, int32_t b) {
        a = find(a);
        b = find(b);
        if (a == b) return;
        if (a < b) std::swap(a, b);
        parent[a] = b;   // root = smaller index
    }
};

Error topo(const std::string& m) { return Error{PGCP_E_TOPOLOGY, m}; }

// Reverse Cuthill-McKee order of a piece's vertices (local indices, adjacency
// in CSR): from a pseudo-peripheral vertex (the end of a second breadth-first
// sweep), breadth-first with neighbours by increasing degree (ties by index),
// reversed.  Rows in this order give each workgroup's contiguous range of rows
// a compact patch of the mesh, hence a small halo (a k-means piece of a sphere
// in global vertex order scatters a workgroup's rows over the whole piece).
void rcm_order(int32_t n, const std::vector<int32_t>& ptr, const std::vector<int32_t>& adj,
               std::vector<int32_t>& order) {
    order.clear();
    order.reserve(n);
    std::vector<int32_t> stamp(n, -1), q, nb;
    std::vector<char> done(n, 0);
    q.reserve(n);
    int32_t sweep = 0;
    auto deg = [&](int32_t v) { return ptr[v + 1] - ptr[v]; };
    auto bfs = [&](int32_t s) -> size_t {   // plain sweep over unplaced vertices; start of its last level
        q.clear();
        q.push_back(s);
        stamp[s] = ++sweep;
        size_t head = 0, last = 0;
        while (head < q.size()) {
            const size_t end = q.size();
            last = head;
            for (; head < end; ++head) {
                const int32_t v = q[head];
                for (int32_t t = ptr[v]; t < ptr[v + 1]; ++t) {
                    const int32_t u = adj[t];
                    if (!done[u] && stamp[u] != sweep) {
                        stamp[u] = sweep;
                        q.push_back(u);
                    }
                }
            }
        }
        return last;
    };
    auto pick = [&](size_t from) {   // smallest degree, then index, among q[from..]
        int32_t best = q[from];
        for (size_t t = from; t < q.size(); ++t) {
            const int32_t v = q[t];
            if (deg(v) < deg(best) || (deg(v) == deg(best) && v < best)) best = v;
        }
        return best;
    };
    for (int32_t s0 = 0; s0 < n; ++s0) {
        if (done[s0]) continue;
        int32_t s = pick(bfs(s0));
        s = pick(bfs(s));
        const size_t first = order.size();
        order.push_back(s);
        done[s] = 1;
        for (size_t h = first; h < order.size(); ++h) {
            const int32_t v = order[h];
            nb.clear();
            for (int32_t t = ptr[v]; t < ptr[v + 1]; ++t)
                if (!done[adj[t]]) nb.push_back(adj[t]);
            std::sort(nb.begin(), nb.end(),
                      [&](int32_t a, int32_t b) { return deg(a) != deg(b) ? deg(a) < deg(b) : a < b; });
            for (int32_t u : nb)
                if (!done[u]) {
                    done[u] = 1;
                    order.push_back(u);
                }
        }
        std::reverse(order.begin() + (int64_t)first, order.end());
    }
}

}  // namespace

Error build_plan(pgcp_part* P, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                 const int32_t* label, int mode) {
    const char* vb = getenv("PGCP_VERBOSE");
    const bool verbose = vb && vb[0] == '1';
    auto t_last = std::chrono::steady_clock::now();
    auto lap = [&](const char* what) {
        if (!verbose) return;
        auto t = std::chrono::steady_clock::now();
        fprintf(stderr, "[pgcp] partition %-12s %8.2f ms\n", what,
                std::chrono::duration<double, std::milli>(t - t_last).count());
        t_last = t;
    };
    if (nv <= 0 || nf <= 0 || nv > INT32_MAX / 2 || nf > INT32_MAX / 4)
        return Error{PGCP_E_INVALID, "mesh size out of range"};
    if (mode < 0 || mode > 2) return Error{PGCP_E_INVALID, "bad mode"};
    P->nv = nv;
    P->nf = nf;
    P->mode = mode;
    for (int64_t f = 0; f < nf; ++f) {
        int32_t a = F[3 * f], b = F[3 * f + 1], c = F[3 * f + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv)
            return Error{PGCP_E_INVALID, "face index out of range"};
        if (a == b || b == c || a == c) return topo("face with a repeated vertex");
    }

    // ---- half-edge twins: outgoing half-edges of every vertex (CSR by source),
    // then the twin of a->b is the b->a entry in b's list.
    const int64_t nh = 3 * nf;
    auto he_b = [&](int64_t h) { return F[(h / 3) * 3 + (h % 3 + 1) % 3]; };
    // (the order inside a vertex's list is not fixed; only membership is used)
    std::vector<int64_t> cnt(nv + 1, 0);
#pragma omp parallel for schedule(static)
    for (int64_t h = 0; h < nh; ++h) __atomic_fetch_add(&cnt[F[h] + 1], (int64_t)1, __ATOMIC_RELAXED);
    for (int64_t v = 0; v < nv; ++v) cnt[v + 1] += cnt[v];
    bigvec<int32_t> out_h(nh), out_b(nh);   // half-edge and its target, grouped by source
    {
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
#pragma omp parallel for schedule(static)
        for (int64_t h = 0; h < nh; ++h) {
            const int64_t q = __atomic_fetch_add(&fill[F[h]], (int64_t)1, __ATOMIC_RELAXED);
            out_h[q] = (int32_t)h;
            out_b[q] = he_b(h);
        }
    }
    bigvec<int32_t> twin(nh);
    int bad_nm = 0, bad_or = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad_nm, bad_or)
    for (int64_t h = 0; h < nh; ++h) {
        const int32_t a = F[h], b = he_b(h);
        int found = 0;
        int32_t t = -1;
        for (int64_t q = cnt[b]; q < cnt[b + 1]; ++q)
            if (out_b[q] == a) {
                found++;
                t = out_h[q];
            }
        int same = 0;
        for (int64_t q = cnt[a]; q < cnt[a + 1]; ++q)
            if (out_b[q] == b) same++;
        if (same > 1) bad_or++;              // two half-edges a->b: faces disagree on orientation
        if (found > 1 || found + same > 2) bad_nm++;
        twin[h] = found == 1 ? t : -1;
    }
    if (bad_or) return topo("inconsistently oriented faces");
    if (bad_nm) return topo("non-manifold edge (more than two faces)");
    lap("twins");
    // ---- pieces: components of the face graph over uncut interior edges
    UnionFind uf(nf);
    for (int64_t h = 0; h < nh; ++h) {
        int32_t t = twin[h];
        if (t < 0 || t < h) continue;
        int32_t f0 = (int32_t)(h / 3), f1 = t / 3;
        if (label[f0] == label[f1]) uf.unite(f0, f1);
    }
    P->face_sub.assign(nf, -1);
    std::vector<int32_t> root_id(nf, -1);
    int K = 0;
    for (int64_t f = 0; f < nf; ++f) {
        int32_t r = uf.find((int32_t)f);
        if (root_id[r] < 0) root_id[r] = K++;
        P->face_sub[f] = root_id[r];
    }
    P->K = K;

    // faces of each piece, ascending
    std::vector<int64_t> fptr(K + 1, 0);
    for (int64_t f = 0; f < nf; ++f) fptr[P->face_sub[f] + 1]++;
    for (int i = 0; i < K; ++i) fptr[i + 1] += fptr[i];
    std::vector<int32_t> faces(nf);
    {
        std::vector<int64_t> fill(fptr.begin(), fptr.end() - 1);
        for (int64_t f = 0; f < nf; ++f) faces[fill[P->face_sub[f]]++] = (int32_t)f;
    }
    P->sub_nf.resize(K);
    for (int i = 0; i < K; ++i) P->sub_nf[i] = (int32_t)(fptr[i + 1] - fptr[i]);

    // vertices of each piece, in reverse Cuthill-McKee order (ties and
    // starting sweeps by ascending global index), packed rows padded to 64
    std::vector<std::vector<int32_t>> verts(K);
    Error err{PGCP_OK, ""};
#pragma omp parallel
    {
        // a thread's vertex stamps (the piece + 1 that last collected it) and
        // global -> local map
        std::vector<int32_t> seen(nv, 0), loc(nv);
        std::vector<int32_t> ptr, adj, fill, order;
#pragma omp for schedule(dynamic)
        for (int i = 0; i < K; ++i) {
            auto& vv = verts[i];
            vv.reserve(fptr[i + 1] - fptr[i]);
            for (int64_t t = fptr[i]; t < fptr[i + 1]; ++t)
                for (int c = 0; c < 3; ++c) {
                    const int32_t g = F[3 * (int64_t)faces[t] + c];
                    if (seen[g] != i + 1) {
                        seen[g] = i + 1;
                        vv.push_back(g);
                    }
                }
            std::sort(vv.begin(), vv.end());
            const int32_t n = (int32_t)vv.size();
            for (int32_t l = 0; l < n; ++l) loc[vv[l]] = l;
            // the piece's vertex graph (each face side once per direction), CSR
            ptr.assign(n + 1, 0);
            for (int64_t t = fptr[i]; t < fptr[i + 1]; ++t)
                for (int c = 0; c < 3; ++c) ptr[loc[F[3 * (int64_t)faces[t] + c]] + 1] += 2;
            for (int32_t l = 0; l < n; ++l) ptr[l + 1] += ptr[l];
            adj.resize(ptr[n]);
            fill.assign(ptr.begin(), ptr.end() - 1);
            for (int64_t t = fptr[i]; t < fptr[i + 1]; ++t) {
                const int64_t f = faces[t];
                for (int c = 0; c < 3; ++c) {
                    const int32_t a = loc[F[3 * f + c]], b = loc[F[3 * f + (c + 1) % 3]];
                    adj[fill[a]++] = b;
                    adj[fill[b]++] = a;
                }
            }
            // sort and drop repeated neighbours in place, then compact
            int32_t w = 0;
            for (int32_t l = 0; l < n; ++l) {
                const int32_t b0 = ptr[l], b1 = ptr[l + 1];
                std::sort(adj.begin() + b0, adj.begin() + b1);
                const int32_t start = w;
                for (int32_t t = b0; t < b1; ++t)
                    if (t == b0 || adj[t] != adj[t - 1]) adj[w++] = adj[t];
                ptr[l] = start;
            }
            ptr[n] = w;
            rcm_order(n, ptr, adj, order);
            std::vector<int32_t> ordered(n);
            for (int32_t l = 0; l < n; ++l) ordered[l] = vv[order[l]];
            vv.swap(ordered);
        }
    }
    P->sub_nv.resize(K);
    P->row0.assign(K + 1, 0);
    for (int i = 0; i < K; ++i) {
        P->sub_nv[i] = (int32_t)verts[i].size();
        int64_t padded = (verts[i].size() + 63) / 64 * 64;
        // the batched CG reaches a piece's vectors through 32-bit byte offsets (16 bytes a row)
        if (padded > (int64_t(1) << 27))
            return Error{PGCP_E_INVALID, "a piece has more than 134,217,728 vertices"};
        if ((int64_t)P->row0[i] + padded > INT32_MAX) return Error{PGCP_E_INVALID, "too many rows"};
        P->row0[i + 1] = P->row0[i] + (int32_t)padded;
    }
    const int64_t N = P->row0[K];
    P->N = N;
    P->nslices = N / 64;
    P->row_gv.assign(N, -1);
    P->row_prev.assign(N, -1);
    P->row_next.assign(N, -1);
    P->row_kind.assign(N, 2);
    P->slice_sub.resize(P->nslices);
    for (int i = 0; i < K; ++i) {
        for (size_t l = 0; l < verts[i].size(); ++l) {
            P->row_gv[P->row0[i] + l] = verts[i][l];
            P->row_kind[P->row0[i] + l] = 0;
        }
        for (int64_t s = P->row0[i] / 64; s < P->row0[i + 1] / 64; ++s) P->slice_sub[s] = i;
    }

    lap("pieces");
    // corner -> packed row (a thread's global-vertex -> row map, refilled per piece)
    bigvec<int32_t> corner_row(nh);
#pragma omp parallel
    {
        bigvec<int32_t> row_of(nv);
#pragma omp for schedule(dynamic)
        for (int i = 0; i < K; ++i) {
            const auto& vv = verts[i];
            for (size_t l = 0; l < vv.size(); ++l) row_of[vv[l]] = P->row0[i] + (int32_t)l;
            for (int64_t t = fptr[i]; t < fptr[i + 1]; ++t) {
                const int64_t f = faces[t];
                for (int c = 0; c < 3; ++c) corner_row[3 * f + c] = row_of[F[3 * f + c]];
            }
        }
    }

    lap("rows");
    // ---- boundary loops, Euler characteristic, pins
    std::vector<std::vector<int32_t>> loops(K);   // packed rows, CCW
    std::vector<std::string> emsg(K);
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < K; ++i) {
        int32_t r0 = P->row0[i];
        int32_t n = (int32_t)verts[i].size();
        std::vector<int32_t> nxt(n, -1);
        int64_t nb = 0;
        for (int64_t t = fptr[i]; t < fptr[i + 1]; ++t) {
            int64_t f = faces[t];
            for (int c = 0; c < 3; ++c) {
                int64_t h = 3 * f + c;
                int32_t tw = twin[h];
                if (tw >= 0 && P->face_sub[tw / 3] == i) continue;
                int32_t a = corner_row[h] - r0, b = corner_row[3 * f + (c + 1) % 3] - r0;
                if (nxt[a] >= 0) {
                    emsg[i] = "piece " + std::to_string(i) + ": pinched boundary vertex";
                    break;
                }
                nxt[a] = b;
                nb++;
            }
            if (!emsg[i].empty()) break;
        }
        if (!emsg[i].empty()) continue;
        if (nb == 0) {
            emsg[i] = "piece " + std::to_string(i) + " has no boundary";
            continue;
        }
        int32_t start = -1;   // the boundary vertex of smallest global index
        for (int32_t l = 0; l < n; ++l)
            if (nxt[l] >= 0 && (start < 0 || verts[i][l] < verts[i][start])) start = l;
        std::vector<int32_t>& L = loops[i];
        int32_t v = start;
        do {
            L.push_back(v + r0);
            v = nxt[v];
        } while (v != start && (int64_t)L.size() <= nb);
        if ((int64_t)L.size() != nb) {
            emsg[i] = "piece " + std::to_string(i) + ": more than one boundary loop";
            continue;
        }
        int64_t nfi = fptr[i + 1] - fptr[i];
        if ((3 * nfi + nb) % 2 != 0 || (int64_t)n - (3 * nfi + nb) / 2 + nfi != 1) {
            emsg[i] = "piece " + std::to_string(i) + ": Euler characteristic is not 1";
            continue;
        }
    }
    for (int i = 0; i < K; ++i)
        if (!emsg[i].empty()) return topo(emsg[i]);

    P->loop_ptr.assign(K + 1, 0);
    for (int i = 0; i < K; ++i) P->loop_ptr[i + 1] = P->loop_ptr[i] + (int32_t)loops[i].size();
    P->n_bdy = P->loop_ptr[K];
    P->loop_row.resize(P->n_bdy);
    P->loop_gv.resize(P->n_bdy);
    P->pin_row.resize(2 * K);
    P->pin_x1.resize(K);
    for (int i = 0; i < K; ++i) {
        const auto& L = loops[i];
        int32_t nb = (int32_t)L.size();
        for (int32_t e = 0; e < nb; ++e) {
            int32_t r = L[e];
            P->loop_row[P->loop_ptr[i] + e] = r;
            P->loop_gv[P->loop_ptr[i] + e] = P->row_gv[r];
            P->row_kind[r] = 1;
            P->row_next[r] = L[(e + 1) % nb];
            P->row_prev[r] = L[(e + nb - 1) % nb];
        }
        // pins: p0 = smallest global index (loop start), p1 = farthest from p0 in R^3
        const double* x0 = V + 3 * (int64_t)P->row_gv[L[0]];
        double best = -1.0;
        int32_t p1 = L[0];
        for (int32_t e = 0; e < nb; ++e) {
            const double* x = V + 3 * (int64_t)P->row_gv[L[e]];
            double dx = x[0] - x0[0], dy = x[1] - x0[1], dz = x[2] - x0[2];
            double d = std::sqrt(dx * dx + dy * dy + dz * dz);
            if (d > best) {
                best = d;
                p1 = L[e];
            }
        }
        if (!(best > 0.0)) return Error{PGCP_E_DEGENERATE, "piece with coincident boundary vertices"};
        P->pin_row[2 * i] = L[0];
        P->pin_row[2 * i + 1] = p1;
        P->pin_x1[i] = best;
    }

    // seam vertices (ascending) and the seam index of each loop entry
    P->seam_gv = P->loop_gv;
    std::sort(P->seam_gv.begin(), P->seam_gv.end());
    P->seam_gv.erase(std::unique(P->seam_gv.begin(), P->seam_gv.end()), P->seam_gv.end());
    P->n_seam = (int64_t)P->seam_gv.size();
    P->loop_seam.resize(P->n_bdy);
    for (int64_t e = 0; e < P->n_bdy; ++e)
        P->loop_seam[e] = (int32_t)(std::lower_bound(P->seam_gv.begin(), P->seam_gv.end(),
                                                     P->loop_gv[e]) - P->seam_gv.begin());

    lap("loops");
    // ---- off-diagonal structure with opposite vertices, per row
    // each corner (k of face (i,j,k)) contributes entries i->j and j->i with
    // opposite vertex k.
    std::vector<int32_t> deg_raw(N, 0);
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < K; ++i)
        for (int64_t t = fptr[i]; t < fptr[i + 1]; ++t)
            for (int c = 0; c < 3; ++c) deg_raw[corner_row[3 * (int64_t)faces[t] + c]] += 2;
    std::vector<int64_t> rptr(N + 1, 0);
    for (int64_t r = 0; r < N; ++r) rptr[r + 1] = rptr[r] + deg_raw[r];
    bigvec<int32_t> ent_col(rptr[N]), ent_opp(rptr[N]);
    bigvec<uint8_t> ent_fwd(rptr[N]);   // 1: (row, column, opposite) is the face's own cyclic order
    {
        std::vector<int64_t> fill(rptr.begin(), rptr.end() - 1);
        // rows of different pieces are disjoint: fill piece by piece in parallel
#pragma omp parallel for schedule(dynamic)
        for (int i = 0; i < K; ++i) {
            for (int64_t t = fptr[i]; t < fptr[i + 1]; ++t) {
                const int64_t f = faces[t];
                for (int c = 0; c < 3; ++c) {
                    int32_t ri = corner_row[3 * f + (c + 1) % 3];
                    int32_t rj = corner_row[3 * f + (c + 2) % 3];
                    int32_t gk = F[3 * f + c];
                    ent_col[fill[ri]] = rj;
                    ent_fwd[fill[ri]] = 1;
                    ent_opp[fill[ri]++] = gk;
                    ent_col[fill[rj]] = ri;
                    ent_fwd[fill[rj]] = 0;
                    ent_opp[fill[rj]++] = gk;
                }
            }
        }
    }
    // merge duplicates: unique columns ascending, up to two opposite vertices
    std::vector<int32_t> deg(N, 0);
    bigvec<int32_t> u_col(rptr[N]), u_o1(rptr[N]), u_o2(rptr[N]);
    bigvec<uint8_t> u_ori(rptr[N]);
    std::vector<std::string> derr(1);
    bool bad_edge = false;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < N; ++r) {
        int64_t s = rptr[r], e = rptr[r + 1];
        // insertion sort by (col, opp): rows are short
        for (int64_t a = s + 1; a < e; ++a) {
            int32_t c = ent_col[a], o = ent_opp[a];
            uint8_t fw = ent_fwd[a];
            int64_t b = a - 1;
            while (b >= s && (ent_col[b] > c || (ent_col[b] == c && ent_opp[b] > o))) {
                ent_col[b + 1] = ent_col[b];
                ent_opp[b + 1] = ent_opp[b];
                ent_fwd[b + 1] = ent_fwd[b];
                b--;
            }
            ent_col[b + 1] = c;
            ent_opp[b + 1] = o;
            ent_fwd[b + 1] = fw;
        }
        int32_t d = 0;
        for (int64_t a = s; a < e;) {
            int64_t b = a;
            while (b < e && ent_col[b] == ent_col[a]) b++;
            if (b - a > 2) bad_edge = true;
            u_col[s + d] = ent_col[a];
            u_o1[s + d] = ent_opp[a];
            u_o2[s + d] = (b - a == 2) ? ent_opp[a + 1] : -1;
            u_ori[s + d] = (uint8_t)(ent_fwd[a] | ((b - a == 2) ? (ent_fwd[a + 1] << 1) : 0));
            d++;
            a = b;
        }
        deg[r] = d;
    }
    if (bad_edge) return topo("edge with more than two faces inside a piece");

    lap("entries");
    // ---- SELL-64 layout
    P->sl_ptr.assign(P->nslices + 1, 0);
    P->sl_w.assign(P->nslices, 0);
    int64_t nnz = 0;
    for (int64_t s = 0; s < P->nslices; ++s) {
        int32_t w = 0;
        for (int l = 0; l < 64; ++l) w = std::max(w, deg[s * 64 + l]);
        P->sl_w[s] = w;
        P->sl_ptr[s + 1] = P->sl_ptr[s] + (int64_t)w * 64;
        for (int l = 0; l < 64; ++l) nnz += deg[s * 64 + l];
    }
    P->nnz_off = nnz;
    P->sub_nnz.assign(K, 0);
    for (int i = 0; i < K; ++i)
        for (int64_t r = P->row0[i]; r < P->row0[i + 1]; ++r) P->sub_nnz[i] += deg[r];
    P->sell_elems = P->sl_ptr[P->nslices];
    if (P->sell_elems > INT32_MAX) return Error{PGCP_E_INVALID, "too many matrix entries for int32 slot indices"};
    P->sl_col.resize(P->sell_elems);
    P->sl_opp.resize(2 * P->sell_elems);
    P->sl_rev.resize(P->sell_elems);
    P->sl_ori.resize(P->sell_elems);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < P->nslices; ++s) {
        int64_t base = P->sl_ptr[s];
        for (int l = 0; l < 64; ++l) {
            int64_t r = s * 64 + l;
            for (int32_t k = 0; k < P->sl_w[s]; ++k) {
                int64_t el = base + (int64_t)k * 64 + l;
                if (k < deg[r]) {
                    const int32_t c = u_col[rptr[r] + k];
                    P->sl_col[el] = c;
                    P->sl_opp[2 * el] = u_o1[rptr[r] + k];
                    P->sl_opp[2 * el + 1] = u_o2[rptr[r] + k];
                    P->sl_ori[el] = u_ori[rptr[r] + k];
                    // the slot of the reverse entry (c, r): columns of a row are ascending
                    const int32_t* cb = u_col.data() + rptr[c];
                    const int32_t kk = (int32_t)(std::lower_bound(cb, cb + deg[c], (int32_t)r) - cb);
                    P->sl_rev[el] = (int32_t)(P->sl_ptr[c / 64] + (int64_t)kk * 64 + c % 64);
                } else {
                    P->sl_col[el] = (int32_t)r;
                    P->sl_opp[2 * el] = -1;
                    P->sl_opp[2 * el + 1] = -1;
                    P->sl_ori[el] = 0;
                    P->sl_rev[el] = -1;
                }
            }
        }
    }

    lap("sell");
    // ---- weld merge tree (depends on the loops only)
    std::vector<std::vector<int>> gl(K);
    std::vector<int64_t> sizes(K);
    for (int i = 0; i < K; ++i) {
        gl[i].assign(P->loop_gv.begin() + P->loop_ptr[i], P->loop_gv.begin() + P->loop_ptr[i + 1]);
        sizes[i] = P->sub_nf[i];
    }
    P->weld_rounds.clear();
    if (K > 1) {
        Error e = merge_plan(gl, sizes, mode, &P->weld_rounds);
        if (e.code != PGCP_OK) return e;
    } else if (mode == PGCP_SPHERE) {
        return Error{PGCP_E_WELD, "sphere mode needs at least two pieces"};
    }
    lap("merge plan");
    return Error{PGCP_OK, ""};
}

}  // namespace pgcp

// Device part of libpgcp (gfx950): cotangent assembly, batched persistent PCG
// for the DNCP and harmonic systems of every piece at once, FP64 residual /
// iterative refinement, boundary gathers and the distortion check.
//
// Data layout.  The vertices of every piece are packed into consecutive rows
// ("packed rows"), each piece padded to a multiple of 64 rows so that one
// 64-row slice (one wavefront) never straddles two pieces.  The off-diagonal
// part of each piece's cotangent Laplacian is stored in SELL-64: slice s holds
// width w_s columns, element (s, k, lane) at sl_ptr[s] + 64 k + lane, so lane l
// of a wavefront reads row 64 s + l and every load is coalesced.  Padding
// slots point at the row itself with value 0.  The diagonal is a separate
// dense vector.  Both coordinates of a vector are interleaved (float2/double2)
// so one matrix read serves x and y.
//
// Batched persistent PCG.  One cooperative launch covers all pieces.  Each
// workgroup owns a contiguous range of slices of exactly one piece; the
// workgroups of a piece meet at per-piece barriers (a monotonically increasing
// arrival counter).  Each writes its partial dot products to a small global
// array; the workgroup that arrives last sums them in a fixed order and
// publishes the sums, so every workgroup of a piece takes the same alpha, beta
// and convergence decision and results are bitwise deterministic.  Per
// iteration there are two barriers:
//   A: beta; p_new = z + beta p_old (own rows, written to the other p buffer);
//      q = A p_new computed by gathering z and p_old of neighbour rows (so
//      p_new need not be visible yet); partial p.q
//   B: alpha; e += alpha p; r -= alpha q; z = D^-1 r, or z = M r with the
//      learned SPAI (neighbours' new r rebuilt from their published old r and
//      q); partial r.z and r.r
// q and p_new stay in registers between the phases.  Every wait is bounded:
// a workgroup that spins too long raises a global abort flag and all
// workgroups leave their loops.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <fstream>
#include <limits>
#include <map>
#include <mutex>
#include <queue>
#include <set>
#include <sstream>
#include <string>
#include <vector>


// Streaming kernel: four waves per SIMD (at most 128 VGPRs), with its slot
// batches of PGCP_STREAM_KB entries sized to fit without spills; measured on
// the 2048^2 / 256-piece DNCP solve, 5% faster than three waves with batches of 8.
#ifndef PGCP_STREAM_WPE
#define PGCP_STREAM_WPE 4
#endif

#include "device_util.h"
#include "pgcp_internal.h"

namespace pgcp {

static void free_workmap(WorkMap& W) {
    for (DevBuf* b : {&W.d_wg_sub, &W.d_wg_rank, &W.d_wg_s0, &W.d_wg_s1, &W.d_sub_pbase, &W.d_sub_nwg, &W.d_wg_h0,
                      &W.d_halo, &W.d_lcol, &W.d_lpn, &W.d_wg_n1, &W.d_rcol, &W.d_expo})
        dev_free(*b);
}

void free_part_device(pgcp_part* P) {
    DevBuf* all[] = {&P->d_row_gv, &P->d_row_prev, &P->d_row_next, &P->d_row_kind, &P->d_slice_sub,
                     &P->d_sl_ptr, &P->d_sl_w, &P->d_sl_col, &P->d_sl_opp, &P->d_sl_rev, &P->d_val64, &P->d_val32,
                     &P->d_diag64, &P->d_diag32, &P->d_pin_row, &P->d_pin_x1, &P->d_loop_ptr,
                     &P->d_loop_row, &P->d_loop_seam, &P->d_seam_gv, &P->d_mask_dncp, &P->d_mask_harm,
                     &P->d_chart, &P->d_u64, &P->d_r64, &P->d_e, &P->d_r, &P->d_z, &P->d_p0, &P->d_p1, &P->d_q, &P->d_r2, &P->d_s1,
                     &P->d_partial, &P->d_bar, &P->d_gen, &P->d_res, &P->d_subinfo, &P->d_bnorm, &P->d_rnorm, &P->d_iters,
                     &P->d_cgs,
                     &P->d_flags, &P->d_row0, &P->d_slicepart,
                     &P->d_scale, &P->d_target, &P->d_active, &P->d_status, &P->d_rrout,
                     &P->d_abort, &P->d_distpart, &P->d_diststat, &P->d_absd, &P->d_sorttmp, &P->d_sl_ori,
                     &P->d_lbs_val64, &P->d_lbs_val32, &P->d_lbs_diag64, &P->d_lbs_diag32, &P->d_face_sub,
                     &P->d_fold_cnt, &P->d_fold_prev};
    for (DevBuf* b : all) dev_free(*b);
    free_workmap(P->wmap32);
    free_workmap(P->wmap64);
    if (P->ev0) (void)hipEventDestroy(P->ev0);
    if (P->ev1) (void)hipEventDestroy(P->ev1);
    P->ev0 = P->ev1 = nullptr;
    lpc_free_part(P);
}

Error upload_plan(pgcp_ctx* ctx, pgcp_part* P) {
    hipStream_t s = ctx->stream;
    Error e{PGCP_OK, ""};
#define UP(buf, vec)                      \
    e = upload(buf, vec, s);              \
    if (e.code != PGCP_OK) return e;
    UP(P->d_row_gv, P->row_gv);
    UP(P->d_row_prev, P->row_prev);
    UP(P->d_row_next, P->row_next);
    UP(P->d_row_kind, P->row_kind);
    UP(P->d_slice_sub, P->slice_sub);
    UP(P->d_sl_ptr, P->sl_ptr);
    UP(P->d_sl_w, P->sl_w);
    UP(P->d_sl_col, P->sl_col);
    UP(P->d_sl_opp, P->sl_opp);
    UP(P->d_sl_rev, P->sl_rev);
    UP(P->d_pin_row, P->pin_row);
    UP(P->d_pin_x1, P->pin_x1);
    UP(P->d_loop_ptr, P->loop_ptr);
    UP(P->d_loop_row, P->loop_row);
    UP(P->d_loop_seam, P->loop_seam);
    UP(P->d_seam_gv, P->seam_gv);
    UP(P->d_row0, P->row0);
    std::vector<uint8_t> md(P->N), mh(P->N);
    for (int64_t r = 0; r < P->N; ++r) {
        md[r] = P->row_kind[r] == 2 ? 1 : 0;
        mh[r] = P->row_kind[r] != 0 ? 1 : 0;
    }
    for (int i = 0; i < P->K; ++i) {
        md[P->pin_row[2 * i]] = 1;
        md[P->pin_row[2 * i + 1]] = 1;
    }
    UP(P->d_mask_dncp, md);
    UP(P->d_mask_harm, mh);
#undef UP
    const size_t N = (size_t)P->N, E = (size_t)P->sell_elems;
    if ((e = dev_alloc(P->d_val64, E * 8)).code) return e;
    if ((e = dev_alloc(P->d_val32, E * 4)).code) return e;
    if ((e = dev_alloc(P->d_diag64, N * 8)).code) return e;
    if ((e = dev_alloc(P->d_diag32, N * 4)).code) return e;
    if ((e = dev_alloc(P->d_u64, N * 16)).code) return e;
    if ((e = dev_alloc(P->d_r64, N * 16)).code) return e;
    if ((e = dev_alloc(P->d_e, N * 16)).code) return e;
    if ((e = dev_alloc(P->d_r, N * 16)).code) return e;
    if ((e = dev_alloc(P->d_z, N * 16)).code) return e;
    if ((e = dev_alloc(P->d_p0, N * 16)).code) return e;
    if ((e = dev_alloc(P->d_p1, N * 16)).code) return e;
    if ((e = dev_alloc(P->d_q, N * 16)).code) return e;
    if ((e = dev_alloc(P->d_r2, N * 16)).code) return e;
    if ((e = dev_alloc(P->d_s1, N * 16)).code) return e;
    const size_t K = (size_t)P->K;
    if ((e = dev_alloc(P->d_rnorm, K * 2 * 8)).code) return e;
    if ((e = dev_alloc(P->d_scale, K * 2 * 8)).code) return e;
    if ((e = dev_alloc(P->d_target, K * 2 * 8)).code) return e;
    if ((e = dev_alloc(P->d_rrout, K * 2 * 8)).code) return e;
    if ((e = dev_alloc(P->d_iters, K * 4)).code) return e;
    if ((e = dev_alloc(P->d_cgs, (size_t)K * 16 * 8)).code) return e;
    if ((e = dev_alloc(P->d_status, K * 4)).code) return e;
    if ((e = dev_alloc(P->d_active, K * 4)).code) return e;
    if ((e = dev_alloc(P->d_bar, K * 4)).code) return e;
    if ((e = dev_alloc(P->d_gen, K * 4)).code) return e;
    if ((e = dev_alloc(P->d_res, K * 8 * 8)).code) return e;
    if ((e = dev_alloc(P->d_abort, 64)).code) return e;
    if ((e = dev_alloc(P->d_flags, 64)).code) return e;
    if ((e = dev_alloc(P->d_chart, K * 3 * 8)).code) return e;
    if ((e = dev_alloc(P->d_slicepart, (size_t)P->nslices * 2 * 8)).code) return e;
    HIPCHK(hipMemsetAsync(P->d_flags.p, 0, 64, s));
    return Error{PGCP_OK, ""};
}

// ----------------------------------------------------------------- assembly

__device__ __forceinline__ double cot_at(const double* __restrict__ V, int a, int b, int k) {
    // cot of the angle at k in triangle (a, b, k): (u.v) / |u x v|, u = v_a - v_k, v = v_b - v_k
    double ux = V[3 * (int64_t)a] - V[3 * (int64_t)k], uy = V[3 * (int64_t)a + 1] - V[3 * (int64_t)k + 1],
           uz = V[3 * (int64_t)a + 2] - V[3 * (int64_t)k + 2];
    double vx = V[3 * (int64_t)b] - V[3 * (int64_t)k], vy = V[3 * (int64_t)b + 1] - V[3 * (int64_t)k + 1],
           vz = V[3 * (int64_t)b + 2] - V[3 * (int64_t)k + 2];
    double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
    double dot = ux * vx + uy * vy + uz * vz;
    return dot / sqrt(cx * cx + cy * cy + cz * cz);
}

// One thread per packed row: every off-diagonal slot of the row gets
// -w_pq = -(cot at opp1 + cot at opp2)/2, the diagonal the sum of w_pq.
// The cotangents of an edge are evaluated with the endpoints in ascending
// global order so that both rows of a symmetric pair compute identical bits.
__global__ void __launch_bounds__(BLOCK) k_assemble(
    int64_t nslices, const int64_t* __restrict__ sl_ptr, const int32_t* __restrict__ sl_w,
    const int32_t* __restrict__ sl_col, const int32_t* __restrict__ sl_opp,
    const int32_t* __restrict__ row_gv, const double* __restrict__ V, double* __restrict__ val64,
    float* __restrict__ val32, double* __restrict__ diag64, float* __restrict__ diag32,
    int* __restrict__ bad) {
    int64_t row = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    int64_t s = row >> 6;
    if (s >= nslices) return;
    int lane = (int)(row & 63);
    int g = row_gv[row];
    int64_t base = sl_ptr[s] + lane;
    int w = sl_w[s];
    double dsum = 0.0;
    for (int k = 0; k < w; ++k) {
        int64_t el = base + (int64_t)k * 64;
        int o1 = sl_opp[2 * el], o2 = sl_opp[2 * el + 1];
        double wv = 0.0;
        if (o1 >= 0 && g >= 0) {
            int h = row_gv[sl_col[el]];
            int a = min(g, h), b = max(g, h);
            double c1 = cot_at(V, a, b, o1);
            double c2 = (o2 >= 0) ? cot_at(V, a, b, o2) : 0.0;
            if (!isfinite(c1) || !isfinite(c2)) atomicExch(bad, 1);
            wv = 0.5 * (c1 + c2);
        }
        val64[el] = -wv;
        val32[el] = (float)(-wv);
        dsum += wv;
    }
    diag64[row] = dsum;
    diag32[row] = (float)dsum;
}

// ----------------------------------------------------------------- FP64 residual

// r = -(A u) on free rows, 0 on Dirichlet rows; per-slice partial |r|^2 (x, y).
__global__ void __launch_bounds__(BLOCK) k_residual64(
    int64_t nslices, const int64_t* __restrict__ sl_ptr, const int32_t* __restrict__ sl_w,
    const int32_t* __restrict__ sl_col, const double* __restrict__ val, const double* __restrict__ diag,
    const int32_t* __restrict__ rprev, const int32_t* __restrict__ rnext, int coupled,
    const uint8_t* __restrict__ mask, const double2* __restrict__ u, double2* __restrict__ r,
    double* __restrict__ slice_part) {
    int64_t row = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    int64_t s = row >> 6;
    if (s >= nslices) return;
    int lane = (int)(row & 63);
    double2 ur = u[row];
    double ax = diag[row] * ur.x, ay = diag[row] * ur.y;
    int64_t base = sl_ptr[s] + lane;
    int w = sl_w[s];
    for (int k = 0; k < w; ++k) {
        int64_t el = base + (int64_t)k * 64;
        double v = val[el];
        double2 uc = u[sl_col[el]];
        ax += v * uc.x;
        ay += v * uc.y;
    }
    if (coupled) {
        int pv = rprev[row], nx = rnext[row];
        if (pv >= 0) {
            double2 un = u[nx], up = u[pv];
            ax -= 0.5 * (un.y - up.y);
            ay += 0.5 * (un.x - up.x);
        }
    }
    double2 out;
    if (mask[row]) {
        out.x = 0.0;
        out.y = 0.0;
    } else {
        out.x = -ax;
        out.y = -ay;
    }
    r[row] = out;
    double px = wave_sum(out.x * out.x), py = wave_sum(out.y * out.y);
    if (lane == 0) {
        slice_part[2 * s] = px;
        slice_part[2 * s + 1] = py;
    }
}

// One block per piece: fixed-order sum of its slices' partials.
__global__ void __launch_bounds__(BLOCK) k_piece_sum(const int32_t* __restrict__ row0,
                                                      const double* __restrict__ slice_part,
                                                      double* __restrict__ out) {
    __shared__ double lds[WAVES * 2];
    int i = blockIdx.x;
    int64_t s0 = row0[i] / 64, s1 = row0[i + 1] / 64;
    double v[2] = {0.0, 0.0};
    for (int64_t s = s0 + threadIdx.x; s < s1; s += BLOCK) {
        v[0] += slice_part[2 * s];
        v[1] += slice_part[2 * s + 1];
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        out[2 * i] = v[0];
        out[2 * i + 1] = v[1];
    }
}

// r_T = r64 / scale (per piece and coordinate), e = 0.
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_prep_inner(int64_t N, const int32_t* __restrict__ slice_sub,
                                                       const double2* __restrict__ r64,
                                                       const double* __restrict__ scale,
                                                       typename Vec2<T>::type* __restrict__ r,
                                                       typename Vec2<T>::type* __restrict__ e) {
    int64_t row = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (row >= N) return;
    int i = slice_sub[row >> 6];
    double sx = scale[2 * i], sy = scale[2 * i + 1];
    double2 v = r64[row];
    typename Vec2<T>::type o, zero;
    o.x = (T)(sx > 0.0 ? v.x / sx : 0.0);
    o.y = (T)(sy > 0.0 ? v.y / sy : 0.0);
    zero.x = (T)0;
    zero.y = (T)0;
    r[row] = o;
    e[row] = zero;
}

// u += scale * e on active pieces.
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_apply_inner(int64_t N, const int32_t* __restrict__ slice_sub,
                                                        const int32_t* __restrict__ active,
                                                        const double* __restrict__ scale,
                                                        const typename Vec2<T>::type* __restrict__ e,
                                                        double2* __restrict__ u) {
    int64_t row = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (row >= N) return;
    int i = slice_sub[row >> 6];
    if (!active[i]) return;
    typename Vec2<T>::type d = e[row];
    double2 x = u[row];
    x.x += scale[2 * i] * (double)d.x;
    x.y += scale[2 * i + 1] * (double)d.y;
    u[row] = x;
}

// ----------------------------------------------------------------- persistent batched PCG

// Matrix slots of a row read per batch of loads in the SpMVs (triangle-mesh
// valences rarely exceed 8; wider rows take several batches).
constexpr int KB = 8;
#ifndef PGCP_STREAM_KB
#define PGCP_STREAM_KB 6
#endif
constexpr int KBR = 4;   // register-resident kernel: own columns come from LDS, fewer registers to spare

template <typename T>
struct CGArgs {
    const int64_t* sl_ptr;
    const int32_t* sl_w;
    const int32_t* sl_col;
    const T* val;
    const T* diag;
    const int32_t* rprev;
    const int32_t* rnext;
    const uint8_t* mask;
    const int32_t* wg_sub;         // [G] piece of each workgroup, -1 = idle
    const int32_t* wg_rank;        // [G] rank of the workgroup inside its piece
    const int32_t* wg_s0;          // [G] first slice
    const int32_t* wg_s1;          // [G] end slice
    const int32_t* sub_pbase;      // [K] first partial record of the piece
    const int32_t* sub_nwg;        // [K] workgroups of the piece
    const int32_t* row0;           // [K+1] first packed row of each piece
    const int32_t* wg_h0;          // [G+1] register kernel: first halo entry of each workgroup
    const int32_t* halo;           // [*] register kernel: packed rows of the halo entries
    const uint16_t* lcol;          // [sell] register kernel: local column of every SELL slot
    const int32_t* lpn;            // [2N] register kernel: local loop neighbours (prev, next) or -1
    int lds_n;                     // register kernel: LDS entries of one vector (own rows + largest ring 1)
    const int32_t* wg_n1;          // [G] register kernels: ring-1 entries of each workgroup's halo
    const uint16_t* rcol;          // [halo * KR] single-reduction kernel: local columns of ring-1 rows
    const uint8_t* expo;           // [N] bit 0: row in some ring 1, bit 1: in some ring 2
    typename Vec2<T>::type* s1;    // single-reduction kernel: sixth published vector buffer
    int lds_nr, lds_nu;            // single-reduction kernel: LDS entries of r and u
    const int32_t* active;         // [K]
    const double* target_rel2;     // [K*2] squared relative tolerance per piece and coordinate
    typename Vec2<T>::type* e;
    typename Vec2<T>::type* r;
    typename Vec2<T>::type* z;
    typename Vec2<T>::type* pa;
    typename Vec2<T>::type* pb;
    typename Vec2<T>::type* q;     // A p (streaming kernel: all rows; SPAI: published halo rows)
    typename Vec2<T>::type* r2;    // second residual buffer (SPAI: r alternates between r and r2)
    const float* mval;             // learned SPAI off-diagonal values (SELL layout, FP32 in every
    const float* mdiag;            //   precision: a preconditioner needs no more), or null; diagonal
    const int32_t* pc;             // [K] 1 = the piece uses the SPAI, 0 = Jacobi (null: all Jacobi)
    double* partial;               // [sum nwg][8]
    unsigned* bar;                 // [K]
    unsigned* gen;                 // [K] reductions published by the last arriving workgroup
    double* res;                   // [K][8] their values
    int* abort_flag;
    int32_t* iters;                // [K] out
    double* rr_out;                // [K*2] out: final recursive |r|^2 / |r0|^2
    int32_t* status;               // [K] out: 0 ok, 1 breakdown, 2 max_iter, 3 abort, 4 stagnation,
                                   //   5 paused at pause_at (streaming kernel; state in cgs)
    double* cgs;                   // [K][16] streaming kernel: scalar state of a paused piece
    int pause_at;                  // streaming kernel: pause every piece when its iteration count reaches this
    int resume;                    // streaming kernel: continue paused pieces from cgs and the vectors
    int coupled;
    int max_iter;
    int n_xcd;                     // workgroup g runs on XCD g % n_xcd (round-robin dispatch)
    int stall;                     // stop after this many iterations without a 10% residual gain
};

// Fixed-order block sum of NV values per thread; result returned to every
// thread.  The per-wave sums go to one of two LDS banks that alternate from
// call to call (par), so one barrier per call suffices: a bank is written
// again only two calls later, after every thread has passed the barrier of
// the call in between and so has finished reading it.
template <int BLK, int NV>
__device__ __forceinline__ void bsum(double (&v)[NV], double* lds, int& par) {
    constexpr int NW = BLK / 64;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double* bank = lds + par * (NW * 8);
    par ^= 1;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) bank[wave * NV + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int w = 0; w < NW; ++w) s += bank[w * NV + i];
        v[i] = s;
    }
}

// Cross-workgroup data (the z and p vectors that neighbours gather, and the
// partial dot products) is published and read with relaxed agent-scope atomic
// stores and loads, which are coherent across the whole device; everything a
// workgroup only reads itself (matrix, diagonal, e, r) uses plain accesses.
__device__ __forceinline__ float2 ld_c(const float2* p) {
    uint64_t u = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    float2 r;
    __builtin_memcpy(&r, &u, 8);
    return r;
}
__device__ __forceinline__ double2 ld_c(const double2* p) {
    const uint64_t* q = reinterpret_cast<const uint64_t*>(p);
    uint64_t a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double2 r;
    __builtin_memcpy(&r.x, &a, 8);
    __builtin_memcpy(&r.y, &b, 8);
    return r;
}
__device__ __forceinline__ void st_c(float2* p, float2 v) {
    uint64_t u;
    __builtin_memcpy(&u, &v, 8);
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_c(double2* p, double2 v) {
    uint64_t a, b;
    __builtin_memcpy(&a, &v.x, 8);
    __builtin_memcpy(&b, &v.y, 8);
    uint64_t* q = reinterpret_cast<uint64_t*>(p);
    __hip_atomic_store(q, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_c(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_c(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One piece's rows [row0, row0 + n) of a vector that other workgroups gather
// or publish within a launch (streaming kernel).  A buffer resource over the
// piece lets a row's pair (16 bytes in FP64, 8 in FP32) move in one
// vector-memory instruction with the agent-scope coherence bit (sc1), the same
// cache policy as the atomics above: an FP64 pair through ld_c / st_c takes two
// 8-byte instructions, each of which fetches or writes through every line the
// wave touches, so the pair costs its bytes twice.  Offsets are 32-bit byte
// counts (pieces hold at most 2^27 rows); an access outside the piece reads 0
// and a store there is dropped.
constexpr int kBufWord3 = 0x00020000;   // raw 32-bit elements, no format conversion
constexpr int kCpolSC1 = 16;            // cache policy: sc1 (coherent at agent scope)

template <typename V2>
struct PieceVec {
    __amdgpu_buffer_rsrc_t rs;
    __device__ __forceinline__ PieceVec(const V2* v, int64_t row0, int64_t n)
        : rs(__builtin_amdgcn_make_buffer_rsrc(const_cast<V2*>(v) + row0, 0, (int)(n * (int64_t)sizeof(V2)),
                                               kBufWord3)) {}
    __device__ __forceinline__ V2 ld(int lrow) const {
        V2 r;
        if constexpr (sizeof(V2) == 16) {
            const auto u = __builtin_amdgcn_raw_buffer_load_b128(rs, lrow * 16, 0, kCpolSC1);
            __builtin_memcpy(&r, &u, 16);
        } else {
            const auto u = __builtin_amdgcn_raw_buffer_load_b64(rs, lrow * 8, 0, kCpolSC1);
            __builtin_memcpy(&r, &u, 8);
        }
        return r;
    }
    __device__ __forceinline__ void st(int lrow, V2 v) const {
        if constexpr (sizeof(V2) == 16) {
            __attribute__((ext_vector_type(4))) unsigned u;
            __builtin_memcpy(&u, &v, 16);
            __builtin_amdgcn_raw_buffer_store_b128(u, rs, lrow * 16, 0, kCpolSC1);
        } else {
            __attribute__((ext_vector_type(2))) unsigned u;
            __builtin_memcpy(&u, &v, 8);
            __builtin_amdgcn_raw_buffer_store_b64(u, rs, lrow * 8, 0, kCpolSC1);
        }
    }
};

// Slot offsets and widths of a wave's slices s, s + nw, s + 2 nw, ... (the
// streaming kernel's walk): lane l holds those of the wave's (j0 + l)-th
// slice, so one load serves 64 slices and a slice reads its own from a lane.
struct SliceMeta {
    int lo = 0, hi = 0, w = 0;
    __device__ __forceinline__ void load(const int64_t* sl_ptr, const int32_t* sl_w, int s, int nw, int s1,
                                         int lane) {
        const int sl = s + lane * nw;
        int64_t b = 0;
        int ww = 0;
        if (sl < s1) {
            b = sl_ptr[sl];
            ww = sl_w[sl];
        }
        lo = (int)b;
        hi = (int)(b >> 32);
        w = ww;
        // wait for them here, once per block: a wait at their first read
        // inside the slice loop would run every slice (and wait for that
        // slice's stores too)
        __asm__ volatile("" ::"v"(lo), "v"(hi), "v"(w));
    }
    __device__ __forceinline__ int64_t base(int jj) const {
        return ((int64_t)__builtin_amdgcn_readlane(hi, jj) << 32) | (uint32_t)__builtin_amdgcn_readlane(lo, jj);
    }
    __device__ __forceinline__ int width(int jj) const { return __builtin_amdgcn_readlane(w, jj); }
};

// A buffer resource over one slice's slots of a SELL array (w slots of 64
// lanes): slot t of lane l is at byte (64 t + l) sizeof(E), a slot past the
// width reads 0.
template <typename E>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slice_rsrc(const E* arr, int64_t sbase, int w) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<E*>(arr) + sbase, 0, w * 64 * (int)sizeof(E), kBufWord3);
}
template <typename E>
__device__ __forceinline__ E slot_ld(__amdgpu_buffer_rsrc_t rs, int lane, int t) {
    if constexpr (sizeof(E) == 8) {
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(rs, lane * 8, t * 512, 0);
        E v;
        __builtin_memcpy(&v, &u, 8);
        return v;
    } else {
        const auto u = __builtin_amdgcn_raw_buffer_load_b32(rs, lane * 4, t * 256, 0);
        E v;
        __builtin_memcpy(&v, &u, 4);
        return v;
    }
}

// Fixed-order sum of the piece's partial records (slots off .. off+NV-1).
template <int BLK, int NV>
__device__ __forceinline__ void piece_sum(const double* partial, int pbase, int nwg, int off, double (&out)[NV],
                                          double* lds, int& par) {
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = 0.0;
    for (int w = threadIdx.x; w < nwg; w += BLK) {
        const double* p = partial + 8 * (int64_t)(pbase + w) + off;
#pragma unroll
        for (int i = 0; i < NV; ++i) out[i] += ld_c(p + i);
    }
    bsum<BLK, NV>(out, lds, par);
}

// z = M r for one row with the learned SPAI (M has the Laplacian's pattern):
// own-workgroup columns from LDS (register kernel) or all from the coherent path.
// Columns outside [lo, hi) take r from rglob, or, when qglob is given, rebuild
// this iteration's residual there as rglob - alpha qglob from the previous
// residual and A p that the owning workgroup published before the barrier, so
// the SPAI needs no barrier of its own.
template <typename T, typename V2, int NB = KB>
__device__ __forceinline__ V2 spai_row(const CGArgs<T>& a, int64_t rw, V2 rown, const V2* lds_r, int64_t lo,
                                       int64_t hi, const V2* rglob, const V2* qglob = nullptr, T ax = (T)0,
                                       T ay = (T)0) {
    const int64_t s = rw >> 6;
    const int64_t base = a.sl_ptr[s] + (rw & 63);
    const int w = a.sl_w[s];
    const T d = (T)a.mdiag[rw];
    T zx = d * rown.x, zy = d * rown.y;
    for (int k0 = 0; k0 < w; k0 += NB) {
        int cc[NB];
        T mm[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int64_t el = base + (int64_t)(k0 + t) * 64;
            const bool in = k0 + t < w;
            mm[t] = in ? (T)a.mval[el] : (T)0;
            cc[t] = in ? a.sl_col[el] : (int)rw;
        }
        V2 rr[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int c = cc[t];
            if (mm[t] == (T)0) {
                rr[t].x = (T)0;
                rr[t].y = (T)0;
            } else if (c >= lo && c < hi) {
                rr[t] = lds_r[c - lo];
            } else {
                rr[t] = ld_c(rglob + c);
                if (qglob) {
                    const V2 qc = ld_c(qglob + c);
                    rr[t].x -= ax * qc.x;
                    rr[t].y -= ay * qc.y;
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            zx += mm[t] * rr[t].x;
            zy += mm[t] * rr[t].y;
        }
    }
    V2 z;
    z.x = zx;
    z.y = zy;
    return z;
}

// z = M r for one row of the streaming kernel (slice s, uniform across the
// wave): the row's SPAI values and columns, then every column's r through the
// piece's coherent vector R, NB slots per batch (slots past the width, or
// whose value is 0, read the own row or a masked one and add nothing).  Six
// slots cover a grid mesh's rows in one batch and keep the FP64 kernel within
// its 128 registers with no scratch (a persistent grid must not need scratch:
// the hardware may run fewer scratch-using waves at once than the grid holds,
// and the missing workgroups would never reach the barriers).
template <typename T, typename V2, int NB = 6>
__device__ __forceinline__ V2 spai_row_stream(const CGArgs<T>& a, int64_t rw, int s, V2 rown, int prow0,
                                              const PieceVec<V2>& R) {
    const int64_t base = a.sl_ptr[s] + (rw & 63);
    const int w = a.sl_w[s];
    const T d = (T)a.mdiag[rw];
    T zx = d * rown.x, zy = d * rown.y;
    for (int k0 = 0; k0 < w; k0 += NB) {
        int cc[NB];
        float mf[NB];   // widened where used, not next to each guarded load
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int64_t el = base + (int64_t)(k0 + t) * 64;
            const bool in = k0 + t < w;
            mf[t] = in ? a.mval[el] : 0.0f;
            cc[t] = in ? a.sl_col[el] : (int)rw;
        }
        V2 rr[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) rr[t] = R.ld(cc[t] - prow0);
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            zx += (T)mf[t] * rr[t].x;
            zy += (T)mf[t] * rr[t].y;
        }
    }
    V2 z;
    z.x = zx;
    z.y = zy;
    return z;
}

// Thread 0 of a workgroup waits until the piece's generation reaches nb.  The
// wait is bounded: past SPIN_MAX polls it raises the abort flag (and every
// other waiter sees it and leaves); the first workgroup to give up records
// where: the barrier it waited at, its piece's workgroups, the arrivals and
// the generation it saw last, its own index.  Returns 1 on abort.
__device__ __forceinline__ int gen_wait(const unsigned* bar, const unsigned* gen, unsigned nb, int nwg,
                                        int* abort_flag) {
    long long spins = 0;
    while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < nb) {
        ++spins;
        if ((spins & 255) == 0) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return 1;
            if (spins > SPIN_MAX) {
                if (__hip_atomic_fetch_add(abort_flag + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                    abort_flag[2] = (int)nb;
                    abort_flag[3] = nwg;
                    abort_flag[4] = (int)__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    abort_flag[5] = (int)__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    abort_flag[6] = (int)blockIdx.x;
                }
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return 1;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return 0;
}

// Barrier of a piece's workgroups fused with the fixed-order sum of their
// partial records: the workgroup that arrives last (it sees the counter at
// target - 1, so every other workgroup's stores have completed) sums the
// records, publishes the sums and bumps the piece's generation; the others wait
// for the generation and read the sums.  One workgroup reads the nwg records
// instead of every workgroup reading all of them.  Returns true on abort.
template <int BLK, int NV>
__device__ __forceinline__ bool piece_reduce(unsigned* bar, unsigned* gen, unsigned nb, int nwg,
                                             const double* partial, int pbase, int off, double* res,
                                             double (&out)[NV], int* abort_flag, int* lds_flag, double* lds,
                                             int& par) {
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned old = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        lds_flag[1] = (old == nb * (unsigned)nwg - 1u) ? 1 : 0;
    }
    __syncthreads();
    if (lds_flag[1]) {
        piece_sum<BLK, NV>(partial, pbase, nwg, off, out, lds, par);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) st_c(res + off + i, out[i]);
            __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __hip_atomic_store(gen, nb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return false;
    }
    if (threadIdx.x == 0) lds_flag[0] = gen_wait(bar, gen, nb, nwg, abort_flag);
    __syncthreads();
    if (lds_flag[0]) return true;
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = ld_c(res + off + i);
    return false;
}

// Barrier of a piece's workgroups without sums: the last to arrive bumps the
// generation, the others wait for it.  Returns true on abort.
template <int BLK>
__device__ __forceinline__ bool piece_barrier(unsigned* bar, unsigned* gen, unsigned nb, int nwg, int* abort_flag,
                                              int* lds_flag) {
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned old = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == nb * (unsigned)nwg - 1u) {
            __hip_atomic_store(gen, nb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            lds_flag[0] = 0;
        } else {
            lds_flag[0] = gen_wait(bar, gen, nb, nwg, abort_flag);
        }
    }
    __syncthreads();
    return lds_flag[0] != 0;
}

// Register-resident batched PCG with LDS-staged vectors.  Thread t of a
// workgroup owns the rows (s0 + wave + NW j) * 64 + lane, j < R, for the whole
// solve: r and z of its rows live in registers, e and p_old in LDS.  The
// workgroup numbers its rows locally (own rows 0 .. nown-1, then the distinct
// columns of other workgroups that its rows reference, the "halo"), and every
// SELL slot carries its local column (lcol), so both sparse products read all
// their operands from LDS.  Each product is preceded by one cooperative fill
// of the halo (every thread loads its entries at once): p_new = z + beta p_old
// (SpMV) or this iteration's residual r_old - alpha q (SPAI), rebuilt from
// values the owning workgroups published before the last barrier.  Only rows
// with a neighbour in another workgroup publish.

// y_j = d_j x_j + sum_k v_jk x[lcol_jk] for the thread's R rows, operands in
// LDS.  The first KS slots of RB rows are loaded together, without branches
// (slots past a row's width are clamped to its last slot and masked), so that
// one memory round trip serves them; a scheduling barrier between row groups
// keeps the compiler from hoisting every group's loads at once (which would
// spill registers).  Wider rows loop over the rest.
constexpr int KS = 6;
constexpr int RB = 2;
constexpr int KR = 8;   // slots per ring-1 row the single-reduction kernel applies M with

template <typename TV, typename T, typename V2, int R>
__device__ __forceinline__ void lds_spmv(const uint16_t* __restrict__ lcol, const TV* __restrict__ val,
                                         const TV* __restrict__ diag, const int32_t (&rv)[R],
                                         const int32_t (&base)[R], const int (&w)[R], const V2 (&x)[R],
                                         const V2* lv, V2 (&y)[R]) {
    // the slot loads do not depend on the iteration; an opaque zero keeps the
    // compiler from hoisting them out of the CG loop into registers for good
    int32_t opq = 0;
    __asm__ volatile("" : "+v"(opq));
#pragma unroll
    for (int j0 = 0; j0 < R; j0 += RB) {
        __builtin_amdgcn_sched_barrier(0);
        constexpr int G = RB < R ? RB : R;
        int lc[G][KS];
        TV vv[G][KS], dd[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int j = j0 + g < R ? j0 + g : R - 1;
            dd[g] = diag[rv[j]];
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                const int32_t el = base[j] + opq + min(t, w[j] - 1) * 64;
                lc[g][t] = lcol[el];
                vv[g][t] = val[el];
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int j = j0 + g;
            if (j >= R) break;
            T yx = (T)dd[g] * x[j].x, yy = (T)dd[g] * x[j].y;
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                const V2 c = lv[lc[g][t]];
                const T v = t < w[j] ? (T)vv[g][t] : (T)0;
                yx += v * c.x;
                yy += v * c.y;
            }
            for (int t = KS; t < w[j]; ++t) {
                const int32_t el = base[j] + t * 64;
                const V2 c = lv[lcol[el]];
                const T v = (T)val[el];
                yx += v * c.x;
                yy += v * c.y;
            }
            y[j].x = yx;
            y[j].y = yy;
        }
    }
}

// 256-thread workgroups are asked to fit two per CU (two waves per SIMD): the
// register budget that lets a 1024-row workgroup shape hold C2-sized batches
// in one cooperative grid.
template <int BLK>
constexpr int pcg_waves_per_eu() { return BLK == 256 ? 2 : BLK / 256; }

template <typename T, int BLK, int R>
__global__ void __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(pcg_waves_per_eu<BLK>())))
k_pcg(CGArgs<T> a) {
    using V2 = typename Vec2<T>::type;
    constexpr int NW = BLK / 64;
    extern __shared__ unsigned char smem_raw[];
    V2* lv = reinterpret_cast<V2*>(smem_raw);   // [lds_n] p: own rows, then the halo
    V2* lrs = lv + a.lds_n;                     // [lds_n] SPAI operand r: own rows, then the halo
    // e of the own rows: in LDS up to 1024 rows per workgroup; larger shapes
    // keep it in memory (plain accesses, each thread its own rows) so that two
    // workgroups still share a CU's LDS
    constexpr bool ELDS = BLK * R <= 1024;
    V2* le = lv + 2 * (int64_t)a.lds_n;         // [BLK R] (ELDS only)
    __shared__ double lds[2 * NW * 8];
    int bpar = 0;   // LDS bank of the next block sum
    __shared__ int lds_flag[2];
    const int wg = blockIdx.x;
    const int sub = a.wg_sub[wg];
    if (sub < 0 || !a.active[sub]) return;
    const int s0 = a.wg_s0[wg], s1 = a.wg_s1[wg];
    const int rank = a.wg_rank[wg];
    const int pbase = a.sub_pbase[sub], nwg = a.sub_nwg[sub];
    const bool leader = rank == 0 && threadIdx.x == 0;
    const bool spai = a.pc != nullptr && a.pc[sub] != 0;
    // the wave index is uniform: slice numbers, widths and offsets stay in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t lo = (int64_t)s0 * 64;
    const int nown = (s1 - s0) * 64;
    const int hb = a.wg_h0[wg], nh = a.wg_n1[wg];   // ring 1 only
    V2* lh = lv + nown;
    V2* lrh = lrs + nown;
    unsigned* bar = a.bar + sub;
    unsigned nbar = 0;
    double* mypart = a.partial + 8 * (int64_t)(pbase + rank);

    int32_t rows[R], rv[R], base[R];   // row, a row safe to load (rows past the range: slice s0), slots
    int w[R], lp[R], ln[R];
    bool valid[R], msk[R], expo[R];
    V2 r[R], z[R];   // e and p_old of the own rows live in LDS
    T dinv[R];
    V2 zero;
    zero.x = (T)0;
    zero.y = (T)0;
    // the thread's first two halo entries stay in registers (row lo when absent)
    const bool h0ok = threadIdx.x < nh, h1ok = threadIdx.x + BLK < nh;
    const int hc0 = h0ok ? a.halo[hb + threadIdx.x] : (int)lo;
    const int hc1 = h1ok ? a.halo[hb + threadIdx.x + BLK] : (int)lo;

    // ---- start: registers, export flags, z = D^-1 r or M r, p_old = 0
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int s = s0 + wave + NW * j;
        valid[j] = s < s1;
        const int sv = valid[j] ? s : s0;   // rows past the range read a valid slice, results discarded
        rows[j] = s * 64 + lane;
        rv[j] = sv * 64 + lane;
        base[j] = (int32_t)a.sl_ptr[sv] + lane;
        w[j] = a.sl_w[sv];
        r[j] = zero;
        z[j] = zero;
        dinv[j] = (T)0;
        msk[j] = true;
        expo[j] = false;
        lp[j] = -1;
        ln[j] = -1;
        if (!valid[j]) continue;
        const int32_t rw = rows[j];
        lv[rw - lo] = zero;
        if constexpr (ELDS) le[rw - lo] = zero;
        else a.e[rw] = zero;
        msk[j] = a.mask[rw] != 0;
        if (!msk[j]) {
            dinv[j] = (T)1 / a.diag[rw];
            r[j] = a.r[rw];
            if (!spai) {
                z[j].x = dinv[j] * r[j].x;
                z[j].y = dinv[j] * r[j].y;
            }
        }
        bool ex = false;
        for (int k = 0; k < w[j]; ++k) ex |= a.lcol[base[j] + (int64_t)k * 64] >= nown;
        if (a.coupled) {
            lp[j] = a.lpn[2 * rw];
            ln[j] = a.lpn[2 * rw + 1];
            ex |= lp[j] >= nown || ln[j] >= nown;
        }
        expo[j] = ex;
    }
    if (spai) {
        // z = M r on the input residual (written by the previous kernel)
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (valid[j]) lrs[rows[j] - lo] = r[j];
        {
            const V2 v0 = a.r[hc0], v1 = a.r[hc1];
            if (h0ok) lrh[threadIdx.x] = v0;
            if (h1ok) lrh[threadIdx.x + BLK] = v1;
            for (int h = threadIdx.x + 2 * BLK; h < nh; h += BLK) lrh[h] = a.r[a.halo[hb + h]];
        }
        __syncthreads();
        V2 mz[R];
        lds_spmv<float, T, V2, R>(a.lcol, a.mval, a.mdiag, rv, base, w, r, lrs, mz);
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (valid[j] && !msk[j]) z[j] = mz[j];
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (!valid[j]) continue;
        if (expo[j]) {
            st_c(a.z + rows[j], z[j]);
            st_c(a.pa + rows[j], zero);
        }
        acc[0] += (double)r[j].x * (double)z[j].x;
        acc[1] += (double)r[j].y * (double)z[j].y;
        acc[2] += (double)r[j].x * (double)r[j].x;
        acc[3] += (double)r[j].y * (double)r[j].y;
    }
    bsum<BLK, 4>(acc, lds, bpar);
    if (threadIdx.x == 0) {
        for (int i = 0; i < 4; ++i) st_c(mypart + 2 + i, acc[i]);
    }
    nbar++;
    double st[4];
    if (piece_reduce<BLK, 4>(bar, a.gen + sub, nbar, nwg, a.partial, pbase, 2, a.res + 8 * (int64_t)sub, st,
                             a.abort_flag, lds_flag, lds, bpar)) {
        if (leader) a.status[sub] = 3;
        return;
    }
    double rz[2] = {st[0], st[1]};
    double rr0[2] = {st[2], st[3]};
    if (a.coupled) {
        rz[0] = rz[1] = st[0] + st[1];
        rr0[0] = rr0[1] = st[2] + st[3];
    }
    const double tgt[2] = {a.target_rel2[2 * sub] * rr0[0], a.target_rel2[2 * sub + 1] * rr0[1]};
    bool done[2] = {rr0[0] <= tgt[0] || !(rz[0] > 0.0), rr0[1] <= tgt[1] || !(rz[1] > 0.0)};
    double rrc[2] = {rr0[0], rr0[1]};
    double beta[2] = {0.0, 0.0};
    double best = (done[0] ? 0.0 : 1.0) + (done[1] ? 0.0 : 1.0);
    int it_best = 0;
    int it = 0;
    int stat = 0;
    V2* pold = a.pa;
    V2* pnew = a.pb;
    V2* rcur = a.r;    // residual of the previous iteration as published (SPAI halo)
    V2* rnext = a.r2;

    while (!(done[0] && done[1])) {
        if (it >= a.max_iter) {
            stat = 2;
            break;
        }
        // ---- phase A: p_new = z + beta p_old (registers, LDS, publish); halo
        // p_new rebuilt from the published z and p_old; q = A p_new; p.q
        const T bx = done[0] ? (T)0 : (T)beta[0], by = done[1] ? (T)0 : (T)beta[1];
        V2 pn[R], q[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const V2 po = valid[j] ? lv[rows[j] - lo] : zero;
            V2 p;
            p.x = done[0] ? (T)0 : z[j].x + bx * po.x;
            p.y = done[1] ? (T)0 : z[j].y + by * po.y;
            pn[j] = p;
            if (valid[j]) {
                lv[rows[j] - lo] = p;
                if (expo[j]) st_c(pnew + rows[j], p);
            }
        }
        {
            const V2 z0 = ld_c(a.z + hc0), o0 = ld_c(pold + hc0);
            const V2 z1 = ld_c(a.z + hc1), o1 = ld_c(pold + hc1);
            V2 v0, v1;
            v0.x = done[0] ? (T)0 : z0.x + bx * o0.x;
            v0.y = done[1] ? (T)0 : z0.y + by * o0.y;
            v1.x = done[0] ? (T)0 : z1.x + bx * o1.x;
            v1.y = done[1] ? (T)0 : z1.y + by * o1.y;
            if (h0ok) lh[threadIdx.x] = v0;
            if (h1ok) lh[threadIdx.x + BLK] = v1;
            for (int h = threadIdx.x + 2 * BLK; h < nh; h += BLK) {
                const int c = a.halo[hb + h];
                const V2 zc = ld_c(a.z + c), oc = ld_c(pold + c);
                V2 v;
                v.x = done[0] ? (T)0 : zc.x + bx * oc.x;
                v.y = done[1] ? (T)0 : zc.y + by * oc.y;
                lh[h] = v;
            }
        }
        __syncthreads();
        lds_spmv<T, T, V2, R>(a.lcol, a.val, a.diag, rv, base, w, pn, lv, q);
        double pq[2] = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (!valid[j] || msk[j]) {
                // a Dirichlet row's A p is zero; neighbours rebuild its residual from it
                q[j] = zero;
                if (spai && valid[j] && expo[j]) st_c(a.q + rows[j], zero);
                continue;
            }
            if (a.coupled && lp[j] >= 0) {
                // (L + L - M/2): the boundary term couples x and y along the loop
                const V2 pN = lv[ln[j]], pP = lv[lp[j]];
                q[j].x -= (T)0.5 * (pN.y - pP.y);
                q[j].y += (T)0.5 * (pN.x - pP.x);
            }
            if (spai && expo[j]) st_c(a.q + rows[j], q[j]);
            pq[0] += (double)pn[j].x * (double)q[j].x;
            pq[1] += (double)pn[j].y * (double)q[j].y;
        }
        bsum<BLK, 2>(pq, lds, bpar);
        if (threadIdx.x == 0) {
            st_c(mypart + 0, pq[0]);
            st_c(mypart + 1, pq[1]);
        }
        nbar++;
        double pqs[2];
        if (piece_reduce<BLK, 2>(bar, a.gen + sub, nbar, nwg, a.partial, pbase, 0, a.res + 8 * (int64_t)sub, pqs,
                                 a.abort_flag, lds_flag, lds, bpar)) {
            stat = 3;
            break;
        }
        double alpha[2] = {0.0, 0.0};
        if (a.coupled) {
            double den = pqs[0] + pqs[1];
            if (!(den > 0.0) || !isfinite(den)) {
                stat = 1;
                break;
            }
            alpha[0] = alpha[1] = rz[0] / den;
        } else {
            for (int c = 0; c < 2; ++c) {
                if (done[c]) continue;
                if (!(pqs[c] > 0.0) || !isfinite(pqs[c])) {
                    stat = 1;
                    break;
                }
                alpha[c] = rz[c] / pqs[c];
            }
            if (stat) break;
        }
        // ---- phase B: e += alpha p; r -= alpha q; z = D^-1 r (Jacobi) or M r
        // (learned SPAI, halo residual rebuilt as r_old - alpha q); r.z, r.r
        const T ax = (T)alpha[0], ay = (T)alpha[1];
        double acc2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (!valid[j] || msk[j]) continue;
            const V2 p = lv[rows[j] - lo];
            V2 ev = ELDS ? le[rows[j] - lo] : a.e[rows[j]];
            ev.x += ax * p.x;
            ev.y += ay * p.y;
            if constexpr (ELDS) le[rows[j] - lo] = ev;
            else a.e[rows[j]] = ev;
            r[j].x -= ax * q[j].x;
            r[j].y -= ay * q[j].y;
            if (spai) continue;
            z[j].x = dinv[j] * r[j].x;
            z[j].y = dinv[j] * r[j].y;
            if (expo[j]) st_c(a.z + rows[j], z[j]);
            acc2[0] += (double)r[j].x * (double)z[j].x;
            acc2[1] += (double)r[j].y * (double)z[j].y;
            acc2[2] += (double)r[j].x * (double)r[j].x;
            acc2[3] += (double)r[j].y * (double)r[j].y;
        }
        if (spai) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (!valid[j]) continue;
                lrs[rows[j] - lo] = r[j];
                if (expo[j]) st_c(rnext + rows[j], r[j]);
            }
            {
                const V2 r0 = ld_c(rcur + hc0), q0 = ld_c(a.q + hc0);
                const V2 r1 = ld_c(rcur + hc1), q1 = ld_c(a.q + hc1);
                V2 v0, v1;
                v0.x = r0.x - ax * q0.x;
                v0.y = r0.y - ay * q0.y;
                v1.x = r1.x - ax * q1.x;
                v1.y = r1.y - ay * q1.y;
                if (h0ok) lrh[threadIdx.x] = v0;
                if (h1ok) lrh[threadIdx.x + BLK] = v1;
                for (int h = threadIdx.x + 2 * BLK; h < nh; h += BLK) {
                    const int c = a.halo[hb + h];
                    const V2 rc = ld_c(rcur + c), qc = ld_c(a.q + c);
                    V2 v;
                    v.x = rc.x - ax * qc.x;
                    v.y = rc.y - ay * qc.y;
                    lrh[h] = v;
                }
            }
            __syncthreads();
            V2 mz[R];
            lds_spmv<float, T, V2, R>(a.lcol, a.mval, a.mdiag, rv, base, w, r, lrs, mz);
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (!valid[j] || msk[j]) continue;
                z[j] = mz[j];
                if (expo[j]) st_c(a.z + rows[j], z[j]);
                acc2[0] += (double)r[j].x * (double)z[j].x;
                acc2[1] += (double)r[j].y * (double)z[j].y;
                acc2[2] += (double)r[j].x * (double)r[j].x;
                acc2[3] += (double)r[j].y * (double)r[j].y;
            }
        }
        bsum<BLK, 4>(acc2, lds, bpar);
        if (threadIdx.x == 0) {
            for (int i = 0; i < 4; ++i) st_c(mypart + 2 + i, acc2[i]);
        }
        nbar++;
        if (piece_reduce<BLK, 4>(bar, a.gen + sub, nbar, nwg, a.partial, pbase, 2, a.res + 8 * (int64_t)sub, st,
                                 a.abort_flag, lds_flag, lds, bpar)) {
            stat = 3;
            break;
        }
        double rzn[2] = {st[0], st[1]};
        double rrn[2] = {st[2], st[3]};
        if (a.coupled) {
            rzn[0] = rzn[1] = st[0] + st[1];
            rrn[0] = rrn[1] = st[2] + st[3];
        }
        double prog = 0.0;
        for (int c = 0; c < 2; ++c) {
            if (done[c]) continue;
            rrc[c] = rrn[c];
            beta[c] = rzn[c] / rz[c];
            rz[c] = rzn[c];
            if (rrn[c] <= tgt[c] || !(rzn[c] > 0.0)) done[c] = true;
            else prog += rrn[c] / rr0[c];
        }
        if (a.coupled) done[1] = done[0];
        ++it;
        // stagnation: no 10% gain of the relative residual in `stall` iterations
        if (prog < 0.9 * best) {
            best = prog;
            it_best = it;
        } else if (!(done[0] && done[1]) && it - it_best > a.stall) {
            stat = 4;
            break;
        }
        V2* t = pold;
        pold = pnew;
        pnew = t;
        t = rcur;
        rcur = rnext;
        rnext = t;
    }
    // the correction leaves through plain stores (read by the next kernel)
#pragma unroll
    for (int j = 0; j < R; ++j)
        if (ELDS && valid[j]) a.e[rows[j]] = le[rows[j] - lo];
    if (leader) {
        a.iters[sub] = it;
        a.status[sub] = stat;
        a.rr_out[2 * sub] = rr0[0] > 0.0 ? rrc[0] / rr0[0] : 0.0;
        a.rr_out[2 * sub + 1] = rr0[1] > 0.0 ? rrc[1] / rr0[1] : 0.0;
    }
}

// Single-reduction batched PCG (Chronopoulos and Gear's recurrences): one
// per-piece barrier per iteration instead of two.  With u = M r and w = A u,
// the scalars gamma = (r, u), delta = (w, u) and |r|^2 of an iteration are
// reduced together; beta = gamma'/gamma, alpha = gamma' / (delta' - beta
// gamma' / alpha), and p = u + beta p, s = w + beta s (= A p) follow by
// recurrence, so that x += alpha p and r -= alpha s.  The next residual of a
// neighbouring row, r - alpha (w + beta s_prev), is rebuilt from the three
// vectors its owner published before the barrier (double-buffered by
// iteration parity), on ring 1 and, when M is the learned SPAI, on ring 2 too:
// the workgroup applies M on its own rows and on ring 1 itself, so w = A u
// needs no second exchange.  Own rows' w, p, s live in registers; r (own rows
// and rings), u (own rows and ring 1) and e in LDS.  Same work map, local
// numbering, barriers and bounded polls as k_pcg.
template <typename T, int BLK, int R>
__global__ void __launch_bounds__(BLK) k_pcg1(CGArgs<T> a) {
    using V2 = typename Vec2<T>::type;
    constexpr int NW = BLK / 64;
    extern __shared__ unsigned char smem_raw[];
    V2* lr = reinterpret_cast<V2*>(smem_raw);   // [lds_nr] r: own rows, ring 1, ring 2
    V2* lu = lr + a.lds_nr;                     // [lds_nu] u = M r: own rows, ring 1
    V2* le = lu + a.lds_nu;                     // [BLK R] e of the own rows
    __shared__ double lds[2 * NW * 8];
    __shared__ int lds_flag[2];
    int bpar = 0;
    const int wg = blockIdx.x;
    const int sub = a.wg_sub[wg];
    if (sub < 0 || !a.active[sub]) return;
    const int s0 = a.wg_s0[wg], s1 = a.wg_s1[wg];
    const int rank = a.wg_rank[wg];
    const int pbase = a.sub_pbase[sub], nwg = a.sub_nwg[sub];
    const bool leader = rank == 0 && threadIdx.x == 0;
    const bool spai = a.pc != nullptr && a.pc[sub] != 0;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t lo = (int64_t)s0 * 64;
    const int nown = (s1 - s0) * 64;
    const int hb = a.wg_h0[wg], nh = a.wg_h0[wg + 1] - hb, n1 = a.wg_n1[wg];
    const int nfill = spai ? nh : n1;               // ring entries whose residual the products need
    const uint8_t pubmask = spai ? 3 : 1;           // rows in some ring 1 (and ring 2) publish
    unsigned* bar = a.bar + sub;
    unsigned nbar = 0;
    double* mypart = a.partial + 8 * (int64_t)(pbase + rank);

    int32_t rows[R], rv[R], base[R];
    int w[R], lp[R], ln[R];
    bool valid[R], msk[R], pub[R];
    V2 wv[R], pv[R], sv[R];
    T dinv[R];
    V2 zero;
    zero.x = (T)0;
    zero.y = (T)0;
    // the thread's first two ring entries stay in registers (row lo when absent)
    const bool h0ok = threadIdx.x < nfill, h1ok = threadIdx.x + BLK < nfill;
    const int hc0 = h0ok ? a.halo[hb + threadIdx.x] : (int)lo;
    const int hc1 = h1ok ? a.halo[hb + threadIdx.x + BLK] : (int)lo;

#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int s = s0 + wave + NW * j;
        valid[j] = s < s1;
        const int sv_ = valid[j] ? s : s0;
        rows[j] = s * 64 + lane;
        rv[j] = sv_ * 64 + lane;
        base[j] = (int32_t)a.sl_ptr[sv_] + lane;
        w[j] = a.sl_w[sv_];
        wv[j] = zero;
        pv[j] = zero;
        sv[j] = zero;
        dinv[j] = (T)0;
        msk[j] = true;
        pub[j] = false;
        lp[j] = -1;
        ln[j] = -1;
        if (!valid[j]) continue;
        const int32_t rw = rows[j];
        msk[j] = a.mask[rw] != 0;
        V2 r0 = zero;
        if (!msk[j]) {
            dinv[j] = (T)1 / a.diag[rw];
            r0 = a.r[rw];
        }
        lr[rw - lo] = r0;
        le[rw - lo] = zero;
        pub[j] = (a.expo[rw] & pubmask) != 0;
        if (a.coupled) {
            lp[j] = a.lpn[2 * rw];
            ln[j] = a.lpn[2 * rw + 1];
        }
    }
    {
        // ring residuals of the input (written by the previous kernel)
        const V2 v0 = a.r[hc0], v1 = a.r[hc1];
        if (h0ok) lr[nown + threadIdx.x] = v0;
        if (h1ok) lr[nown + threadIdx.x + BLK] = v1;
        for (int h = threadIdx.x + 2 * BLK; h < nfill; h += BLK) lr[nown + h] = a.r[a.halo[hb + h]];
    }

    // u = M r on the own rows and ring 1
    auto apply_m = [&]() {
        V2 rr[R];
#pragma unroll
        for (int j = 0; j < R; ++j) rr[j] = valid[j] ? lr[rows[j] - lo] : zero;
        if (spai) {
            V2 mz[R];
            lds_spmv<float, T, V2, R>(a.lcol, a.mval, a.mdiag, rv, base, w, rr, lr, mz);
#pragma unroll
            for (int j = 0; j < R; ++j)
                if (valid[j]) lu[rows[j] - lo] = msk[j] ? zero : mz[j];
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j)
                if (valid[j]) {
                    V2 u;
                    u.x = dinv[j] * rr[j].x;
                    u.y = dinv[j] * rr[j].y;
                    lu[rows[j] - lo] = u;
                }
        }
        for (int h = threadIdx.x; h < n1; h += BLK) {
            const int c = h < BLK ? hc0 : (h < 2 * BLK ? hc1 : a.halo[hb + h]);
            const V2 rc = lr[nown + h];
            V2 u = zero;
            if (!a.mask[c]) {
                if (spai) {
                    const int64_t sc = c >> 6;
                    const int wc = a.sl_w[sc];
                    const int64_t bc = a.sl_ptr[sc] + (c & 63);
                    const T md = (T)a.mdiag[c];
                    T ux = md * rc.x, uy = md * rc.y;
#pragma unroll
                    for (int t = 0; t < KR; ++t) {
                        const int tt = min(t, wc - 1);
                        const T m = t < wc ? (T)a.mval[bc + (int64_t)tt * 64] : (T)0;
                        const V2 x = lr[a.rcol[(int64_t)(hb + h) * KR + tt]];
                        ux += m * x.x;
                        uy += m * x.y;
                    }
                    u.x = ux;
                    u.y = uy;
                } else {
                    const T di = (T)1 / a.diag[c];
                    u.x = di * rc.x;
                    u.y = di * rc.y;
                }
            }
            lu[nown + h] = u;
        }
    };
    // w = A u on the own rows
    auto apply_a = [&]() {
        V2 uu[R];
#pragma unroll
        for (int j = 0; j < R; ++j) uu[j] = valid[j] ? lu[rows[j] - lo] : zero;
        lds_spmv<T, T, V2, R>(a.lcol, a.val, a.diag, rv, base, w, uu, lu, wv);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (!valid[j] || msk[j]) {
                wv[j] = zero;
                continue;
            }
            if (a.coupled && lp[j] >= 0) {
                // (L + L - M/2): the boundary term couples x and y along the loop
                const V2 pN = lu[ln[j]], pP = lu[lp[j]];
                wv[j].x -= (T)0.5 * (pN.y - pP.y);
                wv[j].y += (T)0.5 * (pN.x - pP.x);
            }
        }
    };
    // (r, u), (w, u), (r, r) per coordinate; publish r, w and s_prev of the
    // rows other workgroups rebuild, into the buffers of this parity
    auto dots_publish = [&](int parity, double (&acc)[6]) {
        V2* PR = parity ? a.z : a.r2;
        V2* PW = parity ? a.pb : a.pa;
        V2* PS = parity ? a.s1 : a.q;
#pragma unroll
        for (int i = 0; i < 6; ++i) acc[i] = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (!valid[j]) continue;
            const V2 r = lr[rows[j] - lo], u = lu[rows[j] - lo];
            acc[0] += (double)r.x * (double)u.x;
            acc[1] += (double)r.y * (double)u.y;
            acc[2] += (double)wv[j].x * (double)u.x;
            acc[3] += (double)wv[j].y * (double)u.y;
            acc[4] += (double)r.x * (double)r.x;
            acc[5] += (double)r.y * (double)r.y;
            if (pub[j]) {
                st_c(PR + rows[j], r);
                st_c(PW + rows[j], wv[j]);
                st_c(PS + rows[j], sv[j]);
            }
        }
    };

    __syncthreads();
    apply_m();
    __syncthreads();
    apply_a();
    double acc[6];
    dots_publish(0, acc);
    bsum<BLK, 6>(acc, lds, bpar);
    if (threadIdx.x == 0) {
        for (int i = 0; i < 6; ++i) st_c(mypart + i, acc[i]);
    }
    nbar++;
    double st[6];
    if (piece_reduce<BLK, 6>(bar, a.gen + sub, nbar, nwg, a.partial, pbase, 0, a.res + 8 * (int64_t)sub, st,
                             a.abort_flag, lds_flag, lds, bpar)) {
        if (leader) a.status[sub] = 3;
        return;
    }
    double g[2] = {st[0], st[1]}, dl[2] = {st[2], st[3]}, rr0[2] = {st[4], st[5]};
    if (a.coupled) {
        g[0] = g[1] = st[0] + st[1];
        dl[0] = dl[1] = st[2] + st[3];
        rr0[0] = rr0[1] = st[4] + st[5];
    }
    const double tgt[2] = {a.target_rel2[2 * sub] * rr0[0], a.target_rel2[2 * sub + 1] * rr0[1]};
    bool done[2] = {rr0[0] <= tgt[0] || !(g[0] > 0.0), rr0[1] <= tgt[1] || !(g[1] > 0.0)};
    double rrc[2] = {rr0[0], rr0[1]};
    double alpha[2] = {0.0, 0.0}, beta[2] = {0.0, 0.0};
    int stat = 0;
    for (int c = 0; c < 2; ++c) {
        if (done[c]) continue;
        if (!(dl[c] > 0.0) || !isfinite(dl[c])) stat = 1;
        else alpha[c] = g[c] / dl[c];
    }
    double best = (done[0] ? 0.0 : 1.0) + (done[1] ? 0.0 : 1.0);
    int it_best = 0;
    int it = 0;

    while (stat == 0 && !(done[0] && done[1])) {
        if (it >= a.max_iter) {
            stat = 2;
            break;
        }
        const T ax = done[0] ? (T)0 : (T)alpha[0], ay = done[1] ? (T)0 : (T)alpha[1];
        const T bx = done[0] ? (T)0 : (T)beta[0], by = done[1] ? (T)0 : (T)beta[1];
        // own rows: p = u + beta p, s = w + beta s, e += alpha p, r -= alpha s
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (!valid[j] || msk[j]) continue;
            const int32_t l = rows[j] - (int32_t)lo;
            const V2 u = lu[l];
            pv[j].x = u.x + bx * pv[j].x;
            pv[j].y = u.y + by * pv[j].y;
            sv[j].x = wv[j].x + bx * sv[j].x;
            sv[j].y = wv[j].y + by * sv[j].y;
            V2 ev = le[l], rv_ = lr[l];
            ev.x += ax * pv[j].x;
            ev.y += ay * pv[j].y;
            rv_.x -= ax * sv[j].x;
            rv_.y -= ay * sv[j].y;
            le[l] = ev;
            lr[l] = rv_;
        }
        // ring rows: r - alpha (w + beta s_prev) from this iteration's published vectors
        {
            const int par = it & 1;
            const V2* PR = par ? a.z : a.r2;
            const V2* PW = par ? a.pb : a.pa;
            const V2* PS = par ? a.s1 : a.q;
            const V2 r0 = ld_c(PR + hc0), w0 = ld_c(PW + hc0), q0 = ld_c(PS + hc0);
            const V2 r1 = ld_c(PR + hc1), w1 = ld_c(PW + hc1), q1 = ld_c(PS + hc1);
            V2 v0, v1;
            v0.x = r0.x - ax * (w0.x + bx * q0.x);
            v0.y = r0.y - ay * (w0.y + by * q0.y);
            v1.x = r1.x - ax * (w1.x + bx * q1.x);
            v1.y = r1.y - ay * (w1.y + by * q1.y);
            if (h0ok) lr[nown + threadIdx.x] = v0;
            if (h1ok) lr[nown + threadIdx.x + BLK] = v1;
            for (int h = threadIdx.x + 2 * BLK; h < nfill; h += BLK) {
                const int c = a.halo[hb + h];
                const V2 rc = ld_c(PR + c), wc = ld_c(PW + c), qc = ld_c(PS + c);
                V2 v;
                v.x = rc.x - ax * (wc.x + bx * qc.x);
                v.y = rc.y - ay * (wc.y + by * qc.y);
                lr[nown + h] = v;
            }
        }
        __syncthreads();
        apply_m();
        __syncthreads();
        apply_a();
        double acc2[6];
        dots_publish((it + 1) & 1, acc2);
        bsum<BLK, 6>(acc2, lds, bpar);
        if (threadIdx.x == 0) {
            for (int i = 0; i < 6; ++i) st_c(mypart + i, acc2[i]);
        }
        nbar++;
        if (piece_reduce<BLK, 6>(bar, a.gen + sub, nbar, nwg, a.partial, pbase, 0, a.res + 8 * (int64_t)sub, st,
                                 a.abort_flag, lds_flag, lds, bpar)) {
            stat = 3;
            break;
        }
        double gn[2] = {st[0], st[1]}, dn[2] = {st[2], st[3]}, rrn[2] = {st[4], st[5]};
        if (a.coupled) {
            gn[0] = gn[1] = st[0] + st[1];
            dn[0] = dn[1] = st[2] + st[3];
            rrn[0] = rrn[1] = st[4] + st[5];
        }
        ++it;
        double prog = 0.0;
        for (int c = 0; c < 2; ++c) {
            if (done[c]) continue;
            rrc[c] = rrn[c];
            if (rrn[c] <= tgt[c] || !(gn[c] > 0.0)) {
                done[c] = true;
                continue;
            }
            const double bn = gn[c] / g[c];
            const double den = dn[c] - bn * gn[c] / alpha[c];
            if (!(den > 0.0) || !isfinite(den)) {
                stat = 1;
                break;
            }
            beta[c] = bn;
            alpha[c] = gn[c] / den;
            g[c] = gn[c];
            prog += rrn[c] / rr0[c];
        }
        if (stat) break;
        if (a.coupled) done[1] = done[0];
        // stagnation: no 10% gain of the relative residual in `stall` iterations
        if (prog < 0.9 * best) {
            best = prog;
            it_best = it;
        } else if (!(done[0] && done[1]) && it - it_best > a.stall) {
            stat = 4;
            break;
        }
    }
    // the correction leaves through plain stores (read by the next kernel)
#pragma unroll
    for (int j = 0; j < R; ++j)
        if (valid[j]) a.e[rows[j]] = le[rows[j] - lo];
    if (leader) {
        a.iters[sub] = it;
        a.status[sub] = stat;
        a.rr_out[2 * sub] = rr0[0] > 0.0 ? rrc[0] / rr0[0] : 0.0;
        a.rr_out[2 * sub + 1] = rr0[1] > 0.0 ? rrc[1] / rr0[1] : 0.0;
    }
}

// Streaming batched PCG, for batches whose rows do not fit in the registers of
// one cooperative grid.  The same preconditioned CG and the same fixed-order
// reductions as k_pcg, but e, r, z, p and q live in memory and each wave walks
// any number of its workgroup's slices (s0 + wave + NW j).  An iteration here
// costs hundreds of microseconds of memory round trips, so the kernel spends
// barriers to gather one vector per sparse product instead of two:
//   A1: p = z + beta p (own rows, in place), published;        barrier
//   A2: q = A p gathering p; partial p.q;                      barrier + sums
//   B1: e += alpha p; r -= alpha q; Jacobi: z = D^-1 r and the partials
//       r.z, r.r; SPAI: r published;                            (SPAI: barrier)
//   B2 (SPAI): z = M r gathering r; partials r.z, r.r;         barrier + sums
// Only p (and r with the SPAI) is read by other workgroups: it is published
// and gathered through the piece's coherent vectors, one instruction per row
// pair; everything else, and a thread's own rows of p and r, use plain
// accesses (only the owning thread writes a row within the launch, and a
// thread sees its own stores).  Every vector is updated in place: a row is
// next written two barriers after its last remote read.
template <typename T, int BLK>
__global__ void __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(PGCP_STREAM_WPE)))
k_pcg_stream(CGArgs<T> a) {
    using V2 = typename Vec2<T>::type;
    constexpr int NW = BLK / 64;
    __shared__ double lds[2 * NW * 8];
    int bpar = 0;   // LDS bank of the next block sum
    __shared__ int lds_flag[2];
    const int wg = blockIdx.x;
    const int sub = a.wg_sub[wg];
    if (sub < 0 || !a.active[sub]) return;
    const int s0 = a.wg_s0[wg], s1 = a.wg_s1[wg];
    const int rank = a.wg_rank[wg];
    const int pbase = a.sub_pbase[sub], nwg = a.sub_nwg[sub];
    const bool leader = rank == 0 && threadIdx.x == 0;
    const bool spai = a.pc != nullptr && a.pc[sub] != 0;
    // the wave index as a uniform value: slice numbers, widths and offsets stay in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    unsigned* bar = a.bar + sub;
    unsigned nbar = 0;
    double* mypart = a.partial + 8 * (int64_t)(pbase + rank);
    const int prow0 = a.row0[sub];
    const int64_t prows = (int64_t)a.row0[sub + 1] - prow0;
    V2 zero;
    zero.x = (T)0;
    zero.y = (T)0;

    double st[4];
    double rz[2], rr0[2], rrc[2], beta[2] = {0.0, 0.0};
    bool done[2];
    double best;
    int it_best = 0, it = 0;
    double* cs = a.cgs + 16 * (int64_t)sub;
    if (!a.resume) {
        // ---- start: e = 0, z = D^-1 r, p_old = 0
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int s = s0 + wave; s < s1; s += NW) {
            const int64_t rw = (int64_t)s * 64 + lane;
            V2 r = zero, z = zero;
            if (!a.mask[rw]) {
                r = a.r[rw];
                if (spai) {
                    z = spai_row_stream<T, V2>(a, rw, s, r, prow0, PieceVec<V2>(a.r, prow0, prows));
                } else {
                    const T dinv = (T)1 / a.diag[rw];
                    z.x = dinv * r.x;
                    z.y = dinv * r.y;
                }
            }
            a.e[rw] = zero;
            a.z[rw] = z;
            a.pa[rw] = zero;
            acc[0] += (double)r.x * (double)z.x;
            acc[1] += (double)r.y * (double)z.y;
            acc[2] += (double)r.x * (double)r.x;
            acc[3] += (double)r.y * (double)r.y;
        }
        bsum<BLK, 4>(acc, lds, bpar);
        if (threadIdx.x == 0) {
            for (int i = 0; i < 4; ++i) st_c(mypart + 2 + i, acc[i]);
        }
        nbar++;
        if (piece_reduce<BLK, 4>(bar, a.gen + sub, nbar, nwg, a.partial, pbase, 2, a.res + 8 * (int64_t)sub, st,
                                 a.abort_flag, lds_flag, lds, bpar)) {
            if (leader) a.status[sub] = 3;
            return;
        }
        rz[0] = st[0];
        rz[1] = st[1];
        rr0[0] = st[2];
        rr0[1] = st[3];
        if (a.coupled) {
            rz[0] = rz[1] = st[0] + st[1];
            rr0[0] = rr0[1] = st[2] + st[3];
        }
        rrc[0] = rr0[0];
        rrc[1] = rr0[1];
    } else {
        // ---- continue a paused piece: e, r, z and p are in memory, the
        // scalars in cgs
        rz[0] = cs[0];
        rz[1] = cs[1];
        rr0[0] = cs[2];
        rr0[1] = cs[3];
        rrc[0] = cs[4];
        rrc[1] = cs[5];
        beta[0] = cs[6];
        beta[1] = cs[7];
        it = (int)cs[8];
        it_best = (int)cs[9];
    }
    const double tgt[2] = {a.target_rel2[2 * sub] * rr0[0], a.target_rel2[2 * sub + 1] * rr0[1]};
    if (!a.resume) {
        done[0] = rr0[0] <= tgt[0] || !(rz[0] > 0.0);
        done[1] = rr0[1] <= tgt[1] || !(rz[1] > 0.0);
        best = (done[0] ? 0.0 : 1.0) + (done[1] ? 0.0 : 1.0);
    } else {
        done[0] = cs[10] != 0.0;
        done[1] = cs[11] != 0.0;
        best = cs[12];
    }
    int stat = 0;
    const PieceVec<V2> Pv(a.pa, prow0, prows), Rv(a.r, prow0, prows);

    while (!(done[0] && done[1])) {
        if (it >= a.max_iter) {
            stat = 2;
            break;
        }
        if (it >= a.pause_at) {
            stat = 5;
            break;
        }
        // ---- A1: p = z + beta p on the own rows (a finished coordinate keeps p = 0)
        const T bx = done[0] ? (T)0 : (T)beta[0], by = done[1] ? (T)0 : (T)beta[1];
        const T cx = done[0] ? (T)0 : (T)1, cy = done[1] ? (T)0 : (T)1;
        for (int s = s0 + wave; s < s1; s += 2 * NW) {
            // two slices at a time: both slices' loads before either's store
            const int64_t rA = (int64_t)s * 64 + lane, rB = rA + 64 * NW;
            const bool hasB = s + NW < s1;
            const V2 zA = a.z[rA], oA = a.pa[rA];
            V2 zB = zero, oB = zero;
            if (hasB) {
                zB = a.z[rB];
                oB = a.pa[rB];
            }
            V2 p;
            p.x = cx * zA.x + bx * oA.x;
            p.y = cy * zA.y + by * oA.y;
            Pv.st((int)(rA - prow0), p);
            if (hasB) {
                p.x = cx * zB.x + bx * oB.x;
                p.y = cy * zB.y + by * oB.y;
                Pv.st((int)(rB - prow0), p);
            }
        }
        nbar++;
        if (piece_barrier<BLK>(bar, a.gen + sub, nbar, nwg, a.abort_flag, lds_flag)) {
            stat = 3;
            break;
        }
        // ---- A2: q = A p, gathering p; p.q.  Per slice two memory round
        // trips: the row's own data, its slots' columns and values and its
        // loop neighbours together (no branch on the mask before them), then
        // every gather of p (the first KS slots and the loop neighbours).  The
        // slice's slot offset and width were loaded one slice ahead, so the
        // slot loads wait for nothing.
        double pq[2] = {0.0, 0.0};
        SliceMeta sm;
        // blocks of 64 of the wave's slices: their offsets and widths in one
        // load, outside the slice loop (whose readlanes then wait for nothing)
        for (int sb = s0 + wave; sb < s1; sb += 64 * NW) {
          sm.load(a.sl_ptr, a.sl_w, sb, NW, s1, lane);
          const int se = min(s1, sb + 64 * NW);
          for (int j = 0, s = sb; s < se; ++j, s += NW) {
            const int64_t sbase = sm.base(j);
            const int w = sm.width(j);
            const int64_t rw = (int64_t)s * 64 + lane;
            const int64_t base = sbase + lane;
            const __amdgpu_buffer_rsrc_t rcol = slice_rsrc(a.sl_col, sbase, w), rval = slice_rsrc(a.val, sbase, w);
            const bool msk = a.mask[rw] != 0;
            const V2 p = a.pa[rw];
            const T d = a.diag[rw];
            constexpr int KS = PGCP_STREAM_KB;
            int cc[KS];
            T vv[KS];
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                // through the slice's buffer resources: no branch, one
                // address register for every slot; a slot past the width
                // reads column 0 and value 0, so it adds 0 (its gather reads
                // the piece's first row, or 0 outside the piece)
                cc[t] = slot_ld<int>(rcol, lane, t);
                vv[t] = slot_ld<T>(rval, lane, t);
            }
            // the loop neighbours after the slot loads, both at once, so that
            // waiting for them does not hold the slot loads back
            int ix = (int)rw, iy = (int)rw;
            bool lp = false;
            if (a.coupled) {
                const int pv = a.rprev[rw], nx = a.rnext[rw];
                lp = pv >= 0;
                ix = lp ? nx : (int)rw;
                iy = lp ? pv : (int)rw;
            }
            V2 pp[KS];
#pragma unroll
            for (int t = 0; t < KS; ++t) pp[t] = Pv.ld(cc[t] - prow0);
            const V2 pN = Pv.ld(ix - prow0), pP = Pv.ld(iy - prow0);
            T qx = d * p.x, qy = d * p.y;
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                qx += vv[t] * pp[t].x;
                qy += vv[t] * pp[t].y;
            }
            // rows wider than KS slots (few): the rest in further batches
            for (int k0 = KS; k0 < w; k0 += KS) {
#pragma unroll
                for (int t = 0; t < KS; ++t) {
                    const int64_t el = base + (int64_t)(k0 + t) * 64;
                    const bool in = k0 + t < w;
                    cc[t] = in ? a.sl_col[el] : (int)rw;
                    vv[t] = in ? a.val[el] : (T)0;
                }
#pragma unroll
                for (int t = 0; t < KS; ++t) pp[t] = Pv.ld(cc[t] - prow0);
#pragma unroll
                for (int t = 0; t < KS; ++t) {
                    qx += vv[t] * pp[t].x;
                    qy += vv[t] * pp[t].y;
                }
            }
            if (lp) {
                qx -= (T)0.5 * (pN.y - pP.y);
                qy += (T)0.5 * (pN.x - pP.x);
            }
            if (msk) {
                qx = (T)0;
                qy = (T)0;
            }
            V2 q;
            q.x = qx;
            q.y = qy;
            a.q[rw] = q;
            pq[0] += (double)p.x * (double)qx;
            pq[1] += (double)p.y * (double)qy;
          }
        }
        bsum<BLK, 2>(pq, lds, bpar);
        if (threadIdx.x == 0) {
            st_c(mypart + 0, pq[0]);
            st_c(mypart + 1, pq[1]);
        }
        nbar++;
        double pqs[2];
        if (piece_reduce<BLK, 2>(bar, a.gen + sub, nbar, nwg, a.partial, pbase, 0, a.res + 8 * (int64_t)sub, pqs,
                                 a.abort_flag, lds_flag, lds, bpar)) {
            stat = 3;
            break;
        }
        double alpha[2] = {0.0, 0.0};
        if (a.coupled) {
            double den = pqs[0] + pqs[1];
            if (!(den > 0.0) || !isfinite(den)) {
                stat = 1;
                break;
            }
            alpha[0] = alpha[1] = rz[0] / den;
        } else {
            for (int c = 0; c < 2; ++c) {
                if (done[c]) continue;
                if (!(pqs[c] > 0.0) || !isfinite(pqs[c])) {
                    stat = 1;
                    break;
                }
                alpha[c] = rz[c] / pqs[c];
            }
            if (stat) break;
        }
        // ---- B1: e += alpha p; r -= alpha q; Jacobi: z = D^-1 r, r.z, r.r;
        // SPAI: r published for B2
        const T ax = (T)alpha[0], ay = (T)alpha[1];
        double acc2[4] = {0.0, 0.0, 0.0, 0.0};
        // one row's update from its loaded values; a masked row keeps its values
        auto b1_row = [&](int64_t rw, bool msk, V2 p, V2 q, V2 e, V2 r, T dg) {
            if (msk) return;
            e.x += ax * p.x;
            e.y += ay * p.y;
            r.x -= ax * q.x;
            r.y -= ay * q.y;
            a.e[rw] = e;
            if (spai) {
                Rv.st((int)(rw - prow0), r);
                return;
            }
            const T dinv = (T)1 / dg;
            V2 z;
            z.x = dinv * r.x;
            z.y = dinv * r.y;
            a.r[rw] = r;
            a.z[rw] = z;
            acc2[0] += (double)r.x * (double)z.x;
            acc2[1] += (double)r.y * (double)z.y;
            acc2[2] += (double)r.x * (double)r.x;
            acc2[3] += (double)r.y * (double)r.y;
        };
        for (int s = s0 + wave; s < s1; s += 2 * NW) {
            // two slices at a time, every load of both before either's
            // stores: one memory round trip per pair (the sums keep the
            // order of the slices)
            const int64_t rA = (int64_t)s * 64 + lane, rB = rA + 64 * NW;
            const bool hasB = s + NW < s1;
            const bool mA = a.mask[rA] != 0;
            const V2 pA = a.pa[rA], qA = a.q[rA], eA = a.e[rA], xA = a.r[rA];
            const T dA = a.diag[rA];
            bool mB = true;
            V2 pB = zero, qB = zero, eB = zero, xB = zero;
            T dB = (T)1;
            if (hasB) {
                mB = a.mask[rB] != 0;
                pB = a.pa[rB];
                qB = a.q[rB];
                eB = a.e[rB];
                xB = a.r[rB];
                dB = a.diag[rB];
            }
            b1_row(rA, mA, pA, qA, eA, xA, dA);
            if (hasB) b1_row(rB, mB, pB, qB, eB, xB, dB);
        }
        if (spai) {
            // ---- B2: z = M r, gathering r; r.z, r.r
            nbar++;
            if (piece_barrier<BLK>(bar, a.gen + sub, nbar, nwg, a.abort_flag, lds_flag)) {
                stat = 3;
                break;
            }
            // per slice two memory round trips, as in A2: the row's own data
            // and its first NB slots' values and columns together, then their
            // gathers (the products in spai_row_stream's order).  The FP32
            // values are loaded without a branch and widened where they are
            // used: a conversion inside each guarded load's branch made every
            // load wait for the one before it.
            constexpr int NB = 6;
            SliceMeta sm;
            for (int sb = s0 + wave; sb < s1; sb += 64 * NW) {   // as in A2
              sm.load(a.sl_ptr, a.sl_w, sb, NW, s1, lane);
              const int se = min(s1, sb + 64 * NW);
              for (int j = 0, s = sb; s < se; ++j, s += NW) {
                const int64_t sbase = sm.base(j);
                const int w = sm.width(j);
                const int64_t rw = (int64_t)s * 64 + lane;
                const int64_t base = sbase + lane;
                const __amdgpu_buffer_rsrc_t rcol = slice_rsrc(a.sl_col, sbase, w),
                                             rmv = slice_rsrc(a.mval, sbase, w);
                const bool msk = a.mask[rw] != 0;
                const V2 r = a.r[rw];
                const float dmf = a.mdiag[rw];
                int cc[NB];
                float mf[NB];
#pragma unroll
                for (int t = 0; t < NB; ++t) {
                    // as in A2: a slot past the width reads column 0 and
                    // value 0 and adds 0
                    cc[t] = slot_ld<int>(rcol, lane, t);
                    mf[t] = slot_ld<float>(rmv, lane, t);
                }
                V2 rr[NB];
#pragma unroll
                for (int t = 0; t < NB; ++t) rr[t] = Rv.ld(cc[t] - prow0);
                const T dm = (T)dmf;
                T zx = dm * r.x, zy = dm * r.y;
#pragma unroll
                for (int t = 0; t < NB; ++t) {
                    zx += (T)mf[t] * rr[t].x;
                    zy += (T)mf[t] * rr[t].y;
                }
                for (int k0 = NB; k0 < w; k0 += NB) {   // rows wider than NB slots (few)
#pragma unroll
                    for (int t = 0; t < NB; ++t) {
                        const int64_t el = base + (int64_t)(k0 + t) * 64;
                        const bool in = k0 + t < w;
                        mf[t] = in ? a.mval[el] : 0.0f;
                        cc[t] = in ? a.sl_col[el] : (int)rw;
                    }
#pragma unroll
                    for (int t = 0; t < NB; ++t) rr[t] = Rv.ld(cc[t] - prow0);
#pragma unroll
                    for (int t = 0; t < NB; ++t) {
                        zx += (T)mf[t] * rr[t].x;
                        zy += (T)mf[t] * rr[t].y;
                    }
                }
                if (msk) continue;
                V2 z;
                z.x = zx;
                z.y = zy;
                a.z[rw] = z;
                acc2[0] += (double)r.x * (double)z.x;
                acc2[1] += (double)r.y * (double)z.y;
                acc2[2] += (double)r.x * (double)r.x;
                acc2[3] += (double)r.y * (double)r.y;
              }
            }
        }
        bsum<BLK, 4>(acc2, lds, bpar);
        if (threadIdx.x == 0) {
            for (int i = 0; i < 4; ++i) st_c(mypart + 2 + i, acc2[i]);
        }
        nbar++;
        if (piece_reduce<BLK, 4>(bar, a.gen + sub, nbar, nwg, a.partial, pbase, 2, a.res + 8 * (int64_t)sub, st,
                                 a.abort_flag, lds_flag, lds, bpar)) {
            stat = 3;
            break;
        }
        double rzn[2] = {st[0], st[1]};
        double rrn[2] = {st[2], st[3]};
        if (a.coupled) {
            rzn[0] = rzn[1] = st[0] + st[1];
            rrn[0] = rrn[1] = st[2] + st[3];
        }
        double prog = 0.0;
        for (int c = 0; c < 2; ++c) {
            if (done[c]) continue;
            rrc[c] = rrn[c];
            beta[c] = rzn[c] / rz[c];
            rz[c] = rzn[c];
            if (rrn[c] <= tgt[c] || !(rzn[c] > 0.0)) done[c] = true;
            else prog += rrn[c] / rr0[c];
        }
        if (a.coupled) done[1] = done[0];
        ++it;
        if (prog < 0.9 * best) {
            best = prog;
            it_best = it;
        } else if (!(done[0] && done[1]) && it - it_best > a.stall) {
            stat = 4;
            break;
        }
    }
    if (leader) {
        a.iters[sub] = it;
        a.status[sub] = stat;
        a.rr_out[2 * sub] = rr0[0] > 0.0 ? rrc[0] / rr0[0] : 0.0;
        a.rr_out[2 * sub + 1] = rr0[1] > 0.0 ? rrc[1] / rr0[1] : 0.0;
        if (stat == 5) {
            cs[0] = rz[0];
            cs[1] = rz[1];
            cs[2] = rr0[0];
            cs[3] = rr0[1];
            cs[4] = rrc[0];
            cs[5] = rrc[1];
            cs[6] = beta[0];
            cs[7] = beta[1];
            cs[8] = (double)it;
            cs[9] = (double)it_best;
            cs[10] = done[0] ? 1.0 : 0.0;
            cs[11] = done[1] ? 1.0 : 0.0;
            cs[12] = best;
        }
    }
}

// ----------------------------------------------------------------- DNCP / harmonic set-up and gathers

__global__ void k_init_dncp(int K, const int32_t* __restrict__ pin_row, const double* __restrict__ pin_x1,
                            double2* __restrict__ u) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    u[pin_row[2 * i]] = make_double2(0.0, 0.0);
    u[pin_row[2 * i + 1]] = make_double2(pin_x1[i], 0.0);
}

__device__ __forceinline__ double2 chart_fwd(double2 z, double2 c, int cinf) {
    // w = (z - c) / (1 + conj(c) z); infinity -> 1/conj(c)
    if (isinf(z.x) || isinf(z.y)) {
        if (cinf) return make_double2(0.0, 0.0);
        double d = c.x * c.x + c.y * c.y;
        if (d == 0.0) return make_double2(INFINITY, INFINITY);
        return make_double2(c.x / d, c.y / d);
    }
    if (cinf) {   // chart centred at infinity: w = -1/z
        double d = z.x * z.x + z.y * z.y;
        return make_double2(-z.x / d, z.y / d);
    }
    double nx = z.x - c.x, ny = z.y - c.y;
    double dx = 1.0 + (c.x * z.x + c.y * z.y), dy = c.x * z.y - c.y * z.x;
    double d = dx * dx + dy * dy;
    return make_double2((nx * dx + ny * dy) / d, (ny * dx - nx * dy) / d);
}

__device__ __forceinline__ double2 chart_inv(double2 w, double2 c, int cinf, bool* isinfz) {
    // z = (w + c) / (1 - conj(c) w)
    *isinfz = false;
    if (cinf) {
        double d = w.x * w.x + w.y * w.y;
        if (d == 0.0) {
            *isinfz = true;
            return w;
        }
        return make_double2(-w.x / d, w.y / d);
    }
    double nx = w.x + c.x, ny = w.y + c.y;
    double dx = 1.0 - (c.x * w.x + c.y * w.y), dy = -(c.x * w.y - c.y * w.x);
    double d = dx * dx + dy * dy;
    if (d == 0.0) {
        *isinfz = true;
        return w;
    }
    return make_double2((nx * dx + ny * dy) / d, (ny * dx - nx * dy) / d);
}

__device__ __forceinline__ void inv_stereo(double2 z, bool zinf, double* out) {
    if (zinf || isinf(z.x) || isinf(z.y)) {
        out[0] = 0.0;
        out[1] = 0.0;
        out[2] = 1.0;
        return;
    }
    double r2 = z.x * z.x + z.y * z.y, den = r2 + 1.0;
    out[0] = 2.0 * z.x / den;
    out[1] = -2.0 * z.y / den;
    out[2] = (r2 - 1.0) / den;
}

// One block per piece: the piece's rotation chart for the sphere.  The centre
// is the stereographic image of the normalised mean of the piece's welded
// boundary points on the sphere; chart[3i..3i+2] = (Re c, Im c, c is infinity).
__global__ void __launch_bounds__(BLOCK) k_sphere_charts(const int32_t* __restrict__ loop_ptr,
                                                          const int32_t* __restrict__ loop_seam,
                                                          const double2* __restrict__ welded,
                                                          double* __restrict__ chart) {
    __shared__ double lds[32];
    int i = blockIdx.x;
    int e0 = loop_ptr[i], e1 = loop_ptr[i + 1];
    double m[3] = {0.0, 0.0, 0.0};
    for (int e = e0 + threadIdx.x; e < e1; e += BLOCK) {
        double p[3];
        inv_stereo(welded[loop_seam[e]], false, p);
        m[0] += p[0];
        m[1] += p[1];
        m[2] += p[2];
    }
    block_sum<3>(m, lds);
    if (threadIdx.x == 0) {
        double nrm = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
        double x = m[0] / nrm, y = m[1] / nrm, z = m[2] / nrm;
        double d = 1.0 - z;
        if (d > 0.0) {
            chart[3 * i] = x / d;
            chart[3 * i + 1] = -y / d;
            chart[3 * i + 2] = 0.0;
        } else {
            chart[3 * i] = 0.0;
            chart[3 * i + 1] = 0.0;
            chart[3 * i + 2] = 1.0;
        }
    }
}

// u = welded values (in the piece's chart for the sphere) on loop rows, 0 elsewhere.
__global__ void __launch_bounds__(BLOCK) k_init_harm(int64_t nbdy, int K, const int32_t* __restrict__ loop_ptr,
                                                      const int32_t* __restrict__ loop_row,
                                                      const int32_t* __restrict__ loop_seam,
                                                      const int32_t* __restrict__ slice_sub,
                                                      const double2* __restrict__ welded,
                                                      const double* __restrict__ chart, int sphere,
                                                      double2* __restrict__ u) {
    int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (e >= nbdy) return;
    int r = loop_row[e];
    double2 v = welded[loop_seam[e]];
    if (sphere) {
        int i = slice_sub[r >> 6];
        v = chart_fwd(v, make_double2(chart[3 * i], chart[3 * i + 1]), (int)chart[3 * i + 2]);
    }
    u[r] = v;
}

// One block per piece: translate so the loop mean is 0 and gather the loop.
__global__ void __launch_bounds__(BLOCK) k_dncp_bdy(const int32_t* __restrict__ loop_ptr,
                                                     const int32_t* __restrict__ loop_row,
                                                     const double2* __restrict__ u, double* __restrict__ bdy) {
    __shared__ double lds[32];
    int i = blockIdx.x;
    int e0 = loop_ptr[i], e1 = loop_ptr[i + 1];
    double v[2] = {0.0, 0.0};
    for (int e = e0 + threadIdx.x; e < e1; e += BLOCK) {
        double2 x = u[loop_row[e]];
        v[0] += x.x;
        v[1] += x.y;
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        lds[20] = v[0] / (double)(e1 - e0);
        lds[21] = v[1] / (double)(e1 - e0);
    }
    __syncthreads();
    double mx = lds[20], my = lds[21];
    for (int e = e0 + threadIdx.x; e < e1; e += BLOCK) {
        double2 x = u[loop_row[e]];
        bdy[2 * (int64_t)e] = x.x - mx;
        bdy[2 * (int64_t)e + 1] = x.y - my;
    }
}

// Interior rows write their own value; seam vertices come from the weld.
__global__ void __launch_bounds__(BLOCK) k_harm_out(int64_t N, const uint8_t* __restrict__ row_kind,
                                                     const int32_t* __restrict__ row_gv,
                                                     const int32_t* __restrict__ slice_sub,
                                                     const double2* __restrict__ u, const double* __restrict__ chart,
                                                     int sphere, double* __restrict__ out) {
    int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (r >= N || row_kind[r] != 0) return;
    int64_t g = row_gv[r];
    double2 w = u[r];
    if (sphere) {
        int i = slice_sub[r >> 6];
        bool zi;
        double2 z = chart_inv(w, make_double2(chart[3 * i], chart[3 * i + 1]), (int)chart[3 * i + 2], &zi);
        inv_stereo(z, zi, out + 3 * g);
    } else {
        out[2 * g] = w.x;
        out[2 * g + 1] = w.y;
    }
}

__global__ void __launch_bounds__(BLOCK) k_seam_out(int64_t nseam, const int32_t* __restrict__ seam_gv,
                                                     const double2* __restrict__ welded, int sphere,
                                                     double* __restrict__ out) {
    int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (s >= nseam) return;
    int64_t g = seam_gv[s];
    double2 w = welded[s];
    if (sphere) {
        inv_stereo(w, false, out + 3 * g);
    } else {
        out[2 * g] = w.x;
        out[2 * g + 1] = w.y;
    }
}

// ----------------------------------------------------------------- quasi-conformal fold repair

// Flipped faces of a planar map per piece (signed area <= 0).
__global__ void __launch_bounds__(BLOCK) k_fold_count(int64_t nf, const int32_t* __restrict__ F,
                                                       const int32_t* __restrict__ face_sub,
                                                       const double* __restrict__ X, unsigned* __restrict__ cnt) {
    const int64_t f = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (f >= nf) return;
    const int64_t a = F[3 * f], b = F[3 * f + 1], c = F[3 * f + 2];
    const double ax = X[2 * a], ay = X[2 * a + 1];
    const double o = (X[2 * b] - ax) * (X[2 * c + 1] - ay) - (X[2 * b + 1] - ay) * (X[2 * c] - ax);
    if (!(o > 0.0)) atomicAdd(cnt + (face_sub ? face_sub[f] : 0), 1u);
}

// Contribution of face (t0, t1, t2), in the face's own cyclic order, to entry
// (p, q) of the linear Beltrami solver's matrix: area * grad phi_p . A grad
// phi_q in the face's isometric frame, with
//   A = [[(rho-1)^2 + tau^2, -2 tau], [-2 tau, (rho+1)^2 + tau^2]] / (1 - |mu|^2),
// mu = rho + i tau the map's Beltrami coefficient on the face, its modulus cut
// at mu_max.  The frame starts at the cycle's smallest vertex id and p, q are
// taken in ascending order, so both rows of a symmetric pair get the same bits.
__device__ double lbs_face_entry(const double* __restrict__ V, const double* __restrict__ X, int t0, int t1, int t2,
                                 int p, int q, double mu_max) {
    int a = t0, b = t1, c = t2;
    if (t1 < t0 && t1 < t2) {
        a = t1;
        b = t2;
        c = t0;
    } else if (t2 < t0 && t2 < t1) {
        a = t2;
        b = t0;
        c = t1;
    }
    const double e1x = V[3 * (int64_t)b] - V[3 * (int64_t)a], e1y = V[3 * (int64_t)b + 1] - V[3 * (int64_t)a + 1],
                 e1z = V[3 * (int64_t)b + 2] - V[3 * (int64_t)a + 2];
    const double e2x = V[3 * (int64_t)c] - V[3 * (int64_t)a], e2y = V[3 * (int64_t)c + 1] - V[3 * (int64_t)a + 1],
                 e2z = V[3 * (int64_t)c + 2] - V[3 * (int64_t)a + 2];
    const double l1 = sqrt(e1x * e1x + e1y * e1y + e1z * e1z);
    const double x3 = (e1x * e2x + e1y * e2y + e1z * e2z) / l1;
    const double px = e2x - x3 * e1x / l1, py = e2y - x3 * e1y / l1, pz = e2z - x3 * e1z / l1;
    const double y3 = sqrt(px * px + py * py + pz * pz);
    // the map on the frame: a z + b conj(z), mu = b / a
    //   = (l1 d2 - (x3 + i y3) d1) / (d1 (x3 - i y3) - l1 d2)
    const double d1x = X[2 * (int64_t)b] - X[2 * (int64_t)a], d1y = X[2 * (int64_t)b + 1] - X[2 * (int64_t)a + 1];
    const double d2x = X[2 * (int64_t)c] - X[2 * (int64_t)a], d2y = X[2 * (int64_t)c + 1] - X[2 * (int64_t)a + 1];
    const double nx = l1 * d2x - (x3 * d1x - y3 * d1y), ny = l1 * d2y - (x3 * d1y + y3 * d1x);
    const double dx = d1x * x3 + d1y * y3 - l1 * d2x, dy = d1y * x3 - d1x * y3 - l1 * d2y;
    const double nn = sqrt(nx * nx + ny * ny), dn = sqrt(dx * dx + dy * dy);
    double rho = 0.0, tau = 0.0;
    if (nn >= mu_max * dn) {
        // |mu| >= mu_max: modulus mu_max, direction of num / den (of num if den = 0)
        if (nn > 0.0 && dn > 0.0) {
            rho = mu_max * (nx * dx + ny * dy) / (nn * dn);
            tau = mu_max * (ny * dx - nx * dy) / (nn * dn);
        } else if (nn > 0.0) {
            rho = mu_max * nx / nn;
            tau = mu_max * ny / nn;
        }
    } else {
        const double dd = dx * dx + dy * dy;
        rho = (nx * dx + ny * dy) / dd;
        tau = (ny * dx - nx * dy) / dd;
    }
    const double sc = 1.0 / (1.0 - rho * rho - tau * tau);
    const double A11 = sc * ((rho - 1.0) * (rho - 1.0) + tau * tau), A12 = sc * (-2.0 * tau),
                 A22 = sc * ((rho + 1.0) * (rho + 1.0) + tau * tau);
    // corners Q0 = (0, 0), Q1 = (l1, 0), Q2 = (x3, y3); the gradient of corner k
    // is the opposite edge Q_{k+2} - Q_{k+1} turned by +90 degrees over 2 area
    const int lo = min(p, q), hi = max(p, q);
    const int kl = lo == a ? 0 : (lo == b ? 1 : 2), kh = hi == a ? 0 : (hi == b ? 1 : 2);
    const double Qx[3] = {0.0, l1, x3}, Qy[3] = {0.0, 0.0, y3};
    const double ex_l = Qx[(kl + 2) % 3] - Qx[(kl + 1) % 3], ey_l = Qy[(kl + 2) % 3] - Qy[(kl + 1) % 3];
    const double ex_h = Qx[(kh + 2) % 3] - Qx[(kh + 1) % 3], ey_h = Qy[(kh + 2) % 3] - Qy[(kh + 1) % 3];
    // area * (g_l . A g_h) with g = (-ey, ex) / (2 area), area = l1 y3 / 2
    const double glx = -ey_l, gly = ex_l, ghx = -ey_h, ghy = ex_h;
    return (glx * (A11 * ghx + A12 * ghy) + gly * (A12 * ghx + A22 * ghy)) / (2.0 * l1 * y3);
}

// One thread per packed row: the Beltrami-solver matrix of the current map X
// on the plan's structure (off-diagonal slot = sum over the edge's one or two
// faces, diagonal = minus the row's sum).
__global__ void __launch_bounds__(BLOCK) k_assemble_lbs(
    int64_t nslices, const int64_t* __restrict__ sl_ptr, const int32_t* __restrict__ sl_w,
    const int32_t* __restrict__ sl_col, const int32_t* __restrict__ sl_opp, const uint8_t* __restrict__ sl_ori,
    const int32_t* __restrict__ row_gv, const double* __restrict__ V, const double* __restrict__ X, double mu_max,
    double* __restrict__ val64, float* __restrict__ val32, double* __restrict__ diag64, float* __restrict__ diag32) {
    const int64_t row = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t s = row >> 6;
    if (s >= nslices) return;
    const int lane = (int)(row & 63);
    const int g = row_gv[row];
    const int64_t base = sl_ptr[s] + lane;
    const int w = sl_w[s];
    double dsum = 0.0;
    for (int k = 0; k < w; ++k) {
        const int64_t el = base + (int64_t)k * 64;
        const int o1 = sl_opp[2 * el], o2 = sl_opp[2 * el + 1];
        double v = 0.0;
        if (o1 >= 0 && g >= 0) {
            const int h = row_gv[sl_col[el]];
            const int ori = sl_ori[el];
            v = (ori & 1) ? lbs_face_entry(V, X, g, h, o1, g, h, mu_max) : lbs_face_entry(V, X, h, g, o1, g, h, mu_max);
            if (o2 >= 0)
                v += (ori & 2) ? lbs_face_entry(V, X, g, h, o2, g, h, mu_max)
                               : lbs_face_entry(V, X, h, g, o2, g, h, mu_max);
        }
        val64[el] = v;
        val32[el] = (float)v;
        dsum -= v;
    }
    diag64[row] = dsum;
    diag32[row] = (float)dsum;
}

// Dirichlet values of the repair solve: the map's own values on boundary rows,
// 0 elsewhere.
__global__ void __launch_bounds__(BLOCK) k_fold_init(int64_t N, const uint8_t* __restrict__ row_kind,
                                                      const int32_t* __restrict__ row_gv,
                                                      const double* __restrict__ X, double2* __restrict__ u) {
    const int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (r >= N) return;
    double2 v = make_double2(0.0, 0.0);
    if (row_kind[r] == 1) {
        const int64_t g = row_gv[r];
        v = make_double2(X[2 * g], X[2 * g + 1]);
    }
    u[r] = v;
}

// Interior rows of the pieces whose pass is undone take back their value from
// before the pass.
__global__ void __launch_bounds__(BLOCK) k_fold_undo(int64_t N, const uint8_t* __restrict__ row_kind,
                                                      const int32_t* __restrict__ row_gv,
                                                      const int32_t* __restrict__ slice_sub,
                                                      const unsigned* __restrict__ undo,
                                                      const double* __restrict__ prev, double* __restrict__ X) {
    const int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (r >= N || row_kind[r] != 0 || undo[slice_sub[r >> 6]] == 0) return;
    const int64_t g = row_gv[r];
    X[2 * g] = prev[2 * g];
    X[2 * g + 1] = prev[2 * g + 1];
}

// Interior rows of the pieces repaired in this pass write their new value.
__global__ void __launch_bounds__(BLOCK) k_fold_out(int64_t N, const uint8_t* __restrict__ row_kind,
                                                     const int32_t* __restrict__ row_gv,
                                                     const int32_t* __restrict__ slice_sub,
                                                     const unsigned* __restrict__ cnt,
                                                     const double2* __restrict__ u, double* __restrict__ X) {
    const int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (r >= N || row_kind[r] != 0 || cnt[slice_sub[r >> 6]] == 0) return;
    const int64_t g = row_gv[r];
    X[2 * g] = u[r].x;
    X[2 * g + 1] = u[r].y;
}

// ----------------------------------------------------------------- distortion

__device__ __forceinline__ double angle3(double ux, double uy, double uz, double vx, double vy, double vz) {
    double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
    return atan2(sqrt(cx * cx + cy * cy + cz * cz), ux * vx + uy * vy + uz * vz);
}

struct DistPart {
    double sum, sum2, maxd, maxmu;
    double nflip, nmu1, pad0, pad1;
};

__global__ void __launch_bounds__(BLOCK) k_distortion(int64_t nf, const double* __restrict__ V,
                                                       const int32_t* __restrict__ F, const double* __restrict__ X,
                                                       int dim, double* __restrict__ dout, double* __restrict__ muout,
                                                       uint8_t* __restrict__ flipout, DistPart* __restrict__ part) {
    __shared__ double lds[WAVES * 6 + 32];
    int64_t f = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double s = 0.0, s2 = 0.0, mx = 0.0, mmu = 0.0, nfl = 0.0, nmu = 0.0;
    if (f < nf) {
        int id[3] = {F[3 * f], F[3 * f + 1], F[3 * f + 2]};
        double P[3][3], Q[3][3];
        for (int c = 0; c < 3; ++c) {
            for (int t = 0; t < 3; ++t) P[c][t] = V[3 * (int64_t)id[c] + t];
            Q[c][0] = X[(int64_t)dim * id[c]];
            Q[c][1] = X[(int64_t)dim * id[c] + 1];
            Q[c][2] = dim == 3 ? X[(int64_t)dim * id[c] + 2] : 0.0;
        }
        const double rad2deg = 57.29577951308232;
        for (int c = 0; c < 3; ++c) {
            int i1 = (c + 1) % 3, i2 = (c + 2) % 3;
            double as = angle3(P[i1][0] - P[c][0], P[i1][1] - P[c][1], P[i1][2] - P[c][2], P[i2][0] - P[c][0],
                               P[i2][1] - P[c][1], P[i2][2] - P[c][2]);
            double ap = angle3(Q[i1][0] - Q[c][0], Q[i1][1] - Q[c][1], Q[i1][2] - Q[c][2], Q[i2][0] - Q[c][0],
                               Q[i2][1] - Q[c][1], Q[i2][2] - Q[c][2]);
            double d = (ap - as) * rad2deg;
            if (dout) dout[3 * f + c] = d;
            double ad = fabs(d);
            s += ad;
            s2 += ad * ad;
            mx = fmax(mx, ad);
        }
        // orientation
        double ori;
        if (dim == 2) {
            ori = (Q[1][0] - Q[0][0]) * (Q[2][1] - Q[0][1]) - (Q[1][1] - Q[0][1]) * (Q[2][0] - Q[0][0]);
        } else {
            ori = Q[0][0] * (Q[1][1] * Q[2][2] - Q[1][2] * Q[2][1]) - Q[0][1] * (Q[1][0] * Q[2][2] - Q[1][2] * Q[2][0]) +
                  Q[0][2] * (Q[1][0] * Q[2][1] - Q[1][1] * Q[2][0]);
        }
        bool flip = !(ori > 0.0);
        // Beltrami coefficient between isometric frames: source (0, l1, x3 + i y3)
        double e1[3], e2[3];
        for (int t = 0; t < 3; ++t) {
            e1[t] = P[1][t] - P[0][t];
            e2[t] = P[2][t] - P[0][t];
        }
        double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        double x3 = (e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2]) / l1;
        double py[3];
        for (int t = 0; t < 3; ++t) py[t] = e2[t] - x3 * e1[t] / l1;
        double y3 = sqrt(py[0] * py[0] + py[1] * py[1] + py[2] * py[2]);
        double w2x, w2y, w3x, w3y;
        if (dim == 2) {
            w2x = Q[1][0] - Q[0][0];
            w2y = Q[1][1] - Q[0][1];
            w3x = Q[2][0] - Q[0][0];
            w3y = Q[2][1] - Q[0][1];
        } else {
            double f1[3], f2[3];
            for (int t = 0; t < 3; ++t) {
                f1[t] = Q[1][t] - Q[0][t];
                f2[t] = Q[2][t] - Q[0][t];
            }
            double m1 = sqrt(f1[0] * f1[0] + f1[1] * f1[1] + f1[2] * f1[2]);
            double xx = (f1[0] * f2[0] + f1[1] * f2[1] + f1[2] * f2[2]) / m1;
            double qq[3];
            for (int t = 0; t < 3; ++t) qq[t] = f2[t] - xx * f1[t] / m1;
            double yy = sqrt(qq[0] * qq[0] + qq[1] * qq[1] + qq[2] * qq[2]);
            w2x = m1;
            w2y = 0.0;
            w3x = xx;
            w3y = ori > 0.0 ? yy : -yy;
        }
        // f(z) = a z + b conj(z); e1 = l1, e2 = x3 + i y3; d1 = w2, d2 = w3
        // det = e1 conj(e2) - e2 conj(e1) = -2 i l1 y3
        // a = (d1 conj(e2) - d2 conj(e1)) / det, b = (e1 d2 - e2 d1) / det
        double anx = w2x * x3 + w2y * y3 - w3x * l1, any = w2y * x3 - w2x * y3 - w3y * l1;
        double bnx = l1 * w3x - (x3 * w2x - y3 * w2y), bny = l1 * w3y - (x3 * w2y + y3 * w2x);
        double mu = sqrt((bnx * bnx + bny * bny) / (anx * anx + any * any));
        if (muout) muout[f] = mu;
        if (flipout) flipout[f] = flip ? 1 : 0;
        mmu = mu;
        nfl = flip ? 1.0 : 0.0;
        nmu = (mu >= 1.0 - 1e-8) ? 1.0 : 0.0;
    }
    // block reduction (fixed order)
    double v[6] = {s, s2, mx, mmu, nfl, nmu};
    for (int o = 32; o >= 1; o >>= 1) {
        v[0] += __shfl_xor(v[0], o, 64);
        v[1] += __shfl_xor(v[1], o, 64);
        v[2] = fmax(v[2], __shfl_xor(v[2], o, 64));
        v[3] = fmax(v[3], __shfl_xor(v[3], o, 64));
        v[4] += __shfl_xor(v[4], o, 64);
        v[5] += __shfl_xor(v[5], o, 64);
    }
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int i = 0; i < 6; ++i) lds[wave * 6 + i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        DistPart p{0, 0, 0, 0, 0, 0, 0, 0};
        for (int w = 0; w < WAVES; ++w) {
            p.sum += lds[w * 6];
            p.sum2 += lds[w * 6 + 1];
            p.maxd = fmax(p.maxd, lds[w * 6 + 2]);
            p.maxmu = fmax(p.maxmu, lds[w * 6 + 3]);
            p.nflip += lds[w * 6 + 4];
            p.nmu1 += lds[w * 6 + 5];
        }
        part[blockIdx.x] = p;
    }
}

__global__ void __launch_bounds__(BLOCK) k_dist_final(int64_t nblk, const DistPart* __restrict__ part,
                                                       DistPart* __restrict__ out) {
    __shared__ double lds[WAVES * 6 + 32];
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < nblk; b += BLOCK) {
        DistPart p = part[b];
        v[0] += p.sum;
        v[1] += p.sum2;
        v[2] = fmax(v[2], p.maxd);
        v[3] = fmax(v[3], p.maxmu);
        v[4] += p.nflip;
        v[5] += p.nmu1;
    }
    for (int o = 32; o >= 1; o >>= 1) {
        v[0] += __shfl_xor(v[0], o, 64);
        v[1] += __shfl_xor(v[1], o, 64);
        v[2] = fmax(v[2], __shfl_xor(v[2], o, 64));
        v[3] = fmax(v[3], __shfl_xor(v[3], o, 64));
        v[4] += __shfl_xor(v[4], o, 64);
        v[5] += __shfl_xor(v[5], o, 64);
    }
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int i = 0; i < 6; ++i) lds[wave * 6 + i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        DistPart p{0, 0, 0, 0, 0, 0, 0, 0};
        for (int w = 0; w < WAVES; ++w) {
            p.sum += lds[w * 6];
            p.sum2 += lds[w * 6 + 1];
            p.maxd = fmax(p.maxd, lds[w * 6 + 2]);
            p.maxmu = fmax(p.maxmu, lds[w * 6 + 3]);
            p.nflip += lds[w * 6 + 4];
            p.nmu1 += lds[w * 6 + 5];
        }
        *out = p;
    }
}

// Order statistics of |d| for the median and the quartiles (Section 5's
// distortion summaries): a radix select, most significant digit first, on the
// bit patterns of |d|.  For non-negative IEEE doubles (+inf and NaN included)
// the unsigned order of the bit patterns is the numeric order, NaN last.  Each
// pass counts, per target, the 8-bit digit at `shift` of every element whose
// higher digits equal the target's prefix; one workgroup then picks the digit
// bucket that holds the target's rank.  Eight passes fix all 64 bits, so a
// target ends as the exact bit pattern of its order statistic.
constexpr int kQSelMax = 6;
constexpr int kQSelGrid = 2048;

struct QSelState {
    uint64_t prefix[kQSelMax];   // digits fixed so far, lower bits zero
    int64_t rank[kQSelMax];      // 0-based rank among the elements sharing prefix
};

__global__ void __launch_bounds__(BLOCK) k_qsel_hist(int64_t n, const double* __restrict__ d, int nq, int shift,
                                                     const QSelState* __restrict__ qs, unsigned* __restrict__ hist) {
    __shared__ unsigned lh[kQSelMax * 256];
    __shared__ uint64_t pre[kQSelMax];
    for (int i = threadIdx.x; i < nq * 256; i += BLOCK) lh[i] = 0u;
    if ((int)threadIdx.x < nq) pre[threadIdx.x] = qs->prefix[threadIdx.x];
    __syncthreads();
    const uint64_t hi = shift >= 56 ? 0ull : ~0ull << (shift + 8);
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    // the trip count is the same for the whole workgroup, so every lane takes
    // part in the ballots below
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < n; base += stride) {
        const int64_t i = base + threadIdx.x;
        const bool ok = i < n;
        const uint64_t key = ok ? (uint64_t)__double_as_longlong(fabs(d[i])) : 0ull;
        const unsigned dig = (unsigned)(key >> shift) & 255u;
        for (int t = 0; t < nq; ++t) {
            bool m = ok && (key & hi) == pre[t];
            // one LDS atomic per distinct digit among the wave's matching lanes
            unsigned long long todo = __ballot(m);
            while (todo) {
                const int lead = __ffsll(todo) - 1;
                const unsigned ld = __shfl(dig, lead, 64);
                const unsigned long long same = __ballot(m && dig == ld);
                if (lane == lead) atomicAdd(&lh[t * 256 + ld], (unsigned)__popcll(same));
                m = m && dig != ld;
                todo &= ~same;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nq * 256; i += BLOCK)
        if (lh[i]) atomicAdd(&hist[i], lh[i]);
}

// One workgroup of 256 threads, one per digit value.  Clears the histogram for
// the next pass; after the last pass (shift 0) writes each target's value.
__global__ void __launch_bounds__(256) k_qsel_pick(int nq, int shift, QSelState* qs, unsigned* hist, double* out) {
    __shared__ int64_t sc[256];
    const int tid = threadIdx.x;
    for (int t = 0; t < nq; ++t) {
        const unsigned c = hist[t * 256 + tid];
        hist[t * 256 + tid] = 0u;
        sc[tid] = c;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int64_t v = tid >= off ? sc[tid - off] : 0;
            __syncthreads();
            sc[tid] += v;
            __syncthreads();
        }
        const int64_t incl = sc[tid], excl = incl - (int64_t)c;
        const int64_t r = qs->rank[t];
        __syncthreads();   // every thread has read the rank before its owner rewrites it
        if (excl <= r && r < incl) {
            const uint64_t pf = qs->prefix[t] | ((uint64_t)tid << shift);
            qs->rank[t] = r - excl;
            qs->prefix[t] = pf;
            if (shift == 0) out[t] = __longlong_as_double((long long)pf);
        }
        __syncthreads();
    }
}

__global__ void k_zero_u32(int64_t n, unsigned* p) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_zero_d2(int64_t n, double2* p) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_double2(0.0, 0.0);
}

// ----------------------------------------------------------------- host side: launches


Error launch_assemble(pgcp_ctx* ctx, pgcp_part* P, const double* V) {
    hipStream_t s = ctx->stream;
    HIPCHK(hipMemsetAsync(P->d_flags.p, 0, 4, s));
    k_assemble<<<grid_for(P->N), BLOCK, 0, s>>>(P->nslices, (const int64_t*)P->d_sl_ptr.p,
                                                 (const int32_t*)P->d_sl_w.p, (const int32_t*)P->d_sl_col.p,
                                                 (const int32_t*)P->d_sl_opp.p, (const int32_t*)P->d_row_gv.p, V,
                                                 (double*)P->d_val64.p, (float*)P->d_val32.p,
                                                 (double*)P->d_diag64.p, (float*)P->d_diag32.p,
                                                 (int*)P->d_flags.p);
    HIPCHK(hipGetLastError());
    P->assembled = true;
    return Error{PGCP_OK, ""};
}

// Size-weighted streaming maps fill the grid (PGCP_STREAM_FILL=0: leave the
// rounding's leftover workgroups idle); PGCP_STREAM_WGCU caps the streaming
// kernel's workgroups per CU below what its registers allow.
static bool stream_fill_enabled() {
    const char* v = getenv("PGCP_STREAM_FILL");
    return !(v && v[0] == '0');
}
// Weighted maps give a piece at most one workgroup per PGCP_STREAM_MINSPW x NW
// slices (default 2: when a few large pieces are left, fewer and fuller
// workgroups meet at their barriers faster than they lose in work per wave).
static int stream_min_spw() {
    const char* v = getenv("PGCP_STREAM_MINSPW");
    const int n = v ? atoi(v) : 0;
    return n > 0 ? n : 2;
}
static int stream_wg_per_cu() {
    const char* v = getenv("PGCP_STREAM_WGCU");
    const int n = v ? atoi(v) : 0;
    return n > 0 ? n : 1 << 20;
}

// Launch shapes of the batched PCG: threads per workgroup, 64-row slices per
// wave, and which kernel (register-resident, or streaming through memory).
struct PcgCfg {
    int blk, R, stream;
};
static const PcgCfg kPcgCfgs[] = {{256, 1, 0}, {256, 2, 0}, {256, 4, 0}, {256, 6, 0}, {256, 8, 0}, {512, 1, 0},
                                  {512, 2, 0}, {512, 4, 0}, {1024, 1, 0}, {1024, 2, 0}};

template <typename T>
static const void* pcg_stream_kernel(int blk) {
    if (blk == 512) return reinterpret_cast<const void*>(&k_pcg_stream<T, 512>);
    return reinterpret_cast<const void*>(&k_pcg_stream<T, 256>);
}

template <typename T>
static const void* pcg_kernel(int blk, int R) {
    if (blk == 256) {
        switch (R) {
            case 1: return reinterpret_cast<const void*>(&k_pcg<T, 256, 1>);
            case 2: return reinterpret_cast<const void*>(&k_pcg<T, 256, 2>);
            case 4: return reinterpret_cast<const void*>(&k_pcg<T, 256, 4>);
            case 6: return reinterpret_cast<const void*>(&k_pcg<T, 256, 6>);
            default: return reinterpret_cast<const void*>(&k_pcg<T, 256, 8>);
        }
    }
    if (blk == 512) {
        switch (R) {
            case 1: return reinterpret_cast<const void*>(&k_pcg<T, 512, 1>);
            case 2: return reinterpret_cast<const void*>(&k_pcg<T, 512, 2>);
            default: return reinterpret_cast<const void*>(&k_pcg<T, 512, 4>);
        }
    }
    if (R == 1) return reinterpret_cast<const void*>(&k_pcg<T, 1024, 1>);
    return reinterpret_cast<const void*>(&k_pcg<T, 1024, 2>);
}

template <typename T>
static const void* pcg1_kernel(int blk, int R) {
    if (blk == 256) {
        switch (R) {
            case 1: return reinterpret_cast<const void*>(&k_pcg1<T, 256, 1>);
            case 2: return reinterpret_cast<const void*>(&k_pcg1<T, 256, 2>);
            case 4: return reinterpret_cast<const void*>(&k_pcg1<T, 256, 4>);
            default: return reinterpret_cast<const void*>(&k_pcg1<T, 256, 8>);
        }
    }
    if (blk == 512) {
        switch (R) {
            case 1: return reinterpret_cast<const void*>(&k_pcg1<T, 512, 1>);
            case 2: return reinterpret_cast<const void*>(&k_pcg1<T, 512, 2>);
            default: return reinterpret_cast<const void*>(&k_pcg1<T, 512, 4>);
        }
    }
    if (R == 1) return reinterpret_cast<const void*>(&k_pcg1<T, 1024, 1>);
    return reinterpret_cast<const void*>(&k_pcg1<T, 1024, 2>);
}

// Local numbering of the register-resident kernels.  For each workgroup range
// [s0, s1) of 64-row slices: ring 1 = the sorted distinct columns outside it
// that its rows reference (SELL slots and loop neighbours), ring 2 = the sorted
// distinct columns of ring-1 rows outside the range and ring 1.  Local index:
// own row c -> c - 64 s0, ring-1 entry i -> nown + i, ring-2 entry i ->
// nown + n1 + i (16-bit; larger workgroups are rejected by the caller).
// lcol: local column of every SELL slot of the range's rows; lpn: local loop
// neighbours of its boundary rows; rcol: local columns of the slots of its
// ring-1 rows (KR per row, for the single-reduction kernel, which applies M on
// ring 1); expo: bit 0 if a row is in some workgroup's ring 1, bit 1 if in some
// ring 2 (the rows whose values their owners publish).  The ranges are
// disjoint, so each writes its own slots and rows.
struct LocalNum {
    std::vector<std::vector<int32_t>> halo;    // per range: ring 1, then ring 2
    std::vector<int32_t> n1;                   // per range: ring-1 entries
    std::vector<uint16_t> lcol;                // [sell]
    std::vector<int32_t> lpn;                  // [2N]
    std::vector<std::vector<uint16_t>> rcol;   // per range: [n1 * KR]
    std::vector<uint8_t> expo;                 // [N]
    bool rings_ok = true;                      // ring-1 rows have at most KR slots
};

static void local_numbering(const pgcp_part* P, const std::vector<std::pair<int32_t, int32_t>>& ranges,
                            LocalNum& L) {
    const size_t G = ranges.size();
    L.lcol.assign(P->sell_elems, 0);
    L.lpn.assign(2 * P->N, -1);
    L.halo.assign(G, {});
    L.n1.assign(G, 0);
    L.rcol.assign(G, {});
    L.expo.assign(P->N, 0);
    std::vector<uint8_t> ok(G, 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < (int64_t)G; ++g) {
        const int64_t lo = (int64_t)ranges[g].first * 64, hi = (int64_t)ranges[g].second * 64;
        const int32_t nown = (int32_t)(hi - lo);
        const int64_t e0 = P->sl_ptr[ranges[g].first], e1 = P->sl_ptr[ranges[g].second];
        auto outside = [&](int64_t c) { return c < lo || c >= hi; };
        std::vector<int32_t> r1, r2;
        for (int64_t el = e0; el < e1; ++el)
            if (outside(P->sl_col[el])) r1.push_back(P->sl_col[el]);
        for (int64_t rw = lo; rw < hi; ++rw)
            if (P->row_prev[rw] >= 0 && P->row_next[rw] >= 0) {
                if (outside(P->row_prev[rw])) r1.push_back(P->row_prev[rw]);
                if (outside(P->row_next[rw])) r1.push_back(P->row_next[rw]);
            }
        std::sort(r1.begin(), r1.end());
        r1.erase(std::unique(r1.begin(), r1.end()), r1.end());
        auto in_r1 = [&](int32_t c) { return std::binary_search(r1.begin(), r1.end(), c); };
        for (int32_t c : r1) {
            const int64_t sc = c / 64, lane = c % 64;
            for (int32_t k = 0; k < P->sl_w[sc]; ++k) {
                const int32_t q = P->sl_col[P->sl_ptr[sc] + (int64_t)k * 64 + lane];
                if (outside(q) && !in_r1(q)) r2.push_back(q);
            }
            if (P->sl_w[sc] > KR) ok[g] = 0;
        }
        std::sort(r2.begin(), r2.end());
        r2.erase(std::unique(r2.begin(), r2.end()), r2.end());
        const int32_t n1 = (int32_t)r1.size();
        auto local = [&](int32_t c) -> int32_t {
            if (!outside(c)) return (int32_t)(c - lo);
            auto it = std::lower_bound(r1.begin(), r1.end(), c);
            if (it != r1.end() && *it == c) return nown + (int32_t)(it - r1.begin());
            return nown + n1 + (int32_t)(std::lower_bound(r2.begin(), r2.end(), c) - r2.begin());
        };
        for (int64_t el = e0; el < e1; ++el) L.lcol[el] = (uint16_t)local(P->sl_col[el]);
        for (int64_t rw = lo; rw < hi; ++rw)
            if (P->row_prev[rw] >= 0 && P->row_next[rw] >= 0) {
                L.lpn[2 * rw] = local(P->row_prev[rw]);
                L.lpn[2 * rw + 1] = local(P->row_next[rw]);
            }
        std::vector<uint16_t>& rc = L.rcol[g];
        rc.assign((size_t)n1 * KR, 0);
        for (int32_t i = 0; i < n1; ++i) {
            const int32_t c = r1[i];
            const int64_t sc = c / 64, lane = c % 64;
            for (int32_t k = 0; k < std::min(P->sl_w[sc], KR); ++k)
                rc[(size_t)i * KR + k] = (uint16_t)local(P->sl_col[P->sl_ptr[sc] + (int64_t)k * 64 + lane]);
        }
        L.n1[g] = n1;
        std::vector<int32_t>& h = L.halo[g];
        h = r1;
        h.insert(h.end(), r2.begin(), r2.end());
    }
    for (size_t g = 0; g < G; ++g) {
        L.rings_ok = L.rings_ok && ok[g];
        for (int32_t i = 0; i < (int32_t)L.halo[g].size(); ++i)
            L.expo[L.halo[g][i]] |= (i < L.n1[g]) ? 1 : 2;
    }
}

// Workgroup map for one launch shape.  Pieces are placed on XCDs by
// longest-processing-time first (workgroups g with g % n_xcd == x run on XCD x
// under the hardware's round-robin dispatch), every piece on exactly one XCD,
// so that its per-piece barrier only involves workgroups sharing one L2.
static Error build_workmap(pgcp_ctx* ctx, pgcp_part* P, int prec, PcgCfg cfg, WorkMap* W, bool* fits,
                           const int32_t* only = nullptr, double wexp = 1.5) {
    *fits = false;
    int n_cu = 0, coop = 0;
    HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    HIPCHK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, ctx->device));
    if (!coop) return Error{PGCP_E_HIP, "device does not support cooperative launches"};
    const int n_xcd = (n_cu >= 64 && n_cu % 32 == 0) ? n_cu / 32 : 1;
    const int64_t spw = (int64_t)(cfg.blk / 64) * cfg.R;   // slices per workgroup
    const int K = P->K;
    std::vector<int64_t> nw(K, 1);
    if (cfg.R <= 0 && !cfg.stream) return Error{PGCP_E_INVALID, "slices per wave must be positive"};
    if (spw > 0)
        for (int i = 0; i < K; ++i) {
            int64_t ns = (P->row0[i + 1] - P->row0[i]) / 64;
            nw[i] = std::max<int64_t>(1, (ns + spw - 1) / spw);
        }
    // slice range of workgroup t of piece i (every map but the size-weighted
    // one), and for the register-resident kernel the local numbering of each
    // workgroup's rows and halo
    std::vector<std::pair<int32_t, int32_t>> ranges;
    std::vector<int64_t> range0(K + 1, 0);
    LocalNum L;
    size_t lds_bytes = 0, lds1_bytes = 0;
    int64_t lds_n = 0, lds_nr = 0, lds_nu = 0;
    bool cg1 = false;
    if (spw > 0)
        for (int i = 0; i < K; ++i) {
            const int64_t sb = P->row0[i] / 64, ns = (P->row0[i + 1] - P->row0[i]) / 64;
            range0[i + 1] = range0[i] + nw[i];
            for (int64_t t = 0; t < nw[i]; ++t)
                ranges.emplace_back((int32_t)(sb + ns * t / nw[i]), (int32_t)(sb + ns * (t + 1) / nw[i]));
        }
    if (!cfg.stream) {
        local_numbering(P, ranges, L);
        int64_t max_n1 = 0, max_nh = 0;
        for (size_t g = 0; g < L.halo.size(); ++g) {
            max_n1 = std::max<int64_t>(max_n1, L.n1[g]);
            max_nh = std::max<int64_t>(max_nh, (int64_t)L.halo[g].size());
        }
        int lds_max = 0;
        HIPCHK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
        const int64_t own = (int64_t)cfg.blk * cfg.R;
        const size_t vsz = prec == 0 ? 16 : 8;
        // two-barrier kernel: p and the SPAI operand (own rows + ring 1 each), e (own rows)
        lds_n = own + max_n1;
        lds_bytes = (size_t)(2 * lds_n + (own <= 1024 ? own : 0)) * vsz;   // e in LDS up to 1024 rows
        // local columns are 16-bit; a shape whose workgroup has more entries does not fit
        if (lds_n > 65536 || lds_bytes + 4096 > (size_t)lds_max) return Error{PGCP_OK, ""};
        // single-reduction kernel: r (own rows + both rings), u (own rows + ring 1), e
        lds_nr = own + max_nh;
        lds_nu = own + max_n1;
        lds1_bytes = (size_t)(lds_nr + lds_nu + own) * vsz;
        cg1 = L.rings_ok && lds_nr <= 65536 && lds1_bytes + 4096 <= (size_t)lds_max && cfg.R != 6;
    }
    int per_cu = 0;
    const void* kern = cfg.stream ? (prec == 0 ? pcg_stream_kernel<double>(cfg.blk) : pcg_stream_kernel<float>(cfg.blk))
                                  : (prec == 0 ? pcg_kernel<double>(cfg.blk, cfg.R) : pcg_kernel<float>(cfg.blk, cfg.R));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, cfg.blk, lds_bytes));
    if (cfg.stream) per_cu = std::min(per_cu, stream_wg_per_cu());
    const int64_t cap = (int64_t)per_cu * n_cu;
    int64_t cap1 = 0;
    if (cg1) {
        int pc1 = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &pc1, prec == 0 ? pcg1_kernel<double>(cfg.blk, cfg.R) : pcg1_kernel<float>(cfg.blk, cfg.R), cfg.blk,
            lds1_bytes));
        cap1 = (int64_t)pc1 * n_cu;
    }
    if (cfg.stream && cfg.R <= 0) {
        // Streaming, weighted: fill the cooperative grid, giving piece i workgroups
        // in proportion to ns_i^wexp, at least one and at most one per 2 NW slices.
        // wexp = 1.5 (a whole solve in one launch): rows times expected CG
        // iterations, which grow like sqrt(ns_i) for these Laplacians; 1 (a
        // phase in which every piece runs the same iterations): equal slices
        // per workgroup.  Pieces span all XCDs.
        // (`only`: the pieces to map, the others get no workgroup)
        double tw = 0.0;
        int k_on = 0;
        for (int i = 0; i < K; ++i)
            if (!only || only[i]) {
                tw += std::pow((double)((P->row0[i + 1] - P->row0[i]) / 64), wexp);
                k_on++;
            }
        // every mapped piece needs a workgroup of its own: with more pieces
        // than the grid holds there is no weighted map (the loop below would
        // not run and leave G = 0 while the pieces still took a workgroup each)
        if (k_on == 0 || k_on > cap) return Error{PGCP_OK, ""};
        // at most one workgroup per stream_min_spw() x NW slices (two slices
        // for every wave): more would leave waves short of work and only add
        // participants to the piece's barriers (it matters when a few large
        // pieces are left alone)
        const int64_t nwv = (int64_t)(cfg.blk / 64) * stream_min_spw();
        int64_t G = 0;
        for (double target = (double)cap; target >= k_on; target *= 0.97) {
            G = 0;
            for (int i = 0; i < K; ++i) {
                const int64_t ns = (P->row0[i + 1] - P->row0[i]) / 64;
                const double want = target * std::pow((double)ns, wexp) / tw;
                const int64_t most = std::max<int64_t>(1, ns / nwv);
                nw[i] = (only && !only[i]) ? 0 : std::min<int64_t>(most, std::max<int64_t>(1, (int64_t)std::floor(want)));
                G += nw[i];
            }
            if (G <= cap) break;
        }
        if (G > cap) return Error{PGCP_OK, ""};
        if (stream_fill_enabled()) {
            // the workgroups the rounding left over go, one at a time, to the
            // piece with the most slices per workgroup that can take one: the
            // grid is then full, so every CU holds the same number of them
            std::priority_queue<std::pair<double, int>> pq;
            for (int i = 0; i < K; ++i)
                if (nw[i] > 0) pq.push({(double)((P->row0[i + 1] - P->row0[i]) / 64) / (double)nw[i], i});
            while (G < cap && !pq.empty()) {
                const int i = pq.top().second;
                pq.pop();
                const int64_t ns = (P->row0[i + 1] - P->row0[i]) / 64;
                if (nw[i] >= std::max<int64_t>(1, ns / nwv)) continue;
                nw[i]++;
                G++;
                pq.push({(double)ns / (double)nw[i], i});
            }
        }
        W->blk = cfg.blk;
        W->rows_per_thread = 0;
        W->stream = 1;
        W->lds_bytes = 0;
        W->n_xcd = n_xcd;
        W->n_wg = (int)G;
        W->wg_sub.assign(G, -1);
        W->wg_rank.assign(G, 0);
        W->wg_s0.assign(G, 0);
        W->wg_s1.assign(G, 0);
        W->sub_pbase.assign(K, 0);
        W->sub_nwg.assign(K, 0);
        int32_t pb = 0;
        int64_t g = 0;
        for (int i = 0; i < K; ++i) {
            W->sub_pbase[i] = pb;
            W->sub_nwg[i] = (int32_t)nw[i];
            pb += (int32_t)nw[i];
            const int64_t sb = P->row0[i] / 64, ns = (P->row0[i + 1] - P->row0[i]) / 64;
            for (int64_t t = 0; t < nw[i]; ++t, ++g) {
                W->wg_sub[g] = i;
                W->wg_rank[g] = (int32_t)t;
                W->wg_s0[g] = (int32_t)(sb + ns * t / nw[i]);
                W->wg_s1[g] = (int32_t)(sb + ns * (t + 1) / nw[i]);
            }
        }
        W->n_partials = pb;
        Error e{PGCP_OK, ""};
        if ((e = upload(W->d_wg_sub, W->wg_sub, ctx->stream)).code) return e;
        if ((e = upload(W->d_wg_rank, W->wg_rank, ctx->stream)).code) return e;
        if ((e = upload(W->d_wg_s0, W->wg_s0, ctx->stream)).code) return e;
        if ((e = upload(W->d_wg_s1, W->wg_s1, ctx->stream)).code) return e;
        if ((e = upload(W->d_sub_pbase, W->sub_pbase, ctx->stream)).code) return e;
        if ((e = upload(W->d_sub_nwg, W->sub_nwg, ctx->stream)).code) return e;
        if ((e = dev_alloc(P->d_partial, (size_t)pb * 8 * 8)).code) return e;
        *fits = true;
        return Error{PGCP_OK, ""};
    }
    std::vector<int> order(K);
    for (int i = 0; i < K; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nw[a] > nw[b]; });
    std::vector<int64_t> load(n_xcd, 0);
    std::vector<std::vector<int>> on(n_xcd);
    for (int i : order) {
        int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        on[x].push_back(i);
        load[x] += nw[i];
    }
    const int64_t slots = *std::max_element(load.begin(), load.end());
    const int64_t G = slots * n_xcd;
    if (G > cap) return Error{PGCP_OK, ""};
    W->blk = cfg.blk;
    W->rows_per_thread = cfg.R;
    W->stream = cfg.stream;
    W->n_xcd = n_xcd;
    W->n_wg = (int)G;
    W->wg_sub.assign(G, -1);
    W->wg_rank.assign(G, 0);
    W->wg_s0.assign(G, 0);
    W->wg_s1.assign(G, 0);
    W->sub_pbase.assign(K, 0);
    W->sub_nwg.assign(K, 0);
    int32_t pb = 0;
    for (int i = 0; i < K; ++i) {
        W->sub_pbase[i] = pb;
        W->sub_nwg[i] = (int32_t)nw[i];
        pb += (int32_t)nw[i];
    }
    W->n_partials = pb;
    W->lds_bytes = lds_bytes;
    W->lds_n = (int)lds_n;
    W->cg1 = cg1 && G <= cap1;
    W->lds1_bytes = lds1_bytes;
    W->lds_nr = (int)lds_nr;
    W->lds_nu = (int)lds_nu;
    for (int x = 0; x < n_xcd; ++x) {
        int64_t slot = 0;
        for (int i : on[x]) {
            for (int64_t t = 0; t < nw[i]; ++t, ++slot) {
                int64_t g = slot * n_xcd + x;
                W->wg_sub[g] = i;
                W->wg_rank[g] = (int32_t)t;
                W->wg_s0[g] = ranges[range0[i] + t].first;
                W->wg_s1[g] = ranges[range0[i] + t].second;
            }
        }
    }
    // halo entries in workgroup order (register-resident kernel only)
    std::vector<int32_t> wg_h0(G + 1, 0), wg_n1(G, 0), hcat;
    std::vector<uint16_t> rcat;
    for (int64_t g = 0; g < G && !cfg.stream; ++g) {
        if (W->wg_sub[g] >= 0) {
            const int64_t rg = range0[W->wg_sub[g]] + W->wg_rank[g];
            const auto& h = L.halo[rg];
            hcat.insert(hcat.end(), h.begin(), h.end());
            wg_n1[g] = L.n1[rg];
            // KR local columns per halo entry (ring-2 entries unused), indexed like the halo
            rcat.insert(rcat.end(), L.rcol[rg].begin(), L.rcol[rg].end());
            rcat.resize(hcat.size() * KR, 0);
        }
        if (hcat.size() * KR > (size_t)INT32_MAX) return Error{PGCP_E_INVALID, "halo too large for int32 offsets"};
        wg_h0[g + 1] = (int32_t)hcat.size();
    }
    if (hcat.empty()) hcat.push_back(0);
    if (rcat.empty()) rcat.push_back(0);
    Error e{PGCP_OK, ""};
    if (!cfg.stream) {
        if ((e = upload(W->d_wg_h0, wg_h0, ctx->stream)).code) return e;
        if ((e = upload(W->d_halo, hcat, ctx->stream)).code) return e;
        if ((e = upload(W->d_wg_n1, wg_n1, ctx->stream)).code) return e;
        if ((e = upload(W->d_lcol, L.lcol, ctx->stream)).code) return e;
        if ((e = upload(W->d_lpn, L.lpn, ctx->stream)).code) return e;
        if ((e = upload(W->d_rcol, rcat, ctx->stream)).code) return e;
        if ((e = upload(W->d_expo, L.expo, ctx->stream)).code) return e;
    }
    if ((e = upload(W->d_wg_sub, W->wg_sub, ctx->stream)).code) return e;
    if ((e = upload(W->d_wg_rank, W->wg_rank, ctx->stream)).code) return e;
    if ((e = upload(W->d_wg_s0, W->wg_s0, ctx->stream)).code) return e;
    if ((e = upload(W->d_wg_s1, W->wg_s1, ctx->stream)).code) return e;
    if ((e = upload(W->d_sub_pbase, W->sub_pbase, ctx->stream)).code) return e;
    if ((e = upload(W->d_sub_nwg, W->sub_nwg, ctx->stream)).code) return e;
    if ((e = dev_alloc(P->d_partial, (size_t)pb * 8 * 8)).code) return e;
    *fits = true;
    return Error{PGCP_OK, ""};
}

template <typename T>
static CGArgs<T> cg_args(pgcp_part* P, const WorkMap& W, const uint8_t* mask, int coupled, int max_iter,
                         const T* val, const T* diag) {
    using V2 = typename Vec2<T>::type;
    CGArgs<T> a;
    a.sl_ptr = (const int64_t*)P->d_sl_ptr.p;
    a.sl_w = (const int32_t*)P->d_sl_w.p;
    a.sl_col = (const int32_t*)P->d_sl_col.p;
    a.val = val;
    a.diag = diag;
    a.rprev = (const int32_t*)P->d_row_prev.p;
    a.rnext = (const int32_t*)P->d_row_next.p;
    a.mask = mask;
    a.wg_sub = (const int32_t*)W.d_wg_sub.p;
    a.wg_rank = (const int32_t*)W.d_wg_rank.p;
    a.wg_s0 = (const int32_t*)W.d_wg_s0.p;
    a.wg_s1 = (const int32_t*)W.d_wg_s1.p;
    a.sub_pbase = (const int32_t*)W.d_sub_pbase.p;
    a.sub_nwg = (const int32_t*)W.d_sub_nwg.p;
    a.row0 = (const int32_t*)P->d_row0.p;
    a.wg_h0 = (const int32_t*)W.d_wg_h0.p;
    a.halo = (const int32_t*)W.d_halo.p;
    a.lcol = (const uint16_t*)W.d_lcol.p;
    a.lpn = (const int32_t*)W.d_lpn.p;
    a.lds_n = W.lds_n;
    a.wg_n1 = (const int32_t*)W.d_wg_n1.p;
    a.rcol = (const uint16_t*)W.d_rcol.p;
    a.expo = (const uint8_t*)W.d_expo.p;
    a.s1 = (V2*)P->d_s1.p;
    a.lds_nr = W.lds_nr;
    a.lds_nu = W.lds_nu;
    a.active = (const int32_t*)P->d_active.p;
    a.target_rel2 = (const double*)P->d_target.p;
    a.e = (V2*)P->d_e.p;
    a.r = (V2*)P->d_r.p;
    a.z = (V2*)P->d_z.p;
    a.pa = (V2*)P->d_p0.p;
    a.pb = (V2*)P->d_p1.p;
    a.q = (V2*)P->d_q.p;
    a.r2 = (V2*)P->d_r2.p;
    a.mval = nullptr;
    a.mdiag = nullptr;
    a.pc = nullptr;
    a.partial = (double*)P->d_partial.p;
    a.bar = (unsigned*)P->d_bar.p;
    a.gen = (unsigned*)P->d_gen.p;
    a.res = (double*)P->d_res.p;
    a.abort_flag = (int*)P->d_abort.p;
    a.iters = (int32_t*)P->d_iters.p;
    a.rr_out = (double*)P->d_rrout.p;
    a.status = (int32_t*)P->d_status.p;
    a.cgs = (double*)P->d_cgs.p;
    a.pause_at = INT32_MAX;
    a.resume = 0;
    a.coupled = coupled;
    a.max_iter = max_iter;
    a.n_xcd = W.n_xcd;
    a.stall = 600;
    return a;
}

static Error prep_inner(pgcp_part* P, int prec, hipStream_t s) {
    if (prec) {
        k_prep_inner<float><<<grid_for(P->N), BLOCK, 0, s>>>(P->N, (const int32_t*)P->d_slice_sub.p,
                                                              (const double2*)P->d_r64.p,
                                                              (const double*)P->d_scale.p, (float2*)P->d_r.p,
                                                              (float2*)P->d_e.p);
    } else {
        k_prep_inner<double><<<grid_for(P->N), BLOCK, 0, s>>>(P->N, (const int32_t*)P->d_slice_sub.p,
                                                               (const double2*)P->d_r64.p,
                                                               (const double*)P->d_scale.p, (double2*)P->d_r.p,
                                                               (double2*)P->d_e.p);
    }
    k_zero_u32<<<grid_for(P->K), BLOCK, 0, s>>>(P->K, (unsigned*)P->d_bar.p);
    k_zero_u32<<<grid_for(P->K), BLOCK, 0, s>>>(P->K, (unsigned*)P->d_gen.p);
    k_zero_u32<<<1, 64, 0, s>>>(16, (unsigned*)P->d_abort.p);
    HIPCHK(hipGetLastError());
    return Error{PGCP_OK, ""};
}

// The runtime runs cooperative launches on a queue of its own, not on the
// stream's (a kernel trace of a multi-lane stream shows every lane's batched-CG
// kernel on one queue and the lanes' other kernels on theirs), so the kernels
// the stream ran just before (the right-hand side, the zeroed barrier counters
// and abort words) would be ordered before it only by the runtime's
// cross-queue dependency.  The host waits for the stream before every
// cooperative launch instead.
static Error launch_pcg(pgcp_part* P, const WorkMap& W, int prec, const uint8_t* mask, int coupled, int max_iter,
                        int stall, hipStream_t s, const int32_t* pc = nullptr, bool single = false,
                        int pause_at = INT32_MAX, int resume = 0) {
    HIPCHK(hipStreamSynchronize(s));
    single = single && W.cg1 && !W.stream;
    dim3 grid(W.n_wg), block(W.blk);
    if (prec) {
        CGArgs<float> a = cg_args<float>(P, W, mask, coupled, max_iter, (const float*)P->d_val32.p,
                                         (const float*)P->d_diag32.p);
        a.stall = stall;
        a.pause_at = pause_at;
        a.resume = resume;
        if (pc) {
            a.pc = pc;
            a.mval = (const float*)P->d_mval32.p;
            a.mdiag = (const float*)P->d_mdiag32.p;
        }
        void* args[] = {&a};
        if (W.stream)
            HIPCHK(hipLaunchCooperativeKernel(pcg_stream_kernel<float>(W.blk), grid, block, args, 0, s));
        else if (single)
            HIPCHK(hipLaunchCooperativeKernel(pcg1_kernel<float>(W.blk, W.rows_per_thread), grid, block, args,
                                              W.lds1_bytes, s));
        else
            HIPCHK(hipLaunchCooperativeKernel(pcg_kernel<float>(W.blk, W.rows_per_thread), grid, block, args,
                                              W.lds_bytes, s));
    } else {
        CGArgs<double> a = cg_args<double>(P, W, mask, coupled, max_iter, (const double*)P->d_val64.p,
                                           (const double*)P->d_diag64.p);
        a.stall = stall;
        a.pause_at = pause_at;
        a.resume = resume;
        if (pc) {
            a.pc = pc;
            a.mval = (const float*)P->d_mval32.p;
            a.mdiag = (const float*)P->d_mdiag32.p;
        }
        void* args[] = {&a};
        if (W.stream)
            HIPCHK(hipLaunchCooperativeKernel(pcg_stream_kernel<double>(W.blk), grid, block, args, 0, s));
        else if (single)
            HIPCHK(hipLaunchCooperativeKernel(pcg1_kernel<double>(W.blk, W.rows_per_thread), grid, block, args,
                                              W.lds1_bytes, s));
        else
            HIPCHK(hipLaunchCooperativeKernel(pcg_kernel<double>(W.blk, W.rows_per_thread), grid, block, args,
                                              W.lds_bytes, s));
    }
    return Error{PGCP_OK, ""};
}

// Smallest power-of-two slices per wave with which the streaming kernel's
// grid fits in one cooperative launch (0 if none does).
static Error stream_fit(pgcp_ctx* ctx, pgcp_part* P, int prec, int blk, int* R) {
    *R = 0;
    for (int r = 1; r <= 1 << 16; r *= 2) {
        WorkMap T;
        bool fits;
        Error e = build_workmap(ctx, P, prec, PcgCfg{blk, r, 1}, &T, &fits);
        free_workmap(T);
        if (e.code) return e;
        if (fits) {
            *R = r;
            return Error{PGCP_OK, ""};
        }
    }
    return Error{PGCP_OK, ""};
}

// Choose the launch shape: PGCP_PCG_CFG64 / PGCP_PCG_CFG32 (per inner
// precision) or PGCP_PCG_CFG = "blk,R" (register-resident) or "blk,R,1"
// (streaming; R = 0: size-weighted map) forces one; otherwise every shape that
// fits is timed (best of two 40-iteration probes) on the real batch the first
// time a batch of that shape is solved on the device, and the fastest (by more
// than 3% over the earlier candidates) is kept
// for every context on that device (contexts that solve side by side share
// it), and in the PGCP_TUNE_CACHE file if one is named.  The streaming kernel is tried with the fewest and twice the fewest
// slices per wave that fit.
static std::mutex g_tuned_mu;

// A batched-CG launch needs every workgroup resident at once and sized for
// the whole device, so two of them must not share it: contexts that solve
// side by side on their own streams take this lock from the launch to the
// kernel's end (their other kernels run freely around it).
// Error for a batched-CG launch whose barrier wait gave up, with the record
// the first workgroup to give up left in the abort words.
static Error barrier_error(pgcp_part* P, const std::vector<int32_t>& wg_sub, hipStream_t s, const char* what) {
    int rec[16] = {0};
    if (hipMemcpyAsync(rec, P->d_abort.p, sizeof rec, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return Error{PGCP_E_HIP, what};
    const int wg = rec[6];
    const int sub = (wg >= 0 && wg < (int)wg_sub.size()) ? wg_sub[wg] : -1;
    char msg[320];
    snprintf(msg, sizeof msg,
             "%s (workgroup %d of %d, piece %d, waited at barrier %d of its piece's %d workgroups: %d arrivals "
             "of %lld, generation %d)",
             what, wg, (int)wg_sub.size(), sub, rec[2], rec[3], rec[4], (long long)rec[2] * rec[3], rec[5]);
    return Error{PGCP_E_HIP, msg};
}

static std::mutex& coop_mutex(int device) {
    static std::mutex mu[16];
    return mu[(unsigned)device % 16];
}
static std::map<std::string, std::array<int, 3>> g_tuned;   // {threads per workgroup, slices per wave, streaming}

// PGCP_TUNE_CACHE names a text file that keeps tuned shapes across processes,
// one line per batch: "<tag> <batch key> <threads> <slices per wave>
// <streaming>".  The tag is the device's architecture and compute-unit count
// and the time this library was built, so lines written for another GPU or by
// another build are ignored.  The file is read once per process (under
// g_tuned_mu) and each new result is appended as one line.
static std::string tune_tag(pgcp_ctx* ctx) {
    hipDeviceProp_t pr;
    std::string t = hipGetDeviceProperties(&pr, ctx->device) == hipSuccess ? pr.gcnArchName : "unknown";
    t += "/" + std::to_string(ctx->n_cu) + "/" __DATE__ "/" __TIME__;
    for (char& c : t)
        if (c == ' ') c = '_';
    return t;
}

static void tune_cache_load(pgcp_ctx* ctx) {   // g_tuned_mu held
    static std::set<std::string> loaded;       // "<device>|<path>"
    const char* path = getenv("PGCP_TUNE_CACHE");
    if (!path || !path[0]) return;
    if (!loaded.insert(std::to_string(ctx->device) + "|" + path).second) return;
    std::ifstream in(path);
    const std::string tag = tune_tag(ctx);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string t, bkey;
        std::array<int, 3> v{};
        if (!(ls >> t >> bkey >> v[0] >> v[1] >> v[2]) || t != tag) continue;
        g_tuned[std::to_string(ctx->device) + "/" + bkey] = v;
    }
}

static void tune_cache_append(pgcp_ctx* ctx, const std::string& bkey, const std::array<int, 3>& v) {
    const char* path = getenv("PGCP_TUNE_CACHE");
    if (!path || !path[0]) return;
    const std::string line = tune_tag(ctx) + " " + bkey + " " + std::to_string(v[0]) + " " +
                             std::to_string(v[1]) + " " + std::to_string(v[2]) + "\n";
    if (FILE* f = fopen(path, "a")) {   // one write per line: appends from several processes do not interleave
        fwrite(line.data(), 1, line.size(), f);
        fclose(f);
    }
}

static Error choose_workmap(pgcp_ctx* ctx, pgcp_part* P, int prec, const uint8_t* mask, int coupled) {
    WorkMap& W = prec ? P->wmap32 : P->wmap64;
    if (W.n_wg > 0) return Error{PGCP_OK, ""};
    hipStream_t s = ctx->stream;
    const char* force = getenv(prec ? "PGCP_PCG_CFG32" : "PGCP_PCG_CFG64");
    if (!force) force = getenv("PGCP_PCG_CFG");
    if (force) {
        PcgCfg c{256, 1, 0};
        if (sscanf(force, "%d,%d,%d", &c.blk, &c.R, &c.stream) >= 2) {
            bool fits;
            Error e = build_workmap(ctx, P, prec, c, &W, &fits);
            if (e.code) return e;
            if (fits) return Error{PGCP_OK, ""};
        }
    }
    std::string bkey = std::to_string(prec) + ":" + std::to_string(coupled) + ":" + std::to_string(P->K);
    for (int i = 0; i < P->K; ++i) bkey += "," + std::to_string((P->row0[i + 1] - P->row0[i]) / 64);
    const std::string key = std::to_string(ctx->device) + "/" + bkey;
    bool known = false;
    std::array<int, 3> shape{};
    {
        std::lock_guard<std::mutex> g(g_tuned_mu);
        tune_cache_load(ctx);
        auto hit = g_tuned.find(key);
        if (hit != g_tuned.end()) {
            known = true;
            shape = hit->second;
        }
    }
    if (known) {
        bool fits;
        Error e = build_workmap(ctx, P, prec, PcgCfg{shape[0], shape[1], shape[2]}, &W, &fits);
        if (e.code) return e;
        if (fits) return Error{PGCP_OK, ""};
    }
    const char* tune = getenv("PGCP_TUNE");
    const bool do_tune = !(tune && tune[0] == '0');
    float best_ms = 1e30f;
    PcgCfg best{0, 0, 0};
    const int probe_iters = 40;
    std::vector<PcgCfg> cands(std::begin(kPcgCfgs), std::end(kPcgCfgs));
    for (int blk : {256, 512}) {
        int r = 0;
        Error e = stream_fit(ctx, P, prec, blk, &r);
        if (e.code) return e;
        if (r > 0) {
            cands.push_back(PcgCfg{blk, r, 1});
            cands.push_back(PcgCfg{blk, 2 * r, 1});
        }
    }
    // The probes time every piece for the same number of iterations, which
    // cannot show that the streaming kernel's size-weighted map lets large
    // pieces (that need more iterations) finish sooner; when the pieces'
    // sizes differ by more than 2x it is used whenever the register-resident
    // kernel does not fit.
    int64_t ns_min = INT64_MAX, ns_max = 0;
    for (int i = 0; i < P->K; ++i) {
        const int64_t ns = (P->row0[i + 1] - P->row0[i]) / 64;
        ns_min = std::min(ns_min, ns);
        ns_max = std::max(ns_max, ns);
    }
    const bool uneven = ns_max > 2 * ns_min;
    bool reg_fits = false;
    for (const PcgCfg& c : cands) {
        if (c.stream) continue;
        WorkMap T;
        bool fits;
        Error e = build_workmap(ctx, P, prec, c, &T, &fits);
        free_workmap(T);
        if (e.code) return e;
        reg_fits |= fits;
    }
    if (uneven && !reg_fits) {
        // the weighted maps that fit replace the other candidates; with more
        // pieces than a weighted grid holds, the streaming shapes with equal
        // slices per workgroup stay
        std::vector<PcgCfg> wc;
        for (int blk : {256, 512}) {
            WorkMap T;
            bool fits;
            Error e = build_workmap(ctx, P, prec, PcgCfg{blk, 0, 1}, &T, &fits);
            free_workmap(T);
            if (e.code) return e;
            if (fits) wc.push_back(PcgCfg{blk, 0, 1});
        }
        if (!wc.empty()) cands = wc;
    }
    for (const PcgCfg& c : cands) {
        WorkMap T;
        bool fits;
        Error e = build_workmap(ctx, P, prec, c, &T, &fits);
        if (e.code) return e;
        if (!fits) continue;
        if (!do_tune) {
            best = c;
            break;
        }
        float ms = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {   // best of two probes
            if ((e = prep_inner(P, prec, s)).code) return e;
            {
                std::lock_guard<std::mutex> g(coop_mutex(ctx->device));
                HIPCHK(hipEventRecord(P->ev0, s));
                if ((e = launch_pcg(P, T, prec, mask, coupled, probe_iters, 1 << 30, s)).code) return e;
                HIPCHK(hipEventRecord(P->ev1, s));
                HIPCHK(hipEventSynchronize(P->ev1));
            }
            float m1 = 0.f;
            HIPCHK(hipEventElapsedTime(&m1, P->ev0, P->ev1));
            int ab = 0;
            HIPCHK(hipMemcpy(&ab, P->d_abort.p, 4, hipMemcpyDeviceToHost));
            if (ab) return barrier_error(P, T.wg_sub, s, "batched CG barrier timed out while tuning");
            ms = std::min(ms, m1);
        }
        const char* vb = getenv("PGCP_VERBOSE");
        if (vb && vb[0] == '1')
            fprintf(stderr, "[pgcp] tune prec=%d coupled=%d shape %d,%d,%d: %d workgroups, %.3f ms / %d iterations\n",
                    prec, coupled, c.blk, c.R, c.stream, T.n_wg, ms, probe_iters);
        // a later shape must be clearly faster: shapes within timing noise of
        // each other keep the earlier one, so that the choice is repeatable
        if (ms < 0.97f * best_ms) {
            best_ms = ms;
            best = c;
        }
        free_workmap(T);
    }
    if (best.blk == 0) return Error{PGCP_E_INVALID, "problem too large for one cooperative launch"};
    bool fits;
    Error e = build_workmap(ctx, P, prec, best, &W, &fits);
    if (e.code) return e;
    {
        std::lock_guard<std::mutex> g(g_tuned_mu);
        g_tuned[key] = {best.blk, best.R, best.stream};
        if (do_tune) tune_cache_append(ctx, bkey, g_tuned[key]);
    }
    return Error{PGCP_OK, ""};
}

// Phased streaming solves (PGCP_PCG_PHASES=0 turns them off; PGCP_PCG_PHASE0
// sets the first phase's iteration cap).
static bool phases_enabled() {
    const char* v = getenv("PGCP_PCG_PHASES");
    return !(v && v[0] == '0');
}
static int phase_wide() {   // pieces left below which phases use 512-thread workgroups
    const char* v = getenv("PGCP_PCG_PHASE_WIDE");
    return v ? atoi(v) : 16;
}
static int phase0_cap() {
    const char* v = getenv("PGCP_PCG_PHASE0");
    const int c = v ? atoi(v) : 0;
    return c > 0 ? c : 1024;
}

// Iterative refinement driver.  u64 holds the Dirichlet values on masked rows
// and the current iterate elsewhere; solves A u = 0 on the free rows of every
// piece to ||r||_2 <= tol ||b||_2 (per coordinate unless coupled), where
// b = -A_FD u_D is the first residual (u_F = 0 on entry).  Each pass evaluates
// the FP64 residual, then runs one batched PCG (FP64, or FP32 on the scaled
// residual) on the pieces that have not converged, and adds its correction.
static Error refine_solve(pgcp_ctx* ctx, pgcp_part* P, int coupled, const uint8_t* mask,
                          const pgcp_solve_opts* o, pgcp_solve_stats* st, int system,
                          const int32_t* only = nullptr) {
    hipStream_t s = ctx->stream;
    const int K = P->K;
    // learned preconditioner: network outputs for this system, every piece on
    // the SPAI until it breaks down or stagnates (then Jacobi)
    const bool learned = o && o->precond == PGCP_PC_LEARNED;
    std::vector<int32_t> pc(K, learned ? 1 : 0);
    int n_fallback = 0;
    if (learned) {
        if (!o->lpc) return Error{PGCP_E_INVALID, "PGCP_PC_LEARNED needs opts.lpc"};
        if (P->spai_sys != system) {
            Error e0 = lpc_infer(ctx, P, o->lpc, system);
            if (e0.code) return e0;
        }
        Error e0 = dev_alloc(P->d_pc, (size_t)K * 4);
        if (e0.code) return e0;
    }
    const int prec = (o && o->precision == PGCP_FP32_REFINE) ? 1 : 0;
    const double tol = (o && o->tol > 0) ? o->tol : 1e-10;
    const double inner_tol = (o && o->inner_tol > 0) ? o->inner_tol : 1e-4;
    const int max_iter = (o && o->max_iter > 0) ? o->max_iter : 20000;
    const int max_refine = (o && o->max_refine > 0) ? o->max_refine : 30;
    const int stall = (o && o->stall_iters > 0) ? o->stall_iters : 4000;
    const char* vb = getenv("PGCP_VERBOSE");
    const bool verbose = vb && vb[0] == '1';
    if (!P->ev0) {
        // the host waits for the end of each batched-CG launch on ev1: a
        // blocking wait leaves the core to other host work meanwhile (the
        // partition of the next mesh, another lane's weld)
        HIPCHK(hipEventCreate(&P->ev0));
        HIPCHK(hipEventCreateWithFlags(&P->ev1, hipEventBlockingSync));
    }
    Error e{PGCP_OK, ""};
    const WorkMap& W = prec ? P->wmap32 : P->wmap64;
    // two-barrier kernel unless PGCP_PCG_KERNEL=single (the single-reduction
    // kernel measured slower on C2 and drifts at tight tolerances); a pass whose
    // pieces break down or stagnate with it is repeated with the two-barrier kernel
    const char* kv = getenv("PGCP_PCG_KERNEL");
    bool single = kv && std::strcmp(kv, "single") == 0;
    bool used_single = false;

    std::vector<double> bnorm(2 * K, 0.0), rnorm(2 * K, 0.0), scale(2 * K, 0.0), target(2 * K, 0.0);
    std::vector<int32_t> active(K, 0), iters(K, 0), status(K, 0), it_total(K, 0), fail(K, 0);
    std::vector<double> relres(2 * K, 0.0);
    int steps = 0;
    int64_t total = 0;
    bool all_conv = false;
    double cg_ms = 0.0, cg_bytes = 0.0, cg_bytes_native = 0.0;
    int cg_launches = 0;
    // Minimal bytes of one CG iteration of piece i, in the FP32 accounting of
    // the method's cost model: per row its matrix entries with the diagonal
    // (FP32 value + int32 index, 8 B each), the FP32 inverse diagonal (4 B),
    // and the interleaved (x, y) state vectors x, r, p, q read and written once
    // plus one gather of p and the preconditioner's diagonal (76 B); the learned
    // SPAI adds its own value and index stream (8 B per entry with the diagonal).
    auto iter_bytes_min = [&](int i) {
        const double entries = (double)P->sub_nnz[i] + (double)P->sub_nv[i];
        double b = 8.0 * entries + 80.0 * (double)P->sub_nv[i];
        if (pc[i]) b += 8.0 * entries;
        return b;
    };
    // The same iteration as this launch moves it, at the precision of its
    // recurrences: matrix values + column indices once, and per row z, p_old
    // read, p_new written (phase A), e and r read+written, z written (phase B),
    // the diagonal twice and the mask twice.
    const double tsz = prec ? 4.0 : 8.0;
    auto iter_bytes = [&](int i) {
        double b = (double)P->sub_nnz[i] * (tsz + 4.0) + (double)P->sub_nv[i] * (8.0 * 2.0 * tsz + 2.0 * tsz + 2.0);
        // the SPAI apply reads M (FP32 values + column indices, diagonal) and writes and gathers r once more
        if (pc[i]) b += (double)P->sub_nnz[i] * (4.0 + 4.0) + (double)P->sub_nv[i] * (4.0 + 2.0 * 2.0 * tsz);
        return b;
    };
    for (int outer = 0; outer < max_refine; ++outer) {
        k_residual64<<<grid_for(P->N), BLOCK, 0, s>>>(
            P->nslices, (const int64_t*)P->d_sl_ptr.p, (const int32_t*)P->d_sl_w.p, (const int32_t*)P->d_sl_col.p,
            (const double*)P->d_val64.p, (const double*)P->d_diag64.p, (const int32_t*)P->d_row_prev.p,
            (const int32_t*)P->d_row_next.p, coupled, mask, (const double2*)P->d_u64.p, (double2*)P->d_r64.p,
            (double*)P->d_slicepart.p);
        HIPCHK(hipGetLastError());
        k_piece_sum<<<K, BLOCK, 0, s>>>((const int32_t*)P->d_row0.p, (const double*)P->d_slicepart.p,
                                        (double*)P->d_rnorm.p);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(rnorm.data(), P->d_rnorm.p, 2 * K * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        steps++;
        if (outer == 0) bnorm = rnorm;
        int n_active = 0;
        for (int i = 0; i < K; ++i) {
            double rel[2];
            if (coupled) {
                double b = bnorm[2 * i] + bnorm[2 * i + 1], r = rnorm[2 * i] + rnorm[2 * i + 1];
                rel[0] = rel[1] = b > 0 ? std::sqrt(r / b) : (r > 0 ? INFINITY : 0.0);
            } else {
                for (int c = 0; c < 2; ++c) {
                    double b = bnorm[2 * i + c], r = rnorm[2 * i + c];
                    rel[c] = b > 0 ? std::sqrt(r / b) : (r > 0 ? INFINITY : 0.0);
                }
            }
            relres[2 * i] = rel[0];
            relres[2 * i + 1] = rel[1];
            bool conv = (only && !only[i]) || (rel[0] <= tol && rel[1] <= tol);   // `only`: pieces to solve
            active[i] = (!conv && !fail[i]) ? 1 : 0;
            n_active += active[i];
            for (int c = 0; c < 2; ++c) {
                double r = coupled ? rnorm[2 * i] + rnorm[2 * i + 1] : rnorm[2 * i + c];
                scale[2 * i + c] = prec ? std::sqrt(r) : 1.0;
                // inner target: reach tol with margin; FP32 stops at inner_tol
                double need = rel[c] > 0 ? 0.25 * (tol / rel[c]) * (tol / rel[c]) : 1.0;
                if (coupled && c == 1) need = target[2 * i];
                if (prec) need = std::max(need, inner_tol * inner_tol);
                target[2 * i + c] = std::min(need, 1.0);
            }
        }
        if (verbose) {
            double worst = 0.0;
            for (int i = 0; i < K; ++i) worst = std::max(worst, std::max(relres[2 * i], relres[2 * i + 1]));
            fprintf(stderr, "[pgcp] %s %s pass %d: active %d/%d worst relres %.3e\n", coupled ? "dncp" : "harmonic",
                    prec ? "fp32" : "fp64", outer, n_active, K, worst);
        }
        if (n_active == 0) {
            all_conv = true;
            break;
        }
        if (outer == max_refine - 1) break;
        HIPCHK(hipMemcpyAsync(P->d_active.p, active.data(), K * 4, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(P->d_scale.p, scale.data(), 2 * K * 8, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(P->d_target.p, target.data(), 2 * K * 8, hipMemcpyHostToDevice, s));
        // launch shape: chosen once per plan and precision, on this residual
        if ((e = choose_workmap(ctx, P, prec, mask, coupled)).code) return e;
        if ((e = prep_inner(P, prec, s)).code) return e;
        if (learned) HIPCHK(hipMemcpyAsync(P->d_pc.p, pc.data(), K * 4, hipMemcpyHostToDevice, s));
        const bool this_single = single && W.cg1 && !W.stream;
        // Streaming batches run in phases: every piece pauses when its iteration
        // count reaches the phase's cap (1,024, then doubling) and the pieces
        // that have not converged continue, from their state in memory, on a
        // map over them alone, so that the workgroups of finished pieces go to
        // the slow ones (with at most 16 pieces left, 512-thread workgroups:
        // fewer of them meet at each per-piece barrier).
        const bool phased = W.stream && K > 1 && phases_enabled();
        int cap = phased ? phase0_cap() : INT32_MAX;
        std::vector<int32_t> last_map;   // piece of every workgroup of the last launch (error reports)
        {
            // every phase runs its pieces for the same iterations: equal slices per workgroup
            WorkMap W1;
            bool fits1 = false;
            if (phased && (e = build_workmap(ctx, P, prec, PcgCfg{W.blk, 0, 1}, &W1, &fits1, active.data(), 1.0)).code)
                return e;
            std::lock_guard<std::mutex> g(coop_mutex(ctx->device));
            HIPCHK(hipEventRecord(P->ev0, s));
            last_map = (fits1 ? W1 : W).wg_sub;
            e = launch_pcg(P, fits1 ? W1 : W, prec, mask, coupled, max_iter, stall, s,
                           learned ? (const int32_t*)P->d_pc.p : nullptr, this_single, cap, 0);
            if (e.code == PGCP_OK) HIPCHK(hipEventRecord(P->ev1, s));
            if (e.code == PGCP_OK) HIPCHK(hipEventSynchronize(P->ev1));
            free_workmap(W1);
            if (e.code) return e;
        }
        int n_phase = 1;
        while (phased) {
            float pm = 0.f;
            HIPCHK(hipEventElapsedTime(&pm, P->ev0, P->ev1));
            cg_ms += pm;
            cg_launches++;
            if (verbose) fprintf(stderr, "[pgcp]   phase %d took %.2f ms\n", n_phase, pm);
            int abort_flag = 0;
            HIPCHK(hipMemcpyAsync(&abort_flag, P->d_abort.p, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(status.data(), P->d_status.p, K * 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (abort_flag) return barrier_error(P, last_map, s, "batched CG barrier timed out");
            std::vector<int32_t> paused(K, 0);
            int n_paused = 0;
            for (int i = 0; i < K; ++i)
                if (active[i] && status[i] == 5) {
                    paused[i] = 1;
                    n_paused++;
                }
            if (n_paused == 0) break;
            WorkMap Wp;
            bool fits = false;
            const PcgCfg pcfg{n_paused <= phase_wide() ? 512 : W.blk, 0, 1};
            if ((e = build_workmap(ctx, P, prec, pcfg, &Wp, &fits, paused.data(), 1.0)).code) return e;
            cap = cap > INT32_MAX / 2 ? INT32_MAX : 2 * cap;
            HIPCHK(hipMemcpyAsync(P->d_active.p, paused.data(), K * 4, hipMemcpyHostToDevice, s));
            k_zero_u32<<<grid_for(K), BLOCK, 0, s>>>(K, (unsigned*)P->d_bar.p);
            k_zero_u32<<<grid_for(K), BLOCK, 0, s>>>(K, (unsigned*)P->d_gen.p);
            k_zero_u32<<<1, 64, 0, s>>>(16, (unsigned*)P->d_abort.p);
            HIPCHK(hipGetLastError());
            {
                std::lock_guard<std::mutex> g(coop_mutex(ctx->device));
                HIPCHK(hipEventRecord(P->ev0, s));
                last_map = (fits ? Wp : W).wg_sub;
                e = launch_pcg(P, fits ? Wp : W, prec, mask, coupled, max_iter, stall, s,
                               learned ? (const int32_t*)P->d_pc.p : nullptr, false, cap, 1);
                if (e.code == PGCP_OK) HIPCHK(hipEventRecord(P->ev1, s));
                if (e.code == PGCP_OK) HIPCHK(hipEventSynchronize(P->ev1));
            }
            free_workmap(Wp);
            if (e.code) return e;
            n_phase++;
            if (verbose)
                fprintf(stderr, "[pgcp]   phase %d: %d pieces on %d workgroups of %d threads, pause at %d\n",
                        n_phase, n_paused, fits ? Wp.n_wg : W.n_wg, fits ? pcfg.blk : W.blk, cap);
        }
        if (phased) {
            // the pass's correction is applied to every piece it started with
            HIPCHK(hipMemcpyAsync(P->d_active.p, active.data(), K * 4, hipMemcpyHostToDevice, s));
        }
        used_single = this_single;
        if (prec) {
            k_apply_inner<float><<<grid_for(P->N), BLOCK, 0, s>>>(P->N, (const int32_t*)P->d_slice_sub.p,
                                                                   (const int32_t*)P->d_active.p,
                                                                   (const double*)P->d_scale.p,
                                                                   (const float2*)P->d_e.p, (double2*)P->d_u64.p);
        } else {
            k_apply_inner<double><<<grid_for(P->N), BLOCK, 0, s>>>(P->N, (const int32_t*)P->d_slice_sub.p,
                                                                    (const int32_t*)P->d_active.p,
                                                                    (const double*)P->d_scale.p,
                                                                    (const double2*)P->d_e.p, (double2*)P->d_u64.p);
        }
        HIPCHK(hipGetLastError());
        int abort_flag = 0;
        HIPCHK(hipMemcpyAsync(&abort_flag, P->d_abort.p, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(iters.data(), P->d_iters.p, K * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(status.data(), P->d_status.p, K * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (abort_flag) return barrier_error(P, last_map, s, "batched CG barrier timed out");
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, P->ev0, P->ev1));
        if (!phased) {   // a phased pass has counted each of its launches
            cg_ms += ms;
            cg_launches++;
        }
        if (verbose) {
            int mx = 0, nst[5] = {0, 0, 0, 0, 0};
            for (int i = 0; i < K; ++i)
                if (active[i]) {
                    mx = std::max(mx, iters[i]);
                    nst[std::min(std::max(status[i], 0), 4)]++;
                }
            fprintf(stderr, "[pgcp]   cg launch %.2f ms (last phase), max iters %d, status ok/brk/maxit/abort/stall "
                    "%d/%d/%d/%d/%d\n", ms, mx, nst[0], nst[1], nst[2], nst[3], nst[4]);
        }
        bool bad = false;
        for (int i = 0; i < K; ++i)
            if (active[i] && (status[i] == 1 || status[i] == 4)) bad = true;
        if (this_single && bad) {
            // repeat with the two-barrier kernel (the residual is recomputed first)
            single = false;
            for (int i = 0; i < K; ++i) {
                if (!active[i]) continue;
                it_total[i] += iters[i];
                total += iters[i];
                cg_bytes += iters[i] * iter_bytes_min(i);
                cg_bytes_native += iters[i] * iter_bytes(i);
            }
            continue;
        }
        for (int i = 0; i < K; ++i) {
            if (!active[i]) continue;
            it_total[i] += iters[i];
            total += iters[i];
            cg_bytes += iters[i] * iter_bytes_min(i);
            cg_bytes_native += iters[i] * iter_bytes(i);
            if (pc[i] && (status[i] == 1 || status[i] == 4)) {
                pc[i] = 0;   // learned SPAI broke down or stagnated: Jacobi from here on
                n_fallback++;
                continue;
            }
            if (status[i] == 1 && iters[i] == 0) fail[i] = 1;   // breakdown before any progress
        }
    }
    bool noconv = false;
    for (int i = 0; i < K; ++i) {
        bool conv = (only && !only[i]) || (relres[2 * i] <= tol && relres[2 * i + 1] <= tol);
        if (!conv) noconv = true;
        if (st) {
            if (st->iters) st->iters[i] = it_total[i];
            if (st->relres) {
                st->relres[2 * i] = relres[2 * i];
                st->relres[2 * i + 1] = relres[2 * i + 1];
            }
            if (st->status) st->status[i] = conv ? 0 : (fail[i] ? PGCP_E_BREAKDOWN : PGCP_E_NOCONV);
        }
    }
    (void)all_conv;
    if (st) {
        st->n_sub = K;
        st->refine_steps = steps;
        st->total_iters = total;
        st->cg_kernel_ms = cg_ms;
        st->cg_bytes = cg_bytes;
        st->cg_bytes_native = cg_bytes_native;
        st->cg_launches = cg_launches;
        st->rows_per_thread = W.rows_per_thread;
        st->cg_workgroups = W.n_wg;
        st->cg_block = W.blk;
        st->cg_stream = W.stream;
        st->n_fallback = n_fallback;
        st->cg_single = used_single ? 1 : 0;
    }
    if (noconv) return Error{PGCP_E_NOCONV, "some piece missed the residual tolerance"};
    return Error{PGCP_OK, ""};
}

Error run_local_param(pgcp_ctx* ctx, pgcp_part* P, const pgcp_solve_opts* o, double* bdy,
                      pgcp_solve_stats* st) {
    if (!P->assembled) return Error{PGCP_E_INVALID, "pgcp_assemble_cotan has not run"};
    hipStream_t s = ctx->stream;
    k_zero_d2<<<grid_for(P->N), BLOCK, 0, s>>>(P->N, (double2*)P->d_u64.p);
    k_init_dncp<<<grid_for(P->K), BLOCK, 0, s>>>(P->K, (const int32_t*)P->d_pin_row.p,
                                                  (const double*)P->d_pin_x1.p, (double2*)P->d_u64.p);
    HIPCHK(hipGetLastError());
    Error e = refine_solve(ctx, P, 1, (const uint8_t*)P->d_mask_dncp.p, o, st, 0);
    if (e.code != PGCP_OK && e.code != PGCP_E_NOCONV) return e;
    P->solved = PGCP_SYS_DNCP;
    k_dncp_bdy<<<P->K, BLOCK, 0, s>>>((const int32_t*)P->d_loop_ptr.p, (const int32_t*)P->d_loop_row.p,
                                       (const double2*)P->d_u64.p, bdy);
    HIPCHK(hipGetLastError());
    return e;
}

Error run_harmonic(pgcp_ctx* ctx, pgcp_part* P, const double* welded, const pgcp_solve_opts* o, double* out,
                   pgcp_solve_stats* st) {
    if (!P->assembled) return Error{PGCP_E_INVALID, "pgcp_assemble_cotan has not run"};
    hipStream_t s = ctx->stream;
    const int sphere = P->mode == PGCP_SPHERE;
    if (sphere)
        k_sphere_charts<<<P->K, BLOCK, 0, s>>>((const int32_t*)P->d_loop_ptr.p, (const int32_t*)P->d_loop_seam.p,
                                                (const double2*)welded, (double*)P->d_chart.p);
    k_zero_d2<<<grid_for(P->N), BLOCK, 0, s>>>(P->N, (double2*)P->d_u64.p);
    k_init_harm<<<grid_for(P->n_bdy), BLOCK, 0, s>>>(P->n_bdy, P->K, (const int32_t*)P->d_loop_ptr.p,
                                                      (const int32_t*)P->d_loop_row.p,
                                                      (const int32_t*)P->d_loop_seam.p,
                                                      (const int32_t*)P->d_slice_sub.p, (const double2*)welded,
                                                      (const double*)P->d_chart.p, sphere, (double2*)P->d_u64.p);
    HIPCHK(hipGetLastError());
    Error e = refine_solve(ctx, P, 0, (const uint8_t*)P->d_mask_harm.p, o, st, 1);
    if (e.code != PGCP_OK && e.code != PGCP_E_NOCONV) return e;
    P->solved = PGCP_SYS_HARMONIC;
    k_harm_out<<<grid_for(P->N), BLOCK, 0, s>>>(P->N, (const uint8_t*)P->d_row_kind.p, (const int32_t*)P->d_row_gv.p,
                                                 (const int32_t*)P->d_slice_sub.p, (const double2*)P->d_u64.p,
                                                 (const double*)P->d_chart.p, sphere, out);
    k_seam_out<<<grid_for(P->n_seam), BLOCK, 0, s>>>(P->n_seam, (const int32_t*)P->d_seam_gv.p,
                                                      (const double2*)welded, sphere, out);
    HIPCHK(hipGetLastError());
    return e;
}

// Quasi-conformal fold repair of the planar maps of every piece (Sections 3.5
// and 4.5): while a piece's map X has a flipped face, X on its interior is
// replaced by the solution of the linear Beltrami solver for X's own
// coefficient cut at modulus 1 - delta, with X's boundary values (batched CG,
// Jacobi, on the pieces concerned only).
Error run_fold_repair(pgcp_ctx* ctx, pgcp_part* P, const int32_t* F, const double* V, double* X, double delta,
                      int max_passes, const pgcp_solve_opts* o, pgcp_fold_stats* fs) {
    if (!P->assembled) return Error{PGCP_E_INVALID, "pgcp_assemble_cotan has not run"};
    if (P->mode == PGCP_SPHERE) return Error{PGCP_E_INVALID, "fold repair takes planar (free or disk) maps"};
    if (!(delta > 0.0 && delta < 1.0)) return Error{PGCP_E_INVALID, "delta must lie in (0, 1)"};
    if (max_passes < 0) return Error{PGCP_E_INVALID, "max_passes must be >= 0"};
    hipStream_t s = ctx->stream;
    const int K = P->K;
    Error e{PGCP_OK, ""};
    pgcp_fold_stats out{};
    if ((e = dev_alloc(P->d_fold_cnt, (size_t)K * 4)).code) return e;
    // a folding-free map (the usual case) costs one counting pass
    {
        unsigned total = 0;
        k_zero_u32<<<1, 64, 0, s>>>(1, (unsigned*)P->d_fold_cnt.p);
        k_fold_count<<<grid_for(P->nf), BLOCK, 0, s>>>(P->nf, F, nullptr, X, (unsigned*)P->d_fold_cnt.p);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&total, P->d_fold_cnt.p, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (total == 0) {
            if (fs) *fs = out;
            return e;
        }
    }
    // face -> piece and the slots' face orientation, on first use
    if (!P->d_face_sub.p && (e = upload(P->d_face_sub, P->face_sub, s)).code) return e;
    if (!P->d_sl_ori.p && (e = upload(P->d_sl_ori, P->sl_ori, s)).code) return e;
    if (!P->d_lbs_val64.p) {
        if ((e = dev_alloc(P->d_lbs_val64, (size_t)P->sell_elems * 8)).code) return e;
        if ((e = dev_alloc(P->d_lbs_val32, (size_t)P->sell_elems * 4)).code) return e;
        if ((e = dev_alloc(P->d_lbs_diag64, (size_t)P->N * 8)).code) return e;
        if ((e = dev_alloc(P->d_lbs_diag32, (size_t)P->N * 4)).code) return e;
    }
    pgcp_solve_opts lo{};
    if (o) lo = *o;
    lo.precond = PGCP_PC_JACOBI;   // the network was trained on cotangent Laplacians
    lo.lpc = nullptr;
    // the map before the current pass, for pieces whose pass has to be undone
    if ((e = dev_alloc(P->d_fold_prev, (size_t)P->nv * 16)).code) return e;
    std::vector<unsigned> cnt(K, 0), prev(K, 0), undo(K, 0), go(K, 0);
    std::vector<int32_t> only(K, 0), kept(K, 0), stopped(K, 0);
    int64_t flips = 0;
    for (int pass = 0;; ++pass) {
        k_zero_u32<<<grid_for(K), BLOCK, 0, s>>>(K, (unsigned*)P->d_fold_cnt.p);
        k_fold_count<<<grid_for(P->nf), BLOCK, 0, s>>>(P->nf, F, (const int32_t*)P->d_face_sub.p, X,
                                                        (unsigned*)P->d_fold_cnt.p);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(cnt.data(), P->d_fold_cnt.p, (size_t)K * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (pass > 0) {
            // a pass that did not lower a piece's flip count is undone and ends
            // that piece's repair (its welded boundary itself may fold)
            bool any = false;
            for (int i = 0; i < K; ++i) {
                undo[i] = (only[i] && cnt[i] >= prev[i]) ? 1u : 0u;
                if (undo[i]) {
                    any = true;
                    stopped[i] = 1;
                    cnt[i] = prev[i];
                } else if (only[i]) {
                    kept[i] = 1;
                }
            }
            if (any) {
                HIPCHK(hipMemcpyAsync(P->d_fold_cnt.p, undo.data(), (size_t)K * 4, hipMemcpyHostToDevice, s));
                k_fold_undo<<<grid_for(P->N), BLOCK, 0, s>>>(P->N, (const uint8_t*)P->d_row_kind.p,
                                                             (const int32_t*)P->d_row_gv.p,
                                                             (const int32_t*)P->d_slice_sub.p,
                                                             (const unsigned*)P->d_fold_cnt.p,
                                                             (const double*)P->d_fold_prev.p, X);
                HIPCHK(hipGetLastError());
            }
        }
        flips = 0;
        for (int i = 0; i < K; ++i) flips += cnt[i];
        if (pass == 0) out.flips_before = flips;
        int n_go = 0;
        for (int i = 0; i < K; ++i) {
            only[i] = (cnt[i] > 0 && !stopped[i]) ? 1 : 0;
            n_go += only[i];
        }
        if (n_go == 0 || pass == max_passes) break;
        for (int i = 0; i < K; ++i) prev[i] = cnt[i];
        HIPCHK(hipMemcpyAsync(P->d_fold_prev.p, X, (size_t)P->nv * 16, hipMemcpyDeviceToDevice, s));
        // the pieces of this pass (k_fold_out reads them from d_fold_cnt)
        for (int i = 0; i < K; ++i) go[i] = (unsigned)only[i];
        HIPCHK(hipMemcpyAsync(P->d_fold_cnt.p, go.data(), (size_t)K * 4, hipMemcpyHostToDevice, s));
        k_assemble_lbs<<<grid_for(P->N), BLOCK, 0, s>>>(
            P->nslices, (const int64_t*)P->d_sl_ptr.p, (const int32_t*)P->d_sl_w.p, (const int32_t*)P->d_sl_col.p,
            (const int32_t*)P->d_sl_opp.p, (const uint8_t*)P->d_sl_ori.p, (const int32_t*)P->d_row_gv.p, V, X,
            1.0 - delta, (double*)P->d_lbs_val64.p, (float*)P->d_lbs_val32.p, (double*)P->d_lbs_diag64.p,
            (float*)P->d_lbs_diag32.p);
        k_fold_init<<<grid_for(P->N), BLOCK, 0, s>>>(P->N, (const uint8_t*)P->d_row_kind.p,
                                                      (const int32_t*)P->d_row_gv.p, X, (double2*)P->d_u64.p);
        HIPCHK(hipGetLastError());
        // the solver reads the plan's matrix: lend it the Beltrami-solver values
        std::swap(P->d_val64, P->d_lbs_val64);
        std::swap(P->d_val32, P->d_lbs_val32);
        std::swap(P->d_diag64, P->d_lbs_diag64);
        std::swap(P->d_diag32, P->d_lbs_diag32);
        pgcp_solve_stats st{};
        e = refine_solve(ctx, P, 0, (const uint8_t*)P->d_mask_harm.p, &lo, &st, PGCP_SYS_HARMONIC + 1, only.data());
        std::swap(P->d_val64, P->d_lbs_val64);
        std::swap(P->d_val32, P->d_lbs_val32);
        std::swap(P->d_diag64, P->d_lbs_diag64);
        std::swap(P->d_diag32, P->d_lbs_diag32);
        P->solved = -1;
        out.total_iters += st.total_iters;
        out.cg_kernel_ms += st.cg_kernel_ms;
        if (e.code != PGCP_OK) break;
        k_fold_out<<<grid_for(P->N), BLOCK, 0, s>>>(P->N, (const uint8_t*)P->d_row_kind.p,
                                                     (const int32_t*)P->d_row_gv.p, (const int32_t*)P->d_slice_sub.p,
                                                     (const unsigned*)P->d_fold_cnt.p, (const double2*)P->d_u64.p, X);
        HIPCHK(hipGetLastError());
        out.passes++;
    }
    out.flips_after = flips;
    for (int i = 0; i < K; ++i) {
        out.pieces_repaired += kept[i];     // pieces with at least one kept pass
        out.pieces_stopped += stopped[i];   // pieces whose last pass was undone
    }
    if (fs) *fs = out;
    return e;
}

// Distortion check without allocation (pgcp_distortion_noalloc).  The
// per-workgroup partial records of k_distortion and the final record live in a
// fixed device array: kNoAllocBlocks workgroups of BLOCK faces, so at most
// kNoAllocMaxFaces faces per call (2 MiB + one record per device, held until
// the process ends).  In host code `scratch` is only a symbol: its device
// address on each device comes from hipGetSymbolAddress, taken once per device
// at context creation with that device current.
constexpr int64_t kNoAllocBlocks = 32768;
constexpr int64_t kNoAllocMaxFaces = kNoAllocBlocks * BLOCK;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) DistPart scratch[kNoAllocBlocks + 1];
static DistPart* g_scratch_ptr[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices];
static std::mutex g_scratch_mu;

Error noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return Error{PGCP_E_INVALID, "device ordinal out of range"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return Error{PGCP_OK, ""};
    void* ptr = nullptr;
    const hipError_t rc = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (rc != hipSuccess || !ptr) {
        g_scratch_err[device] = rc != hipSuccess ? rc : hipErrorInvalidSymbol;
        (void)hipGetLastError();   // the failure belongs to this entry point only
        return Error{PGCP_E_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(g_scratch_err[device])};
    }
    g_scratch_ptr[device] = (DistPart*)ptr;
    return Error{PGCP_OK, ""};
}

int64_t noalloc_max_faces() { return kNoAllocMaxFaces; }

Error run_distortion_noalloc(pgcp_ctx* ctx, const double* V, const int32_t* F, int64_t nf, const double* X,
                             int dim, double* d, double* mu, uint8_t* flip, pgcp_dist_stats* st) {
    if (nf > kNoAllocMaxFaces) return Error{PGCP_E_INVALID, "more faces than the fixed scratch array holds"};
    DistPart* part = nullptr;
    if (ctx->device >= 0 && ctx->device < kMaxDevices) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        part = g_scratch_ptr[ctx->device];
    }
    if (!part)
        return Error{PGCP_E_HIP, std::string("scratch address of this device not set up: ") +
                                     hipGetErrorString(g_scratch_err[ctx->device])};
    hipStream_t s = ctx->stream;
    const int64_t nblk = (nf + BLOCK - 1) / BLOCK;
    DistPart* fin = part + kNoAllocBlocks;
    // every record k_dist_final reads ([0, nblk)) is written by k_distortion
    // first, so nothing needs clearing between calls
    k_distortion<<<(unsigned)nblk, BLOCK, 0, s>>>(nf, V, F, X, dim, d, mu, flip, part);
    HIPCHK(hipGetLastError());
    k_dist_final<<<1, BLOCK, 0, s>>>(nblk, part, fin);
    HIPCHK(hipGetLastError());
    if (st) {
        DistPart h;
        HIPCHK(hipMemcpyAsync(&h, fin, sizeof(DistPart), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double n = 3.0 * (double)nf;
        st->mean_abs_d = h.sum / n;
        st->sd_abs_d = n > 1 ? std::sqrt(std::max(0.0, (h.sum2 - h.sum * h.sum / n) / (n - 1.0))) : 0.0;
        st->max_abs_d = h.maxd;
        st->median_abs_d = NAN;
        st->iqr_abs_d = NAN;
        st->max_mu = h.maxmu;
        st->n_flipped = (int64_t)llround(h.nflip);
        st->n_mu_ge1 = (int64_t)llround(h.nmu1);
    }
    return Error{PGCP_OK, ""};
}

// Distortion check.  Scratch buffers live in the context-independent statics
// of this call (allocated per call size).
Error run_distortion(pgcp_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf, const double* X,
                     int dim, double* d, double* mu, uint8_t* flip, int want_q, pgcp_dist_stats* st) {
    (void)nv;
    hipStream_t s = ctx->stream;
    const int64_t nblk = (nf + BLOCK - 1) / BLOCK;
    DevBuf part, fin, dtmp, qsel;
    Error e{PGCP_OK, ""};
    if ((e = dev_alloc(part, nblk * sizeof(DistPart))).code) return e;
    if ((e = dev_alloc(fin, sizeof(DistPart))).code) return e;
    double* dd = d;
    if (want_q && !dd) {
        if ((e = dev_alloc(dtmp, nf * 3 * 8)).code) return e;
        dd = (double*)dtmp.p;
    }
    k_distortion<<<(unsigned)nblk, BLOCK, 0, s>>>(nf, V, F, X, dim, dd, mu, flip, (DistPart*)part.p);
    HIPCHK(hipGetLastError());
    k_dist_final<<<1, BLOCK, 0, s>>>(nblk, (const DistPart*)part.p, (DistPart*)fin.p);
    HIPCHK(hipGetLastError());
    double med = NAN, iqr = NAN;
    if (want_q) {
        // midpoint-rule percentiles: position q*n + 1/2 (1-based), linear
        // between its two neighbours in sorted order; the six order
        // statistics come from one radix select
        const int64_t n = 3 * nf;
        const double qv[3] = {0.25, 0.50, 0.75};
        QSelState h0{};
        double tpos[3];
        for (int j = 0; j < 3; ++j) {
            const double pos = qv[j] * (double)n + 0.5;
            const int64_t lo = (int64_t)std::floor(pos);
            tpos[j] = pos;
            h0.rank[2 * j] = std::min<int64_t>(std::max<int64_t>(lo, 1), n) - 1;
            h0.rank[2 * j + 1] = std::min<int64_t>(std::max<int64_t>(lo + 1, 1), n) - 1;
        }
        const size_t hist_bytes = kQSelMax * 256 * sizeof(unsigned);
        if ((e = dev_alloc(qsel, sizeof(QSelState) + hist_bytes + kQSelMax * sizeof(double))).code) return e;
        QSelState* qs = (QSelState*)qsel.p;
        unsigned* hist = (unsigned*)((char*)qsel.p + sizeof(QSelState));
        double* qout = (double*)((char*)hist + hist_bytes);
        HIPCHK(hipMemcpyAsync(qs, &h0, sizeof(QSelState), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemsetAsync(hist, 0, hist_bytes, s));
        const unsigned g = (unsigned)std::min<int64_t>((n + BLOCK - 1) / BLOCK, kQSelGrid);
        for (int shift = 56; shift >= 0; shift -= 8) {
            k_qsel_hist<<<g, BLOCK, 0, s>>>(n, dd, kQSelMax, shift, qs, hist);
            HIPCHK(hipGetLastError());
            k_qsel_pick<<<1, 256, 0, s>>>(kQSelMax, shift, qs, hist, qout);
            HIPCHK(hipGetLastError());
        }
        double v[kQSelMax];
        HIPCHK(hipMemcpyAsync(v, qout, sizeof(v), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double p[3];
        for (int j = 0; j < 3; ++j) {
            const double pos = tpos[j], t = pos - std::floor(pos);
            const double v0 = v[2 * j], v1 = v[2 * j + 1];
            p[j] = pos <= 1.0 ? v0 : pos >= (double)n ? v1 : v0 + t * (v1 - v0);
        }
        med = p[1];
        iqr = p[2] - p[0];
    }
    if (st) {
        DistPart h;
        HIPCHK(hipMemcpyAsync(&h, fin.p, sizeof(DistPart), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double n = 3.0 * (double)nf;
        st->mean_abs_d = h.sum / n;
        st->sd_abs_d = n > 1 ? std::sqrt(std::max(0.0, (h.sum2 - h.sum * h.sum / n) / (n - 1.0))) : 0.0;
        st->max_abs_d = h.maxd;
        st->median_abs_d = med;
        st->iqr_abs_d = iqr;
        st->max_mu = h.maxmu;
        st->n_flipped = (int64_t)llround(h.nflip);
        st->n_mu_ge1 = (int64_t)llround(h.nmu1);
    }
    HIPCHK(hipStreamSynchronize(s));
    dev_free(part);
    dev_free(fin);
    dev_free(dtmp);
    dev_free(qsel);
    return Error{PGCP_OK, ""};
}

Error assembled_ok(pgcp_ctx* ctx, pgcp_part* P) {
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, P->d_flags.p, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (bad) return Error{PGCP_E_DEGENERATE, "zero-area triangle in assembly"};
    return Error{PGCP_OK, ""};
}

}  // namespace pgcp

namespace pgcp {

// Copy one piece's FP64 matrix back to host CSR (local indices = ranks of the
// global vertices, diagonal included).
Error export_laplacian(pgcp_ctx* ctx, const pgcp_part* P, int piece, int32_t* rowptr, int32_t* col, double* val) {
    const int32_t r0 = P->row0[piece];
    const int32_t n = P->sub_nv[piece];
    const int64_t s0 = r0 / 64, s1 = (r0 + (int64_t)n + 63) / 64;
    const int64_t e0 = P->sl_ptr[s0], e1 = P->sl_ptr[s1];
    std::vector<double> v(e1 - e0), dg(n);
    HIPCHK(hipMemcpyAsync(v.data(), (const double*)P->d_val64.p + e0, (e1 - e0) * 8, hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipMemcpyAsync(dg.data(), (const double*)P->d_diag64.p + r0, (size_t)n * 8, hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::vector<int32_t> by_rank, rank_of;
    piece_global_order(P, piece, by_rank, rank_of);
    rowptr[0] = 0;
    std::vector<std::pair<int32_t, double>> ent;
    for (int32_t t = 0; t < n; ++t) {
        const int32_t l = by_rank[t];
        const int64_t r = r0 + l, s = r / 64;
        const int lane = (int)(r & 63);
        ent.clear();
        ent.emplace_back(t, dg[l]);
        for (int k = 0; k < P->sl_w[s]; ++k) {
            const int64_t el = P->sl_ptr[s] + (int64_t)k * 64 + lane;
            const int32_t c = P->sl_col[el];
            if (c == r) continue;   // padding slot
            ent.emplace_back(rank_of[c - r0], v[el - e0]);
        }
        std::sort(ent.begin(), ent.end());
        rowptr[t + 1] = rowptr[t] + (int32_t)ent.size();
        if (col && val) {
            for (size_t q = 0; q < ent.size(); ++q) {
                col[rowptr[t] + q] = ent[q].first;
                val[rowptr[t] + q] = ent[q].second;
            }
        }
    }
    return Error{PGCP_OK, ""};
}

}  // namespace pgcp

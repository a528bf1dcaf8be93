// Internal declarations shared by the host (C++) and device (HIP) parts of libpgcp.
#pragma once

#include <algorithm>
#include <complex>
#include <array>
#include <map>
#include <cstdint>
#include <string>
#include <memory>
#include <type_traits>
#include <utility>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/pgcp.h"

namespace pgcp {

using cplx = std::complex<double>;

// Allocator whose new elements are default-initialised (no zero fill): the
// plan's large arrays are written in parallel right after they are sized, and
// a serial zero fill of tens of MB would cost more than writing them.
template <class T>
struct NoFillAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = NoFillAlloc<U>;
    };
    NoFillAlloc() = default;
    template <class U>
    NoFillAlloc(const NoFillAlloc<U>&) noexcept {}
    template <class U>
    void construct(U* p) noexcept(std::is_nothrow_default_constructible<U>::value) {
        ::new ((void*)p) U;
    }
    template <class U, class... A>
    void construct(U* p, A&&... a) {
        ::new ((void*)p) U(std::forward<A>(a)...);
    }
};
template <class T>
using bigvec = std::vector<T, NoFillAlloc<T>>;

// Error carried from internal code to the C ABI.
struct Error {
    pgcp_status code;
    std::string msg;
};

// Device buffer owned by a plan or context.  Buffers made inside a context's
// call come from the device's stream-ordered pool (hipMallocAsync on the
// context's stream) and go back to it with hipFreeAsync, so neither waits for
// work on other streams: a plain hipFree waits for the whole device, which
// would serialise contexts that run meshes side by side on their own streams.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipStream_t s = nullptr;   // stream of the allocation (pooled buffers)
    bool pooled = false;
};

// Stream that the calling thread's allocations and releases are ordered on;
// set for the duration of an entry point from the context (or plan) it works on.
inline thread_local bool tls_alloc_set = false;
inline thread_local hipStream_t tls_alloc_stream = nullptr;

struct AllocScope {
    bool prev_set;
    hipStream_t prev;
    explicit AllocScope(hipStream_t s) : prev_set(tls_alloc_set), prev(tls_alloc_stream) {
        tls_alloc_set = true;
        tls_alloc_stream = s;
    }
    ~AllocScope() {
        tls_alloc_set = prev_set;
        tls_alloc_stream = prev;
    }
    AllocScope(const AllocScope&) = delete;
    AllocScope& operator=(const AllocScope&) = delete;
};

// A device-side work assignment for the persistent batched CG: each workgroup
// owns a contiguous range of 64-row slices of exactly one piece.
struct WorkMap {
    int blk = 0;                 // threads per workgroup
    int rows_per_thread = 0;     // 64-row slices per wave (register-resident kernel)
    int stream = 0;              // 1: vectors stream through memory, any number of slices per wave
    int n_xcd = 1;
    int n_wg = 0;                // grid size (0 = not built)
    int n_partials = 0;
    std::vector<int32_t> wg_sub, wg_rank, wg_s0, wg_s1;   // per workgroup
    std::vector<int32_t> sub_pbase, sub_nwg;              // per piece
    DevBuf d_wg_sub, d_wg_rank, d_wg_s0, d_wg_s1, d_sub_pbase, d_sub_nwg;
    // register-resident kernel: local numbering of each workgroup's rows and halo
    size_t lds_bytes = 0;        // dynamic LDS per workgroup
    int lds_n = 0;               // LDS entries of one vector: own rows + largest ring 1
    DevBuf d_wg_h0, d_halo, d_lcol, d_lpn, d_wg_n1, d_rcol, d_expo;
    // single-reduction kernel (both rings): usable, its LDS and vector sizes
    bool cg1 = false;
    size_t lds1_bytes = 0;
    int lds_nr = 0, lds_nu = 0;
};

}  // namespace pgcp

// Opaque handles of the C ABI.
struct pgcp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_cu = 0;
    std::string last_error;
};

struct pgcp_part {
    int64_t nv = 0, nf = 0;
    int K = 0;
    int mode = 0;
    int64_t N = 0;          // packed rows (pieces padded to multiples of 64)
    int64_t nslices = 0;    // N / 64
    int64_t n_bdy = 0, n_seam = 0, nnz_off = 0, sell_elems = 0;

    // ---------------- host plan
    std::vector<int32_t> face_sub;            // [nf]
    std::vector<int32_t> sub_nv, sub_nf;      // [K]
    std::vector<int64_t> sub_nnz;             // [K] off-diagonal entries of each piece
    std::vector<int32_t> row0;                // [K+1]
    std::vector<int32_t> row_gv;              // [N]  -1 = padding row
    std::vector<int32_t> row_prev, row_next;  // [N]  CCW loop neighbours (packed rows), -1 inside
    std::vector<uint8_t> row_kind;            // [N]  0 interior, 1 boundary loop, 2 padding
    std::vector<int32_t> slice_sub;           // [nslices]
    std::vector<int64_t> sl_ptr;              // [nslices+1] first element of each slice
    std::vector<int32_t> sl_w;                // [nslices] slice width (max off-diagonals per row)
    pgcp::bigvec<int32_t> sl_col;                 // [sell_elems] packed column; padding = own row
    pgcp::bigvec<int32_t> sl_opp;                 // [2*sell_elems] opposite vertices (global ids) or -1
    pgcp::bigvec<int32_t> sl_rev;                 // [sell_elems] slot of the reverse entry, -1 for padding
    pgcp::bigvec<uint8_t> sl_ori;                 // [sell_elems] bit t: (row, column, opposite t) is that
                                                  // face's own (counter-clockwise) vertex order
    std::vector<int32_t> pin_row;             // [2K] DNCP pins p0, p1 (packed rows)
    std::vector<double> pin_x1;               // [K] x coordinate of p1 (|v_p1 - v_p0|)
    std::vector<int32_t> loop_ptr;            // [K+1]
    std::vector<int32_t> loop_gv, loop_row, loop_seam;   // [n_bdy]
    std::vector<int32_t> seam_gv;             // [n_seam]
    std::vector<std::vector<std::pair<int, int>>> weld_rounds;

    // ---------------- device mirrors
    pgcp::DevBuf d_row_gv, d_row_prev, d_row_next, d_row_kind, d_slice_sub;
    pgcp::DevBuf d_sl_ptr, d_sl_w, d_sl_col, d_sl_opp, d_sl_rev, d_sl_ori;
    pgcp::DevBuf d_val64, d_val32, d_diag64, d_diag32;
    pgcp::DevBuf d_pin_row, d_pin_x1, d_loop_ptr, d_loop_row, d_loop_seam, d_seam_gv;
    pgcp::DevBuf d_mask_dncp, d_mask_harm;    // [N] uint8: 1 = Dirichlet row
    pgcp::DevBuf d_chart;                     // [3K] doubles: sphere chart centre (re, im, is-infinity)

    // ---------------- solver work space
    pgcp::DevBuf d_u64, d_r64, d_e, d_r, d_z, d_p0, d_p1, d_q, d_r2, d_s1;
    pgcp::DevBuf d_partial, d_bar, d_gen, d_res, d_subinfo, d_bnorm, d_rnorm, d_iters, d_flags;
    pgcp::DevBuf d_row0, d_slicepart, d_scale, d_target, d_active, d_status, d_rrout, d_abort;
    pgcp::DevBuf d_cgs;                       // [K][16] scalar state of pieces paused between phases
    pgcp::DevBuf d_distpart, d_diststat, d_absd, d_sorttmp;
    // quasi-conformal fold repair: Beltrami-solver matrix, face -> piece, per-piece counts
    pgcp::DevBuf d_lbs_val64, d_lbs_val32, d_lbs_diag64, d_lbs_diag32, d_face_sub, d_fold_cnt, d_fold_prev;
    pgcp::WorkMap wmap32, wmap64;

    // ---------------- learned preconditioner (network states, SPAI values, training work space)
    int spai_sys = -1;                        // system whose SPAI values are current, -1 = none
    pgcp::DevBuf d_lpc_val, d_lpc_h, d_lpc_e, d_lpc_oe, d_lpc_ov;
    pgcp::DevBuf d_mval32, d_mdiag32, d_mval64, d_mdiag64;
    pgcp::DevBuf d_lpc_av, d_lpc_R, d_lpc_sp, d_lpc_piece, d_lpc_c, d_lpc_goe, d_lpc_gov;
    pgcp::DevBuf d_lpc_dh, d_lpc_dhown, d_lpc_de0, d_lpc_de1, d_lpc_dx, d_pc;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t stream = nullptr;   // stream of the context that last worked on the plan

    bool assembled = false;
    int solved = -1;        // system of the last solve whose iterate d_u64 holds (-1: none)
    bool welded = false;
    bool host_only = false;
};

// Learned preconditioner: fp32 master parameters, Adam moments, the bf16
// weight blocks the kernels read, and gradient work space.
struct pgcp_lpc {
    int device = 0;
    pgcp::DevBuf theta, adam_m, adam_v, wb, grad, gp;
    int64_t step = 0;
};

namespace pgcp {

// weld with the point replay on the device (weld_dev.hip)
Error weld_all_device(pgcp_ctx* ctx, pgcp_part* P, const double* bdy_uv, double* welded_uv);

// learned preconditioner (lpc.hip)
int64_t lpc_num_params();
Error lpc_create(pgcp_ctx* ctx, const float* params, pgcp_lpc** out);
void lpc_destroy(pgcp_lpc* L);
Error lpc_get_params(pgcp_ctx* ctx, const pgcp_lpc* L, float* out);
Error lpc_save(pgcp_ctx* ctx, const pgcp_lpc* L, const char* path);
Error lpc_load(pgcp_ctx* ctx, const char* path, pgcp_lpc** out);
Error lpc_infer(pgcp_ctx* ctx, pgcp_part* P, const pgcp_lpc* L, int system);
Error lpc_export(pgcp_ctx* ctx, const pgcp_part* P, int piece, double* o_off, double* o_diag, double* m_off,
                 double* m_diag);
Error lpc_grad(pgcp_ctx* ctx, pgcp_part* P, pgcp_lpc* L, int system, const float* probes, int n_probes,
               double* loss, float* grad_host, int adam, float lr);
void lpc_free_part(pgcp_part* P);

// host plan (partition.cpp)
Error build_plan(pgcp_part* part, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                 const int32_t* label, int mode);

// weld (weld.cpp)
int shared_arc(const std::vector<int>& la, const std::vector<int>& lb, int* start);
Error merge_plan(const std::vector<std::vector<int>>& loops, const std::vector<int64_t>& sizes,
                 int mode, std::vector<std::vector<std::pair<int, int>>>* rounds);
Error weld_all(pgcp_part* part, const double* bdy_uv, double* welded_uv);

// A piece's packed rows by ascending global vertex: row row0 + by_rank[t]
// holds the piece's t-th smallest global vertex, rank_of is the inverse.  The
// exports list a piece in this order whatever order its rows are packed in.
inline void piece_global_order(const pgcp_part* P, int piece, std::vector<int32_t>& by_rank,
                               std::vector<int32_t>& rank_of) {
    const int32_t r0 = P->row0[piece], n = P->sub_nv[piece];
    by_rank.resize(n);
    rank_of.resize(n);
    for (int32_t l = 0; l < n; ++l) by_rank[l] = l;
    std::sort(by_rank.begin(), by_rank.end(),
              [&](int32_t a, int32_t b) { return P->row_gv[r0 + a] < P->row_gv[r0 + b]; });
    for (int32_t t = 0; t < n; ++t) rank_of[by_rank[t]] = t;
}

// device side (device.hip)
Error upload_plan(pgcp_ctx* ctx, pgcp_part* part);
void free_part_device(pgcp_part* part);
Error launch_assemble(pgcp_ctx* ctx, pgcp_part* P, const double* V);
Error assembled_ok(pgcp_ctx* ctx, pgcp_part* P);
Error export_laplacian(pgcp_ctx* ctx, const pgcp_part* P, int piece, int32_t* rowptr, int32_t* col,
                       double* val);
Error run_local_param(pgcp_ctx* ctx, pgcp_part* P, const pgcp_solve_opts* o, double* bdy,
                      pgcp_solve_stats* st);
Error run_harmonic(pgcp_ctx* ctx, pgcp_part* P, const double* welded, const pgcp_solve_opts* o,
                   double* out, pgcp_solve_stats* st);
Error run_fold_repair(pgcp_ctx* ctx, pgcp_part* P, const int32_t* F, const double* V, double* X, double delta,
                      int max_passes, const pgcp_solve_opts* o, pgcp_fold_stats* fs);
Error noalloc_scratch_init(int device);
int64_t noalloc_max_faces();
Error run_distortion_noalloc(pgcp_ctx* ctx, const double* V, const int32_t* F, int64_t nf, const double* X,
                             int dim, double* d, double* mu, uint8_t* flip, pgcp_dist_stats* st);
Error run_distortion(pgcp_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                     const double* X, int dim, double* d, double* mu, uint8_t* flip, int want_q,
                     pgcp_dist_stats* st);

// area distortion (area.hip)
Error run_area_distortion(pgcp_ctx* ctx, const double* V, const int32_t* F, int64_t nf, const double* X, int dim,
                          double* d, double* mean_abs);
Error run_area_objective(pgcp_ctx* ctx, const double* V, const int32_t* F, int64_t nf, const double* X, int mode,
                         const double* params, double* value);
Error run_area_mobius_opt(pgcp_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf, const double* X,
                          int mode, int max_evals, double* params, double* before, double* after, int32_t* n_evals,
                          double* Y);

}  // namespace pgcp

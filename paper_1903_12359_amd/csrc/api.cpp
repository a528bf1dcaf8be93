// C ABI of libpgcp: argument checks, error strings and timing around the
// host (partition, weld) and device (assembly, solves, distortion) stages.
// Every entry point that does work opens a roctx range named after itself, so
// `rocprofv3 --marker-trace` shows each call beside the kernels it launched.

#include <rocprofiler-sdk-roctx/roctx.h>

#include <chrono>
#include <cstdlib>
#include <cstring>
#include <new>

#include "pgcp_internal.h"

using pgcp::Error;

extern "C" void kmp_set_defaults(char const* str);   // LLVM OpenMP runtime

namespace {

// Host stages run OpenMP regions from several threads at once (a partition
// worker and the solve lanes of a stream, each with a team of its own): idle
// team members must go to sleep soon instead of spinning for the runtime's
// default 200 ms, or they take the cores the other teams need.  An explicit
// KMP_BLOCKTIME in the environment wins.
struct OmpDefaults {
    OmpDefaults() {
        if (!getenv("KMP_BLOCKTIME")) kmp_set_defaults("KMP_BLOCKTIME=1");
    }
} omp_defaults;

pgcp_status fail(pgcp_ctx* ctx, const Error& e) {
    if (ctx && e.code != PGCP_OK) ctx->last_error = e.msg;
    return e.code;
}

pgcp_status bad(pgcp_ctx* ctx, const char* m) { return fail(ctx, Error{PGCP_E_INVALID, m}); }

// message of the last failure of a call made without a context on this
// thread (context creation), read by pgcp_last_error(NULL)
thread_local std::string no_ctx_error = "no context";

pgcp_status no_ctx_fail(pgcp_status code, const std::string& msg) {
    no_ctx_error = msg;
    return code;
}

// roctx range over one entry point (a no-op unless a tool is attached)
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

pgcp_status pgcp_ctx_create(pgcp_ctx** out, int hip_device, void* hip_stream) {
    if (!out) return no_ctx_fail(PGCP_E_INVALID, "null output pointer");
    *out = nullptr;
    int n = 0;
    hipError_t rc = hipGetDeviceCount(&n);
    if (rc != hipSuccess) return no_ctx_fail(PGCP_E_HIP, std::string("hipGetDeviceCount: ") + hipGetErrorString(rc));
    if (hip_device < 0 || hip_device >= n)
        return no_ctx_fail(PGCP_E_HIP, "device " + std::to_string(hip_device) + " of " + std::to_string(n));
    rc = hipSetDevice(hip_device);
    if (rc != hipSuccess) return no_ctx_fail(PGCP_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(rc));
    pgcp_ctx* c = new (std::nothrow) pgcp_ctx();
    if (!c) return no_ctx_fail(PGCP_E_NOMEM, "out of host memory");
    c->device = hip_device;
    c->stream = (hipStream_t)hip_stream;
    (void)hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, hip_device);
    // device address of the fixed scratch array of pgcp_distortion_noalloc,
    // once per device, with the device current (a failure is reported by that
    // entry point; every other call works without the array)
    (void)pgcp::noalloc_scratch_init(hip_device);
    // keep released pool memory for reuse instead of returning it at every
    // synchronisation (plans of a stream of meshes reuse the same sizes)
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, hip_device) == hipSuccess && pool) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    *out = c;
    return PGCP_OK;
}

void pgcp_ctx_destroy(pgcp_ctx* ctx) { delete ctx; }

const char* pgcp_last_error(const pgcp_ctx* ctx) { return ctx ? ctx->last_error.c_str() : no_ctx_error.c_str(); }

pgcp_status pgcp_ctx_set_stream(pgcp_ctx* ctx, void* hip_stream) {
    if (!ctx) return PGCP_E_INVALID;
    ctx->stream = (hipStream_t)hip_stream;
    return PGCP_OK;
}

pgcp_status pgcp_partition(pgcp_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                           const int32_t* label, int32_t mode, pgcp_part** out) {
    Range range("pgcp_partition");
    if (!V || !F || !label || !out) return bad(ctx, "null argument");
    *out = nullptr;
    pgcp_part* P = new (std::nothrow) pgcp_part();
    if (!P) return fail(ctx, Error{PGCP_E_NOMEM, "out of host memory"});
    Error e{PGCP_OK, ""};
    try {
        e = pgcp::build_plan(P, V, nv, F, nf, label, mode);
    } catch (const std::bad_alloc&) {
        e = Error{PGCP_E_NOMEM, "out of host memory"};
    }
    if (e.code == PGCP_OK && ctx) {
        P->stream = ctx->stream;
        pgcp::AllocScope scope(ctx->stream);
        if (hipSetDevice(ctx->device) != hipSuccess) e = Error{PGCP_E_HIP, "hipSetDevice failed"};
        else e = pgcp::upload_plan(ctx, P);
        if (e.code == PGCP_OK && hipStreamSynchronize(ctx->stream) != hipSuccess)
            e = Error{PGCP_E_HIP, "plan upload failed"};
    }
    if (e.code != PGCP_OK) {
        pgcp::AllocScope scope(P->stream);
        pgcp::free_part_device(P);
        delete P;
        if (!ctx) return e.code;
        return fail(ctx, e);
    }
    P->host_only = ctx == nullptr;
    *out = P;
    return PGCP_OK;
}

pgcp_status pgcp_part_query(const pgcp_part* P, pgcp_part_info* info) {
    if (!P || !info) return PGCP_E_INVALID;
    std::memset(info, 0, sizeof(*info));
    info->nv = P->nv;
    info->nf = P->nf;
    info->n_sub = P->K;
    info->mode = P->mode;
    info->n_rows = P->N;
    info->n_bdy = P->n_bdy;
    info->n_seam = P->n_seam;
    info->nnz_offdiag = P->nnz_off;
    info->sell_elems = P->sell_elems;
    info->weld_rounds = (int32_t)P->weld_rounds.size();
    return PGCP_OK;
}

pgcp_status pgcp_part_export(const pgcp_part* P, int32_t* face_sub, int32_t* sub_nv, int32_t* loop_ptr,
                             int32_t* loop_gv, int32_t* seam_gv) {
    if (!P) return PGCP_E_INVALID;
    if (face_sub) std::memcpy(face_sub, P->face_sub.data(), P->face_sub.size() * 4);
    if (sub_nv) std::memcpy(sub_nv, P->sub_nv.data(), P->sub_nv.size() * 4);
    if (loop_ptr) std::memcpy(loop_ptr, P->loop_ptr.data(), P->loop_ptr.size() * 4);
    if (loop_gv) std::memcpy(loop_gv, P->loop_gv.data(), P->loop_gv.size() * 4);
    if (seam_gv) std::memcpy(seam_gv, P->seam_gv.data(), P->seam_gv.size() * 4);
    return PGCP_OK;
}

void pgcp_part_destroy(pgcp_part* P) {
    if (!P) return;
    pgcp::AllocScope scope(P->stream);
    pgcp::free_part_device(P);
    delete P;
}

pgcp_status pgcp_assemble_cotan(pgcp_ctx* ctx, pgcp_part* P, const double* V_dev) {
    Range range("pgcp_assemble_cotan");
    if (!ctx || !P || !V_dev) return bad(ctx, "null argument");
    if (P->host_only) return bad(ctx, "host-only plan");
    pgcp::AllocScope scope(ctx->stream);
    P->stream = ctx->stream;
    return fail(ctx, pgcp::launch_assemble(ctx, P, V_dev));
}

pgcp_status pgcp_local_param(pgcp_ctx* ctx, pgcp_part* P, const pgcp_solve_opts* opts, double* bdy_uv_dev,
                             pgcp_solve_stats* stats) {
    Range range("pgcp_local_param");
    if (!ctx || !P || !bdy_uv_dev) return bad(ctx, "null argument");
    if (P->host_only) return bad(ctx, "host-only plan");
    pgcp::AllocScope scope(ctx->stream);
    P->stream = ctx->stream;
    double t0 = now();
    if (!P->assembled) return bad(ctx, "pgcp_assemble_cotan has not run");
    Error e = pgcp::assembled_ok(ctx, P);
    if (e.code == PGCP_OK) e = pgcp::run_local_param(ctx, P, opts, bdy_uv_dev, stats);
    if (stats) {
        (void)hipStreamSynchronize(ctx->stream);
        stats->seconds = now() - t0;
    }
    return fail(ctx, e);
}

pgcp_status pgcp_weld(pgcp_ctx* ctx, pgcp_part* P, const double* bdy_uv_host, double* welded_uv_host) {
    Range range("pgcp_weld");
    if (!P || !bdy_uv_host || !welded_uv_host) return bad(ctx, "null argument");
    if (ctx && !P->host_only) {
        pgcp::AllocScope scope(ctx->stream);
        P->stream = ctx->stream;
        return fail(ctx, pgcp::weld_all_device(ctx, P, bdy_uv_host, welded_uv_host));
    }
    return fail(ctx, pgcp::weld_all(P, bdy_uv_host, welded_uv_host));
}

pgcp_status pgcp_laplacian_export(pgcp_ctx* ctx, const pgcp_part* P, int32_t piece, int32_t* rowptr,
                                  int32_t* col, double* val) {
    Range range("pgcp_laplacian_export");
    if (!ctx || !P || !rowptr) return bad(ctx, "null argument");
    if (P->host_only || !P->assembled) return bad(ctx, "plan has no assembled device matrix");
    if (piece < 0 || piece >= P->K) return bad(ctx, "piece out of range");
    pgcp::AllocScope scope(ctx->stream);
    return fail(ctx, pgcp::export_laplacian(ctx, P, piece, rowptr, col, val));
}

pgcp_status pgcp_harmonic_solve(pgcp_ctx* ctx, pgcp_part* P, const double* welded_uv_dev,
                                const pgcp_solve_opts* opts, double* out_dev, pgcp_solve_stats* stats) {
    Range range("pgcp_harmonic_solve");
    if (!ctx || !P || !welded_uv_dev || !out_dev) return bad(ctx, "null argument");
    if (P->host_only) return bad(ctx, "host-only plan");
    pgcp::AllocScope scope(ctx->stream);
    P->stream = ctx->stream;
    double t0 = now();
    Error e = pgcp::run_harmonic(ctx, P, welded_uv_dev, opts, out_dev, stats);
    if (stats) {
        (void)hipStreamSynchronize(ctx->stream);
        stats->seconds = now() - t0;
    }
    return fail(ctx, e);
}

pgcp_status pgcp_fold_repair(pgcp_ctx* ctx, pgcp_part* P, const double* V_dev, const int32_t* F_dev,
                             double* param_dev, double delta, int32_t max_passes, const pgcp_solve_opts* opts,
                             pgcp_fold_stats* stats) {
    Range range("pgcp_fold_repair");
    if (!ctx || !P || !V_dev || !F_dev || !param_dev) return bad(ctx, "null argument");
    if (P->host_only) return bad(ctx, "host-only plan");
    pgcp::AllocScope scope(ctx->stream);
    P->stream = ctx->stream;
    return fail(ctx, pgcp::run_fold_repair(ctx, P, F_dev, V_dev, param_dev, delta, max_passes, opts, stats));
}

pgcp_status pgcp_distortion(pgcp_ctx* ctx, const double* V_dev, int64_t nv, const int32_t* F_dev, int64_t nf,
                            const double* param_dev, int32_t dim, double* d_dev, double* mu_dev, uint8_t* flip_dev,
                            int32_t want_quantiles, pgcp_dist_stats* stats) {
    Range range("pgcp_distortion");
    if (!ctx || !V_dev || !F_dev || !param_dev) return bad(ctx, "null argument");
    if (dim != 2 && dim != 3) return bad(ctx, "dim must be 2 or 3");
    if (nf <= 0 || nv <= 0) return bad(ctx, "empty mesh");
    pgcp::AllocScope scope(ctx->stream);
    return fail(ctx, pgcp::run_distortion(ctx, V_dev, nv, F_dev, nf, param_dev, dim, d_dev, mu_dev, flip_dev,
                                          want_quantiles, stats));
}

pgcp_status pgcp_distortion_noalloc(pgcp_ctx* ctx, const double* V_dev, int64_t nv, const int32_t* F_dev,
                                    int64_t nf, const double* param_dev, int32_t dim, double* d_dev, double* mu_dev,
                                    uint8_t* flip_dev, pgcp_dist_stats* stats) {
    // the size limit is checked first, so that it holds whatever else is wrong
    if (nf > pgcp::noalloc_max_faces()) return bad(ctx, "nf exceeds pgcp_distortion_noalloc's fixed scratch array");
    if (!ctx || !V_dev || !F_dev || !param_dev) return bad(ctx, "null argument");
    if (dim != 2 && dim != 3) return bad(ctx, "dim must be 2 or 3");
    if (nf <= 0 || nv <= 0) return bad(ctx, "empty mesh");
    return fail(ctx, pgcp::run_distortion_noalloc(ctx, V_dev, F_dev, nf, param_dev, dim, d_dev, mu_dev, flip_dev,
                                                  stats));
}

int64_t pgcp_distortion_noalloc_max_faces(void) { return pgcp::noalloc_max_faces(); }

static pgcp_status area_args(pgcp_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                             const double* X, int32_t dim) {
    if (!ctx || !V || !F || !X) return bad(ctx, "null argument");
    if (dim != 2 && dim != 3) return bad(ctx, "dim must be 2 or 3");
    if (nf <= 0 || nv <= 0) return bad(ctx, "empty mesh");
    return PGCP_OK;
}

static pgcp_status area_mode(pgcp_ctx* ctx, int32_t mode, int32_t dim) {
    if (mode != PGCP_FREE && mode != PGCP_DISK && mode != PGCP_SPHERE) return bad(ctx, "unknown mode");
    if ((mode == PGCP_SPHERE) != (dim == 3)) return bad(ctx, "sphere mode takes dim 3, free and disk dim 2");
    return PGCP_OK;
}

pgcp_status pgcp_area_distortion(pgcp_ctx* ctx, const double* V_dev, int64_t nv, const int32_t* F_dev, int64_t nf,
                                 const double* param_dev, int32_t dim, double* d_dev, double* mean_abs) {
    Range range("pgcp_area_distortion");
    pgcp_status r = area_args(ctx, V_dev, nv, F_dev, nf, param_dev, dim);
    if (r != PGCP_OK) return r;
    if (!mean_abs) return bad(ctx, "null argument");
    pgcp::AllocScope scope(ctx->stream);
    return fail(ctx, pgcp::run_area_distortion(ctx, V_dev, F_dev, nf, param_dev, dim, d_dev, mean_abs));
}

pgcp_status pgcp_area_objective(pgcp_ctx* ctx, const double* V_dev, int64_t nv, const int32_t* F_dev, int64_t nf,
                                const double* param_dev, int32_t dim, int32_t mode, const double* mobius,
                                double* value) {
    Range range("pgcp_area_objective");
    pgcp_status r = area_args(ctx, V_dev, nv, F_dev, nf, param_dev, dim);
    if (r != PGCP_OK) return r;
    if ((r = area_mode(ctx, mode, dim)) != PGCP_OK) return r;
    if (!mobius || !value) return bad(ctx, "null argument");
    pgcp::AllocScope scope(ctx->stream);
    return fail(ctx, pgcp::run_area_objective(ctx, V_dev, F_dev, nf, param_dev, mode, mobius, value));
}

pgcp_status pgcp_area_mobius_opt(pgcp_ctx* ctx, const double* V_dev, int64_t nv, const int32_t* F_dev, int64_t nf,
                                 const double* param_dev, int32_t dim, int32_t mode, int32_t max_evals,
                                 double* mobius, double* before, double* after, int32_t* n_evals, double* out_dev) {
    Range range("pgcp_area_mobius_opt");
    pgcp_status r = area_args(ctx, V_dev, nv, F_dev, nf, param_dev, dim);
    if (r != PGCP_OK) return r;
    if ((r = area_mode(ctx, mode, dim)) != PGCP_OK) return r;
    if (!mobius || !before || !after) return bad(ctx, "null argument");
    if (max_evals < 1) return bad(ctx, "max_evals must be positive");
    pgcp::AllocScope scope(ctx->stream);
    return fail(ctx, pgcp::run_area_mobius_opt(ctx, V_dev, nv, F_dev, nf, param_dev, mode, max_evals, mobius, before,
                                               after, n_evals, out_dev));
}

}  // extern "C"

extern "C" {

int64_t pgcp_lpc_num_params(void) { return pgcp::lpc_num_params(); }

pgcp_status pgcp_lpc_create(pgcp_ctx* ctx, const float* params_host, pgcp_lpc** out) {
    Range range("pgcp_lpc_create");
    if (!ctx || !out) return bad(ctx, "null argument");
    *out = nullptr;
    pgcp::AllocScope scope(ctx->stream);
    return fail(ctx, pgcp::lpc_create(ctx, params_host, out));
}

pgcp_status pgcp_lpc_get_params(pgcp_ctx* ctx, const pgcp_lpc* lpc, float* params_host) {
    Range range("pgcp_lpc_get_params");
    if (!ctx || !lpc || !params_host) return bad(ctx, "null argument");
    pgcp::AllocScope scope(ctx->stream);
    return fail(ctx, pgcp::lpc_get_params(ctx, lpc, params_host));
}

pgcp_status pgcp_part_solution(pgcp_ctx* ctx, const pgcp_part* P, int32_t* system, double* out_dev) {
    Range range("pgcp_part_solution");
    if (!ctx || !P || !out_dev) return bad(ctx, "null argument");
    if (P->host_only || P->solved < 0 || !P->d_u64.p) return bad(ctx, "no solve has run on this plan");
    if (system) *system = P->solved;
    if (hipMemcpyAsync(out_dev, P->d_u64.p, (size_t)P->N * 16, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess)
        return fail(ctx, Error{PGCP_E_HIP, "solution copy failed"});
    return PGCP_OK;
}

pgcp_status pgcp_lpc_save(pgcp_ctx* ctx, const pgcp_lpc* lpc, const char* path) {
    Range range("pgcp_lpc_save");
    if (!ctx || !lpc || !path) return bad(ctx, "null argument");
    pgcp::AllocScope scope(ctx->stream);
    return fail(ctx, pgcp::lpc_save(ctx, lpc, path));
}

pgcp_status pgcp_lpc_load(pgcp_ctx* ctx, const char* path, pgcp_lpc** out) {
    Range range("pgcp_lpc_load");
    if (!ctx || !path || !out) return bad(ctx, "null argument");
    *out = nullptr;
    pgcp::AllocScope scope(ctx->stream);
    return fail(ctx, pgcp::lpc_load(ctx, path, out));
}

pgcp_status pgcp_lpc_step(const pgcp_lpc* lpc, int64_t* step) {
    if (!lpc || !step) return PGCP_E_INVALID;
    *step = lpc->step;
    return PGCP_OK;
}

void pgcp_lpc_destroy(pgcp_lpc* lpc) {
    if (!lpc) return;
    // the network may be read by several contexts' streams: let all of them finish
    (void)hipDeviceSynchronize();
    pgcp::lpc_destroy(lpc);
}

pgcp_status pgcp_lpc_infer(pgcp_ctx* ctx, pgcp_part* P, const pgcp_lpc* lpc, int32_t system) {
    Range range("pgcp_lpc_infer");
    if (!ctx || !P || !lpc) return bad(ctx, "null argument");
    if (P->host_only) return bad(ctx, "host-only plan");
    pgcp::AllocScope scope(ctx->stream);
    P->stream = ctx->stream;
    return fail(ctx, pgcp::lpc_infer(ctx, P, lpc, system));
}

pgcp_status pgcp_lpc_export(pgcp_ctx* ctx, const pgcp_part* P, int32_t piece, double* o_off, double* o_diag,
                            double* m_off, double* m_diag) {
    Range range("pgcp_lpc_export");
    if (!ctx || !P) return bad(ctx, "null argument");
    if (P->host_only) return bad(ctx, "host-only plan");
    if (piece < 0 || piece >= P->K) return bad(ctx, "piece out of range");
    pgcp::AllocScope scope(ctx->stream);
    return fail(ctx, pgcp::lpc_export(ctx, P, piece, o_off, o_diag, m_off, m_diag));
}

pgcp_status pgcp_lpc_grad(pgcp_ctx* ctx, pgcp_part* P, pgcp_lpc* lpc, int32_t system, const float* probes_dev,
                          int32_t n_probes, double* loss, float* grad_host) {
    Range range("pgcp_lpc_grad");
    if (!ctx || !P || !lpc || !probes_dev) return bad(ctx, "null argument");
    if (P->host_only) return bad(ctx, "host-only plan");
    pgcp::AllocScope scope(ctx->stream);
    P->stream = ctx->stream;
    return fail(ctx, pgcp::lpc_grad(ctx, P, lpc, system, probes_dev, n_probes, loss, grad_host, 0, 0.f));
}

pgcp_status pgcp_lpc_train_step(pgcp_ctx* ctx, pgcp_part* P, pgcp_lpc* lpc, int32_t system,
                                const float* probes_dev, int32_t n_probes, float lr, double* loss) {
    Range range("pgcp_lpc_train_step");
    if (!ctx || !P || !lpc || !probes_dev) return bad(ctx, "null argument");
    if (P->host_only) return bad(ctx, "host-only plan");
    if (!(lr > 0.f)) return bad(ctx, "learning rate must be positive");
    pgcp::AllocScope scope(ctx->stream);
    P->stream = ctx->stream;
    return fail(ctx, pgcp::lpc_grad(ctx, P, lpc, system, probes_dev, n_probes, loss, nullptr, 1, lr));
}

pgcp_status pgcp_part_rows(const pgcp_part* P, int64_t* row0) {
    if (!P || !row0) return PGCP_E_INVALID;
    for (int i = 0; i <= P->K; ++i) row0[i] = P->row0[i];
    return PGCP_OK;
}

pgcp_status pgcp_part_row_vertices(const pgcp_part* P, int32_t* row_gv) {
    if (!P || !row_gv) return PGCP_E_INVALID;
    for (int64_t r = 0; r < P->N; ++r) row_gv[r] = P->row_gv[r];
    return PGCP_OK;
}

}  // extern "C"

/*
 * pgcp.h -- C ABI of the MI355X (gfx950) implementation of parallelizable
 * global conformal parameterization via partial welding (PGCP; Choi,
 * Leung-Liu, Gu, Lui).  Algorithm 3 of the paper, stage by stage:
 *
 *   pgcp_partition       Section 4.1   cut the mesh into simply-connected pieces
 *   pgcp_assemble_cotan  Section 4.2   cotangent Laplacian of every piece
 *   pgcp_local_param     Section 4.2   DNCP free-boundary flattening of every piece
 *   pgcp_weld            Sections 4.3, 4.4   partial welding (+ disk / sphere step)
 *   pgcp_harmonic_solve  Section 4.5   Laplace equation with the welded boundary
 *   pgcp_distortion      Sections 3.5, 5   angle distortion, Beltrami |mu|, flips
 *   pgcp_area_*          Section 6     area distortion and its Moebius post-optimisation
 *
 * Conventions
 *  - Plain C types only; no exceptions cross this boundary.  Every call returns
 *    a pgcp_status; pgcp_last_error(ctx) gives a message for the last failure.
 *  - "_host" pointers are host memory, "_dev" pointers are device memory on the
 *    context's device.  The caller owns every array it passes; the library never
 *    frees them.  Device arrays must stay valid until the context's stream has
 *    passed the call.
 *  - The library owns pgcp_ctx and pgcp_part; release them with the matching
 *    *_destroy call.
 *  - Device work is enqueued on the context's stream.  Calls that return host
 *    results (partition, query/export, weld, and any call given a non-NULL stats
 *    pointer) synchronise that stream before returning.
 *  - Device memory the library allocates inside a context's call comes from the
 *    device's stream-ordered pool (hipMallocAsync) on that context's stream and
 *    goes back to it in the order of the stream of the context that last worked
 *    on the object (pgcp_part_destroy included), so no call waits for work on
 *    other streams.  A plan is meant for one context at a time: a caller that
 *    moves a plan to another context's stream orders the two streams itself.
 *  - Several contexts (threads, streams) may work on one device at once.  A
 *    batched-CG launch needs every workgroup of the device resident, so the
 *    library runs one such launch per device at a time (a lock held from launch
 *    to completion); all other work of the contexts overlaps.  Autotuned launch
 *    shapes are shared by the contexts of a device (and kept in the file that
 *    the environment variable PGCP_TUNE_CACHE names, if set).  Use one process
 *    per GPU: a second process's cooperative launches have failed with
 *    PGCP_E_HIP while another process held the GPU.
 *  - Coordinates are float64.  Indices are int32.  Planar coordinates are stored
 *    as interleaved (x, y) pairs; spherical ones as (x, y, z) triples.
 *  - Boundary arrays ("bdy") list every piece's boundary loop, piece by piece
 *    in piece order, each loop counter-clockwise (the piece on its left) from
 *    its smallest global vertex index.  Seam arrays list every vertex that lies
 *    on some piece's boundary once, in ascending global index.
 */
#ifndef PGCP_H
#define PGCP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PGCP_OK = 0,
    PGCP_E_INVALID = -1,    /* bad argument, shape or call order                        */
    PGCP_E_TOPOLOGY = -2,   /* a piece is not a disk: non-manifold edge, pinched vertex,
                               several boundary loops, wrong Euler characteristic        */
    PGCP_E_DEGENERATE = -3, /* zero-area triangle                                        */
    PGCP_E_NOCONV = -4,     /* some piece missed the residual tolerance (see stats)       */
    PGCP_E_BREAKDOWN = -5,  /* CG breakdown (p.Ap <= 0 or not finite)                     */
    PGCP_E_WELD = -6,       /* welding precondition failed (arc order, short arc, ...)    */
    PGCP_E_HIP = -7,        /* HIP runtime error                                          */
    PGCP_E_NOMEM = -8
} pgcp_status;

typedef enum { PGCP_FREE = 0, PGCP_DISK = 1, PGCP_SPHERE = 2 } pgcp_mode;
typedef enum { PGCP_FP64 = 0, PGCP_FP32_REFINE = 1 } pgcp_precision;

typedef enum { PGCP_PC_JACOBI = 0, PGCP_PC_LEARNED = 1 } pgcp_precond;
typedef enum { PGCP_SYS_DNCP = 0, PGCP_SYS_HARMONIC = 1 } pgcp_system;

typedef struct pgcp_ctx pgcp_ctx;
typedef struct pgcp_part pgcp_part;
typedef struct pgcp_lpc pgcp_lpc;

/* Solver options.  tol: relative residual ||b - A x||_2 / ||b||_2 in FP64 with
 * the FP64 matrix, per piece (per coordinate for the harmonic solve).
 * inner_tol: relative residual reduction of each FP32 inner solve (FP32_REFINE).
 * max_iter: cap on CG iterations per inner solve; max_refine: cap on FP64
 * residual evaluations; stall_iters: an inner solve stops early after this
 * many iterations without a 10% reduction of its residual (restarted from the
 * FP64 residual by the next refinement pass).  Zero fields take the defaults
 * (1e-10, 1e-4, 20000, 30, 4000).  PGCP_VERBOSE=1 in the environment prints
 * one line per refinement pass to stderr.
 * precond: PGCP_PC_JACOBI (default) or PGCP_PC_LEARNED with lpc set: the
 * network's sparse approximate inverse of each piece is computed before the
 * solve (pgcp_lpc_infer) and replaces D^-1; a piece whose learned solve breaks
 * down or stagnates is finished with Jacobi (counted in stats.n_fallback), so
 * the tolerance is met either way. */
typedef struct {
    int32_t precision;        /* pgcp_precision */
    int32_t max_iter;
    int32_t max_refine;
    int32_t stall_iters;
    double tol;
    double inner_tol;
    int32_t precond;          /* pgcp_precond */
    int32_t reserved;
    pgcp_lpc* lpc;            /* required for PGCP_PC_LEARNED */
} pgcp_solve_opts;

/* Per-call solver report.  Arrays are optional (NULL = not wanted), sized n_sub. */
typedef struct {
    int32_t n_sub;            /* out */
    int32_t refine_steps;     /* out: FP64 residual evaluations performed            */
    int64_t total_iters;      /* out: CG iterations summed over pieces and passes    */
    int32_t* iters;           /* in/out [n_sub] CG iterations per piece (all passes) */
    double* relres;           /* in/out [n_sub*2] final FP64 relative residual (x, y) */
    int32_t* status;          /* in/out [n_sub] 0 = converged                         */
    double seconds;           /* out: wall time of the call                          */
    double cg_kernel_ms;      /* out: summed duration of the batched-CG launches (HIP events) */
    double cg_bytes;          /* out: minimal algorithmic bytes of those launches in FP32
                                 accounting, summed over pieces and iterations: per row, 8 B per
                                 matrix entry (FP32 value + int32 column, diagonal included), 4 B
                                 of inverse diagonal and 76 B of (x, y) state vectors; the learned
                                 SPAI adds 8 B per entry of M                                     */
    int32_t cg_launches;      /* out: number of batched-CG launches                    */
    int32_t rows_per_thread;  /* out: 64-row slices per wave of the batched-CG launch  */
    int32_t cg_workgroups;    /* out: workgroups of the batched-CG launch              */
    int32_t cg_block;         /* out: threads per workgroup of the batched-CG launch   */
    int32_t cg_stream;        /* out: 1 if the launch streamed its vectors through memory
                                 (rows beyond what registers of one cooperative grid hold) */
    int32_t n_fallback;       /* out: pieces finished with Jacobi after the learned
                                 preconditioner broke down or stagnated              */
    int32_t cg_single;        /* out: 1 if the last batched-CG launch used the single-reduction
                                 kernel (one per-piece barrier per iteration; opt-in with
                                 PGCP_PCG_KERNEL=single in the environment), 0 if the
                                 two-barrier or the streaming kernel                     */
    double cg_bytes_native;   /* out: the same launches' bytes at the precision their
                                 recurrences ran in (8 B values and vectors for FP64 solves):
                                 matrix value + column per entry, ten passes over the (x, y)
                                 vectors, the diagonal and the mask twice per row             */
} pgcp_solve_stats;

/* Distortion statistics over all 3|F| angles (Table 5 of the paper). */
typedef struct {
    double mean_abs_d, sd_abs_d, max_abs_d;  /* degrees; sd with N-1 */
    double median_abs_d, iqr_abs_d;          /* midpoint-rule percentiles; NaN unless requested */
    double max_mu;                           /* max |mu| of the piecewise-linear map */
    int64_t n_flipped;                       /* signed area (plane) or det (sphere) <= 0 */
    int64_t n_mu_ge1;                        /* faces with |mu| >= 1 - 1e-8 */
} pgcp_dist_stats;

/* Report of pgcp_fold_repair. */
typedef struct {
    int32_t passes;           /* repair passes run                                   */
    int32_t pieces_repaired;  /* pieces with at least one kept pass                  */
    int64_t flips_before;     /* flipped faces of the map given                      */
    int64_t flips_after;      /* flipped faces of the map returned                   */
    int64_t total_iters;      /* CG iterations of the repair solves, summed over pieces */
    double cg_kernel_ms;      /* summed duration of their batched-CG launches        */
    int32_t pieces_stopped;   /* pieces whose last pass did not lower their flip count
                                 and was undone                                       */
    int32_t reserved;
} pgcp_fold_stats;

typedef struct {
    int64_t nv, nf;
    int32_t n_sub;
    int32_t mode;
    int64_t n_rows;           /* packed rows (piece vertices, each piece padded to 64) */
    int64_t n_bdy;            /* total boundary-loop entries                            */
    int64_t n_seam;           /* distinct boundary vertices                             */
    int64_t nnz_offdiag;      /* stored off-diagonal entries (without padding)          */
    int64_t sell_elems;       /* stored off-diagonal slots including SELL-64 padding    */
    int32_t weld_rounds;      /* rounds of the balanced merge tree                      */
    int32_t reserved;
} pgcp_part_info;

/* Context on device `hip_device`, enqueuing on `hip_stream` (hipStream_t; NULL =
 * the null stream). */
pgcp_status pgcp_ctx_create(pgcp_ctx** out, int hip_device, void* hip_stream);
void pgcp_ctx_destroy(pgcp_ctx* ctx);
/* Message of the last failed call on ctx; with ctx NULL, of the last failed
 * pgcp_ctx_create on the calling thread. */
const char* pgcp_last_error(const pgcp_ctx* ctx);
/* Change the stream later calls enqueue on (work already enqueued on the old
 * stream must be ordered before the new stream's by the caller). */
pgcp_status pgcp_ctx_set_stream(pgcp_ctx* ctx, void* hip_stream);

/* Section 4.1.  Cut edges are interior edges whose two faces carry different
 * labels; the connected components of the face graph over the remaining
 * interior edges are the pieces, numbered by their smallest face index.  Every
 * piece must be a topological disk (one boundary loop, no pinched vertex,
 * V - E + F = 1), else PGCP_E_TOPOLOGY.  Builds the full plan: piece vertex
 * lists, SELL-64 matrix structure, boundary loops, DNCP pins, seam list and the
 * weld merge tree, and uploads it to the device.
 * V_host [nv][3] float64, F_host [nf][3] int32 (counter-clockwise), label_host
 * [nf] int32.  Synchronous.  ctx may be NULL: the plan is then host-only (no
 * device mirrors) and serves pgcp_part_query/export and pgcp_weld only.
 * Limits (PGCP_E_INVALID): nv < 2^30, nf < 2^29, at most 134,217,728 vertices
 * in one piece (the batched CG addresses a piece's vectors with 32-bit byte
 * offsets). */
pgcp_status pgcp_partition(pgcp_ctx* ctx, const double* V_host, int64_t nv,
                           const int32_t* F_host, int64_t nf, const int32_t* label_host,
                           int32_t mode, pgcp_part** out);
pgcp_status pgcp_part_query(const pgcp_part* part, pgcp_part_info* info);
/* Copy plan arrays to host buffers (each may be NULL):
 * face_sub [nf], sub_nv [n_sub] (vertices per piece), loop_ptr [n_sub+1],
 * loop_gv [n_bdy] (boundary loops), seam_gv [n_seam]. */
pgcp_status pgcp_part_export(const pgcp_part* part, int32_t* face_sub, int32_t* sub_nv,
                             int32_t* loop_ptr, int32_t* loop_gv, int32_t* seam_gv);
/* Release a plan.  Its device memory returns to the pool in the order of the
 * stream of the context that last worked on it; the stream must still exist. */
void pgcp_part_destroy(pgcp_part* part);

/* Copy the assembled FP64 cotangent Laplacian of one piece to host CSR arrays
 * (local vertex order = ascending global index, columns ascending, diagonal
 * included).  rowptr [n+1] with n = sub_nv[piece]; col/val sized rowptr[n]
 * (call first with col = val = NULL to get rowptr).  Synchronous. */
pgcp_status pgcp_laplacian_export(pgcp_ctx* ctx, const pgcp_part* part, int32_t piece,
                                  int32_t* rowptr, int32_t* col, double* val);

/* Section 4.2.  Cotangent Laplacian of every piece in its PSD form:
 * L[p][q] = -(cot a_pq + cot b_pq)/2, L[p][p] = -sum_q L[p][q], cot of the
 * angle at k in triangle (i,j,k) = (u.v)/|u x v|, u = v_i - v_k, v = v_j - v_k.
 * Kept on the device in FP64 and FP32.  V_dev [nv][3].  Async. */
pgcp_status pgcp_assemble_cotan(pgcp_ctx* ctx, pgcp_part* part, const double* V_dev);

/* Section 4.2.  DNCP of every piece: solves (L (+) L - M/2) z = 0 with two
 * pinned boundary vertices (the loop's smallest global index at (0,0), the
 * loop vertex farthest from it in R^3 at (distance, 0)), by batched
 * preconditioned CG on all pieces at once (Jacobi, or the learned sparse
 * approximate inverse when opts->precond is PGCP_PC_LEARNED; FP64 recurrences,
 * or FP32 ones with FP64 residual refinement per opts->precision); then
 * translates each piece so the mean of its boundary points is 0.  Writes
 * bdy_uv_dev [n_bdy][2].  Requires pgcp_assemble_cotan.  opts may be NULL
 * (defaults), stats may be NULL.  The refinement passes are decided on the
 * host, so the call returns once the solve has finished; the boundary gather
 * into bdy_uv_dev is enqueued on the stream. */
pgcp_status pgcp_local_param(pgcp_ctx* ctx, pgcp_part* part, const pgcp_solve_opts* opts,
                             double* bdy_uv_dev, pgcp_solve_stats* stats);

/* Sections 4.3-4.4.  Partial welding (Algorithms 1 and 2) of the boundary
 * coordinates along the plan's balanced merge tree; in disk mode followed by
 * the geodesic algorithm on the outer boundary and the Cayley map onto the unit
 * disk; in sphere mode the last two components are closed-welded.  With a
 * context the maps of every merge round run on the device (one workgroup per
 * pair zips its two arcs; every other tracked point is replayed through its
 * pair's recorded maps in parallel); the merge bookkeeping, the Moebius
 * normalisation and arcs longer than 8,192 points run on the host.  ctx may be
 * NULL for a host-only plan (everything on the host).
 * bdy_uv_host [n_bdy][2] in, welded_uv_host [n_seam][2] out (sphere mode: a
 * point at infinity is written as (+inf, +inf)).  Synchronous. */
pgcp_status pgcp_weld(pgcp_ctx* ctx, pgcp_part* part, const double* bdy_uv_host,
                      double* welded_uv_host);

/* Section 4.5.  Harmonic map of every piece with the welded boundary as
 * Dirichlet data (same L, boundary rows eliminated), batched CG; then the
 * global gather: interior vertices from their piece, seam vertices from the
 * weld.  Sphere mode solves each piece in its own rotation chart
 * w = (z - c)/(1 + conj(c) z), c = stereographic image of the normalised mean of
 * the piece's welded boundary points on the sphere (computed on the device from
 * welded_uv_dev), and finishes with the stereographic projection
 * (2Re w, -2Im w, |w|^2-1)/(|w|^2+1).  welded_uv_dev [n_seam][2] (a point at
 * infinity as an infinite coordinate); out_dev [nv][2] (free/disk) or [nv][3]
 * (sphere).  Requires pgcp_assemble_cotan. */
pgcp_status pgcp_harmonic_solve(pgcp_ctx* ctx, pgcp_part* part, const double* welded_uv_dev,
                                const pgcp_solve_opts* opts, double* out_dev,
                                pgcp_solve_stats* stats);

/* Sections 3.5 and 5.  Per face: the three angle distortions in degrees
 * (parameter angle minus surface angle, atan2(|u x v|, u.v)), |mu| of the
 * piecewise-linear map between isometric frames, and the flip flag (signed
 * area <= 0 in the plane, det[phi_i, phi_j, phi_k] <= 0 on the sphere).
 * V_dev [nv][3], F_dev [nf][3], param_dev [nv][dim], dim 2 or 3.  d_dev [nf][3],
 * mu_dev [nf], flip_dev [nf] may be NULL.  want_quantiles != 0 also computes the
 * median and IQR of |d| (exact order statistics by a device radix select).
 * stats may be NULL (then async). */
pgcp_status pgcp_distortion(pgcp_ctx* ctx, const double* V_dev, int64_t nv,
                            const int32_t* F_dev, int64_t nf, const double* param_dev,
                            int32_t dim, double* d_dev, double* mu_dev, uint8_t* flip_dev,
                            int32_t want_quantiles, pgcp_dist_stats* stats);

/* Sections 3.5 and 4.5 (last step of Algorithm 3).  Quasi-conformal fold
 * repair of a planar (free or disk) map.  A map folds exactly where its
 * Beltrami coefficient has |mu| >= 1 (a flipped face).  Every piece whose map
 * has a flipped face gets, on its interior vertices, the map with the same
 * boundary values whose Beltrami coefficient is the map's own with its modulus
 * cut at 1 - delta (direction kept): the linear Beltrami solver
 * div(A_mu grad u) = div(A_mu grad v) = 0 with piecewise-linear elements on
 * the faces' isometric frames (A_0 = identity gives the cotangent Laplacian),
 * solved for the pieces concerned by the batched CG (Jacobi, opts'
 * precision and tolerances; opts may be NULL).  Repeated while a piece still
 * has a flipped face, up to max_passes passes; a pass that does not lower a
 * piece's count of flipped faces is undone and ends that piece's repair (its
 * welded boundary itself may fold).  Boundary and seam vertices
 * keep their values, so the pieces still glue.  V_dev [nv][3] and F_dev
 * [nf][3] are the mesh given to pgcp_partition; param_dev [nv][2] is the map
 * (pgcp_harmonic_solve's output), repaired in place.  delta in (0, 1), 0.1 is
 * the usual choice.  Requires pgcp_assemble_cotan; sphere plans are rejected
 * (PGCP_E_INVALID).  A repair solve that misses the tolerance returns
 * PGCP_E_NOCONV with the map as the last completed pass left it.  stats may be
 * NULL.  Synchronous (the flip count of every pass comes back to the host). */
pgcp_status pgcp_fold_repair(pgcp_ctx* ctx, pgcp_part* part, const double* V_dev, const int32_t* F_dev,
                             double* param_dev, double delta, int32_t max_passes,
                             const pgcp_solve_opts* opts, pgcp_fold_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * per-face outputs and statistics as pgcp_distortion (same kernels, bitwise
 * the same results), without quantiles (median_abs_d and iqr_abs_d are NaN).
 * Allocates nothing: the per-workgroup partial sums live in a fixed device
 * array of the library (about 2 MiB per device, held until the process ends),
 * which limits a call to pgcp_distortion_noalloc_max_faces() faces
 * (8,388,608); larger nf is PGCP_E_INVALID, checked before anything else.
 * Every call on one device shares that array: calls that overlap on one device
 * (contexts on several streams or threads) race and must be ordered by the
 * caller.  stats may be NULL (then asynchronous on the context's stream);
 * otherwise the call copies the final record to the host and synchronises. */
pgcp_status pgcp_distortion_noalloc(pgcp_ctx* ctx, const double* V_dev, int64_t nv,
                                    const int32_t* F_dev, int64_t nf, const double* param_dev,
                                    int32_t dim, double* d_dev, double* mu_dev, uint8_t* flip_dev,
                                    pgcp_dist_stats* stats);
int64_t pgcp_distortion_noalloc_max_faces(void);

/* Section 6, area distortion.  Per face
 *   d_area(T) = log[(A(phi(T)) / sum A(phi)) / (A(T) / sum A)],
 * A the area of the flat triangle through the face's points (in R^3 for the
 * mesh and for spherical parameterizations).  V_dev [nv][3], F_dev [nf][3]
 * (indices < nv, not checked), param_dev [nv][dim], dim 2 or 3; d_dev [nf]
 * may be NULL; *mean_abs = mean of |d_area|.  A zero-area or non-finite
 * triangle of the mesh is PGCP_E_DEGENERATE; one of the parameterization
 * makes *mean_abs +inf.  Synchronous. */
pgcp_status pgcp_area_distortion(pgcp_ctx* ctx, const double* V_dev, int64_t nv,
                                 const int32_t* F_dev, int64_t nf, const double* param_dev,
                                 int32_t dim, double* d_dev, double* mean_abs);
/* Section 6, area distortion: mean |d_area| of param composed with a Moebius
 * map.  mode PGCP_FREE (dim 2): f(z) = (a z + b)/(c z + d), mobius[8] = Re a,
 * Im a, Re b, Im b, Re c, Im c, Re d, Im d.  PGCP_DISK (dim 2): f(z) = (z -
 * alpha)/(1 - conj(alpha) z), mobius[2] = Re alpha, Im alpha.  PGCP_SPHERE
 * (dim 3): sigma^-1 o f o sigma with the eight-parameter f and sigma(p) =
 * (x - i y)/(1 - z).  Parameters with ad - bc = 0 or |alpha| >= 1 give +inf.
 * Synchronous. */
pgcp_status pgcp_area_objective(pgcp_ctx* ctx, const double* V_dev, int64_t nv,
                                const int32_t* F_dev, int64_t nf, const double* param_dev,
                                int32_t dim, int32_t mode, const double* mobius, double* value);
/* Section 6, area distortion: the Moebius map of the mode (as in
 * pgcp_area_objective) minimising mean |d_area|, by Nelder-Mead from the
 * identity (initial simplex of step 0.1 per parameter), one evaluation on the
 * device per objective value; no step starts once max_evals evaluations have
 * been made (the last step adds at most n + 1, n = 8 or 2).  Writes the parameters to mobius[8] (mobius[2]
 * for the disk), the objective at the identity and at the result, the number
 * of evaluations (n_evals may be NULL) and, if out_dev is not NULL, the
 * composed parameterization out_dev [nv][dim].  Synchronous. */
pgcp_status pgcp_area_mobius_opt(pgcp_ctx* ctx, const double* V_dev, int64_t nv,
                                 const int32_t* F_dev, int64_t nf, const double* param_dev,
                                 int32_t dim, int32_t mode, int32_t max_evals, double* mobius,
                                 double* before, double* after, int32_t* n_evals, double* out_dev);

/* ---------------------------------------------------------------------------
 * Learned sparse approximate inverse (the GPU path's preconditioner; the paper
 * solves each piece directly).  One message-passing network (width 64, three
 * rounds, 62,466 parameters; weight matrices used in bf16 on the matrix cores,
 * fp32 accumulation) reads a piece's cotangent Laplacian and Dirichlet mask and
 * emits M = D^-1/2 (diag(exp(o_p) + sum_q |o_pq|) + O) D^-1/2 with L's
 * sparsity: symmetric positive definite for any parameters, and equal to the
 * Jacobi preconditioner D^-1 when the outputs are zero.  The flat parameter
 * vector (fp32) is W_x[3][64], b_x[64], W_y[3][64], b_y[64], per round
 * W_e[192][64], b_e[64], W_v[128][64], b_v[64], then u_e[64], c_e, u_v[64], c_v.
 * A system is PGCP_SYS_DNCP (pins masked) or PGCP_SYS_HARMONIC (boundary masked).
 * ------------------------------------------------------------------------- */

int64_t pgcp_lpc_num_params(void);
/* params_host [num_params] fp32, or NULL for all zeros (= Jacobi).  The
 * network lives on the context's device; release with pgcp_lpc_destroy. */
pgcp_status pgcp_lpc_create(pgcp_ctx* ctx, const float* params_host, pgcp_lpc** out);
pgcp_status pgcp_lpc_get_params(pgcp_ctx* ctx, const pgcp_lpc* lpc, float* params_host);
/* Any context's solves may read the network; destroying it waits for the device
 * to finish everything enqueued. */
void pgcp_lpc_destroy(pgcp_lpc* lpc);
/* Write the network's whole training state to `path`: the fp32 master
 * parameters, Adam's first and second moments and its step count, in a small
 * binary file (magic "PGCPLPC1", int64 parameter count, int64 step, three fp32
 * arrays of num_params, a 64-bit FNV-1a hash of the preceding bytes; written
 * to path.tmp and renamed).  Synchronous.  PGCP_E_INVALID if the file cannot
 * be written. */
pgcp_status pgcp_lpc_save(pgcp_ctx* ctx, const pgcp_lpc* lpc, const char* path);
/* Create a network on the context's device from a file written by
 * pgcp_lpc_save: parameters, Adam moments and step restored, so training
 * resumes where it stopped and inference uses the saved weights.  A file of
 * the wrong size, magic, parameter count or hash is PGCP_E_INVALID.  Release
 * with pgcp_lpc_destroy.  Synchronous. */
pgcp_status pgcp_lpc_load(pgcp_ctx* ctx, const char* path, pgcp_lpc** out);
/* Number of Adam steps the network has taken (restored by pgcp_lpc_load). */
pgcp_status pgcp_lpc_step(const pgcp_lpc* lpc, int64_t* step);
/* Run the network on every piece of an assembled plan and store the SPAI
 * values for `system` in the plan.  Async. */
pgcp_status pgcp_lpc_infer(pgcp_ctx* ctx, pgcp_part* part, const pgcp_lpc* lpc, int32_t system);
/* Copy one piece's network outputs and SPAI values (after pgcp_lpc_infer) to
 * host arrays, off-diagonal entries in the order of pgcp_laplacian_export
 * without the diagonal: o_off/m_off [sub_nnz], o_diag/m_diag [sub_nv]; any may
 * be NULL.  Masked rows and columns of M are zero.  Synchronous. */
pgcp_status pgcp_lpc_export(pgcp_ctx* ctx, const pgcp_part* part, int32_t piece, double* o_off,
                            double* o_diag, double* m_off, double* m_diag);
/* Training loss over every piece of the plan:
 *   loss = mean over pieces of mean over probes k of |M A v_k - v_k|^2 / |v_k|^2
 * with A the piece's Laplacian on its free rows.  probes_dev [n_probes][n_rows]
 * fp32 in packed-row order (pgcp_part_rows), 1 <= n_probes <= 16; values on
 * masked rows are ignored.  pgcp_lpc_grad also writes the gradient
 * (grad_host [num_params], may be NULL); pgcp_lpc_train_step takes one Adam
 * step (beta 0.9, 0.999, eps 1e-8) of size lr on the parameters.  Synchronous. */
pgcp_status pgcp_lpc_grad(pgcp_ctx* ctx, pgcp_part* part, pgcp_lpc* lpc, int32_t system,
                          const float* probes_dev, int32_t n_probes, double* loss, float* grad_host);
pgcp_status pgcp_lpc_train_step(pgcp_ctx* ctx, pgcp_part* part, pgcp_lpc* lpc, int32_t system,
                                const float* probes_dev, int32_t n_probes, float lr, double* loss);
/* Packed-row ranges of the pieces: piece i owns rows row0[i] .. row0[i+1]-1,
 * its sub_nv[i] vertices on the first sub_nv[i] of them, the rest padding.
 * row0 [n_sub+1]. */
pgcp_status pgcp_part_rows(const pgcp_part* part, int64_t* row0);
/* Copy the packed-row iterate of the last DNCP or harmonic solve on the plan
 * (interleaved (x, y) float64 per packed row, in pgcp_part_row_vertices
 * order; masked rows hold their pinned or Dirichlet values; for the sphere the
 * harmonic values are in each piece's chart) to out_dev [row0[n_sub]][2], and
 * which system it was to *system (PGCP_SYS_*; may be NULL).  The training
 * driver of the network builds its error probes from these.  Async.
 * PGCP_E_INVALID if no solve has run on the plan. */
pgcp_status pgcp_part_solution(pgcp_ctx* ctx, const pgcp_part* part, int32_t* system, double* out_dev);
/* Global vertex of every packed row, -1 on padding rows: row_gv [row0[n_sub]].
 * Within a piece the rows follow a reverse Cuthill-McKee order of the piece's
 * vertex graph (a workgroup's consecutive rows form a compact patch), not the
 * global order; probe vectors (pgcp_lpc_grad) are laid out by this map. */
pgcp_status pgcp_part_row_vertices(const pgcp_part* part, int32_t* row_gv);

#ifdef __cplusplus
}
#endif
#endif /* PGCP_H */

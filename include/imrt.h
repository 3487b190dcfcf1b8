/*
 * imrt.h -- C ABI of libimrt, a gfx950 (MI355X) implementation of the
 * fluence-map optimiser of "GPU-based ultra fast IMRT plan optimization"
 * (Men, Gu, Choi, Majumdar, Zheng, Mueller, Jiang; arXiv:0908.4421).
 *
 * Model (Section 2.1, Eqs. (1)-(4)): voxel dose z = D x over the voxels x
 * beamlets dose-deposition matrix D; one-sided quadratic penalties
 *   F_j(z_j) = w_u,j * min(z_j - T_u,j, 0)^2 + w_o,j * max(z_j - T_o,j, 0)^2
 * summed over voxels into G(x), minimised over x >= 0.
 * Method (Section 2.2, Eq. (5), steps 1-5): gradient projection
 *   x_{k+1} = max(0, x_k - lambda grad G(x_k)),  grad G = 2 D^T r,
 *   r_j = w_u,j * min(z_j - T_u,j, 0) + w_o,j * max(z_j - T_o,j, 0),
 * with Armijo's rule: accept lambda when
 *   G(x_{k+1}) < G(x_k) - (eps/lambda) * ||x_{k+1} - x_k||^2,
 * else lambda <- lambda/alpha; stop when |G_{k+1} - G_k| / G_{k+1} < delta.
 *
 * Conventions for every entry point:
 *  - Return value: IMRT_OK (0) or a negative imrt_error; the message of the
 *    last error on the calling thread is returned by imrt_last_error().
 *  - Pointers named *_dev are device memory owned by the caller (for example
 *    PyTorch tensors); they must stay valid until the call returns.  Every
 *    other array pointer is host memory read (or written) during the call
 *    only.  Opaque handles are owned by the library and freed by the
 *    matching *_destroy; destroying NULL is a no-op.
 *  - All device work is ordered on the context's stream.  Calls that return
 *    a host value (objective, step norm, solve result, export) synchronise
 *    that stream before returning; the others only enqueue work.
 *  - Dense vectors are float32: x and g have nb entries, dose and residual
 *    nv entries.  Objective values, step sizes and norms are float64.
 *  - One context must not be used from two threads at once.
 */
#ifndef IMRT_H
#define IMRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IMRT_API __attribute__((visibility("default")))

typedef struct imrt_ctx imrt_ctx;
typedef struct imrt_dose imrt_dose;
typedef struct imrt_plan imrt_plan;

/* Error codes returned by every entry point. */
typedef enum {
  IMRT_OK = 0,
  IMRT_EINVAL = -1,      /* bad argument: null handle, size mismatch, unsorted or out-of-range index, negative weight, ... */
  IMRT_ENOMEM = -2,      /* device or host allocation failed */
  IMRT_EHIP = -3,        /* a HIP runtime call failed; the message carries hipGetErrorString */
  IMRT_ENOTREADY = -4,   /* structures or penalties not set on the plan */
  IMRT_EUNSUPPORTED = -5,/* valid request outside what the library supports (message says which limit) */
  IMRT_ETIMEDOUT = -6    /* a bounded wait ended before its result was ready */
} imrt_error;

/* Final state of a solve (imrt_solve_result.status). */
typedef enum {
  IMRT_CONVERGED = 0,    /* relative objective change below delta, or G == 0 (step 5) */
  IMRT_MAX_ITER = 1,     /* max_iter accepted iterations done (always the case with fixed_iters) */
  IMRT_STALLED = 2,      /* a trial equalled x_k (||x_t - x_k|| == 0): x_k is stationary */
  IMRT_LS_FAIL = 3,      /* more than max_backtracks step reductions in one line search */
  IMRT_NUMERIC = 4       /* a trial objective was not finite */
} imrt_solve_status;

/* Storage of D's values.  IMRT_F32: float32 values, int32 indices.
 * IMRT_BF16 / IMRT_F16: for every beamlet i a float32 scale s_i = max_j D_ij
 * (1 if no entry of the column is positive) and 16-bit codes
 * q_ij = RN(D_ij / s_i), the exact quotient rounded once to bfloat16 or
 * IEEE binary16 (nearest, ties to even); every product then uses
 * D~_ij = s_i q_ij, and the CSR column indices are 16-bit (nb <= 65536).
 * Both sparse products still accumulate in float32 (forward) and float64
 * (adjoint); the objective, the Armijo test and the stopping test stay in
 * float64.  The 16-bit forms need the "fwd_wave" option at 1.  The paper
 * stores D in float32; the 16-bit forms halve the bytes of the values. */
typedef enum { IMRT_F32 = 0, IMRT_BF16 = 1, IMRT_F16 = 2 } imrt_dtype;

/* Penalty parameters of one structure (Eq. (1), generalised to separate
 * under/over thresholds and weights).  Weights must be finite and >= 0. */
typedef struct {
  double T_under, T_over, w_under, w_over;
} imrt_penalty;

/* Synthetic phantom geometry for imrt_build_dose_matrix (all lengths in mm).
 * Water box of nx*ny*nz voxels at spacing h centred on the isocentre; PTV
 * sphere of radius r_ptv at the origin, rectum cylinder along z of radius
 * r_rectum tangent at -y, bladder sphere of radius r_bladder tangent at +y
 * (structure ids 0 normal, 1 PTV, 2 rectum, 3 bladder, priority
 * PTV > rectum > bladder > normal).  n_beams coplanar parallel beams at
 * angles 2*pi*b/n_beams; square beamlets of side `beamlet` whose closest
 * point to the beam axis lies within r_ptv + margin; D_ij =
 * float32(exp(-(mu*depth + r^2/(2 sigma^2)))) kept where it is >= tau times
 * the beamlet's maximum over the grid.
 * coarse_normal (0 or 1): unspecified tissue at twice the voxel size in each
 * dimension (Section 3.1).  Every aligned, complete 2x2x2 block of grid
 * voxels that are all normal tissue is then one voxel (structure 0) centred
 * at c_a = (2*b_a + 1)*h - (n_a*h)/2; the voxels of D are the remaining grid
 * voxels (grid index ascending) followed by the coarse voxels (block index
 * bx + (nx/2)*(by + (ny/2)*bz) ascending), and imrt_dose_info reports
 * their count. */
typedef struct {
  int32_t nx, ny, nz;
  double h;
  double r_ptv, r_rectum, r_bladder;
  int32_t n_beams;
  double beamlet, sigma, tau, mu, margin;
  int32_t coarse_normal;
} imrt_geometry;

/* Solver settings (Section 2.2). */
typedef struct {
  double eps;             /* Armijo sufficient-decrease parameter, 0 < eps < 1 */
  double alpha;           /* step reduction factor, alpha > 1 */
  double lambda0;         /* initial step of every line search, > 0 */
  double delta;           /* relative-change stopping tolerance, >= 0 */
  int32_t max_iter;       /* cap on accepted iterations, >= 0 */
  int32_t max_backtracks; /* cap on reductions per line search, >= 0 */
  int32_t fixed_iters;    /* non-zero: run exactly max_iter iterations, no stopping test */
  int32_t trials_per_pass;/* trial step sizes evaluated per pass over D: 1, 2 or 4 (0 = 1) */
  int32_t profile;        /* >= 0; n > 0: time every n-th forward and every n-th adjoint launch
                           * with HIP events on the context stream (1 = every launch) */
  int32_t warm_start;     /* 0: every line search starts at lambda0 (Section 2.2,
                             step 2); 1: iteration k+1 starts at alpha times the
                             step accepted in iteration k (the first at lambda0) */
  void* trace;            /* nullable host buffer of max_iter imrt_trace_entry, filled on return */
  /* Resuming an interrupted solve (checkpoint and restart of Section 2.2's
   * iteration).  resume = 0: a fresh start at x_1, the other three fields
   * unused.  resume = 1: x holds the iterate x_K of an earlier solve after
   * K = k0 >= 1 accepted iterations, G_prev is G(x_{K-1}) (G(x_1) when
   * K = 1) and lambda_prev > 0 the step accepted in iteration K.  The solve
   * then applies step 5's stopping test to the pair (G(x_K), G_prev) before
   * its first iteration (and stops with 0 iterations, IMRT_CONVERGED, when
   * it holds; not with fixed_iters), a warm-started line search begins at
   * alpha * lambda_prev, and trace entries are numbered from k0 + 1;
   * max_iter caps this call's iterations.  A solve continued this way from
   * the x, G and lambda of iteration K reproduces the uninterrupted
   * trajectory bit for bit. */
  int32_t resume;
  int32_t k0;
  double G_prev;
  double lambda_prev;
} imrt_solve_params;

/* One accepted iteration. */
typedef struct {
  int32_t k;              /* accepted iterations so far (1-based) */
  int32_t backtracks;     /* step reductions in this line search */
  double lambda;          /* accepted step size */
  double step_sq;         /* ||x_{k+1} - x_k||^2 */
  double G;               /* G(x_{k+1}) */
} imrt_trace_entry;

typedef struct {
  int32_t iterations;     /* accepted iterations */
  int32_t forward_passes; /* passes over D in CSR form (including the initial evaluation) */
  int32_t adjoint_passes; /* passes over D in CSC form */
  int32_t status;         /* imrt_solve_status */
  double G_initial;       /* G(x_1) */
  double G_final;         /* G at the returned x */
  double device_ms;       /* stream time of the solve, HIP events */
  /* With params.profile: mean HIP-event duration of a forward pass kernel
   * and of an adjoint pass kernel over the timed launches among those that
   * did work (the first forward_passes and adjoint_passes launches), else 0. */
  double forward_kernel_ms;
  double adjoint_kernel_ms;
} imrt_solve_result;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`.  All work is enqueued on
 * hip_stream (a hipStream_t, borrowed; it must outlive the context).  NULL
 * selects the device's null stream, which orders with every blocking stream
 * (PyTorch's default stream is the null stream). */
IMRT_API int imrt_ctx_create(int device, void* hip_stream, imrt_ctx** out);
IMRT_API int imrt_ctx_destroy(imrt_ctx* ctx);
/* The stream the context enqueues on (a hipStream_t). */
IMRT_API int imrt_ctx_stream(const imrt_ctx* ctx, void** hip_stream_out);

/* Launch-shape settings of a context, by name:
 *   "fwd_wg_per_cu"  forward-pass workgroups per compute unit (1..64; default
 *                    3).  A "fwd_wave" workgroup has 16 waves, or 8 on a
 *                    matrix partitioned by per-plan targets
 *                    (imrt_dose_repartition_targets), that take row blocks
 *                    from a shared counter; the grid never holds more per
 *                    compute unit than fit side by side (one of 16 waves;
 *                    three of 8 with one trial per pass, two with more;
 *                    fewer when the staged vectors of a large nb fill the
 *                    LDS).  Otherwise the value is scaled by four
 *                    workgroups of 4 waves.
 *   "adj_wg_per_cu"  adjoint-pass workgroups per compute unit (1..64)
 *   "adj_min_nnz"    fewest nonzeros per adjoint workgroup (>= 16)
 *   "adj_xcd"        1: consecutive adjoint ranges on the same accelerator die,
 *                    which then share their residual gathers in its L2
 *                    (default); 0: dispatch order
 *   "voxel_tiles"    1: imrt_build_dose_matrix stores the rows of D in tiles of
 *                    4 x 4 x 2 voxels (default), so that the residual gathers
 *                    of every beam direction touch few cache lines; 0: in
 *                    grid order.  Voxel-indexed arrays passed to or from the
 *                    API are in grid order either way.
 *   "fwd_blocks_per_wave"  fewest forward row blocks per wave (1..1024,
 *                    default 1) of dose matrices created afterwards
 *   "serve_adjoint_workgroups", "serve_forward_workgroups"  per-plan
 *                    partition targets of the matrices servers created
 *                    afterwards build (defaults 128 and 32; see
 *                    imrt_dose_repartition_targets)
 *   "serve_groups_per_poll"  (adjoint, forward) dispatch groups a server
 *                    created afterwards runs between polls (1..4096,
 *                    default 16): more groups poll less often, fewer admit
 *                    and retire sooner
 *   "serve_shared_adjoint"  1: live solves of a server created afterwards
 *                    that share a resident dose matrix (re-plans of one
 *                    patient) take their gradients from one pass over its
 *                    CSC, up to four solves per pass, each solve's
 *                    arithmetic unchanged; 0 (default): one pass per solve.
 *                    Sharing saves the matrix's reads but puts several
 *                    solves' work in each workgroup: for matrices that stay
 *                    in the last-level cache one pass per solve is faster
 *   "stream_nt"      cache policy of the matrix streams in the passes of
 *                    imrt_solve and imrt_solve_batch: 0 default policy, 1
 *                    non-temporal, 2 (default) non-temporal when the CSR and
 *                    CSC bytes one iteration reads (a batch: its unfinished
 *                    plans' distinct matrices together) exceed the 256 MB
 *                    last-level cache.  Results are the same under every
 *                    policy; a server's passes keep the default policy
 *   "fwd_wave"       1: each wave of a forward workgroup streams its own row
 *                    blocks; 0: the whole workgroup shares each row block
 *   "fwd_col16"      1 (default): float32 matrices with nb <= 65536 created
 *                    afterwards keep a 16-bit copy of the CSR column indices,
 *                    which the wave forward pass reads (6 instead of 8 bytes
 *                    per nonzero, 768-entry row blocks); 0: 32-bit indices
 *   "batch_iters"    solver iterations enqueued between host polls (>= 1)
 * "adj_wg_per_cu", "adj_min_nnz", "fwd_blocks_per_wave", "fwd_col16" and
 * "fwd_wg_per_cu" are read when a dose matrix is created (its work
 * partitions and layout);
 * "fwd_wg_per_cu" and "adj_wg_per_cu" also at launch.
 * Results are deterministic for given settings; the settings change only the
 * grouping of the float32 row sums and of the float64 partial sums of G and
 * of shared columns.
 * Unknown names or out-of-range values return IMRT_EINVAL. */
IMRT_API int imrt_ctx_set_option(imrt_ctx* ctx, const char* name, int64_t value);
IMRT_API int imrt_ctx_get_option(const imrt_ctx* ctx, const char* name, int64_t* value);

/* ---- dose-deposition matrix (Section 2.1; stored as CSR, Section 2.3) ---- */

/* Build the synthetic phantom's structure ids and D on the device (CSR and
 * CSC in the given storage, from float32 values; columns ascending in each row, rows
 * ascending in each column; the rows are held in the internal voxel order
 * of the "voxel_tiles" option, and imrt_dose_export returns grid order).
 * voxel_struct_out: nullable host array receiving the nv structure ids
 * (grid order j = ix + nx*(iy + ny*iz); with coarse_normal the layout's
 * voxel order, nv <= nx*ny*nz, so nx*ny*nz bytes always suffice).  Beamlet order:
 * beam-major, then lateral index, then axial index. */
IMRT_API int imrt_build_dose_matrix(imrt_ctx* ctx, const imrt_geometry* geom, imrt_dtype storage,
                           imrt_dose** out, uint8_t* voxel_struct_out);

/* Upload a caller-built D given in CSR form (host arrays, copied).  row_ptr
 * has nv+1 entries starting at 0 and non-decreasing; col_idx entries lie in
 * [0, nb) and increase strictly within each row; values are finite and
 * >= 0.  The CSC copy is derived on the host; 16-bit storage is then
 * coded on the device from the float32 values. */
IMRT_API int imrt_dose_from_csr(imrt_ctx* ctx, int32_t nv, int32_t nb, int64_t nnz,
                       const int32_t* row_ptr, const int32_t* col_idx, const float* val,
                       imrt_dtype storage, imrt_dose** out);

IMRT_API int imrt_dose_info(const imrt_dose* dose, int32_t* nv, int32_t* nb, int64_t* nnz);

/* Copy D back to host arrays (each nullable): CSR row_ptr[nv+1],
 * col_idx[nnz], val[nnz]; CSC col_ptr[nb+1], row_idx[nnz], cval[nnz];
 * voxel_struct[nv] (only for matrices from imrt_build_dose_matrix).  With
 * 16-bit storage val and cval receive the float32 rounding of s_i q_ij. */
IMRT_API int imrt_dose_export(const imrt_dose* dose, int32_t* row_ptr, int32_t* col_idx, float* val,
                     int32_t* col_ptr, int32_t* row_idx, float* cval, uint8_t* voxel_struct);

/* 16-bit storage only (else IMRT_EINVAL): the codes q_ij as bit patterns in
 * CSR order (val_code[nnz]) and CSC order (cval_code[nnz]), and the scales
 * col_scale[nb]; each nullable; same orders as imrt_dose_export. */
IMRT_API int imrt_dose_export_codes(const imrt_dose* dose, uint16_t* val_code, uint16_t* cval_code,
                                    float* col_scale);

/* The imrt_dtype D is stored in. */
IMRT_API int imrt_dose_storage(const imrt_dose* dose, int32_t* storage);

/* d = D x (CSR, voxel-parallel).  x_dev: nb floats; d_dev: nv floats. */
IMRT_API int imrt_dose_apply(const imrt_dose* dose, const float* x_dev, float* d_dev);
/* y = D^T r (CSC, beamlet-parallel).  r_dev: nv floats; y_dev: nb floats. */
IMRT_API int imrt_dose_apply_transpose(const imrt_dose* dose, const float* r_dev, float* y_dev);

IMRT_API int imrt_dose_destroy(imrt_dose* dose);

/* ---- plan: D plus penalties --------------------------------------------- */

/* A plan borrows `dose`, which must outlive it; several plans may share
 * one dose matrix. */
IMRT_API int imrt_plan_create(imrt_ctx* ctx, const imrt_dose* dose, imrt_plan** out);

/* Structure id of every voxel (host, nv bytes, each < nstruct <= 256).
 * NULL takes the ids computed by imrt_build_dose_matrix. */
IMRT_API int imrt_set_structures(imrt_plan* plan, const uint8_t* voxel_struct, int32_t nstruct);

/* Penalty table, one entry per structure (host, nstruct entries). */
IMRT_API int imrt_set_penalties(imrt_plan* plan, const imrt_penalty* table);

/* Optional per-voxel thresholds (host, nv floats each) replacing the
 * structure thresholds: the paper's T_j, the dose of an original plan.
 * Weights still come from the structure table.  NULL, NULL clears them. */
IMRT_API int imrt_set_voxel_targets(imrt_plan* plan, const float* T_under, const float* T_over);

/* G(x) (Eqs. (2)-(4)) in float64, returned in *G_out (host).  dose_dev
 * (nullable, nv floats) receives D x. */
IMRT_API int imrt_evaluate_objective(imrt_plan* plan, const float* x_dev, double* G_out, float* dose_dev);

/* Gradient of step 1 (Section 2.2; the derivative of Eqs. (1)-(2)):
 * g = grad G(x) = 2 D^T r(D x), r_j = w_u,j min(z_j - T_u,j, 0) +
 * w_o,j max(z_j - T_o,j, 0).  x_dev, g_dev: nb floats.  G_out (nullable
 * host) receives G(x); when it is given the call synchronises the stream.
 * Uses the plan's own buffers (a plan whose dose matrix was repartitioned
 * may grow them on first use). */
IMRT_API int imrt_gradient(imrt_plan* plan, const float* x_dev, float* g_dev, double* G_out);

/* Size of the per-device scratch of imrt_gradient_noalloc (bytes): the
 * residual (4 nv bytes) plus a few kilobytes of partial sums, so plans of up
 * to about 4 million voxels. */
#define IMRT_NOALLOC_SCRATCH_BYTES (16u << 20)

/* imrt_gradient for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops): the same kernels and partition,
 * so the same g and G bit for bit, but every intermediate lives in a static
 * device array of IMRT_NOALLOC_SCRATCH_BYTES per device, held until the
 * process ends; the call allocates nothing (no hipMalloc, no plan buffer).
 * Arguments as imrt_gradient.  IMRT_EINVAL if the plan needs more scratch
 * than that (the message gives both sizes).  Every call on one device shares
 * its scratch: calls that overlap on a device (two streams, two threads)
 * race and must be serialised by the caller.  Nothing in the scratch needs
 * to start at zero.  With G_out NULL it only enqueues kernels (no memset,
 * no copy) on the context's stream. */
IMRT_API int imrt_gradient_noalloc(imrt_plan* plan, const float* x_dev, float* g_dev, double* G_out);

/* Trial point of step 2/4: x_out = max(0, x - lambda g) (computed in
 * float64, stored as float32) and *step_sq_out = ||x_out - x||^2 (float64,
 * host; nullable). */
IMRT_API int imrt_project(imrt_plan* plan, const float* x_dev, const float* g_dev, double lambda,
                 float* x_out_dev, double* step_sq_out);

/* Initial step size lambda_0 = smallest power of two >= 2/L, where
 * L = 2 * (largest penalty weight) * s^2 and s^2 = ||D v||^2 for the unit
 * vector v reached by `iters` power iterations v <- D^T D v / ||D^T D v||
 * started from v0_dev (nb floats, not all zero).  Writes lambda_0 and s. */
IMRT_API int imrt_estimate_lambda0(imrt_plan* plan, const float* v0_dev, int32_t iters,
                          double* lambda0_out, double* sigma_out);

/* The method of Section 2.2 (Eq. (5), steps 1-5): gradient projection with
 * Armijo's line search on G, from x_dev (in: x_1 >= 0, finite, nb floats;
 * out: the final iterate).  The Armijo decision and the stopping test run on
 * the device; the call synchronises the stream and fills *result. */
IMRT_API int imrt_solve(imrt_plan* plan, const imrt_solve_params* params, float* x_dev,
               imrt_solve_result* result);

/* Batched solve of n plans (the method of Section 2.2 run for several
 * independent plans at once, e.g. re-plans of several patients).  The plans must be
 * distinct and share one context; their dose matrices must have one storage
 * and forward layout and the params one trials_per_pass; several plans may share a dose matrix.
 * Each plan is solved exactly as imrt_solve solves it alone -- the same
 * passes, work partitions and reduction orders, so its result is
 * bit-identical -- but every forward and every adjoint pass of the batch is
 * one dispatch over the workgroups of all unfinished plans, batches of
 * iterations are replayed from a captured HIP graph, and a finished plan
 * leaves the dispatches at the next poll.  params, x_dev and results are
 * arrays of n; x_dev[i] (device, nb_i floats) holds x_1 on entry and the
 * result on return.  results[i].device_ms is the stream time of the whole
 * batch; forward_kernel_ms and adjoint_kernel_ms are 0.  Needs the
 * "fwd_wave" option at 1 (IMRT_EUNSUPPORTED otherwise); argument errors as
 * for imrt_solve, IMRT_EINVAL for a repeated plan, mixed contexts, storage
 * or trials_per_pass. */
IMRT_API int imrt_solve_batch(int32_t n, imrt_plan* const* plans, const imrt_solve_params* params,
                              float* const* x_dev, imrt_solve_result* results);

/* Work partitions of a dose matrix: the fewest nonzeros per adjoint
 * workgroup (the CSC is split into ranges of equal nonzero counts) and the
 * fewest row blocks per forward wave.  A plan alone fills the GPU with fine
 * partitions (the defaults, from the context's "adj_min_nnz" and
 * "fwd_blocks_per_wave" options); in a batch coarser ones spend less on each
 * workgroup's start.  Results depend on the partition only through the
 * grouping of float64 sums.  Waits for the context's stream; no solve may be
 * running on the matrix.  adj_min_nnz >= 16, fwd_blocks_per_wave in
 * [1, 1024], else IMRT_EINVAL. */
IMRT_API int imrt_dose_repartition(imrt_dose* dose, int32_t adj_min_nnz, int32_t fwd_blocks_per_wave);
IMRT_API int imrt_dose_partition(const imrt_dose* dose, int32_t* adj_min_nnz, int32_t* fwd_blocks_per_wave);
/* imrt_dose_repartition with the partition of the per-plan targets that
 * imrt_batch_autotune and the server use: about adj_workgroups adjoint and
 * fwd_workgroups forward workgroups (>= 1 each), i.e. nnz/adj_workgroups
 * nonzeros per adjoint workgroup within [1024, 32768] and
 * (nnz/512 + 1)/(8 fwd_workgroups) row blocks per forward wave within [1, 4].
 * Such a matrix's forward workgroups have 8 waves (several side by side on a
 * compute unit, so that the starts of one plan's workgroups overlap the
 * others' streams in shared dispatches); a new matrix's have 16 (one per
 * compute unit), which imrt_dose_repartition keeps.  One batched solve needs
 * matrices with the same forward workgroup size (else IMRT_EINVAL). */
IMRT_API int imrt_dose_repartition_targets(imrt_dose* dose, int32_t adj_workgroups, int32_t fwd_workgroups);

/* Launch-shape search for a batch.  A candidate is a pair of per-plan
 * targets (ta adjoint workgroups, tf forward workgroups): every dose matrix
 * of the batch gets nnz/ta nonzeros per adjoint workgroup (within
 * [1024, 32768]) and nnz/(8 tf 512) row blocks per forward wave (within
 * [1, 4]), so small plans keep enough workgroups to run fast once they run
 * alone while large ones start few.  Each candidate is applied in turn and a
 * batched solve from copies of x_dev (params as for imrt_solve_batch) is
 * timed with stream events: tune_iters > 0 fixed iterations, or with
 * tune_iters == 0 every plan to its own stopping rule (the whole batch).  The
 * fastest candidate is left applied and its targets returned in ta_out and
 * tf_out (nullable).  Solving afterwards, alone or batched, uses it. */
IMRT_API int imrt_batch_autotune(int32_t n, imrt_plan* const* plans, const imrt_solve_params* params,
                                 const float* const* x_dev, int32_t tune_iters, int32_t* ta_out,
                                 int32_t* tf_out);

IMRT_API int imrt_plan_destroy(imrt_plan* plan);

/* ---- re-plan server -------------------------------------------------------
 * A worker thread keeps every dose matrix, plan and solver state resident on
 * the device and runs the iterations of all live solves batched (as
 * imrt_solve_batch does), admitting queued requests between polls when a
 * slot and HBM are free and retiring finished solves at once: continuous
 * batching.  Each result equals imrt_solve's for the same plan, lambda_0 and
 * start point.  Memory: the budget covers resident dose matrices and live
 * plans; a new patient's matrix is admitted only when the largest matrix
 * built so far (initially a quarter of a GiB, at most half the budget) still
 * fits, and unused resident matrices are evicted least recently used first.
 * One dispatch holds one storage, forward layout and trials_per_pass: a
 * request that differs from the live solves in these waits until they have
 * finished (requests keep their arrival order).  Matrices the
 * server builds take the partition of the context's per-plan targets
 * "serve_adjoint_workgroups" and "serve_forward_workgroups" (read at server
 * creation; imrt_dose_repartition_targets); a result equals imrt_solve's on
 * a matrix with that partition. */
typedef struct imrt_server imrt_server;

typedef struct {
  int64_t patient;                  /* resident dose matrix reused if present */
  const imrt_geometry* geometry;    /* builds the matrix otherwise (copied) */
  imrt_dtype storage;
  const imrt_penalty* penalties;    /* structure table (copied), 1..256 entries */
  int32_t nstruct;
  double x0;                        /* every beamlet's start intensity, >= 0 */
  imrt_solve_params params;         /* lambda0 <= 0: 50 power iterations from the
                                       all-ones vector; profile ignored; a trace
                                       buffer (max_iter entries) is filled by the
                                       ticket's imrt_server_wait and must stay
                                       valid until that wait returns */
} imrt_request;

typedef struct {
  double queue_ms;                  /* arrival (submit) to admission */
  double plan_ms;                   /* arrival to result: time to plan */
  double lambda0;                   /* the lambda_0 the solve used */
  int64_t nnz;                      /* the dose matrix's nonzeros, voxels, beamlets */
  int32_t nv, nb;
} imrt_serve_times;

IMRT_API int imrt_server_create(imrt_ctx* ctx, int64_t hbm_budget_bytes, int32_t max_live, imrt_server** out);
/* Queue a request (thread-safe, returns at once with a ticket > 0). */
IMRT_API int imrt_server_submit(imrt_server* server, const imrt_request* request, int64_t* ticket_out);
/* Wait at most timeout_ms milliseconds (> 0) for the ticket's solve; x_out
 * (nullable host array of nb floats) receives its plan.  A failed request
 * returns its error.  When the time runs out first the call returns
 * IMRT_ETIMEDOUT and the ticket stays pending (it may be waited on again);
 * the device work of the live solves is not affected.  A ticket's result is
 * handed out once (IMRT_EINVAL for an unknown ticket, for a ticket already
 * handed out, or while another thread waits on it).  An x_out whose nb
 * differs from the plan's beamlet count is IMRT_EINVAL and leaves the
 * result pending for a later wait. */
IMRT_API int imrt_server_wait(imrt_server* server, int64_t ticket, float* x_out, int32_t nb,
                              imrt_solve_result* result, imrt_serve_times* times, int64_t timeout_ms);
IMRT_API int imrt_server_stats(imrt_server* server, int64_t* used_bytes, int64_t* peak_bytes,
                               int64_t* resident_matrices, int64_t* served);
/* Adjoint dispatch groups the server has run: *shared counts those that
 * served two or more solves on one resident matrix in one pass over its
 * CSC (the shared-matrix adjoint), *total all of them.  Either may be NULL. */
IMRT_API int imrt_server_adjoint_groups(imrt_server* server, int64_t* shared, int64_t* total);
/* Finishes the queued and live requests, then frees everything. */
IMRT_API int imrt_server_destroy(imrt_server* server);

/* Measurement aid, outside the method: the best of `reps` timed streaming
 * reads (after one untimed) of `bytes` of the device buffer `buf` (16-byte
 * aligned, nonnegative float32 values, not modified) on the context's
 * stream, in GB/s (1e9 bytes/s); the read rate the products' streams can be
 * compared with.  Synchronous.  IMRT_EINVAL for NULL pointers, misalignment,
 * bytes < 16 or reps < 1. */
IMRT_API int imrt_read_probe(imrt_ctx* ctx, const void* buf, int64_t bytes, int32_t reps, double* gbs_out);

/* Message of the last error on this thread ("" if none). */
IMRT_API const char* imrt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* IMRT_H */

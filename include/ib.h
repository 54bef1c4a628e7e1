/*
 * ibops: immersed-boundary spreading and interpolation on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library libibops.so.  All pointers named "device" are HIP device
 * pointers owned by the caller; all calls are asynchronous and ordered on the given
 * HIP stream (a hipStream_t passed as void*, NULL = the null stream) unless stated.
 *
 * Operations (Kassen, Shankar & Fogelson, arXiv 2012.06646):
 *   spreading      f = S(X) F, eq. (disc-spread) of Sec. 2 in matrix form (matrix-spread):
 *                  f_c(x_i) = sum_j delta_h(x_i - X_j) F_{j,c}, delta_h = prod_k h_k^-1 phi(./h_k)
 *   interpolation  U = J(X) u, eq. (disc-interp):  U_{j,c} = sum_i delta_h(x_i - X_j) u_c(x_i) h^d
 *   plan           cell keys, stable key/index sort, unique-key count and segment offsets,
 *                  the preparatory steps of Alg. 4 (Sec. 3.4).
 * Grid points of component c are x = h (i + xi_c), i taken modulo n (periodic box,
 * Sec. 3.1), except along walled dimensions (ib_grid_desc.walls); phi is Peskin's 4-point
 * kernel, the cosine kernel (Sec. 2) or the 3-point kernel (ib_kernel).
 *
 * Layouts:
 *   points X, forces F, velocities U : row-major (npts x dim) and (npts x ncomp)
 *   grid fields f, u                 : [ncomp][n2][n1][n0], x (index 0) fastest; 2-D: [ncomp][n1][n0]
 *   keys                             : key = c0 + n0 * (c1 + n1 * c2), the x-fastest cell index
 *                                      counted from 0 (Fig. 2 counts from 1)
 * Cells (Sec. 3.1, Fig. 1): with y_k = t_k - xi_k, t_k = X_k * (n_k / L_k) rounded once in the
 * plan's precision, c_k = floor(y_k) for the 4-point kernels (even support) and the nearest
 * node floor(y_k + 1/2), half-way points going up, for the 3-point kernel (odd support,
 * Fig. 1(b)); then taken modulo n_k.  A point's weights fall on the nodes c_k - 1 .. c_k + 2
 * (even) or c_k - 1 .. c_k + 1 (odd) of each dimension.
 * Dtype: one per plan, IB_F64 or IB_F32, shared by X, F, f, u and U.  Keys, permutations
 * and offsets are int32.
 *
 * Errors: every call returns an ib_status; negative values are errors and leave outputs
 * untouched (argument errors are detected on the host before any launch).  Data errors
 * found on the device (a non-finite coordinate, or |X_k / h_k| >= 2^30) set a device flag
 * reported by ib_plan_status; the results of that update are then unspecified but every
 * memory access stays in bounds.
 */
#ifndef IBOPS_IB_H
#define IBOPS_IB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IB_OK = 0,
    IB_ERR_ARG = -1,          /* invalid argument (null pointer, bad size, bad descriptor) */
    IB_ERR_OOM = -2,          /* workspace too small / host allocation failed */
    IB_ERR_HIP = -3,          /* a HIP runtime call failed */
    IB_ERR_UNSUPPORTED = -4,  /* n_k < 4, more than 2^31-1 cells, unsupported dtype/kernel */
    IB_ERR_BUSY = -5,         /* server queue full */
    IB_ERR_DEVICE_FLAG = -6,  /* a device-side data error was flagged (see above) */
    IB_PENDING = 1            /* batch job not finished yet */
} ib_status;

typedef enum { IB_F64 = 0, IB_F32 = 1 } ib_dtype;

typedef enum {
    IB_KERNEL_PESKIN4 = 0,    /* Peskin's 4-point kernel */
    IB_KERNEL_COSINE4 = 1,    /* phi(r) = (1 + cos(pi r / 2)) / 4 on |r| <= 2 (the paper's choice) */
    IB_KERNEL_ROMA3 = 2       /* the 3-point kernel of Roma, Peskin & Berger (1999): odd support
                                 s = 3, Fig. 1(b): its plans key points by their nearest node and
                                 the operators take the 3^d shifts -1, 0, 1 around it */
} ib_kernel;

#define IB_KERNEL_COUNT 3

typedef struct {
    int32_t dim;              /* 2 or 3 */
    int32_t n[3];             /* cells per dimension, each >= 4; product <= 2^31 - 1 */
    double  length[3];        /* periodic box edge per dimension (> 0); h_k = length_k / n_k */
    int32_t ncomp;            /* grid components, 1..3 (a MAC velocity grid has ncomp = dim) */
    double  stagger[3][3];    /* xi_c in [0,1)^dim per component; MAC: 0.5 - 0.5 e_c */
    int32_t kernel;           /* ib_kernel */
    int32_t walls;            /* non-periodic dimensions: bit k set = dimension k is walled */
} ib_grid_desc;

/* Walled dimensions (the non-periodic boundaries of Sec. 3.1).  Along a walled dimension
 * the grid points are x = h (i + xi) for i = 0 .. n_k - 1 only, with no wrap: a stencil
 * point outside that range is no grid point (the grid indexing function # gives no index),
 * so spreading drops its contribution and interpolation reads nothing there.  Points
 * belong in [0, length_k); a point up to two cells outside still reaches the grid points
 * near the wall; results for points further out are unspecified (no fault).  Positions are
 * advanced without wrap along walled dimensions (ib_advect, ib_interpolate_advect).
 * A walled plan runs on a periodic grid with 4 ghost indices added per walled dimension
 * (n_k + 4; the stencil indices -2 and -1 wrap to n_k + 2 and n_k + 3), whose ghost values
 * are dropped after spreading and zero for interpolation; ib_plan_export's keys index that
 * padded grid.  Batches and the server take periodic jobs only (IB_ERR_UNSUPPORTED). */
#define IB_WALL_GHOSTS 4

typedef struct ib_plan_s *ib_plan;

/* Tuning of a plan; all-zero fields select the built-in choices.
 *   spread_tile   3-D spreading tile (x*y*z cells owned by one block): 1 = 32x16x13,
 *                 2 = 32x8x13, 3 = 64x8x8; 0 = 64x8x8 (2-D grids always use 64x32)
 *   split_points  sharing of a spreading tile by several blocks (at most 256 per tile),
 *                 whose partial tiles a second kernel adds in block order: > 0 = at least
 *                 that many points per block; 0 = about 512 blocks in all, with at least
 *                 128 points per block; < 0 = never share
 *   radix_bits    bucket bits of the key sort (its first pass groups the points by the top
 *                 radix_bits bits of their keys; each bucket is then sorted by one block),
 *                 4..10 for FP64 plans, 4..11 for FP32: 0 = enough buckets for about 2048
 *                 points each, and for at most 8192 cells each
 * Batches take the built-in choices, or one tuning for all their jobs (ib_batch_run_tuned).
 * Results do not depend on the tuning: keys, permutations and offsets are identical, and
 * so are spread and interpolated values, bit for bit (spreading's fixed-point scale depends
 * on the forces and the plan's largest cell count only, and its integer sums on nothing
 * else). */
typedef struct {
    int32_t spread_tile;
    int32_t split_points;
    int32_t radix_bits;
} ib_tuning;

/* Human-readable name of a status code (static string). */
const char *ib_status_string(int32_t status);

/* ---- plans: keys, stable sort, segments (Alg. 4, Sec. 3.4; Fig. 2) -------------------- */

/* Bytes of device workspace a plan for `npts` points needs (0 on invalid arguments).
 * npts may be 0. */
size_t ib_plan_workspace_bytes(const ib_grid_desc *grid, int32_t dtype, int64_t npts);

/* Create a plan.  `workspace` is caller-owned device memory of at least
 * ib_plan_workspace_bytes() bytes (256-byte aligned), kept alive and left untouched by the
 * caller until ib_plan_destroy: it holds the plan's state between calls (its first update
 * clears the counters there; later updates find them cleared by the previous sort).
 * The library never allocates device memory.  The host-side plan object is freed by
 * ib_plan_destroy.  Errors: IB_ERR_ARG, IB_ERR_UNSUPPORTED, IB_ERR_OOM, IB_ERR_HIP. */
int32_t ib_plan_create(const ib_grid_desc *grid, int32_t dtype, int64_t npts,
                       void *workspace, size_t workspace_bytes, ib_plan *out);

/* Number of distinct staggerings among the plan's components (each gets its own keys and
 * sort), and the stagger index of component c. */
int32_t ib_plan_num_staggers(ib_plan plan);
int32_t ib_plan_stagger_of(ib_plan plan, int32_t comp);

/* Recompute the plan for positions X (device, npts x dim, plan dtype): the cell key of
 * every point on the staggering of component 0, the stable ascending sort of the point
 * indices by key (ties keep input order), the first sorted position of every cell, and
 * the positions in that order, which the operators use.  The other staggerings are keyed
 * and sorted, and the number q of distinct keys and the first sorted position of each run
 * are computed, only when ib_plan_export asks for them (from the positions of this update,
 * which the plan keeps).  X is read by this call only. */
int32_t ib_plan_update(ib_plan plan, const void *X, void *stream);

/* The plan of the positions that the last ib_interpolate_advect on this plan produced
 * (written into its X), computed without reading X: the same keys, permutation, offsets
 * and operator results as ib_plan_update(plan, X) with those positions.  The advanced
 * positions are kept by the plan in its sorted order, so the sort reads its input nearly
 * in order.  Needs an ib_interpolate_advect on this plan since its last update (else
 * IB_ERR_ARG; walled plans: always IB_ERR_ARG, use ib_plan_update). */
int32_t ib_plan_update_advected(ib_plan plan, void *stream);

/* Copy one staggering's plan arrays into caller device buffers (any may be NULL):
 * keys[npts] (input order), sorted_keys[npts], perm[npts] (sorted position -> point index),
 * seg_off[q+1] (seg_off[q] = npts; buffer must hold npts+1), q[1].  Stream-ordered after
 * the plan's last update: another staggering is keyed and sorted, and the runs found, by
 * every call that needs them, so a plan updated by a replayed graph exports that update. */
int32_t ib_plan_export(ib_plan plan, int32_t stagger_id, int32_t *keys, int32_t *sorted_keys,
                       int32_t *perm, int32_t *seg_off, int32_t *q, void *stream);

/* Wait for all work on the current device (the plan's work may run on any stream, or
 * replay from a captured graph), then report IB_ERR_DEVICE_FLAG if the last update
 * flagged a data error, else IB_OK (or IB_ERR_HIP).  Clears the flag. */
int32_t ib_plan_status(ib_plan plan);

void ib_plan_destroy(ib_plan plan);

/* As ib_plan_workspace_bytes / ib_plan_create, with a tuning (NULL = defaults).  An
 * out-of-range tuning field gives 0 bytes / IB_ERR_ARG. */
size_t ib_plan_workspace_bytes_tuned(const ib_grid_desc *grid, int32_t dtype, int64_t npts,
                                     const ib_tuning *tuning);
int32_t ib_plan_create_tuned(const ib_grid_desc *grid, int32_t dtype, int64_t npts,
                             const ib_tuning *tuning, void *workspace, size_t workspace_bytes,
                             ib_plan *out);

/* ---- operators ---------------------------------------------------------------------- */

/* Spreading, eq. (disc-spread): f_c(x_i) = (prod_k h_k)^-1 sum_j W_{c,i,j} F_{j,c}, with
 * W = prod_k phi((x_{i,k} - X_{j,k}) / h_k) taken at the nearest periodic image.  F is
 * (npts x ncomp) device, already multiplied by the Lagrangian weights dtheta_j.  f is
 * (ncomp x grid) device; overwritten, or added to when accumulate != 0.  Every grid value
 * is written exactly once.  The sum at each grid value is exact integer arithmetic on its
 * contributions F_{j,c} W, each rounded once to a multiple of 2^-S, where S depends only on
 * max_j |F_{j,c}| and the point counts of the value's tile: so no floating-point atomics
 * are used and the result is bitwise reproducible run to run, whatever the order of work.
 * The rounding adds at most 2^-(S+1) per contribution, below 2^-52 max_j |F_{j,c}| times the
 * bound on contributions per grid value.  A non-finite force makes its component's values
 * NaN. */
int32_t ib_spread(ib_plan plan, const void *F, void *f, int32_t accumulate, void *stream);

/* Interpolation, eq. (disc-interp): U_{j,c} = sum_i W_{c,i,j} u_c(x_i).  u (ncomp x grid)
 * device; U (npts x ncomp) device, overwritten. */
int32_t ib_interpolate(ib_plan plan, const void *u, void *U, void *stream);

/* Interpolation followed by the position update of the IB step, in one pass:
 * U = J(X) u as ib_interpolate, then X <- X + dt U with each coordinate wrapped into
 * [0, length_k) exactly as ib_advect does (bitwise the same results as the two calls).
 * Needs ncomp == dim.  X (npts x dim, device) is the array of the last update (or any
 * array with the same values): it is overwritten in place, after which the plan still
 * serves spreading, interpolation and export at the update's positions.  The advanced
 * positions are also kept by the plan (in its sorted order) for ib_plan_update_advected. */
int32_t ib_interpolate_advect(ib_plan plan, const void *u, void *U, void *X, double dt,
                              void *stream);

/* Position gradient of interpolation, for differentiating through J(X):
 * dX_{j,k} (+)= sum_c W_{j,c} dU_{j,c}/dX_{j,k}, U = J(X) u as in ib_interpolate, where
 * dW/dX_k = (1/h_k) phi'-term: the derivative of the tensor-product weight along axis k.
 * With W = U this is the X-gradient of (1/2)|J(X)u|^2; with u = g and W = F it is the
 * X-gradient of <S(X)F, g>_h (the adjoint pair of eqs. (matrix-interp), (matrix-spread)).
 * u (ncomp x grid), W (npts x ncomp), dX (npts x dim): device, plan dtype.  dX is
 * overwritten, or added to when accumulate != 0. */
int32_t ib_interpolate_grad(ib_plan plan, const void *u, const void *W, void *dX,
                            int32_t accumulate, void *stream);

/* Scaled operators, for the adjoints of Sec. 2's pair J = S^T taken in the grid inner
 * product weighted by prod_k h_k (gradients through spreading and interpolation): each is
 * the operator above with its result multiplied by scale inside the same kernels, with no
 * extra pass over the grid or the points.
 *   ib_spread_scaled:           f (+)= scale * S(X) F; the factor scale * (prod_k h_k)^-1 is
 *                               formed once in FP64 and applied to the exact sums, so the
 *                               result is bitwise reproducible as for ib_spread.
 *   ib_interpolate_scaled:      U = scale * J(X) u, each result times scale (rounded to the
 *                               plan's precision) after its sum.
 *   ib_interpolate_grad_scaled: dX (+)= scale * (the gradient of ib_interpolate_grad), the
 *                               product taken before any accumulation.
 * Arguments, layouts and ownership as for the unscaled calls (which are these with scale 1,
 * bit for bit).  Errors: IB_ERR_ARG for a non-finite scale, plus those of the unscaled calls. */
int32_t ib_spread_scaled(ib_plan plan, const void *F, void *f, double scale, int32_t accumulate,
                         void *stream);
int32_t ib_interpolate_scaled(ib_plan plan, const void *u, void *U, double scale, void *stream);
int32_t ib_interpolate_grad_scaled(ib_plan plan, const void *u, const void *W, void *dX,
                                   double scale, int32_t accumulate, void *stream);

/* Position update of the IB time step, steps (b)/(g) of Sec. 2 with the interpolated
 * velocity: X <- X + dt * U, each coordinate of a periodic dimension wrapped back into
 * [0, length_k) (walled dimensions: no wrap).  X (npts x dim)
 * device, updated in place; U (npts x ncomp) device with ncomp == dim; grid supplies dim and
 * the box.  Errors: IB_ERR_ARG. */
int32_t ib_advect(const ib_grid_desc *grid, int32_t dtype, int64_t npts, void *X, const void *U,
                  double dt, void *stream);

/* Tether force of the unstructured-point test of Sec. 4.1 (each point tied by a Hookean
 * spring of constant k to its initial position): F_{j,c} = k d_{j,c}, where d = X0 - X per
 * coordinate, moved by one box length into [-length_c / 2, length_c / 2) when it lies
 * outside (the nearest periodic image; exact for displacements below half a box); along
 * walled dimensions d is the plain difference.
 * X0, X (npts x dim) and F (npts x ncomp, overwritten) are device arrays of the dtype, with
 * ncomp == dim; grid supplies dim and the box.  Errors: IB_ERR_ARG (k not finite, ncomp !=
 * dim, null pointers with npts > 0), and the descriptor checks of ib_advect. */
int32_t ib_tether_force(const ib_grid_desc *grid, int32_t dtype, int64_t npts, const void *X0,
                        const void *X, double k, void *F, void *stream);

/* ---- batches of independent jobs ---------------------------------------------------- */

/* One job of a batch: a point set on its own grid, with spreading (F -> f) and/or
 * interpolation (u -> U) requested.  Pointers are device pointers in the batch's dtype,
 * with the layouts of ib_spread / ib_interpolate; f == NULL skips spreading, u == NULL
 * skips interpolation.  f and U are overwritten. */
typedef struct {
    ib_grid_desc grid;
    int64_t npts;
    const void *X;   /* npts x dim */
    const void *F;   /* npts x ncomp (may be NULL when f is NULL or npts == 0) */
    void *f;         /* ncomp x grid, or NULL */
    const void *u;   /* ncomp x grid, or NULL */
    void *U;         /* npts x ncomp (may be NULL when u is NULL or npts == 0) */
} ib_job;

#define IB_BATCH_MAX_JOBS 128

/* Bytes of device workspace for a batch (0 on invalid arguments).  All jobs share the
 * dtype, the dimension and the kernel; grids and point counts may differ. */
size_t ib_batch_workspace_bytes(const ib_job *jobs, int32_t njobs, int32_t dtype);

/* Bytes of host staging memory ib_batch_run uses for the job table (0 if njobs is out of
 * range). */
size_t ib_batch_staging_bytes(int32_t njobs);

/* Run the plan (Alg. 4 preparation: keys, stable sort, segments), the spreading and the
 * interpolation of every job of the batch, with one launch per stage for all jobs: each
 * launch covers the blocks of every job, mapped through a job table in the workspace.
 * Results equal those of ib_plan_update + ib_spread + ib_interpolate per job, bit for bit.
 * workspace: caller-owned device memory, >= ib_batch_workspace_bytes, 256-byte aligned,
 * not touched by anyone else until the batch has finished.  host_staging: pinned host
 * memory of ib_batch_staging_bytes(njobs) bytes, left unchanged until the batch has
 * finished; or NULL, in which case the table is uploaded from pageable memory, which makes
 * this call wait for earlier work on the stream.  Asynchronous otherwise.
 * Errors: IB_ERR_ARG, IB_ERR_UNSUPPORTED (njobs > IB_BATCH_MAX_JOBS, mixed dimension or
 * kernel, a bad grid), IB_ERR_OOM (workspace too small), IB_ERR_HIP. */
int32_t ib_batch_run(const ib_job *jobs, int32_t njobs, int32_t dtype, void *workspace,
                     size_t workspace_bytes, void *host_staging, void *stream);

/* A batch with one ib_tuning for all its jobs (NULL: the built-in choices, as above): each
 * job's plan takes the tuning as ib_plan_create_tuned does, so a job's results equal those
 * of a plan created with the same tuning, bit for bit.  The workspace size depends on the
 * tuning; ib_batch_status works as for ib_batch_run.  Errors: those of
 * ib_batch_workspace_bytes (0) and ib_batch_run, and IB_ERR_ARG for a tuning outside its
 * documented ranges. */
size_t ib_batch_workspace_bytes_tuned(const ib_job *jobs, int32_t njobs, int32_t dtype,
                                      const ib_tuning *tuning);
int32_t ib_batch_run_tuned(const ib_job *jobs, int32_t njobs, int32_t dtype, const ib_tuning *tuning,
                           void *workspace, size_t workspace_bytes, void *host_staging, void *stream);

/* Synchronise the stream, then report per job (job_status[j], may be NULL) whether the
 * device flagged a data error in its positions; returns IB_ERR_DEVICE_FLAG if any did.
 * The jobs and workspace must be those of the last ib_batch_run on that workspace. */
int32_t ib_batch_status(const ib_job *jobs, int32_t njobs, int32_t dtype, const void *workspace,
                        int32_t *job_status, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ib_batch_run with the workspace taken
 * from a fixed array of IB_STATIC_SCRATCH_BYTES bytes that the library holds in device memory
 * (one per GPU, until the process ends).  Runs on the current device, whose stream `stream`
 * must be; results equal those of ib_batch_run on the same jobs, bit for bit.  Calls no
 * device or host memory allocator of HIP (no hipMalloc, hipFree, hipHostMalloc).
 * job_flags: device array of njobs words, or NULL; once the batch has finished it holds each
 * job's device error flag (0: none; else the job's positions were flagged as for
 * ib_plan_status), written in stream order.  host_staging as for ib_batch_run.
 * Every call on one GPU uses that GPU's one array, which keeps the last call's contents
 * (each call sets up what it needs itself): calls whose work overlaps on one GPU (other
 * streams, other threads) race and give wrong results; order them on one stream.
 * Errors: IB_ERR_OOM when ib_batch_workspace_bytes(jobs, njobs, dtype) exceeds
 * IB_STATIC_SCRATCH_BYTES (checked before any device work), IB_ERR_HIP if the array's
 * address cannot be taken, and those of ib_batch_run. */
#define IB_STATIC_SCRATCH_BYTES (64u << 20)
int32_t ib_batch_run_static(const ib_job *jobs, int32_t njobs, int32_t dtype, void *host_staging,
                            uint32_t *job_flags, void *stream);

/* ---- serving loop ------------------------------------------------------------------- */

/* A server takes independent jobs one at a time (ib_batch_submit), queues them, and runs
 * them in batches as ib_batch_run does, on a HIP stream of its own (default priority),
 * from a worker thread.  Jobs are admitted into a batch in arrival order while they share
 * the first queued job's dimension and kernel, the batch holds at most
 * max_jobs_per_batch jobs, and the batch's whole device footprint (its plans and job
 * table) fits in the free part of the arena: the caller-owned device memory given at
 * creation, handed out to batches in order and returned as they finish.  At most
 * max_inflight batches are queued on the GPU at once; a new batch takes every compatible
 * job waiting, so batches grow with the load.  A job's latency runs from its arrival (the
 * submit time, or a scheduled arrival time given by the caller) to the moment the worker
 * sees its batch finished.  The server allocates pinned host memory for job tables and
 * flags, and no device memory. */
typedef struct ib_server_s *ib_server;

typedef struct {
    int32_t dtype;               /* ib_dtype of every job */
    int32_t max_jobs_per_batch;  /* 1 .. IB_BATCH_MAX_JOBS (1: one job per launch sequence) */
    int32_t max_inflight;        /* 1 .. 4 batches queued on the GPU at once */
    int32_t max_queue;           /* jobs waiting; ib_batch_submit returns IB_ERR_BUSY beyond */
    int32_t use_graph;           /* which batches replay a captured HIP graph (fixed grids that
                                    loop over the batch's blocks) instead of direct launches:
                                    0 none, k > 0 those of at most k jobs, < 0 all */
} ib_server_opts;

typedef struct {
    uint64_t jobs_done;
    uint64_t batches;
    uint64_t points;
} ib_server_stats;

/* arena: device memory (256-byte aligned) of arena_bytes, kept alive until destroy; its
 * first 4 job-table slots (about 0.6 MB) are reserved, the rest holds the batches' plans.
 * The current HIP device is the server's.  Errors: IB_ERR_ARG, IB_ERR_UNSUPPORTED,
 * IB_ERR_OOM (arena too small for the tables), IB_ERR_HIP. */
int32_t ib_server_create(const ib_server_opts *opts, void *arena, size_t arena_bytes,
                         ib_server *out);

/* Microseconds since the server was created (the clock of arrival times and latencies). */
double ib_server_clock_us(ib_server server);

/* Queue a job (non-blocking).  arrival_us < 0 means now.  The job's input buffers must
 * already hold their final values when this is called: the server reads them on its own
 * stream without waiting for work queued on any other stream (synchronise the stream that
 * produced them first).  The job's buffers must stay valid and unchanged until
 * ib_batch_poll reports it finished.  Errors: IB_ERR_ARG (bad job),
 * IB_ERR_OOM (its footprint exceeds the whole arena), IB_ERR_BUSY (queue full). */
int32_t ib_batch_submit(ib_server server, const ib_job *job, double arrival_us, uint64_t *ticket);

/* IB_PENDING while the job waits or runs; then, once, its final status (IB_OK,
 * IB_ERR_DEVICE_FLAG, IB_ERR_HIP) with its latency in microseconds.  IB_ERR_ARG for an
 * unknown or already reported ticket. */
int32_t ib_batch_poll(ib_server server, uint64_t ticket, double *latency_us);

/* Block until every submitted job has finished. */
int32_t ib_server_drain(ib_server server);

int32_t ib_server_get_stats(ib_server server, ib_server_stats *out);

/* Finish all queued and running jobs, then free the server. */
void ib_server_destroy(ib_server server);

#ifdef __cplusplus
}
#endif

#endif /* IBOPS_IB_H */

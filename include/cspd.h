/*
 * cspd -- batched cross-scale (zero-tree) orthogonal matching pursuit on
 * AMD Instinct MI355X (gfx950).
 *
 * The problem every call solves, per patch (Section III-C of Saragadam, Li,
 * Sankaranarayanan, "Cross-Scale Predictive Dictionaries"):
 *
 *     y = Phi x + e,   x = D_high s_high,   ||s_high||_0 <= K_high,
 *
 * with a chain of S dictionaries D_0 (coarsest) ... D_{S-1} = D_high in
 * which fine atom j is a child of atom floor(j / Q_s) one scale up (the
 * non-overlapping child blocks of Section III-B, 0-based).  Scale 0 is
 * problem (P_low): OMP against the effective dictionary Phi U D_0, where U
 * replicates a coarse sample over its block (nearest-neighbour upsampler,
 * W U = I for the box-average down-sampler W).  Every finer scale is
 * problem (P_high): OMP restarted from y over the children of the previous
 * scale's support only (Algorithm 2, chained down the tree of Fig. 2).
 * cspd_omp_full is Algorithm 1 over every atom of D_high.
 *
 * Conventions for every entry point:
 *   - "host" pointers are read during the call only; "device" pointers are
 *     device memory of the plan's device, owned by the caller, and must stay
 *     valid until the stream passed to the call has completed the work.
 *   - Compute calls are stream-ordered: they enqueue kernels on `hip_stream`
 *     (a hipStream_t; NULL = the default stream) and return without waiting.
 *   - Matrices are dense; "column-major R x C" means element (r, c) at
 *     c * R + r; "row-major R x C" means element (r, c) at r * C + c.
 *   - Floating-point device buffers have the plan's dtype (double for
 *     CSPD_F64, float for CSPD_F32).
 *   - Errors are returned as negative cspd_status codes; nothing aborts or
 *     throws across this interface.  On error the outputs are undefined.  A
 *     message for the last error on the calling thread is available from
 *     cspd_last_error().
 *   - Early termination of one patch (its candidates ran out, or the picked
 *     atom is numerically dependent on the atoms already chosen) is not an
 *     error: it shows as k_used < K and -1 padding in the support.
 */
#ifndef CSPD_H
#define CSPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSPD_MAX_SCALES 4

typedef int32_t cspd_status;
enum {
    CSPD_OK = 0,
    CSPD_E_INVALID = -1,     /* null pointer, bad enum, negative size */
    CSPD_E_SHAPE = -2,       /* inconsistent dimensions (e.g. T_s != Q T_{s-1}, K > k_max) */
    CSPD_E_NOMEM = -3,       /* device or host allocation failed */
    CSPD_E_DEVICE = -4,      /* a HIP runtime call or kernel launch failed */
    CSPD_E_BUSY = -5,        /* serving: the job has not finished yet */
    CSPD_E_NOTFOUND = -6,    /* serving: unknown job id */
    CSPD_E_CAPACITY = -7,    /* serving: the job can never fit the HBM budget */
    CSPD_E_UNSUPPORTED = -8  /* a shape the library has no kernel for */
};

/* Measurement operator Phi (Section III-C). */
enum {
    CSPD_PHI_IDENTITY = 0,   /* Phi = I (denoising); M = N */
    CSPD_PHI_DENSE = 1,      /* one dense M x N matrix shared by all patches */
    CSPD_PHI_MASK = 2        /* Phi = diag(mask_b) per patch (inpainting); M = N */
};

enum { CSPD_F64 = 0, CSPD_F32 = 1 };

/* How the full-dictionary proxy is evaluated (not in the paper: a precision
 * option).  NATIVE computes correlations in the plan's dtype; the two
 * RESCORE modes compute them with bf16 / fp16 matrix cores and FP32
 * accumulation, and re-score in FP32 (exact correlations and norms) the
 * rescore_m candidates of each patch with the best reduced-precision scores
 * (an exact per-patch top-m, ties to the lower atom index) before the argmax:
 * in full OMP at every iteration; in cross-scale OMP at the first scale,
 * whose correlations with y come from one batched contraction (shared dense
 * operator), the top rescore_m by current score at every iteration (a
 * candidate re-scored once stays exact). */
enum { CSPD_CORR_NATIVE = 0, CSPD_CORR_BF16_RESCORE = 1, CSPD_CORR_F16_RESCORE = 2 };

/*
 * Plan description (Section III-A's model, Section III-B's map, Section
 * III-C's operators).
 *   n_scales   S, 1 <= S <= CSPD_MAX_SCALES (S = 1 is plain OMP).
 *   dim[s]     N_s, signal dimension at scale s (coarse -> fine); N = dim[S-1].
 *   atoms[s]   T_s; must satisfy T_s = Q_s T_{s-1} with integer Q_s >= 1.
 *   dict[s]    host, column-major dim[s] x atoms[s], FP64 (converted on the
 *              device to the plan's dtype).
 *   up_map[s]  host, s < S-1: length dim[s+1]; entry j is the scale-s
 *              coordinate that fine coordinate j copies under U (and that W
 *              averages it into).  Must be onto [0, dim[s]).
 *   phi_kind   CSPD_PHI_*.
 *   m          M, rows of Phi (must equal N unless CSPD_PHI_DENSE).
 *   phi        host, row-major M x N, FP64 (CSPD_PHI_DENSE only, else NULL).
 *   dtype      CSPD_F32 or CSPD_F64.
 *   corr_mode  CSPD_CORR_* (RESCORE modes need CSPD_F32).
 *   rescore_m  candidates re-scored per patch in RESCORE modes (1..16; 0 = 8).
 *   k_max      largest sparsity any call will ask for at any scale; the
 *              row stride of the support / coef outputs.
 *   device     HIP device ordinal the plan lives on.
 *   n_phases   CSPD_PHI_DENSE only: number of dense operators (0 or 1: one).
 *              With P > 1, phi holds P row-major M x N operators back to back
 *              and every patch is measured with one of them, chosen per call
 *              (cspd_omp_cross_scale_phased): location-dependent measurement
 *              such as a coded-exposure shutter pattern whose tile differs
 *              with the patch position (Section IV, videos).  1 <= P <= 4096.
 */
typedef struct cspd_plan_desc {
    int32_t n_scales;
    int32_t dim[CSPD_MAX_SCALES];
    int32_t atoms[CSPD_MAX_SCALES];
    const double *dict[CSPD_MAX_SCALES];
    const int32_t *up_map[CSPD_MAX_SCALES];
    int32_t phi_kind;
    int32_t m;
    const double *phi;
    int32_t dtype;
    int32_t corr_mode;
    int32_t rescore_m;
    int32_t k_max;
    int32_t device;
    int32_t n_phases;
} cspd_plan_desc;

typedef struct cspd_plan_s *cspd_plan_t;
typedef struct cspd_graph_s *cspd_graph_t;

/*
 * Build a plan: validate the description, upload the dictionaries and Phi,
 * and compute on the device the effective dictionaries A_s = Phi U D_s
 * (Section III-C, (P_low) / (P_high)) with their column norms, plus the
 * block tables of U.  Blocks until the plan is resident.  The plan owns all
 * of its device memory; release it with cspd_plan_destroy.  The compute
 * calls take their workspace from the device's default stream-ordered memory
 * pool and free it at the end of the call; the first plan on a device raises
 * that pool's release threshold to 2 GiB (never lowers it), so that freed
 * workspace stays in the pool between calls instead of being mapped afresh.
 * Errors: E_INVALID, E_SHAPE (among others: atoms[s] not a multiple of
 * atoms[s-1], or 2^22 or more children per atom), E_NOMEM, E_DEVICE.
 */
cspd_status cspd_plan(const cspd_plan_desc *desc, cspd_plan_t *out);

/* Release a plan (waits for the device; NULL is ignored). */
void cspd_plan_destroy(cspd_plan_t plan);

/* Bytes of device memory the plan holds (dictionaries, tables). */
int64_t cspd_plan_device_bytes(cspd_plan_t plan);

/*
 * Algorithm 1 (orthogonal matching pursuit) over every atom of D_high, for B
 * independent patches.
 *   B          number of patches (0 is allowed: nothing is launched).
 *   y          device, row-major B x M measurements.
 *   mask       device, row-major B x N uint8 (nonzero = observed), required
 *              for CSPD_PHI_MASK and ignored otherwise.
 *   k          device int32[B] per-patch sparsity, or NULL to use k_uniform.
 *              Each K must lie in [0, k_max]; K is capped at T and at M.
 *   support    device, row-major B x k_max int32 out: indices into D_high in
 *              selection order, -1 padded.
 *   coef       device, row-major B x k_max out: coefficients of those
 *              columns of D_high (least-squares solution on the support).
 *   k_used     device int32[B] out: atoms actually selected.
 *   xhat       device, row-major B x N out (may be NULL): D_high s_high.
 * Errors: E_INVALID, E_SHAPE, E_UNSUPPORTED, E_DEVICE, E_NOMEM.
 */
cspd_status cspd_omp_full(cspd_plan_t plan, int64_t B, const void *y, const uint8_t *mask,
                          const int32_t *k, int32_t k_uniform, int32_t *support, void *coef,
                          int32_t *k_used, void *xhat, void *hip_stream);

/*
 * Zero-tree OMP (Algorithm 2, chained over the S scales of the plan).
 *   k_scale        host int32[S-1]: sparsity of scales 0..S-2 (each capped
 *                  at the number of candidates, Q_s times the previous k).
 *   k_fine         device int32[B] per-patch sparsity of the finest scale,
 *                  or NULL to use k_fine_uniform (capped at Q k_{S-2}).
 *   support_coarse device, row-major B x (k_scale[0] + ... + k_scale[S-2])
 *                  int32 out (may be NULL): each coarser scale's support in
 *                  selection order, -1 padded, scales concatenated.
 *   other arguments as for cspd_omp_full.  With S = 1 this is cspd_omp_full.
 */
cspd_status cspd_omp_cross_scale(cspd_plan_t plan, int64_t B, const void *y, const uint8_t *mask,
                                 const int32_t *k_scale, const int32_t *k_fine,
                                 int32_t k_fine_uniform, int32_t *support, void *coef,
                                 int32_t *k_used, void *xhat, int32_t *support_coarse,
                                 void *hip_stream);

/*
 * Zero-tree OMP (or, for S = 1, full OMP) with a per-patch operator chosen
 * from the plan's n_phases dense operators (Section III-C's y = Phi x + e
 * with Phi depending on the patch's position, e.g. a coded-exposure pattern
 * that is not the same over every patch).
 *   phase      device int32[B]: the operator of each patch, in [0, n_phases);
 *              a patch whose phase is outside that range is not solved
 *              (k_used 0, support -1, coefficients and x-hat 0).
 *   other arguments as for cspd_omp_cross_scale.
 * Plans with one operator accept phase = NULL (every patch uses it).
 * Errors: as for cspd_omp_cross_scale; E_INVALID for a NULL phase on a plan
 * with several operators.
 */
cspd_status cspd_omp_cross_scale_phased(cspd_plan_t plan, int64_t B, const int32_t *phase, const void *y,
                                        const uint8_t *mask, const int32_t *k_scale, const int32_t *k_fine,
                                        int32_t k_fine_uniform, int32_t *support, void *coef, int32_t *k_used,
                                        void *xhat, int32_t *support_coarse, void *hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as cspd_omp_cross_scale, same arguments, same kernels and results,
 * but its workspace (the coarse scales' k_used and supports, and scale 0's
 * correlations under a shared dense Phi) lives in a static device array of
 * CSPD_NOALLOC_SCRATCH_BYTES per GPU, reserved when the library's code loads
 * and held until the process ends; its address on a device is resolved once,
 * by the first cspd_plan on that device.  The call allocates nothing.  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams, or from different threads) race and must be serialised
 * by the caller (e.g. one stream).  Passing support_coarse lowers the
 * workspace to 4 (S - 1) bytes per patch (plus 4 T_0 under a dense Phi).
 * Errors: as for cspd_omp_cross_scale (no E_NOMEM), and E_CAPACITY when the
 * call's workspace exceeds CSPD_NOALLOC_SCRATCH_BYTES (checked on the host,
 * before anything is launched).
 */
#define CSPD_NOALLOC_SCRATCH_BYTES 33554432 /* 32 MiB */
cspd_status cspd_omp_cross_scale_noalloc(cspd_plan_t plan, int64_t B, const void *y, const uint8_t *mask,
                                         const int32_t *k_scale, const int32_t *k_fine,
                                         int32_t k_fine_uniform, int32_t *support, void *coef,
                                         int32_t *k_used, void *xhat, int32_t *support_coarse,
                                         void *hip_stream);

/*
 * A cross-scale call (or, for S = 1, a full-dictionary call) captured once
 * into a HIP graph for a fixed batch and fixed buffers: every scale's kernel
 * is one node, and a replay launches them all with one graph launch, without
 * host work or allocation per call.  The graph owns its workspace (allocated
 * here).  Arguments as for cspd_omp_cross_scale, without a stream; the
 * buffers must outlive the graph, and their contents may change between
 * replays (the graph reads them when it runs).  Replays on one graph must not
 * overlap (they share the workspace).  Errors as for the call, E_INVALID for
 * B = 0, E_DEVICE when capture or instantiation fails.
 */
cspd_status cspd_graph_cross_scale(cspd_plan_t plan, int64_t B, const void *y, const uint8_t *mask,
                                   const int32_t *k_scale, const int32_t *k_fine,
                                   int32_t k_fine_uniform, int32_t *support, void *coef,
                                   int32_t *k_used, void *xhat, int32_t *support_coarse,
                                   cspd_graph_t *out);
/* Replay a captured call on a HIP stream (stream-ordered). */
cspd_status cspd_graph_launch(cspd_graph_t graph, void *hip_stream);
/* Free the graph (waits until the device is idle) and its workspace. */
void cspd_graph_destroy(cspd_graph_t graph);

/*
 * Autotuner (not in the paper: kernel selection for Algorithm 2's scales).
 * Runs the cross-scale call once on the caller's batch, then, scale by
 * scale, times every kernel variant that can run that scale (the
 * first-scale matrix-core kernel, the per-patch Gram on the matrix cores,
 * each vector layout, the precomputed-Gram kernel), `reps` launches each,
 * and keeps the fastest in the plan, keyed by scale, by the scale's
 * sparsity bucket (K <= 4, <= 8, <= 16) and by its candidate count.  Later
 * cross-scale calls (and graphs captured after) with the same key use it;
 * other keys keep the shape rules.  Every variant computes the same result
 * up to FP32 rounding order.  Arguments as for cspd_omp_cross_scale (inputs
 * only: outputs go to scratch allocated and freed here); blocks until done.
 * FP32 plans with S >= 2 only (others: no-op).  Errors: as for the call,
 * E_INVALID for reps outside 1..1000, E_NOMEM for the scratch.
 */
cspd_status cspd_autotune(cspd_plan_t plan, int64_t B, const void *y, const uint8_t *mask,
                          const int32_t *k_scale, const int32_t *k_fine, int32_t k_fine_uniform,
                          int32_t reps, void *hip_stream);
/*
 * The plan's tuned kernel for (scale, bucket 0..2): kind 0 = none (shape
 * rules), 1 = first-scale matrix-core, 2 = vector layout (nc column chunks,
 * ppw patches per wavefront), 3 = precomputed Gram, 4 = per-patch Gram on
 * the matrix cores, 5 = batched correlation GEMM then precomputed Gram
 * (scale 0 under a shared dense operator); cand = candidate count it was
 * timed on.
 * Errors: E_INVALID for a NULL argument or an index out of range.
 */
cspd_status cspd_tuned_kernel(cspd_plan_t plan, int32_t scale, int32_t bucket, int32_t *kind, int32_t *nc,
                              int32_t *ppw, int32_t *cand);
/*
 * Pin a kernel for (scale, bucket, cand), e.g. one read back from
 * cspd_tuned_kernel in an earlier process, without timing; kind 0 clears
 * the entry (shape rules again).  Errors: E_INVALID for an index out of
 * range or cand outside 1..T of the scale, E_UNSUPPORTED when the variant
 * cannot run that scale at that candidate count.
 */
cspd_status cspd_set_tuned_kernel(cspd_plan_t plan, int32_t scale, int32_t bucket, int32_t kind, int32_t nc,
                                  int32_t ppw, int32_t cand);

/* ---------------------------------------------------------------------- */
/* Whole signals: overlapping patches in, averaged estimates out.           */
/* (Section IV processes images, videos and light fields as overlapping     */
/* patches; the grid and the averaging below are this library's reading.)  */
/* ---------------------------------------------------------------------- */

/*
 * A patch grid over a signal of ndim (1..4) axes, row-major (last axis
 * fastest): along axis d patches of patch[d] samples start at 0, stride[d],
 * 2 stride[d], ... and, when the last of these does not reach the end, once
 * more at dims[d] - patch[d], so every sample is covered.  Patches are
 * numbered row-major over the grid; a patch is vectorised row-major over its
 * own axes (image (y, x), video (t, y, x), light field (u, v, y, x)), which
 * is the coordinate order of the plan's finest dictionary.
 */
typedef struct cspd_patch_grid {
    int32_t ndim;
    int32_t dims[4];
    int32_t patch[4];
    int32_t stride[4];
} cspd_patch_grid;

/* Number of patches of the grid, or -1 for an invalid grid (message in
 * cspd_last_error): 1 <= patch <= dims, stride >= 1, patch volume <= 65,536. */
int64_t cspd_patch_count(const cspd_patch_grid *grid);

/*
 * Cut a signal into its patches (stream-ordered).
 *   signal      device float, the signal (prod(dims) samples).
 *   mask        device uint8 of the same shape (nonzero = observed), or NULL.
 *   y           device float out, count x prod(patch), row-major.
 *   patch_mask  device uint8 out of the same shape as y (the mask's samples,
 *               or all 1 when mask is NULL), or NULL.
 * Errors: E_INVALID, E_SHAPE, E_DEVICE.
 */
cspd_status cspd_extract_patches(const cspd_patch_grid *grid, const float *signal, const uint8_t *mask, float *y,
                                 uint8_t *patch_mask, void *hip_stream);

/*
 * Put patch estimates back together (stream-ordered): every sample of
 * signal_out is the mean (accumulated in FP64) of the estimates of all the
 * patches that cover it, visited in grid order.
 *   estimates   device float, count x prod(patch) (e.g. the x-hat of an OMP call).
 *   signal_out  device float out, prod(dims) samples.
 * Errors: E_INVALID, E_SHAPE, E_DEVICE.
 */
cspd_status cspd_aggregate_patches(const cspd_patch_grid *grid, const float *estimates, float *signal_out,
                                   void *hip_stream);

/* ---------------------------------------------------------------------- */
/* Learning the dictionaries (Section III-E): the K-SVD dictionary update.  */
/* ---------------------------------------------------------------------- */

/*
 * One sweep of the K-SVD dictionary update after a sparse-approximation step
 * (cspd_omp_full for plain K-SVD, cspd_omp_cross_scale for the cross-scale
 * variant whose supports stay inside the children of the coarse support).
 * Atoms are updated in index order, each seeing the previous updates: the
 * users of atom k (signals whose support holds it), the error without it
 * E_k = R_users + s_k d_k^T, the new atom = leading left singular vector of
 * E_k^T (sign kept towards the old atom), the users' coefficients E_k d_k,
 * and the residual minus the new rank-1 term.  An atom without users keeps
 * its value.  The sweep is deterministic.
 *   x        device float, row-major P x N training signals.
 *   dict     device float, row-major T x N atoms (one atom per row), in/out;
 *            N <= 64.
 *   support  device int32, row-major P x kstride (the OMP call's support,
 *            -1 padded; entries must be distinct per row).
 *   coef     device float, row-major P x kstride, in/out (the OMP call's
 *            coefficients; updated for every used slot).
 * Stream-ordered (workspace allocated and freed on the stream).
 * Errors: E_INVALID, E_SHAPE, E_NOMEM, E_DEVICE.
 */
cspd_status cspd_ksvd_update(const float *x, int64_t P, int32_t N, float *dict, int32_t T, const int32_t *support,
                             float *coef, int32_t kstride, void *hip_stream);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of reconstruction jobs on one device.      */
/* (Not in the paper: a request loop around the calls above.)             */
/* ---------------------------------------------------------------------- */
typedef struct cspd_server_s *cspd_server_t;

/*
 * One reconstruction job.  With on_device = 0, inputs and outputs are HOST
 * buffers, read and written by the server's copy engine; with on_device != 0
 * they are DEVICE buffers on the server's device, which the launches read
 * and write in place (no copies; the job's pieces are not packed with other
 * jobs; per-patch k_fine is then not checked on the host, the kernels clamp
 * it to [0, k_max]).  Either way they must stay valid until cspd_serve_poll
 * has returned CSPD_OK for the job.
 *   plan      a resident plan (jobs of several plans may be in flight).
 *   B         patches; y: B x M; mask: B x N or NULL; k_fine: int32[B] or
 *             NULL (then k_fine_uniform); k_scale: int32[S-1] (copied at
 *             submit).
 *   full      nonzero: Algorithm 1 over D_high instead of zero-tree OMP.
 *   outputs   support / k_used required, coef / xhat optional (NULL).
 */
typedef struct cspd_job {
    cspd_plan_t plan;
    int64_t B;
    const void *y;
    const uint8_t *mask;
    const int32_t *k_fine;
    int32_t k_fine_uniform;
    int32_t k_scale[CSPD_MAX_SCALES];
    int32_t full;
    int32_t *support;
    void *coef;
    int32_t *k_used;
    void *xhat;
    int32_t on_device;
} cspd_job;

/* Timestamps (CLOCK_MONOTONIC nanoseconds) of one finished job. */
typedef struct cspd_job_stats {
    int64_t submit_ns;   /* cspd_serve_submit called */
    int64_t admit_ns;    /* device memory and a slot granted (first piece) */
    int64_t start_ns;    /* its first launch was enqueued */
    int64_t finish_ns;   /* its results were back in host memory */
    int64_t patches;
    int32_t batched_with; /* most other jobs that shared one of its launches */
    int32_t status;      /* CSPD_OK or the error that failed the job */
    int64_t server_resident_bytes; /* device bytes the server held when the job finished */
} cspd_job_stats;

/*
 * Create a server on `device` with an HBM budget for job buffers (bytes,
 * > 0) and at most `max_slots` (1..64) launches in flight, each on its own
 * stream.  Jobs are cut into pieces of at most 65,536 patches.  A
 * background thread admits queued pieces when their buffers fit in the
 * budget, packs waiting pieces of the same plan and kind into one launch (at
 * most 65,536 patches), copies in, launches, copies out and retires them; a
 * job finishes with its last piece.  Pieces are admitted in arrival order,
 * except that pieces of small jobs (at most 8,192 patches) go first while the
 * oldest waiting piece has waited less than 5 ms, and with three or more
 * slots the last free slot is kept for small jobs.  Each slot keeps its device buffers from
 * launch to launch (grown to its largest launch); the budget bounds every
 * byte the server holds on the device: all slots' buffers, in flight or
 * idle, and an idle slot's buffers are released when a launch would not fit
 * otherwise.  Everything is freed by cspd_serve_destroy.
 * Errors: E_INVALID, E_DEVICE, E_NOMEM.
 */
cspd_status cspd_serve_create(int32_t device, int64_t hbm_budget_bytes, int32_t max_slots,
                              cspd_server_t *out);

/* Queue a job (non-blocking).  E_CAPACITY if one of its pieces can never
 * fit the budget; E_INVALID / E_SHAPE for a malformed job. */
cspd_status cspd_serve_submit(cspd_server_t server, const cspd_job *job, uint64_t *job_id);

/* Wait up to timeout_us (0 = just look, < 0 = forever) for a job.  Returns
 * CSPD_OK and fills *stats when it has finished (the job is then forgotten),
 * E_BUSY if still pending, E_NOTFOUND for an unknown id, or the job's own
 * error code if it failed. */
cspd_status cspd_serve_poll(cspd_server_t server, uint64_t job_id, int64_t timeout_us,
                            cspd_job_stats *stats);

/* Drain the queue, stop the thread and free everything. */
void cspd_serve_destroy(cspd_server_t server);

/* ---------------------------------------------------------------------- */
/* Kernel timing (measurement tools; not in the paper).                    */
/* ---------------------------------------------------------------------- */
/*
 * cspd_profile_enable(1) makes every kernel launch of the compute calls
 * record a pair of HIP events on the stream it is launched on, labelled with
 * the kernel's name; 0 stops recording.  cspd_profile_read synchronizes the
 * recorded events and reports entry `idx` (0-based, in order of first
 * appearance): its label (copied into `name`, at most name_len bytes with the
 * terminator), the number of launches and their summed duration in
 * milliseconds.  It returns the number of entries, or a negative status.
 * cspd_profile_reset drops every record.  Recording costs two events per
 * launch; leave it off outside measurements.
 */
cspd_status cspd_profile_enable(int32_t on);
int32_t cspd_profile_read(int32_t idx, char *name, int32_t name_len, int64_t *launches,
                          double *total_ms);
void cspd_profile_reset(void);

/* Message for the last error raised on the calling thread ("" if none). */
const char *cspd_last_error(void);

/* Library version string. */
const char *cspd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CSPD_H */

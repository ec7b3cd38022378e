/*
 * vgicp.h -- C ABI of the MI355X (gfx950) VGICP factor-linearization library.
 *
 * What it computes (GLIM, Koide et al. 2024, Sec. III-C "Matching Cost Factor"):
 * a factor matches a source Gaussian point cloud {(mu_k, C_k)} into the
 * multi-resolution Gaussian voxel map of a target cloud {(mu~, C~) per voxel,
 * levels r_l = r_0 2^(l-1)}.  At a relative pose T = (R, t) that maps source
 * points into the target frame, every source point is transformed
 * (y = R mu + t), its voxel q = floor(y / r_l) is looked up at every level
 * (Sec. III-C "Correspondence search"), and each hit contributes
 *     d = mu~ - y,  W = (C~ + R C R^T)^-1,  e += d^T W d      (Eq. (em), Eq. (d2d))
 *     J = [R (mu)x, -R],  H += J^T W J,  b += J^T W d         (Sec. III-C "Linearization")
 * with W frozen at the linearization point.  All factors of a batch are
 * linearized with one upload of the poses and one download of the results
 * (Sec. III-C "Implementation").
 *
 * Conventions shared by every entry point:
 *   - A pose is 12 doubles, row-major R (9) then t (3); it maps source-frame
 *     points into the target frame.
 *   - H (6x6, row-major) and b (6) are derivatives w.r.t. a right perturbation
 *     T Exp(xi), xi = [omega; v] (rotation first).  e has no factor 1/2, so
 *     e(T Exp(xi)) ~ e + 2 b^T xi + xi^T H xi and the Gauss-Newton step is
 *     -H^-1 b.
 *   - Covariances are 6 doubles per point: xx, xy, xz, yy, yz, zz.
 *   - Resolutions are ascending and each is the previous one times a power of
 *     two, and every resolution is itself a power of two (so y / r is exact).
 *   - Voxel keys are limited to |q - q_origin| < 8192 per axis around the map
 *     origin (the first point snapped to the coarsest voxel), and a level holds
 *     fewer than 67,108,864 voxels.
 *
 * Error behaviour: every call returns a vg_status (0 = VG_OK).  No exception
 * crosses the ABI.  On failure vg_last_error() returns a message that stays
 * valid until the next call on the same thread.  Arguments are validated on
 * the host before any device work is queued; a failed call leaves its outputs
 * unspecified and its handles usable.
 *
 * Ownership: input arrays are read during the call and never retained;
 * handles are owned by the caller and released with the matching *_destroy.
 * A batch keeps references to its sources and voxel maps: destroying one of
 * them while a batch uses it fails with VG_ERR_STATE.  Device pointers passed
 * to *_async calls stay owned by the caller and must remain valid until the
 * queued work completes on the context stream.
 *
 * Threading: a context and everything created from it must be used by one
 * thread at a time.  Calls that share a context are ordered on its stream.
 */
#ifndef VGICP_H
#define VGICP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VG_OK = 0,
    VG_ERR_INVALID_ARG = -1, /* a pointer, size, pose or option is invalid */
    VG_ERR_HIP = -2,         /* a HIP runtime call failed (message has the HIP string) */
    VG_ERR_OOM = -3,         /* device or pinned host allocation failed */
    VG_ERR_KEY_RANGE = -4,   /* a target voxel key lies outside the packable range */
    VG_ERR_CAPACITY = -5,    /* too many voxels in one level */
    VG_ERR_NOT_SPD = -6,     /* an input covariance is not symmetric positive definite */
    VG_ERR_STATE = -7        /* handle in use, destroyed, or from another context */
} vg_status;

/* Precision of a batch.  Re-centring is part of the compensated mode, not a
 * separate switch: that mode stores every source point as an FP32 offset from
 * an FP64 anchor of its 64-point chunk and every voxel mean relative to its
 * voxel centre, so there are no absolute FP32 coordinates to re-centre, and
 * VG_FP32 is the absolute-coordinate (not re-centred) form.  The compensated
 * mode is value 0 so that zero-initialised options select it. */
typedef enum {
    VG_FP32_COMPENSATED = 0, /* FP32 terms in re-centred coordinates; residual and fused
                                covariance formed in FP64; FP64 sums across lanes, waves,
                                tiles and factors (the default).  Sources must lie within
                                500 m of their origin (the first point rounded to a metre):
                                the per-point lever arms are FP32, and beyond that the
                                relative error of b can exceed 1e-5.  A batch with a larger
                                source is refused (VG_ERR_INVALID_ARG); use VG_FP64. */
    VG_FP32 = 1,             /* absolute FP32 coordinates, FP32 accumulation end to end */
    VG_FP64 = 2              /* FP64 data and arithmetic throughout */
} vg_precision;

typedef struct vg_context vg_context;
typedef struct vg_voxelmap vg_voxelmap;
typedef struct vg_source vg_source;
typedef struct vg_batch vg_batch;

/* Options of a factor batch.  Zero-initialize, then set what you need; a zero
 * tuning field means "use the default, or the tuned value if tune_cache is set". */
typedef struct {
    int32_t precision;          /* a vg_precision value */
    int32_t surface_validation; /* 1: discard a point when (mu - T^-1 c) . n > 0 (Sec. III-C,
                                   Correspondence search); sources need normals, c is the
                                   target viewpoint of the factor */
    int32_t use_graph;          /* 1: replay a captured hipGraph [H2D, kernels, D2H] */
    int32_t plain_per_factor;   /* 1: one launch, one upload, one download and one host
                                   synchronization per factor (the per-factor loop the
                                   batched mechanism replaces) */
    int32_t block_threads;      /* 64, 128, 256 or 512 threads per workgroup; 0 = default */
    int32_t tile_points;        /* source points per work tile, a multiple of 64 up to 32768;
                                   0 = default */
    int32_t blocks_per_cu;      /* persistent workgroups per compute unit; 0 = default */
    int32_t lane_kahan;         /* VG_FP32_COMPENSATED only: 1 = Kahan-compensated FP32 sums
                                   inside each lane (sums above a lane are FP64 either way) */
    const char* tune_cache;     /* NULL: no autotuning.  Otherwise a file path: tuned shapes
                                   are read from it, or measured and appended to it */
    int32_t tile_order;         /* order in which the persistent grid takes tiles: 0 default
                                   (1), 1 = eight contiguous ranges, one per XCD, 2 = tiles
                                   dealt round-robin to the eight XCDs (all XCDs work in
                                   the same window of factors); results are identical */
} vg_batch_options;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t that
 * all work is queued on (borrowed, not destroyed); NULL creates a private one. */
vg_status vg_context_create(int32_t device, void* hip_stream, vg_context** out);
vg_status vg_context_destroy(vg_context* ctx);
/* Thread-local message of the last failed call ("" if none). */
const char* vg_last_error(void);
/* Library version: major * 10000 + minor * 100 + patch. */
int32_t vg_version(void);

/* ---- voxel maps (Sec. III-C, Preprocessing) ------------------------------ */

/* Build the Gaussian voxel map of a target cloud: for every level l, each point
 * x falls in voxel floor(x / r_l); a voxel stores the average of its points'
 * means and the average of their covariances (summed in FP64 in ascending point
 * order).  xyz: n x 3, cov: n x 6 (host, FP64).  n may be 0 (empty map).
 * Errors: VG_ERR_INVALID_ARG (non-finite input, bad resolutions, L outside
 * 1..4), VG_ERR_KEY_RANGE, VG_ERR_CAPACITY, VG_ERR_OOM, VG_ERR_HIP. */
vg_status vg_build_voxelmap(vg_context* ctx, const double* xyz, const double* cov, int64_t n,
                            const double* resolutions, int32_t L, vg_voxelmap** out);
/* Number of voxels of a level and the capacity (entries) of its block table:
 * voxels are grouped in 4x4x4 blocks, one hash entry per occupied block. */
vg_status vg_voxelmap_info(const vg_voxelmap* map, int32_t level, int64_t* n_voxels,
                           int64_t* capacity);
/* Copy a level to the host in canonical order (ascending lexicographic key):
 * the per-voxel mean of the member points' means and mean of their
 * covariances (Sec. III-C, Preprocessing), for parity checks.
 * Any output may be NULL.  keys: V x 3 absolute voxel coordinates; means: V x 3
 * and covs: V x 6 in FP64; counts: V.  `n_voxels` is in/out: capacity of the
 * outputs on entry, voxel count on return (VG_ERR_INVALID_ARG if too small). */
vg_status vg_voxelmap_export(const vg_voxelmap* map, int32_t level, int64_t* n_voxels, int64_t* keys,
                             double* means, double* covs, int64_t* counts);
vg_status vg_voxelmap_destroy(vg_voxelmap* map);

/* ---- source clouds ---------------------------------------------------- */

/* Upload a source Gaussian cloud (host FP64: xyz n x 3, cov n x 6, normals n x 3
 * or NULL).  The library reorders points internally along a Morton curve and
 * stores them relative to per-64-point anchors, with a ball and a box that
 * bound each 64-point chunk (chunks that cannot reach a target's voxels are
 * skipped by the kernels); every per-point output of the library is reported
 * in the caller's order.  Covariances must be SPD (VG_ERR_NOT_SPD otherwise).
 * n < 2^27 (the kernels address a source's arrays with 32-bit offsets). */
vg_status vg_create_source(vg_context* ctx, const double* xyz, const double* cov, const double* normals,
                           int64_t n, vg_source** out);
/* Replace the source positions from a device buffer in caller order (n x 3,
 * dtype 0 = float32, 1 = float64), stream-ordered; covariances and normals are
 * kept, the anchors too (offsets are taken from the old anchors), and the chunk
 * bounds are recomputed.  Used to differentiate with respect to the points. */
vg_status vg_source_set_points_async(vg_source* src, const void* d_xyz, int32_t dtype);
vg_status vg_source_destroy(vg_source* src);

/* ---- preprocessing (Sec. IV-A; Sec. III-C, Preprocessing) ---------------- */

/* A preprocessed frame resident on the device: downsampled points with their
 * k nearest neighbours, regularised covariances and oriented normals. */
typedef struct vg_cloud vg_cloud;

/* Sec. IV-A: a raw frame is downsampled, then each kept point gets its k
 * nearest neighbours (exact search) and, from them, a covariance (Sec. III-C,
 * Preprocessing).  The steps as computed here:
 *   1. voxel-grid downsampling: every input point falls in voxel floor(x / r);
 *      each occupied voxel gives one point, the mean of its input points
 *      (FP64 sums in input order); outputs in ascending lexicographic order of
 *      the voxel key (|floor(x / r)| < 2^20 per axis, else VG_ERR_KEY_RANGE);
 *   2. exact k-NN among the downsampled points, the point itself included;
 *      squared distances in FP64 as (dx*dx + dy*dy) + dz*dz with each operation
 *      rounded, ties by the smaller index; fewer than k points: all of them,
 *      the rest of the row padded with -1;
 *   3. covariance (1/k') sum (p - pbar)(p - pbar)^T over the k' found
 *      neighbours; its eigenvalues are replaced by (1e-3, 1, 1) in ascending
 *      order (plane-to-plane regularisation), i.e. C = I - 0.999 n n^T;
 *   4. normal n: eigenvector of the smallest eigenvalue (FP64 Jacobi), oriented
 *      so that n . (sensor - p) >= 0.
 * xyz: n x 3 host FP64 (n >= 0, finite); r > 0; 1 <= k <= 32; sensor: 3 host
 * doubles (the frame's sensor position).  Synchronous (the output size is read
 * back).  Errors: VG_ERR_INVALID_ARG, VG_ERR_KEY_RANGE, VG_ERR_OOM, VG_ERR_HIP. */
vg_status vg_preprocess(vg_context* ctx, const double* xyz, int64_t n, double r, int32_t k, const double* sensor,
                        vg_cloud** out);
/* Number of downsampled points and the neighbour count k of a cloud. */
vg_status vg_cloud_info(const vg_cloud* cloud, int64_t* n_points, int32_t* k);
/* Copy a cloud to the host; any output may be NULL.  xyz m x 3, cov m x 6
 * (regularised), cov_raw m x 6 (before regularisation), normals m x 3,
 * counts m (input points per voxel), nbr m x k (indices into the cloud),
 * nbr_d2 m x k (squared distances, +inf where padded). */
vg_status vg_cloud_export(const vg_cloud* cloud, double* xyz, double* cov, double* cov_raw, double* normals,
                          int64_t* counts, int32_t* nbr, double* nbr_d2);
/* A source cloud / voxel map made from a preprocessed cloud without leaving the
 * device (same semantics as vg_create_source with normals / vg_build_voxelmap
 * on the cloud's FP64 points and regularised covariances). */
vg_status vg_create_source_from_cloud(vg_context* ctx, const vg_cloud* cloud, vg_source** out);
vg_status vg_build_voxelmap_from_cloud(vg_context* ctx, const vg_cloud* cloud, const double* resolutions,
                                       int32_t L, vg_voxelmap** out);
vg_status vg_cloud_destroy(vg_cloud* cloud);

/* ---- factor batches (Sec. III-C, Implementation) ----------------------- */

/* A batch of F factors; factor f matches src[f] into tgt[f].
 * target_viewpoints: F x 3 (host) sensor positions in each target frame, used
 * only with surface_validation (NULL = origin).  Every voxel map in a batch must
 * have the same number of levels L.  opts may be NULL (defaults). */
vg_status vg_create_factor_batch(vg_context* ctx, int64_t F, vg_source* const* src,
                                 vg_voxelmap* const* tgt, const double* target_viewpoints,
                                 const vg_batch_options* opts, vg_batch** out);
/* Shape of a batch: total source points, number of work tiles, and the launch
 * shape in use (block threads, tile points, persistent workgroups, tile order).
 * Any output may be NULL. */
vg_status vg_batch_info(const vg_batch* batch, int64_t* total_points, int64_t* n_tiles,
                        int32_t* block_threads, int32_t* tile_points, int32_t* grid_blocks,
                        int32_t* tile_order);
vg_status vg_batch_destroy(vg_batch* batch);

/* Linearize every factor at its pose (host arrays): poses F x 12 in; e F,
 * H F x 36, b F x 6 out; inliers F x L (number of points with a voxel at each
 * level) or NULL.  One upload and one download per call; synchronous. */
vg_status vg_linearize(vg_batch* batch, const double* poses, double* e, double* H, double* b,
                       int64_t* inliers);
/* Error only, e = sum d^T W d over points and levels (Eq. (em), Eq. (d2d)), with
 * correspondences and W recomputed at the given poses (host arrays: poses
 * F x 12 in, e F out; synchronous).  In the compensated FP32 mode e equals the
 * e vg_linearize returns at the same poses bit for bit (same hits, same
 * operations, same order of summation), so comparing the two, as an LM step
 * does, reflects the pose change only. */
vg_status vg_evaluate(vg_batch* batch, const double* poses, double* e);

/* Overlap rate of every factor at its pose (GLIM Sec. IV-B and V: the
 * fraction of source points that fall in an occupied voxel of the target,
 * used to pick keyframes and submap pairs): overlap F x L, one fraction per
 * level (points discarded by surface validation count as outside).  Runs the
 * key/lookup path only. */
vg_status vg_overlap(vg_batch* batch, const double* poses, double* overlap);

/* Stream-ordered variants on device pointers (no host synchronization).
 * d_poses: F x 12 FP64.  d_out: F x 43 FP64 rows [e, H (36), b (6)];
 * d_inliers: F x L int64 or NULL.  d_e: F FP64. */
vg_status vg_linearize_async(vg_batch* batch, const double* d_poses, double* d_out, int64_t* d_inliers);
vg_status vg_evaluate_async(vg_batch* batch, const double* d_poses, double* d_e);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as vg_linearize_async, bit for bit, with no
 * allocation, free or allocating library call.  The kernels' scratch (tile
 * counters, staged FP32 poses, one partial row of 40 doubles per tile) lives in
 * a fixed 32 MiB device array, one per device, held until the process ends; a
 * batch needing more (roughly 256 B + 64 B per factor + 320 B per tile, i.e.
 * about 100,000 tiles) fails with VG_ERR_CAPACITY.  Every call on a device
 * shares that device's array, so calls that overlap in time on one device (two
 * streams, two threads) race and must be serialized by the caller.  The work
 * counts of vg_batch_work are not updated by this call. */
vg_status vg_linearize_noalloc(vg_batch* batch, const double* d_poses, double* d_out, int64_t* d_inliers);

/* Exact gradient of e (Eq. (em), Eq. (d2d); W recomputed, not frozen;
 * correspondences held at the given poses), scaled by d_grad_e (F).  d_jr: F x 36 FP64 right Jacobians
 * J_r(xi) to apply (grad_xi = J_r^T de/dxi') or NULL for the plain tangent
 * gradient at T.  d_grad_xi: F x 6 FP64.  d_grad_points: per-point gradient of
 * every source of the batch in caller order, sources concatenated in order of
 * first use (n_total x 3; dtype 0 = float32, 1 = float64), or NULL.  A source
 * used by several factors receives the sum of their gradients, formed in FP64
 * in factor order (deterministic); the first such call on a batch allocates a
 * per-factor gradient buffer (3 values per point of every factor whose source
 * is shared) that the batch keeps. */
vg_status vg_backward_async(vg_batch* batch, const double* d_poses, const double* d_grad_e,
                            const double* d_jr, double* d_grad_xi, void* d_grad_points,
                            int32_t points_dtype);

/* T = T0 Exp(xi) for F poses (device FP64: d_T0 F x 12, d_xi F x 6, d_T F x 12),
 * and the SE(3) right Jacobian J_r(xi) (F x 36) when d_jr is not NULL. */
vg_status vg_se3_retract_async(vg_context* ctx, int64_t F, const double* d_T0, const double* d_xi,
                               double* d_T, double* d_jr);

/* Levenberg-Marquardt, device resident, FP64 6x6 solves (Sec. V-A cites
 * Levenberg's method): each iteration linearizes at T, solves
 * (H + lambda diag(H)) delta = -b by Cholesky, evaluates T Exp(delta), accepts
 * it if e decreases (lambda /= 10) and otherwise keeps T (lambda *= 10).
 * poses_in/poses_out F x 12, accepted F x iters (may be NULL), e_hist F x iters
 * (e at each linearization, may be NULL).  One upload and one download. */
vg_status vg_lm_run(vg_batch* batch, const double* poses_in, int32_t iters, double lambda0,
                    double* poses_out, int32_t* accepted, double* e_hist);

/* Correspondences of one factor at a pose (Sec. III-C, Correspondence search:
 * the voxel holding the transformed point at each level), for parity checks: keys
 * n x L x 3 absolute voxel coordinates of the transformed points, found n x L
 * (1 = voxel exists, 0 = none, -1 = point discarded by surface validation),
 * both in caller order.  Uses the batch's precision mode. */
vg_status vg_correspondences(vg_batch* batch, const double* pose, int64_t factor, int64_t* keys,
                             int32_t* found);

/* One Levenberg-Marquardt iteration for every factor (Sec. V-A), stream-ordered
 * on device pointers with no host synchronization: linearize at d_poses (F x 12,
 * in/out), solve (H + lambda diag(H)) delta = -b by FP64 Cholesky, evaluate
 * T Exp(delta), and accept it iff e decreases (T <- T Exp(delta), lambda /= 10);
 * otherwise T is kept and lambda *= 10 (a damped matrix that is not positive
 * definite counts as a rejection).  d_lambda: F FP64, in/out.  d_e: F FP64, the
 * error at the input poses, or NULL.  d_accepted: F int32 (1 = accepted), or
 * NULL.  Uses the batch's result buffers, so calls on one batch must not overlap. */
vg_status vg_lm_step_async(vg_batch* batch, double* d_poses, double* d_lambda, double* d_e, int32_t* d_accepted);

/* Work done by the most recent linearize / evaluate / overlap call on the batch
 * (synchronizes the context stream): per factor the source points and 64-point
 * chunks walked (chunks whose bounds cannot reach any level's voxels are culled
 * before their points are read), and the table lookups per level (F x L: point
 * levels inside the level's key box; the rest are rejected without a memory
 * access).  Any output may be NULL. */
vg_status vg_batch_work(vg_batch* batch, int64_t* walked_points, int64_t* walked_chunks, int64_t* lookups);

/* Autotune the launch shape of a batch at representative poses (host F x 12):
 * every candidate (block threads x tile points x workgroups per CU) is timed
 * with HIP events over `reps` launches of the tile kernel and reduction; the
 * fastest is kept for this batch (candidates are visited in a fixed order of
 * preference and a later one wins only when faster by more than 1.5 %, so the
 * choice is stable under timing noise) and, when the batch was created with a
 * tune_cache path, appended to that file under a key made of the device
 * (architecture, compute units) and the batch signature (precision, F, total
 * points, levels, validation).
 * chosen (may be NULL) receives {block_threads, tile_points, blocks_per_cu,
 * tile_order}.  Both tile orders are candidates.  When the batch's tune_cache
 * already holds a shape for this device and batch signature, that shape is
 * applied without timing anything.  A batch created with
 * plain_per_factor is tuned for its own loop instead: tile points x block
 * threads candidates, each timed over whole calls of that loop (so a single
 * factor's launch can fill the device with small tiles). */
vg_status vg_batch_tune(vg_batch* batch, const double* poses, int32_t reps, int32_t* chosen);

/* ---- pose graphs: two-node expansion and normal-equation assembly ------- */

/* A graph of N pose nodes and F factors; factor f connects source node
 * node_i[f] (whose cloud is transformed) and target node node_j[f], and its
 * relative pose is T_f = T_j^-1 T_i (the pose the factor is linearized at).
 * Sec. III-C: each factor's quadratic expands to H_ii = H, H_ij = -H A,
 * H_jj = A^T H A, b_i = b, b_j = -A^T b with A = Ad(T_f^-1) (right
 * perturbations of T_i and T_j, xi = [omega; v]).  The structure is a BSR
 * matrix of 6x6 blocks: every diagonal block plus (i, j) and (j, i) for every
 * factor, columns ascending within a row.  Node indices must be distinct and
 * in [0, N). */
typedef struct vg_graph vg_graph;
vg_status vg_create_graph(vg_context* ctx, int64_t N, int64_t F, const int64_t* node_i, const int64_t* node_j,
                          vg_graph** out);
/* nnz_blocks (may be NULL); row_ptr N + 1 and col_idx nnz_blocks (host, may be NULL). */
vg_status vg_graph_structure(const vg_graph* graph, int64_t* nnz_blocks, int64_t* row_ptr, int64_t* col_idx);
/* Assemble on the context stream: d_poses F x 12 relative poses, d_lin F x 43
 * rows [e, H, b] from vg_linearize_async; d_values nnz_blocks x 36 (row-major
 * blocks), d_rhs N x 6.  Contributions are summed in factor order in FP64, so
 * results are deterministic. */
vg_status vg_graph_assemble_async(vg_graph* graph, const double* d_poses, const double* d_lin, double* d_values,
                                  double* d_rhs);
vg_status vg_graph_destroy(vg_graph* graph);

/* Time the batched kernels on the context stream with HIP events: reps
 * launches of the tile kernel and of the factor reduction at device-resident
 * poses (host poses are uploaded once first).  ms[0] = average tile-kernel
 * time, ms[1] = average reduction time, ms[2] = average whole-call time of
 * vg_linearize (upload, kernels, download, synchronization). */
vg_status vg_batch_time_kernels(vg_batch* batch, const double* poses, int32_t reps, float* ms);

#ifdef __cplusplus
}
#endif

#endif /* VGICP_H */

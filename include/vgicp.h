/*
 * vgicp.h - C ABI of the VGICP matching-cost factor library for MI355X (gfx950).
 *
 * Implements the GPU part of Koide et al., "Globally Consistent 3D LiDAR
 * Mapping with GPU-accelerated GICP Matching Cost Factors" (IEEE RA-L 2021):
 *   - voxel maps of point clouds with per-point covariances   (Sec. III-A, VGICP
 *     voxel data association)
 *   - linearization of matching-cost factors into Hessian factors
 *     H_ii, H_ij, H_jj, b_i, b_j and the cost e^M                (Sec. III-A, Eqs. (2)-(6))
 *   - the matching cost alone, for trial steps                   (Sec. III-A, Eq. (3))
 *   - the voxel overlap metric                                   (Sec. III-B, Eqs. (7)-(8))
 *
 * Conventions shared by every entry point
 *   - Pointers named in comments as "device" are HIP device pointers (for example
 *     the data_ptr() of a torch tensor on the GPU); "host" pointers are read
 *     before the call returns.
 *   - Work is enqueued on the context's HIP stream.  Device outputs are valid
 *     once that stream has been synchronized.  vgicp_voxelize is the one call
 *     that synchronizes itself (it sizes the map).
 *   - Every function returns VGICP_OK (0) or a negative status.  The message of
 *     the last failure is available from vgicp_last_error(ctx) (or with a NULL
 *     ctx for failures that had no valid context).  On failure no output is
 *     specified and no handle is created.
 *   - Arguments are validated on the host before anything is enqueued.
 *   - Clouds are frame-local.  A cloud of n points is two arrays:
 *       xyz: float32 [3][n]  (x[0..n), then y[0..n), then z[0..n)); the
 *                              rounds stream the library's own copies, which
 *                              keep the coordinates point by point
 *       cov: float32 [n][6]  (per point xx, xy, xz, yy, yz, zz of the
 *                              symmetric 3x3 covariance; 8-byte aligned): only
 *                              points that fall in a voxel read theirs
 *     The caller owns them.  vgicp_voxelize and vgicp_factorset_create read
 *     them during the call only (a factor set keeps its own copy of every
 *     source cloud), so they may be freed once those calls return.
 *   - A pose is 12 float64 values: R (3x3, row-major) then t; it maps sensor
 *     coordinates to world coordinates, x_world = R x + t.
 *   - Factor (i, j) matches the source cloud (in frame i) against the voxel map
 *     of the target cloud (in frame j): every source point is carried into
 *     frame j by T_j^-1 T_i and looked up in the single voxel that contains it.
 *   - Hessian factors use right perturbations T <- T Exp(xi), xi = (omega, rho),
 *     rotation first; the 12-vector order is [xi_i; xi_j], and
 *       H = [[H_ii, H_ij], [H_ij^T, H_jj]],  b = [b_i; b_j],
 *       e = sum_k e_k^T Omega_k e_k,  e_k = mu'_k - T_j^-1 T_i mu_k,
 *       Omega_k = (C'_k + R C_k R^T)^-1,
 *     with the correspondences and Omega_k frozen at the linearization point.
 *   - One context per host thread; calls that share a context are serialized by
 *     the caller.  No C++ exception crosses this interface.
 */
#ifndef VGICP_H
#define VGICP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VGICP_OK 0
#define VGICP_EINVAL (-1)     /* invalid argument                                  */
#define VGICP_ENOMEM (-2)     /* device or host allocation failed                  */
#define VGICP_ERANGE (-3)     /* a voxel key of a cloud lies outside [-2^20, 2^20) */
#define VGICP_ENONFINITE (-4) /* a point coordinate is NaN or infinite             */
#define VGICP_EHIP (-5)       /* a HIP runtime call failed                         */
#define VGICP_EFULL (-6)      /* a server's memory budget would be exceeded        */

/* Accumulation of the per-point Hessian, gradient and cost terms. */
#define VGICP_ACC_MIXED 0    /* (default) FP32 per lane; the sum over a wave's lanes,
                                the waves and the tiles in FP64                        */
#define VGICP_ACC_F32 1      /* FP32 per lane and across the workgroup (plain)      */
#define VGICP_ACC_F32_COMP 3 /* FP32 per lane, two-sum compensated across the lanes of
                                a wave, FP64 across waves and tiles                   */
#define VGICP_ACC_F64 2      /* FP64 from the first per-point term                  */

/* Residual e_k = mu'_k - T mu_k of the per-point terms.  The correspondence
 * decision always uses the FP32 lookup coordinates (fused multiply-adds with the
 * rotation and translation scaled by fl32(1/r)); these modes only change how the
 * residual itself is evaluated. */
#define VGICP_RESID_F64 0 /* T mu_k and the difference in FP64 from the FP32 point and voxel
                             mean and the FP64 relative pose, then rounded to FP32: accurate
                             to the rounding of the residual itself                       */
#define VGICP_RESID_F32 1 /* plain FP32 transform: absolute error ~ |mu| * 2^-23        */

/* Precision of the fused covariance F' = R^T C'_k R + C_k of a correspondence
 * (Eq. (2), in the source frame) and of its inverse, the point's weight.  With
 * covariances regularized to eigenvalues (1, 1, 1e-3), F' of a point on a
 * surface has a condition number near 1e3, so forming it in FP32 moves the
 * weight along the surface normal by about 1e3 FP32 ulp (relative errors up to
 * about 1e-4 in single entries of a small factor's H). */
#define VGICP_FUSED_F64 0 /* F', its adjugate and determinant in FP64 from the FP32
                             inputs and the FP64 relative rotation, the weight rounded
                             to FP32 (default)                                        */
#define VGICP_FUSED_F32 1 /* all in FP32 (optionally gated to FP64 by fp64_kappa)    */

/* How a linearization forms and sums the per-correspondence terms.  Both give
 * the same H, b, e (up to FP32 rounding) in the same layout. */
#define VGICP_FORM_AUTO 0   /* (default) the factor set's form: the source-frame form
                               unless vgicp_factorset_tune chose the pair form          */
#define VGICP_FORM_SOURCE 1 /* 21 + 6 + 1 sums per correspondence in the source frame
                               (Omega' = (R^T C' R + C)^-1, J' = [[mu]x, -I]), expanded
                               exactly to the 12 x 12 H_ii, H_ij, H_jj once per factor  */
#define VGICP_FORM_PAIR 2   /* Eqs. (5)-(6) term by term: each correspondence adds its
                               J^T Omega J (78 upper-triangle entries of the 12 x 12),
                               J^T Omega e (12) and e^T Omega e in the target frame, J =
                               [A, B] with A = [R [mu]x, -R], B = [-[q]x, I]; accum
                               VGICP_ACC_MIXED, _F32 or _F32_COMP, no corr output; about
                               200 VGPRs per lane (2 waves per SIMD)                    */

/* How the factors of one call are launched. */
#define VGICP_SCHED_BATCHED 0    /* one launch over the tiles of all factors, one reduce   */
#define VGICP_SCHED_PER_FACTOR 1 /* one linearize launch and one reduce launch per factor */

/* Layout of a factor set's tile table (point ranges of one factor, of the
 * factor set's tile size).  The grouped and interleaved layouts give the same
 * bits; the balanced one cuts some factors into shorter tiles, which changes
 * only their FP32 summation order (integer outputs are the same). */
#define VGICP_LAYOUT_GROUPED 0     /* factors grouped by target map, each factor's tiles
                                      consecutive (default)                            */
#define VGICP_LAYOUT_INTERLEAVED 1 /* the factors that read one source copy side by
                                      side, tile by tile, so that tiles streaming the
                                      same source points run together and share L2   */
#define VGICP_LAYOUT_BALANCED 2    /* the grouped order in 8 runs of about equal points,
                                      one per XCD, whose factors ending in the run's
                                      last tenth of points get quarter-size tiles, so
                                      that each XCD's last blocks are short; the runs
                                      are padded to one length with empty tiles      */

typedef struct vgicp_context_s *vgicp_ctx;
typedef struct vgicp_voxelmap_s *vgicp_map;
typedef struct vgicp_factorset_s *vgicp_factorset;

typedef struct {
  const float *xyz; /* device, [3][n] */
  const float *cov; /* device, [n][6], 8-byte aligned */
  int64_t n;        /* number of points, 0 <= n <= 2^26 */
} vgicp_cloud;

/* One matching-cost factor (Eq. (1)): indices into the source-cloud list, the
 * voxel-map list and the pose array. */
typedef struct {
  int32_t src;
  int32_t tgt;
  int32_t pose_i;
  int32_t pose_j;
} vgicp_factor;

typedef struct {
  int32_t accum;     /* VGICP_ACC_*                                                  */
  int32_t schedule;  /* VGICP_SCHED_*                                                */
  int32_t use_graph; /* nonzero: the batched schedule is captured once into a HIP
                        graph per (poses, outputs) pointer set and replayed          */
  int32_t resid;     /* VGICP_RESID_*                                                */
  float fp64_kappa;  /* with VGICP_FUSED_F32 only: > 0 makes points whose FP32 fused
                        covariance F' = R^T C' R + C has a condition estimate
                        trace^3 / (27 det) above this value (or is not positive
                        definite in FP32) form and invert F' in FP64; 0 = FP32 always.
                        Ignored with VGICP_FUSED_F64                                 */
  int32_t fused;     /* VGICP_FUSED_*: precision of the fused covariance and its
                        inverse (0 = VGICP_FUSED_F64, the default)                   */
  int32_t form;      /* VGICP_FORM_*: 0 = VGICP_FORM_AUTO, the factor set's form     */
} vgicp_opts;

/* Library version as major*10000 + minor*100 + patch. */
int vgicp_version(void);

/* Message of the last failure on ctx (ctx may be NULL: message of the last
 * failure on this thread that had no valid context).  Never NULL. */
const char *vgicp_last_error(vgicp_ctx ctx);

/* Create a context on HIP device `device` that enqueues on `hip_stream` (a
 * hipStream_t; NULL means the default stream).  The stream is borrowed.
 * Errors: EINVAL (out NULL, device out of range), EHIP. */
int vgicp_ctx_create(int device, void *hip_stream, vgicp_ctx *out);

/* Change the stream later calls enqueue on.  Errors: EINVAL. */
int vgicp_ctx_set_stream(vgicp_ctx ctx, void *hip_stream);

/* Wait for the context's stream.  Errors: EINVAL, EHIP. */
int vgicp_ctx_synchronize(vgicp_ctx ctx);

/* Kernel timing.  While enabled, later calls bracket each kernel they launch
 * outside a HIP graph with a pair of HIP events on the context's stream; the
 * durations are added per kernel kind.  vgicp_ctx_read_timing synchronizes the
 * stream, folds the pending event pairs in and returns the total milliseconds
 * and launch count of `kernel` since the last reset.  Errors: EINVAL, EHIP. */
#define VGICP_KERNEL_LINEARIZE 0 /* per-tile linearization kernel            */
#define VGICP_KERNEL_REDUCE 1    /* per-factor reduce / expand kernel          */
#define VGICP_KERNEL_OVERLAP 2   /* per-tile overlap kernel                    */
#define VGICP_KERNEL_EVALUATE 3  /* per-tile cost-only kernel                  */
#define VGICP_KERNEL_KINDS 4
int vgicp_ctx_set_timing(vgicp_ctx ctx, int enable);
int vgicp_ctx_read_timing(vgicp_ctx ctx, int kernel, double *total_ms, int64_t *launches);
int vgicp_ctx_reset_timing(vgicp_ctx ctx);

/* Destroy a context and its workspace.  Maps and factor sets created from it
 * must be freed first.  NULL is accepted. */
int vgicp_ctx_destroy(vgicp_ctx ctx);

/* --------------------------------------------------------------------------
 * Voxel maps (Sec. III-A): the cloud is discretized at resolution r; voxel v
 * holds the points whose key floor(fl32(x * fl32(1/r))) (per axis, FP32) equals
 * its key.  Its mean is fl32 of the FP64 mean of those points, its covariance
 * fl32 of the FP64 mean of their covariances (VGICP aggregates point
 * distributions, it does not take the sample covariance of positions).  Voxel
 * ordinals number the voxels in lexicographic (kx, ky, kz) key order.
 * ------------------------------------------------------------------------ */

/* Build the voxel map of `cloud` (host struct, device arrays) at `resolution`
 * metres.  Synchronizes the stream once.  The map is library-owned device
 * memory; free it with vgicp_map_free.  The cloud is not referenced after the
 * call returns.
 * Errors: EINVAL (NULL pointers with n > 0, n outside [0, 2^26], resolution
 * not finite or <= 0, more than 2^24 occupied 4 x 4 x 4 bricks), ENONFINITE,
 * ERANGE, ENOMEM, EHIP. */
int vgicp_voxelize(vgicp_ctx ctx, const vgicp_cloud *cloud, double resolution, vgicp_map *out);

/* Map facts: number of voxels, capacity of its brick table (records; voxels
 * are indexed through bricks of 4 x 4 x 4), device bytes held and the
 * resolution.  Any output pointer may be NULL.  Errors: EINVAL. */
int vgicp_map_info(vgicp_map map, int64_t *n_voxels, int64_t *capacity, int64_t *device_bytes,
                   double *resolution);

/* Copy the map out in ordinal order into device arrays: keys int32 [V][3],
 * mean float32 [V][3], cov float32 [V][6], count int32 [V].  Any may be NULL.
 * Enqueued on the stream.  Errors: EINVAL, EHIP. */
int vgicp_map_export(vgicp_ctx ctx, vgicp_map map, int32_t *keys, float *mean, float *cov,
                     int32_t *count);

/* Free a map (NULL accepted).  The caller makes sure no enqueued work still
 * reads it (synchronize first). */
int vgicp_map_free(vgicp_map map);

/* --------------------------------------------------------------------------
 * Factor sets: the factor list F^M of Eq. (1) bound to its clouds and maps.
 * Creating one validates every index and uploads the device tables once, so
 * that each optimizer iteration only passes new poses.
 * ------------------------------------------------------------------------ */

/* sources: host array of n_sources cloud descriptors (device data, caller
 * owned, read during this call only): the factor set keeps its own copy of
 * every source cloud a factor uses, its points in Morton order of cells of the
 * finest resolution among the maps that cloud is matched against, so that
 * neighbouring points of a wave look up neighbouring voxels, coordinates
 * stored point by point (40 bytes of device memory per point; results differ
 * from the caller's order only by FP32 summation order, and per-point outputs
 * keep the caller's order);
 * maps: host array of n_maps handles (they must outlive the factor set);
 * factors: host array of n_factors rows; n_poses: length of the pose arrays
 * later calls pass; tile_points: source points per workgroup tile, a multiple
 * of 256 in [256, 1<<20], or 0 for automatic: the first of 4608, 3072, 2304,
 * 1536 and 768 (whole lookup phases of a workgroup) that gives the factor set
 * at least 3072 tiles, else 768.
 * Outputs of later calls are indexed in the order of `factors`.  Per-point
 * outputs (corr) are laid out factor after factor, n_src points each.
 * Errors: EINVAL (any index out of range, NULL pointers with nonzero counts,
 * bad tile_points, a source of more than 2^26 points), ENOMEM, EHIP. */
int vgicp_factorset_create(vgicp_ctx ctx, const vgicp_cloud *sources, int32_t n_sources,
                           const vgicp_map *maps, int32_t n_maps, const vgicp_factor *factors,
                           int64_t n_factors, int32_t n_poses, int32_t tile_points,
                           vgicp_factorset *out);

/* Factor-set facts (tile_points: the tile size in use; n_tiles: entries of
 * the tile table, the balanced layout's padding included); any output may be
 * NULL.  Errors: EINVAL. */
int vgicp_factorset_info(vgicp_factorset fs, int64_t *n_factors, int64_t *n_tiles,
                         int64_t *total_points, int32_t *tile_points);

/* Schedule autotuning (the batched schedule of Sec. III-D's one-launch
 * linearization round): after 10 warm-up rounds, time a linearization round of
 * this factor set at these poses for each candidate tile size (host int32 array
 * of multiples of 256 in [256, 2^20]; NULL = 32256, 23040, 18432, 13824, 9216,
 * 4608, 3072, 2304, 1536, 768, whole lookup phases of a workgroup) on each of
 * two grids (one workgroup per tile, and a persistent grid of as many
 * workgroups as the device's CUs hold at once for opts' kernel, each walking
 * several tiles), twice in forward and reverse order keeping each pair's best,
 * and keep the fastest pair. Every candidate is timed in the grouped and
 * balanced tile-table layouts (VGICP_LAYOUT_*), and in the interleaved one when
 * some source copy is read by more than one factor; the fastest is kept. With
 * opts' form VGICP_FORM_AUTO (the default) and an accumulation the pair form
 * supports, every candidate is also timed in the pair form and the factor set
 * keeps the faster form for VGICP_FORM_AUTO calls; with another form only that
 * form is timed (and the kept form is not changed). H, b, e, inliers are device
 * buffers as for vgicp_linearize_factors, overwritten by the trial rounds. The
 * factor set's tiles and grid change (results change only by FP32 summation
 * order; the grid alone does not change them) and its captured graphs are
 * dropped. best_tile and best_ms (mean device time of a round) may be NULL; the
 * grid chosen is read with vgicp_factorset_grid, the layout with
 * vgicp_factorset_layout and the form with vgicp_factorset_form. Synchronizes
 * ctx's stream. Errors: EINVAL, EHIP. */
int vgicp_factorset_tune(vgicp_ctx ctx, vgicp_factorset fs, const double *poses,
                         const vgicp_opts *opts, double *H, double *b, double *e,
                         int64_t *inliers, const int32_t *candidates, int32_t n_candidates,
                         int32_t *best_tile, double *best_ms);

/* Measurement of one kernel of a round: `reps` (1..10000) back-to-back
 * launches of the linearization (VGICP_KERNEL_LINEARIZE), cost-only
 * (VGICP_KERNEL_EVALUATE) or overlap (VGICP_KERNEL_OVERLAP) kernel over every
 * tile of the factor set at `poses`, with opts' variant (NULL: defaults),
 * bracketed by one pair of HIP events on ctx's stream and no event between
 * launches; *avg_ms receives the mean duration of a launch.  The call writes
 * only the factor set's tile partials and, once before the timed launches,
 * its table of per-factor pose constants (the next call overwrites both).
 * Synchronizes ctx's stream.  Errors: EINVAL (unknown or reduce kernel, reps
 * out of range), EHIP. */
int vgicp_factorset_time_kernel(vgicp_ctx ctx, vgicp_factorset fs, const double *poses,
                                const vgicp_opts *opts, int32_t kernel, int32_t reps,
                                double *avg_ms);

/* Grid of the factor set's linearize, evaluate and overlap launches:
 * persist_blocks = 0 runs one workgroup per tile; a positive multiple of 8
 * runs at most that many workgroups, the tiles dealt to the 8 XCDs in eighths
 * of the tile table and walked in order by each XCD's workgroups.  Results
 * are the same bits on either grid.  Drops captured graphs (synchronizes
 * ctx's stream when the grid changes).  Errors: EINVAL (not 0 or a multiple
 * of 8 in [8, 2^24]). */
int vgicp_factorset_set_grid(vgicp_ctx ctx, vgicp_factorset fs, int32_t persist_blocks);

/* The grid in use (see vgicp_factorset_set_grid).  Errors: EINVAL. */
int vgicp_factorset_grid(vgicp_factorset fs, int32_t *persist_blocks);

/* The form VGICP_FORM_AUTO calls use (VGICP_FORM_SOURCE unless
 * vgicp_factorset_tune chose VGICP_FORM_PAIR).  Errors: EINVAL. */
int vgicp_factorset_form(vgicp_factorset fs, int32_t *form);

/* Tile-table layout (VGICP_LAYOUT_*): rebuilds the tile table at the current
 * tile size and drops captured graphs (synchronizes ctx's stream).  After
 * vgicp_factorset_reorder every factor reads its own copy, so the interleaved
 * layout then only puts the factors of one source next to each other.
 * Errors: EINVAL, EHIP. */
int vgicp_factorset_set_layout(vgicp_ctx ctx, vgicp_factorset fs, int32_t layout);

/* The layout in use.  Errors: EINVAL. */
int vgicp_factorset_layout(vgicp_factorset fs, int32_t *layout);

/* Target-order source copies.  A round streams every source point once and
 * gathers the statistics of the target voxel it falls in (Sec. III-A, Eq. (3)
 * correspondences); the gathers share cache lines when consecutive points of a
 * wave fall in neighbouring voxels.  This call gives every factor its own copy
 * of its source cloud (40 bytes of device memory per point, replacing the
 * per-cloud Morton-ordered copies) with the points in the order of the target
 * voxels they fall in at `poses` (device float64 [n_poses][12]): voxel after
 * voxel in the order of the map's statistics records (bricks of 4 x 4 x 4,
 * Morton order within a brick), points of one voxel in their previous order,
 * and points that fall in no voxel last.  The order stays good while the
 * poses move by small steps (an optimizer's iterations); call it again after
 * large moves.  Results at any poses are unchanged up to FP32 summation order
 * (integer and per-point outputs are identical).  Captured graphs are
 * dropped.  Synchronizes ctx's stream.
 * Errors: EINVAL (NULL or foreign arguments, more than 2^31 - 1 source points
 * in the set), ENOMEM, EHIP (on failure the set is unchanged). */
int vgicp_factorset_reorder(vgicp_ctx ctx, vgicp_factorset fs, const double *poses);

/* Precision diagnostics (the ill-conditioned case of Sec. III-A's fused
 * covariance C'_k + R C_k R^T): the number of correspondences of the last
 * vgicp_linearize_factors or vgicp_evaluate_errors call on fs that formed and
 * inverted the fused covariance in FP64: every inlier with VGICP_FUSED_F64, the
 * inliers the opts.fp64_kappa gate sent to FP64 with VGICP_FUSED_F32 (0 with
 * fp64_kappa = 0, and before any call).  Overlap calls do not change
 * it.  Synchronizes ctx's stream.  n_points: host int64.
 * Errors: EINVAL (NULL or foreign arguments), EHIP. */
int vgicp_factorset_fp64_points(vgicp_ctx ctx, vgicp_factorset fs, int64_t *n_points);

/* Input checks.  The rounds do not scan their inputs (a source point whose
 * transform is not finite is a miss, a hit whose fused covariance is not
 * positive definite adds nothing), so that a round reads each input once.
 * The checks come from passes that read the inputs anyway:
 *   nonfinite_points, nonfinite_covs: points of the source clouds the set uses
 *     with a non-finite coordinate, and with a non-finite covariance entry,
 *     counted when the set was created (making its ordered copies reads every
 *     point; the set keeps no pointer to the caller's clouds, so later changes
 *     of those clouds are not seen);
 *   degenerate_hits: correspondences of the last vgicp_linearize_factors or
 *     vgicp_evaluate_errors call whose fused covariance C'_k + R C_k R^T
 *     (Eq. (2)) was not positive definite or not finite, and so added nothing
 *     though counted as inliers (0 before any call; synchronizes ctx's stream).
 * Target clouds are checked by vgicp_voxelize (ENONFINITE for a non-finite
 * point; a non-finite covariance makes its voxel's hits degenerate).  Any
 * output may be NULL.  Errors: EINVAL, EHIP. */
int vgicp_factorset_check(vgicp_ctx ctx, vgicp_factorset fs, int64_t *nonfinite_points,
                          int64_t *nonfinite_covs, int64_t *degenerate_hits);

/* Number of HIP graphs the factor set holds.  Graph replay (opts.use_graph)
 * captures one graph per (poses, outputs, options) set and keeps at most 8:
 * capturing another first waits for the context's stream and drops the least
 * recently replayed one.  Errors: EINVAL. */
int vgicp_factorset_graph_count(vgicp_factorset fs, int64_t *n_graphs);

/* Free a factor set and its captured graphs (NULL accepted). */
int vgicp_factorset_destroy(vgicp_factorset fs);

/* Host-side check of a factor list without any device (used by the factor-set
 * constructor).  Errors: EINVAL with a message naming the first bad row. */
int vgicp_validate_factors(int32_t n_sources, int32_t n_maps, int32_t n_poses,
                           const vgicp_factor *factors, int64_t n_factors);

/* --------------------------------------------------------------------------
 * Linearization (Sec. III-A, Eqs. (2)-(6)) and cost evaluation (Eq. (3)).
 * ------------------------------------------------------------------------ */

/* Linearize every factor of `fs` at `poses` (device float64 [n_poses][12]).
 * Outputs (device): H float64 [n_factors][12][12] (row-major, symmetric),
 * b float64 [n_factors][12], e float64 [n_factors], inliers int64 [n_factors]
 * (points that fell in a voxel of the target map), and optionally corr int32
 * [total_points] with the voxel ordinal of each source point or -1 (NULL to
 * skip).  A factor with no inlier returns H = 0, b = 0, e = 0.
 * opts may be NULL (the defaults: FP32 per-lane sums carried in FP64 beyond the lane,
 * batched schedule, no graph, FP64 residual, FP64 fused covariance; a zero-filled
 * vgicp_opts is the same).  Results
 * are deterministic and do not depend on the schedule or on the other factors
 * of the set.  Device inputs are not scanned here: a source point whose
 * transform is not finite or falls outside the key range is a miss, and a hit
 * whose fused covariance is not positive definite (including non-finite) adds
 * nothing but counts as an inlier; vgicp_factorset_check reports both kinds of
 * bad input.  The pair form (opts->form, or the factor set's tuned form under
 * VGICP_FORM_AUTO) allocates its tile partials (96 doubles per tile) at its
 * first call; VGICP_FORM_AUTO takes the source-frame form where the pair form
 * does not apply (corr requested, VGICP_ACC_F64).  Errors: EINVAL (also for
 * VGICP_FORM_PAIR with corr or with VGICP_ACC_F64), EHIP. */
int vgicp_linearize_factors(vgicp_ctx ctx, vgicp_factorset fs, const double *poses,
                            const vgicp_opts *opts, double *H, double *b, double *e,
                            int64_t *inliers, int32_t *corr);

/* The cost e (device float64 [n_factors]) and inliers (device int64
 * [n_factors]) alone, without Jacobians; equal to the e and inliers of
 * vgicp_linearize_factors with the same accumulation in the source-frame form
 * (the pair form's e, summed in the target frame, agrees to FP32 rounding;
 * inliers are always equal).  A call uses the factor set's tile partials and
 * its table of per-factor pose constants:
 * calls on one factor set that overlap in time (on two streams) race.
 * Errors: EINVAL, EHIP. */
int vgicp_evaluate_errors(vgicp_ctx ctx, vgicp_factorset fs, const double *poses,
                          const vgicp_opts *opts, double *e, int64_t *inliers);

/* For callers that cannot allocate device memory during a round (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * vgicp_linearize_factors with the same arguments, kernels and results (bit
 * for bit), but the per-tile partial sums go to a fixed scratch array that the
 * library holds on each device it runs on (VGICP_NOALLOC_MAX_TILES tiles of
 * 32 doubles, 8 MiB, kept until the process ends) instead of the factor
 * set's buffer, and the call allocates nothing: no device or pinned memory,
 * no events, no graph (opts->use_graph must be 0).  It linearizes in the
 * source-frame form only: VGICP_FORM_PAIR is EINVAL and VGICP_FORM_AUTO means
 * VGICP_FORM_SOURCE here, whatever form the factor set was tuned to.  Every
 * call on a device shares that device's array, so calls that overlap on one device (on two
 * streams, or from two threads) race and give wrong results; calls on one
 * stream are ordered and safe.  Nothing in the array needs clearing between
 * calls: each launch writes every partial its reduce reads.
 * Errors: EINVAL (as vgicp_linearize_factors, or use_graph != 0), ERANGE (the
 * factor set has more than VGICP_NOALLOC_MAX_TILES tiles: use larger tiles),
 * EHIP. */
#define VGICP_NOALLOC_MAX_TILES 32768
int vgicp_linearize_factors_noalloc(vgicp_ctx ctx, vgicp_factorset fs, const double *poses,
                                    const vgicp_opts *opts, double *H, double *b, double *e,
                                    int64_t *inliers, int32_t *corr);

/* --------------------------------------------------------------------------
 * Assembly of the linearized system (Sec. III-D: the optimizer collects the
 * per-factor results into one linear system).  With one 6-vector per pose in
 * (omega, rho) order, every factor (i, j) adds H_ii to block (i, i), H_jj to
 * (j, j), H_ij to (i, j), H_ij^T to (j, i), b_i to pose i and b_j to pose j
 * (a factor with i == j adds all four blocks to (i, i)).  Sums run in factor
 * order in FP64, so the result is deterministic.
 * ------------------------------------------------------------------------ */

/* Number of distinct unordered pose pairs {i, j}, i != j, of the factor set
 * and, if `pairs` is not NULL, the pairs as host int32 [n_pairs][2] with
 * pairs[k][0] < pairs[k][1], in increasing lexicographic order.  Errors: EINVAL. */
int vgicp_factorset_pairs(vgicp_factorset fs, int64_t *n_pairs, int32_t *pairs);

/* Assemble from per-factor H (device float64 [n_factors][12][12]) and b
 * (device float64 [n_factors][12]), as written by vgicp_linearize_factors:
 * Hdiag device float64 [n_poses][6][6], bvec device float64 [n_poses][6], and
 * Hoff device float64 [n_pairs][6][6] (may be NULL) holding block (p, q) of
 * pair k = (p, q) (block (q, p) is its transpose).  Poses no factor touches
 * get zeros.  Errors: EINVAL, EHIP. */
int vgicp_assemble_system(vgicp_ctx ctx, vgicp_factorset fs, const double *H, const double *b,
                          double *Hdiag, double *bvec, double *Hoff);

/* --------------------------------------------------------------------------
 * Overlap (Sec. III-B, Eqs. (7)-(8)): for each factor row (i, j), hits = number
 * of source points falling in a voxel of the target map under T_j^-1 T_i and
 * overlap = hits / N (0 when N = 0).
 * ------------------------------------------------------------------------ */

/* hits: device int64 [n_factors]; overlap: device float64 [n_factors] (may be
 * NULL).  Errors: EINVAL, EHIP. */
int vgicp_overlap(vgicp_ctx ctx, vgicp_factorset fs, const double *poses, int64_t *hits,
                  double *overlap);

/* --------------------------------------------------------------------------
 * Keyframe control by overlap (Sec. III-B local mapping, Sec. III-C global
 * mapping).  The overlap of a cloud against a map is Eq. (8) with the pose
 * T_map^-1 T_cloud, counted exactly on the GPU as in vgicp_overlap; the
 * comparisons with the thresholds are made on the host in FP64.
 * ------------------------------------------------------------------------ */

/* Admission rule of a factor by its overlap. */
#define VGICP_GATE_ABOVE 0    /* admit when overlap > threshold (the paper's th^G_min rule) */
#define VGICP_GATE_AT_LEAST 1 /* admit when overlap >= threshold                          */

/* Overlap-gated factor creation (Sec. III-C: a matching-cost factor joins
 * the new keyframe and every earlier one whose overlap exceeds th^G_min,
 * e.g. 2.5 %).  `cloud` (host struct, device xyz [3][n]; cov is not read) at
 * host pose h_pose [12] is checked against each of the n_maps maps at host
 * poses h_map_poses [n_maps][12]: h_hits [n_maps] (host int64, may be NULL)
 * and h_overlap [n_maps] (host float64, may be NULL) receive the counts and
 * rates, h_admitted [n_maps] (host int32) 1 for every map admitted by
 * `threshold` under `rule` (VGICP_GATE_*), *n_admitted (may be NULL) their
 * number.  Synchronizes ctx's stream (the outputs are on the host).
 * Errors: EINVAL (NULL or foreign arguments, a non-finite pose or threshold,
 * an unknown rule), ENOMEM, EHIP. */
int vgicp_connect(vgicp_ctx ctx, const vgicp_cloud *cloud, const double *h_pose,
                  const vgicp_map *maps, const double *h_map_poses, int32_t n_maps,
                  double threshold, int32_t rule, int64_t *h_hits, double *h_overlap,
                  int32_t *h_admitted, int32_t *n_admitted);

/* Local-mapping rules (Sec. III-B). */
typedef struct {
  double skip_above;  /* th^L_max: a frame whose overlap with the submap's last frame
                         is above this is skipped (the sensor has not moved), e.g. 0.95 */
  double close_below; /* th^L_min: the submap closes when the overlap between its newest
                         and first frames is below this, e.g. 0.10                     */
  int32_t max_frames; /* N^L_max: the submap closes when it would hold more frames     */
  int32_t reserved;   /* must be 0                                                     */
} vgicp_submap_rules;

/* Decisions of vgicp_submap_step for an arriving frame. */
#define VGICP_SUBMAP_START 0  /* the submap was empty: the frame starts it                  */
#define VGICP_SUBMAP_SKIP 1   /* overlap with the last frame > skip_above: not inserted     */
#define VGICP_SUBMAP_INSERT 2 /* inserted (factors to every frame of the submap follow)     */
#define VGICP_SUBMAP_CLOSE 3  /* inserted, and the submap closes: overlap with the first
                                 frame < close_below, or n_submap + 1 > max_frames        */

/* The local-mapping decision for `frame` (host struct, device xyz) at host
 * pose h_pose, arriving at a submap of n_submap frames whose first and last
 * frames have maps `first` and `last` at host poses h_first_pose and
 * h_last_pose (equal when n_submap is 1; all ignored when n_submap is 0).
 * *overlap_last and *overlap_first (may be NULL) receive the overlaps of the
 * frame against the last and first maps (0 when n_submap is 0).  The
 * decision is made in that order: START, SKIP, CLOSE, INSERT.  Synchronizes
 * ctx's stream.  Errors: EINVAL, ENOMEM, EHIP. */
int vgicp_submap_step(vgicp_ctx ctx, const vgicp_submap_rules *rules, const vgicp_cloud *frame,
                      const double *h_pose, vgicp_map first, const double *h_first_pose,
                      vgicp_map last, const double *h_last_pose, int32_t n_submap,
                      int32_t *decision, double *overlap_first, double *overlap_last);

/* --------------------------------------------------------------------------
 * Serving: continuous batching of factor requests over resident keyframes.
 *
 * The paper's optimizer issues every cost task of an iteration to the GPU,
 * synchronizes once and collects the results (Sec. III-D).  A server keeps the
 * keyframes (clouds and voxel maps) resident in device memory under a byte
 * budget and serves requests from several optimizers at once: requests that
 * arrive while batches are on the device are admitted into the next batch as
 * soon as a batch slot frees up, and up to `inflight` batches run on their own
 * streams at the same time.  A factor's result depends only on its own points
 * and tiles, so it is bit-identical whether its request ran alone or in a mix.
 * All functions are thread-safe.
 * ------------------------------------------------------------------------ */

typedef struct vgicp_server_s *vgicp_server;

#define VGICP_REQ_LINEARIZE 0 /* outputs H, b, e, inliers                  */
#define VGICP_REQ_EVALUATE 1  /* outputs e, inliers                        */
#define VGICP_REQ_OVERLAP 2   /* outputs inliers (= hits), overlap         */

typedef struct {
  int64_t memory_budget_bytes; /* device bytes for resident frames; 0 = no limit     */
  int32_t max_batch_factors;   /* factors per batch (slot size), >= 1               */
  int32_t max_batch_points;    /* source points per batch, >= 1                     */
  int32_t max_batch_poses;     /* poses per batch, >= 1                             */
  int32_t inflight;            /* batches on the device at once, 1..8                */
  int32_t tile_points;         /* 0 = 4608 (whole lookup phases of a workgroup)     */
  int32_t reserved;            /* must be 0                                         */
  vgicp_opts opts;             /* accumulation, residual, kappa of every batch
                                  (schedule and use_graph are ignored; form must be
                                  VGICP_FORM_AUTO or VGICP_FORM_SOURCE: batches are
                                  linearized in the source-frame form)              */
} vgicp_server_config;

/* Create a server on HIP device `device` with its own streams and worker
 * thread.  Errors: EINVAL, ENOMEM, EHIP. */
int vgicp_server_create(int device, const vgicp_server_config *cfg, vgicp_server *out);

/* Stop the worker after the submitted requests complete and free everything
 * (NULL accepted). */
int vgicp_server_destroy(vgicp_server srv);

/* Message of the last failure on srv. */
const char *vgicp_server_last_error(vgicp_server srv);

/* Register a keyframe: host arrays h_xyz [3][n] and h_cov [n][6] are copied
 * to server-owned device memory and voxelized at `resolution`; the copy then
 * keeps the points in Morton order of cells of that resolution.  That is the
 * order a factor set gives a source cloud whose maps all have this resolution,
 * so a server factor and a factor-set factor agree bit for bit when every
 * target of that source in the factor set has the source frame's resolution
 * and both use the same tile_points, the factor set in the grouped or
 * interleaved layout without target-order copies; otherwise the points are
 * summed in another order and they agree within FP32 summation error (integer
 * outputs always agree).  Requests have no per-point outputs.  Returns its id.
 * Errors: EINVAL (n outside [0, 2^26], NULL arrays, bad resolution), ENONFINITE,
 * ERANGE, EFULL (the frame would exceed the memory
 * budget; nothing is kept), ENOMEM, EHIP. */
int vgicp_server_add_frame(vgicp_server srv, const float *h_xyz, const float *h_cov, int64_t n,
                           double resolution, int32_t *frame_id);

/* Remove a keyframe once every request that references it has completed.
 * Errors: EINVAL (unknown id). */
int vgicp_server_remove_frame(vgicp_server srv, int32_t frame_id);

/* Device bytes held by resident frames, and the budget (0 = no limit). */
int vgicp_server_memory(vgicp_server srv, int64_t *used_bytes, int64_t *budget_bytes);

/* Submit a request of `kind` over n factors (src and tgt are frame ids, pose_i
 * and pose_j index h_poses [n_poses][12]).  Factors and poses are copied before
 * the call returns.  The host output arrays (H [n][144], b [n][12], e [n],
 * inliers [n], overlap [n]; those the kind does not produce may be NULL) must
 * stay valid until the request completes, and two requests in flight must not
 * share one (the library does not check).  Returns a ticket.
 * Errors: EINVAL (unknown frame, index out of range, NULL outputs, more poses
 * than max_batch_poses). */
int vgicp_server_submit(vgicp_server srv, int kind, const vgicp_factor *factors, int64_t n,
                        const double *h_poses, int32_t n_poses, double *H, double *b, double *e,
                        int64_t *inliers, double *overlap, int64_t *ticket);

/* One request of vgicp_server_submit_many: the arguments of
 * vgicp_server_submit (host arrays, same ownership and sizes). */
typedef struct {
  int32_t kind;                 /* VGICP_REQ_* */
  int32_t n_poses;
  int64_t n;                    /* factors */
  const vgicp_factor *factors;  /* [n] */
  const double *h_poses;        /* [n_poses][12] */
  double *H, *b, *e;            /* outputs as for vgicp_server_submit */
  int64_t *inliers;
  double *overlap;
} vgicp_server_request;

/* Several requests queued at once (Sec. III-D: an optimizer issues all of its
 * cost-evaluation tasks, then synchronizes once): the worker finds them
 * together, so requests of one kind share a batch and its launches (fewer
 * launches and copies; small requests submitted one by one can instead finish
 * sooner on separate in-flight slots, whose copies and launches overlap).
 * Each request as for vgicp_server_submit; tickets [n_reqs] receives their
 * tickets in order.  All or nothing: on an error no request is queued.
 * Errors: as vgicp_server_submit, and EINVAL for n_reqs < 0 or NULL arrays
 * with n_reqs > 0. */
int vgicp_server_submit_many(vgicp_server srv, const vgicp_server_request *reqs, int32_t n_reqs,
                             int64_t *tickets);

/* Nonzero in *done once the request's outputs are written.  Errors: EINVAL. */
int vgicp_server_poll(vgicp_server srv, int64_t ticket, int *done);

/* Block until the request completes; *latency_ms (may be NULL) receives the
 * time from submit to outputs written.  Errors: EINVAL, EHIP (a batch failed). */
int vgicp_server_wait(vgicp_server srv, int64_t ticket, double *latency_ms);

/* vgicp_connect over resident frames: frame id `frame` at h_pose against the
 * frames candidates [n_candidates] at h_candidate_poses [n_candidates][12],
 * as overlap requests batched with the server's other work (split so that
 * each carries at most max_batch_poses poses) and waited for.  Outputs as for
 * vgicp_connect.  Errors: EINVAL (unknown frames, bad arguments,
 * max_batch_poses < 2), EHIP. */
int vgicp_server_connect(vgicp_server srv, int32_t frame, const double *h_pose,
                         const int32_t *candidates, const double *h_candidate_poses,
                         int32_t n_candidates, double threshold, int32_t rule, int64_t *h_hits,
                         double *h_overlap, int32_t *h_admitted, int32_t *n_admitted);

/* vgicp_submap_step over resident frames (`first` and `last` are frame ids;
 * one overlap request of two rows, which needs max_batch_poses >= 3).
 * Errors: EINVAL, EHIP. */
int vgicp_server_submap_step(vgicp_server srv, const vgicp_submap_rules *rules, int32_t frame,
                             const double *h_pose, int32_t first, const double *h_first_pose,
                             int32_t last, const double *h_last_pose, int32_t n_submap,
                             int32_t *decision, double *overlap_first, double *overlap_last);

/* Counters: batches launched and requests completed so far, the largest number
 * of requests merged into one batch, and the largest number of batches that
 * were on the device at once.  Any pointer may be NULL. */
int vgicp_server_stats(vgicp_server srv, int64_t *batches, int64_t *requests,
                       int64_t *max_requests_per_batch, int64_t *max_inflight);

#ifdef __cplusplus
}
#endif

#endif /* VGICP_H */

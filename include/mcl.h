/*
 * mcl.h - C ABI of the MI355X (gfx950) sensor update for 6-DoF Monte Carlo
 * localisation in TSDF maps (Eisoldt et al., "Towards 6D MCL for LiDARs in 3D
 * TSDF Maps on Embedded Systems with GPUs", arXiv 2310.04172).
 *
 * One MCL iteration (§III) is motion update, sensor update, resampling; the
 * sensor update is the costly step the paper moves to the GPU (§IV, §V-B).
 * This library runs the sensor update, the weight normalisation, the pose
 * estimate and the resampling on the GPU, so particle state never leaves device
 * memory.
 *
 * Conventions shared by every call:
 *  - Device pointers are plain HIP device addresses (for example a torch
 *    tensor's data_ptr()); the caller owns them and keeps them alive until the
 *    stream has executed the work.  `stream` is a hipStream_t (NULL = the
 *    default stream); every call only enqueues work on it and returns.
 *  - Argument errors are detected on the host before anything is enqueued; a
 *    failing call enqueues nothing.  Launch failures return MCL_EDEVICE.  The
 *    text of the last error on the calling thread is mcl_last_error().
 *  - Poses: 12 float32 rows of length N (structure of arrays), in this order:
 *    r00 r01 r02 r10 r11 r12 r20 r21 r22 tx ty tz - the rotation R (row-major)
 *    and translation t of the sensor in the map frame, the 6-DoF particle state
 *    of Eq. (2) in matrix form.
 *  - Scan points: 3 float32 rows x, y, z of length K in the sensor frame, in
 *    metres.  Any order is correct; ring-major order (neighbouring beams next to
 *    each other) makes the map reads of neighbouring lanes hit the same lines.
 */
#ifndef MCL_H
#define MCL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mcl_status;
#define MCL_OK 0
#define MCL_EINVAL (-1)  /* bad argument (NULL, size, value)                 */
#define MCL_ENOMEM (-2)  /* device allocation failed                          */
#define MCL_EDEVICE (-3) /* HIP runtime / launch error                        */
#define MCL_ERANGE (-4)  /* a size beyond the limits below                    */
#define MCL_EBUSY (-5)   /* a resource is held by earlier work (MCL_TICK_NOWAIT) */

#define MCL_MAX_PARTICLES (1 << 21) /* N per call                                */
#define MCL_MAX_POINTS (1 << 20)    /* K per call                                */
#define MCL_WQ_SHIFT 42             /* fixed-point weights are floor(w * 2^42)   */

/* Storage type of the TSDF values. */
typedef enum {
    MCL_TSDF_I16 = 0, /* q = rint(d / tau * 32767), int16               */
    MCL_TSDF_I8 = 1,  /* q = rint(d / tau * 127), int8                  */
    MCL_TSDF_F32 = 2  /* d itself, metres, float32                      */
} mcl_dtype;

/* A dense TSDF map (§III: a voxelised truncated signed distance field; values
 * are positive in free space, negative inside objects and clamped to the
 * truncation band [-tau, tau]).  Voxel (i, j, k) covers the half-open box
 * [origin + i*voxel, origin + (i+1)*voxel) per axis and holds the clamped
 * signed distance at its centre. */
typedef struct {
    int32_t nx, ny, nz; /* voxels per axis, >= 1                               */
    float voxel;        /* edge length v in metres, > 0                        */
    float origin[3];    /* map-frame position of the min corner of voxel (0,0,0) */
    float tau;          /* truncation distance in metres, > 0                  */
    int32_t dtype;      /* mcl_dtype                                           */
} mcl_map_desc;

typedef struct mcl_map_s *mcl_map; /* opaque; device-resident, immutable */

/* Upload a map.  host_values: HOST memory, nx*ny*nz values of the storage
 * type, x fastest (index i + nx*(j + ny*k)).  The library copies them to the
 * current device in its own brick layout and owns that copy; host_values may be
 * freed when the call returns (the call synchronises `stream`).  Limit: the
 * device copy must stay below 4 GiB.  *out receives the handle. */
mcl_status mcl_map_upload(const mcl_map_desc *desc, const void *host_values, void *stream,
                          mcl_map *out);

/* Upload a sparse coarse/fine map (§III: the map holds fine data only for the
 * parts of the coarse grid with distances inside the truncation band, after
 * Akai et al.).  The grid is cut into 4x4x4 bricks (brick (bx, by, bz) holds
 * voxels 4bx..4bx+3 etc.); only the listed bricks are stored, every other
 * voxel reads +Q (+tau): free or unobserved space.  Memory grows with the
 * number of stored bricks (the library keeps them in 8x32x4-voxel blocks, a
 * block being stored when any of its bricks is listed; mcl_map_bytes reports
 * the total), and the map may exceed the 4 GiB limit of the dense layout
 * (limits: nbx*nby*nbz < 2^31 bricks, ceil(nx/8)*ceil(ny/32) < 2^24).  The sensor
 * update gives exactly the results of the dense map with the same values; the
 * trilinear lookup and the uniform initialisation reject sparse maps, and
 * mcl_tick those whose blocks take 4 GiB or more.
 *   nstored:      number of listed bricks, >= 0.
 *   brick_coords: HOST [nstored][3] int32 (bx, by, bz), each brick at most once.
 *   brick_values: HOST [nstored][64] values of the storage type, in-brick index
 *                 x + 4 y + 16 z (voxels beyond the map edge are never read).
 * The call copies everything and synchronises `stream`. */
mcl_status mcl_map_upload_bricks(const mcl_map_desc *desc, int64_t nstored, const int32_t *brick_coords,
                                 const void *brick_values, void *stream, mcl_map *out);

/* Release a map.  Deferred: the call first waits for the work this library
 * has enqueued on the map (every call that reads it records an event on its
 * stream), then frees the device memory; the handle is invalid afterwards.
 * Work captured into a graph by the caller is not tracked (the events are
 * recorded only outside stream capture): keep such maps alive while the graph
 * may run.  A NULL map returns MCL_EINVAL. */
mcl_status mcl_map_free(mcl_map map);

/* Device bytes a map holds: its values, coarse level and sentinels, plus the
 * trilinear corner-cell copy once mcl_sensor_update_trilinear has built it.
 * 0 for a NULL map. */
size_t mcl_map_bytes(mcl_map map);

/* Sensor update, endpoint model (§III, Eq. 3).  For every particle n:
 *     logw[n] = -(1 / (2 sigma^2)) * sum_k m(x_n, z_k)^2
 * where m(x_n, z_k) is the map value of the voxel containing the scan point z_k
 * transformed by particle pose x_n (R p + t), and +tau for points outside the
 * map.  This is the log of the product of Eq. (3) over the scan without its
 * constant factor, which cancels in normalisation (the full log-likelihood is
 * logw[n] - (K / 2) ln(2 pi sigma^2)).
 * The voxel of a point follows a fixed float32 recipe (round-to-nearest-even;
 * fma is the IEEE fused multiply-add, one rounding): with
 * inv_v = (float)(1.0 / (double)voxel),
 *     a_jk = r_jk * inv_v,  b_j = (t_j - origin_j) * inv_v + 0,
 *     g_j  = fma(a_j2, z, fma(a_j1, y, fma(a_j0, x, b_j))),
 * valid iff 0 <= g_j < n_j on every axis with -0.0 counted below 0 (NaN is
 * outside), voxel index (int)g_j.
 * Sums of squares are accumulated in float32 in an order that depends only on
 * K (not on N or on how the work is split), with a relative error below 3e-6.
 *   points: device, [3][K] float32; K in [0, MCL_MAX_POINTS]; may be NULL if K = 0.
 *   poses:  device, [12][N] float32; N in [1, MCL_MAX_PARTICLES].
 *   sigma:  Eq. (3) standard deviation in metres, finite and > 0.
 *   logw:   device output, [N] float32; must not overlap the inputs. */
mcl_status mcl_sensor_update(mcl_map map, const float *points, int32_t K, const float *poses,
                             int32_t N, float sigma, float *logw, void *stream);

/* Sensor update with the sum reading of the same model (§III, Eq. 3: the
 * paper does not say how the points' likelihoods combine; this entry point
 * takes their sum instead of their product).  For every particle n:
 *     logw[n] = log sum_k exp(-(1 / (2 sigma^2)) * m(x_n, z_k)^2),
 * the log of the sum of Eq. (3) over the scan without its constant factor
 * (the full log of the sum is logw[n] - (1 / 2) ln(2 pi sigma^2));
 * logw[n] = 0 when K = 0 (no evidence: equal weights, as mcl_sensor_update
 * gives).  Lookup and voxel recipe as for mcl_sensor_update.  Each likelihood
 * is computed in float32 as 2^(k2 q^2) with k2 = -c log2(e) (c the score
 * constant of mcl_sensor_update) by the hardware base-2 exponential, and the
 * likelihoods are summed in float32 in the order of mcl_sensor_update; the
 * absolute error of logw[n] stays below
 *     2.2e-6 + 1.8e-7 * tau^2 / (2 sigma^2) + 1.8e-7 * |logw[n]|.
 * Dense maps only, and sigma >= tau / 8, so that no likelihood underflows
 * (MCL_EINVAL otherwise).  Other arguments and errors as for mcl_sensor_update. */
mcl_status mcl_sensor_update_sum(mcl_map map, const float *points, int32_t K, const float *poses,
                                 int32_t N, float sigma, float *logw, void *stream);

/* The sensor update for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Results are bit for bit those of mcl_sensor_update (same kernels, the same
 * arithmetic).  Instead of the stream's workspace (the piece partials and a
 * table of the particles' 12 pose constants), the piece partials
 * (N * ceil(K / 4096) floats when K > 4096; none otherwise) live in a fixed
 * device array, and the pose constants are passed between lanes; the array is
 * of MCL_NOALLOC_SCRATCH_BYTES, which the library holds on each GPU it runs on until
 * the process ends.  The call allocates nothing and records no map-use event
 * (so mcl_map_free does not wait for this work: keep the map alive until the
 * stream has run it).  Every call on one GPU shares that GPU's array: calls
 * that may overlap on one GPU race and must be ordered by the caller (one
 * stream, or events).  MCL_ERANGE if the partials exceed the array (for
 * example N = 10^6 needs K <= 16 * 4096).  Other arguments and errors as for
 * mcl_sensor_update. */
#define MCL_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
mcl_status mcl_sensor_update_noalloc(mcl_map map, const float *points, int32_t K, const float *poses,
                                     int32_t N, float sigma, float *logw, void *stream);

/* Sensor update with a trilinear lookup (§III: a pseudo-continuous map value by
 * interpolation).  As mcl_sensor_update, except that m(x_n, z_k) is the
 * trilinear interpolation of the 8 voxel centres around the transformed point
 * (the stored values sit at the centres; a centre outside the map reads +tau).
 * With g_j from the recipe above, in float32:
 *     h_j = min(max(g_j - 0.5, -2), n_j + 1),  i_j = floor(h_j),  f_j = h_j - i_j,
 * and m = sum over the 8 corners (i_x + a, i_y + b, i_z + c), a, b, c in {0, 1},
 * of (a ? f_x : 1 - f_x)(b ? f_y : 1 - f_y)(c ? f_z : 1 - f_z) * value, computed
 * as lerps along x, then y, then z, lerp(p, q, t) = fma(t, q - p, p).
 * Each interpolated value is within 10 eps M of the exact one (M the largest
 * stored magnitude, eps = 2^-24: three levels of lerps, each adding at most one
 * rounding of its fma and one of its difference), so the relative error of logw
 * is at most the float32 sum bound above plus
 * (20 eps M sum|m| + 100 K eps^2 M^2) / sum m^2.  Arguments and errors as for
 * mcl_sensor_update. */
mcl_status mcl_sensor_update_trilinear(mcl_map map, const float *points, int32_t K, const float *poses,
                                       int32_t N, float sigma, float *logw, void *stream);

/* Weight normalisation (§V-A: the particle weights are summed for
 * normalisation), float64 log-sum-exp:
 *     log_z = max_n l_n + log sum_n exp(l_n - max l),  w_n = exp(l_n - log_z),
 *     wq_n  = floor(w_n * 2^42)   (64-bit fixed point for an exact integer scan).
 *   logw:  device, [N] float32, finite; N in [1, MCL_MAX_PARTICLES].
 *   w:     device output [N] float64, or NULL.
 *   wq:    device output [N] uint64 (required).
 *   log_z: device output [1] float64, or NULL. */
mcl_status mcl_normalize(const float *logw, int32_t N, double *w, uint64_t *wq, double *log_z,
                         void *stream);

/* Low-variance (systematic) resampling (§III: a new particle set is drawn from
 * the weighted one).  With C_i = wq_0 + ... + wq_i and T = C_{N-1}, the offset
 * is r = floor(u * T / 2^64) for one uniform 64-bit draw u, and output slot m
 * takes the particle i with N*C_{i-1} <= m*T + r < N*C_i.  Integer only: the
 * result is exact.  T = 0 is treated as equal weights (idx[m] = m).
 * The draw (the paper names no generator; reading): u = splitmix64(seed XOR
 * splitmix64(tick)), splitmix64(x) being the output of SplitMix64 (Steele, Lea
 * and Flood, OOPSLA 2014) from state x: z = x + 0x9E3779B97F4A7C15,
 * z = (z ^ z >> 30) * 0xBF58476D1CE4E5B9, z = (z ^ z >> 27) * 0x94D049BB133111EB,
 * z ^ z >> 31 (all modulo 2^64).  A filter keeps one seed and counts its updates
 * in tick, so a resampling step is reproducible from (seed, tick) alone.
 * Precondition: N * T < 2^64 (true for the output of mcl_normalize).
 *   wq:        device, [N] uint64; N in [1, MCL_MAX_PARTICLES].
 *   seed, tick: select the draw.
 *   idx:       device output [N] int32, non-decreasing ancestor indices.
 *   poses_in / poses_out: device [12][N] float32, both NULL (indices only) or
 *              both set; poses_out[:, m] = poses_in[:, idx[m]]; no overlap. */
mcl_status mcl_resample(const uint64_t *wq, int32_t N, uint64_t seed, uint64_t tick, int32_t *idx,
                        const float *poses_in, float *poses_out, void *stream);

/* Pose estimate of a weighted particle set (§III: the weighted average of the
 * particles, or the particle of highest weight; §V: a second reduction forms
 * the weighted sum of the poses).  The paper does not say how rotations are
 * averaged; here:
 *   position  t* = sum_n w_n t_n / sum_n w_n
 *   rotation  R* = the rotation nearest to S = sum_n w_n R_n, the maximiser of
 *             trace(R^T S) over SO(3) (weighted chordal L2 mean; for exact
 *             rotations equal to the eigenvector quaternion average).  When S
 *             has a repeated largest singular-value combination the maximiser is
 *             not unique and any maximiser may be returned.
 *   sum_n w_n = 0 is read as equal weights.
 *   w:         device [N] float64 weights, finite and >= 0 (as mcl_normalize
 *              writes them); other values give an unspecified estimate.
 *   poses:     device [12][N] float32 particle poses.
 *   mean:      device output [12] float64, the estimate in the particle layout
 *              (r00 r01 r02 r10 r11 r12 r20 r21 r22 tx ty tz).
 *   best_idx:  device output [1] int32 or NULL: the smallest index among the
 *              largest weights (-1 if no weight exceeds -inf).
 *   best_pose: device output [12] float32 or NULL: poses[:, best_idx] exactly
 *              (NaN if best_idx is -1).
 * Float64 sums in an order fixed by N alone: results are reproducible. */
mcl_status mcl_pose_estimate(const double *w, const float *poses, int32_t N, double *mean,
                             int32_t *best_idx, float *best_pose, void *stream);

/* ---------------------------------------------------- motion and initialisation
 * Random numbers: Philox4x32-10 (Salmon et al., SC 2011), counter (n, lo32(step),
 * hi32(step), c), key (lo32(seed), hi32(seed)): particle n's draws depend only on
 * (seed, step, n), never on the launch.  Uniforms from a 32-bit word x:
 * ((x >> 8) + 1) 2^-24 in (0, 1] and (x >> 8) 2^-24 in [0, 1). */

/* Motion update (§III: every iteration first moves each particle by the motion
 * model; §VI: odometry from dead reckoning or an IMU, with noise on velocity
 * and angular velocity).  The paper gives no formula; here the odometry
 * increment is a rigid motion (dR, dt) in the robot frame and each particle
 * moves by its own noisy copy:
 *     n0..n5 = six standard normals (Box-Muller on Philox words 0..5 of
 *              counters (n, step, 0) and (n, step, 1)),
 *     dt' = dt + sigma_t (n0, n1, n2),   dR' = dR Exp(sigma_r (n3, n4, n5)),
 *     R <- R dR',   t <- R dt' + t        (float32).
 *   poses_in:  device [12][N] float32; poses_out: device [12][N], may equal
 *              poses_in (in place) but must not overlap it otherwise.
 *   delta:     HOST [12] float32, the increment (dR row-major, dt), finite.
 *   sigma_t, sigma_r: standard deviations of the increment's translation (m)
 *              and rotation (rad) noise, >= 0 (velocity noise times the step).
 *   seed, step: select the random numbers (use a new step every update). */
mcl_status mcl_motion_update(const float *poses_in, float *poses_out, int32_t N, const float *delta,
                             float sigma_t, float sigma_r, uint64_t seed, uint64_t step, void *stream);

/* Initialisation round a pose estimate (§III: with an initial estimate the
 * particles are spread with a preset variance around it).  Exactly the motion
 * update above applied to N copies of `mean` with the identity increment:
 *     R = R_mean Exp(sigma_r (n3, n4, n5)),  t = t_mean + R_mean sigma_t (n0, n1, n2)
 * (noise in the frame of the estimate), same random numbers and float32 steps
 * as mcl_motion_update(copies of mean, identity, sigma_t, sigma_r, seed, step).
 *   poses:   device output [12][N] float32.
 *   mean:    HOST [12] float32, the estimate (R row-major, t), finite.
 *   sigma_t, sigma_r: deviations (m, rad), >= 0. */
mcl_status mcl_init_gaussian(float *poses, int32_t N, const float *mean, float sigma_t, float sigma_r,
                             uint64_t seed, uint64_t step, void *stream);

/* Uniform initialisation in free space (§III: without an initial pose estimate
 * the particles are distributed uniformly in free space).  Free voxels are
 * those with a stored value > 0, counted in x-fastest order; with F of them,
 * particle n takes the free voxel of rank floor(U F / 2^64), U = w0 + 2^32 w1
 * from counter (n, 0, 0, 2), a position uniform inside it,
 *     p_j = origin_j + ((float) i_j + u) * voxel   (float32, each step rounded),
 * u from w2, w3, w4 in [0, 1), and the orientation Rz(yaw) Ry(pitch) Rx(roll)
 * with yaw = pi (2 u5 - 1) and pitch, roll = max_tilt (2 u - 1) from w6, w7
 * (counter (n, 0, 0, 3)).  The first call on a map counts its free voxels
 * (one kernel and a host prefix sum; synchronises `stream`).
 *   poses:    device output [12][N] float32.
 *   max_tilt: largest |roll| and |pitch| in radians, >= 0.
 * Returns MCL_EINVAL if the map has no free voxel. */
mcl_status mcl_init_uniform(mcl_map map, float *poses, int32_t N, float max_tilt, uint64_t seed,
                            void *stream);

/* ------------------------------------------------------------- batching
 * One MCL update of many filters at once (the filters may use different maps,
 * particle counts and scan sizes).  mcl_tick runs, for every filter, exactly
 * mcl_sensor_update, then mcl_normalize, then (for filters that ask for it)
 * mcl_pose_estimate on the normalised weights and the input poses, then
 * mcl_resample: each stage is one launch over all filters together (the
 * sensor update one launch per storage type and lookup: nearest on dense
 * maps, nearest on sparse maps, trilinear on dense maps, nearest on dense maps
 * with the sum reading), and every filter's
 * results are bit for bit those of the single-filter calls (the trilinear
 * lookup's corner cells are built on the map's first trilinear use, as by
 * mcl_sensor_update_trilinear).  Sparse maps are accepted when their blocks
 * take less than 4 GiB (MCL_EINVAL otherwise).  Buffers follow the rules of the single-filter
 * calls; all buffers of all jobs must be distinct. */
#define MCL_MAX_JOBS 4096

typedef struct {
    mcl_map map;            /* the filter's map                                   */
    const float *points;    /* device [3][K]; may be NULL if K = 0                */
    int32_t K;              /* scan points, [0, MCL_MAX_POINTS]                   */
    const float *poses;     /* device [12][N] particle poses                      */
    int32_t N;              /* particles, [1, MCL_MAX_PARTICLES]                  */
    float sigma;            /* Eq. (3) sigma, metres                              */
    float *logw;            /* device out [N]                                     */
    double *w;              /* device out [N], or NULL                            */
    uint64_t *wq;           /* device out [N]                                     */
    double *log_z;          /* device out [1], or NULL                            */
    uint64_t seed, tick;    /* resampling draw, as for mcl_resample               */
    int32_t *idx;           /* device out [N] ancestor indices                    */
    float *poses_out;       /* device out [12][N] resampled poses, or NULL        */
    double *est_mean;       /* device out [12], or NULL: the pose estimate of the
                               weighted set (as mcl_pose_estimate); needs w       */
    int32_t *est_idx;       /* device out [1] best particle, or NULL              */
    float *est_pose;        /* device out [12] best particle's pose, or NULL      */
    int32_t lookup;         /* MCL_LOOKUP_NEAREST (as mcl_sensor_update) or
                               MCL_LOOKUP_TRILINEAR (as mcl_sensor_update_trilinear,
                               dense maps only)                                   */
    int32_t score;          /* MCL_SCORE_PRODUCT (0: as mcl_sensor_update) or
                               MCL_SCORE_SUM (as mcl_sensor_update_sum: dense maps,
                               nearest lookup, sigma >= tau / 8)                  */
} mcl_filter_job;

#define MCL_LOOKUP_NEAREST 0
#define MCL_LOOKUP_TRILINEAR 1
#define MCL_SCORE_PRODUCT 0
#define MCL_SCORE_SUM 1

/* Flag for mcl_tick: the launch chain is captured into a HIP graph the first
 * time (per stream and per mix of storage types and lookups) and replayed afterwards;
 * job tables are copied to the device before each replay.  Needs a
 * non-default stream. */
#define MCL_TICK_GRAPH 1
/* Flag for mcl_tick: do not wait for the stream's table staging buffer.  A tick
 * copies its job tables from a pinned host buffer (one per stream); while the
 * copy of the previous tick on that stream has not run yet (it runs in stream
 * order, after the work enqueued before it), the call returns MCL_EBUSY and
 * enqueues nothing, instead of blocking the calling thread. */
#define MCL_TICK_NOWAIT 2

/* Run one tick for n_jobs filters (1..MCL_MAX_JOBS) on `stream`.  The job array
 * is read during the call (it may be reused when the call returns).  Returns
 * the first argument error with the failing job's index in mcl_last_error(). */
mcl_status mcl_tick(const mcl_filter_job *jobs, int32_t n_jobs, int32_t flags, void *stream);

/* Device bytes one filter of N particles and K points needs in a tick: the
 * caller's buffers (poses in and out, logw, w, wq, idx, scan) plus the
 * library's workspace for it.  For admission control; 0 for invalid sizes. */
size_t mcl_job_bytes(int32_t N, int32_t K);

/* --------------------------------------------------------------- tuning
 * Launch settings of the sensor kernel; none changes a result (the summation
 * order depends only on K):
 *   waves_per_block: 2, 4 or 8;
 *   blocks_per_cu:   0 = one wave per work item, else a persistent grid of that
 *                    many workgroups per compute unit;
 *   coarse:          where the nearest lookup reads the coarse level: 0 = chosen
 *                    per wave and chunk (default), 1 = bytes in global memory,
 *                    2 = bits copied into LDS (only for maps whose bit table fits
 *                    64 KiB, and in mcl_tick only for a storage type whose filters
 *                    all share one map; otherwise 1);
 *   runs:            runs per 64-particle group (work items per group and
 *                    4096-point piece): 0 = from the launch's size (more runs for
 *                    small launches, so they spread over the chip), else 1, 2, 4,
 *                    .., 64;
 *   lds_threshold:   with coarse = 0, a wave reads the bits in LDS when more than
 *                    lds_threshold / 8 of its probe lookups read in place (1..8;
 *                    0 = the default 6).
 * Sparse maps use a fixed shape.  mcl_tick uses, per storage type, the shape and
 * runs stored for the largest filter of that type (which also decides whether
 * the launch holds the bits in LDS), and for each filter the coarse mode and
 * threshold stored for its own size class. */
typedef struct {
    int32_t waves_per_block;
    int32_t blocks_per_cu;
    int32_t coarse;
    int32_t runs;
    int32_t lds_threshold;
} mcl_launch_config;

/* Time launch settings on the given filter by coordinate descent (the launch
 * shape, then runs, then the coarse level; each the median of three batches of
 * back-to-back launches, a batch lasting about 2 ms; synchronises `stream`), keep the fastest for its storage type and
 * size class (K and N rounded up to powers of two) for later mcl_sensor_update
 * / mcl_tick calls, and return it in *best (may be NULL).  With the environment
 * variable MCL_TUNE_CACHE naming a file, results are appended to it and read
 * back by later processes on the same kind of GPU.  logw_scratch: device [N]
 * float32 the trials write. */
mcl_status mcl_autotune(mcl_map map, const float *points, int32_t K, const float *poses, int32_t N, float sigma,
                        float *logw_scratch, void *stream, mcl_launch_config *best);

/* Set (or with NULL clear) the setting used for a storage type and size class,
 * as mcl_autotune would (in this process only). */
mcl_status mcl_set_launch_config(int32_t dtype, int32_t K, int32_t N, const mcl_launch_config *cfg);

/* The setting mcl_sensor_update would use for a storage type and sizes: the
 * stored one for their size class (set, tuned, or read from MCL_TUNE_CACHE),
 * else the default {4, 0, 0, 0, 0}. */
mcl_status mcl_get_launch_config(int32_t dtype, int32_t K, int32_t N, mcl_launch_config *out);

/* Launch shape of the normalisation and resampling (Sec. V-A, Sec. III):
 * mcl_normalize and mcl_resample on a filter of at most max_n particles, and
 * mcl_tick when none of its filters has more, run one workgroup per filter in
 * one launch instead of a chain of three launches over the chip (six in a
 * tick).  Both shapes perform the same floating-point operations in the same
 * order, so every output is bit-identical either way; only the time differs.
 * max_n in [0, 4096]; 0 turns the one-launch shape off; the default is 4096.
 * Process-wide; a tick replayed from a graph uses the graph of the shape its
 * filters select.  Errors: MCL_ERANGE for max_n out of range. */
mcl_status mcl_set_weights_fused_max(int32_t max_n);

/* The current max_n of mcl_set_weights_fused_max. */
int32_t mcl_get_weights_fused_max(void);

/* Order in which the sensor update (Sec. III, Eq. 3) visits a filter's
 * particles: mcl_sensor_update, mcl_sensor_update_sum and mcl_tick sort a
 * dense-map filter of at least min_evals particle-point evaluations (N * K) by
 * the cell of its particles' x-y positions (64 x 64 cells over the map, in
 * Morton order) before the lookups, so that particles evaluated together, and
 * by the same part of the chip, read nearby map regions and share cache lines.
 * Each particle's log-weight is computed by exactly the same operations and
 * written to its own index, so every output is bit-identical with or without
 * the order; only the time differs.  The order costs four short launches and
 * 8 bytes per particle of workspace.  A negative min_evals turns it off; the
 * default is 2^30.  Process-wide; the sparse-map and trilinear lookups and
 * mcl_sensor_update_noalloc never order.  Always MCL_OK. */
mcl_status mcl_set_spatial_order_min(int64_t min_evals);

/* The current min_evals of mcl_set_spatial_order_min. */
int64_t mcl_get_spatial_order_min(void);

/* Test support: the voxel each (particle, point) pair reads, by the same
 * device code as mcl_sensor_update.  lin_idx: device output [N][K] int64,
 * i + nx*(j + ny*k), or -1 outside the map.  N*K must not exceed 2^31. */
mcl_status mcl_debug_voxel_indices(mcl_map map, const float *points, int32_t K,
                                   const float *poses, int32_t N, int64_t *lin_idx,
                                   void *stream);

/* Test support: Philox4x32-10 of one counter and key on the device, by the same
 * device code as the motion update and the initialisation.  counter_key: HOST
 * [6] (counter words 0..3, key words 0..1); out: HOST [4].  Synchronous, on the
 * default stream. */
mcl_status mcl_debug_philox(const uint32_t *counter_key, uint32_t *out);

/* ------------------------------------------------------- measurement support
 * The sensor update is bound by its map gathers (the TSDF look-ups, §VI-C).
 * These calls measure the ceilings it is judged against; they compute nothing
 * of the method.  Every kernel writes one float per thread to `sink` (device,
 * at least blocks * 256 floats) so that no load can be dropped. */

/* The byte offset, within the map's value allocation, that the nearest lookup
 * of mcl_sensor_update reads for every (particle, point) pair, computed by the
 * same device code: the voxel's offset or 0 outside the map; with masked != 0
 * the brick's read mask applied (the offset actually read: 0, the +Q sentinel,
 * for bricks wholly at +-Q).  offs: device output [N][K] uint32.  Dense maps. */
mcl_status mcl_bench_gather_offsets(mcl_map map, const float *points, int32_t K, const float *poses, int32_t N,
                                    int32_t masked, uint32_t *offs, void *stream);

/* Replay of the sensor kernel's gathers for S particles (a multiple of 64)
 * whose offsets mcl_bench_gather_offsets wrote (offs [S][K]): work items of 64
 * particles x 4096 points, lanes holding points l, l + 64, ... of each 1024-point
 * chunk as in the sensor kernel; per particle and chunk each lane loads its 16
 * offsets, then issues `reps` times its 16 gathers: with two_gathers the read
 * mask byte and the value at (offset AND mask) (offs unmasked), else the value
 * at the offset (offs masked).  `blocks` workgroups of 4 waves. */
mcl_status mcl_bench_gather_replay(mcl_map map, const uint32_t *offs, int32_t S, int32_t K, int32_t reps,
                                   int32_t two_gathers, int32_t blocks, float *sink, size_t sink_floats,
                                   void *stream);

/* Random 128-byte line gathers: each 64-lane gather reads bytes_per_lane (1, 2
 * or 4) bytes per lane from `lines` (1..64, a power of two) lines chosen at
 * random among the first 2^log2_lines lines of `region` (device, region_bytes
 * >= 128 * 2^log2_lines), the lanes sharing a line at consecutive addresses;
 * 16 gathers in flight per wave, `steps` x 16 gathers per wave. */
mcl_status mcl_bench_line_gather(const void *region, size_t region_bytes, int32_t log2_lines, int32_t lines,
                                 int32_t bytes_per_lane, int32_t steps, uint32_t seed, int32_t blocks, float *sink,
                                 size_t sink_floats, void *stream);

/* Texture-path cost of a gather: each 64-lane gather reads bytes_per_lane (1, 2
 * or 4) bytes per lane from exactly `lines` (1..64, a power of two) 128-byte
 * lines of one 8 KiB block (block_bytes >= 8192), which stays in the L1 cache;
 * the address is a scalar base plus a fixed lane offset, so no vector
 * arithmetic competes with the loads; `steps` x 16 gathers per wave. */
mcl_status mcl_bench_l1_gather(const void *block, size_t block_bytes, int32_t lines, int32_t bytes_per_lane,
                               int32_t steps, int32_t blocks, float *sink, size_t sink_floats, void *stream);

/* Coalesced 16-byte loads over `bytes` (a multiple of 16) of device memory. */
mcl_status mcl_bench_stream_read(const void *src, size_t bytes, int32_t blocks, float *sink, size_t sink_floats,
                                 void *stream);

/* Text of the last error on the calling thread ("" if none). */
const char *mcl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCL_H */

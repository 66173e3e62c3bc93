/*
 * CPU oracle for the 6-DoF MCL sensor update, weight normalisation and
 * resampling of Eisoldt et al., "Towards 6D MCL for LiDARs in 3D TSDF Maps on
 * Embedded Systems with GPUs" (arXiv 2310.04172).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  The product (the HIP library) never
 * calls it, and the two share no code.
 *
 * Plain and slow on purpose: one particle at a time, one scan point at a time,
 * in the order of the definitions.  Arithmetic is float64 or exact integer,
 * except the voxel-index step, whose float32 operations are a fixed recipe (so
 * that voxel indices can be compared bit for bit with any other implementation
 * of the same recipe).  Build with -ffp-contract=off: the recipe's fused
 * multiply-adds are explicit fmaf calls (IEEE fusedMultiplyAdd, one rounding).
 *
 * Definitions, with the reading taken where the paper is silent:
 *
 *  Particle (Eq. 1, Eq. 2): p = (s, w), s a 6-DoF pose.  Handed over as the
 *    rotation matrix R (row-major) and translation t of the sensor in the world,
 *    12 float32 rows r00 r01 r02 r10 r11 r12 r20 r21 r22 tx ty tz, each of
 *    length N (structure of arrays).
 *
 *  Map (§III): dense TSDF, voxel (i,j,k) covers [o + i v, o + (i+1) v) per axis,
 *    values clamped to the truncation band; stored x-fastest
 *    (index i + nx (j + ny k)) as int16 / int8 fixed point q = d / tau * Q
 *    (Q = 32767 / 127) or float32 metres.  Reading: nearest-voxel lookup (the
 *    voxel that contains the point, half-open cells); a point outside the map
 *    reads +Q (+tau), truncated free space.
 *
 *  Voxel-index recipe (float32, IEEE round-to-nearest-even):
 *      inv_v = (float)(1.0 / (double)v)                        once per map
 *      a_jk  = r_jk * inv_v ;  b_j = (t_j - o_j) * inv_v + 0      once per particle
 *      g_j   = fma(a_j2, pz, fma(a_j1, py, fma(a_j0, px, b_j)))  per point
 *      valid iff 0 <= g_j < n_j for j = x, y, z, where -0.0 counts as below 0
 *      (the sign bit decides) ;  i_j = (int) g_j.
 *    The "+ 0" maps an offset of -0.0 to +0.0 (so that t = -0.0 and t = +0.0
 *    select alike); a g_j of -0.0 can then only come from a negative exact value
 *    too small to represent, which lies below 0.
 *
 *  Sensor model (Eq. 3, endpoint model): a point's likelihood is a Gaussian in
 *    the map distance m(x, z).  Reading: a particle's weight is the product over
 *    the scan points (independent beams), kept in the log domain without the
 *    constant factor (it cancels in normalisation):
 *        l_n = -(s^2 / (2 sigma^2)) * sum_k q_k^2,   s = tau / Q (s = 1 for float32).
 *    The sum of squares is exact (int64) for fixed-point maps and float64 for
 *    float32 maps (each square is exact in float64).  A float64 map (the
 *    unquantised distances) serves as the precision reference of the storage
 *    types.
 *    The other reading (a mode of its own): the weight is the sum of the
 *    points' likelihoods instead of their product, again without the constant
 *    factor,
 *        l_n = log sum_k exp(-(s^2 / (2 sigma^2)) q_k^2),
 *    float64 terms added in point order; an empty scan gives l_n = 0 (no
 *    evidence: equal weights, as the product reading gives).
 *
 *  Sparse coarse/fine map (§III, after Akai et al.: fine data only where the
 *    coarse grid holds distances inside the truncation band).  A storage form
 *    only: 4x4x4 bricks of the voxel grid are listed with their values and
 *    every voxel of an unlisted brick reads +Q (+tau); the score is the dense
 *    definition on those values.
 *
 *  Trilinear lookup (§III: a pseudo-continuous state by interpolation).
 *    Reading: the stored values sit at the voxel centres, grid coordinate
 *    i + 1/2; a point's map value is the trilinear interpolation of the 8
 *    centres around it, a centre outside the map reading +Q (+tau).  Recipe:
 *    g_j as above (float32), then in float32
 *        h_j = g_j - 0.5 ;  h_j = min(max(h_j, -2), n_j + 1) ;
 *        i_j = (int) floor(h_j) ;  f_j = h_j - floor(h_j)   (exact),
 *    (the clamp only moves points whose 8 centres are all outside, and sends
 *    NaN there), then in float64
 *        m = sum over a, b, c in {0, 1} of
 *            (a ? f_x : 1 - f_x)(b ? f_y : 1 - f_y)(c ? f_z : 1 - f_z) d(i_x + a, i_y + b, i_z + c)
 *    with d the stored value (int16 / int8 in units of Q, or metres), and
 *        l_n = -(s^2 / (2 sigma^2)) * sum_k m_k^2.
 *
 *  Normalisation (§V-A sums the weights for normalisation), float64:
 *        m = max_n l_n ;  S = sum_n exp(l_n - m) ;
 *        log Z = m + log S ;  w_n = exp(l_n - log Z) ;
 *    S is meant exactly: the terms are added with compensation (Neumaier's
 *    variant of Kahan summation), so the computed S is within 2 units of
 *    rounding of the terms' exact sum whatever N is, where a plain sum in index
 *    order could drift by up to N - 1 units.
 *        W_n = floor(w_n * 2^42)  (64-bit fixed point, for an integer scan).
 *
 *  Resampling (§III: a new particle set is drawn from the weighted one).
 *    Reading: low-variance (systematic) resampling on the fixed-point weights.
 *    With C_i = W_0 + ... + W_i, T = C_{N-1} and one uniform 64-bit draw u,
 *    the offset is r = floor(u T / 2^64) in [0, T), and output slot m takes the
 *    particle i whose scaled cell [N C_{i-1}, N C_i) holds m T + r.  Written
 *    below as the familiar single sweep with a moving threshold.  T = 0 (every
 *    weight zero) is read as equal weights: slot m takes particle m.
 *    The draw: the paper names no generator.  Reading: a filter keeps one
 *    64-bit seed and counts its updates (tick); the update's draw is
 *        u = splitmix64(seed XOR splitmix64(tick)),
 *    splitmix64(x) being the output of SplitMix64 (Steele, Lea and Flood,
 *    "Fast splittable pseudorandom number generators", OOPSLA 2014) from state
 *    x: the state advances by the golden-ratio increment 0x9E3779B97F4A7C15,
 *    then two xor-shift-multiply rounds and a final xor-shift mix it.
 */

#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORACLE_I16 = 0, ORACLE_I8 = 1, ORACLE_F32 = 2, ORACLE_F64 = 3 };

typedef struct {
    int32_t n[3];
    float inv_v;
    float o[3];
} grid_t;

static grid_t make_grid(const int32_t dims[3], float voxel, const float origin[3]) {
    grid_t g;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = dims[a];
        g.o[a] = origin[a];
    }
    g.inv_v = (float)(1.0 / (double)voxel);
    return g;
}

/* Per-particle constants of the index recipe. */
static void particle_consts(const float *poses, int64_t N, int64_t n, const grid_t *g,
                            float a[9], float b[3]) {
    for (int j = 0; j < 3; ++j) {
        for (int k = 0; k < 3; ++k) {
            float r = poses[(int64_t)(3 * j + k) * N + n];
            a[3 * j + k] = r * g->inv_v;
        }
        float shifted = poses[(int64_t)(9 + j) * N + n] - g->o[j];
        b[j] = shifted * g->inv_v + 0.0f; /* -0.0 -> +0.0, every other value unchanged */
    }
}

/* Linear voxel index i + nx (j + ny k) of one point, or -1 outside the map. */
static int64_t voxel_index(const float a[9], const float b[3], float px, float py, float pz,
                           const grid_t *g) {
    int32_t idx[3];
    for (int j = 0; j < 3; ++j) {
        float s = fmaf(a[3 * j + 0], px, b[j]);
        s = fmaf(a[3 * j + 1], py, s);
        s = fmaf(a[3 * j + 2], pz, s);
        /* inside iff 0 <= s < n with -0.0 taken as below 0; NaN fails too */
        if (signbit(s) || !(s < (float)g->n[j])) return -1;
        idx[j] = (int32_t)s;
    }
    return (int64_t)idx[0] + (int64_t)g->n[0] * ((int64_t)idx[1] + (int64_t)g->n[1] * idx[2]);
}

int oracle_voxel_indices(const int32_t dims[3], float voxel, const float origin[3],
                         const float *points, int32_t K, const float *poses, int32_t N,
                         int64_t *lin) {
    if (K < 0 || N < 0) return -1;
    grid_t g = make_grid(dims, voxel, origin);
    for (int64_t n = 0; n < N; ++n) {
        float a[9], b[3];
        particle_consts(poses, N, n, &g, a, b);
        for (int64_t k = 0; k < K; ++k)
            lin[n * K + k] = voxel_index(a, b, points[k], points[K + k], points[2 * (int64_t)K + k], &g);
    }
    return 0;
}

/* ------------------------------------------------------------ sensor update */

typedef struct {
    grid_t g;
    int32_t dtype;
    const void *values;
    double tau;
    int32_t Q;
    const float *points;
    int64_t K;
    const float *poses;
    int64_t N;
    double c;          /* s^2 / (2 sigma^2) */
    double *logw;
    double *ssum;
    int64_t n0, n1;    /* this worker's particle range */
    /* sparse coarse/fine map: slot per 4x4x4 brick (-1: not stored), bricks of 64 values */
    const int32_t *table;
    const void *bricks;
    int64_t nbx, nby, nbz;
} su_job_t;

/* Stored value of voxel v (linear index) of a sparse map as an exact double:
 * the listed brick's value, or Q (tau) for bricks that are not listed. */
static double sparse_value(const su_job_t *J, int64_t v) {
    const int64_t nx = J->g.n[0], ny = J->g.n[1];
    const int64_t i = v % nx, j = (v / nx) % ny, k = v / (nx * ny);
    const int64_t b = (k >> 2) + J->nbz * ((i >> 2) + J->nbx * (j >> 2));
    const int32_t slot = J->table[b];
    if (slot < 0) return J->dtype == ORACLE_F32 ? (double)(float)J->tau : (double)J->Q;
    const int64_t e = (int64_t)slot * 64 + (i & 3) + 4 * (j & 3) + 16 * (k & 3);
    switch (J->dtype) {
    case ORACLE_I16: return ((const int16_t *)J->bricks)[e];
    case ORACLE_I8: return ((const int8_t *)J->bricks)[e];
    default: return ((const float *)J->bricks)[e];
    }
}

/* Sum of squared map values over the scan for particle n: exact for fixed point. */
static double particle_sum_sq(const su_job_t *J, int64_t n) {
    float a[9], b[3];
    particle_consts(J->poses, J->N, n, &J->g, a, b);
    const float *px = J->points, *py = J->points + J->K, *pz = J->points + 2 * J->K;
    if (J->table) { /* sparse map; exact for fixed point (integers < 2^53 in total) */
        double acc = 0.0;
        for (int64_t k = 0; k < J->K; ++k) {
            int64_t v = voxel_index(a, b, px[k], py[k], pz[k], &J->g);
            double d = v < 0 ? (J->dtype == ORACLE_F32 ? (double)(float)J->tau : (double)J->Q) : sparse_value(J, v);
            acc += d * d;
        }
        return acc;
    }
    if (J->dtype == ORACLE_F32) {
        const float *vals = (const float *)J->values;
        double acc = 0.0;
        for (int64_t k = 0; k < J->K; ++k) {
            int64_t v = voxel_index(a, b, px[k], py[k], pz[k], &J->g);
            double d = v < 0 ? (double)(float)J->tau : (double)vals[v];
            acc += d * d;
        }
        return acc;
    }
    if (J->dtype == ORACLE_F64) { /* precision reference: the unquantised distances */
        const double *vals = (const double *)J->values;
        double acc = 0.0;
        for (int64_t k = 0; k < J->K; ++k) {
            int64_t v = voxel_index(a, b, px[k], py[k], pz[k], &J->g);
            double d = v < 0 ? (double)(float)J->tau : vals[v];
            acc += d * d;
        }
        return acc;
    }
    int64_t acc = 0;
    for (int64_t k = 0; k < J->K; ++k) {
        int64_t v = voxel_index(a, b, px[k], py[k], pz[k], &J->g);
        int64_t q;
        if (v < 0)
            q = J->Q;
        else if (J->dtype == ORACLE_I16)
            q = ((const int16_t *)J->values)[v];
        else
            q = ((const int8_t *)J->values)[v];
        acc += q * q;
    }
    return (double)acc; /* < 2^50, exact */
}

static void *su_worker(void *arg) {
    su_job_t *J = (su_job_t *)arg;
    for (int64_t n = J->n0; n < J->n1; ++n) {
        double S = particle_sum_sq(J, n);
        if (J->ssum) J->ssum[n] = S;
        J->logw[n] = -(S * J->c);
    }
    return NULL;
}

/*
 * l_n for every particle (see the header comment).  ssum may be NULL; else it
 * receives the sum of squared stored values (exact integers for fixed point).
 * nthreads > 1 splits the particles into that many contiguous groups, one
 * thread each, as the paper's CPU implementation does (§V-A); the result does
 * not depend on the thread count.
 */
int oracle_sensor_update(const int32_t dims[3], float voxel, const float origin[3], float tau,
                         int32_t dtype, const void *values, const float *points, int32_t K,
                         const float *poses, int32_t N, float sigma, double *logw, double *ssum,
                         int32_t nthreads) {
    if (K < 0 || N < 0 || dtype < 0 || dtype > 3 || !(sigma > 0.0f)) return -1;
    su_job_t base;
    memset(&base, 0, sizeof base);
    base.g = make_grid(dims, voxel, origin);
    base.dtype = dtype;
    base.values = values;
    base.tau = (double)tau;
    base.Q = dtype == ORACLE_I16 ? 32767 : dtype == ORACLE_I8 ? 127 : 1;  /* 1: metres (float32 / float64) */
    base.points = points;
    base.K = K;
    base.poses = poses;
    base.N = N;
    double s = dtype >= ORACLE_F32 ? 1.0 : (double)tau / (double)base.Q;
    double sg = (double)sigma;
    base.c = (s * s) / (2.0 * sg * sg);
    base.logw = logw;
    base.ssum = ssum;
    if (nthreads <= 1 || N < 2) {
        base.n0 = 0;
        base.n1 = N;
        su_worker(&base);
        return 0;
    }
    if (nthreads > N) nthreads = N;
    su_job_t *jobs = (su_job_t *)malloc(sizeof(su_job_t) * (size_t)nthreads);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return -2;
    }
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = base;
        jobs[t].n0 = (int64_t)N * t / nthreads;
        jobs[t].n1 = (int64_t)N * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, su_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(jobs);
    free(th);
    return 0;
}

/* ------------------------------------------- sensor update, sum reading */

/* Stored value read for point k under the particle constants (a, b): the
 * voxel's value as an exact double, or Q (tau) outside the map. */
static double point_value(const su_job_t *J, const float a[9], const float b[3], int64_t k) {
    const float *px = J->points, *py = J->points + J->K, *pz = J->points + 2 * J->K;
    const int64_t v = voxel_index(a, b, px[k], py[k], pz[k], &J->g);
    if (v < 0) return J->dtype >= ORACLE_F32 ? (double)(float)J->tau : (double)J->Q;
    switch (J->dtype) {
    case ORACLE_I16: return ((const int16_t *)J->values)[v];
    case ORACLE_I8: return ((const int8_t *)J->values)[v];
    case ORACLE_F32: return ((const float *)J->values)[v];
    default: return ((const double *)J->values)[v];
    }
}

static void *su_sum_worker(void *arg) {
    su_job_t *J = (su_job_t *)arg;
    for (int64_t n = J->n0; n < J->n1; ++n) {
        float a[9], b[3];
        particle_consts(J->poses, J->N, n, &J->g, a, b);
        double S = 0.0;
        for (int64_t k = 0; k < J->K; ++k) {
            const double d = point_value(J, a, b, k);
            S += exp(-J->c * (d * d));
        }
        if (J->ssum) J->ssum[n] = S;
        J->logw[n] = J->K == 0 ? 0.0 : log(S);
    }
    return NULL;
}

/*
 * l_n under the sum reading (see the header comment) on a dense map.  ssum
 * may be NULL; else it receives sum_k exp(-c q_k^2).  nthreads as for
 * oracle_sensor_update.
 */
int oracle_sensor_update_sum(const int32_t dims[3], float voxel, const float origin[3], float tau, int32_t dtype,
                             const void *values, const float *points, int32_t K, const float *poses, int32_t N,
                             float sigma, double *logw, double *ssum, int32_t nthreads) {
    if (K < 0 || N < 0 || dtype < 0 || dtype > 3 || !(sigma > 0.0f)) return -1;
    su_job_t base;
    memset(&base, 0, sizeof base);
    base.g = make_grid(dims, voxel, origin);
    base.dtype = dtype;
    base.values = values;
    base.tau = (double)tau;
    base.Q = dtype == ORACLE_I16 ? 32767 : dtype == ORACLE_I8 ? 127 : 1;
    base.points = points;
    base.K = K;
    base.poses = poses;
    base.N = N;
    const double sc = dtype >= ORACLE_F32 ? 1.0 : (double)tau / (double)base.Q, sg = (double)sigma;
    base.c = (sc * sc) / (2.0 * sg * sg);
    base.logw = logw;
    base.ssum = ssum;
    if (nthreads > N) nthreads = (int32_t)N;
    if (nthreads <= 1) {
        base.n0 = 0;
        base.n1 = N;
        su_sum_worker(&base);
        return 0;
    }
    su_job_t *jobs = (su_job_t *)malloc(sizeof(su_job_t) * (size_t)nthreads);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return -2;
    }
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = base;
        jobs[t].n0 = (int64_t)N * t / nthreads;
        jobs[t].n1 = (int64_t)N * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, su_sum_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(jobs);
    free(th);
    return 0;
}

/*
 * l_n for a sparse coarse/fine map given as a list of bricks (the definition is
 * the dense one; only the storage differs): nstored bricks, coords [nstored][3]
 * (bx, by, bz), values [nstored][64] (index x + 4 y + 16 z within the brick);
 * every voxel of an unlisted brick reads Q (tau).
 */
int oracle_sensor_update_bricks(const int32_t dims[3], float voxel, const float origin[3], float tau, int32_t dtype,
                                int64_t nstored, const int32_t *coords, const void *values, const float *points,
                                int32_t K, const float *poses, int32_t N, float sigma, double *logw, double *ssum,
                                int32_t nthreads) {
    if (K < 0 || N < 0 || dtype < 0 || dtype > 2 || !(sigma > 0.0f) || nstored < 0) return -1;
    const int64_t nbx = (dims[0] + 3) / 4, nby = (dims[1] + 3) / 4, nbz = (dims[2] + 3) / 4;
    int32_t *table = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nbx * nby * nbz));
    if (!table) return -2;
    for (int64_t b = 0; b < nbx * nby * nbz; ++b) table[b] = -1;
    for (int64_t s = 0; s < nstored; ++s) {
        int64_t bx = coords[3 * s], by = coords[3 * s + 1], bz = coords[3 * s + 2];
        if (bx < 0 || by < 0 || bz < 0 || bx >= nbx || by >= nby || bz >= nbz) {
            free(table);
            return -1;
        }
        table[bz + nbz * (bx + nbx * by)] = (int32_t)s;
    }
    su_job_t base;
    memset(&base, 0, sizeof base);
    base.g = make_grid(dims, voxel, origin);
    base.dtype = dtype;
    base.tau = (double)tau;
    base.Q = dtype == ORACLE_I16 ? 32767 : dtype == ORACLE_I8 ? 127 : 1;
    base.points = points;
    base.K = K;
    base.poses = poses;
    base.N = N;
    double s = dtype == ORACLE_F32 ? 1.0 : (double)tau / (double)base.Q;
    double sg = (double)sigma;
    base.c = (s * s) / (2.0 * sg * sg);
    base.logw = logw;
    base.ssum = ssum;
    base.table = table;
    base.bricks = values;
    base.nbx = nbx;
    base.nby = nby;
    base.nbz = nbz;
    int rc = 0;
    if (nthreads <= 1 || N < 2) {
        base.n0 = 0;
        base.n1 = N;
        su_worker(&base);
    } else {
        if (nthreads > N) nthreads = N;
        su_job_t *jobs = (su_job_t *)malloc(sizeof(su_job_t) * (size_t)nthreads);
        pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
        if (!jobs || !th) {
            rc = -2;
        } else {
            for (int t = 0; t < nthreads; ++t) {
                jobs[t] = base;
                jobs[t].n0 = (int64_t)N * t / nthreads;
                jobs[t].n1 = (int64_t)N * (t + 1) / nthreads;
                pthread_create(&th[t], NULL, su_worker, &jobs[t]);
            }
            for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
        }
        free(jobs);
        free(th);
    }
    free(table);
    return rc;
}

/* ------------------------------------------------------- trilinear lookup */

/* Stored value at voxel (i, j, k), or the out-of-map value. */
static double stored_value(const su_job_t *J, int64_t i, int64_t j, int64_t k) {
    const grid_t *g = &J->g;
    if (i < 0 || j < 0 || k < 0 || i >= g->n[0] || j >= g->n[1] || k >= g->n[2])
        return J->dtype >= ORACLE_F32 ? (double)(float)J->tau : (double)J->Q;
    int64_t v = i + (int64_t)g->n[0] * (j + (int64_t)g->n[1] * k);
    switch (J->dtype) {
    case ORACLE_I16: return ((const int16_t *)J->values)[v];
    case ORACLE_I8: return ((const int8_t *)J->values)[v];
    case ORACLE_F32: return ((const float *)J->values)[v];
    default: return ((const double *)J->values)[v];
    }
}

/* Interpolated map value of one point for particle constants a, b. */
static double trilinear_value(const su_job_t *J, const float a[9], const float b[3], float px, float py,
                              float pz) {
    int64_t i0[3];
    double f[3];
    for (int j = 0; j < 3; ++j) {
        float s = fmaf(a[3 * j + 0], px, b[j]);
        s = fmaf(a[3 * j + 1], py, s);
        s = fmaf(a[3 * j + 2], pz, s);
        float h = s - 0.5f;
        h = fminf(fmaxf(h, -2.0f), (float)J->g.n[j] + 1.0f);
        float fl = floorf(h);
        i0[j] = (int64_t)fl;
        f[j] = (double)(h - fl);
    }
    double m = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int bb = 0; bb < 2; ++bb)
            for (int aa = 0; aa < 2; ++aa) {
                double wgt = (aa ? f[0] : 1.0 - f[0]) * (bb ? f[1] : 1.0 - f[1]) * (c ? f[2] : 1.0 - f[2]);
                m += wgt * stored_value(J, i0[0] + aa, i0[1] + bb, i0[2] + c);
            }
    return m;
}

typedef struct {
    su_job_t base;
    double *sabs;
} tri_job_t;

static void *tri_worker(void *arg) {
    tri_job_t *T = (tri_job_t *)arg;
    const su_job_t *J = &T->base;
    const float *px = J->points, *py = J->points + J->K, *pz = J->points + 2 * J->K;
    for (int64_t n = J->n0; n < J->n1; ++n) {
        float a[9], b[3];
        particle_consts(J->poses, J->N, n, &J->g, a, b);
        double S = 0.0, A = 0.0;
        for (int64_t k = 0; k < J->K; ++k) {
            double m = trilinear_value(J, a, b, px[k], py[k], pz[k]);
            S += m * m;
            A += fabs(m);
        }
        if (J->ssum) J->ssum[n] = S;
        if (T->sabs) T->sabs[n] = A;
        J->logw[n] = -(S * J->c);
    }
    return NULL;
}

/*
 * l_n with the trilinear lookup (see the header comment).  ssum / sabs may be
 * NULL; else they receive sum m^2 and sum |m| per particle (stored units).
 */
int oracle_sensor_update_trilinear(const int32_t dims[3], float voxel, const float origin[3], float tau,
                                   int32_t dtype, const void *values, const float *points, int32_t K,
                                   const float *poses, int32_t N, float sigma, double *logw, double *ssum,
                                   double *sabs, int32_t nthreads) {
    if (K < 0 || N < 0 || dtype < 0 || dtype > 3 || !(sigma > 0.0f)) return -1;
    tri_job_t base;
    memset(&base, 0, sizeof base);
    su_job_t *B = &base.base;
    B->g = make_grid(dims, voxel, origin);
    B->dtype = dtype;
    B->values = values;
    B->tau = (double)tau;
    B->Q = dtype == ORACLE_I16 ? 32767 : dtype == ORACLE_I8 ? 127 : 1;
    B->points = points;
    B->K = K;
    B->poses = poses;
    B->N = N;
    double s = dtype >= ORACLE_F32 ? 1.0 : (double)tau / (double)B->Q;
    double sg = (double)sigma;
    B->c = (s * s) / (2.0 * sg * sg);
    B->logw = logw;
    B->ssum = ssum;
    base.sabs = sabs;
    if (nthreads <= 1 || N < 2) {
        B->n0 = 0;
        B->n1 = N;
        tri_worker(&base);
        return 0;
    }
    if (nthreads > N) nthreads = N;
    tri_job_t *jobs = (tri_job_t *)malloc(sizeof(tri_job_t) * (size_t)nthreads);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return -2;
    }
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = base;
        jobs[t].base.n0 = (int64_t)N * t / nthreads;
        jobs[t].base.n1 = (int64_t)N * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, tri_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(jobs);
    free(th);
    return 0;
}

/* ------------------------------------------------------------ normalisation */

int oracle_normalize(const double *logw, int32_t N, double *w, uint64_t *wq, double *log_z) {
    if (N < 1) return -1;
    double m = logw[0];
    for (int32_t n = 1; n < N; ++n)
        if (logw[n] > m) m = logw[n];
    double S = 0.0, comp = 0.0;
    for (int32_t n = 0; n < N; ++n) {
        const double t = exp(logw[n] - m);
        const double y = S + t;
        comp += fabs(S) >= fabs(t) ? (S - y) + t : (t - y) + S;  /* the rounding error of S + t, exactly */
        S = y;
    }
    S += comp;
    double lz = m + log(S);
    for (int32_t n = 0; n < N; ++n) {
        double wn = exp(logw[n] - lz);
        if (w) w[n] = wn;
        if (wq) wq[n] = (uint64_t)floor(ldexp(wn, 42));
    }
    if (log_z) *log_z = lz;
    return 0;
}

/* -------------------------------------------------------------- resampling */

/* SplitMix64 output from state x (see the header): advance, then mix. */
uint64_t oracle_splitmix64(uint64_t x) {
    uint64_t z = x + UINT64_C(0x9E3779B97F4A7C15);
    z = (z ^ (z >> 30)) * UINT64_C(0xBF58476D1CE4E5B9);
    z = (z ^ (z >> 27)) * UINT64_C(0x94D049BB133111EB);
    return z ^ (z >> 31);
}

/* The resampling draw of update `tick` of a filter seeded with `seed`. */
uint64_t oracle_resample_draw(uint64_t seed, uint64_t tick) {
    return oracle_splitmix64(seed ^ oracle_splitmix64(tick));
}

int oracle_resample(const uint64_t *wq, int32_t N, uint64_t u, int32_t *idx) {
    if (N < 1) return -1;
    uint64_t T = 0;
    for (int32_t i = 0; i < N; ++i) T += wq[i];
    if (T == 0) {
        for (int32_t m = 0; m < N; ++m) idx[m] = m;
        return 0;
    }
    uint64_t r = (uint64_t)(((unsigned __int128)u * T) >> 64);
    /* Sweep the slots in order; the threshold for slot m is m T + r, and the
       particle cursor advances past every particle whose scaled cumulative
       weight N C_i does not exceed the threshold. */
    int32_t i = 0;
    uint64_t C = wq[0];
    for (int32_t m = 0; m < N; ++m) {
        uint64_t x = (uint64_t)m * T + r;
        while (x >= (uint64_t)N * C) {
            ++i;
            C += wq[i];
        }
        idx[m] = i;
    }
    return 0;
}

/*
 * CPU oracle for the motion update and the uniform initialisation of the
 * particle set (Eisoldt et al., arXiv 2310.04172, §III: particles start
 * uniformly in free space when no initial estimate exists, and each iteration
 * first applies the motion model to every particle; §VI: odometry from dead
 * reckoning or an IMU, with noise on the velocity and angular velocity).
 *
 * TEST INFRASTRUCTURE ONLY (see mcl_oracle.c).  Shares no code with the HIP
 * library.  Float64 except where a float32 step is part of a definition below.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC 2011): a 128-bit counter and a 64-bit key
 * give four 32-bit words; ten rounds, each multiplying two counter words by the
 * constants 0xD2511F53 and 0xCD9E8D57 (full 64-bit products), mixing the high
 * halves with the other two words and the key, the key advanced by the Weyl
 * constants 0x9E3779B9 and 0xBB67AE85 between rounds.
 *   Counter of particle n: (n, lo32(step), hi32(step), c), key (lo32(seed),
 *   hi32(seed)); the motion update uses c = 0, 1, the initialisation c = 2, 3
 *   with step = 0: 8 words per particle, w0..w3 from the first call.
 *
 * Readings (the paper gives no formulas for either step):
 *
 *  Uniform in (0, 1] and [0, 1) from a word x: ((x >> 8) + 1) 2^-24 and
 *  (x >> 8) 2^-24.  Standard normals by Box-Muller: for words (x, y),
 *  r = sqrt(-2 ln u1), u1 from x in (0, 1]; a = 2 pi u2, u2 from y in [0, 1);
 *  the pair r cos a, r sin a.  Words (w0, w1), (w2, w3), (w4, w5) give the six
 *  normals n0..n5.
 *
 *  Motion update: the odometry increment is a rigid motion (dR, dt) in the
 *  robot frame (R|t, 12 numbers like a pose); each particle gets its own noisy
 *  copy, translation noise xi_t = sigma_t (n0, n1, n2) and rotation noise
 *  xi_r = sigma_r (n3, n4, n5) (a rotation vector):
 *      dt' = dt + xi_t,   dR' = dR Exp(xi_r),
 *      R_new = R dR',     t_new = R dt' + t,
 *  Exp by Rodrigues' formula.  sigma_t, sigma_r are the standard deviations of
 *  the increment (velocity noise times the time step).
 *
 *  Uniform initialisation in free space: free voxels are those with a stored
 *  value > 0, counted in the x-fastest order of the map (index i + nx (j + ny
 *  k)); particle n takes the free voxel of rank floor(U F / 2^64), F the number
 *  of free voxels, U = w0 + 2^32 w1; its position is, per axis in float32 with
 *  each operation rounded,
 *      p = o + ((float) i + u) * v,   u from w2, w3, w4 in [0, 1),
 *  and its orientation R = Rz(yaw) Ry(pitch) Rx(roll) with yaw = pi (2 u5 - 1),
 *  pitch = a (2 u6 - 1), roll = a (2 u7 - 1), u5..u7 from w5..w7 in [0, 1), a
 *  the largest tilt.
 */

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const double PI = 3.14159265358979323846;

/* Philox4x32-10 of counter c and key k into out. */
void oracle_philox4x32(const uint32_t c[4], const uint32_t k[2], uint32_t out[4]) {
    uint32_t x0 = c[0], x1 = c[1], x2 = c[2], x3 = c[3];
    uint32_t k0 = k[0], k1 = k[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* The 8 words of particle n for the given step and seed, calls c0, c0 + 1. */
static void particle_words(uint64_t seed, uint64_t step, uint32_t n, uint32_t c0, uint32_t w[8]) {
    uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t h = 0; h < 2; ++h) {
        uint32_t c[4] = {n, (uint32_t)step, (uint32_t)(step >> 32), c0 + h};
        oracle_philox4x32(c, k, w + 4 * h);
    }
}

static double unit_open(uint32_t x) { return ((double)(x >> 8) + 1.0) * (1.0 / 16777216.0); }
static double unit_closed(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* Rotation matrix (row-major) of a rotation vector, Rodrigues' formula. */
static void rodrigues(const double v[3], double R[9]) {
    double th = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double a, b; /* sin(th)/th, (1 - cos(th))/th^2 */
    if (th < 1e-8) {
        a = 1.0 - th * th / 6.0;
        b = 0.5 - th * th / 24.0;
    } else {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / (th * th);
    }
    double K[9] = {0, -v[2], v[1], v[2], 0, -v[0], -v[1], v[0], 0};
    double K2[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int m = 0; m < 3; ++m) s += K[3 * r + m] * K[3 * m + c];
            K2[3 * r + c] = s;
        }
    for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0 ? 1.0 : 0.0) + a * K[i] + b * K2[i];
}

/* Six standard normals from words w0..w5. */
static void normals6(const uint32_t w[8], double nrm[6]) {
    for (int p = 0; p < 3; ++p) {
        double r = sqrt(-2.0 * log(unit_open(w[2 * p])));
        double a = 2.0 * PI * unit_closed(w[2 * p + 1]);
        nrm[2 * p] = r * cos(a);
        nrm[2 * p + 1] = r * sin(a);
    }
}

/*
 * Motion update (see the header).  poses_in / poses_out: [12][N] float32
 * (may be the same array); delta: 12 float32 (dR row-major, dt); out_normals:
 * NULL or [6][N] float64, the normals drawn.  Result in float64 (poses_out64,
 * [12][N]) so that tests can compare with their own tolerance.
 */
int oracle_motion_update(const float *poses_in, double *poses_out64, int32_t N, const float delta[12],
                         float sigma_t, float sigma_r, uint64_t seed, uint64_t step, double *out_normals) {
    if (N < 0) return -1;
    for (int32_t n = 0; n < N; ++n) {
        uint32_t w[8];
        particle_words(seed, step, (uint32_t)n, 0, w);
        double nr[6];
        normals6(w, nr);
        if (out_normals)
            for (int q = 0; q < 6; ++q) out_normals[(int64_t)q * N + n] = nr[q];
        double xr[3] = {sigma_r * nr[3], sigma_r * nr[4], sigma_r * nr[5]};
        double E[9];
        rodrigues(xr, E);
        double dR[9], dRn[9], R[9], t[3], dtn[3];
        for (int i = 0; i < 9; ++i) dR[i] = delta[i];
        for (int j = 0; j < 3; ++j) dtn[j] = (double)delta[9 + j] + (double)sigma_t * nr[j];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int m = 0; m < 3; ++m) s += dR[3 * r + m] * E[3 * m + c];
                dRn[3 * r + c] = s;
            }
        for (int i = 0; i < 9; ++i) R[i] = poses_in[(int64_t)i * N + n];
        for (int j = 0; j < 3; ++j) t[j] = poses_in[(int64_t)(9 + j) * N + n];
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int m = 0; m < 3; ++m) s += R[3 * r + m] * dRn[3 * m + c];
                poses_out64[(int64_t)(3 * r + c) * N + n] = s;
            }
            double s = t[r];
            for (int m = 0; m < 3; ++m) s += R[3 * r + m] * dtn[m];
            poses_out64[(int64_t)(9 + r) * N + n] = s;
        }
    }
    return 0;
}

/*
 * Uniform initialisation in free space (see the header).  values: the dense
 * map (x fastest) of the storage type dtype (0 int16, 1 int8, 2 float32).
 * poses_out64: [12][N] float64 (positions are float32 values); voxel_out:
 * NULL or [N] int64 linear indices of the chosen voxels.  Returns -3 if the
 * map has no free voxel.
 */
int oracle_init_uniform(const int32_t dims[3], float voxel, const float origin[3], int32_t dtype,
                        const void *values, int32_t N, float max_tilt, uint64_t seed, double *poses_out64,
                        int64_t *voxel_out) {
    int64_t nvox = (int64_t)dims[0] * dims[1] * dims[2];
    int64_t F = 0;
    for (int64_t v = 0; v < nvox; ++v) {
        int free_ = dtype == 0 ? ((const int16_t *)values)[v] > 0
                    : dtype == 1 ? ((const int8_t *)values)[v] > 0
                                 : ((const float *)values)[v] > 0.0f;
        F += free_;
    }
    if (F == 0) return -3;
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)F);
    if (!list) return -2;
    int64_t f = 0;
    for (int64_t v = 0; v < nvox; ++v) {
        int free_ = dtype == 0 ? ((const int16_t *)values)[v] > 0
                    : dtype == 1 ? ((const int8_t *)values)[v] > 0
                                 : ((const float *)values)[v] > 0.0f;
        if (free_) list[f++] = v;
    }
    for (int32_t n = 0; n < N; ++n) {
        uint32_t w[8];
        particle_words(seed, 0, (uint32_t)n, 2, w);
        uint64_t U = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
        /* floor(U F / 2^64) with a 128-bit product */
        unsigned __int128 prod = (unsigned __int128)U * (unsigned __int128)(uint64_t)F;
        int64_t rank = (int64_t)(prod >> 64);
        int64_t v = list[rank];
        if (voxel_out) voxel_out[n] = v;
        int64_t ijk[3] = {v % dims[0], (v / dims[0]) % dims[1], v / ((int64_t)dims[0] * dims[1])};
        for (int j = 0; j < 3; ++j) {
            float u = (float)(w[2 + j] >> 8) * (1.0f / 16777216.0f);
            float s = (float)ijk[j] + u;
            s = s * voxel;
            s = origin[j] + s;
            poses_out64[(int64_t)(9 + j) * N + n] = (double)s;
        }
        double yaw = PI * (2.0 * unit_closed(w[5]) - 1.0);
        double pitch = (double)max_tilt * (2.0 * unit_closed(w[6]) - 1.0);
        double roll = (double)max_tilt * (2.0 * unit_closed(w[7]) - 1.0);
        double cy = cos(yaw), sy = sin(yaw), cp = cos(pitch), sp = sin(pitch), cr = cos(roll), sr = sin(roll);
        double R[9] = {cy * cp, cy * sp * sr - sy * cr, cy * sp * cr + sy * sr,
                       sy * cp, sy * sp * sr + cy * cr, sy * sp * cr - cy * sr,
                       -sp, cp * sr, cp * cr};
        for (int i = 0; i < 9; ++i) poses_out64[(int64_t)i * N + n] = R[i];
    }
    free(list);
    return 0;
}

// Motion update and uniform initialisation of the particle set, on the device
// (§III: without an initial estimate the particles start uniformly in free
// space; every iteration first moves each particle by the motion model, here
// the odometry increment with noise on its translation and rotation, §VI).
// One thread per particle; random numbers from Philox (rng.h), so every
// particle's draw is fixed by (seed, step, particle index).
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "jobs.h"
#include "rng.h"
#include "voxel.h"

namespace mcl {

constexpr float kPi = 3.14159265358979323846f;

// Box-Muller: the pair r cos a, r sin a for r = sqrt(-2 ln u1), a = 2 pi u2.
__device__ inline void box_muller(uint32_t x, uint32_t y, float &n0, float &n1) {
    const float r = sqrtf(-2.0f * logf(unit_open(x)));
    float s, c;
    sincosf(2.0f * kPi * unit_closed(y), &s, &c);
    n0 = r * c;
    n1 = r * s;
}

// Rotation matrix of a rotation vector (Rodrigues), float32.  For small angles
// the series of sin(t)/t and (1 - cos t)/t^2 = 2 sin^2(t/2)/t^2.
__device__ inline void exp_so3(float vx, float vy, float vz, float (&E)[9]) {
    const float t2 = vx * vx + vy * vy + vz * vz;
    float a, b;
    if (t2 < 1e-8f) {
        a = 1.0f - t2 * (1.0f / 6.0f);
        b = 0.5f - t2 * (1.0f / 24.0f);
    } else {
        const float t = sqrtf(t2);
        const float h = sinf(0.5f * t) / t;
        a = sinf(t) / t;
        b = 2.0f * h * h;
    }
    // I + a K + b K^2, K = [v]x, K^2 = v v^T - t2 I
    E[0] = 1.0f + b * (vx * vx - t2);
    E[1] = -a * vz + b * vx * vy;
    E[2] = a * vy + b * vx * vz;
    E[3] = a * vz + b * vx * vy;
    E[4] = 1.0f + b * (vy * vy - t2);
    E[5] = -a * vx + b * vy * vz;
    E[6] = -a * vy + b * vx * vz;
    E[7] = a * vx + b * vy * vz;
    E[8] = 1.0f + b * (vz * vz - t2);
}

struct Delta {
    float m[12];  // dR row-major, dt
};

// pin and pout may be the same array (each thread reads its particle before
// writing it), so neither is declared restrict.  kMean: every particle starts
// from the same pose `mean` (pin unused) - the initialisation round a pose
// estimate, which is the motion update of N copies of the estimate.
template <bool kMean>
__global__ __launch_bounds__(256) void motion_kernel(const float *pin, float *pout, int N, Delta d, Delta mean,
                                                     float sigma_t, float sigma_r, uint64_t seed, uint64_t step) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    uint32_t w[8];
    particle_words(seed, step, (uint32_t)n, 0u, w);
    float nr[6];
    box_muller(w[0], w[1], nr[0], nr[1]);
    box_muller(w[2], w[3], nr[2], nr[3]);
    box_muller(w[4], w[5], nr[4], nr[5]);
    float E[9];
    exp_so3(sigma_r * nr[3], sigma_r * nr[4], sigma_r * nr[5], E);
    float dR[9], dt[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            dR[3 * r + c] = d.m[3 * r] * E[c] + d.m[3 * r + 1] * E[3 + c] + d.m[3 * r + 2] * E[6 + c];
        dt[r] = d.m[9 + r] + sigma_t * nr[r];
    }
    float P[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) P[j] = kMean ? mean.m[j] : pin[(size_t)j * N + n];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            pout[(size_t)(3 * r + c) * N + n] = P[3 * r] * dR[c] + P[3 * r + 1] * dR[3 + c] + P[3 * r + 2] * dR[6 + c];
        pout[(size_t)(9 + r) * N + n] = P[9 + r] + (P[3 * r] * dt[0] + P[3 * r + 1] * dt[1] + P[3 * r + 2] * dt[2]);
    }
}

// ---------------------------------------------------------------- initialisation
// Free voxels (stored value > 0) in x-fastest order, counted per chunk of 64
// consecutive x of one row; prefix[c] = free voxels before chunk c.
constexpr int kChunkX = 64;

template <typename T>
__device__ inline bool voxel_free(const MapView &m, int x, int y, int z) {
    const T v = *reinterpret_cast<const T *>(m.base + brick_offset<sizeof(T)>(m, (uint32_t)x, (uint32_t)y, (uint32_t)z));
    return v > T(0);
}

template <typename T>
__global__ __launch_bounds__(256) void free_count_kernel(MapView m, int qx, int64_t nchunks, uint8_t *__restrict__ cnt) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nchunks) return;
    const int q = (int)(c % qx);
    const int64_t row = c / qx;
    const int y = (int)(row % m.ny), z = (int)(row / m.ny);
    const int x1 = min(m.nx, (q + 1) * kChunkX);
    int k = 0;
    for (int x = q * kChunkX; x < x1; ++x) k += voxel_free<T>(m, x, y, z);
    cnt[c] = (uint8_t)k;
}

template <typename T>
__global__ __launch_bounds__(256) void init_kernel(MapView m, float voxel, const uint64_t *__restrict__ prefix,
                                                   int64_t nchunks, int qx, uint64_t nfree, float *__restrict__ poses,
                                                   int N, float tilt, uint64_t seed) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    uint32_t w[8];
    particle_words(seed, 0, (uint32_t)n, 2u, w);
    const uint64_t U = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
    const uint64_t rank = __umul64hi(U, nfree);  // floor(U F / 2^64) < F
    // last chunk whose prefix <= rank (prefix[0] = 0, prefix[nchunks] = F > rank)
    int64_t lo = 0, hi = nchunks - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= rank) lo = mid;
        else hi = mid - 1;
    }
    uint64_t left = rank - prefix[lo];  // rank within the chunk
    const int q = (int)(lo % qx);
    const int64_t row = lo / qx;
    const int y = (int)(row % m.ny), z = (int)(row / m.ny);
    const int x1 = min(m.nx, (q + 1) * kChunkX);
    int x = q * kChunkX;
    for (; x < x1; ++x) {
        if (voxel_free<T>(m, x, y, z)) {
            if (left == 0) break;
            --left;
        }
    }
    // the chunk holds more than `left` free voxels, so x < x1 here
    const int ijk[3] = {x, y, z};
    const float org[3] = {m.ox, m.oy, m.oz};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        float s = (float)ijk[j] + unit_closed(w[2 + j]);
        s = s * voxel;
        poses[(size_t)(9 + j) * N + n] = org[j] + s;
    }
    const float yaw = kPi * (2.0f * unit_closed(w[5]) - 1.0f);
    const float pitch = tilt * (2.0f * unit_closed(w[6]) - 1.0f);
    const float roll = tilt * (2.0f * unit_closed(w[7]) - 1.0f);
    float sy, cy, sp, cp, sr, cr;
    sincosf(yaw, &sy, &cy);
    sincosf(pitch, &sp, &cp);
    sincosf(roll, &sr, &cr);
    const float R[9] = {cy * cp, cy * sp * sr - sy * cr, cy * sp * cr + sy * sr,
                        sy * cp, sy * sp * sr + cy * cr, sy * sp * cr - cy * sr,
                        -sp,     cp * sr,                cp * cr};
#pragma unroll
    for (int i = 0; i < 9; ++i) poses[(size_t)i * N + n] = R[i];
}

// Free-voxel prefix of a map, built on first use (synchronous).
struct FreeIndex {
    uint64_t *prefix = nullptr;  // device [nchunks + 1]
    int64_t nchunks = 0;
    int qx = 0;
    uint64_t nfree = 0;
};

static std::mutex g_free_mu;

static mcl_status ensure_free_index(mcl_map_s *m, hipStream_t stream, FreeIndex &out) {
    std::lock_guard<std::mutex> lk(g_free_mu);
    if (m->free_prefix) {
        out.prefix = static_cast<uint64_t *>(m->free_prefix);
        out.qx = (m->view.nx + kChunkX - 1) / kChunkX;
        out.nchunks = (int64_t)out.qx * m->view.ny * m->view.nz;
        out.nfree = m->free_total;
        return MCL_OK;
    }
    const MapView &v = m->view;
    const int qx = (v.nx + kChunkX - 1) / kChunkX;
    const int64_t nchunks = (int64_t)qx * v.ny * v.nz;
    uint8_t *cnt = nullptr;
    uint64_t *prefix = nullptr;
    if (hipMalloc(&cnt, (size_t)nchunks) != hipSuccess) return fail(MCL_ENOMEM, "init_uniform: allocation failed");
    if (hipMalloc(&prefix, (size_t)(nchunks + 1) * 8) != hipSuccess) {
        (void)hipFree(cnt);
        return fail(MCL_ENOMEM, "init_uniform: allocation failed");
    }
    const unsigned blocks = (unsigned)((nchunks + 255) / 256);
    if (m->dtype == MCL_TSDF_I16) free_count_kernel<int16_t><<<blocks, 256, 0, stream>>>(v, qx, nchunks, cnt);
    else if (m->dtype == MCL_TSDF_I8) free_count_kernel<int8_t><<<blocks, 256, 0, stream>>>(v, qx, nchunks, cnt);
    else free_count_kernel<float><<<blocks, 256, 0, stream>>>(v, qx, nchunks, cnt);
    mcl_status st = check_launch("free_count_kernel");
    std::vector<uint8_t> hc;
    std::vector<uint64_t> hp;
    if (st == MCL_OK) {
        hc.resize((size_t)nchunks);
        if (hipMemcpyAsync(hc.data(), cnt, (size_t)nchunks, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            st = fail(MCL_EDEVICE, "init_uniform: count copy failed");
    }
    if (st == MCL_OK) {
        hp.resize((size_t)nchunks + 1);
        uint64_t acc = 0;
        for (int64_t c = 0; c < nchunks; ++c) {
            hp[(size_t)c] = acc;
            acc += hc[(size_t)c];
        }
        hp[(size_t)nchunks] = acc;
        if (hipMemcpyAsync(prefix, hp.data(), hp.size() * 8, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            st = fail(MCL_EDEVICE, "init_uniform: prefix copy failed");
    }
    (void)hipFree(cnt);
    if (st != MCL_OK) {
        (void)hipFree(prefix);
        return st;
    }
    m->free_prefix = prefix;
    m->free_total = hp[(size_t)nchunks];
    out.prefix = prefix;
    out.qx = qx;
    out.nchunks = nchunks;
    out.nfree = m->free_total;
    return MCL_OK;
}

__global__ void philox_kernel(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                              uint32_t *out) {
    const Words4 r = philox4x32_10(c0, c1, c2, c3, k0, k1);
    if (threadIdx.x < 4) out[threadIdx.x] = r.w[threadIdx.x];
}

}  // namespace mcl

using namespace mcl;

extern "C" mcl_status mcl_debug_philox(const uint32_t *counter_key, uint32_t *out) {
    if (!counter_key || !out) return fail(MCL_EINVAL, "debug_philox: NULL argument");
    uint32_t *dev = static_cast<uint32_t *>(workspace(nullptr, 16));
    if (!dev) return fail(MCL_ENOMEM, "debug_philox: workspace allocation failed");
    philox_kernel<<<1, 64>>>(counter_key[0], counter_key[1], counter_key[2], counter_key[3], counter_key[4],
                             counter_key[5], dev);
    mcl_status st = check_launch("philox_kernel");
    if (st != MCL_OK) return st;
    if (hipMemcpy(out, dev, 16, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(MCL_EDEVICE, "debug_philox: copy failed");
    return MCL_OK;
}

extern "C" mcl_status mcl_motion_update(const float *poses_in, float *poses_out, int32_t N, const float *delta,
                                        float sigma_t, float sigma_r, uint64_t seed, uint64_t step, void *stream) {
    if (!poses_in || !poses_out || !delta) return fail(MCL_EINVAL, "motion_update: NULL poses or delta");
    if (N < 1) return fail(MCL_EINVAL, "motion_update: need N >= 1");
    if (N > MCL_MAX_PARTICLES) return fail(MCL_ERANGE, "motion_update: N above the limit");
    if (!(std::isfinite(sigma_t) && sigma_t >= 0.0f && std::isfinite(sigma_r) && sigma_r >= 0.0f))
        return fail(MCL_EINVAL, "motion_update: noise deviations must be finite and >= 0");
    const size_t pb = (size_t)12 * N * 4;
    const auto a = reinterpret_cast<uintptr_t>(poses_in), b = reinterpret_cast<uintptr_t>(poses_out);
    if (a != b && a < b + pb && b < a + pb) return fail(MCL_EINVAL, "motion_update: poses_out partly overlaps poses_in");
    Delta d, none{};
    for (int i = 0; i < 12; ++i) {
        if (!std::isfinite(delta[i])) return fail(MCL_EINVAL, "motion_update: delta must be finite");
        d.m[i] = delta[i];
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    motion_kernel<false><<<(N + 255) / 256, 256, 0, s>>>(poses_in, poses_out, N, d, none, sigma_t, sigma_r, seed, step);
    return check_launch("motion_kernel");
}

extern "C" mcl_status mcl_init_gaussian(float *poses, int32_t N, const float *mean, float sigma_t, float sigma_r,
                                        uint64_t seed, uint64_t step, void *stream) {
    if (!poses || !mean) return fail(MCL_EINVAL, "init_gaussian: NULL poses or mean");
    if (N < 1) return fail(MCL_EINVAL, "init_gaussian: need N >= 1");
    if (N > MCL_MAX_PARTICLES) return fail(MCL_ERANGE, "init_gaussian: N above the limit");
    if (!(std::isfinite(sigma_t) && sigma_t >= 0.0f && std::isfinite(sigma_r) && sigma_r >= 0.0f))
        return fail(MCL_EINVAL, "init_gaussian: deviations must be finite and >= 0");
    Delta id{}, m;
    id.m[0] = id.m[4] = id.m[8] = 1.0f;
    for (int i = 0; i < 12; ++i) {
        if (!std::isfinite(mean[i])) return fail(MCL_EINVAL, "init_gaussian: mean must be finite");
        m.m[i] = mean[i];
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    motion_kernel<true><<<(N + 255) / 256, 256, 0, s>>>(nullptr, poses, N, id, m, sigma_t, sigma_r, seed, step);
    return check_launch("motion_kernel (initialisation round a pose)");
}

extern "C" mcl_status mcl_init_uniform(mcl_map map, float *poses, int32_t N, float max_tilt, uint64_t seed,
                                       void *stream) {
    if (!map || !poses) return fail(MCL_EINVAL, "init_uniform: NULL map or poses");
    if (N < 1) return fail(MCL_EINVAL, "init_uniform: need N >= 1");
    if (N > MCL_MAX_PARTICLES) return fail(MCL_ERANGE, "init_uniform: N above the limit");
    if (!(std::isfinite(max_tilt) && max_tilt >= 0.0f)) return fail(MCL_EINVAL, "init_uniform: max_tilt must be >= 0");
    if (map->sparse) return fail(MCL_EINVAL, "init_uniform: not available for sparse maps (mcl_map_upload_bricks)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    FreeIndex fi;
    mcl_status st = ensure_free_index(map, s, fi);
    if (st != MCL_OK) return st;
    if (fi.nfree == 0) return fail(MCL_EINVAL, "init_uniform: the map has no free voxel (stored value > 0)");
    const MapView &v = map->view;
    const unsigned blocks = (unsigned)((N + 255) / 256);
    if (map->dtype == MCL_TSDF_I16)
        init_kernel<int16_t><<<blocks, 256, 0, s>>>(v, map->voxel, fi.prefix, fi.nchunks, fi.qx, fi.nfree, poses, N, max_tilt, seed);
    else if (map->dtype == MCL_TSDF_I8)
        init_kernel<int8_t><<<blocks, 256, 0, s>>>(v, map->voxel, fi.prefix, fi.nchunks, fi.qx, fi.nfree, poses, N, max_tilt, seed);
    else
        init_kernel<float><<<blocks, 256, 0, s>>>(v, map->voxel, fi.prefix, fi.nchunks, fi.qx, fi.nfree, poses, N, max_tilt, seed);
    st = check_launch("init_kernel");
    return st == MCL_OK ? note_map_use(map, s) : st;
}

// C-ABI entry points: argument checks, error reporting, per-stream workspace.
#include <cmath>
#include <mutex>
#include <unordered_map>
#include <utility>

#include "jobs.h"

namespace mcl {

mcl_status launch_sensor(const mcl_map_s *, const float *, int, const float *, int, float, float *, hipStream_t,
                         float *);
mcl_status launch_sensor_trilinear(mcl_map_s *, const float *, int, const float *, int, float, float *,
                                   hipStream_t);
mcl_status launch_sensor_sum(const mcl_map_s *, const float *, int, const float *, int, float, float *, hipStream_t);
mcl_status launch_debug_indices(const mcl_map_s *, const float *, int, const float *, int, int64_t *, hipStream_t);
mcl_status launch_normalize(const float *, int, double *, uint64_t *, double *, hipStream_t);
mcl_status launch_resample(const uint64_t *, int, uint64_t, int32_t *, const float *, float *, hipStream_t);
mcl_status launch_estimate(const double *, const float *, int, double *, int32_t *, float *, hipStream_t);

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

mcl_status fail(mcl_status code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

mcl_status check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) return MCL_OK;
    return fail(MCL_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {
struct WsKey {
    int device;
    hipStream_t stream;
    bool operator==(const WsKey &o) const { return device == o.device && stream == o.stream; }
};
struct WsHash {
    size_t operator()(const WsKey &k) const { return std::hash<void *>()(k.stream) ^ (size_t)k.device * 0x9e3779b97f4a7c15ull; }
};
std::mutex g_ws_mu;
std::unordered_map<WsKey, std::pair<void *, size_t>, WsHash> g_ws;
}  // namespace

void *workspace(hipStream_t stream, size_t bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto &slot = g_ws[WsKey{dev, stream}];
    if (slot.second >= bytes && slot.first) return slot.first;
    if (slot.first) {
        // work already enqueued on this stream may still read the old buffer
        if (hipStreamSynchronize(stream) != hipSuccess) return nullptr;
        (void)hipFree(slot.first);
        slot = {nullptr, 0};
    }
    size_t want = bytes < ((size_t)1 << 20) ? ((size_t)1 << 20) : bytes + bytes / 4;
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) return nullptr;
    slot = {p, want};
    return p;
}

static bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    if (!a || !b) return false;
    auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

}  // namespace mcl

using namespace mcl;

extern "C" const char *mcl_last_error(void) { return g_last_error.c_str(); }

mcl_status sensor_args(const char *what, mcl_map map, const float *points, int32_t K, const float *poses,
                              int32_t N, float sigma, float *logw, float *c) {
    const std::string w(what);
    if (!map) return fail(MCL_EINVAL, w + ": NULL map");
    if (!poses || !logw) return fail(MCL_EINVAL, w + ": NULL poses or logw");
    if (K < 0 || N < 1) return fail(MCL_EINVAL, w + ": need K >= 0 and N >= 1");
    if (K > MCL_MAX_POINTS || N > MCL_MAX_PARTICLES) return fail(MCL_ERANGE, w + ": K or N above the limit");
    if (K > 0 && !points) return fail(MCL_EINVAL, w + ": NULL points with K > 0");
    if (!(std::isfinite(sigma) && sigma > 0.0f)) return fail(MCL_EINVAL, w + ": sigma must be finite and > 0");
    if (overlaps(logw, (size_t)N * 4, poses, (size_t)12 * N * 4) || overlaps(logw, (size_t)N * 4, points, (size_t)3 * K * 4))
        return fail(MCL_EINVAL, w + ": logw overlaps an input");
    const double s = map->scale, sg = (double)sigma;
    *c = (float)((s * s) / (2.0 * sg * sg));
    return MCL_OK;
}

extern "C" mcl_status mcl_sensor_update(mcl_map map, const float *points, int32_t K, const float *poses, int32_t N,
                                        float sigma, float *logw, void *stream) {
    float c = 0.0f;
    mcl_status st = sensor_args("sensor_update", map, points, K, poses, N, sigma, logw, &c);
    if (st != MCL_OK) return st;
    st = launch_sensor(map, points, K, poses, N, c, logw, static_cast<hipStream_t>(stream), nullptr);
    return st == MCL_OK ? note_map_use(map, static_cast<hipStream_t>(stream)) : st;
}

extern "C" mcl_status mcl_sensor_update_trilinear(mcl_map map, const float *points, int32_t K, const float *poses,
                                                  int32_t N, float sigma, float *logw, void *stream) {
    float c = 0.0f;
    mcl_status st = sensor_args("sensor_update_trilinear", map, points, K, poses, N, sigma, logw, &c);
    if (st != MCL_OK) return st;
    st = launch_sensor_trilinear(map, points, K, poses, N, c, logw, static_cast<hipStream_t>(stream));
    return st == MCL_OK ? note_map_use(map, static_cast<hipStream_t>(stream)) : st;
}

extern "C" mcl_status mcl_sensor_update_sum(mcl_map map, const float *points, int32_t K, const float *poses,
                                            int32_t N, float sigma, float *logw, void *stream) {
    float c = 0.0f;
    mcl_status st = sensor_args("sensor_update_sum", map, points, K, poses, N, sigma, logw, &c);
    if (st != MCL_OK) return st;
    if (map->sparse) return fail(MCL_EINVAL, "sensor_update_sum: the sum reading needs a dense map");
    if (!sum_sigma_ok(map, sigma)) return fail(MCL_EINVAL, "sensor_update_sum: the sum reading needs sigma >= tau / 8");
    st = launch_sensor_sum(map, points, K, poses, N, sum_k2(map, sigma), logw, static_cast<hipStream_t>(stream));
    return st == MCL_OK ? note_map_use(map, static_cast<hipStream_t>(stream)) : st;
}

extern "C" mcl_status mcl_normalize(const float *logw, int32_t N, double *w, uint64_t *wq, double *log_z,
                                    void *stream) {
    if (!logw || !wq) return fail(MCL_EINVAL, "normalize: NULL logw or wq");
    if (N < 1) return fail(MCL_EINVAL, "normalize: need N >= 1");
    if (N > MCL_MAX_PARTICLES) return fail(MCL_ERANGE, "normalize: N above the limit");
    if (overlaps(wq, (size_t)N * 8, logw, (size_t)N * 4) || overlaps(w, (size_t)N * 8, logw, (size_t)N * 4) ||
        overlaps(w, (size_t)N * 8, wq, (size_t)N * 8))
        return fail(MCL_EINVAL, "normalize: overlapping buffers");
    return launch_normalize(logw, N, w, wq, log_z, static_cast<hipStream_t>(stream));
}

extern "C" mcl_status mcl_resample(const uint64_t *wq, int32_t N, uint64_t seed, uint64_t tick, int32_t *idx,
                                   const float *poses_in, float *poses_out, void *stream) {
    if (!wq || !idx) return fail(MCL_EINVAL, "resample: NULL wq or idx");
    if (N < 1) return fail(MCL_EINVAL, "resample: need N >= 1");
    if (N > MCL_MAX_PARTICLES) return fail(MCL_ERANGE, "resample: N above the limit");
    if ((poses_in == nullptr) != (poses_out == nullptr))
        return fail(MCL_EINVAL, "resample: poses_in and poses_out must both be set or both be NULL");
    const size_t pb = (size_t)12 * N * 4;
    if (overlaps(poses_out, pb, poses_in, pb) || overlaps(poses_out, pb, wq, (size_t)N * 8) ||
        overlaps(poses_out, pb, idx, (size_t)N * 4) || overlaps(idx, (size_t)N * 4, wq, (size_t)N * 8) ||
        overlaps(idx, (size_t)N * 4, poses_in, pb))
        return fail(MCL_EINVAL, "resample: overlapping buffers");
    return launch_resample(wq, N, resample_draw(seed, tick), idx, poses_in, poses_out,
                           static_cast<hipStream_t>(stream));
}

extern "C" mcl_status mcl_pose_estimate(const double *w, const float *poses, int32_t N, double *mean,
                                        int32_t *best_idx, float *best_pose, void *stream) {
    if (!w || !poses || !mean) return fail(MCL_EINVAL, "pose_estimate: NULL w, poses or mean");
    if (N < 1) return fail(MCL_EINVAL, "pose_estimate: need N >= 1");
    if (N > MCL_MAX_PARTICLES) return fail(MCL_ERANGE, "pose_estimate: N above the limit");
    const size_t pb = (size_t)12 * N * 4, wb = (size_t)N * 8;
    const void *outs[3] = {mean, best_idx, best_pose};
    const size_t ob[3] = {12 * 8, 4, 12 * 4};
    for (int a = 0; a < 3; ++a) {
        if (overlaps(outs[a], ob[a], w, wb) || overlaps(outs[a], ob[a], poses, pb))
            return fail(MCL_EINVAL, "pose_estimate: overlapping buffers");
        for (int b = a + 1; b < 3; ++b)
            if (overlaps(outs[a], ob[a], outs[b], ob[b])) return fail(MCL_EINVAL, "pose_estimate: overlapping buffers");
    }
    return launch_estimate(w, poses, N, mean, best_idx, best_pose, static_cast<hipStream_t>(stream));
}

extern "C" mcl_status mcl_debug_voxel_indices(mcl_map map, const float *points, int32_t K, const float *poses,
                                              int32_t N, int64_t *lin_idx, void *stream) {
    if (!map || !poses || !lin_idx) return fail(MCL_EINVAL, "debug_voxel_indices: NULL argument");
    if (K < 0 || N < 1) return fail(MCL_EINVAL, "debug_voxel_indices: need K >= 0 and N >= 1");
    if (K > 0 && !points) return fail(MCL_EINVAL, "debug_voxel_indices: NULL points with K > 0");
    if ((int64_t)N * K > ((int64_t)1 << 31)) return fail(MCL_ERANGE, "debug_voxel_indices: N*K above 2^31");
    mcl_status st = launch_debug_indices(map, points, K, poses, N, lin_idx, static_cast<hipStream_t>(stream));
    return st == MCL_OK ? note_map_use(map, static_cast<hipStream_t>(stream)) : st;
}

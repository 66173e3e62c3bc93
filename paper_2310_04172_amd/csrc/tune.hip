// Launch-shape tuning of the sensor kernel.  Shapes differ only in how waves
// are grouped into workgroups and whether the grid is persistent; the
// per-particle summation order is fixed by K, so every shape gives the same
// bits and the tuner only ever changes speed.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "jobs.h"

namespace mcl {

mcl_status launch_sensor_cfg(const mcl_map_s *, const float *, int, const float *, int, float, float *, LaunchCfg,
                             hipStream_t);

namespace {
std::mutex g_tmu;
std::map<std::tuple<int, int, int>, LaunchCfg> g_tuned;

int size_class(int x) {  // ceil(log2(x)) for x >= 1
    int b = 0;
    while (b < 31 && (1 << b) < x) ++b;
    return b;
}

bool valid_cfg(const LaunchCfg &c) {
    return (c.waves_per_block == 2 || c.waves_per_block == 4 || c.waves_per_block == 8) && c.blocks_per_cu >= 0 &&
           c.blocks_per_cu <= 64 && c.coarse >= kCoarseAuto && c.coarse <= kCoarseBits;
}
}  // namespace

LaunchCfg tuned_config(int32_t dtype, int K, int N) {
    std::lock_guard<std::mutex> lk(g_tmu);
    auto it = g_tuned.find({dtype, size_class(std::max(K, 1)), size_class(std::max(N, 1))});
    if (it != g_tuned.end()) return it->second;
    return LaunchCfg{4, 0, kCoarseAuto};
}

}  // namespace mcl

using namespace mcl;

extern "C" mcl_status mcl_set_launch_config(int32_t dtype, int32_t K, int32_t N, const mcl_launch_config *cfg) {
    if (dtype < MCL_TSDF_I16 || dtype > MCL_TSDF_F32 || K < 0 || N < 1)
        return fail(MCL_EINVAL, "set_launch_config: bad storage type or size");
    std::lock_guard<std::mutex> lk(g_tmu);
    auto key = std::make_tuple((int)dtype, size_class(std::max(K, 1)), size_class(N));
    if (!cfg) {
        g_tuned.erase(key);
        return MCL_OK;
    }
    LaunchCfg c{cfg->waves_per_block, cfg->blocks_per_cu, cfg->coarse};
    if (!valid_cfg(c))
        return fail(MCL_EINVAL, "set_launch_config: waves_per_block must be 2, 4 or 8, blocks_per_cu 0..64, coarse 0..2");
    g_tuned[key] = c;
    return MCL_OK;
}

extern "C" mcl_status mcl_autotune(mcl_map map, const float *points, int32_t K, const float *poses, int32_t N,
                                   float sigma, float *logw, void *stream_, mcl_launch_config *best) {
    if (!map || !poses || !logw) return fail(MCL_EINVAL, "autotune: NULL argument");
    if (K < 1 || N < 1 || K > MCL_MAX_POINTS || N > MCL_MAX_PARTICLES)
        return fail(MCL_EINVAL, "autotune: need 1 <= K <= MCL_MAX_POINTS and 1 <= N <= MCL_MAX_PARTICLES");
    if (!points) return fail(MCL_EINVAL, "autotune: NULL points");
    if (!(std::isfinite(sigma) && sigma > 0.0f)) return fail(MCL_EINVAL, "autotune: sigma must be finite and > 0");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const double s = map->scale, sg = (double)sigma;
    const float c = (float)((s * s) / (2.0 * sg * sg));
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(MCL_EDEVICE, "autotune: event creation failed");
    LaunchCfg bestc{4, 0, kCoarseAuto};
    float best_ms = INFINITY;
    mcl_status st = MCL_OK;
    for (int wpb : {2, 4, 8}) {
        for (int bpc : {0, 2, 4, 8, 16}) {
            LaunchCfg cfg{wpb, bpc, kCoarseAuto};
            if ((st = launch_sensor_cfg(map, points, K, poses, N, c, logw, cfg, stream)) != MCL_OK) break;
            float t[3];
            for (int r = 0; r < 3 && st == MCL_OK; ++r) {
                if (hipEventRecord(e0, stream) != hipSuccess) st = fail(MCL_EDEVICE, "autotune: event record failed");
                if (st == MCL_OK) st = launch_sensor_cfg(map, points, K, poses, N, c, logw, cfg, stream);
                if (st == MCL_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                     hipEventElapsedTime(&t[r], e0, e1) != hipSuccess))
                    st = fail(MCL_EDEVICE, "autotune: timing failed");
            }
            if (st != MCL_OK) break;
            std::sort(t, t + 3);
            if (t[1] < best_ms) {
                best_ms = t[1];
                bestc = cfg;
            }
        }
        if (st != MCL_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MCL_OK) return st;
    if ((st = note_map_use(map, stream)) != MCL_OK) return st;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        g_tuned[{map->dtype, size_class(K), size_class(N)}] = bestc;
    }
    if (best) {
        best->waves_per_block = bestc.waves_per_block;
        best->blocks_per_cu = bestc.blocks_per_cu;
        best->coarse = bestc.coarse;
    }
    return MCL_OK;
}

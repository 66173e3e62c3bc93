// Launch tuning of the sensor kernel.  Every setting here only regroups work:
// waves per workgroup and a persistent grid, runs per 64-particle group (which
// particles' loops a wave executes), and where the nearest lookup reads the
// coarse level (mask bytes in global memory or bits in LDS, and the threshold
// of the per-wave choice).  The per-particle summation order is fixed by K, so
// every setting gives the same bits and the tuner only ever changes speed.
//
// Choices are kept per storage type and size class (K and N rounded up to
// powers of two), whatever the spread of the particles they were timed on; so
// the tuner keeps the per-wave coarse-level choice, which adapts to the spread,
// unless a forced mode is more than 1 % faster.  With the environment variable MCL_TUNE_CACHE naming a file,
// they persist across processes: the file is read at the first lookup and a
// line is appended per tuning result (later lines win), tagged with the GPU's
// architecture and compute-unit count so that another GPU ignores them.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "jobs.h"

namespace mcl {

mcl_status launch_sensor_cfg(const mcl_map_s *, const float *, int, const float *, int, float, float *, LaunchCfg,
                             hipStream_t, float *);

namespace {
std::mutex g_tmu;
std::map<std::tuple<int, int, int>, LaunchCfg> g_tuned;
bool g_loaded = false;

int size_class(int x) {  // ceil(log2(x)) for x >= 1
    int b = 0;
    while (b < 31 && (1 << b) < x) ++b;
    return b;
}

bool valid_cfg(const LaunchCfg &c) {
    const bool runs_ok = c.runs == 0 || (c.runs >= 1 && c.runs <= kGroup && (c.runs & (c.runs - 1)) == 0);
    return (c.waves_per_block == 2 || c.waves_per_block == 4 || c.waves_per_block == 8) && c.blocks_per_cu >= 0 &&
           c.blocks_per_cu <= 64 && c.coarse >= kCoarseAuto && c.coarse <= kCoarseBits && runs_ok && c.lds8 >= 0 &&
           c.lds8 <= 8;
}

std::string device_tag() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string arch(p.gcnArchName);
    for (char &ch : arch)
        if (ch == ' ') ch = '_';
    return arch + "/" + std::to_string(p.multiProcessorCount);
}

// Reads the cache file once (caller holds g_tmu).
void load_cache() {
    if (g_loaded) return;
    g_loaded = true;
    const char *path = std::getenv("MCL_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    const std::string tag = device_tag();
    char t[256];
    int dt, kc, nc;
    LaunchCfg c{};
    while (std::fscanf(f, "%255s %d %d %d %d %d %d %d %d", t, &dt, &kc, &nc, &c.waves_per_block, &c.blocks_per_cu,
                       &c.coarse, &c.runs, &c.lds8) == 9) {
        if (tag == t && valid_cfg(c)) g_tuned[{dt, kc, nc}] = c;
    }
    std::fclose(f);
}

void store(int dtype, int kc, int nc, const LaunchCfg &c) {  // caller holds g_tmu
    g_tuned[{dtype, kc, nc}] = c;
    const char *path = std::getenv("MCL_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %d %d %d %d\n", device_tag().c_str(), dtype, kc, nc, c.waves_per_block,
                 c.blocks_per_cu, c.coarse, c.runs, c.lds8);
    std::fclose(f);
}
}  // namespace

LaunchCfg tuned_config(int32_t dtype, int K, int N) {
    std::lock_guard<std::mutex> lk(g_tmu);
    load_cache();
    auto it = g_tuned.find({dtype, size_class(std::max(K, 1)), size_class(std::max(N, 1))});
    if (it != g_tuned.end()) return it->second;
    return kDefaultCfg;
}

}  // namespace mcl

using namespace mcl;

extern "C" mcl_status mcl_set_launch_config(int32_t dtype, int32_t K, int32_t N, const mcl_launch_config *cfg) {
    if (dtype < MCL_TSDF_I16 || dtype > MCL_TSDF_F32 || K < 0 || N < 1)
        return fail(MCL_EINVAL, "set_launch_config: bad storage type or size");
    std::lock_guard<std::mutex> lk(g_tmu);
    load_cache();
    auto key = std::make_tuple((int)dtype, size_class(std::max(K, 1)), size_class(N));
    if (!cfg) {
        g_tuned.erase(key);
        return MCL_OK;
    }
    LaunchCfg c{cfg->waves_per_block, cfg->blocks_per_cu, cfg->coarse, cfg->runs, cfg->lds_threshold};
    if (!valid_cfg(c))
        return fail(MCL_EINVAL, "set_launch_config: waves_per_block must be 2, 4 or 8, blocks_per_cu 0..64, coarse 0..2, "
                                "runs 0 or a power of two up to 64, lds_threshold 0..8");
    g_tuned[key] = c;
    return MCL_OK;
}

extern "C" mcl_status mcl_get_launch_config(int32_t dtype, int32_t K, int32_t N, mcl_launch_config *out) {
    if (dtype < MCL_TSDF_I16 || dtype > MCL_TSDF_F32 || K < 0 || N < 1 || !out)
        return fail(MCL_EINVAL, "get_launch_config: bad storage type, size or NULL output");
    const LaunchCfg c = tuned_config(dtype, K, N);
    out->waves_per_block = c.waves_per_block;
    out->blocks_per_cu = c.blocks_per_cu;
    out->coarse = c.coarse;
    out->runs = c.runs;
    out->lds_threshold = c.lds8;
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
    mcl_status st = MCL_OK;
    // Median over three batches of `reps` back-to-back launches (after one
    // untimed launch), per launch: a batch lasts at least about 2 ms, so short
    // launches are timed without the events' own resolution and jitter.
    int reps = 1;
    auto batch = [&](const LaunchCfg &cfg, int n, float &ms) -> mcl_status {
        mcl_status r = MCL_OK;
        if (hipEventRecord(e0, stream) != hipSuccess) return fail(MCL_EDEVICE, "autotune: event record failed");
        for (int i = 0; i < n && r == MCL_OK; ++i)
            r = launch_sensor_cfg(map, points, K, poses, N, c, logw, cfg, stream, nullptr);
        if (r == MCL_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            r = fail(MCL_EDEVICE, "autotune: timing failed");
        ms /= (float)n;
        return r;
    };
    auto time_cfg = [&](const LaunchCfg &cfg, float &ms) -> mcl_status {
        mcl_status r = launch_sensor_cfg(map, points, K, poses, N, c, logw, cfg, stream, nullptr);
        float t[3];
        for (int i = 0; i < 3 && r == MCL_OK; ++i) r = batch(cfg, reps, t[i]);
        if (r == MCL_OK) {
            std::sort(t, t + 3);
            ms = t[1];
        }
        return r;
    };
    {   // the batch length, from the default setting's time
        float once = 0.0f;
        if ((st = launch_sensor_cfg(map, points, K, poses, N, c, logw, kDefaultCfg, stream, nullptr)) == MCL_OK)
            st = batch(kDefaultCfg, 1, once);
        if (st == MCL_OK) reps = std::max(1, std::min(64, (int)std::ceil(2.0f / std::max(once, 1e-3f))));
    }
    LaunchCfg bestc = kDefaultCfg, best_auto = kDefaultCfg;
    float best_ms = INFINITY, best_auto_ms = INFINITY;
    // auto: the coarse level chosen per wave with a threshold below 8/8 - the
    // settings that adapt to the particle spread of whatever workload later
    // runs in this size class
    auto adaptive = [](const LaunchCfg &c) { return c.coarse == kCoarseAuto && c.lds8 < 8; };
    auto try_cfg = [&](const LaunchCfg &cfg) {
        float ms = INFINITY;
        if (st == MCL_OK) st = time_cfg(cfg, ms);
        if (st != MCL_OK) return;
        if (ms < best_ms) {
            best_ms = ms;
            bestc = cfg;
        }
        if (adaptive(cfg) && ms < best_auto_ms) {
            best_auto_ms = ms;
            best_auto = cfg;
        }
    };
    // coordinate descent: launch shape, then runs per group, then the coarse level
    for (int wpb : {2, 4, 8})
        for (int bpc : {0, 2, 4, 8, 16}) try_cfg(LaunchCfg{wpb, bpc, kCoarseAuto, 0, 0});
    const LaunchCfg shape = bestc;
    for (int runs : {1, 2, 4, 8, 16, 64}) try_cfg(LaunchCfg{shape.waves_per_block, shape.blocks_per_cu, kCoarseAuto, runs, 0});
    const LaunchCfg shaped = bestc;
    if (!map->sparse) {
        for (int l8 : {4, 5, 7, 8}) try_cfg(LaunchCfg{shaped.waves_per_block, shaped.blocks_per_cu, kCoarseAuto, shaped.runs, l8});
        for (int co : {kCoarseBytes, kCoarseBits})
            try_cfg(LaunchCfg{shaped.waves_per_block, shaped.blocks_per_cu, co, shaped.runs, 0});
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MCL_OK) return st;
    // a forced coarse mode suits the spread of the particles it was timed on
    // (mask bytes for particles spread over the map, LDS bits for converged
    // ones); the per-wave choice serves both, so it is kept when it is within
    // 1 % of the fastest
    if (!adaptive(bestc) && best_auto_ms <= 1.01f * best_ms) bestc = best_auto;
    if ((st = note_map_use(map, stream)) != MCL_OK) return st;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        load_cache();
        store(map->dtype, size_class(K), size_class(N), bestc);
    }
    if (best) {
        best->waves_per_block = bestc.waves_per_block;
        best->blocks_per_cu = bestc.blocks_per_cu;
        best->coarse = bestc.coarse;
        best->runs = bestc.runs;
        best->lds_threshold = bestc.lds8;
    }
    return MCL_OK;
}

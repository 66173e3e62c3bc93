// The sensor update for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid it).
//
// mcl_sensor_update keeps its piece partials (one float per particle and
// 4096-point piece of the scan, for scans of more than 4096 points) in a
// per-stream workspace that grows with hipMalloc.  This variant runs the same
// kernels with the partials in a fixed device array that the library holds for
// the life of the process, one per GPU; it allocates nothing.  The array is
// shared by every call on a GPU: calls that overlap on one GPU (on different
// streams, or on one stream from different threads without ordering) race on
// it.  The partials are written before they are read in every call, so the
// array needs no clearing.
#include <mutex>

#include "jobs.h"

// Partials of the no-allocation sensor update (see MCL_NOALLOC_SCRATCH_BYTES).
static __device__ __align__(256) float scratch[MCL_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace mcl {
mcl_status launch_sensor(const mcl_map_s *, const float *, int, const float *, int, float, float *, hipStream_t,
                         float *);
}  // namespace mcl

mcl_status sensor_args(const char *what, mcl_map map, const float *points, int32_t K, const float *poses, int32_t N,
                       float sigma, float *logw, float *c);

namespace {
// The device address of `scratch` on each GPU, taken once per device with that
// device current.  In host code the array's name is only a host-side handle,
// never a device address: kernels get these pointers.
constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void *g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];

float *scratch_ptr(int dev) {
    std::call_once(g_once[dev], [dev]() {
        void *p = nullptr;
        g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[dev] = g_err[dev] == hipSuccess ? p : nullptr;
    });
    return static_cast<float *>(g_ptr[dev]);
}
}  // namespace

using namespace mcl;

extern "C" mcl_status mcl_sensor_update_noalloc(mcl_map map, const float *points, int32_t K, const float *poses,
                                                int32_t N, float sigma, float *logw, void *stream) {
    float c = 0.0f;
    mcl_status st = sensor_args("sensor_update_noalloc", map, points, K, poses, N, sigma, logw, &c);
    if (st != MCL_OK) return st;
    const size_t need = sensor_pieces(K) > 1 ? (size_t)sensor_pieces(K) * N * sizeof(float) : 0;
    if (need > (size_t)MCL_NOALLOC_SCRATCH_BYTES)
        return fail(MCL_ERANGE, "sensor_update_noalloc: the piece partials need " + std::to_string(need) +
                                    " bytes (N times ceil(K / 4096) floats), above the fixed " +
                                    std::to_string((size_t)MCL_NOALLOC_SCRATCH_BYTES) + "-byte scratch array");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(MCL_EDEVICE, "sensor_update_noalloc: no usable current device");
    float *part = scratch_ptr(dev);
    if (!part)
        return fail(MCL_EDEVICE, std::string("sensor_update_noalloc: the scratch array's device address: ") +
                                     hipGetErrorString(g_err[dev]));
    return launch_sensor(map, points, K, poses, N, c, logw, static_cast<hipStream_t>(stream), part);
}

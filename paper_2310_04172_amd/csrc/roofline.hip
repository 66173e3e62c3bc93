// Measurement support: the ceilings the sensor update is measured against.
//
// The nearest lookup is bound by its map gathers (the TSDF look-ups the paper
// names as the bottleneck, §VI-C): each 64-lane gather instruction costs the
// texture path about one cycle per cache line it touches, and its misses cost
// fabric bandwidth.  Neither a flop count nor a byte count of the algorithm
// describes that, so the ceilings are measured:
//
//  * gather_replay_kernel issues exactly the sensor kernel's gathers - the
//    read-mask byte and the value of every (particle, point) pair, same lanes,
//    same 16-point batches, same order of chunks and particles - from byte
//    offsets exported by the sensor kernel's own device code, with no other
//    work than loading those offsets and adding the values.  Each
//    (particle, chunk) set of 1024 gathers is issued `reps` times in a row
//    (the compiler may not reuse the loaded values); from the timings at two
//    repeat counts the time of one extra pass is the cost of the gathers alone
//    with their lines in cache: the texture-path ceiling for this pattern.
//  * line_gather_kernel: random 128-byte lines within a region (sized to stay
//    in L2, in the Infinity Cache, or in HBM), `lines` distinct lines per
//    64-lane gather: the memory system's line rate.
//  * stream_read_kernel: a coalesced read of a large buffer (HBM bandwidth).
#include <algorithm>

#include "jobs.h"
#include "voxel.h"

namespace mcl {

// Byte offset (within the map's value allocation) each (particle, point) pair
// reads, by the sensor kernel's own recipe: the voxel's offset, or 0 (the +Q
// sentinel) outside the map; with `masked`, the read mask is applied (the
// offset of the value actually read, which for bricks wholly at +-Q is the
// sentinel's).  out: [N][K].
template <int ESIZE>
__global__ __launch_bounds__(256) void gather_offsets_kernel(MapView m, const float *__restrict__ pts, int K,
                                                             const float *__restrict__ poses, int N, int masked,
                                                             uint32_t *__restrict__ out) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)N * K) return;
    const int n = (int)(id / K), k = (int)(id - (int64_t)n * K);
    float pa[12];
    pose_consts(poses, N, n, m, pa);
    const float x = pts[k], y = pts[(size_t)K + k], z = pts[(size_t)2 * K + k];
    const float gx = grid_coord(pa[0], pa[1], pa[2], pa[9], x, y, z);
    const float gy = grid_coord(pa[3], pa[4], pa[5], pa[10], x, y, z);
    const float gz = grid_coord(pa[6], pa[7], pa[8], pa[11], x, y, z);
    uint32_t off = voxel_offset<ESIZE>(m, gx, gy, gz);
    if (masked) off &= (uint32_t)(int)m.mask[off >> (kBrickLog2 + (ESIZE == 1 ? 0 : ESIZE == 2 ? 1 : 2))];
    out[id] = off;
}

template <typename T>
__device__ inline int replay_load(const char *base, uint32_t off) {
    if constexpr (sizeof(T) == 4)
        return __float_as_int(*gp(reinterpret_cast<const float *>(base + off)));
    else
        return (int)*gp(reinterpret_cast<const T *>(base + off));
}

// Waves stride over work items (group of 64 particles, piece of 4096 points)
// of the exported sample, as the sensor kernel does; per chunk of 1024 points
// and particle, lane l loads its 16 offsets (points l, l + 64, ...), then issues
// the 16 gathers (16 mask bytes first, then 16 values at offset AND mask, or
// with two_gathers = 0 only the 16 values at pre-masked offsets) `reps` times.
template <typename T>
__global__ __launch_bounds__(256) void gather_replay_kernel(MapView m, const uint32_t *__restrict__ offs, int S,
                                                            int K, int reps, int two_gathers, float *__restrict__ sink) {
    constexpr int kShift = kBrickLog2 + (sizeof(T) == 1 ? 0 : sizeof(T) == 2 ? 1 : 2);
    const int lane = threadIdx.x & (kWave - 1);
    const int ngroups = S / kGroup;
    const int npiece = (K + kPiece - 1) / kPiece;
    const int64_t nitems = (int64_t)ngroups * npiece;
    float acc = 0.0f;
    for (int64_t item = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); item < nitems;
         item += (int64_t)gridDim.x * 4) {
        const int g = (int)(item / npiece), piece = (int)(item - (int64_t)g * npiece);
        const int kb = piece * kPiece, ke = min(K, kb + kPiece);
        for (int kc = kb; kc < ke; kc += kChunk) {
            for (int p = 0; p < kGroup; ++p) {
                const uint32_t *row = offs + (size_t)(g * kGroup + p) * K;
                uint32_t off[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int k = kc + u * kWave + lane;
                    off[u] = k < ke ? gp(row)[k] : m.zero_off;
                }
                for (int r = 0; r < reps; ++r) {
                    asm volatile("" ::: "memory");   // every pass loads again
                    int raw[kU];
                    if (two_gathers) {
                        int msk[kU];
#pragma unroll
                        for (int u = 0; u < kU; ++u) msk[u] = gp(m.mask)[off[u] >> kShift];
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int u = 0; u < kU; ++u) raw[u] = replay_load<T>(m.base, off[u] & (uint32_t)msk[u]);
                    } else {
#pragma unroll
                        for (int u = 0; u < kU; ++u) raw[u] = replay_load<T>(m.base, off[u]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    float s = 0.0f;
#pragma unroll
                    for (int u = 0; u < kU; ++u) {
                        const float f = sizeof(T) == 4 ? __int_as_float(raw[u]) : (float)raw[u];
                        s = __builtin_fmaf(f, f, s);
                    }
                    acc += s;
                }
            }
        }
    }
    sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// Random 128-byte lines of a region of 2^log2_lines lines: lane l of a wave
// reads W bytes of line x_(l / (64 / lines)), at byte W (l mod (64 / lines))
// of it (modulo 128), x a per-lane-group 32-bit LCG, 16 loads in flight per step.
template <int W>
__device__ inline uint32_t load_w(const char *p) {
    if constexpr (W == 1) return (uint32_t)(int)*gp(reinterpret_cast<const int8_t *>(p));
    else if constexpr (W == 2) return (uint32_t)(int)*gp(reinterpret_cast<const int16_t *>(p));
    else return *gp(reinterpret_cast<const uint32_t *>(p));
}

template <int W>
__global__ __launch_bounds__(256) void line_gather_kernel(const char *__restrict__ base, int log2_lines, int lines,
                                                          int steps, uint32_t seed, float *__restrict__ sink) {
    const int lane = threadIdx.x & (kWave - 1);
    const int per = kWave / lines;                    // lanes per line
    const uint32_t wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    uint32_t x = (seed ^ (wave * 0x9E3779B9u)) + (uint32_t)(lane / per) * 0x85EBCA6Bu;
    const uint32_t byte = ((uint32_t)(lane % per) * W) & 127u;   // within the 128-byte line
    const int sh = 32 - log2_lines;
    uint32_t acc = 0;
    for (int s = 0; s < steps; ++s) {
        uint32_t v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            x = x * 1664525u + 1013904223u;
            const uint32_t line = sh >= 32 ? 0u : (x >> sh);
            v[u] = load_w<W>(base + (size_t)line * 128 + byte);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += v[u];
    }
    sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = (float)acc;
}

// Texture-path cost of a gather against the lines it touches, data resident
// in L1: lane l reads W bytes at byte offset 128 (l / (64 / lines)) + W (l mod
// (64 / lines)) (mod 128) of an 8 KiB block, so a gather touches exactly
// `lines` lines; the block's base is a scalar and the lane offsets fixed, so a
// load costs no vector instruction besides the sum.
template <int W>
__global__ __launch_bounds__(256) void l1_gather_kernel(const char *base, int lines, int steps, float *__restrict__ sink) {
    const int lane = threadIdx.x & (kWave - 1);
    const int per = kWave / lines;
    const uint32_t lo = (uint32_t)(lane / per) * 128u + (((uint32_t)(lane % per) * W) & 127u);
    uint32_t acc = 0;
    for (int s = 0; s < steps; ++s) {
        uint32_t v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            // the same lane offset every time, opaque to the compiler, so that
            // no load is merged with another or hoisted out of the loop; the
            // address is the scalar base plus this 32-bit offset, as in the
            // sensor kernel's gathers
            uint32_t o = lo;
            asm volatile("" : "+v"(o));
            v[u] = load_w<W>(base + o);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += v[u];
    }
    sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = (float)acc;
}

typedef uint32_t u32x4r __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void stream_read_kernel(const u32x4r *__restrict__ src, size_t n16,
                                                          float *__restrict__ sink) {
    uint32_t acc = 0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u32x4r a = gp(src)[i], b = gp(src)[i + stride], c = gp(src)[i + 2 * stride], d = gp(src)[i + 3 * stride];
        acc += a.x + a.y + a.z + a.w + b.x + b.y + b.z + b.w + c.x + c.y + c.z + c.w + d.x + d.y + d.z + d.w;
    }
    for (; i < n16; i += stride) {
        const u32x4r a = gp(src)[i];
        acc += a.x + a.y + a.z + a.w;
    }
    sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = (float)acc;
}

}  // namespace mcl

using namespace mcl;

extern "C" mcl_status mcl_bench_gather_offsets(mcl_map map, const float *points, int32_t K, const float *poses,
                                               int32_t N, int32_t masked, uint32_t *offs, void *stream) {
    if (!map || !points || !poses || !offs) return fail(MCL_EINVAL, "bench_gather_offsets: NULL argument");
    if (K < 1 || N < 1 || K > MCL_MAX_POINTS || N > MCL_MAX_PARTICLES)
        return fail(MCL_EINVAL, "bench_gather_offsets: need 1 <= K <= MCL_MAX_POINTS and 1 <= N <= MCL_MAX_PARTICLES");
    if (map->sparse) return fail(MCL_EINVAL, "bench_gather_offsets: dense maps only");
    const int64_t total = (int64_t)N * K;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned blocks = (unsigned)((total + 255) / 256);
    const int e = elem_size(map->dtype);
    if (e == 2) gather_offsets_kernel<2><<<blocks, 256, 0, s>>>(map->view, points, K, poses, N, masked, offs);
    else if (e == 1) gather_offsets_kernel<1><<<blocks, 256, 0, s>>>(map->view, points, K, poses, N, masked, offs);
    else gather_offsets_kernel<4><<<blocks, 256, 0, s>>>(map->view, points, K, poses, N, masked, offs);
    mcl_status st = check_launch("gather_offsets_kernel");
    return st == MCL_OK ? note_map_use(map, s) : st;
}

extern "C" mcl_status mcl_bench_gather_replay(mcl_map map, const uint32_t *offs, int32_t S, int32_t K, int32_t reps,
                                              int32_t two_gathers, int32_t blocks, float *sink, size_t sink_floats,
                                              void *stream) {
    if (!map || !offs || !sink) return fail(MCL_EINVAL, "bench_gather_replay: NULL argument");
    if (S < kGroup || S % kGroup || K < 1 || K > MCL_MAX_POINTS || reps < 1 || blocks < 1)
        return fail(MCL_EINVAL, "bench_gather_replay: need S a positive multiple of 64, 1 <= K, reps >= 1, blocks >= 1");
    if (sink_floats < (size_t)blocks * 256) return fail(MCL_EINVAL, "bench_gather_replay: sink shorter than blocks * 256");
    if (map->sparse) return fail(MCL_EINVAL, "bench_gather_replay: dense maps only");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (map->dtype == MCL_TSDF_I16)
        gather_replay_kernel<int16_t><<<(unsigned)blocks, 256, 0, s>>>(map->view, offs, S, K, reps, two_gathers, sink);
    else if (map->dtype == MCL_TSDF_I8)
        gather_replay_kernel<int8_t><<<(unsigned)blocks, 256, 0, s>>>(map->view, offs, S, K, reps, two_gathers, sink);
    else
        gather_replay_kernel<float><<<(unsigned)blocks, 256, 0, s>>>(map->view, offs, S, K, reps, two_gathers, sink);
    mcl_status st = check_launch("gather_replay_kernel");
    return st == MCL_OK ? note_map_use(map, s) : st;
}

extern "C" mcl_status mcl_bench_line_gather(const void *region, size_t region_bytes, int32_t log2_lines, int32_t lines,
                                            int32_t bytes_per_lane, int32_t steps, uint32_t seed, int32_t blocks,
                                            float *sink, size_t sink_floats, void *stream) {
    if (!region || !sink) return fail(MCL_EINVAL, "bench_line_gather: NULL argument");
    if (sink_floats < (size_t)blocks * 256) return fail(MCL_EINVAL, "bench_line_gather: sink shorter than blocks * 256");
    if (log2_lines < 0 || log2_lines > 31 || !(lines == 1 || lines == 2 || lines == 4 || lines == 8 || lines == 16 ||
                                                lines == 32 || lines == 64) || steps < 1 || blocks < 1 ||
        !(bytes_per_lane == 1 || bytes_per_lane == 2 || bytes_per_lane == 4))
        return fail(MCL_EINVAL, "bench_line_gather: need 0 <= log2_lines <= 31, lines a power of two <= 64, "
                                "1, 2 or 4 bytes per lane");
    if (((size_t)128 << log2_lines) > region_bytes)
        return fail(MCL_EINVAL, "bench_line_gather: 2^log2_lines lines of 128 bytes exceed the region");
    const char *b = static_cast<const char *>(region);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (bytes_per_lane == 1) line_gather_kernel<1><<<(unsigned)blocks, 256, 0, s>>>(b, log2_lines, lines, steps, seed, sink);
    else if (bytes_per_lane == 2) line_gather_kernel<2><<<(unsigned)blocks, 256, 0, s>>>(b, log2_lines, lines, steps, seed, sink);
    else line_gather_kernel<4><<<(unsigned)blocks, 256, 0, s>>>(b, log2_lines, lines, steps, seed, sink);
    return check_launch("line_gather_kernel");
}

extern "C" mcl_status mcl_bench_l1_gather(const void *block, size_t block_bytes, int32_t lines, int32_t bytes_per_lane,
                                          int32_t steps, int32_t blocks, float *sink, size_t sink_floats,
                                          void *stream) {
    if (!block || !sink) return fail(MCL_EINVAL, "bench_l1_gather: NULL argument");
    if (block_bytes < 8192) return fail(MCL_EINVAL, "bench_l1_gather: the block must hold 8 KiB");
    if (sink_floats < (size_t)blocks * 256) return fail(MCL_EINVAL, "bench_l1_gather: sink shorter than blocks * 256");
    if (!(lines == 1 || lines == 2 || lines == 4 || lines == 8 || lines == 16 || lines == 32 || lines == 64) ||
        steps < 1 || blocks < 1 || !(bytes_per_lane == 1 || bytes_per_lane == 2 || bytes_per_lane == 4))
        return fail(MCL_EINVAL, "bench_l1_gather: lines a power of two <= 64, 1, 2 or 4 bytes per lane");
    const char *b = static_cast<const char *>(block);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (bytes_per_lane == 1) l1_gather_kernel<1><<<(unsigned)blocks, 256, 0, s>>>(b, lines, steps, sink);
    else if (bytes_per_lane == 2) l1_gather_kernel<2><<<(unsigned)blocks, 256, 0, s>>>(b, lines, steps, sink);
    else l1_gather_kernel<4><<<(unsigned)blocks, 256, 0, s>>>(b, lines, steps, sink);
    return check_launch("l1_gather_kernel");
}

extern "C" mcl_status mcl_bench_stream_read(const void *src, size_t bytes, int32_t blocks, float *sink,
                                            size_t sink_floats, void *stream) {
    if (!src || !sink || bytes % 16 || blocks < 1) return fail(MCL_EINVAL, "bench_stream_read: bad argument");
    if (sink_floats < (size_t)blocks * 256) return fail(MCL_EINVAL, "bench_stream_read: sink shorter than blocks * 256");
    stream_read_kernel<<<(unsigned)blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<const u32x4r *>(src), bytes / 16, sink);
    return check_launch("stream_read_kernel");
}

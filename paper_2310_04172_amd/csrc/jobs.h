// Per-filter work descriptions shared by the single-filter entry points and the
// batched tick.  A kernel reads its filters through a job source: either one
// job passed by value (single filter) or a table in device memory (batch),
// searched by the prefix offsets each job carries.
#pragma once

#include "mcl_internal.h"

namespace mcl {

// Sensor-update decomposition.  The summation order depends only on these
// constants and K (see sensor.hip), never on the launch shape.
constexpr int kU = 16;                            // points per lane per chunk
constexpr int kChunk = kWave * kU;                // 1024
constexpr int kChunksPerPiece = 4;
constexpr int kPiece = kChunk * kChunksPerPiece;  // 4096 points
constexpr int kGroup = 64;                        // particles per group (lane p holds particle p's pose)

inline int sensor_pieces(int K) { return K <= 0 ? 1 : (K + kPiece - 1) / kPiece; }

// Launches of at least this many particle-point evaluations first write every
// particle's pose constants to a table that the sensor kernel reads with scalar
// loads; smaller ones broadcast them between lanes (the table's extra launch
// costs more than it saves there).  The same values either way.
constexpr int64_t kPoseTableMinEvals = int64_t(1) << 29;

// Spatial order of a filter's particles for the sensor launch.  A filter of at
// least spatial_order_min() evaluations is counting-sorted by the cell of its
// particles' x-y position (kOrderSide x kOrderSide cells over the map's extent,
// cells in Morton order) as its pose-constant table is written: slot s of the
// table holds particle orig[s], so a wave's particles lie close together and so
// do those of neighbouring work items, whose lookups then share cache lines.
// Each particle's sum is formed exactly as before and written back to its own
// index, so results do not depend on the order.
constexpr int kOrderSide = 64;
constexpr int kOrderCells = kOrderSide * kOrderSide;
constexpr int kOrderBlock = 4096;                 // particles per counting block (256 threads x 16)
constexpr int64_t kOrderDefaultMin = int64_t(1) << 30;
int64_t spatial_order_min();                      // < 0: never
inline bool spatial_order(int64_t evals) {
    const int64_t m = spatial_order_min();
    return m >= 0 && evals >= m;
}
inline int order_blocks(int N) { return (N + kOrderBlock - 1) / kOrderBlock; }

// Work items are (group, piece, run): a launch with few (group, piece) pairs
// splits each group's particles into nsub runs of 64 / nsub (a power of two up
// to 64), one work item each, until it has about kTargetItems items (four per
// wave slot of the chip), so small filters still spread over the chip.  A run
// only selects which particles' loops a wave executes: every particle's sum is
// formed in the same order whatever nsub is.
constexpr int64_t kTargetItems = 16384;
inline int sensor_runs(int64_t pairs) {
    int s = 1;
    while (s < kGroup && pairs * s < kTargetItems) s *= 2;
    return s;
}

struct SensorJob {
    MapView map;
    TriView tri;          // corner cells (trilinear lookup only)
    SparseView sp;        // coarse table + pool (sparse maps only)
    const float *pts;     // [3][K]
    const float *poses;   // [12][N]
    float *logw;          // [N] output
    float *part;          // [npiece][N] piece partials (npiece > 1)
    int64_t item0;        // first work item of this job in the launch
    int64_t elem0;        // first particle of this job in the launch
    float c;              // s^2 / (2 sigma^2)
    int32_t K, N, npiece, ngroups;
    int32_t coarse;       // where the nearest lookup reads the coarse level (kCoarse*)
    int32_t nsub;         // runs per group (work items per (group, piece) pair)
    int32_t lds8;         // auto coarse level: LDS when over lds8 / 8 of the probe lookups read in place
    int32_t score;        // kScoreProduct or kScoreSum (how the points' likelihoods combine)
    float k2;             // sum reading: -c log2(e), so a point's likelihood is 2^(k2 q^2)
    int32_t pad_;
    const float *pc;      // [N][12] the pose constants of the particle in each slot, or null: broadcast from the lanes
    int32_t *ocell;       // spatial order: [kOrderCells] particles per cell, then the cell's first slot
    int32_t *orank;       // spatial order: [N] a particle's rank within its cell
    int32_t *orig;        // spatial order: [N] the particle in each slot; null: slot n holds particle n
    int64_t oblk0;        // spatial order: first counting block of this job in the launch
};

// How a particle's points combine: the product of their likelihoods (l = -c sum q^2)
// or their sum (l = log sum exp(-c q^2)).
constexpr int32_t kScoreProduct = 0, kScoreSum = 1;

// Sum reading, host side: a point's likelihood exp(-c q^2) is 2^(k2 q^2) with
// k2 = -c log2(e).  The smallest likelihood, at q = Q (tau for float32 maps),
// is exp(-tau^2 / (2 sigma^2)); sigma >= tau / 8 keeps it at or above e^-32, a
// normal float, so no term underflows.
inline double score_c(const mcl_map_s *m, float sigma) {
    const double s = m->scale, sg = (double)sigma;
    return (s * s) / (2.0 * sg * sg);
}
inline bool sum_sigma_ok(const mcl_map_s *m, float sigma) { return 8.0 * (double)sigma >= (double)m->tau; }
inline float sum_k2(const mcl_map_s *m, float sigma) { return (float)(-score_c(m, sigma) * 1.4426950408889634); }

// Coarse level of the nearest lookup: chosen per wave and chunk (auto), or
// forced to the mask bytes in global memory or the bits in LDS.  Results are
// the same bits in every mode.
constexpr int32_t kCoarseAuto = 0, kCoarseBytes = 1, kCoarseBits = 2;
constexpr int kProbe = 2;      // probe particles per chunk
constexpr int kLdsEighths = 6;  // default: LDS when over 6/8 of the probe lookups read in place

// The resampling draw of a filter's update: u = splitmix64(seed ^ splitmix64(tick)),
// splitmix64(x) the output of SplitMix64 (Steele, Lea and Flood, 2014) from
// state x.  Host code: the draw is computed when the work is enqueued.
inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
inline uint64_t resample_draw(uint64_t seed, uint64_t tick) { return splitmix64(seed ^ splitmix64(tick)); }

// Weight normalisation and resampling of one filter.
constexpr int kWThreads = 256;
constexpr int kWPer = 16;
constexpr int kWBlock = kWThreads * kWPer;  // 4096 particles per block

inline int weight_blocks(int N) { return (N + kWBlock - 1) / kWBlock; }

struct WeightJob {
    const float *logw;    // [N]
    double *w;            // [N] or null
    uint64_t *wq;         // [N]
    double *log_z;        // [1] or null (output)
    int32_t *idx;         // [N] or null (normalise only)
    const float *pin;     // [12][N] or null
    float *pout;          // [12][N] or null
    double *lse_part;     // workspace [2 nblk]
    double *lz;           // workspace [1]
    uint64_t *bsum;       // workspace [nblk]
    uint64_t *total;      // workspace [1]
    uint64_t *C;          // workspace [N]
    uint64_t u;           // resampling draw
    int64_t elem0;        // first particle of this job in the launch
    int32_t blk0;         // first weight block of this job in the launch
    int32_t nblk, N, pad_;
};

// Pose estimate of one filter (weighted mean and best particle).
struct EstJob {
    const double *w;      // [N] normalised weights
    const float *poses;   // [12][N]
    double *mean;         // [12] output
    int32_t *best_idx;    // [1] output or null
    float *best_pose;     // [12] output or null
    double *part;         // workspace [accumulators][nblk]
    void *pbest;          // workspace [nblk] (weight, index) pairs
    int32_t N;
    int32_t nblk;         // blocks of this job (a function of N alone)
    int32_t blk0;         // first block of this job in the launch
    int32_t pad_;
};

int estimate_blocks(int N);
size_t estimate_ws_bytes(int N);
void bind_estimate_ws(EstJob &J, void *ws);

// ------------------------------------------------------------ job sources
// Copy a descriptor at a wave-uniform address into scalar registers.  The
// job tables are written before the kernels that read them start and never
// during them, so they are read as constant memory: scalar loads, which the
// compiler may repeat where registers run short.  (Read as ordinary memory
// through vector loads and readfirstlane, the sensor kernel's descriptor
// fields had to be spilled to vector-register lanes and restored once per
// particle, 9 extra instructions per 16 evaluations.)
template <typename T>
__device__ __attribute__((always_inline)) inline T load_uniform(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "descriptor size must be a multiple of 4");
    union {
        T v;
        int w[sizeof(T) / 4];
    } u;
    const __attribute__((address_space(4))) int *q = (const __attribute__((address_space(4))) int *)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) u.w[i] = q[i];
    return u.v;
}

// Totals of a launch: jobs, sensor work items, particles, weight blocks.
struct Counts {
    int64_t njobs, items, elems, blocks;
};

template <typename J>
struct OneJob {
    J job;
    Counts n;
    __device__ const J &get(int) const { return job; }
    __device__ J load(int) const { return job; }
    __device__ int count() const { return 1; }
    __device__ int64_t items() const { return n.items; }
    __device__ int64_t elems() const { return n.elems; }
    __device__ int64_t blocks() const { return n.blocks; }
};

// Jobs and totals in device memory, so one captured launch chain serves any
// job set written there before it runs.
template <typename J>
struct JobTable {
    const J *jobs;
    const Counts *n;
    __device__ const J &get(int j) const { return jobs[j]; }
    __device__ J load(int j) const { return load_uniform(jobs + j); }
    __device__ int count() const { return (int)n->njobs; }
    __device__ int64_t items() const { return n->items; }
    __device__ int64_t elems() const { return n->elems; }
    __device__ int64_t blocks() const { return n->blocks; }
};

// Index of the last job whose key(job) <= x (jobs sorted by key), per lane:
// for element-indexed work, where lanes of one wave may belong to different
// jobs.
template <typename Src, typename Key>
__device__ inline int find_job(const Src &src, int64_t x, Key key) {
    int lo = 0, hi = src.count() - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (key(src.get(mid)) <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The same for an x that is equal on all lanes of the wave (a work item or a
// block index): the search and its result are provably wave-uniform.
template <typename Src, typename Key>
__device__ inline int find_job_uniform(const Src &src, int64_t x, Key key) {
    int lo = 0, hi = src.count() - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        int64_t k = key(src.get(mid));
        k = ((int64_t)__builtin_amdgcn_readfirstlane((int)(k >> 32)) << 32) |
            (uint32_t)__builtin_amdgcn_readfirstlane((int)(k & 0xffffffff));
        if (k <= x) lo = mid;
        else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Launch shape of the sensor kernel; any shape gives bit-identical results.
struct LaunchCfg {
    int waves_per_block;  // 2, 4 or 8
    int blocks_per_cu;    // 0: one wave per work item; else a persistent grid
    int coarse;           // kCoarseAuto, kCoarseBytes or kCoarseBits
    int runs;             // runs per 64-particle group: 0 = from the launch's size, else 1, 2, 4, .., 64
    int lds8;             // auto coarse level threshold in eighths (1..8); 0 = kLdsEighths
};
constexpr LaunchCfg kDefaultCfg{4, 0, kCoarseAuto, 0, 0};

LaunchCfg tuned_config(int32_t dtype, int K, int N);
int device_cus();

}  // namespace mcl

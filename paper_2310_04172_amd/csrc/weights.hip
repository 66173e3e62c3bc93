// Weight normalisation (float64 log-sum-exp, §V-A) and low-variance resampling
// on 64-bit fixed-point weights (§III), for one filter or a batch of filters.
// Every reduction runs in a fixed order (no atomics), so results are
// reproducible bit for bit and identical whether a filter runs alone or in a
// batch.  Blocks of 4096 particles are the unit of work; a launch strides
// over the (filter, block) pairs of all its filters.
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "jobs.h"

namespace mcl {

constexpr double kWqScale = 4398046511104.0;  // 2^42

// Fixed-order tree over the block: at stride 128, 64, ..., 1 the value of
// thread t becomes op(value t, value t + stride).  The two strides that cross
// waves go through LDS; the six inside wave 0 through lane shuffles (lane t
// reads lane t + stride; lanes at or above the stride compute values the tree
// never uses), so the additions and their order are those of the plain loop
// over LDS, with three barriers instead of nine.
static_assert(kWThreads == 256, "the tree is written for four waves of 64");
template <typename V, typename Op>
__device__ inline V block_tree(V x, V *sh, Op op) {
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    if (t < 128) sh[t] = op(sh[t], sh[t + 128]);
    __syncthreads();
    if (t < 64) {
        V y = op(sh[t], sh[t + 64]);
#pragma unroll
        for (int st = 32; st > 0; st >>= 1) y = op(y, __shfl_down(y, st));
        if (t == 0) sh[0] = y;
    }
    __syncthreads();
    V r = sh[0];
    __syncthreads();
    return r;
}

// Inclusive scan of one value per thread over the block (integer, so exact in
// any order): lane shuffles inside each wave, then the totals of the waves
// before.  *total receives the block's sum.
__device__ inline uint64_t block_scan(uint64_t x, uint64_t *sh, uint64_t *total) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kWThreads / 64; ++w) {
        const uint64_t v = sh[w];
        if (w < wave) before += v;
        all += v;
    }
    __syncthreads();
    *total = all;
    return before + x;
}

// LDS slot of element k of a 4096-value block: one pad slot after every 16, so
// that a thread walking its own 16 consecutive values and the 64 lanes of a
// wave walking theirs hit different banks.
constexpr int kPadBlock = kWBlock + kWBlock / 16;
__device__ inline int pad16(int k) { return k + (k >> 4); }

// Global load and store at a 32-bit byte offset from a wave-uniform base: the
// base stays in scalar registers and each lane holds one offset register.
typedef __attribute__((address_space(1))) char gchar;
__device__ inline float load_at(const float *base, uint32_t off) {
    return *(const __attribute__((address_space(1))) float *)((const gchar *)base + off);
}
__device__ inline void store_at(float *base, uint32_t off, float v) {
    *(__attribute__((address_space(1))) float *)((gchar *)base + off) = v;
}

struct MaxF { __device__ float operator()(float a, float b) const { return fmaxf(a, b); } };
struct MaxD { __device__ double operator()(double a, double b) const { return fmax(a, b); } };
struct AddD { __device__ double operator()(double a, double b) const { return a + b; } };
struct AddU { __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a + b; } };

struct BlkKey { __device__ int64_t operator()(const WeightJob &J) const { return J.blk0; } };
struct ElemKey { __device__ int64_t operator()(const WeightJob &J) const { return J.elem0; } };

// Per block: m_b = max l, S_b = sum exp(l - m_b).
template <typename Src>
__global__ __launch_bounds__(kWThreads) void lse_partial_kernel(Src src) {
    const int64_t nblocks = src.blocks();
    __shared__ float shf[kWThreads];
    __shared__ double shd[kWThreads];
    for (int64_t gb = blockIdx.x; gb < nblocks; gb += gridDim.x) {
        const WeightJob &J = src.get(find_job_uniform(src, gb, BlkKey()));
        const int b = (int)(gb - J.blk0);
        const int base = b * kWBlock + threadIdx.x;
        float mx = -INFINITY;
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            int n = base + i * kWThreads;
            if (n < J.N) mx = fmaxf(mx, J.logw[n]);
        }
        mx = block_tree(mx, shf, MaxF());
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            int n = base + i * kWThreads;
            if (n < J.N) s += exp((double)J.logw[n] - (double)mx);
        }
        s = block_tree(s, shd, AddD());
        if (threadIdx.x == 0) {
            J.lse_part[2 * b] = (double)mx;
            J.lse_part[2 * b + 1] = s;
        }
    }
}

// One block per filter: log Z = m + log sum_b S_b exp(m_b - m).
template <typename Src>
__global__ __launch_bounds__(kWThreads) void lse_reduce_kernel(Src src) {
    __shared__ double shd[kWThreads];
    for (int j = blockIdx.x; j < src.count(); j += gridDim.x) {
        const WeightJob &J = src.get(j);
        double mx = -INFINITY;
        for (int b = threadIdx.x; b < J.nblk; b += kWThreads) mx = fmax(mx, J.lse_part[2 * b]);
        mx = block_tree(mx, shd, MaxD());
        double s = 0.0;
        for (int b = threadIdx.x; b < J.nblk; b += kWThreads) s += J.lse_part[2 * b + 1] * exp(J.lse_part[2 * b] - mx);
        s = block_tree(s, shd, AddD());
        if (threadIdx.x == 0) {
            double lz = mx + log(s);
            J.lz[0] = lz;
            if (J.log_z) J.log_z[0] = lz;
        }
    }
}

template <typename Src>
__global__ __launch_bounds__(kWThreads) void weights_kernel(Src src) {
    const int64_t nelems = src.elems();
    for (int64_t e = (int64_t)blockIdx.x * kWThreads + threadIdx.x; e < nelems; e += (int64_t)gridDim.x * kWThreads) {
        const WeightJob &J = src.get(find_job(src, e, ElemKey()));
        const int n = (int)(e - J.elem0);
        double wn = exp((double)J.logw[n] - J.lz[0]);
        if (J.w) J.w[n] = wn;
        J.wq[n] = (uint64_t)(wn * kWqScale);  // w >= 0: truncation is floor; scaling by 2^42 is exact
    }
}

// ---------------------------------------------------------------- resampling
template <typename Src>
__global__ __launch_bounds__(kWThreads) void rs_blocksum_kernel(Src src) {
    const int64_t nblocks = src.blocks();
    __shared__ uint64_t sh[kWThreads];
    for (int64_t gb = blockIdx.x; gb < nblocks; gb += gridDim.x) {
        const WeightJob &J = src.get(find_job_uniform(src, gb, BlkKey()));
        const int b = (int)(gb - J.blk0);
        const int base = b * kWBlock + threadIdx.x;
        uint64_t s = 0;
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            int n = base + i * kWThreads;
            if (n < J.N) s += J.wq[n];
        }
        s = block_tree(s, sh, AddU());
        if (threadIdx.x == 0) J.bsum[b] = s;
    }
}

// Inclusive scan C of wq: block prefix from the filter's block sums, then a scan
// of the block's 4096 values staged in LDS.  Block 0 also writes the total T.
template <typename Src>
__global__ __launch_bounds__(kWThreads) void rs_scan_kernel(Src src) {
    const int64_t nblocks = src.blocks();
    __shared__ uint64_t vals[kPadBlock];
    __shared__ uint64_t sh[kWThreads];
    const int t = threadIdx.x;
    for (int64_t gb = blockIdx.x; gb < nblocks; gb += gridDim.x) {
        const WeightJob &J = src.get(find_job_uniform(src, gb, BlkKey()));
        const int b = (int)(gb - J.blk0);
        uint64_t pre = 0, tot = 0;
        for (int j = t; j < J.nblk; j += kWThreads) {
            uint64_t v = J.bsum[j];
            tot += v;
            if (j < b) pre += v;
        }
        pre = block_tree(pre, sh, AddU());
        tot = block_tree(tot, sh, AddU());
        const int base = b * kWBlock;
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            int n = base + i * kWThreads + t;
            vals[pad16(i * kWThreads + t)] = n < J.N ? J.wq[n] : 0;
        }
        __syncthreads();
        uint64_t run = 0;
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            run += vals[pad16(t * kWPer + i)];
            vals[pad16(t * kWPer + i)] = run;
        }
        uint64_t btot;
        const uint64_t excl = pre + block_scan(run, sh, &btot) - run;
#pragma unroll
        for (int i = 0; i < kWPer; ++i) vals[pad16(t * kWPer + i)] += excl;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            int n = base + i * kWThreads + t;
            if (n < J.N) J.C[n] = vals[pad16(i * kWThreads + t)];
        }
        if (b == 0 && t == 0) J.total[0] = tot;
        __syncthreads();
    }
}

// Output slot m: x = m T + r; the ancestor is the first i with N C_i > x, i.e.
// C_i > floor(x / N) (C_i is an integer).  Found by binary search; since
// x < N T, i exists.  Then the pose is gathered.
template <typename Src>
__global__ __launch_bounds__(kWThreads) void rs_search_kernel(Src src) {
    const int64_t nelems = src.elems();
    for (int64_t e = (int64_t)blockIdx.x * kWThreads + threadIdx.x; e < nelems; e += (int64_t)gridDim.x * kWThreads) {
        const WeightJob &J = src.get(find_job(src, e, ElemKey()));
        const int m = (int)(e - J.elem0);
        const int N = J.N;
        const uint64_t T = J.total[0];
        int i;
        if (T == 0) {
            i = m;
        } else {
            const uint64_t r = __umul64hi(J.u, T);
            const uint64_t x = (uint64_t)m * T + r;
            const uint64_t y = x / (uint64_t)N;
            int lo = 0, hi = N - 1;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (J.C[mid] > y) hi = mid;
                else lo = mid + 1;
            }
            i = lo;
        }
        J.idx[m] = i;
        if (J.pout) {
#pragma unroll
            for (int j = 0; j < 12; ++j) J.pout[(size_t)j * N + m] = J.pin[(size_t)j * N + i];
        }
    }
}

// ----------------------------------------------- one workgroup per filter
// Normalisation and/or resampling of filters of at most 4096 particles (one
// weight block), one workgroup each, in one launch.  The floating-point work
// repeats the launches above operation for operation and in the same order
// (the block's max and its tree sum of exp(l - m), the reduction over blocks,
// which with a single block leaves that partial as it is, then the weights),
// and the scan and search are integer, exact in any order, so every output is
// bit-identical to the three-launch chains.  One CU serves a filter, so the
// work is latency-bound: each thread keeps its 16 log-weights in registers
// from the first load to the weights, the fixed-point weights and their scan
// stay in LDS, and the 16 searches of a thread advance together.
struct FusedShared {
    float f[kWThreads];
    double d[kWThreads];
    uint64_t u[kWThreads];
    uint64_t C[kPadBlock];  // wq, then its inclusive scan, at pad16(k)
};

template <bool NORM, bool RS>
__device__ __attribute__((always_inline)) inline void weights_fused_filter(const WeightJob &J, FusedShared &sm) {
    float *shf = sm.f;
    double *shd = sm.d;
    uint64_t *shu = sm.u;
    uint64_t *C = sm.C;
    const int t = threadIdx.x;
    const int N = J.N;  // <= kWBlock
    if (NORM) {
        float v[kWPer];
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            const int n = i * kWThreads + t;
            v[i] = n < N ? J.logw[n] : -INFINITY;
        }
        float mx = -INFINITY;  // as lse_partial_kernel on block 0
#pragma unroll
        for (int i = 0; i < kWPer; ++i)
            if (i * kWThreads + t < N) mx = fmaxf(mx, v[i]);
        mx = block_tree(mx, shf, MaxF());
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < kWPer; ++i)
            if (i * kWThreads + t < N) s += exp((double)v[i] - (double)mx);
        s = block_tree(s, shd, AddD());
        // lse_reduce_kernel on one partial: its max is m_0 and its tree sum
        // adds zeros to 0 + S_0 exp(m_0 - m_0)
        const double m0 = (double)mx;
        double s0 = 0.0;
        s0 += s * exp(m0 - m0);
        const double lz = m0 + log(s0);
        if (t == 0 && J.log_z) J.log_z[0] = lz;
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {  // as weights_kernel
            const int n = i * kWThreads + t;
            const double wn = exp((double)v[i] - lz);
            const uint64_t q = (uint64_t)(wn * kWqScale);
            if (n < N) {
                if (J.w) J.w[n] = wn;
                J.wq[n] = q;
            }
            if (RS) C[pad16(n)] = n < N ? q : 0;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            const int n = i * kWThreads + t;
            C[pad16(n)] = n < N ? J.wq[n] : 0;
        }
    }
    if (RS) {
        __syncthreads();
        uint64_t run = 0;  // inclusive scan of this thread's 16 consecutive values
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            run += C[pad16(t * kWPer + i)];
            C[pad16(t * kWPer + i)] = run;
        }
        uint64_t T;
        const uint64_t excl = block_scan(run, shu, &T) - run;
#pragma unroll
        for (int i = 0; i < kWPer; ++i) C[pad16(t * kWPer + i)] += excl;
        __syncthreads();
        // ancestors of the slots m = i 256 + t as rs_search_kernel finds them
        // (the first i with C_i > y_m = floor((m T + r) / N); identity when
        // T = 0), by a branch-free search whose trip count depends on N alone.
        // y_m from one division per thread: with 256 T = Q N + R,
        // y_{m+256} = y_m + Q + [rem_m + R >= N].  Every m T + r of a slot
        // m < N is below N T < 2^64, and so is 256 T when N > 256; keys of
        // slots beyond N are unused and any key keeps the search in bounds.
        uint64_t y[kWPer];
        int at[kWPer];
        if (T != 0) {
            const uint64_t r = __umul64hi(J.u, T), n64 = (uint64_t)N;
            const uint64_t x0 = (uint64_t)t * T + r;
            uint64_t q = x0 / n64, rem = x0 - q * n64;
            uint64_t Q = 0, R = 0;
            if (N > kWThreads) {
                Q = ((uint64_t)kWThreads * T) / n64;
                R = (uint64_t)kWThreads * T - Q * n64;
            }
#pragma unroll
            for (int i = 0; i < kWPer; ++i) {
                y[i] = q;
                at[i] = 0;
                rem += R;
                const bool carry = rem >= n64;
                rem -= carry ? n64 : 0;
                q += Q + (carry ? 1 : 0);
            }
            for (int n = N; n > 1;) {  // the answer lies in [at, at + n); y < T = C_{N-1}
                const int half = n >> 1;
#pragma unroll
                for (int i = 0; i < kWPer; ++i) at[i] = C[pad16(at[i] + half - 1)] <= y[i] ? at[i] + half : at[i];
                n -= half;
            }
        } else {
#pragma unroll
            for (int i = 0; i < kWPer; ++i) at[i] = min(i * kWThreads + t, N - 1);
        }
        // every at[i] is in [0, N), so the loads need no guard; the stores
        // of slots beyond N are skipped
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            const int m = i * kWThreads + t;
            if (m < N) J.idx[m] = at[i];
        }
        if (J.pout) {
            // two batches of 8 slots, 96 loads in flight each; a batch with
            // no slot below N is skipped
#pragma unroll
            for (int i0 = 0; i0 < kWPer; i0 += 8) {
                if (i0 * kWThreads >= N) break;
                float p[8][12];
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const float *row = J.pin + (size_t)c * N;
#pragma unroll
                    for (int k = 0; k < 8; ++k) p[k][c] = load_at(row, (uint32_t)at[i0 + k] * 4u);
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int m = (i0 + k) * kWThreads + t;
                    if (m < N) {
#pragma unroll
                        for (int c = 0; c < 12; ++c) store_at(J.pout + (size_t)c * N, (uint32_t)m * 4u, p[k][c]);
                    }
                }
            }
        }
    }
}

template <typename S>
struct is_one_job : std::false_type {};
template <typename J>
struct is_one_job<OneJob<J>> : std::true_type {};

template <typename Src, bool NORM, bool RS>
__global__ __launch_bounds__(kWThreads) void weights_fused_kernel(Src src) {
    __shared__ FusedShared sm;
    if constexpr (is_one_job<Src>::value) {
        // one filter, no loop: nothing of it is held live across iterations
        if (blockIdx.x == 0) weights_fused_filter<NORM, RS>(src.get(0), sm);
    } else {
        for (int j = blockIdx.x; j < src.count(); j += gridDim.x) {
            weights_fused_filter<NORM, RS>(src.get(j), sm);
            __syncthreads();  // the next filter reuses the shared arrays
        }
    }
}

// ------------------------------------------------------------------ host side
// Filters of at most this many particles (one weight block at most) take the
// one-launch shape; mcl_set_weights_fused_max changes it.
static std::atomic<int> g_fused_max{kWBlock};

int weights_fused_max() { return g_fused_max.load(std::memory_order_relaxed); }

static unsigned grid_for(int64_t units, int per_cu) {
    int64_t g = std::min<int64_t>(units, (int64_t)device_cus() * per_cu);
    return (unsigned)std::max<int64_t>(g, 1);
}

template <typename Src>
mcl_status launch_normalize_src(const Src &src, int njobs, int64_t nblocks, int64_t nelems, hipStream_t stream) {
    lse_partial_kernel<<<grid_for(nblocks, 8), kWThreads, 0, stream>>>(src);
    mcl_status st = check_launch("lse_partial_kernel");
    if (st != MCL_OK) return st;
    lse_reduce_kernel<<<grid_for(njobs, 4), kWThreads, 0, stream>>>(src);
    if ((st = check_launch("lse_reduce_kernel")) != MCL_OK) return st;
    weights_kernel<<<grid_for((nelems + kWThreads - 1) / kWThreads, 16), kWThreads, 0, stream>>>(src);
    return check_launch("weights_kernel");
}

template <typename Src>
mcl_status launch_resample_src(const Src &src, int64_t nblocks, int64_t nelems, hipStream_t stream) {
    rs_blocksum_kernel<<<grid_for(nblocks, 8), kWThreads, 0, stream>>>(src);
    mcl_status st = check_launch("rs_blocksum_kernel");
    if (st != MCL_OK) return st;
    rs_scan_kernel<<<grid_for(nblocks, 4), kWThreads, 0, stream>>>(src);
    if ((st = check_launch("rs_scan_kernel")) != MCL_OK) return st;
    rs_search_kernel<<<grid_for((nelems + kWThreads - 1) / kWThreads, 16), kWThreads, 0, stream>>>(src);
    return check_launch("rs_search_kernel");
}

// One launch for `njobs` filters (a device count may be lower; surplus
// workgroups exit at once).
template <bool NORM, bool RS, typename Src>
mcl_status launch_weights_fused_src(const Src &src, int njobs, hipStream_t stream) {
    weights_fused_kernel<Src, NORM, RS><<<grid_for(njobs, 4), kWThreads, 0, stream>>>(src);
    return check_launch("weights_fused_kernel");
}

template mcl_status launch_weights_fused_src<true, true, JobTable<WeightJob>>(const JobTable<WeightJob> &, int,
                                                                              hipStream_t);
template mcl_status launch_weights_fused_src<true, false, JobTable<WeightJob>>(const JobTable<WeightJob> &, int,
                                                                               hipStream_t);
template mcl_status launch_weights_fused_src<false, true, JobTable<WeightJob>>(const JobTable<WeightJob> &, int,
                                                                               hipStream_t);
template mcl_status launch_normalize_src<OneJob<WeightJob>>(const OneJob<WeightJob> &, int, int64_t, int64_t,
                                                            hipStream_t);
template mcl_status launch_resample_src<OneJob<WeightJob>>(const OneJob<WeightJob> &, int64_t, int64_t, hipStream_t);
template mcl_status launch_normalize_src<JobTable<WeightJob>>(const JobTable<WeightJob> &, int, int64_t, int64_t,
                                                              hipStream_t);
template mcl_status launch_resample_src<JobTable<WeightJob>>(const JobTable<WeightJob> &, int64_t, int64_t,
                                                             hipStream_t);

// Workspace of one filter's weights stage: [2 nblk + 1] doubles, then
// [nblk + 1 + N] u64 (8-byte aligned pieces of one region).
size_t weight_ws_bytes(int N) {
    const int nb = weight_blocks(N);
    return (size_t)(2 * nb + 1) * sizeof(double) + (size_t)(nb + 1 + N) * sizeof(uint64_t);
}

void bind_weight_ws(WeightJob &J, void *ws) {
    const int nb = weight_blocks(J.N);
    double *d = static_cast<double *>(ws);
    J.lse_part = d;
    J.lz = d + 2 * nb;
    uint64_t *u = reinterpret_cast<uint64_t *>(d + 2 * nb + 1);
    J.bsum = u;
    J.total = u + nb;
    J.C = u + nb + 1;
    J.nblk = nb;
}

mcl_status launch_normalize(const float *logw, int N, double *w, uint64_t *wq, double *log_z, hipStream_t stream) {
    void *ws = workspace(stream, weight_ws_bytes(N));
    if (!ws) return fail(MCL_ENOMEM, "normalize: workspace allocation failed");
    OneJob<WeightJob> src{};
    src.n = Counts{1, 0, N, weight_blocks(N)};
    WeightJob &J = src.job;
    J.logw = logw;
    J.w = w;
    J.wq = wq;
    J.log_z = log_z;
    J.N = N;
    bind_weight_ws(J, ws);
    if (N <= weights_fused_max()) return launch_weights_fused_src<true, false>(src, 1, stream);
    return launch_normalize_src(src, 1, J.nblk, N, stream);
}

mcl_status launch_resample(const uint64_t *wq, int N, uint64_t u, int32_t *idx, const float *pin, float *pout,
                           hipStream_t stream) {
    void *ws = workspace(stream, weight_ws_bytes(N));
    if (!ws) return fail(MCL_ENOMEM, "resample: workspace allocation failed");
    OneJob<WeightJob> src{};
    src.n = Counts{1, 0, N, weight_blocks(N)};
    WeightJob &J = src.job;
    J.wq = const_cast<uint64_t *>(wq);
    J.u = u;
    J.idx = idx;
    J.pin = pin;
    J.pout = pout;
    J.N = N;
    bind_weight_ws(J, ws);
    if (N <= weights_fused_max()) return launch_weights_fused_src<false, true>(src, 1, stream);
    return launch_resample_src(src, J.nblk, N, stream);
}

}  // namespace mcl

using namespace mcl;

extern "C" mcl_status mcl_set_weights_fused_max(int32_t max_n) {
    if (max_n < 0 || max_n > kWBlock) return fail(MCL_ERANGE, "set_weights_fused_max: max_n must be in [0, 4096]");
    g_fused_max.store(max_n, std::memory_order_relaxed);
    return MCL_OK;
}

extern "C" int32_t mcl_get_weights_fused_max(void) { return weights_fused_max(); }

namespace mcl {

}  // namespace mcl

// Weight normalisation (float64 log-sum-exp, §V-A) and low-variance resampling
// on 64-bit fixed-point weights (§III), for one filter or a batch of filters.
// Every reduction runs in a fixed order (no atomics), so results are
// reproducible bit for bit and identical whether a filter runs alone or in a
// batch.  Blocks of 4096 particles are the unit of work; a launch strides
// over the (filter, block) pairs of all its filters.
#include <algorithm>

#include "jobs.h"

namespace mcl {

constexpr double kWqScale = 4398046511104.0;  // 2^42

// Fixed-order tree over the block (thread t adds t + stride).
template <typename V, typename Op>
__device__ inline V block_tree(V x, V *sh, Op op) {
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
#pragma unroll
    for (int st = kWThreads / 2; st > 0; st >>= 1) {
        if (t < st) sh[t] = op(sh[t], sh[t + st]);
        __syncthreads();
    }
    V r = sh[0];
    __syncthreads();
    return r;
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
    __shared__ uint64_t vals[kWBlock];
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
            vals[i * kWThreads + t] = n < J.N ? J.wq[n] : 0;
        }
        __syncthreads();
        uint64_t run = 0;
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            run += vals[t * kWPer + i];
            vals[t * kWPer + i] = run;
        }
        sh[t] = run;
        __syncthreads();
        for (int d = 1; d < kWThreads; d <<= 1) {  // inclusive scan of the per-thread totals
            uint64_t add = t >= d ? sh[t - d] : 0;
            __syncthreads();
            sh[t] += add;
            __syncthreads();
        }
        const uint64_t excl = pre + sh[t] - run;
#pragma unroll
        for (int i = 0; i < kWPer; ++i) vals[t * kWPer + i] += excl;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            int n = base + i * kWThreads + t;
            if (n < J.N) J.C[n] = vals[i * kWThreads + t];
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

// ------------------------------------------------------------------ host side
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
    return launch_resample_src(src, J.nblk, N, stream);
}

}  // namespace mcl

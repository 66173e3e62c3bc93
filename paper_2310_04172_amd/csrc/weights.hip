// Weight normalisation (float64 log-sum-exp, §V-A) and low-variance resampling
// on 64-bit fixed-point weights (§III).  Every reduction runs in a fixed order
// (no atomics), so results are reproducible bit for bit.
#include "mcl_internal.h"

namespace mcl {

constexpr int kThreads = 256;
constexpr int kPer = 16;
constexpr int kBlockElems = kThreads * kPer;  // 4096 elements per block
constexpr double kWqScale = 4398046511104.0;  // 2^42

int weight_blocks(int N) { return (N + kBlockElems - 1) / kBlockElems; }

// Fixed-order tree over the block (thread t adds t + stride).
template <typename V, typename Op>
__device__ inline V block_tree(V x, V *sh, Op op) {
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
#pragma unroll
    for (int st = kThreads / 2; st > 0; st >>= 1) {
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

// Per block: m_b = max l, S_b = sum exp(l - m_b).
__global__ __launch_bounds__(kThreads) void lse_partial_kernel(const float *__restrict__ logw, int N,
                                                               double *__restrict__ part) {
    __shared__ float shf[kThreads];
    __shared__ double shd[kThreads];
    const int base = blockIdx.x * kBlockElems + threadIdx.x;
    float mx = -INFINITY;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        int n = base + i * kThreads;
        if (n < N) mx = fmaxf(mx, logw[n]);
    }
    mx = block_tree(mx, shf, MaxF());
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        int n = base + i * kThreads;
        if (n < N) s += exp((double)logw[n] - (double)mx);
    }
    s = block_tree(s, shd, AddD());
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = (double)mx;
        part[2 * blockIdx.x + 1] = s;
    }
}

// One block: log Z = m + log sum_b S_b exp(m_b - m).
__global__ __launch_bounds__(kThreads) void lse_reduce_kernel(const double *__restrict__ part, int nb,
                                                              double *__restrict__ lz_ws, double *__restrict__ log_z) {
    __shared__ double shd[kThreads];
    double mx = -INFINITY;
    for (int b = threadIdx.x; b < nb; b += kThreads) mx = fmax(mx, part[2 * b]);
    mx = block_tree(mx, shd, MaxD());
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) s += part[2 * b + 1] * exp(part[2 * b] - mx);
    s = block_tree(s, shd, AddD());
    if (threadIdx.x == 0) {
        double lz = mx + log(s);
        lz_ws[0] = lz;
        if (log_z) log_z[0] = lz;
    }
}

__global__ __launch_bounds__(kThreads) void weights_kernel(const float *__restrict__ logw, int N,
                                                           const double *__restrict__ lz_ws, double *__restrict__ w,
                                                           uint64_t *__restrict__ wq) {
    int n = blockIdx.x * kThreads + threadIdx.x;
    if (n >= N) return;
    const double lz = lz_ws[0];
    double wn = exp((double)logw[n] - lz);
    if (w) w[n] = wn;
    wq[n] = (uint64_t)(wn * kWqScale);  // w >= 0: truncation is floor; scaling by 2^42 is exact
}

// ---------------------------------------------------------------- resampling
__global__ __launch_bounds__(kThreads) void rs_blocksum_kernel(const uint64_t *__restrict__ wq, int N,
                                                               uint64_t *__restrict__ bsum) {
    __shared__ uint64_t sh[kThreads];
    const int base = blockIdx.x * kBlockElems + threadIdx.x;
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        int n = base + i * kThreads;
        if (n < N) s += wq[n];
    }
    s = block_tree(s, sh, AddU());
    if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

// Inclusive scan C of wq: block prefix from the block sums, then a scan of the
// block's 4096 values staged in LDS.  Block 0 also writes the total T.
__global__ __launch_bounds__(kThreads) void rs_scan_kernel(const uint64_t *__restrict__ wq, int N,
                                                           const uint64_t *__restrict__ bsum, int nb,
                                                           uint64_t *__restrict__ C, uint64_t *__restrict__ total) {
    __shared__ uint64_t vals[kBlockElems];
    __shared__ uint64_t sh[kThreads];
    const int t = threadIdx.x;
    const int b = blockIdx.x;
    uint64_t pre = 0, tot = 0;
    for (int j = t; j < nb; j += kThreads) {
        uint64_t v = bsum[j];
        tot += v;
        if (j < b) pre += v;
    }
    pre = block_tree(pre, sh, AddU());
    tot = block_tree(tot, sh, AddU());
    const int base = b * kBlockElems;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        int n = base + i * kThreads + t;
        vals[i * kThreads + t] = n < N ? wq[n] : 0;
    }
    __syncthreads();
    uint64_t run = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        run += vals[t * kPer + i];
        vals[t * kPer + i] = run;
    }
    // inclusive Hillis-Steele scan of the per-thread totals
    sh[t] = run;
    __syncthreads();
    for (int d = 1; d < kThreads; d <<= 1) {
        uint64_t add = t >= d ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const uint64_t excl = pre + sh[t] - run;
#pragma unroll
    for (int i = 0; i < kPer; ++i) vals[t * kPer + i] += excl;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        int n = base + i * kThreads + t;
        if (n < N) C[n] = vals[i * kThreads + t];
    }
    if (b == 0 && t == 0) total[0] = tot;
}

// Output slot m: x = m T + r; the ancestor is the first i with N C_i > x, i.e.
// C_i > floor(x / N) (C_i is an integer).  Found by binary search; since
// x < N T, i exists.  Then the pose is gathered.
__global__ __launch_bounds__(kThreads) void rs_search_kernel(const uint64_t *__restrict__ C, int N,
                                                             const uint64_t *__restrict__ total, uint64_t u,
                                                             int32_t *__restrict__ idx, const float *__restrict__ pin,
                                                             float *__restrict__ pout) {
    int m = blockIdx.x * kThreads + threadIdx.x;
    if (m >= N) return;
    const uint64_t T = total[0];
    int i;
    if (T == 0) {
        i = m;
    } else {
        const uint64_t r = __umul64hi(u, T);
        const uint64_t x = (uint64_t)m * T + r;
        const uint64_t y = x / (uint64_t)N;
        int lo = 0, hi = N - 1;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (C[mid] > y) hi = mid;
            else lo = mid + 1;
        }
        i = lo;
    }
    idx[m] = i;
    if (pout) {
#pragma unroll
        for (int j = 0; j < 12; ++j) pout[(size_t)j * N + m] = pin[(size_t)j * N + i];
    }
}

// ------------------------------------------------------------------ host side
mcl_status launch_normalize(const float *logw, int N, double *w, uint64_t *wq, double *log_z, hipStream_t stream) {
    const int nb = weight_blocks(N);
    double *ws = static_cast<double *>(workspace(stream, (size_t)(2 * nb + 2) * sizeof(double)));
    if (!ws) return fail(MCL_ENOMEM, "normalize: workspace allocation failed");
    double *part = ws, *lz = ws + 2 * nb;
    lse_partial_kernel<<<nb, kThreads, 0, stream>>>(logw, N, part);
    mcl_status st = check_launch("lse_partial_kernel");
    if (st != MCL_OK) return st;
    lse_reduce_kernel<<<1, kThreads, 0, stream>>>(part, nb, lz, log_z);
    if ((st = check_launch("lse_reduce_kernel")) != MCL_OK) return st;
    weights_kernel<<<(N + kThreads - 1) / kThreads, kThreads, 0, stream>>>(logw, N, lz, w, wq);
    return check_launch("weights_kernel");
}

mcl_status launch_resample(const uint64_t *wq, int N, uint64_t u, int32_t *idx, const float *pin, float *pout,
                           hipStream_t stream) {
    const int nb = weight_blocks(N);
    uint64_t *ws = static_cast<uint64_t *>(workspace(stream, (size_t)(nb + 2 + N) * sizeof(uint64_t)));
    if (!ws) return fail(MCL_ENOMEM, "resample: workspace allocation failed");
    uint64_t *bsum = ws, *total = ws + nb, *C = ws + nb + 2;
    rs_blocksum_kernel<<<nb, kThreads, 0, stream>>>(wq, N, bsum);
    mcl_status st = check_launch("rs_blocksum_kernel");
    if (st != MCL_OK) return st;
    rs_scan_kernel<<<nb, kThreads, 0, stream>>>(wq, N, bsum, nb, C, total);
    if ((st = check_launch("rs_scan_kernel")) != MCL_OK) return st;
    rs_search_kernel<<<(N + kThreads - 1) / kThreads, kThreads, 0, stream>>>(C, N, total, u, idx, pin, pout);
    return check_launch("rs_search_kernel");
}

}  // namespace mcl

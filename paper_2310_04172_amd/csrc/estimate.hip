// Pose estimate of a weighted particle set (§III: the estimate is the weighted
// average of the particles or the particle of highest weight; §V: a second GPU
// reduction forms the weighted sum of the poses).
//
//   position  t* = sum_n w_n t_n / sum_n w_n
//   rotation  R* = the rotation closest to S = sum_n w_n R_n, i.e. the maximiser
//             of trace(R^T S) over SO(3): the weighted chordal L2 mean of the
//             particle rotations (for exact rotations the same rotation as the
//             eigenvector quaternion average of Markley et al. 2007).  Found as
//             the unit quaternion q maximising q^T K q, K the symmetric 4x4
//             matrix whose quadratic form is trace(R(q)^T S) (Horn 1987), by
//             cyclic Jacobi rotations.
//   best      the smallest index of the largest weight, and that particle's pose.
//   sum w = 0 is read as equal weights.
//
// Float64 sums in a fixed order: each thread adds its particles in index order
// (4 per step, strided by the block size so loads coalesce; steps strided by
// the grid, at most 256 blocks of 1024 particles), then a wave tree, then the 4
// waves in order; the final block adds the block partials (stored
// accumulator-major, so its loads coalesce) the same way.
#include <algorithm>
#include <cmath>

#include "jobs.h"

namespace mcl {

constexpr int kEThreads = 256;
constexpr int kEPer = 4;
constexpr int kEBlock = kEThreads * kEPer;
// At most this many blocks; a block strides over the particle set in steps of
// the grid (the grid, and so the summation order, depends on N alone).
constexpr int kEMaxBlocks = 256;
constexpr int kEWaves = kEThreads / 64;
// accumulators: sum w | sum w t (3) | sum w R (9) | sum t (3) | sum R (9)
constexpr int kEAcc = 25;

struct Best {
    double w;
    int i;
};

// larger weight wins; among equal weights the smaller index
__device__ inline Best better(Best a, Best b) { return (b.w > a.w || (b.w == a.w && b.i < a.i)) ? b : a; }

// Sum of acc[] over the block (lane tree, then waves 0..3 in order) and the
// block's best; valid in thread 0 (sums also in tot[] for threads < kEAcc).
__device__ inline void block_reduce(double acc[kEAcc], Best &b, double (*red)[kEAcc], Best *rb, double *tot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int a = 0; a < kEAcc; ++a) acc[a] += __shfl_down(acc[a], off, 64);
        Best o{__shfl_down(b.w, off, 64), __shfl_down(b.i, off, 64)};
        if (lane + off < 64) b = better(b, o);
    }
    if (lane == 0) {
#pragma unroll
        for (int a = 0; a < kEAcc; ++a) red[wave][a] = acc[a];
        rb[wave] = b;
    }
    __syncthreads();
    if (threadIdx.x < kEAcc) {
        double s = red[0][threadIdx.x];
        for (int v = 1; v < kEWaves; ++v) s += red[v][threadIdx.x];
        tot[threadIdx.x] = s;
    }
    if (threadIdx.x == 0) {
        Best r = rb[0];
        for (int v = 1; v < kEWaves; ++v) r = better(r, rb[v]);
        rb[0] = r;
    }
    __syncthreads();
    b = rb[0];
}

// Block b of the launch works for the job whose blocks [blk0, blk0 + nblk) hold
// b; its particles are those of index local + k nblk (in blocks of kEBlock).
template <typename Src>
__global__ __launch_bounds__(kEThreads) void estimate_partial_kernel(Src src) {
    __shared__ double red[kEWaves][kEAcc];
    __shared__ Best rb[kEWaves];
    __shared__ double tot[kEAcc];
    const int blk = blockIdx.x;
    if (blk >= src.blocks()) return;  // surplus blocks of a replayed launch
    const EstJob J = src.load(find_job_uniform(src, blk, [](const EstJob &e) { return (int64_t)e.blk0; }));
    const int local = blk - J.blk0, N = J.N;
    const double *__restrict__ w = J.w;
    const float *__restrict__ poses = J.poses;
    double acc[kEAcc];
#pragma unroll
    for (int a = 0; a < kEAcc; ++a) acc[a] = 0.0;
    Best b{-INFINITY, 0x7fffffff};
    for (int base = local * kEBlock + threadIdx.x; base < N; base += J.nblk * kEBlock) {
        double wv[kEPer];
        float pv[kEPer][12];
#pragma unroll
        for (int i = 0; i < kEPer; ++i) {
            const int n = base + i * kEThreads;
            wv[i] = 0.0;
#pragma unroll
            for (int j = 0; j < 12; ++j) pv[i][j] = 0.0f;
            if (n < N) {
                wv[i] = w[n];
#pragma unroll
                for (int j = 0; j < 12; ++j) pv[i][j] = poses[(size_t)j * N + n];
            }
        }
#pragma unroll
        for (int i = 0; i < kEPer; ++i) {
            const int n = base + i * kEThreads;
            if (n < N) {
                const double wn = wv[i];
                acc[0] += wn;
#pragma unroll
                for (int j = 0; j < 3; ++j) acc[1 + j] += wn * (double)pv[i][9 + j];
#pragma unroll
                for (int j = 0; j < 9; ++j) acc[4 + j] += wn * (double)pv[i][j];
#pragma unroll
                for (int j = 0; j < 3; ++j) acc[13 + j] += (double)pv[i][9 + j];
#pragma unroll
                for (int j = 0; j < 9; ++j) acc[16 + j] += (double)pv[i][j];
                if (wn > b.w) b = Best{wn, n};  // n grows along the loops: a later equal weight never wins
            }
        }
    }
    block_reduce(acc, b, red, rb, tot);
    if (threadIdx.x < kEAcc) J.part[(size_t)threadIdx.x * J.nblk + local] = tot[threadIdx.x];
    if (threadIdx.x == 0) static_cast<Best *>(J.pbest)[local] = b;
}

// 1/x and 1/sqrt(x) for x > 0 normal: the hardware estimates refined by two
// Newton steps each (error a few ulps; the rotations below only need to be
// orthogonal to working precision, not to zero an entry exactly).
__device__ inline double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ inline double rsq_nr(double x) {
    double r = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    r = r * fma(-h * r, r, 1.5);
    return r * fma(-h * r, r, 1.5);
}

// Off-diagonal entries at most this large (the matrix scaled so that its
// largest entry lies in [1, 2)) count as zero: a few units of rounding, the
// level the rotations themselves leave behind.
constexpr double kJacobiTol = 0x1p-50;

// Rotation (c, s) of the plane (p, q) that zeroes the entry apq of a symmetric
// matrix (Golub and Van Loan §8.5.2, with t = tan written as
// sign(d) e / (|d| + sqrt(d^2 + e^2)), d = aqq - app, e = 2 apq); the identity
// when apq is negligible.  Entries are scaled to at most 2 in magnitude.
__device__ inline void jacobi_cs(double app, double aqq, double apq, double &c, double &s) {
    if (fabs(apq) <= kJacobiTol) {
        c = 1.0;
        s = 0.0;
        return;
    }
    const double d = aqq - app, e = 2.0 * apq;
    const double q = fma(d, d, e * e);
    const double h = q * rsq_nr(q);
    const double t = (d >= 0.0 ? e : -e) * rcp_nr(fabs(d) + h);
    c = rsq_nr(fma(t, t, 1.0));
    s = t * c;
}

// A <- J^T A J and V <- V J for the rotations of the disjoint planes (p1, q1)
// and (p2, q2); J(p,p) = J(q,q) = c, J(p,q) = s, J(q,p) = -s.
template <int P1, int Q1, int P2, int Q2>
__device__ inline void jacobi_pair(double (&A)[4][4], double (&V)[4][4]) {
    double c1, s1, c2, s2;
    jacobi_cs(A[P1][P1], A[Q1][Q1], A[P1][Q1], c1, s1);
    jacobi_cs(A[P2][P2], A[Q2][Q2], A[P2][Q2], c2, s2);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double a1 = A[k][P1], b1 = A[k][Q1], a2 = A[k][P2], b2 = A[k][Q2];
        A[k][P1] = c1 * a1 - s1 * b1;
        A[k][Q1] = s1 * a1 + c1 * b1;
        A[k][P2] = c2 * a2 - s2 * b2;
        A[k][Q2] = s2 * a2 + c2 * b2;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double a1 = A[P1][k], b1 = A[Q1][k], a2 = A[P2][k], b2 = A[Q2][k];
        A[P1][k] = c1 * a1 - s1 * b1;
        A[Q1][k] = s1 * a1 + c1 * b1;
        A[P2][k] = c2 * a2 - s2 * b2;
        A[Q2][k] = s2 * a2 + c2 * b2;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double a1 = V[k][P1], b1 = V[k][Q1], a2 = V[k][P2], b2 = V[k][Q2];
        V[k][P1] = c1 * a1 - s1 * b1;
        V[k][Q1] = s1 * a1 + c1 * b1;
        V[k][P2] = c2 * a2 - s2 * b2;
        V[k][Q2] = s2 * a2 + c2 * b2;
    }
}

// Eigenvector of the largest eigenvalue of a symmetric 4x4 matrix by Jacobi
// rotations (Golub and Van Loan §8.5) in the parallel ordering of Brent and Luk
// (the six planes as three pairs of disjoint planes, whose two rotations are
// independent), after scaling by a power of two so that the largest entry lies
// in [1, 2).  Sweeps until every off-diagonal entry is negligible, at most 10
// (4x4 needs 3 or 4: the method converges quadratically down to the rounding
// level).
struct Quat {
    double w, x, y, z;
};

__device__ inline Quat sym4_top_eigvec(double (&A)[4][4]) {
    double mx = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) mx = fmax(mx, fabs(A[r][c]));
    if (!(mx > 0.0) || !(mx < INFINITY)) return Quat{1.0, 0.0, 0.0, 0.0};  // zero (or not finite)
    const int ex = ilogb(mx);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) A[r][c] = ldexp(A[r][c], -ex);
    double V[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) V[r][c] = r == c ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 10; ++sweep) {
        bool done = true;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = p + 1; q < 4; ++q)
                done = done && fabs(A[p][q]) <= kJacobiTol;
        if (done) break;
        jacobi_pair<0, 1, 2, 3>(A, V);
        jacobi_pair<0, 2, 1, 3>(A, V);
        jacobi_pair<0, 3, 1, 2>(A, V);
    }
    int m = 0;
#pragma unroll
    for (int k = 1; k < 4; ++k)
        if (A[k][k] > A[m][m]) m = k;
    double col[4], nrm = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        col[k] = m == 0 ? V[k][0] : m == 1 ? V[k][1] : m == 2 ? V[k][2] : V[k][3];
        nrm = fma(col[k], col[k], nrm);
    }
    nrm = sqrt(nrm);
    return Quat{col[0] / nrm, col[1] / nrm, col[2] / nrm, col[3] / nrm};
}

// One block per job: the job's block partials, then the estimate.
template <typename Src>
__global__ __launch_bounds__(kEThreads) void estimate_final_kernel(Src src) {
    __shared__ double red[kEWaves][kEAcc];
    __shared__ Best rb[kEWaves];
    __shared__ double tot[kEAcc];
    if ((int)blockIdx.x >= src.count()) return;
    const EstJob J = src.load(blockIdx.x);
    const int nb = J.nblk, N = J.N;
    const double *__restrict__ part = J.part;
    const Best *__restrict__ pbest = static_cast<const Best *>(J.pbest);
    const float *__restrict__ poses = J.poses;
    double *__restrict__ mean = J.mean;
    int32_t *__restrict__ best_idx = J.best_idx;
    float *__restrict__ best_pose = J.best_pose;
    double acc[kEAcc];
#pragma unroll
    for (int a = 0; a < kEAcc; ++a) acc[a] = 0.0;
    Best b{-INFINITY, 0x7fffffff};
    for (int k = threadIdx.x; k < nb; k += kEThreads) {
#pragma unroll
        for (int a = 0; a < kEAcc; ++a) acc[a] += part[(size_t)a * nb + k];
        b = better(b, pbest[k]);
    }
    block_reduce(acc, b, red, rb, tot);
    const bool found = b.i != 0x7fffffff;
    if (threadIdx.x < 12 && best_pose)
        best_pose[threadIdx.x] = found ? poses[(size_t)threadIdx.x * N + b.i] : NAN;
    if (threadIdx.x != 0) return;
    if (best_idx) best_idx[0] = found ? b.i : -1;
    const bool weighted = tot[0] > 0.0;
    const double *ts = weighted ? tot + 1 : tot + 13;
    const double *S = weighted ? tot + 4 : tot + 16;
    const double den = weighted ? tot[0] : (double)N;
    // trace(R(q)^T S) = q^T K q for q = (w, x, y, z)
    double K[4][4];
    K[0][0] = S[0] + S[4] + S[8];
    K[1][1] = S[0] - S[4] - S[8];
    K[2][2] = -S[0] + S[4] - S[8];
    K[3][3] = -S[0] - S[4] + S[8];
    K[0][1] = K[1][0] = S[7] - S[5];
    K[0][2] = K[2][0] = S[2] - S[6];
    K[0][3] = K[3][0] = S[3] - S[1];
    K[1][2] = K[2][1] = S[1] + S[3];
    K[1][3] = K[3][1] = S[2] + S[6];
    K[2][3] = K[3][2] = S[5] + S[7];
    const Quat q = sym4_top_eigvec(K);
    const double qw = q.w, x = q.x, y = q.y, z = q.z;
    mean[0] = qw * qw + x * x - y * y - z * z;
    mean[1] = 2.0 * (x * y - qw * z);
    mean[2] = 2.0 * (x * z + qw * y);
    mean[3] = 2.0 * (x * y + qw * z);
    mean[4] = qw * qw - x * x + y * y - z * z;
    mean[5] = 2.0 * (y * z - qw * x);
    mean[6] = 2.0 * (x * z - qw * y);
    mean[7] = 2.0 * (y * z + qw * x);
    mean[8] = qw * qw - x * x - y * y + z * z;
    for (int j = 0; j < 3; ++j) mean[9 + j] = ts[j] / den;
}

int estimate_blocks(int N) { return std::min((N + kEBlock - 1) / kEBlock, kEMaxBlocks); }

size_t estimate_ws_bytes(int N) {
    const size_t nb = estimate_blocks(N);
    return nb * kEAcc * sizeof(double) + nb * sizeof(Best);
}

void bind_estimate_ws(EstJob &J, void *ws) {
    J.nblk = estimate_blocks(J.N);
    J.part = static_cast<double *>(ws);
    J.pbest = J.part + (size_t)J.nblk * kEAcc;
}

template <typename Src>
mcl_status launch_estimate_src(const Src &src, int64_t blocks, int64_t jobs, hipStream_t stream) {
    estimate_partial_kernel<Src><<<(unsigned)blocks, kEThreads, 0, stream>>>(src);
    mcl_status st = check_launch("estimate_partial_kernel");
    if (st != MCL_OK) return st;
    estimate_final_kernel<Src><<<(unsigned)jobs, kEThreads, 0, stream>>>(src);
    return check_launch("estimate_final_kernel");
}

template mcl_status launch_estimate_src<JobTable<EstJob>>(const JobTable<EstJob> &, int64_t, int64_t, hipStream_t);

mcl_status launch_estimate(const double *w, const float *poses, int N, double *mean, int32_t *best_idx,
                           float *best_pose, hipStream_t stream) {
    char *ws = static_cast<char *>(workspace(stream, estimate_ws_bytes(N)));
    if (!ws) return fail(MCL_ENOMEM, "pose_estimate: workspace allocation failed");
    EstJob J{};
    J.w = w;
    J.poses = poses;
    J.mean = mean;
    J.best_idx = best_idx;
    J.best_pose = best_pose;
    J.N = N;
    bind_estimate_ws(J, ws);
    OneJob<EstJob> one{J, Counts{1, 0, N, J.nblk}};
    return launch_estimate_src(one, J.nblk, 1, stream);
}

}  // namespace mcl

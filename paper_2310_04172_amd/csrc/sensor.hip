// Sensor update (§III, Eq. 3, endpoint model): for every particle, transform
// every scan point by the particle pose, read the TSDF value of the voxel that
// holds it, and sum the squared values; l_n = -c * sum, c = s^2 / (2 sigma^2).
//
// Work decomposition (gfx950, 64-lane waves):
//  * a wave owns a group of up to 64 particles, or a run of them when the
//    launch has few groups; lane p keeps particle p's pose constants in 12
//    registers and its running sum;
//  * the scan is cut into chunks of 1024 points; a wave loads a chunk into
//    registers (16 points per lane, lane l holding points l, l+64, ...), then for
//    each particle of its run broadcasts that pose to scalar registers and
//    evaluates the 16 points of every lane: 16 independent gathers in flight;
//  * neighbouring lanes hold neighbouring beams, so one wave-wide gather touches
//    few 128-byte lines of the flat bricks of the map;
//  * a chunk's 64 lane sums are reduced across the wave in a fixed pairwise tree;
//  * the scan is also split into pieces of 4 chunks (4096 points) so small
//    particle counts still fill the GPU; pieces are combined pairwise;
//  * a large launch visits the particles in spatial order (sorted by map cell
//    as their pose constants are written), and each die of the chip takes
//    consecutive work items, so lookups made together share cache lines; each
//    log-weight goes back to its particle's index.
// The summation order is a function of K only (lane partials of 16 terms,
// 6-level wave tree, 4 chunks per piece in order, pairwise over pieces): the
// same particle gives the same bits whatever N, grid or batch it runs in.
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "jobs.h"
#include "voxel.h"

namespace mcl {

__device__ inline float bcast(float x, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

// Sum over the 64 lanes without LDS, in a fixed pairwise tree: DPP quad
// permutations (xor 1, xor 2) and the half-row and row mirrors (pairing lane i
// with 7-i, 15-i once the groups below are uniform) leave every lane of row i
// with its row's sum r_i; then each row adds the previous row's lane 15 (row 3
// gets r2 + r3) and rows 2 and 3 add lane 31 (row 1's r0 + r1), so lane 63
// holds (r0 + r1) + (r2 + r3), which is read into a scalar register.  IEEE
// addition is commutative, so the order of a pair's operands does not matter;
// rows other than row 3 end with partial or zero-filled sums that are never read.
template <int CTRL>
__device__ inline float dpp_add(float x) {
    return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

__device__ inline float wave_sum(float x) {
    x = dpp_add<0xB1>(x);   // quad_perm [1,0,3,2]
    x = dpp_add<0x4E>(x);   // quad_perm [2,3,0,1]
    x = dpp_add<0x141>(x);  // row_half_mirror
    x = dpp_add<0x140>(x);  // row_mirror
    x = dpp_add<0x142>(x);  // row_bcast:15
    x = dpp_add<0x143>(x);  // row_bcast:31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Raw map value as a 32-bit register (sign-extended integer or float bits).
template <typename T>
__device__ inline int load_raw(const char *base, uint32_t off) {
    if constexpr (sizeof(T) == 4)
        return __float_as_int(*gp(reinterpret_cast<const float *>(base + off)));
    else
        return (int)*gp(reinterpret_cast<const T *>(base + off));
}

template <typename T>
__device__ inline float as_value(int raw) {
    if constexpr (sizeof(T) == 4)
        return __int_as_float(raw);
    else
        return (float)raw;
}

template <typename T>
constexpr int class_shift() { return kBrickLog2 + (sizeof(T) == 1 ? 0 : sizeof(T) == 2 ? 1 : 2); }

// A lane's partial score over its kU values, in point order.  Product reading:
// sum q^2 (one fused multiply-add per point).  Sum reading: sum 2^(k2 q^2), the
// points' likelihoods exp(-c q^2) by the hardware base-2 exponential (k2 q^2
// lies in [k2 Q^2, 0], which the library keeps above -47, so every term is a
// normal float); padding slots of a ragged chunk read 0 and add nothing in
// either reading.
template <bool TAIL, bool SUM, typename T>
__device__ __attribute__((always_inline)) inline float lane_score(const int (&raw)[kU], int lane, int nvalid,
                                                                  float k2) {
    float s = 0.0f;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        float f = as_value<T>(raw[u]);
        if constexpr (SUM) {
            float e = __builtin_amdgcn_exp2f((f * f) * k2);
            if (TAIL) e = (u * kWave + lane < nvalid) ? e : 0.0f;
            s = s + e;
        } else {
            s = __builtin_fmaf(f, f, s);
        }
    }
    return s;
}

// Lane partial sum of one particle (pose in A) over this lane's kU points.
// Coarse level first: the read mask of each point's brick (a signed byte in
// global memory): a brick wholly at +-Q reads offset 0, the +Q sentinel, so
// only points in bricks with values inside the truncation band read their own
// value; a gather then touches one shared line for all the others, needs no
// branches, and all kU gathers stay in flight.  Padding lanes point at the
// zero sentinel brick, which is read in place.
template <typename T, bool TAIL, bool SUM>
__device__ __attribute__((always_inline)) inline float lane_chunk_sum(const MapView &m, const float (&A)[12], const float (&px)[kU],
                                       const float (&py)[kU], const float (&pz)[kU], int lane, int nvalid,
                                       float k2, bool count = false, int *nmixed = nullptr) {
    uint32_t off[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        float gx = grid_coord(A[0], A[1], A[2], A[9], px[u], py[u], pz[u]);
        float gy = grid_coord(A[3], A[4], A[5], A[10], px[u], py[u], pz[u]);
        float gz = grid_coord(A[6], A[7], A[8], A[11], px[u], py[u], pz[u]);
        uint32_t o = voxel_offset<sizeof(T)>(m, gx, gy, gz);
        if (TAIL) o = (u * kWave + lane < nvalid) ? o : m.zero_off;
        off[u] = o;
    }
    int msk[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) msk[u] = gp(m.mask)[off[u] >> class_shift<T>()];
    __builtin_amdgcn_sched_barrier(0);
    int raw[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) raw[u] = load_raw<T>(m.base, off[u] & (uint32_t)msk[u]);
    __builtin_amdgcn_sched_barrier(0);
    if (count) {
        // lookups of the wave that read in place (wave-uniform)
        int c = 0;
#pragma unroll
        for (int u = 0; u < kU; ++u) c += __builtin_popcountll(__ballot(msk[u] != 0));
        *nmixed += c;
    }
    return lane_score<TAIL, SUM, T>(raw, lane, nvalid, k2);
}

// The same lookup with the coarse level read from LDS: the workgroup holds the
// map's read masks as bits, so a point costs one global gather instead of two
// (and three more instructions).  The bit of slot b sign-extended is the mask
// (0 or -1).  All 16 LDS reads are issued before the first gather.
template <typename T, bool TAIL, bool SUM>
__device__ __attribute__((always_inline)) inline float lane_chunk_sum_lds(const MapView &m, const uint32_t *sbits,
                                                                          const float (&A)[12], const float (&px)[kU],
                                                                          const float (&py)[kU], const float (&pz)[kU],
                                                                          int lane, int nvalid, float k2) {
    uint32_t off[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        float gx = grid_coord(A[0], A[1], A[2], A[9], px[u], py[u], pz[u]);
        float gy = grid_coord(A[3], A[4], A[5], A[10], px[u], py[u], pz[u]);
        float gz = grid_coord(A[6], A[7], A[8], A[11], px[u], py[u], pz[u]);
        uint32_t o = voxel_offset<sizeof(T)>(m, gx, gy, gz);
        if (TAIL) o = (u * kWave + lane < nvalid) ? o : m.zero_off;
        off[u] = o;
    }
    uint32_t word[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) word[u] = sbits[off[u] >> (class_shift<T>() + 5)];
    __builtin_amdgcn_sched_barrier(0);
    int raw[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        // bit (slot & 31), sign-extended: the mask
        const int mk = __builtin_amdgcn_sbfe((int)word[u], (int)(off[u] >> class_shift<T>()), 1);
        raw[u] = load_raw<T>(m.base, off[u] & (uint32_t)mk);
    }
    __builtin_amdgcn_sched_barrier(0);
    return lane_score<TAIL, SUM, T>(raw, lane, nvalid, k2);
}

// Trilinear lookup (§III: a pseudo-continuous map value by interpolation): one
// gather of the point's corner cell (the 8 voxel values around it; corners
// outside the map hold +Q; cells of bricks wholly at +Q or wholly at -Q read
// the shared +Q sentinel after a read-mask lookup), interpolated along x, then y, then z by
// lerp(a, b, t) = fma(t, b - a, a) in float32.  A point clamped to h = -1 has
// weight 0 on its inside corner and a point clamped to h = n reads two +Q
// corners, so both give exactly Q.  Padding slots contribute 0.  Points go in
// batches of kTriU, whose gathers are all in flight together.
constexpr int kTriU = 8;

__device__ inline float lerp(float a, float b, float t) { return __builtin_fmaf(t, b - a, a); }

template <typename T>
struct CellRaw;
template <>
struct CellRaw<int16_t> {
    uint4 q;
};
template <>
struct CellRaw<int8_t> {
    uint2 q;
};
template <>
struct CellRaw<float> {
    float4 a, b;
};

// clang vector types (the HIP vector structs do not load through
// address-space-qualified pointers)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ inline CellRaw<T> load_cell(const char *base, uint32_t off) {
    CellRaw<T> r;
    if constexpr (sizeof(T) == 2) {
        const u32x4 v = *gp(reinterpret_cast<const u32x4 *>(base + off));
        r.q = make_uint4(v.x, v.y, v.z, v.w);
    } else if constexpr (sizeof(T) == 1) {
        const u32x2 v = *gp(reinterpret_cast<const u32x2 *>(base + off));
        r.q = make_uint2(v.x, v.y);
    } else {
        const f32x4 a = *gp(reinterpret_cast<const f32x4 *>(base + off));
        const f32x4 b = *gp(reinterpret_cast<const f32x4 *>(base + off + 16));
        r.a = make_float4(a.x, a.y, a.z, a.w);
        r.b = make_float4(b.x, b.y, b.z, b.w);
    }
    return r;
}

// The 8 corner values as floats, corner a + 2 b + 4 c (sign-extended fields).
template <typename T>
__device__ inline void unpack_cell(const CellRaw<T> &r, float (&d)[8]) {
    if constexpr (sizeof(T) == 2) {
        const uint32_t w[4] = {r.q.x, r.q.y, r.q.z, r.q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            d[2 * i] = (float)((int32_t)(w[i] << 16) >> 16);
            d[2 * i + 1] = (float)((int32_t)w[i] >> 16);
        }
    } else if constexpr (sizeof(T) == 1) {
        const uint32_t w[2] = {r.q.x, r.q.y};
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k) d[4 * i + k] = (float)((int32_t)(w[i] << (24 - 8 * k)) >> 24);
    } else {
        d[0] = r.a.x, d[1] = r.a.y, d[2] = r.a.z, d[3] = r.a.w;
        d[4] = r.b.x, d[5] = r.b.y, d[6] = r.b.z, d[7] = r.b.w;
    }
}

template <typename T, bool TAIL>
__device__ __attribute__((always_inline)) inline float lane_chunk_sum_tri(const TriView &tv, const float (&A)[12],
                                                                          const float (&px)[kU], const float (&py)[kU],
                                                                          const float (&pz)[kU], int lane, int nvalid) {
    constexpr int E = 8 * sizeof(T);  // bytes per cell
    constexpr int kShift = kCellBrickLog2 + (E == 8 ? 3 : E == 16 ? 4 : 5);
    float s = 0.0f;
#pragma unroll
    for (int u0 = 0; u0 < kU; u0 += kTriU) {
        CellRaw<T> raw[kTriU];
        uint32_t off[kTriU];
        float fx[kTriU], fy[kTriU], fz[kTriU];
#pragma unroll
        for (int v = 0; v < kTriU; ++v) {
            const int u = u0 + v;
            const float gx = grid_coord(A[0], A[1], A[2], A[9], px[u], py[u], pz[u]);
            const float gy = grid_coord(A[3], A[4], A[5], A[10], px[u], py[u], pz[u]);
            const float gz = grid_coord(A[6], A[7], A[8], A[11], px[u], py[u], pz[u]);
            const uint32_t ix = tri_axis(gx, tv.hx, fx[v]);
            const uint32_t iy = tri_axis(gy, tv.hy, fy[v]);
            const uint32_t iz = tri_axis(gz, tv.hz, fz[v]);
            off[v] = cell_offset<E>(tv, ix, iy, iz);
        }
        int msk[kTriU];
#pragma unroll
        for (int v = 0; v < kTriU; ++v) msk[v] = gp(tv.mask)[off[v] >> kShift];
        __builtin_amdgcn_sched_barrier(0);
        // cells of bricks wholly at +Q or wholly at -Q read the +Q sentinel
        // brick at offset 0 (same square)
#pragma unroll
        for (int v = 0; v < kTriU; ++v) raw[v] = load_cell<T>(tv.base, off[v] & (uint32_t)msk[v]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < kTriU; ++v) {
            float d[8];
            unpack_cell<T>(raw[v], d);
            const float c00 = lerp(d[0], d[1], fx[v]), c10 = lerp(d[2], d[3], fx[v]);
            const float c01 = lerp(d[4], d[5], fx[v]), c11 = lerp(d[6], d[7], fx[v]);
            const float c0 = lerp(c00, c10, fy[v]), c1 = lerp(c01, c11, fy[v]);
            float mv = lerp(c0, c1, fz[v]);
            if (TAIL) mv = (u0 + v) * kWave + lane < nvalid ? mv : 0.0f;
            s = __builtin_fmaf(mv, mv, s);
        }
        // Keep batches apart so that only one batch's cells are live: the
        // empty statement takes s as an operand, so this batch's arithmetic must
        // be done here, not sunk below the next batch's gathers.
        asm volatile("" : "+v"(s));
    }
    return s;
}

// Sparse map (offset table + super-brick pool): the super-brick's table entry
// first, then the value in the pool; points outside the map read slot 0 (+Q)
// and padding slots slot 1 (zeros).  Same index recipe, values and summation order
// as the dense layout, so a map gives the same bits in either form.
template <typename T>
__device__ inline int load_raw64(const char *p) {
    if constexpr (sizeof(T) == 4)
        return __float_as_int(*gp(reinterpret_cast<const float *>(p)));
    else
        return (int)*gp(reinterpret_cast<const T *>(p));
}

template <typename T, bool TAIL, bool WIDE>
__device__ __attribute__((always_inline)) inline float lane_chunk_sum_sparse(const MapView &m, const SparseView &sp,
                                                                             const float (&A)[12], const float (&px)[kU],
                                                                             const float (&py)[kU], const float (&pz)[kU],
                                                                             int lane, int nvalid) {
    constexpr uint32_t ES = sizeof(T);
    uint32_t sidx[kU], wv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const float gx = grid_coord(A[0], A[1], A[2], A[9], px[u], py[u], pz[u]);
        const float gy = grid_coord(A[3], A[4], A[5], A[10], px[u], py[u], pz[u]);
        const float gz = grid_coord(A[6], A[7], A[8], A[11], px[u], py[u], pz[u]);
        uint32_t ix, iy, iz;
        const bool ok = voxel_ijk(m, gx, gy, gz, ix, iy, iz);
        // two 24-bit multiply-adds (the empty asm keeps the compiler from
        // turning them into multiplies and a three-way add)
        uint32_t b = __umul24(iy >> kSLY, sp.nsx) + (ix >> kSLX);
        asm volatile("" : "+v"(b));
        b = __umul24(iz >> kSLZ, sp.nsxy) + b;
        b = ok ? b : sp.outside;
        if (TAIL) b = (u * kWave + lane < nvalid) ? b : sp.pad;
        sidx[u] = b << 2;   // byte offset of the entry: 32 bits (the table has under 2^28 entries), so
                            // the gather takes the table base in scalar registers and no 64-bit add
        wv[u] = ((ix & (kSX - 1u)) + ((iy & (kSY - 1u)) << kSLX) + ((iz & (kSZ - 1u)) << (kSLX + kSLY))) * ES;
    }
    uint32_t ent[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) ent[u] = *gp(reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(sp.table) + sidx[u]));
    __builtin_amdgcn_sched_barrier(0);
    int raw[kU];
    if constexpr (!WIDE) {
        // pool below 4 GiB: the entry is the slot's byte offset; slot 0 (+Q)
        // is read at its first value, so such lanes share one line
#pragma unroll
        for (int u = 0; u < kU; ++u) raw[u] = load_raw<T>(sp.pool, ent[u] ? ent[u] + wv[u] : 0u);
    } else {
#pragma unroll
        for (int u = 0; u < kU; ++u)
            raw[u] = load_raw64<T>(sp.pool + (ent[u] ? (uint64_t)ent[u] * ((uint32_t)kSuperVals * ES) + wv[u] : 0u));
    }
    __builtin_amdgcn_sched_barrier(0);
    float s = 0.0f;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const float f = as_value<T>(raw[u]);
        s = __builtin_fmaf(f, f, s);
    }
    return s;
}

// Lookup kinds of the sensor kernel (sparse: pools below / above 4 GiB).
constexpr int kLookNearest = 0, kLookTrilinear = 1, kLookSparse = 2, kLookSparseWide = 3, kLookNearestLds = 4;

// Particles [p0, p1) of the wave's group (particles n0 + p) against one chunk,
// with lookup LK (kLookNearestLds here: the coarse level read from LDS).
// probe: count the in-place reads of the nearest lookup into *nmixed
// (wave-uniform).  A particle's 12 pose constants, the same for every lane,
// come into scalar registers: with PCT by scalar loads from the job's table of
// them, issued one particle ahead so that they arrive while the previous
// particle's lookups run (no vector instruction), else by a read of lane p's
// registers (one vector instruction each); the values, and so the results, are
// the same.
template <typename T, bool TAIL, int LK, bool SUM, bool PCT = false>
__device__ __attribute__((always_inline)) inline void chunk_range(const SensorJob &J, const float (&pa)[12], const float (&px)[kU],
                                   const float (&py)[kU], const float (&pz)[kU], int lane, int nvalid,
                                   int p0, int p1, float &acc, const uint32_t *sbits, int n0, bool probe = false,
                                   int *nmixed = nullptr) {
    static_assert(!SUM || LK == kLookNearest || LK == kLookNearestLds, "the sum reading has the nearest lookup only");
    // the run's bounds and the group's first particle are the same on every
    // lane: said so, the particle loop and the table addresses are scalar work
    p0 = __builtin_amdgcn_readfirstlane(p0);
    p1 = __builtin_amdgcn_readfirstlane(p1);
    n0 = __builtin_amdgcn_readfirstlane(n0);
    typedef const __attribute__((address_space(4))) float *cptr;
    float nx[12];  // with the table: the next particle's constants, loaded one particle ahead
    if constexpr (PCT) {
        if (p0 < p1) {
            cptr q = (cptr)(J.pc + (size_t)(n0 + p0) * 12);
#pragma unroll
            for (int j = 0; j < 12; ++j) nx[j] = q[j];
        }
    }
    for (int p = p0; p < p1; ++p) {
        float A[12];
        if constexpr (PCT) {
#pragma unroll
            for (int j = 0; j < 12; ++j) A[j] = nx[j];
            cptr q = (cptr)(J.pc + (size_t)(n0 + min(p + 1, p1 - 1)) * 12);
#pragma unroll
            for (int j = 0; j < 12; ++j) nx[j] = q[j];
        } else {
#pragma unroll
            for (int j = 0; j < 12; ++j) A[j] = bcast(pa[j], p);
        }
        float t;
        if constexpr (LK == kLookTrilinear)
            t = wave_sum(lane_chunk_sum_tri<T, TAIL>(J.tri, A, px, py, pz, lane, nvalid));
        else if constexpr (LK == kLookSparse || LK == kLookSparseWide)
            t = wave_sum(lane_chunk_sum_sparse<T, TAIL, LK == kLookSparseWide>(J.map, J.sp, A, px, py, pz, lane, nvalid));
        else if constexpr (LK == kLookNearestLds)
            t = wave_sum(lane_chunk_sum_lds<T, TAIL, SUM>(J.map, sbits, A, px, py, pz, lane, nvalid, J.k2));
        else
            t = wave_sum(lane_chunk_sum<T, TAIL, SUM>(J.map, A, px, py, pz, lane, nvalid, J.k2, probe, nmixed));
        if (lane == p) acc += t;
    }
}

// The wave's run of particles [p0, p1) against one chunk.  With the LDS
// coarse level available, the coarse level is read from LDS or from global
// memory, whichever suits this wave's particles (same bits either way): the
// first kProbe particles run with the global masks and count the in-place
// reads; the rest take LDS when over 3/4 of those were in place (tracking:
// most points land in the band, and LDS saves a gather per point), else stay
// on the global masks (global localisation: most points read the shared
// sentinel line, and the global path issues fewer instructions).
template <typename T, bool TAIL, int LK, bool SUM, bool PCT = false>
__device__ __attribute__((always_inline)) inline void chunk_group(const SensorJob &J, const float (&pa)[12], const float (&px)[kU],
                                   const float (&py)[kU], const float (&pz)[kU], int lane, int nvalid,
                                   int p0, int p1, float &acc, const uint32_t *sbits, int n0) {
    if constexpr (LK == kLookNearestLds) {
        int q0 = p0;
        bool lds = J.coarse == kCoarseBits;
        if (J.coarse == kCoarseAuto) {
            int nmixed = 0;
            q0 = min(p0 + kProbe, p1);
            chunk_range<T, TAIL, kLookNearest, SUM, PCT>(J, pa, px, py, pz, lane, nvalid, p0, q0, acc, sbits, n0, true, &nmixed);
            lds = nmixed * 8 > J.lds8 * kChunk * (q0 - p0);
        }
        if (lds)
            chunk_range<T, TAIL, kLookNearestLds, SUM, PCT>(J, pa, px, py, pz, lane, nvalid, q0, p1, acc, sbits, n0);
        else
            chunk_range<T, TAIL, kLookNearest, SUM, PCT>(J, pa, px, py, pz, lane, nvalid, q0, p1, acc, sbits, n0);
    } else {
        chunk_range<T, TAIL, LK, SUM, PCT>(J, pa, px, py, pz, lane, nvalid, p0, p1, acc, sbits, n0);
    }
}

// Coordinates of work item `local` of a job: its group of 64 particles, its
// piece of 4096 points and its run [p0, p1) of the group's particles (empty
// when the group is short).
struct ItemPos {
    int n0, piece, p0, p1;
};
__device__ __attribute__((always_inline)) inline ItemPos item_pos(const SensorJob &J, int local) {
    const int per = J.npiece * J.nsub;
    const int group = local / per;
    const int rem = local - group * per;
    const int piece = rem / J.nsub;
    const int run = kGroup / J.nsub;
    const int p0 = (rem - piece * J.nsub) * run;
    const int n0 = group * kGroup;
    return ItemPos{n0, piece, p0, min(p0 + run, min(kGroup, J.N - n0))};
}

// One work item: particles 64 g + [p0, p1) of a job against points
// [4096 piece, 4096 piece + 4096).  Returns lane p's sum for particle 64 g + p.
template <typename T, int LK, bool SUM, bool PCT = false>
__device__ __attribute__((always_inline)) inline float sensor_item(const SensorJob &J, int local, int lane,
                                                                   const uint32_t *sbits) {
    const ItemPos ip = item_pos(J, local);
    if (ip.p0 >= ip.p1) return 0.0f;
    const int n0 = ip.n0, piece = ip.piece;
    const int gcount = min(kGroup, J.N - n0);
    const MapView &m = J.map;
    const int K = J.K;

    float pa[12];  // this lane's particle's pose constants (read only without the table)
    if constexpr (!PCT) pose_consts(J.poses, J.N, n0 + min(lane, gcount - 1), m, pa);

    float acc = 0.0f;
    const int kb = piece * kPiece;
    const int ke = min(K, kb + kPiece);
    for (int kc = kb; kc < ke; kc += kChunk) {
        const int nvalid = min(kChunk, ke - kc);
        float px[kU], py[kU], pz[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            int k = min(kc + u * kWave + lane, ke - 1);  // padding slots are masked later
            px[u] = gp(J.pts)[k];
            py[u] = gp(J.pts)[(size_t)K + k];
            pz[u] = gp(J.pts)[(size_t)2 * K + k];
        }
        if (nvalid == kChunk)
            chunk_group<T, false, LK, SUM, PCT>(J, pa, px, py, pz, lane, nvalid, ip.p0, ip.p1, acc, sbits, n0);
        else
            chunk_group<T, true, LK, SUM, PCT>(J, pa, px, py, pz, lane, nvalid, ip.p0, ip.p1, acc, sbits, n0);
    }
    return acc;
}

// A particle's log-weight from its total: -(S c) for the product reading,
// log S for the sum reading (0 for an empty scan: no evidence, equal weights).
template <bool SUM>
__device__ __attribute__((always_inline)) inline float particle_logw(const SensorJob &J, float S) {
    if constexpr (SUM) return J.K > 0 ? logf(S) : 0.0f;
    else return -(S * J.c);
}

// Output of a work item: l directly (one piece) or the piece's partial sums.
template <bool SUM>
__device__ __attribute__((always_inline)) inline void sensor_store(const SensorJob &J, int local, int lane,
                                                                   float acc) {
    const ItemPos ip = item_pos(J, local);
    if (lane >= ip.p0 && lane < ip.p1) {
        const int slot = ip.n0 + lane;
        if (J.npiece == 1)
            J.logw[J.orig ? J.orig[slot] : slot] = particle_logw<SUM>(J, acc);
        else
            J.part[(size_t)ip.piece * J.N + slot] = acc;
    }
}

// Waves stride over the work items of all jobs of the launch (one item per
// wave for a full grid, several for a persistent one).  The job descriptor is
// read into scalar registers per item and read again for the store, so it need
// not stay live across the item.
template <typename T, int WPB, typename Src, int LK = kLookNearest, bool SUM = false, bool PCT = false>
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(LK == kLookTrilinear ? 2 : (LK == kLookNearest || LK == kLookNearestLds || LK == kLookSparse) ? 4 : 3))) void sensor_kernel(Src src) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nitems = src.items();
    const int64_t stride = (int64_t)gridDim.x * WPB;
    extern __shared__ __align__(16) uint32_t sbits[];
    if constexpr (LK == kLookNearestLds) {
        // one map per launch: its read bits into LDS, in 16-byte pieces, four
        // loads in flight per thread before the stores (the bit table sits in
        // a 256-byte aligned, 256-byte padded region; the LDS allocation is
        // rounded up to 16 bytes).  Indexes past the end are clamped to the
        // last piece, which is then loaded and stored again with its own value.
        const SensorJob J0 = src.load(0);
        const uint32_t n4 = (J0.map.nrwords + 3u) >> 2;
        const u32x4 *from = reinterpret_cast<const u32x4 *>(J0.map.rbits);
        u32x4 *to = reinterpret_cast<u32x4 *>(sbits);
        constexpr uint32_t kT = WPB * 64;
        for (uint32_t w0 = threadIdx.x; w0 < n4; w0 += 4 * kT) {
            u32x4 v[4];
#pragma unroll
            for (uint32_t i = 0; i < 4; ++i) v[i] = gp(from)[min(w0 + i * kT, n4 - 1u)];
#pragma unroll
            for (uint32_t i = 0; i < 4; ++i) to[min(w0 + i * kT, n4 - 1u)] = v[i];
        }
        __syncthreads();
    }
    // Workgroups go to the chip's 8 dies (XCDs, each with its own L2) in turn:
    // workgroup b to die b mod 8.  Die x takes the x-th eighth of the work items
    // instead, consecutive ones, so with the particles in spatial order each
    // die's L2 holds the lines of one region of the map (a permutation of the
    // workgroups that have work, so every die gets its share also when a
    // replayed graph's grid is larger than the launch needs; any order gives
    // the same results).
    int64_t first = blockIdx.x;
    const int64_t used = std::min<int64_t>(gridDim.x, (nitems + WPB - 1) / WPB);
    if (used >= 8 && (int64_t)blockIdx.x < used) {
        const uint32_t g = (uint32_t)used, per = g >> 3, extra = g & 7u, x = blockIdx.x & 7u;
        first = (int64_t)(x * per + min(x, extra) + (blockIdx.x >> 3));
    }
    for (int64_t item = first * WPB + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); item < nitems;
         item += stride) {
        const int j = find_job_uniform(src, item, [](const SensorJob &J) { return J.item0; });
        float acc;
        int local;
        {
            const SensorJob J = src.load(j);
            local = (int)(item - J.item0);
            acc = sensor_item<T, LK, SUM, PCT>(J, local, lane, sbits);
        }
        const SensorJob J = src.load(j);
        sensor_store<SUM>(J, local, lane, acc);
    }
}

// Pairwise sum of the piece partials in a fixed tree (a binary counter over the
// pieces in order), then l = -(S * c) (or log S, sum reading).  Jobs with one
// piece are done already.
template <typename Src>
__global__ __launch_bounds__(256) void combine_kernel(Src src) {
    const int64_t nelems = src.elems();
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nelems; e += (int64_t)gridDim.x * 256) {
        const int j = find_job(src, e, [](const SensorJob &J) { return J.elem0; });
        const SensorJob &J = src.get(j);
        if (J.npiece == 1) continue;
        const int n = (int)(e - J.elem0);
        float stack[12];
        int depth = 0;
        for (int p = 0; p < J.npiece; ++p) {
            float v = J.part[(size_t)p * J.N + n];
            for (int t = p + 1; (t & 1) == 0; t >>= 1) v = stack[--depth] + v;
            stack[depth++] = v;
        }
        float s = stack[--depth];
        while (depth > 0) s = stack[--depth] + s;
        J.logw[J.orig ? J.orig[n] : n] = J.score == kScoreSum ? particle_logw<true>(J, s) : particle_logw<false>(J, s);
    }
}

// Spatial order.  The cell of a particle: its x-y position in cells of
// 1/kOrderSide of the map's extent per axis (clamped to the map; NaN to cell 0),
// numbered in Morton order (the bits of the cell's x and y interleaved), so
// cells close in number lie close in the map.
__device__ inline uint32_t spread_bits(uint32_t v) {
    uint32_t r = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) r |= ((v >> b) & 1u) << (2 * b);
    return r;
}

__device__ inline int order_cell(const SensorJob &J, int n) {
    static_assert(kOrderSide == 64, "six bits per axis");
    const MapView &m = J.map;
    const float tx = gp(J.poses)[(size_t)9 * J.N + n], ty = gp(J.poses)[(size_t)10 * J.N + n];
    const float hx = (float)kOrderSide / (float)m.nx, hy = (float)kOrderSide / (float)m.ny;
    const float top = (float)(kOrderSide - 1);
    // fmaxf returns the other operand for a NaN, so NaN lands in cell 0
    const float fx = fminf(fmaxf((tx - m.ox) * m.inv_v * hx, 0.0f), top);
    const float fy = fminf(fmaxf((ty - m.oy) * m.inv_v * hy, 0.0f), top);
    return (int)(spread_bits((uint32_t)fx) | (spread_bits((uint32_t)fy) << 1));
}

// Clears the cell counters of every ordered job (one workgroup per job).
template <typename Src>
__global__ __launch_bounds__(256) void order_zero_kernel(Src src) {
    for (int j = blockIdx.x; j < src.count(); j += gridDim.x) {
        const SensorJob &J = src.get(j);
        if (!J.orig) continue;
        for (int c = threadIdx.x; c < kOrderCells; c += 256) J.ocell[c] = 0;
    }
}

// Counts the particles of each cell and gives each particle its rank within its
// cell: per block of kOrderBlock particles of one job a histogram in LDS (the
// LDS adds give the ranks within the block), then one global add per occupied
// cell, which returns the block's first rank in that cell.  Which block comes
// first in a cell depends on timing; every particle still gets a distinct slot
// and the results do not depend on the slots.
template <typename Src>
__global__ __launch_bounds__(256) void order_count_kernel(Src src) {
    __shared__ int hist[kOrderCells];
    constexpr int kPer = kOrderBlock / 256;
    const int64_t nblk = src.blocks();
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int j = find_job_uniform(src, b, [](const SensorJob &J) { return J.oblk0; });
        const SensorJob &J = src.get(j);
        for (int c = threadIdx.x; c < kOrderCells; c += 256) hist[c] = 0;
        __syncthreads();
        const int n0 = (int)(b - J.oblk0) * kOrderBlock;
        int cell[kPer], rank[kPer];
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int n = n0 + i * 256 + (int)threadIdx.x;
            cell[i] = n < J.N ? order_cell(J, n) : -1;
            rank[i] = cell[i] >= 0 ? atomicAdd(&hist[cell[i]], 1) : 0;
        }
        __syncthreads();
        for (int c = threadIdx.x; c < kOrderCells; c += 256) {
            const int k = hist[c];
            if (k) hist[c] = atomicAdd(&J.ocell[c], k);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kPer; ++i)
            if (cell[i] >= 0) J.orank[n0 + i * 256 + (int)threadIdx.x] = hist[cell[i]] + rank[i];
        __syncthreads();
    }
}

// Each cell's count becomes its first slot: the exclusive prefix sum over the
// cells in order (one workgroup per ordered job).
template <typename Src>
__global__ __launch_bounds__(256) void order_scan_kernel(Src src) {
    __shared__ int tot[256];
    constexpr int kPer = kOrderCells / 256;
    const int t = threadIdx.x;
    for (int j = blockIdx.x; j < src.count(); j += gridDim.x) {
        const SensorJob &J = src.get(j);
        if (!J.orig) continue;
        int v[kPer], s = 0;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            v[i] = J.ocell[t * kPer + i];
            s += v[i];
        }
        tot[t] = s;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {
            const int x = t >= d ? tot[t - d] : 0;
            __syncthreads();
            tot[t] += x;
            __syncthreads();
        }
        int run = tot[t] - s;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            J.ocell[t * kPer + i] = run;
            run += v[i];
        }
        __syncthreads();
    }
}

// The pose constants of every particle (pose prologue), by the same device code
// the lanes use, into the table the sensor kernel reads with scalar loads (jobs
// whose pc is set; elements by the jobs' particle offsets).  An ordered job's
// particle goes to slot (first slot of its cell) + (its rank in the cell), and
// the slot records the particle.
template <typename Src>
__global__ __launch_bounds__(256) void pose_consts_jobs_kernel(Src src) {
    const int64_t nelems = src.elems();
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nelems; e += (int64_t)gridDim.x * 256) {
        const int j = find_job(src, e, [](const SensorJob &J) { return J.elem0; });
        const SensorJob &J = src.get(j);
        if (!J.pc) continue;
        const int n = (int)(e - J.elem0);
        float pa[12];
        pose_consts(J.poses, J.N, n, J.map, pa);
        int slot = n;
        if (J.orig) {
            slot = J.ocell[order_cell(J, n)] + J.orank[n];
            J.orig[slot] = n;
        }
        // a slot's 48 bytes as three 16-byte stores (tables are 256-byte aligned)
        f32x4 *out = reinterpret_cast<f32x4 *>(const_cast<float *>(J.pc) + (size_t)slot * 12);
#pragma unroll
        for (int k = 0; k < 3; ++k) out[k] = f32x4{pa[4 * k], pa[4 * k + 1], pa[4 * k + 2], pa[4 * k + 3]};
    }
}

__global__ __launch_bounds__(256) void fill_kernel(float *__restrict__ out, int n, float v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

__global__ __launch_bounds__(256) void debug_index_kernel(MapView m, const float *__restrict__ pts, int K,
                                                          const float *__restrict__ poses, int N,
                                                          int64_t *__restrict__ lin) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)N * K) return;
    int n = (int)(id / K), k = (int)(id - (int64_t)n * K);
    float pa[12];
    pose_consts(poses, N, n, m, pa);
    float x = pts[k], y = pts[(size_t)K + k], z = pts[(size_t)2 * K + k];
    float gx = grid_coord(pa[0], pa[1], pa[2], pa[9], x, y, z);
    float gy = grid_coord(pa[3], pa[4], pa[5], pa[10], x, y, z);
    float gz = grid_coord(pa[6], pa[7], pa[8], pa[11], x, y, z);
    uint32_t ix, iy, iz;
    bool ok = voxel_ijk(m, gx, gy, gz, ix, iy, iz);
    lin[id] = ok ? (int64_t)ix + (int64_t)m.nx * ((int64_t)iy + (int64_t)m.ny * iz) : -1;
}

// ------------------------------------------------------------------ host side
int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            cus = p.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

// LDS bytes a compute unit holds (64 KiB if the device does not say).
static size_t device_lds_per_cu() {
    static size_t lds = 0;
    if (!lds) {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            lds = p.maxSharedMemoryPerMultiProcessor;
        if (lds == 0) lds = 64 * 1024;
    }
    return lds;
}

// Waves per workgroup of a launch whose workgroups each hold `lds` bytes of read
// bits: the requested number, raised (up to 8) until the workgroups that fit a
// compute unit's LDS hold the 16 waves its registers allow (4 per SIMD), so
// that a large bit table does not cut the occupancy.  Any shape gives the same
// bits.
static int lds_waves_per_block(int wpb, size_t lds) {
    if (lds == 0) return wpb;
    const size_t fit = device_lds_per_cu() / lds;
    while (wpb < 8 && fit * (size_t)wpb < 16) wpb *= 2;
    return wpb;
}

// nitems: the item count when known on the host (sizes a one-wave-per-item
// grid); a persistent grid does not need it.
template <typename T, typename Src, int LK = kLookNearest, bool SUM = false, bool PCT = false>
static void launch_sensor_t(const Src &src, int64_t nitems, LaunchCfg cfg, hipStream_t stream, size_t lds = 0) {
    const int wpb = lds_waves_per_block(cfg.waves_per_block, lds);
    int64_t blocks = (nitems + wpb - 1) / wpb;
    if (cfg.blocks_per_cu > 0) blocks = std::min<int64_t>(blocks, (int64_t)device_cus() * cfg.blocks_per_cu);
    if (blocks < 1) blocks = 1;
    switch (wpb) {
        case 2: sensor_kernel<T, 2, Src, LK, SUM, PCT><<<(unsigned)blocks, 128, lds, stream>>>(src); break;
        case 8: sensor_kernel<T, 8, Src, LK, SUM, PCT><<<(unsigned)blocks, 512, lds, stream>>>(src); break;
        default: sensor_kernel<T, 4, Src, LK, SUM, PCT><<<(unsigned)blocks, 256, lds, stream>>>(src); break;
    }
}

template <typename Src, bool SUM, bool PCT>
static void launch_sensor_dense(int32_t dtype, const Src &src, int64_t nitems, LaunchCfg cfg, hipStream_t stream,
                                size_t lds) {
    if (lds > 0) {
        if (dtype == MCL_TSDF_I16) launch_sensor_t<int16_t, Src, kLookNearestLds, SUM, PCT>(src, nitems, cfg, stream, lds);
        else if (dtype == MCL_TSDF_I8) launch_sensor_t<int8_t, Src, kLookNearestLds, SUM, PCT>(src, nitems, cfg, stream, lds);
        else launch_sensor_t<float, Src, kLookNearestLds, SUM, PCT>(src, nitems, cfg, stream, lds);
    } else if (dtype == MCL_TSDF_I16) launch_sensor_t<int16_t, Src, kLookNearest, SUM, PCT>(src, nitems, cfg, stream);
    else if (dtype == MCL_TSDF_I8) launch_sensor_t<int8_t, Src, kLookNearest, SUM, PCT>(src, nitems, cfg, stream);
    else launch_sensor_t<float, Src, kLookNearest, SUM, PCT>(src, nitems, cfg, stream);
}

template <typename Src, bool SUM>
static void launch_sensor_dense(int32_t dtype, const Src &src, int64_t nitems, LaunchCfg cfg, hipStream_t stream,
                                size_t lds, bool pct) {
    if (pct) launch_sensor_dense<Src, SUM, true>(dtype, src, nitems, cfg, stream, lds);
    else launch_sensor_dense<Src, SUM, false>(dtype, src, nitems, cfg, stream, lds);
}

// lds > 0: every job of the launch reads the same dense map, whose read bits
// (nrwords * 4 <= lds bytes) each workgroup copies into LDS; the coarse level
// is then chosen per wave (the jobs' `coarse` field).  sum: the jobs take the
// sum reading (kScoreSum), else the product reading.
// pct: every job of the launch has its pose-constant table (pc), filled here
// first.  ord: some jobs are put in spatial order (orig set) as their tables
// are filled: src.blocks() counting blocks, oblocks (at least as many) sizing
// the grid, and ojobs workgroups for the per-job passes.
template <typename Src>
mcl_status launch_sensor_src(int32_t dtype, const Src &src, int64_t nitems, int64_t nelems, bool combine,
                             LaunchCfg cfg, hipStream_t stream, size_t lds, bool sum, bool pct, bool ord,
                             int64_t oblocks, int ojobs) {
    if (pct) {
        if (ord) {
            const unsigned jb = (unsigned)std::max(ojobs, 1);
            order_zero_kernel<<<jb, 256, 0, stream>>>(src);
            mcl_status st = check_launch("order_zero_kernel");
            if (st != MCL_OK) return st;
            order_count_kernel<<<(unsigned)std::max<int64_t>(std::min<int64_t>(oblocks, 2048), 1), 256, 0, stream>>>(src);
            st = check_launch("order_count_kernel");
            if (st != MCL_OK) return st;
            order_scan_kernel<<<jb, 256, 0, stream>>>(src);
            st = check_launch("order_scan_kernel");
            if (st != MCL_OK) return st;
        }
        const int64_t blocks = std::min<int64_t>((nelems + 255) / 256, (int64_t)device_cus() * 16);
        pose_consts_jobs_kernel<<<(unsigned)std::max<int64_t>(blocks, 1), 256, 0, stream>>>(src);
        mcl_status st = check_launch("pose_consts_jobs_kernel");
        if (st != MCL_OK) return st;
    }
    if (sum) launch_sensor_dense<Src, true>(dtype, src, nitems, cfg, stream, lds, pct);
    else launch_sensor_dense<Src, false>(dtype, src, nitems, cfg, stream, lds, pct);
    mcl_status st = check_launch("sensor_kernel");
    if (st != MCL_OK || !combine) return st;
    int64_t blocks = std::min<int64_t>((nelems + 255) / 256, (int64_t)device_cus() * 16);
    combine_kernel<<<(unsigned)std::max<int64_t>(blocks, 1), 256, 0, stream>>>(src);
    return check_launch("combine_kernel");
}

template mcl_status launch_sensor_src<JobTable<SensorJob>>(int32_t, const JobTable<SensorJob> &, int64_t, int64_t,
                                                           bool, LaunchCfg, hipStream_t, size_t, bool, bool, bool,
                                                           int64_t, int);

// Sparse maps with pools below 4 GiB (the offset table holds byte offsets):
// one wave per work item, four waves per workgroup, as for a single call.
template <typename Src>
mcl_status launch_sensor_sparse_src(int32_t dtype, const Src &src, int64_t nitems, int64_t nelems, bool combine,
                                    hipStream_t stream) {
    const unsigned blocks = (unsigned)std::max<int64_t>((nitems + 3) / 4, 1);
    if (dtype == MCL_TSDF_I16) sensor_kernel<int16_t, 4, Src, kLookSparse><<<blocks, 256, 0, stream>>>(src);
    else if (dtype == MCL_TSDF_I8) sensor_kernel<int8_t, 4, Src, kLookSparse><<<blocks, 256, 0, stream>>>(src);
    else sensor_kernel<float, 4, Src, kLookSparse><<<blocks, 256, 0, stream>>>(src);
    mcl_status st = check_launch("sensor_kernel (sparse map)");
    if (st != MCL_OK || !combine) return st;
    int64_t cb = std::min<int64_t>((nelems + 255) / 256, (int64_t)device_cus() * 16);
    combine_kernel<<<(unsigned)std::max<int64_t>(cb, 1), 256, 0, stream>>>(src);
    return check_launch("combine_kernel");
}

template mcl_status launch_sensor_sparse_src<JobTable<SensorJob>>(int32_t, const JobTable<SensorJob> &, int64_t,
                                                                  int64_t, bool, hipStream_t);

// Trilinear lookup (the jobs' corner cells built): one wave per work item,
// four waves per workgroup, as for a single call.
template <typename Src>
mcl_status launch_sensor_tri_src(int32_t dtype, const Src &src, int64_t nitems, int64_t nelems, bool combine,
                                 hipStream_t stream) {
    const unsigned blocks = (unsigned)std::max<int64_t>((nitems + 3) / 4, 1);
    if (dtype == MCL_TSDF_I16) sensor_kernel<int16_t, 4, Src, kLookTrilinear><<<blocks, 256, 0, stream>>>(src);
    else if (dtype == MCL_TSDF_I8) sensor_kernel<int8_t, 4, Src, kLookTrilinear><<<blocks, 256, 0, stream>>>(src);
    else sensor_kernel<float, 4, Src, kLookTrilinear><<<blocks, 256, 0, stream>>>(src);
    mcl_status st = check_launch("sensor_kernel (trilinear)");
    if (st != MCL_OK || !combine) return st;
    int64_t cb = std::min<int64_t>((nelems + 255) / 256, (int64_t)device_cus() * 16);
    combine_kernel<<<(unsigned)std::max<int64_t>(cb, 1), 256, 0, stream>>>(src);
    return check_launch("combine_kernel");
}

template mcl_status launch_sensor_tri_src<JobTable<SensorJob>>(int32_t, const JobTable<SensorJob> &, int64_t,
                                                               int64_t, bool, hipStream_t);
template mcl_status launch_sensor_src<OneJob<SensorJob>>(int32_t, const OneJob<SensorJob> &, int64_t, int64_t,
                                                         bool, LaunchCfg, hipStream_t, size_t, bool, bool, bool,
                                                         int64_t, int);

SensorJob make_sensor_job(const mcl_map_s *map, const float *pts, int K, const float *poses, int N, float c,
                          float *logw, float *part) {
    SensorJob J{};
    J.map = map->view;
    J.sp = map->sp;
    J.pts = pts;
    J.poses = poses;
    J.logw = logw;
    J.part = part;
    J.c = c;
    J.K = K;
    J.N = N;
    J.npiece = sensor_pieces(K);
    J.ngroups = (N + kGroup - 1) / kGroup;
    J.nsub = sensor_runs((int64_t)J.ngroups * J.npiece);
    J.lds8 = kLdsEighths;
    J.score = kScoreProduct;
    J.k2 = 0.0f;
    return J;
}

// The launch shape's settings of a job: runs per group and the coarse-level
// threshold (neither changes a result).
void apply_cfg(SensorJob &J, const LaunchCfg &cfg) {
    if (cfg.runs > 0) J.nsub = cfg.runs;
    J.lds8 = cfg.lds8 > 0 ? cfg.lds8 : kLdsEighths;
}

// The stream's workspace of a single-filter update: the piece partials
// [npiece][N] (npiece > 1), then, with the table, the pose-constant table
// [N][12] (filled by the launch), then, with the spatial order, the cell
// counters and the particles' ranks and slots.  part given (the no-allocation
// call): the partials go there, and neither the table nor the order is used
// (the lanes broadcast the pose constants; same bits).
static mcl_status sensor_workspace(SensorJob &J, int N, int npiece, bool table, bool ord, hipStream_t stream,
                                   float *part) {
    J.pc = nullptr;
    J.ocell = J.orank = J.orig = nullptr;
    J.oblk0 = 0;
    if (part) {
        J.part = npiece > 1 ? part : nullptr;
        return MCL_OK;
    }
    auto a256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t part_bytes = npiece > 1 ? a256((size_t)npiece * N * sizeof(float)) : 0;
    const size_t pc_bytes = table ? a256((size_t)N * 12 * sizeof(float)) : 0;
    const size_t idx_bytes = a256((size_t)N * sizeof(int32_t));
    const size_t ord_bytes = ord ? a256(kOrderCells * sizeof(int32_t)) + 2 * idx_bytes : 0;
    J.part = nullptr;
    if (part_bytes + pc_bytes + ord_bytes == 0) return MCL_OK;
    char *ws = static_cast<char *>(workspace(stream, part_bytes + pc_bytes + ord_bytes));
    if (!ws) return fail(MCL_ENOMEM, "sensor_update: workspace allocation failed");
    if (npiece > 1) J.part = reinterpret_cast<float *>(ws);
    ws += part_bytes;
    if (table) J.pc = reinterpret_cast<const float *>(ws);
    ws += pc_bytes;
    if (ord) {
        J.ocell = reinterpret_cast<int32_t *>(ws);
        ws += a256(kOrderCells * sizeof(int32_t));
        J.orank = reinterpret_cast<int32_t *>(ws);
        J.orig = reinterpret_cast<int32_t *>(ws + idx_bytes);
    }
    return MCL_OK;
}

// part: the piece partials [npiece][N] (npiece > 1), or null for the stream's
// workspace.  score / k2: the reading (kScoreSum needs a dense map; k2 = -c log2 e).
static mcl_status launch_sensor_job(const mcl_map_s *map, const float *pts, int K, const float *poses, int N, float c,
                                    float *logw, LaunchCfg cfg, hipStream_t stream, float *part, int32_t score,
                                    float k2) {
    const bool sum = score == kScoreSum;
    if (sum && map->sparse) return fail(MCL_EINVAL, "sensor update: the sum reading needs a dense map");
    if (K == 0) {
        // no points: l = 0 for every particle in either reading
        fill_kernel<<<(N + 255) / 256, 256, 0, stream>>>(logw, N, sum ? 0.0f : -(0.0f * c));
        return check_launch("fill_kernel");
    }
    const int npiece = sensor_pieces(K);
    using Src = OneJob<SensorJob>;
    Src src{make_sensor_job(map, pts, K, poses, N, c, logw, nullptr), {}};
    // the pose-constant table and the spatial order: dense maps, not the no-allocation call
    const int64_t evals = (int64_t)N * K;
    const bool ord = !map->sparse && !part && spatial_order(evals);
    const bool table = !map->sparse && !part && (evals >= kPoseTableMinEvals || ord);
    mcl_status wst = sensor_workspace(src.job, N, npiece, table, ord, stream, part);
    if (wst != MCL_OK) return wst;
    src.job.score = score;
    src.job.k2 = k2;
    if (!map->sparse) apply_cfg(src.job, cfg);
    const int64_t nitems = (int64_t)src.job.ngroups * npiece * src.job.nsub;
    const int64_t oblocks = ord ? order_blocks(N) : 0;
    src.n = Counts{1, nitems, N, oblocks};
    const size_t lds_bytes = (((size_t)map->view.nrwords + 3) & ~(size_t)3) * 4;  // 16-byte pieces
    if (!map->sparse && lds_bytes <= kMaxLdsBits && cfg.coarse != kCoarseBytes) {
        src.job.coarse = cfg.coarse;
        return launch_sensor_src(map->dtype, src, nitems, N, npiece > 1, cfg, stream, lds_bytes, sum, table, ord,
                                 oblocks, 1);
    }
    if (!map->sparse)
        return launch_sensor_src(map->dtype, src, nitems, N, npiece > 1, cfg, stream, 0, sum, table, ord, oblocks, 1);
    // sparse map: one wave per work item, four waves per workgroup
    const unsigned blocks = (unsigned)((nitems + 3) / 4);
    if (map->sp.small) {
        if (map->dtype == MCL_TSDF_I16) sensor_kernel<int16_t, 4, Src, kLookSparse><<<blocks, 256, 0, stream>>>(src);
        else if (map->dtype == MCL_TSDF_I8) sensor_kernel<int8_t, 4, Src, kLookSparse><<<blocks, 256, 0, stream>>>(src);
        else sensor_kernel<float, 4, Src, kLookSparse><<<blocks, 256, 0, stream>>>(src);
    } else {
        if (map->dtype == MCL_TSDF_I16) sensor_kernel<int16_t, 4, Src, kLookSparseWide><<<blocks, 256, 0, stream>>>(src);
        else if (map->dtype == MCL_TSDF_I8) sensor_kernel<int8_t, 4, Src, kLookSparseWide><<<blocks, 256, 0, stream>>>(src);
        else sensor_kernel<float, 4, Src, kLookSparseWide><<<blocks, 256, 0, stream>>>(src);
    }
    mcl_status st = check_launch("sensor_kernel (sparse map)");
    if (st != MCL_OK || npiece == 1) return st;
    int64_t cb = std::min<int64_t>((N + 255) / 256, (int64_t)device_cus() * 16);
    combine_kernel<<<(unsigned)std::max<int64_t>(cb, 1), 256, 0, stream>>>(src);
    return check_launch("combine_kernel");
}

// Trilinear lookup: the same decomposition and summation order, one wave per
// work item, four waves per workgroup.
mcl_status launch_sensor_trilinear(mcl_map_s *map, const float *pts, int K, const float *poses, int N, float c,
                                   float *logw, hipStream_t stream) {
    mcl_status est = ensure_trilinear(map, stream);
    if (est != MCL_OK) return est;
    if (K == 0) {
        fill_kernel<<<(N + 255) / 256, 256, 0, stream>>>(logw, N, -(0.0f * c));
        return check_launch("fill_kernel");
    }
    const int npiece = sensor_pieces(K);
    using Src = OneJob<SensorJob>;
    Src src{make_sensor_job(map, pts, K, poses, N, c, logw, nullptr), {}};
    mcl_status wst = sensor_workspace(src.job, N, npiece, false, false, stream, nullptr);
    if (wst != MCL_OK) return wst;
    src.job.tri = map->tri;
    const int64_t nitems = (int64_t)src.job.ngroups * npiece * src.job.nsub;
    src.n = Counts{1, nitems, N, 0};
    const unsigned blocks = (unsigned)((nitems + 3) / 4);
    if (map->dtype == MCL_TSDF_I16) sensor_kernel<int16_t, 4, Src, kLookTrilinear><<<blocks, 256, 0, stream>>>(src);
    else if (map->dtype == MCL_TSDF_I8) sensor_kernel<int8_t, 4, Src, kLookTrilinear><<<blocks, 256, 0, stream>>>(src);
    else sensor_kernel<float, 4, Src, kLookTrilinear><<<blocks, 256, 0, stream>>>(src);
    mcl_status st = check_launch("sensor_kernel (trilinear)");
    if (st != MCL_OK || npiece == 1) return st;
    int64_t cb = std::min<int64_t>((N + 255) / 256, (int64_t)device_cus() * 16);
    combine_kernel<<<(unsigned)std::max<int64_t>(cb, 1), 256, 0, stream>>>(src);
    return check_launch("combine_kernel");
}

mcl_status launch_sensor_cfg(const mcl_map_s *map, const float *pts, int K, const float *poses, int N, float c,
                             float *logw, LaunchCfg cfg, hipStream_t stream, float *part) {
    return launch_sensor_job(map, pts, K, poses, N, c, logw, cfg, stream, part, kScoreProduct, 0.0f);
}

mcl_status launch_sensor(const mcl_map_s *map, const float *pts, int K, const float *poses, int N, float c,
                         float *logw, hipStream_t stream, float *part) {
    return launch_sensor_cfg(map, pts, K, poses, N, c, logw, tuned_config(map->dtype, K, N), stream, part);
}

// Sum reading, launched as the product reading's tuned shape for (dtype, K, N).
mcl_status launch_sensor_sum(const mcl_map_s *map, const float *pts, int K, const float *poses, int N, float k2,
                             float *logw, hipStream_t stream) {
    return launch_sensor_job(map, pts, K, poses, N, 0.0f, logw, tuned_config(map->dtype, K, N), stream, nullptr,
                             kScoreSum, k2);
}

mcl_status launch_debug_indices(const mcl_map_s *map, const float *pts, int K, const float *poses, int N,
                                int64_t *lin, hipStream_t stream) {
    int64_t total = (int64_t)N * K;
    if (total == 0) return MCL_OK;
    debug_index_kernel<<<(unsigned)((total + 255) / 256), 256, 0, stream>>>(map->view, pts, K, poses, N, lin);
    return check_launch("debug_index_kernel");
}

}  // namespace mcl

// ------------------------------------------------------------------ spatial order
namespace mcl {
static std::atomic<int64_t> g_order_min{kOrderDefaultMin};
int64_t spatial_order_min() { return g_order_min.load(std::memory_order_relaxed); }
}  // namespace mcl

extern "C" mcl_status mcl_set_spatial_order_min(int64_t min_evals) {
    mcl::g_order_min.store(min_evals, std::memory_order_relaxed);
    return MCL_OK;
}

extern "C" int64_t mcl_get_spatial_order_min(void) { return mcl::spatial_order_min(); }

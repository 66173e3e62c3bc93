// Device-side voxel addressing: the float32 index recipe and the brick layout.
// Shared by the sensor-update kernel and the index export, so both read the
// same voxel for every (particle, point) pair.
#pragma once

#include "mcl_internal.h"

namespace mcl {

// Per-particle constants of the index recipe (pose prologue):
//   a_jk = r_jk * inv_v  (pa[0..8]),  b_j = (t_j - o_j) * inv_v  (pa[9..11]).
// poses: [12][N] rows r00 .. r22 tx ty tz.
__device__ inline void pose_consts(const float *__restrict__ poses, int N, int n, const MapView &m,
                                   float pa[12]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int j = 0; j < 9; ++j) pa[j] = poses[(size_t)j * N + n] * m.inv_v;
    float dx = poses[(size_t)9 * N + n] - m.ox;
    float dy = poses[(size_t)10 * N + n] - m.oy;
    float dz = poses[(size_t)11 * N + n] - m.oz;
    pa[9] = dx * m.inv_v;
    pa[10] = dy * m.inv_v;
    pa[11] = dz * m.inv_v;
}

// One grid coordinate: ((a0 x + a1 y) + a2 z) + b, every operation rounded.
__device__ inline float grid_coord(float a0, float a1, float a2, float b, float x, float y, float z) {
#pragma clang fp contract(off)
    float s = a0 * x;
    float t = a1 * y;
    s = s + t;
    t = a2 * z;
    s = s + t;
    return s + b;
}

// Voxel (ix, iy, iz) holding grid coordinates g, if 0 <= g < n on every axis
// (NaN is outside).  g is clamped into [0, h] with h the largest float below n:
// a coordinate inside [0, n) is left unchanged (and -0.0 compares equal to its
// clamp, as -0.0 >= 0), anything else changes, NaN compares unequal; the clamped
// value converts to the voxel index exactly as (int)g would.
__device__ inline bool voxel_ijk(const MapView &m, float gx, float gy, float gz, uint32_t &ix,
                                 uint32_t &iy, uint32_t &iz) {
    float cx = __builtin_amdgcn_fmed3f(gx, 0.0f, m.hx);
    float cy = __builtin_amdgcn_fmed3f(gy, 0.0f, m.hy);
    float cz = __builtin_amdgcn_fmed3f(gz, 0.0f, m.hz);
    bool ok = (cx == gx) & (cy == gy) & (cz == gz);
    ix = (uint32_t)(int)cx;
    iy = (uint32_t)(int)cy;
    iz = (uint32_t)(int)cz;
    return ok;
}

// Byte offset of a voxel's value in the brick layout (bricks z-fastest, then x,
// then y; inside a brick z, y, x weigh 16, 4, 1).  The element index
//   64 (bz + nbz (bx + nbx by)) + 16 (iz & 3) + 4 (iy & 3) + (ix & 3)
// is separable per axis, with c = ~3:
//   Z = 16 iz,  X = ix + (16 nbz - 1)(ix & c),  Y = 4 iy + (16 nbz nbx - 4)(iy & c).
// cx, cy hold the two coefficients times ESIZE; the upload keeps them below 2^24.
template <int ESIZE>
__device__ inline uint32_t brick_offset(const MapView &m, uint32_t ix, uint32_t iy, uint32_t iz) {
    uint32_t a = __umul24(ix & ~3u, m.cx) + iz * (16u * ESIZE);
    uint32_t b = __umul24(iy & ~3u, m.cy) + a;
    return b + ix * (uint32_t)ESIZE + iy * (4u * ESIZE);
}

// Byte offset read for grid coordinates g: the voxel's, or the +Q sentinel outside.
template <int ESIZE>
__device__ inline uint32_t voxel_offset(const MapView &m, float gx, float gy, float gz) {
    uint32_t ix, iy, iz;
    bool ok = voxel_ijk(m, gx, gy, gz, ix, iy, iz);
    uint32_t off = brick_offset<ESIZE>(m, ix, iy, iz);
    return ok ? off : m.out_off;
}

}  // namespace mcl

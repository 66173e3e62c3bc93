// Device-side voxel addressing: the float32 index recipe and the brick layout.
// Shared by the sensor-update kernel and the index export, so both read the
// same voxel for every (particle, point) pair.
#pragma once

#include "mcl_internal.h"

namespace mcl {

// The same pointer in the global address space.  Pointers that reach a kernel
// through a job table in memory are generic to the compiler, which then emits
// FLAT loads with a 64-bit address add per load; every pointer here is to
// device memory, so loads through gp() are plain global loads.
template <typename T>
__device__ inline const __attribute__((address_space(1))) T *gp(const T *p) {
    return (const __attribute__((address_space(1))) T *)p;
}

// Per-particle constants of the index recipe (pose prologue):
//   a_jk = r_jk * inv_v  (pa[0..8]),  b_j = (t_j - o_j) * inv_v  (pa[9..11]).
// poses: [12][N] rows r00 .. r22 tx ty tz.
__device__ inline void pose_consts(const float *__restrict__ poses, int N, int n, const MapView &m,
                                   float pa[12]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int j = 0; j < 9; ++j) pa[j] = gp(poses)[(size_t)j * N + n] * m.inv_v;
    float dx = gp(poses)[(size_t)9 * N + n] - m.ox;
    float dy = gp(poses)[(size_t)10 * N + n] - m.oy;
    float dz = gp(poses)[(size_t)11 * N + n] - m.oz;
    // adding +0.0 turns a -0.0 offset into +0.0 and leaves every other value
    // unchanged, so that translations of -0.0 and +0.0 select alike
    pa[9] = dx * m.inv_v + 0.0f;
    pa[10] = dy * m.inv_v + 0.0f;
    pa[11] = dz * m.inv_v + 0.0f;
}

// One grid coordinate: fma(a2, z, fma(a1, y, fma(a0, x, b))), three fused
// multiply-adds, each rounded once.  With b not -0.0 an exact zero sum rounds
// to +0.0, so g is -0.0 only when a negative exact value is too small to be
// represented: such a point lies below 0.
__device__ inline float grid_coord(float a0, float a1, float a2, float b, float x, float y, float z) {
    return __builtin_fmaf(a2, z, __builtin_fmaf(a1, y, __builtin_fmaf(a0, x, b)));
}

// Voxel (ix, iy, iz) holding grid coordinates g, if 0 <= g < n on every axis,
// -0.0 counting as below 0 and NaN as outside: exactly when the bit pattern of
// g, read as an unsigned integer, is below that of n (non-negative floats order
// like their bit patterns; negative values, -0.0 and NaNs of either sign have
// patterns above any finite positive n).  The integer coordinates are (int)g;
// for a point outside the map they are meaningless and the caller must not
// use them (voxel_offset replaces the address by the sentinel's).
__device__ inline bool voxel_ijk(const MapView &m, float gx, float gy, float gz, uint32_t &ix,
                                 uint32_t &iy, uint32_t &iz) {
    bool ok = (int)(__float_as_uint(gx) < m.bx) & (int)(__float_as_uint(gy) < m.by) & (int)(__float_as_uint(gz) < m.bz);
    ix = (uint32_t)(int)gx;
    iy = (uint32_t)(int)gy;
    iz = (uint32_t)(int)gz;
    return ok;
}

// Byte offset of a voxel's value in the brick layout (bricks z-fastest, then x,
// then y; inside a brick x, y, z weigh 1, BX, BX BY).  With V = BX BY BZ the
// element index
//   V (bz + nbz (bx + nbx by)) + (ix & (BX-1)) + BX (iy & (BY-1)) + BX BY (iz & (BZ-1))
// is separable per axis (z is the fastest brick axis, so its two parts merge):
//   Z = BX BY iz,  X = ix + (V nbz / BX - 1)(ix & ~(BX-1)),
//   Y = BX iy + (V nbz nbx / BY - BX)(iy & ~(BY-1)).
// cx, cy hold the two coefficients times ESIZE; the upload keeps them below
// 2^24.  data0 skips the +Q sentinel brick in front.  Sums wrap modulo 2^32
// and the true offset is below 2^32, so the wrapped sum is exact.
//
// Evaluated as three shift-adds (ix + BX iy, + BX BY iz, ESIZE * that +
// data0) and two 24-bit multiply-adds: 7 instructions with the two masks.
// Left to itself the compiler merges the sums into shifts and three-way adds
// around plain 24-bit multiplies, 9 instructions; the empty asm statements
// pin each partial sum, so every step maps to one instruction.  The sensor
// kernel is partly bound by instruction issue, and the two saved instructions
// per evaluation took the global-localisation update from 19.96 to 19.08 ms.
template <int ESIZE>
__device__ inline uint32_t brick_offset(const MapView &m, uint32_t ix, uint32_t iy, uint32_t iz) {
    uint32_t lin = ix + (iy << kBLX);
    asm volatile("" : "+v"(lin));
    lin += iz << (kBLX + kBLY);
    asm volatile("" : "+v"(lin));
    uint32_t base = lin * (uint32_t)ESIZE + m.data0;
    asm volatile("" : "+v"(base));
    uint32_t t = __umul24(iy & ~(uint32_t)(kBY - 1), m.cy) + base;
    asm volatile("" : "+v"(t));
    return __umul24(ix & ~(uint32_t)(kBX - 1), m.cx) + t;
}

// Byte offset read for grid coordinates g: the voxel's, or the +Q sentinel
// (offset 0) outside.
template <int ESIZE>
__device__ inline uint32_t voxel_offset(const MapView &m, float gx, float gy, float gz) {
    uint32_t ix, iy, iz;
    bool ok = voxel_ijk(m, gx, gy, gz, ix, iy, iz);
    uint32_t off = brick_offset<ESIZE>(m, ix, iy, iz);
    return ok ? off : 0u;
}

// Trilinear lookup, one axis: the stored values sit at the voxel centres (grid
// coordinate i + 1/2), so the interpolation coordinate is h = g - 1/2, clamped
// to [-1, n] (this only moves points whose two centres are both outside, and
// sends NaN there: such points read +Q exactly, see the kernel); the lower
// centre is i = floor(h), the weight of the upper one f = h - floor(h) (exact).
// Returns i + 1, the index of the cell with lower corner i in the cell grid.
__device__ inline uint32_t tri_axis(float g, float hmax, float &f) {
    float h = g - 0.5f;
    h = fminf(fmaxf(h, -1.0f), hmax);
    const float fl = floorf(h);
    f = h - fl;
    return (uint32_t)((int32_t)fl + 1);
}

// Byte offset of cell (i, j, k) of the trilinear corner-cell grid (bricks of
// CX x CY x CZ cells, z-fastest, then x, then y; ESIZE bytes per cell):
//   data0 + ESIZE (i + CX j + CX CY k) + cx (i & ~(CX-1)) + cy (j & ~(CY-1)),
// separable as for the values, with the coefficients of TriView, and
// evaluated the same way (shift-add chain, two 24-bit multiply-adds).
template <int ESIZE>
__device__ inline uint32_t cell_offset(const TriView &tv, uint32_t ix, uint32_t iy, uint32_t iz) {
    uint32_t lin = ix + (iy << kCLX);
    asm volatile("" : "+v"(lin));
    lin += iz << (kCLX + kCLY);
    asm volatile("" : "+v"(lin));
    uint32_t base = lin * (uint32_t)ESIZE + tv.data0;
    asm volatile("" : "+v"(base));
    uint32_t t = __umul24(iy & ~(uint32_t)(kCY - 1), tv.cy) + base;
    asm volatile("" : "+v"(t));
    return __umul24(ix & ~(uint32_t)(kCX - 1), tv.cx) + t;
}

}  // namespace mcl

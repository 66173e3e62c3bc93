// TSDF map upload: dense x-fastest host array -> device brick layout + sentinels.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mcl_internal.h"
#include "voxel.h"

namespace mcl {

// Element e of the brick layout: brick bi = e / V = bz + nbz (bx + nbx by),
// value w = e % V = (ix % BX) + BX (iy % BY) + BX BY (iz % BZ), V = BX BY BZ.
// Padding voxels get 0 (never read).
__device__ inline void brick_voxel(int64_t bi, int w, int nbx, int nbz, int &ix, int &iy, int &iz) {
    const int bz = (int)(bi % nbz);
    const int64_t r = bi / nbz;
    const int bx = (int)(r % nbx);
    const int by = (int)(r / nbx);
    ix = bx * kBX + (w & (kBX - 1));
    iy = by * kBY + ((w >> kBLX) & (kBY - 1));
    iz = bz * kBZ + (w >> (kBLX + kBLY));
}

template <typename T>
__global__ __launch_bounds__(256) void brick_kernel(const T *__restrict__ dense, T *__restrict__ bricked,
                                                    int nx, int ny, int nz, int nbx, int nbz,
                                                    int64_t nvals) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nvals) return;
    int ix, iy, iz;
    brick_voxel(e >> kBrickLog2, (int)(e & (kBrickVals - 1)), nbx, nbz, ix, iy, iz);
    T v = T(0);
    if (ix < nx && iy < ny && iz < nz) v = dense[(int64_t)ix + (int64_t)nx * ((int64_t)iy + (int64_t)ny * iz)];
    bricked[e] = v;
}

// Read mask of every brick, stored at slot brick + 1 (slot 0 is the +Q
// sentinel in front): 0 if all its voxels inside the map hold +-Q (padding
// voxels beyond the map are ignored), else -1.
template <typename T>
__global__ __launch_bounds__(256) void brick_mask_kernel(const T *__restrict__ bricked, int8_t *__restrict__ mask,
                                                         int nx, int ny, int nz, int nbx, int nbz, int64_t nbricks,
                                                         T qpos, T qneg) {
    int64_t bi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (bi >= nbricks) return;
    const T *b = bricked + bi * kBrickVals;
    bool trunc = true;
    for (int w = 0; w < kBrickVals; ++w) {
        int ix, iy, iz;
        brick_voxel(bi, w, nbx, nbz, ix, iy, iz);
        if (ix < nx && iy < ny && iz < nz) trunc &= (b[w] == qpos) | (b[w] == qneg);
    }
    mask[bi + 1] = trunc ? int8_t(0) : int8_t(-1);
}

// The masks as bits: bit b of word w is set when slot 32 w + b is read in place.
__global__ __launch_bounds__(256) void read_bits_kernel(const int8_t *__restrict__ mask, int64_t nslots,
                                                        uint32_t *__restrict__ bits, int64_t nwords) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    uint32_t v = 0;
    for (int b = 0; b < 32; ++b) {
        const int64_t i = w * 32 + b;
        if (i < nslots && mask[i] != 0) v |= 1u << b;
    }
    bits[w] = v;
}

template <typename T>
static void fill_sentinels(char *qpos, char *zero, T outside) {
    for (int w = 0; w < kBrickVals; ++w) {
        reinterpret_cast<T *>(qpos)[w] = outside;  // +Q sentinel brick at offset 0
        reinterpret_cast<T *>(zero)[w] = T(0);     // zero sentinel brick after the data
    }
}

// Cell e of the corner-cell layout (see TriView): cell (i, j, k) of the cell
// grid holds map voxels (i - 1 + a, j - 1 + b, k - 1 + c), a, b, c in {0, 1},
// as value a + 2 b + 4 c, read from the main brick layout, or +Q outside.
template <typename T>
__global__ __launch_bounds__(256) void tri_build_kernel(MapView src, T *__restrict__ dst, int nbx, int nbz,
                                                        int64_t ncells, T outside) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ncells) return;
    const int64_t bi = e >> kCellBrickLog2;
    const int w = (int)(e & (kCellBrickVals - 1));
    const int bz = (int)(bi % nbz);
    const int64_t r = bi / nbz;
    const int bx = (int)(r % nbx);
    const int by = (int)(r / nbx);
    const int ix = bx * kCX + (w & (kCX - 1)) - 1;
    const int iy = by * kCY + ((w >> kCLX) & (kCY - 1)) - 1;
    const int iz = bz * kCZ + (w >> (kCLX + kCLY)) - 1;
    for (int c = 0; c < 8; ++c) {
        int x = ix + (c & 1), y = iy + ((c >> 1) & 1), z = iz + (c >> 2);
        T v = outside;
        if (x >= 0 && y >= 0 && z >= 0 && x < src.nx && y < src.ny && z < src.nz)
            v = *reinterpret_cast<const T *>(src.base + brick_offset<sizeof(T)>(src, (uint32_t)x, (uint32_t)y, (uint32_t)z));
        dst[e * 8 + c] = v;
    }
}

// Read mask of every brick of cells, at slot brick + 1 (slot 0: the sentinel):
// 0 if all 8 corners of all its cells are +Q, or all are -Q, else -1.
template <typename T>
__global__ __launch_bounds__(256) void tri_mask_kernel(const T *__restrict__ cells, int8_t *__restrict__ mask,
                                                       int64_t nbricks, T qpos, T qneg) {
    int64_t bi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (bi >= nbricks) return;
    const T *b = cells + bi * kCellBrickVals * 8;
    bool pos = true, neg = true;
    for (int w = 0; w < kCellBrickVals * 8; ++w) {
        pos &= b[w] == qpos;
        neg &= b[w] == qneg;
    }
    mask[bi + 1] = (pos || neg) ? int8_t(0) : int8_t(-1);
}

static std::mutex g_tri_mu;

mcl_status ensure_trilinear(mcl_map_s *m, hipStream_t stream) {
    if (m->sparse) return fail(MCL_EINVAL, "trilinear: not available for sparse maps (mcl_map_upload_bricks)");
    std::lock_guard<std::mutex> lk(g_tri_mu);
    if (m->tri_dev) return MCL_OK;
    const MapView &v = m->view;
    const int es = 8 * elem_size(m->dtype);  // bytes per cell
    const int64_t px = v.nx + 2, py = v.ny + 2, pz = v.nz + 2;
    const int64_t nbx = (px + kCX - 1) / kCX, nby = (py + kCY - 1) / kCY, nbz = (pz + kCZ - 1) / kCZ;
    const int64_t nvals = nbx * nby * nbz * kCellBrickVals;  // cells
    const int64_t nbricks = nvals / kCellBrickVals;
    const int64_t brick_bytes = (int64_t)kCellBrickVals * es;
    const int64_t data0 = brick_bytes;  // +Q sentinel brick of cells in front
    const int64_t mask_off = (data0 + nvals * es + 255) / 256 * 256;
    const int64_t bytes = mask_off + (nbricks + 1 + 255) / 256 * 256;
    const int64_t cx = (int64_t)es * (kCellBrickVals / kCX * nbz - 1);
    const int64_t cy = (int64_t)es * (kCellBrickVals / kCY * nbz * nbx - kCX);
    if (bytes >= ((int64_t)1 << 32) || cy >= ((int64_t)1 << 24) || cx >= ((int64_t)1 << 24))
        return fail(MCL_ERANGE, "trilinear: the corner-cell map exceeds the brick addressing limits");
    void *dev = nullptr;
    if (hipMalloc(&dev, (size_t)bytes) != hipSuccess) return fail(MCL_ENOMEM, "trilinear: device allocation failed");
    char *base = static_cast<char *>(dev);
    int8_t *mask = reinterpret_cast<int8_t *>(base + mask_off);
    std::vector<char> sent((size_t)brick_bytes);
    for (int64_t c = 0; c < kCellBrickVals * 8; ++c) {
        if (m->dtype == MCL_TSDF_I16) reinterpret_cast<int16_t *>(sent.data())[c] = 32767;
        else if (m->dtype == MCL_TSDF_I8) reinterpret_cast<int8_t *>(sent.data())[c] = 127;
        else reinterpret_cast<float *>(sent.data())[c] = m->tau;
    }
    const int8_t sent_mask = 0;
    mcl_status st = MCL_OK;
    if (hipMemcpyAsync(base, sent.data(), (size_t)brick_bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(mask, &sent_mask, 1, hipMemcpyHostToDevice, stream) != hipSuccess)
        st = fail(MCL_EDEVICE, "trilinear: sentinel copy failed");
    const unsigned blocks = (unsigned)((nvals + 255) / 256);
    const unsigned cblocks = (unsigned)((nbricks + 255) / 256);
    if (st == MCL_OK) {
        char *cells = base + data0;
        if (m->dtype == MCL_TSDF_I16) {
            tri_build_kernel<int16_t><<<blocks, 256, 0, stream>>>(v, (int16_t *)cells, (int)nbx, (int)nbz, nvals, (int16_t)32767);
            tri_mask_kernel<int16_t><<<cblocks, 256, 0, stream>>>((const int16_t *)cells, mask, nbricks, (int16_t)32767,
                                                                  (int16_t)-32767);
        } else if (m->dtype == MCL_TSDF_I8) {
            tri_build_kernel<int8_t><<<blocks, 256, 0, stream>>>(v, (int8_t *)cells, (int)nbx, (int)nbz, nvals, (int8_t)127);
            tri_mask_kernel<int8_t><<<cblocks, 256, 0, stream>>>((const int8_t *)cells, mask, nbricks, (int8_t)127,
                                                                 (int8_t)-127);
        } else {
            tri_build_kernel<float><<<blocks, 256, 0, stream>>>(v, (float *)cells, (int)nbx, (int)nbz, nvals, m->tau);
            tri_mask_kernel<float><<<cblocks, 256, 0, stream>>>((const float *)cells, mask, nbricks, m->tau, -m->tau);
        }
        st = check_launch("tri_build_kernel / tri_mask_kernel");
    }
    if (st == MCL_OK && hipStreamSynchronize(stream) != hipSuccess)
        st = fail(MCL_EDEVICE, "trilinear: synchronisation failed");
    if (st != MCL_OK) {
        (void)hipFree(dev);
        return st;
    }
    TriView t{};
    t.base = static_cast<const char *>(dev);
    t.cx = (uint32_t)cx;
    t.cy = (uint32_t)cy;
    t.data0 = (uint32_t)data0;
    t.hx = (float)v.nx;
    t.hy = (float)v.ny;
    t.hz = (float)v.nz;
    t.mask = mask;
    m->tri = t;
    m->tri_bytes = (size_t)bytes;
    m->tri_dev = dev;
    return MCL_OK;
}

static mcl_status check_desc(const mcl_map_desc &d, const char *what) {
    const std::string w(what);
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) return fail(MCL_EINVAL, w + ": dimensions must be >= 1");
    if (d.nx >= (1 << 24) || d.ny >= (1 << 24) || d.nz >= (1 << 24))
        return fail(MCL_ERANGE, w + ": dimensions must be below 2^24");
    if (!(std::isfinite(d.voxel) && d.voxel > 0.0f)) return fail(MCL_EINVAL, w + ": voxel must be finite and > 0");
    if (!(std::isfinite(d.tau) && d.tau > 0.0f)) return fail(MCL_EINVAL, w + ": tau must be finite and > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(d.origin[a])) return fail(MCL_EINVAL, w + ": origin must be finite");
    if (d.dtype < MCL_TSDF_I16 || d.dtype > MCL_TSDF_F32) return fail(MCL_EINVAL, w + ": unknown dtype");
    return MCL_OK;
}

// The fields of a map handle that both layouts share: grid, index recipe, scale.
static void fill_common(mcl_map_s *m, const mcl_map_desc &d) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    m->device = dev;
    m->dtype = d.dtype;
    m->Q = d.dtype == MCL_TSDF_I16 ? 32767 : d.dtype == MCL_TSDF_I8 ? 127 : 1;
    m->tau = d.tau;
    m->voxel = d.voxel;
    m->scale = d.dtype == MCL_TSDF_F32 ? 1.0 : (double)d.tau / (double)m->Q;
    MapView &v = m->view;
    v.nx = d.nx; v.ny = d.ny; v.nz = d.nz;
    v.nbx = (d.nx + kBX - 1) / kBX; v.nby = (d.ny + kBY - 1) / kBY; v.nbz = (d.nz + kBZ - 1) / kBZ;
    float fx = (float)d.nx, fy = (float)d.ny, fz = (float)d.nz;
    std::memcpy(&v.bx, &fx, 4);
    std::memcpy(&v.by, &fy, 4);
    std::memcpy(&v.bz, &fz, 4);
    v.inv_v = (float)(1.0 / (double)d.voxel);
    v.ox = d.origin[0]; v.oy = d.origin[1]; v.oz = d.origin[2];
}

}  // namespace mcl

using namespace mcl;

extern "C" mcl_status mcl_map_upload_bricks(const mcl_map_desc *desc, int64_t nstored, const int32_t *brick_coords,
                                            const void *brick_values, void *stream_, mcl_map *out) {
    if (!desc || !out || (nstored > 0 && (!brick_coords || !brick_values)))
        return fail(MCL_EINVAL, "map_upload_bricks: NULL argument");
    *out = nullptr;
    const mcl_map_desc &d = *desc;
    mcl_status st = check_desc(d, "map_upload_bricks");
    if (st != MCL_OK) return st;
    if (nstored < 0) return fail(MCL_EINVAL, "map_upload_bricks: nstored must be >= 0");
    const int64_t nbx = (d.nx + 3) / 4, nby = (d.ny + 3) / 4, nbz = (d.nz + 3) / 4;
    const int64_t nbricks = nbx * nby * nbz;
    // super-brick grid: kSX x kSY x kSZ voxels = (kSX/4) x (kSY/4) x (kSZ/4) listed bricks
    constexpr int PX = kSX / 4, PY = kSY / 4, PZ = kSZ / 4;
    const int64_t nsx = (nbx + PX - 1) / PX, nsy = (nby + PY - 1) / PY, nsz = (nbz + PZ - 1) / PZ;
    const int64_t nsuper = nsx * nsy * nsz;
    if (nbricks >= ((int64_t)1 << 31) || nsx * nsy >= ((int64_t)1 << 24) || nstored + 2 >= ((int64_t)1 << 31))
        return fail(MCL_ERANGE,
                    "map_upload_bricks: too many bricks (need nbx*nby*nbz < 2^31 and ceil(nx/8)*ceil(ny/32) < 2^24)");
    const int es = elem_size(d.dtype);
    // which input brick sits at each brick index (-1: not stored), and which super-bricks hold one
    std::vector<int32_t> at((size_t)nbricks, -1);
    std::vector<uint8_t> held((size_t)nsuper, 0);
    for (int64_t i = 0; i < nstored; ++i) {
        const int32_t bx = brick_coords[3 * i], by = brick_coords[3 * i + 1], bz = brick_coords[3 * i + 2];
        if (bx < 0 || by < 0 || bz < 0 || bx >= nbx || by >= nby || bz >= nbz)
            return fail(MCL_EINVAL, "map_upload_bricks: brick " + std::to_string(i) + " outside the grid");
        int32_t &slot = at[(size_t)(bz + nbz * (bx + nbx * (int64_t)by))];
        if (slot >= 0) return fail(MCL_EINVAL, "map_upload_bricks: brick " + std::to_string(i) + " listed twice");
        slot = (int32_t)i;
        held[(size_t)(bx / PX + nsx * (by / PY + nsy * (int64_t)(bz / PZ)))] = 1;
    }
    // the pool (slot 0 +Q, slot 1 zeros, then the stored super-bricks in index order)
    int64_t nheld = 0;
    for (uint8_t h : held) nheld += h;
    const size_t super_bytes = (size_t)kSuperVals * es;
    const size_t pool_bytes = (size_t)(nheld + 2) * super_bytes;
    const bool small = pool_bytes < ((size_t)1 << 32);
    if (!small && nheld + 2 >= ((int64_t)1 << 32)) return fail(MCL_ERANGE, "map_upload_bricks: too many stored super-bricks");
    std::vector<char> pool_h(pool_bytes, 0);
    auto fill_q = [&](char *dst) {
        for (int w = 0; w < kSuperVals; ++w) {
            if (d.dtype == MCL_TSDF_I16) reinterpret_cast<int16_t *>(dst)[w] = 32767;
            else if (d.dtype == MCL_TSDF_I8) reinterpret_cast<int8_t *>(dst)[w] = 127;
            else reinterpret_cast<float *>(dst)[w] = d.tau;
        }
    };
    fill_q(pool_h.data());
    // table: per super-brick the byte offset (or slot) of its pool slot; then outside, padding
    std::vector<uint32_t> table((size_t)nsuper + 2, 0u);
    auto entry = [&](int64_t slot) { return small ? (uint32_t)((size_t)slot * super_bytes) : (uint32_t)slot; };
    table[(size_t)nsuper] = entry(0);
    table[(size_t)nsuper + 1] = entry(1);
    const char *src = static_cast<const char *>(brick_values);
    int64_t next = 2;
    for (int64_t si = 0; si < nsuper; ++si) {
        if (!held[(size_t)si]) {
            table[(size_t)si] = entry(0);
            continue;
        }
        table[(size_t)si] = entry(next);
        char *dst = pool_h.data() + (size_t)next * super_bytes;
        ++next;
        fill_q(dst);
        const int64_t sx = si % nsx, rr = si / nsx, sy = rr % nsy, sz = rr / nsy;
        for (int c = 0; c < PX * PY * PZ; ++c) {
            const int64_t bx = sx * PX + c % PX, by = sy * PY + (c / PX) % PY, bz = sz * PZ + c / (PX * PY);
            if (bx >= nbx || by >= nby || bz >= nbz) continue;
            const int32_t i = at[(size_t)(bz + nbz * (bx + nbx * by))];
            if (i < 0) continue;
            const char *b = src + (size_t)i * 64 * es;  // listed brick, in-brick index x + 4 y + 16 z
            for (int v = 0; v < 64; ++v) {
                const int x = (int)(bx - sx * PX) * 4 + (v & 3), y = (int)(by - sy * PY) * 4 + ((v >> 2) & 3),
                          z = (int)(bz - sz * PZ) * 4 + (v >> 4);
                std::memcpy(dst + (size_t)(x + kSX * (y + kSY * z)) * es, b + (size_t)v * es, es);
            }
        }
    }
    mcl_map_s *m = new (std::nothrow) mcl_map_s();
    if (!m) return fail(MCL_ENOMEM, "map_upload_bricks: host allocation failed");
    if (hipMalloc(&m->sp_table, table.size() * 4) != hipSuccess) {
        delete m;
        return fail(MCL_ENOMEM, "map_upload_bricks: device allocation failed");
    }
    if (hipMalloc(&m->sp_pool, pool_bytes) != hipSuccess) {
        (void)hipFree(m->sp_table);
        delete m;
        return fail(MCL_ENOMEM, "map_upload_bricks: device allocation failed");
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    bool ok = hipMemcpyAsync(m->sp_table, table.data(), table.size() * 4, hipMemcpyHostToDevice, stream) == hipSuccess &&
              hipMemcpyAsync(m->sp_pool, pool_h.data(), pool_bytes, hipMemcpyHostToDevice, stream) == hipSuccess &&
              hipStreamSynchronize(stream) == hipSuccess;
    if (!ok) {
        (void)hipFree(m->sp_table);
        (void)hipFree(m->sp_pool);
        delete m;
        return fail(MCL_EDEVICE, "map_upload_bricks: copy to device failed");
    }
    fill_common(m, d);
    m->sparse = true;
    m->bytes = table.size() * 4 + pool_bytes;
    m->sp.table = static_cast<const uint32_t *>(m->sp_table);
    m->sp.pool = static_cast<const char *>(m->sp_pool);
    m->sp.nsx = (uint32_t)nsx;
    m->sp.nsxy = (uint32_t)(nsx * nsy);
    m->sp.outside = (uint32_t)nsuper;
    m->sp.pad = (uint32_t)nsuper + 1;
    m->sp.small = small ? 1u : 0u;
    *out = m;
    return MCL_OK;
}

extern "C" mcl_status mcl_map_upload(const mcl_map_desc *desc, const void *host_values, void *stream_,
                                     mcl_map *out) {
    if (!desc || !host_values || !out) return fail(MCL_EINVAL, "map_upload: NULL argument");
    *out = nullptr;
    const mcl_map_desc &d = *desc;
    {
        mcl_status cst = check_desc(d, "map_upload");
        if (cst != MCL_OK) return cst;
    }
    const int es = elem_size(d.dtype);
    const int64_t nbx = (d.nx + kBX - 1) / kBX, nby = (d.ny + kBY - 1) / kBY, nbz = (d.nz + kBZ - 1) / kBZ;
    const int64_t nvals = nbx * nby * nbz * kBrickVals;
    const int64_t nbricks = nvals / kBrickVals;
    const int64_t brick_bytes = (int64_t)kBrickVals * es;
    const int64_t data0 = brick_bytes;                              // +Q sentinel brick in front
    const int64_t zero_off = data0 + nvals * es;                    // zero sentinel brick after the data
    const int64_t nslots = nbricks + 2;
    const int64_t mask_off = (zero_off + brick_bytes + 255) / 256 * 256;
    const int64_t nrwords = (nslots + 31) / 32;
    const int64_t bits_off = mask_off + (nslots + 255) / 256 * 256;
    const int64_t total = bits_off + (nrwords * 4 + 255) / 256 * 256;
    if (total >= ((int64_t)1 << 32)) return fail(MCL_ERANGE, "map_upload: map exceeds the 4 GiB device layout limit");
    const int64_t cx = (int64_t)es * (kBrickVals / kBX * nbz - 1);
    const int64_t cy = (int64_t)es * (kBrickVals / kBY * nbz * nbx - kBX);
    if (cy >= ((int64_t)1 << 24) || cx >= ((int64_t)1 << 24))
        return fail(MCL_ERANGE, "map_upload: nz * nx too large for the brick addressing (need 16*nbz*nbx*esize < 2^24)");
    const int64_t dense_vals = (int64_t)d.nx * d.ny * d.nz;
    hipStream_t stream = static_cast<hipStream_t>(stream_);

    mcl_map_s *m = new (std::nothrow) mcl_map_s();
    if (!m) return fail(MCL_ENOMEM, "map_upload: host allocation failed");
    void *dense_dev = nullptr;
    if (hipMalloc(&m->dev, (size_t)total) != hipSuccess) {
        delete m;
        return fail(MCL_ENOMEM, "map_upload: device allocation failed");
    }
    if (hipMalloc(&dense_dev, (size_t)(dense_vals * es)) != hipSuccess) {
        (void)hipFree(m->dev);
        delete m;
        return fail(MCL_ENOMEM, "map_upload: staging allocation failed");
    }
    mcl_status st = MCL_OK;
    char sent_q[kBrickVals * 4] = {0}, sent_z[kBrickVals * 4] = {0};
    if (d.dtype == MCL_TSDF_I16) fill_sentinels<int16_t>(sent_q, sent_z, (int16_t)32767);
    else if (d.dtype == MCL_TSDF_I8) fill_sentinels<int8_t>(sent_q, sent_z, (int8_t)127);
    else fill_sentinels<float>(sent_q, sent_z, d.tau);
    const int8_t sent_mask[2] = {0, -1};  // +Q sentinel: read slot 0 (itself); zero sentinel: read in place
    char *base = static_cast<char *>(m->dev);
    int8_t *mask = reinterpret_cast<int8_t *>(base + mask_off);
    if (hipMemcpyAsync(dense_dev, host_values, (size_t)(dense_vals * es), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(base, sent_q, (size_t)brick_bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(base + zero_off, sent_z, (size_t)brick_bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(mask, &sent_mask[0], 1, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(mask + nbricks + 1, &sent_mask[1], 1, hipMemcpyHostToDevice, stream) != hipSuccess) {
        st = fail(MCL_EDEVICE, "map_upload: copy to device failed");
    } else {
        unsigned blocks = (unsigned)((nvals + 255) / 256);
        char *data = base + data0;
        if (d.dtype == MCL_TSDF_I16)
            brick_kernel<int16_t><<<blocks, 256, 0, stream>>>((const int16_t *)dense_dev, (int16_t *)data, d.nx, d.ny, d.nz, (int)nbx, (int)nbz, nvals);
        else if (d.dtype == MCL_TSDF_I8)
            brick_kernel<int8_t><<<blocks, 256, 0, stream>>>((const int8_t *)dense_dev, (int8_t *)data, d.nx, d.ny, d.nz, (int)nbx, (int)nbz, nvals);
        else
            brick_kernel<float><<<blocks, 256, 0, stream>>>((const float *)dense_dev, (float *)data, d.nx, d.ny, d.nz, (int)nbx, (int)nbz, nvals);
        st = check_launch("brick_kernel");
        unsigned cblocks = (unsigned)((nbricks + 255) / 256);
        if (st == MCL_OK) {
            if (d.dtype == MCL_TSDF_I16)
                brick_mask_kernel<int16_t><<<cblocks, 256, 0, stream>>>((const int16_t *)data, mask, d.nx, d.ny, d.nz, (int)nbx, (int)nbz, nbricks, (int16_t)32767, (int16_t)-32767);
            else if (d.dtype == MCL_TSDF_I8)
                brick_mask_kernel<int8_t><<<cblocks, 256, 0, stream>>>((const int8_t *)data, mask, d.nx, d.ny, d.nz, (int)nbx, (int)nbz, nbricks, (int8_t)127, (int8_t)-127);
            else
                brick_mask_kernel<float><<<cblocks, 256, 0, stream>>>((const float *)data, mask, d.nx, d.ny, d.nz, (int)nbx, (int)nbz, nbricks, d.tau, -d.tau);
            st = check_launch("brick_mask_kernel");
        }
        if (st == MCL_OK) {
            read_bits_kernel<<<(unsigned)((nrwords + 255) / 256), 256, 0, stream>>>(
                mask, nslots, reinterpret_cast<uint32_t *>(base + bits_off), nrwords);
            st = check_launch("read_bits_kernel");
        }
        if (st == MCL_OK && hipStreamSynchronize(stream) != hipSuccess) st = fail(MCL_EDEVICE, "map_upload: synchronisation failed");
    }
    (void)hipFree(dense_dev);
    if (st != MCL_OK) {
        (void)hipFree(m->dev);
        delete m;
        return st;
    }
    fill_common(m, d);
    m->bytes = (size_t)total;
    MapView &v = m->view;
    v.base = static_cast<const char *>(m->dev);
    v.cx = (uint32_t)cx;
    v.cy = (uint32_t)cy;
    v.data0 = (uint32_t)data0;
    v.zero_off = (uint32_t)zero_off;
    v.mask = reinterpret_cast<const int8_t *>(base + mask_off);
    v.rbits = reinterpret_cast<const uint32_t *>(base + bits_off);
    v.nrwords = (uint32_t)nrwords;
    *out = m;
    return MCL_OK;
}

extern "C" size_t mcl_map_bytes(mcl_map map) { return map ? map->bytes + map->tri_bytes : 0; }

namespace mcl {
mcl_status note_map_use(mcl_map_s *map, hipStream_t stream) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return fail(MCL_EDEVICE, "map use: stream query failed");
    if (cs != hipStreamCaptureStatusNone) return MCL_OK;
    std::lock_guard<std::mutex> lk(map->uses_mu);
    hipEvent_t ev = nullptr;
    for (auto &u : map->uses)
        if (u.first == stream) ev = u.second;
    if (!ev) {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            return fail(MCL_EDEVICE, "map use: event creation failed");
        map->uses.emplace_back(stream, ev);
    }
    if (hipEventRecord(ev, stream) != hipSuccess) return fail(MCL_EDEVICE, "map use: event record failed");
    return MCL_OK;
}
}  // namespace mcl

extern "C" mcl_status mcl_map_free(mcl_map map) {
    if (!map) return fail(MCL_EINVAL, "map_free: NULL map");
    hipError_t e = hipSuccess;
    {
        // deferred: the work enqueued on the map completes before its memory goes
        std::lock_guard<std::mutex> lk(map->uses_mu);
        for (auto &u : map->uses) {
            if (hipEventSynchronize(u.second) != hipSuccess) e = hipErrorInvalidValue;
            (void)hipEventDestroy(u.second);
        }
        map->uses.clear();
    }
    if (e != hipSuccess) {
        delete map;
        return fail(MCL_EDEVICE, "map_free: waiting for the map's work failed (its memory is kept)");
    }
    if (map->dev) e = hipFree(map->dev);
    if (map->sp_table && hipFree(map->sp_table) != hipSuccess) e = hipErrorInvalidValue;
    if (map->sp_pool && hipFree(map->sp_pool) != hipSuccess) e = hipErrorInvalidValue;
    if (map->tri_dev && hipFree(map->tri_dev) != hipSuccess) e = hipErrorInvalidValue;
    if (map->free_prefix && hipFree(map->free_prefix) != hipSuccess) e = hipErrorInvalidValue;
    delete map;
    return e == hipSuccess ? MCL_OK : fail(MCL_EDEVICE, "map_free: hipFree failed");
}

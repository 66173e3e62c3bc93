// Internal declarations of the HIP library (device layout, launch helpers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "mcl.h"

namespace mcl {

constexpr int kWave = 64;

// ---------------------------------------------------------------- map layout
// The dense grid is padded to whole bricks of 8 x 32 x 4 voxels (x, y, z); one
// brick (1024 values) is one contiguous run, x fastest, then y, then z, so an
// int16 line of 128 bytes holds an 8 x 8 patch of one z-layer.  Bricks are
// ordered z fastest, then x, then y (maps are flat: nz is the short axis),
// which keeps every address coefficient below 2^24 for 24-bit multiplies.  The
// allocation starts with a sentinel brick of +Q (read by points outside the map
// and instead of every brick wholly at +-Q), then the bricks, then a sentinel
// brick of zeros (read by padding lanes past the end of a scan, contributing
// nothing).
//
// Why this shape: the texture units spend their cycles per cache line a
// wave-wide gather touches.  The 64 lanes of a gather hold consecutive beams of
// one LiDAR ring, which sweep sideways at nearly one height; flat, elongated
// bricks put those points in fewer value lines, and a brick read mask (below)
// then covers a larger horizontal patch, so the mask lines touched per gather
// drop too.  Measured against 4 x 4 x 4 bricks on a 1024 x 1024 x 128 map with
// a VLP-16-shaped scan, 10^6 particles: 12 % less time under global
// localisation, 32 % less with the particles converged round one pose.
//
// Beside the values sits the coarse level of the map: per brick (and per
// sentinel, in address order) a read mask, -1 if the brick has any value
// inside the truncation band (read in place) and 0 if every voxel holds +-Q.
// Only q^2 enters the score, so such a brick scores Q^2 for any point: the
// lookup reads address (offset AND mask), which is the +Q sentinel at offset 0.
// The masks are kept twice: as signed bytes in global memory, and as bits
// (1 = read in place) small enough for the sensor kernel to hold in LDS.
constexpr int kBLX = 3, kBLY = 5, kBLZ = 2;                 // log2 of the brick shape
constexpr int kBX = 1 << kBLX, kBY = 1 << kBLY, kBZ = 1 << kBLZ;
constexpr int kBrickLog2 = kBLX + kBLY + kBLZ;
constexpr int kBrickVals = 1 << kBrickLog2;                 // 1024

struct MapView {
    const char *base;        // device: bricked values, then the sentinels
    int32_t nx, ny, nz;      // true dimensions
    int32_t nbx, nby, nbz;   // bricks per axis (dense layout)
    uint32_t bx, by, bz;     // bit patterns of (float)nx, ny, nz (bounds test)
    float inv_v;             // (float)(1.0 / (double)voxel)
    float ox, oy, oz;        // origin
    uint32_t cx, cy;         // ESIZE (V nbz / BX - 1), ESIZE (V nbz nbx / BY - BX), V = BX BY BZ
    uint32_t data0;          // byte offset of the first brick (after the +Q sentinel brick at 0)
    uint32_t zero_off;       // byte offset of the 0 sentinel brick
    const int8_t *mask;      // device: read mask per brick slot, indexed by byte offset >> (kBrickLog2 + log2 esize)
    const uint32_t *rbits;   // device: the same masks as bits, bit b of word w for slot 32 w + b
    uint32_t nrwords;        // words of rbits (bricks + 2 sentinels, rounded up to 32)
};
// Largest read-bit table the sensor kernel copies into LDS (bytes); maps with
// more bricks use the mask bytes in global memory.
constexpr uint32_t kMaxLdsBits = 64 * 1024;

// The map for the trilinear lookup, one gather per point: cell (i, j, k) holds
// the 8 voxel values at its corners (i..i+1, j..j+1, k..k+1), x fastest, so an
// interpolation reads one 16-byte run (int16; 8 bytes int8, 32 bytes float32).
// Cells span i in [-1, n] per axis (corners outside the map hold +Q) and are
// stored at index i + 1 in bricks of CX x CY x CZ cells, x fastest inside a
// brick, bricks ordered like the value bricks; a +Q sentinel brick of cells
// comes first, at offset 0.  Eight times the map's memory (HBM is plentiful,
// gathers are not).  As for the values, each brick of cells has a read mask,
// -1 (read in place) unless every corner of its cells is +Q or every one is
// -Q: such a cell interpolates to exactly +-Q, and only the square enters the
// score, so the lookup reads offset (offset AND mask) = 0, the sentinel.
// Built on first use of the trilinear lookup.
struct TriView {
    const char *base;        // device: sentinel brick, then the bricked corner cells
    uint32_t cx, cy;         // brick address coefficients of the cell grid (bytes)
    uint32_t data0;          // byte offset of the first brick of cells
    float hx, hy, hz;        // (float)n per axis: upper clamp of h
    const int8_t *mask;      // read mask per brick slot, indexed by byte offset >> (log2 cells per brick + log2 cell bytes)
};
constexpr int kCLX = 2, kCLY = 2, kCLZ = 2;                      // log2 of the cell-brick shape
constexpr int kCX = 1 << kCLX, kCY = 1 << kCLY, kCZ = 1 << kCLZ;
constexpr int kCellBrickLog2 = kCLX + kCLY + kCLZ;
constexpr int kCellBrickVals = 1 << kCellBrickLog2;

// Sparse coarse/fine map (§III: the map holds fine data only for the coarse
// cells with distances inside the truncation band, after Akai et al.).  The
// caller lists 4x4x4 bricks; the library stores them in super-bricks of
// SX x SY x SZ voxels (flat, like the dense bricks and for the same reason: the
// beams of one gather fall in fewer lines), a super-brick being stored when
// any of its bricks is listed, its unlisted bricks holding +Q.  A pool of the
// stored super-bricks (x fastest inside) and the coarse level: a table with one
// 32-bit entry per super-brick, the byte offset of its slot in the pool, or of
// slot 0 (all +Q) when it is not stored.  The table runs x fastest, then y,
// then z (super index = sx + nsx (sy + nsy sz)): a 128-byte line of entries is
// a 12.8 m x 1.6 m strip (at 5 cm voxels) of one height layer, and the beams of
// one gather sweep sideways at nearly one height, so they share few lines
// (2.4 lines per gather on the warehouse workload against 3.8 with z fastest).
// Two more entries follow for points outside the map (slot 0) and for padding
// lanes (slot 1, all zeros).  With super-bricks the table is small (0.5 MiB for a
// 1024 x 1024 x 128 map) and stays in L2, so a lookup is two dependent gathers
// (table entry, then value) and no rank arithmetic.  Pools of 4 GiB and more
// keep slot numbers in the table and 64-bit addresses.
constexpr int kSLX = 3, kSLY = 5, kSLZ = 2;                      // log2 of the super-brick shape (voxels)
constexpr int kSX = 1 << kSLX, kSY = 1 << kSLY, kSZ = 1 << kSLZ;
constexpr int kSuperLog2 = kSLX + kSLY + kSLZ;
constexpr int kSuperVals = 1 << kSuperLog2;
struct SparseView {
    const uint32_t *table;   // device [nsuper + 2]: byte offset (or slot, wide pools) per super-brick
    const char *pool;        // device [nslots][kSuperVals] values
    uint32_t nsx, nsxy;      // super index = sx + nsx sy + nsx nsy sz (both < 2^24)
    uint32_t outside, pad;   // table indices of the outside (+Q) and padding (zero) entries
    uint32_t small;          // pool below 4 GiB: the table holds byte offsets
};

}  // namespace mcl

struct mcl_map_s {
    mcl::MapView view;
    void *dev;          // allocation holding bricks + sentinels
    size_t bytes;
    int device;
    int32_t dtype;
    int32_t Q;          // 32767, 127 or 1
    float tau;
    float voxel;
    double scale;       // metres per stored unit: tau / Q, or 1 for float32
    void *tri_dev;      // corner cells for the trilinear lookup, or null
    size_t tri_bytes;
    mcl::TriView tri;
    void *free_prefix;  // free voxels before each 64-voxel row chunk (uniform initialisation), or null
    uint64_t free_total;
    bool sparse;        // coarse table + brick pool (view.base and view.mask unused)
    mcl::SparseView sp;
    void *sp_table, *sp_pool;
    // Work enqueued on the map: one event per stream that has read it, recorded
    // after the last such work (mcl_map_free waits for all of them).
    std::mutex uses_mu;
    std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
};

namespace mcl {
// Builds map->tri on first use (allocation + one kernel, then a synchronisation
// of `stream`); later calls return at once.
mcl_status ensure_trilinear(mcl_map_s *map, hipStream_t stream);
}  // namespace mcl

namespace mcl {

// thread-local last error
void set_error(const std::string &msg);
mcl_status fail(mcl_status code, const std::string &msg);
mcl_status check_launch(const char *what);

// Workspace per stream, grown on demand (never shrinks until unload).
void *workspace(hipStream_t stream, size_t bytes);

// Record that work reading `map` has been enqueued on `stream` (an event after
// it, so that mcl_map_free can wait for it).  Nothing is recorded while the
// stream is being captured into a graph.
mcl_status note_map_use(mcl_map_s *map, hipStream_t stream);

inline int elem_size(int32_t dtype) { return dtype == MCL_TSDF_I16 ? 2 : dtype == MCL_TSDF_I8 ? 1 : 4; }

}  // namespace mcl

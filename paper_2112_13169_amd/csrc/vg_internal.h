// vg_internal.h -- parameter blocks and kernel launchers shared by the host
// API (vg_api.cpp) and the gfx950 kernels (vg_kernels.hip).  Not installed.
//
// Device layout of a grid: rows of gx voxels are stored with a pitch of
// gxp = 32 * ceil(gx / 32) bytes (voxel (x, y, z) at x + gxp * (y + gy * z)),
// so that the same linear index addresses a voxel's byte in a per-frame mark
// plane and its bit in the per-frame occupancy plane (32-voxel words never
// straddle rows).  The padding bytes x >= gx are never part of the grid.
//
// The local grid itself is a ring buffer: voxel (x, y, z) of the grid lives
// at ((x + rx) mod gx, (y + ry) mod gy, (z + rz) mod gz) of its buffer, where
// (rx, ry, rz) are the grid's ring offsets.  A shift (Sec. IV-E) moves the
// offsets and clears only the slabs that enter the grid.  The per-frame
// planes use the plain (unrotated) layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vg_frustum.h"
#include "vg_walk.h"

namespace vg {

// Voxel values in the local grid.
constexpr uint8_t kUnknown = 0;
constexpr uint8_t kFree = 1;
constexpr uint8_t kOccupied = 2;

// Input forms of steps 2-3.
constexpr int kPinhole = 0;
constexpr int kSpinning = 1;
constexpr int kPoints = 2;

// Largest supported vox_inf: the x dilation works on a 64-bit window of
// 32 output voxels plus 2 * vox_inf neighbours.
constexpr int kMaxInflation = 16;

// Most per-frame plane sets one grid's scratch may hold: a batch runs up to
// that many consecutive frames of one grid together, each on its own set.
constexpr int32_t kMaxPlaneSets = 16;

// Row pitch of the device grid layout.
inline int32_t grid_pitch(int32_t gx) { return 32 * ((gx + 31) / 32); }

// The merge and the x dilation have two forms: a narrow one, one lane per
// 16-column chunk / 32-voxel word, for small launches (more lanes hide more
// latency), and a wide one, one lane per 64 columns / 128 voxels, that reads
// only the columns the frame can change (vg_frustum.h).  A launch whose
// narrow form would have at least kWideLanes lanes (8 wavefronts per SIMD of
// the chip) takes the wide form.
constexpr int64_t kWideLanes = (int64_t)1 << 19;

// Wide merge lanes per grid row.
__host__ __device__ inline int32_t merge_lanes_per_row(int32_t gx) { return (gx + 63) / 64; }
// Wide x-dilation lanes per padded row (wx: 32-voxel words per row).
__host__ __device__ inline int32_t dilate_x_lanes_per_row(int32_t wx) { return (wx + 3) / 4; }

inline int64_t merge_lanes(int32_t gx, bool wide)
{
    return wide ? merge_lanes_per_row(gx) : grid_pitch(gx) / 16;
}
inline bool merge_wide(int32_t gx, int64_t rows) { return merge_lanes(gx, false) * rows >= kWideLanes; }
inline int64_t dilate_x_lanes(int32_t wx, bool wide) { return wide ? dilate_x_lanes_per_row(wx) : wx; }
inline bool dilate_x_wide(int64_t narrow_lanes) { return narrow_lanes >= kWideLanes; }

// A box of rows [y0, y1] x [z0, z1] (inclusive; empty if y0 > y1).
struct RowBox {
    int32_t y0, y1, z0, z1;
};

// Per-frame planes.  Seeds live on the grid padded by vox_inf on every side
// (a point just outside the grid still inflates into it); padded coordinate =
// voxel coordinate + vox_inf.
struct Planes {
    int32_t n[3];        // grid size
    int32_t r;           // vox_inf
    int32_t wx;          // 32-voxel words per grid row: gxp / 32
    int32_t py, pz;      // padded rows: gy + 2r, gz + 2r
    int32_t seed_pitch;  // bytes per padded seed row (multiple of 64, >= 32*wx + 64)
    uint8_t *seed;       // seed stamps, [pz][py][seed_pitch]
    uint32_t *bitx;      // seeds dilated along x, [pz][py][wx] words
    uint32_t *occ;       // occupied voxels of the frame, bit i = grid index i
    uint8_t *occb;       // or (direct stamping, non-null) the frame's stamp at
                         // byte i for an occupied voxel of grid index i; it
                         // takes the seed plane's place
    uint8_t *marks;      // free stamps [0, nbytes), "unknown and traced" stamps
                         // [nbytes, 2 nbytes), one byte per grid index each
    uint32_t nbytes;     // bytes of the device-layout grid
    int32_t lo[3], hi[3];  // padded box that holds every seed (lo > hi: none)
    uint32_t epoch;      // stamp of this frame (1..255)
    const RowLimits *lim;  // device: the columns of each row the frame can change
                           // or seed, written by its seed pass (null: all)
};

// Step 2a: transform and quantise every measured point, stamp its voxel (or,
// with Planes::occb, every voxel of its cube).
struct SeedParams {
    Planes pl;
    float R[9];       // R^v_c = R^w_c, row-major
    float tv[3];      // t^v = t^w_c - origin_w
    float s;          // vox_size
    int32_t kind;     // kPinhole, kSpinning or kPoints
    int32_t W, H;     // image size (kPoints: W = number of points, H = 1)
    int64_t pitch;    // image row pitch in floats
    double fx, fy, cx, cy;
    float dmin, dmax;
    const float *img;     // depth / range image, or points[W][3]
    const float *col_tab; // spinning: cos/sin azimuth per column
    const float *row_tab; // spinning: cos/sin elevation per row
    // the frame's regions (vg_frustum.h), computed by the pass's first lane
    // into lim_out (= pl.lim) from these: a pinhole fan of half sizes hw x hh
    // at vox_depth vd (lim_fan), an image with the corner slopes lim_k (ku0,
    // ku1, kv0, kv1; lim_img)
    RowLimits *lim_out;
    int32_t vd, hw, hh;
    int32_t lim_fan, lim_img;
    float lim_k[4];
};

// Step 3: the bundled ray fan.  One wavefront owns a tile of 64 fan targets,
// (1 << tile_log2w) along a (pinhole column / ring column) by
// (64 >> tile_log2w) along b (pinhole row / height).
struct RayParams {
    float R[9];
    WalkFrame wf;     // camera position / voxel, grid size and pitch
    int32_t kind;     // kPinhole (also points) or kSpinning
    int32_t vd, hw, hh;   // pinhole fan; spinning: hh = largest half height
    int32_t na, nb;       // fan extent along a and b
    int32_t tile_log2w;   // 0..6
    int32_t tiles_a, tiles;
    const int32_t *hz;    // spinning: half height per column
    const void *occ;      // occupancy: bits, or stamp bytes if occ_is_bytes
    uint32_t occ_bytes;
    int32_t occ_is_bytes;
    uint8_t *marks;       // as Planes::marks
    uint32_t nbytes;
    uint32_t epoch;
    // order of the ray blocks (WalkOrder), used if it was built for this
    // launch's blocks; null: block order
    const int32_t *order_in;
};

// Ray wavefronts up to which a launch has at most one per SIMD (gfx950:
// 256 compute units x 4 SIMDs) and its ray blocks go to the XCDs in ranges.
constexpr int64_t kLoneWaves = 1024;

// Order of the ray blocks of a large one-frame walk.  Every workgroup of a
// launch runs as soon as a compute unit has room, in block order, so the
// launch ends with the wavefronts that started last; when those are the
// shortest, fewer SIMDs idle at the end.  So the frame's earlier launches
// also build the order in which its walk takes the ray blocks: by an
// estimate of each block's walk length from the frame's pose, longest first.
// The seed launch's extra workgroups rate the blocks (a level per block);
// one extra workgroup of the x dilation launch sorts them, in runs that keep
// the XCD runs of the walk's blocks (the launch boundary orders the two).
// The marks do not depend on the order.  In scratch (plane set 0): a tag --
// the launch shape the order was built for, 0 while none is valid -- and a
// permutation of [0, ray_blocks); then the levels.
constexpr int32_t kOrderMaxBlocks = 8192;
constexpr int32_t kOrderTagInts = 16;
constexpr int32_t kOrderMaxParts = 64;   // rating workgroups
constexpr int32_t kOrderLevels = 256;
struct WalkOrderTag {
    int32_t ray_blocks, tiles_a, tiles, tile_log2w;
};
constexpr size_t kOrderBufBytes = 4 * ((size_t)kOrderTagInts + kOrderMaxBlocks);
constexpr size_t kOrderKeyBytes = kOrderMaxBlocks;
constexpr size_t kOrderBytes = kOrderBufBytes + kOrderKeyBytes;

// A walk-order build: the walk's parameters and ray blocks, the rating
// workgroups (parts), and where the order (tag + blocks) and the levels go;
// order null: none.
struct OrderBuild {
    RayParams rp;
    int32_t ray_blocks;
    int32_t parts;
    int32_t *order;
    uint8_t *keys;
};

// Step 5 on a ring-buffered grid: after the ring offsets moved, the voxels
// whose grid coordinate lies in an exposed slab [lo, hi) of some axis become
// unknown.  Lanes of 16 buffer columns, in three parts: (A) every grid row,
// over the 16-column buffer chunks xrun[0] .. xrun[1] and xrun[2] .. xrun[3]
// (half-open) that hold the exposed x slab (every chunk if it is the whole
// row); (B) the rows of the exposed y slab and (C) those of the exposed z
// slab, whole.  lanes[] counts each part's lanes.
struct SlabClear {
    uint8_t *loc;
    int32_t n[3];
    int32_t gxp;
    int32_t ring[3];        // ring offsets after the shift
    int32_t lo[3], hi[3];   // exposed grid coordinates per axis (lo == hi: none)
    int32_t xrun[4];
    int64_t lanes[3];
};

inline int64_t clear_lanes(const SlabClear &c) { return c.lanes[0] + c.lanes[1] + c.lanes[2]; }

// One frame of a batch round, as the batch kernels read it from device memory.
struct FrameDesc {
    SeedParams sp;              // transform, image and the frame's planes
    RayParams rp;               // the ray fan
    uint8_t *loc;               // the grid's buffer
    SlabClear clear;            // the frame's shift (if it shifts)
    RowBox rows;                // rows of the resolve pass
    int32_t ring[3];            // ring offsets the frame's merge uses
    int32_t inside;             // the camera voxel lies in the grid
    int32_t seed_bx;            // image seed blocks along x (points: 0)
    // Merge of a round that holds several consecutive frames of one grid:
    // on the first frame of each grid's run of frames (in order, contiguous
    // in the table), the run's length and the rows the merge covers, in the
    // grid coordinates of the run's last frame; 0 on the run's other frames.
    int32_t group;
    RowBox dom;
};

// The y/z dilation runs on tiles staged through LDS when a row's words fit a
// fixed slot width kW (8 or 16 words, so rows up to 256 / 512 voxels) and
// vox_inf <= 3: a block of kBlock threads is kW word lanes by kBlock / kW row
// slots, and a tile is kBlock / kW output rows along y by tz along z -- 2, or
// 8 for launches with many tiles (fewer z rows read twice: an 8-deep tile
// reads 8 + 2 vox_inf input z rows, four 2-deep tiles 4 (2 + 2 vox_inf)).
// kw 0: untiled.
constexpr int kTileMaxR = 3;
constexpr int kTileDeep = 8;
constexpr int64_t kDeepTileMin = 512;   // 8-deep tiles per launch to use them
constexpr size_t kMaxTileLds = 48 * 1024;

struct YzTile {
    int kw, tz;
};

// The slot width for a frame at tile depth tz (0: the frame cannot be tiled).
inline int dilate_tile_width(const Planes &pl, int tz)
{
    const int kw = pl.wx <= 8 ? 8 : (pl.wx <= 16 ? 16 : 0);
    const size_t ty = kw ? 256 / kw : 0, iz = (size_t)tz + 2 * pl.r, iy = ty + 2 * pl.r;
    // each thread loads at most 2 input rows of every z row: iy <= 2 ty
    if (kw == 0 || pl.r > kTileMaxR || iy > 2 * ty)
        return 0;
    return 4 * (size_t)kw * iz * iy <= kMaxTileLds ? kw : 0;
}

// LDS bytes of one tile: its padded input rows.
inline size_t dilate_tile_lds(const Planes &pl, YzTile t)
{
    const size_t ty = 256 / t.kw, iz = (size_t)t.tz + 2 * pl.r, iy = ty + 2 * pl.r;
    return 4 * (size_t)t.kw * iz * iy;
}

inline int64_t dilate_tiles(const Planes &pl, YzTile t)
{
    const int ty = 256 / t.kw;
    return (int64_t)((pl.n[1] + ty - 1) / ty) * ((pl.n[2] + t.tz - 1) / t.tz);
}

// Batch stages, in launch order within a round.
enum { kBatchShift, kBatchSeed, kBatchDilateX, kBatchDilateYZ, kBatchRays, kBatchResolve,
       kBatchStages };

// Batch frame tables: per round, kBatchStages block prefixes of m + 1
// entries (16-byte aligned), then m frame descriptors.
constexpr int32_t kMaxBatch = 4096;

constexpr size_t batch_starts_bytes(int32_t m)
{
    return ((size_t)kBatchStages * (m + 1) * sizeof(int32_t) + 15) / 16 * 16;
}

constexpr size_t batch_table_bytes(int32_t m)
{
    return (batch_starts_bytes(m) + (size_t)m * sizeof(FrameDesc) + 15) / 16 * 16;
}

// Workspace of a batch of up to m frames: a round of k frames needs at most
// k times a one-frame round (256-byte aligned, plus slack).
constexpr size_t batch_workspace_bytes(int32_t m)
{
    return ((size_t)m * batch_table_bytes(1) + 256 + 255) / 256 * 256;
}

// Frames per call of the batch entry point whose frame tables live in a
// device array of the library (for callers that cannot allocate), and that
// array's size.
constexpr int32_t kStaticBatchFrames = 256;
constexpr size_t kStaticBatchBytes = batch_workspace_bytes(kStaticBatchFrames);

// Bytes to copy into device memory, carried as a kernel argument (so that a
// batch needs no host staging buffer that must outlive the call).
constexpr int kUploadWords = 1016;
struct UploadBlob {
    uint32_t *dst;
    uint32_t words;
    uint32_t w[kUploadWords];
};

// Optional timing of one stage: `start` takes the start time of the stage's
// first kernel dispatch and `stop` the end time of its last (recorded by the
// dispatches themselves, so no marker sits between the kernels).  A stage
// that launches nothing records both as plain markers.  Null: not recorded.
struct StageEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

hipError_t launch_fill(void *dst, uint8_t value, size_t bytes, hipStream_t st);
hipError_t launch_seeds(const SeedParams &p, hipStream_t st, const StageEvents &ev = {},
                        const OrderBuild *order = nullptr);
// Seeds -> occupied bit plane (dilation by vox_inf along x, then y and z).
hipError_t launch_dilate(const Planes &pl, hipStream_t st, const StageEvents &ev = {},
                         const OrderBuild *order = nullptr);
// The walk of every fan ray.  camera_inside: the camera voxel lies in the grid.
// clear (optional): a slab clear of the local grid run by extra workgroups of
// the same launch (it touches no memory the walk uses).
hipError_t launch_rays(const RayParams &p, bool camera_inside, hipStream_t st,
                       const StageEvents &ev = {}, const SlabClear *clear = nullptr);
// Marks and occupied bits -> the local grid (ring offsets `ring`), over the
// given rows.
hipError_t launch_resolve(const Planes &pl, uint8_t *loc, const RowBox &rows,
                          const int32_t ring[3], hipStream_t st, const StageEvents &ev = {});
hipError_t launch_clear(const SlabClear &c, hipStream_t st, const StageEvents &ev = {});
// Records the events of a stage that launches no kernel.
hipError_t record_empty_stage(const StageEvents &ev, hipStream_t st);

// The library's own batch workspace on the current device (kStaticBatchBytes,
// 256-byte aligned): its device address, looked up once per device.
hipError_t static_batch_workspace(void **ptr);
// Batch: copy host words to device memory through kernel arguments.
hipError_t launch_upload(uint32_t *dst, const uint32_t *src, size_t words, hipStream_t st);
// Batch: one launch of stage `stage` (kBatch*) over the n frames of a round;
// fd and start (n + 1 block prefixes) live in device memory; blocks = start[n].
// tile.kw > 0 (kBatchDilateYZ only): the tiled y/z dilation of that shape
// with `lds` bytes of LDS per block; the block prefixes then count
// dilate_tiles(pl, tile) per frame.
// seq (kBatchResolve only): the merge takes each grid's run of frames
// together (FrameDesc::group), and the block prefixes count its domain's
// blocks on the run's first frame and none on the others.
// wide (kBatchDilateX and kBatchResolve without seq): the wide form of the
// stage, whose block prefixes count its lanes.
hipError_t launch_batch_stage(int stage, const FrameDesc *fd, const int32_t *start, int32_t n,
                              int32_t blocks, hipStream_t st, const StageEvents &ev = {},
                              YzTile tile = {0, 0}, size_t lds = 0, bool seq = false,
                              bool wide = false);
// Linear (pitch gx) <-> device layout (pitch gxp) copies of a whole grid.
hipError_t copy_grid(uint8_t *dst, int64_t dst_pitch, const uint8_t *src, int64_t src_pitch,
                     const int32_t n[3], hipMemcpyKind kind, hipStream_t st);
// Device layout with ring offsets -> linear: up to 8 box copies.
hipError_t copy_grid_from_ring(uint8_t *dst, const uint8_t *src, int64_t src_pitch,
                               const int32_t n[3], const int32_t ring[3], hipMemcpyKind kind,
                               hipStream_t st);

}  // namespace vg

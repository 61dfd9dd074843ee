// vg_kernels.hip -- gfx950 kernels for depth-frame -> voxel-grid generation
// (Toumieh & Lambert, arXiv 2112.13169, Sec. IV).
//
// One frame is a chain of launches on one stream (k_clear, for a shift of the
// ring-buffered grid, runs before it when the grid is re-centred):
//   k_seed        Alg. 1, transform and quantise: one lane per pixel / point: unproject,
//                 transform, quantise; stamp the point's voxel in a seed plane
//                 padded by vox_inf (byte stores of the frame's stamp: no
//                 clearing between frames, no atomics).  For small frames it
//                 stamps the point's whole cube into a byte occupancy plane
//                 instead, and the two dilations do not run.
//   k_dilate_x    Alg. 1, inflation, separably: seeds -> bits dilated by
//   k_dilate_yz   vox_inf along x, then along y and z.  The union of the
//                 (2 vox_inf + 1)^3 cubes is exactly this separable dilation.
//   k_rays_w      Alg. 2: one wavefront (and workgroup) per tile of 64 fan
//                 targets (8 x 8 by default), one lane per ray.  Each step stamps its voxel in
//                 one of two per-frame mark planes: "free" before the ray's
//                 first occupied voxel, "unknown and traced" from it on.
//                 Occupancy words are fetched for 8 walk steps at a time so
//                 that the loads overlap.
//   k_resolve     Alg. 3: occupied bits, then traced stamps, then free stamps
//                 decide each voxel of the local grid the frame reaches.
// All stores are idempotent byte stores; no atomics.
//
// Floating point: contraction is off (also on the command line) so every fp32
// operation rounds exactly as written; fp32 division is the correctly rounded
// one, fp32 denormals are kept.  The fixed operation orders are those of the
// transform (R p + t, left to right) and of the Amanatides & Woo walk.
#include "vg_internal.h"
#include "vg_walk.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <mutex>

#pragma clang fp contract(off)

// Frame tables of vg_integrate_batch_static: one copy per GPU, held until the
// process ends.  Host code never passes this name to a kernel (on the host it
// is only a stand-in for the symbol); it uses the device address that
// static_batch_workspace() looks up per device.
static __device__ __align__(256) uint8_t scratch[vg::kStaticBatchBytes];

namespace vg {

namespace {

constexpr int kBlock = 256;
// Larger walk launches give each XCD runs of this many consecutive ray blocks.
constexpr int32_t kXcdRun = 4;

// ----------------------------------------------------------------- helpers

// A frame's row limits as the kernels read them: through the constant address
// space (the seed pass wrote them in an earlier launch and no kernel that
// reads them writes them), so that they load with scalar loads also where
// the pointer itself was read from memory (a batch's frame table).
// (The host pass of this file, which never runs the kernels, keeps the plain
// pointer.)
#ifdef __HIP_DEVICE_COMPILE__
typedef const __attribute__((address_space(4))) RowLimits *ConstLimits;
#else
typedef const RowLimits *ConstLimits;
#endif

__device__ __forceinline__ ConstLimits const_limits(const RowLimits *p)
{
    return (ConstLimits)p;
}

// Workgroup b of a launch runs on XCD b mod 8, and each of the 8 XCDs has an
// L2 of its own.  Neighbouring ray tiles mark the same mark-plane lines, and a
// line dirtied in several L2s is written back from each of them.  The block
// that runs as workgroup b takes block xcd_runs(b, n) instead, so that each
// XCD walks runs of kXcdRun consecutive blocks: most lines then stay in one
// L2, and the runs still spread the costly tiles over every XCD.  A
// permutation of [0, n) (blocks past the last whole round of 8 runs keep
// their numbers).
__device__ __forceinline__ int32_t xcd_runs(int32_t b, int32_t n)
{
    constexpr int32_t round = 8 * kXcdRun;
    if (b >= n / round * round)
        return b;
    const int32_t k = b >> 3, x = b & 7;
    return ((k / kXcdRun) * 8 + x) * kXcdRun + k % kXcdRun;
}

// Row i of R p: ((R_i0 x + R_i1 y) + R_i2 z), each operation rounded.
__device__ __forceinline__ float row_dot(const float *Ri, float x, float y, float z)
{
    float a = Ri[0] * x;
    float b = Ri[1] * y;
    float s = a + b;
    float c = Ri[2] * z;
    return s + c;
}

// Square-ring column of a spinning fan: 8*vd lattice columns with
// max(|x|,|y|) = vd, counter-clockwise from just above (vd, -vd).
__device__ __forceinline__ void ring_column(int32_t c, int32_t vd, int32_t &x, int32_t &y)
{
    int32_t side = c / (2 * vd), k = c - side * (2 * vd);
    if (side == 0) {
        x = vd;
        y = -vd + 1 + k;
    } else if (side == 1) {
        x = vd - 1 - k;
        y = vd;
    } else if (side == 2) {
        x = -vd;
        y = vd - 1 - k;
    } else {
        x = -vd + 1 + k;
        y = -vd;
    }
}

// Fan target of (ia, ib): the ray direction in the camera frame (lattice
// integers) and the squared termination length.  False if out of the fan.
__device__ __forceinline__ bool fan_target(const RayParams &p, int32_t ia, int32_t ib,
                                           int32_t &tx, int32_t &ty, int32_t &tz, int32_t &m2)
{
    if (ia >= p.na || ib >= p.nb)
        return false;
    if (p.kind == kSpinning) {
        int32_t z = ib - p.hh;
        int32_t lim = p.hz[ia];
        if (z < -lim || z > lim)
            return false;
        ring_column(ia, p.vd, tx, ty);
        tz = z;
        m2 = p.vd * p.vd;
    } else {
        tx = ia - p.hw;
        ty = ib - p.hh;
        tz = p.vd;
        m2 = tx * tx + ty * ty + p.vd * p.vd;
    }
    return true;
}

__device__ __forceinline__ void ray_direction(const RayParams &p, int32_t tx, int32_t ty,
                                              int32_t tz, float dir[3])
{
    float x = (float)tx, y = (float)ty, z = (float)tz;
    dir[0] = row_dot(p.R + 0, x, y, z);
    dir[1] = row_dot(p.R + 3, x, y, z);
    dir[2] = row_dot(p.R + 6, x, y, z);
}

// Bit 0 of byte j set iff byte j of w equals the byte replicated in rep (the
// other bits clear).
__device__ __forceinline__ uint32_t byte_eq_ones(uint32_t w, uint32_t rep)
{
    uint32_t x = w ^ rep;                                  // zero bytes = matches
    uint32_t y = (x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
    y = ~(y | x | 0x7F7F7F7Fu);                            // 0x80 exactly in zero bytes
    return y >> 7;
}

// The flags of two such words in bits 0 .. 7: a's bytes 0 .. 3, then b's.
// One multiply gathers all eight: flag k of a sits at bit 8k and of b at
// 8k + 4, and the multiplier's bits 24 - 7i move flag i of each to bit
// 24 + i (a) and 28 + i (b); the other products land on distinct bits below
// 24 or at 32 and above, so nothing carries into bits 24 .. 31.
__device__ __forceinline__ uint32_t gather8(uint32_t a, uint32_t b)
{
    return ((a | (b << 4)) * 0x01020408u) >> 24;
}

// Bit j (j < 16) set iff byte j of q (x's bytes first) equals the byte
// replicated in rep.
__device__ __forceinline__ uint32_t byte_eq_mask16(const uint4 &q, uint32_t rep)
{
    return gather8(byte_eq_ones(q.x, rep), byte_eq_ones(q.y, rep)) |
           (gather8(byte_eq_ones(q.z, rep), byte_eq_ones(q.w, rep)) << 8);
}

// ----------------------------------------------------------------- kernels

__global__ __launch_bounds__(kBlock) void k_fill(uint8_t *dst, uint8_t value, size_t bytes)
{
    const uintptr_t base = (uintptr_t)dst & ~(uintptr_t)15;
    const uintptr_t end = (uintptr_t)dst + bytes;
    size_t chunk = (size_t)blockIdx.x * kBlock + threadIdx.x;
    uintptr_t c0 = base + chunk * 16;
    if (c0 >= end)
        return;
    if (c0 >= (uintptr_t)dst && c0 + 16 <= end) {
        uint32_t w = value * 0x01010101u;
        *reinterpret_cast<uint4 *>(c0) = make_uint4(w, w, w, w);
    } else {
        for (uintptr_t q = c0; q < c0 + 16; ++q)
            if (q >= (uintptr_t)dst && q < end)
                *reinterpret_cast<uint8_t *>(q) = value;
    }
}

// ------------------------------------------------------------ stage bodies
// Each stage is a device function of (parameters, work index); the one-frame
// kernels take their parameters as kernel arguments, the batch kernels read
// them from a frame table in device memory.

// Alg. 1, transform and quantise.  Images: block = 64 x 4 pixels (bx, by), one wavefront
// per image row segment (coalesced row reads).  Points: 256 points per block.
// The point of lane (bx, by, threadIdx.x): its padded voxel coordinates, or
// false if it has none (no pixel, invalid depth, or a cube that cannot reach
// the grid).
__device__ __forceinline__ bool seed_point(const SeedParams &p, int32_t bx, int32_t by,
                                           int32_t pp[3])
{
    float pc[3];
    if (p.kind == kPoints) {
        int64_t i = (int64_t)bx * kBlock + threadIdx.x;
        if (i >= p.W)
            return false;
        const float *q = p.img + 3 * i;
        float x = q[0], y = q[1], z = q[2];
        if (!(__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z)))
            return false;
        pc[0] = x;
        pc[1] = y;
        pc[2] = z;
    } else {
        int32_t u = bx * 64 + (threadIdx.x & 63);
        int32_t v = by * 4 + (threadIdx.x >> 6);
        if (u >= p.W || v >= p.H)
            return false;
        float d = p.img[(int64_t)v * p.pitch + u];
        if (!(d >= p.dmin && d <= p.dmax))
            return false;
        if (p.kind == kPinhole) {
            // pixel slopes in double, rounded once
            float ku = (float)(((double)u - p.cx) / p.fx);
            float kv = (float)(((double)v - p.cy) / p.fy);
            pc[0] = d * ku;
            pc[1] = d * kv;
            pc[2] = d;
        } else {
            float ce = p.row_tab[2 * v + 0], se = p.row_tab[2 * v + 1];
            float ca = p.col_tab[2 * u + 0], sa = p.col_tab[2 * u + 1];
            float horiz = d * ce;
            pc[0] = horiz * ca;
            pc[1] = horiz * sa;
            pc[2] = d * se;
        }
    }
    const Planes &pl = p.pl;
    for (int a = 0; a < 3; ++a) {
        float pv = row_dot(p.R + 3 * a, pc[0], pc[1], pc[2]) + p.tv[a];
        float q = floorf(pv / p.s);
        // the cube cannot reach the grid: drop the point
        if (!(q >= (float)(-pl.r) && q <= (float)(pl.n[a] - 1 + pl.r)))
            return false;
        pp[a] = (int32_t)q + pl.r;   // padded coordinate
    }
    return true;
}

__device__ __forceinline__ void seed_body(const SeedParams &p, int32_t bx, int32_t by)
{
    const Planes &pl = p.pl;
    if (bx == 0 && by == 0 && threadIdx.x < 64 && p.lim_out) {
        // the frame's regions, for the x dilation and the merge: lanes 0..7
        // of the first wavefront build one plane each; the camera position as
        // the walk's (the same fp32 quotients)
        const int k = (int)threadIdx.x;
        const int planes = p.lim_fan ? (p.lim_img ? 8 : 4) : 0;
        bool ok = true;
        if (k < planes) {
            const float o[3] = {p.tv[0] / p.s, p.tv[1] / p.s, p.tv[2] / p.s};
            RowPlane q;
            ok = make_region_plane(k, p.R, o, p.vd, p.hw, p.hh, p.lim_k[0], p.lim_k[1],
                                   p.lim_k[2], p.lim_k[3], pl.r, pl.n[0], q);
            (k < 4 ? p.lim_out->fan.p[k] : p.lim_out->img.p[k - 4]) = q;
        }
        const bool all = __all(ok);
        if (k == 0) {
            p.lim_out->has_fan = planes > 0 && all ? 1 : 0;
            p.lim_out->has_img = planes == 8 && all ? 1 : 0;
        }
    }
    int32_t pp[3] = {0, 0, 0};
    const bool ok = seed_point(p, bx, by, pp);
    if (!pl.occb) {
        if (ok)
            pl.seed[(int64_t)pl.seed_pitch * (pp[1] + (int64_t)pl.py * pp[2]) + pp[0]] =
                (uint8_t)pl.epoch;
        return;
    }
    // Stamp the cube of the point's voxel, clipped to the grid: padded
    // coordinates pp - r .. pp + r are grid coordinates pp - 2r .. pp.
    if (!ok)
        return;
    const int32_t gxp = pl.wx * 32;
    const int32_t x0 = max(pp[0] - 2 * pl.r, 0), x1 = min(pp[0], pl.n[0] - 1);
    const int32_t y0 = max(pp[1] - 2 * pl.r, 0), y1 = min(pp[1], pl.n[1] - 1);
    const int32_t z0 = max(pp[2] - 2 * pl.r, 0), z1 = min(pp[2], pl.n[2] - 1);
    for (int32_t z = z0; z <= z1; ++z)
        for (int32_t y = y0; y <= y1; ++y) {
            uint8_t *row = pl.occb + (int64_t)gxp * (y + (int64_t)pl.n[1] * z);
            for (int32_t x = x0; x <= x1; ++x)
                row[x] = (uint8_t)pl.epoch;
        }
}

// Bit j of the result set iff some bit j .. j + span - 1 of w is (span >= 1):
// shift-or doublings up to the largest power of two p <= span, then one
// shifted or for the rest.
__device__ __forceinline__ uint64_t or_span(uint64_t w, int32_t span)
{
    int32_t p = 1;
    while (2 * p <= span) {
        w |= w >> p;
        p *= 2;
    }
    return span > p ? (w | (w >> (span - p))) : w;
}

// Seeds -> bits dilated along x: output voxel x is set iff a seed lies at
// padded x .. x + 2r of the same padded row, for the padded rows of the seed
// box.  kWide (large launches): one lane per four 32-voxel output words (128
// voxels), which reads the row's stamp bytes x0 .. x0 + 127 + 2r once
// (16-byte loads, SWAR compares) unless the seed box or the image's region of
// the row (grid coordinates = padded - r) leaves them out.  Otherwise one lane
// per output word, reading x0 .. x0 + 63 (more lanes for small launches).
template <bool kWide>
__device__ __forceinline__ void dilate_x_body(const Planes &pl, int64_t gid)
{
    const int32_t ny = pl.hi[1] - pl.lo[1] + 1;
    const int32_t nz = pl.hi[2] - pl.lo[2] + 1;
    if (!kWide) {
        if (pl.lo[0] > pl.hi[0] || ny <= 0 || nz <= 0 || gid >= (int64_t)pl.wx * ny * nz)
            return;
        const uint32_t g32 = (uint32_t)gid, wx = (uint32_t)pl.wx;
        const int32_t w = (int32_t)(g32 % wx);
        const uint32_t row = g32 / wx;
        const int32_t y = pl.lo[1] + (int32_t)(row % (uint32_t)ny);
        const int32_t z = pl.lo[2] + (int32_t)(row / (uint32_t)ny);
        const int32_t x0 = 32 * w;
        uint32_t out = 0;
        if (x0 <= pl.hi[0] && x0 + 31 + 2 * pl.r >= pl.lo[0]) {
            const uint4 *src = reinterpret_cast<const uint4 *>(
                pl.seed + (int64_t)pl.seed_pitch * (y + (int64_t)pl.py * z) + x0);
            const uint32_t rep = (pl.epoch & 0xFFu) * 0x01010101u;
            uint32_t m[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                m[k] = byte_eq_mask16(src[k], rep);
            }
            const uint64_t w64 = (uint64_t)(m[0] | (m[1] << 16)) |
                                 ((uint64_t)(m[2] | (m[3] << 16)) << 32);
            out = (uint32_t)or_span(w64, 2 * pl.r + 1);
            const int32_t valid = pl.n[0] - x0;   // output voxels of this word inside the grid
            if (valid < 32)
                out &= (1u << valid) - 1u;
        }
        pl.bitx[(int64_t)pl.wx * (y + (int64_t)pl.py * z) + w] = out;
        return;
    }
    const int32_t lanes = dilate_x_lanes_per_row(pl.wx);
    if (pl.lo[0] > pl.hi[0] || ny <= 0 || nz <= 0 || gid >= (int64_t)lanes * ny * nz)
        return;
    // fewer lanes than a padded grid has bytes: 32-bit index arithmetic
    const uint32_t g32 = (uint32_t)gid;
    const int32_t k = (int32_t)(g32 % (uint32_t)lanes);
    const uint32_t row = g32 / (uint32_t)lanes;
    const int32_t y = pl.lo[1] + (int32_t)(row % (uint32_t)ny);
    const int32_t z = pl.lo[2] + (int32_t)(row / (uint32_t)ny);
    const int32_t x0 = 128 * k;
    const int32_t words = min(4, pl.wx - 4 * k);           // output words of this lane
    const int32_t need = 32 * words + 2 * pl.r;            // stamp bytes they read
    uint32_t m[5] = {0u, 0u, 0u, 0u, 0u};                  // bit j: byte x0 + j is a seed
    if (x0 <= pl.hi[0] && x0 + need - 1 >= pl.lo[0] &&
        (!pl.lim || row_run_seeded(*const_limits(pl.lim), y - pl.r, z - pl.r, x0 - pl.r,
                                   x0 + need - 1 - pl.r))) {
        const uint4 *src = reinterpret_cast<const uint4 *>(
            pl.seed + (int64_t)pl.seed_pitch * (y + (int64_t)pl.py * z) + x0);
        const uint32_t rep = (pl.epoch & 0xFFu) * 0x01010101u;
        uint4 q[10];
#pragma unroll
        for (int j = 0; j < 10; ++j)
            q[j] = 16 * j < need ? src[j] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            m[j >> 1] |= byte_eq_mask16(q[j], rep) << (16 * (j & 1));
        }
    }
    uint32_t *dst = pl.bitx + (int64_t)pl.wx * (y + (int64_t)pl.py * z) + 4 * k;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i >= words)
            break;
        uint32_t out =
            (uint32_t)or_span(((uint64_t)m[i + 1] << 32) | (uint64_t)m[i], 2 * pl.r + 1);
        const int32_t valid = pl.n[0] - (x0 + 32 * i);   // output voxels inside the grid
        if (valid < 32)
            out = valid > 0 ? out & ((1u << valid) - 1u) : 0u;
        dst[i] = out;
    }
}

// x-dilated rows -> occupied bit plane: OR over the (2r+1) x (2r+1) padded
// rows y .. y+2r, z .. z+2r.  Every word of the plane is written.
__device__ __forceinline__ void dilate_yz_body(const Planes &pl, int64_t gid)
{
    if (gid >= (int64_t)pl.wx * pl.n[1] * pl.n[2])
        return;
    const uint32_t g32 = (uint32_t)gid, wx = (uint32_t)pl.wx;   // < 2^26 words
    const int32_t w = (int32_t)(g32 % wx);
    const uint32_t row = g32 / wx;
    const int32_t y = (int32_t)(row % (uint32_t)pl.n[1]);
    const int32_t z = (int32_t)(row / (uint32_t)pl.n[1]);
    const int32_t y0 = max(y, pl.lo[1]), y1 = min(y + 2 * pl.r, pl.hi[1]);
    const int32_t z0 = max(z, pl.lo[2]), z1 = min(z + 2 * pl.r, pl.hi[2]);
    uint32_t out = 0;
    if (pl.lo[0] <= pl.hi[0]) {
        for (int32_t zz = z0; zz <= z1; ++zz) {
            const uint32_t *src = pl.bitx + (int64_t)pl.wx * ((int64_t)pl.py * zz) + w;
            for (int32_t yy = y0; yy <= y1; ++yy)
                out |= src[(int64_t)pl.wx * yy];
        }
    }
    pl.occ[gid] = out;
}

// The same dilation for one tile (tile_y, tile_z) of kBlock / kW rows along y
// by kTZ along z (vox_inf <= kTileMaxR).  Thread = (word lane w, row slot);
// the padded rows the tile reads are loaded once into LDS (rows outside the
// seed box as 0).  Each thread then ORs its column along y, one input z row
// at a time, into registers, and ORs those along z.  Both passes read a fixed
// 2 kTileMaxR + 1 rows (rows past the window are read, at clamped addresses,
// and not used), so that the reads of a pass issue together.  No divisions:
// rows are walked by slot, words by lane.
template <int kW, int kTZ>
__device__ __forceinline__ void dilate_yz_tile_body(const Planes &pl, int32_t tile_y,
                                                    int32_t tile_z, uint32_t *lds)
{
    constexpr int32_t kTY = kBlock / kW;
    constexpr int kTileMaxIz = kTZ + 2 * kTileMaxR;   // input z rows a tile may need
    const int32_t w = (int32_t)threadIdx.x % kW, slot = (int32_t)threadIdx.x / kW;
    const int32_t r2 = 2 * pl.r, wx = pl.wx;
    const int32_t iy = kTY + r2, iz = kTZ + r2;
    const int32_t y0 = tile_y * kTY, z0 = tile_z * kTZ;   // first output row = padded row
    uint32_t *in = lds;                   // [iz][iy][kW]
    const bool any = pl.lo[0] <= pl.hi[0];
    const bool lane = w < wx;
    // all loads of a thread first, so that they are in flight together: the
    // thread's word lane w of padded rows y0 + slot (+ kTY) of every input z
    // row (at most 2 x kTileMaxIz, unrolled, no divisions); then the stores
    // Buffer loads: the lane's byte offset of padded row (py, z0) once (kOob,
    // which reads 0, for rows outside the seed box), and the z row's offset
    // as the uniform scalar offset, so that a load costs no vector
    // arithmetic.  Rows of at most 16 words: the padded plane holds fewer than
    // 2^31 bytes.
    const uint32_t zs = 4u * (uint32_t)wx * (uint32_t)pl.py;   // bytes per padded z row
    const __amdgpu_buffer_rsrc_t rb = buffer_rsrc(pl.bitx, zs * (uint32_t)pl.pz);
    uint32_t ld[2][kTileMaxIz];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int32_t yy = slot + h * kTY;
        const int32_t py = y0 + yy;
        const bool yin = any && lane && yy < iy && py >= pl.lo[1] && py <= pl.hi[1];
        const uint32_t off =
            yin ? 4u * ((uint32_t)wx * (uint32_t)py + (uint32_t)w) + (uint32_t)z0 * zs : kOob;
#pragma unroll
        for (int zz = 0; zz < kTileMaxIz; ++zz) {
            const int32_t pz = z0 + zz;
            ld[h][zz] = (zz < iz && pz >= pl.lo[2] && pz <= pl.hi[2])
                            ? __builtin_amdgcn_raw_buffer_load_b32(rb, (int)off,
                                                                   (int)((uint32_t)zz * zs), 0)
                            : 0u;
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int32_t yy = slot + h * kTY;
#pragma unroll
        for (int zz = 0; zz < kTileMaxIz; ++zz)
            if (yy < iy && zz < iz)
                in[(zz * iy + yy) * kW + w] = ld[h][zz];
    }
    __syncthreads();
    // along y: t[zz] = OR of input rows slot .. slot + r2 of input z row zz
    // (z rows past iz are read at row iz - 1 and not used either)
    uint32_t t[kTileMaxIz];
#pragma unroll
    for (int zz = 0; zz < kTileMaxIz; ++zz) {
        const int32_t zr = min(zz, iz - 1);
        uint32_t v = 0;
#pragma unroll
        for (int d = 0; d <= 2 * kTileMaxR; ++d) {
            const uint32_t x = in[(zr * iy + min(slot + d, iy - 1)) * kW + w];
            v |= d <= r2 ? x : 0u;
        }
        t[zz] = zz < iz ? v : 0u;
    }
    const int32_t gy = y0 + slot;
    if (!lane || gy >= pl.n[1])
        return;
    // along z: output z row z0 + z = OR of t[z .. z + r2]
    // stores as the loads: the lane's offset once, the z row's as the scalar
    const uint32_t os = 4u * (uint32_t)wx * (uint32_t)pl.n[1];   // bytes per grid z row
    const __amdgpu_buffer_rsrc_t ro = buffer_rsrc(pl.occ, os * (uint32_t)pl.n[2]);
    const uint32_t out = 4u * ((uint32_t)wx * (uint32_t)gy + (uint32_t)w) + (uint32_t)z0 * os;
#pragma unroll
    for (int z = 0; z < kTZ; ++z) {
        const int32_t gz = z0 + z;
        if (gz >= pl.n[2])
            break;
        uint32_t v = 0;
#pragma unroll
        for (int d = 0; d <= 2 * kTileMaxR; ++d)
            v |= d <= r2 ? t[z + d] : 0u;
        __builtin_amdgcn_raw_buffer_store_b32(v, ro, (int)out, (int)((uint32_t)z * os), 0);
    }
}

// Alg. 2 for the 64 rays of fan tile `tile` (one wavefront).
template <bool kGeneral, bool kBytes, bool kLone>
__device__ __forceinline__ void rays_body(const RayParams &p, int32_t tile)
{
    const int lane = threadIdx.x & 63;
    const int32_t lw = p.tile_log2w;
    const int32_t ta = tile % p.tiles_a, tb = tile / p.tiles_a;
    const int32_t ia = (ta << lw) + (lane & ((1 << lw) - 1));
    const int32_t ib = tb * (64 >> lw) + (lane >> lw);
    int32_t tx, ty, tz, m2;
    if (tile >= p.tiles || !fan_target(p, ia, ib, tx, ty, tz, m2))
        return;
    float dir[3];
    ray_direction(p, tx, ty, tz, dir);
    if (kGeneral && (axis_dead(sgn(dir[0]), p.wf.v0[0], p.wf.n[0]) ||
                     axis_dead(sgn(dir[1]), p.wf.v0[1], p.wf.n[1]) ||
                     axis_dead(sgn(dir[2]), p.wf.v0[2], p.wf.n[2])))
        return;
    Walk w;
    walk_setup(w, p.wf, dir);
    walk_ray<kGeneral, kBytes, kLone>(w, m2, walk_mem(p.occ, p.occ_bytes, p.marks, p.nbytes,
                                                      p.epoch & 0xFFu));
}

// (v + r) mod n for v, r in [0, n).
__device__ __forceinline__ int32_t wrap_add(int32_t v, int32_t r, int32_t n)
{
    const int32_t s = v + r;
    return s >= n ? s - n : s;
}

// The 16 bytes at any byte address p: five aligned dword loads from p
// rounded down to 4 (so up to 4 bytes past p + 16 are read), realigned with
// v_alignbyte.
__device__ __forceinline__ uint4 load16_unaligned(const uint8_t *p)
{
    // pointer arithmetic, not an integer round trip, keeps the global
    // address space (global rather than flat loads)
    const uint32_t sh = (uint32_t)((uintptr_t)p & 3);
    const uint32_t *w = reinterpret_cast<const uint32_t *>(p - sh);
    uint32_t v[5];
#pragma unroll
    for (int k = 0; k < 5; ++k)
        v[k] = w[k];
    return make_uint4(__builtin_amdgcn_alignbyte(v[1], v[0], sh),
                      __builtin_amdgcn_alignbyte(v[2], v[1], sh),
                      __builtin_amdgcn_alignbyte(v[3], v[2], sh),
                      __builtin_amdgcn_alignbyte(v[4], v[3], sh));
}

// 0xFF in each byte of w that equals the byte replicated in rep, 0 in the
// others (SWAR: no carry crosses a byte).
__device__ __forceinline__ uint32_t byte_eq_ff(uint32_t w, uint32_t rep)
{
    const uint32_t x = w ^ rep;
    const uint32_t y = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;   // bit 7 set in non-zero bytes
    return ((~y >> 7) & 0x01010101u) * 0xFFu;
}

__device__ __forceinline__ uint4 byte_eq_ff16(const uint4 &q, uint32_t rep)
{
    return make_uint4(byte_eq_ff(q.x, rep), byte_eq_ff(q.y, rep), byte_eq_ff(q.z, rep),
                      byte_eq_ff(q.w, rep));
}

// 0xFF in byte j (j < 4) of the result iff bit j of b is set.
__device__ __forceinline__ uint32_t spread4(uint32_t b)
{
    return ((b & 0xFu) * 0x00204081u & 0x01010101u) * 0xFFu;
}

__device__ __forceinline__ uint4 spread16(uint32_t b)
{
    return make_uint4(spread4(b), spread4(b >> 4), spread4(b >> 8), spread4(b >> 12));
}

// A frame's states of 16 consecutive voxels as byte masks (0xFF in byte j
// iff voxel j is): occupied, traced, free.
struct Masks16 {
    uint4 o, t, f;
};

__device__ __forceinline__ bool any16(const Masks16 &m)
{
    return ((m.o.x | m.o.y | m.o.z | m.o.w) | (m.t.x | m.t.y | m.t.z | m.t.w) |
            (m.f.x | m.f.y | m.f.z | m.f.w)) != 0u;
}

// The frame's states of 16 grid columns of one plane row: columns x0 .. x0 +
// 15, wrapping at the grid's width, of which the first nvalid are grid
// columns.  The bytes are one aligned 16-byte run, one unaligned run (aligned
// dwords + v_alignbyte), or a run that wraps (per byte, zero past nvalid).
// The stamps are compared once, after the loads.  A plane byte or bit of a
// column past the grid's width never holds the frame's stamp or bit (the
// passes write grid voxels only), so no column mask is needed.
template <bool kBytes>
__device__ __forceinline__ void gather16(const Planes &pl, int64_t prow, int32_t x0,
                                         int32_t nvalid, Masks16 &m)
{
    const int32_t gx = pl.n[0];
    const uint32_t rep = (pl.epoch & 0xFFu) * 0x01010101u;
    uint4 fr, tr, oc = make_uint4(0u, 0u, 0u, 0u);
    uint32_t obits = 0;
    if ((x0 & 15) == 0 && x0 + nvalid <= gx) {
        // one run of grid columns starting on a 16-column boundary
        const int64_t b = prow + x0;
        fr = *reinterpret_cast<const uint4 *>(pl.marks + b);
        tr = *reinterpret_cast<const uint4 *>(pl.marks + pl.nbytes + b);
        if (kBytes)
            oc = *reinterpret_cast<const uint4 *>(pl.occb + b);
        else
            obits = (pl.occ[b >> 5] >> (b & 16)) & 0xFFFFu;
    } else if (x0 + nvalid <= gx) {
        const int64_t b = prow + x0;
        fr = load16_unaligned(pl.marks + b);
        tr = load16_unaligned(pl.marks + pl.nbytes + b);
        if (kBytes) {
            oc = load16_unaligned(pl.occb + b);
        } else {
            const uint64_t two =
                (uint64_t)pl.occ[b >> 5] | ((uint64_t)pl.occ[(b >> 5) + 1] << 32);
            obits = (uint32_t)(two >> (b & 31)) & 0xFFFFu;
        }
    } else {
        uint32_t f[4] = {0u, 0u, 0u, 0u}, t[4] = {0u, 0u, 0u, 0u}, o[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            if (j >= nvalid)
                break;
            int32_t x = x0 + j;
            if (x >= gx)
                x -= gx;
            const int64_t b = prow + x;
            f[j >> 2] |= (uint32_t)pl.marks[b] << (8 * (j & 3));
            t[j >> 2] |= (uint32_t)pl.marks[pl.nbytes + b] << (8 * (j & 3));
            if (kBytes)
                o[j >> 2] |= (uint32_t)pl.occb[b] << (8 * (j & 3));
            else
                obits |= ((pl.occ[b >> 5] >> (b & 31)) & 1u) << j;
        }
        fr = make_uint4(f[0], f[1], f[2], f[3]);
        tr = make_uint4(t[0], t[1], t[2], t[3]);
        oc = make_uint4(o[0], o[1], o[2], o[3]);
    }
    m.o = kBytes ? byte_eq_ff16(oc, rep) : spread16(obits);
    m.t = byte_eq_ff16(tr, rep);
    m.f = byte_eq_ff16(fr, rep);
}

// The four 16-column chunks a wide merge lane reads, and the loads they need.
// Chunk s holds grid columns x0[s] .. (nv[s] of them, wrapping at the grid's
// width); want[s]: the lane reads it.  Chunks that lie in one run of grid
// columns load through buffer resources -- 20 bytes from the dword below the
// run's first byte, realigned with v_alignbyte -- and the others (not read,
// or wrapping at the seam) at an offset past every range, which reads 0
// without a branch; so every load of the lane is issued before the first is
// used.  The wrapping chunks are read byte by byte afterwards.
struct Lane64 {
    int32_t x0[4], nv[4];
    bool want[4];
};

template <bool kBytes>
struct Loads64 {
    uint4 f4[4], t4[4], o4[4];
    uint32_t f1[4], t1[4], o1[4];
    uint32_t sh[4];
    uint32_t ob[4][2], osh[4];
};

template <bool kBytes>
__device__ __forceinline__ void issue64(const Planes &pl, uint32_t prow, const Lane64 &c,
                                        Loads64<kBytes> &ld)
{
    const uint32_t nb = pl.nbytes;
    // one dword of slack past each plane: the plane that follows, or the
    // scratch region after the traced plane
    const __amdgpu_buffer_rsrc_t rm = buffer_rsrc(pl.marks, 2u * nb + 4u);
    const __amdgpu_buffer_rsrc_t ro =
        kBytes ? buffer_rsrc(pl.occb, nb + 4u) : buffer_rsrc(pl.occ, nb / 8u + 4u);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const uint32_t b = prow + (uint32_t)c.x0[s];
        const bool run = c.want[s] && c.x0[s] + c.nv[s] <= pl.n[0];
        const uint32_t off = run ? (b & ~3u) : kOob;
        ld.sh[s] = b & 3u;
        const auto f = __builtin_amdgcn_raw_buffer_load_b128(rm, (int)off, 0, 0);
        const auto t = __builtin_amdgcn_raw_buffer_load_b128(rm, (int)(off + nb), 0, 0);
        ld.f4[s] = make_uint4(f[0], f[1], f[2], f[3]);
        ld.t4[s] = make_uint4(t[0], t[1], t[2], t[3]);
        ld.f1[s] = __builtin_amdgcn_raw_buffer_load_b32(rm, (int)(off + 16u), 0, 0);
        ld.t1[s] = __builtin_amdgcn_raw_buffer_load_b32(rm, (int)(off + nb + 16u), 0, 0);
        if (kBytes) {
            const auto o = __builtin_amdgcn_raw_buffer_load_b128(ro, (int)off, 0, 0);
            ld.o4[s] = make_uint4(o[0], o[1], o[2], o[3]);
            ld.o1[s] = __builtin_amdgcn_raw_buffer_load_b32(ro, (int)(off + 16u), 0, 0);
        } else {
            const auto o = __builtin_amdgcn_raw_buffer_load_b64(ro, (int)(run ? (b >> 5) << 2 : kOob),
                                                                0, 0);
            ld.ob[s][0] = o[0];
            ld.ob[s][1] = o[1];
            ld.osh[s] = b & 31u;
        }
    }
}

__device__ __forceinline__ uint4 align16(const uint4 &v, uint32_t next, uint32_t sh)
{
    return make_uint4(__builtin_amdgcn_alignbyte(v.y, v.x, sh),
                      __builtin_amdgcn_alignbyte(v.z, v.y, sh),
                      __builtin_amdgcn_alignbyte(v.w, v.z, sh),
                      __builtin_amdgcn_alignbyte(next, v.w, sh));
}

template <bool kBytes>
__device__ __forceinline__ void finish64(const Planes &pl, uint32_t prow, const Lane64 &c,
                                         const Loads64<kBytes> &ld, Masks16 mk[4])
{
    const uint32_t rep = (pl.epoch & 0xFFu) * 0x01010101u;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        mk[s].f = byte_eq_ff16(align16(ld.f4[s], ld.f1[s], ld.sh[s]), rep);
        mk[s].t = byte_eq_ff16(align16(ld.t4[s], ld.t1[s], ld.sh[s]), rep);
        if (kBytes)
            mk[s].o = byte_eq_ff16(align16(ld.o4[s], ld.o1[s], ld.sh[s]), rep);
        else
            mk[s].o = spread16(__builtin_amdgcn_alignbit(ld.ob[s][1], ld.ob[s][0], ld.osh[s]) &
                               0xFFFFu);
        if (c.want[s] && c.x0[s] + c.nv[s] > pl.n[0])
            gather16<kBytes>(pl, prow, c.x0[s], c.nv[s], mk[s]);
    }
}

// Four voxels of the local grid: the bytes of cm become unknown (a shift's
// clear), then Alg. 3 -- an occupied voxel becomes occupied, else a traced
// one unknown, else a free one free; the others keep their value.
__device__ __forceinline__ uint32_t merge4(uint32_t v, uint32_t cm, uint32_t om, uint32_t tm,
                                          uint32_t fm)
{
    tm &= ~om;
    fm &= ~(om | tm);
    return (v & ~(cm | om | tm | fm)) | (0x02020202u & om) | (0x01010101u & fm);
}

__device__ __forceinline__ void apply16(uint4 &v, const uint4 &cm, const Masks16 &m)
{
    v.x = merge4(v.x, cm.x, m.o.x, m.t.x, m.f.x);
    v.y = merge4(v.y, cm.y, m.o.y, m.t.y, m.f.y);
    v.z = merge4(v.z, cm.z, m.o.z, m.t.z, m.f.z);
    v.w = merge4(v.w, cm.w, m.o.w, m.t.w, m.f.w);
}

// Whether the frame may change one of the nvalid grid columns x0 .. (wrapping
// at gx) given its runs of the row (bounded false: every column).
__device__ __forceinline__ bool run_touched(bool bounded, const int32_t run[4], int32_t gx,
                                            int32_t x0, int32_t nvalid)
{
    if (!bounded)
        return true;
    const int32_t e = x0 + nvalid - 1;
    if (e < gx)
        return runs_meet(run, x0, e);
    return runs_meet(run, x0, gx - 1) || runs_meet(run, 0, e - gx);
}

// Alg. 3: the frame's marks merged into the local grid, over the buffer rows
// that hold the grid rows of the row box: occupied bit -> occupied; else a
// traced stamp -> unknown; else a free stamp -> free; else unchanged.  The
// frame's planes are read at the grid columns each 16-column chunk holds (one
// run, or two where the ring wraps).  kWide (large launches): one lane per 64
// buffer columns (four chunks); only chunks within the frame's runs of the
// row (vg_frustum.h) are read, and every gather is issued before the local
// grid is read and written.  Otherwise one lane per chunk (more lanes for
// small launches).
template <bool kBytes, bool kWide>
__device__ __forceinline__ void resolve_body(const Planes &pl, uint8_t *loc, const RowBox &rows,
                                             const int32_t ring[3], int64_t gid)
{
    const int32_t ny = rows.y1 - rows.y0 + 1, nz = rows.z1 - rows.z0 + 1;
    const int32_t gx = pl.n[0];
    if (!kWide) {
        const int32_t chunks = pl.wx * 2;   // 16-column chunks per row
        if (ny <= 0 || nz <= 0 || gid >= (int64_t)chunks * ny * nz)
            return;
        const uint32_t g32 = (uint32_t)gid;   // < 2^26 chunks in a grid
        const int32_t k = (int32_t)(g32 % (uint32_t)chunks);
        const uint32_t row = g32 / (uint32_t)chunks;
        const int32_t y = rows.y0 + (int32_t)(row % (uint32_t)ny);
        const int32_t z = rows.z0 + (int32_t)(row / (uint32_t)ny);
        const int32_t c0 = 16 * k;   // buffer column of the chunk
        if (c0 >= gx)
            return;                  // row padding only
        const int32_t nvalid = min(16, gx - c0);
        const int32_t by = wrap_add(y, ring[1], pl.n[1]), bz = wrap_add(z, ring[2], pl.n[2]);
        const int64_t prow = 32 * (int64_t)pl.wx * (y + (int64_t)pl.n[1] * z);
        const int64_t brow = 32 * (int64_t)pl.wx * (by + (int64_t)pl.n[1] * bz);
        int32_t x0 = c0 - ring[0];   // grid column of buffer column c0
        if (x0 < 0)
            x0 += gx;
        Masks16 mk;
        gather16<kBytes>(pl, prow, x0, nvalid, mk);
        if (!any16(mk))
            return;
        uint8_t *dst = loc + brow + c0;
        uint4 v = *reinterpret_cast<const uint4 *>(dst);
        apply16(v, make_uint4(0u, 0u, 0u, 0u), mk);
        *reinterpret_cast<uint4 *>(dst) = v;
        return;
    }
    const int32_t lanes = merge_lanes_per_row(gx);
    if (ny <= 0 || nz <= 0 || gid >= (int64_t)lanes * ny * nz)
        return;
    const uint32_t g32 = (uint32_t)gid;   // < 2^26 lanes in a grid
    const int32_t k = (int32_t)(g32 % (uint32_t)lanes);
    const uint32_t row = g32 / (uint32_t)lanes;
    const int32_t y = rows.y0 + (int32_t)(row % (uint32_t)ny);
    const int32_t z = rows.z0 + (int32_t)(row / (uint32_t)ny);
    const int32_t by = wrap_add(y, ring[1], pl.n[1]), bz = wrap_add(z, ring[2], pl.n[2]);
    const int64_t prow = 32 * (int64_t)pl.wx * (y + (int64_t)pl.n[1] * z);    // planes
    const int64_t brow = 32 * (int64_t)pl.wx * (by + (int64_t)pl.n[1] * bz);  // buffer
    int32_t run[4];
    const bool bounded = pl.lim && row_runs(*const_limits(pl.lim), y, z, gx, run);
    // chunks within the runs: their planes and the local grid's 16 voxels
    // are loaded together (the runs are tight, so nearly all of them change)
    Lane64 c;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int32_t c0 = 64 * k + 16 * s;   // buffer column of the chunk
        int32_t x0 = c0 - ring[0];             // grid column of buffer column c0
        if (x0 < 0)
            x0 += gx;
        c.x0[s] = x0;
        c.nv[s] = min(16, gx - c0);
        // c0 >= gx: row padding only
        c.want[s] = c0 < gx && run_touched(bounded, run, gx, x0, c.nv[s]);
    }
    Loads64<kBytes> ld;
    issue64<kBytes>(pl, (uint32_t)prow, c, ld);
    const __amdgpu_buffer_rsrc_t rl = buffer_rsrc(loc, pl.nbytes);
    uint4 v[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const uint32_t off = c.want[s] ? (uint32_t)brow + 64u * k + 16u * s : kOob;
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(rl, (int)off, 0, 0);
        v[s] = make_uint4(q[0], q[1], q[2], q[3]);
    }
    Masks16 mk[4];
    finish64<kBytes>(pl, (uint32_t)prow, c, ld, mk);
#pragma unroll
    for (int s = 0; s < 4; ++s)
        if (c.want[s] && any16(mk[s])) {
            apply16(v[s], make_uint4(0u, 0u, 0u, 0u), mk[s]);
            *reinterpret_cast<uint4 *>(loc + brow + 64 * k + 16 * s) = v[s];
        }
}

// Bits a .. b - 1 of a 16-bit mask, clamped to 0 .. 16.
__device__ __forceinline__ uint32_t range_mask16(int32_t a, int32_t b)
{
    a = max(a, 0);
    b = min(b, 16);
    return a < b ? ((1u << b) - 1u) & ~((1u << a) - 1u) : 0u;
}

// Columns of 16 grid columns (x0 .. , wrapping; nvalid of them) in row (y, z)
// that a frame's shift clears (clear_body's rule); none if it does not shift.
// Column j holds grid column x0 + j, or x0 + j - gx past the seam.
__device__ __forceinline__ uint32_t clear_mask16(const SlabClear &c, int32_t y, int32_t z,
                                                 int32_t x0, int32_t nvalid)
{
    if (!c.loc)
        return 0u;
    const uint32_t valid = nvalid >= 16 ? 0xFFFFu : (1u << nvalid) - 1u;
    if ((y >= c.lo[1] && y < c.hi[1]) || (z >= c.lo[2] && z < c.hi[2]) ||
        c.hi[0] - c.lo[0] >= c.n[0])
        return valid;
    if (c.lo[0] >= c.hi[0])
        return 0u;
    // j with x0 + j in [lo, hi), and past the seam j with x0 + j - gx in it
    const uint32_t m = range_mask16(c.lo[0] - x0, c.hi[0] - x0) |
                       range_mask16(c.lo[0] - x0 + c.n[0], c.hi[0] - x0 + c.n[0]);
    return m & valid;
}

// Alg. 3 for a run of consecutive frames of one grid (fd[0 .. group), in
// order), each walked into its own planes in its own grid coordinates, with
// the shifts between them (Sec. IV-E): every voxel ends as if the frames had
// been merged one after another -- per frame, first its shift's clear, then
// its marks, so the latest frame that saw the voxel decides.  The shifts'
// clears have already run over the whole grid (the batch's shift stage);
// here they are applied again in order, so that they also undo the marks of
// earlier frames of the run.  One lane per 64 buffer columns (four 16-column
// chunks) of a buffer row that holds a grid row (in the coordinates of the
// run's last frame) of the merge's domain; each frame's planes are read at
// its own grid coordinates of those voxels, where its row box and its runs
// of the row hold them.
__device__ __forceinline__ void resolve_seq_body(const FrameDesc *fd, int64_t gid)
{
    const FrameDesc &f0 = fd[0];
    const int32_t m = f0.group;
    const RowBox &dom = f0.dom;
    const Planes &pl0 = f0.sp.pl;
    const int32_t ny = dom.y1 - dom.y0 + 1, nz = dom.z1 - dom.z0 + 1;
    const int32_t gx = pl0.n[0], gy = pl0.n[1], gz = pl0.n[2];
    const int32_t lanes = merge_lanes_per_row(gx);
    if (m <= 0 || ny <= 0 || nz <= 0 || gid >= (int64_t)lanes * ny * nz)
        return;
    const uint32_t g32 = (uint32_t)gid;   // < 2^26 lanes in a grid
    const int32_t k = (int32_t)(g32 % (uint32_t)lanes);
    const uint32_t row = g32 / (uint32_t)lanes;
    const FrameDesc &fl = fd[m - 1];
    const int32_t by = wrap_add(dom.y0 + (int32_t)(row % (uint32_t)ny), fl.ring[1], gy);
    const int32_t bz = wrap_add(dom.z0 + (int32_t)(row / (uint32_t)ny), fl.ring[2], gz);
    uint8_t *dst = f0.loc + 32 * (int64_t)pl0.wx * (by + (int64_t)gy * bz) + 64 * k;
    uint4 v[4];
    uint32_t loaded = 0;   // bit s: v[s] holds the grid's 16 voxels of chunk s
    for (int32_t j = 0; j < m; ++j) {
        const FrameDesc &f = fd[j];
        int32_t y = by - f.ring[1], z = bz - f.ring[2];
        if (y < 0)
            y += gy;
        if (z < 0)
            z += gz;
        const bool in_rows = y >= f.rows.y0 && y <= f.rows.y1 && z >= f.rows.z0 && z <= f.rows.z1;
        int32_t run[4];
        const bool bounded =
            in_rows && f.sp.pl.lim && row_runs(*const_limits(f.sp.pl.lim), y, z, gx, run);
        const uint32_t prow = 32u * (uint32_t)pl0.wx * (uint32_t)(y + gy * z);
        Lane64 c;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int32_t c0 = 64 * k + 16 * s;
            int32_t x0 = c0 - f.ring[0];
            if (x0 < 0)
                x0 += gx;
            c.x0[s] = x0;
            c.nv[s] = min(16, gx - c0);
            c.want[s] = c0 < gx && in_rows && run_touched(bounded, run, gx, x0, c.nv[s]);
        }
        Loads64<false> ld;
        issue64<false>(f.sp.pl, prow, c, ld);
        Masks16 mk[4];
        finish64<false>(f.sp.pl, prow, c, ld, mk);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int32_t c0 = 64 * k + 16 * s;
            if (c0 >= gx)
                continue;
            const uint32_t cm = clear_mask16(f.clear, y, z, c.x0[s], c.nv[s]);
            if (cm == 0u && !(c.want[s] && any16(mk[s])))
                continue;
            if (!((loaded >> s) & 1u)) {
                v[s] = *reinterpret_cast<const uint4 *>(dst + 16 * s);
                loaded |= 1u << s;
            }
            apply16(v[s], spread16(cm), mk[s]);
        }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
        if ((loaded >> s) & 1u)
            *reinterpret_cast<uint4 *>(dst + 16 * s) = v[s];
}

// Sec. IV-E on the ring buffer: the voxels of the exposed slabs become
// unknown, 16 buffer columns per lane (the lane parts of SlabClear).  Part A
// clears, in every grid row, the buffer columns of its chunks that hold grid
// columns of the exposed x slab; parts B and C clear whole rows of the
// exposed y and z slabs (16-byte stores).  Lanes of different parts may
// clear the same voxel; every store writes unknown.
__device__ __forceinline__ void clear_body(const SlabClear &c, int64_t gid)
{
    const int32_t cpr = c.gxp >> 4;   // 16-column chunks per buffer row
    int32_t y, z, chunk;
    bool whole;
    if (gid < c.lanes[0]) {
        const int32_t na = c.xrun[1] - c.xrun[0];
        const int32_t per = na + (c.xrun[3] - c.xrun[2]);
        const uint32_t g32 = (uint32_t)gid, row = g32 / (uint32_t)per;
        const int32_t j = (int32_t)(g32 - row * (uint32_t)per);
        chunk = j < na ? c.xrun[0] + j : c.xrun[2] + (j - na);
        y = (int32_t)(row % (uint32_t)c.n[1]);
        z = (int32_t)(row / (uint32_t)c.n[1]);
        whole = c.hi[0] - c.lo[0] >= c.n[0];
    } else if (gid < c.lanes[0] + c.lanes[1]) {
        const uint32_t g32 = (uint32_t)(gid - c.lanes[0]), row = g32 / (uint32_t)cpr;
        chunk = (int32_t)(g32 - row * (uint32_t)cpr);
        const int32_t ny = c.hi[1] - c.lo[1];
        y = c.lo[1] + (int32_t)(row % (uint32_t)ny);
        z = (int32_t)(row / (uint32_t)ny);
        whole = true;
    } else if (gid < c.lanes[0] + c.lanes[1] + c.lanes[2]) {
        const uint32_t g32 = (uint32_t)(gid - c.lanes[0] - c.lanes[1]);
        const uint32_t row = g32 / (uint32_t)cpr;
        chunk = (int32_t)(g32 - row * (uint32_t)cpr);
        y = (int32_t)(row % (uint32_t)c.n[1]);
        z = c.lo[2] + (int32_t)(row / (uint32_t)c.n[1]);
        whole = true;
    } else {
        return;
    }
    const int32_t c0 = 16 * chunk;
    const int32_t by = wrap_add(y, c.ring[1], c.n[1]), bz = wrap_add(z, c.ring[2], c.n[2]);
    uint8_t *dst = c.loc + (int64_t)c.gxp * (by + (int64_t)c.n[1] * bz) + c0;
    if (whole) {
        *reinterpret_cast<uint4 *>(dst) = make_uint4(0u, 0u, 0u, 0u);
        return;
    }
    for (int j = 0; j < 16; ++j) {
        const int32_t col = c0 + j;
        if (col >= c.n[0])
            break;
        int32_t x = col - c.ring[0];       // grid column held by buffer column col
        if (x < 0)
            x += c.n[0];
        if (x >= c.lo[0] && x < c.hi[0])
            dst[j] = kUnknown;
    }
}

// ------------------------------------------------------- one-frame kernels

// Walk length estimate of the pinhole target (ia, ib) from inside the grid:
// the distance to the target or to the grid's boundary along the ray,
// whichever is nearer, times the steps per unit length (|u_x| + |u_y| +
// |u_z| for the unit direction u).  It only orders blocks, so approximate
// reciprocals do.
__device__ __forceinline__ float walk_cost(const RayParams &p, int32_t ia, int32_t ib)
{
    const float x = (float)(ia - p.hw), y = (float)(ib - p.hh), z = (float)p.vd;
    float d[3];
    ray_direction(p, ia - p.hw, ib - p.hh, p.vd, d);
    const float len = sqrtf(x * x + y * y + z * z);
    const float il = __builtin_amdgcn_rcpf(len);
    float t = len, l1 = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = d[a] * il;
        l1 += fabsf(u);
        const float o = p.wf.o[a], n = (float)p.wf.n[a];
        const float ta = u > 0.0f   ? (n - o) * __builtin_amdgcn_rcpf(u)
                         : u < 0.0f ? -o * __builtin_amdgcn_rcpf(u)
                                    : len;
        t = fminf(t, fmaxf(ta, 0.0f));
    }
    return t * l1;
}

// Rating workgroup `part` (< ob.parts) of a walk-order build (WalkOrder):
// the level of each of its ray blocks -- the highest walk-length estimate at
// the corner targets of the block's tiles (of the box of its four tiles
// where they share a row of tiles), in kOrderLevels steps.  Four consecutive
// lanes take the four corners of a block.
__device__ __forceinline__ void rate_walk_blocks(const OrderBuild &ob, int32_t part)
{
    const RayParams &p = ob.rp;
    const int32_t t = (int32_t)threadIdx.x;
    const int32_t tw = 1 << p.tile_log2w, th = 64 >> p.tile_log2w;
    const float top = 1.7321f * sqrtf((float)p.hw * p.hw + (float)p.hh * p.hh +
                                      (float)p.vd * p.vd);
    const float scale = (float)(kOrderLevels - 1) / fmaxf(top, 1.0f);
    const int32_t corner = t & 3;
    const int32_t per = ob.parts * (kBlock / 4);   // blocks per round of the parts
    // every lane runs the same rounds (the shuffles need all four lanes)
    for (int32_t j0 = part * (kBlock / 4); j0 < ob.ray_blocks; j0 += per) {
        const int32_t j = j0 + (t >> 2);
        float c = 0.0f;
        if (j < ob.ray_blocks) {
            const int32_t first = 4 * j, lastt = min(4 * j + 3, p.tiles - 1);
            if (first / p.tiles_a == lastt / p.tiles_a) {   // one row of tiles: the box
                const int32_t a0 = (first % p.tiles_a) * tw, b0 = (first / p.tiles_a) * th;
                const int32_t a1 = min((lastt % p.tiles_a + 1) * tw, p.na) - 1;
                const int32_t b1 = min(b0 + th, p.nb) - 1;
                c = walk_cost(p, corner & 1 ? a1 : a0, corner & 2 ? b1 : b0);
            } else {   // across two rows of tiles: each lane one tile's corners
                const int32_t tile = first + corner;
                if (tile <= lastt) {
                    const int32_t a0 = (tile % p.tiles_a) * tw, b0 = (tile / p.tiles_a) * th;
                    const int32_t a1 = min(a0 + tw, p.na) - 1, b1 = min(b0 + th, p.nb) - 1;
                    c = fmaxf(fmaxf(walk_cost(p, a0, b0), walk_cost(p, a1, b0)),
                              fmaxf(walk_cost(p, a0, b1), walk_cost(p, a1, b1)));
                }
            }
        }
        c = fmaxf(c, __shfl_xor(c, 1));
        c = fmaxf(c, __shfl_xor(c, 2));
        if (j < ob.ray_blocks && corner == 0)
            ob.keys[j] = (uint8_t)min(max((int32_t)(c * scale), 0), kOrderLevels - 1);
    }
}

// The sorting workgroup of a walk-order build, in the launch after the
// rating one.  It orders runs of kXcdRun consecutive blocks, not blocks, so
// that each run still lands on one XCD (xcd_runs deals positions out in such
// runs): every whole run by its highest level, highest first (a counting sort
// in LDS); the blocks past the last whole run keep their positions.  Then
// the tag.
__device__ __forceinline__ void sort_walk_blocks(const OrderBuild &ob)
{
    constexpr int32_t kRunsPerThread = kOrderMaxBlocks / kXcdRun / kBlock;
    __shared__ int32_t cnt[kOrderLevels], pos[kOrderLevels];
    const RayParams &p = ob.rp;
    const int32_t nblk = ob.ray_blocks, nrun = nblk / kXcdRun;
    const int32_t t = (int32_t)threadIdx.x;   // kBlock == kOrderLevels threads
    WalkOrderTag *tag = reinterpret_cast<WalkOrderTag *>(ob.order);
    if (t == 0)
        tag->ray_blocks = 0;   // no valid order while it is rewritten
    cnt[t] = 0;
    __syncthreads();
    // each thread's runs' levels: all their blocks' levels load together
    int32_t lv[kRunsPerThread];
#pragma unroll
    for (int32_t r = 0; r < kRunsPerThread; ++r) {
        const int32_t run = min(t + r * kBlock, max(nrun - 1, 0));
        uint32_t k[kXcdRun];
#pragma unroll
        for (int32_t i = 0; i < kXcdRun; ++i)
            k[i] = ob.keys[min(run * kXcdRun + i, nblk - 1)];
        uint32_t m = 0;
#pragma unroll
        for (int32_t i = 0; i < kXcdRun; ++i)
            m = max(m, k[i]);
        lv[r] = (int32_t)m;
        if (t + r * kBlock < nrun)
            atomicAdd(&cnt[m], 1);
    }
    __syncthreads();
    // pos[k] = runs of levels above k (Hillis-Steele over the levels from
    // the top: thread t holds level kOrderLevels - 1 - t)
    const int32_t v = cnt[kOrderLevels - 1 - t];
    pos[t] = v;
    __syncthreads();
    for (int32_t off = 1; off < kOrderLevels; off <<= 1) {
        const int32_t w = t >= off ? pos[t - off] : 0;
        __syncthreads();
        pos[t] += w;
        __syncthreads();
    }
    const bool whole = pos[kOrderLevels - 1] == nrun;   // every run counted once
    cnt[kOrderLevels - 1 - t] = pos[t] - v;   // next free position of each level
    __syncthreads();
    if (!whole)
        return;
    int32_t *out = ob.order + kOrderTagInts;
#pragma unroll
    for (int32_t r = 0; r < kRunsPerThread; ++r) {
        const int32_t run = t + r * kBlock;
        if (run < nrun) {
            const int32_t at = atomicAdd(&cnt[lv[r]], 1);
            if (at < nrun)
#pragma unroll
                for (int32_t i = 0; i < kXcdRun; ++i)
                    out[at * kXcdRun + i] = run * kXcdRun + i;
        }
    }
    for (int32_t j = nrun * kXcdRun + t; j < nblk; j += kBlock)
        out[j] = j;
    __syncthreads();
    if (t == 0) {
        tag->tiles_a = p.tiles_a;
        tag->tiles = p.tiles;
        tag->tile_log2w = p.tile_log2w;
        tag->ray_blocks = nblk;
    }
}

// The ray block that takes position rb: the frame's order if it was built
// for this launch's blocks, else rb.
__device__ __forceinline__ int32_t ordered_block(const RayParams &p, int32_t nblk, int32_t rb)
{
    const WalkOrderTag tag = *reinterpret_cast<const WalkOrderTag *>(p.order_in);
    if (tag.ray_blocks != nblk || tag.tiles_a != p.tiles_a || tag.tiles != p.tiles ||
        tag.tile_log2w != p.tile_log2w)
        return rb;
    return p.order_in[kOrderTagInts + rb];
}

// The seed pass; with ob.order, an extra row of workgroups rates the walk's
// ray blocks instead.
__global__ __launch_bounds__(kBlock) void k_seed(SeedParams p, OrderBuild ob)
{
    int32_t by = (int32_t)blockIdx.y;
    if (ob.order) {   // the first row, so that it runs beside the seeds
        if (by == 0) {
            if ((int32_t)blockIdx.x < ob.parts)
                rate_walk_blocks(ob, (int32_t)blockIdx.x);
            return;
        }
        --by;
    }
    seed_body(p, blockIdx.x, by);
}

// The x dilation; with ob.order, workgroup 0 sorts the frame's walk order
// instead.
template <bool kWide>
__global__ __launch_bounds__(kBlock) void k_dilate_x(Planes pl, OrderBuild ob)
{
    int32_t b = (int32_t)blockIdx.x;
    if (ob.order) {
        if (b == 0) {
            sort_walk_blocks(ob);
            return;
        }
        --b;
    }
    dilate_x_body<kWide>(pl, (int64_t)b * kBlock + threadIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_dilate_yz(Planes pl)
{
    dilate_yz_body(pl, (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

template <int kW, int kTZ>
__global__ __launch_bounds__(kBlock) void k_dilate_yz_tile(Planes pl)
{
    extern __shared__ uint32_t lds[];
    dilate_yz_tile_body<kW, kTZ>(pl, blockIdx.x, blockIdx.y, lds);
}

// The walk, one wavefront per workgroup: a compute unit starts the next
// wavefront as soon as one of its SIMDs has a free slot, where a workgroup of
// four waits for a slot on each (the walk took 139 -> 135 us on the 1280x720
// frame), and a small launch spreads over more compute units.  In a launch of
// more than kLoneWaves wavefronts wavefront u walks tile w of ray block
// position bb; the four tiles of a position go to one XCD, as workgroup bb of
// four wavefronts would (workgroups go to the 8 XCDs in turn), so the
// positions keep their XCD runs and their walk order.  Workgroups from
// 4 ray_blocks on run the slab clear c, 64 lanes each.  kLone: the walk form
// that overlaps each chunk's loads with the next chunk's steps.
constexpr int32_t kTiles = kBlock / 64;   // tiles per ray block

// Wavefront u (< kTiles * ray_blocks) of a launch with one wavefront per
// workgroup: tile w of ray block position bb.  Whole rounds of 8 positions x
// 4 tiles: wavefront u = 32 j + 8 w + x walks tile w of position 8 j + x; the
// last partial round in order.
__device__ __forceinline__ void wave_position(int32_t ray_blocks, int32_t u, int32_t &bb,
                                              int32_t &w)
{
    const int32_t full = 8 * kTiles * (ray_blocks / 8);
    if (u < full) {
        const int32_t k = u >> 3, x = u & 7;
        bb = (k / kTiles) * 8 + x;
        w = k % kTiles;
    } else {
        bb = ray_blocks / 8 * 8 + (u - full) / kTiles;
        w = (u - full) % kTiles;
    }
}

template <bool kGeneral, bool kBytes, bool kLone>
__global__ __launch_bounds__(64) void k_rays_w(RayParams p, SlabClear c, int32_t ray_blocks)
{
    const int32_t units = kTiles * ray_blocks, u = (int32_t)blockIdx.x;
    if (u >= units) {
        clear_body(c, (int64_t)(u - units) * 64 + threadIdx.x);
        return;
    }
    if (kLone && units <= kLoneWaves) {
        // every wavefront resident at once: each XCD takes a contiguous range
        // of tiles, whose neighbours share cache lines in its L2
        const int32_t q = units / 8, rem = units % 8, x = u % 8;
        rays_body<kGeneral, kBytes, kLone>(p, x * q + min(x, rem) + u / 8);
        return;
    }
    int32_t bb, w;
    wave_position(ray_blocks, u, bb, w);
    int32_t rb = xcd_runs(bb, ray_blocks);
    if (p.order_in)
        rb = ordered_block(p, ray_blocks, rb);
    rays_body<kGeneral, kBytes, kLone>(p, rb * kTiles + w);
}

// One wavefront per workgroup, as the walk of large launches: at 4 wavefronts
// per SIMD (117 VGPRs on the wide path) a wavefront starts wherever a slot
// frees (19.2 -> 18.9 us on the 1280x720 frame).
template <bool kBytes, bool kWide>
__global__ __launch_bounds__(64) void k_resolve(Planes pl, uint8_t *loc, RowBox rows, int32_t rx,
                                                int32_t ry, int32_t rz)
{
    const int32_t ring[3] = {rx, ry, rz};
    resolve_body<kBytes, kWide>(pl, loc, rows, ring, (int64_t)blockIdx.x * 64 + threadIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_clear(SlabClear c)
{
    clear_body(c, (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

// ----------------------------------------------------------- batch kernels
// One launch per stage for every frame of a batch round.  start[0..n] is the
// stage's block prefix over the round's frames; a block finds its frame by a
// (wavefront-uniform) binary search and works on that frame's local block.

__device__ __forceinline__ int32_t frame_of(const int32_t *__restrict__ start, int32_t n,
                                            int32_t block, int32_t &local)
{
    int32_t lo = 0, hi = n - 1;   // start[lo] <= block < start[hi + 1]
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (start[mid] <= block)
            lo = mid;
        else
            hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    local = block - start[lo];
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_upload(UploadBlob b)
{
    for (uint32_t i = threadIdx.x; i < b.words; i += kBlock)
        b.dst[i] = b.w[i];
}

__global__ __launch_bounds__(kBlock) void kb_clear(const FrameDesc *__restrict__ fd,
                                                   const int32_t *__restrict__ start, int32_t n)
{
    int32_t local;
    const FrameDesc &f = fd[frame_of(start, n, blockIdx.x, local)];
    clear_body(f.clear, (int64_t)local * kBlock + threadIdx.x);
}

__global__ __launch_bounds__(kBlock) void kb_seed(const FrameDesc *__restrict__ fd,
                                                  const int32_t *__restrict__ start, int32_t n)
{
    int32_t local;
    const FrameDesc &f = fd[frame_of(start, n, blockIdx.x, local)];
    if (f.seed_bx > 0)
        seed_body(f.sp, local % f.seed_bx, local / f.seed_bx);
    else
        seed_body(f.sp, local, 0);
}

template <bool kWide>
__global__ __launch_bounds__(kBlock) void kb_dilate_x(const FrameDesc *__restrict__ fd,
                                                      const int32_t *__restrict__ start, int32_t n)
{
    int32_t local;
    const FrameDesc &f = fd[frame_of(start, n, blockIdx.x, local)];
    dilate_x_body<kWide>(f.sp.pl, (int64_t)local * kBlock + threadIdx.x);
}

__global__ __launch_bounds__(kBlock) void kb_dilate_yz(const FrameDesc *__restrict__ fd,
                                                       const int32_t *__restrict__ start,
                                                       int32_t n)
{
    int32_t local;
    const FrameDesc &f = fd[frame_of(start, n, blockIdx.x, local)];
    dilate_yz_body(f.sp.pl, (int64_t)local * kBlock + threadIdx.x);
}

template <int kW, int kTZ>
__global__ __launch_bounds__(kBlock) void kb_dilate_yz_tile(const FrameDesc *__restrict__ fd,
                                                            const int32_t *__restrict__ start,
                                                            int32_t n)
{
    extern __shared__ uint32_t lds[];
    int32_t local;
    const FrameDesc &f = fd[frame_of(start, n, blockIdx.x, local)];
    constexpr int32_t kTY = kBlock / kW;
    const int32_t tiles_y = (f.sp.pl.n[1] + kTY - 1) / kTY;
    dilate_yz_tile_body<kW, kTZ>(f.sp.pl, local % tiles_y, local / tiles_y, lds);
}

// One wavefront per workgroup, as k_rays_w: wavefront u walks tile w of the
// stage's ray block position bb.
__global__ __launch_bounds__(64) void kb_rays(const FrameDesc *__restrict__ fd,
                                              const int32_t *__restrict__ start, int32_t n)
{
    int32_t bb, w, local;
    wave_position(start[n], (int32_t)blockIdx.x, bb, w);
    const FrameDesc &f = fd[frame_of(start, n, xcd_runs(bb, start[n]), local)];
    const int32_t tile = local * kTiles + w;
    if (f.inside)
        rays_body<false, false, true>(f.rp, tile);
    else
        rays_body<true, false, false>(f.rp, tile);
}

template <bool kWide>
// One wavefront per workgroup, as k_resolve: workgroup u is wavefront u % 4
// of the stage's block u / 4 (start[] counts blocks of kBlock = 256 lanes).
__global__ __launch_bounds__(64) void kb_resolve(const FrameDesc *__restrict__ fd,
                                                 const int32_t *__restrict__ start, int32_t n)
{
    int32_t local;
    const FrameDesc &f = fd[frame_of(start, n, (int32_t)blockIdx.x >> 2, local)];
    resolve_body<false, kWide>(f.sp.pl, f.loc, f.rows, f.ring,
                               (int64_t)local * kBlock + (blockIdx.x & 3u) * 64u + threadIdx.x);
}

// The merge of a round that holds runs of frames of one grid: a block finds
// the first frame of its run (the run's other frames have no blocks).
__global__ __launch_bounds__(64) void kb_resolve_seq(const FrameDesc *__restrict__ fd,
                                                     const int32_t *__restrict__ start,
                                                     int32_t n)
{
    int32_t local;
    const int32_t i = frame_of(start, n, (int32_t)blockIdx.x >> 2, local);
    resolve_seq_body(fd + i, (int64_t)local * kBlock + (blockIdx.x & 3u) * 64u + threadIdx.x);
}

uint32_t blocks_for(int64_t threads) { return (uint32_t)((threads + kBlock - 1) / kBlock); }

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_fill(void *dst, uint8_t value, size_t bytes, hipStream_t st)
{
    if (bytes == 0)
        return hipSuccess;
    uintptr_t base = (uintptr_t)dst & ~(uintptr_t)15;
    size_t chunks = ((uintptr_t)dst + bytes - base + 15) / 16;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for((int64_t)chunks)), dim3(kBlock), 0, st,
                       (uint8_t *)dst, value, bytes);
    return hipGetLastError();
}

hipError_t record_empty_stage(const StageEvents &ev, hipStream_t st)
{
    hipError_t e = hipSuccess;
    if (ev.start)
        e = hipEventRecord(ev.start, st);
    if (e == hipSuccess && ev.stop)
        e = hipEventRecord(ev.stop, st);
    return e;
}

hipError_t launch_seeds(const SeedParams &p, hipStream_t st, const StageEvents &ev,
                        const OrderBuild *order)
{
    dim3 grid;
    if (p.kind == kPoints)
        grid = dim3(std::max<uint32_t>(blocks_for(p.W), 1u), 1);
    else
        grid = dim3((uint32_t)std::max((p.W + 63) / 64, 1), (uint32_t)std::max((p.H + 3) / 4, 1));
    OrderBuild ob{};
    if (order && order->order) {
        // an extra row of workgroups rates the walk's blocks
        ob = *order;
        ob.parts = (int32_t)std::min<uint32_t>(grid.x, (uint32_t)kOrderMaxParts);
        grid.y += 1;
    }
    hipExtLaunchKernelGGL(k_seed, grid, dim3(kBlock), 0, st, ev.start, ev.stop, 0, p, ob);
    return hipGetLastError();
}

hipError_t launch_dilate(const Planes &pl, hipStream_t st, const StageEvents &ev,
                         const OrderBuild *order)
{
    const bool any = pl.lo[0] <= pl.hi[0] && pl.lo[1] <= pl.hi[1] && pl.lo[2] <= pl.hi[2];
    hipEvent_t start = ev.start;
    if (any) {
        const int64_t rows = (int64_t)(pl.hi[1] - pl.lo[1] + 1) * (pl.hi[2] - pl.lo[2] + 1);
        const bool wide = dilate_x_wide((int64_t)pl.wx * rows);
        const int64_t n = (int64_t)dilate_x_lanes(pl.wx, wide) * rows;
        OrderBuild ob{};
        if (order && order->order)
            ob = *order;
        hipExtLaunchKernelGGL(wide ? k_dilate_x<true> : k_dilate_x<false>,
                              dim3(blocks_for(n) + (ob.order ? 1u : 0u)), dim3(kBlock), 0, st,
                              start, (hipEvent_t) nullptr, 0, pl, ob);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        start = nullptr;
    }
    // 8-deep tiles where there are enough of them to fill the chip, else 2-deep
    YzTile t{dilate_tile_width(pl, kTileDeep), kTileDeep};
    if (t.kw == 0 || dilate_tiles(pl, t) < kDeepTileMin)
        t = YzTile{dilate_tile_width(pl, 2), 2};
    if (t.kw > 0) {
        const uint32_t lds = (uint32_t)dilate_tile_lds(pl, t);
        const int32_t ty = kBlock / t.kw;
        const dim3 tiles((uint32_t)((pl.n[1] + ty - 1) / ty),
                         (uint32_t)((pl.n[2] + t.tz - 1) / t.tz));
        auto kern = t.kw == 8 ? (t.tz == 2 ? k_dilate_yz_tile<8, 2> : k_dilate_yz_tile<8, 8>)
                              : (t.tz == 2 ? k_dilate_yz_tile<16, 2> : k_dilate_yz_tile<16, 8>);
        hipExtLaunchKernelGGL(kern, tiles, dim3(kBlock), lds, st, start, ev.stop, 0, pl);
        return hipGetLastError();
    }
    int64_t n = (int64_t)pl.wx * pl.n[1] * pl.n[2];
    hipExtLaunchKernelGGL(k_dilate_yz, dim3(blocks_for(n)), dim3(kBlock), 0, st, start, ev.stop,
                          0, pl);
    return hipGetLastError();
}

hipError_t launch_rays(const RayParams &p, bool camera_inside, hipStream_t st,
                       const StageEvents &ev, const SlabClear *clear)
{
    const int64_t ray_blocks = (p.tiles + kTiles - 1) / kTiles;
    SlabClear c{};
    int64_t clear_blocks = 0;
    if (clear) {
        c = *clear;
        clear_blocks = blocks_for(clear_lanes(c));
    }
    if (ray_blocks + clear_blocks == 0)
        return record_empty_stage(ev, st);
    // one wavefront per workgroup, kTiles per block of rays or of the clear;
    // the camera inside the grid: the walk form that keeps its loads in
    // flight; from outside, every step takes the tested path anyway
    const dim3 g((uint32_t)(kTiles * (ray_blocks + clear_blocks))), b(64);
    if (camera_inside && !p.occ_is_bytes)
        hipExtLaunchKernelGGL((k_rays_w<false, false, true>), g, b, 0, st, ev.start, ev.stop, 0,
                              p, c, (int32_t)ray_blocks);
    else if (camera_inside)
        hipExtLaunchKernelGGL((k_rays_w<false, true, true>), g, b, 0, st, ev.start, ev.stop, 0, p,
                              c, (int32_t)ray_blocks);
    else if (!p.occ_is_bytes)
        hipExtLaunchKernelGGL((k_rays_w<true, false, false>), g, b, 0, st, ev.start, ev.stop, 0,
                              p, c, (int32_t)ray_blocks);
    else
        hipExtLaunchKernelGGL((k_rays_w<true, true, false>), g, b, 0, st, ev.start, ev.stop, 0, p,
                              c, (int32_t)ray_blocks);
    return hipGetLastError();
}

hipError_t launch_resolve(const Planes &pl, uint8_t *loc, const RowBox &rows,
                          const int32_t ring[3], hipStream_t st, const StageEvents &ev)
{
    if (rows.y0 > rows.y1 || rows.z0 > rows.z1)
        return record_empty_stage(ev, st);
    const int32_t ny = rows.y1 - rows.y0 + 1, nz = rows.z1 - rows.z0 + 1;
    const bool wide = merge_wide(pl.n[0], (int64_t)ny * nz);
    const int64_t n = (int64_t)merge_lanes(pl.n[0], wide) * ny * nz;
    auto kern = pl.occb ? (wide ? k_resolve<true, true> : k_resolve<true, false>)
                        : (wide ? k_resolve<false, true> : k_resolve<false, false>);
    hipExtLaunchKernelGGL(kern, dim3((uint32_t)((n + 63) / 64)), dim3(64), 0, st, ev.start,
                          ev.stop, 0, pl, loc, rows, ring[0], ring[1], ring[2]);
    return hipGetLastError();
}

hipError_t launch_clear(const SlabClear &c, hipStream_t st, const StageEvents &ev)
{
    const int64_t lanes = clear_lanes(c);
    if (lanes == 0)
        return record_empty_stage(ev, st);
    hipExtLaunchKernelGGL(k_clear, dim3(blocks_for(lanes)), dim3(kBlock), 0, st, ev.start,
                          ev.stop, 0, c);
    return hipGetLastError();
}

hipError_t static_batch_workspace(void **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!p || ((uintptr_t)p % 256) != 0)
            return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_upload(uint32_t *dst, const uint32_t *src, size_t words, hipStream_t st)
{
    UploadBlob b;
    for (size_t at = 0; at < words; at += kUploadWords) {
        b.dst = dst + at;
        b.words = (uint32_t)std::min<size_t>(kUploadWords, words - at);
        std::copy(src + at, src + at + b.words, b.w);
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(kBlock), 0, st, b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_batch_stage(int stage, const FrameDesc *fd, const int32_t *start, int32_t n,
                              int32_t blocks, hipStream_t st, const StageEvents &ev, YzTile tile,
                              size_t lds, bool seq, bool wide)
{
    if (blocks <= 0 || n <= 0)
        return record_empty_stage(ev, st);
    const dim3 g((uint32_t)blocks), b(kBlock);
    switch (stage) {
    case kBatchShift:
        hipExtLaunchKernelGGL(kb_clear, g, b, 0, st, ev.start, ev.stop, 0, fd, start, n);
        break;
    case kBatchSeed:
        hipExtLaunchKernelGGL(kb_seed, g, b, 0, st, ev.start, ev.stop, 0, fd, start, n);
        break;
    case kBatchDilateX:
        if (wide)
            hipExtLaunchKernelGGL(kb_dilate_x<true>, g, b, 0, st, ev.start, ev.stop, 0, fd, start,
                                  n);
        else
            hipExtLaunchKernelGGL(kb_dilate_x<false>, g, b, 0, st, ev.start, ev.stop, 0, fd,
                                  start, n);
        break;
    case kBatchDilateYZ:
        if (tile.kw > 0) {
            auto kern = tile.kw == 8
                            ? (tile.tz == 2 ? kb_dilate_yz_tile<8, 2> : kb_dilate_yz_tile<8, 8>)
                            : (tile.tz == 2 ? kb_dilate_yz_tile<16, 2> : kb_dilate_yz_tile<16, 8>);
            hipExtLaunchKernelGGL(kern, g, b, (uint32_t)lds, st, ev.start, ev.stop, 0, fd, start,
                                  n);
        } else {
            hipExtLaunchKernelGGL(kb_dilate_yz, g, b, 0, st, ev.start, ev.stop, 0, fd, start, n);
        }
        break;
    case kBatchRays:
        hipExtLaunchKernelGGL(kb_rays, dim3((uint32_t)(kTiles * blocks)), dim3(64), 0, st,
                              ev.start, ev.stop, 0, fd, start, n);
        break;
    case kBatchResolve: {
        // one wavefront per workgroup, kBlock / 64 per block of the stage's prefix
        const dim3 g4((uint32_t)(kBlock / 64) * (uint32_t)blocks), b64(64);
        if (seq)
            hipExtLaunchKernelGGL(kb_resolve_seq, g4, b64, 0, st, ev.start, ev.stop, 0, fd, start,
                                  n);
        else if (wide)
            hipExtLaunchKernelGGL(kb_resolve<true>, g4, b64, 0, st, ev.start, ev.stop, 0, fd,
                                  start, n);
        else
            hipExtLaunchKernelGGL(kb_resolve<false>, g4, b64, 0, st, ev.start, ev.stop, 0, fd,
                                  start, n);
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t copy_grid(uint8_t *dst, int64_t dst_pitch, const uint8_t *src, int64_t src_pitch,
                     const int32_t n[3], hipMemcpyKind kind, hipStream_t st)
{
    return hipMemcpy2DAsync(dst, (size_t)dst_pitch, src, (size_t)src_pitch, (size_t)n[0],
                            (size_t)n[1] * n[2], kind, st);
}

hipError_t copy_grid_from_ring(uint8_t *dst, const uint8_t *src, int64_t src_pitch,
                               const int32_t n[3], const int32_t ring[3], hipMemcpyKind kind,
                               hipStream_t st)
{
    // along each axis, grid coordinates [0, n - r) sit at buffer r.., and
    // [n - r, n) at buffer 0..
    for (int iz = 0; iz < 2; ++iz)
        for (int iy = 0; iy < 2; ++iy)
            for (int ix = 0; ix < 2; ++ix) {
                const int idx[3] = {ix, iy, iz};
                size_t g0[3], b0[3], len[3];
                bool empty = false;
                for (int a = 0; a < 3; ++a) {
                    const int32_t r = ring[a];
                    g0[a] = idx[a] ? (size_t)(n[a] - r) : 0;
                    b0[a] = idx[a] ? 0 : (size_t)r;
                    len[a] = idx[a] ? (size_t)r : (size_t)(n[a] - r);
                    empty = empty || len[a] == 0;
                }
                if (empty)
                    continue;
                hipMemcpy3DParms p = {};
                p.srcPtr = make_hipPitchedPtr(const_cast<uint8_t *>(src), (size_t)src_pitch,
                                              (size_t)n[0], (size_t)n[1]);
                p.srcPos = make_hipPos(b0[0], b0[1], b0[2]);
                p.dstPtr = make_hipPitchedPtr(dst, (size_t)n[0], (size_t)n[0], (size_t)n[1]);
                p.dstPos = make_hipPos(g0[0], g0[1], g0[2]);
                p.extent = make_hipExtent(len[0], len[1], len[2]);
                p.kind = kind;
                hipError_t e = hipMemcpy3DAsync(&p, st);
                if (e != hipSuccess)
                    return e;
            }
    return hipSuccess;
}

}  // namespace vg

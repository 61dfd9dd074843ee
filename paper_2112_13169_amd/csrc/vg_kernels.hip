// vg_kernels.hip -- gfx950 kernels for depth-frame -> voxel-grid generation
// (Toumieh & Lambert, arXiv 2112.13169, Sec. IV).
//
// One frame is a chain of launches on one stream:
//   k_seed        Alg. 1 lines 2-5: one lane per pixel / point: unproject,
//                 transform, quantise; stamp the point's voxel in a seed plane
//                 padded by vox_inf (byte stores of the frame's stamp: no
//                 clearing between frames, no atomics).
//   k_dilate_x    Alg. 1 lines 6-9, separably: seeds -> bits dilated by
//   k_dilate_yz   vox_inf along x, then along y and z.  The union of the
//                 (2 vox_inf + 1)^3 cubes is exactly this separable dilation.
//   k_ray_free    Alg. 2 up to the first occupied voxel: one wavefront per 8x8
//                 tile of fan targets; every voxel walked before the hit
//                 becomes free in the local grid.  Rays that hit park their
//                 walk state.  Occupancy words are fetched for 8 walk steps at
//                 a time so the loads overlap.
//   k_ray_traced  Alg. 2 after the hit: parked rays continue and mark every
//                 voxel they walk "unknown and traced" (stored as unknown).
//   k_mark_occ    the frame's occupied voxels become occupied in the grid.
// Alg. 3 (merge) needs no pass of its own: the launches write the merged
// values straight into the local grid and their order gives the merge's
// priorities (traced beats free, occupied beats both).
//
// Floating point: contraction is off (also on the command line) so every fp32
// operation rounds exactly as written; fp32 division is the correctly rounded
// one, fp32 denormals are kept.  The fixed operation orders are those of the
// transform (R p + t, left to right) and of the Amanatides & Woo walk.
#include "vg_internal.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace vg {

namespace {

constexpr int kBlock = 256;
constexpr int kChunk = 8;   // walk steps whose occupancy words load together

// ----------------------------------------------------------------- helpers

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

// Amanatides & Woo set-up on one axis.
__device__ __forceinline__ void axis_setup(float o, int32_t v0, float d, int32_t &step,
                                           float &tmax, float &tdelta)
{
    if (d > 0.0f) {
        step = 1;
        tmax = ((float)(v0 + 1) - o) / d;
        tdelta = 1.0f / d;
    } else if (d < 0.0f) {
        step = -1;
        tmax = ((float)v0 - o) / d;
        tdelta = -1.0f / d;
    } else {
        step = 0;
        tmax = __builtin_inff();
        tdelta = __builtin_inff();
    }
}

// Walk state of one ray (scalar fields: a per-axis array indexed by the
// stepping axis would be demoted to private memory).
struct Walker {
    int32_t vx, vy, vz;       // current voxel
    int32_t sx, sy, sz;       // step per axis (-1, 0, +1)
    int32_t cx, cy, cz;       // |v - v0| per axis: steps taken on that axis
    float tmx, tmy, tmz;      // ray parameter of the next boundary per axis
    float tdx, tdy, tdz;      // ray parameter per voxel per axis
    int32_t d2;               // squared lattice distance from the camera voxel
};

__device__ __forceinline__ void walker_setup(Walker &w, const float o[3], const int32_t v0[3],
                                             const float dir[3])
{
    axis_setup(o[0], v0[0], dir[0], w.sx, w.tmx, w.tdx);
    axis_setup(o[1], v0[1], dir[1], w.sy, w.tmy, w.tdy);
    axis_setup(o[2], v0[2], dir[2], w.sz, w.tmz, w.tdz);
    w.vx = v0[0];
    w.vy = v0[1];
    w.vz = v0[2];
    w.cx = w.cy = w.cz = 0;
    w.d2 = 0;
}

// One walk step: move along the axis whose boundary is nearest (ties go to
// the later axis).  Returns false when the walk cannot continue: zero
// direction, or the ray left the grid on an axis it keeps moving away on
// (the grid is convex, so it can never come back).
__device__ __forceinline__ bool walk_step(Walker &w, const int32_t n[3])
{
    const bool cxy = w.tmx < w.tmy, cxz = w.tmx < w.tmz, cyz = w.tmy < w.tmz;
    const bool ax = cxy && cxz;
    const bool ay = !cxy && cyz;
    int32_t st, va, na;
    if (ax) {
        st = w.sx;
        w.vx += st;
        w.tmx += w.tdx;
        w.d2 += 2 * w.cx + 1;
        w.cx += 1;
        va = w.vx;
        na = n[0];
    } else if (ay) {
        st = w.sy;
        w.vy += st;
        w.tmy += w.tdy;
        w.d2 += 2 * w.cy + 1;
        w.cy += 1;
        va = w.vy;
        na = n[1];
    } else {
        st = w.sz;
        w.vz += st;
        w.tmz += w.tdz;
        w.d2 += 2 * w.cz + 1;
        w.cz += 1;
        va = w.vz;
        na = n[2];
    }
    if (st == 0)
        return false;
    return !((va < 0 && st < 0) || (va >= na && st > 0));
}

__device__ __forceinline__ bool in_grid(const Walker &w, const int32_t n[3])
{
    return (uint32_t)w.vx < (uint32_t)n[0] && (uint32_t)w.vy < (uint32_t)n[1] &&
           (uint32_t)w.vz < (uint32_t)n[2];
}

// A ray that starts outside the grid and does not move towards it on that
// axis never enters.
__device__ __forceinline__ bool never_enters(const Walker &w, const int32_t n[3])
{
    return (w.vx < 0 && w.sx <= 0) || (w.vx >= n[0] && w.sx >= 0) ||
           (w.vy < 0 && w.sy <= 0) || (w.vy >= n[1] && w.sy >= 0) ||
           (w.vz < 0 && w.sz <= 0) || (w.vz >= n[2] && w.sz >= 0);
}

__device__ __forceinline__ void ray_direction(const RayParams &p, int32_t tx, int32_t ty,
                                              int32_t tz, float dir[3])
{
    float x = (float)tx, y = (float)ty, z = (float)tz;
    dir[0] = row_dot(p.R + 0, x, y, z);
    dir[1] = row_dot(p.R + 3, x, y, z);
    dir[2] = row_dot(p.R + 6, x, y, z);
}

// Bit j (j < 4) set iff byte j of w equals the byte replicated in rep.
__device__ __forceinline__ uint32_t byte_eq_mask(uint32_t w, uint32_t rep)
{
    uint32_t x = w ^ rep;                                  // zero bytes = matches
    uint32_t y = (x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
    y = ~(y | x | 0x7F7F7F7Fu);                            // 0x80 exactly in zero bytes
    uint32_t t = (y >> 7) & 0x01010101u;
    return (t * 0x01020408u) >> 24;                        // gather the four flags
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

// Alg. 1 lines 2-5.  Images: block = 64 x 4 pixels, one wavefront per image
// row segment (coalesced row reads).  Points: 256 points per block.
__global__ __launch_bounds__(kBlock) void k_seed(SeedParams p)
{
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
        *p.parked_count = 0;   // the traced pass of this frame starts empty

    float pc[3];
    if (p.kind == kPoints) {
        int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
        if (i >= p.W)
            return;
        const float *q = p.img + 3 * i;
        float x = q[0], y = q[1], z = q[2];
        if (!(__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z)))
            return;
        pc[0] = x;
        pc[1] = y;
        pc[2] = z;
    } else {
        int32_t u = blockIdx.x * 64 + (threadIdx.x & 63);
        int32_t v = blockIdx.y * 4 + (threadIdx.x >> 6);
        if (u >= p.W || v >= p.H)
            return;
        float d = p.img[(int64_t)v * p.pitch + u];
        if (!(d >= p.dmin && d <= p.dmax))
            return;
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
    int32_t pp[3];
    for (int a = 0; a < 3; ++a) {
        float pv = row_dot(p.R + 3 * a, pc[0], pc[1], pc[2]) + p.tv[a];
        float q = floorf(pv / p.s);
        // the cube cannot reach the grid: drop the point
        if (!(q >= (float)(-pl.r) && q <= (float)(pl.n[a] - 1 + pl.r)))
            return;
        pp[a] = (int32_t)q + pl.r;   // padded coordinate
    }
    pl.seed[(int64_t)pl.seed_pitch * (pp[1] + (int64_t)pl.py * pp[2]) + pp[0]] =
        (uint8_t)pl.epoch;
}

// Seeds -> bits dilated along x.  One lane per 32-voxel word of a padded row
// inside the seed box; output voxel x is set iff a seed lies at padded
// x .. x + 2r of the same padded row.
__global__ __launch_bounds__(kBlock) void k_dilate_x(Planes pl)
{
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int32_t ny = pl.hi[1] - pl.lo[1] + 1;
    const int32_t nz = pl.hi[2] - pl.lo[2] + 1;
    if (gid >= (int64_t)pl.wx * ny * nz)
        return;
    const int32_t w = (int32_t)(gid % pl.wx);
    const int64_t row = gid / pl.wx;
    const int32_t y = pl.lo[1] + (int32_t)(row % ny);
    const int32_t z = pl.lo[2] + (int32_t)(row / ny);
    const int32_t x0 = 32 * w;
    uint32_t out = 0;
    if (x0 <= pl.hi[0] && x0 + 31 + 2 * pl.r >= pl.lo[0]) {
        const uint4 *src = reinterpret_cast<const uint4 *>(
            pl.seed + (int64_t)pl.seed_pitch * (y + (int64_t)pl.py * z) + x0);
        const uint32_t rep = (pl.epoch & 0xFFu) * 0x01010101u;
        uint64_t m = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint4 q = src[k];
            uint32_t b = byte_eq_mask(q.x, rep) | (byte_eq_mask(q.y, rep) << 4) |
                         (byte_eq_mask(q.z, rep) << 8) | (byte_eq_mask(q.w, rep) << 12);
            m |= (uint64_t)b << (16 * k);
        }
        uint64_t acc = m;
        for (int d = 1; d <= 2 * pl.r; ++d)
            acc |= m >> d;
        out = (uint32_t)acc;
        const int32_t valid = pl.n[0] - x0;   // output voxels of this word inside the grid
        if (valid < 32)
            out &= (1u << valid) - 1u;
    }
    pl.bitx[(int64_t)pl.wx * (y + (int64_t)pl.py * z) + w] = out;
}

// x-dilated rows -> occupied bit plane: OR over the (2r+1) x (2r+1) padded
// rows y .. y+2r, z .. z+2r.  Every word of the plane is written.
__global__ __launch_bounds__(kBlock) void k_dilate_yz(Planes pl)
{
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gid >= (int64_t)pl.wx * pl.n[1] * pl.n[2])
        return;
    const int32_t w = (int32_t)(gid % pl.wx);
    const int64_t row = gid / pl.wx;
    const int32_t y = (int32_t)(row % pl.n[1]);
    const int32_t z = (int32_t)(row / pl.n[1]);
    const int32_t y0 = max(y, pl.lo[1]), y1 = min(y + 2 * pl.r, pl.hi[1]);
    const int32_t z0 = max(z, pl.lo[2]), z1 = min(z + 2 * pl.r, pl.hi[2]);
    uint32_t out = 0;
    for (int32_t zz = z0; zz <= z1; ++zz) {
        const uint32_t *src = pl.bitx + (int64_t)pl.wx * ((int64_t)pl.py * zz) + w;
        for (int32_t yy = y0; yy <= y1; ++yy)
            out |= src[(int64_t)pl.wx * yy];
    }
    pl.occ[gid] = out;
}

// Alg. 2 before the first occupied voxel.
__global__ __launch_bounds__(kBlock) void k_ray_free(RayParams p)
{
    const int lane = threadIdx.x & 63;
    const int32_t tile = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int32_t ta = tile % p.tiles_a, tb = tile / p.tiles_a;
    const int32_t ia = ta * 8 + (lane & 7), ib = tb * 8 + (lane >> 3);

    int32_t tx, ty, tz, m2;
    bool park = false;
    Walker w;
    if (tile < p.tiles && fan_target(p, ia, ib, tx, ty, tz, m2)) {
        float dir[3];
        ray_direction(p, tx, ty, tz, dir);
        walker_setup(w, p.o, p.v0, dir);
        bool more = !never_enters(w, p.n);
        while (more) {
            const Walker snap = w;
            uint32_t widx[kChunk], lidx[kChunk], bit[kChunk];
            bool val[kChunk];
#pragma unroll
            for (int s = 0; s < kChunk; ++s) {
                val[s] = false;
                widx[s] = lidx[s] = bit[s] = 0;
                if (more) {
                    if (w.d2 < m2 && walk_step(w, p.n)) {
                        if (in_grid(w, p.n)) {
                            val[s] = true;
                            uint32_t row = (uint32_t)w.vy + (uint32_t)p.n[1] * (uint32_t)w.vz;
                            widx[s] = ((uint32_t)w.vx >> 5) + (uint32_t)p.wx * row;
                            bit[s] = (uint32_t)w.vx & 31u;
                            lidx[s] = (uint32_t)w.vx + (uint32_t)p.n[0] * row;
                        }
                    } else {
                        more = false;
                    }
                }
            }
            uint32_t word[kChunk];
#pragma unroll
            for (int s = 0; s < kChunk; ++s)
                word[s] = val[s] ? p.occ[widx[s]] : 0u;
            int hit = kChunk;
#pragma unroll
            for (int s = kChunk - 1; s >= 0; --s)
                if ((word[s] >> bit[s]) & 1u)
                    hit = s;
#pragma unroll
            for (int s = 0; s < kChunk; ++s)
                if (val[s] && s < hit)
                    p.loc[lidx[s]] = kFree;
            if (hit < kChunk) {
                // replay the walk up to and including the hit voxel
                w = snap;
                for (int s = 0; s <= hit; ++s)
                    walk_step(w, p.n);
                park = w.d2 < m2;   // anything left to walk after the hit?
                break;
            }
        }
    }

    // Park the rays that hit: one atomic per wavefront.
    const uint64_t mask = __ballot(park);
    if (mask == 0)
        return;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader)
        base = atomicAdd(p.parked_count, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (park) {
        uint32_t slot = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        if (slot < p.parked_cap) {
            ParkedRay r;
            r.ta = ia;
            r.tb = ib;
            r.vx = w.vx;
            r.vy = w.vy;
            r.vz = w.vz;
            r.tmx = w.tmx;
            r.tmy = w.tmy;
            r.tmz = w.tmz;
            p.parked[slot] = r;
        }
    }
}

// Alg. 2 after the hit: continue each parked ray, marking "unknown and
// traced" (stored as unknown) on every voxel it walks.  Occupied voxels are
// restored by k_mark_occ afterwards, so this pass needs no loads.
__global__ __launch_bounds__(kBlock) void k_ray_traced(RayParams p)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t count = min(*p.parked_count, p.parked_cap);
    if (i >= count)
        return;
    const ParkedRay r = p.parked[i];
    int32_t tx, ty, tz, m2;
    if (!fan_target(p, r.ta, r.tb, tx, ty, tz, m2))
        return;
    float dir[3];
    ray_direction(p, tx, ty, tz, dir);
    Walker w;
    walker_setup(w, p.o, p.v0, dir);   // steps and step sizes of this ray
    w.vx = r.vx;                       // resume right after the hit voxel
    w.vy = r.vy;
    w.vz = r.vz;
    w.tmx = r.tmx;
    w.tmy = r.tmy;
    w.tmz = r.tmz;
    w.cx = abs(w.vx - p.v0[0]);
    w.cy = abs(w.vy - p.v0[1]);
    w.cz = abs(w.vz - p.v0[2]);
    w.d2 = w.cx * w.cx + w.cy * w.cy + w.cz * w.cz;
    while (w.d2 < m2) {
        if (!walk_step(w, p.n))
            break;
        if (in_grid(w, p.n))
            p.loc[(uint32_t)w.vx + (uint32_t)p.n[0] * ((uint32_t)w.vy +
                                                        (uint32_t)p.n[1] * (uint32_t)w.vz)] =
                kUnknown;
    }
}

// The frame's occupied voxels become occupied in the local grid.  One lane
// per occupancy word of the rows the seed box can reach.
__global__ __launch_bounds__(kBlock) void k_mark_occ(Planes pl, uint8_t *loc, int32_t y0,
                                                     int32_t ny, int32_t z0, int32_t nz)
{
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gid >= (int64_t)pl.wx * ny * nz)
        return;
    const int32_t w = (int32_t)(gid % pl.wx);
    const int64_t row = gid / pl.wx;
    const int32_t y = y0 + (int32_t)(row % ny);
    const int32_t z = z0 + (int32_t)(row / ny);
    const int64_t r = y + (int64_t)pl.n[1] * z;
    uint32_t m = pl.occ[(int64_t)pl.wx * r + w];
    uint8_t *dst = loc + (int64_t)pl.n[0] * r + 32 * w;
    while (m) {
        int b = __ffs(m) - 1;
        dst[b] = kOccupied;
        m &= m - 1u;
    }
}

// Sec. IV-E: dst[x,y,z] = src[x+dx, y+dy, z+dz] inside, else unknown.
__global__ __launch_bounds__(kBlock) void k_shift(const uint8_t *src, uint8_t *dst, int32_t nx,
                                                  int32_t ny, int32_t nz, int32_t dx, int32_t dy,
                                                  int32_t dz)
{
    int32_t x = blockIdx.x * kBlock + threadIdx.x;
    int32_t y = blockIdx.y, z = blockIdx.z;
    if (x >= nx)
        return;
    int64_t sx = (int64_t)x + dx, sy = (int64_t)y + dy, sz = (int64_t)z + dz;
    uint8_t val = kUnknown;
    if (sx >= 0 && sx < nx && sy >= 0 && sy < ny && sz >= 0 && sz < nz)
        val = src[(sz * ny + sy) * nx + sx];
    dst[((int64_t)z * ny + y) * nx + x] = val;
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

hipError_t launch_seeds(const SeedParams &p, hipStream_t st)
{
    dim3 grid;
    if (p.kind == kPoints)
        grid = dim3(std::max<uint32_t>(blocks_for(p.W), 1u), 1);
    else
        grid = dim3((uint32_t)std::max((p.W + 63) / 64, 1), (uint32_t)std::max((p.H + 3) / 4, 1));
    hipLaunchKernelGGL(k_seed, grid, dim3(kBlock), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_dilate(const Planes &pl, hipStream_t st)
{
    const bool any = pl.lo[0] <= pl.hi[0] && pl.lo[1] <= pl.hi[1] && pl.lo[2] <= pl.hi[2];
    if (any) {
        int64_t n = (int64_t)pl.wx * (pl.hi[1] - pl.lo[1] + 1) * (pl.hi[2] - pl.lo[2] + 1);
        hipLaunchKernelGGL(k_dilate_x, dim3(blocks_for(n)), dim3(kBlock), 0, st, pl);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    int64_t n = (int64_t)pl.wx * pl.n[1] * pl.n[2];
    hipLaunchKernelGGL(k_dilate_yz, dim3(blocks_for(n)), dim3(kBlock), 0, st, pl);
    return hipGetLastError();
}

hipError_t launch_rays(const RayParams &p, hipStream_t st, hipEvent_t mid)
{
    const int waves = kBlock / 64;
    uint32_t blocks = (uint32_t)((p.tiles + waves - 1) / waves);
    if (blocks == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_ray_free, dim3(blocks), dim3(kBlock), 0, st, p);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && mid)
        e = hipEventRecord(mid, st);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_ray_traced, dim3(blocks_for((int64_t)p.tiles * 64)), dim3(kBlock), 0,
                       st, p);
    return hipGetLastError();
}

hipError_t launch_mark_occupied(const Planes &pl, uint8_t *loc, hipStream_t st)
{
    // output rows y with a seed row in y .. y + 2r inside the box
    const int32_t y0 = std::max(pl.lo[1] - 2 * pl.r, 0), y1 = std::min(pl.hi[1], pl.n[1] - 1);
    const int32_t z0 = std::max(pl.lo[2] - 2 * pl.r, 0), z1 = std::min(pl.hi[2], pl.n[2] - 1);
    if (pl.lo[0] > pl.hi[0] || y0 > y1 || z0 > z1)
        return hipSuccess;
    int64_t n = (int64_t)pl.wx * (y1 - y0 + 1) * (z1 - z0 + 1);
    hipLaunchKernelGGL(k_mark_occ, dim3(blocks_for(n)), dim3(kBlock), 0, st, pl, loc, y0,
                       y1 - y0 + 1, z0, z1 - z0 + 1);
    return hipGetLastError();
}

hipError_t launch_shift(const uint8_t *src, uint8_t *dst, const int32_t n[3], const int32_t d[3],
                        hipStream_t st)
{
    dim3 grid((uint32_t)((n[0] + kBlock - 1) / kBlock), (uint32_t)n[1], (uint32_t)n[2]);
    hipLaunchKernelGGL(k_shift, grid, dim3(kBlock), 0, st, src, dst, n[0], n[1], n[2], d[0], d[1],
                       d[2]);
    return hipGetLastError();
}

}  // namespace vg

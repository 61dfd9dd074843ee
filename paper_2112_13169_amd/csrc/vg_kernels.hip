// vg_kernels.hip -- gfx950 kernels for depth-frame -> voxel-grid generation
// (Toumieh & Lambert, arXiv 2112.13169, Sec. IV).
//
// Frame = three launches on one stream:
//   k_occupied  Alg. 1: one lane per pixel / point: unproject, transform,
//               quantise, mark the vox_inf cube occupied in the local grid and
//               stamp it in the per-frame occupancy plane.
//   k_ray_free  Alg. 2 up to the first occupied voxel: one wavefront per 8x8
//               tile of fan targets; every voxel walked before the hit becomes
//               free in the local grid.  Rays that hit park their walk state.
//   k_ray_traced Alg. 2 after the hit: parked rays continue; the voxels they
//               walk ("unknown and traced") become unknown in the local grid.
// Alg. 3 (merge) needs no pass of its own: the three launches write the merged
// values straight into the local grid, and their stream order gives the
// merge's priorities (traced beats free; rays never touch occupied voxels).
// All stores are idempotent byte stores; no atomics on voxels.
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

__device__ __forceinline__ bool in_grid(const Walker &w, const int32_t n[3], int64_t &idx)
{
    if ((uint32_t)w.vx >= (uint32_t)n[0] || (uint32_t)w.vy >= (uint32_t)n[1] ||
        (uint32_t)w.vz >= (uint32_t)n[2])
        return false;
    idx = (int64_t)w.vx + (int64_t)n[0] * ((int64_t)w.vy + (int64_t)n[1] * w.vz);
    return true;
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

// Alg. 1.  Images: block = 64 x 4 pixels, one wavefront per image row
// segment (coalesced row reads).  Points: 256 points per block.
__global__ __launch_bounds__(kBlock) void k_occupied(OccParams p)
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

    int32_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        float pv = row_dot(p.R + 3 * a, pc[0], pc[1], pc[2]) + p.tv[a];
        float q = floorf(pv / p.s);
        if (!(q >= (float)(-p.r) && q <= (float)(p.n[a] - 1 + p.r)))
            return;   // the cube cannot reach the grid
        int32_t qi = (int32_t)q;
        lo[a] = max(qi - p.r, 0);
        hi[a] = min(qi + p.r, p.n[a] - 1);
    }
    const uint8_t stamp = (uint8_t)p.epoch;
    for (int32_t z = lo[2]; z <= hi[2]; ++z)
        for (int32_t y = lo[1]; y <= hi[1]; ++y) {
            int64_t row = ((int64_t)z * p.n[1] + y) * p.n[0];
            for (int32_t x = lo[0]; x <= hi[0]; ++x) {
                p.occ[row + x] = stamp;
                p.loc[row + x] = kOccupied;
            }
        }
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
        if (!never_enters(w, p.n)) {
            const uint8_t stamp = (uint8_t)p.epoch;
            while (w.d2 < m2) {
                if (!walk_step(w, p.n))
                    break;
                int64_t idx;
                if (in_grid(w, p.n, idx)) {
                    if (p.occ[idx] == stamp) {
                        park = w.d2 < m2;   // anything left to walk after the hit?
                        break;
                    }
                    p.loc[idx] = kFree;
                }
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
// traced" (stored as unknown) on every non-occupied voxel it walks.
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
    const uint8_t stamp = (uint8_t)p.epoch;
    while (w.d2 < m2) {
        if (!walk_step(w, p.n))
            break;
        int64_t idx;
        if (in_grid(w, p.n, idx) && p.occ[idx] != stamp)
            p.loc[idx] = kUnknown;
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

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_fill(void *dst, uint8_t value, size_t bytes, hipStream_t st)
{
    if (bytes == 0)
        return hipSuccess;
    uintptr_t base = (uintptr_t)dst & ~(uintptr_t)15;
    size_t chunks = ((uintptr_t)dst + bytes - base + 15) / 16;
    size_t blocks = (chunks + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_fill, dim3((uint32_t)blocks), dim3(kBlock), 0, st, (uint8_t *)dst, value,
                       bytes);
    return hipGetLastError();
}

hipError_t launch_occupied(const OccParams &p, hipStream_t st)
{
    dim3 grid;
    if (p.kind == kPoints)
        grid = dim3((uint32_t)std::max<int64_t>(((int64_t)p.W + kBlock - 1) / kBlock, 1), 1);
    else
        grid = dim3((uint32_t)std::max((p.W + 63) / 64, 1), (uint32_t)std::max((p.H + 3) / 4, 1));
    hipLaunchKernelGGL(k_occupied, grid, dim3(kBlock), 0, st, p);
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
    uint32_t tblocks = (uint32_t)(((uint64_t)p.tiles * 64 + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_ray_traced, dim3(tblocks), dim3(kBlock), 0, st, p);
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

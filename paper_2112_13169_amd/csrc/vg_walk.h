// vg_walk.h -- the ray walk of Alg. 2 (Toumieh & Lambert, arXiv 2112.13169,
// Sec. IV-C): Amanatides & Woo traversal from the camera voxel, termination
// at the target's length, free / traced marking around the first occupied
// voxel.  Used by the k_rays kernel; plain C++ without HIP so that the same
// code can also be compiled for the host (VG_HD expands accordingly).
#pragma once

#include <stdint.h>

#ifdef __HIPCC__
#define VG_HD __device__ __forceinline__
#define VG_INF __builtin_inff()
#define vg_any(p) __any(p)
#else
#include <cmath>
#define VG_HD static inline
#define VG_INF INFINITY
#define vg_any(p) (p)   // host build: one lane per "wavefront"
#endif

namespace vg {

constexpr int kChunk = 8;   // walk steps whose occupancy words load together
constexpr uint8_t kWalkFree = 1;   // local-grid value of a free voxel

// Per-frame constants of the walk.
struct WalkFrame {
    float o[3];       // camera position in voxel units
    int32_t v0[3];    // camera voxel
    int32_t n[3];     // grid size
    int32_t gxp;      // device-layout row pitch
};

VG_HD int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }
VG_HD float fmin3(float a, float b, float c) { return fminf(fminf(a, b), c); }

// Amanatides & Woo set-up on one axis.
VG_HD void axis_setup(float o, int32_t v0, float d, int32_t &step, float &tmax, float &tdelta)
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
        tmax = VG_INF;
        tdelta = VG_INF;
    }
}

// Walk state of one ray.  Scalar fields and value selects: an array indexed
// by the stepping axis would be demoted to private memory, and a conditional
// over lvalues selects an address (also forcing memory).  Steps taken on an
// axis are kept as q = 2 * steps + 1, so that the squared lattice distance
// grows by q at each step on that axis.
struct Walk {
    float tmx, tmy, tmz;      // ray parameter of the next boundary per axis
    float tdx, tdy, tdz;      // ray parameter per voxel per axis
    int32_t qx, qy, qz;       // 2 * (steps on the axis) + 1
    int32_t lx, ly, lz;       // q must stay below this: 2 * (steps until outside) - 1
    int32_t ex, ey, ez;       // q from which the ray is inside: 2 * (steps until inside) + 1
    int32_t sx, sy, sz;       // index stride of one step on each axis
    int32_t d2;               // squared lattice distance from the camera voxel
    uint32_t idx;             // device-layout index of the current voxel (mod 2^32)
};

// Steps along one axis before the walk leaves the grid (0 for an axis the
// ray does not move on: choosing it ends the walk) and before it enters.
VG_HD void axis_limits(int32_t step, int32_t v0, int32_t n, int32_t &leave, int32_t &enter)
{
    leave = step > 0 ? n - v0 : (step < 0 ? v0 + 1 : 0);
    enter = step > 0 ? imax(-v0, 0) : (step < 0 ? imax(v0 - n + 1, 0) : 0);
}

VG_HD void walk_setup(Walk &w, const WalkFrame &p, const float dir[3])
{
    int32_t sx, sy, sz, lx, ly, lz, ex, ey, ez;
    axis_setup(p.o[0], p.v0[0], dir[0], sx, w.tmx, w.tdx);
    axis_setup(p.o[1], p.v0[1], dir[1], sy, w.tmy, w.tdy);
    axis_setup(p.o[2], p.v0[2], dir[2], sz, w.tmz, w.tdz);
    axis_limits(sx, p.v0[0], p.n[0], lx, ex);
    axis_limits(sy, p.v0[1], p.n[1], ly, ey);
    axis_limits(sz, p.v0[2], p.n[2], lz, ez);
    w.lx = 2 * lx - 1;
    w.ly = 2 * ly - 1;
    w.lz = 2 * lz - 1;
    w.ex = 2 * ex + 1;
    w.ey = 2 * ey + 1;
    w.ez = 2 * ez + 1;
    w.sx = sx;
    w.sy = sy * p.gxp;
    w.sz = sz * p.gxp * p.n[1];
    w.qx = w.qy = w.qz = 1;
    w.d2 = 0;
    w.idx = (uint32_t)((int64_t)p.v0[0] + (int64_t)p.gxp * (p.v0[1] + (int64_t)p.n[1] * p.v0[2]));
}

// An axis on which the camera lies outside the grid and the ray does not
// move towards it: such a ray never enters the grid.
VG_HD bool axis_dead(int32_t step, int32_t v0, int32_t n)
{
    const bool outside = v0 < 0 || v0 >= n;
    const bool towards = (step > 0 && v0 < 0) || (step < 0 && v0 >= n);
    return outside && !towards;
}

VG_HD int32_t sgn(float d) { return d > 0.0f ? 1 : (d < 0.0f ? -1 : 0); }

// Value selects (see Walk).
VG_HD int32_t sel(bool c, int32_t a, int32_t b) { return c ? a : b; }
VG_HD float self(bool c, float a, float b) { return c ? a : b; }

// One step of Alg. 2: move along the axis whose next boundary is nearest
// (ties go to the later axis).  Returns false when the walk is over: its
// length is reached, the direction is zero, or the ray left the grid on an
// axis it keeps moving away on (the grid is convex: it cannot return).  The
// state moves on even then -- a finished walk is never read again -- so the
// step has no branches.  kGeneral: the camera may be outside the grid, and
// `in` reports whether the new voxel lies in it; otherwise every voxel of a
// live walk does.
template <bool kGeneral>
VG_HD bool walk_step(Walk &w, int32_t m2, bool live, bool &in)
{
    const float tmx = w.tmx, tmy = w.tmy, tmz = w.tmz;
    // tMx<tMy ? (tMx<tMz ? x : z) : (tMy<tMz ? y : z) == "z if tMz is a
    // minimum, else y if tMy is, else x" (the boundary parameters are never NaN)
    const float mn = fmin3(tmx, tmy, tmz);
    const bool az = tmz == mn;
    const bool ayr = tmy == mn;
    const int32_t q = sel(az, w.qz, sel(ayr, w.qy, w.qx));
    const int32_t lim = sel(az, w.lz, sel(ayr, w.ly, w.lx));
    const int32_t stride = sel(az, w.sz, sel(ayr, w.sy, w.sx));
    const bool go = live && w.d2 < m2 && q < lim;
    const bool ay = !az && ayr, ax = !az && !ayr;
    w.tmx = self(ax, tmx + w.tdx, tmx);
    w.tmy = self(ay, tmy + w.tdy, tmy);
    w.tmz = self(az, tmz + w.tdz, tmz);
    w.qx = sel(ax, q + 2, w.qx);
    w.qy = sel(ay, q + 2, w.qy);
    w.qz = sel(az, q + 2, w.qz);
    w.d2 += q;
    w.idx += (uint32_t)stride;
    if (kGeneral)
        in = w.qx >= w.ex && w.qy >= w.ey && w.qz >= w.ez;
    return go;
}

// The walk runs in chunks of kChunk steps, two chunks in flight: the
// occupancy words of one chunk load while the previous chunk is resolved.
// Every chunk issues exactly kChunk loads (word 0 where none is needed) so
// that the wait for a chunk's words never has to cover the next chunk's loads.
struct Chunk {
    uint32_t ids[kChunk];     // device-layout index of each step's voxel
    uint32_t words[kChunk];   // occupancy word of that voxel (garbage when not needed)
    uint32_t valid;           // bit s: step s was taken and its voxel is in the grid
};

template <bool kGeneral>
VG_HD bool walk_chunk(Walk &w, int32_t m2, bool alive, Chunk &c, bool load,
                                           const uint32_t *occ)
{
    c.valid = 0;
#pragma unroll
    for (int s = 0; s < kChunk; ++s) {
        bool in = true;
        alive = walk_step<kGeneral>(w, m2, alive, in);
        c.ids[s] = w.idx;
        c.valid |= (alive && in) ? (1u << s) : 0u;
    }
    // a wavefront whose rays have all met their obstacle loads nothing
    if (vg_any(load)) {
#pragma unroll
        for (int s = 0; s < kChunk; ++s) {
            const bool need = load && ((c.valid >> s) & 1u);
            c.words[s] = occ[need ? c.ids[s] >> 5 : 0u];
        }
    } else {
#pragma unroll
        for (int s = 0; s < kChunk; ++s)
            c.words[s] = 0u;
    }
    return alive;
}

// Marks of one chunk: free before the ray's first occupied voxel, traced
// after it, nothing on it.  Returns whether the chunk held the hit.
VG_HD bool resolve_chunk(const Chunk &c, bool before_hit, uint8_t *loc,
                                              uint8_t *traced, uint8_t stamp)
{
    int hit = kChunk;
    if (before_hit) {
#pragma unroll
        for (int s = kChunk - 1; s >= 0; --s)
            if (((c.valid >> s) & 1u) && ((c.words[s] >> (c.ids[s] & 31u)) & 1u))
                hit = s;
    }
#pragma unroll
    for (int s = 0; s < kChunk; ++s) {
        if (!((c.valid >> s) & 1u))
            continue;
        if (before_hit && s < hit)
            loc[c.ids[s]] = kWalkFree;
        else if (s != hit)
            traced[c.ids[s]] = stamp;
    }
    return hit < kChunk;
}

// Alg. 2 for one ray: walk, test occupancy before the first hit, mark free
// before it and "unknown and traced" after it.
template <bool kGeneral>
VG_HD void walk_ray(Walk &w, int32_t m2, const uint32_t *occ, uint8_t *loc, uint8_t *traced,
                    uint8_t stamp)
{
    bool before_hit = true;   // Alg. 2: vox_val is still "free"
    Chunk a, b;
    bool alive = walk_chunk<kGeneral>(w, m2, true, a, true, occ);
    while (true) {
        bool more = alive;
        alive = walk_chunk<kGeneral>(w, m2, alive, b, before_hit, occ);
        if (resolve_chunk(a, before_hit, loc, traced, stamp))
            before_hit = false;
        if (!more && b.valid == 0)
            break;
        more = alive;
        alive = walk_chunk<kGeneral>(w, m2, alive, a, before_hit, occ);
        if (resolve_chunk(b, before_hit, loc, traced, stamp))
            before_hit = false;
        if (!more && a.valid == 0)
            break;
    }
}

}  // namespace vg

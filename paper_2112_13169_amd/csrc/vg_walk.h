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
#define vg_all(p) __all(p)
#else
#include <cmath>
#define VG_HD static inline
#define VG_INF INFINITY
#define vg_any(p) (p)   // host build: one lane per "wavefront"
#define vg_all(p) (p)
#endif

namespace vg {

constexpr int kChunk = 8;   // walk steps whose occupancy words load together

// Memory the walk touches: the frame's occupancy bits (32-bit words) and its
// mark planes -- byte stamps, free marks at [0, n) and "unknown and traced"
// marks at [n, 2n), both indexed like the device-layout grid.  Offsets at or
// beyond a buffer's size read 0 and write nothing (on the device these are
// buffer-resource range checks, so masked lanes need no branches).
constexpr uint32_t kOob = 0x80000000u;

#ifdef __HIPCC__
struct WalkMem {
    __amdgpu_buffer_rsrc_t occ, marks;
    uint32_t n;        // bytes per mark plane
    uint32_t stamp;    // the frame's stamp
};

// raw buffer descriptor, word 3 of the gfx9 family (no swizzle, no format)
VG_HD __amdgpu_buffer_rsrc_t buffer_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000);
}

VG_HD WalkMem walk_mem(const uint32_t *occ, uint32_t occ_bytes, uint8_t *marks, uint32_t n,
                       uint32_t stamp)
{
    WalkMem m;
    m.occ = buffer_rsrc(occ, occ_bytes);
    m.marks = buffer_rsrc(marks, 2 * n);
    m.n = n;
    m.stamp = stamp;
    return m;
}

VG_HD uint32_t load_occ(const WalkMem &m, uint32_t byte_off)
{
    return __builtin_amdgcn_raw_buffer_load_b32(m.occ, (int)byte_off, 0, 0);
}

VG_HD void store_mark(const WalkMem &m, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b8((unsigned char)m.stamp, m.marks, (int)off, 0, 0);
}
#else
struct WalkMem {
    const uint32_t *occ;
    uint32_t occ_bytes;
    uint8_t *marks;
    uint32_t n;
    uint32_t stamp;
};

VG_HD WalkMem walk_mem(const uint32_t *occ, uint32_t occ_bytes, uint8_t *marks, uint32_t n,
                       uint32_t stamp)
{
    return WalkMem{occ, occ_bytes, marks, n, stamp};
}

VG_HD uint32_t load_occ(const WalkMem &m, uint32_t byte_off)
{
    return byte_off + 4 <= m.occ_bytes ? m.occ[byte_off / 4] : 0u;
}

VG_HD void store_mark(const WalkMem &m, uint32_t off)
{
    if (off < 2 * m.n)
        m.marks[off] = (uint8_t)m.stamp;
}
#endif

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

// Move one voxel along the axis whose next boundary is nearest (ties go to
// the later axis): its boundary parameter advances by its per-voxel
// increment, its step count by one, the squared lattice distance by the old
// q of that axis and the index by that axis' stride.  Returns the old q and
// the axis' limit (a step with q >= limit leaves the grid).
VG_HD void advance(Walk &w, int32_t &q, int32_t &lim)
{
    const float tmx = w.tmx, tmy = w.tmy, tmz = w.tmz;
    // tMx<tMy ? (tMx<tMz ? x : z) : (tMy<tMz ? y : z) == "z if tMz is a
    // minimum, else y if tMy is, else x" (the boundary parameters are never NaN)
    const float mn = fmin3(tmx, tmy, tmz);
    const bool az = tmz == mn;
    const bool ayr = tmy == mn;
    q = sel(az, w.qz, sel(ayr, w.qy, w.qx));
    lim = sel(az, w.lz, sel(ayr, w.ly, w.lx));
    const int32_t stride = sel(az, w.sz, sel(ayr, w.sy, w.sx));
    const bool ay = !az && ayr, ax = !az && !ayr;
    w.tmx = self(ax, tmx + w.tdx, tmx);
    w.tmy = self(ay, tmy + w.tdy, tmy);
    w.tmz = self(az, tmz + w.tdz, tmz);
    w.qx = sel(ax, q + 2, w.qx);
    w.qy = sel(ay, q + 2, w.qy);
    w.qz = sel(az, q + 2, w.qz);
    w.d2 += q;
    w.idx += (uint32_t)stride;
}

// One step of Alg. 2.  Returns false when the walk is over: its length is
// reached, the direction is zero, or the ray left the grid on an axis it
// keeps moving away on (the grid is convex: it cannot return).  The state
// moves on even then -- a finished walk is never read again -- so the step
// has no branches.  kGeneral: the camera may be outside the grid, and `in`
// reports whether the new voxel lies in it; otherwise every voxel of a live
// walk does.
template <bool kGeneral>
VG_HD bool walk_step(Walk &w, int32_t m2, bool live, bool &in)
{
    const bool near = w.d2 < m2;
    int32_t q, lim;
    advance(w, q, lim);
    if (kGeneral)
        in = w.qx >= w.ex && w.qy >= w.ey && w.qz >= w.ez;
    return live && near && q < lim;
}

// Bit `i mod 32` of an occupancy word.
VG_HD uint32_t bit_of(uint32_t word, uint32_t i)
{
#ifdef __HIPCC__
    return __builtin_amdgcn_ubfe(word, i, 1u);
#else
    return (word >> (i & 31u)) & 1u;
#endif
}

// Index of the lowest set bit of a non-zero word.
VG_HD int lowest_set(uint32_t v)
{
    return __builtin_ctz(v);
}

// The walk runs in chunks of kChunk steps, two chunks in flight: the
// occupancy words of one chunk load while the previous chunk is resolved.
// A step that was not taken, or whose voxel is outside the grid, has index
// kOob: its load reads 0 and its mark store writes nothing (kOob is at least
// twice any plane size, so kOob + n stays out of range too).
struct Chunk {
    uint32_t ids[kChunk];     // device-layout index of each step's voxel, or kOob
    uint32_t words[kChunk];   // occupancy word of that voxel (0 when not loaded)
};

// A live walk whose next kChunk steps can neither reach its length nor leave
// the grid: every axis has room for kChunk more steps (an axis the ray does
// not move on has none, so such rays never qualify) and the distance stays
// below the length even if every step is taken on the axis with the largest q.
VG_HD bool chunk_safe(const Walk &w, int32_t m2)
{
    constexpr int32_t room = 2 * (kChunk - 1);
    const int32_t qm = imax(w.qx, imax(w.qy, w.qz));
    return w.qx + room < w.lx && w.qy + room < w.ly && w.qz + room < w.lz &&
           w.d2 + (kChunk - 1) * qm + (kChunk - 1) * (kChunk - 2) < m2;
}

template <bool kGeneral>
VG_HD bool walk_chunk(Walk &w, int32_t m2, bool alive, Chunk &c, bool load, const WalkMem &m)
{
    if (!kGeneral && vg_all(!alive || chunk_safe(w, m2))) {
        // No step of this chunk can end a walk, so the steps skip the tests
        // and the bookkeeping of q and the distance: the steps per axis are
        // counted in one word (10 bits each) and applied at the end.  The
        // boundary parameters and the index move exactly as in advance().
        uint32_t cnt = 0;
#pragma unroll
        for (int s = 0; s < kChunk; ++s) {
            const float tmx = w.tmx, tmy = w.tmy, tmz = w.tmz;
            const float mn = fmin3(tmx, tmy, tmz);
            const bool az = tmz == mn;
            const bool ayr = tmy == mn;
            const bool ay = !az && ayr, ax = !az && !ayr;
            w.tmx = self(ax, tmx + w.tdx, tmx);
            w.tmy = self(ay, tmy + w.tdy, tmy);
            w.tmz = self(az, tmz + w.tdz, tmz);
            cnt += (uint32_t)sel(az, 1 << 20, sel(ayr, 1 << 10, 1));
            w.idx += (uint32_t)sel(az, w.sz, sel(ayr, w.sy, w.sx));
            c.ids[s] = alive ? w.idx : kOob;
        }
        // c steps on an axis whose q was q0 add q0 + (q0+2) + ... = c (q0 + c - 1)
        const int32_t cx = (int32_t)(cnt & 1023u), cy = (int32_t)((cnt >> 10) & 1023u);
        const int32_t cz = (int32_t)(cnt >> 20);
        w.d2 += cx * (w.qx + cx - 1) + cy * (w.qy + cy - 1) + cz * (w.qz + cz - 1);
        w.qx += 2 * cx;
        w.qy += 2 * cy;
        w.qz += 2 * cz;
    } else {
#pragma unroll
        for (int s = 0; s < kChunk; ++s) {
            bool in = true;
            alive = walk_step<kGeneral>(w, m2, alive, in);
            c.ids[s] = (alive && in) ? w.idx : kOob;
        }
    }
    // a wavefront whose rays have all met their obstacle loads nothing.  For
    // kOob the word's byte offset is 2^28, beyond any occupancy plane (grids
    // hold fewer than 2^30 voxels): a step outside the grid reads 0.
    if (vg_any(load)) {
#pragma unroll
        for (int s = 0; s < kChunk; ++s)
            c.words[s] = load_occ(m, load ? (c.ids[s] >> 5) << 2 : kOob);
    } else {
#pragma unroll
        for (int s = 0; s < kChunk; ++s)
            c.words[s] = 0u;
    }
    return alive;
}

// Marks of one chunk: free before the ray's first occupied voxel, traced from
// it on (the occupied voxel itself becomes occupied whatever its marks say).
// Returns whether the chunk held the hit.
VG_HD bool resolve_chunk(const Chunk &c, bool before_hit, const WalkMem &m)
{
    // occupied bits of the chunk's voxels as a mask (words of steps not taken
    // are 0); the hit is its lowest set bit.  Steps before `hit` are free:
    // none once the ray has hit (hit = 0), all of them if this chunk has no
    // occupied voxel (hit = kChunk).
    uint32_t hits = 1u;
    if (before_hit) {
        hits = 1u << kChunk;
#pragma unroll
        for (int s = 0; s < kChunk; ++s)
            hits |= bit_of(c.words[s], c.ids[s]) << s;
    }
    const int hit = lowest_set(hits);
#pragma unroll
    for (int s = 0; s < kChunk; ++s)
        store_mark(m, c.ids[s] + (s < hit ? 0u : m.n));
    return before_hit && hit < kChunk;
}

// Alg. 2 for one ray: walk, test occupancy before the first hit, mark free
// before it and "unknown and traced" from it on.  A chunk walked after the
// walk ended holds no step, so the loop ends once the chunk that ended it is
// resolved.
template <bool kGeneral>
VG_HD void walk_ray(Walk &w, int32_t m2, const WalkMem &m)
{
    bool before_hit = true;   // Alg. 2: vox_val is still "free"
    Chunk a, b;
    bool alive = walk_chunk<kGeneral>(w, m2, true, a, true, m);
    while (true) {
        bool more = alive;
        alive = walk_chunk<kGeneral>(w, m2, alive, b, before_hit, m);
        if (resolve_chunk(a, before_hit, m))
            before_hit = false;
        if (!more)
            break;
        more = alive;
        alive = walk_chunk<kGeneral>(w, m2, alive, a, before_hit, m);
        if (resolve_chunk(b, before_hit, m))
            before_hit = false;
        if (!more)
            break;
    }
}

}  // namespace vg

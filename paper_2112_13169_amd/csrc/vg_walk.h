// vg_walk.h -- the ray walk of Alg. 2 (Toumieh & Lambert, arXiv 2112.13169,
// Sec. IV-C): Amanatides & Woo traversal from the camera voxel, termination
// at the target's length, free / traced marking around the first occupied
// voxel.  Used by the walk kernels; plain C++ without HIP so that the same
// code can also be compiled for the host (VG_HD expands accordingly).
#pragma once

#include <stdint.h>

#ifdef __HIPCC__
#define VG_HD __device__ __forceinline__
#define VG_INF __builtin_inff()
#define vg_any(p) __any(p)
#define vg_all(p) __all(p)
// a vote the compiler can see is the same on every lane
#define vg_any_u(p) (__builtin_amdgcn_readfirstlane(__any(p)) != 0)
#else
#include <cmath>
#define VG_HD static inline
#define VG_INF INFINITY
// Host build: one lane per "wavefront".  A test can stand in for the other
// lanes of a wavefront with vg_host_vote: each call returns whether some
// other lane votes the other way (so a wavefront vote can be true although
// this lane's predicate is false, for any, or false although it is true, for
// all).  The walk's results must not depend on it.
inline bool (*vg_host_vote)() = nullptr;
#define vg_any(p) ((p) || (vg_host_vote && vg_host_vote()))
#define vg_all(p) ((p) && !(vg_host_vote && vg_host_vote()))
#define vg_any_u(p) vg_any(p)
#endif

namespace vg {

constexpr int kChunk = 8;   // walk steps whose occupancy words load together
constexpr int32_t kNoLimit = 0x3FFFFFFF;   // a q limit no walk reaches

// Memory the walk touches: the frame's occupancy -- bits (32-bit words), or
// byte stamps (one per device-layout voxel) for frames whose occupied cubes
// were stamped directly -- and its mark planes -- byte stamps, free marks at
// [0, n) and "unknown and traced" marks at [n, 2n), both indexed like the
// device-layout grid.  Offsets at or beyond a buffer's size read 0 and write
// nothing (on the device these are buffer-resource range checks, so masked
// lanes need no branches).
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

VG_HD WalkMem walk_mem(const void *occ, uint32_t occ_bytes, uint8_t *marks, uint32_t n,
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

VG_HD uint32_t load_occ_byte(const WalkMem &m, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b8(m.occ, (int)off, 0, 0);
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

VG_HD WalkMem walk_mem(const void *occ, uint32_t occ_bytes, uint8_t *marks, uint32_t n,
                       uint32_t stamp)
{
    return WalkMem{static_cast<const uint32_t *>(occ), occ_bytes, marks, n, stamp};
}

VG_HD uint32_t load_occ(const WalkMem &m, uint32_t byte_off)
{
    return byte_off + 4 <= m.occ_bytes ? m.occ[byte_off / 4] : 0u;
}

VG_HD uint32_t load_occ_byte(const WalkMem &m, uint32_t off)
{
    return off < m.occ_bytes ? reinterpret_cast<const uint8_t *>(m.occ)[off] : 0u;
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
    // An axis the ray does not move on is never chosen while another one
    // moves (its boundary parameter is infinite): give it a limit no walk
    // reaches, so that chunks of such a ray may skip the tests.  A ray that
    // moves on no axis keeps the limit that ends its walk at once.
    const bool moves = sx != 0 || sy != 0 || sz != 0;
    w.lx = sx == 0 && moves ? kNoLimit : 2 * lx - 1;
    w.ly = sy == 0 && moves ? kNoLimit : 2 * ly - 1;
    w.lz = sz == 0 && moves ? kNoLimit : 2 * lz - 1;
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

// The axis of the next step: the one whose boundary parameter is smallest,
// ties going to the later axis -- tMx<tMy ? (tMx<tMz ? x : z) : (tMy<tMz ?
// y : z) -- as three compares: z if tMz <= tMy and tMz <= tMx, else y if
// tMy <= tMx, else x (the boundary parameters are never NaN).
VG_HD void pick_axis(float tmx, float tmy, float tmz, bool &ax, bool &ay, bool &az)
{
    const bool zy = tmz <= tmy, zx = tmz <= tmx, yx = tmy <= tmx;
    az = zy && zx;
    ay = !az && yx;
    ax = !az && !yx;
}

// Move one voxel along the axis whose next boundary is nearest: its boundary
// parameter advances by its per-voxel increment, its step count by one, the
// squared lattice distance by the old q of that axis and the index by that
// axis' stride.  Returns the old q and the axis' limit (a step with q >=
// limit leaves the grid).
VG_HD void advance(Walk &w, int32_t &q, int32_t &lim)
{
    const float tmx = w.tmx, tmy = w.tmy, tmz = w.tmz;
    bool ax, ay, az;
    pick_axis(tmx, tmy, tmz, ax, ay, az);
    q = sel(az, w.qz, sel(ay, w.qy, w.qx));
    lim = sel(az, w.lz, sel(ay, w.ly, w.lx));
    const int32_t stride = sel(az, w.sz, sel(ay, w.sy, w.sx));
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

// a * b for a, b < 2^24 and a product below 2^32 (one full-rate multiply on
// the device).
VG_HD uint32_t mul24(uint32_t a, uint32_t b)
{
#ifdef __HIPCC__
    return __umul24(a, b);
#else
    return a * b;
#endif
}

// The walk runs in chunks of kChunk steps, two chunks in flight: the
// occupancy words of one chunk load while the previous chunk is resolved.
//
// Indices: a walk's index runs over the free mark plane until the ray meets
// its first occupied voxel, over the traced plane from then on (it moves up
// by n there), and is kOob once the walk is over (its strides become 0, so it
// stays kOob).  A step that was not taken, or whose voxel is outside the
// grid, has index kOob.  Loads at traced-plane indices or at kOob fall beyond
// the occupancy plane and read 0 (the word of index i is at byte
// (i >> 5) << 2, at least n / 8 for i >= n, and 2^28 for kOob; with kBytes
// the stamp of index i is at byte i, at least n); stores at kOob or kOob + n
// write nothing (kOob is at least twice any plane size).  So a ray after its
// hit needs no test for its loads or for the plane of its marks.  A stamp
// byte of a voxel stamped in an earlier frame holds that frame's number,
// never this frame's (the numbers only grow until the planes are cleared).
struct Chunk {
    uint32_t ids[kChunk];     // index of each step's voxel, or kOob
    uint32_t words[kChunk];   // occupancy word (kBytes: stamp byte) of that voxel, 0 when not loaded
    bool loaded;              // some lane of the wavefront loaded words
};

// A live walk whose next kChunk steps can neither reach its length nor leave
// the grid: every axis has room for kChunk more steps (an axis the ray does
// not move on always has) and the distance stays below the length even if
// every step is taken on the axis with the largest q.
VG_HD bool chunk_safe(const Walk &w, int32_t m2)
{
    constexpr int32_t room = 2 * (kChunk - 1);
    // q = 2 * steps + 1 < 2^20 (a wavefront's walks end within 3 * 65535
    // steps, a finished walk's q moving with the live ones' chunks): the
    // full-rate 24-bit multiply is exact
    const int32_t qm = imax(w.qx, imax(w.qy, w.qz));
    return w.qx + room < w.lx && w.qy + room < w.ly && w.qz + room < w.lz &&
           w.d2 + (int32_t)mul24((uint32_t)qm, kChunk - 1) + (kChunk - 1) * (kChunk - 2) < m2;
}

// kLone selects the form for wavefronts that each have a SIMD to themselves
// (see walk_ray).
// kChunk steps of a walk: the index of each step's voxel into c.ids.
template <bool kGeneral>
VG_HD bool step_chunk(Walk &w, int32_t m2, bool alive, Chunk &c)
{
    if (!kGeneral && vg_all(!alive || chunk_safe(w, m2))) {
        // No step of this chunk can end a walk, so the steps skip the tests
        // and the bookkeeping of q and the distance: the steps per axis are
        // counted in one word (10 bits each) and applied at the end.  The
        // boundary parameters and the index move exactly as in advance(); a
        // finished walk's index stays kOob.
        uint32_t cnt = 0;
#pragma unroll
        for (int s = 0; s < kChunk; ++s) {
            const float tmx = w.tmx, tmy = w.tmy, tmz = w.tmz;
            bool ax, ay, az;
            pick_axis(tmx, tmy, tmz, ax, ay, az);
            w.tmx = self(ax, tmx + w.tdx, tmx);
            w.tmy = self(ay, tmy + w.tdy, tmy);
            w.tmz = self(az, tmz + w.tdz, tmz);
            cnt += (uint32_t)sel(az, 1 << 20, sel(ay, 1 << 10, 1));
            w.idx += (uint32_t)sel(az, w.sz, sel(ay, w.sy, w.sx));
            c.ids[s] = w.idx;
        }
        // c steps on an axis whose q was q0 add q0 + (q0+2) + ... = c (q0 + c - 1);
        // a live walk's distance stays below 2^31, so q and c (q0 + c - 1) fit
        // the 24-bit multiply
        const uint32_t cx = cnt & 1023u, cy = (cnt >> 10) & 1023u, cz = cnt >> 20;
        w.d2 += (int32_t)(mul24(cx, (uint32_t)w.qx + cx - 1u) +
                          mul24(cy, (uint32_t)w.qy + cy - 1u) +
                          mul24(cz, (uint32_t)w.qz + cz - 1u));
        w.qx += (int32_t)(2u * cx);
        w.qy += (int32_t)(2u * cy);
        w.qz += (int32_t)(2u * cz);
    } else {
#pragma unroll
        for (int s = 0; s < kChunk; ++s) {
            bool in = true;
            alive = walk_step<kGeneral>(w, m2, alive, in);
            c.ids[s] = (alive && in) ? w.idx : kOob;
        }
        if (!alive) {   // over: the index parks at kOob
            w.idx = kOob;
            w.sx = w.sy = w.sz = 0;
        }
    }
    return alive;
}

// kChunk steps and the occupancy of their voxels.
template <bool kGeneral, bool kBytes, bool kLone>
VG_HD bool walk_chunk(Walk &w, int32_t m2, bool alive, Chunk &c, bool load, const WalkMem &m)
{
    alive = step_chunk<kGeneral>(w, m2, alive, c);
    // A wavefront whose rays have all met their obstacle need not load (its
    // indices lie in the traced plane or at kOob, past the occupancy plane,
    // and would read 0).  The lone form loads anyway: with the same memory
    // operations on every path, the compiler's wait counts let the hit test
    // of a chunk wait for that chunk's loads only, not for the next chunk's,
    // which then stay in flight during the next chunk's steps.  Only the hit
    // test is skipped.
    c.loaded = vg_any(load);
    if (kLone || c.loaded) {
#pragma unroll
        for (int s = 0; s < kChunk; ++s)
            c.words[s] = kBytes ? load_occ_byte(m, c.ids[s]) : load_occ(m, (c.ids[s] >> 5) << 2);
    } else {
#pragma unroll
        for (int s = 0; s < kChunk; ++s)
            c.words[s] = 0u;
    }
    return alive;
}

// Marks of chunk c: free before the ray's first occupied voxel, traced from
// it on (the occupied voxel itself becomes occupied whatever its marks say).
// The hit is the lowest occupied slot of a ray still before its hit.  A lane
// that hits here moves to the traced plane: its walk index and the indices
// of the chunk walked after c (`next`) move up by n.  That chunk's words
// were loaded from the free plane and must no longer count: they are zeroed,
// or, in the lone form, whose registers are left alone while their loads are
// in flight, the hit test skips lanes whose before_hit is false.
template <bool kBytes, bool kLone>
VG_HD void resolve_chunk(const Chunk &c, bool &before_hit, Walk &w, Chunk &next,
                         const WalkMem &m)
{
    int hit = kChunk;
    // the lone form tests every chunk it loads (in its loading loop some ray
    // is still before its hit), so that every path consumes the loads
    if (kLone || c.loaded) {
        uint32_t hits = 1u << kChunk;
#pragma unroll
        for (int s = 0; s < kChunk; ++s)
            hits |= (kBytes ? (uint32_t)(c.words[s] == m.stamp) : bit_of(c.words[s], c.ids[s]))
                    << s;
        hit = lowest_set(hits);
        if (kLone && !before_hit)
            hit = kChunk;
    }
    if (vg_any(hit < kChunk)) {
#pragma unroll
        for (int s = 0; s < kChunk; ++s)
            store_mark(m, c.ids[s] + (s < hit ? 0u : m.n));
        if (hit < kChunk) {
            before_hit = false;
            w.idx += m.n;
#pragma unroll
            for (int s = 0; s < kChunk; ++s) {
                next.ids[s] += m.n;
                if (!kLone)
                    next.words[s] = 0u;
            }
        }
    } else {
#pragma unroll
        for (int s = 0; s < kChunk; ++s)
            store_mark(m, c.ids[s]);
    }
}

// Alg. 2 for one ray: walk, test occupancy before the first hit, mark free
// before it and "unknown and traced" from it on.  Chunks alternate: while one
// chunk's loads are in flight the other is walked.  A chunk walked after the
// walk ended holds no step (its indices are kOob: it loads 0 and stores
// nothing), so a lane is done once it has resolved the chunk that ended its
// walk.
//
// Two forms.  The first does the least work per chunk: a lane leaves the
// loop as soon as it is done, and a wavefront past all its obstacles loads
// nothing; other wavefronts on its SIMD may hide its load latency.  The lone
// form, made for a wavefront that has its SIMD to itself (a small frame,
// which waits out every latency), keeps the next chunk's loads in flight:
// each iteration walks and resolves both chunks, its only exit, at the end,
// is wave-uniform, and every chunk loads and is hit-tested, so that one
// sequence of memory operations runs through each iteration (otherwise the
// compiler's wait counts, merged over the paths, make each hit test wait for
// the next chunk's loads too).  Once every ray of the wavefront has met its
// obstacle (for good: before_hit never turns true again) either form goes on
// in a second loop that only steps and stores traced marks.  With that loop
// the lone form measured as fast as the first also where SIMDs are shared, and
// the kernels use it whenever the camera is inside the grid.
template <bool kGeneral, bool kBytes, bool kLone>
VG_HD void walk_ray(Walk &w, int32_t m2, const WalkMem &m)
{
    bool before_hit = true;   // Alg. 2: vox_val is still "free"
    Chunk a, b;
    bool alive = walk_chunk<kGeneral, kBytes, kLone>(w, m2, true, a, true, m);
    if (kLone) {
        while (true) {
            alive = walk_chunk<kGeneral, kBytes, kLone>(w, m2, alive, b, before_hit, m);
            resolve_chunk<kBytes, kLone>(a, before_hit, w, b, m);
            const bool more = alive;   // b was not the chunk that ended the walk
            alive = walk_chunk<kGeneral, kBytes, kLone>(w, m2, alive, a, before_hit, m);
            resolve_chunk<kBytes, kLone>(b, before_hit, w, a, m);
            if (!vg_any_u(more))
                return;
            if (!vg_any_u(before_hit))
                break;
        }
        // Chunk a is walked but not resolved; its indices are in the traced
        // plane (or kOob) on every lane.
        while (true) {
#pragma unroll
            for (int s = 0; s < kChunk; ++s)
                store_mark(m, a.ids[s]);
            if (!vg_any_u(alive))
                return;
            alive = step_chunk<kGeneral>(w, m2, alive, a);
        }
    } else {
        bool traced_only = false;
        while (true) {
            bool more = alive;
            alive = walk_chunk<kGeneral, kBytes, kLone>(w, m2, alive, b, before_hit, m);
            resolve_chunk<kBytes, kLone>(a, before_hit, w, b, m);
            if (!more)
                break;
            more = alive;
            alive = walk_chunk<kGeneral, kBytes, kLone>(w, m2, alive, a, before_hit, m);
            resolve_chunk<kBytes, kLone>(b, before_hit, w, a, m);
            if (!more)
                break;
            if (!vg_any(before_hit)) {
                traced_only = true;
                break;
            }
        }
        if (traced_only) {
            // as in the lone form: chunk a is walked but not resolved, its
            // indices in the traced plane or at kOob
            while (true) {
#pragma unroll
                for (int s = 0; s < kChunk; ++s)
                    store_mark(m, a.ids[s]);
                if (!alive)
                    break;
                alive = step_chunk<kGeneral>(w, m2, alive, a);
            }
        }
    }
}

}  // namespace vg

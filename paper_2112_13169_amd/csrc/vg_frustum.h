// vg_frustum.h -- which columns of a grid row one frame can change
// (Toumieh & Lambert, arXiv 2112.13169, Sec. IV-B and IV-C).
//
// Every voxel a ray of the fan visits meets that ray, and every ray lies in
// the fan's pyramid: the apex is the camera, the edges are the corner
// targets (+-hw, +-hh, vox_depth) (Sec. IV-C).  Every occupied voxel of a
// pinhole frame lies within vox_inf voxels of a measured point, and every
// measured point lies in the image's pyramid: the apex is the camera, the
// edges are the corner pixels' rays (Alg. 1).  So a voxel whose centre lies
// outside both pyramids, widened by a margin, keeps its value, and the merge
// need not read its marks; a seed row segment outside the image's pyramid
// holds no seed, and the x dilation need not read it.  Both regions are
// convex; a grid row meets each in one run of columns.
//
// Plain C++ without HIP (VG_FR_HD), so that the host tests can check the
// regions against the oracle's measurement grids.
#pragma once

#include <stdint.h>

#include <cmath>

#ifdef __HIPCC__
#define VG_FR_HD __host__ __device__ __forceinline__
#else
#define VG_FR_HD static inline
#endif

namespace vg {

// One bounding plane of a region, n . (c - apex) <= m for a voxel centre c,
// as the row test evaluates it: with t = e + f y + g z for grid row (y, z)
// (in double, so that rounding stays far below a column),
//   kind  1: columns x <= t * inv + c0 are admitted  (n_x > 0)
//   kind -1: columns x >= t * inv + c0 are admitted  (n_x < 0)
//   kind  0: every column if t >= 0, none otherwise   (n_x ~ 0)
struct RowPlane {
    double e, f, g, inv, c0;
    int32_t kind;
    int32_t pad;
};

struct Region {
    RowPlane p[4];
};

// The two regions of one frame, in the voxel units of its grid.  has_fan /
// has_img false: that region is unbounded (a spinning sensor's fan, whose
// ring of targets is not convex, and the occupied voxels of a spinning frame,
// of a point cloud or of an image whose valid range reaches behind the
// camera); the merge then reads whole rows.
struct RowLimits {
    int32_t has_fan, has_img;
    Region fan, img;
};

// Columns [lo, hi] of grid row (y, z), clipped to [xmin, xmax], whose voxel
// centres satisfy every plane of the region (lo > hi: none), widened by one
// column on each side.
VG_FR_HD void region_columns(const Region &R, int32_t y, int32_t z, int32_t xmin, int32_t xmax,
                             int32_t &lo, int32_t &hi)
{
    const double yd = (double)y, zd = (double)z;
    double flo = (double)xmin, fhi = (double)xmax;
    bool none = false;
    // selects, no branches: the device loads every plane before the first
    // is used
    for (int k = 0; k < 4; ++k) {
        const RowPlane &q = R.p[k];
        // a conservative bound: fused multiply-adds are fine here
        const double t = fma(q.g, zd, fma(q.f, yd, q.e));
        const double b = fma(t, q.inv, q.c0);   // kind 0: inv 0, b finite and unused
        fhi = q.kind > 0 ? fmin(fhi, b + 1.0) : fhi;
        flo = q.kind < 0 ? fmax(flo, b - 1.0) : flo;
        none = none || (q.kind == 0 && t < 0.0);
    }
    if (none || !(flo <= fhi)) {
        lo = 1;
        hi = 0;
        return;
    }
    lo = (int32_t)ceil(flo);
    hi = (int32_t)floor(fhi);
}

// The runs of grid row (y, z) that a frame may change: the fan's and the
// image's, each [lo, hi] within [0, gx - 1] (lo > hi: empty).  False: the
// frame's regions do not bound the row (every column may change).
VG_FR_HD bool row_runs(const RowLimits &L, int32_t y, int32_t z, int32_t gx, int32_t run[4])
{
    if (!L.has_fan || !L.has_img)
        return false;
    region_columns(L.fan, y, z, 0, gx - 1, run[0], run[1]);
    region_columns(L.img, y, z, 0, gx - 1, run[2], run[3]);
    return true;
}

// Whether columns [a, b] meet one of the runs.
VG_FR_HD bool runs_meet(const int32_t run[4], int32_t a, int32_t b)
{
    return (run[0] <= run[1] && a <= run[1] && b >= run[0]) ||
           (run[2] <= run[3] && a <= run[3] && b >= run[2]);
}

// Whether columns [a, b] of grid row (y, z) may hold a measured point's
// voxel; rows and columns may lie in the vox_inf padding around the grid
// (the image's region; always true with no such region).
VG_FR_HD bool row_run_seeded(const RowLimits &L, int32_t y, int32_t z, int32_t a, int32_t b)
{
    if (!L.has_img)
        return true;
    int32_t lo, hi;
    region_columns(L.img, y, z, a, b, lo, hi);
    return lo <= hi;
}

// Margin of the fan's region, in voxels: a visited voxel meets its ray, so
// its centre lies within sqrt(3)/2 of the pyramid; the rest covers the drift
// of the fp32 walk from the exact ray.
constexpr double kFanMargin = 1.5;

// One plane of a region from its grid-frame normal n (any length), margin m
// (voxels) and the apex o (voxels).  reach bounds |x + 1/2 - o_x| over every
// column a test asks about.
VG_FR_HD bool make_row_plane(const double n_in[3], double m, const float o[3], double reach,
                             RowPlane &q)
{
    const double len = sqrt(n_in[0] * n_in[0] + n_in[1] * n_in[1] + n_in[2] * n_in[2]);
    if (!(len > 1e-12))
        return false;
    const double n[3] = {n_in[0] / len, n_in[1] / len, n_in[2] / len};
    // n_x (x + 1/2 - o_x) <= m - n_y (y + 1/2 - o_y) - n_z (z + 1/2 - o_z) = t
    q.f = -n[1];
    q.g = -n[2];
    q.e = m - n[1] * (0.5 - (double)o[1]) - n[2] * (0.5 - (double)o[2]);
    q.c0 = (double)o[0] - 0.5;
    q.pad = 0;
    if (fabs(n[0]) > 1e-9) {
        q.kind = n[0] > 0.0 ? 1 : -1;
        q.inv = 1.0 / n[0];
    } else {
        // |n_x (x + 1/2 - o_x)| <= |n_x| reach: the row is admitted unless t
        // stays below that for every column
        q.kind = 0;
        q.inv = 0.0;
        q.e += fabs(n[0]) * reach + 1e-9;
    }
    return true;
}

// Plane `which` of one frame's regions: 0..3 the fan's sides (a <= hw,
// a >= -hw, b <= hh, b >= -hh of a pinhole fan of half sizes hw x hh at
// vox_depth vd), 4..7 the image's (x <= ku1 z, x >= ku0 z, y <= kv1 z,
// y >= kv0 z for an image whose corner pixels have the fp32 slopes ku0 <= ku
// <= ku1, kv0 <= kv <= kv1).  R: T^v_c's rotation (row-major); o: the camera
// in voxel units; gx: grid width (the columns the tests ask about lie in
// [-vox_inf, gx + vox_inf)).  The image's region is widened by
// (vox_inf + 1/2) sqrt(3) + 1 voxels: an occupied voxel's centre lies within
// vox_inf + 1/2 voxels per axis of a measured point, plus fp32 rounding.
// False if the plane is degenerate.
VG_FR_HD bool make_region_plane(int which, const float R[9], const float o[3], int32_t vd,
                                int32_t hw, int32_t hh, float ku0, float ku1, float kv0,
                                float kv1, int32_t vox_inf, int32_t gx, RowPlane &q)
{
    double c[3];
    switch (which) {
    case 0: c[0] = vd; c[1] = 0.0; c[2] = -(double)hw; break;
    case 1: c[0] = -(double)vd; c[1] = 0.0; c[2] = -(double)hw; break;
    case 2: c[0] = 0.0; c[1] = vd; c[2] = -(double)hh; break;
    case 3: c[0] = 0.0; c[1] = -(double)vd; c[2] = -(double)hh; break;
    case 4: c[0] = 1.0; c[1] = 0.0; c[2] = -(double)ku1; break;
    case 5: c[0] = -1.0; c[1] = 0.0; c[2] = (double)ku0; break;
    case 6: c[0] = 0.0; c[1] = 1.0; c[2] = -(double)kv1; break;
    default: c[0] = 0.0; c[1] = -1.0; c[2] = (double)kv0; break;
    }
    double n[3];
    for (int i = 0; i < 3; ++i)
        n[i] = (double)R[3 * i] * c[0] + (double)R[3 * i + 1] * c[1] + (double)R[3 * i + 2] * c[2];
    const double reach = (double)gx + 2.0 * vox_inf + fabs((double)o[0]) + 2.0;
    const double m = which < 4 ? kFanMargin : (vox_inf + 0.5) * sqrt(3.0) + 1.0;
    return make_row_plane(n, m, o, reach, q);
}

// The regions of one frame (fan: a pinhole fan, else unbounded; img: an
// image whose valid depths are not negative, else unbounded; the other
// arguments as for make_region_plane).
VG_FR_HD void make_row_limits(const float R[9], const float o[3], bool fan, int32_t vd,
                              int32_t hw, int32_t hh, bool img, float ku0, float ku1, float kv0,
                              float kv1, int32_t vox_inf, int32_t gx, RowLimits &L)
{
    L.has_fan = L.has_img = 0;
    if (!fan)
        return;
    bool ok = true;
    for (int which = 0; which < (img ? 8 : 4); ++which)
        ok = make_region_plane(which, R, o, vd, hw, hh, ku0, ku1, kv0, kv1, vox_inf, gx,
                               which < 4 ? L.fan.p[which] : L.img.p[which - 4]) && ok;
    L.has_fan = ok ? 1 : 0;
    L.has_img = ok && img ? 1 : 0;
}

}  // namespace vg

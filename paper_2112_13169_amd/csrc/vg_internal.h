// vg_internal.h -- parameter blocks and kernel launchers shared by the host
// API (vg_api.cpp) and the gfx950 kernels (vg_kernels.hip).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// A ray that met an occupied voxel in the free pass, parked for the traced
// pass: its fan coordinates (to rebuild direction and step sizes) and the
// walk state right after the hit voxel.
struct alignas(16) ParkedRay {
    int32_t ta, tb;      // fan target: pinhole (a, b); spinning (column, z)
    int32_t vx, vy, vz;  // current voxel
    float tmx, tmy, tmz; // next boundary crossing per axis
};
static_assert(sizeof(ParkedRay) == 32, "ParkedRay is 32 bytes");

// Occupancy planes of one frame.  Seeds live on the grid padded by vox_inf on
// every side (a point just outside the grid still inflates into it); padded
// coordinate = voxel coordinate + vox_inf.
struct Planes {
    int32_t n[3];        // grid size
    int32_t r;           // vox_inf
    int32_t wx;          // 32-voxel words per grid row: ceil(gx / 32)
    int32_t py, pz;      // padded rows: gy + 2r, gz + 2r
    int32_t seed_pitch;  // bytes per padded seed row (multiple of 64, >= 32*wx + 64)
    uint8_t *seed;       // per-frame seed stamps, [pz][py][seed_pitch]
    uint32_t *bitx;      // seeds dilated along x, [pz][py][wx] words
    uint32_t *occ;       // occupied voxels of the frame, [gz][gy][wx] words
    int32_t lo[3], hi[3];  // padded box that holds every seed (lo > hi: none)
    uint32_t epoch;      // stamp of this frame (1..255)
};

// Step 2a: transform and quantise every measured point, stamp its voxel.
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
    uint32_t *parked_count;
};

// Step 3: the bundled ray fan.  One wavefront owns an 8 x 8 tile of fan
// targets (tile_a along a / column, tile_b along b / z).
struct RayParams {
    float R[9];
    float o[3];       // camera position in voxel units
    int32_t v0[3];    // camera voxel
    int32_t n[3];
    int32_t wx;       // occupancy words per row
    int32_t kind;     // kPinhole (also points) or kSpinning
    int32_t vd, hw, hh;   // pinhole fan; spinning: hh = largest half height
    int32_t na, nb;       // fan extent along a and b
    int32_t tiles_a, tiles;
    const int32_t *hz;    // spinning: half height per column
    uint8_t *loc;
    const uint32_t *occ;
    ParkedRay *parked;
    uint32_t *parked_count;
    uint32_t parked_cap;
};

hipError_t launch_fill(void *dst, uint8_t value, size_t bytes, hipStream_t st);
hipError_t launch_seeds(const SeedParams &p, hipStream_t st);
// Seeds -> occupied bit plane (dilation by vox_inf along x, then y and z).
hipError_t launch_dilate(const Planes &pl, hipStream_t st);
// mid: optional event recorded between the free and the traced pass.
hipError_t launch_rays(const RayParams &p, hipStream_t st, hipEvent_t mid);
// Occupied bit plane -> local grid (runs after the traced pass).
hipError_t launch_mark_occupied(const Planes &pl, uint8_t *loc, hipStream_t st);
hipError_t launch_shift(const uint8_t *src, uint8_t *dst, const int32_t n[3],
                        const int32_t d[3], hipStream_t st);

}  // namespace vg

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

// A ray that met an occupied voxel in the free pass, parked for the traced
// pass: its fan coordinates (to rebuild direction and step sizes) and the
// walk state right after the hit voxel.
struct alignas(16) ParkedRay {
    int32_t ta, tb;      // fan target: pinhole (a, b); spinning (column, z)
    int32_t vx, vy, vz;  // current voxel
    float tmx, tmy, tmz; // next boundary crossing per axis
};
static_assert(sizeof(ParkedRay) == 32, "ParkedRay is 32 bytes");

// Step 2: transform, quantise and inflate every measured point.
struct OccParams {
    float R[9];       // R^v_c = R^w_c, row-major
    float tv[3];      // t^v = t^w_c - origin_w
    float s;          // vox_size
    int32_t n[3];     // grid size
    int32_t r;        // vox_inf
    int32_t kind;     // kPinhole, kSpinning or kPoints
    int32_t W, H;     // image size (kPoints: W = number of points, H = 1)
    int64_t pitch;    // image row pitch in floats
    double fx, fy, cx, cy;
    float dmin, dmax;
    const float *img;     // depth / range image, or points[W][3]
    const float *col_tab; // spinning: cos/sin azimuth per column
    const float *row_tab; // spinning: cos/sin elevation per row
    uint8_t *loc;         // local grid
    uint8_t *occ;         // per-frame occupancy stamps
    uint32_t *parked_count;
    uint32_t epoch;       // stamp of this frame (1..255)
};

// Step 3: the bundled ray fan.  One wavefront owns an 8 x 8 tile of fan
// targets (tile_a along a / column, tile_b along b / z).
struct RayParams {
    float R[9];
    float o[3];       // camera position in voxel units
    int32_t v0[3];    // camera voxel
    int32_t n[3];
    int32_t kind;     // kPinhole (also points) or kSpinning
    int32_t vd, hw, hh;   // pinhole fan; spinning: hh = largest half height
    int32_t na, nb;       // fan extent along a and b
    int32_t tiles_a, tiles;
    const int32_t *hz;    // spinning: half height per column
    uint8_t *loc;
    const uint8_t *occ;
    ParkedRay *parked;
    uint32_t *parked_count;
    uint32_t parked_cap;
    uint32_t epoch;
};

hipError_t launch_fill(void *dst, uint8_t value, size_t bytes, hipStream_t st);
hipError_t launch_occupied(const OccParams &p, hipStream_t st);
// mid: optional event recorded between the free and the traced pass.
hipError_t launch_rays(const RayParams &p, hipStream_t st, hipEvent_t mid);
hipError_t launch_shift(const uint8_t *src, uint8_t *dst, const int32_t n[3],
                        const int32_t d[3], hipStream_t st);

}  // namespace vg

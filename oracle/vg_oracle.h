/*
 * vg_oracle.h -- plain, single-threaded CPU oracle for depth-frame -> voxel-grid
 * generation (Toumieh & Lambert, "GPU Accelerated Voxel Grid Generation for fast
 * MAV Exploration", arXiv 2112.13169).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no source, header, table or helper with the GPU library, and the
 * GPU library never calls it.
 *
 * Every function follows the paper's steps in its order and notation:
 *   Sec. IV-A  voxel grid setup (two grids, ms reset before every measurement)
 *   Sec. IV-B  populate occupied voxels, Alg. 1 (transform, quantise, inflate)
 *   Sec. IV-C  ray-trace to free voxels, Alg. 2 (bundled fan, Amanatides-Woo walk)
 *   Sec. IV-D  update the local grid, Alg. 3
 *   Sec. IV-E  shift the local grid
 * Where the paper is silent or garbled the implementation takes a written reading;
 * each reading is named at the place it is used (R1..R27).
 *
 * Voxel states.  loc grid: 0 unknown, 1 free, 2 occupied.  ms grid additionally
 * uses 3 = "unknown and traced" (Sec. IV-C, Fig. 2).
 *
 * Floating point: every fp32 operation is written out in a fixed order and must
 * be compiled with -ffp-contract=off and without fast-math.  Integer decisions
 * that depend on trigonometry (ray-fan sizes) are made once, in double.
 */
#ifndef VG_ORACLE_H
#define VG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OG_UNKNOWN 0
#define OG_FREE 1
#define OG_OCCUPIED 2
#define OG_TRACED 3
#define OG_OUTSIDE 255 /* og_trace_ray: a walk step that left the grid */

/* Ray-fan sizes, Sec. IV-C (R9, R10).  out[0] = vox_depth, out[1] = half width
 * hw, out[2] = half height hh; vox_width = 2*hw+1, vox_height = 2*hh+1.
 * Returns 0, or -1 if the sizes are out of the supported range. */
int og_fan_sizes(float depth, float vox_size, double fov_x, double fov_y, int32_t out[3]);

/* Number of rays of a spinning-sensor fan (R27) and its half height table:
 * hz_out (optional, 8*vox_depth entries, column order of og_spin_column). */
int64_t og_spin_ray_count(int32_t vox_depth, double tan_half_vfov, int32_t *hz_out);

/* Grid origin after integer shifts (state of Sec. IV-A/IV-E):
 * origin = base + (float)shift * vox_size, per component, each op rounded. */
void og_origin(const float base[3], const int32_t shift[3], float vox_size, float origin[3]);

/* Alg. 1, transform and quantise, for one camera-frame point: p^v = R p^c + t^v (R8) and
 * q = floor(p^v / vox_size) (R1).  Writes the floored values as floats. */
void og_quantize(const float R[9], const float tv[3], float vox_size, const float pc[3], float q[3]);

/* Alg. 2 for one ray.  o = ray start in voxel units, dir = ray direction in voxel
 * units, m2 = squared termination length (R15).  ms (may be NULL = all unknown)
 * supplies occupancy and receives FREE / TRACED marks with the priority of R18.
 * If out_xyz / out_val are given, the walk's voxels (every step, in order, also
 * those outside the grid) and the value assigned to each (OG_FREE, OG_TRACED,
 * OG_OCCUPIED for a hit, OG_OUTSIDE) are written, up to max_out entries.
 * Returns the number of walk steps. */
int64_t og_trace_ray(const float o[3], const float dir[3], int64_t m2,
                     int32_t gx, int32_t gy, int32_t gz, uint8_t *ms,
                     int32_t *out_xyz, uint8_t *out_val, int64_t max_out);

/* Steps 1-4 for one pinhole z-depth image (Sec. IV-A..IV-D).
 * loc: in/out local grid (gx*gy*gz bytes, x fastest).  ms_out: optional copy of
 * the measurement grid after step 3.  depth: width*height floats, row-major.
 * R (row-major), t: T^w_c.  origin: current grid origin in the world frame.
 * stats (optional, 5 entries): voxel updates (ms != unknown), in-grid walk steps,
 * occupied voxels, rays, in-grid walk steps after each ray's first hit.
 * Returns 0 or -1 on invalid arguments. */
int og_integrate_pinhole(int32_t gx, int32_t gy, int32_t gz, float vox_size,
                         const float origin[3], int32_t vox_inf,
                         uint8_t *loc, uint8_t *ms_out,
                         const float *depth, int32_t width, int32_t height,
                         double fx, double fy, double cx, double cy,
                         double fov_x, double fov_y, float depth_min, float depth_max,
                         const float R[9], const float t[3], int64_t stats[5]);

/* Steps 1-4 for one spinning range image (R27).  col_tab: 2*width floats
 * (cos az, sin az per column), row_tab: 2*height floats (cos el, sin el per row).
 * vfov: full vertical field of view in radians. */
int og_integrate_spinning(int32_t gx, int32_t gy, int32_t gz, float vox_size,
                          const float origin[3], int32_t vox_inf,
                          uint8_t *loc, uint8_t *ms_out,
                          const float *range, int32_t width, int32_t height,
                          const float *col_tab, const float *row_tab,
                          double vfov, float depth_min, float depth_max,
                          const float R[9], const float t[3], int64_t stats[5]);

/* Steps 1-4 for a dense point cloud given in the camera frame (Sec. IV input
 * form "dense point cloud"); the ray fan is the pinhole fan of fov_x/fov_y. */
int og_integrate_points(int32_t gx, int32_t gy, int32_t gz, float vox_size,
                        const float origin[3], int32_t vox_inf,
                        uint8_t *loc, uint8_t *ms_out,
                        const float *points, int64_t n_points,
                        double fov_x, double fov_y, float depth,
                        const float R[9], const float t[3], int64_t stats[5]);

/* Alg. 3 applied to whole grids (R19). */
void og_merge(int64_t n, const uint8_t *ms, uint8_t *loc);

/* Sec. IV-E (R21): out[i] = in[i + delta] if inside, else unknown. */
void og_shift(int32_t gx, int32_t gy, int32_t gz, const uint8_t *in, uint8_t *out,
              int32_t dx, int32_t dy, int32_t dz);

/* R21 helper: integer offset that re-centres the grid on a camera at t_w_c. */
void og_center_offset(int32_t gx, int32_t gy, int32_t gz, float vox_size,
                      const float origin[3], const float t_w_c[3], int32_t delta[3]);

#ifdef __cplusplus
}
#endif
#endif

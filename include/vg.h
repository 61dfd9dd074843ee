/*
 * vg.h -- C ABI of the MI355X (gfx950) voxel-grid library: one dense depth
 * frame -> a robot-centred uint8 grid of occupied / free / unknown voxels.
 *
 * Method: Toumieh & Lambert, "GPU Accelerated Voxel Grid Generation for fast
 * MAV Exploration" (arXiv 2112.13169), Sec. IV:
 *   step 1 voxel grid setup (Sec. IV-A)        -> vg_create_grid
 *   steps 2-4 populate occupied (Alg. 1), ray-trace to free (Alg. 2) and
 *   update the local grid (Alg. 3)             -> vg_integrate_frame
 *   step 5 shift the local grid (Sec. IV-E)    -> vg_shift_grid
 * Argument names follow the paper's nomenclature (Table I).
 *
 * Conventions for every entry point:
 *  - Ownership: the caller owns every device buffer (the local grid, the
 *    scratch workspace, depth images).  The library never allocates
 *    or frees device memory; a vg_grid handle owns host metadata only.
 *  - Asynchrony: device work is enqueued on `stream` (a hipStream_t; NULL is
 *    the default stream) and nothing blocks the host, except where stated.
 *    One handle must not be used from two streams at once; distinct handles
 *    are independent.
 *  - Errors: argument errors are detected before any device work is enqueued,
 *    return VG_ERR_ARG and leave the grid unchanged.  HIP launch / copy errors
 *    return VG_ERR_HIP; the grid's content is then undefined (launches of
 *    the failed call may have run), and its next frame first clears the
 *    per-frame planes, so no stamp of the failed call is taken for its own.
 *    Nothing throws across the ABI.
 *  - Layout: vg_read_grid / vg_write_grid exchange grids as
 *    uint8[grid_size_z][grid_size_y][grid_size_x] with the paper's linear index
 *    idx = x + y*grid_size_x + z*grid_size_x*grid_size_y (Sec. IV-D); grid
 *    axes are aligned with the world (ENU) frame.  The device buffers bound to
 *    a grid hold it with rows padded to a multiple of 32 voxels (row pitch
 *    32*ceil(grid_size_x/32) bytes); their content is for the library only.
 *  - Voxel values: VG_UNKNOWN 0, VG_FREE 1, VG_OCCUPIED 2.  Other byte values
 *    written by vg_write_grid are kept until a frame overwrites them.
 */
#ifndef VG_H
#define VG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vg_grid vg_grid;
typedef int32_t vg_status;

#define VG_OK 0
#define VG_ERR_ARG (-1)    /* invalid argument; nothing was enqueued          */
#define VG_ERR_HIP (-2)    /* a HIP runtime call failed                       */
#define VG_ERR_BUDGET (-3) /* a caller buffer is smaller than required         */
#define VG_ERR_STATE (-4)  /* handle used on a different device than created  */

#define VG_UNKNOWN 0
#define VG_FREE 1
#define VG_OCCUPIED 2

#define VG_PINHOLE 0  /* z-depth image (depth along the optical axis)      */
#define VG_SPINNING 1 /* range image of a spinning sensor, 360 deg azimuth */

/* T^w_c: camera -> world.  R row-major (columns are the camera axes in the
 * world frame), t = camera centre in metres.  Pinhole camera frame: z along
 * the optical axis, x right (across fov_x), y down (across fov_y).  Spinning
 * sensor frame: z up.  All 12 entries must be finite. */
typedef struct vg_pose {
    float R[9];
    float t[3];
} vg_pose;

/* Sensor model.
 * VG_PINHOLE: pixel (u, v) looks along ((u - cx) / fx, (v - cy) / fy, 1); the
 *   image holds z-depth in metres.  fov_x / fov_y (radians, in (0, pi)) set
 *   the ray fan of Sec. IV-C.
 * VG_SPINNING: column u has azimuth cos/sin col_tab[2u], col_tab[2u+1]; row v
 *   has elevation cos/sin row_tab[2v], row_tab[2v+1] (device pointers,
 *   float32); the image holds range in metres; fov_y is the full vertical
 *   field of view (radians) that bounds the ray fan; fov_x, fx..cy unused.
 * Image sizes are at most 65535 x 65535.
 * A pixel is a measurement iff depth_min <= value <= depth (NaN is not).
 * `depth` is also the range the fan clears: vox_depth = round(depth/vox_size). */
typedef struct vg_sensor {
    int32_t kind;
    int32_t width, height;
    int32_t reserved;
    double fx, fy, cx, cy;
    double fov_x, fov_y;
    float depth_min, depth;
    const float *col_tab;
    const float *row_tab;
} vg_sensor;

/* Ray-fan sizes of Sec. IV-C for a sensor on a grid of voxel size vox_size:
 * out[0] = vox_depth, out[1] = half width, out[2] = half height (pinhole; the
 * fan is (2*out[1]+1) x (2*out[2]+1) rays), out[3] = number of rays.
 * Host-only; returns VG_ERR_ARG when the sizes are out of range
 * (vox_depth > 16384, half sizes > 16384). */
vg_status vg_fan_sizes(const vg_sensor *sensor, float vox_size, int64_t out[4]);

/* Bytes of the device buffer of a grid of this size.  Host-only; 0 for
 * invalid sizes. */
size_t vg_grid_bytes(int32_t grid_size_x, int32_t grid_size_y, int32_t grid_size_z);

/* Bytes of device scratch workspace a grid of this size and vox_inf needs
 * for one set of per-frame planes (stamp and bit planes of steps 2-3, Alg. 1
 * and 2; with the frame's row regions and, in the first set, the order in
 * which large walks take their ray blocks).  A scratch of k times this size (k <= VG_MAX_PLANE_SETS) holds k
 * sets: vg_integrate_batch then runs up to k consecutive frames of the grid
 * together (see there).  Host-only; 0 for invalid sizes. */
size_t vg_scratch_bytes(int32_t grid_size_x, int32_t grid_size_y, int32_t grid_size_z,
                        int32_t vox_inf);

/* Most plane sets a grid's scratch is used for (scratch beyond that many
 * sets is left alone). */
#define VG_MAX_PLANE_SETS 16

/* Step 1 (Sec. IV-A): bind caller buffers to a new grid and set every voxel
 * of loc_grid to unknown (enqueued on `stream`).
 *   loc_grid: device, 16-byte aligned, grid_bytes >= vg_grid_bytes(...).  It
 *     holds the grid as a ring buffer, so shifts work in place.
 *   loc_spare: unused (may be NULL).
 *   scratch: device, scratch_bytes >= vg_scratch_bytes(..., vox_inf), 256-byte
 *     aligned; it is cleared here and owned by the grid until destroyed.
 *     floor(scratch_bytes / vg_scratch_bytes(...)) plane sets, at most
 *     VG_MAX_PLANE_SETS, are used.
 *   origin_w: world position (m) of the grid corner (voxel (0,0,0)'s minimum
 *     corner); vox_size > 0 m; vox_inf in [0, 16] voxels of inflation.
 *   Dimensions in [1, 65535] with vg_grid_bytes(...) < 2^30.
 * Returns VG_ERR_BUDGET if grid_bytes or scratch_bytes is too small.
 * On success *out receives the handle. */
vg_status vg_create_grid(int32_t grid_size_x, int32_t grid_size_y, int32_t grid_size_z,
                         float vox_size, const float origin_w[3], int32_t vox_inf,
                         uint8_t *loc_grid, uint8_t *loc_spare, size_t grid_bytes,
                         void *scratch, size_t scratch_bytes, void *stream, vg_grid **out);

/* Bind new device buffers to an existing grid (same sizes as for
 * vg_create_grid), keeping its host state: sizes, vox_size, origin and the
 * accumulated integer shift, vox_inf.  The new scratch is cleared here; the
 * content of loc_grid is the caller's (restore it with vg_write_grid).  This
 * lets a caller release a grid's device memory while it is idle (after
 * vg_read_grid) and resume it later with results identical to never having
 * released it.  All work on the old buffers must have been enqueued on
 * `stream` or completed. */
vg_status vg_rebind_grid(vg_grid *g, uint8_t *loc_grid, uint8_t *loc_spare, size_t grid_bytes,
                         void *scratch, size_t scratch_bytes, void *stream);

/* Steps 2-4 (Alg. 1, 2, 3) for one frame, enqueued on `stream`:
 *   depth: device, sensor->height rows of sensor->width float32, rows
 *     row_pitch_bytes apart (>= 4*width, multiple of 4).
 *   T_w_c: camera pose for this frame (host struct, read before returning).
 * The frame's occupied voxels (vox_inf cubes around the measured points,
 * clipped to the grid) become VG_OCCUPIED; voxels the ray fan crosses before
 * its first occupied voxel become VG_FREE unless some ray crosses them after
 * a hit, in which case they become VG_UNKNOWN; every other voxel keeps its
 * value.  Returns VG_ERR_ARG if the ray fan is too large (more than 2^31
 * ray lanes). */
vg_status vg_integrate_frame(vg_grid *g, const float *depth, int64_t row_pitch_bytes,
                             const vg_sensor *sensor, const vg_pose *T_w_c, void *stream);

/* Step 5 then steps 2-4 (Sec. IV-E; Alg. 1, 2, 3): the same as
 * vg_shift_grid(g, dx, dy, dz, stream) followed by vg_integrate_frame(g, ...)
 * -- the same grid, the same errors (VG_ERR_ARG leaves the grid untouched,
 * shift included) -- in one call.  The shift's clear of the exposed slabs
 * runs as extra workgroups of the frame's ray-walk launch, on compute units
 * the walk leaves idle, instead of a launch of its own.  With the
 * measurement hook set, the frame's shift pair records markers only (the
 * clear's time is inside the walk's pair). */
vg_status vg_integrate_frame_shifted(vg_grid *g, const float *depth, int64_t row_pitch_bytes,
                                     const vg_sensor *sensor, const vg_pose *T_w_c, int32_t dx,
                                     int32_t dy, int32_t dz, void *stream);

/* Same as vg_integrate_frame for a dense point cloud (the paper's stereo input
 * form, Sec. IV): `points` is device float32[n_points][3] in the camera frame;
 * an entry is a measurement iff all three coordinates are finite.  The ray fan
 * is the pinhole fan of sensor->fov_x, fov_y and depth (kind must be
 * VG_PINHOLE; width, height, fx..cy are ignored). */
vg_status vg_integrate_points(vg_grid *g, const float *points, int64_t n_points,
                              const vg_sensor *sensor, const vg_pose *T_w_c, void *stream);

/* Step 5 (Sec. IV-E): shift the grid content by an integer voxel offset:
 * new[x,y,z] = old[x+dx, y+dy, z+dz] where that lies inside, else unknown; the
 * grid origin moves by (dx,dy,dz)*vox_size (kept as an integer count so it
 * never drifts).  The buffer is a ring: the shift moves its offsets and
 * clears only the slabs that enter the grid (|dx|*gy*gz + |dy|*gx*gz +
 * |dz|*gx*gy voxels at most).  Enqueued on `stream`; (0,0,0) does nothing. */
vg_status vg_shift_grid(vg_grid *g, int32_t dx, int32_t dy, int32_t dz, void *stream);

/* Offset that re-centres the grid on a camera at t_w_c (metres), the shift
 * of Sec. IV-E that keeps the robot at the centre of its local grid:
 * delta = floor((t_w_c - origin_w) / vox_size) - grid_size / 2 (fp32 as
 * written, integer halving).  Host-only. */
vg_status vg_center_offset(const vg_grid *g, const float t_w_c[3], int32_t delta_out[3]);

/* vg_center_offset as it will be once shifts totalling pending[3] voxels
 * have been applied (NULL: none) -- the offsets of consecutive frames of one
 * grid in a batch.  Host-only. */
vg_status vg_center_offset_after(const vg_grid *g, const int32_t pending[3], const float t_w_c[3],
                                 int32_t delta_out[3]);

/* Current grid origin in the world frame: the corner of voxel (0,0,0), the
 * translation of T^v_w (Table I; Sec. IV-A), moved by vox_size per voxel of
 * accumulated shift (Sec. IV-E): origin = origin_w + (float)shift * vox_size
 * per axis, in fp32.  Host-only. */
vg_status vg_grid_origin(const vg_grid *g, float origin_w_out[3]);

/* Copy the local grid (Sec. IV-A: occupied / free / unknown voxels) to dst
 * in the linear layout of Sec. IV-D (idx = x + y*gx + z*gx*gy, whatever the
 * ring offsets of the device buffer): dst holds gx*gy*gz bytes, device
 * memory if dst_is_device, else host memory.  Enqueued on `stream` --
 * synchronise the stream before reading a host destination. */
vg_status vg_read_grid(const vg_grid *g, uint8_t *dst, int32_t dst_is_device, void *stream);

/* Overwrite the local grid from src (gx*gy*gz bytes, the linear layout of
 * vg_read_grid; device memory if src_is_device, else host memory), e.g. to
 * restore a checkpoint; the ring offsets restart at 0.  Not a step of the
 * paper: it lets a server release an idle grid's device memory and resume
 * it later (see vg_rebind_grid). */
vg_status vg_write_grid(vg_grid *g, const uint8_t *src, int32_t src_is_device, void *stream);

/* One frame of a batch. */
typedef struct vg_frame {
    vg_grid *grid;            /* grid the frame is integrated into                 */
    int32_t shift[3];         /* shift of `grid` applied right before the frame    */
    int32_t is_points;        /* 0: image (sensor.kind), 1: point cloud            */
    const float *data;        /* device: image rows, or float32[n_points][3]        */
    int64_t row_pitch_bytes;  /* images: as for vg_integrate_frame                  */
    int64_t n_points;         /* point clouds: as for vg_integrate_points           */
    vg_sensor sensor;
    vg_pose T_w_c;
} vg_frame;

/* Bytes of device workspace vg_integrate_batch needs for up to max_frames
 * frames (at most 4096).  Host-only; 0 for invalid counts. */
size_t vg_batch_workspace_bytes(int32_t max_frames);

/* Steps 2-5 for a batch of frames, enqueued on `stream`.  The result equals,
 * for i = 0 .. n_frames-1 in order, vg_shift_grid(frames[i].grid,
 * frames[i].shift) followed by vg_integrate_frame (or vg_integrate_points)
 * of frames[i] -- voxel for voxel.  Frames may target any mix of grids on the
 * current device; frames of one grid are applied in their order.  Frames
 * run together in rounds: a grid whose scratch holds S plane sets (see
 * vg_create_grid) puts its k-th frame of the batch into round floor(k / S),
 * on plane set k mod S, and each round is one launch per stage over all its
 * frames, whatever their image sizes, sensors, poses and grid sizes.  Steps
 * 2-3 of a round's frames of one grid run in parallel, each frame on its own
 * planes in its own (shifted) grid coordinates, since they read only their
 * own measurements (Alg. 1, 2); the round's merge then takes each grid's
 * frames in order, every frame's shift clear (Sec. IV-E) and marks (Alg. 3)
 * applied in turn, so the latest frame that saw a voxel decides it.  A round
 * of a single frame runs the one-frame launches instead (the shift's clear
 * inside its walk launch, as vg_integrate_frame_shifted), unless stage
 * events are given (vg_integrate_batch_timed).
 *   workspace: device, 256-byte aligned, workspace_bytes >=
 *     vg_batch_workspace_bytes(n_frames) (else VG_ERR_BUDGET).  The frame
 *     tables are written into it through kernel arguments (no host staging
 *     buffer, no host synchronisation), so a later call may reuse it on the
 *     same stream at once.
 * Every frame is checked before anything is enqueued (VG_ERR_ARG: no grid
 * changes).  The call enqueues kernels only, so it can be captured into a
 * HIP graph.  A replay repeats the captured call exactly: the same poses,
 * shifts, per-frame stamps and ring offsets, taken from the kernel
 * arguments, with the image buffers read at replay time.  The host state of
 * the grids (origin, ring offsets, stamp) advances once, at capture.  So a
 * replay gives the eager call's result only when it repeats that call's
 * inputs -- the same image contents, and no call on its grids in between
 * (the marks a replay leaves then carry the stamps the replay itself
 * writes); a replay after new image contents, or after other calls on the
 * grids, is not a valid integration. */
vg_status vg_integrate_batch(const vg_frame *frames, int32_t n_frames, void *workspace,
                             size_t workspace_bytes, void *stream);

/* vg_integrate_batch with a measurement hook: events (hipEvent_t, NULL
 * entries skipped) holds 12 entries, the (start, stop) pair of each batch
 * stage in launch order -- shift, seed, dilation x, dilation yz, ray walk,
 * merge.  A stage's start event takes the start time of its first launch and
 * its stop event the end time of its last (recorded by the launches; a stage
 * that launches nothing records markers).  events NULL: vg_integrate_batch. */
vg_status vg_integrate_batch_timed(const vg_frame *frames, int32_t n_frames, void *workspace,
                                   size_t workspace_bytes, void *const *events, void *stream);

/* Most frames one vg_integrate_batch_static call takes. */
#define VG_STATIC_BATCH_MAX_FRAMES 256

/* vg_integrate_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no workspace argument -- the frame tables go to a device array
 * the library holds, one per GPU (172 288 bytes, VG_STATIC_BATCH_MAX_FRAMES
 * frames' worth, held until the process ends).  The call allocates no device
 * memory.  n_frames > VG_STATIC_BATCH_MAX_FRAMES returns VG_ERR_BUDGET and
 * enqueues nothing.  Every call on one GPU shares that GPU's array, and each
 * call overwrites it before reading it: calls enqueued one after another on
 * one stream are safe, while calls whose work can overlap on one GPU (other
 * streams, or other host threads' calls not ordered with this one) race and
 * give undefined grids.  Everything else -- results, errors, HIP-graph
 * capture and its replays -- is as for vg_integrate_batch. */
vg_status vg_integrate_batch_static(const vg_frame *frames, int32_t n_frames, void *stream);

/* Shape of the ray bundle one wavefront walks: tiles of (1 << log2_width)
 * fan targets along the fan's width (pinhole columns, or ring columns of a
 * spinning fan) by (64 >> log2_width) along its height; log2_width in
 * [0, 6], default 3 (8 x 8).  Results do not depend on it (every ray is
 * walked alone); speed does.  Host-only; applies to later frames of g. */
vg_status vg_set_ray_tile(vg_grid *g, int32_t log2_width);

/* Measurement hook.  events holds n_sets sets of 10 hipEvent_t: per set the
 * (start, stop) pairs of five stages in this order: seed pass, dilation, ray
 * walk, resolve pass, shift.  With n_sets > 0, frame k (each following
 * vg_integrate_frame / vg_integrate_points call) uses set j = k mod n_sets,
 * and a vg_shift_grid call uses the set of the frame that follows it.  A
 * stage's start event takes the start time of its first kernel dispatch and
 * its stop event the end time of its last (the dispatches record them, so
 * hipEventElapsedTime gives device execution time with no marker in
 * between); a stage that launches nothing records both events as markers on
 * the stream.  NULL entries are not recorded.  The array is copied; the
 * events must stay alive while set.  n_sets = 0 (events may be NULL) turns
 * recording off. */
vg_status vg_set_profile_events(vg_grid *g, void *const *events, int32_t n_sets);

/* Release the handle (host metadata only; caller buffers are untouched).
 * The caller must make sure no work using the handle is still queued if it
 * frees the buffers afterwards. */
vg_status vg_destroy_grid(vg_grid *g);

/* Static description of a status code. */
const char *vg_status_str(vg_status s);

#ifdef __cplusplus
}
#endif
#endif

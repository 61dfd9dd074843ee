/*
 * vg_oracle.c -- plain CPU oracle for depth-frame -> voxel-grid generation.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg; never by the GPU library.  Single-threaded,
 * written for reading, not for speed.  Build with
 *     gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared
 * so that every fp32 operation below is rounded exactly as written.
 *
 * Parity status per function (pins live in tests/test_oracle_*.py):
 *   og_fan_sizes          pinned (paper's standard parameters, closed forms)
 *   og_quantize           pinned (exact binary hand cases, brute force)
 *   og_trace_ray          pinned (hand rays, brute-force segment/box order)
 *   og_integrate_pinhole  pinned (union-of-cubes brute force, invariants,
 *                         hand scenes); the free/traced priority (R18) and the
 *                         traced->unknown merge (R19) are readings: parity
 *                         unpinned by the paper, pinned by hand-built cases
 *   og_integrate_spinning parity unpinned (the paper has no spinning sensor);
 *                         checked by invariants and hand columns only
 *   og_integrate_points   pinned through the same cases as the pinhole path
 *   og_merge, og_shift    pinned (exhaustive truth table, closed form)
 */
#include "vg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ helpers */

static int64_t lin(int32_t gx, int32_t gy, int32_t x, int32_t y, int32_t z)
{
    /* Sec. IV-D: idx = x + y*grid_size_x + z*grid_size_x*grid_size_y */
    return (int64_t)x + (int64_t)y * gx + (int64_t)z * gx * gy;
}

static int inside(int32_t gx, int32_t gy, int32_t gz, int32_t x, int32_t y, int32_t z)
{
    return x >= 0 && y >= 0 && z >= 0 && x < gx && y < gy && z < gz;
}

/* Round half away from zero, in double (R9, R10, R27). */
static double round_half_away(double v)
{
    return v < 0.0 ? -floor(-v + 0.5) : floor(v + 0.5);
}

/* ---------------------------------------------------- ray-fan sizes (IV-C) */

int og_fan_sizes(float depth, float vox_size, double fov_x, double fov_y, int32_t out[3])
{
    /* R9: vox_depth = depth / vox_size, rounded to the closest integer. */
    double vd = round_half_away((double)depth / (double)vox_size);
    if (!(vd >= 1.0 && vd <= 16384.0))
        return -1;
    /* R10: vox_width = 2*tan(fov_x/2)*vox_depth + 1 is odd by construction:
     * the half width tan(fov_x/2)*vox_depth is rounded, then doubled, plus 1. */
    double hw = round_half_away(tan(fov_x / 2.0) * vd);
    double hh = round_half_away(tan(fov_y / 2.0) * vd);
    if (!(hw >= 0.0 && hw <= 16384.0 && hh >= 0.0 && hh <= 16384.0))
        return -1;
    out[0] = (int32_t)vd;
    out[1] = (int32_t)hw;
    out[2] = (int32_t)hh;
    return 0;
}

/* R27: the spinning fan's columns walk the square ring max(|x|,|y|) = vox_depth
 * counter-clockwise, starting just above (VD, -VD): 8*VD lattice columns. */
static void spin_column(int32_t c, int32_t vd, int32_t *x, int32_t *y)
{
    int32_t side = c / (2 * vd), k = c % (2 * vd);
    switch (side) {
    case 0: *x = vd;          *y = -vd + 1 + k; break;
    case 1: *x = vd - 1 - k;  *y = vd;          break;
    case 2: *x = -vd;         *y = vd - 1 - k;  break;
    default: *x = -vd + 1 + k; *y = -vd;        break;
    }
}

static int32_t spin_half_height(int32_t x, int32_t y, double tan_half_vfov)
{
    /* R27: |z| <= round(tan(vfov/2) * sqrt(x^2 + y^2)), decided in double. */
    return (int32_t)round_half_away(tan_half_vfov * sqrt((double)x * x + (double)y * y));
}

int64_t og_spin_ray_count(int32_t vd, double tan_half_vfov, int32_t *hz_out)
{
    int64_t n = 0;
    for (int32_t c = 0; c < 8 * vd; ++c) {
        int32_t x, y;
        spin_column(c, vd, &x, &y);
        int32_t hz = spin_half_height(x, y, tan_half_vfov);
        if (hz_out)
            hz_out[c] = hz;
        n += 2 * (int64_t)hz + 1;
    }
    return n;
}

/* ------------------------------------------------------ grid frame (IV-A) */

void og_origin(const float base[3], const int32_t shift[3], float vox_size, float origin[3])
{
    for (int a = 0; a < 3; ++a) {
        float off = (float)shift[a] * vox_size;
        origin[a] = base[a] + off;
    }
}

/* R8: row i of T^v_c p = ((R_i0*x + R_i1*y) + R_i2*z) + t_i, every op rounded. */
static void transform(const float R[9], const float t[3], const float p[3], float out[3])
{
    for (int i = 0; i < 3; ++i) {
        float a = R[3 * i + 0] * p[0];
        float b = R[3 * i + 1] * p[1];
        float s = a + b;
        float c = R[3 * i + 2] * p[2];
        s = s + c;
        out[i] = s + t[i];
    }
}

/* R11: ray direction = rotation part only (w = 0), same op order as R8. */
static void rotate(const float R[9], const float p[3], float out[3])
{
    for (int i = 0; i < 3; ++i) {
        float a = R[3 * i + 0] * p[0];
        float b = R[3 * i + 1] * p[1];
        float s = a + b;
        float c = R[3 * i + 2] * p[2];
        out[i] = s + c;
    }
}

/* A4 / R7: T^v_w is the pure translation -origin (grid axes are ENU-aligned),
 * so T^v_c = (R^w_c, t^w_c - origin). */
static void grid_translation(const float t[3], const float origin[3], float tv[3])
{
    for (int a = 0; a < 3; ++a)
        tv[a] = t[a] - origin[a];
}

/* ----------------------------------------- Alg. 1: populate occupied (IV-B) */

void og_quantize(const float R[9], const float tv[3], float vox_size, const float pc[3], float q[3])
{
    float pv[3];
    transform(R, tv, pc, pv);              /* Alg. 1: the transform */
    for (int a = 0; a < 3; ++a)            /* Alg. 1: quantise, R1: floor */
        q[a] = floorf(pv[a] / vox_size);
}

/* Alg. 1, inflation, for one point already transformed; R2 clips the cube to the
 * grid and drops points whose cube cannot reach it. */
static void add_occ(int32_t gx, int32_t gy, int32_t gz, int32_t r, const float q[3], uint8_t *ms)
{
    const int32_t n[3] = {gx, gy, gz};
    for (int a = 0; a < 3; ++a) {
        if (!(q[a] >= (float)(-r) && q[a] <= (float)(n[a] - 1 + r)))
            return;
    }
    int32_t qi[3] = {(int32_t)q[0], (int32_t)q[1], (int32_t)q[2]};
    for (int32_t i = qi[0] - r; i <= qi[0] + r; ++i)
        for (int32_t j = qi[1] - r; j <= qi[1] + r; ++j)
            for (int32_t k = qi[2] - r; k <= qi[2] + r; ++k)
                if (inside(gx, gy, gz, i, j, k))
                    ms[lin(gx, gy, i, j, k)] = OG_OCCUPIED;
}

/* --------------------------------------------- Alg. 2: ray trace (IV-C) */

/* R18: a voxel reached after a hit becomes "unknown and traced" whatever other
 * rays wrote; "free" only lands on a voxel no ray has marked yet; occupied
 * voxels are never written by rays. */
static void mark(uint8_t *ms, int64_t idx, uint8_t val)
{
    if (val == OG_TRACED)
        ms[idx] = OG_TRACED;
    else if (ms[idx] == OG_UNKNOWN)
        ms[idx] = OG_FREE;
}

/* One walk of Alg. 2.  Optional outputs: the visited voxels and the value
 * assigned to each (og_trace_ray), and the number of in-grid voxels. */
static int64_t walk(const float o[3], const float dir[3], int64_t m2,
                    int32_t gx, int32_t gy, int32_t gz, uint8_t *ms,
                    int32_t *out_xyz, uint8_t *out_val, int64_t max_out, int64_t *in_grid,
                    int64_t *after_hit)
{
    /* R12: start voxel = floor of the camera position in voxel units. */
    int32_t v0[3], v[3], step[3];
    float tmax[3], tdelta[3];
    for (int a = 0; a < 3; ++a) {
        v0[a] = (int32_t)floorf(o[a]);
        v[a] = v0[a];
        /* R13: Amanatides & Woo initialisation, per axis. */
        if (dir[a] > 0.0f) {
            step[a] = 1;
            tmax[a] = ((float)(v0[a] + 1) - o[a]) / dir[a];
            tdelta[a] = 1.0f / dir[a];
        } else if (dir[a] < 0.0f) {
            step[a] = -1;
            tmax[a] = ((float)v0[a] - o[a]) / dir[a];
            tdelta[a] = -1.0f / dir[a];
        } else {
            step[a] = 0;
            tmax[a] = INFINITY;
            tdelta[a] = INFINITY;
        }
    }

    uint8_t vox_val = OG_FREE;   /* Alg. 2: vox_val <- free */
    int64_t d2 = 0;              /* R15: squared lattice distance from v0 */
    int64_t nsteps = 0, ingrid = 0, post = 0;
    while (d2 < m2) {
        /* R13: move by one voxel along the axis whose boundary is nearest;
         * on ties the later axis wins.  R14: the start voxel is never
         * processed, because the walk moves before it tests. */
        int a = tmax[0] < tmax[1] ? (tmax[0] < tmax[2] ? 0 : 2) : (tmax[1] < tmax[2] ? 1 : 2);
        if (step[a] == 0)
            break;               /* zero direction: no voxel boundary is ever reached */
        v[a] += step[a];
        tmax[a] += tdelta[a];

        uint8_t assigned = OG_OUTSIDE;
        if (inside(gx, gy, gz, v[0], v[1], v[2])) {       /* R17 */
            int64_t idx = lin(gx, gy, v[0], v[1], v[2]);
            ++ingrid;
            post += vox_val == OG_TRACED;
            /* R16: the occupancy test reads this measurement's grid. */
            if (ms && ms[idx] == OG_OCCUPIED) {
                vox_val = OG_TRACED;                       /* Alg. 2: after the hit */
                assigned = OG_OCCUPIED;
            } else {
                if (ms)
                    mark(ms, idx, vox_val);
                assigned = vox_val;
            }
        }
        if (out_xyz && nsteps < max_out) {
            out_xyz[3 * nsteps + 0] = v[0];
            out_xyz[3 * nsteps + 1] = v[1];
            out_xyz[3 * nsteps + 2] = v[2];
        }
        if (out_val && nsteps < max_out)
            out_val[nsteps] = assigned;
        ++nsteps;

        /* R15: traversed distance as an integer squared norm from v0. */
        int64_t dx = v[0] - v0[0], dy = v[1] - v0[1], dz = v[2] - v0[2];
        d2 = dx * dx + dy * dy + dz * dz;
    }
    if (in_grid)
        *in_grid += ingrid;
    if (after_hit)
        *after_hit += post;
    return nsteps;
}

int64_t og_trace_ray(const float o[3], const float dir[3], int64_t m2,
                     int32_t gx, int32_t gy, int32_t gz, uint8_t *ms,
                     int32_t *out_xyz, uint8_t *out_val, int64_t max_out)
{
    for (int a = 0; a < 3; ++a)
        if (!(fabsf(o[a]) < 16777216.0f) || !isfinite(dir[a]))
            return -1;
    return walk(o, dir, m2, gx, gy, gz, ms, out_xyz, out_val, max_out, NULL, NULL);
}

/* ------------------------------------------ Alg. 3: update local grid (IV-D) */

void og_merge(int64_t n, const uint8_t *ms, uint8_t *loc)
{
    for (int64_t i = 0; i < n; ++i) {
        if (ms[i] != OG_UNKNOWN) {
            /* R19: "unknown and traced" is stored in loc as unknown. */
            loc[i] = ms[i] == OG_TRACED ? OG_UNKNOWN : ms[i];
        }
    }
}

/* ------------------------------------------------------ shared frame driver */

typedef struct {
    int32_t gx, gy, gz;
    float vox_size;
    int32_t vox_inf;
    float tv[3];
    const float *R;
    uint8_t *ms;
    int64_t after_hit;   /* in-grid walk steps after the ray's first hit */
} frame_ctx;

static int check_grid(int32_t gx, int32_t gy, int32_t gz, float vox_size, int32_t vox_inf)
{
    if (gx < 1 || gy < 1 || gz < 1)
        return -1;
    if ((int64_t)gx * gy * gz >= ((int64_t)1 << 31))
        return -1;
    if (!(vox_size > 0.0f) || !isfinite(vox_size) || vox_inf < 0 || vox_inf > 64)
        return -1;
    return 0;
}

static void point_to_grid(frame_ctx *f, const float pc[3])
{
    float q[3];
    og_quantize(f->R, f->tv, f->vox_size, pc, q);
    add_occ(f->gx, f->gy, f->gz, f->vox_inf, q, f->ms);
}

/* Step 3 for the pinhole fan of Sec. IV-C: targets (x_i, y_i, vox_depth) with
 * |x_i| <= hw, |y_i| <= hh, each ray cut at the target's own length (R15). */
static int64_t trace_pinhole_fan(frame_ctx *f, int32_t vd, int32_t hw, int32_t hh)
{
    float o[3], dir[3], tgt[3];
    int64_t steps = 0;
    for (int a = 0; a < 3; ++a)
        o[a] = f->tv[a] / f->vox_size;     /* R12: p^v_c in voxel units */
    for (int32_t yi = -hh; yi <= hh; ++yi) {
        for (int32_t xi = -hw; xi <= hw; ++xi) {
            tgt[0] = (float)xi;
            tgt[1] = (float)yi;
            tgt[2] = (float)vd;
            rotate(f->R, tgt, dir);        /* Alg. 2: ray direction, R11 */
            int64_t m2 = (int64_t)xi * xi + (int64_t)yi * yi + (int64_t)vd * vd;
            walk(o, dir, m2, f->gx, f->gy, f->gz, f->ms, NULL, NULL, 0, &steps, &f->after_hit);
        }
    }
    return steps;
}

static void finish_frame(frame_ctx *f, uint8_t *loc, uint8_t *ms_out, int64_t rays,
                         int64_t steps, int64_t stats[5])
{
    int64_t n = (int64_t)f->gx * f->gy * f->gz;
    int64_t upd = 0, occ = 0;
    for (int64_t i = 0; i < n; ++i) {
        upd += f->ms[i] != OG_UNKNOWN;
        occ += f->ms[i] == OG_OCCUPIED;
    }
    if (ms_out)
        memcpy(ms_out, f->ms, (size_t)n);
    og_merge(n, f->ms, loc);              /* step 4 */
    if (stats) {
        stats[0] = upd;
        stats[1] = steps;
        stats[2] = occ;
        stats[3] = rays;
        stats[4] = f->after_hit;
    }
}

static int start_frame(frame_ctx *f, int32_t gx, int32_t gy, int32_t gz, float vox_size,
                       const float origin[3], int32_t vox_inf, const float R[9], const float t[3])
{
    if (check_grid(gx, gy, gz, vox_size, vox_inf))
        return -1;
    for (int i = 0; i < 9; ++i)
        if (!isfinite(R[i]))
            return -1;
    for (int a = 0; a < 3; ++a)
        if (!isfinite(t[a]) || !isfinite(origin[a]))
            return -1;
    f->gx = gx;
    f->gy = gy;
    f->gz = gz;
    f->vox_size = vox_size;
    f->vox_inf = vox_inf;
    f->R = R;
    f->after_hit = 0;
    grid_translation(t, origin, f->tv);
    /* Integer voxel coordinates of the camera must stay far from int32 limits. */
    for (int a = 0; a < 3; ++a)
        if (!(fabsf(f->tv[a] / vox_size) < 16777216.0f))
            return -1;
    /* Step 1 (Sec. IV-A): the measurement grid starts all unknown. */
    f->ms = (uint8_t *)calloc((size_t)gx * gy * gz, 1);
    return f->ms ? 0 : -1;
}

/* ------------------------------------------------------------ entry points */

int og_integrate_pinhole(int32_t gx, int32_t gy, int32_t gz, float vox_size,
                         const float origin[3], int32_t vox_inf,
                         uint8_t *loc, uint8_t *ms_out,
                         const float *depth, int32_t width, int32_t height,
                         double fx, double fy, double cx, double cy,
                         double fov_x, double fov_y, float depth_min, float depth_max,
                         const float R[9], const float t[3], int64_t stats[5])
{
    int32_t fan[3];
    if (width < 0 || height < 0 || og_fan_sizes(depth_max, vox_size, fov_x, fov_y, fan))
        return -1;
    frame_ctx f;
    if (start_frame(&f, gx, gy, gz, vox_size, origin, vox_inf, R, t))
        return -1;

    /* Step 2, Alg. 1, one depth pixel at a time. */
    for (int32_t v = 0; v < height; ++v) {
        /* R5: pixel ray slopes, computed in double and rounded once. */
        float kv = (float)(((double)v - cy) / fy);
        for (int32_t u = 0; u < width; ++u) {
            float d = depth[(int64_t)v * width + u];
            if (!(d >= depth_min && d <= depth_max))      /* R3 */
                continue;
            float ku = (float)(((double)u - cx) / fx);
            float pc[3] = {d * ku, d * kv, d};            /* R4, R6: z-depth */
            point_to_grid(&f, pc);
        }
    }

    /* Step 3, Alg. 2 over the bundled fan. */
    int64_t steps = trace_pinhole_fan(&f, fan[0], fan[1], fan[2]);
    int64_t rays = (2 * (int64_t)fan[1] + 1) * (2 * (int64_t)fan[2] + 1);
    finish_frame(&f, loc, ms_out, rays, steps, stats);
    free(f.ms);
    return 0;
}

int og_integrate_points(int32_t gx, int32_t gy, int32_t gz, float vox_size,
                        const float origin[3], int32_t vox_inf,
                        uint8_t *loc, uint8_t *ms_out,
                        const float *points, int64_t n_points,
                        double fov_x, double fov_y, float depth,
                        const float R[9], const float t[3], int64_t stats[5])
{
    int32_t fan[3];
    if (n_points < 0 || og_fan_sizes(depth, vox_size, fov_x, fov_y, fan))
        return -1;
    frame_ctx f;
    if (start_frame(&f, gx, gy, gz, vox_size, origin, vox_inf, R, t))
        return -1;
    for (int64_t i = 0; i < n_points; ++i) {
        const float *p = points + 3 * i;
        /* A point cloud entry is a measurement iff all coordinates are finite. */
        if (!(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2])))
            continue;
        point_to_grid(&f, p);
    }
    int64_t steps = trace_pinhole_fan(&f, fan[0], fan[1], fan[2]);
    int64_t rays = (2 * (int64_t)fan[1] + 1) * (2 * (int64_t)fan[2] + 1);
    finish_frame(&f, loc, ms_out, rays, steps, stats);
    free(f.ms);
    return 0;
}

int og_integrate_spinning(int32_t gx, int32_t gy, int32_t gz, float vox_size,
                          const float origin[3], int32_t vox_inf,
                          uint8_t *loc, uint8_t *ms_out,
                          const float *range, int32_t width, int32_t height,
                          const float *col_tab, const float *row_tab,
                          double vfov, float depth_min, float depth_max,
                          const float R[9], const float t[3], int64_t stats[5])
{
    double vd_d = round_half_away((double)depth_max / (double)vox_size);   /* R9 */
    if (!(vd_d >= 1.0 && vd_d <= 16384.0) || !(vfov > 0.0 && vfov < 3.14159))
        return -1;
    int32_t vd = (int32_t)vd_d;
    frame_ctx f;
    if (start_frame(&f, gx, gy, gz, vox_size, origin, vox_inf, R, t))
        return -1;

    /* Step 2 (R27): sensor frame z up; elevation per row, azimuth per column. */
    for (int32_t v = 0; v < height; ++v) {
        float ce = row_tab[2 * v + 0], se = row_tab[2 * v + 1];
        for (int32_t u = 0; u < width; ++u) {
            float rho = range[(int64_t)v * width + u];
            if (!(rho >= depth_min && rho <= depth_max))
                continue;
            float ca = col_tab[2 * u + 0], sa = col_tab[2 * u + 1];
            float horiz = rho * ce;
            float pc[3] = {horiz * ca, horiz * sa, rho * se};
            point_to_grid(&f, pc);
        }
    }

    /* Step 3 (R27): one ray per lattice target on the square ring of half side
     * vox_depth, inside the vertical fov; every ray is cut at vox_depth. */
    double thv = tan(vfov / 2.0);
    float o[3], dir[3], tgt[3];
    for (int a = 0; a < 3; ++a)
        o[a] = f.tv[a] / f.vox_size;
    int64_t steps = 0, rays = 0, m2 = (int64_t)vd * vd;
    for (int32_t c = 0; c < 8 * vd; ++c) {
        int32_t x, y;
        spin_column(c, vd, &x, &y);
        int32_t hz = spin_half_height(x, y, thv);
        for (int32_t z = -hz; z <= hz; ++z) {
            tgt[0] = (float)x;
            tgt[1] = (float)y;
            tgt[2] = (float)z;
            rotate(R, tgt, dir);
            walk(o, dir, m2, gx, gy, gz, f.ms, NULL, NULL, 0, &steps, &f.after_hit);
            ++rays;
        }
    }
    finish_frame(&f, loc, ms_out, rays, steps, stats);
    free(f.ms);
    return 0;
}

/* -------------------------------------------------------- shift (IV-E) */

void og_shift(int32_t gx, int32_t gy, int32_t gz, const uint8_t *in, uint8_t *out,
              int32_t dx, int32_t dy, int32_t dz)
{
    for (int32_t z = 0; z < gz; ++z)
        for (int32_t y = 0; y < gy; ++y)
            for (int32_t x = 0; x < gx; ++x) {
                int64_t sx = (int64_t)x + dx, sy = (int64_t)y + dy, sz = (int64_t)z + dz;
                uint8_t val = OG_UNKNOWN;   /* newly exposed voxels are unknown */
                if (sx >= 0 && sy >= 0 && sz >= 0 && sx < gx && sy < gy && sz < gz)
                    val = in[lin(gx, gy, (int32_t)sx, (int32_t)sy, (int32_t)sz)];
                out[lin(gx, gy, x, y, z)] = val;
            }
}

void og_center_offset(int32_t gx, int32_t gy, int32_t gz, float vox_size,
                      const float origin[3], const float t_w_c[3], int32_t delta[3])
{
    const int32_t n[3] = {gx, gy, gz};
    for (int a = 0; a < 3; ++a) {
        float rel = t_w_c[a] - origin[a];
        float c = floorf(rel / vox_size);
        delta[a] = (int32_t)c - n[a] / 2;
    }
}

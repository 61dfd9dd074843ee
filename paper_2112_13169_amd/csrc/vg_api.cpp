// vg_api.cpp -- host side of the C ABI declared in include/vg.h:
// argument validation, the host-computed per-frame constants (T^v_c, the ray
// fan sizes of Sec. IV-C, the camera voxel), scratch layout and launches.
#include "../../include/vg.h"
#include "vg_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#pragma clang fp contract(off)

using namespace vg;

namespace {

constexpr size_t kAlign = 256;
constexpr int32_t kMaxFan = 16384;
constexpr size_t kHzBytes = (size_t)8 * kMaxFan * sizeof(int32_t);

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Scratch layout of one plane set (all offsets 256-aligned):
//   seed      seed stamps on the grid padded by vox_inf, rows of seed_pitch bytes
//   bitx      seeds dilated along x, one 32-bit word per 32 voxels of a padded row
//   occ       occupied voxels of the frame, one bit per device-layout voxel
//   marks     free stamps, then "unknown and traced" stamps, one byte per
//             device-layout voxel each
//   hz        spinning fan: half height per ring column
//   lim       the frame's row regions (vg_frustum.h), written by its seed pass
struct Layout {
    int32_t gxp, wx, py, pz, seed_pitch;
    size_t seed, bitx, occ, marks, hz, lim, order, fixed;
};

Layout layout_for(int32_t gx, int32_t gy, int32_t gz, int32_t r)
{
    Layout l;
    l.gxp = grid_pitch(gx);
    l.wx = l.gxp / 32;
    l.py = gy + 2 * r;
    l.pz = gz + 2 * r;
    l.seed_pitch = (32 * l.wx + 64 + 63) / 64 * 64;
    l.seed = 0;
    l.bitx = l.seed + align_up((size_t)l.seed_pitch * l.py * l.pz);
    l.occ = l.bitx + align_up((size_t)4 * l.wx * l.py * l.pz);
    l.marks = l.occ + align_up((size_t)4 * l.wx * gy * gz);
    l.hz = l.marks + align_up((size_t)2 * l.gxp * gy * gz);
    l.lim = l.hz + kHzBytes;
    l.order = l.lim + align_up(sizeof(RowLimits));
    l.fixed = l.order + align_up(kOrderBytes);
    return l;
}

double round_half_away(double v) { return v < 0.0 ? -std::floor(-v + 0.5) : std::floor(v + 0.5); }

struct Fan {
    int32_t vd = 0, hw = 0, hh = 0;   // hh: largest half height for spinning fans
    int64_t rays = 0;
    std::vector<int32_t> hz;          // spinning only
};

// Sec. IV-C: vox_depth = depth / vox_size rounded; the half width / height of
// the fan is tan(fov/2) * vox_depth rounded, so the full sizes are odd.  A
// spinning fan (no pinhole fov) uses every lattice column on the square ring
// of half side vox_depth, each as high as tan(vfov/2) times its distance.
bool fan_for(const vg_sensor &s, float vox_size, Fan &f)
{
    double vd = round_half_away((double)s.depth / (double)vox_size);
    if (!(vd >= 1.0 && vd <= kMaxFan))
        return false;
    f.vd = (int32_t)vd;
    if (s.kind == VG_SPINNING) {
        if (!(s.fov_y > 0.0 && s.fov_y < 3.14159))
            return false;
        const double thv = std::tan(s.fov_y / 2.0);
        f.hz.resize((size_t)8 * f.vd);
        f.rays = 0;
        f.hh = 0;
        f.hw = 0;
        for (int32_t c = 0; c < 8 * f.vd; ++c) {
            int32_t side = c / (2 * f.vd), k = c % (2 * f.vd), x, y;
            if (side == 0) {
                x = f.vd;
                y = -f.vd + 1 + k;
            } else if (side == 1) {
                x = f.vd - 1 - k;
                y = f.vd;
            } else if (side == 2) {
                x = -f.vd;
                y = f.vd - 1 - k;
            } else {
                x = -f.vd + 1 + k;
                y = -f.vd;
            }
            double h = round_half_away(thv * std::sqrt((double)x * x + (double)y * y));
            if (!(h >= 0.0 && h <= kMaxFan))
                return false;
            f.hz[c] = (int32_t)h;
            if (f.hz[c] > f.hh)
                f.hh = f.hz[c];
            f.rays += 2 * (int64_t)f.hz[c] + 1;
        }
        return true;
    }
    if (!(s.fov_x > 0.0 && s.fov_x < 3.14159 && s.fov_y > 0.0 && s.fov_y < 3.14159))
        return false;
    double hw = round_half_away(std::tan(s.fov_x / 2.0) * vd);
    double hh = round_half_away(std::tan(s.fov_y / 2.0) * vd);
    if (!(hw >= 0.0 && hw <= kMaxFan && hh >= 0.0 && hh <= kMaxFan))
        return false;
    f.hw = (int32_t)hw;
    f.hh = (int32_t)hh;
    f.rays = (2 * (int64_t)f.hw + 1) * (2 * (int64_t)f.hh + 1);
    return true;
}

bool finite_pose(const vg_pose *T)
{
    for (float v : T->R)
        if (!std::isfinite(v))
            return false;
    for (float v : T->t)
        if (!std::isfinite(v))
            return false;
    return true;
}

}  // namespace

struct vg_grid {
    int32_t n[3];
    float s;
    float base[3];
    int32_t shift[3];
    int32_t r;
    uint8_t *loc;            // ring buffer of the local grid
    int32_t ring[3];         // its ring offsets
    uint8_t *scratch;
    size_t scratch_bytes;
    Layout lay;
    uint32_t epoch;          // stamp of the last frame, 0 = none yet
    int device;
    int32_t sets = 1;        // plane sets in scratch, lay.fixed bytes apart
    // spinning fan table currently in each set
    int32_t hz_vd[kMaxPlaneSets] = {};
    double hz_fov[kMaxPlaneSets] = {};
    int32_t tile_log2w = 3;  // ray tiles of (1 << tile_log2w) x (64 >> tile_log2w) targets
    // measurement hook: sets of kStages (start, stop) pairs, one set per frame
    std::vector<StageEvents> prof;
    uint64_t prof_next = 0;
};

namespace {

// Stages timed by the measurement hook, in the order of a set's event pairs.
enum { kStageSeed, kStageDilate, kStageRays, kStageResolve, kStageShift, kStages };

// The event pairs of the frame in turn (the set a vg_shift_grid call uses is
// that of the frame that follows it), or null when recording is off.
const StageEvents *stage_events(const vg_grid *g)
{
    if (g->prof.empty())
        return nullptr;
    const size_t sets = g->prof.size() / kStages;
    return &g->prof[kStages * (size_t)(g->prof_next % sets)];
}

vg_status hip_status(hipError_t e) { return e == hipSuccess ? VG_OK : VG_ERR_HIP; }

bool same_device(const vg_grid *g)
{
    int d = -1;
    return hipGetDevice(&d) == hipSuccess && d == g->device;
}

// Origin after integer shifts: base + (float)shift * vox_size (no drift).
void current_origin(const vg_grid *g, float o[3])
{
    for (int a = 0; a < 3; ++a) {
        float off = (float)g->shift[a] * g->s;
        o[a] = g->base[a] + off;
    }
}

bool valid_sensor(const vg_sensor *s)
{
    if (!s)
        return false;
    if (s->kind != VG_PINHOLE && s->kind != VG_SPINNING)
        return false;
    if (s->width < 0 || s->height < 0 || s->width > 65535 || s->height > 65535)
        return false;
    if (!std::isfinite(s->depth) || !(s->depth > 0.0f) || std::isnan(s->depth_min))
        return false;
    if (s->kind == VG_PINHOLE) {
        if (!(std::isfinite(s->fx) && std::isfinite(s->fy) && s->fx != 0.0 && s->fy != 0.0 &&
              std::isfinite(s->cx) && std::isfinite(s->cy)))
            return false;
    } else if (s->width > 0 && s->height > 0 && (!s->col_tab || !s->row_tab)) {
        return false;
    }
    return true;
}

// Padded-coordinate box that holds every seed a frame can produce, from the
// sensor's frustum (pinhole: the 8 corners of the depth range over the image;
// spinning: a ball of the largest range), widened by a bound on the fp32
// rounding of the device's transform.  Points: the whole padded grid.
void seed_box(const vg_grid *g, int kind, const vg_sensor &s, const vg_pose &T,
              const float tv[3], int32_t lo[3], int32_t hi[3])
{
    const int32_t r = g->r;
    for (int a = 0; a < 3; ++a) {
        lo[a] = 0;
        hi[a] = g->n[a] - 1 + 2 * r;
    }
    if (kind == kPoints || !std::isfinite(s.depth_min))
        return;
    if (s.width == 0 || s.height == 0 || s.depth_min > s.depth) {
        lo[0] = 1;
        hi[0] = 0;   // no measurement can exist
        return;
    }
    double qmin[3], qmax[3], mag = 0.0, tmag = 0.0;
    for (int a = 0; a < 3; ++a) {
        qmin[a] = INFINITY;
        qmax[a] = -INFINITY;
        tmag = std::max(tmag, std::fabs((double)tv[a]));
    }
    if (kind == kPinhole) {
        const double ku[2] = {(0.0 - s.cx) / s.fx, ((double)s.width - 1.0 - s.cx) / s.fx};
        const double kv[2] = {(0.0 - s.cy) / s.fy, ((double)s.height - 1.0 - s.cy) / s.fy};
        const double dd[2] = {(double)s.depth_min, (double)s.depth};
        for (double d : dd)
            for (double u : ku)
                for (double v : kv) {
                    const double pc[3] = {d * u, d * v, d};
                    double m = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        double pv = (double)tv[a];
                        for (int j = 0; j < 3; ++j) {
                            pv += (double)T.R[3 * a + j] * pc[j];
                            m += std::fabs((double)T.R[3 * a + j] * pc[j]);
                        }
                        qmin[a] = std::min(qmin[a], pv / g->s);
                        qmax[a] = std::max(qmax[a], pv / g->s);
                    }
                    mag = std::max(mag, m);
                }
    } else {
        const double rho = std::max(std::fabs((double)s.depth_min), std::fabs((double)s.depth));
        for (int a = 0; a < 3; ++a) {
            double ext = 0.0;
            for (int j = 0; j < 3; ++j)
                ext += std::fabs((double)T.R[3 * a + j]) * rho * 1.0001;
            qmin[a] = ((double)tv[a] - ext) / g->s;
            qmax[a] = ((double)tv[a] + ext) / g->s;
            mag = std::max(mag, 3.0 * ext);
        }
    }
    const double slack = 4.0 + 4e-6 * (mag + tmag) / g->s;
    for (int a = 0; a < 3; ++a) {
        double l = std::floor(qmin[a] - slack) + r, h = std::floor(qmax[a] + slack) + r;
        l = std::max(l, 0.0);
        h = std::min(h, (double)(g->n[a] - 1 + 2 * r));
        if (!(l <= h)) {
            lo[0] = 1;
            hi[0] = 0;
            return;
        }
        lo[a] = (int32_t)l;
        hi[a] = (int32_t)h;
    }
}

// Rows of the grid the ray fan can reach: the fan is the pyramid with apex at
// the camera and the targets as base (a ball of radius vox_depth for a
// spinning fan); a walk ends within one voxel of its target's length, and
// every voxel it visits touches the ray.  The box of the pyramid scaled by
// (1 + 3 / vox_depth), widened by 3 voxels, holds all of them.
RowBox fan_rows(const vg_grid *g, int kind, const Fan &fan, const vg_pose &T, const float o[3])
{
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a)
        lo[a] = hi[a] = (double)o[a];
    if (kind == kSpinning) {
        for (int a = 0; a < 3; ++a) {
            lo[a] -= fan.vd + 3.0;
            hi[a] += fan.vd + 3.0;
        }
    } else {
        const double k = 1.0 + 3.0 / fan.vd;
        for (int sa = -1; sa <= 1; sa += 2)
            for (int sb = -1; sb <= 1; sb += 2) {
                const double t[3] = {(double)sa * fan.hw * k, (double)sb * fan.hh * k,
                                     (double)fan.vd * k};
                for (int a = 0; a < 3; ++a) {
                    double c = (double)o[a];
                    for (int j = 0; j < 3; ++j)
                        c += (double)T.R[3 * a + j] * t[j];
                    lo[a] = std::min(lo[a], c);
                    hi[a] = std::max(hi[a], c);
                }
            }
        for (int a = 0; a < 3; ++a) {
            lo[a] -= 3.0;
            hi[a] += 3.0;
        }
    }
    RowBox b;
    b.y0 = (int32_t)std::max(std::floor(lo[1]), 0.0);
    b.y1 = (int32_t)std::min(std::floor(hi[1]), (double)(g->n[1] - 1));
    b.z0 = (int32_t)std::max(std::floor(lo[2]), 0.0);
    b.z1 = (int32_t)std::min(std::floor(hi[2]), (double)(g->n[2] - 1));
    if (std::floor(hi[0]) < 0.0 || std::floor(lo[0]) > g->n[0] - 1)
        b.y0 = 1, b.y1 = 0;
    return b;
}

RowBox row_union(const RowBox &a, const RowBox &b)
{
    const bool ea = a.y0 > a.y1 || a.z0 > a.z1, eb = b.y0 > b.y1 || b.z0 > b.z1;
    if (ea)
        return b;
    if (eb)
        return a;
    return RowBox{std::min(a.y0, b.y0), std::max(a.y1, b.y1), std::min(a.z0, b.z0),
                  std::max(a.z1, b.z1)};
}

// Grid state a frame's plan depends on; a batch advances a copy of it frame
// by frame and writes it back only when every frame has been planned.
struct GridState {
    int32_t shift[3];
    int32_t ring[3];
    uint32_t epoch;
    int32_t hz_vd[kMaxPlaneSets];
    double hz_fov[kMaxPlaneSets];
};

GridState state_of(const vg_grid *g)
{
    GridState s;
    std::memcpy(s.shift, g->shift, sizeof s.shift);
    std::memcpy(s.ring, g->ring, sizeof s.ring);
    s.epoch = g->epoch;
    std::memcpy(s.hz_vd, g->hz_vd, sizeof s.hz_vd);
    std::memcpy(s.hz_fov, g->hz_fov, sizeof s.hz_fov);
    return s;
}

void store_state(vg_grid *g, const GridState &s)
{
    std::memcpy(g->shift, s.shift, sizeof s.shift);
    std::memcpy(g->ring, s.ring, sizeof s.ring);
    g->epoch = s.epoch;
    std::memcpy(g->hz_vd, s.hz_vd, sizeof s.hz_vd);
    std::memcpy(g->hz_fov, s.hz_fov, sizeof s.hz_fov);
}

// No fan table in any set: the next spinning frame writes its own.
void forget_fan_tables(vg_grid *g)
{
    for (int k = 0; k < kMaxPlaneSets; ++k) {
        g->hz_vd[k] = 0;
        g->hz_fov[k] = -1.0;
    }
}

// Step 5 on the ring buffer (Sec. IV-E): grid coordinate x now holds what
// x + d held, so the ring offsets move by d and the coordinates whose source
// lay outside the grid -- [n - d, n) for d > 0, [0, -d) for d < 0 -- are
// cleared.  Fills `c` (loc excepted) and moves the state's offsets and shift.
void plan_shift(const vg_grid *g, GridState &gs, const int32_t d[3], SlabClear &c)
{
    for (int a = 0; a < 3; ++a) {
        const int32_t n = g->n[a];
        int64_t r = ((int64_t)gs.ring[a] + d[a]) % n;
        if (r < 0)
            r += n;
        gs.ring[a] = (int32_t)r;
        gs.shift[a] += d[a];
        c.n[a] = n;
        c.ring[a] = gs.ring[a];
        if (d[a] > 0) {
            c.lo[a] = (int32_t)std::max<int64_t>((int64_t)n - d[a], 0);
            c.hi[a] = n;
        } else if (d[a] < 0) {
            c.lo[a] = 0;
            c.hi[a] = (int32_t)std::min<int64_t>(-(int64_t)d[a], n);
        } else {
            c.lo[a] = c.hi[a] = 0;
        }
    }
    c.gxp = g->lay.gxp;
    // a shift past the grid on some axis clears everything: restart the ring
    // at 0 (the plain layout keeps the merge on its aligned path)
    bool all = false;
    for (int a = 0; a < 3; ++a)
        all = all || (c.hi[a] - c.lo[a] >= c.n[a]);
    if (all)
        for (int a = 0; a < 3; ++a)
            gs.ring[a] = c.ring[a] = 0;
    // lanes: the buffer chunks of the exposed x slab in every row (all of
    // them when everything is cleared), the rows of the y and z slabs whole
    const int32_t cpr = c.gxp / 16;
    for (int k = 0; k < 4; ++k)
        c.xrun[k] = 0;
    if (all) {
        c.lo[0] = 0;
        c.hi[0] = c.n[0];
        c.xrun[1] = cpr;
    } else if (c.lo[0] < c.hi[0]) {
        const int32_t b0 = (c.lo[0] + c.ring[0]) % c.n[0], len = c.hi[0] - c.lo[0];
        if (b0 + len <= c.n[0]) {
            c.xrun[0] = b0 / 16;
            c.xrun[1] = (b0 + len - 1) / 16 + 1;
        } else {
            c.xrun[0] = b0 / 16;
            c.xrun[1] = (c.n[0] - 1) / 16 + 1;
            c.xrun[2] = 0;
            c.xrun[3] = (b0 + len - c.n[0] - 1) / 16 + 1;
        }
    }
    const int64_t rows = (int64_t)c.n[1] * c.n[2];
    c.lanes[0] = rows * ((c.xrun[1] - c.xrun[0]) + (c.xrun[3] - c.xrun[2]));
    c.lanes[1] = all ? 0 : (int64_t)(c.hi[1] - c.lo[1]) * c.n[2] * cpr;
    c.lanes[2] = all ? 0 : (int64_t)(c.hi[2] - c.lo[2]) * c.n[1] * cpr;
}

// What the seed pass needs to compute the regions of vg_frustum.h for one
// frame: the pinhole fan (images and point clouds), and the image's pyramid
// for pinhole images whose valid depths are not negative.  The corner
// pixels' slopes are the fp32 slopes the seed pass uses (rounding is
// monotonic, so every pixel's lies between).
void region_inputs(int kind, const vg_sensor &s, const Fan &fan, int32_t W, int32_t H,
                   SeedParams &sp)
{
    sp.vd = fan.vd;
    sp.hw = fan.hw;
    sp.hh = fan.hh;
    sp.lim_fan = kind != kSpinning ? 1 : 0;
    sp.lim_img = kind == kPinhole && s.depth_min >= 0.0f && W > 0 && H > 0 ? 1 : 0;
    float ku[2] = {0.0f, 0.0f}, kv[2] = {0.0f, 0.0f};
    if (sp.lim_img) {
        ku[0] = (float)((0.0 - s.cx) / s.fx);
        ku[1] = (float)(((double)W - 1.0 - s.cx) / s.fx);
        kv[0] = (float)((0.0 - s.cy) / s.fy);
        kv[1] = (float)(((double)H - 1.0 - s.cy) / s.fy);
    }
    sp.lim_k[0] = std::min(ku[0], ku[1]);
    sp.lim_k[1] = std::max(ku[0], ku[1]);
    sp.lim_k[2] = std::min(kv[0], kv[1]);
    sp.lim_k[3] = std::max(kv[0], kv[1]);
}

// Host plan of steps 2-4 for one frame: every per-frame constant and launch
// size.  Nothing is launched and no state changes.
struct FramePlan {
    int kind;
    Fan fan;
    SeedParams sp;
    RayParams rp;
    RowBox rows;
    bool inside;
    bool wrap;        // the stamp planes must be cleared first (stamp wrapped)
    bool upload_hz;   // the spinning fan table must be (re)written
    bool direct;      // occupied cubes stamped directly into bytes (no dilation)
    int32_t set;      // plane set of the grid's scratch the frame uses
    uint32_t epoch;
    int32_t ring[3];  // ring offsets of the grid when the frame merges
};

// Stamping each point's (2 vox_inf + 1)^3 cube directly costs that many
// byte stores per point; the separable dilation costs three launches over the
// seed box.  Frames whose points times cube stay below this stamp directly
// (one launch) when walked one per call.
constexpr int64_t kDirectStores = 16 << 20;

vg_status plan_frame(const vg_grid *g, const GridState &gs, int kind, const float *data,
                     int64_t pitch_floats, int32_t W, int32_t H, const vg_sensor *sensor,
                     const vg_pose *T, FramePlan &p, bool allow_direct = false, int32_t set = 0)
{
    p.kind = kind;
    p.set = set;
    uint8_t *const sc = g->scratch + (size_t)set * g->lay.fixed;   // the set's planes
    if (!fan_for(*sensor, g->s, p.fan))
        return VG_ERR_ARG;
    if ((W > 0 && H > 0) && !data)
        return VG_ERR_ARG;
    const Fan &fan = p.fan;

    // T^v_c = T^v_w T^w_c: the grid frame is the world frame translated by
    // -origin (axes aligned), so R is unchanged and t^v = t^w_c - origin.
    float origin[3], tv[3], o[3];
    int32_t v0[3];
    for (int a = 0; a < 3; ++a) {
        float off = (float)gs.shift[a] * g->s;
        origin[a] = g->base[a] + off;
    }
    for (int a = 0; a < 3; ++a) {
        tv[a] = T->t[a] - origin[a];
        o[a] = tv[a] / g->s;   // camera position in voxel units
        if (!(std::fabs(o[a]) < 16777216.0f))
            return VG_ERR_ARG;
        v0[a] = (int32_t)std::floor(o[a]);
    }
    // fan tiles of tw x th targets, one wavefront each
    const int32_t tw = 1 << g->tile_log2w, th = 64 >> g->tile_log2w;
    const int32_t fan_a = kind == kSpinning ? 8 * fan.vd : 2 * fan.hw + 1;
    const int32_t fan_b = 2 * fan.hh + 1;
    const int64_t tiles = (int64_t)((fan_a + tw - 1) / tw) * ((fan_b + th - 1) / th);
    if (tiles * 64 > (int64_t)0x7fffffff)
        return VG_ERR_ARG;

    // Per-frame stamp 1..255; the stamp planes are cleared when it wraps.
    p.wrap = gs.epoch == 255;
    p.epoch = p.wrap ? 1 : gs.epoch + 1;
    p.upload_hz =
        kind == kSpinning && (gs.hz_vd[set] != fan.vd || gs.hz_fov[set] != sensor->fov_y);
    std::memcpy(p.ring, gs.ring, sizeof p.ring);

    Planes pl;
    std::memcpy(pl.n, g->n, sizeof pl.n);
    pl.r = g->r;
    pl.wx = g->lay.wx;
    pl.py = g->lay.py;
    pl.pz = g->lay.pz;
    pl.seed_pitch = g->lay.seed_pitch;
    pl.seed = sc + g->lay.seed;
    pl.bitx = reinterpret_cast<uint32_t *>(sc + g->lay.bitx);
    pl.occ = reinterpret_cast<uint32_t *>(sc + g->lay.occ);
    pl.marks = sc + g->lay.marks;
    pl.nbytes = (uint32_t)((size_t)g->lay.gxp * g->n[1] * g->n[2]);
    seed_box(g, kind, *sensor, *T, tv, pl.lo, pl.hi);
    pl.epoch = p.epoch;
    pl.lim = reinterpret_cast<const RowLimits *>(sc + g->lay.lim);
    const int64_t side = 2 * g->r + 1;
    p.direct = allow_direct && (int64_t)W * H * side * side * side <= kDirectStores;
    pl.occb = p.direct ? pl.seed : nullptr;   // grid-layout stamps in the seed plane's place

    SeedParams &sp = p.sp;
    sp.pl = pl;
    std::memcpy(sp.R, T->R, sizeof sp.R);
    std::memcpy(sp.tv, tv, sizeof sp.tv);
    sp.s = g->s;
    sp.kind = kind;
    sp.W = W;
    sp.H = H;
    sp.pitch = pitch_floats;
    sp.fx = sensor->fx;
    sp.fy = sensor->fy;
    sp.cx = sensor->cx;
    sp.cy = sensor->cy;
    sp.dmin = sensor->depth_min;
    sp.dmax = sensor->depth;
    sp.img = data;
    sp.col_tab = sensor->col_tab;
    sp.row_tab = sensor->row_tab;
    sp.lim_out = reinterpret_cast<RowLimits *>(sc + g->lay.lim);
    region_inputs(kind, *sensor, fan, W, H, sp);

    RayParams &rp = p.rp;
    std::memcpy(rp.R, T->R, sizeof rp.R);
    std::memcpy(rp.wf.o, o, sizeof rp.wf.o);
    std::memcpy(rp.wf.v0, v0, sizeof rp.wf.v0);
    std::memcpy(rp.wf.n, g->n, sizeof rp.wf.n);
    rp.wf.gxp = g->lay.gxp;
    rp.kind = kind == kSpinning ? kSpinning : kPinhole;
    rp.vd = fan.vd;
    rp.hw = fan.hw;
    rp.hh = fan.hh;
    rp.na = fan_a;
    rp.nb = fan_b;
    rp.tile_log2w = g->tile_log2w;
    rp.tiles_a = (fan_a + tw - 1) / tw;
    rp.tiles = (int32_t)tiles;
    rp.hz = reinterpret_cast<const int32_t *>(sc + g->lay.hz);
    rp.occ = p.direct ? static_cast<const void *>(pl.occb) : static_cast<const void *>(pl.occ);
    rp.occ_bytes = p.direct ? pl.nbytes : pl.nbytes / 8;
    rp.occ_is_bytes = p.direct ? 1 : 0;
    rp.marks = pl.marks;
    rp.nbytes = pl.nbytes;
    rp.epoch = p.epoch;
    rp.order_in = nullptr;
    p.inside = v0[0] >= 0 && v0[0] < g->n[0] && v0[1] >= 0 && v0[1] < g->n[1] && v0[2] >= 0 &&
               v0[2] < g->n[2];

    // rows holding occupied voxels (seed box minus padding, widened by the
    // inflation) or traced stamps (the fan's reach)
    RowBox seed_rows{1, 0, 1, 0};
    if (pl.lo[0] <= pl.hi[0])
        seed_rows = RowBox{std::max(pl.lo[1] - 2 * pl.r, 0), std::min(pl.hi[1], g->n[1] - 1),
                           std::max(pl.lo[2] - 2 * pl.r, 0), std::min(pl.hi[2], g->n[2] - 1)};
    p.rows = row_union(seed_rows, fan_rows(g, kind, fan, *T, o));
    return VG_OK;
}

// The grid state after a planned frame.
void advance(GridState &gs, const FramePlan &p, const vg_sensor *sensor)
{
    gs.epoch = p.epoch;
    if (p.upload_hz) {
        gs.hz_vd[p.set] = p.fan.vd;
        gs.hz_fov[p.set] = sensor->fov_y;
    }
}

// Work done before a planned frame's stages: the stamp planes of every set
// cleared on a wrap (stamps restart at 1, so no set may keep an old one),
// the spinning fan table of the frame's set written.
hipError_t prepare_frame(const vg_grid *g, const FramePlan &p, hipStream_t st)
{
    hipError_t e = hipSuccess;
    for (int32_t k = 0; p.wrap && k < g->sets && e == hipSuccess; ++k) {
        uint8_t *const sc = g->scratch + (size_t)k * g->lay.fixed;
        e = launch_fill(sc + g->lay.seed, 0, g->lay.bitx - g->lay.seed, st);
        if (e == hipSuccess)
            e = launch_fill(sc + g->lay.marks, 0, g->lay.hz - g->lay.marks, st);
    }
    if (e == hipSuccess && p.upload_hz)
        e = launch_upload(
            reinterpret_cast<uint32_t *>(g->scratch + (size_t)p.set * g->lay.fixed + g->lay.hz),
            reinterpret_cast<const uint32_t *>(p.fan.hz.data()), p.fan.hz.size(), st);
    return e;
}


// Blocks of 256 lanes each batch stage launches for a planned frame.
void batch_blocks(const vg_grid *g, const FramePlan &p, bool moved, const SlabClear &clear,
                  YzTile tile, bool wide_x, bool wide_res, int64_t blocks[kBatchStages])
{
    auto per = [](int64_t lanes) { return (lanes + 255) / 256; };
    const Planes &pl = p.sp.pl;
    const int64_t wx = pl.wx;
    blocks[kBatchShift] = moved ? per(clear_lanes(clear)) : 0;
    // at least one seed block: its first lane writes the frame's regions
    if (p.kind == kPoints)
        blocks[kBatchSeed] = std::max<int64_t>(per(p.sp.W), 1);
    else
        blocks[kBatchSeed] = (p.sp.W > 0 && p.sp.H > 0)
                                 ? (int64_t)((p.sp.W + 63) / 64) * ((p.sp.H + 3) / 4)
                                 : 1;
    const bool any = pl.lo[0] <= pl.hi[0] && pl.lo[1] <= pl.hi[1] && pl.lo[2] <= pl.hi[2];
    blocks[kBatchDilateX] =
        any ? per(dilate_x_lanes(pl.wx, wide_x) * (pl.hi[1] - pl.lo[1] + 1) *
                  (int64_t)(pl.hi[2] - pl.lo[2] + 1))
            : 0;
    blocks[kBatchDilateYZ] =
        tile.kw > 0 ? dilate_tiles(pl, tile) : per(wx * g->n[1] * (int64_t)g->n[2]);
    blocks[kBatchRays] = ((int64_t)p.rp.tiles + 3) / 4;
    const RowBox &b = p.rows;
    blocks[kBatchResolve] = (b.y0 <= b.y1 && b.z0 <= b.z1)
                                ? per(merge_lanes(g->n[0], wide_res) * (b.y1 - b.y0 + 1) *
                                      (int64_t)(b.z1 - b.z0 + 1))
                                : 0;
}

// Steps 2-4 of one frame, one launch per stage.
// A shift of the grid's offset by d stays within +-2^24 voxels.
bool shift_in_range(const vg_grid *g, const int32_t d[3])
{
    for (int a = 0; a < 3; ++a) {
        const int64_t s = (int64_t)g->shift[a] + d[a];
        if (s > (1 << 24) || s < -(1 << 24))
            return false;
    }
    return true;
}

// A pinhole walk from inside the grid with more ray wavefronts than the GPU
// has SIMDs (and no more blocks than an order holds) takes its ray blocks in
// the order its frame's x dilation launch builds (WalkOrder), in plane set 0.
void use_walk_order(vg_grid *g, FramePlan &p, OrderBuild &ob)
{
    ob.order = nullptr;
    const int64_t ray_blocks = ((int64_t)p.rp.tiles + 3) / 4;
    if (p.rp.kind != kPinhole || !p.inside || p.direct || ray_blocks * 4 <= kLoneWaves ||
        ray_blocks > kOrderMaxBlocks)
        return;
    uint8_t *base = g->scratch + g->lay.order;
    p.rp.order_in = reinterpret_cast<const int32_t *>(base);
    ob.rp = p.rp;
    ob.ray_blocks = (int32_t)ray_blocks;
    ob.parts = kOrderMaxParts;
    ob.order = reinterpret_cast<int32_t *>(base);
    ob.keys = base + kOrderBufBytes;
}

// Steps 2-4 of one frame, after the shift d (step 5) if d is given and not
// zero: its slab clear runs as extra workgroups of the walk launch.
vg_status integrate(vg_grid *g, int kind, const float *data, int64_t pitch_floats, int32_t W,
                    int32_t H, const vg_sensor *sensor, const vg_pose *T, hipStream_t st,
                    const int32_t *d = nullptr)
{
    GridState gs = state_of(g);
    SlabClear clear;
    const bool shifted = d && (d[0] != 0 || d[1] != 0 || d[2] != 0);
    if (shifted) {
        if (!shift_in_range(g, d))
            return VG_ERR_ARG;
        plan_shift(g, gs, d, clear);
        clear.loc = g->loc;
    }
    FramePlan p;
    vg_status rc = plan_frame(g, gs, kind, data, pitch_floats, W, H, sensor, T, p, true);
    if (rc != VG_OK)
        return rc;
    if (!same_device(g))
        return VG_ERR_STATE;
    hipError_t e = prepare_frame(g, p, st);
    if (e == hipSuccess && p.wrap)
        g->epoch = 0;   // planes cleared: no stale stamp can match
    if (e != hipSuccess)
        return VG_ERR_HIP;

    const StageEvents *ev = stage_events(g);
    StageEvents none;
    auto stage = [&](int k) -> const StageEvents & { return ev ? ev[k] : none; };
    if (d)   // the shift's own pair: markers (its clear is timed with the walk)
        e = record_empty_stage(stage(kStageShift), st);
    OrderBuild ob;
    use_walk_order(g, p, ob);
    if (e == hipSuccess)
        e = launch_seeds(p.sp, st, stage(kStageSeed), &ob);
    if (e == hipSuccess)   // direct stamping has nothing to dilate
        e = p.direct ? record_empty_stage(stage(kStageDilate), st)
                     : launch_dilate(p.sp.pl, st, stage(kStageDilate), &ob);
    if (e == hipSuccess)
        e = launch_rays(p.rp, p.inside, st, stage(kStageRays), shifted ? &clear : nullptr);
    if (e == hipSuccess)
        e = launch_resolve(p.sp.pl, g->loc, p.rows, p.ring, st, stage(kStageResolve));
    if (ev)
        ++g->prof_next;
    if (e != hipSuccess) {
        // launches already enqueued may have written this frame's stamp: the
        // next frame must not take it again, so it starts by clearing the
        // planes (the stamp wraps)
        g->epoch = 255;
        return VG_ERR_HIP;
    }
    advance(gs, p, sensor);
    store_state(g, gs);
    return VG_OK;
}

}  // namespace

extern "C" {

vg_status vg_fan_sizes(const vg_sensor *sensor, float vox_size, int64_t out[4])
{
    if (!valid_sensor(sensor) || !out || !(vox_size > 0.0f) || !std::isfinite(vox_size))
        return VG_ERR_ARG;
    Fan f;
    if (!fan_for(*sensor, vox_size, f))
        return VG_ERR_ARG;
    out[0] = f.vd;
    out[1] = f.hw;
    out[2] = f.hh;
    out[3] = f.rays;
    return VG_OK;
}

size_t vg_grid_bytes(int32_t gx, int32_t gy, int32_t gz)
{
    if (gx < 1 || gy < 1 || gz < 1 || gx > 65535 || gy > 65535 || gz > 65535)
        return 0;
    // below 2^30: the two mark planes (2x) stay inside 31-bit buffer offsets
    if ((int64_t)grid_pitch(gx) * gy * gz >= ((int64_t)1 << 30))
        return 0;
    return (size_t)grid_pitch(gx) * gy * gz;
}

size_t vg_scratch_bytes(int32_t gx, int32_t gy, int32_t gz, int32_t vox_inf)
{
    if (vg_grid_bytes(gx, gy, gz) == 0 || vox_inf < 0 || vox_inf > kMaxInflation)
        return 0;
    return layout_for(gx, gy, gz, vox_inf).fixed;
}

vg_status vg_create_grid(int32_t gx, int32_t gy, int32_t gz, float vox_size,
                         const float origin_w[3], int32_t vox_inf, uint8_t *loc_grid,
                         uint8_t *loc_spare, size_t grid_bytes, void *scratch,
                         size_t scratch_bytes, void *stream, vg_grid **out)
{
    if (!out)
        return VG_ERR_ARG;
    *out = nullptr;
    if (vg_grid_bytes(gx, gy, gz) == 0)
        return VG_ERR_ARG;
    if (!(vox_size > 0.0f) || !std::isfinite(vox_size) || vox_inf < 0 || vox_inf > kMaxInflation)
        return VG_ERR_ARG;
    if (!origin_w || !std::isfinite(origin_w[0]) || !std::isfinite(origin_w[1]) ||
        !std::isfinite(origin_w[2]))
        return VG_ERR_ARG;
    (void)loc_spare;   // not needed: the local grid is a ring buffer
    if (!loc_grid || !scratch || ((uintptr_t)scratch % kAlign) != 0 ||
        ((uintptr_t)loc_grid % 16) != 0)
        return VG_ERR_ARG;
    const size_t n = vg_grid_bytes(gx, gy, gz);
    Layout lay = layout_for(gx, gy, gz, vox_inf);
    if (scratch_bytes < lay.fixed || grid_bytes < n)
        return VG_ERR_BUDGET;

    vg_grid *g = new (std::nothrow) vg_grid;
    if (!g)
        return VG_ERR_ARG;
    g->n[0] = gx;
    g->n[1] = gy;
    g->n[2] = gz;
    g->s = vox_size;
    for (int a = 0; a < 3; ++a) {
        g->base[a] = origin_w[a];
        g->shift[a] = 0;
    }
    g->r = vox_inf;
    g->loc = loc_grid;
    for (int a = 0; a < 3; ++a)
        g->ring[a] = 0;
    g->scratch = static_cast<uint8_t *>(scratch);
    g->scratch_bytes = scratch_bytes;
    g->lay = lay;
    g->sets = (int32_t)std::min<size_t>(scratch_bytes / lay.fixed, kMaxPlaneSets);
    forget_fan_tables(g);
    g->epoch = 0;
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return VG_ERR_HIP;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    // Step 1: every voxel of the local grid starts unknown; stamps start clear.
    if (launch_fill(loc_grid, VG_UNKNOWN, n, st) != hipSuccess ||
        launch_fill(scratch, 0, (size_t)g->sets * lay.fixed, st) != hipSuccess) {
        delete g;
        return VG_ERR_HIP;
    }
    *out = g;
    return VG_OK;
}

vg_status vg_rebind_grid(vg_grid *g, uint8_t *loc_grid, uint8_t *loc_spare, size_t grid_bytes,
                         void *scratch, size_t scratch_bytes, void *stream)
{
    if (!g)
        return VG_ERR_ARG;
    (void)loc_spare;
    if (!loc_grid || !scratch || ((uintptr_t)scratch % kAlign) != 0 ||
        ((uintptr_t)loc_grid % 16) != 0)
        return VG_ERR_ARG;
    if (scratch_bytes < g->lay.fixed || grid_bytes < vg_grid_bytes(g->n[0], g->n[1], g->n[2]))
        return VG_ERR_BUDGET;
    if (!same_device(g))
        return VG_ERR_STATE;
    // fresh stamp planes: no stamp of an earlier frame is left to match
    const int32_t sets = (int32_t)std::min<size_t>(scratch_bytes / g->lay.fixed, kMaxPlaneSets);
    if (launch_fill(scratch, 0, (size_t)sets * g->lay.fixed, static_cast<hipStream_t>(stream)) !=
        hipSuccess)
        return VG_ERR_HIP;
    g->loc = loc_grid;
    g->scratch = static_cast<uint8_t *>(scratch);
    g->scratch_bytes = scratch_bytes;
    g->sets = sets;
    g->epoch = 0;
    forget_fan_tables(g);
    return VG_OK;
}

vg_status vg_integrate_frame(vg_grid *g, const float *depth, int64_t row_pitch_bytes,
                             const vg_sensor *sensor, const vg_pose *T_w_c, void *stream)
{
    if (!g || !valid_sensor(sensor) || !T_w_c || !finite_pose(T_w_c))
        return VG_ERR_ARG;
    if (row_pitch_bytes % 4 != 0 || row_pitch_bytes < 4 * (int64_t)sensor->width)
        return VG_ERR_ARG;
    int kind = sensor->kind == VG_SPINNING ? kSpinning : kPinhole;
    return integrate(g, kind, depth, row_pitch_bytes / 4, sensor->width, sensor->height, sensor,
                     T_w_c, static_cast<hipStream_t>(stream));
}

vg_status vg_integrate_points(vg_grid *g, const float *points, int64_t n_points,
                              const vg_sensor *sensor, const vg_pose *T_w_c, void *stream)
{
    if (!g || !valid_sensor(sensor) || sensor->kind != VG_PINHOLE || !T_w_c ||
        !finite_pose(T_w_c) || n_points < 0 || n_points > 0x7fffffff)
        return VG_ERR_ARG;
    return integrate(g, kPoints, points, 0, (int32_t)n_points, 1, sensor, T_w_c,
                     static_cast<hipStream_t>(stream));
}

vg_status vg_integrate_frame_shifted(vg_grid *g, const float *depth, int64_t row_pitch_bytes,
                                     const vg_sensor *sensor, const vg_pose *T_w_c, int32_t dx,
                                     int32_t dy, int32_t dz, void *stream)
{
    if (!g || !valid_sensor(sensor) || !T_w_c || !finite_pose(T_w_c))
        return VG_ERR_ARG;
    if (row_pitch_bytes % 4 != 0 || row_pitch_bytes < 4 * (int64_t)sensor->width)
        return VG_ERR_ARG;
    const int32_t d[3] = {dx, dy, dz};
    int kind = sensor->kind == VG_SPINNING ? kSpinning : kPinhole;
    return integrate(g, kind, depth, row_pitch_bytes / 4, sensor->width, sensor->height, sensor,
                     T_w_c, static_cast<hipStream_t>(stream), d);
}

vg_status vg_shift_grid(vg_grid *g, int32_t dx, int32_t dy, int32_t dz, void *stream)
{
    if (!g)
        return VG_ERR_ARG;
    const int32_t d[3] = {dx, dy, dz};
    if (!shift_in_range(g, d))
        return VG_ERR_ARG;
    const StageEvents *ev = stage_events(g);
    const StageEvents none;
    const StageEvents &sev = ev ? ev[kStageShift] : none;
    if (dx == 0 && dy == 0 && dz == 0) {
        if (ev && !same_device(g))
            return VG_ERR_STATE;
        return hip_status(record_empty_stage(sev, static_cast<hipStream_t>(stream)));
    }
    if (!same_device(g))
        return VG_ERR_STATE;
    GridState gs = state_of(g);
    SlabClear c;
    plan_shift(g, gs, d, c);
    c.loc = g->loc;
    hipError_t e = launch_clear(c, static_cast<hipStream_t>(stream), sev);
    if (e != hipSuccess)
        return VG_ERR_HIP;
    store_state(g, gs);
    return VG_OK;
}

vg_status vg_center_offset_after(const vg_grid *g, const int32_t pending[3], const float t_w_c[3],
                                 int32_t delta_out[3])
{
    if (!g || !t_w_c || !delta_out)
        return VG_ERR_ARG;
    float origin[3];
    for (int a = 0; a < 3; ++a) {
        const int64_t s = (int64_t)g->shift[a] + (pending ? pending[a] : 0);
        if (s > (1 << 24) || s < -(1 << 24))
            return VG_ERR_ARG;
        float off = (float)s * g->s;
        origin[a] = g->base[a] + off;
    }
    int32_t d[3];
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(t_w_c[a]))
            return VG_ERR_ARG;
        float rel = t_w_c[a] - origin[a];
        float c = std::floor(rel / g->s);
        if (!(std::fabs(c) < 16777216.0f))
            return VG_ERR_ARG;
        d[a] = (int32_t)c - g->n[a] / 2;
    }
    for (int a = 0; a < 3; ++a)
        delta_out[a] = d[a];
    return VG_OK;
}

vg_status vg_center_offset(const vg_grid *g, const float t_w_c[3], int32_t delta_out[3])
{
    return vg_center_offset_after(g, nullptr, t_w_c, delta_out);
}

vg_status vg_grid_origin(const vg_grid *g, float origin_w_out[3])
{
    if (!g || !origin_w_out)
        return VG_ERR_ARG;
    current_origin(g, origin_w_out);
    return VG_OK;
}

vg_status vg_read_grid(const vg_grid *g, uint8_t *dst, int32_t dst_is_device, void *stream)
{
    if (!g || !dst)
        return VG_ERR_ARG;
    const hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (g->ring[0] == 0 && g->ring[1] == 0 && g->ring[2] == 0)
        return hip_status(copy_grid(dst, g->n[0], g->loc, g->lay.gxp, g->n, kind, st));
    return hip_status(copy_grid_from_ring(dst, g->loc, g->lay.gxp, g->n, g->ring, kind, st));
}

vg_status vg_write_grid(vg_grid *g, const uint8_t *src, int32_t src_is_device, void *stream)
{
    if (!g || !src)
        return VG_ERR_ARG;
    hipError_t e = copy_grid(g->loc, g->lay.gxp, src, g->n[0], g->n,
                             src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                             static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return VG_ERR_HIP;
    for (int a = 0; a < 3; ++a)
        g->ring[a] = 0;   // written in the plain layout
    return VG_OK;
}

vg_status vg_set_profile_events(vg_grid *g, void *const *events, int32_t n_sets)
{
    if (!g || n_sets < 0 || (n_sets > 0 && !events))
        return VG_ERR_ARG;
    std::vector<StageEvents> v;
    for (int64_t i = 0; i < kStages * (int64_t)n_sets; ++i)
        v.push_back(StageEvents{static_cast<hipEvent_t>(events[2 * i]),
                                static_cast<hipEvent_t>(events[2 * i + 1])});
    g->prof.swap(v);
    g->prof_next = 0;
    return VG_OK;
}

vg_status vg_set_ray_tile(vg_grid *g, int32_t log2_width)
{
    if (!g || log2_width < 0 || log2_width > 6)
        return VG_ERR_ARG;
    g->tile_log2w = log2_width;
    return VG_OK;
}

size_t vg_batch_workspace_bytes(int32_t max_frames)
{
    if (max_frames < 0 || max_frames > kMaxBatch)
        return 0;
    return batch_workspace_bytes(max_frames);
}

vg_status vg_integrate_batch(const vg_frame *frames, int32_t n_frames, void *workspace,
                             size_t workspace_bytes, void *stream)
{
    return vg_integrate_batch_timed(frames, n_frames, workspace, workspace_bytes, nullptr, stream);
}

vg_status vg_integrate_batch_timed(const vg_frame *frames, int32_t n_frames, void *workspace,
                                   size_t workspace_bytes, void *const *events, void *stream)
{
    if (n_frames < 0 || n_frames > kMaxBatch || (n_frames > 0 && !frames))
        return VG_ERR_ARG;
    if (n_frames == 0)
        return VG_OK;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0)
        return VG_ERR_ARG;
    if (workspace_bytes < vg_batch_workspace_bytes(n_frames))
        return VG_ERR_BUDGET;
    hipStream_t st = static_cast<hipStream_t>(stream);

    // Plan every frame against the state its grid will have by then.
    std::vector<vg_grid *> grids;
    std::vector<GridState> states;
    std::vector<int32_t> grid_frames;   // frames planned so far per grid
    std::vector<FramePlan> plans((size_t)n_frames);
    std::vector<int32_t> grid_of((size_t)n_frames), round_of((size_t)n_frames);
    std::vector<uint8_t> moved_of((size_t)n_frames);
    std::vector<SlabClear> clears((size_t)n_frames);
    std::vector<std::array<int32_t, 3>> shift_at((size_t)n_frames);   // grid shift after the frame's
    for (int32_t i = 0; i < n_frames; ++i) {
        const vg_frame &f = frames[i];
        vg_grid *g = f.grid;
        if (!g || !valid_sensor(&f.sensor) || !finite_pose(&f.T_w_c))
            return VG_ERR_ARG;
        int kind;
        int32_t W, H;
        int64_t pitch;
        if (f.is_points) {
            if (f.sensor.kind != VG_PINHOLE || f.n_points < 0 || f.n_points > 0x7fffffff)
                return VG_ERR_ARG;
            kind = kPoints;
            W = (int32_t)f.n_points;
            H = 1;
            pitch = 0;
        } else {
            if (f.row_pitch_bytes % 4 != 0 || f.row_pitch_bytes < 4 * (int64_t)f.sensor.width)
                return VG_ERR_ARG;
            kind = f.sensor.kind == VG_SPINNING ? kSpinning : kPinhole;
            W = f.sensor.width;
            H = f.sensor.height;
            pitch = f.row_pitch_bytes / 4;
        }
        size_t k = 0;
        while (k < grids.size() && grids[k] != g)
            ++k;
        if (k == grids.size()) {
            grids.push_back(g);
            states.push_back(state_of(g));
            grid_frames.push_back(0);
        }
        GridState &gs = states[k];
        bool moved = false;
        for (int a = 0; a < 3; ++a) {
            int64_t s = (int64_t)gs.shift[a] + f.shift[a];
            if (s > (1 << 24) || s < -(1 << 24))
                return VG_ERR_ARG;
            moved = moved || f.shift[a] != 0;
        }
        moved_of[i] = moved ? 1 : 0;
        std::memset(&clears[i], 0, sizeof clears[i]);
        if (moved) {
            plan_shift(g, gs, f.shift, clears[i]);
            clears[i].loc = g->loc;
        }
        // the grid's k-th frame of the batch runs in round k / sets on plane
        // set k mod sets: a round holds up to `sets` consecutive frames of a grid
        const int32_t kth = grid_frames[k]++;
        vg_status rc = plan_frame(g, gs, kind, f.data, pitch, W, H, &f.sensor, &f.T_w_c, plans[i],
                                  false, kth % g->sets);
        if (rc != VG_OK)
            return rc;
        advance(gs, plans[i], &f.sensor);
        grid_of[i] = (int32_t)k;
        round_of[i] = kth / g->sets;
        std::memcpy(shift_at[i].data(), gs.shift, sizeof gs.shift);
    }
    for (vg_grid *g : grids)
        if (!same_device(g))
            return VG_ERR_STATE;

    // Frame tables, one per round, packed into the workspace.
    int32_t rounds = 0;
    for (int32_t i = 0; i < n_frames; ++i)
        rounds = std::max(rounds, round_of[i] + 1);
    std::vector<std::vector<int32_t>> members((size_t)rounds);
    for (int32_t i = 0; i < n_frames; ++i)
        members[(size_t)round_of[i]].push_back(i);
    // a grid's frames of a round contiguous and in batch order (the merge
    // takes them as one run)
    for (std::vector<int32_t> &mem : members)
        std::stable_sort(mem.begin(), mem.end(),
                         [&](int32_t a, int32_t b) { return grid_of[a] < grid_of[b]; });
    // rounds with a run of several frames of one grid merge run by run
    std::vector<uint8_t> seq_round((size_t)rounds, 0);
    for (int32_t r = 0; r < rounds; ++r) {
        const std::vector<int32_t> &mem = members[(size_t)r];
        for (size_t j = 1; j < mem.size(); ++j)
            if (grid_of[mem[j]] == grid_of[mem[j - 1]])
                seq_round[(size_t)r] = 1;
    }
    std::vector<size_t> table_at((size_t)rounds);
    size_t used = 0;
    for (int32_t r = 0; r < rounds; ++r) {
        table_at[(size_t)r] = used;
        used += batch_table_bytes((int32_t)members[(size_t)r].size());
    }
    if (used > workspace_bytes)
        return VG_ERR_BUDGET;
    std::vector<uint32_t> host(used / 4, 0u);
    std::vector<std::array<int32_t, kBatchStages>> totals((size_t)rounds);
    // tiled y/z dilation per round: the widest slot any frame needs, if every
    // frame of the round can use tiles (kw 0: the untiled kernel), 8 deep if
    // every frame can and the round has enough 8-deep tiles
    std::vector<YzTile> round_tile((size_t)rounds, YzTile{0, 0});
    std::vector<size_t> round_lds((size_t)rounds, 0);
    // wide forms of the x dilation and the merge where the round's narrow
    // forms would have many lanes
    std::vector<uint8_t> wide_x((size_t)rounds, 0), wide_res((size_t)rounds, 0);
    for (int32_t r = 0; r < rounds; ++r) {
        int64_t nx = 0, nres = 0;
        for (int32_t i : members[(size_t)r]) {
            const Planes &pl = plans[(size_t)i].sp.pl;
            if (pl.lo[0] <= pl.hi[0] && pl.lo[1] <= pl.hi[1] && pl.lo[2] <= pl.hi[2])
                nx += dilate_x_lanes(pl.wx, false) * (pl.hi[1] - pl.lo[1] + 1) *
                      (int64_t)(pl.hi[2] - pl.lo[2] + 1);
            const RowBox &b = plans[(size_t)i].rows;
            if (b.y0 <= b.y1 && b.z0 <= b.z1)
                nres += merge_lanes(pl.n[0], false) * (b.y1 - b.y0 + 1) *
                        (int64_t)(b.z1 - b.z0 + 1);
        }
        wide_x[(size_t)r] = dilate_x_wide(nx) ? 1 : 0;
        wide_res[(size_t)r] = nres >= kWideLanes ? 1 : 0;
    }
    for (int32_t r = 0; r < rounds; ++r) {
        const std::vector<int32_t> &mem = members[(size_t)r];
        const int32_t m = (int32_t)mem.size();
        YzTile pick{0, 0};
        size_t pick_lds = 0;
        for (int tz : {kTileDeep, 2}) {
            int tw = 8;
            for (int32_t i : mem) {
                const int k = dilate_tile_width(plans[(size_t)i].sp.pl, tz);
                tw = k == 0 ? 0 : (tw == 0 ? 0 : std::max(tw, k));
            }
            size_t lds = 0;
            int64_t tiles = 0;
            for (int32_t i : mem)
                if (tw > 0) {
                    lds = std::max(lds, dilate_tile_lds(plans[(size_t)i].sp.pl, YzTile{tw, tz}));
                    tiles += dilate_tiles(plans[(size_t)i].sp.pl, YzTile{tw, tz});
                }
            if (tw == 0 || lds > kMaxTileLds || (tz == kTileDeep && tiles < kDeepTileMin))
                continue;
            pick = YzTile{tw, tz};
            pick_lds = lds;
            break;
        }
        round_tile[(size_t)r] = pick;
        round_lds[(size_t)r] = pick_lds;
        uint8_t *base = reinterpret_cast<uint8_t *>(host.data()) + table_at[(size_t)r];
        int32_t *start = reinterpret_cast<int32_t *>(base);
        FrameDesc *fd = reinterpret_cast<FrameDesc *>(base + batch_starts_bytes(m));
        std::array<int64_t, kBatchStages> acc{};
        for (int32_t j = 0; j < m; ++j) {
            const int32_t i = mem[(size_t)j];
            const FramePlan &p = plans[(size_t)i];
            const vg_grid *g = grids[(size_t)grid_of[i]];
            int64_t blocks[kBatchStages];
            batch_blocks(g, p, moved_of[i] != 0, clears[i], round_tile[(size_t)r],
                         wide_x[(size_t)r] != 0, wide_res[(size_t)r] != 0, blocks);
            // a run of frames of one grid: its first frame carries the run and
            // the merge's rows -- the union of the frames' row boxes moved into
            // the grid coordinates of the run's last frame (a row a frame's
            // box holds that has left the grid by then was cleared by a later
            // shift of the run, which the merge re-applies in order)
            int32_t group = 0;
            RowBox dom{1, 0, 1, 0};
            if (seq_round[(size_t)r] && (j == 0 || grid_of[mem[(size_t)j - 1]] != grid_of[i])) {
                int32_t e = j;
                while (e < m && grid_of[mem[(size_t)e]] == grid_of[i])
                    ++e;
                group = e - j;
                const std::array<int32_t, 3> &last = shift_at[(size_t)mem[(size_t)e - 1]];
                for (int32_t t = j; t < e; ++t) {
                    const int32_t it = mem[(size_t)t];
                    const RowBox &b = plans[(size_t)it].rows;
                    if (b.y0 > b.y1 || b.z0 > b.z1)
                        continue;
                    const int32_t dy = last[1] - shift_at[(size_t)it][1];
                    const int32_t dz = last[2] - shift_at[(size_t)it][2];
                    const RowBox moved{std::max(b.y0 - dy, 0), std::min(b.y1 - dy, g->n[1] - 1),
                                       std::max(b.z0 - dz, 0), std::min(b.z1 - dz, g->n[2] - 1)};
                    dom = row_union(dom, moved);
                }
                blocks[kBatchResolve] =
                    (dom.y0 <= dom.y1 && dom.z0 <= dom.z1)
                        ? ((int64_t)merge_lanes_per_row(g->n[0]) * (dom.y1 - dom.y0 + 1) *
                               (int64_t)(dom.z1 - dom.z0 + 1) + 255) / 256
                        : 0;
            } else if (seq_round[(size_t)r]) {
                blocks[kBatchResolve] = 0;
            }
            FrameDesc d;
            std::memset(&d, 0, sizeof d);
            d.sp = p.sp;
            d.rp = p.rp;
            d.loc = g->loc;
            d.clear = clears[i];
            d.rows = p.rows;
            std::memcpy(d.ring, p.ring, sizeof d.ring);
            d.inside = p.inside ? 1 : 0;
            d.seed_bx = p.kind == kPoints ? 0 : std::max((p.sp.W + 63) / 64, 1);
            d.group = group;
            d.dom = dom;
            std::memcpy(&fd[j], &d, sizeof d);
            for (int s = 0; s < kBatchStages; ++s) {
                start[s * (m + 1) + j] = (int32_t)acc[s];
                acc[s] += blocks[s];
                if (acc[s] > 0x7fffffff)
                    return VG_ERR_ARG;
            }
        }
        for (int s = 0; s < kBatchStages; ++s) {
            start[s * (m + 1) + m] = (int32_t)acc[s];
            totals[(size_t)r][s] = (int32_t)acc[s];
        }
    }

    // A round of one frame (untimed) runs the one-frame launches instead: no
    // table, the shift's clear inside the walk launch.
    std::vector<uint8_t> direct((size_t)rounds);
    bool all_direct = true;
    for (int32_t r = 0; r < rounds; ++r) {
        direct[(size_t)r] = !events && members[(size_t)r].size() == 1;
        all_direct = all_direct && direct[(size_t)r];
    }

    // Upload the tables, then per round: per-frame preparation and one
    // launch per stage.
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    hipError_t e = all_direct ? hipSuccess
                              : launch_upload(reinterpret_cast<uint32_t *>(ws), host.data(),
                                              host.size(), st);
    for (int32_t r = 0; r < rounds && e == hipSuccess; ++r) {
        const std::vector<int32_t> &mem = members[(size_t)r];
        const int32_t m = (int32_t)mem.size();
        for (int32_t i : mem)
            if (e == hipSuccess)
                e = prepare_frame(grids[(size_t)grid_of[i]], plans[(size_t)i], st);
        if (direct[(size_t)r]) {
            const int32_t i = mem[0];
            const FramePlan &p = plans[(size_t)i];
            const vg_grid *g = grids[(size_t)grid_of[i]];
            if (e == hipSuccess)
                e = launch_seeds(p.sp, st);
            if (e == hipSuccess)
                e = launch_dilate(p.sp.pl, st);
            if (e == hipSuccess)
                e = launch_rays(p.rp, p.inside, st, {}, moved_of[i] ? &clears[i] : nullptr);
            if (e == hipSuccess)
                e = launch_resolve(p.sp.pl, g->loc, p.rows, p.ring, st);
            continue;
        }
        const int32_t *start = reinterpret_cast<const int32_t *>(ws + table_at[(size_t)r]);
        const FrameDesc *fd =
            reinterpret_cast<const FrameDesc *>(ws + table_at[(size_t)r] + batch_starts_bytes(m));
        for (int s = 0; s < kBatchStages && e == hipSuccess; ++s) {
            StageEvents ev;
            if (events) {   // stage s: start of its first launch, end of its last
                ev.start = r == 0 ? static_cast<hipEvent_t>(events[2 * s]) : nullptr;
                ev.stop = r == rounds - 1 ? static_cast<hipEvent_t>(events[2 * s + 1]) : nullptr;
            }
            const bool yz = s == kBatchDilateYZ;
            const bool wide = (s == kBatchDilateX && wide_x[(size_t)r]) ||
                              (s == kBatchResolve && wide_res[(size_t)r]);
            e = launch_batch_stage(s, fd, start + s * (m + 1), m, totals[(size_t)r][s], st, ev,
                                   yz ? round_tile[(size_t)r] : YzTile{0, 0},
                                   yz ? round_lds[(size_t)r] : 0,
                                   s == kBatchResolve && seq_round[(size_t)r], wide);
        }
    }
    if (e != hipSuccess) {
        // as for one frame: stamps of this batch may already be in the planes
        for (vg_grid *g : grids)
            g->epoch = 255;
        return VG_ERR_HIP;
    }
    for (size_t k = 0; k < grids.size(); ++k)
        store_state(grids[k], states[k]);
    return VG_OK;
}

vg_status vg_integrate_batch_static(const vg_frame *frames, int32_t n_frames, void *stream)
{
    if (n_frames > kStaticBatchFrames)
        return VG_ERR_BUDGET;
    if (n_frames < 0 || (n_frames > 0 && !frames))
        return VG_ERR_ARG;
    if (n_frames == 0)
        return VG_OK;
    void *ws = nullptr;
    if (static_batch_workspace(&ws) != hipSuccess)
        return VG_ERR_HIP;
    return vg_integrate_batch_timed(frames, n_frames, ws, kStaticBatchBytes, nullptr, stream);
}

vg_status vg_destroy_grid(vg_grid *g)
{
    if (!g)
        return VG_ERR_ARG;
    delete g;
    return VG_OK;
}

const char *vg_status_str(vg_status s)
{
    switch (s) {
    case VG_OK:
        return "ok";
    case VG_ERR_ARG:
        return "invalid argument";
    case VG_ERR_HIP:
        return "HIP runtime error";
    case VG_ERR_BUDGET:
        return "scratch workspace too small";
    case VG_ERR_STATE:
        return "handle used on another device";
    default:
        return "unknown status";
    }
}

}  // extern "C"

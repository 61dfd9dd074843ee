// vg_api.cpp -- host side of the C ABI declared in include/vg.h:
// argument validation, the host-computed per-frame constants (T^v_c, the ray
// fan sizes of Sec. IV-C, the camera voxel), scratch layout and launches.
#include "../../include/vg.h"
#include "vg_internal.h"

#include <hip/hip_runtime.h>

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

// Scratch layout (all offsets 256-aligned):
//   seed      seed stamps on the grid padded by vox_inf, rows of seed_pitch bytes
//   bitx      seeds dilated along x, one 32-bit word per 32 voxels of a padded row
//   occ       occupied voxels of the frame, one bit per device-layout voxel
//   traced    "unknown and traced" stamps, one byte per device-layout voxel
//   hz        spinning fan: half height per ring column
struct Layout {
    int32_t gxp, wx, py, pz, seed_pitch;
    size_t seed, bitx, occ, traced, hz, fixed;
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
    l.traced = l.occ + align_up((size_t)4 * l.wx * gy * gz);
    l.hz = l.traced + align_up((size_t)l.gxp * gy * gz);
    l.fixed = l.hz + kHzBytes;
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
    uint8_t *loc, *spare;
    uint8_t *scratch;
    size_t scratch_bytes;
    Layout lay;
    uint32_t epoch;          // stamp of the last frame, 0 = none yet
    int device;
    // spinning fan table currently in scratch
    int32_t hz_vd = 0;
    double hz_fov = -1.0;
    std::vector<int32_t> hz_host;   // kept alive for the asynchronous upload
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

// Common part of steps 2-4: per-frame constants, stamp, launches.
vg_status integrate(vg_grid *g, int kind, const float *data, int64_t pitch_floats, int32_t W,
                    int32_t H, const vg_sensor *sensor, const vg_pose *T, hipStream_t st)
{
    Fan fan;
    if (!fan_for(*sensor, g->s, fan))
        return VG_ERR_ARG;
    if ((W > 0 && H > 0) && !data)
        return VG_ERR_ARG;

    // T^v_c = T^v_w T^w_c: the grid frame is the world frame translated by
    // -origin (axes aligned), so R is unchanged and t^v = t^w_c - origin.
    float origin[3], tv[3], o[3];
    int32_t v0[3];
    current_origin(g, origin);
    for (int a = 0; a < 3; ++a) {
        tv[a] = T->t[a] - origin[a];
        o[a] = tv[a] / g->s;   // camera position in voxel units
        if (!(std::fabs(o[a]) < 16777216.0f))
            return VG_ERR_ARG;
        v0[a] = (int32_t)std::floor(o[a]);
    }
    // fan tiles of 8 x 8 targets, one wavefront each
    const int32_t fan_a = kind == kSpinning ? 8 * fan.vd : 2 * fan.hw + 1;
    const int32_t fan_b = 2 * fan.hh + 1;
    const int64_t tiles = (int64_t)((fan_a + 7) / 8) * ((fan_b + 7) / 8);
    if (tiles * 64 > (int64_t)0x7fffffff)
        return VG_ERR_ARG;
    if (!same_device(g))
        return VG_ERR_STATE;

    // Per-frame stamp 1..255; the stamp planes are cleared when it wraps.
    hipError_t e = hipSuccess;
    if (g->epoch == 255) {
        e = launch_fill(g->scratch + g->lay.seed, 0, g->lay.bitx - g->lay.seed, st);
        if (e == hipSuccess)
            e = launch_fill(g->scratch + g->lay.traced, 0, g->lay.hz - g->lay.traced, st);
        if (e != hipSuccess)
            return VG_ERR_HIP;
        g->epoch = 0;
    }
    const uint32_t epoch = g->epoch + 1;

    if (kind == kSpinning && (g->hz_vd != fan.vd || g->hz_fov != sensor->fov_y)) {
        g->hz_host = fan.hz;
        e = hipMemcpyAsync(g->scratch + g->lay.hz, g->hz_host.data(),
                           g->hz_host.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
        // The table changes only with the sensor; wait so the host copy can
        // be replaced safely next time.
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return VG_ERR_HIP;
        g->hz_vd = fan.vd;
        g->hz_fov = sensor->fov_y;
    }

    const StageEvents *ev = stage_events(g);
    StageEvents none;
    auto stage = [&](int k) -> const StageEvents & { return ev ? ev[k] : none; };

    Planes pl;
    std::memcpy(pl.n, g->n, sizeof pl.n);
    pl.r = g->r;
    pl.wx = g->lay.wx;
    pl.py = g->lay.py;
    pl.pz = g->lay.pz;
    pl.seed_pitch = g->lay.seed_pitch;
    pl.seed = g->scratch + g->lay.seed;
    pl.bitx = reinterpret_cast<uint32_t *>(g->scratch + g->lay.bitx);
    pl.occ = reinterpret_cast<uint32_t *>(g->scratch + g->lay.occ);
    pl.traced = g->scratch + g->lay.traced;
    seed_box(g, kind, *sensor, *T, tv, pl.lo, pl.hi);
    pl.epoch = epoch;

    SeedParams sp;
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

    RayParams rp;
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
    rp.tiles_a = (fan_a + 7) / 8;
    rp.tiles = (int32_t)tiles;
    rp.hz = reinterpret_cast<const int32_t *>(g->scratch + g->lay.hz);
    rp.loc = g->loc;
    rp.occ = pl.occ;
    rp.traced = pl.traced;
    rp.epoch = epoch;
    const bool inside = v0[0] >= 0 && v0[0] < g->n[0] && v0[1] >= 0 && v0[1] < g->n[1] &&
                        v0[2] >= 0 && v0[2] < g->n[2];

    // rows holding occupied voxels (seed box minus padding, widened by the
    // inflation) or traced stamps (the fan's reach)
    RowBox seed_rows{1, 0, 1, 0};
    if (pl.lo[0] <= pl.hi[0])
        seed_rows = RowBox{std::max(pl.lo[1] - 2 * pl.r, 0), std::min(pl.hi[1], g->n[1] - 1),
                           std::max(pl.lo[2] - 2 * pl.r, 0), std::min(pl.hi[2], g->n[2] - 1)};
    const RowBox rows = row_union(seed_rows, fan_rows(g, kind, fan, *T, o));

    if (e == hipSuccess)
        e = launch_seeds(sp, st, stage(kStageSeed));
    if (e == hipSuccess)
        e = launch_dilate(pl, st, stage(kStageDilate));
    if (e == hipSuccess)
        e = launch_rays(rp, inside, st, stage(kStageRays));
    if (e == hipSuccess)
        e = launch_resolve(pl, g->loc, rows, st, stage(kStageResolve));
    if (ev)
        ++g->prof_next;
    if (e != hipSuccess)
        return VG_ERR_HIP;
    g->epoch = epoch;
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
    if ((int64_t)grid_pitch(gx) * gy * gz >= ((int64_t)1 << 31))
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
    if (!loc_grid || !loc_spare || loc_grid == loc_spare || !scratch ||
        ((uintptr_t)scratch % kAlign) != 0 || ((uintptr_t)loc_grid % 16) != 0 ||
        ((uintptr_t)loc_spare % 16) != 0)
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
    g->spare = loc_spare;
    g->scratch = static_cast<uint8_t *>(scratch);
    g->scratch_bytes = scratch_bytes;
    g->lay = lay;
    g->epoch = 0;
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return VG_ERR_HIP;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    // Step 1: every voxel of the local grid starts unknown; stamps start clear.
    if (launch_fill(loc_grid, VG_UNKNOWN, n, st) != hipSuccess ||
        launch_fill(scratch, 0, lay.fixed, st) != hipSuccess) {
        delete g;
        return VG_ERR_HIP;
    }
    *out = g;
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

vg_status vg_shift_grid(vg_grid *g, int32_t dx, int32_t dy, int32_t dz, void *stream)
{
    if (!g)
        return VG_ERR_ARG;
    const int32_t d[3] = {dx, dy, dz};
    for (int a = 0; a < 3; ++a) {
        int64_t s = (int64_t)g->shift[a] + d[a];
        if (s > (1 << 24) || s < -(1 << 24))
            return VG_ERR_ARG;
    }
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
    hipError_t e = launch_shift(g->loc, g->spare, g->n, d, static_cast<hipStream_t>(stream), sev);
    if (e != hipSuccess)
        return VG_ERR_HIP;
    uint8_t *t = g->loc;
    g->loc = g->spare;
    g->spare = t;
    for (int a = 0; a < 3; ++a)
        g->shift[a] += d[a];
    return VG_OK;
}

vg_status vg_center_offset(const vg_grid *g, const float t_w_c[3], int32_t delta_out[3])
{
    if (!g || !t_w_c || !delta_out)
        return VG_ERR_ARG;
    float origin[3];
    current_origin(g, origin);
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
    return hip_status(copy_grid(dst, g->n[0], g->loc, g->lay.gxp, g->n,
                                dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                static_cast<hipStream_t>(stream)));
}

vg_status vg_write_grid(vg_grid *g, const uint8_t *src, int32_t src_is_device, void *stream)
{
    if (!g || !src)
        return VG_ERR_ARG;
    return hip_status(copy_grid(g->loc, g->lay.gxp, src, g->n[0], g->n,
                                src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                static_cast<hipStream_t>(stream)));
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

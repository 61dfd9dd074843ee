// Host build of the kernel's ray walk (paper_2112_13169_amd/csrc/vg_walk.h),
// checked ray by ray against the CPU oracle's walk.  Random grids, random
// occupancy, random rays from inside and outside the grid.  In every other
// trial the lane's wavefront votes at random (vg_host_vote): other lanes may
// still need occupancy loads after this ray's hit, or force the chunk path
// with per-step tests.  Occupancy as bits, or (every third trial) as stamp
// bytes with stale stamps of other frames on free voxels.  Either buffer is
// followed by set words / this frame's stamp, which reads beyond the plane's
// size must not see.  Prints the number of mismatching voxels and exits
// non-zero if there is any.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../oracle/vg_oracle.h"
#include "../paper_2112_13169_amd/csrc/vg_walk.h"

using namespace vg;

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd()
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (uint32_t)(rng_state >> 11);
}

static bool random_vote() { return rnd() % 3 == 0; }

int main(int argc, char **argv)
{
    const int trials = argc > 1 ? atoi(argv[1]) : 2000;
    rng_state += argc > 2 ? (uint64_t)atoll(argv[2]) : 0;
    long long bad = 0, voxels = 0, steps = 0;
    for (int trial = 0; trial < trials; ++trial) {
        // every third trial: a large grid and long rays, so that most chunks
        // take the path without per-step tests
        const bool big = trial % 3 == 1;
        WalkFrame f;
        f.n[0] = 1 + rnd() % (big ? 200 : 48);
        f.n[1] = 1 + rnd() % (big ? 160 : 40);
        f.n[2] = 1 + rnd() % (big ? 120 : 24);
        f.gxp = 32 * ((f.n[0] + 31) / 32);
        const int nx = f.n[0], ny = f.n[1], nz = f.n[2];
        const bool outside = trial % 4 == 3;
        for (int a = 0; a < 3; ++a) {
            float span = outside ? 3.0f * f.n[a] : (float)f.n[a];
            float off = outside ? -1.0f * f.n[a] : 0.0f;
            f.o[a] = off + span * (float)(rnd() % 100000) / 100000.0f;
            if (!outside && f.o[a] >= f.n[a])
                f.o[a] = f.n[a] - 0.5f;
            if (trial % 7 == 0)
                f.o[a] = floorf(f.o[a]) + 0.5f;   // voxel centres: ties in the walk
            f.v0[a] = (int32_t)floorf(f.o[a]);
        }
        const bool inside = f.v0[0] >= 0 && f.v0[0] < nx && f.v0[1] >= 0 && f.v0[1] < ny &&
                            f.v0[2] >= 0 && f.v0[2] < nz;
        const size_t words = (size_t)f.gxp / 32 * ny * nz;
        std::vector<uint32_t> occ(words + 4096, 0xFFFFFFFFu);   // the plane, then set words
        std::fill(occ.begin(), occ.begin() + words, 0u);
        const bool bytes = trial % 3 == 2;
        const uint8_t stamp = 1 + rnd() % 255;
        // byte stamps: the plane (one byte per device-layout voxel), then bytes
        // holding this frame's stamp that reads beyond the plane must not see
        const size_t nvox = (size_t)f.gxp * ny * nz;
        std::vector<uint8_t> occb(nvox + 4096, stamp);
        for (size_t j = 0; j < nvox; ++j)
            occb[j] = (uint8_t)(rnd() % 4 == 0 ? (stamp + 1 + rnd() % 254) & 0xFF : 0);
        vg_host_vote = trial % 2 ? random_vote : nullptr;
        std::vector<uint8_t> ms((size_t)nx * ny * nz, 0);
        const uint32_t density = big ? 200 + rnd() % 4000 : 8 + rnd() % 120;
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    if (rnd() % density == 0) {
                        size_t j = (size_t)x + (size_t)f.gxp * (y + (size_t)ny * z);
                        occ[j >> 5] |= 1u << (j & 31);
                        occb[j] = stamp;
                        ms[x + (size_t)nx * (y + (size_t)ny * z)] = OG_OCCUPIED;
                    }
        float dir[3];
        for (int a = 0; a < 3; ++a) {
            int k = (int)(rnd() % 61) - 30;
            dir[a] = trial % 5 == 0 ? (float)k : (float)k * 0.37f + (float)(rnd() % 1000) * 1e-4f;
            if (trial % 11 == 0 && a == trial % 3)
                dir[a] = 0.0f;
        }
        const int32_t m2 = 1 + (int32_t)(rnd() % (big ? 60000 : 4000));
        const uint32_t n = (uint32_t)((size_t)f.gxp * ny * nz);
        std::vector<uint8_t> marks(2 * (size_t)n, 0);

        bool dead = false;
        for (int a = 0; a < 3; ++a)
            dead = dead || axis_dead(sgn(dir[a]), f.v0[a], f.n[a]);
        if (!dead) {
            Walk w;
            walk_setup(w, f, dir);
            // both walk forms (the lone one for wavefronts alone on a SIMD)
            const bool lone = trial / 4 % 2 == 1;
            if (bytes) {
                const WalkMem m = walk_mem(occb.data(), (uint32_t)nvox, marks.data(), n, stamp);
                if (inside && lone)
                    walk_ray<false, true, true>(w, m2, m);
                else if (inside)
                    walk_ray<false, true, false>(w, m2, m);
                else
                    walk_ray<true, true, false>(w, m2, m);
            } else {
                const WalkMem m = walk_mem(occ.data(), (uint32_t)(4 * words), marks.data(), n,
                                           stamp);
                if (inside && lone)
                    walk_ray<false, false, true>(w, m2, m);
                else if (inside)
                    walk_ray<false, false, false>(w, m2, m);
                else
                    walk_ray<true, false, false>(w, m2, m);
            }
        }
        std::vector<uint8_t> ref = ms;
        steps += og_trace_ray(f.o, dir, m2, nx, ny, nz, ref.data(), nullptr, nullptr, 0);
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    size_t i = x + (size_t)nx * (y + (size_t)ny * z);
                    size_t j = x + (size_t)f.gxp * (y + (size_t)ny * z);
                    int got = ms[i] == OG_OCCUPIED       ? OG_OCCUPIED
                              : marks[n + j] == stamp    ? OG_TRACED
                              : marks[j] == stamp        ? OG_FREE
                                                         : OG_UNKNOWN;
                    if (got != ref[i]) {
                        if (bad < 5)
                            fprintf(stderr, "trial %d voxel (%d,%d,%d): oracle %d walk %d\n", trial,
                                    x, y, z, ref[i], got);
                        ++bad;
                    }
                    ++voxels;
                }
    }
    printf("trials %d voxels %lld oracle-steps %lld mismatches %lld\n", trials, voxels, steps, bad);
    return bad != 0;
}

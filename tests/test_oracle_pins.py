"""Pins of the CPU oracle against what the paper and plain mathematics fix.

None of these tests re-types the oracle's formulas: expected values come from
the paper's printed numbers (tests/golden/standard_params.txt), hand-computed
cases with exact binary inputs (tests/golden/single_*.txt), brute force over
voxels in double / exact rationals, and invariants.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([c.strip() for c in line.split("|")])
    return rows


def _nums(s, typ=float):
    return [typ(v) for v in s.split()]


# ------------------------------------------------------- ray-fan sizes (IV-C)

def test_standard_parameters_voxel_and_ray_counts():
    """Sec. V: the standard parameters give exactly 200 000 voxels and about
    8 500 rays."""
    kv = {r[0].split()[0]: r[0].split()[1] for r in _read_table("standard_params.txt")}
    s = float(kv["vox_size_m"])
    dims = [round(float(kv[f"grid_size_{a}_m"]) / s) for a in "xyz"]
    assert dims[0] * dims[1] * dims[2] == int(kv["voxels_exact"])
    vd, hw, hh = oracle.fan_sizes(float(kv["depth_m"]), s, math.radians(float(kv["fov_x_deg"])),
                                  math.radians(float(kv["fov_y_deg"])))
    assert vd == 43                      # 6.5 / 0.15 = 43.3 -> 43
    rays = (2 * hw + 1) * (2 * hh + 1)
    # "about 8 500": the reading gives 79 x 105 = 8 295 (2.4 % below).
    assert abs(rays - int(kv["rays_approx"])) / int(kv["rays_approx"]) < 0.05
    assert (2 * hw + 1) % 2 == 1 and (2 * hh + 1) % 2 == 1   # odd by construction


def test_fan_sizes_closed_forms():
    # 90 degrees: tan(45 deg) = 1, so the half width equals vox_depth.
    for depth, s, vd in [(5.0, 0.1, 50), (8.0, 0.05, 160), (12.0, 0.025, 480)]:
        got = oracle.fan_sizes(depth, s, math.pi / 2, math.pi / 2)
        assert got == (vd, vd, vd)
    # fov = 2 atan(k / vd) gives half width k exactly.
    for k in range(0, 30):
        vd, hw, hh = oracle.fan_sizes(5.0, 0.25, 2 * math.atan(k / 20), 2 * math.atan((k + 1) / 20))
        assert (vd, hw, hh) == (20, k, k + 1)
    # vox_depth rounds half away from zero: 0.625 / 0.25 = 2.5 -> 3.
    assert oracle.fan_sizes(0.625, 0.25, 1.0, 1.0)[0] == 3
    assert oracle.fan_sizes(0.375, 0.25, 1.0, 1.0)[0] == 2     # 1.5 -> 2
    # out of range
    assert oracle.fan_sizes(0.01, 1.0, 1.0, 1.0) is None


# ---------------------------------------------- Alg. 1 quantisation (IV-B)

def test_single_points_hand_cases():
    for name, Rs, tvs, ss, pcs, qs in _read_table("single_points.txt"):
        q = oracle.quantize(_nums(Rs), _nums(tvs), float(ss), _nums(pcs))
        assert list(q.astype(int)) == _nums(qs, int), name


def _exact_q(R, tv, s, p):
    """floor((R p + tv) / s) in exact rationals."""
    out = []
    for i in range(3):
        acc = Fraction(tv[i]) + sum(Fraction(float(R[i][j])) * Fraction(float(p[j])) for j in range(3))
        out.append(math.floor(acc / Fraction(s)))
    return out


def _perm_rotations():
    mats = []
    for perm in [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]:
        for signs in np.ndindex(2, 2, 2):
            M = np.zeros((3, 3))
            for i in range(3):
                M[i, perm[i]] = -1.0 if signs[i] else 1.0
            if np.linalg.det(M) > 0:
                mats.append(M)
    return mats


def test_quantize_exact_brute_force():
    """Permutation rotations and dyadic inputs: every fp32 op is exact, so the
    oracle must equal the exact rational floor."""
    rng = np.random.default_rng(7)
    rots = _perm_rotations()
    assert len(rots) == 24
    for _ in range(2000):
        R = rots[rng.integers(len(rots))]
        s = [0.25, 0.5, 0.125, 1.0][rng.integers(4)]
        tv = rng.integers(-256, 256, 3) / 64.0
        p = rng.integers(-512, 512, 3) / 64.0
        q = oracle.quantize(R.reshape(-1), tv, s, p)
        assert list(q.astype(int)) == _exact_q(R, tv, s, p)


# ---------------------------------------- Alg. 1 occupied cubes (IV-B, R2)

def _points_frame(dims, s, r, pts, tv, R=np.eye(3)):
    gx, gy, gz = dims
    loc = np.zeros((gz, gy, gx), np.uint8)
    # camera at tv with origin 0; a narrow fan keeps rays short
    ms, st = oracle.integrate_points(loc, [0, 0, 0], s, r, pts, 0.2, 0.2, 2 * s, R.reshape(-1),
                                     tv)
    return ms, st


def test_occupied_cube_clipping_hand_cases():
    s = 1.0
    # point voxels (0,0,0), (-1,2,2), (-2,2,2) [too far], (4,2,2), (5,2,2) [too far]
    pts = np.array([[0.5, 0.5, 0.5], [-0.5, 2.5, 2.5], [-1.5, 2.5, 2.5],
                    [4.5, 2.5, 2.5], [5.5, 2.5, 2.5]])
    ms, _ = _points_frame((4, 4, 4), s, 1, pts, [0.0, 0.0, 0.0])
    occ = ms == oracle.OCCUPIED
    expect = np.zeros((4, 4, 4), bool)
    expect[0:2, 0:2, 0:2] = True          # cube of (0,0,0) clipped at the corner
    expect[1:4, 1:4, 0] = True            # (-1,2,2) reaches in: x = 0 only
    expect[1:4, 1:4, 3] = True            # (4,2,2) reaches in: x = 3 only
    assert np.array_equal(occ, expect)


@pytest.mark.parametrize("r", [0, 1, 2, 3])
def test_occupied_union_of_cubes_brute_force(r):
    """Voxel v is occupied iff some point's voxel is within Chebyshev r of v
    (brute force over voxels, exact point voxels)."""
    rng = np.random.default_rng(100 + r)
    dims = (11, 9, 7)
    s = 0.5
    rots = _perm_rotations()
    for trial in range(6):
        R = rots[rng.integers(len(rots))]
        tv = rng.integers(0, 6 * 64, 3) / 64.0
        n = int(rng.integers(1, 40))
        pts = rng.integers(-8 * 64, 8 * 64, (n, 3)) / 64.0
        ms, _ = _points_frame(dims, s, r, pts, tv, R)
        q = np.array([_exact_q(R, tv, s, p) for p in pts])
        zz, yy, xx = np.meshgrid(*[np.arange(d) for d in dims[::-1]], indexing="ij")
        vox = np.stack([xx, yy, zz], -1).reshape(-1, 1, 3)
        cheb = np.abs(vox - q[None, :, :]).max(-1)
        expect = (cheb <= r).any(-1).reshape(dims[::-1])
        assert np.array_equal(ms == oracle.OCCUPIED, expect), trial


# ------------------------------------------------ Alg. 2 single rays (IV-C)

_VAL = {"F": oracle.FREE, "T": oracle.TRACED, "O": oracle.OCCUPIED, "X": oracle.OUTSIDE}


def test_single_rays_hand_cases():
    for name, dims, o, d, m2, occs, walk in _read_table("single_rays.txt"):
        gx, gy, gz = _nums(dims, int)
        ms = np.zeros((gz, gy, gx), np.uint8)
        if occs != "-":
            for c in occs.split(";"):
                x, y, z = (int(v) for v in c.split(","))
                ms[z, y, x] = oracle.OCCUPIED
        before = ms.copy()
        xyz, val = oracle.trace_ray(_nums(o), _nums(d), int(m2), (gx, gy, gz), ms)
        exp = [(tuple(int(v) for v in w.split(":")[0].split(",")), _VAL[w.split(":")[1]])
               for w in walk.split()]
        assert [tuple(v) for v in xyz] == [e[0] for e in exp], name
        assert list(val) == [e[1] for e in exp], name
        # the start voxel is never written (R14)
        v0 = [math.floor(c) for c in _nums(o)]
        if all(0 <= v0[a] < (gx, gy, gz)[a] for a in range(3)):
            assert ms[v0[2], v0[1], v0[0]] == before[v0[2], v0[1], v0[0]], name


def test_axis_ray_processes_exactly_vox_depth_voxels():
    for vd in [1, 2, 7, 43, 160]:
        xyz, val = oracle.trace_ray([0.5, 0.5, 0.5], [0, 0, vd], vd * vd, (1, 1, 1))
        assert len(xyz) == vd
        assert list(xyz[:, 2]) == list(range(1, vd + 1))


def _brute_walk(o, d, m2):
    """Voxels a straight segment enters, ordered by entry time, by a slab test
    of every voxel box in a bounding region (double precision); then cut by the
    integer termination of Alg. 2.  Returns (voxels, min gap between entry
    times) -- callers skip near-ties."""
    o = np.asarray(o, float)
    d = np.asarray(d, float)
    L = math.sqrt(m2) + 3.0
    tend = L / np.linalg.norm(d)
    end = o + tend * d
    lo = np.floor(np.minimum(o, end)).astype(int) - 2
    hi = np.floor(np.maximum(o, end)).astype(int) + 2
    axes = [np.arange(lo[a], hi[a] + 1) for a in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    V = np.stack([X, Y, Z], -1).reshape(-1, 3).astype(float)
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = (V - o) / d
        t1 = (V + 1.0 - o) / d
    tn = np.where(d == 0, np.where((o >= V) & (o < V + 1), -np.inf, np.inf), np.minimum(t0, t1))
    tf = np.where(d == 0, np.where((o >= V) & (o < V + 1), np.inf, -np.inf), np.maximum(t0, t1))
    t_in = tn.max(1)
    t_out = tf.min(1)
    hit = (t_out > t_in) & (t_out > 0) & (t_in < tend)
    order = np.argsort(t_in[hit])
    vox = V[hit][order].astype(int)
    tins = t_in[hit][order]
    v0 = np.floor(o).astype(int)
    assert tuple(vox[0]) == tuple(v0)
    vox, tins = vox[1:], tins[1:]
    out = []
    for v in vox:
        out.append(tuple(v))
        if int(((v - v0) ** 2).sum()) >= m2:
            break
    k = len(out)
    t = tins[:k + 1]
    gaps = np.diff(t) / np.maximum(1.0, np.abs(t[1:]))
    return out, (gaps.min() if gaps.size else 1.0)


def test_walk_matches_brute_force_segment_boxes():
    """Generic poses: the walk equals the ordered list of voxels the segment
    passes through (Amanatides & Woo visit every voxel the ray touches)."""
    rng = np.random.default_rng(11)
    checked = skipped = 0
    for _ in range(400):
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                      [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                      [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
        vd = int(rng.integers(3, 25))
        a, b = int(rng.integers(-vd, vd + 1)), int(rng.integers(-vd, vd + 1))
        dirf = (R.astype(np.float32) @ np.array([a, b, vd], np.float32)).astype(np.float32)
        o = (rng.uniform(-20, 20, 3)).astype(np.float32)
        m2 = a * a + b * b + vd * vd
        exp, gap = _brute_walk(o.astype(float), dirf.astype(float), m2)
        if gap < 1e-4:
            skipped += 1
            continue
        xyz, _ = oracle.trace_ray(o, dirf, m2, (1, 1, 1))
        assert [tuple(v) for v in xyz] == exp
        checked += 1
    assert checked >= 300, (checked, skipped)


def test_walk_is_six_connected_and_terminates_by_length():
    rng = np.random.default_rng(5)
    for _ in range(200):
        o = rng.uniform(-5, 5, 3).astype(np.float32)
        d = rng.standard_normal(3).astype(np.float32) * 10
        m2 = int(rng.integers(1, 900))
        xyz, _ = oracle.trace_ray(o, d, m2, (1, 1, 1))
        v0 = np.floor(o).astype(int)
        path = np.vstack([v0, xyz])
        steps = np.abs(np.diff(path, axis=0)).sum(1)
        assert np.all(steps == 1)                       # face-adjacent
        dist2 = ((xyz - v0) ** 2).sum(1)
        assert dist2[-1] >= m2 and np.all(dist2[:-1] < m2)
        assert np.all(np.diff(dist2) > 0)               # strictly increasing


def test_traced_wins_over_free_in_any_ray_order():
    """The paper leaves concurrent free / traced writes undefined (Sec. IV-C);
    the reading used here is order-independent: any post-hit visit makes the
    voxel "unknown and traced".  Find two rays that share a voxel X, one
    before its hit and one after, and run them in both orders."""
    dims = (24, 24, 3)
    o = [0.5, 12.5, 1.5]
    found = None
    for occ_y in range(8, 17):
        for occ_x in range(3, 12):
            ms = np.zeros(dims[::-1], np.uint8)
            ms[1, occ_y, occ_x] = oracle.OCCUPIED
            walks = {}
            for b in range(-12, 13):
                xyz, val = oracle.trace_ray(o, [20, b, 0], 400 + b * b, dims, ms.copy())
                walks[b] = (xyz, val)
            pre = {}
            post = {}
            for b, (xyz, val) in walks.items():
                for v, s in zip(map(tuple, xyz), val):
                    (pre if s == oracle.FREE else post if s == oracle.TRACED else {}).setdefault(v, b)
            both = [v for v in pre if v in post and pre[v] != post[v]]
            if both:
                found = (occ_x, occ_y, both[0], pre[both[0]], post[both[0]])
                break
        if found:
            break
    assert found is not None
    occ_x, occ_y, X, b_free, b_traced = found
    results = []
    for order in [(b_free, b_traced), (b_traced, b_free)]:
        ms = np.zeros(dims[::-1], np.uint8)
        ms[1, occ_y, occ_x] = oracle.OCCUPIED
        for b in order:
            oracle.trace_ray(o, [20, b, 0], 400 + b * b, dims, ms)
        results.append(ms[X[2], X[1], X[0]])
    assert results == [oracle.TRACED, oracle.TRACED]


# --------------------------------------------- Alg. 3 merge, shift (IV-D/E)

def test_merge_truth_table():
    ms = np.repeat(np.arange(4, dtype=np.uint8), 3)
    loc = np.tile(np.arange(3, dtype=np.uint8), 4)
    out = loc.copy()
    oracle.merge(ms, out)
    expect = {0: None, 1: 1, 2: 2, 3: 0}      # unknown keeps, traced -> unknown
    for m, l0, l1 in zip(ms, loc, out):
        assert l1 == (l0 if expect[m] is None else expect[m])


def test_shift_closed_form_and_composition():
    rng = np.random.default_rng(3)
    loc = rng.integers(0, 3, (5, 6, 7)).astype(np.uint8)    # gz, gy, gx
    for _ in range(30):
        d = rng.integers(-8, 9, 3)
        out = oracle.shift(loc, d)
        expect = np.zeros_like(loc)
        gz, gy, gx = loc.shape
        for z in range(gz):
            for y in range(gy):
                for x in range(gx):
                    sx, sy, sz = x + d[0], y + d[1], z + d[2]
                    if 0 <= sx < gx and 0 <= sy < gy and 0 <= sz < gz:
                        expect[z, y, x] = loc[sz, sy, sx]
        assert np.array_equal(out, expect)
        e = rng.integers(-4, 5, 3)
        two = oracle.shift(out, e)
        one = oracle.shift(loc, d + e)
        zz, yy, xx = np.meshgrid(*[np.arange(n) for n in loc.shape], indexing="ij")
        keep = ((xx + e[0] >= 0) & (xx + e[0] < gx) & (yy + e[1] >= 0) & (yy + e[1] < gy)
                & (zz + e[2] >= 0) & (zz + e[2] < gz))
        assert np.array_equal(two[keep], one[keep])
        assert np.all(two[~keep] == 0)


def test_center_offset_recentres():
    dims = (100, 100, 50)
    s = np.float32(0.1)
    origin = np.array([-5.0, -5.0, -1.5], np.float32)
    assert oracle.center_offset(dims, s, origin, [0.05, 0.05, 1.05]) == (0, 0, 0)
    assert oracle.center_offset(dims, s, origin, [0.35, -0.25, 1.05]) == (3, -3, 0)


def test_origin_after_shift():
    o = oracle.origin([-5.0, -2.5, 0.0], [4, -3, 0], 0.25)
    assert list(o) == [-4.0, -3.25, 0.0]

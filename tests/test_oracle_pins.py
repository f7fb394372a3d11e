"""Pins for the CPU oracle: each check compares it with something other than itself.

* exact rational arithmetic (the first-hit definition without rounding);
* closed forms (axis-aligned rays through voxel centres, empty and full volumes);
* the edge-case suite (parallel axes, lattice corners, clipping, NaN, subnormals, ...);
* the paper's worked facts (Morton figure, table of formats, layout word counts,
  extents of the composition example, whole-level de-duplication never growing size);
* losslessness (decoding the built buffer returns the input occupancy) and
  cross-format invariance (every format of one volume gives the flat-DDA hits).
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from tests.exact import first_hit_exact

GOLD = os.path.join(os.path.dirname(__file__), "golden")
INF = float("inf")


def ray(o, d, tmin=0.0, tmax=INF):
    return np.array([[o[0], o[1], o[2], tmin, d[0], d[1], d[2], tmax]], dtype=np.float32)


def codes_of(voxels):
    v = np.array(sorted(voxels), dtype=np.int32).reshape(-1, 3)
    c = W.morton_encode(v) if len(v) else np.zeros(0, np.uint64)
    return np.sort(c)


def dense_of(voxels, ext):
    g = np.zeros((1 << ext[2], 1 << ext[1], 1 << ext[0]), np.uint8)
    for x, y, z in voxels:
        g[z, y, x] = 1
    return g


def as_tuple(h):
    return (int(h[0]), int(h[1]), int(h[2]), float(np.int32(h[3]).view(np.float32)))


# Formats for an 8^3 volume covering every 1-, 2- and 3-level type sequence.
SPECS_8 = [
    "R(3,3,3)", "S(3)", "G(3)",
    "R(1,1,1) R(2,2,2)", "R(2,2,2) S(1)", "R(1,1,1) G(2)", "S(1) R(2,2,2)", "S(2) S(1)", "S(1) G(2)",
    "G(2) R(1,1,1)", "G(1) S(2)", "G(1) G(2)",
    "R(1,1,1) R(1,1,1) R(1,1,1)", "R(1,1,1) S(1) G(1)", "R(1,1,1) G(1) S(1)", "S(1) R(1,1,1) G(1)",
    "S(1) S(1) S(1)", "S(1) G(1) R(1,1,1)", "G(1) R(1,1,1) S(1)", "G(1) G(1) G(1)", "G(1) S(1) R(1,1,1)",
    "R(1,1,1) R(1,1,1) S(1)", "S(1) S(1) R(1,1,1)", "G(1) G(1) R(1,1,1)", "R(1,1,1) G(1) G(1)",
    "G(2) R(1,1,1) --whole-level-dedup", "R(1,1,1) G(2) --whole-level-dedup", "G(1) G(1) G(1) --whole-level-dedup",
]


# ------------------------------------------------------------------ paper facts
def test_morton_order_matches_paper_figure():
    rows = [list(map(int, l.split())) for l in open(os.path.join(GOLD, "morton_figure_4x4.txt"))
            if l.strip() and not l.startswith("#")]
    for idx, col, row in rows:
        # The 2-D figure is the z = 0 slice: its visit order is the Morton order of (x=col, y=row).
        code = W.morton_encode(np.array([[col, row, 0]], np.int32))[0]
        two_d = int(code)
        # Drop the (zero) z bits to get the 2-D interleave index.
        bits = [(two_d >> (3 * b)) & 1 for b in range(4)] + [(two_d >> (3 * b + 1)) & 1 for b in range(4)]
        idx2 = sum(bits[b] << (2 * b) for b in range(4)) + sum(bits[4 + b] << (2 * b + 1) for b in range(4))
        assert idx2 == idx


def test_table_of_formats_extents():
    """Every signature of the evaluated-format table represents its stated grid side."""
    n = 0
    for line in open(os.path.join(GOLD, "table_formats.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        label, side, spec = line.split(maxsplit=2)
        spec = spec.strip()
        nlev, ext = oracle.parse(spec)
        assert ext == (int(side).bit_length() - 1,) * 3, (label, spec, ext)
        assert nlev == spec.count("(")
        n += 1
    assert n == 40


def test_composition_example_extents():
    # R(1,0,2) R(2,2,2): a 2x1x4 grid of 4x4x4 sub-volumes is 8x4x16 voxels (Sec. 3.2).
    assert oracle.parse("R(1,0,2) R(2,2,2)") == (2, (3, 2, 4))


@pytest.mark.parametrize("spec", ["R(2,2,2) S(1,1,1)", "S(2) R(1,0,2)", "R(1,1,1) R(1,2,1)", "Q(3)", "R(3,3)",
                                  "S(0)", "", "R(3,3,3) --bogus"])
def test_parse_rejects(spec):
    with pytest.raises(oracle.OracleError):
        oracle.parse(spec)


def test_layout_word_counts_single_voxel():
    """Word counts of the layout figure: SVO node 2 words, SVDAG node 1 + #children, leaf 1."""
    c = codes_of([(5, 2, 7)])
    for L in (1, 2, 3):
        v = oracle.Volume("S(%d)" % L, c if L == 3 else codes_of([(1, 0, 1)]))
        assert v.num_words == 1 + 2 * (L + 1)  # root pointer + one 2-word node per depth incl. leaf
        g = oracle.Volume("G(%d)" % L, c if L == 3 else codes_of([(1, 0, 1)]))
        assert g.num_words == 1 + 2 * L + 1  # internal nodes: mask + 1 pointer; leaf: 1 word
    r = oracle.Volume("R(3,3,3)", c)
    assert r.num_words == 1 + 512
    w = r.words()
    assert w[0] == 1 and w[1 + 5 + 8 * (2 + 8 * 7)] == 0xFFFFFFFF and np.count_nonzero(w[1:]) == 1


def test_layout_full_volume_counts():
    full = np.arange(512, dtype=np.uint64)
    g = oracle.Volume("G(3)", full)
    # De-duplication leaves one node per depth: 3 internal nodes of 9 words, one 1-word leaf.
    assert g.num_words == 1 + 3 * 9 + 1
    s = oracle.Volume("S(3)", full)
    assert s.num_words == 1 + 2 * (1 + 8 + 64 + 512)
    r = oracle.Volume("R(1,1,1) R(2,2,2)", full)
    assert r.num_words == 1 + 8 + 8 * 64
    e = oracle.Volume("G(3)", np.zeros(0, np.uint64))
    assert e.num_words == 1 and e.words()[0] == 0


def test_whole_level_dedup_never_grows():
    codes = W.scene_shell(11, 6, 6, 3, 1.0)
    for spec in ["R(3,3,3) G(3)", "R(2,2,2) G(4)", "S(2) G(4)", "R(4,4,4) G(2)", "G(2) G(2) G(2)"]:
        a = oracle.Volume(spec, codes).num_words
        b = oracle.Volume(spec + " --whole-level-dedup", codes).num_words
        assert b <= a, spec
    # a repetitive volume must actually shrink: identical sub-volumes share nodes
    rep = codes_of([(x, y, z) for x in range(16) for y in range(16) for z in range(16) if (x + y + z) % 3 == 0])
    a = oracle.Volume("R(2,2,2) G(2)", rep).num_words
    b = oracle.Volume("R(2,2,2) G(2) --whole-level-dedup", rep).num_words
    assert b < a


def test_build_rejects_bad_codes():
    with pytest.raises(oracle.OracleError):
        oracle.Volume("R(3,3,3)", np.array([5, 3], np.uint64))
    with pytest.raises(oracle.OracleError):
        oracle.Volume("R(3,3,3)", np.array([5, 5], np.uint64))
    with pytest.raises(oracle.OracleError):
        oracle.Volume("R(1,0,2) R(2,2,2)", codes_of([(0, 4, 0)]))  # y beyond extent 4


# ------------------------------------------------------------------ losslessness
@pytest.mark.parametrize("spec", SPECS_8)
def test_decode_is_lossless(spec):
    codes = W.scene_bernoulli(7, 3, 3, 3, 0.2)
    assert np.array_equal(oracle.Volume(spec, codes).decode(), codes)


def test_decode_noncubic():
    codes = W.scene_bernoulli(3, 3, 2, 4, 0.15)
    for spec in ["R(1,0,2) R(2,2,2)", "R(1,0,2) S(2)", "R(1,0,2) G(1) R(1,1,1)", "R(3,2,4)"]:
        assert np.array_equal(oracle.Volume(spec, codes).decode(), codes), spec


# ------------------------------------------------------------------ exact arithmetic
def test_brute_force_matches_exact_arithmetic():
    rng = np.random.default_rng(0)
    checked = 0
    for seed in range(6):
        codes = W.scene_bernoulli(100 + seed, 3, 3, 3, 0.08)
        vox = [tuple(v) for v in W.morton_decode(codes)]
        rays = W.random_rays(200 + seed, (8, 8, 8), 120)
        # plus rays from outside, aimed at the box
        o = rng.uniform(-6, 14, size=(60, 3))
        tgt = rng.uniform(0, 8, size=(60, 3))
        d = tgt - o
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        out = np.concatenate([o, np.zeros((60, 1)), d, np.full((60, 1), np.inf)], axis=1).astype(np.float32)
        rays = np.concatenate([rays, out])
        got = oracle.brute(codes, (3, 3, 3), rays)
        for r, h in zip(rays, got):
            v, te, margin = first_hit_exact(vox, (3, 3, 3), r)
            if margin < 1e-5:
                continue
            checked += 1
            if v is None:
                assert h[0] == -1
            else:
                assert tuple(h[:3]) == v
                t = float(np.int32(h[3]).view(np.float32))
                assert abs(t - float(te)) <= 1e-6 * max(1.0, abs(float(te)))
    assert checked > 800


def test_noncubic_exact():
    codes = W.scene_bernoulli(5, 3, 2, 4, 0.05)
    vox = [tuple(v) for v in W.morton_decode(codes)]
    rays = W.random_rays(9, (8, 4, 16), 200)
    got = oracle.Volume("R(1,0,2) G(1) R(1,1,1)", codes).trace(rays)
    for r, h in zip(rays, got):
        v, te, margin = first_hit_exact(vox, (3, 2, 4), r)
        if margin < 1e-5:
            continue
        assert (tuple(h[:3]) == v) if v is not None else h[0] == -1


# ------------------------------------------------------------------ closed forms
@pytest.mark.parametrize("spec", ["R(3,3,3)", "S(3)", "G(3)", "R(1,1,1) S(1) R(1,1,1)", "G(2) R(1,1,1)"])
def test_axis_rays_through_voxel_centres(spec):
    codes = W.scene_bernoulli(17, 3, 3, 3, 0.12)
    occ = dense_of([tuple(v) for v in W.morton_decode(codes)], (3, 3, 3))  # occ[z, y, x]
    vol = oracle.Volume(spec, codes)
    rays, expect = [], []
    for j in range(8):
        for k in range(8):
            for axis in range(3):
                for sgn in (1, -1):
                    o = [0.0, 0.0, 0.0]
                    d = [0.0, 0.0, 0.0]
                    others = [a for a in range(3) if a != axis]
                    o[others[0]] = j + 0.5
                    o[others[1]] = k + 0.5
                    o[axis] = -3.0 if sgn > 0 else 11.0
                    d[axis] = float(sgn)
                    rays.append(ray(o, d)[0])
                    idx = [0, 0, 0]
                    idx[others[0]] = j
                    idx[others[1]] = k
                    line = []
                    for i in range(8):
                        idx[axis] = i
                        line.append(occ[idx[2], idx[1], idx[0]])
                    order = range(8) if sgn > 0 else range(7, -1, -1)
                    hit = next((i for i in order if line[i]), None)
                    if hit is None:
                        expect.append(None)
                    else:
                        idx[axis] = hit
                        t = (hit + 3.0) if sgn > 0 else (11.0 - (hit + 1))
                        expect.append((idx[0], idx[1], idx[2], t))
    got = vol.trace(np.array(rays))
    for g, e in zip(got, expect):
        if e is None:
            assert g[0] == -1 and math.isinf(as_tuple(g)[3])
        else:
            assert as_tuple(g) == e


def test_empty_and_full_volumes():
    rays = W.random_rays(3, (8, 8, 8), 300)
    empty = np.zeros(0, np.uint64)
    full = np.arange(512, dtype=np.uint64)
    for spec in ["R(3,3,3)", "S(3)", "G(1) G(2)", "R(1,1,1) S(1) R(1,1,1)"]:
        assert np.all(oracle.Volume(spec, empty).trace(rays)[:, 0] == -1)
        h = oracle.Volume(spec, full).trace(rays)
        # origins are inside the grid and tmin = 0: the hit is the origin's voxel at t = 0
        assert np.array_equal(h[:, :3], np.floor(rays[:, :3]).astype(np.int32))
        assert np.all(h[:, 3].view(np.float32) == 0.0)


def test_ray_missing_the_box_and_tmax_clip():
    full = oracle.Volume("S(3)", np.arange(512, dtype=np.uint64))
    assert full.trace(ray((-5, -5, -5), (-1, 0.3, 0.2)))[0, 0] == -1        # pointing away
    assert full.trace(ray((-5, 20, 3), (1, 0, 0)))[0, 0] == -1              # passes beside it
    assert full.trace(ray((-5, 3.5, 3.5), (1, 0, 0), tmax=4.99))[0, 0] == -1  # stops short
    assert as_tuple(full.trace(ray((-5, 3.5, 3.5), (1, 0, 0), tmax=5.01))[0]) == (0, 3, 3, 5.0)


# ------------------------------------------------------------------ edge-case suite
EDGE_VOX = [(5, 3, 2), (5, 2, 2), (2, 1, 1), (1, 2, 1), (3, 3, 3), (2, 2, 2), (6, 6, 6), (0, 7, 0), (7, 0, 7)]
EDGE_SPECS = ["R(3,3,3)", "S(3)", "G(3)", "R(1,1,1) G(2)", "S(1) R(1,1,1) S(1)", "G(2) R(1,1,1) --whole-level-dedup"]

# (ray, expected) with expected = (x, y, z, t) or None; derived by hand.
EDGE_CASES = [
    # E1: lying in the integer plane y = 3 (parallel axis): cell floor(3.0) = 3
    (ray((-1.0, 3.0, 2.5), (1, 0, 0)), (5, 3, 2, 6.0)),
    # E2: through lattice corners, diagonal steps only; (2,1,1)/(1,2,1) are touched at a point
    (ray((-0.5, -0.5, -0.5), (1, 1, 1)), (2, 2, 2, 2.5)),
    # E3: origin inside an occupied voxel: t = t0 = tmin
    (ray((2.5, 2.5, 2.5), (1, 0.3, 0.2)), (2, 2, 2, 0.0)),
    # E4: origin inside an empty voxel of the grid, marching +x along y=3.5, z=3.5
    (ray((0.25, 3.5, 3.5), (1, 0, 0)), (3, 3, 3, 2.75)),
    # E5: tmin beyond the first voxel skips it; tmax before the next one misses
    (ray((0.25, 2.5, 2.5), (1, 0, 0), tmin=2.0), (2, 2, 2, 2.0)),
    (ray((0.25, 2.5, 2.5), (1, 0, 0), tmin=2.9), (5, 2, 2, 4.75)),
    (ray((-1.0, 2.5, 2.5), (1, 0, 0), tmin=7.5), None),
    (ray((-1.0, 6.5, 6.5), (1, 0, 0), tmax=6.999), None),
    (ray((-1.0, 6.5, 6.5), (1, 0, 0), tmax=7.001), (6, 6, 6, 7.0)),
    (ray((-1.0, 6.5, 6.5), (1, 0, 0), tmax=7.0), None),  # intervals are half-open at tmax
    # E6: negative direction and -0.0 components (parallel)
    (ray((9.0, 3.5, 2.5), (-1, -0.0, 0.0)), (5, 3, 2, 3.0)),
    (ray((7.5, 0.5, 9.0), (-0.0, 0.0, -2.0)), (7, 0, 7, 0.5)),
    # E7: subnormal component: 1/d overflows, so the axis is parallel
    (ray((-2.0, 3.5, 2.5), (1, 1e-45, 0)), (5, 3, 2, 7.0)),
    # E8: grazing the boundary face x = N with d_x = 0: outside the half-open grid
    (ray((8.0, -1.0, 0.5), (0, 1, 0)), None),
    (ray((7.999, -1.0, 7.5), (0, 1, 0)), (7, 0, 7, 1.0)),
    # E9: NaN components miss
    (ray((float("nan"), 3.5, 2.5), (1, 0, 0)), None),
    (ray((-1.0, 3.5, 2.5), (float("nan"), 0, 0)), None),
    (ray((-1.0, 3.5, 2.5), (1, 0, 0), tmax=float("nan")), None),
    # E10: far origin, |o| = 2^20: plane times are exact integers here
    (ray((-1048576.0, 3.5, 2.5), (1, 0, 0)), (5, 3, 2, 1048581.0)),
    # zero direction misses
    (ray((3.5, 3.5, 3.5), (0, 0, 0)), None),
]


@pytest.mark.parametrize("spec", EDGE_SPECS)
def test_edge_suite(spec):
    codes = codes_of(EDGE_VOX)
    vol = oracle.Volume(spec, codes)
    rays = np.concatenate([r for r, _ in EDGE_CASES])
    got = vol.trace(rays)
    brute = oracle.brute(codes, (3, 3, 3), rays)
    flat = oracle.flat_dda(dense_of(EDGE_VOX, (3, 3, 3)), (3, 3, 3), rays)
    for i, ((r, e), g) in enumerate(zip(EDGE_CASES, got)):
        if e is None:
            assert g[0] == -1 and g[1] == -1 and g[2] == -1, (i, g)
            assert math.isinf(as_tuple(g)[3])
        else:
            assert as_tuple(g) == e, (i, as_tuple(g), e)
    assert np.array_equal(got, brute)
    assert np.array_equal(got, flat)


# ------------------------------------------------------------------ cross-format invariance
@pytest.mark.parametrize("seed", [1, 2])
def test_every_format_matches_flat_dda(seed):
    codes = W.scene_bernoulli(seed, 3, 3, 3, 0.06 * seed)
    occ = dense_of([tuple(v) for v in W.morton_decode(codes)], (3, 3, 3))
    rays = np.concatenate([W.random_rays(seed, (8, 8, 8), 400), W.camera_rays(seed, 0, (8, 8, 8), 24, 16),
                           W.camera_rays(seed, 1, (8, 8, 8), 24, 16)])
    flat = oracle.flat_dda(occ, (3, 3, 3), rays)
    brute, ties = oracle.brute(codes, (3, 3, 3), rays, return_ties=True)
    assert ties.max() == 0  # the first hit is unique
    assert np.array_equal(flat, brute)
    for spec in SPECS_8:
        assert np.array_equal(oracle.Volume(spec, codes).trace(rays), flat), spec


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_split_buffers_match_flat_dda(seed):
    """One buffer per level (the oracle's answer past 2^32 words, forced here by
    --depth-buffers): every type sequence of the 8^3 suite, and DF levels, give the flat
    DDA's hits, decode losslessly, and hold the single buffer's words (each level's buffer
    starts with a reserved word, so pointer values differ)."""
    codes = W.scene_bernoulli(seed, 3, 3, 3, 0.06 * seed)
    occ = dense_of([tuple(v) for v in W.morton_decode(codes)], (3, 3, 3))
    rays = np.concatenate([W.random_rays(seed, (8, 8, 8), 400), W.camera_rays(seed, 0, (8, 8, 8), 24, 16),
                           np.concatenate([r for r, _ in EDGE_CASES])])
    flat = oracle.flat_dda(occ, (3, 3, 3), rays)
    for spec in SPECS_8 + ["D(1,1,1,2) R(2,2,2)", "D(2,2,2,3) S(1)", "R(1,1,1) D(1,1,1,2) G(1)"]:
        one, split = oracle.Volume(spec, codes), oracle.Volume(spec + " --depth-buffers", codes)
        assert split.split_buffers() and not one.split_buffers()
        assert np.array_equal(split.trace(rays), flat), spec
        assert np.array_equal(split.decode(), codes), spec
        nlev = len(spec.split(" --")[0].split())
        assert split.num_words == one.num_words + nlev  # plus one reserved word per level


def test_shell_scene_formats_agree():
    codes = W.scene_shell(4, 6, 8, 4, 1.4)
    occ = dense_of([tuple(v) for v in W.morton_decode(codes)], (6, 6, 6))
    rays = np.concatenate([W.camera_rays(4, 0, (64, 64, 64), 48, 32), W.random_rays(4, (64, 64, 64), 1500)])
    flat = oracle.flat_dda(occ, (6, 6, 6), rays)
    assert (flat[:, 0] >= 0).mean() > 0.1
    for spec in ["R(2,2,2) S(2) R(2,2,2)", "G(6)", "S(6)", "G(4) R(2,2,2) --whole-level-dedup", "S(2) G(2) R(2,2,2)",
                 "R(3,3,3) R(3,3,3)", "R(2,2,2) G(4)"]:
        assert np.array_equal(oracle.Volume(spec, codes).trace(rays), flat), spec


def test_multithreaded_trace_matches_single():
    codes = W.scene_solid_noise(1)
    vol = oracle.Volume("R(2,2,2) S(2) R(2,2,2)", codes)
    rays = W.camera_rays(1, 0, (64, 64, 64), 64, 48)
    assert np.array_equal(vol.trace(rays, 1), vol.trace(rays, 4))


# ------------------------------------------------------------------ distance-field levels
def _l1_brute(occ, cap):
    """Capped L1 distance from every cell to the nearest occupied cell, by exhaustive search."""
    nz, ny, nx = occ.shape
    pts = np.argwhere(occ)  # (z, y, x)
    out = np.full(occ.shape, cap, np.int64)
    if len(pts) == 0:
        return out
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                d = np.abs(pts - np.array([z, y, x])).sum(axis=1).min()
                out[z, y, x] = min(cap, d)
    return out


@pytest.mark.parametrize("p,cap", [(0.02, 6), (0.1, 2), (0.004, 100), (0.3, 1)])
def test_df_distances_brute_force(p, cap):
    """A one-level DF grid stores (terminating integer, capped L1 distance) per cell (Sec. 3.3)."""
    codes = W.scene_bernoulli(int(p * 1000) + cap, 3, 2, 4, p)
    occ = dense_of([tuple(v) for v in W.morton_decode(codes)], (3, 2, 4))
    w = oracle.Volume("D(3,2,4,%d)" % cap, codes).words()
    assert w[0] == 1 and len(w) == 1 + 2 * occ.size
    term = w[1::2].reshape(occ.shape)
    dist = w[2::2].reshape(occ.shape)
    assert np.array_equal(term != 0, occ.astype(bool))
    assert np.array_equal(dist, _l1_brute(occ, cap))


def test_df_distances_two_levels():
    """Above a lower level, the distance counts non-empty sub-volumes of the DF grid (Sec. 4.1)."""
    codes = W.scene_bernoulli(21, 4, 4, 4, 0.004)
    sub = np.zeros((4, 4, 4), np.uint8)  # occupancy of the 4x4x4 grid of 4^3 sub-volumes
    for x, y, z in W.morton_decode(codes):
        sub[z >> 2, y >> 2, x >> 2] = 1
    w = oracle.Volume("D(2,2,2,5) R(2,2,2)", codes).words()
    root = int(w[0])  # children are written before the grid that points at them
    dist = w[root + 1:root + 2 * 64:2].reshape(4, 4, 4)
    assert np.array_equal(dist, _l1_brute(sub, 5))


def test_df_full_and_single_voxel():
    full = oracle.Volume("D(2,2,2,6)", np.arange(64, dtype=np.uint64)).words()
    assert np.all(full[2::2] == 0)
    one = oracle.Volume("D(3,3,3,30)", codes_of([(0, 0, 0)])).words()
    d = one[2::2].reshape(8, 8, 8)
    z, y, x = np.mgrid[0:8, 0:8, 0:8]
    assert np.array_equal(d, x + y + z)  # closed form: distance to the corner voxel


DF_SPECS = ["D(3,3,3,6)", "D(3,3,3,1)", "D(1,1,1,2) R(2,2,2)", "R(1,1,1) D(2,2,2,3)", "D(2,2,2,6) S(1)",
            "G(1) D(2,2,2,4)", "D(1,1,1,3) D(1,1,1,3) D(1,1,1,3)", "S(1) D(1,1,1,1) G(1)",
            "D(2,2,2,6) G(1) --whole-level-dedup"]


@pytest.mark.parametrize("spec", DF_SPECS)
def test_df_decode_is_lossless(spec):
    codes = W.scene_bernoulli(7, 3, 3, 3, 0.2)
    assert np.array_equal(oracle.Volume(spec, codes).decode(), codes)


@pytest.mark.parametrize("seed,p", [(1, 0.01), (2, 0.03), (3, 0.12)])
def test_df_formats_match_flat_dda(seed, p):
    """Skipping by the stored distance never skips an occupied cell: hits equal the flat DDA."""
    codes = W.scene_bernoulli(seed + 40, 3, 3, 3, p)
    occ = dense_of([tuple(v) for v in W.morton_decode(codes)], (3, 3, 3))
    rays = np.concatenate([W.random_rays(seed, (8, 8, 8), 600), W.camera_rays(seed, 0, (8, 8, 8), 24, 16)])
    flat = oracle.flat_dda(occ, (3, 3, 3), rays)
    for spec in DF_SPECS:
        assert np.array_equal(oracle.Volume(spec, codes).trace(rays), flat), spec


@pytest.mark.parametrize("spec", ["D(3,3,3,6)", "D(1,1,1,3) R(2,2,2)", "S(1) D(2,2,2,6)"])
def test_df_edge_suite(spec):
    codes = codes_of(EDGE_VOX)
    got = oracle.Volume(spec, codes).trace(np.concatenate([r for r, _ in EDGE_CASES]))
    for i, ((r, e), g) in enumerate(zip(EDGE_CASES, got)):
        if e is None:
            assert g[0] == -1, (i, g)
        else:
            assert as_tuple(g) == e, (i, as_tuple(g), e)


def test_df_shell_scene():
    codes = W.scene_shell(4, 6, 8, 4, 1.4)
    occ = dense_of([tuple(v) for v in W.morton_decode(codes)], (6, 6, 6))
    rays = np.concatenate([W.camera_rays(4, 0, (64, 64, 64), 48, 32), W.random_rays(4, (64, 64, 64), 1500)])
    flat = oracle.flat_dda(occ, (6, 6, 6), rays)
    for spec in ["D(6,6,6,6)", "D(4,4,4,6) R(2,2,2)", "D(3,3,3,6) D(3,3,3,6)", "D(2,2,2,6) G(4) --wld"]:
        assert np.array_equal(oracle.Volume(spec, codes).trace(rays), flat), spec

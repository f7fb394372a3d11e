"""GPU parity at the benchmark's full sizes and launch configuration, on sampled rays.

* 512^3 surface volume, nine formats: every 1080p view is traced in full on the GPU
  (as the benchmark does); the oracle, built in the same format, traces a seeded sample
  of each view; one low-resolution view is compared in full. The plain Raw format
  R(9,9,9) is checked against the oracle's flat DDA, which is that format's traversal.
* 2048^3 surface volume, both formats: 1080p primary rays traced in full on the GPU,
  a sample checked against the oracle; bounce rays are generated from the ORACLE's hits
  on that sample and traced by both. The oracle traces the same volume built as G(11):
  every format of one volume has the same first hits (pinned on the CPU), and G(11) is
  the format the oracle builds in seconds at this size.
* The distance-field formats of the table at 512^3 and one at 2048^3, the same way
  (D(9,9,9,6) against the flat DDA, like R(9,9,9)).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import compare
from workloads import configs as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2410_14128_amd as H
    H.lib()
    return H


@pytest.fixture(scope="module")
def surf512():
    cfg = C.SURF512
    codes = C.scene(cfg)
    views = [C.primary_rays(cfg, v) for v in range(cfg["views"])]
    return cfg, codes, views


def _dense(codes, log2n):
    n = 1 << log2n
    xyz = W.morton_decode(codes)
    g = np.zeros((n, n, n), np.uint8)
    g[xyz[:, 2], xyz[:, 1], xyz[:, 0]] = 1
    return g


def _trace_full(vol, rays):
    import torch
    d = torch.from_numpy(rays).cuda()
    h = vol.trace(d)
    torch.cuda.synchronize()
    return h.cpu().numpy()


@pytest.mark.parametrize("spec", C.SURF512["specs"] + C.SURF512_DF)
def test_surface512(H, surf512, spec):
    cfg, codes, views = surf512
    vol = H.Volume(spec, codes)
    if spec.startswith("R(9,9,9)") or spec.startswith("D(9,9,9"):
        dense = _dense(codes, 9)
        ref_fn = lambda r: oracle.flat_dda(dense, (9, 9, 9), r)
    else:
        ov = oracle.Volume(spec, codes)
        ref_fn = lambda r: ov.trace(r, nthreads=8)
    rng = np.random.default_rng(2024)
    hits_total = 0
    for j, rays in enumerate(views):
        got = _trace_full(vol, rays)
        idx = rng.choice(len(rays), 6000, replace=False)
        assert compare(got[idx], ref_fn(rays[idx]), f"{spec} view {j}") == 0
        hits_total += int((got[:, 0] >= 0).sum())
    assert hits_total > 0.1 * sum(len(r) for r in views)
    small = C.primary_rays(cfg, 1, 240, 135)
    assert compare(_trace_full(vol, small), ref_fn(small), f"{spec} 240x135") == 0


@pytest.fixture(scope="module")
def surf2048():
    cfg = C.SURF2048
    codes = C.scene(cfg)
    prim = C.primary_rays(cfg, 0)
    ov = oracle.Volume("G(11) --whole-level-dedup", codes)
    rng = np.random.default_rng(77)
    idx = np.sort(rng.choice(len(prim), 20000, replace=False))
    ref_p = ov.trace(prim[idx], nthreads=8)
    bounce, src = W.bounce_rays(cfg["bounce_seed"], prim[idx], ref_p)
    ref_b = ov.trace(bounce, nthreads=8)
    rnd = W.random_rays(5, (2048,) * 3, 20000)
    ref_r = ov.trace(rnd, nthreads=8)
    return cfg, codes, prim, idx, ref_p, bounce, ref_b, rnd, ref_r


@pytest.mark.parametrize("spec", C.SURF2048["specs"] + ["G(7) R(4,4,4) --whole-level-dedup --restart-sv",
                                                        "D(4,4,4,6) G(7) --whole-level-dedup"])
def test_surface2048(H, surf2048, spec):
    cfg, codes, prim, idx, ref_p, bounce, ref_b, rnd, ref_r = surf2048
    vol = H.Volume(spec, codes)
    got = _trace_full(vol, prim)
    assert compare(got[idx], ref_p, f"{spec} primary") == 0
    assert (ref_p[:, 0] >= 0).mean() > 0.1 and len(bounce) > 2000
    assert compare(_trace_full(vol, bounce), ref_b, f"{spec} bounce") == 0
    assert compare(_trace_full(vol, rnd), ref_r, f"{spec} random") == 0


@pytest.mark.parametrize("sd", [dict(split=8, split_budget=32), dict(split=16, split_budget=64),
                                dict(split=4, split_budget=16, lds_depths=3),
                                dict(split=64, split_budget=32, split_rounds=2),
                                dict(split=16, split_budget=8, split_rounds=4, lds_depths=3),
                                dict(split=64, split_budget=2)], ids=lambda d: str(d))
def test_surface2048_split_schedule(H, surf2048, sd):
    """Whole 1080p frames traced with split walks equal the plain schedule bit for bit. With a
    2-step budget most of the 2 M primary rays survive, so the second launch's K falls to 1
    (more survivors than half its grid's lanes)."""
    import torch
    cfg, codes, prim, idx, ref_p, bounce, ref_b, rnd, ref_r = surf2048
    vol = H.Volume("G(7) R(4,4,4) --whole-level-dedup", codes)
    sc = H.schedule(**sd)
    plain = _trace_full(vol, prim)
    got = vol.trace(torch.from_numpy(prim).cuda(), sched=sc)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert np.array_equal(got, plain)
    assert compare(got[idx], ref_p, f"split {sd} primary") == 0
    b_full, _ = W.bounce_rays(cfg["bounce_seed"], prim, plain)
    bp = _trace_full(vol, b_full)
    bs = vol.trace(torch.from_numpy(b_full).cuda(), sched=sc)
    torch.cuda.synchronize()
    assert np.array_equal(bs.cpu().numpy(), bp)
    for rays, ref, what in ((bounce, ref_b, "bounce"), (rnd, ref_r, "random")):
        g = vol.trace(torch.from_numpy(rays).cuda(), sched=sc)
        torch.cuda.synchronize()
        assert compare(g.cpu().numpy(), ref, f"split {sd} {what}") == 0


@pytest.mark.parametrize("sd", [dict(steal=1, steal_len=8), dict(steal=4, steal_len=16),
                                dict(steal=8, steal_len=64),
                                dict(steal=4, steal_len=8, lds_depths=3),
                                dict(steal=1, steal_len=2, steal_idle=16, interleave=1),
                                dict(interleave=1)], ids=lambda d: str(d))
def test_surface2048_steal_schedule(H, surf2048, sd):
    """Whole 1080p frames, primary and bounce rays, traced with walks split among the idle
    lanes of each wave (and with rays interleaved across waves, the benchmark's schedule of
    the one-frame bounce launch) equal the plain schedule bit for bit, and sampled rays the
    oracle."""
    import torch
    cfg, codes, prim, idx, ref_p, bounce, ref_b, rnd, ref_r = surf2048
    vol = H.Volume("G(7) R(4,4,4) --whole-level-dedup", codes)
    sc = H.schedule(**sd)
    plain = _trace_full(vol, prim)
    got = vol.trace(torch.from_numpy(prim).cuda(), sched=sc)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert np.array_equal(got, plain)
    assert compare(got[idx], ref_p, f"steal {sd} primary") == 0
    b_full, _ = W.bounce_rays(cfg["bounce_seed"], prim, plain)
    bp = _trace_full(vol, b_full)
    bs = vol.trace(torch.from_numpy(b_full).cuda(), sched=sc)
    torch.cuda.synchronize()
    assert np.array_equal(bs.cpu().numpy(), bp)
    for rays, ref, what in ((bounce, ref_b, "bounce"), (rnd, ref_r, "random")):
        g = vol.trace(torch.from_numpy(rays).cuda(), sched=sc)
        torch.cuda.synchronize()
        assert compare(g.cpu().numpy(), ref, f"steal {sd} {what}") == 0


def test_counting_variant_matches_plain(H, surf512):
    import torch
    cfg, codes, views = surf512
    vol = H.Volume("G(6) R(3,3,3) --whole-level-dedup", codes)
    rays = torch.from_numpy(views[0][::97].copy()).cuda()
    plain = vol.trace(rays)
    hits, logt, cnt = vol.trace_count(rays, cap=2048)
    torch.cuda.synchronize()
    assert torch.equal(plain, hits)
    c = cnt.cpu().numpy()
    assert c.max() <= 2048
    # a ray that misses the root box reads nothing; every other ray reads word 0 first
    entered = c > 0
    assert entered.mean() > 0.3 and np.all(c[hits.cpu().numpy()[:, 0] >= 0] >= 2)
    lg = logt.cpu().numpy()
    nw = vol.info()["num_words"]
    for i in np.nonzero(entered)[0][::101]:
        assert lg[i, 0] == 0  # the root pointer
        assert np.all(lg[i, : c[i]] < nw)


def test_max_extent_volume(H):
    """The largest supported side (2^16): a few voxels in G(16), rays from outside."""
    pts = np.array([[0, 0, 0], [65535, 65535, 65535], [40000, 123, 65000], [32768, 32767, 32768]], np.int32)
    codes = np.sort(W.morton_encode(pts))
    spec = "G(16)"
    rays = []
    for p in pts:
        c = p.astype(np.float64) + 0.5
        o = c + np.array([-70000.0, 3000.0, -1234.0])
        d = (c - o) / np.linalg.norm(c - o)
        rays.append([o[0], o[1], o[2], 0, d[0], d[1], d[2], np.inf])
    rays = np.array(rays, np.float32)
    got = _trace_full(H.Volume(spec, codes), rays)
    ref = oracle.brute(codes, (16, 16, 16), rays)
    assert compare(got, ref, "max extent") == 0
    assert np.all(got[:, 0] >= 0)


# ------------------------------------------------------------------ the paper's 40 formats
@pytest.mark.parametrize("label,k,spec", [t for t in C.TABLE_FORMATS if t[1] == 9], ids=lambda x: str(x))
def test_table_format_512(H, surf512, label, k, spec):
    """Every 512^3 row of the format table against the flat DDA (the same occupancy)."""
    cfg, codes, views = surf512
    dense = _dense(codes, 9)
    vol = H.Volume(C.table_spec(spec), codes)
    rays = views[label % 4]
    got = _trace_full(vol, rays)
    idx = np.random.default_rng(label).choice(len(rays), 4000, replace=False)
    assert compare(got[idx], oracle.flat_dda(dense, (9, 9, 9), rays[idx]), f"row {label} {spec}") == 0


@pytest.mark.parametrize("label,k,spec", [t for t in C.TABLE_FORMATS if t[1] == 11], ids=lambda x: str(x))
def test_table_format_2048(H, surf2048, label, k, spec):
    """Every 2048^3 row of the format table against the oracle's G(11) hits (every format
    of one volume has the same first hits)."""
    cfg, codes, prim, idx, ref_p, bounce, ref_b, rnd, ref_r = surf2048
    vol = H.Volume(C.table_spec(spec), codes)
    got = _trace_full(vol, prim)
    assert compare(got[idx], ref_p, f"row {label} {spec} primary") == 0
    assert compare(_trace_full(vol, bounce), ref_b, f"row {label} {spec} bounce") == 0
    assert compare(_trace_full(vol, rnd[:5000]), ref_r[:5000], f"row {label} {spec} random") == 0

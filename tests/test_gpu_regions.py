"""Buffers with per-depth regions (the paper's multiple buffers with indirection, Sec. 3.3):
each depth's nodes in their own region, pointers relative to the region they point into,
so a format may pass 2^32 words.

* Small volumes built with --depth-buffers trace bit for bit like the single-buffer layout
  under every schedule, and read the very same words (the counting kernel's logs match:
  nodes sit at the same places, only pointer values differ).
* A volume past 2^32 words (R(3,4,4) R(7,7,7) R(5,5,5) over 32768 x 65536 x 65536: a
  depth of pointer grids just below 2^32 words and a depth of bricks, 4.31 G words in all)
  builds, uploads and traces at parity with the oracle, which traces the same voxels built
  as R(3,4,4) G(12) (every format of one volume has the same first hits, pinned on the CPU).
* Batches and the server hold such volumes beside others (the batched launch then runs the
  region-aware kernel), and device construction builds them word for word like the host.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2410_14128_amd as H
    H.lib()
    return H


SCHEDS = [dict(), dict(steal=1, steal_len=2, steal_idle=16), dict(steal=2, steal_len=1), dict(split=8, split_budget=4),
          dict(split=64, split_budget=2, split_rounds=2), dict(persistent=1, refill=8, inner=4), dict(sort=1, sort_bits=3),
          dict(lds_depths=2), dict(stack_depth=2)]


@pytest.mark.parametrize("spec", ["G(4) R(3,3,3) --whole-level-dedup", "S(3) R(4,4,4)", "R(2,2,2) S(2) G(3)",
                                  "D(3,3,3,6) R(2,2,2) R(2,2,2)", "S(2) G(2) R(3,3,3) --restart-sv", "R(3,3,3) R(4,4,4)"])
def test_regions_trace_like_one_buffer(H, spec):
    import torch
    codes = W.scene_shell(12, 7, 8, 4, 1.4)
    rays = np.concatenate([W.random_rays(12, (128,) * 3, 20000), W.camera_rays(12, 0, (128,) * 3, 160, 120)])
    one, reg = H.Volume(spec, codes), H.Volume(spec + " --depth-buffers", codes)
    assert reg.info()["depth_buffers"]
    d = torch.from_numpy(rays).cuda()
    want = one.trace(d, sched=H.schedule())
    for sd in SCHEDS:
        try:
            got = reg.trace(d, sched=H.schedule(**sd))
        except H.HvfError as e:  # a staged prefix larger than the LDS limit is refused
            assert "lds_depths" in sd and e.name == "HVF_E_INPUT"
            continue
        torch.cuda.synchronize()
        assert torch.equal(got, want), f"{spec} {sd}"
    idx = np.arange(0, len(rays), 11)
    ov = oracle.Volume(spec + " --depth-buffers", codes)  # the oracle's own buffers per level
    assert ov.split_buffers()
    assert compare(want.cpu().numpy()[idx], ov.trace(rays[idx], nthreads=8), spec) == 0
    small = torch.from_numpy(rays[:3000]).cuda()
    h1, l1, c1 = one.trace_count(small, cap=512)
    h2, l2, c2 = reg.trace_count(small, cap=512)
    torch.cuda.synchronize()
    assert torch.equal(h1, h2) and torch.equal(c1, c2)
    mask = torch.arange(512, device="cuda")[None, :] < c1[:, None]
    assert torch.equal(torch.where(mask, l1, 0), torch.where(mask, l2, 0))


def test_regions_in_batches_and_server(H):
    """Volumes with per-depth regions batch and serve beside volumes without them (the
    batched launch then runs the region-aware kernel with every node kind): every batch's
    and request's hits equal hvf_trace of that volume alone."""
    import torch
    specs = ["G(4) R(3,3,3) --whole-level-dedup --depth-buffers", "S(3) R(4,4,4)", "R(2,2,2) S(2) G(3) --depth-buffers",
             "S(2) G(2) R(3,3,3) --paper-layout", "D(3,3,3,6) R(2,2,2) R(2,2,2) --depth-buffers", "G(7)"]
    vols, rays, refs = [], [], []
    for j, spec in enumerate(specs):
        codes = W.scene_shell(30 + j, 7, 8, 4, 1.4)
        r = np.concatenate([W.random_rays(40 + j, (128,) * 3, 3000), W.camera_rays(40 + j, j % 3, (128,) * 3, 80, 60)])
        v = H.Volume(spec, codes)
        d = torch.from_numpy(r).cuda()
        vols.append(v)
        rays.append(d)
        refs.append(v.trace(d, sched=H.schedule()))
    torch.cuda.synchronize()
    for order in (list(range(len(specs))), [1, 3, 5, 0, 2, 4], [0]):
        bt = H.Batch([vols[j] for j in order], [rays[j] for j in order])
        got = bt.run()
        torch.cuda.synchronize()
        for j, g in zip(order, got):
            assert torch.equal(g, refs[j]), (order, specs[j])
        bt.close()
    srv = H.Server(256 << 20, max_slots=8, max_steps=2)
    ids = [srv.add_volume(v) for v in vols]
    host = [r.cpu().numpy() for r in rays]
    reqs = [(j, srv.submit(ids[j], host[j][k::3])) for j in range(len(specs)) for k in range(3)]
    for j, rid in reqs:
        h, _ = srv.wait(rid)
        k = [r for jj, r in reqs if jj == j].index(rid)
        assert np.array_equal(h, refs[j].cpu().numpy()[k::3]), specs[j]
    srv.close()


def test_paper_layout_regions_refused_by_device_build(H):
    import torch
    codes = W.scene_shell(12, 6, 6, 2, 1.4)
    with pytest.raises(H.HvfError) as e:
        H.Volume.from_device("G(3) R(3,3,3) --paper-layout --depth-buffers", torch.from_numpy(codes.view(np.int64)).cuda())
    assert e.value.name == "HVF_E_UNSUPPORTED"


def test_volume_past_2_32_words(H):
    import torch
    rng = np.random.default_rng(2032)
    # R(3,4,4) R(7,7,7) R(5,5,5) over 32768 x 65536 x 65536: 2,047 of the 2,048 top cells
    # hold ten random voxels each, so the depth of 128^3-cell pointer grids takes
    # 2,047 x 2^21 words (just below 2^32) and the bricks 20,470 x 1,024 more.
    top = np.array([(x, y, z) for z in range(16) for y in range(16) for x in range(8) if (x, y, z) != (7, 15, 15)])
    xyz = (np.repeat(top, 10, axis=0) << 12) + rng.integers(0, 1 << 12, size=(len(top) * 10, 3))
    codes = np.unique(W.morton_encode(xyz.astype(np.int32)))
    spec = "R(3,4,4) R(7,7,7) R(5,5,5)"
    print(f"building {spec} over {len(codes)} voxels", flush=True)
    v = H.Volume(spec, codes)
    info = v.info()
    print(f"built: {info['num_words']} words, depth offsets {info['depth_offset'][:info['num_depths']]}", flush=True)
    assert info["depth_buffers"] and info["num_words"] > (1 << 32) and info["extent_log2"] == (15, 16, 16)
    v.upload()
    # rays aimed at occupied voxels from random points of the volume, and random rays
    ext = (1 << 15, 1 << 16, 1 << 16)
    tgt = W.morton_decode(codes[rng.choice(len(codes), 3000, replace=False)]).astype(np.float64) + 0.5
    org = rng.uniform(0, 1, size=(3000, 3)) * np.array(ext)
    dirs = tgt - org
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    aimed = np.zeros((3000, 8), np.float32)
    aimed[:, 0:3], aimed[:, 4:7], aimed[:, 7] = org, dirs, np.inf
    rays = np.ascontiguousarray(np.concatenate([aimed, W.random_rays(2032, ext, 3000)]))
    d = torch.from_numpy(rays).cuda()
    got = v.trace(d, sched=H.schedule())
    stolen = v.trace(d, sched=H.schedule(steal=1, steal_len=2, steal_idle=16))
    # the same rays in a batched launch beside a small volume (64-bit word indices there too)
    small = H.Volume("G(3) R(2,2,2)", W.scene_shell(5, 5, 4, 2, 1.4))
    ds = torch.from_numpy(W.random_rays(5, (32,) * 3, 2000)).cuda()
    bt = H.Batch([small, v, small], [ds, d, ds])
    bh = bt.run()
    torch.cuda.synchronize()
    assert torch.equal(got, stolen) and torch.equal(bh[1], got)
    assert torch.equal(bh[0], small.trace(ds)) and torch.equal(bh[2], bh[0])
    bt.close()
    # the same volume built on the device (the builder picks per-depth regions by itself)
    print("device build", flush=True)
    dv = H.Volume.from_device(spec, torch.from_numpy(codes.view(np.int64)).cuda())
    assert dv.info()["depth_buffers"] and dv.info()["num_words"] == info["num_words"]
    dgot = dv.trace(d, sched=H.schedule())
    torch.cuda.synchronize()
    assert torch.equal(dgot, got)
    wh = v.words()
    wd = dv.words()
    assert np.array_equal(wh, wd)
    del wh, wd, dgot
    dv.close()
    del dv
    got = got.cpu().numpy()
    assert (got[:3000, 0] >= 0).mean() > 0.5
    v.close()
    del v
    ref = oracle.Volume("R(3,4,4) G(12)", codes).trace(rays, nthreads=8)
    assert compare(got, ref, "past 2^32 words") == 0

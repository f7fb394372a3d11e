"""Batched persistent launch: every batch's hits equal hvf_trace of that batch alone
(bit-exact), which the oracle pins on samples; hipGraph replays are checked one by one."""
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
def cases(H):
    import torch
    cfg = dict(C.BATCHED)
    cfg["kmax"] = 8  # keep the oracle builds small
    out = []
    for i in range(14):
        spec, k, codes, rays = C.batched_case(cfg, i, scale_rays=0.03)
        v = H.Volume(spec, codes)
        d = torch.from_numpy(rays).cuda()
        ref = v.trace(d, sched=H.schedule())
        out.append((spec, k, codes, rays, v, d, ref))
    # distance-field levels (the batch then runs the all-kinds kernel)
    for spec, k in (("D(2,2,2,4) G(3) --whole-level-dedup", 5), ("D(3,3,3,6) D(3,3,3,6)", 6)):
        codes = W.scene_shell(90 + k, k, 6, 2, 1.4)
        rays = np.concatenate([W.random_rays(k, (1 << k,) * 3, 3000), W.camera_rays(k, 0, (1 << k,) * 3, 64, 48)])
        v = H.Volume(spec, codes)
        d = torch.from_numpy(rays).cuda()
        out.append((spec, k, codes, rays, v, d, v.trace(d, sched=H.schedule())))
    # an empty volume and an empty ray batch
    v = H.Volume("G(3) R(2,2,2)", np.zeros(0, np.uint64))
    r = W.random_rays(1, (32,) * 3, 1000)
    d = torch.from_numpy(r).cuda()
    out.append(("G(3) R(2,2,2)", 5, np.zeros(0, np.uint64), r, v, d, v.trace(d)))
    e = torch.empty((0, 8), dtype=torch.float32, device="cuda")
    out.append(("S(3)", 3, np.zeros(0, np.uint64), np.zeros((0, 8), np.float32), H.Volume("S(3)", np.arange(5, dtype=np.uint64)), e,
                torch.empty((0, 4), dtype=torch.int32, device="cuda")))
    torch.cuda.synchronize()
    return out


def test_plain_reference_matches_oracle(H, cases):
    rng = np.random.default_rng(3)
    for spec, k, codes, rays, v, d, ref in cases:
        if len(rays) == 0:
            continue
        idx = rng.choice(len(rays), min(2000, len(rays)), replace=False)
        got = ref.cpu().numpy()[idx]
        want = oracle.Volume(spec, codes).trace(rays[idx], nthreads=8)
        assert compare(got, want, spec) == 0


@pytest.mark.parametrize("opts", [dict(), dict(refill=1, inner=1), dict(refill=64, inner=64, blocks_per_cu=1),
                                  dict(use_graph=0)], ids=["default", "refill1", "refill64-bpc1", "nograph"])
def test_batched_equals_per_volume(H, cases, opts):
    import torch
    b = H.Batch([c[4] for c in cases], [c[5] for c in cases], opts=H.batch_opts(**opts))
    for h in b.hits:
        h.fill_(-7)
    b.run()
    torch.cuda.synchronize()
    for (spec, *_, ref), h in zip(cases, b.hits):
        assert torch.equal(h, ref), spec
    b.close()


def test_graph_replays_each_correct(H, cases):
    import torch
    b = H.Batch([c[4] for c in cases], [c[5] for c in cases])
    for rep in range(4):
        for h in b.hits:
            h.fill_(rep - 9)                            # eager work between replays
        x = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager kernels
        b.run()
        torch.cuda.synchronize()
        for (spec, *_, ref), h in zip(cases, b.hits):
            assert torch.equal(h, ref), (rep, spec)
        assert torch.isfinite(x)
    b.close()


def test_batch_autotune_keeps_results(H, cases):
    import torch
    b = H.Batch([c[4] for c in cases], [c[5] for c in cases])
    o = b.autotune()
    assert 1 <= o.refill <= 64 and o.inner >= 1
    for h in b.hits:
        h.fill_(-3)
    b.run()
    torch.cuda.synchronize()
    for (spec, *_, ref), h in zip(cases, b.hits):
        assert torch.equal(h, ref), spec
    b.close()


@pytest.mark.parametrize("family", [["G(3) R(2,2,2)", "G(4) R(3,3,3) --whole-level-dedup", "G(2) G(2) R(2,2,2)"],
                                    ["S(3) R(2,2,2)", "S(4) R(3,3,3)", "S(2) S(1) R(2,2,2)"],
                                    ["S(2) G(2) R(2,2,2)", "G(3) R(2,2,2)", "S(3) R(3,3,3)"],
                                    ["R(2,2,2) R(3,3,3)", "R(3,3,3) R(2,2,2)", "R(1,1,1) R(2,2,2) R(2,2,2)"]],
                         ids=["svdag-brick", "svo-brick", "octree-brick", "raw-brick"])
def test_batches_of_one_family(H, family):
    """Batches whose volumes all fall in one brick-final family run that family's own
    batched kernel; every batch's hits still equal hvf_trace of that batch alone, and the
    server's steps over such volumes too."""
    import torch
    vols, rays, refs = [], [], []
    for i, spec in enumerate(family * 2):
        k = H.Volume(spec).info()["extent_log2"][0]
        codes = W.scene_shell(200 + i, k, max(4, (1 << k) // 16), 2, 1.4)
        v = H.Volume(spec, codes)
        r = np.concatenate([W.random_rays(300 + i, (1 << k,) * 3, 2000), W.camera_rays(300 + i, 0, (1 << k,) * 3, 48, 32)])
        d = torch.from_numpy(r).cuda()
        vols.append(v)
        rays.append(d)
        refs.append(v.trace(d, sched=H.schedule()).clone())
    b = H.Batch(vols, rays)
    for h in b.hits:
        h.fill_(-7)
    b.run()
    torch.cuda.synchronize()
    for spec, h, ref in zip(family * 2, b.hits, refs):
        assert torch.equal(h, ref), spec
    b.close()
    srv = H.Server(64 << 20, max_slots=16, max_steps=2)
    ids = [srv.add_volume(v) for v in vols]
    rid = [srv.submit(ids[i], rays[i].cpu().numpy()) for i in range(len(vols))]
    for r, ref in zip(rid, refs):
        assert np.array_equal(srv.wait(r)[0], ref.cpu().numpy())
    srv.close()

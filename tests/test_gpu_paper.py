"""Tracing the paper's own word layout (--paper-layout) on the GPU through the C-ABI.

Hits must equal the oracle's (hit flag and xyz bit-exact, t within 1e-6 relative) and,
being the same first-hit query, equal those of the library's own layout bit for bit.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import compare, gpu_trace
from tests.test_oracle_pins import DF_SPECS, EDGE_CASES, EDGE_SPECS, EDGE_VOX, SPECS_8, codes_of
from tests.test_paper_layout import MORE
from workloads import configs as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2410_14128_amd as H
    H.lib()
    return H


def rays_for(ext, seed=3):
    return np.concatenate([W.camera_rays(seed, seed % 3, ext, 96, 80), W.random_rays(seed, ext, 12000),
                           np.concatenate([r for r, _ in EDGE_CASES])]).astype(np.float32)


@pytest.mark.parametrize("spec", SPECS_8 + DF_SPECS + MORE)
def test_paper_layout_matches_oracle_and_own_layout(H, spec):
    ex = H.Volume(spec).info()["extent_log2"]
    ext = tuple(1 << e for e in ex)
    for seed, p in ((1, 0.05), (2, 0.4)):
        codes = W.scene_bernoulli(seed, ex[0], ex[1], ex[2], p)
        rays = rays_for(ext, seed)
        got = gpu_trace(H.Volume(spec + " --paper-layout", codes), rays)
        assert compare(got, oracle.Volume(spec, codes).trace(rays, nthreads=8), f"{spec} paper") == 0
        assert np.array_equal(got, gpu_trace(H.Volume(spec, codes), rays)), spec


@pytest.mark.parametrize("spec", EDGE_SPECS + ["D(3,3,3,6)", "S(1) D(2,2,2,6)"])
def test_paper_layout_edge_suite(H, spec):
    codes = codes_of(EDGE_VOX)
    rays = np.concatenate([r for r, _ in EDGE_CASES])
    got = gpu_trace(H.Volume(spec + " --paper-layout", codes), rays)
    assert compare(got, oracle.Volume(spec, codes).trace(rays), spec) == 0


def test_paper_layout_surface_512(H):
    cfg = C.SURF512
    codes = C.scene(cfg)
    view = C.primary_rays(cfg, 0)
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(len(view), 20000, replace=False))
    for spec in ["S(9)", "G(9) --whole-level-dedup", "G(6) R(3,3,3) --whole-level-dedup", "R(3,3,3) R(3,3,3) R(3,3,3)",
                 "D(4,4,4,6) G(5) --whole-level-dedup"]:
        got = gpu_trace(H.Volume(spec + " --paper-layout", codes), view)
        assert np.array_equal(got, gpu_trace(H.Volume(spec, codes), view)), spec
        assert compare(got[idx], oracle.Volume(spec, codes).trace(view[idx], nthreads=8), spec) == 0


@pytest.mark.parametrize("sd", [dict(persistent=1, refill=8, inner=4), dict(sort=1, sort_bits=3),
                                dict(split=8, split_budget=3), dict(split=64, split_budget=2, split_rounds=2),
                                dict(steal=1, steal_len=1), dict(steal=4, steal_len=8)],
                         ids=lambda d: str(d))
def test_paper_layout_schedules(H, sd):
    import torch
    codes = W.scene_shell(3, 7, 8, 4, 1.4)
    rays = rays_for((128,) * 3)
    d = torch.from_numpy(rays).cuda()
    for spec in ["G(4) R(3,3,3) --whole-level-dedup --paper-layout", "R(2,2,2) S(2) D(3,3,3,5) --paper-layout",
                 "S(3) G(4) --paper-layout"]:
        v = H.Volume(spec, codes)
        plain = v.trace(d)
        got = v.trace(d, sched=H.schedule(**sd))
        torch.cuda.synchronize()
        assert torch.equal(got, plain), spec


def test_paper_layout_counting_and_refusals(H):
    import torch
    codes = W.scene_shell(3, 7, 8, 4, 1.4)
    v = H.Volume("G(4) R(3,3,3) --whole-level-dedup --paper-layout", codes)
    d = torch.from_numpy(rays_for((128,) * 3)).cuda()
    hits, log, cnt = v.trace_count(d, cap=256)
    torch.cuda.synchronize()
    assert torch.equal(hits, v.trace(d))
    hit = hits[:, 0] >= 0
    assert bool(hit.any()) and int(cnt[hit].min()) >= 2  # a hit reads word 0 and the nodes on its way
    for sd in (dict(stack_depth=2), dict(lds_depths=1)):
        with pytest.raises(H.HvfError) as e:
            v.trace(d, sched=H.schedule(**sd))
        assert e.value.name == "HVF_E_INPUT"
    sc = v.autotune(d)  # skips the schedules this layout refuses
    assert sc.stack_depth == 0 and sc.lds_depths == 0


def test_paper_layout_batched_and_served(H):
    """Volumes in the paper's layout, alone and mixed with the library's own layout (DF
    levels included), in one batched launch and through the server: each batch's hits equal
    its volume's own trace."""
    import torch
    codes = W.scene_shell(3, 7, 8, 4, 1.4)
    specs = ["G(4) R(3,3,3) --whole-level-dedup --paper-layout", "R(2,2,2) S(2) D(3,3,3,5) --paper-layout",
             "S(3) G(4) --paper-layout", "G(4) R(3,3,3) --whole-level-dedup", "D(2,2,2,4) S(5)"]
    vols = [H.Volume(sp, codes) for sp in specs]
    rays = [torch.from_numpy(W.random_rays(10 + i, (128,) * 3, 3000 + 997 * i)).cuda() for i in range(len(vols))]
    want = [v.trace(r) for v, r in zip(vols, rays)]
    torch.cuda.synchronize()
    for group in (vols[:3], vols):
        b = H.Batch(group, rays[:len(group)])
        hits = b.run()
        torch.cuda.synchronize()
        for i, h in enumerate(hits):
            assert torch.equal(h, want[i]), (len(group), specs[i])
        b.close()
    srv = H.Server(1 << 26, max_slots=8, max_steps=2)
    ids = [srv.add_volume(v) for v in vols]
    rid = [srv.submit(ids[i], rays[i].cpu().numpy()) for i in range(len(vols))]
    for i, r in enumerate(rid):
        got = srv.wait(r)[0]
        assert np.array_equal(got, want[i].cpu().numpy()), specs[i]
    srv.close()

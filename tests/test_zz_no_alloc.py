"""The allocation-free split trace (hvf_trace_split_noalloc) against hvf_trace_sched with
the same split schedule, through the C-ABI: two calls in a row, the second with fewer rays,
so the fixed scratch array carries the first call's lists into the second; plus its
refusals (no allocation may happen, so an un-uploaded volume and oversized calls fail)."""
import ctypes

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


def test_noalloc_split_matches_allocating_entry_point(H):
    import torch
    codes = W.scene_shell(3, 7, 8, 4, 1.4)
    spec = "G(4) R(3,3,3) --whole-level-dedup"
    v = H.Volume(spec, codes)
    v.upload()
    ov = oracle.Volume(spec, codes)
    big = np.concatenate([W.camera_rays(3, 0, (128,) * 3, 320, 240), W.random_rays(3, (128,) * 3, 60000)])
    small = np.ascontiguousarray(W.random_rays(4, (128,) * 3, 5000))
    for sd in (dict(split=8, split_budget=4), dict(split=64, split_budget=2, split_rounds=2)):
        sc = H.schedule(**sd)
        for rays in (big, small):  # the second call is smaller: the array keeps the first call's contents
            d = torch.from_numpy(rays).cuda()
            want = v.trace(d, sched=sc)
            got = torch.full((len(rays), 4), 7, dtype=torch.int32, device="cuda")
            v.trace_split_noalloc(d, got, sc)
            torch.cuda.synchronize()
            assert torch.equal(got, want), f"{sd} {len(rays)} rays"
            idx = np.arange(0, len(rays), 7)
            assert compare(got.cpu().numpy()[idx], ov.trace(rays[idx], nthreads=8), f"noalloc {sd}") == 0


def test_noalloc_refusals(H):
    import torch
    codes = W.scene_shell(3, 7, 8, 4, 1.4)
    v = H.Volume("G(4) R(3,3,3) --whole-level-dedup", codes)
    d = torch.from_numpy(W.random_rays(5, (128,) * 3, 1000)).cuda()
    hits = torch.empty((1000, 4), dtype=torch.int32, device="cuda")
    sc = H.schedule(split=8, split_budget=4)
    with pytest.raises(H.HvfError) as e:  # not uploaded: the upload would allocate
        v.trace_split_noalloc(d, hits, sc)
    assert e.value.name == "HVF_E_STATE"
    v.upload()
    with pytest.raises(H.HvfError) as e:  # not a split schedule
        v.trace_split_noalloc(d, hits, H.schedule())
    assert e.value.name == "HVF_E_INPUT"
    st = H.lib().hvf_trace_split_noalloc(v.handle, d.data_ptr(), H.NOALLOC_MAX_RAYS + 1, hits.data_ptr(),
                                         ctypes.byref(sc), None)
    assert H.STATUS[st] == "HVF_E_INPUT"
    assert b"at most" in H.lib().hvf_last_error()
    v.trace_split_noalloc(d, hits, sc)
    torch.cuda.synchronize()
    assert torch.equal(hits, v.trace(d))

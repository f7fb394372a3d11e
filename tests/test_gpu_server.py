"""Serving: each request's hits are the same alone and in the mix (bit-exact), equal to
hvf_trace of the request (which the oracle pins on samples); admission respects the
memory budget and makes requests wait when it is small."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import compare, gpu_trace

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2410_14128_amd as H
    H.lib()
    return H


@pytest.fixture(scope="module")
def world(H):
    vols = []
    for i, (log2n, spec) in enumerate([(6, "G(2) R(4,4,4) --whole-level-dedup"), (7, "G(3) R(4,4,4) --whole-level-dedup"),
                                       (8, "G(4) R(4,4,4) --whole-level-dedup"), (7, "R(3,3,3) S(4)")]):
        n = 1 << log2n
        codes = W.scene_shell(50 + i, log2n, max(4, n // 16), max(1, n // 64), 1.4)
        vols.append((spec, log2n, codes, H.Volume(spec, codes)))
    rng = np.random.default_rng(5)
    reqs = []
    for k in range(40):
        vi = int(rng.integers(0, len(vols)))
        res = [(64, 64), (128, 96), (320, 180), (7, 3)][int(rng.integers(0, 4))]
        n = 1 << vols[vi][1]
        rays = W.camera_rays(900 + k, 0, (n,) * 3, *res)
        if k % 5 == 0:
            rays = np.concatenate([rays, W.random_rays(k, (n,) * 3, 500)])
        reqs.append((vi, np.ascontiguousarray(rays)))
    reqs.append((0, np.zeros((0, 8), np.float32)))  # an empty request
    return vols, reqs


def _serve(H, world, budget, slots, steps, gaps=False):
    vols, reqs = world
    srv = H.Server(budget, max_slots=slots, max_steps=steps)
    ids = [srv.add_volume(v[3]) for v in vols]
    import time
    rid = []
    for k, (vi, rays) in enumerate(reqs):
        rid.append(srv.submit(ids[vi], rays))
        if gaps and k % 7 == 0:
            time.sleep(0.002)
    out = [srv.wait(r)[0] for r in rid]
    st = srv.stats()
    srv.close()
    return out, st


def test_alone_equals_mix_equals_trace(H, world):
    vols, reqs = world
    alone = []
    srv = H.Server(64 << 20, max_slots=1, max_steps=1)  # one request at a time, in order
    ids = [srv.add_volume(v[3]) for v in vols]
    for vi, rays in reqs:
        alone.append(srv.wait(srv.submit(ids[vi], rays))[0])
    srv.close()
    mix, st = _serve(H, world, 256 << 20, 64, 3, gaps=True)
    assert st["completed"] == len(reqs) and st["steps"] >= 2
    for k, ((vi, rays), a, m) in enumerate(zip(reqs, alone, mix)):
        assert np.array_equal(a, m), k
        if len(rays):
            assert np.array_equal(m, gpu_trace(vols[vi][3], rays)), k
    # oracle spot check of a few requests
    for k in range(0, len(reqs), 9):
        vi, rays = reqs[k]
        if len(rays) == 0:
            continue
        idx = np.arange(0, len(rays), max(1, len(rays) // 400))
        spec, log2n, codes, _ = vols[vi]
        assert compare(mix[k][idx], oracle.Volume(spec, codes).trace(rays[idx], nthreads=8), f"request {k}") == 0


def test_small_budget_forces_admission_waits(H, world):
    vols, reqs = world
    biggest = max(len(r) for _, r in reqs)
    budget = 3 * (48 * biggest + 512)
    out, st = _serve(H, world, budget, 64, 2)
    assert st["admission_waits"] > 0
    assert st["peak_bytes"] <= st["budget_bytes"] == ((budget + 255) // 256) * 256
    for (vi, rays), m in zip(reqs, out):
        if len(rays):
            assert np.array_equal(m, gpu_trace(vols[vi][3], rays))


def test_oversize_request_rejected(H, world):
    vols, reqs = world
    srv = H.Server(1 << 16, max_slots=4, max_steps=1)
    vid = srv.add_volume(vols[0][3])
    with pytest.raises(H.HvfError) as e:
        srv.submit(vid, W.random_rays(1, (64,) * 3, 5000))
    assert e.value.name == "HVF_E_NOMEM"
    srv.close()


def test_pinned_rays_and_held_results(H, world):
    import torch
    vols, reqs = world
    srv = H.Server(128 << 20, max_slots=16, max_steps=2)
    ids = [srv.add_volume(v[3]) for v in vols]
    pinned, rid = [], []
    for vi, rays in reqs[:12]:
        p = torch.empty(rays.shape, dtype=torch.float32, pin_memory=True).numpy()
        p[...] = rays
        pinned.append(p)
        rid.append(srv.submit(ids[vi], p, hold=True))
    for (vi, rays), r in zip(reqs[:12], rid):
        h, lat = srv.wait(r)
        assert h is None and lat >= 0
        got = srv.result(r).copy()
        assert np.array_equal(got, gpu_trace(vols[vi][3], rays))
        srv.release(r)
    with pytest.raises(H.HvfError):
        srv.result(rid[0])  # released
    st = srv.stats()
    assert st["completed"] == 12 and st["peak_bytes"] <= st["budget_bytes"]
    srv.close()


def test_failed_step_completes_its_requests_with_the_error(H, world):
    """A step that fails at launch (forced from the host) finishes its requests with
    HVF_E_DEVICE: the wait reports the error instead of stale hits, the caller's hit array
    is left untouched, the request's memory and slot are returned, and the server then
    refuses new requests."""
    vols, reqs = world
    srv = H.Server(1 << 24, max_slots=8, max_steps=2)
    vid = srv.add_volume(vols[0][3])
    rays = np.ascontiguousarray(W.camera_rays(7, 0, (64,) * 3, 32, 32))
    ok = np.full((len(rays), 4), 7, np.int32)
    srv.wait(srv.submit(vid, rays, ok))
    assert np.array_equal(ok, gpu_trace(vols[0][3], rays))
    srv.fail_steps(1)
    bad = np.full((len(rays), 4), 7, np.int32)
    rid = srv.submit(vid, rays, bad)
    with pytest.raises(H.HvfError) as e:
        srv.wait(rid)
    assert e.value.name == "HVF_E_DEVICE"
    assert (bad == 7).all()
    with pytest.raises(H.HvfError) as e:
        srv.poll(rid)
    assert e.value.name == "HVF_E_DEVICE"
    with pytest.raises(H.HvfError) as e:
        srv.submit(vid, rays, bad)
    assert e.value.name == "HVF_E_DEVICE"
    st = srv.stats()
    assert st["completed"] == 1
    srv.close()

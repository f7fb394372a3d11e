"""Oracle-checked parity of the batched and served workloads at their full stated sizes.

* Batched: all 64 volumes of the batched workload (sides 2^6 to 2^10, random 2- and
  3-level hybrid formats) with their full ray batches (22 M rays, up to 2 M per batch) in
  one graph-captured persistent launch. Every batch equals hvf_trace of that batch alone
  (plain schedule), and a seeded sample of 2,000 rays per batch equals the oracle, which
  traces each volume built as G(k) --whole-level-dedup: every format of one volume has the
  same first hits (pinned on the CPU), and G(k) is the format the oracle builds quickly.
* Served: one 2048^3 and one 4096^3 volume of the served workload
  (G(k-4) R(4,4,4) --whole-level-dedup) behind the server, with a short stream of requests
  at the served resolutions and their bounce follow-ups; each request's hits are the same
  alone (one request at a time) and in the mix, and equal the oracle on a sample of
  2,000 rays per request.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import compare
from workloads import configs as C

pytestmark = pytest.mark.gpu
THREADS = min(16, len(os.sched_getaffinity(0)))


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2410_14128_amd as H
    H.lib()
    return H


def _oracles(jobs):
    """Oracle volumes built concurrently (the build runs without the GIL)."""
    with ThreadPoolExecutor(THREADS) as ex:
        return list(ex.map(lambda j: oracle.Volume(*j), jobs))


def test_batched_full_config(H):
    import torch
    cfg = C.BATCHED
    cases = [C.batched_case(cfg, i) for i in range(cfg["nvol"])]
    print(f"batched: {len(cases)} volumes, {sum(len(c[3]) for c in cases)} rays", flush=True)
    oras = _oracles([(f"G({k}) --whole-level-dedup", codes) for spec, k, codes, rays in cases])
    vols = [H.Volume(spec, codes) for spec, k, codes, rays in cases]
    d_rays = [torch.from_numpy(rays).cuda() for spec, k, codes, rays in cases]
    b = H.Batch(vols, d_rays)
    b.autotune()
    hits = b.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(2025)
    for i, ((spec, k, codes, rays), v, d, h) in enumerate(zip(cases, vols, d_rays, hits)):
        alone = v.trace(d, sched=H.schedule())
        torch.cuda.synchronize()
        assert torch.equal(h, alone), f"batch {i} {spec}"
        idx = np.sort(rng.choice(len(rays), min(2000, len(rays)), replace=False))
        got = h.cpu().numpy()[idx]
        assert compare(got, oras[i].trace(rays[idx], nthreads=THREADS), f"batch {i} {spec} (2^{k})") == 0
    b.close()


def test_served_full_size_volumes(H):
    import torch
    cfg = C.SERVED
    picks = [13, 15]  # a 2048^3 and a 4096^3 volume
    built = [C.served_volume(cfg, i) for i in picks]
    for spec, k, codes in built:
        print(f"served: {spec} at {1 << k}^3, {len(codes)} voxels", flush=True)
    oras = _oracles([(f"G({k}) --whole-level-dedup", codes) for spec, k, codes in built])
    vols = [H.Volume(spec, codes) for spec, k, codes in built]
    # requests: each volume at every served resolution, then bounce follow-ups of half of them
    reqs = []
    for vi, (spec, k, codes) in enumerate(built):
        n = 1 << k
        for j, (w, h) in enumerate(cfg["resolutions"]):
            reqs.append((vi, np.ascontiguousarray(W.camera_rays(cfg["seed"] * 100 + picks[vi], j, (n,) * 3, w, h))))
    for q in list(range(0, len(reqs), 2)):
        vi, prim = reqs[q]
        hp = vols[vi].trace(torch.from_numpy(prim).cuda()).cpu().numpy()
        bounce, _ = W.bounce_rays(cfg["seed"] * 100 + picks[vi] + 7, prim, hp)
        reqs.append((vi, np.ascontiguousarray(bounce)))
    del built
    # alone: one request at a time, in order
    srv = H.Server(1 << 30, max_slots=1, max_steps=1)
    ids = [srv.add_volume(v) for v in vols]
    alone = [srv.wait(srv.submit(ids[vi], rays))[0] for vi, rays in reqs]
    srv.close()
    # mix: every request submitted at once, batched as they are admitted
    srv = H.Server(1 << 30, max_slots=64, max_steps=3)
    ids = [srv.add_volume(v) for v in vols]
    rid = [srv.submit(ids[vi], rays) for vi, rays in reqs]
    mix = [srv.wait(r)[0] for r in rid]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["max_step_requests"] >= 2
    rng = np.random.default_rng(77)
    for q, ((vi, rays), a, m) in enumerate(zip(reqs, alone, mix)):
        assert np.array_equal(a, m), f"request {q}"
        idx = np.sort(rng.choice(len(rays), min(2000, len(rays)), replace=False))
        assert compare(m[idx], oras[vi].trace(rays[idx], nthreads=THREADS), f"request {q}") == 0

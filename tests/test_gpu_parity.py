"""GPU parity: hvf_trace through the C-ABI against the CPU oracle, element by element.

Bar: hit flag and voxel xyz bit-exact; t within 1e-6 relative (observed: bit-exact).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import compare, gpu_trace
from tests.test_oracle_pins import DF_SPECS, EDGE_CASES, EDGE_SPECS, EDGE_VOX, SPECS_8, codes_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2410_14128_amd as H
    H.lib()  # raises if the HIP library is not built: no fallback
    return H


def test_small_config_full_frame(H):
    """64^3 solid spheres + noise, R(2,2,2) S(2) R(2,2,2), 256x256 primary rays."""
    codes = W.scene_solid_noise(1, log2n=6, n_sph=8, rmin=4, rmax=16, noise=0.05)
    spec = "R(2,2,2) S(2) R(2,2,2)"
    rays = W.camera_rays(1, 0, (64, 64, 64), 256, 256)
    got = gpu_trace(H.Volume(spec, codes), rays)
    ref = oracle.Volume(spec, codes).trace(rays, nthreads=8)
    assert compare(got, ref, spec) == 0
    assert 0.2 < (ref[:, 0] >= 0).mean() < 0.9


@pytest.mark.parametrize("spec", SPECS_8 + DF_SPECS)
def test_every_type_sequence_tiny(H, spec):
    for seed in (1, 2, 3):
        codes = W.scene_bernoulli(seed, 3, 3, 3, 0.05 * seed)
        rays = np.concatenate([W.random_rays(seed, (8, 8, 8), 2000), W.camera_rays(seed, 0, (8, 8, 8), 40, 30),
                               np.concatenate([r for r, _ in EDGE_CASES])])
        got = gpu_trace(H.Volume(spec, codes), rays)
        ref = oracle.Volume(spec, codes).trace(rays)
        assert compare(got, ref, f"{spec} seed {seed}") == 0


@pytest.mark.parametrize("spec", EDGE_SPECS + ["D(3,3,3,6)", "D(1,1,1,3) R(2,2,2)", "S(1) D(2,2,2,6)"])
def test_edge_suite(H, spec):
    codes = codes_of(EDGE_VOX)
    rays = np.concatenate([r for r, _ in EDGE_CASES])
    got = gpu_trace(H.Volume(spec, codes), rays)
    ref = oracle.Volume(spec, codes).trace(rays)
    assert compare(got, ref, spec) == 0
    for (r, e), g in zip(EDGE_CASES, got):
        if e is None:
            assert g[0] == -1
        else:
            assert (int(g[0]), int(g[1]), int(g[2]), float(np.int32(g[3]).view(np.float32))) == e


@pytest.mark.parametrize("spec", ["R(1,0,2) R(2,2,2)", "R(1,0,2) S(2)", "R(1,0,2) G(1) R(1,1,1)", "R(3,2,4)",
                                  "D(1,0,2,3) R(2,2,2)", "D(3,2,4,6)", "D(1,0,2,2) D(2,2,2,4)"])
def test_noncubic_top(H, spec):
    codes = W.scene_bernoulli(3, 3, 2, 4, 0.08)
    rays = np.concatenate([W.random_rays(4, (8, 4, 16), 3000), W.camera_rays(4, 0, (8, 4, 16), 48, 32)])
    got = gpu_trace(H.Volume(spec, codes), rays)
    ref = oracle.Volume(spec, codes).trace(rays)
    assert compare(got, ref, spec) == 0


def test_empty_volume_and_empty_batch(H):
    import torch
    v = H.Volume("G(3) R(2,2,2)", np.zeros(0, np.uint64))
    rays = W.random_rays(1, (32, 32, 32), 500)
    got = gpu_trace(v, rays)
    assert np.all(got[:, :3] == -1) and np.all(np.isinf(got[:, 3].view(np.float32)))
    v.trace(torch.empty((0, 8), dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()


def test_deterministic(H):
    codes = W.scene_shell(3, 7, 8, 4, 1.4)
    v = H.Volume("G(4) R(3,3,3) --whole-level-dedup", codes)
    rays = np.concatenate([W.random_rays(5, (128,) * 3, 50000), W.camera_rays(5, 0, (128,) * 3, 200, 150)])
    a = gpu_trace(v, rays)
    b = gpu_trace(v, rays)
    assert np.array_equal(a, b)
    ref = oracle.Volume("G(4) R(3,3,3) --whole-level-dedup", codes).trace(rays, nthreads=8)
    assert compare(a, ref, "shell 128") == 0


SCHEDULES = [dict(stack_depth=1), dict(stack_depth=2), dict(stack_depth=3, persistent=1, refill=8),
             dict(persistent=1, refill=1, inner=1), dict(persistent=1, refill=16, inner=8),
             dict(persistent=1, refill=8, inner=4, blocks_per_cu=1), dict(persistent=1, refill=32, inner=16, blocks_per_cu=2),
             dict(persistent=1, refill=64, inner=64), dict(sort=1, sort_bits=0), dict(sort=1, sort_bits=4),
             dict(sort=1, sort_bits=9), dict(lds_depths=1), dict(lds_depths=2), dict(lds_depths=16),
             dict(lds_depths=3, persistent=1, refill=16, inner=8), dict(lds_depths=2, stack_depth=2),
             dict(lds_depths=2, sort=1, sort_bits=4),
             dict(split=2, split_budget=1), dict(split=4, split_budget=3), dict(split=8, split_budget=8),
             dict(split=64, split_budget=2), dict(split=16, split_budget=32), dict(split=32, split_budget=5),
             dict(split=8, split_budget=4, lds_depths=2), dict(split=4, split_budget=2, stack_depth=2),
             dict(split=8, split_budget=2, split_rounds=2), dict(split=64, split_budget=1, split_rounds=6),
             dict(split=2, split_budget=3, split_rounds=1), dict(split=4, split_budget=3, split_rounds=1, lds_depths=2),
             dict(split=16, split_budget=4, split_rounds=3, stack_depth=2),
             dict(steal=1, steal_len=1), dict(steal=2, steal_len=3),
             dict(steal=8, steal_len=16), dict(steal=64, steal_len=1),
             dict(steal=4, steal_len=1, lds_depths=2), dict(steal=1, steal_len=2, stack_depth=2),
             dict(steal=16, steal_len=1 << 20), dict(steal=1, steal_len=1, steal_idle=16),
             dict(steal=2, steal_len=2, steal_idle=64), dict(interleave=1), dict(interleave=1, lds_depths=2),
             dict(interleave=1, stack_depth=2), dict(steal=1, steal_len=2, steal_idle=16, interleave=1),
             dict(steal=4, steal_len=1, interleave=1, lds_depths=2),
             dict(steal=1, steal_len=2, steal_idle=16, interleave=1, rays_per_wave=32),
             dict(steal=1, steal_len=1, steal_idle=1, interleave=1, rays_per_wave=1),
             dict(steal=2, steal_len=2, steal_idle=8, interleave=1, rays_per_wave=17, lds_depths=2)]


@pytest.mark.parametrize("sd", SCHEDULES, ids=lambda d: "-".join(f"{k}{v}" for k, v in d.items()))
def test_schedules_give_identical_results(H, sd):
    import torch
    sc = H.schedule(**sd)
    cases = [("R(2,2,2) S(2) R(2,2,2)", W.scene_solid_noise(1), (64,) * 3),
             ("G(4) R(3,3,3) --whole-level-dedup", W.scene_shell(3, 7, 8, 4, 1.4), (128,) * 3),
             ("S(1) G(1) R(1,1,1)", W.scene_bernoulli(2, 3, 3, 3, 0.1), (8,) * 3),
             ("D(2,2,2,4) D(2,2,2,6) D(3,3,3,6)", W.scene_shell(3, 7, 8, 4, 1.4), (128,) * 3)]
    for spec, codes, ext in cases:
        rays = np.concatenate([W.camera_rays(3, 0, ext, 160, 120), W.random_rays(3, ext, 30000),
                               np.concatenate([r for r, _ in EDGE_CASES])])
        v = H.Volume(spec, codes)
        d = torch.from_numpy(rays).cuda()
        plain = v.trace(d).cpu().numpy()
        info = v.info()
        k = sd.get("lds_depths", 0)
        staged = 0 if k == 0 else (info["depth_offset"][k] if k < info["num_depths"] else info["num_words"] & ~3)
        if staged > 8192:
            with pytest.raises(H.HvfError) as e:  # the prefix does not fit the LDS limit
                v.trace(d, sched=sc)
            assert e.value.name == "HVF_E_INPUT"
            continue
        got = v.trace(d, sched=sc)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        assert np.array_equal(got, plain), f"{spec} {sd}"
        ref = oracle.Volume(spec, codes).trace(rays, nthreads=8)
        assert compare(got, ref, f"{spec} {sd}") == 0


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 255, 256, 257, 1000, 4097])
def test_interleaved_rays_ragged_counts(H, n):
    """Interleaved launches (lane l < R of wave w takes ray l * W + w) at counts that leave the
    last waves partly or wholly empty, with 64 and with fewer rays per wave: every ray is
    traced once, hits land at each ray's index, equal to the plain launch's."""
    import torch
    codes, ext = W.scene_shell(11, 7, 8, 4, 1.4), (128,) * 3
    v = H.Volume("G(4) R(3,3,3) --whole-level-dedup", codes)
    rays = np.concatenate([W.camera_rays(11, 0, ext, 64, 48), W.random_rays(11, ext, 4000)])[:n]
    d = torch.from_numpy(np.ascontiguousarray(rays)).cuda()
    plain = v.trace(d).cpu().numpy()
    for sd in (dict(interleave=1), dict(steal=1, steal_len=1, interleave=1),
               dict(steal=1, steal_len=2, steal_idle=16, interleave=1),
               dict(steal=1, steal_len=2, steal_idle=16, interleave=1, rays_per_wave=32),
               dict(steal=1, steal_len=1, steal_idle=4, interleave=1, rays_per_wave=7),
               dict(steal=1, steal_len=1, steal_idle=1, interleave=1, rays_per_wave=1)):
        hb = torch.full((n, 4), 7, dtype=torch.int32, device="cuda")
        v.trace(d, hb, sched=H.schedule(**sd))
        assert np.array_equal(hb.cpu().numpy(), plain), f"n={n} {sd}"


def test_autotune_keeps_results(H):
    import torch
    codes = W.scene_shell(3, 7, 8, 4, 1.4)
    spec = "R(3,3,3) G(4) --whole-level-dedup"
    v = H.Volume(spec, codes)
    sample = torch.from_numpy(W.camera_rays(9, 1, (128,) * 3, 320, 240)).cuda()
    sc = v.autotune(sample)
    assert H.schedule_dict(v.get_schedule()) == H.schedule_dict(sc)
    rays = np.concatenate([W.camera_rays(9, 0, (128,) * 3, 320, 240), W.random_rays(9, (128,) * 3, 20000)])
    got = gpu_trace(v, rays)
    ref = oracle.Volume(spec, codes).trace(rays, nthreads=8)
    assert compare(got, ref, f"autotuned {H.schedule_dict(sc)}") == 0


@pytest.mark.parametrize("spec", ["G(4) R(3,3,3) --whole-level-dedup --restart-sv", "S(2) G(2) R(2,2,2) --restart-sv",
                                  "D(3,3,3,6) S(4)", "R(2,2,2) R(2,2,2) R(3,3,3)"])
def test_steal_forks_keep_results(H, spec):
    """Forked walks (stealing) with restart-sv stacks, distance fields and Raw pointer grids
    give the plain schedule's hits bit for bit, at every check period."""
    import torch
    small = spec.startswith("S(2) G(2)")  # the only 64^3 format of this list
    codes, ext = (W.scene_solid_noise(5), (64,) * 3) if small else (W.scene_shell(5, 7, 8, 4, 1.4), (128,) * 3)
    rays = np.concatenate([W.random_rays(5, ext, 20000), W.camera_rays(5, 1, ext, 96, 64),
                           np.concatenate([r for r, _ in EDGE_CASES])])
    v = H.Volume(spec, codes)
    d = torch.from_numpy(rays).cuda()
    plain = v.trace(d).cpu().numpy()
    for sd in (dict(steal=1, steal_len=1), dict(steal=2, steal_len=4), dict(steal=4, steal_len=1, stack_depth=3)):
        got = v.trace(d, sched=H.schedule(**sd)).cpu().numpy()
        assert np.array_equal(got, plain), f"{spec} {sd}"


@pytest.mark.parametrize("spec", [sp + " --restart-sv" for sp in SPECS_8 if "--" not in sp] +
                         ["G(4) R(3,3,3) --whole-level-dedup --restart-sv", "S(2) G(2) R(2,2,2) --restart-sv"])
def test_restart_sv(H, spec):
    """Restarting sparse-voxel intersection (no stack inside SVO/SVDAG levels) gives the
    same hits as the oracle."""
    for seed in (1, 2):
        big = spec.startswith("G(4) R(3,3,3)")  # the only 128^3 format of this list
        codes = W.scene_shell(seed, 7, 8, 4, 1.4) if big else W.scene_bernoulli(seed, 3, 3, 3, 0.06 * seed)
        ext = (128,) * 3 if big else (8,) * 3
        if "S(2) G(2)" in spec:
            codes, ext = W.scene_solid_noise(seed), (64,) * 3
        rays = np.concatenate([W.random_rays(seed, ext, 3000), W.camera_rays(seed, 0, ext, 64, 48),
                               np.concatenate([r for r, _ in EDGE_CASES])])
        got = gpu_trace(H.Volume(spec, codes), rays)
        ref = oracle.Volume(spec, codes).trace(rays, nthreads=8)
        assert compare(got, ref, f"{spec} seed {seed}") == 0


@pytest.mark.parametrize("spec", ["D(6,6,6,6)", "D(4,4,4,6) R(2,2,2)", "D(3,3,3,6) D(3,3,3,6)",
                                  "D(2,2,2,6) G(4) --whole-level-dedup", "D(3,3,3,99) S(3)", "D(2,2,2,1) D(4,4,4,1)"])
def test_distance_field_sparse_scene(H, spec):
    """DF levels skip cells by their stored distance (Sec. 4.2); a sparse shell scene makes
    long skips. Hits must equal the oracle's, on primary and random rays."""
    codes = W.scene_shell(4, 6, 8, 4, 1.4)
    rays = np.concatenate([W.camera_rays(4, 0, (64, 64, 64), 96, 64), W.random_rays(4, (64, 64, 64), 6000)])
    got = gpu_trace(H.Volume(spec, codes), rays)
    ref = oracle.Volume(spec, codes).trace(rays, nthreads=8)
    assert compare(got, ref, spec) == 0


def test_concurrent_traces_of_one_volume(H):
    """Sorted, split and persistent traces of one volume in flight together on two streams,
    from two host threads on streams of their own and from four host threads on the default
    stream each equal the plain trace."""
    import threading
    import torch
    codes = W.scene_shell(3, 7, 8, 4, 1.4)
    v = H.Volume("G(4) R(3,3,3) --whole-level-dedup", codes)
    rays = [torch.from_numpy(np.concatenate([W.camera_rays(s, s % 3, (128,) * 3, 200, 150),
                                             W.random_rays(s, (128,) * 3, 20000)])).cuda() for s in range(6)]
    plain = [v.trace(r) for r in rays]
    torch.cuda.synchronize()
    scheds = [H.schedule(sort=1, sort_bits=2), H.schedule(split=8, split_budget=4, split_rounds=1), H.schedule(persistent=1),
              H.schedule(sort=1, sort_bits=4), H.schedule(split=4, split_budget=2), H.schedule(persistent=1, refill=8)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.full((r.shape[0], 4), 7, dtype=torch.int32, device="cuda") for r in rays]
    torch.cuda.synchronize()
    for i, (r, sc) in enumerate(zip(rays, scheds)):
        with torch.cuda.stream(streams[i % 2]):
            v.trace(r, outs[i], sched=sc)
    torch.cuda.synchronize()
    for i in range(len(rays)):
        assert torch.equal(outs[i], plain[i]), f"stream case {i}"
    outs2 = [torch.full((r.shape[0], 4), 7, dtype=torch.int32, device="cuda") for r in rays]
    torch.cuda.synchronize()

    def worker(k):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            for i in range(k, len(rays), 2):
                v.trace(rays[i], outs2[i], sched=scheds[i])
        s.synchronize()

    ts = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    torch.cuda.synchronize()
    for i in range(len(rays)):
        assert torch.equal(outs2[i], plain[i]), f"thread case {i}"
    # Split traces on the default stream from four host threads: they share the volume's
    # survivor list when it is free, take their own scratch when it is held, and the shared
    # list grows for the larger ray sets mid-way.
    split = [H.schedule(split=8, split_budget=4), H.schedule(split=4, split_budget=2, split_rounds=2)]
    order = [rays[0][:5000], rays[1], rays[2][:777]] + rays[3:]
    want = [v.trace(r) for r in order]
    torch.cuda.synchronize()
    outs3 = [[torch.full((r.shape[0], 4), 7, dtype=torch.int32, device="cuda") for r in order] for _ in range(4)]
    torch.cuda.synchronize()

    def default_worker(k):
        for i, r in enumerate(order):
            v.trace(r, outs3[k][i], sched=split[(i + k) % 2], stream=0)

    ts = [threading.Thread(target=default_worker, args=(k,)) for k in range(4)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    torch.cuda.synchronize()
    for k in range(4):
        for i in range(len(order)):
            assert torch.equal(outs3[k][i], want[i]), f"default-stream thread {k} case {i}"

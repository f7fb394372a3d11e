"""Device construction (hvf_build_device) through the C-ABI.

A device-built volume must hold the host builder's word buffer word for word (same
layout, same SVDAG de-duplication, same statistics), in the library's layout and in the
paper's (--paper-layout, whose host words the oracle pins on the CPU), and tracing it must
match the oracle element by element (hit and xyz bit-exact, t within 1e-6 relative).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import compare, gpu_trace
from tests.test_oracle_pins import DF_SPECS, EDGE_CASES, EDGE_SPECS, EDGE_VOX, SPECS_8, codes_of
from workloads import configs as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2410_14128_amd as H
    H.lib()
    return H


def dev_codes(codes):
    import torch
    return torch.from_numpy(np.ascontiguousarray(codes, dtype=np.uint64).view(np.int64)).cuda()


def same_volume(H, spec, codes):
    host = H.Volume(spec, codes)
    dev = H.Volume.from_device(spec, dev_codes(codes))
    wh, wd = host.words(), dev.words()
    assert len(wh) == len(wd), f"{spec}: {len(wd)} words, host {len(wh)}"
    bad = np.nonzero(wh != wd)[0]
    assert len(bad) == 0, f"{spec}: {len(bad)} words differ, first at {bad[:5].tolist()}: " \
                          f"{wd[bad[:5]].tolist()} vs host {wh[bad[:5]].tolist()}"
    ih, idv = host.info(), dev.info()
    for k in ("num_words", "depth_nodes", "depth_offset", "level_nodes", "num_voxels", "kernel_family"):
        assert ih[k] == idv[k], (spec, k, ih[k], idv[k])
    return host, dev


@pytest.mark.parametrize("spec", SPECS_8 + DF_SPECS)
def test_every_type_sequence_words(H, spec):
    for seed, p in ((1, 0.05), (2, 0.2), (3, 0.6), (4, 1.0)):
        same_volume(H, spec, W.scene_bernoulli(seed, 3, 3, 3, p))


@pytest.mark.parametrize("spec", ["R(1,0,2) R(2,2,2)", "R(3,2,4)", "R(1,0,2) S(2)", "R(1,0,2) G(1) R(1,1,1)",
                                  "R(0,0,0) R(2,2,2)", "R(2,1,0) G(2) --whole-level-dedup", "R(1,1,1)", "S(1)",
                                  "G(1)", "R(0,1,2) R(1,1,1)", "D(3,2,4,5) R(1,1,1)", "D(3,2,4,3)", "D(1,0,2,2) S(2)",
                                  "D(2,1,0,9) D(2,2,2,1)"])
def test_noncubic_and_tiny_tops(H, spec):
    ex = H.Volume(spec).info()["extent_log2"]
    for seed, p in ((5, 0.1), (6, 0.5)):
        same_volume(H, spec, W.scene_bernoulli(seed, ex[0], ex[1], ex[2], p))


@pytest.mark.parametrize("spec", ["G(6)", "G(3) G(3)", "G(6) --whole-level-dedup", "G(3) G(3) --whole-level-dedup",
                                  "S(2) G(4)", "G(4) R(2,2,2)", "R(2,2,2) G(2) R(2,2,2)"])
def test_repetitive_scene_dedup(H, spec):
    """A periodic pattern: many equal subtrees, inside and across sub-volumes."""
    xyz = np.stack(np.meshgrid(np.arange(64), np.arange(64), np.arange(64), indexing="ij"), -1).reshape(-1, 3)
    keep = ((xyz[:, 0] % 8) < 3) & ((xyz[:, 1] % 4) != 1) & (((xyz[:, 2] + xyz[:, 0] // 16) % 8) < 5)
    codes = np.sort(W.morton_encode(xyz[keep].astype(np.uint32)))
    host, dev = same_volume(H, spec, codes)
    if spec.startswith("G(6)"):
        assert host.info()["depth_nodes"][3] < 64  # de-duplication did merge nodes


def test_scenes_256(H):
    codes = W.scene_shell(4, 8, 12, 6, 1.2)
    for spec in ["R(4,4,4) R(4,4,4)", "S(8)", "G(8)", "G(8) --whole-level-dedup", "R(6,6,6) G(2)",
                 "S(4) G(2) R(2,2,2)", "G(5) R(3,3,3)", "R(2,2,2) S(3) G(3) --whole-level-dedup"]:
        same_volume(H, spec, codes)


def test_surface_512_formats(H):
    codes = C.scene(C.SURF512)
    for spec in C.SURF512["specs"] + C.SURF512_DF:
        same_volume(H, spec, codes)


def test_distance_field_caps_and_sparse_scene(H):
    """Distances that hit the cap and distances far below it, in grids and in bricks."""
    xyz = np.array([[0, 0, 0], [63, 63, 63], [5, 40, 17], [33, 2, 60]], np.uint32)
    codes = np.sort(W.morton_encode(xyz))
    for spec in ["D(6,6,6,99)", "D(6,6,6,1)", "D(3,3,3,40) D(3,3,3,7)", "D(2,2,2,5) D(2,2,2,5) D(2,2,2,5)",
                 "G(2) D(4,4,4,12)", "D(4,4,4,20) G(2) --whole-level-dedup"]:
        same_volume(H, spec, codes)


def test_trace_device_built_against_oracle(H):
    codes = W.scene_solid_noise(1, log2n=6, n_sph=8, rmin=4, rmax=16, noise=0.05)
    rays = W.camera_rays(1, 0, (64, 64, 64), 128, 128)
    for spec in ["R(2,2,2) S(2) R(2,2,2)", "G(4) R(2,2,2)", "S(2) G(4) --whole-level-dedup"]:
        dev = H.Volume.from_device(spec, dev_codes(codes))
        got = gpu_trace(dev, rays)
        ref = oracle.Volume(spec, codes).trace(rays, nthreads=8)
        assert compare(got, ref, spec) == 0


@pytest.mark.parametrize("spec", EDGE_SPECS + ["D(3,3,3,6)", "D(1,1,1,3) R(2,2,2)", "S(1) D(2,2,2,6)"])
def test_edge_suite_device_built(H, spec):
    codes = codes_of(EDGE_VOX)
    rays = np.concatenate([r for r, _ in EDGE_CASES])
    got = gpu_trace(H.Volume.from_device(spec, dev_codes(codes)), rays)
    ref = oracle.Volume(spec, codes).trace(rays)
    assert compare(got, ref, spec) == 0


def test_depth_buffers_save_and_load(H, tmp_path):
    """A device-built volume with per-depth regions saves and loads like a host-built one."""
    import torch
    spec = "G(3) R(3,3,3) --whole-level-dedup --depth-buffers"
    codes = W.scene_bernoulli(11, 3, 3, 3, 0.3)
    host, dev = same_volume(H, spec, codes)
    p = str(tmp_path / "dev.hvf")
    dev.save(p)
    back = H.Volume.load(p)
    assert back.info() == host.info() and np.array_equal(back.words(), host.words())
    rays = torch.from_numpy(W.random_rays(12, (64,) * 3, 2000)).cuda()
    assert torch.equal(back.trace(rays), host.trace(rays))


@pytest.mark.parametrize("spec", SPECS_8 + DF_SPECS)
def test_depth_buffers_words(H, spec):
    """Per-depth regions built on the device: region-relative pointers and the same word
    positions as the host build, word for word; traces and batched traces agree."""
    import torch
    for seed, p in ((1, 0.05), (3, 0.6)):
        host, dev = same_volume(H, spec + " --depth-buffers", W.scene_bernoulli(seed, 3, 3, 3, p))
        assert dev.info()["depth_buffers"] and host.info()["depth_buffers"]
    ext = host.info()["extent_log2"]
    rays = torch.from_numpy(W.random_rays(8, tuple(1 << e for e in ext), 3000)).cuda()
    want = host.trace(rays)
    bt = H.Batch([dev, host], [rays, rays])
    got = bt.run()
    torch.cuda.synchronize()
    assert torch.equal(dev.trace(rays), want) and torch.equal(got[0], want) and torch.equal(got[1], want)
    bt.close()


def test_empty_single_and_full(H):
    for spec in ["R(3,3,3)", "G(3)", "S(1) R(2,2,2)"]:
        same_volume(H, spec, np.zeros(0, np.uint64))
        same_volume(H, spec, np.array([0], np.uint64))
        same_volume(H, spec, np.array([511], np.uint64))
        same_volume(H, spec, np.arange(512, dtype=np.uint64))
        same_volume(H, spec + " --depth-buffers", np.zeros(0, np.uint64))
        same_volume(H, spec + " --depth-buffers", np.arange(512, dtype=np.uint64))


def test_errors(H):
    import torch
    codes = W.scene_bernoulli(1, 3, 3, 3, 0.3)
    with pytest.raises(H.HvfError) as e:
        H.Volume.from_device("R(3,3,3)", dev_codes(codes[::-1].copy()))
    assert e.value.name == "HVF_E_INPUT"
    with pytest.raises(H.HvfError) as e:
        H.Volume.from_device("R(2,2,2)", dev_codes(codes))  # codes beyond a 4^3 volume
    assert e.value.name == "HVF_E_INPUT"
    dup = np.concatenate([codes[:3], codes[2:]])
    with pytest.raises(H.HvfError) as e:
        H.Volume.from_device("R(3,3,3)", dev_codes(dup))
    assert e.value.name == "HVF_E_INPUT"
    with pytest.raises(H.HvfError) as e:
        H.Volume.from_device("Q(3)", dev_codes(codes))
    assert e.value.name == "HVF_E_SPEC"
    with pytest.raises(TypeError):
        H.Volume.from_device("R(3,3,3)", torch.from_numpy(codes.view(np.int64)))
    # the failed calls leave nothing behind: a build right after still matches
    same_volume(H, "G(3)", codes)


def test_host_copy_on_demand(H, tmp_path):
    """The host copy of a device-built volume is fetched when first read: size first, then
    save/load, then the words; a loaded copy traces like the original."""
    codes = W.scene_shell(2, 7, 6, 3, 1.3)
    spec = "R(2,2,2) G(3) R(2,2,2)"
    dev = H.Volume.from_device(spec, dev_codes(codes))
    host = H.Volume(spec, codes)
    assert dev.info()["num_words"] == host.info()["num_words"]
    path = str(tmp_path / "dev.hvf")
    dev.save(path)
    back = H.Volume.load(path)
    assert np.array_equal(back.words(), host.words())
    assert np.array_equal(dev.words(), host.words())
    rays = W.random_rays(3, (128, 128, 128), 20000)
    assert np.array_equal(gpu_trace(back, rays), gpu_trace(dev, rays))


# ---------------------------------------------------------------- the paper's word layout
PAPER_MORE = ["R(1,0,2) R(2,2,2)", "R(3,2,4)", "R(1,0,2) S(2)", "R(1,0,2) G(1) R(1,1,1)", "D(3,2,4,5) R(1,1,1)",
              "G(6) --whole-level-dedup", "G(3) G(3) --whole-level-dedup", "S(2) G(2) R(1,1,1) --whole-level-dedup",
              "D(2,2,2,4) D(2,2,2,6) D(3,3,3,6)", "S(1) G(1) R(1,1,1)", "R(0,0,0) R(2,2,2)", "G(1)", "S(1)",
              "R(1,1,1)", "D(2,1,0,9) D(2,2,2,1)", "R(2,1,0) G(2) --whole-level-dedup"]


@pytest.mark.parametrize("spec", SPECS_8 + DF_SPECS + PAPER_MORE)
def test_paper_layout_words(H, spec):
    """Every type sequence, DF levels and non-cubic or one-cell tops, at four densities."""
    ex = H.Volume(spec).info()["extent_log2"]
    for seed, p in ((1, 0.05), (2, 0.2), (3, 0.6), (4, 1.0)):
        same_volume(H, spec + " --paper-layout", W.scene_bernoulli(seed, ex[0], ex[1], ex[2], p))


@pytest.mark.parametrize("spec", ["G(6)", "G(3) G(3)", "G(6) --whole-level-dedup", "G(3) G(3) --whole-level-dedup",
                                  "S(2) G(4)", "G(4) R(2,2,2)", "R(2,2,2) G(2) R(2,2,2)", "G(2) G(2) G(2)",
                                  "S(2) G(2) G(2) --whole-level-dedup"])
def test_paper_layout_repetitive_scene(H, spec):
    """A periodic pattern: the first of many equal SVDAG children (and leaves) is the stored one."""
    xyz = np.stack(np.meshgrid(np.arange(64), np.arange(64), np.arange(64), indexing="ij"), -1).reshape(-1, 3)
    keep = ((xyz[:, 0] % 8) < 3) & ((xyz[:, 1] % 4) != 1) & (((xyz[:, 2] + xyz[:, 0] // 16) % 8) < 5)
    codes = np.sort(W.morton_encode(xyz[keep].astype(np.uint32)))
    same_volume(H, spec + " --paper-layout", codes)


def test_paper_layout_scenes(H):
    """A 256^3 shell scene in mixed formats, the 512^3 surface formats, and DF caps."""
    codes = W.scene_shell(4, 8, 12, 6, 1.2)
    for spec in ["R(4,4,4) R(4,4,4)", "S(8)", "G(8)", "G(8) --whole-level-dedup", "R(6,6,6) G(2)",
                 "S(4) G(2) R(2,2,2)", "G(5) R(3,3,3)", "R(2,2,2) S(3) G(3) --whole-level-dedup", "D(4,4,4,6) G(4)"]:
        same_volume(H, spec + " --paper-layout", codes)
    codes = C.scene(C.SURF512)
    for spec in C.SURF512["specs"] + C.SURF512_DF:
        same_volume(H, spec + " --paper-layout", codes)
    xyz = np.array([[0, 0, 0], [63, 63, 63], [5, 40, 17], [33, 2, 60]], np.uint32)
    sparse = np.sort(W.morton_encode(xyz))
    for spec in ["D(6,6,6,99)", "D(6,6,6,1)", "D(3,3,3,40) D(3,3,3,7)", "G(2) D(4,4,4,12)"]:
        same_volume(H, spec + " --paper-layout", sparse)


def test_paper_layout_empty_single_and_full(H):
    for spec in ["R(3,3,3)", "G(3)", "S(1) R(2,2,2)", "D(3,3,3,4)", "G(1) G(2)"]:
        for codes in (np.zeros(0, np.uint64), np.array([0], np.uint64), np.array([511], np.uint64),
                      np.arange(512, dtype=np.uint64)):
            same_volume(H, spec + " --paper-layout", codes)


@pytest.mark.parametrize("spec", EDGE_SPECS + ["D(3,3,3,6)", "S(1) D(2,2,2,6)"])
def test_paper_layout_device_built_traces(H, spec):
    """Device-built paper-layout volumes against the oracle: the edge suite, and a 64^3 scene."""
    codes = codes_of(EDGE_VOX)
    rays = np.concatenate([r for r, _ in EDGE_CASES])
    got = gpu_trace(H.Volume.from_device(spec + " --paper-layout", dev_codes(codes)), rays)
    assert compare(got, oracle.Volume(spec, codes).trace(rays), spec) == 0
    if spec == EDGE_SPECS[0]:
        scene = W.scene_solid_noise(1, log2n=6, n_sph=8, rmin=4, rmax=16, noise=0.05)
        rays = W.camera_rays(1, 0, (64, 64, 64), 128, 128)
        for sp in ["R(2,2,2) S(2) R(2,2,2)", "G(4) R(2,2,2)", "S(2) G(4) --whole-level-dedup"]:
            dev = H.Volume.from_device(sp + " --paper-layout", dev_codes(scene))
            assert compare(gpu_trace(dev, rays), oracle.Volume(sp, scene).trace(rays, nthreads=8), sp) == 0

"""The paper's own word layout (--paper-layout), host side: no GPU needed.

The library's builder for this layout and the oracle's builder are written separately
from the same construction pass (Sec. 4.1) and memory layout (Sec. 3.3); their word
buffers must agree word for word, which pins both.
"""
import os

import numpy as np
import pytest

import oracle
import paper_2410_14128_amd as H
import workloads as W
from tests.test_oracle_pins import DF_SPECS, SPECS_8

MORE = ["R(1,0,2) R(2,2,2)", "R(3,2,4)", "R(1,0,2) S(2)", "R(1,0,2) G(1) R(1,1,1)", "D(3,2,4,5) R(1,1,1)",
        "G(6) --whole-level-dedup", "G(3) G(3) --whole-level-dedup", "S(2) G(2) R(1,1,1) --whole-level-dedup",
        "D(2,2,2,4) D(2,2,2,6) D(3,3,3,6)", "S(1) G(1) R(1,1,1)"]


@pytest.mark.parametrize("spec", SPECS_8 + DF_SPECS + MORE)
def test_words_equal_the_oracle(spec):
    ex = H.Volume(spec).info()["extent_log2"]
    for seed, p in ((1, 0.05), (2, 0.3), (3, 1.0)):
        codes = W.scene_bernoulli(seed, ex[0], ex[1], ex[2], p)
        got = H.Volume(spec + " --paper-layout", codes).words()
        want = oracle.Volume(spec, codes).words()
        assert len(got) == len(want), (spec, seed, len(got), len(want))
        bad = np.nonzero(got != want)[0]
        assert len(bad) == 0, (spec, seed, bad[:5].tolist())


def test_repetitive_scene_dedup_words():
    xyz = np.stack(np.meshgrid(np.arange(64), np.arange(64), np.arange(64), indexing="ij"), -1).reshape(-1, 3)
    keep = ((xyz[:, 0] % 8) < 3) & ((xyz[:, 1] % 4) != 1) & (((xyz[:, 2] + xyz[:, 0] // 16) % 8) < 5)
    codes = np.sort(W.morton_encode(xyz[keep].astype(np.uint32)))
    for spec in ["G(6)", "G(6) --whole-level-dedup", "G(3) G(3) --whole-level-dedup", "R(2,2,2) G(2) R(2,2,2)"]:
        got = H.Volume(spec + " --paper-layout", codes).words()
        assert np.array_equal(got, oracle.Volume(spec, codes).words()), spec


def test_empty_and_full():
    for spec in ["R(3,3,3)", "G(3)", "S(1) R(2,2,2)", "D(3,3,3,4)"]:
        for codes in (np.zeros(0, np.uint64), np.array([0], np.uint64), np.arange(512, dtype=np.uint64)):
            got = H.Volume(spec + " --paper-layout", codes).words()
            assert np.array_equal(got, oracle.Volume(spec, codes).words()), (spec, len(codes))


def test_layout_flags_and_limits(tmp_path):
    with pytest.raises(H.HvfError) as e:
        H.Volume("S(3) --restart-sv --paper-layout", np.array([1], np.uint64))
    assert e.value.name == "HVF_E_UNSUPPORTED"
    with pytest.raises(H.HvfError) as e:
        H.Volume("R(16,1,1) --paper-layout", np.array([1], np.uint64))
    assert e.value.name == "HVF_E_SPEC"
    codes = W.scene_bernoulli(4, 4, 4, 4, 0.2)
    v = H.Volume("S(2) G(2) --paper-layout", codes)
    info = v.info()
    assert info["num_voxels"] == len(codes)
    # Raw-final and mixed SVO/SVDAG formats take the paper family; octree-only ones an octree family.
    raw = H.Volume("R(2,2,2) R(2,2,2) --paper-layout", codes).info()
    assert raw["paper_layout"] and (raw["kernel_family"] >> 9) & 1  # the RGBA-voxel Raw kind is compiled in
    assert not H.Volume("R(2,2,2) R(2,2,2)", codes).info()["paper_layout"]
    path = str(tmp_path / "p.hvf")
    v.save(path)
    back = H.Volume.load(path)
    assert np.array_equal(back.words(), v.words())
    assert back.info()["paper_layout"] and back.info()["num_depths"] == info["num_depths"]

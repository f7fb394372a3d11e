"""Pins for the reference read model (tests/read_model.py) that the byte accounting is
checked against: hand-counted word sets for small cases worked out from the documented
layout, and the model's hit voxel equal to the oracle's on random rays (so the model
visits the cells of the traversal in the right order and stops where it does)."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.read_model import Model

H = pytest.importorskip("paper_2410_14128_amd")
INF = float("inf")


def ray(o, d, tmin=0.0, tmax=INF):
    return np.array([o[0], o[1], o[2], tmin, d[0], d[1], d[2], tmax], dtype=np.float32)


def vol(spec, voxels):
    v = np.array(sorted(voxels), dtype=np.int32).reshape(-1, 3)
    codes = np.sort(W.morton_encode(v))
    h = H.Volume(spec, codes)
    return h, Model(h.info(), h.words(), v)


def test_one_voxel_in_g3():
    """G(3), one voxel: word 0, the root node's mask word and its descriptor for the child
    octant, then the depth-1 descriptor; the deepest node's mask comes with that descriptor
    and its voxel bit is tested in registers. Nodes of depth d start at depth_offset[d]."""
    h, m = vol("G(3)", [(5, 2, 6)])
    off = h.info()["depth_offset"]
    words = h.words()
    reads, hit = m.reads(ray((-1.0, 2.5, 6.5), (1.0, 0.0, 0.0)))
    assert hit == (5, 2, 6)
    # root node at off[0]: mask, then one descriptor (child pointer, child mask)
    assert words[0] == off[0] and words[off[0] + 1] == off[1]
    assert reads == {0, off[0], off[0] + 1, off[0] + 2, off[1] + 1, off[1] + 2}
    assert len({w >> 4 for w in reads}) == 3


def test_axis_ray_through_a_brick():
    """R(3,3,3): one brick of 2x2x2 blocks of 4^3 voxels; an axis ray along +x reads the two
    blocks of its row (two words each), then walks the voxels of the occupied one."""
    h, m = vol("R(3,3,3)", [(6, 1, 1), (2, 5, 5)])
    b = h.words()[0]
    reads, hit = m.reads(ray((-1.0, 1.5, 1.5), (1.0, 0.0, 0.0)))
    assert hit == (6, 1, 1)
    assert reads == {0, b, b + 1, b + 2, b + 3}
    reads, hit = m.reads(ray((-1.0, 1.5, 1.5), (1.0, 0.0, 0.0), tmax=4.5))  # stops inside block 0
    assert hit is None and reads == {0, b, b + 1}


def test_distance_field_skip():
    """D(2,2,2,3) R(2,2,2): a 4^3 DF grid of 4^3-voxel cells. Along +x the first cell is
    empty at L1 distance 3 from the occupied cell (3,0,0), so the cells at L1 distance 1
    and 2 are not read; the occupied cell's pointer is read, then the one-block brick's mask."""
    h, m = vol("D(2,2,2,3) R(2,2,2)", [(13, 1, 1)])
    g = h.words()[0]
    words = h.words()
    assert words[g] == 0x80000000 | 3 and words[g + 1] == 0x80000000 | 2
    reads, hit = m.reads(ray((-1.0, 1.5, 1.5), (1.0, 0.0, 0.0)))
    assert hit == (13, 1, 1)
    brick = words[g + 3]
    assert reads == {0, g, g + 3, brick, brick + 1}


def test_paper_layout_svdag_leaf():
    """G(2) R(2,2,2) in the paper's layout: the SVDAG's last depth points to a leaf word that
    holds the Raw sub-volume's pointer; the Raw level holds one RGBA word per voxel. A ray
    along +x reads word 0, the root's mask word and child pointer, the child's mask word and
    leaf pointer, the leaf word, then the voxel words up to the hit (2 here): 8 words."""
    h, m = vol("G(2) R(2,2,2) --paper-layout", [(5, 9, 2)])
    w = h.words()
    reads, hit = m.reads(ray((-3.0, 9.5, 2.5), (1.0, 0.0, 0.0)))
    assert hit == (5, 9, 2)
    root = int(w[0])
    c1 = int(w[root + 1])          # the root has one child: pointer at root + 1
    leaf = int(w[c1 + 1])          # the child's only child: pointer to the leaf word
    sub = int(w[leaf])             # the leaf word: the Raw sub-volume's first word
    # voxels (4, 9, 2) and (5, 9, 2) of the 4^3 sub-volume at (4, 8, 0): x-fastest
    vox = [sub + 0 + 4 * 1 + 16 * 2, sub + 1 + 4 * 1 + 16 * 2]
    assert reads == {0, root, root + 1, c1, c1 + 1, leaf, *vox} and len(reads) == 8
    assert w[vox[1]] == 0xFFFFFFFF and w[vox[0]] == 0


@pytest.mark.parametrize("spec", ["R(2,2,2) S(2) R(2,2,2)", "G(4) R(2,2,2) --whole-level-dedup", "S(3) R(3,3,3)",
                                  "R(3,3,3) G(3)", "D(2,2,2,4) D(2,2,2,4) R(2,2,2)", "R(1,2,3) S(3)",
                                  "G(3) R(3,3,3) --paper-layout", "S(2) D(2,2,2,5) R(2,2,2) --paper-layout",
                                  "R(2,2,2) S(2) G(2) --paper-layout"])
def test_model_hits_equal_the_oracle(spec):
    """The model stops at the oracle's first hit on random rays and camera rays."""
    codes = W.scene_solid_noise(3)
    ext = H.Volume(spec, np.zeros(0, np.uint64)).info()["extent_log2"]
    n = [1 << e for e in ext]
    if n != [64, 64, 64]:
        xyz = W.morton_decode(codes)
        keep = (xyz[:, 0] < n[0]) & (xyz[:, 1] < n[1]) & (xyz[:, 2] < n[2])
        codes = np.sort(W.morton_encode(xyz[keep]))
    h = H.Volume(spec, codes)
    m = Model(h.info(), h.words(), W.morton_decode(codes))
    rays = np.concatenate([W.random_rays(3, tuple(n), 200), W.camera_rays(3, 0, tuple(n), 12, 12)])
    ref = oracle.Volume(spec.replace(" --paper-layout", ""), codes).trace(rays)
    for r, want in zip(rays, ref):
        _, hit = m.reads(r)
        got = (-1, -1, -1) if hit is None else hit
        assert got == tuple(int(x) for x in want[:3]), (spec, r)

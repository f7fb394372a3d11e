"""The seeded input generators: deterministic, sorted, in bounds, of the stated shape."""
import numpy as np

import workloads as W


def test_morton_roundtrip():
    rng = np.random.default_rng(1)
    xyz = rng.integers(0, 1 << 20, size=(1000, 3)).astype(np.int32)
    assert np.array_equal(W.morton_decode(W.morton_encode(xyz)), xyz)


def test_scenes_deterministic_sorted_in_bounds():
    for gen in (lambda: W.scene_solid_noise(3), lambda: W.scene_shell(5, 7, 8, 4, 1.4),
                lambda: W.scene_bernoulli(2, 3, 2, 4, 0.3)):
        a, b = gen(), gen()
        assert np.array_equal(a, b) and len(a) > 0
        assert np.all(np.diff(a.astype(np.int64)) > 0)
    xyz = W.morton_decode(W.scene_bernoulli(2, 3, 2, 4, 0.3))
    assert xyz[:, 0].max() < 8 and xyz[:, 1].max() < 4 and xyz[:, 2].max() < 16


def test_shell_thread_count_independent():
    assert np.array_equal(W.scene_shell(9, 7, 6, 3, 1.4, nthreads=1), W.scene_shell(9, 7, 6, 3, 1.4, nthreads=7))


def test_shell_voxels_touch_empty_space():
    codes = W.scene_shell(6, 6, 6, 3, 1.4)
    xyz = W.morton_decode(codes)
    occ = np.zeros((66, 66, 66), bool)
    occ[xyz[:, 2] + 1, xyz[:, 1] + 1, xyz[:, 0] + 1] = True
    # a shell voxel has an empty 6-neighbour (inside the grid) or lies on the grid boundary
    nb_empty = np.zeros(len(xyz), bool)
    for a in range(3):
        for s in (-1, 1):
            q = xyz.copy() + 1
            q[:, a] += s
            nb_empty |= ~occ[q[:, 2], q[:, 1], q[:, 0]]
    assert nb_empty.all()


def test_camera_rays_shape_and_norm():
    r = W.camera_rays(1, 0, (64, 64, 64), 32, 16)
    assert r.shape == (512, 8)
    assert np.allclose(np.linalg.norm(r[:, 4:7], axis=1), 1.0, atol=1e-6)
    assert np.all(r[:, 3] == 0) and np.all(np.isinf(r[:, 7]))
    eye = r[0, :3] - 32.0
    assert 1.2 * 64 - 1 <= np.linalg.norm(eye) <= 2.0 * 64 + 1


def test_bounce_rays_leave_the_surface():
    rays = np.array([[-3, 0.5, 0.5, 0, 1, 0, 0, np.inf]], np.float32)
    hits = np.array([[2, 0, 0, 0]], np.int32)
    hits[0, 3] = np.float32(5.0).view(np.int32)
    b, src = W.bounce_rays(1, rays, hits)
    assert len(b) == 1 and src[0] == 0
    assert abs(b[0, 0] - (2.0 - 2 ** -6)) < 1e-6 and b[0, 4] < 0  # leaves through the -x face


def test_table_formats_recipe_matches_the_pinned_table():
    """The sweep's format list is the paper's table (pinned in tests/golden)."""
    import os
    import re
    from workloads import configs as C
    gold = [l.split(maxsplit=2) for l in open(os.path.join(os.path.dirname(__file__), "golden", "table_formats.txt"))
            if l.strip() and not l.startswith("#")]

    def norm(s):
        s = re.sub(r"D\((\d+)\^3,(\d+)\)", r"D(\1,\1,\1,\2)", s)
        return re.sub(r"R\((\d+)\^3\)", r"R(\1,\1,\1)", s).strip()

    assert len(gold) == len(C.TABLE_FORMATS) == 40
    for (lab, side, spec), (l2, k, sp) in zip(gold, C.TABLE_FORMATS):
        assert int(lab) == l2 and int(side) == 1 << k and norm(spec) == sp

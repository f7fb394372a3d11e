"""The byte accounting (B_ray) against the reference read model: for every ray, the set of
format words the counting kernel logs equals the set the traversal must read
(tests/read_model.py, pinned on the CPU by tests/test_read_model.py). B_ray is
32 + 16 bytes plus 4 bytes per distinct word (word model) or 64 bytes per distinct
64-byte sector (sector model), so equal word sets give equal B_ray in both models."""
import numpy as np
import pytest

import workloads as W
from tests.read_model import Model
from workloads import configs as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2410_14128_amd as H
    H.lib()
    return H


def _check(H, spec, codes, rays, cap=2048):
    import torch
    v = H.Volume(spec, codes)
    m = Model(v.info(), v.words(), W.morton_decode(codes))
    d = torch.from_numpy(np.ascontiguousarray(rays)).cuda()
    hits, log, cnt = v.trace_count(d, cap=cap)
    torch.cuda.synchronize()
    hits, log, cnt = hits.cpu().numpy(), log.cpu().numpy(), cnt.cpu().numpy()
    assert int(cnt.max()) <= cap
    words_k = sectors_k = words_m = sectors_m = 0
    for i, r in enumerate(rays):
        got = set(int(x) for x in log[i, :cnt[i]])
        want, hit = m.reads(r)
        assert got == want, f"{spec} ray {i}: kernel-only {sorted(got - want)[:8]}, model-only {sorted(want - got)[:8]}"
        assert (tuple(int(x) for x in hits[i, :3]) == (hit if hit is not None else (-1, -1, -1))), f"{spec} ray {i}"
        words_k += len(got)
        sectors_k += len({w >> 4 for w in got})
        words_m += len(want)
        sectors_m += len({w >> 4 for w in want})
    assert (words_k, sectors_k) == (words_m, sectors_m)
    return words_k / len(rays), sectors_k / len(rays)


def test_hand_counted_cases(H):
    cases = [("G(3)", [(5, 2, 6)], (-1.0, 2.5, 6.5), 6), ("R(3,3,3)", [(6, 1, 1), (2, 5, 5)], (-1.0, 1.5, 1.5), 5),
             ("D(2,2,2,3) R(2,2,2)", [(13, 1, 1)], (-1.0, 1.5, 1.5), 5),
             ("G(2) R(2,2,2) --paper-layout", [(5, 9, 2)], (-3.0, 9.5, 2.5), 8)]
    for spec, vox, o, nwords in cases:
        v = np.array(vox, dtype=np.int32)
        codes = np.sort(W.morton_encode(v))
        r = np.array([[o[0], o[1], o[2], 0.0, 1.0, 0.0, 0.0, np.inf]], dtype=np.float32)
        words, _ = _check(H, spec, codes, r)
        assert words == nwords, spec


def test_small_config(H):
    """The 64^3 small case R(2,2,2) S(2) R(2,2,2): a sample of its 256x256 view plus random rays."""
    cfg = C.SMALL
    codes = C.scene(cfg)
    view = C.primary_rays(cfg, 0)
    rng = np.random.default_rng(31)
    rays = np.concatenate([view[rng.choice(len(view), 2000, replace=False)], W.random_rays(31, (64,) * 3, 500)])
    w, s = _check(H, cfg["spec"], codes, rays)
    assert w > 4 and s > 1


@pytest.mark.parametrize("spec", ["G(3) R(4,4,4) --whole-level-dedup", "S(3) R(4,4,4)", "G(4) R(3,3,3) --whole-level-dedup",
                                  "D(3,3,3,6) S(4)", "R(2,2,2) R(2,2,2) R(3,3,3)", "D(4,4,4,5) R(3,3,3)",
                                  "S(2) G(2) R(3,3,3) --restart-sv", "G(4) R(3,3,3) --paper-layout",
                                  "R(3,3,3) S(2) D(2,2,2,4) --paper-layout"])
def test_formats_128(H, spec):
    """128^3 shell scene: camera and random rays (incoherent, as the bounce launches)."""
    codes = W.scene_shell(8, 7, 8, 4, 1.4)
    rays = np.concatenate([W.camera_rays(8, 0, (128,) * 3, 24, 20), W.random_rays(8, (128,) * 3, 400)])
    _check(H, spec, codes, rays)

"""Helpers for GPU parity tests: trace through the C-ABI, compare with the oracle."""
import numpy as np


def gpu_trace(vol, rays: np.ndarray) -> np.ndarray:
    import torch
    r = torch.from_numpy(np.ascontiguousarray(rays, dtype=np.float32)).cuda()
    h = vol.trace(r)
    torch.cuda.synchronize()
    return h.cpu().numpy()


def compare(got: np.ndarray, ref: np.ndarray, what: str = "", rtol: float = 1e-6):
    """Hit flag and voxel xyz bit-exact; t within rtol relative (+-0 equal, inf == inf).

    Returns the number of rays whose t differs in any bit (expected 0).
    """
    assert got.shape == ref.shape, (got.shape, ref.shape)
    xyz_bad = np.any(got[:, :3] != ref[:, :3], axis=1)
    if xyz_bad.any():
        idx = np.nonzero(xyz_bad)[0][:5]
        raise AssertionError(f"{what}: {int(xyz_bad.sum())}/{len(got)} rays hit a different voxel; "
                             f"first {idx.tolist()}: got {got[idx].tolist()} want {ref[idx].tolist()}")
    tg = got[:, 3].view(np.float32).astype(np.float64)
    tr = ref[:, 3].view(np.float32).astype(np.float64)
    both_inf = np.isinf(tg) & np.isinf(tr) & (np.sign(tg) == np.sign(tr))
    with np.errstate(invalid="ignore"):
        close = both_inf | (np.abs(tg - tr) <= rtol * np.maximum(np.abs(tg), np.abs(tr)))
    if not close.all():
        idx = np.nonzero(~close)[0][:5]
        raise AssertionError(f"{what}: {int((~close).sum())} rays with t outside {rtol} relative; "
                             f"first {idx.tolist()}: got {tg[idx].tolist()} want {tr[idx].tolist()}")
    assert not np.any(got[:, 0] == -2), f"{what}: iteration guard tripped"
    return int(np.count_nonzero(got[:, 3] != ref[:, 3]))

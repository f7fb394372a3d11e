"""Exact-arithmetic statement of the first-hit definition, for pinning the oracle.

Rays are taken at their exact fp32 values as rationals; plane crossing times are exact
rationals (p - o) / d, so nothing here rounds. Used only on tiny volumes.
"""
from fractions import Fraction
import math

import numpy as np


def first_hit_exact(voxels, ext, ray):
    """Return (voxel, t_exact, margin) or (None, None, margin).

    voxels: iterable of (x, y, z) ints; ext: per-axis log2 extents; ray: 8 floats.
    margin: the smallest relative gap among the decisions that fix the answer (entry vs
    exit of the winner, winner vs runner-up, clip), so callers can skip near-ties where
    fp32 rounding may legitimately decide differently.
    """
    ox, oy, oz, tmin, dx, dy, dz, tmax = [float(np.float32(v)) for v in ray]
    o = (ox, oy, oz)
    d = (dx, dy, dz)
    if not all(math.isfinite(v) for v in o + d):
        return None, None, math.inf
    N = [1 << e for e in ext]
    if all(v == 0.0 for v in d):
        return None, None, math.inf
    F = Fraction
    lo_t = F(tmin) if math.isfinite(tmin) else (None if tmin > 0 else "-inf")
    hi_t = F(tmax) if math.isfinite(tmax) else "inf"
    best = None
    second = None
    graze = math.inf  # least relative |x - e| over every candidate box, visited or not
    for v in voxels:
        v = tuple(int(c) for c in v)
        e = None
        x = None
        ok = True
        for a in range(3):
            if d[a] == 0.0:
                if not (v[a] <= o[a] < v[a] + 1):
                    ok = False
                    break
                continue
            t_lo = (F(v[a]) - F(o[a])) / F(d[a])
            t_hi = (F(v[a] + 1) - F(o[a])) / F(d[a])
            ne, fa = (t_lo, t_hi) if d[a] > 0 else (t_hi, t_lo)
            e = ne if e is None or ne > e else e
            x = fa if x is None or fa < x else x
        if not ok:
            continue
        if lo_t == "-inf":
            pass
        elif lo_t is None:
            continue
        else:
            e = lo_t if lo_t > e else e
        if hi_t != "inf":
            x = hi_t if hi_t < x else x
        sc = max(abs(e), abs(x), Fraction(1))
        graze = min(graze, float(abs(x - e) / sc))
        if not (e < x):
            continue
        item = (e, x, tuple(v))
        if best is None or e < best[0]:
            second = best
            best = item
        elif second is None or e < second[0]:
            second = item
    if best is None:
        return None, None, graze
    e, x, v = best
    scale = max(abs(e), abs(x), Fraction(1))
    margin = graze
    if second is not None:
        margin = min(margin, float(abs(second[0] - e) / scale))
    return v, e, margin

"""Workload recipes (inputs only): seeded scenes, format specs and ray sets.

The paper evaluates voxelized mesh models (San Miguel, Hairball, Buddha, Sponza) at
512^3 and 2048^3; those models are not available, so seeded synthetic SDF scenes of the
same resolutions stand in for them. Format specs follow the paper's grammar (R(k,k,k)
has 2^k cells per axis); several come from its table of evaluated formats.
"""
from __future__ import annotations

import numpy as np

from . import camera_rays, random_rays, scene_shell, scene_solid_noise

# Small case: 64^3 solid spheres (radii U[4,16]) OR 5% Bernoulli noise; 256x256 pinhole.
SMALL = dict(name="small-64", log2n=6, seed=1, spec="R(2,2,2) S(2) R(2,2,2)", width=256, height=256, views=1)

# 512^3 surface volume: shell of 32 spheres + 16 tori; nine formats; 4 views at 1080p.
SURF512 = dict(
    name="surface-512", log2n=9, seed=2, n_sph=32, n_tor=16, scale=1.4, width=1920, height=1080, views=4,
    specs=[
        "R(9,9,9)",                          # plain Raw
        "S(9)",                              # plain SVO
        "G(9) --whole-level-dedup",          # plain SVDAG (table row 40)
        "G(6) R(3,3,3) --whole-level-dedup",  # SVDAG -> Raw 8^3 bricks
        "S(3) G(4) R(2,2,2) --whole-level-dedup",  # SVO -> SVDAG -> Raw 4^3
        "R(4,4,4) G(5) --whole-level-dedup",  # table row 29
        "R(4,4,4) S(5)",                     # table row 28
        "R(3,3,3) R(3,3,3) R(3,3,3)",        # table row 24
        "S(5) R(4,4,4)",                     # table row 32
    ])

# Distance-field formats of the table at 512^3 (rows 21, 22, 26, 27, 34, 35, 38), traced on
# the same volume and views; measured beside the nine formats above, not part of them.
SURF512_DF = ["D(3,3,3,6) D(3,3,3,6) G(3) --whole-level-dedup", "D(3,3,3,6) R(3,3,3) G(3) --whole-level-dedup",
              "D(4,4,4,6) S(5)", "D(4,4,4,6) G(5) --whole-level-dedup", "D(5,5,5,6) D(4,4,4,6)",
              "D(5,5,5,6) R(4,4,4)", "D(9,9,9,6)"]

# The 40 evaluated format signatures of the paper's table (Sec. 6): (label, log2 side,
# spec). Rows 1-20 represent a 2048^3 grid, rows 21-40 a 512^3 grid; R(k^3) is R(k,k,k)
# and D(k^3,M) is D(k,k,k,M). SVDAG levels are built with whole-level de-duplication.
TABLE_FORMATS = [
    (1, 11, "D(4,4,4,6) D(3,3,3,6) G(4)"), (2, 11, "D(4,4,4,6) R(3,3,3) G(4)"), (3, 11, "R(4,4,4) R(3,3,3) G(4)"),
    (4, 11, "R(4,4,4) S(3) G(4)"), (5, 11, "R(4,4,4) R(4,4,4) R(3,3,3)"), (6, 11, "D(4,4,4,6) S(7)"),
    (7, 11, "D(4,4,4,6) G(7)"), (8, 11, "D(6,6,6,6) S(5)"), (9, 11, "D(6,6,6,6) G(5)"), (10, 11, "R(4,4,4) S(7)"),
    (11, 11, "R(4,4,4) G(7)"), (12, 11, "R(6,6,6) S(5)"), (13, 11, "R(6,6,6) G(5)"), (14, 11, "R(3,3,3) G(8)"),
    (15, 11, "R(8,8,8) G(3)"), (16, 11, "S(7) G(4)"), (17, 11, "S(5) G(6)"), (18, 11, "S(3) G(8)"), (19, 11, "S(11)"),
    (20, 11, "G(11)"),
    (21, 9, "D(3,3,3,6) D(3,3,3,6) G(3)"), (22, 9, "D(3,3,3,6) R(3,3,3) G(3)"), (23, 9, "R(3,3,3) R(3,3,3) G(3)"),
    (24, 9, "R(3,3,3) R(3,3,3) R(3,3,3)"), (25, 9, "R(4,4,4) R(1,1,1) R(4,4,4)"), (26, 9, "D(4,4,4,6) S(5)"),
    (27, 9, "D(4,4,4,6) G(5)"), (28, 9, "R(4,4,4) S(5)"), (29, 9, "R(4,4,4) G(5)"), (30, 9, "R(2,2,2) G(7)"),
    (31, 9, "R(7,7,7) G(2)"), (32, 9, "S(5) R(4,4,4)"), (33, 9, "G(5) R(4,4,4)"), (34, 9, "D(5,5,5,6) D(4,4,4,6)"),
    (35, 9, "D(5,5,5,6) R(4,4,4)"), (36, 9, "R(5,5,5) R(4,4,4)"), (37, 9, "R(9,9,9)"), (38, 9, "D(9,9,9,6)"),
    (39, 9, "S(9)"), (40, 9, "G(9)"),
]


def table_spec(spec: str) -> str:
    return spec + " --whole-level-dedup" if "G(" in spec else spec


# 2048^3 surface volume: 96 spheres + 32 tori; SVDAG top 7 levels -> Raw 16^3 bricks, and
# SVO -> Raw 8^3; 1080p primary rays plus one cosine-weighted bounce per primary hit.
SURF2048 = dict(name="surface-2048", log2n=11, seed=3, n_sph=96, n_tor=32, scale=1.2, width=1920, height=1080,
                views=1, specs=["G(7) R(4,4,4) --whole-level-dedup", "S(8) R(3,3,3)"], bounce_seed=33,
                # 8 frames whose bounce rays are traced in one launch (view 1 is the autotuner's
                # held-out view of the one-frame launches), and 8 held-out frames to tune it on
                frame_views=[0, 2, 3, 4, 5, 6, 7, 8], tune_frame_views=list(range(9, 17)))


# Formats of the 2048^3 volume whose construction (host against device) the bench line reports.
BUILD_2048 = ["S(11)", "G(11) --whole-level-dedup", "R(6,6,6) G(5) --whole-level-dedup", "R(4,4,4) R(4,4,4) R(3,3,3)"]


def scene(cfg: dict) -> np.ndarray:
    if cfg["name"].startswith("small"):
        return scene_solid_noise(cfg["seed"], log2n=cfg["log2n"], n_sph=8, rmin=4.0, rmax=16.0, noise=0.05)
    return scene_shell(cfg["seed"], cfg["log2n"], cfg["n_sph"], cfg["n_tor"], cfg["scale"])


def primary_rays(cfg: dict, view: int, width: int | None = None, height: int | None = None) -> np.ndarray:
    n = 1 << cfg["log2n"]
    return camera_rays(cfg["seed"], view, (n, n, n), width or cfg["width"], height or cfg["height"])


# Batched: 64 volumes, side 2^k with k ~ U{6..10}; shell scenes with max(4, N/16)
# primitives; each a seeded random hybrid format of 2 or 3 levels with kinds uniform over
# {R, S, G} (k split into positive parts, Raw exponents <= 5); 64 ray batches of size
# round(exp(U[ln 4096, ln 2^21])), half pinhole rays, half random origins and directions.
BATCHED = dict(name="batched-64", seed=4, nvol=64, kmin=6, kmax=10, nmin=4096, nmax=1 << 21)


def batched_format(rng: np.random.Generator, k: int) -> str:
    while True:
        nlev = int(rng.integers(2, 4))
        kinds = [str(rng.choice(["R", "S", "G"])) for _ in range(nlev)]
        cuts = np.sort(rng.choice(np.arange(1, k), size=nlev - 1, replace=False)) if k > nlev - 1 else None
        if cuts is None:
            continue
        parts = np.diff(np.concatenate([[0], cuts, [k]])).tolist()
        if any(kd == "R" and p > 5 for kd, p in zip(kinds, parts)):
            continue
        spec = " ".join(f"R({p},{p},{p})" if kd == "R" else f"{kd}({p})" for kd, p in zip(kinds, parts))
        if "G" in kinds and rng.random() < 0.5:
            spec += " --whole-level-dedup"
        return spec


def batched_case(cfg: dict, i: int, scale_rays: float = 1.0):
    """Volume i of the batched workload: (spec, log2 side, Morton codes, rays)."""
    rng = np.random.default_rng([cfg["seed"], i])
    k = int(rng.integers(cfg["kmin"], cfg["kmax"] + 1))
    spec = batched_format(rng, k)
    n_side = 1 << k
    prims = max(4, n_side // 16)
    codes = scene_shell(cfg["seed"] * 1000 + i, k, prims - prims // 4, prims // 4, 1.4)
    n = int(round(np.exp(rng.uniform(np.log(cfg["nmin"]), np.log(cfg["nmax"])))) * scale_rays)
    n = max(64, n)
    half = n // 2
    w = max(1, int(round(np.sqrt(half * 16 / 9))))
    h = (half + w - 1) // w
    cam = camera_rays(cfg["seed"] * 1000 + i, 0, (n_side,) * 3, w, h)[:half]
    rnd = random_rays(cfg["seed"] * 1000 + i, (n_side,) * 3, n - half)
    return spec, k, codes, np.ascontiguousarray(np.concatenate([cam, rnd]))


# Served: 16 resident volumes -- 4 each at 256^3, 512^3, 1024^3 and 2 each at 2048^3,
# 4096^3 -- shells of 32*N/512 primitives in the format G(k-4) R(4,4,4) with whole-level
# de-duplication; requests are seeded cameras at a resolution uniform over
# {256x256, 512x512, 1280x720, 1920x1080}, half of them followed by one bounce per hit.
SERVED = dict(name="served-16", seed=5, sides=[8, 8, 8, 8, 9, 9, 9, 9, 10, 10, 10, 10, 11, 11, 12, 12],
              resolutions=[(256, 256), (512, 512), (1280, 720), (1920, 1080)], bounce_p=0.5)


def served_volume(cfg: dict, i: int):
    k = cfg["sides"][i]
    n = 1 << k
    prims = 32 * n // 512
    codes = scene_shell(cfg["seed"] * 100 + i, k, prims - prims // 4, prims // 4, 1.2)
    return f"G({k - 4}) R(4,4,4) --whole-level-dedup", k, codes

"""Workload recipes (inputs only): seeded scenes, format specs and ray sets.

The paper evaluates voxelized mesh models (San Miguel, Hairball, Buddha, Sponza) at
512^3 and 2048^3; those models are not available, so seeded synthetic SDF scenes of the
same resolutions stand in for them. Format specs follow the paper's grammar (R(k,k,k)
has 2^k cells per axis); several come from its table of evaluated formats.
"""
from __future__ import annotations

import numpy as np

from . import camera_rays, scene_shell, scene_solid_noise

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

# 2048^3 surface volume: 96 spheres + 32 tori; SVDAG top 7 levels -> Raw 16^3 bricks, and
# SVO -> Raw 8^3; 1080p primary rays plus one cosine-weighted bounce per primary hit.
SURF2048 = dict(name="surface-2048", log2n=11, seed=3, n_sph=96, n_tor=32, scale=1.2, width=1920, height=1080,
                views=1, specs=["G(7) R(4,4,4) --whole-level-dedup", "S(8) R(3,3,3)"], bounce_seed=33)


def scene(cfg: dict) -> np.ndarray:
    if cfg["name"].startswith("small"):
        return scene_solid_noise(cfg["seed"], log2n=cfg["log2n"], n_sph=8, rmin=4.0, rmax=16.0, noise=0.05)
    return scene_shell(cfg["seed"], cfg["log2n"], cfg["n_sph"], cfg["n_tor"], cfg["scale"])


def primary_rays(cfg: dict, view: int, width: int | None = None, height: int | None = None) -> np.ndarray:
    n = 1 << cfg["log2n"]
    return camera_rays(cfg["seed"], view, (n, n, n), width or cfg["width"], height or cfg["height"])

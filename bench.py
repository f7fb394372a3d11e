#!/usr/bin/env python3
"""Benchmark: ray intersection through hybrid voxel formats on one MI355X.

Default workload (one "step"): the 512^3 surface volume (shell of 32 spheres + 16
tori) in nine formats, four seeded 1920x1080 pinhole views each, i.e. 36 hvf_trace
launches over 74,649,600 primary rays. Inputs are resident in HBM before timing.
value = rays traced per second over the timed steps (Mrays/s).

Also reported (extra keys): the 2048^3 surface volume in its two formats, 1080p
primary rays and one cosine-weighted bounce ray per primary hit (incoherent).

roofline: algorithmic bytes per ray (32 B ray + 16 B hit + 64 B per distinct 64-byte
sector of the format the traversal reads, from the counting kernel on a ray sample)
times rays per launch, over the launch time measured with HIP events on the stream the
kernels run on; peak = 8 TB/s HBM.

cpu_baseline: the CPU oracle on a bounded sample of the same rays and formats.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
RAY_B, HIT_B = 32, 16


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("hvf_trace.hip", "hvf_build.cpp", "hvf_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2410_14128_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def distinct_per_ray(logt, cnt, shift: int):
    """Distinct (word_index >> shift) values per ray, from the counting kernel's log."""
    import torch
    cap = logt.shape[1]
    k = torch.clamp(cnt, max=cap)
    valid = torch.arange(cap, device=logt.device)[None, :] < k[:, None]
    v = torch.where(valid, logt >> shift, torch.full_like(logt, 2 ** 31 - 1))
    v, _ = torch.sort(v, dim=1)
    new = torch.ones_like(v, dtype=torch.bool)
    new[:, 1:] = v[:, 1:] != v[:, :-1]
    new &= v != 2 ** 31 - 1
    return new.sum(dim=1)


def byte_model(vol, rays_sample, cap=4096):
    """Mean algorithmic bytes per ray: (word model, sector model), plus overflow count."""
    import torch
    hits, logt, cnt = vol.trace_count(rays_sample, cap=cap)
    torch.cuda.synchronize()
    words = distinct_per_ray(logt, cnt, 0).double()
    sectors = distinct_per_ray(logt, cnt, 4).double()
    over = int((cnt > cap).sum())
    return (RAY_B + HIT_B + 4.0 * words.mean().item(), RAY_B + HIT_B + 64.0 * sectors.mean().item(),
            float(cnt.double().mean().item()), over, hits)


# VALU issue peak of MI355X: 256 CUs x 4 SIMDs, each issuing one wave64 VALU instruction per
# 4 cycles (16 lanes per cycle) at 2.4 GHz, in wave instructions per second.
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4


def profile_entry(name: str, kernel: str):
    """The committed rocprofv3 summary entry of `kernel` on workload `name`
    (profiles/pmc_traffic.json), or None when absent, taken for another kernel or with a
    different kernel source."""
    p = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("kernel_hash") != kernel_source_hash():
        return None
    w = d.get("workloads", {}).get(name)
    if w is None or w.get("kernel") != kernel:
        return None
    return w


def traffic_from_profile(name: str, kernel: str):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, each scaled by the same
    counter's reading for a plain 1 GiB copy) from the committed rocprofv3 PMC summary, or
    None when absent, taken for another kernel or with a different kernel source."""
    w = profile_entry(name, kernel)
    return None if w is None else round(float(w["bytes_per_launch"]))


def time_launches(fn_list, steps, warmup):
    """Run a step = every fn in fn_list once, with events on the current (launch) stream
    around the timed steps. Returns (ms_per_step, per-launch mean ms list). A step of one
    launch is timed by the events around its `steps` back-to-back launches alone (event
    pairs around each launch would add their own gaps to it); steps of several launches also
    record an event pair around each launch, to split the step between them."""
    import torch
    for _ in range(warmup):
        for fn in fn_list:
            fn()
    torch.cuda.synchronize()
    if len(fn_list) == 1:
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(steps):
            fn_list[0]()
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / steps
        return ms, [ms]
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in fn_list]
          for _ in range(steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for s in range(steps):
        for j, fn in enumerate(fn_list):
            ev[s][j][0].record()
            fn()
            ev[s][j][1].record()
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    per = [float(np.mean([ev[s][j][0].elapsed_time(ev[s][j][1]) for s in range(steps)])) for j in range(len(fn_list))]
    return total_ms / steps, per


SCHEDULE_BOUNCE = os.path.join(ROOT, "workloads", "schedule_bounce2048.json")


def run_headline(args, torch, H, W, C):
    """The bench step: one trace call over the bounce (incoherent) rays of one 1920x1080 frame
    of the 2048^3 surface volume in G(7) R(4,4,4) --whole-level-dedup, rays and hits resident
    in HBM. The primary frame is traced once (plain schedule, untimed) to derive the bounce
    rays. The schedule comes from the committed autotuner result unless --retune (then the
    autotuner picks it on the bounce rays of a held-out view, truncated to the same count).
    Roofline of the call's kernel: algorithmic bytes per launch (B_ray, sector model, from the
    counting kernel on a seeded sample of the same rays, times the rays) over its mean launch
    time from HIP events on the launch stream."""
    cfg = C.SURF2048
    n = 1 << cfg["log2n"]
    t0 = time.time()
    codes = C.scene(cfg)
    spec = cfg["specs"][0]
    log(f"[bench] headline: 2048^3 scene {len(codes)} voxels ({len(codes) / n ** 3:.4%}) in {time.time() - t0:.1f}s")
    prim = C.primary_rays(cfg, 0)
    v = H.Volume(spec, codes)
    v.upload()
    plain = H.schedule()
    h = v.trace(torch.from_numpy(prim).cuda(), sched=plain)
    torch.cuda.synchronize()
    b, _ = W.bounce_rays(cfg["bounce_seed"], prim, h.cpu().numpy())
    del h
    d_b = torch.from_numpy(b).cuda()
    hb = torch.empty((len(b), 4), dtype=torch.int32, device="cuda")
    fixed = {} if (args.retune or args.no_tune) else load_schedules(SCHEDULE_BOUNCE)
    if args.no_tune:
        sched = H.schedule_dict(plain)
    elif spec in fixed:
        v.set_schedule(H.schedule(**fixed[spec]))
        sched = H.schedule_dict(v.get_schedule())
    else:
        held = C.primary_rays(cfg, 1)
        hh = v.trace(torch.from_numpy(held).cuda(), sched=plain)
        torch.cuda.synchronize()
        bt, _ = W.bounce_rays(cfg["bounce_seed"] + 1, held, hh.cpu().numpy())
        sched = H.schedule_dict(v.autotune(torch.from_numpy(np.ascontiguousarray(bt[:len(b)])).cuda()))
        del hh, bt
    source = ("autotuned on a held-out view's bounce rays" if not fixed else
              f"from {os.path.relpath(SCHEDULE_BOUNCE, ROOT)}")
    log(f"[bench] headline: {len(b)} bounce rays, schedule {sched} ({source}); warmup {args.warmup}, "
        f"timing {args.steps} steps")
    # The untimed reference trace and byte accounting run first, so the GPU is busy right
    # before the warm-up launches.
    ref = v.trace(d_b, sched=plain)
    info = v.info()
    kernel = H.kernel_name(info, sched)
    if args.sample > 0:
        rng = np.random.default_rng(4242)
        smp = torch.from_numpy(b[np.sort(rng.choice(len(b), min(args.sample, len(b)), replace=False))]).cuda()
        bw, bs, loads, over, _ = byte_model(v, smp)
    else:
        bw = bs = loads = float("nan")
        over = 0
    ms, per = time_launches([lambda: v.trace(d_b, hb)], args.steps, args.warmup)
    torch.cuda.synchronize()
    same = bool(torch.equal(hb, ref))
    value = len(b) / (ms * 1e-3) / 1e6
    avg_ms = per[0]
    bytes_launch = bs * len(b)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    fin = bool(np.isfinite(achieved))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1) if fin else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4) if fin else None,
                "traffic": traffic_from_profile("headline-bounce-2048", kernel),
                "kernel": kernel, "launches_per_step": 1, "avg_launch_us": round(avg_ms * 1e3, 2),
                "algorithmic_bytes_per_launch": round(bytes_launch) if fin else None,
                "B_ray_sector": round(bs, 1), "B_ray_word": round(bw, 1), "loads_per_ray": round(loads, 1),
                "log_overflow_rays": over, "grid_threads": ((len(b) + 255) // 256) * 256,
                "roof_mrays_s": round(HBM_PEAK_GBS * 1e9 / bs / 1e6, 1) if fin else None}
    # `achieved` counts algorithmic bytes (the sector model); the measured HBM bytes (FETCH_SIZE +
    # WRITE_SIZE from the committed counters) over the same launch time sit beside it.
    if roofline["traffic"] is not None:
        roofline["traffic_gbs"] = round(roofline["traffic"] / (avg_ms * 1e-3) / 1e9, 1)
        roofline["traffic_frac"] = round(roofline["traffic_gbs"] / HBM_PEAK_GBS, 4)
    # The launch is bound by VALU issue rather than HBM: the committed SQ_INSTS_VALU count per
    # launch over the same launch time, against the chip's issue rate.
    ent = profile_entry("headline-bounce-2048", kernel)
    if ent is not None and "valu_wave_insts_per_launch" in ent:
        rate = ent["valu_wave_insts_per_launch"] / (avg_ms * 1e-3)
        roofline["valu_issue"] = {"bound": "alu", "achieved": round(rate / 1e9, 1),
                                  "peak": round(VALU_PEAK_WAVE_INSTS / 1e9, 1),
                                  "unit": "G wave64 VALU instructions/s",
                                  "frac": round(rate / VALU_PEAK_WAVE_INSTS, 4),
                                  "insts_per_launch": ent["valu_wave_insts_per_launch"]}
    log(f"[bench] headline: {ms * 1e3:.1f} us per step, {value:.1f} Mrays/s; {kernel} {avg_ms * 1e3:.1f} us, "
        f"B_ray {bs:.0f} B, {achieved:.0f} GB/s algorithmic ({achieved / HBM_PEAK_GBS:.1%} of HBM roofline); "
        f"hits identical to the plain schedule: {same}")
    out = {"value": value, "ms": ms, "rays": len(b), "roofline": roofline, "schedule": sched,
           "schedule_source": source, "identical_to_plain": same, "format": spec, "format_bytes": info["bytes"],
           "occupancy": len(codes) / n ** 3, "bounce": b}
    v.close()
    return out


def run_small(args, torch, H, W, C):
    """The small case: 64^3 solid spheres with 5% noise in R(2,2,2) S(2) R(2,2,2), one 256x256
    view of primary rays, autotuned on a held-out view of the same size."""
    cfg = C.SMALL
    codes = C.scene(cfg)
    rays = C.primary_rays(cfg, 0)
    v = H.Volume(cfg["spec"], codes)
    v.upload()
    d = torch.from_numpy(rays).cuda()
    hits = torch.empty((len(rays), 4), dtype=torch.int32, device="cuda")
    sched = (H.schedule_dict(v.get_schedule()) if args.no_tune else
             H.schedule_dict(v.autotune(torch.from_numpy(C.primary_rays(cfg, 1)).cuda())))
    ms, per = time_launches([lambda: v.trace(d, hits)], args.steps, args.warmup)
    if args.sample > 0:
        bw, bs, loads, _, _ = byte_model(v, d)
    else:
        bw = bs = loads = float("nan")
    r = {"format": cfg["spec"], "rays": len(rays), "ms": ms, "mrays_s": len(rays) / (ms * 1e-3) / 1e6,
         "B_ray_sector": bs, "B_ray_word": bw, "loads_per_ray": loads, "schedule": sched,
         "kernel": H.kernel_name(v.info(), sched), "format_bytes": v.info()["bytes"],
         "occupancy": len(codes) / 64 ** 3}
    r["frac_roofline"] = r["mrays_s"] * 1e6 * bs / (HBM_PEAK_GBS * 1e9)
    r.update({k: round(x, 4) for k, x in r.items() if isinstance(x, float)})
    log(f"[bench] small-64 {cfg['spec']}: {r['mrays_s']:.1f} Mrays/s ({r['frac_roofline']:.1%}, B_ray {bs:.0f} B, "
        f"{sched})")
    v.close()
    return r


def run_surface512(args, torch, H, W, C):
    cfg = C.SURF512
    n = 1 << cfg["log2n"]
    t0 = time.time()
    codes = C.scene(cfg)
    log(f"[bench] surface-512: {len(codes)} voxels ({len(codes) / n ** 3:.4%}) in {time.time() - t0:.1f}s")
    views = [C.primary_rays(cfg, v) for v in range(cfg["views"])]
    d_views = [torch.from_numpy(r).cuda() for r in views]
    hits = [torch.empty((len(r), 4), dtype=torch.int32, device="cuda") for r in views]
    vols = []
    for spec in cfg["specs"]:
        v = H.Volume(spec, codes)
        v.upload()
        vols.append(v)
    torch.cuda.synchronize()
    fns = []
    for v in vols:
        for j in range(len(views)):
            fns.append(lambda v=v, j=j: v.trace(d_views[j], hits[j]))
    # Autotune each format on a held-out view (a fifth seeded camera at the timed 1920x1080:
    # schedules that shorten a launch's tail pay off differently at other ray counts), then time
    # the tuned schedules: the timed region. The untuned comparison (--untuned) runs after
    # it, so a profile of the timed kernels is not mixed with it.
    # Schedules come from the committed autotuner results (workloads/schedules_surface512.json,
    # written by a --retune run on this GPU) when present: the autotuner's choice between
    # schedules within a few percent of each other varies from run to run, and the profiles
    # of the dominant kernel must see the same launches as the bench line.
    fixed = {} if (args.retune or args.no_tune) else load_schedules(args.schedules)
    tune = torch.from_numpy(C.primary_rays(cfg, cfg["views"])).cuda()
    scheds = []
    for spec, v in zip(cfg["specs"], vols):
        if args.no_tune:
            scheds.append(H.schedule_dict(v.get_schedule()))
        elif spec in fixed:
            v.set_schedule(H.schedule(**fixed[spec]))
            scheds.append(H.schedule_dict(v.get_schedule()))
        else:
            scheds.append(H.schedule_dict(v.autotune(tune)))
    del tune
    tuned_from = "autotuned on a held-out view" if not fixed else f"from {os.path.relpath(args.schedules, ROOT)}"
    log(f"[bench] surface-512: {len(fns)} launches per step; warmup {args.warmup}, timing {args.steps} steps")
    ms, per = time_launches(fns, args.steps, args.warmup)
    rays_per_step = sum(len(r) for r in views) * len(vols)
    value = rays_per_step / (ms * 1e-3) / 1e6
    log(f"[bench] surface-512: {ms:.2f} ms/step, {value:.1f} Mrays/s")
    per_plain = None
    if args.untuned:
        plain = H.schedule()
        fns_plain = [lambda v=v, j=j: v.trace(d_views[j], hits[j], sched=plain) for v in vols for j in range(len(views))]
        _, per_plain = time_launches(fns_plain, args.steps, args.warmup)
    # Byte model per format and view on a seeded sample of each view's pixels.
    rng = np.random.default_rng(12345)
    sample_idx = [np.sort(rng.choice(len(r), size=min(args.sample, len(r)), replace=False)) for r in views]
    per_format = []
    launch_bytes = []  # algorithmic bytes of each timed launch (format-major, like fns)
    kernels = []       # trace kernel of each timed launch
    for fi, (spec, v) in enumerate(zip(cfg["specs"], vols)):
        info = v.info()
        bw, bs, loads, over = [], [], [], 0
        for j, r in enumerate(views):
            if args.sample <= 0:
                bw.append(float("nan")), bs.append(float("nan")), loads.append(float("nan"))
            else:
                smp = torch.from_numpy(r[sample_idx[j]]).cuda()
                w_, s_, l_, o_, _ = byte_model(v, smp)
                bw.append(w_)
                bs.append(s_)
                loads.append(l_)
                over += o_
            launch_bytes.append(bs[-1] * len(r))
            kernels.append(H.kernel_name(info, scheds[fi]))
        launch_ms = per[fi * len(views):(fi + 1) * len(views)]
        nrays = sum(len(r) for r in views)
        fmt_ms = float(np.sum(launch_ms))
        per_format.append({
            "format": spec, "format_bytes": info["bytes"], "mrays_s": nrays / (fmt_ms * 1e-3) / 1e6,
            "schedule": scheds[fi], "kernel": kernels[-1],
            "ms": fmt_ms, "B_ray_sector": round(float(np.mean(bs)), 1), "B_ray_word": round(float(np.mean(bw)), 1),
            "loads_per_ray": round(float(np.mean(loads)), 1), "log_overflow_rays": over,
            "roof_mrays_s": HBM_PEAK_GBS * 1e9 / float(np.mean(bs)) / 1e6,
        })
        if per_plain is not None:
            plain_ms = float(np.sum(per_plain[fi * len(views):(fi + 1) * len(views)]))
            per_format[-1]["mrays_s_untuned"] = nrays / (plain_ms * 1e-3) / 1e6
        per_format[-1]["frac_roofline"] = per_format[-1]["mrays_s"] / per_format[-1]["roof_mrays_s"]
        log(f"[bench]   {spec:42s} {per_format[-1]['mrays_s']:8.1f} Mrays/s ({scheds[fi]}, {kernels[-1]})  "
            f"B_ray {np.mean(bs):7.1f} B ({per_format[-1]['frac_roofline']:.1%} of HBM roof)  "
            f"size {info['bytes'] / 2 ** 20:.1f} MiB")
    # Roofline of the dominant kernel: the trace kernel with the largest share of the step.
    # achieved = its algorithmic bytes per launch / its mean launch time (HIP events on the
    # launch stream); both are means over its launches in one step.
    tot = {}
    for k, t in zip(kernels, per):
        tot[k] = tot.get(k, 0.0) + t
    dom = max(tot, key=tot.get)
    idx = [i for i, k in enumerate(kernels) if k == dom]
    avg_ms = float(np.mean([per[i] for i in idx]))
    bytes_launch = float(np.mean([launch_bytes[i] for i in idx]))
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    all_achieved = float(np.sum(launch_bytes)) / (float(np.sum(per)) * 1e-3) / 1e9
    fin = bool(np.isfinite(achieved))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1) if fin else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4) if fin else None,
                "traffic": traffic_from_profile("surface-512", dom),
                "kernel": dom, "launches_per_step": len(idx), "share_of_step": round(tot[dom] / float(np.sum(per)), 3),
                "avg_launch_us": round(avg_ms * 1e3, 2),
                "algorithmic_bytes_per_launch": round(bytes_launch) if np.isfinite(bytes_launch) else None,
                "grid_threads": len(views[0]),
                "formats": sorted({cfg["specs"][i // len(views)] for i in idx}),
                "all_launches_achieved": round(all_achieved, 1) if np.isfinite(all_achieved) else None}
    log(f"[bench] surface-512 dominant kernel {dom}: {len(idx)} launches/step, {avg_ms * 1e3:.1f} us each, "
        f"{achieved:.0f} GB/s algorithmic ({achieved / HBM_PEAK_GBS:.1%}); all launches {all_achieved:.0f} GB/s")
    return {
        "value": value, "ms": ms, "rays_per_step": rays_per_step, "roofline": roofline,
        "per_format": per_format, "schedules": tuned_from,
        "codes": codes, "views": views, "sample_idx": sample_idx, "occupancy": len(codes) / n ** 3,
    }


def raw_twin(spec):
    """The same hierarchy with every distance-field level D(W,H,D,M) replaced by Raw R(W,H,D)."""
    import re
    return re.sub(r"D\((\d+),(\d+),(\d+),\d+\)", r"R(\1,\2,\3)", spec)


def run_df512(args, torch, H, C, res):
    """Distance-field formats of the table at 512^3, each beside its Raw twin (same levels,
    no distances), autotuned like the nine headline formats and timed over the 4 views."""
    cfg = C.SURF512
    codes, views = res["codes"], res["views"]
    d_views = [torch.from_numpy(r).cuda() for r in views]
    hits = [torch.empty((len(r), 4), dtype=torch.int32, device="cuda") for r in views]
    tune = torch.from_numpy(C.primary_rays(cfg, cfg["views"])).cuda()
    nrays = sum(len(r) for r in views)
    out = []
    for spec in C.SURF512_DF:
        row = {"format": spec, "raw_twin": raw_twin(spec)}
        for key, sp in (("df", spec), ("raw", row["raw_twin"])):
            v = H.Volume(sp, codes)
            v.upload()
            sched = H.schedule_dict(v.get_schedule() if args.no_tune else v.autotune(tune))
            ms, _ = time_launches([lambda v=v, j=j: v.trace(d_views[j], hits[j]) for j in range(len(views))],
                                  args.steps, args.warmup)
            row[key] = {"mrays_s": round(nrays / (ms * 1e-3) / 1e6, 1), "bytes": v.info()["bytes"], "schedule": sched}
            del v
        row["df_over_raw"] = round(row["df"]["mrays_s"] / row["raw"]["mrays_s"], 3)
        log(f"[bench]   DF {spec:46s} {row['df']['mrays_s']:8.1f} Mrays/s  twin {row['raw_twin']:36s} "
            f"{row['raw']['mrays_s']:8.1f}  x{row['df_over_raw']:.2f}  size {row['df']['bytes'] / 2 ** 20:.1f} MiB "
            f"vs {row['raw']['bytes'] / 2 ** 20:.1f}")
        out.append(row)
    return out


SCHEDULES_512 = os.path.join(ROOT, "workloads", "schedules_surface512.json")


def load_schedules(path: str) -> dict:
    """Per-format schedules of the 512^3 formats from a bench JSON line (or its
    per_format list); {} when the file is absent or unreadable."""
    try:
        d = json.load(open(path))
    except Exception:
        return {}
    rows = d.get("per_format", []) if isinstance(d, dict) else d
    keys = set(H_schedule_fields())
    out = {}
    for r in rows:
        sc = r.get("schedule")
        if isinstance(sc, dict) and set(sc) <= keys:
            out[r["format"]] = sc
    return out


def H_schedule_fields():
    import paper_2410_14128_amd as H
    return [f for f, _ in H.hvf_schedule._fields_]


def run_sweep(args, torch, H, W, C):
    """Every format of the paper's table on the matching synthetic volume: GPU-layout size
    against Mrays/s, one lane per ray (1080p primary rays of view 0; at 2048^3 also the
    bounce rays of those hits), and the Pareto set of (size, primary Mrays/s)."""
    out = []
    for log2n, cfg in ((9, C.SURF512), (11, C.SURF2048)):
        codes = C.scene(cfg)
        prim = C.primary_rays(cfg, 0)
        d_prim = torch.from_numpy(prim).cuda()
        h = torch.empty((len(prim), 4), dtype=torch.int32, device="cuda")
        d_b = hb = None
        for label, k, spec in C.TABLE_FORMATS:
            if k != log2n:
                continue
            sp = C.table_spec(spec)
            t0 = time.time()
            v = H.Volume(sp, codes)
            tb = time.time() - t0
            v.upload()
            plain = H.schedule()
            ms, _ = time_launches([lambda: v.trace(d_prim, h, sched=plain)], args.steps, args.warmup)
            rec = {"label": label, "format": sp, "side": 1 << k, "bytes": v.info()["bytes"], "build_s": round(tb, 2),
                   "primary_mrays_s": round(len(prim) / ms / 1e3, 1)}
            if k == 11:
                if d_b is None:
                    torch.cuda.synchronize()
                    b, _ = W.bounce_rays(cfg["bounce_seed"], prim, h.cpu().numpy())
                    d_b = torch.from_numpy(b).cuda()
                    hb = torch.empty((len(b), 4), dtype=torch.int32, device="cuda")
                msb, _ = time_launches([lambda: v.trace(d_b, hb, sched=plain)], args.steps, args.warmup)
                rec["bounce_mrays_s"] = round(d_b.shape[0] / msb / 1e3, 1)
            log(f"[bench] sweep {label:2d} {sp:44s} {rec['bytes'] / 2 ** 20:9.1f} MiB  primary {rec['primary_mrays_s']:8.1f}"
                + (f"  bounce {rec['bounce_mrays_s']:8.1f}" if "bounce_mrays_s" in rec else "") + " Mrays/s")
            out.append(rec)
            v.close()
    for side in (512, 2048):
        rows = sorted([r for r in out if r["side"] == side], key=lambda r: (r["bytes"], -r["primary_mrays_s"]))
        best = -1.0
        for r in rows:
            r["pareto"] = r["primary_mrays_s"] > best
            best = max(best, r["primary_mrays_s"])
    return out


def run_sweep_paper(args, torch, H, W, C):
    """The format sweep in both layouts: every format of the paper's table built in the
    library's own layout and in the paper's word layout (--paper-layout, RGBA voxel words),
    each traced with one lane per ray on 1080p primary rays of view 0 (at 2048^3 also their
    bounce rays). The two layouts' hits are compared bit for bit on every launch."""
    out = []
    for log2n, cfg in ((9, C.SURF512), (11, C.SURF2048)):
        codes = C.scene(cfg)
        prim = C.primary_rays(cfg, 0)
        d_prim = torch.from_numpy(prim).cuda()
        h = torch.empty((len(prim), 4), dtype=torch.int32, device="cuda")
        h_own = torch.empty_like(h)
        d_b = hb = hb_own = None
        plain = H.schedule()
        for label, k, spec in C.TABLE_FORMATS:
            if k != log2n:
                continue
            sp = C.table_spec(spec)
            own = H.Volume(sp, codes)
            t0 = time.time()
            v = H.Volume(sp + " --paper-layout", codes)
            tb = time.time() - t0
            own.trace(d_prim, h_own, sched=plain)
            ms_own, _ = time_launches([lambda: own.trace(d_prim, h_own, sched=plain)], args.steps, args.warmup)
            ms, _ = time_launches([lambda: v.trace(d_prim, h, sched=plain)], args.steps, args.warmup)
            torch.cuda.synchronize()
            if not torch.equal(h, h_own):
                raise RuntimeError(f"paper layout and own layout differ on {sp} primary rays")
            rec = {"label": label, "format": sp, "side": 1 << k, "bytes": own.info()["bytes"],
                   "paper_bytes": v.info()["bytes"], "paper_build_s": round(tb, 2),
                   "primary_mrays_s": round(len(prim) / ms_own / 1e3, 1),
                   "paper_primary_mrays_s": round(len(prim) / ms / 1e3, 1)}
            if k == 11:
                if d_b is None:
                    b, _ = W.bounce_rays(cfg["bounce_seed"], prim, h_own.cpu().numpy())
                    d_b = torch.from_numpy(b).cuda()
                    hb = torch.empty((len(b), 4), dtype=torch.int32, device="cuda")
                    hb_own = torch.empty_like(hb)
                msb_own, _ = time_launches([lambda: own.trace(d_b, hb_own, sched=plain)], args.steps, args.warmup)
                msb, _ = time_launches([lambda: v.trace(d_b, hb, sched=plain)], args.steps, args.warmup)
                torch.cuda.synchronize()
                if not torch.equal(hb, hb_own):
                    raise RuntimeError(f"paper layout and own layout differ on {sp} bounce rays")
                rec["bounce_mrays_s"] = round(d_b.shape[0] / msb_own / 1e3, 1)
                rec["paper_bounce_mrays_s"] = round(d_b.shape[0] / msb / 1e3, 1)
            log(f"[bench] sweep-paper {label:2d} {sp:44s} own {rec['bytes'] / 2 ** 20:8.1f} MiB "
                f"{rec['primary_mrays_s']:8.1f}  paper {rec['paper_bytes'] / 2 ** 20:8.1f} MiB "
                f"{rec['paper_primary_mrays_s']:8.1f} Mrays/s primary"
                + (f"; bounce own {rec['bounce_mrays_s']:7.1f} paper {rec['paper_bounce_mrays_s']:7.1f}"
                   if "bounce_mrays_s" in rec else "") + f" (paper build {tb:.1f} s)")
            out.append(rec)
            v.close()
            own.close()
    return out


def run_construction(args, torch, H, C, formats_2048=None):
    """Format construction from sorted Morton codes: the host builder plus the upload of its
    buffer, against hvf_build_device on codes already resident on the device (median of
    three builds each; the device figure includes the download of the host copy). The two
    word buffers are compared word for word."""
    out = []
    specs = formats_2048 or [C.table_spec(sp) for _, k, sp in C.TABLE_FORMATS if k == 11]
    # the paper's word layout: a few 512^3 formats, and one 2048^3 format beside the others
    paper512 = [sp + " --paper-layout" for sp in ("G(9) --whole-level-dedup", "R(4,4,4) G(5) --whole-level-dedup",
                                                  "R(4,4,4) S(5)", "D(4,4,4,6) G(5) --whole-level-dedup")]
    paper2048 = ["G(11) --whole-level-dedup --paper-layout"]
    for cfg, fmts in ((C.SURF512, C.SURF512["specs"] + C.SURF512_DF + paper512), (C.SURF2048, specs + paper2048)):
        codes = C.scene(cfg)
        d_codes = torch.from_numpy(codes.view(np.int64)).cuda()
        H.Volume.from_device("S(3)", d_codes[:1] * 0).close()  # load the construction kernels
        for sp in fmts:
            th, td = [], []
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                vh = H.Volume(sp, codes)
                vh.upload()
                torch.cuda.synchronize()
                th.append(time.perf_counter() - t0)
                t0 = time.perf_counter()
                vd = H.Volume.from_device(sp, d_codes)
                torch.cuda.synchronize()
                td.append(time.perf_counter() - t0)
                same = bool(np.array_equal(vh.words(), vd.words()))
                nbytes = vh.info()["bytes"]
                vh.close()
                vd.close()
                if not same:
                    raise RuntimeError(f"device construction differs from the host builder for {sp}")
            rec = {"format": sp, "side": 1 << cfg["log2n"], "voxels": int(len(codes)), "bytes": nbytes,
                   "host_ms": round(1e3 * float(np.median(th)), 2), "device_ms": round(1e3 * float(np.median(td)), 2),
                   "identical": same}
            rec["speedup"] = round(rec["host_ms"] / rec["device_ms"], 1)
            log(f"[bench] build {rec['side']:4d}^3 {sp:44s} {nbytes / 2 ** 20:8.1f} MiB  host+upload "
                f"{rec['host_ms']:8.1f} ms  device {rec['device_ms']:7.1f} ms  x{rec['speedup']}")
            out.append(rec)
        del d_codes
    return out


def run_restart(args, torch, H, W, C):
    """Restarting sparse-voxel intersection (--restart-sv) against the stacked walk, for every
    2048^3 format of the paper's table with an SVO or SVDAG level (Sec. 4.3): 1080p primary
    rays of view 0 and their bounce rays, plain schedule, one lane per ray."""
    cfg = C.SURF2048
    codes = C.scene(cfg)
    prim = C.primary_rays(cfg, 0)
    d_prim = torch.from_numpy(prim).cuda()
    h = torch.empty((len(prim), 4), dtype=torch.int32, device="cuda")
    plain = H.schedule()
    out = []
    d_b = hb = None
    for label, k, spec in C.TABLE_FORMATS:
        if k != 11 or not any(c in spec for c in ("S(", "G(")):
            continue
        base = C.table_spec(spec)
        rec = {"label": label, "format": base}
        for key, sp in (("stacked", base), ("restart", base + " --restart-sv")):
            v = H.Volume(sp, codes)
            v.upload()
            ms, _ = time_launches([lambda: v.trace(d_prim, h, sched=plain)], args.steps, args.warmup)
            if d_b is None:
                torch.cuda.synchronize()
                b, _ = W.bounce_rays(cfg["bounce_seed"], prim, h.cpu().numpy())
                d_b = torch.from_numpy(b).cuda()
                hb = torch.empty((len(b), 4), dtype=torch.int32, device="cuda")
            msb, _ = time_launches([lambda: v.trace(d_b, hb, sched=plain)], args.steps, args.warmup)
            rec[key] = {"primary_mrays_s": round(len(prim) / ms / 1e3, 1), "bounce_mrays_s": round(d_b.shape[0] / msb / 1e3, 1)}
            v.close()
        rec["primary_ratio"] = round(rec["restart"]["primary_mrays_s"] / rec["stacked"]["primary_mrays_s"], 3)
        rec["bounce_ratio"] = round(rec["restart"]["bounce_mrays_s"] / rec["stacked"]["bounce_mrays_s"], 3)
        log(f"[bench] restart {label:2d} {base:44s} primary x{rec['primary_ratio']:.3f}  bounce x{rec['bounce_ratio']:.3f}")
        out.append(rec)
    return out


def run_surface2048(args, torch, H, W, C):
    cfg = C.SURF2048
    n = 1 << cfg["log2n"]
    t0 = time.time()
    codes = C.scene(cfg)
    log(f"[bench] surface-2048: {len(codes)} voxels ({len(codes) / n ** 3:.4%}) in {time.time() - t0:.1f}s")
    prim = C.primary_rays(cfg, 0)
    d_prim = torch.from_numpy(prim).cuda()
    held = C.primary_rays(cfg, 1)  # held-out camera at the timed resolution, for the autotuner
    d_held = torch.from_numpy(held).cuda()
    out = []
    for spec in cfg["specs"]:
        v = H.Volume(spec, codes)
        v.upload()
        h = v.trace(d_prim)
        hh = v.trace(d_held)
        torch.cuda.synchronize()
        b, _ = W.bounce_rays(cfg["bounce_seed"], prim, h.cpu().numpy())
        bh, _ = W.bounce_rays(cfg["bounce_seed"] + 1, held, hh.cpu().numpy())
        d_b = torch.from_numpy(b).cuda()
        hb = torch.empty((len(b), 4), dtype=torch.int32, device="cuda")
        plain = H.schedule()
        sched_p = H.schedule_dict(v.autotune(d_held)) if not args.no_tune else H.schedule_dict(plain)
        ms_p, _ = time_launches([lambda: v.trace(d_prim, h)], args.steps, args.warmup)
        # Tune on as many held-out bounce rays as the timed launch traces (the held-out view
        # has more hits than view 0, and a schedule's gain depends on the launch size).
        sched_b = H.schedule_dict(v.autotune(torch.from_numpy(bh[:len(b)].copy()).cuda())) if not args.no_tune else sched_p
        ms_b, _ = time_launches([lambda: v.trace(d_b, hb)], args.steps, args.warmup)
        frames = run_frames2048(args, torch, H, W, C, v, cfg, b)
        # untuned comparison after the timed launches (a profile of those stays unmixed; the
        # one-lane-per-ray launches of both grids are the run's last ones)
        ms_p0, _ = time_launches([lambda: v.trace(d_prim, h, sched=plain)], args.steps, args.warmup)
        ms_b0, _ = time_launches([lambda: v.trace(d_b, hb, sched=plain)], args.steps, args.warmup)
        rng = np.random.default_rng(7)
        if args.sample > 0:
            sp = torch.from_numpy(prim[rng.choice(len(prim), min(args.sample, len(prim)), replace=False)]).cuda()
            sb = torch.from_numpy(b[rng.choice(len(b), min(args.sample, len(b)), replace=False)]).cuda()
            wp, bp, lp, _, _ = byte_model(v, sp)
            wb, bb, lb, _, _ = byte_model(v, sb)
        else:
            wp = bp = lp = wb = bb = lb = float("nan")
        info = v.info()
        rec = {"format": spec, "format_bytes": info["bytes"],
               "primary": {"rays": len(prim), "ms": ms_p, "mrays_s": len(prim) / ms_p / 1e3, "B_ray_sector": bp,
                           "B_ray_word": wp, "loads_per_ray": lp, "schedule": sched_p,
                           "kernel": H.kernel_name(info, sched_p), "avg_launch_us": ms_p * 1e3,
                           "mrays_s_untuned": len(prim) / ms_p0 / 1e3},
               "incoherent": {"rays": len(b), "ms": ms_b, "mrays_s": len(b) / ms_b / 1e3, "B_ray_sector": bb,
                              "B_ray_word": wb, "loads_per_ray": lb, "schedule": sched_b,
                              "kernel": H.kernel_name(info, sched_b), "avg_launch_us": ms_b * 1e3,
                              "mrays_s_untuned": len(b) / ms_b0 / 1e3}}
        for k in ("primary", "incoherent"):
            r = rec[k]
            r["achieved_gbs"] = r["B_ray_sector"] * r["rays"] / (r["ms"] * 1e-3) / 1e9
            r["frac_roofline"] = r["achieved_gbs"] / HBM_PEAK_GBS
            r.update({kk: round(vv, 4) for kk, vv in r.items() if isinstance(vv, float)})
        rec["incoherent_8_frames"] = frames
        log(f"[bench]   2048 {spec:36s} primary {rec['primary']['mrays_s']:8.1f} Mrays/s "
            f"({rec['primary']['frac_roofline']:.1%}, untuned {rec['primary']['mrays_s_untuned']:.1f}, {sched_p})  "
            f"incoherent {rec['incoherent']['mrays_s']:8.1f} Mrays/s ({rec['incoherent']['frac_roofline']:.1%}, "
            f"B_ray {bb:.0f} B, untuned {rec['incoherent']['mrays_s_untuned']:.1f}, {sched_b})")
        out.append(rec)
        v.close()
    return {"occupancy": len(codes) / n ** 3, "formats": out}


def frame_bounces(torch, H, W, C, v, cfg, views, seed0):
    """Bounce rays of several 1080p frames of the 2048^3 volume, concatenated: each view's
    primary rays are traced (plain schedule) and one cosine-weighted bounce is drawn per hit
    with a seed of its own."""
    out = []
    for j in views:
        prim = C.primary_rays(cfg, j)
        h = v.trace(torch.from_numpy(prim).cuda(), sched=H.schedule())
        torch.cuda.synchronize()
        b, _ = W.bounce_rays(seed0 + j, prim, h.cpu().numpy())
        out.append(b)
    return np.concatenate(out)


def run_frames2048(args, torch, H, W, C, v, cfg, b0):
    """The bounce rays of 8 frames (8 seeded views; view 0's are the one-frame launch's)
    traced in one launch, as a wavefront renderer gathers secondary rays over frames or
    samples: the one-frame launch leaves most of the device idle in its tail. Tuned on 8
    held-out frames, truncated to the same ray count."""
    views = cfg["frame_views"]
    b8 = np.concatenate([b0, frame_bounces(torch, H, W, C, v, cfg, views[1:], cfg["bounce_seed"])])
    d8 = torch.from_numpy(b8).cuda()
    h8 = torch.empty((len(b8), 4), dtype=torch.int32, device="cuda")
    plain = H.schedule()
    if args.no_tune:
        sched = H.schedule_dict(plain)
    else:
        bt = frame_bounces(torch, H, W, C, v, cfg, cfg["tune_frame_views"], cfg["bounce_seed"] + 1000)[:len(b8)]
        sched = H.schedule_dict(v.autotune(torch.from_numpy(np.ascontiguousarray(bt)).cuda()))
        del bt
    ms, _ = time_launches([lambda: v.trace(d8, h8)], args.steps, args.warmup)
    ms0, _ = time_launches([lambda: v.trace(d8, h8, sched=plain)], args.steps, args.warmup)
    if args.sample > 0:
        rng = np.random.default_rng(8)
        _, bs, lb, _, _ = byte_model(v, torch.from_numpy(b8[rng.choice(len(b8), min(args.sample, len(b8)),
                                                                            replace=False)]).cuda())
    else:
        bs = lb = float("nan")
    r = {"frames": len(views), "views": views, "rays": len(b8), "ms": ms, "mrays_s": len(b8) / ms / 1e3,
         "B_ray_sector": bs, "loads_per_ray": lb, "schedule": sched, "kernel": H.kernel_name(v.info(), sched),
         "avg_launch_us": ms * 1e3, "mrays_s_untuned": len(b8) / ms0 / 1e3}
    r["achieved_gbs"] = r["B_ray_sector"] * r["rays"] / (r["ms"] * 1e-3) / 1e9
    r["frac_roofline"] = r["achieved_gbs"] / HBM_PEAK_GBS
    r.update({k: round(x, 4) for k, x in r.items() if isinstance(x, float)})
    log(f"[bench]   2048 incoherent, {len(views)} frames in one launch: {r['mrays_s']:8.1f} Mrays/s "
        f"({r['frac_roofline']:.1%}, untuned {r['mrays_s_untuned']:.1f}, {sched})")
    del d8, h8
    return r


def run_bounce2048(args, torch, H, W, C):
    """Only the incoherent launch of the 2048^3 leg (first format, plain schedule), for
    counter profiles: the primary frame is traced once to derive the bounce rays, then the
    bounce rays are traced warmup + steps times."""
    cfg = C.SURF2048
    codes = C.scene(cfg)
    prim = C.primary_rays(cfg, 0)
    v = H.Volume(cfg["specs"][0], codes)
    v.upload()
    h = v.trace(torch.from_numpy(prim).cuda())
    torch.cuda.synchronize()
    b, _ = W.bounce_rays(cfg["bounce_seed"], prim, h.cpu().numpy())
    d_b = torch.from_numpy(b).cuda()
    hb = torch.empty((len(b), 4), dtype=torch.int32, device="cuda")
    ms, _ = time_launches([lambda: v.trace(d_b, hb, sched=H.schedule())], args.steps, args.warmup)
    log(f"[bench] bounce-2048 {cfg['specs'][0]}: {len(b)} rays, {ms * 1e3:.1f} us per launch, "
        f"{len(b) / ms / 1e3:.1f} Mrays/s")


def run_batched(args, torch, H, W, C):
    """64 volumes of random hybrid formats, 64 ray batches of uneven size: one graph-captured
    persistent launch versus one hvf_trace launch per volume on the same stream."""
    cfg = C.BATCHED
    t0 = time.time()
    vols, d_rays, specs, ns = [], [], [], []
    for i in range(cfg["nvol"]):
        spec, k, codes, rays = C.batched_case(cfg, i)
        v = H.Volume(spec, codes)
        v.upload()
        vols.append(v)
        d_rays.append(torch.from_numpy(rays).cuda())
        specs.append(spec)
        ns.append(len(rays))
    total = int(sum(ns))
    log(f"[bench] batched: {len(vols)} volumes, {total} rays, built in {time.time() - t0:.1f}s")
    hits_plain = [torch.empty((n, 4), dtype=torch.int32, device="cuda") for n in ns]
    plain = H.schedule()
    fns = [lambda v=v, r=r, h=h: v.trace(r, h, sched=plain) for v, r, h in zip(vols, d_rays, hits_plain)]
    ms_plain, _ = time_launches(fns, args.steps, args.warmup)
    b = H.Batch(vols, d_rays)
    opts = b.autotune() if not args.no_tune else H.batch_opts()
    ms_b, _ = time_launches([b.run], args.steps, args.warmup)
    torch.cuda.synchronize()
    same = all(torch.equal(x, y) for x, y in zip(b.hits, hits_plain))
    b.close()
    rec = {"volumes": len(vols), "rays": total, "ms_batched": round(ms_b, 3), "ms_per_volume_launches": round(ms_plain, 3),
           "mrays_s_batched": round(total / ms_b / 1e3, 1), "mrays_s_per_volume": round(total / ms_plain / 1e3, 1),
           "speedup": round(ms_plain / ms_b, 3), "identical_hits": bool(same),
           "opts": {"refill": opts.refill, "inner": opts.inner, "blocks_per_cu": opts.blocks_per_cu,
                    "use_graph": opts.use_graph}}
    log(f"[bench] batched: graph {rec['mrays_s_batched']} Mrays/s vs per-volume {rec['mrays_s_per_volume']} Mrays/s "
        f"(x{rec['speedup']}), identical={same}, {rec['opts']}")
    for v in vols:
        v.close()
    return rec


def run_served(args, torch, H, W, C):
    """Poisson request streams against the server; p50/p99 latency and Mrays/s at 0.5, 0.8
    and 0.95 of the closed-loop saturation rate, plus a one-request-at-a-time baseline."""
    cfg = C.SERVED
    t0 = time.time()
    vols, pools = [], []
    for i in range(len(cfg["sides"])):
        spec, k, codes = C.served_volume(cfg, i)
        v = H.Volume(spec, codes)
        v.upload()
        vols.append(v)
        del codes
        n = 1 << k
        per = []

        def pinned(a):
            p = torch.empty(a.shape, dtype=torch.float32, pin_memory=True).numpy()
            p[...] = a
            return p

        for j, (w, h) in enumerate(cfg["resolutions"]):
            prim = W.camera_rays(cfg["seed"] * 100 + i, j, (n, n, n), w, h)
            hp = v.trace(torch.from_numpy(prim).cuda()).cpu().numpy()
            b, _ = W.bounce_rays(cfg["seed"] * 100 + i + 7, prim, hp)
            per.append((pinned(prim), pinned(np.ascontiguousarray(b))))
        pools.append(per)
    torch.cuda.synchronize()
    log(f"[bench] served: {len(vols)} volumes resident "
        f"({sum(v.info()['bytes'] for v in vols) / 2 ** 30:.2f} GiB), ray pools ready in {time.time() - t0:.1f}s")
    rng = np.random.default_rng(cfg["seed"])
    nreq = args.serve_requests + args.serve_warmup
    plan = [(int(rng.integers(0, len(vols))), int(rng.integers(0, 4)), bool(rng.random() < cfg["bounce_p"]))
            for _ in range(nreq)]

    def run(arrivals, slots, steps):
        srv = H.Server(args.serve_budget << 20, max_slots=slots, max_steps=steps)
        ids = [srv.add_volume(v) for v in vols]
        start = time.perf_counter()
        pending = {}  # primary request id -> plan index
        follow = {}   # bounce request id -> plan index
        t_sub = {}
        lat = {}
        rays_total = 0
        k = 0
        while k < nreq or pending or follow:
            now = time.perf_counter() - start
            while k < nreq and arrivals[k] <= now:
                vi, ri, bounce = plan[k]
                prim = pools[vi][ri][0]
                rid = srv.submit(ids[vi], prim, hold=True)
                pending[rid] = k
                t_sub[k] = start + arrivals[k]
                rays_total += len(prim)
                k += 1
            for rid in list(pending):
                done, _ = srv.poll(rid)
                if done:
                    j = pending.pop(rid)
                    srv.release(rid)
                    vi, ri, bounce = plan[j]
                    if bounce and len(pools[vi][ri][1]):
                        b = pools[vi][ri][1]
                        follow[srv.submit(ids[vi], b, hold=True)] = j
                        rays_total += len(b)
                    else:
                        lat[j] = (time.perf_counter() - t_sub[j]) * 1e3
            for rid in list(follow):
                done, _ = srv.poll(rid)
                if done:
                    j = follow.pop(rid)
                    srv.release(rid)
                    lat[j] = (time.perf_counter() - t_sub[j]) * 1e3
            if k < nreq and not pending and not follow:
                time.sleep(max(0.0, min(0.0005, arrivals[k] - (time.perf_counter() - start))))
        span = time.perf_counter() - start
        st = srv.stats()
        srv.close()
        L = np.array([lat[j] for j in range(args.serve_warmup, nreq)])
        return {"p50_ms": round(float(np.percentile(L, 50)), 3), "p99_ms": round(float(np.percentile(L, 99)), 3),
                "mean_ms": round(float(L.mean()), 3), "mrays_s": round(rays_total / span / 1e6, 1),
                "requests_per_s": round(nreq / span, 1), "steps": int(st["steps"]),
                "max_step_requests": int(st["max_step_requests"]), "admission_waits": int(st["admission_waits"]),
                "peak_mib": round(st["peak_bytes"] / 2 ** 20, 1)}

    burst = run(np.zeros(nreq), args.serve_slots, 3)
    sat = burst["requests_per_s"]
    log(f"[bench] served: closed-loop saturation {sat:.0f} requests/s, {burst['mrays_s']} Mrays/s")
    levels = {}
    arrivals = {}
    for frac in (0.5, 0.8, 0.95):
        gaps = rng.exponential(1.0 / (frac * sat), size=nreq)
        arrivals[frac] = np.cumsum(gaps) - gaps[0]
        levels[str(frac)] = run(arrivals[frac], args.serve_slots, 3)
        log(f"[bench] served @ {frac:.2f} S: p50 {levels[str(frac)]['p50_ms']} ms, p99 {levels[str(frac)]['p99_ms']} ms, "
            f"{levels[str(frac)]['mrays_s']} Mrays/s")
    fifo = run(arrivals[0.8], 1, 1)  # the same arrival trace as the 0.8 S level
    log(f"[bench] served FIFO one-at-a-time @ 0.80 S: p50 {fifo['p50_ms']} ms, p99 {fifo['p99_ms']} ms, "
        f"{fifo['mrays_s']} Mrays/s")
    for v in vols:
        v.close()
    return {"volumes": len(vols), "saturation_requests_per_s": sat, "closed_loop": burst, "poisson": levels,
            "fifo_at_0.8": fifo, "budget_mib": args.serve_budget, "slots": args.serve_slots,
            "requests_per_level": args.serve_requests, "warmup_requests_per_level": args.serve_warmup}


def host_cpu():
    """CPU model, logical CPU count and the CPUs this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def start_oracle_build(C):
    """Build the oracle's volume of the headline format in a background thread (the oracle's
    build is a long single-threaded host computation; ctypes releases the GIL while it runs,
    so the GPU legs proceed meanwhile). Returns a function that waits and yields
    (volume, build seconds)."""
    import threading
    import oracle
    cfg = C.SURF2048
    box = {}

    def work():
        t0 = time.time()
        box["vol"] = oracle.Volume(cfg["specs"][0], C.scene(cfg))
        box["s"] = time.time() - t0

    th = threading.Thread(target=work, daemon=True)
    th.start()

    def wait():
        th.join()
        return box["vol"], box["s"]
    return wait


def cpu_baseline(wait_oracle, rays):
    """The oracle, as it stands, on the headline workload: the same format and the same bounce
    rays, every usable host core (the oracle's static thread split), median of three runs;
    one core on every 8th ray, scaled. The build is not timed."""
    ov, build_s = wait_oracle()
    model, nproc, usable = host_cpu()
    t_all = []
    for _ in range(3):
        t0 = time.perf_counter()
        ov.trace(rays, nthreads=usable)
        t_all.append(time.perf_counter() - t0)
    one = rays[::8]
    t_one = []
    for _ in range(3):
        t0 = time.perf_counter()
        ov.trace(one, nthreads=1)
        t_one.append(time.perf_counter() - t0)
    v_all = len(rays) / float(np.median(t_all)) / 1e6
    v_one = len(one) / float(np.median(t_one)) / 1e6
    log(f"[bench] oracle on {usable} of {nproc} host CPUs ({model}): {v_all:.3f} Mrays/s; one core {v_one:.3f}; "
        f"oracle build {build_s:.0f} s (not timed)")
    return {"value": round(v_all, 4), "unit": "Mrays/s", "cores": usable, "kind": "oracle",
            "value_1core": round(v_one, 4), "nproc": nproc, "cpu_model": model,
            "sample": f"all {len(rays)} bounce rays of the headline frame (one core: every 8th ray), oracle built in "
                      f"the same format (build {build_s:.0f} s, not timed); median of 3 runs; static thread split"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--sample", type=int, default=16384, help="rays per view for the byte model")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-2048", action="store_true", help="skip the 2048^3 leg (both formats, 8 frames)")
    ap.add_argument("--no-512", action="store_true", help="skip the 512^3 leg")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (one lane per ray)")
    ap.add_argument("--retune", action="store_true",
                    help="autotune the headline and the 512^3 formats even when a schedule file is present")
    ap.add_argument("--schedules", default=SCHEDULES_512,
                    help="per-format 512^3 schedules (a bench JSON line; default: the committed autotuner results)")
    ap.add_argument("--untuned", action="store_true", help="also time the 512^3 formats with the plain schedule")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (PMC calibration of FETCH/WRITE_SIZE)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-df", action="store_true", help="skip the distance-field format leg")
    ap.add_argument("--no-build", action="store_true", help="skip the construction (host vs device) leg")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-budget", type=int, default=4096, help="server memory budget, MiB")
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--only", choices=["headline", "small", "surface512", "surface2048", "bounce2048", "batched",
                                       "served", "df", "sweep", "sweep-paper", "build", "restart"],
                    default=None,
                    help="run one workload only (for profiling); prints no bench line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; sharding over several GPUs is designed, not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        x = torch.ones(256 << 20, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4, "copies": 3}))
        return
    import paper_2410_14128_amd as H
    import workloads as W
    from workloads import configs as C

    assert torch.cuda.is_available(), "bench needs a HIP device"
    H.lib()
    torch.cuda.set_device(0)
    if args.only == "surface2048":
        run_surface2048(args, torch, H, W, C)
        return
    if args.only == "bounce2048":
        run_bounce2048(args, torch, H, W, C)
        return
    if args.only == "sweep":
        print(json.dumps({"format_sweep": run_sweep(args, torch, H, W, C)}))
        return
    if args.only == "sweep-paper":
        print(json.dumps({"format_sweep_layouts": run_sweep_paper(args, torch, H, W, C)}))
        return
    if args.only == "batched":
        run_batched(args, torch, H, W, C)
        return
    if args.only == "restart":
        print(json.dumps({"restart_sv": run_restart(args, torch, H, W, C)}))
        return
    if args.only == "build":
        print(json.dumps({"construction": run_construction(args, torch, H, C)}))
        return
    if args.only == "served":
        print(json.dumps(run_served(args, torch, H, W, C)))
        return
    if args.only == "headline":
        run_headline(args, torch, H, W, C)
        return
    if args.only == "small":
        print(json.dumps({"small_64": run_small(args, torch, H, W, C)}))
        return
    if args.only in ("surface512", "df"):
        res = run_surface512(args, torch, H, W, C)
        if args.only == "df":
            run_df512(args, torch, H, C, res)
        return
    wait_oracle = None if args.no_cpu_baseline else start_oracle_build(C)
    head = run_headline(args, torch, H, W, C)
    small = run_small(args, torch, H, W, C)
    res = None if args.no_512 else run_surface512(args, torch, H, W, C)
    df = None if (args.no_df or res is None) else run_df512(args, torch, H, C, res)
    extra = None if args.no_2048 else run_surface2048(args, torch, H, W, C)
    batched = None if args.no_batched else run_batched(args, torch, H, W, C)
    served = None if args.no_served else run_served(args, torch, H, W, C)
    construction = None if args.no_build else run_construction(args, torch, H, C, formats_2048=C.BUILD_2048)
    cpu = None if wait_oracle is None else cpu_baseline(wait_oracle, head["bounce"])
    s512 = None
    if res is not None:
        s512 = {"mrays_s": round(res["value"], 2), "ms_per_step": round(res["ms"], 3),
                "rays_per_step": res["rays_per_step"], "occupancy": round(res["occupancy"], 5),
                "schedules": res["schedules"], "roofline": res["roofline"], "per_format": res["per_format"]}
    line = {
        "metric": "Mrays/s (primary & incoherent) per format; % HBM roofline; p50/p99 ms served",
        "value": round(head["value"], 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(head["ms"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded SDF shell scenes, seeded pinhole cameras, "
                                                      "seeded cosine-weighted bounces)",
        "config": {"workload": "surface-2048 incoherent: the bounce rays of one 1920x1080 frame (one cosine-weighted "
                               "bounce per primary hit) of the 2048^3 shell of 96 spheres + 32 tori, traced through "
                               "G(7) R(4,4,4) --whole-level-dedup in one call",
                   "rays_per_step": head["rays"], "format": head["format"], "format_bytes": head["format_bytes"],
                   "occupancy": round(head["occupancy"], 5), "schedule": head["schedule"],
                   "schedule_source": head["schedule_source"]},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "identical_to_plain_schedule": head["identical_to_plain"],
        "small_64": small,
        "surface_512": s512,
        "surface_2048": extra,
        "distance_field_512": df,
        "batched": batched,
        "served": served,
        "construction": construction,
        "kernel_hash": kernel_source_hash(),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()

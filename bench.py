"""Benchmark of the per-frame GI pass on one MI355X.

One step = one frame of the whole pass (gi_spawn_probes -> gi_trace_probes -> gi_cache_update
(update, gather, SH) -> gi_interpolate_probes, plus the moving light's upload) on the 1080p
field workload: 1920x1080 G-buffer over a seeded ~1.0M-triangle scene, 32,400 probes x 64
rays, 2^20 world-cache slots, a camera orbit and one light on a circle.  G-buffers of every
frame are rendered into HBM before the timed region (the paper rasterises them; they are an
input of the pass).

Prints one JSON line: ms/frame (value), probe Mrays/s, per-kernel times, the roofline of the
dominant kernel and the CPU oracle's time on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
NODE_BYTES, TRI_BYTES = 128, 48
# fp32 ALU operations of the traversal tests (adds, multiplies, min/max, compares, one divide
# per triangle): 26 per child box of a 4-wide node (12 for the slab distances, 12 for entry and
# exit, 2 compares), 53 per watertight triangle test (9 translations, 12 for the shear, 9 for
# the edge functions, 9 sign and zero tests, 3 for the determinant, 8 for the scaled distance,
# the divide and 2 range compares)
NODE_OPS, TRI_OPS = 104, 53
# one fp32 operation per lane per cycle without packed or fused forms: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz (the 157.3 TFLOP/s vector peak counts a packed FMA as 4)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
ALU_BOUND = ("trace_probes", "shade_hits")


def _traffic(kernel, workload, form):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this workload and
    form, if it was taken on the current kernel sources; else None"""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{form}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    k = d.get("kernels", {}).get(kernel)
    from paper_2310_19855_amd import pmc
    if not k or k.get("src_hash") is None or k.get("src_hash") != pmc.kernel_src_hash(kernel):
        return None
    return k.get("bytes_per_launch")


# Table 1 of the paper splits a frame into three columns; each kernel of the pass falls in one
# (the paper's passes to columns, Section 5): probe rays are "raytracing"; spawn, the world
# cache's insert / light sample / shadow ray / update and the probe gather are "caching &
# sampling"; SH projection (fused into the gather here), interpolation and filtering are
# "interpolate & denoise".  The learned surrogate is not in the paper: its own column.
TABLE1 = {"trace_probes": "raytracing",
          "spawn": "caching_sampling", "mask_mip": "caching_sampling", "shade_hits": "caching_sampling",
          "cache_update": "caching_sampling", "cache_update_tiles": "caching_sampling",
          "gather_sh": "caching_sampling", "reproject": "caching_sampling", "reconstruct": "caching_sampling",
          "lg_box": "caching_sampling", "lg_box_final": "caching_sampling", "light_grid": "caching_sampling",
          "restir_clear": "caching_sampling", "restir_store": "caching_sampling",
          "interpolate": "interpolate_denoise", "filter_x": "interpolate_denoise", "filter_y": "interpolate_denoise"}


def table1_buckets(kern, frames):
    """ms per frame per Table-1 column from per-kernel totals"""
    out = {"raytracing": 0.0, "caching_sampling": 0.0, "interpolate_denoise": 0.0, "learned": 0.0, "other": 0.0}
    for name, v in kern.items():
        b = TABLE1.get(name, "learned" if name.startswith(("learned_", "mlp_", "train", "infer", "adam", "judge",
                                                             "select", "sort")) else "other")
        out[b] += v["avg_ms"] * v["launches"] / max(frames, 1)
    return {k: round(v, 5) for k, v in out.items() if v or k != "other"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=55)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="field1080")
    ap.add_argument("--profile-frames", type=int, default=5)
    ap.add_argument("--cpu-frames", type=int, default=40,
                    help="oracle frames timed for cpu_baseline (about 0.2 s each on 16 host threads)")
    ap.add_argument("--cpu-single-frames", type=int, default=2, help="oracle frames timed on one host thread")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", metavar="PATH", default=None,
                    help="after the headline line, run the optional sweeps (cache forms, 4K, furnace, probe "
                         "filter, temporal reuse, light sampling) and write them as JSON to PATH")
    ap.add_argument("--equal-error", metavar="PATH", default=None,
                    help="after the headline line, run the equal-error protocol (field sequence of 60 frames, "
                         "evaluation frames 0, 29, 59, R in 8..128, plain / MLP-BF16 / MLP-FP8) and write it to PATH")
    ap.add_argument("--form", default="plain", choices=("plain", "mlp_bf16", "mlp_fp8"),
                    help="cache form of the timed frames (learned forms train and infer every frame)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (scale of HBM byte counters)")
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))
    line = headline(args, log)
    print(json.dumps(line), flush=True)
    if args.equal_error:
        res = equal_error_protocol(log)
        with open(args.equal_error, "w") as fh:
            json.dump(res, fh, indent=1)
        log(f"[bench] equal-error protocol written to {args.equal_error}")
    if args.forms:
        forms = optional_sweeps(log)
        with open(args.forms, "w") as fh:
            json.dump(forms, fh, indent=1)
        log(f"[bench] optional sweeps written to {args.forms}")


def optional_sweeps(log):
    import torch
    torch.cuda.empty_cache()
    forms = forms_comparison(log)
    forms.update(field4k_and_furnace(log))
    forms["probe_filter"] = probe_filter_measure(log)
    forms["temporal_reuse"] = temporal_measure(log)
    forms["temporal_upscale_2x2"] = temporal_measure(log, upscale=2, with_cpu=False)
    forms["temporal_upscale_2x2_guided"] = temporal_measure(log, upscale=2, ray_guiding=1, with_cpu=False)
    forms["temporal_quality"] = temporal_quality(log)
    forms["light_sampling"] = light_sampling_measure(log)
    return forms


def headline(args, log):
    """The timed frames of the workload, per-kernel times, the roofline of the dominant kernel
    and the CPU oracle on a bounded sample of the same workload: the benchmark's one line."""
    import numpy as np  # noqa: F401
    import torch

    from paper_2310_19855_amd import gi
    from paper_2310_19855_amd import inputs as I

    preset = dict(I.PRESETS[args.workload])
    W, H, R = preset["width"], preset["height"], preset["rays_per_probe"]
    scene = I.make_scene(preset["scene"])
    cfg = dict(width=W, height=H, rays_per_probe=R, table_log2=preset["table_log2"],
               bounces=preset["bounces"], sky=scene.sky, cache_mode=FORMS[args.form])
    if args.form != "plain":
        cfg.update(MLP_CFG)
    torch.cuda.set_device(0)
    ctx = gi.Context(**cfg)
    t0 = time.time()
    ctx.build_bvh(scene)
    t_bvh = time.time() - t0
    dims = ctx.dims()
    log(f"[bench] scene {scene.name}: {scene.n_tris} tris, BVH {int(dims[9])} nodes depth {int(dims[10])} "
        f"built in {t_bvh:.2f}s")

    n_frames = args.warmup + args.steps
    n_gb = max(n_frames, args.profile_frames)
    cams = [I.camera_for(scene.name, f) for f in range(n_gb)]
    for f, c in enumerate(cams):
        c.index = f
    gbs = []
    for f in range(n_gb):
        if scene.dynamic is not None:
            tv, m = scene.dynamic(f)
            ctx.set_dynamic(tv, m)
        g = gi.GBuffer(H, W)
        ctx.render_gbuffer(cams[f], g.pos, g.nrm, g.alb, g.prim)
        gbs.append(g)
    torch.cuda.synchronize()
    dyn = [scene.dynamic(f) if scene.dynamic is not None else None for f in range(n_gb)]
    out = torch.zeros((H, W, 4), dtype=torch.float32, device="cuda")
    log(f"[bench] {n_gb} G-buffers resident ({n_gb * W * H * 52 / 2**30:.1f} GiB)")

    def frame(f, fi):
        g = gbs[f]
        if dyn[f] is not None:
            ctx.set_dynamic(*dyn[f])
        cam = cams[f]
        cam.index = fi
        ctx.spawn_probes(cam, g.pos, g.nrm, g.prim)
        ctx.trace_probes(cam)
        if args.form != "plain":
            ctx.learned_train(cam)
        ctx.cache_update(cam)
        ctx.interpolate_probes(cam, g.pos, g.nrm, g.prim, out)

    for f in range(args.warmup):
        frame(f, f)
    torch.cuda.synchronize()
    ctx.reset_stats()
    # the traversal kernel's own launches are timed inside the timed frames (two events on its
    # launch stream per frame; the library's events skip the system fence); every other
    # kernel is timed in a separate pass below
    ctx.profile(2)
    ctx.profile_read()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for k in range(args.steps):
        f = args.warmup + k
        frame(f, f)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    live = ctx.profile_read().get("trace_probes")
    ctx.profile(False)
    stats = ctx.stats()
    ms_per_frame = wall * 1e3 / args.steps
    log(f"[bench] {args.steps} frames: {ms_per_frame:.3f} ms/frame wall, {gpu_ms / args.steps:.3f} ms/frame events")
    if stats["wraps"]:
        raise RuntimeError(f"{stats['wraps']} fixed-point cell sums wrapped: the cached averages are corrupt")

    # per-kernel device times (HIP events on the launch stream), separate pass over frames
    # already seen (the cache is warm, as in the timed frames)
    ctx.profile(True)
    ctx.profile_read()
    for k in range(args.profile_frames):
        f = k % n_gb
        frame(f, n_frames + k)
    prof = ctx.profile_read()
    ctx.profile(False)
    trav = ctx.measure_traversal()
    kern = {name: dict(launches=c, avg_ms=ms / max(c, 1)) for name, (c, ms) in prof.items()}

    rays_per_frame = stats["rays"] / args.steps
    hits_per_frame = stats["hits"] / args.steps
    # the traversal's launch time from the timed frames themselves (the separate pass's value
    # stays in "kernels")
    live_ms = live[1] / live[0] if live and live[0] else None
    trace_ms = live_ms if live_ms else kern.get("trace_probes", {}).get("avg_ms", float("nan"))
    mrays = rays_per_frame / (trace_ms * 1e-3) / 1e6 if trace_ms == trace_ms else None
    total_rays = (stats["rays"] + stats["shadow"] + stats["bounce"]) / args.steps
    frame_ms_events = gpu_ms / args.steps

    # algorithmic bytes per launch (the traffic the method must move), per kernel
    P = int(dims[0])
    N = int(dims[2])
    pr_rays = max(trav["probe_rays"], 1)
    alg = {
        "trace_probes": trav["probe_nodes"] * NODE_BYTES + trav["probe_tris"] * TRI_BYTES
        + 16 * trav["probe_rays"] + 32 * P,
        "shade_hits": trav["shadow_nodes"] * NODE_BYTES + trav["shadow_tris"] * TRI_BYTES
        + hits_per_frame * (128 + 16 + 4 + 32 + 8 + 32),
        "cache_update": 4 * N + 96 * stats["live"],
        "gather_sh": rays_per_frame * 32 + P * (64 * 16 + 112 + 16),
        "interpolate": W * H * (52 + 16) + P * 144,
    }
    if args.form in ("mlp_bf16", "mlp_fp8"):
        # one optimiser step's gradient sort: 8 corner pairs per level and sample, each pass of
        # the 8-bit LSD sort reads the 4-B key for its histogram, then reads and writes the
        # 12-B pair
        n_pairs = (1 << MLP_CFG["mlp_batch_log2"]) * MLP_CFG["mlp_levels"] * 8
        key_bits = (MLP_CFG["mlp_levels"] - 1).bit_length() + MLP_CFG["mlp_table_log2"]
        alg["learned_grad_sort"] = n_pairs * 28 * ((key_bits + 7) // 8)
    total_ms = sum(v["avg_ms"] * v["launches"] for v in kern.values()) / max(args.profile_frames, 1)
    # the dominant kernel among those with algorithmic bytes (stages such as the learned
    # training, a mix of gathers and matrix work, have none)
    dom = max(((k, v) for k, v in kern.items() if k in alg),
              key=lambda kv: kv[1]["avg_ms"] * kv[1]["launches"])[0]
    for name, v in kern.items():
        if name in alg:
            v["alg_bytes"] = int(alg[name])
            v["gbs"] = alg[name] / (v["avg_ms"] * 1e-3) / 1e9
            v["frac_hbm"] = v["gbs"] / HBM_PEAK_GBS
        v["share"] = v["avg_ms"] * v["launches"] / max(args.profile_frames, 1) / total_ms if total_ms else None
    # the traversal's arithmetic view beside its HBM view: the fp32 operations of the tests
    # the walk runs against the VALU issue peak (its node and triangle bytes come mostly from
    # L2 and the Infinity Cache, so the byte roofline is an upper bound on what it could take)
    alg_ops = {"trace_probes": trav["probe_nodes"] * NODE_OPS + trav["probe_tris"] * TRI_OPS,
               "shade_hits": trav["shadow_nodes"] * NODE_OPS + trav["shadow_tris"] * TRI_OPS}
    for name, v in kern.items():
        if name in alg_ops:
            v["alg_ops"] = int(alg_ops[name])
            v["tops"] = alg_ops[name] / (v["avg_ms"] * 1e-3) / 1e12
            v["frac_alu"] = v["tops"] / VALU_PEAK_TOPS
    dk = dict(kern[dom])
    if dom == "trace_probes" and live_ms:
        dk["avg_ms"] = live_ms
        dk["gbs"] = alg[dom] / (live_ms * 1e-3) / 1e9
        dk["frac_hbm"] = dk["gbs"] / HBM_PEAK_GBS
        dk["tops"] = alg_ops[dom] / (live_ms * 1e-3) / 1e12
        dk["frac_alu"] = dk["tops"] / VALU_PEAK_TOPS
    traffic = _traffic(dom, args.workload, args.form)
    roofline = {"kernel": dom, "bound": "hbm", "achieved": round(dk.get("gbs", 0.0), 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(dk.get("frac_hbm", 0.0), 5), "traffic": traffic,
                "alg_bytes_per_launch": dk.get("alg_bytes"), "avg_launch_ms": round(dk["avg_ms"], 5),
                "timing": ("HIP events on the launch stream around each of the timed frames' launches"
                           if dom == "trace_probes" and live_ms else
                           "HIP events on the launch stream, separate pass over warm frames")}
    if traffic:
        roofline["dram_frac_of_alg_bytes"] = round(traffic / max(dk.get("alg_bytes", 1), 1), 4)
    if dom in alg_ops:
        roofline["alu_view"] = {"alg_ops_per_launch": dk["alg_ops"], "achieved": round(dk["tops"], 3),
                                "peak": round(VALU_PEAK_TOPS, 2), "unit": "T fp32 op/s",
                                "frac": round(dk["frac_alu"], 5)}
    if dom in ("trace_probes", "shade_hits"):
        roofline.update({"bytes_per_probe_ray": round((trav["probe_nodes"] * NODE_BYTES
                                                       + trav["probe_tris"] * TRI_BYTES) / pr_rays, 1),
                         "nodes_per_probe_ray": round(trav["probe_nodes"] / pr_rays, 3),
                         "tris_per_probe_ray": round(trav["probe_tris"] / pr_rays, 3)})
    log(f"[bench] kernels: " + ", ".join(f"{k} {v['avg_ms']:.3f}ms x{v['launches'] // max(args.profile_frames, 1)}"
                                         for k, v in sorted(kern.items(), key=lambda kv: -kv[1]['avg_ms'] * kv[1]['launches'])))
    buckets = table1_buckets(kern, args.profile_frames)
    log(f"[bench] Table-1 columns (ms/frame): {buckets}")

    cpu = None
    if not args.no_cpu_baseline and args.form == "plain":
        del gbs
        torch.cuda.empty_cache()
        cpu = cpu_baseline(scene, cfg, args.cpu_frames, log, single_frames=args.cpu_single_frames)

    return {
        "metric": "GI ms/frame & probe Mrays/s at 1080p; plain vs MLP cache at fixed rel. error",
        "value": round(ms_per_frame, 4), "unit": "ms/frame", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_frame, 4), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+u32",
        "data": "synthetic (seeded procedural scene, camera orbit, moving light)",
        "config": {"workload": f"{args.workload}: {W}x{H} G-buffer, {scene.n_tris} tris ({scene.name}), "
                               f"{P} probe tiles x {R} rays, 2^{preset['table_log2']} cache slots, "
                               f"{preset['bounces']} bounce(s), frames {args.warmup}..{n_frames - 1}",
                   "cache": args.form},
        "probe_mrays_per_s": round(mrays, 1) if mrays else None,
        "total_mrays_per_s": round(total_rays / (frame_ms_events * 1e-3) / 1e6, 1),
        "probe_rays_per_frame": int(rays_per_frame), "hits_per_frame": int(hits_per_frame),
        "shadow_rays_per_frame": int(stats["shadow"] / args.steps),
        "gpu_event_ms_per_frame": round(frame_ms_events, 4),
        "table1_ms_per_frame": buckets,
        "fixed_point_wraps": int(stats["wraps"]), "overflow_drops": int(stats["overflow"]),
        "bvh_build_s": round(t_bvh, 2),
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }


FORMS = {"plain": 0, "plain_lod": 0, "plain_tiles": 0, "plain_lod_tiles": 0, "mlp_bf16": 1, "mlp_fp8": 2}
# two-level cache forms: 2^16 tiles of 64 cells, queries from the finest level with 16 samples
TILES_CFG = dict(cache_tiles=1, table_log2=16, tile_min_samples=16)
MLP_CFG = dict(mlp_batch_log2=14, mlp_levels=16, mlp_table_log2=19, mlp_steps=4, mlp_lr_grid=1e-2,
               mlp_lr_mlp=1e-2, mlp_judge=0.5)
SWEEP_R = (8, 16, 32, 64, 128)
SWEEP_FRAMES, SWEEP_TIMED_FROM = 16, 8


def run_form(scene_name, scene, W, H, R, form, frames, timed_from, points=None, profile=False, extra=None,
             want_out=False):
    """Frames of the pass with the camera and lights frozen at frame 0 (the reference's frame
    state).  Returns GPU ms per timed frame, per-kernel ms, learned stats and, with points
    (pos, nrm device tensors), the plain cache's lookups and the form's radiance there; with
    want_out the last frame's irradiance image (rgb, flag)."""
    import torch

    from paper_2310_19855_amd import gi
    from paper_2310_19855_amd import inputs as I
    cfg = dict(width=W, height=H, rays_per_probe=R, table_log2=20, sky=scene.sky, cache_mode=FORMS[form])
    if form in ("mlp_bf16", "mlp_fp8"):
        cfg.update(MLP_CFG)
    if form in ("plain_lod", "plain_lod_tiles"):
        # levels of detail that follow Algorithm 6's adaptive cell size of this view
        fov = I.camera_for(scene_name, 0).fov_y
        cfg["lod_scale"] = math.tan(fov * 8.0 * max(1.0 / H, H / (W * W)))
    if form in ("plain_tiles", "plain_lod_tiles"):
        cfg.update(TILES_CFG)
    cfg.update(extra or {})
    ctx = gi.Context(**cfg)
    ctx.build_bvh(scene)
    if scene.dynamic is not None:
        ctx.set_dynamic(*scene.dynamic(0))
    gb = gi.GBuffer(H, W)
    out = torch.zeros((H, W, 4), dtype=torch.float32, device="cuda")
    ctx.render_gbuffer(I.camera_for(scene_name, 0), gb.pos, gb.nrm, gb.alb, gb.prim)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    for f in range(frames):
        if f == timed_from:
            torch.cuda.synchronize()
            if profile:
                ctx.profile(True)
                ctx.profile_read()
            ev0.record()
        cam = I.camera_for(scene_name, 0)
        cam.index = f
        ctx.spawn_probes(cam, gb.pos, gb.nrm, gb.prim)
        ctx.trace_probes(cam)
        if form in ("mlp_bf16", "mlp_fp8"):
            ctx.learned_train(cam)
        ctx.cache_update(cam)
        ctx.interpolate_probes(cam, gb.pos, gb.nrm, gb.prim, out)
    ev1.record()
    torch.cuda.synchronize()
    n = max(frames - timed_from, 1)
    ms = ev0.elapsed_time(ev1) / n
    kern = {}
    if profile:
        prof = ctx.profile_read()
        ctx.profile(False)
        kern = {k: round(v[1] / n, 4) for k, v in prof.items()}
    learned = form in ("mlp_bf16", "mlp_fp8")
    res = {"ms": ms, "kernels": kern, "learned": ctx.learned_stats() if learned else None}
    if want_out:
        res["out"] = out.cpu().numpy()
    if points is not None:
        pp, pn = points
        q = torch.zeros((pp.shape[0], 4), dtype=torch.float32, device="cuda")
        ctx.cache_query(pp, pn, q)
        res["plain_at_points"] = q.cpu().numpy()
        if learned:
            ctx.learned_query(pp, pn, q)
            res["form_at_points"] = q.cpu().numpy()
        else:
            res["form_at_points"] = res["plain_at_points"]
        torch.cuda.synchronize()
    ctx.close()
    return res


EE_FORMS = ("plain", "mlp_bf16", "mlp_fp8")
EE_FRAMES, EE_EVAL = 60, (0, 29, 59)
EE_CAPS = (4, 16, 64)


def _point_reference(frame):
    """the float64 point reference of a frame of the field sequence (its camera and lights
    frozen): seeded visible surface points of its 480x270 view and the converged radiance there"""
    import numpy as np
    g = os.path.join(ROOT, "tests", "golden")
    path = os.path.join(g, f"field480x270_f{frame}_points.npz")
    if frame == 0 and not os.path.exists(path):
        path = os.path.join(g, "field480x270_reference.npz")
    if not os.path.exists(path):
        return None
    return np.load(path)


def equal_error_protocol(log, W=1920, H=1080, frames=EE_FRAMES, eval_frames=EE_EVAL, sweep_R=SWEEP_R,
                         timed_from=5):
    """The equal-error comparison on the benchmark workload's own sequence: the 1920x1080 field
    with its orbiting camera and moving light, 60 frames, for each cache form (plain, MLP with
    BF16 inference, MLP with FP8 e4m3 inference) and each rays-per-probe R.  At the evaluation
    frames 0, 29 and 59 the cache's radiance (the plain cell, or the surrogate) is compared with
    the float64 oracle's converged radiance at that frame's reference points (relMAE over the
    points whose cell the plain cache holds); ms/frame is the GPU time of the pass (spawn to
    interpolation, learned training and inference included) over frames 5..59, from HIP events
    around each frame.  Beside it, the per-pixel reading: the irradiance image of a 480x270 run
    with the frame-0 camera and lights frozen (16 frames) against the oracle's converged
    irradiance image of that view (relMAE over pixels with a probe on both sides)."""
    import numpy as np
    import torch

    from paper_2310_19855_amd import gi
    from paper_2310_19855_amd import inputs as I
    refs = {f: _point_reference(f) for f in eval_frames}
    missing = [f for f, r in refs.items() if r is None]
    if missing:
        return {"error": f"no point reference for frames {missing} (python -m oracle.make_reference --scene field "
                         f"--frame F --points-only)"}
    scene = I.make_scene("field")
    pts = {f: (torch.from_numpy(r["point_pos"]).cuda(), torch.from_numpy(r["point_nrm"]).cuda(),
               r["point_L"].astype(np.float64)) for f, r in refs.items()}
    out = {"protocol": f"field {W}x{H}, frames 0..{frames - 1} (orbit camera, moving light), evaluation frames "
                       f"{list(eval_frames)}; relMAE of the cache radiance at each evaluation frame's seeded surface "
                       f"points vs the float64 oracle's converged radiance there (light and camera of that frame), "
                       f"over the points whose cell the plain cache holds; ms/frame over frames {timed_from}.."
                       f"{frames - 1}", "mlp": dict(MLP_CFG), "sweep": {}}
    def run(form, R, extra=None):
        cfg = dict(width=W, height=H, rays_per_probe=R, table_log2=20, sky=scene.sky, cache_mode=FORMS[form])
        if form != "plain":
            cfg.update(MLP_CFG)
        cfg.update(extra or {})
        ctx = gi.Context(**cfg)
        ctx.build_bvh(scene)
        gb = gi.GBuffer(H, W)
        o = torch.zeros((H, W, 4), dtype=torch.float32, device="cuda")
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        ms, errs = [], {}
        for f in range(frames):
            cam = I.camera_for("field", f)
            cam.index = f
            ctx.set_dynamic(*scene.dynamic(f))
            ctx.render_gbuffer(cam, gb.pos, gb.nrm, gb.alb, gb.prim)
            e0.record()
            ctx.spawn_probes(cam, gb.pos, gb.nrm, gb.prim)
            ctx.trace_probes(cam)
            if form != "plain":
                ctx.learned_train(cam)
            ctx.cache_update(cam)
            ctx.interpolate_probes(cam, gb.pos, gb.nrm, gb.prim, o)
            e1.record()
            torch.cuda.synchronize()
            if f >= timed_from:
                ms.append(e0.elapsed_time(e1))
            if f in pts:
                pp, pn, Lr = pts[f]
                q = torch.zeros((pp.shape[0], 4), dtype=torch.float32, device="cuda")
                ctx.cache_query(pp, pn, q)
                plain_q = q.cpu().numpy()
                if form != "plain":
                    ctx.learned_query(pp, pn, q)
                val = q.cpu().numpy()
                found = plain_q[:, 3] > 0
                L = val[found, :3].astype(np.float64)
                errs[f] = {"relMAE": round(float(np.abs(L - Lr[found]).sum() / max(np.abs(Lr[found]).sum(), 1e-30)), 5),
                           "points": int(found.sum())}
        ctx.close()
        row = {"ms_per_frame": round(float(np.mean(ms)), 4), "eval": errs,
               "max_relMAE": max(v["relMAE"] for v in errs.values())}
        log(f"[bench] equal error {form} R={R} {extra or ''}: {row['ms_per_frame']:.3f} ms/frame, relMAE "
            + ", ".join(f"f{f} {v['relMAE']:.3f}" for f, v in errs.items()))
        return row

    for form in EE_FORMS:
        out["sweep"][form] = {R: run(form, R) for R in sweep_R}
    # the plain cache's history cap (samples in its moving average): with a moving light a long
    # history averages the radiance of the light's earlier positions
    out["plain_history_cap"] = {f"R{R}_cap{cap}": run("plain", R, {"n_cap": cap})
                                for R in (64, 128) for cap in EE_CAPS}

    def cheapest(form, level):
        ok = [(v["ms_per_frame"], R) for R, v in out["sweep"][form].items() if v["max_relMAE"] <= level]
        if not ok:
            return None
        m, R = min(ok)
        return {"rays_per_probe": R, "ms_per_frame": m, "max_relMAE": out["sweep"][form][R]["max_relMAE"]}
    out["equal_error_5pct"] = {f: cheapest(f, 0.05) for f in EE_FORMS}
    common = max(min(v["max_relMAE"] for v in out["sweep"][f].values()) for f in EE_FORMS)
    out["equal_error_common"] = {"level": round(common, 5), **{f: cheapest(f, common) for f in EE_FORMS}}
    out["nominal_R64"] = {f: out["sweep"][f].get(64) for f in EE_FORMS}
    # per-pixel reading at frame 0 (480x270, the converged irradiance image of the frozen view)
    ref = np.load(os.path.join(ROOT, "tests", "golden", "field480x270_reference.npz"))
    w, h = int(ref["width"]), int(ref["height"])
    pix = {}
    for form in EE_FORMS:
        r = run_form("field", scene, w, h, 64, form, SWEEP_FRAMES, SWEEP_TIMED_FROM, want_out=True)
        img = r["out"]
        ok = (img[..., 3] == 0) & (ref["flag"] == 0)
        E = img[ok][:, :3].astype(np.float64)
        Er = ref["irradiance"][ok].astype(np.float64)
        pix[form] = {"relMAE": round(float(np.abs(E - Er).sum() / max(np.abs(Er).sum(), 1e-30)), 5),
                     "pixels": int(ok.sum())}
    out["per_pixel_frame0_480x270_R64"] = pix
    log(f"[bench] equal error at 5%: {out['equal_error_5pct']}; common level {out['equal_error_common']}; "
        f"per-pixel {pix}")
    return out


def forms_comparison(log, W=1920, H=1080):
    """Plain vs learned cache forms at equal relative radiance error.  For each scene with a
    stored float64 reference (the oracle converged at seeded visible surface points), each
    form and each rays-per-probe R: 16 frames with the frame-0 camera and lights, GPU time of
    frames 8..15, then the relative mean absolute error of the form's radiance at the points
    whose cell the plain cache holds at that R.  Reported: the cheapest R (and its ms/frame)
    with error <= 5% per form, and at the lowest error level every form reaches."""
    import numpy as np
    import torch

    from paper_2310_19855_amd import inputs as I
    out = {"protocol": f"{W}x{H}, frames 0..{SWEEP_FRAMES - 1} with the frame-0 camera and lights, "
                       f"ms/frame over frames {SWEEP_TIMED_FROM}..{SWEEP_FRAMES - 1}; relMAE of the cache "
                       "radiance at seeded visible surface points vs the float64 oracle's converged NEE "
                       "radiance there, over the points whose cell the plain cache holds",
           "mlp": dict(MLP_CFG), "scenes": {}}
    for scene_name in ("room", "field"):
        path = os.path.join(ROOT, "tests", "golden", f"{scene_name}480x270_reference.npz")
        if not os.path.exists(path):
            continue
        ref = np.load(path)
        scene = I.make_scene(scene_name)
        pts = (torch.from_numpy(ref["point_pos"]).cuda(), torch.from_numpy(ref["point_nrm"]).cuda())
        Lr = ref["point_L"].astype(np.float64)
        table = {}
        for form in FORMS:
            table[form] = {}
            for R in SWEEP_R:
                r = run_form(scene_name, scene, W, H, R, form, SWEEP_FRAMES, SWEEP_TIMED_FROM, points=pts,
                             profile=(R == 64))
                found = r["plain_at_points"][:, 3] > 0
                L = r["form_at_points"][found, :3].astype(np.float64)
                e = float(np.abs(L - Lr[found]).sum() / max(np.abs(Lr[found]).sum(), 1e-30))
                row = {"ms_per_frame": round(r["ms"], 4), "relMAE": round(e, 5), "points": int(found.sum())}
                if r["kernels"]:
                    row["kernels_ms"] = r["kernels"]
                if r["learned"]:
                    row["loss"] = round(r["learned"]["loss"], 5)
                    row["fallback"] = r["learned"]["fallback"]
                table[form][R] = row
            log(f"[bench] {scene_name} {form}: " + ", ".join(
                f"R={R} {v['relMAE']:.3f} @ {v['ms_per_frame']:.2f}ms" for R, v in table[form].items()))

        def cheapest(form, level):
            ok = [(v["ms_per_frame"], R) for R, v in table[form].items() if v["relMAE"] <= level]
            if not ok:
                return None
            ms, R = min(ok)
            return {"rays_per_probe": R, "ms_per_frame": ms, "relMAE": table[form][R]["relMAE"]}
        common = max(min(v["relMAE"] for v in table[f].values()) for f in FORMS)
        out["scenes"][scene_name] = {
            "sweep": table,
            "reference": f"{len(Lr)} points, {int(ref['point_samples'])} NEE samples each, relative "
                         f"standard error {float(ref['point_se'].sum() / ref['point_L'].sum()):.4f}",
            "equal_error_5pct": {f: cheapest(f, 0.05) for f in FORMS},
            "equal_error_common": {"level": round(common, 5), **{f: cheapest(f, common) for f in FORMS}},
        }
        log(f"[bench] {scene_name} equal error at {common:.3f}: " + ", ".join(
            f"{f} {v['ms_per_frame']:.2f}ms (R={v['rays_per_probe']})"
            for f, v in out["scenes"][scene_name]["equal_error_common"].items() if isinstance(v, dict)))
    return out


def field4k_and_furnace(log, W=3840, H=2160, R=64):
    """The field scene at 3840x2160 with FP8 e4m3 inference beside BF16 and the plain cache:
    ms/frame and the cache radiance's relMAE at the stored float64 point reference (seeded
    world positions, valid at any resolution of the frame-0 view), 16 frozen frames.  Beside
    it the closed furnace (Le = 1, albedo 0.8, two bounces, cache values replaced each frame):
    after frame f every cell holds L_f = albedo (Le + L_{f-1}), L_0 = albedo Le, so a pixel's
    irradiance is pi (Le + L_f); reported per form is the relMAE of the irradiance image of
    the last frame against that value."""
    import numpy as np
    import torch

    from paper_2310_19855_amd import inputs as I
    res = {"field4k": {"protocol": f"{W}x{H}, R={R}, frames 0..{SWEEP_FRAMES - 1} with the frame-0 camera "
                                   f"and lights, ms/frame over frames {SWEEP_TIMED_FROM}..{SWEEP_FRAMES - 1}; "
                                   "relMAE vs the float64 point reference over the points the plain cache holds"},
           "furnace": {}}
    path = os.path.join(ROOT, "tests", "golden", "field480x270_reference.npz")
    if os.path.exists(path):
        ref = np.load(path)
        scene = I.make_scene("field")
        pts = (torch.from_numpy(ref["point_pos"]).cuda(), torch.from_numpy(ref["point_nrm"]).cuda())
        Lr = ref["point_L"].astype(np.float64)
        for form in FORMS:
            r = run_form("field", scene, W, H, R, form, SWEEP_FRAMES, SWEEP_TIMED_FROM, points=pts)
            found = r["plain_at_points"][:, 3] > 0
            L = r["form_at_points"][found, :3].astype(np.float64)
            e = float(np.abs(L - Lr[found]).sum() / max(np.abs(Lr[found]).sum(), 1e-30))
            res["field4k"][form] = {"ms_per_frame": round(r["ms"], 4), "relMAE": round(e, 5),
                                    "points": int(found.sum())}
            log(f"[bench] field {W}x{H} {form}: relMAE {e:.3f} @ {r['ms']:.2f} ms/frame")
        del scene
    fsc = I.make_scene("furnace")
    fp = I.PRESETS["furnace"]
    rho, le, frames = 0.8, 1.0, 42
    L = rho * le
    for _ in range(1, frames):
        L = rho * (le + L)
    E = math.pi * (le + L)
    res["furnace"]["protocol"] = (f"{fp['width']}x{fp['height']}, R={fp['rays_per_probe']}, two bounces, cache "
                                  f"values replaced each frame, {frames} frames; closed-form irradiance {E:.6f} "
                                  f"(limit 5 pi); relMAE of the last frame's irradiance over pixels with a probe")
    for form in FORMS:
        r = run_form("furnace", fsc, fp["width"], fp["height"], fp["rays_per_probe"], form, frames, frames - 8,
                     extra=dict(bounces=2, n_cap=0, cell_scale=0.5, leak_bit=0,
                                # no history (n_cap 0) counts no samples: tiles answer from level 0
                                **({"tile_min_samples": 0} if "tiles" in form else {})),
                     want_out=True)
        o = r["out"]
        ok = o[..., 3] != 2
        e = float(np.abs(o[ok][:, :3].astype(np.float64) - E).sum() / (E * 3 * max(int(ok.sum()), 1)))
        res["furnace"][form] = {"ms_per_frame": round(r["ms"], 4), "relMAE": round(e, 6), "pixels": int(ok.sum())}
        log(f"[bench] furnace {form}: relMAE {e:.2e} @ {r['ms']:.3f} ms/frame")
    return res


def probe_filter_measure(log, scene_name="field", W=1920, H=1080, R=64, with_cpu=True):
    """The probe-space filter of Algorithm 5 on the benchmark workload's view: 16 frames with
    the frame-0 camera and lights, filter on, per-pass launch time (HIP events) and the
    fraction of the HBM peak at its algorithmic bytes: per probe and pass, its atlas read once
    and written once (2 x 1 KiB; neighbours' cells are re-read from L2), plus the SH (112 B) on
    the y pass, plus position and normal (32 B)."""
    from paper_2310_19855_amd import inputs as I
    scene = I.make_scene(scene_name)
    r = run_form(scene_name, scene, W, H, R, "plain", SWEEP_FRAMES, SWEEP_TIMED_FROM, profile=True,
                 extra=dict(probe_filter=1))
    P = ((W + 7) // 8) * ((H + 7) // 8)
    out = {"workload": f"{scene_name} {W}x{H}, R={R}, frozen frame-0 view", "ms_per_frame_with_filter": round(r["ms"], 4)}
    for name, extra in (("filter_x", 0), ("filter_y", 112)):
        ms = r["kernels"].get(name)
        if not ms:
            continue
        b = P * (2 * 1024 + 32 + extra)
        out[name] = {"avg_ms": ms, "alg_bytes": b, "gbs": round(b / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"[bench] probe filter: " + ", ".join(f"{k} {v['avg_ms']:.4f} ms ({v['frac_hbm']:.2f} of HBM peak)"
                                            for k, v in out.items() if isinstance(v, dict)))
    if with_cpu:
        out["cpu_baseline"] = probe_filter_cpu(scene, scene_name, W, H, R)
        log(f"[bench] probe filter, CPU oracle: {out['cpu_baseline']['value']:.1f} ms for both passes")
    return out


def temporal_measure(log, scene_name="field", W=1920, H=1080, R=64, frames=24, timed_from=8, with_cpu=True,
                     upscale=1, ray_guiding=0):
    """Temporal reuse of screen probes (Algorithm 1 reprojection, Algorithm 3 hysteresis) on the
    benchmark workload's moving camera: frames 0..23 of the orbit with the moving light,
    ms/frame over frames 8..23, the reprojection kernel's launch time and its fraction of the
    HBM peak at its algorithmic bytes (per pixel the G-buffer position, normal and primary hit,
    36 B; per tile the winner and history, 8 B; the previous probes come from L2).  With
    upscale 2, temporal upscaling and adaptive sampling (Algorithm 2) on top: probe rays per
    frame and the placement kernels' time.  With ray guiding, the reconstruction kernel against
    the HBM peak at its algorithmic bytes: per probe the previous atlas (1 KiB, each previous
    probe read from HBM once, its other readers hit L2), position and normal (32 B), and the
    written reconstruction and weight sums (1 KiB + 256 B)."""
    import torch

    from paper_2310_19855_amd import gi
    from paper_2310_19855_amd import inputs as I
    scene = I.make_scene(scene_name)
    ctx = gi.Context(width=W, height=H, rays_per_probe=R, table_log2=20, sky=scene.sky, temporal=1,
                     upscale=upscale, ray_guiding=ray_guiding)
    ctx.build_bvh(scene)
    gb = gi.GBuffer(H, W)
    out = torch.zeros((H, W, 4), dtype=torch.float32, device="cuda")
    for f in range(frames):
        cam = I.camera_for(scene_name, f)
        cam.index = f
        if scene.dynamic is not None:
            ctx.set_dynamic(*scene.dynamic(f))
        ctx.render_gbuffer(cam, gb.pos, gb.nrm, gb.alb, gb.prim)
        if f == timed_from:
            torch.cuda.synchronize()
            ctx.profile(True)
            ctx.profile_read()
            rays0 = ctx.stats()["rays"]
        ctx.spawn_probes(cam, gb.pos, gb.nrm, gb.prim)
        ctx.trace_probes(cam)
        ctx.cache_update(cam)
        ctx.interpolate_probes(cam, gb.pos, gb.nrm, gb.prim, out)
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    dn_ms = None
    if upscale == 1 and not ray_guiding:
        # the screen-space denoiser on this workload's last frame, 8 calls (history growing)
        dn = gi.Denoiser(W, H)
        den = torch.zeros_like(out)
        dn(cam, gb.pos, gb.nrm, gb.prim, out, den)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(8):
            dn(cam, gb.pos, gb.nrm, gb.prim, out, den)
        e1.record()
        torch.cuda.synchronize()
        dn_ms = e0.elapsed_time(e1) / 8
        dn.close()
    n = frames - timed_from
    P = ((W + 7) // 8) * ((H + 7) // 8)
    rays = (ctx.stats()["rays"] - rays0) / n
    res = {"workload": f"{scene_name} {W}x{H}, R={R}, orbit camera and moving light, frames {timed_from}..{frames - 1}"
                       + (f", temporal upscaling {upscale}x{upscale}" if upscale > 1 else "")
                       + (", ray guiding" if ray_guiding else ""),
           "probe_rays_per_frame": int(rays), "ray_fraction": round(rays / (P * R), 4),
           "kernels_ms_per_frame": {k: round(v[1] / n, 5) for k, v in sorted(prof.items()) if k != "gbuffer"}}
    if dn_ms is not None:
        res["denoiser_ms_per_frame"] = round(dn_ms, 5)
    if "reconstruct" in prof:
        ms = prof["reconstruct"][1] / max(prof["reconstruct"][0], 1)
        b = P * (1024 + 32 + 1024 + 256)
        res["reconstruct"] = {"avg_ms": round(ms, 5), "alg_bytes": b, "gbs": round(b / (ms * 1e-3) / 1e9, 1),
                              "frac_hbm": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if upscale > 1:
        up = [k for k in prof if k.startswith("upscale_")]
        res["placement_ms_per_frame"] = round(sum(prof[k][1] for k in up) / n, 5)
    if "reproject" in prof:
        # the pass's kernels (each frame also renders its G-buffer, which is not part of it)
        pass_ms = sum(v[1] for k, v in prof.items() if k != "gbuffer") / n
        res["pass_ms_per_frame"] = round(pass_ms, 4)
        ms = prof["reproject"][1] / max(prof["reproject"][0], 1)
        b = W * H * 36 + P * 8
        res["reproject"] = {"avg_ms": round(ms, 5), "alg_bytes": b, "gbs": round(b / (ms * 1e-3) / 1e9, 1),
                            "frac_hbm": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    ctx.close()
    log(f"[bench] temporal reuse (upscale {upscale}, guiding {ray_guiding}): pass {res.get('pass_ms_per_frame')} ms/frame, "
        f"{res['ray_fraction']} of the rays, reproject "
        f"{res.get('reproject', {}).get('avg_ms')} ms ({res.get('reproject', {}).get('frac_hbm')} of HBM peak)")
    if with_cpu:
        res["cpu_baseline"] = temporal_cpu(scene, scene_name, W, H, R)
        log(f"[bench] temporal reuse, CPU oracle spawn with reprojection: {res['cpu_baseline']['value']:.1f} ms")
    return res


def temporal_quality(log, W=512, H=288, R=64, frames=32, ref_R=256, ref_frames=96):
    """What the temporal screen cache buys per ray (room, fixed camera, 512x288, 64 rays per
    probe): the per-pixel irradiance of frames 24..31 against a converged reference (the mean
    of 88 frames of 256 rays per probe without temporal reuse), as the relative L1 error over
    the image and the ratio of mean levels, for: no reuse; reuse (Algorithms 1, 3); reuse with
    ray guiding; 2x2 upscaling with adaptive sampling; upscaling with guiding; and the last
    two modes' ends followed by the screen-space denoiser (Section 2.4.3).  The rays per frame
    are measured by the context's counters."""
    import torch

    from paper_2310_19855_amd import gi
    from paper_2310_19855_amd import inputs as I
    scene = I.room_scene()
    cam = I.room_camera(0)

    def run(R_, nframes, keep_from, denoise=False, **kw):
        ctx = gi.Context(width=W, height=H, rays_per_probe=R_, table_log2=18, bounces=2, **kw)
        ctx.build_bvh(scene)
        gb = gi.GBuffer(H, W)
        out = torch.zeros((H, W, 4), dtype=torch.float32, device="cuda")
        dn = gi.Denoiser(W, H) if denoise else None
        den = torch.zeros((H, W, 4), dtype=torch.float32, device="cuda")
        acc, kept, rays0 = [], 0, 0
        for f in range(nframes):
            cam.index = f
            if f == keep_from:
                rays0 = ctx.stats()["rays"]
            ctx.render_gbuffer(cam, gb.pos, gb.nrm, gb.alb, gb.prim)
            ctx.spawn_probes(cam, gb.pos, gb.nrm, gb.prim)
            ctx.trace_probes(cam)
            ctx.cache_update(cam)
            ctx.interpolate_probes(cam, gb.pos, gb.nrm, gb.prim, out)
            if dn is not None:
                dn(cam, gb.pos, gb.nrm, gb.prim, out, den)
            if f >= keep_from:
                acc.append((den if dn is not None else out)[..., :3].clone())
                kept += 1
        rays = (ctx.stats()["rays"] - rays0) / max(kept, 1)
        ctx.close()
        if dn is not None:
            dn.close()
        return torch.stack(acc), rays

    ref_frames_t, _ = run(ref_R, ref_frames, 8)
    ref = ref_frames_t.mean(0)
    lum = ref.mean(-1)
    on = lum > 1e-3 * lum.max()
    modes = {"no_reuse": {}, "reuse": dict(temporal=1), "reuse_guided": dict(temporal=1, ray_guiding=1),
             "upscale_2x2": dict(temporal=1, upscale=2), "upscale_2x2_guided": dict(temporal=1, upscale=2, ray_guiding=1),
             "no_reuse_denoised": dict(denoise=True),
             "upscale_2x2_guided_denoised": dict(temporal=1, upscale=2, ray_guiding=1, denoise=True)}
    res = {"workload": f"room {W}x{H}, fixed camera, R={R}, two bounces, frames 24..{frames - 1}; reference "
                       f"R={ref_R} without reuse, mean of {ref_frames} frames", "modes": {}}
    for name, kw in modes.items():
        fr, rays = run(R, frames, 24, **kw)
        err = ((fr - ref).abs().mean(-1)[:, on] / lum[on]).mean().item()
        level = (fr.mean(-1)[:, on].mean() / lum[on].mean()).item()
        res["modes"][name] = {"rel_l1": round(err, 4), "level": round(level, 4), "rays_per_frame": int(rays)}
        log(f"[bench] temporal quality {name}: rel L1 {err:.4f}, level {level:.3f}, {int(rays)} rays/frame")
    return res


def light_sampling_measure(log, W=1920, H=1080, R=64, frames=16, timed_from=8, ref_R=128, ref_frames=96):
    """Light sampling on the room lit by 64 small quads of very different radiance: the plain
    cache's radiance at visible surface points (every 61st pixel of the frame-0 G-buffer)
    after 16 frames, against a converged run (area-proportional sampling, 128 rays per probe,
    96 frames, a long moving average), for area-proportional sampling and for RIS over the
    light grid with 1, 4 and 8 candidates and cell lists of 16, 64 and all 128 emitter
    triangles, and with world-space reservoir reuse (with the default cache history of 256
    samples, and with 8); the mean level against the reference's, ms/frame over frames 8..15
    and the light grid's kernels."""
    import numpy as np
    import torch

    from paper_2310_19855_amd import gi
    from paper_2310_19855_amd import inputs as I
    scene = I.lights_room_scene()
    cam = I.room_camera(0)

    def run(R_, nframes, n_cap_default, **kw):
        kw = dict(kw)
        n_cap = kw.pop("n_cap", n_cap_default)
        ctx = gi.Context(width=W, height=H, rays_per_probe=R_, table_log2=20, bounces=1, n_cap=n_cap, **kw)
        ctx.build_bvh(scene)
        gb = gi.GBuffer(H, W)
        out = torch.zeros((H, W, 4), dtype=torch.float32, device="cuda")
        ctx.render_gbuffer(cam, gb.pos, gb.nrm, gb.alb, gb.prim)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        for f in range(nframes):
            cam.index = f
            if f == timed_from:
                torch.cuda.synchronize()
                ctx.profile(True)
                ctx.profile_read()
                e0.record()
            ctx.spawn_probes(cam, gb.pos, gb.nrm, gb.prim)
            ctx.trace_probes(cam)
            ctx.cache_update(cam)
            ctx.interpolate_probes(cam, gb.pos, gb.nrm, gb.prim, out)
        e1.record()
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        ctx.profile(False)
        ms = e0.elapsed_time(e1) / max(nframes - timed_from, 1)
        hit = gb.prim.reshape(-1) != 0xFFFFFFFF
        pos = gb.pos.reshape(-1, 4)[hit][::61].clone()
        nrm = gb.nrm.reshape(-1, 4)[hit][::61].clone()
        pos[:, 3] = -1.0
        q = torch.zeros((pos.shape[0], 4), dtype=torch.float32, device="cuda")
        ctx.cache_query(pos, nrm, q)
        torch.cuda.synchronize()
        ctx.close()
        n = max(nframes - timed_from, 1)
        return ms, q.cpu().numpy(), {k: round(v[1] / n, 5) for k, v in prof.items()}

    _, ref, _ = run(ref_R, ref_frames, 1024)
    modes = {"area": {}, "ris4_k16": dict(light_grid=1, ris_candidates=4, lgrid_k=16),
             "ris4_k64": dict(light_grid=1, ris_candidates=4, lgrid_k=64),
             "ris1_k128": dict(light_grid=1, ris_candidates=1, lgrid_k=128),
             "ris4_k128": dict(light_grid=1, ris_candidates=4, lgrid_k=128),
             "ris8_k128": dict(light_grid=1, ris_candidates=8, lgrid_k=128),
             "ris4_k128_reuse": dict(light_grid=1, ris_candidates=4, lgrid_k=128, restir=1, restir_log2=20),
             # a cache that keeps little history (8 samples), as reservoir reuse is meant to allow
             "ris4_k128_ncap8": dict(light_grid=1, ris_candidates=4, lgrid_k=128, n_cap=8),
             "ris4_k128_reuse_ncap8": dict(light_grid=1, ris_candidates=4, lgrid_k=128, restir=1, restir_log2=20,
                                           n_cap=8),
             "ris4_k128_reuse_cap1": dict(light_grid=1, ris_candidates=4, lgrid_k=128, restir=1, restir_log2=20,
                                          restir_cap=1),
             "ris4_k128_reuse_cap1_ncap8": dict(light_grid=1, ris_candidates=4, lgrid_k=128, restir=1,
                                                restir_log2=20, restir_cap=1, n_cap=8)}
    res = {"workload": f"lights_room (64 emissive quads, radiance 2..200) {W}x{H}, R={R}, one bounce, frames "
                       f"0..{frames - 1}, ms/frame over {timed_from}..{frames - 1}; relMAE of the cache radiance at "
                       f"visible points vs area sampling at R={ref_R} over {ref_frames} frames", "modes": {}}
    for name, kw in modes.items():
        ms, q, kern = run(R, frames, 256, **kw)   # n_cap in kw overrides the 256
        both = (q[:, 3] > 0) & (ref[:, 3] > 0)
        e = float(np.abs(q[both, :3] - ref[both, :3]).sum() / max(np.abs(ref[both, :3]).sum(), 1e-30))
        level = float(q[both, :3].sum() / max(ref[both, :3].sum(), 1e-30))
        lg = {k: v for k, v in kern.items()
              if k in ("lg_box", "lg_box_final", "light_grid", "shade_hits", "restir_clear", "restir_store")}
        res["modes"][name] = {"ms_per_frame": round(ms, 4), "relMAE": round(e, 5), "level": round(level, 4),
                              "points": int(both.sum()), "kernels_ms": lg}
        log(f"[bench] light sampling {name}: relMAE {e:.4f}, level {level:.3f} @ {ms:.3f} ms/frame {lg}")
    return res


def temporal_cpu(scene, scene_name, W, H, R):
    """The oracle's spawn with reprojection (plain C, all host threads) for frame 1 of the orbit,
    after a full oracle frame 0 that leaves the history"""
    import oracle as O
    from paper_2310_19855_amd import inputs as I
    cores = O.set_threads(1)
    O.set_threads(cores)
    osc = O.OracleScene(scene)
    st = O.OracleFrameState(osc, dict(O.default_config(), width=W, height=H, rays_per_probe=R, table_log2=20,
                                      sky=scene.sky, temporal=1))
    f0 = I.camera_for(scene_name, 0)
    f0.index = 0
    osc.set_frame_dynamic(0)
    st.frame(f0, osc.gbuffer(f0, W, H))
    f1 = I.camera_for(scene_name, 1)
    f1.index = 1
    osc.set_frame_dynamic(1)
    gp, gn, ga, gprim = osc.gbuffer(f1, W, H)
    t0 = time.time()
    st.spawn(f1, gp, gn, gprim)
    ms = (time.time() - t0) * 1e3
    return {"value": round(ms, 1), "unit": "ms (spawn with reprojection, one frame)", "cores": cores, "kind": "oracle",
            "sample": "frame 1 of the orbit after an oracle frame 0"}


def probe_filter_cpu(scene, scene_name, W, H, R):
    """The oracle's two filter passes (plain C, all host threads) over the same view's probes,
    on a seeded synthetic atlas (radiance U[0,1], travelled distance U[0.1, 50] m)"""
    import numpy as np

    import oracle as O
    from paper_2310_19855_amd import inputs as I
    cores = O.set_threads(1)
    O.set_threads(cores)
    osc = O.OracleScene(scene)
    st = O.OracleFrameState(osc, dict(O.default_config(), width=W, height=H, rays_per_probe=R, table_log2=20,
                                      probe_filter=1))
    fr = I.camera_for(scene_name, 0)
    gp, gn, ga, gprim = osc.gbuffer(fr, W, H)
    st.spawn(fr, gp, gn, gprim)
    P = ((W + 7) // 8) * ((H + 7) // 8)
    rng = np.random.default_rng(21)
    atlas = np.concatenate([rng.uniform(0, 1, (P, 64, 3)), rng.uniform(0.1, 50.0, (P, 64, 1))], -1).astype(np.float32)
    t0 = time.time()
    a1 = st.filter_atlas(fr, 0, atlas)
    st.filter_atlas(fr, 1, a1)
    ms = (time.time() - t0) * 1e3
    return {"value": round(ms, 1), "unit": "ms per frame (x and y passes)", "cores": cores, "kind": "oracle",
            "sample": f"{P} probe tiles of the frame-0 view, one frame"}


def calibrate_copy(mib):
    """A plain elementwise device copy (read mib MiB, write mib MiB), five times: profiled with
    rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE it gives the scale of those counters."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_read_bytes": n * 4, "copy_write_bytes": n * 4, "launches": 5}), flush=True)


def cpu_baseline(scene, cfg, frames, log, single_frames=2):
    """The oracle (plain C, float32 parity mode, all host threads) on the same scene, config and
    frames at full resolution: spawn -> trace -> cache update -> gather + SH -> interpolate per
    frame, each stage timed; G-buffer rendering and the oracle's BVH build excluded.  Then the
    same on one thread over the first single_frames frames with a fresh cache."""
    import oracle as O
    from paper_2310_19855_amd import inputs as I
    cores = O.set_threads(1)        # the threads the parallel loops use (OMP_NUM_THREADS or all)
    O.set_threads(cores)
    t0 = time.time()
    osc = O.OracleScene(scene)
    t_build = time.time() - t0
    stage_names = ("spawn", "trace", "update", "gather_sh", "interpolate")

    def run(nframes):
        st = O.OracleFrameState(osc, dict(O.default_config(), **cfg))
        tot = dict.fromkeys(stage_names, 0.0)
        for f in range(nframes):
            cam = I.camera_for(scene.name, f)
            cam.index = f
            osc.set_frame_dynamic(f)
            pos, nrm, _alb, prim = osc.gbuffer(cam, cfg["width"], cfg["height"])
            t = [time.perf_counter()]
            st.spawn(cam, pos, nrm, prim)
            t.append(time.perf_counter())
            st.trace(cam)
            t.append(time.perf_counter())
            st.cache_update_only()
            t.append(time.perf_counter())
            st.probe_pass(cam)
            t.append(time.perf_counter())
            st.interpolate(cam, pos, nrm, prim)
            t.append(time.perf_counter())
            for i, k in enumerate(stage_names):
                tot[k] += t[i + 1] - t[i]
            log(f"[bench] cpu oracle frame {f}: {t[-1] - t[0]:.2f}s")
        return {k: v * 1e3 / max(nframes, 1) for k, v in tot.items()}

    stages = run(frames)
    ms = sum(stages.values())
    one = None
    if single_frames:
        prev = O.set_threads(1)
        s1 = run(single_frames)
        O.set_threads(prev)
        one = {"value": round(sum(s1.values()), 1), "unit": "ms/frame", "cores": 1,
               "stages_ms": {k: round(v, 2) for k, v in s1.items()},
               "sample": f"frames 0..{single_frames - 1}, fresh cache"}
        log(f"[bench] cpu oracle, one thread: {one['value']:.0f} ms/frame")
    return {"value": round(ms, 1), "unit": "ms/frame", "cores": cores, "kind": "oracle",
            "stages_ms": {k: round(v, 2) for k, v in stages.items()},
            "sample": f"{frames} full frames (frames 0..{frames - 1}) of the same workload, fresh cache, "
                      f"spawn..interpolate, G-buffer and the oracle's BVH build ({t_build:.1f}s) excluded",
            "host": _host_cpu(), "single_thread": one}


def _host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()

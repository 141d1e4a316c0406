"""Host-side legs of bench.py: the CPU oracle baseline and the Table-1 grouping run without a
GPU, so that a mistake in them cannot keep the benchmark from printing its line."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2310_19855_amd import inputs as I  # noqa: E402


def test_cpu_baseline_times_more_frames_than_the_gpu_run_renders():
    # the oracle leg builds its own cameras: more oracle frames than warmup + steps is fine
    scene = I.room_scene()
    cfg = dict(width=64, height=48, rays_per_probe=8, table_log2=14, bounces=1, sky=scene.sky, cache_mode=0)
    logs = []
    r = bench.cpu_baseline(scene, cfg, 4, logs.append, single_frames=1)
    assert r["kind"] == "oracle" and r["unit"] == "ms/frame" and r["cores"] >= 1
    assert set(r["stages_ms"]) == {"spawn", "trace", "update", "gather_sh", "interpolate"}
    assert all(v >= 0 for v in r["stages_ms"].values())
    assert abs(sum(r["stages_ms"].values()) - r["value"]) < 0.2
    assert r["single_thread"]["cores"] == 1
    assert sum(1 for m in logs if "cpu oracle frame" in m) == 4 + 1
    json.dumps(r)


def test_split_update_equals_update():
    # cache_update_only + probe_pass is the oracle's update, bit for bit
    import numpy as np

    import oracle as O
    scene = I.room_scene()
    cfg = dict(O.default_config(), width=48, height=40, rays_per_probe=8, table_log2=14, bounces=2)
    osc = O.OracleScene(scene)
    a = O.OracleFrameState(osc, cfg)
    b = O.OracleFrameState(osc, cfg)
    for f in range(3):
        cam = I.room_camera(f)
        cam.index = f
        pos, nrm, alb, prim = osc.gbuffer(cam, 48, 40)
        ea = a.frame(cam, (pos, nrm, alb, prim))
        b.spawn(cam, pos, nrm, prim)
        b.trace(cam)
        b.cache_update_only()
        b.probe_pass(cam)
        eb = b.interpolate(cam, pos, nrm, prim)
        assert np.array_equal(ea.view(np.uint32), eb.view(np.uint32))
        pa, pb = a.probes(), b.probes()
        for k in pa:
            assert np.array_equal(np.asarray(pa[k]), np.asarray(pb[k])), k


def test_table1_columns():
    kern = {"trace_probes": dict(launches=2, avg_ms=0.3), "shade_hits": dict(launches=2, avg_ms=0.2),
            "gather_sh": dict(launches=2, avg_ms=0.05), "interpolate": dict(launches=2, avg_ms=0.04),
            "spawn": dict(launches=2, avg_ms=0.01)}
    b = bench.table1_buckets(kern, 2)
    assert b["raytracing"] == 0.3
    assert abs(b["caching_sampling"] - 0.26) < 1e-9
    assert b["interpolate_denoise"] == 0.04


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr

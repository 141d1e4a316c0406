"""Writes the converged float64 references used by the equal-error comparison.

Calls only the oracle (float64 reference mode): a scene with its frame-0 camera and lights
frozen, R* = 1024 rays per probe, a world cache without history cap or eviction, run for K
frames.  Stored: the irradiance of the last frame (its Halton jitter fixes the probe
placement) and the world-cache cells whose history reached min_hist samples (key, radiance,
sample count).

    python -m oracle.make_reference [--scene room --width 480 --height 270 --frames 24 --rays 1024]

With --frame F --points-only: only the point reference of frame F of the scene's sequence
(its camera and its lights frozen at F), written to <scene><W>x<H>_f<F>_points.npz.
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2310_19855_amd import inputs as I  # noqa: E402


def reference(scene, width, height, frames, rays, seed=3):
    sc = I.make_scene(scene)
    osc = O.OracleScene(sc, f64=True)
    osc.set_frame_dynamic(0)
    cfg = O.default_config(width=width, height=height, rays_per_probe=rays, table_log2=22,
                           n_cap=0xFFFFFFFF, max_life=0xFFFFFFFF, seed=seed, sky=sc.sky)
    st = O.OracleFrameState(osc, cfg)
    out = None
    g = osc.gbuffer(I.camera_for(scene, 0), width, height)
    for f in range(frames):
        fr = I.camera_for(scene, 0)
        fr.index = f
        t0 = time.time()
        out = st.frame(fr, g)
        print(f"frame {f}: {time.time() - t0:.1f}s", flush=True)
    return out, st.table(), g, st


def point_reference(st, g, n_points, n_samples, seed=17, scene="room"):
    """Converged reflected radiance at seeded visible surface points: for one bounce a cell's
    sample is albedo * E / pi with E the one-light-sample NEE estimate (Sections 2.2.4, 2.3.1),
    so its expectation at a point is albedo times the mean of n_samples such estimates there.
    Points are G-buffer pixels (primary hits of the frozen camera) drawn without replacement."""
    pos, nrm, alb, prim = g
    valid = np.nonzero(prim.reshape(-1) != 0xFFFFFFFF)[0]
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(valid, size=min(n_points, len(valid)), replace=False))
    P = pos.reshape(-1, 4)[pick].astype(np.float64)
    Nn = nrm.reshape(-1, 4)[pick].astype(np.float64)
    A = alb.reshape(-1, 4)[pick, :3].astype(np.float64)
    fr = I.camera_for(scene, 0)   # only the frame index enters NEE: it picks the RNG stream
    fr.index = 1 << 20            # a stream of its own, apart from the frames' streams
    ids = np.arange(n_samples, dtype=np.uint32)
    L = np.zeros((len(pick), 3))
    se = np.zeros((len(pick), 3))
    t0 = time.time()
    for i in range(len(pick)):
        e = st.nee(fr, P[i, :3], Nn[i, :3], ids)
        L[i] = A[i] * e.mean(0)
        se[i] = A[i] * e.std(0) / np.sqrt(n_samples)
        if i % 1024 == 0:
            print(f"point {i}: {time.time() - t0:.1f}s", flush=True)
    P[:, 3] = -1.0              # lookups without the leak bit
    Nn[:, 3] = 0.0
    return pick, P.astype(np.float32), Nn.astype(np.float32), L, se


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scene", default="room", choices=("room", "field"))
    ap.add_argument("--min-hist", type=int, default=4096)
    ap.add_argument("--width", type=int, default=480)
    ap.add_argument("--height", type=int, default=270)
    ap.add_argument("--frames", type=int, default=24)
    ap.add_argument("--rays", type=int, default=1024)
    ap.add_argument("--points", type=int, default=8192)
    ap.add_argument("--point-samples", type=int, default=16384)
    ap.add_argument("--frame", type=int, default=0, help="frame of the sequence whose camera and lights are frozen")
    ap.add_argument("--points-only", action="store_true", help="only the point reference of --frame")
    args = ap.parse_args()
    if args.points_only:
        sc = I.make_scene(args.scene)
        osc = O.OracleScene(sc, f64=True)
        osc.set_frame_dynamic(args.frame)
        st = O.OracleFrameState(osc, O.default_config(width=args.width, height=args.height, rays_per_probe=1,
                                                       table_log2=10, sky=sc.sky))
        g = osc.gbuffer(I.camera_for(args.scene, args.frame), args.width, args.height)
        pix, ppos, pnrm, pL, pse = point_reference(st, g, args.points, args.point_samples, scene=args.scene)
        path = os.path.join(ROOT, "tests", "golden", f"{args.scene}{args.width}x{args.height}_f{args.frame}_points.npz")
        np.savez_compressed(path, frame=args.frame, width=args.width, height=args.height, scene=args.scene,
                            point_pixel=pix.astype(np.uint32), point_pos=ppos, point_nrm=pnrm,
                            point_L=pL.astype(np.float32), point_se=pse.astype(np.float32),
                            point_samples=args.point_samples)
        print(f"point reference of frame {args.frame}: relative standard error {pse.sum() / pL.sum():.4f}")
        print("wrote", path)
        return
    E, tab, g, st = reference(args.scene, args.width, args.height, args.frames, args.rays)
    pix, ppos, pnrm, pL, pse = point_reference(st, g, args.points, args.point_samples, scene=args.scene)
    # converged world-cache cells: those with at least min_hist samples of history
    min_hist = args.min_hist
    keep = tab["nhist"] >= min_hist
    path = os.path.join(ROOT, "tests", "golden", f"{args.scene}{args.width}x{args.height}_reference.npz")
    np.savez_compressed(path, irradiance=E[..., :3].astype(np.float32), flag=E[..., 3].astype(np.uint8),
                        frames=args.frames, rays=args.rays, width=args.width, height=args.height,
                        cell_key=tab["key"][keep], cell_L=tab["L"][keep].astype(np.float32),
                        cell_nhist=tab["nhist"][keep], min_hist=min_hist, scene=args.scene,
                        point_pixel=pix.astype(np.uint32), point_pos=ppos, point_nrm=pnrm,
                        point_L=pL.astype(np.float32), point_se=pse.astype(np.float32),
                        point_samples=args.point_samples)
    print(f"{keep.sum()} converged cells of {len(keep)}; point reference: relative standard error "
          f"{pse.sum() / pL.sum():.4f} (sum over points)")
    print("wrote", path)


if __name__ == "__main__":
    main()

"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Integers (probe mask, hit triangle, hit distance bits, cell keys, fixed-point sums and counts,
flags) must be bit-exact; float radiance within 1e-4 relative error (float64 evaluation)."""
import math

import numpy as np
import pytest

from gpu_common import SH_FLOOR, Pair, assert_close, bits

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_2310_19855_amd import gi  # noqa: E402
from paper_2310_19855_amd import inputs as I  # noqa: E402

SENT = 0xFFFFFFFF


def _compare_table(gt, ot):
    assert np.array_equal(gt["id"], ot["id"]), "cell id sets differ"
    assert np.array_equal(gt["key"], ot["key"])
    assert np.array_equal(gt["acc"], ot["acc"]), "fixed-point sums differ"


def _run_stage_parity(scene, cfg, frames, check_every=True, camera=None):
    pr = Pair(scene, cfg)
    for f in frames:
        if camera is not None:
            fr = camera(f)
        else:
            fr = I.camera_for(scene.name, f) if scene.name != "room" else I.room_camera(0)
        fr.index = f
        pr.set_frame_dynamic(f)
        (gp, gn, ga, gprim), (op, on, oa, oprim) = pr.gbuffer(fr)
        # G-buffer: bit-exact
        assert np.array_equal(gprim, oprim), "primary hits differ"
        assert np.array_equal(bits(gp), bits(op)) and np.array_equal(bits(gn), bits(on))
        assert np.array_equal(bits(ga), bits(oa))
        # spawn + mask MIPs
        pr.ctx.spawn_probes(fr, pr.gb.pos, pr.gb.nrm, pr.gb.prim)
        pr.ost.spawn(fr, op, on, oprim)
        gpr, opr = pr.ctx.probes(), pr.ost.probes()
        assert np.array_equal(gpr["mask"], opr["mask"]), "probe mask differs"
        assert np.array_equal(bits(gpr["pos"]), bits(opr["pos"]))
        assert np.array_equal(bits(gpr["nrm"]), bits(opr["nrm"]))
        # trace: rays, hits, keys, fixed-point sums
        pr.ctx.trace_probes(fr)
        pr.ost.trace(fr)
        gr, orr = pr.ctx.rays(), pr.ost.rays()
        assert np.array_equal(gr["tri"], orr["tri"]), "hit triangles differ"
        assert np.array_equal(bits(gr["t"]), bits(orr["t"])), "hit distances differ"
        assert np.array_equal(gr["cell"], orr["cell"]), "ray flags / atlas cells differ"
        hit = (orr["cell"] & gi.RAY_HIT) != 0
        assert np.array_equal(gr["key"][hit], orr["key"][hit]), "cell keys differ"
        assert np.array_equal(gr["slot"] >= 0, orr["slot"] >= 0)
        tiled = cfg.get("cache_tiles", 0)
        gt, ot = (pr.ctx.tiles(), pr.ost.tiles()) if tiled else (pr.ctx.table(), pr.ost.table())
        _compare_table(gt, ot)
        if cfg.get("light_grid", 0):
            gl, ol = pr.ctx.light_grid(), pr.ost.light_grid()
            assert np.array_equal(gl["dims"], ol["dims"]), "light grid dims differ"
            assert np.array_equal(bits(gl["lo"]), bits(ol["lo"].astype(np.float32))) and gl["h"] == ol["h"]
            assert np.array_equal(gl["count"], ol["count"]), "light list lengths differ"
            for c in np.nonzero(ol["count"])[0]:
                assert np.array_equal(gl["list"][c, :ol["count"][c]], ol["list"][c, :ol["count"][c]]), c
        if cfg.get("restir", 0):
            gv, ov = pr.ctx.reservoirs(), pr.ost.reservoirs()
            assert np.array_equal(gv["id"], ov["id"]) and np.array_equal(gv["key"], ov["key"]), "reservoir cells"
            for k in ("k", "M"):
                assert np.array_equal(gv[k], ov[k]), f"reservoir {k} differs"
            for k in ("y", "W", "n"):
                assert np.array_equal(bits(gv[k]), bits(ov[k].astype(np.float32))), f"reservoir {k} differs"
        gs, os_ = pr.ctx.stats(), pr.ost.stats()
        for k in ("rays", "hits", "inserts", "overflow", "nonfinite", "wraps", "shadow", "occluded", "bounce"):
            assert gs[k] == os_[k], f"stat {k}: gpu {gs[k]} oracle {os_[k]}"
        # update + gather + SH
        pr.ctx.cache_update(fr)
        pr.ost.update(fr)
        gt, ot = (pr.ctx.tiles(), pr.ost.tiles()) if tiled else (pr.ctx.table(), pr.ost.table())
        assert np.array_equal(gt["id"], ot["id"])
        assert np.array_equal(gt["nhist"], ot["nhist"]) and np.array_equal(gt["life"], ot["life"])
        assert_close(gt["L"], ot["L"], what="cached radiance")
        if tiled:
            assert_close(gt["Lq"], ot["Lq"], what="prefiltered radiance")
        gpr, opr = pr.ctx.probes(), pr.ost.probes()
        # radiance and travelled distance apart (a miss records 1e4 m, which would set the
        # floor of a joint comparison far above the radiance values)
        assert_close(gpr["atlas"][..., :3], opr["atlas"][..., :3], what="probe atlas radiance")
        assert_close(gpr["atlas"][..., 3], opr["atlas"][..., 3], what="probe atlas distance")
        assert_close(gpr["sh"], opr["sh"], what="SH coefficients", floor_frac=SH_FLOOR)
        # interpolate
        pr.ctx.interpolate_probes(fr, pr.gb.pos, pr.gb.nrm, pr.gb.prim, pr.out)
        go = pr.out.cpu().numpy()
        oo = pr.ost.interpolate(fr, op, on, oprim)
        assert np.array_equal(go[..., 3], oo[..., 3]), "interpolation flags differ"
        assert_close(go[..., :3], oo[..., :3], what="irradiance")
        gs, os_ = pr.ctx.stats(), pr.ost.stats()
        for k in ("live", "evict", "relaxed", "noprobe"):
            assert gs[k] == os_[k], f"stat {k}: gpu {gs[k]} oracle {os_[k]}"
    return pr


def test_room128_one_frame_stage_parity():
    """128x128 room, 16 rays per probe, 2^16 slots, one bounce, one frame"""
    _run_stage_parity(I.room_scene(), dict(width=128, height=128, rays_per_probe=16, table_log2=16), [0])


def test_room_multi_frame_two_bounces_ragged():
    """ragged tiles (100x76), 33 rays, cached bounce reading the previous update, eviction"""
    _run_stage_parity(I.room_scene(), dict(width=100, height=76, rays_per_probe=33, table_log2=14,
                                           bounces=2, max_life=2, n_cap=16), [0, 1, 2, 3])


def test_room_probe_filter_frames_ragged():
    """the probe-space filter of Algorithm 5 on (x pass, y pass, SH of the result): ragged
    100x76 room, 33 rays, two bounces, three frames; filtered atlas, SH and irradiance"""
    _run_stage_parity(I.room_scene(), dict(width=100, height=76, rays_per_probe=33, table_log2=14, bounces=2,
                                           probe_filter=1), [0, 1, 2])


def test_field_probe_filter_frames():
    """the filter on the ~1.0M-triangle field at 320x192 (sky tiles, depth discontinuities,
    misses with 1e4 m travelled distance), two frames with the moving light"""
    sc = I.field_scene()
    _run_stage_parity(sc, dict(width=320, height=192, rays_per_probe=64, table_log2=18, sky=sc.sky,
                               probe_filter=1), [0, 1])


def test_room_levels_of_detail_frames():
    """descriptor levels of detail on (lod_scale 0.065, Algorithm 6's distance scale at
    128x128): room distances of 1-6 m give levels 0-3; two bounces, so the bounce lookups use
    the levels too; keys, fixed-point sums, cells, atlas and irradiance as everywhere"""
    pr = _run_stage_parity(I.room_scene(), dict(width=128, height=128, rays_per_probe=16, table_log2=16,
                                                bounces=2, lod_scale=0.065), [0, 1])
    lods = (pr.ost.table()["key"].astype(np.int64) >> 58) & 7
    assert len(np.unique(lods)) >= 3, np.unique(lods)


def test_field_levels_of_detail_frames_and_query():
    """levels of detail on the field at 160x96 (lod_scale 0.05: 2-80 m give levels 0-6), two
    frames with the moving light, then lookup-only queries at random points and at the
    frame's hit points (measured from the last spawn's camera on both sides)"""
    sc = I.field_scene()
    pr = _run_stage_parity(sc, dict(width=160, height=96, rays_per_probe=64, table_log2=18, sky=sc.sky,
                                    lod_scale=0.05), [0, 1])
    lods = (pr.ost.table()["key"].astype(np.int64) >> 58) & 7
    assert len(np.unique(lods)) >= 4, np.unique(lods)
    pos, nrm = I.query_points(4000, -40.0, 40.0)
    pos[:, 1] = np.abs(pos[:, 1]) % 3.0
    # visible surface points of the last frame (the oracle's G-buffer), where probe rays of
    # neighbouring probes have created cells
    fr = I.camera_for("field", 1)
    fr.index = 1
    _, (op, on, oa, oprim) = pr.gbuffer(fr)
    vis = np.nonzero(oprim.reshape(-1) != 0xFFFFFFFF)[0][::7]
    sp = op.reshape(-1, 4)[vis].copy()
    sp[:, 3] = -1.0
    sn = on.reshape(-1, 4)[vis].copy()
    sn[:, 3] = 0.0
    pos = np.concatenate([pos, sp.astype(np.float32)])
    nrm = np.concatenate([nrm, sn.astype(np.float32)])
    out = torch.zeros((len(pos), 4), dtype=torch.float32, device="cuda")
    pr.ctx.cache_query(torch.from_numpy(pos).cuda(), torch.from_numpy(nrm).cuda(), out)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    o = pr.ost.query(pos, nrm)
    assert np.array_equal(g[:, 3], o[:, 3])
    assert o[4000:, 3].sum() > 100, "the surface queries should find cells"
    assert_close(g[:, :3], o[:, :3], what="query")


@pytest.mark.parametrize("R", [1, 64, 65, 256])
def test_extreme_rays_per_probe(R):
    """the smallest and the largest number of rays per probe (256 rays: four waves per probe
    in the trace, four chunks in the gather's per-cell sums), and both sides of the gather's
    64-entry ray stage (64 rays fill it; 65 take the full stage with a ragged second chunk)"""
    _run_stage_parity(I.room_scene(), dict(width=72, height=40, rays_per_probe=R, table_log2=16, bounces=2), [0, 1])


def test_minimum_frame_one_tile():
    """an 8x8 frame: one probe tile, a MIP chain of one level"""
    _run_stage_parity(I.room_scene(), dict(width=8, height=8, rays_per_probe=32, table_log2=10), [0, 1, 2])


def test_all_sky_view_has_no_probes():
    """a camera looking straight up over the field: every primary ray misses, so every tile
    is empty, no probe ray is traced and every pixel is flagged as sky"""
    sc = I.field_scene()
    cam = lambda f: I.look_frame(f, (0.0, 30.0, 0.0), (0.0, 1.0, 0.0), world_up=(0.0, 0.0, 1.0))
    pr = _run_stage_parity(sc, dict(width=64, height=48, rays_per_probe=16, table_log2=12, sky=sc.sky), [0],
                           camera=cam)
    assert pr.ctx.stats()["rays"] == 0
    assert (pr.out.cpu().numpy()[..., 3] == gi.INTERP_SKY).all()


@pytest.mark.parametrize("n_tris", [1, 2])
def test_one_and_two_triangle_scenes(n_tris):
    """the smallest scenes: a floor triangle (and, with two, an emitting triangle above it
    facing down); the BVH is a root holding one leaf"""
    v = np.array([[-5, 0, -5], [5, 0, -5], [0, 0, 8], [-1, 3, -1], [0, 3, 1], [1, 3, -1]], np.float32)
    idx = np.array([[0, 2, 1], [3, 4, 5]], np.uint32)[:n_tris]
    mats = np.array([[0.6, 0.5, 0.4, 0, 0, 0], [0, 0, 0, 20, 20, 20]], np.float32)
    sc = I.Scene(name="tri", verts=v, idx=idx, tri_mat=np.arange(n_tris, dtype=np.uint32), materials=mats,
                 sky=(0.1, 0.1, 0.1))
    cam = lambda f: I.look_frame(f, (0.0, 1.5, -4.0), (0.0, -0.3, 1.0))
    _run_stage_parity(sc, dict(width=48, height=40, rays_per_probe=32, table_log2=10, sky=sc.sky), [0, 1],
                      camera=cam)


def test_temporal_reuse_static_camera():
    """temporal reuse (Algorithm 1 reprojection, Algorithm 3 hysteresis) with a fixed camera:
    every probe stays on its pixel from frame 1 on, and the atlas is the new estimate blended
    with the history; masks, atlas, SH and irradiance against the oracle over four frames"""
    pr = _run_stage_parity(I.room_scene(), dict(width=96, height=72, rays_per_probe=32, table_log2=17, bounces=2,
                                                temporal=1), [0, 1, 2, 3], camera=lambda f: I.room_camera(0))
    assert pr.ctx.stats()["overflow"] == 0
    m = pr.ctx.probes()["mask"][:pr.ost.dims()[0]]
    win, hist = pr.ost.temporal()
    valid = m != SENT
    assert np.array_equal(win[valid], m[valid])


def test_temporal_reuse_orbit_and_filter():
    """temporal reuse on the field with the orbiting camera (1 degree per frame) and the moving
    light, the probe filter on: reprojection under motion, blending, filtering of the blended
    atlas; three frames"""
    sc = I.field_scene()
    pr = _run_stage_parity(sc, dict(width=160, height=96, rays_per_probe=64, table_log2=18, sky=sc.sky, temporal=1,
                                    probe_filter=1), [0, 1, 2])
    win, hist = pr.ost.temporal()
    assert (hist != SENT).sum() > 100, "the orbit should keep most probes"


def test_temporal_upscale_fixed_camera_ragged():
    """temporal upscaling 2x2 with adaptive sampling (Algorithm 2) on a ragged 100x76 room
    (spawn tiles cut by both screen edges), fixed camera, six frames: one traced probe per
    spawn tile, kept probes copying their history, empty tiles taking override tiles' rays;
    the traced flags of every ray, masks, atlas, SH and irradiance against the oracle"""
    pr = _run_stage_parity(I.room_scene(), dict(width=100, height=76, rays_per_probe=32, table_log2=17, bounces=2,
                                                temporal=1, upscale=2), list(range(6)),
                           camera=lambda f: I.room_camera(0))
    assert pr.ctx.stats()["overflow"] == 0
    win, hist, traced = pr.ost.temporal(with_traced=True)
    m = pr.ctx.probes()["mask"][:pr.ost.dims()[0]]
    assert (m != SENT).sum() > 0.9 * len(m) and traced.sum() < len(m) // 3


def test_temporal_upscale_orbit_and_filter():
    """temporal upscaling 2x2 on the field with the orbiting camera, the moving light and the
    filter on: sky tiles, probes lost to motion, adaptive sampling into them; four frames"""
    sc = I.field_scene()
    pr = _run_stage_parity(sc, dict(width=160, height=96, rays_per_probe=64, table_log2=18, sky=sc.sky, temporal=1,
                                    upscale=2, probe_filter=1), [0, 1, 2, 3])
    win, hist, traced = pr.ost.temporal(with_traced=True)
    assert 0 < traced.sum() < len(traced) // 2


def test_ray_guiding_fixed_camera_ragged():
    """ray guiding (Section 2.1.2) with temporal reuse on a ragged 100x76 room, fixed camera,
    two bounces, four frames: the parallax-corrected reconstruction, the integer inverse-CDF
    cell picks and the in-cell directions (every ray's cell, hit and distance bit-exact), the
    reconstruction as Algorithm 3's history; atlas, SH and irradiance against the oracle"""
    pr = _run_stage_parity(I.room_scene(), dict(width=100, height=76, rays_per_probe=32, table_log2=17, bounces=2,
                                                temporal=1, ray_guiding=1), [0, 1, 2, 3],
                           camera=lambda f: I.room_camera(0))
    recon, cdf = pr.ost.guiding()
    assert (cdf[:, 63] > 0).sum() > 0.9 * (pr.ost.probes()["mask"][:pr.ost.P] != SENT).sum()


def test_ray_guiding_upscale_orbit_and_filter():
    """everything of the temporal screen cache at once on the field: the orbit, the moving
    light, 2x2 upscaling with adaptive sampling, ray guiding (kept probes take the
    reconstruction) and the filter; four frames"""
    sc = I.field_scene()
    pr = _run_stage_parity(sc, dict(width=160, height=96, rays_per_probe=64, table_log2=18, sky=sc.sky, temporal=1,
                                    upscale=2, ray_guiding=1, probe_filter=1), [0, 1, 2, 3])
    recon, cdf = pr.ost.guiding()
    assert (cdf[:, 63] > 0).sum() > 50


def test_two_level_cache_room_frames_ragged():
    """the two-level world cache (Section 2.2.3) on a ragged 100x76 room, two bounces (bounce
    lookups read the prefiltered radiance), four frames with eviction (max_life 2): tile ids,
    keys and per-cell fixed-point sums bit-exact, per-cell moving averages, sample counts, tile
    lives, the prefiltered radiance of every cell, atlas, SH and irradiance"""
    pr = _run_stage_parity(I.room_scene(), dict(width=100, height=76, rays_per_probe=33, table_log2=10, bounces=2,
                                                max_life=2, n_cap=16, cache_tiles=1, tile_min_samples=8),
                           [0, 1, 2, 3])
    t = pr.ctx.tiles()
    assert len(t["id"]) > 10 and pr.ctx.stats()["overflow"] == 0
    # cells below the threshold read a coarser level
    few = (t["nhist"] > 0) & (t["nhist"] < 8)
    assert few.any() and not np.allclose(t["Lq"][few], t["L"][few])


def test_two_level_cache_field_levels_of_detail_and_query():
    """tiles on the field with levels of detail, the moving light and temporal reuse, two
    frames; then lookup-only queries at visible surface points read the prefiltered cells"""
    sc = I.field_scene()
    cfg = dict(width=160, height=96, rays_per_probe=64, table_log2=14, sky=sc.sky, cache_tiles=1,
               tile_min_samples=16, lod_scale=0.05, temporal=1)
    pr = _run_stage_parity(sc, cfg, [0, 1])
    (gp, gn, ga, gprim), _ = pr.gbuffer(I.camera_for(sc.name, 1))
    hit = gprim.reshape(-1) != 0xFFFFFFFF
    pos = gp.reshape(-1, 4)[hit][::7].copy()
    nrm = gn.reshape(-1, 4)[hit][::7].copy()
    pos[:, 3] = -1.0
    import torch
    out = torch.zeros((len(pos), 4), dtype=torch.float32, device="cuda")
    pr.ctx.cache_query(torch.from_numpy(pos).cuda(), torch.from_numpy(nrm).cuda(), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = pr.ost.query(pos, nrm)
    assert np.array_equal(got[:, 3], want[:, 3]) and got[:, 3].sum() > 0.5 * len(pos)
    assert_close(got[:, :3], want[:, :3], what="queried prefiltered radiance")


def test_light_grid_ris_many_light_room():
    """light sampling by RIS over the light grid (Section 2.3) on the room lit by 64 small
    quads, ragged 100x76, two bounces, three frames: the box of the hits, the grid and every
    cell's light list bit-exact, then every ray's record, the shadow-ray counts and the
    fixed-point sums (the picks of the reservoirs) bit-exact, atlas, SH and irradiance"""
    sc = I.lights_room_scene()
    pr = _run_stage_parity(sc, dict(width=100, height=76, rays_per_probe=32, table_log2=16, bounces=2,
                                    light_grid=1, lgrid_dim=8, lgrid_k=12, ris_candidates=4, lgrid_threshold=1e-3),
                           [0, 1, 2], camera=lambda f: I.room_camera(0))
    g = pr.ctx.light_grid()
    assert (g["count"] > 0).mean() > 0.5 and pr.ctx.stats()["shadow"] > 0


def test_restir_reservoir_reuse_many_light_room():
    """world-space reservoir reuse (Section 2.3.1) on the many-light room over four frames:
    the reservoir table of every frame (cells, light, point, weight, count, normal) and all
    that follows from the resampled picks bit-exact, then atlas, SH and irradiance"""
    sc = I.lights_room_scene()
    pr = _run_stage_parity(sc, dict(width=100, height=76, rays_per_probe=32, table_log2=16, bounces=2, light_grid=1,
                                    lgrid_dim=8, lgrid_k=128, ris_candidates=4, restir=1, restir_log2=16),
                           [0, 1, 2, 3], camera=lambda f: I.room_camera(0))
    r = pr.ctx.reservoirs()
    assert len(r["M"]) > 100 and r["M"].max() > 4


def test_every_option_together():
    """every part beyond the hot path at once on the many-light room with a turning camera:
    2x2 temporal upscaling with adaptive sampling and ray guiding, the probe filter, the
    two-level cache with levels of detail, the light grid with RIS and reservoir reuse, two
    bounces; four frames, every stage against the oracle"""
    import math
    sc = I.lights_room_scene()

    def cam(f):
        fr = I.room_camera(0)
        yaw = math.radians(1.5 * f)
        c, s = math.cos(yaw), math.sin(yaw)
        rot = lambda v: np.array([c * v[0] + s * v[2], v[1], -s * v[0] + c * v[2]], np.float32)
        fr.fwd, fr.right, fr.up = rot(fr.fwd), rot(fr.right), rot(fr.up)
        return fr
    _run_stage_parity(sc, dict(width=100, height=76, rays_per_probe=32, table_log2=12, bounces=2, temporal=1,
                               upscale=2, ray_guiding=1, probe_filter=1, cache_tiles=1, tile_min_samples=8,
                               lod_scale=0.06, light_grid=1, lgrid_dim=8, lgrid_k=32, ris_candidates=4, restir=1,
                               restir_log2=16), [0, 1, 2, 3], camera=cam)


def test_light_grid_field_moving_light():
    """the grid and RIS on the field, whose moving light changes the emitters every frame;
    one candidate (a uniform pick from the cell's list) and the default grid"""
    sc = I.field_scene()
    _run_stage_parity(sc, dict(width=160, height=96, rays_per_probe=32, table_log2=17, sky=sc.sky, light_grid=1,
                               ris_candidates=1), [0, 1])


def test_room_overflowing_table_invariants():
    pr = Pair(I.room_scene(), dict(width=64, height=64, rays_per_probe=32, table_log2=6))
    fr = I.room_camera(0)
    (gp, gn, ga, gprim), _ = pr.gbuffer(fr)
    pr.ctx.spawn_probes(fr, pr.gb.pos, pr.gb.nrm, pr.gb.prim)
    pr.ctx.trace_probes(fr)
    t = pr.ctx.table()
    s = pr.ctx.stats()
    r = pr.ctx.rays()
    assert len(t["id"]) <= 64 and s["overflow"] > 0
    hit = (r["cell"] & gi.RAY_HIT) != 0
    assert ((r["slot"] < 0) & hit).sum() == s["overflow"]
    assert len(np.unique(t["id"])) == len(t["id"])
    assert t["acc"][:, 3].sum() == (r["slot"] >= 0).sum()
    # every ray that holds a slot sees its own key in that cell
    for slot_key in np.unique(r["key"][r["slot"] >= 0]):
        assert slot_key in set(t["key"].tolist())


def test_field_traversal_matches_oracle_bvh():
    """~1.0M-triangle field: GPU 4-wide BVH walk == oracle's binary BVH, bit for bit"""
    sc = I.field_scene()
    pr = Pair(sc, dict(width=64, height=64))
    o, d = I.random_rays(200000, [-40, 0.05, -40], [40, 10, 40], seed=31)
    n = len(o)
    o4 = torch.zeros((n, 4), dtype=torch.float32)
    d4 = torch.zeros((n, 4), dtype=torch.float32)
    o4[:, :3] = torch.from_numpy(o)
    o4[:, 3] = 3.0e38
    d4[:, :3] = torch.from_numpy(d)
    o4, d4 = o4.cuda(), d4.cuda()
    tri = torch.zeros(n, dtype=torch.int32, device="cuda")
    t = torch.zeros(n, dtype=torch.float32, device="cuda")
    pr.ctx.trace_rays(o4, d4, tri, t)
    torch.cuda.synchronize()
    otri, ot = pr.osc.closest(o, d)
    assert np.array_equal(tri.cpu().numpy().view(np.uint32), otri)
    assert np.array_equal(t.cpu().numpy().view(np.uint32), ot.view(np.uint32))
    # any-hit with finite segments
    tm = np.random.default_rng(5).uniform(0.1, 20.0, n).astype(np.float32)
    o4[:, 3] = torch.from_numpy(tm).cuda()
    pr.ctx.trace_rays(o4, d4, tri, t, any_hit=True)
    torch.cuda.synchronize()
    assert np.array_equal(tri.cpu().numpy().view(np.uint32), pr.osc.any(o, d, tm))


def test_field_small_frames_with_moving_light():
    """the ~1.0M-triangle field at 160x96, 64 rays, a light moving between frames"""
    _run_stage_parity(I.field_scene(), dict(width=160, height=96, rays_per_probe=64, table_log2=18,
                                            sky=(0.05, 0.05, 0.05)), [0, 1])


def test_field1080_full_frames_in_the_benchmark_configuration():
    """the benchmark's own configuration at full size: 1920x1080 over the ~1.0M-triangle
    field, 64 rays per probe, 2^20 slots, camera orbit and moving light, frames 0 and 1 (every
    pixel, probe, ray, cell and atlas entry compared)"""
    p = I.PRESETS["field1080"]
    sc = I.field_scene()
    _run_stage_parity(sc, dict(width=p["width"], height=p["height"], rays_per_probe=p["rays_per_probe"],
                               table_log2=p["table_log2"], bounces=p["bounces"], sky=sc.sky), [0, 1])


def test_city4k_full_frames_two_bounces():
    """the 4K city at full size: 3840x2160 over ~9.4M triangles, 128 rays per probe, two
    bounces (the second read from the previous frame's cache), frames 0 and 1.  Most of the
    16.6M rays hit a 10 cm cell of their own on this 4 km city, so the table has 2^26 slots
    here and no bucket overflows (which keys win a full bucket depends on the order of
    insertion; the configured 2^22 slots are checked by the next test)"""
    p = I.PRESETS["city4k"]
    sc = I.city_scene()
    pr = _run_stage_parity(sc, dict(width=p["width"], height=p["height"], rays_per_probe=p["rays_per_probe"],
                                    table_log2=26, bounces=p["bounces"], sky=sc.sky), [0, 1])
    assert pr.ctx.stats()["overflow"] == 0


def test_city4k_configured_table_overflow():
    """the 4K city with its configured 2^22 slots, where buckets overflow: hits, keys and the
    per-key fixed-point sums of every key both sides hold are bit-exact; a key held by one
    side only sits in a bucket the other side filled; a held key received all its samples;
    a ray holds a slot exactly when its key is held"""
    p = I.PRESETS["city4k"]
    sc = I.city_scene()
    pr = Pair(sc, dict(width=p["width"], height=p["height"], rays_per_probe=p["rays_per_probe"],
                       table_log2=p["table_log2"], bounces=p["bounces"], sky=sc.sky))
    fr = I.camera_for("city", 0)
    fr.index = 0
    (gp, gn, ga, gprim), (op, on, oa, oprim) = pr.gbuffer(fr)
    assert np.array_equal(gprim, oprim)
    pr.ctx.spawn_probes(fr, pr.gb.pos, pr.gb.nrm, pr.gb.prim)
    pr.ost.spawn(fr, op, on, oprim)
    pr.ctx.trace_probes(fr)
    pr.ost.trace(fr)
    gr, orr = pr.ctx.rays(), pr.ost.rays()
    assert np.array_equal(gr["tri"], orr["tri"]) and np.array_equal(bits(gr["t"]), bits(orr["t"]))
    hit = (orr["cell"] & gi.RAY_HIT) != 0
    assert np.array_equal(gr["key"][hit], orr["key"][hit])
    gt, ot = pr.ctx.table(), pr.ost.table()
    gs, os_ = pr.ctx.stats(), pr.ost.stats()
    assert gs["overflow"] > 0 and os_["overflow"] > 0
    keys, n_rays = np.unique(orr["key"][hit], return_counts=True)
    per_key = dict(zip(keys.tolist(), n_rays.tolist()))
    for t, r, st in ((gt, gr, gs), (ot, orr, os_)):
        held = t["key"]
        # each held key received all its samples, and rays hold a slot exactly for held keys
        assert np.array_equal(t["acc"][:, 3], np.array([per_key[int(k)] for k in held], np.uint32))
        assert np.array_equal(r["slot"][hit] >= 0, np.isin(r["key"][hit], held))
        assert st["overflow"] + st["nonfinite"] == int(hit.sum()) - int(t["acc"][:, 3].sum())
    # keys held by both sides: identical sums; keys held by one side: the other side's bucket is full
    common, gi_idx, oi_idx = np.intersect1d(gt["key"], ot["key"], return_indices=True)
    assert np.array_equal(gt["acc"][gi_idx], ot["acc"][oi_idx])
    assert np.array_equal(gt["id"][gi_idx], ot["id"][oi_idx])
    for t_one, t_other in ((gt, ot), (ot, gt)):
        only = ~np.isin(t_one["key"], t_other["key"])
        buckets_other, fill_other = np.unique(t_other["id"] >> np.uint64(32), return_counts=True)
        fill = dict(zip(buckets_other.tolist(), fill_other.tolist()))
        for b in np.unique(t_one["id"][only] >> np.uint64(32)).tolist():
            assert fill.get(b, 0) == 32, f"bucket {b} not full on the other side"


def test_furnace_parity_and_closed_form():
    """closed diffuse sphere (Le = 1, albedo 0.8, ~200k triangles), feedback through the
    cache with replacement: two frames against the oracle, then the GPU alone follows the
    recurrence L_f = albedo (Le + L_{f-1}) towards Le / (1 - albedo) = 5"""
    sc = I.furnace_scene()
    cfg = dict(width=96, height=96, rays_per_probe=64, table_log2=18, cell_scale=0.5, n_cap=0, leak_bit=0,
               bounces=2)
    pr = _run_stage_parity(sc, cfg, [0, 1])
    rho, le = 0.8, 1.0
    L = rho * (le + rho * le)
    for f in range(2, 40):
        fr = I.camera_for("furnace", 0)
        fr.index = f
        pr.ctx.spawn_probes(fr, pr.gb.pos, pr.gb.nrm, pr.gb.prim)
        pr.ctx.trace_probes(fr)
        pr.ctx.cache_update(fr)
        L = rho * (le + L)
        p = pr.ctx.probes()
        valid = p["mask"][:len(p["pos"])] != SENT
        atlas = p["atlas"][valid][..., :3].astype(np.float64)
        # every probe ray returns Le + L_f of the cell it hits: the mean over the GPU atlas
        # follows the recurrence (cells created late lag a frame early on; single cells spread
        # up to a few % from the facets and the 2^-12 steps)
        assert abs(atlas.mean() / (le + L) - 1) < (1.5e-3 if f < 20 else 3e-4), f
        assert np.abs(atlas / (le + L) - 1).max() < 0.1, f
    # and converges to the closed-form limit Le / (1 - rho) = 5 (rho^41 = 1.1e-4 away)
    assert abs(atlas.mean() / (le / (1 - rho)) - 1) < 7e-4
    # the cells the last frame's rays touched hold L_39 = rho Le (1 - rho^40) / (1 - rho)
    t = pr.ctx.table()
    live = t["life"] == cfg.get("max_life", 32)
    assert live.sum() > 100
    assert abs(t["L"][live].astype(np.float64).mean() / L - 1) < 5e-4
    pr.ctx.interpolate_probes(fr, pr.gb.pos, pr.gb.nrm, pr.gb.prim, pr.out)
    o = pr.out.cpu().numpy()
    assert (o[..., 3] == 0).all()
    assert abs(o[..., :3].mean() / (math.pi * (le + L)) - 1) < 2e-3


def test_cache_query_matches_oracle():
    pr = _run_stage_parity(I.room_scene(), dict(width=96, height=96, rays_per_probe=16, table_log2=14), [0])
    t = pr.ost.table()
    keys = t["key"].astype(np.int64)
    q = np.stack([(keys >> s) & 0x3FFFF for s in (0, 18, 36)], 1)
    q = np.where(q >= (1 << 17), q - (1 << 18), q)
    cls = (keys >> 54) & 7
    leak = (keys >> 57) & 1
    n = len(keys)
    nrm = np.zeros((n, 4), np.float32)
    nrm[np.arange(n), cls // 2] = np.where(cls % 2 == 1, -1.0, 1.0)
    pos = np.zeros((n, 4), np.float32)
    pos[:, :3] = (q + 0.5) / 10.0
    pos[:, 3] = np.where(leak == 1, 0.05, 1.0)
    extra_p, extra_n = I.query_points(1000, -2.0, 8.0)
    pos = np.concatenate([pos, extra_p])
    nrm = np.concatenate([nrm, extra_n])
    out = torch.zeros((len(pos), 4), dtype=torch.float32, device="cuda")
    pr.ctx.cache_query(torch.from_numpy(pos).cuda(), torch.from_numpy(nrm).cuda(), out)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    o = pr.ost.query(pos, nrm)
    assert np.array_equal(g[:, 3], o[:, 3])
    assert (g[:n, 3] == 1).all()
    assert_close(g[:, :3], o[:, :3], what="query")


def test_determinism_repeated_runs():
    res = []
    for _ in range(2):
        pr = Pair(I.room_scene(), dict(width=128, height=128, rays_per_probe=64, table_log2=16))
        fr = I.room_camera(0)
        pr.gbuffer(fr)
        pr.ctx.spawn_probes(fr, pr.gb.pos, pr.gb.nrm, pr.gb.prim)
        pr.ctx.trace_probes(fr)
        t = pr.ctx.table()
        pr.ctx.cache_update(fr)
        pr.ctx.interpolate_probes(fr, pr.gb.pos, pr.gb.nrm, pr.gb.prim, pr.out)
        assert pr.ctx.stats()["overflow"] == 0
        res.append((t["id"], t["acc"], pr.ctx.probes()["atlas"], pr.out.cpu().numpy()))
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_cache_save_load_resume():
    """N frames, save, restore into a fresh context, M frames == N + M frames, bit for bit"""
    sc = I.room_scene()
    cfg = dict(width=64, height=64, rays_per_probe=16, table_log2=16, bounces=2)

    def run(ctx, gb, out, frames):
        for f in frames:
            fr = I.room_camera(0)
            fr.index = f
            ctx.render_gbuffer(fr, gb.pos, gb.nrm, gb.alb, gb.prim)
            ctx.spawn_probes(fr, gb.pos, gb.nrm, gb.prim)
            ctx.trace_probes(fr)
            ctx.cache_update(fr)
            ctx.interpolate_probes(fr, gb.pos, gb.nrm, gb.prim, out)
        torch.cuda.synchronize()
        return out.cpu().numpy()

    a = gi.Context(**cfg)
    a.build_bvh(sc)
    gb = gi.GBuffer(64, 64)
    out = torch.zeros((64, 64, 4), dtype=torch.float32, device="cuda")
    full = run(a, gb, out, range(5))
    ta = a.table()
    b = gi.Context(**cfg)
    b.build_bvh(sc)
    run(b, gb, out, range(3))
    blob = b.cache_save()
    c = gi.Context(**cfg)
    c.build_bvh(sc)
    c.cache_load(blob)
    resumed = run(c, gb, out, range(3, 5))
    tc = c.table()
    # bit-exact resume needs an order-free run: no bucket may overflow
    assert a.stats()["overflow"] == 0 and c.stats()["overflow"] == 0
    assert np.array_equal(bits(full), bits(resumed))
    assert np.array_equal(ta["id"], tc["id"]) and np.array_equal(bits(ta["L"]), bits(tc["L"]))


def test_invalid_arguments_and_frame_order():
    ctx = gi.Context(width=64, height=64)
    with pytest.raises(gi.GIError, match="STATE"):
        ctx.trace_probes(I.room_camera(0))
    with pytest.raises(gi.GIError):
        gi.Context(width=4, height=64)
    with pytest.raises(gi.GIError):
        gi.Context(rays_per_probe=1000)
    with pytest.raises(gi.GIError, match="INVALID"):
        gi.Context(width=64, height=64, upscale=2)          # upscaling needs temporal reuse
    with pytest.raises(gi.GIError):
        gi.Context(width=64, height=64, temporal=1, upscale=5)
    with pytest.raises(gi.GIError, match="INVALID"):
        gi.Context(width=64, height=64, ray_guiding=1)      # guiding needs temporal reuse
    with pytest.raises(gi.GIError, match="INVALID"):
        gi.Context(width=64, height=64, cache_tiles=1, cache_mode=gi.CACHE_MLP_BF16)   # tiles: plain cache only
    with pytest.raises(gi.GIError, match="INVALID"):
        gi.Context(width=64, height=64, restir=1)            # reservoirs need the light grid
    with pytest.raises(gi.GIError, match="INVALID"):
        gi.Context(width=64, height=64, frac_bits=16, r_max=1024.0)   # a wave's group sum would wrap
    gi.Context(width=64, height=64, frac_bits=16, r_max=1000.0).close()
    ctx = gi.Context(width=64, height=64, cache_tiles=1, table_log2=8)
    with pytest.raises(gi.GIError, match="UNSUPPORTED"):
        ctx.table()                                          # per-cell export of the single-level cache
    with pytest.raises(gi.GIError, match="INVALID"):
        ctx.profile(3)                                       # timer levels are 0, 1 and 2
    ctx.close()


def test_denoiser_frames_with_a_turning_camera():
    """the screen-space denoiser (Section 2.4.3) after the GPU and oracle frames of a ragged
    100x76 room whose camera turns 2 degrees a frame (disocclusion at one edge): history
    lengths and radii bit-exact, accumulated history and denoised irradiance against the
    oracle's (each side denoising its own interpolation)"""
    import math
    import torch
    W, H = 100, 76
    pr = Pair(I.room_scene(), dict(width=W, height=H, rays_per_probe=16, table_log2=15, denoise=1, dn_hist_max=8,
                                   dn_radius=4))
    dn = gi.Denoiser(W, H, hist_max=8, radius_max=4)
    out = torch.zeros((H, W, 4), dtype=torch.float32, device="cuda")
    for f in range(4):
        fr = I.room_camera(0)
        fr.index = f
        yaw = math.radians(2.0 * f)
        c, s = math.cos(yaw), math.sin(yaw)
        rot = lambda v: np.array([c * v[0] + s * v[2], v[1], -s * v[0] + c * v[2]], np.float32)
        fr.fwd, fr.right, fr.up = rot(fr.fwd), rot(fr.right), rot(fr.up)
        (gp, gn, ga, gprim), (op, on, oa, oprim) = pr.gbuffer(fr)
        pr.ctx.spawn_probes(fr, pr.gb.pos, pr.gb.nrm, pr.gb.prim)
        pr.ost.spawn(fr, op, on, oprim)
        pr.ctx.trace_probes(fr)
        pr.ost.trace(fr)
        pr.ctx.cache_update(fr)
        pr.ost.update(fr)
        pr.ctx.interpolate_probes(fr, pr.gb.pos, pr.gb.nrm, pr.gb.prim, pr.out)
        oirr = pr.ost.interpolate(fr, op, on, oprim)
        dn(fr, pr.gb.pos, pr.gb.nrm, pr.gb.prim, pr.out, out)
        torch.cuda.synchronize()
        oout = pr.ost.denoise(fr, op, on, oprim.reshape(H, W), oirr)
        gh, grad = dn.state()
        oh, orad = pr.ost.denoise_state()
        assert np.array_equal(gh[..., 3], oh[..., 3]), f"history lengths differ at frame {f}"
        assert np.array_equal(grad, orad), f"radii differ at frame {f}"
        assert_close(gh[..., :3], oh[..., :3], what="denoiser history")
        go = out.cpu().numpy()
        assert np.array_equal(go[..., 3], oout[..., 3])
        assert_close(go[..., :3], oout[..., :3], what="denoised irradiance")
    assert (gh[..., 3] == 4).mean() > 0.6 and (gh[..., 3] == 1).any()
    dn.close()

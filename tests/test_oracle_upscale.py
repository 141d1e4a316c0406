"""Pins of the oracle's temporal upscaling and adaptive sampling (Section 2.1.1 spawn tiles,
Section 2.1.2 and Algorithm 2), upscale u = 2: 16x16-pixel spawn tiles, one new probe per
spawn tile and frame.

What the method fixes, checked here without re-running the oracle's code path:
- the spawn jitter is floor(16 * Halton) in bases 2 and 3 (closed forms for the first frames;
  halving it gives the 8-pixel jitter of upscale 1);
- on the first frame exactly the probe tiles that hold the jittered pixel of their spawn tile
  trace, at that pixel, and nothing else holds a probe;
- the rays are conserved: adaptive sampling moves rays between tiles, so the number of
  traced probes always equals the number of spawned tiles, and the ray count is that times
  the rays per probe (a quarter of upscale 1's on a screen of whole spawn tiles);
- with a fixed camera a probe, once placed, stays on its pixel; a kept probe that does not
  trace keeps its previous radiance exactly; after the four quadrants of the spawn tile have
  each been jittered into (frames 0, 1, 3, 4 of the Halton sequence) every tile holds a probe;
  such a kept probe keeps its SH as well (SH reprojection);
- Algorithm 2 under this implementation's reading (override tiles in tile order, pick by the
  counter hash of dimension 7, the lowest-numbered picker wins) on a frame where override and
  empty tiles exist (frame 2 of the fixed camera)."""
import numpy as np
import pytest

import oracle as O
from paper_2310_19855_amd import inputs as I

SENT = 0xFFFFFFFF


def test_spawn_jitter_closed_forms():
    # frames 0..4 use Halton indices 1..5: base 2 -> 1/2, 1/4, 3/4, 1/8, 5/8; base 3 -> 1/3,
    # 2/3, 1/9, 4/9, 7/9; times 16, floored
    want = [(8, 5), (4, 10), (12, 1), (2, 7), (10, 12)]
    assert [O.halton_jitter(f, 16) for f in range(5)] == want
    for f in range(200):
        a, b = O.halton_jitter(f, 16)
        c, d = O.halton_jitter(f, 8)
        assert (a // 2, b // 2) == (c, d)


def _run(cfg, frames, cam=None):
    sc = I.room_scene()
    osc = O.OracleScene(sc, f64=True)
    st = O.OracleFrameState(osc, O.default_config(**cfg))
    out = []
    prev_rays = 0
    for f in frames:
        fr = cam(f) if cam else I.room_camera(0)
        fr.index = f
        g = osc.gbuffer(fr, cfg["width"], cfg["height"])
        st.frame(fr, g)
        P = int(st.dims()[0])
        pr = st.probes()
        win, hist, traced = st.temporal(with_traced=True)
        rays = int(st.stats()["rays"])
        out.append(dict(mask=pr["mask"][:P].copy(), atlas=pr["atlas"].copy(), sh=pr["sh"].copy(), win=win, hist=hist,
                        traced=traced.astype(bool), rays=rays - prev_rays, prim=g[3].reshape(-1)))
        prev_rays = rays
    return st, out


def _spawned(f, W, H, TW, TH, prim, u=2):
    sx, sy = O.halton_jitter(f, 8 * u)
    s = np.zeros(TW * TH, bool)
    pix = np.full(TW * TH, SENT, np.uint32)
    for ty in range(TH):
        for tx in range(TW):
            px, py = 8 * u * (tx // u) + sx, 8 * u * (ty // u) + sy
            if px // 8 == tx and py // 8 == ty and px < W and py < H and prim[py * W + px] != SENT:
                s[ty * TW + tx] = True
                pix[ty * TW + tx] = (py << 16) | px
    return s, pix


CFG = dict(width=64, height=48, rays_per_probe=16, table_log2=15, temporal=1, upscale=2)


def test_first_frame_traces_one_tile_per_spawn_tile():
    st, out = _run(CFG, [0])
    o = out[0]
    TW, TH = 8, 6
    assert (o["prim"] != SENT).all()          # the room is closed: no sky
    s, pix = _spawned(0, 64, 48, TW, TH, o["prim"])
    # jitter (8, 5): the right-hand, upper probe tile of every spawn tile
    tiles = np.nonzero(s)[0]
    assert sorted(tiles) == sorted(ty * TW + tx for ty in range(0, TH, 2) for tx in range(1, TW, 2))
    assert np.array_equal(o["traced"], s)
    assert np.array_equal(o["mask"][s], pix[s])
    assert (o["mask"][~s] == SENT).all()
    assert o["rays"] == s.sum() * 16 == TW * TH * 16 // 4


def test_fixed_camera_sequence():
    W, H, TW, TH = 64, 48, 8, 6
    st, out = _run(CFG, list(range(6)))
    for f, o in enumerate(out):
        s, _ = _spawned(f, W, H, TW, TH, o["prim"])
        # rays conserved: as many traced probes as spawned tiles, R rays each
        assert o["traced"].sum() == s.sum(), f
        assert o["rays"] == s.sum() * 16, f
        placed = o["mask"] != SENT
        assert not (o["traced"] & ~placed).any()
        if f == 0:
            continue
        p = out[f - 1]
        prev_placed = p["mask"] != SENT
        # a placed probe stays on its pixel, with itself as history
        assert np.array_equal(o["mask"][prev_placed], p["mask"][prev_placed]), f
        assert np.array_equal(o["hist"][prev_placed], np.nonzero(prev_placed)[0].astype(np.uint32))
        assert (placed >= prev_placed).all()
        # kept probes that did not trace keep their radiance exactly, and their SH with it
        # (SH reprojection: no projection for them)
        kept = prev_placed & ~o["traced"]
        assert kept.any()
        assert np.array_equal(o["atlas"][kept], p["atlas"][kept]), f
        assert np.array_equal(o["sh"][kept], p["sh"][kept]), f
        # kept probes that traced blend new rays into it
        fresh = prev_placed & o["traced"]
        if fresh.any():
            assert not np.array_equal(o["atlas"][fresh], p["atlas"][fresh])
    # quadrants jittered so far: (1,0) frames 0 and 2, (0,1) frame 1, (0,0) frame 3, (1,1)
    # frame 4: from frame 4 on every tile holds a probe
    assert (out[3]["mask"] == SENT).any()
    assert (out[4]["mask"] != SENT).all() and (out[5]["mask"] != SENT).all()


def test_adaptive_sampling_reading_on_frame_two():
    """frame 2 jitters into the quadrant of frame 0 again: those tiles are spawned and kept
    (override tiles); the quadrants never jittered so far are empty.  Each empty tile picks
    override tile over[hash(seed, 2, tile, 7) % count]; an override tile picked by anyone
    gives its rays to the lowest-numbered tile that picked it, whose probe is placed at its
    own pixel of the jitter (12 % 8, 1 % 8) = (4, 1)"""
    W, H, TW, TH = 64, 48, 8, 6
    st, out = _run(CFG, [0, 1, 2])
    o, p = out[2], out[1]
    s, _ = _spawned(2, W, H, TW, TH, o["prim"])
    kept = p["mask"] != SENT
    over = np.nonzero(s & kept)[0]
    empty = np.nonzero(~s & ~kept)[0]
    assert len(over) == TW * TH // 4 and len(empty) == TW * TH // 2
    seed = O.default_config()["seed"]
    winner = {}
    for e in empty:
        k = over[O.rng(seed, 2, int(e), 7) % len(over)]
        winner[k] = min(winner.get(k, 1 << 30), int(e))
    assert 0 < len(winner) < len(over)         # some override tiles keep their rays
    for t in over:
        assert o["traced"][t] == (t not in winner), t
    took = set(winner.values())
    for e in empty:
        if e in took:
            tx, ty = e % TW, e // TW
            assert o["traced"][e]
            assert o["mask"][e] == ((8 * ty + 1) << 16) | (8 * tx + 4)
        else:
            assert not o["traced"][e] and o["mask"][e] == SENT


def test_upscale_one_equals_off():
    cfg0 = dict(width=40, height=24, rays_per_probe=8, table_log2=12, temporal=1)
    _, a = _run(dict(cfg0, upscale=0), [0, 1])
    _, b = _run(dict(cfg0, upscale=1), [0, 1])
    for x, y in zip(a, b):
        assert np.array_equal(x["mask"], y["mask"]) and np.array_equal(x["atlas"], y["atlas"])
        assert x["traced"].sum() == (x["mask"] != SENT).sum()

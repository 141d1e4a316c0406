"""Pins of the oracle's temporal reuse of screen probes: probe reprojection (Algorithm 1) and
the biased shadow-preserving hysteresis of Algorithm 3.

The half-precision packing of Algorithm 1 is checked against numpy's float16 conversion; the
hysteresis against values worked out by hand; reprojection against two camera motions whose
answer is fixed by geometry: none (every probe stays on its pixel) and a sideways move of
exactly 16 pixels' footprint over a floor seen from above (every probe reappears 16 pixels
away, its history two tiles over)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2310_19855_amd import inputs as I

SENT = 0xFFFFFFFF


def test_half_packing_matches_float16_rounding():
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.uniform(0, 1, 3000), rng.uniform(0, 70000, 3000), 10.0 ** rng.uniform(-9, 5, 3000),
                        [0.0, 65504.0, 65519.99, 65520.0, 6.1035156e-05, 5.9604645e-08, 2.9802322e-08, 1e-30]])
    x = x.astype(np.float32)
    with np.errstate(over="ignore"):      # values from 65520 up round to infinity
        want = x.astype(np.float16).view(np.uint16).astype(np.uint32)
    got = np.array([O.half_bits(float(v)) for v in x], np.uint32)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(float(x[i]), hex(got[i]), hex(want[i])) for i in bad[:5]]
    assert O.half_bits(65504.0) == 0x7BFF


@pytest.mark.parametrize("f64", [True, False])
def test_hysteresis_hand_cases(f64):
    # new, history -> luminance ratio; alpha = clamp((l1 - l2 - min) / max, 0, 0.95)^2
    cases = [
        (4.0, 1.0, 3.25),                 # alpha = (4-1-1)/4 = 0.5 -> 0.25: 4 + 0.25 (1 - 4)
        (1.0, 4.0, 1.0),                  # darker than the history: alpha = 0, taken at once
        (2.0, 2.0, 2.0),                  # unchanged
        (10.0, 1.0, 10.0 - 0.64 * 9.0),   # alpha = 0.8^2
        (100.0, 1.0, 100.0 - 0.9025 * 99.0),  # alpha clamped to 0.95, squared
        (0.0, 0.0, 0.0),                  # both dark: max(l1, l2) floored at 1e-4
        (2.0, 1.0, 2.0),                  # exactly twice: alpha = 0
    ]
    curr = np.array([[c, c, c, 5.0] for c, _, _ in cases])
    prev = np.array([[q, q, q, 9.0] for _, q, _ in cases])
    out = O.temporal_blend(curr, prev, f64=f64)
    tol = 1e-12 if f64 else 1e-6
    for (c, q, want), o in zip(cases, out):
        assert abs(o[0] - want) <= tol * max(1.0, abs(want)), (c, q, o[0], want)
        assert o[0] == o[1] == o[2]
    # the travelled distance follows the same alpha: 5 + 0.25 (9 - 5) in the first case
    assert abs(out[0][3] - 6.0) <= tol * 6
    # colour: luminance is the channel mean, so a pure-red brightening is judged on r / 3
    o = O.temporal_blend([[6.0, 0.0, 0.0, 1.0]], [[0.5, 0.5, 0.5, 1.0]], f64=f64)[0]
    a = ((2.0 - 0.5 - 0.5) / 2.0) ** 2
    assert abs(o[0] - (6.0 + a * (0.5 - 6.0))) <= tol * 6


def _frames(sc, cfg, cams, temporal=1):
    osc = O.OracleScene(sc, f64=True)
    st = O.OracleFrameState(osc, O.default_config(temporal=temporal, **cfg))
    masks, temps = [], []
    for f, fr in enumerate(cams):
        fr.index = f
        g = osc.gbuffer(fr, cfg["width"], cfg["height"])
        st.frame(fr, g)
        masks.append(st.probes()["mask"][:st.dims()[0]].copy())
        temps.append(st.temporal())
    return st, masks, temps


def test_static_camera_keeps_every_probe_in_place():
    """same camera in frames 0 and 1: a previous probe is seen at distance 0 from its own
    pixel, so every tile keeps its probe (and the Halton pixel of frame 1 is not used)"""
    cfg = dict(width=64, height=48, rays_per_probe=16, table_log2=14)
    cams = [I.room_camera(0), I.room_camera(0)]
    st, masks, temps = _frames(I.room_scene(), cfg, cams)
    win, hist = temps[1]
    valid = masks[0] != SENT
    assert valid.sum() > 20
    assert np.array_equal(win[valid], masks[0][valid])
    assert np.array_equal(hist[valid], np.nonzero(valid)[0].astype(np.uint32))
    assert np.array_equal(masks[1][valid], masks[0][valid])
    # without temporal reuse frame 1 uses its own jitter: the probes move
    st2, masks2, _ = _frames(I.room_scene(), cfg, [I.room_camera(0), I.room_camera(0)], temporal=0)
    assert not np.array_equal(masks2[1][valid], masks2[0][valid])


def test_sideways_move_by_sixteen_pixels():
    """a floor seen from 10 m above; the camera moves along its right vector by the footprint
    of exactly 16 pixels, so the point seen at pixel x in frame 1 was at x + 16 in frame 0:
    the probe of tile t + 2 reappears 16 pixels left of where it was, in tile t"""
    W, H = 96, 64
    floor = I.Scene(name="floor", verts=np.array([[-100, 0, -100], [100, 0, -100], [100, 0, 100], [-100, 0, 100]],
                                                 np.float32),
                    idx=np.array([[0, 2, 1], [0, 3, 2]], np.uint32), tri_mat=np.zeros(2, np.uint32),
                    materials=np.array([[0.5, 0.5, 0.5, 0, 0, 0]], np.float32), sky=(0.2, 0.2, 0.2))
    h = 10.0
    cam0 = I.look_frame(0, (0.0, h, 0.0), (0.0, -1.0, 0.0), world_up=(0.0, 0.0, 1.0))
    foot = 2.0 * h * cam0.tan_half / H          # metres per pixel at the floor
    d = 16.0 * foot
    cam1 = I.look_frame(1, (0.0 + d * float(cam0.right[0]), h, d * float(cam0.right[2])), (0.0, -1.0, 0.0),
                        world_up=(0.0, 0.0, 1.0))
    assert np.allclose(cam1.right, cam0.right)
    cfg = dict(width=W, height=H, rays_per_probe=16, table_log2=12, sky=floor.sky)
    st, masks, temps = _frames(floor, cfg, [cam0, cam1])
    win, hist = temps[1]
    TW = W // 8
    checked = 0
    for t in range(len(win)):
        tx = t % TW
        if tx + 2 >= TW:
            continue
        m0 = int(masks[0][t + 2])
        assert m0 != SENT
        assert hist[t] == t + 2, (t, hist[t])
        assert win[t] == (((m0 >> 16) << 16) | ((m0 & 0xFFFF) - 16)), (t, hex(win[t]), hex(m0))
        checked += 1
    assert checked == (TW - 2) * (H // 8)


def test_first_frame_has_no_history():
    cfg = dict(width=32, height=32, rays_per_probe=8, table_log2=10)
    st, masks, temps = _frames(I.room_scene(), cfg, [I.room_camera(0)])
    win, hist = temps[0]
    assert (win == SENT).all() and (hist == SENT).all()

"""Pins of the oracle's screen-space denoiser (Section 2.4.3): temporal accumulation with a
capped history and a spatial filter whose radius follows the history length.

- Fixed camera, constant input images c_0, c_1, ...: the history length is f + 1 after frame
  f (capped at dn_hist_max) and the accumulated value is the mean of the inputs so far (after
  the cap, the moving average with weight 1 / cap); the radius is floor(4 / n); the output
  of a constant image is that constant (the filter's weights are normalised).
- Disocclusion: after a sideways camera move, pixels whose previous position falls off the
  screen restart (n = 1, radius 4), the others continue.
- Edges: on a first frame (radius 4), a pixel beside a perpendicular surface takes nothing
  from it (normal weight 0), and a pixel beside a parallel surface at another depth takes it
  with the depth weight cs / (cs + difference), worked out by hand.
- A pixel without a probe keeps its history as it is."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2310_19855_amd import inputs as I


def _room(W=64, H=48, **kw):
    sc = I.room_scene()
    osc = O.OracleScene(sc, f64=True)
    st = O.OracleFrameState(osc, O.default_config(width=W, height=H, denoise=1, **kw))
    return osc, st


def test_running_mean_and_radius_with_a_fixed_camera():
    W, H = 64, 48
    osc, st = _room(W, H, dn_hist_max=4)
    fr = I.room_camera(0)
    g = osc.gbuffer(fr, W, H)
    prim = g[3].reshape(H, W)
    vals = [1.0, 4.0, 2.5, 7.0, 3.0, 6.0]
    mean = None
    for f, v in enumerate(vals):
        fr.index = f
        irr = np.zeros((H, W, 4))
        irr[..., :3] = v
        out = st.denoise(fr, g[0], g[1], prim, irr)
        hist, rad = st.denoise_state()
        n = min(f + 1, 4)
        mean = v if f == 0 else mean + (v - mean) / n
        assert np.all(hist[..., 3] == n), f
        assert np.allclose(hist[..., 0], mean, rtol=1e-12), f
        assert np.all(rad == 4 // n), f
        assert np.allclose(out[..., :3], mean, rtol=1e-12), f
    # the mean of the first four frames (3.625), then weight 1/4: 3.46875, 4.1015625
    assert mean == 4.1015625 and np.all(hist[..., 0] == 4.1015625)


def test_disocclusion_after_a_sideways_move():
    W, H = 64, 48
    osc, st = _room(W, H)
    fr0 = I.room_camera(0)
    g0 = osc.gbuffer(fr0, W, H)
    irr = np.ones((H, W, 4))
    irr[..., 3] = 0
    st.denoise(fr0, g0[0], g0[1], g0[3].reshape(H, W), irr)
    # turn the camera a little: the right edge of the view is new
    fr1 = I.room_camera(0)
    fr1.index = 1
    yaw = math.radians(3.0)
    c, s = math.cos(yaw), math.sin(yaw)
    rot = lambda v: np.array([c * v[0] + s * v[2], v[1], -s * v[0] + c * v[2]], np.float32)
    fr1.fwd, fr1.right, fr1.up = rot(fr1.fwd), rot(fr1.right), rot(fr1.up)
    g1 = osc.gbuffer(fr1, W, H)
    st.denoise(fr1, g1[0], g1[1], g1[3].reshape(H, W), irr)
    hist, rad = st.denoise_state()
    n = hist[..., 3]
    assert (n == 2).mean() > 0.7                     # most pixels continue
    new = n == 1
    assert new.any() and (rad[new] == 4).all()
    # the view turned by 3 degrees (about 4 pixels' worth of the 64 x 60 degree field at this
    # size): a strip on one side restarts entirely
    assert new[:, :3].all() or new[:, -3:].all()


def _planes(W, H, depth_r, normal_r):
    """left half: the plane z = 10 facing the camera (-z), right half: depth depth_r"""
    gpos = np.zeros((H, W, 4))
    gnrm = np.zeros((H, W, 4))
    xs = (np.arange(W) - W / 2 + 0.5) * 0.01
    ys = (np.arange(H) - H / 2 + 0.5) * 0.01
    for y in range(H):
        for x in range(W):
            d = 10.0 if x < W // 2 else depth_r
            gpos[y, x, :3] = (xs[x], ys[y], d)
            gpos[y, x, 3] = d
            gnrm[y, x, :3] = (0.0, 0.0, -1.0) if x < W // 2 else normal_r
    return gpos, gnrm


@pytest.mark.parametrize("case", ["perpendicular", "parallel"])
def test_edge_weights_on_a_first_frame(case):
    W, H = 16, 8
    osc, st = _room(W, H)
    fr = I.Frame(index=0, pos=np.array([0.0, 0.0, 0.0], np.float32), fwd=np.array([0.0, 0.0, 1.0], np.float32),
                 right=np.array([1.0, 0.0, 0.0], np.float32), up=np.array([0.0, 1.0, 0.0], np.float32),
                 fov_y=0.5, tan_half=float(np.float32(math.tan(0.25))))
    if case == "perpendicular":
        gpos, gnrm = _planes(W, H, 10.0, (-1.0, 0.0, 0.0))
    else:
        gpos, gnrm = _planes(W, H, 12.0, (0.0, 0.0, -1.0))
    prim = np.zeros((H, W), np.uint32)
    irr = np.zeros((H, W, 4))
    irr[:, : W // 2, :3] = 1.0
    irr[:, W // 2:, :3] = 5.0
    out = st.denoise(fr, gpos.reshape(-1, 4), gnrm.reshape(-1, 4), prim, irr)
    x, y = W // 2 - 1, H // 2                 # left of the edge; radius 4 reaches 4 columns right
    if case == "perpendicular":
        assert out[y, x, 0] == pytest.approx(1.0, rel=1e-12)
    else:
        kappa = O.distance_scale(0.5, W, H)
        X = gpos[y, x, :3]
        cs = kappa * np.linalg.norm(X)
        w = cs / (cs + 2.0)
        # window rows y-4..y+3 (8 rows: the image), columns x-4..x+4: 5 left, 4 right
        rows = min(H, y + 5) - max(0, y - 4)
        nl, nr = 5 * rows, 4 * rows
        want = (nl * 1.0 + nr * w * 5.0) / (nl + nr * w)
        assert out[y, x, 0] == pytest.approx(want, rel=1e-9)


def test_pixel_without_probe_keeps_its_history():
    W, H = 32, 24
    osc, st = _room(W, H)
    fr = I.room_camera(0)
    g = osc.gbuffer(fr, W, H)
    prim = g[3].reshape(H, W)
    irr = np.full((H, W, 4), 3.0)
    irr[..., 3] = 0
    st.denoise(fr, g[0], g[1], prim, irr)
    irr2 = np.full((H, W, 4), 9.0)
    irr2[..., 3] = 0
    irr2[5, 7, 3] = 2.0                       # no probe here this frame
    fr.index = 1
    st.denoise(fr, g[0], g[1], prim, irr2)
    hist, _ = st.denoise_state()
    assert hist[5, 7, 3] == 1 and hist[5, 7, 0] == 3.0
    assert hist[6, 7, 3] == 2 and hist[6, 7, 0] == 6.0

"""Pins of the oracle's probe-space filter (Algorithm 5: separable 7x7 sparse blur).

Probes are placed through the oracle's own spawn on a synthetic G-buffer: a row of 8x8 tiles
on the floor plane y = 0 (normal +y), every pixel of a tile at the tile's probe position, so
the Halton jitter does not matter.  The camera sits far above, with a field of view that makes
Algorithm 6's cell size large enough to accept coplanar neighbours.  Expected values are
worked out by hand from the algorithm's statement (taps at -1, +1, -2, +2, -3, +3 tiles,
plane and normal rejection, the pi/50 angle test, depth weights, re-averaged hit distance).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2310_19855_amd import inputs as I

NT = 9            # tiles in the row
W, H = 8 * NT, 8


def _frame(fov=0.05, index=0):
    # camera 100 m above the middle of the row, looking down; kappa = tan(fov) for H = 8
    up = np.array([0.0, 0.0, 1.0], np.float32)
    return I.Frame(index=index, pos=np.array([36.0, 100.0, 4.0], np.float32),
                   fwd=np.array([0.0, -1.0, 0.0], np.float32), right=np.array([1.0, 0.0, 0.0], np.float32),
                   up=up, fov_y=fov, tan_half=float(np.float32(math.tan(fov / 2))))


def _state(pos, nrm=None, depth=None, f64=True, sky_tiles=()):
    """oracle state with one probe per tile at pos[k] (x, y, z), normal nrm[k]"""
    pos = np.asarray(pos, np.float64)
    nrm = np.tile([0.0, 1.0, 0.0], (NT, 1)) if nrm is None else np.asarray(nrm, np.float64)
    depth = np.full(NT, 100.0) if depth is None else np.asarray(depth, np.float64)
    gpos = np.zeros((H, W, 4))
    gnrm = np.zeros((H, W, 4))
    prim = np.zeros((H, W), np.uint32)
    for k in range(NT):
        gpos[:, 8 * k:8 * k + 8, :3] = pos[k]
        gpos[:, 8 * k:8 * k + 8, 3] = depth[k]
        gnrm[:, 8 * k:8 * k + 8, :3] = nrm[k]
        if k in sky_tiles:
            prim[:, 8 * k:8 * k + 8] = 0xFFFFFFFF
    sc = O.OracleScene(I.room_scene(), f64=f64)
    st = O.OracleFrameState(sc, O.default_config(width=W, height=H, rays_per_probe=16))
    st.spawn(_frame(), gpos.reshape(-1, 4), gnrm.reshape(-1, 4), prim.reshape(-1))
    return sc, st


def _row(dx=1.0):
    return [[4.0 + dx * (k - 4), 0.0, 4.0] for k in range(NT)]


def _atlas(values, alpha=1e4):
    a = np.zeros((NT, 64, 4))
    for k, v in enumerate(values):
        a[k, :, :3] = v
        a[k, :, 3] = alpha if np.isscalar(alpha) else alpha[k]
    return a


def test_taps_reach_three_tiles_each_way():
    """coplanar probes at equal depth, misses (large hit distance): every neighbour within 3
    tiles contributes with weight 1, so the centre probe gets the mean of 7 and the end
    probes the mean of 4"""
    sc, st = _state(_row())
    v = np.arange(NT, dtype=np.float64) * 10.0 + 1.0
    out = st.filter_atlas(_frame(), 0, _atlas(v))
    assert np.allclose(out[4, :, 0], v[1:8].mean(), rtol=1e-12)
    assert np.allclose(out[0, :, 0], v[0:4].mean(), rtol=1e-12)
    assert np.allclose(out[8, :, 0], v[5:9].mean(), rtol=1e-12)
    assert np.allclose(out[2, :, 0], v[0:6].mean(), rtol=1e-12)


def test_vertical_pass_of_a_single_row_changes_nothing():
    sc, st = _state(_row())
    a = _atlas(np.arange(NT, dtype=np.float64) + 1.0)
    out = st.filter_atlas(_frame(), 1, a)
    assert np.array_equal(out, a)


def test_constant_field_is_invariant():
    """same radiance everywhere: the normalised weighted mean returns it, whatever the
    geometry (depths differ here, so the weights differ)"""
    depth = 100.0 + 3.0 * np.arange(NT)
    sc, st = _state(_row(), depth=depth, f64=False)
    a = _atlas([2.5] * NT)
    out = st.filter_atlas(_frame(), 0, a)
    assert np.allclose(out[..., :3], 2.5, rtol=1e-6)


def test_plane_distance_rejects_a_raised_probe():
    """probe 5 lifted above the plane by more than the cell size (kappa * distance = tan(0.05)
    * ~100 m = 5 m) takes no part in probe 4's mean, and sees no neighbour itself"""
    pos = _row()
    pos[5][1] = 20.0
    sc, st = _state(pos)
    v = np.arange(NT, dtype=np.float64) * 10.0 + 1.0
    out = st.filter_atlas(_frame(), 0, _atlas(v))
    assert np.allclose(out[4, :, 0], np.mean([v[1], v[2], v[3], v[4], v[6], v[7]]), rtol=1e-12)
    assert np.allclose(out[5, :, 0], v[5], rtol=1e-12)


def test_sky_tile_is_skipped_by_the_search():
    """tile 5 has no probe: the tap at +1 from tile 4 finds nothing at MIP 0 and continues
    at MIP 1 from x = 4 / 2 = 2, where x + 1 = 3 covers tiles 6 and 7 and returns the first
    valid one, tile 6; the +2 tap finds tile 6 directly.  Probe 4 therefore averages itself
    with 3, 6, 2, 6, 1, 7"""
    sc, st = _state(_row(), sky_tiles=(5,))
    v = np.arange(NT, dtype=np.float64) * 10.0 + 1.0
    out = st.filter_atlas(_frame(), 0, _atlas(v))
    m = st.probes()["mask"][:NT]
    assert m[5] == 0xFFFFFFFF
    assert st.find_probe(4 * 8, 0, 1, 0) == m[6]
    assert np.allclose(out[4, :, 0], np.mean([v[4], v[3], v[6], v[2], v[6], v[1], v[7]]), rtol=1e-12)


def test_normal_check_rejects_cells_below_the_neighbour():
    """neighbour normals tilted 90 degrees about z (pointing -x): cells whose direction has a
    positive x component point below those surfaces and keep their own value"""
    nrm = np.tile([0.0, 1.0, 0.0], (NT, 1))
    nrm[[3, 5]] = [-1.0, 0.0, 0.0]
    pos = _row()
    sc, st = _state(pos, nrm=nrm)
    v = np.zeros(NT)
    v[3] = v[5] = 100.0
    a = _atlas(v)
    out = st.filter_atlas(_frame(), 0, a)
    # cell direction for a +y normal: local (a, b, z) -> world (a, z, -b) for this basis
    for cell in range(64):
        u = (2 * (cell & 7) + 1) / 8 - 1
        w = (2 * (cell >> 3) + 1) / 8 - 1
        ax = (u + w) / 2
        if ax > 0:          # points along +x: below the -x surfaces of probes 3 and 5
            assert out[4, cell, 0] == 0.0, cell
    assert (out[4, :, 0] > 0).any()


def test_angle_threshold_hand_case():
    """cell 27 of a +y probe points along (-1, 7, 0)/sqrt(50).  A neighbour 1 m along +x with
    hit distance h is accepted iff the angle between the cell direction and (offset + h dir)
    is within pi/50: tan = (7/sqrt(50)) / (h - 1/sqrt(50)) <= tan(pi/50), i.e. h >= 15.88 m"""
    pos = _row(1.0)
    sc, st = _state(pos)
    v = np.zeros(NT)
    v[5] = 100.0
    for h, accepted in ((20.0, True), (12.0, False)):
        alpha = np.full(NT, 1e4)
        alpha[5] = h
        out = st.filter_atlas(_frame(), 0, _atlas(v, alpha))
        # probe 4, cell 27: neighbour 5 at +1 m (the others have zero radiance, miss distance)
        assert (out[4, 27, 0] > 0) == accepted, h
    tan_t = math.tan(math.pi / 50)
    h0 = 7 / math.sqrt(50) / tan_t + 1 / math.sqrt(50)
    assert 15.8 < h0 < 15.95


def test_depth_weight_reading_and_hit_distance_average():
    """READING of the undefined depth weight: cs / (cs + |d_q - d_p|).  Probe 4 with one
    accepted neighbour (5) at depth difference equal to its cell size gets weight 1/2; the
    travelled distance is averaged with the neighbour's clamped distance the same way"""
    pos = _row()
    depth = np.full(NT, 100.0)
    kappa = math.tan(0.05)
    cam = np.array([36.0, 100.0, 4.0])
    cs = kappa * float(np.linalg.norm(np.array(pos[4]) - cam))
    depth[5] = 100.0 + cs
    sc, st = _state(pos, depth=depth)
    # only probe 5 contributes to probe 4: the others are lifted out of the plane
    for k in (1, 2, 3, 6, 7):
        pos[k][1] = 50.0
    sc, st = _state(pos, depth=depth)
    v = np.zeros(NT)
    v[4], v[5] = 3.0, 9.0
    alpha = np.full(NT, 1e4)
    alpha[4], alpha[5] = 40.0, 30.0
    out = st.filter_atlas(_frame(), 0, _atlas(v, alpha))
    w = cs / (cs + cs)
    assert np.allclose(out[4, :, 0], (3.0 + w * 9.0) / (1 + w), rtol=1e-9)
    assert np.allclose(out[4, :, 3], (40.0 + w * 30.0) / (1 + w), rtol=1e-9)


def test_isolated_probe_is_unchanged():
    pos = _row()
    for k in range(NT):
        if k != 4:
            pos[k][1] = 50.0 + k
    sc, st = _state(pos)
    a = _atlas(np.arange(NT) + 1.0, alpha=np.arange(NT) + 5.0)
    out = st.filter_atlas(_frame(), 0, a)
    assert np.array_equal(out[4], a[4])


@pytest.mark.parametrize("f64", [False, True])
def test_frame_with_filter_keeps_energy_of_a_uniform_room(f64):
    """whole oracle frame with the filter on, room scene: filtering only redistributes cell
    values, so the mean atlas radiance over probes stays within a few percent of the
    unfiltered frame's"""
    sc = I.room_scene()
    osc = O.OracleScene(sc, f64=f64)
    fr = I.room_camera(0)
    means = []
    for pf in (0, 1):
        st = O.OracleFrameState(osc, O.default_config(width=64, height=64, rays_per_probe=16, probe_filter=pf))
        g = osc.gbuffer(fr, 64, 64)
        st.frame(fr, g)
        p = st.probes()
        valid = p["mask"][:len(p["pos"])] != 0xFFFFFFFF
        means.append(p["atlas"][valid][..., :3].mean())
    assert abs(means[1] / means[0] - 1) < 0.05

"""Pins of the oracle's ray guiding (Section 2.1.2): the parallax-corrected reconstruction of a
new probe's hemisphere from the previous frame's probes, and sampling in proportion to it.

- The cell pick is an integer inverse CDF: hand cases fix which cell a 32-bit number picks.
- A guided direction is a uniform point of the picked cell's square in the hemi-octahedral
  domain: for the normals +z and -z (whose orthonormal bases are the axes, up to sign) the
  direction's own square coordinates, worked out from the mapping's definition, are the
  point that was asked for.
- Reconstruction: a previous probe at the new probe's own position and normal gives every
  cell back to itself with its distance; a probe one metre to the side sends each of its
  cells to the cell of the direction from the new probe to the cell's hit point, worked out
  here from the geometry (the parallax), and the distances become the lengths from the new
  probe; probes that fail the plane or normal test give nothing.
- Whole frames: the rays keep their count and fall only into cells of positive weight, and
  with guiding the temporal irradiance stays near the per-frame estimate's level, which
  Algorithm 3's darkening bias pulls the unguided temporal estimate well below."""
import numpy as np
import pytest

import oracle as O
from paper_2310_19855_amd import inputs as I

SENT = 0xFFFFFFFF


def test_cell_pick_hand_cases():
    cdf = np.zeros(64, np.uint32)
    cdf[10:] = 1
    cdf[40:] = 4            # weights: cell 10 -> 1, cell 40 -> 3
    r = np.array([0, (1 << 30) - 1, 1 << 30, (1 << 32) - 1, 3 << 30], np.uint32)
    _, cell = O.guided_dirs([0.0, 0.0, 1.0], cdf, r, np.full(5, 0.5), np.full(5, 0.5), f64=True)
    assert cell.tolist() == [10, 10, 40, 40, 40]
    # equal weights: r = k * 2^26 picks cell k exactly
    cdf = np.arange(1, 65, dtype=np.uint32)
    r = (np.arange(64, dtype=np.uint64) << 26).astype(np.uint32)
    _, cell = O.guided_dirs([0.0, 0.0, 1.0], cdf, r, np.full(64, 0.5), np.full(64, 0.5), f64=True)
    assert cell.tolist() == list(range(64))


def _square_coords(lx, ly, lz):
    s = np.abs(lx) + np.abs(ly) + lz
    a, b = lx / s, ly / s
    return a + b, a - b


@pytest.mark.parametrize("nz", [1.0, -1.0])
def test_guided_direction_is_the_asked_point_of_its_cell(nz):
    rng = np.random.default_rng(4)
    n = 4000
    cells = rng.integers(0, 64, n).astype(np.uint32)
    cdf = np.zeros(64, np.uint32)
    u0, u1 = rng.uniform(0, 1, n), rng.uniform(0, 1, n)
    d = np.zeros((n, 3))
    for k in range(64):
        sel = np.nonzero(cells == k)[0]
        if not len(sel):
            continue
        cdf[:] = 0
        cdf[k:] = 1
        dd, c = O.guided_dirs([0.0, 0.0, nz], cdf, np.zeros(len(sel), np.uint32), u0[sel], u1[sel], f64=True)
        assert (c == k).all()
        d[sel] = dd
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
    # normal +z: basis x, y; normal -z: basis x, -y (local z along the normal)
    lx, ly, lz = d[:, 0], d[:, 1] * nz, d[:, 2] * nz
    assert (lz >= 0).all()
    uu, vv = _square_coords(lx, ly, lz)
    assert np.allclose(uu, ((cells & 7) + u0) / 4 - 1, atol=1e-12)
    assert np.allclose(vv, ((cells >> 3) + u1) / 4 - 1, atol=1e-12)


def _cell_of(lx, ly, lz):
    uu, vv = _square_coords(lx, ly, lz)
    ix = np.clip(np.floor(4 * (uu + 1)), 0, 7).astype(int)
    iy = np.clip(np.floor(4 * (vv + 1)), 0, 7).astype(int)
    return 8 * iy + ix


def _centre_local(c):
    """unit local direction of the centre of atlas cell c (hemi-octahedral square)"""
    uu = (2 * (c & 7) + 1) / 8 - 1
    vv = (2 * (c >> 3) + 1) / 8 - 1
    a, b = (uu + vv) / 2, (uu - vv) / 2
    z = 1 - abs(a) - abs(b)
    L = np.sqrt(a * a + b * b + z * z)
    return a / L, b / L, z / L


def _atlas(vals, dist):
    a = np.zeros((64, 4))
    a[:, 0] = vals
    a[:, 1] = vals
    a[:, 2] = vals
    a[:, 3] = dist
    return a


UP = [0.0, 1.0, 0.0, 0.0]


def test_same_probe_gives_every_cell_back():
    vals = np.arange(64, dtype=np.float64) + 1.0
    recon, cdf = O.reconstruct_probe(np.zeros(3), np.array(UP), 0.5, [[0, 0, 0, 0]], [UP], [_atlas(vals, 3.0)])
    assert np.allclose(recon[:, 0], vals, rtol=1e-12)
    assert np.allclose(recon[:, 3], 3.0, rtol=1e-12)
    w = np.diff(np.concatenate([[0], cdf.astype(np.int64)]))
    assert w[63] == 1 << 20
    want = np.floor(vals / 64.0 * (1 << 20))
    assert (np.abs(w - want) <= 1).all() and (np.diff(w) > 0).all()


@pytest.mark.parametrize("h", [0.7, 2.0, 9.0])
def test_parallax_of_a_probe_one_metre_aside(h):
    """previous probe q at (1, 0, 0), new probe p at the origin, both facing +y.  For +y the
    orthonormal basis is t = +x, b = -z, so a local direction (a, b, z) is the world vector
    (a, z, -b), and a world vector v is local (v_x, -v_z, v_y).  q's cell c with travelled
    distance h was hit at q + h * centre(c); p sees it along v = (1, 0, 0) + h * centre(c)."""
    vals = np.arange(64, dtype=np.float64) + 1.0
    recon, _ = O.reconstruct_probe(np.zeros(3), np.array(UP), 0.5, [[1, 0, 0, 0]], [UP], [_atlas(vals, h)])
    sums, cnt, dsum = np.zeros(64), np.zeros(64), np.zeros(64)
    for c in range(64):
        a, b, z = _centre_local(c)
        v = np.array([1.0 + h * a, h * z, -h * b])
        lx, ly, lz = v[0], -v[2], v[1]
        assert lz > 0
        k = _cell_of(np.array([lx]), np.array([ly]), np.array([lz]))[0]
        sums[k] += vals[c]
        dsum[k] += np.linalg.norm(v)
        cnt[k] += 1
    full = cnt > 0
    assert np.allclose(recon[full, 0], sums[full] / cnt[full], rtol=1e-12)
    assert np.allclose(recon[full, 3], dsum[full] / cnt[full], rtol=1e-12)
    assert (recon[~full, 3] == -1).all()
    if h < 1:
        # a close hit point moves far in direction: the cells really are remapped
        assert not np.allclose(recon[full, 0], vals[full])


def test_rejected_previous_probes_give_nothing():
    vals = np.ones(64)
    # lifted above p's plane by more than the cell size
    recon, cdf = O.reconstruct_probe(np.zeros(3), np.array(UP), 0.5, [[0, 0.6, 0, 0]], [UP], [_atlas(vals, 2.0)])
    assert (recon[:, 3] == -1).all() and cdf[63] == 0
    # normal 20 degrees away (cosine 0.94 < 0.95)
    t = np.radians(20.0)
    n = [np.sin(t), np.cos(t), 0.0, 0.0]
    recon, cdf = O.reconstruct_probe(np.zeros(3), np.array(UP), 0.5, [[0, 0, 0, 0]], [n], [_atlas(vals, 2.0)])
    assert (recon[:, 3] == -1).all() and cdf[63] == 0
    # 15 degrees (0.966) is accepted
    t = np.radians(15.0)
    n = [np.sin(t), np.cos(t), 0.0, 0.0]
    recon, cdf = O.reconstruct_probe(np.zeros(3), np.array(UP), 0.5, [[0, 0, 0, 0]], [n], [_atlas(vals, 2.0)])
    assert (recon[:, 3] > 0).sum() > 40 and cdf[63] > 0
    # no candidates at all
    recon, cdf = O.reconstruct_probe(np.zeros(3), np.array(UP), 0.5, [], [], [])
    assert (recon[:, 3] == -1).all() and cdf[63] == 0


def _frames(guiding, frames=4, W=64, H=48, R=32, temporal=1):
    sc = I.room_scene()
    osc = O.OracleScene(sc, f64=False)
    cfg = O.default_config(width=W, height=H, rays_per_probe=R, table_log2=15, temporal=temporal,
                           ray_guiding=guiding, bounces=2)
    st = O.OracleFrameState(osc, cfg)
    fr = I.room_camera(0)
    out = []
    for f in range(frames):
        fr.index = f
        g = osc.gbuffer(fr, W, H)
        st.spawn(fr, g[0], g[1], g[3])
        recon, cdf = st.guiding()
        st.trace(fr)
        rays = st.rays()
        st.update(fr)
        pr = st.probes()
        irr = st.interpolate(fr, g[0], g[1], g[3])
        out.append(dict(cdf=cdf.copy(), cell=rays["cell"].copy(), mask=pr["mask"][:st.P].copy(),
                        irr=float(irr[..., :3].mean()), rays=st.stats()["rays"]))
    return st, out


def test_guided_frames_room():
    st, g = _frames(1)
    _, u = _frames(0)
    R = 32
    for f in range(4):
        assert g[f]["rays"] == u[f]["rays"]
        valid = g[f]["mask"] != SENT
        guided = valid & (g[f]["cdf"][:, 63] > 0)
        if f == 0:
            assert not guided.any()
            continue
        assert guided.sum() > 0.9 * valid.sum()
        cells = (g[f]["cell"] & 63).reshape(-1, R)
        w = np.diff(np.concatenate([np.zeros((len(valid), 1), np.int64), g[f]["cdf"].astype(np.int64)], 1), axis=1)
        for p in np.nonzero(guided)[0]:
            assert (w[p, cells[p]] > 0).all(), p


def test_guiding_keeps_the_level_that_hysteresis_darkens():
    """Algorithm 3 is biased towards darkening (the paper accepts some darkening to keep
    shadows); with noisy per-cell estimates the unguided temporal irradiance falls well below
    the per-frame estimate's.  Guided rays cut the noise of the bright cells, and the level
    stays near the per-frame estimate's (room, fixed camera, 64 rays, frames 2-5)"""
    fr = slice(2, 6)
    lvl = {}
    for name, guiding, temporal in (("frame", 0, 0), ("unguided", 0, 1), ("guided", 1, 1)):
        _, o = _frames(guiding, frames=6, R=64, temporal=temporal)
        lvl[name] = np.mean([x["irr"] for x in o[fr]])
    assert abs(lvl["guided"] / lvl["frame"] - 1) < 0.15, lvl
    assert lvl["unguided"] < 0.8 * lvl["frame"], lvl

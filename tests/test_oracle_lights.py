"""Pins of the oracle's light grid and resampled light sampling (Section 2.3: RIS with
weighted reservoir sampling over candidates from the light grid of Section 2.3.2).

- RIS is unbiased when the cell's list holds every light: the mean of many estimates at a
  point equals the sum of Lambert's polygon irradiance over two quads of different radiance
  (one candidate: a uniform light pick; four candidates: resampling), within 5 standard errors.
- Grid geometry: cubic cells, the longest axis split into lgrid_dim, the others rounded up.
- Lists: a light facing away from a cell (the cell's bounding sphere behind its plane) and a
  light out of range (its range from the threshold) are culled; the cell under a light lists
  it first; lists are ordered by importance, at most lgrid_k long.
- Whole frames on the many-light room: the rays and hits do not change, every shadow ray
  comes from a hit, and the radiance level agrees with area-proportional sampling."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2310_19855_amd import inputs as I

from test_oracle_geometry import _lambert_polygon, _tri_scene


def _quad(cx, y, cz, half, down=True):
    q = np.array([[cx - half, y, cz - half], [cx + half, y, cz - half], [cx + half, y, cz + half],
                  [cx - half, y, cz + half]])
    return q, ([q[[0, 1, 2]], q[[0, 2, 3]]] if down else [q[[0, 2, 1]], q[[0, 3, 2]]])


@pytest.mark.parametrize("m", [1, 4])
def test_ris_is_unbiased_with_full_lists(m):
    qa, ta = _quad(0.0, 2.0, 0.0, 0.5)
    qb, tb = _quad(1.5, 2.5, 0.5, 0.25)
    sc = _tri_scene(ta + tb, [[0, 0, 0, 10, 10, 10]] * 2 + [[0, 0, 0, 40, 20, 10]] * 2)
    osc = O.OracleScene(sc, f64=True)
    st = O.OracleFrameState(osc, O.default_config(light_grid=1, lgrid_dim=4, lgrid_k=8, ris_candidates=m, lgrid_threshold=1e-9))
    st.light_grid_set([-2.0, -1.0, -2.0], [2.0, 3.0, 2.0])
    g = st.light_grid()
    p = np.array([0.3, 0.0, -0.2])
    i = [int(np.floor((v - o) / g["h"])) for v, o in zip(p, g["lo"])]
    c = (i[2] * g["dims"][1] + i[1]) * g["dims"][0] + i[0]
    assert g["count"][c] == 4                   # the point's cell lists all four triangles
    n = np.array([0.1, 1.0, 0.05])
    n = n / np.linalg.norm(n)
    ids = np.arange(300000, dtype=np.uint32)
    e = st.nee(I.room_camera(0), p, n, ids)
    for ch, (la, lb) in enumerate(((10, 40), (10, 20), (10, 10))):
        exact = (_lambert_polygon(p, n, qa, la) + _lambert_polygon(p, n, qb, lb)) / math.pi
        x = e[:, ch]
        assert abs(x.mean() - exact) < 5 * x.std() / math.sqrt(len(x)), (ch, x.mean(), exact)


def test_grid_geometry():
    qa, ta = _quad(0.0, 2.0, 0.0, 0.5)
    sc = _tri_scene(ta, [[0, 0, 0, 10, 10, 10]] * 2)
    st = O.OracleFrameState(O.OracleScene(sc, f64=True), O.default_config(light_grid=1, lgrid_dim=16, lgrid_k=4))
    st.light_grid_set([0.0, 0.0, 0.0], [10.0, 5.0, 2.5])
    g = st.light_grid()
    assert g["h"] == 0.625 and g["dims"].tolist() == [16, 8, 4]
    st.light_grid_set([1.0, 1.0, 1.0], [1.0, 1.0, 1.0])     # a single point: one cell of side 1
    g = st.light_grid()
    assert g["h"] == 1.0 and g["dims"].tolist() == [1, 1, 1]


def test_culling_and_order():
    # light A at x = -3 facing down, light B at x = +3 facing up, both at y = 2
    qa, ta = _quad(-3.0, 2.0, 0.0, 0.25, down=True)
    qb, tb = _quad(3.0, 2.0, 0.0, 0.25, down=False)
    sc = _tri_scene(ta + tb, [[0, 0, 0, 20, 20, 20]] * 2 + [[0, 0, 0, 20, 20, 20]] * 2)
    cfg = O.default_config(light_grid=1, lgrid_dim=8, lgrid_k=8, lgrid_threshold=1e-6)
    st = O.OracleFrameState(O.OracleScene(sc, f64=True), cfg)
    st.light_grid_set([-4.0, -2.5, -4.0], [4.0, 5.5, 4.0])      # cells of 1 m, y from -2.5
    g = st.light_grid()
    D = g["dims"]
    assert D.tolist() == [8, 8, 8]

    def cell(x, y, z):
        i = [int(np.floor((v - o) / g["h"])) for v, o in zip((x, y, z), g["lo"])]
        return (i[2] * D[1] + i[1]) * D[0] + i[0]

    def lights(x, y, z):
        c = cell(x, y, z)
        return g["list"][c, :g["count"][c]].tolist()
    # under A (cell y in [-1.5, -0.5]): A's two triangles; B faces up and its plane y = 2 lies
    # above the whole cell (sphere radius 0.87): culled
    low_a = lights(-3.0, -1.5, 0.5)
    assert sorted(low_a) == [0, 1]
    # above B (cell y in [4.5, 5.5]): B listed, A faces down and the cell lies above its plane
    assert sorted(lights(3.0, 5.0, 0.5)) == [2, 3]
    # the cell y in [1.5, 2.5] straddles both planes: corners in front of each light; A is
    # 0.7 m away, B 5.5 m, so A's triangles come first
    both = lights(-2.5, 2.0, 0.5)
    assert set(both) == {0, 1, 2, 3} and set(both[:2]) == {0, 1}
    # a tiny range (large threshold) culls the far light: the threshold makes sqrt(phi / tau) 1 m
    phi = 20.0 * 0.5 * 0.5 / 2          # luminance 20, area 0.125 per triangle
    st2 = O.OracleFrameState(O.OracleScene(sc, f64=True), dict(cfg, lgrid_threshold=phi))
    st2.light_grid_set([-4.0, -2.5, -4.0], [4.0, 5.5, 4.0])
    g2 = st2.light_grid()
    c = cell(-3.0, -1.5, 0.5)
    assert g2["count"][c] == 0                   # 3.1 m below A: beyond 1 m + 0.87 m
    c = cell(-3.0, 2.0, 0.5)
    assert sorted(g2["list"][c, :g2["count"][c]].tolist()) == [0, 1]


def test_lists_are_ordered_and_capped():
    sc = I.lights_room_scene()
    cfg = O.default_config(light_grid=1, lgrid_dim=6, lgrid_k=5)
    st = O.OracleFrameState(O.OracleScene(sc, f64=True), cfg)
    st.light_grid_set([0.0, 0.0, 0.0], [6.0, 3.0, 6.0])
    g = st.light_grid()
    # 64 lights on the walls and ceiling: every 1 m cell of the room has at least 5 in front
    # of it and within range, and keeps exactly 5, all distinct
    assert g["dims"].tolist() == [6, 3, 6]
    assert (g["count"] == 5).all()
    assert all(len(set(row.tolist())) == 5 for row in g["list"])


def _frames(sc, light_grid, frames=3, W=64, H=48, R=32):
    osc = O.OracleScene(sc, f64=False)
    cfg = O.default_config(width=W, height=H, rays_per_probe=R, table_log2=15, light_grid=light_grid,
                           lgrid_dim=8, lgrid_k=16, ris_candidates=4)
    st = O.OracleFrameState(osc, cfg)
    fr = I.room_camera(0)
    irr = []
    for f in range(frames):
        fr.index = f
        g = osc.gbuffer(fr, W, H)
        out = st.frame(fr, g)
        irr.append(float(out[..., :3].mean()))
    return st, irr


def test_frames_on_the_many_light_room():
    sc = I.lights_room_scene()
    st_r, irr_r = _frames(sc, 1)
    st_a, irr_a = _frames(sc, 0)
    sr, sa = st_r.stats(), st_a.stats()
    assert sr["rays"] == sa["rays"] and sr["hits"] == sa["hits"]
    assert 0 < sr["shadow"] <= sr["hits"]
    assert abs(np.mean(irr_r) / np.mean(irr_a) - 1) < 0.15, (irr_r, irr_a)


# --- world-space reservoir reuse (Section 2.3.1) -------------------------------------------

def _restir_frames(sc, restir, frames, W=64, H=48, R=16, m=4):
    osc = O.OracleScene(sc, f64=False)
    cfg = O.default_config(width=W, height=H, rays_per_probe=R, table_log2=15, light_grid=1, lgrid_dim=8,
                           lgrid_k=128, ris_candidates=m, restir=restir, restir_log2=15)
    st = O.OracleFrameState(osc, cfg)
    fr = I.room_camera(0)
    out = []
    for f in range(frames):
        fr.index = f
        g = osc.gbuffer(fr, W, H)
        st.spawn(fr, g[0], g[1], g[3])
        st.trace(fr)
        res = st.reservoirs() if restir else None
        st.update(fr)
        irr = st.interpolate(fr, g[0], g[1], g[3])
        out.append(dict(res=res, irr=float(irr[..., :3].mean())))
    return st, out


def test_reservoirs_accumulate_counts_up_to_the_cap():
    """frame 0 has nothing to reuse: every stored reservoir holds the 4 candidates of its
    hit; from frame 1 on the stored counts grow by reuse, and never pass 4 + 20 * 4"""
    sc = I.lights_room_scene()
    st, out = _restir_frames(sc, 1, 6)
    r0 = out[0]["res"]
    assert len(r0["M"]) > 20 and (r0["M"] == 4).all()
    assert np.allclose(np.linalg.norm(r0["n"], axis=1), 1.0, atol=1e-5)
    assert (r0["W"] > 0).all() and (r0["k"] < 128).all()
    grown = [o["res"]["M"].max() for o in out[1:]]
    assert grown[0] > 4 and max(grown) <= 84 and grown[-1] >= grown[0]
    # one reservoir per quantised position: keys are distinct and keep no normal class bits
    k = out[-1]["res"]["key"]
    assert len(np.unique(k)) == len(k) and ((k >> np.uint64(54)) & np.uint64(0xF) == 0).all()


def test_reservoir_reuse_keeps_the_radiance_level():
    """reuse resamples the same target (unshadowed contribution), so the irradiance level
    over frames stays that of RIS alone (within the noise of a few frames)"""
    sc = I.lights_room_scene()
    _, on = _restir_frames(sc, 1, 6)
    _, off = _restir_frames(sc, 0, 6)
    a = np.mean([o["irr"] for o in on[2:]])
    b = np.mean([o["irr"] for o in off[2:]])
    assert abs(a / b - 1) < 0.1, (a, b)

"""Pins of the oracle's ray queries, G-buffer, emitter sampling and next-event estimation:
brute force, closed-form geometry, watertightness, and Lambert's polygon irradiance."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2310_19855_amd import inputs as I


def _tri_scene(tris, mats=None):
    tris = np.asarray(tris, np.float32).reshape(-1, 3, 3)
    n = len(tris)
    mats = np.array([[0.5, 0.5, 0.5, 0, 0, 0]] * n if mats is None else mats, np.float32)
    return I.Scene("t", verts=tris.reshape(-1, 3), idx=np.arange(3 * n, dtype=np.uint32).reshape(-1, 3),
                   tri_mat=np.arange(n, dtype=np.uint32) if len(mats) == n else np.zeros(n, np.uint32),
                   materials=mats)


def test_hand_triangle_exact_distance():
    sc = O.OracleScene(_tri_scene([[-1, -1, 1], [1, -1, 1], [0, 1, 1]]))
    tri, t = sc.closest(np.zeros((1, 3)), np.array([[0, 0, 1.0]]))
    assert tri[0] == 0 and t[0] == np.float32(1.0)
    # behind the origin and parallel rays miss; t > 0 strictly
    tri, t = sc.closest(np.array([[0, 0, 1.0], [0, 0, 2.0], [0, 0, 0.0]]),
                        np.array([[0, 0, 1.0], [0, 0, 1.0], [1.0, 0, 0]]))
    assert (tri == 0xFFFFFFFF).all()
    # any-hit respects the open interval (0, tmax)
    assert sc.any(np.zeros((2, 3)), np.array([[0, 0, 1.0]] * 2), np.array([1.0, 1.0001]))[0] == 0
    assert sc.any(np.zeros((1, 3)), np.array([[0, 0, 1.0]]), np.array([1.0001]))[0] == 1


def test_shared_edge_goes_to_lower_index_and_is_watertight():
    # two triangles sharing the edge x = 0 of the z = 2 plane; the duplicate of triangle 0
    # (index 2) ties exactly and must lose to index 0
    tris = [[[0, -1, 2], [0, 1, 2], [-1, 0, 2]], [[0, 1, 2], [0, -1, 2], [1, 0, 2]],
            [[0, -1, 2], [0, 1, 2], [-1, 0, 2]]]
    sc = O.OracleScene(_tri_scene(tris))
    ys = np.linspace(-0.9, 0.9, 181).astype(np.float32)
    o = np.stack([np.zeros_like(ys), ys, np.zeros_like(ys)], 1)
    d = np.tile([0, 0, 1.0], (len(ys), 1))
    tri, t = sc.closest(o, d)
    assert (tri != 0xFFFFFFFF).all() and (t == np.float32(2.0)).all()
    assert set(np.unique(tri)) <= {0, 1}


def test_closed_mesh_has_no_leaks():
    v, f = I.uv_sphere(5.0, 64, 64, inward=True)
    sc = I.Scene("s", verts=v.astype(np.float32), idx=f.astype(np.uint32),
                 tri_mat=np.zeros(len(f), np.uint32), materials=np.array([[0.5] * 3 + [0] * 3], np.float32))
    o_, d_ = I.random_rays(100000, -2.8, 2.8, seed=21)   # |o| < 4.9: inside
    osc = O.OracleScene(sc, use_bvh=True)
    tri, t = osc.closest(o_, d_)
    assert (tri != 0xFFFFFFFF).all()
    # distances agree with the float64 chord length to the polyhedron within its sagitta
    p = o_.astype(np.float64) + t[:, None] * d_.astype(np.float64)
    r = np.linalg.norm(p, axis=1)
    sag = 5.0 * (1 - math.cos(math.pi / 64)) * 2.5
    assert (r <= 5.0 + 1e-4).all() and (r >= 5.0 - sag).all()


def test_bvh_equals_brute_force_room_and_field_subset():
    sc = I.room_scene()
    a = O.OracleScene(sc, use_bvh=False)
    b = O.OracleScene(sc, use_bvh=True)
    o, d = I.random_rays(20000, 0.1, 2.9, seed=3)
    ta, tta = a.closest(o, d)
    tb, ttb = b.closest(o, d)
    assert (ta == tb).all() and (tta.view(np.uint32) == ttb.view(np.uint32)).all()
    tm = np.full(len(o), 2.0, np.float32)
    assert (a.any(o, d, tm) == b.any(o, d, tm)).all()
    # a 60k-triangle window of the field scene
    f = I.field_scene(n_boxes=4000, n_spheres=8)
    a = O.OracleScene(f, use_bvh=False)
    b = O.OracleScene(f, use_bvh=True)
    o, d = I.random_rays(3000, [-30, 0.2, -30], [30, 4, 30], seed=4)
    ta, tta = a.closest(o, d)
    tb, ttb = b.closest(o, d)
    assert (ta == tb).all() and (tta.view(np.uint32) == ttb.view(np.uint32)).all()


def test_gbuffer_brute_force_room():
    sc = I.room_scene()
    fr = I.room_camera(0)
    ga = O.OracleScene(sc, use_bvh=False).gbuffer(fr, 128, 128)
    gb = O.OracleScene(sc, use_bvh=True).gbuffer(fr, 128, 128)
    for x, y in zip(ga, gb):
        assert np.array_equal(x.view(np.uint32) if x.dtype != np.uint32 else x,
                              y.view(np.uint32) if y.dtype != np.uint32 else y)
    pos, nrm, alb, prim = ga
    assert (prim != 0xFFFFFFFF).all()             # closed room
    assert (pos[..., :3] >= -1e-4).all() and (pos[..., 0] <= 6 + 1e-4).all()
    # face-forwarded normals point back towards the camera
    view = pos[..., :3] - fr.pos
    assert ((view * nrm[..., :3]).sum(-1) <= 1e-6).all()
    # the pixel-centre ray of a centred square image hits the wall straight ahead at the
    # float64 plane distance
    d = fr.fwd.astype(np.float64)
    ts = [((6.0 if d[k] > 0 else 0.0) - fr.pos[k]) / d[k] for k in range(3) if abs(d[k]) > 1e-9]
    tmin = min(t for t in ts if t > 0)
    assert pos[..., 3].max() > 0 and pos[..., 3].min() < tmin + 1e-3


def test_emitter_selection_proportional_to_area():
    # 4 emitters of areas 1, 2, 3, 4 (right triangles with legs sqrt(2a))
    tris, mats = [], []
    for a in (1.0, 2.0, 3.0, 4.0):
        l = math.sqrt(2 * a)
        tris.append([[0, 0, 0], [l, 0, 0], [0, l, 0]])
    mats = [[0, 0, 0, 1, 1, 1]] * 4
    sc = O.OracleScene(_tri_scene(tris, mats))
    etri, ethr, area = sc.emitters()
    assert abs(area - 10.0) < 1e-5
    assert list(etri) == [0, 1, 2, 3] and ethr[-1] == 0xFFFFFFFF
    # exact preimage sizes of the threshold table
    edges = np.concatenate([[0], ethr.astype(np.float64)])
    frac = np.diff(edges) / 2**32
    assert np.allclose(frac, [0.1, 0.2, 0.3, 0.4], atol=1e-9)
    rng = np.random.default_rng(0)
    picks = [sc.pick_emitter(int(r)) for r in rng.integers(0, 2**32, 20000)]
    hist = np.bincount(picks, minlength=4) / 20000
    assert np.allclose(hist, [0.1, 0.2, 0.3, 0.4], atol=0.015)
    assert sc.pick_emitter(0) == 0 and sc.pick_emitter(0xFFFFFFFF) == 3


def _lambert_polygon(p, n, verts, le):
    """irradiance from a uniform polygonal emitter (Lambert's formula)"""
    u = [(v - p) / np.linalg.norm(v - p) for v in verts]
    s = 0.0
    for i in range(len(u)):
        a, b = u[i], u[(i + 1) % len(u)]
        g = np.cross(a, b)
        s += math.acos(np.clip(a @ b, -1, 1)) * (n @ (g / np.linalg.norm(g)))
    return 0.5 * le * abs(s)


@pytest.mark.parametrize("p,n", [((0.2, 0.0, -0.3), (0.0, 1.0, 0.0)),
                                 ((1.5, 0.5, 0.7), (-0.3, 0.9, -0.2))])
def test_nee_matches_lambert_polygon_formula(p, n):
    # one 1x1 quad at y = 2, facing down, Le = 10
    quad = np.array([[-0.5, 2.0, -0.5], [0.5, 2.0, -0.5], [0.5, 2.0, 0.5], [-0.5, 2.0, 0.5]])
    tris = [quad[[0, 1, 2]], quad[[0, 2, 3]]]
    sc = _tri_scene(tris, [[0, 0, 0, 10, 10, 10]] * 2)
    osc = O.OracleScene(sc, f64=True)
    st = O.OracleFrameState(osc, O.default_config())
    n = np.array(n) / np.linalg.norm(n)
    ids = np.arange(400000, dtype=np.uint32)
    e = st.nee(I.room_camera(0), np.array(p, np.float64), n, ids)[:, 0]
    exact = _lambert_polygon(np.array(p), n, quad, 10.0) / math.pi
    assert abs(e.mean() - exact) < 5 * e.std() / math.sqrt(len(e)) + 1e-9
    assert abs(e.mean() / exact - 1) < 5e-3


def test_nee_shadow_ray_occlusion():
    quad = np.array([[-0.5, 2.0, -0.5], [0.5, 2.0, -0.5], [0.5, 2.0, 0.5], [-0.5, 2.0, 0.5]])
    blocker = np.array([[-5, 1.0, -5], [5, 1.0, -5], [0, 1.0, 5]])
    sc = _tri_scene([quad[[0, 1, 2]], quad[[0, 2, 3]], blocker],
                    [[0, 0, 0, 10, 10, 10]] * 2 + [[0.5, 0.5, 0.5, 0, 0, 0]])
    st = O.OracleFrameState(O.OracleScene(sc), O.default_config())
    e = st.nee(I.room_camera(0), np.zeros(3, np.float32), np.array([0, 1, 0], np.float32),
               np.arange(1000, dtype=np.uint32))
    assert (e == 0).all()

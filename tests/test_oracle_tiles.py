"""Pins of the oracle's two-level world cache (Section 2.2.3, prefiltering): tiles of 8x8 2D
cells indexed by projecting along the normal's main axis, and MIP levels that answer queries
from the finest level holding enough samples.

- Tile descriptor: the tiled key of a point equals the single-level key of the point whose
  quantised position is the tile's (floor division by 8), so the tile layout reuses the
  checked descriptor; the in-tile cell is the remainder modulo 8 along the two axes other than
  the main one, checked by hand for each main axis and negative coordinates; points that
  differ along the main axis inside a tile share their cell.
- MIP levels and the level choice: hand cases (sample-weighted 2x2 means, the fallback to
  coarser levels, the coarsest level when no level has enough samples), the constant tile.
- Whole frames: the furnace closed forms hold with tiles (one bounce: every probe ray returns
  Le + rho Le; the feedback recurrence L_f = rho (Le + L_{f-1})), and the per-cell fixed-point
  counts add up to the hits."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2310_19855_amd import inputs as I

SENT = 0xFFFFFFFF


def _cfg(**kw):
    return O.default_config(cell_scale=1.0, leak_bit=0, **kw)


@pytest.mark.parametrize("normal,axes", [((0.0, 0.0, 1.0), (0, 1)), ((1.0, 0.0, 0.0), (1, 2)),
                                         ((0.0, -1.0, 0.0), (0, 2))])
def test_tile_key_and_cell(normal, axes):
    q = np.array([13, -3, 40])
    y = (q + 0.5).astype(np.float64)[None, :]
    n = np.array([normal])
    key, cell = O.tile_keys(_cfg(), y, n, np.array([100.0]), f64=True)
    tile = np.floor_divide(q, 8)
    ref, _, _ = O.keys(_cfg(), (tile + 0.5)[None, :].astype(np.float64), n, np.array([100.0]), f64=True)
    assert key[0] == ref[0]
    u, v = q[axes[0]] % 8, q[axes[1]] % 8          # Python's % is the floor remainder
    assert cell[0] == 8 * v + u
    # moving along the main axis inside the tile keeps key and cell
    main = int(np.argmax(np.abs(normal)))
    y2 = y.copy()
    y2[0, main] = 8 * tile[main] + 7.25
    key2, cell2 = O.tile_keys(_cfg(), y2, n, np.array([100.0]), f64=True)
    assert key2[0] == key[0] and cell2[0] == cell[0]
    # the next tile along u changes the key
    y3 = y.copy()
    y3[0, axes[0]] += 8.0
    key3, _ = O.tile_keys(_cfg(), y3, n, np.array([100.0]), f64=True)
    assert key3[0] != key[0]


def test_every_cell_of_a_tile_is_reached_once():
    xs, ys = np.meshgrid(np.arange(8), np.arange(8), indexing="xy")
    y = np.stack([16 + xs.ravel() + 0.5, -8 + ys.ravel() + 0.5, np.full(64, 3.5)], 1)
    n = np.tile([0.0, 0.0, -1.0], (64, 1))
    key, cell = O.tile_keys(_cfg(), y, n, np.full(64, 100.0), f64=True)
    assert len(set(key.tolist())) == 1
    assert sorted(cell.tolist()) == list(range(64))
    assert np.array_equal(cell, (8 * ys.ravel() + xs.ravel()).astype(np.uint32))


def _tile(cells):
    L0 = np.zeros((64, 3))
    n0 = np.zeros(64, np.uint32)
    for (x, y), (n, L) in cells.items():
        n0[8 * y + x] = n
        L0[8 * y + x] = L
    return L0, n0


def test_prefilter_hand_cases():
    T = 5
    # block A: cells (0,0) (1,0) (0,1) (1,1) with 1, 2, 3, 4 samples of 10, 20, 30, 40;
    # cell (6,6): 8 samples of 100
    L0, n0 = _tile({(0, 0): (1, 10.0), (1, 0): (2, 20.0), (0, 1): (3, 30.0), (1, 1): (4, 40.0), (6, 6): (8, 100.0)})
    Lq = O.prefilter(L0, n0, T)[:, 0].reshape(8, 8)      # [y, x]
    a = (1 * 10 + 2 * 20 + 3 * 30 + 4 * 40) / 10.0        # block A's level-1 mean, 10 samples
    # block A's cells: level 0 has < 5 samples, the level-1 parent has 10
    for x, y in ((0, 0), (1, 0), (0, 1), (1, 1)):
        assert Lq[y, x] == pytest.approx(a, rel=1e-15)
    # the rest of A's level-2 quadrant (x, y < 4): level-1 parents empty, level-2 parent = A
    assert Lq[3, 2] == pytest.approx(a, rel=1e-15)
    # cell (6,6) has 8 >= 5 samples: its own value; its level-1 siblings take the parent (8)
    assert Lq[6, 6] == 100.0 and Lq[7, 7] == 100.0 and Lq[6, 7] == 100.0
    # (4,4): level-1 parent (2,2) empty; level-2 parent (1,1) holds the 8 samples
    assert Lq[4, 4] == 100.0
    # (0,4): level-2 parent (0,1) empty; level 3 holds all 18 samples
    assert Lq[4, 0] == pytest.approx((a * 10 + 800.0) / 18.0, rel=1e-15)


def test_prefilter_fallbacks():
    # one cell with T-1 samples: no level reaches T, the coarsest level answers everywhere
    L0, n0 = _tile({(5, 2): (4, 7.0)})
    assert np.all(O.prefilter(L0, n0, 5)[:, 1] == 7.0)
    # an empty tile answers zero
    L0, n0 = _tile({})
    assert np.all(O.prefilter(L0, n0, 5) == 0.0)
    # every cell with enough samples: level 0 everywhere
    rng = np.random.default_rng(1)
    L0 = rng.uniform(0, 5, (64, 3))
    n0 = rng.integers(5, 40, 64).astype(np.uint32)
    assert np.array_equal(O.prefilter(L0, n0, 5), L0)
    # a constant tile stays constant whatever the counts
    L0 = np.full((64, 3), 2.5)
    n0 = rng.integers(0, 9, 64).astype(np.uint32)
    assert np.allclose(O.prefilter(L0, n0, 6), 2.5, rtol=1e-15)


@pytest.fixture(scope="module")
def furnace():
    sc = I.furnace_scene()
    return sc, O.OracleScene(sc, f64=True)


def test_furnace_one_bounce_with_tiles(furnace):
    sc, osc = furnace
    fr = I.furnace_camera(0)
    g = osc.gbuffer(fr, 64, 64)
    st = O.OracleFrameState(osc, O.default_config(width=64, height=64, rays_per_probe=64, table_log2=14,
                                                   cell_scale=2.0, cache_tiles=1, tile_min_samples=4))
    st.spawn(fr, g[0], g[1], g[3])
    st.trace(fr)
    t = st.tiles()
    # every hit lands in exactly one cell of one tile
    assert t["acc"][..., 3].sum() == st.stats()["hits"]
    st.update(fr)
    out = st.interpolate(fr, g[0], g[1], g[3])
    pr = st.probes()
    valid = pr["mask"][:st.P] != SENT
    at = pr["atlas"][valid][..., :3]
    assert abs(at.mean() / 1.8 - 1) < 5e-4
    assert np.allclose(out[..., :3], math.pi * 1.8, rtol=5e-3)
    t = st.tiles()
    live = t["nhist"] > 0
    cells = t["L"][live][:, 0]
    # the cells' moving averages hold rho * Le = 0.8 up to the one-frame estimator's noise;
    # the query radiance (a level's sample-weighted mean for every cell of a live tile) keeps
    # the mean and, being prefiltered, spreads less
    assert abs(cells.mean() / 0.8 - 1) < 3e-3
    q = t["Lq"][..., 0].ravel()
    assert abs(q.mean() / 0.8 - 1) < 3e-3
    assert q.std() < cells.std()


def test_furnace_feedback_with_tiles(furnace):
    sc, osc = furnace
    fr = I.furnace_camera(0)
    g = osc.gbuffer(fr, 64, 64)
    st = O.OracleFrameState(osc, O.default_config(width=64, height=64, rays_per_probe=64, table_log2=14,
                                                   cell_scale=0.5, n_cap=0, leak_bit=0, bounces=2, cache_tiles=1,
                                                   tile_min_samples=0))
    # n_cap = 0 keeps no history (each update takes the frame's mean and counts no samples), so
    # the levels are reached with tile_min_samples = 0: every cell answers with its own value
    rho, le = 0.8, 1.0
    L = 0.0
    for f in range(8):
        st.frame(fr, g)
        L = rho * (le + L)
        pr = st.probes()
        valid = pr["mask"][:st.P] != SENT
        assert abs(pr["atlas"][valid][..., :3].mean() / (le + L) - 1) < 8e-3, f

"""Pins of the float64 oracle of the learned surrogate: library interpolation, finite
differences, Adam's closed-form first step, torch's float8_e4m3fn codec."""
import math

import numpy as np
import pytest

from oracle import learned as L


def test_resolutions_span_min_to_max():
    s = L.Spec()
    r = s.resolutions()
    assert r[0] == 16 and r[-1] == 4096 and len(r) == 16
    assert all(b > a for a, b in zip(r, r[1:]))
    # geometric progression
    ratios = np.array(r[1:]) / np.array(r[:-1])
    assert np.allclose(ratios, 4096 ** (1 / 15) / 16 ** (1 / 15), rtol=0.05)


def test_dense_level_matches_library_trilinear_interpolation():
    scipy_interp = pytest.importorskip("scipy.interpolate")
    s = L.Spec(levels=1, table_log2=9, n_min=6, n_max=6)    # (6+1)^3 = 343 <= 512: dense
    p = L.init_params(s, seed=5)
    rng = np.random.default_rng(0)
    p["grid"][0] = rng.normal(size=(512, 2))
    N = 6
    vals = p["grid"][0][:(N + 1) ** 3].reshape(N + 1, N + 1, N + 1, 2)   # index vx + vy*7 + vz*49
    vals = np.transpose(vals, (2, 1, 0, 3))                               # -> [x][y][z]
    x = rng.uniform(0, 1, size=(500, 3)).astype(np.float32)
    x[:5] = np.float32([[0, 0, 0], [1, 1, 1], [0.5, 0.5, 0.5], [1 / 6, 2 / 6, 5 / 6], [1, 0, 1]])
    X, _ = L.features(s, p, x, np.zeros((500, 3)))
    g = np.arange(N + 1) / N
    for f in range(2):
        ref = scipy_interp.RegularGridInterpolator((g, g, g), vals[..., f])(x.astype(np.float64) * np.float32(N) / N)
        assert np.allclose(X[:, f], ref, atol=1e-6)
    # vertices return the stored value exactly
    v = np.array([[2, 3, 4]]) / 4.0
    s4 = L.Spec(levels=1, table_log2=8, n_min=4, n_max=4)
    p4 = L.init_params(s4, seed=1)
    X4, c = L.features(s4, p4, v.astype(np.float32), np.zeros((1, 3)))
    assert X4[0, 0] == p4["grid"][0][2 + 3 * 5 + 4 * 25, 0]


def test_hashed_levels_index_range_and_spread():
    s = L.Spec(levels=4, table_log2=10, n_min=32, n_max=256)
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, size=(20000, 3)).astype(np.float32)
    for (idx, w), N in zip(L.corner_indices(s, x), s.resolutions()):
        assert idx.min() >= 0 and idx.max() < s.T
        assert np.allclose(w.sum(1), 1.0)
        if (N + 1) ** 3 > s.T:
            h = np.bincount(idx.ravel(), minlength=s.T)
            assert (h > 0).mean() > 0.95


def _tiny():
    s = L.Spec(levels=2, table_log2=6, n_min=2, n_max=6)
    p = L.init_params(s, seed=3)
    rng = np.random.default_rng(4)
    p["grid"] = rng.normal(scale=0.5, size=p["grid"].shape)
    p["W3"][:3] = rng.normal(scale=0.3, size=(3, 64))
    x = rng.uniform(0, 1, size=(12, 3)).astype(np.float32)
    n = rng.normal(size=(12, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    t = rng.uniform(0, 2, size=(12, 3))
    return s, p, x, n, t


def test_gradients_match_central_finite_differences():
    s, p, x, n, t = _tiny()
    _, g = L.loss_and_grads(s, p, x, n, t)
    y0, _ = L.forward(s, p, x, n)
    den = y0 * y0 + 0.01     # the stopped-gradient denominator, frozen for the differences
    rng = np.random.default_rng(7)
    checked = 0
    for k in ("W1", "W2", "W3", "grid"):
        flat = p[k].reshape(-1)
        gk = g[k].reshape(-1)
        cand = np.nonzero(np.abs(gk) > 1e-6)[0]
        for i in rng.choice(cand, size=min(8, len(cand)), replace=False):
            h = 1e-6 * max(1.0, abs(flat[i]))
            old = flat[i]
            flat[i] = old + h
            lp, _ = L.loss_and_grads(s, p, x, n, t, den)
            flat[i] = old - h
            lm, _ = L.loss_and_grads(s, p, x, n, t, den)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gk[i]) <= 1e-5 * max(abs(fd), 1e-3), (k, i, fd, gk[i])
            checked += 1
    assert checked >= 24


def test_loss_hand_value():
    s = L.Spec(levels=1, table_log2=6, n_min=2, n_max=2)
    p = L.init_params(s, seed=0)
    for k in ("W1", "W2", "W3", "grid"):
        p[k] = np.zeros_like(p[k])
    # y = W3 relu(W2 relu(W1 x)); make y = 0.5 on every channel via the constant input
    p["W1"][0, 35] = 1.0
    p["W2"][0, 0] = 1.0
    p["W3"][:3, 0] = 0.5
    x = np.zeros((2, 3), np.float32)
    y, _ = L.forward(s, p, x, np.zeros((2, 3)))
    assert np.allclose(y, 0.5)
    t = np.array([[0.5, 0.5, 0.5], [1.5, 0.5, 0.5]])
    loss, _ = L.loss_and_grads(s, p, x, np.zeros((2, 3)), t)
    assert abs(loss - (1.0 / 0.26) / 6) < 1e-12


def test_adam_first_step_closed_form_and_skip():
    s, p, x, n, t = _tiny()
    _, g = L.loss_and_grads(s, p, x, n, t)
    before = {k: v.copy() for k, v in p.items()}
    opt = L.Adam(s, p)
    assert opt.step(p, g)
    for k in p:
        lr, eps = (s.lr_grid, s.eps_grid) if k == "grid" else (s.lr_mlp, s.eps_mlp)
        assert np.allclose(p[k] - before[k], -lr * g[k] / (np.abs(g[k]) + eps), rtol=1e-9, atol=1e-15)
    g["W1"][0, 0] = np.inf
    snap = {k: v.copy() for k, v in p.items()}
    assert not opt.step(p, g)
    assert all(np.array_equal(p[k], snap[k]) for k in p) and opt.t == 1


def test_lazy_grid_adam_moves_only_entries_with_a_gradient():
    """The lazy grid step equals the dense step (pinned by the closed form above) wherever the
    gradient is non-zero, and leaves an entry whose gradient is zero exactly as it was."""
    import dataclasses
    s, p, x, n, t = _tiny()
    _, g1 = L.loss_and_grads(s, p, x, n, t)
    g1["grid"][g1["grid"] == 0] = 1e-3            # step 1 touches every entry
    g2 = {k: v * -0.5 for k, v in g1.items()}
    g2["grid"].flat[0] = 0.0                       # an entry no sample touched at step 2
    pd = {k: v.copy() for k, v in p.items()}
    dense = L.Adam(dataclasses.replace(s, lazy_grid=False), pd)
    lazy = L.Adam(s, p)
    assert dense.step(pd, g1) and lazy.step(p, g1)
    assert np.array_equal(p["grid"], pd["grid"])
    after1 = p["grid"].flat[0]
    assert dense.step(pd, g2) and lazy.step(p, g2)
    on = g2["grid"] != 0
    assert np.array_equal(p["grid"][on], pd["grid"][on])
    assert np.array_equal(p["W1"], pd["W1"])
    assert p["grid"].flat[0] == after1 and pd["grid"].flat[0] != after1
    assert lazy.m["grid"].flat[0] == (1 - s.beta1) * g1["grid"].flat[0]


def test_training_fits_a_smooth_radiance_field():
    s = L.Spec(levels=4, table_log2=10, n_min=4, n_max=32, lr_grid=1e-2, lr_mlp=1e-2)
    p = L.init_params(s, seed=2)
    rng = np.random.default_rng(8)
    opt = L.Adam(s, p)
    f = lambda x: np.stack([1 + np.sin(3 * x[:, 0]), 0.5 + x[:, 1], 1 + 0 * x[:, 2]], 1)
    losses = []
    for it in range(150):
        x = rng.uniform(0, 1, size=(256, 3)).astype(np.float32)
        n = np.tile([0, 1, 0.0], (256, 1))
        loss, g = L.loss_and_grads(s, p, x, n, f(x))
        opt.step(p, g)
        losses.append(loss)
    assert np.mean(losses[-10:]) < 0.1 * np.mean(losses[:5])


def test_e4m3_codec_matches_torch():
    torch = pytest.importorskip("torch")
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy()
    got = L.e4m3_decode(codes)
    assert np.array_equal(np.isnan(ref), np.isnan(got))
    assert np.array_equal(ref[~np.isnan(ref)], got[~np.isnan(got)])
    assert got[0x38] == 1.0 and got[0x7E] == 448.0 and got[0x01] == 2.0 ** -9
    x = np.concatenate([np.random.default_rng(0).uniform(-448, 448, 200000),
                        (got[:126][1:] + got[:126][:-1]) / 2])   # exact midpoints: ties to even
    enc = L.e4m3_encode(x)
    tref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(enc, tref)
    assert L.e4m3_encode(np.array([1e6]))[0] == 0x7E and L.e4m3_encode(np.array([-1e6]))[0] == 0xFE


def test_init_values_are_seeded_uniform():
    v = L.init_values(3, 1, 100000, 1.0)
    assert v.dtype == np.float32 and -1 <= v.min() and v.max() < 1
    assert abs(v.mean()) < 0.01 and abs(v.var() - 1 / 3) < 0.01
    assert np.array_equal(v, L.init_values(3, 1, 100000, 1.0))
    assert not np.array_equal(v, L.init_values(4, 1, 100000, 1.0))


# ---- the frame's training batch --------------------------------------------------------

def test_training_rays_hand_flags():
    # rays: 0 hit with a cell, 1 miss, 2 hit that overflowed (no cell), 3 hit with a non-finite
    # sample, 4 hit with a cell
    flags = np.array([0x100 | 5, 3, 0x100, 0x100 | 0x10000, 0x100 | 0x200], np.uint32)
    slot = np.array([7, -1, -1, 3, 0], np.int32)
    sample = np.array([[1, 1, 1], [0, 0, 0], [1, 1, 1], [np.inf, 0, 0], [0, 0, 0]], np.float32)
    assert L.training_rays(slot, flags, sample).tolist() == [0, 4]


def test_select_picks_hand_values_and_strata():
    # floor((k + 1/2) * 10 / 4) = floor(1.25), floor(3.75), floor(6.25), floor(8.75)
    assert L.select_picks(10, 4, 0.5).tolist() == [1, 3, 6, 8]
    # fewer training rays than rows: floor(3k / 8) repeats rays in order
    assert L.select_picks(3, 8, 0.0).tolist() == [0, 0, 0, 1, 1, 1, 2, 2]
    # u just below 1 never reaches n
    u = np.float32(1.0) - np.float32(2.0 ** -24)
    assert L.select_picks(5, 5, u).tolist() == [0, 1, 2, 3, 4]
    # with n >= rows, pick k lies in stratum [k n / rows, (k + 1) n / rows): exact rationals
    from fractions import Fraction
    n, rows = 1000003, 4096
    u = L.frame_u(3, 7)
    picks = L.select_picks(n, rows, u)
    for k in range(0, rows, 97):
        exact = (Fraction(k) + Fraction(float(u))) * n / rows
        assert picks[k] == math.floor(exact)
        assert Fraction(k * n, rows) <= picks[k] < Fraction((k + 1) * n, rows)


def test_frame_u_is_the_top_24_bits_of_the_seeded_hash():
    for seed, f in ((3, 0), (3, 1), (17, 59)):
        u = L.frame_u(seed, f)
        assert u.dtype == np.float32 and 0.0 <= u < 1.0
        assert float(u) * 2 ** 24 == int(L.rng_u32(seed, f, 0x7FFFFFFF, 9)) >> 8
    assert L.frame_u(3, 0) != L.frame_u(3, 1)


def test_morton15_hand_codes():
    c = lambda q: L.morton15(np.array([q], np.float32) / np.float32(32))[0]  # noqa: E731
    assert c([1, 0, 0]) == 1 and c([0, 1, 0]) == 2 and c([0, 0, 1]) == 4
    assert c([2, 0, 0]) == 8 and c([0, 0, 16]) == 1 << 14
    assert c([31, 31, 31]) == (1 << 15) - 1 and c([5, 9, 3]) == c([5, 9, 3])
    # the top of the domain clamps into the last cell
    assert L.morton15(np.array([[1.0, 1.0, 1.0]], np.float32))[0] == (1 << 15) - 1
    # interleaving by brute force over random cells
    rng = np.random.default_rng(0)
    q = rng.integers(0, 32, size=(200, 3))
    got = L.morton15((q.astype(np.float32) + np.float32(0.5)) / np.float32(32))
    for (a, b, cc), g in zip(q, got):
        bits = "".join(f"{z:05b}"[4 - i] + f"{y:05b}"[4 - i] + f"{x:05b}"[4 - i]
                       for i in reversed(range(5)) for x, y, z in [(a, b, cc)])
        assert g == int(bits, 2)


def test_group_order_is_a_stable_sort_by_code():
    rng = np.random.default_rng(1)
    x = rng.integers(0, 4, size=(500, 3)).astype(np.float32) / np.float32(4)   # many equal codes
    order = L.group_order(x)
    codes = L.morton15(x)
    assert sorted(range(500), key=lambda i: (int(codes[i]), i)) == order.tolist()


def test_step_rows_partition_the_batch():
    B, steps = 16, 4
    rows = L.batch_rows(B, steps)
    assert rows == 64 and L.batch_rows(1 << 19, 4) == 1 << 20 and L.batch_rows(1 << 20, 4) == 1 << 20
    got = np.concatenate([L.step_rows(rows, B, k) for k in range(steps)])
    assert sorted(got.tolist()) == list(range(rows))
    assert L.step_rows(rows, B, 1).tolist() == list(range(1, 64, 4))

"""Pins of the CPU oracle's small building blocks against what mathematics and third-party
definitions fix (closed forms, exhaustive bounds, library routines, invariants)."""
import ctypes as C
import math
import struct

import numpy as np
import pytest

import oracle as O


# --- sin/cos of 2*pi*u without a library transcendental -------------------------------------

def test_sincos_exhaustive_bound():
    # every float32 input u = k * 2^-24 the ray generator can produce
    u = (np.arange(1 << 24, dtype=np.float64) * 2.0 ** -24).astype(np.float32)
    c, s = O.sincos2pi(u)
    ref_c = np.cos(2.0 * np.pi * u.astype(np.float64))
    ref_s = np.sin(2.0 * np.pi * u.astype(np.float64))
    assert np.max(np.abs(c - ref_c)) < 3.0e-7
    assert np.max(np.abs(s - ref_s)) < 3.0e-7
    # special angles are exact
    c0, s0 = O.sincos2pi(np.array([0.0, 0.25, 0.5, 0.75], np.float32))
    assert list(c0) == [1.0, 0.0, -1.0, 0.0] and list(s0) == [0.0, 1.0, 0.0, -1.0]


# --- hashes ------------------------------------------------------------------------------

def test_xxh32_matches_xxhash_library():
    xxhash = pytest.importorskip("xxhash")
    rng = np.random.default_rng(0)
    vals = [0, 1, 2, 0xFFFFFFFF, 0x80000000] + [int(v) for v in rng.integers(0, 2**32, 200)]
    for v in vals:
        assert O.xxh32(v) == xxhash.xxh32_intdigest(struct.pack("<I", v), 0)


def _collisions(which, n):
    lib, p = O._lib(False)
    f = getattr(lib, p + "hash_collisions")
    f.restype = C.c_uint64
    f.argtypes = [C.c_uint32, C.c_uint64]
    return f(which, n)


def test_hashes_are_injective_and_avalanche():
    # both hashes are bijections of u32: no repeated output over 2^24 inputs (a random
    # function would repeat ~32k times)
    assert _collisions(0, 1 << 24) == 0
    assert _collisions(1, 1 << 24) == 0
    # avalanche: flipping one input bit flips each output bit with probability ~1/2
    rng = np.random.default_rng(1)
    xs = [int(v) for v in rng.integers(0, 2**32, 400)]
    for h in (O.pcg, O.xxh32):
        flips = np.zeros((32, 32))
        for x in xs:
            hx = h(x)
            for b in range(32):
                d = hx ^ h(x ^ (1 << b))
                flips[b] += [(d >> k) & 1 for k in range(32)]
        p = flips / len(xs)
        assert 0.35 < p.min() and p.max() < 0.65


def test_rng_uniform_24bit():
    n = 200000
    u = np.array([O.rng(3, 0, i, 0) >> 8 for i in range(n)], np.float64) / 2**24
    assert u.min() >= 0.0 and u.max() < 1.0
    hist = np.bincount((u * 64).astype(int), minlength=64)
    exp = n / 64
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 120.0   # 63 dof, p ~ 1e-5
    # different dimensions / frames / ids are decorrelated
    a = np.array([O.rng(3, 0, i, 0) for i in range(4000)], np.float64)
    b = np.array([O.rng(3, 0, i, 1) for i in range(4000)], np.float64)
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.06


# --- Halton jitter (Section 2.1.1) ---------------------------------------------------------

def test_halton_closed_forms():
    # Phi_2(1..4) = 1/2, 1/4, 3/4, 1/8 ; Phi_3(1..4) = 1/3, 2/3, 1/9, 4/9
    got = [O.halton_jitter(f) for f in range(4)]
    assert got == [(4, 2), (2, 5), (6, 0), (1, 3)]
    # base-2 stratification: 64 consecutive frames visit every column exactly 8 times
    jx = [O.halton_jitter(f)[0] for f in range(64)]
    assert np.bincount(jx, minlength=8).tolist() == [8] * 8
    for f in range(200):
        x, y = O.halton_jitter(f)
        assert 0 <= x < 8 and 0 <= y < 8
        i = f + 1
        # floor(8 * radical inverse) from exact rational arithmetic
        def phi(i, b):
            num, den = 0, 1
            while i:
                num, den, i = num * b + i % b, den * b, i // b
            return num, den
        n2, d2 = phi(i, 2)
        n3, d3 = phi(i, 3)
        assert (x, y) == (8 * n2 // d2, 8 * n3 // d3)


# --- Algorithm 6 --------------------------------------------------------------------------

def test_adaptive_cell_size_closed_form():
    fov = math.radians(60.0)
    k = O.distance_scale(np.float32(fov), 1920, 1080)
    # tan(fov * 8 * max(1/1080, 1080/1920^2)) with 1/H the larger term for landscape
    assert abs(k - math.tan(fov * 8.0 / 1080.0)) < 1e-9
    assert abs(k * 10.0 - 0.07757) < 1e-4
    # portrait: H/W^2 wins
    k2 = O.distance_scale(np.float32(fov), 100, 400)
    assert abs(k2 - math.tan(fov * 8.0 * 400.0 / 100.0 ** 2)) < 1e-6


# --- hemi-octahedral cells and cosine sampling (Section 2.1, 2.1.3) -----------------------

def test_cell_moment_sums():
    m = O.cell_moments()
    assert abs(m[:, 0].sum() - 2.0 * math.pi) < 1e-10
    assert np.allclose(m[:, 1:4].sum(0), [0.0, 0.0, math.pi], atol=1e-10)
    M = m[:, 4:].sum(0)  # xx, yy, zz, xy, xz, yz
    assert np.allclose(M, [2 * math.pi / 3] * 3 + [0.0] * 3, atol=1e-10)
    # symmetry of the map: cell (ix, iy) and its mirror have the same solid angle
    om = m[:, 0].reshape(8, 8)
    assert np.allclose(om, om[::-1, ::-1], rtol=1e-12)
    assert np.allclose(om, om.T, rtol=1e-12)
    assert (om > 0).all()


def test_cell_solid_angle_monte_carlo():
    # independent check of the quadrature: uniform hemisphere directions binned by the map
    rng = np.random.default_rng(5)
    n = 2_000_000
    z = rng.uniform(0.0, 1.0, n)
    ph = rng.uniform(0.0, 2 * math.pi, n)
    r = np.sqrt(1 - z * z)
    x, y = r * np.cos(ph), r * np.sin(ph)
    s = np.abs(x) + np.abs(y) + z
    a, b = x / s, y / s
    ix = np.clip(np.floor(4 * (a + b + 1)), 0, 7).astype(int)
    iy = np.clip(np.floor(4 * (a - b + 1)), 0, 7).astype(int)
    frac = np.bincount(8 * iy + ix, minlength=64) / n
    m = O.cell_moments()
    assert np.allclose(frac, m[:, 0] / (2 * math.pi), atol=4 * np.sqrt(frac.max() / n))


def test_cosine_sampling_chi2_per_cell():
    rng = np.random.default_rng(2)
    n = 400000
    nrm = rng.normal(size=3)
    nrm /= np.linalg.norm(nrm)
    u0 = (rng.integers(0, 1 << 24, n) * 2.0 ** -24).astype(np.float32)
    u1 = (rng.integers(0, 1 << 24, n) * 2.0 ** -24).astype(np.float32)
    d, cell = O.cosine_dirs(np.tile(nrm.astype(np.float32), (n, 1)), u0, u1)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=2e-6)
    assert (d @ nrm.astype(np.float32) > -1e-6).all()
    # cosine-distributed: the probability of a cell is its projected solid angle / pi
    m = O.cell_moments()
    p = m[:, 3] / math.pi
    hist = np.bincount(cell, minlength=64)
    chi2 = ((hist - n * p) ** 2 / (n * p)).sum()
    assert chi2 < 130.0   # 63 dof
    # mean cos(theta) of a cosine distribution is 2/3
    assert abs((d @ nrm).mean() - 2.0 / 3.0) < 3e-3
    # the direction l = (0,0,1) (u0 = 0) lies in the centre cells 27, 28, 35, 36
    d0, c0 = O.cosine_dirs(np.array([[0, 0, 1.0]], np.float32), np.zeros(1, np.float32),
                           np.zeros(1, np.float32))
    assert np.allclose(d0, [[0, 0, 1]]) and int(c0[0]) in (27, 28, 35, 36)


# --- world-cache descriptor (Section 2.2.1, 2.2.2) ------------------------------------------

def test_key_hand_cases():
    cfg = O.default_config()
    key, b, fp = O.keys(cfg, [[0.05, 0.15, -0.05]], [[0.0, 1.0, 0.0]], [0.5])
    k = int(key[0])
    q = [(k >> s) & 0x3FFFF for s in (0, 18, 36)]
    sx = [v - (1 << 18) if v >= (1 << 17) else v for v in q]
    assert sx == [0, 1, -1]
    assert (k >> 54) & 7 == 2 and (k >> 57) & 1 == 0
    assert fp[0] != 0 and b[0] < (1 << 16) // 32
    # leak bit: ray shorter than one cell (t * S < 1)
    k2 = int(O.keys(cfg, [[0.05, 0.15, -0.05]], [[0, 1, 0]], [0.05])[0][0])
    assert (k2 >> 57) & 1 == 1 and (k2 & ((1 << 57) - 1)) == (k & ((1 << 57) - 1))
    # normal classes: +x 0, -x 1, +y 2, -y 3, +z 4, -z 5; ties go to the lower axis
    ns = [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
          [0.6, 0.6, 0.5], [-0.5, -0.6, 0.6]]
    ks = O.keys(cfg, np.zeros((8, 3)), ns, np.ones(8))[0]
    assert [(int(v) >> 54) & 7 for v in ks] == [0, 1, 2, 3, 4, 5, 0, 3]


@pytest.mark.parametrize("f64", [False, True])
def test_key_levels_of_detail_hand_cases(f64):
    """Section 2.2.1 levels of detail (READING: cell size = base size x 2^lod, lod the smallest
    integer <= 7 with 2^lod >= lod_scale * d * S).  Camera at the origin, S = 10 (0.1 m cells),
    lod_scale = 0.01: x = 0.1 d, so d = 5, 15, 19, 21, 45 m give lod 0, 1, 1, 2, 3 and a point
    100 km away is capped at 7.  The position is quantised at the level's cell size and the
    leak test uses it too."""
    cfg = O.default_config(lod_scale=0.01)
    d = np.array([5.0, 15.0, 19.0, 21.0, 45.0, 1e5])
    y = np.stack([d, np.zeros(6), np.zeros(6)], 1)
    key = O.keys(cfg, y, np.tile([0, 1, 0], (6, 1)), np.ones(6), f64=f64)[0].astype(np.int64)
    assert list((key >> 58) & 7) == [0, 1, 1, 2, 3, 7]
    qx = key & 0x3FFFF
    # floor(d * 10 / 2^lod): 50, 75, 95, 52 (52.5), 56 (56.25), (1e6 / 128 = 7812) mod 2^18
    assert list(qx) == [50, 75, 95, 52, 56, 7812]
    # leak bit: t = 0.15 m is shorter than a 0.2 m cell (lod 1) but not than a 0.1 m cell
    k0 = int(O.keys(cfg, [[5.0, 0, 0]], [[0, 1, 0]], [0.15], f64=f64)[0][0])
    k1 = int(O.keys(cfg, [[15.0, 0, 0]], [[0, 1, 0]], [0.15], f64=f64)[0][0])
    assert (k0 >> 57) & 1 == 0 and (k1 >> 57) & 1 == 1
    # lod_scale 0: one level, the same keys as without levels
    k_off = O.keys(O.default_config(), y, np.tile([0, 1, 0], (6, 1)), np.ones(6), f64=f64)[0].astype(np.int64)
    assert ((k_off >> 58) == 0).all()
    assert list(k_off & 0x3FFFF) == [50, 150, 190, 210, 450, 1000000 % (1 << 18)]
    # the distance is measured from the camera
    k_cam = O.keys(cfg, y, np.tile([0, 1, 0], (6, 1)), np.ones(6), f64=f64, cam=(15.0, 0.0, 0.0))[0].astype(np.int64)
    assert int(k_cam[1] >> 58) == 0


def test_key_quantiser_is_the_float32_product():
    cfg = O.default_config()
    rng = np.random.default_rng(3)
    y = rng.uniform(-50, 50, size=(20000, 3)).astype(np.float32)
    # add decimal boundary values whose float32 products round across an integer
    y[:6, 0] = np.float32([0.3, 0.7, 0.1, -0.1, 2.9, -0.7])
    key = O.keys(cfg, y, np.tile([0, 1, 0], (len(y), 1)), np.ones(len(y)))[0].astype(np.int64)
    q = np.stack([(key >> s) & 0x3FFFF for s in (0, 18, 36)], 1)
    q = np.where(q >= (1 << 17), q - (1 << 18), q)
    # float64 evaluation of the float32 operation: exact product, one rounding to float32
    prod = (y.astype(np.float64) * 10.0).astype(np.float32).astype(np.float64)
    assert (q == np.floor(prod)).all()
    assert q[1, 0] == 7   # 0.7f * 10 rounds up to 7.0f although the exact product is 6.99999988


def test_key_packing_injective():
    cfg = O.default_config()
    rng = np.random.default_rng(4)
    qi = rng.integers(-(1 << 17), 1 << 17, size=(50000, 3))
    y = ((qi + 0.5) / 10.0).astype(np.float32)
    key = O.keys(cfg, y, np.tile([0, 1, 0], (len(y), 1)), np.ones(len(y)))[0]
    uq = np.unique(qi, axis=0)
    assert len(np.unique(key)) == len(uq)


def test_bucket_uniformity():
    cfg = O.default_config(table_log2=16)
    q = np.stack(np.meshgrid(np.arange(64), np.arange(16), np.arange(32), indexing="ij"), -1).reshape(-1, 3)
    y = ((q + 0.5) / 10.0).astype(np.float32)
    _, b, fp = O.keys(cfg, y, np.tile([0, 1, 0], (len(y), 1)), np.ones(len(y)))
    nb = (1 << 16) // 32
    hist = np.bincount(b, minlength=nb)
    exp = len(y) / nb
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < nb + 6 * math.sqrt(2 * nb)
    assert len(np.unique(fp)) > len(fp) - 5


# --- spherical harmonics (Section 2.4.2) ----------------------------------------------------

def _random_frame_normals(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_sh_hemisphere_constant_gives_pi_L(oracle_mod):
    from paper_2310_19855_amd import inputs as I
    sc = O.OracleScene(I.room_scene(), f64=True)
    st = O.OracleFrameState(sc, O.default_config())
    nrm = _random_frame_normals(50, 6)
    nrm[0] = [0, 0, 1]
    nrm[1] = [0, 0, -1]
    atlas = np.zeros((50, 64, 4))
    atlas[..., :3] = [2.0, 0.5, 1.0]
    coef = st.sh_project(atlas, nrm)
    E = O.sh_eval(coef, nrm, f64=True)
    assert np.allclose(E, np.pi * np.array([2.0, 0.5, 1.0]), rtol=1e-9)


def test_sh_projection_matches_brute_force_integral():
    """coefficients of a piecewise-constant atlas equal the integral of Y_lm * L over the
    hemisphere, computed by dense Monte Carlo with the textbook real SH basis"""
    from paper_2310_19855_amd import inputs as I
    sc = O.OracleScene(I.room_scene(), f64=True)
    st = O.OracleFrameState(sc, O.default_config())
    rng = np.random.default_rng(9)
    n = np.array([0.3, -0.5, 0.81])
    n /= np.linalg.norm(n)
    atlas = np.zeros((1, 64, 4))
    atlas[0, :, :3] = rng.uniform(0, 2, size=(64, 3))
    coef = st.sh_project(atlas, n[None])[0].reshape(9, 3)
    # Monte Carlo over uniform world directions in the hemisphere of n
    N = 4_000_000
    w = rng.normal(size=(N, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    w[w @ n < 0] *= -1
    # local frame used by the oracle: Duff et al. branchless basis
    sgn = 1.0 if n[2] >= 0 else -1.0
    a = -1.0 / (sgn + n[2])
    b = n[0] * n[1] * a
    t = np.array([1 + sgn * n[0] * n[0] * a, sgn * b, -sgn * n[0]])
    bb = np.array([b, sgn + n[1] * n[1] * a, -n[1]])
    lx, ly, lz = w @ t, w @ bb, w @ n
    s = np.abs(lx) + np.abs(ly) + lz
    A, B = lx / s, ly / s
    ix = np.clip(np.floor(4 * (A + B + 1)), 0, 7).astype(int)
    iy = np.clip(np.floor(4 * (A - B + 1)), 0, 7).astype(int)
    L = atlas[0, 8 * iy + ix, :3]
    x, y, z = w[:, 0], w[:, 1], w[:, 2]
    Y = np.stack([0.5 * np.sqrt(1 / np.pi) * np.ones(N), np.sqrt(3 / (4 * np.pi)) * y,
                  np.sqrt(3 / (4 * np.pi)) * z, np.sqrt(3 / (4 * np.pi)) * x,
                  0.5 * np.sqrt(15 / np.pi) * x * y, 0.5 * np.sqrt(15 / np.pi) * y * z,
                  0.25 * np.sqrt(5 / np.pi) * (3 * z * z - 1), 0.5 * np.sqrt(15 / np.pi) * x * z,
                  0.25 * np.sqrt(15 / np.pi) * (x * x - y * y)], 1)
    mc = 2 * np.pi * (Y[:, :, None] * L[:, None, :]).mean(0)
    assert np.allclose(coef, mc, atol=6e-3)


# --- Algorithm 4 and the mask MIP chain (Section 2.1.5) --------------------------------------

def _morton_first(mask0, TW, TH, lvl, x, y):
    """first valid entry in Morton (recursive 2x2 raster) order of the level-lvl block"""
    size = 1 << lvl
    best = None
    for dy in range(size):
        for dx in range(size):
            cx, cy = x * size + dx, y * size + dy
            if cx >= TW or cy >= TH:
                continue
            v = int(mask0[cy * TW + cx])
            if v == 0xFFFFFFFF:
                continue
            code = 0
            for bit in range(lvl):
                code |= ((dx >> bit) & 1) << (2 * bit) | ((dy >> bit) & 1) << (2 * bit + 1)
            if best is None or code < best[0]:
                best = (code, v)
    return 0xFFFFFFFF if best is None else best[1]


def test_mask_mips_first_valid_in_morton_order():
    from paper_2310_19855_amd import inputs as I
    sc = O.OracleScene(I.room_scene())
    W, H = 88, 56
    st = O.OracleFrameState(sc, O.default_config(width=W, height=H))
    rng = np.random.default_rng(12)
    pos = np.zeros((H, W, 4), np.float32)
    nrm = np.zeros((H, W, 4), np.float32)
    nrm[..., 1] = 1
    prim = np.where(rng.uniform(size=(H, W)) < 0.7, 0xFFFFFFFF, 5).astype(np.uint32)
    fr = I.room_camera(0)
    st.spawn(fr, pos, nrm, prim)
    pr = st.probes()
    d = st.dims()
    TW, TH, nmip = int(d[3]), int(d[4]), int(d[5])
    jx, jy = int(d[7]), int(d[8])
    m0 = pr["mask"][:TW * TH]
    for ty in range(TH):
        for tx in range(TW):
            px, py = 8 * tx + jx, 8 * ty + jy
            v = int(m0[ty * TW + tx])
            if px < W and py < H and prim[py, px] != 0xFFFFFFFF:
                assert v == (py << 16) | px
            else:
                assert v == 0xFFFFFFFF
    off, w, h = 0, TW, TH
    for lvl in range(nmip):
        for y in range(h):
            for x in range(w):
                assert int(pr["mask"][off + y * w + x]) == _morton_first(m0, TW, TH, lvl, x, y)
        off += w * h
        w, h = (w + 1) // 2, (h + 1) // 2
    assert w == 1 and h == 1 or nmip >= 1


def test_find_closest_probe_hand_cases():
    from paper_2310_19855_amd import inputs as I
    sc = O.OracleScene(I.room_scene())
    W = H = 64   # 8x8 tiles
    st = O.OracleFrameState(sc, O.default_config(width=W, height=H))
    pos = np.zeros((H, W, 4), np.float32)
    nrm = np.zeros((H, W, 4), np.float32)
    prim = np.full((H, W), 0xFFFFFFFF, np.uint32)
    fr = I.room_camera(0)          # frame 0 jitter = (4, 2)
    for tx, ty in ((0, 0), (5, 5), (7, 2)):
        prim[8 * ty + 2, 8 * tx + 4] = 1
    st.spawn(fr, pos, nrm, prim)
    enc = lambda tx, ty: ((8 * ty + 2) << 16) | (8 * tx + 4)
    # a valid probe in the very tile is returned at mip 0
    assert st.find_probe(8 * 5, 8 * 5, 0, 0) == enc(5, 5)
    # empty neighbour (tile (6,5)): mip 1 looks at tile block (3,2)+(1,0) -> (4,2) = tiles 8..9
    # x 4..5 (out of range/empty) -> continue to mip 2 ((1,1)+(1,0) = block (2,1): tiles 8.. empty)
    assert st.find_probe(8 * 5, 8 * 5, 1, 0) == 0xFFFFFFFF
    # from tile (6,4) towards -x: mip0 (5,4) empty; mip1 (3,2)-(1,0) = (2,2) covers tiles
    # (4..5, 4..5) whose first valid in raster order is (5,5)
    assert st.find_probe(8 * 6, 8 * 4, -1, 0) == enc(5, 5)
    # out of bounds stops the search
    assert st.find_probe(0, 0, -1, 0) == 0xFFFFFFFF
    assert st.find_probe(0, 0, 0, 0) == enc(0, 0)

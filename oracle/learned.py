"""Float64 oracle of the learned radiance-cache surrogate -- TEST INFRASTRUCTURE ONLY.

Not part of the GI-1.0 paper: the surrogate follows the mathematical definitions of the
multiresolution hash encoding (Mueller, Evans, Schied and Keller 2022) and of an online-trained
radiance cache (Mueller, Rousselle, Novak and Keller 2021).  No code of those works is used.

Definitions (every one mirrored by the HIP kernels):
  * input: x = clamp((y - lo) / (hi - lo), 0, 1) per axis; normal feature (n + 1) / 2.
  * encoding: level l of L has resolution N_l = floor(N_min * exp(l ln b) + 1e-6), ln b =
    (ln N_max - ln N_min) / (L - 1).  p = x * N_l (float32), v = min(floor(p), N_l - 1),
    f = p - v; the 8 corners v + c
    (c in {0,1}^3) have trilinear weights prod(c ? f : 1 - f).  A corner's table index is
    dense, vx + vy (N_l+1) + vz (N_l+1)^2, when (N_l+1)^3 <= T, else the spatial hash
    (vx * 1 ^ vy * 2654435761 ^ vz * 805459861) mod T in uint32 arithmetic.  Each entry holds
    2 features; the level's output is the weighted sum.  Levels are concatenated: 2L values.
  * MLP input (64): columns 0..2L-1 the encoding (columns up to 31 zero when L < 16), 32..34
    the normal feature, 35 the constant 1, the rest zero; W1 (64x64) -> ReLU ->
    W2 (64x64) -> ReLU -> W3 (16x64); outputs 0..2 are radiance.  No biases (the constant
    input plays that role).
  * loss: mean over samples and 3 channels of (y - t)^2 / (sg(y)^2 + 0.01) (relative L2 with
    the prediction's square treated as a constant).
  * Adam (Kingma and Ba 2015) with bias correction on the unscaled gradient; a step whose
    gradient holds a non-finite value is skipped.
  * initial values: (2u - 1) * scale in float32 with u = the top 24 bits of the nested PCG
    hash rng(seed, stream, index, 0) (streams: W1 1, W2 2, W3 3, grid level l 100 + l);
    scale = 1e-4 for the grid, sqrt(6 / 64) for the weights; rows 3..15 of W3 are zero.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

PRIME_Y = 2654435761
PRIME_Z = 805459861


def _pcg(v):
    v = np.asarray(v, np.uint64) & 0xFFFFFFFF
    state = (v * 747796405 + 2891336453) & 0xFFFFFFFF
    word = (((state >> ((state >> 28) + 4)) ^ state) * 277803737) & 0xFFFFFFFF
    return ((word >> 22) ^ word) & 0xFFFFFFFF


def rng_u32(seed, stream, idx, dim=0):
    """nested PCG hash: pcg(dim + pcg(idx + pcg(stream + pcg(seed)))) in uint32 arithmetic"""
    s = _pcg(np.uint64(seed))
    s = _pcg((np.uint64(stream) + s) & 0xFFFFFFFF)
    s = _pcg((np.asarray(idx, np.uint64) + s) & 0xFFFFFFFF)
    return _pcg((np.uint64(dim) + s) & 0xFFFFFFFF)


def init_values(seed, stream, n, scale):
    u = ((rng_u32(seed, stream, np.arange(n, dtype=np.uint64)) >> 8).astype(np.float32)
         * np.float32(5.9604644775390625e-08))
    return ((u * np.float32(2.0) - np.float32(1.0)) * np.float32(scale)).astype(np.float32)


@dataclass
class Spec:
    levels: int = 16
    table_log2: int = 19
    n_min: int = 16
    n_max: int = 4096
    hidden: int = 64
    beta1: float = 0.9
    beta2: float = 0.99
    eps_grid: float = 1e-15
    eps_mlp: float = 1e-8
    lr_grid: float = 1e-2
    lr_mlp: float = 1e-3
    loss_scale: float = 128.0
    lazy_grid: bool = True      # grid entries with a zero gradient skip the step (m, v, value kept)

    @property
    def T(self):
        return 1 << self.table_log2

    def resolutions(self):
        if self.levels == 1:
            return [self.n_min]
        lb = (math.log(self.n_max) - math.log(self.n_min)) / (self.levels - 1)
        return [int(math.floor(self.n_min * math.exp(l * lb) + 1e-6)) for l in range(self.levels)]


def init_params(spec: Spec, seed: int):
    grid = np.stack([init_values(seed, 100 + l, spec.T * 2, 1e-4).reshape(spec.T, 2)
                     for l in range(spec.levels)]).astype(np.float64)
    s = math.sqrt(6.0 / 64.0)
    W1 = init_values(seed, 1, 64 * 64, s).reshape(64, 64).astype(np.float64)
    W2 = init_values(seed, 2, 64 * 64, s).reshape(64, 64).astype(np.float64)
    W3 = np.zeros((16, 64))
    W3[:3] = init_values(seed, 3, 3 * 64, s).reshape(3, 64)
    return dict(grid=grid, W1=W1, W2=W2, W3=W3)


def corner_indices(spec: Spec, x32):
    """per level: indices [n,8] and trilinear weights [n,8] of the 8 corners; x32 float32 [n,3]"""
    out = []
    T = spec.T
    for l, N in enumerate(spec.resolutions()):
        p = (x32 * np.float32(N)).astype(np.float32)
        v = np.minimum(np.floor(p), np.float32(N - 1)).astype(np.int64)
        f = (p - v.astype(np.float32)).astype(np.float64)
        idx = np.zeros((len(x32), 8), np.int64)
        w = np.ones((len(x32), 8))
        dense = (N + 1) ** 3 <= T
        for c in range(8):
            cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
            vx, vy, vz = v[:, 0] + cx, v[:, 1] + cy, v[:, 2] + cz
            if dense:
                idx[:, c] = vx + vy * (N + 1) + vz * (N + 1) ** 2
            else:
                h = (vx.astype(np.uint64) * 1) ^ (vy.astype(np.uint64) * PRIME_Y & 0xFFFFFFFF) \
                    ^ (vz.astype(np.uint64) * PRIME_Z & 0xFFFFFFFF)
                idx[:, c] = (h & 0xFFFFFFFF) & (T - 1)
            w[:, c] = (f[:, 0] if cx else 1 - f[:, 0]) * (f[:, 1] if cy else 1 - f[:, 1]) * \
                (f[:, 2] if cz else 1 - f[:, 2])
        out.append((idx, w))
    return out


def normalize_pos(y, lo, hi):
    """float32 x = clamp((y - lo) / (hi - lo), 0, 1), the same rounding as the kernels"""
    y = np.asarray(y, np.float32)
    lo = np.asarray(lo, np.float32)
    hi = np.asarray(hi, np.float32)
    return np.clip((y - lo) / (hi - lo), np.float32(0), np.float32(1)).astype(np.float32)


def features(spec: Spec, params, x32, nrm):
    corners = corner_indices(spec, x32)
    enc = np.zeros((len(x32), 2 * spec.levels))
    for l, (idx, w) in enumerate(corners):
        g = params["grid"][l]
        enc[:, 2 * l] = (w * g[idx, 0]).sum(1)
        enc[:, 2 * l + 1] = (w * g[idx, 1]).sum(1)
    X = np.zeros((len(x32), 64))
    X[:, :2 * spec.levels] = enc
    X[:, 32:35] = (np.asarray(nrm, np.float64) + 1.0) / 2.0
    X[:, 35] = 1.0
    return X, corners


def forward(spec: Spec, params, x32, nrm):
    X, corners = features(spec, params, x32, nrm)
    z1 = X @ params["W1"].T
    h1 = np.maximum(z1, 0)
    z2 = h1 @ params["W2"].T
    h2 = np.maximum(z2, 0)
    y = h2 @ params["W3"].T
    return y[:, :3], dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2, y=y, corners=corners)


def loss_and_grads(spec: Spec, params, x32, nrm, target, den=None):
    """loss and exact gradients (float64) with respect to grid and weights; the denominator
    y^2 + 0.01 is a constant of the gradient (pass `den` to evaluate the loss with it frozen)"""
    y, c = forward(spec, params, x32, nrm)
    t = np.asarray(target, np.float64)
    n = len(y)
    if den is None:
        den = y * y + 0.01
    loss = ((y - t) ** 2 / den).sum() / (3 * n)
    dy = np.zeros((n, 16))
    dy[:, :3] = 2.0 * (y - t) / den / (3 * n)
    gW3 = dy.T @ c["h2"]
    dh2 = dy @ params["W3"]
    dz2 = dh2 * (c["z2"] > 0)
    gW2 = dz2.T @ c["h1"]
    dh1 = dz2 @ params["W2"]
    dz1 = dh1 * (c["z1"] > 0)
    gW1 = dz1.T @ c["X"]
    dX = dz1 @ params["W1"]
    ggrid = np.zeros_like(params["grid"])
    for l, (idx, w) in enumerate(c["corners"]):
        for f in range(2):
            np.add.at(ggrid[l][:, f], idx.ravel(), (w * dX[:, 2 * l + f][:, None]).ravel())
    return loss, dict(grid=ggrid, W1=gW1, W2=gW2, W3=gW3)


class Adam:
    def __init__(self, spec: Spec, params):
        self.spec = spec
        self.m = {k: np.zeros_like(v) for k, v in params.items()}
        self.v = {k: np.zeros_like(v) for k, v in params.items()}
        self.t = 0

    def step(self, params, grads):
        """returns False (and changes nothing) if any gradient is non-finite"""
        if not all(np.isfinite(g).all() for g in grads.values()):
            return False
        s = self.spec
        self.t += 1
        for k in params:
            lr, eps = (s.lr_grid, s.eps_grid) if k == "grid" else (s.lr_mlp, s.eps_mlp)
            g = grads[k]
            m = s.beta1 * self.m[k] + (1 - s.beta1) * g
            v = s.beta2 * self.v[k] + (1 - s.beta2) * g ** 2
            mh = m / (1 - s.beta1 ** self.t)
            vh = v / (1 - s.beta2 ** self.t)
            p = params[k] - lr * mh / (np.sqrt(vh) + eps)
            if k == "grid" and s.lazy_grid:
                # lazy form: only entries that received a gradient in this step move
                on = g != 0
                m = np.where(on, m, self.m[k])
                v = np.where(on, v, self.v[k])
                p = np.where(on, p, params[k])
            self.m[k], self.v[k], params[k] = m, v, p
        return True


# ---- the frame's training batch (not in the paper; the surrogate's own data path) --------
#
#   * training rays: the frame's probe rays whose hit found or created a world-cache cell
#     (slot >= 0) and whose cache sample is finite, in ray order (ray id = probe * R + ray);
#     their samples (before quantisation) are the targets.
#   * rows = steps * B picks (at most 2^20, a whole number of B), pick k = training ray
#     floor((k + u) n / rows), n training rays, u the frame's uniform number.
#   * grouping: the rows stably sorted by the 15-bit Morton code of the normalised position
#     (32 cells per axis); optimiser step k trains on grouped rows k, k + s, k + 2s, ...,
#     s = rows / B.

def training_rays(slot, flags, sample):
    """ids (ascending) of the rays whose hit (flag bit 8) has a cell (slot >= 0) and a finite
    sample"""
    hit = (np.asarray(flags) & 0x100) != 0
    ok = hit & (np.asarray(slot) >= 0) & np.isfinite(np.asarray(sample, np.float64)).all(1)
    return np.nonzero(ok)[0]


def frame_u(seed, frame):
    """the selection's uniform number of a frame: the top 24 bits of the nested PCG hash
    rng(seed, frame, 2^31 - 1, 9), times 2^-24 (float32)"""
    h = int(rng_u32(seed, frame, 0x7FFFFFFF, 9))
    return np.float32(h >> 8) * np.float32(5.9604644775390625e-08)


def batch_rows(B, steps):
    """rows of a frame's batch: one sub-batch of B per step, at most 2^20 rows"""
    return B * max(1, min(steps, (1 << 20) // B))


def select_picks(n, rows, u):
    """indices into the training-ray list: floor((k + u) n / rows) for k < rows, in float64 (each
    product is rounded once, as written), at most n - 1"""
    k = np.arange(rows, dtype=np.float64)
    r = np.floor((k + np.float64(u)) * np.float64(n) / np.float64(rows)).astype(np.int64)
    return np.minimum(r, n - 1)


def morton15(x32):
    """15-bit Morton code of positions in [0, 1]^3 (float32): cell q_a = min(trunc(32 x_a), 31)
    per axis; bit 3i + a of the code is bit i of q_a"""
    x32 = np.asarray(x32, np.float32)
    q = np.minimum((x32 * np.float32(32.0)).astype(np.int64), 31)
    code = np.zeros(len(x32), np.int64)
    for i in range(5):
        for a in range(3):
            code |= ((q[:, a] >> i) & 1) << (3 * i + a)
    return code


def group_order(x32):
    """row order of the grouped batch: by Morton code, ties in pick order"""
    return np.argsort(morton15(x32), kind="stable")


def step_rows(rows, B, k):
    """grouped rows of optimiser step k"""
    sub = rows // B
    return np.arange(k % sub, rows, sub)[:B]


# ---- FP8 (OCP e4m3: 1 sign, 4 exponent bits with bias 7, 3 mantissa bits, max 448, no
#      infinities, S.1111.111 = NaN) ----

def e4m3_decode(code):
    code = np.asarray(code, np.int64) & 0xFF
    s = np.where(code & 0x80, -1.0, 1.0)
    e = (code >> 3) & 0xF
    m = code & 7
    val = np.where(e == 0, m / 8.0 * 2.0 ** -6, (1 + m / 8.0) * 2.0 ** (e - 7))
    val = np.where((e == 15) & (m == 7), np.nan, val)
    return s * val


def e4m3_encode(x):
    """round-half-to-even to the nearest e4m3 value, saturating to +-448 (NaN stays NaN)"""
    x = np.asarray(x, np.float64)
    vals = e4m3_decode(np.arange(128))            # non-negative codes in increasing order
    finite = vals[:127]                           # drop NaN code 0x7F
    a = np.minimum(np.abs(x), 448.0)
    pos = np.searchsorted(finite, a)              # first value >= a
    pos = np.clip(pos, 1, 126)
    lo, hi = finite[pos - 1], finite[pos]
    pick_hi = (a - lo > hi - a) | ((a - lo == hi - a) & ((pos & 1) == 0))
    code = np.where(a <= finite[0], 0, np.where(pick_hi, pos, pos - 1))
    code = np.where(a >= 448.0, 126, code)
    code = code | np.where(np.signbit(x), 0x80, 0)
    return np.where(np.isnan(x), 0x7F, code).astype(np.uint8)

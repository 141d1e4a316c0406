"""CPU oracle of the GI-1.0 indirect-lighting pass -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import this package.
It wraps ``gi_oracle.c`` (plain C, built in FP32 parity mode and FP64 reference mode) through
ctypes, and ``learned.py`` (float64 numpy) for the learned radiance-cache surrogate.
It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS = {}

U32P = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
I32P = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
U64P = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
F32P = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
F64P = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")

NCELL = 64
STAT_NAMES = ["rays", "hits", "inserts", "overflow", "nonfinite", "wraps", "shadow", "occluded",
              "evict", "live", "relaxed", "noprobe", "bounce"]


class OrcConfig(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("rays_per_probe", C.c_uint32),
                ("table_log2", C.c_uint32), ("bounces", C.c_uint32), ("leak_bit", C.c_uint32),
                ("max_life", C.c_uint32), ("n_cap", C.c_uint32), ("seed", C.c_uint32),
                ("frac_bits", C.c_uint32), ("probe_filter", C.c_uint32), ("lod_scale", C.c_float),
                ("cell_scale", C.c_float), ("r_max", C.c_float), ("eps_scale", C.c_float),
                ("t_sky", C.c_float), ("sky", C.c_float * 4),
                ("temporal", C.c_uint32), ("upscale", C.c_uint32), ("ray_guiding", C.c_uint32),
                ("cache_tiles", C.c_uint32), ("tile_min_samples", C.c_uint32), ("light_grid", C.c_uint32),
                ("lgrid_dim", C.c_uint32), ("lgrid_k", C.c_uint32), ("ris_candidates", C.c_uint32), ("lgrid_threshold", C.c_float),
                ("restir", C.c_uint32), ("restir_log2", C.c_uint32), ("restir_cap", C.c_uint32),
                ("denoise", C.c_uint32), ("dn_hist_max", C.c_uint32), ("dn_radius", C.c_uint32),
                ("pad11", C.c_uint32), ("pad12", C.c_uint32)]


class OrcFrame(C.Structure):
    _fields_ = [("index", C.c_uint32), ("fov_y", C.c_float), ("tan_half", C.c_float),
                ("pad", C.c_float), ("pos", C.c_float * 4), ("fwd", C.c_float * 4),
                ("right", C.c_float * 4), ("up", C.c_float * 4)]


def default_config(**kw) -> dict:
    cfg = dict(width=128, height=128, rays_per_probe=16, table_log2=16, bounces=1, leak_bit=1,
               max_life=32, n_cap=256, seed=3, frac_bits=12, cell_scale=10.0, r_max=64.0,
               eps_scale=1e-4, t_sky=1e4, sky=(0.0, 0.0, 0.0), probe_filter=0, lod_scale=0.0,
               temporal=0, upscale=0, ray_guiding=0, cache_tiles=0, tile_min_samples=16, light_grid=0,
               lgrid_dim=16, lgrid_k=8, ris_candidates=4, lgrid_threshold=1e-3,
               restir=0, restir_log2=16, restir_cap=20, denoise=0, dn_hist_max=16, dn_radius=4)
    cfg.update(kw)
    return cfg


def set_threads(n: int) -> int:
    """Sets the OpenMP thread count of the oracle's parallel loops (the libgomp the oracle
    libraries link); returns the previous count."""
    _lib(False)
    gomp = C.CDLL("libgomp.so.1")
    prev = int(gomp.omp_get_max_threads())
    gomp.omp_set_num_threads(C.c_int(int(n)))
    return prev


def _lib(f64: bool):
    key = "64" if f64 else "32"
    if key in _LIBS:
        return _LIBS[key]
    path = os.path.join(HERE, f"liboracle{key}.so")
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    lib = C.CDLL(path)
    p = f"orc{key}_"
    R = F64P if f64 else F32P
    vp = C.c_void_p

    def fn(name, res, *args):
        f = getattr(lib, p + name)
        f.restype = res
        f.argtypes = list(args)
        return f
    fn("pcg", C.c_uint32, C.c_uint32)
    fn("xxh32", C.c_uint32, C.c_uint32)
    fn("rng", C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32)
    fn("sincos2pi", None, R, C.c_uint32, R, R)
    fn("halton_jitter", None, C.c_uint32, C.c_uint32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32))
    fn("scene_create", vp, F32P, C.c_uint32, U32P, C.c_uint32, U32P, F32P, C.c_uint32, C.c_uint32,
       C.c_int)
    fn("scene_set_dynamic", C.c_int, vp, F32P, U32P, C.c_uint32)
    fn("scene_destroy", None, vp)
    fn("scene_emitters", None, vp, C.POINTER(C.c_uint32), U32P, U32P, C.POINTER(C.c_double))
    fn("scene_normals", None, vp, R)
    fn("trace_closest", None, vp, R, R, C.c_uint32, C.c_double if f64 else C.c_float, U32P, R)
    fn("trace_any", None, vp, R, R, C.c_uint32, R, U32P)
    fn("pick_emitter", C.c_uint32, vp, C.c_uint32)
    fn("render_gbuffer", None, vp, C.POINTER(OrcFrame), C.c_uint32, C.c_uint32, R, R, R, U32P)
    fn("cell_moments", None, F64P)
    fn("cosine_dirs", None, R, R, R, C.c_uint32, R, U32P)
    fn("keys", None, C.POINTER(OrcConfig), R, R, R, R, C.c_uint32, U64P, U32P, U32P)
    fn("create", vp, C.POINTER(OrcConfig), vp)
    fn("destroy", None, vp)
    fn("distance_scale", C.c_float, C.c_float, C.c_uint32, C.c_uint32)
    fn("spawn", None, vp, C.POINTER(OrcFrame), R, R, U32P)
    fn("trace", None, vp, C.POINTER(OrcFrame))
    fn("update", None, vp, C.POINTER(OrcFrame))
    fn("probe_pass", None, vp, C.POINTER(OrcFrame))
    fn("interpolate", None, vp, C.POINTER(OrcFrame), R, R, U32P, R)
    fn("query", None, vp, R, R, C.c_uint32, R)
    fn("dims", None, vp, U32P)
    fn("export_probes", None, vp, U32P, R, R, R, R)
    fn("export_rays", None, vp, I32P, R, U32P, U32P, U64P, R)
    fn("export_hits", None, vp, R, R)
    fn("export_table", C.c_uint32, vp, U64P, U64P, U32P, R, U32P, U32P, C.c_uint32)
    fn("export_tiles", C.c_uint32, vp, U64P, U64P, U32P, U32P, R, U32P, R, C.c_uint32)
    fn("tile_keys", None, C.POINTER(OrcConfig), R, R, R, R, C.c_uint32, U64P, U32P)
    fn("prefilter", None, R, U32P, C.c_uint32, R)
    fn("light_grid_export", None, vp, R, U32P, U32P, U32P)
    fn("light_grid_set", None, vp, R, R)
    fn("restir_export", C.c_uint32, vp, U64P, U64P, R, R, R, U32P, U32P, C.c_uint32)
    fn("denoise", None, vp, C.POINTER(OrcFrame), R, R, U32P, R, R)
    fn("denoise_export", None, vp, R, U32P)
    fn("poke_cell", C.c_int, vp, C.c_uint64, U32P, R, C.c_uint32, C.c_uint32, C.c_uint32)
    fn("cache_update_only", None, vp)
    fn("stats", None, vp, U64P)
    fn("find_probe", C.c_uint32, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32)
    fn("sh_eval", None, R, R, C.c_uint32, R)
    fn("sh_project_atlas", None, vp, R, R, C.c_uint32, R)
    fn("filter_atlas", None, vp, C.POINTER(OrcFrame), C.c_int32, C.c_int32, R, R)
    fn("half_bits", C.c_uint32, C.c_float)
    fn("temporal_blend_atlas", None, R, R, C.c_uint32, R)
    fn("temporal_export", None, vp, U32P, U32P, U32P)
    fn("guiding_export", None, vp, R, U32P)
    fn("guided_dirs", None, R, U32P, U32P, R, R, C.c_uint32, R, U32P)
    fn("reconstruct_probe", None, R, R, C.c_double if f64 else C.c_float, C.c_uint32, R, R, R, R, U32P)
    fn("nee_samples", None, vp, C.POINTER(OrcFrame), R, R, U32P, C.c_uint32, R)
    fn("config_size", C.c_uint32)
    got = int(getattr(lib, p + "config_size")())
    if got != C.sizeof(OrcConfig):
        raise RuntimeError(f"oracle config struct is {got} bytes, its Python mirror {C.sizeof(OrcConfig)}")
    _LIBS[key] = (lib, p)
    return _LIBS[key]


def _call(f64, name, *args):
    lib, p = _lib(f64)
    return getattr(lib, p + name)(*args)


# ---------------------------------------------------------------------------------------
# small functions
# ---------------------------------------------------------------------------------------

def pcg(v: int) -> int:
    return _call(False, "pcg", v)


def xxh32(v: int) -> int:
    return _call(False, "xxh32", v)


def rng(seed, frame, gid, dim) -> int:
    return _call(False, "rng", seed, frame, gid, dim)


def sincos2pi(u, f64=False):
    dt = np.float64 if f64 else np.float32
    u = np.ascontiguousarray(u, dt)
    c = np.empty_like(u)
    s = np.empty_like(u)
    _call(f64, "sincos2pi", u, u.size, c, s)
    return c, s


def halton_jitter(frame: int, n: int = 8):
    """floor(n * Halton(frame + 1)) in bases 2 and 3"""
    jx, jy = C.c_uint32(), C.c_uint32()
    _call(False, "halton_jitter", frame, n, C.byref(jx), C.byref(jy))
    return jx.value, jy.value


def cell_moments() -> np.ndarray:
    out = np.zeros((64, 10), np.float64)
    _call(False, "cell_moments", out)
    return out


def distance_scale(fov_y: float, W: int, H: int) -> float:
    return _call(False, "distance_scale", fov_y, W, H)


def cosine_dirs(n, u0, u1, f64=False):
    dt = np.float64 if f64 else np.float32
    n = np.ascontiguousarray(n, dt)
    u0 = np.ascontiguousarray(u0, dt)
    u1 = np.ascontiguousarray(u1, dt)
    d = np.zeros((len(u0), 3), dt)
    cell = np.zeros(len(u0), np.uint32)
    _call(f64, "cosine_dirs", n, u0, u1, len(u0), d, cell)
    return d, cell


def guided_dirs(n, cdf, r, u0, u1, f64=False):
    """ray guiding's sampling for one probe with unit normal n and inclusive weight sums cdf
    [64]: per ray, the cell picked by the 32-bit number r and the direction of the point
    (u0, u1) inside it"""
    dt = np.float64 if f64 else np.float32
    n = np.ascontiguousarray(n, dt)
    cdf = np.ascontiguousarray(cdf, np.uint32)
    r = np.ascontiguousarray(r, np.uint32)
    u0 = np.ascontiguousarray(u0, dt)
    u1 = np.ascontiguousarray(u1, dt)
    d = np.zeros((len(r), 3), dt)
    cell = np.zeros(len(r), np.uint32)
    _call(f64, "guided_dirs", n, cdf, r, u0, u1, len(r), d, cell)
    return d, cell


def reconstruct_probe(pp, pn, cs, qpos, qnrm, qatlas, f64=True):
    """ray guiding's parallax-corrected reconstruction of one probe (position pp, unit normal
    pn, cell size cs) from up to 9 previous probes (positions, normals, atlases [n, 64, 4]);
    returns the reconstruction [64, 4] (distance -1 where empty) and the weight sums [64]"""
    dt = np.float64 if f64 else np.float32
    qpos = np.zeros((0, 4), dt) if len(qpos) == 0 else np.ascontiguousarray(np.asarray(qpos, dt).reshape(-1, 4))
    qnrm = np.zeros((0, 4), dt) if len(qnrm) == 0 else np.ascontiguousarray(np.asarray(qnrm, dt).reshape(-1, 4))
    qatlas = np.zeros((0, NCELL, 4), dt) if len(qatlas) == 0 else np.ascontiguousarray(qatlas, dt)
    recon = np.zeros((NCELL, 4), dt)
    cdf = np.zeros(NCELL, np.uint32)
    p3 = np.zeros(4, dt)
    p3[:3] = pp[:3]
    n3 = np.zeros(4, dt)
    n3[:3] = pn[:3]
    _call(f64, "reconstruct_probe", p3, n3, cs, len(qpos), qpos, qnrm, qatlas, recon, cdf)
    return recon, cdf


def half_bits(x: float) -> int:
    """IEEE binary16 bits of a non-negative float32, round to nearest even"""
    return int(_call(False, "half_bits", float(x)))


def temporal_blend(curr, prev, f64=True):
    """Algorithm 3 on cells [n][4] (rgb, travelled distance)"""
    dt = np.float64 if f64 else np.float32
    c = np.ascontiguousarray(curr, dt).reshape(-1, 4)
    q = np.ascontiguousarray(prev, dt).reshape(-1, 4)
    out = np.zeros_like(c)
    _call(f64, "temporal_blend_atlas", c, q, len(c), out)
    return out


def keys(cfg: dict, y, n, t, f64=False, cam=(0.0, 0.0, 0.0)):
    """descriptor, bucket and fingerprint of points y with normals n and ray lengths t; cam is
    the camera position the levels of detail are measured from"""
    dt = np.float64 if f64 else np.float32
    cam = np.ascontiguousarray(cam, dt)
    y = np.ascontiguousarray(y, dt)
    n = np.ascontiguousarray(n, dt)
    t = np.ascontiguousarray(t, dt)
    cnt = len(t)
    key = np.zeros(cnt, np.uint64)
    b = np.zeros(cnt, np.uint32)
    fp = np.zeros(cnt, np.uint32)
    c = make_config(cfg)
    _call(f64, "keys", C.byref(c), cam, y, n, t, cnt, key, b, fp)
    return key, b, fp


def tile_keys(cfg: dict, y, n, t, f64=False, cam=(0.0, 0.0, 0.0)):
    """two-level cache: tile descriptor and the cell inside the tile of points y with normals n"""
    dt = np.float64 if f64 else np.float32
    cam = np.ascontiguousarray(cam, dt)
    y = np.ascontiguousarray(y, dt)
    n = np.ascontiguousarray(n, dt)
    t = np.ascontiguousarray(t, dt)
    key = np.zeros(len(t), np.uint64)
    cell = np.zeros(len(t), np.uint32)
    c = make_config(dict(cfg, cache_tiles=1))
    _call(f64, "tile_keys", C.byref(c), cam, y, n, t, len(t), key, cell)
    return key, cell


def prefilter(L0, n0, T, f64=True):
    """the tile MIP levels and query radiance of one tile's 64 cells (rgb [64, 3], samples [64])"""
    dt = np.float64 if f64 else np.float32
    out = np.zeros((NCELL, 3), dt)
    _call(f64, "prefilter", np.ascontiguousarray(L0, dt), np.ascontiguousarray(n0, np.uint32), T, out)
    return out


def sh_eval(coef, n, f64=False):
    dt = np.float64 if f64 else np.float32
    coef = np.ascontiguousarray(coef, dt).reshape(-1, 27)
    n = np.ascontiguousarray(n, dt).reshape(-1, 3)
    E = np.zeros((len(n), 3), dt)
    _call(f64, "sh_eval", coef, n, len(n), E)
    return E


def make_config(cfg: dict) -> OrcConfig:
    c = OrcConfig()
    for k, v in cfg.items():
        if k == "sky":
            for i in range(3):
                c.sky[i] = float(v[i])
        elif hasattr(c, k):
            setattr(c, k, v)
    return c


def make_frame(fr) -> OrcFrame:
    f = OrcFrame()
    f.index = fr.index
    f.fov_y = fr.fov_y
    f.tan_half = fr.tan_half
    for name in ("pos", "fwd", "right", "up"):
        v = getattr(fr, name)
        arr = getattr(f, name)
        for i in range(3):
            arr[i] = float(v[i])
    return f


# ---------------------------------------------------------------------------------------
# scene and frame state
# ---------------------------------------------------------------------------------------

class OracleScene:
    def __init__(self, scene, f64=False, use_bvh=None, nd_cap=64):
        self.f64 = f64
        self.dt = np.float64 if f64 else np.float32
        if use_bvh is None:
            use_bvh = scene.n_tris > 2048
        self.src = scene
        self.h = _call(f64, "scene_create", np.ascontiguousarray(scene.verts, np.float32),
                       len(scene.verts), np.ascontiguousarray(scene.idx, np.uint32), scene.n_tris,
                       np.ascontiguousarray(scene.tri_mat, np.uint32),
                       np.ascontiguousarray(scene.materials, np.float32), len(scene.materials),
                       nd_cap, int(use_bvh))
        self.nt = scene.n_tris
        self.nd = 0

    def set_dynamic(self, tv, mats):
        tv = np.ascontiguousarray(tv, np.float32).reshape(-1, 9)
        mats = np.ascontiguousarray(mats, np.uint32)
        if _call(self.f64, "scene_set_dynamic", self.h, tv, mats, len(mats)) != 0:
            raise ValueError("too many dynamic triangles")
        self.nd = len(mats)

    def set_frame_dynamic(self, frame_index: int):
        if self.src.dynamic is not None:
            tv, m = self.src.dynamic(frame_index)
            self.set_dynamic(tv, m)

    def emitters(self):
        ne = C.c_uint32()
        n = self.nt + 64
        etri = np.zeros(n, np.uint32)
        ethr = np.zeros(n, np.uint32)
        area = C.c_double()
        _call(self.f64, "scene_emitters", self.h, C.byref(ne), etri, ethr, C.byref(area))
        return etri[:ne.value].copy(), ethr[:ne.value].copy(), area.value

    def normals(self):
        out = np.zeros((self.nt + self.nd, 3), self.dt)
        _call(self.f64, "scene_normals", self.h, out)
        return out

    def closest(self, o, d, tmax=3.0e38):
        o = np.ascontiguousarray(o, self.dt)
        d = np.ascontiguousarray(d, self.dt)
        n = len(o)
        tri = np.zeros(n, np.uint32)
        t = np.zeros(n, self.dt)
        _call(self.f64, "trace_closest", self.h, o, d, n, tmax, tri, t)
        return tri, t

    def any(self, o, d, tmax):
        o = np.ascontiguousarray(o, self.dt)
        d = np.ascontiguousarray(d, self.dt)
        tm = np.ascontiguousarray(np.broadcast_to(tmax, (len(o),)), self.dt)
        hit = np.zeros(len(o), np.uint32)
        _call(self.f64, "trace_any", self.h, o, d, len(o), tm, hit)
        return hit

    def pick_emitter(self, r: int) -> int:
        return _call(self.f64, "pick_emitter", self.h, r)

    def gbuffer(self, frame, W, H):
        pos = np.zeros((H, W, 4), self.dt)
        nrm = np.zeros((H, W, 4), self.dt)
        alb = np.zeros((H, W, 4), self.dt)
        prim = np.zeros((H, W), np.uint32)
        f = make_frame(frame)
        _call(self.f64, "render_gbuffer", self.h, C.byref(f), W, H, pos, nrm, alb, prim)
        return pos, nrm, alb, prim

    def __del__(self):
        try:
            _call(self.f64, "scene_destroy", self.h)
        except Exception:
            pass


class OracleFrameState:
    """World cache, probes and rays of one context; methods follow the frame order."""

    def __init__(self, scene: OracleScene, cfg: dict):
        self.scene = scene
        self.f64 = scene.f64
        self.dt = scene.dt
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        self.h = _call(self.f64, "create", C.byref(self._c), scene.h)
        d = np.zeros(9, np.uint32)
        _call(self.f64, "dims", self.h, d)
        self.P, self.R, self.N, self.TW, self.TH, self.nmip, self.mask_total = (int(x) for x in d[:7])

    def dims(self):
        d = np.zeros(9, np.uint32)
        _call(self.f64, "dims", self.h, d)
        return d

    def spawn(self, frame, gpos, gnrm, gprim):
        self._f = make_frame(frame)
        self._g = (np.ascontiguousarray(gpos, self.dt), np.ascontiguousarray(gnrm, self.dt),
                   np.ascontiguousarray(gprim, np.uint32))
        _call(self.f64, "spawn", self.h, C.byref(self._f), *self._g)

    def trace(self, frame):
        f = make_frame(frame)
        _call(self.f64, "trace", self.h, C.byref(f))

    def update(self, frame):
        f = make_frame(frame)
        _call(self.f64, "update", self.h, C.byref(f))

    def interpolate(self, frame, gpos, gnrm, gprim):
        H, W = gprim.shape
        out = np.zeros((H, W, 4), self.dt)
        f = make_frame(frame)
        _call(self.f64, "interpolate", self.h, C.byref(f), np.ascontiguousarray(gpos, self.dt),
              np.ascontiguousarray(gnrm, self.dt), np.ascontiguousarray(gprim, np.uint32), out)
        return out

    def frame(self, frame, gbuf):
        """spawn -> trace -> update (+gather, SH) -> interpolate for one frame"""
        pos, nrm, _alb, prim = gbuf
        self.spawn(frame, pos, nrm, prim)
        self.trace(frame)
        self.update(frame)
        return self.interpolate(frame, pos, nrm, prim)

    def query(self, pos, nrm):
        pos = np.ascontiguousarray(pos, self.dt)
        nrm = np.ascontiguousarray(nrm, self.dt)
        out = np.zeros((len(pos), 4), self.dt)
        _call(self.f64, "query", self.h, pos, nrm, len(pos), out)
        return out

    def probes(self):
        mask = np.zeros(self.mask_total, np.uint32)
        ppos = np.zeros((self.P, 4), self.dt)
        pnrm = np.zeros((self.P, 4), self.dt)
        atlas = np.zeros((self.P, NCELL, 4), self.dt)
        sh = np.zeros((self.P, 27), self.dt)
        _call(self.f64, "export_probes", self.h, mask, ppos, pnrm, atlas, sh)
        return dict(mask=mask, pos=ppos, nrm=pnrm, atlas=atlas, sh=sh)

    def rays(self):
        n = self.P * self.R
        slot = np.zeros(n, np.int32)
        t = np.zeros(n, self.dt)
        tri = np.zeros(n, np.uint32)
        cell = np.zeros(n, np.uint32)
        key = np.zeros(n, np.uint64)
        sample = np.zeros((n, 3), self.dt)
        _call(self.f64, "export_rays", self.h, slot, t, tri, cell, key, sample)
        return dict(slot=slot, t=t, tri=tri, cell=cell, key=key, sample=sample)

    def hits(self):
        """hit point y and face-forwarded normal ny [P*R, 3] of the last trace (rows of rays
        that missed hold stale values)"""
        n = self.P * self.R
        y = np.zeros((n, 3), self.dt)
        ny = np.zeros((n, 3), self.dt)
        _call(self.f64, "export_hits", self.h, y, ny)
        return y, ny

    def table(self):
        cap = self.N
        ident = np.zeros(cap, np.uint64)
        key = np.zeros(cap, np.uint64)
        acc = np.zeros((cap, 4), np.uint32)
        L = np.zeros((cap, 3), self.dt)
        nh = np.zeros(cap, np.uint32)
        life = np.zeros(cap, np.uint32)
        n = _call(self.f64, "export_table", self.h, ident, key, acc, L, nh, life, cap)
        order = np.argsort(ident[:n], kind="stable")
        return dict(id=ident[:n][order], key=key[:n][order], acc=acc[:n][order], L=L[:n][order],
                    nhist=nh[:n][order], life=life[:n][order])

    def tiles(self):
        """two-level cache: live tiles sorted by (bucket, fingerprint), with per-cell fixed-point
        sums, moving averages, sample counts and the prefiltered query radiance"""
        cap = self.N
        ident = np.zeros(cap, np.uint64)
        key = np.zeros(cap, np.uint64)
        life = np.zeros(cap, np.uint32)
        acc = np.zeros((cap, NCELL, 4), np.uint32)
        L = np.zeros((cap, NCELL, 3), self.dt)
        nh = np.zeros((cap, NCELL), np.uint32)
        Lq = np.zeros((cap, NCELL, 3), self.dt)
        n = _call(self.f64, "export_tiles", self.h, ident, key, life, acc, L, nh, Lq, cap)
        o = np.argsort(ident[:n], kind="stable")
        return dict(id=ident[:n][o], key=key[:n][o], life=life[:n][o], acc=acc[:n][o], L=L[:n][o],
                    nhist=nh[:n][o], Lq=Lq[:n][o])

    def denoise(self, frame, gpos, gnrm, gprim, irr):
        """the denoiser over this frame's interpolated irradiance irr [H, W, 4] (rgb, flag)"""
        H, W = gprim.shape
        out = np.zeros((H, W, 4), self.dt)
        f = make_frame(frame)
        _call(self.f64, "denoise", self.h, C.byref(f), np.ascontiguousarray(gpos, self.dt),
              np.ascontiguousarray(gnrm, self.dt), np.ascontiguousarray(gprim, np.uint32),
              np.ascontiguousarray(irr, self.dt), out)
        return out

    def denoise_state(self):
        """the accumulated irradiance and history length [H, W, 4], and the radius per pixel"""
        H, W = int(self.cfg["height"]), int(self.cfg["width"])
        hist = np.zeros((H, W, 4), self.dt)
        rad = np.zeros((H, W), np.uint32)
        _call(self.f64, "denoise_export", self.h, hist, rad)
        return hist, rad

    def reservoirs(self):
        """the reservoir table written by the last trace (restir): sorted by (bucket,
        fingerprint): key, light point, contribution weight, normal, light, count"""
        cap = 1 << int(self.cfg.get("restir_log2", 16))
        ident = np.zeros(cap, np.uint64)
        key = np.zeros(cap, np.uint64)
        y = np.zeros((cap, 3), self.dt)
        W = np.zeros(cap, self.dt)
        n = np.zeros((cap, 3), self.dt)
        k = np.zeros(cap, np.uint32)
        M = np.zeros(cap, np.uint32)
        c = _call(self.f64, "restir_export", self.h, ident, key, y, W, n, k, M, cap)
        o = np.argsort(ident[:c], kind="stable")
        return dict(id=ident[:c][o], key=key[:c][o], y=y[:c][o], W=W[:c][o], n=n[:c][o], k=k[:c][o], M=M[:c][o])

    def light_grid_set(self, lo, hi):
        """build the light grid over the box [lo, hi] (as a trace does over its hit points)"""
        _call(self.f64, "light_grid_set", self.h, np.ascontiguousarray(lo, self.dt), np.ascontiguousarray(hi, self.dt))

    def light_grid(self):
        """after a trace with light_grid: origin and cell side, dims, per cell the light list
        (indices into the emitter list) and its length"""
        geom = np.zeros(4, self.dt)
        dims = np.zeros(3, np.uint32)
        D = int(self.cfg.get("lgrid_dim", 16))
        K = int(self.cfg.get("lgrid_k", 8))
        lst = np.zeros(D * D * D * K, np.uint32)
        cnt = np.zeros(D * D * D, np.uint32)
        _call(self.f64, "light_grid_export", self.h, geom, dims, lst, cnt)
        n = int(np.prod(dims))
        return dict(lo=geom[:3].copy(), h=float(geom[3]), dims=dims, list=lst[:n * K].reshape(n, K), count=cnt[:n])

    def poke_cell(self, key, acc4, L3, nhist, life, accessed):
        return _call(self.f64, "poke_cell", self.h, key, np.ascontiguousarray(acc4, np.uint32),
                     np.ascontiguousarray(L3, self.dt), nhist, life, accessed)

    def cache_update_only(self):
        _call(self.f64, "cache_update_only", self.h)

    def probe_pass(self, frame):
        """the per-probe half of update(): gather, backup, blend / filter if configured, SH;
        cache_update_only() followed by probe_pass() is update()"""
        f = make_frame(frame)
        _call(self.f64, "probe_pass", self.h, C.byref(f))

    def stats(self):
        out = np.zeros(16, np.uint64)
        _call(self.f64, "stats", self.h, out)
        return {k: int(out[i]) for i, k in enumerate(STAT_NAMES)}

    def find_probe(self, px, py, ox, oy):
        return _call(self.f64, "find_probe", self.h, px, py, ox, oy)

    def nee(self, frame, y, ny, ids):
        """E/pi estimates (one light sample and one shadow ray each) at a point"""
        ids = np.ascontiguousarray(ids, np.uint32)
        out = np.zeros((len(ids), 3), self.dt)
        f = make_frame(frame)
        _call(self.f64, "nee_samples", self.h, C.byref(f), np.ascontiguousarray(y, self.dt),
              np.ascontiguousarray(ny, self.dt), ids, len(ids), out)
        return out

    def temporal(self, with_traced=False):
        """per tile: the pixel (mask encoding) the previous frame's probe moved to and the
        previous tile it came from (SENTINEL where none), after the last spawn; with_traced
        adds whether the tile's probe traces rays this frame"""
        P = int(self.dims()[0])
        win = np.zeros(P, np.uint32)
        hist = np.zeros(P, np.uint32)
        traced = np.zeros(P, np.uint32)
        _call(self.f64, "temporal_export", self.h, win, hist, traced)
        return (win, hist, traced) if with_traced else (win, hist)

    def guiding(self):
        """after a spawn with ray guiding: the reconstruction [P, 64, 4] (rgb, distance; the
        distance is -1 in empty cells) and the inclusive weight sums [P, 64]"""
        recon = np.zeros((self.P, NCELL, 4), self.dt)
        cdf = np.zeros((self.P, NCELL), np.uint32)
        _call(self.f64, "guiding_export", self.h, recon, cdf)
        return recon, cdf

    def filter_atlas(self, frame, axis, atlas):
        """one pass of the probe-space filter (Algorithm 5) along axis 0 (x) or 1 (y) over an
        atlas [P][64][4], with the probes of the last spawn"""
        a = np.ascontiguousarray(atlas, self.dt).reshape(-1, NCELL, 4)
        out = np.zeros_like(a)
        f = make_frame(frame)
        _call(self.f64, "filter_atlas", self.h, C.byref(f), 1 if axis == 0 else 0, 1 if axis == 1 else 0, a, out)
        return out

    def sh_project(self, atlas, nrm):
        atlas = np.ascontiguousarray(atlas, self.dt).reshape(-1, NCELL, 4)
        nrm = np.ascontiguousarray(nrm, self.dt).reshape(-1, 3)
        out = np.zeros((len(nrm), 27), self.dt)
        _call(self.f64, "sh_project_atlas", self.h, atlas, nrm, len(nrm), out)
        return out

    def __del__(self):
        try:
            _call(self.f64, "destroy", self.h)
        except Exception:
            pass

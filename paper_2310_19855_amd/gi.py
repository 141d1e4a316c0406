"""Python binding of libgi.so (the C ABI in include/gi.h): argument marshalling only.

Device memory and streams come from PyTorch tensors; every step of the pass runs in the
library's HIP kernels.  Importing this module does not need a GPU; creating a Context does,
and fails loudly if the library is missing or the device is not gfx950.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgi.so")

GI_OK = 0
ERRORS = {-1: "GI_ERR_INVALID_ARG", -2: "GI_ERR_OOM", -3: "GI_ERR_HIP", -4: "GI_ERR_STATE",
          -5: "GI_ERR_UNSUPPORTED", -6: "GI_ERR_INTERNAL"}
CACHE_PLAIN, CACHE_MLP_BF16, CACHE_MLP_FP8 = 0, 1, 2
RAY_HIT, RAY_FRONT, RAY_EMIT, RAY_TRACED = 0x100, 0x200, 0x400, 0x10000
# per-pixel flags of the interpolation output (alpha channel): GI_INTERP_* of include/gi.h
INTERP_OK, INTERP_RELAXED, INTERP_NO_PROBE, INTERP_SKY = 0.0, 1.0, 2.0, 3.0
STAT_NAMES = ["rays", "hits", "inserts", "overflow", "nonfinite", "wraps", "shadow", "occluded",
              "evict", "live", "relaxed", "noprobe", "bounce", "mlp_skipped", "mlp_fallback", "_15"]


class GIError(RuntimeError):
    pass


class Config(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("rays_per_probe", C.c_uint32),
                ("table_log2", C.c_uint32), ("bounces", C.c_uint32), ("leak_bit", C.c_uint32),
                ("max_life", C.c_uint32), ("n_cap", C.c_uint32), ("seed", C.c_uint32),
                ("frac_bits", C.c_uint32), ("cache_mode", C.c_uint32), ("probe_filter", C.c_uint32),
                ("cell_scale", C.c_float), ("r_max", C.c_float), ("eps_scale", C.c_float),
                ("t_sky", C.c_float), ("sky", C.c_float * 4),
                ("mlp_batch_log2", C.c_uint32), ("mlp_levels", C.c_uint32),
                ("mlp_table_log2", C.c_uint32), ("mlp_steps", C.c_uint32),
                ("mlp_lr_grid", C.c_float), ("mlp_lr_mlp", C.c_float),
                ("mlp_loss_scale", C.c_float), ("mlp_judge", C.c_float),
                ("scene_min", C.c_float * 4), ("scene_max", C.c_float * 4),
                ("lod_scale", C.c_float), ("temporal", C.c_uint32), ("upscale", C.c_uint32),
                ("ray_guiding", C.c_uint32), ("cache_tiles", C.c_uint32), ("tile_min_samples", C.c_uint32),
                ("light_grid", C.c_uint32), ("ris_candidates", C.c_uint32), ("lgrid_dim", C.c_uint32),
                ("lgrid_k", C.c_uint32), ("lgrid_threshold", C.c_float), ("restir", C.c_uint32),
                ("restir_log2", C.c_uint32), ("restir_cap", C.c_uint32)]


class Frame(C.Structure):
    _fields_ = [("index", C.c_uint32), ("fov_y", C.c_float), ("tan_half", C.c_float),
                ("pad", C.c_float), ("pos", C.c_float * 4), ("fwd", C.c_float * 4),
                ("right", C.c_float * 4), ("up", C.c_float * 4)]


DEFAULTS = dict(width=128, height=128, rays_per_probe=16, table_log2=16, bounces=1, leak_bit=1,
                max_life=32, n_cap=256, seed=3, frac_bits=12, cache_mode=CACHE_PLAIN,
                cell_scale=10.0, r_max=64.0, eps_scale=1e-4, t_sky=1e4, sky=(0.0, 0.0, 0.0),
                mlp_batch_log2=14, mlp_levels=16, mlp_table_log2=19, mlp_steps=4,
                mlp_lr_grid=1e-2, mlp_lr_mlp=1e-2, mlp_loss_scale=128.0, mlp_judge=0.1, tile_min_samples=16,
                ris_candidates=4, lgrid_dim=16, lgrid_k=8, lgrid_threshold=1e-3, restir_log2=16,
                restir_cap=20)

_lib = None


def lib():
    """Load libgi.so; raises if it was not built (no fallback of any kind)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GIError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, u32, u64, f32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_float
    sz = C.c_size_t
    P = C.POINTER

    def fn(name, res, *args):
        f = getattr(L, name)
        f.restype = res
        f.argtypes = list(args)
    st = C.c_int32
    fn("gi_version", C.c_char_p)
    fn("gi_create", st, P(Config), P(vp))
    fn("gi_destroy", None, vp)
    fn("gi_last_error", C.c_char_p, vp)
    fn("gi_build_bvh", st, vp, vp, u32, vp, u32, vp, vp, u32)
    fn("gi_bvh_build_host", st, vp, u32, vp, u32, vp, u32, P(u32), P(u32), P(u32))
    fn("gi_tiles_export", st, vp, vp, vp, vp, vp, vp, vp, vp, u32, P(u32))
    fn("gi_light_grid_export", st, vp, vp, vp, vp, vp, u32)
    fn("gi_restir_export", st, vp, vp, vp, vp, vp, vp, vp, u32, P(u32))
    fn("gi_denoiser_create", st, u32, u32, u32, u32, P(vp))
    fn("gi_denoiser_destroy", None, vp)
    fn("gi_denoiser_reset", st, vp)
    fn("gi_denoise", st, vp, P(Frame), vp, vp, vp, vp, vp, vp)
    fn("gi_denoiser_export", st, vp, vp, vp)
    fn("gi_set_dynamic_triangles", st, vp, vp, vp, u32, vp)
    fn("gi_render_gbuffer", st, vp, P(Frame), vp, vp, vp, vp, vp)
    fn("gi_spawn_probes", st, vp, P(Frame), vp, vp, vp, vp)
    fn("gi_trace_probes", st, vp, P(Frame), vp)
    fn("gi_cache_update", st, vp, P(Frame), vp)
    fn("gi_interpolate_probes", st, vp, P(Frame), vp, vp, vp, vp, vp)
    fn("gi_cache_query", st, vp, vp, vp, u32, vp, vp)
    fn("gi_trace_rays", st, vp, vp, vp, u32, u32, vp, vp, vp)
    fn("gi_trace_rays_noalloc", st, vp, vp, vp, u32, u32, vp, vp, vp)
    fn("gi_measure_traversal", st, vp, vp, vp)
    fn("gi_learned_train", st, vp, P(Frame), vp)
    fn("gi_learned_query", st, vp, vp, vp, u32, vp, vp)
    fn("gi_e4m3_encode", st, vp, vp, vp, u32, vp)
    fn("gi_learned_step", st, vp, vp, vp, vp, u32, u32, vp)
    fn("gi_cache_export", st, vp, vp, vp, vp, vp, vp, vp, u32, P(u32))
    fn("gi_cache_save", st, vp, vp, sz, P(sz))
    fn("gi_cache_load", st, vp, vp, sz)
    fn("gi_cache_import", st, vp, vp, sz)
    fn("gi_rays_export", st, vp, vp, vp, vp, vp, vp)
    fn("gi_probes_export", st, vp, vp, vp, vp, vp, vp)
    fn("gi_get_dims", st, vp, vp)
    fn("gi_get_stats", st, vp, vp)
    fn("gi_reset_stats", st, vp, vp)
    fn("gi_profile_enable", st, vp, u32)
    fn("gi_profile_read", st, vp, vp, sz, vp, vp, u32, P(u32))
    fn("gi_learned_save", st, vp, vp, sz, P(sz))
    fn("gi_learned_load", st, vp, vp, sz)
    fn("gi_learned_export", st, vp, vp, sz, P(sz))
    fn("gi_learned_import", st, vp, vp, sz)
    fn("gi_learned_stats", st, vp, vp)
    fn("gi_learned_batch_export", st, vp, vp, vp, u32, P(u32), P(u32))
    _lib = L
    return L


NODE_DTYPE = np.dtype([("lo_x", "<f4", 4), ("hi_x", "<f4", 4), ("lo_y", "<f4", 4), ("hi_y", "<f4", 4),
                       ("lo_z", "<f4", 4), ("hi_z", "<f4", 4), ("child", "<u4", 4), ("pad", "<u4", 4)])


def build_bvh_host(tri_verts):
    """The 4-wide BVH that gi_build_bvh builds, on the host: (nodes as a NODE_DTYPE array,
    triangle index of every leaf slot, depth).  tri_verts: float32 [n][9]."""
    tv = np.ascontiguousarray(tri_verts, np.float32).reshape(-1, 9)
    n = C.c_uint32(0)
    ns = C.c_uint32(0)
    d = C.c_uint32(0)
    L = lib()
    st = L.gi_bvh_build_host(tv.ctypes.data, tv.shape[0], None, 0, None, 0, C.byref(n), C.byref(ns), C.byref(d))
    if st != 0:
        raise GIError(f"gi_bvh_build_host: status {st}")
    nodes = np.zeros(n.value, NODE_DTYPE)
    slots = np.zeros(ns.value, np.uint32)
    st = L.gi_bvh_build_host(tv.ctypes.data, tv.shape[0], nodes.ctypes.data, n.value, slots.ctypes.data, ns.value,
                             C.byref(n), C.byref(ns), C.byref(d))
    if st != 0:
        raise GIError(f"gi_bvh_build_host: status {st}")
    return nodes, slots, int(d.value)


def make_config(**kw) -> Config:
    d = dict(DEFAULTS)
    d.update(kw)
    c = Config()
    for k, v in d.items():
        if k in ("sky", "scene_min", "scene_max"):
            arr = getattr(c, k)
            for i, x in enumerate(v):
                arr[i] = float(x)
        else:
            setattr(c, k, v)
    return c


def make_frame(fr) -> Frame:
    f = Frame()
    f.index = fr.index
    f.fov_y = fr.fov_y
    f.tan_half = fr.tan_half
    for name in ("pos", "fwd", "right", "up"):
        v = getattr(fr, name)
        a = getattr(f, name)
        for i in range(3):
            a[i] = float(v[i])
    return f


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


class Context:
    """One world cache, probe set and scene on the current device (calls in frame order)."""

    def __init__(self, **cfg):
        L = lib()
        self.cfg = make_config(**cfg)
        self.cfg_dict = dict(DEFAULTS, **cfg)
        h = C.c_void_p()
        st = L.gi_create(C.byref(self.cfg), C.byref(h))
        if st != GI_OK:
            raise GIError(f"gi_create failed: {ERRORS.get(st, st)}")
        self.h = h
        self._keep = []

    def _check(self, st, what):
        if st != GI_OK:
            msg = lib().gi_last_error(self.h)
            raise GIError(f"{what}: {ERRORS.get(st, st)}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "h", None):
            lib().gi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- scene ---
    def build_bvh(self, scene):
        v = np.ascontiguousarray(scene.verts, np.float32)
        i = np.ascontiguousarray(scene.idx, np.uint32)
        m = np.ascontiguousarray(scene.tri_mat, np.uint32)
        mats = np.ascontiguousarray(scene.materials, np.float32)
        self._check(lib().gi_build_bvh(self.h, v.ctypes.data, len(v), i.ctypes.data, len(i),
                                       m.ctypes.data, mats.ctypes.data, len(mats)), "gi_build_bvh")

    def set_dynamic(self, tv, mats, stream=None):
        tv = np.ascontiguousarray(tv, np.float32).reshape(-1, 9)
        mats = np.ascontiguousarray(mats, np.uint32)
        self._check(lib().gi_set_dynamic_triangles(self.h, tv.ctypes.data, mats.ctypes.data, len(mats),
                                                   _stream(stream)), "gi_set_dynamic_triangles")

    def render_gbuffer(self, frame, pos, nrm, alb, prim, stream=None):
        f = make_frame(frame)
        self._check(lib().gi_render_gbuffer(self.h, C.byref(f), _ptr(pos), _ptr(nrm), _ptr(alb),
                                            _ptr(prim), _stream(stream)), "gi_render_gbuffer")

    # --- frame ---
    def spawn_probes(self, frame, pos, nrm, prim, stream=None):
        f = make_frame(frame)
        self._check(lib().gi_spawn_probes(self.h, C.byref(f), _ptr(pos), _ptr(nrm), _ptr(prim),
                                          _stream(stream)), "gi_spawn_probes")

    def trace_probes(self, frame, stream=None):
        f = make_frame(frame)
        self._check(lib().gi_trace_probes(self.h, C.byref(f), _stream(stream)), "gi_trace_probes")

    def learned_train(self, frame, stream=None):
        f = make_frame(frame)
        self._check(lib().gi_learned_train(self.h, C.byref(f), _stream(stream)), "gi_learned_train")

    def cache_update(self, frame, stream=None):
        f = make_frame(frame)
        self._check(lib().gi_cache_update(self.h, C.byref(f), _stream(stream)), "gi_cache_update")

    def interpolate_probes(self, frame, pos, nrm, prim, out, stream=None):
        f = make_frame(frame)
        self._check(lib().gi_interpolate_probes(self.h, C.byref(f), _ptr(pos), _ptr(nrm), _ptr(prim),
                                                _ptr(out), _stream(stream)), "gi_interpolate_probes")

    def cache_query(self, pos, nrm, out, stream=None):
        self._check(lib().gi_cache_query(self.h, _ptr(pos), _ptr(nrm), pos.shape[0], _ptr(out),
                                          _stream(stream)), "gi_cache_query")

    def learned_query(self, pos, nrm, out, stream=None):
        self._check(lib().gi_learned_query(self.h, _ptr(pos), _ptr(nrm), pos.shape[0], _ptr(out),
                                           _stream(stream)), "gi_learned_query")

    def e4m3_encode(self, x, out, stream=None):
        """OCP e4m3 codes of the float32 device array x into the uint8 device array out"""
        self._check(lib().gi_e4m3_encode(self.h, _ptr(x), _ptr(out), x.numel(), _stream(stream)), "gi_e4m3_encode")

    def learned_step(self, pos, nrm, target, apply=True, stream=None):
        self._check(lib().gi_learned_step(self.h, _ptr(pos), _ptr(nrm), _ptr(target), pos.shape[0], int(apply),
                                          _stream(stream)), "gi_learned_step")

    def trace_rays(self, o, d, tri, t, any_hit=False, stream=None):
        self._check(lib().gi_trace_rays(self.h, _ptr(o), _ptr(d), o.shape[0], int(any_hit), _ptr(tri),
                                        _ptr(t), _stream(stream)), "gi_trace_rays")

    def trace_rays_noalloc(self, o, d, tri, t, any_hit=False, stream=None):
        self._check(lib().gi_trace_rays_noalloc(self.h, _ptr(o), _ptr(d), o.shape[0], int(any_hit), _ptr(tri),
                                                _ptr(t), _stream(stream)), "gi_trace_rays_noalloc")

    def measure_traversal(self, stream=None):
        out = np.zeros(8, np.uint64)
        self._check(lib().gi_measure_traversal(self.h, out.ctypes.data, _stream(stream)),
                    "gi_measure_traversal")
        keys = ["probe_rays", "probe_nodes", "probe_tris", "shadow_rays", "shadow_nodes", "shadow_tris"]
        return {k: int(out[i]) for i, k in enumerate(keys)}

    # --- exports ---
    def dims(self):
        out = np.zeros(16, np.uint32)
        self._check(lib().gi_get_dims(self.h, out.ctypes.data), "gi_get_dims")
        return out

    def stats(self):
        out = np.zeros(16, np.uint64)
        self._check(lib().gi_get_stats(self.h, out.ctypes.data), "gi_get_stats")
        return {k: int(out[i]) for i, k in enumerate(STAT_NAMES)}

    def reset_stats(self, stream=None):
        self._check(lib().gi_reset_stats(self.h, _stream(stream)), "gi_reset_stats")

    def rays(self):
        d = self.dims()
        n = int(d[0]) * int(d[1])
        slot = np.zeros(n, np.int32)
        t = np.zeros(n, np.float32)
        tri = np.zeros(n, np.uint32)
        fl = np.zeros(n, np.uint32)
        key = np.zeros(n, np.uint64)
        self._check(lib().gi_rays_export(self.h, slot.ctypes.data, t.ctypes.data, tri.ctypes.data,
                                         fl.ctypes.data, key.ctypes.data), "gi_rays_export")
        return dict(slot=slot, t=t, tri=tri, cell=fl, key=key)

    def probes(self):
        d = self.dims()
        P, mt = int(d[0]), int(d[6])
        mask = np.zeros(mt, np.uint32)
        pos = np.zeros((P, 4), np.float32)
        nrm = np.zeros((P, 4), np.float32)
        atlas = np.zeros((P, 64, 4), np.float32)
        sh = np.zeros((P, 27), np.float32)
        self._check(lib().gi_probes_export(self.h, mask.ctypes.data, pos.ctypes.data, nrm.ctypes.data,
                                           atlas.ctypes.data, sh.ctypes.data), "gi_probes_export")
        return dict(mask=mask, pos=pos, nrm=nrm, atlas=atlas, sh=sh)

    def table(self):
        N = int(self.dims()[2])
        ident = np.zeros(N, np.uint64)
        key = np.zeros(N, np.uint64)
        acc = np.zeros((N, 4), np.uint32)
        L = np.zeros((N, 3), np.float32)
        nh = np.zeros(N, np.uint32)
        life = np.zeros(N, np.uint32)
        n = C.c_uint32()
        self._check(lib().gi_cache_export(self.h, ident.ctypes.data, key.ctypes.data, acc.ctypes.data,
                                          L.ctypes.data, nh.ctypes.data, life.ctypes.data, N,
                                          C.byref(n)), "gi_cache_export")
        k = n.value
        order = np.argsort(ident[:k], kind="stable")
        return dict(id=ident[:k][order], key=key[:k][order], acc=acc[:k][order], L=L[:k][order],
                    nhist=nh[:k][order], life=life[:k][order])

    def tiles(self):
        """two-level cache (cache_tiles = 1): live tiles sorted by (bucket, fingerprint) with
        per-cell sums, moving averages, sample counts and prefiltered radiance"""
        N = int(self.dims()[2])
        ident = np.zeros(N, np.uint64)
        key = np.zeros(N, np.uint64)
        life = np.zeros(N, np.uint32)
        acc = np.zeros((N, 64, 4), np.uint32)
        L = np.zeros((N, 64, 3), np.float32)
        nh = np.zeros((N, 64), np.uint32)
        Lq = np.zeros((N, 64, 3), np.float32)
        n = C.c_uint32()
        self._check(lib().gi_tiles_export(self.h, ident.ctypes.data, key.ctypes.data, life.ctypes.data,
                                          acc.ctypes.data, L.ctypes.data, nh.ctypes.data, Lq.ctypes.data, N,
                                          C.byref(n)), "gi_tiles_export")
        k = n.value
        o = np.argsort(ident[:k], kind="stable")
        return dict(id=ident[:k][o], key=key[:k][o], life=life[:k][o], acc=acc[:k][o], L=L[:k][o],
                    nhist=nh[:k][o], Lq=Lq[:k][o])

    def reservoirs(self):
        """world-space reservoirs written by the last trace (restir = 1), sorted by (bucket,
        fingerprint): key, light point, contribution weight, normal, light, count"""
        N = 1 << int(self.cfg_dict["restir_log2"])
        ident = np.zeros(N, np.uint64)
        key = np.zeros(N, np.uint64)
        yw = np.zeros((N, 4), np.float32)
        nr = np.zeros((N, 3), np.float32)
        k = np.zeros(N, np.uint32)
        m = np.zeros(N, np.uint32)
        n = C.c_uint32()
        self._check(lib().gi_restir_export(self.h, ident.ctypes.data, key.ctypes.data, yw.ctypes.data, nr.ctypes.data,
                                           k.ctypes.data, m.ctypes.data, N, C.byref(n)), "gi_restir_export")
        c = n.value
        o = np.argsort(ident[:c], kind="stable")
        return dict(id=ident[:c][o], key=key[:c][o], y=yw[:c, :3][o], W=yw[:c, 3][o], n=nr[:c][o], k=k[:c][o],
                    M=m[:c][o])

    def light_grid(self):
        """light grid of the last trace (light_grid = 1): origin, cell side, dims, per-cell
        lists (emitter indices) and counts"""
        D = int(self.cfg_dict["lgrid_dim"])
        K = int(self.cfg_dict["lgrid_k"])
        geom = np.zeros(4, np.float32)
        dims = np.zeros(3, np.uint32)
        lst = np.zeros(D * D * D * K, np.uint32)
        cnt = np.zeros(D * D * D, np.uint32)
        self._check(lib().gi_light_grid_export(self.h, geom.ctypes.data, dims.ctypes.data, lst.ctypes.data,
                                               cnt.ctypes.data, D * D * D), "gi_light_grid_export")
        n = int(np.prod(dims))
        return dict(lo=geom[:3].copy(), h=float(geom[3]), dims=dims, list=lst[:n * K].reshape(n, K), count=cnt[:n])

    def cache_save(self) -> bytes:
        n = C.c_size_t()
        self._check(lib().gi_cache_save(self.h, None, 0, C.byref(n)), "gi_cache_save")
        buf = C.create_string_buffer(n.value)
        self._check(lib().gi_cache_save(self.h, buf, n.value, C.byref(n)), "gi_cache_save")
        return buf.raw

    def cache_load(self, blob: bytes):
        self._check(lib().gi_cache_import(self.h, blob, len(blob)), "gi_cache_import")

    def learned_save(self) -> bytes:
        n = C.c_size_t()
        self._check(lib().gi_learned_export(self.h, None, 0, C.byref(n)), "gi_learned_export")
        buf = C.create_string_buffer(n.value)
        self._check(lib().gi_learned_export(self.h, buf, n.value, C.byref(n)), "gi_learned_export")
        return buf.raw

    def learned_load(self, blob: bytes):
        self._check(lib().gi_learned_import(self.h, blob, len(blob)), "gi_learned_import")

    def learned_stats(self):
        out = np.zeros(8, np.float32)
        self._check(lib().gi_learned_stats(self.h, out.ctypes.data), "gi_learned_stats")
        return dict(loss=float(out[0]), judged_err=float(out[1]), fallback=bool(out[2]),
                    steps=int(out[3]), skipped=int(out[4]))

    def learned_batch(self):
        """the last gi_learned_train's batch: dict(raw, grouped [rows, 3, 4] float32 (pos+t,
        normal + ray-id bits, target + 1), gid [rows] (raw order), n_train)"""
        rows, n = C.c_uint32(0), C.c_uint32(0)
        self._check(lib().gi_learned_batch_export(self.h, None, None, 0, C.byref(rows), C.byref(n)),
                    "gi_learned_batch_export")
        raw = np.zeros((rows.value, 3, 4), np.float32)
        grouped = np.zeros((rows.value, 3, 4), np.float32)
        self._check(lib().gi_learned_batch_export(self.h, raw.ctypes.data, grouped.ctypes.data, rows.value,
                                                  C.byref(rows), C.byref(n)), "gi_learned_batch_export")
        return dict(raw=raw, grouped=grouped, gid=raw[:, 1, 3].view(np.uint32).copy(), n_train=int(n.value))

    def profile(self, on):
        """True / 1: time every kernel; 2: only the probe-ray traversal; False / 0: off"""
        self._check(lib().gi_profile_enable(self.h, int(on)), "gi_profile_enable")

    def profile_read(self):
        cap = 64
        names = C.create_string_buffer(4096)
        counts = np.zeros(cap, np.uint32)
        ms = np.zeros(cap, np.float64)
        n = C.c_uint32()
        self._check(lib().gi_profile_read(self.h, names, 4096, counts.ctypes.data, ms.ctypes.data, cap,
                                          C.byref(n)), "gi_profile_read")
        parts = names.raw.split(b"\0")
        return {parts[i].decode(): (int(counts[i]), float(ms[i])) for i in range(min(n.value, cap))}


class GBuffer:
    """Device G-buffer tensors of one frame: pos, nrm, alb [H,W,4] float32, prim [H,W] int32."""

    def __init__(self, H, W, device="cuda"):
        import torch
        self.pos = torch.zeros((H, W, 4), dtype=torch.float32, device=device)
        self.nrm = torch.zeros((H, W, 4), dtype=torch.float32, device=device)
        self.alb = torch.zeros((H, W, 4), dtype=torch.float32, device=device)
        self.prim = torch.zeros((H, W), dtype=torch.int32, device=device)

    def host(self):
        return (self.pos.cpu().numpy(), self.nrm.cpu().numpy(), self.alb.cpu().numpy(),
                self.prim.cpu().numpy().view(np.uint32))


class Denoiser:
    """The screen-space denoiser (gi_denoiser_*): temporal accumulation with a capped history
    and a spatial filter whose radius follows the history length."""

    def __init__(self, width, height, hist_max=16, radius_max=4):
        L = lib()
        h = C.c_void_p()
        st = L.gi_denoiser_create(width, height, hist_max, radius_max, C.byref(h))
        if st != GI_OK:
            raise GIError(f"gi_denoiser_create failed: {ERRORS.get(st, st)}")
        self.h, self.W, self.H = h, width, height

    def _check(self, st, what):
        if st != GI_OK:
            raise GIError(f"{what} failed: {ERRORS.get(st, st)}")

    def __call__(self, frame, pos, nrm, prim, irradiance, out, stream=None):
        f = make_frame(frame)
        self._check(lib().gi_denoise(self.h, C.byref(f), _ptr(pos), _ptr(nrm), _ptr(prim), _ptr(irradiance),
                                     _ptr(out), _stream(stream)), "gi_denoise")

    def reset(self):
        self._check(lib().gi_denoiser_reset(self.h), "gi_denoiser_reset")

    def state(self):
        hist = np.zeros((self.H, self.W, 4), np.float32)
        rad = np.zeros((self.H, self.W), np.uint32)
        self._check(lib().gi_denoiser_export(self.h, hist.ctypes.data, rad.ctypes.data), "gi_denoiser_export")
        return hist, rad

    def close(self):
        if self.h:
            lib().gi_denoiser_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Seeded synthetic inputs for the indirect-lighting pass: scenes, cameras, moving lights.

This module produces input data only (triangle soups, materials, camera frames).  It holds
none of the lighting method's arithmetic, so both the HIP path and the CPU oracle may consume
its output.  All geometry is generated in float64 and rounded once to float32.

Scenes stand in for the paper's test scenes, which are not available (Section 5, Table 1):
  * ``room``     -- a closed 6x3x6 m room, 8 random boxes and one emissive ceiling quad
                    (110 triangles).
  * ``field``    -- ~1.0M triangles: a tessellated 80x80 m ground, 40,000 random boxes,
                    100 subdivided icospheres and 4 emissive quads, one of which circles.
  * ``city``     -- ~10M triangles of extruded random convex building footprints.
  * ``furnace``  -- an inward-facing closed UV sphere (radius 5 m, 316x316), emission 1,
                    albedo 0.8.

Materials are rows of 6 float32: albedo rgb, emitted radiance rgb.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

SCENE_SEED = 1
CAMERA_SEED = 2
RNG_SEED = 3


@dataclasses.dataclass
class Scene:
    name: str
    verts: np.ndarray          # float32 [V,3]
    idx: np.ndarray            # uint32  [T,3]
    tri_mat: np.ndarray        # uint32  [T]
    materials: np.ndarray      # float32 [M,6]  (albedo rgb, Le rgb)
    sky: tuple = (0.0, 0.0, 0.0)
    # moving emitters: frame -> (float32 [D,9] vertices, uint32 [D] materials); None if static
    dynamic: Optional[Callable[[int], tuple]] = None

    @property
    def n_tris(self) -> int:
        return int(self.idx.shape[0])


@dataclasses.dataclass
class Frame:
    """One camera frame.  Vectors are float32 unit vectors from a float64 construction."""
    index: int
    pos: np.ndarray
    fwd: np.ndarray
    right: np.ndarray
    up: np.ndarray
    fov_y: float
    tan_half: float


# ----------------------------------------------------------------------------------------
# geometry builders (float64)
# ----------------------------------------------------------------------------------------

def _box(lo, hi, outward=True):
    """12 triangles of an axis-aligned box; winding gives outward (or inward) normals."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    v = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], dtype=np.float64)
    # outward CCW faces
    f = np.array([[0, 2, 1], [0, 3, 2],      # z0 face, normal -z
                  [4, 5, 6], [4, 6, 7],      # z1 face, normal +z
                  [0, 1, 5], [0, 5, 4],      # y0 face, normal -y
                  [3, 7, 6], [3, 6, 2],      # y1 face, normal +y
                  [0, 4, 7], [0, 7, 3],      # x0 face, normal -x
                  [1, 2, 6], [1, 6, 5]],     # x1 face, normal +x
                 dtype=np.int64)
    if not outward:
        f = f[:, [0, 2, 1]]
    return v, f


def _quad(center, half_u, half_v, normal_sign_flip=False):
    """Two triangles of a parallelogram centre +- half_u +- half_v; winding normal = u x v."""
    c = np.asarray(center, np.float64)
    u = np.asarray(half_u, np.float64)
    w = np.asarray(half_v, np.float64)
    v = np.array([c - u - w, c + u - w, c + u + w, c - u + w])
    f = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int64)
    if normal_sign_flip:
        f = f[:, [0, 2, 1]]
    return v, f


def _icosphere(level):
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t], [0, -1, -t],
         [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]]
    f = [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4],
         [11, 10, 2], [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8],
         [3, 8, 9], [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]]
    v = [np.array(p, np.float64) / np.linalg.norm(p) for p in v]
    for _ in range(level):
        cache = {}
        nf = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = v[a] + v[b]
                v.append(m / np.linalg.norm(m))
                cache[key] = len(v) - 1
            return cache[key]
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = nf
    return np.array(v), np.array(f, dtype=np.int64)


def uv_sphere(radius, n_seg, n_ring, inward=True):
    """UV sphere with pole fans: 2*n_seg*(n_ring-2) + 2*n_seg triangles."""
    verts = [[0.0, radius, 0.0]]
    for r in range(1, n_ring):
        th = math.pi * r / n_ring
        for s in range(n_seg):
            ph = 2.0 * math.pi * s / n_seg
            verts.append([radius * math.sin(th) * math.cos(ph), radius * math.cos(th),
                          radius * math.sin(th) * math.sin(ph)])
    verts.append([0.0, -radius, 0.0])
    v = np.array(verts)
    faces = []
    ring = lambda r, s: 1 + (r - 1) * n_seg + (s % n_seg)
    for s in range(n_seg):
        faces.append([0, ring(1, s + 1), ring(1, s)])
    for r in range(1, n_ring - 1):
        for s in range(n_seg):
            a, b = ring(r, s), ring(r, s + 1)
            c, d = ring(r + 1, s), ring(r + 1, s + 1)
            faces.append([a, b, d])
            faces.append([a, d, c])
    last = len(verts) - 1
    for s in range(n_seg):
        faces.append([last, ring(n_ring - 1, s), ring(n_ring - 1, s + 1)])
    f = np.array(faces, dtype=np.int64)
    # the construction above winds faces outward; flip for inward normals
    if inward:
        f = f[:, [0, 2, 1]]
    return v, f


class _Builder:
    def __init__(self):
        self.v: List[np.ndarray] = []
        self.f: List[np.ndarray] = []
        self.m: List[np.ndarray] = []
        self.nv = 0
        self.mats: List[List[float]] = []

    def material(self, albedo, le=(0.0, 0.0, 0.0)):
        self.mats.append(list(albedo) + list(le))
        return len(self.mats) - 1

    def add(self, v, f, mat):
        self.v.append(v)
        self.f.append(f + self.nv)
        self.m.append(np.full(len(f), mat, np.uint32))
        self.nv += len(v)

    def scene(self, name, sky=(0.0, 0.0, 0.0), dynamic=None):
        return Scene(name=name,
                     verts=np.concatenate(self.v).astype(np.float32),
                     idx=np.concatenate(self.f).astype(np.uint32),
                     tri_mat=np.concatenate(self.m).astype(np.uint32),
                     materials=np.array(self.mats, np.float32).reshape(-1, 6),
                     sky=tuple(float(s) for s in sky), dynamic=dynamic)


# ----------------------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------------------

def room_scene(seed: int = SCENE_SEED, light_le: float = 10.0) -> Scene:
    """6x3x6 m room (inward faces, albedo 0.7), 8 non-overlapping random boxes on the floor
    (albedo U[0.3,0.8] per channel) and a 1x1 m emissive quad 1 cm below the ceiling."""
    rng = np.random.default_rng(seed)
    b = _Builder()
    wall = b.material((0.7, 0.7, 0.7))
    v, f = _box((0.0, 0.0, 0.0), (6.0, 3.0, 6.0), outward=False)
    b.add(v, f, wall)
    placed = []
    while len(placed) < 8:
        sx, sz = rng.uniform(0.3, 1.0, size=2)
        h = rng.uniform(0.3, 1.5)
        x0 = rng.uniform(0.2, 5.8 - sx)
        z0 = rng.uniform(0.2, 5.8 - sz)
        ok = all(x0 + sx + 0.05 < p[0] or p[0] + p[2] + 0.05 < x0 or
                 z0 + sz + 0.05 < p[1] or p[1] + p[3] + 0.05 < z0 for p in placed)
        if not ok:
            continue
        placed.append((x0, z0, sx, sz))
        alb = rng.uniform(0.3, 0.8, size=3)
        v, f = _box((x0, 0.0, z0), (x0 + sx, h, z0 + sz))
        b.add(v, f, b.material(alb))
    light = b.material((0.0, 0.0, 0.0), (light_le, light_le, light_le))
    # facing down: u x v must be -y
    v, f = _quad((3.0, 2.99, 3.0), (0.5, 0.0, 0.0), (0.0, 0.0, 0.5))
    b.add(v, f, light)
    return b.scene("room")


def lights_room_scene(seed: int = SCENE_SEED, n_lights: int = 64) -> Scene:
    """The room of room_scene (same walls and boxes) lit by n_lights small emissive quads
    instead of one: 0.2x0.2 m, 1 cm off the ceiling (facing down) or the four walls (facing
    in), random colours, radiance log-uniform over [2, 200] so that a few lights dominate."""
    base = room_scene(seed)
    rng = np.random.default_rng(seed + 101)
    b = _Builder()
    b.mats = [list(m) for m in base.materials[:-1]]   # without the ceiling light
    keep = base.tri_mat < len(base.materials) - 1
    b.v.append(base.verts.astype(np.float32))
    b.f.append(base.idx[keep])
    b.m.append(base.tri_mat[keep])
    b.nv = len(base.verts)
    s = 0.1
    for _ in range(n_lights):
        le = 10.0 ** rng.uniform(np.log10(2.0), np.log10(200.0)) * rng.uniform(0.4, 1.0, size=3)
        mat = b.material((0.0, 0.0, 0.0), le)
        face = rng.integers(0, 5)
        a, c = rng.uniform(0.3, 5.7, size=2)
        h = rng.uniform(1.0, 2.7)
        if face == 0:      # ceiling, facing down
            v, f = _quad((a, 2.99, c), (s, 0.0, 0.0), (0.0, 0.0, s))
        elif face == 1:    # wall x = 0, facing +x
            v, f = _quad((0.01, h, c), (0.0, s, 0.0), (0.0, 0.0, s))
        elif face == 2:    # wall x = 6, facing -x
            v, f = _quad((5.99, h, c), (0.0, 0.0, s), (0.0, s, 0.0))
        elif face == 3:    # wall z = 0, facing +z
            v, f = _quad((a, h, 0.01), (s, 0.0, 0.0), (0.0, s, 0.0))
        else:              # wall z = 6, facing -z
            v, f = _quad((a, h, 5.99), (0.0, s, 0.0), (s, 0.0, 0.0))
        b.add(v, f, mat)
    return b.scene("lights_room")


def _field_light_quad(center):
    v, f = _quad(center, (1.0, 0.0, 0.0), (0.0, 0.0, 1.0))   # normal -y (down)
    return v[f].reshape(-1, 9)


def field_scene(seed: int = SCENE_SEED, n_boxes: int = 40000, n_spheres: int = 100,
                ground_res: int = 64, sphere_level: int = 4, light_le: float = 50.0,
                light_orbit_deg_per_frame: float = 6.0) -> Scene:
    """~1.0M-triangle outdoor field: tessellated ground, instanced boxes, icospheres,
    4 emissive 2x2 m quads at 8 m; quad 0 circles the centre at radius 15 m."""
    rng = np.random.default_rng(seed)
    b = _Builder()
    ground_mat = b.material((0.5, 0.5, 0.5))
    n = ground_res
    xs = np.linspace(-40.0, 40.0, n + 1)
    gx, gz = np.meshgrid(xs, xs, indexing="xy")
    gv = np.stack([gx.ravel(), np.zeros(gx.size), gz.ravel()], axis=1)
    i = np.arange(n)
    ii, jj = np.meshgrid(i, i, indexing="xy")
    a = (jj * (n + 1) + ii).ravel()
    bq = a + 1
    c = a + (n + 1)
    d = c + 1
    # +y facing: (b-a) x (c-a) with b-a=+x, c-a=+z gives -y, so wind a,c,b
    gf = np.concatenate([np.stack([a, c, bq], 1), np.stack([bq, c, d], 1)])
    b.add(gv, gf, ground_mat)

    # boxes: all instances of a unit box, scaled/translated
    bv, bf = _box((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    sizes = rng.uniform(0.2, 2.0, size=(n_boxes, 3))
    pos = np.stack([rng.uniform(-38.0, 38.0, n_boxes), np.zeros(n_boxes),
                    rng.uniform(-38.0, 38.0, n_boxes)], 1)
    alb = rng.uniform(0.1, 0.9, size=(n_boxes, 3))
    mat0 = len(b.mats)
    b.mats.extend([list(al) + [0.0, 0.0, 0.0] for al in alb])
    verts = (bv[None, :, :] * sizes[:, None, :] + pos[:, None, :]).reshape(-1, 3)
    faces = (bf[None, :, :] + 8 * np.arange(n_boxes)[:, None, None]).reshape(-1, 3)
    mats = np.repeat(np.arange(mat0, mat0 + n_boxes, dtype=np.uint32), 12)
    b.v.append(verts)
    b.f.append(faces + b.nv)
    b.m.append(mats)
    b.nv += len(verts)

    sv, sf = _icosphere(sphere_level)
    for _ in range(n_spheres):
        r = rng.uniform(0.5, 3.0)
        cpos = np.array([rng.uniform(-35.0, 35.0), r, rng.uniform(-35.0, 35.0)])
        m = b.material(rng.uniform(0.1, 0.9, size=3))
        b.add(sv * r + cpos, sf, m)

    le = (light_le, light_le, light_le)
    light_mat = b.material((0.0, 0.0, 0.0), le)
    for cx, cz in ((12.0, -12.0), (-12.0, 12.0), (-12.0, -12.0)):
        v, f = _quad((cx, 8.0, cz), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0))
        b.add(v, f, light_mat)
    step = math.radians(light_orbit_deg_per_frame)

    def dynamic(frame: int):
        ang = step * frame
        tri = _field_light_quad((15.0 * math.cos(ang), 8.0, 15.0 * math.sin(ang)))
        return tri.astype(np.float32), np.full(2, light_mat, np.uint32)
    return b.scene("field", sky=(0.05, 0.05, 0.05), dynamic=dynamic)


def city_scene(seed: int = SCENE_SEED, blocks: int = 100, block_size: float = 40.0,
               facade_quad: float = 3.0, light_le: float = 500.0) -> Scene:
    """Procedural city: one extruded convex 4-8-gon building per block, facades tessellated
    into ~facade_quad-metre quads, fan roofs; a tessellated ground plane; 4 emissive quads."""
    rng = np.random.default_rng(seed)
    b = _Builder()
    ground_mat = b.material((0.4, 0.4, 0.4))
    extent = blocks * block_size
    gn = 128
    xs = np.linspace(0.0, extent, gn + 1)
    gx, gz = np.meshgrid(xs, xs, indexing="xy")
    gv = np.stack([gx.ravel(), np.zeros(gx.size), gz.ravel()], axis=1)
    i = np.arange(gn)
    ii, jj = np.meshgrid(i, i, indexing="xy")
    a = (jj * (gn + 1) + ii).ravel()
    c = a + (gn + 1)
    gf = np.concatenate([np.stack([a, c, a + 1], 1), np.stack([a + 1, c, c + 1], 1)])
    b.add(gv, gf, ground_mat)
    all_v, all_f, all_m = [], [], []
    nv = b.nv
    mat_base = len(b.mats)
    for by in range(blocks):
        for bx in range(blocks):
            k = int(rng.integers(4, 9))
            ang = np.sort(rng.uniform(0.0, 2.0 * math.pi, k))
            rad = rng.uniform(8.0, 16.0)
            cx = (bx + 0.5) * block_size
            cz = (by + 0.5) * block_size
            px = cx + rad * np.cos(ang)
            pz = cz + rad * np.sin(ang)
            h = rng.uniform(10.0, 120.0)
            ny = max(1, int(round(h / facade_quad)))
            ys = np.linspace(0.0, h, ny + 1)
            mat = len(b.mats)
            b.mats.append(list(rng.uniform(0.1, 0.9, 3)) + [0.0, 0.0, 0.0])
            # all facades of the building as one vertex grid: (ny + 1) rows by the edges'
            # columns side by side; quads never join the last column of an edge to the next
            x0, z0 = px, pz
            x1, z1 = np.roll(px, -1), np.roll(pz, -1)
            nxs = np.maximum(1, np.rint(np.hypot(x1 - x0, z1 - z0) / facade_quad).astype(np.int64))
            ncol = nxs + 1
            C = int(ncol.sum())
            first = np.concatenate([[0], np.cumsum(ncol)[:-1]])
            edge = np.repeat(np.arange(k), ncol)
            t = (np.arange(C) - first[edge]) / nxs[edge]
            ex = x0[edge] + (x1 - x0)[edge] * t
            ez = z0[edge] + (z1 - z0)[edge] * t
            fv = np.stack([np.tile(ex, ny + 1), np.repeat(ys, C), np.tile(ez, ny + 1)], 1)
            cols = np.nonzero(np.arange(C) != (first + nxs)[edge])[0]
            cc, rr = np.meshgrid(cols, np.arange(ny), indexing="xy")
            q0 = (rr * C + cc).ravel()
            q1 = q0 + 1
            q2 = q0 + C
            q3 = q2 + 1
            # counter-clockwise footprint -> outward facade normals with this winding
            ff = np.concatenate([np.stack([q0, q2, q1], 1), np.stack([q1, q2, q3], 1)])
            all_v.append(fv)
            all_f.append(ff + nv)
            all_m.append(np.full(len(ff), mat, np.uint32))
            nv += len(fv)
            rv = np.concatenate([[[cx, h, cz]], np.stack([px, np.full(k, h), pz], 1)])
            rf = np.array([[0, 1 + (e + 1) % k, 1 + e] for e in range(k)])
            all_v.append(rv)
            all_f.append(rf + nv)
            all_m.append(np.full(k, mat, np.uint32))
            nv += len(rv)
    b.v += all_v
    b.f += all_f
    b.m += all_m
    b.nv = nv
    light_mat = b.material((0.0, 0.0, 0.0), (light_le, light_le, light_le))
    mid = extent / 2.0
    for cx, cz in ((mid + 120, mid - 120), (mid - 120, mid + 120), (mid - 120, mid - 120),
                   (mid + 120, mid + 120)):
        v, f = _quad((cx, 80.0, cz), (10.0, 0.0, 0.0), (0.0, 0.0, 10.0))
        b.add(v, f, light_mat)
    del mat_base
    return b.scene("city", sky=(0.2, 0.2, 0.2))


def furnace_scene(radius: float = 5.0, n_seg: int = 316, n_ring: int = 316,
                  le: float = 1.0, albedo: float = 0.8) -> Scene:
    """Closed inward-facing sphere: every surface emits `le` and reflects `albedo`."""
    b = _Builder()
    m = b.material((albedo, albedo, albedo), (le, le, le))
    v, f = uv_sphere(radius, n_seg, n_ring, inward=True)
    b.add(v, f, m)
    return b.scene("furnace")


# ----------------------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------------------

def look_frame(index, pos, fwd, fov_y_deg=60.0, world_up=(0.0, 1.0, 0.0)) -> Frame:
    pos = np.asarray(pos, np.float64)
    fwd = np.asarray(fwd, np.float64)
    fwd = fwd / np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(world_up, np.float64))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    fov = math.radians(fov_y_deg)
    return Frame(index=index, pos=pos.astype(np.float32), fwd=fwd.astype(np.float32),
                 right=right.astype(np.float32), up=up.astype(np.float32),
                 fov_y=float(np.float32(fov)), tan_half=float(np.float32(math.tan(fov / 2.0))))


def room_camera(index: int = 0, seed: int = CAMERA_SEED) -> Frame:
    rng = np.random.default_rng(seed)
    x, z = rng.uniform(1.0, 5.0, size=2)
    yaw = rng.uniform(0.0, 2.0 * math.pi)
    pitch = rng.uniform(-0.3, 0.0)
    fwd = (math.cos(pitch) * math.sin(yaw), math.sin(pitch), math.cos(pitch) * math.cos(yaw))
    return look_frame(index, (x, 1.6, z), fwd)


def orbit_camera(index: int, radius: float = 30.0, height: float = 6.0,
                 deg_per_frame: float = 1.0, target=(0.0, 0.0, 0.0)) -> Frame:
    ang = math.radians(deg_per_frame * index)
    pos = np.array([radius * math.cos(ang), height, radius * math.sin(ang)])
    fwd = np.asarray(target, np.float64) - pos
    return look_frame(index, pos, fwd)


def city_camera(index: int, extent: float = 4000.0) -> Frame:
    mid = extent / 2.0
    t = index * 2.0
    pos = (mid - 300.0 + t, 150.0, mid - 300.0 + 0.5 * t)
    return look_frame(index, pos, (1.0, -0.35, 1.0))


def furnace_camera(index: int = 0) -> Frame:
    ang = 0.3 * index
    return look_frame(index, (0.0, 0.0, 0.0), (math.cos(ang), 0.1, math.sin(ang)))


# ----------------------------------------------------------------------------------------
# workload presets (sizes of the benchmark configurations)
# ----------------------------------------------------------------------------------------

PRESETS = {
    # 128x128, 16 rays, 2^16 slots, 1 bounce, 1 frame, room scene
    "room128": dict(scene="room", width=128, height=128, rays_per_probe=16, table_log2=16,
                    bounces=1, frames=1),
    # 1920x1080, 64 rays, 2^20 slots, 60 frames, field scene with a moving light
    "field1080": dict(scene="field", width=1920, height=1080, rays_per_probe=64,
                      table_log2=20, bounces=1, frames=60),
    # 3840x2160, 128 rays, 2^22 slots, 2 bounces, 30 frames, city scene
    "city4k": dict(scene="city", width=3840, height=2160, rays_per_probe=128, table_log2=22,
                   bounces=2, frames=30),
    # room scene at 1080p for the learned cache
    "room1080": dict(scene="room", width=1920, height=1080, rays_per_probe=64, table_log2=20,
                     bounces=1, frames=60),
    "furnace": dict(scene="furnace", width=256, height=256, rays_per_probe=64, table_log2=20,
                    bounces=2, frames=1),
}


def make_scene(name: str) -> Scene:
    return {"room": room_scene, "field": field_scene, "city": city_scene,
            "furnace": furnace_scene, "lights_room": lights_room_scene}[name]()


def camera_for(scene_name: str, index: int) -> Frame:
    if scene_name in ("room", "lights_room"):
        return room_camera(index)
    if scene_name == "field":
        return orbit_camera(index)
    if scene_name == "city":
        return city_camera(index)
    return furnace_camera(index)


def random_rays(n: int, lo, hi, seed: int = 7):
    """Seeded ray origins uniform in a box and directions uniform on the sphere (float32)."""
    rng = np.random.default_rng(seed)
    o = rng.uniform(lo, hi, size=(n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


def query_points(n: int, lo, hi, seed: int = 11):
    """Seeded points and unit normals (float32 [n,4]) for cache queries; .w of points = -1."""
    rng = np.random.default_rng(seed)
    p = np.concatenate([rng.uniform(lo, hi, size=(n, 3)), -np.ones((n, 1))], 1)
    nrm = rng.normal(size=(n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    nrm = np.concatenate([nrm, np.zeros((n, 1))], 1)
    return p.astype(np.float32), nrm.astype(np.float32)


"""Seeded synthetic scenes shaped like the workloads of the paper's evaluation.

This module only draws inputs: vertex positions, indices, camera matrices,
attributes and textures.  It holds none of the rendering arithmetic (no
transform, snapping, coverage, depth or shading), so both the HIP path and the
CPU oracle can consume the same arrays without sharing any of the method.

The paper's scenes (Sec. 7.2, Fig. "rastpics": Fairy Forest, Buddha, Mecha,
Dragon at 1024x768) are public models that are not available here; the
generators below stand in for them by shape class:

* ``tiny64``   -- 256 large random triangles on a 64x64 screen (mixed sizes,
                  high depth complexity; the parity workhorse).
* ``grid1080`` -- a displaced 1024x512-quad grid (~1.05M shared-vertex
                  triangles of ~2 px^2) seen through a perspective camera at
                  1920x1080; it stands in for the "very small"/"small"
                  triangle scenes (Buddha, Dragon).
* ``micro``    -- independent micropolygons with log-normal area around
                  0.5 px^2 (the Reyes Sample-stage load after dicing).
* ``batch``    -- many independent small scenes of uneven triangle counts.
* ``diffgrid`` -- the grid mesh with per-vertex UVs and a texture, seen from
                  many viewpoints.
* ``patches``  -- a bumpy sheet of bicubic Bezier patches seen at a grazing
                  angle, for the Reyes front end (the paper's Bigguy and
                  Teapot patch models are not available).

All arrays are NumPy, float32 unless noted, with positions and per-vertex
attributes stored as SoA planes ``[channels][V]``.  Every generator takes a
seed and uses ``numpy.random.default_rng`` (PCG64).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Scene:
    """Inputs for one render call (one or many scenes/views)."""

    width: int
    height: int
    pos: np.ndarray                      # [3][V] float32
    color: np.ndarray                    # [3][V] float32
    idx: Optional[np.ndarray] = None     # [T][3] int32, None -> vertex 3t+k
    num_tris: int = 0                    # T over all scenes (indexed or not)
    mvp: Optional[np.ndarray] = None     # [S][16] float32 row-major, None -> identity
    num_scenes: int = 1
    scene_tri_off: Optional[np.ndarray] = None  # [S+1] int32 (concatenated scenes)
    scene_vtx_off: Optional[np.ndarray] = None  # [S+1] int32
    instanced: bool = False              # S views of one mesh (scene_*_off unused)
    uv: Optional[np.ndarray] = None      # [2][V] float32
    normal: Optional[np.ndarray] = None  # [3][V] float32
    texture: Optional[np.ndarray] = None  # [Nh][Nw][3] float32
    lights: Optional[np.ndarray] = None  # [L][3] float32 unit vectors
    bin_size: int = 16
    shading: str = "gouraud"             # gouraud | textured | deferred | lit
    name: str = ""

    @property
    def num_vertices(self) -> int:
        return int(self.pos.shape[1])


def default_light() -> np.ndarray:
    """The fragment shader's light direction normalize(1,1,1) of the paper's
    example stage (Sec. 4.1, listing "kernels"), computed in float64 and
    rounded once to float32."""
    v = np.array([1.0, 1.0, 1.0], dtype=np.float64)
    return (v / math.sqrt(3.0)).astype(np.float32).reshape(1, 3)


def lights(num: int) -> np.ndarray:
    """``num`` unit light directions: the first is normalize(1,1,1); the others
    sit on a cone around +z at 45 degrees elevation, evenly spaced in azimuth.
    Float64 then rounded to float32 (shader complexity knob, Sec. 7.2)."""
    out = [default_light()[0].astype(np.float64)]
    for k in range(1, num):
        a = 2.0 * math.pi * k / max(num - 1, 1)
        v = np.array([math.cos(a), math.sin(a), 1.0])
        out.append(v / np.linalg.norm(v))
    return np.asarray(out, dtype=np.float64).astype(np.float32)


def with_lighting(sc: Scene, num_lights: int = 1, seed: int = 7,
                  shading: str = "lit") -> Scene:
    """A copy of ``sc`` lit by ``num_lights`` lights (see ``lights``): per-vertex
    unit normals drawn as normalize(N(0, I)) with z made non-negative, and
    forward-lit (or deferred) shading."""
    rng = np.random.default_rng(seed)
    n = rng.standard_normal(size=(3, sc.pos.shape[1]))
    n[2] = np.abs(n[2])
    n /= np.linalg.norm(n, axis=0, keepdims=True)
    return dataclasses.replace(sc, normal=n.astype(np.float32), lights=lights(num_lights),
                               shading=shading, name=f"{sc.name}_{shading}{num_lights}")


# ---------------------------------------------------------------------------
# tiny64: 256 random triangles, NDC input, w = 1
# ---------------------------------------------------------------------------
def tiny(seed: int = 1001, width: int = 64, height: int = 64, num_tris: int = 256,
         bin_size: int = 8) -> Scene:
    rng = np.random.default_rng(seed)
    V = 3 * num_tris
    xy = rng.uniform(-1.0, 1.0, size=(2, V))
    z = rng.uniform(0.0, 1.0, size=(1, V))
    pos = np.concatenate([xy, z], axis=0).astype(np.float32)
    color = rng.uniform(0.0, 1.0, size=(3, V)).astype(np.float32)
    return Scene(width, height, pos, color, None, num_tris, bin_size=bin_size,
                 name=f"tiny{width}x{height}_T{num_tris}_s{seed}")


# ---------------------------------------------------------------------------
# Perspective camera helpers (float64, rounded to float32 at the end)
# ---------------------------------------------------------------------------
def perspective(fovy_deg: float, aspect: float, near: float, far: float) -> np.ndarray:
    """Left-handed perspective matrix that maps view-space depth z in
    [near, far] to NDC depth in [0, 1] and puts view z into clip w."""
    f = 1.0 / math.tan(math.radians(fovy_deg) / 2.0)
    m = np.zeros((4, 4))
    m[0, 0] = f / aspect
    m[1, 1] = f
    m[2, 2] = far / (far - near)
    m[2, 3] = -near * far / (far - near)
    m[3, 2] = 1.0
    return m


def translate(x: float, y: float, z: float) -> np.ndarray:
    m = np.eye(4)
    m[:3, 3] = (x, y, z)
    return m


def rot_x(deg: float) -> np.ndarray:
    c, s = math.cos(math.radians(deg)), math.sin(math.radians(deg))
    m = np.eye(4)
    m[1, 1], m[1, 2], m[2, 1], m[2, 2] = c, -s, s, c
    return m


def rot_y(deg: float) -> np.ndarray:
    c, s = math.cos(math.radians(deg)), math.sin(math.radians(deg))
    m = np.eye(4)
    m[0, 0], m[0, 2], m[2, 0], m[2, 2] = c, s, -s, c
    return m


# ---------------------------------------------------------------------------
# grid: displaced regular grid of nx x ny quads, two CCW triangles per quad
# ---------------------------------------------------------------------------
def grid_mesh(nx: int, ny: int, seed: int, half_w: float = 2.3, half_h: float = 1.3):
    """Vertices (nx+1)*(ny+1) on a regular (u, v) grid; world position
    x = (2u-1)*half_w, y = (2v-1)*half_h, z = 0.5 + 0.1 sin(2pi(3u+p1)) sin(2pi(2v+p2))."""
    rng = np.random.default_rng(seed)
    p1, p2 = rng.uniform(0.0, 1.0, size=2)
    u = np.arange(nx + 1, dtype=np.float64) / nx
    v = np.arange(ny + 1, dtype=np.float64) / ny
    U, Vv = np.meshgrid(u, v)            # [ny+1][nx+1]
    x = (2.0 * U - 1.0) * half_w
    y = (2.0 * Vv - 1.0) * half_h
    z = 0.5 + 0.1 * np.sin(2 * math.pi * (3 * U + p1)) * np.sin(2 * math.pi * (2 * Vv + p2))
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()]).astype(np.float32)
    uv = np.stack([U.ravel(), Vv.ravel()]).astype(np.float32)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    v00 = (j * (nx + 1) + i).ravel()
    v10 = v00 + 1
    v01 = v00 + (nx + 1)
    v11 = v01 + 1
    # two counter-clockwise triangles per quad (fixed diagonal v00-v11),
    # interleaved so that triangle 2q and 2q+1 belong to quad q
    idx = np.empty((2 * v00.size, 3), dtype=np.int32)
    idx[0::2] = np.stack([v00, v10, v11], axis=1)
    idx[1::2] = np.stack([v00, v11, v01], axis=1)
    return pos, uv, idx


def grid(seed: int = 1002, width: int = 1920, height: int = 1080, nx: int = 1024,
         ny: int = 512, bin_size: int = 16) -> Scene:
    pos, _, idx = grid_mesh(nx, ny, seed)
    rng = np.random.default_rng(seed + 1)
    color = rng.uniform(0.0, 1.0, size=(3, pos.shape[1])).astype(np.float32)
    mvp = perspective(60.0, width / height, 0.1, 10.0) @ translate(0.0, 0.0, 1.5)
    return Scene(width, height, pos, color, idx, idx.shape[0],
                 mvp=mvp.astype(np.float32).reshape(1, 16), bin_size=bin_size,
                 name=f"grid{nx}x{ny}_{width}x{height}")


# ---------------------------------------------------------------------------
# micro: independent micropolygons with log-normal area (deferred shading)
# ---------------------------------------------------------------------------
def micro(seed: int = 3003, width: int = 1920, height: int = 1080,
          num_tris: int = 1 << 23, mean_log_area: float = math.log(0.5),
          sigma: float = 0.5, z_levels: int = 0, num_lights: int = 1,
          bin_size: int = 16) -> Scene:
    rng = np.random.default_rng(seed)
    T = num_tris
    cx = rng.uniform(0.0, width, size=T)
    cy = rng.uniform(0.0, height, size=T)
    area = rng.lognormal(mean_log_area, sigma, size=T)
    ang = rng.uniform(0.0, 2 * math.pi, size=(3, T))
    px, py = np.cos(ang), np.sin(ang)
    a0 = 0.5 * np.abs((px[1] - px[0]) * (py[2] - py[0]) - (px[2] - px[0]) * (py[1] - py[0]))
    a0 = np.maximum(a0, 1e-3)
    k = np.sqrt(area / a0)
    gx, gy = px.mean(axis=0), py.mean(axis=0)
    sx = cx + k * (px - gx)                  # [3][T] pixels
    sy = cy + k * (py - gy)
    z = rng.uniform(0.0, 1.0, size=T)
    if z_levels:
        z = np.floor(z * z_levels) / z_levels
    V = 3 * T
    pos = np.empty((3, V), dtype=np.float32)
    # vertex 3t+k
    pos[0] = (2.0 * sx.T.ravel() / width - 1.0).astype(np.float32)
    pos[1] = (2.0 * sy.T.ravel() / height - 1.0).astype(np.float32)
    pos[2] = np.repeat(z, 3).astype(np.float32)
    color = rng.uniform(0.0, 1.0, size=(3, V)).astype(np.float32)
    n = rng.standard_normal(size=(3, V))
    n[2] = np.abs(n[2])
    n /= np.linalg.norm(n, axis=0, keepdims=True)
    return Scene(width, height, pos, color, None, T, normal=n.astype(np.float32),
                 lights=lights(num_lights), bin_size=bin_size, shading="deferred",
                 name=f"micro{T}_{width}x{height}")


# ---------------------------------------------------------------------------
# batch: many small scenes of uneven triangle counts, concatenated
# ---------------------------------------------------------------------------
def batch(num_scenes: int = 256, size: int = 256, tmin: int = 1000, tmax: int = 200000,
          seed0: int = 4000, mean_log_len: float = math.log(4.0), sigma: float = 0.5,
          bin_size: int = 16) -> Scene:
    pos_l, col_l, tri_off, vtx_off = [], [], [0], [0]
    for s in range(num_scenes):
        rng = np.random.default_rng(seed0 + s)
        Ts = int(math.floor(math.exp(rng.uniform(math.log(tmin), math.log(tmax)))))
        v0 = rng.uniform(0.0, size, size=(2, Ts))
        L = rng.lognormal(mean_log_len, sigma, size=(2, Ts))
        th = rng.uniform(0.0, 2 * math.pi, size=(2, Ts))
        v1 = v0 + L[0] * np.stack([np.cos(th[0]), np.sin(th[0])])
        v2 = v0 + L[1] * np.stack([np.cos(th[1]), np.sin(th[1])])
        xy = np.stack([v0, v1, v2], axis=2).reshape(2, 3 * Ts)   # vertex 3t+k
        ndc = xy / (size / 2.0) - 1.0
        z = rng.uniform(0.0, 1.0, size=(1, 3 * Ts))
        pos_l.append(np.concatenate([ndc, z]).astype(np.float32))
        col_l.append(rng.uniform(0.0, 1.0, size=(3, 3 * Ts)).astype(np.float32))
        tri_off.append(tri_off[-1] + Ts)
        vtx_off.append(vtx_off[-1] + 3 * Ts)
    pos = np.concatenate(pos_l, axis=1)
    color = np.concatenate(col_l, axis=1)
    return Scene(size, size, pos, color, None, tri_off[-1], num_scenes=num_scenes,
                 scene_tri_off=np.asarray(tri_off, dtype=np.int32),
                 scene_vtx_off=np.asarray(vtx_off, dtype=np.int32),
                 bin_size=bin_size, name=f"batch{num_scenes}x{size}")


def mixed(seed: int = 6006, width: int = 1920, height: int = 1080, num_small: int = 1 << 20,
          num_large: int = 512, small_len: float = math.log(4.0), large_len: float = math.log(150.0),
          sigma: float = 0.5) -> Scene:
    """One frame of many small and some large triangles (the Fairy Forest
    class, "many small and large"): ``num_small`` triangles with edges
    log-normal around 4 px and ``num_large`` around 150 px, in random
    submission order, one z ~ U[0, 1) per vertex, RGB ~ U[0, 1); NDC input,
    w = 1."""
    rng = np.random.default_rng(seed)
    T = num_small + num_large
    mu = np.where(rng.permutation(T) < num_large, large_len, small_len)
    v0 = rng.uniform(0.0, 1.0, size=(2, T)) * np.array([[width], [height]])
    L = rng.lognormal(mu, sigma, size=(2, T))
    th = rng.uniform(0.0, 2 * math.pi, size=(2, T))
    v1 = v0 + L[0] * np.stack([np.cos(th[0]), np.sin(th[0])])
    v2 = v0 + L[1] * np.stack([np.cos(th[1]), np.sin(th[1])])
    xy = np.stack([v0, v1, v2], axis=2).reshape(2, 3 * T)        # vertex 3t+k
    ndc = xy / np.array([[width / 2.0], [height / 2.0]]) - 1.0
    z = rng.uniform(0.0, 1.0, size=(1, 3 * T))
    pos = np.concatenate([ndc, z]).astype(np.float32)
    color = rng.uniform(0.0, 1.0, size=(3, 3 * T)).astype(np.float32)
    return Scene(width, height, pos, color, None, T, name=f"mixed{num_small}+{num_large}")


def split_batch(sc: Scene, s: int) -> Scene:
    """Scene ``s`` of a concatenated batch as a plain single-scene input."""
    t0, t1 = int(sc.scene_tri_off[s]), int(sc.scene_tri_off[s + 1])
    v0, v1 = int(sc.scene_vtx_off[s]), int(sc.scene_vtx_off[s + 1])
    idx = None if sc.idx is None else np.ascontiguousarray(sc.idx[t0:t1])
    mvp = None if sc.mvp is None else sc.mvp[s:s + 1].copy()
    return Scene(sc.width, sc.height, np.ascontiguousarray(sc.pos[:, v0:v1]),
                 np.ascontiguousarray(sc.color[:, v0:v1]), idx, t1 - t0, mvp=mvp,
                 bin_size=sc.bin_size, shading=sc.shading, name=f"{sc.name}[{s}]")


# ---------------------------------------------------------------------------
# diffgrid: textured grid seen from many viewpoints (instanced views)
# ---------------------------------------------------------------------------
def view_mvps(num_views: int, aspect: float = 1.0) -> np.ndarray:
    """View j: yaw -15 + 30*(j mod 8)/7 degrees, pitch -10 + 20*floor(j/8)/7
    degrees about the grid centre (0, 0, 0.5), eye 2 units in front."""
    proj = perspective(60.0, aspect, 0.1, 10.0)
    out = []
    for j in range(num_views):
        yaw = -15.0 + 30.0 * (j % 8) / 7.0
        pitch = -10.0 + 20.0 * (j // 8) / 7.0
        view = translate(0.0, 0.0, 2.0) @ rot_x(pitch) @ rot_y(yaw) @ translate(0.0, 0.0, -0.5)
        out.append((proj @ view).astype(np.float32).reshape(16))
    return np.stack(out)


def diffgrid(seed: int = 5000, size: int = 512, num_views: int = 64, nx: int = 1024,
             ny: int = 512, tex_size: int = 512, bin_size: int = 16) -> Scene:
    pos, uv, idx = grid_mesh(nx, ny, 1002)
    rng = np.random.default_rng(seed)
    color = rng.uniform(0.0, 1.0, size=(3, pos.shape[1])).astype(np.float32)
    tex = rng.uniform(0.0, 1.0, size=(tex_size, tex_size, 3)).astype(np.float32)
    return Scene(size, size, pos, color, idx, idx.shape[0], mvp=view_mvps(num_views),
                 num_scenes=num_views, instanced=True, uv=uv, texture=tex,
                 bin_size=bin_size, shading="textured", name=f"diffgrid{num_views}x{size}")


# ---------------------------------------------------------------------------
# patches: a bumpy surface of bicubic Bezier patches for the Reyes front end
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class PatchScene:
    """Inputs of the Reyes front end: bicubic Bezier patches, each 16 control
    points row-major over (v, u) (point 4i + j has u index j, v index i), a
    colour per patch, one camera, the dice threshold and grid, and lights."""

    width: int
    height: int
    patches: np.ndarray                  # [P][16][3] float32
    patch_color: np.ndarray              # [P][3] float32
    mvp: Optional[np.ndarray]            # [16] float32 row-major, None -> identity
    dice_px: float = 16.0                # dice once the screen box is <= this on both axes
    max_depth: int = 20                  # splits per patch at most
    dice_n: int = 8                      # n x n quads per diced patch
    lights: Optional[np.ndarray] = None  # [L][3] float32 unit vectors
    name: str = ""

    @property
    def num_patches(self) -> int:
        return int(self.patches.shape[0])


def patches(seed: int = 7007, width: int = 1920, height: int = 1080, pa: int = 64,
            pb: int = 32, dice_px: float = 16.0, dice_n: int = 8, max_depth: int = 20,
            num_lights: int = 1, tilt_deg: float = -60.0, noise: float = 0.03) -> PatchScene:
    """A pa x pb sheet of patches sharing their border control points (a C0
    surface): the control net spans x in [-2.3, 2.3], y in [-1.3, 1.3] with
    z = 0.1 sin(2pi(3u+p1)) sin(2pi(2v+p2)) plus N(0, noise^2) bumps per
    control point, tilted about x so that it recedes from the camera (near
    patches are many times larger on screen than far ones: uneven split
    depths, as in the paper's Reyes scenes)."""
    rng = np.random.default_rng(seed)
    p1, p2 = rng.uniform(0.0, 1.0, size=2)
    nu, nv = 3 * pa + 1, 3 * pb + 1
    u = np.arange(nu, dtype=np.float64) / (nu - 1)
    v = np.arange(nv, dtype=np.float64) / (nv - 1)
    U, Vv = np.meshgrid(u, v)            # [nv][nu]
    x = (2.0 * U - 1.0) * 2.3
    y = (2.0 * Vv - 1.0) * 1.3
    z = 0.1 * np.sin(2 * math.pi * (3 * U + p1)) * np.sin(2 * math.pi * (2 * Vv + p2))
    z = z + noise * rng.standard_normal(z.shape)
    net = np.stack([x, y, z], axis=-1)   # [nv][nu][3]
    out = np.empty((pb, pa, 4, 4, 3), np.float64)
    for b in range(pb):
        for a in range(pa):
            out[b, a] = net[3 * b:3 * b + 4, 3 * a:3 * a + 4]
    color = rng.uniform(0.2, 1.0, size=(pa * pb, 3)).astype(np.float32)
    mvp = (perspective(60.0, width / height, 0.1, 10.0) @ translate(0.0, 0.1, 2.0)
           @ rot_x(tilt_deg))
    return PatchScene(width, height, out.reshape(pa * pb, 16, 3).astype(np.float32), color,
                      mvp.astype(np.float32).reshape(16), dice_px, max_depth, dice_n,
                      lights(num_lights), name=f"patches{pa}x{pb}_{width}x{height}")

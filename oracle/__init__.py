"""CPU oracle of the binned raster pipeline (ctypes wrapper around oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the HIP path; the only thing both sides consume is the seeded input
arrays.

Scenes are duck-typed: any object with the attributes ``width, height, pos,
color, idx, num_tris, mvp, num_scenes, scene_tri_off, scene_vtx_off,
instanced, uv, normal, texture, lights, shading`` works (NumPy arrays, planes
stored as ``[channels][V]``).  Batched inputs (several scenes, or several views
of one mesh) are rendered one scene at a time, which is their definition.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from types import SimpleNamespace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wno-misleading-indentation"]

SHADING = {"gouraud": 0, "textured": 1, "deferred": 2, "lit": 3}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32),
                ("pos", C.c_void_p), ("num_vertices", C.c_int64),
                ("idx", C.c_void_p), ("num_tris", C.c_int64),
                ("mvp", C.c_void_p), ("color", C.c_void_p), ("uv", C.c_void_p),
                ("normal", C.c_void_p), ("texture", C.c_void_p),
                ("tex_w", C.c_int32), ("tex_h", C.c_int32),
                ("lights", C.c_void_p), ("num_lights", C.c_int32), ("shading", C.c_int32)]


class _Targets(C.Structure):
    _fields_ = [("color", C.c_void_p), ("depth", C.c_void_p), ("primid", C.c_void_p),
                ("bary", C.c_void_p), ("gbuf_normal", C.c_void_p), ("gbuf_albedo", C.c_void_p),
                ("cover_count", C.c_void_p), ("frag_count", C.c_void_p)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        sig = {"orc_vertices": (C.c_int, [P, P, P, P, P, P]),
               "orc_setup": (C.c_int, [P, P, P, P]),
               "orc_assign_bin": (C.c_int64, [P, C.c_int32, P, P, C.c_int64]),
               "orc_render": (C.c_int, [P, P]),
               "orc_render_rows": (C.c_int, [P, P, C.c_int32, C.c_int32]),
               "orc_depth_keys": (C.c_int, [P, C.c_int64, C.c_int64, P, P, P]),
               "orc_resolve_rows": (C.c_int, [P, P, P, C.c_int32, C.c_int32]),
               "orc_render_oit": (C.c_int, [P, P, C.c_int32, P, P, P, P]),
               "orc_backward": (C.c_int, [P, P, P, P, P, P]),
               "orc_reyes_halve": (None, [P, C.c_int, P, P]),
               "orc_reyes_decide": (C.c_int, [P, P, C.c_int, C.c_int, C.c_float, C.c_int]),
               "orc_reyes_split": (C.c_int64, [P, C.c_int64, P, C.c_int, C.c_int, C.c_float,
                                               C.c_int, P, P, C.c_int64]),
               "orc_reyes_dice": (None, [P, P, P, C.c_int64, C.c_int, P, P, P, P])}
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype, fn.argtypes = res, args
        _lib = lib
    return _lib


class using_library:
    """Temporarily route every oracle call to another build of oracle.c
    (the mutation tests compile planted mistakes into a scratch library)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _load()                      # make sure the real one is set up first
        lib = C.CDLL(self.path)
        for name in ("orc_vertices", "orc_setup", "orc_assign_bin", "orc_render", "orc_render_rows",
                     "orc_depth_keys", "orc_resolve_rows", "orc_render_oit", "orc_backward",
                     "orc_reyes_halve", "orc_reyes_decide", "orc_reyes_split", "orc_reyes_dice"):
            src, dst = getattr(_lib, name), getattr(lib, name)
            dst.restype, dst.argtypes = src.restype, src.argtypes
        _lib = lib
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


class _Keep:
    """Holds the contiguous copies alive while the C structure points at them."""


def _scene_struct(sc, keep: _Keep):
    pos = _c(sc.pos, np.float32)
    idx = _c(getattr(sc, "idx", None), np.int32)
    mvp = getattr(sc, "mvp", None)
    mvp = None if mvp is None else _c(np.asarray(mvp).reshape(-1)[:16], np.float32)
    color = _c(sc.color, np.float32)
    uv = _c(getattr(sc, "uv", None), np.float32)
    normal = _c(getattr(sc, "normal", None), np.float32)
    tex = _c(getattr(sc, "texture", None), np.float32)
    lights = getattr(sc, "lights", None)
    if lights is None:
        lights = np.array([[1.0, 1.0, 1.0]], dtype=np.float64) / np.sqrt(3.0)
    lights = _c(np.asarray(lights, dtype=np.float64).astype(np.float32).reshape(-1, 3), np.float32)
    keep.arrays = [pos, idx, mvp, color, uv, normal, tex, lights]
    shading = SHADING[getattr(sc, "shading", "gouraud")]
    s = _Scene(int(sc.width), int(sc.height), _ptr(pos), pos.shape[1], _ptr(idx),
               int(sc.num_tris), _ptr(mvp), _ptr(color), _ptr(uv), _ptr(normal), _ptr(tex),
               0 if tex is None else tex.shape[1], 0 if tex is None else tex.shape[0],
               _ptr(lights), lights.shape[0], shading)
    return s


def scene_parts(sc):
    """Yield single-scene views of a (possibly batched) scene."""
    S = int(getattr(sc, "num_scenes", 1) or 1)
    if S == 1:
        yield sc
        return
    if getattr(sc, "instanced", False):
        for s in range(S):
            d = dict(vars(sc))
            d.update(mvp=np.asarray(sc.mvp)[s].reshape(16), num_scenes=1, instanced=False)
            yield SimpleNamespace(**d)
        return
    for s in range(S):
        t0, t1 = int(sc.scene_tri_off[s]), int(sc.scene_tri_off[s + 1])
        v0, v1 = int(sc.scene_vtx_off[s]), int(sc.scene_vtx_off[s + 1])
        d = dict(vars(sc))
        d.update(pos=sc.pos[:, v0:v1], color=sc.color[:, v0:v1], num_tris=t1 - t0,
                 idx=None if sc.idx is None else sc.idx[t0:t1],
                 mvp=None if sc.mvp is None else np.asarray(sc.mvp)[s].reshape(16),
                 uv=None if getattr(sc, "uv", None) is None else sc.uv[:, v0:v1],
                 normal=None if getattr(sc, "normal", None) is None else sc.normal[:, v0:v1],
                 num_scenes=1)
        yield SimpleNamespace(**d)


def vertices(sc):
    """Per-vertex snap: (X, Y, z, iw, valid) for one scene."""
    lib = _load()
    keep = _Keep()
    s = _scene_struct(sc, keep)
    V = s.num_vertices
    X = np.zeros(V, np.int32); Y = np.zeros(V, np.int32)
    z = np.zeros(V, np.float32); iw = np.zeros(V, np.float32); valid = np.zeros(V, np.uint8)
    lib.orc_vertices(C.byref(s), _ptr(X), _ptr(Y), _ptr(z), _ptr(iw), _ptr(valid))
    return X, Y, z, iw, valid.astype(bool)


def setup(sc):
    """Per-triangle setup: (live[T] bool, bbox[T][4] = x0,x1,y0,y1, A2[T] int64)."""
    lib = _load()
    keep = _Keep()
    s = _scene_struct(sc, keep)
    T = int(sc.num_tris)
    live = np.zeros(T, np.uint8); bbox = np.zeros((T, 4), np.int32); A2 = np.zeros(T, np.int64)
    lib.orc_setup(C.byref(s), _ptr(live), _ptr(bbox), _ptr(A2))
    return live.astype(bool), bbox, A2


def assign_bin(sc, bin_size: int):
    """CSR bin lists (offsets[nbins+1], tris ascending per bin) for one scene."""
    lib = _load()
    keep = _Keep()
    s = _scene_struct(sc, keep)
    bw = bin_size if bin_size > 0 else sc.width
    bh = bin_size if bin_size > 0 else sc.height
    nbins = ((sc.width + bw - 1) // bw) * ((sc.height + bh - 1) // bh)
    off = np.zeros(nbins + 1, np.int32)
    total = lib.orc_assign_bin(C.byref(s), int(bin_size), _ptr(off), None, 0)
    tris = np.zeros(max(total, 1), np.int32)
    lib.orc_assign_bin(C.byref(s), int(bin_size), _ptr(off), _ptr(tris), int(total))
    return off, tris[:total]


def render(sc, want_bary: bool = True, want_gbuf: bool = None, want_cover: bool = False,
           threads: int = 1):
    """Render every scene of ``sc``.  Returns a dict of arrays with a leading
    scene axis: color [S][H][W][4], depth, primid, bary, gbuf_normal,
    gbuf_albedo, cover_count, frag_count [S].

    ``threads`` > 1 renders on that many host threads (the C calls release
    the interpreter lock).  Several scenes run side by side.  A single scene
    splits its triangles into one range per thread, each range's depth test
    into a key buffer of its own (orc_depth_keys); the element-wise minimum
    of those buffers is the scene's (the test is a minimum over keys), and
    bands of pixel rows are then resolved and shaded on the threads
    (orc_resolve_rows).  The result is the single-threaded one bit for
    bit."""
    lib = _load()
    parts = list(scene_parts(sc))
    S, H, W = len(parts), int(sc.height), int(sc.width)
    if want_gbuf is None:
        want_gbuf = getattr(sc, "shading", "gouraud") == "deferred"
    out = dict(color=np.zeros((S, H, W, 4), np.float32), depth=np.zeros((S, H, W), np.float32),
               primid=np.zeros((S, H, W), np.int32),
               bary=np.zeros((S, H, W, 2), np.float32) if want_bary else None,
               gbuf_normal=np.zeros((S, H, W, 3), np.float32) if want_gbuf else None,
               gbuf_albedo=np.zeros((S, H, W, 3), np.float32) if want_gbuf else None,
               cover_count=np.zeros((S, H, W), np.int32) if want_cover else None,
               frag_count=np.zeros(S, np.uint64))
    structs = []
    for part in parts:
        keep = _Keep()
        structs.append((_scene_struct(part, keep), keep))

    def targets(i, fc):
        sel = lambda a: None if a is None else a[i].ctypes.data  # noqa: E731
        return _Targets(sel(out["color"]), sel(out["depth"]), sel(out["primid"]),
                        sel(out["bary"]), sel(out["gbuf_normal"]), sel(out["gbuf_albedo"]),
                        sel(out["cover_count"]), None if fc is None else fc.ctypes.data)

    if threads <= 1 or S > 1:
        fc = np.zeros((S, 1), np.uint64)

        def one(i):
            t = targets(i, fc[i])
            return lib.orc_render_rows(C.byref(structs[i][0]), C.byref(t), 0, H)
        if threads <= 1:
            rcs = [one(i) for i in range(S)]
        else:
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(max_workers=threads) as ex:
                rcs = list(ex.map(one, range(S)))
        if any(rc != 0 for rc in rcs):
            raise MemoryError("oracle render failed")
        out["frag_count"][:] = fc[:, 0]
        return out

    from concurrent.futures import ThreadPoolExecutor
    s0 = C.byref(structs[0][0])
    T = int(parts[0].num_tris)
    edges = [T * k // threads for k in range(threads + 1)]
    zbs = [np.full(H * W, np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64) for _ in range(threads)]
    covs = [np.zeros(H * W, np.int32) if want_cover else None for _ in range(threads)]
    fcs = np.zeros((threads, 1), np.uint64)

    def keys(k):
        return lib.orc_depth_keys(s0, edges[k], edges[k + 1], zbs[k].ctypes.data,
                                  None if covs[k] is None else covs[k].ctypes.data,
                                  fcs[k].ctypes.data)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(keys, range(threads)))
    zbuf = zbs[0]
    for zb in zbs[1:]:
        np.minimum(zbuf, zb, out=zbuf)
    del zbs
    if want_cover:
        out["cover_count"][0] = np.sum(covs, axis=0).reshape(H, W)
    out["frag_count"][0] = fcs.sum()
    nb = min(H, 4 * threads)
    rows = [H * k // nb for k in range(nb + 1)]
    t = targets(0, None)

    def shade(b):
        return lib.orc_resolve_rows(s0, zbuf.ctypes.data, C.byref(t), rows[b], rows[b + 1])
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(shade, range(nb)))
    return out


def render_oit(sc, alpha, layers: int):
    """Order-independent transparency of a one-scene Gouraud scene: the
    `layers` nearest fragments of every pixel composited nearest first with
    the per-vertex opacities `alpha` [V] (see orc_render_oit).  Returns
    color [1][H][W][4], depth, primid, bary with a leading scene axis."""
    lib = _load()
    parts = list(scene_parts(sc))
    assert len(parts) == 1, "one scene"
    H, W = int(sc.height), int(sc.width)
    out = dict(color=np.zeros((1, H, W, 4), np.float32), depth=np.zeros((1, H, W), np.float32),
               primid=np.zeros((1, H, W), np.int32), bary=np.zeros((1, H, W, 2), np.float32))
    keep = _Keep()
    s = _scene_struct(parts[0], keep)
    a = np.ascontiguousarray(alpha, np.float32)
    rc = lib.orc_render_oit(C.byref(s), _ptr(a), int(layers), _ptr(out["color"]),
                            _ptr(out["depth"]), _ptr(out["primid"]), _ptr(out["bary"]))
    if rc != 0:
        raise MemoryError("oracle render failed")
    return out


def backward(sc, primid, bary, grad):
    """Reference gradients (float64) for every scene of ``sc``, accumulated
    over scenes: (grad_vcolor [3][V], grad_tex [th][tw][3] or None)."""
    lib = _load()
    V = sc.pos.shape[1]
    gv = np.zeros((3, V), np.float64)
    tex = getattr(sc, "texture", None)
    gt = np.zeros(tex.shape, np.float64) if tex is not None else np.zeros(1, np.float64)
    instanced = getattr(sc, "instanced", False)
    for i, part in enumerate(scene_parts(sc)):
        keep = _Keep()
        s = _scene_struct(part, keep)
        pid = np.ascontiguousarray(primid[i], np.int32)
        ba = np.ascontiguousarray(bary[i], np.float32)
        g = np.ascontiguousarray(grad[i], np.float32)
        if instanced or int(getattr(sc, "num_scenes", 1) or 1) == 1:
            lib.orc_backward(C.byref(s), _ptr(pid), _ptr(ba), _ptr(g), _ptr(gv), _ptr(gt))
        else:
            v0, v1 = int(sc.scene_vtx_off[i]), int(sc.scene_vtx_off[i + 1])
            sub = np.zeros((3, v1 - v0), np.float64)
            lib.orc_backward(C.byref(s), _ptr(pid), _ptr(ba), _ptr(g), _ptr(sub), _ptr(gt))
            gv[:, v0:v1] += sub
    return gv, (gt if tex is not None else None)


# ---------------------------------------------------------------------------
# Reyes front end (Split and Dice of bicubic Bezier patches, Sec. 7.1)
# ---------------------------------------------------------------------------
def _mvp(mvp):
    return None if mvp is None else np.ascontiguousarray(np.asarray(mvp, np.float32).reshape(16))


def reyes_halve(cp, direction: int):
    """Halves of one patch [16][3] at u = 1/2 (direction 0) or v = 1/2 (1)."""
    lib = _load()
    cp = np.ascontiguousarray(cp, np.float32).reshape(16, 3)
    lo, hi = np.zeros((16, 3), np.float32), np.zeros((16, 3), np.float32)
    lib.orc_reyes_halve(_ptr(cp), int(direction), _ptr(lo), _ptr(hi))
    return lo, hi


def reyes_decide(cp, mvp, width: int, height: int, dice_px: float, last: bool = False) -> int:
    """0 drop, 1 dice, 2 split in u, 3 split in v (see orc_reyes_decide)."""
    lib = _load()
    cp = np.ascontiguousarray(cp, np.float32).reshape(16, 3)
    m = _mvp(mvp)
    return int(lib.orc_reyes_decide(_ptr(cp), _ptr(m), int(width), int(height),
                                    float(dice_px), int(bool(last))))


def reyes_split(patches, mvp, width: int, height: int, dice_px: float, max_depth: int):
    """Breadth-first Split of patches [P][16][3]: (leaves [L][16][3], source
    patch of each leaf [L]) in the order the rounds emit them."""
    lib = _load()
    pt = np.ascontiguousarray(patches, np.float32).reshape(-1, 16, 3)
    m = _mvp(mvp)
    cap = max(4 * len(pt), 16)
    while True:
        leaves = np.zeros((cap, 16, 3), np.float32)
        src = np.zeros(cap, np.int32)
        n = int(lib.orc_reyes_split(_ptr(pt), len(pt), _ptr(m), int(width), int(height),
                                    float(dice_px), int(max_depth), _ptr(leaves), _ptr(src), cap))
        if n < 0:
            raise MemoryError("oracle split failed")
        if n <= cap:
            return leaves[:n].copy(), src[:n].copy()
        cap = n


def reyes_dice(leaves, src, patch_color, n: int):
    """Dice every leaf into an (n+1) x (n+1) vertex grid: (pos [3][V], color
    [3][V], normal [3][V], idx [2 n^2 L][3]) with V = L (n+1)^2."""
    lib = _load()
    lv = np.ascontiguousarray(leaves, np.float32).reshape(-1, 16, 3)
    sr = np.ascontiguousarray(src, np.int32)
    pc = np.ascontiguousarray(patch_color, np.float32).reshape(-1, 3)
    L, m = len(lv), int(n) + 1
    V, T = L * m * m, 2 * int(n) * int(n) * L
    pos, col, nrm = (np.zeros((3, V), np.float32) for _ in range(3))
    idx = np.zeros((T, 3), np.int32)
    lib.orc_reyes_dice(_ptr(lv), _ptr(sr), _ptr(pc), L, int(n), _ptr(pos), _ptr(col), _ptr(nrm),
                       _ptr(idx))
    return pos, col, nrm, idx


def reyes_scene(ps):
    """The micropolygon scene a patch scene dices into: Split, then Dice, as
    a one-scene indexed mesh with forward-lit shading (Shade's diffuse model)
    that ``render`` draws.  ``ps`` carries width, height, mvp, patches
    [P][16][3], patch_color [P][3], dice_px, max_depth, dice_n and lights."""
    leaves, src = reyes_split(ps.patches, ps.mvp, ps.width, ps.height, ps.dice_px, ps.max_depth)
    pos, col, nrm, idx = reyes_dice(leaves, src, ps.patch_color, ps.dice_n)
    return SimpleNamespace(width=int(ps.width), height=int(ps.height), pos=pos, color=col, idx=idx,
                           num_tris=len(idx), mvp=ps.mvp, num_scenes=1, scene_tri_off=None,
                           scene_vtx_off=None, instanced=False, uv=None, normal=nrm, texture=None,
                           lights=ps.lights, shading="lit", num_leaves=len(leaves),
                           leaf_src=src)

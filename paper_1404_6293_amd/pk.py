"""Python binding of libpk (include/pk.h): argument marshalling only.

Every step of the pipeline runs in the HIP kernels of ``libpk.so``; this
module mirrors the C structs with ctypes, hands device pointers of torch
tensors to the library and enqueues on torch's current stream.  PyTorch is
used for device memory and streams only.  If the library is missing the
calls raise: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpk.so")

# enums of pk.h
PK_OK, PK_ERR_INVALID_ARGUMENT, PK_ERR_CAPACITY, PK_ERR_HIP, PK_ERR_UNSUPPORTED = range(5)
PK_SCHED_LOAD_BALANCE, PK_SCHED_DIRECT_MAP, PK_SCHED_DYNAMIC, PK_SCHED_SPLIT, PK_SCHED_FRAGMENT_BINS = range(5)
PK_SHADE_GOURAUD, PK_SHADE_TEXTURED, PK_SHADE_DEFERRED, PK_SHADE_LIT = range(4)
PK_FLAG_COUNT_FRAGS = 1
PK_FLAG_FUSE_RESOLVE = 2
PK_FLAG_DEFER_SHADE = 4
PK_FLAG_TWO_LEVEL_BINS = 8

SCHEDULES = {"load_balance": PK_SCHED_LOAD_BALANCE, "direct_map": PK_SCHED_DIRECT_MAP,
             "dynamic": PK_SCHED_DYNAMIC, "split": PK_SCHED_SPLIT,
             "fragment_bins": PK_SCHED_FRAGMENT_BINS}
SHADINGS = {"gouraud": PK_SHADE_GOURAUD, "textured": PK_SHADE_TEXTURED,
            "deferred": PK_SHADE_DEFERRED, "lit": PK_SHADE_LIT}

EXPORTS = ("pk_workspace_bytes", "pk_setup", "pk_assign_bin", "pk_raster_shade", "pk_shade",
           "pk_backward", "pk_bin_lists", "pk_status_string", "pk_render_static",
           "pk_reyes_workspace_bytes", "pk_reyes_split", "pk_reyes_dice")
# size of the library's static workspace used by pk_render_static (pk.h)
PK_STATIC_WORKSPACE_BYTES = 64 << 20


class PkError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {msg} (status {status})")
        self.status = status


class Params(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("bin_size", C.c_int32),
                ("schedule", C.c_int32), ("threads_per_bin", C.c_int32), ("shading", C.c_int32),
                ("flags", C.c_int32), ("num_scenes", C.c_int32), ("instanced", C.c_int32),
                ("persistent_groups", C.c_int32), ("split_size", C.c_int32),
                ("layers", C.c_int32)]


class Mesh(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("num_vertices", C.c_int32), ("indices", C.c_void_p),
                ("num_tris", C.c_int32), ("mvp", C.c_void_p), ("scene_tri_off", C.c_void_p),
                ("scene_vtx_off", C.c_void_p)]


class Attribs(C.Structure):
    _fields_ = [("color", C.c_void_p), ("uv", C.c_void_p), ("normal", C.c_void_p),
                ("texture", C.c_void_p), ("tex_w", C.c_int32), ("tex_h", C.c_int32),
                ("lights", C.c_void_p), ("num_lights", C.c_int32), ("alpha", C.c_void_p)]


class ReyesParams(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("dice_px", C.c_float),
                ("max_depth", C.c_int32), ("dice_n", C.c_int32)]


# most patches one Split round may queue (pk_reyes.h)
PK_REYES_MAX_QUEUE = 1 << 28


class BinView(C.Structure):
    _fields_ = [("bin_offsets", C.c_void_p), ("bin_tris", C.c_void_p), ("num_bins", C.c_int64)]


class Targets(C.Structure):
    _fields_ = [("color", C.c_void_p), ("depth", C.c_void_p), ("primid", C.c_void_p),
                ("bary", C.c_void_p), ("gbuf_normal", C.c_void_p), ("gbuf_albedo", C.c_void_p),
                ("frag_count", C.c_void_p)]


_lib = None


def lib():
    """Load libpk.so (built in-tree by ``paper_1404_6293_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1404_6293_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.pk_workspace_bytes.restype = C.c_size_t
        L.pk_workspace_bytes.argtypes = [P, P, C.c_int64]
        L.pk_setup.restype = C.c_int
        L.pk_setup.argtypes = [P, P, P, P]
        L.pk_assign_bin.restype = C.c_int
        L.pk_assign_bin.argtypes = [P, P, P, C.c_int64, P, P]
        L.pk_raster_shade.restype = C.c_int
        L.pk_raster_shade.argtypes = [P, P, P, P, P, P]
        L.pk_shade.restype = C.c_int
        L.pk_shade.argtypes = [P, P, P, P, P, P]
        L.pk_backward.restype = C.c_int
        L.pk_backward.argtypes = [P, P, P, P, P, P, P, P, P]
        L.pk_bin_lists.restype = C.c_int
        L.pk_bin_lists.argtypes = [P, P, P, P]
        L.pk_render_static.restype = C.c_int
        L.pk_render_static.argtypes = [P, P, P, P, P, P]
        L.pk_reyes_workspace_bytes.restype = C.c_size_t
        L.pk_reyes_workspace_bytes.argtypes = [P, C.c_int64, C.c_int64]
        L.pk_reyes_split.restype = C.c_int
        L.pk_reyes_split.argtypes = [P, P, C.c_int64, P, P, C.c_int64, P, P, C.c_int64,
                                     C.c_int32, C.c_int32, P, P]
        L.pk_reyes_dice.restype = C.c_int
        L.pk_reyes_dice.argtypes = [P, P, P, C.c_int64, P, C.c_int64, P, P, P, P, P]
        L.pk_status_string.restype = C.c_char_p
        L.pk_status_string.argtypes = [C.c_int]
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().pk_status_string(status).decode()


def _check(fn: str, status: int):
    if status != PK_OK:
        raise PkError(fn, status, status_string(status))


def _ref(x):
    return None if x is None else C.byref(x)


# --- the four calls of the ABI, same names -------------------------------
def pk_workspace_bytes(params: Params, mesh: Mesh, pair_capacity: int) -> int:
    return int(lib().pk_workspace_bytes(C.byref(params), C.byref(mesh), int(pair_capacity)))


def pk_setup(params: Params, mesh: Mesh, ws: int, stream: int = 0):
    _check("pk_setup", lib().pk_setup(_ref(params), _ref(mesh), ws, stream))


def pk_assign_bin(params: Params, mesh: Mesh, ws: int, pair_capacity: int, pairs_needed: int,
                  stream: int = 0):
    _check("pk_assign_bin", lib().pk_assign_bin(_ref(params), _ref(mesh), ws, int(pair_capacity),
                                                pairs_needed, stream))


def pk_raster_shade(params: Params, mesh: Mesh, attribs: Attribs, ws: int, targets: Targets,
                    stream: int = 0):
    _check("pk_raster_shade", lib().pk_raster_shade(_ref(params), _ref(mesh), _ref(attribs), ws,
                                                    _ref(targets), stream))


def pk_shade(params: Params, mesh: Mesh, attribs: Attribs, ws: int, targets: Targets,
             stream: int = 0):
    _check("pk_shade", lib().pk_shade(_ref(params), _ref(mesh), _ref(attribs), ws,
                                      _ref(targets), stream))


def pk_backward(params: Params, mesh: Mesh, attribs: Attribs, primid: int, bary: int,
                grad_color: int, grad_vcolor: int, grad_tex: int, stream: int = 0):
    _check("pk_backward", lib().pk_backward(_ref(params), _ref(mesh), _ref(attribs), primid, bary,
                                            grad_color, grad_vcolor, grad_tex, stream))


def pk_render_static(params: Params, mesh: Mesh, attribs: Attribs, targets: Targets,
                     pairs_needed: Optional[int] = None, stream: int = 0):
    _check("pk_render_static", lib().pk_render_static(_ref(params), _ref(mesh), _ref(attribs),
                                                      _ref(targets), pairs_needed, stream))


def pk_bin_lists(params: Params, mesh: Mesh, ws: int) -> BinView:
    v = BinView()
    _check("pk_bin_lists", lib().pk_bin_lists(_ref(params), _ref(mesh), ws, C.byref(v)))
    return v


# --- the Reyes front end (include/pk_reyes.h) ---------------------------
def pk_reyes_workspace_bytes(params: ReyesParams, num_patches: int, queue_capacity: int) -> int:
    return int(lib().pk_reyes_workspace_bytes(C.byref(params), int(num_patches),
                                              int(queue_capacity)))


def pk_reyes_split(params: ReyesParams, patches: int, num_patches: int, mvp: Optional[int],
                   ws: int, queue_capacity: int, leaves: Optional[int], leaf_src: Optional[int],
                   leaf_capacity: int, round_begin: int, round_end: int, counts: int,
                   stream: int = 0):
    _check("pk_reyes_split", lib().pk_reyes_split(_ref(params), patches, int(num_patches), mvp, ws,
                                                  int(queue_capacity), leaves, leaf_src,
                                                  int(leaf_capacity), int(round_begin),
                                                  int(round_end), counts, stream))


def pk_reyes_dice(params: ReyesParams, leaves: int, leaf_src: int, num_leaves: int,
                  patch_color: int, num_patches: int, pos: int, color: int, normal: int,
                  indices: int, stream: int = 0):
    _check("pk_reyes_dice", lib().pk_reyes_dice(_ref(params), leaves, leaf_src, int(num_leaves),
                                                patch_color, int(num_patches), pos, color, normal,
                                                indices, stream))


# --- convenience layer over torch device memory ---------------------------
def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    import torch
    return torch.cuda.current_stream().cuda_stream


@dataclass
class RenderConfig:
    bin_size: int = 16
    schedule: str = "direct_map"
    threads_per_bin: int = 0
    persistent_groups: int = 0
    split_size: int = 0            # schedule "split": pairs per work item (0 = 256)
    layers: int = 0                # > 0: order-independent transparency with the
                                   # scene's per-vertex `alpha` (that many layers)
    count_frags: bool = False
    want_bary: bool = True
    fuse_resolve: bool = False
    # raster_shade() stops after the depth test and shade() resolves; frame()
    # calls both (lets a caller time or overlap the two passes)
    defer_shade: bool = False
    # two bin levels: large triangles go to coarse bins of 4x the size
    two_level: bool = False


def _light_default():
    return np.array([[1.0, 1.0, 1.0]]) / np.sqrt(3.0)


class DeviceScene:
    """Inputs of one render call resident in device memory.

    ``scene`` is any object with the attributes of
    ``paper_1404_6293_amd.scenes.Scene``.  NumPy arrays are copied to the
    device once; torch tensors already on the device (e.g. vertex colours that
    require grad) are used in place.
    """

    def __init__(self, scene, device: str = "cuda"):
        import torch
        self.torch = torch
        dev = torch.device(device)
        self.device = dev

        def up(a, dtype):
            if a is None:
                return None
            if isinstance(a, torch.Tensor):
                t = a.detach() if a.requires_grad else a
                return t.to(device=dev, dtype=dtype).contiguous()
            return torch.from_numpy(np.ascontiguousarray(np.asarray(a), dtype=np.dtype(
                {torch.float32: np.float32, torch.int32: np.int32}[dtype]))).to(dev)

        sc = scene
        f32, i32 = torch.float32, torch.int32
        self.S = int(getattr(sc, "num_scenes", 1) or 1)
        self.W, self.H = int(sc.width), int(sc.height)
        self.instanced = bool(getattr(sc, "instanced", False)) and self.S > 1
        self.pos = up(sc.pos, f32)
        self.num_vertices = int(self.pos.shape[1])
        self.num_tris = int(sc.num_tris)
        self.idx = up(sc.idx, i32) if sc.idx is not None else None
        self.mvp = up(sc.mvp, f32).reshape(-1, 16) if sc.mvp is not None else None
        if self.mvp is not None and self.mvp.shape[0] != self.S:
            raise ValueError(f"mvp has {self.mvp.shape[0]} matrices for {self.S} scenes")
        batched = self.S > 1 and not self.instanced
        self.tri_off = up(sc.scene_tri_off, i32) if batched else None
        self.vtx_off = up(sc.scene_vtx_off, i32) if batched else None
        self.color = up(sc.color, f32)
        self.uv = up(getattr(sc, "uv", None), f32)
        self.normal = up(getattr(sc, "normal", None), f32)
        self.texture = up(getattr(sc, "texture", None), f32)
        self.alpha = up(getattr(sc, "alpha", None), f32)
        lights = getattr(sc, "lights", None)
        if lights is None:
            lights = _light_default()
        self.lights = up(np.asarray(lights, np.float64).astype(np.float32).reshape(-1, 3), f32)
        self.shading = SHADINGS[getattr(sc, "shading", "gouraud")]
        self.items = self.num_tris * (self.S if self.instanced else 1)

    def mesh(self) -> Mesh:
        return Mesh(_ptr(self.pos), self.num_vertices, _ptr(self.idx), self.num_tris,
                    _ptr(self.mvp), _ptr(self.tri_off), _ptr(self.vtx_off))

    def attribs(self) -> Attribs:
        tex = self.texture
        return Attribs(_ptr(self.color), _ptr(self.uv), _ptr(self.normal), _ptr(tex),
                       0 if tex is None else int(tex.shape[1]),
                       0 if tex is None else int(tex.shape[0]), _ptr(self.lights),
                       int(self.lights.shape[0]), _ptr(self.alpha))


class Renderer:
    """Renders one scene (or batch of scenes / views) held in device memory.

    ``frame()`` enqueues setup, assign-bin and raster/shade on the current
    stream without synchronizing; ``render()`` also makes sure the bin-pair
    capacity sufficed (one device-to-host read) and retries if not.
    ``capture()`` records one frame into a HIP graph for ``replay()``.
    """

    def __init__(self, scene, cfg: RenderConfig = RenderConfig(), device: str = "cuda"):
        import torch
        lib()  # fail early and loudly when the library is missing
        self.torch = torch
        self.cfg = cfg
        self.dev = scene if isinstance(scene, DeviceScene) else DeviceScene(scene, device)
        d = self.dev
        self.device = d.device
        self.S, self.W, self.H = d.S, d.W, d.H
        self.shading = d.shading
        self.params = Params(self.W, self.H, int(cfg.bin_size), SCHEDULES[cfg.schedule],
                             int(cfg.threads_per_bin), self.shading,
                             (PK_FLAG_COUNT_FRAGS if cfg.count_frags else 0)
                             | (PK_FLAG_FUSE_RESOLVE if cfg.fuse_resolve else 0)
                             | (PK_FLAG_DEFER_SHADE if cfg.defer_shade else 0)
                             | (PK_FLAG_TWO_LEVEL_BINS if cfg.two_level else 0), self.S,
                             int(d.instanced), int(cfg.persistent_groups), int(cfg.split_size),
                             int(cfg.layers))
        self.mesh = d.mesh()
        self.attribs = d.attribs()
        S, H, W = self.S, self.H, self.W
        f32 = torch.float32
        dev = self.device
        self.out_color = torch.empty((S, H, W, 4), dtype=f32, device=dev)
        self.out_depth = torch.empty((S, H, W), dtype=f32, device=dev)
        self.out_primid = torch.empty((S, H, W), dtype=torch.int32, device=dev)
        self.out_bary = torch.empty((S, H, W, 2), dtype=f32, device=dev) if cfg.want_bary else None
        deferred = self.shading == PK_SHADE_DEFERRED
        self.gbuf_n = torch.empty((S, H, W, 3), dtype=f32, device=dev) if deferred else None
        self.gbuf_a = torch.empty((S, H, W, 3), dtype=f32, device=dev) if deferred else None
        self.frag_count = torch.zeros(1, dtype=torch.int64, device=dev)
        self.targets = Targets(_ptr(self.out_color), _ptr(self.out_depth), _ptr(self.out_primid),
                               _ptr(self.out_bary), _ptr(self.gbuf_n), _ptr(self.gbuf_a),
                               _ptr(self.frag_count))
        self.pairs_needed = torch.zeros(1, dtype=torch.int64, device=dev)
        self.items = d.items
        self.graph = None
        self._alloc_ws(max(4 * self.items, 1024))

    def _alloc_ws(self, capacity: int):
        nbytes = pk_workspace_bytes(self.params, self.mesh, capacity)
        if nbytes == 0:
            raise PkError("pk_workspace_bytes", PK_ERR_INVALID_ARGUMENT, "invalid parameters")
        self.capacity = capacity
        self.ws = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
        self.graph = None   # a captured graph holds the old workspace address

    # stages, one call each
    def setup(self):
        pk_setup(self.params, self.mesh, self.ws.data_ptr(), _stream())

    def assign_bin(self):
        pk_assign_bin(self.params, self.mesh, self.ws.data_ptr(), self.capacity,
                      self.pairs_needed.data_ptr(), _stream())

    def raster_shade(self):
        pk_raster_shade(self.params, self.mesh, self.attribs, self.ws.data_ptr(), self.targets,
                        _stream())

    def shade(self):
        """Per-pixel resolve and shading of a frame whose raster_shade() ran
        with ``defer_shade``; a no-op otherwise."""
        if self.cfg.defer_shade:
            pk_shade(self.params, self.mesh, self.attribs, self.ws.data_ptr(), self.targets,
                     _stream())

    def count_fragments(self, on: bool):
        """Switch the covered-sample counter (PK_FLAG_COUNT_FRAGS) on or off
        for the following frames; the images do not change."""
        if on:
            self.params.flags |= PK_FLAG_COUNT_FRAGS
        else:
            self.params.flags &= ~PK_FLAG_COUNT_FRAGS
        self.graph = None   # a captured graph holds the old flags

    def frame(self):
        """Enqueue one whole frame; no synchronization."""
        if self.params.flags & PK_FLAG_COUNT_FRAGS:
            self.frag_count.zero_()
        self.setup()
        self.assign_bin()
        self.raster_shade()
        self.shade()

    def ensure_capacity(self) -> bool:
        """Read the pair count of the last frame; grow the workspace and return
        True when it did not fit (the frame must then be rendered again)."""
        need = int(self.pairs_needed.item())
        if need > self.capacity:
            self._alloc_ws(int(need * 1.25) + 1024)
            return True
        return False

    def render(self) -> dict:
        self.frame()
        if self.ensure_capacity():
            self.frame()
            if self.ensure_capacity():
                raise PkError("render", PK_ERR_CAPACITY, "pair capacity still exceeded")
        return self.outputs()

    def capture(self, warmup: int = 2):
        """Record one frame into a HIP graph (after sizing the workspace with a
        checked render).  Replays reuse this workspace and these outputs; a
        replay whose bin pairs outgrow the capacity writes empty pixels, which
        ``ensure_capacity`` detects afterwards (then capture again)."""
        torch = self.torch
        self.render()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self.frame()
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.frame()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("no captured graph: call capture() first")
        self.graph.replay()

    def outputs(self) -> dict:
        return dict(color=self.out_color, depth=self.out_depth, primid=self.out_primid,
                    bary=self.out_bary, gbuf_normal=self.gbuf_n, gbuf_albedo=self.gbuf_a,
                    frag_count=self.frag_count)

    def bin_lists(self):
        """CSR bin lists of the last frame, copied to the host for checking:
        (offsets[nbins_total+1], triangle numbers) as NumPy arrays."""
        import torch
        v = pk_bin_lists(self.params, self.mesh, self.ws.data_ptr())
        base = self.ws.data_ptr()
        o0 = v.bin_offsets - base
        off = self.ws[o0:o0 + 4 * (v.num_bins + 1)].view(torch.int32).cpu().numpy().copy()
        n = int(off[-1])
        o1 = v.bin_tris - base
        pairs = self.ws[o1:o1 + 4 * n].view(torch.int32).cpu().numpy().copy()
        return off, pairs

    def backward(self, grad_color, grad_vcolor, grad_tex=None):
        """Accumulate dL/d(vertex colour) (and dL/d(texel)) from the saved
        primid/bary of the last frame and the upstream colour gradient."""
        if self.out_bary is None:
            raise ValueError("backward needs the saved barycentrics (want_bary=True)")
        pk_backward(self.params, self.mesh, self.attribs, _ptr(self.out_primid),
                    _ptr(self.out_bary), _ptr(grad_color), _ptr(grad_vcolor), _ptr(grad_tex),
                    _stream())


class Reyes:
    """The Reyes pipeline of a patch scene on the GPU (Sec. 7.1): Split and
    Dice (include/pk_reyes.h), then Sample and Shade by the binned
    rasterizer drawing the diced micropolygons with forward-lit diffuse
    shading.

    ``split()`` enqueues every Split round; ``leaves()`` reads the leaf count
    (one device-to-host read, the host's check that the self-loop drained)
    and grows the queue or leaf buffer and splits again when they were too
    small; ``dice()`` enqueues Dice; ``render()`` runs the whole frame.
    ``ps`` carries width, height, patches [P][16][3], patch_color [P][3],
    mvp [16] (or None), dice_px, max_depth, dice_n and lights.
    """

    def __init__(self, ps, cfg: Optional[RenderConfig] = None, device: str = "cuda",
                 queue_capacity: Optional[int] = None, leaf_capacity: Optional[int] = None):
        import torch
        lib()
        self.torch = torch
        dev = torch.device(device)
        self.device = dev
        self.cfg = cfg if cfg is not None else RenderConfig(bin_size=16)
        self.W, self.H = int(ps.width), int(ps.height)
        f32 = torch.float32
        self.patches = torch.from_numpy(np.ascontiguousarray(
            np.asarray(ps.patches, np.float32).reshape(-1, 16, 3))).to(dev)
        self.num_patches = int(self.patches.shape[0])
        self.patch_color = torch.from_numpy(np.ascontiguousarray(
            np.asarray(ps.patch_color, np.float32).reshape(-1, 3))).to(dev)
        self.mvp = (None if ps.mvp is None else torch.from_numpy(np.ascontiguousarray(
            np.asarray(ps.mvp, np.float32).reshape(16))).to(dev))
        lights = ps.lights if getattr(ps, "lights", None) is not None else _light_default()
        self.lights = np.asarray(lights, np.float64).astype(np.float32).reshape(-1, 3)
        self.params = ReyesParams(self.W, self.H, float(ps.dice_px), int(ps.max_depth),
                                  int(ps.dice_n))
        self.counts = torch.zeros(6, dtype=torch.int64, device=dev)
        self._rounds_hint = int(ps.max_depth) + 1
        self._enqueued = 0
        P = max(self.num_patches, 1)
        self._alloc_queue(queue_capacity if queue_capacity is not None else 8 * P + 1024)
        self._alloc_leaves(leaf_capacity if leaf_capacity is not None else 8 * P + 1024)
        self.num_leaves = None
        self._mesh_leaves = None
        self.renderer = None
        del f32

    def _alloc_queue(self, cap: int):
        nbytes = pk_reyes_workspace_bytes(self.params, self.num_patches, cap)
        if nbytes == 0:
            raise PkError("pk_reyes_workspace_bytes", PK_ERR_INVALID_ARGUMENT,
                          "invalid parameters")
        self.queue_capacity = int(cap)
        self.ws = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)

    def _alloc_leaves(self, cap: int):
        self.leaf_capacity = int(cap)
        self.leaf_cp = self.torch.empty((max(cap, 1), 16, 3), dtype=self.torch.float32,
                                        device=self.device)
        self.leaf_src = self.torch.empty(max(cap, 1), dtype=self.torch.int32, device=self.device)

    def split(self, rounds: Optional[int] = None):
        """Enqueue the first ``rounds`` Split rounds (default: as many as the
        last split needed, or all of them the first time); no
        synchronization.  ``leaves()`` enqueues the rest if they were not
        enough."""
        total = int(self.params.max_depth) + 1
        k = self._rounds_hint if rounds is None else int(rounds)
        k = min(max(k, 1), total)
        self._enqueued = k
        self._split_rounds(0, k)

    def _split_rounds(self, r0: int, r1: int):
        pk_reyes_split(self.params, self.patches.data_ptr(), self.num_patches, _ptr(self.mvp),
                       self.ws.data_ptr(), self.queue_capacity, self.leaf_cp.data_ptr(),
                       self.leaf_src.data_ptr(), self.leaf_capacity, r0, r1,
                       self.counts.data_ptr(), _stream())

    def read_counts(self):
        """(leaves, largest queue, patches visited, overflow, patches queued
        for the next round, rounds with work) of the rounds run so far."""
        return tuple(int(x) for x in self.counts.cpu().tolist())

    def leaves(self) -> int:
        """Number of leaves of the last split(), after enqueueing the rounds
        it still needed, and after growing the buffers and splitting again
        when the queue or the leaf list were too small."""
        total = int(self.params.max_depth) + 1
        for _ in range(64):
            nl, need, _, overflow, pending, worked = self.read_counts()
            if overflow:
                self._alloc_queue(max(int(need * 1.25) + 1024, 2 * self.queue_capacity))
                self._split_rounds(0, self._enqueued)
            elif nl > self.leaf_capacity:
                self._alloc_leaves(int(nl * 1.25) + 1024)
                self._split_rounds(0, self._enqueued)
            elif pending and self._enqueued < total:
                # the self-loop has not drained: run the remaining rounds
                self._split_rounds(self._enqueued, total)
                self._enqueued = total
            else:
                self.num_leaves = nl
                self._rounds_hint = max(worked, 1)
                return nl
        raise PkError("pk_reyes_split", PK_ERR_CAPACITY, "queue kept overflowing")

    def _alloc_mesh(self, nl: int):
        torch = self.torch
        n = int(self.params.dice_n)
        V, T = nl * (n + 1) ** 2, 2 * n * n * nl
        f32 = torch.float32
        self.pos = torch.empty((3, V), dtype=f32, device=self.device)
        self.color = torch.empty((3, V), dtype=f32, device=self.device)
        self.normal = torch.empty((3, V), dtype=f32, device=self.device)
        self.idx = torch.empty((T, 3), dtype=torch.int32, device=self.device)
        self._mesh_leaves = nl
        self.renderer = None

    def dice(self, nl: Optional[int] = None):
        """Enqueue Dice of the first ``nl`` leaves (default: the last count)."""
        nl = self.num_leaves if nl is None else int(nl)
        if self._mesh_leaves != nl:
            self._alloc_mesh(nl)
        pk_reyes_dice(self.params, self.leaf_cp.data_ptr(), self.leaf_src.data_ptr(), nl,
                      self.patch_color.data_ptr(), self.num_patches, self.pos.data_ptr(),
                      self.color.data_ptr(), self.normal.data_ptr(), self.idx.data_ptr(),
                      _stream())

    def mesh_scene(self):
        """The diced micropolygons as a one-scene indexed, forward-lit scene
        (device tensors, used in place)."""
        from types import SimpleNamespace
        return SimpleNamespace(width=self.W, height=self.H, pos=self.pos, color=self.color,
                               idx=self.idx, num_tris=int(self.idx.shape[0]),
                               mvp=None if self.mvp is None else self.mvp.reshape(1, 16),
                               num_scenes=1, scene_tri_off=None, scene_vtx_off=None,
                               instanced=False, uv=None, normal=self.normal, texture=None,
                               lights=self.lights, shading="lit")

    def sample_shade(self) -> "Renderer":
        """The rasterizer for the current dice buffers (built once per leaf
        count); its frame() runs Sample and Shade."""
        if self.renderer is None:
            self.renderer = Renderer(self.mesh_scene(), self.cfg, device=str(self.device))
        return self.renderer

    def frame(self):
        """One whole frame: Split, the leaf-count read, Dice, Sample and
        Shade (the rasterizer's pair capacity is checked by render())."""
        self.split()
        nl = self.leaves()
        self.dice(nl)
        self.sample_shade().frame()

    def render(self) -> dict:
        self.split()
        nl = self.leaves()
        self.dice(nl)
        out = self.sample_shade().render()
        out = dict(out)
        out["num_leaves"] = nl
        return out

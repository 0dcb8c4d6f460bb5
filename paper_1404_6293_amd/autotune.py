"""Autotuner for the bin size and schedule of the screen-space stage.

The paper explores bin sizes and schedules by editing stage parameters and
observes that the best choice flips with the scene (triangle size and count)
and the target (Sec. 7.2: binning helps mixed-size scenes and hurts tiny
regular triangles; fusing Rasterizer and Fragment Shader trades load balance
for locality).  Here that exploration is automatic: every candidate
(bin size, schedule, threads per bin, fused resolve) renders the scene a few
times on the GPU, timed with HIP events, and the fastest wins.  Results are
cached in a JSON file keyed by the screen, the batch shape, the triangle
count and the measured fragments per triangle (a proxy for triangle size).
Every candidate produces the same image, so tuning never changes results.
"""
from __future__ import annotations

import itertools
import json
import math
import os
from dataclasses import asdict
from typing import Iterable, Optional

from . import pk

CACHE_ENV = "PK_AUTOTUNE_CACHE"
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pk_autotune.json")

BIN_SIZES = (0, 8, 16, 32, 64)   # 0: whole-screen bins (unbinned, Sec. 4.4)
SCHEDULES = ("direct_map", "load_balance", "dynamic", "split", "fragment_bins")
THREADS = (64, 128, 256)


def candidates(bins: Iterable[int] = BIN_SIZES, schedules: Iterable[str] = SCHEDULES,
               threads: Iterable[int] = THREADS, fused: Iterable[bool] = (False, True),
               two_level: bool = True):
    if 0 in bins:
        # whole-screen bins ignore the schedule, the bin workgroup size and
        # fusion: one candidate
        yield pk.RenderConfig(bin_size=0)
    for b, s, t, f in itertools.product([b for b in bins if b], schedules, threads, fused):
        if s == "split" and f:
            continue                      # pieces of a bin merge before the resolve
        if s == "fragment_bins":
            # fragments binned after shading: 16-64 px bins, one candidate
            # each (threads per bin and fusion do not apply)
            if b >= 16 and t == min(threads) and not f:
                yield pk.RenderConfig(bin_size=b, schedule=s)
            continue
        yield pk.RenderConfig(bin_size=b, schedule=s, threads_per_bin=t, fuse_resolve=f)
        if (two_level and b <= 16 and s in ("load_balance", "direct_map") and not f):
            # large triangles to coarse bins of 4x the size
            yield pk.RenderConfig(bin_size=b, schedule=s, threads_per_bin=t, two_level=True)


def _key(dev: "pk.DeviceScene", frags_per_tri: float, want_bary: bool) -> str:
    tb = int(round(math.log2(max(dev.items, 1))))
    fb = int(round(2 * math.log2(max(frags_per_tri, 1e-3))))
    return f"{dev.W}x{dev.H}x{dev.S}|inst{int(dev.instanced)}|T2^{tb}|fpt{fb}|sh{dev.shading}|bary{int(want_bary)}"


def _time(r: "pk.Renderer", reps: int) -> float:
    torch = r.torch
    r.render()
    for _ in range(2):
        r.frame()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        r.frame()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    if r.ensure_capacity():
        return _time(r, reps)
    ts.sort()
    return ts[len(ts) // 2]


def autotune(scene, want_bary: bool = False, cands: Optional[Iterable] = None, reps: int = 5,
             cache_path: Optional[str] = None, use_cache: bool = True, verbose: bool = False):
    """Return (best RenderConfig, {description: ms}) for ``scene`` (a Scene or
    a pk.DeviceScene)."""
    dev = scene if isinstance(scene, pk.DeviceScene) else pk.DeviceScene(scene)
    probe = pk.Renderer(dev, pk.RenderConfig(bin_size=16, count_frags=True, want_bary=False))
    probe.render()
    frags = int(probe.frag_count.item())
    del probe
    key = _key(dev, frags / max(dev.items, 1), want_bary)
    path = cache_path or os.environ.get(CACHE_ENV, DEFAULT_CACHE)
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        return pk.RenderConfig(**cache[key]["config"]), cache[key]["times"]
    times, best, best_ms = {}, None, float("inf")
    for c in (cands if cands is not None else candidates()):
        c.want_bary = want_bary
        try:
            r = pk.Renderer(dev, c)
            ms = _time(r, reps)
        except pk.PkError:
            continue
        finally:
            r = None
        desc = (f"B{c.bin_size}/{c.schedule}/t{c.threads_per_bin}/"
                f"{'fused' if c.fuse_resolve else 'split'}{'/two_level' if c.two_level else ''}")
        times[desc] = ms
        if verbose:
            print(f"autotune {key}: {desc} {ms:.4f} ms", flush=True)
        if ms < best_ms:
            best, best_ms = c, ms
    if best is None:
        raise RuntimeError("no autotuning candidate ran")
    if use_cache:
        cache[key] = {"config": asdict(best), "times": times}
        try:
            os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
            tmp = path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1)
            os.replace(tmp, path)
        except OSError:
            pass
    return best, times

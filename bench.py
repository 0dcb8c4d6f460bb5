"""Benchmark: binned software raster throughput on one MI355X.

One step = one whole frame of the hot path on resident inputs: vertex
transform + setup + bin counts (pk_setup), prefix sum + scatter of the bin
lists (pk_assign_bin), per-bin coverage and depth test (pk_raster_shade with
the shading deferred) and the per-pixel resolve / shading pass (pk_shade).
Consecutive frames rotate over three renderers on three streams (each
frame complete and in order on its stream; `single_stream` reports the same
frames run one after another).  Prints one JSON line.  Default workload: the
1920x1080
displaced grid of 1024x512 quads (1,048,576 triangles) through a perspective
camera, Gouraud shading, 16x16 bins.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


WORKLOADS = {
    "grid1080": dict(desc="1920x1080 displaced grid, 1024x512 quads (1,048,576 triangles, "
                          "shared vertices), perspective camera, Gouraud, 16x16 bins",
                     bin=16, schedule="direct_map", tpb=0, bary=False),
    "micro8m": dict(desc="1920x1080, 8,388,608 independent micropolygons (log-normal area "
                         "around 0.5 px^2), deferred shading over an fp32 G-buffer, 1 light, "
                         "whole-screen bins (the autotuned choice)",
                    bin=0, schedule="direct_map", tpb=0, bary=False),
    "batch256": dict(desc="256 scenes at 256x256, log-uniform 1K-200K random triangles each "
                          "(edge ~ log-normal around 4 px), one batched launch",
                     bin=16, schedule="direct_map", tpb=0, bary=False),
    "tiny64": dict(desc="64x64, 256 random triangles, Gouraud, 8x8 bins", bin=8,
                   schedule="direct_map", tpb=64, bary=False),
}


def make_scene(name: str):
    from paper_1404_6293_amd import scenes
    if name == "grid1080":
        return scenes.grid()
    if name == "micro8m":
        return scenes.micro()
    if name == "batch256":
        return scenes.batch()
    if name == "tiny64":
        return scenes.tiny()
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(sc, npairs: int, covered: int, want_bary: bool, B: int) -> dict:
    """Algorithmic HBM bytes of one whole frame, split over the frame's four
    stages: every input read once, every (bin, triangle) pair written once
    and read once (4 B each way), every output written once (and the
    deferred G-buffer read back once by the lighting pass).  What a stage
    passes to the next through the workspace (setup records, boxes, keys)
    is an implementation choice and is not counted.  A vertex attribute
    plane counts as read whole, or as the visible triangles' three vertex
    values per covered pixel when that is less (independent
    micropolygons, where most triangles are hidden or cover no sample).
    Instanced views read the mesh once per view.

    Stages: `setup` reads positions (and indices); `assign_bin` writes the
    pairs and the CSR offsets; `raster` reads the pairs and offsets and
    writes every pixel's depth and primitive ID; `shade` gathers the
    attributes and writes colour (bary; G-buffer, then reads it back and
    writes colour for deferred shading).  With whole-screen bins the
    triangle setup runs in the raster stage's kernel: the raster stage then
    reads the indices (indexed meshes, whose vertices the setup stage still
    transforms) or the positions.  Returns {stage: bytes, "frame": total}."""
    S = int(getattr(sc, "num_scenes", 1) or 1)
    views = S if getattr(sc, "instanced", False) else 1
    V = int(sc.pos.shape[1]) * views
    T = int(sc.num_tris) * views
    npix = S * sc.width * sc.height
    nbins = 0 if not B else S * (-(-sc.width // B)) * (-(-sc.height // B))
    shading = getattr(sc, "shading", "gouraud")
    indexed = sc.idx is not None

    def plane(ch):   # one attribute of ch float32 channels
        return min(4 * ch * V, 3 * 4 * ch * covered)
    setup = 12 * V + (12 * T if indexed else 0)
    assign = 4 * npairs + 4 * (nbins + 1)
    raster = 4 * npairs + 4 * (nbins + 1) + 8 * npix
    if not B:
        # setup fused into the per-triangle depth-test kernel
        moved = 12 * T if indexed else 12 * V
        setup -= moved
        raster += moved
    shade = plane(3)
    if shading == "textured":
        tex = getattr(sc, "texture", None)
        shade += plane(2) + min(int(tex.size) * 4 * views, 4 * 12 * covered)
    if shading == "deferred":
        shade += plane(3) + 24 * npix + 24 * npix + 16 * npix
    else:
        shade += 16 * npix
    if want_bary:
        shade += 8 * npix
    out = {"setup": setup, "assign_bin": assign, "raster": raster, "shade": shade}
    out["frame"] = sum(out.values())
    return out


def kernel_source_hash() -> str:
    """SHA-256 over the HIP sources and the public header with comments and
    whitespace removed, so that a profiled traffic figure is only reported
    for the code it was measured on (and survives comment edits)."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1404_6293_amd", "csrc")
    srcs = [f for f in sorted(os.listdir(csrc)) if not f.startswith("probe_")]
    for path in srcs + ["../../include/pk.h"]:
        with open(os.path.join(csrc, path), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(os.path.basename(path).encode())
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def profiled_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 summary
    of `workload` (FETCH_SIZE + WRITE_SIZE, each scaled by a plain copy's
    reading), or None when there is none or the kernels have changed since."""
    path = os.path.join(ROOT, "profiles", f"{workload}_kernels.md")
    if not os.path.exists(path):
        return None
    want = kernel_source_hash()
    for line in open(path):
        # "traffic <kernel> <bytes> bytes/launch sources <sha256>"
        parts = line.split()
        if (len(parts) == 6 and parts[0] == "traffic" and parts[1] == kernel
                and parts[5] == want):
            return int(parts[2])
    return None


def profiled_valu_busy(workload: str, kernel: str):
    """Percent of the time the VALU was busy during `kernel` (rocprofv3's
    VALUBusy) from the committed summary of `workload`, or None when there is
    none or the kernels have changed since."""
    path = os.path.join(ROOT, "profiles", f"{workload}_kernels.md")
    if not os.path.exists(path):
        return None
    want = kernel_source_hash()
    for line in open(path):
        # "valubusy <kernel> <percent> percent sources <sha256>"
        parts = line.split()
        if (len(parts) == 6 and parts[0] == "valubusy" and parts[1] == kernel
                and parts[5] == want):
            return float(parts[2])
    return None


def host_cpus() -> int:
    """Host threads the oracle may use: this process's CPU set, at most 16
    (a GPU machine's CPU share per GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _oracle_rate(parts, budget_s, threads, frags_of=None):
    """Render the single-scene parts one after another (cycling) with the
    oracle on `threads` host threads until `budget_s` is used (at least one).
    Returns (triangles, fragments, scenes, seconds)."""
    import oracle
    done_tris = done_frags = done = 0
    t0 = time.perf_counter()
    while True:
        part = parts[done % len(parts)]
        o = oracle.render(part, want_bary=False, threads=threads)
        done_tris += int(part.num_tris)
        done_frags += int(o["frag_count"].sum())
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    return done_tris, done_frags, done, time.perf_counter() - t0


def cpu_baseline(sc, budget_s: float = 6.0):
    """The oracle as it stands (plain C; one scene's pixel rows cut into
    bands over host threads) timed on this host on the same workload, on
    every host thread this process may use and on one: whole scenes, one
    after another, until each time budget is used (at least one)."""
    parts = list(__import__("oracle").scene_parts(sc))
    n = host_cpus()
    tris, frags, done, dt = _oracle_rate(parts, budget_s, n)
    tris1, _, done1, dt1 = _oracle_rate(parts, budget_s, 1)
    return {"value": round(tris / dt / 1e6, 3), "unit": "Mtris/s", "cores": n,
            "kind": "oracle",
            "sample": f"{done} whole-frame render(s) of the workload ({tris} triangles) on "
                      f"{n} threads in {dt:.1f} s; {done1} on one thread in {dt1:.1f} s",
            "gfrags_per_s": round(frags / dt / 1e9, 4),
            "ms_per_frame": round(dt / done * 1e3, 2),
            "single_thread": {"value": round(tris1 / dt1 / 1e6, 3), "unit": "Mtris/s",
                              "ms_per_frame": round(dt1 / done1 * 1e3, 2)},
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def cpu_baseline_configs(budget_s: float = 4.0) -> dict:
    """The oracle on the other workloads (all host threads this process may
    use), each on a bounded sample: micro8m whole frames; batch256 scenes
    (scaled to the 256-scene frame by triangles); diff64 views forward, and
    the float64 reference backward of those views, scaled to 64 views."""
    import numpy as np

    import oracle
    from paper_1404_6293_amd import scenes
    n = host_cpus()
    out = {}
    sc = scenes.micro()
    tris, frags, done, dt = _oracle_rate([sc], budget_s, n)
    out["micro8m"] = {"ms_per_frame": round(dt / done * 1e3, 1),
                      "mtris_per_s": round(tris / dt / 1e6, 3),
                      "gfrags_per_s": round(frags / dt / 1e9, 4), "frames": done}
    del sc
    sc = scenes.batch()
    parts = list(oracle.scene_parts(sc))
    total = int(sc.num_tris)
    t0 = time.perf_counter()
    done_tris = done_frags = k = 0
    while time.perf_counter() - t0 < budget_s and k < len(parts):
        o = oracle.render(parts[k], want_bary=False, threads=1)
        done_tris += int(parts[k].num_tris)
        done_frags += int(o["frag_count"].sum())
        k += 1
    dt = time.perf_counter() - t0
    # scenes are independent: n threads render n scenes side by side; the
    # sample ran on one thread, so the n-thread frame is scaled by n
    out["batch256"] = {"ms_per_frame_one_thread": round(dt * total / done_tris * 1e3, 1),
                       "ms_per_frame_est_all_threads": round(dt * total / done_tris / n * 1e3, 1),
                       "mtris_per_s_one_thread": round(done_tris / dt / 1e6, 3),
                       "scenes_sampled": k}
    del sc, parts
    sc = scenes.diffgrid()
    views = list(oracle.scene_parts(sc))
    t0 = time.perf_counter()
    fwd = bwd = 0.0
    k = 0
    rng = np.random.default_rng(0)
    while k < len(views) and time.perf_counter() - t0 < budget_s:
        a = time.perf_counter()
        o = oracle.render(views[k], want_bary=True, threads=n)
        b = time.perf_counter()
        g = rng.standard_normal((1, sc.height, sc.width, 4)).astype(np.float32)
        oracle.backward(views[k], o["primid"], o["bary"], g)
        c = time.perf_counter()
        fwd += b - a
        bwd += c - b
        k += 1
    out["diff64"] = {"forward_ms_per_64_views": round(fwd / k * 64 * 1e3, 1),
                     "backward_fp64_ms_per_64_views": round(bwd / k * 64 * 1e3, 1),
                     "views_sampled": k,
                     "note": "forward on all threads; the reference backward is single-threaded"}
    out["threads"] = n
    return out


def _median_ms(torch, fn, reps):
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def _tuned(sc, cands, want_bary=False):
    """Autotuned configuration for a scene, tuned afresh on every run (no
    cache: a stale entry from other kernels would skip the tuning)."""
    from paper_1404_6293_amd import autotune
    best, times = autotune.autotune(sc, want_bary=want_bary, cands=cands, reps=3,
                                    use_cache=False)
    return best, times


def bench_batched(reps: int = 10) -> dict:
    """256 scenes at 256x256 (log-uniform 1K-200K triangles each): one batched
    frame replayed from a captured HIP graph with an autotuned bin size and
    schedule, against the same 256 scenes rendered as 256 sequential plain
    frames with the same configuration."""
    import torch
    from paper_1404_6293_amd import autotune, pk, scenes
    sc = scenes.batch()
    dev = pk.DeviceScene(sc)
    cands = list(autotune.candidates(bins=(0, 8, 16, 32, 64),
                                     schedules=("direct_map", "dynamic", "split"),
                                     threads=(64, 128), fused=(False,)))
    cfg, times = _tuned(dev, cands)
    cfg.count_frags = True
    rb = pk.Renderer(dev, cfg)
    rb.render()
    torch.cuda.synchronize()
    frags = int(rb.frag_count.item())
    rb.count_fragments(False)
    rb.capture()
    torch.cuda.synchronize()
    ms_b = _median_ms(torch, rb.replay, reps)
    assert not rb.ensure_capacity()
    del rb
    cfg.count_frags = False
    plain = [pk.Renderer(scenes.split_batch(sc, s), cfg) for s in range(sc.num_scenes)]
    for r in plain:
        r.render()
    torch.cuda.synchronize()

    def seq():
        for r in plain:
            r.frame()
    ms_p = _median_ms(torch, seq, max(3, reps // 3))
    tris = int(sc.num_tris)
    # algorithmic bytes of the batched frame (pairs and covered pixels of the
    # tuned configuration)
    rb = pk.Renderer(dev, cfg)
    rb.render()
    torch.cuda.synchronize()
    npairs = int(rb.pairs_needed.item())
    covered = int((rb.out_primid >= 0).sum().item())
    del rb
    alg = algorithmic_bytes(sc, npairs, covered, False, cfg.bin_size)["frame"]
    return {"workload": "batch256: 256 scenes at 256x256, log-uniform 1K-200K random triangles "
                        "each (edge ~ log-normal around 4 px)",
            "roofline_frame": {"alg_bytes": alg,
                               "frac": round(alg / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "tuned": {"bin_size": cfg.bin_size, "schedule": cfg.schedule,
                      "threads_per_bin": cfg.threads_per_bin},
            "tuning_ms": {k: round(v, 4) for k, v in times.items()},
            "triangles": tris, "fragments": frags,
            "batched_graph_ms": round(ms_b, 4), "sequential_plain_ms": round(ms_p, 4),
            "speedup": round(ms_p / ms_b, 3),
            "batched_mtris_per_s": round(tris / ms_b / 1e3, 1),
            "batched_gfrags_per_s": round(frags / ms_b / 1e6, 3)}


def _stage_ms(torch, r, reps):
    """Mean ms of each of a frame's four calls (setup, assign_bin, raster,
    shade), HIP events on the launch stream; `r` renders with defer_shade."""
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(reps)]
    torch.cuda.synchronize()
    for e in ev:
        e[0].record(stream)
        r.setup()
        e[1].record(stream)
        r.assign_bin()
        e[2].record(stream)
        r.raster_shade()
        e[3].record(stream)
        r.shade()
        e[4].record(stream)
    torch.cuda.synchronize()
    names = ("setup", "assign_bin", "raster", "shade")
    return {n: sum(e[i].elapsed_time(e[i + 1]) for e in ev) / reps for i, n in enumerate(names)}


def bench_micro(reps: int = 10) -> dict:
    """2^23 micropolygons at 1920x1080 with deferred shading, bin size
    autotuned in {0 (whole-screen bins), 8, 16, 32, 64}; frame and stage
    times, the frame's fraction of the HBM roofline and, with whole-screen
    bins, the depth test's device-scope atomics against the probe's rate at
    the same address distribution (uniform over the screen)."""
    import torch
    from paper_1404_6293_amd import autotune, pk, probe, scenes
    sc = scenes.micro()
    dev = pk.DeviceScene(sc)
    cands = list(autotune.candidates(bins=(0, 8, 16, 32, 64), schedules=("direct_map",),
                                     threads=(64, 128), fused=(False,)))
    cfg, times = _tuned(dev, cands)
    cfg.count_frags = True
    cfg.defer_shade = True
    cfg.want_bary = False
    r = pk.Renderer(dev, cfg)
    r.render()
    torch.cuda.synchronize()
    frags = int(r.frag_count.item())
    npairs = int(r.pairs_needed.item())
    covered = int((r.out_primid >= 0).sum().item())
    r.count_fragments(False)
    ms = _median_ms(torch, r.frame, reps)
    st = _stage_ms(torch, r, reps)
    tris = int(sc.num_tris)
    alg = algorithmic_bytes(sc, npairs, covered, False, cfg.bin_size)
    out = {"workload": "micro8m: 1920x1080, 8,388,608 micropolygons (log-normal area around "
                       "0.5 px^2), deferred shading over an fp32 G-buffer, 1 light",
           "tuned": {"bin_size": cfg.bin_size, "schedule": cfg.schedule},
           "tuning_ms": {k: round(v, 4) for k, v in times.items()},
           "frame_ms": round(ms, 4), "mtris_per_s": round(tris / ms / 1e3, 1),
           "gfrags_per_s": round(frags / ms / 1e6, 3),
           "stage_ms": {k: round(v, 4) for k, v in st.items()},
           "covered_pixels": covered, "bin_pairs": npairs,
           "roofline_frame": {"alg_bytes": alg["frame"],
                              "frac": round(alg["frame"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
           "roofline_stages": {n: round(alg[n] / (st[n] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                               for n in st if st[n] > 0}}
    if cfg.bin_size == 0:
        npix = sc.width * sc.height
        g = torch.Generator(device="cuda")
        g.manual_seed(3)
        addr = torch.randint(0, npix, (frags,), device="cuda", dtype=torch.int32, generator=g)
        peak = probe.global_min_u64_rate(addr, npix)
        del addr
        rate = frags / (st["raster"] * 1e-3) / 1e9
        out["atomic_roofline"] = {"ops": frags, "kind": "device-scope 64-bit atomic min",
                                  "rate_g_per_s": round(rate, 2),
                                  "probe_peak_g_per_s": round(peak, 2),
                                  "probe": "pkp_global_min_u64, uniform pixel addresses",
                                  "frac": round(rate / peak, 4)}
    return out


def bench_lights(reps: int = 5) -> dict:
    """The paper's fusion and binning experiments (Sec. 7.2) with shader
    complexity as a light count: forward lighting in the fragment shader
    (colour = vertex colour x the sum of max(0, n . l) over L lights), one
    whole frame for L = 1, 4, 16, 64 in four pipelines:
      baseline       whole-screen bins, one kernel per stage (vertex/setup,
                     raster with a device-scope depth test, per-pixel
                     resolve that shades the visible fragment);
      freepipe       Rasterizer and Fragment Shader fused per triangle (every
                     covered fragment shaded, before the depth test), then
                     Depth Test + Composite per 32-px bin (fragment bins);
      binned         16-px bins, LOAD_BALANCE, shading in a per-pixel pass;
      binned_fused   16-px bins, DIRECT_MAP, shading fused into the bin kernel.
    Scenes: the 1080p grid (about 1M tiny regular triangles), micro8m (8.4M
    micropolygons) and a mixed frame of 1M small and 512 large triangles
    (many small and large), each with random unit normals."""
    import torch
    from paper_1404_6293_amd import pk, scenes
    pipes = {"baseline": dict(bin_size=0),
             "freepipe": dict(bin_size=32, schedule="fragment_bins"),
             "binned": dict(bin_size=16, schedule="load_balance"),
             "binned_fused": dict(bin_size=16, schedule="direct_map", fuse_resolve=True)}
    out = {}
    for name, make in (("grid1080", scenes.grid), ("micro8m", scenes.micro),
                       ("mixed", scenes.mixed)):
        base = make()
        res = {}
        for L in (1, 4, 16, 64):
            dev = pk.DeviceScene(scenes.with_lighting(base, L))
            for pname, c in pipes.items():
                r = pk.Renderer(dev, pk.RenderConfig(want_bary=False, **c))
                r.render()
                torch.cuda.synchronize()
                res[f"{pname}/L{L}"] = round(_median_ms(torch, r.frame, reps), 4)
                del r
            del dev
        out[name] = res
        del base
    return {"workload": "forward-lit frames (L lights) of grid1080, micro8m and a mixed "
                        "1M-small + 512-large frame in four pipelines", "frame_ms": out}


def bench_two_level(reps: int = 5) -> dict:
    """Two bin levels (hierarchical bins, the paper's non-uniform bins of
    Sec. 8) against one level: one whole frame per configuration on one
    stream (ms), with the (bin, triangle) pairs of each, on the mixed frame
    (1M small + 512 large triangles), batch256 and grid1080."""
    import torch
    from paper_1404_6293_amd import pk, scenes
    out = {}
    for name, make in (("mixed", scenes.mixed), ("batch256", scenes.batch),
                       ("grid1080", scenes.grid)):
        dev = pk.DeviceScene(make())
        res = {}
        for B in (8, 16):
            for sched in ("load_balance", "direct_map"):
                for tl in (False, True):
                    r = pk.Renderer(dev, pk.RenderConfig(bin_size=B, schedule=sched,
                                                         two_level=tl, want_bary=False))
                    r.render()
                    torch.cuda.synchronize()
                    key = f"B{B}/{sched}/{'two_level' if tl else 'one_level'}"
                    res[key] = {"frame_ms": round(_median_ms(torch, r.frame, reps), 4),
                                "pairs": int(r.pairs_needed.item())}
                    del r
        out[name] = res
        del dev
    return {"workload": "mixed, batch256 and grid1080 with 8/16-px bins, one or two bin levels "
                        "(coarse bins of 4x the size for triangles spanning more than 2x2 bins)",
            "frames": out}


def bench_reyes(reps: int = 10) -> dict:
    """The Reyes pipeline (Sec. 7.1) on a 2048-patch bumpy sheet at 1920x1080
    (dice at 16 px, 8 x 8 grids, one light): Split (every round, one stream),
    Dice, Sample + Shade of the diced micropolygons under a few rasterizer
    configurations, and the whole frame including the host's read of the
    leaf count; medians of HIP-event timings (ms).  A frame's Split enqueues
    the rounds the previous frame needed (the count of rounds with work)
    and only then the rest if the queue has not drained; Split's rate counts
    the patches visited over all rounds; the oracle's Split + Dice on the
    host is timed beside it."""
    import time
    import torch
    import oracle
    from paper_1404_6293_amd import pk, scenes
    ps = scenes.patches()
    r = pk.Reyes(ps)
    r.split()
    nl = r.leaves()
    r.dice(nl)
    torch.cuda.synchronize()
    _, largest, visits, _, _, worked = r.read_counts()
    # a frame enqueues the rounds the last one needed (then checks that the
    # queue drained); all max_depth + 1 rounds for comparison
    split_ms = _median_ms(torch, r.split, reps)
    split_all_ms = _median_ms(torch, lambda: r.split(ps.max_depth + 1), reps)
    r.split()
    torch.cuda.synchronize()
    assert r.read_counts()[4] == 0
    # the same rounds replayed from a HIP graph (launch costs only)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        r.split()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        r.split()
    g.replay()
    torch.cuda.synchronize()
    graph_ok = r.read_counts()[0] == nl
    split_graph_ms = _median_ms(torch, g.replay, reps)
    del g
    dice_ms = _median_ms(torch, lambda: r.dice(nl), reps)
    tris = int(r.idx.shape[0])
    raster = {}
    best, best_ms = None, float("inf")
    for name, cfg in (("B0", pk.RenderConfig(bin_size=0, want_bary=False)),
                      ("B8/direct_map", pk.RenderConfig(bin_size=8, want_bary=False)),
                      ("B16/direct_map", pk.RenderConfig(bin_size=16, want_bary=False)),
                      ("B32/fragment_bins", pk.RenderConfig(bin_size=32, schedule="fragment_bins",
                                                            want_bary=False))):
        r.cfg, r.renderer = cfg, None
        rr = r.sample_shade()
        rr.render()
        torch.cuda.synchronize()
        raster[name] = round(_median_ms(torch, rr.frame, reps), 4)
        if raster[name] < best_ms:
            best, best_ms = cfg, raster[name]
    r.cfg, r.renderer = best, None
    r.render()
    torch.cuda.synchronize()

    def whole():
        r.frame()
    frame_ms = _median_ms(torch, whole, reps)
    t0 = time.perf_counter()
    lv, src = oracle.reyes_split(ps.patches, ps.mvp, ps.width, ps.height, ps.dice_px,
                                 ps.max_depth)
    t1 = time.perf_counter()
    oracle.reyes_dice(lv, src, ps.patch_color, ps.dice_n)
    t2 = time.perf_counter()
    # algorithmic bytes: Split reads every visited patch (192 B) and its
    # decision, and writes each half it queues and each leaf once (192 B +
    # a 4-B source); Dice reads each leaf and its source and writes 36 B per
    # vertex (position, colour, normal) and 12 B per triangle
    n = ps.dice_n
    split_bytes = 193 * visits + 196 * (visits - ps.num_patches) + 196 * nl
    dice_bytes = 196 * nl + 36 * nl * (n + 1) ** 2 + 12 * tris

    def roof(nbytes, ms):
        a_ = nbytes / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "alg_bytes": int(nbytes), "achieved": round(a_, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(a_ / HBM_PEAK_GBS, 4)}
    return {"workload": f"{ps.name}: {ps.num_patches} bicubic patches, dice at {ps.dice_px} px "
                        f"into {ps.dice_n}x{ps.dice_n} grids, forward-lit, 1 light",
            "leaves": nl, "micropolygons": tris, "largest_queue": largest,
            "patches_visited": visits, "rounds_with_work": worked,
            "max_rounds": ps.max_depth + 1, "split_ms": round(split_ms, 4),
            "split_all_rounds_ms": round(split_all_ms, 4),
            "split_mpatches_per_s": round(visits / (split_ms * 1e-3) / 1e6, 1),
            "split_graph_ms": round(split_graph_ms, 4), "split_graph_same_leaves": graph_ok,
            "split_roofline": roof(split_bytes, split_ms),
            "dice_ms": round(dice_ms, 4),
            "dice_mtris_per_s": round(tris / (dice_ms * 1e-3) / 1e6, 1),
            "dice_roofline": roof(dice_bytes, dice_ms),
            "sample_shade_ms": raster, "frame_ms": round(frame_ms, 4),
            "frame_config": {"bin_size": best.bin_size, "schedule": best.schedule},
            "cpu_oracle": {"split_s": round(t1 - t0, 3), "dice_s": round(t2 - t1, 3),
                           "split_mpatches_per_s": round(visits / (t1 - t0) / 1e6, 2),
                           "threads": 1}}


# the paper's raster scenes at 1024x768 (triangle counts) and its K40c
# frame times (Table "cudaraster"); context only: the models are not here,
# grids of the same triangle counts stand in
PAPER_SCENES = (("Fairy Forest", 174000, 8.80), ("Mecha", 254000, 6.40),
                ("Dragon", 871000, 10.20), ("Buddha", 1100000, 11.20))


def bench_paper_resolution(reps: int = 20) -> dict:
    """The grid workload at the paper's resolution (1024x768) with the
    triangle counts of its four raster scenes: 16-px bins, DIRECT_MAP, one
    stream; medians of HIP-event frame times beside the paper's K40c times
    for the scenes of the same counts (other scenes, other hardware)."""
    import math
    import torch
    from paper_1404_6293_amd import pk, scenes
    out = {}
    for name, T, paper_ms in PAPER_SCENES:
        ny = int(round(math.sqrt(T / 4.0)))
        nx = int(round(T / (2.0 * ny)))
        sc = scenes.grid(width=1024, height=768, nx=nx, ny=ny)
        r = pk.Renderer(sc, pk.RenderConfig(bin_size=16, schedule="direct_map", want_bary=False))
        r.render()
        torch.cuda.synchronize()
        ms = _median_ms(torch, r.frame, reps)
        out[name] = {"grid_quads": [nx, ny], "triangles": int(sc.num_tris),
                     "frame_ms": round(ms, 4),
                     "mtris_per_s": round(sc.num_tris / (ms * 1e-3) / 1e6, 1),
                     "paper_k40c_ms": paper_ms,
                     "paper_k40c_mtris_per_s": round(T / (paper_ms * 1e-3) / 1e6, 1)}
        del r
    return {"workload": "1024x768 displaced grids with the triangle counts of the paper's "
                        "four raster scenes (16-px bins, one stream)", "frames": out}


def bench_ablation(reps: int = 5) -> dict:
    """The schedule ablation of Sec. 7.2 on grid1080: whole-screen bins (the
    unbinned baseline) and every bin size with each schedule, the resolve in
    its own pass or fused into the bin kernel.  One whole frame per
    configuration on one stream (median of HIP-event timings, ms); every
    configuration renders the same image."""
    from paper_1404_6293_amd import autotune, pk, scenes
    dev = pk.DeviceScene(scenes.grid())
    cands = list(autotune.candidates(bins=(0, 8, 16, 32, 64),
                                     schedules=("direct_map", "load_balance", "dynamic", "split"),
                                     threads=(0,), fused=(False, True)))
    best, times = autotune.autotune(dev, cands=cands, reps=reps, use_cache=False)
    return {"workload": "grid1080", "frame_ms": {k: round(v, 4) for k, v in times.items()},
            "fastest": {"bin_size": best.bin_size, "schedule": best.schedule,
                        "fused_resolve": best.fuse_resolve}}


def bench_transparency(reps: int = 5, bins=(8, 16, 32), layers=(0, 1, 2, 4, 8)) -> dict:
    """Order-independent transparency on batch256 (random triangles, depth
    complexity about 3.75) with per-vertex opacity ~ U[0.2, 0.8): one whole
    frame (one workgroup per bin) for 1, 2, 4 and 8 layers against the
    opaque frame.  8- and 16-px bins keep every pixel's K nearest keys in LDS
    and pass over each bin's list once; so do 32-px bins up to 3 layers, and
    peel beyond, one pass per layer.
    Each layer is one more resolved fragment per pixel."""
    import numpy as np
    import torch
    from types import SimpleNamespace
    from paper_1404_6293_amd import pk, scenes
    sc = scenes.batch()
    sc = SimpleNamespace(**{**vars(sc), "alpha": np.random.default_rng(7).uniform(
        0.2, 0.8, sc.pos.shape[1]).astype(np.float32)})
    dev = pk.DeviceScene(sc)
    out = {}
    for B in bins:
        for K in layers:
            r = pk.Renderer(dev, pk.RenderConfig(bin_size=B, schedule="load_balance",
                                                 want_bary=False, layers=K))
            r.render()
            torch.cuda.synchronize()
            name = "opaque" if K == 0 else f"layers{K}"
            out[f"B{B}/{name}"] = round(_median_ms(torch, r.frame, reps), 4)
            del r
    return {"workload": "batch256 with per-vertex opacity U[0.2, 0.8), LOAD_BALANCE, "
                        "default threads per bin; one pass with K keys per pixel in "
                        "LDS, except B32 beyond 3 layers (depth peeling)",
            "frame_ms": out}


def measured_stream_bandwidth(torch, mib: int = 1024, reps: int = 5) -> float:
    """GB/s of a plain device-to-device copy of `mib` MiB (read + write bytes
    over time), buffers far larger than the 256 MB MALL: the achievable HBM
    stream rate beside the 8 TB/s spec."""
    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    ms = _median_ms(torch, lambda: b.copy_(a), reps)
    del a, b
    return 2 * n / (ms * 1e-3) / 1e9


def scatter_rates(torch, r, sc, reps: int = 3) -> dict:
    """Rates (G/s) of plain float32 atomic scatters over the same addresses,
    in the same order, as the textured backward's: per covered pixel (pixel
    by pixel) 3 vertices x 3 channels of the winning triangle and 4 bilinear
    taps x 3 channels of the texture.  `probe`: one device-scope atomic add
    per address (pkp_global_add_f32), the atomic roofline's denominator;
    `index_add`: torch's index_add_ for comparison."""
    from paper_1404_6293_amd import probe
    prim = r.out_primid.reshape(-1)
    cov = prim >= 0
    t = prim[cov].long()
    V = sc.pos.shape[1]
    idx = torch.as_tensor(sc.idx, device="cuda").long().reshape(-1, 3)
    tri = idx[t]                                     # [N, 3] vertex numbers
    parts = [tri[:, k] + ch * V for k in range(3) for ch in range(3)]
    bary = r.out_bary.reshape(-1, 2)[cov]
    b1, b2 = bary[:, 0], bary[:, 1]
    b0 = 1.0 - b1 - b2
    uv = torch.as_tensor(sc.uv, device="cuda")
    th, tw = sc.texture.shape[0], sc.texture.shape[1]
    u = b0 * uv[0][tri[:, 0]] + b1 * uv[0][tri[:, 1]] + b2 * uv[0][tri[:, 2]]
    v = b0 * uv[1][tri[:, 0]] + b1 * uv[1][tri[:, 1]] + b2 * uv[1][tri[:, 2]]
    i0 = torch.clamp(torch.floor(u * tw - 0.5), -1, tw).long()
    j0 = torch.clamp(torch.floor(v * th - 0.5), -1, th).long()
    base = 3 * V
    for dj in (0, 1):
        for di in (0, 1):
            ii = torch.clamp(i0 + di, 0, tw - 1)
            jj = torch.clamp(j0 + dj, 0, th - 1)
            for ch in range(3):
                parts.append(base + (jj * tw + ii) * 3 + ch)
    addr = torch.stack(parts, dim=1).reshape(-1)     # pixel by pixel
    del parts, tri, bary, u, v, i0, j0
    n = 3 * V + th * tw * 3
    m = int(addr.numel())
    out = {"scatters": m,
           "probe": probe.global_add_f32_rate(addr.to(torch.int32).contiguous(), n)}
    # the same number of atomics into the same buffer, a wave's addresses
    # consecutive (one cache line per 16 lanes) or uniformly random
    seq = (torch.arange(m, device="cuda", dtype=torch.int64) % n).to(torch.int32)
    out["coalesced"] = probe.global_add_f32_rate(seq, n)
    del seq
    rnd = torch.randint(0, n, (m,), device="cuda", dtype=torch.int32)
    out["random"] = probe.global_add_f32_rate(rnd, n)
    del rnd
    vals = torch.ones(addr.numel(), dtype=torch.float32, device="cuda")
    dst = torch.zeros(n, dtype=torch.float32, device="cuda")
    ms = _median_ms(torch, lambda: dst.index_add_(0, addr, vals), reps)
    out["index_add"] = addr.numel() / (ms * 1e-3) / 1e9
    del addr, vals, dst
    return out


def bench_backward(reps: int = 10) -> dict:
    """64 views at 512x512 of the 1024x512-quad grid, textured (512x512x3):
    forward with saved barycentrics against the backward pass to vertex
    colours and texels."""
    import numpy as np
    import torch
    from paper_1404_6293_amd import pk, scenes
    sc = scenes.diffgrid()
    r = pk.Renderer(sc, pk.RenderConfig(bin_size=16, schedule="direct_map", threads_per_bin=0,
                                        want_bary=True))
    r.render()
    torch.cuda.synchronize()
    covered = int((r.out_primid >= 0).sum().item())
    ms_f = _median_ms(torch, r.frame, reps)
    g = torch.from_numpy(np.random.default_rng(0).standard_normal(
        (sc.num_scenes, sc.height, sc.width, 4)).astype(np.float32)).cuda()
    gv = torch.zeros((3, sc.pos.shape[1]), dtype=torch.float32, device="cuda")
    gt = torch.zeros(sc.texture.shape, dtype=torch.float32, device="cuda")

    def bwd():
        gv.zero_()
        gt.zero_()
        r.backward(g, gv, gt)
    ms_b = _median_ms(torch, bwd, reps)
    scatters = covered * 21
    rates = scatter_rates(torch, r, sc)
    rate = scatters / ms_b / 1e6
    return {"workload": "diff64: 64 views at 512x512 of a 1024x512-quad grid (1,048,576 "
                        "triangles), per-vertex RGB modulated by a bilinear 512x512x3 texture",
            "covered_pixels": covered, "forward_ms": round(ms_f, 4),
            "backward_ms": round(ms_b, 4), "backward_over_forward": round(ms_b / ms_f, 3),
            "fp32_scatters": scatters,
            "scatter_rate_g_per_s": round(rate, 2),
            "atomic_roofline": {"peak_g_per_s": round(rates["probe"], 2),
                                "peak_kind": "pkp_global_add_f32: one device-scope float32 "
                                             "atomic add per scatter, same addresses and order",
                                "frac": round(rate / rates["probe"], 4),
                                "coalesced_g_per_s": round(rates["coalesced"], 2),
                                "frac_of_coalesced": round(rate / rates["coalesced"], 4),
                                "random_g_per_s": round(rates["random"], 2),
                                "index_add_g_per_s": round(rates["index_add"], 2)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="grid1080", choices=sorted(WORKLOADS))
    ap.add_argument("--bin", type=int, default=-1,
                    help="bin size (0 = whole-screen bins); default: the workload's")
    ap.add_argument("--schedule", default="")
    ap.add_argument("--tpb", type=int, default=-1)
    ap.add_argument("--streams", type=int, default=3,
                    help="frames alternate between this many renderers and streams")
    ap.add_argument("--groups", type=int, default=0,
                    help="persistent workgroups of the bin kernel (0 = library default)")
    ap.add_argument("--bary", action="store_true", help="also save barycentrics")
    ap.add_argument("--fuse-resolve", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and backward comparisons")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times "
                         "(calibrates the HBM byte counters of a profiler run)")
    ap.add_argument("--transparency", type=int, default=-1, metavar="K",
                    help="only time the transparency frame of batch256 with K layers "
                         "(bin size --bin, default 16; 20 frames) and print its JSON")
    ap.add_argument("--reyes", action="store_true",
                    help="only run the Reyes pipeline's timings and print their JSON")
    ap.add_argument("--backward", action="store_true",
                    help="only time the diff64 forward and backward and print their JSON")
    args = ap.parse_args()
    if args.backward:
        print(json.dumps(bench_backward(reps=max(args.steps, 3) if args.steps < 400 else 10)),
              flush=True)
        return
    if args.reyes:
        print(json.dumps(bench_reyes(reps=max(args.steps, 3) if args.steps < 400 else 10)),
              flush=True)
        return
    if args.transparency >= 0:
        print(json.dumps(bench_transparency(reps=20, bins=(16 if args.bin < 0 else args.bin,),
                                            layers=(args.transparency,))), flush=True)
        return
    if args.copy_probe:
        import torch
        n = args.copy_probe << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "launches": 5}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(scenes/views shard across GPUs with no exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1404_6293_amd import pk

    wl = WORKLOADS[args.workload]
    sc = make_scene(args.workload)
    B = wl["bin"] if args.bin < 0 else args.bin
    sched = args.schedule or wl["schedule"]
    tpb = wl["tpb"] if args.tpb < 0 else args.tpb
    bary = args.bary or wl["bary"]
    sc.bin_size = B
    fused = args.fuse_resolve
    # the frame's raster/shade step runs as two calls (bin kernel, then the
    # per-pixel pass) so that each kernel is timed on its own
    cfg = pk.RenderConfig(bin_size=B, schedule=sched, threads_per_bin=tpb, count_frags=True,
                          want_bary=bary, fuse_resolve=fused, defer_shade=not fused,
                          persistent_groups=args.groups)
    print(f"bench: {args.workload} B={B} {sched} tpb={tpb} bary={bary} "
          f"fused={fused} steps={args.steps} warmup={args.warmup}",
          file=sys.stderr, flush=True)
    r = pk.Renderer(sc, cfg)
    r.render()                       # sizes the bin-pair capacity once
    torch.cuda.synchronize()
    frags = int(r.frag_count.item())
    npairs = int(r.pairs_needed.item())
    covered = int((r.out_primid >= 0).sum().item())
    # the fragment count is a statistic of the (deterministic) frame, taken
    # once above; the timed frames render without the counter
    r.count_fragments(False)
    for _ in range(args.warmup):
        r.frame()
    torch.cuda.synchronize()

    K = args.steps
    stream = torch.cuda.current_stream()
    # Headline: K whole frames, each one complete (setup, binning, bin kernel,
    # resolve) and in order on its stream, rotating over three renderers
    # (own workspace and outputs, shared inputs) on three streams so that one
    # frame's small kernels overlap another's large ones (grid1080: 0.068 ms
    # per frame with three, 0.071 with two, 0.075 with four).  No event inside
    # a frame (an event record costs the queue a few microseconds).
    nst = max(1, args.streams)
    rs = [r] + [pk.Renderer(r.dev, cfg) for _ in range(nst - 1)]
    for x in rs[1:]:
        x.count_fragments(False)
        x.render()
    streams = [torch.cuda.Stream() for _ in range(nst)]   # default priority
    for _ in range(args.warmup):
        for x, st in zip(rs, streams):
            with torch.cuda.stream(st):
                x.frame()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        with torch.cuda.stream(streams[k % nst]):
            rs[k % nst].frame()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for x in rs:
        assert not x.ensure_capacity(), "bin-pair capacity changed during the timed region"
    for x in rs[1:]:
        assert torch.equal(x.out_primid, r.out_primid), "pipelined frames differ"
        assert torch.equal(x.out_color, r.out_color), "pipelined frames differ"
    # the same frames one after another on one stream (a frame's latency)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(K):
        r.frame()
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t1
    # cold frames: a 512 MB scratch write before each flushes the 256 MB
    # last-level cache (MALL), so the frame reads its inputs from HBM; the
    # median of HIP-event timings around the frame alone
    cold_ms = None
    try:
        scratch = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        cold = []
        for _ in range(min(K, 20)):
            scratch.fill_(1)
            c0 = torch.cuda.Event(enable_timing=True)
            c1 = torch.cuda.Event(enable_timing=True)
            c0.record(stream)
            r.frame()
            c1.record(stream)
            torch.cuda.synchronize()
            cold.append(c0.elapsed_time(c1))
        cold.sort()
        cold_ms = cold[len(cold) // 2]
        del scratch
    except RuntimeError:      # not enough free memory for the scratch buffer
        pass
    # the same K frames again with HIP events around each stage on the launch
    # stream: per-stage (per-kernel) durations for the roofline
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(K)]
    torch.cuda.synchronize()
    for k in range(K):
        e = ev[k]
        e[0].record(stream)
        r.setup()
        e[1].record(stream)
        r.assign_bin()
        e[2].record(stream)
        r.raster_shade()
        e[3].record(stream)
        r.shade()
        e[4].record(stream)
    torch.cuda.synchronize()
    names = ("setup", "assign_bin", "raster", "shade")
    stage = {n: sum(e[i].elapsed_time(e[i + 1]) for e in ev) / K for i, n in enumerate(names)}
    ms = dt * 1e3 / K
    S = int(getattr(sc, "num_scenes", 1) or 1)
    tris = int(sc.num_tris) * (S if getattr(sc, "instanced", False) else 1)
    mtris = tris / (ms * 1e-3) / 1e6
    gfrags = frags / (ms * 1e-3) / 1e9

    # algorithmic bytes per stage; the dominant kernel is the longest stage's
    alg = algorithmic_bytes(sc, npairs, covered, bary, B)
    deferred = getattr(sc, "shading", "gouraud") == "deferred"
    kernels = {"setup": ("k_vertex + k_setup" if sc.idx is not None else "k_setup") if B
               else ("k_vertex" if sc.idx is not None else "(none: setup runs in k_direct)"),
               "assign_bin": "k_scan + k_scatter" if B else "(none: whole-screen bins)",
               "raster": "k_direct" if B == 0 else "k_raster",
               "shade": "k_resolve" + (" + k_deferred" if deferred else "")}
    shares = dict(alg)
    if fused and B:
        # the resolve runs inside the bin kernel: its bytes are that launch's
        kernels["raster"] = "k_raster (fused resolve)"
        shares["raster"] += shares["shade"] - 8 * S * sc.width * sc.height
        shares["shade"] = 0
    stages = {}
    for n in names:
        t_n = stage[n]
        a_n = shares[n] / (t_n * 1e-3) / 1e9 if t_n > 0 else 0.0
        stages[n] = {"kernel": kernels[n], "alg_bytes": shares[n], "avg_ms": round(t_n, 4),
                     "achieved": round(a_n, 1), "frac": round(a_n / HBM_PEAK_GBS, 4)}
    dom = max(("raster", "shade"), key=lambda n: stage[n])
    kern = stages[dom]["kernel"]
    t_ms, alg_k = stage[dom], shares[dom]
    achieved = alg_k / (t_ms * 1e-3) / 1e9
    # the committed profile's name for the stage's kernels (no spaces)
    prof_name = kern.replace(" ", "") if not kern.startswith("(") else None
    roofline = {"bound": "hbm", "kernel": kern, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic(args.workload, prof_name) if prof_name else None,
                "alg_bytes_per_launch": alg_k, "avg_launch_ms": round(t_ms, 4),
                "valu_busy_pct": profiled_valu_busy(args.workload, prof_name) if prof_name else None,
                "alg_bytes_definition": "inputs read once + 8 B per (bin, triangle) pair + "
                                        "outputs written once; workspace records excluded",
                "frame": {"alg_bytes": alg["frame"],
                          "achieved": round(alg["frame"] / (ms * 1e-3) / 1e9, 1),
                          "frac": round(alg["frame"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "frac_single_stream": round(alg["frame"] / (dt1 / K) / 1e9
                                                      / HBM_PEAK_GBS, 4),
                          "frac_sum_of_stages": round(alg["frame"] / (sum(stage.values()) * 1e-3)
                                                      / 1e9 / HBM_PEAK_GBS, 4)},
                "stages": stages}
    if B and not fused:
        # the bin kernel's depth test: one LDS 64-bit atomic min per covered
        # sample in range, against the probe's rate into 16x16-pixel tiles
        try:
            from paper_1404_6293_amd import probe
            lds_rate = probe.lds_min_u64_rate(B * B if B <= 64 else 4096, True)
            roofline["lds_atomic"] = {"ops": frags, "rate_g_per_s": round(frags / (stage["raster"] * 1e-3) / 1e9, 2),
                                      "probe_peak_g_per_s": round(lds_rate, 1),
                                      "frac": round(frags / (stage["raster"] * 1e-3) / 1e9 / lds_rate, 4)}
        except (RuntimeError, OSError):
            roofline["lds_atomic"] = None
    try:
        roofline["measured_stream_gbs"] = round(measured_stream_bandwidth(torch), 1)
        roofline["frac_of_measured"] = round(achieved / roofline["measured_stream_gbs"], 4)
    except RuntimeError:      # not enough free memory for the probe
        roofline["measured_stream_gbs"] = None
    out = {
        "metric": "Mtris/s + Gfrags/s at 1080p (binned raster); batched/backward vs plain, 1 GPU",
        "value": round(mtris, 2), "unit": "Mtris/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64+f64+f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}", "bin_size": B,
                   "schedule": sched, "threads_per_bin": tpb, "fused_resolve": fused,
                   "saved_bary": bary, "triangles": tris,
                   "resolution": f"{sc.width}x{sc.height}", "scenes": S},
        "streams": nst,
        "single_stream": {"ms_per_step": round(dt1 * 1e3 / K, 4),
                          "value": round(tris / (dt1 * 1e3 / K * 1e-3) / 1e6, 2)},
        "gfrags_per_s": round(gfrags, 3), "fragments_per_frame": frags,
        "bin_pairs_per_frame": npairs, "stage_ms": {k: round(v, 4) for k, v in stage.items()},
        "cold_ms_per_frame": None if cold_ms is None else round(cold_ms, 4),
        "roofline": roofline,
    }
    if not args.no_extras and args.workload == "grid1080":
        print("bench: batched vs plain", file=sys.stderr, flush=True)
        out["batched"] = bench_batched()
        print("bench: backward vs forward", file=sys.stderr, flush=True)
        out["backward"] = bench_backward()
        print("bench: micropolygons", file=sys.stderr, flush=True)
        out["micro"] = bench_micro()
        print("bench: schedule ablation", file=sys.stderr, flush=True)
        out["ablation"] = bench_ablation()
        print("bench: transparency layers", file=sys.stderr, flush=True)
        out["transparency"] = bench_transparency()
        print("bench: light count", file=sys.stderr, flush=True)
        out["lights"] = bench_lights()
        print("bench: two bin levels", file=sys.stderr, flush=True)
        out["two_level"] = bench_two_level()
        print("bench: reyes", file=sys.stderr, flush=True)
        out["reyes"] = bench_reyes()
        print("bench: paper resolution", file=sys.stderr, flush=True)
        out["paper_resolution"] = bench_paper_resolution()
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        cb = cpu_baseline(sc)
        if not args.no_extras and args.workload == "grid1080":
            cb["other_workloads"] = cpu_baseline_configs()
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""GPU tests of the growths on top of the plain pipeline: batched rendering
replayed from a captured HIP graph, the differentiable wrapper (against the
oracle's reference gradient and against central differences of the GPU
forward), the autotuner, and full-size checks of the micropolygon and
batched workloads."""
import sys
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from paper_1404_6293_amd import pk, scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pk.lib()


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_graph_replays_match_eager():
    import torch
    _note("graph replay, batched scenes")
    sc = scenes.batch(num_scenes=12, size=96, tmin=200, tmax=20000, seed0=77)
    eager = pk.Renderer(sc, pk.RenderConfig(bin_size=16, schedule="dynamic", count_frags=True))
    ref = {k: v.clone() for k, v in eager.render().items() if v is not None}
    g = pk.Renderer(eager.dev, pk.RenderConfig(bin_size=16, schedule="dynamic", count_frags=True))
    g.capture()
    for rep in range(4):
        for k in ("color", "depth", "primid", "bary"):
            g.outputs()[k].fill_(7)
        eager.render()                       # unrelated eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert not g.ensure_capacity()
        for k in ("color", "depth", "primid", "bary", "frag_count"):
            assert torch.equal(g.outputs()[k], ref[k]), (rep, k)
    o = oracle.render(sc)
    np.testing.assert_array_equal(ref["primid"].cpu().numpy(), o["primid"])


def _loss(img, tgt, crop):
    y0, y1, x0, x1 = crop
    d = img[:, y0:y1, x0:x1, :3].double() - tgt[:, y0:y1, x0:x1, :3].double()
    return (d * d).sum()


def test_autograd_matches_oracle_and_central_differences():
    import torch
    from paper_1404_6293_amd.autograd import rasterize
    _note("autograd textured views")
    sc = scenes.diffgrid(size=64, num_views=3, nx=48, ny=24, tex_size=32)
    dev = "cuda"
    vcolor = torch.tensor(sc.color, device=dev, requires_grad=True)
    tex = torch.tensor(sc.texture, device=dev, requires_grad=True)
    pos = torch.tensor(sc.pos, device=dev)
    idx = torch.tensor(sc.idx, device=dev)
    uv = torch.tensor(sc.uv, device=dev)
    mvp = torch.tensor(sc.mvp, device=dev)
    rng = np.random.default_rng(5)
    tgt = torch.tensor(rng.uniform(0, 1, (3, 64, 64, 4)).astype(np.float32), device=dev)
    crop = (16, 48, 16, 48)
    kw = dict(width=64, height=64, mvp=mvp, uv=uv, texture=tex, num_views=3, bin_size=16)
    img, depth, primid = rasterize(vcolor, pos, idx, **kw)
    L = _loss(img, tgt, crop)
    L.backward()
    gv = vcolor.grad.cpu().numpy().astype(np.float64)
    gt = tex.grad.cpu().numpy().astype(np.float64)
    # reference gradient from the oracle's own forward
    o = oracle.render(sc)
    np.testing.assert_array_equal(primid.cpu().numpy(), o["primid"])
    G = np.zeros((3, 64, 64, 4), np.float32)
    y0, y1, x0, x1 = crop
    G[:, y0:y1, x0:x1, :3] = 2.0 * (o["color"][:, y0:y1, x0:x1, :3].astype(np.float64)
                                    - tgt.cpu().numpy()[:, y0:y1, x0:x1, :3])
    ov, ot = oracle.backward(sc, o["primid"], o["bary"], G)
    av, at = oracle.backward(sc, o["primid"], o["bary"], np.abs(G))
    eps = 2.0 ** -24
    assert (np.abs(gv - ov) <= 1e-4 * np.abs(ov) + 64 * eps * av + 1e-6).all()
    assert (np.abs(gt - ot) <= 1e-4 * np.abs(ot) + 64 * eps * at + 1e-6).all()
    # central differences (exact for this quadratic loss up to float32 image rounding)
    h = 1e-3
    base = img.detach()
    checked = 0
    with torch.no_grad():
        for which, param, grad in (("vcolor", vcolor, gv), ("tex", tex, gt)):
            flat = grad.reshape(-1)
            nz = np.flatnonzero(np.abs(flat) > 1e-3)
            for j in rng.choice(nz, size=min(12, nz.size), replace=False):
                vals = []
                for sgn in (1, -1):
                    p2 = param.detach().clone()
                    p2.view(-1)[j] += sgn * h
                    args = dict(kw)
                    if which == "tex":
                        args["texture"] = p2
                        im = rasterize(vcolor.detach(), pos, idx, **args)[0]
                    else:
                        im = rasterize(p2, pos, idx, **args)[0]
                    vals.append((float(_loss(im, tgt, crop)), im))
                fd = (vals[0][0] - vals[1][0]) / (2 * h)
                changed = int((vals[0][1] != base).any(dim=-1).sum())
                bound = 1e-3 * abs(flat[j]) + 1e-5 + changed * 3 * 4 * 6e-8 / (2 * h)
                assert abs(fd - flat[j]) <= bound, (which, j, fd, flat[j])
                checked += 1
    assert checked >= 12


def test_autotuner_picks_a_config_with_the_same_image(tmp_path):
    import torch
    from paper_1404_6293_amd import autotune
    _note("autotune small scene")
    sc = scenes.tiny(seed=9, width=160, height=96, num_tris=3000)
    cands = list(autotune.candidates(bins=(8, 32), schedules=("direct_map", "load_balance"),
                                     threads=(64, 256), fused=(False,)))
    best, times = autotune.autotune(sc, cands=cands, reps=3, cache_path=str(tmp_path / "c.json"))
    assert len(times) == len(cands)
    assert best.bin_size in (8, 32)
    again, _ = autotune.autotune(sc, cands=cands, reps=3, cache_path=str(tmp_path / "c.json"))
    assert again == best                      # served from the cache
    a = pk.Renderer(sc, best).render()
    b = pk.Renderer(sc, pk.RenderConfig(bin_size=16)).render()
    for k in ("color", "depth", "primid"):
        assert torch.equal(a[k], b[k])


_MICRO = {}


def _micro8m():
    """The micro8m scene and its oracle render, made once for the module."""
    if not _MICRO:
        sc = scenes.micro()
        _MICRO["scene"] = sc
        _MICRO["oracle"] = oracle.render(sc, want_bary=False)
    return _MICRO["scene"], _MICRO["oracle"]


@pytest.mark.parametrize("bin_size,schedule", [(16, "direct_map"), (0, "direct_map"),
                                               (32, "fragment_bins"), (64, "fragment_bins")])
def test_micro8m_full_frame_deferred(bin_size, schedule):
    """8,388,608 micropolygons at 1920x1080, deferred, full frame against the
    oracle: with 16-px bins, and with whole-screen bins, the benchmark's
    (autotuned) launch configuration for this workload."""
    import torch
    _note(f"micro8m full frame bin_size={bin_size} {schedule}")
    sc, o = _micro8m()
    r = pk.Renderer(sc, pk.RenderConfig(bin_size=bin_size, schedule=schedule, threads_per_bin=0,
                                        count_frags=True, want_bary=False))
    out = r.render()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out["primid"].cpu().numpy(), o["primid"])
    assert (out["depth"].cpu().numpy() == o["depth"]).all()
    np.testing.assert_allclose(out["color"].cpu().numpy(), o["color"], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(out["gbuf_normal"].cpu().numpy(), o["gbuf_normal"], rtol=1e-5, atol=1e-6)
    assert int(out["frag_count"].item()) == int(o["frag_count"].sum())


def test_batch256_sampled_scenes_and_plain_equivalence():
    """The 256-scene batch at 256x256 in one launch: 8 sampled scenes against
    the oracle, and every scene against its own plain (S=1) render."""
    import torch
    _note("batch256 full")
    sc = scenes.batch()
    rb = pk.Renderer(sc, pk.RenderConfig(bin_size=16, schedule="direct_map", threads_per_bin=0,
                                         want_bary=False))
    ob = rb.render()
    torch.cuda.synchronize()
    pid = ob["primid"].cpu().numpy()
    col = ob["color"].cpu().numpy()
    rng = np.random.default_rng(0)
    for s in rng.choice(256, size=8, replace=False):
        part = scenes.split_batch(sc, int(s))
        o = oracle.render(part, want_bary=False)
        np.testing.assert_array_equal(pid[s], o["primid"][0])
        np.testing.assert_allclose(col[s], o["color"][0], rtol=1e-5, atol=1e-6)
    for s in range(0, 256, 15):
        r1 = pk.Renderer(scenes.split_batch(sc, s), pk.RenderConfig(bin_size=16, want_bary=False))
        o1 = r1.render()
        assert torch.equal(o1["primid"][0], ob["primid"][s])
        assert torch.equal(o1["color"][0], ob["color"][s])


def _one_view(sc, j):
    d = dict(vars(sc))
    d.update(mvp=np.asarray(sc.mvp)[j:j + 1].copy(), num_scenes=1, instanced=False)
    return SimpleNamespace(**d)


def test_diff64_full_size_views_backward_and_central_differences():
    """The differentiable workload at full size: 64 views at 512x512 of the
    1,048,576-triangle grid, textured, in the benchmark's launch
    configuration.  Sampled views match the oracle element by element
    (primid and depth bit-exact); the backward of an image loss on those
    views matches the oracle's float64 gradient; and on view 0 the gradient
    of the sum-of-squares loss over the 32x32 crop at (240, 240) matches
    central differences (h = 1e-3) of the GPU forward for 256 vertex-colour
    and 256 texel scalars that reach the crop."""
    import torch
    _note("diff64 full size: forward of 64 views")
    sc = scenes.diffgrid()
    tgt_sc = scenes.diffgrid(seed=5001)
    cfg = pk.RenderConfig(bin_size=16, schedule="direct_map", threads_per_bin=0, want_bary=True)
    r = pk.Renderer(sc, cfg)
    out = r.render()
    torch.cuda.synchronize()
    views = [0, 27, 63]
    pid_v = out["primid"][views].cpu().numpy()
    bary_v = out["bary"][views].cpu().numpy()
    col_v = out["color"][views].cpu().numpy()
    dep_v = out["depth"][views].cpu().numpy()
    for i, j in enumerate(views):
        _note(f"diff64 view {j} vs oracle")
        o = oracle.render(_one_view(sc, j))
        np.testing.assert_array_equal(pid_v[i], o["primid"][0])
        assert (dep_v[i] == o["depth"][0]).all()
        np.testing.assert_allclose(col_v[i], o["color"][0], rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(bary_v[i], o["bary"][0], rtol=1e-5, atol=1e-6)
    assert (pid_v >= 0).sum() > 0.5 * pid_v.size

    # backward over all 64 views with the upstream gradient non-zero on the
    # sampled views only: the oracle's gradient of those views is the answer
    _note("diff64 backward vs oracle gradient")
    rng = np.random.default_rng(51)
    G = np.zeros((64, 512, 512, 4), np.float32)
    G[views] = rng.standard_normal((len(views), 512, 512, 4)).astype(np.float32)
    gv = torch.zeros((3, sc.pos.shape[1]), dtype=torch.float32, device="cuda")
    gt = torch.zeros(sc.texture.shape, dtype=torch.float32, device="cuda")
    r.backward(torch.from_numpy(G).cuda(), gv, gt)
    torch.cuda.synchronize()
    sub = SimpleNamespace(**{**vars(sc), "mvp": np.asarray(sc.mvp)[views].copy(),
                             "num_scenes": len(views)})
    ov, ot = oracle.backward(sub, pid_v, bary_v, G[views])
    av, at = oracle.backward(sub, pid_v, bary_v, np.abs(G[views]))
    # float32 atomics summing n terms in any order: |error| <= n eps sum|terms|
    n, eps = 1024, 2.0 ** -24
    assert (np.abs(gv.cpu().numpy() - ov) <= 1e-4 * np.abs(ov) + n * eps * av + 1e-6).all()
    assert (np.abs(gt.cpu().numpy() - ot) <= 1e-4 * np.abs(ot) + n * eps * at + 1e-6).all()
    del r, out, gv, gt
    torch.cuda.empty_cache()

    # view 0: loss over the crop against a render of a second colour set
    # and texture, its gradient, and central differences
    _note("diff64 view 0: crop gradient and central differences")
    y0, x0, cs = 240, 240, 32
    v0 = _one_view(sc, 0)
    r0 = pk.Renderer(v0, pk.RenderConfig(bin_size=16, want_bary=True))
    img = r0.render()["color"].clone()
    tgt = pk.Renderer(_one_view(tgt_sc, 0), pk.RenderConfig(bin_size=16)).render()["color"].clone()

    def loss(im):
        d = im[0, y0:y0 + cs, x0:x0 + cs, :3].double() - tgt[0, y0:y0 + cs, x0:x0 + cs, :3].double()
        return float((d * d).sum())

    Gc = torch.zeros_like(img)
    Gc[0, y0:y0 + cs, x0:x0 + cs, :3] = (2.0 * (img[0, y0:y0 + cs, x0:x0 + cs, :3].double()
                                               - tgt[0, y0:y0 + cs, x0:x0 + cs, :3].double())).float()
    gv0 = torch.zeros((3, sc.pos.shape[1]), dtype=torch.float32, device="cuda")
    gt0 = torch.zeros(sc.texture.shape, dtype=torch.float32, device="cuda")
    r0.backward(Gc, gv0, gt0)
    torch.cuda.synchronize()
    gv0, gt0 = gv0.cpu().numpy().astype(np.float64), gt0.cpu().numpy().astype(np.float64)
    pid0 = r0.out_primid.cpu().numpy()
    b0 = r0.out_bary.cpu().numpy()
    o0v, o0t = oracle.backward(v0, pid0, b0, Gc.cpu().numpy())
    a0v, a0t = oracle.backward(v0, pid0, b0, np.abs(Gc.cpu().numpy()))
    assert (np.abs(gv0 - o0v) <= 1e-4 * np.abs(o0v) + 64 * eps * a0v + 1e-6).all()
    assert (np.abs(gt0 - o0t) <= 1e-4 * np.abs(o0t) + 64 * eps * a0t + 1e-6).all()
    # parameters that reach the crop: vertices of the visible triangles, and
    # texels with a non-zero gradient there
    crop_t = np.unique(pid0[0, y0:y0 + cs, x0:x0 + cs])
    crop_t = crop_t[crop_t >= 0]
    verts = np.unique(sc.idx[crop_t].ravel())
    vpar = [(int(c), int(v)) for c, v in zip(rng.integers(0, 3, 256), rng.choice(verts, 256))]
    tnz = np.argwhere(np.abs(o0t) > 0)
    tpar = [tuple(int(x) for x in tnz[k]) for k in rng.choice(len(tnz), 256, replace=False)]
    h = 1e-3
    col_t, tex_t = r0.dev.color, r0.dev.texture
    base = img
    worst = 0.0
    for which, plist in (("vcolor", vpar), ("tex", tpar)):
        for key in plist:
            ref = float(gv0[key]) if which == "vcolor" else float(gt0[key])
            T = col_t if which == "vcolor" else tex_t
            orig = T[key].clone()
            vals = []
            for sgn in (1.0, -1.0):
                T[key] = orig + sgn * h
                r0.frame()
                im = r0.out_color
                vals.append((loss(im), float(T[key].item()), int((im != base).any(dim=-1).sum())))
            T[key] = orig
            fd = (vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1])
            changed = max(vals[0][2], vals[1][2])
            bound = 1e-3 * abs(ref) + 1e-5 + changed * 3 * 4 * 6e-8 / (2 * h)
            assert abs(fd - ref) <= bound, (which, key, fd, ref, bound)
            worst = max(worst, abs(fd - ref) / bound)
    _note(f"diff64 central differences: 512 scalars, worst error / bound = {worst:.3f}")

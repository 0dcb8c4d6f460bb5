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


def test_micro8m_full_frame_deferred():
    """8,388,608 micropolygons at 1920x1080, deferred, in the benchmark's
    launch configuration: full-frame comparison with the oracle."""
    import torch
    _note("micro8m full frame")
    sc = scenes.micro()
    r = pk.Renderer(sc, pk.RenderConfig(bin_size=16, schedule="direct_map", threads_per_bin=0,
                                        count_frags=True, want_bary=False))
    out = r.render()
    torch.cuda.synchronize()
    o = oracle.render(sc, want_bary=False)
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

"""GPU parity of PK_SCHED_FRAGMENT_BINS (fragments shaded per triangle, then
binned by pixel for the depth test and composite) against the CPU oracle,
through the C ABI.  Same bar as every other schedule: primitive IDs and
depth bit for bit, colours, barycentrics and G-buffers within 1e-5 relative
+ 1e-6 absolute, fragment counts exact, and the image bit-identical to the
triangle-binned pipeline's."""
import sys
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from paper_1404_6293_amd import pk, scenes

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-5, 1e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pk.lib()  # must load: no fallback


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_render(sc, **cfg):
    import torch
    r = pk.Renderer(sc, pk.RenderConfig(count_frags=True, **cfg))
    out = r.render()
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    res["renderer"] = r
    return res


def compare(g, o, check_bary=True, gbuf=False):
    np.testing.assert_array_equal(g["primid"], o["primid"])
    assert (g["depth"] == o["depth"]).all(), "depth expected bit-exact"
    np.testing.assert_allclose(g["color"], o["color"], rtol=RTOL, atol=ATOL)
    if check_bary and o.get("bary") is not None and g.get("bary") is not None:
        np.testing.assert_allclose(g["bary"], o["bary"], rtol=RTOL, atol=ATOL)
    if gbuf:
        np.testing.assert_allclose(g["gbuf_normal"], o["gbuf_normal"], rtol=RTOL, atol=ATOL)
        np.testing.assert_allclose(g["gbuf_albedo"], o["gbuf_albedo"], rtol=RTOL, atol=ATOL)
    assert int(g["frag_count"][0]) == int(o["frag_count"].sum())


FB = dict(schedule="fragment_bins")


@pytest.mark.parametrize("seed", range(24))
def test_tiny64_random(seed):
    B = (16, 32, 64)[seed % 3]
    _note(f"fragment bins tiny64 seed={seed} B={B}")
    sc = scenes.tiny(seed=seed)
    compare(gpu_render(sc, bin_size=B, **FB), oracle.render(sc))


@pytest.mark.parametrize("W,H,B,T", [(37, 29, 16, 40), (1, 1, 16, 20), (257, 3, 32, 100),
                                     (130, 66, 64, 500), (64, 200, 16, 1000), (300, 17, 64, 60)])
def test_ragged_screens(W, H, B, T):
    _note(f"fragment bins ragged {W}x{H} B={B} T={T}")
    sc = scenes.tiny(seed=W * 31 + H, width=W, height=H, num_tris=T)
    compare(gpu_render(sc, bin_size=B, **FB), oracle.render(sc))


def test_same_image_as_triangle_bins():
    """Binning fragments instead of triangles regroups the work only: the
    image equals the triangle-binned pipeline's bit for bit."""
    sc = scenes.tiny(seed=77, width=150, height=110, num_tris=600)
    ref = gpu_render(sc, bin_size=16, schedule="load_balance")
    compare(ref, oracle.render(sc))
    for B in (16, 32, 64):
        for defer in (False, True):
            _note(f"fragment bins vs triangle bins B={B} defer={defer}")
            g = gpu_render(sc, bin_size=B, defer_shade=defer, **FB)
            for k in ("color", "depth", "primid", "bary"):
                assert (g[k] == ref[k]).all(), (B, defer, k)
            assert int(g["frag_count"][0]) == int(ref["frag_count"][0])


@pytest.mark.parametrize("defer", [False, True])
@pytest.mark.parametrize("B", [16, 64])
def test_deferred_micropolygons(B, defer):
    _note(f"fragment bins deferred micropolygons B={B} defer={defer}")
    sc = scenes.micro(seed=11, width=256, height=128, num_tris=60000, num_lights=3)
    compare(gpu_render(sc, bin_size=B, defer_shade=defer, **FB), oracle.render(sc), gbuf=True)


def test_deferred_tie_heavy_many_lights():
    """Depth quantised to 8 levels (the smaller index must win every tie)
    and 16 lights in the fused lighting."""
    sc = scenes.micro(seed=12, width=200, height=120, num_tris=80000, z_levels=8, num_lights=16)
    compare(gpu_render(sc, bin_size=32, **FB), oracle.render(sc), gbuf=True)


def test_textured_perspective_view():
    """One view of the textured, indexed grid through a perspective matrix."""
    sc = scenes.diffgrid(size=96, num_views=3, nx=32, ny=16, tex_size=16)
    d = dict(vars(sc))
    d.update(mvp=np.asarray(sc.mvp)[1:2].copy(), num_scenes=1, instanced=False)
    v = SimpleNamespace(**d)
    compare(gpu_render(v, bin_size=32, **FB), oracle.render(v))


def test_indexed_perspective_grid():
    sc = scenes.grid(seed=3, width=200, height=120, nx=64, ny=32)
    g = gpu_render(sc, bin_size=16, **FB)
    o = oracle.render(sc)
    compare(g, o)
    assert (g["primid"] >= 0).all()


def test_empty_and_culled_inputs():
    sc = scenes.tiny(seed=1, width=40, height=30, num_tris=1)
    sc0 = SimpleNamespace(**{**vars(sc), "num_tris": 0})
    g = gpu_render(sc0, bin_size=16, **FB)
    assert (g["primid"] == -1).all() and (g["depth"] == 1).all() and (g["color"] == 0).all()
    P = [(0.0, 0.0, 0.5), (0.5, 0.0, 0.5), (0.0, 0.5, 0.5),                  # kept
         (0.0, 0.0, 0.5), (0.0, 0.0, 0.5), (0.3, 0.3, 0.5),                  # zero area
         (np.nan, 0.0, 0.5), (0.5, 0.0, 0.5), (0.0, 0.5, 0.5),               # NaN
         (3.0, 3.0, 0.5), (3.5, 3.0, 0.5), (3.0, 3.5, 0.5),                  # off screen
         (2000.0, 0.0, 0.5), (0.5, 0.0, 0.5), (0.0, 0.5, 0.5),               # guard band
         (-0.5, -0.5, 1.5), (0.5, -0.5, 1.5), (0.0, 0.5, 1.5)]               # z >= 1
    pos = np.asarray(P, np.float32).T.copy()
    col = np.random.default_rng(0).uniform(0, 1, pos.shape).astype(np.float32)
    sc = SimpleNamespace(width=32, height=32, pos=pos, color=col, idx=None,
                         num_tris=pos.shape[1] // 3, mvp=None, num_scenes=1, scene_tri_off=None,
                         scene_vtx_off=None, instanced=False, uv=None, normal=None, texture=None,
                         lights=None, shading="gouraud")
    g = gpu_render(sc, bin_size=16, **FB)
    compare(g, oracle.render(sc))
    assert set(np.unique(g["primid"])) <= {-1, 0}


def test_capacity_overflow_then_retry():
    import torch
    sc = scenes.tiny(seed=8, width=128, height=128, num_tris=500)
    r = pk.Renderer(sc, pk.RenderConfig(bin_size=32, **FB))
    r._alloc_ws(10)                      # room for 10 fragments: far too small
    r.frame()
    torch.cuda.synchronize()
    need = int(r.pairs_needed.item())
    assert need > 10
    assert (r.out_primid.cpu().numpy() == -1).all()
    assert r.ensure_capacity()
    r.frame()
    assert not r.ensure_capacity()
    o = oracle.render(sc)
    np.testing.assert_array_equal(r.out_primid.cpu().numpy(), o["primid"])


def test_unsupported_requests_are_refused():
    sc = scenes.batch(num_scenes=2, size=32, tmin=10, tmax=20)
    with pytest.raises(pk.PkError):
        pk.Renderer(sc, pk.RenderConfig(bin_size=16, **FB)).render()
    with pytest.raises(pk.PkError):
        pk.Renderer(scenes.tiny(seed=2), pk.RenderConfig(bin_size=8, **FB)).render()


# ---------------------------------------------------------------------------
# forward lighting in the fragment shader (PK_SHADE_LIT), every pipeline
# ---------------------------------------------------------------------------
LIT_MODES = {"split": dict(bin_size=16), "fused": dict(bin_size=16, fuse_resolve=True),
             "defer": dict(bin_size=32, defer_shade=True), "unbinned": dict(bin_size=0),
             "fragment_bins": dict(bin_size=32, schedule="fragment_bins"),
             "load_balance": dict(bin_size=8, schedule="load_balance", fuse_resolve=True)}


@pytest.mark.parametrize("mode", sorted(LIT_MODES))
@pytest.mark.parametrize("L", [1, 5])
def test_forward_lit_matches_oracle(mode, L):
    """colour = vertex colour x the sum over the lights of max(0, n . l),
    computed in the fragment shader: the oracle's forward-lit image (whose
    colour equals the deferred one bit for bit) on random triangles and on
    an indexed perspective grid."""
    _note(f"forward lit mode={mode} lights={L}")
    for sc in (scenes.with_lighting(scenes.tiny(seed=21 + L, width=90, height=70, num_tris=300), L),
               scenes.with_lighting(scenes.grid(seed=4, width=160, height=96, nx=48, ny=24), L,
                                    seed=9)):
        compare(gpu_render(sc, **LIT_MODES[mode]), oracle.render(sc))


def test_forward_lit_batched_scenes():
    sc = scenes.with_lighting(scenes.batch(num_scenes=4, size=64, tmin=50, tmax=2000), 3)
    o = oracle.render(sc)
    for cfg in (dict(bin_size=16), dict(bin_size=0), dict(bin_size=8, schedule="split",
                                                          split_size=16)):
        compare(gpu_render(sc, **cfg), o)

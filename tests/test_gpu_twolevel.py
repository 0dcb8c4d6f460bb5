"""GPU parity of two bin levels (PK_FLAG_TWO_LEVEL_BINS, hierarchical
bins): triangles whose box spans more than 2 x 2 bins go to coarse bins of
four times the size.  The image must equal the oracle's (and the one-level
pipeline's bit for bit), and the two levels' bin lists must hold exactly
the triangles the rule assigns them, worked out here from the oracle's
setup boxes."""
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


def gpu_render(sc, two_level=True, **cfg):
    import torch
    r = pk.Renderer(sc, pk.RenderConfig(count_frags=True, two_level=two_level, **cfg))
    out = r.render()
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    res["renderer"] = r
    return res


def compare(g, o, check_bary=True):
    np.testing.assert_array_equal(g["primid"], o["primid"])
    assert (g["depth"] == o["depth"]).all(), "depth expected bit-exact"
    np.testing.assert_allclose(g["color"], o["color"], rtol=RTOL, atol=ATOL)
    if check_bary and o.get("bary") is not None and g.get("bary") is not None:
        np.testing.assert_allclose(g["bary"], o["bary"], rtol=RTOL, atol=ATOL)
    assert int(g["frag_count"][0]) == int(o["frag_count"].sum())


def expected_lists(sc, B):
    """{bin number: sorted triangles} of one scene under the two-level rule:
    fine bins (B px) numbered row-major first, then coarse bins (4B px)."""
    live, bbox, _ = oracle.setup(sc)
    W, H = sc.width, sc.height
    nbx, nby = -(-W // B), -(-H // B)
    nbx_c = -(-W // (4 * B))
    out = {}
    for t in np.nonzero(live)[0]:
        x0, x1, y0, y1 = (int(v) for v in bbox[t])
        bx0, bx1, by0, by1 = x0 // B, x1 // B, y0 // B, y1 // B
        if bx1 - bx0 + 1 > 2 or by1 - by0 + 1 > 2:
            C = 4 * B
            for by in range(y0 // C, y1 // C + 1):
                for bx in range(x0 // C, x1 // C + 1):
                    out.setdefault(nbx * nby + by * nbx_c + bx, []).append(int(t))
        else:
            for by in range(by0, by1 + 1):
                for bx in range(bx0, bx1 + 1):
                    out.setdefault(by * nbx + bx, []).append(int(t))
    return out


@pytest.mark.parametrize("seed", range(12))
def test_tiny64_random(seed):
    B = (8, 16)[seed % 2]
    sched = ("load_balance", "direct_map")[(seed // 2) % 2]
    _note(f"two-level tiny64 seed={seed} B={B} {sched}")
    sc = scenes.tiny(seed=seed)
    compare(gpu_render(sc, bin_size=B, schedule=sched), oracle.render(sc))


@pytest.mark.parametrize("W,H,B,T", [(37, 29, 8, 40), (1, 1, 8, 20), (257, 3, 16, 100),
                                     (130, 66, 16, 500), (64, 200, 8, 1000)])
def test_ragged_screens(W, H, B, T):
    _note(f"two-level ragged {W}x{H} B={B} T={T}")
    sc = scenes.tiny(seed=W * 31 + H, width=W, height=H, num_tris=T)
    compare(gpu_render(sc, bin_size=B), oracle.render(sc))


@pytest.mark.parametrize("B", [8, 16])
def test_bin_lists_follow_the_rule(B):
    sc = scenes.tiny(seed=5, width=120, height=90, num_tris=400)
    g = gpu_render(sc, bin_size=B)
    off, pairs = g["renderer"].bin_lists()
    want = expected_lists(sc, B)
    nbins = len(off) - 1
    nbx, nby = -(-120 // B), -(-90 // B)
    assert nbins == nbx * nby + (-(-120 // (4 * B))) * (-(-90 // (4 * B)))
    coarse = 0
    for b in range(nbins):
        got = sorted(int(x) for x in pairs[off[b]:off[b + 1]])
        assert got == sorted(want.get(b, [])), b
        if b >= nbx * nby:
            coarse += len(got)
    assert coarse > 0                       # some triangles are large here
    compare(g, oracle.render(sc))


def test_same_image_as_one_level_and_modes():
    """Two levels regroup the work only: bit-identical to one level, with
    the shading deferred or not, over batched scenes, a perspective grid
    and deferred micropolygons."""
    for sc in (scenes.tiny(seed=77, width=150, height=110, num_tris=600),
               scenes.batch(num_scenes=5, size=64, tmin=50, tmax=3000),
               scenes.grid(seed=3, width=200, height=120, nx=64, ny=32),
               scenes.micro(seed=11, width=256, height=128, num_tris=30000, num_lights=3)):
        ref = gpu_render(sc, two_level=False, bin_size=8)
        compare(ref, oracle.render(sc))
        for B in (8, 16):
            for sched in ("load_balance", "direct_map"):
                for defer in (False, True):
                    _note(f"two-level {sc.name} B={B} {sched} defer={defer}")
                    g = gpu_render(sc, bin_size=B, schedule=sched, defer_shade=defer)
                    for k in ("color", "depth", "primid", "bary"):
                        assert (g[k] == ref[k]).all(), (sc.name, B, sched, defer, k)
                    assert int(g["frag_count"][0]) == int(ref["frag_count"][0])


def test_capacity_overflow_then_retry():
    import torch
    sc = scenes.tiny(seed=8, width=128, height=128, num_tris=500)
    r = pk.Renderer(sc, pk.RenderConfig(bin_size=8, two_level=True))
    r._alloc_ws(10)
    r.frame()
    torch.cuda.synchronize()
    assert int(r.pairs_needed.item()) > 10
    assert (r.out_primid.cpu().numpy() == -1).all()
    assert r.ensure_capacity()
    r.frame()
    assert not r.ensure_capacity()
    np.testing.assert_array_equal(r.out_primid.cpu().numpy(), oracle.render(sc)["primid"])


def test_unsupported_combinations_are_refused():
    sc = scenes.tiny(seed=2)
    for cfg in (dict(bin_size=32), dict(bin_size=0), dict(bin_size=8, schedule="dynamic"),
                dict(bin_size=8, schedule="split"), dict(bin_size=8, fuse_resolve=True)):
        with pytest.raises(pk.PkError):
            pk.Renderer(sc, pk.RenderConfig(two_level=True, **cfg)).render()

"""Pins of the order-independent-transparency oracle (orc_render_oit).

The compositing rule is this project's reading of the paper's EndBin example
(Depth Test, EndBin, Composite): every pixel's K nearest fragments, by the
same (depth, triangle) keys as the opaque depth test, composited nearest
first with interpolated per-vertex opacity:
    T = 1, C = 0; per fragment: w = T * a; C += w * c; T = T * (1 - a).
Pinned against (1) the opaque oracle when every opacity is 1, (2) a single
layer, which is the opaque colour times its opacity, and (3) an independent
composition: each triangle rendered alone by the opaque oracle, the
fragments of every pixel sorted and composited here in float32.
"""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from paper_1404_6293_amd import scenes

f32 = np.float32


def _alpha_of(bary, a, vid):
    """Interpolated opacity with the oracle's operation order."""
    b1, b2 = f32(bary[0]), f32(bary[1])
    b0 = (f32(1.0) - b1) - b2
    t = b0 * a[vid[0]]
    t = t + b1 * a[vid[1]]
    t = t + b2 * a[vid[2]]
    return f32(t)


def test_unit_opacity_is_the_opaque_image():
    sc = scenes.tiny(seed=3, width=48, height=40, num_tris=60)
    V = sc.pos.shape[1]
    o = oracle.render(sc)
    for K in (1, 3, 8):
        r = oracle.render_oit(sc, np.ones(V, np.float32), K)
        np.testing.assert_array_equal(r["primid"], o["primid"])
        np.testing.assert_array_equal(r["depth"], o["depth"])
        np.testing.assert_array_equal(r["bary"], o["bary"])
        # the interpolated opacity is 1 up to rounding, so later layers add
        # at most a few ulp
        np.testing.assert_allclose(r["color"], o["color"], rtol=1e-6, atol=1e-7)


def test_one_layer_is_opacity_times_colour():
    sc = scenes.tiny(seed=4, width=40, height=32, num_tris=50)
    V = sc.pos.shape[1]
    a = np.random.default_rng(1).uniform(0.0, 1.0, V).astype(np.float32)
    o = oracle.render(sc)
    r = oracle.render_oit(sc, a, 1)
    H, W = sc.height, sc.width
    for y in range(H):
        for x in range(W):
            t = int(o["primid"][0, y, x])
            if t < 0:
                assert (r["color"][0, y, x] == 0).all()
                continue
            al = _alpha_of(o["bary"][0, y, x], a, [3 * t, 3 * t + 1, 3 * t + 2])
            want = [f32(0.0) + (f32(1.0) * al) * o["color"][0, y, x, c] for c in range(3)]
            assert list(r["color"][0, y, x, :3]) == want
            assert r["color"][0, y, x, 3] == f32(1.0) - f32(1.0) * (f32(1.0) - al)


@pytest.mark.parametrize("K", [1, 2, 4, 16])
def test_independent_composition(K):
    """Every triangle rendered alone (opaque oracle), then per pixel: sort the
    fragments by (depth bits, triangle), keep K, composite in float32."""
    sc = scenes.tiny(seed=9, width=24, height=20, num_tris=40)
    V = sc.pos.shape[1]
    a = np.random.default_rng(2).uniform(0.05, 0.95, V).astype(np.float32)
    H, W, T = sc.height, sc.width, sc.num_tris
    frags = [[[] for _ in range(W)] for _ in range(H)]
    for t in range(T):
        one = SimpleNamespace(**{**vars(sc), "pos": sc.pos[:, 3 * t:3 * t + 3].copy(),
                                 "color": sc.color[:, 3 * t:3 * t + 3].copy(), "num_tris": 1})
        o = oracle.render(one)
        for y, x in zip(*np.nonzero(o["primid"][0] >= 0)):
            d = o["depth"][0, y, x]
            key = (int(d.view(np.uint32)), t)
            al = _alpha_of(o["bary"][0, y, x], a[3 * t:3 * t + 3], [0, 1, 2])
            frags[y][x].append((key, al, o["color"][0, y, x, :3].copy(), d, o["bary"][0, y, x]))
    r = oracle.render_oit(sc, a, K)
    for y in range(H):
        for x in range(W):
            fl = sorted(frags[y][x], key=lambda f: f[0])[:K]
            C = [f32(0.0)] * 3
            Tr = f32(1.0)
            for (_, al, c, _, _) in fl:
                w = Tr * al
                C = [C[i] + w * c[i] for i in range(3)]
                Tr = Tr * (f32(1.0) - al)
            assert list(r["color"][0, y, x, :3]) == C, (y, x)
            if fl:
                assert r["color"][0, y, x, 3] == f32(1.0) - Tr
                assert r["primid"][0, y, x] == fl[0][0][1]
                assert r["depth"][0, y, x] == fl[0][3]
                assert (r["bary"][0, y, x] == fl[0][4]).all()
            else:
                assert r["color"][0, y, x, 3] == 0 and r["primid"][0, y, x] == -1

"""GPU parity of the Reyes front end (include/pk_reyes.h) against the CPU
oracle, through the C ABI.  Split and Dice follow a fixed operation order in
float32, so the bar is bit-exactness: the same leaves (all 48 control
values), in the same order, with the same source patches; the same diced
positions, colours, normals and triangles.  The drawn frame meets the
rasterizer's bar: primitive IDs and depth bit for bit, colours within
1e-5 relative + 1e-6 absolute."""
import sys
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
import reyes_pins
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


def gpu_split(ps, **kw):
    import torch
    r = pk.Reyes(ps, **kw)
    r.split()
    nl = r.leaves()
    torch.cuda.synchronize()
    return r, r.leaf_cp[:nl].cpu().numpy(), r.leaf_src[:nl].cpu().numpy()


def check_split(ps, **kw):
    r, lv, src = gpu_split(ps, **kw)
    olv, osrc = oracle.reyes_split(ps.patches, ps.mvp, ps.width, ps.height, ps.dice_px,
                                   ps.max_depth)
    assert lv.shape == olv.shape, (lv.shape, olv.shape)
    np.testing.assert_array_equal(src, osrc)
    assert (lv.view(np.uint32) == olv.view(np.uint32)).all(), "leaves expected bit-exact"
    return r, olv, osrc


def check_dice(r, olv, osrc, ps):
    import torch
    r.dice(len(olv))
    torch.cuda.synchronize()
    pos, col, nrm, idx = oracle.reyes_dice(olv, osrc, ps.patch_color, ps.dice_n)
    for g, o, name in ((r.pos, pos, "pos"), (r.color, col, "color"), (r.normal, nrm, "normal")):
        assert (g.cpu().numpy().view(np.uint32) == o.view(np.uint32)).all(), name
    np.testing.assert_array_equal(r.idx.cpu().numpy(), idx)


def small(**kw):
    d = dict(pa=8, pb=4, width=320, height=180, dice_px=8.0, dice_n=4)
    d.update(kw)
    return scenes.patches(**d)


@pytest.mark.parametrize("seed", range(6))
def test_split_and_dice_small_sheets(seed):
    ps = small(seed=seed, tilt_deg=-40.0 - 5 * seed, noise=0.01 * (seed + 1),
               dice_n=(1, 2, 4, 5, 8, 16)[seed])
    _note(f"reyes small sheet seed={seed} n={ps.dice_n}")
    r, olv, osrc = check_split(ps)
    assert len(olv) > ps.num_patches
    check_dice(r, olv, osrc, ps)


@pytest.mark.parametrize("W,H,D", [(1, 1, 4.0), (37, 29, 3.0), (257, 3, 8.0), (64, 200, 2.5)])
def test_ragged_screens(W, H, D):
    _note(f"reyes ragged {W}x{H} D={D}")
    ps = small(seed=W + H, width=W, height=H, dice_px=D, max_depth=14)
    r, olv, osrc = check_split(ps)
    check_dice(r, olv, osrc, ps)


def test_depth_cap_and_depth_zero():
    for depth in (0, 1, 3):
        _note(f"reyes max_depth={depth}")
        ps = dataclass_replace(small(seed=9), max_depth=depth)
        r, olv, osrc = check_split(ps)
        check_dice(r, olv, osrc, ps)


def dataclass_replace(ps, **kw):
    d = dict(vars(ps))
    d.update(kw)
    return SimpleNamespace(**d)


def test_pin_configurations():
    """The pins' hand-built cases (exact leaf counts, off-screen culling,
    breadth-first order, w <= 0 and NaN patches) through the GPU."""
    sq = reyes_pins.square
    cases = [
        (np.stack([sq(-0.5, -0.5, 1.0)]), None, 256, 256, 8.0, 20, 256),
        (np.stack([sq(-0.5, -0.5, 1.0)]), None, 256, 256, 8.0, 3, 8),
        (np.stack([sq(-1.25, -1.25, 2.0)]), None, 64, 64, 4.0, 20, 225),
        (np.stack([sq(-1.375, -1.375, 2.0)]), None, 64, 64, 4.0, 20, 196),
        (np.stack([sq(-0.5, -0.5, 0.5), sq(0.5, 0.5, 0.125)]), None, 64, 64, 8.0, 20, 5),
    ]
    nan = sq(0.0, 0.0, 0.4)
    nan[5, 1] = np.nan
    mvp = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, -0.1], [0, 0, 1, 0]], np.float32)
    behind = reyes_pins.net(lambda u, v: (0.1 * u, 0.1 * v, 1.0 - 1.2 * u * v))
    front = reyes_pins.net(lambda u, v: (0.01 * u, 0.01 * v, 1.0))
    cases.append((np.stack([nan, sq(2.0, 2.0, 0.3), sq(0.1, 0.1, 0.02)]), None, 256, 256, 8.0,
                  20, 1))
    cases.append((np.stack([behind, front, behind]), mvp.reshape(16), 256, 256, 8.0, 20, 1))
    for k, (P, m, W, H, D, depth, want) in enumerate(cases):
        _note(f"reyes pin case {k}")
        ps = SimpleNamespace(width=W, height=H, patches=P.astype(np.float32),
                             patch_color=np.ones((len(P), 3), np.float32), mvp=m, dice_px=D,
                             max_depth=depth, dice_n=3, lights=None)
        r, olv, osrc = check_split(ps)
        assert len(olv) == want
        check_dice(r, olv, osrc, ps)


def test_largest_screen():
    """8192 x 8192, the largest screen: leaves and diced meshes bit-exact."""
    ps = small(seed=13, width=8192, height=8192, dice_px=64.0, dice_n=4)
    _note("reyes 8192x8192")
    r, olv, osrc = check_split(ps)
    assert len(olv) > 1000
    check_dice(r, olv, osrc, ps)


def test_empty_input_and_all_culled():
    import torch
    ps = SimpleNamespace(width=64, height=64, patches=np.zeros((0, 16, 3), np.float32),
                         patch_color=np.zeros((0, 3), np.float32), mvp=None, dice_px=8.0,
                         max_depth=5, dice_n=4, lights=None)
    r, lv, src = gpu_split(ps)
    assert len(lv) == 0 and r.read_counts() == (0, 0, 0, 0, 0, 0)
    ps.patches = np.stack([reyes_pins.square(2.0, 2.0, 0.5)] * 3)
    ps.patch_color = np.ones((3, 3), np.float32)
    r, lv, src = gpu_split(ps)
    assert len(lv) == 0 and r.read_counts() == (0, 0, 3, 0, 0, 1)
    r.dice(0)
    torch.cuda.synchronize()


def test_queue_and_leaf_overflow_then_retry():
    """A queue of 16 patches and a leaf list of 8: the counts report the
    overflow, the binding grows both and splits again to the same leaves."""
    ps = small(seed=4)
    r = pk.Reyes(ps, queue_capacity=16, leaf_capacity=8)
    r.split()
    nl, need, visits, overflow = r.read_counts()[:4]
    assert overflow == 1 and need > 16
    check_split(ps, queue_capacity=16, leaf_capacity=8)
    r2 = pk.Reyes(ps, queue_capacity=1 << 16, leaf_capacity=8)
    r2.split()
    nl, need, visits, overflow = r2.read_counts()[:4]
    olv, _ = oracle.reyes_split(ps.patches, ps.mvp, ps.width, ps.height, ps.dice_px,
                                ps.max_depth)
    assert overflow == 0 and nl == len(olv) > 8          # counted beyond the leaf list
    assert r2.leaves() == len(olv) and r2.leaf_capacity >= len(olv)


def test_counts_visits_and_largest_queue():
    """The counts: the largest queue of rounds >= 1, the patches visited and
    the rounds with work, from a breadth-first walk of the oracle's
    decisions; nothing left queued at the end."""
    ps = small(seed=2)
    r, _, _ = gpu_split(ps)
    q = [p for p in ps.patches]
    visits, largest, worked = 0, 0, 0
    for depth in range(ps.max_depth + 1):
        visits += len(q)
        worked += 1 if q else 0
        nxt = []
        for cp in q:
            d = oracle.reyes_decide(cp, ps.mvp, ps.width, ps.height, ps.dice_px,
                                    depth == ps.max_depth)
            if d >= 2:
                nxt.extend(oracle.reyes_halve(cp, d - 2))
        q = nxt
        largest = max(largest, len(q))
    _, need, got_visits, overflow, pending, got_worked = r.read_counts()
    assert (need, got_visits, overflow, pending, got_worked) == (largest, visits, 0, 0, worked)
    assert r._rounds_hint == worked


@pytest.mark.parametrize("rounds", [1, 2, 5])
def test_split_in_batches_of_rounds(rounds):
    """Enqueueing the first rounds only, then the rest when the counts say
    the queue has not drained, gives the same leaves as one call; so does a
    later frame that enqueues just the rounds the last one needed."""
    ps = small(seed=6)
    _note(f"reyes rounds in batches: first {rounds}")
    olv, osrc = oracle.reyes_split(ps.patches, ps.mvp, ps.width, ps.height, ps.dice_px,
                                   ps.max_depth)
    r = pk.Reyes(ps, queue_capacity=1 << 16)
    for it in range(2):
        r.split(rounds)
        # the first rounds alone do not drain the sheet; the hint does
        assert (r.read_counts()[4] > 0) == (it == 0)
        nl = r.leaves()
        assert nl == len(olv)
        np.testing.assert_array_equal(r.leaf_src[:nl].cpu().numpy(), osrc)
        assert (r.leaf_cp[:nl].cpu().numpy().view(np.uint32) == olv.view(np.uint32)).all()
        rounds = None                           # next: the hint from the counts
    assert r.read_counts()[4] == 0


@pytest.mark.parametrize("cfg", [dict(bin_size=16), dict(bin_size=32, fuse_resolve=True),
                                 dict(bin_size=0), dict(bin_size=16, defer_shade=True)])
def test_frame_matches_oracle(cfg):
    """Split, Dice, Sample and Shade: the drawn frame equals the oracle's
    drawing of the oracle's diced scene."""
    ps = scenes.patches(pa=12, pb=6, width=240, height=136, dice_px=6.0, dice_n=4, num_lights=3)
    _note(f"reyes frame {cfg}")
    r = pk.Reyes(ps, cfg=pk.RenderConfig(count_frags=True, **cfg))
    g = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.render().items()}
    o = oracle.render(oracle.reyes_scene(ps))
    np.testing.assert_array_equal(g["primid"], o["primid"])
    assert (g["depth"] == o["depth"]).all()
    np.testing.assert_allclose(g["color"], o["color"], rtol=RTOL, atol=ATOL)
    np.testing.assert_allclose(g["bary"], o["bary"], rtol=RTOL, atol=ATOL)
    assert int(g["frag_count"][0]) == int(o["frag_count"].sum())
    assert (g["primid"] >= 0).mean() > 0.3


def test_full_size_sheet():
    """The benchmark's patch sheet (2048 patches at 1920x1080, dice 16 px,
    8 x 8 grids): every leaf and its source bit-exact, Dice bit-exact on a
    sample of leaves, and the whole frame against the oracle."""
    import torch
    ps = scenes.patches()
    _note("reyes full-size sheet")
    r, olv, osrc = check_split(ps)
    r.dice(len(olv))
    torch.cuda.synchronize()
    n = ps.dice_n
    m, per = (n + 1) ** 2, 2 * n * n
    V = len(olv) * m
    rng = np.random.default_rng(0)
    pick = np.sort(rng.choice(len(olv), 64, replace=False))
    pos, col, nrm, idx = oracle.reyes_dice(olv[pick], osrc[pick], ps.patch_color, n)
    gp, gc, gn = (t.cpu().numpy() for t in (r.pos, r.color, r.normal))
    gi = r.idx.cpu().numpy()
    assert gp.shape == (3, V) and gi.shape == (per * len(olv), 3)
    for k, l in enumerate(pick):
        vs = slice(l * m, (l + 1) * m)
        ov = slice(k * m, (k + 1) * m)
        for g, o in ((gp, pos), (gc, col), (gn, nrm)):
            assert (g[:, vs].view(np.uint32) == o[:, ov].view(np.uint32)).all(), l
        np.testing.assert_array_equal(gi[l * per:(l + 1) * per] - l * m, idx[k * per:(k + 1) * per] - k * m)
    out = r.sample_shade().render()
    torch.cuda.synchronize()
    sc = oracle.reyes_scene(ps)
    o = oracle.render(sc)
    np.testing.assert_array_equal(out["primid"].cpu().numpy(), o["primid"])
    np.testing.assert_allclose(out["color"].cpu().numpy(), o["color"], rtol=RTOL, atol=ATOL)

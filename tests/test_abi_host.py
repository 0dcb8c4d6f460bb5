"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/pk.h and include/pk_reyes.h declare, validates arguments before it enqueues
anything, and computes the workspace size and status strings on the host."""
import ctypes as C
import os
import re

import pytest

from paper_1404_6293_amd import pk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the headers of libpk (include/pk_probe.h belongs to the probe library)
HEADERS = [os.path.join(ROOT, "include", h) for h in ("pk.h", "pk_reyes.h")]


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(pk.LIB_PATH):
        from paper_1404_6293_amd import build
        build.build()
    return pk.lib()


def declared_functions():
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(pk_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_abi():
    names = declared_functions()
    for n in ("pk_setup", "pk_assign_bin", "pk_raster_shade", "pk_shade", "pk_backward",
              "pk_workspace_bytes", "pk_status_string", "pk_bin_lists"):
        assert n in names
    assert set(names) == set(pk.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    for n in declared_functions():
        assert hasattr(L, n), n


def _params(**kw):
    d = dict(width=64, height=64, bin_size=8, schedule=0, threads_per_bin=0, shading=0, flags=0,
             num_scenes=1, instanced=0, persistent_groups=0)
    d.update(kw)
    return pk.Params(**d)


FAKE = 0x1000  # never dereferenced: every call below fails validation first


def _mesh(**kw):
    d = dict(pos=FAKE, num_vertices=3, indices=None, num_tris=1, mvp=None, scene_tri_off=None,
             scene_vtx_off=None)
    d.update(kw)
    return pk.Mesh(**d)


@pytest.mark.parametrize("bad", [
    dict(width=0), dict(height=-1), dict(width=8193), dict(bin_size=12), dict(bin_size=128),
    dict(bin_size=-8), dict(schedule=5), dict(schedule=-1), dict(threads_per_bin=32),
    dict(split_size=-1), dict(schedule=3, flags=2), dict(layers=-1), dict(layers=9),
    dict(layers=2, flags=2),
    dict(threads_per_bin=512), dict(shading=4), dict(flags=16), dict(flags=6), dict(num_scenes=0),
    dict(instanced=2), dict(persistent_groups=-1)])
def test_invalid_params_rejected_on_host(L, bad):
    p = _params(**bad)
    assert L.pk_setup(C.byref(p), C.byref(_mesh()), FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert L.pk_assign_bin(C.byref(p), C.byref(_mesh()), FAKE, 16, FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert L.pk_workspace_bytes(C.byref(p), C.byref(_mesh()), 100) == 0


def test_whole_screen_bins(L):
    """bin_size 0: one bin per scene, no lists (their view is refused), the
    rest of the validation unchanged."""
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    T = 1000
    m = _mesh(num_tris=T, num_vertices=3 * T)
    for S in (1, 3):
        p = _params(width=100, height=70, bin_size=0, num_scenes=S, instanced=int(S > 1))
        nb = S
        want = (al(32 * S * T) + al(16 * S * T) + al(8 * S * T) + al(4 * nb) + al(4 * 4672)
                + al(4 * (nb + 1)) + al(4 * nb) + al(8 * S * 100 * 70))
        assert L.pk_workspace_bytes(C.byref(p), C.byref(m), 0) == want
        v = pk.BinView()
        assert L.pk_bin_lists(C.byref(p), C.byref(m), 1 << 20, C.byref(v)) == pk.PK_ERR_UNSUPPORTED
    for bad in (dict(schedule=5), dict(threads_per_bin=32), dict(width=0)):
        p = _params(bin_size=0, **bad)
        assert L.pk_setup(C.byref(p), C.byref(_mesh()), FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT


def test_null_and_inconsistent_pointers_rejected(L):
    p = _params()
    assert L.pk_setup(None, C.byref(_mesh()), FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert L.pk_setup(C.byref(p), None, FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert L.pk_setup(C.byref(p), C.byref(_mesh()), None, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert L.pk_setup(C.byref(p), C.byref(_mesh(pos=None)), FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert L.pk_setup(C.byref(p), C.byref(_mesh(num_tris=-1)), FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    # concatenated batches need the scene offsets
    pb = _params(num_scenes=4)
    assert L.pk_setup(C.byref(pb), C.byref(_mesh()), FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    # pair capacity bounds
    assert L.pk_assign_bin(C.byref(p), C.byref(_mesh()), FAKE, -1, FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert L.pk_assign_bin(C.byref(p), C.byref(_mesh()), FAKE, 1 << 31, FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    # raster/shade requirements
    a = pk.Attribs(color=None)
    t = pk.Targets()
    assert L.pk_raster_shade(C.byref(p), C.byref(_mesh()), C.byref(a), FAKE, C.byref(t), None) == pk.PK_ERR_INVALID_ARGUMENT
    a = pk.Attribs(color=FAKE)
    pt = _params(shading=1)
    assert L.pk_raster_shade(C.byref(pt), C.byref(_mesh()), C.byref(a), FAKE, C.byref(t), None) == pk.PK_ERR_INVALID_ARGUMENT
    pd = _params(shading=2)
    assert L.pk_raster_shade(C.byref(pd), C.byref(_mesh()), C.byref(a), FAKE, C.byref(t), None) == pk.PK_ERR_INVALID_ARGUMENT
    pf = _params(flags=1)
    assert L.pk_raster_shade(C.byref(pf), C.byref(_mesh()), C.byref(a), FAKE, C.byref(t), None) == pk.PK_ERR_INVALID_ARGUMENT
    # the deferred shading pass needs the flag and the same attribute checks
    assert L.pk_shade(C.byref(p), C.byref(_mesh()), C.byref(pk.Attribs(color=FAKE)), FAKE,
                      C.byref(t), None) == pk.PK_ERR_INVALID_ARGUMENT
    pdef = _params(flags=pk.PK_FLAG_DEFER_SHADE)
    assert L.pk_shade(C.byref(pdef), C.byref(_mesh()), None, FAKE, C.byref(t),
                      None) == pk.PK_ERR_INVALID_ARGUMENT
    assert L.pk_shade(C.byref(pdef), C.byref(_mesh()), C.byref(pk.Attribs(color=None)), FAKE,
                      C.byref(t), None) == pk.PK_ERR_INVALID_ARGUMENT
    assert L.pk_shade(C.byref(pdef), C.byref(_mesh()), C.byref(pk.Attribs(color=FAKE)), None,
                      C.byref(t), None) == pk.PK_ERR_INVALID_ARGUMENT
    pdt = _params(flags=pk.PK_FLAG_DEFER_SHADE, shading=1)
    assert L.pk_shade(C.byref(pdt), C.byref(_mesh()), C.byref(pk.Attribs(color=FAKE)), FAKE,
                      C.byref(t), None) == pk.PK_ERR_INVALID_ARGUMENT
    # backward
    assert L.pk_backward(C.byref(p), C.byref(_mesh()), C.byref(a), None, FAKE, FAKE, FAKE, None, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert L.pk_backward(C.byref(pd), C.byref(_mesh()), C.byref(a), FAKE, FAKE, FAKE, FAKE, None, None) == pk.PK_ERR_UNSUPPORTED
    assert L.pk_backward(C.byref(pt), C.byref(_mesh()), C.byref(a), FAKE, FAKE, FAKE, FAKE, None, None) == pk.PK_ERR_INVALID_ARGUMENT


def test_workspace_bytes_arithmetic(L):
    p = _params(width=100, height=70, bin_size=16)
    T = 1000
    m = _mesh(num_tris=T, num_vertices=3 * T)
    b0 = L.pk_workspace_bytes(C.byref(p), C.byref(m), 0)
    b1 = L.pk_workspace_bytes(C.byref(p), C.byref(m), 64)
    b2 = L.pk_workspace_bytes(C.byref(p), C.byref(m), 64 + 1)
    assert b0 > 0 and b1 - b0 == 256 and b2 - b1 == 256
    nbins = 7 * 5
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    # 32-byte setup records, 16 bytes of 1/w per triangle (unindexed only),
    # 8-byte bboxes, counts, misc words, offsets, cursors, keys
    common = (al(8 * T) + al(4 * nbins) + al(4 * 4672) + al(4 * (nbins + 1)) + al(4 * nbins)
              + al(8 * 100 * 70))
    assert b0 == al(32 * T) + al(16 * T) + common
    # an indexed mesh has one 16-byte snapped record per vertex (per view)
    # instead of the per-triangle 1/w slice
    mi = _mesh(num_tris=T, num_vertices=600, indices=FAKE)
    assert L.pk_workspace_bytes(C.byref(p), C.byref(mi), 0) == al(16 * 600) + al(32 * T) + common
    # instanced views multiply the per-triangle and per-vertex slices
    pi = _params(width=100, height=70, bin_size=16, num_scenes=3, instanced=1)
    nb3 = 3 * nbins
    common3 = (al(8 * 3 * T) + al(4 * nb3) + al(4 * 4672) + al(4 * (nb3 + 1)) + al(4 * nb3)
               + al(8 * 3 * 100 * 70))
    assert L.pk_workspace_bytes(C.byref(pi), C.byref(m), 0) == al(32 * 3 * T) + al(16 * 3 * T) + common3
    assert L.pk_workspace_bytes(C.byref(pi), C.byref(mi), 0) == (al(16 * 3 * 600) + al(32 * 3 * T)
                                                                 + common3)
    assert L.pk_workspace_bytes(C.byref(p), C.byref(_mesh(num_tris=-1)), 0) == 0
    assert L.pk_workspace_bytes(C.byref(p), C.byref(m), -5) == 0
    assert L.pk_workspace_bytes(C.byref(p), None, 0) == 0


def test_split_schedule_workspace(L):
    """PK_SCHED_SPLIT adds one work-item number per bin (+1) to the
    workspace and PK_SCHED_DYNAMIC one bin number per bin; other schedules
    and whole-screen bins add nothing."""
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    m = _mesh(num_tris=1000, num_vertices=3000)
    base = L.pk_workspace_bytes(C.byref(_params(width=100, height=70, bin_size=16, schedule=1)),
                                C.byref(m), 0)
    for sp in (0, 1, 500):
        p = _params(width=100, height=70, bin_size=16, schedule=3, split_size=sp)
        assert L.pk_workspace_bytes(C.byref(p), C.byref(m), 0) == base + al(4 * 36)
    p0 = _params(width=100, height=70, bin_size=0, schedule=3)
    assert L.pk_workspace_bytes(C.byref(p0), C.byref(m), 0) == L.pk_workspace_bytes(
        C.byref(_params(width=100, height=70, bin_size=0)), C.byref(m), 0)
    # DYNAMIC keeps each die's bins in heaviest-first order: one word per bin
    pd = _params(width=100, height=70, bin_size=16, schedule=2)
    assert L.pk_workspace_bytes(C.byref(pd), C.byref(m), 0) == base + al(4 * 35)


@pytest.mark.parametrize("kw", [dict(shading=1), dict(shading=2), dict(bin_size=0), dict(bin_size=64),
                                dict(schedule=3)])
def test_transparency_layers_unsupported_combinations(L, kw):
    p = _params(**{"layers": 2, **kw})
    assert L.pk_setup(C.byref(p), C.byref(_mesh()), FAKE, None) == pk.PK_ERR_UNSUPPORTED


def test_transparency_layers_workspace_and_alpha(L):
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    m = _mesh(num_tris=1000, num_vertices=3000)
    b0 = L.pk_workspace_bytes(C.byref(_params(width=100, height=70, bin_size=16)), C.byref(m), 0)
    for K in (1, 3, 8):
        p = _params(width=100, height=70, bin_size=16, layers=K)
        assert L.pk_workspace_bytes(C.byref(p), C.byref(m), 0) == b0 + al(8 * 7000 * K) - al(8 * 7000)
    # the opacity plane is required, and there is no backward
    p = _params(layers=2)
    t = pk.Targets(FAKE, FAKE, FAKE, None, None, None, None)
    assert L.pk_raster_shade(C.byref(p), C.byref(_mesh()), C.byref(pk.Attribs(color=FAKE)), FAKE,
                             C.byref(t), None) == pk.PK_ERR_INVALID_ARGUMENT
    assert L.pk_backward(C.byref(p), C.byref(_mesh()), C.byref(pk.Attribs(color=FAKE, alpha=FAKE)),
                         FAKE, FAKE, FAKE, FAKE, None, None) == pk.PK_ERR_UNSUPPORTED


def test_bin_lists_view_points_into_workspace(L):
    p = _params(width=100, height=70, bin_size=16)
    m = _mesh(num_tris=1000, num_vertices=3000)
    v = pk.BinView()
    base = 1 << 20
    assert L.pk_bin_lists(C.byref(p), C.byref(m), base, C.byref(v)) == pk.PK_OK
    assert v.num_bins == 35
    size = L.pk_workspace_bytes(C.byref(p), C.byref(m), 0)
    assert base < v.bin_offsets < v.bin_tris == base + size
    assert L.pk_bin_lists(C.byref(p), C.byref(m), None, C.byref(v)) == pk.PK_ERR_INVALID_ARGUMENT


def test_status_strings(L):
    for s in range(5):
        assert pk.status_string(s)
    assert pk.status_string(99) == "unknown status"
    assert pk.status_string(pk.PK_ERR_INVALID_ARGUMENT) == "invalid argument"


def test_static_workspace_rejects_frames_that_do_not_fit(L):
    """pk_render_static checks on the host, before anything is enqueued, that
    every workspace slice but the pair list fits its static workspace."""
    at = pk.Attribs(FAKE, None, None, None, 0, 0, None, 0, None)
    tg = pk.Targets(FAKE, FAKE, FAKE, None, None, None, None)
    # 8192 x 8192 keys alone take 512 MiB
    p = _params(width=8192, height=8192, bin_size=0)
    assert L.pk_workspace_bytes(C.byref(p), C.byref(_mesh()), 0) > pk.PK_STATIC_WORKSPACE_BYTES
    assert L.pk_render_static(C.byref(p), C.byref(_mesh()), C.byref(at), C.byref(tg), None,
                              None) == pk.PK_ERR_CAPACITY
    # invalid arguments are still invalid
    bad = _params(bin_size=12)
    assert L.pk_render_static(C.byref(bad), C.byref(_mesh()), C.byref(at), C.byref(tg), None,
                              None) == pk.PK_ERR_INVALID_ARGUMENT
    assert L.pk_render_static(C.byref(_params()), C.byref(_mesh()), None, C.byref(tg), None,
                              None) == pk.PK_ERR_INVALID_ARGUMENT
    assert "static workspace" in pk.status_string(pk.PK_ERR_CAPACITY)


def test_fragment_bins_restrictions_and_workspace(L):
    """PK_SCHED_FRAGMENT_BINS: one opaque scene, 16-64 px bins, at most 8192
    bins; its workspace holds no per-triangle records or keys, a count
    matrix (one row of bin counts per workgroup of 1024-triangle rounds) and
    the fragments (2 planes of 16 bytes, 3 for deferred shading, in blocks
    of 64)."""
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    m = _mesh(num_tris=1000, num_vertices=3000)
    for bad in (dict(bin_size=8), dict(bin_size=0), dict(num_scenes=2, instanced=1),
                dict(layers=2, bin_size=16), dict(width=8192, height=8192, bin_size=16)):
        p = _params(schedule=4, **{"bin_size": 16, **bad})
        assert L.pk_setup(C.byref(p), C.byref(m), FAKE, None) == pk.PK_ERR_UNSUPPORTED, bad
        assert L.pk_workspace_bytes(C.byref(p), C.byref(m), 100) == 0
    p = _params(width=100, height=70, bin_size=32, schedule=4)         # 4 x 3 bins
    nb = 12
    for shading, planes in ((0, 2), (2, 3)):
        p.shading = shading
        want = (al(4 * 1 * nb) + al(4 * nb) + al(4 * nb) + al(4 * 4672) + al(4 * (nb + 1))
                + al(16 * planes * 128))
        assert L.pk_workspace_bytes(C.byref(p), C.byref(m), 100) == want
    v = pk.BinView()
    assert L.pk_bin_lists(C.byref(p), C.byref(m), 1 << 20, C.byref(v)) == pk.PK_ERR_UNSUPPORTED


def test_two_level_bins_workspace_and_restrictions(L):
    """PK_FLAG_TWO_LEVEL_BINS: each scene's coarse bins (4x the size) follow
    its fine bins in the counts, cursors and offsets; 8- or 16-px bins,
    LOAD_BALANCE or DIRECT_MAP, opaque and not fused."""
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    m = _mesh(num_tris=1000, num_vertices=3000)
    one = L.pk_workspace_bytes(C.byref(_params(width=100, height=70, bin_size=8)), C.byref(m), 0)
    two = L.pk_workspace_bytes(C.byref(_params(width=100, height=70, bin_size=8, flags=8)),
                               C.byref(m), 0)
    nf, nc = 13 * 9, 4 * 3                  # fine 8-px bins, coarse 32-px bins
    assert two - one == ((al(4 * (nf + nc)) - al(4 * nf)) * 2
                         + al(4 * (nf + nc + 1)) - al(4 * (nf + 1)))
    for bad in (dict(bin_size=32), dict(bin_size=0), dict(schedule=2), dict(schedule=3),
                dict(flags=8 | 2), dict(layers=2)):
        p = _params(**{"flags": 8, **bad})
        p.flags |= 8
        assert L.pk_setup(C.byref(p), C.byref(m), FAKE, None) in (pk.PK_ERR_UNSUPPORTED,
                                                                   pk.PK_ERR_INVALID_ARGUMENT)


# ---------------------------------------------------------------------------
# Reyes front end (include/pk_reyes.h): host-side validation and sizes
# ---------------------------------------------------------------------------
def _rp(**kw):
    d = dict(width=64, height=48, dice_px=8.0, max_depth=10, dice_n=4)
    d.update(kw)
    return pk.ReyesParams(**d)


def test_reyes_workspace_bytes(L):
    f = L.pk_reyes_workspace_bytes
    base = f(C.byref(_rp()), 0, 0)
    assert base > 0 and base % 256 == 0
    # two queues of 192-byte patches and int32 sources, a decision byte per patch
    big = f(C.byref(_rp()), 1000, 1 << 16)
    assert big - base >= 2 * (1 << 16) * (192 + 4) + (1 << 16)
    # the decision bytes cover the input round too
    assert f(C.byref(_rp()), 1 << 20, 16) >= f(C.byref(_rp()), 0, 16) + (1 << 20) - 256
    for bad in (dict(width=0), dict(height=8193), dict(dice_px=0.0), dict(dice_px=float("nan")),
                dict(dice_px=float("inf")), dict(max_depth=-1), dict(max_depth=31),
                dict(dice_n=0), dict(dice_n=17)):
        assert f(C.byref(_rp(**bad)), 10, 10) == 0, bad
    assert f(C.byref(_rp()), -1, 10) == 0
    assert f(C.byref(_rp()), 10, pk.PK_REYES_MAX_QUEUE + 1) == 0
    assert f(None, 10, 10) == 0


def test_reyes_split_and_dice_validate_before_launch(L):
    ok = _rp()
    bad = _rp(dice_n=0)
    cnt = FAKE
    S = L.pk_reyes_split
    assert S(C.byref(bad), FAKE, 4, None, 0x10000, 64, FAKE, FAKE, 64, 0, 21, cnt, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert S(C.byref(ok), None, 4, None, 0x10000, 64, FAKE, FAKE, 64, 0, 21, cnt, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert S(C.byref(ok), FAKE, 4, None, None, 64, FAKE, FAKE, 64, 0, 21, cnt, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert S(C.byref(ok), FAKE, 4, None, 0x10010, 64, FAKE, FAKE, 64, 0, 21, cnt, None) == pk.PK_ERR_INVALID_ARGUMENT  # ws alignment
    assert S(C.byref(ok), FAKE + 4, 4, None, 0x10000, 64, FAKE, FAKE, 64, 0, 21, cnt, None) == pk.PK_ERR_INVALID_ARGUMENT  # patches alignment
    assert S(C.byref(ok), FAKE, 4, None, 0x10000, 64, None, FAKE, 64, 0, 21, cnt, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert S(C.byref(ok), FAKE, 4, None, 0x10000, 64, FAKE, FAKE, 64, 0, 21, None, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert S(C.byref(ok), FAKE, -1, None, 0x10000, 64, FAKE, FAKE, 64, 0, 21, cnt, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert S(C.byref(ok), FAKE, 4, None, 0x10000, -1, FAKE, FAKE, 64, 0, 21, cnt, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert S(C.byref(ok), FAKE, 4, None, 0x10000, 64, FAKE, FAKE, -1, 0, 21, cnt, None) == pk.PK_ERR_INVALID_ARGUMENT
    # rounds: 0 <= round_begin <= round_end
    assert S(C.byref(ok), FAKE, 4, None, 0x10000, 64, FAKE, FAKE, 64, -1, 21, cnt, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert S(C.byref(ok), FAKE, 4, None, 0x10000, 64, FAKE, FAKE, 64, 5, 4, cnt, None) == pk.PK_ERR_INVALID_ARGUMENT
    D = L.pk_reyes_dice
    assert D(C.byref(bad), FAKE, FAKE, 4, FAKE, 4, FAKE, FAKE, FAKE, FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert D(C.byref(ok), FAKE, FAKE, -1, FAKE, 4, FAKE, FAKE, FAKE, FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert D(C.byref(ok), None, FAKE, 4, FAKE, 4, FAKE, FAKE, FAKE, FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    assert D(C.byref(ok), FAKE, FAKE, 4, FAKE, 4, FAKE, None, FAKE, FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    # V = L (n+1)^2 must stay below 2^31 (mesh vertex numbers are int32)
    assert D(C.byref(_rp(dice_n=16)), FAKE, FAKE, (1 << 31) // 289 + 1, FAKE, 4, FAKE, FAKE,
             FAKE, FAKE, None) == pk.PK_ERR_INVALID_ARGUMENT
    # nothing to dice: nothing enqueued, OK
    assert D(C.byref(ok), None, None, 0, None, 0, None, None, None, None, None) == pk.PK_OK

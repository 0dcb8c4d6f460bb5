"""Host-side logic of bench.py: the JSON contract's refusals, the
algorithmic-byte formulas behind `roofline`, and the profile lookup that
feeds `roofline.traffic` (valid only for the code it was measured on)."""
import os
import shutil
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def _scene(W, H, V, T, S=1, idx=True, shading="gouraud", instanced=False, texture=None):
    import numpy as np
    return SimpleNamespace(width=W, height=H, num_scenes=S, idx=object() if idx else None,
                           shading=shading, pos=np.zeros((3, V), np.float32), num_tris=T,
                           instanced=instanced, texture=texture)


def test_algorithmic_bytes_formulas():
    # indexed Gouraud mesh, 16-px bins (7 x 5 bins on 100 x 70), no bary
    sc = _scene(100, 70, V=50, T=80)
    a = bench.algorithmic_bytes(sc, npairs=1000, covered=300, want_bary=False, B=16)
    assert a["setup"] == 12 * 50 + 12 * 80                # positions + indices
    assert a["assign_bin"] == 4 * 1000 + 4 * 36           # pairs written, CSR offsets
    assert a["raster"] == 4 * 1000 + 4 * 36 + 8 * 7000    # pairs read, depth + primid
    assert a["shade"] == 12 * 50 + 16 * 7000              # colour plane (less than
                                                          # 36 B x 300 gathers), RGBA
    assert a["frame"] == sum(a[k] for k in ("setup", "assign_bin", "raster", "shade"))
    a2 = bench.algorithmic_bytes(sc, 1000, 300, True, 16)
    assert a2["shade"] == a["shade"] + 8 * 7000           # saved barycentrics
    # independent deferred micropolygons, whole-screen bins: the visible
    # triangles' colours and normals (36 B each per covered pixel) are less
    # than the planes; G-buffer written and read back, colour written
    sd = _scene(100, 70, V=3000, T=1000, idx=False, shading="deferred")
    d = bench.algorithmic_bytes(sd, 0, 300, False, 0)
    # (whole-screen bins: the setup runs in the depth-test kernel, which
    # reads the positions)
    assert d["setup"] == 0
    assert d["assign_bin"] == 4 and d["raster"] == 12 * 3000 + 4 + 8 * 7000
    assert d["shade"] == 2 * 36 * 300 + 24 * 7000 * 2 + 16 * 7000
    # textured instanced views read the mesh once per view
    import numpy as np
    tv = _scene(32, 32, V=100, T=150, S=4, shading="textured", instanced=True,
                texture=np.zeros((8, 8, 3), np.float32))
    t = bench.algorithmic_bytes(tv, 500, 2000, True, 8)
    assert t["setup"] == 4 * (12 * 100 + 12 * 150)
    assert t["shade"] == (4 * 12 * 100 + 4 * 8 * 100 + 4 * 8 * 8 * 3 * 4
                          + (16 + 8) * 4 * 1024)
    # indexed mesh, whole-screen bins: the Vertex Shader still reads the
    # positions in the setup stage, the depth-test kernel the indices
    w = bench.algorithmic_bytes(sc, 0, 300, False, 0)
    assert w["setup"] == 12 * 50 and w["raster"] == 12 * 80 + 4 + 8 * 7000
    assert w["frame"] == a["frame"] - 8 * 1000 - 8 * 35


def test_grid1080_frame_bytes_match_the_workload_sizes():
    """The 1920x1080 grid (525,825 vertices, 1,048,576 triangles, 975,046
    pairs with 16-px bins, one fragment per pixel): pos 6.31 + RGB 6.31 +
    indices 12.58 + pairs 7.80 + outputs 49.77 MB."""
    sc = _scene(1920, 1080, V=525825, T=1048576)
    a = bench.algorithmic_bytes(sc, 975046, 2073600, False, 16)
    expect = 12 * 525825 * 2 + 12 * 1048576 + 8 * 975046 + 8 * 8161 + 24 * 2073600
    assert a["frame"] == expect
    assert abs(a["frame"] / 1e6 - 82.8) < 0.2
    assert a["raster"] == 4 * 975046 + 4 * 8161 + 8 * 2073600      # about 20.55 MB


@pytest.fixture
def tree(tmp_path, monkeypatch):
    """A copy of the sources the hash covers, with bench pointed at it."""
    (tmp_path / "paper_1404_6293_amd").mkdir()
    shutil.copytree(os.path.join(ROOT, "paper_1404_6293_amd", "csrc"),
                    tmp_path / "paper_1404_6293_amd" / "csrc")
    shutil.copytree(os.path.join(ROOT, "include"), tmp_path / "include")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def test_source_hash_ignores_comments_not_code(tree):
    h0 = bench.kernel_source_hash()
    assert h0 == bench.kernel_source_hash()
    f = tree / "paper_1404_6293_amd" / "csrc" / "k_setup.hip"
    text = f.read_text()
    f.write_text("// an added comment\n/* and a block\n comment */\n" + text.replace("\n", "\n\n", 3))
    assert bench.kernel_source_hash() == h0
    changed = text.replace("kItemsPerThread = ", "kItemsPerThread = 1 + ", 1)
    assert changed != text
    f.write_text(changed)
    assert bench.kernel_source_hash() != h0


def test_profiled_traffic_needs_the_measured_code(tree):
    h = bench.kernel_source_hash()
    p = tree / "profiles" / "grid1080_kernels.md"
    p.write_text("# summary\n```\n"
                 f"traffic k_raster 47616223 bytes/launch sources {h}\n"
                 f"traffic k_direct 123 bytes/launch sources {'0' * 64}\n```\n")
    assert bench.profiled_traffic("grid1080", "k_raster") == 47616223
    assert bench.profiled_traffic("grid1080", "k_direct") is None      # other code
    assert bench.profiled_traffic("micro8m", "k_raster") is None       # no summary

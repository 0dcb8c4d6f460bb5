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


def _scene(W, H, S=1, idx=True, shading="gouraud"):
    return SimpleNamespace(width=W, height=H, num_scenes=S, idx=object() if idx else None,
                           shading=shading)


def test_algorithmic_bytes_formulas():
    sc = _scene(100, 70)
    # 40 B per pair, two 4-byte offsets per bin (7 x 5 bins of 16 px), 8 B per pixel
    assert bench.bin_kernel_algorithmic_bytes(sc, 1000, 16) == 40 * 1000 + 8 * 35 + 8 * 7000
    assert bench.bin_kernel_algorithmic_bytes(sc, 0, 64) == 8 * 4 + 8 * 7000   # 2 x 2 bins
    # unbinned: 36 B per input triangle, 16 B of key per pixel
    assert bench.direct_kernel_algorithmic_bytes(_scene(100, 70, S=3), 500) == 36 * 500 + 16 * 21000
    # resolve: per pixel 4 B primitive ID + 16 B colour (+8 bary); per covered
    # pixel 12 B indices (indexed) + 36 B colours (+36 B normals, deferred)
    assert bench.shade_pass_algorithmic_bytes(sc, 300, False) == 20 * 7000 + 48 * 300
    assert bench.shade_pass_algorithmic_bytes(sc, 300, True) == 28 * 7000 + 48 * 300
    sd = _scene(100, 70, idx=False, shading="deferred")
    assert bench.shade_pass_algorithmic_bytes(sd, 300, False) == 28 * 7000 + 72 * 300


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
    f.write_text(text.replace("kItemsPerThread = 4", "kItemsPerThread = 2"))
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

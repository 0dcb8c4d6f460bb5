"""The oracle's Reyes front end (Split and Dice of bicubic Bezier patches,
Sec. 7.1) against its pins: the Bernstein definition of a patch, affine
patches' closed forms, exact leaf counts of axis-aligned squares, the split
decision's cases, the breadth-first leaf order and a diced scene drawn end to
end.  The pins themselves live in reyes_pins.py so that the mutation tests
can run them against planted mistakes."""
import numpy as np
import pytest

import oracle
import reyes_pins
from paper_1404_6293_amd import scenes


@pytest.mark.parametrize("name", sorted(reyes_pins.PINS))
def test_pin(name):
    assert reyes_pins.PINS[name](), name


def test_patch_scene_is_a_c0_sheet():
    """Neighbouring patches of the generator share their border control
    points, so the split surface has no cracks between input patches."""
    ps = scenes.patches(pa=4, pb=3, width=320, height=180)
    P = ps.patches.reshape(3, 4, 4, 4, 3)       # [pb][pa][i][j][3]
    assert (P[:, :-1, :, 3] == P[:, 1:, :, 0]).all()
    assert (P[:-1, :, 3, :] == P[1:, :, 0, :]).all()
    assert ps.patch_color.shape == (12, 3) and ps.mvp.shape == (16,)


def test_split_leaves_are_small_or_at_depth_cap():
    """Every leaf of a perspective patch scene passes the dice test, except
    when the depth cap forced it; sources are non-decreasing per round."""
    ps = scenes.patches(pa=8, pb=4, width=320, height=180, dice_px=8.0)
    leaves, src = oracle.reyes_split(ps.patches, ps.mvp, ps.width, ps.height, ps.dice_px,
                                     ps.max_depth)
    assert len(leaves) > 4 * ps.num_patches
    for lf in leaves[:: max(1, len(leaves) // 200)]:
        assert oracle.reyes_decide(lf, ps.mvp, ps.width, ps.height, ps.dice_px) == 1
    capped, _ = oracle.reyes_split(ps.patches, ps.mvp, ps.width, ps.height, ps.dice_px, 2)
    assert len(capped) <= 4 * ps.num_patches


def test_empty_and_all_culled():
    leaves, src = oracle.reyes_split(np.zeros((0, 16, 3), np.float32), None, 64, 64, 8.0, 10)
    assert leaves.shape == (0, 16, 3) and src.shape == (0,)
    off = reyes_pins.square(2.0, 2.0, 0.5)
    leaves, _ = oracle.reyes_split(off[None], None, 64, 64, 8.0, 10)
    assert len(leaves) == 0
    pos, col, nrm, idx = oracle.reyes_dice(leaves, np.zeros(0, np.int32),
                                           np.ones((1, 3), np.float32), 4)
    assert pos.shape == (3, 0) and idx.shape == (0, 3)

"""Model of the transparency slots' atomic-min cascade under concurrency.

With 8- and 16-px bins the bin kernel keeps each pixel's K nearest keys in K
LDS slots: an arriving key takes an atomic minimum with slot 0, and whatever
it displaced (the larger of the old value and the key) moves on to slot 1,
and so on; the last slot drops what it displaces, and a cascade stops early
when it meets an empty slot.  The kernel relies on slot j ending as the
(j+1)-th smallest key whatever the interleaving of the threads' atomic steps.
Here many simulated threads run their cascades one atomic step at a time in
random interleavings, and the final slots must equal the sorted K smallest
keys.  The skip that was measured and taken out (a plain read showing a slot
already below the key passes the key on without an atomic) is checked too:
it gives the same slots, because slot values only ever decrease.
"""
import random

import pytest

EMPTY = (1 << 64) - 1


def _run(keys, K, rng, skip_smaller=False):
    slots = [EMPTY] * K
    # per thread: (key in flight, next slot); None when finished
    state = [[k, 0] for k in keys]
    live = list(range(len(keys)))
    while live:
        i = rng.choice(live)
        key, j = state[i]
        if skip_smaller and slots[j] < key and j < K - 1:
            state[i][1] = j + 1                         # plain read: pass it on
            continue
        old = slots[j]                                  # one atomic min step
        slots[j] = min(old, key)
        if j == K - 1 or old == EMPTY:
            live.remove(i)
            continue
        state[i] = [max(old, key), j + 1]
    return slots


@pytest.mark.parametrize("skip_smaller", [False, True])
@pytest.mark.parametrize("K", [1, 2, 3, 5, 8])
def test_cascade_keeps_the_k_smallest_in_order(K, skip_smaller):
    rng = random.Random(1000 * K + skip_smaller)
    for trial in range(300):
        n = rng.randrange(0, 3 * K + 4)
        keys = rng.sample(range(1, 1 << 40), n)
        got = _run(keys, K, rng, skip_smaller)
        want = sorted(keys)[:K] + [EMPTY] * max(0, K - n)
        assert got == want, (trial, keys)


def test_cascade_needs_the_carry():
    """The planted mistake: dropping the displaced key instead of carrying it
    on loses keys, which the model detects."""
    rng = random.Random(5)
    K = 3
    keys = [50, 40, 30, 20, 10]
    slots = [EMPTY] * K
    for key in keys:                       # one thread at a time, no carry
        for j in range(K):
            if slots[j] == EMPTY or key < slots[j]:
                slots[j] = key
                break
    assert slots != sorted(keys)[:K]
    assert _run(keys, K, rng) == sorted(keys)[:K]

"""Two-level completion ticket of the step kernel, modelled on the host.

Every slot of a running system takes one ticket per launch: a ticket of its
group (slot index mod G, G = min(slots, 16)); the last arrival of a group
resets the group counter and takes a ticket of the top counter; the arrival
that completes the top counter finalizes and resets it.  Whatever the arrival
order, exactly one arrival finalizes, it is the last one, and every counter
is zero again at the end of the launch.  The last test shows why the count
has to be the phase-independent slot count: one extra arrival leaves an
offset that a later launch with single-slot groups never clears.
"""
import random

import pytest

GROUPS = 16


def group_of(tk, ntk):
    G = min(ntk, GROUPS)
    g = tk % G
    gsize = ntk // G + (1 if g < ntk % G else 0)
    return G, g, gsize


def run_launch(order, ntk, ctr):
    """Arrivals in the given order; ctr = [top, g0, g1, ...]. Returns the arrival positions that finalize."""
    fin = []
    for pos, tk in enumerate(order):
        G, g, gsize = group_of(tk, ntk)
        pg = ctr[1 + g]
        ctr[1 + g] += 1
        if pg == gsize - 1:
            ctr[1 + g] = 0
            pt = ctr[0]
            ctr[0] += 1
            if pt == G - 1:
                ctr[0] = 0
                fin.append(pos)
    return fin


@pytest.mark.parametrize("ntk", [1, 2, 7, 15, 16, 17, 31, 32, 33, 100, 2048])
def test_group_sizes_partition_the_slots(ntk):
    G = min(ntk, GROUPS)
    sizes = [group_of(g, ntk)[2] for g in range(G)]
    assert sum(sizes) == ntk and min(sizes) >= 1
    counts = [0] * G
    for tk in range(ntk):
        counts[group_of(tk, ntk)[1]] += 1
    assert counts == sizes


@pytest.mark.parametrize("ntk", [1, 3, 9, 16, 17, 25, 40, 257])
def test_one_finalize_at_the_last_arrival_and_counters_reset(ntk):
    rng = random.Random(ntk)
    ctr = [0] * (1 + GROUPS)
    for _ in range(20):
        order = list(range(ntk))
        rng.shuffle(order)
        assert run_launch(order, ntk, ctr) == [ntk - 1]
        assert ctr == [0] * (1 + GROUPS)


def test_an_extra_arrival_stalls_a_later_launch():
    """One stray arrival in a launch of 17 slots leaves an offset; a later launch of
    9 slots (single-slot groups) then never finalizes."""
    ctr = [0] * (1 + GROUPS)
    run_launch([0], 17, ctr)                       # the stray
    assert run_launch(list(range(17)), 17, ctr) != []
    assert ctr != [0] * (1 + GROUPS)
    assert run_launch(list(range(9)), 9, ctr) == []

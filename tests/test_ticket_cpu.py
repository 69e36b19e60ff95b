"""Two-level completion ticket of the step kernel, modelled on the host.

Every slot of a running system takes one ticket per launch: a ticket of its
group (slot index mod G, G = 16); the last arrival of a group resets the group
counter and takes a ticket of the top counter; the arrival that completes the
top counter finalizes and resets it.  A system of at most 16 slots takes
tickets of the top counter directly.  Whatever the arrival
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
    """Arrivals in the given order; ctr = [top, g0, g1, ...]. Returns the arrival positions that finalize.

    A system of at most GROUPS slots takes tickets of the top counter directly."""
    fin = []
    for pos, tk in enumerate(order):
        if ntk <= GROUPS:
            pt = ctr[0]
            ctr[0] += 1
            if pt == ntk - 1:
                ctr[0] = 0
                fin.append(pos)
            continue
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
    """One stray arrival in a launch of 17 slots leaves an offset in a group counter;
    the slots of a later launch then never complete that group and no launch
    finalizes.  With at most 16 slots a stray arrival shifts the single counter and
    the finalize comes one arrival early, before every slot has arrived."""
    ctr = [0] * (1 + GROUPS)
    run_launch([0], 17, ctr)                       # the stray
    assert run_launch(list(range(17)), 17, ctr) != []
    assert ctr != [0] * (1 + GROUPS)
    for _ in range(3):
        assert run_launch(list(range(17)), 17, ctr) != [16]
    ctr = [0] * (1 + GROUPS)
    run_launch([0], 9, ctr)                        # the stray
    assert run_launch(list(range(9)), 9, ctr) == [7]


def _launch_schedule(lim, rng):
    """Random start / arrival times of the lim slots of one launch (start before arrival)."""
    ev = []
    for sl in range(lim):
        a, b = sorted(rng.random() for _ in range(2))
        ev.append((a, "start", sl))
        ev.append((b, "arrive", sl))
    ev.sort()
    return ev


def _single_system_launch(ev, ntiles, phase0, lim, count_slots):
    """One launch of a single system whose two tilings have ntiles[phase] tiles.

    Each slot reads the phase when it starts.  count_slots=False: the rule before the
    fix, a slot with no tile of the phase it read leaves without a ticket and the
    ticket target is that phase's tile count.  count_slots=True: every slot takes a
    ticket and the target is the phase-independent slot count lim.  Returns (slots
    that read a phase other than phase0, number of finalizes, tickets taken toward a
    phase other than phase0)."""
    phase = phase0
    seen = {}
    count = 0
    finals = 0
    stray = 0
    for _, kind, sl in ev:
        if kind == "start":
            seen[sl] = phase
            continue
        ph = seen[sl]
        if not count_slots and sl >= ntiles[ph]:
            continue
        if ph != phase0:
            stray += 1
            continue
        count += 1
        target = lim if count_slots else ntiles[phase0]
        if count == target:
            finals += 1
            phase = 1 - phase0               # the finalize sets the next phase
    late = sum(1 for ph in seen.values() if ph != phase0)
    return late, finals, stray


def test_single_system_late_slot_reads_the_next_phase_only_with_the_tile_count_ticket():
    """A single system whose inner tiling has 3 tiles and whose FP64 tiling has 5 runs
    on lim = 8 slots.  With tickets counting the phase's tiles, a slot that starts after
    the finalize reads the next phase, runs one of its tiles inside the launch and takes
    a ticket toward it (the offset that stalls a later launch, as above).  With tickets
    counting every slot, the finalize is the last event of the launch."""
    rng = random.Random(5)
    ntiles, lim = {0: 3, 1: 5}, 8
    strays_old = 0
    for _ in range(2000):
        ev = _launch_schedule(lim, rng)
        late, finals, stray = _single_system_launch(ev, ntiles, 0, lim, count_slots=False)
        assert finals == 1
        strays_old += stray
        late, finals, stray = _single_system_launch(ev, ntiles, 0, lim, count_slots=True)
        assert (late, finals, stray) == (0, 1, 0)
    assert strays_old > 0

"""Model of the binning fill pass's workgroup tile table, run on the CPU.

The fill pass writes each triangle's record index into every tile list it
overlaps.  A workgroup first counts its entries per tile in an LDS hash
table (pass 1), reserves one contiguous range per tabled tile with one
global atomic on the tile's counter, then writes its entries (pass 2): a
tile found in the (now frozen) table takes the next position of the
workgroup's range, any other tile a position from its global counter.
This is only correct if pass 1 and pass 2 agree, entry by entry, on which
tiles are in the table.

The model below steps the lanes of one workgroup through the same shared
memory operations as the kernel's table functions (one read, compare-and-
swap or add per step), under a scheduler that picks which lane moves next,
and checks the result: every tile's list positions
[offs, offs + entries) are each written exactly once, and every tile
counter ends at zero.

An earlier protocol let pass 1 refuse a tile whenever the table held 3/4 of
its slots, even when the tile's key was about to be inserted by another
lane; pass 2 then found the key and wrote one past the workgroup's range.
`test_cutoff_protocol_overruns` replays that interleaving and shows the
overrun and the slot left unwritten.  The protocol the kernel uses refuses
only when the key's whole probe window holds other keys, which no later
insert can change (`test_fill_protocol_*`).
"""
from __future__ import annotations

import random

EMPTY = -1


class Table:
    """Workgroup table: slot keys, per-slot counts and offsets, occupancy."""

    def __init__(self, slots, probe, full):
        self.slots, self.probe, self.full = slots, probe, full
        self.key = [EMPTY] * slots
        self.cnt = [0] * slots
        self.off = [0] * slots
        self.nocc = 0

    def home(self, k):
        # any fixed hash works for the model; colliding keys are chosen by tests
        return (k * 7) % self.slots


def tile_slot(T, k, insert, cutoff):
    """Generator: the slot of key k (inserting when `insert`), or -1.

    Yields once before every shared-memory access so the scheduler can
    interleave lanes there; the final value is returned.  `cutoff` applies
    the refusal at occupancy >= T.full when an empty slot is met.
    """
    h = T.home(k)
    for p in range(T.probe):
        sl = (h + p) % T.slots
        yield
        cur = T.key[sl]
        if cur == k:
            return sl
        if cur == EMPTY:
            if not insert:
                return -1
            if cutoff:
                yield
                if T.nocc >= T.full:
                    return -1
            yield
            old = T.key[sl]  # compare-and-swap: one atomic step
            if old == EMPTY:
                T.key[sl] = k
                yield
                T.nocc += 1
                return sl
            if old == k:
                return sl
    return -1


def lane_pass1(T, keys, cutoff, log):
    for k in keys:
        sl = yield from tile_slot(T, k, True, cutoff)
        log.append((k, sl))
        if sl >= 0:
            yield
            T.cnt[sl] += 1


def lane_pass2(T, keys, offs, count, bins, who):
    for k in keys:
        sl = yield from tile_slot(T, k, False, False)
        yield
        if sl >= 0:
            pos = T.off[sl] + T.cnt[sl]
            T.cnt[sl] += 1
        else:
            count[k] -= 1
            pos = offs[k] + count[k]
        bins.setdefault(pos, []).append(who)


def run(gens, schedule):
    """Run generators to completion.  `schedule` = (script, seed): the
    script's lane indices are stepped in order (an entry for a lane that
    has finished is skipped), then lanes are picked at random from a
    generator seeded with `seed` until all have finished."""
    live = dict(enumerate(gens))
    script, seed = schedule
    rng = random.Random(seed)

    def step(i):
        try:
            next(live[i])
        except StopIteration:
            del live[i]

    for i in script:
        if i in live:
            step(i)
    while live:
        step(rng.choice(sorted(live)))


def fill(lane_keys, table_args, cutoff, sched1=((), 0), sched2=((), 0)):
    """One workgroup's fill pass over lanes' tile lists.  Returns (offs,
    count after fill, bins: position -> writers)."""
    tiles = sorted({k for ks in lane_keys for k in ks})
    entries = {k: sum(ks.count(k) for ks in lane_keys) for k in tiles}
    offs, o = {}, 0
    for k in tiles:
        offs[k] = o
        o += entries[k]
    count = dict(entries)  # the count pass left every tile's total here
    T = Table(*table_args)
    log = []
    run([lane_pass1(T, ks, cutoff, log) for ks in lane_keys], sched1)
    # barrier; reserve one range per tabled tile
    for sl in range(T.slots):
        k = T.key[sl]
        if k >= 0:
            n = T.cnt[sl]
            T.off[sl] = offs[k]
            count[k] -= n
            T.cnt[sl] = count[k]
    # barrier; pass 2 with frozen lookups
    bins = {}
    run([lane_pass2(T, ks, offs, count, bins, who) for who, ks in enumerate(lane_keys)], sched2)
    return offs, entries, count, bins


def check(offs, entries, count, bins):
    """Every position of every tile's range written once, nothing outside,
    every counter back at zero.  Returns a list of violations."""
    bad = []
    want = {offs[k] + j for k in offs for j in range(entries[k])}
    for pos, who in bins.items():
        if pos not in want:
            bad.append(("outside", pos))
        elif len(who) != 1:
            bad.append(("written twice", pos))
    for pos in want - set(bins):
        bad.append(("never written", pos))
    for k, c in count.items():
        if c != 0:
            bad.append(("counter", k, c))
    return bad


# Table of 8 slots, probe window 8, cutoff at 6 occupied: small enough to
# reach full occupancy with a handful of lanes.
SMALL = (8, 8, 6)


def adversarial_lanes():
    # lanes 0..4 insert five distinct tiles (home slots 7, 6, 5, 4, 3:
    # occupancy 5); lanes 5 and 6 both have tile 8 (home slot 0, empty);
    # lane 7 adds tile 6 (home slot 2), pushing occupancy to the cutoff
    # between lane 5's occupancy check and its compare-and-swap
    return [[1], [2], [3], [4], [5], [8], [8], [6]]


def adversarial_schedule():
    s = []
    for lane in range(5):  # lanes 0..4 run to completion: 5 slots taken
        s += [lane] * 8
    # lane 5: reads its home slot (empty); with the cutoff, its occupancy
    # check passes (5 < 6) and it stops before the compare-and-swap
    s += [5, 5, 5]
    # lane 7 inserts tile 6: occupancy 6
    s += [7] * 8
    # lane 6 reads the same slot, still empty; with the cutoff it is refused
    s += [6, 6, 6]
    # lane 5 completes its insert of tile 8, then lane 6 (if still live)
    s += [5] * 8 + [6] * 8
    return s


def test_cutoff_protocol_overruns():
    """The replaced protocol: a refusal at full occupancy while another lane
    inserts the same key makes pass 2 write one past the workgroup's range
    (overwriting an entry of the next tile) and leaves one position of the
    tile never written, its counter at 1."""
    lanes = adversarial_lanes()
    offs, entries, count, bins = fill(lanes, SMALL, cutoff=True, sched1=(adversarial_schedule(), 0))
    bad = check(offs, entries, count, bins)
    kinds = {b[0] for b in bad}
    assert "never written" in kinds
    assert "counter" in kinds and count[8] == 1
    # the extra write lands one past tile 8's range: on the next tile's
    # first entry, or here (tile 8 is the last tile) outside every range
    assert ("outside", offs[8] + entries[8]) in bad


def test_fill_protocol_adversarial_schedule():
    """The kernel's protocol on the same lanes and schedule: consistent."""
    lanes = adversarial_lanes()
    res = fill(lanes, SMALL, cutoff=False, sched1=(adversarial_schedule(), 0))
    assert check(*res) == []


def random_lanes(rng, n_lanes, n_tiles, per_lane):
    return [rng.sample(range(n_tiles), rng.randint(0, min(per_lane, n_tiles))) for _ in range(n_lanes)]


def test_fill_protocol_random_interleavings():
    """Many random interleavings of both passes, tables driven to and past
    full occupancy (more distinct tiles than slots, short probe windows so
    that exhaustion refusals happen): always consistent."""
    rng = random.Random(1)
    exhausted = 0
    for trial in range(400):
        slots = rng.choice([4, 8, 16])
        probe = rng.choice([1, 2, 4, slots])
        lanes = random_lanes(rng, rng.randint(2, 12), rng.randint(1, 3 * slots), 6)
        res = fill(lanes, (slots, probe, slots * 3 // 4), cutoff=False, sched1=((), trial), sched2=((), 10_000 + trial))
        assert check(*res) == [], (trial, lanes)
        exhausted += len({k for ks in lanes for k in ks}) > slots
    assert exhausted > 50  # the overfull case was exercised


def test_cutoff_protocol_fails_under_random_interleavings():
    """The same random search finds failures of the replaced protocol (so
    the search is strong enough to tell the two apart)."""
    rng = random.Random(2)
    failures = 0
    for trial in range(400):
        lanes = random_lanes(rng, 10, 12, 4)
        res = fill(lanes, SMALL, cutoff=True, sched1=((), trial), sched2=((), 10_000 + trial))
        failures += check(*res) != []
    assert failures > 0

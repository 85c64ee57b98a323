"""A lockstep model of the clip kernel's per-wave deposit tile (the opt-in
SIMPROJ_TILED_DEPOSIT path, DepF32::tile_add and the flush at a wave's end):
64 lanes deposit one piece each per step; every lane reads its cell's hashed
slot, the lanes whose cell holds the slot add there, then the others take the
slot over by compare-and-swap in lane order (the winner flushes the evicted
cell, a loser deposits directly), and at the end every resident cell is
flushed.  The model checks that each piece lands exactly once, in its own
cell, whatever the collisions: integer masses make the comparison exact.
The GPU tests (test_gpu_tiled_deposit.py) check the kernel itself against
the oracle."""
import random
from collections import defaultdict

EMPTY = 0xFFFFFFFF
TILE = 64


def slot(cell):
    # the kernel's multiplicative hash onto 64 slots
    return ((cell * 2654435761) & 0xFFFFFFFF) >> 26


def tiled(steps, adds_first=True):
    key = [EMPTY] * TILE
    val = [0] * TILE
    grid = defaultdict(int)
    for lanes in steps:
        reads = [(cell, x, slot(cell)) for cell, x in lanes]
        reads = [(cell, x, t, key[t]) for cell, x, t in reads]  # one load for every lane

        def adds():  # pieces of resident cells
            for cell, x, t, k in reads:
                if k == cell:
                    val[t] += x

        def takeovers():  # the others, in lane order
            for cell, x, t, k in reads:
                if k == cell:
                    continue
                if key[t] == k:  # compare-and-swap won
                    key[t] = cell
                    old, val[t] = val[t], x
                    if k != EMPTY:
                        grid[k] += old
                else:
                    grid[cell] += x

        if adds_first:
            adds()
            takeovers()
        else:
            takeovers()
            adds()
    for t in range(TILE):  # the wave's end
        if key[t] != EMPTY:
            grid[key[t]] += val[t]
    return grid


def direct(steps):
    grid = defaultdict(int)
    for lanes in steps:
        for cell, x in lanes:
            grid[cell] += x
    return grid


def _steps(rng, n_steps, n_cells, lanes=64):
    cells = rng.sample(range(1 << 24), n_cells)
    return [[(rng.choice(cells), rng.randrange(1, 1 << 20)) for _ in range(rng.randrange(1, lanes + 1))]
            for _ in range(n_steps)]


def test_every_piece_lands_once_in_its_cell():
    rng = random.Random(7)
    for n_cells in (1, 3, 40, 64, 200, 5000):
        steps = _steps(rng, 300, n_cells)
        assert tiled(steps) == direct(steps), n_cells


def test_colliding_cells_of_one_slot():
    # many distinct cells hashing to the same slot, in the same step
    rng = random.Random(11)
    same = [c for c in range(1 << 16) if slot(c) == 5][:20]
    steps = [[(rng.choice(same), rng.randrange(1, 1000)) for _ in range(64)] for _ in range(200)]
    assert tiled(steps) == direct(steps)


def test_hash_covers_every_slot():
    assert {slot(c) for c in range(1 << 14)} == set(range(TILE))


def test_phase_order_matters():
    """With the take-overs before the adds (the order the kernel's wave
    barrier rules out) pieces of an evicted cell land in its successor."""
    rng = random.Random(3)
    steps = _steps(rng, 300, 100)
    assert tiled(steps, adds_first=False) != direct(steps)

"""Host logic of the grouped-GEMM workgroup schedules (hp2sph_schedule_map, no
GPU needed): the map from workgroup id to (problem, tile) that each schedule
hands the GEMM kernel.

What every schedule must satisfy, checked on seeded problem lists (sizes of
the per-order problems: up to 9 row tiles, 1..3 column tiles, ragged edges):
* every 128 x 128 output tile of every problem is run by exactly one
  workgroup, and a workgroup without a tile holds (-1, -1);
* XCD schedules: the hardware deals workgroup w to XCD w mod 8, so all tiles
  of a problem sit at one residue mod 8, all XCDs get equally many slots, and
  each XCD runs its problems in list order and their tiles in order;
  round robin puts problem i on XCD i mod 8; balanced keeps the XCD loads
  (tiles x K) within the largest single problem's load of each other, the
  bound of greedy least-loaded placement;
* linear: workgroup w runs the w-th tile of the list in order, no padding;
* linear_rows: problems in list order, within each the row tiles of one column
  panel back to back (tile index = row * column_tiles + column), no padding."""

import ctypes

import numpy as np
import pytest

import paper_1904_10514_amd as P

TILE = 128
XCD = 8


def _tiles(M, N):
    return [(-(-m // TILE)) * (-(-n // TILE)) for m, n in zip(M, N)]


def _problem_lists():
    rng = np.random.default_rng(np.random.SeedSequence([1904, 10514, 77]))
    out = [([1], [2], [1]), ([128], [128], [16]), ([129], [130], [17])]
    for n in (5, 8, 9, 31, 300):
        M = rng.integers(1, 1100, n)
        N = 2 * rng.integers(1, 192, n)
        K = rng.integers(1, 1100, n)
        order = np.argsort(-(M.astype(np.int64) * K), kind="stable")   # longest first, as plans launch them
        out.append((M[order].tolist(), N[order].tolist(), K[order].tolist()))
    return out


def _coverage(mp, tiles):
    seen = {}
    for w, (p, t) in enumerate(mp):
        if p < 0:
            assert t == -1
            continue
        assert 0 <= p < len(tiles) and 0 <= t < tiles[p], (w, p, t)
        assert (p, t) not in seen, f"tile {(p, t)} run twice"
        seen[(p, t)] = w
    assert len(seen) == sum(tiles), "a tile is never run"
    return seen


@pytest.mark.parametrize("case", range(8))
def test_every_schedule_runs_each_tile_once(case):
    M, N, K = _problem_lists()[case]
    tiles = _tiles(M, N)
    for name in P.SCHEDULES:
        _coverage(P.schedule_map(name, M, N, K), tiles)


@pytest.mark.parametrize("case", range(8))
def test_linear_schedule_is_list_order(case):
    M, N, K = _problem_lists()[case]
    tiles = _tiles(M, N)
    mp = P.schedule_map("linear", M, N, K)
    expect = [(i, t) for i in range(len(M)) for t in range(tiles[i])]
    assert [tuple(x) for x in mp] == expect


@pytest.mark.parametrize("case", range(8))
def test_linear_rows_schedule_runs_row_tiles_of_a_panel_together(case):
    M, N, K = _problem_lists()[case]
    mp = P.schedule_map("linear_rows", M, N, K)
    expect = []
    for i in range(len(M)):
        rows, cols = -(-M[i] // TILE), -(-N[i] // TILE)
        expect += [(i, r * cols + c) for c in range(cols) for r in range(rows)]
    assert [tuple(x) for x in mp] == expect


def _xcd_lanes(mp, tiles):
    """Per XCD, the (problem, tile) sequence it runs; checks one XCD per problem."""
    assert len(mp) % XCD == 0
    lanes = [[tuple(mp[w]) for w in range(x, len(mp), XCD) if mp[w][0] >= 0] for x in range(XCD)]
    home = {}
    for x, lane in enumerate(lanes):
        for p, _ in lane:
            assert home.setdefault(p, x) == x, f"problem {p} split over XCDs"
        # problems in list order, tiles of each in order, each problem contiguous
        assert lane == sorted(lane)
        ps = [p for p, _ in lane]
        assert all(ps.count(p) == tiles[p] for p in set(ps))
    return lanes, home


@pytest.mark.parametrize("case", range(8))
def test_round_robin_deals_problems_to_xcds_in_turn(case):
    M, N, K = _problem_lists()[case]
    tiles = _tiles(M, N)
    lanes, home = _xcd_lanes(P.schedule_map("xcd_round_robin", M, N, K), tiles)
    assert all(home[i] == i % XCD for i in range(len(M)))


@pytest.mark.parametrize("case", range(8))
def test_balanced_schedule_bounds_the_xcd_loads(case):
    M, N, K = _problem_lists()[case]
    tiles = _tiles(M, N)
    mp = P.schedule_map("xcd_balanced", M, N, K)
    lanes, home = _xcd_lanes(mp, tiles)
    work = [tiles[i] * K[i] for i in range(len(M))]
    load = [0] * XCD
    for p, x in home.items():
        load[x] += work[p]
    assert max(load) - min(load) <= max(work)
    # padding only fills the XCDs up to the longest one
    assert len(mp) // XCD == max(len(lane) for lane in lanes)


def test_balanced_beats_round_robin_on_a_skewed_list():
    # one long problem per round of eight, then seven tiny ones: round robin
    # stacks every long problem on XCD 0
    M, N, K = [], [], []
    for _ in range(4):
        M += [1024] + [16] * 7
        N += [128] * 8
        K += [1024] + [16] * 7
    tiles = _tiles(M, N)
    work = [t * k for t, k in zip(tiles, K)]

    def max_load(name):
        _, home = _xcd_lanes(P.schedule_map(name, M, N, K), tiles)
        load = [0] * XCD
        for p, x in home.items():
            load[x] += work[p]
        return max(load)

    assert max_load("xcd_balanced") < max_load("xcd_round_robin") / 3


def test_schedule_map_errors():
    lib = P.lib()
    cnt = ctypes.c_int64(0)
    one = np.ones(1, dtype=np.int32)
    zero = np.zeros(1, dtype=np.int32)
    assert lib.hp2sph_schedule_map(len(P.SCHEDULES), one.ctypes.data, one.ctypes.data, one.ctypes.data, 1, None, 0,
                                   ctypes.byref(cnt)) == -1
    assert lib.hp2sph_schedule_map(0, one.ctypes.data, one.ctypes.data, one.ctypes.data, -1, None, 0,
                                   ctypes.byref(cnt)) == -1
    assert lib.hp2sph_schedule_map(0, zero.ctypes.data, one.ctypes.data, one.ctypes.data, 1, None, 0,
                                   ctypes.byref(cnt)) == -1
    assert lib.hp2sph_schedule_map(0, None, None, None, 1, None, 0, ctypes.byref(cnt)) == -1
    assert lib.hp2sph_schedule_map(0, None, None, None, 0, None, 0, ctypes.byref(cnt)) == 0
    assert cnt.value == 0
    with pytest.raises(ValueError):
        P.schedule_map("nonexistent", [1], [2], [1])

"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these re-types the oracle's own code: they check it against hand
traces, an external Philox implementation (rocRAND's open-source engine),
closed forms derived from the tile model, an independent brute-force
explorer of every growth order, exact invariances of the model and textbook
polyomino counts.
"""
import itertools
import math
import os
import random
import shutil
import subprocess

import numpy as np
import pytest

from oracle import ref
from tests import brute_force as bf

HERE = os.path.dirname(os.path.abspath(__file__))


def encode(tiles, c=8):
    """Genome of a tile list, seed first, colours N,E,S,W, MSB first."""
    bits = c.bit_length() - 1
    g = 0
    for tile in tiles:
        for col in tile:
            g = (g << bits) | col
    return g


def word_fn(run, rng_id, seed=1):
    def word(s):
        ctr = (s >> 2, run, rng_id & 0xFFFFFFFF, rng_id >> 32)
        return ref.philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))[s & 3]
    return word


# --------------------------------------------------------------------------
# Philox4x32-10 against rocRAND's engine (an implementation we did not write)
# --------------------------------------------------------------------------
def test_philox_matches_rocrand(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND probe")
    exe = tmp_path / "probe"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1",
                    os.path.join(HERE, "rocrand_philox_probe.cpp"), "-o", str(exe)],
                   check=True, cwd=str(tmp_path), capture_output=True)
    rng = random.Random(12345)
    cases = [(0, 0, 0, 0, 0, 0), (1, 0, 0, 0, 0, 0), (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF,
             0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF)]
    for _ in range(300):
        cases.append((rng.getrandbits(32), rng.getrandbits(32), rng.getrandbits(32),
                      rng.getrandbits(30), rng.getrandbits(32), rng.getrandbits(32)))
    # the counters the assembly uses: (step/4, run, rng_id lo, rng_id hi)
    for s, r in itertools.product(range(0, 12), range(0, 3)):
        g = rng.getrandbits(24)
        rid = g | (2 << 56)
        cases.append((1, 0, s, r, rid & 0xFFFFFFFF, rid >> 32))
    stdin = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
    out = subprocess.run([str(exe)], input=stdin, capture_output=True, text=True, check=True)
    lines = out.stdout.strip().splitlines()
    assert len(lines) == len(cases)
    for case, line in zip(cases, lines):
        k0, k1, c0, c1, c2, c3 = case
        want = tuple(int(v) for v in line.split())
        assert ref.philox4x32_10((c0, c1, c2, c3), (k0, k1)) == want, case


# --------------------------------------------------------------------------
# One-at-a-time hash: hand traces (App. F.4)
# --------------------------------------------------------------------------
def load_oaat_traces():
    cases = []
    with open(os.path.join(HERE, "golden", "oaat_hand_traces.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lhs, rhs = line.split("=")
            cases.append((bytes(int(b) for b in lhs.split(",")), int(rhs)))
    return cases


@pytest.mark.parametrize("data,want", load_oaat_traces())
def test_oaat_hand_traces(data, want):
    assert ref.oaat(data) == want


def test_collision_bound_eq2():
    """Eq. 2: 1 - prod_{i<=1000}(1 - i 2^-32) is about 0.01 % (1.16e-4)."""
    p = 1.0 - math.prod(1.0 - i * 2.0 ** -32 for i in range(1001))
    assert 1.1e-4 < p < 1.2e-4


# --------------------------------------------------------------------------
# Shape hash: D4 invariance and discrimination on free polyominoes
# --------------------------------------------------------------------------
def fixed_polyominoes(n):
    shapes = {frozenset([(0, 0)])}
    for _ in range(n - 1):
        nxt = set()
        for s in shapes:
            for (x, y) in s:
                for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                    c = (x + dx, y + dy)
                    if c not in s:
                        t = s | {c}
                        mx = min(p[0] for p in t)
                        my = min(p[1] for p in t)
                        nxt.add(frozenset((p[0] - mx, p[1] - my) for p in t))
        shapes = nxt
    return shapes


def to_mask(shape):
    w = max(p[0] for p in shape) + 1
    h = max(p[1] for p in shape) + 1
    m = np.zeros((h, w), dtype=np.uint8)
    for x, y in shape:
        m[y, x] = 1
    return m


def d4_images(mask):
    out = []
    for k in range(4):
        r = np.rot90(mask, k)
        out.append(r)
        out.append(np.fliplr(r))
    return out


def test_d4_hash_separates_free_polyominoes():
    # free polyomino counts for n = 1..6 (a textbook sequence): 1, 1, 2, 5, 12, 35
    want_free = [1, 1, 2, 5, 12, 35]
    all_hashes = set()
    for n, free in zip(range(1, 7), want_free):
        hashes = {ref.shape_hash_d4(to_mask(s)) for s in fixed_polyominoes(n)}
        assert len(hashes) == free, n
        assert not (hashes & all_hashes)
        all_hashes |= hashes


def test_d4_hash_invariance_random_shapes():
    rng = np.random.default_rng(3)
    for _ in range(200):
        h, w = rng.integers(1, 12, size=2)
        m = (rng.random((h, w)) < 0.5).astype(np.uint8)
        if not m.any():
            m[0, 0] = 1
        base = ref.shape_hash_d4(m)
        for img in d4_images(m):
            assert ref.shape_hash_d4(np.ascontiguousarray(img)) == base
        # padding with empty rows/cols does not change the hash
        padded = np.zeros((h + 3, w + 2), dtype=np.uint8)
        padded[1:1 + h, 2:2 + w] = m
        assert ref.shape_hash_d4(padded) == base


def test_monomer_and_square_hash_values():
    # monomer: one cell (0,0) in all 8 orientations -> OAAT of bytes 0,0 = 0
    # -> OAAT of 32 zero bytes = 0
    assert ref.shape_hash_d4(np.ones((1, 1), np.uint8)) == 0
    # 2x2 square: every orientation lists (0,0),(1,0),(0,1),(1,1)
    h = ref.oaat(bytes([0, 0, 1, 0, 0, 1, 1, 1]))
    assert ref.shape_hash_d4(np.ones((2, 2), np.uint8)) == ref.oaat(h.to_bytes(4, "little") * 8)


# --------------------------------------------------------------------------
# Genome layout (App. B.3) and the closed forms of S_{1,8}
# --------------------------------------------------------------------------
def test_genome_bit_order_and_seed_position():
    sq = encode([(1, 2, 0, 0)])          # N=1, E=2: a 2x2 square
    assert sq == 640
    cells, ev, choice = ref.trace_run(sq, 1, run=0)
    assert ev == ref.EV_NONE and choice == 1
    # the seed sits at (G/2, G/2); N is y-1 and E is x+1
    assert cells[0] == (8, 8)
    assert set(cells) == {(8, 8), (8, 7), (9, 8), (9, 7)}
    # tile 0 is the seed: an inert seed assembles nothing
    assert ref.classify_one(encode([(0, 0, 0, 0), (1, 2, 0, 0)]), 2)[:3] == (ref.DET, 1, 0)
    assert ref.classify_one(encode([(1, 2, 0, 0), (0, 0, 0, 0)]), 2)[:2] == (ref.DET, 4)


def s18_groups():
    """Partition S_{1,8} by hand-derivable behaviour (from the pair rule)."""
    pairs = [(1, 2), (3, 4), (5, 6)]
    mono, square, line = [], [], []
    for g in range(4096):
        tile = bf.decode(g, 1, 8)[0]
        present = [p for p in pairs if p[0] in tile and p[1] in tile]
        if not present:
            mono.append(g)
            continue
        if len(present) == 1:
            a, b = present[0]
            ia = [i for i in range(4) if tile[i] == a]
            ib = [i for i in range(4) if tile[i] == b]
            rest = [tile[i] for i in range(4) if i not in ia + ib]
            if len(ia) == 1 and len(ib) == 1 and all(x in (0, 7) for x in rest):
                if (ia[0] - ib[0]) % 2:
                    square.append(g)
                else:
                    line.append(g)
    return mono, square, line


def test_s18_closed_forms():
    recs = ref.classify_range(0, 4096, 1, grid=16, runs=20, seed=1)
    mono, square, line = s18_groups()
    assert (len(mono), len(square), len(line)) == (2398, 96, 48)
    for g in mono:      # no colour meets its partner: the seed stays alone
        assert tuple(recs[g]) == (ref.DET, 1, 0, 0)
    sq_hash = ref.shape_hash_d4(np.ones((2, 2), np.uint8))
    for g in square:    # one pair on adjacent edges: the 2x2 square
        cls, size, h, steps = (int(v) for v in recs[g])
        assert (cls, size, h) == (ref.DET, 4, sq_hash)
        assert steps == 20 * 3   # run 0 had a choice, so all 20 runs are made
    for g in line:      # one pair on opposite edges: an endless straight line
        assert recs[g]["cls"] == ref.UNBOUND
        # the line reaches the ring after 7 to 14 placements on a 16-grid
        assert 8 <= recs[g]["size"] <= 15


# --------------------------------------------------------------------------
# Brute force over every growth order
# --------------------------------------------------------------------------
def check_against_brute(g, t, grid, rec, runs=20, cap=50_000):
    cls, size, h, steps = (int(v) for v in rec)
    if cls == ref.UNBOUND:
        ex = bf.explore(g, t, 8, grid, cap=cap, stop_at={"UNBOUND"})
        assert "UNBOUND" in ex.events, (g, t, grid)
    elif cls == ref.ND_SITE:
        ex = bf.explore(g, t, 8, grid, cap=cap, stop_at={"AMBIG"})
        assert "AMBIG" in ex.events, (g, t, grid)
    elif cls == ref.ND_RUNS:
        ex = bf.explore(g, t, 8, grid, cap=cap)
        assert ex.capped or len(ex.terminals) >= 2 or ex.events
    else:
        ex = bf.explore(g, t, 8, grid, cap=cap)
        if ex.capped:
            return "capped"
        # the oracle's shape is reachable
        (_, occ) = ref.classify_one(g, t, grid=grid, runs=runs, with_occupancy=True)
        shape = frozenset((x, y) for y in range(grid + 1) for x in range(grid + 1) if occ[y, x])
        assert shape in ex.terminals, (g, t, grid)
        assert size == len(shape)
        assert h == ref.shape_hash_d4(occ)
        if ex.truly_det:
            # every run places size-1 tiles; all runs are made iff run 0 chose
            assert steps == (size - 1) * (1 if ex.choice_free else runs)
            return "det"
        return "misclassified"
    return "ok"


@pytest.mark.parametrize("grid", [8, 16])
def test_brute_force_all_of_s18(grid):
    recs = ref.classify_range(0, 4096, 1, grid=grid, runs=20)
    tally = {}
    for g in range(4096):
        k = check_against_brute(g, 1, grid, recs[g])
        tally[k] = tally.get(k, 0) + 1
    assert tally.get("capped", 0) == 0
    # truly deterministic single tiles are never misclassified at R = 20
    assert tally.get("misclassified", 0) == 0


def test_brute_force_sampled_s28_s38():
    rng = random.Random(7)
    recs_by = {}
    for t, n in ((2, 400), (3, 250)):
        gs = [rng.getrandbits(12 * t) for _ in range(n)]
        recs = ref.classify(np.array(gs, dtype=np.uint64), t, grid=16)
        recs_by[t] = (gs, recs)
    # bias towards the interesting classes: all non-trivial ones in the sample
    for t, (gs, recs) in recs_by.items():
        for g, rec in zip(gs, recs):
            if rec["steps"] == 0 and rec["cls"] == ref.DET:
                continue
            check_against_brute(g, t, 16, rec, cap=20_000)


def test_every_det_shape_of_s28_is_truly_det():
    """One genotype per DET shape of S_{2,8} (G=16), found by scanning a
    stride of the space: its shape is the unique terminal of every order."""
    rng = np.random.default_rng(11)
    gs = rng.integers(0, 1 << 24, size=200_000, dtype=np.uint64)
    recs = ref.classify(gs, 2, grid=16)
    seen = {}
    for g, rec in zip(gs.tolist(), recs):
        if rec["cls"] == ref.DET and int(rec["hash"]) not in seen:
            seen[int(rec["hash"])] = (g, rec)
    assert len(seen) >= 10
    for h, (g, rec) in seen.items():
        assert check_against_brute(g, 2, 16, rec, cap=100_000) in ("det", "misclassified")


def test_trace_equals_from_scratch_replay():
    """Each oracle run equals a replay that recomputes the whole frontier
    from scratch at every step (eager update == isotropic re-check)."""
    rng = random.Random(99)
    cases = [(g, 1) for g in rng.sample(range(4096), 120)]
    cases += [(rng.getrandbits(24), 2) for _ in range(150)]
    cases += [(rng.getrandbits(36), 3) for _ in range(100)]
    for g, t in cases:
        rid = ref.default_rng_id(g, t)
        for run in (0, 1, 7):
            cells, ev, choice = ref.trace_run(g, t, run, grid=16)
            order, event, bchoice, _ = bf.replay(g, t, 8, 16, word_fn(run, rid))
            assert cells == order, (g, t, run)
            want_ev = {None: ref.EV_NONE, "UNBOUND": ref.EV_UNBOUND, "AMBIG": ref.EV_AMBIG}[event]
            assert ev == want_ev and choice == int(bchoice), (g, t, run)


# --------------------------------------------------------------------------
# Exact invariances of the model (records bit-identical with rng_id fixed)
# --------------------------------------------------------------------------
def relabel(tiles, sigma):
    return [tuple(sigma[c] for c in tile) for tile in tiles]


COLOUR_MAPS = [
    {0: 0, 1: 2, 2: 1, 3: 3, 4: 4, 5: 5, 6: 6, 7: 7},   # swap within a pair
    {0: 0, 1: 3, 2: 4, 3: 5, 4: 6, 5: 1, 6: 2, 7: 7},   # permute the pairs
    {0: 7, 1: 1, 2: 2, 3: 3, 4: 4, 5: 5, 6: 6, 7: 0},   # swap the two inert colours
]


def test_exact_invariances():
    rng = random.Random(5)
    for _ in range(300):
        t = rng.choice((2, 3))
        g = rng.getrandbits(12 * t)
        tiles = bf.decode(g, t, 8)
        rid = ref.default_rng_id(g, t)
        base = ref.classify_one(g, t, rng_id=rid)
        variants = []
        # rotate a non-seed tile's edge list
        variants.append((tiles[:1] + [bf.rotate(tiles[1], rng.randrange(1, 4))] + tiles[2:], t))
        # permute the non-seed tiles
        if t == 3:
            variants.append(([tiles[0], tiles[2], tiles[1]], t))
        # relabel colours preserving the pairing
        for sigma in COLOUR_MAPS:
            variants.append((relabel(tiles, sigma), t))
        # pad with a duplicate tile or with an inert tile
        if t == 2:
            variants.append((tiles + [tiles[1]], 3))
            variants.append((tiles + [(0, 7, 0, 0)], 3))
            variants.append((tiles + [bf.rotate(tiles[0], 2)], 3))
        for vt, vtn in variants:
            assert ref.classify_one(encode(vt), vtn, rng_id=rid) == base, (g, t, vt)


def test_single_tile_padding():
    for g in range(0, 4096, 7):
        rid = ref.default_rng_id(g, 1)
        base = ref.classify_one(g, 1)
        tile = bf.decode(g, 1, 8)[0]
        assert ref.classify_one(encode([tile, tile]), 2, rng_id=rid) == base
        assert ref.classify_one(encode([tile, (0, 0, 0, 0)]), 2, rng_id=rid) == base


def test_shape_invariance_of_truly_det():
    """Rotating every tile (seed included) rotates the assembly; mirroring
    every tile mirrors it.  Truly deterministic genotypes keep their class and
    D4 hash."""
    rng = np.random.default_rng(21)
    gs = rng.integers(0, 1 << 24, size=20_000, dtype=np.uint64)
    recs = ref.classify(gs, 2, grid=16)
    picked = [int(g) for g, r in zip(gs, recs) if r["cls"] == ref.DET and r["size"] > 1][:150]
    checked = 0
    for g in picked:
        ex = bf.explore(g, 2, 8, 16, cap=20_000)
        if not ex.truly_det:
            continue
        tiles = bf.decode(g, 2, 8)
        base = ref.classify_one(g, 2)
        for r in (1, 2, 3):
            rot = [bf.rotate(tl, r) for tl in tiles]
            got = ref.classify_one(encode(rot), 2)
            assert (got[0], got[1], got[2]) == base[:3]
        mir = [(tl[0], tl[3], tl[2], tl[1]) for tl in tiles]
        got = ref.classify_one(encode(mir), 2)
        assert (got[0], got[1], got[2]) == base[:3]
        checked += 1
    assert checked >= 50


def test_misclassification_never_grows_with_runs():
    """Runs 0..R-1 are a prefix of runs 0..R'-1: once a witness is found at R
    it is found at every R' >= R (§3.2: error falls as k grows)."""
    rng = np.random.default_rng(4)
    gs = rng.integers(0, 1 << 24, size=20_000, dtype=np.uint64)
    prev = None
    for R in (1, 2, 4, 8, 20):
        recs = ref.classify(gs, 2, grid=16, runs=R)
        det = recs["cls"] == ref.DET
        if prev is not None:
            assert not np.any(det & ~prev)
        prev = det


# --------------------------------------------------------------------------
# Argument checking
# --------------------------------------------------------------------------
@pytest.mark.parametrize("t,c,grid,runs", [(0, 8, 16, 20), (5, 8, 16, 20), (2, 3, 16, 20),
                                           (2, 8, 15, 20), (2, 8, 6, 20), (2, 8, 66, 20),
                                           (2, 8, 16, 0), (2, 8, 16, 65), (4, 32, 16, 1)])
def test_invalid_arguments(t, c, grid, runs):
    assert ref.check_args(t, c, grid, runs) != 0


def test_genome_with_stray_bits_rejected():
    with pytest.raises(ValueError):
        ref.classify_one(1 << 24, 2)
    with pytest.raises(ValueError):
        ref.classify_range((1 << 24) - 1, 2, 2)


def test_widest_genome_c16_t4():
    g = (1 << 64) - 1
    rec = ref.classify_one(g, 4, c=16)
    assert rec[0] in (ref.UNBOUND, ref.ND_SITE, ref.ND_RUNS, ref.DET)


# ---------------------------------------------------------------------------
# Forced shapes: a first-run shape in which every cell's occupied neighbours
# bond to that cell's own tile only.  Pinned against the classification
# itself (every forced genotype is DET with (size - 1) * R placements, for
# every R) and against the independent brute-force explorer (every growth
# order ends in that one shape, with no event).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("t,grid,space", [(1, 16, 4096), (2, 16, 1 << 24), (3, 16, 1 << 36),
                                          (3, 32, 1 << 36)])
def test_forced_shapes_classify_det_for_every_run_count(t, grid, space):
    rng = np.random.default_rng(t * 100 + grid)
    n = min(2048, space)
    seen = 0
    for first in rng.integers(0, max(1, space - n), size=4):
        for runs in (2, 7, 20):
            recs, s0, e0, c0, f0 = ref.classify_range_run0(int(first), n, t, grid=grid,
                                                           runs=runs, forced=True)
            forced = (f0 & 1) != 0
            seen += int(np.sum(forced & (c0 == 1)))
            assert np.all(e0[forced] == 0)
            assert np.all(recs["cls"][forced] == ref.DET)
            placed = recs["size"][forced].astype(np.int64) - 1
            want = np.where(c0[forced] == 1, placed * runs, placed)
            assert np.array_equal(recs["steps"][forced].astype(np.int64), want)
    assert seen > 0     # forced shapes whose first run drew random words


def test_forced_shapes_are_the_only_terminal_of_every_order():
    """Forced genotypes of S_{2,8} whose first run drew random words: the
    brute-force explorer finds no event and exactly one terminal assembly,
    the first run's shape."""
    rng = np.random.default_rng(77)
    starts = rng.integers(0, (1 << 24) - 4096, size=4)
    checked = 0
    for first in starts:
        recs, s0, e0, c0, f0 = ref.classify_range_run0(int(first), 4096, 2, forced=True)
        for i in np.nonzero(((f0 & 1) != 0) & (c0 == 1))[0][:12]:
            g = int(first) + int(i)
            ex = bf.explore(g, 2, 8, 16, cap=20_000)
            if ex.capped:
                continue
            assert not ex.events, g
            assert len(ex.terminals) == 1, g
            shape = next(iter(ex.terminals))
            assert len(shape) == recs["size"][i], g
            checked += 1
    assert checked >= 20


# ---------------------------------------------------------------------------
# Guarded shapes: a first-run shape in which, for every cell p other than the
# seed and every occupied neighbour q whose tile admits at p something other
# than p's tile, q cannot be reached from the seed over exact bonds without
# passing through p.  Every forced shape is guarded.  Pinned like the forced
# shapes: against the classification at several run counts (DET, first-run
# size, (size - 1) * R placements) and against the brute-force explorer
# (every growth order ends in the first run's shape, with no event).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("t,grid,space", [(2, 16, 1 << 24), (3, 16, 1 << 36), (3, 32, 1 << 36),
                                          (4, 10, 1 << 48)])
def test_guarded_shapes_classify_det_for_every_run_count(t, grid, space):
    rng = np.random.default_rng(t * 1000 + grid)
    beyond_forced = 0
    for first in rng.integers(0, space - 4096, size=3):
        for runs in (2, 7, 20):
            recs, s0, e0, c0, f0 = ref.classify_range_run0(int(first), 2048, t, grid=grid,
                                                           runs=runs, forced=True)
            forced = (f0 & 1) != 0
            guarded = (f0 & 2) != 0
            assert not np.any(forced & ~guarded)         # forced implies guarded
            assert np.all(e0[guarded] == 0)
            assert np.all(recs["cls"][guarded] == ref.DET)
            placed = recs["size"][guarded].astype(np.int64) - 1
            want = np.where(c0[guarded] == 1, placed * runs, placed)
            assert np.array_equal(recs["steps"][guarded].astype(np.int64), want)
            beyond_forced += int(np.sum(guarded & ~forced & (c0 == 1)))
    assert beyond_forced > 0


def test_guarded_shapes_are_the_only_terminal_of_every_order():
    """Guarded genotypes of S_{2,8} and of the three-tile space that are not
    forced (so a neighbour of some cell admits another tile there): the
    brute-force explorer finds no event and exactly one terminal assembly,
    the first run's shape."""
    rng = np.random.default_rng(78)
    checked = 0
    for t, space in ((2, 1 << 24), (3, 1 << 36)):
        for first in rng.integers(0, space - 4096, size=3):
            recs, s0, e0, c0, f0 = ref.classify_range_run0(int(first), 4096, t, forced=True)
            pick = np.nonzero(((f0 & 2) != 0) & ((f0 & 1) == 0) & (c0 == 1))[0]
            for i in pick[:10]:
                g = int(first) + int(i)
                ex = bf.explore(g, t, 8, 16, cap=20_000)
                if ex.capped:
                    continue
                assert not ex.events, (t, g)
                assert len(ex.terminals) == 1, (t, g)
                assert len(next(iter(ex.terminals))) == recs["size"][i], (t, g)
                checked += 1
    assert checked >= 30


# ---------------------------------------------------------------------------
# The 16 x 16 window: a genotype classified with G = 16 gets the record of its
# own G > 16 unless that record is UNBOUND (no run up to the deciding one
# reached the window's ring, and such runs are the runs in the larger grid).
# A pipeline may classify G > 16 in the window and rerun only the UNBOUND
# ones; pinned here on the oracle for t = 2..4 and G = 18..32.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("t,grid", [(2, 32), (3, 32), (3, 20), (4, 24), (2, 18)])
def test_window_records_equal_unless_unbound(t, grid):
    rng = np.random.default_rng(500 + 10 * t + grid)
    g = rng.integers(0, 1 << (12 * t), size=4000, dtype=np.uint64)
    small = ref.classify(g, t, grid=16)
    big = ref.classify(g, t, grid=grid)
    inside = small["cls"] != ref.UNBOUND
    assert np.array_equal(small[inside], big[inside])
    # and the window is not vacuous: some records differ, all of them UNBOUND at 16
    assert np.any(~inside)
    assert np.all(small["cls"][small != big] == ref.UNBOUND)

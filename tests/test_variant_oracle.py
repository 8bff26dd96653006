"""Pins of the oracle's classification variants: the C4 shape hash (§3.3:
the four rotations hashed, sorted and hashed again) and the LIFO movelist
traversal (§3.2: frontier sites on a stack, inserted at random positions,
taken from the top).

C4 hash:
  - invariant under the four rotations of random masks;
  - exactly 1, 1, 2, 7, 18, 60 distinct values over the polyominoes of
    1..6 cells (the one-sided polyomino counts, a textbook sequence);
  - tells a chiral shape from its mirror image, which D4 does not.
LIFO traversal (against the brute-force explorer, tests/brute_force.py):
  - every run is a valid growth order (each placed cell was a frontier
    site of the configuration before it, recomputed from scratch) and ends
    as the explorer says that configuration ends;
  - every UNBOUND or ND verdict has a witness among the explorer's
    outcomes and every DET shape is a terminal the explorer reaches;
  - genotypes whose growth never offers a choice give the same records as
    the uniform traversal (no draw is made in either);
  - a site's insertion slot is uniform: the first of two sites that join an
    empty-started stack together is on top half of the time.
"""
import numpy as np
import pytest

from oracle import ref
from tests import brute_force as bf
from tests.test_oracle_pins import fixed_polyominoes, to_mask


def rotations(mask):
    return [np.rot90(mask, k) for k in range(4)]


def test_c4_hash_is_rotation_invariant():
    rng = np.random.default_rng(3)
    for _ in range(200):
        h, w = rng.integers(1, 8, size=2)
        m = (rng.random((h, w)) < 0.5).astype(np.uint8)
        if not m.any():
            continue
        m = m[np.ix_(m.any(axis=1), m.any(axis=0))]
        hs = {ref.shape_hash_c4(r) for r in rotations(m)}
        assert len(hs) == 1


def test_c4_hash_counts_one_sided_polyominoes():
    want = [1, 1, 2, 7, 18, 60]
    seen = set()
    for n, k in zip(range(1, 7), want):
        hs = {ref.shape_hash_c4(to_mask(s)) for s in fixed_polyominoes(n)}
        assert len(hs) == k, n
        assert not (hs & seen)
        seen |= hs


def test_c4_separates_mirror_images_d4_does_not():
    ell = np.array([[1, 0], [1, 0], [1, 1]], dtype=np.uint8)
    jay = np.fliplr(ell)
    assert ref.shape_hash_c4(ell) != ref.shape_hash_c4(jay)
    assert ref.shape_hash_d4(ell) == ref.shape_hash_d4(jay)
    square = np.ones((2, 2), dtype=np.uint8)
    assert ref.shape_hash_c4(square) == ref.shape_hash_c4(np.fliplr(square))


def test_c4_records_differ_from_d4_only_in_the_hash():
    g = np.arange(4096, dtype=np.uint64)
    d4 = ref.classify(g, 1)
    c4 = ref.classify_variant(g, 1, ref.VARIANT_C4)
    for f in ("cls", "size", "steps"):
        assert np.array_equal(d4[f], c4[f])
    assert np.array_equal(d4["hash"] == 0, c4["hash"] == 0)


def replay_is_valid(genome, t, cells, event, grid=16):
    """The placements are a growth order: each cell was a frontier site of
    the configuration before it; the run ends as that configuration does."""
    m = bf.Model(genome, t, 8, grid)
    centre = m.centre
    off = (centre[0] - (grid // 2), centre[1] - (grid // 2))
    placed = {centre: m.seed_tile}
    for (x, y) in cells[1:]:
        q = (x + off[0], y + off[1])
        ev, frontier = m.analyse(placed)
        assert ev is None, (genome, ev)
        assert q in frontier, (genome, q)
        placed[q] = frontier[q]
    ev, frontier = m.analyse(placed)
    want = {0: None, 1: "UNBOUND", 2: "AMBIG"}[event]
    assert ev == want, (genome, ev, want)
    if ev is None:
        assert not frontier
    return placed


@pytest.mark.parametrize("t", [1, 2])
def test_lifo_runs_are_growth_orders(t):
    rng = np.random.default_rng(10 + t)
    for g in rng.integers(0, 1 << (12 * t), size=60, dtype=np.uint64):
        for run in (0, 3):
            cells, ev, _ = ref.trace_run_variant(int(g), t, run, ref.VARIANT_LIFO)
            replay_is_valid(int(g), t, cells, ev)


def test_lifo_verdicts_have_witnesses():
    rng = np.random.default_rng(21)
    pool = rng.integers(0, 1 << 24, size=150, dtype=np.uint64)
    rec = ref.classify_variant(pool, 2, ref.VARIANT_LIFO)
    for g, r in zip(pool, rec):
        ex = bf.explore(int(g), 2, 8, 16, cap=3_000)
        if ex.capped:
            continue
        if r["cls"] == ref.UNBOUND:
            assert "UNBOUND" in ex.events
        elif r["cls"] == ref.ND_SITE:
            assert "AMBIG" in ex.events
        elif r["cls"] == ref.ND_RUNS:
            assert len(ex.terminals) >= 2 or ex.events
        elif r["cls"] == ref.DET:
            sizes = {len(s) for s in ex.terminals}
            assert r["size"] in sizes
        if ex.truly_det:
            assert r["cls"] == ref.DET


def test_choice_free_genotypes_agree_with_uniform_traversal():
    g = np.arange(4096, dtype=np.uint64)
    uni = ref.classify(g, 1)
    lifo = ref.classify_variant(g, 1, ref.VARIANT_LIFO)
    rng = np.random.default_rng(2)
    g2 = rng.integers(0, 1 << 24, size=3000, dtype=np.uint64)
    uni2 = ref.classify(g2, 2)
    lifo2 = ref.classify_variant(g2, 2, ref.VARIANT_LIFO)
    for u, l, gs, t in ((uni, lifo, g, 1), (uni2, lifo2, g2, 2)):
        free = []
        for i, x in enumerate(gs[:300]):
            ex = bf.explore(int(x), t, 8, 16, cap=300)
            if not ex.capped and ex.choice_free:
                free.append(i)
        assert len(free) > 50
        free = np.array(free)
        assert np.array_equal(u[free], l[free])


def test_insertion_slot_is_uniform():
    """A tile with two bonding sides facing partners on one tile: the seed's
    update inserts the E site into an empty stack, then the S site at slot
    0 or 1 with one draw; the top is placed first."""
    # seed N,E,S,W = 0,1,1,0 (E and S show colour 1) and a second tile
    # 2,2,2,2 bonds to both: the seed's E and S sites join the frontier
    genome = (0 << 21) | (1 << 18) | (1 << 15) | (0 << 12) | (2 << 9) | (2 << 6) | (2 << 3) | 2
    firsts = []
    for rid in range(2000):
        cells, _, _ = ref.trace_run_variant(genome, 2, 0, ref.VARIANT_LIFO, rng_id=rid)
        firsts.append(cells[1])
    xs = {c for c in firsts}
    assert len(xs) == 2
    share = np.mean([c == firsts[0] for c in firsts])
    assert abs(share - 0.5) < 5 * np.sqrt(0.25 / 2000)

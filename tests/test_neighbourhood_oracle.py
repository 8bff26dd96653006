"""Pins of the oracle's robustness and evolvability (§1.1: the proportion of
single mutations that keep the phenotype, the number of different
phenotypes single mutations reach), against the independent brute-force
explorer (tests/brute_force.py).

The explorer (its model and from-scratch site options) follows every growth
order.  Where every order ends the same
way - one terminal shape and no event (DET), or only UNBOUND events, or only
ambiguous sites (ND) - the phenotype is fixed whatever the random stream,
so it can be derived without the classifier.  For every genotype whose own
phenotype and whose mutants' phenotypes are all fixed that way, the
explorer's counts must equal the oracle's.  The mutants are made here from
the decoded colour digits (flip bit j of the colour of side d of tile i),
not from the genome word.
"""
import numpy as np

from oracle import ref
from tests import brute_force as bf


def shape_hash(cells):
    xs = [x for x, _ in cells]
    ys = [y for _, y in cells]
    w, h = max(xs) - min(xs) + 1, max(ys) - min(ys) + 1
    m = np.zeros((h, w), dtype=np.uint8)
    for x, y in cells:
        m[y - min(ys), x - min(xs)] = 1
    return ref.shape_hash_d4(m)


def fixed_phenotype(genome, t, c=8, grid=16, cap=800):
    """('DET', size, hash), ('UNBOUND',), ('ND',) or None when the outcome
    depends on the random stream (two different outcomes are reachable) or
    more than `cap` configurations would have to be visited to tell.
    Depth first over every growth order, memoised on the configuration."""
    m = bf.Model(genome, t, c, grid)
    seen = set()
    stack = [{m.centre: m.seed_tile}]
    outcome = None
    while stack:
        placed = stack.pop()
        key = frozenset(placed.items())
        if key in seen:
            continue
        seen.add(key)
        if len(seen) > cap:
            return None
        event, frontier = m.analyse(placed)
        if event is not None:
            o = ("UNBOUND",) if event == "UNBOUND" else ("ND",)
        elif not frontier:
            o = ("DET", frozenset(placed))
        else:
            for q, tile in frontier.items():
                nxt = dict(placed)
                nxt[q] = tile
                stack.append(nxt)
            continue
        if outcome is not None and o != outcome:
            return None
        outcome = o
    if outcome[0] == "DET":
        return ("DET", len(outcome[1]), shape_hash(outcome[1]))
    return outcome


def encode(tiles, c):
    bits = c.bit_length() - 1
    g = 0
    for tile in tiles:
        for colour in tile:
            g = (g << bits) | colour
    return g


def digit_mutants(genome, t, c=8):
    bits = c.bit_length() - 1
    tiles = [list(x) for x in bf.decode(genome, t, c)]
    out = []
    for i in range(t):
        for d in range(4):
            for j in range(bits):
                m = [list(x) for x in tiles]
                m[i][d] ^= 1 << j
                out.append(encode(m, c))
    return out


def test_single_mutants_are_the_bit_flips():
    rng = np.random.default_rng(4)
    for t in (1, 2, 3):
        for g in rng.integers(0, 1 << (12 * t), size=20, dtype=np.uint64):
            assert sorted(digit_mutants(int(g), t)) == sorted(ref.mutants(np.array([g]), t)[0]
                                                              .tolist())


def brute_counts(genomes, t):
    pheno = {}

    def ph(g):
        if g not in pheno:
            pheno[g] = fixed_phenotype(g, t)
        return pheno[g]

    got = {}
    for g in genomes:
        own = ph(int(g))
        if own is None:
            continue
        ms = [ph(m) for m in digit_mutants(int(g), t)]
        if any(p is None for p in ms):
            continue
        got[int(g)] = (sum(p == own for p in ms), len({p for p in ms if p != own}))
    return got


def test_s18_robustness_and_evolvability_match_brute_force():
    g = np.arange(4096, dtype=np.uint64)
    robust, evolv = ref.neighbourhood(g, 1)
    want = brute_counts(g, 1)
    assert len(want) > 3000
    for k, (r, e) in want.items():
        assert (robust[k], evolv[k]) == (r, e), k


def test_s28_sample_robustness_and_evolvability_match_brute_force():
    rng = np.random.default_rng(8)
    g = rng.integers(0, 1 << 24, size=200, dtype=np.uint64)
    robust, evolv = ref.neighbourhood(g, 2)
    want = brute_counts(g, 2)
    assert len(want) > 60
    idx = {int(x): i for i, x in enumerate(g)}
    for k, (r, e) in want.items():
        assert (robust[idx[k]], evolv[idx[k]]) == (r, e), k


def test_counts_are_consistent():
    """robust + (mutants with another phenotype) = 4 t b; evolv is at most
    the number of mutants with another phenotype, and 0 exactly when every
    mutant keeps the phenotype."""
    rng = np.random.default_rng(9)
    g = rng.integers(0, 1 << 24, size=2000, dtype=np.uint64)
    robust, evolv = ref.neighbourhood(g, 2)
    assert np.all((robust >= 0) & (robust <= 24))
    assert np.all(evolv <= 24 - robust)
    assert np.array_equal(evolv == 0, robust == 24)

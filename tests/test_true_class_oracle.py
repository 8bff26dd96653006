"""Pins of the oracle's exhaustive true class (every growth order followed,
§3.2; the misclassification of §4.1 is measured against it).

  - every genotype of S_{1,8} and a sample of S_{2,8}: deterministic exactly
    when the independent brute-force explorer (tests/brute_force.py: its
    own decoding, bond rule and from-scratch site options, depth first)
    finds no event and one terminal shape, and then the same shape;
  - soundness of the stochastic classifier: a genotype it classes non-DET
    (a witness run exists) is never truly deterministic;
  - a guarded first-run shape or a choice-free first run is truly
    deterministic, with the stochastic record's size and hash.
"""
import numpy as np
import pytest

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


def check_against_brute_force(genomes, t):
    tr = ref.true_class(genomes, t, grid=16)
    assert np.all(tr["cls"] != ref.TRUE_CAPPED)
    for g, r in zip(genomes, tr):
        ex = bf.explore(int(g), t, 8, 16, cap=400_000, stop_at={"UNBOUND", "AMBIG"})
        assert not ex.capped, int(g)
        assert ex.truly_det == (r["cls"] == ref.DET), int(g)
        if ex.truly_det:
            (shape,) = ex.terminals
            assert r["size"] == len(shape), int(g)
            assert r["hash"] == shape_hash(shape), int(g)
        else:
            assert r["size"] == 0 and r["hash"] == 0


def test_true_class_of_s18_matches_brute_force():
    check_against_brute_force(np.arange(4096, dtype=np.uint64), 1)


def test_true_class_of_s28_sample_matches_brute_force():
    rng = np.random.default_rng(31)
    pool = rng.integers(0, 1 << 24, size=1 << 15, dtype=np.uint64)
    rec = ref.classify(pool, 2, grid=16, runs=20, seed=1)
    # every class, weighted towards deterministic records with a choice (the
    # ones a few runs can get wrong)
    cand = pool[(rec["cls"] == ref.DET) & (rec["steps"] == (rec["size"] - 1) * 20)
                & (rec["size"] >= 3)]
    rest = pool[:400]
    check_against_brute_force(np.concatenate([cand[:300], rest]), 2)


def test_stochastic_witness_implies_true_nd_and_proofs_imply_true_det():
    n = 1 << 16
    first = 5 << 20
    rec, s0, e0, c0, f0 = ref.classify_range_run0(first, n, 2, grid=16, runs=20, seed=1,
                                                  forced=True)
    g = np.arange(first, first + n, dtype=np.uint64)
    tr = ref.true_class(g, 2, grid=16)
    assert np.all(tr["cls"] != ref.TRUE_CAPPED)
    nd = rec["cls"] != ref.DET
    assert not np.any(tr["cls"][nd] == ref.DET)
    proven = (e0 == 0) & ((c0 == 0) | ((f0 & 2) != 0))
    assert np.all(tr["cls"][proven] == ref.DET)
    assert np.array_equal(tr["size"][proven], rec["size"][proven])
    assert np.array_equal(tr["hash"][proven], rec["hash"][proven])

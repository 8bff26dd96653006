"""Pins of the oracle of the paper's GA (oracle/jatam_roulette_oracle.c):
global roulette wheel selection (§2.2, App. C.1), single-point crossover
(App. D.2), Poisson bit-flip mutation (§3.1, App. D.1) and the Fujiyama
test bed (§4.2).

  - the lookup returns the paper's own worked example (App. C.1), stored in
    tests/golden/roulette_lookup_example.txt;
  - selection frequencies follow the roulette law f_i / sum f (chi-square),
    and are uniform when every fitness is zero;
  - the Poisson thresholds equal scipy's Poisson CDF, and the drawn flip
    counts have the Poisson mean, variance and zero-class share;
  - a child is the crossover of its parents at one point: a prefix of one
    parent and the suffix of the other, up to the flipped bits, and flips
    are distinct (Hamming distance = drawn count);
  - on the Fujiyama landscape the population adapts, and discovery comes
    sooner at a higher mutation rate below the error threshold.
"""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "roulette_lookup_example.txt")


def test_lookup_reproduces_the_papers_example():
    fields = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        fields[key] = [int(v) for v in vals]
    assert ref.roulette_lookup(fields["weights"], fields["cutoff"][0]) == fields["index"][0]
    # every cut-off 1..10 lands in the area of its weight
    want = [i for i, w in enumerate(fields["weights"]) for _ in range(w)]
    assert [ref.roulette_lookup(fields["weights"], c) for c in range(1, 11)] == want
    assert ref.roulette_lookup(fields["weights"], 11) == -1


def parents_of(children, pop):
    """Index of each child in pop (children made without crossover or flips)."""
    where = {int(g): i for i, g in enumerate(pop)}
    return np.array([where[int(c)] for c in children])


def test_selection_follows_the_roulette_law():
    n = 8
    pop = np.arange(1, n + 1, dtype=np.uint64) << np.uint64(8)   # distinct genomes
    fit = np.array([0, 1, 2, 3, 5, 8, 13, 0], dtype=np.uint32)
    kids = ref.roulette_offspring(pop, fit, 3, 16, 0.0, crossover=False, n_out=200_000)
    counts = np.bincount(parents_of(kids, pop), minlength=n)
    assert counts[0] == 0 and counts[7] == 0
    expect = fit / fit.sum() * len(kids)
    live = fit > 0
    chi2 = ((counts[live] - expect[live]) ** 2 / expect[live]).sum()
    assert chi2 < stats.chi2.ppf(1 - 1e-6, live.sum() - 1), (counts, expect)


def test_zero_fitness_selects_uniformly():
    n = 10
    pop = np.arange(1, n + 1, dtype=np.uint64) << np.uint64(4)
    kids = ref.roulette_offspring(pop, np.zeros(n, dtype=np.uint32), 0, 16, 0.0,
                                  crossover=False, n_out=100_000)
    counts = np.bincount(parents_of(kids, pop), minlength=n)
    chi2 = ((counts - 10_000) ** 2 / 10_000).sum()
    assert chi2 < stats.chi2.ppf(1 - 1e-6, n - 1)


@pytest.mark.parametrize("lam", [0.1, 0.5, 1.0, 3.0])
def test_poisson_thresholds_and_counts(lam):
    L = 32
    thr = ref.poisson_thresholds(lam, L)
    cdf = stats.poisson.cdf(np.arange(L + 1), lam)
    want = np.minimum(np.floor(cdf * 2.0 ** 32), 2.0 ** 32)
    assert np.all(np.abs(thr.astype(np.float64) - want) <= 1.0)
    # drawn flip counts: a one-genome population, no crossover, the child's
    # distance from the parent is the number of flips
    kids = ref.roulette_offspring(np.zeros(1, dtype=np.uint64), np.ones(1, dtype=np.uint32), 0,
                                  L, lam, crossover=False, n_out=200_000)
    k = np.array([bin(int(x)).count("1") for x in kids])
    se = np.sqrt(lam / len(k))
    assert abs(k.mean() - lam) < 6 * se
    assert abs(k.var() - lam) < 6 * np.sqrt(2 * lam * lam + lam) / np.sqrt(len(k)) + 1e-3
    assert abs(np.mean(k == 0) - np.exp(-lam)) < 6 * np.sqrt(np.exp(-lam) / len(k))


def test_single_point_crossover_structure():
    """Parents all-ones and all-zeros of L bits with equal fitness, no
    mutation: every child is a run of ones followed by zeros or of zeros
    followed by ones, and the crossover points cover 0..L-1 uniformly."""
    L = 20
    ones = (1 << L) - 1
    pop = np.array([ones, 0], dtype=np.uint64)
    kids = ref.roulette_offspring(pop, np.array([1, 1], dtype=np.uint32), 7, L, 0.0,
                                  crossover=True, n_out=50_000)
    prefixes = []
    for x in kids.tolist():
        bits = format(x, f"0{L}b")            # position 0 first
        changes = sum(bits[i] != bits[i + 1] for i in range(L - 1))
        assert changes <= 1, bits
        prefixes.append(len(bits) - len(bits.lstrip(bits[0])) if changes else None)
    # a child that differs from its first parent took a prefix of length p >= 1
    p = np.array([q for q in prefixes if q is not None])
    assert p.min() >= 1 and p.max() <= L - 1
    counts = np.bincount(p, minlength=L)[1:]
    assert counts.min() > 0.5 * counts.mean()


def test_flips_are_distinct_and_within_the_genome():
    L = 12
    kids = ref.roulette_offspring(np.zeros(1, dtype=np.uint64), np.ones(1, dtype=np.uint32), 2,
                                  L, 6.0, crossover=False, n_out=20_000)
    assert np.all(kids >> np.uint64(L) == 0)
    # at lambda = 6 on 12 bits the count is often above half the genome: the
    # distinct-position retry still gives exactly k set bits (mean near 6)
    k = np.array([bin(int(x)).count("1") for x in kids])
    assert abs(k.mean() - 6.0) < 0.15


def test_fujiyama_adapts_and_faster_with_more_mutation():
    """All-zero start, L = 32, target weight 25, population 128: every
    simulation discovers the target, and the median discovery time at
    mu L = 1 is below that at mu L = 0.1 (§4.2: discovery time falls with
    the mutation rate)."""
    times = {}
    for lam in (0.1, 1.0):
        d = [ref.fujiyama(128, 32, lam, 25, 5000, seed=100 + s)[0] for s in range(15)]
        assert min(d) > 0
        times[lam] = np.median(d)
    assert times[1.0] < times[0.1], times
    d, a, final = ref.fujiyama(128, 32, 0.5, 25, 5000, seed=3)
    assert 0 < d <= a
    w = np.array([bin(int(x)).count("1") for x in final])
    assert np.mean(w >= 25) >= 0.5

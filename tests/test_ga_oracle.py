"""Pins of the GA oracle (one generation of tournament selection, uniform
per-edge crossover and per-edge mutation) against closed forms and the
paper's own test bed for its GA, the single-peak 'Fujiyama' landscape of
Hamming weight (§4.2)."""
import math

import numpy as np
import pytest

from oracle import ref


def uniform_genome(colour, t=3):
    g = 0
    for _ in range(4 * t):
        g = (g << 3) | colour
    return g


def edge_colours(genomes, t=3):
    g = genomes.astype(np.uint64)
    return np.stack([(g >> np.uint64(3 * (4 * t - 1 - e))) & np.uint64(7) for e in range(4 * t)],
                    axis=1)


def test_tournament_selection_law():
    """Fitness k for individual k of 8; tournament of 4 with replacement:
    P(winner = k) = ((k+1)^4 - k^4) / 8^4.  Mutation off, so every child edge
    is a parent's colour, each parent drawn by the same law."""
    pop = np.array([uniform_genome(k) for k in range(8)], dtype=np.uint64)
    fit = np.arange(8, dtype=np.int32)
    kids = ref.ga_offspring(pop, fit, 3, generation=0, n_out=200_000, mut=(0, 12), seed=9)
    counts = np.bincount(edge_colours(kids).ravel(), minlength=8)
    total = counts.sum()
    for k in range(8):
        p = ((k + 1) ** 4 - k ** 4) / 8 ** 4
        sigma = math.sqrt(p * (1 - p) * total / 12)   # 12 edges share one child's parents
        assert abs(counts[k] - p * total) < 6 * sigma * 12 ** 0.5, (k, counts[k], p * total)


def test_equal_fitness_selects_uniformly():
    pop = np.array([uniform_genome(k) for k in range(8)], dtype=np.uint64)
    fit = np.zeros(8, dtype=np.int32)
    kids = ref.ga_offspring(pop, fit, 3, generation=3, n_out=100_000, mut=(0, 12), seed=1)
    counts = np.bincount(edge_colours(kids).ravel(), minlength=8) / (12 * 100_000)
    assert np.all(np.abs(counts - 1 / 8) < 0.01)


def test_mutation_rate_and_replacement_colours():
    pop = np.full(16, uniform_genome(3), dtype=np.uint64)
    fit = np.zeros(16, dtype=np.int32)
    kids = ref.ga_offspring(pop, fit, 3, generation=1, n_out=200_000, mut=(1, 12), seed=2)
    cols = edge_colours(kids).ravel()
    changed = cols != 3
    rate = changed.mean()
    assert abs(rate - 1 / 12) < 5 * math.sqrt((1 / 12) * (11 / 12) / cols.size)
    new = np.bincount(cols[changed], minlength=8)
    assert new[3] == 0                       # never "mutates" to the same colour
    share = new[[0, 1, 2, 4, 5, 6, 7]] / changed.sum()
    assert np.all(np.abs(share - 1 / 7) < 0.01)
    # rate 0: children are parents; rate 1: every edge changes
    assert np.all(ref.ga_offspring(pop, fit, 3, 0, n_out=1000, mut=(0, 1)) == pop[0])
    assert np.all(edge_colours(ref.ga_offspring(pop, fit, 3, 0, n_out=1000, mut=(1, 1))) != 3)


def test_uniform_crossover_mixes_edges():
    pop = np.array([uniform_genome(1), uniform_genome(2)], dtype=np.uint64)
    fit = np.zeros(2, dtype=np.int32)
    kids = ref.ga_offspring(pop, fit, 3, generation=0, n_out=100_000, mut=(0, 12), seed=4)
    cols = edge_colours(kids)
    mixed = np.mean((cols == 1).any(axis=1) & (cols == 2).any(axis=1))
    # parents differ with probability 1/2; then all 12 mask bits agree w.p. 2^-11
    assert abs(mixed - 0.5 * (1 - 2.0 ** -11)) < 0.01
    # per edge, each parent's colour half the time
    assert abs((cols == 1).mean() - 0.5) < 0.01


def test_fujiyama_landscape_adapts():
    """§4.2: on the single broad peak of Hamming weight the population climbs
    to the peak (36 set bits for t=3)."""
    rng = np.random.default_rng(0)
    pop = rng.integers(0, 1 << 36, size=512, dtype=np.uint64)

    def hamming(g):
        return np.array([bin(int(x)).count("1") for x in g], dtype=np.int32)

    fit = hamming(pop)
    start = fit.mean()
    for gen in range(60):
        pop = ref.ga_offspring(pop, fit, 3, generation=gen, seed=11)
        fit = hamming(pop)
    assert start < 20 and fit.mean() > 28 and fit.max() >= 34


def test_ga_step_fitness_is_det_size():
    """The generation's fitness is the size of the structure for a
    deterministic offspring, else 0: checked against the brute-force
    explorer (its own decoding and from-scratch options) on the offspring
    whose outcome every growth order fixes (one terminal shape and no event:
    fitness = its cell count; only events reachable: fitness 0)."""
    from tests import brute_force as bf
    rng = np.random.default_rng(8)
    pop = rng.integers(0, 1 << 24, size=300, dtype=np.uint64)
    fit = np.zeros(300, dtype=np.int32)
    nxt, nfit = ref.ga_step(pop, fit, 2, generation=0, grid=16, runs=20)
    checked = {"det": 0, "nd": 0}
    for g, f in zip(nxt.tolist(), nfit.tolist()):
        ex = bf.explore(int(g), 2, 8, 16, cap=800)
        if ex.capped:
            continue
        if ex.truly_det:
            (shape,) = ex.terminals
            assert f == len(shape), g
            checked["det"] += 1
        elif ex.events and not ex.terminals:
            assert f == 0, g
            checked["nd"] += 1
    assert checked["det"] > 25 and checked["nd"] > 25, checked


@pytest.mark.parametrize("bad", [dict(tournament=0), dict(tournament=9), dict(mut=(2, 1)),
                                 dict(mut=(1, 0))])
def test_ga_invalid_params(bad):
    pop = np.zeros(4, dtype=np.uint64)
    fit = np.zeros(4, dtype=np.int32)
    with pytest.raises(ValueError):
        ref.ga_offspring(pop, fit, 3, 0, **bad)

"""The paper's GA on the GPU (roulette selection, single-point crossover,
Poisson bit flips; §2.2, §3.1, App. C.1, D.1, D.2) against the oracle
(oracle/jatam_roulette_oracle.c, pinned in tests/test_roulette_oracle.py):
offspring bit for bit, whole Fujiyama simulations (§4.2) generation by
generation to the same discovery and adaptation times and final
population, and generations with JaTAM fitness (DET size from the
classifier) chained on the device."""
import numpy as np
import pytest

from oracle import ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def jt():
    if not torch.cuda.is_available():
        pytest.fail("gpu test run without a GPU")
    import paper_2205_15311_amd as pkg
    pkg.lib()
    return pkg


def dev64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


@pytest.mark.parametrize("L,lam,cross", [(32, 0.0, True), (32, 0.3, True), (32, 2.5, False),
                                         (64, 1.0, True), (1, 0.5, True), (12, 8.0, True)])
def test_offspring_bit_exact(jt, L, lam, cross):
    rng = np.random.default_rng(L * 10 + int(lam * 10))
    n = 1000
    mask = (1 << L) - 1 if L < 64 else (1 << 64) - 1
    pop = rng.integers(0, 1 << 63, size=n, dtype=np.uint64) & np.uint64(mask)
    fit = rng.integers(0, 41, size=n).astype(np.uint32)
    for gen in (0, 7):
        got = jt.roulette_offspring(dev64(pop), dev32(fit), gen, L, lam, crossover=cross,
                                    seed=11, n_out=3000).cpu().numpy().view(np.uint64)
        want = ref.roulette_offspring(pop, fit, gen, L, lam, crossover=cross, seed=11,
                                      n_out=3000)
        assert np.array_equal(got, want), (gen, np.nonzero(got != want)[0][:5])


def test_offspring_edge_cases(jt):
    # every fitness zero (uniform parents), a single parent, the largest
    # population and fitness
    rng = np.random.default_rng(2)
    pop = rng.integers(0, 1 << 20, size=777, dtype=np.uint64)
    zero = np.zeros(777, dtype=np.uint32)
    got = jt.roulette_offspring(dev64(pop), dev32(zero), 3, 20, 0.7, n_out=2000)
    assert np.array_equal(got.cpu().numpy().view(np.uint64),
                          ref.roulette_offspring(pop, zero, 3, 20, 0.7, n_out=2000))
    one = pop[:1]
    got = jt.roulette_offspring(dev64(one), dev32(np.array([5], np.uint32)), 0, 20, 1.5,
                                n_out=500)
    assert np.array_equal(got.cpu().numpy().view(np.uint64),
                          ref.roulette_offspring(one, np.array([5], np.uint32), 0, 20, 1.5,
                                                 n_out=500))
    big = rng.integers(0, 1 << 30, size=1 << 16, dtype=np.uint64)
    fit = rng.integers(0, 1 << 16, size=1 << 16).astype(np.uint32)
    got = jt.roulette_offspring(dev64(big), dev32(fit), 9, 30, 0.2, n_out=1 << 16)
    assert np.array_equal(got.cpu().numpy().view(np.uint64),
                          ref.roulette_offspring(big, fit, 9, 30, 0.2))
    # no offspring: nothing launched for them
    jt.roulette_offspring(dev64(pop), dev32(zero), 0, 20, 0.7, n_out=0)


@pytest.mark.parametrize("pop,L,target", [(100, 24, 18), (64, 16, 12), (512, 32, 25)])
def test_fujiyama_simulations_match_oracle(jt, pop, L, target):
    lambdas = [0.2, 1.0, 3.0]
    sims, cutoff = 4, 300
    disc, adap, fin = jt.fujiyama(lambdas, sims, pop, L, target, cutoff, seed=40,
                                  final_pop=True)
    disc, adap = disc.cpu().numpy(), adap.cpu().numpy()
    fin = fin.cpu().numpy().view(np.uint64)
    for s in range(sims):
        for k, lam in enumerate(lambdas):
            d, a, f = ref.fujiyama(pop, L, lam, target, cutoff, seed=40 + s)
            assert (disc[s, k], adap[s, k]) == (d, a), (s, lam)
            assert np.array_equal(fin[s, k], f), (s, lam)


def test_jatam_fitness_generations_chain(jt):
    """Three generations of the paper's GA with JaTAM fitness: three-tile
    genomes (L = 36 bits), fitness = DET size at G = 32, R = 20."""
    rng = np.random.default_rng(6)
    n = 4096
    pop = rng.integers(0, 1 << 36, size=n, dtype=np.uint64)
    rec = ref.classify(pop, 3, grid=32, runs=20, seed=1)
    fit = np.where(rec["cls"] == ref.DET, rec["size"], 0).astype(np.uint32)
    dpop, dfit = dev64(pop), dev32(fit)
    for gen in range(3):
        kids = jt.roulette_offspring(dpop, dfit, gen, 36, 0.5, seed=5)
        rec_d = jt.classify(kids, 3, 8, 32, 20, 1)
        dfit = torch.where(rec_d[:, 0] == 3, rec_d[:, 1], torch.zeros_like(rec_d[:, 1]))
        dfit = dfit.contiguous()
        dpop = kids
        pop = ref.roulette_offspring(pop, fit, gen, 36, 0.5, seed=5)
        rec = ref.classify(pop, 3, grid=32, runs=20, seed=1)
        fit = np.where(rec["cls"] == ref.DET, rec["size"], 0).astype(np.uint32)
        assert np.array_equal(dpop.cpu().numpy().view(np.uint64), pop), gen
        assert np.array_equal(dfit.cpu().numpy().view(np.uint32), fit), gen

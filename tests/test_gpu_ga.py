"""Parity of the GPU genetic algorithm with the oracle: offspring genomes and
fitness bit-exact, over chained generations."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("tournament,mut", [(4, (1, 12)), (1, (0, 12)), (8, (1, 1)), (2, (5, 7))])
def test_offspring_bit_exact(jt, tournament, mut):
    rng = np.random.default_rng(tournament)
    n = 65_536
    pop = rng.integers(0, 1 << 36, size=n, dtype=np.uint64)
    fit = rng.integers(0, 40, size=n, dtype=np.int32)
    p = jt.GAParams(seed=5, tournament=tournament, mut_num=mut[0], mut_den=mut[1])
    got = jt.ga_offspring(dev(pop.view(np.int64)), dev(fit), 3, p, generation=17, n_out=4 * n)
    torch.cuda.synchronize()
    want = ref.ga_offspring(pop, fit, 3, generation=17, n_out=4 * n, seed=5,
                            tournament=tournament, mut=mut)
    assert np.array_equal(got.cpu().numpy().view(np.uint64), want)


def test_offspring_other_space(jt):
    rng = np.random.default_rng(3)
    pop = rng.integers(0, 1 << 48, size=1000, dtype=np.uint64)
    fit = rng.integers(0, 3, size=1000, dtype=np.int32)
    p = jt.GAParams(seed=(1 << 40) + 3)
    got = jt.ga_offspring(dev(pop.view(np.int64)), dev(fit), 4, p, generation=2, c=16)
    torch.cuda.synchronize()
    want = ref.ga_offspring(pop, fit, 4, generation=2, c=16, seed=(1 << 40) + 3)
    assert np.array_equal(got.cpu().numpy().view(np.uint64), want)


def test_ga_steps_chain_bit_exact(jt):
    """Three generations, population 8192, t=3, G=32, R=20: every genome and
    fitness equal to the oracle's after each generation."""
    rng = np.random.default_rng(2026)
    n = 8192
    pop = rng.integers(0, 1 << 36, size=n, dtype=np.uint64)
    fit = np.zeros(n, dtype=np.int32)
    p = jt.GAParams(seed=5)
    with jt.Batch(n) as b:
        gpop, gfit = dev(pop.view(np.int64)), dev(fit)
        for gen in range(3):
            gpop, gfit = b.ga_step(gpop, gfit, 3, p, gen, grid_limit=32, runs=20, seed=1)
            pop, fit = ref.ga_step(pop, fit, 3, generation=gen, grid=32, runs=20, seed=1,
                                   ga_seed=5)
            torch.cuda.synchronize()
            assert np.array_equal(gpop.cpu().numpy().view(np.uint64), pop), gen
            assert np.array_equal(gfit.cpu().numpy(), fit), gen
        assert fit.max() > 1

"""Robustness and evolvability on the GPU (§1.1) against the oracle's
(oracle/ref.py neighbourhood, pinned in tests/test_neighbourhood_oracle.py
against the brute-force explorer): the single mutants bit for bit, and
[robust, evolv] per genotype exactly, through both GPU routes - mutants
classified by the batched path, and mutants' records gathered from the
records of a whole space."""
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
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


@pytest.mark.parametrize("t,c", [(1, 8), (2, 8), (3, 8), (2, 4), (4, 16)])
def test_single_mutants_bit_exact(jt, t, c):
    rng = np.random.default_rng(t * 16 + c)
    bits = 4 * t * (c.bit_length() - 1)
    g = rng.integers(0, 1 << min(bits, 63), size=1000, dtype=np.uint64)
    got = jt.single_mutants(dev(g), t, c).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, ref.mutants(g, t, c))
    first = max(0, (1 << min(bits, 40)) - 700) if bits <= 40 else 12345
    got_r = jt.single_mutants(None, t, c, first=first, n=700).cpu().numpy().view(np.uint64)
    assert np.array_equal(got_r, ref.mutants(np.arange(first, first + 700, dtype=np.uint64),
                                             t, c))
    # an empty call launches nothing
    jt.single_mutants(None, t, c, first=0, n=0)


def neighbourhood_by_classification(jt, genomes, t, grid):
    n = len(genomes)
    m = jt.mutant_count(t)
    dg = dev(genomes)
    mut = jt.single_mutants(dg, t)
    with jt.Batch(n * m) as b:
        own = b.classify(dg, t, 8, grid, 20, 1)
        mrec = b.classify(mut.reshape(-1), t, 8, grid, 20, 1)
        out = jt.neighbourhood(own, mrec, t)
        torch.cuda.synchronize()
    return out.cpu().numpy()


def test_s18_whole_space(jt):
    space = jt.classify_range(0, 4096, 1, 8, 16, 20, 1, device="cuda:0")
    got = jt.neighbourhood_space(space, 1).cpu().numpy()
    robust, evolv = ref.neighbourhood(np.arange(4096, dtype=np.uint64), 1)
    assert np.array_equal(got[:, 0], robust)
    assert np.array_equal(got[:, 1], evolv)
    got2 = neighbourhood_by_classification(jt, np.arange(4096, dtype=np.uint64), 1, 16)
    assert np.array_equal(got2, got)


def test_s28_whole_space_and_sample(jt):
    """All of S_{2,8} classified once; a contiguous range of it and a random
    sample (by classifying its mutants) against the oracle."""
    with jt.Batch(1 << 24) as b:
        space = b.classify_range(0, 1 << 24, 2, 8, 16, 20, 1)
        first, n = 9_000_000, 1 << 13
        got = jt.neighbourhood_space(space, 2, first=first, n=n).cpu().numpy()
        full = jt.neighbourhood_space(space, 2)
        torch.cuda.synchronize()
    robust, evolv = ref.neighbourhood(np.arange(first, first + n, dtype=np.uint64), 2)
    assert np.array_equal(got[:, 0], robust)
    assert np.array_equal(got[:, 1], evolv)
    full = full.cpu().numpy()
    assert np.array_equal(full[first:first + n], got)
    assert np.all((full[:, 0] >= 0) & (full[:, 0] <= 24) & (full[:, 1] <= 24 - full[:, 0]))
    rng = np.random.default_rng(3)
    sample = rng.integers(0, 1 << 24, size=1 << 12, dtype=np.uint64)
    got_s = neighbourhood_by_classification(jt, sample, 2, 16)
    assert np.array_equal(got_s, full[sample.astype(np.int64)])
    robust, evolv = ref.neighbourhood(sample[:1024], 2)
    assert np.array_equal(got_s[:1024, 0], robust)
    assert np.array_equal(got_s[:1024, 1], evolv)


def test_three_tile_sample_grid32(jt):
    rng = np.random.default_rng(5)
    g = rng.integers(0, 1 << 36, size=1500, dtype=np.uint64)
    got = neighbourhood_by_classification(jt, g, 3, 32)
    robust, evolv = ref.neighbourhood(g, 3, grid=32)
    assert np.array_equal(got[:, 0], robust)
    assert np.array_equal(got[:, 1], evolv)

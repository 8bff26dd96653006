"""The GPU true class (every growth order followed, §3.2 and §4.1) against
the oracle's exhaustive exploration, which tests/test_true_class_oracle.py
pins against the independent brute-force explorer (tests/brute_force.py).

Class, size and hash are compared on every genotype the oracle decides
(the `steps` field counts states in each side's own visiting order and is
not compared; a genotype the oracle leaves undecided past its cap is
skipped).  Also checked: soundness against the R-run classifier (a true DET
genotype is classed DET by the classifier with the same size and hash) and
the undecided path (a cap too small for the search)."""
import numpy as np
import pytest

from oracle import ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CAP = 1 << 20


@pytest.fixture(scope="module")
def jt():
    if not torch.cuda.is_available():
        pytest.fail("gpu test run without a GPU")
    import paper_2205_15311_amd as pkg
    pkg.lib()
    return pkg


@pytest.fixture(scope="module")
def truth(jt):
    with jt.Truth(1 << 18, max_level=4096, waves=64) as w:
        yield w


def records(rec):
    torch.cuda.synchronize()
    return rec.cpu().numpy().view(ref.RECORD).reshape(-1)


def compare(got, want, genomes, label):
    decided = want["cls"] != ref.TRUE_CAPPED
    assert np.all(got["cls"][decided] != ref.TRUE_CAPPED), label
    for f in ("cls", "size", "hash"):
        bad = np.nonzero(decided & (got[f] != want[f]))[0]
        assert len(bad) == 0, (label, f, [(int(genomes[i]), tuple(got[i]), tuple(want[i]))
                                          for i in bad[:5]])
    return int(decided.sum())


def test_true_class_of_s18(jt, truth):
    got = records(truth.true_class_range(0, 4096, 1, grid_limit=16, cap=CAP))
    want = ref.true_class(np.arange(4096, dtype=np.uint64), 1, grid=16, cap=CAP)
    assert compare(got, want, np.arange(4096), "S_1,8") == 4096


def test_true_class_of_s28_candidates_and_sample(jt, truth):
    """Genotypes the classifier calls DET after choosing between sites (the
    ones a few runs can get wrong, and the ones the explorer takes), plus a
    uniform sample."""
    rng = np.random.default_rng(31)
    pool = rng.integers(0, 1 << 24, size=1 << 17, dtype=np.uint64)
    rec = ref.classify(pool, 2, grid=16, runs=20, seed=1)
    cand = pool[(rec["cls"] == ref.DET) & (rec["steps"] == (rec["size"] - 1) * 20)
                & (rec["size"] >= 3)]
    g = np.concatenate([cand, pool[:8192]])
    got = records(truth.true_class(torch.from_numpy(g.view(np.int64)).cuda(), 2, cap=CAP))
    want = ref.true_class(g, 2, grid=16, cap=CAP)
    assert compare(got, want, g, "S_2,8 sample") == len(g)
    # some genotypes needed the exhaustive search, some of them are not DET
    assert np.any(got["steps"] > 0)
    assert np.any((got["steps"] > 0) & (got["cls"] == ref.ND_SITE))


def test_true_class_of_a_contiguous_s28_slice(jt, truth):
    first, n = 11 << 20, 1 << 16
    got = records(truth.true_class_range(first, n, 2, cap=CAP))
    want = ref.true_class(np.arange(first, first + n, dtype=np.uint64), 2, grid=16, cap=CAP)
    assert compare(got, want, np.arange(first, first + n), "S_2,8 slice") == n


def test_true_class_three_tiles_grid32(jt, truth):
    rng = np.random.default_rng(77)
    pool = rng.integers(0, 1 << 36, size=1 << 14, dtype=np.uint64)
    rec = ref.classify(pool, 3, grid=32, runs=20, seed=1)
    g = np.concatenate([pool[rec["cls"] == ref.DET], pool[:2048]])
    got = records(truth.true_class(torch.from_numpy(g.view(np.int64)).cuda(), 3,
                                   grid_limit=32, cap=CAP))
    want = ref.true_class(g, 3, grid=32, cap=CAP)
    assert compare(got, want, g, "three tiles G=32") >= len(g) - 8


def test_true_det_is_classified_det_with_the_same_shape(jt, truth):
    first, n = 3 << 20, 1 << 18
    tr = records(truth.true_class_range(first, n, 2, cap=CAP))
    cl = ref.classify_range(first, n, 2, grid=16, runs=20, seed=1)
    det = tr["cls"] == ref.DET
    assert det.sum() > 1000
    assert np.all(cl["cls"][det] == ref.DET)
    assert np.array_equal(cl["size"][det], tr["size"][det])
    assert np.array_equal(cl["hash"][det], tr["hash"][det])
    # and a genotype with a witness run is never truly deterministic
    assert not np.any(det & (cl["cls"] != ref.DET))


def test_small_cap_leaves_the_search_undecided(jt):
    """Genotypes whose search needs more than `cap` states come back
    UNDECIDED; the others are unchanged, and the workspace is clean for the
    next call."""
    rng = np.random.default_rng(31)
    pool = rng.integers(0, 1 << 24, size=1 << 16, dtype=np.uint64)
    rec = ref.classify(pool, 2, grid=16, runs=20, seed=1)
    g = pool[(rec["cls"] == ref.DET) & (rec["steps"] == (rec["size"] - 1) * 20)
             & (rec["size"] >= 3)]
    dg = torch.from_numpy(g.view(np.int64)).cuda()
    with jt.Truth(len(g), max_level=64, waves=8) as w:
        full = records(w.true_class(dg, 2, cap=CAP))
        small = records(w.true_class(dg, 2, cap=3))
        again = records(w.true_class(dg, 2, cap=CAP))
    explored = full["steps"] > 3
    assert np.any(explored)
    assert np.all(small["cls"][explored] == ref.TRUE_CAPPED)
    assert np.array_equal(small[~explored], full[~explored])
    assert np.array_equal(again, full)

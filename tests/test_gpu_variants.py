"""Classification variants on the GPU against the oracle's
(oracle/jatam_oracle.c, pinned in tests/test_variant_oracle.py): the C4
shape hash (§3.3) and the LIFO movelist traversal (§3.2), apart and
together, record for record."""
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


def records(rec):
    torch.cuda.synchronize()
    return rec.cpu().numpy().view(ref.RECORD).reshape(-1)


def same(got, want, label):
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (label, bad[:5], got[bad[:3]], want[bad[:3]])


VARIANTS = [1, 2, 3]


@pytest.mark.parametrize("variant", VARIANTS)
def test_s18_whole_space(jt, variant):
    got = records(jt.classify_variant(None, 1, variant, first=0, n=4096))
    same(got, ref.classify_variant(None, 1, variant, first=0, n=4096), variant)


@pytest.mark.parametrize("variant", VARIANTS)
def test_s28_sample_and_range(jt, variant):
    rng = np.random.default_rng(40 + variant)
    g = rng.integers(0, 1 << 24, size=1 << 14, dtype=np.uint64)
    dg = torch.from_numpy(g.view(np.int64)).cuda()
    same(records(jt.classify_variant(dg, 2, variant)), ref.classify_variant(g, 2, variant),
         variant)
    first = (1 << 24) - 5000   # a ragged tail at the end of the space
    same(records(jt.classify_variant(None, 2, variant, first=first, n=5000)),
         ref.classify_variant(None, 2, variant, first=first, n=5000), variant)


@pytest.mark.parametrize("variant,grid", [(1, 32), (1, 20), (2, 16), (3, 12), (2, 10)])
def test_three_tiles(jt, variant, grid):
    rng = np.random.default_rng(grid * 4 + variant)
    g = rng.integers(0, 1 << 36, size=3000, dtype=np.uint64)
    dg = torch.from_numpy(g.view(np.int64)).cuda()
    same(records(jt.classify_variant(dg, 3, variant, grid_limit=grid)),
         ref.classify_variant(g, 3, variant, grid=grid), (variant, grid))


def test_no_variant_is_the_plain_path(jt):
    rng = np.random.default_rng(5)
    g = rng.integers(0, 1 << 24, size=4096, dtype=np.uint64)
    dg = torch.from_numpy(g.view(np.int64)).cuda()
    same(records(jt.classify_variant(dg, 2, 0)), records(jt.classify(dg, 2)), 0)


def test_lifo_needs_the_small_layout(jt):
    dg = torch.zeros(4, dtype=torch.int64, device="cuda")
    with pytest.raises(jt.JatamError):
        jt.classify_variant(dg, 2, jt.VARIANT_LIFO, grid_limit=32)

"""The device tallies: class counts and the histogram of DET shapes
(jatam_shape_histogram), against counts of oracle records."""
import json
import os

import numpy as np
import pytest

from oracle import ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def jt():
    if not torch.cuda.is_available():
        pytest.fail("gpu test run without a GPU")
    import paper_2205_15311_amd as pkg
    pkg.lib()
    return pkg


def expected_shapes(recs):
    det = recs[recs["cls"] == ref.DET]
    pairs = np.stack([det["size"].astype(np.int64), det["hash"].astype(np.int64)])
    if pairs.shape[1] == 0:
        return []
    keys, counts = np.unique(pairs, axis=1, return_counts=True)
    return [(int(h), int(z), int(c)) for (z, h), c in zip(keys.T, counts)]


def got_shapes(jt, table):
    arr = jt.shape_table_to_numpy(table)
    return [(int(e["hash"]), int(e["size"]), int(e["count"])) for e in arr]


def to_dev(recs):
    return torch.from_numpy(np.ascontiguousarray(recs).view(np.int32).reshape(-1, 4)).cuda()


def test_histogram_of_oracle_records(jt):
    """S_{1,8} in full, a sample of S_{2,8} and of the three-tile space at
    G=32: the table holds exactly the oracle records' (hash, size) counts."""
    rng = np.random.default_rng(8)
    parts = [ref.classify_range(0, 4096, 1, grid=16, runs=20, seed=1),
             ref.classify(rng.integers(0, 1 << 24, size=1 << 16, dtype=np.uint64), 2, grid=16),
             ref.classify(rng.integers(0, 1 << 36, size=1 << 14, dtype=np.uint64), 3, grid=32)]
    recs = np.concatenate(parts)
    table = jt.shape_histogram(to_dev(recs), capacity=4096)
    torch.cuda.synchronize()
    assert got_shapes(jt, table) == expected_shapes(recs)


def test_histogram_accumulates_over_slices(jt):
    rng = np.random.default_rng(9)
    recs = ref.classify(rng.integers(0, 1 << 24, size=1 << 15, dtype=np.uint64), 2, grid=16)
    dev = to_dev(recs)
    table = torch.zeros((1024, 2), dtype=torch.int64, device="cuda")
    for lo in range(0, len(recs), 5000):
        jt.shape_histogram(dev[lo:lo + 5000], table)
    torch.cuda.synchronize()
    assert got_shapes(jt, table) == expected_shapes(recs)


def test_histogram_many_keys_and_overflow(jt):
    """Synthetic records: 3000 distinct shapes, a few of them very frequent
    (the contended case); then the same records into a table too small for
    them, where every DET record is either counted or reported lost."""
    rng = np.random.default_rng(10)
    n = 1 << 20
    recs = np.zeros(n, dtype=ref.RECORD)
    recs["cls"] = rng.integers(-1, 4, size=n)
    keys = rng.integers(0, 1 << 32, size=3000, dtype=np.uint64)
    pick = np.where(rng.random(n) < 0.8, rng.integers(0, 3, size=n), rng.integers(0, 3000, size=n))
    recs["hash"] = keys[pick].astype(np.uint32)
    recs["size"] = 1 + (pick % 7)
    dev = to_dev(recs)
    table = jt.shape_histogram(dev, capacity=8192)
    torch.cuda.synchronize()
    want = expected_shapes(recs)
    assert got_shapes(jt, table) == want

    small = torch.zeros((1024, 2), dtype=torch.int64, device="cuda")
    lost = torch.zeros(1, dtype=torch.int64, device="cuda")
    jt.shape_histogram(dev, small, overflow=lost)
    torch.cuda.synchronize()
    got = got_shapes(jt, small)
    assert len(got) == 1024                                  # every entry used
    exact = {(h, z): c for h, z, c in want}
    assert all(exact[(h, z)] == c for h, z, c in got)       # no partial counts lost
    assert sum(c for _, _, c in got) + int(lost.item()) == int(np.sum(recs["cls"] == ref.DET))


def test_s28_tally_and_shapes_from_one_batched_call(jt):
    """All of S_{2,8}: the batched call's device tally and the histogram of
    its records equal the oracle's (tests/golden/s28_digests.json)."""
    with open(os.path.join(HERE, "golden", "s28_digests.json")) as f:
        gold = json.load(f)
    tally = torch.zeros(4, dtype=torch.int64, device="cuda")
    with jt.Batch(1 << 24) as b:
        rec = b.classify_range(0, 1 << 24, 2, 8, 16, 20, 1, tally=tally)
        table = jt.shape_histogram(rec, capacity=256)
        torch.cuda.synchronize()
    assert tally.cpu().tolist() == gold["tally"]
    assert got_shapes(jt, table) == [(s["hash"], s["size"], s["count"]) for s in gold["shapes"]]

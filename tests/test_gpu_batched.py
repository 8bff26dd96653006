"""Parity of the pipelined (batched) path with the CPU oracle, through the C
ABI: same records as the plain kernel, bit for bit, whatever the queue order,
slice size or mix of tile counts and grids."""
import hashlib
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


@pytest.fixture(scope="module")
def batch(jt):
    b = jt.Batch(1 << 24)
    yield b
    b.close()


def records(rec):
    torch.cuda.synchronize()
    return rec.cpu().numpy().view(ref.RECORD).reshape(-1)


def assert_same(got, want, label):
    bad = np.nonzero(got != want)[0]
    if len(bad):
        lines = [f"{label}: {len(bad)} of {len(want)} records differ"]
        for i in bad[:8]:
            lines.append(f"  [{i}] gpu={tuple(got[i])} oracle={tuple(want[i])}")
        pytest.fail("\n".join(lines))


def tally_of(recs):
    return [int(np.sum(recs["cls"] == k)) for k in range(4)]


def test_s18_batched(jt, batch):
    tally = torch.zeros(4, dtype=torch.int64, device="cuda")
    got = records(batch.classify_range(0, 4096, 1, 8, 16, 20, 1, tally=tally))
    want = ref.classify_range(0, 4096, 1, grid=16, runs=20, seed=1)
    assert_same(got, want, "S_{1,8} batched")
    assert tally.cpu().tolist() == tally_of(want)


def test_s28_batched_one_call(jt, batch):
    """All 2^24 genotypes of S_{2,8} in a single pipelined call; every 2^20
    slice of records hashed and compared with the oracle's digest."""
    with open(os.path.join(HERE, "golden", "s28_digests.json")) as f:
        gold = json.load(f)
    tally = torch.zeros(4, dtype=torch.int64, device="cuda")
    rec = batch.classify_range(0, 1 << 24, 2, 8, 16, 20, 1, tally=tally)
    got = records(rec)
    for s in gold["slices"]:
        part = got[s["first"]:s["first"] + s["n"]]
        if hashlib.sha256(part.tobytes()).hexdigest() != s["sha256"]:
            want = ref.classify_range(s["first"], s["n"], 2, grid=16, runs=20, seed=1)
            assert_same(part, want, f"S_{{2,8}} slice at {s['first']}")
            pytest.fail("digest mismatch without a record mismatch")
    assert tally.cpu().tolist() == gold["tally"]


@pytest.mark.parametrize("t,grid,runs", [(2, 16, 20), (3, 16, 20), (3, 32, 20), (2, 32, 20),
                                         (4, 16, 5), (2, 16, 1), (2, 16, 2), (2, 16, 64),
                                         (3, 10, 33), (1, 8, 20)])
def test_batched_random_lists(jt, batch, t, grid, runs):
    rng = np.random.default_rng(7 * t + grid + runs)
    n = 30_000 if grid <= 16 else 8_000
    gs = rng.integers(0, 1 << (12 * t), size=n, dtype=np.uint64)
    got = records(batch.classify(torch.from_numpy(gs.view(np.int64)).cuda(), t, 8, grid, runs, 1))
    assert_same(got, ref.classify(gs, t, grid=grid, runs=runs, seed=1), f"t={t} G={grid} R={runs}")


def test_batched_mixed_items(jt, batch):
    """Items of mixed tile count (1..3) and grid (16, 32) in one call, some
    with their own rng_id, one invalid."""
    rng = np.random.default_rng(2026)
    n = 20_000
    t = rng.integers(1, 4, size=n)
    grid = np.where(rng.random(n) < 0.5, 16, 32)
    gs = rng.integers(0, 1 << 36, size=n, dtype=np.uint64) >> (36 - 12 * t).astype(np.uint64)
    rid = gs | (t.astype(np.uint64) << np.uint64(56))
    rid[::5] ^= rng.integers(0, 1 << 40, size=rid[::5].shape[0], dtype=np.uint64)
    items = jt.make_items(gs, t, grid, rid)
    items[17, 16] = 9   # t = 9: outside the limits
    dev = torch.from_numpy(items).cuda()
    got = records(batch.classify_items(dev, 8, 20, 1))
    ok = np.ones(n, bool)
    ok[17] = False
    want_items = np.zeros(n, dtype=ref.ITEM)
    want_items["genome"], want_items["rng_id"] = gs, rid
    want_items["t"], want_items["grid"] = t, grid
    want = np.zeros(n, dtype=ref.RECORD)
    want[ok] = ref.classify_items(want_items[ok], c=8, runs=20, seed=1)
    want[~ok] = (-1, 0, 0, 0)
    assert_same(got, want, "mixed items")


@pytest.mark.parametrize("n", [0, 1, 2, 63, 65, 1000, 4097])
def test_batched_ragged(jt, batch, n):
    first = 9_000_000
    got = records(batch.classify_range(first, n, 2, 8, 16, 20, 1))
    if n:
        assert_same(got, ref.classify_range(first, n, 2, grid=16, runs=20, seed=1), f"n={n}")


def test_batched_equals_plain_on_three_tiles(jt, batch):
    """A 2^20 slice of S_{3,8} at G=32 through both paths; and the workspace
    reused right after for a smaller call."""
    first = 12_345_678_901      # < 8^12 - 2^20
    n = 1 << 20
    plain = records(jt.classify_range(first, n, 3, 8, 32, 20, 1))
    piped = records(batch.classify_range(first, n, 3, 8, 32, 20, 1))
    assert_same(piped, plain, "batched vs plain, S_{3,8} G=32")
    sample = np.random.default_rng(3).choice(n, 3000, replace=False)
    want = ref.classify(np.uint64(first) + sample.astype(np.uint64), 3, grid=32, runs=20, seed=1)
    assert_same(plain[sample], want, "sampled oracle")
    small = records(batch.classify_range(first, 1000, 3, 8, 32, 20, 1))
    assert_same(small, plain[:1000], "reused workspace")


def test_batched_argument_errors(jt, batch):
    with pytest.raises(jt.JatamError):
        batch.classify_range(0, (1 << 24) + 1, 3, 8, 16, 20, 1)   # beyond max_n
    with pytest.raises(jt.JatamError):
        batch.classify_range(0, 10, 2, 8, 40, 20, 1)              # unsupported grid
    with pytest.raises(jt.JatamError):
        batch.classify_range((1 << 24) - 5, 10, 2, 8, 16, 20, 1)  # beyond the space


def test_stage_timing_hook(jt, batch):
    batch.set_timing(True)
    batch.classify_range(0, 1 << 16, 2, 8, 16, 20, 1)
    batch.classify_range(0, 1 << 16, 2, 8, 16, 20, 1)
    times = batch.stage_times()
    batch.set_timing(False)
    assert times["first_run_kernel<16>"][1] == 2 and times["repeat_kernel<16>"][1] == 2
    assert all(ms >= 0 for ms, _ in times.values())


def test_refill_threshold_does_not_change_records(jt, batch):
    rng = np.random.default_rng(77)
    gs = rng.integers(0, 1 << 24, size=50_000, dtype=np.uint64)
    dev = torch.from_numpy(gs.view(np.int64)).cuda()
    want = ref.classify(gs, 2, grid=16, runs=20, seed=1)
    try:
        for refill in (1, 5, 33, 64):
            batch.set_refill(refill)
            got = records(batch.classify(dev, 2, 8, 16, 20, 1))
            assert_same(got, want, f"refill={refill}")
    finally:
        batch.set_refill(24)


@pytest.mark.parametrize("grid", [16, 32])
def test_rare_paths_three_tiles(jt, batch, grid):
    """400k random three-tile genotypes: enough to contain ND_RUNS genotypes
    and DET shapes of 20-33 cells (bounding boxes beyond 8 x 8), through both
    paths."""
    rng = np.random.default_rng(123 + grid)
    gs = rng.integers(0, 1 << 36, size=400_000, dtype=np.uint64)
    want = ref.classify(gs, 3, grid=grid, runs=20, seed=1)
    assert np.sum(want["cls"] == ref.ND_RUNS) > 10
    assert np.sum((want["cls"] == ref.DET) & (want["size"] >= 20)) > 10
    dev = torch.from_numpy(gs.view(np.int64)).cuda()
    assert_same(records(batch.classify(dev, 3, 8, grid, 20, 1)), want, f"batched G={grid}")
    assert_same(records(jt.classify(dev, 3, 8, grid, 20, 1)), want, f"plain G={grid}")

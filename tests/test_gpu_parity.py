"""Parity of the HIP path with the CPU oracle, through the C ABI.

Every record (class, size, shape hash, steps) must be bit-identical.  Full
spaces are compared against digests written by tests/golden/make_golden.py
from the oracle; everything else against the oracle run here on the same
seeded inputs.
"""
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
    pkg.lib()   # raises if the HIP library is missing: no fallback
    return pkg


def gpu_records(rec):
    torch.cuda.synchronize()
    return rec.cpu().numpy().view(ref.RECORD).reshape(-1)


def assert_same(got, want, label):
    bad = np.nonzero(got != want)[0]
    if len(bad):
        lines = [f"{label}: {len(bad)} of {len(want)} records differ"]
        for i in bad[:8]:
            lines.append(f"  [{i}] gpu={tuple(got[i])} oracle={tuple(want[i])}")
        pytest.fail("\n".join(lines))


def test_s18_all_genotypes(jt):
    """All 4096 single-tile genotypes, G=16, R=20, seed 1."""
    got = gpu_records(jt.classify_range(0, 4096, 1, 8, 16, 20, 1))
    assert_same(got, ref.classify_range(0, 4096, 1, grid=16, runs=20, seed=1), "S_{1,8}")
    with open(os.path.join(HERE, "golden", "s18_digests.json")) as f:
        gold = json.load(f)
    assert hashlib.sha256(got.tobytes()).hexdigest() == gold["slices"][0]["sha256"]


def test_s28_all_genotypes_by_digest(jt):
    """All 2^24 two-tile genotypes in 16 range launches of 2^20 (the plain
    kernel's launch configuration), each slice's records hashed and compared
    with the oracle's digest."""
    with open(os.path.join(HERE, "golden", "s28_digests.json")) as f:
        gold = json.load(f)
    n = gold["slice"]
    out = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    for s in gold["slices"]:
        jt.classify_range(s["first"], s["n"], 2, 8, 16, 20, 1, out=out)
        got = gpu_records(out)
        if hashlib.sha256(got.tobytes()).hexdigest() != s["sha256"]:
            want = ref.classify_range(s["first"], s["n"], 2, grid=16, runs=20, seed=1)
            assert_same(got, want, f"S_{{2,8}} slice at {s['first']}")
            pytest.fail("digest mismatch without a record mismatch")
        assert [int(np.sum(got["cls"] == k)) for k in range(4)] == s["tally"]


@pytest.mark.parametrize("t,grid", [(1, 8), (2, 16), (3, 16), (4, 16), (2, 32), (3, 32),
                                    (2, 10), (3, 24), (1, 32)])
def test_random_genotypes(jt, t, grid):
    rng = np.random.default_rng(1000 + 10 * t + grid)
    n = 20_000 if grid <= 16 else 6_000
    gs = rng.integers(0, 1 << (12 * t), size=n, dtype=np.uint64)
    dev = torch.from_numpy(gs.view(np.int64)).cuda()
    got = gpu_records(jt.classify(dev, t, 8, grid, 20, 1))
    assert_same(got, ref.classify(gs, t, grid=grid, runs=20, seed=1), f"t={t} G={grid}")


@pytest.mark.parametrize("grid", [18, 22, 26, 30])
def test_wide_layout_long_runs(jt, grid):
    """Grids of 17 < G < 32 run in the 32 x 32 layout, whose frontier select
    keeps per-group counts of four rows: genotypes whose runs place many
    tiles (UNBOUND runs that fill the box, large DET shapes) put frontier
    sites in every group and across group edges.  The sample is the
    three-tile genotypes of a seeded draw whose oracle record has at least
    40 placements, plus as many ordinary ones."""
    rng = np.random.default_rng(4100 + grid)
    gs = rng.integers(0, 1 << 36, size=40_000, dtype=np.uint64)
    want = ref.classify(gs, 3, grid=grid, runs=20, seed=1)
    long = np.nonzero(want["steps"] >= 40)[0][:3000]
    assert len(long) >= 200, f"only {len(long)} long runs at G={grid}"
    pick = np.concatenate([long, np.arange(len(long))])
    sub = np.ascontiguousarray(gs[pick])
    dev = torch.from_numpy(sub.view(np.int64)).cuda()
    got = gpu_records(jt.classify(dev, 3, 8, grid, 20, 1))
    assert_same(got, want[pick], f"plain G={grid}")
    with jt.Batch(len(sub)) as b:
        got = gpu_records(b.classify(dev, 3, 8, grid, 20, 1))
    assert_same(got, want[pick], f"batched G={grid}")


@pytest.mark.parametrize("runs,seed", [(1, 1), (7, 123456789), (64, (1 << 63) + 5)])
def test_runs_and_seeds(jt, runs, seed):
    rng = np.random.default_rng(runs)
    gs = rng.integers(0, 1 << 24, size=8_000, dtype=np.uint64)
    dev = torch.from_numpy(gs.view(np.int64)).cuda()
    got = gpu_records(jt.classify(dev, 2, 8, 16, runs, seed))
    assert_same(got, ref.classify(gs, 2, grid=16, runs=runs, seed=seed), f"R={runs}")


@pytest.mark.parametrize("c,t", [(2, 4), (4, 3), (16, 2), (16, 4)])
def test_other_colour_counts(jt, c, t):
    bits = 4 * t * (c.bit_length() - 1)
    rng = np.random.default_rng(c * 10 + t)
    hi = 1 << min(bits, 63)
    gs = rng.integers(0, hi, size=6_000, dtype=np.uint64)
    if bits == 64:
        gs |= rng.integers(0, 2, size=gs.shape[0], dtype=np.uint64) << np.uint64(63)
    dev = torch.from_numpy(gs.view(np.int64)).cuda()
    got = gpu_records(jt.classify(dev, t, c, 16, 20, 1))
    assert_same(got, ref.classify(gs, t, c=c, grid=16, runs=20, seed=1), f"c={c} t={t}")


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 255, 257, 1000])
def test_ragged_sizes(jt, n):
    first = 5_000_000
    rec = jt.classify_range(first, n, 2, 8, 16, 20, 1)
    got = gpu_records(rec)
    if n:
        assert_same(got, ref.classify_range(first, n, 2, grid=16, runs=20, seed=1), f"n={n}")


def test_slicing_does_not_change_records(jt):
    first, n = 3 << 20, 50_000
    whole = gpu_records(jt.classify_range(first, n, 2, 8, 16, 20, 1))
    parts, at = [], 0
    for size in (1, 999, 4097, 12_345, n - 1 - 999 - 4097 - 12_345):
        parts.append(gpu_records(jt.classify_range(first + at, size, 2, 8, 16, 20, 1)))
        at += size
    assert_same(np.concatenate(parts), whole, "sliced")
    # list mode in shuffled order gives the same records
    perm = np.random.default_rng(0).permutation(n)
    gs = (first + perm).astype(np.uint64)
    shuf = gpu_records(jt.classify(torch.from_numpy(gs.view(np.int64)).cuda(), 2, 8, 16, 20, 1))
    assert_same(shuf, whole[perm], "shuffled")


def test_stray_genome_bits_give_invalid_records(jt):
    gs = np.array([5, (1 << 24) | 5, 1 << 63, 77], dtype=np.uint64)
    got = gpu_records(jt.classify(torch.from_numpy(gs.view(np.int64)).cuda(), 2, 8, 16, 20, 1))
    assert tuple(got[1]) == (jt.INVALID, 0, 0, 0) and tuple(got[2]) == (jt.INVALID, 0, 0, 0)
    want = ref.classify(gs[[0, 3]], 2, grid=16)
    assert_same(got[[0, 3]], want, "valid neighbours")


def test_three_tile_space_slice_and_sample(jt):
    """S_{3,8} at G=32: a contiguous lexicographic slice at a seeded offset
    and a uniform sample (the three-tile workload at reduced size)."""
    rng = np.random.default_rng(11)
    first = int(rng.integers(0, (1 << 36) - (1 << 14)))
    got = gpu_records(jt.classify_range(first, 1 << 14, 3, 8, 32, 20, 1))
    assert_same(got, ref.classify_range(first, 1 << 14, 3, grid=32, runs=20, seed=1), "slice")
    gs = rng.integers(0, 1 << 36, size=1 << 14, dtype=np.uint64)
    got = gpu_records(jt.classify(torch.from_numpy(gs.view(np.int64)).cuda(), 3, 8, 32, 20, 1))
    assert_same(got, ref.classify(gs, 3, grid=32, runs=20, seed=1), "sample")


def test_largest_supported_grid_and_runs(jt):
    rng = np.random.default_rng(64)
    gs = rng.integers(0, 1 << 36, size=3000, dtype=np.uint64)
    got = gpu_records(jt.classify(torch.from_numpy(gs.view(np.int64)).cuda(), 3, 8, 32, 64, 9))
    assert_same(got, ref.classify(gs, 3, grid=32, runs=64, seed=9), "G=32 R=64")

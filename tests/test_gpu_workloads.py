"""The larger workloads at their full sizes, through the C ABI, in the launch
configuration the library uses for them (one pipelined call per slice).

Parity here is on stratified subsets of 2^22 records each, compared with the
oracle's records of the same inputs through tests/golden/workload_strata.json
(per-2^18-record SHA-256 digests written by tests/golden/make_strata.py,
which calls only the oracle; a differing chunk is re-run on the oracle here
and its differing records are printed): every (t, G) stratum of the mixed
stream, every 256th genotype of the 2^30 slice, every 64th of the 2^28
sample.  Also on every record of a class of inputs small enough to enumerate
(one-tile items) and on properties that hold at any size:
  - the device tally equals the class counts of the records;
  - a non-DET record has hash 0; a DET record has size >= 1 and
    steps = (size - 1) * R, or size - 1 when run 0 drew no random word
    (its runs are then identical, §3.2);
  - equal items (genome, t, grid, rng_id) give equal records.
Inputs: tests/inputs.py (numpy's Philox generator, seeded)."""
import hashlib
import json
import os
import time

import numpy as np
import pytest

from oracle import ref
from tests import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = 20
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def strata():
    with open(os.path.join(HERE, "golden", "workload_strata.json")) as f:
        return json.load(f)


def check_stratum(recs, gold, oracle_chunk, label):
    """recs: the GPU's records of a stratum; gold: its digests and tally;
    oracle_chunk(lo, hi): the oracle's records of positions lo..hi-1, run
    only for a chunk whose digest differs."""
    assert len(recs) == gold["n"], label
    ch = gold["chunk"]
    for k, want in enumerate(gold["sha256"]):
        part = recs[k * ch:(k + 1) * ch]
        if hashlib.sha256(part.tobytes()).hexdigest() != want:
            assert_same(part, oracle_chunk(k * ch, (k + 1) * ch), f"{label} chunk {k}")
            pytest.fail(f"{label} chunk {k}: digest differs, records equal the oracle's")
    assert [int(np.sum(recs["cls"] == k)) for k in range(4)] == gold["tally"], label


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


def assert_same(got, want, label):
    bad = np.nonzero(got != want)[0]
    if len(bad):
        lines = [f"{label}: {len(bad)} of {len(want)} records differ"]
        for i in bad[:8]:
            lines.append(f"  [{i}] gpu={tuple(got[i])} oracle={tuple(want[i])}")
        pytest.fail("\n".join(lines))


def check_properties(recs, tally, label):
    cls = recs["cls"]
    assert np.all((cls >= ref.UNBOUND) & (cls <= ref.DET)), label
    assert tally == [int(np.count_nonzero(cls == k)) for k in range(4)], label
    assert np.all(recs["hash"][cls != ref.DET] == 0), label
    det = recs[cls == ref.DET]
    assert np.all(det["size"] >= 1), label
    placed = det["size"].astype(np.int64) - 1
    ok = (det["steps"] == placed) | (det["steps"] == placed * R)
    assert np.all(ok), (label, det[~ok][:4])


def test_mixed_stream_2e26_one_call(jt, strata):
    """2^26 items of 1-3 tiles on 16x16 or 32x32 grids in ONE call.  Every
    one-tile record (about a third) is checked against the oracle, since the
    4096 x 2 distinct one-tile items are few; the first 2^22 items of each
    (t, G) stratum against the oracle's digests."""
    n = 1 << 26
    g, t, grid = inputs.mixed_stream(n)
    items = jt.make_items(g, t, grid)
    dev = torch.from_numpy(items).cuda()
    del items
    tally = torch.zeros(4, dtype=torch.int64, device="cuda")
    with jt.Batch(n) as b:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = b.classify_items(dev, 8, R, 1, tally=tally)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    print(f"mixed stream: {n / dt / 1e6:.1f} M items/s ({dt:.2f} s)", flush=True)
    del dev
    recs = records(rec)
    del rec
    check_properties(recs, tally.cpu().tolist(), "mixed stream")

    # every one-tile item
    one = np.nonzero(t == 1)[0]
    uniq = np.arange(4096, dtype=np.uint64)
    for G in (16, 32):
        want = ref.classify(uniq, 1, grid=G, runs=R, seed=1)
        sel = one[grid[one] == G]
        assert_same(recs[sel], want[g[sel].astype(np.int64)], f"one-tile items, G={G}")

    # 2^22 items of every (t, G) stratum
    assert strata["mixed"]["total"] == n
    for tt in (1, 2, 3):
        for G in (16, 32):
            gold = strata["mixed"]["strata"][f"t{tt}_g{G}"]
            idx = np.nonzero((t == tt) & (grid == G))[0][:gold["n"]]

            def oracle_chunk(lo, hi, idx=idx):
                sel = idx[lo:hi]
                it = np.zeros(len(sel), dtype=ref.ITEM)
                it["genome"], it["t"], it["grid"] = g[sel], t[sel], grid[sel]
                it["rng_id"] = g[sel] | (t[sel].astype(np.uint64) << np.uint64(56))
                return ref.classify_items(it, 8, R, 1)

            check_stratum(recs[idx], gold, oracle_chunk, f"mixed t={tt} G={G}")


def test_three_tile_slice_2e30_g32(jt, strata):
    """A contiguous 2^30-genotype slice of the three-tile space at G=32, in
    four pipelined calls of 2^28: the slice's first and last 4096 records
    and every 256th record equal the oracle's; properties on all."""
    n, per = 1 << 30, 1 << 28
    first = inputs.three_tile_slice_start(n)
    gold = strata["slice"]
    assert gold["first"] == first and gold["total"] == n and per % gold["stride"] == 0
    out = torch.empty((per, 4), dtype=torch.int32, device="cuda")
    total = np.zeros(4, dtype=np.int64)
    strided = []
    t_gpu = 0.0
    with jt.Batch(per) as b:
        for k in range(n // per):
            lo = first + k * per
            tally = torch.zeros(4, dtype=torch.int64, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.classify_range(lo, per, 3, 8, 32, R, 1, out=out, tally=tally)
            torch.cuda.synchronize()
            t_gpu += time.perf_counter() - t0
            recs = records(out)
            tl = tally.cpu().tolist()
            check_properties(recs, tl, f"slice part {k}")
            total += tl
            strided.append(recs[::gold["stride"]].copy())
            if k == 0:
                assert_same(recs[:4096], ref.classify_range(lo, 4096, 3, grid=32, runs=R, seed=1),
                            "slice head")
            if k == n // per - 1:
                assert_same(recs[-4096:], ref.classify_range(lo + per - 4096, 4096, 3, grid=32,
                                                             runs=R, seed=1), "slice tail")
    print(f"three-tile slice at {first}: {n / t_gpu / 1e6:.1f} M genotypes/s, tally {total.tolist()}",
          flush=True)
    stride = gold["stride"]
    check_stratum(np.concatenate(strided), gold,
                  lambda lo, hi: ref.classify(np.uint64(first) + np.arange(lo, hi, dtype=np.uint64)
                                              * np.uint64(stride), 3, grid=32, runs=R, seed=1),
                  "slice, every 256th")


def test_three_tile_sample_2e28_g32(jt, strata):
    """2^28 uniform three-tile genotypes at G=32 in one call: every 64th
    record equals the oracle's; properties on all."""
    n = 1 << 28
    g = inputs.three_tile_sample(n)
    dg = torch.from_numpy(g.view(np.int64)).cuda()
    tally = torch.zeros(4, dtype=torch.int64, device="cuda")
    with jt.Batch(n) as b:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = b.classify(dg, 3, 8, 32, R, 1, tally=tally)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    print(f"three-tile sample: {n / dt / 1e6:.1f} M genotypes/s ({dt:.2f} s)", flush=True)
    del dg
    recs = records(rec)
    del rec
    check_properties(recs, tally.cpu().tolist(), "three-tile sample")
    gold = strata["sample"]
    assert gold["total"] == n
    gs = g[::gold["stride"]]
    check_stratum(recs[::gold["stride"]].copy(), gold,
                  lambda lo, hi: ref.classify(gs[lo:hi], 3, grid=32, runs=R, seed=1),
                  "sample, every 64th")


def test_ga_population_65536_g32_chain(jt):
    """The GA at its full shape: population 65,536 of three-tile genotypes,
    G=32, R=20, tournament 4, mutation 1/12; three generations chained, every
    genome and fitness equal to the oracle's after each."""
    n = 65_536
    pop = inputs.population(n, 3)
    fit = np.zeros(n, dtype=np.int32)
    p = jt.GAParams(seed=5)
    with jt.Batch(n) as b:
        gpop = torch.from_numpy(pop.view(np.int64)).cuda()
        gfit = torch.from_numpy(fit).cuda()
        for gen in range(3):
            gpop, gfit = b.ga_step(gpop, gfit, 3, p, gen, grid_limit=32, runs=R, seed=1)
            pop, fit = ref.ga_step(pop, fit, 3, generation=gen, grid=32, runs=R, seed=1,
                                   ga_seed=5)
            torch.cuda.synchronize()
            assert np.array_equal(gpop.cpu().numpy().view(np.uint64), pop), gen
            assert np.array_equal(gfit.cpu().numpy(), fit), gen


def test_screened_ga_generation_full_size(jt):
    """A screened generation at full size: 4 x 65,536 offspring scored by the
    surrogate, the top 65,536 kept and assembled.  Offspring equal the
    oracle's; the kept set is exactly the top-k of the scores; fitness of the
    kept genotypes equals the oracle's."""
    n, k = 65_536, 4
    pop = inputs.population(n, 3)
    fit = (pop % np.uint64(17)).astype(np.int32)
    params = jt.GAParams(seed=5)
    dpop = torch.from_numpy(pop.view(np.int64)).cuda()
    dfit = torch.from_numpy(fit).cuda()
    with jt.MLP(4096) as net, jt.GA(k * n) as ga, jt.Batch(n) as b:
        net.init(3)
        nxt, nfit = ga.step_screened(b, net, dpop, dfit, 3, params, generation=1, oversample=k,
                                     grid_limit=32)
        cand = jt.ga_offspring(dpop, dfit, 3, params, generation=1, n_out=k * n)
        scores = net.score(cand, 3).cpu().numpy()
        torch.cuda.synchronize()
    cand = cand.cpu().numpy().view(np.uint64)
    assert np.array_equal(cand, ref.ga_offspring(pop, fit, 3, 1, n_out=k * n, seed=5))
    key = scores.astype(np.float32).view(np.uint32).astype(np.uint64)
    key = np.where(key & 0x80000000, (~key) & 0xFFFFFFFF, key | 0x80000000)
    key = (~key) & 0xFFFFFFFF
    key[np.isnan(scores)] = 0xFFFFFFFF
    kept = np.sort(np.lexsort((np.arange(len(scores)), key))[:n])
    got_pop = nxt.cpu().numpy().view(np.uint64)
    assert np.array_equal(got_pop, cand[kept])
    rec = ref.classify(got_pop, 3, grid=32, runs=R, seed=1)
    assert np.array_equal(nfit.cpu().numpy(), np.where(rec["cls"] == ref.DET, rec["size"], 0))

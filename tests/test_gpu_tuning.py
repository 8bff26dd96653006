"""Launch parameters of the pipeline: the autotuner and explicit tunings never
change a record, and neither does the order of the item queue (including an
order by the surrogate's predicted cost).  Records are checked against the
oracle or its golden digests."""
import hashlib
import json
import os

import numpy as np
import pytest

from oracle import ref
from tests import inputs

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


def test_autotune_on_s28_keeps_the_golden_records(jt):
    with open(os.path.join(HERE, "golden", "s28_digests.json")) as f:
        gold = json.load(f)
    n = gold["slice"]
    with jt.Batch(1 << 22) as b:
        best, log = b.autotune(0, 1 << 22, 2, 8, 16, 20, 1)
        print("autotune:", best, [(e, round(ms, 3)) for e, ms in log], flush=True)
        assert len(log) >= 8
        best_ms = [ms for e, ms in log if e == best][-1]
        assert best_ms <= log[0][1]          # never worse than where it started
        assert b.get_tuning(16) == best
        out = torch.empty((4 * n, 4), dtype=torch.int32, device="cuda")
        b.classify_range(0, 4 * n, 2, 8, 16, 20, 1, out=out)
        rec = out.cpu().numpy()
    for s in gold["slices"][:4]:
        blob = rec[s["first"]:s["first"] + s["n"]].tobytes()
        assert hashlib.sha256(blob).hexdigest() == s["sha256"], s["first"]


@pytest.mark.parametrize("grid,tuning", [
    (16, dict(refill=1, first_waves=1, repeat_waves=1)),
    (16, dict(refill=64, first_waves=3, repeat_waves=2)),
    (16, dict(wide_layout=1)),
    (32, dict(refill=8, first_waves=1, repeat_waves=2)),
    (32, dict(wide_layout=1)),
    (32, dict(wide_layout=2)),
    (16, dict(claim_share=0)),
    (16, dict(claim_share=16)),
    (16, dict(claim_share=16, first_waves=1, refill=64)),
    (32, dict(claim_share=16, first_waves=1)),
    (32, dict(claim_share=12, wide_layout=2)),
    (16, dict(claim_chunks=1, claim_share=16)),
    (16, dict(claim_chunks=8)),
    (16, dict(repeat_mapping=1)),
    (16, dict(repeat_mapping=1, repeat_waves=1, wide_layout=1)),
    (32, dict(repeat_mapping=1)),
    (32, dict(repeat_mapping=1, wide_layout=2)),
    (16, dict(repeat_mapping=2)),
    (16, dict(repeat_mapping=2, repeat_waves=1, claim_share=0)),
    (32, dict(repeat_mapping=2)),
    (32, dict(repeat_mapping=2, wide_layout=2)),
])
def test_explicit_tunings_keep_records(jt, grid, tuning):
    rng = np.random.default_rng(grid + len(tuning))
    g = rng.integers(0, 1 << 36, size=20_000, dtype=np.uint64)
    with jt.Batch(1 << 16) as b:
        b.set_tuning(grid, **tuning)
        got = records(b.classify(torch.from_numpy(g.view(np.int64)).cuda(), 3, 8, grid, 20, 1))
    assert_same(got, ref.classify(g, 3, grid=grid, runs=20, seed=1), f"G={grid} {tuning}")


@pytest.mark.parametrize("share", [8, 16])
def test_claimed_chunks_keep_records(jt, share):
    """Enough chunks per wave (one wave per CU, 2^18 genotypes) that the
    waves claim chunks from the device counter, up to four at a time, with
    segments sized for one claim beyond each wave's dealt-out share."""
    rng = np.random.default_rng(60 + share)
    g = rng.integers(0, 1 << 24, size=1 << 18, dtype=np.uint64)
    with jt.Batch(1 << 18) as b:
        b.set_tuning(16, claim_share=share, first_waves=1, refill=16)
        tally = torch.zeros(4, dtype=torch.int64, device="cuda")
        got = records(b.classify(torch.from_numpy(g.view(np.int64)).cuda(), 2, 8, 16, 20, 1,
                                 tally=tally))
    want = ref.classify(g, 2, grid=16, runs=20, seed=1)
    assert_same(got, want, f"claim_share={share}")
    assert tally.cpu().tolist() == [int(np.sum(want["cls"] == k)) for k in range(4)]


def test_bad_tunings_rejected(jt):
    with jt.Batch(1024) as b:
        for bad in (dict(refill=0), dict(refill=65), dict(first_waves=0), dict(repeat_waves=0),
                    dict(wide_layout=2), dict(claim_share=-1), dict(claim_share=17),
                    dict(claim_chunks=0), dict(claim_chunks=9), dict(repeat_mapping=-1),
                    dict(repeat_mapping=3)):
            with pytest.raises(jt.JatamError):
                b.set_tuning(16, **bad)
        with pytest.raises(jt.JatamError):
            b.set_tuning(32, wide_layout=3)
        with pytest.raises(jt.JatamError):
            b.set_tuning(16, wide_layout=2)


def mixed_items(jt, n):
    g, t, grid = inputs.mixed_stream(n, key=17)
    items = np.zeros(n, dtype=ref.ITEM)
    items["genome"], items["t"], items["grid"] = g, t, grid
    items["rng_id"] = g | (t.astype(np.uint64) << np.uint64(56))
    return g, t, grid, items


def test_queue_order_does_not_change_records(jt):
    n = 1 << 15
    g, t, grid, items = mixed_items(jt, n)
    want = ref.classify_items(items)
    dev = torch.from_numpy(jt.make_items(g, t, grid)).cuda()
    rng = np.random.default_rng(4)
    orders = {"identity": np.arange(n), "reversed": np.arange(n)[::-1].copy(),
              "random": rng.permutation(n), "grid-major": np.argsort(-grid.astype(np.int64),
                                                                     kind="stable")}
    with jt.Batch(n) as b:
        for name, order in orders.items():
            tally = torch.zeros(4, dtype=torch.int64, device="cuda")
            o = torch.from_numpy(order.astype(np.int32)).cuda()
            got = records(b.classify_items(dev, 8, 20, 1, tally=tally, order=o))
            assert_same(got, want, name)
            assert tally.cpu().tolist() == [int(np.sum(want["cls"] == k)) for k in range(4)]


def test_surrogate_cost_order_keeps_records(jt):
    """The queue ordered by an (untrained) surrogate's predicted cost, most
    expensive first: records equal the oracle's."""
    n = 1 << 15
    g, t, grid, items = mixed_items(jt, n)
    dg = torch.from_numpy(g.view(np.int64)).cuda()
    dt = torch.from_numpy(t.astype(np.uint8)).cuda()
    with jt.MLP(4096) as net, jt.Batch(n) as b:
        net.init(5)
        order = jt.order_by_cost(net.score(dg, dt))
        dev = torch.from_numpy(jt.make_items(g, t, grid)).cuda()
        got = records(b.classify_items(dev, 8, 20, 1, order=order))
    assert_same(got, ref.classify_items(items), "surrogate order")


def spearman(a, b):
    """Rank correlation with tied values given their mean rank (most exact
    step counts are 0)."""
    from scipy.stats import spearmanr
    return float(spearmanr(a, b).correlation)


def test_trained_cost_order_follows_the_exact_work(jt):
    """A network trained on exact classifications orders a range of S_{2,8}
    it has not seen by its exact work: the order is a permutation whose
    predicted-cost buckets never rise, the ordered pipeline gives the
    oracle's records, and the predicted cost (the size of the deciding run)
    ranks genotypes by the exact placement count of their first run, the
    work of the first-run queue it orders (Spearman), far better than the
    untrained network's."""
    rng = np.random.default_rng(12)
    train = rng.integers(0, 1 << 23, size=1 << 17, dtype=np.uint64)   # lower half of S_2,8
    dtrain = torch.from_numpy(train.view(np.int64)).cuda()
    lab = jt.classify(dtrain, 2, 8, 16, 20, 1)
    first, n = 3 << 22, 1 << 15                                        # upper half
    want, steps0, _, _ = ref.classify_range_run0(first, n, 2, grid=16, runs=20, seed=1)
    genomes = torch.arange(first, first + n, dtype=torch.int64, device="cuda")
    corr = {}
    with jt.MLP(4096) as net, jt.Batch(n) as b:
        net.init(7)
        corr["untrained"] = spearman(net.predict(genomes, 2, jt.PREDICT_COST).cpu().numpy(),
                                     steps0)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        for step in range(400):
            lo = (step * 4096) % (1 << 17)
            net.train_step(dtrain[lo:lo + 4096], 2, lab[lo:lo + 4096], lr=1e-3, loss=loss)
        scores = net.predict(genomes, 2, jt.PREDICT_COST)
        screen = net.score(genomes, 2).cpu().numpy()
        order = jt.order_by_cost(scores)
        got = records(b.classify_range_ordered(first, n, order, 2, 8, 16, 20, 1))
        sc = scores.cpu().numpy()
        o = order.cpu().numpy().astype(np.int64)
    assert_same(got, want, "trained cost order")
    assert np.array_equal(np.sort(o), np.arange(n))
    # buckets of 16 log2(score + 2), never rising along the order (the kernel's
    # fast log2 may put a score on a bucket boundary one bucket off)
    key = np.floor(16 * np.log2(np.maximum(sc[o], -1.0) + 2.0)).clip(0, 255)
    assert np.all(np.diff(key) <= 1) and np.sum(np.diff(key) > 0) <= n // 100
    corr["trained"] = spearman(sc, steps0)
    corr["trained_screen_score"] = spearman(screen, steps0)
    corr["trained_vs_all_runs"] = spearman(sc, want["steps"])
    print("Spearman(predicted cost, exact steps):", corr)
    # measured: 0.31 trained, 0.02 untrained (ties at zero steps, 61% of
    # genotypes, get their mean rank)
    assert corr["trained"] > 0.25 and corr["trained"] > corr["untrained"] + 0.2, corr


@pytest.mark.parametrize("t,grid", [(3, 32), (2, 32), (3, 24), (4, 20)])
def test_window_and_direct_wide_layout_agree(jt, t, grid):
    """16 < G <= 32: the 16 x 16 window with a 32 x 32 rerun of the items
    that left it, the direct 32 x 32 classification, and the default (direct
    at this call size) give the oracle's records and tallies."""
    rng = np.random.default_rng(40 + t + grid)
    g = rng.integers(0, 1 << (12 * t), size=40_000, dtype=np.uint64)
    want = ref.classify(g, t, grid=grid, runs=20, seed=1)
    dev = torch.from_numpy(g.view(np.int64)).cuda()
    with jt.Batch(1 << 16) as b:
        for wide in (2, 1, 0):
            b.set_tuning(32, wide_layout=wide)
            tally = torch.zeros(4, dtype=torch.int64, device="cuda")
            got = records(b.classify(dev, t, 8, grid, 20, 1, tally=tally))
            assert_same(got, want, f"t={t} G={grid} wide_layout={wide}")
            assert tally.cpu().tolist() == [int(np.sum(want["cls"] == k)) for k in range(4)]


@pytest.mark.parametrize("mapping,runs", [(0, 20), (1, 20), (2, 20)])
def test_repeat_mappings_keep_the_golden_records(jt, mapping, runs):
    """One lane per repeat candidate (runs in turn, stopping at the first
    witness), and two passes (4 lanes per candidate, then R lanes for the
    undecided), over the first 2^22 genotypes of S_{2,8}: the oracle's
    digests."""
    with open(os.path.join(HERE, "golden", "s28_digests.json")) as f:
        gold = json.load(f)
    n = gold["slice"]
    with jt.Batch(4 * n) as b:
        b.set_tuning(16, repeat_mapping=mapping)
        tally = torch.zeros(4, dtype=torch.int64, device="cuda")
        out = b.classify_range(0, 4 * n, 2, 8, 16, runs, 1, tally=tally)
        torch.cuda.synchronize()
        rec = out.cpu().numpy()
    for s in gold["slices"][:4]:
        blob = rec[s["first"]:s["first"] + s["n"]].tobytes()
        assert hashlib.sha256(blob).hexdigest() == s["sha256"], s["first"]
    want = np.sum([s["tally"] for s in gold["slices"][:4]], axis=0).tolist()
    assert tally.cpu().tolist() == want


@pytest.mark.parametrize("runs", [1, 2, 4, 5, 7, 8, 12, 20, 33, 64])
def test_two_pass_repeat_at_every_run_count(jt, runs):
    """Two repeat passes at run counts below, at and above the first pass's
    4 runs, on S_{2,8} and three-tile genotypes: the oracle's records."""
    rng = np.random.default_rng(runs)
    g2 = rng.integers(0, 1 << 24, size=30_000, dtype=np.uint64)
    g3 = rng.integers(0, 1 << 36, size=10_000, dtype=np.uint64)
    with jt.Batch(1 << 15) as b:
        b.set_tuning(16, repeat_mapping=2)
        b.set_tuning(32, repeat_mapping=2)
        got2 = records(b.classify(torch.from_numpy(g2.view(np.int64)).cuda(), 2, 8, 16, runs, 1))
        got3 = records(b.classify(torch.from_numpy(g3.view(np.int64)).cuda(), 3, 8, 32, runs, 1))
    assert_same(got2, ref.classify(g2, 2, grid=16, runs=runs, seed=1), f"t=2 R={runs}")
    assert_same(got3, ref.classify(g3, 3, grid=32, runs=runs, seed=1), f"t=3 R={runs}")


def test_classify_batch_with_order_and_call_tuning(jt):
    """jatam_classify_batch: a mixed stream with a queue order and per-call
    launch parameters gives the oracle's records and leaves the workspace's
    own parameters as they were."""
    n = 1 << 14
    g, t, grid, items = mixed_items(jt, n)
    want = ref.classify_items(items)
    dev = torch.from_numpy(jt.make_items(g, t, grid)).cuda()
    order = torch.from_numpy(np.random.default_rng(9).permutation(n).astype(np.int32)).cuda()
    tunes = [None,
             {16: dict(repeat_mapping=1, claim_chunks=2), 32: dict(repeat_mapping=1)},
             {16: dict(refill=8, first_waves=2), 32: dict(wide_layout=2, claim_share=16)}]
    with jt.Batch(n) as b:
        before = (b.get_tuning(16), b.get_tuning(32))
        for tune in tunes:
            for o in (None, order):
                tally = torch.zeros(4, dtype=torch.int64, device="cuda")
                got = records(b.classify_batch(dev, 8, 20, 1, order=o, tune=tune, tally=tally))
                assert_same(got, want, f"tune={tune} order={o is not None}")
                assert tally.cpu().tolist() == [int(np.sum(want["cls"] == k)) for k in range(4)]
        assert (b.get_tuning(16), b.get_tuning(32)) == before
        with pytest.raises(jt.JatamError):
            b.classify_batch(dev, 8, 20, 1, tune={16: dict(repeat_mapping=3)})


def test_staging_back_pressure_keeps_records(jt):
    """Every item a DET candidate (run 0 drew a random word and ended clean):
    with every chunk claimed by one wave per CU, segments fill up and waves
    stop claiming once a claim would not fit; every item is still
    classified."""
    rng = np.random.default_rng(70)
    pool = rng.integers(0, 1 << 24, size=1 << 16, dtype=np.uint64)
    rec = ref.classify(pool, 2, grid=16, runs=20, seed=1)
    cand = pool[(rec["cls"] == ref.DET) & (rec["size"] >= 3)
                & (rec["steps"] == (rec["size"] - 1) * 20)]
    assert len(cand) > 1000
    g = np.resize(cand, 1 << 18)
    want = ref.classify(g, 2, grid=16, runs=20, seed=1)
    with jt.Batch(1 << 18) as b:
        b.set_tuning(16, claim_share=16, first_waves=1, refill=16, claim_chunks=1)
        tally = torch.zeros(4, dtype=torch.int64, device="cuda")
        got = records(b.classify(torch.from_numpy(g.view(np.int64)).cuda(), 2, 8, 16, 20, 1,
                                 tally=tally))
    assert_same(got, want, "all candidates")
    assert tally.cpu().tolist() == [0, 0, 0, len(g)]


def test_claim_parts_run_dry_unevenly(jt):
    """First-run claims come from eight parts of the claimed chunks, one
    counter each; a wave whose part runs dry moves on to the next.  Here the
    last part holds only long runs and the others only genotypes the seed
    decides, so most waves finish their own part early and take chunks of
    the last one: every item is still classified exactly once."""
    rng = np.random.default_rng(71)
    pool = rng.integers(0, 1 << 24, size=1 << 17, dtype=np.uint64)
    rec = ref.classify(pool, 2, grid=16, runs=20, seed=1)
    # long run 0: an event after 40 or more placements, or a DET shape of 16
    # or more cells; cheap: decided at the seed (no placement)
    heavy = pool[((rec["cls"] != ref.DET) & (rec["steps"] >= 40))
                 | ((rec["cls"] == ref.DET) & (rec["size"] >= 16))]
    cheap = pool[rec["steps"] == 0]
    assert len(heavy) > 500 and len(cheap) > 10000
    n = 1 << 18
    # 256 waves, 4,096 chunks: a quarter dealt out, 3,072 claimed one at a
    # time in eight parts of 384 chunks; the last part is the list's last
    # 384 * 64 entries
    tail = 384 * 64
    g = np.concatenate([np.resize(cheap, n - tail), np.resize(heavy, tail)])
    want = ref.classify(g, 2, grid=16, runs=20, seed=1)
    with jt.Batch(n) as b:
        b.set_tuning(16, claim_share=12, claim_chunks=4, first_waves=1)
        tally = torch.zeros(4, dtype=torch.int64, device="cuda")
        got = records(b.classify(torch.from_numpy(g.view(np.int64)).cuda(), 2, 8, 16, 20, 1,
                                 tally=tally))
    assert_same(got, want, "uneven claim parts")
    assert tally.cpu().tolist() == [int(np.sum(want["cls"] == k)) for k in range(4)]


def test_autotune_cache_file(jt, tmp_path):
    """The tuning found for a key is written to the cache file and read back
    instead of searching again; another key adds a line; a broken line of a
    key is searched again and replaced."""
    path = tmp_path / "tuning.jsonl"
    n = 1 << 18
    with jt.Batch(n) as b:
        t1, hit1 = b.autotune_cached(str(path), 0, n, 2, 8, 16, 20, 2)
        assert not hit1
        lines = path.read_text().splitlines()
        assert len(lines) == 1 and '"key": "' in lines[0] and "|R20|" in lines[0]
        b.set_tuning(16, refill=64)
        t2, hit2 = b.autotune_cached(str(path), 0, n, 2, 8, 16, 20, 2)
        assert hit2 and t2 == t1 and b.get_tuning(16) == t1
        _, hit3 = b.autotune_cached(str(path), 0, n, 2, 8, 16, 7, 2)
        assert not hit3 and len(path.read_text().splitlines()) == 2
    path.write_text(lines[0].replace('"refill": ', '"refill": x') + "\n")
    with jt.Batch(n) as b:
        _, hit4 = b.autotune_cached(str(path), 0, n, 2, 8, 16, 20, 2)
        assert not hit4
        fixed = path.read_text().splitlines()
        assert len(fixed) == 1 and '"refill": x' not in fixed[0]

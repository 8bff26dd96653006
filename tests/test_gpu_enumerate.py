"""Graph-replayed enumeration (jatam_batch_enumerate): one captured slice
pipeline launched once per slice.  Every replay's records, and the tally and
shape histogram accumulated over the replays, equal the oracle's (golden
digests or direct oracle calls).  Eager calls run between enumerations."""
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


def golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


def shapes_of(jt, table):
    return [(int(e["hash"]), int(e["size"]), int(e["count"]))
            for e in jt.shape_table_to_numpy(table)]


def test_s28_in_16_graph_replays(jt):
    gold = golden("s28_digests.json")
    n = gold["slice"]
    out = torch.empty((16 * n, 4), dtype=torch.int32, device="cuda")
    tally = torch.zeros(4, dtype=torch.int64, device="cuda")
    table = torch.zeros((256, 2), dtype=torch.int64, device="cuda")
    with jt.Batch(n) as b:
        b.enumerate(0, n, 16, 2, 8, 16, 20, 1, out=out, tally=tally, shapes=table)
        torch.cuda.synchronize()
        rec = out.cpu().numpy()
        for s in gold["slices"]:
            blob = rec[s["first"]:s["first"] + s["n"]].tobytes()
            assert hashlib.sha256(blob).hexdigest() == s["sha256"], s["first"]
        assert tally.cpu().tolist() == gold["tally"]
        assert shapes_of(jt, table) == [(s["hash"], s["size"], s["count"]) for s in gold["shapes"]]

        # eager work on the same workspace, then a second enumeration with a
        # new capture: S_{1,8} kept only as tally and histogram
        b.classify_range(0, 4096, 1, 8, 16, 20, 1)
        torch.cuda.synchronize()
        g18 = golden("s18_digests.json")
        tally.zero_()
        table.zero_()
        b.enumerate(0, 1024, 4, 1, 8, 16, 20, 1, tally=tally, shapes=table)
        torch.cuda.synchronize()
        assert tally.cpu().tolist() == g18["tally"]
        assert shapes_of(jt, table) == [(s["hash"], s["size"], s["count"]) for s in g18["shapes"]]


def test_s28_tally_and_shapes_without_records(jt):
    gold = golden("s28_digests.json")
    tally = torch.zeros(4, dtype=torch.int64, device="cuda")
    table = torch.zeros((256, 2), dtype=torch.int64, device="cuda")
    with jt.Batch(1 << 22) as b:
        b.enumerate(0, 1 << 22, 4, 2, 8, 16, 20, 1, tally=tally, shapes=table)
        torch.cuda.synchronize()
    assert tally.cpu().tolist() == gold["tally"]
    assert shapes_of(jt, table) == [(s["hash"], s["size"], s["count"]) for s in gold["shapes"]]


def test_three_tile_g32_replays(jt):
    first, n, k = 8_000_000_000, 1 << 16, 5
    out = torch.empty((k * n, 4), dtype=torch.int32, device="cuda")
    with jt.Batch(n) as b:
        for _ in range(2):      # the same enumeration twice: replays agree with the oracle
            out.fill_(-7)
            b.enumerate(first, n, k, 3, 8, 32, 20, 1, out=out)
            torch.cuda.synchronize()
            rec = out.cpu().numpy().view(ref.RECORD).reshape(-1)
            pick = np.sort(np.random.default_rng(2).choice(k * n, size=4096, replace=False))
            want = ref.classify(np.uint64(first) + pick.astype(np.uint64), 3, grid=32)
            assert np.array_equal(rec[pick], want)
            for lo in (0, n - 512, 2 * n, k * n - 512):
                assert np.array_equal(rec[lo:lo + 512],
                                      ref.classify_range(first + lo, 512, 3, grid=32)), lo


def test_enumerate_argument_errors(jt):
    with jt.Batch(1024) as b:
        for args in ((0, 0, 1), (0, 2048, 1), (0, 1024, 0), ((1 << 24) - 1024, 1024, 2)):
            with pytest.raises(jt.JatamError):
                b.enumerate(args[0], args[1], args[2], 2, 8, 16, 20, 1)
        bad = torch.zeros((100, 2), dtype=torch.int64, device="cuda")
        with pytest.raises(jt.JatamError):
            b.enumerate(0, 1024, 1, 2, 8, 16, 20, 1, shapes=bad)


def test_window_in_graph_replays(jt):
    """Three-tile slices at G = 32 through the 16 x 16 window (forced on),
    the list of items that left it and their 32 x 32 rerun all inside the
    captured slice pipeline: records, tally and shape histogram equal the
    oracle's, and some items did leave the window."""
    first, n, k = 8_592_194_344, 1 << 15, 4
    want = ref.classify_range(first, k * n, 3, grid=32)
    assert np.sum(want["cls"] == ref.UNBOUND) > 100
    out = torch.empty((k * n, 4), dtype=torch.int32, device="cuda")
    tally = torch.zeros(4, dtype=torch.int64, device="cuda")
    table = torch.zeros((1024, 2), dtype=torch.int64, device="cuda")
    with jt.Batch(n) as b:
        b.set_tuning(32, wide_layout=2)
        b.enumerate(first, n, k, 3, 8, 32, 20, 1, out=out, tally=tally, shapes=table)
        torch.cuda.synchronize()
        rec = out.cpu().numpy().view(ref.RECORD).reshape(-1)
    assert np.array_equal(rec, want)
    assert tally.cpu().tolist() == [int(np.sum(want["cls"] == c)) for c in range(4)]
    det = want[want["cls"] == ref.DET]
    keys, counts = np.unique(np.stack([det["size"].astype(np.int64), det["hash"].astype(np.int64)]),
                             axis=1, return_counts=True)
    assert shapes_of(jt, table) == [(int(h), int(z), int(c)) for (z, h), c in zip(keys.T, counts)]


def test_s28_resumable_with_a_manifest(jt, tmp_path):
    """All of S_{2,8} in 16 slices through the manifest driver, stopped after
    5 slices and resumed: every slice digest and tally is the golden one, as
    is the total."""
    import hashlib as hl

    from paper_2205_15311_amd import manifest
    gold = golden("s28_digests.json")
    n = gold["slice"]
    header = {"space": "S_2,8", "t": 2, "c": 8, "grid": 16, "runs": 20, "seed": 1}
    with jt.Batch(n) as b:
        def gpu_slice(first, count):
            rec = b.classify_range(first, count, 2, 8, 16, 20, 1)
            torch.cuda.synchronize()
            return rec.cpu().numpy()

        path = str(tmp_path / "s28.jsonl")
        part = manifest.enumerate_slices(path, header, 0, n, 16, gpu_slice, stop_after=5)
        assert part["slices_done"] == 5 and not part["complete"]
        res = manifest.enumerate_slices(path, header, 0, n, 16, gpu_slice)
    assert res["complete"]
    entries = [json.loads(x) for x in open(path).read().splitlines()[1:]]
    for e, s in zip(sorted(entries, key=lambda e: e["slice"]), gold["slices"]):
        assert e["sha256"] == s["sha256"] and e["tally"] == s["tally"]
    want = hl.sha256("".join(s["sha256"] for s in gold["slices"]).encode()).hexdigest()
    assert res["digest"] == want
    assert res["tally"] == np.sum([s["tally"] for s in gold["slices"]], axis=0).tolist()

"""jatam_classify_static (the pipelined classification with the library's
static device array as its workspace) against jatam_batch_classify (the same
pipeline with an allocated workspace) and the oracle: two calls in a row,
the second smaller, through the C ABI."""
import ctypes

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


@pytest.mark.parametrize("t,grid,n1,n2", [(2, 16, 1 << 18, 5000), (3, 32, 100_000, 777)])
def test_static_workspace_equals_allocated_workspace(jt, t, grid, n1, n2):
    rng = np.random.default_rng(100 + t)
    L = jt.lib()
    with jt.Batch(1 << 18) as b:
        for n in (n1, n2):
            g = rng.integers(0, 1 << (12 * t), size=n, dtype=np.uint64)
            dg = torch.from_numpy(g.view(np.int64)).cuda()
            out = torch.full((n, 4), -7, dtype=torch.int32, device="cuda")
            tally = torch.zeros(4, dtype=torch.int64, device="cuda")
            rc = L.jatam_classify_static(dg.data_ptr(), n, t, 8, grid, 20, 1, out.data_ptr(),
                                         tally.data_ptr(), None)
            assert rc == 0
            got = records(out)
            want = records(b.classify(dg, t, 8, grid, 20, 1))
            assert np.array_equal(got, want), (t, grid, n)
            pick = np.sort(rng.choice(n, size=min(n, 4096), replace=False))
            assert np.array_equal(got[pick], ref.classify(g[pick], t, grid=grid, runs=20, seed=1))
            assert tally.cpu().tolist() == [int(np.sum(want["cls"] == k)) for k in range(4)]


def test_static_workspace_limits(jt):
    L = jt.lib()
    buf = torch.zeros(8, dtype=torch.int64, device="cuda")
    out = torch.zeros((8, 4), dtype=torch.int32, device="cuda")
    assert L.jatam_classify_static(buf.data_ptr(), (1 << 18) + 1, 2, 8, 16, 20, 1,
                                   out.data_ptr(), None, None) == -1
    assert L.jatam_classify_static(buf.data_ptr(), -1, 2, 8, 16, 20, 1, out.data_ptr(), None,
                                   None) == -1
    assert L.jatam_classify_static(None, 0, 2, 8, 16, 20, 1, None, None, None) == 0

"""Surrogate use on the GPU: scores against the reference network, the top-k
rule exactly, the screened GA generation exactly given the surrogate's
scores (fitness from assembly, checked against the oracle), and what the
trained surrogate gains over unscreened offspring."""
import numpy as np
import pytest

from oracle import mlp_ref as M
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


def desc_order_key(scores):
    """Ascending key == descending score in IEEE total order, NaN last."""
    u = scores.astype(np.float32).view(np.uint32).astype(np.uint64)
    asc = np.where(u & 0x80000000, (~u) & 0xFFFFFFFF, u | 0x80000000)
    key = (~asc) & 0xFFFFFFFF
    nan = np.isnan(scores)
    key[nan] = 0xFFFFFFFF
    return key


def top_k_reference(scores, k):
    key = desc_order_key(scores)
    order = np.lexsort((np.arange(len(scores)), key))
    return np.sort(order[:k])


def test_select_top_with_ties_nan_and_signed_zero(jt):
    rng = np.random.default_rng(0)
    n, k = 262_144, 65_536
    s = rng.integers(-50, 50, size=n).astype(np.float32) / 4
    s[rng.random(n) < 0.01] = np.nan
    s[rng.random(n) < 0.01] = -0.0
    s[rng.random(n) < 0.001] = np.inf
    with jt.GA(n) as ga:
        for kk in (1, 7, k, n):
            got = ga.select_top(torch.from_numpy(s).cuda(), kk).cpu().numpy()
            assert np.array_equal(got, top_k_reference(s, kk)), kk


def test_scores_match_reference(jt):
    p = M.random_params(11)
    rng = np.random.default_rng(2)
    g = rng.integers(0, 1 << 36, size=3000, dtype=np.uint64)
    with jt.MLP(1024) as net:
        net.set_params(torch.from_numpy(M.flatten(p).astype(np.float32)).cuda())
        got = net.score(torch.from_numpy(g.view(np.int64)).cuda(), 3).cpu().numpy()
    out, _ = M.forward(p, M.encode(g, 3))
    z = out[:, :3] - out[:, :3].max(axis=1, keepdims=True)
    pdet = np.exp(z[:, 2]) / np.exp(z).sum(axis=1)
    want = pdet * np.exp(out[:, 3]) - 1
    assert np.abs(got - want).max() <= 1e-3 * (np.abs(want).max() + 1)


def test_predictions_match_reference(jt):
    """jatam_mlp_predict's three kinds against the reference network's
    outputs: the screening score, the predicted size exp(o3) - 1 and the
    softmax probability of UNBOUND."""
    p = M.random_params(13)
    rng = np.random.default_rng(5)
    g = rng.integers(0, 1 << 36, size=3000, dtype=np.uint64)
    dg = torch.from_numpy(g.view(np.int64)).cuda()
    with jt.MLP(1024) as net:
        net.set_params(torch.from_numpy(M.flatten(p).astype(np.float32)).cuda())
        got = {k: net.predict(dg, 3, k).cpu().numpy().astype(np.float64)
               for k in (jt.PREDICT_SCREEN, jt.PREDICT_COST, jt.PREDICT_P_UNBOUND)}
        score = net.score(dg, 3).cpu().numpy()
    out, _ = M.forward(p, M.encode(g, 3))
    z = out[:, :3] - out[:, :3].max(axis=1, keepdims=True)
    prob = np.exp(z) / np.exp(z).sum(axis=1, keepdims=True)
    want = {jt.PREDICT_SCREEN: prob[:, 2] * np.exp(out[:, 3]) - 1,
            jt.PREDICT_COST: np.exp(out[:, 3]) - 1,
            jt.PREDICT_P_UNBOUND: prob[:, 0]}
    assert np.array_equal(got[jt.PREDICT_SCREEN], score.astype(np.float64))
    for k, w in want.items():
        assert np.abs(got[k] - w).max() <= 2e-3 * (np.abs(w).max() + 1), k


def test_screened_generation_is_exact_given_scores(jt):
    rng = np.random.default_rng(5)
    n, k = 4096, 4
    pop = rng.integers(0, 1 << 36, size=n, dtype=np.uint64)
    fit = rng.integers(0, 20, size=n, dtype=np.int32)
    params = jt.GAParams(seed=5)
    dpop = torch.from_numpy(pop.view(np.int64)).cuda()
    dfit = torch.from_numpy(fit).cuda()
    with jt.MLP(4096) as net, jt.GA(k * n) as ga, jt.Batch(n) as b:
        net.init(3)
        nxt, nfit = ga.step_screened(b, net, dpop, dfit, 3, params, generation=4, oversample=k,
                                     grid_limit=32)
        cand = jt.ga_offspring(dpop, dfit, 3, params, generation=4, n_out=k * n)
        scores = net.score(cand, 3).cpu().numpy()
        torch.cuda.synchronize()
    cand = cand.cpu().numpy().view(np.uint64)
    assert np.array_equal(cand, ref.ga_offspring(pop, fit, 3, 4, n_out=k * n, seed=5))
    kept = top_k_reference(scores, n)
    got_pop = nxt.cpu().numpy().view(np.uint64)
    assert np.array_equal(got_pop, cand[kept])
    rec = ref.classify(got_pop, 3, grid=32, runs=20, seed=1)
    want_fit = np.where(rec["cls"] == ref.DET, rec["size"], 0)
    assert np.array_equal(nfit.cpu().numpy(), want_fit)


def test_trained_surrogate_raises_offspring_fitness(jt):
    """The gain of the learned part: train on exact classifications of random
    three-tile genotypes (G=32), then keep the best quarter of 4x offspring
    by surrogate score.  Their mean exact fitness must beat that of the
    unscreened offspring by a clear margin."""
    rng = np.random.default_rng(21)
    n_train = 1 << 17
    tg = torch.from_numpy(rng.integers(0, 1 << 36, size=n_train, dtype=np.uint64).view(np.int64)).cuda()
    with jt.Batch(1 << 17) as b, jt.MLP(4096) as net, jt.GA(1 << 16) as ga:
        labels = b.classify(tg, 3, 8, 32, 20, 1)
        net.init(1)
        for step in range(600):
            lo = (step * 4096) % n_train
            net.train_step(tg[lo:lo + 4096], 3, labels[lo:lo + 4096], lr=1e-3)
        n = 1 << 14
        pop = torch.from_numpy(rng.integers(0, 1 << 36, size=n, dtype=np.uint64).view(np.int64)).cuda()
        rec = b.classify(pop, 3, 8, 32, 20, 1)
        fit = torch.where(rec[:, 0] == 3, rec[:, 1], torch.zeros_like(rec[:, 1])).contiguous()
        params = jt.GAParams(seed=9)
        cand = jt.ga_offspring(pop, fit, 3, params, generation=0, n_out=4 * n)
        crec = b.classify(cand, 3, 8, 32, 20, 1)
        cfit = torch.where(crec[:, 0] == 3, crec[:, 1], torch.zeros_like(crec[:, 1])).float()
        kept = ga.select_top(net.score(cand, 3), n).long()
        screened = float(cfit[kept].mean())
        unscreened = float(cfit.mean())
    print(f"mean fitness: unscreened {unscreened:.3f}, screened {screened:.3f}")
    assert screened > 1.3 * unscreened


def test_ga_step_with_surrogate_is_the_screened_generation(jt):
    """jatam_ga_step with a surrogate argument makes the screened generation
    (same population and fitness as jatam_ga_step_screened), and without one
    the plain generation of the oracle."""
    rng = np.random.default_rng(6)
    n, k = 2048, 4
    pop = rng.integers(0, 1 << 36, size=n, dtype=np.uint64)
    fit = rng.integers(0, 20, size=n, dtype=np.int32)
    params = jt.GAParams(seed=5)
    dpop = torch.from_numpy(pop.view(np.int64)).cuda()
    dfit = torch.from_numpy(fit).cuda()
    with jt.MLP(4096) as net, jt.GA(k * n) as ga, jt.Batch(n) as b:
        net.init(3)
        a_pop, a_fit = ga.step_screened(b, net, dpop, dfit, 3, params, generation=2,
                                        oversample=k, grid_limit=32)
        a_pop, a_fit = a_pop.cpu().numpy(), a_fit.cpu().numpy()
        s_pop, s_fit = b.ga_step(dpop, dfit, 3, params, 2, grid_limit=32,
                                 surrogate=jt.Screen(net, ga, k))
        p_pop, p_fit = b.ga_step(dpop, dfit, 3, params, 2, grid_limit=32)
        torch.cuda.synchronize()
    assert np.array_equal(s_pop.cpu().numpy(), a_pop)
    assert np.array_equal(s_fit.cpu().numpy(), a_fit)
    want_pop, want_fit = ref.ga_step(pop, fit, 3, generation=2, grid=32, runs=20, seed=1,
                                     ga_seed=5)
    assert np.array_equal(p_pop.cpu().numpy().view(np.uint64), want_pop)
    assert np.array_equal(p_fit.cpu().numpy(), want_fit)

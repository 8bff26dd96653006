"""Pins of the reference surrogate MLP (oracle/mlp_ref.py): its gradients
against central finite differences (pure fp64), its bf16 rounding against
torch's conversion, its input encoding against the independent genome
decoder, and Adam's first step against its closed form."""
import numpy as np
import pytest

from oracle import mlp_ref as M
from tests import brute_force as bf

torch = pytest.importorskip("torch")


def batch(n=48, seed=0):
    rng = np.random.default_rng(seed)
    g = rng.integers(0, 1 << 36, size=n, dtype=np.uint64)
    t = rng.integers(1, 4, size=n)
    g = g >> (36 - 12 * t).astype(np.uint64)
    cls = rng.integers(0, 4, size=n)
    size = rng.integers(1, 60, size=n)
    return g, t, cls, size


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000) * 10 ** rng.uniform(-8, 8, 20000),
                        [0.0, -0.0, 1.0, 3.0, 1e-40, 65504.0]])
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.to_bf16(x), want)


def test_encoding_matches_decoder():
    g, t, _, _ = batch(200, seed=3)
    x = M.encode(g, t)
    for i in range(len(g)):
        tiles = bf.decode(int(g[i]), int(t[i]), 8)
        want = np.zeros(96)
        for e in range(4 * int(t[i])):
            want[e * 8 + tiles[e // 4][e % 4]] = 1.0
        assert np.array_equal(x[i], want)
    assert np.array_equal(x.sum(axis=1), 4 * t)


def test_gradients_match_finite_differences():
    p = M.random_params(7, scale=0.5)
    g, t, cls, size = batch(32, seed=5)
    loss, grads, _ = M.loss_and_grads(p, g, t, cls, size, bf16=False)
    rng = np.random.default_rng(9)
    eps = 1e-6
    for key in M.ORDER:
        shape = M.SHAPES[key]
        for _ in range(12):
            idx = tuple(int(rng.integers(0, s)) for s in shape)
            if key == "w1":   # only rows that some input activates have a gradient
                x = M.encode(g, t)
                idx = (int(rng.choice(np.nonzero(x.sum(axis=0))[0])), idx[1])
            q_plus = {k: v.copy() for k, v in p.items()}
            q_minus = {k: v.copy() for k, v in p.items()}
            q_plus[key][idx] += eps
            q_minus[key][idx] -= eps
            lp = M.loss_and_grads(q_plus, g, t, cls, size, bf16=False)[0]
            lm = M.loss_and_grads(q_minus, g, t, cls, size, bf16=False)[0]
            fd = (lp - lm) / (2 * eps)
            an = grads[key][idx]
            assert abs(fd - an) <= 1e-6 + 1e-5 * abs(an), (key, idx, fd, an)


def test_cross_entropy_gradient_sums_to_zero():
    p = M.random_params(2)
    g, t, cls, size = batch(64, seed=8)
    x = M.encode(g, t)
    k, y = M.targets(cls, size)
    out, _ = M.forward(p, x)
    _, dout = M.loss_and_dout(out, k, y)
    assert np.allclose(dout[:, :3].sum(axis=1), 0.0, atol=1e-15)


def test_adam_first_step_is_signed_lr():
    p = M.random_params(4)
    g = {k: np.random.default_rng(1).standard_normal(v.shape) for k, v in p.items()}
    zero = {k: np.zeros_like(v) for k, v in p.items()}
    q, m, v = M.adam(p, g, zero, zero, step=1, lr=1e-3)
    for k in M.ORDER:
        # m_hat = g, v_hat = g^2: the step is lr * g / (|g| + eps)
        assert np.allclose(p[k] - q[k], 1e-3 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-12)


def test_parameter_count():
    assert M.n_params() == 96 * 256 + 256 + 256 * 256 + 256 + 256 * 4 + 4 == 91652

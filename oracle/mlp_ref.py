"""Reference surrogate MLP: forward, loss, backward and Adam, in numpy fp64.

TEST INFRASTRUCTURE ONLY (never imported by the product path).  The paper
has no learned part; this network is the library's surrogate for screening
GA offspring: it predicts, from a genotype's edge colours, its class
(UNBOUND / ND / DET) and log(1 + size), so that only the most promising
offspring are assembled.  Every reported class still comes from exact
assembly.

Network: x = one-hot of the 12 edge colours (12 x 8 = 96 inputs; the edges
of absent tiles are all-zero), h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2)
(256 wide each), out = h2 W3 + b3 (3 class logits, 1 log1p-size).
Loss = mean cross-entropy + mean squared error of log1p(size), weighted 1:1.

Precision model (mirrors the kernels): weights are held in fp32 and used
rounded to bf16; h1, h2 and the hidden-layer gradients are rounded to bf16
(round to nearest even, after rounding to fp32) where the kernels store
them; every sum is exact here (fp64) where the kernels accumulate in fp32.
With `bf16=False` no rounding happens at all (pure fp64), which is what the
finite-difference pins check.  `rounding` names the points that round (all
of ROUNDING by default); a test leaves one out to show that each of them is
needed to match the kernels.
"""
from __future__ import annotations

import numpy as np

D_IN, H, D_OUT, N_CLASS = 96, 256, 4, 3
EDGES = 12
SHAPES = {"w1": (D_IN, H), "b1": (H,), "w2": (H, H), "b2": (H,), "w3": (H, D_OUT),
          "b3": (D_OUT,)}
ORDER = ("w1", "b1", "w2", "b2", "w3", "b3")
# where the kernels round to bf16: the weights as used, the two hidden
# activations and the two hidden-layer gradients
ROUNDING = ("w", "h1", "h2", "dh2", "dh1")


def n_params() -> int:
    return sum(int(np.prod(s)) for s in SHAPES.values())


def to_bf16(x: np.ndarray) -> np.ndarray:
    """Round to fp32, then to bf16 with round-to-nearest-even; returns fp64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    nan = np.isnan(f)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def encode(genomes: np.ndarray, t: np.ndarray | int, c: int = 8) -> np.ndarray:
    """One-hot inputs [n, 96]: edge e of tile e//4 (sides N, E, S, W) sets
    column e*8 + colour; tiles beyond t contribute nothing."""
    g = np.asarray(genomes, dtype=np.uint64)
    n = g.shape[0]
    t = np.broadcast_to(np.asarray(t, dtype=np.int64), (n,))
    bits = c.bit_length() - 1
    x = np.zeros((n, D_IN), dtype=np.float64)
    for e in range(EDGES):
        present = e < 4 * t
        shift = (bits * (4 * t - 1 - e)).clip(min=0).astype(np.uint64)
        colour = ((g >> shift) & np.uint64(c - 1)).astype(np.int64)
        rows = np.nonzero(present)[0]
        x[rows, e * 8 + colour[rows]] = 1.0
    return x


def targets(cls: np.ndarray, size: np.ndarray):
    """Class index (0 UNBOUND, 1 ND_SITE or ND_RUNS, 2 DET) and log1p(size)."""
    cls = np.asarray(cls)
    k = np.where(cls == 0, 0, np.where(cls == 3, 2, 1))
    return k.astype(np.int64), np.log1p(np.asarray(size, dtype=np.float64))


def _rounder(bf16: bool, rounding, point: str):
    if bf16 and point in (ROUNDING if rounding is None else rounding):
        return to_bf16
    return lambda a: np.asarray(a, dtype=np.float64)


def forward(p: dict, x: np.ndarray, bf16: bool = True, rounding=None):
    rw = _rounder(bf16, rounding, "w")
    w1, w2, w3 = rw(p["w1"]), rw(p["w2"]), rw(p["w3"])
    a1 = x @ w1 + p["b1"]
    h1 = _rounder(bf16, rounding, "h1")(np.maximum(a1, 0.0))
    a2 = h1 @ w2 + p["b2"]
    h2 = _rounder(bf16, rounding, "h2")(np.maximum(a2, 0.0))
    out = h2 @ w3 + p["b3"]
    return out, {"h1": h1, "h2": h2, "w1": w1, "w2": w2, "w3": w3}


def loss_and_dout(out: np.ndarray, k: np.ndarray, y: np.ndarray):
    n = out.shape[0]
    logits = out[:, :N_CLASS]
    z = logits - logits.max(axis=1, keepdims=True)
    prob = np.exp(z) / np.exp(z).sum(axis=1, keepdims=True)
    ce = -np.log(prob[np.arange(n), k])
    err = out[:, N_CLASS] - y
    loss = ce.mean() + (err ** 2).mean()
    dout = np.zeros_like(out)
    dout[:, :N_CLASS] = prob
    dout[np.arange(n), k] -= 1.0
    dout[:, :N_CLASS] /= n
    dout[:, N_CLASS] = 2.0 * err / n
    return loss, dout


def backward(p: dict, x: np.ndarray, cache: dict, dout: np.ndarray, bf16: bool = True,
             rounding=None):
    h1, h2 = cache["h1"], cache["h2"]
    g = {}
    g["w3"] = h2.T @ dout
    g["b3"] = dout.sum(axis=0)
    dh2 = _rounder(bf16, rounding, "dh2")((dout @ cache["w3"].T) * (h2 > 0))
    g["w2"] = h1.T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = _rounder(bf16, rounding, "dh1")((dh2 @ cache["w2"].T) * (h1 > 0))
    g["w1"] = x.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return g


def loss_and_grads(p: dict, genomes, t, cls, size, c: int = 8, bf16: bool = True,
                   rounding=None):
    x = encode(genomes, t, c)
    k, y = targets(cls, size)
    out, cache = forward(p, x, bf16, rounding)
    loss, dout = loss_and_dout(out, k, y)
    return loss, backward(p, x, cache, dout, bf16, rounding), out


def adam(p: dict, g: dict, m: dict, v: dict, step: int, lr=1e-3, beta1=0.9, beta2=0.999,
         eps=1e-8):
    """One Adam step (step counts from 1); returns new (p, m, v)."""
    np_, nm, nv = {}, {}, {}
    for key in ORDER:
        nm[key] = beta1 * m[key] + (1 - beta1) * g[key]
        nv[key] = beta2 * v[key] + (1 - beta2) * g[key] ** 2
        mhat = nm[key] / (1 - beta1 ** step)
        vhat = nv[key] / (1 - beta2 ** step)
        np_[key] = p[key] - lr * mhat / (np.sqrt(vhat) + eps)
    return np_, nm, nv


def random_params(seed: int, scale: float = 1.0) -> dict:
    """Seeded He-scaled parameters (a test input, not the library's init)."""
    rng = np.random.default_rng(seed)
    p = {}
    for key in ORDER:
        shape = SHAPES[key]
        fan_in = shape[0] if len(shape) == 2 else 1
        std = np.sqrt(2.0 / fan_in) if len(shape) == 2 else 0.05
        p[key] = (rng.standard_normal(shape) * std * scale).astype(np.float32).astype(np.float64)
    return p


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in ORDER])


def unflatten(v: np.ndarray) -> dict:
    out, at = {}, 0
    for k in ORDER:
        n = int(np.prod(SHAPES[k]))
        out[k] = np.asarray(v[at:at + n], dtype=np.float64).reshape(SHAPES[k])
        at += n
    return out

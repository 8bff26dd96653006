"""ctypes binding of the CPU oracle (libjatam_oracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark.  The product path never imports this module.
Records are numpy structured arrays with the 16-byte layout
{int32 cls, int32 size, uint32 hash, int32 steps}.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjatam_oracle.so")

UNBOUND, ND_SITE, ND_RUNS, DET = 0, 1, 2, 3
CLASS_NAMES = {UNBOUND: "UNBOUND", ND_SITE: "ND_SITE", ND_RUNS: "ND_RUNS", DET: "DET"}
EV_NONE, EV_UNBOUND, EV_AMBIG = 0, 1, 2

RECORD = np.dtype([("cls", "<i4"), ("size", "<i4"), ("hash", "<u4"), ("steps", "<i4")])
ITEM = np.dtype([("genome", "<u8"), ("rng_id", "<u8"), ("t", "u1"), ("grid", "u1"),
                 ("pad", "u1", (6,))])

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _build
            _build.build()
        L = ctypes.CDLL(LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.jref_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.jref_philox4x32_10.restype = None
        L.jref_oaat.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.jref_oaat.restype = ctypes.c_uint32
        L.jref_default_rng_id.argtypes = [ctypes.c_uint64, ctypes.c_int]
        L.jref_default_rng_id.restype = ctypes.c_uint64
        L.jref_shape_hash_d4.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        L.jref_shape_hash_d4.restype = ctypes.c_uint32
        L.jref_check_args.argtypes = [ctypes.c_int] * 4
        L.jref_check_args.restype = ctypes.c_int
        L.jref_classify_one.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
        L.jref_classify_one.restype = ctypes.c_int
        L.jref_classify.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                    ctypes.c_void_p, ctypes.c_int]
        L.jref_classify.restype = ctypes.c_int
        L.jref_classify_range.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int]
        L.jref_classify_range.restype = ctypes.c_int
        L.jref_classify_items.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p,
                                          ctypes.c_int]
        L.jref_classify_items.restype = ctypes.c_int
        L.jref_classify_range_run0.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_int]
        L.jref_classify_range_run0.restype = ctypes.c_int
        L.jref_ga_offspring.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p]
        L.jref_ga_offspring.restype = ctypes.c_int
        L.jref_ga_step.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                   ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int]
        L.jref_ga_step.restype = ctypes.c_int
        L.jref_true_class.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int64, ctypes.c_void_p]
        L.jref_true_class.restype = ctypes.c_int
        L.jref_trace_run.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                     ctypes.c_void_p, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.jref_trace_run.restype = ctypes.c_int
        _lib = L
    return _lib


def philox4x32_10(ctr, key) -> tuple:
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().jref_philox4x32_10(c, k, o)
    return tuple(int(v) for v in o)


def oaat(data: bytes) -> int:
    buf = ctypes.create_string_buffer(bytes(data), max(len(data), 1))
    return int(lib().jref_oaat(buf, len(data)))


def default_rng_id(genome: int, t: int) -> int:
    return int(lib().jref_default_rng_id(genome, t))


def shape_hash_d4(mask: np.ndarray) -> int:
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    h, w = m.shape
    return int(lib().jref_shape_hash_d4(m.ctypes.data, w, h))


def shape_hash_c4(mask: np.ndarray) -> int:
    """Shape hash over the four rotations only (§3.3)."""
    L = lib()
    L.jref_shape_hash_c4.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    L.jref_shape_hash_c4.restype = ctypes.c_uint32
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    h, w = m.shape
    return int(L.jref_shape_hash_c4(m.ctypes.data, w, h))


VARIANT_C4, VARIANT_LIFO = 1, 2


def classify_variant(genomes, t: int, variant: int, c: int = 8, grid: int = 16, runs: int = 20,
                     seed: int = 1, first: int = 0, n: int | None = None,
                     threads: int = 0) -> np.ndarray:
    """Classification with the C4 hash and/or the LIFO movelist traversal;
    genomes None means the range first .. first + n - 1."""
    L = lib()
    L.jref_classify_variant.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_int]
    L.jref_classify_variant.restype = ctypes.c_int
    g = None if genomes is None else np.ascontiguousarray(genomes, dtype=np.uint64)
    n = len(g) if g is not None else n
    out = np.zeros(n, dtype=RECORD)
    rc = L.jref_classify_variant(g.ctypes.data if g is not None else None, first, n, t, c, grid,
                                 runs, seed, variant, out.ctypes.data, threads)
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (rc={rc})")
    return out


def trace_run_variant(genome: int, t: int, run: int, variant: int, c: int = 8, grid: int = 16,
                      seed: int = 1, rng_id: int | None = None):
    """trace_run with a traversal variant."""
    L = lib()
    L.jref_trace_run_variant.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.jref_trace_run_variant.restype = ctypes.c_int
    rid = default_rng_id(genome, t) if rng_id is None else rng_id
    cap = (grid + 1) * (grid + 1)
    cells = np.zeros(cap, dtype=np.int32)
    ev, ch = ctypes.c_int(0), ctypes.c_int(0)
    n = L.jref_trace_run_variant(genome, rid, t, c, grid, run, seed, variant, cells.ctypes.data,
                                 cap, ctypes.byref(ev), ctypes.byref(ch))
    if n < 0:
        raise ValueError("oracle rejected arguments")
    W = grid + 1
    return [(int(p) % W, int(p) // W) for p in cells[:n]], int(ev.value), int(ch.value)


def check_args(t: int, c: int, grid: int, runs: int) -> int:
    return int(lib().jref_check_args(t, c, grid, runs))


def classify_one(genome: int, t: int, c: int = 8, grid: int = 16, runs: int = 20,
                 seed: int = 1, rng_id: int | None = None, with_occupancy: bool = False):
    """Returns (cls, size, hash, steps) [, occupancy (G+1)x(G+1) uint8]."""
    rid = default_rng_id(genome, t) if rng_id is None else rng_id
    out = np.zeros(1, dtype=RECORD)
    occ = np.zeros((grid + 1, grid + 1), dtype=np.uint8) if with_occupancy else None
    rc = lib().jref_classify_one(genome, rid, t, c, grid, runs, seed, out.ctypes.data,
                                 occ.ctypes.data if occ is not None else None)
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (rc={rc})")
    rec = tuple(int(out[0][f]) for f in ("cls", "size", "hash", "steps"))
    return (rec, occ) if with_occupancy else rec


def classify(genomes: np.ndarray, t: int, c: int = 8, grid: int = 16, runs: int = 20,
             seed: int = 1, threads: int = 0) -> np.ndarray:
    g = np.ascontiguousarray(genomes, dtype=np.uint64)
    out = np.zeros(g.shape[0], dtype=RECORD)
    rc = lib().jref_classify(g.ctypes.data, g.shape[0], t, c, grid, runs, seed,
                             out.ctypes.data, threads)
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (rc={rc})")
    return out


def classify_range(first: int, n: int, t: int, c: int = 8, grid: int = 16, runs: int = 20,
                   seed: int = 1, threads: int = 0) -> np.ndarray:
    out = np.zeros(n, dtype=RECORD)
    rc = lib().jref_classify_range(first, n, t, c, grid, runs, seed, out.ctypes.data, threads)
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (rc={rc})")
    return out


def classify_range_run0(first: int, n: int, t: int, c: int = 8, grid: int = 16,
                        runs: int = 20, seed: int = 1, threads: int = 0, forced: bool = False):
    """Records plus (steps, event, choice) of every genotype's first run, and
    with forced=True also a flag per genotype: bit 0 set if the first run's
    shape is forced, bit 1 set if it is guarded."""
    out = np.zeros(n, dtype=RECORD)
    s0 = np.zeros(n, dtype=np.int32)
    e0 = np.zeros(n, dtype=np.int8)
    c0 = np.zeros(n, dtype=np.int8)
    f0 = np.zeros(n, dtype=np.int8)
    rc = lib().jref_classify_range_run0(first, n, t, c, grid, runs, seed, out.ctypes.data,
                                        s0.ctypes.data, e0.ctypes.data, c0.ctypes.data,
                                        f0.ctypes.data, threads)
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (rc={rc})")
    return (out, s0, e0, c0, f0) if forced else (out, s0, e0, c0)


def classify_items(items: np.ndarray, c: int = 8, runs: int = 20, seed: int = 1,
                   threads: int = 0) -> np.ndarray:
    it = np.ascontiguousarray(items, dtype=ITEM)
    out = np.zeros(it.shape[0], dtype=RECORD)
    rc = lib().jref_classify_items(it.ctypes.data, it.shape[0], c, runs, seed,
                                   out.ctypes.data, threads)
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (rc={rc})")
    return out


def trace_run(genome: int, t: int, run: int, c: int = 8, grid: int = 16, seed: int = 1,
              rng_id: int | None = None):
    """Placed cells of one run in placement order as (x, y), plus event and choice."""
    rid = default_rng_id(genome, t) if rng_id is None else rng_id
    cap = (grid + 1) * (grid + 1)
    cells = np.zeros(cap, dtype=np.int32)
    ev, ch = ctypes.c_int(0), ctypes.c_int(0)
    n = lib().jref_trace_run(genome, rid, t, c, grid, run, seed, cells.ctypes.data, cap,
                             ctypes.byref(ev), ctypes.byref(ch))
    if n < 0:
        raise ValueError("oracle rejected arguments")
    W = grid + 1
    return [(int(p) % W, int(p) // W) for p in cells[:n]], int(ev.value), int(ch.value)


class GAParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("tournament", ctypes.c_int),
                ("mut_num", ctypes.c_int), ("mut_den", ctypes.c_int)]


def ga_offspring(pop: np.ndarray, fit: np.ndarray, t: int, generation: int, n_out: int | None = None,
                 c: int = 8, seed: int = 5, tournament: int = 4, mut=(1, 12)) -> np.ndarray:
    pop = np.ascontiguousarray(pop, dtype=np.uint64)
    fit = np.ascontiguousarray(fit, dtype=np.int32)
    n_out = pop.shape[0] if n_out is None else n_out
    out = np.zeros(n_out, dtype=np.uint64)
    p = GAParams(seed, tournament, mut[0], mut[1])
    rc = lib().jref_ga_offspring(pop.ctypes.data, fit.ctypes.data, pop.shape[0], t, c,
                                 ctypes.byref(p), generation, n_out, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (rc={rc})")
    return out


def ga_step(pop: np.ndarray, fit: np.ndarray, t: int, generation: int, c: int = 8,
            grid: int = 32, runs: int = 20, seed: int = 1, ga_seed: int = 5,
            tournament: int = 4, mut=(1, 12), threads: int = 0):
    pop = np.ascontiguousarray(pop, dtype=np.uint64)
    fit = np.ascontiguousarray(fit, dtype=np.int32)
    nxt = np.zeros_like(pop)
    nfit = np.zeros_like(fit)
    p = GAParams(ga_seed, tournament, mut[0], mut[1])
    rc = lib().jref_ga_step(pop.ctypes.data, fit.ctypes.data, pop.shape[0], t, c, grid, runs,
                            seed, ctypes.byref(p), generation, nxt.ctypes.data, nfit.ctypes.data,
                            threads)
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (rc={rc})")
    return nxt, nfit


TRUE_CAPPED = -2


def true_class(genomes: np.ndarray, t: int, c: int = 8, grid: int = 16,
               cap: int = 1 << 20) -> np.ndarray:
    """Exhaustive true class of each genome: records with cls DET (size, hash
    of the only terminal shape), ND_SITE (not deterministic) or TRUE_CAPPED;
    steps = states visited."""
    g = np.ascontiguousarray(genomes, dtype=np.uint64)
    out = np.zeros(g.shape[0], dtype=RECORD)
    rc = lib().jref_true_class(g.ctypes.data, g.shape[0], t, c, grid, cap, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (rc={rc})")
    return out


# ---------------------------------------------------------------------------
# Robustness and evolvability (§1.1): the proportion of single mutations that
# leave the phenotype unchanged, and the number of different phenotypes that
# single mutations reach.  A single mutation flips one genome bit (the
# mutation operator of App. B.3 flips bits), so a t-tile genotype with
# b = log2 c bits per colour has 4*t*b single mutants.  The phenotype of a
# record is UNBOUND, non-deterministic (ND_SITE or ND_RUNS) or the
# deterministic shape (size and D4 hash).
# ---------------------------------------------------------------------------
def mutants(genomes: np.ndarray, t: int, c: int = 8) -> np.ndarray:
    """[n, 4*t*b] genomes: column k has bit k flipped (bit 0 the lowest)."""
    g = np.asarray(genomes, dtype=np.uint64)
    nbits = 4 * t * (c.bit_length() - 1)
    flips = np.uint64(1) << np.arange(nbits, dtype=np.uint64)
    return g[:, None] ^ flips[None, :]


def phenotype_keys(rec: np.ndarray) -> np.ndarray:
    """One uint64 per record: 1 for UNBOUND, 2 for either ND class, and for a
    DET record 4 + size * 2^32 + hash (never 1 or 2)."""
    cls = rec["cls"].astype(np.int64)
    det = (np.uint64(4) + (rec["size"].astype(np.uint64) << np.uint64(32))
           + rec["hash"].astype(np.uint64))
    key = np.where(cls == DET, det, np.where(cls == UNBOUND, np.uint64(1), np.uint64(2)))
    return key.astype(np.uint64)


def neighbourhood(genomes: np.ndarray, t: int, c: int = 8, grid: int = 16, runs: int = 20,
                  seed: int = 1, threads: int = 0):
    """(robust, evolv) per genotype: robust = how many of its single mutants
    have its phenotype; evolv = how many distinct phenotypes other than its
    own its single mutants have.  Every genotype and mutant is classified by
    the oracle with its default rng_id."""
    g = np.ascontiguousarray(genomes, dtype=np.uint64)
    m = mutants(g, t, c)
    own = phenotype_keys(classify(g, t, c=c, grid=grid, runs=runs, seed=seed,
                                  threads=threads))
    mk = phenotype_keys(classify(m.ravel(), t, c=c, grid=grid, runs=runs, seed=seed,
                                 threads=threads)).reshape(m.shape)
    robust = np.sum(mk == own[:, None], axis=1).astype(np.int32)
    evolv = np.zeros(len(g), dtype=np.int32)
    for i in range(len(g)):
        others = set(mk[i].tolist())
        others.discard(int(own[i]))
        evolv[i] = len(others)
    return robust, evolv


# ---------------------------------------------------------------------------
# The paper's GA (roulette selection, single-point crossover, Poisson bit
# flips) and its Fujiyama test bed (jatam_roulette_oracle.c).
# ---------------------------------------------------------------------------
class RouletteParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("length", ctypes.c_int32),
                ("crossover", ctypes.c_int32), ("lambda_", ctypes.c_double)]


def _roulette_lib():
    L = lib()
    if not getattr(L, "_roulette_ready", False):
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        L.jref_roulette_lookup.argtypes = [vp, i64, ctypes.c_uint64]
        L.jref_roulette_lookup.restype = i64
        L.jref_poisson_thresholds.argtypes = [ctypes.c_double, ctypes.c_int, vp]
        L.jref_poisson_thresholds.restype = None
        L.jref_roulette_offspring.argtypes = [vp, vp, i64, vp, ctypes.c_int32, i64, vp]
        L.jref_roulette_offspring.restype = ctypes.c_int
        L.jref_fujiyama.argtypes = [vp, i64, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
        L.jref_fujiyama.restype = ctypes.c_int
        L._roulette_ready = True
    return L


def roulette_lookup(weights, cutoff: int) -> int:
    w = np.ascontiguousarray(weights, dtype=np.uint32)
    return int(_roulette_lib().jref_roulette_lookup(w.ctypes.data, len(w), cutoff))


def poisson_thresholds(lam: float, length: int) -> np.ndarray:
    thr = np.zeros(length + 1, dtype=np.uint64)
    _roulette_lib().jref_poisson_thresholds(lam, length, thr.ctypes.data)
    return thr


def roulette_offspring(pop, fit, generation: int, length: int, lam: float, crossover: bool = True,
                       seed: int = 5, n_out: int | None = None) -> np.ndarray:
    pop = np.ascontiguousarray(pop, dtype=np.uint64)
    fit = np.ascontiguousarray(fit, dtype=np.uint32)
    n_out = len(pop) if n_out is None else n_out
    out = np.zeros(n_out, dtype=np.uint64)
    p = RouletteParams(seed, length, 1 if crossover else 0, lam)
    rc = _roulette_lib().jref_roulette_offspring(pop.ctypes.data, fit.ctypes.data, len(pop),
                                                 ctypes.byref(p), generation, n_out,
                                                 out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (rc={rc})")
    return out


def fujiyama(n: int, length: int, lam: float, target: int, cutoff: int, seed: int = 5,
             crossover: bool = True):
    """(discovery, adaptation, final population) of one simulation."""
    p = RouletteParams(seed, length, 1 if crossover else 0, lam)
    d, a = ctypes.c_int32(0), ctypes.c_int32(0)
    final = np.zeros(n, dtype=np.uint64)
    rc = _roulette_lib().jref_fujiyama(ctypes.byref(p), n, target, cutoff, ctypes.byref(d),
                                       ctypes.byref(a), final.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (rc={rc})")
    return int(d.value), int(a.value), final

"""Python binding of the HIP library (libjatam.so): argument marshalling only.

Every entry point mirrors an extern "C" function of include/jatam.h; the
tensors' device pointers and torch's current HIP stream are handed straight
to the library, which does all the work in its own kernels.  There is no
CPU fallback: if the library or a GPU is missing, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjatam.so")

UNBOUND, ND_SITE, ND_RUNS, DET, INVALID, UNDECIDED = 0, 1, 2, 3, -1, -2
CLASS_NAMES = {UNBOUND: "UNBOUND", ND_SITE: "ND_SITE", ND_RUNS: "ND_RUNS", DET: "DET",
               INVALID: "INVALID"}
E_INVALID_ARG, E_UNSUPPORTED, E_HIP = -1, -2, -3

# jatam_result_t: int32 cls, int32 size, uint32 hash, int32 steps
RECORD_FIELDS = ("cls", "size", "hash", "steps")

_lib = None


class JatamError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {strerror(code)} ({code})")
        self.code = code


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2205_15311_amd.build_lib`")
        L = ctypes.CDLL(LIB_PATH)
        i64, i32, u64, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p
        L.jatam_classify.argtypes = [vp, i64, i32, i32, i32, i32, u64, vp, vp]
        L.jatam_classify.restype = i32
        L.jatam_classify_range.argtypes = [u64, i64, i32, i32, i32, i32, u64, vp, vp]
        L.jatam_classify_range.restype = i32
        L.jatam_strerror.argtypes = [i32]
        L.jatam_strerror.restype = ctypes.c_char_p
        L.jatam_abi_version.argtypes = []
        L.jatam_abi_version.restype = i32
        L.jatam_batch_create.argtypes = [i64, ctypes.POINTER(vp)]
        L.jatam_batch_create.restype = i32
        L.jatam_batch_destroy.argtypes = [vp]
        L.jatam_batch_destroy.restype = i32
        L.jatam_batch_classify.argtypes = [vp, vp, i64, i32, i32, i32, i32, u64, vp, vp, vp]
        L.jatam_batch_classify.restype = i32
        L.jatam_batch_classify_range.argtypes = [vp, u64, i64, i32, i32, i32, i32, u64, vp, vp,
                                                 vp]
        L.jatam_batch_classify_range.restype = i32
        L.jatam_batch_classify_items.argtypes = [vp, vp, i64, i32, i32, u64, vp, vp, vp]
        L.jatam_batch_classify_items.restype = i32
        L.jatam_ga_offspring.argtypes = [vp, vp, i64, i32, i32, vp, ctypes.c_int32, i64, vp, vp]
        L.jatam_ga_offspring.restype = i32
        L.jatam_ga_step.argtypes = [vp, vp, vp, i64, i32, i32, i32, i32, u64, vp,
                                    ctypes.c_int32, vp, vp, vp, vp]
        L.jatam_ga_step.restype = i32
        L.jatam_mlp_create.argtypes = [i64, i32, ctypes.POINTER(vp)]
        L.jatam_mlp_create.restype = i32
        L.jatam_mlp_destroy.argtypes = [vp]
        L.jatam_mlp_destroy.restype = i32
        L.jatam_mlp_init.argtypes = [vp, u64, vp]
        L.jatam_mlp_init.restype = i32
        L.jatam_mlp_set_params.argtypes = [vp, vp, vp]
        L.jatam_mlp_set_params.restype = i32
        L.jatam_mlp_get_params.argtypes = [vp, vp, vp, vp]
        L.jatam_mlp_get_params.restype = i32
        L.jatam_mlp_forward.argtypes = [vp, vp, vp, i32, i64, vp, vp]
        L.jatam_mlp_forward.restype = i32
        L.jatam_mlp_train_step.argtypes = [vp, vp, vp, i32, vp, i64, ctypes.c_float, vp, vp]
        L.jatam_mlp_train_step.restype = i32
        L.jatam_mlp_score.argtypes = [vp, vp, vp, i32, i64, vp, vp]
        L.jatam_mlp_score.restype = i32
        L.jatam_mlp_predict.argtypes = [vp, i32, vp, vp, i32, i64, vp, vp]
        L.jatam_mlp_predict.restype = i32
        L.jatam_ga_create.argtypes = [i64, ctypes.POINTER(vp)]
        L.jatam_ga_create.restype = i32
        L.jatam_ga_destroy.argtypes = [vp]
        L.jatam_ga_destroy.restype = i32
        L.jatam_select_top.argtypes = [vp, vp, i64, i64, vp, vp]
        L.jatam_select_top.restype = i32
        L.jatam_ga_step_screened.argtypes = [vp, vp, vp, vp, vp, i64, i32, i32, i32, i32, u64, vp,
                                             ctypes.c_int32, i32, vp, vp, vp]
        L.jatam_ga_step_screened.restype = i32
        L.jatam_batch_set_refill.argtypes = [vp, i32]
        L.jatam_batch_set_refill.restype = i32
        L.jatam_batch_set_timing.argtypes = [vp, i32]
        L.jatam_batch_set_timing.restype = i32
        L.jatam_batch_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int), i32]
        L.jatam_batch_stage_times.restype = i32
        L.jatam_batch_stage_name.argtypes = [i32]
        L.jatam_batch_stage_name.restype = ctypes.c_char_p
        L.jatam_batch_classify_items_ordered.argtypes = [vp, vp, vp, i64, i32, i32, u64, vp, vp,
                                                         vp]
        L.jatam_batch_classify_items_ordered.restype = i32
        L.jatam_batch_get_tuning.argtypes = [vp, i32, ctypes.POINTER(Tuning)]
        L.jatam_batch_get_tuning.restype = i32
        L.jatam_batch_set_tuning.argtypes = [vp, i32, ctypes.POINTER(Tuning)]
        L.jatam_batch_set_tuning.restype = i32
        L.jatam_batch_autotune.argtypes = [vp, u64, i64, i32, i32, i32, i32, u64, vp,
                                           ctypes.POINTER(Tuning), vp]
        L.jatam_batch_autotune.restype = i32
        L.jatam_batch_autotune_cached.argtypes = [vp, ctypes.c_char_p, u64, i64, i32, i32, i32,
                                                  i32, u64, vp, ctypes.POINTER(Tuning),
                                                  ctypes.POINTER(ctypes.c_int), vp]
        L.jatam_batch_autotune_cached.restype = i32
        L.jatam_batch_autotune_log.argtypes = [vp, i32, ctypes.POINTER(Tuning),
                                               ctypes.POINTER(ctypes.c_double)]
        L.jatam_batch_autotune_log.restype = i32
        L.jatam_batch_enumerate.argtypes = [vp, u64, i64, i64, i32, i32, i32, i32, u64, vp, vp,
                                            vp, i64, vp]
        L.jatam_classify_batch.argtypes = [vp, vp, i64, i32, i32, u64, vp, vp, vp, vp, vp]
        L.jatam_classify_batch.restype = i32
        L.jatam_classify_static.argtypes = [vp, i64, i32, i32, i32, i32, u64, vp, vp, vp]
        L.jatam_classify_static.restype = i32
        L.jatam_batch_enumerate.restype = i32
        L.jatam_shape_histogram.argtypes = [vp, i64, vp, i64, vp, vp]
        L.jatam_classify_variant.argtypes = [vp, u64, i64, i32, i32, i32, i32, u64, i32, vp, vp]
        L.jatam_classify_variant.restype = i32
        L.jatam_single_mutants.argtypes = [vp, u64, i64, i32, i32, vp, vp]
        L.jatam_single_mutants.restype = i32
        L.jatam_neighbourhood.argtypes = [vp, vp, i64, i32, i32, vp, vp]
        L.jatam_neighbourhood.restype = i32
        L.jatam_neighbourhood_space.argtypes = [vp, u64, i64, i32, i32, vp, vp]
        L.jatam_neighbourhood_space.restype = i32
        L.jatam_roulette_work_words.argtypes = [i64]
        L.jatam_roulette_work_words.restype = i64
        L.jatam_roulette_offspring.argtypes = [vp, vp, i64, vp, ctypes.c_int32, i64, vp, vp, vp]
        L.jatam_roulette_offspring.restype = i32
        L.jatam_fujiyama.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp]
        L.jatam_fujiyama.restype = i32
        L.jatam_shape_histogram.restype = i32
        L.jatam_batch_classify_range_ordered.argtypes = [vp, u64, i64, i32, i32, i32, i32, u64,
                                                         vp, vp, vp, vp]
        L.jatam_batch_classify_range_ordered.restype = i32
        L.jatam_order_work_words.argtypes = [i64]
        L.jatam_order_work_words.restype = i64
        L.jatam_order_by_cost.argtypes = [vp, i64, vp, vp, vp]
        L.jatam_order_by_cost.restype = i32
        L.jatam_truth_create.argtypes = [i64, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(vp)]
        L.jatam_truth_create.restype = i32
        L.jatam_truth_destroy.argtypes = [vp]
        L.jatam_truth_destroy.restype = i32
        L.jatam_true_class.argtypes = [vp, vp, i64, i32, i32, i32, i64, vp, vp]
        L.jatam_true_class.restype = i32
        L.jatam_true_class_range.argtypes = [vp, u64, i64, i32, i32, i32, i64, vp, vp]
        L.jatam_true_class_range.restype = i32
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().jatam_strerror(code).decode()


def abi_version() -> int:
    return int(lib().jatam_abi_version())


def _stream_handle(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _check(rc: int, where: str) -> None:
    if rc != 0:
        raise JatamError(rc, where)


def _records(n: int, device, out):
    if out is None:
        return torch.empty((n, 4), dtype=torch.int32, device=device)
    if out.dtype != torch.int32 or tuple(out.shape) != (n, 4) or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 tensor of shape (n, 4)")
    return out


def classify(genotypes: torch.Tensor, t: int, c: int = 8, grid_limit: int = 16,
             runs: int = 20, seed: int = 1, out: torch.Tensor | None = None,
             stream=None) -> torch.Tensor:
    """jatam_classify: records (n, 4) int32 [cls, size, hash bits, steps]."""
    if genotypes.dtype not in (torch.int64, torch.uint64) or genotypes.dim() != 1:
        raise ValueError("genotypes must be a 1-D int64/uint64 tensor")
    if not genotypes.is_cuda or not genotypes.is_contiguous():
        raise ValueError("genotypes must be a contiguous device tensor")
    n = genotypes.shape[0]
    rec = _records(n, genotypes.device, out)
    rc = lib().jatam_classify(genotypes.data_ptr(), n, t, c, grid_limit, runs, seed,
                              rec.data_ptr(), _stream_handle(stream))
    _check(rc, "jatam_classify")
    return rec


def classify_range(first: int, n: int, t: int, c: int = 8, grid_limit: int = 16,
                   runs: int = 20, seed: int = 1, out: torch.Tensor | None = None,
                   device="cuda", stream=None) -> torch.Tensor:
    """jatam_classify_range: genome i = first + i."""
    rec = _records(n, device, out)
    rc = lib().jatam_classify_range(first, n, t, c, grid_limit, runs, seed, rec.data_ptr(),
                                    _stream_handle(stream))
    _check(rc, "jatam_classify_range")
    return rec


VARIANT_C4, VARIANT_LIFO = 1, 2   # jatam_classify_variant flags


def classify_variant(genotypes: torch.Tensor | None, t: int, variant: int, c: int = 8,
                     grid_limit: int = 16, runs: int = 20, seed: int = 1, first: int = 0,
                     n: int | None = None, out: torch.Tensor | None = None, device="cuda",
                     stream=None) -> torch.Tensor:
    """jatam_classify_variant: VARIANT_C4 and/or VARIANT_LIFO; genotypes None
    means the range first + i."""
    if genotypes is not None:
        n = genotypes.shape[0]
        device = genotypes.device
    rec = _records(n, device, out)
    rc = lib().jatam_classify_variant(genotypes.data_ptr() if genotypes is not None else None,
                                      first, n, t, c, grid_limit, runs, seed, variant,
                                      rec.data_ptr(), _stream_handle(stream))
    _check(rc, "jatam_classify_variant")
    return rec


STATIC_MAX_N = 1 << 18


def classify_static(genotypes: torch.Tensor, t: int, c: int = 8, grid_limit: int = 16,
                    runs: int = 20, seed: int = 1, out: torch.Tensor | None = None,
                    tally: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """jatam_classify_static: the pipelined path with the library's static
    device array as its workspace (n <= 2^18; no device allocation by the
    library)."""
    if genotypes.dtype not in (torch.int64, torch.uint64) or genotypes.dim() != 1:
        raise ValueError("genotypes must be a 1-D int64/uint64 tensor")
    if not genotypes.is_cuda or not genotypes.is_contiguous():
        raise ValueError("genotypes must be a contiguous device tensor")
    n = genotypes.shape[0]
    rec = _records(n, genotypes.device, out)
    rc = lib().jatam_classify_static(genotypes.data_ptr(), n, t, c, grid_limit, runs, seed,
                                     rec.data_ptr(), Batch._tally_ptr(tally),
                                     _stream_handle(stream))
    _check(rc, "jatam_classify_static")
    return rec


def order_by_cost(scores: torch.Tensor, order: torch.Tensor | None = None,
                  work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """jatam_order_by_cost: a queue order (int32 tensor, a permutation of
    0..n-1) by descending score bucket.  `work` (int32, at least
    jatam_order_work_words(n) elements) may be passed to avoid allocating."""
    if scores.dtype != torch.float32 or scores.dim() != 1 or not scores.is_cuda \
            or not scores.is_contiguous():
        raise ValueError("scores must be a contiguous 1-D float32 device tensor")
    n = scores.shape[0]
    words = int(lib().jatam_order_work_words(n))
    if order is None:
        order = torch.empty(n, dtype=torch.int32, device=scores.device)
    if work is None:
        work = torch.empty(max(words, 1), dtype=torch.int32, device=scores.device)
    if order.numel() != n or work.numel() < words:
        raise ValueError("order must hold n entries and work the scratch words")
    rc = lib().jatam_order_by_cost(scores.data_ptr(), n, order.data_ptr(), work.data_ptr(),
                                   _stream_handle(stream))
    _check(rc, "jatam_order_by_cost")
    return order


def records_to_numpy(rec: torch.Tensor):
    """(n, 4) int32 records -> numpy structured array (cls, size, hash, steps)."""
    import numpy as np
    dt = np.dtype([("cls", "<i4"), ("size", "<i4"), ("hash", "<u4"), ("steps", "<i4")])
    return rec.detach().cpu().contiguous().numpy().view(dt).reshape(-1)


class GAParams(ctypes.Structure):
    """jatam_ga_params_t."""
    _fields_ = [("seed", ctypes.c_uint64), ("tournament", ctypes.c_int32),
                ("mut_num", ctypes.c_int32), ("mut_den", ctypes.c_int32),
                ("pad", ctypes.c_int32)]

    def __init__(self, seed=5, tournament=4, mut_num=1, mut_den=12):
        super().__init__(seed, tournament, mut_num, mut_den, 0)


def _check_pop(pop, fit):
    if pop.dtype not in (torch.int64, torch.uint64) or pop.dim() != 1 or not pop.is_cuda:
        raise ValueError("pop must be a 1-D int64/uint64 device tensor")
    if fit.dtype != torch.int32 or fit.shape != pop.shape or not fit.is_cuda:
        raise ValueError("fit must be an int32 device tensor shaped like pop")
    if not pop.is_contiguous() or not fit.is_contiguous():
        raise ValueError("pop and fit must be contiguous")


def ga_offspring(pop: torch.Tensor, fit: torch.Tensor, t: int, params: GAParams,
                 generation: int, c: int = 8, n_out: int | None = None,
                 out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """jatam_ga_offspring: n_out offspring genomes (int64 tensor)."""
    _check_pop(pop, fit)
    n_out = pop.shape[0] if n_out is None else n_out
    if out is None:
        out = torch.empty(n_out, dtype=torch.int64, device=pop.device)
    rc = lib().jatam_ga_offspring(pop.data_ptr(), fit.data_ptr(), pop.shape[0], t, c,
                                  ctypes.byref(params), generation, n_out, out.data_ptr(),
                                  _stream_handle(stream))
    _check(rc, "jatam_ga_offspring")
    return out


# jatam_item_t: uint64 genome, uint64 rng_id, uint8 t, uint8 grid, 6 pad bytes
ITEM_BYTES = 24


class Tuning(ctypes.Structure):
    """jatam_tuning_t: launch parameters of one grid class."""
    _fields_ = [("refill", ctypes.c_int), ("first_waves", ctypes.c_int),
                ("repeat_waves", ctypes.c_int), ("wide_layout", ctypes.c_int),
                ("claim_share", ctypes.c_int), ("claim_chunks", ctypes.c_int),
                ("repeat_mapping", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


SHAPE_COUNT_BYTES = 16


def shape_histogram(records: torch.Tensor, table: torch.Tensor | None = None,
                    capacity: int = 4096, overflow: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    """jatam_shape_histogram: adds the DET records to a device table of
    jatam_shape_count_t entries, held as an int64 tensor (capacity, 2)
    [hash | size << 32, count]; a new zeroed table if none is given."""
    if records.dtype != torch.int32 or records.dim() != 2 or records.shape[1] != 4 \
            or not records.is_cuda or not records.is_contiguous():
        raise ValueError("records must be a contiguous device int32 tensor (n, 4)")
    if table is None:
        table = torch.zeros((capacity, 2), dtype=torch.int64, device=records.device)
    if table.dtype != torch.int64 or table.dim() != 2 or table.shape[1] != 2 \
            or not table.is_cuda or not table.is_contiguous():
        raise ValueError("table must be a contiguous device int64 tensor (capacity, 2)")
    if overflow is not None and (overflow.dtype != torch.int64 or overflow.numel() != 1):
        raise ValueError("overflow must be a device int64 tensor of one element")
    rc = lib().jatam_shape_histogram(records.data_ptr(), records.shape[0], table.data_ptr(),
                                     table.shape[0],
                                     overflow.data_ptr() if overflow is not None else None,
                                     _stream_handle(stream))
    _check(rc, "jatam_shape_histogram")
    return table


def _records_arg(rec: torch.Tensor, name: str) -> None:
    if rec.dtype != torch.int32 or rec.dim() != 2 or rec.shape[1] != 4 or not rec.is_cuda \
            or not rec.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device int32 tensor (n, 4)")


def mutant_count(t: int, c: int = 8) -> int:
    """Single mutants per genotype: one per genome bit."""
    return 4 * t * (c.bit_length() - 1)


def single_mutants(genotypes: torch.Tensor | None, t: int, c: int = 8, first: int = 0,
                   n: int | None = None, out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
    """jatam_single_mutants: (n, m) int64 device tensor, entry [i, k] =
    genotype i with bit k flipped; genotypes None means the range first + i."""
    if genotypes is not None:
        n = genotypes.shape[0]
        dev = genotypes.device
    else:
        dev = torch.device("cuda", torch.cuda.current_device())
    m = mutant_count(t, c)
    if out is None:
        out = torch.empty((n, m), dtype=torch.int64, device=dev)
    _check(lib().jatam_single_mutants(genotypes.data_ptr() if genotypes is not None else None,
                                      first, n, t, c, out.data_ptr(), _stream_handle(stream)),
           "jatam_single_mutants")
    return out


def neighbourhood(own: torch.Tensor, mutant_records: torch.Tensor, t: int, c: int = 8,
                  out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """jatam_neighbourhood: (n, 2) int32 [robust, evolv] from the genotypes'
    records and their mutants' records ((n * m, 4), mutant k of genotype i
    at row i * m + k)."""
    _records_arg(own, "own")
    _records_arg(mutant_records, "mutant_records")
    n = own.shape[0]
    if mutant_records.shape[0] != n * mutant_count(t, c):
        raise ValueError("mutant_records must hold n * m records")
    if out is None:
        out = torch.empty((n, 2), dtype=torch.int32, device=own.device)
    _check(lib().jatam_neighbourhood(own.data_ptr(), mutant_records.data_ptr(), n, t, c,
                                     out.data_ptr(), _stream_handle(stream)),
           "jatam_neighbourhood")
    return out


def neighbourhood_space(space: torch.Tensor, t: int, c: int = 8, first: int = 0,
                        n: int | None = None, out: torch.Tensor | None = None,
                        stream=None) -> torch.Tensor:
    """jatam_neighbourhood_space: (n, 2) int32 [robust, evolv] of genotypes
    first .. first + n - 1, space holding the records of the whole space."""
    _records_arg(space, "space")
    if space.shape[0] != c ** (4 * t):
        raise ValueError("space must hold the records of all c^(4t) genotypes")
    n = space.shape[0] - first if n is None else n
    if out is None:
        out = torch.empty((n, 2), dtype=torch.int32, device=space.device)
    _check(lib().jatam_neighbourhood_space(space.data_ptr(), first, n, t, c, out.data_ptr(),
                                           _stream_handle(stream)),
           "jatam_neighbourhood_space")
    return out


class RouletteParams(ctypes.Structure):
    """jatam_roulette_params_t."""
    _fields_ = [("seed", ctypes.c_uint64), ("length", ctypes.c_int32),
                ("crossover", ctypes.c_int32), ("lambda_", ctypes.c_double)]


def roulette_offspring(pop: torch.Tensor, fit: torch.Tensor, generation: int, length: int,
                       lam: float, crossover: bool = True, seed: int = 5,
                       n_out: int | None = None, out: torch.Tensor | None = None,
                       work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """jatam_roulette_offspring: pop int64 (n,), fit int32/uint32 (n,) device
    tensors; returns n_out offspring (int64)."""
    n = pop.shape[0]
    n_out = n if n_out is None else n_out
    if pop.dtype != torch.int64 or fit.dtype not in (torch.int32, torch.uint32) \
            or fit.shape[0] != n or not pop.is_contiguous() or not fit.is_contiguous():
        raise ValueError("pop must be int64 (n,), fit int32 (n,), both contiguous")
    if out is None:
        out = torch.empty(n_out, dtype=torch.int64, device=pop.device)
    if work is None:
        work = torch.empty(int(lib().jatam_roulette_work_words(n)), dtype=torch.int32,
                           device=pop.device)
    p = RouletteParams(seed, length, 1 if crossover else 0, lam)
    _check(lib().jatam_roulette_offspring(pop.data_ptr(), fit.data_ptr(), n, ctypes.byref(p),
                                          generation, n_out, work.data_ptr(), out.data_ptr(),
                                          _stream_handle(stream)), "jatam_roulette_offspring")
    return out


def fujiyama(lambdas, sims: int, pop: int, length: int, target: int, cutoff: int,
             seed: int = 5, crossover: bool = True, final_pop: bool = False, device="cuda",
             stream=None):
    """jatam_fujiyama: (discovery, adaptation) int32 device tensors (sims,
    rates), and the final populations (sims, rates, pop) if asked."""
    lam = (ctypes.c_double * len(lambdas))(*[float(x) for x in lambdas])
    rates = len(lambdas)
    disc = torch.empty((sims, rates), dtype=torch.int32, device=device)
    adap = torch.empty((sims, rates), dtype=torch.int32, device=device)
    fin = torch.empty((sims, rates, pop), dtype=torch.int64, device=device) if final_pop \
        else None
    p = RouletteParams(seed, length, 1 if crossover else 0, 0.0)
    _check(lib().jatam_fujiyama(ctypes.byref(p), lam, rates, sims, pop, target, cutoff,
                                disc.data_ptr(), adap.data_ptr(),
                                fin.data_ptr() if fin is not None else None,
                                _stream_handle(stream)), "jatam_fujiyama")
    return (disc, adap, fin) if final_pop else (disc, adap)


def shape_table_to_numpy(table: torch.Tensor):
    """Non-empty entries of a shape table as a numpy structured array
    (hash uint32, size int32, count uint64), sorted by (size, hash)."""
    import numpy as np
    dt = np.dtype([("hash", "<u4"), ("size", "<i4"), ("count", "<u8")])
    arr = table.cpu().numpy().view(dt).reshape(-1)
    arr = arr[arr["size"] != 0]
    return np.sort(arr, order=("size", "hash"))


def make_items(genomes, t, grid, rng_ids=None):
    """Packs per-item genomes, tile counts and grids (numpy arrays) into the
    24-byte jatam_item_t layout; returns a uint8 numpy array of shape (n, 24)."""
    import numpy as np
    genomes = np.asarray(genomes, dtype=np.uint64)
    n = genomes.shape[0]
    t = np.broadcast_to(np.asarray(t, dtype=np.uint8), (n,))
    grid = np.broadcast_to(np.asarray(grid, dtype=np.uint8), (n,))
    if rng_ids is None:
        rng_ids = genomes | (t.astype(np.uint64) << np.uint64(56))
    dt = np.dtype([("genome", "<u8"), ("rng_id", "<u8"), ("t", "u1"), ("grid", "u1"),
                   ("pad", "u1", (6,))])
    arr = np.zeros(n, dtype=dt)
    arr["genome"] = genomes
    arr["rng_id"] = rng_ids
    arr["t"] = t
    arr["grid"] = grid
    return arr.view(np.uint8).reshape(n, ITEM_BYTES)


class Truth:
    """A jatam_truth_t workspace and the true-class calls (every growth order
    followed): records (n, 4) int32 [cls, size, hash bits, states], cls one
    of DET, ND_SITE, UNDECIDED (past `cap` states) or INVALID."""

    def __init__(self, max_n: int, max_level: int = 4096, waves: int = 64):
        handle = ctypes.c_void_p()
        _check(lib().jatam_truth_create(int(max_n), int(max_level), int(waves),
                                        ctypes.byref(handle)), "jatam_truth_create")
        self._h = handle
        self.max_n = int(max_n)

    def close(self) -> None:
        if self._h is not None and self._h.value:
            _check(lib().jatam_truth_destroy(self._h), "jatam_truth_destroy")
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def true_class(self, genotypes: torch.Tensor, t: int, c: int = 8, grid_limit: int = 16,
                   cap: int = 1 << 20, out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
        """jatam_true_class over a device genome array."""
        if genotypes.dtype not in (torch.int64, torch.uint64) or genotypes.dim() != 1:
            raise ValueError("genotypes must be a 1-D int64/uint64 tensor")
        if not genotypes.is_cuda or not genotypes.is_contiguous():
            raise ValueError("genotypes must be a contiguous device tensor")
        n = genotypes.shape[0]
        rec = _records(n, genotypes.device, out)
        rc = lib().jatam_true_class(self._h, genotypes.data_ptr(), n, t, c, grid_limit, cap,
                                    rec.data_ptr(), _stream_handle(stream))
        _check(rc, "jatam_true_class")
        return rec

    def true_class_range(self, first: int, n: int, t: int, c: int = 8, grid_limit: int = 16,
                         cap: int = 1 << 20, out: torch.Tensor | None = None, device="cuda",
                         stream=None) -> torch.Tensor:
        """jatam_true_class_range: genome i = first + i."""
        rec = _records(n, device, out)
        rc = lib().jatam_true_class_range(self._h, first, n, t, c, grid_limit, cap,
                                          rec.data_ptr(), _stream_handle(stream))
        _check(rc, "jatam_true_class_range")
        return rec


class Batch:
    """A jatam_batch_t workspace (device queues for up to max_n genotypes per
    call) and the pipelined calls that use it."""

    def __init__(self, max_n: int):
        handle = ctypes.c_void_p()
        _check(lib().jatam_batch_create(int(max_n), ctypes.byref(handle)), "jatam_batch_create")
        self._h = handle
        self.max_n = int(max_n)

    def close(self) -> None:
        if self._h is not None and self._h.value:
            _check(lib().jatam_batch_destroy(self._h), "jatam_batch_destroy")
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _tally_ptr(tally):
        if tally is None:
            return None
        if tally.dtype != torch.int64 or tuple(tally.shape) != (4,) or not tally.is_cuda:
            raise ValueError("tally must be a device int64 tensor of shape (4,)")
        return tally.data_ptr()

    def classify(self, genotypes: torch.Tensor, t: int, c: int = 8, grid_limit: int = 16,
                 runs: int = 20, seed: int = 1, out: torch.Tensor | None = None,
                 tally: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """jatam_batch_classify."""
        if genotypes.dtype not in (torch.int64, torch.uint64) or genotypes.dim() != 1:
            raise ValueError("genotypes must be a 1-D int64/uint64 tensor")
        if not genotypes.is_cuda or not genotypes.is_contiguous():
            raise ValueError("genotypes must be a contiguous device tensor")
        n = genotypes.shape[0]
        rec = _records(n, genotypes.device, out)
        rc = lib().jatam_batch_classify(self._h, genotypes.data_ptr(), n, t, c, grid_limit,
                                        runs, seed, rec.data_ptr(), self._tally_ptr(tally),
                                        _stream_handle(stream))
        _check(rc, "jatam_batch_classify")
        return rec

    def classify_range(self, first: int, n: int, t: int, c: int = 8, grid_limit: int = 16,
                       runs: int = 20, seed: int = 1, out: torch.Tensor | None = None,
                       tally: torch.Tensor | None = None, device="cuda",
                       stream=None) -> torch.Tensor:
        """jatam_batch_classify_range."""
        rec = _records(n, device, out)
        rc = lib().jatam_batch_classify_range(self._h, first, n, t, c, grid_limit, runs, seed,
                                              rec.data_ptr(), self._tally_ptr(tally),
                                              _stream_handle(stream))
        _check(rc, "jatam_batch_classify_range")
        return rec

    def classify_range_ordered(self, first: int, n: int, order: torch.Tensor, t: int,
                               c: int = 8, grid_limit: int = 16, runs: int = 20, seed: int = 1,
                               out: torch.Tensor | None = None,
                               tally: torch.Tensor | None = None, device="cuda",
                               stream=None) -> torch.Tensor:
        """jatam_batch_classify_range_ordered: queue position p holds genotype
        first + order[p] (order: int32 device tensor of n entries)."""
        if order.dtype != torch.int32 or order.numel() != n or not order.is_cuda \
                or not order.is_contiguous():
            raise ValueError("order must be a contiguous int32 device tensor of n entries")
        rec = _records(n, device, out)
        rc = lib().jatam_batch_classify_range_ordered(self._h, first, n, t, c, grid_limit, runs,
                                                      seed, order.data_ptr(), rec.data_ptr(),
                                                      self._tally_ptr(tally),
                                                      _stream_handle(stream))
        _check(rc, "jatam_batch_classify_range_ordered")
        return rec

    def classify_items(self, items: torch.Tensor, c: int = 8, runs: int = 20, seed: int = 1,
                       out: torch.Tensor | None = None, tally: torch.Tensor | None = None,
                       order: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """jatam_batch_classify_items (or _ordered, given a queue order);
        items is a device uint8 tensor (n, 24), order a device int32 tensor
        (n,) holding a permutation of 0..n-1."""
        if items.dtype != torch.uint8 or items.dim() != 2 or items.shape[1] != ITEM_BYTES:
            raise ValueError("items must be a uint8 tensor of shape (n, 24)")
        if not items.is_cuda or not items.is_contiguous():
            raise ValueError("items must be a contiguous device tensor")
        n = items.shape[0]
        rec = _records(n, items.device, out)
        if order is None:
            rc = lib().jatam_batch_classify_items(self._h, items.data_ptr(), n, c, runs, seed,
                                                  rec.data_ptr(), self._tally_ptr(tally),
                                                  _stream_handle(stream))
        else:
            if order.dtype not in (torch.int32, torch.uint32) or tuple(order.shape) != (n,) \
                    or not order.is_cuda or not order.is_contiguous():
                raise ValueError("order must be a contiguous device int32 tensor of shape (n,)")
            rc = lib().jatam_batch_classify_items_ordered(self._h, items.data_ptr(),
                                                          order.data_ptr(), n, c, runs, seed,
                                                          rec.data_ptr(), self._tally_ptr(tally),
                                                          _stream_handle(stream))
        _check(rc, "jatam_batch_classify_items")
        return rec

    def classify_batch(self, items: torch.Tensor, c: int = 8, runs: int = 20, seed: int = 1,
                       order: torch.Tensor | None = None, tune: dict | None = None,
                       out: torch.Tensor | None = None, tally: torch.Tensor | None = None,
                       stream=None) -> torch.Tensor:
        """jatam_classify_batch: items (device uint8 (n, 24)) in the queue order
        `order` (None: as given), with launch parameters `tune` ({16: {...},
        32: {...}} overriding fields of the workspace's for this call; None:
        the workspace's own)."""
        if items.dtype != torch.uint8 or items.dim() != 2 or items.shape[1] != ITEM_BYTES:
            raise ValueError("items must be a uint8 tensor of shape (n, 24)")
        if not items.is_cuda or not items.is_contiguous():
            raise ValueError("items must be a contiguous device tensor")
        n = items.shape[0]
        rec = _records(n, items.device, out)
        if order is not None and (order.dtype not in (torch.int32, torch.uint32)
                                  or tuple(order.shape) != (n,) or not order.is_cuda
                                  or not order.is_contiguous()):
            raise ValueError("order must be a contiguous device int32 tensor of shape (n,)")
        tp = None
        if tune is not None:
            pair = (Tuning * 2)()
            for k, g in enumerate((16, 32)):
                _check(lib().jatam_batch_get_tuning(self._h, g, ctypes.byref(pair[k])),
                       "jatam_batch_get_tuning")
                for f, v in tune.get(g, {}).items():
                    setattr(pair[k], f, int(v))
            tp = pair
        rc = lib().jatam_classify_batch(self._h, items.data_ptr(), n, c, runs, seed,
                                        order.data_ptr() if order is not None else None, tp,
                                        rec.data_ptr(), self._tally_ptr(tally),
                                        _stream_handle(stream))
        _check(rc, "jatam_classify_batch")
        return rec

    def enumerate(self, first: int, slice_n: int, slices: int, t: int, c: int = 8,
                  grid_limit: int = 16, runs: int = 20, seed: int = 1,
                  out: torch.Tensor | None = None, tally: torch.Tensor | None = None,
                  shapes: torch.Tensor | None = None, stream=None):
        """jatam_batch_enumerate: `slices` graph replays of one slice's
        pipeline over [first, first + slice_n * slices).  out: None or an
        int32 (slice_n * slices, 4) tensor; shapes: None or a table as for
        shape_histogram (int64 (capacity, 2))."""
        if out is not None:
            _records(slice_n * slices, out.device, out)
        if shapes is not None and (shapes.dtype != torch.int64 or shapes.dim() != 2
                                   or shapes.shape[1] != 2 or not shapes.is_cuda):
            raise ValueError("shapes must be a device int64 tensor (capacity, 2)")
        rc = lib().jatam_batch_enumerate(self._h, first, slice_n, slices, t, c, grid_limit, runs,
                                         seed, out.data_ptr() if out is not None else None,
                                         self._tally_ptr(tally),
                                         shapes.data_ptr() if shapes is not None else None,
                                         shapes.shape[0] if shapes is not None else 0,
                                         _stream_handle(stream))
        _check(rc, "jatam_batch_enumerate")
        return out

    def get_tuning(self, grid_limit: int) -> dict:
        t = Tuning()
        _check(lib().jatam_batch_get_tuning(self._h, grid_limit, ctypes.byref(t)),
               "jatam_batch_get_tuning")
        return t.as_dict()

    def set_tuning(self, grid_limit: int, **fields) -> None:
        t = Tuning()
        _check(lib().jatam_batch_get_tuning(self._h, grid_limit, ctypes.byref(t)),
               "jatam_batch_get_tuning")
        for k, v in fields.items():
            setattr(t, k, int(v))
        _check(lib().jatam_batch_set_tuning(self._h, grid_limit, ctypes.byref(t)),
               "jatam_batch_set_tuning")

    def autotune(self, first: int, n: int, t: int, c: int = 8, grid_limit: int = 16,
                 runs: int = 20, seed: int = 1, stream=None):
        """jatam_batch_autotune over [first, first + n); returns (best
        parameters, [(parameters, median ms), ...] in the order tried)."""
        scratch = torch.empty((2 * n, 4), dtype=torch.int32, device="cuda")
        best = Tuning()
        rc = lib().jatam_batch_autotune(self._h, first, n, t, c, grid_limit, runs, seed,
                                        scratch.data_ptr(), ctypes.byref(best),
                                        _stream_handle(stream))
        _check(rc, "jatam_batch_autotune")
        log = []
        count = lib().jatam_batch_autotune_log(self._h, -1, None, None)
        for i in range(count):
            e, ms = Tuning(), ctypes.c_double()
            lib().jatam_batch_autotune_log(self._h, i, ctypes.byref(e), ctypes.byref(ms))
            log.append((e.as_dict(), ms.value))
        return best.as_dict(), log

    def autotune_cached(self, path: str, first: int, n: int, t: int, c: int = 8,
                        grid_limit: int = 16, runs: int = 20, seed: int = 1, stream=None):
        """jatam_batch_autotune_cached; returns (parameters, from_cache)."""
        scratch = torch.empty((2 * n, 4), dtype=torch.int32, device="cuda")
        best, hit = Tuning(), ctypes.c_int(0)
        rc = lib().jatam_batch_autotune_cached(self._h, os.fsencode(path), first, n, t, c,
                                               grid_limit, runs, seed, scratch.data_ptr(),
                                               ctypes.byref(best), ctypes.byref(hit),
                                               _stream_handle(stream))
        _check(rc, "jatam_batch_autotune_cached")
        return best.as_dict(), bool(hit.value)

    def ga_step(self, pop: torch.Tensor, fit: torch.Tensor, t: int, params: GAParams,
                generation: int, c: int = 8, grid_limit: int = 32, runs: int = 20,
                seed: int = 1, next_pop: torch.Tensor | None = None,
                next_fit: torch.Tensor | None = None, surrogate: "Screen | None" = None,
                stream=None):
        """jatam_ga_step: (next_pop, next_fit) of one generation; with a
        Screen, the surrogate-screened generation."""
        _check_pop(pop, fit)
        if next_pop is None:
            next_pop = torch.empty_like(pop)
        if next_fit is None:
            next_fit = torch.empty_like(fit)
        scr = surrogate.struct() if surrogate is not None else None
        rc = lib().jatam_ga_step(self._h, pop.data_ptr(), fit.data_ptr(), pop.shape[0], t, c,
                                 grid_limit, runs, seed, ctypes.byref(params), generation,
                                 ctypes.byref(scr) if scr is not None else None,
                                 next_pop.data_ptr(), next_fit.data_ptr(), _stream_handle(stream))
        _check(rc, "jatam_ga_step")
        return next_pop, next_fit

    def set_refill(self, idle_lanes: int) -> None:
        _check(lib().jatam_batch_set_refill(self._h, idle_lanes), "jatam_batch_set_refill")

    def set_timing(self, enable: bool) -> None:
        _check(lib().jatam_batch_set_timing(self._h, 1 if enable else 0),
               "jatam_batch_set_timing")

    def stage_times(self) -> dict:
        """{stage name: (summed ms, calls)} over the calls made while timing."""
        ms = (ctypes.c_double * 8)()
        calls = (ctypes.c_int * 8)()
        k = lib().jatam_batch_stage_times(self._h, ms, calls, 8)
        if k < 0:
            raise JatamError(k, "jatam_batch_stage_times")
        return {lib().jatam_batch_stage_name(s).decode(): (ms[s], calls[s]) for s in range(k)
                if calls[s] > 0}


MLP_PARAMS = 91652
PREDICT_SCREEN, PREDICT_COST, PREDICT_P_UNBOUND = 0, 1, 2   # jatam_mlp_predict kinds


class MLP:
    """jatam_mlp_t: the surrogate network, trained and evaluated on the GPU."""

    def __init__(self, max_batch: int = 4096, c: int = 8):
        handle = ctypes.c_void_p()
        _check(lib().jatam_mlp_create(int(max_batch), c, ctypes.byref(handle)), "jatam_mlp_create")
        self._h = handle
        self.max_batch = int(max_batch)

    def close(self) -> None:
        if self._h is not None and self._h.value:
            _check(lib().jatam_mlp_destroy(self._h), "jatam_mlp_destroy")
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, seed: int, stream=None) -> None:
        _check(lib().jatam_mlp_init(self._h, seed, _stream_handle(stream)), "jatam_mlp_init")

    def set_params(self, params: torch.Tensor, stream=None) -> None:
        if params.dtype != torch.float32 or params.numel() != MLP_PARAMS or not params.is_cuda:
            raise ValueError("params must be a device float32 tensor of 91652 values")
        _check(lib().jatam_mlp_set_params(self._h, params.contiguous().data_ptr(),
                                          _stream_handle(stream)), "jatam_mlp_set_params")

    def get_params(self, grads: bool = False, stream=None):
        """(params, grads or None) as device float32 tensors."""
        p = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
        g = torch.empty_like(p) if grads else None
        _check(lib().jatam_mlp_get_params(self._h, p.data_ptr(), g.data_ptr() if grads else None,
                                          _stream_handle(stream)), "jatam_mlp_get_params")
        return p, g

    @staticmethod
    def _tiles(t, n):
        if isinstance(t, int):
            return None, t
        if t.dtype != torch.uint8 or t.shape[0] != n or not t.is_cuda:
            raise ValueError("t must be an int or a device uint8 tensor of length n")
        return t.contiguous().data_ptr(), 0

    def forward(self, genomes: torch.Tensor, t, out: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
        n = genomes.shape[0]
        tp, ta = self._tiles(t, n)
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float32, device=genomes.device)
        _check(lib().jatam_mlp_forward(self._h, genomes.data_ptr(), tp, ta, n, out.data_ptr(),
                                       _stream_handle(stream)), "jatam_mlp_forward")
        return out

    def score(self, genomes: torch.Tensor, t, out: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
        """jatam_mlp_score: P(DET) * exp(predicted log1p size) - 1 per genome."""
        n = genomes.shape[0]
        tp, ta = self._tiles(t, n)
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=genomes.device)
        _check(lib().jatam_mlp_score(self._h, genomes.data_ptr(), tp, ta, n, out.data_ptr(),
                                     _stream_handle(stream)), "jatam_mlp_score")
        return out

    def predict(self, genomes: torch.Tensor, t, kind: int, out: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
        """jatam_mlp_predict: PREDICT_SCREEN, PREDICT_COST or PREDICT_P_UNBOUND."""
        n = genomes.shape[0]
        tp, ta = self._tiles(t, n)
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=genomes.device)
        _check(lib().jatam_mlp_predict(self._h, int(kind), genomes.data_ptr(), tp, ta, n,
                                       out.data_ptr(), _stream_handle(stream)),
               "jatam_mlp_predict")
        return out

    def train_step(self, genomes: torch.Tensor, t, labels: torch.Tensor, lr: float = 1e-3,
                   loss: torch.Tensor | None = None, stream=None):
        """labels: (n, 4) int32 records of the genomes."""
        n = genomes.shape[0]
        tp, ta = self._tiles(t, n)
        _check(lib().jatam_mlp_train_step(self._h, genomes.data_ptr(), tp, ta,
                                          labels.data_ptr(), n, float(lr),
                                          loss.data_ptr() if loss is not None else None,
                                          _stream_handle(stream)), "jatam_mlp_train_step")
        return loss


class GA:
    """jatam_ga_t: workspace of the surrogate-screened GA (and top-k select)."""

    def __init__(self, max_candidates: int):
        handle = ctypes.c_void_p()
        _check(lib().jatam_ga_create(int(max_candidates), ctypes.byref(handle)), "jatam_ga_create")
        self._h = handle

    def close(self) -> None:
        if self._h is not None and self._h.value:
            _check(lib().jatam_ga_destroy(self._h), "jatam_ga_destroy")
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def select_top(self, scores: torch.Tensor, k: int, stream=None) -> torch.Tensor:
        """Indices (int32 tensor, ascending) of the k best scores."""
        if scores.dtype != torch.float32 or not scores.is_cuda or not scores.is_contiguous():
            raise ValueError("scores must be a contiguous device float32 tensor")
        out = torch.empty(k, dtype=torch.int32, device=scores.device)
        _check(lib().jatam_select_top(self._h, scores.data_ptr(), scores.shape[0], k,
                                      out.data_ptr(), _stream_handle(stream)), "jatam_select_top")
        return out

    def step_screened(self, batch: "Batch", mlp: "MLP", pop: torch.Tensor, fit: torch.Tensor,
                      t: int, params: GAParams, generation: int, oversample: int = 4, c: int = 8,
                      grid_limit: int = 32, runs: int = 20, seed: int = 1, stream=None):
        """jatam_ga_step_screened: (next_pop, next_fit)."""
        _check_pop(pop, fit)
        next_pop, next_fit = torch.empty_like(pop), torch.empty_like(fit)
        rc = lib().jatam_ga_step_screened(self._h, batch._h, mlp._h, pop.data_ptr(),
                                          fit.data_ptr(), pop.shape[0], t, c, grid_limit, runs,
                                          seed, ctypes.byref(params), generation, oversample,
                                          next_pop.data_ptr(), next_fit.data_ptr(),
                                          _stream_handle(stream))
        _check(rc, "jatam_ga_step_screened")
        return next_pop, next_fit


class ScreenStruct(ctypes.Structure):
    """jatam_screen_t."""
    _fields_ = [("mlp", ctypes.c_void_p), ("ga", ctypes.c_void_p),
                ("oversample", ctypes.c_int32), ("pad", ctypes.c_int32)]


class Screen:
    """What screens a GA generation (jatam_screen_t): a surrogate network, a
    candidate workspace and the oversampling factor."""

    def __init__(self, mlp: MLP, ga: GA, oversample: int = 4):
        self.mlp, self.ga, self.oversample = mlp, ga, int(oversample)

    def struct(self) -> ScreenStruct:
        return ScreenStruct(self.mlp._h.value, self.ga._h.value, self.oversample, 0)

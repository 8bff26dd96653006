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

UNBOUND, ND_SITE, ND_RUNS, DET, INVALID = 0, 1, 2, 3, -1
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


def records_to_numpy(rec: torch.Tensor):
    """(n, 4) int32 records -> numpy structured array (cls, size, hash, steps)."""
    import numpy as np
    dt = np.dtype([("cls", "<i4"), ("size", "<i4"), ("hash", "<u4"), ("steps", "<i4")])
    return rec.detach().cpu().contiguous().numpy().view(dt).reshape(-1)

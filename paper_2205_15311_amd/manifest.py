"""Resumable slice-by-slice enumeration of a lexicographic genotype range.

The paper classifies its spaces batch by batch (§3.4); an enumeration that
takes hours must survive a stopped process.  This keeps a manifest file next
to the work: a header line naming the enumeration, then one JSON line per
finished slice with its class tally and the SHA-256 of its records.  A run
that stops - killed, or told to stop after a number of slices - resumes at
the first slice the manifest lacks; the total tally and the combined digest
(SHA-256 over the slice digests in slice order) do not depend on where it
stopped.

The classification of a slice is the caller's: `classify_slice(first, n)`
returns the n records (the library's batched call on the GPU), as an array
whose bytes are the 16-byte records.  Nothing here computes the method.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np


class ManifestMismatch(RuntimeError):
    """The manifest on disk belongs to another enumeration."""


def _tally(records: np.ndarray) -> list[int]:
    cls = np.asarray(records).view(np.int32).reshape(-1, 4)[:, 0]
    return [int(np.sum(cls == k)) for k in range(4)]


def _read(path: str, header: dict) -> dict[int, dict]:
    done: dict[int, dict] = {}
    if not os.path.exists(path):
        return done
    with open(path) as f:
        lines = [ln for ln in (x.strip() for x in f) if ln]
    if not lines:
        return done
    if json.loads(lines[0]) != {"enumeration": header}:
        raise ManifestMismatch(f"{path} records another enumeration")
    for ln in lines[1:]:
        try:
            entry = json.loads(ln)
        except json.JSONDecodeError:
            break                    # a line cut short by a stop: redo that slice
        done[int(entry["slice"])] = entry
    return done


def enumerate_slices(path: str, header: dict, first: int, slice_n: int, slices: int,
                     classify_slice, stop_after: int | None = None) -> dict:
    """Classifies slices first + s*slice_n .. of the range, s < slices, that
    the manifest at `path` does not hold yet, appending a line after each.
    header: what identifies the enumeration (space, grid, runs, seed, ...);
    a manifest with another header raises ManifestMismatch.  stop_after:
    return after classifying that many new slices (the rest stay for a
    later call).  Returns {"complete", "slices_done", "tally", "digest"}."""
    header = dict(header, first=int(first), slice=int(slice_n), slices=int(slices))
    done = _read(path, header)
    if not os.path.exists(path) or os.path.getsize(path) == 0:
        with open(path, "w") as f:
            f.write(json.dumps({"enumeration": header}) + "\n")
    else:
        # rewrite without a trailing partial line before appending
        with open(path, "w") as f:
            f.write(json.dumps({"enumeration": header}) + "\n")
            for s in sorted(done):
                f.write(json.dumps(done[s]) + "\n")
    new = 0
    for s in range(slices):
        if s in done:
            continue
        if stop_after is not None and new >= stop_after:
            break
        lo = first + s * slice_n
        rec = np.ascontiguousarray(classify_slice(lo, slice_n))
        entry = {"slice": s, "first": lo, "n": slice_n, "tally": _tally(rec),
                 "sha256": hashlib.sha256(rec.tobytes()).hexdigest()}
        with open(path, "a") as f:
            f.write(json.dumps(entry) + "\n")
            f.flush()
            os.fsync(f.fileno())
        done[s] = entry
        new += 1
    complete = len(done) == slices
    tally = [sum(done[s]["tally"][k] for s in done) for k in range(4)]
    digest = hashlib.sha256("".join(done[s]["sha256"] for s in sorted(done)).encode())
    return {"complete": complete, "slices_done": len(done), "tally": tally,
            "digest": digest.hexdigest() if complete else None}

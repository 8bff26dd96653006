"""Writes tests/golden/s28_digests.json and s18_digests.json.

Calls only the CPU oracle: every expected value in those files comes from
oracle/ (never from the HIP library).  Per 2^20-genotype slice of a space it
stores the SHA-256 of the little-endian 16-byte records, the class tally, the
summed steps and the summed size of DET genotypes.

    python tests/golden/make_golden.py            # both files
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import ref  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def slice_summary(recs, s0, e0, c0, f0, runs):
    det = recs["cls"] == 3
    size = recs["size"].astype(np.int64)
    steps = recs["steps"].astype(np.int64)
    s0 = s0.astype(np.int64)
    # how the work splits over a pipeline: genotypes the seed alone decides
    # (0 placements) and first runs; then the candidates (first run drew a
    # random word and ended without an event): those whose first-run shape
    # is guarded (forced shapes among them) are final after that run, the
    # others need the repeat runs
    cand = (e0 == 0) & (c0 == 1) & (runs > 1)
    forced = cand & ((f0 & 1) != 0)
    proven = cand & ((f0 & 2) != 0)
    unproven = cand & ((f0 & 2) == 0)
    first_only = ~cand
    return {
        "sha256": hashlib.sha256(recs.tobytes()).hexdigest(),
        "tally": [int(np.sum(recs["cls"] == k)) for k in range(4)],
        "steps": int(steps.sum()),
        "det_size": int(size[det].sum()),
        "work": {
            "run0_steps": int(s0.sum()),
            "monomer_det": int(np.sum(det & (size == 1))),
            "run0_det": int(np.sum(det & first_only & (size > 1))),
            "run0_det_size": int(size[det & first_only & (size > 1)].sum()),
            "candidates": int(cand.sum()),
            "cand_steps0": int(s0[cand].sum()),
            "cand_size": int(size[cand].sum()),
            "forced": int(forced.sum()),
            "forced_size": int(size[forced].sum()),
            "proven": int(proven.sum()),
            "proven_size": int(size[proven].sum()),
            "unproven": int(unproven.sum()),
            "unproven_steps": int(steps[unproven].sum()),
            "unproven_det": int(np.sum(det & unproven)),
            "unproven_det_size": int(size[det & unproven].sum()),
        },
    }


def shape_counts(recs):
    """{(hash, size): count} over the DET records."""
    det = recs[recs["cls"] == 3]
    keys, counts = np.unique(np.stack([det["hash"].astype(np.int64), det["size"].astype(np.int64)]),
                             axis=1, return_counts=True)
    return {(int(h), int(z)): int(c) for (h, z), c in zip(keys.T, counts)}


def make(t, grid, runs, seed, total, slice_n, path):
    t0 = time.time()
    slices = []
    shapes = {}
    for first in range(0, total, slice_n):
        n = min(slice_n, total - first)
        recs, s0, e0, c0, f0 = ref.classify_range_run0(first, n, t, grid=grid, runs=runs,
                                                       seed=seed, forced=True)
        s = slice_summary(recs, s0, e0, c0, f0, runs)
        for key, cnt in shape_counts(recs).items():
            shapes[key] = shapes.get(key, 0) + cnt
        s["first"] = first
        s["n"] = n
        slices.append(s)
    doc = {
        "space": f"S_{{{t},8}}", "t": t, "c": 8, "grid": grid, "runs": runs, "seed": seed,
        "total": total, "slice": slice_n, "record": "int32 cls, int32 size, uint32 hash, int32 steps",
        "writer": "tests/golden/make_golden.py (oracle only)",
        "slices": slices,
        "tally": [sum(s["tally"][k] for s in slices) for k in range(4)],
        "steps": sum(s["steps"] for s in slices),
        "det_size": sum(s["det_size"] for s in slices),
        "work": {k: sum(s["work"][k] for s in slices) for k in slices[0]["work"]},
        "shapes": [{"hash": h, "size": z, "count": shapes[(h, z)]}
                   for (h, z) in sorted(shapes, key=lambda k: (k[1], k[0]))],
    }
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"{path}: {time.time() - t0:.1f}s tally={doc['tally']}")


if __name__ == "__main__":
    make(1, 16, 20, 1, 4096, 4096, os.path.join(HERE, "s18_digests.json"))
    make(2, 16, 20, 1, 1 << 24, 1 << 20, os.path.join(HERE, "s28_digests.json"))

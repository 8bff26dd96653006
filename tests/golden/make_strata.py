"""Writes tests/golden/workload_strata.json: the oracle's records of stratified
subsets of the three larger workloads, as SHA-256 digests per chunk of 2^18
records (so a mismatch on the GPU names its chunk) and class tallies.

Calls only the CPU oracle and the seeded input generators (tests/inputs.py);
no expected value comes from the HIP library.

  mixed   the 2^26-item mixed stream (t in {1,2,3}, G in {16,32}): for each
          (t, G) stratum, its first 2^22 items in stream order
  slice   the contiguous 2^30-genotype slice of the three-tile space at
          G = 32: every 256th genotype (2^22 records, spread over the slice)
  sample  the 2^28-genotype uniform three-tile sample at G = 32: every 64th
          (2^22 records)

    python tests/golden/make_strata.py        (a few minutes on 8 cores)
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
from tests import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
R, SEED = 20, 1
STRATUM = 1 << 22
CHUNK = 1 << 18
MIXED_N = 1 << 26
SLICE_N, SLICE_STRIDE = 1 << 30, 256
SAMPLE_N, SAMPLE_STRIDE = 1 << 28, 64


def summary(recs):
    chunks = [hashlib.sha256(recs[i:i + CHUNK].tobytes()).hexdigest()
              for i in range(0, len(recs), CHUNK)]
    return {"n": int(len(recs)), "chunk": CHUNK, "sha256": chunks,
            "tally": [int(np.sum(recs["cls"] == k)) for k in range(4)]}


def mixed_items(g, t, grid):
    it = np.zeros(len(g), dtype=ref.ITEM)
    it["genome"], it["t"], it["grid"] = g, t, grid
    it["rng_id"] = g | (t.astype(np.uint64) << np.uint64(56))
    return it


def main():
    out = {"runs": R, "seed": SEED}
    t0 = time.time()
    g, t, grid = inputs.mixed_stream(MIXED_N)
    strata = {}
    for tt in (1, 2, 3):
        for G in (16, 32):
            idx = np.nonzero((t == tt) & (grid == G))[0][:STRATUM]
            assert len(idx) == STRATUM
            recs = ref.classify_items(mixed_items(g[idx], t[idx], grid[idx]), 8, R, SEED)
            strata[f"t{tt}_g{G}"] = summary(recs)
            print(f"mixed t={tt} G={G}: {time.time() - t0:.0f} s", flush=True)
    out["mixed"] = {"total": MIXED_N, "strata": strata}
    del g, t, grid

    first = inputs.three_tile_slice_start(SLICE_N)
    gs = np.uint64(first) + np.arange(0, SLICE_N, SLICE_STRIDE, dtype=np.uint64)
    out["slice"] = {"first": int(first), "total": SLICE_N, "stride": SLICE_STRIDE,
                    **summary(ref.classify(gs, 3, grid=32, runs=R, seed=SEED))}
    print(f"slice: {time.time() - t0:.0f} s", flush=True)

    gsamp = inputs.three_tile_sample(SAMPLE_N)[::SAMPLE_STRIDE]
    out["sample"] = {"total": SAMPLE_N, "stride": SAMPLE_STRIDE,
                     **summary(ref.classify(gsamp, 3, grid=32, runs=R, seed=SEED))}
    print(f"sample: {time.time() - t0:.0f} s", flush=True)
    with open(os.path.join(HERE, "workload_strata.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()

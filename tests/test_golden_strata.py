"""The stored oracle digests of the larger workloads match the oracle as it
stands (one chunk, recomputed here on the CPU)."""
import hashlib
import json
import os

import numpy as np

from oracle import ref
from tests import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def test_slice_stratum_first_chunk_matches_the_oracle():
    with open(os.path.join(HERE, "golden", "workload_strata.json")) as f:
        gold = json.load(f)["slice"]
    assert gold["first"] == inputs.three_tile_slice_start(gold["total"])
    k = np.arange(gold["chunk"], dtype=np.uint64)
    g = np.uint64(gold["first"]) + k * np.uint64(gold["stride"])
    recs = ref.classify(g, 3, grid=32, runs=20, seed=1)
    assert hashlib.sha256(recs.tobytes()).hexdigest() == gold["sha256"][0]

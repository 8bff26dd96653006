"""Resumable enumeration (paper_2205_15311_amd/manifest.py) on the CPU, with
the oracle classifying each slice: a run stopped after k slices and resumed
ends with the same tally and digest as an uninterrupted run, whatever k; a
manifest cut mid-line redoes that slice; another enumeration's manifest is
refused; the slice digests are those of the golden S_{2,8} records."""
import json
import os

import numpy as np
import pytest

from oracle import ref
from paper_2205_15311_amd import manifest

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = {"space": "S_2,8", "t": 2, "c": 8, "grid": 16, "runs": 20, "seed": 1}


def oracle_slice(first, n):
    return ref.classify_range(first, n, 2, grid=16, runs=20, seed=1)


def test_stop_and_resume_give_the_uninterrupted_result(tmp_path):
    whole = manifest.enumerate_slices(str(tmp_path / "whole.jsonl"), HEADER, 0, 4096, 6,
                                      oracle_slice)
    assert whole["complete"] and whole["slices_done"] == 6
    for k in (1, 3, 5):
        path = str(tmp_path / f"stop{k}.jsonl")
        part = manifest.enumerate_slices(path, HEADER, 0, 4096, 6, oracle_slice, stop_after=k)
        assert not part["complete"] and part["slices_done"] == k and part["digest"] is None
        rest = manifest.enumerate_slices(path, HEADER, 0, 4096, 6, oracle_slice)
        assert rest == whole
    rec = oracle_slice(0, 6 * 4096)
    assert whole["tally"] == [int(np.sum(rec["cls"] == c)) for c in range(4)]


def test_a_line_cut_short_is_redone(tmp_path):
    path = tmp_path / "cut.jsonl"
    manifest.enumerate_slices(str(path), HEADER, 0, 2048, 4, oracle_slice, stop_after=3)
    text = path.read_text()
    path.write_text(text[:-20])              # the third slice's line loses its end
    res = manifest.enumerate_slices(str(path), HEADER, 0, 2048, 4, oracle_slice)
    whole = manifest.enumerate_slices(str(tmp_path / "w.jsonl"), HEADER, 0, 2048, 4,
                                      oracle_slice)
    assert res == whole
    assert len(path.read_text().splitlines()) == 5


def test_another_enumeration_is_refused(tmp_path):
    path = str(tmp_path / "m.jsonl")
    manifest.enumerate_slices(path, HEADER, 0, 1024, 2, oracle_slice, stop_after=1)
    with pytest.raises(manifest.ManifestMismatch):
        manifest.enumerate_slices(path, dict(HEADER, runs=7), 0, 1024, 2, oracle_slice)


def test_slice_digests_are_the_golden_ones(tmp_path):
    with open(os.path.join(HERE, "golden", "s28_digests.json")) as f:
        gold = json.load(f)
    first, n = gold["slices"][0]["first"], gold["slices"][0]["n"]
    path = tmp_path / "g.jsonl"
    manifest.enumerate_slices(str(path), HEADER, first, n, 1, oracle_slice)
    entry = json.loads(path.read_text().splitlines()[1])
    assert entry["sha256"] == gold["slices"][0]["sha256"]
    assert entry["tally"] == gold["slices"][0]["tally"]

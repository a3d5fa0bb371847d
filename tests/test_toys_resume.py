"""Checkpointed toy studies (paper_1706_01420_amd/toys.py): the JSONL record
reader on the CPU (other seeds and a torn last line ignored); on the GPU, a
study interrupted after its first batch and started again writes exactly
the records of an uninterrupted study (counter-based toys, batch-independent
fits)."""
import json
import sys

import numpy as np
import pytest

from paper_1706_01420_amd import toys


def test_completed_ids_reads_records_of_its_seed(tmp_path):
    p = tmp_path / "study.jsonl"
    assert toys.completed_ids(str(p), 7) == set()
    with open(p, "w") as fh:
        for seed, j in ((7, 0), (7, 3), (8, 1), (7, 2)):
            fh.write(json.dumps({"seed": seed, "toy_id": j, "theta": [0.0]}) + "\n")
        fh.write('{"seed": 7, "toy_id": 5, "the')          # torn by an interruption
    assert toys.completed_ids(str(p), 7) == {0, 2, 3}
    assert toys.completed_ids(str(p), 8) == {1}


@pytest.mark.gpu
def test_interrupted_study_resumes_to_the_same_records(tmp_path):
    from paper_1706_01420_amd import ipx, workloads
    ctx = ipx.ipx_create(0)
    try:
        th = np.array(workloads.THETA_GEN[1])
        a, b = str(tmp_path / "a.jsonl"), str(tmp_path / "b.jsonl")
        print("[gpu] toy study resume", file=sys.stderr, flush=True)
        assert toys.study(ipx, ctx, 1, th, 31, 10, a, batch=4) == 10
        # "interrupted" after 3 toys (so the resumed batches differ from a's)
        assert toys.study(ipx, ctx, 1, th, 31, 10, b, batch=4, limit=3) == 3
        with open(b, "a") as fh:
            fh.write('{"seed": 31, "toy_id": 3, "th')                          # torn write
        assert toys.study(ipx, ctx, 1, th, 31, 10, b, batch=4) == 7
        assert toys.study(ipx, ctx, 1, th, 31, 10, b, batch=4) == 0              # nothing left

        def records(path):
            out = {}
            with open(path) as fh:
                for line in fh:
                    try:
                        r = json.loads(line)
                    except ValueError:
                        continue
                    out[r["toy_id"]] = r
            return out
        ra, rb = records(a), records(b)
        assert sorted(ra) == list(range(10)) and sorted(rb) == list(range(10))
        for j in range(10):
            assert ra[j] == rb[j], j
        assert np.mean([ra[j]["converged"] for j in ra]) > 0.8
    finally:
        ipx.ipx_destroy(ctx)

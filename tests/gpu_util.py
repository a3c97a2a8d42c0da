"""Helpers for the GPU parity tests (call the HIP library through the C ABI)."""
import hashlib
import json
import os

import numpy as np

import paper_2110_12511_amd as pb

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def u64(t):
    return pb.to_numpy_u64(t)


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def golden(workload, quantity):
    p = os.path.join(GOLDEN, f"{workload}__{quantity}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        return json.load(f)


def check_golden(rec, res, graph_digest):
    assert rec["graph_sha256"] == graph_digest, "input graph differs from the one the oracle ran on"
    assert rec["n"] == res.size
    for i, v in rec["sample"]:
        assert int(res[i]) == int(v), (i, int(res[i]), v)
    assert str(int(res.max())) == rec["max"] if res.size else True
    assert digest(res) == rec["sha256"]

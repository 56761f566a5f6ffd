"""Every gate of the 4096-gate benchmark batch against the CPU oracle, in every blind-rotation
form and key-switch form that can run it. The oracle's outputs for this batch are committed as
per-gate SHA-256 digests (tests/golden/config2_oracle_digest.json, written by
tests/golden/make_config2_digest.py from the oracle alone); the test first checks that it
encrypted the same inputs, then compares all 4096 output rows."""
import hashlib
import json
import os

import numpy as np
import pytest

import workloads as W
from paper_2010_09410_amd import client
from paper_2010_09410_amd.device import to_host

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "config2_oracle_digest.json")
B = 4096

# (blind-rotation shape, key-switch form): the matrix-core form, the 8-, 4- and 3-wave NTT
# forms, the split matrix-core form; key-switch forms 3 (matrix cores), 2 (LDS-staged split), 1 (row tiles), 0 (gather).
FORMS = [(32, 3), (32, 2), (8, 3), (8, 2), (4, 1), (3, 0), (33, 3)]


def row_digest(row) -> str:
    return hashlib.sha256(np.ascontiguousarray(row, dtype="<u4").tobytes()).hexdigest()[:16]


@pytest.fixture(scope="module")
def batch(keys):
    doc = json.load(open(GOLDEN))
    cfg = W.config2(B)
    in0 = client.tlwe_encrypt_bits(keys["s0"], cfg["bits0"], *cfg["enc0"])
    in1 = client.tlwe_encrypt_bits(keys["s0"], cfg["bits1"], *cfg["enc1"])
    inputs = hashlib.sha256(np.ascontiguousarray(cfg["ops"]).tobytes() + in0.astype("<u4").tobytes()
                            + in1.astype("<u4").tobytes()).hexdigest()
    assert inputs == doc["inputs_sha256"], "the encrypted inputs differ from the ones the digests were made from"
    return cfg, in0, in1, doc


@pytest.mark.parametrize("waves,ks", FORMS)
def test_every_gate_matches_oracle(gpu, batch, waves, ks):
    cfg, in0, in1, doc = batch
    d0, d1, dops = gpu.tensor(in0), gpu.tensor(in1), gpu.tensor(cfg["ops"])
    saved = gpu.tuning(B)
    try:
        gpu.set_tuning(B, waves, ks)
        assert gpu.tuning(B) == (waves, ks)
        out = to_host(gpu.gates(dops, d0, d1))
        gpu.sync()
    finally:
        gpu.set_tuning(B, 0, saved[1])
    want = doc["gate_sha256_prefix"]
    bad = [k for k in range(B) if row_digest(out[k]) != want[k]]
    assert not bad, f"{len(bad)} of {B} gates differ from the oracle (shape {waves}, key switch {ks}); first {bad[:8]}"
    assert hashlib.sha256(out.astype("<u4").tobytes()).hexdigest() == doc["outputs_sha256"]


@pytest.mark.parametrize("nb", [1, 16, 64, 1000, 2048])
def test_split_matrix_form_prefixes_match_oracle(gpu, batch, nb):
    """The split matrix-core form on the first nb gates (one tile, partial tiles, a ragged
    1000-gate batch, a 2048-gate batch with fewer row groups) against the oracle's digests."""
    cfg, in0, in1, doc = batch
    d0, d1, dops = gpu.tensor(in0[:nb]), gpu.tensor(in1[:nb]), gpu.tensor(cfg["ops"][:nb])
    saved = gpu.tuning(nb)
    try:
        gpu.set_tuning(nb, 33, 2)
        assert gpu.tuning(nb) == (33, 2)
        out = to_host(gpu.gates(dops, d0, d1))
        gpu.sync()
    finally:
        gpu.set_tuning(nb, 0, saved[1])
    want = doc["gate_sha256_prefix"]
    bad = [k for k in range(nb) if row_digest(out[k]) != want[k]]
    assert not bad, f"{len(bad)} of {nb} gates differ from the oracle; first {bad[:8]}"


@pytest.mark.parametrize("nb,groups", [(1, 6), (1, 12), (1, 24), (2, 12), (3, 24), (4, 6), (5, 24), (16, 24),
                                       (37, 12), (64, 24), (64, 1), (256, 6), (1, -6), (16, -6), (37, -3),
                                       (64, -6), (256, -3), (1000, -2), (2048, -1), (16, -12), (37, -24),
                                       (256, -12), (300, -24)])
def test_split_form_workgroup_counts_match_oracle(gpu, batch, nb, groups):
    """Every way of cutting a step of the split form (row groups, single rows with the byte
    planes in two or four ranges; up to four gates with the digits formed inside the step
    kernel, five gates just above; negative counts: shares stored as partial sums and added by
    the digit launch, 300 gates with -24 falling back to atomics) on prefixes of the batch,
    against the oracle's digests."""
    cfg, in0, in1, doc = batch
    d0, d1, dops = gpu.tensor(in0[:nb]), gpu.tensor(in1[:nb]), gpu.tensor(cfg["ops"][:nb])
    saved = gpu.tuning(nb)
    prev = gpu.set_split_groups(nb, groups)
    try:
        gpu.set_tuning(nb, 33, 2)
        out = to_host(gpu.gates(dops, d0, d1))
        gpu.sync()
    finally:
        gpu.set_tuning(nb, 0, saved[1])
        gpu.set_split_groups(nb, prev)
    want = doc["gate_sha256_prefix"]
    bad = [k for k in range(nb) if row_digest(out[k]) != want[k]]
    assert not bad, f"{len(bad)} of {nb} gates differ from the oracle (groups {groups}); first {bad[:8]}"

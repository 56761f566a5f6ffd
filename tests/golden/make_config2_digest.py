"""Writes config2_oracle_digest.json: the CPU oracle's outputs for the whole 4096-gate batch
(NAND/AND/OR/XOR/XNOR on fresh encrypted bits, seeds 0/1/2 for the keys, 12 and 22 for the
bits and the encryption randomness), stored as SHA-256 digests per gate.

Only the oracle and the seeded draws are used: the keys, the encryptions and the gate outputs
are all computed by ``oracle`` (the library is not imported). The GPU parity test compares
every gate of its batch against these digests; the input digest lets it check first that it
encrypted the same ciphertexts.

Run from the repository root:  python tests/golden/make_config2_digest.py   (about 3-4 minutes
on 8 cores).
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_oracle_digest.json")
PREFIX = 16  # hex digits kept of each gate's SHA-256 (64 bits)


def row_digest(row: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(row, dtype="<u4").tobytes()).hexdigest()[:PREFIX]


def main():
    t0 = time.time()
    s0, s1 = W.secret_keys()
    bk, ksk = oracle.keyset(s0, s1, W.bk_draws(), W.ksk_draws())
    cfg = W.config2()
    in0 = oracle.tlwe_encrypt_bits(s0, cfg["bits0"], *cfg["enc0"])
    in1 = oracle.tlwe_encrypt_bits(s0, cfg["bits1"], *cfg["enc1"])
    out = oracle.gates(bk, ksk, cfg["ops"], in0, in1)
    inputs = hashlib.sha256(np.ascontiguousarray(cfg["ops"]).tobytes() + in0.astype("<u4").tobytes()
                            + in1.astype("<u4").tobytes()).hexdigest()
    doc = {
        "what": "CPU oracle outputs of the 4096-gate batch: per-gate SHA-256 (first 16 hex digits) of the "
                "631 little-endian uint32 words of each output TLWE, and of all outputs concatenated",
        "workload": "4096 independent gates, opcode uniform over NAND/AND/OR/XOR/XNOR, fresh TLWE inputs; "
                    "n=630 N=1024 l=3 Bgbit=6 t=8 basebit=2; keys from seeds 0/1/2",
        "written_by": "tests/golden/make_config2_digest.py (oracle only)",
        "inputs_sha256": inputs,
        "outputs_sha256": hashlib.sha256(out.astype("<u4").tobytes()).hexdigest(),
        "gate_sha256_prefix": [row_digest(r) for r in out],
    }
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=0)
        fh.write("\n")
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()

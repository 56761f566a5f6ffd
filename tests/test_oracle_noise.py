"""Noise-variance pins of the oracle's blind rotation and key switch.

Predictions follow the standard TFHE average-case analysis, evaluated with the actual key
weights: per blind-rotation step, 2l N E[d^2] V1 from the key noise plus, when the key bit
is 1, (1 + |s1|) (2^-18)^2 / 12 from the gadget rounding; for the key switch, the number of
non-zero digits times V0 plus |s1| (2^-16)^2 / 12 from its rounding. E[d^2] = 341.5 for
digits uniform on [-32, 31]; V0 = 2^-30, V1 = 2^-50.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
import workloads as W
from conftest import signed

P = oracle.DEFAULT
N, n, l = P.N, P.n, P.l
MU = 1 << 29
T2 = 2.0 ** -32  # one torus unit of the uint32 discretisation


def test_blind_rotation_variance(keys):
    s0, s1 = keys["s0"], keys["s1"]
    w0, w1 = int(s0.sum()), int(s1.sum())
    pred = n * 2 * l * N * 341.5 * 2.0 ** -50 + w0 * (1 + w1) * (2.0 ** -18) ** 2 / 12
    g = W.rng(200)
    cs = W.uniform_u32(g, (8, n + 1))
    tv = np.full(N, MU, dtype=np.uint32)
    with ThreadPoolExecutor(8) as ex:
        accs = list(ex.map(lambda c: oracle.blind_rotate(keys["bk"], c, tv), cs))
    errs = []
    for c, acc in zip(cs, accs):
        abar = np.array([oracle.modswitch(v) for v in c[:n]], dtype=np.int64)
        phi = (oracle.modswitch(c[n]) - int(np.sum(abar * s0))) % (2 * N)
        k = (2 * N - phi) % (2 * N)
        want = oracle.rotate(tv, k)
        errs.append(signed(oracle.trlwe_phase(s1, acc) - want))
    e = np.concatenate(errs) * T2
    var = float(np.mean(e ** 2))
    print(f"blind rotation variance {var:.3e} predicted {pred:.3e} ratio {var / pred:.3f}")
    assert 0.8 < var / pred < 1.25


def test_keyswitch_variance(keys):
    """For one fixed key and uniform inputs, digit v_{j,p} is uniform on {0..3}, so the
    phase error X = -sum_{j,p} e_{j,p,v} - rounding has E[X^2] = sum_{jp} E[e^2]
    + (sum_{jp} E[e])^2 - sum_{jp} E[e]^2 + |s1| (2^-16)^2 / 12, with E over the digit."""
    s0, s1 = keys["s0"], keys["s1"]
    w1 = int(s1.sum())
    e = keys["kskd"][1].astype(np.float64) * T2            # [N][t][3] key noise
    m1 = e.sum(axis=2) / 4.0                              # E[e] per (j, p)
    m2 = (e ** 2).sum(axis=2) / 4.0                       # E[e^2] per (j, p)
    pred = m2.sum() + m1.sum() ** 2 - (m1 ** 2).sum() + w1 * (2.0 ** -16) ** 2 / 12
    g = W.rng(201)
    cs = W.uniform_u32(g, (768, N + 1))
    with ThreadPoolExecutor(8) as ex:
        outs = list(ex.map(lambda c: oracle.keyswitch(keys["ksk"], c), cs))
    d = np.array([(int(oracle.tlwe_phase(s0, o)) - int(oracle.tlwe_phase(s1, c)) + 2 ** 31) % 2 ** 32 - 2 ** 31
                  for c, o in zip(cs, outs)], dtype=np.float64) * T2
    var = float(np.mean(d ** 2))
    print(f"key switch mean-square error {var:.3e} predicted {pred:.3e} ratio {var / pred:.3f}")
    assert 0.85 < var / pred < 1.15

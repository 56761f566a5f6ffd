"""Pins of the oracle's TFHE steps against closed forms, exact identities and decryption.

* Encryption (Sec. 2.1.2): phases equal message + noise exactly; TRGSW rows carry the gadget.
* External product: exact phase identity (noise terms + gadget recomposition), trivial
  TRGSW(1) = coefficientwise rounding to multiples of 2^-18, TRGSW(0) = 0.
* SampleExtract: the TLWE phase equals the chosen TRLWE phase coefficient, bit for bit.
* Key switching: with a noise-free key the phase error is exactly the rounding term.
* Blind rotation with a noise-free, mask-free key: exactly X^-(bbar - sum abar_i s_i) tv.
* Gates: trivial inputs give exactly (0, +-1/8); every gate decrypts its full truth table;
  the paper's half adder (Eq. halfadder) with its printed case A = B = 1 -> S = 0, C = 1.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from conftest import signed

P = oracle.DEFAULT
N, n, l = P.N, P.n, P.l
MU = 1 << 29
HERE = os.path.dirname(os.path.abspath(__file__))

TRUTH = {
    oracle.NAND: lambda a, b: 1 - (a & b), oracle.AND: lambda a, b: a & b,
    oracle.OR: lambda a, b: a | b, oracle.NOR: lambda a, b: 1 - (a | b),
    oracle.XOR: lambda a, b: a ^ b, oracle.XNOR: lambda a, b: 1 - (a ^ b),
    oracle.ANDNOT: lambda a, b: a & (1 - b), oracle.ORNOT: lambda a, b: a | (1 - b),
}


def round14(x):
    """Nearest multiple of 2^14 (ties up), mod 2^32: the value l = 3 digits of base 64 represent."""
    return ((np.asarray(x, dtype=np.uint64) + (1 << 13)) & 0xFFFFC000 & 0xFFFFFFFF).astype(np.uint32)


def test_tlwe_phase_is_message_plus_noise(keys):
    g = W.rng(100)
    bits = g.integers(0, 2, 64)
    a, e = W.tlwe_draws(g, 64)
    c = oracle.tlwe_encrypt_bits(keys["s0"], bits, a, e)
    ph = signed(oracle.tlwe_phase(keys["s0"], c))
    np.testing.assert_array_equal(ph, np.where(bits == 1, MU, -MU) + e)
    np.testing.assert_array_equal(oracle.tlwe_decrypt(keys["s0"], c), bits)


def test_trlwe_and_trgsw_structure(keys):
    s1 = keys["s1"]
    g = W.rng(101)
    bits = g.integers(0, 2, N).astype(np.uint8)
    a, e = W.trlwe_draws(g, 1)
    c = oracle.trlwe_encrypt_bits(s1, bits, a[0], e[0])
    np.testing.assert_array_equal(signed(oracle.trlwe_phase(s1, c)), np.where(bits == 1, MU, -MU) + e[0])
    # TRGSW(m): row r < l has phase e_r - m s/Bg^(r+1); row r >= l has phase e_r + m/Bg^(r-l+1).
    ma, me = W.trgsw_draws(g, 1)
    for m in (0, 1):
        C = oracle.trgsw_encrypt(s1, m, ma[0], me[0])
        for r in range(2 * l):
            ph = oracle.trlwe_phase(s1, C[r])
            if r < l:
                expect = me[0][r].astype(np.uint32) - np.uint32(m) * (s1.astype(np.uint32) << (32 - 6 * (r + 1)))
            else:
                expect = me[0][r].astype(np.uint32).copy()
                expect[0] += np.uint32(m << (32 - 6 * (r - l + 1)))
            np.testing.assert_array_equal(ph, expect)


def test_gadget_trgsw_is_rounding(keys):
    g = W.rng(102)
    x = W.uniform_u32(g, (2, N))
    G = np.zeros((2 * l, 2, N), dtype=np.uint32)
    for r in range(l):
        G[r, 0, 0] = 1 << (32 - 6 * (r + 1))
        G[l + r, 1, 0] = 1 << (32 - 6 * (r + 1))
    np.testing.assert_array_equal(oracle.trgsw_gadget(), G)
    np.testing.assert_array_equal(oracle.external_product(G, x), round14(x))
    np.testing.assert_array_equal(oracle.external_product(np.zeros_like(G), x), np.zeros_like(x))


def test_external_product_exact_phase_identity(keys):
    """phase(C(m) [x] x) = sum_q d_q * e_q + m (round(B) - round(A) s), exactly (mod 2^32)."""
    s1 = keys["s1"]
    g = W.rng(103)
    ma, me = W.trgsw_draws(g, 1)
    x = W.uniform_u32(g, (2, N))
    digits = np.array([[oracle.decompose(v) for v in x[h]] for h in range(2)])  # [2][N][l]
    noise_term = np.zeros(N, dtype=np.uint32)
    for q in range(2 * l):
        h, r = divmod(q, l)
        noise_term += oracle.polymul(digits[h, :, r].astype(np.int64).astype(np.uint32),
                                     me[0][q].astype(np.int64).astype(np.uint32))
    for m in (0, 1):
        C = oracle.trgsw_encrypt(s1, m, ma[0], me[0])
        ph = oracle.trlwe_phase(s1, oracle.external_product(C, x))
        rA, rB = round14(x[0]), round14(x[1])
        expect = noise_term + np.uint32(m) * (rB - oracle.polymul(rA, s1))
        np.testing.assert_array_equal(ph, expect)


def test_cmux_selects(keys):
    s1 = keys["s1"]
    g = W.rng(104)
    ma, me = W.trgsw_draws(g, 2)
    a, e = W.trlwe_draws(g, 2)
    b0 = g.integers(0, 2, N).astype(np.uint8)
    b1 = g.integers(0, 2, N).astype(np.uint8)
    x0 = oracle.trlwe_encrypt_bits(s1, b0, a[0], e[0])
    x1 = oracle.trlwe_encrypt_bits(s1, b1, a[1], e[1])
    for m in (0, 1):
        C = oracle.trgsw_encrypt(s1, m, ma[m], me[m])
        ph = signed(oracle.trlwe_phase(s1, oracle.cmux(C, x0, x1)))
        want = np.where((b1 if m else b0) == 1, MU, -MU)
        assert np.abs(ph - want).max() < (1 << 22)


def test_sample_extract_phase_identity(keys):
    s1 = keys["s1"]
    g = W.rng(105)
    c = W.uniform_u32(g, (2, N))
    phase = oracle.trlwe_phase(s1, c)
    for h in (0, 1, 2, 31, 511, 1022, 1023):
        t = oracle.sample_extract(c, h)
        assert oracle.tlwe_phase(s1, t) == phase[h]


def test_keyswitch_noise_free_exact_rounding(keys):
    """With a noise-free key, phase_out - phase_in = sum_j s1_j (a_j - round16(a_j)) exactly."""
    s0, s1 = keys["s0"], keys["s1"]
    kskd = W.ksk_draws()
    ksk0 = oracle.ksk_gen(s0, s1, kskd[0], np.zeros_like(kskd[1]))
    g = W.rng(106)
    for _ in range(4):
        c = W.uniform_u32(g, (N + 1,))
        out = oracle.keyswitch(ksk0, c)
        rnd = ((c[:N].astype(np.uint64) + (1 << 15)) & 0xFFFF0000).astype(np.uint32)
        err = int(np.sum((c[:N] - rnd).astype(np.uint64) * s1.astype(np.uint64)))
        assert int(oracle.tlwe_phase(s0, out)) == (int(oracle.tlwe_phase(s1, c)) + err) & 0xFFFFFFFF


def test_keyswitch_with_noise_keeps_phase(keys):
    g = W.rng(107)
    for _ in range(4):
        c = W.uniform_u32(g, (N + 1,))
        out = oracle.keyswitch(keys["ksk"], c)
        d = int(np.int32(np.uint32(oracle.tlwe_phase(keys["s0"], out) - oracle.tlwe_phase(keys["s1"], c))))
        assert abs(d) < (1 << 27)


def trivial_bk(s0):
    """Noise-free, mask-free bootstrapping key: BK[i] = s0[i] * G."""
    G = oracle.trgsw_gadget()
    return (s0.astype(np.uint32)[:, None, None, None] * G[None]).astype(np.uint32)


def monomial(k):
    p = np.zeros(N, dtype=np.uint32)
    k %= 2 * N
    p[k % N] = 1 if k < N else 0xFFFFFFFF
    return p


def test_blind_rotate_noise_free_closed_form(keys):
    s0 = keys["s0"]
    bk0 = trivial_bk(s0)
    g = W.rng(108)
    for _ in range(3):
        c = W.uniform_u32(g, (n + 1,))
        tv = (g.integers(0, 1 << 18, N, dtype=np.uint32) << 14).astype(np.uint32)  # exact under rounding
        acc = oracle.blind_rotate(bk0, c, tv)
        abar = np.array([oracle.modswitch(v) for v in c[:n]], dtype=np.int64)
        bbar = oracle.modswitch(c[n])
        phi = (bbar - int(np.sum(abar * s0))) % (2 * N)
        np.testing.assert_array_equal(acc[0], np.zeros(N, dtype=np.uint32))
        np.testing.assert_array_equal(acc[1], oracle.polymul(monomial(2 * N - phi), tv))


def test_trivial_inputs_give_exact_outputs(keys):
    """Inputs (0, +-1/8): every abar is 0, so the output is exactly (0, +-1/8)."""
    ops, i0, i1, want = [], [], [], []
    for op, f in TRUTH.items():
        for a in (0, 1):
            for b in (0, 1):
                ops.append(op)
                t0 = np.zeros(n + 1, dtype=np.uint32); t0[n] = MU if a else (-MU) & 0xFFFFFFFF
                t1 = np.zeros(n + 1, dtype=np.uint32); t1[n] = MU if b else (-MU) & 0xFFFFFFFF
                i0.append(t0); i1.append(t1); want.append(f(a, b))
    out = oracle.gates(keys["bk"], keys["ksk"], np.array(ops), np.array(i0), np.array(i1))
    exp = np.zeros_like(out)
    exp[:, n] = np.where(np.array(want) == 1, MU, (-MU) & 0xFFFFFFFF)
    np.testing.assert_array_equal(out, exp)


def test_every_gate_truth_table(keys):
    s0 = keys["s0"]
    g = W.rng(109)
    ops, a_bits, b_bits = [], [], []
    for op in TRUTH:
        for a in (0, 1):
            for b in (0, 1):
                ops.append(op); a_bits.append(a); b_bits.append(b)
    ops, a_bits, b_bits = np.array(ops), np.array(a_bits), np.array(b_bits)
    ea, eb = W.tlwe_draws(g, ops.size), W.tlwe_draws(g, ops.size)
    c0 = oracle.tlwe_encrypt_bits(s0, a_bits, *ea)
    c1 = oracle.tlwe_encrypt_bits(s0, b_bits, *eb)
    out = oracle.gates(keys["bk"], keys["ksk"], ops, c0, c1)
    want = np.array([TRUTH[o](a, b) for o, a, b in zip(ops, a_bits, b_bits)])
    np.testing.assert_array_equal(oracle.tlwe_decrypt(s0, out), want)
    # output noise is far inside the +-1/16 decision margin
    err = signed(oracle.tlwe_phase(s0, out)) - np.where(want == 1, MU, -MU)
    assert np.abs(err).max() < (1 << 26)
    # NOT needs no bootstrap: it negates the ciphertext
    notc, boot = oracle.gate_linear(oracle.NOT, c0[0], c0[0])
    assert not boot
    np.testing.assert_array_equal(notc, (0 - c0[0].astype(np.uint64)).astype(np.uint32))
    assert oracle.tlwe_decrypt(s0, notc) == 1 - a_bits[0]


def test_half_adder_from_paper(keys):
    spec = json.load(open(os.path.join(HERE, "golden", "half_adder.json")))
    s0 = keys["s0"]
    g = W.rng(110)
    rows = [(a, b) for a in (0, 1) for b in (0, 1)]
    A = np.array([r[0] for r in rows]); B = np.array([r[1] for r in rows])
    wires = {"A": oracle.tlwe_encrypt_bits(s0, A, *W.tlwe_draws(g, 4)),
             "B": oracle.tlwe_encrypt_bits(s0, B, *W.tlwe_draws(g, 4))}
    for name, op, *ins in spec["circuit"]:
        if op == "NOT":
            wires[name] = np.array([oracle.gate_linear(oracle.NOT, c, c)[0] for c in wires[ins[0]]])
        else:
            code = getattr(oracle, op)
            wires[name] = oracle.gates(keys["bk"], keys["ksk"], np.full(4, code), wires[ins[0]], wires[ins[1]])
    S = oracle.tlwe_decrypt(s0, wires["S"]); C = oracle.tlwe_decrypt(s0, wires["C"])
    np.testing.assert_array_equal(S, A ^ B)
    np.testing.assert_array_equal(C, A & B)
    for case in spec["printed_cases"]:
        k = rows.index((case["A"], case["B"]))
        assert (S[k], C[k]) == (case["S"], case["C"])


MUX_ROWS = [(s, a, b) for s in (0, 1) for a in (0, 1) for b in (0, 1)]


def trivial_bit(bit):
    t = np.zeros(n + 1, dtype=np.uint32)
    t[n] = MU if bit else (-MU) & 0xFFFFFFFF
    return t


def test_mux_trivial_inputs_exact(keys):
    """MUX(s, a, b) = s ? a : b: with trivial inputs every abar is 0, both halves bootstrap to
    exactly (0, +-1/8), and the result is exactly (0, +-1/8) for the selected bit."""
    S = np.array([trivial_bit(r[0]) for r in MUX_ROWS])
    A = np.array([trivial_bit(r[1]) for r in MUX_ROWS])
    Bb = np.array([trivial_bit(r[2]) for r in MUX_ROWS])
    out = oracle.muxes(keys["bk"], keys["ksk"], S, A, Bb)
    want = np.array([a if s else b for s, a, b in MUX_ROWS])
    np.testing.assert_array_equal(out, np.array([trivial_bit(w) for w in want]))


def test_mux_truth_table_and_control_unit(keys):
    """Encrypted inputs decrypt to s ? a : b over the full truth table (two draws), and the
    result is the SampleExtract + key switch of the RAM control unit's HomMUX without SE and
    IKS (Sec. 2.1.2) on the same inputs."""
    s0 = keys["s0"]
    g = W.rng(111)
    rows = MUX_ROWS * 2
    enc = lambda bits: oracle.tlwe_encrypt_bits(s0, np.array(bits), *W.tlwe_draws(g, len(bits)))
    S, A, Bb = enc([r[0] for r in rows]), enc([r[1] for r in rows]), enc([r[2] for r in rows])
    out = oracle.muxes(keys["bk"], keys["ksk"], S, A, Bb)
    want = np.array([a if s else b for s, a, b in rows])
    np.testing.assert_array_equal(oracle.tlwe_decrypt(s0, out), want)
    err = signed(oracle.tlwe_phase(s0, out)) - np.where(want == 1, MU, -MU)
    assert np.abs(err).max() < (1 << 26)
    for k in (0, 5, 11):
        u = oracle.ram_control(keys["bk"], S[k], A[k:k + 1], Bb[k:k + 1])[0]
        np.testing.assert_array_equal(out[k], oracle.keyswitch(keys["ksk"], oracle.sample_extract(u, 0)))

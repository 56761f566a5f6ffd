"""Pins of the oracle's circuit bootstrapping (TLWE -> TRGSW, Sec. 2.1.2 "Circuit
Bootstrapping"; used on the CMUX memory's address bits, Sec. 8.2) on the 2^64 torus, on
small parameter sets so that every check is brute force in Python integers: the level-2
products against the negacyclic definition, the decomposition against its defining bound,
the blind rotation with a noise-free key against its closed form, the private key switch
against the exact sum of its selected noise terms, and the whole conversion against the
gadget TRGSW's phases (noise-free keys) and as a CMUX selector (noisy keys)."""
import numpy as np
import pytest

import oracle
import workloads as W

M64 = (1 << 64) - 1
M32 = (1 << 32) - 1
P = oracle.Params(8, 16, 2, 4, 4, 2)       # level 0/1: n, N, output gadget l x 2^4
Q = oracle.Params2(32, 3, 8, 8, 2)         # level 2: N2, l2 x 2^8, private key switch 8 x 2 bits


def negacyclic(a, b, mod):
    """Brute-force product in Z[X]/(X^N+1) over Python integers, reduced mod `mod`."""
    N = len(a)
    out = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            if k < N:
                out[k] += int(a[i]) * int(b[j])
            else:
                out[k - N] -= int(a[i]) * int(b[j])
    return [x % mod for x in out]


def to_u64(xs):
    return np.array([int(x) & M64 for x in xs], dtype=np.uint64)


def test_polymul64_against_brute_force_and_limb_convolution():
    g = W.rng(600)
    for N in (1, 2, 4, 8, 16):
        a = W.uniform_u64(g, N)
        b = W.uniform_u64(g, N)
        assert [int(x) for x in oracle.polymul64(a, b)] == negacyclic(a, b, 1 << 64)
    # N = 2048 with small signed digits (the blind rotation's operands): 16-bit limbs of b,
    # numpy convolution of exact int64 partial sums, folded by X^N = -1
    N = 2048
    d = g.integers(-256, 256, N)
    b = W.uniform_u64(g, N)
    acc = [0] * N
    for limb in range(4):
        bl = ((b >> np.uint64(16 * limb)) & np.uint64(0xFFFF)).astype(np.int64)
        full = np.convolve(d, bl)
        folded = full[:N].copy()
        folded[:N - 1] -= full[N:]
        for i in range(N):
            acc[i] += int(folded[i]) << (16 * limb)
    got = oracle.polymul64(to_u64(d), b)
    assert [int(x) for x in got] == [x % (1 << 64) for x in acc]


def test_rotate64_is_the_monomial_product():
    g = W.rng(601)
    p = W.uniform_u64(g, 16)
    for k in range(32):
        mono = [0] * 16
        mono[k % 16] = 1 if k < 16 else -1
        assert [int(x) for x in oracle.rotate64(p, k)] == negacyclic(mono, p, 1 << 64), k


def test_decompose64_defining_bound():
    g = W.rng(602)
    xs = [0, 1, M64, 1 << 63, (1 << 63) - 1] + [int(x) for x in W.uniform_u64(g, 400)]
    step = 64 - Q.l * Q.bgbit
    for x in xs:
        d = [int(v) for v in oracle.decompose64(x, Q)]
        assert all(-(1 << (Q.bgbit - 1)) <= v < (1 << (Q.bgbit - 1)) for v in d)
        rec = sum(v << (64 - Q.bgbit * (r + 1)) for r, v in enumerate(d)) % (1 << 64)
        want = (((x + (1 << (step - 1))) >> step) << step) % (1 << 64)   # nearest multiple of 2^step
        assert rec == want, hex(x)


def test_trlwe64_phase_is_message_plus_noise():
    g = W.rng(603)
    s2 = W.secret_key2(3, Q.N)
    a, m = W.uniform_u64(g, Q.N), W.uniform_u64(g, Q.N)
    e = W.gaussian_i64(g, 2.0 ** -44, Q.N)
    c = oracle.trlwe64_encrypt_torus(s2, m, a, e)
    assert [int(x) for x in c[1]] == [(int(x) + int(y) + int(z)) % (1 << 64)
                                       for x, y, z in zip(negacyclic(a, s2, 1 << 64), m, e)]
    assert [int(x) for x in oracle.trlwe64_phase(s2, c)] == [(int(x) + int(y)) % (1 << 64) for x, y in zip(m, e)]


def gadget64(m):
    """Trivial level-2 TRGSW of a bit (zero masks, zero noise)."""
    return oracle.trgsw64_encrypt(np.zeros(Q.N, np.uint64), m, np.zeros((2 * Q.l, Q.N), np.uint64),
                                  np.zeros((2 * Q.l, Q.N), np.int64), Q)


def test_external_product64_exact_identities():
    g = W.rng(604)
    x = W.uniform_u64(g, (2, Q.N))
    step = 64 - Q.l * Q.bgbit
    rounded = [(((int(v) + (1 << (step - 1))) >> step) << step) % (1 << 64) for v in x.reshape(-1)]
    assert [int(v) for v in oracle.external_product64(gadget64(1), x, Q).reshape(-1)] == rounded
    assert not oracle.external_product64(gadget64(0), x, Q).any()
    # encrypted selector: phase(out) = m round(phase(x)) + sum_q d_q e_q exactly (the masks cancel)
    s2 = W.secret_key2(3, Q.N)
    masks, noise = W.uniform_u64(g, (2 * Q.l, Q.N)), W.gaussian_i64(g, 2.0 ** -44, (2 * Q.l, Q.N))
    for m in (0, 1):
        C = oracle.trgsw64_encrypt(s2, m, masks, noise, Q)
        out = oracle.external_product64(C, x, Q)
        digs = [[int(v) for v in oracle.decompose64(int(x[h, j]), Q)] for h in range(2) for j in range(Q.N)]
        err = [0] * Q.N
        for h in range(2):
            for r in range(Q.l):
                dq = [digs[h * Q.N + j][r] for j in range(Q.N)]
                for k, v in enumerate(negacyclic(dq, noise[h * Q.l + r], 1 << 64)):
                    err[k] += v
        ra = to_u64(rounded[:Q.N]); rb = to_u64(rounded[Q.N:])
        ph_round = [(int(b_) - int(v)) % (1 << 64) for b_, v in zip(rb, negacyclic(ra, s2, 1 << 64))]
        want = [(m * p + e_) % (1 << 64) for p, e_ in zip(ph_round, err)]
        assert [int(v) for v in oracle.trlwe64_phase(s2, out)] == want, m


def test_blind_rotate64_noise_free_closed_form():
    g = W.rng(605)
    s0 = g.integers(0, 2, P.n).astype(np.uint32)
    bk2 = np.stack([gadget64(int(b)) for b in s0])
    tv = np.full(Q.N, 1 << 50, dtype=np.uint64)
    for trial in range(6):
        c = W.uniform_u32(g, P.n + 1)
        acc = oracle.blind_rotate64(bk2, c, tv, Q)
        sh = 32 - (2 * Q.N).bit_length() + 1
        ms = [((int(x) + (1 << (sh - 1))) >> sh) % (2 * Q.N) for x in c]     # round(x 2N2 / 2^32)
        k = (ms[P.n] - sum(ms[i] * int(s0[i]) for i in range(P.n))) % (2 * Q.N)
        mono = [0] * Q.N                                                    # X^{-k}
        kk = (2 * Q.N - k) % (2 * Q.N)
        mono[kk % Q.N] = 1 if kk < Q.N else -1
        assert not acc[0].any()
        assert [int(v) for v in acc[1]] == negacyclic(mono, tv, 1 << 64), trial


def test_sample_extract64_phase():
    g = W.rng(606)
    s2 = W.secret_key2(3, Q.N)
    c = W.uniform_u64(g, (2, Q.N))
    t = oracle.sample_extract64(c)
    ph = (int(t[Q.N]) - sum(int(t[j]) * int(s2[j]) for j in range(Q.N))) % (1 << 64)
    assert ph == int(oracle.trlwe64_phase(s2, c)[0])


def small_keys(g, sigma2, sigma_pks):
    s0 = g.integers(0, 2, P.n).astype(np.uint32)
    s1 = g.integers(0, 2, P.N).astype(np.uint32)
    s2 = g.integers(0, 2, Q.N).astype(np.uint64)
    m2 = W.uniform_u64(g, (P.n, 2 * Q.l, Q.N)) if sigma2 is not None else np.zeros((P.n, 2 * Q.l, Q.N), np.uint64)
    e2 = W.gaussian_i64(g, sigma2 or 0.0, (P.n, 2 * Q.l, Q.N))
    shape = (2, Q.N + 1, Q.t, (1 << Q.basebit) - 1, P.N)
    mk = W.uniform_u32(g, shape) if sigma_pks is not None else np.zeros(shape, np.uint32)
    ek = W.gaussian_i32(g, sigma_pks or 0.0, shape)
    bk2 = oracle.bk2_gen(s0, s2, m2, e2, Q)
    pksk = oracle.pksk_gen(s1, s2, mk, ek, P, Q)
    return s0, s1, s2, bk2, pksk, ek


def f_message(u, s1, x32):
    """f_0(x) = -s1 x, f_1(x) = x (constant polynomial), on the 2^32 torus."""
    if u == 0:
        return [(-int(s) * x32) % (1 << 32) for s in s1]
    return [x32 % (1 << 32)] + [0] * (len(s1) - 1)


def rounded_phase32(s2, c):
    """sum_k z_k chat_k with z = (-s2, 1) and chat_k = c_k rounded to t2 basebit2 bits, as a
    2^32 torus value."""
    tb = Q.t * Q.basebit
    ch = [((int(v) + (1 << (64 - tb - 1))) >> (64 - tb)) % (1 << tb) for v in c]
    tot = ch[Q.N] - sum(ch[k] * int(s2[k]) for k in range(Q.N))
    return (tot << (32 - tb)) % (1 << 32)


def test_private_keyswitch_exact_with_noise_terms():
    g = W.rng(607)
    s0, s1, s2, bk2, pksk, ek = small_keys(g, None, 2.0 ** -30)
    base = 1 << Q.basebit
    tb = Q.t * Q.basebit
    for trial in range(4):
        c = W.uniform_u64(g, Q.N + 1)
        x = rounded_phase32(s2, c)
        for u in (0, 1):
            out = oracle.private_keyswitch(pksk, u, c, P, Q)
            noise = [0] * P.N
            for k in range(Q.N + 1):
                chat = ((int(c[k]) + (1 << (64 - tb - 1))) >> (64 - tb)) % (1 << tb)
                for p in range(Q.t):
                    v = (chat >> (Q.basebit * (Q.t - 1 - p))) & (base - 1)
                    if v:
                        for j in range(P.N):
                            noise[j] += int(ek[u, k, p, v - 1, j])
            ph = [(int(b_) - int(v)) % (1 << 32) for b_, v in zip(out[1], negacyclic(out[0], s1, 1 << 32))]
            want = [(m + e) % (1 << 32) for m, e in zip(f_message(u, s1, x), noise)]
            assert ph == want, (trial, u)


def gadget_phase_rows(s1, m):
    """Phases of the gadget TRGSW of m under s1: row r < l: -m s1 / Bg^(r+1); row l + r:
    m / Bg^(r+1) in the constant coefficient."""
    rows = []
    for r in range(2 * P.l):
        j = r % P.l + 1
        g_ = 1 << (32 - P.bgbit * j)
        rows.append(f_message(0 if r < P.l else 1, s1, m * g_))
    return rows


def test_circuit_bootstrap_noise_free_equals_gadget_phases():
    g = W.rng(608)
    s0, s1, s2, bk2, pksk, _ = small_keys(g, None, None)
    for trial in range(8):
        bit = trial & 1
        a = W.uniform_u32(g, P.n)
        e = int(g.integers(-(1 << 20), 1 << 20))
        c = oracle.tlwe_encrypt_bits(s0, [bit], a[None, :], np.array([e], np.int32))[0]
        C = oracle.circuit_bootstrap(bk2, pksk, c, P, Q)
        want = gadget_phase_rows(s1, bit)
        for r in range(2 * P.l):
            ph = [(int(b_) - int(v)) % (1 << 32) for b_, v in zip(C[r, 1], negacyclic(C[r, 0], s1, 1 << 32))]
            assert ph == want[r], (trial, r)


def test_circuit_bootstrap_output_selects_in_a_cmux():
    """Noisy keys: the TRGSW made from an encrypted bit picks the right one of two encrypted
    TRLWE in a CMUX, and its rows' phases are within a small bound of the gadget's."""
    g = W.rng(609)
    s0, s1, s2, bk2, pksk, _ = small_keys(g, 2.0 ** -44, 2.0 ** -30)
    for trial in range(6):
        bit = trial & 1
        c = oracle.tlwe_encrypt_bits(s0, [bit], W.uniform_u32(g, (1, P.n)), W.gaussian_i32(g, 2.0 ** -15, 1))[0]
        C = oracle.circuit_bootstrap(bk2, pksk, c, P, Q)
        want = gadget_phase_rows(s1, bit)
        for r in range(2 * P.l):
            ph = [(int(b_) - int(v)) % (1 << 32) for b_, v in zip(C[r, 1], negacyclic(C[r, 0], s1, 1 << 32))]
            dev = [((p - w + (1 << 31)) % (1 << 32)) - (1 << 31) for p, w in zip(ph, want[r])]
            # key-switch rounding (t2 basebit2 bits per key coefficient) plus noise
            bound = (Q.N + 1) * (1 << (32 - Q.t * Q.basebit - 1)) + (1 << 14)
            assert max(abs(d) for d in dev) < bound, (trial, r)
        bits0, bits1 = g.integers(0, 2, P.N), g.integers(0, 2, P.N)
        x0 = oracle.trlwe_encrypt_bits(s1, bits0, W.uniform_u32(g, P.N), W.gaussian_i32(g, 2.0 ** -25, P.N))
        x1 = oracle.trlwe_encrypt_bits(s1, bits1, W.uniform_u32(g, P.N), W.gaussian_i32(g, 2.0 ** -25, P.N))
        out = oracle.cmux(C, x0, x1, P)
        ph = oracle.trlwe_phase(s1, out)
        got = (ph.view(np.int32) >= 0).astype(int)
        assert np.array_equal(got, bits1 if bit else bits0), trial


def test_batched_circuit_bootstraps_equal_single_ones():
    g = W.rng(610)
    s0, s1, s2, bk2, pksk, _ = small_keys(g, 2.0 ** -44, 2.0 ** -30)
    cs = oracle.tlwe_encrypt_bits(s0, [1, 0, 1], W.uniform_u32(g, (3, P.n)), W.gaussian_i32(g, 2.0 ** -15, 3))
    many = oracle.circuit_bootstraps(bk2, pksk, cs, P, Q, threads=4)
    for i in range(3):
        assert np.array_equal(many[i], oracle.circuit_bootstrap(bk2, pksk, cs[i], P, Q)), i

"""The algebra the matrix-core blind rotation relies on when its operands carry the gadget digits
plus 32 (Sec. 2.1.2, external product): with the offset, each row's product gains 32 times the
row key times the all-ones polynomial, and the correction C[i] = 64 S_i - 32 S_{N-1} (S the
prefix sums of the six row keys' sum, all mod 2^32) removes it exactly; and the sum segment
x0 + x1 of two offset digit words is a plain 32-bit add, as no byte sum reaches 256. Checked
here with the oracle's schoolbook negacyclic product and its gadget decomposition."""
import numpy as np

import oracle
import workloads as W

N, ROWS, L, BG_BIT = 1024, 6, 3, 6


def correction(keys):
    """C[i] = 64 S_i - 32 S_{N-1} mod 2^32 for S the prefix sums of the row keys' sum."""
    s = np.cumsum(keys.astype(np.uint64).sum(axis=0) % (1 << 32)) % (1 << 32)
    return ((64 * s - 32 * s[-1]) % (1 << 32)).astype(np.uint32)


def digit_rows(g):
    """Balanced gadget digits of two random torus polynomials (rows 3h + k), by the oracle."""
    acc = W.uniform_u32(g, (2, N))
    d = np.zeros((ROWS, N), np.int64)
    for h in range(2):
        for j in range(N):
            d[3 * h:3 * h + 3, j] = oracle.decompose(int(acc[h, j]))
    return d


def test_offset_correction_restores_the_products():
    g = W.rng(9100)
    keys = W.uniform_u32(g, (ROWS, N))
    d = digit_rows(g)
    assert d.min() >= -32 and d.max() <= 31
    plain = np.zeros(N, np.uint64)
    offset = np.zeros(N, np.uint64)
    for r in range(ROWS):
        plain += oracle.polymul(keys[r], (d[r] % (1 << 32)).astype(np.uint32)).astype(np.uint64)
        offset += oracle.polymul(keys[r], (d[r] + 32).astype(np.uint32)).astype(np.uint64)
    plain %= 1 << 32
    got = (offset + (1 << 32) - correction(keys).astype(np.uint64)) % (1 << 32)
    np.testing.assert_array_equal(got, plain)


def test_correction_of_a_single_coefficient_key():
    # K = X^t in one row: K * (1 + .. + X^{N-1}) is -1 below t and +1 from t on
    for t in (0, 1, 511, 1023):
        keys = np.zeros((ROWS, N), np.uint32)
        keys[2, t] = 1
        want = np.where(np.arange(N) >= t, 32, -32) % (1 << 32)
        np.testing.assert_array_equal(correction(keys), want.astype(np.uint32))


def test_sum_segment_is_a_carry_free_word_add():
    g = W.rng(9101)
    x0 = g.integers(0, 64, (4096, 4)).astype(np.uint32)  # digits plus 32, four per word
    x1 = g.integers(0, 64, (4096, 4)).astype(np.uint32)
    pack = lambda b: (b[:, 0] | b[:, 1] << 8 | b[:, 2] << 16 | b[:, 3] << 24).astype(np.uint32)
    np.testing.assert_array_equal(pack(x0) + pack(x1), pack(x0 + x1))
    assert (x0 + x1).max() <= 126

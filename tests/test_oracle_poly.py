"""Pins of the oracle's negacyclic product in Z[X]/(X^N+1) mod 2^32 (the ring of Sec. 2.1.2).

Checked against things other than the oracle: big-integer brute force on tiny N, numpy's
linear convolution folded by X^N = -1 (exact via 16-bit limbs), and closed forms
(monomial products, identity, linearity, commutativity).
"""
import itertools

import numpy as np
import pytest

import oracle

M32 = (1 << 32) - 1


def brute_negacyclic(a, b):
    """Python big-int schoolbook in Z[X]/(X^N+1), reduced mod 2^32."""
    N = len(a)
    out = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            if k < N:
                out[k] += int(a[i]) * int(b[j])
            else:
                out[k - N] -= int(a[i]) * int(b[j])
    return np.array([x & M32 for x in out], dtype=np.uint32)


def numpy_negacyclic(a, b):
    """np.convolve on 16-bit limbs (exact in int64), folded with X^N = -1, mod 2^32."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    N = a.size
    a0, a1 = (a & 0xFFFF).astype(np.int64), (a >> 16).astype(np.int64)
    b0, b1 = (b & 0xFFFF).astype(np.int64), (b >> 16).astype(np.int64)

    def fold(c):
        full = np.zeros(2 * N, dtype=np.int64)
        full[: 2 * N - 1] = c
        return full[:N] - full[N:]

    lo = fold(np.convolve(a0, b0))
    mid = fold(np.convolve(a0, b1)) + fold(np.convolve(a1, b0))
    tot = (lo.astype(object) + (mid.astype(object) << 16))
    return np.array([int(x) & M32 for x in tot], dtype=np.uint32)


@pytest.mark.parametrize("N", [1, 2])
def test_exhaustive_tiny(N):
    alphabet = [0, 1, 2, 0x80000000, M32]
    for a in itertools.product(alphabet, repeat=N):
        for b in itertools.product(alphabet, repeat=N):
            a_ = np.array(a, dtype=np.uint32)
            b_ = np.array(b, dtype=np.uint32)
            np.testing.assert_array_equal(oracle.polymul(a_, b_), brute_negacyclic(a_, b_))


def test_exhaustive_n4_small_alphabet():
    alphabet = [0, 1, M32]
    for a in itertools.product(alphabet, repeat=4):
        a_ = np.array(a, dtype=np.uint32)
        for b in itertools.product(alphabet, repeat=4):
            b_ = np.array(b, dtype=np.uint32)
            np.testing.assert_array_equal(oracle.polymul(a_, b_), brute_negacyclic(a_, b_))


@pytest.mark.parametrize("N", [8, 16, 64])
def test_random_vs_bigint(N):
    g = np.random.default_rng(N)
    for _ in range(5):
        a = g.integers(0, 2 ** 32, N, dtype=np.uint64).astype(np.uint32)
        b = g.integers(0, 2 ** 32, N, dtype=np.uint64).astype(np.uint32)
        np.testing.assert_array_equal(oracle.polymul(a, b), brute_negacyclic(a, b))


def test_random_n1024_vs_numpy_convolve():
    g = np.random.default_rng(1024)
    for _ in range(3):
        a = g.integers(0, 2 ** 32, 1024, dtype=np.uint64).astype(np.uint32)
        b = g.integers(0, 2 ** 32, 1024, dtype=np.uint64).astype(np.uint32)
        np.testing.assert_array_equal(oracle.polymul(a, b), numpy_negacyclic(a, b))
    # small signed digits times torus values, as in the external product
    d = g.integers(-32, 32, 1024).astype(np.int64).astype(np.uint32)
    a = g.integers(0, 2 ** 32, 1024, dtype=np.uint64).astype(np.uint32)
    np.testing.assert_array_equal(oracle.polymul(d, a), numpy_negacyclic(d, a))


def monomial(N, k):
    """X^k for k in [0, 2N): X^N = -1."""
    p = np.zeros(N, dtype=np.uint32)
    k %= 2 * N
    if k < N:
        p[k] = 1
    else:
        p[k - N] = M32
    return p


def test_monomial_closed_form():
    N = 16
    for a in range(2 * N):
        for b in range(2 * N):
            np.testing.assert_array_equal(oracle.polymul(monomial(N, a), monomial(N, b)), monomial(N, a + b))


def test_rotate_is_monomial_product():
    g = np.random.default_rng(7)
    for N in (16, 1024):
        p = g.integers(0, 2 ** 32, N, dtype=np.uint64).astype(np.uint32)
        for k in [0, 1, 5, N - 1, N, N + 1, 2 * N - 1] + list(g.integers(0, 2 * N, 4)):
            np.testing.assert_array_equal(oracle.rotate(p, k), oracle.polymul(monomial(N, int(k)), p))


def test_identity_linearity_commutativity():
    g = np.random.default_rng(11)
    N = 1024
    a, b, c = (g.integers(0, 2 ** 32, N, dtype=np.uint64).astype(np.uint32) for _ in range(3))
    np.testing.assert_array_equal(oracle.polymul(monomial(N, 0), a), a)
    np.testing.assert_array_equal(oracle.polymul(a, b), oracle.polymul(b, a))
    np.testing.assert_array_equal(oracle.polymul(a, b + c), oracle.polymul(a, b) + oracle.polymul(a, c))

"""Pins of the oracle's scalar steps: gadget decomposition, modulus switch, key-switch digits.

The exhaustive check runs every 32-bit torus value through the oracle and tests the
defining bounds (digit ranges and reconstruction error), in a small C program under
tests/c. Spot values below are worked by hand.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("exh") / "exhaustive")
    subprocess.run(["gcc", "-O2", "-pthread", "-o", exe, os.path.join(HERE, "c", "exhaustive.c"), "-ldl"],
                   check=True)
    return exe


def test_exhaustive_all_32bit_values(checker):
    threads = max(1, len(os.sched_getaffinity(0)))
    r = subprocess.run([checker, oracle.build(force=False), str(threads)], capture_output=True, text=True,
                       timeout=900)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr


def test_decompose_hand_values():
    # 0 decomposes to all-zero digits (the rounding offset cancels exactly).
    np.testing.assert_array_equal(oracle.decompose(0), [0, 0, 0])
    # 1/Bg = 2^26 -> (1, 0, 0); 1/Bg^3 = 2^14 -> (0, 0, 1); -1/Bg^2 = -2^20 -> (0, -1, 0).
    np.testing.assert_array_equal(oracle.decompose(1 << 26), [1, 0, 0])
    np.testing.assert_array_equal(oracle.decompose(1 << 14), [0, 0, 1])
    np.testing.assert_array_equal(oracle.decompose((-(1 << 20)) & 0xFFFFFFFF), [0, -1, 0])
    # 2^13 rounds up to 2^14; 2^13 - 1 rounds down to 0.
    np.testing.assert_array_equal(oracle.decompose(1 << 13), [0, 0, 1])
    np.testing.assert_array_equal(oracle.decompose((1 << 13) - 1), [0, 0, 0])
    # -1/2 = 2^31 -> most significant digit -32.
    np.testing.assert_array_equal(oracle.decompose(1 << 31), [-32, 0, 0])


def test_modswitch_hand_values():
    assert oracle.modswitch(0) == 0
    assert oracle.modswitch((1 << 20) - 1) == 0      # just below half a bucket
    assert oracle.modswitch(1 << 20) == 1            # half a bucket rounds up
    assert oracle.modswitch(0xFFFFFFFF) == 0         # wraps to 0
    assert oracle.modswitch(1 << 29) == 256          # 1/8 -> 2N/8
    assert oracle.modswitch(1 << 31) == 1024         # 1/2 -> N


def test_ks_digits_hand_values():
    np.testing.assert_array_equal(oracle.ks_digits(0), [0] * 8)
    np.testing.assert_array_equal(oracle.ks_digits(1 << 30), [1, 0, 0, 0, 0, 0, 0, 0])
    np.testing.assert_array_equal(oracle.ks_digits(3 << 16), [0, 0, 0, 0, 0, 0, 0, 3])
    np.testing.assert_array_equal(oracle.ks_digits((1 << 15) - 1), [0] * 8)   # rounds down
    np.testing.assert_array_equal(oracle.ks_digits(1 << 15), [0, 0, 0, 0, 0, 0, 0, 1])  # rounds up

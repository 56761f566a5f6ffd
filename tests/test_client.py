"""The library's client side (key generation, encryption, decryption in numpy) against the
oracle: both compute from the same seeded draws, independently, and must agree bit for bit."""
import numpy as np

import oracle
import workloads as W
from paper_2010_09410_amd import client


def test_keys_match_oracle(keys):
    bk, ksk = client.keyset(keys["s0"], keys["s1"], keys["bkd"], keys["kskd"])
    np.testing.assert_array_equal(bk, keys["bk"])
    np.testing.assert_array_equal(ksk, keys["ksk"])


def test_encryptions_match_oracle(keys):
    s0, s1 = keys["s0"], keys["s1"]
    g = W.rng(400)
    bits = g.integers(0, 2, 32)
    a, e = W.tlwe_draws(g, 32)
    np.testing.assert_array_equal(client.tlwe_encrypt_bits(s0, bits, a, e), oracle.tlwe_encrypt_bits(s0, bits, a, e))
    np.testing.assert_array_equal(client.tlwe_decrypt(s0, client.tlwe_encrypt_bits(s0, bits, a, e)), bits)
    ma, me = W.trlwe_draws(g, 3)
    msg = W.uniform_u32(g, (3, 1024))
    for i in range(3):
        np.testing.assert_array_equal(client.trlwe_encrypt_torus(s1, msg[i], ma[i], me[i]),
                                      oracle.trlwe_encrypt_torus(s1, msg[i], ma[i], me[i]))
    ta, te = W.trgsw_draws(g, 2)
    for m in (0, 1):
        np.testing.assert_array_equal(client.trgsw_encrypt(s1, m, ta[m], te[m]), oracle.trgsw_encrypt(s1, m, ta[m], te[m]))
    np.testing.assert_array_equal(client.trivial_trgsw(1), oracle.trgsw_gadget())


def test_phase_and_decrypt(keys):
    s1 = keys["s1"]
    g = W.rng(401)
    c = W.uniform_u32(g, (2, 1024))
    np.testing.assert_array_equal(client.trlwe_phase(s1, c), oracle.trlwe_phase(s1, c))
    t = W.uniform_u32(g, (5, 631))
    np.testing.assert_array_equal(client.tlwe_phase(keys["s0"], t), oracle.tlwe_phase(keys["s0"], t))


def test_memory_encodings():
    words = np.array([0x80000001, 0x00000002] + [0] * 30, dtype=np.uint32)
    msg = client.pack_rom(words)
    assert msg.shape == (1, 1024)
    mu, neg = 1 << 29, (-(1 << 29)) & 0xFFFFFFFF
    assert msg[0, 0] == mu and msg[0, 31] == mu and msg[0, 1] == neg   # word 0: bits 0 and 31
    assert msg[0, 32 + 1] == mu and msg[0, 32] == neg                  # word 1: bit 1
    cells = client.ram_cell_messages(np.array([[1, 0]]))
    assert cells[0, 0, 0] == mu and cells[0, 1, 0] == neg and (cells[0, :, 1:] == neg).all()

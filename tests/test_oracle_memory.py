"""Pins of the oracle's CMUX Memory (Sec. 8): ROM and RAM reads, the RAM write, and the
CMUX counts of the paper's appendix table.

* With trivial (noise-free, mask-free) selectors and cells every CMUX selects exactly, so
  every ROM address and every RAM address is checked against the plaintext exactly.
* With encrypted selectors and cells, sampled reads and a write-then-read decrypt correctly.
* CMUX counts: RAM read w(2^v - 1), RAM write unit w 2^v v, ROM (#polys - 1) + log2(words per
  polynomial), and the paper's own figures 4,080 / 32,768 / 8 for its 512-byte memories.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

P = oracle.DEFAULT
N, n, l = P.N, P.n, P.l
MU = 1 << 29
NEG = (-MU) & 0xFFFFFFFF
HERE = os.path.dirname(os.path.abspath(__file__))


def pack_rom(words, N=N, wbits=32):
    """Plaintext polynomials: coefficient wbits*q + b of polynomial h holds bit b of word
    (N/wbits)*h + q, encoded mu(2m - 1)."""
    per = N // wbits
    npoly = len(words) // per
    msg = np.zeros((npoly, N), dtype=np.uint32)
    for h in range(npoly):
        for q in range(per):
            w = int(words[per * h + q])
            for b in range(wbits):
                msg[h, wbits * q + b] = MU if (w >> b) & 1 else NEG
    return msg


def trivial_selectors(value, bits, P=P):
    G = oracle.trgsw_gadget(P)
    return np.array([((value >> j) & 1) * G for j in range(bits)], dtype=np.uint32)


def trivial_trlwe(msg):
    return np.stack([np.zeros_like(msg), msg], axis=-2)


def test_rom_every_address_exact_with_trivial_selectors():
    wl = W.rom_workload()
    words = wl["words"]
    msg = pack_rom(words)
    rom = trivial_trlwe(msg)                              # [16][2][N]
    sels = np.array([trivial_selectors(a, 9) for a in range(512)])
    out = oracle.rom_reads(np.zeros((N, 8, 3, n + 1), dtype=np.uint32), rom, sels)
    want_bits = (words[:, None] >> np.arange(32)[None, :]) & 1          # [512][32]
    want = np.zeros_like(out)
    want[:, :, n] = np.where(want_bits == 1, MU, NEG)
    np.testing.assert_array_equal(out, want)


def test_rom_encrypted_sample(keys):
    s0, s1 = keys["s0"], keys["s1"]
    wl = W.rom_workload(reads=4)
    msg = pack_rom(wl["words"])
    ca, ce = wl["cells"]
    rom = np.array([oracle.trlwe_encrypt_torus(s1, msg[h], ca[h], ce[h]) for h in range(16)])
    sa, se = wl["sel"]
    sels = np.array([[oracle.trgsw_encrypt(s1, (int(wl["addr"][r]) >> j) & 1, sa[r, j], se[r, j])
                      for j in range(9)] for r in range(4)])
    out = oracle.rom_reads(keys["ksk"], rom, sels)
    for r in range(4):
        bits = (int(wl["words"][wl["addr"][r]]) >> np.arange(32)) & 1
        np.testing.assert_array_equal(oracle.tlwe_decrypt(s0, out[r]), bits)


def ram_cells_msg(contents):
    """Cell message m X^0: constant coefficient +-mu, the others -mu."""
    w, A = contents.shape
    msg = np.full((w, A, N), NEG, dtype=np.uint32)
    msg[:, :, 0] = np.where(contents == 1, MU, NEG)
    return msg


def test_ram_read_every_address_exact_with_trivial_selectors():
    g = W.rng(300)
    v, w = 5, 3
    contents = g.integers(0, 2, (w, 2 ** v)).astype(np.uint8)
    ram = trivial_trlwe(ram_cells_msg(contents))          # [w][2^v][2][N]
    sels = np.array([trivial_selectors(a, v) for a in range(2 ** v)])
    out = oracle.ram_reads(np.zeros((N, 8, 3, n + 1), dtype=np.uint32), ram, sels)
    want = np.zeros_like(out)
    want[:, :, n] = np.where(contents.T == 1, MU, NEG)
    np.testing.assert_array_equal(out, want)


@pytest.mark.parametrize("flag", [1, 0])
def test_ram_write_exact_with_trivial_inputs(keys, flag):
    """Trivial RAM, selectors, flag and data: every refreshed cell is exactly the blind
    rotation of its new bit, (0, X^{-bbar} tv) with bbar = 256 for 1 and 1792 for 0."""
    g = W.rng(301 + flag)
    v, w = 4, 2
    contents = g.integers(0, 2, (w, 2 ** v)).astype(np.uint8)
    waddr = int(g.integers(0, 2 ** v))
    data = g.integers(0, 2, w).astype(np.uint8)
    ram = trivial_trlwe(ram_cells_msg(contents))
    sel = trivial_selectors(waddr, v)
    fl = np.zeros(n + 1, dtype=np.uint32); fl[n] = MU if flag else NEG
    dat = np.zeros((w, n + 1), dtype=np.uint32); dat[:, n] = np.where(data == 1, MU, NEG)
    new = oracle.ram_write(keys["bk"], keys["ksk"], ram, sel, fl, dat)
    tv = np.full(N, MU, dtype=np.uint32)
    for i in range(w):
        for A in range(2 ** v):
            bit = int(data[i]) if (A == waddr and flag) else int(contents[i, A])
            bbar = 256 if bit else 1792
            np.testing.assert_array_equal(new[i, A, 0], np.zeros(N, dtype=np.uint32))
            np.testing.assert_array_equal(new[i, A, 1], oracle.rotate(tv, 2 * N - bbar))


@pytest.mark.parametrize("flag", [1, 0])
def test_ram_write_then_read_encrypted(keys, flag):
    s0, s1 = keys["s0"], keys["s1"]
    v, w = 3, 2
    wl = W.ram_workload(v=v, w=w, reads=2 ** v, flag=flag, seed_off=flag)
    ca, ce = wl["cells"]
    msg = ram_cells_msg(wl["contents"])
    ram = np.array([[oracle.trlwe_encrypt_torus(s1, msg[i, A], ca[i, A], ce[i, A]) for A in range(2 ** v)]
                    for i in range(w)])
    sa, se = wl["wsel"]
    sel = np.array([oracle.trgsw_encrypt(s1, (wl["waddr"] >> j) & 1, sa[j], se[j]) for j in range(v)])
    fl = oracle.tlwe_encrypt_bits(s0, [flag], *wl["fenc"])[0]
    dat = oracle.tlwe_encrypt_bits(s0, wl["wdata"], *wl["denc"])
    new = oracle.ram_write(keys["bk"], keys["ksk"], ram, sel, fl, dat)
    # read back every address with fresh encrypted selectors
    ra, re_ = wl["rsel"]
    rsels = np.array([[oracle.trgsw_encrypt(s1, (A >> j) & 1, ra[A, j], re_[A, j]) for j in range(v)]
                      for A in range(2 ** v)])
    out = oracle.ram_reads(keys["ksk"], new, rsels)
    expect = wl["contents"].copy()
    if flag:
        expect[:, wl["waddr"]] = wl["wdata"]
    for A in range(2 ** v):
        np.testing.assert_array_equal(oracle.tlwe_decrypt(s0, out[A]), expect[:, A])


def test_write_bars_equal_the_full_write(keys):
    """The sampled write-bar routine (the checker of large RAM writes) over every (bit,
    address) pair, in a shuffled order and again for a repeated subset, returns exactly the
    cells of the whole RAM write, given the read unit's and the control unit's outputs."""
    s0, s1 = keys["s0"], keys["s1"]
    v, w = 3, 2
    wl = W.ram_workload(v=v, w=w, reads=1, flag=1, seed_off=7)
    ca, ce = wl["cells"]
    msg = ram_cells_msg(wl["contents"])
    ram = np.array([[oracle.trlwe_encrypt_torus(s1, msg[i, A], ca[i, A], ce[i, A]) for A in range(2 ** v)]
                    for i in range(w)])
    sa, se = wl["wsel"]
    sel = np.array([oracle.trgsw_encrypt(s1, (wl["waddr"] >> j) & 1, sa[j], se[j]) for j in range(v)])
    fl = oracle.tlwe_encrypt_bits(s0, [1], *wl["fenc"])[0]
    dat = oracle.tlwe_encrypt_bits(s0, wl["wdata"], *wl["denc"])
    new = oracle.ram_write(keys["bk"], keys["ksk"], ram, sel, fl, dat).reshape(-1, 2, N)
    rd = oracle.ram_read(keys["ksk"], ram, sel)
    u = oracle.ram_control(keys["bk"], fl, dat, rd)
    idx = W.rng(302).permutation(w * 2 ** v)
    np.testing.assert_array_equal(oracle.ram_write_bars(keys["bk"], keys["ksk"], ram, sel, u, idx), new[idx])
    few = np.array([idx[3], idx[0], idx[3]])
    np.testing.assert_array_equal(oracle.ram_write_bars(keys["bk"], keys["ksk"], ram, sel, u, few), new[few])


SMALL = oracle.Params(16, 64, 3, 6, 8, 2)


def test_cmux_counts_match_paper_table():
    spec = json.load(open(os.path.join(HERE, "golden", "cmux_counts.json")))
    # RAM read unit and write unit, v = 8, w = 16 (structure does not depend on N; small N for speed)
    Ps = SMALL
    v, w = spec["ram_read"]["v"], spec["ram_read"]["w"]
    ram = np.zeros((w, 2 ** v, 2, Ps.N), dtype=np.uint32)
    sel = trivial_selectors(5, v, Ps)
    bk = np.zeros((Ps.n, 2 * Ps.l, 2, Ps.N), dtype=np.uint32)
    ksk = np.zeros((Ps.N, Ps.t, 3, Ps.n + 1), dtype=np.uint32)
    oracle.reset_counters()
    oracle.ram_read(ksk, ram, sel, P=Ps)
    read_cmux = oracle.cmux_count()
    assert read_cmux == w * (2 ** v - 1) == spec["ram_read"]["cmux"]
    oracle.reset_counters()
    oracle.ram_write(bk, ksk, ram, sel, np.zeros(Ps.n + 1, np.uint32), np.zeros((w, Ps.n + 1), np.uint32), P=Ps)
    assert oracle.cmux_count() - read_cmux == w * 2 ** v * v == spec["ram_write"]["cmux"]
    assert oracle.br_count() == 2 * w + w * 2 ** v      # control unit + refresh of every cell
    # ROM: 512 bytes of 32-bit words at N = 1024 -> 4 polynomials of 32 words
    words = np.zeros(spec["rom"]["bytes"] // 4, dtype=np.uint32)
    rom = trivial_trlwe(pack_rom(words))
    assert rom.shape[0] == 4
    oracle.reset_counters()
    oracle.rom_read(np.zeros((N, 8, 3, n + 1), np.uint32), rom, trivial_selectors(77, 7))
    assert oracle.cmux_count() == (4 - 1) + 5 == spec["rom"]["cmux"]
    # the 16-polynomial ROM of the 512-word workload: 15 tree CMUXes + 5 rotations
    oracle.reset_counters()
    oracle.rom_read(np.zeros((N, 8, 3, n + 1), np.uint32), trivial_trlwe(pack_rom(np.zeros(512, np.uint32))),
                    trivial_selectors(77, 9))
    assert oracle.cmux_count() == 20

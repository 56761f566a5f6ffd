"""GPU parity of CMUX Memory (Sec. 8): ROM reads, RAM reads and the RAM write, bit-exact
against the oracle. At the workload's own sizes (512-word ROM, 256 reads; RAM v = 8, w = 8)
every ROM read, sixteen RAM reads with encrypted selectors and 263 write bars (one whole bit
block and every bit at the written address) are compared with the oracle, and every read and
every written cell is decrypted."""
import numpy as np
import pytest

import oracle
import workloads as W
from paper_2010_09410_amd import client
from paper_2010_09410_amd.device import to_host

pytestmark = pytest.mark.gpu
N, n = 1024, 630


def rom_setup(keys, reads):
    s1 = keys["s1"]
    wl = W.rom_workload(reads=reads)
    msg = client.pack_rom(wl["words"])
    ca, ce = wl["cells"]
    rom = client.trlwe_encrypt_torus(s1, msg, ca, ce)                      # [16][2][N]
    abits = (wl["addr"][:, None] >> np.arange(9)[None, :]) & 1
    sa, se = wl["sel"]
    sel = client.trgsw_encrypt(s1, abits, sa, se)                          # [R][9][6][2][N]
    return wl, rom, sel


def test_rom_read_parity_and_full_workload(gpu, keys):
    wl, rom, sel = rom_setup(keys, 256)
    out = to_host(gpu.rom_read(gpu.tensor(rom), gpu.tensor(sel), 9, 32))
    gpu.sync()
    bits = (wl["words"][wl["addr"]][:, None] >> np.arange(32)[None, :]) & 1
    np.testing.assert_array_equal(client.tlwe_decrypt(keys["s0"], out), bits)
    ref = oracle.rom_reads(keys["ksk"], rom, sel)                           # all 256 reads
    bad = np.nonzero((out != ref).any(axis=(1, 2)))[0]
    assert bad.size == 0, f"{bad.size} of 256 ROM reads differ from the oracle, first {bad[:8]}"


def test_rom_read_small_and_single_cell(gpu, keys):
    """A 2-cell ROM (v = 6) and a single-cell ROM (v = 5, no tree), ragged read count."""
    s1 = keys["s1"]
    g = W.rng(600)
    for v in (6, 5):
        P = 1 << (v - 5)
        words = W.uniform_u32(g, (32 * P,))
        a, e = W.trlwe_draws(g, P)
        rom = client.trlwe_encrypt_torus(s1, client.pack_rom(words), a, e)
        addr = g.integers(0, 32 * P, 3)
        sa, se = W.trgsw_draws(g, 3 * v)
        sel = client.trgsw_encrypt(s1, (addr[:, None] >> np.arange(v)[None, :]) & 1,
                                   sa.reshape(3, v, 6, N), se.reshape(3, v, 6, N))
        out = to_host(gpu.rom_read(gpu.tensor(rom), gpu.tensor(sel), v, 32))
        np.testing.assert_array_equal(out, oracle.rom_reads(keys["ksk"], rom, sel))


def test_ram_read_parity(gpu, keys):
    s1 = keys["s1"]
    v, w, R = 4, 3, 5
    g = W.rng(601)
    contents = g.integers(0, 2, (w, 2 ** v))
    a, e = W.trlwe_draws(g, w * 2 ** v)
    ram = client.trlwe_encrypt_torus(s1, client.ram_cell_messages(contents), a.reshape(w, 2 ** v, N),
                                     e.reshape(w, 2 ** v, N))
    addr = g.integers(0, 2 ** v, R)
    sa, se = W.trgsw_draws(g, R * v)
    sel = client.trgsw_encrypt(s1, (addr[:, None] >> np.arange(v)[None, :]) & 1, sa.reshape(R, v, 6, N),
                               se.reshape(R, v, 6, N))
    out = to_host(gpu.ram_read(gpu.tensor(ram), gpu.tensor(sel)))
    np.testing.assert_array_equal(out, oracle.ram_reads(keys["ksk"], ram, sel))
    np.testing.assert_array_equal(client.tlwe_decrypt(keys["s0"], out), contents[:, addr].T)


def test_ram_read_full_size_encrypted_selectors(gpu, keys):
    """v = 8, w = 8 (2,048 cells): sixteen reads at uniform addresses with encrypted selectors,
    bit-exact against the oracle and decrypting to the stored bits."""
    s1 = keys["s1"]
    wl = W.ram_workload(v=8, w=8, reads=16, flag=1)
    ca, ce = wl["cells"]
    ram = client.trlwe_encrypt_torus(s1, client.ram_cell_messages(wl["contents"]), ca, ce)
    sa, se = wl["rsel"]
    sel = client.trgsw_encrypt(s1, (wl["raddr"][:, None] >> np.arange(8)[None, :]) & 1, sa, se)
    out = to_host(gpu.ram_read(gpu.tensor(ram), gpu.tensor(sel)))
    gpu.sync()
    np.testing.assert_array_equal(client.tlwe_decrypt(keys["s0"], out), wl["contents"][:, wl["raddr"]].T)
    np.testing.assert_array_equal(out, oracle.ram_reads(keys["ksk"], ram, sel))


def encrypted_ram(keys, wl):
    s0, s1 = keys["s0"], keys["s1"]
    v, w = wl["v"], wl["w"]
    ca, ce = wl["cells"]
    ram = client.trlwe_encrypt_torus(s1, client.ram_cell_messages(wl["contents"]), ca, ce)
    sa, se = wl["wsel"]
    sel = client.trgsw_encrypt(s1, (wl["waddr"] >> np.arange(v)) & 1, sa, se)
    flag = client.tlwe_encrypt_bits(s0, [wl["flag"]], *wl["fenc"])[0]
    data = client.tlwe_encrypt_bits(s0, wl["wdata"], *wl["denc"])
    return ram, sel, flag, data


@pytest.mark.parametrize("flag", [1, 0])
def test_ram_write_parity_small(gpu, keys, flag):
    wl = W.ram_workload(v=3, w=2, reads=1, flag=flag, seed_off=10 + flag)
    ram, sel, fl, data = encrypted_ram(keys, wl)
    d_ram = gpu.tensor(ram)
    gpu.ram_write(d_ram, gpu.tensor(sel), gpu.tensor(fl), gpu.tensor(data))
    new = to_host(d_ram)
    gpu.sync()
    ref = oracle.ram_write(keys["bk"], keys["ksk"], ram, sel, fl, data)
    np.testing.assert_array_equal(new, ref)


def test_ram_write_then_read_full_workload(gpu, keys):
    """v = 8, w = 8: write under f = 1, then read every address back; 263 write bars (the whole
    block of bit 3 and every bit at the written address) are bit-exact against the oracle given
    the oracle's own read-unit and control-unit outputs."""
    s0, s1 = keys["s0"], keys["s1"]
    wl = W.ram_workload(v=8, w=8, reads=1, flag=1)
    ram, sel, fl, data = encrypted_ram(keys, wl)
    d_ram = gpu.tensor(ram)
    gpu.ram_write(d_ram, gpu.tensor(sel), gpu.tensor(fl), gpu.tensor(data))
    new = to_host(d_ram)
    # read back all 256 addresses with fresh selectors (trivial ones: exact selection)
    rsel = client.trivial_trgsw((np.arange(256)[:, None] >> np.arange(8)[None, :]) & 1)
    out = to_host(gpu.ram_read(gpu.tensor(new), gpu.tensor(rsel)))
    gpu.sync()
    expect = wl["contents"].copy()
    expect[:, wl["waddr"]] = wl["wdata"]
    np.testing.assert_array_equal(client.tlwe_decrypt(s0, out).T, expect)
    # sampled bars against the oracle (read unit and control unit recomputed on the CPU)
    rd = oracle.ram_read(keys["ksk"], ram, sel)
    u = oracle.ram_control(keys["bk"], fl, data, rd)
    idx = np.unique(np.r_[3 * 256 + np.arange(256), np.arange(8) * 256 + wl["waddr"]])
    assert idx.size == 263
    bars = oracle.ram_write_bars(keys["bk"], keys["ksk"], ram, sel, u, idx)
    bad = idx[(new.reshape(-1, 2, N)[idx] != bars).any(axis=(1, 2))]
    assert bad.size == 0, f"{bad.size} of {idx.size} write bars differ from the oracle, first {bad[:8]}"


def test_memory_size_limits_rejected(gpu):
    """Requests beyond the launch limit (R w or w 2^v above 2^22) are refused before any work."""
    from paper_2010_09410_amd import VspError
    from paper_2010_09410_amd import _native as nv
    buf = gpu.empty(16, 2, N)
    ptr = buf.data_ptr()
    with pytest.raises(VspError):
        nv.vsp_rom_read(gpu.handle, ptr, 16, ptr, 9, 32, ptr, 1 << 18, gpu.stream())
    with pytest.raises(VspError):
        nv.vsp_ram_read(gpu.handle, ptr, 8, 1024, ptr, ptr, 1 << 13, gpu.stream())
    with pytest.raises(VspError):
        nv.vsp_ram_write(gpu.handle, ptr, 16, 128, ptr, ptr, ptr, gpu.stream())

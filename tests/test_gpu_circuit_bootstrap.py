"""Circuit bootstrapping on the GPU (TLWE -> TRGSW, Sec. 2.1.2; the CMUX memory's address
conversion, Sec. 8.2) against the oracle, bit for bit, at the full parameter set; and its
output used as the address selectors of a RAM read."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2010_09410_amd import VspError, client
from paper_2010_09410_amd import _native as nv
from paper_2010_09410_amd.device import to_host

pytestmark = pytest.mark.gpu
n, N = 630, 1024


@pytest.fixture(scope="module")
def cb(gpu, keys):
    s2 = W.secret_key2()
    bk2d, pkskd = W.bk2_draws(), W.pksk_draws()
    bk2, pksk = client.keyset2(keys["s0"], keys["s1"], s2, bk2d, pkskd)
    key = gpu.cbkey(bk2, pksk)
    del bk2, pksk
    obk2, opksk = oracle.keyset2(keys["s0"], keys["s1"], s2, bk2d, pkskd)
    del bk2d, pkskd
    yield dict(key=key, bk2=obk2, pksk=opksk)
    key.close()


def test_circuit_bootstrap_matches_oracle(gpu, keys, cb):
    """Five conversions against the oracle in both forms of the level-2 blind rotation (one
    four-wave workgroup per job, and eight waves per job), and in the form picked by size."""
    g = W.rng(700)
    bits = np.array([1, 0, 1, 1, 0])
    cs = client.tlwe_encrypt_bits(keys["s0"], bits, *W.tlwe_draws(g, bits.size))
    cs[4] = client.trivial_tlwe_bits([0])[0]          # a noise-free, mask-free input
    want = oracle.circuit_bootstraps(cb["bk2"], cb["pksk"], cs)
    try:
        for form in (1, 2, 0):
            cb["key"].set_form(form)
            out = to_host(cb["key"].bootstrap(gpu.tensor(cs)))
            gpu.sync()
            for r in range(bits.size):
                np.testing.assert_array_equal(out[r].reshape(6, 2, N), want[r], err_msg=f"form {form}, input {r}")
    finally:
        cb["key"].set_form(0)
    # every row's phase is the gadget TRGSW's phase of the bit, within the noise
    s1 = keys["s1"]
    for r, b in enumerate(bits):
        for row in range(6):
            ph = client.trlwe_phase(s1, out[r].reshape(6, 2, N)[row]).view(np.int32).astype(np.int64)
            g_ = 1 << (32 - 6 * (row % 3 + 1))
            if row < 3:
                exp = (-(s1.astype(np.int64)) * b * g_)
            else:
                exp = np.zeros(N, np.int64)
                exp[0] = b * g_
            dev = ((ph - exp + (1 << 31)) % (1 << 32)) - (1 << 31)
            assert np.abs(dev).max() < 1 << 16, (r, row, int(np.abs(dev).max()))


def test_circuit_bootstrap_forms_agree_on_a_larger_batch(gpu, keys, cb):
    """90 conversions (270 jobs, beyond one eight-wave round, so the default takes the four-wave
    form): every output equals the eight-wave form's, and two sampled conversions equal the
    oracle's."""
    g = W.rng(701)
    R = 90
    bits = g.integers(0, 2, R)
    cs = client.tlwe_encrypt_bits(keys["s0"], bits, *W.tlwe_draws(g, R))
    d = gpu.tensor(cs)
    try:
        cb["key"].set_form(0)
        auto = to_host(cb["key"].bootstrap(d))
        cb["key"].set_form(2)
        wide = to_host(cb["key"].bootstrap(d))
        gpu.sync()
    finally:
        cb["key"].set_form(0)
    np.testing.assert_array_equal(auto, wide)
    pick = [0, R - 1]
    want = oracle.circuit_bootstraps(cb["bk2"], cb["pksk"], cs[pick])
    for k, r in enumerate(pick):
        np.testing.assert_array_equal(auto[r].reshape(6, 2, N), want[k], err_msg=f"input {r}")


def test_circuit_bootstrapped_address_drives_a_ram_read(gpu, keys, cb):
    """A RAM read (v = 8, w = 8) whose address arrives as level-0 TLWE bits: circuit
    bootstrapping gives the selectors, the read returns the stored bits."""
    s0, s1 = keys["s0"], keys["s1"]
    wl = W.ram_workload(v=8, w=8, reads=4, flag=1)
    ca, ce = wl["cells"]
    ram = client.trlwe_encrypt_torus(s1, client.ram_cell_messages(wl["contents"]), ca, ce)
    addr_bits = (wl["raddr"][:, None] >> np.arange(8)[None, :]) & 1             # [4][8]
    tl = client.tlwe_encrypt_bits(s0, addr_bits.reshape(-1), *W.tlwe_draws(W.rng(701), addr_bits.size))
    sel = cb["key"].bootstrap(gpu.tensor(tl)).reshape(4, 8, 6, 2, N)
    out = to_host(gpu.ram_read(gpu.tensor(ram), sel))
    gpu.sync()
    np.testing.assert_array_equal(client.tlwe_decrypt(s0, out), wl["contents"][:, wl["raddr"]].T)


def test_circuit_bootstrap_argument_errors(gpu, cb):
    d = gpu.empty(2, n + 1)
    o = gpu.empty(2, 6, 2, N)
    nv.vsp_circuit_bootstrap(gpu.handle, cb["key"].handle, d.data_ptr(), o.data_ptr(), 0, gpu.stream())
    with pytest.raises(VspError):
        nv.vsp_circuit_bootstrap(gpu.handle, None, d.data_ptr(), o.data_ptr(), 2, gpu.stream())
    host = np.zeros((2, 6, 2, N), np.uint32)
    with pytest.raises(VspError) as ei:                                   # host output
        nv.vsp_circuit_bootstrap(gpu.handle, cb["key"].handle, d.data_ptr(), host.ctypes.data, 2, gpu.stream())
    assert ei.value.status == nv.VSP_E_ARG
    with pytest.raises(VspError) as ei:                                   # output overlaps the input
        nv.vsp_circuit_bootstrap(gpu.handle, cb["key"].handle, o.data_ptr(), o.data_ptr(), 2, gpu.stream())
    assert ei.value.status == nv.VSP_E_ARG
    for bad in (-1, 3):
        with pytest.raises(VspError) as ei:                               # unknown level-2 form
            cb["key"].set_form(bad)
        assert ei.value.status == nv.VSP_E_ARG


def counter_machine_netlist():
    """A clocked netlist with a RAM port (v = 4, w = 4): address register A (flip-flops 0-3)
    counts up each cycle; the read port loads register D (flip-flops 4-7) with RAM[A]; the
    write data is D XOR A under the external write-flag input. Wires: 0 the flag, 1-4 A,
    5-8 D, then the gates."""
    NOT, XOR, AND = 8, 4, 1
    A, D = [1, 2, 3, 4], [5, 6, 7, 8]
    gates = []
    def gate(op, a, b):
        gates.append((op, a, b))
        return 9 + len(gates) - 1
    s0 = gate(NOT, A[0], A[0])
    c = A[0]
    nxt = [s0]
    for b in range(1, 4):
        nxt.append(gate(XOR, A[b], c))
        if b < 3:
            c = gate(AND, A[b], c)
    wd = [gate(XOR, D[b], A[b]) for b in range(4)]
    next_state = nxt + D            # the D entries are taken over by the read port
    return np.array(gates, np.int64), next_state, A, wd


def test_clocked_netlist_with_ram_in_the_loop(gpu, keys, cb):
    """Cycles of a netlist whose RAM is read and written every clock from TLWE wires (circuit
    bootstrapping of the address): the state and the RAM follow the plaintext model for four
    cycles; the first cycle's read and write are bit-exact against the oracle fed the same
    ciphertexts; and a fresh machine resumed from the host snapshot taken after the first cycle
    (flip-flops and RAM, the paper's snapshot for resumption) runs the other three cycles to the
    same bits."""
    s0, s1 = keys["s0"], keys["s1"]
    gates, next_state, A_w, wd_w = counter_machine_netlist()
    g = W.rng(702)
    contents = g.integers(0, 2, (4, 16))
    a0, d0 = 13, int(g.integers(0, 16))
    flags = [1, 0, 1, 1]
    state_bits = [(a0 >> b) & 1 for b in range(4)] + [(d0 >> b) & 1 for b in range(4)]
    state = client.tlwe_encrypt_bits(s0, state_bits, *W.tlwe_draws(g, 8))
    ca, ce = W.trlwe_draws(g, 64)
    ram0 = client.trlwe_encrypt_torus(s1, client.ram_cell_messages(contents), ca.reshape(4, 16, N), ce.reshape(4, 16, N))
    fin = client.tlwe_encrypt_bits(s0, flags, *W.tlwe_draws(g, 4)).reshape(4, 1, n + 1)
    m = gpu.machine(gates, 1, next_state)
    d_ram = gpu.tensor(ram0)
    m.attach_ram(cb["key"], d_ram, A_w, 0, wd_w, [4, 5, 6, 7])
    d_state = gpu.tensor(state)
    # cycle 1, then the oracle on the same ciphertexts: selectors from circuit bootstrapping
    # of the address flip-flops, the read into D, the write of D xor A under the flag
    m.run(d_state, 1, gpu.tensor(fin[:1]))
    st1 = to_host(d_state)
    ram1 = to_host(d_ram)
    gpu.sync()
    sel = oracle.circuit_bootstraps(cb["bk2"], cb["pksk"], state[:4])
    np.testing.assert_array_equal(st1[4:8], oracle.ram_read(keys["ksk"], ram0, sel))
    wdata = np.stack([oracle.gate(keys["bk"], keys["ksk"], 4, state[4 + b], state[b]) for b in range(4)])
    np.testing.assert_array_equal(ram1, oracle.ram_write(keys["bk"], keys["ksk"], ram0, sel, fin[0, 0], wdata))
    # three more cycles against the plaintext model
    m.run(d_state, 3, gpu.tensor(fin[1:]))
    st_full = to_host(d_state)
    st = client.tlwe_decrypt(s0, st_full)
    ram = to_host(d_ram)
    gpu.sync()
    # resumption: a new machine from the snapshot after cycle 1
    m2 = gpu.machine(gates, 1, next_state)
    d_ram2 = gpu.tensor(ram1)
    m2.attach_ram(cb["key"], d_ram2, A_w, 0, wd_w, [4, 5, 6, 7])
    d_state2 = gpu.tensor(st1)
    m2.run(d_state2, 3, gpu.tensor(fin[1:]))
    np.testing.assert_array_equal(to_host(d_state2), st_full)
    np.testing.assert_array_equal(to_host(d_ram2), ram)
    gpu.sync()
    m2.close()
    mem = contents.copy()
    A, Dv = a0, d0
    for f in flags:
        rd = mem[:, A].copy()
        if f:
            mem[:, A] = [((Dv >> b) & 1) ^ ((A >> b) & 1) for b in range(4)]
        A, Dv = (A + 1) % 16, int(sum(int(rd[b]) << b for b in range(4)))
    assert [int(x) for x in st] == [(A >> b) & 1 for b in range(4)] + [(Dv >> b) & 1 for b in range(4)]
    got = (client.trlwe_phase(s1, ram)[..., 0].view(np.int32) >= 0).astype(int)
    np.testing.assert_array_equal(got, mem)
    m.close()

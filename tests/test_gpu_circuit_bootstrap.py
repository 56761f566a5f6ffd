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
    g = W.rng(700)
    bits = np.array([1, 0, 1, 1, 0])
    cs = client.tlwe_encrypt_bits(keys["s0"], bits, *W.tlwe_draws(g, bits.size))
    cs[4] = client.trivial_tlwe_bits([0])[0]          # a noise-free, mask-free input
    out = to_host(cb["key"].bootstrap(gpu.tensor(cs)))
    gpu.sync()
    want = oracle.circuit_bootstraps(cb["bk2"], cb["pksk"], cs)
    for r in range(bits.size):
        np.testing.assert_array_equal(out[r].reshape(6, 2, N), want[r], err_msg=f"input {r}")
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

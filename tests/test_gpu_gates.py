"""GPU parity of the NTT product, the external product and the homomorphic gates against the
oracle: bit-exact ciphertexts (integer arithmetic; the tolerance is zero)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2010_09410_amd import VSP_BATCHED, VSP_PER_GATE, VspError, client
from paper_2010_09410_amd.device import to_host

pytestmark = pytest.mark.gpu
N, n = 1024, 630
MU = 1 << 29


def dev(ctx, a):
    return ctx.tensor(a)


def test_ntt_polymul_matches_schoolbook(gpu):
    g = W.rng(500)
    J = 9  # spans several workgroups and a ragged tail
    a = g.integers(-32, 32, (J, N)).astype(np.int32)
    b = W.uniform_u32(g, (J, N))
    # edge cases: zero, one-hot, extreme digits, all-ones torus values
    a[0] = 0
    a[1] = 0; a[1, 5] = 1
    a[2] = -32; b[2] = 0xFFFFFFFF
    a[3] = 31; b[3] = 0x80000000
    a[4] = 0; a[4, N - 1] = -1
    a[5] = g.integers(-(1 << 20), (1 << 20) + 1, N)
    out = to_host(gpu.debug_polymul(dev(gpu, a), dev(gpu, b)))
    torch.cuda.synchronize()
    for j in range(J):
        np.testing.assert_array_equal(out[j], oracle.polymul(a[j].astype(np.int64).astype(np.uint32), b[j]), err_msg=f"j={j}")


def test_external_product_matches_oracle(gpu, keys):
    s1 = keys["s1"]
    g = W.rng(501)
    J = 6
    ma, me = W.trgsw_draws(g, J)
    C = np.stack([client.trgsw_encrypt(s1, j & 1, ma[j], me[j]) for j in range(J)])
    C[4] = client.trivial_trgsw(1)
    C[5] = 0
    x = W.uniform_u32(g, (J, 2, N))
    x[3] = 0xFFFFFFFF
    out = to_host(gpu.debug_external_product(dev(gpu, C), dev(gpu, x)))
    for j in range(J):
        np.testing.assert_array_equal(out[j], oracle.external_product(C[j], x[j]), err_msg=f"j={j}")


def encrypt_pair(keys, cfg):
    s0 = keys["s0"]
    in0 = client.tlwe_encrypt_bits(s0, cfg["bits0"], *cfg["enc0"])
    in1 = client.tlwe_encrypt_bits(s0, cfg["bits1"], *cfg["enc1"])
    return in0, in1


def test_config1_eight_nand_bit_exact(gpu, keys):
    cfg = W.config1()
    in0, in1 = encrypt_pair(keys, cfg)
    out = to_host(gpu.gates(dev(gpu, cfg["ops"]), dev(gpu, in0), dev(gpu, in1)))
    ref = oracle.gates(keys["bk"], keys["ksk"], cfg["ops"], in0, in1)
    np.testing.assert_array_equal(out, ref)
    np.testing.assert_array_equal(client.tlwe_decrypt(keys["s0"], out), 1 - (cfg["bits0"] & cfg["bits1"]))


ALL_OPS = [oracle.NAND, oracle.AND, oracle.OR, oracle.NOR, oracle.XOR, oracle.XNOR, oracle.ANDNOT, oracle.ORNOT,
           oracle.NOT]
TRUTH = {0: lambda a, b: 1 - (a & b), 1: lambda a, b: a & b, 2: lambda a, b: a | b, 3: lambda a, b: 1 - (a | b),
         4: lambda a, b: a ^ b, 5: lambda a, b: 1 - (a ^ b), 6: lambda a, b: a & (1 - b), 7: lambda a, b: a | (1 - b),
         8: lambda a, b: 1 - a}


def truth_table_inputs(keys, seed):
    g = W.rng(seed)
    ops, A, Bb = [], [], []
    for op in ALL_OPS:
        for a in (0, 1):
            for b in (0, 1):
                ops.append(op); A.append(a); Bb.append(b)
    ops, A, Bb = np.array(ops, np.uint8), np.array(A), np.array(Bb)
    in0 = client.tlwe_encrypt_bits(keys["s0"], A, *W.tlwe_draws(g, ops.size))
    in1 = client.tlwe_encrypt_bits(keys["s0"], Bb, *W.tlwe_draws(g, ops.size))
    return ops, A, Bb, in0, in1


def test_every_gate_truth_table_bit_exact(gpu, keys):
    ops, A, Bb, in0, in1 = truth_table_inputs(keys, 502)
    out = to_host(gpu.gates(dev(gpu, ops), dev(gpu, in0), dev(gpu, in1)))
    ref = oracle.gates(keys["bk"], keys["ksk"], ops, in0, in1)
    np.testing.assert_array_equal(out, ref)
    want = np.array([TRUTH[o](a, b) for o, a, b in zip(ops, A, Bb)])
    np.testing.assert_array_equal(client.tlwe_decrypt(keys["s0"], out), want)


def test_per_gate_mode_equals_batched(gpu, keys):
    ops, A, Bb, in0, in1 = truth_table_inputs(keys, 503)
    ops, in0, in1 = ops[:13], in0[:13], in1[:13]   # ragged: not a multiple of the workgroup
    o_b = to_host(gpu.gates(dev(gpu, ops), dev(gpu, in0), dev(gpu, in1), mode=VSP_BATCHED))
    o_p = to_host(gpu.gates(dev(gpu, ops), dev(gpu, in0), dev(gpu, in1), mode=VSP_PER_GATE))
    np.testing.assert_array_equal(o_b, o_p)
    np.testing.assert_array_equal(o_b, oracle.gates(keys["bk"], keys["ksk"], ops, in0, in1))


def test_key_copies_equal_oracle(gpu, keys):
    """Gates whose gate g reads its own device copy g mod c of the bootstrapping key (a batch
    without key reuse): the same bits as the oracle in every NTT form and for several copy
    counts (one per gate, fewer, one), with NOT gates and a ragged batch; bad forms and copy
    counts are refused."""
    from paper_2010_09410_amd import _native as nv
    ops, A, Bb, in0, in1 = truth_table_inputs(keys, 505)
    ref = oracle.gates(keys["bk"], keys["ksk"], ops, in0, in1)
    d = [dev(gpu, x) for x in (ops, in0, in1)]
    for waves, copies in ((8, 1), (8, ops.size), (4, 5), (3, ops.size), (8, 7)):
        out, ms = gpu.gates_key_copies(*d, waves=waves, copies=copies)
        assert ms > 0
        np.testing.assert_array_equal(to_host(out), ref, err_msg=f"waves={waves} copies={copies}")
    for waves, copies in ((32, 1), (8, 0), (8, 65537)):
        with pytest.raises(VspError) as ei:
            gpu.gates_key_copies(*d, waves=waves, copies=copies)
        assert ei.value.status == nv.VSP_E_ARG


def test_trivial_inputs_exact_closed_form(gpu):
    ops, A, Bb = [], [], []
    for op in ALL_OPS[:8]:
        for a in (0, 1):
            for b in (0, 1):
                ops.append(op); A.append(a); Bb.append(b)
    ops = np.array(ops, np.uint8)
    out = to_host(gpu.gates(dev(gpu, ops), dev(gpu, client.trivial_tlwe_bits(A)), dev(gpu, client.trivial_tlwe_bits(Bb))))
    want = np.array([TRUTH[o](a, b) for o, a, b in zip(ops, A, Bb)])
    np.testing.assert_array_equal(out, client.trivial_tlwe_bits(want))


def test_bootstrap_trlwe_matches_oracle(gpu, keys):
    ops, A, Bb, in0, in1 = truth_table_inputs(keys, 504)
    sel = ops != oracle.NOT
    ops, in0, in1 = ops[sel][::3], in0[sel][::3], in1[sel][::3]
    out = to_host(gpu.bootstrap_trlwe(dev(gpu, ops), dev(gpu, in0), dev(gpu, in1)))
    for k in range(ops.size):
        lin, _ = oracle.gate_linear(int(ops[k]), in0[k], in1[k])
        np.testing.assert_array_equal(out[k], oracle.bootstrap_to_trlwe(keys["bk"], lin), err_msg=f"k={k}")


@pytest.mark.parametrize("groups", [6, 24])
def test_tiny_split_batches_with_idle_gates(gpu, keys, groups):
    """Batches of at most four gates in the split matrix-core form (digits formed inside the
    step kernel, the accumulator rotating through three buffers), with a gate that does not
    bootstrap among them: gate outputs and TRLWE accumulators equal the oracle."""
    ops, A, Bb, in0, in1 = truth_table_inputs(keys, 506)
    pick = [32, 1, 0]                      # NOT, NAND, NAND: the first gate does not bootstrap
    ops3, a3, b3 = ops[pick], in0[pick], in1[pick]
    assert ops3[0] == oracle.NOT
    saved = {B: gpu.tuning(B) for B in (3, 4)}
    prev = gpu.set_split_groups(3, groups)
    try:
        for B in (3, 4):
            gpu.set_tuning(B, 33, 2)
        out = to_host(gpu.gates(dev(gpu, ops3), dev(gpu, a3), dev(gpu, b3)))
        np.testing.assert_array_equal(out, oracle.gates(keys["bk"], keys["ksk"], ops3, a3, b3))
        t_ops, t0, t1 = ops[[1, 5, 9, 13]], in0[[1, 5, 9, 13]], in1[[1, 5, 9, 13]]
        tr = to_host(gpu.bootstrap_trlwe(dev(gpu, t_ops), dev(gpu, t0), dev(gpu, t1)))
        for k in range(4):
            lin, _ = oracle.gate_linear(int(t_ops[k]), t0[k], t1[k])
            np.testing.assert_array_equal(tr[k], oracle.bootstrap_to_trlwe(keys["bk"], lin), err_msg=f"k={k}")
        gpu.sync()
    finally:
        for B, (w, t) in saved.items():
            gpu.set_tuning(B, 0, t)
        gpu.set_split_groups(3, prev)


def test_empty_batch_is_noop(gpu):
    t = gpu.empty(1, n + 1)
    ops = torch.zeros(1, dtype=torch.uint8, device=gpu.device)
    from paper_2010_09410_amd import _native as nv
    nv.vsp_gates(gpu.handle, ops.data_ptr(), t.data_ptr(), t.data_ptr(), t.data_ptr(), 0, VSP_BATCHED, gpu.stream())


def test_argument_errors(gpu):
    from paper_2010_09410_amd import _native as nv
    ops = torch.zeros(4, dtype=torch.uint8, device=gpu.device)
    a = gpu.empty(4, n + 1)
    b = gpu.empty(4, n + 1)
    small = gpu.empty(2, n + 1)
    host = np.zeros((4, n + 1), np.uint32)
    cases = [
        (0, a.data_ptr(), b.data_ptr(), small.data_ptr()),          # null ops
        (ops.data_ptr(), host.ctypes.data, b.data_ptr(), small.data_ptr()),  # host pointer
        (ops.data_ptr(), a.data_ptr(), b.data_ptr(), a.data_ptr()),  # output aliases input
        (ops.data_ptr(), a.data_ptr() + 2, b.data_ptr(), small.data_ptr()),  # misaligned
    ]
    for (o, x, y, z) in cases:
        with pytest.raises(VspError) as ei:
            nv.vsp_gates(gpu.handle, o, x, y, z, 4, VSP_BATCHED, gpu.stream())
        assert ei.value.status == nv.VSP_E_ARG
    with pytest.raises(VspError):
        nv.vsp_gates(gpu.handle, ops.data_ptr(), a.data_ptr(), b.data_ptr(), gpu.empty(4, n + 1).data_ptr(), 4, 7,
                     gpu.stream())
    with pytest.raises(VspError) as ei:
        nv.vsp_context_create(np.zeros(1, np.uint32), np.zeros(1, np.uint32), 0, params=(500, 1024, 1, 3, 6, 8, 2))
    assert ei.value.status == nv.VSP_E_PARAMS


def test_invalid_opcode_zeroes_output_and_is_reported(gpu, keys):
    from paper_2010_09410_amd import _native as nv
    ops = np.array([oracle.NAND, 200, oracle.AND], np.uint8)
    in0 = client.trivial_tlwe_bits([1, 1, 1])
    in1 = client.trivial_tlwe_bits([1, 0, 1])
    out = gpu.gates(dev(gpu, ops), dev(gpu, in0), dev(gpu, in1))
    with pytest.raises(VspError) as ei:
        gpu.sync()
    assert ei.value.status == nv.VSP_E_ARG
    o = to_host(out)
    assert (o[1] == 0).all()
    np.testing.assert_array_equal(o[[0, 2]], client.trivial_tlwe_bits([0, 1]))
    gpu.sync()  # flag cleared


def test_config2_sampled_parity_and_full_decryption(gpu, keys):
    """The 4096-gate batch (the benchmark workload): all outputs decrypt to the plaintext gate
    results, and a sample is bit-exact against the oracle."""
    cfg = W.config2()
    in0, in1 = encrypt_pair(keys, cfg)
    out = to_host(gpu.gates(dev(gpu, cfg["ops"]), dev(gpu, in0), dev(gpu, in1)))
    want = np.array([TRUTH[o](a, b) for o, a, b in zip(cfg["ops"], cfg["bits0"], cfg["bits1"])])
    np.testing.assert_array_equal(client.tlwe_decrypt(keys["s0"], out), want)
    idx = np.array([0, 1, 2, 1023, 2048, 3071, 4094, 4095] + list(W.rng(505).integers(0, 4096, 8)))
    ref = oracle.gates(keys["bk"], keys["ksk"], cfg["ops"][idx], in0[idx], in1[idx])
    np.testing.assert_array_equal(out[idx], ref)


MUX_ROWS = [(s, a, b) for s in (0, 1) for a in (0, 1) for b in (0, 1)]


def test_mux_matches_oracle_and_truth_table(gpu, keys):
    """HomMUX s ? c1 : c0 over the full truth table twice plus a ragged random batch: bit-exact
    against the oracle, and every row decrypts to the selected bit."""
    s0 = keys["s0"]
    g = W.rng(510)
    rows = MUX_ROWS * 2 + [tuple(g.integers(0, 2, 3)) for _ in range(21)]   # 37 rows
    enc = lambda bits: client.tlwe_encrypt_bits(s0, np.array(bits), *W.tlwe_draws(g, len(bits)))
    S, A, Bb = enc([r[0] for r in rows]), enc([r[1] for r in rows]), enc([r[2] for r in rows])
    out = to_host(gpu.mux(dev(gpu, S), dev(gpu, A), dev(gpu, Bb)))
    gpu.sync()
    want = np.array([a if s else b for s, a, b in rows])
    np.testing.assert_array_equal(client.tlwe_decrypt(s0, out), want)
    np.testing.assert_array_equal(out, oracle.muxes(keys["bk"], keys["ksk"], S, A, Bb))
    # trivial inputs give exactly (0, +-1/8)
    T = lambda bits: client.trivial_tlwe_bits(np.array(bits))
    tout = to_host(gpu.mux(dev(gpu, T([r[0] for r in MUX_ROWS])), dev(gpu, T([r[1] for r in MUX_ROWS])),
                           dev(gpu, T([r[2] for r in MUX_ROWS]))))
    np.testing.assert_array_equal(tout, T([a if s else b for s, a, b in MUX_ROWS]))


def test_mux_rejects_overlap_and_accepts_empty(gpu):
    x = gpu.empty(4, n + 1)
    y = gpu.empty(4, n + 1)
    with pytest.raises(VspError):
        gpu.mux(x, y, y, out=x)
    gpu.mux(x[:0], y[:0], y[:0], out=gpu.empty(0, n + 1))

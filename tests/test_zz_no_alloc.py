"""The allocation-free gate entry point (vsp_gates_noalloc, fixed device scratch) against
vsp_gates, through the C ABI: two calls in a row, the second smaller, bit for bit."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2010_09410_amd import VSP_BATCHED, VSP_PER_GATE, VspError, client
from paper_2010_09410_amd import _native as nv
from paper_2010_09410_amd.device import to_host

pytestmark = pytest.mark.gpu
n = 630


def batch(keys, seed, B):
    g = W.rng(seed)
    ops = g.integers(0, 9, B).astype(np.uint8)          # every opcode, NOT included
    bits0, bits1 = g.integers(0, 2, B), g.integers(0, 2, B)
    in0 = client.tlwe_encrypt_bits(keys["s0"], bits0, *W.tlwe_draws(g, B))
    in1 = client.tlwe_encrypt_bits(keys["s0"], bits1, *W.tlwe_draws(g, B))
    return ops, in0, in1


def run(ctx, fn, ops, in0, in1, mode=VSP_BATCHED):
    B = len(ops)
    d_ops, d0, d1 = ctx.tensor(ops), ctx.tensor(in0), ctx.tensor(in1)
    out = ctx.empty(B, n + 1)
    fn(ctx.handle, d_ops.data_ptr(), d0.data_ptr(), d1.data_ptr(), out.data_ptr(), B, mode, ctx.stream())
    torch.cuda.synchronize()
    return to_host(out)


def test_noalloc_equals_gates_on_consecutive_calls(gpu, keys):
    for seed, B in ((900, 1500), (901, 37)):           # the second call smaller than the first
        ops, in0, in1 = batch(keys, seed, B)
        want = run(gpu, nv.vsp_gates, ops, in0, in1)
        got = run(gpu, nv.vsp_gates_noalloc, ops, in0, in1)
        np.testing.assert_array_equal(got, want, err_msg=f"B={B}")
    gpu.sync()


def test_noalloc_largest_batch_per_gate_mode_and_matrix_tuning(gpu, keys):
    ops, in0, in1 = batch(keys, 902, 2048)
    want = run(gpu, nv.vsp_gates, ops, in0, in1)
    # a tuning that picks the matrix-core form for this size runs the NTT form here: same bits
    br, ks = gpu.tuning(2048)
    gpu.set_tuning(2048, 32, ks)
    try:
        got = run(gpu, nv.vsp_gates_noalloc, ops, in0, in1)
    finally:
        gpu.set_tuning(2048, 0, ks)
    np.testing.assert_array_equal(got, want)
    got3 = run(gpu, nv.vsp_gates_noalloc, ops[:3], in0[:3], in1[:3], mode=VSP_PER_GATE)
    np.testing.assert_array_equal(got3, want[:3])
    gpu.sync()


def test_noalloc_rejects_oversized_batch(gpu):
    B = 2049
    d_ops = gpu.tensor(np.zeros(B, np.uint8))
    d0 = gpu.empty(B, n + 1)
    d1 = gpu.empty(B, n + 1)
    out = gpu.empty(B, n + 1)
    with pytest.raises(VspError, match="at most 2048"):
        nv.vsp_gates_noalloc(gpu.handle, d_ops.data_ptr(), d0.data_ptr(), d1.data_ptr(), out.data_ptr(), B,
                             VSP_BATCHED, gpu.stream())
    nv.vsp_gates_noalloc(gpu.handle, d_ops.data_ptr(), d0.data_ptr(), d1.data_ptr(), out.data_ptr(), 0,
                         VSP_BATCHED, gpu.stream())

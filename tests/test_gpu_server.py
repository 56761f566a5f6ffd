"""The continuous-batching server: results are bit-identical alone and in the mix (and equal
to the circuit executor's), admission respects the memory budget, oversize requests are
refused, and malformed circuits are rejected at submission."""
import time

import numpy as np
import pytest

import workloads as W
from paper_2010_09410_amd import VspError, client
from paper_2010_09410_amd import _native as nv
from paper_2010_09410_amd.device import to_host

pytestmark = pytest.mark.gpu
ROWB = 631 * 4


def wait(srv, ticket, nwires, timeout=120.0):
    t0 = time.time()
    while time.time() - t0 < timeout:
        done, wires, lat = srv.poll(ticket, nwires)
        if done:
            return wires, lat
        time.sleep(0.005)
    raise TimeoutError(f"ticket {ticket} not done after {timeout} s")


def requests(keys, count, seed):
    out = []
    for k in range(count):
        c = W.small_circuit(seed=seed + k, levels=2 + k % 4, wmin=2, wmax=12 + 6 * k, ninputs=8 + k)
        inputs = client.tlwe_encrypt_bits(keys["s0"], c["bits"], *c["enc"])
        out.append((c, inputs))
    return out


def test_alone_equals_mixed_equals_circuit(gpu, keys):
    reqs = requests(keys, 6, 800)
    # alone: one request at a time on a fresh server
    alone = []
    srv = gpu.server(mem_budget_bytes=64 << 20, max_batch=256)
    for c, inputs in reqs:
        t = srv.submit(c["gates"], c["ninputs"], inputs)
        alone.append(wait(srv, t, c["ninputs"] + len(c["gates"]))[0])
    srv.close()
    # mixed: all at once, small batches so that requests share batches and levels interleave
    srv = gpu.server(mem_budget_bytes=64 << 20, max_batch=40)
    tickets = [srv.submit(c["gates"], c["ninputs"], inputs) for c, inputs in reqs]
    mixed = [wait(srv, t, c["ninputs"] + len(c["gates"]))[0] for t, (c, _) in zip(tickets, reqs)]
    gates, batches, peak = srv.stats()
    srv.close()
    assert gates == sum(len(c["gates"]) for c, _ in reqs)
    assert batches < sum(int(c["level"].max()) + 1 for c, _ in reqs)   # batches were shared
    for (c, inputs), a, m in zip(reqs, alone, mixed):
        np.testing.assert_array_equal(a, m)
        circ = gpu.circuit(c["gates"], c["ninputs"])
        ref = to_host(circ.run(gpu.tensor(inputs)))
        gpu.sync()
        circ.close()
        np.testing.assert_array_equal(m, ref)


def test_admission_by_memory_budget(gpu, keys):
    reqs = requests(keys, 4, 900)
    biggest = max(c["ninputs"] + len(c["gates"]) for c, _ in reqs)
    budget = int(1.5 * biggest) * ROWB            # at most one or two requests resident at once
    srv = gpu.server(mem_budget_bytes=budget, max_batch=512)
    tickets = [srv.submit(c["gates"], c["ninputs"], inputs) for c, inputs in reqs]
    outs = [wait(srv, t, c["ninputs"] + len(c["gates"]))[0] for t, (c, _) in zip(tickets, reqs)]
    _, _, peak = srv.stats()
    assert peak <= budget
    for (c, _), o in zip(reqs, outs):
        dec = client.tlwe_decrypt(keys["s0"], o)
        assert dec.shape[0] == c["ninputs"] + len(c["gates"])
    srv.close()


def test_capacity_and_malformed_rejected(gpu, keys):
    c = W.small_circuit(seed=950, levels=3, wmin=4, wmax=8, ninputs=8)
    inputs = client.tlwe_encrypt_bits(keys["s0"], c["bits"], *c["enc"])
    srv = gpu.server(mem_budget_bytes=4 * ROWB, max_batch=16)
    with pytest.raises(VspError) as ei:
        srv.submit(c["gates"], c["ninputs"], inputs)
    assert ei.value.status == nv.VSP_E_CAPACITY
    with pytest.raises(VspError) as ei:
        srv.submit(np.array([[0, 0, 3]]), 2, inputs[:2])
    assert ei.value.status == nv.VSP_E_ARG
    with pytest.raises(VspError) as ei:
        srv.poll(12345)
    assert ei.value.status == nv.VSP_E_STATE
    srv.close()


def test_per_client_key_sets(gpu, keys):
    """Two clients with their own key sets (each client generates and ships its own keys,
    Sec. 4.1) served together, so that batches hold gates of both key sets: client B's results
    equal the oracle evaluated with B's keys and decrypt under B's secret key, and client A's
    equal the circuit executor."""
    import oracle
    from test_gpu_circuit import oracle_eval, plaintext_eval
    s0b, s1b = W.secret_keys(5)
    bkd, kskd = W.bk_draws(6), W.ksk_draws(7)
    kb = gpu.keyset(*client.keyset(s0b, s1b, bkd, kskd))
    reqs_a = requests(keys, 3, 1000)
    reqs_b = []
    for k in range(3):
        c = W.small_circuit(seed=1100 + k, levels=2 + k, wmin=2, wmax=10, ninputs=6 + k)
        reqs_b.append((c, client.tlwe_encrypt_bits(s0b, c["bits"], *c["enc"])))
    srv = gpu.server(mem_budget_bytes=64 << 20, max_batch=64)
    ta = [srv.submit(c["gates"], c["ninputs"], x) for c, x in reqs_a]
    tb = [srv.submit(c["gates"], c["ninputs"], x, keyset=kb) for c, x in reqs_b]
    outs_a = [wait(srv, t, c["ninputs"] + len(c["gates"]))[0] for t, (c, _) in zip(ta, reqs_a)]
    outs_b = [wait(srv, t, c["ninputs"] + len(c["gates"]))[0] for t, (c, _) in zip(tb, reqs_b)]
    _, batches, _ = srv.stats()
    srv.close()
    assert batches < sum(int(c["level"].max()) + 1 for c, _ in reqs_a + reqs_b)   # batches mixed clients
    for (c, x), o in zip(reqs_b, outs_b):
        np.testing.assert_array_equal(client.tlwe_decrypt(s0b, o), plaintext_eval(c["gates"], c["bits"]))
    bk_b, ksk_b = oracle.keyset(s0b, s1b, bkd, kskd)
    c, x = reqs_b[0]
    ref = oracle_eval({"bk": bk_b, "ksk": ksk_b}, c["gates"], c["level"], x)
    np.testing.assert_array_equal(outs_b[0], ref)
    for (c, x), o in zip(reqs_a, outs_a):
        circ = gpu.circuit(c["gates"], c["ninputs"])
        np.testing.assert_array_equal(o, to_host(circ.run(gpu.tensor(x))))
        gpu.sync()
        circ.close()
    kb.close()


TRUTH = {0: lambda a, b: 1 - (a & b), 1: lambda a, b: a & b, 2: lambda a, b: a | b, 3: lambda a, b: 1 - (a | b),
         4: lambda a, b: a ^ b, 5: lambda a, b: 1 - (a ^ b), 6: lambda a, b: a & (1 - b), 7: lambda a, b: a | (1 - b),
         8: lambda a, b: 1 - a}


def test_served_trace_decrypts_and_matches_oracle(gpu, keys):
    """The first 24 circuits of the serving workload (64 clients, log-uniform sizes in
    [100, 20000], Poisson arrivals at 50/s), all submitted at once so that their ready gates
    share batches: every wire of every circuit decrypts to the plaintext evaluation, and two
    random gates per circuit are bit-exact against the oracle fed the served input wires."""
    import oracle
    trace = W.serving_trace(rate=50.0, duration=10.0)[:24]
    assert len(trace) == 24
    enc = [client.tlwe_encrypt_bits(keys["s0"], r["bits"], *W.tlwe_draws(W.rng(r["enc_seed"]), r["ninputs"]))
           for r in trace]
    srv = gpu.server(mem_budget_bytes=2 << 30, max_batch=4096)
    tickets = [srv.submit(r["gates"], r["ninputs"], e) for r, e in zip(trace, enc)]
    served = [wait(srv, t, r["ninputs"] + len(r["gates"]), timeout=300.0)[0] for t, r in zip(tickets, trace)]
    gates, batches, _ = srv.stats()
    srv.close()
    assert gates == sum(len(r["gates"]) for r in trace)
    assert batches < sum(int(r["level"].max()) + 1 for r in trace)     # circuits shared batches
    g = W.rng(870)
    ops, a, b, got = [], [], [], []
    for r, wires in zip(trace, served):
        plain = [int(x) for x in r["bits"]]
        for op, i0, i1 in r["gates"]:
            plain.append(TRUTH[int(op)](plain[i0], plain[i1]))
        np.testing.assert_array_equal(client.tlwe_decrypt(keys["s0"], wires), np.array(plain, dtype=np.uint8))
        for k in g.choice(len(r["gates"]), 2, replace=False):
            op, i0, i1 = r["gates"][k]
            ops.append(op)
            a.append(wires[i0])
            b.append(wires[i1])
            got.append(wires[r["ninputs"] + k])
    ref = oracle.gates(keys["bk"], keys["ksk"], np.array(ops, np.uint8), np.array(a), np.array(b))
    np.testing.assert_array_equal(np.array(got), ref)


def test_mixed_key_set_batches_on_the_matrix_cores(gpu, keys):
    """Two clients with different key sets, each with a wide three-level circuit, served with
    the matrix-core forms forced for large batches: batches hold both key sets (each key set's
    range padded to whole 32-gate tiles, every tile naming its key), and every output of client
    B equals the oracle under B's keys gate by gate (fed the served input wires), while client
    A's equal the circuit executor."""
    import oracle
    from test_gpu_circuit import plaintext_eval
    s0b, s1b = W.secret_keys(8)
    bkd, kskd = W.bk_draws(9), W.ksk_draws(10)
    kb = gpu.keyset(*client.keyset(s0b, s1b, bkd, kskd))
    ca = W.small_circuit(seed=1200, levels=3, wmin=1100, wmax=1300, ninputs=64)
    cb = W.small_circuit(seed=1201, levels=3, wmin=1100, wmax=1300, ninputs=64)
    xa = client.tlwe_encrypt_bits(keys["s0"], ca["bits"], *ca["enc"])
    xb = client.tlwe_encrypt_bits(s0b, cb["bits"], *cb["enc"])
    saved = {B: gpu.tuning(B) for B in (1024, 2048, 4096)}
    try:
        for B in (1024, 2048, 4096):
            gpu.set_tuning(B, 33, 3)
        srv = gpu.server(mem_budget_bytes=256 << 20, max_batch=4096)
        ta = srv.submit(ca["gates"], ca["ninputs"], xa)
        tb = srv.submit(cb["gates"], cb["ninputs"], xb, keyset=kb)
        oa, _ = wait(srv, ta, ca["ninputs"] + len(ca["gates"]))
        ob, _ = wait(srv, tb, cb["ninputs"] + len(cb["gates"]))
        gates_launched, batches, _ = srv.stats()
        srv.close()
    finally:
        for B, (w, t) in saved.items():
            gpu.set_tuning(B, 0, t)
    assert batches < 6                                     # levels of both clients shared batches
    np.testing.assert_array_equal(client.tlwe_decrypt(s0b, ob), plaintext_eval(cb["gates"], cb["bits"]))
    np.testing.assert_array_equal(client.tlwe_decrypt(keys["s0"], oa), plaintext_eval(ca["gates"], ca["bits"]))
    bk_b, ksk_b = oracle.keyset(s0b, s1b, bkd, kskd)
    g = cb["gates"]
    idx = np.unique(np.r_[0, len(g) - 1, W.rng(1202).choice(len(g), 30, replace=False)])
    ref = oracle.gates(bk_b, ksk_b, g[idx, 0].astype(np.uint8), ob[g[idx, 1]], ob[g[idx, 2]])
    np.testing.assert_array_equal(ob[cb["ninputs"] + idx], ref)
    circ = gpu.circuit(ca["gates"], ca["ninputs"])
    np.testing.assert_array_equal(oa, to_host(circ.run(gpu.tensor(xa))))
    gpu.sync()
    circ.close()
    kb.close()

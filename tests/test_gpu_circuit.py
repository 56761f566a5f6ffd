"""Levelled circuits on the GPU: full bit-exact parity on a small layered DAG, graph replay ==
eager launches, and the 64-level / 75k-gate DAG decrypted in full with gate-local parity of
two sampled gates per level (the oracle recomputes them from the GPU's own input wires)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import workloads as W
from paper_2010_09410_amd import VspError, client
from paper_2010_09410_amd import _native as nv
from paper_2010_09410_amd.device import to_host

pytestmark = pytest.mark.gpu
n = 630

TRUTH = {0: lambda a, b: 1 - (a & b), 1: lambda a, b: a & b, 2: lambda a, b: a | b, 3: lambda a, b: 1 - (a | b),
         4: lambda a, b: a ^ b, 5: lambda a, b: 1 - (a ^ b), 6: lambda a, b: a & (1 - b), 7: lambda a, b: a | (1 - b),
         8: lambda a, b: 1 - a}


def plaintext_eval(gates, bits):
    wires = list(int(b) for b in bits)
    for op, a, b in gates:
        wires.append(TRUTH[int(op)](wires[a], wires[b]))
    return np.array(wires, dtype=np.uint8)


def oracle_eval(keys, gates, level, inputs):
    """Level by level, gates of a level in parallel on the CPU oracle."""
    wires = np.zeros((len(inputs) + len(gates), n + 1), dtype=np.uint32)
    wires[: len(inputs)] = inputs
    ni = len(inputs)
    for L in range(int(level.max()) + 1):
        idx = np.nonzero(level == L)[0]
        ops = gates[idx, 0].astype(np.uint8)
        a = wires[gates[idx, 1]]
        b = wires[gates[idx, 2]]
        wires[ni + idx] = oracle.gates(keys["bk"], keys["ksk"], ops, a, b)
    return wires


def test_small_circuit_bit_exact_and_graph_equals_eager(gpu, keys):
    c = W.small_circuit(seed=700, levels=4, wmin=3, wmax=9, ninputs=12)
    gates = c["gates"].copy()
    gates[5, 0] = nv.NOT                      # exercise the no-bootstrap path inside a level
    gates[7, 0] = nv.ANDNOT
    inputs = client.tlwe_encrypt_bits(keys["s0"], c["bits"], *c["enc"])
    circ = gpu.circuit(gates, c["ninputs"])
    wires = to_host(circ.run(gpu.tensor(inputs)))
    wires_eager, ms = circ.run_timed(gpu.tensor(inputs))
    gpu.sync()
    np.testing.assert_array_equal(wires, to_host(wires_eager))
    assert len(ms) == circ.nlevels and all(t > 0 for t in ms)
    # levels as the library computes them (NOT takes one input)
    level = np.zeros(len(gates), dtype=np.int64)
    lv = [0] * c["ninputs"]
    for g, (op, a, b) in enumerate(gates):
        L = lv[a] if op == nv.NOT else max(lv[a], lv[b])
        lv.append(L + 1)
        level[g] = L
    ref = oracle_eval(keys, gates, level, inputs)
    np.testing.assert_array_equal(wires, ref)
    np.testing.assert_array_equal(client.tlwe_decrypt(keys["s0"], wires), plaintext_eval(gates, c["bits"]))
    circ.close()


def test_circuit_rejects_malformed(gpu):
    with pytest.raises(VspError):
        gpu.circuit(np.array([[0, 0, 5]]), 2)           # reads a wire not yet computed
    with pytest.raises(VspError):
        gpu.circuit(np.array([[11, 0, 1]]), 2)          # invalid opcode
    with pytest.raises(VspError):
        gpu.circuit(np.array([[0, 2, 0]]), 2)           # reads its own output


def test_config3_full_decrypt_and_sampled_parity(gpu, keys):
    c = W.config3()
    inputs = client.tlwe_encrypt_bits(keys["s0"], c["bits"], *c["enc"])
    circ = gpu.circuit(c["gates"], c["ninputs"])
    assert circ.nlevels == 64
    wires = to_host(circ.run(gpu.tensor(inputs)))
    gpu.sync()
    np.testing.assert_array_equal(client.tlwe_decrypt(keys["s0"], wires), plaintext_eval(c["gates"], c["bits"]))
    # gate-local parity: two random gates of every level (plus the first and last gate), the
    # oracle fed the GPU's own input wires
    g = W.rng(701)
    per_level = [g.choice(np.nonzero(c["level"] == L)[0], 2, replace=False) for L in range(64)]
    sample = np.unique(np.concatenate([[0, len(c["gates"]) - 1], *per_level]))
    assert np.array_equal(np.unique(c["level"][sample]), np.arange(64))
    ops = c["gates"][sample, 0].astype(np.uint8)
    ref = oracle.gates(keys["bk"], keys["ksk"], ops, wires[c["gates"][sample, 1]], wires[c["gates"][sample, 2]])
    np.testing.assert_array_equal(wires[c["ninputs"] + sample], ref)
    circ.close()


def test_graph_replays_with_eager_work_between(gpu, keys):
    """The captured level sequence is replayed several times, with unrelated eager launches and
    synchronisations in between; every replay equals the eager result."""
    c = W.small_circuit(seed=702, levels=5, wmin=4, wmax=40, ninputs=16)
    inputs = gpu.tensor(client.tlwe_encrypt_bits(keys["s0"], c["bits"], *c["enc"]))
    circ = gpu.circuit(c["gates"], c["ninputs"])
    eager, _ = circ.run_timed(inputs)
    eager = to_host(eager)
    g = W.rng(703)
    other = W.gate_batch(7, 50)
    o0 = gpu.tensor(client.tlwe_encrypt_bits(keys["s0"], other["bits0"], *other["enc0"]))
    o1 = gpu.tensor(client.tlwe_encrypt_bits(keys["s0"], other["bits1"], *other["enc1"]))
    ops = gpu.tensor(other["ops"])
    for rep in range(3):
        gpu.gates(ops, o0, o1)                     # eager work on the same stream
        gpu.sync()
        replay = to_host(circ.run(inputs))
        np.testing.assert_array_equal(replay, eager, err_msg=f"replay {rep}")
        o0 = gpu.tensor(W.uniform_u32(g, (50, n + 1)))
    circ.close()
    np.testing.assert_array_equal(client.tlwe_decrypt(keys["s0"], eager), plaintext_eval(c["gates"], c["bits"]))


# A 4-bit counter with an enable input: next = state + e, as XOR / AND gates.
COUNTER_GATES = np.array([[nv.XOR, 1, 0], [nv.AND, 1, 0],        # bit 0, carry into bit 1
                          [nv.XOR, 2, 6], [nv.AND, 2, 6],        # bit 1, carry into bit 2
                          [nv.XOR, 3, 8], [nv.AND, 3, 8],        # bit 2, carry into bit 3
                          [nv.XOR, 4, 10]])                      # bit 3
COUNTER_NEXT = [5, 7, 9, 11]


def counter_oracle(keys, state, ins):
    """The same cycles on the oracle: gates level by level, then the latch."""
    for e in ins:
        wires = np.zeros((12, n + 1), dtype=np.uint32)
        wires[0], wires[1:5] = e, state
        for lo, hi in ((0, 2), (2, 4), (4, 6), (6, 7)):
            g = COUNTER_GATES[lo:hi]
            wires[5 + lo:5 + hi] = oracle.gates(keys["bk"], keys["ksk"], g[:, 0].astype(np.uint8), wires[g[:, 1]],
                                                wires[g[:, 2]])
        state = wires[COUNTER_NEXT].copy()
    return state


def test_machine_counter_cycles(gpu, keys):
    """Six clock cycles of the counter with enable bits 1,1,0,1,1,1 from state 0: the state
    decrypts to 5, is bit-exact against the oracle, and two runs of three cycles equal one of six."""
    s0 = keys["s0"]
    g = W.rng(704)
    en = [1, 1, 0, 1, 1, 1]
    ins = client.tlwe_encrypt_bits(s0, np.array(en), *W.tlwe_draws(g, len(en))).reshape(len(en), 1, n + 1)
    st0 = client.tlwe_encrypt_bits(s0, np.zeros(4, dtype=np.int64), *W.tlwe_draws(g, 4))
    m = gpu.machine(COUNTER_GATES, 1, COUNTER_NEXT)
    state = gpu.tensor(st0)
    wires = gpu.empty(m.nwires, n + 1)
    m.run(state, 6, gpu.tensor(ins), wires)
    full = to_host(state)
    state2 = gpu.tensor(st0)
    m.run(state2, 3, gpu.tensor(ins[:3]))
    m.run(state2, 3, gpu.tensor(ins[3:]))
    halves = to_host(state2)
    gpu.sync()
    m.close()
    np.testing.assert_array_equal(client.tlwe_decrypt(s0, full), [1, 0, 1, 0])   # 5, least significant bit first
    np.testing.assert_array_equal(full, halves)
    np.testing.assert_array_equal(full, counter_oracle(keys, st0, ins[:, 0]))
    np.testing.assert_array_equal(to_host(wires)[1:5], full)                   # flip-flop rows hold the latched state


def test_machine_rejects_bad_latch(gpu):
    with pytest.raises(VspError):
        gpu.machine(COUNTER_GATES, 1, [5, 7, 9, 99])

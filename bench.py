"""Benchmark: gate bootstraps per second on one MI355X, batched vs per-gate, with the
per-level latency of a layered circuit.

A step is one batched homomorphic-gate pass (gate linear combination, modulus switch,
blind rotation by 630 CMUX external products, SampleExtract, identity key switch) over a
batch of 4096 independent random gates (NAND/AND/OR/XOR/XNOR, uniform) on fresh TLWE
ciphertexts with the 80-bit parameter set (n = 630, N = 1024, l = 3, Bg = 64, t = 8, base 4).
Keys and inputs are synthetic (seeded) and resident in HBM before the timed region.

Prints one JSON line (rank 0). Extra fields: the per-gate rate (one launch sequence per
gate), the batched / per-gate ratio, per-level p50/p99 latency of the 64-level circuit, a
serving run (Poisson arrivals of layered circuits from 64 clients: throughput and p50/p99
circuit latency), the roofline of the dominant kernel (the matrix-core step kernel against the
int8 MFMA peak, or the NTT blind-rotation kernel against the integer-ALU peak, whichever form
the autotuner picks for the batch) with the HBM side, and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

B_GATES = 4096
N_LWE, N_RING, GL, STEPS_BR = 630, 1024, 3, 630

# ---------------------------------------------------------------- work model
# 32-bit VALU lane-operations of one blind-rotation step: the modular operations of the
# algorithm (per lane of a wave; lanes 0-31 and 32-63 each carry one polynomial) priced at
# the instruction counts of the compiled gfx950 routines they use. Butterflies multiply
# their second input by 2^E (canonical result) and then add and subtract with one carry fix:
# 17.5 instructions for E mod 96 below 32, 25 in [32, 64), 20 in [64, 96), 14 for E = 0,
# 8 for the first stage on small digits. A general product mod p is 22, a canonical 2^E
# product 9 / 15 / 10 by the same classes, an add mod p 7, a gadget digit with its rotation
# 8, an exact lift 4; the key MAC adds two products with one reduction (40) and the two
# half-wave swaps (2) to the accumulator (7).
C_MUL, C_ADD, C_DIGIT, C_LIFT, C_DOT2, C_SWAP = 22, 7, 8, 4, 40, 2
BF_LO, BF_MID, BF_HI, BF_TRIV, BF_SMALL = 17.5, 25, 20, 14, 8
P2_LO, P2_MID, P2_HI = 9, 15, 10


def _exp_class(E: int) -> int:
    e = E % 96
    return 3 if e == 0 else (0 if e < 32 else (1 if e < 64 else 2))


def _brv5(k: int) -> int:
    return int(f"{k:05b}"[::-1], 2)


def br_step_lane_ops() -> int:
    cost = {0: BF_LO, 1: BF_MID, 2: BF_HI, 3: BF_TRIV}
    # pass 1 (negacyclic, twiddle 2^(3 brv5(m)) at stage s for blocks m in [2^s, 2^(s+1)))
    pass1 = 16 * BF_SMALL + sum((16 >> s) * cost[_exp_class(3 * _brv5(m))]
                                for s in range(1, 5) for m in range(1 << s, 2 << s))
    # cyclic DFT32 with w = 2^6 (decimation in time: span H uses w^(j 16 / H))
    dft = sum(cost[_exp_class(6 * j * (16 // H))] * (32 // (2 * H)) for H in (1, 2, 4, 8, 16) for j in range(H))
    table = 31 * C_MUL
    twist = sum({0: P2_LO, 1: P2_MID, 2: P2_HI}[_exp_class(96 - 3 * t)] for t in range(1, 32))
    forward = pass1 + table + dft
    inverse = dft + table + dft + twist + 32 * C_LIFT
    mac = GL * 32 * (C_DOT2 + C_SWAP + C_ADD)    # per lane: 32 slots, 3 rounds
    digits = GL * 32 * C_DIGIT
    return int(round(64 * (GL * forward + inverse + mac + digits)))


LANE_OPS_PER_GATE = STEPS_BR * br_step_lane_ops()
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9            # CUs x SIMDs x lanes/clk x clock: 39.3 T/s
BK_NTT_BYTES = N_LWE * 2 * GL * 2 * N_RING * 8  # key stream read by every gate (61.93 MB)
HBM_PEAK = 8.0e12                               # bytes/s


# The method's own arithmetic per gate bootstrap (independent of how a kernel organises it):
# 630 external products, each with 6 forward and 2 inverse negacyclic transforms of N = 1024
# points (N/2 log2 N = 5,120 butterflies, one product and one sum and one difference mod p
# each) and 12 pointwise key products of N points (one product and one sum each).
BUTTERFLIES = N_RING // 2 * 10
MULMOD_PER_GATE = STEPS_BR * (8 * BUTTERFLIES + 2 * 2 * GL * N_RING)      # 33.5 M
ADDMOD_PER_GATE = STEPS_BR * (2 * 8 * BUTTERFLIES + 2 * 2 * GL * N_RING)  # 59.4 M


def algorithmic(gates_per_s: float, ceiling):
    """Gates/s against the method's work priced at the measured register-resident rates of a
    product and of a sum mod p on the whole chip (`vsp_measure_modp`)."""
    if ceiling is None:
        return None
    mul, add = ceiling
    g_mul = mul / MULMOD_PER_GATE                                   # products alone
    g_both = 1.0 / (MULMOD_PER_GATE / mul + ADDMOD_PER_GATE / add)  # products and sums, same VALU
    return {"mulmod_per_gate": MULMOD_PER_GATE, "addmod_per_gate": ADDMOD_PER_GATE,
            "mulmod_per_s": round(mul / 1e12, 4), "addmod_per_s": round(add / 1e12, 4), "unit": "T/s",
            "ceiling_gates_per_s_mulmod_only": round(g_mul, 1), "frac_mulmod_only": round(gates_per_s / g_mul, 4),
            "ceiling_gates_per_s": round(g_both, 1), "frac": round(gates_per_s / g_both, 4)}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def br_hbm_bytes(B: int) -> int:
    """Algorithmic HBM bytes of one blind-rotation launch over B gates: the key once, the
    opcodes and modulus-switched inputs read, the extracted TLWE rows written."""
    return BK_NTT_BYTES + B * (1 + (N_LWE + 1) * 4 + (N_RING + 1) * 4)


# ---------------------------------------------------------------- matrix-core form
# One step kernel launch computes, per tile of 32 gates and output polynomial, the three
# half-size Toeplitz products of one Karatsuba level (P1, P2, P3: 3 x 512 x 512 multiply-adds)
# for the 6 TRGSW rows and the 4 byte planes of the key, as int8 MFMA (2 ops per multiply-add).
MF_TILE = 32
MF_OPS_PER_TILE = 2 * MF_TILE * 2 * 3 * (N_RING // 2) ** 2 * 2 * GL * 4
MF_A_TILE_BYTES = 2 * GL * 3 * (N_RING // 2) * MF_TILE      # digit operands of a tile (int8)
MF_KEY_STEP_BYTES = (2 * GL * 2 * 4 * 3 * N_RING             # three key sequences per row, output, plane,
                     + 2 * N_RING * 4)                      # and the digit-offset correction per output
PEAK_INT8 = 5.0e15                                          # dense int8 MFMA, ops/s
PROF_PERIOD = 16                                            # event-timed launches: one in PROF_PERIOD


def mf_step_ops(B: int) -> int:
    return (B + MF_TILE - 1) // MF_TILE * MF_OPS_PER_TILE


def mf_step_hbm_bytes(B: int) -> int:
    """Compulsory HBM bytes of one step kernel launch: the step's digit operands read once and
    the next step's written once (segments x1 and x0 only: the step forms their sum segment
    itself), the step's key (with its offset correction) read once, the accumulators read and
    written."""
    operands = (B + MF_TILE - 1) // MF_TILE * MF_A_TILE_BYTES * 2 // 3
    return 2 * operands + MF_KEY_STEP_BYTES + B * 2 * N_RING * 4 * 2


def src_fingerprint(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2010_09410_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def br_fingerprint() -> str:
    return src_fingerprint(("gl64.h", "ntt.h", "blind_rotate.h"))


def mf_fingerprint() -> str:
    return src_fingerprint(("gl64.h", "ntt.h", "vsp_internal.h", "blind_rotate_mfma.hip"))


def measured_traffic(fp: str):
    """HBM bytes per launch of the kernel whose sources have fingerprint fp, from a committed
    rocprofv3 summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), else None."""
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        fields = {}
        with open(path) as fh:
            for line in fh:
                if line.startswith("traffic_"):
                    k, _, v = line.partition(":")
                    fields[k.strip()] = v.strip()
        if fields.get("traffic_fingerprint") == fp and "traffic_bytes_per_launch" in fields:
            return int(fields["traffic_bytes_per_launch"]), os.path.basename(path)
    return None, None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--per-gate", type=int, default=64, help="gates timed in per-gate mode")
    ap.add_argument("--no-circuit", action="store_true", help="skip the per-level circuit latency")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--cpu-gates", type=int, default=0, help="oracle sample size (default: about 12 s of work)")
    ap.add_argument("--no-memory", action="store_true", help="skip the CMUX-memory timings")
    ap.add_argument("--no-machine", action="store_true", help="skip the clocked-netlist cycle timing")
    ap.add_argument("--serving", type=float, default=10.0, metavar="SECONDS",
                    help="arrival window of the serving run at 50 circuits/s (0 skips it)")
    ap.add_argument("--serving-light", type=float, default=0.7, metavar="FRACTION",
                    help="also serve about 30 circuits offered at this fraction of the measured batched "
                         "throughput (0 skips it)")
    ap.add_argument("--no-ntt-form", action="store_true",
                    help="skip timing the 4096-gate batch in the NTT form when the tuning picks the matrix form")
    ap.add_argument("--no-key-reuse", action="store_true",
                    help="skip the 4096-gate NTT-form batch without key reuse (one key copy per resident gate)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of MIB MiB (reference for HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(s0, s1, bkd, kskd, cfg, in0, in1, ngates):
    """The CPU oracle (test infrastructure) on this host's cores, on a bounded sample sized
    to about 12 s of work from a short first pass; also one gate on one thread and 16 ROM
    reads (512-word ROM, 9-bit addresses) on all threads."""
    import oracle
    import workloads as W
    from paper_2010_09410_amd import client
    threads = max(1, len(os.sched_getaffinity(0)))
    bk, ksk = oracle.keyset(s0, s1, bkd, kskd)
    if not ngates:
        n0 = 2 * threads
        t0 = time.perf_counter()
        oracle.gates(bk, ksk, cfg["ops"][:n0], in0[:n0], in1[:n0], threads=threads)
        rate0 = n0 / (time.perf_counter() - t0)
        ngates = int(min(len(cfg["ops"]), max(n0, round(rate0 * 12.0 / threads) * threads)))
    t0 = time.perf_counter()
    oracle.gates(bk, ksk, cfg["ops"][:ngates], in0[:ngates], in1[:ngates], threads=threads)
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    oracle.gates(bk, ksk, cfg["ops"][:1], in0[:1], in1[:1], threads=1)
    single = time.perf_counter() - t1
    wl = W.rom_workload(reads=16)
    rom = client.trlwe_encrypt_torus(s1, client.pack_rom(wl["words"]), *wl["cells"])
    sel = client.trgsw_encrypt(s1, (wl["addr"][:, None] >> np.arange(9)[None, :]) & 1, *wl["sel"])
    t2 = time.perf_counter()
    oracle.rom_reads(ksk, rom, sel, threads=threads)
    rom_dt = time.perf_counter() - t2
    return {"value": round(ngates / dt, 2), "unit": "gate bootstraps/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"first {ngates} gates of the 4096-gate batch, {threads} threads, {dt:.1f} s",
            "single_thread_s_per_gate": round(single, 3), "rom_reads_per_s": round(16 / rom_dt, 1)}


def memory_run(ctx, s0, s1, reps: int = 3):
    """CMUX memory (Sec. 8): 256 ROM reads of 32 bits from a 512-word ROM, 256 RAM reads and
    one RAM write of an 8-bit word over 256 addresses, timed with events on the library's
    stream (median of `reps` after one warm-up). Encrypted inputs from the seeded workloads."""
    import torch

    import workloads as W
    from paper_2010_09410_amd import client
    wl = W.rom_workload(reads=256)
    rom = client.trlwe_encrypt_torus(s1, client.pack_rom(wl["words"]), *wl["cells"])
    sel = client.trgsw_encrypt(s1, (wl["addr"][:, None] >> np.arange(9)[None, :]) & 1, *wl["sel"])
    rw = W.ram_workload(v=8, w=8, reads=1, flag=1)
    ram = client.trlwe_encrypt_torus(s1, client.ram_cell_messages(rw["contents"]), *rw["cells"])
    wsel = client.trgsw_encrypt(s1, (rw["waddr"] >> np.arange(8)) & 1, *rw["wsel"])
    flag = client.tlwe_encrypt_bits(s0, [rw["flag"]], *rw["fenc"])[0]
    data = client.tlwe_encrypt_bits(s0, rw["wdata"], *rw["denc"])
    rsel = client.trgsw_encrypt(s1, (wl["addr"][:, None] % 256 >> np.arange(8)[None, :]) & 1,
                                wl["sel"][0][:, :8], wl["sel"][1][:, :8])
    d_rom, d_sel, d_ram0 = ctx.tensor(rom), ctx.tensor(sel), ctx.tensor(ram)
    d_wsel, d_flag, d_data, d_rsel = ctx.tensor(wsel), ctx.tensor(flag), ctx.tensor(data), ctx.tensor(rsel)
    d_ram = d_ram0.clone()
    st = torch.cuda.current_stream(ctx.device)

    def timed(fn):
        fn()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fn()
            e1.record(st)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    rom_ms = timed(lambda: ctx.rom_read(d_rom, d_sel, 9, 32))
    rd_ms = timed(lambda: ctx.ram_read(d_ram0, d_rsel))

    def write():
        d_ram.copy_(d_ram0)
        ctx.ram_write(d_ram, d_wsel, d_flag, d_data)
    wr_ms = timed(write)
    ctx.sync()
    return {"rom_256_reads_ms": round(rom_ms, 2), "rom_reads_per_s": round(256 / (rom_ms / 1e3), 1),
            "ram_256_reads_ms": round(rd_ms, 2), "ram_write_ms": round(wr_ms, 2),
            "workload": "ROM 512 x 32-bit words (16 packed TRLWE), 9-bit encrypted addresses; RAM v = 8, "
                        "w = 8 (2,048 TRLWE cells); write = read + control unit + 2,048 write bars + "
                        "2,048 refresh bootstraps"}


def circuit_bootstrap_run(ctx, s0, s1, reps: int = 2):
    """Circuit bootstrapping (TLWE -> TRGSW) of the address bits of 256 ROM reads (9 bits each,
    2,304 conversions), then the ROM read from those selectors; and one cycle of the clocked
    netlist's RAM port (v = 8, w = 8): 8 address bits converted, one read, one write."""
    import torch

    import workloads as W
    from paper_2010_09410_amd import client
    t0 = time.perf_counter()
    bk2, pksk = client.keyset2(s0, s1, W.secret_key2(), W.bk2_draws(), W.pksk_draws())
    keygen_s = time.perf_counter() - t0
    key = ctx.cbkey(bk2, pksk)
    del bk2, pksk
    wl = W.rom_workload(reads=256)
    rom = client.trlwe_encrypt_torus(s1, client.pack_rom(wl["words"]), *wl["cells"])
    bits = (wl["addr"][:, None] >> np.arange(9)[None, :]) & 1
    tl = client.tlwe_encrypt_bits(s0, bits.reshape(-1), *W.tlwe_draws(W.rng(44), bits.size))
    d_rom, d_tl = ctx.tensor(rom), ctx.tensor(tl)
    st = torch.cuda.current_stream(ctx.device)

    def timed(fn):
        fn()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fn()
            e1.record(st)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    sel = ctx.empty(bits.size, 6, 2, 1024)
    cb_ms = timed(lambda: key.bootstrap(d_tl, out=sel))
    one_ms = timed(lambda: key.bootstrap(d_tl[:1], out=sel[:1]))
    rom_ms = timed(lambda: ctx.rom_read(d_rom, sel.reshape(256, 9, 6, 2, 1024), 9, 32))
    tl8 = ctx.tensor(client.tlwe_encrypt_bits(s0, bits[0, :8], *W.tlwe_draws(W.rng(45), 8)))
    rw = W.ram_workload(v=8, w=8, reads=1, flag=1)
    d_ram = ctx.tensor(client.trlwe_encrypt_torus(s1, client.ram_cell_messages(rw["contents"]), *rw["cells"]))
    flag = ctx.tensor(client.tlwe_encrypt_bits(s0, [1], *rw["fenc"])[0])
    data = ctx.tensor(client.tlwe_encrypt_bits(s0, rw["wdata"], *rw["denc"]))
    rsel = ctx.empty(8, 6, 2, 1024)

    def ram_cycle():
        key.bootstrap(tl8, out=rsel)
        ctx.ram_read(d_ram, rsel.reshape(1, 8, 6, 2, 1024))
        ctx.ram_write(d_ram, rsel, flag, data)
    cyc_ms = timed(ram_cycle)
    ctx.sync()
    key.close()
    return {"conversions": int(bits.size), "batch_ms": round(cb_ms, 2),
            "per_s": round(bits.size / (cb_ms / 1e3), 1), "single_ms": round(one_ms, 2),
            "rom_256_reads_from_tlwe_addresses_ms": round(cb_ms + rom_ms, 2),
            "ram_port_cycle_ms": round(cyc_ms, 2), "client_keygen_s": round(keygen_s, 1),
            "params": "level 2: N2 = 2048, l2 = 4, Bg2 = 2^9 on the 2^64 torus; private key switch t = 12, base 4",
            "workload": "address bits of 256 ROM reads (512 x 32-bit words, 9-bit addresses) as fresh TLWE; RAM "
                        "port cycle v = 8, w = 8: 8 conversions, one read, one write"}


def machine_run(ctx, s0, cycles: int = 3):
    """Clock cycles of a synthetic clocked netlist of a small processor's size (2,422 gates in
    32 levels, 256 flip-flops), one HIP graph replay per cycle, timed with events."""
    import torch

    import workloads as W
    from paper_2010_09410_amd import client
    net = W.clocked_netlist()
    m = ctx.machine(net["gates"], 0, net["next_state"])
    state = ctx.tensor(client.tlwe_encrypt_bits(s0, net["bits"], *net["enc"]))
    m.run(state, 1)
    st = torch.cuda.current_stream(ctx.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    m.run(state, cycles)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / cycles
    m.close()
    return {"gates": len(net["gates"]), "levels": int(net["level"].max()) + 1, "flip_flops": net["nstate"],
            "s_per_cycle": round(ms / 1e3, 4), "gates_per_s": round(len(net["gates"]) / (ms / 1e3), 1),
            "workload": "synthetic layered netlist of the paper's pipelined-processor gate count (2,422 two-input "
                        "gates), 32 levels, 256 flip-flops; no CMUX memory"}


MEAN_CIRCUIT_GATES = (20000 - 100) / np.log(20000 / 100)   # log-uniform sizes in [100, 20000]


def serving_run(ctx, s0, duration: float, rate: float = 50.0, mem_budget: int = 2 << 30, nkeys: int = 1):
    """Replays Poisson arrivals of layered circuits from 64 clients in real time against the
    continuous-batching server; inputs are encrypted before the clock starts. With nkeys > 1,
    client c encrypts under key set c mod nkeys (set 0 is the context's keys, the others are
    drawn from seeds 30 + 3k) and the server batches per key set."""
    import workloads as W
    from paper_2010_09410_amd import client
    trace = W.serving_trace(rate=rate, duration=duration)
    sks, keysets = [s0], [None]
    for k in range(1, nkeys):
        a0, a1 = W.secret_keys(30 + 3 * k)
        sks.append(a0)
        keysets.append(ctx.keyset(*client.keyset(a0, a1, W.bk_draws(31 + 3 * k), W.ksk_draws(32 + 3 * k))))
    which = [r["client"] % nkeys for r in trace]
    enc = [client.tlwe_encrypt_bits(sks[w], r["bits"], *W.tlwe_draws(W.rng(r["enc_seed"]), r["ninputs"]))
           for r, w in zip(trace, which)]
    srv = ctx.server(mem_budget, max_batch=4096)
    pending, lat, done_t = {}, [], []
    i = 0
    t0 = time.perf_counter()
    while i < len(trace) or pending:
        now = time.perf_counter() - t0
        while i < len(trace) and trace[i]["t"] <= now:
            r = trace[i]
            pending[srv.submit(r["gates"], r["ninputs"], enc[i], keyset=keysets[which[i]])] = i
            i += 1
        for tk, j in list(pending.items()):
            done, _, ms = srv.poll(tk, trace[j]["ninputs"] + len(trace[j]["gates"]))
            if done:
                lat.append(ms)
                done_t.append(time.perf_counter() - t0)
                del pending[tk]
        time.sleep(0.002)
    gates, batches, peak = srv.stats()
    srv.close()
    for k in keysets[1:]:
        k.close()
    total = sum(len(r["gates"]) for r in trace)
    span = max(done_t) - trace[0]["t"]
    lat = np.array(lat)
    return {"circuits": len(trace), "clients": 64, "key_sets": nkeys, "gates": total,
            "rate_circuits_per_s": round(rate, 2),
            "arrival_window_s": round(duration, 2),
            "offered_gates_per_s": round(total / duration, 1), "served_gates_per_s": round(total / span, 1),
            "makespan_s": round(span, 3), "p50_latency_ms": round(float(np.percentile(lat, 50)), 1),
            "p99_latency_ms": round(float(np.percentile(lat, 99)), 1), "batches": int(batches),
            "mean_batch": round(gates / max(batches, 1), 1), "peak_resident_MB": round(peak / 1e6, 1),
            "memory_budget_MB": round(mem_budget / 1e6, 1)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is a "
              "design note, not a measured path.", file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads as W
    from paper_2010_09410_amd import VSP_PER_GATE, client
    from paper_2010_09410_amd import _native as nv
    from paper_2010_09410_amd.device import Context

    s0, s1 = W.secret_keys()
    bkd, kskd = W.bk_draws(), W.ksk_draws()
    bk, ksk = client.keyset(s0, s1, bkd, kskd)
    cfg = W.config2(B_GATES)
    in0 = client.tlwe_encrypt_bits(s0, cfg["bits0"], *cfg["enc0"])
    in1 = client.tlwe_encrypt_bits(s0, cfg["bits1"], *cfg["enc1"])
    ctx = Context(bk, ksk, device=0)
    ops_d, a_d, b_d = ctx.tensor(cfg["ops"]), ctx.tensor(in0), ctx.tensor(in1)
    out = ctx.empty(B_GATES, N_LWE + 1)
    tune = None
    if not args.no_autotune:
        import tempfile
        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "tune.json")
            ctx.autotune(max_batch=B_GATES, cache_path=path)
            with open(path) as fh:
                (_, tune), = json.load(fh).items()
    br_waves, ks_form = ctx.tuning(B_GATES)

    for _ in range(args.warmup):
        ctx.gates(ops_d, a_d, b_d, out=out)
    ctx.sync()
    # kernel times live over the timed region, from HIP events around every PROF_PERIOD-th
    # launch of each kind (event pairs around all 630 step launches of a batch would cost
    # about 6% of its time)
    nv.vsp_profile_enable(ctx.handle, PROF_PERIOD)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.gates(ops_d, a_d, b_d, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    br_ms, br_n = nv.vsp_profile_read(ctx.handle, 0)
    ks_ms, ks_n = nv.vsp_profile_read(ctx.handle, 1)
    step_ms, step_n = nv.vsp_profile_read(ctx.handle, 3)
    nv.vsp_profile_enable(ctx.handle, False)
    ctx.sync()
    ms_per_step = dt * 1e3 / args.steps
    value = B_GATES * args.steps / dt

    # register-resident throughput of a product and of a sum mod p on the whole chip
    ceiling = nv.vsp_measure_modp(0, 4096)

    # the same batch in the NTT form (the transform-domain method), when the tuning picked the
    # matrix-core form for it
    ntt_form = None
    if br_waves == 32 and not args.no_ntt_form:
        ctx.set_tuning(B_GATES, 8, ks_form)
        ctx.gates(ops_d, a_d, b_d, out=out)
        ctx.sync()
        nv.vsp_profile_enable(ctx.handle, True)
        reps = 3
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.gates(ops_d, a_d, b_d, out=out)
        torch.cuda.synchronize()
        ndt = time.perf_counter() - t0
        nbr_ms, nbr_n = nv.vsp_profile_read(ctx.handle, 0)
        nv.vsp_profile_enable(ctx.handle, False)
        ctx.set_tuning(B_GATES, 32, ks_form)
        ctx.sync()
        nrate = B_GATES * reps / ndt
        navg = nbr_ms / max(nbr_n, 1)
        nach = B_GATES * LANE_OPS_PER_GATE / (navg * 1e-3)
        ntraffic, nsrc = measured_traffic(br_fingerprint())
        ntt_form = {"kernel": "k_blind_rotate<8>", "value": round(nrate, 1), "unit": "gate bootstraps/s",
                    "ms_per_step": round(ndt * 1e3 / reps, 3), "blind_rotation_avg_ms": round(navg, 3),
                    "alu": {"achieved": round(nach / 1e12, 3), "peak": round(PEAK_LANE_OPS / 1e12, 3),
                            "unit": "T int32 lane-ops/s (compiled-routine instruction model)",
                            "frac": round(nach / PEAK_LANE_OPS, 4)},
                    "algorithmic": algorithmic(B_GATES / (navg * 1e-3), ceiling),
                    "hbm": {"algorithmic_bytes_per_launch": br_hbm_bytes(B_GATES),
                            "frac": round(br_hbm_bytes(B_GATES) / (navg * 1e-3) / HBM_PEAK, 6),
                            "measured_bytes_per_launch": ntraffic, "traffic_source": nsrc,
                            "measured_GBps": None if ntraffic is None else round(ntraffic / (navg * 1e-3) / 1e9, 1)}}

    # What key reuse contributes: the same batch in the eight-wave NTT form with one shared key,
    # then with gate g reading its own device copy g mod C, C = the gates the form holds at once
    # (eight per CU), so that no resident gate shares key bytes with another; and one gate alone
    # in the three-wave latency form (occupancy: one workgroup on the chip).
    key_reuse = None
    if not args.no_key_reuse:
        resident = 8 * torch.cuda.get_device_properties(ctx.device).multi_processor_count
        kr = {"form": "k_blind_rotate<8>", "gates": B_GATES, "key_bytes_per_gate": BK_NTT_BYTES}
        for name, copies in (("shared", 1), ("unshared", resident)):
            ctx.gates_key_copies(ops_d[:16], a_d[:16], b_d[:16], waves=8, copies=1)
            _, ms = ctx.gates_key_copies(ops_d, a_d, b_d, waves=8, copies=copies, out=out)
            kb = B_GATES * BK_NTT_BYTES if copies > 1 else BK_NTT_BYTES
            kr[name] = {"copies": copies, "blind_rotation_ms": round(ms, 3),
                        "gates_per_s": round(B_GATES / (ms * 1e-3), 1),
                        "key_bytes_requested": kb, "key_GBps": round(kb / (ms * 1e-3) / 1e9, 1),
                        "key_frac_of_hbm": round(kb / (ms * 1e-3) / HBM_PEAK, 4)}
        _, one = ctx.gates_key_copies(ops_d[:1], a_d[:1], b_d[:1], waves=3, copies=1)
        kr["one_gate"] = {"form": "k_blind_rotate_wide", "blind_rotation_ms": round(one, 3),
                          "gates_per_s": round(1e3 / one, 2),
                          "key_GBps": round(BK_NTT_BYTES / (one * 1e-3) / 1e9, 2)}
        kr["occupancy_gain"] = round(kr["unshared"]["gates_per_s"] / kr["one_gate"]["gates_per_s"], 1)
        kr["reuse_gain"] = round(kr["shared"]["gates_per_s"] / kr["unshared"]["gates_per_s"], 3)
        key_reuse = kr
        torch.cuda.synchronize()

    # per-gate mode: one launch sequence per gate, each streaming the whole key
    per_gate = None
    pg = args.per_gate
    if pg > 0:
        ctx.gates(ops_d[:1], a_d[:1], b_d[:1], mode=VSP_PER_GATE)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.gates(ops_d[:pg], a_d[:pg], b_d[:pg], mode=VSP_PER_GATE)
        torch.cuda.synchronize()
        per_gate = pg / (time.perf_counter() - t0)

    # homomorphic MUX (two bootstraps and one key switch per MUX), 2048 rows of the same inputs
    mux_rate = None
    if pg > 0:
        M = B_GATES // 2
        mo = ctx.empty(M, N_LWE + 1)
        ctx.mux(a_d[:M], b_d[:M], a_d[M:2 * M], out=mo)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.mux(a_d[:M], b_d[:M], a_d[M:2 * M], out=mo)
        torch.cuda.synchronize()
        mux_rate = M / (time.perf_counter() - t0)
        del mo

    if args.calibrate_copy > 0:
        src = torch.empty(args.calibrate_copy << 18, dtype=torch.int32, device=ctx.device).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # per-level latency of the 64-level circuit (eager levels timed with events)
    levels = None
    if not args.no_circuit and hasattr(nv.lib(), "vsp_circuit_create"):
        c3 = W.config3()
        cin = client.tlwe_encrypt_bits(s0, c3["bits"], *c3["enc"])
        circ = ctx.circuit(c3["gates"], c3["ninputs"])
        d_cin = ctx.tensor(cin)
        circ.run(d_cin)  # warm-up: the first launch of each kernel loads its code
        torch.cuda.synchronize()
        _, lv_ms = circ.run_timed(d_cin)
        lv = np.array(lv_ms)
        # the captured level sequence (one HIP graph launch), timed with events
        wires = circ.run(d_cin)
        st = torch.cuda.current_stream(ctx.device)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        circ.run(d_cin, wires)
        e1.record(st)
        e1.synchronize()
        graph_ms = e0.elapsed_time(e1)
        widths = np.asarray(c3["widths"])
        levels = {"levels": int(lv.size), "gates": int(len(c3["gates"])),
                  "p50_ms": round(float(np.percentile(lv, 50)), 3), "p99_ms": round(float(np.percentile(lv, 99)), 3),
                  "min_width": int(widths.min()), "max_width": int(widths.max()),
                  "eager_circuit_ms": round(float(lv.sum()), 2),
                  "eager_gates_per_s": round(float(len(c3["gates"]) / (lv.sum() / 1e3)), 1),
                  "graph_circuit_ms": round(graph_ms, 2),
                  "graph_gates_per_s": round(len(c3["gates"]) / (graph_ms / 1e3), 1)}
        del wires
        circ.close()

    memory = None
    if not args.no_memory:
        memory = memory_run(ctx, s0, s1)
    machine = None
    if not args.no_machine:
        machine = machine_run(ctx, s0)
    cbs = None
    if not args.no_memory:
        cbs = circuit_bootstrap_run(ctx, s0, s1)

    serving = None
    if args.serving > 0:
        serving = serving_run(ctx, s0, args.serving)
    if args.serving_light > 0:
        rate = args.serving_light * value / MEAN_CIRCUIT_GATES
        light = serving_run(ctx, s0, 30.0 / rate, rate=rate)
        light["offered_fraction_of_batched_throughput"] = args.serving_light
        keyed = serving_run(ctx, s0, 30.0 / rate, rate=rate, nkeys=4)
        keyed["offered_fraction_of_batched_throughput"] = args.serving_light
        serving = dict(config=serving, light=light, light_4_key_sets=keyed)

    per_gate_key = None
    if per_gate is not None:
        # each gate of the per-gate path streams the whole key of its form once: the byte-plane
        # key in the matrix-core forms, the NTT-domain key otherwise
        pg_form = ctx.tuning(1)[0]
        pg_bytes = N_LWE * MF_KEY_STEP_BYTES if pg_form in (32, 33) else BK_NTT_BYTES
        per_gate_key = {"GBps": round(per_gate * pg_bytes / 1e9, 2),
                        "frac_of_hbm": round(per_gate * pg_bytes / HBM_PEAK, 6), "gates_timed": pg,
                        "form": pg_form, "key_bytes_per_gate": pg_bytes}
    br_avg_ms = br_ms / max(br_n, 1)
    launch = {"br_shape": br_waves, "keyswitch": ["gather", "tiled", "split", "matrix"][ks_form], "autotune": tune}
    if br_waves == 32:
        # matrix-core form: the dominant kernel is the step kernel (630 launches per batch)
        mf_ms, mf_n = step_ms, step_n
        mf_avg = mf_ms / max(mf_n, 1)
        achieved = mf_step_ops(B_GATES) / (mf_avg * 1e-3)
        traffic, traffic_src = measured_traffic(mf_fingerprint())
        hbm = mf_step_hbm_bytes(B_GATES) / (mf_avg * 1e-3)
        roof = {"bound": "mfma", "kernel": "k_mf_step", "achieved": round(achieved / 1e12, 1),
                "peak": PEAK_INT8 / 1e12, "unit": "TOP/s (int8)", "frac": round(achieved / PEAK_INT8, 4),
                "work": "issued int8 multiply-adds of the one-level Karatsuba Toeplitz products over four "
                        "balanced byte planes (utilisation of issued work, not the method's arithmetic)",
                "algorithmic": algorithmic(value, ceiling),
                "traffic": traffic, "traffic_source": traffic_src, "avg_launch_ms": round(mf_avg, 4),
                "launches_per_batch": N_LWE, "timed_launches": mf_n, "event_sample_period": PROF_PERIOD,
                "int8_ops_per_launch": mf_step_ops(B_GATES),
                "hbm": {"achieved": round(hbm / 1e9, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                        "frac": round(hbm / HBM_PEAK, 4), "algorithmic_bytes_per_launch": mf_step_hbm_bytes(B_GATES),
                        "measured_GBps": None if traffic is None else round(traffic / (mf_avg * 1e-3) / 1e9, 1)},
                "blind_rotation_avg_ms": round(br_avg_ms, 3),
                "keyswitch_avg_ms": round(ks_ms / max(ks_n, 1), 3), "launch": launch}
    else:
        achieved = B_GATES * LANE_OPS_PER_GATE / (br_avg_ms * 1e-3) / 1e12
        traffic, traffic_src = measured_traffic(br_fingerprint())
        hbm = br_hbm_bytes(B_GATES) / (br_avg_ms * 1e-3)
        roof = {"bound": "alu", "kernel": f"k_blind_rotate<{br_waves}>", "achieved": round(achieved, 3),
                "algorithmic": algorithmic(B_GATES / (br_avg_ms * 1e-3), ceiling),
                "peak": round(PEAK_LANE_OPS / 1e12, 3), "unit": "T int32 lane-ops/s",
                "frac": round(achieved * 1e12 / PEAK_LANE_OPS, 4), "traffic": traffic, "traffic_source": traffic_src,
                "avg_launch_ms": round(br_avg_ms, 3), "lane_ops_per_gate": LANE_OPS_PER_GATE,
                "hbm": {"achieved": round(hbm / 1e9, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                        "frac": round(hbm / HBM_PEAK, 4), "algorithmic_bytes_per_launch": br_hbm_bytes(B_GATES),
                        "measured_GBps": None if traffic is None else round(traffic / (br_avg_ms * 1e-3) / 1e9, 1)},
                "key_stream_GBps_requested": round(B_GATES * BK_NTT_BYTES / (br_avg_ms * 1e-3) / 1e9, 1),
                "keyswitch_avg_ms": round(ks_ms / max(ks_n, 1), 3), "launch": launch}
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(s0, s1, bkd, kskd, cfg, in0, in1, args.cpu_gates)
    ctx.close()

    line = {
        "metric": "gate bootstraps/sec on 1 MI355X, batched vs per-gate; p50/p99 per-level latency",
        "value": round(value, 1), "unit": "gate bootstraps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "dtype_note": "exact torus arithmetic mod 2^32; " + ("int8 byte-plane MFMA operands with int32 "
                      "accumulation" if br_waves == 32 else "NTT mod 2^64 - 2^32 + 1 in u64"),
        "config": {"workload": "4096 independent random gates (NAND/AND/OR/XOR/XNOR) on fresh TLWE, "
                               "n=630 N=1024 l=3 Bg=64 ks t=8 base=4, one batched launch",
                   "batch": B_GATES, "parallelism": "single GPU"},
        "per_gate_value": None if per_gate is None else round(per_gate, 2),
        "batched_over_per_gate": None if per_gate is None else round(value / per_gate, 1),
        "per_gate_key_stream": per_gate_key, "ntt_form_4096": ntt_form, "key_reuse": key_reuse,
        "mux_per_s": None if mux_rate is None else round(mux_rate, 1),
        "per_level": levels, "clocked_netlist": machine, "cmux_memory": memory, "circuit_bootstrapping": cbs, "serving": serving, "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Seeded synthetic inputs: every random draw the method makes, and nothing else.

This module holds no TFHE arithmetic. It only draws, from numpy ``PCG64`` generators
with fixed seeds, the random objects the method consumes:

* secret-key bits (uniform binary keys of the TLWE and TRLWE definitions, Sec. 2.1.2),
* uniform torus masks ``a`` (as ``uint32``, the torus discretised to Z/2^32),
* Gaussian noise integers ``e = rint(sigma * 2^32 * z)`` with ``z ~ N(0, 1)``
  (the modular Gaussian of Sec. 2.1.2, sampled at torus resolution 2^-32),
* plaintext bits, gate opcodes, circuit wiring, memory words, addresses and
  request arrival times of the synthetic workloads.

Both the CPU oracle and the GPU library's client take these arrays as inputs; neither
computes them, and this module imports neither.

Seeds: 0 secret keys (s0 then s1), 1 bootstrapping-key masks and noise, 2 key-switching
key masks and noise, 10 + c plaintexts / circuits / arrivals of workload c, 20 + c the
encryption randomness of workload c; for circuit bootstrapping 3 the level-2 key s2,
4 the level-2 bootstrapping-key masks and noise, 5 the private key-switching-key masks and
noise.
"""
from __future__ import annotations

import numpy as np

# Parameter set of the workloads (the 80-bit TFHE set the paper adopts, Sec. 2.1.2).
LWE_N = 630          # TLWE dimension n
RING_N = 1024        # TRLWE degree N
GADGET_L = 3         # TRGSW rows per column l
KS_T = 8             # key-switch digits per coefficient
KS_BASE = 4          # key-switch base (basebit = 2)
SIGMA0 = 2.0 ** -15  # TLWE / key-switching-key noise sd (torus units)
SIGMA1 = 2.0 ** -25  # TRLWE / TRGSW / bootstrapping-key noise sd (torus units)

# Circuit bootstrapping (level 2, a reading: the paper names the operation but fixes no
# parameters): ring degree, gadget, 2^64-torus noise of the level-2 bootstrapping key, and
# the private key switch to level-1 TRLWE with its key's noise.
RING_N2 = 2048
GADGET_L2 = 4
BG_BIT2 = 9
PKS_T = 12
PKS_BASE = 4          # basebit 2
SIGMA2 = 2.0 ** -44   # level-2 bootstrapping-key noise sd (torus units)
SIGMA_PKS = 2.0 ** -30  # private key-switching-key noise sd (torus units)

# Gate opcodes as the C ABI numbers them.
NAND, AND, OR, NOR, XOR, XNOR, ANDNOT, ORNOT, NOT = range(9)
BENCH_OPS = np.array([NAND, AND, OR, XOR, XNOR], dtype=np.uint8)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_u32(g: np.random.Generator, shape) -> np.ndarray:
    return g.integers(0, 2 ** 32, size=shape, dtype=np.uint64).astype(np.uint32)


def gaussian_i32(g: np.random.Generator, sigma: float, shape) -> np.ndarray:
    """Noise integers rint(sigma * 2^32 * z), z ~ N(0,1); sigma = 0 gives zeros."""
    z = g.standard_normal(size=shape)
    return np.rint(z * (sigma * 2.0 ** 32)).astype(np.int64).astype(np.int32)


# --------------------------------------------------------------------------- keys
def secret_keys(seed: int = 0, n: int = LWE_N, N: int = RING_N):
    g = rng(seed)
    s0 = g.integers(0, 2, size=n, dtype=np.uint32)
    s1 = g.integers(0, 2, size=N, dtype=np.uint32)
    return s0, s1


def bk_draws(seed: int = 1, n: int = LWE_N, N: int = RING_N, l: int = GADGET_L,
             sigma: float = SIGMA1):
    """Masks [n][2l][N] and noise [n][2l][N] of the n TRGSW rows of the bootstrapping key."""
    g = rng(seed)
    masks = uniform_u32(g, (n, 2 * l, N))
    noise = gaussian_i32(g, sigma, (n, 2 * l, N))
    return masks, noise


def ksk_draws(seed: int = 2, n: int = LWE_N, N: int = RING_N, t: int = KS_T,
              base: int = KS_BASE, sigma: float = SIGMA0):
    """Masks [N][t][base-1][n] and noise [N][t][base-1] of the key-switching key."""
    g = rng(seed)
    masks = uniform_u32(g, (N, t, base - 1, n))
    noise = gaussian_i32(g, sigma, (N, t, base - 1))
    return masks, noise


def uniform_u64(g: np.random.Generator, shape) -> np.ndarray:
    return g.integers(0, 2 ** 64, size=shape, dtype=np.uint64)


def gaussian_i64(g: np.random.Generator, sigma: float, shape) -> np.ndarray:
    """Noise integers rint(sigma * 2^64 * z) on the 2^64 torus, z ~ N(0,1)."""
    z = g.standard_normal(size=shape)
    return np.rint(z * (sigma * 2.0 ** 64)).astype(np.int64)


def secret_key2(seed: int = 3, N2: int = RING_N2):
    """Binary level-2 TRLWE key (uint64 coefficients)."""
    return rng(seed).integers(0, 2, size=N2, dtype=np.uint64)


def bk2_draws(seed: int = 4, n: int = LWE_N, N2: int = RING_N2, l2: int = GADGET_L2, sigma: float = SIGMA2):
    """Masks [n][2 l2][N2] (uint64) and noise [n][2 l2][N2] (int64) of the level-2
    bootstrapping key."""
    g = rng(seed)
    return uniform_u64(g, (n, 2 * l2, N2)), gaussian_i64(g, sigma, (n, 2 * l2, N2))


def pksk_draws(seed: int = 5, N: int = RING_N, N2: int = RING_N2, t: int = PKS_T, base: int = PKS_BASE,
               sigma: float = SIGMA_PKS):
    """Masks [2][N2+1][t][base-1][N] and noise of the same shape of the two private
    key-switching keys (level-1 TRLWE rows)."""
    g = rng(seed)
    shape = (2, N2 + 1, t, base - 1, N)
    return uniform_u32(g, shape), gaussian_i32(g, sigma, shape)


def tlwe_draws(g: np.random.Generator, count: int, n: int = LWE_N, sigma: float = SIGMA0):
    return uniform_u32(g, (count, n)), gaussian_i32(g, sigma, (count,))


def trlwe_draws(g: np.random.Generator, count: int, N: int = RING_N, sigma: float = SIGMA1):
    return uniform_u32(g, (count, N)), gaussian_i32(g, sigma, (count, N))


def trgsw_draws(g: np.random.Generator, count: int, N: int = RING_N, l: int = GADGET_L,
                sigma: float = SIGMA1):
    return uniform_u32(g, (count, 2 * l, N)), gaussian_i32(g, sigma, (count, 2 * l, N))


# ---------------------------------------------------------------- gate workloads
def gate_batch(config: int, B: int, ops=None):
    """B independent gates on fresh random bits (8 NAND: config 1; 4096 mixed: config 2).

    Returns dict(ops [B] u8, bits0 [B], bits1 [B], enc0=(masks, noise), enc1=(masks, noise)).
    """
    gp = rng(10 + config)
    if ops is None:
        ops = gp.choice(BENCH_OPS, size=B)
    ops = np.asarray(ops, dtype=np.uint8)
    bits = gp.integers(0, 2, size=(2, B), dtype=np.uint8)
    ge = rng(20 + config)
    enc = tlwe_draws(ge, 2 * B)
    return dict(ops=ops, bits0=bits[0], bits1=bits[1],
                enc0=(enc[0][:B], enc[1][:B]), enc1=(enc[0][B:], enc[1][B:]))


def config1():
    """Eight NAND gates on sixteen fresh random encrypted bits."""
    return gate_batch(1, 8, ops=np.full(8, NAND, dtype=np.uint8))


def config2(B: int = 4096):
    """4096 independent gates, opcode uniform over NAND/AND/OR/XOR/XNOR."""
    return gate_batch(2, B)


# ------------------------------------------------------------------- circuits
def layered_circuit(g: np.random.Generator, ninputs: int, widths, ops_pool=BENCH_OPS):
    """Random layered DAG. Gate k of level L takes its first input uniformly from the
    wires of level L-1 (the primary inputs for L = 0) and its second uniformly from all
    earlier wires. Wire ids: primary inputs 0..ninputs-1, then gates in level order.

    Returns (gates [G][3] int64 as (op, in0, in1), level_of_gate [G]).
    """
    widths = [int(w) for w in widths]
    G = sum(widths)
    gates = np.zeros((G, 3), dtype=np.int64)
    level = np.zeros(G, dtype=np.int32)
    prev_lo, prev_hi = 0, ninputs          # wire range of the previous level
    nxt = ninputs                          # next wire id
    k = 0
    for L, w in enumerate(widths):
        ops = g.choice(ops_pool, size=w)
        in0 = g.integers(prev_lo, prev_hi, size=w)
        in1 = g.integers(0, nxt, size=w)
        gates[k:k + w, 0] = ops
        gates[k:k + w, 1] = in0
        gates[k:k + w, 2] = in1
        level[k:k + w] = L
        prev_lo, prev_hi = nxt, nxt + w
        nxt += w
        k += w
    return gates, level


def config3(levels: int = 64, wmin: int = 16, wmax: int = 2048, ninputs: int = 2048):
    """64-level layered DAG with widths uniform in [16, 2048] on 2048 fresh input bits."""
    g = rng(13)
    widths = g.integers(wmin, wmax + 1, size=levels)
    gates, level = layered_circuit(g, ninputs, widths)
    bits = g.integers(0, 2, size=ninputs, dtype=np.uint8)
    enc = tlwe_draws(rng(23), ninputs)
    return dict(ninputs=ninputs, widths=widths, gates=gates, level=level, bits=bits, enc=enc)


def small_circuit(seed: int, levels: int, wmin: int, wmax: int, ninputs: int):
    """A smaller layered DAG of the same recipe (tests)."""
    g = rng(seed)
    widths = g.integers(wmin, wmax + 1, size=levels)
    gates, level = layered_circuit(g, ninputs, widths)
    bits = g.integers(0, 2, size=ninputs, dtype=np.uint8)
    enc = tlwe_draws(rng(seed + 1000), ninputs)
    return dict(ninputs=ninputs, widths=widths, gates=gates, level=level, bits=bits, enc=enc)


def clocked_netlist(gates: int = 2422, levels: int = 32, nstate: int = 256, seed: int = 16):
    """A synthetic clocked netlist of a small processor's size (2,422 two-input gates, the
    gate count of the paper's pipelined processor without its MUX and NOT cells): a layered
    DAG over 256 flip-flop outputs with equal level widths; flip-flop k latches the k-th of
    the last 256 gate outputs. Wire ids: flip-flops 0..nstate-1, then the gates."""
    g = rng(seed)
    widths = np.full(levels, gates // levels, dtype=np.int64)
    widths[: gates - int(widths.sum())] += 1
    gl, level = layered_circuit(g, nstate, widths)
    next_state = (nstate + gates - nstate + np.arange(nstate)).astype(np.uint32)
    bits = g.integers(0, 2, size=nstate, dtype=np.uint8)
    enc = tlwe_draws(rng(seed + 10), nstate)
    return dict(gates=gl, level=level, nstate=nstate, next_state=next_state, bits=bits, enc=enc)


# ------------------------------------------------------------- CMUX memory
def rom_workload(reads: int = 256, words: int = 512, seed_off: int = 0):
    """ROM of 512 uniform 32-bit words and `reads` uniform 9-bit addresses.

    Returns dict(words [512] u32, addr [reads] u32, cell draws for the 16 TRLWE cells,
    selector draws [reads][9] TRGSW).
    """
    g = rng(14 + seed_off)
    W = uniform_u32(g, (words,))
    abits = int(np.log2(words))
    addr = g.integers(0, words, size=reads, dtype=np.uint32)
    ge = rng(24 + seed_off)
    npoly = words * 32 // RING_N
    cells = trlwe_draws(ge, npoly)
    sel = trgsw_draws(ge, reads * abits)
    sel = (sel[0].reshape(reads, abits, 2 * GADGET_L, RING_N),
           sel[1].reshape(reads, abits, 2 * GADGET_L, RING_N))
    return dict(words=W, addr=addr, abits=abits, cells=cells, sel=sel)


def ram_workload(v: int = 8, w: int = 8, reads: int = 4, flag: int = 1, seed_off: int = 0):
    """RAM of 2^v words of w bits: uniform contents, a write of uniform data at a uniform
    address under an encrypted write flag, and `reads` uniform read addresses.
    """
    g = rng(14 + 100 + seed_off)
    contents = g.integers(0, 2, size=(w, 2 ** v), dtype=np.uint8)
    waddr = int(g.integers(0, 2 ** v))
    wdata = g.integers(0, 2, size=w, dtype=np.uint8)
    raddr = g.integers(0, 2 ** v, size=reads, dtype=np.uint32)
    ge = rng(24 + 100 + seed_off)
    cells = trlwe_draws(ge, w * 2 ** v)
    cells = (cells[0].reshape(w, 2 ** v, RING_N), cells[1].reshape(w, 2 ** v, RING_N))
    wsel = trgsw_draws(ge, v)
    rsel = trgsw_draws(ge, reads * v)
    rsel = (rsel[0].reshape(reads, v, 2 * GADGET_L, RING_N),
            rsel[1].reshape(reads, v, 2 * GADGET_L, RING_N))
    fenc = tlwe_draws(ge, 1)
    denc = tlwe_draws(ge, w)
    return dict(v=v, w=w, contents=contents, waddr=waddr, wdata=wdata, flag=int(flag),
                raddr=raddr, cells=cells, wsel=wsel, rsel=rsel, fenc=fenc, denc=denc)


# ------------------------------------------------------------------ serving
def serving_trace(clients: int = 64, rate: float = 50.0, duration: float = 10.0,
                  gmin: int = 100, gmax: int = 20000, seed: int = 15):
    """Poisson arrivals of random layered circuits from `clients` clients.

    Circuit size G ~ log-uniform[gmin, gmax]; depth max(2, round(sqrt(G)/2)); level widths
    proportional to U[0.5, 1.5]; primary inputs = width of the first level; wiring as in
    the layered DAG. Returns a list of dicts sorted by arrival time.
    """
    g = rng(seed)
    t = 0.0
    reqs = []
    while True:
        t += g.exponential(1.0 / rate)
        if t > duration:
            break
        G = int(round(np.exp(g.uniform(np.log(gmin), np.log(gmax)))))
        depth = max(2, int(round(np.sqrt(G) / 2)))
        wts = g.uniform(0.5, 1.5, size=depth)
        widths = np.maximum(1, np.floor(wts / wts.sum() * G)).astype(np.int64)
        widths[-1] += G - int(widths.sum())
        if widths[-1] < 1:
            widths[-1] = 1
        ninputs = max(2, int(widths[0]))
        gates, level = layered_circuit(g, ninputs, widths)
        bits = g.integers(0, 2, size=ninputs, dtype=np.uint8)
        reqs.append(dict(t=t, client=int(g.integers(0, clients)), ninputs=ninputs,
                         gates=gates, level=level, bits=bits,
                         enc_seed=int(g.integers(0, 2 ** 31))))
    return reqs

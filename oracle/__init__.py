"""Python binding of the CPU oracle (``liboracle.so``, built from ``oracle.c``).

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` import this package. The GPU library never does, and this package
imports nothing from it.

Each wrapper marshals numpy arrays to the C oracle; the arithmetic is all in ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

# Gate opcodes (the library's C ABI numbering).
NAND, AND, OR, NOR, XOR, XNOR, ANDNOT, ORNOT, NOT = range(9)
MU = 1 << 29


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (portable x86-64 + AVX2 code, pthreads)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O3", "-mavx2", "-std=c11", "-Wall", "-fPIC", "-shared", "-pthread",
               "-o", _SO + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("N", ctypes.c_int32), ("l", ctypes.c_int32),
                ("bgbit", ctypes.c_int32), ("t", ctypes.c_int32), ("basebit", ctypes.c_int32)]

    def __repr__(self):
        return f"Params(n={self.n}, N={self.N}, l={self.l}, bgbit={self.bgbit}, t={self.t}, basebit={self.basebit})"


DEFAULT = Params(630, 1024, 3, 6, 8, 2)


class Params2(ctypes.Structure):
    """Level-2 parameters of circuit bootstrapping: ring degree, gadget rows and base bits on
    the 2^64 torus, private key-switch digits and base bits."""
    _fields_ = [("N", ctypes.c_int32), ("l", ctypes.c_int32), ("bgbit", ctypes.c_int32),
                ("t", ctypes.c_int32), ("basebit", ctypes.c_int32)]

    def __repr__(self):
        return f"Params2(N={self.N}, l={self.l}, bgbit={self.bgbit}, t={self.t}, basebit={self.basebit})"


DEFAULT2 = Params2(2048, 4, 9, 12, 2)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_SO)
        _declare(_lib)
    return _lib


_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_P = ctypes.POINTER(Params)
_Q = ctypes.POINTER(Params2)
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_c = ctypes


def _declare(L):
    sig = {
        "or_polymul": (None, [_c.c_int, _u32p, _u32p, _u32p]),
        "or_rotate": (None, [_c.c_int, _u32p, _c.c_uint32, _u32p]),
        "or_tlwe_encrypt_torus": (None, [_c.c_int, _u32p, _u32p, _c.c_int32, _c.c_uint32, _u32p]),
        "or_tlwe_encrypt_bit": (None, [_c.c_int, _u32p, _u32p, _c.c_int32, _c.c_int, _u32p]),
        "or_tlwe_phase": (_c.c_uint32, [_c.c_int, _u32p, _u32p]),
        "or_tlwe_decrypt": (_c.c_int, [_c.c_int, _u32p, _u32p]),
        "or_trlwe_encrypt_torus": (None, [_c.c_int, _u32p, _u32p, _i32p, _u32p, _u32p]),
        "or_trlwe_encrypt_bits": (None, [_c.c_int, _u32p, _u32p, _i32p, _u8p, _u32p]),
        "or_trlwe_phase": (None, [_c.c_int, _u32p, _u32p, _u32p]),
        "or_trgsw_encrypt": (None, [_P, _u32p, _u32p, _i32p, _c.c_int, _u32p]),
        "or_trgsw_gadget": (None, [_P, _u32p]),
        "or_bk_gen": (None, [_P, _u32p, _u32p, _u32p, _i32p, _u32p, _c.c_int]),
        "or_ksk_gen": (None, [_P, _u32p, _u32p, _u32p, _i32p, _u32p]),
        "or_decompose": (None, [_P, _c.c_uint32, _i32p]),
        "or_modswitch": (_c.c_uint32, [_c.c_uint32, _c.c_int]),
        "or_external_product": (None, [_P, _u32p, _u32p, _u32p]),
        "or_cmux": (None, [_P, _u32p, _u32p, _u32p, _u32p]),
        "or_blind_rotate": (None, [_P, _u32p, _u32p, _u32p, _u32p]),
        "or_sample_extract": (None, [_c.c_int, _u32p, _c.c_int, _u32p]),
        "or_keyswitch": (None, [_P, _u32p, _u32p, _u32p]),
        "or_ks_digits": (None, [_P, _c.c_uint32, _u32p]),
        "or_gate_linear": (_c.c_int, [_c.c_int, _c.c_int, _u32p, _u32p, _u32p]),
        "or_bootstrap_to_trlwe": (None, [_P, _u32p, _u32p, _u32p]),
        "or_gate": (None, [_P, _u32p, _u32p, _c.c_int, _u32p, _u32p, _u32p]),
        "or_gates": (None, [_P, _u32p, _u32p, _u8p, _u32p, _u32p, _u32p, _c.c_int64, _c.c_int]),
        "or_mux": (None, [_P, _u32p, _u32p, _u32p, _u32p, _u32p, _u32p]),
        "or_muxes": (None, [_P, _u32p, _u32p, _u32p, _u32p, _u32p, _u32p, _c.c_int64, _c.c_int]),
        "or_rom_read": (None, [_P, _u32p, _u32p, _c.c_int, _u32p, _c.c_int, _c.c_int, _u32p]),
        "or_ram_read": (None, [_P, _u32p, _u32p, _c.c_int, _c.c_int, _u32p, _u32p]),
        "or_ram_control": (None, [_P, _u32p, _u32p, _u32p, _u32p, _c.c_int, _u32p]),
        "or_ram_write_bars": (None, [_P, _u32p, _u32p, _u32p, _c.c_int, _u32p, _u32p, _i64p,
                                     _c.c_int64, _u32p, _c.c_int]),
        "or_ram_write": (None, [_P, _u32p, _u32p, _u32p, _c.c_int, _c.c_int, _u32p, _u32p,
                                _u32p, _c.c_int]),
        "or_rom_reads": (None, [_P, _u32p, _u32p, _c.c_int, _u32p, _c.c_int, _c.c_int, _u32p,
                                _c.c_int64, _c.c_int]),
        "or_ram_reads": (None, [_P, _u32p, _u32p, _c.c_int, _c.c_int, _u32p, _u32p, _c.c_int64, _c.c_int]),
        "or_polymul64": (None, [_c.c_int, _u64p, _u64p, _u64p]),
        "or_rotate64": (None, [_c.c_int, _u64p, _c.c_uint32, _u64p]),
        "or_trlwe64_encrypt_torus": (None, [_c.c_int, _u64p, _u64p, _i64p, _u64p, _u64p]),
        "or_trlwe64_phase": (None, [_c.c_int, _u64p, _u64p, _u64p]),
        "or_trgsw64_encrypt": (None, [_Q, _u64p, _u64p, _i64p, _c.c_int, _u64p]),
        "or_bk2_gen": (None, [_c.c_int, _Q, _u32p, _u64p, _u64p, _i64p, _u64p, _c.c_int]),
        "or_decompose64": (None, [_Q, _c.c_uint64, _i64p]),
        "or_external_product64": (None, [_Q, _u64p, _u64p, _u64p]),
        "or_blind_rotate64": (None, [_c.c_int, _Q, _u64p, _u32p, _u64p, _u64p]),
        "or_sample_extract64": (None, [_c.c_int, _u64p, _u64p]),
        "or_pksk_gen": (None, [_P, _Q, _u32p, _u64p, _u32p, _i32p, _u32p, _c.c_int]),
        "or_private_keyswitch": (None, [_P, _Q, _u32p, _c.c_int, _u64p, _u32p]),
        "or_circuit_bootstrap": (None, [_P, _Q, _u64p, _u32p, _u32p, _u32p]),
        "or_circuit_bootstraps": (None, [_P, _Q, _u64p, _u32p, _u32p, _u32p, _c.c_int64, _c.c_int]),
        "or_cmux_count": (_c.c_uint64, []),
        "or_br_count": (_c.c_uint64, []),
        "or_reset_counters": (None, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _u32(x):
    return np.ascontiguousarray(x, dtype=np.uint32)


def _i32(x):
    return np.ascontiguousarray(x, dtype=np.int32)


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


# ----------------------------------------------------------------- polynomials
def polymul(a, b):
    a, b = _u32(a), _u32(b)
    out = np.zeros_like(a)
    lib().or_polymul(a.size, a, b, out)
    return out


def rotate(p, k):
    p = _u32(p)
    out = np.zeros_like(p)
    lib().or_rotate(p.size, p, int(k) % (2 * p.size), out)
    return out


# ----------------------------------------------------------------- encryption
def tlwe_encrypt_bits(s, bits, masks, noise):
    s, masks, noise = _u32(s), _u32(masks), _i32(noise)
    n = s.size
    bits = np.asarray(bits).reshape(-1)
    out = np.zeros((bits.size, n + 1), dtype=np.uint32)
    for k in range(bits.size):
        row = out[k]
        lib().or_tlwe_encrypt_bit(n, s, masks[k], int(noise[k]), int(bits[k]), row)
    return out


def tlwe_encrypt_torus(s, m, a, e):
    s, a = _u32(s), _u32(a)
    out = np.zeros(s.size + 1, dtype=np.uint32)
    lib().or_tlwe_encrypt_torus(s.size, s, a, int(e), int(m) & 0xFFFFFFFF, out)
    return out


def tlwe_phase(s, c):
    s, c = _u32(s), _u32(c)
    if c.ndim == 1:
        return np.uint32(lib().or_tlwe_phase(s.size, s, c))
    return np.array([lib().or_tlwe_phase(s.size, s, _u32(row)) for row in c], dtype=np.uint32)


def tlwe_decrypt(s, c):
    ph = tlwe_phase(s, c)
    return (np.asarray(ph).view(np.int32) >= 0).astype(np.uint8)


def trlwe_encrypt_bits(s, bits, a, e):
    s, a, e = _u32(s), _u32(a), _i32(e)
    out = np.zeros(2 * s.size, dtype=np.uint32)
    lib().or_trlwe_encrypt_bits(s.size, s, a, e, np.ascontiguousarray(bits, dtype=np.uint8), out)
    return out.reshape(2, s.size)


def trlwe_encrypt_torus(s, m, a, e):
    s, a, e, m = _u32(s), _u32(a), _i32(e), _u32(m)
    out = np.zeros(2 * s.size, dtype=np.uint32)
    lib().or_trlwe_encrypt_torus(s.size, s, a, e, m, out)
    return out.reshape(2, s.size)


def trlwe_phase(s, c):
    s, c = _u32(s), _u32(c)
    out = np.zeros(s.size, dtype=np.uint32)
    lib().or_trlwe_phase(s.size, s, c.reshape(-1), out)
    return out


def trgsw_encrypt(s, m, masks, noise, P=DEFAULT):
    s, masks, noise = _u32(s), _u32(masks), _i32(noise)
    out = np.zeros((2 * P.l, 2, P.N), dtype=np.uint32)
    lib().or_trgsw_encrypt(ctypes.byref(P), s, masks.reshape(-1), noise.reshape(-1), int(m), out.reshape(-1))
    return out


def trgsw_gadget(P=DEFAULT):
    out = np.zeros((2 * P.l, 2, P.N), dtype=np.uint32)
    lib().or_trgsw_gadget(ctypes.byref(P), out.reshape(-1))
    return out


def bk_gen(s0, s1, masks, noise, P=DEFAULT, threads=None):
    s0, s1, masks, noise = _u32(s0), _u32(s1), _u32(masks), _i32(noise)
    out = np.zeros((P.n, 2 * P.l, 2, P.N), dtype=np.uint32)
    lib().or_bk_gen(ctypes.byref(P), s0, s1, masks.reshape(-1), noise.reshape(-1), out.reshape(-1),
                    threads or default_threads())
    return out


def ksk_gen(s0, s1, masks, noise, P=DEFAULT):
    s0, s1, masks, noise = _u32(s0), _u32(s1), _u32(masks), _i32(noise)
    base = 1 << P.basebit
    out = np.zeros((P.N, P.t, base - 1, P.n + 1), dtype=np.uint32)
    lib().or_ksk_gen(ctypes.byref(P), s0, s1, masks.reshape(-1), noise.reshape(-1), out.reshape(-1))
    return out


# ----------------------------------------------------------------- steps
def decompose(x, P=DEFAULT):
    d = np.zeros(16, dtype=np.int32)
    lib().or_decompose(ctypes.byref(P), int(x) & 0xFFFFFFFF, d)
    return d[:P.l].copy()


def modswitch(x, N=1024):
    return int(lib().or_modswitch(int(x) & 0xFFFFFFFF, N))


def ks_digits(a, P=DEFAULT):
    v = np.zeros(64, dtype=np.uint32)
    lib().or_ks_digits(ctypes.byref(P), int(a) & 0xFFFFFFFF, v)
    return v[:P.t].copy()


def external_product(C, x, P=DEFAULT):
    out = np.zeros((2, P.N), dtype=np.uint32)
    lib().or_external_product(ctypes.byref(P), _u32(C).reshape(-1), _u32(x).reshape(-1), out.reshape(-1))
    return out


def cmux(C, x0, x1, P=DEFAULT):
    out = np.zeros((2, P.N), dtype=np.uint32)
    lib().or_cmux(ctypes.byref(P), _u32(C).reshape(-1), _u32(x0).reshape(-1), _u32(x1).reshape(-1),
                  out.reshape(-1))
    return out


def blind_rotate(bk, c, tv, P=DEFAULT):
    out = np.zeros((2, P.N), dtype=np.uint32)
    lib().or_blind_rotate(ctypes.byref(P), _u32(bk).reshape(-1), _u32(c), _u32(tv), out.reshape(-1))
    return out


def sample_extract(c, h=0):
    c = _u32(c).reshape(-1)
    N = c.size // 2
    out = np.zeros(N + 1, dtype=np.uint32)
    lib().or_sample_extract(N, c, int(h), out)
    return out


def keyswitch(ksk, c, P=DEFAULT):
    out = np.zeros(P.n + 1, dtype=np.uint32)
    lib().or_keyswitch(ctypes.byref(P), _u32(ksk).reshape(-1), _u32(c), out)
    return out


def gate_linear(op, c1, c2):
    c1, c2 = _u32(c1), _u32(c2)
    out = np.zeros_like(c1)
    boot = lib().or_gate_linear(c1.size - 1, int(op), c1, c2, out)
    return out, bool(boot)


def bootstrap_to_trlwe(bk, c, P=DEFAULT):
    out = np.zeros((2, P.N), dtype=np.uint32)
    lib().or_bootstrap_to_trlwe(ctypes.byref(P), _u32(bk).reshape(-1), _u32(c), out.reshape(-1))
    return out


def gate(bk, ksk, op, c1, c2, P=DEFAULT):
    out = np.zeros(P.n + 1, dtype=np.uint32)
    lib().or_gate(ctypes.byref(P), _u32(bk).reshape(-1), _u32(ksk).reshape(-1), int(op), _u32(c1), _u32(c2), out)
    return out


def gates(bk, ksk, ops, in0, in1, P=DEFAULT, threads=None):
    ops = np.ascontiguousarray(ops, dtype=np.uint8)
    B = ops.size
    out = np.zeros((B, P.n + 1), dtype=np.uint32)
    lib().or_gates(ctypes.byref(P), _u32(bk).reshape(-1), _u32(ksk).reshape(-1), ops,
                   _u32(in0).reshape(-1), _u32(in1).reshape(-1), out.reshape(-1), B,
                   threads or default_threads())
    return out


def muxes(bk, ksk, s, c1, c0, P=DEFAULT, threads=None):
    """Homomorphic MUX s ? c1 : c0 over B rows of TLWE inputs."""
    s = _u32(s)
    B = s.shape[0]
    out = np.zeros((B, P.n + 1), dtype=np.uint32)
    lib().or_muxes(ctypes.byref(P), _u32(bk).reshape(-1), _u32(ksk).reshape(-1), s.reshape(-1),
                   _u32(c1).reshape(-1), _u32(c0).reshape(-1), out.reshape(-1), B, threads or default_threads())
    return out


# ----------------------------------------------------------------- CMUX memory
def rom_read(ksk, rom, sel, wbits=32, P=DEFAULT):
    rom = _u32(rom)
    npoly = rom.shape[0]
    abits = sel.shape[0]
    out = np.zeros((wbits, P.n + 1), dtype=np.uint32)
    lib().or_rom_read(ctypes.byref(P), _u32(ksk).reshape(-1), rom.reshape(-1), npoly,
                      _u32(sel).reshape(-1), abits, wbits, out.reshape(-1))
    return out


def rom_reads(ksk, rom, sels, wbits=32, P=DEFAULT, threads=None):
    """Independent ROM reads; sels is [R][abits][2l][2][N]."""
    rom, sels = _u32(rom), _u32(sels)
    R, abits = sels.shape[0], sels.shape[1]
    out = np.zeros((R, wbits, P.n + 1), dtype=np.uint32)
    lib().or_rom_reads(ctypes.byref(P), _u32(ksk).reshape(-1), rom.reshape(-1), rom.shape[0], sels.reshape(-1),
                       abits, wbits, out.reshape(-1), R, threads or default_threads())
    return out


def ram_reads(ksk, ram, sels, P=DEFAULT, threads=None):
    """Independent RAM reads; sels is [R][v][2l][2][N]."""
    ram, sels = _u32(ram), _u32(sels)
    w, cells = ram.shape[0], ram.shape[1]
    v = int(cells).bit_length() - 1
    R = sels.shape[0]
    out = np.zeros((R, w, P.n + 1), dtype=np.uint32)
    lib().or_ram_reads(ctypes.byref(P), _u32(ksk).reshape(-1), ram.reshape(-1), v, w, sels.reshape(-1),
                       out.reshape(-1), R, threads or default_threads())
    return out


def ram_read(ksk, ram, sel, P=DEFAULT):
    ram = _u32(ram)
    w, cells = ram.shape[0], ram.shape[1]
    v = int(cells).bit_length() - 1
    out = np.zeros((w, P.n + 1), dtype=np.uint32)
    lib().or_ram_read(ctypes.byref(P), _u32(ksk).reshape(-1), ram.reshape(-1), v, w,
                      _u32(sel).reshape(-1), out.reshape(-1))
    return out


def ram_control(bk, flag, data, rd, P=DEFAULT):
    data, rd = _u32(data), _u32(rd)
    w = data.shape[0]
    out = np.zeros((w, 2, P.N), dtype=np.uint32)
    lib().or_ram_control(ctypes.byref(P), _u32(bk).reshape(-1), _u32(flag), data.reshape(-1),
                         rd.reshape(-1), w, out.reshape(-1))
    return out


def ram_write_bars(bk, ksk, ram, sel, u, idx, P=DEFAULT, threads=None):
    ram = _u32(ram)
    v = int(ram.shape[1]).bit_length() - 1
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros((idx.size, 2, P.N), dtype=np.uint32)
    lib().or_ram_write_bars(ctypes.byref(P), _u32(bk).reshape(-1), _u32(ksk).reshape(-1), ram.reshape(-1), v,
                            _u32(sel).reshape(-1), _u32(u).reshape(-1), idx, idx.size, out.reshape(-1),
                            threads or default_threads())
    return out


def ram_write(bk, ksk, ram, sel, flag, data, P=DEFAULT, threads=None):
    ram = np.array(ram, dtype=np.uint32, copy=True, order="C")
    w, cells = ram.shape[0], ram.shape[1]
    v = int(cells).bit_length() - 1
    lib().or_ram_write(ctypes.byref(P), _u32(bk).reshape(-1), _u32(ksk).reshape(-1), ram.reshape(-1), v, w,
                       _u32(sel).reshape(-1), _u32(flag), _u32(data).reshape(-1),
                       threads or default_threads())
    return ram


def cmux_count() -> int:
    """CMUX gates evaluated by the memory units since the last reset."""
    return int(lib().or_cmux_count())


def br_count() -> int:
    """Blind rotations since the last reset."""
    return int(lib().or_br_count())


def reset_counters() -> None:
    lib().or_reset_counters()


# ----------------------------------------------------------------- key sets
def keyset(s0, s1, bkd, kskd, P=DEFAULT, threads=None):
    """Bootstrapping key and key-switching key from the given draws."""
    bk = bk_gen(s0, s1, bkd[0], bkd[1], P, threads)
    ksk = ksk_gen(s0, s1, kskd[0], kskd[1], P)
    return bk, ksk


# ----------------------------------------------------------------- circuit bootstrapping
def _u64(x):
    return np.ascontiguousarray(x, dtype=np.uint64)


def _i64(x):
    return np.ascontiguousarray(x, dtype=np.int64)


def polymul64(a, b):
    """Negacyclic product mod 2^64 (schoolbook)."""
    a, b = _u64(a), _u64(b)
    out = np.zeros_like(a)
    lib().or_polymul64(a.size, a, b, out)
    return out


def rotate64(p, k):
    p = _u64(p)
    out = np.zeros_like(p)
    lib().or_rotate64(p.size, p, int(k) % (2 * p.size), out)
    return out


def trlwe64_encrypt_torus(s2, m, a, e):
    a = _u64(a)
    out = np.zeros(2 * a.size, dtype=np.uint64)
    lib().or_trlwe64_encrypt_torus(a.size, _u64(s2), a, _i64(e), _u64(m), out)
    return out.reshape(2, -1)


def trlwe64_phase(s2, c):
    c = _u64(c).reshape(-1)
    out = np.zeros(c.size // 2, dtype=np.uint64)
    lib().or_trlwe64_phase(c.size // 2, _u64(s2), c, out)
    return out


def trgsw64_encrypt(s2, m, masks, noise, Q=DEFAULT2):
    out = np.zeros((2 * Q.l, 2, Q.N), dtype=np.uint64)
    lib().or_trgsw64_encrypt(ctypes.byref(Q), _u64(s2), _u64(masks).reshape(-1), _i64(noise).reshape(-1), int(m),
                             out.reshape(-1))
    return out


def bk2_gen(s0, s2, masks, noise, Q=DEFAULT2, threads=None):
    """Level-2 bootstrapping key [n][2 l2][2][N2]: BK2[i] = TRGSW2_{s2}(s0[i])."""
    n = len(s0)
    out = np.zeros((n, 2 * Q.l, 2, Q.N), dtype=np.uint64)
    lib().or_bk2_gen(n, ctypes.byref(Q), _u32(s0), _u64(s2), _u64(masks).reshape(-1), _i64(noise).reshape(-1),
                     out.reshape(-1), threads or default_threads())
    return out


def decompose64(x, Q=DEFAULT2):
    d = np.zeros(16, dtype=np.int64)
    lib().or_decompose64(ctypes.byref(Q), int(x) & 0xFFFFFFFFFFFFFFFF, d)
    return d[:Q.l].copy()


def external_product64(C, x, Q=DEFAULT2):
    out = np.zeros((2, Q.N), dtype=np.uint64)
    lib().or_external_product64(ctypes.byref(Q), _u64(C).reshape(-1), _u64(x).reshape(-1), out.reshape(-1))
    return out


def blind_rotate64(bk2, c, tv, Q=DEFAULT2):
    c = _u32(c)
    out = np.zeros((2, Q.N), dtype=np.uint64)
    lib().or_blind_rotate64(c.size - 1, ctypes.byref(Q), _u64(bk2).reshape(-1), c, _u64(tv), out.reshape(-1))
    return out


def sample_extract64(c):
    c = _u64(c).reshape(-1)
    N = c.size // 2
    out = np.zeros(N + 1, dtype=np.uint64)
    lib().or_sample_extract64(N, c, out)
    return out


def pksk_gen(s1, s2, masks, noise, P=DEFAULT, Q=DEFAULT2, threads=None):
    """Private functional key-switching keys [2][N2+1][t2][base2-1][2][N]: function 0 is
    x -> -s1 x, function 1 is x -> x."""
    base = 1 << Q.basebit
    out = np.zeros((2, Q.N + 1, Q.t, base - 1, 2, P.N), dtype=np.uint32)
    lib().or_pksk_gen(ctypes.byref(P), ctypes.byref(Q), _u32(s1), _u64(s2), _u32(masks).reshape(-1),
                      _i32(noise).reshape(-1), out.reshape(-1), threads or default_threads())
    return out


def private_keyswitch(pksk, u, c, P=DEFAULT, Q=DEFAULT2):
    out = np.zeros((2, P.N), dtype=np.uint32)
    lib().or_private_keyswitch(ctypes.byref(P), ctypes.byref(Q), _u32(pksk).reshape(-1), int(u), _u64(c),
                               out.reshape(-1))
    return out


def circuit_bootstrap(bk2, pksk, c, P=DEFAULT, Q=DEFAULT2):
    """Level-0 TLWE of a bit -> level-1 TRGSW [2l][2][N] of that bit."""
    out = np.zeros((2 * P.l, 2, P.N), dtype=np.uint32)
    lib().or_circuit_bootstrap(ctypes.byref(P), ctypes.byref(Q), _u64(bk2).reshape(-1), _u32(pksk).reshape(-1),
                               _u32(c), out.reshape(-1))
    return out


def circuit_bootstraps(bk2, pksk, cs, P=DEFAULT, Q=DEFAULT2, threads=None):
    cs = _u32(cs)
    R = cs.shape[0]
    out = np.zeros((R, 2 * P.l, 2, P.N), dtype=np.uint32)
    lib().or_circuit_bootstraps(ctypes.byref(P), ctypes.byref(Q), _u64(bk2).reshape(-1), _u32(pksk).reshape(-1),
                                cs.reshape(-1), out.reshape(-1), R, threads or default_threads())
    return out


def keyset2(s0, s1, s2, bk2d, pkskd, P=DEFAULT, Q=DEFAULT2, threads=None):
    """Circuit-bootstrapping keys from the given draws: (level-2 bootstrapping key, private
    key-switching keys)."""
    return bk2_gen(s0, s2, bk2d[0], bk2d[1], Q, threads), pksk_gen(s1, s2, pkskd[0], pkskd[1], P, Q, threads)

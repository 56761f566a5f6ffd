"""Client side of the protocol (the party that owns the secret keys): key generation,
encryption and decryption with numpy (Sec. 2.1.2, TLWE / TRLWE / TRGSW).

The server-side library never sees secret keys; it receives the bootstrapping key, the
key-switching key and ciphertexts produced here. Random draws (keys, masks, noise) are
inputs, produced by the seeded generators in ``workloads``.

Torus elements are uint32 (arithmetic mod 2^32). Products a(X) s(X) with a binary key s
in Z[X]/(X^N+1) are computed exactly as float64 matrix products on 16-bit limbs: every
partial sum is an integer below 2^26 in magnitude, so the floating-point result is exact.
"""
from __future__ import annotations

import numpy as np

MU = np.uint32(1 << 29)            # 1/8
NEG_MU = np.uint32((1 << 32) - (1 << 29))  # -1/8
N_LWE, N_RING, L, BG_BIT, KS_T, KS_BASEBIT = 630, 1024, 3, 6, 8, 2
M32 = (1 << 32) - 1


def _negacyclic_matrix(s: np.ndarray) -> np.ndarray:
    """M with (a @ M)[k] = (a(X) s(X) mod X^N + 1)[k] for a binary (0/1) key s."""
    N = s.size
    M = np.zeros((N, N), dtype=np.float64)
    sf = s.astype(np.float64)
    for i in range(N):
        # row i: X^i s(X): coefficient k takes s[k - i] (k >= i) or -s[k - i + N] (k < i)
        M[i, i:] = sf[: N - i]
        M[i, :i] = -sf[N - i:]
    return M


def mul_by_key(a: np.ndarray, s: np.ndarray) -> np.ndarray:
    """a(X) s(X) mod (X^N + 1, 2^32) for rows a [..., N] (uint32) and a binary key s [N]."""
    a = np.asarray(a, dtype=np.uint32)
    shape = a.shape
    a2 = a.reshape(-1, shape[-1])
    M = _negacyclic_matrix(np.asarray(s))
    lo = (a2 & 0xFFFF).astype(np.float64) @ M
    hi = (a2 >> 16).astype(np.float64) @ M
    r = (np.rint(lo).astype(np.int64) + (np.rint(hi).astype(np.int64) << 16)) & M32
    return r.astype(np.uint32).reshape(shape)


def dot_key(a: np.ndarray, s: np.ndarray) -> np.ndarray:
    """<a, s> mod 2^32 for rows a [..., n] and a binary key s [n]."""
    a = np.asarray(a, dtype=np.uint32)
    sf = np.asarray(s).astype(np.float64)
    lo = (a & 0xFFFF).astype(np.float64) @ sf
    hi = (a >> 16).astype(np.float64) @ sf
    return ((np.rint(lo).astype(np.int64) + (np.rint(hi).astype(np.int64) << 16)) & M32).astype(np.uint32)


def _u32(x) -> np.ndarray:
    return (np.asarray(x).astype(np.int64) & M32).astype(np.uint32)


# ------------------------------------------------------------------ TLWE
def bit_to_torus(bits) -> np.ndarray:
    """mu(2m - 1): +1/8 for 1, -1/8 for 0."""
    return np.where(np.asarray(bits) != 0, MU, NEG_MU).astype(np.uint32)


def tlwe_encrypt_torus(s0, m, masks, noise) -> np.ndarray:
    """TLWE (a, <a, s> + m + e) for torus messages m [B]; masks [B][n], noise [B]."""
    masks = np.asarray(masks, dtype=np.uint32)
    b = dot_key(masks, s0).astype(np.uint64) + _u32(m) + _u32(noise)
    return np.concatenate([masks, (b & M32).astype(np.uint32)[..., None]], axis=-1)


def tlwe_encrypt_bits(s0, bits, masks, noise) -> np.ndarray:
    return tlwe_encrypt_torus(s0, bit_to_torus(bits), masks, noise)


def trivial_tlwe_bits(bits, n: int = N_LWE) -> np.ndarray:
    """Noise-free, mask-free ciphertexts (0, mu(2m - 1)) (public constants)."""
    bits = np.asarray(bits)
    c = np.zeros(bits.shape + (n + 1,), dtype=np.uint32)
    c[..., n] = bit_to_torus(bits)
    return c


def tlwe_phase(s, c) -> np.ndarray:
    c = np.asarray(c, dtype=np.uint32)
    return ((c[..., -1].astype(np.int64) - dot_key(c[..., :-1], s).astype(np.int64)) & M32).astype(np.uint32)


def tlwe_decrypt(s, c) -> np.ndarray:
    """(1 + sgn(phase)) / 2 with phase 0 read as positive."""
    return (tlwe_phase(s, c).view(np.int32) >= 0).astype(np.uint8)


# ------------------------------------------------------------------ TRLWE / TRGSW
def trlwe_encrypt_torus(s1, m, masks, noise) -> np.ndarray:
    """TRLWE (a, a s + m + e) for torus message polynomials m [..., N]."""
    masks = np.asarray(masks, dtype=np.uint32)
    b = (mul_by_key(masks, s1).astype(np.uint64) + _u32(m) + _u32(noise)) & M32
    return np.stack([masks, b.astype(np.uint32)], axis=-2)


def trlwe_phase(s1, c) -> np.ndarray:
    c = np.asarray(c, dtype=np.uint32)
    return ((c[..., 1, :].astype(np.int64) - mul_by_key(c[..., 0, :], s1).astype(np.int64)) & M32).astype(np.uint32)


def trgsw_encrypt(s1, m, masks, noise) -> np.ndarray:
    """TRGSW of bits m [...]: 2l TRLWE encryptions of zero; rows r < l add m / Bg^(r+1) to the
    constant coefficient of a, rows r >= l add m / Bg^(r-l+1) to that of b.
    masks, noise [..., 2l, N] -> [..., 2l, 2, N]."""
    masks = np.asarray(masks, dtype=np.uint32)
    C = trlwe_encrypt_torus(s1, np.zeros_like(masks), masks, noise)
    m = np.asarray(m, dtype=np.uint64)
    for r in range(L):
        g = np.uint64(1 << (32 - BG_BIT * (r + 1)))
        C[..., r, 0, 0] = ((C[..., r, 0, 0].astype(np.uint64) + m * g) & M32).astype(np.uint32)
        C[..., L + r, 1, 0] = ((C[..., L + r, 1, 0].astype(np.uint64) + m * g) & M32).astype(np.uint32)
    return C


def trivial_trgsw(m, N: int = N_RING) -> np.ndarray:
    """Noise-free, mask-free TRGSW of bits m (m times the gadget G)."""
    m = np.asarray(m, dtype=np.uint32)
    C = np.zeros(m.shape + (2 * L, 2, N), dtype=np.uint32)
    for r in range(L):
        g = np.uint32(1 << (32 - BG_BIT * (r + 1)))
        C[..., r, 0, 0] = m * g
        C[..., L + r, 1, 0] = m * g
    return C


# ------------------------------------------------------------------ keys
def bootstrapping_key(s0, s1, masks, noise) -> np.ndarray:
    """BK[i] = TRGSW_{s1}(s0[i]): [n][2l][2][N]."""
    return trgsw_encrypt(s1, np.asarray(s0), masks, noise)


def keyswitching_key(s0, s1, masks, noise) -> np.ndarray:
    """KSK[j][p][v-1] = TLWE_{s0}(v s1[j] / 4^(p+1)): [N][t][3][n+1]."""
    N, t, B1 = masks.shape[0], masks.shape[1], masks.shape[2]
    v = np.arange(1, B1 + 1, dtype=np.uint64)[None, None, :]
    p = np.arange(t, dtype=np.uint64)[None, :, None]
    m = (np.asarray(s1, dtype=np.uint64)[:, None, None] * v * (np.uint64(1) << (np.uint64(32) - KS_BASEBIT * (p + 1)))) & M32
    return tlwe_encrypt_torus(s0, m.astype(np.uint32), masks, noise)


def keyset(s0, s1, bkd, kskd):
    return bootstrapping_key(s0, s1, *bkd), keyswitching_key(s0, s1, *kskd)


# ------------------------------------------------------------------ memory encodings
def pack_rom(words, wbits: int = 32, N: int = N_RING) -> np.ndarray:
    """ROM plaintext polynomials (vertical + horizontal packing): coefficient wbits*q + b of
    polynomial h holds bit b of word (N / wbits) h + q, encoded mu(2m - 1)."""
    words = np.asarray(words, dtype=np.uint64)
    per = N // wbits
    bits = (words[:, None] >> np.arange(wbits, dtype=np.uint64)[None, :]) & 1   # [W][wbits]
    return bit_to_torus(bits.reshape(-1, per * wbits))


def ram_cell_messages(contents, N: int = N_RING) -> np.ndarray:
    """RAM cell messages m X^0 for bits contents [w][2^v]: constant coefficient mu(2m - 1), the
    other coefficients -mu (one bit per TRLWE, the read unit's layout)."""
    contents = np.asarray(contents)
    msg = np.full(contents.shape + (N,), NEG_MU, dtype=np.uint32)
    msg[..., 0] = bit_to_torus(contents)
    return msg


# ------------------------------------------------------------------ circuit bootstrapping keys
# Level 2 (the conversion TLWE -> TRGSW of Sec. 2.1.2 "Circuit Bootstrapping"): a binary key
# s2 of degree N2 over the 2^64 torus, BK2[i] = TRGSW2_{s2}(s0[i]) with an l2 x 2^bg2 gadget,
# and two private functional key-switching keys to level-1 TRLWE under s1.
N2, L2, BG_BIT2, PKS_T, PKS_BASEBIT = 2048, 4, 9, 12, 2
M64 = (1 << 64) - 1


def mul_by_key64(a: np.ndarray, s: np.ndarray) -> np.ndarray:
    """a(X) s(X) mod (X^N + 1, 2^64) for rows a [..., N] (uint64) and a binary key s [N], as
    float64 matrix products on four 16-bit limbs (partial sums below 2^27: exact)."""
    a = np.asarray(a, dtype=np.uint64)
    shape = a.shape
    a2 = a.reshape(-1, shape[-1])
    M = _negacyclic_matrix(np.asarray(s))
    r = np.zeros(a2.shape, dtype=np.uint64)
    for q in range(4):
        limb = ((a2 >> np.uint64(16 * q)) & np.uint64(0xFFFF)).astype(np.float64)
        part = np.rint(limb @ M).astype(np.int64).astype(np.uint64)   # two's complement mod 2^64
        r += part << np.uint64(16 * q)
    return r.reshape(shape)


def trlwe64_encrypt_torus(s2, m, masks, noise) -> np.ndarray:
    masks = np.asarray(masks, dtype=np.uint64)
    b = mul_by_key64(masks, s2) + np.asarray(m, dtype=np.uint64) + np.asarray(noise).astype(np.int64).astype(np.uint64)
    return np.stack([masks, b], axis=-2)


def trgsw64_encrypt(s2, m, masks, noise) -> np.ndarray:
    """Level-2 TRGSW of bits m [...]: masks, noise [..., 2 l2, N2] -> [..., 2 l2, 2, N2] (rows as
    trgsw_encrypt, gadget entries 2^(64 - bg2 (r+1)))."""
    masks = np.asarray(masks, dtype=np.uint64)
    C = trlwe64_encrypt_torus(s2, np.zeros_like(masks), masks, noise)
    m = np.asarray(m, dtype=np.uint64)
    for r in range(L2):
        g = np.uint64(1 << (64 - BG_BIT2 * (r + 1)))
        C[..., r, 0, 0] += m * g
        C[..., L2 + r, 1, 0] += m * g
    return C


def private_keyswitching_keys(s1, s2, masks, noise, chunk: int = 8192) -> np.ndarray:
    """PKSK[u][k][p][v-1] = TRLWE_{s1}(f_u(v z_k / 4^(p+1))) with z = (-s2, 1), f_0(x) = -s1 x,
    f_1(x) = x: [2][N2+1][t][3][2][N] (uint32)."""
    masks = np.asarray(masks, dtype=np.uint32)
    _, K, t, B1, N = masks.shape
    z = np.concatenate([(-np.asarray(s2, dtype=np.int64)), np.ones(1, np.int64)]) & M32      # [K]
    v = np.arange(1, B1 + 1, dtype=np.uint64)
    sh = np.uint64(32) - np.uint64(PKS_BASEBIT) * (np.arange(t, dtype=np.uint64) + np.uint64(1))
    x = (z.astype(np.uint64)[:, None, None] * v[None, None, :] * (np.uint64(1) << sh)[None, :, None]) & M32  # [K][t][B1]
    out = np.empty(masks.shape[:-1] + (2, N), dtype=np.uint32)
    s1u = np.asarray(s1, dtype=np.uint64)
    for u in range(2):
        flat_m = masks[u].reshape(-1, N)
        flat_e = np.asarray(noise[u]).reshape(-1, N)
        flat_x = x.reshape(-1)
        dst = out[u].reshape(-1, 2, N)
        for lo in range(0, flat_m.shape[0], chunk):
            hi = min(lo + chunk, flat_m.shape[0])
            xs = flat_x[lo:hi].astype(np.uint64)
            if u == 0:
                msg = ((np.uint64(0) - s1u[None, :] * xs[:, None]) & M32).astype(np.uint32)
            else:
                msg = np.zeros((hi - lo, N), dtype=np.uint32)
                msg[:, 0] = xs.astype(np.uint32)
            dst[lo:hi] = trlwe_encrypt_torus(s1, msg, flat_m[lo:hi], flat_e[lo:hi])
    return out


def keyset2(s0, s1, s2, bk2d, pkskd):
    """(BK2 [n][2 l2][2][N2] uint64, PKSK [2][N2+1][t][3][2][N] uint32)."""
    return trgsw64_encrypt(s2, np.asarray(s0), *bk2d), private_keyswitching_keys(s1, s2, *pkskd)

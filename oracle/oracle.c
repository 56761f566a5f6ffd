/*
 * CPU oracle for TFHE gate bootstrapping and the CMUX-memory ROM/RAM.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load this library; the GPU library never does, and the two share no code.
 *
 * It is a plain, slow, obviously correct restatement of what the method computes:
 *   - the torus T = R/Z is discretised to Z/2^32 (uint32, arithmetic wraps mod 2^32);
 *   - every product in T_N[X] = T[X]/(X^N+1) is the schoolbook negacyclic definition;
 *   - encryption, the TRGSW gadget, the external product, CMUX, blind rotation, sample
 *     extraction, identity key switching and the homomorphic gates follow the paper's
 *     Sec. 2.1.2 and, where it delegates the algorithm to TFHE (Chillotti et al.,
 *     J. Cryptology 2020), the published TFHE algorithms, written from their definitions;
 *   - ROM/RAM reads and the RAM write follow Sec. 8 (CMUX Memory).
 * All random draws (keys, masks, noise) are inputs; nothing here draws randomness.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef struct {
  int32_t n;      /* TLWE dimension */
  int32_t N;      /* TRLWE degree (power of two) */
  int32_t l;      /* gadget rows per column */
  int32_t bgbit;  /* log2 of the gadget base Bg */
  int32_t t;      /* key-switch digits */
  int32_t basebit;/* log2 of the key-switch base */
} or_params;

/* Gate opcodes (same numbering as the library's C ABI). */
enum { OR_NAND = 0, OR_AND, OR_OR, OR_NOR, OR_XOR, OR_XNOR, OR_ANDNOT, OR_ORNOT, OR_NOT };

#define MU 0x20000000u /* mu = 1/8 on the 2^32 torus (Sec. 2.1.2 notation) */

/* Structural counters: CMUX gates evaluated by the memory units, and blind rotations. */
static uint64_t g_cmux_count = 0, g_br_count = 0;

uint64_t or_cmux_count(void) { return __atomic_load_n(&g_cmux_count, __ATOMIC_SEQ_CST); }
uint64_t or_br_count(void) { return __atomic_load_n(&g_br_count, __ATOMIC_SEQ_CST); }
void or_reset_counters(void) {
  __atomic_store_n(&g_cmux_count, 0, __ATOMIC_SEQ_CST);
  __atomic_store_n(&g_br_count, 0, __ATOMIC_SEQ_CST);
}

static void *xmalloc(size_t bytes) {
  void *p = calloc(bytes ? bytes : 1, 1);
  if (!p) abort();
  return p;
}

/* ------------------------------------------------------------------ polynomials */

/* out += a * b in Z[X]/(X^N+1) mod 2^32 (schoolbook). X^N = -1 gives the sign flip. */
static void polymul_acc(int N, const uint32_t *a, const uint32_t *b, uint32_t *out) {
  for (int i = 0; i < N; i++) {
    const uint32_t ai = a[i];
    if (ai == 0) continue;
    uint32_t *o = out + i;
    for (int j = 0; j < N - i; j++) o[j] += ai * b[j];          /* i + j < N  */
    uint32_t *w = out + i - N;
    for (int j = N - i; j < N; j++) w[j] -= ai * b[j];          /* i + j >= N */
  }
}

/* out = a * b in Z[X]/(X^N+1) mod 2^32. */
void or_polymul(int N, const uint32_t *a, const uint32_t *b, uint32_t *out) {
  memset(out, 0, sizeof(uint32_t) * N);
  polymul_acc(N, a, b, out);
}

/* out = X^k * p for k in [0, 2N): coefficient j takes p[j-k], negated when it wraps past X^N. */
void or_rotate(int N, const uint32_t *p, uint32_t k, uint32_t *out) {
  k %= (uint32_t)(2 * N);
  for (int j = 0; j < N; j++) {
    int64_t src = (int64_t)j - (int64_t)k;   /* in (-2N, N) */
    int neg = 0;
    while (src < 0) { src += N; neg ^= 1; }
    out[j] = neg ? (uint32_t)(0u - p[src]) : p[src];
  }
}

/* ------------------------------------------------------------------ encryption (Sec. 2.1.2) */

/* TLWE: b = <a, s> + m + e, where m is a torus value. c = (a[0..n), b). */
void or_tlwe_encrypt_torus(int n, const uint32_t *s, const uint32_t *a, int32_t e, uint32_t m,
                           uint32_t *c) {
  uint32_t dot = 0;
  for (int i = 0; i < n; i++) { c[i] = a[i]; dot += a[i] * s[i]; }
  c[n] = dot + m + (uint32_t)e;
}

/* TLWE of a bit: message mu(2m - 1), mu = 1/8. */
void or_tlwe_encrypt_bit(int n, const uint32_t *s, const uint32_t *a, int32_t e, int m, uint32_t *c) {
  or_tlwe_encrypt_torus(n, s, a, e, m ? MU : (uint32_t)(0u - MU), c);
}

/* Phase b - <a, s>. */
uint32_t or_tlwe_phase(int n, const uint32_t *s, const uint32_t *c) {
  uint32_t dot = 0;
  for (int i = 0; i < n; i++) dot += c[i] * s[i];
  return c[n] - dot;
}

/* Decryption (1 + sgn(phase))/2, with phase 0 read as positive. */
int or_tlwe_decrypt(int n, const uint32_t *s, const uint32_t *c) {
  return (int32_t)or_tlwe_phase(n, s, c) >= 0 ? 1 : 0;
}

/* TRLWE: b[X] = a[X] s[X] + m[X] + e[X] with a torus message polynomial m. c = (a, b). */
void or_trlwe_encrypt_torus(int N, const uint32_t *s, const uint32_t *a, const int32_t *e,
                            const uint32_t *m, uint32_t *c) {
  uint32_t *ca = c, *cb = c + N;
  memcpy(ca, a, sizeof(uint32_t) * N);
  or_polymul(N, a, s, cb);
  for (int j = 0; j < N; j++) cb[j] += m[j] + (uint32_t)e[j];
}

/* TRLWE of a bit polynomial: message mu(2m[X] - 1[X]). */
void or_trlwe_encrypt_bits(int N, const uint32_t *s, const uint32_t *a, const int32_t *e,
                           const uint8_t *bits, uint32_t *c) {
  uint32_t *m = xmalloc(sizeof(uint32_t) * N);
  for (int j = 0; j < N; j++) m[j] = bits[j] ? MU : (uint32_t)(0u - MU);
  or_trlwe_encrypt_torus(N, s, a, e, m, c);
  free(m);
}

/* Phase polynomial b - a s. */
void or_trlwe_phase(int N, const uint32_t *s, const uint32_t *c, uint32_t *ph) {
  or_polymul(N, c, s, ph);
  for (int j = 0; j < N; j++) ph[j] = c[N + j] - ph[j];
}

/* Gadget entry 1/Bg^j on the 2^32 torus, j = 1..l. */
static uint32_t gadget(const or_params *P, int j) { return 1u << (32 - P->bgbit * j); }

/* TRGSW of a bit m: 2l rows, each a TRLWE of zero (a_r, a_r s + e_r). Rows r = 0..l-1 add
 * m/Bg^(r+1) to the constant coefficient of a_r; rows l..2l-1 add m/Bg^(r-l+1) to that of
 * b_r (the 2l x 2 matrix of Sec. 2.1.2). C is [2l][2][N]. */
void or_trgsw_encrypt(const or_params *P, const uint32_t *s, const uint32_t *masks,
                      const int32_t *noise, int m, uint32_t *C) {
  const int N = P->N, l = P->l;
  uint32_t *zero = xmalloc(sizeof(uint32_t) * N);
  memset(zero, 0, sizeof(uint32_t) * N);
  for (int r = 0; r < 2 * l; r++) {
    uint32_t *row = C + (size_t)r * 2 * N;
    or_trlwe_encrypt_torus(N, s, masks + (size_t)r * N, noise + (size_t)r * N, zero, row);
    if (m) {
      if (r < l) row[0] += gadget(P, r + 1);
      else row[N] += gadget(P, r - l + 1);
    }
  }
  free(zero);
}

/* The trivial TRGSW of 1 (zero masks, zero noise): G. */
void or_trgsw_gadget(const or_params *P, uint32_t *C) {
  const int N = P->N, l = P->l;
  memset(C, 0, sizeof(uint32_t) * 2 * l * 2 * N);
  for (int r = 0; r < l; r++) C[(size_t)r * 2 * N] = gadget(P, r + 1);
  for (int r = l; r < 2 * l; r++) C[(size_t)r * 2 * N + N] = gadget(P, r - l + 1);
}

/* ------------------------------------------------------------------ parallel helper */

typedef struct { void (*fn)(void *, int64_t); void *ctx; int64_t lo, hi, step; } or_job;

static void *job_run(void *p) {
  or_job *j = p;
  for (int64_t i = j->lo; i < j->hi; i += j->step) j->fn(j->ctx, i);
  return NULL;
}

/* Runs fn(ctx, i) for i in [0, count) on `threads` threads (round-robin split). */
static void parallel_for(int64_t count, int threads, void (*fn)(void *, int64_t), void *ctx) {
  if (threads < 1) threads = 1;
  if (threads > count) threads = (int)(count > 0 ? count : 1);
  if (threads == 1) { for (int64_t i = 0; i < count; i++) fn(ctx, i); return; }
  pthread_t *th = xmalloc(sizeof(pthread_t) * threads);
  or_job *jobs = xmalloc(sizeof(or_job) * threads);
  for (int t = 0; t < threads; t++) {
    jobs[t] = (or_job){fn, ctx, t, count, threads};
    pthread_create(&th[t], NULL, job_run, &jobs[t]);
  }
  for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
  free(th); free(jobs);
}

/* ------------------------------------------------------------------ keys */

typedef struct { const or_params *P; const uint32_t *s0, *s1, *masks; const int32_t *noise; uint32_t *out; } bk_ctx;

static void bk_one(void *p, int64_t i) {
  bk_ctx *c = p;
  const or_params *P = c->P;
  const size_t rowsz = (size_t)2 * P->l * P->N;
  or_trgsw_encrypt(P, c->s1, c->masks + i * rowsz, c->noise + i * rowsz, (int)c->s0[i],
                   c->out + (size_t)i * rowsz * 2);
}

/* Bootstrapping key: BK[i] = TRGSW_{s1}(s0[i]), i < n. masks/noise are [n][2l][N];
 * bk is [n][2l][2][N]. */
void or_bk_gen(const or_params *P, const uint32_t *s0, const uint32_t *s1, const uint32_t *masks,
               const int32_t *noise, uint32_t *bk, int threads) {
  bk_ctx c = {P, s0, s1, masks, noise, bk};
  parallel_for(P->n, threads, bk_one, &c);
}

/* Key-switching key: KSK[j][p][v-1] = TLWE_{s0}(v * s1[j] / base^(p+1)), j < N, p < t,
 * v = 1..base-1. masks are [N][t][base-1][n], noise [N][t][base-1]; ksk is
 * [N][t][base-1][n+1]. */
void or_ksk_gen(const or_params *P, const uint32_t *s0, const uint32_t *s1, const uint32_t *masks,
                const int32_t *noise, uint32_t *ksk) {
  const int n = P->n, base = 1 << P->basebit;
  for (int j = 0; j < P->N; j++)
    for (int p = 0; p < P->t; p++)
      for (int v = 1; v < base; v++) {
        size_t idx = ((size_t)j * P->t + p) * (base - 1) + (v - 1);
        uint32_t m = (uint32_t)v * s1[j] * (1u << (32 - (p + 1) * P->basebit));
        or_tlwe_encrypt_torus(n, s0, masks + idx * n, noise[idx], m, ksk + idx * (n + 1));
      }
}

/* ------------------------------------------------------------------ bootstrapping steps */

/* Signed gadget decomposition of a torus value: x ~ sum_{r=1..l} d_r / Bg^r with
 * d_r in [-Bg/2, Bg/2), rounding to the nearest multiple of 1/Bg^l. d[r-1] = d_r. */
void or_decompose(const or_params *P, uint32_t x, int32_t *d) {
  const int l = P->l, bgbit = P->bgbit;
  const uint32_t half = 1u << (bgbit - 1), mask = (1u << bgbit) - 1;
  uint32_t offset = 0;
  for (int r = 1; r <= l; r++) offset += half << (32 - r * bgbit);
  offset += 1u << (32 - l * bgbit - 1);                   /* round to nearest */
  const uint32_t t = x + offset;
  for (int r = 1; r <= l; r++) d[r - 1] = (int32_t)((t >> (32 - r * bgbit)) & mask) - (int32_t)half;
}

/* Modulus switch of a torus value to Z/2N: round(x * 2N / 2^32) mod 2N. */
uint32_t or_modswitch(uint32_t x, int N) {
  int logtwoN = 0;
  while ((1 << logtwoN) < 2 * N) logtwoN++;
  const int sh = 32 - logtwoN;
  return ((x + (1u << (sh - 1))) >> sh) & (uint32_t)(2 * N - 1);
}

/* External product C [2l][2][N] (TRGSW) times (A, B) (TRLWE): decompose A into rows 0..l-1
 * and B into rows l..2l-1, then sum_q d_q * C[q] over both polynomials of each row. */
void or_external_product(const or_params *P, const uint32_t *C, const uint32_t *in, uint32_t *out) {
  const int N = P->N, l = P->l;
  uint32_t *dig = xmalloc(sizeof(uint32_t) * 2 * l * N);
  int32_t d[16];
  for (int half = 0; half < 2; half++)
    for (int j = 0; j < N; j++) {
      or_decompose(P, in[half * N + j], d);
      for (int r = 0; r < l; r++) dig[(size_t)(half * l + r) * N + j] = (uint32_t)d[r];
    }
  memset(out, 0, sizeof(uint32_t) * 2 * N);
  for (int q = 0; q < 2 * l; q++) {
    const uint32_t *row = C + (size_t)q * 2 * N;
    polymul_acc(N, dig + (size_t)q * N, row, out);          /* a part */
    polymul_acc(N, dig + (size_t)q * N, row + N, out + N);  /* b part */
  }
  free(dig);
}

/* CMUX(C, x0, x1) = x0 + C (ext) (x1 - x0): x1 if C encrypts 1, x0 if it encrypts 0. */
static void cmux(const or_params *P, const uint32_t *C, const uint32_t *x0, const uint32_t *x1, uint32_t *out) {
  const int N = P->N;
  uint32_t *diff = xmalloc(sizeof(uint32_t) * 2 * N);
  for (int j = 0; j < 2 * N; j++) diff[j] = x1[j] - x0[j];
  or_external_product(P, C, diff, out);
  for (int j = 0; j < 2 * N; j++) out[j] += x0[j];
  free(diff);
}

/* CMUX as a memory-unit gate (counted). */
void or_cmux(const or_params *P, const uint32_t *C, const uint32_t *x0, const uint32_t *x1, uint32_t *out) {
  cmux(P, C, x0, x1, out);
  __atomic_fetch_add(&g_cmux_count, 1, __ATOMIC_RELAXED);
}

/* Blind rotation of a TLWE c (n+1) with test vector tv [N]:
 * ACC = (0, X^{-bbar} tv); for i = 0..n-1: ACC <- CMUX(BK[i], ACC, X^{abar_i} ACC),
 * i.e. ACC + BK[i] (ext) (X^{abar_i} ACC - ACC). acc is [2][N]. */
void or_blind_rotate(const or_params *P, const uint32_t *bk, const uint32_t *c, const uint32_t *tv,
                     uint32_t *acc) {
  const int n = P->n, N = P->N;
  const size_t trgsw = (size_t)2 * P->l * 2 * N;
  uint32_t *rot = xmalloc(sizeof(uint32_t) * 2 * N);
  uint32_t *next = xmalloc(sizeof(uint32_t) * 2 * N);
  const uint32_t bbar = or_modswitch(c[n], N);
  memset(acc, 0, sizeof(uint32_t) * N);
  or_rotate(N, tv, (uint32_t)(2 * N) - bbar, acc + N);
  for (int i = 0; i < n; i++) {
    const uint32_t abar = or_modswitch(c[i], N);
    or_rotate(N, acc, abar, rot);
    or_rotate(N, acc + N, abar, rot + N);
    cmux(P, bk + i * trgsw, acc, rot, next);
    memcpy(acc, next, sizeof(uint32_t) * 2 * N);
  }
  free(rot); free(next);
  __atomic_fetch_add(&g_br_count, 1, __ATOMIC_RELAXED);
}

/* SampleExtract at index h: the TLWE (under the coefficients of s1) whose phase is
 * coefficient h of the TRLWE phase. a'_j = A_{h-j} (j <= h), -A_{N+h-j} (j > h); b' = B_h. */
void or_sample_extract(int N, const uint32_t *c, int h, uint32_t *out) {
  for (int j = 0; j < N; j++) out[j] = (j <= h) ? c[h - j] : (uint32_t)(0u - c[N + h - j]);
  out[N] = c[N + h];
}

/* Identity key switching s1 -> s0: out = (0, b') - sum_{j,p} KSK[j][p][v_{j,p}] with v_{j,p}
 * the p-th base-2^basebit digit (most significant first) of a'_j rounded to t*basebit bits. */
void or_keyswitch(const or_params *P, const uint32_t *ksk, const uint32_t *in, uint32_t *out) {
  const int n = P->n, N = P->N, t = P->t, bb = P->basebit, base = 1 << bb;
  const uint32_t round = 1u << (32 - t * bb - 1);
  memset(out, 0, sizeof(uint32_t) * (n + 1));
  out[n] = in[N];
  for (int j = 0; j < N; j++) {
    const uint32_t ahat = in[j] + round;
    for (int p = 0; p < t; p++) {
      const uint32_t v = (ahat >> (32 - (p + 1) * bb)) & (uint32_t)(base - 1);
      if (v == 0) continue;
      const uint32_t *k = ksk + (((size_t)j * t + p) * (base - 1) + (v - 1)) * (n + 1);
      for (int i = 0; i <= n; i++) out[i] -= k[i];
    }
  }
}

/* Key-switch digits of one value (for property checks). */
void or_ks_digits(const or_params *P, uint32_t a, uint32_t *v) {
  const int t = P->t, bb = P->basebit;
  const uint32_t ahat = a + (1u << (32 - t * bb - 1));
  for (int p = 0; p < t; p++) v[p] = (ahat >> (32 - (p + 1) * bb)) & ((1u << bb) - 1);
}

/* Linear combination of a homomorphic gate (the standard TFHE gate combinations on the
 * +-1/8 encoding): c = (0, k) + s1*c1 + s2*c2. Returns 0 for NOT (c = -c1, no bootstrap). */
int or_gate_linear(int n, int op, const uint32_t *c1, const uint32_t *c2, uint32_t *c) {
  const uint32_t E = MU, Q = 2 * MU; /* 1/8 and 1/4 */
  int32_t s1 = 1, s2 = 1; uint32_t k = 0;
  switch (op) {
    case OR_NAND:   k = E;            s1 = -1; s2 = -1; break;
    case OR_AND:    k = 0u - E;       s1 = 1;  s2 = 1;  break;
    case OR_OR:     k = E;            s1 = 1;  s2 = 1;  break;
    case OR_NOR:    k = 0u - E;       s1 = -1; s2 = -1; break;
    case OR_XOR:    k = Q;            s1 = 2;  s2 = 2;  break;
    case OR_XNOR:   k = 0u - Q;       s1 = -2; s2 = -2; break;
    case OR_ANDNOT: k = 0u - E;       s1 = 1;  s2 = -1; break;
    case OR_ORNOT:  k = E;            s1 = 1;  s2 = -1; break;
    case OR_NOT:
      for (int i = 0; i <= n; i++) c[i] = 0u - c1[i];
      return 0;
    default: abort();
  }
  for (int i = 0; i <= n; i++) c[i] = (uint32_t)s1 * c1[i] + (uint32_t)s2 * c2[i];
  c[n] += k;
  return 1;
}

/* Bootstrapping of a TLWE to a TRLWE (no SE, no IKS): blind rotation with the test vector
 * mu in every coefficient. acc is [2][N]. */
void or_bootstrap_to_trlwe(const or_params *P, const uint32_t *bk, const uint32_t *c, uint32_t *acc) {
  uint32_t *tv = xmalloc(sizeof(uint32_t) * P->N);
  for (int j = 0; j < P->N; j++) tv[j] = MU;
  or_blind_rotate(P, bk, c, tv, acc);
  free(tv);
}

/* Homomorphic gate: linear combination, blind rotation, SampleExtract(0), key switch. */
void or_gate(const or_params *P, const uint32_t *bk, const uint32_t *ksk, int op,
             const uint32_t *c1, const uint32_t *c2, uint32_t *out) {
  const int n = P->n, N = P->N;
  uint32_t *lin = xmalloc(sizeof(uint32_t) * (n + 1));
  if (!or_gate_linear(n, op, c1, c2, lin)) { memcpy(out, lin, sizeof(uint32_t) * (n + 1)); free(lin); return; }
  uint32_t *acc = xmalloc(sizeof(uint32_t) * 2 * N);
  uint32_t *ext = xmalloc(sizeof(uint32_t) * (N + 1));
  or_bootstrap_to_trlwe(P, bk, lin, acc);
  or_sample_extract(N, acc, 0, ext);
  or_keyswitch(P, ksk, ext, out);
  free(lin); free(acc); free(ext);
}

typedef struct { const or_params *P; const uint32_t *bk, *ksk; const uint8_t *ops; const uint32_t *in0, *in1; uint32_t *out; } gates_ctx;

static void gate_one(void *p, int64_t g) {
  gates_ctx *c = p;
  const size_t w = (size_t)c->P->n + 1;
  or_gate(c->P, c->bk, c->ksk, c->ops[g], c->in0 + g * w, c->in1 + g * w, c->out + g * w);
}

/* B independent gates, spread over `threads` threads. */
void or_gates(const or_params *P, const uint32_t *bk, const uint32_t *ksk, const uint8_t *ops,
              const uint32_t *in0, const uint32_t *in1, uint32_t *out, int64_t B, int threads) {
  gates_ctx c = {P, bk, ksk, ops, in0, in1, out};
  parallel_for(B, threads, gate_one, &c);
}

/* Homomorphic MUX, s ? c1 : c0 (the three-operand gate of Sec. 2.1.2, TFHE section): the two
 * bootstrapped halves AND(s, c1) and ANDNOT(c0, s) are added as TRLWE together with (0, mu),
 * which is the HomMUX without SE and IKS of Sec. 2.1.2; SampleExtract at 0 and the identity
 * key switch then return a TLWE under the LWE key. */
void or_mux(const or_params *P, const uint32_t *bk, const uint32_t *ksk, const uint32_t *s,
            const uint32_t *c1, const uint32_t *c0, uint32_t *out) {
  const int n = P->n, N = P->N;
  uint32_t *lin = xmalloc(sizeof(uint32_t) * (n + 1));
  uint32_t *acc = xmalloc(sizeof(uint32_t) * 2 * N);
  uint32_t *acc2 = xmalloc(sizeof(uint32_t) * 2 * N);
  uint32_t *ext = xmalloc(sizeof(uint32_t) * (N + 1));
  or_gate_linear(n, OR_AND, s, c1, lin);
  or_bootstrap_to_trlwe(P, bk, lin, acc);
  or_gate_linear(n, OR_ANDNOT, c0, s, lin);
  or_bootstrap_to_trlwe(P, bk, lin, acc2);
  for (int j = 0; j < 2 * N; j++) acc[j] += acc2[j];
  acc[N] += MU;
  or_sample_extract(N, acc, 0, ext);
  or_keyswitch(P, ksk, ext, out);
  free(lin); free(acc); free(acc2); free(ext);
}

typedef struct { const or_params *P; const uint32_t *bk, *ksk, *s, *c1, *c0; uint32_t *out; } mux_ctx;

static void mux_one(void *p, int64_t g) {
  mux_ctx *c = p;
  const size_t w = (size_t)c->P->n + 1;
  or_mux(c->P, c->bk, c->ksk, c->s + g * w, c->c1 + g * w, c->c0 + g * w, c->out + g * w);
}

/* B independent MUXes, spread over `threads` threads. */
void or_muxes(const or_params *P, const uint32_t *bk, const uint32_t *ksk, const uint32_t *s,
              const uint32_t *c1, const uint32_t *c0, uint32_t *out, int64_t B, int threads) {
  mux_ctx c = {P, bk, ksk, s, c1, c0, out};
  parallel_for(B, threads, mux_one, &c);
}

/* ------------------------------------------------------------------ CMUX memory (Sec. 8) */

/* ROM read by a CMUX tree over packed TRLWE cells (LUT with vertical and horizontal
 * packing). `words_per_poly` words of `wbits` bits share one polynomial: coefficient
 * wbits*q + b of cell h holds bit b of word words_per_poly*h + q. Selectors sel[j]
 * ([abits][2l][2][N]) encrypt the address bits, least significant first. The high
 * address bits walk the tree over the npoly cells (first the lowest of them); the low
 * bits rotate the chosen cell by X^{-wbits*q}; output bit b is KS(SE_b(.)).
 * out is [wbits][n+1]. */
void or_rom_read(const or_params *P, const uint32_t *ksk, const uint32_t *rom, int npoly,
                 const uint32_t *sel, int abits, int wbits, uint32_t *out) {
  const int N = P->N, n = P->n;
  const size_t tr = (size_t)2 * N, trgsw = (size_t)2 * P->l * 2 * N;
  int rotbits = 0;
  while ((wbits << rotbits) < N) rotbits++;            /* log2(N / wbits) */
  uint32_t *L = xmalloc(sizeof(uint32_t) * tr * npoly);
  memcpy(L, rom, sizeof(uint32_t) * tr * npoly);
  int width = npoly;
  for (int d = 0; rotbits + d < abits && width > 1; d++) {
    for (int m = 0; m < width / 2; m++) {
      uint32_t *res = xmalloc(sizeof(uint32_t) * tr);
      or_cmux(P, sel + (size_t)(rotbits + d) * trgsw, L + (2 * m) * tr, L + (2 * m + 1) * tr, res);
      memcpy(L + m * tr, res, sizeof(uint32_t) * tr);
      free(res);
    }
    width /= 2;
  }
  uint32_t *R = L, *rot = xmalloc(sizeof(uint32_t) * tr), *res = xmalloc(sizeof(uint32_t) * tr);
  for (int j = 0; j < rotbits; j++) {
    const uint32_t k = (uint32_t)(2 * N) - (uint32_t)(wbits << j);
    or_rotate(N, R, k, rot);
    or_rotate(N, R + N, k, rot + N);
    or_cmux(P, sel + (size_t)j * trgsw, R, rot, res);
    memcpy(R, res, sizeof(uint32_t) * tr);
  }
  uint32_t *ext = xmalloc(sizeof(uint32_t) * (N + 1));
  for (int b = 0; b < wbits; b++) {
    or_sample_extract(N, R, b, ext);
    or_keyswitch(P, ksk, ext, out + (size_t)b * (n + 1));
  }
  free(L); free(rot); free(res); free(ext);
}

/* CMUX tree over the 2^v cells of one RAM bit block, address bits least significant first. */
static void ram_tree(const or_params *P, const uint32_t *cells, int v, const uint32_t *sel, uint32_t *res) {
  const int N = P->N;
  const size_t tr = (size_t)2 * N, trgsw = (size_t)2 * P->l * 2 * N;
  int width = 1 << v;
  uint32_t *L = xmalloc(sizeof(uint32_t) * tr * width);
  memcpy(L, cells, sizeof(uint32_t) * tr * width);
  uint32_t *tmp = xmalloc(sizeof(uint32_t) * tr);
  for (int d = 0; d < v; d++) {
    for (int m = 0; m < width / 2; m++) {
      or_cmux(P, sel + (size_t)d * trgsw, L + (2 * m) * tr, L + (2 * m + 1) * tr, tmp);
      memcpy(L + m * tr, tmp, sizeof(uint32_t) * tr);
    }
    width /= 2;
  }
  memcpy(res, L, sizeof(uint32_t) * tr);
  free(L); free(tmp);
}

/* RAM read unit (Sec. 8.2): the RAM is w blocks of 2^v TRLWE cells (block i holds bit i of
 * every word, in the constant coefficient). Per bit: CMUX tree, SampleExtract(0), key switch.
 * ram is [w][2^v][2][N]; sel is [v][2l][2][N]; out is [w][n+1]. */
void or_ram_read(const or_params *P, const uint32_t *ksk, const uint32_t *ram, int v, int w,
                 const uint32_t *sel, uint32_t *out) {
  const int N = P->N, n = P->n;
  const size_t tr = (size_t)2 * N;
  uint32_t *res = xmalloc(sizeof(uint32_t) * tr), *ext = xmalloc(sizeof(uint32_t) * (N + 1));
  for (int i = 0; i < w; i++) {
    ram_tree(P, ram + (size_t)i * (1u << v) * tr, v, sel, res);
    or_sample_extract(N, res, 0, ext);
    or_keyswitch(P, ksk, ext, out + (size_t)i * (n + 1));
  }
  free(res); free(ext);
}

/* RAM control unit (Sec. 8.2): multiplex write data x_i and read data r_i by the write flag f
 * with a HomMUX without SE and IKS: u_i = BR(AND(f, x_i)) + BR(ANDNOT(r_i, f)) + (0, mu X^0).
 * u is [w][2][N]. The w bits are independent and run on `threads` threads. */
typedef struct { const or_params *P; const uint32_t *bk, *flag, *data, *rd; uint32_t *u; } ctl_ctx;

static void ctl_one(void *p, int64_t i) {
  ctl_ctx *c = p;
  const int n = c->P->n, N = c->P->N;
  uint32_t *lin = xmalloc(sizeof(uint32_t) * (n + 1));
  uint32_t *acc = xmalloc(sizeof(uint32_t) * 2 * N);
  uint32_t *ui = c->u + (size_t)i * 2 * N;
  or_gate_linear(n, OR_AND, c->flag, c->data + (size_t)i * (n + 1), lin);
  or_bootstrap_to_trlwe(c->P, c->bk, lin, ui);
  or_gate_linear(n, OR_ANDNOT, c->rd + (size_t)i * (n + 1), c->flag, lin);
  or_bootstrap_to_trlwe(c->P, c->bk, lin, acc);
  for (int j = 0; j < 2 * N; j++) ui[j] += acc[j];
  ui[N] += MU;
  free(lin); free(acc);
}

void or_ram_control(const or_params *P, const uint32_t *bk, const uint32_t *flag, const uint32_t *data,
                    const uint32_t *rd, int w, uint32_t *u) {
  ctl_ctx c = {P, bk, flag, data, rd, u};
  parallel_for(w, w, ctl_one, &c);
}

/* Selector of write-bar bit d for constant address bit c: C_d if c = 1, G - C_d if c = 0
 * (comparison with 0, Sec. 8.2 Remark). */
static void bar_selector(const or_params *P, const uint32_t *Cd, int c, uint32_t *out) {
  const size_t trgsw = (size_t)2 * P->l * 2 * P->N;
  if (c) { memcpy(out, Cd, sizeof(uint32_t) * trgsw); return; }
  or_trgsw_gadget(P, out);
  for (size_t k = 0; k < trgsw; k++) out[k] -= Cd[k];
}

typedef struct { const or_params *P; const uint32_t *bk, *ksk, *ram, *sel, *u; uint32_t *out; int v; } bar_ctx;

/* One write bar (bit i, address A): y <- u_i; for d = 0..v-1: y <- CMUX(sel_{d,A}, R[i][A], y);
 * then refresh: R'[i][A] = BR(KS(SE_0(y))) as a TRLWE. */
static void bar_one(void *p, int64_t k) {
  bar_ctx *c = p;
  const or_params *P = c->P;
  const int N = P->N, n = P->n, v = c->v;
  const size_t tr = (size_t)2 * N, trgsw = (size_t)2 * P->l * 2 * N;
  const int64_t i = k >> v, A = k & ((1 << v) - 1);
  const uint32_t *old = c->ram + (size_t)k * tr;
  uint32_t *y = xmalloc(sizeof(uint32_t) * tr), *tmp = xmalloc(sizeof(uint32_t) * tr);
  uint32_t *s = xmalloc(sizeof(uint32_t) * trgsw);
  uint32_t *ext = xmalloc(sizeof(uint32_t) * (N + 1)), *lwe = xmalloc(sizeof(uint32_t) * (n + 1));
  memcpy(y, c->u + (size_t)i * tr, sizeof(uint32_t) * tr);
  for (int d = 0; d < v; d++) {
    bar_selector(P, c->sel + (size_t)d * trgsw, (int)((A >> d) & 1), s);
    or_cmux(P, s, old, y, tmp);
    memcpy(y, tmp, sizeof(uint32_t) * tr);
  }
  or_sample_extract(N, y, 0, ext);
  or_keyswitch(P, c->ksk, ext, lwe);
  or_bootstrap_to_trlwe(P, c->bk, lwe, c->out + (size_t)k * tr);
  free(y); free(tmp); free(s); free(ext); free(lwe);
}

typedef struct { bar_ctx base; const int64_t *idx; } sub_ctx;

static void sub_bar(void *p, int64_t k) {
  sub_ctx *c = p;
  const size_t tr = (size_t)2 * c->base.P->N;
  bar_ctx b = c->base;
  b.out = c->base.out + (size_t)k * tr - (size_t)c->idx[k] * tr;   /* bar idx[k] lands in slot k */
  bar_one(&b, c->idx[k]);
}

/* Write bars for a subset of (bit, address) pairs given the controlled data u ([w][2][N]):
 * out[k] = refreshed cell of bar idx[k] = i * 2^v + A (samples large RAMs). */
void or_ram_write_bars(const or_params *P, const uint32_t *bk, const uint32_t *ksk, const uint32_t *ram,
                       int v, const uint32_t *sel, const uint32_t *u, const int64_t *idx, int64_t count,
                       uint32_t *out, int threads) {
  sub_ctx c = {{P, bk, ksk, ram, sel, u, out, v}, idx};
  parallel_for(count, threads, sub_bar, &c);
}

/* RAM write (Sec. 8.2): read unit at the address, control unit, then all w*2^v write bars
 * (each reading the old cell) with a refresh bootstrap. ram is updated in place. */
void or_ram_write(const or_params *P, const uint32_t *bk, const uint32_t *ksk, uint32_t *ram, int v, int w,
                  const uint32_t *sel, const uint32_t *flag, const uint32_t *data, int threads) {
  const int n = P->n, N = P->N;
  const size_t tr = (size_t)2 * N, cells = (size_t)w << v;
  uint32_t *rd = xmalloc(sizeof(uint32_t) * w * (n + 1));
  uint32_t *u = xmalloc(sizeof(uint32_t) * w * tr);
  uint32_t *nw = xmalloc(sizeof(uint32_t) * cells * tr);
  or_ram_read(P, ksk, ram, v, w, sel, rd);
  or_ram_control(P, bk, flag, data, rd, w, u);
  bar_ctx c = {P, bk, ksk, ram, sel, u, nw, v};
  parallel_for((int64_t)cells, threads, bar_one, &c);
  memcpy(ram, nw, sizeof(uint32_t) * cells * tr);
  free(rd); free(u); free(nw);
}

/* ------------------------------------------------------------------ batches of reads */

typedef struct { const or_params *P; const uint32_t *ksk, *mem, *sel; uint32_t *out; int a, b, c; } reads_ctx;

static void rom_one(void *p, int64_t r) {
  reads_ctx *c = p;
  const size_t trgsw = (size_t)2 * c->P->l * 2 * c->P->N;
  or_rom_read(c->P, c->ksk, c->mem, c->a, c->sel + (size_t)r * c->b * trgsw, c->b, c->c,
              c->out + (size_t)r * c->c * (c->P->n + 1));
}

/* R independent ROM reads; sel is [R][abits][2l][2][N], out [R][wbits][n+1]. */
void or_rom_reads(const or_params *P, const uint32_t *ksk, const uint32_t *rom, int npoly, const uint32_t *sel,
                  int abits, int wbits, uint32_t *out, int64_t R, int threads) {
  reads_ctx c = {P, ksk, rom, sel, out, npoly, abits, wbits};
  parallel_for(R, threads, rom_one, &c);
}

static void ram_one(void *p, int64_t r) {
  reads_ctx *c = p;
  const size_t trgsw = (size_t)2 * c->P->l * 2 * c->P->N;
  or_ram_read(c->P, c->ksk, c->mem, c->a, c->b, c->sel + (size_t)r * c->a * trgsw,
              c->out + (size_t)r * c->b * (c->P->n + 1));
}

/* R independent RAM reads; sel is [R][v][2l][2][N], out [R][w][n+1]. */
void or_ram_reads(const or_params *P, const uint32_t *ksk, const uint32_t *ram, int v, int w, const uint32_t *sel,
                  uint32_t *out, int64_t R, int threads) {
  reads_ctx c = {P, ksk, ram, sel, out, v, w, 0};
  parallel_for(R, threads, ram_one, &c);
}

/* ================================================================== circuit bootstrapping
 *
 * TLWE (level 0, a bit as +-1/8) -> TRGSW (level 1, gadget l x Bg), the conversion the paper
 * names "Circuit Bootstrapping" (Sec. 2.1.2, after Chillotti et al.) and applies to the
 * address bits of the CMUX memory (Sec. 8.2). The paper fixes no parameters for it; the
 * reading used here: a level-2 ring of degree N2 over the 2^64 torus (uint64), a level-2
 * bootstrapping key BK2[i] = TRGSW2_{s2}(s0[i]) with gadget l2 x 2^bgbit2, and private
 * functional key switching from level 2 to level-1 TRLWE with t2 digits of basebit2 bits.
 * For each gadget level j = 1..l of the output: a level-2 blind rotation of c with the
 * test vector 1/(2 Bg^j) in every coefficient, SampleExtract at 0, plus 1/(2 Bg^j) (so the
 * TLWE2 holds m/Bg^j), then two private key switches: f(x) = -s1 x gives TRGSW row j-1 (the
 * rows whose a part carries m/Bg^j, phase -m s1/Bg^j) and f(x) = x gives row l+j-1 (phase
 * m/Bg^j), the row layout of or_trgsw_encrypt. */

typedef struct {
  int32_t N;       /* level-2 TRLWE degree */
  int32_t l;       /* level-2 gadget rows per column */
  int32_t bgbit;   /* log2 of the level-2 gadget base */
  int32_t t;       /* private key-switch digits */
  int32_t basebit; /* log2 of the private key-switch base */
} or_params2;

/* out += a * b in Z[X]/(X^N+1) mod 2^64 (schoolbook). */
static void polymul64_acc(int N, const uint64_t *a, const uint64_t *b, uint64_t *out) {
  for (int i = 0; i < N; i++) {
    const uint64_t ai = a[i];
    if (ai == 0) continue;
    uint64_t *o = out + i;
    for (int j = 0; j < N - i; j++) o[j] += ai * b[j];
    uint64_t *w = out + i - N;
    for (int j = N - i; j < N; j++) w[j] -= ai * b[j];
  }
}

void or_polymul64(int N, const uint64_t *a, const uint64_t *b, uint64_t *out) {
  memset(out, 0, sizeof(uint64_t) * N);
  polymul64_acc(N, a, b, out);
}

/* out = X^k p, k in [0, 2N), over the 2^64 torus. */
void or_rotate64(int N, const uint64_t *p, uint32_t k, uint64_t *out) {
  k %= (uint32_t)(2 * N);
  for (int j = 0; j < N; j++) {
    int64_t src = (int64_t)j - (int64_t)k;
    int neg = 0;
    while (src < 0) { src += N; neg ^= 1; }
    out[j] = neg ? (uint64_t)(0ull - p[src]) : p[src];
  }
}

/* Level-2 TRLWE: (a, a s + m + e) over the 2^64 torus. */
void or_trlwe64_encrypt_torus(int N, const uint64_t *s, const uint64_t *a, const int64_t *e,
                              const uint64_t *m, uint64_t *c) {
  memcpy(c, a, sizeof(uint64_t) * N);
  or_polymul64(N, a, s, c + N);
  for (int j = 0; j < N; j++) c[N + j] += m[j] + (uint64_t)e[j];
}

void or_trlwe64_phase(int N, const uint64_t *s, const uint64_t *c, uint64_t *ph) {
  or_polymul64(N, c, s, ph);
  for (int j = 0; j < N; j++) ph[j] = c[N + j] - ph[j];
}

static uint64_t gadget2(const or_params2 *Q, int j) { return 1ull << (64 - Q->bgbit * j); }

/* Level-2 TRGSW of a bit (rows as in or_trgsw_encrypt). masks/noise [2 l2][N2]. */
void or_trgsw64_encrypt(const or_params2 *Q, const uint64_t *s, const uint64_t *masks,
                        const int64_t *noise, int m, uint64_t *C) {
  const int N = Q->N, l = Q->l;
  uint64_t *zero = xmalloc(sizeof(uint64_t) * N);
  for (int r = 0; r < 2 * l; r++) {
    uint64_t *row = C + (size_t)r * 2 * N;
    or_trlwe64_encrypt_torus(N, s, masks + (size_t)r * N, noise + (size_t)r * N, zero, row);
    if (m) {
      if (r < l) row[0] += gadget2(Q, r + 1);
      else row[N] += gadget2(Q, r - l + 1);
    }
  }
  free(zero);
}

typedef struct { const or_params2 *Q; const uint32_t *s0; const uint64_t *s2, *masks; const int64_t *noise; uint64_t *out; } bk2_ctx;

static void bk2_one(void *p, int64_t i) {
  bk2_ctx *c = p;
  const size_t rowsz = (size_t)2 * c->Q->l * c->Q->N;
  or_trgsw64_encrypt(c->Q, c->s2, c->masks + i * rowsz, c->noise + i * rowsz, (int)c->s0[i],
                     c->out + (size_t)i * rowsz * 2);
}

/* Level-2 bootstrapping key: BK2[i] = TRGSW2_{s2}(s0[i]), i < n. masks/noise [n][2 l2][N2];
 * bk2 [n][2 l2][2][N2]. */
void or_bk2_gen(int n, const or_params2 *Q, const uint32_t *s0, const uint64_t *s2, const uint64_t *masks,
                const int64_t *noise, uint64_t *bk2, int threads) {
  bk2_ctx c = {Q, s0, s2, masks, noise, bk2};
  parallel_for(n, threads, bk2_one, &c);
}

/* Signed gadget decomposition on the 2^64 torus: x ~ sum_{r=1..l2} d_r / Bg2^r, d_r in
 * [-Bg2/2, Bg2/2), rounding to the nearest multiple of 1/Bg2^l2. */
void or_decompose64(const or_params2 *Q, uint64_t x, int64_t *d) {
  const int l = Q->l, bgbit = Q->bgbit;
  const uint64_t half = 1ull << (bgbit - 1), mask = (1ull << bgbit) - 1;
  uint64_t offset = 0;
  for (int r = 1; r <= l; r++) offset += half << (64 - r * bgbit);
  offset += 1ull << (64 - l * bgbit - 1);
  const uint64_t t = x + offset;
  for (int r = 1; r <= l; r++) d[r - 1] = (int64_t)((t >> (64 - r * bgbit)) & mask) - (int64_t)half;
}

/* Level-2 external product (as or_external_product, mod 2^64). */
void or_external_product64(const or_params2 *Q, const uint64_t *C, const uint64_t *in, uint64_t *out) {
  const int N = Q->N, l = Q->l;
  uint64_t *dig = xmalloc(sizeof(uint64_t) * 2 * l * N);
  int64_t d[16];
  for (int half = 0; half < 2; half++)
    for (int j = 0; j < N; j++) {
      or_decompose64(Q, in[half * N + j], d);
      for (int r = 0; r < l; r++) dig[(size_t)(half * l + r) * N + j] = (uint64_t)d[r];
    }
  memset(out, 0, sizeof(uint64_t) * 2 * N);
  for (int q = 0; q < 2 * l; q++) {
    const uint64_t *row = C + (size_t)q * 2 * N;
    polymul64_acc(N, dig + (size_t)q * N, row, out);
    polymul64_acc(N, dig + (size_t)q * N, row + N, out + N);
  }
  free(dig);
}

/* Level-2 blind rotation of a level-0 TLWE c (n+1, 2^32 torus): modulus switch to Z/2N2,
 * ACC = (0, X^{-bbar} tv), ACC <- ACC + BK2[i] (ext) (X^{abar_i} ACC - ACC) for i < n. */
void or_blind_rotate64(int n, const or_params2 *Q, const uint64_t *bk2, const uint32_t *c, const uint64_t *tv,
                       uint64_t *acc) {
  const int N = Q->N;
  const size_t trgsw = (size_t)2 * Q->l * 2 * N;
  uint64_t *diff = xmalloc(sizeof(uint64_t) * 2 * N);
  uint64_t *prod = xmalloc(sizeof(uint64_t) * 2 * N);
  const uint32_t bbar = or_modswitch(c[n], N);
  memset(acc, 0, sizeof(uint64_t) * N);
  or_rotate64(N, tv, (uint32_t)(2 * N) - bbar, acc + N);
  for (int i = 0; i < n; i++) {
    const uint32_t abar = or_modswitch(c[i], N);
    or_rotate64(N, acc, abar, diff);
    or_rotate64(N, acc + N, abar, diff + N);
    for (int j = 0; j < 2 * N; j++) diff[j] -= acc[j];
    or_external_product64(Q, bk2 + i * trgsw, diff, prod);
    for (int j = 0; j < 2 * N; j++) acc[j] += prod[j];
  }
  free(diff); free(prod);
  __atomic_fetch_add(&g_br_count, 1, __ATOMIC_RELAXED);
}

/* SampleExtract at 0 over the 2^64 torus: TLWE2 (N2 + 1). */
void or_sample_extract64(int N, const uint64_t *c, uint64_t *out) {
  out[0] = c[0];
  for (int j = 1; j < N; j++) out[j] = 0ull - c[N - j];
  out[N] = c[N];
}

/* Private functional key-switching keys from the level-2 TLWE key to level-1 TRLWE under
 * s1, for f_0(x) = -s1 x and f_1(x) = x: with z = (-s2[0], ..., -s2[N2-1], 1) (so that
 * sum_k c_k z_k is the phase of a TLWE2 c = (a, b)),
 *   PKSK[u][k][p][v-1] = TRLWE_{s1}(f_u(v z_k / base^(p+1))),  k <= N2, p < t2, v = 1..base-1,
 * messages on the 2^32 torus. masks [2][N2+1][t2][base-1][N], noise the same shape (int32);
 * pksk [2][N2+1][t2][base-1][2][N]. */
typedef struct { const or_params *P; const or_params2 *Q; const uint32_t *s1; const uint64_t *s2;
                 const uint32_t *masks; const int32_t *noise; uint32_t *out; } pksk_ctx;

static void pksk_one(void *p, int64_t idx) {
  pksk_ctx *c = p;
  const int N = c->P->N, N2 = c->Q->N, t = c->Q->t, bb = c->Q->basebit, base = 1 << bb;
  /* idx = ((u (N2+1) + k) t + pp) (base-1) + (v-1) */
  int64_t r = idx;
  const int v = (int)(r % (base - 1)) + 1; r /= (base - 1);
  const int pp = (int)(r % t); r /= t;
  const int k = (int)(r % (N2 + 1)); r /= (N2 + 1);
  const int u = (int)r;
  const uint32_t z = (k == N2) ? 1u : (uint32_t)(0u - (uint32_t)c->s2[k]);
  const uint32_t x = (uint32_t)v * z * (1u << (32 - (pp + 1) * bb));   /* v z_k / base^(p+1) */
  uint32_t *m = xmalloc(sizeof(uint32_t) * N);
  if (u == 0) for (int j = 0; j < N; j++) m[j] = 0u - c->s1[j] * x;   /* -s1 x */
  else m[0] = x;                                                      /* x      */
  or_trlwe_encrypt_torus(N, c->s1, c->masks + (size_t)idx * N, c->noise + (size_t)idx * N, m,
                         c->out + (size_t)idx * 2 * N);
  free(m);
}

void or_pksk_gen(const or_params *P, const or_params2 *Q, const uint32_t *s1, const uint64_t *s2,
                 const uint32_t *masks, const int32_t *noise, uint32_t *pksk, int threads) {
  pksk_ctx c = {P, Q, s1, s2, masks, noise, pksk};
  const int64_t count = (int64_t)2 * (Q->N + 1) * Q->t * ((1 << Q->basebit) - 1);
  parallel_for(count, threads, pksk_one, &c);
}

/* Private functional key switch of a TLWE2 c (N2 + 1, 2^64 torus) with key u:
 * out = sum_{k <= N2} sum_{p < t2} PKSK[u][k][p][v_{k,p}], v_{k,p} the p-th base-2^basebit2
 * digit (most significant first) of c_k rounded to t2 basebit2 bits. out [2][N]. */
void or_private_keyswitch(const or_params *P, const or_params2 *Q, const uint32_t *pksk, int u,
                          const uint64_t *c, uint32_t *out) {
  const int N = P->N, N2 = Q->N, t = Q->t, bb = Q->basebit, base = 1 << bb;
  const uint64_t round = 1ull << (64 - t * bb - 1);
  const uint32_t *key = pksk + (size_t)u * (N2 + 1) * t * (base - 1) * 2 * N;
  memset(out, 0, sizeof(uint32_t) * 2 * N);
  for (int k = 0; k <= N2; k++) {
    const uint64_t chat = c[k] + round;
    for (int p = 0; p < t; p++) {
      const uint32_t v = (uint32_t)(chat >> (64 - (p + 1) * bb)) & (uint32_t)(base - 1);
      if (v == 0) continue;
      const uint32_t *e = key + (((size_t)k * t + p) * (base - 1) + (v - 1)) * 2 * N;
      for (int j = 0; j < 2 * N; j++) out[j] += e[j];
    }
  }
}

/* Circuit bootstrapping of a level-0 TLWE c of a bit into a level-1 TRGSW C [2l][2][N]
 * (P: the level-0/1 parameters and the output gadget; Q: level 2). */
/* Gadget level j (1..l) of the conversion: TRGSW rows j-1 and l+j-1 of C. */
static void cb_level(const or_params *P, const or_params2 *Q, const uint64_t *bk2, const uint32_t *pksk,
                     const uint32_t *c, int j, uint32_t *C) {
  const int N = P->N, l = P->l, N2 = Q->N;
  uint64_t *tv = xmalloc(sizeof(uint64_t) * N2);
  uint64_t *acc = xmalloc(sizeof(uint64_t) * 2 * N2);
  uint64_t *ext = xmalloc(sizeof(uint64_t) * (N2 + 1));
  const uint64_t half = 1ull << (63 - P->bgbit * j);       /* 1/(2 Bg^j) */
  for (int i = 0; i < N2; i++) tv[i] = half;
  or_blind_rotate64(P->n, Q, bk2, c, tv, acc);
  or_sample_extract64(N2, acc, ext);
  ext[N2] += half;                                          /* m / Bg^j */
  or_private_keyswitch(P, Q, pksk, 0, ext, C + (size_t)(j - 1) * 2 * N);
  or_private_keyswitch(P, Q, pksk, 1, ext, C + (size_t)(l + j - 1) * 2 * N);
  free(tv); free(acc); free(ext);
}

void or_circuit_bootstrap(const or_params *P, const or_params2 *Q, const uint64_t *bk2, const uint32_t *pksk,
                          const uint32_t *c, uint32_t *C) {
  for (int j = 1; j <= P->l; j++) cb_level(P, Q, bk2, pksk, c, j, C);
}

typedef struct { const or_params *P; const or_params2 *Q; const uint64_t *bk2; const uint32_t *pksk;
                 const uint32_t *in; uint32_t *out; } cb_ctx;

static void cb_one(void *p, int64_t job) {
  cb_ctx *c = p;
  const int l = c->P->l;
  const int64_t i = job / l;
  const size_t trgsw = (size_t)2 * l * 2 * c->P->N;
  cb_level(c->P, c->Q, c->bk2, c->pksk, c->in + (size_t)i * (c->P->n + 1), (int)(job % l) + 1, c->out + i * trgsw);
}

/* R circuit bootstraps, their R l gadget levels spread over `threads` threads.
 * in [R][n+1], out [R][2l][2][N]. */
void or_circuit_bootstraps(const or_params *P, const or_params2 *Q, const uint64_t *bk2, const uint32_t *pksk,
                           const uint32_t *in, uint32_t *out, int64_t R, int threads) {
  cb_ctx c = {P, Q, bk2, pksk, in, out};
  parallel_for(R * P->l, threads, cb_one, &c);
}

/*
 * Exhaustive property checks of the oracle's scalar steps over every 32-bit torus value.
 * The properties are the mathematical definitions, not a re-implementation:
 *   gadget decomposition: digits in [-Bg/2, Bg/2) and x - sum_r d_r 2^(32-6r) in [-2^13, 2^13)
 *     (with the recomposition a multiple of 2^14, this is exactly rounding to the nearest
 *     multiple of 1/Bg^l);
 *   modulus switch: xbar in [0, 2N) and x - xbar 2^21 in [-2^20, 2^20);
 *   key-switch digits: v_p in [0, base) and a - sum_p v_p 2^(30-2p) in [-2^15, 2^15).
 * Usage: exhaustive <liboracle.so> <threads>. Prints failures and exits non-zero on any.
 */
#include <dlfcn.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct { int32_t n, N, l, bgbit, t, basebit; } params;
static void (*f_dec)(const params *, uint32_t, int32_t *);
static uint32_t (*f_ms)(uint32_t, int);
static void (*f_ks)(const params *, uint32_t, uint32_t *);
static params P = {630, 1024, 3, 6, 8, 2};
static int nthreads;

typedef struct { int id; uint64_t bad_dec, bad_ms, bad_ks; uint32_t first_bad; } job;

static void *run(void *arg) {
  job *j = arg;
  uint64_t lo = ((1ull << 32) * j->id) / nthreads, hi = ((1ull << 32) * (j->id + 1)) / nthreads;
  int32_t d[16];
  uint32_t v[64];
  for (uint64_t xx = lo; xx < hi; xx++) {
    uint32_t x = (uint32_t)xx;
    f_dec(&P, x, d);
    uint32_t rec = 0;
    int ok = 1;
    for (int r = 1; r <= P.l; r++) {
      if (d[r - 1] < -32 || d[r - 1] >= 32) ok = 0;
      rec += (uint32_t)d[r - 1] << (32 - 6 * r);
    }
    int32_t err = (int32_t)(x - rec);
    if (!ok || err < -(1 << 13) || err >= (1 << 13) || (rec & 0x3FFF)) { if (!j->bad_dec++) j->first_bad = x; }
    uint32_t xb = f_ms(x, P.N);
    int32_t e2 = (int32_t)(x - (xb << 21));
    if (xb >= 2048u || e2 < -(1 << 20) || e2 >= (1 << 20)) { if (!j->bad_ms++) j->first_bad = x; }
    f_ks(&P, x, v);
    uint32_t rk = 0;
    ok = 1;
    for (int p = 0; p < P.t; p++) { if (v[p] > 3) ok = 0; rk += v[p] << (30 - 2 * p); }
    int32_t e3 = (int32_t)(x - rk);
    if (!ok || e3 < -(1 << 15) || e3 >= (1 << 15)) { if (!j->bad_ks++) j->first_bad = x; }
  }
  return NULL;
}

int main(int argc, char **argv) {
  if (argc < 3) return 2;
  void *h = dlopen(argv[1], RTLD_NOW);
  if (!h) { fprintf(stderr, "dlopen: %s\n", dlerror()); return 2; }
  f_dec = dlsym(h, "or_decompose"); f_ms = dlsym(h, "or_modswitch"); f_ks = dlsym(h, "or_ks_digits");
  if (!f_dec || !f_ms || !f_ks) return 2;
  nthreads = atoi(argv[2]);
  if (nthreads < 1) nthreads = 1;
  pthread_t th[256]; job jobs[256];
  for (int i = 0; i < nthreads; i++) { jobs[i] = (job){i, 0, 0, 0, 0}; pthread_create(&th[i], NULL, run, &jobs[i]); }
  uint64_t bd = 0, bm = 0, bk = 0;
  for (int i = 0; i < nthreads; i++) {
    pthread_join(th[i], NULL);
    bd += jobs[i].bad_dec; bm += jobs[i].bad_ms; bk += jobs[i].bad_ks;
    if (jobs[i].bad_dec || jobs[i].bad_ms || jobs[i].bad_ks) printf("first failure near x=0x%08x\n", jobs[i].first_bad);
  }
  printf("checked 2^32 values: decomposition failures %llu, modswitch failures %llu, ks-digit failures %llu\n",
         (unsigned long long)bd, (unsigned long long)bm, (unsigned long long)bk);
  return (bd || bm || bk) ? 1 : 0;
}

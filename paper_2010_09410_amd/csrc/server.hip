// Continuous-batching server: the evaluating party serving many clients' circuits on one
// GPU (Sec. 4.1, the server evaluates for each client; Sec. 6.2(d), gates of a level are
// independent). Admitted circuits keep their wires resident in a device arena whose size is
// the memory budget; each iteration gathers the ready gates (the next level of every
// admitted circuit, round-robin, up to max_batch) into one batched launch sequence on the
// server's stream. Circuits may come with their own key set (each client's bootstrapping and
// key-switching keys): the batch is ordered by key set, the blind rotation reads each gate's
// key through a per-gate key index, and the key switch runs once per key set over its
// contiguous range. At most two batches are in flight, so host-side assembly and admission
// overlap device execution, and requests that arrive meanwhile join the next batch.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "vsp_internal.h"

using namespace vsp;
using Clock = std::chrono::steady_clock;

namespace {

constexpr size_t ROWB = (LWE_N + 1) * 4;  // bytes of one TLWE wire

struct Request {
  uint64_t ticket = 0;
  uint64_t ninputs = 0, ngates = 0;
  std::vector<vsp_gate_desc> gates;
  std::vector<uint32_t> inputs;
  std::vector<std::vector<uint32_t>> levels;  // gate indices per level
  size_t level = 0, pos = 0;                   // next gate to launch: levels[level][pos]
  uint64_t base = 0, rows = 0;                 // arena rows [base, base + rows)
  int64_t last_batch = -1;                     // batch that launched the final gate
  bool admitted = false, done = false;
  const vsp_keyset* keys = nullptr;            // NULL: the context's keys
  std::vector<uint32_t> result;
  Clock::time_point t_submit, t_done;
};

constexpr int kMaxBatchKeys = 64;  // distinct key sets in one batch

struct Slot {  // one in-flight batch
  uint8_t* h_ops = nullptr;
  uint32_t* h_idx = nullptr;
  uint16_t* h_kid = nullptr;
  const uint64_t** h_keytab = nullptr;
  uint8_t* d_ops = nullptr;
  uint32_t* d_idx = nullptr;
  uint16_t* d_kid = nullptr;
  const uint64_t** d_keytab = nullptr;
  const int8_t** h_tilekeys = nullptr;  // matrix-core key of each tile of a padded batch
  const int8_t** d_tilekeys = nullptr;
  uint32_t* d_abar = nullptr;
  uint32_t* d_tlwe1 = nullptr;
  hipEvent_t ev = nullptr;
  int64_t batch = -1;
  bool busy = false;
};

}  // namespace

struct vsp_server {
  vsp_context* ctx = nullptr;
  uint64_t budget = 0, max_batch = 0, arena_rows = 0;
  uint64_t cap = 0;  // launch entries per batch: max_batch plus tile padding of every key set
  uint32_t* arena = nullptr;
  std::map<uint64_t, uint64_t> free_rows;  // base -> length
  uint64_t resident = 0, peak = 0, gates_launched = 0, batches = 0, next_ticket = 1;
  int64_t batch_no = 0;
  std::deque<Request*> queue;
  std::vector<Request*> active;
  std::map<uint64_t, Request*> all;
  size_t rr = 0;
  Slot slots[2];
  void* mf_work = nullptr;  // matrix-core workspace (the batches run one after the other on st)
  struct Cand {
    uint8_t key, op;
    uint32_t i0, i1, io;
  };
  std::vector<Cand> cand;  // gates of the batch being assembled
  hipStream_t st = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  std::string error;
};

namespace {

bool arena_alloc(vsp_server* s, uint64_t rows, uint64_t* base) {
  for (auto it = s->free_rows.begin(); it != s->free_rows.end(); ++it) {
    if (it->second >= rows) {
      *base = it->first;
      const uint64_t rest = it->second - rows, nb = it->first + rows;
      s->free_rows.erase(it);
      if (rest) s->free_rows[nb] = rest;
      return true;
    }
  }
  return false;
}

void arena_free(vsp_server* s, uint64_t base, uint64_t rows) {
  auto it = s->free_rows.emplace(base, rows).first;
  auto nx = std::next(it);
  if (nx != s->free_rows.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    s->free_rows.erase(nx);
  }
  if (it != s->free_rows.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      s->free_rows.erase(it);
    }
  }
}

// Levelises a validated circuit: gate g goes to level 1 + max(level of its inputs).
vsp_status levelise(const vsp_gate_desc* gates, uint64_t ngates, uint64_t ninputs,
                    std::vector<std::vector<uint32_t>>& levels) {
  std::vector<uint32_t> lvl(ninputs + ngates, 0);
  for (uint64_t g = 0; g < ngates; g++) {
    const vsp_gate_desc& d = gates[g];
    const uint64_t self = ninputs + g;
    if (d.op > VSP_NOT) return fail(VSP_E_ARG, "gate " + std::to_string(g) + " has an invalid opcode");
    if (d.in0 >= self || (d.op != VSP_NOT && d.in1 >= self))
      return fail(VSP_E_ARG, "gate " + std::to_string(g) + " reads a wire that is not computed before it");
    uint32_t L = lvl[d.in0];
    if (d.op != VSP_NOT) L = std::max(L, lvl[d.in1]);
    lvl[self] = L + 1;
    if (levels.size() < L + 1) levels.resize(L + 1);
    levels[L].push_back((uint32_t)g);
  }
  return VSP_OK;
}

// Admits queued requests in arrival order while they fit (caller holds the lock).
void admit(vsp_server* s) {
  while (!s->queue.empty()) {
    Request* r = s->queue.front();
    uint64_t base;
    if (!arena_alloc(s, r->rows, &base)) break;
    r->base = base;
    // the host inputs stay alive until the request retires, so the asynchronous copy is safe
    if (r->ninputs)
      (void)hipMemcpyAsync(s->arena + base * (LWE_N + 1), r->inputs.data(), r->ninputs * ROWB, hipMemcpyHostToDevice,
                           s->st);
    r->admitted = true;
    s->resident += r->rows * ROWB;
    s->peak = std::max(s->peak, s->resident);
    s->active.push_back(r);
    s->queue.pop_front();
  }
}

// Completes requests whose last batch has finished (caller holds the lock).
void retire(vsp_server* s, int64_t finished_batch) {
  for (size_t i = 0; i < s->active.size();) {
    Request* r = s->active[i];
    const bool launched_all = r->level >= r->levels.size();
    if (launched_all && r->last_batch <= finished_batch) {
      const uint64_t n = r->ninputs + r->ngates;
      r->result.resize(n * (LWE_N + 1));
      if (n) (void)hipMemcpy(r->result.data(), s->arena + r->base * (LWE_N + 1), n * ROWB, hipMemcpyDeviceToHost);
      r->t_done = Clock::now();
      r->done = true;
      r->inputs.clear();
      r->inputs.shrink_to_fit();
      arena_free(s, r->base, r->rows);
      s->resident -= r->rows * ROWB;
      s->active.erase(s->active.begin() + i);
    } else {
      i++;
    }
  }
}

void worker_loop(vsp_server* s) {
  (void)hipSetDevice(s->ctx->device);
  int cur = 0;
  int64_t completed = -1;
  for (;;) {
    Slot& sl = s->slots[cur];
    if (sl.busy) {  // wait for the batch that used this slot two iterations ago
      (void)hipEventSynchronize(sl.ev);
      sl.busy = false;
      completed = std::max(completed, sl.batch);
    }
    std::unique_lock<std::mutex> lk(s->mu);
    retire(s, completed);
    admit(s);
    s->cv.notify_all();
    // gather ready gates: the next level of every active request, round-robin
    uint64_t nb = 0;
    const size_t na = s->active.size();
    std::vector<const vsp_keyset*> kset;
    s->cand.clear();
    for (size_t k = 0; k < na && nb < s->max_batch; k++) {
      Request* r = s->active[(s->rr + k) % na];
      if (r->level >= r->levels.size()) continue;
      // a request's next level may only follow its previous one in a later batch
      if (r->last_batch == s->batch_no) continue;
      size_t key = std::find(kset.begin(), kset.end(), r->keys) - kset.begin();
      if (key == kset.size()) {
        if (kset.size() == (size_t)kMaxBatchKeys) continue;  // this key set waits for the next batch
        kset.push_back(r->keys);
      }
      const auto& lv = r->levels[r->level];
      while (r->pos < lv.size() && nb < s->max_batch) {
        const vsp_gate_desc& d = r->gates[lv[r->pos]];
        s->cand.push_back({(uint8_t)key, (uint8_t)d.op, (uint32_t)(r->base + d.in0),
                           (uint32_t)(r->base + (d.op == VSP_NOT ? d.in0 : d.in1)),
                           (uint32_t)(r->base + r->ninputs + lv[r->pos])});
        nb++;
        r->pos++;
      }
      r->last_batch = s->batch_no;
      if (r->pos == lv.size()) {
        r->level++;
        r->pos = 0;
      }
    }
    if (na) s->rr = (s->rr + 1) % na;
    // lay the batch out grouped by key set (counting sort on the key index); when a key set
    // other than the context's takes part and the batch size calls for a matrix-core form, each
    // key set's range starts on a tile boundary (padding entries do nothing) and every tile
    // names its key set's byte-plane key
    const size_t nk = kset.size();
    std::vector<uint64_t> count(nk, 0), start(nk + 1, 0);
    for (const auto& c : s->cand) count[c.key]++;
    const bool keyed = nk > 1 || (nk == 1 && kset[0] != nullptr);
    bool padded = false;
    if (keyed && s->mf_work) {
      uint64_t nbp = 0;
      for (size_t k = 0; k < nk; k++) nbp += (count[k] + MF_TILE - 1) / MF_TILE * MF_TILE;
      padded = br_matrix_form(s->ctx->tune.br_waves(nbp));
    }
    for (size_t k = 0; k < nk; k++)
      start[k + 1] = start[k] + (padded ? (count[k] + MF_TILE - 1) / MF_TILE * MF_TILE : count[k]);
    const uint64_t nbl = start[nk];  // launched entries, padding included
    {
      const uint64_t M = s->cap;
      std::vector<uint64_t> fill(start.begin(), start.end() - 1);
      for (const auto& c : s->cand) {
        const uint64_t i = fill[c.key]++;
        sl.h_ops[i] = c.op;
        sl.h_kid[i] = (uint16_t)c.key;
        sl.h_idx[i] = c.i0;
        sl.h_idx[M + i] = c.i1;
        sl.h_idx[2 * M + i] = c.io;
      }
      for (size_t k = 0; k < nk; k++) {
        for (uint64_t i = fill[k]; i < start[k + 1]; i++) {
          sl.h_ops[i] = OP_SKIP;
          sl.h_kid[i] = (uint16_t)k;
          sl.h_idx[i] = sl.h_idx[M + i] = sl.h_idx[2 * M + i] = 0;
        }
        sl.h_keytab[k] = kset[k] ? kset[k]->bkn : s->ctx->bkn;
        if (padded)
          for (uint64_t t = start[k] / MF_TILE; t < start[k + 1] / MF_TILE; t++)
            sl.h_tilekeys[t] = kset[k] ? kset[k]->mf_key : s->ctx->mf_key;
      }
    }
    if (nb == 0) {
      const bool inflight = s->slots[0].busy || s->slots[1].busy;
      if (inflight) {
        lk.unlock();
        cur ^= 1;
        continue;
      }
      if (s->stop && s->queue.empty() && s->active.empty()) break;
      if (s->active.empty() || s->queue.empty()) s->cv.wait_for(lk, std::chrono::milliseconds(2));
      continue;
    }
    const int64_t b = s->batch_no++;
    s->gates_launched += nb;
    s->batches++;
    lk.unlock();
    hipStream_t st = s->st;
    const uint64_t M = s->cap;
    (void)hipMemcpyAsync(sl.d_ops, sl.h_ops, nbl, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(sl.d_idx, sl.h_idx, nbl * 4, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(sl.d_idx + M, sl.h_idx + M, nbl * 4, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(sl.d_idx + 2 * M, sl.h_idx + 2 * M, nbl * 4, hipMemcpyHostToDevice, st);
    if (nk > 1) {
      (void)hipMemcpyAsync(sl.d_kid, sl.h_kid, nbl * sizeof(uint16_t), hipMemcpyHostToDevice, st);
      (void)hipMemcpyAsync(sl.d_keytab, sl.h_keytab, nk * sizeof(void*), hipMemcpyHostToDevice, st);
    }
    if (padded)
      (void)hipMemcpyAsync(sl.d_tilekeys, sl.h_tilekeys, nbl / MF_TILE * sizeof(void*), hipMemcpyHostToDevice, st);
    hipError_t e = launch_gate_prologue(s->ctx, sl.d_ops, s->arena, s->arena, sl.d_idx, sl.d_idx + M, sl.d_idx + 2 * M,
                                        sl.d_abar, s->arena, nbl, st);
    if (e == hipSuccess)
      e = launch_blind_rotate(s->ctx, sl.d_ops, sl.d_abar, sl.d_tlwe1, nullptr, nbl, 0, st, sl.h_keytab[0],
                              nk > 1 ? sl.d_keytab : nullptr, nk > 1 ? sl.d_kid : nullptr, s->mf_work, false,
                              padded ? sl.d_tilekeys : nullptr);
    for (size_t k = 0; k < nk && e == hipSuccess; k++) {
      const uint64_t a = start[k];
      e = launch_keyswitch(s->ctx, sl.d_ops + a, sl.d_tlwe1 + a * (RING_N + 1), sl.d_idx + 2 * M + a, s->arena, count[k],
                           st, -1, kset[k] ? kset[k]->ksk : nullptr, kset[k] ? kset[k]->ks_mf : nullptr);
    }
    if (e == hipSuccess) e = hipEventRecord(sl.ev, st);
    if (e != hipSuccess) {
      std::lock_guard<std::mutex> g(s->mu);
      s->error = std::string("batch launch failed: ") + hipGetErrorString(e);
    }
    sl.batch = b;
    sl.busy = true;
    cur ^= 1;
  }
}

void free_server(vsp_server* s) {
  if (!s) return;
  (void)hipSetDevice(s->ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& sl : s->slots) {
    for (void* p : {(void*)sl.h_ops, (void*)sl.h_idx, (void*)sl.h_kid, (void*)sl.h_keytab, (void*)sl.h_tilekeys})
      if (p) (void)hipHostFree(p);
    for (void* p : {(void*)sl.d_ops, (void*)sl.d_idx, (void*)sl.d_kid, (void*)sl.d_keytab, (void*)sl.d_tilekeys,
                    (void*)sl.d_abar, (void*)sl.d_tlwe1})
      if (p) (void)hipFree(p);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
  }
  if (s->mf_work) (void)hipFree(s->mf_work);
  if (s->arena) (void)hipFree(s->arena);
  if (s->st) (void)hipStreamDestroy(s->st);
  for (auto& kv : s->all) delete kv.second;
  delete s;
}

}  // namespace

extern "C" {

vsp_status vsp_server_create(vsp_context* ctx, uint64_t mem_budget_bytes, uint64_t max_batch, vsp_server** out) {
  if (out == nullptr) return fail(VSP_E_ARG, "out is NULL");
  *out = nullptr;
  if (ctx == nullptr) return fail(VSP_E_ARG, "context is NULL");
  if (max_batch == 0 || max_batch > (1u << 20)) return fail(VSP_E_ARG, "max_batch must be in [1, 2^20]");
  const uint64_t rows = mem_budget_bytes / ROWB;
  if (rows == 0 || rows > 0xFFFFFFFFull) return fail(VSP_E_ARG, "memory budget out of range");
  auto* s = new vsp_server();
  s->ctx = ctx;
  s->budget = rows * ROWB;
  s->max_batch = max_batch;
  s->cap = max_batch + (uint64_t)MF_TILE * kMaxBatchKeys;
  s->arena_rows = rows;
  s->free_rows[0] = rows;
  auto bail = [&](vsp_status st) {
    free_server(s);
    return st;
  };
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return bail(hip_fail(e, "hipSetDevice"));
  if ((e = hipMalloc(&s->arena, s->budget)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(arena)"));
  if ((e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking)) != hipSuccess) return bail(hip_fail(e, "stream"));
  const uint64_t C = s->cap, tiles = C / MF_TILE + 1;
  for (auto& sl : s->slots) {
    if ((e = hipHostMalloc(&sl.h_ops, C)) != hipSuccess) return bail(hip_fail(e, "hipHostMalloc"));
    if ((e = hipHostMalloc(&sl.h_idx, 3 * C * 4)) != hipSuccess) return bail(hip_fail(e, "hipHostMalloc"));
    if ((e = hipHostMalloc(&sl.h_kid, C * sizeof(uint16_t))) != hipSuccess) return bail(hip_fail(e, "hipHostMalloc"));
    if ((e = hipHostMalloc(&sl.h_keytab, kMaxBatchKeys * sizeof(void*))) != hipSuccess)
      return bail(hip_fail(e, "hipHostMalloc"));
    if ((e = hipHostMalloc(&sl.h_tilekeys, tiles * sizeof(void*))) != hipSuccess) return bail(hip_fail(e, "hipHostMalloc"));
    if ((e = hipMalloc(&sl.d_kid, C * sizeof(uint16_t))) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
    if ((e = hipMalloc(&sl.d_keytab, kMaxBatchKeys * sizeof(void*))) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
    if ((e = hipMalloc(&sl.d_tilekeys, tiles * sizeof(void*))) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
    if ((e = hipMalloc(&sl.d_ops, C)) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
    if ((e = hipMalloc(&sl.d_idx, 3 * C * 4)) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
    if ((e = hipMalloc(&sl.d_abar, C * ROWB)) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
    if ((e = hipMalloc(&sl.d_tlwe1, C * (RING_N + 1) * 4)) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
    if ((e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming)) != hipSuccess) return bail(hip_fail(e, "event"));
  }
  if (ctx->mf_key && (e = hipMalloc(&s->mf_work, mf_work_bytes(C, true))) != hipSuccess)
    return bail(hip_fail(e, "hipMalloc(matrix-core workspace)"));
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return VSP_OK;
}

vsp_status vsp_server_submit(vsp_server* s, const vsp_gate_desc* gates, uint64_t ngates, uint64_t ninputs,
                             const uint32_t* h_inputs, uint64_t* ticket) {
  return vsp_server_submit_keyset(s, nullptr, gates, ngates, ninputs, h_inputs, ticket);
}

vsp_status vsp_server_submit_keyset(vsp_server* s, const vsp_keyset* keys, const vsp_gate_desc* gates,
                                    uint64_t ngates, uint64_t ninputs, const uint32_t* h_inputs, uint64_t* ticket) {
  if (s == nullptr || ticket == nullptr) return fail(VSP_E_ARG, "server or ticket is NULL");
  if (keys != nullptr && keys->ctx != s->ctx) return fail(VSP_E_ARG, "the key set belongs to another context");
  if (ngates > 0 && gates == nullptr) return fail(VSP_E_ARG, "gates is NULL");
  if (ninputs > 0 && h_inputs == nullptr) return fail(VSP_E_ARG, "h_inputs is NULL");
  auto* r = new Request();
  r->ninputs = ninputs;
  r->ngates = ngates;
  r->rows = ninputs + ngates;
  vsp_status st = levelise(gates, ngates, ninputs, r->levels);
  if (st) {
    delete r;
    return st;
  }
  if (r->rows * ROWB > s->budget) {
    delete r;
    return fail(VSP_E_CAPACITY, "circuit needs more device memory than the server budget");
  }
  r->gates.assign(gates, gates + ngates);
  r->inputs.assign(h_inputs, h_inputs + ninputs * (LWE_N + 1));
  r->keys = keys;
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) {
    delete r;
    return fail(VSP_E_STATE, "server is stopping");
  }
  r->ticket = s->next_ticket++;
  s->all[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  s->cv.notify_all();
  return VSP_OK;
}

vsp_status vsp_server_poll(vsp_server* s, uint64_t ticket, uint32_t* h_wires, int* done, double* latency_ms) {
  if (s == nullptr || done == nullptr) return fail(VSP_E_ARG, "server or done is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->error.empty()) return fail(VSP_E_HIP, s->error);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return fail(VSP_E_STATE, "unknown or already collected ticket");
  Request* r = it->second;
  *done = r->done ? 1 : 0;
  if (!r->done) return VSP_OK;
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  if (h_wires) {
    std::copy(r->result.begin(), r->result.end(), h_wires);
    s->all.erase(it);
    delete r;
  }
  return VSP_OK;
}

vsp_status vsp_server_stats(vsp_server* s, uint64_t* gates, uint64_t* batches, uint64_t* peak_bytes) {
  if (s == nullptr) return fail(VSP_E_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (gates) *gates = s->gates_launched;
  if (batches) *batches = s->batches;
  if (peak_bytes) *peak_bytes = s->peak;
  return VSP_OK;
}

vsp_status vsp_server_destroy(vsp_server* s) {
  if (s == nullptr) return VSP_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  free_server(s);
  return VSP_OK;
}

}  // extern "C"

// Request server for continuous batching (pc2_server_*, pc2_serve_*).
//
// Requests -- encryptions, aggregations and decryptions of vectors of any
// length under one key -- arrive one at a time.  Admission by memory, the
// cutting of requests into element groups and the two launch policies are
// the rules of serve_sched.hpp.  Each operation has its own persistent
// launcher (pc2_runner) on its own stream; whenever that stream is idle, the
// next scheduling pass forms one launch over up to tick_groups groups drawn
// from the admitted requests of the operation.  Requests that arrive while
// launches run join the next launch of their operation, and the three
// operations overlap on the device.  A request is complete when the launch
// holding its last group has finished (a HIP event on its stream).
//
// The server drives nothing by itself: every pc2_serve_* call makes one
// scheduling pass (retire finished launches, admit, launch on idle streams),
// so a caller that waits for results keeps calling pc2_serve_poll or
// pc2_serve_progress.  It uses the public runner calls only.
#include <hip/hip_runtime.h>

#include <chrono>
#include <memory>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/pc2.h"
#include "serve_sched.hpp"

namespace {

using pc2s::NOPS;
using pc2s::op_slot;
using pc2s::Piece;
using pc2s::Request;
constexpr uint32_t K_MAX = 128;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

struct pc2_server {
  pc2_ctx* ctx = nullptr;
  int device = 0;
  const pc2_sk* sk = nullptr;
  const pc2_pk* pk = nullptr;
  uint32_t L = 0;
  size_t max_requests = 0;
  pc2s::Sched sch;
  pc2_runner* runner[NOPS] = {};
  hipStream_t stream[NOPS] = {};
  hipEvent_t finished[NOPS] = {};
  bool busy[NOPS] = {};
  std::vector<Piece> tick[NOPS];
  std::vector<uint64_t> completed;  // finished ids not yet drained by pc2_serve_completed
  std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
  uint64_t next_id = 1;
  uint64_t launches = 0;
  // per-launch argument arrays and the retired requests, reused
  std::vector<pc2_job> jobs;
  std::vector<size_t> first, ngroups;
  std::vector<Request*> done;
};

namespace {

size_t request_bytes(const pc2_server* s, const pc2_job& j) {
  const size_t L = s->L, n = j.count;
  if (j.op == PC2_OP_ENCRYPT) return n * (4 * (size_t)j.m_limbs + 4 * L + 8 * L);
  if (j.op == PC2_OP_HOM_SUM) return n * 8 * L * ((size_t)j.K + 1);
  return n * (8 * L + 4 * L);
}

void note_finished(pc2_server* s, uint64_t id) {
  // ids that pc2_serve_poll already reported are dropped here, so the list
  // holds at most about twice the tracked requests
  if (s->completed.size() >= 2 * s->max_requests) {
    auto& c = s->completed;
    c.erase(std::remove_if(c.begin(), c.end(),
                           [s](uint64_t i) { return !s->requests.count(i); }),
            c.end());
  }
  s->completed.push_back(id);
}

// The launch of operation `op` finished: count its groups against their requests.
void retire(pc2_server* s, int op) {
  s->done.clear();
  pc2s::retire(s->sch, op, s->tick[op], s->done);
  for (Request* r : s->done) note_finished(s, r->id);
  s->tick[op].clear();
  s->busy[op] = false;
}

// One launch of operation `op` over the admitted requests' next groups.
int launch(pc2_server* s, int op) {
  auto& tick = s->tick[op];
  pc2s::form_launch(s->sch, op, now_s(), tick);
  if (tick.empty()) return PC2_OK;
  s->jobs.clear();
  s->first.clear();
  s->ngroups.clear();
  for (const Piece& p : tick) {
    s->jobs.push_back(p.req->job);
    s->first.push_back(p.first);
    s->ngroups.push_back(p.n);
  }
  int rc = pc2_runner_launch(s->runner[op], s->jobs.data(), s->first.data(), s->ngroups.data(),
                             s->jobs.size(), s->stream[op]);
  if (rc) {
    tick.clear();
    return rc;
  }
  if (hipEventRecord(s->finished[op], s->stream[op]) != hipSuccess) return PC2_E_DEVICE;
  pc2s::commit(tick);
  s->busy[op] = true;
  ++s->launches;
  return PC2_OK;
}

// Requests are cut into groups of the size the key's current encryption
// tile gives; a tile change (PC2_OPT_TILE, pc2_autotune) while requests of an
// operation are admitted would make the launcher read their group ranges in
// other units, so it is refused; with none admitted the new size is taken.
int refresh_group_sizes(pc2_server* s) {
  static const int ops[NOPS] = {PC2_OP_ENCRYPT, PC2_OP_HOM_SUM, PC2_OP_DECRYPT};
  for (int op = 0; op < NOPS; ++op) {
    uint32_t g = 0;
    if (pc2_runner_group_size(s->pk, ops[op], &g) != PC2_OK || g == 0) return PC2_E_UNSUPPORTED;
    if (g == s->sch.group_elems[op]) continue;
    if (!s->sch.active[op].empty()) return PC2_E_UNSUPPORTED;
    s->sch.group_elems[op] = g;
  }
  return PC2_OK;
}

// One scheduling pass: retire finished launches, admit, launch where idle.
int pass(pc2_server* s) {
  if (hipSetDevice(s->device) != hipSuccess) return PC2_E_DEVICE;
  for (int op = 0; op < NOPS; ++op) {
    if (!s->busy[op]) continue;
    const hipError_t q = hipEventQuery(s->finished[op]);
    if (q == hipSuccess) retire(s, op);
    else if (q != hipErrorNotReady) return PC2_E_DEVICE;
  }
  int rc = refresh_group_sizes(s);
  if (rc) return rc;
  pc2s::admit(s->sch, now_s());
  for (int op = 0; op < NOPS; ++op) {
    if (s->busy[op]) continue;
    rc = launch(s, op);
    if (rc) return rc;
  }
  return PC2_OK;
}

// Two device arrays overlap without being the same array of the same size
// (the only aliasing the library accepts between an output and an input).
bool partial_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  if (x + na <= y || y + nb <= x) return false;
  return !(x == y && na == nb);
}

// The op and the key always; the arrays only when there is work (count > 0).
int check_job(const pc2_server* s, const pc2_job& j) {
  const int slot = op_slot(j.op);
  if (slot < 0) return PC2_E_INVAL;
  if (slot == 2 ? j.sk != s->sk : j.pk != s->pk) return PC2_E_INVAL;
  if (j.count == 0) return PC2_OK;
  if (!j.out || (slot == 2 && !j.in0)) return PC2_E_INVAL;
  if (slot == 0 && (!j.in0 || !j.in1 || j.m_limbs < 1 || j.m_limbs > s->L)) return PC2_E_INVAL;
  if (slot == 1) {
    if (!j.inputs || j.K < 1 || j.K > K_MAX) return PC2_E_INVAL;
    for (uint32_t k = 0; k < j.K; ++k)
      if (!j.inputs[k] || (j.lengths && j.lengths[k] > j.count)) return PC2_E_INVAL;
  }
  const size_t n = j.count, L = s->L;
  if (slot == 0 && (partial_overlap(j.out, 8 * L * n, j.in0, 4 * (size_t)j.m_limbs * n) ||
                    partial_overlap(j.out, 8 * L * n, j.in1, 4 * L * n)))
    return PC2_E_INVAL;
  if (slot == 2 && partial_overlap(j.out, 4 * L * n, j.in0, 8 * L * n)) return PC2_E_INVAL;
  if (slot == 1)
    for (uint32_t k = 0; k < j.K; ++k) {  // input k holds lengths[k] rows (ragged) or count
      const size_t rows = j.lengths ? j.lengths[k] : n;
      if (partial_overlap(j.out, 8 * L * n, j.inputs[k], 8 * L * rows)) return PC2_E_INVAL;
    }
  return PC2_OK;
}

void destroy(pc2_server* s) {
  (void)hipSetDevice(s->device);
  for (int op = 0; op < NOPS; ++op) {
    if (s->stream[op]) (void)hipStreamSynchronize(s->stream[op]);
    if (s->runner[op]) (void)pc2_runner_destroy(s->runner[op]);
    if (s->finished[op]) (void)hipEventDestroy(s->finished[op]);
    if (s->stream[op]) (void)hipStreamDestroy(s->stream[op]);
  }
  delete s;
}

}  // namespace

extern "C" {

int pc2_server_create(pc2_ctx* ctx, const pc2_sk* sk, size_t hbm_budget, size_t tick_groups,
                      size_t max_requests, pc2_server** out) {
  if (!ctx || !sk || !out || tick_groups == 0 || max_requests == 0) return PC2_E_INVAL;
  *out = nullptr;
  const pc2_pk* pk = pc2_sk_public(sk);
  uint32_t nbits = 0, limbs = 0;
  pc2_ctx* key_ctx = nullptr;
  int device = 0;
  if (!pk || pc2_pk_info(pk, &nbits, &limbs) != PC2_OK ||
      pc2_pk_context(pk, &key_ctx, &device) != PC2_OK || key_ctx != ctx)
    return PC2_E_INVAL;
  if (hipSetDevice(device) != hipSuccess) return PC2_E_DEVICE;
  if (hbm_budget == 0) {  // half of the device memory free now
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return PC2_E_DEVICE;
    hbm_budget = free_b / 2;
  }
  pc2_server* s = new (std::nothrow) pc2_server();
  if (!s) return PC2_E_NOMEM;
  s->ctx = ctx;
  s->device = device;
  s->sk = sk;
  s->pk = pk;
  s->L = limbs;
  s->sch.budget = hbm_budget;
  s->sch.tick_groups = tick_groups;
  s->max_requests = max_requests;
  static const int ops[NOPS] = {PC2_OP_ENCRYPT, PC2_OP_HOM_SUM, PC2_OP_DECRYPT};
  int rc = PC2_OK;
  for (int op = 0; op < NOPS && !rc; ++op) {
    rc = pc2_runner_group_size(pk, ops[op], &s->sch.group_elems[op]);
    if (!rc && s->sch.group_elems[op] == 0) rc = PC2_E_UNSUPPORTED;
    if (!rc) rc = pc2_runner_create(ctx, ops[op], nbits, max_requests, tick_groups, &s->runner[op]);
    if (!rc && (hipStreamCreateWithFlags(&s->stream[op], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s->finished[op], hipEventDisableTiming) != hipSuccess))
      rc = PC2_E_DEVICE;
  }
  if (rc) {
    destroy(s);
    return rc;
  }
  s->jobs.reserve(max_requests);
  s->first.reserve(max_requests);
  s->ngroups.reserve(max_requests);
  *out = s;
  return PC2_OK;
}

int pc2_serve_submit(pc2_server* s, const pc2_job* job, uint64_t* req_id) {
  if (!s || !job || !req_id) return PC2_E_INVAL;
  int rc = check_job(s, *job);
  if (rc) return rc;
  if (s->requests.size() >= s->max_requests) return PC2_E_BUSY;
  auto r = std::unique_ptr<Request>(new (std::nothrow) Request());
  if (!r) return PC2_E_NOMEM;
  r->id = s->next_id++;
  r->slot = op_slot(job->op);
  r->job = *job;
  if (job->op == PC2_OP_HOM_SUM && job->count > 0) {
    r->inputs.assign(job->inputs, job->inputs + job->K);
    r->job.inputs = r->inputs.data();
    if (job->lengths) {
      r->lengths.assign(job->lengths, job->lengths + job->K);
      r->job.lengths = r->lengths.data();
    }
  }
  r->bytes = request_bytes(s, r->job);
  if (r->bytes > s->sch.budget) return PC2_E_NOMEM;  // could never be admitted
  Request* raw = r.get();
  s->requests.emplace(raw->id, std::move(r));
  *req_id = raw->id;
  if (raw->job.count == 0) {  // nothing to compute
    raw->state = pc2s::DONE;
    note_finished(s, raw->id);
    return PC2_OK;
  }
  raw->submitted = now_s();
  s->sch.waiting.push_back(raw);
  return pass(s);
}

int pc2_serve_poll(pc2_server* s, uint64_t req_id, int* done) {
  if (!s || !done) return PC2_E_INVAL;
  auto it = s->requests.find(req_id);
  if (it == s->requests.end()) return PC2_E_INVAL;
  const int rc = pass(s);
  if (rc) return rc;
  *done = it->second->state == pc2s::DONE;
  if (*done) s->requests.erase(it);
  return PC2_OK;
}

int pc2_serve_progress(pc2_server* s, size_t* pending) {
  if (!s) return PC2_E_INVAL;
  const int rc = pass(s);
  if (rc) return rc;
  if (pending) {
    size_t n = s->sch.waiting.size();
    for (int op = 0; op < NOPS; ++op) n += s->sch.active[op].size();
    *pending = n;
  }
  return PC2_OK;
}

int pc2_serve_completed(pc2_server* s, uint64_t* ids, size_t cap, size_t* n) {
  if (!s || !n || (cap && !ids)) return PC2_E_INVAL;
  size_t i = 0, k = 0;
  for (; i < s->completed.size() && k < cap; ++i) {
    auto it = s->requests.find(s->completed[i]);
    if (it == s->requests.end()) continue;  // already reported by pc2_serve_poll
    ids[k++] = s->completed[i];
    s->requests.erase(it);
  }
  s->completed.erase(s->completed.begin(), s->completed.begin() + i);
  *n = k;
  return PC2_OK;
}

int pc2_server_set_policy(pc2_server* s, int policy, double max_age_s) {
  if (!s || (policy != PC2_SERVE_FAIR && policy != PC2_SERVE_SHORTEST) || !(max_age_s >= 0))
    return PC2_E_INVAL;
  s->sch.policy = policy;
  s->sch.max_age = max_age_s;
  return PC2_OK;
}

int pc2_server_stats(const pc2_server* s, uint64_t* launches, size_t* max_bytes,
                     size_t* used_bytes) {
  if (!s) return PC2_E_INVAL;
  if (launches) *launches = s->launches;
  if (max_bytes) *max_bytes = s->sch.max_used;
  if (used_bytes) *used_bytes = s->sch.used;
  return PC2_OK;
}

int pc2_server_destroy(pc2_server* s) {
  if (!s) return PC2_E_INVAL;
  destroy(s);
  return PC2_OK;
}

}  // extern "C"

// Host-only simulation of the request server's scheduling passes, for the
// CPU tests: the server's own rules (serve_sched.hpp) over a virtual clock and
// a simulated device on which each operation is one in-order stream and a
// launch of g groups of operation op takes g * cost[op] seconds.  Each pass is
// what pc2_serve_progress does: retire finished launches, admit, launch on
// idle streams.  Built by tests/test_serve_scheduler.py with the host
// compiler; nothing here touches a device.
#include <cstddef>
#include <cstdint>
#include <memory>
#include <vector>

#include "../paper_2601_14980_amd/csrc/serve_sched.hpp"

namespace {
const int OPS[pc2s::NOPS] = {PC2_OP_ENCRYPT, PC2_OP_HOM_SUM, PC2_OP_DECRYPT};
}

extern "C" {

// n requests: arrival time, operation slot (0 encrypt, 1 hom_sum, 2 decrypt),
// element count and admission bytes.  A request whose bytes exceed the budget
// is refused as pc2_serve_submit refuses it (admitted = completed = -1).
// Outputs: admitted[i], completed[i] (the pass at which its last launch was
// seen finished), and a log of 5 int64 per launched piece: launch index,
// operation slot, request index, first group, groups.  Returns the number of
// log rows, -1 if log_cap rows were not enough, or -2 if the trace did not
// finish within 5e7 passes.
long serve_sim(int n, const double* arrival, const int* slot, const uint64_t* count,
               const uint64_t* bytes, uint64_t budget, uint64_t tick_groups, int policy,
               double max_age, const uint32_t* group_elems, const double* cost, double dt,
               double* admitted, double* completed, int64_t* log, long log_cap,
               uint64_t* max_used, double* makespan) {
  pc2s::Sched s;
  s.budget = budget;
  s.tick_groups = tick_groups;
  s.policy = policy;
  s.max_age = max_age;
  for (int op = 0; op < pc2s::NOPS; ++op) s.group_elems[op] = group_elems[op];
  std::vector<std::unique_ptr<pc2s::Request>> reqs(n);
  for (int i = 0; i < n; ++i) {
    reqs[i].reset(new pc2s::Request());
    reqs[i]->id = (uint64_t)i;
    reqs[i]->slot = slot[i];
    reqs[i]->job.op = OPS[slot[i]];
    reqs[i]->job.count = count[i];
    reqs[i]->bytes = bytes[i];
    admitted[i] = completed[i] = -1;
  }
  std::vector<pc2s::Piece> tick[pc2s::NOPS];
  bool busy[pc2s::NOPS] = {};
  double ends[pc2s::NOPS] = {};
  std::vector<pc2s::Request*> done;
  long rows = 0, launches = 0, passes = 0;
  const long max_passes = 50000000;
  int next = 0, live = 0;
  double t = 0;
  while (true) {
    while (next < n && arrival[next] <= t) {  // submissions (arrival order)
      pc2s::Request* r = reqs[next++].get();
      if (r->bytes > s.budget) continue;  // could never be admitted
      r->submitted = t;
      s.waiting.push_back(r);
      ++live;
    }
    for (int op = 0; op < pc2s::NOPS; ++op) {  // one scheduling pass
      if (!busy[op] || ends[op] > t) continue;
      done.clear();
      pc2s::retire(s, op, tick[op], done);
      for (pc2s::Request* r : done) {
        completed[r->id] = t;
        --live;
      }
      tick[op].clear();
      busy[op] = false;
    }
    pc2s::admit(s, t);
    for (pc2s::Request* r : s.active[0]) if (admitted[r->id] < 0) admitted[r->id] = r->admitted;
    for (pc2s::Request* r : s.active[1]) if (admitted[r->id] < 0) admitted[r->id] = r->admitted;
    for (pc2s::Request* r : s.active[2]) if (admitted[r->id] < 0) admitted[r->id] = r->admitted;
    for (int op = 0; op < pc2s::NOPS; ++op) {
      if (busy[op]) continue;
      pc2s::form_launch(s, op, t, tick[op]);
      if (tick[op].empty()) continue;
      size_t groups = 0;
      for (const pc2s::Piece& p : tick[op]) {
        if (rows >= log_cap) return -1;
        int64_t* row = log + 5 * rows++;
        row[0] = launches;
        row[1] = op;
        row[2] = (int64_t)p.req->id;
        row[3] = (int64_t)p.first;
        row[4] = (int64_t)p.n;
        groups += p.n;
      }
      pc2s::commit(tick[op]);
      ++launches;
      busy[op] = true;
      ends[op] = t + (double)groups * cost[op];
    }
    if (next >= n && live == 0) break;
    if (++passes > max_passes) return -2;  // a rule that never finishes the trace
    t += dt;
  }
  *max_used = s.max_used;
  *makespan = t;
  return rows;
}

}  // extern "C"

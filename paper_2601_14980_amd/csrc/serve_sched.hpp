// Scheduling rules of the request server (admission by memory, launch
// formation, retirement), free of any device call so that the same code runs
// under the server (serve.cpp) and under a host-only simulation.
//
// A request is admitted when the bytes of its inputs and output fit in the
// budget beside the requests already admitted.  An admitted request is cut
// into element groups (one wavefront's share each) of the size its
// operation's launcher uses.  A launch of one operation takes up to
// tick_groups groups from the admitted requests of that operation:
//   - shortest remaining first (PC2_SERVE_SHORTEST, the default): requests
//     in increasing order of the groups they have left, each taking all it
//     can, which minimises mean latency; a request admitted longer ago than
//     max_age goes first, oldest first, so long requests are not starved.
//     Admission lets later requests that fit pass one that does not, until
//     that one has waited max_age since it was submitted.
//   - fair share (PC2_SERVE_FAIR): an equal slice each, then what is left to
//     the oldest; admission is first come, first served.
// Time is passed in by the caller (seconds on any monotonic clock).
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <vector>

#include "../../include/pc2.h"

namespace pc2s {

constexpr int NOPS = 3;  // encrypt, hom_sum, decrypt

inline int op_slot(int op) {
  if (op == PC2_OP_ENCRYPT) return 0;
  if (op == PC2_OP_HOM_SUM) return 1;
  if (op == PC2_OP_DECRYPT) return 2;
  return -1;
}

enum : int { WAITING = 0, ACTIVE = 1, DONE = 2 };

struct Request {
  uint64_t id = 0;
  int slot = 0;
  int state = WAITING;
  pc2_job job{};
  std::vector<const uint32_t*> inputs;  // hom_sum: the caller's pointer array, copied
  std::vector<size_t> lengths;          // hom_sum: the caller's lengths, copied (may be empty)
  size_t bytes = 0;                     // inputs + output, for admission
  size_t groups = 0, next = 0, done = 0;
  double submitted = 0, admitted = 0;
};

struct Piece {
  Request* req;
  size_t first, n;
};

struct Sched {
  size_t budget = 0, used = 0, max_used = 0;
  size_t tick_groups = 0;
  int policy = PC2_SERVE_SHORTEST;
  double max_age = 1.0;
  uint32_t group_elems[NOPS] = {};
  std::deque<Request*> waiting;       // submitted, not admitted
  std::deque<Request*> active[NOPS];  // admitted, not finished
};

// Admit the waiting requests that the policy lets in at time t (see above).
inline void admit(Sched& s, double t) {
  const bool first_fit = s.policy == PC2_SERVE_SHORTEST;
  for (auto it = s.waiting.begin(); it != s.waiting.end();) {
    Request* r = *it;
    if (s.used + r->bytes > s.budget) {
      if (!first_fit || t - r->submitted > s.max_age) break;
      ++it;
      continue;
    }
    it = s.waiting.erase(it);
    const size_t g = s.group_elems[r->slot];
    r->groups = (r->job.count + g - 1) / g;
    r->state = ACTIVE;
    r->admitted = t;
    s.used += r->bytes;
    s.max_used = std::max(s.max_used, s.used);
    s.active[r->slot].push_back(r);
  }
}

// The pieces of the next launch of operation slot `op` at time t (empty when
// no admitted request of it has groups left).  Nothing is taken until
// commit() is called on the pieces.
inline void form_launch(const Sched& s, int op, double t, std::vector<Piece>& out) {
  out.clear();
  std::vector<Request*> reqs;
  for (Request* r : s.active[op])
    if (r->next < r->groups) reqs.push_back(r);
  if (reqs.empty()) return;
  size_t room = s.tick_groups;
  std::vector<size_t> take(reqs.size(), 0);
  if (s.policy == PC2_SERVE_SHORTEST) {
    // aged requests first (oldest first), then the rest by groups left
    std::stable_sort(reqs.begin(), reqs.end(), [&](const Request* a, const Request* b) {
      const bool oa = t - a->admitted > s.max_age, ob = t - b->admitted > s.max_age;
      if (oa != ob) return oa;
      if (oa) return a->admitted < b->admitted;
      return a->groups - a->next < b->groups - b->next;
    });
  } else {
    const size_t share = std::max<size_t>(1, room / reqs.size());
    for (size_t i = 0; i < reqs.size() && room; ++i) {
      take[i] = std::min({share, reqs[i]->groups - reqs[i]->next, room});
      room -= take[i];
    }
  }
  for (size_t i = 0; i < reqs.size() && room; ++i) {
    const size_t n = std::min(reqs[i]->groups - reqs[i]->next - take[i], room);
    take[i] += n;
    room -= n;
  }
  for (size_t i = 0; i < reqs.size(); ++i)
    if (take[i]) out.push_back({reqs[i], reqs[i]->next, take[i]});
}

// The launch holding these pieces was issued: their groups are taken.
inline void commit(const std::vector<Piece>& tick) {
  for (const Piece& p : tick) p.req->next += p.n;
}

// The launch holding these pieces finished: count its groups against their
// requests; the requests it completes leave the active list, release their
// bytes and are appended to `finished` (state DONE).
inline void retire(Sched& s, int op, const std::vector<Piece>& tick,
                   std::vector<Request*>& finished) {
  for (const Piece& p : tick) {
    Request* r = p.req;
    r->done += p.n;
    if (r->done == r->groups) {
      auto& q = s.active[op];
      q.erase(std::find(q.begin(), q.end(), r));
      r->state = DONE;
      s.used -= r->bytes;
      finished.push_back(r);
    }
  }
}

}  // namespace pc2s

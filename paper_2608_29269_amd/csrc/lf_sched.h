// lf_sched.h -- admission and tile planning of the relight server
// (continuous batching of forward renders of one resident scene; every
// rearrangement or relighting request re-renders the scene, Sec. 3.4 and the
// interaction loop of Sec. 1).  Plain C++17, no device code: the server
// (lf_server.hip) executes what it decides and reports completed work back.
//
// Model.
//  - A request is a number of primary rays (camera pixels) and a cost in
//    bytes (its working set, charged against the HBM budget while admitted).
//  - Admission is FIFO: the oldest waiting request is admitted when a slot is
//    free and the budget still holds its cost; nothing overtakes it.
//  - Every iteration (one batched wavefront pass) draws tiles of consecutive
//    rays from the admitted requests until the batch is full; only a
//    request's last tile may be ragged, every other tile is whole 128-ray
//    chunks.  Which requests go first is the policy:
//      kShortestFirst  smallest remaining work (rays x (1 + S)) first, each
//                      taking all it can (short requests finish in one pass);
//      kOldestFirst    admission order, each taking all it can (FIFO with
//                      backfill of the room the oldest leaves);
//      kRoundRobin     max(tile_rays, batch_rays / active) rays each,
//                      starting after the request served last.
//  - An iteration's tiles complete together; a request completes when all of
//    its rays have completed, which frees its slot and its budget.
//  - A request whose pass failed (fail()) gets no further tiles; it
//    completes, failed, once every tile already launched for it has retired,
//    so no pass still in flight writes into its outputs after it is reported.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <utility>
#include <vector>

namespace lf {

enum SchedPolicy { kShortestFirst = 0, kOldestFirst = 1, kRoundRobin = 2 };

struct SchedConfig {
  int policy = kShortestFirst;
  int max_slots = 16;
  int64_t budget = int64_t(16) << 30;
  int64_t tile_rays = 65536;   // multiple of chunk
  int64_t batch_rays = 262144; // multiple of chunk, >= tile_rays
  int max_pending = 1024;
  int64_t chunk = 128;
};

struct SchedTile {
  int slot;
  int64_t first;  // first ray id within the request
  int64_t n;      // rays
};

class Scheduler {
 public:
  enum Submit { kOk = 0, kBusy = 1, kTooBig = 2 };

  explicit Scheduler(const SchedConfig &c = SchedConfig()) : cfg_(c), slots_(c.max_slots) {}

  const SchedConfig &config() const { return cfg_; }

  // work_per_ray weighs a ray's cost for kShortestFirst (e.g. 1 + S)
  Submit submit(uint64_t ticket, int64_t rays, int64_t cost, int64_t work_per_ray = 1) {
    if (cost > cfg_.budget) return kTooBig;
    if ((int)pending_.size() >= cfg_.max_pending) return kBusy;
    pending_.push_back({ticket, rays, cost, work_per_ray});
    return kOk;
  }

  // FIFO admission into free slots within the budget; returns (slot, ticket).
  std::vector<std::pair<int, uint64_t>> admit() {
    std::vector<std::pair<int, uint64_t>> out;
    while (!pending_.empty()) {
      const Waiting &w = pending_.front();
      if (used_ + w.cost > cfg_.budget) break;
      int s = free_slot();
      if (s < 0) break;
      Slot &sl = slots_[s];
      sl.busy = true;
      sl.ticket = w.ticket;
      sl.rays = w.rays;
      sl.cost = w.cost;
      sl.next = 0;
      sl.done = 0;
      sl.failed = false;
      sl.wpr = w.wpr;
      sl.seq = seq_++;
      used_ += w.cost;
      out.push_back({s, w.ticket});
      pending_.pop_front();
    }
    return out;
  }

  // Tiles of the next iteration (empty if no admitted request has rays left
  // to schedule).  The padded size of the tiles never exceeds batch_rays.
  std::vector<SchedTile> plan() {
    std::vector<int> act;
    for (int s = 0; s < cfg_.max_slots; ++s)
      if (slots_[s].busy && slots_[s].next < slots_[s].rays) act.push_back(s);
    std::vector<SchedTile> tiles;
    if (act.empty()) return tiles;
    const int64_t ch = cfg_.chunk;
    int64_t quota = cfg_.batch_rays;
    size_t start = 0;
    if (cfg_.policy == kShortestFirst) {
      std::sort(act.begin(), act.end(), [&](int a, int b) {
        const Slot &x = slots_[a], &y = slots_[b];
        const int64_t wx = (x.rays - x.next) * x.wpr, wy = (y.rays - y.next) * y.wpr;
        return wx != wy ? wx < wy : x.seq < y.seq;
      });
    } else {
      std::sort(act.begin(), act.end(), [&](int a, int b) { return slots_[a].seq < slots_[b].seq; });
    }
    if (cfg_.policy == kRoundRobin) {
      quota = std::max(cfg_.tile_rays, round_up(cfg_.batch_rays / (int64_t)act.size(), ch));
      // start after the request served last in the previous iteration
      while (start < act.size() && slots_[act[start]].seq <= last_seq_) ++start;
      if (start == act.size()) start = 0;
    }
    int64_t room = cfg_.batch_rays;
    for (size_t i = 0; i < act.size(); ++i) {
      Slot &sl = slots_[act[(start + i) % act.size()]];
      const int64_t cap = std::min(quota, room);
      if (cap < ch) break;
      const int64_t rem = sl.rays - sl.next;
      const int64_t take = rem <= cap ? rem : (cap / ch) * ch;
      tiles.push_back({act[(start + i) % act.size()], sl.next, take});
      sl.next += take;
      room -= round_up(take, ch);
      last_seq_ = sl.seq;
    }
    return tiles;
  }

  // A pass holding tiles of the request in `slot` failed: plan no more of
  // its rays.  It completes (from retire) when the tiles already launched
  // have all retired, the failed pass's included.
  void fail(int slot) {
    if (slot < 0 || slot >= cfg_.max_slots) return;
    Slot &sl = slots_[slot];
    if (!sl.busy || sl.failed) return;
    sl.failed = true;
    sl.rays = sl.next;
  }

  bool failed(int slot) const { return slot >= 0 && slot < cfg_.max_slots && slots_[slot].failed; }

  // The iteration that held `tiles` has finished; returns (slot, ticket) of
  // the requests it completed (their slots and budget are released).
  std::vector<std::pair<int, uint64_t>> retire(const std::vector<SchedTile> &tiles) {
    std::vector<std::pair<int, uint64_t>> out;
    for (const SchedTile &t : tiles) {
      Slot &sl = slots_[t.slot];
      sl.done += t.n;
      if (sl.busy && sl.done == sl.rays) {
        sl.busy = false;
        used_ -= sl.cost;
        out.push_back({t.slot, sl.ticket});
      }
    }
    return out;
  }

  // Drops every waiting request (returns their tickets).
  std::vector<uint64_t> cancel_pending() {
    std::vector<uint64_t> out;
    for (const Waiting &w : pending_) out.push_back(w.ticket);
    pending_.clear();
    return out;
  }

  int active() const {
    int n = 0;
    for (const Slot &s : slots_) n += s.busy;
    return n;
  }
  int pending() const { return (int)pending_.size(); }
  int64_t used() const { return used_; }
  // admitted requests still holding rays that no iteration has taken yet
  bool has_unscheduled() const {
    for (const Slot &s : slots_)
      if (s.busy && s.next < s.rays) return true;
    return false;
  }

 private:
  struct Waiting {
    uint64_t ticket;
    int64_t rays, cost, wpr;
  };
  struct Slot {
    bool busy = false;
    bool failed = false;
    uint64_t ticket = 0;
    int64_t rays = 0, cost = 0, next = 0, done = 0, wpr = 1;
    uint64_t seq = 0;
  };
  static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
  int free_slot() const {
    for (int s = 0; s < cfg_.max_slots; ++s)
      if (!slots_[s].busy) return s;
    return -1;
  }

  SchedConfig cfg_;
  std::vector<Slot> slots_;
  std::deque<Waiting> pending_;
  int64_t used_ = 0;
  uint64_t seq_ = 1;
  uint64_t last_seq_ = 0;
};

}  // namespace lf

// C entry points over the relight server's scheduler (admission and tile
// planning), built by the CPU tests with the host compiler: the scheduler is
// plain C++ and runs here without a device.
#include <cstdint>
#include <vector>

#include "lf_sched.h"

extern "C" {

void *sched_create(int policy, int max_slots, int64_t budget, int64_t tile_rays, int64_t batch_rays,
                   int max_pending) {
  lf::SchedConfig c;
  c.policy = policy;
  c.max_slots = max_slots;
  c.budget = budget;
  c.tile_rays = tile_rays;
  c.batch_rays = batch_rays;
  c.max_pending = max_pending;
  c.chunk = 128;
  return new lf::Scheduler(c);
}

void sched_destroy(void *s) { delete (lf::Scheduler *)s; }

int sched_submit(void *s, uint64_t ticket, int64_t rays, int64_t cost, int64_t work_per_ray) {
  return (int)((lf::Scheduler *)s)->submit(ticket, rays, cost, work_per_ray);
}

// admitted (slot, ticket) pairs into out[2*i], out[2*i+1]; returns the count
int sched_admit(void *s, int64_t *out, int cap) {
  auto v = ((lf::Scheduler *)s)->admit();
  int n = 0;
  for (auto &p : v) {
    if (n < cap) {
      out[2 * n] = p.first;
      out[2 * n + 1] = (int64_t)p.second;
    }
    ++n;
  }
  return n;
}

// tiles of the next iteration as (slot, first, n) triples; returns the count
int sched_plan(void *s, int64_t *out, int cap) {
  auto v = ((lf::Scheduler *)s)->plan();
  int n = 0;
  for (auto &t : v) {
    if (n < cap) {
      out[3 * n] = t.slot;
      out[3 * n + 1] = t.first;
      out[3 * n + 2] = t.n;
    }
    ++n;
  }
  return n;
}

// retires the given tiles; completed (slot, ticket) pairs into out; returns the count
int sched_retire(void *s, const int64_t *tiles, int n_tiles, int64_t *out, int cap) {
  std::vector<lf::SchedTile> v;
  for (int i = 0; i < n_tiles; ++i) v.push_back({(int)tiles[3 * i], tiles[3 * i + 1], tiles[3 * i + 2]});
  auto done = ((lf::Scheduler *)s)->retire(v);
  int n = 0;
  for (auto &p : done) {
    if (n < cap) {
      out[2 * n] = p.first;
      out[2 * n + 1] = (int64_t)p.second;
    }
    ++n;
  }
  return n;
}

void sched_fail(void *s, int slot) { ((lf::Scheduler *)s)->fail(slot); }
int sched_failed(void *s, int slot) { return ((lf::Scheduler *)s)->failed(slot) ? 1 : 0; }
int sched_active(void *s) { return ((lf::Scheduler *)s)->active(); }
int sched_pending(void *s) { return ((lf::Scheduler *)s)->pending(); }
int64_t sched_used(void *s) { return ((lf::Scheduler *)s)->used(); }
}

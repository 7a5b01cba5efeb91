// lf_server.hip -- relight server: continuous batching of forward renders of
// the resident scene (Sec. 3.4, scene editing and relighting).  A host thread
// admits requests (lf_sched.h), stages each admitted request's transforms,
// camera and environment into its slot (instance records and importance
// sampling tables are built on the device) and launches batched wavefront
// passes over 128-ray chunks of the admitted requests.  Up to max_in_flight
// passes run at once, each on a lane of its own (stream and scratch), so the
// latency-bound tail of one pass overlaps the bulk of the next.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "lf_host.h"
#include "lf_sched.h"

namespace {

using lfh::DevBuf;
using Clock = std::chrono::steady_clock;

double now_ms() {
  return std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count();
}

enum TicketState { kWaiting = 0, kAdmitted = 1, kDone = 2 };

struct TicketRec {
  TicketState state = kWaiting;
  lf_status status = LF_OK;
  lf_request req{};
  int64_t rays = 0;
  double t_submit = 0.0, t_done = 0.0;
};

// Device state of one request slot.
struct SlotDev {
  DevBuf xf;      // [M*9] R then [M*3] t
  DevBuf inst;    // InstRec[n_inst]
  DevBuf bounds;  // 6 doubles
  DevBuf cam;     // CamArgs
  DevBuf tex, cdf_row, cdf_col, lum, rowsum, roww, scal;
  DevBuf status;  // status word of the request's instance records (invalid transforms)
  hipEvent_t staged = nullptr;  // recorded after the slot's staging on the staging lane's stream
};

// What the host reads back after each pass.
struct IterReadback {
  uint32_t status;
  uint32_t secondaries;
};

// One pass at a time on its own stream with its own scratch.
struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<lf::SchedTile> tiles;
  lf::ChunkDesc *h_chunks = nullptr;  // pinned
  IterReadback *h_rb = nullptr;       // pinned
  DevBuf d_chunks, rec1, rec2, queue, work, kbuf1, kbuf2, contrib, skeys, skeys2, svals, svals2, shist;
  DevBuf rbd;  // IterReadback on the device: the pass's status word, then its secondary-queue count
  DevBuf hint2;  // k-th distance per (ray, slot), written by the single-request kernels
};

}  // namespace

struct lf_server {
  lf_ctx *ctx = nullptr;
  lf_server_config cfg{};
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  bool kicked = false;  // a request was submitted since the last plan
  bool failed = false;
  lf_status fail_status = LF_OK;
  std::string err;
  lf::Scheduler sched;
  std::unordered_map<uint64_t, TicketRec> tickets;
  uint64_t next_ticket = 1;
  std::vector<uint64_t> slot_ticket;
  std::vector<lf_status> slot_fail;  // status of a failed pass of the slot's request, until it completes
  std::vector<SlotDev> slots;
  std::vector<Lane> lanes;
  lf::BatchSlot *h_slots = nullptr;   // [max_slots] pinned staging of the slot table
  lf::CamArgs *h_cams = nullptr;      // [max_slots] pinned staging of the cameras
  DevBuf d_slots;                     // BatchSlot[max_slots]
  int64_t max_chunks = 0;
  // statistics
  std::vector<double> lat;
  int64_t completed = 0, rejected = 0, rays_primary = 0, rays_secondary = 0, iterations = 0;
  double t_first = -1.0, t_last = -1.0;
};

namespace {

lf_status sfail(lf_server *s, lf_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  std::lock_guard<std::mutex> lk(s->mu);
  s->err = buf;
  return st;
}

int64_t request_cost(const lf_request &r) {
  const int64_t R = (int64_t)r.cam.w * r.cam.h;
  const int64_t H = r.env.h, W = r.env.w;
  return R * (32 + 44 * (int64_t)r.spp) + 12 * H * W + lfh::env_table_bytes((int)H, (int)W);
}

// Marks a ticket finished (mu held).
void finish_ticket(lf_server *s, uint64_t t, lf_status st, double when) {
  auto it = s->tickets.find(t);
  if (it == s->tickets.end() || it->second.state == kDone) return;
  it->second.state = kDone;
  it->second.status = st;
  it->second.t_done = when;
  if (st == LF_OK) {
    s->lat.push_back(when - it->second.t_submit);
    s->completed += 1;
    s->t_last = when;
  }
}

// True if p is device memory of the server's device, which the kernels can
// read in place (host memory is copied in; the caller keeps every buffer of
// a request valid until it completes either way).
bool device_resident(const void *p, int device) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice && at.device == device;
}

// Stages an admitted request into its slot on stream st: transforms and
// environment (read in place from device memory, else copied in), camera,
// instance records, sampling tables and the slot table entry; records the
// slot's staged event.  Every copy here runs as a small kernel that may wait
// for a compute unit the passes in flight hold, so device inputs are not copied.
bool stage_slot(lf_server *s, int slot, const lf_request &r, hipStream_t st) {
  lf_ctx *c = s->ctx;
  SlotDev &sd = s->slots[slot];
  const int M = c->n_inst - 1;
  const int H = r.env.h, W = r.env.w;
  const bool env_dev = device_resident(r.env.texels, c->device);
  const bool xf_dev = M > 0 && device_resident(r.xf.R, c->device) && device_resident(r.xf.t, c->device);
  if (!sd.xf.ensure(sizeof(float) * 12 * (M > 0 ? M : 1)) ||
      (!env_dev && !sd.tex.ensure(sizeof(float) * 3 * (size_t)H * W)) ||
      !lfh::ensure_env_tables(sd.cdf_row, sd.cdf_col, sd.lum, sd.rowsum, sd.roww, sd.scal, H, W))
    return false;
  const float *xR = nullptr, *xt = nullptr;
  if (M > 0 && xf_dev) {
    xR = r.xf.R;
    xt = r.xf.t;
  } else if (M > 0) {
    float *xf = sd.xf.as<float>();
    if (hipMemcpyAsync(xf, r.xf.R, sizeof(float) * 9 * M, hipMemcpyDefault, st) != hipSuccess ||
        hipMemcpyAsync(xf + 9 * M, r.xf.t, sizeof(float) * 3 * M, hipMemcpyDefault, st) != hipSuccess)
      return false;
    xR = xf;
    xt = xf + 9 * M;
  }
  const float *tex = r.env.texels;
  if (!env_dev) {
    if (hipMemcpyAsync(sd.tex.p, r.env.texels, sizeof(float) * 3 * (size_t)H * W, hipMemcpyDefault, st) !=
        hipSuccess)
      return false;
    tex = sd.tex.as<float>();
  }
  lf::CamArgs &ca = s->h_cams[slot];
  memset(&ca, 0, sizeof ca);
  if (lfh::camera_args(nullptr, r.cam, ca) != LF_OK) return false;  // validated at submission
  if (hipMemcpyAsync(sd.cam.p, &ca, sizeof ca, hipMemcpyHostToDevice, st) != hipSuccess) return false;
  lf::launch_fill_u32(sd.status.as<uint32_t>(), 0u, 1, st);
  lf::launch_instances(xR, xt, c->rootbox.as<float>(),
                       c->d_first.as<int32_t>(), c->d_n.as<int32_t>(), c->d_root.as<int32_t>(), c->n_inst,
                       sd.inst.as<lf::InstRec>(), sd.bounds.as<double>(), sd.status.as<uint32_t>(), st);
  lf::launch_env_tables(tex, H, W, s->cfg.params.flags, sd.cdf_row.as<double>(),
                        sd.cdf_col.as<double>(), sd.lum.as<double>(), sd.rowsum.as<double>(), sd.roww.as<double>(),
                        sd.scal.as<double>(), st);
  lf::BatchSlot &b = s->h_slots[slot];
  memset(&b, 0, sizeof b);
  b.inst = sd.inst.as<lf::InstRec>();
  b.bounds = sd.bounds.as<double>();
  b.cam = sd.cam.as<lf::CamArgs>();
  b.E.tex = tex;
  b.E.H = H;
  b.E.W = W;
  b.E.cdf_row = sd.cdf_row.as<double>();
  b.E.cdf_col = sd.cdf_col.as<double>();
  b.E.lum = sd.lum.as<double>();
  b.E.rowsum = sd.rowsum.as<double>();
  b.E.roww = sd.roww.as<double>();
  b.E.scal = sd.scal.as<double>();
  b.radiance = r.out.radiance;
  b.depth = r.out.depth;
  b.normal = r.out.normal;
  b.alpha = r.out.alpha;
  b.seed = r.seed;
  b.spp = r.spp;
  if (hipMemcpyAsync(s->d_slots.as<lf::BatchSlot>() + slot, &b, sizeof b, hipMemcpyHostToDevice, st) != hipSuccess)
    return false;
  if (hipEventRecord(sd.staged, st) != hipSuccess) return false;
  return hipGetLastError() == hipSuccess;
}

// Launches one batched pass over the tiles on lane L.  A pass that holds one
// whole request runs the single-request kernels instead (those of lf_render,
// with the request's slot data as their arguments): the same results, without
// each ray looking up its chunk and slot.
bool launch_pass(lf_server *s, Lane &L, const std::vector<lf::SchedTile> &tiles) {
  lf_ctx *c = s->ctx;
  hipStream_t st = L.stream;
  lf::ChunkDesc *hc = L.h_chunks;
  int64_t nch = 0;
  for (const lf::SchedTile &t : tiles) {
    // the slot may have been staged on another lane's stream
    if (hipStreamWaitEvent(st, s->slots[t.slot].staged, 0) != hipSuccess) return false;
    // scheduled positions are tiles x 128, so every chunk is one whole tile
    for (int64_t r = 0; r < t.n; r += lf::kChunk) {
      if (nch >= s->max_chunks) return false;  // the planner never exceeds the batch size
      hc[nch].slot = t.slot;
      hc[nch].pad = 0;
      hc[nch].tile = (t.first + r) / lf::kChunk;
      ++nch;
    }
  }
  if (hipMemcpyAsync(L.d_chunks.p, hc, sizeof(lf::ChunkDesc) * nch, hipMemcpyHostToDevice, st) != hipSuccess)
    return false;
  lf::RenderArgs a;
  memset(&a, 0, sizeof a);
  lfh::scene_view(c, a.S);
  lfh::trace_params(c, &s->cfg.params, a.P);
  a.P.abort = nullptr;  // server passes do not read the context's abort word
  a.P.spp = s->cfg.max_spp;  // replaced per request in the shading passes
  a.P.counters = nullptr;
  a.spp_stride = s->cfg.max_spp;
  a.R = nch * lf::kChunk;
  a.chunks = L.d_chunks.as<lf::ChunkDesc>();
  a.slots = s->d_slots.as<lf::BatchSlot>();
  a.rec1 = L.rec1.as<lf::SurfRec>();
  a.rec2 = L.rec2.as<lf::SurfRec>();
  a.queue = L.queue.as<lf::SecEntry>();
  a.queue_count = L.rbd.as<uint32_t>() + 1;
  a.work = L.work.as<uint32_t>();
  a.kbuf1 = L.kbuf1.as<uint32_t>();
  a.kbuf2 = L.kbuf2.as<uint32_t>();
  a.contrib = L.contrib.as<float>();
  a.status = L.rbd.as<uint32_t>();
  const bool sorted = !(s->cfg.params.flags & LF_FLAG_UNSORTED);
  a.order = sorted ? L.svals.as<int32_t>() : nullptr;
  const lf::SchedTile &t0 = tiles[0];
  const lf::CamArgs &hc0 = s->h_cams[t0.slot];
  const bool whole = tiles.size() == 1 && t0.first == 0 && t0.n == hc0.tiles[1] * lf::kChunk;
  const double *bounds6 = nullptr;
  if (whole) {
    const lf::BatchSlot &hs = s->h_slots[t0.slot];
    a.chunks = nullptr;
    a.slots = nullptr;
    a.S.inst = hs.inst;
    a.E = hs.E;
    a.P.seed = hs.seed;
    a.P.spp = hs.spp;
    a.spp_stride = hs.spp;
    a.rays.cams = hs.cam;
    a.n_tiles = hc0.tiles[1];
    a.R = hc0.first[1];
    a.radiance = hs.radiance;
    a.depth = hs.depth;
    a.normal = hs.normal;
    a.alpha = hs.alpha;
    a.hint2 = L.hint2.as<float>();
    a.use_hint = 0;
    bounds6 = hs.bounds;
  }
  lf::launch_fill_u32(a.queue_count, 0u, 1, st);
  lf::launch_trace1(a, st);
  lf::launch_composite1(a, false, st);
  lf::launch_shade1(a, false, st);
  if (sorted) {
    const int64_t cap = a.R * a.spp_stride;
    lf::launch_secondary_keys(a.queue, a.queue_count, cap, bounds6, a.chunks, a.slots, L.skeys.as<uint64_t>(),
                              L.svals.as<int32_t>(), st);
    lf::radix_sort(L.skeys.as<uint64_t>(), L.svals.as<int32_t>(), L.skeys2.as<uint64_t>(), L.svals2.as<int32_t>(),
                   L.shist.as<uint32_t>(), cap, st, 32);
  }
  lf::launch_trace2(a, st);
  lf::launch_composite2(a, st);
  lf::launch_shade2(a, false, st);
  lf::launch_resolve(a, st);
  // one copy for both words (each copy here is a small kernel that waits for
  // a compute unit the other lanes' traversals may hold)
  static_assert(sizeof(IterReadback) == 8, "readback layout");
  if (hipMemcpyAsync(L.h_rb, L.rbd.p, sizeof(IterReadback), hipMemcpyDeviceToHost, st) != hipSuccess) return false;
  lf::launch_fill_u32(a.status, 0u, 1, st);
  if (hipEventRecord(L.done, st) != hipSuccess) return false;
  L.tiles = tiles;
  L.busy = true;
  return hipGetLastError() == hipSuccess;
}

lf_status status_of(uint32_t st) {
  if (st & lf::kStatusOverflow) return LF_EOVERFLOW;
  if (st & lf::kStatusBadTransform) return LF_EINVAL;
  if (st & lf::kStatusBvhCorrupt) return LF_EDEVICE;
  return LF_OK;
}

// Completes the requests of lane L's finished pass.
bool retire(lf_server *s, Lane &L) {
  const double t = now_ms();
  const IterReadback rb = *L.h_rb;
  const lf_status st = status_of(rb.status);
  L.busy = false;
  std::lock_guard<std::mutex> lk(s->mu);
  s->rays_secondary += rb.secondaries;
  if (st != LF_OK) {
    // a device condition ends every request of the pass: none is planned
    // again, and each is reported once its other passes in flight are done
    for (const lf::SchedTile &tl : L.tiles) {
      s->sched.fail(tl.slot);
      if (s->slot_fail[tl.slot] == LF_OK) s->slot_fail[tl.slot] = st;
    }
    s->err = "device status set during a batched pass";
  }
  for (auto &done : s->sched.retire(L.tiles)) {
    lf_status rs = s->slot_fail[done.first];
    s->slot_fail[done.first] = LF_OK;
    if (rs == LF_OK) {
      // the request's own instance status (all of its passes have completed, so the word is final)
      uint32_t ist = 0;
      if (hipMemcpy(&ist, s->slots[done.first].status.p, 4, hipMemcpyDeviceToHost) != hipSuccess) return false;
      rs = status_of(ist);
      if (rs != LF_OK) s->err = "degenerate or non-finite object transform";
      else s->rays_primary += s->tickets[done.second].rays;
    }
    finish_ticket(s, done.second, rs, t);
  }
  L.tiles.clear();
  s->cv_done.notify_all();
  return true;
}

// Retires every lane whose pass has finished; returns how many (-1 on error).
int poll_lanes(lf_server *s) {
  int n = 0;
  for (Lane &L : s->lanes) {
    if (!L.busy) continue;
    const hipError_t q = hipEventQuery(L.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess || !retire(s, L)) return -1;
    ++n;
  }
  return n;
}

void fail_all(lf_server *s, lf_status st, const char *why) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->failed = true;
  s->fail_status = st;
  s->err = why;
  const double t = now_ms();
  for (auto &kv : s->tickets)
    if (kv.second.state != kDone) finish_ticket(s, kv.first, st, t);
  s->cv_done.notify_all();
}

void serve(lf_server *s) {
  if (hipSetDevice(s->ctx->device) != hipSuccess) {
    fail_all(s, LF_EDEVICE, "hipSetDevice failed on the server thread");
    return;
  }
  bool ok = true;
  while (ok) {
    Lane *free_lane = nullptr;
    int busy = 0;
    for (Lane &L : s->lanes) {
      if (L.busy) ++busy;
      else if (!free_lane) free_lane = &L;
    }
    std::vector<std::pair<int, uint64_t>> admitted;
    std::vector<lf_request> reqs;
    std::vector<lf::SchedTile> tiles;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (busy == 0) {
        s->cv_work.wait(lk, [&] { return s->stop || s->sched.pending() > 0 || s->sched.has_unscheduled(); });
        if (s->stop) break;
      }
      if (!s->stop && free_lane) {
        s->kicked = false;
        admitted = s->sched.admit();
        for (auto &ad : admitted) {
          s->slot_ticket[ad.first] = ad.second;
          TicketRec &tr = s->tickets[ad.second];
          tr.state = kAdmitted;
          reqs.push_back(tr.req);
        }
        tiles = s->sched.plan();
      }
    }
    if (free_lane) {
      for (size_t i = 0; i < admitted.size() && ok; ++i)
        ok = stage_slot(s, admitted[i].first, reqs[i], free_lane->stream);
      if (!ok) break;
    }
    if (!tiles.empty()) {
      ok = launch_pass(s, *free_lane, tiles);
      if (!ok) break;
      std::lock_guard<std::mutex> lk(s->mu);
      s->iterations += 1;
      continue;  // fill the other lanes before waiting
    }
    if (busy == 0) continue;
    // every lane busy, or nothing new to launch: wait until a pass finishes
    int n = 0;
    while (ok && (n = poll_lanes(s)) == 0) {
      std::unique_lock<std::mutex> lk(s->mu);
      // wake early for new work when a lane is free
      if (free_lane && (s->kicked || s->sched.has_unscheduled())) break;
      s->cv_work.wait_for(lk, std::chrono::microseconds(100));
    }
    if (n < 0) ok = false;
  }
  // drain
  for (Lane &L : s->lanes) {
    if (!L.busy) continue;
    if (hipEventSynchronize(L.done) != hipSuccess || !retire(s, L)) ok = false;
  }
  if (!ok) {
    const hipError_t e = hipGetLastError();
    char buf[256];
    snprintf(buf, sizeof buf, "server pass failed: %s", hipGetErrorString(e));
    fail_all(s, LF_EDEVICE, buf);
  }
  for (Lane &L : s->lanes) (void)hipStreamSynchronize(L.stream);
}

void free_server(lf_server *s) {
  for (Lane &L : s->lanes) {
    if (L.stream) {
      (void)hipStreamSynchronize(L.stream);
      (void)hipStreamDestroy(L.stream);
    }
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.h_chunks) (void)hipHostFree(L.h_chunks);
    if (L.h_rb) (void)hipHostFree(L.h_rb);
  }
  for (SlotDev &sd : s->slots)
    if (sd.staged) (void)hipEventDestroy(sd.staged);
  if (s->h_slots) (void)hipHostFree(s->h_slots);
  if (s->h_cams) (void)hipHostFree(s->h_cams);
  delete s;
}

}  // namespace

extern "C" {

void lf_server_config_default(lf_server_config *cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof *cfg);
  cfg->max_slots = 16;
  cfg->hbm_budget_bytes = (int64_t)16 << 30;
  cfg->tile_rays = 65536;
  cfg->batch_rays = 1048576;
  cfg->max_spp = 4;
  cfg->max_pending = 4096;
  cfg->policy = LF_SCHED_OLDEST_FIRST;
  cfg->max_in_flight = 2;
  lf_params_default(&cfg->params);
}

lf_status lf_server_create(lf_ctx *c, const lf_server_config *cfg, lf_server **out) {
  if (!c || !out) return LF_EINVAL;
  *out = nullptr;
  if (!cfg) return lfh::fail(c, LF_EINVAL, "config is NULL");
  if (!c->has_scene) return lfh::fail(c, LF_EINVAL, "no scene set");
  if (cfg->max_slots < 1 || cfg->max_slots > 64) return lfh::fail(c, LF_EINVAL, "max_slots not in 1..64");
  if (cfg->tile_rays < lf::kChunk || cfg->tile_rays % lf::kChunk || cfg->batch_rays < cfg->tile_rays ||
      cfg->batch_rays % lf::kChunk)
    return lfh::fail(c, LF_EINVAL, "tile_rays and batch_rays must be multiples of %d with batch >= tile", lf::kChunk);
  if (cfg->max_spp < 1 || cfg->max_spp > 64) return lfh::fail(c, LF_EINVAL, "max_spp not in 1..64");
  if (cfg->max_pending < 1 || cfg->hbm_budget_bytes < 1) return lfh::fail(c, LF_EINVAL, "invalid queue or budget");
  if (cfg->policy < LF_SCHED_SHORTEST_FIRST || cfg->policy > LF_SCHED_ROUND_ROBIN)
    return lfh::fail(c, LF_EINVAL, "unknown scheduling policy %d", cfg->policy);
  if (cfg->max_in_flight < 1 || cfg->max_in_flight > 4) return lfh::fail(c, LF_EINVAL, "max_in_flight not in 1..4");
  lf_params p = cfg->params;
  p.spp = cfg->max_spp;
  lf_status st = lfh::validate_params(c, &p);
  if (st) return st;
  if (p.flags & (LF_FLAG_COUNT | LF_FLAG_NO_SECONDARY | LF_FLAG_NEE))
    return lfh::fail(c, LF_EUNSUPPORTED, "LF_FLAG_COUNT, LF_FLAG_NO_SECONDARY and LF_FLAG_NEE are not served");
  if ((int64_t)cfg->batch_rays * cfg->max_spp >= (int64_t)INT32_MAX)
    return lfh::fail(c, LF_EUNSUPPORTED, "batch_rays x max_spp too large");
  if (!lfh::set_device(c)) return lfh::fail(c, LF_EDEVICE, "hipSetDevice");
  const double sig2 = p.support_sigma * p.support_sigma;
  if (p.alpha_min != c->built_alpha_min || sig2 != c->built_sig2) {
    if (c->servers > 0) return lfh::fail(c, LF_EBUSY, "another server serves other tracing constants");
    if ((st = lfh::refit_impl(c, p.alpha_min, sig2))) return st;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return lfh::check_hip(c, "server create");

  lf_server *s = new lf_server();
  s->ctx = c;
  s->cfg = *cfg;
  lf::SchedConfig sc;
  sc.policy = cfg->policy;
  sc.max_slots = cfg->max_slots;
  sc.budget = cfg->hbm_budget_bytes;
  sc.tile_rays = cfg->tile_rays;
  sc.batch_rays = cfg->batch_rays;
  sc.max_pending = cfg->max_pending;
  sc.chunk = lf::kChunk;
  s->sched = lf::Scheduler(sc);
  s->slot_ticket.assign(cfg->max_slots, 0);
  s->slot_fail.assign(cfg->max_slots, LF_OK);
  s->slots = std::vector<SlotDev>(cfg->max_slots);
  s->lanes = std::vector<Lane>(cfg->max_in_flight);
  const int64_t B = cfg->batch_rays;
  const int64_t BS = B * cfg->max_spp;
  s->max_chunks = B / lf::kChunk;
  bool ok = hipHostMalloc((void **)&s->h_slots, sizeof(lf::BatchSlot) * cfg->max_slots, hipHostMallocDefault) ==
            hipSuccess;
  ok = ok && hipHostMalloc((void **)&s->h_cams, sizeof(lf::CamArgs) * cfg->max_slots, hipHostMallocDefault) ==
                 hipSuccess;
  ok = ok && s->d_slots.ensure(sizeof(lf::BatchSlot) * cfg->max_slots);
  const int M = c->n_inst - 1;
  for (int i = 0; i < cfg->max_slots && ok; ++i) {
    SlotDev &sd = s->slots[i];
    ok = hipEventCreateWithFlags(&sd.staged, hipEventDisableTiming) == hipSuccess &&
         sd.xf.ensure(sizeof(float) * 12 * (M > 0 ? M : 1)) && sd.inst.ensure(sizeof(lf::InstRec) * c->n_inst) &&
         sd.bounds.ensure(6 * sizeof(double)) && sd.cam.ensure(sizeof(lf::CamArgs)) && sd.status.ensure(4) &&
         sd.tex.ensure(sizeof(float) * 3 * 256 * 512) &&
         lfh::ensure_env_tables(sd.cdf_row, sd.cdf_col, sd.lum, sd.rowsum, sd.roww, sd.scal, 256, 512);
  }
  for (Lane &L : s->lanes) {
    if (!ok) break;
    ok = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&L.done, hipEventDisableTiming) == hipSuccess &&
         hipHostMalloc((void **)&L.h_chunks, sizeof(lf::ChunkDesc) * s->max_chunks, hipHostMallocDefault) ==
             hipSuccess &&
         hipHostMalloc((void **)&L.h_rb, sizeof(IterReadback), hipHostMallocDefault) == hipSuccess &&
         L.d_chunks.ensure(sizeof(lf::ChunkDesc) * s->max_chunks) && L.rec1.ensure(sizeof(lf::SurfRec) * B) &&
         L.rec2.ensure(sizeof(lf::SurfRec) * BS) && L.queue.ensure(sizeof(lf::SecEntry) * BS) &&
         L.rbd.ensure(sizeof(IterReadback)) && L.work.ensure(sizeof(uint32_t) * lf::kPoolParts) &&
         L.kbuf1.ensure(sizeof(uint32_t) * 2 * lf::kbucket(s->cfg.params.k) * B) &&
         L.kbuf2.ensure(sizeof(uint32_t) * 2 * lf::kbucket(s->cfg.params.k) * BS) &&
         L.contrib.ensure(sizeof(float) * 3 * BS) && L.skeys.ensure(8 * BS) && L.skeys2.ensure(8 * BS) &&
         L.svals.ensure(4 * BS) && L.svals2.ensure(4 * BS) && L.shist.ensure(4 * lf::radix_sort_hist_words(BS)) &&
         L.hint2.ensure(sizeof(float) * BS);
    if (ok) {
      lf::launch_fill_u32(L.rbd.as<uint32_t>(), 0u, 2, L.stream);
      ok = hipStreamSynchronize(L.stream) == hipSuccess;
    }
  }
  if (!ok) {
    (void)hipGetLastError();
    free_server(s);
    return lfh::fail(c, LF_ENOMEM, "server buffers (batch of %lld rays x %d samples, %d lanes)", (long long)B,
                     cfg->max_spp, cfg->max_in_flight);
  }
  c->servers += 1;
  s->worker = std::thread(serve, s);
  *out = s;
  return LF_OK;
}

lf_status lf_server_submit(lf_server *s, const lf_request *r, uint64_t *ticket) {
  if (!s) return LF_EINVAL;
  if (!r || !ticket) return sfail(s, LF_EINVAL, "request or ticket is NULL");
  const int M = s->ctx->n_inst - 1;
  const lf_camera &cm = r->cam;
  if (cm.w < 1 || cm.h < 1 || !(cm.fov_y_deg > 0.f && cm.fov_y_deg < 180.f))
    return sfail(s, LF_EINVAL, "invalid camera");
  for (int k = 0; k < 12; ++k)
    if (!std::isfinite(cm.pose[k])) return sfail(s, LF_EINVAL, "non-finite camera pose");
  if ((int64_t)cm.w * cm.h >= (int64_t)INT32_MAX) return sfail(s, LF_EUNSUPPORTED, "camera too large");
  if (r->spp < 1 || r->spp > s->cfg.max_spp) return sfail(s, LF_EINVAL, "spp=%d not in 1..%d", r->spp, s->cfg.max_spp);
  if (!r->env.texels || r->env.h < 1 || r->env.w < 1 || r->env.h > 8192 || r->env.w > 8192)
    return sfail(s, LF_EINVAL, "invalid environment map");
  if (M > 0 && (!r->xf.R || !r->xf.t)) return sfail(s, LF_EINVAL, "scene has %d objects but no transforms", M);
  if (!r->out.radiance || !r->out.depth || !r->out.normal || !r->out.alpha)
    return sfail(s, LF_EINVAL, "radiance, depth, normal and alpha outputs are required");
  if (r->out.hit_idx || r->out.sec_hit_idx) return sfail(s, LF_EUNSUPPORTED, "the server does not return hit lists");
  const int64_t cost = request_cost(*r);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->failed) return s->fail_status;
  if (s->stop) return LF_EBUSY;
  const uint64_t t = s->next_ticket;
  // scheduled in whole 16x8-pixel tiles (128 positions each, lanes outside the image idle)
  const int64_t positions = (int64_t)((cm.w + 15) / 16) * ((cm.h + 7) / 8) * lf::kChunk;
  const lf::Scheduler::Submit res = s->sched.submit(t, positions, cost, 1 + (int64_t)r->spp);
  if (res != lf::Scheduler::kOk) {
    s->rejected += 1;
    if (res == lf::Scheduler::kBusy) {
      s->err = "server queue full";
      return LF_EBUSY;
    }
    s->err = "request working set exceeds the HBM budget";
    return LF_EUNSUPPORTED;
  }
  s->next_ticket += 1;
  TicketRec &tr = s->tickets[t];
  tr.req = *r;
  tr.rays = (int64_t)cm.w * cm.h;
  tr.t_submit = now_ms();
  if (s->t_first < 0.0) s->t_first = tr.t_submit;
  *ticket = t;
  s->kicked = true;
  s->cv_work.notify_one();
  return LF_OK;
}

lf_status lf_server_poll(lf_server *s, uint64_t ticket, int *done) {
  if (!s) return LF_EINVAL;
  if (!done) return sfail(s, LF_EINVAL, "done is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) {
    s->err = "unknown ticket";
    return LF_EINVAL;
  }
  *done = it->second.state == kDone;
  return it->second.state == kDone ? it->second.status : LF_OK;
}

lf_status lf_server_wait(lf_server *s, uint64_t ticket) {
  if (!s) return LF_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) {
    s->err = "unknown ticket";
    return LF_EINVAL;
  }
  s->cv_done.wait(lk, [&] { return it->second.state == kDone; });
  return it->second.status;
}

lf_status lf_server_latency(lf_server *s, uint64_t ticket, double *ms) {
  if (!s) return LF_EINVAL;
  if (!ms) return sfail(s, LF_EINVAL, "ms is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end() || it->second.state != kDone) {
    s->err = "unknown or unfinished ticket";
    return LF_EINVAL;
  }
  *ms = it->second.t_done - it->second.t_submit;
  return it->second.status;
}

lf_status lf_server_stats_get(lf_server *s, lf_server_stats *out) {
  if (!s) return LF_EINVAL;
  if (!out) return sfail(s, LF_EINVAL, "stats is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  memset(out, 0, sizeof *out);
  std::vector<double> v = s->lat;
  std::sort(v.begin(), v.end());
  auto rank = [&](double q) {
    if (v.empty()) return 0.0;
    size_t i = (size_t)std::ceil(q * (double)v.size());
    i = i < 1 ? 1 : (i > v.size() ? v.size() : i);
    return v[i - 1];
  };
  out->p50_ms = rank(0.50);
  out->p99_ms = rank(0.99);
  out->completed = s->completed;
  out->rejected = s->rejected;
  out->rays_primary = s->rays_primary;
  out->rays_secondary = s->rays_secondary;
  out->iterations = s->iterations;
  const double span = s->t_last - s->t_first;
  out->rays_per_s = span > 0.0 ? (double)(s->rays_primary + s->rays_secondary) / (span * 1e-3) : 0.0;
  return LF_OK;
}

const char *lf_server_last_error(lf_server *s) {
  if (!s) return "null server";
  std::lock_guard<std::mutex> lk(s->mu);
  thread_local std::string copy;
  copy = s->err;
  return copy.c_str();
}

void lf_server_destroy(lf_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    const double t = now_ms();
    for (auto &kv : s->tickets)
      if (kv.second.state != kDone) finish_ticket(s, kv.first, LF_EBUSY, t);
    s->cv_done.notify_all();
  }
  (void)hipSetDevice(s->ctx->device);
  s->ctx->servers -= 1;
  free_server(s);
}

}  // extern "C"

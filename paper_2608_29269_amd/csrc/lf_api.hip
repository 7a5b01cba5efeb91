// lf_api.hip -- host runtime behind include/lightfuse.h: context, argument
// validation, library-owned device memory, scene build/refit and the launch
// sequences of the forward and backward passes.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "lf_host.h"
#include "lf_kernels.h"

namespace lfh {

lf_status fail(lf_ctx *c, lf_status st, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return st;
}

lf_status check_hip(lf_ctx *c, const char *where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, LF_EDEVICE, "%s: %s", where, hipGetErrorString(e));
  return LF_OK;
}

bool set_device(lf_ctx *c) { return hipSetDevice(c->device) == hipSuccess; }

}  // namespace lfh

using lfh::check_hip;
using lfh::fail;
using lfh::set_device;
using lfh::kPiHost;

namespace {

hipEvent_t take_event(lf_ctx *c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// Names of the phases (lf_profile_enable), also the roctx ranges that
// bracket their host-side launches for a tracer's marker view.
const char *const kPhaseName[LF_NUM_PHASES] = {
    "lf:refit",          "lf:state_env",  "lf:trace1",    "lf:shade1",     "lf:sort2",       "lf:trace2",
    "lf:shade2",         "lf:resolve",    "lf:replay_primary", "lf:replay_secondary", "lf:adj_shade", "lf:unused",
    "lf:zero_grads",     "lf:loss",       "lf:composite1", "lf:composite2", "lf:adj_hits"};

// Brackets one phase with a roctx range and, when profiling is enabled, with
// events on the stream.
struct Phase {
  lf_ctx *c;
  int id;
  hipEvent_t a = nullptr, b = nullptr;
  Phase(lf_ctx *c_, int id_) : c(c_), id(id_) {
    roctxRangePushA(kPhaseName[id]);
    if (!c->profiling) return;
    a = take_event(c);
    b = take_event(c);
    if (a) (void)hipEventRecord(a, c->stream);
  }
  ~Phase() {
    roctxRangePop();
    if (!c->profiling || !a || !b) return;
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back({id, {a, b}});
  }
};

}  // namespace

namespace lfh {

lf_status refit_impl(lf_ctx *c, double alpha_min, double sig2) {
  ++c->scene_epoch;
  c->sig_valid = false;
  Phase ph(c, 0);
  lf::launch_refit(c->s, alpha_min, sig2, c->perm.as<int32_t>(), c->leaf_parent.as<int32_t>(),
                   c->node_parent.as<int32_t>(), c->node_order.as<int32_t>(), c->h_level_off, c->n_nodes, c->n_inst,
                   c->nodes.as<lf::BNode>(), c->rec.as<lf::TraceRec>(), c->filt.as<lf::FiltRec>(),
                   c->leafbox.as<float>(), c->rootbox.as<float>(), c->status.as<uint32_t>(), c->stream);
  lf::launch_wide_quantize(c->nodes.as<lf::BNode>(), c->winfo.as<lf::WideInfo>(), c->n_wide, c->n_nodes,
                           c->qnodes.as<lf::QNode>(), c->status.as<uint32_t>(), c->stream);
  c->built_alpha_min = alpha_min;
  c->built_sig2 = sig2;
  return check_hip(c, "refit");
}

lf_status validate_params(lf_ctx *c, const lf_params *p) {
  if (!p) return fail(c, LF_EINVAL, "params is NULL");
  if (p->k < 1 || p->k > 64) return fail(c, p->k > 64 ? LF_EUNSUPPORTED : LF_EINVAL, "k=%d not in 1..64", p->k);
  if (p->spp < 1 || p->spp > 64) return fail(c, LF_EINVAL, "spp=%d not in 1..64", p->spp);
  if (!(p->alpha_min > 0.0) || !(p->alpha_cap > 0.0 && p->alpha_cap < 1.0) || !(p->support_sigma > 0.0) ||
      !(p->eps >= 0.0) || !(p->t_min >= 0.0) || !std::isfinite(p->secondary_offset))
    return fail(c, LF_EINVAL, "invalid tracing constants");
  if (p->flags & ~0x3FFu) return fail(c, LF_EINVAL, "unknown flags 0x%x", p->flags);
  return LF_OK;
}

lf_status camera_args(lf_ctx *c, const lf_camera &cm, lf::CamArgs &ca) {
  if (cm.w < 1 || cm.h < 1 || !(cm.fov_y_deg > 0.f && cm.fov_y_deg < 180.f))
    return fail(c, LF_EINVAL, "invalid camera");
  const int i = ca.n_cams;
  if (i >= LF_MAX_CAMERAS) return fail(c, LF_EINVAL, "at most %d cameras per call", LF_MAX_CAMERAS);
  for (int k = 0; k < 12; ++k) {
    if (!std::isfinite(cm.pose[k])) return fail(c, LF_EINVAL, "non-finite camera pose");
    ca.pose[i][k] = cm.pose[k];
  }
  ca.tan_half[i] = (float)std::tan((double)cm.fov_y_deg * kPiHost / 360.0);
  ca.w[i] = cm.w;
  ca.h[i] = cm.h;
  ca.first[i + 1] = ca.first[i] + (int64_t)cm.w * cm.h;
  ca.tiles[i + 1] = ca.tiles[i] + (int64_t)((cm.w + 15) / 16) * ((cm.h + 7) / 8);
  ca.n_cams = i + 1;
  return LF_OK;
}

void scene_view(const lf_ctx *c, lf::SceneView &S) {
  S.rec = c->rec.as<lf::TraceRec>();
  S.filt = c->filt.as<lf::FiltRec>();
  S.nodes = c->qnodes.as<lf::QNode>();
  S.inst = nullptr;
  S.n_inst = c->n_inst;
  S.n_rec = (int32_t)c->s.n;
  S.n_nodes = (int32_t)c->n_wide;
  S.mu = c->s.mu; S.q = c->s.q; S.scale = c->s.scale; S.opacity = c->s.opacity;
  S.albedo = c->s.albedo; S.roughness = c->s.roughness; S.metallic = c->s.metallic;
}

void trace_params(const lf_ctx *c, const lf_params *p, lf::TraceParams &P) {
  P.k = p->k;
  P.spp = p->spp;
  P.seed = p->seed;
  P.alpha_min = p->alpha_min;
  P.alpha_cap = p->alpha_cap;
  P.sig2 = p->support_sigma * p->support_sigma;
  P.eps = p->eps;
  P.t_min = p->t_min;
  P.sec_off = p->secondary_offset;
  P.flags = p->flags;
  P.counters = (p->flags & LF_FLAG_COUNT) ? c->counters.as<unsigned long long>() : nullptr;
  P.abort = c->abort_d;
}

bool ensure_env_tables(DevBuf &cdf_row, DevBuf &cdf_col, DevBuf &lum, DevBuf &rowsum, DevBuf &roww, DevBuf &scal,
                       int H, int W) {
  return cdf_row.ensure(sizeof(double) * (H + 1)) && cdf_col.ensure(sizeof(double) * H * (W + 1)) &&
         lum.ensure(sizeof(double) * H * W) && rowsum.ensure(sizeof(double) * H) && roww.ensure(sizeof(double) * H) &&
         scal.ensure(sizeof(double) * 2);
}

int64_t env_table_bytes(int H, int W) {
  return (int64_t)sizeof(double) * ((H + 1) + (int64_t)H * (W + 1) + (int64_t)H * W + 2 * H + 2);
}

}  // namespace lfh

using lfh::refit_impl;
using lfh::validate_params;

namespace {

// Common validation and setup of lf_render / lf_render_backward.
lf_status prepare(lf_ctx *c, const lf_transforms *xf, const lf_envmap *env, const lf_rays *rays,
                  const lf_camera *cams, int32_t n_cams, const lf_params *p, lf::RenderArgs &a) {
  if (!c) return LF_EINVAL;
  if (!c->has_scene) return fail(c, LF_EINVAL, "no scene set");
  lf_status st = validate_params(c, p);
  if (st) return st;
  if (!env || !env->texels || env->h < 1 || env->w < 1 || env->h > 8192 || env->w > 8192)
    return fail(c, LF_EINVAL, "invalid environment map");
  int M = c->n_inst - 1;
  if (M > 0 && (!xf || !xf->R || !xf->t)) return fail(c, LF_EINVAL, "scene has %d objects but no transforms", M);
  if ((rays != nullptr) == (cams != nullptr && n_cams > 0))
    return fail(c, LF_EINVAL, "pass exactly one of rays or cameras");
  memset(&a, 0, sizeof a);
  int64_t R = 0;
  if (rays) {
    if (rays->n < 0 || (rays->n > 0 && (!rays->o || !rays->d))) return fail(c, LF_EINVAL, "invalid rays");
    R = rays->n;
    a.rays.o = rays->o;
    a.rays.d = rays->d;
    a.rays.n = R;
  } else {
    if (n_cams > LF_MAX_CAMERAS) return fail(c, LF_EINVAL, "at most %d cameras per call", LF_MAX_CAMERAS);
    lf::CamArgs &ca = c->h_cams;
    memset(&ca, 0, sizeof ca);
    for (int i = 0; i < n_cams; ++i)
      if ((st = lfh::camera_args(c, cams[i], ca))) return fail(c, st, "camera %d: %s", i, c->err.c_str());
    R = ca.first[n_cams];
    a.n_tiles = ca.tiles[n_cams];
    if (!c->cams.ensure(sizeof(lf::CamArgs))) return fail(c, LF_ENOMEM, "cameras");
    if (hipMemcpyAsync(c->cams.p, &ca, sizeof ca, hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return check_hip(c, "camera upload");
    a.rays.cams = c->cams.as<lf::CamArgs>();
  }
  const int64_t J = (int64_t)p->spp * ((p->flags & LF_FLAG_NEE) ? 2 : 1);  // secondary slots per ray
  if (R * J >= (int64_t)INT32_MAX) return fail(c, LF_EUNSUPPORTED, "too many rays x samples");
  a.R = R;
  double sig2 = p->support_sigma * p->support_sigma;
  if (p->alpha_min != c->built_alpha_min || sig2 != c->built_sig2) {
    if (c->servers > 0) return fail(c, LF_EBUSY, "tracing constants differ from the scene a server is serving");
    if ((st = refit_impl(c, p->alpha_min, sig2))) return st;
  }
  // state assembly: instance records for this state's transforms
  Phase ph(c, 1);
  if (!c->bounds.ensure(6 * sizeof(double))) return fail(c, LF_ENOMEM, "bounds");
  lf::launch_instances(M > 0 ? xf->R : nullptr, M > 0 ? xf->t : nullptr, c->rootbox.as<float>(),
                       c->d_first.as<int32_t>(), c->d_n.as<int32_t>(), c->d_root.as<int32_t>(), c->n_inst,
                       c->inst.as<lf::InstRec>(), c->bounds.as<double>(), c->status.as<uint32_t>(), c->stream);
  // environment importance-sampling tables
  int H = env->h, W = env->w;
  if (!lfh::ensure_env_tables(c->env_cdf_row, c->env_cdf_col, c->env_lum, c->env_rowsum, c->env_roww, c->env_scal,
                              H, W))
    return fail(c, LF_ENOMEM, "environment tables");
  lf::launch_env_tables(env->texels, H, W, p->flags, c->env_cdf_row.as<double>(), c->env_cdf_col.as<double>(),
                        c->env_lum.as<double>(), c->env_rowsum.as<double>(), c->env_roww.as<double>(),
                        c->env_scal.as<double>(), c->stream);
  lfh::scene_view(c, a.S);
  a.S.inst = c->inst.as<lf::InstRec>();
  lfh::trace_params(c, p, a.P);
  a.spp_stride = (int32_t)J;
  a.E.tex = env->texels;
  a.E.H = H;
  a.E.W = W;
  a.E.cdf_row = c->env_cdf_row.as<double>();
  a.E.cdf_col = c->env_cdf_col.as<double>();
  a.E.lum = c->env_lum.as<double>();
  a.E.rowsum = c->env_rowsum.as<double>();
  a.E.roww = c->env_roww.as<double>();
  a.E.scal = c->env_scal.as<double>();
  a.status = c->status.as<uint32_t>();
  const bool trace2 = !(p->flags & LF_FLAG_NO_SECONDARY);
  const int64_t RS = R * J;
  // k-buffers handed from the traversal to the compositing launches: one per
  // primary work item (tile positions or rays; the backward's compositing
  // adjoint reads those of its replayed primary pass) and per secondary
  // queue entry
  const int64_t items1 = a.n_tiles > 0 ? a.n_tiles * lf::kBlock : R, items2 = trace2 ? RS : 0;
  const size_t kb_bytes = sizeof(uint32_t) * 2 * lf::kbucket(p->k);
  if (!c->work.ensure(sizeof(uint32_t) * lf::kPoolParts) ||
      !c->kbuf1.ensure(kb_bytes * (items1 > 0 ? items1 : 1)) || !c->kbuf2.ensure(kb_bytes * (items2 > 0 ? items2 : 1)))
    return fail(c, LF_ENOMEM, "k-buffers for %lld + %lld rays", (long long)items1, (long long)items2);
  a.work = c->work.as<uint32_t>();
  a.kbuf1 = c->kbuf1.as<uint32_t>();
  a.kbuf2 = c->kbuf2.as<uint32_t>();
  const int64_t R1 = R > 0 ? R : 1;
  if (!c->rec1.ensure(sizeof(lf::SurfRec) * R1)) return fail(c, LF_ENOMEM, "surface records");
  a.rec1 = c->rec1.as<lf::SurfRec>();
  if (trace2) {
    if (!c->queue.ensure(sizeof(lf::SecEntry) * (RS > 0 ? RS : 1)) || !c->qcount.ensure(sizeof(uint32_t)) ||
        !c->rec2.ensure(sizeof(lf::SurfRec) * (RS > 0 ? RS : 1)))
      return fail(c, LF_ENOMEM, "secondary queue");
    if (!c->hint2.ensure(sizeof(float) * (RS > 0 ? RS : 1))) return fail(c, LF_ENOMEM, "secondary bounds");
    a.hint2 = c->hint2.as<float>();
    a.queue = c->queue.as<lf::SecEntry>();
    a.queue_count = c->qcount.as<uint32_t>();
    a.rec2 = c->rec2.as<lf::SurfRec>();
    lf::launch_fill_u32(a.queue_count, 0u, 1, c->stream);
    if (!(p->flags & LF_FLAG_UNSORTED)) {
      const int64_t n2 = RS > 0 ? RS : 1;
      if (!c->skeys.ensure(8 * n2) || !c->skeys2.ensure(8 * n2) || !c->svals.ensure(4 * n2) ||
          !c->svals2.ensure(4 * n2) || !c->shist.ensure(4 * lf::radix_sort_hist_words(n2)))
        return fail(c, LF_ENOMEM, "secondary sort buffers");
      a.order = c->svals.as<int32_t>();
    }
  }
  return check_hip(c, "prepare");
}

// Signature of a render call whose arguments prepare() accepted (cameras
// as uploaded to c->h_cams).
lfh::CallSig call_sig(const lf_ctx *c, const lf_transforms *xf, const lf_envmap *env, const lf_rays *rays,
                      const lf_params *p) {
  lfh::CallSig g;
  memset(&g, 0, sizeof g);  // padding included, so signatures compare with memcmp
  if (rays) {
    g.ro = rays->o;
    g.rd = rays->d;
    g.n = rays->n;
  } else {
    g.cams = c->h_cams;
  }
  g.k = p->k;
  g.spp = p->spp;
  g.seed = p->seed;
  g.flags = p->flags & ~(LF_FLAG_COUNT | LF_FLAG_DETERMINISTIC);
  g.alpha_min = p->alpha_min;
  g.alpha_cap = p->alpha_cap;
  g.sigma = p->support_sigma;
  g.eps = p->eps;
  g.t_min = p->t_min;
  g.sec_off = p->secondary_offset;
  g.env = env->texels;
  g.h = env->h;
  g.w = env->w;
  if (c->n_inst > 1 && xf) {
    g.R = xf->R;
    g.t = xf->t;
  }
  g.epoch = c->scene_epoch;
  return g;
}

// regroups the secondary queue by direction octant and origin for coherent traversal
void sort_secondaries(lf_ctx *c, const lf::RenderArgs &a) {
  if (!a.order) return;
  const int64_t cap = a.R * a.spp_stride;
  lf::launch_secondary_keys(a.queue, a.queue_count, cap, c->bounds.as<double>(), nullptr, nullptr,
                            c->skeys.as<uint64_t>(), c->svals.as<int32_t>(), c->stream);
  lf::radix_sort(c->skeys.as<uint64_t>(), c->svals.as<int32_t>(), c->skeys2.as<uint64_t>(), c->svals2.as<int32_t>(),
                 c->shist.as<uint32_t>(), cap, c->stream, 32);
}

}  // namespace

extern "C" {

void lf_params_default(lf_params *p) {
  if (!p) return;
  p->k = 32;
  p->spp = 1;
  p->seed = 0;
  p->alpha_min = 1.0 / 255.0;
  p->alpha_cap = 0.99;
  p->support_sigma = 3.0;
  p->eps = 1e-6;
  p->t_min = 1e-4;
  p->secondary_offset = 1e-3;
  p->flags = 0;
}

// ---- device scratch of the allocation-free L1 objective (lf_l1_loss_noalloc)
// The partial sums of one objective pass (one slot per block of a grid capped
// at kMaxLossBlocks, then the totals) live in this file-scope array: each
// device holds its own copy for the life of the process, and every call on a
// device shares it.  In host code `scratch` names a host-side stand-in, so
// kernels receive the device address looked up by lf_create instead.
static __device__ __align__(256) double scratch[lf::kLossPartDoubles];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxScratchDevices] = {};  // device address of `scratch` on each device

// Looks up the device's copy of `scratch` once, with that device current.
bool scratch_lookup(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return false;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return true;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return false;
  }
  g_scratch[device] = (double *)p;
  return true;
}

double *scratch_ptr(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}
}  // namespace

lf_status lf_create(lf_ctx **out, int device, void *hip_stream) {
  if (!out) return LF_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return LF_EDEVICE;
  }
  lf_ctx *c = new lf_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (!set_device(c) || !scratch_lookup(device) || !c->status.ensure(sizeof(uint32_t)) ||
      !c->acc_secondary.ensure(8) || !c->counters.ensure(8 * LF_NUM_COUNTERS)) {
    delete c;
    return LF_EDEVICE;
  }
  // the abort word: host memory the kernels read uncached, so a store from
  // any host thread reaches traversal loops that are already running
  void *ab = nullptr, *ab_d = nullptr;
  if (hipHostMalloc(&ab, sizeof(uint32_t), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer(&ab_d, ab, 0) != hipSuccess) {
    (void)hipGetLastError();
    if (ab) (void)hipHostFree(ab);
    delete c;
    return LF_EDEVICE;
  }
  c->abort_h = (uint32_t *)ab;
  c->abort_d = (const uint32_t *)ab_d;
  __atomic_store_n(c->abort_h, 0u, __ATOMIC_SEQ_CST);
  lf::launch_fill_u32(c->status.as<uint32_t>(), 0u, 1, c->stream);
  lf::launch_fill_u32(c->acc_secondary.as<uint32_t>(), 0u, 2, c->stream);
  lf::launch_fill_u32(c->counters.as<uint32_t>(), 0u, 2 * LF_NUM_COUNTERS, c->stream);
  if (check_hip(c, "create")) {
    delete c;
    return LF_EDEVICE;
  }
  *out = c;
  return LF_OK;
}

void lf_destroy(lf_ctx *c) {
  if (!c) return;
  set_device(c);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (auto &pe : c->pending) {
    (void)hipEventDestroy(pe.second.first);
    (void)hipEventDestroy(pe.second.second);
  }
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  if (c->abort_h) (void)hipHostFree(c->abort_h);
  delete c;
}

const char *lf_last_error(const lf_ctx *c) { return c ? c->err.c_str() : "null context"; }

// The stream has drained: clears the abort request, then returns (and
// clears) the latched device status.
static lf_status drained(lf_ctx *c) {
  __atomic_store_n(c->abort_h, 0u, __ATOMIC_SEQ_CST);
  uint32_t st = 0;
  if (hipMemcpy(&st, c->status.p, sizeof st, hipMemcpyDeviceToHost) != hipSuccess) return check_hip(c, "sync");
  if (st) {
    lf::launch_fill_u32(c->status.as<uint32_t>(), 0u, 1, c->stream);
    (void)hipStreamSynchronize(c->stream);
    if (st & lf::kStatusOverflow) return fail(c, LF_EOVERFLOW, "traversal stack overflow on the device");
    if (st & lf::kStatusBadTransform) return fail(c, LF_EINVAL, "degenerate or non-finite object transform");
    if (st & lf::kStatusBvhCorrupt) return fail(c, LF_EDEVICE, "out-of-range hierarchy index on the device");
    if (st & lf::kStatusAborted) return fail(c, LF_EABORTED, "traversal cut short by lf_abort");
  }
  return LF_OK;
}

lf_status lf_sync(lf_ctx *c) {
  if (!c) return LF_EINVAL;
  set_device(c);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return check_hip(c, "sync");
  return drained(c);
}

lf_status lf_abort(lf_ctx *c) {
  if (!c) return LF_EINVAL;
  __atomic_store_n(c->abort_h, 1u, __ATOMIC_SEQ_CST);
  return LF_OK;
}

lf_status lf_sync_timeout(lf_ctx *c, double timeout_ms) {
  if (!c) return LF_EINVAL;
  if (!(timeout_ms >= 0.0)) return fail(c, LF_EINVAL, "timeout_ms must be >= 0");
  set_device(c);
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t q = hipStreamQuery(c->stream);
    if (q == hipSuccess) return drained(c);
    if (q != hipErrorNotReady) return check_hip(c, "sync");
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (ms >= timeout_ms) break;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  // the watchdog fires: cut the traversal short and wait for what is enqueued
  __atomic_store_n(c->abort_h, 1u, __ATOMIC_SEQ_CST);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return check_hip(c, "sync");
  (void)drained(c);
  return fail(c, LF_ETIMEOUT, "work not done after %.3f ms: cut short", timeout_ms);
}

lf_status lf_scene_set(lf_ctx *c, const lf_surfels *sf) {
  if (!c) return LF_EINVAL;
  if (!sf) return fail(c, LF_EINVAL, "surfels is NULL");
  if (!sf->mu || !sf->q || !sf->scale || !sf->opacity || !sf->albedo || !sf->roughness || !sf->metallic)
    return fail(c, LF_EINVAL, "surfel array is NULL");
  if (sf->n < 1 || sf->n >= (int64_t)INT32_MAX) return fail(c, LF_EINVAL, "n=%lld out of range", (long long)sf->n);
  if (sf->n_objects < 0 || sf->n_objects > lf::kMaxInst - 1)
    return fail(c, sf->n_objects < 0 ? LF_EINVAL : LF_EUNSUPPORTED, "n_objects=%d not in 0..%d", sf->n_objects,
                lf::kMaxInst - 1);
  if (!sf->object_offset) return fail(c, LF_EINVAL, "object_offset is NULL");
  int n_inst = sf->n_objects + 1;
  const int64_t *off = sf->object_offset;
  if (off[0] != 0 || off[n_inst] != sf->n) return fail(c, LF_EINVAL, "object_offset must start at 0 and end at n");
  for (int i = 0; i < n_inst; ++i)
    if (off[i + 1] < off[i]) return fail(c, LF_EINVAL, "object_offset must be non-decreasing");
  if (c->servers > 0) return fail(c, LF_EBUSY, "a relight server is reading the scene");
  set_device(c);
  // calls still running on the stream read the buffers rebuilt below (some
  // of them written by copies that the stream does not order)
  if (hipStreamSynchronize(c->stream) != hipSuccess) return check_hip(c, "scene set");
  c->has_scene = false;
  c->s = lf::SurfelArrays{sf->mu, sf->q, sf->scale, sf->opacity, sf->albedo, sf->roughness, sf->metallic, sf->n};
  c->n_inst = n_inst;
  c->h_first.assign(n_inst, 0);
  c->h_n.assign(n_inst, 0);
  c->h_node_off.assign(n_inst, 0);
  c->h_root.assign(n_inst, 0);
  int64_t nodes = 0;
  for (int i = 0; i < n_inst; ++i) {
    c->h_first[i] = (int32_t)off[i];
    c->h_n[i] = (int32_t)(off[i + 1] - off[i]);
    c->h_node_off[i] = (int32_t)nodes;
    if (c->h_n[i] >= 2) c->h_root[i] = (int32_t)nodes;
    else if (c->h_n[i] == 1) c->h_root[i] = ~c->h_first[i];
    nodes += c->h_n[i] > 1 ? c->h_n[i] - 1 : 0;
  }
  c->n_nodes = nodes;
  const int64_t n = sf->n;
  bool ok = c->d_first.ensure(4 * n_inst) && c->d_n.ensure(4 * n_inst) && c->d_root.ensure(4 * n_inst) &&
            c->rec.ensure(sizeof(lf::TraceRec) * n) && c->filt.ensure(sizeof(lf::FiltRec) * n) && c->nodes.ensure(sizeof(lf::BNode) * (nodes ? nodes : 1)) &&
            c->perm.ensure(4 * n) && c->leaf_parent.ensure(4 * n) && c->node_parent.ensure(4 * (nodes ? nodes : 1)) &&
            c->flags.ensure(4 * (nodes ? nodes : 1)) && c->leafbox.ensure(24 * n) &&
            c->rootbox.ensure(24 * n_inst) && c->inst.ensure(sizeof(lf::InstRec) * n_inst) &&
            c->keys.ensure(8 * n) && c->keys2.ensure(8 * n) && c->vals2.ensure(4 * n) &&
            c->hist.ensure(4 * lf::radix_sort_hist_words(n)) && c->boxidx.ensure(24 * n) &&
            c->ibounds.ensure(24 * n_inst) && c->depth.ensure(8);
  if (!ok) return fail(c, LF_ENOMEM, "scene buffers for n=%lld", (long long)n);
  if (hipMemcpy(c->d_first.p, c->h_first.data(), 4 * n_inst, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_n.p, c->h_n.data(), 4 * n_inst, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_root.p, c->h_root.data(), 4 * n_inst, hipMemcpyHostToDevice) != hipSuccess)
    return check_hip(c, "scene upload");
  lf_params dp;
  lf_params_default(&dp);
  const double sig2 = dp.support_sigma * dp.support_sigma;
  hipStream_t st = c->stream;
  lf::launch_boxes_by_index(c->s, dp.alpha_min, sig2, c->boxidx.as<float>(), st);
  lf::launch_instance_bounds(c->boxidx.as<float>(), c->d_first.as<int32_t>(), c->d_n.as<int32_t>(), n_inst,
                             c->ibounds.as<float>(), st);
  lf::launch_morton(c->boxidx.as<float>(), c->ibounds.as<float>(), c->d_first.as<int32_t>(), c->d_n.as<int32_t>(),
                    n_inst, n, c->keys.as<uint64_t>(), c->perm.as<int32_t>(), st);
  lf::radix_sort(c->keys.as<uint64_t>(), c->perm.as<int32_t>(), c->keys2.as<uint64_t>(), c->vals2.as<int32_t>(),
                 c->hist.as<uint32_t>(), n, st);
  // hierarchy of every instance by locally-ordered clustering of the sorted boxes
  if (!c->ploc_i.ensure(sizeof(int32_t) * 5 * n) || !c->ploc_f.ensure(sizeof(float) * 12 * n))
    return fail(c, LF_ENOMEM, "clustering scratch for n=%lld", (long long)n);
  int32_t *pi = c->ploc_i.as<int32_t>();
  float *pf = c->ploc_f.as<float>();
  for (int i = 0; i < n_inst; ++i) {
    if (c->h_n[i] < 1) continue;
    if (!lf::launch_ploc(c->perm.as<int32_t>(), c->boxidx.as<float>(), c->h_first[i], c->h_n[i], c->h_node_off[i], i,
                         c->nodes.as<lf::BNode>(), c->node_parent.as<int32_t>(), c->leaf_parent.as<int32_t>(), pi,
                         pi + n, pf, pf + 6 * n, pi + 2 * n, (uint32_t *)(pi + 3 * n), (uint32_t *)(pi + 4 * n), st))
      return fail(c, LF_EDEVICE, "hierarchy clustering of instance %d failed", i);
  }
  lf::launch_fill_u32(c->depth.as<uint32_t>(), 0u, 2, st);
  lf::launch_depth(c->leaf_parent.as<int32_t>(), c->node_parent.as<int32_t>(), n, c->n_nodes,
                   c->depth.as<int32_t>(), c->status.as<uint32_t>(), st);
  if (hipStreamSynchronize(st) != hipSuccess ||
      hipMemcpy(&c->max_depth, c->depth.p, 4, hipMemcpyDeviceToHost) != hipSuccess)
    return check_hip(c, "hierarchy depth");
  // Traversal nodes: surface-area-cost collapse (costs bottom-up by binary
  // depth, then expansion level by level), subtree counts, then depth-first
  // placement with contiguous children and the matching leaf order.
  const int64_t nn = nodes ? nodes : 1;
  const int W = lf::kWide;
  if (!c->wtmp.ensure(sizeof(int32_t) * ((10 + W) * nn + n)) || !c->wdp.ensure((sizeof(float) * W + 16) * nn))
    return fail(c, LF_ENOMEM, "traversal-node scratch for n=%lld", (long long)n);
  int32_t *level = c->wtmp.as<int32_t>(), *sub_w = level + nn, *sub_l = sub_w + nn, *widx = sub_l + nn;
  int32_t *dbase = widx + nn, *lbase = dbase + nn;
  int2 *side_cnt = (int2 *)(lbase + nn);
  int32_t *slot_src = (int32_t *)(side_cnt + 2 * nn), *newpos = slot_src + W * nn;
  int32_t *n_levels_d = c->depth.as<int32_t>() + 1;
  float *wcost = c->wdp.as<float>();
  uint8_t *wchoice = (uint8_t *)(wcost + W * nn);
  // binary nodes by depth for the level-by-level refit
  std::vector<int32_t> h_depth(nodes), h_order(nodes);
  c->h_level_off.assign(1, 0);
  if (!c->node_order.ensure(sizeof(int32_t) * nn)) return fail(c, LF_ENOMEM, "refit order");
  if (nodes > 0) {
    lf::launch_node_depth(c->node_parent.as<int32_t>(), c->n_nodes, level, c->status.as<uint32_t>(), st);
    if (hipMemcpy(h_depth.data(), level, sizeof(int32_t) * nodes, hipMemcpyDeviceToHost) != hipSuccess)
      return check_hip(c, "refit order");
    int32_t dmax = 0;
    for (int64_t i = 0; i < nodes; ++i) {
      if (h_depth[i] < 0 || h_depth[i] > 4096) return fail(c, LF_EDEVICE, "inconsistent node depth");
      dmax = std::max(dmax, h_depth[i]);
    }
    c->h_level_off.assign(dmax + 2, 0);
    for (int64_t i = 0; i < nodes; ++i) ++c->h_level_off[h_depth[i] + 1];
    for (int32_t d = 0; d <= dmax; ++d) c->h_level_off[d + 1] += c->h_level_off[d];
    std::vector<int64_t> fill(c->h_level_off.begin(), c->h_level_off.end() - 1);
    for (int64_t i = 0; i < nodes; ++i) h_order[fill[h_depth[i]]++] = (int32_t)i;
    if (hipMemcpy(c->node_order.p, h_order.data(), sizeof(int32_t) * nodes, hipMemcpyHostToDevice) != hipSuccess)
      return check_hip(c, "refit order");
  }
  lf::launch_wide_cost(c->nodes.as<lf::BNode>(), c->n_nodes, c->node_order.as<int32_t>(), c->h_level_off, wcost,
                       wchoice, c->status.as<uint32_t>(), st);
  lf::launch_fill_u32((uint32_t *)level, 0xffffffffu, nn, st);
  lf::launch_wide_roots(c->d_root.as<int32_t>(), c->d_n.as<int32_t>(), n_inst, level, st);
  for (int32_t it = 0; it <= c->max_depth && nodes > 0; ++it)
    lf::launch_wide_level(c->nodes.as<lf::BNode>(), c->n_nodes, it, wchoice, level, slot_src, n_levels_d,
                          c->status.as<uint32_t>(), st);
  lf::launch_wide_count(c->leaf_parent.as<int32_t>(), c->node_parent.as<int32_t>(), level, n, c->n_nodes,
                        c->flags.as<int32_t>(), side_cnt, sub_w, sub_l, c->status.as<uint32_t>(), st);
  if (hipStreamSynchronize(st) != hipSuccess ||
      hipMemcpy(&c->wide_levels, n_levels_d, 4, hipMemcpyDeviceToHost) != hipSuccess)
    return check_hip(c, "traversal nodes");
  std::vector<int32_t> roots(3 * n_inst, 0), root4(n_inst);
  int64_t n_wide = 0;
  c->h_wide_off.assign(n_inst, 0);
  c->h_wide_n.assign(n_inst, 0);
  for (int i = 0; i < n_inst; ++i) {
    root4[i] = c->h_root[i];
    c->h_wide_off[i] = n_wide;
    if (c->h_n[i] < 2) continue;
    int32_t cnt = 0;
    if (hipMemcpy(&cnt, sub_w + c->h_root[i], 4, hipMemcpyDeviceToHost) != hipSuccess)
      return check_hip(c, "traversal nodes");
    if (cnt < 1 || cnt > c->h_n[i]) return fail(c, LF_EDEVICE, "inconsistent traversal-node count %d", cnt);
    roots[3 * i] = (int32_t)n_wide;
    roots[3 * i + 1] = (int32_t)n_wide + 1;
    roots[3 * i + 2] = c->h_first[i];
    root4[i] = (int32_t)n_wide;
    c->h_wide_n[i] = cnt;
    n_wide += cnt;
  }
  c->n_wide = n_wide;
  if (!c->wroots.ensure(sizeof(int32_t) * 3 * n_inst) || !c->winfo.ensure(sizeof(lf::WideInfo) * (n_wide ? n_wide : 1)) ||
      !c->qnodes.ensure(sizeof(lf::QNode) * (n_wide ? n_wide : 1)))
    return fail(c, LF_ENOMEM, "traversal nodes");
  if (hipMemcpy(c->wroots.p, roots.data(), sizeof(int32_t) * 3 * n_inst, hipMemcpyHostToDevice) != hipSuccess)
    return check_hip(c, "traversal nodes");
  lf::launch_wide_root_pos(c->d_root.as<int32_t>(), c->d_n.as<int32_t>(), c->wroots.as<int32_t>(), n_inst, widx, dbase,
                           lbase, st);
  lf::launch_iota(newpos, n, st);
  for (int32_t it = 0; it < c->wide_levels; ++it)
    lf::launch_wide_assign(c->nodes.as<lf::BNode>(), c->n_nodes, n, it, level, slot_src, sub_w, sub_l, widx, dbase,
                           lbase, newpos, c->winfo.as<lf::WideInfo>(), n_wide, c->status.as<uint32_t>(), st);
  lf::launch_leaf_reorder(newpos, c->perm.as<int32_t>(), c->leaf_parent.as<int32_t>(), n, c->n_nodes,
                          c->vals2.as<int32_t>(), (int32_t *)c->keys2.p, c->nodes.as<lf::BNode>(),
                          c->status.as<uint32_t>(), st);
  if (hipMemcpyAsync(c->perm.p, c->vals2.p, 4 * (size_t)n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(c->leaf_parent.p, c->keys2.p, 4 * (size_t)n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(c->d_root.p, root4.data(), 4 * n_inst, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return check_hip(c, "traversal nodes");
  lf_status s2 = refit_impl(c, dp.alpha_min, sig2);
  if (s2) return s2;
  if (hipStreamSynchronize(st) != hipSuccess) return check_hip(c, "scene build");
  uint32_t bst = 0;
  if (hipMemcpy(&bst, c->status.p, 4, hipMemcpyDeviceToHost) != hipSuccess) return check_hip(c, "scene build");
  if (bst & lf::kStatusBvhCorrupt) {
    lf::launch_fill_u32(c->status.as<uint32_t>(), 0u, 1, st);
    return fail(c, LF_EDEVICE, "hierarchy build produced an out-of-range index");
  }
  // the traversal stack holds one entry per level above the current node,
  // naming a node by 23 bits
  if (c->wide_levels - 1 > lf::kStackL)
    return fail(c, LF_EUNSUPPORTED, "%d node levels need more than the traversal stack (%d entries)",
                c->wide_levels, lf::kStackL);
  if (c->n_wide >= lf::kMaxWideNodes)
    return fail(c, LF_EUNSUPPORTED, "%lld traversal nodes exceed the stack encoding (%d)", (long long)c->n_wide,
                lf::kMaxWideNodes);
  c->has_scene = true;
  return check_hip(c, "scene build");
}

lf_status lf_scene_refit(lf_ctx *c) {
  if (!c) return LF_EINVAL;
  if (!c->has_scene) return fail(c, LF_EINVAL, "no scene set");
  if (c->servers > 0) return fail(c, LF_EBUSY, "a relight server is reading the scene");
  set_device(c);
  return refit_impl(c, c->built_alpha_min, c->built_sig2);
}

lf_status lf_render(lf_ctx *c, const lf_transforms *xf, const lf_envmap *env, const lf_rays *rays,
                    const lf_camera *cams, int32_t n_cams, const lf_params *p, lf_outputs *out) {
  if (!c) return LF_EINVAL;
  if (!out) return fail(c, LF_EINVAL, "outputs struct is NULL");
  set_device(c);
  c->sig_valid = false;
  lf::RenderArgs a;
  lf_status st = prepare(c, xf, env, rays, cams, n_cams, p, a);
  if (st) return st;
  if (a.R == 0) return LF_OK;
  // a backward with the same arguments may start its replay from this call's k-th distances
  const lfh::CallSig sig = call_sig(c, xf, env, rays, p);
  if (!out->radiance || !out->depth || !out->normal || !out->alpha)
    return fail(c, LF_EINVAL, "radiance, depth, normal and alpha outputs are required");
  a.radiance = out->radiance;
  a.depth = out->depth;
  a.normal = out->normal;
  a.alpha = out->alpha;
  a.hit_idx = out->hit_idx;
  a.sec_hit_idx = out->sec_hit_idx;
  const bool trace2 = !(p->flags & LF_FLAG_NO_SECONDARY);
  if (trace2) {
    if (!c->contrib.ensure(sizeof(float) * 3 * a.R * a.spp_stride)) return fail(c, LF_ENOMEM, "contributions");
    a.contrib = c->contrib.as<float>();
  } else if (out->sec_hit_idx) {
    lf::launch_fill_u32((uint32_t *)out->sec_hit_idx, 0xffffffffu, a.R * a.spp_stride * p->k, c->stream);
  }
  {
    Phase ph(c, 2);
    lf::launch_trace1(a, c->stream);
  }
  {
    Phase ph(c, 14);
    lf::launch_composite1(a, false, c->stream);
  }
  {
    Phase ph(c, 3);
    lf::launch_shade1(a, false, c->stream);
  }
  if (trace2) {
    {
      Phase ph(c, 4);
      sort_secondaries(c, a);
    }
    {
      Phase ph(c, 5);
      lf::launch_trace2(a, c->stream);
    }
    {
      Phase ph(c, 15);
      lf::launch_composite2(a, c->stream);
    }
    {
      Phase ph(c, 6);
      lf::launch_shade2(a, false, c->stream);
    }
    Phase ph(c, 7);
    lf::launch_resolve(a, c->stream);
    lf::launch_accum(c->acc_secondary.as<unsigned long long>(), a.queue_count, c->stream);
  }
  c->acc_primary += a.R;
  st = check_hip(c, "render");
  if (st == LF_OK) {
    c->last_sig = sig;
    c->sig_valid = true;
  }
  return st;
}

// A backward call that ran; the next one does not start from its k-buffers.
static lf_status backward_done(lf_ctx *c, const lfh::CallSig &sig) {
  (void)sig;
  c->sig_valid = false;
  return check_hip(c, "backward");
}

// Smallest b with 2^b > n: keys below 2^b sort in ceil(b / 16) * 2 radix passes
// and 2^b - 1 marks unused records.
static int key_bits(int64_t n) {
  int b = 1;
  while (b < 62 && ((int64_t)1 << b) <= n) ++b;
  return b;
}

// Scratch of the order-fixed adjoint (LF_FLAG_DETERMINISTIC) for the call a.
static lf_status deterministic_buffers(lf_ctx *c, const lf::RenderArgs &a, int64_t texels, lf::DetArgs &d) {
  const int64_t J = (int64_t)a.P.spp * ((a.P.flags & LF_FLAG_NEE) ? 2 : 1);
  d.n_hit = lf::adjoint_items(a) * lf::kbucket(a.P.k);
  d.env_cap = (int)(4 * (1 + 3 * J));
  d.n_env = a.R * d.env_cap;
  if (d.n_hit >= ((int64_t)1 << 31) || d.n_env >= ((int64_t)1 << 31))
    return fail(c, LF_EUNSUPPORTED, "deterministic gradients take at most 2^31 records (%lld hit, %lld env)",
                (long long)d.n_hit, (long long)d.n_env);
  d.hit_bits = key_bits(c->s.n);
  d.env_bits = key_bits(texels);
  d.hit_unused = ((uint64_t)1 << d.hit_bits) - 1;
  d.env_unused = ((uint64_t)1 << d.env_bits) - 1;
  const int64_t nmax = d.n_hit > d.n_env ? d.n_hit : d.n_env;
  if (!c->det_key.ensure(8 * nmax) || !c->det_key2.ensure(8 * nmax) || !c->det_idx.ensure(4 * nmax) ||
      !c->det_idx2.ensure(4 * nmax) || !c->det_hval.ensure(sizeof(double) * 15 * d.n_hit) ||
      !c->det_eval.ensure(sizeof(double) * 3 * d.n_env) ||
      !c->det_hist.ensure(4 * lf::radix_sort_hist_words(nmax)))
    return fail(c, LF_ENOMEM, "deterministic gradient records (%lld hit, %lld env)", (long long)d.n_hit,
                (long long)d.n_env);
  // the two sorts run one after the other on the stream, so they share the key and index buffers
  d.hit_key = d.env_key = c->det_key.as<uint64_t>();
  d.hit_key2 = d.env_key2 = c->det_key2.as<uint64_t>();
  d.hit_idx = d.env_idx = c->det_idx.as<int32_t>();
  d.hit_idx2 = d.env_idx2 = c->det_idx2.as<int32_t>();
  d.hit_val = c->det_hval.as<double>();
  d.env_val = c->det_eval.as<double>();
  d.hist = c->det_hist.as<uint32_t>();
  return LF_OK;
}

lf_status lf_render_backward(lf_ctx *c, const lf_transforms *xf, const lf_envmap *env, const lf_rays *rays,
                             const lf_camera *cams, int32_t n_cams, const lf_params *p, const lf_grad_out *g,
                             lf_grad_in *gi) {
  if (!c) return LF_EINVAL;
  if (!g) return fail(c, LF_EINVAL, "upstream gradients struct is NULL");
  if (!gi || !gi->d_mu || !gi->d_q || !gi->d_scale || !gi->d_opacity || !gi->d_albedo || !gi->d_roughness ||
      !gi->d_metallic || !gi->d_env)
    return fail(c, LF_EINVAL, "all eight gradient outputs are required");
  set_device(c);
  const bool had_sig = c->sig_valid;
  c->sig_valid = false;
  lf::RenderArgs a;
  lf_status st = prepare(c, xf, env, rays, cams, n_cams, p, a);
  if (st) return st;
  // the replay traces the rays of the forward call just before it with the
  // same arguments: each starts from the k-th distance that call left in the
  // k-buffers (only then: equal pointers need not mean equal contents, and
  // a wrong bound costs a retrace)
  const lfh::CallSig sig = call_sig(c, xf, env, rays, p);
  a.use_hint = had_sig && memcmp(&sig, &c->last_sig, sizeof sig) == 0;
  // the order-fixed form's record limit and buffers before any work is enqueued
  lf::DetArgs det;
  if ((p->flags & LF_FLAG_DETERMINISTIC) && a.R > 0) {
    st = deterministic_buffers(c, a, (int64_t)env->h * env->w, det);
    if (st) return st;
  }
  const int64_t n = c->s.n;
  hipStream_t s = c->stream;
  {
    Phase ph0(c, 12);
    lf::launch_fill_f32(gi->d_mu, 0.f, 3 * n, s);
    lf::launch_fill_f32(gi->d_q, 0.f, 4 * n, s);
    lf::launch_fill_f32(gi->d_scale, 0.f, 2 * n, s);
    lf::launch_fill_f32(gi->d_opacity, 0.f, n, s);
    lf::launch_fill_f32(gi->d_albedo, 0.f, 3 * n, s);
    lf::launch_fill_f32(gi->d_roughness, 0.f, n, s);
    lf::launch_fill_f32(gi->d_metallic, 0.f, n, s);
    lf::launch_fill_f32(gi->d_env, 0.f, (int64_t)3 * env->h * env->w, s);
  }

  if (a.R == 0) return check_hip(c, "backward");
  const bool trace2 = !(p->flags & LF_FLAG_NO_SECONDARY);
  if (!c->seeds.ensure(sizeof(lf::AdjSeed) * a.R)) return fail(c, LF_ENOMEM, "adjoint seeds");
  a.seeds = c->seeds.as<lf::AdjSeed>();
  if (trace2 && !c->frozen.ensure(sizeof(lf::SecFrozen) * a.R * a.spp_stride))
    return fail(c, LF_ENOMEM, "frozen records");
  a.frozen = trace2 ? c->frozen.as<lf::SecFrozen>() : nullptr;
  {
    Phase ph(c, 8);
    lf::launch_trace1(a, s);
    lf::launch_composite1(a, true, s);
    if (trace2) lf::launch_shade1(a, true, s);
  }
  if (trace2) {
    Phase ph(c, 9);
    sort_secondaries(c, a);
    lf::launch_trace2(a, s);
    lf::launch_composite2(a, s);
    lf::launch_shade2(a, true, s);
  }
  lf::GradArgs ga{g->d_radiance, g->d_depth, g->d_normal, g->d_alpha, gi->d_mu, gi->d_q, gi->d_scale,
                  gi->d_opacity, gi->d_albedo, gi->d_roughness, gi->d_metallic, gi->d_env};
  if (p->flags & LF_FLAG_DETERMINISTIC) {
    {
      Phase ph(c, 10);
      lf::launch_adjoint_shade_det(a, ga, det, s);
    }
    {
      Phase ph(c, 16);
      lf::launch_adjoint_hits_det(a, ga, det, s);
    }
    return backward_done(c, sig);
  }
  {
    // partial copies of the environment gradient, as many as fit in 256 MB
    const int64_t m = (int64_t)3 * env->h * env->w;
    int copies = (int)std::min<int64_t>(lf::kEnvGradCopies, ((int64_t)256 << 20) / (4 * m));
    if (copies > 1 && !c->env_part.ensure(sizeof(float) * copies * m)) copies = 1;
    Phase ph(c, 10);
    lf::launch_adjoint_shade(a, ga, copies > 1 ? c->env_part.as<float>() : nullptr, copies, s);
  }
  {
    Phase ph(c, 16);
    lf::launch_adjoint_hits(a, ga, s);
  }
  return backward_done(c, sig);
}

lf_status lf_l1_loss(lf_ctx *c, const float *pred, const float *target, int64_t n, float *loss, float *grad) {
  if (!c) return LF_EINVAL;
  if (!loss || n < 0 || (n > 0 && (!pred || !target))) return fail(c, LF_EINVAL, "invalid loss arguments");
  set_device(c);
  if (!c->lossbuf.ensure(lf::kLossPartDoubles * sizeof(double))) return fail(c, LF_ENOMEM, "loss scratch");
  Phase ph(c, 13);
  lf::launch_l1(pred, target, n, loss, grad, c->lossbuf.as<double>(), c->stream);
  return check_hip(c, "l1 loss");
}

lf_status lf_l1_loss_noalloc(lf_ctx *c, const float *pred, const float *target, int64_t n, float *loss,
                             float *grad) {
  if (!c) return LF_EINVAL;
  if (!loss || n < 0 || (n > 0 && (!pred || !target))) return fail(c, LF_EINVAL, "invalid loss arguments");
  double *part = scratch_ptr(c->device);
  if (!part) return fail(c, LF_EDEVICE, "no loss scratch on device %d", c->device);
  set_device(c);
  lf::launch_l1(pred, target, n, loss, grad, part, c->stream);
  return check_hip(c, "l1 loss (no allocation)");
}

// Uploads one camera into c->cams (camera 0); validates it first.
static lf_status upload_camera(lf_ctx *c, const lf_camera *cam) {
  if (!cam || cam->w < 1 || cam->h < 1 || !(cam->fov_y_deg > 0.f && cam->fov_y_deg < 180.f))
    return fail(c, LF_EINVAL, "invalid camera");
  lf::CamArgs &ca = c->h_cams;
  memset(&ca, 0, sizeof ca);
  lf_status st = lfh::camera_args(c, *cam, ca);
  if (st) return st;
  if (!c->cams.ensure(sizeof(lf::CamArgs))) return fail(c, LF_ENOMEM, "cameras");
  if (hipMemcpyAsync(c->cams.p, &ca, sizeof ca, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return check_hip(c, "camera upload");
  return LF_OK;
}

lf_status lf_raygen(lf_ctx *c, const lf_camera *cam, float *o, float *d) {
  if (!c) return LF_EINVAL;
  if (!o || !d) return fail(c, LF_EINVAL, "invalid raygen arguments");
  set_device(c);
  lf_status st = upload_camera(c, cam);
  if (st) return st;
  lf::launch_raygen(c->cams.as<lf::CamArgs>(), (int64_t)cam->w * cam->h, o, d, c->stream);
  return check_hip(c, "raygen");
}

// ---- geometry-refinement objectives (Sec. 3.1, 3.2)
static bool loss_acc(lf_ctx *c) { return c->lossbuf.ensure(lf::kLossPartDoubles * sizeof(double)); }

lf_status lf_loss_alpha(lf_ctx *c, const float *alpha, int64_t n, float *loss, float *grad) {
  if (!c) return LF_EINVAL;
  if (!loss || n < 0 || (n > 0 && !alpha)) return fail(c, LF_EINVAL, "invalid coverage-loss arguments");
  set_device(c);
  if (!loss_acc(c)) return fail(c, LF_ENOMEM, "loss scratch");
  Phase ph(c, 13);
  lf::launch_loss_alpha(alpha, n, loss, grad, c->lossbuf.as<double>(), c->stream);
  return check_hip(c, "coverage loss");
}

lf_status lf_loss_scale(lf_ctx *c, const float *scale, int64_t n, float s_max, float *loss, float *grad) {
  if (!c) return LF_EINVAL;
  if (!loss || n < 0 || (n > 0 && !scale) || !(s_max > 0.f) || !std::isfinite(s_max))
    return fail(c, LF_EINVAL, "invalid scale-loss arguments");
  set_device(c);
  if (!loss_acc(c)) return fail(c, LF_ENOMEM, "loss scratch");
  Phase ph(c, 13);
  lf::launch_loss_scale(scale, n, s_max, loss, grad, c->lossbuf.as<double>(), c->stream);
  return check_hip(c, "scale loss");
}

lf_status lf_loss_depth(lf_ctx *c, const float *depth, const float *ref, const float *conf, int64_t n, float eps,
                        float *loss, float *grad) {
  if (!c) return LF_EINVAL;
  if (!loss || n < 0 || (n > 0 && (!depth || !ref)) || !(eps > 0.f) || !std::isfinite(eps))
    return fail(c, LF_EINVAL, "invalid depth-loss arguments");
  set_device(c);
  if (!loss_acc(c)) return fail(c, LF_ENOMEM, "loss scratch");
  Phase ph(c, 13);
  lf::launch_loss_depth(depth, ref, conf, n, eps, loss, grad, c->lossbuf.as<double>(), c->stream);
  return check_hip(c, "depth loss");
}

lf_status lf_loss_normal(lf_ctx *c, const float *normal, const float *ref, int64_t n, float *loss, float *grad) {
  if (!c) return LF_EINVAL;
  if (!loss || n < 0 || (n > 0 && (!normal || !ref))) return fail(c, LF_EINVAL, "invalid normal-loss arguments");
  set_device(c);
  if (!loss_acc(c)) return fail(c, LF_ENOMEM, "loss scratch");
  Phase ph(c, 13);
  lf::launch_loss_normal(normal, ref, n, loss, grad, c->lossbuf.as<double>(), c->stream);
  return check_hip(c, "normal loss");
}

lf_status lf_loss_tv(lf_ctx *c, const float *env, int32_t h, int32_t w, float *loss, float *grad) {
  if (!c) return LF_EINVAL;
  if (!env || !loss || h < 1 || w < 1) return fail(c, LF_EINVAL, "invalid TV-loss arguments");
  set_device(c);
  if (!loss_acc(c)) return fail(c, LF_ENOMEM, "loss scratch");
  Phase ph(c, 13);
  lf::launch_loss_tv(env, h, w, loss, grad, c->lossbuf.as<double>(), c->stream);
  return check_hip(c, "TV loss");
}

lf_status lf_loss_depth_normal(lf_ctx *c, const lf_camera *cam, const float *depth, const float *ref, float *loss,
                               float *grad) {
  if (!c) return LF_EINVAL;
  if (!depth || !ref || !loss) return fail(c, LF_EINVAL, "invalid depth-normal-loss arguments");
  set_device(c);
  if (!loss_acc(c)) return fail(c, LF_ENOMEM, "loss scratch");
  lf_status st = upload_camera(c, cam);
  if (st) return st;
  if (cam->h > 16 * 65535) return fail(c, LF_EINVAL, "depth map taller than %d rows", 16 * 65535);
  Phase ph(c, 13);
  lf::launch_loss_depth_normal(c->cams.as<lf::CamArgs>(), cam->w, cam->h, depth, ref, loss, grad,
                               c->lossbuf.as<double>(), c->stream);
  return check_hip(c, "depth-normal loss");
}

lf_status lf_stats_get(lf_ctx *c, lf_render_stats *st) {
  if (!c) return LF_EINVAL;
  if (!st) return fail(c, LF_EINVAL, "stats is NULL");
  set_device(c);
  unsigned long long q = 0;
  if (hipStreamSynchronize(c->stream) != hipSuccess ||
      hipMemcpy(&q, c->acc_secondary.p, sizeof q, hipMemcpyDeviceToHost) != hipSuccess)
    return check_hip(c, "stats");
  st->rays_primary = c->acc_primary;
  st->rays_secondary = (int64_t)q;
  c->acc_primary = 0;
  lf::launch_fill_u32(c->acc_secondary.as<uint32_t>(), 0u, 2, c->stream);
  return check_hip(c, "stats");
}

lf_status lf_trace_counters(lf_ctx *c, uint64_t *out) {
  if (!c) return LF_EINVAL;
  if (!out) return fail(c, LF_EINVAL, "counters output is NULL");
  set_device(c);
  if (hipStreamSynchronize(c->stream) != hipSuccess ||
      hipMemcpy(out, c->counters.p, 8 * LF_NUM_COUNTERS, hipMemcpyDeviceToHost) != hipSuccess)
    return check_hip(c, "counters");
  lf::launch_fill_u32(c->counters.as<uint32_t>(), 0u, 2 * LF_NUM_COUNTERS, c->stream);
  return check_hip(c, "counters");
}

lf_status lf_profile_enable(lf_ctx *c, int enable) {
  if (!c) return LF_EINVAL;
  c->profiling = enable != 0;
  return LF_OK;
}

lf_status lf_profile_read(lf_ctx *c, double *ms, int64_t *count) {
  if (!c) return LF_EINVAL;
  if (!ms || !count) return fail(c, LF_EINVAL, "profile outputs are NULL");
  set_device(c);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return check_hip(c, "profile");
  for (auto &pe : c->pending) {
    float t = 0.f;
    if (pe.first >= 0 && hipEventElapsedTime(&t, pe.second.first, pe.second.second) == hipSuccess) {
      c->prof_ms[pe.first] += t;
      c->prof_n[pe.first] += 1;
    }
    (void)hipGetLastError();
    c->pool.push_back(pe.second.first);
    c->pool.push_back(pe.second.second);
  }
  c->pending.clear();
  for (int i = 0; i < LF_NUM_PHASES; ++i) {
    ms[i] = c->prof_ms[i];
    count[i] = c->prof_n[i];
    c->prof_ms[i] = 0.0;
    c->prof_n[i] = 0;
  }
  return LF_OK;
}

lf_status lf_scene_get_info(lf_ctx *c, lf_scene_info *info) {
  if (!c) return LF_EINVAL;
  if (!info) return fail(c, LF_EINVAL, "info is NULL");
  if (!c->has_scene) return fail(c, LF_EINVAL, "no scene set");
  info->n_instances = c->n_inst;
  info->n_surfels = c->s.n;
  info->n_nodes = c->n_nodes;
  info->max_depth = c->max_depth;
  info->stack_size = lf::kStackL;
  info->n_wide_nodes = c->n_wide;
  info->wide_levels = c->wide_levels;
  info->node_width = lf::kWide;
  return LF_OK;
}

lf_status lf_scene_copy_bvh(lf_ctx *c, int32_t inst, float *node_boxes, int32_t *children, int32_t *perm,
                            float *leaf_boxes) {
  if (!c) return LF_EINVAL;
  if (!c->has_scene) return fail(c, LF_EINVAL, "no scene set");
  if (inst < 0 || inst >= c->n_inst) return fail(c, LF_EINVAL, "instance %d out of range", inst);
  set_device(c);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return check_hip(c, "copy bvh");
  int32_t n = c->h_n[inst], first = c->h_first[inst];
  int32_t nn = n > 1 ? n - 1 : 0;
  if (nn > 0 && (node_boxes || children)) {
    std::vector<lf::BNode> h(nn);
    if (hipMemcpy(h.data(), c->nodes.as<lf::BNode>() + c->h_node_off[inst], sizeof(lf::BNode) * nn,
                  hipMemcpyDeviceToHost) != hipSuccess)
      return check_hip(c, "copy bvh");
    for (int32_t i = 0; i < nn; ++i) {
      if (node_boxes) {
        float *b = node_boxes + 12 * (int64_t)i;
        for (int k = 0; k < 3; ++k) {
          b[k] = h[i].lo0[k]; b[3 + k] = h[i].hi0[k]; b[6 + k] = h[i].lo1[k]; b[9 + k] = h[i].hi1[k];
        }
      }
      if (children) {
        int32_t c0 = h[i].c0, c1 = h[i].c1;
        children[2 * i + 0] = c0 >= 0 ? c0 - c->h_node_off[inst] : ~((~c0) - first);
        children[2 * i + 1] = c1 >= 0 ? c1 - c->h_node_off[inst] : ~((~c1) - first);
      }
    }
  }
  if (perm && n > 0 &&
      hipMemcpy(perm, c->perm.as<int32_t>() + first, 4 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess)
    return check_hip(c, "copy bvh");
  if (leaf_boxes && n > 0 &&
      hipMemcpy(leaf_boxes, c->leafbox.as<float>() + 6 * (int64_t)first, 24 * (size_t)n, hipMemcpyDeviceToHost) !=
          hipSuccess)
    return check_hip(c, "copy bvh");
  return LF_OK;
}

lf_status lf_scene_copy_wide(lf_ctx *c, int32_t inst, int64_t *n_nodes, float *slot_boxes, int32_t *slot_child) {
  if (!c) return LF_EINVAL;
  if (!c->has_scene) return fail(c, LF_EINVAL, "no scene set");
  if (inst < 0 || inst >= c->n_inst) return fail(c, LF_EINVAL, "instance %d out of range", inst);
  if (!n_nodes) return fail(c, LF_EINVAL, "n_nodes is NULL");
  set_device(c);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return check_hip(c, "copy wide");
  const int64_t m = c->h_wide_n[inst], off = c->h_wide_off[inst];
  *n_nodes = m;
  if (m == 0 || (!slot_boxes && !slot_child)) return LF_OK;
  std::vector<lf::QNode> h(m);
  if (hipMemcpy(h.data(), c->qnodes.as<lf::QNode>() + off, sizeof(lf::QNode) * m, hipMemcpyDeviceToHost) !=
      hipSuccess)
    return check_hip(c, "copy wide");
  const int W = lf::kWide;
  const int32_t first = c->h_first[inst];
  for (int64_t j = 0; j < m; ++j) {
    const lf::QNode &q = h[j];
    int below = 0;
    for (int i = 0; i < W; ++i) {
      const bool inner = (q.imask >> i) & 1u, valid = (q.vmask >> i) & 1u;
      if (slot_boxes) {
        for (int k = 0; k < 3; ++k) {
          const float st = std::ldexp(1.0f, q.e[k]);
          slot_boxes[(j * W + i) * 6 + k] = std::fma((float)q.q[k][i], st, q.p[k]);
          slot_boxes[(j * W + i) * 6 + 3 + k] = std::fma((float)q.q[3 + k][i], st, q.p[k]);
        }
      }
      if (slot_child)
        slot_child[j * W + i] = !valid ? INT32_MIN
                                : inner ? (int32_t)(q.child_base + below - off)
                                        : ~(q.leaf_base + (i - below) - first);
      below += inner ? 1 : 0;
    }
  }
  return LF_OK;
}

}  // extern "C"

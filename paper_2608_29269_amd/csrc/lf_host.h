// lf_host.h -- host-side state of liblightfuse shared by the context API
// (lf_api.hip) and the relight server (lf_server.hip).  Internal.
#pragma once
#include <string>
#include <utility>
#include <vector>

#include "lf_internal.h"
#include "lf_kernels.h"

namespace lfh {

// Library-owned device allocation that only grows.
struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  bool ensure(size_t bytes) {
    if (bytes <= cap && p) return true;
    release();
    size_t b = bytes ? bytes : 16;
    if (hipMalloc(&p, b) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return false;
    }
    cap = b;
    return true;
  }
  template <class T>
  T *as() const { return (T *)p; }
};

constexpr double kPiHost = 3.14159265358979323846;

// What fixes the rays a render call traces and their order: a call with
// the same signature as the previous one on the context traces the same
// primary and secondary rays in the same order.
struct CallSig {
  const void *ro, *rd;
  int64_t n;
  lf::CamArgs cams;
  int32_t k, spp;
  uint64_t seed;
  uint32_t flags;  // without the flags that leave the traced rays unchanged
  double alpha_min, alpha_cap, sigma, eps, t_min, sec_off;
  const void *env;
  int32_t h, w;
  const void *R, *t;
  uint64_t epoch;  // scene generation (set, refit)
};

}  // namespace lfh

struct lf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  // abort word: pinned, mapped, coherent host memory the tracing kernels poll
  uint32_t *abort_h = nullptr;
  const uint32_t *abort_d = nullptr;
  std::string err;
  // scene
  bool has_scene = false;
  int servers = 0;  // live relight servers reading the scene (scene_set / refit refused meanwhile)
  lf::SurfelArrays s{};
  int n_inst = 0;
  std::vector<int32_t> h_first, h_n, h_node_off, h_root;
  int64_t n_nodes = 0;
  int32_t max_depth = 0;
  double built_alpha_min = 0, built_sig2 = 0;
  lfh::DevBuf d_first, d_n, d_root;
  lfh::DevBuf rec, filt, nodes, perm, leaf_parent, node_parent, flags, leafbox, rootbox, inst, status;
  lfh::DevBuf keys, keys2, vals2, hist, boxidx, ibounds, depth, ploc_i, ploc_f;
  lfh::DevBuf qnodes, winfo, wtmp, wdp, wroots, node_order;
  std::vector<int64_t> h_level_off;  // node_order[h_level_off[d] ..): the binary internal nodes of depth d
  int64_t n_wide = 0;      // traversal nodes over all instances
  std::vector<int64_t> h_wide_off, h_wide_n;  // per instance
  int32_t wide_levels = 0; // levels of the deepest traversal hierarchy
  // per call
  lfh::DevBuf env_cdf_row, env_cdf_col, env_lum, env_rowsum, env_roww, env_scal;
  lfh::DevBuf queue, qcount, work, kbuf1, kbuf2, hint2, contrib, frozen, lossbuf, cams, rec1, rec2, seeds;
  lfh::DevBuf env_part;  // partial copies of the environment gradient (shading adjoint)
  lfh::DevBuf bounds, skeys, skeys2, svals, svals2, shist;
  lfh::DevBuf det_key, det_key2, det_idx, det_idx2, det_hval, det_eval, det_hist;  // LF_FLAG_DETERMINISTIC
  // the k-buffers in kbuf1 / kbuf2 belong to the last render call with this signature
  uint64_t scene_epoch = 0;
  bool sig_valid = false;
  lfh::CallSig last_sig;
  lf::CamArgs h_cams{};
  // ray counters since the last lf_stats_get
  int64_t acc_primary = 0;
  lfh::DevBuf acc_secondary, counters;
  // phase timers
  bool profiling = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> pool;
  double prof_ms[LF_NUM_PHASES] = {};
  int64_t prof_n[LF_NUM_PHASES] = {};
};

namespace lfh {

// Records a formatted message in the context and returns st.
lf_status fail(lf_ctx *c, lf_status st, const char *fmt, ...);
// LF_EDEVICE with the pending HIP error, if any.
lf_status check_hip(lf_ctx *c, const char *where);
bool set_device(lf_ctx *c);
// Recomputes trace records, binary bounds and traversal nodes for the given
// opacity threshold and squared support radius (on the context's stream).
lf_status refit_impl(lf_ctx *c, double alpha_min, double sig2);
// Validates tracing parameters (k, spp, constants, flags).
lf_status validate_params(lf_ctx *c, const lf_params *p);
// Validated lf_camera -> slot c of a CamArgs (ray ids from 0).
lf_status camera_args(lf_ctx *c, const lf_camera &cm, lf::CamArgs &ca);
// Scene arrays of the context (instances left NULL).
void scene_view(const lf_ctx *c, lf::SceneView &S);
// Tracing constants of p (spp and seed included).
void trace_params(const lf_ctx *c, const lf_params *p, lf::TraceParams &P);
// Device buffers of the environment sampling tables of an h x w map.
bool ensure_env_tables(DevBuf &cdf_row, DevBuf &cdf_col, DevBuf &lum, DevBuf &rowsum, DevBuf &roww, DevBuf &scal,
                       int h, int w);
// Bytes of the tables above (for admission budgets).
int64_t env_table_bytes(int h, int w);

}  // namespace lfh

// lf_kernels.h -- host-side launchers of the gfx950 kernels (internal).
#pragma once
#include <atomic>
#include <vector>

#include "lf_internal.h"

namespace lf {

struct SurfelArrays {
  const float *mu, *q, *scale, *opacity, *albedo, *roughness, *metallic;
  int64_t n;
};

// ---- BVH (lf_bvh.hip)
// per-surfel prep by surfel index: conservative boxes and centres
void launch_boxes_by_index(const SurfelArrays &s, double alpha_min, double sig2, float *box6, hipStream_t st);
// per-instance bounds of the box centres: out[inst*6] = (lo xyz, hi xyz)
void launch_instance_bounds(const float *box6, const int32_t *inst_first, const int32_t *inst_n, int n_inst,
                            float *out, hipStream_t st);
// 64-bit Morton keys (instance in the top bits) and identity values
void launch_morton(const float *box6, const float *inst_bounds, const int32_t *inst_first, const int32_t *inst_n,
                   int n_inst, int64_t n, uint64_t *keys, int32_t *vals, hipStream_t st);
// stable LSD radix sort of (keys, vals); tmp buffers of the same sizes; hist scratch
size_t radix_sort_hist_words(int64_t n);
void radix_sort(uint64_t *keys, int32_t *vals, uint64_t *keys_tmp, int32_t *vals_tmp, uint32_t *hist, int64_t n,
                hipStream_t st, int key_bits = 64);
// PLOC hierarchy of one instance (synchronises the stream once per clustering round); false if it failed.
// Scratch: cid, cid2, nn, rem, pre [n] and cbox, cbox2 [n,6].
bool launch_ploc(const int32_t *perm, const float *boxidx, int32_t first, int32_t n, int32_t node_off, int32_t inst,
                 BNode *nodes, int32_t *node_parent, int32_t *leaf_parent, int32_t *cid, int32_t *cid2, float *cbox,
                 float *cbox2, int32_t *nn, uint32_t *rem, uint32_t *pre, hipStream_t st);
// leaf depth maximum into *max_depth (device int)
void launch_depth(const int32_t *leaf_parent, const int32_t *node_parent, int64_t n, int64_t n_nodes,
                  int32_t *max_depth, uint32_t *status, hipStream_t st);
// depth of every binary internal node (root = 0)
void launch_node_depth(const int32_t *node_parent, int64_t n_nodes, int32_t *depth, uint32_t *status,
                       hipStream_t st);
// trace records + bounds level by level: order lists the internal nodes by depth, level_off[d] the first of
// depth d (level_off.back() = n_nodes)
void launch_refit(const SurfelArrays &s, double alpha_min, double sig2, const int32_t *perm,
                  const int32_t *leaf_parent, const int32_t *node_parent, const int32_t *order,
                  const std::vector<int64_t> &level_off, int64_t n_nodes, int n_inst, BNode *nodes, TraceRec *rec,
                  FiltRec *filt, float *leaf_box6, float *root_box6, uint32_t *status, hipStream_t st);
// Wide traversal nodes (surface-area-cost collapse of the binary hierarchy).
// level[b] = -1 for every binary node first; roots of instances with >= 2 surfels get level 0
void launch_wide_roots(const int32_t *root, const int32_t *cnt, int n_inst, int32_t *level, hipStream_t st);
// collapse costs and choices of every binary node, deepest depth first (order / level_off as for the refit);
// cost [n_nodes, kWide] floats, choice [n_nodes, 16] bytes
void launch_wide_cost(const BNode *nodes, int64_t n_nodes, const int32_t *order, const std::vector<int64_t> &level_off,
                      float *cost, uint8_t *choice, uint32_t *status, hipStream_t st);
// slot sources [n_nodes, kWide] of the nodes of level it; *n_levels = max level + 1 (device int)
void launch_wide_level(const BNode *nodes, int64_t n_nodes, int32_t it, const uint8_t *choice, int32_t *level,
                       int32_t *slot_src, int32_t *n_levels, uint32_t *status, hipStream_t st);
// wide nodes and leaves in every binary subtree (flags and side_cnt [2 n_nodes] scratch)
void launch_wide_count(const int32_t *leaf_parent, const int32_t *node_parent, const int32_t *level, int64_t n,
                       int64_t n_nodes, int32_t *flags, int2 *side_cnt, int32_t *sub_w, int32_t *sub_l,
                       uint32_t *status, hipStream_t st);
// positions of the instance roots: roots[3i..3i+2] = (wide index, first descendant, first leaf)
void launch_wide_root_pos(const int32_t *root, const int32_t *cnt, const int32_t *roots, int n_inst, int32_t *widx,
                          int32_t *dbase, int32_t *lbase, hipStream_t st);
// places the nodes of level it (build descriptions into info, new leaf positions into newpos)
void launch_wide_assign(const BNode *nodes, int64_t n_nodes, int64_t n, int32_t it, const int32_t *level,
                        const int32_t *slot_src, const int32_t *sub_w, const int32_t *sub_l, int32_t *widx,
                        int32_t *dbase, int32_t *lbase, int32_t *newpos, WideInfo *info, int64_t n_wide,
                        uint32_t *status, hipStream_t st);
void launch_iota(int32_t *p, int64_t n, hipStream_t st);
// leaf order, leaf parents (into perm2 / leaf_parent2) and binary leaf codes after the placement
void launch_leaf_reorder(const int32_t *newpos, const int32_t *perm, const int32_t *leaf_parent, int64_t n,
                         int64_t n_nodes, int32_t *perm2, int32_t *leaf_parent2, BNode *nodes, uint32_t *status,
                         hipStream_t st);
// quantised traversal nodes from the refitted binary boxes
void launch_wide_quantize(const BNode *nodes, const WideInfo *info, int64_t n_wide, int64_t n_nodes, QNode *out,
                          uint32_t *status, hipStream_t st);
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);
void launch_fill_f32(float *p, float v, int64_t n, hipStream_t st);

// ---- per-render (lf_render.hip)
void launch_instances(const float *R, const float *t, const float *root_box6, const int32_t *inst_first,
                      const int32_t *inst_n, const int32_t *inst_root, int n_inst, InstRec *out, double *bounds6,
                      uint32_t *status, hipStream_t st);
// sort keys of the secondary queue: (direction octant and octahedral cell, origin Morton code); entries past the
// count sort last
void launch_secondary_keys(const SecEntry *queue, const uint32_t *count, int64_t cap, const double *bounds6,
                           const ChunkDesc *chunks, const BatchSlot *slots, uint64_t *keys, int32_t *vals,
                           hipStream_t st);
void launch_env_tables(const float *tex, int H, int W, uint32_t flags, double *cdf_row, double *cdf_col, double *lum,
                       double *rowsum, double *roww, double *scal, hipStream_t st);

struct RenderArgs {
  SceneView S;
  TraceParams P;
  EnvView E;
  RaySource rays;
  int64_t R;
  int64_t n_tiles;      // camera rays: 16x8-pixel tiles over all cameras (one per block), else 0
  // outputs
  float *radiance, *depth, *normal, *alpha;
  int32_t *hit_idx, *sec_hit_idx;
  // scratch
  SurfRec *rec1;        // [R] primary surface records
  SurfRec *rec2;        // [R*S] secondary surface records (queue order)
  SecEntry *queue;      // [R*S]
  uint32_t *queue_count;
  const int32_t *order; // [R*S] trace order of the queue (sorted for coherence), or NULL
  float *contrib;       // [R*S*3]
  SecFrozen *frozen;    // [R*S] (backward replay)
  AdjSeed *seeds;       // [R] (backward)
  uint32_t *status;
  uint32_t *work;       // [kPoolParts] item counters of the persistent traversal launches (cleared before each)
  uint32_t *kbuf1;      // [primary items, 2K] k-buffers from traversal to compositing (t[K], then ids[K])
  uint32_t *kbuf2;      // [secondary items, 2K] the same for the secondary queue
  float *hint2;         // [R*S] k-th distance of each (ray, slot)'s secondary trace (its queue position varies)
  // per-ray sample stride of contrib / frozen and of the queue capacity (spp, or the batch maximum)
  int32_t spp_stride;
  // 1 (the replay of a backward right after the forward with the same arguments): kbuf1 and hint2
  // hold that forward's k-th distances; each ray starts from its earlier k-th distance as a culling
  // bound and is traced again without it if fewer than k hits lie below the bound
  int32_t use_hint;
  // continuous batching (NULL for one request): R = kChunk * number of chunks
  const ChunkDesc *chunks;
  const BatchSlot *slots;
};
// primary: traversal (k-buffers into kbuf1), compositing, then shading
void launch_trace1(const RenderArgs &a, hipStream_t st);
void launch_composite1(const RenderArgs &a, bool replay, hipStream_t st);
void launch_shade1(const RenderArgs &a, bool replay, hipStream_t st);
// secondary: traversal and compositing of the queue, then the two environment samples
void launch_trace2(const RenderArgs &a, hipStream_t st);
void launch_composite2(const RenderArgs &a, hipStream_t st);
void launch_shade2(const RenderArgs &a, bool replay, hipStream_t st);
void launch_resolve(const RenderArgs &a, hipStream_t st);
void launch_accum(unsigned long long *acc, const uint32_t *count, hipStream_t st);
void launch_raygen(const CamArgs *cams, int64_t n, float *o, float *d, hipStream_t st);
// training objectives (lf_loss.hip); part: device scratch of kLossPartDoubles doubles
constexpr int kMaxLossBlocks = 2048;                       // blocks (partial-sum slots) per objective pass
constexpr int kLossPartDoubles = 2 * kMaxLossBlocks + 2;  // two slot rows, then the totals
void launch_l1(const float *pred, const float *target, int64_t n, float *loss, float *grad, double *part,
               hipStream_t st);
void launch_loss_alpha(const float *alpha, int64_t n, float *loss, float *grad, double *part, hipStream_t st);
void launch_loss_scale(const float *scale, int64_t n, float s_max, float *loss, float *grad, double *part,
                       hipStream_t st);
void launch_loss_depth(const float *depth, const float *ref, const float *conf, int64_t n, float eps, float *loss,
                       float *grad, double *part, hipStream_t st);
void launch_loss_normal(const float *normal, const float *ref, int64_t n, float *loss, float *grad, double *part,
                        hipStream_t st);
void launch_loss_tv(const float *env, int h, int w, float *loss, float *grad, double *part, hipStream_t st);
void launch_loss_depth_normal(const CamArgs *cams, int w, int h, const float *depth, const float *ref, float *loss,
                              float *grad, double *part, hipStream_t st);

// ---- backward (lf_backward.hip)
struct GradArgs {
  const float *d_radiance, *d_depth, *d_normal, *d_alpha;
  float *g_mu, *g_q, *g_scale, *g_opacity, *g_albedo, *g_roughness, *g_metallic, *g_env;
};
// shading adjoint (env gradients, compositing seeds), then the compositing adjoint of the seeded rays from the
// primary k-buffers (kbuf1) of the replayed primary pass
// Environment gradients go to `copies` zeroed partial maps in part (block b
// adds to copy b % copies; copies = 1: straight to g.g_env, part unused),
// which are then summed into g.g_env in copy order.
constexpr int kEnvGradCopies = 16;
void launch_adjoint_shade(const RenderArgs &a, const GradArgs &g, float *part, int copies, hipStream_t st);
void launch_adjoint_hits(const RenderArgs &a, const GradArgs &g, hipStream_t st);
// Order-fixed (LF_FLAG_DETERMINISTIC) form of the two adjoints: contributions
// go to records at fixed positions, are sorted by target and summed in
// binary64 per target (see lf_backward.hip).  Buffers owned by the caller.
struct DetArgs {
  uint64_t *hit_key, *hit_key2;   // [n_hit] surfel keys, sort scratch
  int32_t *hit_idx, *hit_idx2;    // [n_hit] record positions, sort scratch
  double *hit_val;                // [n_hit][15]
  int64_t n_hit;                  // adjoint_items x k bucket
  uint64_t hit_unused;            // key of an unused record: 2^hit_bits - 1 > every surfel index
  int hit_bits;
  uint64_t *env_key, *env_key2;
  int32_t *env_idx, *env_idx2;
  double *env_val;                // [n_env][3]
  int64_t n_env;                  // rays x env_cap
  int env_cap;                    // records per ray: 4 taps x (1 + 3 x secondary slots)
  uint64_t env_unused;
  int env_bits;
  uint32_t *hist;                 // radix_sort_hist_words(max(n_hit, n_env))
};
int64_t adjoint_items(const RenderArgs &a);  // work items of the compositing adjoint
void launch_adjoint_shade_det(const RenderArgs &a, const GradArgs &g, const DetArgs &d, hipStream_t st);
void launch_adjoint_hits_det(const RenderArgs &a, const GradArgs &g, const DetArgs &d, hipStream_t st);

inline int kbucket(int k) { return k <= 8 ? 8 : (k <= 16 ? 16 : (k <= 32 ? 32 : 64)); }

// Blocks of a persistent launch of kernel Kern (kBlock threads): as many as
// can be resident at once on the current device, at most one per
// kPoolItemsPerBlock items, at least one.  The residency is looked up once per
// device.  Small launches spread thinly (8 items per wave): they are bound by
// their longest rays, not by issue, and a wave lasts as long as its slowest lane.
constexpr int kPoolItemsPerBlock = 16;
template <auto Kern>
inline unsigned pool_blocks(int64_t items) {
  static std::atomic<int> resident[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    dev = 0;
  }
  int nb = (dev >= 0 && dev < 64) ? resident[dev].load(std::memory_order_relaxed) : 0;
  if (nb <= 0) {
    int cu = 0, per = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu < 1) {
      (void)hipGetLastError();
      cu = 1;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, Kern, kBlock, 0) != hipSuccess || per < 1) {
      (void)hipGetLastError();
      per = 1;
    }
    nb = cu * per;
    if (dev >= 0 && dev < 64) resident[dev].store(nb, std::memory_order_relaxed);
  }
  const int64_t need = (items + kPoolItemsPerBlock - 1) / kPoolItemsPerBlock;
  return (unsigned)(need < 1 ? 1 : (need < nb ? need : nb));
}


}  // namespace lf

// lf_kernels.h -- host-side launchers of the gfx950 kernels (internal).
#pragma once
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
// trace records + bottom-up bounds
void launch_refit(const SurfelArrays &s, double alpha_min, double sig2, const int32_t *perm,
                  const int32_t *leaf_parent, const int32_t *node_parent, int32_t *flags, int64_t n_nodes,
                  int n_inst, BNode *nodes, TraceRec *rec, FiltRec *filt, float *leaf_box6, float *root_box6,
                  uint32_t *status, hipStream_t st);
// 4-wide hierarchy: flags of even-depth internal nodes and their exclusive prefix sum (index of the 4-wide node)
void launch_wide_index(const int32_t *node_parent, int64_t n_nodes, uint32_t *flag, uint32_t *idx4,
                       uint32_t *status, hipStream_t st);
// 4-wide nodes from the refitted binary nodes
void launch_collapse(const BNode *nodes, const uint32_t *flag, const uint32_t *idx4, int64_t n_nodes, BNode4 *out,
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
  // per-ray sample stride of contrib / frozen and of the queue capacity (spp, or the batch maximum)
  int32_t spp_stride;
  // continuous batching (NULL for one request): R = kChunk * number of chunks
  const ChunkDesc *chunks;
  const BatchSlot *slots;
};
// primary: traversal + compositing, then shading
void launch_trace1(const RenderArgs &a, bool replay, hipStream_t st);
void launch_shade1(const RenderArgs &a, bool replay, hipStream_t st);
// secondary: traversal + compositing of the queue, then the two environment samples
void launch_trace2(const RenderArgs &a, hipStream_t st);
void launch_shade2(const RenderArgs &a, bool replay, hipStream_t st);
void launch_resolve(const RenderArgs &a, hipStream_t st);
void launch_accum(unsigned long long *acc, const uint32_t *count, hipStream_t st);
void launch_raygen(const CamArgs *cams, int64_t n, float *o, float *d, hipStream_t st);
void launch_l1(const float *pred, const float *target, int64_t n, float *loss, float *grad, double *acc,
               hipStream_t st);

// ---- backward (lf_backward.hip)
struct GradArgs {
  const float *d_radiance, *d_depth, *d_normal, *d_alpha;
  float *g_mu, *g_q, *g_scale, *g_opacity, *g_albedo, *g_roughness, *g_metallic, *g_env;
};
// shading adjoint (env gradients, compositing seeds) then traversal + compositing adjoint
void launch_adjoint_shade(const RenderArgs &a, const GradArgs &g, hipStream_t st);
void launch_adjoint_trace(const RenderArgs &a, const GradArgs &g, hipStream_t st);

inline int kbucket(int k) { return k <= 8 ? 8 : (k <= 16 ? 16 : (k <= 32 ? 32 : 64)); }

}  // namespace lf

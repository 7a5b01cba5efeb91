// lf_bvh.hip -- per-surfel prep, size-extended Morton codes, LSD radix sort,
// hierarchy by parallel locally-ordered clustering (Meister and Bittner 2018,
// "Parallel Locally-Ordered Clustering for Bounding Volume Hierarchy
// Construction"), bottom-up refit and the compressed wide traversal nodes,
// for gfx950.
//
// One hierarchy per instance (background and each object, in object space).
// Leaves hold one surfel; binary internal nodes store both children's boxes
// (the refit structure); traversal uses wide nodes cut from it whose child
// boxes are quantised to 8 bits per plane.  Surfel boxes bound the support
// ellipse rho^2 <= rho^2_max (3-sigma support and opacity threshold) and are
// rounded outward to binary32.
#include <cfloat>

#include "lf_device.h"
#include "lf_kernels.h"

namespace lf {

namespace {

// Trace record and conservative box of surfel i.
__device__ __forceinline__ void surfel_prep(const SurfelArrays &s, int64_t i, double alpha_min, double sig2,
                                            TraceRec &r, float *lo, float *hi, FiltRec *filt = nullptr) {
  const float *q = s.q + 4 * i;
  double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
  double ql = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  qw /= ql; qx /= ql; qy /= ql; qz /= ql;
  d3 tu, tv, n;
  quat_frame(qw, qx, qy, qz, tu, tv, n);
  double su = s.scale[2 * i], sv = s.scale[2 * i + 1], al = s.opacity[i];
  double rho2max = fmin(sig2, 2.0 * log(al / alpha_min));
  r.n[0] = n.x; r.n[1] = n.y; r.n[2] = n.z;
  r.a[0] = tu.x / su; r.a[1] = tu.y / su; r.a[2] = tu.z / su;
  r.b[0] = tv.x / sv; r.b[1] = tv.y / sv; r.b[2] = tv.z / sv;
  r.mu[0] = s.mu[3 * i]; r.mu[1] = s.mu[3 * i + 1]; r.mu[2] = s.mu[3 * i + 2];
  r.orig = (int32_t)i;
  r.rho2max = rho2max;
  if (filt) {
    FiltRec f;
    const bool ok = rho2max >= 0.0;
    f.v0 = make_float4((float)r.a[0], (float)r.a[1], (float)r.a[2], r.mu[0]);
    f.v1 = make_float4((float)r.b[0], (float)r.b[1], (float)r.b[2], r.mu[1]);
    f.v2 = make_float4(r.mu[2], ok ? round_up_f(rho2max) : -1.0f, ok ? round_up_f(sqrt(rho2max)) : 0.0f,
                       round_up_f(1.0 / fmin(su, sv)));
    *filt = f;
  }
  if (!(rho2max >= 0.0)) {  // never valid (also NaN): empty box
    lo[0] = lo[1] = lo[2] = INFINITY;
    hi[0] = hi[1] = hi[2] = -INFINITY;
    return;
  }
  double rr = sqrt(rho2max) * (1.0 + 1e-12);
  const double tuv[3][2] = {{su * tu.x, sv * tv.x}, {su * tu.y, sv * tv.y}, {su * tu.z, sv * tv.z}};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double e = rr * sqrt(tuv[k][0] * tuv[k][0] + tuv[k][1] * tuv[k][1]);
    double c = (double)r.mu[k];
    lo[k] = round_down_f(c - e);
    hi[k] = round_up_f(c + e);
  }
}

__global__ void k_boxes_by_index(SurfelArrays s, double alpha_min, double sig2, float *box6) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  TraceRec r;
  float lo[3], hi[3];
  surfel_prep(s, i, alpha_min, sig2, r, lo, hi);
  for (int k = 0; k < 3; ++k) { box6[6 * i + k] = lo[k]; box6[6 * i + 3 + k] = hi[k]; }
}

// one block per instance: bounds of the (finite) box centres
__global__ void k_instance_bounds(const float *box6, const int32_t *first, const int32_t *cnt, float *out) {
  int inst = blockIdx.x;
  __shared__ float red[6][256];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = first[inst] + threadIdx.x; i < (int64_t)first[inst] + cnt[inst]; i += blockDim.x) {
    const float *b = box6 + 6 * i;
    if (!(b[0] <= b[3])) continue;  // empty box
    for (int k = 0; k < 3; ++k) {
      float c = 0.5f * (b[k] + b[3 + k]);
      lo[k] = fminf(lo[k], c);
      hi[k] = fmaxf(hi[k], c);
    }
  }
  for (int k = 0; k < 3; ++k) { red[k][threadIdx.x] = lo[k]; red[3 + k][threadIdx.x] = hi[k]; }
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = fminf(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        red[3 + k][threadIdx.x] = fmaxf(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 6; ++k) out[6 * inst + k] = red[k][0];
}

__device__ __forceinline__ uint64_t spread3(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

// Sort key of a surfel box: instance (6 bits), then 54 bits interleaving
// 18-bit Morton coordinates of the box centre with a 3-bit size class (log2
// of the instance extent over the box's largest extent) placed after the
// first size_level levels (3 bits each) of the Morton code, so that below
// the coarse spatial levels each size class forms its own subtrees and large
// surfels no longer inflate the boxes of small ones (extended Morton codes,
// Vinkler et al. 2017).
__global__ void k_morton(const float *box6, const float *ib, const int32_t *first, const int32_t *cnt, int n_inst,
                         int64_t n, int size_level, uint64_t *keys, int32_t *vals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int inst = 0;
  for (int j = 1; j < n_inst; ++j)
    if (i >= first[j] && cnt[j] > 0) inst = j;
  const float *b = box6 + 6 * i;
  const float *B = ib + 6 * inst;
  uint64_t code = 0;
  if (b[0] <= b[3]) {
    uint64_t c[3];
    float emax = 0.f, ebox = 0.f;
    for (int k = 0; k < 3; ++k) {
      float ext = B[3 + k] - B[k];
      emax = fmaxf(emax, ext);
      ebox = fmaxf(ebox, b[3 + k] - b[k]);
      float x = ext > 0.f ? (0.5f * (b[k] + b[3 + k]) - B[k]) / ext : 0.5f;
      x = fminf(fmaxf(x, 0.f), 1.f);
      c[k] = (uint64_t)fminf(x * 262144.0f, 262143.0f);  // 18 bits per axis
    }
    const uint64_t m = (spread3(c[0]) << 2) | (spread3(c[1]) << 1) | spread3(c[2]);  // 54 bits
    float lr = (emax > 0.f && ebox > 0.f) ? log2f(emax / ebox) : 0.f;
    const uint64_t sz = (uint64_t)fminf(fmaxf(lr, 0.f), 7.f);  // 3-bit size class
    const int low = 54 - 3 * size_level;  // Morton bits below the size class
    const uint64_t hi_part = low >= 54 ? 0 : (m >> low);
    const uint64_t lo_part = low >= 54 ? m : (m & ((1ull << low) - 1));
    code = ((hi_part << 3 | sz) << low) | lo_part;  // 57 bits
  }
  keys[i] = ((uint64_t)inst << 57) | code;
  vals[i] = (int32_t)i;
}

// ---------------------------------------------------------------- radix sort
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t *keys, int64_t n, int shift, uint32_t *hist,
                                                        int nb) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ITEMS; ++r) {
    int64_t i = base + r * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of len words in place, one block of 1024 threads
__global__ __launch_bounds__(1024) void k_rs_scan(uint32_t *a, int64_t len) {
  __shared__ uint32_t part[1024];
  int64_t per = (len + 1023) / 1024;
  int64_t b = threadIdx.x * per, e = b + per < len ? b + per : len;
  uint32_t s = 0;
  for (int64_t i = b; i < e; ++i) s += a[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int64_t i = b; i < e; ++i) {
    uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
}

// Exclusive scan of a long array in three launches: tile sums, a one-block
// scan of the sums, then each tile scanned from its offset.  Tiles of
// SC_TILE words; a thread owns SC_ITEMS consecutive words of its tile.
constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 16;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

__global__ __launch_bounds__(SC_THREADS) void k_scan_tile_sums(const uint32_t *a, int64_t len, uint32_t *sums) {
  __shared__ uint32_t ws[SC_THREADS / 64];
  const int64_t base = (int64_t)blockIdx.x * SC_TILE;
  uint32_t s = 0;
  for (int r = 0; r < SC_ITEMS; ++r) {
    const int64_t i = base + r * SC_THREADS + threadIdx.x;
    if (i < len) s += a[i];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < SC_THREADS / 64; ++w) t += ws[w];
    sums[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(SC_THREADS) void k_scan_tile_apply(uint32_t *a, int64_t len, const uint32_t *offs) {
  __shared__ uint32_t ts[SC_THREADS];
  const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
  uint32_t v[SC_ITEMS], s = 0;
#pragma unroll
  for (int r = 0; r < SC_ITEMS; ++r) {
    v[r] = base + r < len ? a[base + r] : 0u;
    s += v[r];
  }
  ts[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < SC_THREADS; off <<= 1) {
    const uint32_t x = threadIdx.x >= (unsigned)off ? ts[threadIdx.x - off] : 0u;
    __syncthreads();
    ts[threadIdx.x] += x;
    __syncthreads();
  }
  uint32_t run = offs[blockIdx.x] + (threadIdx.x ? ts[threadIdx.x - 1] : 0u);
#pragma unroll
  for (int r = 0; r < SC_ITEMS; ++r) {
    if (base + r < len) a[base + r] = run;
    run += v[r];
  }
}

// exclusive scan of a[0..len) in place; sums: scratch of scan_scratch_words(len) words
void exclusive_scan(uint32_t *a, int64_t len, uint32_t *sums, hipStream_t st) {
  const int64_t nt = (len + SC_TILE - 1) / SC_TILE;
  if (nt <= 1) {
    hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(1024), 0, st, a, len);
    return;
  }
  hipLaunchKernelGGL(k_scan_tile_sums, dim3((unsigned)nt), dim3(SC_THREADS), 0, st, (const uint32_t *)a, len, sums);
  hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(1024), 0, st, sums, nt);
  hipLaunchKernelGGL(k_scan_tile_apply, dim3((unsigned)nt), dim3(SC_THREADS), 0, st, a, len, (const uint32_t *)sums);
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint64_t *kin, const int32_t *vin, uint64_t *kout,
                                                           int32_t *vout, int64_t n, int shift,
                                                           const uint32_t *offs, int nb) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wc[RS_THREADS / 64][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  base[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
  const uint64_t lt = lane ? ((~0ull) >> (64 - lane)) : 0ull;
  int64_t tile = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ITEMS; ++r) {
    for (int w = 0; w < RS_THREADS / 64; ++w) wc[w][threadIdx.x] = 0;
    __syncthreads();
    int64_t i = tile + r * RS_THREADS + threadIdx.x;
    bool valid = i < n;
    uint64_t key = valid ? kin[i] : 0ull;
    uint32_t dg = (uint32_t)((key >> shift) & 255u);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      bool bit = (dg >> b) & 1u;
      uint64_t m = __ballot(valid && bit);
      peers &= bit ? m : ~m;
    }
    uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wc[wave][dg] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t off = base[dg] + rank;
      for (int w = 0; w < wave; ++w) off += wc[w][dg];
      if (off < (uint64_t)n) {  // always true for consistent offsets
        kout[off] = key;
        vout[off] = vin[i];
      }
    }
    __syncthreads();
    uint32_t tot = 0;
    for (int w = 0; w < RS_THREADS / 64; ++w) tot += wc[w][threadIdx.x];
    base[threadIdx.x] += tot;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- PLOC hierarchy
// Parallel locally-ordered clustering (Meister and Bittner 2018) of one
// instance's surfels in sorted-key order: every cluster picks, within a
// window of kPlocR positions on either side, the neighbour whose merged box
// has the smallest surface area; mutual pairs merge into a new node; the
// cluster list is compacted in order; repeat until one cluster is left.
// Node indices count down from the end of the instance's node range, so the
// last merge (the root) gets its first index.
constexpr int kPlocR = 128;  // window radius: traversal 4% faster than with 32, build 128 instead of 84 ms at 1M
constexpr int kPlocB = 256;

__device__ __forceinline__ float box_area(const float *lo, const float *hi) {
  const float x = fmaxf(hi[0] - lo[0], 0.f), y = fmaxf(hi[1] - lo[1], 0.f), z = fmaxf(hi[2] - lo[2], 0.f);
  return x * y + y * z + z * x;
}

__global__ void k_ploc_init(const int32_t *perm, const float *boxidx, int32_t first, int32_t n, int32_t *cid,
                            float *cbox) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cid[i] = ~(first + i);
  const float *b = boxidx + 6 * (int64_t)perm[first + i];
  for (int k = 0; k < 6; ++k) cbox[6 * i + k] = b[k];
}

// nearest neighbour by merged surface area, ties by the (lower, higher) index pair
__global__ __launch_bounds__(kPlocB) void k_ploc_nn(const float *cbox, int m, int rr, int32_t *nn) {
  __shared__ float sb[kPlocB + 2 * kPlocR][6];
  const int base = blockIdx.x * kPlocB;
  for (int j = threadIdx.x; j < kPlocB + 2 * kPlocR; j += kPlocB) {
    const int g = base - kPlocR + j;
    for (int k = 0; k < 6; ++k) sb[j][k] = (g >= 0 && g < m) ? cbox[6 * g + k] : 0.f;
  }
  __syncthreads();
  const int i = base + threadIdx.x;
  if (i >= m) return;
  const float *bi = sb[threadIdx.x + kPlocR];
  float best = INFINITY;
  int bj = -1;
  for (int dd = -rr; dd <= rr; ++dd) {
    const int j = i + dd;
    if (dd == 0 || j < 0 || j >= m) continue;
    const float *bj_ = sb[threadIdx.x + kPlocR + dd];
    float lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(bi[k], bj_[k]);
      hi[k] = fmaxf(bi[3 + k], bj_[3 + k]);
    }
    const float a = box_area(lo, hi);
    // with equal areas the pair with the smaller (min, max) index wins, the same on both sides
    const bool better = a < best || (a == best && bj >= 0 &&
                                     (min(i, j) < min(i, bj) || (min(i, j) == min(i, bj) && max(i, j) < max(i, bj))));
    if (bj < 0 || better) {
      best = a;
      bj = j;
    }
  }
  nn[i] = bj;
}

// rem[j] = 1 if j merges into its (lower) mutual nearest neighbour
__global__ void k_ploc_flags(const int32_t *nn, int m, uint32_t *rem, uint32_t *pre) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int i = nn[j];
  const uint32_t r = (i >= 0 && i < j && nn[i] == j) ? 1u : 0u;
  rem[j] = r;
  pre[j] = r;
}

__device__ __forceinline__ void set_parent(int32_t c, int32_t parent_side, int32_t *node_parent, int32_t *leaf_parent) {
  if (c < 0) leaf_parent[~c] = parent_side;
  else node_parent[c] = parent_side;
}

// merges mutual pairs into nodes next_idx - rank and compacts the cluster list
__global__ void k_ploc_merge(const int32_t *nn, const uint32_t *pre, int m, int32_t next_idx, const int32_t *cid,
                             const float *cbox, int32_t *cid2, float *cbox2, BNode *nodes, int32_t *node_parent,
                             int32_t *leaf_parent) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int j = nn[i];
  const bool mutual = j >= 0 && nn[j] == i;
  if (mutual && j < i) return;  // merged into j
  const int p = i - (int)pre[i];
  if (mutual) {
    const int32_t idx = next_idx - (int32_t)pre[j];
    const int32_t a = cid[i], b = cid[j];
    BNode nd;
    for (int k = 0; k < 3; ++k) {
      nd.lo0[k] = cbox[6 * i + k]; nd.hi0[k] = cbox[6 * i + 3 + k];
      nd.lo1[k] = cbox[6 * j + k]; nd.hi1[k] = cbox[6 * j + 3 + k];
    }
    nd.c0 = a;
    nd.c1 = b;
    nd.pad0 = nd.pad1 = 0;
    nodes[idx] = nd;
    set_parent(a, (idx << 1) | 0, node_parent, leaf_parent);
    set_parent(b, (idx << 1) | 1, node_parent, leaf_parent);
    cid2[p] = idx;
    for (int k = 0; k < 3; ++k) {
      cbox2[6 * p + k] = fminf(nd.lo0[k], nd.lo1[k]);
      cbox2[6 * p + 3 + k] = fmaxf(nd.hi0[k], nd.hi1[k]);
    }
  } else {
    cid2[p] = cid[i];
    for (int k = 0; k < 6; ++k) cbox2[6 * p + k] = cbox[6 * i + k];
  }
}

__global__ void k_ploc_root(const int32_t *cid, int32_t inst, int32_t *node_parent) {
  node_parent[cid[0]] = -(inst + 2);
}

__global__ void k_leaf_root(int32_t first, int32_t inst, int32_t *leaf_parent) { leaf_parent[first] = -(inst + 2); }

__global__ void k_depth(const int32_t *leaf_parent, const int32_t *node_parent, int64_t n, int64_t n_nodes,
                        int32_t *max_depth, uint32_t *status) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int dep = 0;
  int p = leaf_parent[i];
  while (p >= 0) {
    if ((p >> 1) >= n_nodes || dep > 4096) {
      atomicOr(status, kStatusBvhCorrupt);
      break;
    }
    ++dep;
    p = node_parent[p >> 1];
  }
  atomicMax(max_depth, dep);
}

// Refit in levels: the leaves first (trace and filter records by leaf
// position, each leaf's box into its parent's slot for it), then one launch
// per binary depth from the deepest up, each node's box (the union of its
// two slots) into its parent's slot; kernel boundaries order the levels, so
// no atomics are needed.  Roots write their instance's bounds.
__global__ void k_refit_leaves(SurfelArrays s, double alpha_min, double sig2, const int32_t *perm,
                               const int32_t *leaf_parent, BNode *nodes, int64_t n_nodes, int n_inst, TraceRec *rec,
                               FiltRec *filt, float *leaf_box6, float *root_box6, uint32_t *status) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= s.n) return;
  const int orig = perm[pos];
  if (orig < 0 || orig >= s.n) {
    atomicOr(status, kStatusBvhCorrupt);
    return;
  }
  TraceRec r;
  float lo[3], hi[3];
  surfel_prep(s, orig, alpha_min, sig2, r, lo, hi, filt + pos);
  rec[pos] = r;
  for (int k = 0; k < 3; ++k) { leaf_box6[6 * pos + k] = lo[k]; leaf_box6[6 * pos + 3 + k] = hi[k]; }
  const int pp = leaf_parent[pos];
  if (pp >= 0) {
    if ((pp >> 1) >= n_nodes) {  // never taken for a consistent hierarchy
      atomicOr(status, kStatusBvhCorrupt);
      return;
    }
    BNode *nd = nodes + (pp >> 1);
    float *dlo = (pp & 1) ? nd->lo1 : nd->lo0, *dhi = (pp & 1) ? nd->hi1 : nd->hi0;
    for (int k = 0; k < 3; ++k) { dlo[k] = lo[k]; dhi[k] = hi[k]; }
    return;
  }
  const int inst = -pp - 2;
  if (inst < 0 || inst >= n_inst) {
    atomicOr(status, kStatusBvhCorrupt);
    return;
  }
  for (int k = 0; k < 3; ++k) { root_box6[6 * inst + k] = lo[k]; root_box6[6 * inst + 3 + k] = hi[k]; }
}

__global__ void k_refit_level(const int32_t *order, int64_t begin, int64_t end, const int32_t *node_parent,
                              BNode *nodes, int64_t n_nodes, int n_inst, float *root_box6, uint32_t *status) {
  const int64_t idx = begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= end) return;
  const int p = order[idx];
  if (p < 0 || p >= n_nodes) {
    atomicOr(status, kStatusBvhCorrupt);
    return;
  }
  const BNode nd = nodes[p];
  float lo[3], hi[3];
  for (int k = 0; k < 3; ++k) {
    lo[k] = fminf(nd.lo0[k], nd.lo1[k]);
    hi[k] = fmaxf(nd.hi0[k], nd.hi1[k]);
  }
  const int pp = node_parent[p];
  if (pp >= 0) {
    if ((pp >> 1) >= n_nodes) {
      atomicOr(status, kStatusBvhCorrupt);
      return;
    }
    BNode *q = nodes + (pp >> 1);
    float *dlo = (pp & 1) ? q->lo1 : q->lo0, *dhi = (pp & 1) ? q->hi1 : q->hi0;
    for (int k = 0; k < 3; ++k) { dlo[k] = lo[k]; dhi[k] = hi[k]; }
    return;
  }
  const int inst = -pp - 2;
  if (inst < 0 || inst >= n_inst) {
    atomicOr(status, kStatusBvhCorrupt);
    return;
  }
  for (int k = 0; k < 3; ++k) { root_box6[6 * inst + k] = lo[k]; root_box6[6 * inst + 3 + k] = hi[k]; }
}

// depth of every binary internal node (root = 0)
__global__ void k_node_depth(const int32_t *node_parent, int64_t n_nodes, int32_t *depth, uint32_t *status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_nodes) return;
  int dep = 0;
  int p = node_parent[i];
  while (p >= 0) {
    if ((p >> 1) >= n_nodes || dep > 4096) {  // never taken for a consistent hierarchy
      atomicOr(status, kStatusBvhCorrupt);
      break;
    }
    ++dep;
    p = node_parent[p >> 1];
  }
  depth[i] = dep;
}

// ---------------------------------------------------------------- wide nodes
// The binary hierarchy is cut into traversal nodes of up to kWide slots by the
// surface-area cost (after Ylitie, Karras and Laine 2017).  Bottom-up over the
// binary depths, every internal node n gets C(n, i), i = 1..kWide: the least
// cost of covering its subtree with at most i slots of the node above it, where
// a traversal node costs kCostNode times its box area plus the cost of its own
// kWide slots, and a surfel in a slot costs kCostLeaf times its box area:
//   D(n, j) = min over k of C'(left, k) + C'(right, j - k)   (n opened into j slots)
//   C(n, 1) = kCostNode A(n) + D(n, kWide)                   (n a traversal node)
//   C(n, i) = min(C(n, i - 1), D(n, i))
// with C'(leaf, k) = kCostLeaf A(leaf) for every k >= 1.  Top-down, one launch
// per traversal level, each traversal node expands its recorded choices into
// its slots; every internal slot starts a node of the next level.
constexpr int32_t kNoSlot = -1;
constexpr float kCostNode = 1.0f;  // a visit of one traversal node (all kWide slot tests)
constexpr float kCostLeaf = 0.3f;  // a surfel in a slot whose box is hit (queue entry and pre-filter)

__device__ __forceinline__ float side_area(const BNode &nd, int side) {
  return box_area(side ? nd.lo1 : nd.lo0, side ? nd.hi1 : nd.hi0);
}

__device__ __forceinline__ float node_area(const BNode &nd) {
  float lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = fminf(nd.lo0[a], nd.lo1[a]);
    hi[a] = fmaxf(nd.hi0[a], nd.hi1[a]);
  }
  return box_area(lo, hi);
}

__global__ void k_wide_roots(const int32_t *root, const int32_t *cnt, int n_inst, int32_t *level) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_inst && cnt[i] >= 2) level[root[i]] = 0;
}

// costs of the nodes of one binary depth (order[0..count)); deeper depths are
// done.  cost[n * kWide + i - 1] = C(n, i); choice[n * 16 + i - 1] is the split
// k of D(n, i) that C(n, i) takes, or 0 where it takes C(n, i - 1) (i = 1: the
// node itself); choice[n * 16 + kWide] is the split of D(n, kWide).
__global__ void k_wide_cost(const BNode *nodes, const int32_t *order, int64_t count, int64_t n_nodes, float *cost,
                            uint8_t *choice, uint32_t *status) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int32_t n = order[t];
  const BNode nd = nodes[n];
  float cc[2][kWide];
  for (int side = 0; side < 2; ++side) {
    const int32_t c = side ? nd.c1 : nd.c0;
    if (c >= n_nodes) {  // never taken for a consistent hierarchy
      atomicOr(status, kStatusBvhCorrupt);
      return;
    }
    if (c < 0) {
      const float leaf = kCostLeaf * side_area(nd, side);
      for (int i = 0; i < kWide; ++i) cc[side][i] = leaf;
    } else {
      for (int i = 0; i < kWide; ++i) cc[side][i] = cost[(int64_t)c * kWide + i];
    }
  }
  float D[kWide + 1];
  uint8_t Dk[kWide + 1];
  for (int j = 2; j <= kWide; ++j) {
    D[j] = INFINITY;
    Dk[j] = 1;
    for (int k = 1; k < j; ++k) {
      const float v = cc[0][k - 1] + cc[1][j - k - 1];
      if (v < D[j]) {
        D[j] = v;
        Dk[j] = (uint8_t)k;
      }
    }
  }
  float C = kCostNode * node_area(nd) + D[kWide];
  cost[(int64_t)n * kWide] = C;
  choice[(int64_t)n * 16] = 0;
  for (int i = 2; i <= kWide; ++i) {
    uint8_t ch = 0;
    if (D[i] < C) {
      C = D[i];
      ch = Dk[i];
    }
    cost[(int64_t)n * kWide + i - 1] = C;
    choice[(int64_t)n * 16 + i - 1] = ch;
  }
  choice[(int64_t)n * 16 + kWide] = Dk[kWide];
}

// slots of the traversal nodes of level it: node b is opened into D(b, kWide)
__global__ void k_wide_level(const BNode *nodes, int64_t n_nodes, int32_t it, const uint8_t *choice, int32_t *level,
                             int32_t *slot_src, int32_t *n_levels, uint32_t *status) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_nodes || level[b] != it) return;
  // pending (binary node, slots) pairs whose subtree is opened into that many slots
  int32_t pn[kWide];
  int pj[kWide];
  int np = 1, m = 0;
  pn[0] = (int32_t)b;
  pj[0] = kWide;
  bool inner = false;
  int32_t src[kWide];
  while (np > 0) {
    --np;
    const int32_t p = pn[np];
    const int j = pj[np];
    const BNode nd = nodes[p];
    const int k = choice[(int64_t)p * 16 + (p == (int32_t)b && j == kWide ? kWide : j - 1)];
    for (int side = 0; side < 2; ++side) {
      const int32_t c = side ? nd.c1 : nd.c0;
      int i = side ? j - k : k;
      if (c >= n_nodes || k < 1 || k >= j || m >= kWide) {  // never taken for a consistent hierarchy
        atomicOr(status, kStatusBvhCorrupt);
        return;
      }
      if (c >= 0)
        while (i > 1 && choice[(int64_t)c * 16 + i - 1] == 0) --i;
      if (c < 0 || i == 1) {
        src[m++] = (int32_t)(p << 1 | side);
        if (c >= 0) {
          level[c] = it + 1;
          inner = true;
        }
      } else {
        if (np >= kWide) {
          atomicOr(status, kStatusBvhCorrupt);
          return;
        }
        pn[np] = c;
        pj[np] = i;
        ++np;
      }
    }
  }
  for (int q = 0; q < kWide; ++q) slot_src[b * kWide + q] = q < m ? src[q] : kNoSlot;
  atomicMax(n_levels, inner ? it + 2 : it + 1);
}

// per binary node: wide nodes (sub_w) and leaves (sub_l) in its subtree, from
// the leaves up; the second arriving child combines (release/acquire on the
// arrival count)
__global__ void k_wide_count(const int32_t *leaf_parent, const int32_t *node_parent, const int32_t *level, int64_t n,
                             int64_t n_nodes, int32_t *flags, int2 *side_cnt, int32_t *sub_w, int32_t *sub_l,
                             uint32_t *status) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= n) return;
  int w = 0, l = 1;
  int pp = leaf_parent[pos];
  int steps = 0;
  while (pp >= 0) {
    const int p = pp >> 1, side = pp & 1;
    if (p >= n_nodes || ++steps > 4096) {
      atomicOr(status, kStatusBvhCorrupt);
      return;
    }
    side_cnt[2 * p + side] = make_int2(w, l);
    const int old = __hip_atomic_fetch_add(flags + p, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (old == 0) return;
    const int2 o = side_cnt[2 * p + (side ^ 1)];
    w += o.x + (level[p] >= 0 ? 1 : 0);
    l += o.y;
    sub_w[p] = w;
    sub_l[p] = l;
    pp = node_parent[p];
  }
}

// roots[3i..3i+2] = (wide index, first descendant index, first leaf position) of instance i's root
__global__ void k_wide_root_pos(const int32_t *root, const int32_t *cnt, const int32_t *roots, int n_inst,
                                int32_t *widx, int32_t *dbase, int32_t *lbase) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inst || cnt[i] < 2) return;
  widx[root[i]] = roots[3 * i];
  dbase[root[i]] = roots[3 * i + 1];
  lbase[root[i]] = roots[3 * i + 2];
}

// Places the nodes of level `it` depth-first with contiguous children: a
// node's internal children occupy [dbase, dbase + #internal), followed by
// each child's own descendants in slot order; its leaf slots occupy
// [lbase, lbase + #leaves), followed by each internal child's leaves.
// Writes the node's build description and the new position of its leaves.
__global__ void k_wide_assign(const BNode *nodes, int64_t n_nodes, int64_t n, int32_t it, const int32_t *level,
                              const int32_t *slot_src, const int32_t *sub_w, const int32_t *sub_l, int32_t *widx,
                              int32_t *dbase, int32_t *lbase, int32_t *newpos, WideInfo *info, int64_t n_wide,
                              uint32_t *status) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_nodes || level[b] != it) return;
  const int32_t me = widx[b], db = dbase[b], lb = lbase[b];
  if (me < 0 || me >= n_wide) {
    atomicOr(status, kStatusBvhCorrupt);
    return;
  }
  // The occupied slots, internal children first (a stable partition of the
  // collapse's slot order): internal slot j then holds node child_base + j
  // and leaf slot j leaf leaf_base + j - #internal, and the traversal stack
  // can name a node's unvisited internal children by a mask of slots.
  WideInfo wi;
  int32_t code[kWide], srcs[kWide];
  int m = 0, n_int = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int q = 0; q < kWide; ++q) {
      const int32_t sr = slot_src[b * kWide + q];
      if (sr == kNoSlot) continue;
      if ((sr >> 1) >= n_nodes || sr < 0) {
        atomicOr(status, kStatusBvhCorrupt);
        return;
      }
      const BNode &nd = nodes[sr >> 1];
      const int32_t c = (sr & 1) ? nd.c1 : nd.c0;
      if ((c >= 0) != (pass == 0)) continue;
      srcs[m] = sr;
      code[m] = c;
      ++m;
      n_int += c >= 0;
    }
  }
  // Internal children in order of their box centres along the axis on which
  // those centres spread most (insertion sort, stable); the traversal visits
  // a node's remaining children in this order or its reverse, whichever runs
  // along the ray, so nearer subtrees tend to come first.
  int axis = 0;
  if (n_int > 1) {
    float cen[kWide][3], cmin[3] = {INFINITY, INFINITY, INFINITY}, cmax[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int q = 0; q < n_int; ++q) {
      const BNode &nd = nodes[srcs[q] >> 1];
      const float *bl = (srcs[q] & 1) ? nd.lo1 : nd.lo0, *bh = (srcs[q] & 1) ? nd.hi1 : nd.hi0;
      for (int k = 0; k < 3; ++k) {
        const float c = 0.5f * bl[k] + 0.5f * bh[k];
        cen[q][k] = c == c ? c : 0.0f;
        cmin[k] = fminf(cmin[k], cen[q][k]);
        cmax[k] = fmaxf(cmax[k], cen[q][k]);
      }
    }
    float best = -1.0f;
    for (int k = 0; k < 3; ++k)
      if (cmax[k] - cmin[k] > best) {
        best = cmax[k] - cmin[k];
        axis = k;
      }
    for (int q = 1; q < n_int; ++q) {
      const int32_t sq = srcs[q], cq = code[q];
      const float key = cen[q][axis];
      float c3[3] = {cen[q][0], cen[q][1], cen[q][2]};
      int j = q;
      for (; j > 0 && cen[j - 1][axis] > key; --j) {
        srcs[j] = srcs[j - 1];
        code[j] = code[j - 1];
        for (int k = 0; k < 3; ++k) cen[j][k] = cen[j - 1][k];
      }
      srcs[j] = sq;
      code[j] = cq;
      for (int k = 0; k < 3; ++k) cen[j][k] = c3[k];
    }
  }
  for (int q = 0; q < kWide; ++q) wi.src[q] = q < m ? srcs[q] : kNoSlot;
  wi.imask = ((1u << n_int) - 1u) | ((uint32_t)axis << 8);
  int32_t dnext = db + n_int, lnext = lb + (m - n_int);
  int ki = 0, kl = 0;
  for (int q = 0; q < m; ++q) {
    const int32_t x = code[q];
    if (x >= 0) {
      if (x >= n_nodes) {
        atomicOr(status, kStatusBvhCorrupt);
        return;
      }
      widx[x] = db + ki++;
      dbase[x] = dnext;
      lbase[x] = lnext;
      dnext += sub_w[x] - 1;
      lnext += sub_l[x];
    } else {
      if (~x >= n) {
        atomicOr(status, kStatusBvhCorrupt);
        return;
      }
      newpos[~x] = lb + kl++;
    }
  }
  wi.child_base = db;
  wi.leaf_base = lb;
  wi.n_slots = (uint32_t)m;
  info[me] = wi;
}

// moves every leaf to its new position: the leaf order (perm), the leaf
// parents and the binary nodes' leaf codes
__global__ void k_leaf_reorder(const int32_t *newpos, const int32_t *perm, const int32_t *leaf_parent, int64_t n,
                               int64_t n_nodes, int32_t *perm2, int32_t *leaf_parent2, BNode *nodes,
                               uint32_t *status) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= n) return;
  const int32_t np = newpos[pos];
  if (np < 0 || np >= n) {
    atomicOr(status, kStatusBvhCorrupt);
    return;
  }
  perm2[np] = perm[pos];
  const int32_t pp = leaf_parent[pos];
  leaf_parent2[np] = pp;
  if (pp >= 0) {
    if ((pp >> 1) >= n_nodes) {
      atomicOr(status, kStatusBvhCorrupt);
      return;
    }
    if (pp & 1) nodes[pp >> 1].c1 = ~np;
    else nodes[pp >> 1].c0 = ~np;
  }
}

__global__ void k_iota(int32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

__device__ __forceinline__ float pow2f(int e) { return __uint_as_float((uint32_t)(e + 127) << 23); }

// Quantised traversal nodes from the refitted binary boxes.  Per axis the
// frame origin is the lower bound of the occupied non-empty slots and the
// step 2^e the smallest power of two with fmaf(255, 2^e, p) at or above their
// upper bound; lower codes round down and upper codes up, both checked with
// the same fused multiply-add the traversal evaluates.  A NaN bound decodes
// to the whole frame.
__global__ void k_wide_quantize(const BNode *nodes, const WideInfo *info, int64_t n_wide, int64_t n_nodes,
                                QNode *out, uint32_t *status) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_wide) return;
  const WideInfo wi = info[j];
  float lo[kWide][3], hi[kWide][3];
  float ulo[3] = {INFINITY, INFINITY, INFINITY}, uhi[3] = {-INFINITY, -INFINITY, -INFINITY};
  uint32_t vmask = 0;
  for (int q = 0; q < kWide; ++q) {
    for (int k = 0; k < 3; ++k) {
      lo[q][k] = INFINITY;
      hi[q][k] = -INFINITY;
    }
    if (q >= (int)wi.n_slots) continue;
    const int32_t sr = wi.src[q];
    if (sr < 0 || (sr >> 1) >= n_nodes) {
      atomicOr(status, kStatusBvhCorrupt);
      return;
    }
    const BNode &nd = nodes[sr >> 1];
    const float *bl = (sr & 1) ? nd.lo1 : nd.lo0, *bh = (sr & 1) ? nd.hi1 : nd.hi0;
    bool empty = false;
    for (int k = 0; k < 3; ++k) {
      lo[q][k] = bl[k];
      hi[q][k] = bh[k];
      empty |= bl[k] > bh[k];
    }
    if (empty) continue;
    vmask |= 1u << q;
    for (int k = 0; k < 3; ++k) {
      ulo[k] = fminf(ulo[k], bl[k]);
      uhi[k] = fmaxf(uhi[k], bh[k]);
    }
  }
  QNode nd;
  for (int k = 0; k < 3; ++k) {
    float p = 0.0f;
    int e = -126;
    if (vmask) {
      p = fminf(fmaxf(ulo[k], -FLT_MAX), FLT_MAX);  // NaN -> -FLT_MAX
      const float ext = uhi[k] - p;
      if (ext > 0.0f && ext <= FLT_MAX) e = max(-126, ilogbf(ext) - 8);
      else if (!(ext <= 0.0f)) e = 127;  // infinite or NaN extent
      while (e < 127 && !(__builtin_fmaf(255.0f, pow2f(e), p) >= uhi[k])) ++e;
    }
    const float st = pow2f(e);
    nd.p[k] = p;
    nd.e[k] = (int8_t)e;
    const float top = __builtin_fmaf(255.0f, st, p);
    for (int q = 0; q < kWide; ++q) {
      int ql = 255, qh = 0;
      if ((vmask >> q) & 1u) {
        const float l = lo[q][k], h = hi[q][k];
        if (!(l >= p)) {
          ql = 0;
        } else {
          ql = (int)fmin(floor(((double)l - (double)p) / (double)st), 255.0);
          while (ql > 0 && __builtin_fmaf((float)ql, st, p) > l) --ql;
        }
        if (!(h <= top)) {
          qh = 255;
        } else {
          qh = (int)fmax(fmin(ceil(((double)h - (double)p) / (double)st), 255.0), 0.0);
          while (qh < 255 && __builtin_fmaf((float)qh, st, p) < h) ++qh;
        }
      }
      nd.q[k][q] = (uint8_t)ql;
      nd.q[3 + k][q] = (uint8_t)qh;
    }
  }
  nd.imask = (uint8_t)wi.imask;
  nd.child_base = wi.child_base;
  nd.leaf_base = wi.leaf_base;
  nd.vmask = vmask | (((wi.imask >> 8) & 3u) << 8);
  out[j] = nd;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f32(float *p, float v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_boxes_by_index(const SurfelArrays &s, double alpha_min, double sig2, float *box6, hipStream_t st) {
  if (s.n <= 0) return;
  hipLaunchKernelGGL(k_boxes_by_index, dim3(blocks(s.n, 256)), dim3(256), 0, st, s, alpha_min, sig2, box6);
}

void launch_instance_bounds(const float *box6, const int32_t *inst_first, const int32_t *inst_n, int n_inst,
                            float *out, hipStream_t st) {
  hipLaunchKernelGGL(k_instance_bounds, dim3(n_inst), dim3(256), 0, st, box6, inst_first, inst_n, out);
}

void launch_morton(const float *box6, const float *inst_bounds, const int32_t *inst_first, const int32_t *inst_n,
                   int n_inst, int64_t n, uint64_t *keys, int32_t *vals, hipStream_t st) {
  if (n <= 0) return;
  // one coarse spatial level above the size classes: 21% fewer node visits per ray than plain
  // Morton order on the 1M-surfel scene; with the surface-area-cost collapse and a 128 window, level 0
  // traces 15% slower and level 2 alike; the clustering of plain Morton order builds much deeper trees
  constexpr int kSizeLevel = 1;
  hipLaunchKernelGGL(k_morton, dim3(blocks(n, 256)), dim3(256), 0, st, box6, inst_bounds, inst_first, inst_n, n_inst,
                     n, kSizeLevel, keys, vals);
}

size_t radix_sort_hist_words(int64_t n) {
  const size_t h = (size_t)256 * blocks(n > 0 ? n : 1, RS_TILE);
  return h + h / SC_TILE + 1;  // digit counts, then the scan's tile sums
}

void radix_sort(uint64_t *keys, int32_t *vals, uint64_t *keys_tmp, int32_t *vals_tmp, uint32_t *hist, int64_t n,
                hipStream_t st, int key_bits) {
  if (n <= 1) return;
  int nb = (int)blocks(n, RS_TILE);
  uint64_t *ka = keys, *kb = keys_tmp;
  int32_t *va = vals, *vb = vals_tmp;
  const int passes = (key_bits + 15) / 16 * 2;  // even, so the result lands back in (keys, vals)
  for (int pass = 0; pass < passes; ++pass) {
    int shift = 8 * pass;
    hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(RS_THREADS), 0, st, ka, n, shift, hist, nb);
    exclusive_scan(hist, (int64_t)256 * nb, hist + (int64_t)256 * nb, st);
    hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(RS_THREADS), 0, st, ka, va, kb, vb, n, shift, hist, nb);
    uint64_t *tk = ka; ka = kb; kb = tk;
    int32_t *tv = va; va = vb; vb = tv;
  }
  // an even number of passes: the result is back in (keys, vals)
}

bool launch_ploc(const int32_t *perm, const float *boxidx, int32_t first, int32_t n, int32_t node_off, int32_t inst,
                 BNode *nodes, int32_t *node_parent, int32_t *leaf_parent, int32_t *cid, int32_t *cid2, float *cbox,
                 float *cbox2, int32_t *nn, uint32_t *rem, uint32_t *pre, hipStream_t st) {
  if (n == 1) {
    hipLaunchKernelGGL(k_leaf_root, dim3(1), dim3(1), 0, st, first, inst, leaf_parent);
    return true;
  }
  hipLaunchKernelGGL(k_ploc_init, dim3(blocks(n, 256)), dim3(256), 0, st, perm, boxidx, first, n, cid, cbox);
  int m = n;
  int32_t next_idx = node_off + n - 2;
  for (int it = 0; m > 1; ++it) {
    if (it > 4 * n) return false;  // no progress: never for a consistent clustering
    hipLaunchKernelGGL(k_ploc_nn, dim3(blocks(m, kPlocB)), dim3(kPlocB), 0, st, cbox, m, kPlocR, nn);
    hipLaunchKernelGGL(k_ploc_flags, dim3(blocks(m, 256)), dim3(256), 0, st, nn, m, rem, pre);
    hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(1024), 0, st, pre, (int64_t)m);
    hipLaunchKernelGGL(k_ploc_merge, dim3(blocks(m, 256)), dim3(256), 0, st, nn, pre, m, next_idx, cid, cbox, cid2,
                       cbox2, nodes, node_parent, leaf_parent);
    uint32_t last_pre = 0, last_rem = 0;
    if (hipMemcpyAsync(&last_pre, pre + m - 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&last_rem, rem + m - 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return false;
    const int merged = (int)(last_pre + last_rem);
    if (merged <= 0) return false;
    next_idx -= merged;
    m -= merged;
    int32_t *t = cid; cid = cid2; cid2 = t;
    float *tb = cbox; cbox = cbox2; cbox2 = tb;
  }
  if (next_idx != node_off - 1) return false;
  hipLaunchKernelGGL(k_ploc_root, dim3(1), dim3(1), 0, st, cid, inst, node_parent);
  return true;
}


void launch_depth(const int32_t *leaf_parent, const int32_t *node_parent, int64_t n, int64_t n_nodes,
                  int32_t *max_depth, uint32_t *status, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_depth, dim3(blocks(n, 256)), dim3(256), 0, st, leaf_parent, node_parent, n, n_nodes,
                     max_depth, status);
}

void launch_node_depth(const int32_t *node_parent, int64_t n_nodes, int32_t *depth, uint32_t *status,
                       hipStream_t st) {
  if (n_nodes <= 0) return;
  hipLaunchKernelGGL(k_node_depth, dim3(blocks(n_nodes, 256)), dim3(256), 0, st, node_parent, n_nodes, depth, status);
}

void launch_refit(const SurfelArrays &s, double alpha_min, double sig2, const int32_t *perm,
                  const int32_t *leaf_parent, const int32_t *node_parent, const int32_t *order,
                  const std::vector<int64_t> &level_off, int64_t n_nodes, int n_inst, BNode *nodes, TraceRec *rec,
                  FiltRec *filt, float *leaf_box6, float *root_box6, uint32_t *status, hipStream_t st) {
  if (s.n <= 0) return;
  hipLaunchKernelGGL(k_refit_leaves, dim3(blocks(s.n, 256)), dim3(256), 0, st, s, alpha_min, sig2, perm, leaf_parent,
                     nodes, n_nodes, n_inst, rec, filt, leaf_box6, root_box6, status);
  // level_off[d] .. level_off[d + 1]: the nodes of depth d in order; deepest first
  for (int64_t d = (int64_t)level_off.size() - 2; d >= 0; --d) {
    const int64_t b = level_off[d], e = level_off[d + 1];
    if (e > b)
      hipLaunchKernelGGL(k_refit_level, dim3(blocks(e - b, 256)), dim3(256), 0, st, order, b, e, node_parent, nodes,
                         n_nodes, n_inst, root_box6, status);
  }
}

void launch_wide_roots(const int32_t *root, const int32_t *cnt, int n_inst, int32_t *level, hipStream_t st) {
  hipLaunchKernelGGL(k_wide_roots, dim3(1), dim3(64), 0, st, root, cnt, n_inst, level);
}

void launch_wide_cost(const BNode *nodes, int64_t n_nodes, const int32_t *order, const std::vector<int64_t> &level_off,
                      float *cost, uint8_t *choice, uint32_t *status, hipStream_t st) {
  for (int64_t d = (int64_t)level_off.size() - 2; d >= 0; --d) {
    const int64_t cnt = level_off[d + 1] - level_off[d];
    if (cnt > 0)
      hipLaunchKernelGGL(k_wide_cost, dim3(blocks(cnt, 256)), dim3(256), 0, st, nodes, order + level_off[d], cnt,
                         n_nodes, cost, choice, status);
  }
}

void launch_wide_level(const BNode *nodes, int64_t n_nodes, int32_t it, const uint8_t *choice, int32_t *level,
                       int32_t *slot_src, int32_t *n_levels, uint32_t *status, hipStream_t st) {
  if (n_nodes <= 0) return;
  hipLaunchKernelGGL(k_wide_level, dim3(blocks(n_nodes, 256)), dim3(256), 0, st, nodes, n_nodes, it, choice, level,
                     slot_src, n_levels, status);
}

void launch_wide_count(const int32_t *leaf_parent, const int32_t *node_parent, const int32_t *level, int64_t n,
                       int64_t n_nodes, int32_t *flags, int2 *side_cnt, int32_t *sub_w, int32_t *sub_l,
                       uint32_t *status, hipStream_t st) {
  if (n <= 0 || n_nodes <= 0) return;
  launch_fill_u32((uint32_t *)flags, 0u, n_nodes, st);
  hipLaunchKernelGGL(k_wide_count, dim3(blocks(n, 256)), dim3(256), 0, st, leaf_parent, node_parent, level, n,
                     n_nodes, flags, side_cnt, sub_w, sub_l, status);
}

void launch_wide_root_pos(const int32_t *root, const int32_t *cnt, const int32_t *roots, int n_inst, int32_t *widx,
                          int32_t *dbase, int32_t *lbase, hipStream_t st) {
  hipLaunchKernelGGL(k_wide_root_pos, dim3(1), dim3(64), 0, st, root, cnt, roots, n_inst, widx, dbase, lbase);
}

void launch_wide_assign(const BNode *nodes, int64_t n_nodes, int64_t n, int32_t it, const int32_t *level,
                        const int32_t *slot_src, const int32_t *sub_w, const int32_t *sub_l, int32_t *widx,
                        int32_t *dbase, int32_t *lbase, int32_t *newpos, WideInfo *info, int64_t n_wide,
                        uint32_t *status, hipStream_t st) {
  if (n_nodes <= 0) return;
  hipLaunchKernelGGL(k_wide_assign, dim3(blocks(n_nodes, 256)), dim3(256), 0, st, nodes, n_nodes, n, it, level,
                     slot_src, sub_w, sub_l, widx, dbase, lbase, newpos, info, n_wide, status);
}

void launch_iota(int32_t *p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_iota, dim3(blocks(n, 256)), dim3(256), 0, st, p, n);
}

void launch_leaf_reorder(const int32_t *newpos, const int32_t *perm, const int32_t *leaf_parent, int64_t n,
                         int64_t n_nodes, int32_t *perm2, int32_t *leaf_parent2, BNode *nodes, uint32_t *status,
                         hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_leaf_reorder, dim3(blocks(n, 256)), dim3(256), 0, st, newpos, perm, leaf_parent, n, n_nodes,
                     perm2, leaf_parent2, nodes, status);
}

void launch_wide_quantize(const BNode *nodes, const WideInfo *info, int64_t n_wide, int64_t n_nodes, QNode *out,
                          uint32_t *status, hipStream_t st) {
  if (n_wide <= 0) return;
  hipLaunchKernelGGL(k_wide_quantize, dim3(blocks(n_wide, 256)), dim3(256), 0, st, nodes, info, n_wide, n_nodes, out,
                     status);
}

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks(n, 256)), dim3(256), 0, st, p, v, n);
}
void launch_fill_f32(float *p, float v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f32, dim3(blocks(n, 256)), dim3(256), 0, st, p, v, n);
}

}  // namespace lf

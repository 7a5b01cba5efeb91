// lf_render.hip -- forward path of the gfx950 tracer (wavefront form):
//   instances  : per-state rigid transforms -> instance records (Eq. state-assembly)
//   env tables : piecewise-constant importance-sampling tables of E_k
//   primary    : ray generation, traversal + k-closest buffer, compositing into
//                the surface record (Eq. surface-record), outputs, sampling of
//                S directions and ballot-compacted enqueue of live secondaries
//   secondary  : trace of the compacted queue, secondary record, two
//                unshadowed env samples, per-sample contribution
//   resolve    : pixel radiance = T E(d) + sum_s contributions (fixed order)
#include "lf_device.h"
#include "lf_kernels.h"

namespace lf {

namespace {

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ void k_instances(const float *R, const float *t, const float *root_box6, const int32_t *first,
                            const int32_t *cnt, const int32_t *root, int n_inst, InstRec *out, double *bounds6,
                            uint32_t *status) {
  const int ii = threadIdx.x;  // one block of kMaxInst threads
  __shared__ double sb[kMaxInst][6];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (ii < n_inst) {
    InstRec I;
    I.first = first[ii];
    I.n = cnt[ii];
    I.root = root[ii];
    I.identity = ii == 0;
    const float *rb = root_box6 + 6 * ii;
    const double blo[3] = {rb[0], rb[1], rb[2]}, bhi[3] = {rb[3], rb[4], rb[5]};
    if (ii == 0) {
      for (int k = 0; k < 9; ++k) I.R[k] = (k % 4 == 0) ? 1.0 : 0.0;
      for (int k = 0; k < 3; ++k) I.t[k] = 0.0;
    } else {
      const float *A = R + 9 * (ii - 1);
      // Gram-Schmidt of the first two columns, third = cross product
      d3 c0 = mk(A[0], A[3], A[6]), c1 = mk(A[1], A[4], A[7]);
      const double l0 = sqrt(dot(c0, c0));
      bool bad = !(l0 > 1e-6);
      c0 = (1.0 / l0) * c0;
      c1 = c1 - dot(c0, c1) * c0;
      const double l1 = sqrt(dot(c1, c1));
      bad = bad || !(l1 > 1e-6);
      c1 = (1.0 / l1) * c1;
      const d3 c2 = cross(c0, c1);
      const float *tt = t + 3 * (ii - 1);
      bad = bad || !isfinite(tt[0]) || !isfinite(tt[1]) || !isfinite(tt[2]);
      if (bad) {
        atomicOr(status, kStatusBadTransform);
        I.n = 0;
      }
      I.R[0] = c0.x; I.R[1] = c1.x; I.R[2] = c2.x;
      I.R[3] = c0.y; I.R[4] = c1.y; I.R[5] = c2.y;
      I.R[6] = c0.z; I.R[7] = c1.z; I.R[8] = c2.z;
      for (int k = 0; k < 3; ++k) I.t[k] = tt[k];
    }
    // world bounds: transformed corners of the object-space root box, padded
    if (I.n > 0 && blo[0] <= bhi[0]) {
      for (int c = 0; c < 8; ++c) {
        const d3 p = mk((c & 1) ? bhi[0] : blo[0], (c & 2) ? bhi[1] : blo[1], (c & 4) ? bhi[2] : blo[2]);
        const d3 w = mul(I.R, p) + mk(I.t[0], I.t[1], I.t[2]);
        const double ww[3] = {w.x, w.y, w.z};
        for (int k = 0; k < 3; ++k) { lo[k] = fmin(lo[k], ww[k]); hi[k] = fmax(hi[k], ww[k]); }
      }
      for (int k = 0; k < 3; ++k) {
        const double pad = 1e-9 * (fabs(lo[k]) + fabs(hi[k])) + 1e-30;
        lo[k] -= pad;
        hi[k] += pad;
      }
    } else {
      I.n = 0;
    }
    for (int k = 0; k < 3; ++k) { I.lo[k] = lo[k]; I.hi[k] = hi[k]; }
    I.omag = 0.0f;
    I.oext = 0.0f;
    for (int k = 0; k < 3; ++k) {
      I.omag = fmaxf(I.omag, fmaxf(fabsf(rb[k]), fabsf(rb[3 + k])));
      I.oext = fmaxf(I.oext, rb[3 + k] - rb[k]);
    }
    I.pad[0] = I.pad[1] = 0;
    out[ii] = I;
    for (int k = 0; k < 3; ++k) { sb[ii][k] = lo[k]; sb[ii][3 + k] = hi[k]; }
  }
  __syncthreads();
  // union of the instance bounds
  if (ii == 0) {
    double u[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int j = 0; j < n_inst; ++j)
      for (int k = 0; k < 3; ++k) { u[k] = fmin(u[k], sb[j][k]); u[3 + k] = fmax(u[3 + k], sb[j][3 + k]); }
    for (int k = 0; k < 6; ++k) bounds6[k] = u[k];
  }
}

__device__ __forceinline__ uint32_t spread3_10(uint32_t x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

__global__ void k_secondary_keys(const SecEntry *queue, const uint32_t *count, int64_t cap, const double *bounds6,
                                 const ChunkDesc *chunks, const BatchSlot *slots, uint64_t *keys, int32_t *vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap) return;
  vals[i] = (int32_t)i;
  if (i >= (int64_t)*count) {
    keys[i] = 0xffffffffull;
    return;
  }
  const SecEntry e = queue[i];
  // in a batch every request quantises in its own world bounds (only the grouping depends on it)
  const double *b = chunks ? slots[chunks[e.ray / kChunk].slot].bounds : bounds6;
  uint32_t c[3];
  for (int k = 0; k < 3; ++k) {
    const double ext = b[3 + k] - b[k];
    double x = ext > 0.0 ? (e.o[k] - b[k]) / ext : 0.5;
    x = fmin(fmax(x, 0.0), 1.0);
    c[k] = (uint32_t)fmin(x * 512.0, 511.0);  // 9 bits per axis
  }
  // direction first (octant, then 3+3 bits of the octahedral map), then the
  // origin (7 bits per axis): measured 9% faster secondary traversal at 1M
  // surfels than octant + 9-bit origin, and 24% faster than origin first
  const uint32_t oct = (e.w[0] < 0.0 ? 1u : 0u) | (e.w[1] < 0.0 ? 2u : 0u) | (e.w[2] < 0.0 ? 4u : 0u);
  const double an = fabs(e.w[0]) + fabs(e.w[1]) + fabs(e.w[2]);
  double px = e.w[0] / an, py = e.w[1] / an;
  if (e.w[2] < 0.0) {
    const double qx = (1.0 - fabs(py)) * (px >= 0.0 ? 1.0 : -1.0), qy = (1.0 - fabs(px)) * (py >= 0.0 ? 1.0 : -1.0);
    px = qx;
    py = qy;
  }
  const uint32_t ux = (uint32_t)fmin(fmax(0.5 * (px + 1.0), 0.0) * 8.0, 7.0);
  const uint32_t uy = (uint32_t)fmin(fmax(0.5 * (py + 1.0), 0.0) * 8.0, 7.0);
  const uint32_t m = (spread3_10(c[0] >> 2) << 2) | (spread3_10(c[1] >> 2) << 1) | spread3_10(c[2] >> 2);
  keys[i] = ((uint64_t)oct << 27) | ((uint64_t)ux << 24) | ((uint64_t)uy << 21) | m;
}

// one block per env row: clamped luminance, row sum, conditional CDF (double)
__global__ __launch_bounds__(256) void k_env_rows(const float *tex, int H, int W, double *cdf_col, double *lum,
                                                  double *rowsum, double *roww) {
  int r = blockIdx.x;
  __shared__ double part[256];
  __shared__ double carry;
  if (threadIdx.x == 0) carry = 0.0;
  __syncthreads();
  // pass 1: row sum
  double s = 0.0;
  for (int c = threadIdx.x; c < W; c += 256) {
    const float *p = tex + 3 * ((int64_t)r * W + c);
    double l = 0.2126 * p[0] + 0.7152 * p[1] + 0.0722 * p[2];
    if (!(l > 0.0)) l = 0.0;
    lum[(int64_t)r * W + c] = l;
    s += l;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  double rs = part[0];
  __syncthreads();
  double *cc = cdf_col + (int64_t)r * (W + 1);
  // pass 2: inclusive scan in chunks of 256
  for (int c0 = 0; c0 < W; c0 += 256) {
    int c = c0 + threadIdx.x;
    double v = (c < W) ? lum[(int64_t)r * W + c] : 0.0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      double x = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0.0;
      __syncthreads();
      part[threadIdx.x] += x;
      __syncthreads();
    }
    if (c < W) cc[c + 1] = rs > 0.0 ? (carry + part[threadIdx.x]) / rs : (double)(c + 1) / W;
    __syncthreads();
    if (threadIdx.x == 0) carry += part[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cc[0] = 0.0;
    cc[W] = 1.0;
    rowsum[r] = rs;
    roww[r] = rs * sin((r + 0.5) * kPi / H);
  }
}

// one block: marginal CDF over rows, total weight, c_env
__global__ __launch_bounds__(256) void k_env_marginal(int H, uint32_t flags, const double *roww, double *cdf_row,
                                                      double *scal) {
  __shared__ double part[256];
  __shared__ double carry;
  __shared__ double total;
  double s = 0.0;
  for (int r = threadIdx.x; r < H; r += 256) s += roww[r];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) { total = part[0]; carry = 0.0; }
  __syncthreads();
  double tot = total;
  for (int r0 = 0; r0 < H; r0 += 256) {
    int r = r0 + threadIdx.x;
    part[threadIdx.x] = r < H ? roww[r] : 0.0;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      double x = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0.0;
      __syncthreads();
      part[threadIdx.x] += x;
      __syncthreads();
    }
    if (r < H) cdf_row[r + 1] = tot > 0.0 ? (carry + part[threadIdx.x]) / tot : (double)(r + 1) / H;
    __syncthreads();
    if (threadIdx.x == 0) carry += part[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cdf_row[0] = 0.0;
    cdf_row[H] = 1.0;
    scal[0] = tot;
    scal[1] = (tot > 0.0 && !(flags & LF_FLAG_BSDF_ONLY)) ? 0.5 : 0.0;
  }
}

// ---------------------------------------------------------------- request views
// Where the per-request quantities of a ray live: the launch arguments for a
// single request, the slot of the ray's chunk in a batch.
struct ReqView {
  const InstRec *inst;
  float *radiance, *depth, *normal, *alpha;
  int64_t local;   // ray id within the request (sampler counter, output index)
  bool valid;
};

template <bool B>
__device__ __forceinline__ ReqView req_view(const RenderArgs &a, int64_t ray) {
  ReqView v;
  if constexpr (B) {
    const bool in = ray < a.R;  // a block may extend past the last chunk
    const ChunkDesc cd = a.chunks[in ? ray / kChunk : 0];
    const BatchSlot &sl = a.slots[cd.slot];
    v.inst = sl.inst;
    v.radiance = sl.radiance; v.depth = sl.depth; v.normal = sl.normal; v.alpha = sl.alpha;
    const int w = sl.cam->w[0], h = sl.cam->h[0];
    const int nx = (w + 15) / 16;
    const int lane = (int)(ray % kChunk);
    const int x = (int)(cd.tile % nx) * 16 + (lane >> 6) * 8 + (lane & 7);
    const int y = (int)(cd.tile / nx) * 8 + ((lane & 63) >> 3);
    v.local = (int64_t)y * w + x;
    v.valid = in && x < w && y < h;
  } else {
    v.inst = a.S.inst;
    v.radiance = a.radiance; v.depth = a.depth; v.normal = a.normal; v.alpha = a.alpha;
    v.local = ray;
    v.valid = ray < a.R;
  }
  return v;
}

// environment, sampler seed and S of the ray's request
template <bool B>
__device__ __forceinline__ void req_shading(const RenderArgs &a, int64_t ray, EnvView &E, TraceParams &P) {
  P = a.P;
  if constexpr (B) {
    const BatchSlot &sl = a.slots[a.chunks[ray < a.R ? ray / kChunk : 0].slot];
    E = sl.E;
    P.seed = sl.seed;
    P.spp = sl.spp;
  } else {
    E = a.E;
  }
}

template <bool B>
__device__ __forceinline__ void req_ray(const RenderArgs &a, int64_t ray, const ReqView &v, float *of, float *df) {
  if constexpr (B) raygen_f32(*a.slots[a.chunks[ray / kChunk].slot].cam, 0, v.local, of, df);
  else load_ray(a.rays, ray, of, df);
}

// ---------------------------------------------------------------- primary tracing
template <int K, class B_>
__device__ __forceinline__ void finish_primary(const RenderArgs &a, const SceneView &S, const ReqView &v, bool replay,
                                               int64_t ray, B_ &kb, d3 o, d3 d) {
  Record rc;
  composite<K>(S, a.P, kb, o, d, rc);
  store_record(rc, a.rec1 + ray);
  if (replay) return;
  const int64_t i = v.local;
  v.depth[i] = (float)rc.depth;
  v.alpha[i] = (float)rc.A;
  v.normal[3 * i + 0] = (float)rc.n.x;
  v.normal[3 * i + 1] = (float)rc.n.y;
  v.normal[3 * i + 2] = (float)rc.n.z;
  if (a.hit_idx) write_hits<K>(S, kb, a.P.k, a.hit_idx + ray * a.P.k);
}

// primary rays as a pool of work items: tiles of the cameras, batch chunks, or explicit rays
template <bool B>
__device__ __forceinline__ int64_t primary_items(const RenderArgs &a) {
  return (!B && a.n_tiles) ? a.n_tiles * kBlock : a.R;
}
template <bool B>
__device__ __forceinline__ int64_t primary_ray(const RenderArgs &a, int64_t item) {
  if constexpr (!B)
    if (a.n_tiles) return tile_ray(*a.rays.cams, item);
  return item;
}

template <int K, bool B>
struct PrimaryWork {
  static constexpr int kRefill = 24;  // camera rays of a wave stay alike; refill in larger groups
  static constexpr bool kPrefetch = false;
  const RenderArgs &a;
  __device__ bool begin(int64_t item, d3 &o, d3 &d, const InstRec *&inst) const {
    const int64_t ray = primary_ray<B>(a, item);
    if (ray < 0) return false;
    const ReqView v = req_view<B>(a, ray);
    if (!v.valid) return false;
    float of[3], df[3];
    req_ray<B>(a, ray, v, of, df);
    o = mk(of[0], of[1], of[2]);
    d = mk(df[0], df[1], df[2]);
    inst = v.inst;
    return true;
  }
  __device__ void store(int64_t item, const KBufF<K> &kb) const { store_kbuf<K>(kb, a.kbuf1 + item * 2 * K); }
  // the k-th distance this item's ray had in the earlier call, or +inf
  __device__ float hint(int64_t item) const {
    if (B || !a.use_hint) return INFINITY;
    return __uint_as_float(a.kbuf1[item * 2 * K + K - 1]);
  }
};

template <int K, bool B>
__global__ __launch_bounds__(kBlock, 2) void k_trace1(RenderArgs a) {
  __shared__ int stk[kStackL * kBlock];
  __shared__ int lq[kLeafQ * kBlock];
  const PrimaryWork<K, B> wk{a};
  trace_pool<K>(a.S, a.P, wk, primary_items<B>(a), a.work, stk + threadIdx.x, lq + threadIdx.x, a.status, 0);
}

// the same as wave packets, for camera tiles and batch chunks (8x8 pixels per wave)
template <int K, bool B>
__global__ __launch_bounds__(kBlock, 2) void k_trace1p(RenderArgs a) {
  __shared__ int wstk[(kBlock / 64) * kStackL];
  const PrimaryWork<K, B> wk{a};
  trace_packet<K>(a.S, a.P, wk, primary_items<B>(a), a.work, wstk + (threadIdx.x / 64) * kStackL, a.status, 0);
}

// compositing of every primary ray's k-buffer, record and outputs
template <int K, bool B>
__global__ __launch_bounds__(kBlock) void k_composite1(RenderArgs a, bool replay) {
  const int64_t item = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (item >= primary_items<B>(a)) return;
  const int64_t ray = primary_ray<B>(a, item);
  if (ray < 0) return;
  const ReqView v = req_view<B>(a, ray);
  if (!v.valid) return;
  float of[3], df[3];
  req_ray<B>(a, ray, v, of, df);
  KBufF<K> kb;
  load_kbuf<K>(kb, a.kbuf1 + item * 2 * K);
  SceneView S = a.S;
  S.inst = v.inst;
  finish_primary<K>(a, S, v, replay, ray, kb, mk(of[0], of[1], of[2]), mk(df[0], df[1], df[2]));
}

// ---------------------------------------------------------------- primary shading
// Background term, the sampled directions of every slot (one-sample MIS, or
// next-event + continuation per sample in the two-ray form), ballot-compacted
// enqueue of live secondary rays.  replay = true regenerates the queue only.
template <bool B>
__global__ __launch_bounds__(256) void k_shade1(RenderArgs a, bool replay) {
  const int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const ReqView v = req_view<B>(a, ray);
  const bool active = v.valid;
  EnvView E;
  TraceParams P;
  req_shading<B>(a, ray, E, P);
  const int S = P.spp, J = n_slots(P);
  float of[3] = {0, 0, 0}, df[3] = {0, 0, 1};
  if (active) req_ray<B>(a, ray, v, of, df);
  const d3 d = mk(df[0], df[1], df[2]);
  Record rc;
  rc.nh = 0;
  if (active) rc = load_record(a.rec1 + ray);
  const double c_env = E.scal[1];
  const d3 wo = -d;
  d3 L = mk(0, 0, 0);
  if (active && !replay && !(P.flags & LF_FLAG_NO_BACKGROUND)) L = rc.T * env_eval(E, d);
  const bool trace2 = !(P.flags & LF_FLAG_NO_SECONDARY);
  for (int s = 0; s < J; ++s) {
    d3 w = mk(0, 0, 1);
    double K_ = 0.0, tw = 1.0;
    const bool live = active && primary_slot(E, P, rc, wo, v.local, s, c_env, w, K_, tw);
    d3 thr = mk(0, 0, 0);
    if (live) thr = (K_ * rc.A / S) * fcos(rc.n, w, wo, rc.a, rc.m, rc.r, P.flags);
    if (!trace2) {
      if (live && !replay) {
        const d3 Ev = tw * env_eval(E, w);
        L = L + mk(thr.x * Ev.x, thr.y * Ev.y, thr.z * Ev.z);
      }
      continue;
    }
    SecEntry e;
    if (live) {
      const d3 o2 = rc.x + P.sec_off * rc.n;
      e.o[0] = o2.x; e.o[1] = o2.y; e.o[2] = o2.z;
      e.w[0] = w.x; e.w[1] = w.y; e.w[2] = w.z;
      e.thr[0] = (float)thr.x; e.thr[1] = (float)thr.y; e.thr[2] = (float)thr.z;
      e.ray = (int32_t)ray;
      e.s = s;
      e.tw = (float)tw;
    }
    wave_append<SecEntry>(live, e, a.queue, a.queue_count);
    if (active && !live) {
      const int64_t cs = ray * a.spp_stride + s;
      if (!replay) {
        a.contrib[3 * cs + 0] = 0.f;
        a.contrib[3 * cs + 1] = 0.f;
        a.contrib[3 * cs + 2] = 0.f;
        if (a.sec_hit_idx)
          for (int j = 0; j < P.k; ++j) a.sec_hit_idx[cs * P.k + j] = -1;
      } else {
        SecFrozen f = {};
        f.T2 = 1.0f;
        a.frozen[cs] = f;
      }
    }
  }
  if (active && !replay) {
    v.radiance[3 * v.local + 0] = (float)L.x;
    v.radiance[3 * v.local + 1] = (float)L.y;
    v.radiance[3 * v.local + 2] = (float)L.z;
  }
}

// ---------------------------------------------------------------- secondary tracing
template <int K, class B_>
__device__ __forceinline__ void finish_secondary(const RenderArgs &a, const SceneView &S, uint32_t qi,
                                                 const SecEntry &e, B_ &kb, d3 o, d3 w) {
  Record r2;
  composite<K>(S, a.P, kb, o, w, r2);
  store_record(r2, a.rec2 + qi);
  if (a.sec_hit_idx) {
    const int64_t cs = (int64_t)e.ray * a.spp_stride + e.s;
    write_hits<K>(S, kb, a.P.k, a.sec_hit_idx + cs * a.P.k);
  }
}

// the (regrouped) secondary queue as a pool of work items
template <int K, bool B>
struct SecondaryWork {
  static constexpr int kRefill = 8;
  static constexpr bool kPrefetch = true;
  const RenderArgs &a;
  __device__ bool begin(int64_t item, d3 &o, d3 &w, const InstRec *&inst) const {
    const SecEntry &e = a.queue[a.order ? (uint32_t)a.order[item] : (uint32_t)item];
    o = mk(e.o[0], e.o[1], e.o[2]);
    w = mk(e.w[0], e.w[1], e.w[2]);
    if constexpr (B) inst = a.slots[a.chunks[e.ray / kChunk].slot].inst;
    else inst = a.S.inst;
    return true;
  }
  // the k-th distance is also kept per (ray, slot), which identifies the
  // secondary ray across calls (its queue position depends on the order of
  // the appends)
  __device__ void store(int64_t item, const KBufF<K> &kb) const {
    store_kbuf<K>(kb, a.kbuf2 + item * 2 * K);
    if (!B) {
      const SecEntry &e = a.queue[a.order ? (uint32_t)a.order[item] : (uint32_t)item];
      a.hint2[(int64_t)e.ray * a.spp_stride + e.s] = kb.t[K - 1];
    }
  }
  __device__ float hint(int64_t item) const {
    if (B || !a.use_hint) return INFINITY;
    const SecEntry &e = a.queue[a.order ? (uint32_t)a.order[item] : (uint32_t)item];
    return a.hint2[(int64_t)e.ray * a.spp_stride + e.s];
  }
};

template <int K, bool B>
__global__ __launch_bounds__(kBlock, 2) void k_trace2(RenderArgs a) {
  __shared__ int stk[kStackL * kBlock];
  __shared__ int lq[kLeafQ * kBlock];
  const SecondaryWork<K, B> wk{a};
  trace_pool<K>(a.S, a.P, wk, (int64_t)*a.queue_count, a.work, stk + threadIdx.x, lq + threadIdx.x, a.status, 4);
}

template <int K, bool B>
__global__ __launch_bounds__(kBlock) void k_composite2(RenderArgs a) {
  const uint32_t item = blockIdx.x * kBlock + threadIdx.x;
  if (item >= *a.queue_count) return;
  const uint32_t qi = a.order ? (uint32_t)a.order[item] : item;
  const SecEntry e = a.queue[qi];
  SceneView S = a.S;
  if constexpr (B) S.inst = a.slots[a.chunks[e.ray / kChunk].slot].inst;
  KBufF<K> kb;
  load_kbuf<K>(kb, a.kbuf2 + (int64_t)item * 2 * K);
  finish_secondary<K>(a, S, qi, e, kb, mk(e.o[0], e.o[1], e.o[2]), mk(e.w[0], e.w[1], e.w[2]));
}

// ---------------------------------------------------------------- secondary shading
template <bool B>
__global__ __launch_bounds__(256) void k_shade2(RenderArgs a, bool replay) {
  const uint32_t count = *a.queue_count;
  const uint32_t qi = blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= count) return;
  const SecEntry e = a.queue[qi];
  EnvView E;
  TraceParams P;
  req_shading<B>(a, e.ray, E, P);
  const int64_t local = req_view<B>(a, e.ray).local;
  const d3 w = mk(e.w[0], e.w[1], e.w[2]);
  const Record r2 = load_record(a.rec2 + qi);
  const double c_env = E.scal[1];
  const bool nee = (P.flags & LF_FLAG_NEE) != 0;
  SecCoef sc;
  if (!nee || (e.s & 1)) {  // the indirect term: every ray of the one-ray form, continuations of the two-ray form
    secondary_coefs(E, P, r2, w, local, nee ? e.s >> 1 : e.s, c_env, sc);
  } else {
    sc.ce = sc.cb = sc.we = sc.wb = mk(0, 0, 0);
    sc.has_e = sc.has_b = false;
  }
  const double T2w = (double)e.tw * r2.T;
  const int64_t cs = (int64_t)e.ray * a.spp_stride + e.s;
  if (replay) {
    SecFrozen f;
    f.T2 = (float)T2w;
    f.ce[0] = (float)sc.ce.x; f.ce[1] = (float)sc.ce.y; f.ce[2] = (float)sc.ce.z;
    f.cb[0] = (float)sc.cb.x; f.cb[1] = (float)sc.cb.y; f.cb[2] = (float)sc.cb.z;
    f.we[0] = (float)sc.we.x; f.we[1] = (float)sc.we.y; f.we[2] = (float)sc.we.z;
    f.wb[0] = (float)sc.wb.x; f.wb[1] = (float)sc.wb.y; f.wb[2] = (float)sc.wb.z;
    f.has = (sc.has_e ? 1u : 0u) | (sc.has_b ? 2u : 0u);
    a.frozen[cs] = f;
    return;
  }
  d3 Lin = T2w * env_eval(E, w);
  if (sc.has_e) {
    const d3 Ee = env_eval(E, sc.we);
    Lin = Lin + mk(sc.ce.x * Ee.x, sc.ce.y * Ee.y, sc.ce.z * Ee.z);
  }
  if (sc.has_b) {
    const d3 Eb = env_eval(E, sc.wb);
    Lin = Lin + mk(sc.cb.x * Eb.x, sc.cb.y * Eb.y, sc.cb.z * Eb.z);
  }
  a.contrib[3 * cs + 0] = (float)(e.thr[0] * Lin.x);
  a.contrib[3 * cs + 1] = (float)(e.thr[1] * Lin.y);
  a.contrib[3 * cs + 2] = (float)(e.thr[2] * Lin.z);
}

template <bool B>
__global__ void k_resolve(RenderArgs a) {
  const int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ray >= a.R) return;
  const ReqView v = req_view<B>(a, ray);
  if (!v.valid) return;
  int S = a.spp_stride;  // slots of every ray (the server's requests use the one-ray form)
  if constexpr (B) S = a.slots[a.chunks[ray / kChunk].slot].spp;
  float *rad = v.radiance + 3 * v.local;
  double L[3] = {rad[0], rad[1], rad[2]};
  for (int s = 0; s < S; ++s)
    for (int c = 0; c < 3; ++c) L[c] += (double)a.contrib[3 * (ray * a.spp_stride + s) + c];
  for (int c = 0; c < 3; ++c) rad[c] = (float)L[c];
}

__global__ void k_raygen(const CamArgs *cams, int64_t n, float *o, float *d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  raygen_f32(*cams, 0, i, o + 3 * i, d + 3 * i);
}

__global__ void k_accum(unsigned long long *acc, const uint32_t *count) { *acc += *count; }


template <int K, bool B>
void trace1_k(const RenderArgs &a, hipStream_t st) {
  const int64_t items = (!B && a.n_tiles) ? a.n_tiles * kBlock : a.R;
  launch_fill_u32(a.work, 0u, kPoolParts, st);
  // coherent camera rays as wave packets once every resident block has some
  // to take; smaller launches are bound by their slowest rays, and one ray per
  // lane spreads them thinner
  bool packets = (B || a.n_tiles) && !(a.P.flags & LF_FLAG_BRUTE_FORCE);
  if (packets) packets = items >= (int64_t)pool_blocks<k_trace1p<K, B>>(INT64_MAX / 4) * kBlock;
  if (packets)
    hipLaunchKernelGGL((k_trace1p<K, B>), dim3(pool_blocks<k_trace1p<K, B>>(items)), dim3(kBlock), 0, st, a);
  else
    hipLaunchKernelGGL((k_trace1<K, B>), dim3(pool_blocks<k_trace1<K, B>>(items)), dim3(kBlock), 0, st, a);
}
template <int K, bool B>
void composite1_k(const RenderArgs &a, bool replay, hipStream_t st) {
  const int64_t items = (!B && a.n_tiles) ? a.n_tiles * kBlock : a.R;
  hipLaunchKernelGGL((k_composite1<K, B>), dim3(blocks(items, kBlock)), dim3(kBlock), 0, st, a, replay);
}
template <int K, bool B>
void trace2_k(const RenderArgs &a, hipStream_t st) {
  launch_fill_u32(a.work, 0u, kPoolParts, st);
  hipLaunchKernelGGL((k_trace2<K, B>), dim3(pool_blocks<k_trace2<K, B>>(a.R * a.spp_stride)), dim3(kBlock), 0, st,
                     a);
}
template <int K, bool B>
void composite2_k(const RenderArgs &a, hipStream_t st) {
  hipLaunchKernelGGL((k_composite2<K, B>), dim3(blocks(a.R * a.spp_stride, kBlock)), dim3(kBlock), 0, st, a);
}
// fn<K, B>(args...) for the k-buffer size bucket of a.P.k
#define LF_K_DISPATCH(fn, B, ...)                  \
  switch (kbucket(a.P.k)) {                        \
    case 8: fn<8, B>(__VA_ARGS__); break;          \
    case 16: fn<16, B>(__VA_ARGS__); break;        \
    case 32: fn<32, B>(__VA_ARGS__); break;        \
    default: fn<64, B>(__VA_ARGS__); break;        \
  }

}  // namespace

void launch_instances(const float *R, const float *t, const float *root_box6, const int32_t *inst_first,
                      const int32_t *inst_n, const int32_t *inst_root, int n_inst, InstRec *out, double *bounds6,
                      uint32_t *status, hipStream_t st) {
  hipLaunchKernelGGL(k_instances, dim3(1), dim3(kMaxInst), 0, st, R, t, root_box6, inst_first, inst_n, inst_root,
                     n_inst, out, bounds6, status);
}

void launch_secondary_keys(const SecEntry *queue, const uint32_t *count, int64_t cap, const double *bounds6,
                           const ChunkDesc *chunks, const BatchSlot *slots, uint64_t *keys, int32_t *vals,
                           hipStream_t st) {
  if (cap <= 0) return;
  hipLaunchKernelGGL(k_secondary_keys, dim3(blocks(cap, 256)), dim3(256), 0, st, queue, count, cap, bounds6, chunks,
                     slots, keys, vals);
}

void launch_env_tables(const float *tex, int H, int W, uint32_t flags, double *cdf_row, double *cdf_col, double *lum,
                       double *rowsum, double *roww, double *scal, hipStream_t st) {
  hipLaunchKernelGGL(k_env_rows, dim3(H), dim3(256), 0, st, tex, H, W, cdf_col, lum, rowsum, roww);
  hipLaunchKernelGGL(k_env_marginal, dim3(1), dim3(256), 0, st, H, flags, roww, cdf_row, scal);
}

void launch_trace1(const RenderArgs &a, hipStream_t st) {
  if (a.R <= 0) return;
  if (a.chunks) LF_K_DISPATCH(trace1_k, true, a, st)
  else LF_K_DISPATCH(trace1_k, false, a, st)
}

void launch_composite1(const RenderArgs &a, bool replay, hipStream_t st) {
  if (a.R <= 0) return;
  if (a.chunks) LF_K_DISPATCH(composite1_k, true, a, replay, st)
  else LF_K_DISPATCH(composite1_k, false, a, replay, st)
}

void launch_shade1(const RenderArgs &a, bool replay, hipStream_t st) {
  if (a.R <= 0) return;
  if (a.chunks) hipLaunchKernelGGL(k_shade1<true>, dim3(blocks(a.R, 256)), dim3(256), 0, st, a, replay);
  else hipLaunchKernelGGL(k_shade1<false>, dim3(blocks(a.R, 256)), dim3(256), 0, st, a, replay);
}

void launch_trace2(const RenderArgs &a, hipStream_t st) {
  if (a.R <= 0) return;
  if (a.chunks) LF_K_DISPATCH(trace2_k, true, a, st)
  else LF_K_DISPATCH(trace2_k, false, a, st)
}

void launch_composite2(const RenderArgs &a, hipStream_t st) {
  if (a.R <= 0) return;
  if (a.chunks) LF_K_DISPATCH(composite2_k, true, a, st)
  else LF_K_DISPATCH(composite2_k, false, a, st)
}

void launch_shade2(const RenderArgs &a, bool replay, hipStream_t st) {
  if (a.R <= 0) return;
  const unsigned nb = blocks(a.R * a.spp_stride, 256);
  if (a.chunks) hipLaunchKernelGGL(k_shade2<true>, dim3(nb), dim3(256), 0, st, a, replay);
  else hipLaunchKernelGGL(k_shade2<false>, dim3(nb), dim3(256), 0, st, a, replay);
}

void launch_resolve(const RenderArgs &a, hipStream_t st) {
  if (a.R <= 0) return;
  if (a.chunks) hipLaunchKernelGGL(k_resolve<true>, dim3(blocks(a.R, 256)), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(k_resolve<false>, dim3(blocks(a.R, 256)), dim3(256), 0, st, a);
}

void launch_raygen(const CamArgs *cams, int64_t n, float *o, float *d, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_raygen, dim3(blocks(n, 256)), dim3(256), 0, st, cams, n, o, d);
}

void launch_accum(unsigned long long *acc, const uint32_t *count, hipStream_t st) {
  hipLaunchKernelGGL(k_accum, dim3(1), dim3(1), 0, st, acc, count);
}

}  // namespace lf

// lf_device.h -- device functions of the gfx950 tracer: ray generation,
// BVH traversal with a k-closest hit buffer, front-to-back compositing,
// environment sampling and the metallic-roughness BRDF.
//
// Precision split.  Every discrete decision of the method (which surfels are
// hit, their (t, index) order, the k-truncation, the sampled directions,
// technique/lobe choices, hemisphere tests, texel choices) is taken in double
// precision from the binary32 inputs, so the results agree with exact
// arithmetic except for inputs within a few ulps of a switching point.  The
// BVH is traversed with binary32 boxes and slab tests made conservative by
// construction, so traversal never culls a valid hit.
#pragma once
#include "lf_internal.h"

namespace lf {

// ------------------------------------------------------------------ vectors
struct d3 { double x, y, z; };
__device__ __forceinline__ d3 mk(double x, double y, double z) { return d3{x, y, z}; }
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ d3 operator*(double s, d3 a) { return mk(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ d3 operator-(d3 a) { return mk(-a.x, -a.y, -a.z); }
__device__ __forceinline__ double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 cross(d3 a, d3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double lum(d3 c) { return 0.2126 * c.x + 0.7152 * c.y + 0.0722 * c.z; }
__device__ __forceinline__ double clampd(double x, double lo, double hi) { return fmin(fmax(x, lo), hi); }
__device__ __forceinline__ d3 ld3(const float *p) { return mk(p[0], p[1], p[2]); }
// M (row-major 3x3) times v, and its transpose
__device__ __forceinline__ d3 mul(const double *M, d3 v) {
  return mk(M[0] * v.x + M[1] * v.y + M[2] * v.z, M[3] * v.x + M[4] * v.y + M[5] * v.z,
            M[6] * v.x + M[7] * v.y + M[8] * v.z);
}
__device__ __forceinline__ d3 mulT(const double *M, d3 v) {
  return mk(M[0] * v.x + M[3] * v.y + M[6] * v.z, M[1] * v.x + M[4] * v.y + M[7] * v.z,
            M[2] * v.x + M[5] * v.y + M[8] * v.z);
}

constexpr double kPi = 3.14159265358979323846;
constexpr double kInvPi = 1.0 / kPi;

// ------------------------------------------------------------------ sampler
// SplitMix64 (Steele, Lea & Flood 2014) chained over (seed, ray, sample, dim);
// the top 24 bits give a uniform in [0,1) that is exact in float and double.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double urand(uint64_t seed, uint64_t ray, uint64_t s, uint32_t dim) {
  uint64_t h = splitmix64(seed ^ splitmix64(ray ^ splitmix64((s << 8) | (uint64_t)dim)));
  return (double)(h >> 40) * (1.0 / 16777216.0);
}

// Owen-scrambled Sobol uniforms (the replayed Sobol samples of the PRB
// paragraph, Sec. 3.3).  Direction numbers of 11 dimensions: dimension 0 is
// van der Corput; dimensions 1..10 use the primitive polynomials and initial
// numbers of Joe and Kuo (2008), degree s, inner coefficients a (a_1 the top
// bit), m_1..m_s, extended by V_k = a_1 V_(k-1) ^ ... ^ a_(s-1) V_(k-s+1) ^
// V_(k-s) ^ (V_(k-s) >> s) on the 32-bit fractions V_k = m_k 2^(32-k).
struct SobolDirections {
  uint32_t v[11][32];  // v[d][k-1] = V_k
};

constexpr SobolDirections sobol_directions() {
  constexpr int deg[11] = {0, 1, 2, 3, 3, 4, 4, 5, 5, 5, 5};
  constexpr uint32_t inner[11] = {0, 0, 1, 1, 2, 1, 4, 2, 4, 7, 11};
  constexpr uint32_t init[11][5] = {{0}, {1}, {1, 3}, {1, 3, 1}, {1, 1, 1}, {1, 1, 3, 3}, {1, 3, 5, 13},
                                    {1, 1, 5, 5, 17}, {1, 1, 5, 5, 5}, {1, 1, 7, 11, 19}, {1, 1, 5, 1, 1}};
  SobolDirections t{};
  for (int k = 1; k <= 32; ++k) t.v[0][k - 1] = 1u << (32 - k);
  for (int d = 1; d < 11; ++d) {
    const int s = deg[d];
    for (int k = 1; k <= 32; ++k) {
      uint32_t v = 0;
      if (k <= s) {
        v = init[d][k - 1] << (32 - k);
      } else {
        v = t.v[d][k - s - 1] ^ (t.v[d][k - s - 1] >> s);
        for (int j = 1; j < s; ++j)
          if ((inner[d] >> (s - 1 - j)) & 1u) v ^= t.v[d][k - j - 1];
      }
      t.v[d][k - 1] = v;
    }
  }
  return t;
}

__constant__ SobolDirections kSobol = sobol_directions();

__device__ __forceinline__ uint32_t sobol32(uint32_t i, int d) {
  uint32_t x = 0;
  for (int k = 0; i; ++k, i >>= 1)
    if (i & 1u) x ^= kSobol.v[d][k];
  return x;
}

// Nested uniform (Owen) scramble by Burley's hash ("Practical Hash-based Owen
// Scrambling", 2020): in bit-reversed order an add and four xor-multiplies by
// even constants, so each bit is flipped by a function of the bits above it.
__device__ __forceinline__ uint32_t owen32(uint32_t x, uint32_t seed) {
  x = __builtin_bitreverse32(x);
  x += seed;
  x ^= x * 0x6c50b47cu;
  x ^= x * 0xb82f1e52u;
  x ^= x * 0xc7afe638u;
  x ^= x * 0x8d22f6e6u;
  return __builtin_bitreverse32(x);
}

// 24-bit uniform of (seed, ray, sample, dim): the ray's hash scrambles the
// sample index (each ray draws an aligned block of the sequence) and, per
// dimension, the coordinate.
__device__ __forceinline__ double sobol_u(uint64_t seed, uint64_t ray, uint64_t s, uint32_t dim) {
  const uint64_t h = splitmix64(seed ^ splitmix64(ray));
  const uint32_t i = owen32((uint32_t)s, (uint32_t)h);
  const uint32_t ds = (uint32_t)(splitmix64(h ^ (0x100000000ull + dim)) >> 32);
  return (double)(owen32(sobol32(i, (int)dim), ds) >> 8) * (1.0 / 16777216.0);
}


// ------------------------------------------------------------------ frames
// columns of the rotation of a unit quaternion (w,x,y,z)
__device__ __forceinline__ void quat_frame(double w, double x, double y, double z, d3 &tu, d3 &tv, d3 &n) {
  tu = mk(1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y));
  tv = mk(2 * (x * y - w * z), 1 - 2 * (x * x + z * z), 2 * (y * z + w * x));
  n = mk(2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y));
}

// branchless orthonormal basis about n (Duff et al. 2017)
__device__ __forceinline__ void onb(d3 n, d3 &b1, d3 &b2) {
  double sign = n.z >= 0.0 ? 1.0 : -1.0;
  double a = -1.0 / (sign + n.z);
  double b = n.x * n.y * a;
  b1 = mk(1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x);
  b2 = mk(b, sign + n.y * n.y * a, -n.y);
}

// ------------------------------------------------------------------ raygen
// Pinhole ray through the centre of pixel `pix` of camera c, in binary32
// with a fixed operation order, no contraction, correctly rounded division
// and square root (so every implementation produces the same bits).
__device__ __noinline__ void raygen_f32(const CamArgs &ca, int c, int64_t pix, float *o, float *d) {
#pragma clang fp contract(off)
  const float *P = ca.pose[c];
  int32_t w = ca.w[c], h = ca.h[c];
  float fw = (float)w, fh = (float)h;
  float aspect = fw / fh;
  int64_t px = pix % w, py = pix / w;
  float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  float th = ca.tan_half[c];
  float sx = (2.0f * fx / fw - 1.0f) * th;
  sx = sx * aspect;
  float sy = (1.0f - 2.0f * fy / fh) * th;
  float dx = P[0] * sx, dy = P[4] * sx, dz = P[8] * sx;
  dx = dx + P[1] * sy;
  dy = dy + P[5] * sy;
  dz = dz + P[9] * sy;
  dx = dx - P[2];
  dy = dy - P[6];
  dz = dz - P[10];
  float ss = dx * dx;
  ss = ss + dy * dy;
  ss = ss + dz * dz;
  float len = sqrtf(ss);
  d[0] = dx / len;
  d[1] = dy / len;
  d[2] = dz / len;
  o[0] = P[3];
  o[1] = P[7];
  o[2] = P[11];
}

__device__ __forceinline__ void load_ray(const RaySource &rs, int64_t id, float *o, float *d) {
  if (rs.o) {
    o[0] = rs.o[3 * id + 0]; o[1] = rs.o[3 * id + 1]; o[2] = rs.o[3 * id + 2];
    d[0] = rs.d[3 * id + 0]; d[1] = rs.d[3 * id + 1]; d[2] = rs.d[3 * id + 2];
  } else {
    const CamArgs &ca = *rs.cams;
    int c = 0;
    while (c + 1 < ca.n_cams && id >= ca.first[c + 1]) ++c;
    raygen_f32(ca, c, id - ca.first[c], o, d);
  }
}

// Camera ray of work item `item` when primary rays are traced in 16x8-pixel
// tiles: items 128t..128t+127 cover tile t (row-major over each camera's
// tiles), the first 64 its left 8x8 half, so consecutive items are spatially
// compact.  -1 for an item outside the image.
__device__ __forceinline__ int64_t tile_ray(const CamArgs &ca, int64_t item) {
  const int64_t tile = item / kBlock;
  const int within = (int)(item % kBlock);
  int c = 0;
  while (c + 1 < ca.n_cams && tile >= ca.tiles[c + 1]) ++c;
  const int64_t lt = tile - ca.tiles[c];
  const int nx = (ca.w[c] + 15) / 16;
  const int tx = (int)(lt % nx), ty = (int)(lt / nx);
  const int lane = within & 63, half = within >> 6;
  const int x = tx * 16 + half * 8 + (lane & 7), y = ty * 8 + (lane >> 3);
  if (x >= ca.w[c] || y >= ca.h[c]) return -1;
  return ca.first[c] + (int64_t)y * ca.w[c] + x;
}

// ------------------------------------------------------------------ k-closest buffers
// Hits are ordered by (t, surfel index).  Entries hold the leaf position of
// the surfel and a flip bit (stored normal faces away from the ray).  The
// first K-k slots hold -inf sentinels so the k-th hit always sits in the last
// (static) slot.
//
// Keys are t rounded to binary32, which preserves the order of distinct
// keys; a new key equal to one in the buffer is placed by the exact double t
// and, on exact ties, the surfel index (kinsert_tied), so the buffer always
// holds the k closest hits in exact (t, index) order.
template <int K>
struct KBufF {
  float t[K];
  uint32_t id[K];
};

template <int K>
__device__ __forceinline__ void kinit(KBufF<K> &b, int k) {
  // k is made opaque here, so the sentinels are set where the buffer starts
  // instead of being computed once and kept (spilled) for every later start
  int kk = k;
  asm volatile("" : "+s"(kk));
#pragma unroll
  for (int j = 0; j < K; ++j) {
    b.t[j] = j < K - kk ? -INFINITY : INFINITY;
    b.id[j] = kIdMask;
  }
}

// Insertion into the sorted buffer without a carried dependency: since the
// buffer is non-decreasing, "key < t[j]" is monotone in j, and slot j takes
// t[j-1] if the key also precedes t[j-1], the key if it precedes t[j] only,
// and keeps t[j] otherwise.  Slots are updated from the top down so t[j-1] is
// still the old value; every slot's comparisons are independent.  Only used
// for a key equal to no key in the buffer.
// k-buffer of one ray in device memory: t[K] then id[K] (2K words)
template <int K>
__device__ __forceinline__ void store_kbuf(const KBufF<K> &b, uint32_t *out) {
  uint4 *o = (uint4 *)out;
#pragma unroll
  for (int j = 0; j < K / 4; ++j)
    o[j] = make_uint4(__float_as_uint(b.t[4 * j]), __float_as_uint(b.t[4 * j + 1]), __float_as_uint(b.t[4 * j + 2]),
                      __float_as_uint(b.t[4 * j + 3]));
#pragma unroll
  for (int j = 0; j < K / 4; ++j) o[K / 4 + j] = make_uint4(b.id[4 * j], b.id[4 * j + 1], b.id[4 * j + 2], b.id[4 * j + 3]);
}

template <int K>
__device__ __forceinline__ void load_kbuf(KBufF<K> &b, const uint32_t *in) {
  const uint4 *p = (const uint4 *)in;
#pragma unroll
  for (int j = 0; j < K / 4; ++j) {
    const uint4 v = p[j];
    b.t[4 * j] = __uint_as_float(v.x); b.t[4 * j + 1] = __uint_as_float(v.y);
    b.t[4 * j + 2] = __uint_as_float(v.z); b.t[4 * j + 3] = __uint_as_float(v.w);
    const uint4 w = p[K / 4 + j];
    b.id[4 * j] = w.x; b.id[4 * j + 1] = w.y; b.id[4 * j + 2] = w.z; b.id[4 * j + 3] = w.w;
  }
}

template <int K>
__device__ __forceinline__ void kinsert(KBufF<K> &b, float t, uint32_t id) {
#pragma unroll
  for (int j = K - 1; j >= 0; --j) {
    const float bt = b.t[j];
    const bool here = t < bt;
    const bool below = j > 0 && t < b.t[j > 0 ? j - 1 : 0];
    b.t[j] = here ? (below ? b.t[j > 0 ? j - 1 : 0] : t) : bt;
    b.id[j] = here ? (below ? b.id[j > 0 ? j - 1 : 0] : id) : b.id[j];
  }
}

// Rotations walk a buffer with one loop body (static register indexing):
// after K rotations the buffer is back in its original order.
template <class B, int K>
__device__ __forceinline__ void krotl(B &b) {
  auto t0 = b.t[0];
  uint32_t i0 = b.id[0];
#pragma unroll
  for (int j = 0; j < K - 1; ++j) { b.t[j] = b.t[j + 1]; b.id[j] = b.id[j + 1]; }
  b.t[K - 1] = t0;
  b.id[K - 1] = i0;
}
template <class B, int K>
__device__ __forceinline__ void krotr(B &b) {
  auto t0 = b.t[K - 1];
  uint32_t i0 = b.id[K - 1];
#pragma unroll
  for (int j = K - 1; j > 0; --j) { b.t[j] = b.t[j - 1]; b.id[j] = b.id[j - 1]; }
  b.t[0] = t0;
  b.id[0] = i0;
}

// ------------------------------------------------------------------ traversal
// adjacent binary32 values (finite arguments)
__device__ __forceinline__ float next_up_f(float f) {
  if (f == 0.0f) return 1.4e-45f;
  int b = __float_as_int(f);
  return __int_as_float(f > 0.0f ? b + 1 : b - 1);
}
__device__ __forceinline__ float next_down_f(float f) { return -next_up_f(-f); }
__device__ __forceinline__ float round_up_f(double v) {
  float f = (float)v;
  return ((double)f < v && isfinite(f)) ? next_up_f(f) : f;
}
__device__ __forceinline__ float round_down_f(double v) {
  float f = (float)v;
  return ((double)f > v && isfinite(f)) ? next_down_f(f) : f;
}

// exact slab test of a double ray against a double box: entry/exit t
__device__ __forceinline__ bool slab64(d3 o, d3 d, const double *lo, const double *hi, double &tn, double &tf) {
  tn = -INFINITY;
  tf = INFINITY;
  const double oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (dd[a] == 0.0) {
      if (oo[a] < lo[a] || oo[a] > hi[a]) return false;
    } else {
      double i = 1.0 / dd[a];
      double t0 = (lo[a] - oo[a]) * i, t1 = (hi[a] - oo[a]) * i;
      tn = fmax(tn, fmin(t0, t1));
      tf = fmin(tf, fmax(t0, t1));
    }
  }
  return tn <= tf;
}

// Binary32 view of the object-space ray for the box tests.  Every box is
// grown by pad >= the distance between the exact ray and this binary32 ray
// over the instance's parameter range (rounded origin and direction, and the
// clamping of tiny direction components), so a box the exact ray enters is
// never culled.  On axis a a node's plane of code q is met at
// q * (2^e / d) + fma(p, 1/d, nb) (near planes) or + fma(p, 1/d, fb) (far
// planes), with nb = -o / d - pad / |d| - E and fb = -o / d + pad / |d| + E;
// E bounds every rounding in these (of 1/d, the products, the fused
// multiply-adds and the half ulp between a decoded plane and its real code
// value) for frame origins and steps within the instance's object-space
// bounds (|p| <= omag, 255 * 2^e <= 4 oext), so near distances are never
// overestimated and far ones never underestimated.  An axis whose terms are
// not safely finite is left unconstrained.
struct RayF {
  float ox, oy, oz;      // origin
  float dx, dy, dz;      // direction
  float ix, iy, iz;      // 1/d
  bool sx, sy, sz;       // d >= 0 per axis
  float nbx, nby, nbz;   // near-plane offsets
  float fbx, fby, fbz;   // far-plane offsets
  float oabs;            // max |origin component|
};

__device__ __forceinline__ float inv_dir(float d) {
  float dd = fabsf(d) < 1e-20f ? copysignf(1e-20f, d) : d;
  return 1.0f / dd;
}

__device__ __forceinline__ void plane_offsets(float o, float inv, float pad, float omag, float oext, float &nb,
                                              float &fb) {
  const float ai = fabsf(inv);
  const float span = (omag + 4.0f * oext + fabsf(o) + pad) * ai;
  if (!(span < 0x1p100f)) {
    nb = -INFINITY;
    fb = INFINITY;
    return;
  }
  const float E = 0x1p-18f * span + 1e-30f;
  const float ob = o * inv, g = pad * ai;
  nb = (-ob - g) - E;
  fb = (-ob + g) + E;
}

__device__ __forceinline__ void make_rayf(d3 oo, d3 dd, double tabs, float omag, float oext, RayF &rf) {
  rf.ox = (float)oo.x; rf.oy = (float)oo.y; rf.oz = (float)oo.z;
  rf.dx = (float)dd.x; rf.dy = (float)dd.y; rf.dz = (float)dd.z;
  rf.oabs = fmaxf(fmaxf(fabsf(rf.ox), fabsf(rf.oy)), fabsf(rf.oz));
  const double eo = fmax(fmax(fabs(oo.x - rf.ox), fabs(oo.y - rf.oy)), fabs(oo.z - rf.oz));
  const double ed = fmax(fmax(fabs(dd.x - rf.dx), fabs(dd.y - rf.dy)), fabs(dd.z - rf.dz)) + 1e-20;
  const float pad = (float)((eo + ed * tabs + 1e-30) * 1.001) + 1e-30f;
  rf.ix = inv_dir(rf.dx); rf.iy = inv_dir(rf.dy); rf.iz = inv_dir(rf.dz);
  rf.sx = rf.ix >= 0.f; rf.sy = rf.iy >= 0.f; rf.sz = rf.iz >= 0.f;
  plane_offsets(rf.ox, rf.ix, pad, omag, oext, rf.nbx, rf.fbx);
  plane_offsets(rf.oy, rf.iy, pad, omag, oext, rf.nby, rf.fby);
  plane_offsets(rf.oz, rf.iz, pad, omag, oext, rf.nbz, rf.fbz);
}

// Visits one traversal node: the masks of the internal and leaf slots whose
// decoded boxes (grown by pad) the ray enters within [tlo, thi], each slot's
// entry distance t (meaningful for hit slots; >= tlo), and what locates the
// children: slot i holds node cbase + (internal slots below i) or leaf
// position lbase + (leaf slots below i).
__device__ __forceinline__ void visit_node(const QNode *node, const RayF &rf, float tlo, float thi, float *t,
                                           uint32_t &ihit, uint32_t &lhit, uint32_t &imask, int &cbase,
                                           int &lbase, bool &desc) {
  constexpr int kDw = (int)sizeof(QNode) / 4;
  constexpr int kPw = kWide / 4;  // dwords per plane
  uint32_t dw[kDw];
  const uint4 *src = (const uint4 *)node;
#pragma unroll
  for (int v = 0; v < kDw / 4; ++v) {
    const uint4 x = src[v];
    dw[4 * v] = x.x; dw[4 * v + 1] = x.y; dw[4 * v + 2] = x.z; dw[4 * v + 3] = x.w;
  }
  const uint32_t meta = dw[3];
  // a plane of code q on axis a is met at q * C_a + B_a (see RayF)
  const float px = __uint_as_float(dw[0]), py = __uint_as_float(dw[1]), pz = __uint_as_float(dw[2]);
  const float Cx = __uint_as_float((uint32_t)((int)(int8_t)(meta & 0xffu) + 127) << 23) * rf.ix;
  const float Cy = __uint_as_float((uint32_t)((int)(int8_t)((meta >> 8) & 0xffu) + 127) << 23) * rf.iy;
  const float Cz = __uint_as_float((uint32_t)((int)(int8_t)((meta >> 16) & 0xffu) + 127) << 23) * rf.iz;
  const float Bnx = __builtin_fmaf(px, rf.ix, rf.nbx), Bfx = __builtin_fmaf(px, rf.ix, rf.fbx);
  const float Bny = __builtin_fmaf(py, rf.iy, rf.nby), Bfy = __builtin_fmaf(py, rf.iy, rf.fby);
  const float Bnz = __builtin_fmaf(pz, rf.iz, rf.nbz), Bfz = __builtin_fmaf(pz, rf.iz, rf.fbz);
  imask = meta >> 24;
  cbase = (int)dw[4];
  lbase = (int)dw[5];
  const uint32_t vmask = dw[6];
  // the internal children run along the ray in descending slot order when
  // the ray points down the node's order axis
  const uint32_t oax = (vmask >> 8) & 3u;
  desc = oax == 0 ? !rf.sx : (oax == 1 ? !rf.sy : !rf.sz);
  // codes of the near and far plane of each axis: lower codes for d >= 0
  uint32_t nx[kPw], ny[kPw], nz[kPw], fx[kPw], fy[kPw], fz[kPw];
#pragma unroll
  for (int w = 0; w < kPw; ++w) {
    const uint32_t lx = dw[7 + w], ly = dw[7 + kPw + w], lz = dw[7 + 2 * kPw + w];
    const uint32_t hx = dw[7 + 3 * kPw + w], hy = dw[7 + 4 * kPw + w], hz = dw[7 + 5 * kPw + w];
    nx[w] = rf.sx ? lx : hx; fx[w] = rf.sx ? hx : lx;
    ny[w] = rf.sy ? ly : hy; fy[w] = rf.sy ? hy : ly;
    nz[w] = rf.sz ? lz : hz; fz[w] = rf.sz ? hz : lz;
  }
  uint32_t hits = 0;
#pragma unroll
  for (int i = 0; i < kWide; ++i) {
    const int w = i / 4, b = 8 * (i % 4);
    const float tnx = __builtin_fmaf((float)((nx[w] >> b) & 0xffu), Cx, Bnx);
    const float tny = __builtin_fmaf((float)((ny[w] >> b) & 0xffu), Cy, Bny);
    const float tnz = __builtin_fmaf((float)((nz[w] >> b) & 0xffu), Cz, Bnz);
    const float tfx = __builtin_fmaf((float)((fx[w] >> b) & 0xffu), Cx, Bfx);
    const float tfy = __builtin_fmaf((float)((fy[w] >> b) & 0xffu), Cy, Bfy);
    const float tfz = __builtin_fmaf((float)((fz[w] >> b) & 0xffu), Cz, Bfz);
    const float n = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, tlo));
    const float f = fminf(fminf(tfx, tfy), fminf(tfz, thi));
    hits |= n <= f ? 1u << i : 0u;
    t[i] = n;
  }
  hits &= vmask;
  lhit = hits & ~imask;
  ihit = hits & imask;
}

constexpr int kNodeDw = (int)sizeof(QNode) / 4;

// The same test on a node's words already loaded (dw[kNodeDw]), for the
// wave-packet traversal, whose node words come through the scalar cache.
__device__ __forceinline__ void visit_node_dw(const uint32_t *dw, const RayF &rf, float tlo, float thi, float *t,
                                              uint32_t &ihit, uint32_t &lhit, uint32_t &imask, int &cbase,
                                              int &lbase, bool &desc) {
  constexpr int kPw = kWide / 4;  // dwords per plane
  const uint32_t meta = dw[3];
  // a plane of code q on axis a is met at q * C_a + B_a (see RayF)
  const float px = __uint_as_float(dw[0]), py = __uint_as_float(dw[1]), pz = __uint_as_float(dw[2]);
  const float Cx = __uint_as_float((uint32_t)((int)(int8_t)(meta & 0xffu) + 127) << 23) * rf.ix;
  const float Cy = __uint_as_float((uint32_t)((int)(int8_t)((meta >> 8) & 0xffu) + 127) << 23) * rf.iy;
  const float Cz = __uint_as_float((uint32_t)((int)(int8_t)((meta >> 16) & 0xffu) + 127) << 23) * rf.iz;
  const float Bnx = __builtin_fmaf(px, rf.ix, rf.nbx), Bfx = __builtin_fmaf(px, rf.ix, rf.fbx);
  const float Bny = __builtin_fmaf(py, rf.iy, rf.nby), Bfy = __builtin_fmaf(py, rf.iy, rf.fby);
  const float Bnz = __builtin_fmaf(pz, rf.iz, rf.nbz), Bfz = __builtin_fmaf(pz, rf.iz, rf.fbz);
  imask = meta >> 24;
  cbase = (int)dw[4];
  lbase = (int)dw[5];
  const uint32_t vmask = dw[6];
  // the internal children run along the ray in descending slot order when
  // the ray points down the node's order axis
  const uint32_t oax = (vmask >> 8) & 3u;
  desc = oax == 0 ? !rf.sx : (oax == 1 ? !rf.sy : !rf.sz);
  // codes of the near and far plane of each axis: lower codes for d >= 0
  uint32_t nx[kPw], ny[kPw], nz[kPw], fx[kPw], fy[kPw], fz[kPw];
#pragma unroll
  for (int w = 0; w < kPw; ++w) {
    const uint32_t lx = dw[7 + w], ly = dw[7 + kPw + w], lz = dw[7 + 2 * kPw + w];
    const uint32_t hx = dw[7 + 3 * kPw + w], hy = dw[7 + 4 * kPw + w], hz = dw[7 + 5 * kPw + w];
    nx[w] = rf.sx ? lx : hx; fx[w] = rf.sx ? hx : lx;
    ny[w] = rf.sy ? ly : hy; fy[w] = rf.sy ? hy : ly;
    nz[w] = rf.sz ? lz : hz; fz[w] = rf.sz ? hz : lz;
  }
  uint32_t hits = 0;
#pragma unroll
  for (int i = 0; i < kWide; ++i) {
    const int w = i / 4, b = 8 * (i % 4);
    const float tnx = __builtin_fmaf((float)((nx[w] >> b) & 0xffu), Cx, Bnx);
    const float tny = __builtin_fmaf((float)((ny[w] >> b) & 0xffu), Cy, Bny);
    const float tnz = __builtin_fmaf((float)((nz[w] >> b) & 0xffu), Cz, Bnz);
    const float tfx = __builtin_fmaf((float)((fx[w] >> b) & 0xffu), Cx, Bfx);
    const float tfy = __builtin_fmaf((float)((fy[w] >> b) & 0xffu), Cy, Bfy);
    const float tfz = __builtin_fmaf((float)((fz[w] >> b) & 0xffu), Cz, Bfz);
    const float n = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, tlo));
    const float f = fminf(fminf(tfx, tfy), fminf(tfz, thi));
    hits |= n <= f ? 1u << i : 0u;
    t[i] = n;
  }
  hits &= vmask;
  lhit = hits & ~imask;
  ihit = hits & imask;
}

// Exact (double) plane intersection and support test of the surfel at leaf
// position pos against the object-space ray (o, d).  Returns false if the
// surfel is not hit; otherwise t and the flip bit.
// Plane intersection n.(mu - o) / n.d of the object-space ray with a
// surfel's plane, with a fixed operation order (no contraction): every
// recomputation for the same surfel and ray gives the same double.
__device__ __forceinline__ double plane_den(const TraceRec &r, d3 d) {
#pragma clang fp contract(off)
  return r.n[0] * d.x + r.n[1] * d.y + r.n[2] * d.z;
}
__device__ __forceinline__ double plane_t(const TraceRec &r, d3 o, double den) {
#pragma clang fp contract(off)
  const double mx = (double)r.mu[0] - o.x, my = (double)r.mu[1] - o.y, mz = (double)r.mu[2] - o.z;
  return (r.n[0] * mx + r.n[1] * my + r.n[2] * mz) / den;
}

__device__ __forceinline__ bool exact_hit(const TraceRec &r, d3 o, d3 d, double t_min, double &t, bool &flip) {
  const double den = plane_den(r, d);
  if (!(fabs(den) >= 1e-12)) return false;
  const d3 n = mk(r.n[0], r.n[1], r.n[2]);
  const d3 mu = mk((double)r.mu[0], (double)r.mu[1], (double)r.mu[2]);
  t = plane_t(r, o, den);
  if (!(t > t_min)) return false;
  d3 dl = (o + t * d) - mu;
  double xu = dl.x * r.a[0] + dl.y * r.a[1] + dl.z * r.a[2];
  double xv = dl.x * r.b[0] + dl.y * r.b[1] + dl.z * r.b[2];
  double rho2 = xu * xu + xv * xv;
  flip = den > 0.0;
  return rho2 <= r.rho2max;
}

// Binary32 pre-filter: rejects a surfel only if, with a bound on every
// rounding error of the binary32 evaluation (a factor of about 8 above the
// first-order error of each product and sum), its plane intersection is
// certainly behind t_min or beyond tk_up, or its local radius certainly lies
// outside the support.  Everything else goes to exact_hit.  The unit normal
// is the normalised cross product of the rounded scaled tangents a and b
// (orthogonal, so |a x b| = |a||b|): about 6 ulp per component, against half
// an ulp for a stored normal, so the bound on t takes twice the factor.  Its
// sign is immaterial (t = num / den flips both).
__device__ __forceinline__ bool prefilter(const FiltRec &F, const RayF &r, float t_min_f, float tk_up) {
  const float4 v0 = F.v0, v1 = F.v1, v2 = F.v2;
  const float ax = v0.x, ay = v0.y, az = v0.z, bx = v1.x, by = v1.y, bz = v1.z;
  const float cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
  const float c2 = cx * cx + cy * cy + cz * cz;
  if (!(c2 >= 1e-30f && c2 <= 1e30f)) return true;  // extreme scales: decide exactly
  const float ic = __builtin_amdgcn_rsqf(c2);
  const float nx = cx * ic, ny = cy * ic, nz = cz * ic;
  const float mx = v0.w, my = v1.w, mz = v2.x;
  const float den = nx * r.dx + ny * r.dy + nz * r.dz;
  const float adb = fabsf(den);
  if (!(adb >= 1e-7f)) return true;  // grazing: decide exactly
  const float rx = mx - r.ox, ry = my - r.oy, rz = mz - r.oz;
  const float num = nx * rx + ny * ry + nz * rz;
  const float t = num * __builtin_amdgcn_rcpf(den);
  const float S = r.oabs + fmaxf(fmaxf(fabsf(mx), fabsf(my)), fabsf(mz));
  const float et = 4e-6f * (S * (1.0f + 1.0f / adb) + fabsf(t));
  if (t + et <= t_min_f) return false;
  if (t - et > tk_up) return false;
  const float dx = r.ox + t * r.dx - mx, dy = r.oy + t * r.dy - my, dz = r.oz + t * r.dz - mz;
  const float xu = dx * ax + dy * ay + dz * az;
  const float xv = dx * bx + dy * by + dz * bz;
  const float rho2 = xu * xu + xv * xv;
  const float exi = 1.8f * v2.w * (et + 2e-6f * (S + fabsf(t)));
  const float margin = exi * (2.0f * v2.z + exi) + 1e-6f * fabsf(v2.y);
  return rho2 <= v2.y + margin;
}

// Test one surfel and insert it if valid and among the k closest.
// object-space ray of instance I (fixed operation order, no contraction)
__device__ __forceinline__ void to_object(const InstRec &I, d3 o, d3 d, d3 &oo, d3 &dd) {
#pragma clang fp contract(off)
  if (I.identity) {
    oo = o;
    dd = d;
  } else {
    const double *M = I.R;
    const double px = o.x - I.t[0], py = o.y - I.t[1], pz = o.z - I.t[2];
    oo = mk(M[0] * px + M[3] * py + M[6] * pz, M[1] * px + M[4] * py + M[7] * pz, M[2] * px + M[5] * py + M[8] * pz);
    dd = mk(M[0] * d.x + M[3] * d.y + M[6] * d.z, M[1] * d.x + M[4] * d.y + M[7] * d.z,
            M[2] * d.x + M[5] * d.y + M[8] * d.z);
  }
}

__device__ __forceinline__ int inst_of(const SceneView &S, int pos) {
  int ii = 0;
  for (int j = 1; j < S.n_inst; ++j)
    if (pos >= S.inst[j].first && S.inst[j].n > 0) ii = j;
  return ii;
}

// Exact key of a buffer entry for the world ray (o, d): the same plane_t of
// the same object-space ray that produced it when it was inserted.
__device__ __forceinline__ double entry_t(const SceneView &S, uint32_t id, d3 o, d3 d) {
  const int pos = (int)(id & kIdMask);
  d3 oo, dd;
  to_object(S.inst[inst_of(S, pos)], o, d, oo, dd);
  const TraceRec &r = S.rec[pos];
  return plane_t(r, oo, plane_den(r, dd));
}

// Inserts a hit whose binary32 key equals a key already in the buffer.  The
// buffer is kept in exact (t, original index) order, so its position is the
// number of entries whose binary32 key is smaller plus the number of tied
// entries whose exact key is smaller.  Walks the buffer by rotation (static
// register indexing); returns false if the hit falls beyond the k-th.
template <int K>
__device__ __forceinline__ bool kinsert_tied(const SceneView &S, KBufF<K> &b, float tf, double t, uint32_t id, d3 o,
                                          d3 d) {
  const int32_t orig = S.rec[id & kIdMask].orig;
  int p = 0;
#pragma unroll 1
  for (int r = 0; r < K; ++r) {
    const float bt = b.t[0];
    if (bt < tf) {
      ++p;
    } else if (bt == tf) {
      const double te = entry_t(S, b.id[0], o, d);
      if (te < t || (te == t && S.rec[b.id[0] & kIdMask].orig < orig)) ++p;
    }
    krotl<KBufF<K>, K>(b);
  }
  if (p >= K) return false;
#pragma unroll
  for (int j = K - 1; j >= 0; --j) {
    const int jm = j > 0 ? j - 1 : 0;
    b.t[j] = j > p ? b.t[jm] : (j == p ? tf : b.t[j]);
    b.id[j] = j > p ? b.id[jm] : (j == p ? id : b.id[j]);
  }
  return true;
}

// Exact (FP64) plane hit and support/threshold test of the surfel at leaf
// position pos, which passed the pre-filter, against the object-space ray
// (o, d) of the world ray (wo, wd), and insertion of a valid hit that belongs
// to the k closest.  Binary32 keys are roundings of the exact distances and
// rounding is monotone, so a key above the k-th key is beyond the exact k-th
// distance and distinct keys order exactly; a key equal to one in the buffer
// is placed by exact keys.  Returns bit 0: inserted, bit 1: placed by exact
// keys, bit 2: passed the binary32 pre-filter (always set), bit 3: valid hit.
template <int K>
__device__ __forceinline__ int exact_insert_rec(const SceneView &S, const TraceRec &rec, int pos, d3 o, d3 d,
                                                double t_min, KBufF<K> &kb, d3 wo, d3 wd) {
  const float tk = kb.t[K - 1];
  double t;
  bool flip;
  if (!exact_hit(rec, o, d, t_min, t, flip)) return 4;
  const float tf = (float)t;
  // beyond the k-th key, or at the key of a bound sentinel still in the k-th slot
  if (tf > tk || (tf == tk && kb.id[K - 1] == kIdMask)) return 12;
  const uint32_t id = (uint32_t)pos | (flip ? kFlipBit : 0u);
  bool tie = false;
#pragma unroll
  for (int j = 0; j < K; ++j) tie |= kb.t[j] == tf;
  if (!tie) {
    kinsert<K>(kb, tf, id);
    return 13;
  }
  return kinsert_tied<K>(S, kb, tf, t, id, wo, wd) ? 15 : 14;
}

template <int K>
__device__ __forceinline__ int exact_insert(const SceneView &S, int pos, d3 o, d3 d, double t_min, KBufF<K> &kb,
                                            d3 wo, d3 wd) {
  return exact_insert_rec<K>(S, S.rec[pos], pos, o, d, t_min, kb, wo, wd);
}

// Pre-filter, then exact test and insertion, of one surfel (bits as above; 0
// when the pre-filter rejects it).
template <int K>
__device__ __forceinline__ int test_surfel(const SceneView &S, int pos, d3 o, d3 d, const RayF &rf, double t_min,
                                           float t_min_f, KBufF<K> &kb, d3 wo, d3 wd) {
  const float tk = kb.t[K - 1];
  const float tk_up = tk < INFINITY ? next_up_f(tk) : INFINITY;
  if (!prefilter(S.filt[pos], rf, t_min_f, tk_up)) return 0;
  return exact_insert<K>(S, pos, o, d, t_min, kb, wo, wd);
}


template <int K>
__device__ __forceinline__ double kth(const KBufF<K> &b) { return (double)b.t[K - 1]; }

// Persistent traversal of a pool of `count` work items (rays): every lane
// holds one ray at a time, collects its k closest valid hits over all
// instances and stores them with wk.store; a wave refills its idle lanes from
// the shared counter *next once Work::kRefill of them are idle (or all are),
// taking at most its even share of `count` over the grid's waves at a time,
// so the rays of a wave need not finish together (see kPoolParts for the
// counters).  Work supplies
//   bool begin(int64_t item, d3 &o, d3 &d, const InstRec *&inst)  (false: nothing to trace)
//   void store(int64_t item, const KBufF<K> &kb)
//   float hint(int64_t item)  (a k-th distance the ray had before, or +inf)
//   static constexpr int kRefill; static constexpr bool kPrefetch (see the exact loop)
// Traversal of an instance runs in rounds of two phases (after Aila and
// Laine 2009, "while-while"): in the node phase a lane visits nodes, its hit
// leaves join its leaf queue and its nearest hit internal child is visited
// next (the others are pushed), while some lane that can still visit nodes
// has fewer than kLeafMin leaves queued; a lane pauses while its queue could
// not take a whole node's leaves.  The leaf phase then tests every queued
// leaf.  stk points at this lane's first LDS stack slot (stride kBlock,
// kStackL entries) and lq at its first leaf-queue slot (stride kBlock,
// kLeafQ entries).  A node's internal children occupy its first slots, so a
// stack entry names all the hit internal children of one visited node that
// are still to be visited: (descending << 31) | (child_base << 8) | slot
// mask, taken lowest slot first, or highest first when descending (the
// children are ordered along an axis; descending when the ray points down
// it).  The stack thus holds at most one entry per level above the current
// node, and the build guarantees that the hierarchy is shallow enough.
// Every lane leaves once the pool is empty and its last ray is stored.
//
// With a finite hint h (the k-th distance the forward call before a
// backward found for the same ray) the ray starts with its empty k-buffer slots keyed
// at B = the binary32 successor of h instead of +inf, so nodes and surfels
// beyond B are culled from the start; a hit keyed at B or beyond is not
// taken while such a bound sentinel holds the k-th slot.  If a sentinel
// still holds the k-th slot when the ray is done, fewer than k valid hits
// lie below B, and the ray is traced again from the start with +inf; else
// its k hits are exactly the k nearest (every hit below B was found).  So
// the result never depends on the hint, only the work does.
//
// When the host raises the abort word (P.abort, read every eighth refill of
// a wave), the wave stores every ray it holds or takes from then on with an
// empty hit list and traverses nothing more, so the kernel drains quickly
// and the buffers it hands on stay well formed; kStatusAborted is latched.

template <int K, class Work>
__device__ void trace_pool(const SceneView &S0, const TraceParams &P, const Work &wk, int64_t count, uint32_t *next,
                           int *stk, int *lq, uint32_t *status, int counter_base) {
  constexpr int kDone = (int)0x80000000;  // no node to visit
  const bool brute = (P.flags & LF_FLAG_BRUTE_FORCE) != 0;
  const float t_min_f = round_down_f(P.t_min);
  const float tlo = (float)(0.5 * P.t_min);
  const int lane = (int)(threadIdx.x & 63u);
  uint32_t c_rays = 0, c_nodes = 0, c_tests = 0, c_ins = 0, c_ties = 0, c_pass = 0, c_hits = 0, c_push = 0;
  uint32_t c_hinted = 0, c_retry = 0;
  bool bounded = false;  // the ray's k-buffer started from a finite bound
  int c_deep = 0;
  bool aborted = false;  // the host's abort word was seen (uniform over the wave)
  uint32_t refills = 0;
  auto count_test = [&](int r) {
    c_ins += r & 1;
    c_ties += (r >> 1) & 1;
    c_pass += (r >> 2) & 1;
    c_hits += r >> 3;
    ++c_tests;
  };
  int sp = 0;
  // next node to visit from the top entry: its lowest remaining slot; the
  // entry goes once its mask is empty
  auto pop = [&]() -> int {
    int *e = stk + (sp - 1) * kBlock;
    const uint32_t v = (uint32_t)*e, m = v & 0xffu;
    const int b = (v >> 31) ? 31 - __builtin_clz(m) : __builtin_ctz(m);
    const uint32_t rest = m & ~(1u << b);
    if (rest) *e = (int)((v & ~0xffu) | rest);
    else --sp;
    return (int)((v >> 8) & 0x7fffffu) + b;
  };
  SceneView S = S0;
  KBufF<K> kb;
  kinit<K>(kb, P.k);
  int64_t item = -1;
  bool live = false;       // this lane holds a ray
  bool exhausted = false;  // the pool is empty (uniform over the wave)
  int part = (int)(blockIdx.x % kPoolParts), tried = 0;  // the item range this wave draws from
  int ii = 0;              // the ray's current instance
  d3 o = mk(0, 0, 0), d = mk(0, 0, 1), oo = o, dd = d;
  RayF rf;
  make_rayf(oo, dd, 0.0, 0.0f, 0.0f, rf);
  int cur = kDone, qn = 0;
  // a wave takes at most its even share of the items at a time: when there are
  // fewer items than lanes in the grid, every wave gets a few rays instead of
  // a quarter of the waves holding 64 each, which shortens the longest wave
  const int64_t n_waves = (int64_t)gridDim.x * (kBlock / 64);
  const int cap = (int)min((int64_t)64, max((int64_t)1, (count + n_waves - 1) / n_waves));
  while (true) {
    // idle lanes take the next items, one counter update per wave
    if (!exhausted) {
      const unsigned long long idle = __ballot(!live);
      const int n_idle = __popcll(idle);
      if (n_idle >= Work::kRefill || (n_idle > 0 && !__any(live))) {
        const int leader = __ffsll((long long)idle) - 1;
        if (P.abort && !aborted && (refills++ & 7u) == 0 &&
            __hip_atomic_load(P.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u) {
          aborted = true;
          if (lane == leader) atomicOr(status, kStatusAborted);
          if (live) {  // the ray in flight is given up: stored with no hits
            kinit<K>(kb, P.k);
            wk.store(item, kb);
            live = false;
          }
          cur = kDone;
          qn = 0;
        }
        uint32_t base = 0;
        const int take = n_idle < cap ? n_idle : cap;
        if (lane == leader) base = atomicAdd(next + part, (uint32_t)take);
        base = (uint32_t)__shfl((int)base, leader);
        const int64_t lo = count * part / kPoolParts, hi = count * (part + 1) / kPoolParts;
        const int64_t first = lo + (int64_t)base;
        if (first + take >= hi) {  // this range is used up: move to the next one
          part = part + 1 == kPoolParts ? 0 : part + 1;
          exhausted = ++tried == kPoolParts;
        }
        if ((idle >> lane) & 1ull) {  // the lanes idle at the ballot (not those just given up)
          const int rk = __popcll(idle & ((1ull << lane) - 1ull));
          const int64_t it = first + rk;
          if (rk < take && it < hi) {
            item = it;
            live = wk.begin(item, o, d, S.inst);
            if (live && aborted) {
              kinit<K>(kb, P.k);
              wk.store(item, kb);
              live = false;
            } else if (live) {
              ++c_rays;
              kinit<K>(kb, P.k);
              const float h = wk.hint(item);
              bounded = h >= 0.0f && h < INFINITY;
              if (bounded) {
                const float bnd = next_up_f(h);
#pragma unroll
                for (int j = 0; j < K; ++j) kb.t[j] = kb.t[j] == INFINITY ? bnd : kb.t[j];
                ++c_hinted;
              }
              ii = -1;
              cur = kDone;
              qn = 0;
            }
          }
        }
      }
    }
    // a lane done with an instance moves to the next one its ray enters, or stores the ray's hits
    if (live && cur == kDone && qn == 0) {
      bool found = false;
      while (++ii < S.n_inst) {
        const InstRec &I = S.inst[ii];
        if (I.n <= 0) continue;
        double itn, itf;
        if (!slab64(o, d, I.lo, I.hi, itn, itf)) continue;
        if (itf < P.t_min) continue;
        if (itn > kth<K>(kb) * (1.0 + 1e-6)) continue;
        to_object(I, o, d, oo, dd);
        make_rayf(oo, dd, fmax(fabs(itf), fabs(itn)), I.omag, I.oext, rf);
        found = true;
        break;
      }
      if (!found && bounded && kb.id[K - 1] == kIdMask) {
        // fewer than k valid hits below the bound: trace the ray again without it
        bounded = false;
        ++c_retry;
        kinit<K>(kb, P.k);
        ii = -1;
        cur = kDone;
        qn = 0;
      } else if (!found) {
        wk.store(item, kb);
        live = false;
      } else if (brute) {  // every surfel of the instance; the next round moves on
        const InstRec &I = S.inst[ii];
        const int end = I.first + I.n <= S.n_rec ? I.first + I.n : S.n_rec;
        for (int pos = I.first < 0 ? 0 : I.first; pos < end; ++pos)
          count_test(test_surfel<K>(S, pos, oo, dd, rf, P.t_min, t_min_f, kb, o, d));
      } else {
        cur = S.inst[ii].root;
        sp = 0;
        if (cur < 0) {  // a one-surfel instance
          lq[0] = cur;
          qn = 1;
          cur = kDone;
        }
      }
    }
    if (!__any(live)) {
      if (exhausted) break;
      continue;
    }
    // node phase
    while (true) {
      const bool can = cur >= 0 && qn <= kLeafQ - kWide;
      if (!__any(can && qn < kLeafMin)) break;
      if (!can) continue;
      if (cur >= S.n_nodes) {  // never taken for a consistent hierarchy
        atomicOr(status, kStatusBvhCorrupt);
        cur = kDone;
        continue;
      }
      ++c_nodes;
      // the exact k-th distance is at most the successor of the k-th binary32 key
      const float tkf = kb.t[K - 1];
      const float thi = tkf < INFINITY ? next_up_f(tkf) * (1.0f + 1e-6f) : INFINITY;
      float ts[kWide];
      uint32_t ih, lh, im;
      int cbase, lbase;
      bool desc;
      visit_node(S.nodes + cur, rf, tlo, thi, ts, ih, lh, im, cbase, lbase, desc);
      // hit leaves join the queue, in slot order (leaf slots follow the
      // node's internal ones)
      const int leaf0 = lbase - __builtin_popcount(im);
      for (uint32_t m = lh; m; m &= m - 1u) lq[(qn++) * kBlock] = ~(leaf0 + __builtin_ctz(m));
      if (ih == 0) {
        cur = sp ? pop() : kDone;
        continue;
      }
      // the nearest hit internal child next, the others onto the stack as one entry
      int bj = __builtin_ctz(ih);
      if (ih & (ih - 1u)) {
        // entry distances are >= tlo >= 0, so their bit patterns order as
        // they do (a -0 orders last, which only changes the visiting order);
        // the low three bits carry the slot (ties within 8 ulps go to the lower)
        uint32_t key[kWide];
#pragma unroll
        for (int j = 0; j < kWide; ++j)
          key[j] = ((ih >> j) & 1u) ? (__float_as_uint(ts[j]) & ~7u) | (uint32_t)j : 0xffffffffu;
        static_assert(kWide == 8, "the reduction below is written for eight slots");
        bj = (int)(min(min(min(key[0], key[1]), min(key[2], key[3])), min(min(key[4], key[5]), min(key[6], key[7]))) & 7u);
      }
      const uint32_t rest = ih & ~(1u << bj);
      if (rest) {
        if (sp >= kStackL) {  // never taken for a hierarchy the build accepted
          atomicOr(status, kStatusOverflow);
          cur = kDone;
          continue;
        }
        stk[(sp++) * kBlock] = (int)((desc ? 0x80000000u : 0u) | ((uint32_t)cbase << 8) | rest);
        ++c_push;
        c_deep = sp > c_deep ? sp : c_deep;
      }
      cur = cbase + bj;
    }
    // the leaf phase runs at a raised wave priority: its burst of independent
    // record loads then issues ahead of the other wave's node-phase arithmetic
    // (1% faster traversal than without)
    __builtin_amdgcn_s_setprio(1);
    // leaf phase: the binary32 pre-filter over the whole queue, compacting the
    // survivors to its front, then their exact tests and insertions, so that
    // the rare exact path runs for many lanes at once
    {
      const float tk = kb.t[K - 1];
      const float tk_up = tk < INFINITY ? next_up_f(tk) : INFINITY;
      int np = 0;
      // four records in flight per step
      int j = 0;
      for (; j + 4 <= qn; j += 4) {
        int lv[4];
        FiltRec fr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          lv[u] = lq[(j + u) * kBlock];
          const bool okp = ~lv[u] < S.n_rec;
          if (!okp) atomicOr(status, kStatusBvhCorrupt);
          fr[u] = S.filt[okp ? ~lv[u] : 0];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const bool okp = ~lv[u] < S.n_rec;
          c_tests += okp ? 1u : 0u;
          if (okp && prefilter(fr[u], rf, t_min_f, tk_up)) lq[(np++) * kBlock] = lv[u];
        }
      }
      for (; j < qn; ++j) {
        const int leaf = lq[j * kBlock];
        if (~leaf >= S.n_rec) {  // never taken for a consistent hierarchy
          atomicOr(status, kStatusBvhCorrupt);
          continue;
        }
        ++c_tests;
        if (prefilter(S.filt[~leaf], rf, t_min_f, tk_up)) lq[(np++) * kBlock] = leaf;
      }
      // with Work::kPrefetch the next survivor's record is loaded while the
      // current one is tested (few lanes take this loop at once, so its
      // loads are exposed; worth it for secondary rays, not camera rays)
      // (the prefetched record lives only inside this block: a record held
      // over from an earlier round would stay live across the node phase
      // and be spilled to scratch there)
      auto count_exact = [&](int r) {
        c_ins += r & 1;
        c_ties += (r >> 1) & 1;
        ++c_pass;
        c_hits += r >> 3;
      };
      if constexpr (Work::kPrefetch) {
        if (np > 0) {
          TraceRec rnext = S.rec[~lq[0]];
          for (int j = 0; j < np; ++j) {
            const TraceRec rcur = rnext;
            if (j + 1 < np) rnext = S.rec[~lq[(j + 1) * kBlock]];
            count_exact(exact_insert_rec<K>(S, rcur, ~lq[j * kBlock], oo, dd, P.t_min, kb, o, d));
          }
        }
      } else {
        for (int j = 0; j < np; ++j) count_exact(exact_insert<K>(S, ~lq[j * kBlock], oo, dd, P.t_min, kb, o, d));
      }
    }
    __builtin_amdgcn_s_setprio(0);
    qn = 0;
  }
  if (P.counters && c_rays) {
    atomicAdd(P.counters + counter_base + 0, (unsigned long long)c_rays);
    atomicAdd(P.counters + counter_base + 1, (unsigned long long)c_nodes);
    atomicAdd(P.counters + counter_base + 2, (unsigned long long)c_tests);
    atomicAdd(P.counters + counter_base + 3, (unsigned long long)c_ins);
    atomicAdd(P.counters + 8 + counter_base / 4, (unsigned long long)c_ties);
    atomicAdd(P.counters + 10 + counter_base / 4, (unsigned long long)c_pass);
    atomicAdd(P.counters + 12 + counter_base / 4, (unsigned long long)c_hits);
    atomicAdd(P.counters + 14 + counter_base / 4, (unsigned long long)c_push);
    atomicMax(P.counters + 16 + counter_base / 4, (unsigned long long)c_deep);
    atomicAdd(P.counters + 18 + counter_base / 4, (unsigned long long)c_hinted);
    atomicAdd(P.counters + 20 + counter_base / 4, (unsigned long long)c_retry);
  }
}

// ------------------------------------------------------------ wave packets
// N dwords at a wave-uniform address, read through the scalar data cache
// (loads from the constant address space with a uniform address are scalar).
template <int N>
__device__ __forceinline__ void load_uniform(const void *p, uint32_t *out) {
  const __attribute__((address_space(4))) uint32_t *q = (const __attribute__((address_space(4))) uint32_t *)p;
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = q[i];
}

// OR of v over the 64 lanes of a wave whose lanes are all active: within
// each row of 16 lanes by DPP shifts, then across rows by the row
// broadcasts, so lane 63 holds the result.
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  int x = (int)v;
  x |= __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x |= __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x |= __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x |= __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x |= __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x |= __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane(x, 63);
}

// First item of range `part` of a pool split into kPoolParts ranges that
// start at multiples of 64 (one wave packet).
__device__ __forceinline__ int64_t packet_part_lo(int64_t count, int part) {
  return part >= kPoolParts ? count : ((count * part / kPoolParts) & ~(int64_t)63);
}

// Traversal of a pool of coherent rays as wave packets: a wave takes 64
// consecutive items (half a 16x8-pixel tile of camera rays: 8x8 pixels) and
// its lanes walk one node sequence together.  A node is visited when any
// lane's ray entered its box; every lane tests the node's child boxes with its
// own ray and its own current k-th distance, and a leaf any lane entered is
// tested by each lane that entered it, at once, so the node, filter record
// and trace record come through the scalar cache once per wave.  The next
// node is the hit internal child nearest along the first visiting lane's ray;
// the other hit internal children of all lanes are pushed as one entry on a
// per-wave LDS stack (wstk, kStackL entries) in the format of trace_pool and
// taken along the node's order axis.  Each lane still tests every surfel its own traversal would
// (it takes part in every node its ray entered) and some more, with the same
// pre-filter, exact test and insertion, so its k-buffer ends exactly as with
// trace_pool; hints, retries, the abort word and the counters follow
// trace_pool too.
template <int K, class Work>
__device__ void trace_packet(const SceneView &S0, const TraceParams &P, const Work &wk, int64_t count,
                             uint32_t *next, int *wstk, uint32_t *status, int counter_base) {
  constexpr int kDone = (int)0x80000000;
  const float t_min_f = round_down_f(P.t_min);
  const float tlo = (float)(0.5 * P.t_min);
  const int lane = (int)(threadIdx.x & 63u);
  uint32_t c_rays = 0, c_nodes = 0, c_tests = 0, c_ins = 0, c_ties = 0, c_pass = 0, c_hits = 0, c_push = 0;
  uint32_t c_hinted = 0, c_retry = 0;
  int c_deep = 0;
  auto count_exact = [&](int r) {
    c_ins += r & 1;
    c_ties += (r >> 1) & 1;
    ++c_pass;
    c_hits += r >> 3;
  };
  SceneView S = S0;
  int part = (int)(blockIdx.x % kPoolParts), tried = 0;
  bool aborted = false;
  uint32_t takes = 0;
  while (tried < kPoolParts) {
    if (P.abort && !aborted && (takes & 7u) == 0 &&
        __hip_atomic_load(P.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u) {
      aborted = true;
      if (lane == 0) atomicOr(status, kStatusAborted);
    }
    ++takes;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(next + part, 64u);
    base = (uint32_t)__shfl((int)base, 0);
    const int64_t hi = packet_part_lo(count, part + 1);
    const int64_t first = packet_part_lo(count, part) + (int64_t)base;
    if (first >= hi) {  // this range is used up: move to the next one
      part = part + 1 == kPoolParts ? 0 : part + 1;
      ++tried;
      continue;
    }
    const int64_t item = first + lane;
    d3 o = mk(0, 0, 0), d = mk(0, 0, 1);
    const InstRec *inst = S0.inst;
    const bool live = item < hi && wk.begin(item, o, d, inst);
    KBufF<K> kb;
    kinit<K>(kb, P.k);
    const unsigned long long lv = __ballot(live);
    if (lv == 0ull) continue;
    if (aborted) {  // stored with no hits, nothing traversed
      if (live) wk.store(item, kb);
      continue;
    }
    // the rays of a packet belong to one request: its instance records
    {
      const int ldr = __ffsll((long long)lv) - 1;
      const uint64_t ip = (uint64_t)inst;
      const uint32_t ilo = (uint32_t)__shfl((int)(uint32_t)ip, ldr), ihi = (uint32_t)__shfl((int)(uint32_t)(ip >> 32), ldr);
      S.inst = (const InstRec *)(((uint64_t)ihi << 32) | ilo);
    }
    bool bounded = false;
    if (live) {
      ++c_rays;
      const float h = wk.hint(item);
      bounded = h >= 0.0f && h < INFINITY;
      if (bounded) {
        const float bnd = next_up_f(h);
#pragma unroll
        for (int j = 0; j < K; ++j) kb.t[j] = kb.t[j] == INFINITY ? bnd : kb.t[j];
        ++c_hinted;
      }
    }
    bool act = live;
    for (int round = 0; round < 2; ++round) {
      if (!__any(act)) break;
      for (int ii = 0; ii < S.n_inst; ++ii) {
        const InstRec &I = S.inst[ii];
        if (I.n <= 0) continue;
        bool in = false;
        d3 oo = o, dd = d;
        RayF rf;
        if (act) {
          double itn, itf;
          in = slab64(o, d, I.lo, I.hi, itn, itf) && itf >= P.t_min && !(itn > kth<K>(kb) * (1.0 + 1e-6));
          if (in) {
            to_object(I, o, d, oo, dd);
            make_rayf(oo, dd, fmax(fabs(itf), fabs(itn)), I.omag, I.oext, rf);
          }
        }
        if (!__any(in)) continue;
        const int root = I.root;
        if (root < 0) {  // a one-surfel instance
          if (in) {
            const int r = test_surfel<K>(S, ~root, oo, dd, rf, P.t_min, t_min_f, kb, o, d);
            ++c_tests;
            if (r) count_exact(r);
          }
          continue;
        }
        int sp = 0, cur = root;
        while (true) {
          if (cur < 0 || cur >= S.n_nodes) {  // never taken for a consistent hierarchy
            if (lane == 0) atomicOr(status, kStatusBvhCorrupt);
            break;
          }
          uint32_t dw[kNodeDw];
          load_uniform<kNodeDw>(S.nodes + __builtin_amdgcn_readfirstlane(cur), dw);
          const uint32_t im = dw[3] >> 24;
          const int cbase = (int)dw[4], lbase = (int)dw[5];
          uint32_t ih = 0, lh = 0;
          bool desc = false;
          float tsv[kWide];
          if (in) {
            ++c_nodes;
            const float tkf = kb.t[K - 1];
            const float thi = tkf < INFINITY ? next_up_f(tkf) * (1.0f + 1e-6f) : INFINITY;
            uint32_t im2;
            int cb2, lb2;
            visit_node_dw(dw, rf, tlo, thi, tsv, ih, lh, im2, cb2, lb2, desc);
          }
          // the leaf and internal slots some lane entered (every lane of the wave runs this)
          const uint32_t hu = wave_or(lh | (ih << 8));
          const uint32_t iu = hu >> 8;
          // leaves, in slot order (leaf slots follow the internal ones)
          const int leaf0 = lbase - __builtin_popcount(im);
          for (uint32_t m = hu & 0xffu; m; m &= m - 1u) {
            const int j = __builtin_ctz(m);
            const int pos = __builtin_amdgcn_readfirstlane(leaf0 + j);
            if (pos < 0 || pos >= S.n_rec) {  // never taken for a consistent hierarchy
              if (lane == 0) atomicOr(status, kStatusBvhCorrupt);
              continue;
            }
            uint32_t fw[12];
            load_uniform<12>(S.filt + pos, fw);
            FiltRec fr;
            fr.v0 = make_float4(__uint_as_float(fw[0]), __uint_as_float(fw[1]), __uint_as_float(fw[2]),
                                __uint_as_float(fw[3]));
            fr.v1 = make_float4(__uint_as_float(fw[4]), __uint_as_float(fw[5]), __uint_as_float(fw[6]),
                                __uint_as_float(fw[7]));
            fr.v2 = make_float4(__uint_as_float(fw[8]), __uint_as_float(fw[9]), __uint_as_float(fw[10]),
                                __uint_as_float(fw[11]));
            bool pass = false;
            if ((lh >> j) & 1u) {
              ++c_tests;
              const float tk = kb.t[K - 1];
              pass = prefilter(fr, rf, t_min_f, tk < INFINITY ? next_up_f(tk) : INFINITY);
            }
            if (__any(pass)) {
              uint32_t rw[sizeof(TraceRec) / 4];
              load_uniform<sizeof(TraceRec) / 4>(S.rec + pos, rw);
              TraceRec rec;
              __builtin_memcpy(&rec, rw, sizeof rec);
              if (pass) count_exact(exact_insert_rec<K>(S, rec, pos, oo, dd, P.t_min, kb, o, d));
            }
          }
          if (iu == 0) {  // next from the stack's top entry
            cur = kDone;
            if (sp > 0) {
              const uint32_t v = (uint32_t)__builtin_amdgcn_readfirstlane(wstk[sp - 1]), mk8 = v & 0xffu;
              const int b = (v >> 31) ? 31 - __builtin_clz(mk8) : __builtin_ctz(mk8);
              const uint32_t rest = mk8 & ~(1u << b);
              if (rest) {
                if (lane == 0) wstk[sp - 1] = (int)((v & ~0xffu) | rest);
              } else {
                --sp;
              }
              cur = (int)((v >> 8) & 0x7fffffu) + b;
            }
            if (cur == kDone) break;
            continue;
          }
          // next, the child nearest along the first visiting lane's ray (its
          // own hit children keyed as in trace_pool); the others of every
          // lane onto the stack as one entry, taken along the node's axis in
          // the direction that lane's ray runs
          const int ldr = __ffsll((long long)__ballot(ih != 0u)) - 1;
          const bool dsc = __shfl((int)desc, ldr) != 0;
          int bl = dsc ? 31 - __builtin_clz(ih | 1u) : __builtin_ctz(ih | 0x100u);
          if (ih & (ih - 1u)) {
            uint32_t key[kWide];
#pragma unroll
            for (int j = 0; j < kWide; ++j)
              key[j] = ((ih >> j) & 1u) ? (__float_as_uint(tsv[j]) & ~7u) | (uint32_t)j : 0xffffffffu;
            bl = (int)(min(min(min(key[0], key[1]), min(key[2], key[3])), min(min(key[4], key[5]), min(key[6], key[7]))) & 7u);
          }
          const int bj = __shfl(bl, ldr);
          const uint32_t rest = iu & ~(1u << bj);
          if (rest) {
            if (sp >= kStackL) {  // never taken for a hierarchy the build accepted
              if (lane == 0) atomicOr(status, kStatusOverflow);
              break;
            }
            if (lane == 0) wstk[sp] = (int)((dsc ? 0x80000000u : 0u) | ((uint32_t)cbase << 8) | rest);
            ++sp;
            if (in) ++c_push;
            c_deep = sp > c_deep ? sp : c_deep;
          }
          cur = cbase + bj;
        }
      }
      // fewer than k valid hits below a ray's bound: it is traced again without it
      act = act && bounded && kb.id[K - 1] == kIdMask;
      if (act) {
        bounded = false;
        ++c_retry;
        kinit<K>(kb, P.k);
      }
    }
    if (live) wk.store(item, kb);
  }
  if (P.counters && c_rays) {
    atomicAdd(P.counters + counter_base + 0, (unsigned long long)c_rays);
    atomicAdd(P.counters + counter_base + 1, (unsigned long long)c_nodes);
    atomicAdd(P.counters + counter_base + 2, (unsigned long long)c_tests);
    atomicAdd(P.counters + counter_base + 3, (unsigned long long)c_ins);
    atomicAdd(P.counters + 8 + counter_base / 4, (unsigned long long)c_ties);
    atomicAdd(P.counters + 10 + counter_base / 4, (unsigned long long)c_pass);
    atomicAdd(P.counters + 12 + counter_base / 4, (unsigned long long)c_hits);
    atomicAdd(P.counters + 14 + counter_base / 4, (unsigned long long)c_push);
    atomicMax(P.counters + 16 + counter_base / 4, (unsigned long long)c_deep);
    atomicAdd(P.counters + 18 + counter_base / 4, (unsigned long long)c_hinted);
    atomicAdd(P.counters + 20 + counter_base / 4, (unsigned long long)c_retry);
  }
}

// ------------------------------------------------------------------ compositing
// Surface record of Eq. surface-record, in double precision.
struct Record {
  double A, T;
  d3 x, n, a;   // composited position, unit normal (0 on a miss), base colour
  double m, r, depth;
  double nl;    // length of the composited normal before renormalisation
  int nh;
};

__device__ __forceinline__ void store_record(const Record &rc, SurfRec *out) {
  SurfRec s;
  s.x[0] = rc.x.x; s.x[1] = rc.x.y; s.x[2] = rc.x.z;
  s.n[0] = rc.n.x; s.n[1] = rc.n.y; s.n[2] = rc.n.z;
  s.a[0] = rc.a.x; s.a[1] = rc.a.y; s.a[2] = rc.a.z;
  s.A = rc.A; s.T = rc.T; s.m = rc.m; s.r = rc.r; s.depth = rc.depth; s.nl = rc.nl;
  s.nh = rc.nh;
  s.pad = 0;
  *out = s;
}
__device__ __forceinline__ Record load_record(const SurfRec *in) {
  const SurfRec s = *in;
  Record rc;
  rc.x = mk(s.x[0], s.x[1], s.x[2]);
  rc.n = mk(s.n[0], s.n[1], s.n[2]);
  rc.a = mk(s.a[0], s.a[1], s.a[2]);
  rc.A = s.A; rc.T = s.T; rc.m = s.m; rc.r = s.r; rc.depth = s.depth; rc.nl = s.nl;
  rc.nh = s.nh;
  return rc;
}

// Exact quantities of one hit (leaf position pos) of the world ray (o, d):
// depth t, effective opacity (Eq. gaussian-response, capped) and the world
// normal turned towards the ray.  Uses the same arithmetic as exact_hit.
struct HitE {
  double t, at;
  d3 nw;
  int orig, inst;
};
__device__ __forceinline__ void hit_exact(const SceneView &S, const TraceParams &P, uint32_t id, d3 o, d3 d,
                                          HitE &h) {
  const int pos = (int)(id & kIdMask);
  const TraceRec r = S.rec[pos];
  h.inst = inst_of(S, pos);
  const InstRec &I = S.inst[h.inst];
  d3 oo, dd;
  to_object(I, o, d, oo, dd);
  d3 n = mk(r.n[0], r.n[1], r.n[2]);
  d3 mu = mk((double)r.mu[0], (double)r.mu[1], (double)r.mu[2]);
  h.t = plane_t(r, oo, plane_den(r, dd));
  d3 dl = (oo + h.t * dd) - mu;
  double xu = dl.x * r.a[0] + dl.y * r.a[1] + dl.z * r.a[2];
  double xv = dl.x * r.b[0] + dl.y * r.b[1] + dl.z * r.b[2];
  double raw = (double)S.opacity[r.orig] * exp(-0.5 * (xu * xu + xv * xv));
  h.at = raw > P.alpha_cap ? P.alpha_cap : raw;
  d3 nw = I.identity ? n : mul(I.R, n);
  h.nw = (id & kFlipBit) ? -nw : nw;
  h.orig = r.orig;
}

template <int K, class B>
__device__ void composite(const SceneView &S, const TraceParams &P, B &kb, d3 o, d3 d, Record &rc) {
  double T = 1.0, A = 0.0, Zt = 0.0, Zm = 0.0, Zr = 0.0;
  d3 Zx = mk(0, 0, 0), Zn = mk(0, 0, 0), Za = mk(0, 0, 0);
  int nh = 0;
  for (int it = 0; it < K; ++it) {
    const double t = (double)kb.t[0];
    const uint32_t id = kb.id[0];
    krotl<B, K>(kb);
    if (t > -INFINITY && t < INFINITY) {
      HitE h;
      hit_exact(S, P, id, o, d, h);
      const double w = T * h.at;
      A += w;
      Zt += w * h.t;
      Zx = Zx + w * (o + h.t * d);
      Zn = Zn + w * h.nw;
      Za = Za + w * ld3(S.albedo + 3 * (int64_t)h.orig);
      Zm += w * (double)S.metallic[h.orig];
      Zr += w * (double)S.roughness[h.orig];
      T *= (1.0 - h.at);
      ++nh;
    }
  }
  const double inv = 1.0 / (A + P.eps);
  rc.A = A;
  rc.T = T;
  rc.nh = nh;
  rc.depth = Zt * inv;
  rc.x = inv * Zx;
  rc.a = inv * Za;
  rc.m = Zm * inv;
  rc.r = Zr * inv;
  const d3 N = inv * Zn;
  const double nl = sqrt(dot(N, N));
  rc.nl = nl;
  rc.n = (nh > 0 && nl > 0.0) ? (1.0 / nl) * N : mk(0, 0, 0);
}

// hit list (surfel indices in order, -1 padded) for debugging/parity outputs
template <int K, class B>
__device__ void write_hits(const SceneView &S, const B &kb, int k, int32_t *out) {
  int j = 0;
#pragma unroll
  for (int e = 0; e < K; ++e)
    if (kb.t[e] > -INFINITY) {
      if (j < k) out[j] = kb.t[e] < INFINITY ? S.rec[kb.id[e] & kIdMask].orig : -1;
      ++j;
    }
}

// ------------------------------------------------------------------ environment
__device__ __forceinline__ void dir_to_uv(d3 w, double &u, double &v) {
  double th = acos(clampd(w.y, -1.0, 1.0));
  double ph = atan2(w.z, w.x);
  if (ph < 0.0) ph += 2.0 * kPi;
  u = ph / (2.0 * kPi);
  v = th / kPi;
}

struct Taps {
  int64_t i[4];
  double w[4];
};

// bilinear taps at (v*H - 1/2, u*W - 1/2); wraps in u, clamps in v
__device__ __forceinline__ void env_taps(const EnvView &E, d3 w, Taps &tp) {
  double u, v;
  dir_to_uv(w, u, v);
  double x = u * E.W - 0.5, y = v * E.H - 0.5;
  double x0 = floor(x), y0 = floor(y);
  double fx = x - x0, fy = y - y0;
  int64_t c0 = (((int64_t)x0) % E.W + E.W) % E.W, c1 = (c0 + 1) % E.W;
  int64_t r0 = (int64_t)y0, r1 = r0 + 1;
  r0 = r0 < 0 ? 0 : (r0 > E.H - 1 ? E.H - 1 : r0);
  r1 = r1 < 0 ? 0 : (r1 > E.H - 1 ? E.H - 1 : r1);
  tp.i[0] = r0 * E.W + c0; tp.w[0] = (1 - fy) * (1 - fx);
  tp.i[1] = r0 * E.W + c1; tp.w[1] = (1 - fy) * fx;
  tp.i[2] = r1 * E.W + c0; tp.w[2] = fy * (1 - fx);
  tp.i[3] = r1 * E.W + c1; tp.w[3] = fy * fx;
}

__device__ __forceinline__ d3 env_eval(const EnvView &E, d3 w) {
  Taps tp;
  env_taps(E, w, tp);
  d3 c = mk(0, 0, 0);
#pragma unroll
  for (int k = 0; k < 4; ++k) c = c + tp.w[k] * ld3(E.tex + 3 * tp.i[k]);
  return c;
}

__device__ __forceinline__ int cdf_search(const double *cdf, int n, double u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (cdf[mid + 1] > u) hi = mid; else lo = mid + 1;
  }
  return lo;
}

__device__ __forceinline__ double env_texel_pdf(const EnvView &E, int r, int c, double sin_th) {
  double total = E.scal[0];
  if (!(sin_th > 0.0) || !(total > 0.0) || !(E.rowsum[r] > 0.0)) return 0.0;
  double prow = E.roww[r] / total, pcol = E.lum[(int64_t)r * E.W + c] / E.rowsum[r];
  return prow * pcol * (double)E.H * (double)E.W / (2.0 * kPi * kPi * sin_th);
}

__device__ __forceinline__ double env_pdf(const EnvView &E, d3 w) {
  double u, v;
  dir_to_uv(w, u, v);
  int r = (int)floor(v * E.H), c = (int)floor(u * E.W);
  r = r > E.H - 1 ? E.H - 1 : r;
  c = c > E.W - 1 ? E.W - 1 : c;
  return env_texel_pdf(E, r, c, sin(v * kPi));
}

__device__ __forceinline__ double env_sample(const EnvView &E, double ua, double ub, d3 &w) {
  int r = cdf_search(E.cdf_row, E.H, ua);
  const double *cc = E.cdf_col + (int64_t)r * (E.W + 1);
  int c = cdf_search(cc, E.W, ub);
  double orow = (ua - E.cdf_row[r]) / (E.cdf_row[r + 1] - E.cdf_row[r]);
  double ocol = (ub - cc[c]) / (cc[c + 1] - cc[c]);
  double v = (r + orow) / E.H, u = (c + ocol) / E.W;
  double th = v * kPi, ph = u * 2.0 * kPi;
  double st = sin(th);
  w = mk(st * cos(ph), cos(th), st * sin(ph));
  return env_texel_pdf(E, r, c, st);
}

// ------------------------------------------------------------------ BRDF
// Lambert + GGX (Walter et al. 2007), separable Smith G1, Schlick Fresnel,
// F0 = 0.04 (1 - m) + a m, alpha_g = clamp(r, 0.08, 1)^2.
struct Spec {
  double ci, co, ch, vh, a2, D, G1i, G1o, P, reff;
  bool rclamp;
  d3 h;
};

__device__ __forceinline__ void spec_setup(d3 n, d3 wi, d3 wo, double r, Spec &s) {
  d3 h = wi + wo;
  s.h = (1.0 / sqrt(dot(h, h))) * h;
  s.ci = dot(n, wi);
  s.co = dot(n, wo);
  s.ch = dot(n, s.h);
  s.vh = dot(wo, s.h);
  s.rclamp = (r < 0.08 || r > 1.0);
  s.reff = clampd(r, 0.08, 1.0);
  double ag = s.reff * s.reff;
  s.a2 = ag * ag;
  double den = s.ch * s.ch * (s.a2 - 1.0) + 1.0;
  s.D = s.a2 / (kPi * den * den);
  s.G1i = 2.0 * s.ci / (s.ci + sqrt(s.a2 + (1.0 - s.a2) * s.ci * s.ci));
  s.G1o = 2.0 * s.co / (s.co + sqrt(s.a2 + (1.0 - s.a2) * s.co * s.co));
  double om = 1.0 - s.vh;
  s.P = om * om * om * om * om;
}

// f(wi, wo) (no cosine), zero below either hemisphere
__device__ __forceinline__ d3 brdf(d3 n, d3 wi, d3 wo, d3 a, double m, double r, uint32_t flags) {
  double ci = dot(n, wi), co = dot(n, wo);
  if (!(ci > 0.0) || !(co > 0.0)) return mk(0, 0, 0);
  d3 f = ((1.0 - m) * kInvPi) * a;
  if (flags & LF_FLAG_DIFFUSE_ONLY) return f;
  Spec s;
  spec_setup(n, wi, wo, r, s);
  double sc = s.D * s.G1i * s.G1o / (4.0 * ci * co);
  d3 F0 = mk(0.04 * (1.0 - m) + a.x * m, 0.04 * (1.0 - m) + a.y * m, 0.04 * (1.0 - m) + a.z * m);
  return f + sc * mk(F0.x + (1.0 - F0.x) * s.P, F0.y + (1.0 - F0.y) * s.P, F0.z + (1.0 - F0.z) * s.P);
}

// f(wi, wo) * (n . wi) for a frozen live sample (no hemisphere test)
__device__ __forceinline__ d3 fcos(d3 n, d3 wi, d3 wo, d3 a, double m, double r, uint32_t flags) {
  double ci = dot(n, wi);
  d3 f = ((1.0 - m) * kInvPi * ci) * a;
  if (flags & LF_FLAG_DIFFUSE_ONLY) return f;
  Spec s;
  spec_setup(n, wi, wo, r, s);
  double sc = s.D * s.G1i * s.G1o / (4.0 * s.co);
  d3 F0 = mk(0.04 * (1.0 - m) + a.x * m, 0.04 * (1.0 - m) + a.y * m, 0.04 * (1.0 - m) + a.z * m);
  return f + sc * mk(F0.x + (1.0 - F0.x) * s.P, F0.y + (1.0 - F0.y) * s.P, F0.z + (1.0 - F0.z) * s.P);
}

__device__ __forceinline__ double q_spec(d3 a, double m, uint32_t flags) {
  if (flags & LF_FLAG_DIFFUSE_ONLY) return 0.0;
  d3 F0 = mk(0.04 * (1.0 - m) + a.x * m, 0.04 * (1.0 - m) + a.y * m, 0.04 * (1.0 - m) + a.z * m);
  double lf = lum(F0), ld = lum((1.0 - m) * a);
  if (!(lf + ld > 0.0)) return 0.5;
  return clampd(lf / (lf + ld), 0.1, 0.9);
}

__device__ __forceinline__ double pdf_bsdf(d3 n, d3 wi, d3 wo, d3 a, double m, double r, uint32_t flags) {
  double ci = dot(n, wi);
  if (!(ci > 0.0)) return 0.0;
  double qs = q_spec(a, m, flags);
  double pc = ci * kInvPi;
  if (qs == 0.0) return pc;
  Spec s;
  spec_setup(n, wi, wo, r, s);
  double pg = (s.ci > 0.0 && s.vh > 0.0) ? s.D * s.ch / (4.0 * fabs(s.vh)) : 0.0;
  return qs * pg + (1.0 - qs) * pc;
}

// cosine (Malley) or GGX half-vector (Walter et al. 2007) direction
__device__ __forceinline__ d3 sample_lobe(d3 n, d3 wo, double r, bool spec, double u1, double u2) {
  d3 b1, b2;
  onb(n, b1, b2);
  double ph = 2.0 * kPi * u2;
  if (!spec) {
    double rr = sqrt(u1);
    return (rr * cos(ph)) * b1 + (rr * sin(ph)) * b2 + sqrt(1.0 - u1) * n;
  }
  double reff = clampd(r, 0.08, 1.0), ag = reff * reff, a2 = ag * ag;
  double c2 = (1.0 - u1) / (1.0 + (a2 - 1.0) * u1);
  double ct = sqrt(c2), st = sqrt(1.0 - c2 < 0.0 ? 0.0 : 1.0 - c2);
  d3 h = (st * cos(ph)) * b1 + (st * sin(ph)) * b2 + ct * n;
  double oh = dot(wo, h);
  return (2.0 * oh) * h - wo;
}

// The uniform of (ray, sample, dim) from the sampler the flags select.
__device__ __forceinline__ double draw(const TraceParams &P, int64_t ray, int s, uint32_t dim) {
  return (P.flags & LF_FLAG_SOBOL) ? sobol_u(P.seed, (uint64_t)ray, (uint64_t)s, dim)
                                   : urand(P.seed, (uint64_t)ray, (uint64_t)s, dim);
}

// Secondary-ray slots per primary ray: S, or 2S in the two-ray form.
__device__ __forceinline__ int n_slots(const TraceParams &P) { return P.spp * ((P.flags & LF_FLAG_NEE) ? 2 : 1); }

// Primary direction of slot j and its frozen weights (Eq. path-estimator,
// power heuristic); false for a dead slot.  One-ray form (slot = sample s):
// technique by u0 with probabilities (c_env, 1 - c_env),
// K = c_t p_t / ((c_e p_e)^2 + (c_b p_b)^2), tw = 1.  Two-ray form (Sec. 4.2;
// path sample s = j/2, both techniques always drawn): slot 2s samples the
// environment (dims 9, 10) with K = p_e / (p_e^2 + p_b^2), tw = 1; slot 2s+1
// samples the cosine/GGX mixture (dims 1-3) with K = 1/p_b, and its escaping
// term T2 E(w) carries tw = p_b^2 / (p_e^2 + p_b^2) while the indirect term
// at its secondary hit is not MIS-weighted.
__device__ __forceinline__ bool primary_slot(const EnvView &E, const TraceParams &P, const Record &rc, d3 wo,
                                             int64_t ray, int j, double c_env, d3 &w, double &K, double &tw) {
  if (rc.nh == 0) return false;
  const bool nee = (P.flags & LF_FLAG_NEE) != 0;
  const int s = nee ? j >> 1 : j;
  const int kind = nee ? 1 + (j & 1) : 0;  // 0 one-ray, 1 next-event, 2 continuation
  bool use_env;
  if (kind == 0) {
    use_env = draw(P, ray, s, 0) < c_env;
  } else {
    use_env = kind == 1;
    if (use_env && !(c_env > 0.0)) return false;
  }
  double pe = 0.0, pb;
  if (use_env) {
    const uint32_t da = kind == 1 ? 9u : 2u;
    pe = env_sample(E, draw(P, ray, s, da), draw(P, ray, s, da + 1), w);
  } else {
    const double u1 = draw(P, ray, s, 1);
    const double qs = q_spec(rc.a, rc.m, P.flags);
    w = sample_lobe(rc.n, wo, rc.r, u1 < qs, draw(P, ray, s, 2), draw(P, ray, s, 3));
  }
  if (!(dot(rc.n, w) > 0.0)) return false;
  pb = pdf_bsdf(rc.n, w, wo, rc.a, rc.m, rc.r, P.flags);
  if (!use_env) pe = c_env > 0.0 ? env_pdf(E, w) : 0.0;
  const double pt = use_env ? pe : pb;
  if (!(pt > 0.0)) return false;
  tw = 1.0;
  if (kind == 0) {
    const double c_bsdf = 1.0 - c_env;
    const double ct = use_env ? c_env : c_bsdf;
    const double den = (c_env * pe) * (c_env * pe) + (c_bsdf * pb) * (c_bsdf * pb);
    K = ct * pt / den;
  } else if (kind == 1) {
    K = pe / (pe * pe + pb * pb);
  } else {
    K = 1.0 / pb;
    tw = pb * pb / (pe * pe + pb * pb);
  }
  return true;
}

// Frozen coefficients of the two unshadowed environment samples at a
// secondary record (two-sample power heuristic).
struct SecCoef {
  d3 ce, cb, we, wb;
  bool has_e, has_b;
};

__device__ __forceinline__ void secondary_coefs(const EnvView &E, const TraceParams &P, const Record &r2, d3 w,
                                                int64_t ray, int s, double c_env, SecCoef &sc) {
  sc.ce = mk(0, 0, 0);
  sc.cb = mk(0, 0, 0);
  sc.we = mk(0, 0, 0);
  sc.wb = mk(0, 0, 0);
  sc.has_e = sc.has_b = false;
  if (r2.nh == 0) return;
  d3 wo2 = -w;
  if (c_env > 0.0) {
    double u4 = draw(P, ray, s, 4), u5 = draw(P, ray, s, 5);
    double pe2 = env_sample(E, u4, u5, sc.we);
    double c2 = dot(r2.n, sc.we);
    if (c2 > 0.0 && pe2 > 0.0) {
      d3 f2 = brdf(r2.n, sc.we, wo2, r2.a, r2.m, r2.r, P.flags);
      double pb2 = pdf_bsdf(r2.n, sc.we, wo2, r2.a, r2.m, r2.r, P.flags);
      double wgt = pe2 * pe2 / (pe2 * pe2 + pb2 * pb2);
      sc.ce = (r2.A * wgt * c2 / pe2) * f2;
      sc.has_e = true;
    }
  }
  double u6 = draw(P, ray, s, 6), u7 = draw(P, ray, s, 7), u8 = draw(P, ray, s, 8);
  double qs2 = q_spec(r2.a, r2.m, P.flags);
  sc.wb = sample_lobe(r2.n, wo2, r2.r, u6 < qs2, u7, u8);
  double c2 = dot(r2.n, sc.wb);
  if (c2 > 0.0) {
    double pb2 = pdf_bsdf(r2.n, sc.wb, wo2, r2.a, r2.m, r2.r, P.flags);
    double pe2 = c_env > 0.0 ? env_pdf(E, sc.wb) : 0.0;
    if (pb2 > 0.0) {
      d3 f2 = brdf(r2.n, sc.wb, wo2, r2.a, r2.m, r2.r, P.flags);
      double wgt = pb2 * pb2 / (pe2 * pe2 + pb2 * pb2);
      sc.cb = (r2.A * wgt * c2 / pb2) * f2;
      sc.has_b = true;
    }
  }
}

// Wave-aggregated append: one atomic per wave, slots in lane order.
template <class T>
__device__ __forceinline__ void wave_append(bool live, const T &e, T *queue, uint32_t *count) {
  uint64_t mask = __ballot(live);
  if (mask == 0) return;
  const int lane = __lane_id();
  const int leader = __ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(mask));
  base = __shfl(base, leader);
  if (live) {
    uint64_t lt = lane ? ((~0ull) >> (64 - lane)) : 0ull;
    queue[base + (uint32_t)__popcll(mask & lt)] = e;
  }
}

}  // namespace lf

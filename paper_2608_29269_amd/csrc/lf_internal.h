// lf_internal.h -- data layouts shared by the host runtime and the gfx950
// kernels of liblightfuse.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lightfuse.h"

namespace lf {

constexpr int kBlock = 128;       // threads per block of the tracing kernels (2 wave64)
constexpr int kWide = 8;          // children per traversal node
constexpr int kStackL = 24;       // traversal stack entries per lane, in LDS (12 KB per block): one per
                                  // level above the current node, so hierarchies of up to kStackL + 1 levels
constexpr int kMaxWideNodes = 1 << 23;  // a stack entry holds a node index in 23 bits
constexpr int kLeafQ = 56;        // leaf-queue entries per lane (LDS, 28 KB per block)
constexpr int kLeafMin = 12;       // the node phase goes on while a lane that can visit nodes has fewer queued
// Persistent traversal splits its items into kPoolParts contiguous ranges
// with one counter each; a block starts on range blockIdx % kPoolParts, so
// with round-robin dispatch of blocks over the eight XCDs each XCD's L2
// serves one compact range of (sorted) rays at a time; a wave whose range is
// used up moves on to the next.
constexpr int kPoolParts = 8;
constexpr int kMaxInst = 64;      // background + up to 63 objects
constexpr uint32_t kFlipBit = 0x80000000u;
constexpr uint32_t kIdMask = 0x7fffffffu;

// Status bits latched on the device.
constexpr uint32_t kStatusOverflow = 1u;
constexpr uint32_t kStatusBadTransform = 2u;
constexpr uint32_t kStatusBvhCorrupt = 4u;   // an index read from the hierarchy was out of range
constexpr uint32_t kStatusAborted = 8u;      // the host's abort word cut the traversal short

// Per-surfel trace record, stored in leaf (Morton) order: everything the
// ray-surfel decision needs, in double precision so that hit sets and their
// (t, index) order are decided exactly as in FP64 arithmetic.  96 bytes.
struct alignas(16) TraceRec {
  double n[3];      // object-space unit normal (third frame column)
  double a[3];      // t_u / s_u
  double b[3];      // t_v / s_v
  float mu[3];      // object-space centre (exact in double)
  int32_t orig;     // surfel index in the caller's arrays
  double rho2max;   // min(sigma^2, 2 ln(alpha / alpha_min)): support and threshold as one predicate
};
static_assert(sizeof(TraceRec) == 96, "TraceRec layout");

// Binary32 copy of the trace record used by the pre-filter, 48 bytes (the
// plane normal is recomputed from a x b, which keeps more records in cache):
// v0 = (a.x, a.y, a.z, mu.x), v1 = (b.x, b.y, b.z, mu.y),
// v2 = (mu.z, rho2max rounded up, sqrt(rho2max) rounded up, max(|a|,|b|) rounded up).
struct alignas(16) FiltRec {
  float4 v0, v1, v2;
};
static_assert(sizeof(FiltRec) == 48, "FiltRec layout");

// Binary BVH node holding both children's boxes (one 64-byte fetch per
// visited node).  Child >= 0: internal node index (global); < 0: ~leaf
// position (global).
struct alignas(16) BNode {
  float lo0[3], hi0[3];
  float lo1[3], hi1[3];
  int32_t c0, c1;
  int32_t pad0, pad1;
};
static_assert(sizeof(BNode) == 64, "BNode layout");

// Traversal node with up to kWide children whose boxes are quantised to 8
// bits per plane in a per-node frame (compressed wide BVH, Ylitie et al.
// 2017): on axis a the plane of code q lies at fmaf(q, 2^e[a], p[a]) in
// binary32.  The build picks every lower code so that this value is at or
// below the child's lower bound and every upper code so that it is at or
// above its upper bound, so a decoded box always contains the box it stands
// for.  Slots 0..m-1 are occupied, internal children first: slot i < n_int
// (n_int = popcount(imask), imask = (1 << n_int) - 1) holds node
// child_base + i, slot i >= n_int holds leaf (surfel position)
// leaf_base + i - n_int.  The internal children are ordered by their box
// centres along axis (vmask >> 8) & 3.  80 bytes for kWide = 8.
struct alignas(16) QNode {
  float p[3];
  int8_t e[3];
  uint8_t imask;          // bit i: slot i holds an internal node (the first slots)
  int32_t child_base;
  int32_t leaf_base;
  uint32_t vmask;         // bit i < 8: slot i holds a child with a non-empty box; bits 8-9: order axis
  uint8_t q[6][kWide];    // lower x, y, z then upper x, y, z codes per slot
};
static_assert(sizeof(QNode) == (kWide == 8 ? 80 : 64), "QNode layout");
static_assert(kWide == 4 || kWide == 8, "traversal width");

// Build-time description of one traversal node, kept for every refit: the
// binary (parent << 1 | side) under which each slot's box is stored (-1:
// unoccupied), and the node's child and leaf bases.
struct alignas(16) WideInfo {
  int32_t src[kWide];
  int32_t child_base, leaf_base;
  uint32_t imask, n_slots;
};

// One instance of the two-level scene for the current state: background
// (identity) or an object with its rigid transform.
struct alignas(16) InstRec {
  double R[9];      // object -> world rotation (orthonormalised), row-major
  double t[3];      // object -> world translation
  double lo[3], hi[3];  // world-space bounds of the instance (conservative)
  int32_t root;     // root traversal node (>= 0), ~leaf (< 0) for one surfel; unused if n == 0
  int32_t identity; // 1: background (no transform)
  int32_t first;    // first surfel index / leaf position of the instance
  int32_t n;        // surfel count
  float omag;       // largest |coordinate| of the object-space bounds of the instance's surfels
  float oext;       // their largest extent
  int32_t pad[2];
};

struct SceneView {
  const TraceRec *rec;   // [N] leaf order
  const FiltRec *filt;   // [N] leaf order
  const QNode *nodes;    // traversal nodes of all instances
  const InstRec *inst;   // [n_inst]
  int32_t n_inst;
  int32_t n_rec;         // N
  int32_t n_nodes;       // traversal nodes over all instances
  const float *mu, *q, *scale, *opacity, *albedo, *roughness, *metallic;  // caller arrays (orig index)
};

struct TraceParams {
  int32_t k, spp;
  uint64_t seed;
  double alpha_min, alpha_cap, sig2, eps, t_min, sec_off;
  uint32_t flags;
  unsigned long long *counters;  // [LF_NUM_COUNTERS] traversal counters when LF_FLAG_COUNT is set
  const uint32_t *abort;         // device view of the host's abort word (fine-grained), or null
};

struct EnvView {
  const float *tex;        // [H,W,3]
  int32_t H, W;
  const double *cdf_row;   // [H+1]
  const double *cdf_col;   // [H,(W+1)]
  const double *lum;       // [H,W]  max(lum, 0)
  const double *rowsum;    // [H]
  const double *roww;      // [H]
  const double *scal;      // [0] total weight, [1] c_env
};

struct CamArgs {
  float pose[LF_MAX_CAMERAS][12];
  float tan_half[LF_MAX_CAMERAS];
  int32_t w[LF_MAX_CAMERAS], h[LF_MAX_CAMERAS];
  int64_t first[LF_MAX_CAMERAS + 1];  // ray-id offsets
  int64_t tiles[LF_MAX_CAMERAS + 1];  // offsets of each camera's 16x8-pixel tiles
  int32_t n_cams;
};

struct RaySource {
  const float *o, *d;     // explicit rays, or NULL to use cams
  int64_t n;
  const CamArgs *cams;    // device copy of the cameras
};

// Secondary ray queued by the primary pass (one per live slot).
struct alignas(16) SecEntry {
  double o[3];
  double w[3];
  float thr[3];        // K * f * cos * A / S of the primary slot
  int32_t ray;         // primary ray id
  int32_t s;           // slot: the sample, or 2 * sample + (0 next-event, 1 continuation) in the two-ray form
  float tw;            // weight of the escaping term T2 E(w) (its MIS weight in the two-ray form, else 1)
};
static_assert(sizeof(SecEntry) == 80, "SecEntry layout");

// Composited surface record of one ray (Eq. surface-record), double
// precision, written by the tracing passes and read by the shading passes.
struct alignas(16) SurfRec {
  double x[3], n[3], a[3];
  double A, T, m, r, depth, nl;
  int32_t nh, pad;
};
static_assert(sizeof(SurfRec) == 128, "SurfRec layout");

// Seeds of the compositing adjoint of one ray (from the shading adjoint).
struct alignas(16) AdjSeed {
  float gA, gT, gZt, gZm, gZr;
  float gZn[3], gZa[3];
  float T;
  float pad[4];
};
static_assert(sizeof(AdjSeed) == 64, "AdjSeed layout");

// Frozen secondary quantities of one (ray, sample) for the replayed backward.
struct alignas(16) SecFrozen {
  float T2;
  float ce[3];   // A2 x frozen factors of the environment sample at the secondary record
  float cb[3];   // A2 x frozen factors of the BSDF sample at the secondary record
  float we[3];
  float wb[3];
  uint32_t has;  // bit0: env sample, bit1: BSDF sample
};
static_assert(sizeof(SecFrozen) == 64, "SecFrozen layout");

// ---- continuous batching: several requests share one wavefront pass.
// The batch is a list of 128-ray chunks; every chunk belongs to one request
// (its slot) and is one 16x8-pixel tile of that request's image (8x8 per
// wave64), lanes outside the image idle.
constexpr int kChunk = kBlock;

struct alignas(16) ChunkDesc {
  int32_t slot;    // server slot of the request
  int32_t pad;
  int64_t tile;    // tile index within the request's image (row-major over 16x8 tiles)
};
static_assert(sizeof(ChunkDesc) == 16, "ChunkDesc layout");

// What differs between the requests of a batch.
struct alignas(16) BatchSlot {
  const InstRec *inst;      // [n_inst] this request's instance records
  const double *bounds;     // [6] world bounds of its instances
  const CamArgs *cam;       // camera 0 generates the request's rays
  EnvView E;                // its environment map and sampling tables
  float *radiance, *depth, *normal, *alpha;  // its outputs, indexed by ray id
  uint64_t seed;
  int32_t spp;
  int32_t pad;
};

}  // namespace lf

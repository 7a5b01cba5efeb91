// lf_backward.hip -- reverse mode of the forward path under path replay
// (Sec. 3.3, PRB paragraph).  Per primary ray the hit list is recomputed by a
// fresh traversal (never stored), the surface record is recomposited, the S
// sampling decisions are regenerated from the seed and the frozen secondary
// quantities are read from the replay pass.  The adjoint then runs through
// the primary BRDF and every environment texel read, through the normal
// normalisation and the front-to-back compositing (suffix sums over the hit
// list), and through plane intersection and effective opacity into
// (mu, q, s, alpha, a, m, r), accumulated with float atomics.
#include "lf_device.h"
#include "lf_kernels.h"

namespace lf {

namespace {

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Per-block accumulation of environment-texel gradients in an LDS table
// keyed by texel (open addressing, a few probes), flushed with one atomic per
// texel and channel; a texel that finds no slot goes to device memory
// directly.  The background of neighbouring pixels meets the same few
// texels, and so do importance-sampled directions where the map is bright,
// so this replaces most device-scope atomics on shared addresses.  Other
// texels a block rarely meets twice: they go to device memory directly and
// leave the table's slots to the ones that repeat.
constexpr int kEnvAggBits = 11;
constexpr int kEnvAggSlots = 1 << kEnvAggBits;  // 32 KB of LDS per block with the values
constexpr int kEnvAggProbes = 8;
constexpr double kEnvHot = 16.0;  // pooled: luminance at least this many times the map's mean

struct BlockEnvTable {
  int *key;     // [kEnvAggSlots], -1 when free
  float *val;   // [3][kEnvAggSlots]
  float *genv;  // [H, W, 3] in device memory
  const double *lum;  // [H, W] clamped texel luminance
  double lum_hot;     // texels at or above it are pooled
  // repeats: the caller expects the texel again within the block
  __device__ void add(int texel, double dx, double dy, double dz, bool repeats) {
    const float gx = (float)dx, gy = (float)dy, gz = (float)dz;
    const uint32_t h = (uint32_t)texel * 2654435761u;
    const int probes = repeats || lum[texel] >= lum_hot ? kEnvAggProbes : 0;
#pragma unroll 1
    for (int p = 0; p < probes; ++p) {
      const int slot = (int)((h >> (32 - kEnvAggBits)) + (uint32_t)p) & (kEnvAggSlots - 1);
      const int k = atomicCAS(key + slot, -1, texel);
      if (k == -1 || k == texel) {
        atomicAdd(val + slot, gx);
        atomicAdd(val + kEnvAggSlots + slot, gy);
        atomicAdd(val + 2 * kEnvAggSlots + slot, gz);
        return;
      }
    }
    atomicAdd(genv + 3 * texel + 0, gx);
    atomicAdd(genv + 3 * texel + 1, gy);
    atomicAdd(genv + 3 * texel + 2, gz);
  }
};

// Order-fixed accumulation (LF_FLAG_DETERMINISTIC): every contribution is
// written as a record at a position fixed by its ray (or work item) and its
// rank within that ray, keyed by its target (environment texel or surfel);
// the records are then sorted by key with a stable radix sort, so each
// target's records stay in position order, and every target's sum is taken
// in binary64 in that order and rounded once.  The result does not depend
// on scheduling.
struct EnvRecords {
  uint64_t *key;  // [rays * cap] texel of each record
  int32_t *idx;   // [rays * cap] the record's own position (the sort's payload)
  double *val;    // [rays * cap][3]
  int64_t base;   // first record of this ray
  int n;          // records written so far
  __device__ void add(int texel, double gx, double gy, double gz, bool) {
    const int64_t r = base + n++;
    key[r] = (uint64_t)texel;
    idx[r] = (int32_t)r;
    val[3 * r] = gx;
    val[3 * r + 1] = gy;
    val[3 * r + 2] = gz;
  }
};

template <class EAcc>
__device__ __forceinline__ void env_scatter(const EnvView &E, EAcc &acc, d3 w, d3 g, bool repeats) {
  Taps tp;
  env_taps(E, w, tp);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (tp.w[k] == 0.0) continue;
    acc.add((int)tp.i[k], tp.w[k] * g.x, tp.w[k] * g.y, tp.w[k] * g.z, repeats);
  }
}

// reverse of fcos(): accumulates into gn (unit normal), ga, gm, gr
__device__ __forceinline__ void fcos_bwd(d3 n, d3 wi, d3 wo, d3 a, double m, double r, uint32_t flags, d3 gfc,
                                         d3 &gn, d3 &ga, double &gm, double &gr) {
  double ci = dot(n, wi);
  ga = ga + ((1.0 - m) * kInvPi * ci) * gfc;
  gm += -(gfc.x * a.x + gfc.y * a.y + gfc.z * a.z) * kInvPi * ci;
  double gci = (gfc.x * a.x + gfc.y * a.y + gfc.z * a.z) * (1.0 - m) * kInvPi;
  if (!(flags & LF_FLAG_DIFFUSE_ONLY)) {
    Spec s;
    spec_setup(n, wi, wo, r, s);
    double a2 = s.a2;
    double sc = s.D * s.G1i * s.G1o / (4.0 * s.co);
    const double ac[3] = {a.x, a.y, a.z}, gc[3] = {gfc.x, gfc.y, gfc.z};
    double gsc = 0.0, gac[3];
    for (int c = 0; c < 3; ++c) {
      double F0 = 0.04 * (1.0 - m) + ac[c] * m;
      gsc += gc[c] * (F0 + (1.0 - F0) * s.P);
      double gF0 = gc[c] * sc * (1.0 - s.P);
      gac[c] = gF0 * m;
      gm += gF0 * (ac[c] - 0.04);
    }
    ga = ga + mk(gac[0], gac[1], gac[2]);
    double u = s.ch * s.ch * (a2 - 1.0) + 1.0;
    double dD_dch = -4.0 * a2 * s.ch * (a2 - 1.0) / (kPi * u * u * u);
    double dD_da2 = (u - 2.0 * a2 * s.ch * s.ch) / (kPi * u * u * u);
    double si = sqrt(a2 + (1.0 - a2) * s.ci * s.ci), so = sqrt(a2 + (1.0 - a2) * s.co * s.co);
    double dG1i_dc = 2.0 * a2 / (si * (s.ci + si) * (s.ci + si));
    double dG1o_dc = 2.0 * a2 / (so * (s.co + so) * (s.co + so));
    double dG1i_da2 = -s.ci * (1.0 - s.ci * s.ci) / (si * (s.ci + si) * (s.ci + si));
    double dG1o_da2 = -s.co * (1.0 - s.co * s.co) / (so * (s.co + so) * (s.co + so));
    double gch = gsc * dD_dch * s.G1i * s.G1o / (4.0 * s.co);
    gci += gsc * s.D * dG1i_dc * s.G1o / (4.0 * s.co);
    double gco = gsc * s.D * s.G1i * (dG1o_dc * s.co - s.G1o) / (4.0 * s.co * s.co);
    double ga2 = gsc * (dD_da2 * s.G1i * s.G1o + s.D * (dG1i_da2 * s.G1o + s.G1i * dG1o_da2)) / (4.0 * s.co);
    if (!s.rclamp) gr += ga2 * 4.0 * s.reff * s.reff * s.reff;
    gn = gn + gco * wo + gch * s.h;
  }
  gn = gn + gci * wi;
}

// ---------------------------------------------------------------- shading adjoint
// Per primary ray: reverse of L = A * (1/S) sum_j F_j + T * E(d) over the
// slots j with F_j = K_j f(w_j) (n.w_j) (tw_j T2 E(w_j) + ce E(w_e) + cb E(w_b))
// (the replay stores tw_j T2 as its frozen transmittance); environment
// gradients are scattered here, and the adjoints of the surface record are
// reduced to the seeds of the compositing adjoint.
template <class EAcc>
__device__ __forceinline__ void adj_shade_ray(const RenderArgs &a, const GradArgs &G, int64_t ray, EAcc &acc) {
  const TraceParams &P = a.P;
  const int S = P.spp, J = n_slots(P);
  float of[3], df[3];
  load_ray(a.rays, ray, of, df);
  const d3 d = mk(df[0], df[1], df[2]);
  const Record rc = load_record(a.rec1 + ray);
  const d3 gL = G.d_radiance ? ld3(G.d_radiance + 3 * ray) : mk(0, 0, 0);
  const double gdepth = G.d_depth ? (double)G.d_depth[ray] : 0.0;
  d3 gn = G.d_normal ? ld3(G.d_normal + 3 * ray) : mk(0, 0, 0);
  double gA = G.d_alpha ? (double)G.d_alpha[ray] : 0.0, gT = 0.0;
  if (!(P.flags & LF_FLAG_NO_BACKGROUND)) {
    const d3 Ed = env_eval(a.E, d);
    gT += dot(gL, Ed);
    env_scatter(a.E, acc, d, rc.T * gL, true);
  }
  AdjSeed sd = {};
  sd.T = (float)rc.T;
  if (rc.nh == 0) {
    a.seeds[ray] = sd;
    return;
  }
  const double c_env = a.E.scal[1];
  const bool trace2 = !(P.flags & LF_FLAG_NO_SECONDARY);
  const d3 wo = -d;
  d3 ga = mk(0, 0, 0);
  double gm = 0.0, gr = 0.0;
  for (int s = 0; s < J; ++s) {
    d3 w;
    double K_, tw = 1.0;
    if (!primary_slot(a.E, P, rc, wo, ray, s, c_env, w, K_, tw)) continue;
    double T2 = tw;
    d3 ce = mk(0, 0, 0), cb = mk(0, 0, 0), we = mk(0, 0, 1), wb = mk(0, 0, 1);
    uint32_t has = 0;
    if (trace2) {
      const SecFrozen f = a.frozen[ray * a.spp_stride + s];
      T2 = f.T2;
      ce = ld3(f.ce); cb = ld3(f.cb); we = ld3(f.we); wb = ld3(f.wb);
      has = f.has;
    }
    const d3 E = env_eval(a.E, w);
    d3 Lin = T2 * E;
    if (has & 1u) { const d3 Ee = env_eval(a.E, we); Lin = Lin + mk(ce.x * Ee.x, ce.y * Ee.y, ce.z * Ee.z); }
    if (has & 2u) { const d3 Eb = env_eval(a.E, wb); Lin = Lin + mk(cb.x * Eb.x, cb.y * Eb.y, cb.z * Eb.z); }
    const d3 fc = fcos(rc.n, w, wo, rc.a, rc.m, rc.r, P.flags);
    const d3 Ls = K_ * mk(fc.x * Lin.x, fc.y * Lin.y, fc.z * Lin.z);
    gA += dot(gL, Ls) / S;
    const d3 gF = (rc.A / S) * gL;
    const d3 gfc = K_ * mk(gF.x * Lin.x, gF.y * Lin.y, gF.z * Lin.z);
    const d3 gLin = K_ * mk(gF.x * fc.x, gF.y * fc.y, gF.z * fc.z);
    env_scatter(a.E, acc, w, T2 * gLin, false);
    if (has & 1u) env_scatter(a.E, acc, we, mk(ce.x * gLin.x, ce.y * gLin.y, ce.z * gLin.z), false);
    if (has & 2u) env_scatter(a.E, acc, wb, mk(cb.x * gLin.x, cb.y * gLin.y, cb.z * gLin.z), false);
    fcos_bwd(rc.n, w, wo, rc.a, rc.m, rc.r, P.flags, gfc, gn, ga, gm, gr);
  }
  // normalisation n_bar = N / |N|; z_bar = Z * inv with inv = 1/(A + eps)
  const double inv = 1.0 / (rc.A + P.eps);
  d3 gN = mk(0, 0, 0);
  if (rc.nl > 0.0) gN = (1.0 / rc.nl) * (gn - dot(rc.n, gn) * rc.n);
  const d3 N = rc.nl * rc.n;
  gA += -inv * (gdepth * rc.depth + dot(gN, N) + dot(ga, rc.a) + gm * rc.m + gr * rc.r);
  sd.gA = (float)gA;
  sd.gT = (float)gT;
  sd.gZt = (float)(gdepth * inv);
  sd.gZm = (float)(gm * inv);
  sd.gZr = (float)(gr * inv);
  sd.gZn[0] = (float)(gN.x * inv); sd.gZn[1] = (float)(gN.y * inv); sd.gZn[2] = (float)(gN.z * inv);
  sd.gZa[0] = (float)(ga.x * inv); sd.gZa[1] = (float)(ga.y * inv); sd.gZa[2] = (float)(ga.z * inv);
  sd.pad[0] = 1.0f;  // ray has hits
  a.seeds[ray] = sd;
}

// Every block adds its texel gradients to copy blockIdx % copies of the map
// in G.g_env: device-scope atomics from all blocks on the bright texels would
// otherwise serialise on single addresses.
__global__ __launch_bounds__(256) void k_adj_shade(RenderArgs a, GradArgs G, int copies) {
  __shared__ int key[kEnvAggSlots];
  __shared__ float val[3 * kEnvAggSlots];
  for (int j = threadIdx.x; j < kEnvAggSlots; j += blockDim.x) {
    key[j] = -1;
    val[j] = val[kEnvAggSlots + j] = val[2 * kEnvAggSlots + j] = 0.0f;
  }
  __syncthreads();
  // the map's mean luminance weighted as the sampler weights rows (by sin theta), over the texels
  const double mean = a.E.scal[0] / ((double)a.E.H * a.E.W);
  float *genv = G.g_env + (int64_t)(blockIdx.x % (unsigned)copies) * 3 * a.E.H * a.E.W;
  BlockEnvTable acc{key, val, genv, a.E.lum, kEnvHot * mean};
  const int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ray < a.R) adj_shade_ray(a, G, ray, acc);
  __syncthreads();
  for (int j = threadIdx.x; j < kEnvAggSlots; j += blockDim.x) {
    const int t = key[j];
    if (t < 0) continue;
    for (int c = 0; c < 3; ++c) {
      const float g = val[c * kEnvAggSlots + j];
      if (g != 0.0f) atomicAdd(genv + 3 * t + c, g);
    }
  }
}

// deterministic form: each ray's environment records (at most 4 taps per
// lookup, 1 + 3 J lookups), unused positions keyed past every texel
__global__ __launch_bounds__(256) void k_adj_shade_det(RenderArgs a, GradArgs G, DetArgs d) {
  const int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ray >= a.R) return;
  EnvRecords acc{d.env_key, d.env_idx, d.env_val, ray * d.env_cap, 0};
  adj_shade_ray(a, G, ray, acc);
  for (int j = acc.n; j < d.env_cap; ++j) {
    d.env_key[acc.base + j] = d.env_unused;
    d.env_idx[acc.base + j] = (int32_t)(acc.base + j);
  }
}

// ---------------------------------------------------------------- gradient accumulation
// The fifteen per-surfel gradient values of one hit, in this order: albedo
// (3), metallic, roughness, opacity, scale (2), mu (3), raw quaternion (4).
constexpr int kGradVals = 15;

__device__ __forceinline__ float *grad_slot(const GradArgs &G, int64_t i, int v) {
  switch (v) {
    case 0: case 1: case 2: return G.g_albedo + 3 * i + v;
    case 3: return G.g_metallic + i;
    case 4: return G.g_roughness + i;
    case 5: return G.g_opacity + i;
    case 6: case 7: return G.g_scale + 2 * i + (v - 6);
    case 8: case 9: case 10: return G.g_mu + 3 * i + (v - 8);
    default: return G.g_q + 4 * i + (v - 11);
  }
}

// Per-block accumulation of hit gradients in an LDS table keyed by surfel
// (open addressing, a few probes), flushed to device memory with one atomic
// per surfel and value; a hit that finds no slot goes to device memory
// directly.  Neighbouring rays of a block meet largely the same surfels, so
// this replaces most device-scope atomics on shared addresses.
constexpr int kAggBits = 9;
constexpr int kAggSlots = 1 << kAggBits;  // 32 KB of LDS per block with the values
constexpr int kAggProbes = 8;

struct BlockGradTable {
  int *key;     // [kAggSlots], -1 when free
  float *val;   // [kGradVals][kAggSlots]
  const GradArgs &G;
  __device__ void add(int64_t i, const double *dv, int /*slot*/) {
    float gv[kGradVals];
#pragma unroll
    for (int v = 0; v < kGradVals; ++v) gv[v] = (float)dv[v];
    const uint32_t h = (uint32_t)i * 2654435761u;
#pragma unroll 1
    for (int p = 0; p < kAggProbes; ++p) {
      const int slot = (int)((h >> (32 - kAggBits)) + (uint32_t)p) & (kAggSlots - 1);
      const int k = atomicCAS(key + slot, -1, (int)i);
      if (k == -1 || k == (int)i) {
#pragma unroll
        for (int v = 0; v < kGradVals; ++v) atomicAdd(val + v * kAggSlots + slot, gv[v]);
        return;
      }
    }
#pragma unroll
    for (int v = 0; v < kGradVals; ++v) atomicAdd(grad_slot(G, i, v), gv[v]);
  }
};

// deterministic form: one record per hit slot of each work item
struct HitRecords {
  uint64_t *key;  // [items * K] surfel of each record
  int32_t *idx;   // [items * K] the record's own position
  double *val;    // [items * K][kGradVals]
  int64_t base;   // first record of this item
  __device__ void add(int64_t i, const double *gv, int slot) {
    const int64_t r = base + slot;
    key[r] = (uint64_t)i;
    idx[r] = (int32_t)r;
#pragma unroll
    for (int v = 0; v < kGradVals; ++v) val[kGradVals * r + v] = gv[v];
  }
};

// ---------------------------------------------------------------- compositing adjoint
// Back to front over the recomputed hit list: with v_j = gA + sum_z gZ . z_j
// and the suffix V_j = sum_{i>j} w_i v_i,
//   d/d(alpha_j) = T_j v_j - (V_j + gT T) / (1 - alpha_j),
// then through the effective opacity and the plane intersection into
// (mu, q, s, alpha) and through the composited attributes into (a, m, r).
template <int K, class B, class Acc>
__device__ void adjoint_hits(const RenderArgs &a, const AdjSeed &sd, B &kb, d3 o, d3 d, Acc &acc) {
  const TraceParams &P = a.P;
  const double gA = sd.gA, gT = sd.gT, gZt = sd.gZt, gZm = sd.gZm, gZr = sd.gZr, Tfin = sd.T;
  const d3 gZn = mk(sd.gZn[0], sd.gZn[1], sd.gZn[2]), gZa = mk(sd.gZa[0], sd.gZa[1], sd.gZa[2]);
  double V = 0.0, Tafter = Tfin;
  for (int it = 0; it < K; ++it) {
    const double tkey = (double)kb.t[K - 1];
    const uint32_t id = kb.id[K - 1];
    krotr<B, K>(kb);
    if (!(tkey > -INFINITY && tkey < INFINITY)) continue;
    HitE he;
    hit_exact(a.S, P, id, o, d, he);
    const int64_t i = he.orig;
    const double Tj = Tafter / (1.0 - he.at);
    const double wj = Tj * he.at;
    const d3 aj = ld3(a.S.albedo + 3 * i);
    const double mj = a.S.metallic[i], rj = a.S.roughness[i];
    const double vj = gA + gZt * he.t + gZm * mj + gZr * rj + dot(gZn, he.nw) + dot(gZa, aj);
    const double gat = Tj * vj - (V + gT * Tfin) / (1.0 - he.at);
    V += wj * vj;
    Tafter = Tj;
    // attributes
    double gv[kGradVals];
    gv[0] = gZa.x * wj;
    gv[1] = gZa.y * wj;
    gv[2] = gZa.z * wj;
    gv[3] = gZm * wj;
    gv[4] = gZr * wj;
    // frame of the raw quaternion, object-space ray of the hit's instance
    const InstRec &I = a.S.inst[he.inst];
    d3 oo, dd;
    to_object(I, o, d, oo, dd);
    const float *q = a.S.q + 4 * i;
    const double qlen = sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3]);
    const double w = q[0] / qlen, x = q[1] / qlen, y = q[2] / qlen, z = q[3] / qlen;
    d3 tu, tv, n;
    quat_frame(w, x, y, z, tu, tv, n);
    const d3 mu = ld3(a.S.mu + 3 * i);
    const double su = a.S.scale[2 * i], sv = a.S.scale[2 * i + 1], alpha = a.S.opacity[i];
    const d3 dl = (oo + he.t * dd) - mu;
    const double xu = dot(dl, tu) / su, xv = dot(dl, tv) / sv;
    const double g = exp(-0.5 * (xu * xu + xv * xv));
    const double raw = alpha * g;
    // effective opacity alpha_t = min(cap, alpha exp(-rho^2/2))
    const double graw = raw > P.alpha_cap ? 0.0 : gat;
    gv[5] = graw * g;
    const double grho2 = graw * alpha * g * (-0.5);
    const double gxu = grho2 * 2.0 * xu, gxv = grho2 * 2.0 * xv;
    gv[6] = -gxu * xu / su;
    gv[7] = -gxv * xv / sv;
    const d3 gdl = (gxu / su) * tu + (gxv / sv) * tv;
    const d3 gtu = (gxu / su) * dl, gtv = (gxv / sv) * dl;
    // dl = o + t d - mu ; t = n.(mu - o) / (n.d) ; composited normal = +-R n
    const double gt = gZt * wj + dot(gdl, dd);
    const double den = dot(n, dd);
    const d3 gnw = wj * gZn;
    d3 gno = I.identity ? gnw : mulT(I.R, gnw);
    if (id & kFlipBit) gno = -gno;
    const d3 gmu = (gt / den) * n - gdl;
    const d3 gnn = gno - (gt / den) * dl;
    gv[8] = gmu.x;
    gv[9] = gmu.y;
    gv[10] = gmu.z;
    // columns (t_u, t_v, n) of rot(q_hat) -> q_hat -> raw q;  G[r][c] row-major
    const double G0 = gtu.x, G1 = gtv.x, G2 = gnn.x, G3 = gtu.y, G4 = gtv.y, G5 = gnn.y, G6 = gtu.z, G7 = gtv.z,
                 G8 = gnn.z;
    const double gq0 = G1 * (-2 * z) + G2 * (2 * y) + G3 * (2 * z) + G5 * (-2 * x) + G6 * (-2 * y) + G7 * (2 * x);
    const double gq1 = G1 * (2 * y) + G2 * (2 * z) + G3 * (2 * y) + G4 * (-4 * x) + G5 * (-2 * w) + G6 * (2 * z) +
                       G7 * (2 * w) + G8 * (-4 * x);
    const double gq2 = G0 * (-4 * y) + G1 * (2 * x) + G2 * (2 * w) + G3 * (2 * x) + G5 * (2 * z) + G6 * (-2 * w) +
                       G7 * (2 * z) + G8 * (-4 * y);
    const double gq3 = G0 * (-4 * z) + G1 * (-2 * w) + G2 * (2 * x) + G3 * (2 * w) + G4 * (-4 * z) + G5 * (2 * y) +
                       G6 * (2 * x) + G7 * (2 * y);
    const double pq = gq0 * w + gq1 * x + gq2 * y + gq3 * z;
    gv[11] = (gq0 - w * pq) / qlen;
    gv[12] = (gq1 - x * pq) / qlen;
    gv[13] = (gq2 - y * pq) / qlen;
    gv[14] = (gq3 - z * pq) / qlen;
    acc.add(i, gv, it);
  }
}

// the seeded rays among the primary work items (tiles of the cameras or explicit rays)
__device__ __forceinline__ int64_t adj_items(const RenderArgs &a) { return a.n_tiles ? a.n_tiles * kBlock : a.R; }
inline int64_t adj_items_host(const RenderArgs &a) { return a.n_tiles ? a.n_tiles * kBlock : a.R; }
__device__ __forceinline__ int64_t adj_ray(const RenderArgs &a, int64_t item) {
  const int64_t ray = a.n_tiles ? tile_ray(*a.rays.cams, item) : item;
  return (ray >= 0 && ray < a.R && a.seeds[ray].pad[0] != 0.0f) ? ray : -1;
}

// compositing adjoint of every seeded ray from the k-buffer its replayed
// primary traversal left in kbuf1 (same rays, scene and constants, so the same
// hit list)
template <int K>
__global__ __launch_bounds__(kBlock) void k_adj_hits(RenderArgs a, GradArgs G) {
  __shared__ int key[kAggSlots];
  __shared__ float val[kGradVals * kAggSlots];
  for (int j = threadIdx.x; j < kAggSlots; j += kBlock) {
    key[j] = -1;
#pragma unroll
    for (int v = 0; v < kGradVals; ++v) val[v * kAggSlots + j] = 0.0f;
  }
  __syncthreads();
  BlockGradTable tab{key, val, G};
  const int64_t item = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t ray = item < adj_items(a) ? adj_ray(a, item) : -1;
  if (ray >= 0) {
    float of[3], df[3];
    load_ray(a.rays, ray, of, df);
    KBufF<K> kb;
    load_kbuf<K>(kb, a.kbuf1 + item * 2 * K);
    adjoint_hits<K>(a, a.seeds[ray], kb, mk(of[0], of[1], of[2]), mk(df[0], df[1], df[2]), tab);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kAggSlots; j += kBlock) {
    const int i = key[j];
    if (i < 0) continue;
#pragma unroll
    for (int v = 0; v < kGradVals; ++v) {
      const float g = val[v * kAggSlots + j];
      if (g != 0.0f) atomicAdd(grad_slot(G, i, v), g);
    }
  }
}

// deterministic form: K records per work item, unused slots keyed past every surfel
template <int K>
__global__ __launch_bounds__(kBlock) void k_adj_hits_det(RenderArgs a, GradArgs G, DetArgs d) {
  const int64_t item = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (item >= adj_items(a)) return;
  const int64_t base = item * K;
  for (int j = 0; j < K; ++j) {
    d.hit_key[base + j] = d.hit_unused;
    d.hit_idx[base + j] = (int32_t)(base + j);
  }
  const int64_t ray = adj_ray(a, item);
  if (ray < 0) return;
  float of[3], df[3];
  load_ray(a.rays, ray, of, df);
  KBufF<K> kb;
  load_kbuf<K>(kb, a.kbuf1 + item * 2 * K);
  HitRecords acc{d.hit_key, d.hit_idx, d.hit_val, base};
  adjoint_hits<K>(a, a.seeds[ray], kb, mk(of[0], of[1], of[2]), mk(df[0], df[1], df[2]), acc);
}

// One thread per sorted record; the first record of each key sums the
// key's records in sorted (= position) order in binary64 and writes the
// rounded sums over the target's zero-initialised gradients.
__global__ void k_det_reduce_hits(const uint64_t *key, const int32_t *idx, int64_t n, uint64_t unused,
                                  const double *val, GradArgs G) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint64_t k = key[p];
  if (k == unused || (p > 0 && key[p - 1] == k)) return;
  double s[kGradVals];
#pragma unroll
  for (int v = 0; v < kGradVals; ++v) s[v] = 0.0;
  for (int64_t q = p; q < n && key[q] == k; ++q) {
    const double *r = val + (int64_t)kGradVals * idx[q];
#pragma unroll
    for (int v = 0; v < kGradVals; ++v) s[v] += r[v];
  }
#pragma unroll
  for (int v = 0; v < kGradVals; ++v) *grad_slot(G, (int64_t)k, v) = (float)s[v];
}

__global__ void k_det_reduce_env(const uint64_t *key, const int32_t *idx, int64_t n, uint64_t unused,
                                 const double *val, float *genv) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint64_t k = key[p];
  if (k == unused || (p > 0 && key[p - 1] == k)) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t q = p; q < n && key[q] == k; ++q) {
    const double *r = val + 3 * (int64_t)idx[q];
    s0 += r[0];
    s1 += r[1];
    s2 += r[2];
  }
  genv[3 * k] = (float)s0;
  genv[3 * k + 1] = (float)s1;
  genv[3 * k + 2] = (float)s2;
}

template <int K>
void adjoint_hits_k(const RenderArgs &a, const GradArgs &g, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_hits<K>, dim3(blocks(adj_items_host(a), kBlock)), dim3(kBlock), 0, st, a, g);
}

template <int K>
void adjoint_hits_det_k(const RenderArgs &a, const GradArgs &g, const DetArgs &d, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_hits_det<K>, dim3(blocks(adj_items_host(a), kBlock)), dim3(kBlock), 0, st, a, g, d);
}

}  // namespace

int64_t adjoint_items(const RenderArgs &a) { return adj_items_host(a); }

void launch_adjoint_shade_det(const RenderArgs &a, const GradArgs &g, const DetArgs &d, hipStream_t st) {
  if (a.R <= 0) return;
  hipLaunchKernelGGL(k_adj_shade_det, dim3(blocks(a.R, 256)), dim3(256), 0, st, a, g, d);
  radix_sort(d.env_key, d.env_idx, d.env_key2, d.env_idx2, d.hist, d.n_env, st, d.env_bits);
  hipLaunchKernelGGL(k_det_reduce_env, dim3(blocks(d.n_env, 256)), dim3(256), 0, st, (const uint64_t *)d.env_key,
                     (const int32_t *)d.env_idx, d.n_env, d.env_unused, (const double *)d.env_val, g.g_env);
}

void launch_adjoint_hits_det(const RenderArgs &a, const GradArgs &g, const DetArgs &d, hipStream_t st) {
  if (a.R <= 0) return;
  switch (kbucket(a.P.k)) {
    case 8: adjoint_hits_det_k<8>(a, g, d, st); break;
    case 16: adjoint_hits_det_k<16>(a, g, d, st); break;
    case 32: adjoint_hits_det_k<32>(a, g, d, st); break;
    default: adjoint_hits_det_k<64>(a, g, d, st); break;
  }
  radix_sort(d.hit_key, d.hit_idx, d.hit_key2, d.hit_idx2, d.hist, d.n_hit, st, d.hit_bits);
  hipLaunchKernelGGL(k_det_reduce_hits, dim3(blocks(d.n_hit, 256)), dim3(256), 0, st, (const uint64_t *)d.hit_key,
                     (const int32_t *)d.hit_idx, d.n_hit, d.hit_unused, (const double *)d.hit_val, g);
}

// g_env[i] = the copies' values at i, added in copy order
__global__ void k_env_copies_sum(const float *part, int64_t m, int copies, float *genv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  float s = 0.0f;
  for (int x = 0; x < copies; ++x) s += part[x * m + i];
  genv[i] = s;
}

void launch_adjoint_shade(const RenderArgs &a, const GradArgs &g, float *part, int copies, hipStream_t st) {
  if (a.R <= 0) return;
  if (copies <= 1 || !part) {
    hipLaunchKernelGGL(k_adj_shade, dim3(blocks(a.R, 256)), dim3(256), 0, st, a, g, 1);
    return;
  }
  const int64_t m = (int64_t)3 * a.E.H * a.E.W;
  launch_fill_f32(part, 0.0f, copies * m, st);
  GradArgs gp = g;
  gp.g_env = part;
  hipLaunchKernelGGL(k_adj_shade, dim3(blocks(a.R, 256)), dim3(256), 0, st, a, gp, copies);
  hipLaunchKernelGGL(k_env_copies_sum, dim3(blocks(m, 256)), dim3(256), 0, st, (const float *)part, m, copies,
                     g.g_env);
}

void launch_adjoint_hits(const RenderArgs &a, const GradArgs &g, hipStream_t st) {
  if (a.R <= 0) return;
  switch (kbucket(a.P.k)) {
    case 8: adjoint_hits_k<8>(a, g, st); break;
    case 16: adjoint_hits_k<16>(a, g, st); break;
    case 32: adjoint_hits_k<32>(a, g, st); break;
    default: adjoint_hits_k<64>(a, g, st); break;
  }
}

}  // namespace lf

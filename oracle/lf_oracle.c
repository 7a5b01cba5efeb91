/*
 * lf_oracle.c -- plain FP64 CPU oracle (test infrastructure only; see
 * lf_oracle.h).  Brute force over every surfel for every ray, no BVH, no
 * blocking, no reordering beyond what the method states.  OpenMP parallelises
 * over rays only.
 *
 * Structure: for each primary ray, decide() takes every discrete decision of
 * the estimator at the given parameters (hit lists, sampled directions,
 * technique/lobe choices, MIS and pdf factors, secondary traces and records)
 * and records them as a "frozen" path; evaluate() computes the outputs from the
 * live parameters given a frozen path.  The forward render is
 * evaluate(theta, decide(theta)); the path-replay objective is
 * evaluate(theta, decide(theta0)); the adjoint is the hand-written reverse of
 * evaluate.
 */
#include "lf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846
#define INV_PI (1.0 / PI)
#define KMAX 64
#define LUM_R 0.2126
#define LUM_G 0.7152
#define LUM_B 0.0722

/* ------------------------------------------------------------------------ */
/* small vector helpers                                                     */
/* ------------------------------------------------------------------------ */
static inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static inline double lum3(const double *c) { return LUM_R * c[0] + LUM_G * c[1] + LUM_B * c[2]; }
static inline double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }
static inline double dmin(double a, double b) { return a < b ? a : b; }

/* ------------------------------------------------------------------------ */
/* sampler: SplitMix64 (Steele, Lea & Flood 2014), chained over             */
/* (seed, ray id, sample, dimension); 24-bit uniforms exact in float/double  */
/* ------------------------------------------------------------------------ */
uint64_t ors_splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double ors_uniform(uint64_t seed, uint64_t ray, uint64_t sample, uint32_t dim) {
  uint64_t h = ors_splitmix64(seed ^ ors_splitmix64(ray ^ ors_splitmix64((sample << 8) | (uint64_t)dim)));
  return (double)(h >> 40) * (1.0 / 16777216.0);
}

/* Owen-scrambled Sobol points (Sec. 3.3 PRB paragraph: the forward seed is
 * recorded and the same Sobol samples are replayed).  Sobol's construction
 * with the direction numbers of Joe and Kuo (2008) for dimensions 1..10
 * (primitive polynomial of degree s with inner coefficients a, initial
 * m_1..m_s), dimension 0 the van der Corput sequence; the point of index i
 * XORs the direction numbers V_k of the set bits k of i.  Pinned: the
 * construction (hand-derived first points, nets), primitive polynomials,
 * valid m_k and 2D projections of t <= 4; that the m_k are Joe and Kuo's
 * particular choice among valid ones is parity unpinned. */
#define ORS_SOBOL_DIMS 11
static const int sob_s[ORS_SOBOL_DIMS] = {0, 1, 2, 3, 3, 4, 4, 5, 5, 5, 5};
static const uint32_t sob_a[ORS_SOBOL_DIMS] = {0, 0, 1, 1, 2, 1, 4, 2, 4, 7, 11};
static const uint32_t sob_m[ORS_SOBOL_DIMS][5] = {{0},          {1},          {1, 3},         {1, 3, 1},
                                                  {1, 1, 1},    {1, 1, 3, 3}, {1, 3, 5, 13},  {1, 1, 5, 5, 17},
                                                  {1, 1, 5, 5, 5}, {1, 1, 7, 11, 19}, {1, 1, 5, 1, 1}};

/* direction number V_k (k = 1..32) of dimension d, as a 32-bit fraction:
 * V_k = m_k 2^(32-k), with m_k from the polynomial's recurrence
 * m_k = 2 a_1 m_(k-1) ^ 4 a_2 m_(k-2) ^ ... ^ 2^(s-1) a_(s-1) m_(k-s+1) ^ 2^s m_(k-s) ^ m_(k-s) */
static uint32_t sobol_direction(int d, int k) {
  if (d == 0) return 1u << (32 - k);
  const int s = sob_s[d];
  uint64_t m[33];
  for (int j = 1; j <= 32; ++j) {
    if (j <= s) {
      m[j] = sob_m[d][j - 1];
    } else {
      uint64_t v = (m[j - s] << s) ^ m[j - s];
      for (int i = 1; i < s; ++i)
        if ((sob_a[d] >> (s - 1 - i)) & 1u) v ^= m[j - i] << i;
      m[j] = v;
    }
  }
  return (uint32_t)(m[k] << (32 - k));
}

void ors_sobol_poly(uint32_t d, int32_t *degree, uint32_t *inner) {
  *degree = sob_s[d];
  *inner = sob_a[d];
}

uint32_t ors_sobol(uint32_t i, uint32_t d) {
  uint32_t x = 0;
  for (int k = 1; k <= 32; ++k)
    if ((i >> (k - 1)) & 1u) x ^= sobol_direction((int)d, k);
  return x;
}

static uint32_t reverse_bits32(uint32_t x) {
  uint32_t r = 0;
  for (int b = 0; b < 32; ++b) r |= ((x >> b) & 1u) << (31 - b);
  return r;
}

/* nested uniform (Owen) scramble by Burley's hash (2020, "Practical
 * Hash-based Owen Scrambling"): in bit-reversed order, an add and four
 * xor-multiplies by even constants, so every bit is flipped by a function
 * of the bits above it in the original order only */
uint32_t ors_owen_scramble(uint32_t x, uint32_t seed) {
  x = reverse_bits32(x);
  x += seed;
  x ^= x * 0x6c50b47cu;
  x ^= x * 0xb82f1e52u;
  x ^= x * 0xc7afe638u;
  x ^= x * 0x8d22f6e6u;
  return reverse_bits32(x);
}

/* u = 24-bit uniform of (seed, ray, sample, dim): the ray's seed scrambles
 * the sample index (so every ray uses its own aligned block of the
 * sequence) and, per dimension, the Sobol coordinate */
double ors_sobol_uniform(uint64_t seed, uint64_t ray, uint64_t sample, uint32_t dim) {
  const uint64_t h = ors_splitmix64(seed ^ ors_splitmix64(ray));
  const uint32_t i = ors_owen_scramble((uint32_t)sample, (uint32_t)h);
  const uint32_t ds = (uint32_t)(ors_splitmix64(h ^ (0x100000000ull + dim)) >> 32);
  const uint32_t x = ors_owen_scramble(ors_sobol(i, dim), ds);
  return (double)(x >> 8) * (1.0 / 16777216.0);
}

/* the sampler the parameters select */
static double draw(const ors_params *p, int64_t ray, int s, uint32_t dim) {
  return (p->flags & ORS_SOBOL) ? ors_sobol_uniform(p->seed, (uint64_t)ray, (uint64_t)s, dim)
                                : ors_uniform(p->seed, (uint64_t)ray, (uint64_t)s, dim);
}

/* ------------------------------------------------------------------------ */
/* frames                                                                   */
/* ------------------------------------------------------------------------ */
/* standard rotation matrix of a unit quaternion (w,x,y,z), row-major */
static void quat_matrix(const double *q, double *M) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  M[0] = 1 - 2 * (y * y + z * z); M[1] = 2 * (x * y - w * z);     M[2] = 2 * (x * z + w * y);
  M[3] = 2 * (x * y + w * z);     M[4] = 1 - 2 * (x * x + z * z); M[5] = 2 * (y * z - w * x);
  M[6] = 2 * (x * z - w * y);     M[7] = 2 * (y * z + w * x);     M[8] = 1 - 2 * (x * x + y * y);
}

void ors_quat_to_frame(const double q[4], double tu[3], double tv[3], double n[3]) {
  double len = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double qh[4] = {q[0] / len, q[1] / len, q[2] / len, q[3] / len}, M[9];
  quat_matrix(qh, M);
  for (int r = 0; r < 3; ++r) { tu[r] = M[3 * r + 0]; tv[r] = M[3 * r + 1]; n[r] = M[3 * r + 2]; }
}

/* rotation of an object transform: Gram-Schmidt of the first two columns,
 * third column their cross product (the FP32 input is only approximately
 * orthonormal; both implementations use this same definition) */
static void orthonormalise(const double *A, double *R) {
  double c0[3] = {A[0], A[3], A[6]}, c1[3] = {A[1], A[4], A[7]}, c2[3];
  double l0 = sqrt(dot3(c0, c0));
  for (int i = 0; i < 3; ++i) c0[i] /= l0;
  double p = dot3(c0, c1);
  for (int i = 0; i < 3; ++i) c1[i] -= p * c0[i];
  double l1 = sqrt(dot3(c1, c1));
  for (int i = 0; i < 3; ++i) c1[i] /= l1;
  cross3(c0, c1, c2);
  for (int r = 0; r < 3; ++r) { R[3 * r + 0] = c0[r]; R[3 * r + 1] = c1[r]; R[3 * r + 2] = c2[r]; }
}

/* branchless orthonormal basis (Duff et al. 2017, "Building an Orthonormal
 * Basis, Revisited") */
void ors_onb(const double n[3], double b1[3], double b2[3]) {
  double sign = n[2] >= 0.0 ? 1.0 : -1.0;
  double a = -1.0 / (sign + n[2]);
  double b = n[0] * n[1] * a;
  b1[0] = 1.0 + sign * n[0] * n[0] * a; b1[1] = sign * b; b1[2] = -sign * n[0];
  b2[0] = b; b2[1] = sign + n[1] * n[1] * a; b2[2] = -n[1];
}

/* ------------------------------------------------------------------------ */
/* world-space surfels (Eq. state-assembly; rigid transforms move centres    */
/* and orientations only)                                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  double mu[3], tu[3], tv[3], n[3];
  double su, sv, alpha, rho2max;
  double qh[4], qlen; /* normalised quaternion and the raw norm (for the adjoint) */
  int obj;            /* -1 background, else object index */
} wsurf;

typedef struct {
  const ors_scene *sc;
  const ors_params *p;
  int64_t n;
  int M;
  double *R; /* [M,9] orthonormalised rotations */
  wsurf *ws;
  /* environment sampling distribution */
  int H, W;
  double *lum, *rowsum, *roww, *cdf_row, *cdf_col; /* [H*W],[H],[H],[H+1],[H*(W+1)] */
  double total;
  double c_env, c_bsdf;
} world;

static int surfel_object(const ors_scene *sc, int64_t i) {
  for (int o = 0; o < sc->n_objects; ++o)
    if (i >= sc->object_offset[o + 1] && i < sc->object_offset[o + 2]) return o;
  return -1;
}

static void build_world(world *w, const ors_scene *sc, const ors_params *p) {
  w->sc = sc; w->p = p; w->n = sc->n; w->M = sc->n_objects;
  w->R = (double *)malloc(sizeof(double) * 9 * (w->M > 0 ? w->M : 1));
  for (int o = 0; o < w->M; ++o) orthonormalise(sc->R + 9 * o, w->R + 9 * o);
  w->ws = (wsurf *)malloc(sizeof(wsurf) * (sc->n > 0 ? sc->n : 1));
  double sig2 = p->support_sigma * p->support_sigma;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < sc->n; ++i) {
    wsurf *s = &w->ws[i];
    const double *q = sc->q + 4 * i;
    s->qlen = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int c = 0; c < 4; ++c) s->qh[c] = q[c] / s->qlen;
    double Mq[9];
    quat_matrix(s->qh, Mq);
    s->obj = surfel_object(sc, i);
    double F[9];
    if (s->obj >= 0) {
      const double *Ro = w->R + 9 * s->obj, *to = sc->t + 3 * s->obj;
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
          F[3 * r + c] = Ro[3 * r + 0] * Mq[0 + c] + Ro[3 * r + 1] * Mq[3 + c] + Ro[3 * r + 2] * Mq[6 + c];
        s->mu[r] = Ro[3 * r + 0] * sc->mu[3 * i + 0] + Ro[3 * r + 1] * sc->mu[3 * i + 1] +
                   Ro[3 * r + 2] * sc->mu[3 * i + 2] + to[r];
      }
    } else {
      memcpy(F, Mq, sizeof F);
      for (int r = 0; r < 3; ++r) s->mu[r] = sc->mu[3 * i + r];
    }
    for (int r = 0; r < 3; ++r) { s->tu[r] = F[3 * r + 0]; s->tv[r] = F[3 * r + 1]; s->n[r] = F[3 * r + 2]; }
    s->su = sc->scale[2 * i + 0];
    s->sv = sc->scale[2 * i + 1];
    s->alpha = sc->opacity[i];
    /* support and opacity threshold as one predicate (Sec. 3.2): rho^2 <= sigma^2
     * and alpha*exp(-rho^2/2) >= alpha_min */
    s->rho2max = dmin(sig2, 2.0 * log(s->alpha / p->alpha_min));
  }
  /* environment importance-sampling distribution: rows by luminance times
   * sin(theta) at the row centre, columns by luminance within a row */
  int H = sc->env_h, W = sc->env_w;
  w->H = H; w->W = W;
  w->lum = (double *)calloc((size_t)H * W, sizeof(double));
  w->rowsum = (double *)calloc(H, sizeof(double));
  w->roww = (double *)calloc(H, sizeof(double));
  w->cdf_row = (double *)calloc(H + 1, sizeof(double));
  w->cdf_col = (double *)calloc((size_t)H * (W + 1), sizeof(double));
  w->total = 0.0;
  for (int r = 0; r < H; ++r) {
    double rs = 0.0;
    for (int c = 0; c < W; ++c) {
      double l = lum3(sc->env + 3 * ((size_t)r * W + c));
      if (!(l > 0.0)) l = 0.0;
      w->lum[(size_t)r * W + c] = l;
      rs += l;
    }
    w->rowsum[r] = rs;
    w->roww[r] = rs * sin((r + 0.5) * PI / H);
    w->total += w->roww[r];
    double *cc = w->cdf_col + (size_t)r * (W + 1);
    cc[0] = 0.0;
    for (int c = 0; c < W; ++c) cc[c + 1] = rs > 0.0 ? cc[c] + w->lum[(size_t)r * W + c] / rs : (double)(c + 1) / W;
    cc[W] = 1.0;
  }
  w->cdf_row[0] = 0.0;
  for (int r = 0; r < H; ++r) w->cdf_row[r + 1] = w->total > 0.0 ? w->cdf_row[r] + w->roww[r] / w->total : (double)(r + 1) / H;
  w->cdf_row[H] = 1.0;
  w->c_env = (w->total > 0.0 && !(p->flags & ORS_BSDF_ONLY)) ? 0.5 : 0.0;
  w->c_bsdf = 1.0 - w->c_env;
}

static void free_world(world *w) {
  free(w->R); free(w->ws); free(w->lum); free(w->rowsum); free(w->roww); free(w->cdf_row); free(w->cdf_col);
}

/* ------------------------------------------------------------------------ */
/* environment map: lat-long, +Y up, theta = acos(w_y), phi = atan2(w_z,w_x) */
/* ------------------------------------------------------------------------ */
static void dir_to_uv(const double *w, double *u, double *v) {
  double th = acos(clampd(w[1], -1.0, 1.0));
  double ph = atan2(w[2], w[0]);
  if (ph < 0.0) ph += 2.0 * PI;
  *u = ph / (2.0 * PI);
  *v = th / PI;
}

/* bilinear lookup at (v*H - 1/2, u*W - 1/2): wraps in u, clamps in v.  The
 * four texel indices and weights are returned for gradient scattering. */
static void env_taps(int H, int W, const double *w, int64_t *tap, double *wt) {
  double u, v;
  dir_to_uv(w, &u, &v);
  double x = u * W - 0.5, y = v * H - 0.5;
  double x0 = floor(x), y0 = floor(y);
  double fx = x - x0, fy = y - y0;
  int64_t c0 = ((int64_t)x0 % W + W) % W, c1 = (c0 + 1) % W;
  int64_t r0 = (int64_t)y0, r1 = r0 + 1;
  if (r0 < 0) r0 = 0;
  if (r0 > H - 1) r0 = H - 1;
  if (r1 < 0) r1 = 0;
  if (r1 > H - 1) r1 = H - 1;
  tap[0] = r0 * W + c0; wt[0] = (1 - fy) * (1 - fx);
  tap[1] = r0 * W + c1; wt[1] = (1 - fy) * fx;
  tap[2] = r1 * W + c0; wt[2] = fy * (1 - fx);
  tap[3] = r1 * W + c1; wt[3] = fy * fx;
}

static void env_eval(const double *env, int H, int W, const double *w, double *rgb) {
  int64_t tap[4];
  double wt[4];
  env_taps(H, W, w, tap, wt);
  rgb[0] = rgb[1] = rgb[2] = 0.0;
  for (int k = 0; k < 4; ++k)
    for (int c = 0; c < 3; ++c) rgb[c] += wt[k] * env[3 * tap[k] + c];
}

static void env_scatter(double *genv, int H, int W, const double *w, const double *g) {
  int64_t tap[4];
  double wt[4];
  env_taps(H, W, w, tap, wt);
  for (int k = 0; k < 4; ++k)
    for (int c = 0; c < 3; ++c) {
#pragma omp atomic
      genv[3 * tap[k] + c] += wt[k] * g[c];
    }
}

/* first index i in [0,n) with cdf[i+1] > u (cdf has n+1 entries, cdf[n] = 1) */
static int cdf_search(const double *cdf, int n, double u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    if (cdf[mid + 1] > u) hi = mid; else lo = mid + 1;
  }
  return lo;
}

static double env_texel_pdf(const world *w, int r, int c, double sin_th) {
  if (!(sin_th > 0.0) || !(w->total > 0.0) || !(w->rowsum[r] > 0.0)) return 0.0;
  double prow = w->roww[r] / w->total, pcol = w->lum[(size_t)r * w->W + c] / w->rowsum[r];
  return prow * pcol * (double)w->H * (double)w->W / (2.0 * PI * PI * sin_th);
}

/* solid-angle pdf of environment importance sampling at direction w; *margin
 * receives the distance of the direction to the nearest texel edge (in
 * units of the [0,1) parameterisation) */
static double env_pdf_m(const world *w, const double *dir, double *margin) {
  double u, v;
  dir_to_uv(dir, &u, &v);
  double y = v * w->H, x = u * w->W;
  int r = (int)floor(y), c = (int)floor(x);
  if (r > w->H - 1) r = w->H - 1;
  if (c > w->W - 1) c = w->W - 1;
  if (margin) {
    double my = dmin(y - floor(y), ceil(y) - y) / w->H, mx = dmin(x - floor(x), ceil(x) - x) / w->W;
    if (y == floor(y)) my = 0.0;
    if (x == floor(x)) mx = 0.0;
    *margin = dmin(*margin, dmin(my, mx));
  }
  double st = sin(v * PI);
  return env_texel_pdf(w, r, c, st);
}

/* piecewise-constant sampling: row from the marginal CDF, column from the
 * row's conditional CDF, continuous offset within the texel */
static double env_sample_m(const world *w, double ua, double ub, double *dir, double *margin) {
  int r = cdf_search(w->cdf_row, w->H, ua);
  const double *cc = w->cdf_col + (size_t)r * (w->W + 1);
  int c = cdf_search(cc, w->W, ub);
  if (margin) {
    double m = dmin(fabs(ua - w->cdf_row[r]), fabs(w->cdf_row[r + 1] - ua));
    m = dmin(m, dmin(fabs(ub - cc[c]), fabs(cc[c + 1] - ub)));
    *margin = dmin(*margin, m);
  }
  double orow = (ua - w->cdf_row[r]) / (w->cdf_row[r + 1] - w->cdf_row[r]);
  double ocol = (ub - cc[c]) / (cc[c + 1] - cc[c]);
  double v = (r + orow) / w->H, u = (c + ocol) / w->W;
  double th = v * PI, ph = u * 2.0 * PI;
  double st = sin(th);
  dir[0] = st * cos(ph); dir[1] = cos(th); dir[2] = st * sin(ph);
  return env_texel_pdf(w, r, c, st);
}

/* ------------------------------------------------------------------------ */
/* metallic-roughness BRDF (Sec. 3.3): Lambert diffuse + GGX microfacet      */
/* specular (Walter et al. 2007) with separable Smith G and Schlick Fresnel  */
/* ------------------------------------------------------------------------ */
typedef struct { double ci, co, ch, vh, alpha2, D, G1i, G1o, P; int r_clamped; double reff; } spec_t;

static void spec_setup(const double *n, const double *wi, const double *wo, double r, spec_t *s) {
  double h[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
  double hl = sqrt(dot3(h, h));
  for (int i = 0; i < 3; ++i) h[i] /= hl;
  s->ci = dot3(n, wi); s->co = dot3(n, wo); s->ch = dot3(n, h); s->vh = dot3(wo, h);
  s->r_clamped = (r < 0.08 || r > 1.0);
  s->reff = clampd(r, 0.08, 1.0);
  double ag = s->reff * s->reff;
  s->alpha2 = ag * ag;
  double den = s->ch * s->ch * (s->alpha2 - 1.0) + 1.0;
  s->D = s->alpha2 / (PI * den * den);
  s->G1i = 2.0 * s->ci / (s->ci + sqrt(s->alpha2 + (1.0 - s->alpha2) * s->ci * s->ci));
  s->G1o = 2.0 * s->co / (s->co + sqrt(s->alpha2 + (1.0 - s->alpha2) * s->co * s->co));
  double om = 1.0 - s->vh;
  s->P = om * om * om * om * om;
}

/* f(wi,wo) without the cosine; zero outside the upper hemisphere of n */
void ors_brdf(const double n[3], const double wi[3], const double wo[3], const double a[3],
              double m, double r, uint32_t flags, double f[3]) {
  double ci = dot3(n, wi), co = dot3(n, wo);
  if (!(ci > 0.0) || !(co > 0.0)) { f[0] = f[1] = f[2] = 0.0; return; }
  for (int c = 0; c < 3; ++c) f[c] = (1.0 - m) * a[c] * INV_PI;
  if (flags & ORS_DIFFUSE_ONLY) return;
  spec_t s;
  spec_setup(n, wi, wo, r, &s);
  double sc = s.D * s.G1i * s.G1o / (4.0 * ci * co);
  for (int c = 0; c < 3; ++c) {
    double F0 = 0.04 * (1.0 - m) + a[c] * m;
    f[c] += sc * (F0 + (1.0 - F0) * s.P);
  }
}

double ors_ggx_D(double ch, double r) {
  double reff = clampd(r, 0.08, 1.0), ag = reff * reff, a2 = ag * ag;
  double den = ch * ch * (a2 - 1.0) + 1.0;
  return a2 / (PI * den * den);
}
double ors_smith_G1(double c, double r) {
  double reff = clampd(r, 0.08, 1.0), ag = reff * reff, a2 = ag * ag;
  return 2.0 * c / (c + sqrt(a2 + (1.0 - a2) * c * c));
}
double ors_q_spec(const double a[3], double m, uint32_t flags);

/* probability of picking the GGX lobe in the BSDF mixture */
static double q_spec(const double *a, double m, uint32_t flags) {
  if (flags & ORS_DIFFUSE_ONLY) return 0.0;
  double F0[3], dif[3];
  for (int c = 0; c < 3; ++c) { F0[c] = 0.04 * (1.0 - m) + a[c] * m; dif[c] = (1.0 - m) * a[c]; }
  double lf = lum3(F0), ld = lum3(dif);
  if (!(lf + ld > 0.0)) return 0.5;
  return clampd(lf / (lf + ld), 0.1, 0.9);
}

double ors_q_spec(const double a[3], double m, uint32_t flags) { return q_spec(a, m, flags); }

static double pdf_ggx(const double *n, const double *wi, const double *wo, double r) {
  spec_t s;
  spec_setup(n, wi, wo, r, &s);
  if (!(s.ci > 0.0) || !(s.vh > 0.0)) return 0.0;
  return s.D * s.ch / (4.0 * fabs(s.vh));
}

double ors_pdf_bsdf(const double n[3], const double wi[3], const double wo[3],
                    const double a[3], double m, double r, uint32_t flags) {
  double ci = dot3(n, wi);
  if (!(ci > 0.0)) return 0.0;
  double qs = q_spec(a, m, flags);
  double pc = ci * INV_PI;
  if (qs == 0.0) return pc;
  return qs * pdf_ggx(n, wi, wo, r) + (1.0 - qs) * pc;
}

/* direction from the cosine (Malley) or GGX (Walter et al. 2007) lobe */
static void sample_lobe(const double *n, const double *wo, double r, int spec, double u1, double u2, double *wi) {
  double b1[3], b2[3], l[3];
  ors_onb(n, b1, b2);
  double ph = 2.0 * PI * u2;
  if (!spec) {
    double rr = sqrt(u1);
    l[0] = rr * cos(ph); l[1] = rr * sin(ph); l[2] = sqrt(1.0 - u1);
    for (int i = 0; i < 3; ++i) wi[i] = l[0] * b1[i] + l[1] * b2[i] + l[2] * n[i];
  } else {
    double reff = clampd(r, 0.08, 1.0), ag = reff * reff, a2 = ag * ag;
    double c2 = (1.0 - u1) / (1.0 + (a2 - 1.0) * u1);
    double ct = sqrt(c2), st = sqrt(1.0 - c2 < 0.0 ? 0.0 : 1.0 - c2);
    double h[3];
    l[0] = st * cos(ph); l[1] = st * sin(ph); l[2] = ct;
    for (int i = 0; i < 3; ++i) h[i] = l[0] * b1[i] + l[1] * b2[i] + l[2] * n[i];
    double oh = dot3(wo, h);
    for (int i = 0; i < 3; ++i) wi[i] = 2.0 * oh * h[i] - wo[i];
  }
}

int ors_sample_bsdf(const double n[3], const double wo[3], const double a[3], double m,
                    double r, uint32_t flags, double u_lobe, double u1, double u2, double wi[3]) {
  double qs = q_spec(a, m, flags);
  sample_lobe(n, wo, r, u_lobe < qs, u1, u2, wi);
  return dot3(n, wi) > 0.0;
}

double ors_env_pdf(const ors_scene *scene, const double w[3]) {
  ors_params p;
  memset(&p, 0, sizeof p);
  p.alpha_min = 1.0 / 255.0; p.support_sigma = 3.0;
  world wd;
  ors_scene s = *scene;
  s.n = 0;
  build_world(&wd, &s, &p);
  double r = env_pdf_m(&wd, w, NULL);
  free_world(&wd);
  return r;
}

double ors_env_sample(const ors_scene *scene, double ua, double ub, double w[3]) {
  ors_params p;
  memset(&p, 0, sizeof p);
  p.alpha_min = 1.0 / 255.0; p.support_sigma = 3.0;
  world wd;
  ors_scene s = *scene;
  s.n = 0;
  build_world(&wd, &s, &p);
  double r = env_sample_m(&wd, ua, ub, w, NULL);
  free_world(&wd);
  return r;
}

void ors_env_lookup(const ors_scene *scene, const double w[3], double rgb[3]) {
  env_eval(scene->env, scene->env_h, scene->env_w, w, rgb);
}

/* ------------------------------------------------------------------------ */
/* ray-surfel candidates, depth sort and k-truncation (Sec. 3.2)             */
/* ------------------------------------------------------------------------ */
typedef struct { double t, rho2, rho2max; int64_t i; int flip, valid, in3s; } cand;
typedef struct { cand *c; int64_t n, cap; } cbuf;

static void cbuf_push(cbuf *b, cand c) {
  if (b->n == b->cap) {
    b->cap = b->cap ? 2 * b->cap : 1024;
    b->c = (cand *)realloc(b->c, sizeof(cand) * b->cap);
  }
  b->c[b->n++] = c;
}

static int cand_cmp(const void *pa, const void *pb) {
  const cand *a = (const cand *)pa, *b = (const cand *)pb;
  if (a->t < b->t) return -1;
  if (a->t > b->t) return 1;
  return (a->i > b->i) - (a->i < b->i);
}

typedef struct { int nh; int64_t idx[KMAX]; int flip[KMAX]; } hitlist;

typedef struct { double tgap, rho, tmin; double touch; } trace_stats;

/* Every surfel is tested: plane intersection t = n.(mu-o)/(n.d), hit point
 * projected on the tangent axes and divided by the scales (xi), kept iff
 * t > t_min and rho^2 = |xi|^2 <= rho^2_max.  Kept hits are sorted by
 * (t, index) and the first k form the hit list. */
static void trace_decide(const world *w, const double *o, const double *d, int k, cbuf *buf,
                         hitlist *hl, trace_stats *st) {
  const ors_params *p = w->p;
  double sig2 = p->support_sigma * p->support_sigma;
  buf->n = 0;
  for (int64_t i = 0; i < w->n; ++i) {
    const wsurf *s = &w->ws[i];
    double den = dot3(s->n, d);
    if (fabs(den) < 1e-12) continue;
    double rel[3] = {s->mu[0] - o[0], s->mu[1] - o[1], s->mu[2] - o[2]};
    double t = dot3(s->n, rel) / den;
    double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
    double dl[3] = {x[0] - s->mu[0], x[1] - s->mu[1], x[2] - s->mu[2]};
    double xu = dot3(dl, s->tu) / s->su, xv = dot3(dl, s->tv) / s->sv;
    double rho2 = xu * xu + xv * xv;
    /* keep everything near the support for the margin bookkeeping */
    if (rho2 > (s->rho2max > sig2 ? s->rho2max : sig2) + 1.0) continue;
    cand c;
    c.t = t; c.rho2 = rho2; c.rho2max = s->rho2max; c.i = i; c.flip = den > 0.0;
    c.valid = (t > p->t_min) && (rho2 <= s->rho2max);
    c.in3s = rho2 <= sig2;
    cbuf_push(buf, c);
  }
  /* sort valid ones by (t, index) */
  int64_t nv = 0;
  for (int64_t j = 0; j < buf->n; ++j)
    if (buf->c[j].valid) { cand tmp = buf->c[nv]; buf->c[nv] = buf->c[j]; buf->c[j] = tmp; ++nv; }
  qsort(buf->c, nv, sizeof(cand), cand_cmp);
  hl->nh = (int)(nv < k ? nv : k);
  for (int j = 0; j < hl->nh; ++j) { hl->idx[j] = buf->c[j].i; hl->flip[j] = buf->c[j].flip; }
  if (st) {
    double tk = nv >= k ? buf->c[k - 1].t : INFINITY;
    double tcut = nv > k ? buf->c[k].t : INFINITY;
    int64_t lim = nv < k + 1 ? nv : k + 1;
    for (int64_t j = 0; j + 1 < lim; ++j) {
      double g = buf->c[j + 1].t - buf->c[j].t;
      if (g > 0.0) st->tgap = dmin(st->tgap, g);
    }
    for (int64_t j = 0; j < buf->n; ++j) {
      const cand *c = &buf->c[j];
      if (c->t <= tcut) {
        if (c->t > p->t_min) st->rho = dmin(st->rho, fabs(c->rho2 - c->rho2max));
        if (c->rho2 <= c->rho2max) st->tmin = dmin(st->tmin, fabs(c->t - p->t_min));
      }
      if (c->in3s && c->t > p->t_min && c->t <= tk) st->touch += 1.0;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* front-to-back compositing into a surface record (Eq. surface-record)      */
/* ------------------------------------------------------------------------ */
typedef struct {
  double t, x[3], dl[3], xu, xv, rho2, g, raw, at;
  int capped;
  double nrm[3]; /* world normal turned to face the ray */
  double a[3], m, r;
  double T;      /* transmittance in front of this hit */
} hitv;

typedef struct {
  double A, T, depth, x[3], N[3], nl, n[3], a[3], m, r, inv;
  double Zt, Zn[3], Za[3], Zm, Zr;
} record;

static void composite(const world *w, const hitlist *hl, const double *o, const double *d, hitv *hv, record *rc) {
  const ors_params *p = w->p;
  const ors_scene *sc = w->sc;
  double T = 1.0, A = 0.0, Zt = 0.0, Zx[3] = {0, 0, 0}, Zn[3] = {0, 0, 0}, Za[3] = {0, 0, 0}, Zm = 0.0, Zr = 0.0;
  for (int j = 0; j < hl->nh; ++j) {
    int64_t i = hl->idx[j];
    const wsurf *s = &w->ws[i];
    hitv *h = &hv[j];
    double den = dot3(s->n, d);
    double rel[3] = {s->mu[0] - o[0], s->mu[1] - o[1], s->mu[2] - o[2]};
    h->t = dot3(s->n, rel) / den;
    for (int c = 0; c < 3; ++c) { h->x[c] = o[c] + h->t * d[c]; h->dl[c] = h->x[c] - s->mu[c]; }
    h->xu = dot3(h->dl, s->tu) / s->su;
    h->xv = dot3(h->dl, s->tv) / s->sv;
    h->rho2 = h->xu * h->xu + h->xv * h->xv;
    /* effective opacity (Eq. gaussian-response), capped at alpha_cap */
    h->g = exp(-0.5 * h->rho2);
    h->raw = s->alpha * h->g;
    h->capped = h->raw > p->alpha_cap;
    h->at = h->capped ? p->alpha_cap : h->raw;
    double sg = hl->flip[j] ? -1.0 : 1.0;
    for (int c = 0; c < 3; ++c) h->nrm[c] = sg * s->n[c];
    for (int c = 0; c < 3; ++c) h->a[c] = sc->albedo[3 * i + c];
    h->m = sc->metallic[i];
    h->r = sc->roughness[i];
    h->T = T;
    double wj = T * h->at;
    A += wj;
    Zt += wj * h->t;
    for (int c = 0; c < 3; ++c) { Zx[c] += wj * h->x[c]; Zn[c] += wj * h->nrm[c]; Za[c] += wj * h->a[c]; }
    Zm += wj * h->m;
    Zr += wj * h->r;
    T *= (1.0 - h->at);
  }
  rc->A = A; rc->T = T;
  rc->inv = 1.0 / (A + p->eps);
  rc->Zt = Zt; rc->Zm = Zm; rc->Zr = Zr;
  rc->depth = Zt * rc->inv;
  for (int c = 0; c < 3; ++c) {
    rc->Zn[c] = Zn[c]; rc->Za[c] = Za[c];
    rc->x[c] = Zx[c] * rc->inv; rc->N[c] = Zn[c] * rc->inv; rc->a[c] = Za[c] * rc->inv;
  }
  rc->m = Zm * rc->inv;
  rc->r = Zr * rc->inv;
  rc->nl = sqrt(dot3(rc->N, rc->N));
  for (int c = 0; c < 3; ++c) rc->n[c] = (hl->nh > 0 && rc->nl > 0.0) ? rc->N[c] / rc->nl : 0.0;
}

/* ------------------------------------------------------------------------ */
/* decisions of one primary path (frozen under path replay)                 */
/* ------------------------------------------------------------------------ */
typedef struct {
  int live;
  double w[3];      /* sampled direction */
  double K;         /* MIS weight over (technique probability x pdf) */
  double tw;        /* weight of the T2 E(w) term (its MIS weight in the two-ray form, else 1) */
  double T2;        /* transmittance of the secondary trace */
  double ce[3], cb[3]; /* A2 x (frozen non-env factors) of the two secondary env samples */
  double we[3], wb[3];
  int has_e, has_b;
} samp;

typedef struct {
  hitlist hl;
  samp *s; /* [J] one per slot */
  double margins[ORS_NMARGIN];
  double counts[ORS_NCOUNT];
  hitlist *shl; /* [J] secondary hit lists (for inspection) */
  double *sA2;  /* [J] */
} frozen;

/* secondary-ray slots per primary ray: S, or 2S for the two-ray form */
static int n_slots(const ors_params *p) { return p->spp * ((p->flags & ORS_NEE) ? 2 : 1); }

/* Primary direction of slot j and its frozen weights (Eq. path-estimator,
 * power heuristic).  One-ray form (slot = sample s): technique by u0 with
 * probabilities (c_env, c_bsdf), K = c_t p_t / ((c_env p_e)^2 + (c_bsdf p_b)^2),
 * tw = 1.  Two-ray form (Sec. 4.2: one environment next-event sample and one
 * BSDF continuation per path sample s = j/2, both always drawn): slot 2s
 * samples the environment (dims 9, 10), K = p_e / (p_e^2 + p_b^2), tw = 1;
 * slot 2s+1 samples the cosine/GGX mixture (dims 1-3), K = 1/p_b and the
 * escaping term T2 E(w) carries tw = p_b^2 / (p_e^2 + p_b^2), while the
 * indirect term at its secondary hit is not MIS-weighted.  Returns 0 for a
 * dead slot. */
static int sample_slot(const world *w, const record *rc, const double *wo, int64_t ray_id, int j, frozen *fz,
                       samp *sp) {
  const ors_params *p = w->p;
  const int nee = (p->flags & ORS_NEE) != 0;
  const int s = nee ? j / 2 : j;
  const int kind = nee ? 1 + (j & 1) : 0; /* 0 one-ray, 1 next-event, 2 continuation */
  double qs = q_spec(rc->a, rc->m, p->flags);
  double pe = 0.0, pb = 0.0;
  int use_env;
  if (kind == 0) {
    use_env = draw(p, ray_id, s, 0) < w->c_env;
  } else {
    use_env = kind == 1;
    if (use_env && !(w->c_env > 0.0)) return 0;
  }
  if (use_env) {
    const uint32_t da = kind == 1 ? 9 : 2;
    pe = env_sample_m(w, draw(p, ray_id, s, da), draw(p, ray_id, s, da + 1), sp->w,
                      &fz->margins[ORS_M_ENV]);
  } else {
    double u1 = draw(p, ray_id, s, 1);
    if (qs > 0.0 && qs < 1.0) fz->margins[ORS_M_LOBE] = dmin(fz->margins[ORS_M_LOBE], fabs(u1 - qs));
    sample_lobe(rc->n, wo, rc->r, u1 < qs, draw(p, ray_id, s, 2), draw(p, ray_id, s, 3),
                sp->w);
  }
  double cosw = dot3(rc->n, sp->w);
  fz->margins[ORS_M_COS] = dmin(fz->margins[ORS_M_COS], fabs(cosw));
  if (!(cosw > 0.0)) return 0;
  pb = ors_pdf_bsdf(rc->n, sp->w, wo, rc->a, rc->m, rc->r, p->flags);
  if (!use_env) pe = w->c_env > 0.0 ? env_pdf_m(w, sp->w, &fz->margins[ORS_M_ENV]) : 0.0;
  double pt = use_env ? pe : pb;
  if (!(pt > 0.0)) return 0;
  sp->tw = 1.0;
  if (kind == 0) {
    double ct = use_env ? w->c_env : w->c_bsdf;
    double den = (w->c_env * pe) * (w->c_env * pe) + (w->c_bsdf * pb) * (w->c_bsdf * pb);
    sp->K = ct * pt / den;
  } else if (kind == 1) {
    sp->K = pe / (pe * pe + pb * pb);
  } else {
    sp->K = 1.0 / pb;
    sp->tw = pb * pb / (pe * pe + pb * pb);
  }
  return 1;
}

static void decide(const world *w, const double *o, const double *d, int64_t ray_id, cbuf *buf, frozen *fz) {
  const ors_params *p = w->p;
  for (int m = 0; m < ORS_NMARGIN; ++m) fz->margins[m] = INFINITY;
  for (int c = 0; c < ORS_NCOUNT; ++c) fz->counts[c] = 0.0;
  trace_stats st = {INFINITY, INFINITY, INFINITY, 0.0};
  trace_decide(w, o, d, p->k, buf, &fz->hl, &st);
  fz->margins[ORS_M_TGAP_PRI] = st.tgap;
  fz->margins[ORS_M_RHO_PRI] = st.rho;
  fz->margins[ORS_M_TMIN] = st.tmin;
  fz->counts[ORS_C_TOUCH_PRI] = st.touch;
  fz->counts[ORS_C_COMP_PRI] = fz->hl.nh;
  if (!(p->flags & ORS_NO_BACKGROUND)) fz->counts[ORS_C_ENV] += 1.0;
  hitv hv[KMAX];
  record rc;
  composite(w, &fz->hl, o, d, hv, &rc);
  double wo[3] = {-d[0], -d[1], -d[2]};
  trace_stats st2 = {INFINITY, INFINITY, INFINITY, 0.0};
  const int J = n_slots(p);
  for (int j = 0; j < J; ++j) {
    samp *sp = &fz->s[j];
    memset(sp, 0, sizeof *sp);
    sp->T2 = 1.0;
    sp->tw = 1.0;
    fz->shl[j].nh = 0;
    fz->sA2[j] = -1.0;
    if (fz->hl.nh == 0) continue;
    if (!sample_slot(w, &rc, wo, ray_id, j, fz, sp)) continue;
    sp->live = 1;
    fz->counts[ORS_C_ENV] += 1.0;
    const int s = (p->flags & ORS_NEE) ? j / 2 : j;               /* path sample (uniform stream) */
    const int indirect = !(p->flags & ORS_NEE) || (j & 1);        /* next-event rays see only E */
    if (p->flags & ORS_NO_SECONDARY) continue;
    /* one secondary ray: visibility and indirect path at once */
    double o2[3];
    for (int c = 0; c < 3; ++c) o2[c] = rc.x[c] + p->secondary_offset * rc.n[c];
    hitlist *hl2 = &fz->shl[j];
    trace_decide(w, o2, sp->w, p->k, buf, hl2, &st2);
    fz->counts[ORS_C_SEC_RAYS] += 1.0;
    fz->counts[ORS_C_COMP_SEC] += hl2->nh;
    hitv hv2[KMAX];
    record r2;
    composite(w, hl2, o2, sp->w, hv2, &r2);
    sp->T2 = r2.T;
    fz->sA2[j] = r2.A;
    if (hl2->nh == 0 || !indirect) continue;
    /* two unshadowed environment samples at the secondary record, combined by
     * the two-sample power heuristic */
    double wo2[3] = {-sp->w[0], -sp->w[1], -sp->w[2]};
    if (w->c_env > 0.0) {
      double u4 = draw(p, ray_id, s, 4), u5 = draw(p, ray_id, s, 5);
      double pe2 = env_sample_m(w, u4, u5, sp->we, &fz->margins[ORS_M_ENV]);
      double c2 = dot3(r2.n, sp->we);
      fz->margins[ORS_M_COS] = dmin(fz->margins[ORS_M_COS], fabs(c2));
      if (c2 > 0.0 && pe2 > 0.0) {
        double f2[3];
        ors_brdf(r2.n, sp->we, wo2, r2.a, r2.m, r2.r, p->flags, f2);
        double pb2 = ors_pdf_bsdf(r2.n, sp->we, wo2, r2.a, r2.m, r2.r, p->flags);
        double wgt = pe2 * pe2 / (pe2 * pe2 + pb2 * pb2);
        for (int c = 0; c < 3; ++c) sp->ce[c] = r2.A * wgt * f2[c] * c2 / pe2;
        sp->has_e = 1;
        fz->counts[ORS_C_ENV] += 1.0;
      }
    }
    {
      double u6 = draw(p, ray_id, s, 6), u7 = draw(p, ray_id, s, 7),
             u8 = draw(p, ray_id, s, 8);
      double qs2 = q_spec(r2.a, r2.m, p->flags);
      if (qs2 > 0.0 && qs2 < 1.0) fz->margins[ORS_M_LOBE] = dmin(fz->margins[ORS_M_LOBE], fabs(u6 - qs2));
      sample_lobe(r2.n, wo2, r2.r, u6 < qs2, u7, u8, sp->wb);
      double c2 = dot3(r2.n, sp->wb);
      fz->margins[ORS_M_COS] = dmin(fz->margins[ORS_M_COS], fabs(c2));
      if (c2 > 0.0) {
        double pb2 = ors_pdf_bsdf(r2.n, sp->wb, wo2, r2.a, r2.m, r2.r, p->flags);
        double pe2 = w->c_env > 0.0 ? env_pdf_m(w, sp->wb, &fz->margins[ORS_M_ENV]) : 0.0;
        if (pb2 > 0.0) {
          double f2[3];
          ors_brdf(r2.n, sp->wb, wo2, r2.a, r2.m, r2.r, p->flags, f2);
          double wgt = pb2 * pb2 / (pe2 * pe2 + pb2 * pb2);
          for (int c = 0; c < 3; ++c) sp->cb[c] = r2.A * wgt * f2[c] * c2 / pb2;
          sp->has_b = 1;
          fz->counts[ORS_C_ENV] += 1.0;
        }
      }
    }
  }
  fz->margins[ORS_M_TGAP_SEC] = st2.tgap;
  fz->margins[ORS_M_RHO_SEC] = st2.rho;
  fz->margins[ORS_M_TMIN] = dmin(fz->margins[ORS_M_TMIN], st2.tmin);
  fz->counts[ORS_C_TOUCH_SEC] = st2.touch;
}

/* ------------------------------------------------------------------------ */
/* evaluation of a frozen path and its adjoint                              */
/* ------------------------------------------------------------------------ */
/* fcos = f(wi,wo) * (n.wi) for a frozen live sample (no hemisphere test) */
static void fcos_eval(const double *n, const double *wi, const double *wo, const double *a, double m, double r,
                      uint32_t flags, double *fc) {
  double ci = dot3(n, wi);
  for (int c = 0; c < 3; ++c) fc[c] = (1.0 - m) * a[c] * INV_PI * ci;
  if (flags & ORS_DIFFUSE_ONLY) return;
  spec_t s;
  spec_setup(n, wi, wo, r, &s);
  double sc = s.D * s.G1i * s.G1o / (4.0 * s.co);
  for (int c = 0; c < 3; ++c) {
    double F0 = 0.04 * (1.0 - m) + a[c] * m;
    fc[c] += sc * (F0 + (1.0 - F0) * s.P);
  }
}

/* reverse of fcos_eval: accumulates into gn (w.r.t. the unit normal), ga, gm, gr */
static void fcos_bwd(const double *n, const double *wi, const double *wo, const double *a, double m, double r,
                     uint32_t flags, const double *gfc, double *gn, double *ga, double *gm, double *gr) {
  double ci = dot3(n, wi);
  double gci = 0.0;
  for (int c = 0; c < 3; ++c) {
    ga[c] += gfc[c] * (1.0 - m) * INV_PI * ci;
    *gm += -gfc[c] * a[c] * INV_PI * ci;
    gci += gfc[c] * (1.0 - m) * a[c] * INV_PI;
  }
  if (!(flags & ORS_DIFFUSE_ONLY)) {
    spec_t s;
    spec_setup(n, wi, wo, r, &s);
    double h[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
    double hl = sqrt(dot3(h, h));
    for (int i = 0; i < 3; ++i) h[i] /= hl;
    double a2 = s.alpha2;
    double sc = s.D * s.G1i * s.G1o / (4.0 * s.co);
    /* g_sc = sum_c gfc_c * F_c ; F_c = F0_c (1-P) + P ; F0_c = 0.04(1-m) + a_c m */
    double gsc = 0.0;
    for (int c = 0; c < 3; ++c) {
      double F0 = 0.04 * (1.0 - m) + a[c] * m;
      double F = F0 + (1.0 - F0) * s.P;
      gsc += gfc[c] * F;
      double gF0 = gfc[c] * sc * (1.0 - s.P);
      ga[c] += gF0 * m;
      *gm += gF0 * (a[c] - 0.04);
    }
    /* sc = D(ch, a2) G1(ci, a2) G1(co, a2) / (4 co) */
    double u = s.ch * s.ch * (a2 - 1.0) + 1.0;
    double dD_dch = -4.0 * a2 * s.ch * (a2 - 1.0) / (PI * u * u * u);
    double dD_da2 = (u - 2.0 * a2 * s.ch * s.ch) / (PI * u * u * u);
    double si = sqrt(a2 + (1.0 - a2) * s.ci * s.ci), so = sqrt(a2 + (1.0 - a2) * s.co * s.co);
    double dG1i_dc = 2.0 * a2 / (si * (s.ci + si) * (s.ci + si));
    double dG1o_dc = 2.0 * a2 / (so * (s.co + so) * (s.co + so));
    double dG1i_da2 = -s.ci * (1.0 - s.ci * s.ci) / (si * (s.ci + si) * (s.ci + si));
    double dG1o_da2 = -s.co * (1.0 - s.co * s.co) / (so * (s.co + so) * (s.co + so));
    double gch = gsc * dD_dch * s.G1i * s.G1o / (4.0 * s.co);
    gci += gsc * s.D * dG1i_dc * s.G1o / (4.0 * s.co);
    double gco = gsc * s.D * s.G1i * (dG1o_dc * s.co - s.G1o) / (4.0 * s.co * s.co);
    double ga2 = gsc * (dD_da2 * s.G1i * s.G1o + s.D * (dG1i_da2 * s.G1o + s.G1i * dG1o_da2)) / (4.0 * s.co);
    if (!s.r_clamped) *gr += ga2 * 4.0 * s.reff * s.reff * s.reff;
    for (int i = 0; i < 3; ++i) gn[i] += gco * wo[i] + gch * h[i];
  }
  for (int i = 0; i < 3; ++i) gn[i] += gci * wi[i];
}

typedef struct {
  double L[3], depth, normal[3], alpha, T;
} pixel;

/* value of the frozen path at the live parameters held by `w` */
static void evaluate(const world *w, const frozen *fz, const double *o, const double *d, hitv *hv, record *rc,
                     double (*Ls)[3], double (*fcs)[3], double (*Lins)[3], pixel *px) {
  const ors_params *p = w->p;
  const ors_scene *sc = w->sc;
  composite(w, &fz->hl, o, d, hv, rc);
  double wo[3] = {-d[0], -d[1], -d[2]};
  double Lsurf[3] = {0, 0, 0};
  const int J = n_slots(p);
  for (int s = 0; s < J; ++s) {
    const samp *sp = &fz->s[s];
    Ls[s][0] = Ls[s][1] = Ls[s][2] = 0.0;
    if (!sp->live) continue;
    double E[3], Ee[3] = {0, 0, 0}, Eb[3] = {0, 0, 0};
    env_eval(sc->env, sc->env_h, sc->env_w, sp->w, E);
    if (sp->has_e) env_eval(sc->env, sc->env_h, sc->env_w, sp->we, Ee);
    if (sp->has_b) env_eval(sc->env, sc->env_h, sc->env_w, sp->wb, Eb);
    fcos_eval(rc->n, sp->w, wo, rc->a, rc->m, rc->r, p->flags, fcs[s]);
    for (int c = 0; c < 3; ++c) {
      Lins[s][c] = sp->tw * sp->T2 * E[c] + sp->ce[c] * Ee[c] + sp->cb[c] * Eb[c];
      Ls[s][c] = sp->K * fcs[s][c] * Lins[s][c];
      Lsurf[c] += Ls[s][c];
    }
  }
  double Ed[3] = {0, 0, 0};
  if (!(p->flags & ORS_NO_BACKGROUND)) env_eval(sc->env, sc->env_h, sc->env_w, d, Ed);
  for (int c = 0; c < 3; ++c) px->L[c] = rc->A * (Lsurf[c] / p->spp) + rc->T * Ed[c];
  px->depth = rc->depth;
  for (int c = 0; c < 3; ++c) px->normal[c] = rc->n[c];
  px->alpha = rc->A;
  px->T = rc->T;
}

/* rows of d(rot(q))/d(w,x,y,z) contracted with G (row-major 3x3) */
static void quat_matrix_bwd(const double *q, const double *G, double *gq) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  /* dM/dw */
  gq[0] = G[1] * (-2 * z) + G[2] * (2 * y) + G[3] * (2 * z) + G[5] * (-2 * x) + G[6] * (-2 * y) + G[7] * (2 * x);
  /* dM/dx */
  gq[1] = G[1] * (2 * y) + G[2] * (2 * z) + G[3] * (2 * y) + G[4] * (-4 * x) + G[5] * (-2 * w) + G[6] * (2 * z) +
          G[7] * (2 * w) + G[8] * (-4 * x);
  /* dM/dy */
  gq[2] = G[0] * (-4 * y) + G[1] * (2 * x) + G[2] * (2 * w) + G[3] * (2 * x) + G[5] * (2 * z) + G[6] * (-2 * w) +
          G[7] * (2 * z) + G[8] * (-4 * y);
  /* dM/dz */
  gq[3] = G[0] * (-4 * z) + G[1] * (-2 * w) + G[2] * (2 * x) + G[3] * (2 * w) + G[4] * (-4 * z) + G[5] * (2 * y) +
          G[6] * (2 * x) + G[7] * (2 * y);
}

static inline void atomic_add(double *p, double v) {
#pragma omp atomic
  *p += v;
}

/* reverse mode of evaluate() at the frozen path's own parameters */
static void evaluate_bwd(const world *w, const frozen *fz, const double *o, const double *d, const double *gL,
                         double gdepth, const double *gnormal, double galpha, ors_grads *g) {
  const ors_params *p = w->p;
  const ors_scene *sc = w->sc;
  int S = p->spp, J = n_slots(p);
  hitv hv[KMAX];
  record rc;
  double (*Ls)[3] = (double (*)[3])malloc(sizeof(double) * 3 * J);
  double (*fcs)[3] = (double (*)[3])malloc(sizeof(double) * 3 * J);
  double (*Lins)[3] = (double (*)[3])malloc(sizeof(double) * 3 * J);
  pixel px;
  evaluate(w, fz, o, d, hv, &rc, Ls, fcs, Lins, &px);
  double wo[3] = {-d[0], -d[1], -d[2]};
  int H = sc->env_h, W = sc->env_w;
  /* L = A * Lsurf / S + T * E(d) */
  double gA = galpha, gT = 0.0;
  if (!(p->flags & ORS_NO_BACKGROUND)) {
    double Ed[3], ge[3];
    env_eval(sc->env, H, W, d, Ed);
    for (int c = 0; c < 3; ++c) { gT += gL[c] * Ed[c]; ge[c] = gL[c] * rc.T; }
    env_scatter(g->env, H, W, d, ge);
  }
  double gn[3] = {gnormal[0], gnormal[1], gnormal[2]}, ga[3] = {0, 0, 0}, gm = 0.0, gr = 0.0;
  for (int s = 0; s < J; ++s) {
    const samp *sp = &fz->s[s];
    if (!sp->live) continue;
    double gF[3], gfc[3], gLin[3];
    for (int c = 0; c < 3; ++c) {
      gA += gL[c] * Ls[s][c] / S;
      gF[c] = gL[c] * rc.A / S;
      gfc[c] = gF[c] * sp->K * Lins[s][c];
      gLin[c] = gF[c] * sp->K * fcs[s][c];
    }
    double ge[3];
    for (int c = 0; c < 3; ++c) ge[c] = gLin[c] * sp->tw * sp->T2;
    env_scatter(g->env, H, W, sp->w, ge);
    if (sp->has_e) { for (int c = 0; c < 3; ++c) ge[c] = gLin[c] * sp->ce[c]; env_scatter(g->env, H, W, sp->we, ge); }
    if (sp->has_b) { for (int c = 0; c < 3; ++c) ge[c] = gLin[c] * sp->cb[c]; env_scatter(g->env, H, W, sp->wb, ge); }
    fcos_bwd(rc.n, sp->w, wo, rc.a, rc.m, rc.r, p->flags, gfc, gn, ga, &gm, &gr);
  }
  free(Ls); free(fcs); free(Lins);
  int nh = fz->hl.nh;
  if (nh == 0) return;
  /* normalisation n = N / |N| */
  double gN[3] = {0, 0, 0};
  if (rc.nl > 0.0) {
    double ng = dot3(rc.n, gn);
    for (int c = 0; c < 3; ++c) gN[c] = (gn[c] - rc.n[c] * ng) / rc.nl;
  }
  /* z_bar = Z * inv, inv = 1/(A+eps) */
  double inv = rc.inv;
  double gZt = gdepth * inv, gZn[3], gZa[3], gZm = gm * inv, gZr = gr * inv;
  double ginv = gdepth * rc.Zt + gm * rc.Zm + gr * rc.Zr;
  for (int c = 0; c < 3; ++c) {
    gZn[c] = gN[c] * inv; gZa[c] = ga[c] * inv;
    ginv += gN[c] * rc.Zn[c] + ga[c] * rc.Za[c];
  }
  gA += -ginv * inv * inv;
  /* compositing adjoint: with v_j = gA + sum_z gZ . z_j and suffix
   * V_j = sum_{i>j} w_i v_i, d/d(alpha_j) = T_j v_j - (V_j + gT T)/(1-alpha_j) */
  double V = 0.0;
  for (int j = nh - 1; j >= 0; --j) {
    hitv *h = &hv[j];
    int64_t i = fz->hl.idx[j];
    const wsurf *s = &w->ws[i];
    double wj = h->T * h->at;
    double vj = gA + gZt * h->t + gZm * h->m + gZr * h->r + dot3(gZn, h->nrm) + dot3(gZa, h->a);
    double gat = h->T * vj - (V + gT * rc.T) / (1.0 - h->at);
    V += wj * vj;
    /* attribute gradients */
    double gt = gZt * wj;
    double gnrm[3];
    for (int c = 0; c < 3; ++c) gnrm[c] = gZn[c] * wj;
    for (int c = 0; c < 3; ++c) atomic_add(&g->albedo[3 * i + c], gZa[c] * wj);
    atomic_add(&g->metallic[i], gZm * wj);
    atomic_add(&g->roughness[i], gZr * wj);
    /* effective opacity: alpha_t = min(cap, alpha exp(-rho^2/2)) */
    double graw = h->capped ? 0.0 : gat;
    atomic_add(&g->opacity[i], graw * h->g);
    double grho2 = graw * s->alpha * h->g * (-0.5);
    double gxu = grho2 * 2.0 * h->xu, gxv = grho2 * 2.0 * h->xv;
    atomic_add(&g->scale[2 * i + 0], -gxu * h->xu / s->su);
    atomic_add(&g->scale[2 * i + 1], -gxv * h->xv / s->sv);
    double gdl[3], gtu[3], gtv[3], gmu[3], gnw[3];
    for (int c = 0; c < 3; ++c) {
      gdl[c] = gxu * s->tu[c] / s->su + gxv * s->tv[c] / s->sv;
      gtu[c] = gxu * h->dl[c] / s->su;
      gtv[c] = gxv * h->dl[c] / s->sv;
    }
    /* dl = x - mu, x = o + t d */
    for (int c = 0; c < 3; ++c) gmu[c] = -gdl[c];
    gt += dot3(gdl, d);
    /* t = n.(mu - o)/(n.d) */
    double den = dot3(s->n, d);
    double sg = fz->hl.flip[j] ? -1.0 : 1.0;
    for (int c = 0; c < 3; ++c) {
      gmu[c] += gt * s->n[c] / den;
      gnw[c] = -gt * h->dl[c] / den + sg * gnrm[c];
    }
    /* world frame F = R_o * rot(qh); columns (t_u, t_v, n); mu' = R_o mu + t_o */
    double Gw[9], G[9];
    for (int r = 0; r < 3; ++r) { Gw[3 * r + 0] = gtu[r]; Gw[3 * r + 1] = gtv[r]; Gw[3 * r + 2] = gnw[r]; }
    double gmo[3];
    if (s->obj >= 0) {
      const double *Ro = w->R + 9 * s->obj;
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) G[3 * r + c] = Ro[0 + r] * Gw[0 + c] + Ro[3 + r] * Gw[3 + c] + Ro[6 + r] * Gw[6 + c];
      for (int r = 0; r < 3; ++r) gmo[r] = Ro[0 + r] * gmu[0] + Ro[3 + r] * gmu[1] + Ro[6 + r] * gmu[2];
    } else {
      memcpy(G, Gw, sizeof G);
      memcpy(gmo, gmu, sizeof gmo);
    }
    for (int c = 0; c < 3; ++c) atomic_add(&g->mu[3 * i + c], gmo[c]);
    double gqh[4];
    quat_matrix_bwd(s->qh, G, gqh);
    double pq = gqh[0] * s->qh[0] + gqh[1] * s->qh[1] + gqh[2] * s->qh[2] + gqh[3] * s->qh[3];
    for (int c = 0; c < 4; ++c) atomic_add(&g->q[4 * i + c], (gqh[c] - s->qh[c] * pq) / s->qlen);
  }
}

/* ------------------------------------------------------------------------ */
/* public entry points                                                      */
/* ------------------------------------------------------------------------ */
static int check(const ors_scene *sc, const ors_rays *r, const ors_params *p) {
  if (!sc || !r || !p) return -1;
  if (p->k < 1 || p->k > KMAX || p->spp < 1) return -2;
  if (sc->n < 0 || sc->n_objects < 0 || !sc->object_offset) return -3;
  if (sc->env_h < 1 || sc->env_w < 1 || !sc->env) return -4;
  if (sc->object_offset[0] != 0 || sc->object_offset[sc->n_objects + 1] != sc->n) return -5;
  return 0;
}

static void frozen_alloc(frozen *f, int S) {
  f->s = (samp *)calloc(S, sizeof(samp));
  f->shl = (hitlist *)calloc(S, sizeof(hitlist));
  f->sA2 = (double *)calloc(S, sizeof(double));
}
static void frozen_free(frozen *f) { free(f->s); free(f->shl); free(f->sA2); }

static void write_out(const ors_params *p, const frozen *fz, const pixel *px, int64_t r, ors_outputs *out) {
  int k = p->k, S = n_slots(p);
  if (out->radiance) for (int c = 0; c < 3; ++c) out->radiance[3 * r + c] = px->L[c];
  if (out->depth) out->depth[r] = px->depth;
  if (out->normal) for (int c = 0; c < 3; ++c) out->normal[3 * r + c] = px->normal[c];
  if (out->alpha) out->alpha[r] = px->alpha;
  if (out->transmittance) out->transmittance[r] = px->T;
  if (out->hit_idx)
    for (int j = 0; j < k; ++j) out->hit_idx[(int64_t)r * k + j] = j < fz->hl.nh ? (int32_t)fz->hl.idx[j] : -1;
  if (out->sec_hit_idx)
    for (int s = 0; s < S; ++s)
      for (int j = 0; j < k; ++j)
        out->sec_hit_idx[((int64_t)r * S + s) * k + j] = j < fz->shl[s].nh ? (int32_t)fz->shl[s].idx[j] : -1;
  if (out->sec_alpha) for (int s = 0; s < S; ++s) out->sec_alpha[(int64_t)r * S + s] = fz->sA2[s];
  if (out->margins) for (int m = 0; m < ORS_NMARGIN; ++m) out->margins[(int64_t)r * ORS_NMARGIN + m] = fz->margins[m];
  if (out->counts) for (int c = 0; c < ORS_NCOUNT; ++c) out->counts[(int64_t)r * ORS_NCOUNT + c] = fz->counts[c];
}

static int render_impl(const ors_scene *sc0, const ors_scene *sc, const ors_rays *rays, const ors_params *p,
                       ors_outputs *out, int n_threads) {
  int rcode = check(sc0, rays, p);
  if (rcode) return rcode;
  if ((rcode = check(sc, rays, p))) return rcode;
  if (sc->n != sc0->n || sc->env_h != sc0->env_h || sc->env_w != sc0->env_w) return -6;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
  world w0, w1;
  build_world(&w0, sc0, p);
  int same = (sc == sc0);
  if (!same) build_world(&w1, sc, p);
  const world *wl = same ? &w0 : &w1;
#pragma omp parallel
  {
    cbuf buf = {0, 0, 0};
    frozen fz;
    frozen_alloc(&fz, n_slots(p));
    hitv hv[KMAX];
    record rc;
    double (*Ls)[3] = (double (*)[3])malloc(sizeof(double) * 3 * n_slots(p));
    double (*fcs)[3] = (double (*)[3])malloc(sizeof(double) * 3 * n_slots(p));
    double (*Lins)[3] = (double (*)[3])malloc(sizeof(double) * 3 * n_slots(p));
#pragma omp for schedule(dynamic, 4)
    for (int64_t r = 0; r < rays->n; ++r) {
      const double *o = rays->o + 3 * r, *d = rays->d + 3 * r;
      decide(&w0, o, d, rays->id[r], &buf, &fz);
      pixel px;
      evaluate(wl, &fz, o, d, hv, &rc, Ls, fcs, Lins, &px);
      write_out(p, &fz, &px, r, out);
    }
    free(Ls); free(fcs); free(Lins);
    frozen_free(&fz);
    free(buf.c);
  }
  free_world(&w0);
  if (!same) free_world(&w1);
  return 0;
}

int ors_render(const ors_scene *scene, const ors_rays *rays, const ors_params *p, ors_outputs *out, int n_threads) {
  return render_impl(scene, scene, rays, p, out, n_threads);
}

int ors_frozen_eval(const ors_scene *scene0, const ors_scene *scene, const ors_rays *rays, const ors_params *p,
                    ors_outputs *out, int n_threads) {
  return render_impl(scene0, scene, rays, p, out, n_threads);
}

int ors_backward(const ors_scene *sc, const ors_rays *rays, const ors_params *p, const ors_upstream *up,
                 ors_grads *g, int n_threads) {
  int rcode = check(sc, rays, p);
  if (rcode) return rcode;
  if (!up || !g || !g->mu || !g->q || !g->scale || !g->opacity || !g->albedo || !g->roughness || !g->metallic ||
      !g->env)
    return -7;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
  int64_t n = sc->n;
  memset(g->mu, 0, sizeof(double) * 3 * n);
  memset(g->q, 0, sizeof(double) * 4 * n);
  memset(g->scale, 0, sizeof(double) * 2 * n);
  memset(g->opacity, 0, sizeof(double) * n);
  memset(g->albedo, 0, sizeof(double) * 3 * n);
  memset(g->roughness, 0, sizeof(double) * n);
  memset(g->metallic, 0, sizeof(double) * n);
  memset(g->env, 0, sizeof(double) * 3 * (size_t)sc->env_h * sc->env_w);
  world w;
  build_world(&w, sc, p);
#pragma omp parallel
  {
    cbuf buf = {0, 0, 0};
    frozen fz;
    frozen_alloc(&fz, n_slots(p));
#pragma omp for schedule(dynamic, 4)
    for (int64_t r = 0; r < rays->n; ++r) {
      const double *o = rays->o + 3 * r, *d = rays->d + 3 * r;
      decide(&w, o, d, rays->id[r], &buf, &fz);
      double gL[3] = {0, 0, 0}, gn[3] = {0, 0, 0}, gd = 0.0, ga = 0.0;
      if (up->radiance) for (int c = 0; c < 3; ++c) gL[c] = up->radiance[3 * r + c];
      if (up->normal) for (int c = 0; c < 3; ++c) gn[c] = up->normal[3 * r + c];
      if (up->depth) gd = up->depth[r];
      if (up->alpha) ga = up->alpha[r];
      evaluate_bwd(&w, &fz, o, d, gL, gd, gn, ga, g);
    }
    frozen_free(&fz);
    free(buf.c);
  }
  free_world(&w);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* pinhole ray generation in IEEE single precision, fixed operation order    */
/* ------------------------------------------------------------------------ */
float ors_tan_half(float fov_y_deg) { return (float)tan((double)fov_y_deg * PI / 360.0); }

void ors_raygen(const float pose[12], float tan_half, int32_t w, int32_t h, const int64_t *pix, int64_t n,
                float *o, float *d) {
  float fw = (float)w, fh = (float)h;
  float aspect = fw / fh;
  for (int64_t r = 0; r < n; ++r) {
    int64_t px = pix[r] % w, py = pix[r] / w;
    float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    float sx = (2.0f * fx / fw - 1.0f) * tan_half;
    sx = sx * aspect;
    float sy = (1.0f - 2.0f * fy / fh) * tan_half;
    float dx = pose[0] * sx, dy = pose[4] * sx, dz = pose[8] * sx;
    dx = dx + pose[1] * sy; dy = dy + pose[5] * sy; dz = dz + pose[9] * sy;
    dx = dx - pose[2]; dy = dy - pose[6]; dz = dz - pose[10];
    float ss = dx * dx;
    ss = ss + dy * dy;
    ss = ss + dz * dz;
    float len = sqrtf(ss);
    d[3 * r + 0] = dx / len; d[3 * r + 1] = dy / len; d[3 * r + 2] = dz / len;
    o[3 * r + 0] = pose[3]; o[3 * r + 1] = pose[7]; o[3 * r + 2] = pose[11];
  }
}

/*
 * lf_oracle.h -- plain FP64 CPU oracle for one-bounce ray tracing of 2D
 * Gaussian surfels (LightFuse, arXiv 2608.29269).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, brute-force,
 * obviously-correct reference that the GPU library is checked against.  It
 * tests every surfel for every ray (no BVH), computes everything in double
 * precision, and shares no code, header, table or constant generator with the
 * GPU path.  Only tests, the smoke check and the benchmark's CPU-baseline leg
 * may load it.
 *
 * Everything here follows Sec. 3 of the paper:
 *   - surfel tuple and state assembly: Sec. 3.1, Eq. gaussian-primitive and
 *     Eq. state-assembly (rigid transforms act on centres and orientations);
 *   - ray-surfel intersection, effective opacity, cap, support/threshold
 *     culling, depth sort and front-to-back compositing: Sec. 3.2,
 *     Eq. gaussian-response and Eq. surface-record;
 *   - rendering equation, metallic-roughness BRDF, environment next-event
 *     estimation, cosine/GGX BSDF continuation, power-heuristic MIS, at most
 *     one secondary interaction: Sec. 3.3, Eq. rendering-equation and
 *     Eq. path-estimator;
 *   - path replay backpropagation (frozen sampling decisions, gradients through
 *     the primary BRDF and the environment map; geometry gradients through the
 *     compositing rules): Sec. 3.3 (PRB paragraph) and Sec. 3.2.
 * Constants the paper leaves open (support radius 3 sigma, opacity threshold
 * 1/255 tested before the 0.99 cap, epsilon 1e-6, t_min 1e-4, secondary
 * offset 1e-3) are passed in through ors_params so the same values reach both
 * implementations.  The remaining open points are fixed in the source:
 * Lambert + GGX/Smith/Schlick BRDF with F0 = 0.04(1-m) + a m and
 * alpha_g = clamp(r,0.08,1)^2; one-sample power-heuristic MIS over
 * {environment importance sampling, cosine/GGX mixture} with probability 1/2
 * each; one secondary ray per sample that serves as both visibility and
 * indirect path; two unshadowed environment samples (one per technique) at the
 * secondary record; lat-long environment with +Y up; SplitMix64 sampler.
 *
 * All arrays are caller-owned, row-major, contiguous, double precision unless
 * stated.  Functions return 0 on success and a negative value on invalid
 * arguments; they never free caller memory.
 */
#ifndef LF_ORACLE_H
#define LF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* flags (bit meanings identical to the GPU library's parameter flags) */
#define ORS_NO_SECONDARY  (1u << 0) /* shade with unshadowed E(w); trace no secondary ray */
#define ORS_NO_BACKGROUND (1u << 1) /* drop the T*E(d) background term */
#define ORS_BSDF_ONLY     (1u << 2) /* never use environment importance sampling */
#define ORS_DIFFUSE_ONLY  (1u << 3) /* Lambert lobe only (no GGX term, cosine sampling) */
#define ORS_SOBOL         (1u << 8) /* Owen-scrambled Sobol uniforms instead of the hash */
#define ORS_NEE           (1u << 7) /* two rays per path sample: an environment next-event ray and a
                                       cosine/GGX continuation, multi-sample power MIS; outputs indexed
                                       by slot 2s (next-event) and 2s+1 (continuation) */

typedef struct {
  const double *mu;        /* [n,3] centres (object space for object surfels) */
  const double *q;         /* [n,4] quaternion (w,x,y,z), any nonzero norm */
  const double *scale;     /* [n,2] in-plane scales > 0 */
  const double *opacity;   /* [n] */
  const double *albedo;    /* [n,3] */
  const double *roughness; /* [n] */
  const double *metallic;  /* [n] */
  int64_t n;
  int32_t n_objects;            /* M */
  const int64_t *object_offset; /* [M+2]: background [0,off[1]), object o in [off[o+1],off[o+2]) */
  const double *R;              /* [M,3,3] rotation per object (orthonormalised internally) */
  const double *t;              /* [M,3] translation per object */
  const double *env;            /* [env_h,env_w,3] lat-long, row 0 at +Y */
  int32_t env_h, env_w;
} ors_scene;

typedef struct {
  int32_t k;                /* hit-list length, 1..64 */
  int32_t spp;              /* S >= 1 shading samples per primary hit */
  uint64_t seed;            /* sampler seed */
  double alpha_min;         /* opacity threshold (1/255) */
  double alpha_cap;         /* opacity cap (0.99) */
  double support_sigma;     /* finite support radius in sigmas (3) */
  double eps;               /* epsilon of the composite normalisation (1e-6) */
  double t_min;             /* minimum ray parameter (1e-4) */
  double secondary_offset;  /* secondary origin offset along the normal (1e-3) */
  uint32_t flags;
} ors_params;

typedef struct {
  const double *o, *d;  /* [n,3] origins and unit directions */
  const int64_t *id;    /* [n] sampler ray ids */
  int64_t n;
} ors_rays;

/* per-ray decision margins (distance of each discrete decision from its
 * switching point; a tiny margin means a legitimately ambiguous ray) */
enum {
  ORS_M_TGAP_PRI = 0,  /* smallest nonzero gap between consecutive t of the first k+1 primary hits */
  ORS_M_RHO_PRI,       /* smallest |rho^2 - rho^2_max| among primary candidates before the cut */
  ORS_M_TGAP_SEC,      /* same as TGAP_PRI over all secondary traces */
  ORS_M_RHO_SEC,       /* same as RHO_PRI over all secondary traces */
  ORS_M_ENV,           /* smallest distance of a sampler value to a CDF edge / texel edge */
  ORS_M_LOBE,          /* smallest |u_lobe - q_spec| */
  ORS_M_COS,           /* smallest |n.w| of a hemisphere decision */
  ORS_M_TMIN,          /* smallest |t - t_min| of a culled-or-kept candidate */
  ORS_NMARGIN
};
/* per-ray counts used for algorithmic-byte accounting */
enum {
  ORS_C_TOUCH_PRI = 0, /* surfels whose 3-sigma support the primary ray crosses with t <= t_(k) */
  ORS_C_COMP_PRI,      /* composited primary hits */
  ORS_C_SEC_RAYS,      /* secondary rays traced */
  ORS_C_TOUCH_SEC,     /* sum over secondary rays of crossed supports with t <= t_(k) */
  ORS_C_COMP_SEC,      /* sum over secondary rays of composited hits */
  ORS_C_ENV,           /* bilinear environment lookups */
  ORS_NCOUNT
};

typedef struct {
  double *radiance;      /* [n,3] */
  double *depth;         /* [n] */
  double *normal;        /* [n,3] */
  double *alpha;         /* [n] accumulated opacity A */
  double *transmittance; /* [n] final transmittance T, or NULL */
  int32_t *hit_idx;      /* [n,k] primary hit surfel indices in order, -1 padded, or NULL */
  int32_t *sec_hit_idx;  /* [n,S,k] secondary hit lists, -1 padded (all -1 if not traced), or NULL */
  double *sec_alpha;     /* [n,S] A2 of each sample's secondary record (-1: not traced), or NULL */
  double *margins;       /* [n,ORS_NMARGIN] or NULL */
  double *counts;        /* [n,ORS_NCOUNT] or NULL */
} ors_outputs;

typedef struct { const double *radiance, *depth, *normal, *alpha; } ors_upstream; /* NULL = zero */
typedef struct { double *mu, *q, *scale, *opacity, *albedo, *roughness, *metallic, *env; } ors_grads;

/* Forward render of explicit rays.  n_threads <= 0 uses the OpenMP default. */
int ors_render(const ors_scene *scene, const ors_rays *rays, const ors_params *p,
               ors_outputs *out, int n_threads);

/* Frozen objective of path replay: every discrete decision and frozen factor
 * (hit sets and their order, sampled directions, technique and lobe choices,
 * MIS/pdf factors, secondary origins and records, non-environment factors of
 * the secondary estimate) is taken at scene0; every live quantity is evaluated
 * at scene.  scene and scene0 must have the same n, objects and env size. */
int ors_frozen_eval(const ors_scene *scene0, const ors_scene *scene, const ors_rays *rays,
                    const ors_params *p, ors_outputs *out, int n_threads);

/* Hand-written reverse-mode adjoint of ors_frozen_eval at scene0 == scene.
 * Gradients are OVERWRITTEN (zeroed first).  Quaternion gradients are with
 * respect to the raw (unnormalised) q. */
int ors_backward(const ors_scene *scene, const ors_rays *rays, const ors_params *p,
                 const ors_upstream *up, ors_grads *g, int n_threads);

/* Pinhole ray generation, defined in IEEE single precision with a fixed
 * operation order (no fused multiply-add, correctly rounded division and
 * square root) so that it is reproducible bit for bit.  pix[i] = y*w + x. */
void ors_raygen(const float pose[12], float tan_half, int32_t w, int32_t h,
                const int64_t *pix, int64_t n, float *o, float *d);
float ors_tan_half(float fov_y_deg);

/* sampler (SplitMix64 chain, Steele, Lea & Flood 2014) */
uint64_t ors_splitmix64(uint64_t x);
double ors_uniform(uint64_t seed, uint64_t ray, uint64_t sample, uint32_t dim);
uint32_t ors_sobol(uint32_t i, uint32_t d);                 /* raw Sobol point, d < 11 */
void ors_sobol_poly(uint32_t d, int32_t *degree, uint32_t *inner); /* its primitive polynomial */
uint32_t ors_owen_scramble(uint32_t x, uint32_t seed);      /* nested uniform scramble */
double ors_sobol_uniform(uint64_t seed, uint64_t ray, uint64_t sample, uint32_t dim);

/* building blocks exposed for closed-form tests */
void ors_quat_to_frame(const double q[4], double tu[3], double tv[3], double n[3]);
void ors_onb(const double n[3], double b1[3], double b2[3]);
void ors_brdf(const double n[3], const double wi[3], const double wo[3], const double a[3],
              double m, double r, uint32_t flags, double f[3]);
double ors_ggx_D(double n_dot_h, double roughness);     /* GGX normal distribution */
double ors_smith_G1(double n_dot_v, double roughness);  /* separable Smith masking */
double ors_q_spec(const double a[3], double m, uint32_t flags); /* GGX lobe probability */
double ors_pdf_bsdf(const double n[3], const double wi[3], const double wo[3],
                    const double a[3], double m, double r, uint32_t flags);
/* draws a direction from the cosine/GGX mixture; returns 1 if above the surface */
int ors_sample_bsdf(const double n[3], const double wo[3], const double a[3], double m,
                    double r, uint32_t flags, double u_lobe, double u1, double u2, double wi[3]);
double ors_env_pdf(const ors_scene *scene, const double w[3]);
/* importance-samples the env map; returns the pdf (0 if invalid) */
double ors_env_sample(const ors_scene *scene, double ua, double ub, double w[3]);
void ors_env_lookup(const ors_scene *scene, const double w[3], double rgb[3]);

#ifdef __cplusplus
}
#endif
#endif

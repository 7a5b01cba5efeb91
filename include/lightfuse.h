/*
 * lightfuse.h -- C ABI of the MI355X (gfx950) one-bounce 2D-Gaussian-surfel
 * ray tracer: the data-parallel hot path of LightFuse's relightable
 * reconstruction (arXiv 2608.29269, Sec. 3).
 *
 * Conventions
 *  - Every pointer documented "device" is caller-owned HIP device memory
 *    (e.g. PyTorch tensors); the library never frees it.  Scene arrays passed
 *    to lf_scene_set are retained (not copied) and must stay alive and
 *    unmoved until the next lf_scene_set or lf_destroy.
 *  - The library owns only what lives inside an lf_ctx: BVHs, per-surfel
 *    trace records, environment sampling tables, queues and scratch.
 *  - All calls are asynchronous on the context's stream.  Argument errors are
 *    returned synchronously (LF_EINVAL, nothing is launched).  Conditions
 *    found on the device (invalid transforms, traversal-stack overflow) are
 *    latched in a device status word and returned by the next lf_sync.
 *  - Arrays are row-major and contiguous; float is IEEE binary32.
 *  - A context is not thread-safe; use one context per host thread/stream
 *    (lf_abort excepted).
 */
#ifndef LIGHTFUSE_H
#define LIGHTFUSE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LF_OK = 0,
  LF_EINVAL = 1,       /* invalid argument (synchronous) or invalid device data (latched) */
  LF_ENOMEM = 2,       /* device allocation failed */
  LF_EDEVICE = 3,      /* HIP runtime error */
  LF_EBUSY = 4,        /* server queue full */
  LF_EOVERFLOW = 5,    /* traversal stack or queue overflow seen on the device */
  LF_EUNSUPPORTED = 6, /* valid but unsupported configuration (e.g. k > 64, BVH deeper than the stack) */
  LF_EABORTED = 7,     /* work cut short by lf_abort (latched; outputs of the affected calls undefined) */
  LF_ETIMEOUT = 8      /* lf_sync_timeout gave up waiting and cut the work short */
} lf_status;

typedef struct lf_ctx lf_ctx;

/* Creates a context on HIP device `device` that issues all work on
 * `hip_stream` (a hipStream_t; NULL = the null stream). */
lf_status lf_create(lf_ctx **out, int device, void *hip_stream);
void lf_destroy(lf_ctx *ctx);
/* Message of the last non-OK status of this context (never NULL). */
const char *lf_last_error(const lf_ctx *ctx);
/* Waits for the context's stream and returns (then clears) any latched device
 * status; LF_EABORTED if lf_abort cut work short.  Clears the abort request
 * once the stream has drained. */
lf_status lf_sync(lf_ctx *ctx);
/* Failure detection for the persistent traversal pools.  lf_abort raises the
 * context's abort word (fine-grained host memory that the tracing kernels
 * read while they refill their lanes, every eighth refill of a wave): every
 * ray not yet finished is then stored with an empty hit list and no further
 * traversal is done, so each kernel of the calls already enqueued still
 * completes normally, quickly, and with every buffer it hands on well formed;
 * their outputs are undefined and the next lf_sync returns LF_EABORTED.
 * Calls enqueued before that lf_sync are cut short too.  Safe to call from
 * any host thread, also while another thread waits in lf_sync.  Relight
 * server passes do not read the word. */
lf_status lf_abort(lf_ctx *ctx);
/* lf_sync with a host watchdog: polls the stream; if it has not drained
 * after timeout_ms (>= 0), raises the abort word, waits for the cut-short
 * work, clears the word and the latched status and returns LF_ETIMEOUT. */
lf_status lf_sync_timeout(lf_ctx *ctx, double timeout_ms);

/* ---------------------------------------------------------------------------
 * Scene: shared background B plus M movable objects O_o, each a set of 2D
 * Gaussian surfels G_i = (mu_i, q_i, s_i, alpha_i, a_i, m_i, r_i)
 * (Sec. 3.1, Eq. gaussian-primitive; the splatting feature f_i is not traced).
 * ------------------------------------------------------------------------- */
typedef struct {
  const float *mu;        /* device [n,3] centre; object space for object surfels */
  const float *q;         /* device [n,4] orientation quaternion (w,x,y,z), any nonzero norm */
  const float *scale;     /* device [n,2] in-plane scales s_u, s_v > 0 */
  const float *opacity;   /* device [n]   alpha in (0,1] */
  const float *albedo;    /* device [n,3] base colour a in [0,1]^3 */
  const float *roughness; /* device [n]   r in [0,1] */
  const float *metallic;  /* device [n]   m in [0,1] */
  int64_t n;              /* 1 <= n < 2^31 */
  int32_t n_objects;      /* M, 0 <= M <= 63 */
  const int64_t *object_offset; /* host [M+2], non-decreasing: background surfels are
                                   [0, off[1]), object o (0-based) is [off[o+1], off[o+2]),
                                   off[0] = 0 and off[M+1] = n */
} lf_surfels;

/* Retains the scene pointers and builds one bounding-volume hierarchy per
 * instance (background and each object, in object space): per-surfel trace
 * records, size-extended Morton codes, radix sort, a binary hierarchy by
 * parallel locally-ordered clustering of the sorted boxes (Meister and
 * Bittner 2018), cut into traversal nodes of up to eight children by a
 * surface-area-cost dynamic programme (after Ylitie, Karras and Laine 2017)
 * and placed depth-first with contiguous children, surfel records reordered
 * to match, then the bounds and the
 * traversal nodes with child boxes quantised conservatively to 8 bits per
 * plane.  Synchronous: it first waits for the work already on the context's
 * stream (which reads the buffers it rebuilds) and returns once the hierarchy
 * is built.  LF_EUNSUPPORTED if a hierarchy is deeper than the traversal
 * stack. */
lf_status lf_scene_set(lf_ctx *ctx, const lf_surfels *surfels);
/* Recomputes trace records and bounds bottom-up after in-place updates of the
 * retained arrays (same n, same object ranges), and re-quantises the
 * traversal nodes; the hierarchy is kept. */
lf_status lf_scene_refit(lf_ctx *ctx);

/* Rigid transform T_{k,o} = (R, t) per object for one state k; it moves only
 * centres and orientations (Sec. 3.1, Eq. state-assembly):
 * mu' = R mu + t, frame' = R frame.  R must be a rotation; the library uses
 * the Gram-Schmidt orthonormalisation of its first two columns (third column
 * = their cross product) in double precision. */
typedef struct {
  const float *R; /* device [M,3,3] row-major, or NULL if M == 0 */
  const float *t; /* device [M,3], or NULL if M == 0 */
} lf_transforms;

/* State environment map E_k: lat-long, +Y up, row r covers polar angle
 * [r, r+1) pi/h from +Y, column c covers azimuth [c, c+1) 2pi/w measured
 * from +X towards +Z; scene-linear RGB. */
typedef struct {
  const float *texels; /* device [h,w,3] */
  int32_t h, w;        /* 1 <= h, w <= 8192 */
} lf_envmap;

/* Explicit rays (origins, unit directions); ray id i = array index. */
typedef struct {
  const float *o; /* device [n,3] */
  const float *d; /* device [n,3] unit */
  int64_t n;
} lf_rays;

/* Pinhole camera; pose is the 3x4 camera-to-world matrix (row-major) whose
 * columns are (right, up, back, centre); the camera looks along -back.  The
 * ray of pixel (x, y), y = 0 at the top, passes through the pixel centre;
 * it is computed in binary32 with a fixed operation order so it is
 * reproducible bit for bit.  Ray ids enumerate cameras in order, then pixels
 * row-major: id = offset_c + y*w + x with offset_c = sum of earlier w*h. */
typedef struct {
  float pose[12];
  float fov_y_deg; /* 0 < fov < 180 */
  int32_t w, h;    /* >= 1 */
} lf_camera;
#define LF_MAX_CAMERAS 16

#define LF_FLAG_NO_SECONDARY  (1u << 0) /* shade with the unshadowed E(w); trace no secondary ray */
#define LF_FLAG_NO_BACKGROUND (1u << 1) /* drop the T*E(d) term behind partial coverage */
#define LF_FLAG_BSDF_ONLY     (1u << 2) /* sample only the cosine/GGX mixture (no env importance sampling) */
#define LF_FLAG_DIFFUSE_ONLY  (1u << 3) /* Lambert lobe only */
#define LF_FLAG_BRUTE_FORCE   (1u << 4) /* test every surfel of every instance (no BVH); for testing */
#define LF_FLAG_COUNT         (1u << 5) /* accumulate traversal counters (lf_trace_counters) */
#define LF_FLAG_UNSORTED      (1u << 6) /* trace secondary rays in queue order instead of regrouping them
                                           by direction octant and origin (same results, less coherent) */
/* The paper's two-ray estimator (Sec. 3.3, Eq. path-estimator; Sec. 4.2): per
 * path sample s one environment next-event ray (slot 2s, weight p_e/(p_e^2+p_b^2),
 * its secondary trace used only as transmittance) and one cosine/GGX
 * continuation (slot 2s+1, weight 1/p_b; the escaping term T2 E(w) carries the
 * power-heuristic weight p_b^2/(p_e^2+p_b^2), the two environment samples at
 * its secondary hit do not).  Without it, one ray per sample from one-sample
 * MIS serves both roles.  Secondary outputs are indexed by slot (2S per ray).
 * Not accepted by the relight server. */
#define LF_FLAG_NEE           (1u << 7)
/* Owen-scrambled Sobol uniforms (Sec. 3.3 PRB paragraph: the seed is
 * recorded and the same Sobol samples replayed) instead of the SplitMix64
 * hash: Sobol points of 11 dimensions (van der Corput, then Joe and Kuo's
 * 2008 direction numbers), the sample index and each coordinate
 * nested-uniform scrambled by Burley's hash (2020) seeded per ray, 24-bit
 * uniforms; the samples of one ray form an aligned block of the sequence,
 * so power-of-two spp are stratified in every dimension. */
#define LF_FLAG_SOBOL         (1u << 8)
/* Order-fixed gradient sums in lf_render_backward (Sec. 3.3 PRB paragraph:
 * the replay must reproduce the same path and the same gradient).  Every
 * per-hit and per-environment-tap contribution is written as a binary64
 * record at a position fixed by its ray and its rank within the ray; the
 * records are sorted by target (surfel or texel) with a stable radix sort
 * and each target's records are summed in binary64 in record order, then
 * rounded once to binary32.  Gradients are then bitwise reproducible from
 * run to run.  Costs about 128 B of device scratch per (work item x k
 * bucket) and 32 B per (ray x 4 (1 + 3 J)) environment taps (LF_ENOMEM if
 * that cannot be allocated, LF_EUNSUPPORTED past 2^31 records).  Without
 * it the same contributions are summed by per-block LDS tables and float
 * atomics, whose order varies between runs.  No effect on lf_render. */
#define LF_FLAG_DETERMINISTIC (1u << 9)

/* Tracing and estimator parameters.  Readings of points the paper leaves
 * open (Sec. 3.2 "finite support", "opacity threshold", epsilon of
 * Eq. surface-record; Sec. 3.3 estimator constants) are the defaults set by
 * lf_params_default. */
typedef struct {
  int32_t k;        /* hits kept per ray, 1..64 (default 32) */
  int32_t spp;      /* S shading samples per primary hit, 1..64 (default 1) */
  uint64_t seed;    /* sampler seed; the same seed replays the same paths */
  double alpha_min; /* opacity threshold, hits with alpha*exp(-rho^2/2) < alpha_min are culled (1/255) */
  double alpha_cap; /* effective-opacity cap (0.99) */
  double support_sigma; /* finite support radius in units of sigma (3) */
  double eps;       /* epsilon of the composite normalisation (1e-6) */
  double t_min;     /* smallest accepted ray parameter (1e-4) */
  double secondary_offset; /* secondary origin = x_bar + offset * n_bar (1e-3) */
  uint32_t flags;   /* LF_FLAG_* */
} lf_params;
void lf_params_default(lf_params *p);

typedef struct {
  float *radiance;      /* device [R,3] pixel radiance L (Eq. path-estimator, plus T*E(d)) */
  float *depth;         /* device [R]   composited plane-intersection depth (ray parameter) */
  float *normal;        /* device [R,3] composited unit normal facing the ray (0 on a miss) */
  float *alpha;         /* device [R]   accumulated opacity A */
  int32_t *hit_idx;     /* device [R,k] primary hit surfel indices in order, -1 padded; or NULL */
  int32_t *sec_hit_idx; /* device [R,J,k] secondary hit lists per slot (J = S, or 2S with LF_FLAG_NEE;
                           -1 padded, all -1 if not traced); or NULL */
} lf_outputs;

/* Forward render of one state (Sec. 3.2 tracing and compositing; Sec. 3.3
 * one-bounce estimator): for each ray, the k closest valid hits sorted by
 * (t, surfel index) are composited front to back into a surface record; S
 * directions are drawn by one-sample power-heuristic MIS between environment
 * importance sampling and a cosine/GGX mixture; each live direction traces
 * one secondary ray whose record returns T2*E(w) + A2*L2, L2 being two
 * unshadowed environment samples at the secondary record.  Pixel value
 * L = A * mean_s F_s + T * E(d).
 * Exactly one of `rays` (non-NULL) or `cams`/`n_cams` (1..LF_MAX_CAMERAS,
 * host array) selects the rays.  radiance/depth/normal/alpha must be
 * non-NULL device arrays with R rows. */
lf_status lf_render(lf_ctx *ctx, const lf_transforms *xf, const lf_envmap *env, const lf_rays *rays,
                    const lf_camera *cams, int32_t n_cams, const lf_params *p, lf_outputs *out);

/* Upstream gradients of the outputs (device, same shapes; NULL = zero). */
typedef struct {
  const float *d_radiance, *d_depth, *d_normal, *d_alpha;
} lf_grad_out;
/* Parameter gradients (device, shapes of the scene arrays and env map).
 * All eight must be non-NULL; they are OVERWRITTEN.  d_q is with respect to
 * the raw (unnormalised) quaternion; the rest with respect to the values
 * passed in. */
typedef struct {
  float *d_mu, *d_q, *d_scale, *d_opacity, *d_albedo, *d_roughness, *d_metallic, *d_env;
} lf_grad_in;

/* Reverse mode of lf_render under path replay (Sec. 3.3, PRB paragraph):
 * the same seed replays the same paths; hit sets and their order, sampled
 * directions, technique/lobe choices, MIS and pdf factors, secondary origins
 * and records are held fixed, while gradients flow through the primary
 * compositing (geometry, opacity, materials; Sec. 3.2), the primary BRDF and
 * every environment texel read.  Hit lists are recomputed, never stored.
 * Arguments as for lf_render with identical values. */
lf_status lf_render_backward(lf_ctx *ctx, const lf_transforms *xf, const lf_envmap *env, const lf_rays *rays,
                             const lf_camera *cams, int32_t n_cams, const lf_params *p, const lf_grad_out *g,
                             lf_grad_in *grads);

/* Scene-linear L1 objective of inverse rendering (Sec. 3.4,
 * Eq. training-objectives, data term): loss = mean |pred - target| over n
 * values; grad = sign(pred - target)/n (sign(0) = 0).  loss: device scalar
 * (binary64 sum in a fixed order; 0 for n = 0, where pred and target may be
 * NULL); grad: device [n] or NULL.  LF_EINVAL for n < 0 or a missing pointer. */
lf_status lf_l1_loss(lf_ctx *ctx, const float *pred, const float *target, int64_t n, float *loss, float *grad);

/* lf_l1_loss for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result bit for bit, but the partial sums live in
 * a library-owned device array of 2 x 2048 + 2 doubles (32 KB) that each
 * device holds for the life of the process, located by
 * lf_create; no allocation, no free, no event.  Any n >= 0 fits (the grid
 * is capped at 2048 blocks, one partial-sum slot each).  Every call on one
 * device shares that array (each call overwrites what it reads, so nothing
 * needs clearing): calls that overlap on one device, from any contexts or
 * streams, race and must be ordered by the caller.  Arguments, ownership and
 * errors as for lf_l1_loss; LF_EDEVICE if the array was not located. */
lf_status lf_l1_loss_noalloc(lf_ctx *ctx, const float *pred, const float *target, int64_t n, float *loss,
                             float *grad);

/* ---- Geometry-refinement objectives (Sec. 3.1 and 3.2).  Common contract:
 * every array is a device array; loss is a device float scalar written
 * asynchronously on the context's stream; grad, when non-NULL, is
 * OVERWRITTEN with d(loss)/d(first map) (same shape); sums run in binary64
 * in a fixed order, so the loss does not vary from run to run; sign(0) = 0.  The gradients feed lf_render_backward's d_alpha, d_depth and
 * d_normal.  Errors: LF_EINVAL for NULL maps, n < 0 or an invalid constant. */

/* Coverage term L_alpha = (1/n) sum |A - 1| (Sec. 3.1, Eq. alpha-coverage)
 * over an accumulated-opacity map alpha [n] (lf_outputs.alpha). */
lf_status lf_loss_alpha(lf_ctx *ctx, const float *alpha, int64_t n, float *loss, float *grad);

/* Scale regulariser L_s = (1/n) sum_i max(0, max(|s_u|,|s_v|)/s_max - 1)^2
 * (Sec. 3.1, Eq. scale-regularization) over in-plane scales [n,2]; the
 * gradient goes to the larger component (the first on a tie).  s_max > 0. */
lf_status lf_loss_scale(lf_ctx *ctx, const float *scale, int64_t n, float s_max, float *loss, float *grad);

/* Confidence-weighted depth term L_D = sum |C| |D - D*| / (sum |C| |D*| + eps)
 * (Sec. 3.2, Eq. reconstruction-depth) over a rendered depth map D [n]
 * (lf_outputs.depth), reference D* [n] and confidence C [n] (NULL: C = 1).
 * eps > 0. */
lf_status lf_loss_depth(lf_ctx *ctx, const float *depth, const float *ref, const float *conf, int64_t n, float eps,
                        float *loss, float *grad);

/* Rendered-normal term L_N = 1 - (1/n) sum <N, N*> (Sec. 3.2,
 * Eq. reconstruction-normal) over normal maps [n,3] (lf_outputs.normal and
 * the reference); grad = -N* / n.  n = 0 gives loss 0. */
lf_status lf_loss_normal(lf_ctx *ctx, const float *normal, const float *ref, int64_t n, float *loss, float *grad);

/* Environment regulariser L_TV(E_k) of the inverse-rendering objective
 * (Sec. 3.4, Eq. training-objectives; the paper does not define it): the
 * anisotropic first-order total variation of a lat-long map env [h,w,3]
 * (lf_envmap layout), sum over channels of |E(y,x+1) - E(y,x)| with x wrapping
 * in azimuth plus |E(y+1,x) - E(y,x)| for y < h-1 (no wrap over the poles),
 * divided by 3 h w.  grad: [h,w,3] or NULL.  Errors: LF_EINVAL for h or w < 1. */
lf_status lf_loss_tv(lf_ctx *ctx, const float *env, int32_t h, int32_t w, float *loss, float *grad);

/* Depth-derived-normal term L_DN = 1 - (1/(w h)) sum <N^D, N*> (Sec. 3.2,
 * Eq. reconstruction-normal) for the rendered depth map depth [h*w]
 * (row-major, the rays of `cam` as lf_raygen makes them) and reference
 * normals ref [h*w,3].  N^D at pixel (x, y) is the unit vector along
 * (P(x+1,y) - P(x-1,y)) x (P(x,y-1) - P(x,y+1)), P = o + depth * d the point
 * on the pixel's ray (row 0 at the top), which faces the camera on a smooth
 * surface; N^D = 0 on the image border, next to a pixel with depth <= 0 (no
 * surface) or where the cross product vanishes.  grad: d(loss)/d(depth) [h*w].
 * Errors: LF_EINVAL for an invalid camera or h > 1048560. */
lf_status lf_loss_depth_normal(lf_ctx *ctx, const lf_camera *cam, const float *depth, const float *ref, float *loss,
                               float *grad);

/* Pinhole rays of one camera (device o, d: [w*h,3]) exactly as lf_render
 * generates them. */
lf_status lf_raygen(lf_ctx *ctx, const lf_camera *cam, float *o, float *d);

/* Introspection of the current scene's hierarchies (synchronous). */
typedef struct {
  int32_t n_instances;  /* M + 1 */
  int64_t n_surfels;
  int64_t n_nodes;      /* internal nodes over all instances */
  int32_t max_depth;    /* deepest leaf (root = depth 0) */
  int32_t stack_size;   /* traversal stack entries per ray (one per level above the current node: the
                           scene set fails with LF_EUNSUPPORTED if wide_levels - 1 exceeds it) */
  int64_t n_wide_nodes; /* traversal nodes over all instances */
  int32_t wide_levels;  /* levels of the deepest traversal hierarchy */
  int32_t node_width;   /* children per traversal node */
} lf_scene_info;
lf_status lf_scene_get_info(lf_ctx *ctx, lf_scene_info *info);

/* Copies instance `inst`'s hierarchy to host memory: n-1 internal nodes as
 * child boxes [n-1, 2, 6] (lo xyz, hi xyz), children [n-1, 2] (>= 0 internal
 * node within the instance, < 0 leaf ~position), leaf order perm [n] (surfel
 * index of each leaf position, global), leaf boxes [n, 6] by leaf position.
 * Any pointer may be NULL. */
lf_status lf_scene_copy_bvh(lf_ctx *ctx, int32_t inst, float *node_boxes, int32_t *children, int32_t *perm,
                            float *leaf_boxes);

/* Copies instance `inst`'s traversal nodes to host memory, decoded: *n_nodes
 * receives their count m; if slot_boxes / slot_child are not NULL they must
 * hold m * node_width * 6 floats / m * node_width ints, filled per node and
 * slot with the decoded binary32 box (lo xyz, hi xyz; the box traversal
 * tests) and the child (>= 0 traversal node within the instance, < 0 ~leaf
 * position within the instance, INT32_MIN for a slot without a child or with
 * an empty box).  Node 0 is the root. */
lf_status lf_scene_copy_wide(lf_ctx *ctx, int32_t inst, int64_t *n_nodes, float *slot_boxes, int32_t *slot_child);

/* Rays traced by lf_render calls since the previous lf_stats_get: primary
 * rays and secondary rays actually traced (live samples).  Accumulated on the
 * device without synchronisation; lf_stats_get synchronises, returns and
 * resets them.  Replay passes of lf_render_backward are not counted. */
typedef struct {
  int64_t rays_primary;
  int64_t rays_secondary;
} lf_render_stats;
lf_status lf_stats_get(lf_ctx *ctx, lf_render_stats *stats);

/* Traversal counters accumulated by calls made with LF_FLAG_COUNT since the
 * previous read (synchronous; resets them): [0] primary rays, [1] traversal
 * nodes visited, [2] surfels tested, [3] hits inserted into k-buffers, then
 * [4..7] the same for secondary rays, [8] primary and [9] secondary hits
 * whose binary32 distance key equalled one already held, placed by exact
 * FP64 keys, [10] primary and [11] secondary surfel tests that passed the
 * binary32 pre-filter, [12] primary and [13] secondary valid hits found
 * (support and threshold met, before truncation to k), [14] primary and
 * [15] secondary traversal stack pushes, [16] primary and [17] secondary
 * deepest traversal stack reached (a maximum, not a sum), [18] primary and
 * [19] secondary rays that started from the k-th distance of the same ray
 * in the previous call (the replay of an lf_render_backward directly after
 * the lf_render with the same arguments), [20] primary and [21] secondary
 * rays of those traced again without it (fewer than k hits below it). */
#define LF_NUM_COUNTERS 22
lf_status lf_trace_counters(lf_ctx *ctx, uint64_t *counters /*[LF_NUM_COUNTERS]*/);

/* Per-phase device timers.  When enabled, every phase below is bracketed by
 * HIP events on the context's stream; lf_profile_read synchronises, returns
 * the accumulated milliseconds and launch counts per phase and resets them.
 * Phases: 0 refit, 1 state and environment tables, 2 primary traversal,
 * 3 primary shading, 4 secondary regrouping, 5 secondary traversal,
 * 6 secondary shading, 7 resolve, 8 replay of the primary pass, 9 replay of
 * the secondary pass, 10 shading adjoint, 11 unused (the compositing adjoint
 * reads the hit lists of the replayed primary pass), 12 gradient zeroing,
 * 13 loss, 14 primary compositing, 15 secondary compositing, 16 compositing
 * adjoint.  Phases 2 and 5 each hold one traversal kernel launch per call
 * (after clearing its work counters), phases 14 to 16 one compositing kernel
 * launch. */
#define LF_NUM_PHASES 17
lf_status lf_profile_enable(lf_ctx *ctx, int enable);
lf_status lf_profile_read(lf_ctx *ctx, double *ms /*[LF_NUM_PHASES]*/, int64_t *count /*[LF_NUM_PHASES]*/);

/* ---------------------------------------------------------------------------
 * Relight server.  Rearranging objects or relighting re-renders the resident
 * scene with new object transforms and a new environment map (Sec. 3.4,
 * scene editing and relighting; Sec. 1, appearance recomputed after every
 * interaction).  The server renders many such requests at once by
 * continuous batching: every iteration is one batched forward pass (primary
 * trace, shading, secondary trace, shading, resolve) over 128-ray chunks,
 * each one 16x8-pixel tile of one request's image, drawn from all admitted
 * requests (policy below), each request with its own
 * transforms, environment, camera, S and seed.  A request's outputs equal
 * those of lf_render with the same inputs bit for bit (ray ids and sampler
 * counters are local to the request).
 *
 * Admission is FIFO: a waiting request is admitted when one of max_slots is
 * free and the sum of the working sets of admitted requests stays within
 * hbm_budget_bytes.  The working set of a request of R = w*h rays and S
 * samples is charged as R*(32 + 44*S) bytes (outputs and its share of the
 * secondary-ray state) plus its environment copy and sampling tables.
 * Buffers the server allocates up front (batch scratch sized by batch_rays
 * and max_spp, one environment slot per request slot) are not charged.
 *
 * The server has its own HIP streams and host thread.  It reads the context's
 * scene: lf_scene_set and lf_scene_refit return LF_EBUSY while a server of
 * the context exists, and every server must be destroyed before its context.
 * The server functions are thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct lf_server lf_server;

/* Which admitted requests fill a pass first (admission itself is always FIFO). */
#define LF_SCHED_SHORTEST_FIRST 0 /* smallest remaining work, rays x (1 + S), first; each takes all it can */
#define LF_SCHED_OLDEST_FIRST   1 /* admission order; each takes all it can (FIFO with backfill) */
#define LF_SCHED_ROUND_ROBIN    2 /* max(tile_rays, batch_rays / active) rays each, in turn */

typedef struct {
  int32_t max_slots;        /* requests admitted at once, 1..64 (default 16) */
  int64_t hbm_budget_bytes; /* admission budget of the admitted working sets (default 16 GiB) */
  int32_t tile_rays;        /* smallest share of primary rays a request gets per iteration (round
                               robin); multiple of 128 (default 65536).  Rays are counted in whole
                               16x8-pixel tiles of 128 */
  int32_t batch_rays;       /* primary rays per iteration, multiple of 128, >= tile_rays (default 1048576) */
  int32_t max_spp;          /* largest S a request may ask for, 1..64 (default 4) */
  int32_t max_pending;      /* waiting requests before lf_server_submit returns LF_EBUSY (default 4096) */
  int32_t policy;           /* LF_SCHED_* (default LF_SCHED_OLDEST_FIRST) */
  int32_t max_in_flight;    /* passes running at once, 1..4, each on its own stream with its own
                               scratch (default 2): the latency-bound tail of one pass overlaps
                               the next, and a new arrival starts on a free lane */
  lf_params params;         /* k, constants and flags shared by every request (spp and seed are
                               per request; LF_FLAG_COUNT and LF_FLAG_NO_SECONDARY are not served) */
} lf_server_config;
void lf_server_config_default(lf_server_config *cfg);

/* One render request.  Every buffer must stay valid until the request has
 * completed (lf_server_poll reports done or lf_server_wait returned). */
typedef struct {
  lf_transforms xf;   /* host or device [M,3,3] and [M,3] (NULL if M == 0) */
  lf_envmap env;      /* host or device texels; host arrays (texels, transforms) are copied into
                         the request's slot on admission, device arrays are read in place */
  lf_camera cam;      /* one pinhole camera; R = cam.w * cam.h rays, ids from 0 */
  int32_t spp;        /* S, 1..max_spp */
  uint64_t seed;      /* sampler seed */
  lf_outputs out;     /* device radiance/depth/normal/alpha with R rows; hit_idx and
                         sec_hit_idx must be NULL */
} lf_request;

/* Creates a server over ctx's current scene (synchronises ctx's stream). */
lf_status lf_server_create(lf_ctx *ctx, const lf_server_config *cfg, lf_server **out);
/* Validates and enqueues a request; non-blocking.  LF_EBUSY if max_pending
 * requests are waiting, LF_EUNSUPPORTED if its working set alone exceeds the
 * budget (both count as rejected).  *ticket >= 1 identifies it. */
lf_status lf_server_submit(lf_server *srv, const lf_request *req, uint64_t *ticket);
/* *done = 1 once the request has completed; returns the request's status
 * (LF_OK, or the error that ended it; LF_EINVAL for an unknown ticket). */
lf_status lf_server_poll(lf_server *srv, uint64_t ticket, int *done);
/* Blocks until the request has completed; returns its status. */
lf_status lf_server_wait(lf_server *srv, uint64_t ticket);
/* Milliseconds from submission to completion of a completed request. */
lf_status lf_server_latency(lf_server *srv, uint64_t ticket, double *ms);

typedef struct {
  double p50_ms, p99_ms;   /* latency percentiles over completed requests (nearest rank) */
  double rays_per_s;       /* traced rays (primary + live secondary) per second of serving
                              (first submission to last completion) */
  int64_t completed, rejected;
  int64_t rays_primary, rays_secondary;
  int64_t iterations;      /* batched passes launched */
} lf_server_stats;
lf_status lf_server_stats_get(lf_server *srv, lf_server_stats *stats);
/* Message of the server's last error (never NULL). */
const char *lf_server_last_error(lf_server *srv);
/* Finishes the iterations in flight, cancels requests not yet completed
 * (their status becomes LF_EBUSY) and frees the server. */
void lf_server_destroy(lf_server *srv);

#ifdef __cplusplus
}
#endif
#endif

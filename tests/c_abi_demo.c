/* A plain C99 caller of liblightfuse: device memory from the HIP runtime's C
 * API, every call through include/lightfuse.h, no Python.  One surfel at the
 * origin facing +z (scales 0.2, opacity 0.8) and one ray from (0.05, 0, -2)
 * along +z: the ray meets the plane at t = 2 at local radius rho = 0.25, so
 * (Sec. 3.2, Eq. gaussian-response and surface-record) the accumulated
 * opacity is A = 0.8 exp(-rho^2 / 2), the depth 2 A / (A + eps), the normal
 * faces the ray, and dA/d(opacity) = exp(-rho^2 / 2).  Prints "c abi ok" and
 * exits 0 when all of these hold. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "lightfuse.h"

#define CHECK_HIP(x)                                                  \
  do {                                                                \
    if ((x) != hipSuccess) {                                          \
      fprintf(stderr, "HIP error at line %d: %s\n", __LINE__, #x);    \
      return 2;                                                       \
    }                                                                 \
  } while (0)
#define CHECK_LF(ctx, x)                                                               \
  do {                                                                                 \
    lf_status st_ = (x);                                                               \
    if (st_ != LF_OK) {                                                                \
      fprintf(stderr, "lightfuse error %d at line %d: %s\n", (int)st_, __LINE__,       \
              lf_last_error(ctx));                                                     \
      return 3;                                                                        \
    }                                                                                  \
  } while (0)

static int upload(float **dst, const float *src, size_t n) {
  if (hipMalloc((void **)dst, n * sizeof(float)) != hipSuccess) return 1;
  return hipMemcpy(*dst, src, n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess;
}

int main(void) {
  const float h_mu[3] = {0.f, 0.f, 0.f}, h_q[4] = {1.f, 0.f, 0.f, 0.f}, h_scale[2] = {0.2f, 0.2f};
  const float h_opacity[1] = {0.8f}, h_albedo[3] = {0.5f, 0.5f, 0.5f}, h_rough[1] = {0.5f}, h_metal[1] = {0.f};
  const float h_o[3] = {0.05f, 0.f, -2.f}, h_d[3] = {0.f, 0.f, 1.f};
  float h_env[4 * 8 * 3];
  for (int i = 0; i < 4 * 8 * 3; ++i) h_env[i] = 1.f;
  float *mu, *q, *scale, *opacity, *albedo, *rough, *metal, *o, *d, *env;
  if (upload(&mu, h_mu, 3) || upload(&q, h_q, 4) || upload(&scale, h_scale, 2) || upload(&opacity, h_opacity, 1) ||
      upload(&albedo, h_albedo, 3) || upload(&rough, h_rough, 1) || upload(&metal, h_metal, 1) ||
      upload(&o, h_o, 3) || upload(&d, h_d, 3) || upload(&env, h_env, 4 * 8 * 3)) {
    fprintf(stderr, "upload failed\n");
    return 2;
  }
  float *out;  /* radiance 3, depth 1, normal 3, alpha 1, d_alpha 1, then 8 gradient arrays */
  CHECK_HIP(hipMalloc((void **)&out, 64 * sizeof(float)));
  CHECK_HIP(hipMemset(out, 0, 64 * sizeof(float)));

  lf_ctx *ctx = NULL;
  if (lf_create(&ctx, 0, NULL) != LF_OK) {
    fprintf(stderr, "lf_create failed\n");
    return 3;
  }
  const int64_t off[2] = {0, 1};
  lf_surfels s;
  memset(&s, 0, sizeof s);
  s.mu = mu; s.q = q; s.scale = scale; s.opacity = opacity; s.albedo = albedo; s.roughness = rough;
  s.metallic = metal; s.n = 1; s.n_objects = 0; s.object_offset = off;
  CHECK_LF(ctx, lf_scene_set(ctx, &s));

  lf_envmap e = {env, 4, 8};
  lf_rays r;
  memset(&r, 0, sizeof r);
  r.o = o; r.d = d; r.n = 1;
  lf_params p;
  lf_params_default(&p);
  p.k = 4;
  p.flags = LF_FLAG_NO_SECONDARY;
  /* an argument error is returned at once, with a message */
  p.k = 0;
  lf_outputs outs = {out, out + 3, out + 4, out + 7, NULL, NULL};
  if (lf_render(ctx, NULL, &e, &r, NULL, 0, &p, &outs) != LF_EINVAL || strlen(lf_last_error(ctx)) == 0) {
    fprintf(stderr, "k = 0 was not refused\n");
    return 4;
  }
  p.k = 4;
  CHECK_LF(ctx, lf_render(ctx, NULL, &e, &r, NULL, 0, &p, &outs));
  CHECK_LF(ctx, lf_sync(ctx));

  const float one = 1.f;
  CHECK_HIP(hipMemcpy(out + 8, &one, sizeof one, hipMemcpyHostToDevice));
  lf_grad_out go = {NULL, NULL, NULL, out + 8};
  lf_grad_in gi = {out + 9, out + 12, out + 16, out + 18, out + 19, out + 22, out + 23, out + 24};
  float *g_env;
  CHECK_HIP(hipMalloc((void **)&g_env, sizeof h_env));
  gi.d_env = g_env;
  CHECK_LF(ctx, lf_render_backward(ctx, NULL, &e, &r, NULL, 0, &p, &go, &gi));
  CHECK_LF(ctx, lf_sync(ctx));

  float h[64];
  CHECK_HIP(hipMemcpy(h, out, sizeof h, hipMemcpyDeviceToHost));
  const double g = exp(-0.5 * (0.05 / 0.2) * (0.05 / 0.2));
  const double A = 0.8 * g, depth = 2.0 * A / (A + 1e-6);
  int ok = fabs(h[7] - A) < 1e-6 && fabs(h[3] - depth) < 1e-5 && fabs(h[4]) < 1e-6 && fabs(h[5]) < 1e-6 &&
           fabs(h[6] + 1.0) < 1e-6 && fabs(h[18] - g) < 1e-5;
  printf("alpha %.7f (%.7f) depth %.6f (%.6f) normal %.3f %.3f %.3f d_opacity %.6f (%.6f)\n", h[7], A, h[3], depth,
         h[4], h[5], h[6], h[18], g);
  lf_destroy(ctx);
  hipFree(g_env);
  hipFree(out);
  hipFree(mu); hipFree(q); hipFree(scale); hipFree(opacity); hipFree(albedo); hipFree(rough); hipFree(metal);
  hipFree(o); hipFree(d); hipFree(env);
  if (!ok) {
    fprintf(stderr, "mismatch\n");
    return 1;
  }
  printf("c abi ok\n");
  return 0;
}

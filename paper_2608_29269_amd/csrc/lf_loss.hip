// lf_loss.hip -- geometry-refinement objectives and their gradients:
//   L_alpha  coverage of the accumulated opacity map       (Sec. 3.1, Eq. alpha-coverage)
//   L_s      squared hinge on the largest in-plane scale   (Sec. 3.1, Eq. scale-regularization)
//   L_D      confidence-weighted relative L1 on depth      (Sec. 3.2, Eq. reconstruction-depth)
//   L_N      cosine term on the rendered normal map        (Sec. 3.2, Eq. reconstruction-normal)
//   L_DN     cosine term on the depth-derived normal map   (Sec. 3.2, Eq. reconstruction-normal)
// Each is one streaming pass over its maps (HBM-bound): per-element terms are
// summed in binary64, one wave shuffle tree and one atomic per block, and a
// one-thread kernel turns the sum into the loss.  Gradients are written in
// the same pass, except L_D, whose gradient needs the global denominator
// first.  L_DN gathers, for each pixel, the gradients of the (at most five)
// central-difference normals that read its depth, so it needs no scratch
// and its gradient does not depend on scheduling.
#include "lf_device.h"
#include "lf_kernels.h"

namespace lf {

namespace {

constexpr int kLossBlock = 256;

inline unsigned loss_grid(int64_t n) {
  int64_t nb = (n + kLossBlock - 1) / kLossBlock;
  return (unsigned)(nb < 1 ? 1 : (nb > 2048 ? 2048 : nb));
}

__device__ inline double sgn(double v) { return (double)((v > 0.0) - (v < 0.0)); }

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Adds the block's sum of v (and of v2) to acc[0] (and acc[1]); every thread
// of the 256-thread block must call it.
template <int N>
__device__ inline void block_add(const double (&v)[N], double *acc) {
  __shared__ double part[N][kLossBlock / 64];
  const int t = threadIdx.x + threadIdx.y * blockDim.x;
  for (int k = 0; k < N; ++k) {
    const double s = wave_sum(v[k]);
    if ((t & 63) == 0) part[k][t >> 6] = s;
  }
  __syncthreads();
  if (t < N) {
    double s = 0.0;
    for (int w = 0; w < kLossBlock / 64; ++w) s += part[t][w];
    atomicAdd(acc + t, s);
  }
}

__global__ void k_zero_acc(double *acc) {
  acc[0] = 0.0;
  acc[1] = 0.0;
}

// loss = offset + scale * acc[0]
__global__ void k_loss_final(const double *acc, double scale, double offset, float *loss) {
  *loss = (float)(offset + scale * acc[0]);
}

__global__ __launch_bounds__(kLossBlock) void k_loss_alpha(const float *alpha, int64_t n, float *grad, double *acc) {
  const double inv = 1.0 / (double)n;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kLossBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLossBlock) {
    const double r = (double)alpha[i] - 1.0;
    s += fabs(r);
    if (grad) grad[i] = (float)(sgn(r) * inv);
  }
  block_add<1>({s}, acc);
}

__global__ __launch_bounds__(kLossBlock) void k_loss_scale(const float *scale, int64_t n, double s_max, float *grad,
                                                           double *acc) {
  const double gk = 2.0 / ((double)n * s_max);
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kLossBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLossBlock) {
    const double su = scale[2 * i], sv = scale[2 * i + 1];
    const bool second = fabs(sv) > fabs(su);  // the first component wins ties
    const double h = fmax(0.0, (second ? fabs(sv) : fabs(su)) / s_max - 1.0);
    s += h * h;
    if (grad) {
      const double g = gk * h * sgn(second ? sv : su);
      grad[2 * i] = second ? 0.f : (float)g;
      grad[2 * i + 1] = second ? (float)g : 0.f;
    }
  }
  block_add<1>({s}, acc);
}

__global__ __launch_bounds__(kLossBlock) void k_loss_depth_sums(const float *depth, const float *ref, const float *conf,
                                                                int64_t n, double *acc) {
  double num = 0.0, den = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kLossBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLossBlock) {
    const double c = conf ? fabs((double)conf[i]) : 1.0, r = ref[i];
    num += c * fabs((double)depth[i] - r);
    den += c * fabs(r);
  }
  block_add<2>({num, den}, acc);
}

__global__ __launch_bounds__(kLossBlock) void k_loss_depth_grad(const float *depth, const float *ref, const float *conf,
                                                                int64_t n, double eps, const double *acc, float *grad,
                                                                float *loss) {
  const double inv = 1.0 / (acc[1] + eps);
  if (blockIdx.x == 0 && threadIdx.x == 0) *loss = (float)(acc[0] * inv);
  if (!grad) return;
  for (int64_t i = (int64_t)blockIdx.x * kLossBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLossBlock) {
    const double c = conf ? fabs((double)conf[i]) : 1.0;
    grad[i] = (float)(c * sgn((double)depth[i] - (double)ref[i]) * inv);
  }
}

// m = 3 * pixels, flat over the [pixels, 3] maps
__global__ __launch_bounds__(kLossBlock) void k_loss_normal(const float *normal, const float *ref, int64_t m,
                                                            double inv_n, float *grad, double *acc) {
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * kLossBlock + threadIdx.x; k < m; k += (int64_t)gridDim.x * kLossBlock) {
    const double r = ref[k];
    s += (double)normal[k] * r;
    if (grad) grad[k] = (float)(-r * inv_n);
  }
  block_add<1>({s}, acc);
}

// ---- depth-derived normal
//
// With P = o + D d and one pinhole centre o for all pixels, the central
// differences of P are those of Q = D d, which avoids cancelling the
// camera position; Q is formed in binary64 from the binary32 depth and ray.
__device__ inline void qpoint(const CamArgs &ca, const float *D, int64_t p, double q[3]) {
  float o[3], d[3];
  raygen_f32(ca, 0, p, o, d);
  const double z = D[p];
  q[0] = z * d[0];
  q[1] = z * d[1];
  q[2] = z * d[2];
}

__device__ inline void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

struct DnCenter {
  double a[3], b[3], c[3], len;
};

// Tangent differences a = P(x+1,y) - P(x-1,y), b = P(x,y-1) - P(x,y+1) and
// their cross product at interior pixel (x, y); false where the normal is
// undefined (border, a neighbour without surface, parallel tangents).
__device__ bool dn_center(const CamArgs &ca, const float *D, int w, int h, int x, int y, DnCenter &t) {
  if (x < 1 || y < 1 || x > w - 2 || y > h - 2) return false;
  const int64_t p = (int64_t)y * w + x;
  if (!(fminf(fminf(D[p - 1], D[p + 1]), fminf(D[p - w], D[p + w])) > 0.f)) return false;
  double q0[3], q1[3];
  qpoint(ca, D, p + 1, q0);
  qpoint(ca, D, p - 1, q1);
  for (int k = 0; k < 3; ++k) t.a[k] = q0[k] - q1[k];
  qpoint(ca, D, p - w, q0);
  qpoint(ca, D, p + w, q1);
  for (int k = 0; k < 3; ++k) t.b[k] = q0[k] - q1[k];
  cross3(t.a, t.b, t.c);
  t.len = sqrt(t.c[0] * t.c[0] + t.c[1] * t.c[1] + t.c[2] * t.c[2]);
  return t.len > 0.0;
}

// d(loss)/dc of -(1/n) <c/|c|, r>
__device__ inline void dn_gc(const DnCenter &t, const float *ref, int64_t p, double inv_n, double gc[3]) {
  const double r[3] = {ref[3 * p], ref[3 * p + 1], ref[3 * p + 2]};
  const double il = 1.0 / t.len;
  const double u[3] = {t.c[0] * il, t.c[1] * il, t.c[2] * il};
  const double ur = u[0] * r[0] + u[1] * r[1] + u[2] * r[2];
  for (int k = 0; k < 3; ++k) gc[k] = -(r[k] - u[k] * ur) * il * inv_n;
}

// One pixel per thread on 16 x 16 tiles: the pixel's own term of the sum and
// the gradient of its depth, gathered from the centres that difference it.
__global__ __launch_bounds__(kLossBlock) void k_loss_depth_normal(const CamArgs *cams, const float *D, const float *ref,
                                                                  int w, int h, double inv_n, float *grad,
                                                                  double *acc) {
  const CamArgs &ca = *cams;
  const int x = blockIdx.x * 16 + threadIdx.x, y = blockIdx.y * 16 + threadIdx.y;
  double dot = 0.0;
  if (x < w && y < h) {
    const int64_t p = (int64_t)y * w + x;
    DnCenter t;
    if (dn_center(ca, D, w, h, x, y, t)) {
      const double il = 1.0 / t.len;
      dot = (t.c[0] * ref[3 * p] + t.c[1] * ref[3 * p + 1] + t.c[2] * ref[3 * p + 2]) * il;
    }
    if (grad) {
      double g[3] = {0.0, 0.0, 0.0}, gc[3], v[3];
      // as P(x+1) of the centre (x-1, y): +b x gc; as P(x-1) of (x+1, y): -b x gc
      if (dn_center(ca, D, w, h, x - 1, y, t)) {
        dn_gc(t, ref, p - 1, inv_n, gc);
        cross3(t.b, gc, v);
        for (int k = 0; k < 3; ++k) g[k] += v[k];
      }
      if (dn_center(ca, D, w, h, x + 1, y, t)) {
        dn_gc(t, ref, p + 1, inv_n, gc);
        cross3(t.b, gc, v);
        for (int k = 0; k < 3; ++k) g[k] -= v[k];
      }
      // as P(y-1) of the centre (x, y+1): +gc x a; as P(y+1) of (x, y-1): -gc x a
      if (dn_center(ca, D, w, h, x, y + 1, t)) {
        dn_gc(t, ref, p + w, inv_n, gc);
        cross3(gc, t.a, v);
        for (int k = 0; k < 3; ++k) g[k] += v[k];
      }
      if (dn_center(ca, D, w, h, x, y - 1, t)) {
        dn_gc(t, ref, p - w, inv_n, gc);
        cross3(gc, t.a, v);
        for (int k = 0; k < 3; ++k) g[k] -= v[k];
      }
      float o[3], d[3];
      raygen_f32(ca, 0, p, o, d);
      grad[p] = (float)(g[0] * d[0] + g[1] * d[1] + g[2] * d[2]);
    }
  }
  block_add<1>({dot}, acc);
}

}  // namespace

void launch_loss_alpha(const float *alpha, int64_t n, float *loss, float *grad, double *acc, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_acc, dim3(1), dim3(1), 0, st, acc);
  if (n > 0) hipLaunchKernelGGL(k_loss_alpha, dim3(loss_grid(n)), dim3(kLossBlock), 0, st, alpha, n, grad, acc);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1), 0, st, acc, n > 0 ? 1.0 / (double)n : 0.0, 0.0, loss);
}

void launch_loss_scale(const float *scale, int64_t n, float s_max, float *loss, float *grad, double *acc,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_zero_acc, dim3(1), dim3(1), 0, st, acc);
  if (n > 0)
    hipLaunchKernelGGL(k_loss_scale, dim3(loss_grid(n)), dim3(kLossBlock), 0, st, scale, n, (double)s_max, grad, acc);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1), 0, st, acc, n > 0 ? 1.0 / (double)n : 0.0, 0.0, loss);
}

void launch_loss_depth(const float *depth, const float *ref, const float *conf, int64_t n, float eps, float *loss,
                       float *grad, double *acc, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_acc, dim3(1), dim3(1), 0, st, acc);
  if (n > 0)
    hipLaunchKernelGGL(k_loss_depth_sums, dim3(loss_grid(n)), dim3(kLossBlock), 0, st, depth, ref, conf, n, acc);
  hipLaunchKernelGGL(k_loss_depth_grad, dim3(grad && n > 0 ? loss_grid(n) : 1), dim3(kLossBlock), 0, st, depth, ref,
                     conf, n, (double)eps, (const double *)acc, grad, loss);
}

void launch_loss_normal(const float *normal, const float *ref, int64_t n, float *loss, float *grad, double *acc,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_zero_acc, dim3(1), dim3(1), 0, st, acc);
  const double inv_n = n > 0 ? 1.0 / (double)n : 0.0;
  if (n > 0)
    hipLaunchKernelGGL(k_loss_normal, dim3(loss_grid(3 * n)), dim3(kLossBlock), 0, st, normal, ref, 3 * n, inv_n, grad,
                       acc);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1), 0, st, acc, -inv_n, n > 0 ? 1.0 : 0.0, loss);
}

void launch_loss_depth_normal(const CamArgs *cams, int w, int h, const float *depth, const float *ref, float *loss,
                              float *grad, double *acc, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_acc, dim3(1), dim3(1), 0, st, acc);
  const double inv_n = 1.0 / ((double)w * (double)h);
  hipLaunchKernelGGL(k_loss_depth_normal, dim3((w + 15) / 16, (h + 15) / 16), dim3(16, 16), 0, st, cams, depth, ref, w,
                     h, inv_n, grad, acc);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1), 0, st, acc, -inv_n, 1.0, loss);
}

}  // namespace lf

// lf_loss.hip -- training objectives and their gradients:
//   L1       scene-linear data term of inverse rendering   (Sec. 3.4, Eq. training-objectives)
//   L_alpha  coverage of the accumulated opacity map       (Sec. 3.1, Eq. alpha-coverage)
//   L_s      squared hinge on the largest in-plane scale   (Sec. 3.1, Eq. scale-regularization)
//   L_D      confidence-weighted relative L1 on depth      (Sec. 3.2, Eq. reconstruction-depth)
//   L_N      cosine term on the rendered normal map        (Sec. 3.2, Eq. reconstruction-normal)
//   L_DN     cosine term on the depth-derived normal map   (Sec. 3.2, Eq. reconstruction-normal)
//   L_TV     total variation of the environment map E_k    (Sec. 3.4, Eq. training-objectives)
// Each is one streaming pass over its maps (HBM-bound) on at most
// kMaxLossBlocks blocks: per-element terms are summed in binary64, each
// block stores its partial sum in its own slot (no atomics: one address hit
// by every block serialises), and a one-block kernel adds the slots in a
// fixed order and writes the loss, so the value does not depend on
// scheduling.  Gradients are written in the same pass, except L_D, whose
// gradient needs the global denominator first.  L_DN gathers, for each
// pixel, the gradient terms of the (at most four) central-difference
// normals that read its depth, so its gradient needs no scratch either.
#include "lf_device.h"
#include "lf_kernels.h"

namespace lf {

namespace {

constexpr int kLossBlock = 256;

inline unsigned loss_grid(int64_t n) {
  int64_t nb = (n + kLossBlock - 1) / kLossBlock;
  return (unsigned)(nb < 1 ? 1 : (nb > kMaxLossBlocks ? kMaxLossBlocks : nb));
}

__device__ inline double sgn(double v) { return (double)((v > 0.0) - (v < 0.0)); }

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Stores the block's sums of v[k] in part[k * kMaxLossBlocks + blockIdx.x];
// every thread of the 256-thread block must call it.
template <int N>
__device__ inline void block_store(const double (&v)[N], double *part) {
  __shared__ double ws[N][kLossBlock / 64];
  const int t = threadIdx.x + threadIdx.y * blockDim.x;
  for (int k = 0; k < N; ++k) {
    const double s = wave_sum(v[k]);
    if ((t & 63) == 0) ws[k][t >> 6] = s;
  }
  __syncthreads();
  if (t < N) {
    double s = 0.0;
    for (int w = 0; w < kLossBlock / 64; ++w) s += ws[t][w];
    part[t * kMaxLossBlocks + blockIdx.x] = s;
  }
}

// One block: tot[k] = sum of the nb partial sums of slot row k (fixed
// order); then loss = offset + scale * tot[0], or tot[0] / (tot[1] + eps)
// when eps > 0 (the depth objective).
template <int N>
__global__ __launch_bounds__(kLossBlock) void k_loss_reduce(const double *part, int nb, double scale, double offset,
                                                            double eps, double *tot, float *loss) {
  __shared__ double ws[N][kLossBlock / 64];
  const int t = threadIdx.x;
  for (int k = 0; k < N; ++k) {
    double s = 0.0;
    for (int b = t; b < nb; b += kLossBlock) s += part[k * kMaxLossBlocks + b];
    s = wave_sum(s);
    if ((t & 63) == 0) ws[k][t >> 6] = s;
  }
  __syncthreads();
  if (t == 0) {
    double v[N];
    for (int k = 0; k < N; ++k) v[k] = ws[k][0] + ws[k][1] + ws[k][2] + ws[k][3];
    for (int k = 0; k < N; ++k) tot[k] = v[k];
    *loss = (float)(eps > 0.0 ? v[0] / (v[N - 1] + eps) : offset + scale * v[0]);
  }
}

__global__ __launch_bounds__(kLossBlock) void k_l1(const float *pred, const float *target, int64_t n, float *grad,
                                                   double *part) {
  const double inv = 1.0 / (double)n;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kLossBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLossBlock) {
    const double r = (double)pred[i] - (double)target[i];
    s += fabs(r);
    if (grad) grad[i] = (float)(sgn(r) * inv);
  }
  block_store<1>({s}, part);
}

__global__ __launch_bounds__(kLossBlock) void k_loss_alpha(const float *alpha, int64_t n, float *grad, double *part) {
  const double inv = 1.0 / (double)n;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kLossBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLossBlock) {
    const double r = (double)alpha[i] - 1.0;
    s += fabs(r);
    if (grad) grad[i] = (float)(sgn(r) * inv);
  }
  block_store<1>({s}, part);
}

__global__ __launch_bounds__(kLossBlock) void k_loss_scale(const float *scale, int64_t n, double s_max, float *grad,
                                                           double *part) {
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
  block_store<1>({s}, part);
}

__global__ __launch_bounds__(kLossBlock) void k_loss_depth_sums(const float *depth, const float *ref, const float *conf,
                                                                int64_t n, double *part) {
  double num = 0.0, den = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kLossBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLossBlock) {
    const double c = conf ? fabs((double)conf[i]) : 1.0, r = ref[i];
    num += c * fabs((double)depth[i] - r);
    den += c * fabs(r);
  }
  block_store<2>({num, den}, part);
}

__global__ __launch_bounds__(kLossBlock) void k_loss_depth_grad(const float *depth, const float *ref, const float *conf,
                                                                int64_t n, double eps, const double *tot,
                                                                float *grad) {
  const double inv = 1.0 / (tot[1] + eps);
  for (int64_t i = (int64_t)blockIdx.x * kLossBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLossBlock) {
    const double c = conf ? fabs((double)conf[i]) : 1.0;
    grad[i] = (float)(c * sgn((double)depth[i] - (double)ref[i]) * inv);
  }
}

// m = 3 * pixels, flat over the [pixels, 3] maps
__global__ __launch_bounds__(kLossBlock) void k_loss_normal(const float *normal, const float *ref, int64_t m,
                                                            double inv_n, float *grad, double *part) {
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * kLossBlock + threadIdx.x; k < m; k += (int64_t)gridDim.x * kLossBlock) {
    const double r = ref[k];
    s += (double)normal[k] * r;
    if (grad) grad[k] = (float)(-r * inv_n);
  }
  block_store<1>({s}, part);
}

// L_TV: anisotropic first-order total variation of a lat-long map [H,W,3]:
// |E(y,x+1) - E(y,x)| with x wrapping in azimuth, plus |E(y+1,x) - E(y,x)| for
// y < H-1 (no wrap over the poles), over 3 H W values.  One texel per thread:
// its two forward differences enter the sum, and its gradient gathers the
// signs of the (at most four) differences it takes part in.
__device__ inline float sgn_diff(float a, float b) { return (float)((a > b) - (a < b)); }  // sign(a - b)

__global__ __launch_bounds__(kLossBlock) void k_loss_tv(const float *E, int H, int W, double inv_n, float *grad,
                                                        double *part) {
  const int64_t n = (int64_t)H * W;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kLossBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLossBlock) {
    const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
    const int64_t row = (int64_t)y * W;
    const float *e = E + 3 * i;
    const float *er = E + 3 * (row + (x + 1 == W ? 0 : x + 1));
    const float *el = E + 3 * (row + (x == 0 ? W - 1 : x - 1));
    const bool up = y > 0, down = y + 1 < H;
    for (int c = 0; c < 3; ++c) {
      const float v = e[c];
      s += fabs((double)er[c] - (double)v);
      if (down) s += fabs((double)e[3 * W + c] - (double)v);
      if (grad) {
        float g = sgn_diff(v, el[c]) - sgn_diff(er[c], v);
        if (up) g += sgn_diff(v, e[c - 3 * W]);
        if (down) g -= sgn_diff(e[3 * W + c], v);
        grad[3 * i + c] = (float)((double)g * inv_n);
      }
    }
  }
  block_store<1>({s}, part);
}

// ---- depth-derived normal
//
// With P = o + D d and one pinhole centre o for all pixels, the central
// differences of P are those of Q = D d, which avoids cancelling the camera
// position; Q is formed in binary64 from the binary32 depth and ray.
//
// One 16 x 16 pixel tile per block, staged through LDS: the points Q of the
// tile plus a two-pixel apron (20 x 20, one ray each), then the normals of
// the tile plus a one-pixel apron (18 x 18) reduced to the two vectors their
// gradient sends to the differenced points, ga = b x gc to P(x+1,y) (and -ga
// to P(x-1,y)), gb = gc x a to P(x,y-1) (and -gb to P(x,y+1)), with gc the
// gradient of the loss in the cross product c = a x b; each pixel then
// gathers its four terms.
constexpr int kDnT = 16, kDnP = kDnT + 4, kDnC = kDnT + 2;

__device__ inline void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

__global__ __launch_bounds__(kLossBlock) void k_loss_depth_normal(const CamArgs *cams, const float *D, const float *ref,
                                                                  int w, int h, double inv_n, float *grad,
                                                                  double *part) {
  __shared__ double sq[kDnP * kDnP][3];    // Q = D d, zero outside the image
  __shared__ float sz[kDnP * kDnP];        // depth, zero outside the image
  __shared__ float sdir[kDnP * kDnP][3];   // unit ray directions
  __shared__ double sga[kDnC * kDnC][3], sgb[kDnC * kDnC][3];
  const CamArgs &ca = *cams;
  const int t = threadIdx.x + threadIdx.y * kDnT;
  const int tiles_x = (w + kDnT - 1) / kDnT;
  const int64_t n_tiles = (int64_t)tiles_x * ((h + kDnT - 1) / kDnT);
  double dot = 0.0;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {  // same trip count for the whole block
    const int X0 = (int)(tile % tiles_x) * kDnT, Y0 = (int)(tile / tiles_x) * kDnT;
    for (int k = t; k < kDnP * kDnP; k += kLossBlock) {
      const int x = X0 - 2 + k % kDnP, y = Y0 - 2 + k / kDnP;
      float z = 0.f, o[3], d[3] = {0.f, 0.f, 0.f};
      if (x >= 0 && y >= 0 && x < w && y < h) {
        const int64_t p = (int64_t)y * w + x;
        z = D[p];
        raygen_f32(ca, 0, p, o, d);
      }
      sz[k] = z;
      for (int c = 0; c < 3; ++c) {
        sdir[k][c] = d[c];
        sq[k][c] = (double)z * d[c];
      }
    }
    __syncthreads();
    for (int k = t; k < kDnC * kDnC; k += kLossBlock) {
      const int cx = k % kDnC, cy = k / kDnC;
      const int x = X0 - 1 + cx, y = Y0 - 1 + cy;  // the normal's pixel
      double ga[3] = {0.0, 0.0, 0.0}, gb[3] = {0.0, 0.0, 0.0};
      const int m = (cy + 1) * kDnP + cx + 1;       // its point in sq
      // undefined on the border, next to a pixel without surface, or for parallel tangents
      if (x >= 1 && y >= 1 && x <= w - 2 && y <= h - 2 &&
          fminf(fminf(sz[m - 1], sz[m + 1]), fminf(sz[m - kDnP], sz[m + kDnP])) > 0.f) {
        double a[3], b[3], c[3];
        for (int i = 0; i < 3; ++i) {
          a[i] = sq[m + 1][i] - sq[m - 1][i];
          b[i] = sq[m - kDnP][i] - sq[m + kDnP][i];
        }
        cross3(a, b, c);
        const double len = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        if (len > 0.0) {
          const int64_t p = (int64_t)y * w + x;
          const double r[3] = {ref[3 * p], ref[3 * p + 1], ref[3 * p + 2]};
          const double il = 1.0 / len;
          if (cx >= 1 && cy >= 1 && cx <= kDnT && cy <= kDnT) dot += (c[0] * r[0] + c[1] * r[1] + c[2] * r[2]) * il;
          if (grad) {
            // d(loss)/dc of -(1/n) <c/|c|, r>
            const double u[3] = {c[0] * il, c[1] * il, c[2] * il};
            const double ur = u[0] * r[0] + u[1] * r[1] + u[2] * r[2];
            double gc[3];
            for (int i = 0; i < 3; ++i) gc[i] = -(r[i] - u[i] * ur) * il * inv_n;
            cross3(b, gc, ga);
            cross3(gc, a, gb);
          }
        }
      }
      for (int i = 0; i < 3; ++i) {
        sga[k][i] = ga[i];
        sgb[k][i] = gb[i];
      }
    }
    __syncthreads();
    const int x = X0 + threadIdx.x, y = Y0 + threadIdx.y;
    if (grad && x < w && y < h) {
      const int cl = (threadIdx.y + 1) * kDnC + threadIdx.x;  // normal of (x-1, y); (x+1, y) is cl + 2
      const int cu = threadIdx.y * kDnC + threadIdx.x + 1;    // normal of (x, y-1); (x, y+1) is cu + 2 kDnC
      double g[3];
      for (int i = 0; i < 3; ++i)
        g[i] = sga[cl][i] - sga[cl + 2][i] + sgb[cu + 2 * kDnC][i] - sgb[cu][i];
      const int m = (threadIdx.y + 2) * kDnP + threadIdx.x + 2;
      grad[(int64_t)y * w + x] = (float)(g[0] * sdir[m][0] + g[1] * sdir[m][1] + g[2] * sdir[m][2]);
    }
    __syncthreads();  // the next tile overwrites the LDS arrays
  }
  block_store<1>({dot}, part);
}

}  // namespace

// part: device scratch of kLossPartDoubles doubles (slots, then the totals)
void launch_l1(const float *pred, const float *target, int64_t n, float *loss, float *grad, double *part,
               hipStream_t st) {
  const unsigned nb = n > 0 ? loss_grid(n) : 0;
  if (nb) hipLaunchKernelGGL(k_l1, dim3(nb), dim3(kLossBlock), 0, st, pred, target, n, grad, part);
  hipLaunchKernelGGL(k_loss_reduce<1>, dim3(1), dim3(kLossBlock), 0, st, (const double *)part, (int)nb,
                     n > 0 ? 1.0 / (double)n : 0.0, 0.0, 0.0, part + 2 * kMaxLossBlocks, loss);
}

void launch_loss_alpha(const float *alpha, int64_t n, float *loss, float *grad, double *part, hipStream_t st) {
  const unsigned nb = n > 0 ? loss_grid(n) : 0;
  if (nb) hipLaunchKernelGGL(k_loss_alpha, dim3(nb), dim3(kLossBlock), 0, st, alpha, n, grad, part);
  hipLaunchKernelGGL(k_loss_reduce<1>, dim3(1), dim3(kLossBlock), 0, st, (const double *)part, (int)nb,
                     n > 0 ? 1.0 / (double)n : 0.0, 0.0, 0.0, part + 2 * kMaxLossBlocks, loss);
}

void launch_loss_scale(const float *scale, int64_t n, float s_max, float *loss, float *grad, double *part,
                       hipStream_t st) {
  const unsigned nb = n > 0 ? loss_grid(n) : 0;
  if (nb) hipLaunchKernelGGL(k_loss_scale, dim3(nb), dim3(kLossBlock), 0, st, scale, n, (double)s_max, grad, part);
  hipLaunchKernelGGL(k_loss_reduce<1>, dim3(1), dim3(kLossBlock), 0, st, (const double *)part, (int)nb,
                     n > 0 ? 1.0 / (double)n : 0.0, 0.0, 0.0, part + 2 * kMaxLossBlocks, loss);
}

void launch_loss_depth(const float *depth, const float *ref, const float *conf, int64_t n, float eps, float *loss,
                       float *grad, double *part, hipStream_t st) {
  const unsigned nb = n > 0 ? loss_grid(n) : 0;
  double *tot = part + 2 * kMaxLossBlocks;
  if (nb) hipLaunchKernelGGL(k_loss_depth_sums, dim3(nb), dim3(kLossBlock), 0, st, depth, ref, conf, n, part);
  hipLaunchKernelGGL(k_loss_reduce<2>, dim3(1), dim3(kLossBlock), 0, st, (const double *)part, (int)nb, 0.0, 0.0,
                     (double)eps, tot, loss);
  if (nb && grad)
    hipLaunchKernelGGL(k_loss_depth_grad, dim3(nb), dim3(kLossBlock), 0, st, depth, ref, conf, n, (double)eps,
                       (const double *)tot, grad);
}

void launch_loss_normal(const float *normal, const float *ref, int64_t n, float *loss, float *grad, double *part,
                        hipStream_t st) {
  const unsigned nb = n > 0 ? loss_grid(3 * n) : 0;
  const double inv_n = n > 0 ? 1.0 / (double)n : 0.0;
  if (nb)
    hipLaunchKernelGGL(k_loss_normal, dim3(nb), dim3(kLossBlock), 0, st, normal, ref, 3 * n, inv_n, grad, part);
  hipLaunchKernelGGL(k_loss_reduce<1>, dim3(1), dim3(kLossBlock), 0, st, (const double *)part, (int)nb, -inv_n,
                     n > 0 ? 1.0 : 0.0, 0.0, part + 2 * kMaxLossBlocks, loss);
}

void launch_loss_tv(const float *env, int h, int w, float *loss, float *grad, double *part, hipStream_t st) {
  const int64_t n = (int64_t)h * w;
  const unsigned nb = loss_grid(n);
  const double inv_n = 1.0 / (3.0 * (double)n);
  hipLaunchKernelGGL(k_loss_tv, dim3(nb), dim3(kLossBlock), 0, st, env, h, w, inv_n, grad, part);
  hipLaunchKernelGGL(k_loss_reduce<1>, dim3(1), dim3(kLossBlock), 0, st, (const double *)part, (int)nb, inv_n, 0.0, 0.0,
                     part + 2 * kMaxLossBlocks, loss);
}

void launch_loss_depth_normal(const CamArgs *cams, int w, int h, const float *depth, const float *ref, float *loss,
                              float *grad, double *part, hipStream_t st) {
  const int64_t tiles = (int64_t)((w + kDnT - 1) / kDnT) * ((h + kDnT - 1) / kDnT);
  const unsigned nb = (unsigned)(tiles < kMaxLossBlocks ? tiles : kMaxLossBlocks);
  const double inv_n = 1.0 / ((double)w * (double)h);
  hipLaunchKernelGGL(k_loss_depth_normal, dim3(nb), dim3(kDnT, kDnT), 0, st, cams, depth, ref, w, h, inv_n, grad,
                     part);
  hipLaunchKernelGGL(k_loss_reduce<1>, dim3(1), dim3(kLossBlock), 0, st, (const double *)part, (int)nb, -inv_n, 1.0,
                     0.0, part + 2 * kMaxLossBlocks, loss);
}

}  // namespace lf

// The focusing objective of the differentiable form, fused around the operator:
//   L(m) = sum over the k models of ||W_d (G m - d_obs)||^2 + alpha * sum_i m_i^2 / (m_i^2 + eps^2)
// (the data misfit and the minimum-support stabilizer of Sec. 2.2 with lambda = 0 and W = I) and
// its gradient  dL/dm = G^T (2 W_d^2 (G m - d_obs)) + alpha * 2 m eps^2 / (m^2 + eps^2)^2.
// The operator products are the library's block applies; everything around them is one kernel
// before the reduction, one for the reduction and one after G^T.
#include "common.h"

namespace ff {
namespace {

constexpr int kThreads = 256;
constexpr int kLossBlocks = 256;   // partial sums per term
static_assert(kLossBlocks == kThreads, "k_loss_final sums one partial per thread");

__device__ double block_sum256(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// Blocks [0, kLossBlocks): rw = 2 wd^2 (gm - d) in place of gm (the misfit's gradient with
// respect to G m) and partial sums of (wd (gm - d))^2 into part[b].  Blocks [kLossBlocks, 2 kLossBlocks):
// partial sums of m^2 / (m^2 + eps2) into part[b].  Grid-stride over the km and kn elements.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_loss_terms(T *__restrict__ rw, const T *__restrict__ d, const T *__restrict__ wd, int64_t km,
             const T *__restrict__ m, int64_t kn, double eps2, double *__restrict__ part) {
  __shared__ double red[kThreads];
  double s = 0.0;
  if (blockIdx.x < kLossBlocks) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < km; i += (int64_t)kLossBlocks * kThreads) {
      const double w = (double)wd[i];
      const double r = w * ((double)rw[i] - (double)d[i]);
      s += r * r;
      rw[i] = (T)(2.0 * w * r);
    }
  } else {
    const int b = blockIdx.x - kLossBlocks;
    for (int64_t i = (int64_t)b * kThreads + threadIdx.x; i < kn; i += (int64_t)kLossBlocks * kThreads) {
      const double v = (double)m[i];
      const double q = v * v;
      s += q / (q + eps2);
    }
  }
  s = block_sum256(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// loss = sum of the misfit partials + alpha * sum of the stabilizer partials (fixed order)
__global__ void __launch_bounds__(kThreads)
k_loss_final(const double *__restrict__ part, double alpha, double *__restrict__ loss) {
  __shared__ double red[kThreads];
  const double a = block_sum256(part[threadIdx.x], red);
  __syncthreads();
  const double b = block_sum256(part[kLossBlocks + threadIdx.x], red);
  if (threadIdx.x == 0) loss[0] = a + alpha * b;
}

// g = scale * (g + alpha * 2 m eps2 / (m^2 + eps2)^2), scale = *scale_ptr (1 when NULL)
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_grad_combine(T *__restrict__ g, const T *__restrict__ m, int64_t kn, double alpha, double eps2,
               const double *__restrict__ scale_ptr) {
  const double sc = scale_ptr ? *scale_ptr : 1.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < kn; i += (int64_t)gridDim.x * kThreads) {
    const double v = (double)m[i];
    const double q = v * v + eps2;
    g[i] = (T)(sc * ((double)g[i] + alpha * 2.0 * v * eps2 / (q * q)));
  }
}

unsigned blocks_for(int64_t count) {
  int64_t b = (count + kThreads - 1) / kThreads;
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

ff_status same_device(ff_spectra h) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(FF_EHIP, "hipGetDevice failed");
  if (cur != h->device) return fail(FF_EDEVICE, "current device differs from the handle's device");
  return FF_OK;
}

}  // namespace
}  // namespace ff

using namespace ff;

extern "C" {

ff_status ff_focusing_loss(ff_spectra h, int64_t k, const void *m, const void *d_obs, const void *wd, double alpha,
                           double eps2, void *rw, double *work, ff_stream stream) {
  if (!h || !m || !d_obs || !wd || !rw || !work) return fail(FF_EINVAL, "ff_focusing_loss: NULL argument");
  if (k < 1) return fail(FF_ESHAPE, "ff_focusing_loss: need k >= 1");
  if (!(eps2 > 0.0) || !(alpha >= 0.0)) return fail(FF_EINVAL, "ff_focusing_loss: need eps2 > 0, alpha >= 0");
  ff_status st = same_device(h);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  // rw = G m (k columns), then the two terms
  if ((st = op_apply(h, 0, k, m, h->n, rw, h->m, nullptr, nullptr, h->dtype, s))) return st;
  const int64_t km = k * h->m, kn = k * h->n;
  if (h->dtype == FF_F32)
    k_loss_terms<float><<<2 * kLossBlocks, kThreads, 0, s>>>((float *)rw, (const float *)d_obs, (const float *)wd, km,
                                                             (const float *)m, kn, eps2, work + 1);
  else
    k_loss_terms<double><<<2 * kLossBlocks, kThreads, 0, s>>>((double *)rw, (const double *)d_obs, (const double *)wd,
                                                              km, (const double *)m, kn, eps2, work + 1);
  k_loss_final<<<1, kThreads, 0, s>>>(work + 1, alpha, work);
  FF_LAUNCH_CHECK("ff_focusing_loss");
  return FF_OK;
}

ff_status ff_focusing_grad(ff_spectra h, int64_t k, const void *m, const void *rw, double alpha, double eps2,
                           const double *scale, void *grad, ff_stream stream) {
  if (!h || !m || !rw || !grad) return fail(FF_EINVAL, "ff_focusing_grad: NULL argument");
  if (k < 1) return fail(FF_ESHAPE, "ff_focusing_grad: need k >= 1");
  if (!(eps2 > 0.0) || !(alpha >= 0.0)) return fail(FF_EINVAL, "ff_focusing_grad: need eps2 > 0, alpha >= 0");
  ff_status st = same_device(h);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = op_apply(h, 1, k, rw, h->m, grad, h->n, nullptr, nullptr, h->dtype, s))) return st;
  const int64_t kn = k * h->n;
  if (h->dtype == FF_F32)
    k_grad_combine<float><<<blocks_for(kn), kThreads, 0, s>>>((float *)grad, (const float *)m, kn, alpha, eps2, scale);
  else
    k_grad_combine<double><<<blocks_for(kn), kThreads, 0, s>>>((double *)grad, (const double *)m, kn, alpha, eps2,
                                                               scale);
  FF_LAUNCH_CHECK("ff_focusing_grad");
  return FF_OK;
}

}  // extern "C"

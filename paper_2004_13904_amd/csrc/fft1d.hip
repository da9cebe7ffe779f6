// Stand-alone 1-D transforms through the device FFT of the operator's passes (the Stockham
// transform of fft.h in any of its stage plans), for verification against a reference FFT:
// count transforms of length n, one per block.
#include "common.h"
#include "fft.h"

namespace ff {
namespace {

// tw[e] = exp(-2 pi i e / n), evaluated in double and rounded once
template <typename T> __global__ void k_twiddles(cplx<T> *__restrict__ tw, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double a = 6.283185307179586476925 * (double)e / (double)n;
  tw[e] = mk<T>((T)cos(a), (T)-sin(a));
}

// out[b] = DFT(in[b]) (INV: the unnormalized inverse), b = blockIdx.x; TPF = N/8 threads
template <typename T, int N, bool INV, int P>
__global__ void __launch_bounds__((FFT<T, N, INV, P>::TPF))
k_fft_1d(const cplx<T> *__restrict__ in, cplx<T> *__restrict__ out, const cplx<T> *__restrict__ tw) {
  using F = FFT<T, N, INV, P>;
  __shared__ cplx<T> buf[F::LDS];
  const int j = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * N;
  typename F::Tw t;
  F::load_tw(t, j, tw);   // the inverse multiplies by the conjugates of the same table
  cplx<T> v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) v[u] = in[base + j + u * F::TPF];
  F::run_tw(v, j, buf, t);
#pragma unroll
  for (int u = 0; u < 8; ++u) out[base + j + u * F::TPF] = v[u];
}

template <typename T, int N, int P>
void launch_plan(bool inverse, int64_t count, const void *in, void *out, const void *tw, hipStream_t s) {
  if (inverse)
    k_fft_1d<T, N, true, P><<<(unsigned)count, N / 8, 0, s>>>((const cplx<T> *)in, (cplx<T> *)out,
                                                              (const cplx<T> *)tw);
  else
    k_fft_1d<T, N, false, P><<<(unsigned)count, N / 8, 0, s>>>((const cplx<T> *)in, (cplx<T> *)out,
                                                               (const cplx<T> *)tw);
}

template <typename T, int N>
ff_status launch_fft_1d(int plan, bool inverse, int64_t count, const void *in, void *out, void *tw, hipStream_t s) {
  k_twiddles<T><<<(N + 255) / 256, 256, 0, s>>>((cplx<T> *)tw, N);
  switch (plan_canon(N, plan)) {
    case 0: launch_plan<T, N, 0>(inverse, count, in, out, tw, s); break;
    case 1:
      if constexpr (plan_canon(N, 1) == 1) launch_plan<T, N, 1>(inverse, count, in, out, tw, s);
      break;
    default: launch_plan<T, N, 2>(inverse, count, in, out, tw, s); break;
  }
  FF_LAUNCH_CHECK("ff_fft_1d");
  return FF_OK;
}

}  // namespace
}  // namespace ff

using namespace ff;

extern "C" {

ff_status ff_fft_1d(int32_t n, int32_t dtype, int32_t inverse, int32_t plan, int64_t count, const void *in,
                    void *out, void *twiddles, ff_stream stream) {
  if (!in || !out || !twiddles) return fail(FF_EINVAL, "ff_fft_1d: NULL argument");
  if (dtype != FF_F32 && dtype != FF_F64) return fail(FF_EDTYPE, "ff_fft_1d: dtype must be FF_F32 or FF_F64");
  if (inverse != 0 && inverse != 1) return fail(FF_EINVAL, "ff_fft_1d: inverse must be 0 or 1");
  if (plan < 0 || plan >= kFftPlans) return fail(FF_EINVAL, "ff_fft_1d: plan must be 0, 1 or 2");
  if (count < 0 || count > 2147483647) return fail(FF_ESHAPE, "ff_fft_1d: count out of range");
  if (!is_pow2(n) || n < 8 || n > 2048) return fail(FF_ESHAPE, "ff_fft_1d: n must be a power of two in [8, 2048]");
  if (count == 0) return FF_OK;
  hipStream_t s = (hipStream_t)stream;
  if (dtype == FF_F32) {
    FF_SWITCH_N(n, return launch_fft_1d<float, NN>(plan, inverse == 1, count, in, out, twiddles, s));
  } else {
    FF_SWITCH_N(n, return launch_fft_1d<double, NN>(plan, inverse == 1, count, in, out, twiddles, s));
  }
  return FF_OK;
}

}  // extern "C"

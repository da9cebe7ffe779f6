// The operator's block product for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).  It runs the same pass
// kernels as apply_G_block, with the pass intermediates in a fixed library array instead of the
// handle's workspace, and calls no allocating routine.
//
// The array lives in the code object: every device the library runs on holds its own copy from
// the first call on that device until the process ends.  In host code `scratch` only names the
// symbol; its device address on the current device comes from hipGetSymbolAddress, looked up
// once per device and kept in g_scratch_ptr.  Kernels receive that address.
#include <mutex>

#include "common.h"

namespace ff {
namespace {

constexpr size_t kScratchBytes = FF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // device address of `scratch` on each device, once looked up

// Device address of this device's array; `dev` must be the current device.
ff_status scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FF_EDEVICE, "ff_apply_block_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "ff_apply_block_noalloc: hipGetSymbolAddress(scratch)");
    if (!p) return fail(FF_EHIP, "ff_apply_block_noalloc: hipGetSymbolAddress returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FF_OK;
}

}  // namespace
}  // namespace ff

using namespace ff;

extern "C" ff_status ff_apply_block_noalloc(ff_spectra h, int32_t transpose, int64_t k, const void *X, int64_t ldx,
                                            void *Y, int64_t ldy, const void *w_pre, const void *w_post,
                                            ff_stream stream) {
  if (!h || !X || !Y) return fail(FF_EINVAL, "ff_apply_block_noalloc: NULL argument");
  if (transpose != 0 && transpose != 1) return fail(FF_EINVAL, "ff_apply_block_noalloc: transpose must be 0 or 1");
  if (k < 0) return fail(FF_ESHAPE, "ff_apply_block_noalloc: k < 0");
  const int64_t rin = transpose ? h->m : h->n, rout = transpose ? h->n : h->m;
  if (ldx < rin || ldy < rout) return fail(FF_ESHAPE, "ff_apply_block_noalloc: leading dimension too small");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FF_EHIP, "ff_apply_block_noalloc: hipGetDevice failed");
  if (dev != h->device) return fail(FF_EDEVICE, "ff_apply_block_noalloc: current device differs from the handle's");
  // vectors per launch: as many of the handle's batch as the array holds (row intermediates
  // first, then the column-pass buffer, 256-byte aligned)
  size_t rows_b = 0, cols_b = 0;
  op_ws_per_vector(h, transpose, &rows_b, &cols_b);
  auto need = [&](int64_t kb) { return ((size_t)kb * rows_b + 255) / 256 * 256 + (size_t)kb * cols_b; };
  if (need(1) > kScratchBytes)
    return fail(FF_ENOMEM, "ff_apply_block_noalloc: one vector's pass intermediates (" + std::to_string(need(1)) +
                               " bytes) exceed the fixed scratch array (" + std::to_string(kScratchBytes) + " bytes)");
  void *base = nullptr;
  ff_status st = scratch_address(dev, &base);
  if (st != FF_OK) return st;
  if (k == 0) return FF_OK;
  int64_t kb = h->batch;
  while (kb > 1 && need(kb) > kScratchBytes) --kb;
  const size_t cols_off = ((size_t)kb * rows_b + 255) / 256 * 256;
  const OpWs ws{base, (unsigned char *)base + cols_off, (int)kb};
  return op_apply_ws(h, ws, transpose, k, X, ldx, Y, ldy, w_pre, w_post, h->dtype, (hipStream_t)stream);
}

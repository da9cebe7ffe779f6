// Internal declarations shared by the HIP translation units of libfastfocus.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fastfocus.h"

namespace ff {

// ---------------------------------------------------------------------------------------
// Complex scalars: float2 / double2 so that one element is one vector load.
template <typename T> struct CT;
template <> struct CT<float> { using type = float2; };
template <> struct CT<double> { using type = double2; };
template <typename T> using cplx = typename CT<T>::type;

template <typename T> __host__ __device__ __forceinline__ cplx<T> mk(T re, T im) {
  cplx<T> c;
  c.x = re;
  c.y = im;
  return c;
}
template <typename T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
// Complex products with the fused multiply-adds written out: every kernel then rounds a
// product the same way (left to the compiler's contraction, the same expression could be
// fused differently in different kernels, and paths that should agree bit for bit would not).
__device__ __forceinline__ float ffma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double ffma(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  const T yy = a.y * b.y, yx = a.y * b.x;
  return mk<T>(ffma(a.x, b.x, -yy), ffma(a.x, b.y, yx));
}
// a * conj(b)
template <typename T> __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  const T yy = a.y * b.y, xy = a.x * b.y;
  return mk<T>(ffma(a.x, b.x, yy), ffma(a.y, b.x, -xy));
}
template <typename T> __device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return mk<T>(a.x, -a.y); }
template <typename T> __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }

// ---------------------------------------------------------------------------------------
// Error reporting: the C ABI returns a status and keeps a thread-local message.
void set_error(const std::string &msg);
ff_status fail(ff_status code, const std::string &msg);
ff_status hip_fail(hipError_t e, const char *what);

#define FF_HIP(call)                                                \
  do {                                                              \
    hipError_t e_ = (call);                                         \
    if (e_ != hipSuccess) return ::ff::hip_fail(e_, #call);         \
  } while (0)

#define FF_LAUNCH_CHECK(what)                                       \
  do {                                                              \
    hipError_t e_ = hipGetLastError();                              \
    if (e_ != hipSuccess) return ::ff::hip_fail(e_, what);          \
  } while (0)

// Dispatch a runtime embedding size to a compile-time constant NN.
#define FF_SWITCH_N(N, ...)                                   \
  switch (N) {                                                 \
    case 8: { constexpr int NN = 8; __VA_ARGS__; } break;             \
    case 16: { constexpr int NN = 16; __VA_ARGS__; } break;           \
    case 32: { constexpr int NN = 32; __VA_ARGS__; } break;           \
    case 64: { constexpr int NN = 64; __VA_ARGS__; } break;           \
    case 128: { constexpr int NN = 128; __VA_ARGS__; } break;         \
    case 256: { constexpr int NN = 256; __VA_ARGS__; } break;         \
    case 512: { constexpr int NN = 512; __VA_ARGS__; } break;         \
    case 1024: { constexpr int NN = 1024; __VA_ARGS__; } break;       \
    case 2048: { constexpr int NN = 2048; __VA_ARGS__; } break;       \
    default: return ::ff::fail(FF_ENOTIMPL, "unsupported embedding size"); \
  }


// The same dispatch for code that must release resources first: an unsupported size sets `st`.
#define FF_SWITCH_N_SET(N, st, ...)                            \
  switch (N) {                                                 \
    case 8: { constexpr int NN = 8; __VA_ARGS__; } break;             \
    case 16: { constexpr int NN = 16; __VA_ARGS__; } break;           \
    case 32: { constexpr int NN = 32; __VA_ARGS__; } break;           \
    case 64: { constexpr int NN = 64; __VA_ARGS__; } break;           \
    case 128: { constexpr int NN = 128; __VA_ARGS__; } break;         \
    case 256: { constexpr int NN = 256; __VA_ARGS__; } break;         \
    case 512: { constexpr int NN = 512; __VA_ARGS__; } break;         \
    case 1024: { constexpr int NN = 1024; __VA_ARGS__; } break;       \
    case 2048: { constexpr int NN = 2048; __VA_ARGS__; } break;       \
    default: st = ::ff::fail(FF_ENOTIMPL, "unsupported embedding size"); \
  }

// stage plans of the device FFT (fft.h)
constexpr int kFftPlans = 3;

inline bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Vectors per batched operator launch: each handle picks a batch (a multiple of 4 within
// [kMinBatch, kMaxBatch]) whose row-pass intermediates fit in about kBatchBytes, and sizes its
// pass workspace for it (about twice that).  Larger launches fill more of the chip per pass and
// pay the fixed launch costs fewer times: per vector, G and G^T of the 200 x 150 x 12 survey
// take 3.8-3.9 us at 128 vectors against 4.0-4.2 us at 24, and those of the 100 x 60 x 10
// survey 0.50-0.52 us at 128 against 0.62-0.64 us at 64, although the intermediates then
// exceed the last-level cache.
constexpr int kMinBatch = 16, kMaxBatch = 128;
constexpr size_t kBatchBytes = (size_t)512 << 20;

}  // namespace ff

// ---------------------------------------------------------------------------------------
// The spectra handle.
struct ff_spectra_s {
  int device = 0;
  int dtype = FF_F32;
  // geometry
  int sx = 0, sy = 0, nz = 0, pxl = 0, pxr = 0, pyl = 0, pyr = 0, nx = 0, ny = 0;
  double dx = 0, dy = 0, incl = 0, decl = 0, field = 0;
  int kernel = 0;
  std::vector<double> z_edges;
  // embedding
  int NX = 0, NY = 0, H = 0;         // H = NX/2 + 1 half-spectrum columns
  int ldy = 0, lds = 0;              // column strides of the intermediates (ny, sy rounded up to 16)
  int64_t m = 0, n = 0;
  // device memory
  void *spec = nullptr;              // [nz][H][NY] complex (float2 or double2), scaled by 1/(NX NY)
  void *tw_x = nullptr, *tw_y = nullptr;   // twiddle tables exp(-2 pi i e / N), e in [0, N)
  double *z_dev = nullptr;           // z_edges on the device
  int batch = ff::kMinBatch;          // vectors per batched launch (tunable, <= batch_max)
  int batch_max = ff::kMinBatch;      // vectors the pass workspace holds
  int row_tile = 0;                   // 0 auto, 1 one transform per row block, 2 largest tile
  int col_batched = 2;                // column passes of block applies (ff_tuning)
  int rsvd_qr = 0;                    // RSVD orthonormalization: 0 CholQR2 first, 1 Householder, 2 CholQR3 first
  int pair_fused = 1;                 // grouped plans: G x and G^T d of this survey share one column pass
  int gkb_graph = 0;                  // replay the GKB iteration loop from a captured graph
  int gkb_onesided = 0;               // GKB: 0 both bases reorthogonalized, 1 the data side only, 2 as 1 with A recomputed
  int fft_plan_x = 0, fft_plan_y = 0; // stage plans of the row and column transforms (fft.h)
  uint64_t tune_version = 0;          // bumped by every ff_set_tuning (captured launches depend on it)
  // the captured GKB iteration loop and what it was captured for
  void *gkb_exec = nullptr;           // hipGraphExec_t
  const void *gkb_ws = nullptr;
  size_t gkb_ws_bytes = 0;
  int gkb_tp = 0, gkb_tb = 0;
  uint64_t gkb_tune = 0;
  hipStream_t cap_stream = nullptr;   // the handle's own stream for captures
  void *blas = nullptr;               // rocblas_handle of this handle's solver calls
  void *ws_rows = nullptr;           // batch x nz x H x max(ny, sy) complex: row-pass <-> column-pass
  void *ws_cols = nullptr;           // batch x LG x H x max(sy, ...) complex: column-pass partials / D1
  size_t ws_rows_bytes = 0, ws_cols_bytes = 0;
  int lg_G = 1;                      // layer groups of the G column pass (partial sums)
  int lg_GT = 1;                     // layer groups of the G^T column pass
  // RSVD orthonormalizations so far: by CholeskyQR2, by shifted CholeskyQR3, by Householder QR
  int64_t qr_cholesky2 = 0, qr_cholesky3 = 0, qr_householder = 0;
  // pass profiling: 4 events per profiled call (before pass 1, after passes 1-3)
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_kind;        // transpose flag of each profiled call
  int prof_cap = 0, prof_n = 0, prof_cur = -1;
};

namespace ff {
size_t csize(int dtype);
// Pass workspace of the operator: row-pass <-> column-pass intermediates (`rows`), column-pass
// partial sums or transformed data rows (`cols`), and the vectors per launch they hold.
struct OpWs {
  void *rows, *cols;
  int batch;
};
// operator passes (apply.hip): op_apply runs on the handle's own workspace, op_apply_ws on the
// caller's; op_ws_per_vector gives the bytes one vector of a launch needs in each region
ff_status op_apply(ff_spectra h, int transpose, int64_t k, const void *X, int64_t ldx, void *Y,
                   int64_t ldy, const void *w_pre, const void *w_post, int io_dtype,
                   hipStream_t s);
ff_status op_apply_ws(ff_spectra h, const OpWs &ws, int transpose, int64_t k, const void *X, int64_t ldx,
                      void *Y, int64_t ldy, const void *w_pre, const void *w_post, int io_dtype, hipStream_t s);
void op_ws_per_vector(ff_spectra h, int transpose, size_t *rows_bytes, size_t *cols_bytes);
// vectors of one type in and another out (single-precision handles: FP64 in, FP32 out or the
// reverse); w_pre has the input type, w_post the output type
ff_status op_apply_io(ff_spectra h, int transpose, int64_t k, const void *X, int64_t ldx, void *Y, int64_t ldy,
                      const void *w_pre, const void *w_post, int in_dtype, int out_dtype, hipStream_t s);
ff_status op_time_pass(ff_spectra h, int transpose, int pass, int reps, const void *X, void *Y, hipStream_t s);
// spectra construction (spectra.hip)
ff_status make_spectra(ff_spectra h, hipStream_t s);
ff_status kernel_table(ff_spectra h, double *table, hipStream_t s);
// wave groups per block of the column passes (layer split inside a block)
int col_wave_groups(int dtype, int NY);
// records profiling event `slot` (0..3) of the current profiled call, if profiling is on
void prof_mark(ff_spectra h, int slot, int transpose, hipStream_t s);
// destroys the handle's rocBLAS handle, if it has one (solvers.hip)
void release_blas(ff_spectra h);
}  // namespace ff

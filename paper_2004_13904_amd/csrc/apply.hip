// Host launchers of the three-pass BCCB operator (Appendix A of the paper): G X and G^T Y for
// a batch of vectors, with the diagonal weights of eq. (forwardmult) fused into the first and
// last passes.  Launches are asynchronous on the caller's stream and allocate nothing.
#include <type_traits>

#include "plan_passes.h"

namespace ff {
namespace {


// One pass of G (transpose = 0) or G^T (transpose = 1) for kb vectors: pass 0 = row
// transforms, 1 = column transforms with the spectral products, 2 = inverse row transforms,
// each with the handle's stage plan of its transforms.
template <typename T, typename TI, typename TO>
ff_status run_pass(ff_spectra h, const OpWs &ws, int transpose, int pass, int kb, const TI *X, int64_t ldx, TO *Y,
                   int64_t ldy_out, const TI *pre, const TO *post, hipStream_t s) {
  if (pass == 1) {
    switch (plan_canon(h->NY, h->fft_plan_y)) {
      case 0: return col_pass<0, T>(h, ws, transpose, kb, s);
      case 1: return col_pass<1, T>(h, ws, transpose, kb, s);
      default: return col_pass<2, T>(h, ws, transpose, kb, s);
    }
  }
  const int px = plan_canon(h->NX, h->fft_plan_x);
  if (pass == 0) {
    switch (px) {
      case 0: return r2c_pass<0, T, TI>(h, ws, transpose, kb, X, ldx, pre, s);
      case 1: return r2c_pass<1, T, TI>(h, ws, transpose, kb, X, ldx, pre, s);
      default: return r2c_pass<2, T, TI>(h, ws, transpose, kb, X, ldx, pre, s);
    }
  }
  switch (px) {
    case 0: return c2r_pass<0, T, TO>(h, ws, transpose, kb, Y, ldy_out, post, s);
    case 1: return c2r_pass<1, T, TO>(h, ws, transpose, kb, Y, ldy_out, post, s);
    default: return c2r_pass<2, T, TO>(h, ws, transpose, kb, Y, ldy_out, post, s);
  }
}

template <typename T, typename TI, typename TO>
ff_status run_op(ff_spectra h, const OpWs &ws, int transpose, int kb, const TI *X, int64_t ldx, TO *Y, int64_t ldy,
                 const TI *pre, const TO *post, hipStream_t s) {
  for (int pass = 0; pass < 3; ++pass) {
    prof_mark(h, pass, transpose, s);
    ff_status st = run_pass<T, TI, TO>(h, ws, transpose, pass, kb, X, ldx, Y, ldy, pre, post, s);
    if (st != FF_OK) return st;
  }
  prof_mark(h, 3, transpose, s);
  return FF_OK;
}

// k vectors of type TI in, of type TO out (the pre-weights are TI values, the post-weights TO)
template <typename T, typename TI, typename TO>
ff_status run(ff_spectra h, const OpWs &ws, int transpose, int64_t k, const void *X, int64_t ldx, void *Y,
              int64_t ldy, const void *w_pre, const void *w_post, hipStream_t s) {
  const TI *x = (const TI *)X;
  TO *y = (TO *)Y;
  const int B = ws.batch;
  for (int64_t c0 = 0; c0 < k; c0 += B) {
    const int kb = (int)((k - c0) < B ? (k - c0) : B);
    ff_status st = run_op<T, TI, TO>(h, ws, transpose, kb, x + c0 * ldx, ldx, y + c0 * ldy, ldy,
                                     (const TI *)w_pre, (const TO *)w_post, s);
    if (st != FF_OK) return st;
  }
  return FF_OK;
}

OpWs handle_ws(ff_spectra h) { return OpWs{h->ws_rows, h->ws_cols, h->batch}; }

}  // namespace

int col_wave_groups(int dtype, int NY) {
  int w = 1;
  auto pick = [&](auto tag) {
    using T = decltype(tag);
    switch (NY) {
      case 8: w = ColCfg<T, 8>::WPB; break;
      case 16: w = ColCfg<T, 16>::WPB; break;
      case 32: w = ColCfg<T, 32>::WPB; break;
      case 64: w = ColCfg<T, 64>::WPB; break;
      case 128: w = ColCfg<T, 128>::WPB; break;
      case 256: w = ColCfg<T, 256>::WPB; break;
      case 512: w = ColCfg<T, 512>::WPB; break;
      case 1024: w = ColCfg<T, 1024>::WPB; break;
      case 2048: w = ColCfg<T, 2048>::WPB; break;
      default: w = 1;
    }
  };
  if (dtype == FF_F64) pick(double(0)); else pick(float(0));
  return w;
}

void prof_mark(ff_spectra h, int slot, int transpose, hipStream_t s) {
  if (h->prof_cap == 0) return;
  if (slot == 0) {
    h->prof_cur = -1;
    if (h->prof_n >= h->prof_cap) return;
    h->prof_cur = h->prof_n++;
    h->prof_kind[h->prof_cur] = transpose;
  }
  if (h->prof_cur < 0) return;
  (void)hipEventRecord(h->prof_ev[4 * h->prof_cur + slot], s);   // best effort: a failed mark only loses a timing
}

ff_status op_time_pass(ff_spectra h, int transpose, int pass, int reps, const void *X, void *Y, hipStream_t s) {
  // populate the intermediates with one full application, then repeat the chosen pass
  ff_status st = op_apply(h, transpose, 1, X, transpose ? h->m : h->n, Y, transpose ? h->n : h->m, nullptr, nullptr,
                          h->dtype, s);
  if (st != FF_OK) return st;
  const int64_t ldx = transpose ? h->m : h->n, ldy = transpose ? h->n : h->m;
  const OpWs ws = handle_ws(h);
  for (int r = 0; r < reps && st == FF_OK; ++r) {
    if (h->dtype == FF_F32)
      st = run_pass<float, float, float>(h, ws, transpose, pass, 1, (const float *)X, ldx, (float *)Y, ldy, nullptr,
                                         nullptr, s);
    else
      st = run_pass<double, double, double>(h, ws, transpose, pass, 1, (const double *)X, ldx, (double *)Y, ldy,
                                            nullptr, nullptr, s);
  }
  return st;
}

void op_ws_per_vector(ff_spectra h, int transpose, size_t *rows_bytes, size_t *cols_bytes) {
  const size_t cs = csize(h->dtype), HC = (size_t)(h->NX / 2);
  *rows_bytes = cs * (size_t)h->nz * HC * (size_t)h->ldy;
  *cols_bytes = cs * (transpose ? 1 : (size_t)h->lg_G) * HC * (size_t)h->lds;
}

ff_status op_apply_ws(ff_spectra h, const OpWs &ws, int transpose, int64_t k, const void *X, int64_t ldx, void *Y,
                      int64_t ldy, const void *w_pre, const void *w_post, int io_dtype, hipStream_t s) {
  if (ws.batch < 1 || !ws.rows || !ws.cols) return fail(FF_EINVAL, "operator workspace is empty");
  if (h->dtype == FF_F32 && io_dtype == FF_F32)
    return run<float, float, float>(h, ws, transpose, k, X, ldx, Y, ldy, w_pre, w_post, s);
  if (h->dtype == FF_F32 && io_dtype == FF_F64)
    return run<float, double, double>(h, ws, transpose, k, X, ldx, Y, ldy, w_pre, w_post, s);
  if (h->dtype == FF_F64 && io_dtype == FF_F64)
    return run<double, double, double>(h, ws, transpose, k, X, ldx, Y, ldy, w_pre, w_post, s);
  return fail(FF_EDTYPE, "vector dtype not supported for this handle");
}

ff_status op_apply_io(ff_spectra h, int transpose, int64_t k, const void *X, int64_t ldx, void *Y, int64_t ldy,
                      const void *w_pre, const void *w_post, int in_dtype, int out_dtype, hipStream_t s) {
  if (in_dtype == out_dtype) return op_apply(h, transpose, k, X, ldx, Y, ldy, w_pre, w_post, in_dtype, s);
  const OpWs ws = handle_ws(h);
  if (h->dtype == FF_F32 && in_dtype == FF_F64 && out_dtype == FF_F32)
    return run<float, double, float>(h, ws, transpose, k, X, ldx, Y, ldy, w_pre, w_post, s);
  if (h->dtype == FF_F32 && in_dtype == FF_F32 && out_dtype == FF_F64)
    return run<float, float, double>(h, ws, transpose, k, X, ldx, Y, ldy, w_pre, w_post, s);
  return fail(FF_EDTYPE, "vector dtypes not supported for this handle");
}

ff_status op_apply(ff_spectra h, int transpose, int64_t k, const void *X, int64_t ldx, void *Y, int64_t ldy,
                   const void *w_pre, const void *w_post, int io_dtype, hipStream_t s) {
  return op_apply_ws(h, handle_ws(h), transpose, k, X, ldx, Y, ldy, w_pre, w_post, io_dtype, s);
}

}  // namespace ff

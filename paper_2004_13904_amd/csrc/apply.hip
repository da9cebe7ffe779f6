// Host launchers of the three-pass BCCB operator (Appendix A of the paper): G X and G^T Y for
// a batch of vectors, with the diagonal weights of eq. (forwardmult) fused into the first and
// last passes.  Launches are asynchronous on the caller's stream and allocate nothing.
#include "passes.h"

namespace ff {
namespace {

template <typename T, typename TI, typename TO>
ff_status run_G(ff_spectra h, int kb, const TI *X, int64_t ldx, TO *Y, int64_t ldy, const TI *pre,
                const TO *post, hipStream_t s) {
  const int H = h->H, nz = h->nz, nx = h->nx, ny = h->ny, sx = h->sx, sy = h->sy, LG = h->lg_G;
  cplx<T> *X1 = (cplx<T> *)h->ws_rows;
  cplx<T> *Ap = (cplx<T> *)h->ws_cols;
  const cplx<T> *spec = (const cplx<T> *)h->spec;
  const cplx<T> *twx = (const cplx<T> *)h->tw_x, *twy = (const cplx<T> *)h->tw_y;
  const int64_t lay = (int64_t)ny * nx;
  FF_SWITCH_N(h->NX, {
    using C = RowCfg<T, NN>;
    dim3 g((ny + C::ROWS - 1) / C::ROWS, nz, kb);
    k_row_r2c<T, TI, NN><<<g, C::THREADS, 0, s>>>(X, Idx3{ldx, lay, nx}, pre, Idx3{0, lay, nx}, ny, nx, 0, X1,
                                                   Idx3{(int64_t)nz * H * ny, (int64_t)H * ny, 1}, ny, twx);
  });
  FF_LAUNCH_CHECK("G pass 1 (row transforms)");
  FF_SWITCH_N(h->NY, {
    using CC = ColCfg<NN>;
    dim3 g((H + CC::CPB - 1) / CC::CPB, LG, kb);
    k_col_G<T, NN><<<g, CC::THREADS, 0, s>>>(X1, ny, nz, H, LG, spec, Ap, sy, h->pyl, twy);
  });
  FF_LAUNCH_CHECK("G pass 2 (column transforms and spectral products)");
  FF_SWITCH_N(h->NX, {
    using C = RowCfg<T, NN>;
    dim3 g((sy + C::ROWS - 1) / C::ROWS, 1, kb);
    k_row_c2r<T, TO, NN><<<g, C::THREADS, 0, s>>>(Ap, Idx3{(int64_t)LG * H * sy, 0, 1}, sy, (int64_t)H * sy, LG, sy,
                                                   Y, Idx3{ldy, 0, sx}, post, Idx3{0, 0, sx}, sx, h->pxl, twx);
  });
  FF_LAUNCH_CHECK("G pass 3 (inverse row transforms)");
  return FF_OK;
}

template <typename T, typename TI, typename TO>
ff_status run_GT(ff_spectra h, int kb, const TI *X, int64_t ldx, TO *Y, int64_t ldy, const TI *pre,
                 const TO *post, hipStream_t s) {
  const int H = h->H, nz = h->nz, nx = h->nx, ny = h->ny, sx = h->sx, sy = h->sy, LG = h->lg_GT;
  cplx<T> *X1 = (cplx<T> *)h->ws_rows;
  cplx<T> *D1 = (cplx<T> *)h->ws_cols;
  const cplx<T> *spec = (const cplx<T> *)h->spec;
  const cplx<T> *twx = (const cplx<T> *)h->tw_x, *twy = (const cplx<T> *)h->tw_y;
  const int64_t lay = (int64_t)ny * nx;
  FF_SWITCH_N(h->NX, {
    using C = RowCfg<T, NN>;
    dim3 g((sy + C::ROWS - 1) / C::ROWS, 1, kb);
    k_row_r2c<T, TI, NN><<<g, C::THREADS, 0, s>>>(X, Idx3{ldx, 0, sx}, pre, Idx3{0, 0, sx}, sy, sx, h->pxl, D1,
                                                   Idx3{(int64_t)H * sy, 0, 1}, sy, twx);
  });
  FF_LAUNCH_CHECK("G^T pass 1 (row transforms)");
  FF_SWITCH_N(h->NY, {
    using CC = ColCfg<NN>;
    dim3 g((H + CC::CPB - 1) / CC::CPB, LG, kb);
    k_col_GT<T, NN><<<g, CC::THREADS, 0, s>>>(D1, sy, h->pyl, nz, H, LG, spec, X1, ny, twy);
  });
  FF_LAUNCH_CHECK("G^T pass 2 (column transforms and spectral products)");
  FF_SWITCH_N(h->NX, {
    using C = RowCfg<T, NN>;
    dim3 g((ny + C::ROWS - 1) / C::ROWS, nz, kb);
    k_row_c2r<T, TO, NN><<<g, C::THREADS, 0, s>>>(X1, Idx3{(int64_t)nz * H * ny, (int64_t)H * ny, 1}, ny, 0, 1, ny,
                                                   Y, Idx3{ldy, lay, nx}, post, Idx3{0, lay, nx}, nx, 0, twx);
  });
  FF_LAUNCH_CHECK("G^T pass 3 (inverse row transforms)");
  return FF_OK;
}

template <typename T, typename TIO>
ff_status run(ff_spectra h, int transpose, int64_t k, const void *X, int64_t ldx, void *Y, int64_t ldy,
              const void *w_pre, const void *w_post, hipStream_t s) {
  const TIO *x = (const TIO *)X;
  TIO *y = (TIO *)Y;
  for (int64_t c0 = 0; c0 < k; c0 += kMaxBatch) {
    const int kb = (int)((k - c0) < kMaxBatch ? (k - c0) : kMaxBatch);
    ff_status st = transpose
        ? run_GT<T, TIO, TIO>(h, kb, x + c0 * ldx, ldx, y + c0 * ldy, ldy, (const TIO *)w_pre, (const TIO *)w_post, s)
        : run_G<T, TIO, TIO>(h, kb, x + c0 * ldx, ldx, y + c0 * ldy, ldy, (const TIO *)w_pre, (const TIO *)w_post, s);
    if (st != FF_OK) return st;
  }
  return FF_OK;
}

}  // namespace

ff_status op_apply(ff_spectra h, int transpose, int64_t k, const void *X, int64_t ldx, void *Y, int64_t ldy,
                   const void *w_pre, const void *w_post, int io_dtype, hipStream_t s) {
  if (h->dtype == FF_F32 && io_dtype == FF_F32)
    return run<float, float>(h, transpose, k, X, ldx, Y, ldy, w_pre, w_post, s);
  if (h->dtype == FF_F32 && io_dtype == FF_F64)
    return run<float, double>(h, transpose, k, X, ldx, Y, ldy, w_pre, w_post, s);
  if (h->dtype == FF_F64 && io_dtype == FF_F64)
    return run<double, double>(h, transpose, k, X, ldx, Y, ldy, w_pre, w_post, s);
  return fail(FF_EDTYPE, "vector dtype not supported for this handle");
}

}  // namespace ff

// Host launchers of the three-pass BCCB operator (Appendix A of the paper): G X and G^T Y for
// a batch of vectors, with the diagonal weights of eq. (forwardmult) fused into the first and
// last passes.  Launches are asynchronous on the caller's stream and allocate nothing.
#include <type_traits>

#include "passes.h"

namespace ff {
namespace {


// Row-pass tile: transforms per block (a block of NF transforms writes 2*NF-row contiguous
// segments).  `tile` is the handle's row_tile: 1 = one transform, 2 = the largest that fits LDS,
// 3 = four, 4 = two (capped by the largest); 0 = automatic by the rows of the pass (measured on
// 512- and 256-point rows): one transform below 512 rows and two below 1024, so that small passes
// still spread over the chip; four for larger forward passes; four for inverse passes below 2048
// rows and the largest above (its 2*NF-row write segments fetch fewer partial cache lines).
inline int row_nf(int tile, int64_t rows, int nfm, bool inverse) {
  int nf;
  if (tile == 1) nf = 1;
  else if (tile == 2) nf = nfm;
  else if (tile == 3) nf = 4;
  else if (tile == 4) nf = 2;
  else nf = rows < 512 ? 1 : rows < 1024 ? 2 : (inverse && rows >= 2048) ? nfm : 4;
  return nf < nfm ? nf : nfm;
}

template <typename T, typename TI, int N, int NF>
void launch_r2c_nf(int nrows, int nb, int kb, const TI *in, Idx3 ii, const TI *pre, Idx3 pi, int len, int off,
                   cplx<T> *out, Idx3 oi, int64_t out_kx, const cplx<T> *tw, hipStream_t s) {
  using C = RowCfg<T, N, NF>;
  dim3 g((nrows * nb + C::ROWS - 1) / C::ROWS, 1, kb);
  k_row_r2c<T, TI, N, NF><<<g, C::THREADS, 0, s>>>(in, ii, pre, pi, nrows, nb, len, off, out, oi, out_kx, tw);
}

template <typename T, typename TI, int N>
void launch_r2c(int tile, int nrows, int nb, int kb, const TI *in, Idx3 ii, const TI *pre, Idx3 pi, int len, int off,
                cplx<T> *out, Idx3 oi, int64_t out_kx, const cplx<T> *tw, hipStream_t s) {
  constexpr int NFM = RowMax<T, N>::NF;
  constexpr int NF4 = NFM < 4 ? NFM : 4, NF2 = NFM < 2 ? NFM : 2;
  const int nf = row_nf(tile, (int64_t)nrows * nb * kb, NFM, false);
  if (nf == NFM)
    launch_r2c_nf<T, TI, N, NFM>(nrows, nb, kb, in, ii, pre, pi, len, off, out, oi, out_kx, tw, s);
  else if (nf == NF4)
    launch_r2c_nf<T, TI, N, NF4>(nrows, nb, kb, in, ii, pre, pi, len, off, out, oi, out_kx, tw, s);
  else if (nf == NF2)
    launch_r2c_nf<T, TI, N, NF2>(nrows, nb, kb, in, ii, pre, pi, len, off, out, oi, out_kx, tw, s);
  else
    launch_r2c_nf<T, TI, N, 1>(nrows, nb, kb, in, ii, pre, pi, len, off, out, oi, out_kx, tw, s);
}

template <typename T, typename TO, int N, int NF>
void launch_c2r_nf(int nrows, int nb, int kb, const cplx<T> *in, Idx3 ii, int64_t in_kx, int64_t pstride, int P,
                   TO *out, Idx3 oi, const TO *post, Idx3 qi, int len, int off, const cplx<T> *tw, hipStream_t s) {
  using C = RowCfg<T, N, NF>;
  dim3 g((nrows * nb + C::ROWS - 1) / C::ROWS, 1, kb);
  k_row_c2r<T, TO, N, NF><<<g, C::THREADS, 0, s>>>(in, ii, in_kx, pstride, P, nrows, nb, out, oi, post, qi, len, off, tw);
}

template <typename T, typename TO, int N>
void launch_c2r(int tile, int nrows, int nb, int kb, const cplx<T> *in, Idx3 ii, int64_t in_kx, int64_t pstride,
                int P, TO *out, Idx3 oi, const TO *post, Idx3 qi, int len, int off, const cplx<T> *tw, hipStream_t s) {
  constexpr int NFM = RowMax<T, N>::NF;
  constexpr int NF4 = NFM < 4 ? NFM : 4, NF2 = NFM < 2 ? NFM : 2;
  const int nf = row_nf(tile, (int64_t)nrows * nb * kb, NFM, true);
  if (nf == NFM)
    launch_c2r_nf<T, TO, N, NFM>(nrows, nb, kb, in, ii, in_kx, pstride, P, out, oi, post, qi, len, off, tw, s);
  else if (nf == NF4)
    launch_c2r_nf<T, TO, N, NF4>(nrows, nb, kb, in, ii, in_kx, pstride, P, out, oi, post, qi, len, off, tw, s);
  else if (nf == NF2)
    launch_c2r_nf<T, TO, N, NF2>(nrows, nb, kb, in, ii, in_kx, pstride, P, out, oi, post, qi, len, off, tw, s);
  else
    launch_c2r_nf<T, TO, N, 1>(nrows, nb, kb, in, ii, in_kx, pstride, P, out, oi, post, qi, len, off, tw, s);
}

// One pass of G (transpose = 0) or G^T (transpose = 1) for kb vectors: pass 0 = row
// transforms, 1 = column transforms with the spectral products, 2 = inverse row transforms.
template <typename T, typename TI, typename TO>
ff_status run_pass(ff_spectra h, const OpWs &ws, int transpose, int pass, int kb, const TI *X, int64_t ldx, TO *Y,
                   int64_t ldy_out, const TI *pre, const TO *post, hipStream_t s) {
  const int HC = h->NX / 2, nz = h->nz, nx = h->nx, ny = h->ny, sx = h->sx, sy = h->sy;
  const int ldy = h->ldy, lds = h->lds;
  cplx<T> *X1 = (cplx<T> *)ws.rows;   // [vec][r][c][row] (ld ldy), HC column slots
  cplx<T> *C2 = (cplx<T> *)ws.cols;   // G: partial sums [vec][g][c][j]; G^T: D1 [vec][c][j] (ld lds)
  const cplx<T> *spec = (const cplx<T> *)h->spec;
  const cplx<T> *twx = (const cplx<T> *)h->tw_x, *twy = (const cplx<T> *)h->tw_y;
  const int64_t lay = (int64_t)ny * nx;
  if (!transpose) {
    const int LG = h->lg_G;
    if (pass == 0) {
      FF_SWITCH_N(h->NX, launch_r2c<T, TI, NN>(h->row_tile, ny, nz, kb, X, Idx3{ldx, lay, nx}, pre, Idx3{0, lay, nx}, nx, 0, X1,
                                               Idx3{(int64_t)nz * HC * ldy, (int64_t)HC * ldy, 1}, ldy, twx, s));
      FF_LAUNCH_CHECK("G pass 1 (row transforms)");
    } else if (pass == 1) {
      const bool half = 2 * ny <= h->NY && 2 * (h->pyl + sy) <= h->NY;
      FF_SWITCH_N(h->NY, {
        using CC = ColCfg<T, NN>;
        if constexpr (BatchCfg<T, NN>::OK) {
          if (kb > 1 && h->col_batched) {
            dim3 g((HC + CC::CPB - 1) / CC::CPB, LG, (kb + BatchCfg<T, NN>::V - 1) / BatchCfg<T, NN>::V);
            if (half)
              k_col_G_batch<T, NN, true><<<g, CC::THREADS * CC::WPB, 0, s>>>(X1, ny, ldy, nz, HC, LG, kb, spec,
                                                                          C2, sy, lds, h->pyl, twy);
            else
              k_col_G_batch<T, NN, false><<<g, CC::THREADS * CC::WPB, 0, s>>>(X1, ny, ldy, nz, HC, LG, kb, spec,
                                                                           C2, sy, lds, h->pyl, twy);
            break;
          }
        }
        dim3 g((HC + CC::CPB - 1) / CC::CPB, LG, kb);
        if (half)
          k_col_G<T, NN, true><<<g, CC::THREADS * CC::WPB, 0, s>>>(X1, ny, ldy, nz, HC, LG, spec, C2, sy, lds, h->pyl, twy);
        else
          k_col_G<T, NN, false><<<g, CC::THREADS * CC::WPB, 0, s>>>(X1, ny, ldy, nz, HC, LG, spec, C2, sy, lds, h->pyl, twy);
      });
      FF_LAUNCH_CHECK("G pass 2 (column transforms and spectral products)");
    } else {
      FF_SWITCH_N(h->NX, launch_c2r<T, TO, NN>(h->row_tile, sy, 1, kb, C2, Idx3{(int64_t)LG * HC * lds, 0, 1}, lds, (int64_t)HC * lds,
                                               LG, Y, Idx3{ldy_out, 0, sx}, post, Idx3{0, 0, sx}, sx, h->pxl, twx, s));
      FF_LAUNCH_CHECK("G pass 3 (inverse row transforms)");
    }
  } else {
    const int LG = h->lg_GT;
    if (pass == 0) {
      FF_SWITCH_N(h->NX, launch_r2c<T, TI, NN>(h->row_tile, sy, 1, kb, X, Idx3{ldx, 0, sx}, pre, Idx3{0, 0, sx}, sx, h->pxl, C2,
                                               Idx3{(int64_t)HC * lds, 0, 1}, lds, twx, s));
      FF_LAUNCH_CHECK("G^T pass 1 (row transforms)");
    } else if (pass == 1) {
      const bool half = 2 * ny <= h->NY && 2 * (h->pyl + sy) <= h->NY;
      FF_SWITCH_N(h->NY, {
        using CC = ColCfg<T, NN>;
        if constexpr (BatchCfg<T, NN>::OK) {
          if (kb > 1 && h->col_batched) {
            dim3 g((HC + CC::CPB - 1) / CC::CPB, LG, (kb + BatchCfg<T, NN>::V - 1) / BatchCfg<T, NN>::V);
            if (half)
              k_col_GT_batch<T, NN, true><<<g, CC::THREADS * CC::WPB, 0, s>>>(C2, sy, lds, h->pyl, nz, HC, LG, kb,
                                                                           spec, X1, ny, ldy, twy);
            else
              k_col_GT_batch<T, NN, false><<<g, CC::THREADS * CC::WPB, 0, s>>>(C2, sy, lds, h->pyl, nz, HC, LG, kb,
                                                                            spec, X1, ny, ldy, twy);
            break;
          }
        }
        dim3 g((HC + CC::CPB - 1) / CC::CPB, LG, kb);
        if (half)
          k_col_GT<T, NN, true><<<g, CC::THREADS * CC::WPB, 0, s>>>(C2, sy, lds, h->pyl, nz, HC, LG, spec, X1, ny, ldy, twy);
        else
          k_col_GT<T, NN, false><<<g, CC::THREADS * CC::WPB, 0, s>>>(C2, sy, lds, h->pyl, nz, HC, LG, spec, X1, ny, ldy, twy);
      });
      FF_LAUNCH_CHECK("G^T pass 2 (column transforms and spectral products)");
    } else {
      FF_SWITCH_N(h->NX, launch_c2r<T, TO, NN>(h->row_tile, ny, nz, kb, X1, Idx3{(int64_t)nz * HC * ldy, (int64_t)HC * ldy, 1}, ldy, 0,
                                               1, Y, Idx3{ldy_out, lay, nx}, post, Idx3{0, lay, nx}, nx, 0, twx, s));
      FF_LAUNCH_CHECK("G^T pass 3 (inverse row transforms)");
    }
  }
  return FF_OK;
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

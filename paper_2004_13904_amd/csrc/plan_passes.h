// Host launchers of the three passes of the BCCB operator (Appendix A of the paper) for one
// stage plan FP of the transforms (fft.h): the row passes use the plan of the NX-point row
// transforms, the column pass that of the NY-point column transforms.  Each plan's launchers
// are compiled in a translation unit of their own (plan0.hip .. plan2.hip); apply.hip picks
// the unit by the handle's plans.  A plan that is not canonical for the size (plan_canon) is
// never launched: the dispatcher maps it to the canonical one first.
#pragma once

#include "passes.h"

namespace ff {

// The passes for kb vectors (OpWs: intermediates).  r2c_pass: pass 1 of G (rows of the model,
// input X of type TI, weights pre) or of G^T (rows of the data); col_pass: pass 2; c2r_pass:
// pass 3 of G (station rows out, weights post) or of G^T (model rows out).
template <int FP, typename T, typename TI>
ff_status r2c_pass(ff_spectra h, const OpWs &ws, int transpose, int kb, const TI *X, int64_t ldx, const TI *pre,
                   hipStream_t s);
template <int FP, typename T>
ff_status col_pass(ff_spectra h, const OpWs &ws, int transpose, int kb, hipStream_t s);
template <int FP, typename T, typename TO>
ff_status c2r_pass(ff_spectra h, const OpWs &ws, int transpose, int kb, TO *Y, int64_t ldy_out, const TO *post,
                   hipStream_t s);

// block products whose G column pass is the vector-parallel one (k_col_G_vec), which leaves
// one layer-group partial per vector (G^T keeps the 4-vector pass)
inline bool vec_cols(ff_spectra h, int kb) {
  return kb > 1 && h->col_batched == 2 && h->dtype == FF_F32 && h->NY <= 512;
}

#ifdef FF_PLAN_UNIT
namespace {

// Row-pass tile: transforms per block (a block of NF transforms writes 2*NF-row contiguous
// segments).  `tile` is the handle's row_tile: 1 = one transform, 2 = the largest that fits LDS,
// 3 = four, 4 = two (capped by the largest); 0 = automatic by the rows of the pass (measured on
// 512- and 256-point rows): one transform below 512 rows and two below 1024, so that small passes
// still spread over the chip; four for larger forward passes; four for inverse passes below 2048
// rows and the largest above (its 2*NF-row segments fill whole cache lines); the largest for
// every pass of at least 16384 rows (block products: G of the k = 3750 block of the 200 x 150 x 12
// survey 6 % faster than with four).
inline int row_nf(int tile, int64_t rows, int nfm, bool inverse) {
  int nf;
  if (tile == 1) nf = 1;
  else if (tile == 2) nf = nfm;
  else if (tile == 3) nf = 4;
  else if (tile == 4) nf = 2;
  else nf = rows < 512 ? 1 : rows < 1024 ? 2 : (rows >= 16384 || (inverse && rows >= 2048)) ? nfm : 4;
  return nf < nfm ? nf : nfm;
}

template <typename T, typename TI, int N, int NF, int FP>
void launch_r2c_nf(int nrows, int nb, int kb, const TI *in, Idx3 ii, const TI *pre, Idx3 pi, int len, int off,
                   cplx<T> *out, Idx3 oi, int64_t out_kx, const cplx<T> *tw, hipStream_t s) {
  using C = RowCfg<T, N, NF>;
  dim3 g(row_blocks(nrows, nb, C::ROWS), 1, kb);
  k_row_r2c<T, TI, N, NF, true, FP><<<g, C::THREADS, 0, s>>>(in, ii, pre, pi, nrows, nb, len, off, out, oi, out_kx, tw);
}

template <typename T, typename TI, int N, int FP>
void launch_r2c(int tile, int nrows, int nb, int kb, const TI *in, Idx3 ii, const TI *pre, Idx3 pi, int len, int off,
                cplx<T> *out, Idx3 oi, int64_t out_kx, const cplx<T> *tw, hipStream_t s) {
  constexpr int NFM = RowMax<T, N>::NF;
  constexpr int NF4 = NFM < 4 ? NFM : 4, NF2 = NFM < 2 ? NFM : 2;
  const int nf = row_nf(tile, (int64_t)nrows * nb * kb, NFM, false);
  if (nf == NFM)
    launch_r2c_nf<T, TI, N, NFM, FP>(nrows, nb, kb, in, ii, pre, pi, len, off, out, oi, out_kx, tw, s);
  else if (nf == NF4)
    launch_r2c_nf<T, TI, N, NF4, FP>(nrows, nb, kb, in, ii, pre, pi, len, off, out, oi, out_kx, tw, s);
  else if (nf == NF2)
    launch_r2c_nf<T, TI, N, NF2, FP>(nrows, nb, kb, in, ii, pre, pi, len, off, out, oi, out_kx, tw, s);
  else
    launch_r2c_nf<T, TI, N, 1, FP>(nrows, nb, kb, in, ii, pre, pi, len, off, out, oi, out_kx, tw, s);
}

template <typename T, typename TO, int N, int NF, int FP>
void launch_c2r_nf(int nrows, int nb, int kb, const cplx<T> *in, Idx3 ii, int64_t in_kx, int64_t pstride, int P,
                   TO *out, Idx3 oi, const TO *post, Idx3 qi, int len, int off, const cplx<T> *tw, hipStream_t s) {
  using C = RowCfg<T, N, NF>;
  dim3 g(row_blocks(nrows, nb, C::ROWS), 1, kb);
  k_row_c2r<T, TO, N, NF, FP><<<g, C::THREADS, 0, s>>>(in, ii, in_kx, pstride, P, nrows, nb, out, oi, post, qi, len, off, tw);
}

template <typename T, typename TO, int N, int FP>
void launch_c2r(int tile, int nrows, int nb, int kb, const cplx<T> *in, Idx3 ii, int64_t in_kx, int64_t pstride,
                int P, TO *out, Idx3 oi, const TO *post, Idx3 qi, int len, int off, const cplx<T> *tw, hipStream_t s) {
  constexpr int NFM = RowMax<T, N>::NF;
  constexpr int NF4 = NFM < 4 ? NFM : 4, NF2 = NFM < 2 ? NFM : 2;
  const int nf = row_nf(tile, (int64_t)nrows * nb * kb, NFM, true);
  if (nf == NFM)
    launch_c2r_nf<T, TO, N, NFM, FP>(nrows, nb, kb, in, ii, in_kx, pstride, P, out, oi, post, qi, len, off, tw, s);
  else if (nf == NF4)
    launch_c2r_nf<T, TO, N, NF4, FP>(nrows, nb, kb, in, ii, in_kx, pstride, P, out, oi, post, qi, len, off, tw, s);
  else if (nf == NF2)
    launch_c2r_nf<T, TO, N, NF2, FP>(nrows, nb, kb, in, ii, in_kx, pstride, P, out, oi, post, qi, len, off, tw, s);
  else
    launch_c2r_nf<T, TO, N, 1, FP>(nrows, nb, kb, in, ii, in_kx, pstride, P, out, oi, post, qi, len, off, tw, s);
}

}  // namespace

template <int FP, typename T, typename TI>
ff_status r2c_pass(ff_spectra h, const OpWs &ws, int transpose, int kb, const TI *X, int64_t ldx, const TI *pre,
                   hipStream_t s) {
  const int HC = h->NX / 2, nz = h->nz, nx = h->nx, ny = h->ny, sx = h->sx, sy = h->sy;
  const int ldy = h->ldy, lds = h->lds;
  cplx<T> *X1 = (cplx<T> *)ws.rows;
  cplx<T> *C2 = (cplx<T> *)ws.cols;
  const cplx<T> *twx = (const cplx<T> *)h->tw_x;
  const int64_t lay = (int64_t)ny * nx;
  FF_SWITCH_N(h->NX, {
    if constexpr (plan_canon(NN, FP) != FP) return fail(FF_EINVAL, "stage plan is not canonical for the row size");
    else if (!transpose)
      launch_r2c<T, TI, NN, FP>(h->row_tile, ny, nz, kb, X, Idx3{ldx, lay, nx}, pre, Idx3{0, lay, nx}, nx, 0, X1,
                                Idx3{(int64_t)nz * HC * ldy, (int64_t)HC * ldy, 1}, ldy, twx, s);
    else
      launch_r2c<T, TI, NN, FP>(h->row_tile, sy, 1, kb, X, Idx3{ldx, 0, sx}, pre, Idx3{0, 0, sx}, sx, h->pxl, C2,
                                Idx3{(int64_t)HC * lds, 0, 1}, lds, twx, s);
  });
  FF_LAUNCH_CHECK(transpose ? "G^T pass 1 (row transforms)" : "G pass 1 (row transforms)");
  return FF_OK;
}

template <int FP, typename T, typename TO>
ff_status c2r_pass(ff_spectra h, const OpWs &ws, int transpose, int kb, TO *Y, int64_t ldy_out, const TO *post,
                   hipStream_t s) {
  const int HC = h->NX / 2, nz = h->nz, nx = h->nx, ny = h->ny, sx = h->sx, sy = h->sy;
  const int ldy = h->ldy, lds = h->lds;
  cplx<T> *X1 = (cplx<T> *)ws.rows;
  cplx<T> *C2 = (cplx<T> *)ws.cols;
  const cplx<T> *twx = (const cplx<T> *)h->tw_x;
  const int64_t lay = (int64_t)ny * nx;
  FF_SWITCH_N(h->NX, {
    if constexpr (plan_canon(NN, FP) != FP) return fail(FF_EINVAL, "stage plan is not canonical for the row size");
    else if (!transpose)
      launch_c2r<T, TO, NN, FP>(h->row_tile, sy, 1, kb, C2, Idx3{(int64_t)h->lg_G * HC * lds, 0, 1}, lds,
                                (int64_t)HC * lds, vec_cols(h, kb) ? 1 : h->lg_G, Y, Idx3{ldy_out, 0, sx}, post,
                                Idx3{0, 0, sx}, sx, h->pxl, twx, s);
    else
      launch_c2r<T, TO, NN, FP>(h->row_tile, ny, nz, kb, X1, Idx3{(int64_t)nz * HC * ldy, (int64_t)HC * ldy, 1}, ldy,
                                0, 1, Y, Idx3{ldy_out, lay, nx}, post, Idx3{0, lay, nx}, nx, 0, twx, s);
  });
  FF_LAUNCH_CHECK(transpose ? "G^T pass 3 (inverse row transforms)" : "G pass 3 (inverse row transforms)");
  return FF_OK;
}

template <int FP, typename T>
ff_status col_pass(ff_spectra h, const OpWs &ws, int transpose, int kb, hipStream_t s) {
  const int HC = h->NX / 2, nz = h->nz, ny = h->ny, sy = h->sy;
  const int ldy = h->ldy, lds = h->lds;
  cplx<T> *X1 = (cplx<T> *)ws.rows;
  cplx<T> *C2 = (cplx<T> *)ws.cols;
  const cplx<T> *spec = (const cplx<T> *)h->spec;
  const cplx<T> *twy = (const cplx<T> *)h->tw_y;
  const bool half = 2 * ny <= h->NY && 2 * (h->pyl + sy) <= h->NY;
  const int LG = transpose ? h->lg_GT : h->lg_G;
  FF_SWITCH_N(h->NY, {
    using CC = ColCfg<T, NN>;
    if constexpr (plan_canon(NN, FP) != FP) {
      return fail(FF_EINVAL, "stage plan is not canonical for the column size");
    } else {
      bool done = false;
      if constexpr (VecCfg<T, NN>::OK) {
        if (!transpose && vec_cols(h, kb)) {
          using VC = VecCfg<T, NN>;
          dim3 g((HC + CC::CPB - 1) / CC::CPB, (kb + VC::VV - 1) / VC::VV);
          const int64_t xs = (int64_t)nz * HC * ldy;
          if (half)
            k_col_G_vec<T, NN, true, FP><<<g, VC::THREADS, 0, s>>>(X1, ny, ldy, nz, HC, kb, xs, spec, C2,
                                                                  (int64_t)h->lg_G * HC * lds, sy, lds, h->pyl, twy);
          else
            k_col_G_vec<T, NN, false, FP><<<g, VC::THREADS, 0, s>>>(X1, ny, ldy, nz, HC, kb, xs, spec, C2,
                                                                   (int64_t)h->lg_G * HC * lds, sy, lds, h->pyl, twy);
          done = true;
        }
      }
      if constexpr (BatchCfg<T, NN>::OK) {
        if (!done && kb > 1 && h->col_batched) {
          dim3 g((HC + CC::CPB - 1) / CC::CPB, LG, (kb + BatchCfg<T, NN>::V - 1) / BatchCfg<T, NN>::V);
          if (!transpose && half)
            k_col_G_batch<T, NN, true, FP><<<g, CC::THREADS * CC::WPB, 0, s>>>(X1, ny, ldy, nz, HC, LG, kb, spec, C2,
                                                                            sy, lds, h->pyl, twy);
          else if (!transpose)
            k_col_G_batch<T, NN, false, FP><<<g, CC::THREADS * CC::WPB, 0, s>>>(X1, ny, ldy, nz, HC, LG, kb, spec, C2,
                                                                             sy, lds, h->pyl, twy);
          else if (half)
            k_col_GT_batch<T, NN, true, FP><<<g, CC::THREADS * CC::WPB, 0, s>>>(C2, sy, lds, h->pyl, nz, HC, LG, kb,
                                                                             spec, X1, ny, ldy, twy);
          else
            k_col_GT_batch<T, NN, false, FP><<<g, CC::THREADS * CC::WPB, 0, s>>>(C2, sy, lds, h->pyl, nz, HC, LG, kb,
                                                                              spec, X1, ny, ldy, twy);
          done = true;
        }
      }
      if (!done) {
        dim3 g((HC + CC::CPB - 1) / CC::CPB, LG, kb);
        if (!transpose && half)
          k_col_G<T, NN, true, FP><<<g, CC::THREADS * CC::WPB, 0, s>>>(X1, ny, ldy, nz, HC, LG, spec, C2, sy, lds,
                                                                    h->pyl, twy);
        else if (!transpose)
          k_col_G<T, NN, false, FP><<<g, CC::THREADS * CC::WPB, 0, s>>>(X1, ny, ldy, nz, HC, LG, spec, C2, sy, lds,
                                                                     h->pyl, twy);
        else if (half)
          k_col_GT<T, NN, true, FP><<<g, CC::THREADS * CC::WPB, 0, s>>>(C2, sy, lds, h->pyl, nz, HC, LG, spec, X1, ny,
                                                                     ldy, twy);
        else
          k_col_GT<T, NN, false, FP><<<g, CC::THREADS * CC::WPB, 0, s>>>(C2, sy, lds, h->pyl, nz, HC, LG, spec, X1,
                                                                      ny, ldy, twy);
      }
    }
  });
  FF_LAUNCH_CHECK(transpose ? "G^T pass 2 (column transforms and spectral products)"
                            : "G pass 2 (column transforms and spectral products)");
  return FF_OK;
}

// the explicit instantiations of one plan's translation unit
#define FF_PLAN_INSTANTIATE(FP)                                                                                   \
  template ff_status r2c_pass<FP, float, float>(ff_spectra, const OpWs &, int, int, const float *, int64_t,       \
                                                const float *, hipStream_t);                                      \
  template ff_status r2c_pass<FP, float, double>(ff_spectra, const OpWs &, int, int, const double *, int64_t,     \
                                                 const double *, hipStream_t);                                    \
  template ff_status r2c_pass<FP, double, double>(ff_spectra, const OpWs &, int, int, const double *, int64_t,    \
                                                  const double *, hipStream_t);                                   \
  template ff_status c2r_pass<FP, float, float>(ff_spectra, const OpWs &, int, int, float *, int64_t,             \
                                                const float *, hipStream_t);                                      \
  template ff_status c2r_pass<FP, float, double>(ff_spectra, const OpWs &, int, int, double *, int64_t,           \
                                                 const double *, hipStream_t);                                    \
  template ff_status c2r_pass<FP, double, double>(ff_spectra, const OpWs &, int, int, double *, int64_t,          \
                                                  const double *, hipStream_t);                                   \
  template ff_status col_pass<FP, float>(ff_spectra, const OpWs &, int, int, hipStream_t);                        \
  template ff_status col_pass<FP, double>(ff_spectra, const OpWs &, int, int, hipStream_t);
#endif  // FF_PLAN_UNIT

}  // namespace ff

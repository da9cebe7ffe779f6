// Pass kernels of the BCCB-embedded layered operator (Appendix A of the paper).
//
//   G x   : [row R2C along x of every model row, zero-padded to NX]            (pass 1)
//           [per column kx: FFT along y, multiply by the layer spectrum, sum the
//            layers in the frequency domain, inverse FFT along y, keep the station rows] (pass 2)
//           [row C2R along x of every station row, keep the station columns]    (pass 3)
//   G^T y : pass 1 on the data rows (embedded at the station offset), pass 2 with the
//           conjugate spectra and one inverse per layer, pass 3 on every model row.
//
// Intermediate layout between the passes is column-major per half-spectrum column
// ([batch][kx][row], rows contiguous) so that the column pass reads and writes whole
// contiguous columns and the row passes transpose through LDS.
#pragma once

#include <type_traits>

#include "fft.h"

namespace ff {

// Row-pass blocks: NF transforms (2 NF rows) per block.  NFMAX keeps the LDS of the
// transforms within 64 KB and the block within 1024 threads.
template <typename T, int N> struct RowMax {
  static constexpr int CS = (int)sizeof(cplx<T>);
  static constexpr int H = N / 2 + 1;
  static constexpr int LDSF = FFT<T, N, false>::LDS;
  static constexpr bool fits(int nf) {
    return nf * (N / 8) <= 1024 && (H * (2 * nf + 1) > nf * LDSF ? H * (2 * nf + 1) : nf * LDSF) * CS <= 65536;
  }
  static constexpr int NF = fits(8) ? 8 : fits(4) ? 4 : fits(2) ? 2 : 1;
};

template <typename T, int N, int NF_> struct RowCfg {
  static constexpr int NF = NF_;
  static constexpr int ROWS = 2 * NF;
  static constexpr int THREADS = NF * (N / 8);
  static constexpr int TS = ROWS + 1;                  // padded tile stride (bank conflicts)
  static constexpr int H = N / 2 + 1;
  static constexpr int LDSF = FFT<T, N, false>::LDS;   // per transform
  static constexpr int SH = H * TS > NF * LDSF ? H * TS : NF * LDSF;   // transforms, then tile
};

// Column-pass wave groups: CPB columns per wave group (one wavefront for NY <= 512), WPB
// wave groups per block splitting the layers (LDS of the block within 64 KB).
template <typename T, int NY> struct ColCfg {
  static constexpr int TPF = NY / 8;
  static constexpr int CPB = TPF >= 64 ? 1 : 64 / TPF;  // columns per wave group
  static constexpr int THREADS = CPB * TPF;             // threads per wave group
  static constexpr int GLDS = CPB * FFT<T, NY, false>::LDS;   // LDS elements per wave group
  static constexpr int byLds = 65536 / (GLDS * (int)sizeof(cplx<T>));
  static constexpr int WPB = TPF > 64 ? 1 : (byLds < 8 ? byLds : 8);
};

// Blocks of a row pass over nb batches of nrows rows, ROWS rows per block (RowMap).
inline int row_blocks(int nrows, int nb, int rows) { return nb * ((nrows + rows - 1) / rows); }

// Strides of a 3-level index (vector v, batch b within the vector, row) -> element offset.
struct Idx3 {
  int64_t v, b, row;
  __device__ __forceinline__ int64_t at(int64_t vv, int64_t bb, int64_t rr) const {
    return vv * v + bb * b + rr * row;
  }
};

// Rows of a row pass: each of the nb batches (layers) takes its nrows rows padded to a multiple
// of ROWS, so that a block's ROWS rows lie in one batch and start on a multiple of ROWS (whole
// cache lines of the column-major intermediates, whose row strides are multiples of 16
// elements).  Block bx holds rows row0 .. row0 + ROWS - 1 of batch b; the padding rows are
// neither read nor written.  A pass fills nb * ceil(nrows / ROWS) blocks (row_blocks).
template <class C> struct RowMap {
  int b, row0, nrows;
  bool ok;   // the block lies inside the pass
  __device__ __forceinline__ RowMap(int bx, int nrows_, int nb) : nrows(nrows_) {
    const int per = (nrows + C::ROWS - 1) / C::ROWS;   // blocks per batch
    b = bx / per;
    row0 = (bx - b * per) * C::ROWS;
    ok = b < nb;
  }
  __device__ __forceinline__ bool valid(int row) const { return ok && row < nrows; }
};

// Row of a transposed tile element: tile element idx belongs to tile row idx % ROWS, i.e. to
// row row0 + idx % ROWS of the block's batch.  When THREADS is a multiple of ROWS each thread
// always meets the same tile row.
template <class C> struct TileRow {
  static constexpr bool FIXED = C::THREADS % C::ROWS == 0;
  RowMap<C> m;
  int row;
  __device__ __forceinline__ TileRow(const RowMap<C> &m_) : m(m_) { row = m.row0 + (int)threadIdx.x % C::ROWS; }
  // false for a padding row or a block past the pass; else o = ix.at(vec, b, row)
  __device__ __forceinline__ bool get(int idx, const Idx3 &ix, int64_t vec, int64_t &o) const {
    const int r = FIXED ? row : m.row0 + idx % C::ROWS;
    o = ix.at(vec, m.b, r);
    return m.valid(r);
  }
};

// ---------------------------------------------------------------------------------------
// Pass 1: real rows -> half spectra along x, written transposed.
// Input row (vec, b, row) holds `len` values that sit at x = off .. off+len-1 of the length-N
// embedding (zero elsewhere); `pre` (optional) multiplies them (indexed without the vector
// stride).  Output element (vec, b, kx, row) at out[o.at(vec, b, row) + kx*out_kx], for
// kx < N/2 + 1, or with PACK for the N/2 column slots of the column passes (slot 0 holds the
// real DC and Nyquist bins as one complex value, DC + i Nyquist).  Rows as RowMap numbers them.
// Grid: (row_blocks(nrows, nb, ROWS), 1, nvec).
template <typename T, typename TI, int N, int NF, bool PACK = true, bool HALF = false, int FP = 0>
__device__ __forceinline__ void
row_r2c_body_h(cplx<T> *__restrict__ sh, int bx, int by, int64_t bz, const TI *__restrict__ in, Idx3 ii, const TI *__restrict__ pre, Idx3 pi, int nrows, int nb, int len,
          int off, cplx<T> *__restrict__ out, Idx3 oi, int64_t out_kx,
          const cplx<T> *__restrict__ tw) {
  using C = RowCfg<T, N, NF>;
  using F = FFT<T, N, false, FP>;
  const int f = threadIdx.x / F::TPF, j = threadIdx.x % F::TPF;
  const int64_t vec = bz;
  const RowMap<C> rm(bx, nrows, nb);
  const int qa = rm.row0 + 2 * f, qb = qa + 1, bq = rm.b;
  const bool va = rm.valid(qa), vb = rm.valid(qb);
  cplx<T> v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int c = j + u * F::TPF - off;
    T a = 0, bv = 0;
    if ((!HALF || u < 4) && c >= 0 && c < len) {
      if (va) {
        a = (T)in[ii.at(vec, bq, qa) + c];
        if (pre) a *= (T)pre[pi.at(0, bq, qa) + c];
      }
      if (vb) {
        bv = (T)in[ii.at(vec, bq, qb) + c];
        if (pre) bv *= (T)pre[pi.at(0, bq, qb) + c];
      }
    }
    v[u] = mk<T>(a, bv);
  }
  F::template run<HALF, false>(v, j, sh + f * F::LDS, tw);
  // separate the two packed real transforms: Xa = (Z_k + conj Z_{N-k})/2, Xb = (Z_k - conj Z_{N-k})/(2i)
  cplx<T> *z = sh + f * F::LDS;
#pragma unroll
  for (int u = 0; u < 8; ++u) z[j + u * F::TPF] = v[u];
  group_sync<F::TPF>();
  cplx<T> xa[5], xb[5];
#pragma unroll
  for (int u = 0; u < 5; ++u) {
    const int k = j + u * F::TPF;
    if (u < 4 || j == 0) {
      const cplx<T> zk = z[k], zr = z[(N - k) & (N - 1)];
      xa[u] = mk<T>((zk.x + zr.x) * (T)0.5, (zk.y - zr.y) * (T)0.5);
      xb[u] = mk<T>((zk.y + zr.y) * (T)0.5, (zr.x - zk.x) * (T)0.5);
    }
  }
  __syncthreads();
  cplx<T> *tile = sh;
#pragma unroll
  for (int u = 0; u < 5; ++u) {
    const int k = j + u * F::TPF;
    if (u < 4 || (!PACK && j == 0)) {
      cplx<T> a = xa[u], b = xb[u];
      if (PACK && u == 0 && j == 0) {   // both bins are real: slot 0 = DC + i Nyquist
        a.y = xa[4].x;
        b.y = xb[4].x;
      }
      tile[k * C::TS + 2 * f] = a;
      tile[k * C::TS + 2 * f + 1] = b;
    }
  }
  __syncthreads();
  constexpr int HO = PACK ? N / 2 : N / 2 + 1;   // output columns
  constexpr int PER = (HO * C::ROWS + C::THREADS - 1) / C::THREADS;
  cplx<T> tv[PER];   // every element read (clamped index), so that tv stays in registers
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = min((int)threadIdx.x + q * C::THREADS, HO * C::ROWS - 1);
    const int k = idx / C::ROWS, rr = idx - k * C::ROWS;
    tv[q] = tile[k * C::TS + rr];
  }
  TileRow<C> tr(rm);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = threadIdx.x + q * C::THREADS;
    const int k = idx / C::ROWS;
    int64_t o;
    if (idx < HO * C::ROWS && tr.get(idx, oi, vec, o)) out[o + k * out_kx] = tv[q];
  }
}

// The row values sit at x = off .. off + len - 1: when that lies in the first half of the
// embedding the transform skips the zero half of its input.
template <typename T, typename TI, int N, int NF, bool PACK = true, int FP = 0>
__device__ __forceinline__ void
row_r2c_body(cplx<T> *__restrict__ sh, int bx, int by, int64_t bz, const TI *__restrict__ in, Idx3 ii, const TI *__restrict__ pre, Idx3 pi, int nrows, int nb, int len,
          int off, cplx<T> *__restrict__ out, Idx3 oi, int64_t out_kx,
          const cplx<T> *__restrict__ tw) {
  if (2 * (off + len) <= N)
    row_r2c_body_h<T, TI, N, NF, PACK, true, FP>(sh, bx, by, bz, in, ii, pre, pi, nrows, nb, len, off, out, oi, out_kx, tw);
  else
    row_r2c_body_h<T, TI, N, NF, PACK, false, FP>(sh, bx, by, bz, in, ii, pre, pi, nrows, nb, len, off, out, oi, out_kx, tw);
}

template <typename T, typename TI, int N, int NF, bool PACK = true, int FP = 0>
__global__ void __launch_bounds__((RowCfg<T, N, NF>::THREADS))
k_row_r2c(const TI *__restrict__ in, Idx3 ii, const TI *__restrict__ pre, Idx3 pi, int nrows, int nb, int len,
          int off, cplx<T> *__restrict__ out, Idx3 oi, int64_t out_kx,
          const cplx<T> *__restrict__ tw) {
  __shared__ cplx<T> sh[RowCfg<T, N, NF>::SH];
  row_r2c_body<T, TI, N, NF, PACK, FP>(sh, blockIdx.x, blockIdx.y, blockIdx.z, in, ii, pre, pi, nrows, nb, len, off, out, oi, out_kx, tw);
}

// ---------------------------------------------------------------------------------------
// Pass 3: half spectra (vec, b, c, row) in the N/2 packed column slots of pass 1, summed over
// P partial buffers `pstride` apart, ->
// real rows; keeps x = off .. off+len-1, multiplies by `post` (optional, indexed without the
// vector stride).  Rows as RowMap numbers them.
// Grid: (row_blocks(nrows, nb, ROWS), 1, nvec).
template <typename T, typename TO, int N, int NF, bool HALF, int FP = 0>
__device__ __forceinline__ void
row_c2r_body_h(cplx<T> *__restrict__ sh, int bx, int by, int64_t bz, const cplx<T> *__restrict__ in, Idx3 ii, int64_t in_kx, int64_t pstride, int P, int nrows, int nb,
          TO *__restrict__ out, Idx3 oi, const TO *__restrict__ post, Idx3 qi, int len, int off,
          const cplx<T> *__restrict__ tw) {
  using C = RowCfg<T, N, NF>;
  using F = FFT<T, N, true, FP>;
  const int f = threadIdx.x / F::TPF, j = threadIdx.x % F::TPF;
  const int64_t vec = bz;
  const RowMap<C> rm(bx, nrows, nb);
  cplx<T> *tile = sh;
  // every thread issues all of its tile loads before the first LDS write, so the global
  // load latencies overlap instead of adding up
  constexpr int HI = N / 2;   // input column slots (slot 0 = DC + i Nyquist)
  constexpr int PER = (HI * C::ROWS + C::THREADS - 1) / C::THREADS;
  cplx<T> tv[PER];
  TileRow<C> tr(rm);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = threadIdx.x + q * C::THREADS;
    const int k = idx / C::ROWS;
    int64_t o;
    tv[q] = mk<T>(0, 0);
    if (idx < HI * C::ROWS && tr.get(idx, ii, vec, o)) tv[q] = in[o + k * in_kx];
  }
  for (int p = 1; p < P; ++p) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + q * C::THREADS;
      const int k = idx / C::ROWS;
      int64_t o;
      if (idx < HI * C::ROWS && tr.get(idx, ii, vec, o)) tv[q] = cadd<T>(tv[q], in[o + k * in_kx + p * pstride]);
    }
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = threadIdx.x + q * C::THREADS;
    const int k = idx / C::ROWS, rr = idx - k * C::ROWS;
    if (idx < HI * C::ROWS) tile[k * C::TS + rr] = tv[q];
  }
  __syncthreads();
  cplx<T> v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int k = j + u * F::TPF;
    cplx<T> A, B;
    if (k < N / 2) {
      A = tile[k * C::TS + 2 * f];
      B = tile[k * C::TS + 2 * f + 1];
      if (k == 0) {   // real signal: the DC bin is the real part of slot 0
        A.y = 0;
        B.y = 0;
      }
    } else if (k == N / 2) {   // the Nyquist bin is the imaginary part of slot 0
      A = mk<T>(tile[2 * f].y, 0);
      B = mk<T>(tile[2 * f + 1].y, 0);
    } else {
      A = cconj<T>(tile[(N - k) * C::TS + 2 * f]);
      B = cconj<T>(tile[(N - k) * C::TS + 2 * f + 1]);
    }
    v[u] = mk<T>(A.x - B.y, A.y + B.x);  // Z = A + i B
  }
  __syncthreads();
  F::template run<false, HALF>(v, j, sh + f * F::LDS, tw);
  const int qa = rm.row0 + 2 * f, qb = qa + 1, bq = rm.b;
  const bool va = rm.valid(qa), vb = rm.valid(qb);
#pragma unroll
  for (int u = 0; u < (HALF ? 4 : 8); ++u) {
    const int c = j + u * F::TPF - off;
    if (c >= 0 && c < len) {
      if (va) {
        T a = v[u].x;
        if (post) a *= (T)post[qi.at(0, bq, qa) + c];
        out[oi.at(vec, bq, qa) + c] = (TO)a;
      }
      if (vb) {
        T bv = v[u].y;
        if (post) bv *= (T)post[qi.at(0, bq, qb) + c];
        out[oi.at(vec, bq, qb) + c] = (TO)bv;
      }
    }
  }
}

// The kept values x = off .. off + len - 1: when they lie in the first half of the embedding
// the transform skips the outputs of the other half.
template <typename T, typename TO, int N, int NF, int FP = 0>
__device__ __forceinline__ void
row_c2r_body(cplx<T> *__restrict__ sh, int bx, int by, int64_t bz, const cplx<T> *__restrict__ in, Idx3 ii, int64_t in_kx, int64_t pstride, int P, int nrows, int nb,
          TO *__restrict__ out, Idx3 oi, const TO *__restrict__ post, Idx3 qi, int len, int off,
          const cplx<T> *__restrict__ tw) {
  if (2 * (off + len) <= N)
    row_c2r_body_h<T, TO, N, NF, true, FP>(sh, bx, by, bz, in, ii, in_kx, pstride, P, nrows, nb, out, oi, post, qi, len, off, tw);
  else
    row_c2r_body_h<T, TO, N, NF, false, FP>(sh, bx, by, bz, in, ii, in_kx, pstride, P, nrows, nb, out, oi, post, qi, len, off, tw);
}

template <typename T, typename TO, int N, int NF, int FP = 0>
__global__ void __launch_bounds__((RowCfg<T, N, NF>::THREADS))
k_row_c2r(const cplx<T> *__restrict__ in, Idx3 ii, int64_t in_kx, int64_t pstride, int P, int nrows, int nb,
          TO *__restrict__ out, Idx3 oi, const TO *__restrict__ post, Idx3 qi, int len, int off,
          const cplx<T> *__restrict__ tw) {
  __shared__ cplx<T> sh[RowCfg<T, N, NF>::SH];
  row_c2r_body<T, TO, N, NF, FP>(sh, blockIdx.x, blockIdx.y, blockIdx.z, in, ii, in_kx, pstride, P, nrows, nb, out, oi, post, qi, len, off, tw);
}

// ---------------------------------------------------------------------------------------
// Column passes.  The half spectrum along x has NX/2 + 1 columns, of which kx = 0 (DC) and
// kx = NX/2 (Nyquist) hold real sequences along y (the rows are real).  The row passes store
// them packed in one complex column, slot 0 = DC + i Nyquist, so the intermediates have
// HC = NX/2 column slots (slot c >= 1 is kx = c) and the column passes run over exactly HC
// columns.  For slot 0 the spectra hold, in place of S_r[0] and S_r[NX/2] (both Hermitian),
//   P_r = (S_r[0] + S_r[NX/2]) / 2   (spectrum column 0),
//   M_r = (S_r[0] - S_r[NX/2]) / 2   (spectrum column NX/2).
// With Z = FFT_y(DC + i Nyquist), the packed result of applying S_r[0] to the DC column and
// S_r[NX/2] to the Nyquist column is P_r[k] Z[k] + M_r[k] conj(Z[-k]) (the adjoint: the
// conjugate spectra), i.e. one extra product per layer and one index reversal per column.

// Pass 2 of G: for each column slot c and layer group g:
//   acc = sum_{r in group} S_r[c, :] .* FFT_y(X1[vec, r, c, 0:ny]),
//   out[vec, g, c, j] = IFFT_y(acc)[pyl + j], j in [0, sy).
// Slot 0 also sums accm = sum_r M_r .* FFT_y(...) and adds conj(accm[-k]) to acc[k] (each wave
// group on its own partial sums, before they are added up).
// X1 rows are stored [vec][r][c][y] (ld ldy); spectra [r][kx][ky] (HC + 1 columns).
// A block holds WPB wave groups on the same CPB columns; wave group w takes every WPB-th
// layer of the group (loading the next layer while transforming the current one); the
// partial sums are added up in LDS, each wave group taking a share of the elements, and wave
// group 0 does the inverse transform.
// Grid: (ceil(HC/CPB), LG, nvec).
template <typename T, int NY, bool HALF = false, int FP = 0>
__device__ __forceinline__ void
col_G_body(cplx<T> *__restrict__ sh, int bx, int by, int64_t bz, const cplx<T> *__restrict__ X1, int ny, int ldy, int nz, int HC, int LG,
        const cplx<T> *__restrict__ spec, cplx<T> *__restrict__ outp, int sy, int lds, int pyl,
        const cplx<T> *__restrict__ tw) {
  using CC = ColCfg<T, NY>;
  using Ff = FFT<T, NY, false, FP>;
  using Fi = FFT<T, NY, true, FP>;
  constexpr int TPF = CC::TPF, WPB = CC::WPB;
  const int w = threadIdx.x / CC::THREADS, lt = threadIdx.x % CC::THREADS;
  const int f = lt / TPF, j = lt % TPF;
  const int kx = bx * CC::CPB + f;
  const bool ok = kx < HC;
  const int kxs = ok ? kx : 0;
  const bool pk = bx == 0;   // block-uniform: this block holds the packed slot 0 (f == 0)
  const int64_t SH = HC + 1;         // spectrum columns
  const int g = by;
  const int64_t vec = bz;
  const int r0 = (int)((int64_t)g * nz / LG), r1 = (int)((int64_t)(g + 1) * nz / LG);
  cplx<T> *buf = sh + (w * CC::CPB + f) * Ff::LDS;
  typename Ff::Tw twr;
  Ff::load_tw(twr, j, tw);
  cplx<T> acc[8], xn[8], sn[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = mk<T>(0, 0);
  auto load = [&](int r) {
    const cplx<T> *src = X1 + ((vec * nz + r) * HC + kxs) * (int64_t)ldy;
    const cplx<T> *sp = spec + ((int64_t)r * SH + kxs) * NY;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int y = j + u * TPF;
      xn[u] = ((!HALF || u < 4) && ok && y < ny) ? src[y] : mk<T>(0, 0);
      sn[u] = sp[y];
    }
  };
  // NY <= 512: wave groups are independent, the layer loop may be ragged across them.
  // NY > 512: one wave group per block (WPB = 1), so the loop is uniform in the block.
  int r = r0 + w;
  if (r < r1) load(r);
  if (!pk) {
    for (; r < r1; r += WPB) {
      cplx<T> v[8], s[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        v[u] = xn[u];
        s[u] = sn[u];
      }
      if (r + WPB < r1) load(r + WPB);
      Ff::template run_tw<HALF, false>(v, j, buf, twr);
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = cadd<T>(acc[u], cmul<T>(v[u], s[u]));
    }
  } else {
    // the same loop plus the M_r products.  Single precision prefetches M_r with the rest;
    // double precision loads it at the start of its own iteration (register budget).
    constexpr bool PREFETCH = sizeof(T) == 4;
    cplx<T> accm[8], mn[8];
    auto loadm = [&](int rr) {
      const cplx<T> *mp = spec + ((int64_t)rr * SH + HC) * NY;
#pragma unroll
      for (int u = 0; u < 8; ++u) mn[u] = mp[j + u * TPF];
    };
#pragma unroll
    for (int u = 0; u < 8; ++u) accm[u] = mk<T>(0, 0);
    if (PREFETCH && r < r1) loadm(r);
    for (; r < r1; r += WPB) {
      cplx<T> v[8], s[8], mm[8];
      if (!PREFETCH) loadm(r);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        v[u] = xn[u];
        s[u] = sn[u];
        mm[u] = mn[u];
      }
      if (PREFETCH && r + WPB < r1) {
        load(r + WPB);
        loadm(r + WPB);
      }
      Ff::template run_tw<HALF, false>(v, j, buf, twr);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        acc[u] = cadd<T>(acc[u], cmul<T>(v[u], s[u]));
        accm[u] = cadd<T>(accm[u], cmul<T>(v[u], mm[u]));
      }
      if (!PREFETCH && r + WPB < r1) load(r + WPB);
    }
    // each wave group folds its own M sum in: acc[k] += conj(accm[-k]) (slot 0 lanes)
    group_sync<TPF>();
#pragma unroll
    for (int u = 0; u < 8; ++u) buf[pad8(j + u * TPF)] = accm[u];
    group_sync<TPF>();
    if (f == 0) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = cadd<T>(acc[u], cconj<T>(buf[pad8((NY - j - u * TPF) & (NY - 1))]));
    }
  }
  if constexpr (WPB > 1) {
    // partial sums of the wave groups meet in LDS (each in its own transform buffer).  Wave
    // group w adds up the elements u = w, w + WPB, ... of every lane over the wave groups in
    // order 0, 1, ..., and leaves the sums in wave group 0's buffer.
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) buf[j + u * TPF] = acc[u];
    __syncthreads();
    for (int u = w; u < 8; u += WPB) {
      const int e = f * Ff::LDS + j + u * TPF;
      cplx<T> t = sh[e];
      for (int w2 = 1; w2 < WPB; ++w2) t = cadd<T>(t, sh[w2 * CC::CPB * Ff::LDS + e]);
      sh[e] = t;
    }
    __syncthreads();
    if (w != 0) return;
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = buf[j + u * TPF];
    group_sync<TPF>();
  }
  // the inverse transform uses the conjugate twiddles of the same table
  Fi::template run_tw<false, HALF>(acc, j, buf, *reinterpret_cast<const typename Fi::Tw *>(&twr));
  if (ok) {
    cplx<T> *dst = outp + ((vec * LG + g) * HC + kx) * (int64_t)lds;
#pragma unroll
    for (int u = 0; u < (HALF ? 4 : 8); ++u) {
      const int y = j + u * TPF - pyl;
      if (y >= 0 && y < sy) dst[y] = acc[u];
    }
  }
}

// HALF: the model rows (y < ny) and the kept station rows (pyl .. pyl + sy - 1) lie in the
// first half of the embedding, so the forward transforms skip the zero half of their input and
// the inverse one the discarded half of its output (same results for the values kept).
template <typename T, int NY, bool HALF, int FP = 0>
__global__ void __launch_bounds__((ColCfg<T, NY>::THREADS * ColCfg<T, NY>::WPB))
k_col_G(const cplx<T> *__restrict__ X1, int ny, int ldy, int nz, int HC, int LG,
        const cplx<T> *__restrict__ spec, cplx<T> *__restrict__ outp, int sy, int lds, int pyl,
        const cplx<T> *__restrict__ tw) {
  __shared__ cplx<T> sh[ColCfg<T, NY>::WPB * ColCfg<T, NY>::CPB * FFT<T, NY, false>::LDS];
  col_G_body<T, NY, HALF, FP>(sh, blockIdx.x, blockIdx.y, blockIdx.z, X1, ny, ldy, nz, HC, LG, spec, outp, sy, lds, pyl, tw);
}

// Pass 2 of G^T: for each column slot c: D = FFT_y(D1[vec, c, :] placed at rows pyl..pyl+sy-1);
// for each layer r of the group: X1[vec, r, c, q] = IFFT_y(conj(S_r[c, :]) .* D)[q], q < ny
// (slot 0: conj(P_r) .* D + conj(M_r) .* conj(D[-k])).
// Wave group w of a block takes every WPB-th layer of the group and transforms D itself.
// Grid: (ceil(HC/CPB), LG, nvec).
template <typename T, int NY, bool HALF = false, int FP = 0>
__device__ __forceinline__ void
col_GT_body(cplx<T> *__restrict__ sh, int bx, int by, int64_t bz, const cplx<T> *__restrict__ D1, int sy, int ldd, int pyl, int nz, int HC, int LG,
         const cplx<T> *__restrict__ spec, cplx<T> *__restrict__ X1, int ny, int ldy,
         const cplx<T> *__restrict__ tw) {
  using CC = ColCfg<T, NY>;
  using Ff = FFT<T, NY, false, FP>;
  using Fi = FFT<T, NY, true, FP>;
  constexpr int TPF = CC::TPF, WPB = CC::WPB;
  const int w = threadIdx.x / CC::THREADS, lt = threadIdx.x % CC::THREADS;
  const int f = lt / TPF, j = lt % TPF;
  const int kx = bx * CC::CPB + f;
  const bool ok = kx < HC;
  const int kxs = ok ? kx : 0;
  const bool pk = bx == 0;        // block-uniform
  const bool pk0 = pk && f == 0;          // this lane's column is the packed slot 0
  const int64_t SH = HC + 1;
  const int g = by;
  const int64_t vec = bz;
  const int r0 = (int)((int64_t)g * nz / LG), r1 = (int)((int64_t)(g + 1) * nz / LG);
  if (r0 + w >= r1) return;   // no layer for this wave group (never with WPB = 1)
  cplx<T> *buf = sh + (w * CC::CPB + f) * Ff::LDS;
  typename Ff::Tw twr;
  Ff::load_tw(twr, j, tw);
  const cplx<T> *src = D1 + (vec * HC + kxs) * (int64_t)ldd;
  cplx<T> dh[8], sn[8];
  int r = r0 + w;
  {
    const cplx<T> *sp = spec + ((int64_t)r * SH + kxs) * NY;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int y = j + u * TPF - pyl;
      dh[u] = ((!HALF || u < 4) && ok && y >= 0 && y < sy) ? src[y] : mk<T>(0, 0);
      sn[u] = sp[j + u * TPF];
    }
  }
  Ff::template run_tw<HALF, false>(dh, j, buf, twr);
  auto store = [&](int r, const cplx<T> *v) {
    if (ok) {
      cplx<T> *dst = X1 + ((vec * nz + r) * HC + kx) * (int64_t)ldy;
#pragma unroll
      for (int u = 0; u < (HALF ? 4 : 8); ++u) {
        const int y = j + u * TPF;
        if (y < ny) dst[y] = v[u];
      }
    }
  };
  if (!pk) {
    for (; r < r1; r += WPB) {
      cplx<T> v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = cmulc<T>(dh[u], sn[u]);
      if (r + WPB < r1) {
        const cplx<T> *sp = spec + ((int64_t)(r + WPB) * SH + kxs) * NY;
#pragma unroll
        for (int u = 0; u < 8; ++u) sn[u] = sp[j + u * TPF];
      }
      Fi::template run_tw<false, HALF>(v, j, buf, *reinterpret_cast<const typename Fi::Tw *>(&twr));
      store(r, v);
    }
  } else {
    // dr[k] = conj(D[-k]) for the packed slot 0
    cplx<T> dr[8];
    group_sync<TPF>();
#pragma unroll
    for (int u = 0; u < 8; ++u) buf[pad8(j + u * TPF)] = dh[u];
    group_sync<TPF>();
#pragma unroll
    for (int u = 0; u < 8; ++u) dr[u] = cconj<T>(buf[pad8((NY - j - u * TPF) & (NY - 1))]);
    group_sync<TPF>();
    // M_r is prefetched with S_r in single precision, loaded at use in double (registers)
    constexpr bool PREFETCH = sizeof(T) == 4;
    cplx<T> mn[8];
    auto loadm = [&](int rr) {
      const cplx<T> *mp = spec + ((int64_t)rr * SH + HC) * NY;
#pragma unroll
      for (int u = 0; u < 8; ++u) mn[u] = mp[j + u * TPF];
    };
    if (PREFETCH) loadm(r);
    for (; r < r1; r += WPB) {
      cplx<T> v[8];
      if (!PREFETCH) loadm(r);
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = cmulc<T>(dh[u], sn[u]);
      if (pk0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = cadd<T>(v[u], cmulc<T>(dr[u], mn[u]));
      }
      if (r + WPB < r1) {
        const cplx<T> *sp = spec + ((int64_t)(r + WPB) * SH + kxs) * NY;
#pragma unroll
        for (int u = 0; u < 8; ++u) sn[u] = sp[j + u * TPF];
        if (PREFETCH) loadm(r + WPB);
      }
      Fi::template run_tw<false, HALF>(v, j, buf, *reinterpret_cast<const typename Fi::Tw *>(&twr));
      store(r, v);
    }
  }
}

template <typename T, int NY, bool HALF, int FP = 0>
__global__ void __launch_bounds__((ColCfg<T, NY>::THREADS * ColCfg<T, NY>::WPB))
k_col_GT(const cplx<T> *__restrict__ D1, int sy, int ldd, int pyl, int nz, int HC, int LG,
         const cplx<T> *__restrict__ spec, cplx<T> *__restrict__ X1, int ny, int ldy,
         const cplx<T> *__restrict__ tw) {
  __shared__ cplx<T> sh[ColCfg<T, NY>::WPB * ColCfg<T, NY>::CPB * FFT<T, NY, false>::LDS];
  col_GT_body<T, NY, HALF, FP>(sh, blockIdx.x, blockIdx.y, blockIdx.z, D1, sy, ldd, pyl, nz, HC, LG, spec, X1, ny, ldy, tw);
}

// Pass 2 of an independent pair G x, G^T d of one survey, in one launch: per column slot the
// work of col_G_body and of col_GT_body, with each layer spectrum column read once for both
// products.  D^ = FFT_y(D), the transform of G^T's data column, is computed once per block by
// wave group WD and shared through LDS.  Wave group w then takes the layers L_i = r0 + w + i WPB
// of layer group `by`; per layer it transforms the model column, adds S_r .* FFT_y(x_r) to the
// G sum and stores IFFT_y(conj(S_r) .* D^) as G^T's layer r, the two transforms interleaved
// (fft_dual), while the next layer's columns (and, in the block of the packed slot 0, the
// M_r column) are loaded.  After the wave groups' G sums are added up, wave group WI inverts
// the sum.  Each transform, product and sum is the one col_G_body / col_GT_body computes, in
// the same order, so both results are bit for bit those of the separate passes.  HALF: the
// model and data rows sit in the first half of the embedding (ny <= NY/2 and pyl + sy <= NY/2,
// which the smallest embedding of an unpadded survey always gives), so the forward transforms
// skip the zero half of their input and the inverse ones the half of their output that is
// discarded.
// NY <= 512 (wave-level transforms).  Grid: (ceil(HC/CPB), LG).
template <typename T, int NY> struct PairCfg {
  using CC = ColCfg<T, NY>;
  static constexpr int LDSF = FFT<T, NY, false>::LDS;
  static constexpr int PER_W = 2 * CC::CPB * LDSF;          // exchange buffers per wave group
  static constexpr int SH = CC::WPB * PER_W + CC::CPB * NY;  // + the shared D^ of the columns
  static constexpr int WD = CC::WPB >= 4 ? CC::WPB - 3 : CC::WPB - 1;   // computes D^
  static constexpr int WI = CC::WPB >= 2 ? CC::WPB - 2 : 0;             // inverts the G sum
};

template <typename T, int NY, bool HALF, int FP = 0>
__device__ __forceinline__ void
col_pair_body(cplx<T> *__restrict__ sh, int bx, int by, const cplx<T> *__restrict__ X1, int ny, int ldy,
              cplx<T> *__restrict__ outp, const cplx<T> *__restrict__ D1, cplx<T> *__restrict__ X1t, int sy,
              int lds, int pyl, int nz, int HC, int LG, const cplx<T> *__restrict__ spec,
              const cplx<T> *__restrict__ tw) {
  using CC = ColCfg<T, NY>;
  using PC = PairCfg<T, NY>;
  using Ff = FFT<T, NY, false, FP>;
  using Fi = FFT<T, NY, true, FP>;
  constexpr int TPF = CC::TPF, WPB = CC::WPB, LDSF = PC::LDSF, WD = PC::WD, WI = PC::WI;
  constexpr int UH = HALF ? 4 : 8;   // register slots of a half-pruned transform's input / output
  static_assert(TPF <= 64, "pair column pass: wave-level transforms only");
  const int w = threadIdx.x / CC::THREADS, lt = threadIdx.x % CC::THREADS;
  const int f = lt / TPF, j = lt % TPF;
  const int kx = bx * CC::CPB + f;
  const bool ok = kx < HC;
  const int kxs = ok ? kx : 0;
  const bool pk = bx == 0;            // block-uniform: slot 0 sits at f == 0 of block 0
  const bool pk0 = pk && f == 0;
  const int64_t SH = HC + 1;
  const int g = by;
  const int r0 = (int)((int64_t)g * nz / LG), r1 = (int)((int64_t)(g + 1) * nz / LG);
  const int nl = r0 + w < r1 ? (r1 - r0 - w + WPB - 1) / WPB : 0;   // this wave group's layers
  cplx<T> *wbase = sh + w * PC::PER_W;
  cplx<T> *bufA = wbase + f * LDSF;                        // exchange buffers of this column
  cplx<T> *bufB = wbase + (CC::CPB + f) * LDSF;
  cplx<T> *dsh = sh + WPB * PC::PER_W + f * NY;             // D^ of this column, shared
  typename Ff::Tw twr;
  Ff::load_tw(twr, j, tw);
  cplx<T> acc[8], accm[8], dh[8], xn[8], sn[8], mn[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    acc[u] = mk<T>(0, 0);
    accm[u] = mk<T>(0, 0);
    xn[u] = mk<T>(0, 0);
  }
  auto layer = [&](int i) { return r0 + w + i * WPB; };
  auto load = [&](int rr) {
    const cplx<T> *src = X1 + ((int64_t)rr * HC + kxs) * (int64_t)ldy;
    const cplx<T> *sp = spec + ((int64_t)rr * SH + kxs) * NY;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int y = j + u * TPF;
      if (u < UH) xn[u] = (ok && y < ny) ? src[y] : mk<T>(0, 0);
      sn[u] = sp[y];
    }
    if (pk) {
      const cplx<T> *mp = spec + ((int64_t)rr * SH + HC) * NY;
#pragma unroll
      for (int u = 0; u < 8; ++u) mn[u] = mp[j + u * TPF];
    }
  };
  if (nl > 0) load(layer(0));
  if (w == WD) {
    // the data column of G^T, embedded at rows pyl .. pyl + sy - 1, and its transform, for all
    const cplx<T> *src = D1 + (int64_t)kxs * lds;
    cplx<T> d[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int y = j + u * TPF - pyl;
      d[u] = (u < UH && ok && y >= 0 && y < sy) ? src[y] : mk<T>(0, 0);
    }
    Ff::template run_tw<HALF, false>(d, j, bufB, twr);
#pragma unroll
    for (int u = 0; u < 8; ++u) dsh[j + u * TPF] = d[u];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 8; ++u) dh[u] = dsh[j + u * TPF];
  for (int i = 0; i < nl; ++i) {
    const int rr = layer(i);
    cplx<T> a[8], b[8], sc[8], mc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = xn[u];
      sc[u] = sn[u];
      mc[u] = mn[u];
      b[u] = cmulc<T>(dh[u], sn[u]);     // G^T: conj(S_r) .* D^
    }
    if (pk0) {
      // + conj(M_r) .* conj(D^[-k]) in the packed slot
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const cplx<T> dr = cconj<T>(dsh[(NY - j - u * TPF) & (NY - 1)]);
        b[u] = cadd<T>(b[u], cmulc<T>(dr, mn[u]));
      }
    }
    if (i + 1 < nl) load(layer(i + 1));
    fft_dual<T, NY, false, true, HALF, false, false, HALF, FP>(a, b, j, bufA, bufB, twr);
    // G: the layer sums of S_r .* X and (packed slot) M_r .* X
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = cadd<T>(acc[u], cmul<T>(a[u], sc[u]));
    if (pk) {
#pragma unroll
      for (int u = 0; u < 8; ++u) accm[u] = cadd<T>(accm[u], cmul<T>(a[u], mc[u]));
    }
    if (ok) {
      cplx<T> *dst = X1t + ((int64_t)rr * HC + kx) * (int64_t)ldy;
#pragma unroll
      for (int u = 0; u < UH; ++u) {
        const int y = j + u * TPF;
        if (y < ny) dst[y] = b[u];
      }
    }
  }
  if (pk) {
    // each wave group folds its own M sum into its G sum: acc[k] += conj(accm[-k]) (slot 0)
    group_sync<TPF>();
#pragma unroll
    for (int u = 0; u < 8; ++u) bufA[pad8(j + u * TPF)] = accm[u];
    group_sync<TPF>();
    if (f == 0) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = cadd<T>(acc[u], cconj<T>(bufA[pad8((NY - j - u * TPF) & (NY - 1))]));
    }
  }
  if constexpr (WPB > 1) {
    // the wave groups' G sums meet in LDS (buffer A of each), added in wave-group order; the
    // sums end in wave group 0's buffer A
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) bufA[j + u * TPF] = acc[u];
    __syncthreads();
    for (int u = w; u < 8; u += WPB) {
      const int e = f * LDSF + j + u * TPF;
      cplx<T> t = sh[e];
      for (int w2 = 1; w2 < WPB; ++w2) t = cadd<T>(t, sh[w2 * PC::PER_W + e]);
      sh[e] = t;
    }
    __syncthreads();
    if (w != WI) return;
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = sh[f * LDSF + j + u * TPF];
    group_sync<TPF>();
  }
  Fi::template run_tw<false, HALF>(acc, j, bufA, *reinterpret_cast<const typename Fi::Tw *>(&twr));
  if (ok) {
    cplx<T> *dst = outp + ((int64_t)g * HC + kx) * (int64_t)lds;
#pragma unroll
    for (int u = 0; u < UH; ++u) {
      const int y = j + u * TPF - pyl;
      if (y >= 0 && y < sy) dst[y] = acc[u];
    }
  }
}

// ---------------------------------------------------------------------------------------
// Batched column passes (single precision, NY <= 512): V = 4 vectors per block.  The block's
// WPB wave groups form GL = WPB/2 layer groups times 2 vector pairs: wave group w takes the
// vectors 2p, 2p+1 (p = w mod 2) and the layers r0 + l, r0 + l + GL, ... (l = w / 2), so every
// wave group does the same number of transforms (the layer split alone leaves some wave groups
// with one layer more than others).  A spectrum column is loaded once per wave group for two
// vectors.  Results agree with the single-vector kernels to rounding (the layer sums are taken
// in another order).
template <typename T, int NY> struct BatchCfg {
  static constexpr int V = 4;                    // vectors per block
  static constexpr int GV = 2;                   // vectors per wave group
  static constexpr int GL = ColCfg<T, NY>::WPB / 2;   // layer groups
  static constexpr bool OK = std::is_same<T, float>::value && ColCfg<T, NY>::TPF <= 64 &&
                             ColCfg<T, NY>::WPB >= 4 && ColCfg<T, NY>::WPB % 2 == 0;
};

// Pass 2 of G for vectors vec0 .. vec0+3 (vec0 = 4 blockIdx.z; vectors >= kb are skipped).
// The partial sums of vector 2p + i sit in the wave groups 2l + p (l < GL); wave group 2i + p
// adds them up in layer-group order and does the vector's inverse transform.  Block 0 (slot 0
// at f == 0) also sums the M_r products and folds them in per wave group before the reduction.
template <typename T, int NY, bool HALF, int FP = 0>
__global__ void __launch_bounds__((ColCfg<T, NY>::THREADS * ColCfg<T, NY>::WPB))
k_col_G_batch(const cplx<T> *__restrict__ X1, int ny, int ldy, int nz, int HC, int LG, int kb,
              const cplx<T> *__restrict__ spec, cplx<T> *__restrict__ outp, int sy, int lds, int pyl,
              const cplx<T> *__restrict__ tw) {
  using CC = ColCfg<T, NY>;
  using BC = BatchCfg<T, NY>;
  using Ff = FFT<T, NY, false, FP>;
  using Fi = FFT<T, NY, true, FP>;
  constexpr int TPF = CC::TPF, GL = BC::GL;
  static_assert(BC::OK, "batched column pass configuration");
  __shared__ cplx<T> sh[CC::WPB * CC::CPB * Ff::LDS];
  const int w = threadIdx.x / CC::THREADS, lt = threadIdx.x % CC::THREADS;
  const int f = lt / TPF, j = lt % TPF;
  const int p = w % 2, lgw = w / 2;
  const int kx = blockIdx.x * CC::CPB + f;
  const bool ok = kx < HC;
  const int kxs = ok ? kx : 0;
  const bool pk = blockIdx.x == 0;   // block-uniform
  const int64_t SH = HC + 1;
  const int g = blockIdx.y;
  const int64_t vec0 = (int64_t)blockIdx.z * BC::V;
  const int r0 = (int)((int64_t)g * nz / LG), r1 = (int)((int64_t)(g + 1) * nz / LG);
  cplx<T> *buf = sh + (w * CC::CPB + f) * Ff::LDS;
  typename Ff::Tw twr;
  Ff::load_tw(twr, j, tw);
  cplx<T> acc[2][8], accm[2][8];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      acc[i][u] = mk<T>(0, 0);
      accm[i][u] = mk<T>(0, 0);
    }
  for (int r = r0 + lgw; r < r1; r += GL) {
    cplx<T> sv[8], mv[8];
    const cplx<T> *sp = spec + ((int64_t)r * SH + kxs) * NY;
#pragma unroll
    for (int u = 0; u < 8; ++u) sv[u] = sp[j + u * TPF];
    if (pk) {
      const cplx<T> *mp = spec + ((int64_t)r * SH + HC) * NY;
#pragma unroll
      for (int u = 0; u < 8; ++u) mv[u] = mp[j + u * TPF];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int64_t vec = vec0 + 2 * p + i;
      const bool okv = ok && vec < kb;
      const cplx<T> *src = X1 + ((vec * nz + r) * HC + kxs) * (int64_t)ldy;
      cplx<T> xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int y = j + u * TPF;
        xv[u] = ((!HALF || u < 4) && okv && y < ny) ? src[y] : mk<T>(0, 0);
      }
      Ff::template run_tw<HALF, false>(xv, j, buf, twr);
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[i][u] = cadd<T>(acc[i][u], cmul<T>(xv[u], sv[u]));
      if (pk) {
#pragma unroll
        for (int u = 0; u < 8; ++u) accm[i][u] = cadd<T>(accm[i][u], cmul<T>(xv[u], mv[u]));
      }
    }
  }
  if (pk) {
    // slot 0: acc[k] += conj(accm[-k]), per wave group and vector
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      group_sync<TPF>();
#pragma unroll
      for (int u = 0; u < 8; ++u) buf[pad8(j + u * TPF)] = accm[i][u];
      group_sync<TPF>();
      if (f == 0) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
          acc[i][u] = cadd<T>(acc[i][u], cconj<T>(buf[pad8((NY - j - u * TPF) & (NY - 1))]));
      }
    }
  }
  // two rounds: in round i the wave groups 2i and 2i + 1 collect the vectors 2p + i
  cplx<T> mine[8];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) buf[j + u * TPF] = acc[i][u];
    __syncthreads();
    if (lgw == i) {
#pragma unroll
      for (int u = 0; u < 8; ++u) mine[u] = sh[(p * CC::CPB + f) * Ff::LDS + j + u * TPF];
      for (int l = 1; l < GL; ++l) {
        const cplx<T> *o = sh + ((2 * l + p) * CC::CPB + f) * Ff::LDS;
#pragma unroll
        for (int u = 0; u < 8; ++u) mine[u] = cadd<T>(mine[u], o[j + u * TPF]);
      }
    }
  }
  __syncthreads();
  const int64_t vo = vec0 + 2 * p + lgw;   // the vector this wave group finishes (lgw < 2)
  if (lgw >= 2 || vo >= kb) return;
  Fi::template run_tw<false, HALF>(mine, j, buf, *reinterpret_cast<const typename Fi::Tw *>(&twr));
  if (ok) {
    cplx<T> *dst = outp + ((vo * LG + g) * HC + kx) * (int64_t)lds;
#pragma unroll
    for (int u = 0; u < (HALF ? 4 : 8); ++u) {
      const int y = j + u * TPF - pyl;
      if (y >= 0 && y < sy) dst[y] = mine[u];
    }
  }
}

// Pass 2 of G^T for vectors vec0 .. vec0+3: wave group v < 4 transforms vector v's data column
// into LDS; then wave group w takes the vectors 2p, 2p+1 and the layers r0 + l + k GL as above,
// loading each spectrum column once for its two products and inverse transforms.  Slot 0
// reads the reversed transform conj(D[-k]) from the same LDS copy.
template <typename T, int NY, bool HALF, int FP = 0>
__global__ void __launch_bounds__((ColCfg<T, NY>::THREADS * ColCfg<T, NY>::WPB))
k_col_GT_batch(const cplx<T> *__restrict__ D1, int sy, int ldd, int pyl, int nz, int HC, int LG, int kb,
               const cplx<T> *__restrict__ spec, cplx<T> *__restrict__ X1, int ny, int ldy,
               const cplx<T> *__restrict__ tw) {
  using CC = ColCfg<T, NY>;
  using BC = BatchCfg<T, NY>;
  using Ff = FFT<T, NY, false, FP>;
  using Fi = FFT<T, NY, true, FP>;
  constexpr int TPF = CC::TPF, GL = BC::GL;
  static_assert(BC::OK, "batched column pass configuration");
  __shared__ cplx<T> sh[CC::WPB * CC::CPB * Ff::LDS];
  __shared__ cplx<T> dsh[BC::V * CC::CPB * NY];
  const int w = threadIdx.x / CC::THREADS, lt = threadIdx.x % CC::THREADS;
  const int f = lt / TPF, j = lt % TPF;
  const int p = w % 2, lgw = w / 2;
  const int kx = blockIdx.x * CC::CPB + f;
  const bool ok = kx < HC;
  const int kxs = ok ? kx : 0;
  const bool pk = blockIdx.x == 0;   // block-uniform
  const bool pk0 = pk && f == 0;
  const int64_t SH = HC + 1;
  const int g = blockIdx.y;
  const int64_t vec0 = (int64_t)blockIdx.z * BC::V;
  const int r0 = (int)((int64_t)g * nz / LG), r1 = (int)((int64_t)(g + 1) * nz / LG);
  cplx<T> *buf = sh + (w * CC::CPB + f) * Ff::LDS;
  typename Ff::Tw twr;
  Ff::load_tw(twr, j, tw);
  if (w < BC::V) {
    const bool okv = ok && vec0 + w < kb;
    const cplx<T> *src = D1 + ((vec0 + w) * HC + kxs) * (int64_t)ldd;
    cplx<T> dv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int y = j + u * TPF - pyl;
      dv[u] = ((!HALF || u < 4) && okv && y >= 0 && y < sy) ? src[y] : mk<T>(0, 0);
    }
    Ff::template run_tw<HALF, false>(dv, j, buf, twr);
#pragma unroll
    for (int u = 0; u < 8; ++u) dsh[(w * CC::CPB + f) * NY + j + u * TPF] = dv[u];
  }
  __syncthreads();
  cplx<T> dh[2][8];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int u = 0; u < 8; ++u) dh[i][u] = dsh[((2 * p + i) * CC::CPB + f) * NY + j + u * TPF];
  for (int r = r0 + lgw; r < r1; r += GL) {
    cplx<T> sv[8], mv[8];
    const cplx<T> *sp = spec + ((int64_t)r * SH + kxs) * NY;
#pragma unroll
    for (int u = 0; u < 8; ++u) sv[u] = sp[j + u * TPF];
    if (pk) {
      const cplx<T> *mp = spec + ((int64_t)r * SH + HC) * NY;
#pragma unroll
      for (int u = 0; u < 8; ++u) mv[u] = mp[j + u * TPF];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int64_t vec = vec0 + 2 * p + i;
      cplx<T> xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = cmulc<T>(dh[i][u], sv[u]);
      if (pk0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const cplx<T> dr = cconj<T>(dsh[((2 * p + i) * CC::CPB + f) * NY + ((NY - j - u * TPF) & (NY - 1))]);
          xv[u] = cadd<T>(xv[u], cmulc<T>(dr, mv[u]));
        }
      }
      Fi::template run_tw<false, HALF>(xv, j, buf, *reinterpret_cast<const typename Fi::Tw *>(&twr));
      if (ok && vec < kb) {
        cplx<T> *dst = X1 + ((vec * nz + r) * HC + kx) * (int64_t)ldy;
#pragma unroll
        for (int u = 0; u < (HALF ? 4 : 8); ++u) {
          const int y = j + u * TPF;
          if (y < ny) dst[y] = xv[u];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// Vector-parallel column pass of G for block products (single precision, NY <= 512): a block
// takes CPB column slots and VV = 8 vectors, one vector per wave group, and every wave group
// runs its vector's whole column chain on its own (every layer's forward transform and
// product, the layer sum and the inverse), the next layer's column loaded while the current
// one is transformed.  The wave groups of a block wait for each other only while the block
// stages the layer spectra of its columns in LDS, LC layers at a time: each spectrum column is
// read from memory once per 8 vectors (the 4-vector pass reads it once per 2).  The layers are
// summed in order, so the result agrees with the single-vector pass to rounding.  (The same
// structure for G^T, one forward and nz inverse transforms per vector, was no faster than the
// 4-vector pass.)
template <typename T, int NY> struct VecCfg {
  using CC = ColCfg<T, NY>;
  static constexpr int VV = 8;                       // vectors (wave groups) per block
  static constexpr int THREADS = VV * CC::THREADS;   // 512
  static constexpr int LC = 8;                       // layers of spectra staged per round
  static constexpr int SPL = CC::CPB * NY;           // spectrum elements per layer (512)
  static constexpr int XL = CC::CPB * FFT<T, NY, false>::LDS;   // exchange elements per wave group
  static constexpr int SH = VV * XL + LC * SPL;
  static constexpr bool OK = std::is_same<T, float>::value && CC::TPF <= 64 && CC::THREADS == 64;
};

// stages the spectra of layers r0 .. r0 + lc - 1 of the block's CPB columns (kx0 ..) in LDS:
// dst[l * SPL + f * NY + y]; columns past HC read column HC - 1 (their results are not stored)
template <typename T, int NY>
__device__ __forceinline__ void stage_spectra(cplx<T> *__restrict__ dst, const cplx<T> *__restrict__ spec, int r0,
                                              int lc, int kx0, int HC) {
  using VC = VecCfg<T, NY>;
  const int64_t SH = HC + 1;
  for (int e = threadIdx.x; e < lc * VC::SPL; e += VC::THREADS) {
    const int l = e / VC::SPL, w = e - l * VC::SPL, fc = w / NY, y = w - fc * NY;
    const int kx = min(kx0 + fc, HC - 1);
    dst[e] = spec[((int64_t)(r0 + l) * SH + kx) * NY + y];
  }
}

// Pass 2 of G for vectors 8 blockIdx.y + w: out[vec, 0, c, j] (the single layer-group partial).
template <typename T, int NY, bool HALF, int FP = 0>
__global__ void __launch_bounds__((VecCfg<T, NY>::THREADS))
k_col_G_vec(const cplx<T> *__restrict__ X1, int ny, int ldy, int nz, int HC, int kb, int64_t vstride,
            const cplx<T> *__restrict__ spec, cplx<T> *__restrict__ outp, int64_t ostride, int sy, int lds, int pyl,
            const cplx<T> *__restrict__ tw) {
  using CC = ColCfg<T, NY>;
  using VC = VecCfg<T, NY>;
  using Ff = FFT<T, NY, false, FP>;
  using Fi = FFT<T, NY, true, FP>;
  constexpr int TPF = CC::TPF, UH = HALF ? 4 : 8;
  static_assert(VC::OK, "vector-parallel column pass configuration");
  __shared__ cplx<T> sh[VC::SH];
  const int w = threadIdx.x / CC::THREADS, lt = threadIdx.x % CC::THREADS;
  const int f = lt / TPF, j = lt % TPF;
  const int kx0 = blockIdx.x * CC::CPB, kx = kx0 + f;
  const bool ok = kx < HC;
  const int kxs = ok ? kx : 0;
  const bool pk = blockIdx.x == 0;   // block-uniform: slot 0 sits at f == 0 of block 0
  const int64_t vec = (int64_t)blockIdx.y * VC::VV + w;
  const bool live = vec < kb;         // wave-uniform
  const int64_t SH = HC + 1;
  cplx<T> *buf = sh + w * VC::XL + f * Fi::LDS;
  cplx<T> *sp = sh + VC::VV * VC::XL;
  typename Ff::Tw twr;
  Ff::load_tw(twr, j, tw);
  cplx<T> acc[8], accm[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    acc[u] = mk<T>(0, 0);
    accm[u] = mk<T>(0, 0);
  }
  const cplx<T> *src = X1 + vec * vstride + (int64_t)kxs * ldy;
  cplx<T> xn[UH];   // the next layer's column, loaded while the current one is transformed
  auto load = [&](int rr) {
    const cplx<T> *xr = src + (int64_t)rr * HC * ldy;
#pragma unroll
    for (int u = 0; u < UH; ++u) {
      const int y = j + u * TPF;
      xn[u] = (ok && y < ny) ? xr[y] : mk<T>(0, 0);
    }
  };
  if (live) load(0);
  for (int r0 = 0; r0 < nz; r0 += VC::LC) {
    const int lc = min(VC::LC, nz - r0);
    __syncthreads();   // the previous round's spectra are no longer read
    stage_spectra<T, NY>(sp, spec, r0, lc, kx0, HC);
    __syncthreads();
    if (live) {
      for (int l = 0; l < lc; ++l) {
        const int rr = r0 + l;
        cplx<T> v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = u < UH ? xn[u] : mk<T>(0, 0);
        if (rr + 1 < nz) load(rr + 1);
        Ff::template run_tw<HALF, false>(v, j, buf, twr);
        const cplx<T> *s = sp + l * VC::SPL + f * NY;
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = cadd<T>(acc[u], cmul<T>(v[u], s[j + u * TPF]));
        if (pk) {
          const cplx<T> *mp = spec + ((int64_t)rr * SH + HC) * NY;
#pragma unroll
          for (int u = 0; u < 8; ++u) accm[u] = cadd<T>(accm[u], cmul<T>(v[u], mp[j + u * TPF]));
        }
      }
    }
  }
  if (!live) return;
  if (pk) {
    // acc[k] += conj(accm[-k]) in the packed slot (f == 0)
    group_sync<TPF>();
#pragma unroll
    for (int u = 0; u < 8; ++u) buf[pad8(j + u * TPF)] = accm[u];
    group_sync<TPF>();
    if (f == 0) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = cadd<T>(acc[u], cconj<T>(buf[pad8((NY - j - u * TPF) & (NY - 1))]));
    }
    group_sync<TPF>();
  }
  Fi::template run_tw<false, HALF>(acc, j, buf, *reinterpret_cast<const typename Fi::Tw *>(&twr));
  if (ok) {
    cplx<T> *dst = outp + vec * ostride + (int64_t)kx * lds;
#pragma unroll
    for (int u = 0; u < UH; ++u) {
      const int y = j + u * TPF - pyl;
      if (y >= 0 && y < sy) dst[y] = acc[u];
    }
  }
}

}  // namespace ff

// Projected solvers of the normal equations (Algorithms 1 and 2, Sec. 2.4 of the paper) and the IRLS
// step (Secs. 2.2-2.3).
//
//  gkb_project  -- Algorithm 1: Golub-Kahan bidiagonalization of G~ = diag(wd) G diag(winv)
//                  with reorthogonalization of both bases in FP64, SVD of the bidiagonal B,
//                  regularization parameter from the truncated UPRE (or eq. (eq:alpha1), or
//                  fixed), y = ||r~|| A V Gamma(alpha, Sigma) U(1,:)^T.
//  rsvd_project -- Algorithm 2: randomized SVD with one power iteration; block operator
//                  applications, economic QRs, eigen-decomposition of the symmetrized B^T B.
//  irls_step    -- one focusing IRLS step (Secs. 2.2-2.3).
//
// Operator applications run in the handle's precision with FP64 vectors; every other step is
// FP64 on the device.  The bases are reorthogonalized by classical Gram-Schmidt applied twice
// (same subspace as the paper's modified Gram-Schmidt in exact arithmetic, at least as
// orthogonal in floating point, and two streaming passes over the basis instead of one
// dependent pass per column).  The small dense factorizations use rocSOLVER, the B^T B product
// rocBLAS.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <map>
#include <mutex>

#include "common.h"

namespace ff {
namespace {

constexpr int kThreads = 256;
constexpr int kTLoads = 4;                 // row loads per lane in the transposed products
constexpr int kTCols = 16;                 // basis columns per block of the transposed products
constexpr int kRowsMin = 64 * kTLoads;     // rows per transposed-product block at one row per load
constexpr int kNWaves = 8;                 // waves per block of the basis products A c
constexpr int kMaxPowerIters = 8;          // largest RSVD power-iteration count accepted
constexpr int kNormBlocks = 256;           // blocks (partial sums) of the norm reductions
constexpr int kUpreGrid = 400;
constexpr double kUpreLo = 1e-3;
constexpr double kGoldenTol = 1e-10;

// ---------------------------------------------------------------------------------------
// FP64 reductions and vector kernels

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum; result valid in thread 0
__device__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
  }
  __syncthreads();
  return s;
}

__global__ void k_sumsq_partial(const double *__restrict__ x, int64_t n, double *__restrict__ part) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += x[i] * x[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// nrm = sqrt(sum of partials); inv = 1/nrm (0 for a zero vector: the Krylov space is exhausted)
__global__ void k_norm_finalize(const double *__restrict__ part, int P, double *nrm, double *inv) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < P; i += blockDim.x) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    const double v = sqrt(s);
    *nrm = v;
    if (inv) *inv = v > 0.0 ? 1.0 / v : 0.0;
  }
}

__global__ void k_scale(const double *__restrict__ x, const double *__restrict__ sc, double *__restrict__ y, int64_t n) {
  const double a = *sc;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

// Basis storage of the GKB factors: FP64 (default) or FP32 (half the memory and traffic; the
// arithmetic stays FP64).  load_rows reads RPL consecutive rows of a basis column with one
// vector load (16 bytes: RPL = 2 for double, 4 for float) and widens them to double.  The bases
// are streamed once per pass, so the loads carry the non-temporal hint.
template <typename TB, int RPL> __device__ __forceinline__ void load_rows(const TB *p, double (&o)[RPL]) {
  if constexpr (RPL == 1) {
    o[0] = (double)__builtin_nontemporal_load(p);
  } else {
    typedef TB V __attribute__((ext_vector_type(RPL)));
    const V v = __builtin_nontemporal_load((const V *)p);
#pragma unroll
    for (int q = 0; q < RPL; ++q) o[q] = (double)v[q];
  }
}

// y += sign * (*sc) * x, and the block's partial sum of the updated y^2 in part[blockIdx.x]
// (grid-stride; launched with a fixed grid of kNormBlocks blocks)
template <typename TX>
__global__ void k_axpy_sumsq(double *__restrict__ y, const TX *__restrict__ x, const double *__restrict__ sc,
                             double sign, int64_t n, double *__restrict__ part) {
  __shared__ double red[16];
  const double a = sign * (*sc);
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = y[i] + a * (double)x[i];
    y[i] = v;
    s += v * v;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// b <- (TB)(b * (*sc)) rounded back to double, also stored as a basis column: the operator
// is then applied to exactly the vector the basis holds.
template <typename TB>
__global__ void k_scale_store(double *__restrict__ b, const double *__restrict__ sc, TB *__restrict__ col, int64_t n) {
  const double a = *sc;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const TB t = (TB)(a * b[i]);
    col[i] = t;
    b[i] = (double)t;
  }
}

// k_norm_cond fused into k_scale_store: when the second Gram-Schmidt pass ran (*flag), or
// always when flag is NULL, every block forms the norm from the P partial sums (the order of
// k_norm_cond and k_norm_finalize) and block 0 writes *nrm and *inv; otherwise the blocks take
// *inv as k_norm_flag left it.  Then as k_scale_store with that inverse norm.
template <typename TB>
__global__ void __launch_bounds__(kThreads)
k_scale_store_cond(double *__restrict__ b, TB *__restrict__ col, int64_t n, const double *__restrict__ part, int P,
                   const int *__restrict__ flag, double *__restrict__ nrm, double *__restrict__ inv) {
  __shared__ double red[16];
  __shared__ double a_sh;
  if (!flag || *flag) {
    double s = 0.0;
    for (int i = threadIdx.x; i < P; i += blockDim.x) s += part[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
      const double v = sqrt(s);
      const double a = v > 0.0 ? 1.0 / v : 0.0;
      a_sh = a;
      if (blockIdx.x == 0) {
        *nrm = v;
        *inv = a;
      }
    }
  } else if (threadIdx.x == 0) {
    a_sh = *inv;
  }
  __syncthreads();
  const double a = a_sh;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const TB t = (TB)(a * b[i]);
    col[i] = t;
    b[i] = (double)t;
  }
}

// out = (*sc) * x with x given in double, stored as TB and (rounded) as double
template <typename TB>
__global__ void k_scale_from(const double *__restrict__ x, const double *__restrict__ sc, TB *__restrict__ col,
                             double *__restrict__ dbl, int64_t n) {
  const double a = *sc;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const TB t = (TB)(a * x[i]);
    col[i] = t;
    dbl[i] = (double)t;
  }
}

// dbl = (double) col
template <typename TB>
__global__ void k_widen(const TB *__restrict__ col, double *__restrict__ dbl, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dbl[i] = (double)col[i];
}

// y = (*sc) * x
template <typename TB>
__global__ void k_scaled(const TB *__restrict__ x, const double *__restrict__ sc, double *__restrict__ y, int64_t n) {
  const double a = *sc;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * (double)x[i];
}

// After the first Gram-Schmidt pass: n0 = ||v0|| (before the pass) and n1 = ||v1|| (after it)
// from their partial sums of squares, the second-pass test flag = n1 < n0 / sqrt 2
// (Daniel-Gragg-Kaufman-Stewart), and the norm and its inverse as they stand if the second
// pass is skipped.
__global__ void k_norm_flag(const double *__restrict__ part0, int P0, const double *__restrict__ part1, int P1,
                            int *__restrict__ flag, double *__restrict__ nrm, double *__restrict__ inv) {
  __shared__ double red[16];
  double s0 = 0.0, s1 = 0.0;
  for (int i = threadIdx.x; i < P0; i += blockDim.x) s0 += part0[i];
  for (int i = threadIdx.x; i < P1; i += blockDim.x) s1 += part1[i];
  s0 = block_sum(s0, red);
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    const double v = sqrt(s1);
    *flag = (v < 0.70710678118654752 * sqrt(s0)) ? 1 : 0;
    *nrm = v;
    *inv = v > 0.0 ? 1.0 / v : 0.0;
  }
}

// After a second pass that ran (*flag != 0): the norm from the partials of the pass's update.
__global__ void k_norm_cond(const double *__restrict__ part, int P, const int *__restrict__ flag,
                            double *__restrict__ nrm, double *__restrict__ inv) {
  if (*flag == 0) return;
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < P; i += blockDim.x) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    const double v = sqrt(s);
    *nrm = v;
    *inv = v > 0.0 ? 1.0 / v : 0.0;
  }
}

// Gaussian test matrix from a counter-based generator: Philox4x32-10 (Salmon, Moraes, Dror and
// Shaw, SC 2011).  Pair p of the output (elements 2p, 2p+1) is drawn from the counter
// (p mod 2^32, p / 2^32, stream, 0) under the key (seed mod 2^32, seed / 2^32): two 53-bit
// uniforms u1 in (0, 1], u2 in [0, 1) from the four output words, then Box-Muller:
// sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__global__ void k_gaussian(double *__restrict__ out, int64_t count, uint64_t seed, uint32_t stream) {
  const int64_t npair = (count + 1) / 2;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npair; p += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)p, (uint32_t)((uint64_t)p >> 32), stream, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double a = (double)(((uint64_t)(c[0] >> 5) << 26) | (c[1] >> 6));
    const double b = (double)(((uint64_t)(c[2] >> 5) << 26) | (c[3] >> 6));
    const double u1 = (a + 1.0) * 0x1.0p-53, u2 = b * 0x1.0p-53;
    const double rho = sqrt(-2.0 * log(u1)), th = 6.283185307179586476925 * u2;
    out[2 * p] = rho * cos(th);
    if (2 * p + 1 < count) out[2 * p + 1] = rho * sin(th);
  }
}

// partial[p][j] = sum over the rows of row block p of A[row, j] * x[row]  (A column-major, ld
// lda).  Each lane loads RPL consecutive rows at once (RPL = 2: 16-byte loads), kTLoads times,
// so a block covers kRowsMin * RPL rows and kTCols columns; each of its four waves takes
// kTCols/4 columns (x held in registers).  Grid: (ceil(nrows / (kRowsMin * RPL)), ceil(ncols / kTCols)).
template <int RPL, typename TB>
__global__ void __launch_bounds__(kThreads)
k_gemv_t_partial(const TB *__restrict__ A, int64_t lda, int64_t nrows, int ncols, const double *__restrict__ x,
                 double *__restrict__ part, const int *__restrict__ run) {
  if (run && *run == 0) return;   // conditional pass switched off on the device
  constexpr int K = kTLoads, CW = kTCols / (kThreads / 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t r0 = (int64_t)blockIdx.x * kRowsMin * RPL;
  double xv[K][RPL];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int64_t r = r0 + (int64_t)(l + 64 * k) * RPL + q;
      xv[k][q] = r < nrows ? x[r] : 0.0;
    }
  const int c0 = blockIdx.y * kTCols + w * CW;
  double s[CW];
#pragma unroll
  for (int c = 0; c < CW; ++c) {
    s[c] = 0.0;
    const int j = c0 + c;
    if (j < ncols) {
      const TB *a = A + (int64_t)j * lda;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int64_t r = r0 + (int64_t)(l + 64 * k) * RPL;
        if (r + RPL <= nrows) {
          double e[RPL];
          load_rows<TB, RPL>(a + r, e);
#pragma unroll
          for (int q = 0; q < RPL; ++q) s[c] += e[q] * xv[k][q];
        } else {
#pragma unroll
          for (int q = 0; q < RPL; ++q)
            if (r + q < nrows) s[c] += (double)a[r + q] * xv[k][q];
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CW; ++c) {
    const double t = wave_sum(s[c]);
    if (l == 0 && c0 + c < ncols) part[(int64_t)blockIdx.x * ncols + c0 + c] = t;
  }
}

// out[j] = scale * sum_p part[p][j]: kCSumCols columns per block, the row-block range split over
// the block's kThreads / kCSumCols groups of threads (consecutive threads of a group read
// consecutive columns), then the groups' sums added in LDS in group order.  Narrow blocks and
// short per-thread chains: at a few hundred columns the sums take a few dozen blocks.
constexpr int kCSumCols = 16;
__global__ void __launch_bounds__(kThreads)
k_colsum(const double *__restrict__ part, int P, int ncols, double *__restrict__ out, double scale,
         const int *__restrict__ run) {
  if (run && *run == 0) return;
  __shared__ double red[kThreads];
  constexpr int NG = kThreads / kCSumCols;
  const int c = threadIdx.x % kCSumCols, g = threadIdx.x / kCSumCols;
  const int j = blockIdx.x * kCSumCols + c;
  const int p0 = (int)((int64_t)P * g / NG), p1 = (int)((int64_t)P * (g + 1) / NG);
  double s = 0.0;
  if (j < ncols)
    for (int p = p0; p < p1; ++p) s += part[(int64_t)p * ncols + j];
  red[threadIdx.x] = s;
  __syncthreads();
  if (g == 0 && j < ncols) {
    double t = red[c];
    for (int q = 1; q < NG; ++q) t += red[q * kCSumCols + c];
    out[j] = scale * t;
  }
}

// y = beta * y + alpha * A c   (A column-major nrows x ncols, ld lda).  A block of NW waves
// covers 64 * RPL rows (RPL consecutive rows per lane, 16-byte loads when RPL = 2); wave w takes
// the columns [w ncols / NW, (w + 1) ncols / NW), so that many column loads of a lane are in
// flight; the waves' sums meet in LDS and are added in wave order.
// Grid: ceil(nrows / (64 * RPL)) blocks of 64 * NW threads.
template <int RPL, typename TB, int NW = kNWaves>
__global__ void __launch_bounds__(64 * NW)
k_gemv_n(const TB *__restrict__ A, int64_t lda, int64_t nrows, int ncols, const double *__restrict__ c,
         double *__restrict__ y, double alpha, double beta, const int *__restrict__ run, double *__restrict__ sq) {
  if (run && *run == 0) return;
  __shared__ double red[NW][64 * RPL];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t r = ((int64_t)blockIdx.x * 64 + l) * RPL;
  const int j0 = (int)((int64_t)ncols * w / NW), j1 = (int)((int64_t)ncols * (w + 1) / NW);
  double s[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) s[q] = 0.0;
  if (r + RPL <= nrows) {
    const TB *a = A + r;
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
      double v[4][RPL];
#pragma unroll
      for (int t = 0; t < 4; ++t) load_rows<TB, RPL>(a + (int64_t)(j + t) * lda, v[t]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double cj = c[j + t];
#pragma unroll
        for (int q = 0; q < RPL; ++q) s[q] += v[t][q] * cj;
      }
    }
    for (; j < j1; ++j) {
      const double cj = c[j];
#pragma unroll
      for (int q = 0; q < RPL; ++q) s[q] += (double)a[(int64_t)j * lda + q] * cj;
    }
  } else {
    for (int j = j0; j < j1; ++j) {
      const double cj = c[j];
#pragma unroll
      for (int q = 0; q < RPL; ++q)
        if (r + q < nrows) s[q] += (double)A[(int64_t)j * lda + r + q] * cj;
    }
  }
#pragma unroll
  for (int q = 0; q < RPL; ++q) red[w][l * RPL + q] = s[q];
  __syncthreads();
  double ss = 0.0;
  for (int e = threadIdx.x; e < 64 * RPL; e += 64 * NW) {
    const int64_t rr = (int64_t)blockIdx.x * 64 * RPL + e;
    if (rr < nrows) {
      double t = red[0][e];
      for (int q = 1; q < NW; ++q) t += red[q][e];
      const double v = (beta == 0.0 ? 0.0 : beta * y[rr]) + alpha * t;
      y[rr] = v;
      ss += v * v;
    }
  }
  if (sq) {   // this block's partial sum of the updated y^2
    __shared__ double rs[16];
    ss = block_sum(ss, rs);
    if (threadIdx.x == 0) sq[blockIdx.x] = ss;
  }
}

// ---------------------------------------------------------------------------------------
// Small kernels of the projected problems

// The SVD of the (tp+1) x tp lower-bidiagonal B (diagonal gamma_i, subdiagonal beta_{i+1}) from
// the symmetric eigenproblem of its Golub-Kahan tridiagonal: zero diagonal of order 2 tp + 1 and
// off-diagonal (gamma_0, beta_1, gamma_1, beta_2, ..., gamma_{tp-1}, beta_tp).  For a singular
// triplet (s, u, v) of B the vector interleaving u and v (u_0, v_0, u_1, v_1, ..., u_tp), scaled
// by 1/sqrt(2), is an eigenvector with eigenvalue s; B is never squared.
__global__ void k_tgk_build(const double *__restrict__ gamma, const double *__restrict__ beta, int tp,
                            double *__restrict__ d, double *__restrict__ e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2 * tp + 1) d[i] = 0.0;
  if (i < tp) {
    e[2 * i] = gamma[i];
    e[2 * i + 1] = beta[i + 1];
  }
}

// S[j] = j-th largest eigenvalue, V[:, j] = sqrt2 * odd entries of its eigenvector (V column-major
// tp x tp), u0[j] = sqrt2 * first entry (the first row of U).
__global__ void k_tgk_extract(const double *__restrict__ lam, const double *__restrict__ C, int tp,
                              double *__restrict__ S, double *__restrict__ V, double *__restrict__ u0) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)tp * tp) return;
  const int n2 = 2 * tp + 1;
  const int i = (int)(idx % tp), j = (int)(idx / tp);
  const int jj = n2 - 1 - j;
  const double r2 = 1.4142135623730950488;
  const double *z = C + (int64_t)jj * n2;
  V[idx] = r2 * z[2 * i + 1];
  if (i == 0) {
    u0[j] = r2 * z[0];
    S[j] = lam[jj] > 0.0 ? lam[jj] : 0.0;
  }
}

struct UpreIn {
  const double *s;      // singular values, descending (first t used)
  const double *c;      // coefficients of the right-hand side (first t used), or NULL
  const double *u0;     // GKB: first row of U with stride ldu (c_i = *scale * u0[i*ldu])
  int64_t ldu;
  const double *scale;  // device scalar (||r~||)
  int t;
};

__device__ __forceinline__ double coef(const UpreIn &q, int i) {
  return q.c ? q.c[i] : (*q.scale) * q.u0[(int64_t)i * q.ldu];
}

// U(alpha) = sum (alpha^2/(s^2+alpha^2))^2 c^2 + 2 sum s^2/(s^2+alpha^2) - t, block-parallel
__device__ double upre_eval(const UpreIn &q, double alpha, double *red) {
  const double a2 = alpha * alpha;
  double acc = 0.0;
  for (int i = threadIdx.x; i < q.t; i += blockDim.x) {
    const double s2 = q.s[i] * q.s[i];
    const double f = a2 / (s2 + a2);
    const double c = coef(q, i);
    acc += f * f * c * c + 2.0 * s2 / (s2 + a2);
  }
  double tot = block_sum(acc, red);
  __shared__ double bc;
  if (threadIdx.x == 0) bc = tot - q.t;
  __syncthreads();
  return bc;
}

// alpha minimizing the UPRE: logarithmic grid on [1e-3 max(s_t, 1e-14 s_1), s_1], the grid
// point with the smallest value (larger alpha on ties), golden-section search in log(alpha)
// over the two neighbouring grid cells.  Single block.
__global__ void k_upre_alpha(UpreIn q, double *alpha_out) {
  __shared__ double red[16];
  __shared__ double vals[kUpreGrid];
  __shared__ double lgrid[kUpreGrid];
  const double s1 = q.s[0];
  double st = q.s[q.t - 1];
  if (st < 1e-14 * s1) st = 1e-14 * s1;
  const double llo = log(kUpreLo * st), lhi = log(s1);
  const double step = (lhi - llo) / (kUpreGrid - 1);
  for (int k = threadIdx.x; k < kUpreGrid; k += blockDim.x) lgrid[k] = k == kUpreGrid - 1 ? lhi : llo + step * k;
  __syncthreads();
  // grid values: one thread per grid point (t terms each)
  for (int k = threadIdx.x; k < kUpreGrid; k += blockDim.x) {
    const double a = exp(lgrid[k]), a2 = a * a;
    double acc = 0.0;
    for (int i = 0; i < q.t; ++i) {
      const double s2 = q.s[i] * q.s[i];
      const double f = a2 / (s2 + a2);
      const double c = coef(q, i);
      acc += f * f * c * c + 2.0 * s2 / (s2 + a2);
    }
    vals[k] = acc - q.t;
  }
  __syncthreads();
  __shared__ int kbest;
  __shared__ double best;
  if (threadIdx.x == 0) {
    int kb = 0;
    double b = vals[0];
    for (int k = 1; k < kUpreGrid; ++k)
      if (vals[k] <= b) {
        b = vals[k];
        kb = k;
      }
    kbest = kb;
    best = b;
  }
  __syncthreads();
  const int k = kbest;
  double a = lgrid[k > 0 ? k - 1 : 0];
  double b = lgrid[k < kUpreGrid - 1 ? k + 1 : kUpreGrid - 1];
  const double g = (sqrt(5.0) - 1.0) / 2.0;
  double x1 = b - g * (b - a), x2 = a + g * (b - a);
  double f1 = upre_eval(q, exp(x1), red), f2 = upre_eval(q, exp(x2), red);
  while (b - a > kGoldenTol) {
    if (f1 <= f2) {
      b = x2;
      x2 = x1;
      f2 = f1;
      x1 = b - g * (b - a);
      f1 = upre_eval(q, exp(x1), red);
    } else {
      a = x1;
      x1 = x2;
      f1 = f2;
      x2 = a + g * (b - a);
      f2 = upre_eval(q, exp(x2), red);
    }
  }
  double alpha = exp(0.5 * (a + b));
  const double fa = upre_eval(q, alpha, red);
  if (threadIdx.x == 0) *alpha_out = fa > best ? exp(lgrid[k]) : alpha;
}

// eq. (eq:alpha1): (n/m)^3.5 * s_1 / mean(s_i > 0), over cnt values (descending).  Single block.
__global__ void k_alpha1(const double *__restrict__ s, int cnt, double nm, double *alpha_out) {
  __shared__ double red[16];
  double sum = 0.0, num = 0.0;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x)
    if (s[i] > 0.0) {
      sum += s[i];
      num += 1.0;
    }
  sum = block_sum(sum, red);
  num = block_sum(num, red);
  if (threadIdx.x == 0) *alpha_out = pow(nm, 3.5) * s[0] / (sum / num);
}

// g[i] = scale * s_i / (s_i^2 + alpha^2) * coef_i  for i < cnt (coef from c or from u0 rows)
__global__ void k_filter(const double *__restrict__ s, const double *__restrict__ alpha, UpreIn q, int cnt,
                         double *__restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const double a = *alpha;
  g[i] = s[i] / (s[i] * s[i] + a * a) * coef(q, i);
}

// RSVD: S = sqrt(|lambda|) sorted descending (lambda ascending from the eigensolver), and the
// eigenvector columns in the same order: Vs[:, i] = V[:, perm(i)]
// S = sqrt|lambda| in descending order with perm its source indices; equal magnitudes keep their
// ascending eigenvalue order (NaN ranks last).  One thread per value counts the values ranked
// before it.
__global__ void k_rsvd_sort(const double *__restrict__ lam, int tp, double *__restrict__ S, int *__restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tp) return;
  const double li = lam[i];
  const double v = isnan(li) ? -1.0 : sqrt(fabs(li));
  int rank = 0;
  for (int j = 0; j < tp; ++j) {
    const double lj = lam[j];
    const double u = isnan(lj) ? -1.0 : sqrt(fabs(lj));
    rank += (u > v) || (u == v && j < i);
  }
  perm[rank] = i;
  S[rank] = li != li ? 0.0 : v;
}

// Shifted Cholesky QR helpers (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, SIAM J. Sci.
// Comput. 2020).  k_gram_shift adds s = 11 (rows cols + cols (cols + 1)) u trace(G) to the
// diagonal of the Gram matrix G (cols x cols): trace(G) = ||Y||_F^2 bounds ||Y||_2^2.
__global__ void __launch_bounds__(kThreads) k_gram_shift(double *__restrict__ G, int cols, int64_t rows) {
  __shared__ double red[kThreads / 64];
  double tr = 0.0;
  for (int i = threadIdx.x; i < cols; i += kThreads) tr += G[(int64_t)i * cols + i];
  tr = block_sum(tr, red);
  __shared__ double trs;
  if (threadIdx.x == 0) trs = tr;
  __syncthreads();
  tr = trs;
  const double u = 1.1102230246251565e-16;   // 2^-53
  const double shift = 11.0 * ((double)rows * cols + (double)cols * (cols + 1)) * u * tr;
  for (int i = threadIdx.x; i < cols; i += kThreads) G[(int64_t)i * cols + i] += shift;
}

// G[i] = sum over p < P of Gs[p * cc + i], in slice order (cc = cols^2 entries)
__global__ void k_sum_slices(const double *__restrict__ Gs, int P, int64_t cc, double *__restrict__ G) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cc; i += (int64_t)gridDim.x * blockDim.x) {
    double t = 0.0;
    for (int p = 0; p < P; ++p) t += Gs[p * cc + i];
    G[i] = t;
  }
}

// zero the strictly lower triangle of the column-major cols x cols R^-1, so that a plain product
// with it reads only the triangle
// rows r0 .. r0 + rows - 1 of the column-major single-precision matrix Q (ld rows) to the
// rows x cols double matrix C, and back
__global__ void k_rows_to64(const float *__restrict__ Q, int64_t ld, int64_t r0, int64_t rows, int cols,
                            double *__restrict__ C) {
  for (int c = blockIdx.y; c < cols; c += gridDim.y)
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x)
      C[(int64_t)c * rows + r] = (double)Q[(int64_t)c * ld + r0 + r];
}
__global__ void k_rows_to32(const double *__restrict__ C, int64_t rows, int cols, float *__restrict__ Q, int64_t ld,
                            int64_t r0) {
  for (int c = blockIdx.y; c < cols; c += gridDim.y)
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x)
      Q[(int64_t)c * ld + r0 + r] = (float)C[(int64_t)c * rows + r];
}
__global__ void k_to_f32(const double *__restrict__ x, int64_t n, float *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

__global__ void k_zero_lower(double *__restrict__ A, int cols) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)cols * cols) return;
  const int r = (int)(idx % cols), c = (int)(idx / cols);
  if (r > c) A[idx] = 0.0;
}

// out[0] = max |G - I| over the cols x cols Gram matrix (NaN counts as +inf), as the bits of a
// non-negative double (whose integer order is its numeric order); out[0] must start at 0.
// Block b takes the columns b, b + gridDim.x, ...
__global__ void __launch_bounds__(kThreads) k_orth_defect(const double *__restrict__ G, int cols,
                                                          unsigned long long *__restrict__ out) {
  __shared__ double red[kThreads];
  double mx = 0.0;
  for (int c = blockIdx.x; c < cols; c += gridDim.x)
    for (int r = threadIdx.x; r < cols; r += kThreads) {
      const double d = fabs(G[(int64_t)c * cols + r] - (r == c ? 1.0 : 0.0));
      mx = d != d ? INFINITY : fmax(mx, d);
    }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

__global__ void k_gather_cols(const double *__restrict__ V, int64_t ldv, int nrows, const int *__restrict__ perm, int ncols,
                              double *__restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nrows * ncols) return;
  const int r = (int)(idx % nrows), c = (int)(idx / nrows);
  out[idx] = V[(int64_t)perm[c] * ldv + r];
}

// c_i = (V~_i . btr) / S_i  for i < t (U~ = V~ ./ S)
__global__ void k_rsvd_coef(const double *__restrict__ Vs, int tp, const double *__restrict__ btr, const double *__restrict__ S,
                            int t, double *__restrict__ c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= t) return;
  double acc = 0.0;
  for (int r = 0; r < tp; ++r) acc += Vs[(int64_t)i * tp + r] * btr[r];
  c[i] = acc / S[i];
}

// IRLS pieces
// winv = 1 / (W_z W_L): layer-constant depth weight (mid-depth)^(-beta) times the focusing
// weight ((m_prev - m_prev2)^2 + eps2)^((lambda-2)/4) (identity at k = 1)
__global__ void k_irls_winv(const double *__restrict__ zmid_w, int64_t nlay, int64_t n, const double *__restrict__ mp,
                            const double *__restrict__ mp2, int k, double lam, double eps2, double *__restrict__ winv) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double w = zmid_w[i / nlay];
    if (k > 1) {
      const double dm = mp[i] - mp2[i];
      w *= pow(dm * dm + eps2, (lam - 2.0) / 4.0);
    }
    winv[i] = 1.0 / w;
  }
}

// r = wd * (d_obs - gm)
__global__ void k_residual(const double *__restrict__ wd, const double *__restrict__ dobs, const double *__restrict__ gm,
                           int64_t m, double *__restrict__ r) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = wd[i] * (dobs[i] - gm[i]);
}

// m_new = clip(m_prev + winv * y, lo, hi)
__global__ void k_update_clip(const double *__restrict__ mp, const double *__restrict__ winv, const double *__restrict__ y,
                              int64_t n, double lo, double hi, double *__restrict__ mn) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = mp[i] + winv[i] * y[i];
    mn[i] = v < lo ? lo : (v > hi ? hi : v);
  }
}

// ---------------------------------------------------------------------------------------
// Host helpers

unsigned grid_for(int64_t n, int threads = kThreads, int64_t cap = 4096) {
  int64_t g = (n + threads - 1) / threads;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Rows per lane load of a basis: 16 bytes (2 doubles or 4 floats) when every column start is
// 16-byte aligned, else 1.
template <typename TB> int rows_per_load(const TB *Q, int64_t ld) {
  constexpr int R = 16 / (int)sizeof(TB);
  return (ld % R == 0 && ((uintptr_t)Q % 16) == 0) ? R : 1;
}
int partials_for(int64_t nrows, int rpl) {
  const int64_t rows = (int64_t)kRowsMin * rpl;
  return (int)((nrows + rows - 1) / rows);
}

// The spectra handle's rocBLAS handle, created on first use on the handle's device and bound to
// the caller's stream: solver calls on different spectra handles (and so on different streams)
// never share one.
rocblas_handle blas(ff_spectra sh, hipStream_t s, ff_status *st) {
  if (!sh->blas) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) {
      *st = fail(FF_EHIP, "rocblas_create_handle failed");
      return nullptr;
    }
    sh->blas = h;
  }
  rocblas_handle h = (rocblas_handle)sh->blas;
  if (rocblas_set_stream(h, s) != rocblas_status_success) {
    *st = fail(FF_EHIP, "rocblas_set_stream failed");
    return nullptr;
  }
  *st = FF_OK;
  return h;
}

}  // namespace

void release_blas(ff_spectra sh) {
  if (sh->blas) rocblas_destroy_handle((rocblas_handle)sh->blas);
  sh->blas = nullptr;
}

namespace {

#define FF_BLAS(call, what)                                                       \
  do {                                                                            \
    rocblas_status bs_ = (call);                                                  \
    if (bs_ != rocblas_status_success)                                            \
      return fail(FF_EHIP, std::string(what) + ": " + rocblas_status_to_string(bs_)); \
  } while (0)

// bump allocator over the caller's workspace (256-byte aligned pieces)
struct Arena {
  char *base;
  size_t cap, used = 0;
  bool dry;   // size query only
  template <typename T> T *take(size_t count) {
    size_t off = (used + 255) & ~(size_t)255;
    used = off + sizeof(T) * count;
    return dry ? nullptr : (T *)(base + off);
  }
};

// out = Q^T v (partials in part, then summed) and y = beta y + alpha Q c, with the launch shapes
// of the kernels above.
// `run` (device flag, may be NULL): the kernels return at once when it is 0.
template <typename TB>
void launch_gemv_t(const TB *Q, int64_t ld, int64_t nrows, int ncols, const double *v, double *out, double *part,
                   hipStream_t s, const int *run = nullptr) {
  const int rpl = rows_per_load(Q, ld);
  const int P = partials_for(nrows, rpl);
  const dim3 gt(P, (ncols + kTCols - 1) / kTCols);
  constexpr int R = 16 / (int)sizeof(TB);
  if (rpl == R)
    k_gemv_t_partial<R, TB><<<gt, kThreads, 0, s>>>(Q, ld, nrows, ncols, v, part, run);
  else
    k_gemv_t_partial<1, TB><<<gt, kThreads, 0, s>>>(Q, ld, nrows, ncols, v, part, run);
  k_colsum<<<(ncols + kCSumCols - 1) / kCSumCols, kThreads, 0, s>>>(part, P, ncols, out, 1.0, run);
}

// Returns the number of blocks (= partial sums written to sq, if given).
template <typename TB>
int launch_gemv_n(const TB *Q, int64_t ld, int64_t nrows, int ncols, const double *c, double *y, double alpha,
                  double beta, hipStream_t s, const int *run = nullptr, double *sq = nullptr) {
  // 16-byte loads pay off on long bases; short ones want more blocks
  constexpr int R = 16 / (int)sizeof(TB);
  if (rows_per_load(Q, ld) == R && nrows >= 32768) {
    const unsigned nb = (unsigned)((nrows + 64 * R - 1) / (64 * R));
    k_gemv_n<R, TB><<<nb, 64 * kNWaves, 0, s>>>(Q, ld, nrows, ncols, c, y, alpha, beta, run, sq);
    return (int)nb;
  }
  // shorter bases: twice the waves per block, half the columns per wave
  const unsigned nb = (unsigned)((nrows + 63) / 64);
  k_gemv_n<1, TB, 2 * kNWaves><<<nb, 128 * kNWaves, 0, s>>>(Q, ld, nrows, ncols, c, y, alpha, beta, run, sq);
  return (int)nb;
}

// v <- (I - Q Q^T) v over the first ncols columns of Q (classical Gram-Schmidt), repeated once
// when the first pass cancelled most of v (k_norm_flag); the test stays on the device.  On
// return *nrm = ||v|| and *inv = 1/||v|| (0 for a zero vector).  sq0 holds, on entry when
// have_sq, the kNormBlocks partial sums of v^2 (else they are formed here); sq1 receives the
// block sums of the updated v^2 (one per A c block); part is the scratch of the products.
// flag: 1 int of scratch.
// When deferred is non-NULL and the second pass has at most kDeferMax partial sums, its final
// norm is left to k_scale_store_cond: *deferred receives that count (0 when the norm is final).
constexpr int kDeferMax = 2048;
template <typename TB>
ff_status reorth_norm(const TB *Q, int64_t ld, int64_t nrows, int ncols, double *v, double *coef, double *part,
                      double *sq0, bool have_sq, double *sq1, int *flag, double *nrm, double *inv, hipStream_t s,
                      int *deferred = nullptr) {
  if (deferred) *deferred = 0;
  if (!have_sq) k_sumsq_partial<<<kNormBlocks, kThreads, 0, s>>>(v, nrows, sq0);
  if (ncols <= 0) {
    k_norm_finalize<<<1, kThreads, 0, s>>>(sq0, kNormBlocks, nrm, inv);
    FF_LAUNCH_CHECK("norm");
    return FF_OK;
  }
  launch_gemv_t(Q, ld, nrows, ncols, v, coef, part, s);
  const int nb1 = launch_gemv_n(Q, ld, nrows, ncols, coef, v, -1.0, 1.0, s, nullptr, sq1);
  k_norm_flag<<<1, kThreads, 0, s>>>(sq0, kNormBlocks, sq1, nb1, flag, nrm, inv);
  launch_gemv_t(Q, ld, nrows, ncols, v, coef, part, s, flag);
  const int nb2 = launch_gemv_n(Q, ld, nrows, ncols, coef, v, -1.0, 1.0, s, flag, sq1);
  if (deferred && nb2 <= kDeferMax)
    *deferred = nb2;
  else
    k_norm_cond<<<1, kThreads, 0, s>>>(sq1, nb2, flag, nrm, inv);
  FF_LAUNCH_CHECK("reorthogonalization");
  return FF_OK;
}

// y = alpha * Q c   (Q nrows x ncols)
ff_status gemv_n(const double *Q, int64_t ld, int64_t nrows, int ncols, const double *c, double *y, double alpha,
                 hipStream_t s) {
  launch_gemv_n(Q, ld, nrows, ncols, c, y, alpha, 0.0, s);
  FF_LAUNCH_CHECK("gemv");
  return FF_OK;
}

// out = Q^T v   (ncols values)
ff_status gemv_t(const double *Q, int64_t ld, int64_t nrows, int ncols, const double *v, double *out, double *part,
                 hipStream_t s) {
  launch_gemv_t(Q, ld, nrows, ncols, v, out, part, s);
  FF_LAUNCH_CHECK("gemv_t");
  return FF_OK;
}

// nrm = ||x||, inv = 1/nrm (device scalars)
ff_status norm2(const double *x, int64_t n, double *nrm, double *inv, double *part, hipStream_t s) {
  const int P = 256;
  k_sumsq_partial<<<P, kThreads, 0, s>>>(x, n, part);
  k_norm_finalize<<<1, kThreads, 0, s>>>(part, P, nrm, inv);
  FF_LAUNCH_CHECK("norm");
  return FF_OK;
}

// Workspace of Algorithm 1 for a handle and tp (also used for sizing when a.dry); the bases A
// (n x tp) and H (m x (tp + 1)) are stored as TB.
// Leading dimension of a stored basis: the rows rounded up to 64 elements, so that every column
// starts on a 256-byte boundary and the products use 16-byte loads for any n and m.
inline int64_t basis_ld(int64_t rows) { return (rows + 63) / 64 * 64; }

// Columns of the model-side basis A kept by gkb_run: all t_p, or a ring of two when the handle's
// gkb_onesided tuning is 2 (A is then recomputed in a second pass instead of stored).
inline int gkb_acols(ff_spectra h, int tp) { return h->gkb_onesided == 2 ? (tp < 2 ? tp : 2) : tp; }

template <typename TB> struct GkbWs {
  TB *A, *H;
  int64_t ldA, ldH;
  double *b, *c, *gamma, *beta, *ginv, *binv, *coef, *part, *dT, *eT, *C, *S, *V, *u0, *g, *w, *alpha, *sq0, *sq1;
  double *wdc, *winvc;   // copies of the weights, so that a captured iteration loop reads fixed addresses
  int *flag;
  rocblas_int *info;
  void carve(Arena &a, int64_t n, int64_t m, int tp, int acols) {
    const int64_t P = ((n > m ? n : m) + kRowsMin - 1) / kRowsMin + 1;   // partial rows at one row per load
    const int64_t Pn = ((n > m ? n : m) + 63) / 64 + 1;                  // blocks of the A c products
    const int64_t npart = ((P > 256 ? P : 256) + 1) * (tp + 2);
    ldA = basis_ld(n);
    ldH = basis_ld(m);
    A = a.take<TB>((size_t)ldA * acols);
    H = a.take<TB>((size_t)ldH * (tp + 1));
    b = a.take<double>(n);
    c = a.take<double>(m);
    gamma = a.take<double>(tp + 1);
    beta = a.take<double>(tp + 2);
    ginv = a.take<double>(tp + 1);
    binv = a.take<double>(tp + 2);
    coef = a.take<double>(tp + 2);
    part = a.take<double>((size_t)(npart > Pn ? npart : Pn));
    dT = a.take<double>(2 * (size_t)tp + 1);
    eT = a.take<double>(2 * (size_t)tp + 1);
    C = a.take<double>((2 * (size_t)tp + 1) * (2 * (size_t)tp + 1));
    S = a.take<double>(tp);
    V = a.take<double>((size_t)tp * tp);
    u0 = a.take<double>(tp);
    g = a.take<double>(tp);
    w = a.take<double>(tp);
    alpha = a.take<double>(2);
    sq0 = a.take<double>(kNormBlocks);
    sq1 = a.take<double>((size_t)Pn);
    wdc = a.take<double>(m);
    winvc = a.take<double>(n);
    flag = a.take<int>(1);
    info = a.take<rocblas_int>(4);
  }
};

// Row chunks of a split Gram product Y^T Y (rows x cols Y): a single product has only
// (cols / tile)^2 output tiles, too few for the chip when cols is small, so the rows are cut into
// S chunks of at least 4 max(cols, 256) rows whose Gram matrices come from one batched product;
// at most 64 chunks and 2^26 doubles (512 MB) of partial matrices.
constexpr int64_t kGramScratch = (int64_t)1 << 26;
int gram_chunks(int64_t rows, int cols) {
  int64_t S = rows / (4 * (int64_t)(cols > 256 ? cols : 256));
  if (S > 64) S = 64;
  const int64_t budget = kGramScratch / ((int64_t)cols * cols) - 1;
  if (S > budget) S = budget;
  return S < 2 ? 1 : (int)S;
}
size_t gram_scratch(int64_t rows, int cols) {
  const int S = gram_chunks(rows, cols);
  return S > 1 ? (size_t)(S + 1) * cols * cols : 1;
}

struct RsvdWs {
  double *Q, *Bm, *Y, *lam, *E, *S, *Vs, *btr, *c, *g, *w, *tau, *alpha, *part, *T, *U, *Gs, *dev;
  int *perm;
  rocblas_int *info;
  void carve(Arena &a, int64_t n, int64_t m, int tp) {
    const int64_t P = ((n > m ? n : m) + kRowsMin - 1) / kRowsMin + 1;   // partial rows at one row per load
    Q = a.take<double>((size_t)n * tp);     // n x tp (also holds the m x tp factors)
    Bm = a.take<double>((size_t)m * tp);    // G~ Q
    T = a.take<double>((size_t)(n > m ? n : m) * tp);   // QR scratch
    U = a.take<double>((size_t)(n > m ? n : m) * tp);
    Gs = a.take<double>(gram_scratch(n > m ? n : m, tp));
    dev = a.take<double>(1);
    Y = a.take<double>((size_t)tp * tp);    // B^T B, then its eigenvectors
    lam = a.take<double>(tp);
    E = a.take<double>(tp);
    S = a.take<double>(tp);
    Vs = a.take<double>((size_t)tp * tp);
    btr = a.take<double>(tp);
    c = a.take<double>(tp);
    g = a.take<double>(tp);
    w = a.take<double>(tp);
    tau = a.take<double>(tp);
    alpha = a.take<double>(2);
    part = a.take<double>((size_t)((P > 256 ? P : 256) + 1) * (tp + 2));
    perm = a.take<int>(tp);
    info = a.take<rocblas_int>(8);
  }
};

// Algorithm 2 with the n x t_p matrices (Q and the copy kept for a second Cholesky QR attempt)
// stored in single precision: they are streamed through FP64 row chunks (Ca, Cb) for the Gram
// products and the products with R^-1, so every product and sum is still formed in double.
// The m x t_p matrices and the projected problem stay FP64.
int64_t lean_chunk_rows(int64_t n, int tp) {
  int64_t r = ((int64_t)1 << 27) / (tp > 0 ? tp : 1);   // 1 GB of doubles per staging buffer
  if (r < 4096) r = 4096;
  return r > n ? n : r;
}

struct RsvdWs32 {
  float *Q, *M, *winv32;
  double *Bm, *T, *U, *Gs, *Ca, *Cb, *dev, *Y, *lam, *E, *S, *Vs, *btr, *c, *g, *w, *tau, *alpha, *part;
  int *perm;
  rocblas_int *info;
  int64_t CH;
  void carve(Arena &a, int64_t n, int64_t m, int tp) {
    const int64_t P = ((n > m ? n : m) + kRowsMin - 1) / kRowsMin + 1;
    CH = lean_chunk_rows(n, tp);
    Q = a.take<float>((size_t)n * tp);
    M = a.take<float>((size_t)n * tp);
    winv32 = a.take<float>(n);
    Bm = a.take<double>((size_t)m * tp);     // G~ Q, and Omega when drawn here
    T = a.take<double>((size_t)m * tp);      // QR scratch of the m x t_p factors
    U = a.take<double>((size_t)m * tp);
    Gs = a.take<double>(gram_scratch(m > CH ? m : CH, tp));
    Ca = a.take<double>((size_t)CH * tp);
    Cb = a.take<double>((size_t)CH * tp);
    dev = a.take<double>(1);
    Y = a.take<double>((size_t)tp * tp);
    lam = a.take<double>(tp);
    E = a.take<double>(tp);
    S = a.take<double>(tp);
    Vs = a.take<double>((size_t)tp * tp);
    btr = a.take<double>(tp);
    c = a.take<double>(tp);
    g = a.take<double>(tp);
    w = a.take<double>(tp);
    tau = a.take<double>(tp);
    alpha = a.take<double>(2);
    part = a.take<double>((size_t)((P > 256 ? P : 256) + 1) * (tp + 2));
    perm = a.take<int>(tp);
    info = a.take<rocblas_int>(8);
  }
};

struct IrlsWs {
  double *winv, *r, *gm, *y, *zw, *sig, *part, *nrm;
  void carve(Arena &a, int64_t n, int64_t m, int nz, int tp) {
    winv = a.take<double>(n);
    r = a.take<double>(m);
    gm = a.take<double>(m);
    y = a.take<double>(n);
    zw = a.take<double>(nz);
    sig = a.take<double>(tp);
    part = a.take<double>(256);
    nrm = a.take<double>(2);
  }
};

ff_status check_solver_args(const char *who, ff_spectra h, int t, int tp, const void *r, const void *wd,
                            const void *winv, const void *y, const void *alpha, const void *sigma, const void *ws) {
  const std::string w(who);
  if (!h || !r || !wd || !winv || !y || !alpha || !sigma || !ws) return fail(FF_EINVAL, w + ": NULL argument");
  if (t < 1 || tp < t || tp > h->m) return fail(FF_ESHAPE, w + ": need 1 <= t <= tp <= m");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(FF_EHIP, w + ": hipGetDevice failed");
  if (cur != h->device) return fail(FF_EDEVICE, w + ": current device differs from the handle's device");
  return FF_OK;
}

enum { ALPHA_UPRE = 0, ALPHA_ONE = 1, ALPHA_FIXED = 2 };

// the regularization parameter into *dev_alpha (device) according to mode
ff_status choose_alpha(ff_spectra h, int mode, double fixed, UpreIn q, const double *s_all, int cnt,
                       double *dev_alpha, hipStream_t s) {
  if (mode == ALPHA_FIXED) {
    FF_HIP(hipMemcpyAsync(dev_alpha, &fixed, sizeof(double), hipMemcpyHostToDevice, s));
    // the host value must stay alive until the copy has run
    FF_HIP(hipStreamSynchronize(s));
  } else if (mode == ALPHA_ONE) {
    k_alpha1<<<1, kThreads, 0, s>>>(s_all, cnt, (double)h->n / (double)h->m, dev_alpha);
  } else if (mode == ALPHA_UPRE) {
    k_upre_alpha<<<1, kThreads, 0, s>>>(q, dev_alpha);
  } else {
    return fail(FF_EINVAL, "alpha_mode must be 0 (UPRE), 1 (alpha1) or 2 (fixed)");
  }
  FF_LAUNCH_CHECK("regularization parameter");
  return FF_OK;
}

// Runs `loop` (launches only, on the stream it is given) on stream s: eagerly, or, when the
// handle allows it, from a graph captured on the handle's own stream the first time and replayed
// while the key (workspace, t_p, basis type, tuning) stays the same.  Graphs are not used while
// the caller's stream is itself being captured (the launches then join that capture) or while
// pass profiling is on.
template <class Loop>
ff_status run_captured(ff_spectra h, hipStream_t s, const void *ws, size_t ws_bytes, int tp, int tb, Loop &&loop) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) cs = hipStreamCaptureStatusActive;
  if (!h->gkb_graph || h->prof_cap > 0 || cs != hipStreamCaptureStatusNone) return loop(s);
  const bool hit = h->gkb_exec && h->gkb_ws == ws && h->gkb_ws_bytes == ws_bytes && h->gkb_tp == tp &&
                   h->gkb_tb == tb && h->gkb_tune == h->tune_version;
  if (!hit) {
    if (h->gkb_exec) {
      FF_HIP(hipGraphExecDestroy((hipGraphExec_t)h->gkb_exec));
      h->gkb_exec = nullptr;
    }
    if (!h->cap_stream) FF_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    FF_HIP(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    ff_status st = loop(h->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (st != FF_OK) {
      if (g) hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "gkb_project: capture of the iteration loop");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "gkb_project: instantiation of the iteration graph");
    h->gkb_exec = ex;
    h->gkb_ws = ws;
    h->gkb_ws_bytes = ws_bytes;
    h->gkb_tp = tp;
    h->gkb_tb = tb;
    h->gkb_tune = h->tune_version;
  }
  FF_HIP(hipGraphLaunch((hipGraphExec_t)h->gkb_exec, s));
  return FF_OK;
}

template <typename TB>
ff_status gkb_run(ff_spectra h, const double *rt, const double *wd, const double *winv, int t, int tp, int mode,
                  double *y, double *alpha, double *sigma, void *ws, size_t ws_bytes, hipStream_t s) {
  const int64_t n = h->n, m = h->m;
  Arena ar{(char *)ws, ws_bytes, 0, false};
  GkbWs<TB> W;
  // gkb_onesided: 0 = both bases reorthogonalized (Algorithm 1); 1 = only the data-side basis H,
  // the model-side basis A kept orthogonal by the recurrence itself (one-sided reorthogonalization
  // of the Golub-Kahan process, Simon and Zha 2000); 2 = as 1, with A recomputed in a second pass
  // instead of stored
  const int onesided = h->gkb_onesided;
  const bool ring = onesided == 2 && tp >= 2;
  W.carve(ar, n, m, tp, gkb_acols(h, tp));
  if (ar.used > ws_bytes) return fail(FF_ENOMEM, "gkb_project: workspace too small");
  auto acol = [&](int i) { return W.A + (int64_t)(ring ? (i & 1) : i) * W.ldA; };
  const double fixed = *alpha;
  ff_status st;
  // beta_1 = ||r~||, h_1 = r~ / beta_1 (stored in H; c holds the same values in double, the
  // operand of the next G^T)
  if ((st = norm2(rt, m, W.beta, W.binv, W.part, s))) return st;
  k_scale_from<TB><<<grid_for(m), kThreads, 0, s>>>(rt, W.binv, W.H, W.c, m);
  FF_HIP(hipMemsetAsync(W.b, 0, sizeof(double) * n, s));
  FF_HIP(hipMemcpyAsync(W.wdc, wd, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
  FF_HIP(hipMemcpyAsync(W.winvc, winv, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  // The t_p iterations: about 24 launches each, none of which waits for the host.  With the
  // handle's gkb_graph tuning they are captured once into a graph per (handle, workspace, t_p,
  // basis type, tuning) and replayed on later solves; the graph reads only the workspace (the
  // weights are copied there above), the handle's spectra and its pass buffers.
  auto iterate = [&](hipStream_t s) -> ff_status {
  ff_status st;
  for (int i = 0; i < tp; ++i) {
    TB *ai = acol(i);
    const TB *hi = W.H + (int64_t)i * W.ldH;
    // b = G~^T h_i - beta_i a_{i-1}, reorthogonalized (both-sided); gamma_i = ||b||
    if ((st = op_apply(h, 1, 1, W.c, m, W.b, n, W.wdc, W.winvc, FF_F64, s))) return st;
    if (i > 0)
      k_axpy_sumsq<TB><<<kNormBlocks, kThreads, 0, s>>>(W.b, acol(i - 1), W.beta + i, -1.0, n, W.sq0);
    int dn = 0;
    if (onesided) {
      // no reorthogonalization against A: gamma_i from the partial sums of b, fused into the scaling
      if (i == 0) k_sumsq_partial<<<kNormBlocks, kThreads, 0, s>>>(W.b, n, W.sq0);
      k_scale_store_cond<TB><<<grid_for(n), kThreads, 0, s>>>(W.b, ai, n, W.sq0, kNormBlocks, nullptr, W.gamma + i,
                                                              W.ginv + i);
    } else if ((st = reorth_norm<TB>(W.A, W.ldA, n, i, W.b, W.coef, W.part, W.sq0, i > 0, W.sq1, W.flag,
                                     W.gamma + i, W.ginv + i, s, &dn))) {
      return st;
    } else if (dn > 0)     // b = a_i as stored
      k_scale_store_cond<TB><<<grid_for(n), kThreads, 0, s>>>(W.b, ai, n, W.sq1, dn, W.flag, W.gamma + i, W.ginv + i);
    else
      k_scale_store<TB><<<grid_for(n), kThreads, 0, s>>>(W.b, W.ginv + i, ai, n);
    // c = G~ a_i - gamma_i h_i, reorthogonalized; beta_{i+1} = ||c||
    if ((st = op_apply(h, 0, 1, W.b, n, W.c, m, W.winvc, W.wdc, FF_F64, s))) return st;
    k_axpy_sumsq<TB><<<kNormBlocks, kThreads, 0, s>>>(W.c, hi, W.gamma + i, -1.0, m, W.sq0);
    if ((st = reorth_norm<TB>(W.H, W.ldH, m, i + 1, W.c, W.coef, W.part, W.sq0, true, W.sq1, W.flag,
                              W.beta + i + 1, W.binv + i + 1, s, &dn)))
      return st;
    TB *hn = W.H + (int64_t)(i + 1) * W.ldH;
    if (dn > 0)
      k_scale_store_cond<TB><<<grid_for(m), kThreads, 0, s>>>(W.c, hn, m, W.sq1, dn, W.flag, W.beta + i + 1,
                                                              W.binv + i + 1);
    else
      k_scale_store<TB><<<grid_for(m), kThreads, 0, s>>>(W.c, W.binv + i + 1, hn, m);
  }
  FF_LAUNCH_CHECK("gkb iteration");
  return FF_OK;
  };
  if ((st = run_captured(h, s, (const void *)ws, ws_bytes, tp, (int)sizeof(TB), iterate))) return st;

  // SVD of the (tp+1) x tp bidiagonal through its Golub-Kahan tridiagonal
  const int n2 = 2 * tp + 1;
  k_tgk_build<<<(n2 + 255) / 256, 256, 0, s>>>(W.gamma, W.beta, tp, W.dT, W.eT);
  rocblas_handle bh = blas(h, s, &st);
  if (st) return st;
  FF_BLAS(rocsolver_dstedc(bh, rocblas_evect_tridiagonal, n2, W.dT, W.eT, W.C, n2, W.info), "rocsolver_dstedc");
  k_tgk_extract<<<grid_for((int64_t)tp * tp, 256, 1 << 30), 256, 0, s>>>(W.dT, W.C, tp, W.S, W.V, W.u0);
  FF_LAUNCH_CHECK("bidiagonal SVD");
  // alpha from the first t singular values and c_i = ||r~|| U(1, i)  (||r~|| = beta_1)
  UpreIn q{W.S, nullptr, W.u0, 1, W.beta, t};
  if ((st = choose_alpha(h, mode, fixed, q, W.S, tp, W.alpha, s))) return st;
  // y = ||r~|| A V Gamma(alpha) U(1,:)^T
  UpreIn qa = q;
  qa.t = tp;
  k_filter<<<(tp + 255) / 256, 256, 0, s>>>(W.S, W.alpha, qa, tp, W.g);
  if ((st = gemv_n(W.V, tp, tp, tp, W.g, W.w, 1.0, s))) return st;
  if (onesided == 2) {
    // y = sum_i w_i a_i with a_i rebuilt by the same launches, on the same values, as in the
    // first pass (h_i from H exactly as the operator saw it, gamma_i and beta_i as computed
    // there), so every a_i is the first pass's bit for bit
    for (int i = 0; i < tp; ++i) {
      k_widen<TB><<<grid_for(m), kThreads, 0, s>>>(W.H + (int64_t)i * W.ldH, W.c, m);
      if ((st = op_apply(h, 1, 1, W.c, m, W.b, n, W.wdc, W.winvc, FF_F64, s))) return st;
      if (i > 0)
        k_axpy_sumsq<TB><<<kNormBlocks, kThreads, 0, s>>>(W.b, acol(i - 1), W.beta + i, -1.0, n, W.sq0);
      k_scale_store<TB><<<grid_for(n), kThreads, 0, s>>>(W.b, W.ginv + i, acol(i), n);
      if (i == 0)
        k_scaled<TB><<<grid_for(n), kThreads, 0, s>>>(acol(0), W.w, y, n);
      else
        k_axpy_sumsq<TB><<<kNormBlocks, kThreads, 0, s>>>(y, acol(i), W.w + i, 1.0, n, W.sq0);
    }
  } else {
    launch_gemv_n<TB>(W.A, W.ldA, n, tp, W.w, y, 1.0, 0.0, s);
  }
  FF_LAUNCH_CHECK("gkb solution");
  FF_HIP(hipMemcpyAsync(sigma, W.S, sizeof(double) * tp, hipMemcpyDeviceToDevice, s));
  FF_HIP(hipMemcpyAsync(alpha, W.alpha, sizeof(double), hipMemcpyDeviceToHost, s));
  FF_HIP(hipStreamSynchronize(s));
  return FF_OK;
}

// G = Y^T Y (cols x cols, full) for the column-major rows x cols Y; Gs is the scratch of
// gram_scratch(rows, cols) doubles.  The chunk products and the remainder rows' product are
// summed in chunk order.
ff_status gram(rocblas_handle bh, const double *Y, int64_t rows, int cols, double *G, double *Gs, hipStream_t s) {
  const double one = 1.0, zero = 0.0;
  const int S = gram_chunks(rows, cols);
  const rocblas_int r = (rocblas_int)rows, c = cols;
  if (S == 1) {
    FF_BLAS(rocblas_dgemm(bh, rocblas_operation_transpose, rocblas_operation_none, c, c, r, &one, Y, r, Y, r, &zero, G,
                          c),
            "rocblas_dgemm (Gram)");
    return FF_OK;
  }
  const int64_t K = rows / S, rem = rows - K * S, cc = (int64_t)cols * cols;
  FF_BLAS(rocblas_dgemm_strided_batched(bh, rocblas_operation_transpose, rocblas_operation_none, c, c, (rocblas_int)K,
                                        &one, Y, r, K, Y, r, K, &zero, Gs, c, cc, S),
          "rocblas_dgemm_strided_batched (Gram chunks)");
  int P = S;
  if (rem > 0) {
    const double *Yr = Y + K * S;
    FF_BLAS(rocblas_dgemm(bh, rocblas_operation_transpose, rocblas_operation_none, c, c, (rocblas_int)rem, &one, Yr, r,
                          Yr, r, &zero, Gs + cc * S, c),
            "rocblas_dgemm (Gram remainder)");
    P = S + 1;
  }
  k_sum_slices<<<grid_for(cc), kThreads, 0, s>>>(Gs, P, cc, G);
  FF_LAUNCH_CHECK("Gram sum");
  return FF_OK;
}

ff_status householder_qr(rocblas_handle bh, double *M, int64_t rows, int cols, double *tau) {
  FF_BLAS(rocsolver_dgeqrf(bh, (rocblas_int)rows, cols, M, (rocblas_int)rows, tau), "rocsolver_dgeqrf");
  FF_BLAS(rocsolver_dorgqr(bh, (rocblas_int)rows, cols, cols, M, (rocblas_int)rows, tau), "rocsolver_dorgqr");
  return FF_OK;
}

// One Cholesky QR attempt on the rows x cols matrix M (kept): `passes` passes of Gram product,
// Cholesky (potrf), triangular inverse (trtri) and product, the first one with the Gram matrix
// shifted when `shift`; then the Gram matrix of the result.  Returns through *ok whether every
// factorization succeeded and max |Q^T Q - I| <= 1e-8, and through *q the buffer (T or U)
// holding Q.
ff_status cholesky_qr(rocblas_handle bh, const double *M, int64_t rows, int cols, int passes, bool shift, double *T,
                      double *U, double *G, double *Gs, double *dev, rocblas_int *info, hipStream_t s, bool *ok,
                      const double **q) {
  const double one = 1.0, zero = 0.0;
  const rocblas_int r = (rocblas_int)rows, c = cols;
  FF_HIP(hipMemsetAsync(info, 0, 8 * sizeof(rocblas_int), s));
  const double *in = M;
  double *outs[3] = {T, U, T};
  for (int p = 0; p < passes; ++p) {
    double *out = outs[p];
    ff_status st = gram(bh, in, rows, cols, G, Gs, s);
    if (st) return st;
    if (p == 0 && shift) {
      k_gram_shift<<<1, kThreads, 0, s>>>(G, c, rows);
      FF_LAUNCH_CHECK("gram shift");
    }
    FF_BLAS(rocsolver_dpotrf(bh, rocblas_fill_upper, c, G, c, info + 2 * p), "rocsolver_dpotrf");
    FF_BLAS(rocsolver_dtrtri(bh, rocblas_fill_upper, rocblas_diagonal_non_unit, c, G, c, info + 2 * p + 1),
            "rocsolver_dtrtri");
    k_zero_lower<<<grid_for((int64_t)c * c, 256, 1 << 30), 256, 0, s>>>(G, c);
    FF_LAUNCH_CHECK("zero lower");
    FF_BLAS(rocblas_dgemm(bh, rocblas_operation_none, rocblas_operation_none, r, c, c, &one, in, r, G, c, &zero, out,
                          r),
            "rocblas_dgemm (Q R^-1)");
    in = out;
  }
  ff_status st = gram(bh, in, rows, cols, G, Gs, s);
  if (st) return st;
  FF_HIP(hipMemsetAsync(dev, 0, sizeof(double), s));
  k_orth_defect<<<c < 1024 ? c : 1024, kThreads, 0, s>>>(G, c, (unsigned long long *)dev);
  FF_LAUNCH_CHECK("orthogonality check");
  struct {
    rocblas_int info[8];
    double defect;
  } hs;
  FF_HIP(hipMemcpyAsync(hs.info, info, sizeof(hs.info), hipMemcpyDeviceToHost, s));
  FF_HIP(hipMemcpyAsync(&hs.defect, dev, sizeof(double), hipMemcpyDeviceToHost, s));
  FF_HIP(hipStreamSynchronize(s));
  bool good = hs.defect <= 1e-8;
  for (int i = 0; i < 2 * passes; ++i) good = good && hs.info[i] == 0;
  *ok = good;
  *q = in;
  return FF_OK;
}

// Orthonormal basis of the columns of the tall rows x cols matrix M, in place, by Cholesky QR:
// first plain CholeskyQR2 (two passes; enough while the columns' condition number stays below
// about 1e7), then, if its result is not orthonormal, shifted CholeskyQR3 (Fukaya, Kannan,
// Nakatsukasa, Yamamoto, Yanagisawa, SIAM J. Sci. Comput. 2020: the first of three passes
// factors the Gram matrix plus 11 (rows cols + cols (cols + 1)) u ||M||_F^2 I), then Householder
// QR (geqrf + orgqr).  Each attempt is accepted only if max |Q^T Q - I| <= 1e-8 and all of its
// factorizations succeeded.  T and U are rows x cols scratch, G is cols x cols, Gs the Gram
// scratch, dev one double and info eight ints.  Synchronizes s after each attempt.
ff_status qr_inplace(ff_spectra h, rocblas_handle bh, double *M, int64_t rows, int cols, double *tau, double *T,
                     double *U, double *G, double *Gs, double *dev, rocblas_int *info, hipStream_t s) {
  if (h->rsvd_qr != 1) {
    for (int attempt = h->rsvd_qr == 2 ? 1 : 0; attempt < 2; ++attempt) {
      bool ok = false;
      const double *q = nullptr;
      ff_status st = cholesky_qr(bh, M, rows, cols, attempt == 0 ? 2 : 3, attempt == 1, T, U, G, Gs, dev, info, s,
                                 &ok, &q);
      if (st) return st;
      if (ok) {
        FF_HIP(hipMemcpyAsync(M, q, sizeof(double) * rows * cols, hipMemcpyDeviceToDevice, s));
        (attempt == 0 ? h->qr_cholesky2 : h->qr_cholesky3) += 1;
        return FF_OK;
      }
    }
  }
  h->qr_householder += 1;
  return householder_qr(bh, M, rows, cols, tau);
}

// ---- Cholesky QR of the single-precision basis --------------------------------------------
dim3 chunk_grid(int64_t rows, int cols) {
  const int64_t bx = (rows + kThreads - 1) / kThreads;
  return dim3((unsigned)(bx < 64 ? bx : 64), (unsigned)(cols < 65535 ? cols : 65535));
}

// G = Q^T Q over row chunks staged in FP64 (the chunks' products accumulated in order)
ff_status gram32(rocblas_handle bh, const float *Q, int64_t n, int tp, RsvdWs32 &W, double *G, hipStream_t s) {
  // Each staging round converts S row blocks of R rows (S R <= CH) to FP64 side by side, and one
  // strided-batched product adds their Gram matrices to S partial sums (as gram() splits the
  // rows, so that the product has S times the output tiles); the partials are summed in order at
  // the end.  A last round of fewer rows adds its product to the first partial.
  const double one = 1.0, zero = 0.0;
  const int S = gram_chunks(W.CH, tp);
  const int64_t R = W.CH / S, cc = (int64_t)tp * tp;
  double *Gp = S > 1 ? W.Gs : G;
  bool first = true;
  for (int64_t r0 = 0; r0 < n;) {
    const int64_t left = n - r0;
    if (left >= (int64_t)S * R) {
      for (int p = 0; p < S; ++p)
        k_rows_to64<<<chunk_grid(R, tp), kThreads, 0, s>>>(Q, n, r0 + p * R, R, tp, W.Ca + p * R * tp);
      FF_LAUNCH_CHECK("basis chunk to FP64");
      FF_BLAS(rocblas_dgemm_strided_batched(bh, rocblas_operation_transpose, rocblas_operation_none, tp, tp,
                                            (rocblas_int)R, &one, W.Ca, (rocblas_int)R, R * tp, W.Ca, (rocblas_int)R,
                                            R * tp, first ? &zero : &one, Gp, tp, cc, S),
              "rocblas_dgemm_strided_batched (chunked Gram)");
      r0 += (int64_t)S * R;
    } else {
      if (first && S > 1) {   // fewer rows than one round: the partials are not used
        Gp = G;
      }
      k_rows_to64<<<chunk_grid(left, tp), kThreads, 0, s>>>(Q, n, r0, left, tp, W.Ca);
      FF_LAUNCH_CHECK("basis chunk to FP64");
      FF_BLAS(rocblas_dgemm(bh, rocblas_operation_transpose, rocblas_operation_none, tp, tp, (rocblas_int)left, &one,
                            W.Ca, (rocblas_int)left, W.Ca, (rocblas_int)left, first ? &zero : &one, Gp, tp),
              "rocblas_dgemm (chunked Gram)");
      r0 = n;
    }
    first = false;
  }
  if (Gp != G) {
    k_sum_slices<<<grid_for(cc), kThreads, 0, s>>>(Gp, S, cc, G);
    FF_LAUNCH_CHECK("Gram sum");
  }
  return FF_OK;
}

// Q <- Q Rinv over row chunks (Rinv upper triangular, lower part zero)
ff_status right_mult32(rocblas_handle bh, float *Q, int64_t n, int tp, const double *Rinv, RsvdWs32 &W,
                       hipStream_t s) {
  const double one = 1.0, zero = 0.0;
  for (int64_t r0 = 0; r0 < n; r0 += W.CH) {
    const int64_t rows = n - r0 < W.CH ? n - r0 : W.CH;
    k_rows_to64<<<chunk_grid(rows, tp), kThreads, 0, s>>>(Q, n, r0, rows, tp, W.Ca);
    FF_LAUNCH_CHECK("basis chunk to FP64");
    FF_BLAS(rocblas_dgemm(bh, rocblas_operation_none, rocblas_operation_none, (rocblas_int)rows, tp, tp, &one, W.Ca,
                          (rocblas_int)rows, Rinv, tp, &zero, W.Cb, (rocblas_int)rows),
            "rocblas_dgemm (chunked Q R^-1)");
    k_rows_to32<<<chunk_grid(rows, tp), kThreads, 0, s>>>(W.Cb, rows, tp, Q, n, r0);
    FF_LAUNCH_CHECK("basis chunk to FP32");
  }
  return FF_OK;
}

// The stored single-precision Q is orthonormal to about its own rounding; an attempt is
// accepted at max |Q^T Q - I| <= this bound.
constexpr double kDefect32 = 1e-6;

// One Cholesky QR attempt in place on the single-precision W.Q (as cholesky_qr, chunked).
ff_status cholesky_qr32(rocblas_handle bh, int64_t n, int tp, int passes, bool shift, RsvdWs32 &W, hipStream_t s,
                        bool *ok) {
  const rocblas_int c = tp;
  FF_HIP(hipMemsetAsync(W.info, 0, 8 * sizeof(rocblas_int), s));
  for (int p = 0; p < passes; ++p) {
    ff_status st = gram32(bh, W.Q, n, tp, W, W.Y, s);
    if (st) return st;
    if (p == 0 && shift) {
      k_gram_shift<<<1, kThreads, 0, s>>>(W.Y, c, n);
      FF_LAUNCH_CHECK("gram shift");
    }
    FF_BLAS(rocsolver_dpotrf(bh, rocblas_fill_upper, c, W.Y, c, W.info + 2 * p), "rocsolver_dpotrf");
    FF_BLAS(rocsolver_dtrtri(bh, rocblas_fill_upper, rocblas_diagonal_non_unit, c, W.Y, c, W.info + 2 * p + 1),
            "rocsolver_dtrtri");
    k_zero_lower<<<grid_for((int64_t)c * c, 256, 1 << 30), 256, 0, s>>>(W.Y, c);
    FF_LAUNCH_CHECK("zero lower");
    if ((st = right_mult32(bh, W.Q, n, tp, W.Y, W, s))) return st;
  }
  ff_status st = gram32(bh, W.Q, n, tp, W, W.Y, s);
  if (st) return st;
  FF_HIP(hipMemsetAsync(W.dev, 0, sizeof(double), s));
  k_orth_defect<<<c < 1024 ? c : 1024, kThreads, 0, s>>>(W.Y, c, (unsigned long long *)W.dev);
  FF_LAUNCH_CHECK("orthogonality check");
  struct {
    rocblas_int info[8];
    double defect;
  } hs;
  FF_HIP(hipMemcpyAsync(hs.info, W.info, sizeof(hs.info), hipMemcpyDeviceToHost, s));
  FF_HIP(hipMemcpyAsync(&hs.defect, W.dev, sizeof(double), hipMemcpyDeviceToHost, s));
  FF_HIP(hipStreamSynchronize(s));
  bool good = hs.defect <= kDefect32;
  for (int i = 0; i < 2 * passes; ++i) good = good && hs.info[i] == 0;
  *ok = good;
  return FF_OK;
}

// Orthonormal basis of the columns of the single-precision n x tp matrix W.Q, in place:
// CholeskyQR2, then shifted CholeskyQR3 on the kept input (as qr_inplace).  Householder QR, the
// last resort of the double-precision path, would need the FP64 matrix this variant avoids: if
// both Cholesky attempts fail the call fails (FF_ENOTIMPL).
ff_status qr32(ff_spectra h, rocblas_handle bh, int64_t n, int tp, RsvdWs32 &W, hipStream_t s) {
  if (h->rsvd_qr == 1)
    return fail(FF_ENOTIMPL, "rsvd_project: Householder QR needs FP64 basis storage (rsvd_qr = 1)");
  FF_HIP(hipMemcpyAsync(W.M, W.Q, sizeof(float) * n * tp, hipMemcpyDeviceToDevice, s));
  for (int attempt = h->rsvd_qr == 2 ? 1 : 0; attempt < 2; ++attempt) {
    if (attempt == 1) FF_HIP(hipMemcpyAsync(W.Q, W.M, sizeof(float) * n * tp, hipMemcpyDeviceToDevice, s));
    bool ok = false;
    ff_status st = cholesky_qr32(bh, n, tp, attempt == 0 ? 2 : 3, attempt == 1, W, s, &ok);
    if (st) return st;
    if (ok) {
      (attempt == 0 ? h->qr_cholesky2 : h->qr_cholesky3) += 1;
      return FF_OK;
    }
  }
  return fail(FF_ENOTIMPL, "rsvd_project: Cholesky QR of the single-precision basis failed; use FP64 storage");
}

// Algorithm 2 with the n x t_p matrices stored in single precision (see RsvdWs32); the steps
// are those of rsvd_run.
ff_status rsvd_run32(ff_spectra h, const double *rt, const double *wd, const double *winv, int t, int tp,
                     const double *omega, uint64_t seed, uint32_t stream, int power_iters, int mode, double *y,
                     double *alpha, double *sigma, void *ws, size_t ws_bytes, hipStream_t s) {
  const int64_t n = h->n, m = h->m;
  if (h->dtype != FF_F32) return fail(FF_EDTYPE, "rsvd_project: FP32 basis storage needs an FP32 handle");
  Arena ar{(char *)ws, ws_bytes, 0, false};
  RsvdWs32 W;
  W.carve(ar, n, m, tp);
  if (ar.used > ws_bytes) return fail(FF_ENOMEM, "rsvd_project: workspace too small");
  if (n > INT32_MAX) return fail(FF_ENOTIMPL, "rsvd_project: n exceeds the eigensolver's index range");
  const double fixed = *alpha;
  ff_status st;
  rocblas_handle bh = blas(h, s, &st);
  if (st) return st;
  // W^-1 as the post-weights of the products that produce the single-precision n x tp matrices
  k_to_f32<<<grid_for(n), kThreads, 0, s>>>(winv, n, W.winv32);
  if (!omega) {
    k_gaussian<<<grid_for((int64_t)tp * m), kThreads, 0, s>>>(W.Bm, (int64_t)tp * m, seed, stream);
    omega = W.Bm;
  }
  FF_LAUNCH_CHECK("rsvd setup");
  // Y^T = G~^T Omega^T (n x tp, stored FP32), Q = qr(Y^T)
  if ((st = op_apply_io(h, 1, tp, omega, m, W.Q, n, wd, W.winv32, FF_F64, FF_F32, s))) return st;
  if ((st = qr32(h, bh, n, tp, W, s))) return st;
  for (int q = 0; q < power_iters; ++q) {
    if ((st = op_apply_io(h, 0, tp, W.Q, n, W.Bm, m, W.winv32, wd, FF_F32, FF_F64, s))) return st;
    if ((st = qr_inplace(h, bh, W.Bm, m, tp, W.tau, W.T, W.U, W.Y, W.Gs, W.dev, W.info, s))) return st;
    if ((st = op_apply_io(h, 1, tp, W.Bm, m, W.Q, n, wd, W.winv32, FF_F64, FF_F32, s))) return st;
    if ((st = qr32(h, bh, n, tp, W, s))) return st;
  }
  // B = G~ Q
  if ((st = op_apply_io(h, 0, tp, W.Q, n, W.Bm, m, W.winv32, wd, FF_F32, FF_F64, s))) return st;
  const double one = 1.0, zero = 0.0;
  FF_BLAS(rocblas_dgemm(bh, rocblas_operation_transpose, rocblas_operation_none, tp, tp, (rocblas_int)m, &one, W.Bm,
                        (rocblas_int)m, W.Bm, (rocblas_int)m, &zero, W.Y, tp),
          "rocblas_dgemm");
  FF_BLAS(rocsolver_dsyevd(bh, rocblas_evect_original, rocblas_fill_lower, tp, W.Y, tp, W.lam, W.E, W.info),
          "rocsolver_dsyevd");
  k_rsvd_sort<<<(tp + 255) / 256, 256, 0, s>>>(W.lam, tp, W.S, W.perm);
  k_gather_cols<<<grid_for((int64_t)tp * t, 256, 1 << 30), 256, 0, s>>>(W.Y, tp, tp, W.perm, t, W.Vs);
  if ((st = gemv_t(W.Bm, m, m, tp, rt, W.btr, W.part, s))) return st;
  k_rsvd_coef<<<(t + 255) / 256, 256, 0, s>>>(W.Vs, tp, W.btr, W.S, t, W.c);
  UpreIn q{W.S, W.c, nullptr, 0, nullptr, t};
  if ((st = choose_alpha(h, mode, fixed, q, W.S, tp, W.alpha, s))) return st;
  k_filter<<<(t + 255) / 256, 256, 0, s>>>(W.S, W.alpha, q, t, W.g);
  if ((st = gemv_n(W.Vs, tp, tp, t, W.g, W.w, 1.0, s))) return st;
  launch_gemv_n<float>(W.Q, n, n, tp, W.w, y, 1.0, 0.0, s);
  FF_LAUNCH_CHECK("rsvd solution");
  FF_HIP(hipMemcpyAsync(sigma, W.S, sizeof(double) * tp, hipMemcpyDeviceToDevice, s));
  FF_HIP(hipMemcpyAsync(alpha, W.alpha, sizeof(double), hipMemcpyDeviceToHost, s));
  FF_HIP(hipStreamSynchronize(s));
  return FF_OK;
}

ff_status rsvd_run(ff_spectra h, const double *rt, const double *wd, const double *winv, int t, int tp,
                   const double *omega, uint64_t seed, uint32_t stream, int power_iters, int mode, double *y,
                   double *alpha, double *sigma, void *ws, size_t ws_bytes, hipStream_t s) {
  const int64_t n = h->n, m = h->m;
  Arena ar{(char *)ws, ws_bytes, 0, false};
  RsvdWs W;
  W.carve(ar, n, m, tp);
  if (ar.used > ws_bytes) return fail(FF_ENOMEM, "rsvd_project: workspace too small");
  if (n > INT32_MAX) return fail(FF_ENOTIMPL, "rsvd_project: n exceeds the eigensolver's index range");
  const double fixed = *alpha;
  ff_status st;
  rocblas_handle bh = blas(h, s, &st);
  if (st) return st;
  // Omega from the counter-based generator when not given (its tp x m values fill Bm, which
  // is not needed before the first product has read them)
  if (!omega) {
    k_gaussian<<<grid_for((int64_t)tp * m), kThreads, 0, s>>>(W.Bm, (int64_t)tp * m, seed, stream);
    FF_LAUNCH_CHECK("rsvd test matrix");
    omega = W.Bm;
  }
  // Y^T = G~^T Omega^T (n x tp), Q = qr(Y^T)
  if ((st = op_apply(h, 1, tp, omega, m, W.Q, n, wd, winv, FF_F64, s))) return st;
  if ((st = qr_inplace(h, bh, W.Q, n, tp, W.tau, W.T, W.U, W.Y, W.Gs, W.dev, W.info, s))) return st;
  for (int q = 0; q < power_iters; ++q) {
    // Y = G~ Q (m x tp), Q = qr(Y); Y^T = G~^T Q (n x tp), Q = qr(Y^T)
    if ((st = op_apply(h, 0, tp, W.Q, n, W.Bm, m, winv, wd, FF_F64, s))) return st;
    if ((st = qr_inplace(h, bh, W.Bm, m, tp, W.tau, W.T, W.U, W.Y, W.Gs, W.dev, W.info, s))) return st;
    if ((st = op_apply(h, 1, tp, W.Bm, m, W.Q, n, wd, winv, FF_F64, s))) return st;
    if ((st = qr_inplace(h, bh, W.Q, n, tp, W.tau, W.T, W.U, W.Y, W.Gs, W.dev, W.info, s))) return st;
  }
  // B = G~ Q
  if ((st = op_apply(h, 0, tp, W.Q, n, W.Bm, m, winv, wd, FF_F64, s))) return st;
  // B^T B (symmetric by construction of the product; the eigensolver reads one triangle,
  // which is the symmetrized (Y + Y^T)/2 of the algorithm up to rounding)
  const double one = 1.0, zero = 0.0;
  FF_BLAS(rocblas_dgemm(bh, rocblas_operation_transpose, rocblas_operation_none, tp, tp, (rocblas_int)m, &one, W.Bm,
                        (rocblas_int)m, W.Bm, (rocblas_int)m, &zero, W.Y, tp),
          "rocblas_dgemm");
  FF_BLAS(rocsolver_dsyevd(bh, rocblas_evect_original, rocblas_fill_lower, tp, W.Y, tp, W.lam, W.E, W.info),
          "rocsolver_dsyevd");
  k_rsvd_sort<<<(tp + 255) / 256, 256, 0, s>>>(W.lam, tp, W.S, W.perm);
  k_gather_cols<<<grid_for((int64_t)tp * t, 256, 1 << 30), 256, 0, s>>>(W.Y, tp, tp, W.perm, t, W.Vs);
  // B^T r~, c = U~^T (B^T r~)
  if ((st = gemv_t(W.Bm, m, m, tp, rt, W.btr, W.part, s))) return st;
  k_rsvd_coef<<<(t + 255) / 256, 256, 0, s>>>(W.Vs, tp, W.btr, W.S, t, W.c);
  UpreIn q{W.S, W.c, nullptr, 0, nullptr, t};
  if ((st = choose_alpha(h, mode, fixed, q, W.S, tp, W.alpha, s))) return st;
  // y = Q V~ Gamma(alpha) c
  k_filter<<<(t + 255) / 256, 256, 0, s>>>(W.S, W.alpha, q, t, W.g);
  if ((st = gemv_n(W.Vs, tp, tp, t, W.g, W.w, 1.0, s))) return st;
  if ((st = gemv_n(W.Q, n, n, tp, W.w, y, 1.0, s))) return st;
  FF_HIP(hipMemcpyAsync(sigma, W.S, sizeof(double) * tp, hipMemcpyDeviceToDevice, s));
  FF_HIP(hipMemcpyAsync(alpha, W.alpha, sizeof(double), hipMemcpyDeviceToHost, s));
  FF_HIP(hipStreamSynchronize(s));
  return FF_OK;
}

size_t irls_own_bytes(ff_spectra h, int tp) {
  Arena ar{nullptr, 0, 0, true};
  IrlsWs I;
  I.carve(ar, h->n, h->m, h->nz, tp);
  return ar.used + 256;
}

// bytes of a solver's workspace; the IRLS workspace is the solver's followed by the step's own
// (basis: FF_F64 or FF_F32 storage of the GKB bases)
size_t solver_bytes(ff_spectra h, int which, int solver, int basis, int tp) {
  Arena ar{nullptr, 0, 0, true};
  const int sol = which == FF_WS_IRLS ? solver : (which == FF_WS_RSVD ? 1 : 0);
  if (sol == 1 && basis == FF_F32) {
    RsvdWs32 W;
    W.carve(ar, h->n, h->m, tp);
  } else if (sol == 1) {
    RsvdWs W;
    W.carve(ar, h->n, h->m, tp);
  } else if (basis == FF_F32) {
    GkbWs<float> W;
    W.carve(ar, h->n, h->m, tp, gkb_acols(h, tp));
  } else {
    GkbWs<double> W;
    W.carve(ar, h->n, h->m, tp, gkb_acols(h, tp));
  }
  size_t b = ar.used + 256;
  if (which == FF_WS_IRLS) b += irls_own_bytes(h, tp);
  return b;
}

}  // namespace
}  // namespace ff

using namespace ff;

extern "C" {

ff_status ff_workspace_size(ff_spectra h, int32_t which, int32_t solver, int32_t basis_dtype, int32_t tp,
                            size_t *bytes) {
  if (!h || !bytes) return fail(FF_EINVAL, "ff_workspace_size: NULL argument");
  if (which < FF_WS_GKB || which > FF_WS_IRLS) return fail(FF_EINVAL, "ff_workspace_size: unknown solver");
  if (tp < 1 || tp > h->m) return fail(FF_ESHAPE, "ff_workspace_size: need 1 <= tp <= m");
  if (which == FF_WS_IRLS && solver != 0 && solver != 1) return fail(FF_EINVAL, "ff_workspace_size: solver must be 0 or 1");
  if (basis_dtype != FF_F64 && basis_dtype != FF_F32) return fail(FF_EDTYPE, "ff_workspace_size: basis dtype");
  *bytes = solver_bytes(h, which, solver, basis_dtype, tp);
  return FF_OK;
}

ff_status gkb_project(ff_spectra h, const double *r_tilde, const double *wd, const double *winv, int32_t t,
                      int32_t tp, int32_t alpha_mode, int32_t basis_dtype, double *y, double *alpha, double *sigma,
                      void *workspace, size_t ws_bytes, ff_stream stream) {
  ff_status st = check_solver_args("gkb_project", h, t, tp, r_tilde, wd, winv, y, alpha, sigma, workspace);
  if (st) return st;
  if (alpha_mode < 0 || alpha_mode > 2) return fail(FF_EINVAL, "gkb_project: alpha_mode must be 0, 1 or 2");
  if (basis_dtype == FF_F64)
    return gkb_run<double>(h, r_tilde, wd, winv, t, tp, alpha_mode, y, alpha, sigma, workspace, ws_bytes,
                           (hipStream_t)stream);
  if (basis_dtype == FF_F32)
    return gkb_run<float>(h, r_tilde, wd, winv, t, tp, alpha_mode, y, alpha, sigma, workspace, ws_bytes,
                          (hipStream_t)stream);
  return fail(FF_EDTYPE, "gkb_project: basis_dtype must be FF_F64 or FF_F32");
}

ff_status ff_solver_stats(ff_spectra h, int64_t *qr_cholesky2, int64_t *qr_cholesky3, int64_t *qr_householder) {
  if (!h || !qr_cholesky2 || !qr_cholesky3 || !qr_householder) return fail(FF_EINVAL, "ff_solver_stats: NULL argument");
  *qr_cholesky2 = h->qr_cholesky2;
  *qr_cholesky3 = h->qr_cholesky3;
  *qr_householder = h->qr_householder;
  return FF_OK;
}

ff_status rsvd_project(ff_spectra h, const double *r_tilde, const double *wd, const double *winv, int32_t t,
                       int32_t tp, const double *omega, uint64_t seed, int32_t power_iters, int32_t alpha_mode,
                       int32_t basis_dtype, double *y, double *alpha, double *sigma, void *workspace, size_t ws_bytes,
                       ff_stream stream) {
  ff_status st = check_solver_args("rsvd_project", h, t, tp, r_tilde, wd, winv, y, alpha, sigma, workspace);
  if (st) return st;
  if (power_iters < 0 || power_iters > kMaxPowerIters)
    return fail(FF_EINVAL, "rsvd_project: power_iters must lie in [0, 8]");
  if (alpha_mode < 0 || alpha_mode > 2) return fail(FF_EINVAL, "rsvd_project: alpha_mode must be 0, 1 or 2");
  if (basis_dtype != FF_F64 && basis_dtype != FF_F32)
    return fail(FF_EDTYPE, "rsvd_project: basis_dtype must be FF_F64 or FF_F32");
  if (basis_dtype == FF_F32)
    return rsvd_run32(h, r_tilde, wd, winv, t, tp, omega, seed, 0u, power_iters, alpha_mode, y, alpha, sigma,
                      workspace, ws_bytes, (hipStream_t)stream);
  return rsvd_run(h, r_tilde, wd, winv, t, tp, omega, seed, 0u, power_iters, alpha_mode, y, alpha, sigma, workspace,
                  ws_bytes, (hipStream_t)stream);
}

ff_status irls_step(ff_spectra h, const ff_irls_params *p, const double *d_obs, const double *wd,
                    const double *m_prev, const double *m_prev2, const double *omega, double *m_new, double *alpha,
                    double *chi2_scaled, void *workspace, size_t ws_bytes, ff_stream stream) {
  if (!h || !p || !d_obs || !wd || !m_prev || !m_new || !alpha || !chi2_scaled || !workspace)
    return fail(FF_EINVAL, "irls_step: NULL argument");
  if (p->k < 1) return fail(FF_EINVAL, "irls_step: k must be >= 1");
  if (p->k > 1 && !m_prev2) return fail(FF_EINVAL, "irls_step: m_prev2 is needed for k > 1");
  if (p->solver != 0 && p->solver != 1) return fail(FF_EINVAL, "irls_step: solver must be 0 (GKB) or 1 (RSVD)");
  if (p->solver == 1 && (p->power_iters < 0 || p->power_iters > kMaxPowerIters))
    return fail(FF_EINVAL, "irls_step: power_iters must lie in [0, 8]");
  if (!(p->eps2 > 0) || !(p->m_max >= p->m_min)) return fail(FF_EINVAL, "irls_step: need eps2 > 0, m_max >= m_min");
  if (p->t < 1 || p->tp < p->t || p->tp > h->m) return fail(FF_ESHAPE, "irls_step: need 1 <= t <= tp <= m");
  if (p->basis_dtype != FF_F64 && p->basis_dtype != FF_F32)
    return fail(FF_EDTYPE, "irls_step: basis_dtype must be FF_F64 or FF_F32");
  int cur = -1;
  hipGetDevice(&cur);
  if (cur != h->device) return fail(FF_EDEVICE, "irls_step: current device differs from the handle's device");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = h->n, m = h->m;
  const size_t need = solver_bytes(h, FF_WS_IRLS, p->solver, p->basis_dtype, p->tp);
  if (ws_bytes < need) return fail(FF_ENOMEM, "irls_step: workspace too small");
  // the solver's workspace first, the step's own vectors after it
  const size_t sol = solver_bytes(h, p->solver == 1 ? FF_WS_RSVD : FF_WS_GKB, 0, p->basis_dtype, p->tp);
  Arena ar{(char *)workspace + sol, ws_bytes - sol, 0, false};
  IrlsWs I;
  I.carve(ar, n, m, h->nz, p->tp);
  if (sol + ar.used > ws_bytes) return fail(FF_ENOMEM, "irls_step: workspace too small");
  // depth weights per layer: (mid-depth)^(-beta)
  std::vector<double> zw(h->nz);
  for (int r = 0; r < h->nz; ++r) zw[r] = std::pow(0.5 * (h->z_edges[r] + h->z_edges[r + 1]), -p->beta_depth);
  FF_HIP(hipMemcpyAsync(I.zw, zw.data(), sizeof(double) * h->nz, hipMemcpyHostToDevice, s));
  k_irls_winv<<<grid_for(n), kThreads, 0, s>>>(I.zw, (int64_t)h->nx * h->ny, n, m_prev, m_prev2, p->k, p->lambda,
                                                p->eps2, I.winv);
  // r~ = wd (d_obs - G m_prev)
  ff_status st;
  if ((st = op_apply(h, 0, 1, m_prev, n, I.gm, m, nullptr, nullptr, FF_F64, s))) return st;
  k_residual<<<grid_for(m), kThreads, 0, s>>>(wd, d_obs, I.gm, m, I.r);
  FF_LAUNCH_CHECK("irls_step setup");
  {
    // a non-finite r~ (NaN or Inf in d_obs, wd or m_prev) is rejected before the solve
    if ((st = norm2(I.r, m, I.nrm, nullptr, I.part, s))) return st;
    double r0 = 0.0;
    FF_HIP(hipMemcpyAsync(&r0, I.nrm, sizeof(double), hipMemcpyDeviceToHost, s));
    FF_HIP(hipStreamSynchronize(s));
    if (!std::isfinite(r0)) return fail(FF_EINVAL, "irls_step: non-finite residual (NaN or Inf in d_obs, wd or m_prev)");
  }
  const int mode = p->alpha_fixed > 0 ? ALPHA_FIXED : (p->k == 1 ? ALPHA_ONE : ALPHA_UPRE);
  double a = p->alpha_fixed;
  // the solvers synchronize the stream before returning, so zw (host) has been consumed
  if (p->solver == 0)
    st = p->basis_dtype == FF_F32 ? gkb_run<float>(h, I.r, wd, I.winv, p->t, p->tp, mode, I.y, &a, I.sig, workspace, sol, s)
                                  : gkb_run<double>(h, I.r, wd, I.winv, p->t, p->tp, mode, I.y, &a, I.sig, workspace, sol, s);
  else if (p->basis_dtype == FF_F32)
    st = rsvd_run32(h, I.r, wd, I.winv, p->t, p->tp, omega, p->seed, (uint32_t)p->k, p->power_iters, mode, I.y, &a,
                    I.sig, workspace, sol, s);
  else
    st = rsvd_run(h, I.r, wd, I.winv, p->t, p->tp, omega, p->seed, (uint32_t)p->k, p->power_iters, mode, I.y, &a,
                  I.sig, workspace, sol, s);
  if (st) return st;
  // m^(k) = clip(m^(k-1) + W^{-1} y), then the scaled chi^2 of the clipped iterate
  k_update_clip<<<grid_for(n), kThreads, 0, s>>>(m_prev, I.winv, I.y, n, p->m_min, p->m_max, m_new);
  if ((st = op_apply(h, 0, 1, m_new, n, I.gm, m, nullptr, nullptr, FF_F64, s))) return st;
  k_residual<<<grid_for(m), kThreads, 0, s>>>(wd, d_obs, I.gm, m, I.r);
  if ((st = norm2(I.r, m, I.nrm, nullptr, I.part, s))) return st;
  double nrm = 0.0;
  FF_HIP(hipMemcpyAsync(&nrm, I.nrm, sizeof(double), hipMemcpyDeviceToHost, s));
  FF_HIP(hipStreamSynchronize(s));
  *alpha = a;
  *chi2_scaled = nrm * nrm / ((double)m + std::sqrt(2.0 * (double)m));
  if (!std::isfinite(*chi2_scaled) || !std::isfinite(a))
    return fail(FF_EINVAL, "irls_step: the step produced non-finite values");
  return FF_OK;
}

}  // extern "C"

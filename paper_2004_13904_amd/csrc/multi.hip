// Several surveys applied together: every survey's G and G^T passes run in three grouped
// launches (all row transforms, all column passes, all inverse row transforms) instead of six
// launches per survey.  A survey alone is a chain of small, latency-bound kernels; grouped, the
// chains of all surveys share each launch's ramp and fill the chip together.
//
// Block b of a launch finds its task (survey and product) in a table of first-block indices and
// runs the same pass body as the per-survey kernels for that task's transform length.  The row
// passes take 2048/N transforms per 256-thread block for every N up to 512; the column passes
// have 8 wave groups of 64 threads (512 threads) for every NY up to 512.
#include <algorithm>
#include <new>
#include <vector>

#include "passes.h"

namespace ff {
namespace {

constexpr int kMultiThreads = 512;      // column blocks
constexpr int kMultiRowThreads = 256;   // row blocks
constexpr int kMultiMaxN = 512;     // largest embedding side of a grouped survey

template <int N> struct MultiRow {
  static constexpr int NF = 8 * kMultiRowThreads / N;
  using C = RowCfg<float, N, NF>;
  static_assert(C::THREADS == kMultiRowThreads, "grouped row blocks have kMultiRowThreads threads");
};

template <int NY> struct MultiCol {
  using CC = ColCfg<float, NY>;
  static_assert(CC::THREADS * CC::WPB == kMultiThreads, "grouped column blocks have 512 threads");
  static constexpr int SH = CC::WPB * CC::CPB * FFT<float, NY, false>::LDS;
  static constexpr int SHP = SH > PairCfg<float, NY>::SH ? SH : PairCfg<float, NY>::SH;
};

constexpr int max3(int a, int b, int c) { return a > b ? (a > c ? a : c) : (b > c ? b : c); }
constexpr int kRowSH = max3(max3(MultiRow<8>::C::SH, MultiRow<16>::C::SH, MultiRow<32>::C::SH),
                            max3(MultiRow<64>::C::SH, MultiRow<128>::C::SH, MultiRow<256>::C::SH),
                            MultiRow<512>::C::SH);
constexpr int kColSH = max3(max3(MultiCol<8>::SH, MultiCol<16>::SH, MultiCol<32>::SH),
                            max3(MultiCol<64>::SH, MultiCol<128>::SH, MultiCol<256>::SH), MultiCol<512>::SH);
// the pair's column pass keeps two exchange buffers per wave group and the shared transform of
// the data column (about 76 KB at 512 points); plans without pair tasks keep the smaller blocks
constexpr int kColPairSH = max3(max3(MultiCol<8>::SHP, MultiCol<16>::SHP, MultiCol<32>::SHP),
                                max3(MultiCol<64>::SHP, MultiCol<128>::SHP, MultiCol<256>::SHP), MultiCol<512>::SHP);

// Row transforms of one product of one survey (pass 1), arguments as k_row_r2c's.
struct R2CTask {
  int block0, N;
  const float *in;
  Idx3 ii;
  int nrows, nb, len, off;
  float2 *out;
  Idx3 oi;
  int64_t out_kx;
  const float2 *tw;
};

// Inverse row transforms (pass 3), arguments as k_row_c2r's.
struct C2RTask {
  int block0, N;
  const float2 *in;
  Idx3 ii;
  int64_t in_kx, pstride;
  int P, nrows, nb;
  float *out;
  Idx3 oi;
  int len, off;
  const float2 *tw;
};

// Column pass (pass 2) of G (op 0), of G^T (op 1), or of both products of one survey with one
// read of the spectra (op 2, col_pair_body), arguments as k_col_G's / k_col_GT's; the task's
// blocks are nbx column blocks times LG layer groups.
struct ColTask {
  int block0, NY, op, nbx;
  const float2 *src;       // G and the pair: X1; G^T: D1
  float2 *dst;             // G and the pair: partial sums; G^T: X1
  int ny, ldy, nz, HC, LG, sy, lds, pyl;
  const float2 *spec, *tw;
  const float2 *src2;      // the pair: G^T's D1
  float2 *dst2;            // the pair: G^T's X1
};

template <class Task> __device__ __forceinline__ int find_task(const Task *__restrict__ t, int nt) {
  int i = 0;
  while (i + 1 < nt && t[i + 1].block0 <= (int)blockIdx.x) ++i;
  return i;
}

template <int N> __device__ __forceinline__ void r2c_task(float2 *sh, int lb, const R2CTask &t) {
  row_r2c_body<float, float, N, MultiRow<N>::NF, true>(sh, lb, 0, 0, t.in, t.ii, nullptr, Idx3{0, 0, 0}, t.nrows,
                                                      t.nb, t.len, t.off, t.out, t.oi, t.out_kx, t.tw);
}

template <int N> __device__ __forceinline__ void c2r_task(float2 *sh, int lb, const C2RTask &t) {
  row_c2r_body<float, float, N, MultiRow<N>::NF>(sh, lb, 0, 0, t.in, t.ii, t.in_kx, t.pstride, t.P, t.nrows, t.nb,
                                                 t.out, t.oi, nullptr, Idx3{0, 0, 0}, t.len, t.off, t.tw);
}

template <int NY, bool PAIR> __device__ __forceinline__ void col_task(float2 *sh, int lb, const ColTask &t) {
  const int bx = lb % t.nbx, by = lb / t.nbx;
  if (PAIR && t.op == 2) {
    if (2 * t.ny <= NY && 2 * (t.pyl + t.sy) <= NY)
      col_pair_body<float, NY, true>(sh, bx, by, t.src, t.ny, t.ldy, t.dst, t.src2, t.dst2, t.sy, t.lds, t.pyl,
                                     t.nz, t.HC, t.LG, t.spec, t.tw);
    else
      col_pair_body<float, NY, false>(sh, bx, by, t.src, t.ny, t.ldy, t.dst, t.src2, t.dst2, t.sy, t.lds, t.pyl,
                                      t.nz, t.HC, t.LG, t.spec, t.tw);
  }
  else if (t.op == 0) {
    if (2 * t.ny <= NY && 2 * (t.pyl + t.sy) <= NY)
      col_G_body<float, NY, true>(sh, bx, by, 0, t.src, t.ny, t.ldy, t.nz, t.HC, t.LG, t.spec, t.dst, t.sy, t.lds,
                                  t.pyl, t.tw);
    else
      col_G_body<float, NY, false>(sh, bx, by, 0, t.src, t.ny, t.ldy, t.nz, t.HC, t.LG, t.spec, t.dst, t.sy, t.lds,
                                   t.pyl, t.tw);
  } else {
    if (2 * t.ny <= NY && 2 * (t.pyl + t.sy) <= NY)
      col_GT_body<float, NY, true>(sh, bx, by, 0, t.src, t.sy, t.lds, t.pyl, t.nz, t.HC, t.LG, t.spec, t.dst, t.ny,
                                   t.ldy, t.tw);
    else
      col_GT_body<float, NY, false>(sh, bx, by, 0, t.src, t.sy, t.lds, t.pyl, t.nz, t.HC, t.LG, t.spec, t.dst, t.ny,
                                    t.ldy, t.tw);
  }
}

#define FF_MULTI_SWITCH(N, CALL)                                                                             \
  switch (N) {                                                                                               \
    case 8: CALL(8); break;                                                                                  \
    case 16: CALL(16); break;                                                                                \
    case 32: CALL(32); break;                                                                                \
    case 64: CALL(64); break;                                                                                \
    case 128: CALL(128); break;                                                                              \
    case 256: CALL(256); break;                                                                              \
    case 512: CALL(512); break;                                                                              \
    default: break;                                                                                          \
  }

__global__ void __launch_bounds__(kMultiRowThreads) k_multi_r2c(const R2CTask *__restrict__ tasks, int nt) {
  __shared__ float2 sh[kRowSH];
  const R2CTask &t = tasks[find_task(tasks, nt)];
  const int lb = (int)blockIdx.x - t.block0;
#define FF_R2C(NN) r2c_task<NN>(sh, lb, t)
  FF_MULTI_SWITCH(t.N, FF_R2C)
#undef FF_R2C
}

__global__ void __launch_bounds__(kMultiThreads) k_multi_col(const ColTask *__restrict__ tasks, int nt) {
  __shared__ float2 sh[kColSH];
  const ColTask &t = tasks[find_task(tasks, nt)];
  const int lb = (int)blockIdx.x - t.block0;
#define FF_COL(NN) col_task<NN, false>(sh, lb, t)
  FF_MULTI_SWITCH(t.NY, FF_COL)
#undef FF_COL
}

__global__ void __launch_bounds__(kMultiThreads) k_multi_col_pair(const ColTask *__restrict__ tasks, int nt) {
  __shared__ float2 sh[kColPairSH];
  const ColTask &t = tasks[find_task(tasks, nt)];
  const int lb = (int)blockIdx.x - t.block0;
#define FF_COL(NN) col_task<NN, true>(sh, lb, t)
  FF_MULTI_SWITCH(t.NY, FF_COL)
#undef FF_COL
}

__global__ void __launch_bounds__(kMultiRowThreads) k_multi_c2r(const C2RTask *__restrict__ tasks, int nt) {
  __shared__ float2 sh[kRowSH];
  const C2RTask &t = tasks[find_task(tasks, nt)];
  const int lb = (int)blockIdx.x - t.block0;
#define FF_C2R(NN) c2r_task<NN>(sh, lb, t)
  FF_MULTI_SWITCH(t.N, FF_C2R)
#undef FF_C2R
}

constexpr int MultiRowNF(int N) { return 8 * kMultiRowThreads / N; }
int rows_per_block(int N) { return 2 * MultiRowNF(N); }
int col_blocks_x(int NY, int HC) {
  const int tpf = NY / 8, cpb = tpf >= 64 ? 1 : 64 / tpf;
  return (HC + cpb - 1) / cpb;
}

}  // namespace
}  // namespace ff

using namespace ff;

struct ff_multi_s {
  int device = 0;
  int n_r2c = 0, n_col = 0, n_c2r = 0;          // tasks per launch
  int b_r2c = 0, b_col = 0, b_c2r = 0;          // blocks per launch
  bool col_pair = false;                        // the column launch holds a pair task
  R2CTask *r2c = nullptr;
  ColTask *col = nullptr;
  C2RTask *c2r = nullptr;
};

namespace {

void launch_col(ff_multi p, hipStream_t s) {
  if (!p->n_col) return;
  if (p->col_pair)
    k_multi_col_pair<<<p->b_col, kMultiThreads, 0, s>>>(p->col, p->n_col);
  else
    k_multi_col<<<p->b_col, kMultiThreads, 0, s>>>(p->col, p->n_col);
}

void free_plan(ff_multi p) {
  if (!p) return;
  hipFree(p->r2c);
  hipFree(p->col);
  hipFree(p->c2r);
  delete p;
}

template <class Task> ff_status upload(const std::vector<Task> &v, Task **dst) {
  if (v.empty()) return FF_OK;
  if (hipMalloc((void **)dst, sizeof(Task) * v.size()) != hipSuccess)
    return fail(FF_ENOMEM, "ff_multi_create: device allocation failed");
  if (hipMemcpy(*dst, v.data(), sizeof(Task) * v.size(), hipMemcpyHostToDevice) != hipSuccess)
    return fail(FF_EHIP, "ff_multi_create: table upload failed");
  return FF_OK;
}

}  // namespace

extern "C" {

ff_status ff_multi_create(int32_t count, const ff_spectra *handles, const void *const *x, void *const *gx,
                          const void *const *d, void *const *gtd, ff_multi *out) {
  if (!out) return fail(FF_EINVAL, "ff_multi_create: NULL output");
  *out = nullptr;
  if (count < 1 || !handles) return fail(FF_EINVAL, "ff_multi_create: need at least one handle");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FF_EHIP, "ff_multi_create: no HIP device");
  std::vector<R2CTask> r2c;
  std::vector<ColTask> col;
  std::vector<C2RTask> c2r;
  int b_r2c = 0, b_col = 0, b_c2r = 0;
  bool any_pair = false;
  for (int i = 0; i < count; ++i) {
    const ff_spectra h = handles[i];
    if (!h) return fail(FF_EINVAL, "ff_multi_create: NULL handle");
    for (int k = 0; k < i; ++k)
      if (handles[k] == h) return fail(FF_EINVAL, "ff_multi_create: a handle appears twice");
    if (h->device != dev) return fail(FF_EDEVICE, "ff_multi_create: handle on another device");
    if (h->dtype != FF_F32) return fail(FF_EDTYPE, "ff_multi_create: single-precision handles only");
    if (h->NX > kMultiMaxN || h->NY > kMultiMaxN)
      return fail(FF_ENOTIMPL, "ff_multi_create: embedding larger than 512 x 512");
    const bool doG = x && gx && x[i] && gx[i], doT = d && gtd && d[i] && gtd[i];
    if ((x && gx) && (!x[i]) != (!gx[i])) return fail(FF_EINVAL, "ff_multi_create: x and gx must both be set");
    if ((d && gtd) && (!d[i]) != (!gtd[i])) return fail(FF_EINVAL, "ff_multi_create: d and gtd must both be set");
    const int HC = h->NX / 2, nz = h->nz, nx = h->nx, ny = h->ny, sx = h->sx, sy = h->sy;
    const int ldy = h->ldy, lds = h->lds;
    const int64_t lay = (int64_t)ny * nx;
    // G uses vector slot 0 of the pass workspaces, G^T slot 1, so both run in the same launches
    const size_t need_rows = sizeof(float2) * 2 * (size_t)nz * HC * ldy;
    const size_t need_cols = sizeof(float2) * 2 * (size_t)nz * HC * lds;
    if (h->ws_rows_bytes < need_rows || h->ws_cols_bytes < need_cols || h->lg_G > nz)
      return fail(FF_ENOTIMPL, "ff_multi_create: pass workspace too small for a grouped apply");
    float2 *X1 = (float2 *)h->ws_rows, *C2 = (float2 *)h->ws_cols;
    float2 *X1t = X1 + (size_t)nz * HC * ldy, *C2t = C2 + (size_t)nz * HC * lds;
    const float2 *twx = (const float2 *)h->tw_x, *twy = (const float2 *)h->tw_y;
    const float2 *spec = (const float2 *)h->spec;
    const int rpb = rows_per_block(h->NX), nbx = col_blocks_x(h->NY, HC);
    // a pair task halves the column blocks of the two products and needs more LDS per block: by
    // default (pair_fused = 1) it is used for a single survey whose pair alone fills the chip
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    const bool pair = doG && doT && (h->pair_fused == 2 || (h->pair_fused == 1 && count == 1 && nbx * h->lg_G >= cus));
    any_pair = any_pair || pair;
    if (pair) {
      // one column task for both products: each spectrum column is read once
      ColTask c{b_col, h->NY, 2, nbx, X1, C2, ny, ldy, nz, HC, h->lg_G, sy, lds, h->pyl, spec, twy, C2t, X1t};
      col.push_back(c);
      b_col += nbx * h->lg_G;
    }
    if (doG) {
      R2CTask a{b_r2c, h->NX, (const float *)x[i], Idx3{0, lay, nx}, ny, nz, nx, 0, X1, Idx3{0, (int64_t)HC * ldy, 1},
                ldy, twx};
      r2c.push_back(a);
      b_r2c += row_blocks(ny, nz, rpb);
      if (!pair) {
        ColTask c{b_col, h->NY, 0, nbx, X1, C2, ny, ldy, nz, HC, h->lg_G, sy, lds, h->pyl, spec, twy, nullptr, nullptr};
        col.push_back(c);
        b_col += nbx * h->lg_G;
      }
      C2RTask e{b_c2r, h->NX, C2, Idx3{0, 0, 1}, lds, (int64_t)HC * lds, h->lg_G, sy, 1, (float *)gx[i],
                Idx3{0, 0, sx}, sx, h->pxl, twx};
      c2r.push_back(e);
      b_c2r += row_blocks(sy, 1, rpb);
    }
    if (doT) {
      R2CTask a{b_r2c, h->NX, (const float *)d[i], Idx3{0, 0, sx}, sy, 1, sx, h->pxl, C2t, Idx3{0, 0, 1}, lds, twx};
      r2c.push_back(a);
      b_r2c += row_blocks(sy, 1, rpb);
      if (!pair) {
        ColTask c{b_col, h->NY, 1, nbx, C2t, X1t, ny, ldy, nz, HC, h->lg_GT, sy, lds, h->pyl, spec, twy, nullptr,
                  nullptr};
        col.push_back(c);
        b_col += nbx * h->lg_GT;
      }
      C2RTask e{b_c2r, h->NX, X1t, Idx3{0, (int64_t)HC * ldy, 1}, ldy, 0, 1, ny, nz, (float *)gtd[i],
                Idx3{0, lay, nx}, nx, 0, twx};
      c2r.push_back(e);
      b_c2r += row_blocks(ny, nz, rpb);
    }
  }
  ff_multi p = new (std::nothrow) ff_multi_s();
  if (!p) return fail(FF_ENOMEM, "ff_multi_create: host allocation failed");
  p->device = dev;
  p->n_r2c = (int)r2c.size();
  p->n_col = (int)col.size();
  p->n_c2r = (int)c2r.size();
  p->b_r2c = b_r2c;
  p->b_col = b_col;
  p->b_c2r = b_c2r;
  p->col_pair = any_pair;
  ff_status st = upload(r2c, &p->r2c);
  if (st == FF_OK) st = upload(col, &p->col);
  if (st == FF_OK) st = upload(c2r, &p->c2r);
  if (st != FF_OK) {
    free_plan(p);
    return st;
  }
  *out = p;
  return FF_OK;
}

ff_status ff_multi_apply(ff_multi p, ff_stream stream) {
  if (!p) return fail(FF_EINVAL, "ff_multi_apply: NULL plan");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(FF_EDEVICE, "ff_multi_apply: plan built on another device");
  hipStream_t s = (hipStream_t)stream;
  if (p->n_r2c) k_multi_r2c<<<p->b_r2c, kMultiRowThreads, 0, s>>>(p->r2c, p->n_r2c);
  FF_LAUNCH_CHECK("grouped row transforms");
  launch_col(p, s);
  FF_LAUNCH_CHECK("grouped column passes");
  if (p->n_c2r) k_multi_c2r<<<p->b_c2r, kMultiRowThreads, 0, s>>>(p->c2r, p->n_c2r);
  FF_LAUNCH_CHECK("grouped inverse row transforms");
  return FF_OK;
}

ff_status ff_multi_time_pass(ff_multi p, int32_t pass, int32_t reps, ff_stream stream) {
  if (!p) return fail(FF_EINVAL, "ff_multi_time_pass: NULL plan");
  if (pass < 0 || pass > 2 || reps < 0) return fail(FF_EINVAL, "ff_multi_time_pass: pass in {0,1,2}, reps >= 0");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(FF_EDEVICE, "ff_multi_time_pass: plan built on another device");
  hipStream_t s = (hipStream_t)stream;
  for (int r = 0; r < reps; ++r) {
    if (pass == 0 && p->n_r2c) k_multi_r2c<<<p->b_r2c, kMultiRowThreads, 0, s>>>(p->r2c, p->n_r2c);
    if (pass == 1) launch_col(p, s);
    if (pass == 2 && p->n_c2r) k_multi_c2r<<<p->b_c2r, kMultiRowThreads, 0, s>>>(p->c2r, p->n_c2r);
  }
  FF_LAUNCH_CHECK("ff_multi_time_pass");
  return FF_OK;
}

ff_status ff_multi_free(ff_multi p) {
  if (!p) return FF_OK;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(p->device);
  free_plan(p);
  hipSetDevice(cur);
  return FF_OK;
}

}  // extern "C"

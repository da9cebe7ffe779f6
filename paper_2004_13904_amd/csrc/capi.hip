// C ABI entry points: argument validation, handle lifetime and error reporting.  Every
// failure is reported as a negative status plus a thread-local message; nothing throws
// across the boundary.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"

namespace ff {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

ff_status fail(ff_status code, const std::string &msg) {
  g_err = msg;
  return code;
}

ff_status hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return FF_EHIP;
}

size_t csize(int dtype) { return dtype == FF_F64 ? sizeof(double2) : sizeof(float2); }

namespace {

int next_pow2(int64_t v) {
  int p = 8;
  while (p < v) p *= 2;
  return p;
}

void prof_release(ff_spectra h) {
  for (hipEvent_t e : h->prof_ev) hipEventDestroy(e);
  h->prof_ev.clear();
  h->prof_kind.clear();
  h->prof_cap = h->prof_n = 0;
  h->prof_cur = -1;
}

void free_handle(ff_spectra h) {
  if (!h) return;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(h->device);
  prof_release(h);
  hipFree(h->spec);
  hipFree(h->tw_x);
  hipFree(h->tw_y);
  hipFree(h->z_dev);
  hipFree(h->ws_rows);
  hipFree(h->ws_cols);
  if (h->gkb_exec) hipGraphExecDestroy((hipGraphExec_t)h->gkb_exec);
  if (h->cap_stream) hipStreamDestroy(h->cap_stream);
  release_blas(h);
  hipSetDevice(cur);
  delete h;
}

ff_status check_device(ff_spectra h) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(FF_EHIP, "hipGetDevice failed");
  if (cur != h->device) return fail(FF_EDEVICE, "current device differs from the handle's device");
  return FF_OK;
}

template <typename T> ff_status upload_twiddles(int N, void **dst) {
  std::vector<cplx<T>> tw(N);
  for (int e = 0; e < N; ++e) {
    // exp(-2 pi i e / N) evaluated in double and rounded once
    const double a = 2.0 * M_PI * (double)e / (double)N;
    tw[e] = mk<T>((T)std::cos(a), (T)-std::sin(a));
  }
  if (hipMalloc(dst, sizeof(cplx<T>) * N) != hipSuccess) return fail(FF_ENOMEM, "twiddle table allocation failed");
  if (hipMemcpy(*dst, tw.data(), sizeof(cplx<T>) * N, hipMemcpyHostToDevice) != hipSuccess)
    return fail(FF_EHIP, "twiddle table upload failed");
  return FF_OK;
}

int column_blocks(int H, int NY) {
  const int tpf = NY / 8;
  const int cpb = tpf >= 64 ? 1 : 64 / tpf;
  return (H + cpb - 1) / cpb;
}

// Validates the geometry, fills the handle's fields and allocates its device memory and
// twiddle tables; the spectra are left to the caller (computed or loaded).
ff_status create_handle(const ff_geometry *g, int32_t dtype, const std::string &who, ff_spectra *out) {
  if (!g || !out) return fail(FF_EINVAL, who + ": NULL geometry or output");
  *out = nullptr;
  if (dtype != FF_F32 && dtype != FF_F64) return fail(FF_EDTYPE, who + ": dtype must be FF_F32 or FF_F64");
  if (g->sx < 1 || g->sy < 1 || g->nz < 1) return fail(FF_ESHAPE, who + ": sx, sy, nz must be >= 1");
  if (g->pad_xl < 0 || g->pad_xr < 0 || g->pad_yl < 0 || g->pad_yr < 0)
    return fail(FF_ESHAPE, who + ": negative padding");
  if (!(g->dx > 0) || !(g->dy > 0) || !std::isfinite(g->dx) || !std::isfinite(g->dy))
    return fail(FF_EINVAL, who + ": dx, dy must be positive and finite");
  if (!g->z_edges) return fail(FF_EINVAL, who + ": z_edges is NULL");
  if (g->z_edges[0] != 0.0) return fail(FF_EINVAL, who + ": z_edges[0] must be 0 (station plane)");
  for (int r = 0; r < g->nz; ++r)
    if (!(g->z_edges[r + 1] > g->z_edges[r]) || !std::isfinite(g->z_edges[r + 1]))
      return fail(FF_EINVAL, who + ": z_edges must increase strictly");
  if (g->kernel != FF_GRAVITY_GZ && g->kernel != FF_MAGNETIC_TFA)
    return fail(FF_EINVAL, who + ": unknown kernel");
  if (g->kernel == FF_MAGNETIC_TFA &&
      (!std::isfinite(g->incl_deg) || !std::isfinite(g->decl_deg) || !std::isfinite(g->field_nT)))
    return fail(FF_EINVAL, who + ": magnetic field parameters must be finite");
  const int64_t nx = (int64_t)g->sx + g->pad_xl + g->pad_xr;
  const int64_t ny = (int64_t)g->sy + g->pad_yl + g->pad_yr;
  const int64_t minx = g->sx + nx - 1, miny = g->sy + ny - 1;
  if (minx > 2048 || miny > 2048) return fail(FF_ENOTIMPL, who + ": embedding would exceed 2048");
  int NX = g->nfft_x, NY = g->nfft_y;
  if (NX == 0) NX = next_pow2(minx);
  if (NY == 0) NY = next_pow2(miny);
  if (!is_pow2(NX) || !is_pow2(NY) || NX < 8 || NY < 8 || NX > 2048 || NY > 2048)
    return fail(FF_ENOTIMPL, who + ": embedding sizes must be powers of two in [8, 2048]");
  if (NX < minx || NY < miny)
    return fail(FF_ESHAPE, who + ": embedding smaller than s + n - 1 would wrap around");

  ff_spectra h = new (std::nothrow) ff_spectra_s();
  if (!h) return fail(FF_ENOMEM, who + ": host allocation failed");
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(FF_EHIP, who + ": no HIP device");
  }
  h->dtype = dtype;
  h->sx = g->sx; h->sy = g->sy; h->nz = g->nz;
  h->pxl = g->pad_xl; h->pxr = g->pad_xr; h->pyl = g->pad_yl; h->pyr = g->pad_yr;
  h->nx = (int)nx; h->ny = (int)ny;
  h->dx = g->dx; h->dy = g->dy;
  h->incl = g->incl_deg; h->decl = g->decl_deg; h->field = g->field_nT;
  h->kernel = g->kernel;
  h->z_edges.assign(g->z_edges, g->z_edges + g->nz + 1);
  h->NX = NX; h->NY = NY; h->H = NX / 2 + 1;
  // intermediate columns start on 128-byte (complex64) boundaries
  h->ldy = (h->ny + 15) / 16 * 16;
  h->lds = (h->sy + 15) / 16 * 16;
  h->m = (int64_t)g->sx * g->sy;
  h->n = nx * ny * g->nz;
  // Layer groups across blocks of the column passes: enough wavefronts to fill the chip
  // (about 2048), while every group keeps at least one layer per wave group of its block.
  const int cb = column_blocks(NX / 2, NY);   // NX/2 packed column slots
  const int wpb = col_wave_groups(dtype, NY);
  int lg = (2048 + cb * wpb - 1) / (cb * wpb);
  const int lgmax_layers = h->nz / wpb > 0 ? h->nz / wpb : 1;
  if (lg > lgmax_layers) lg = lgmax_layers;
  if (lg < 1) lg = 1;
  h->lg_G = lg;
  h->lg_GT = lg;

  const size_t cs = csize(dtype);
  const int64_t rows = h->ldy > h->lds ? h->ldy : h->lds;
  const size_t per_vec = cs * (size_t)h->nz * (NX / 2) * rows;   // row-pass intermediates of a vector
  size_t b = kBatchBytes / per_vec;
  b = b < (size_t)kMinBatch ? kMinBatch : b > (size_t)kMaxBatch ? kMaxBatch : b;
  h->batch = (int)(b / 4 * 4);
  h->batch_max = h->batch;
  h->ws_rows_bytes = cs * (size_t)h->batch * h->nz * h->H * rows;
  // room for the G partial sums of up to nz layer groups (ff_set_tuning may raise lg_G)
  h->ws_cols_bytes = cs * (size_t)h->batch * h->nz * h->H * h->lds;
  ff_status st = FF_OK;
  if (hipMalloc(&h->spec, cs * (size_t)h->nz * h->H * NY) != hipSuccess ||
      hipMalloc(&h->ws_rows, h->ws_rows_bytes) != hipSuccess ||
      hipMalloc(&h->ws_cols, h->ws_cols_bytes) != hipSuccess ||
      hipMalloc((void **)&h->z_dev, sizeof(double) * (h->nz + 1)) != hipSuccess) {
    free_handle(h);
    return fail(FF_ENOMEM, who + ": device allocation failed");
  }
  if (hipMemcpy(h->z_dev, g->z_edges, sizeof(double) * (h->nz + 1), hipMemcpyHostToDevice) != hipSuccess) {
    free_handle(h);
    return fail(FF_EHIP, who + ": z_edges upload failed");
  }
  st = dtype == FF_F32 ? upload_twiddles<float>(NX, &h->tw_x) : upload_twiddles<double>(NX, &h->tw_x);
  if (st == FF_OK) st = dtype == FF_F32 ? upload_twiddles<float>(NY, &h->tw_y) : upload_twiddles<double>(NY, &h->tw_y);
  if (st != FF_OK) {
    std::string msg = g_err;
    free_handle(h);
    return fail(st, msg);
  }
  *out = h;
  return FF_OK;
}

}  // namespace
}  // namespace ff

using namespace ff;

extern "C" {

const char *ff_last_error(void) { return g_err.c_str(); }

ff_status build_spectra(const ff_geometry *g, int32_t dtype, ff_stream stream, ff_spectra *out) {
  ff_spectra h = nullptr;
  ff_status st = create_handle(g, dtype, "build_spectra", &h);
  if (st != FF_OK) return st;
  st = make_spectra(h, (hipStream_t)stream);
  if (st != FF_OK) {
    std::string msg = g_err;
    free_handle(h);
    return fail(st, msg);
  }
  *out = h;
  return FF_OK;
}

// ---- spectra checkpoints -------------------------------------------------------------
// File layout (host byte order): magic "FFSPEC", u16 version; i32 dtype, sx, sy, nz, pad_xl,
// pad_xr, pad_yl, pad_yr, kernel, NX, NY; f64 dx, dy, incl, decl, field; f64 z_edges[nz + 1];
// i64 byte count of the spectra; the spectra ([nz][NX/2 + 1][NY] complex, as on the device);
// u64 FNV-1a hash of the spectra bytes.
static const char kMagic[6] = {'F', 'F', 'S', 'P', 'E', 'C'};
static const uint16_t kVersion = 1;

static uint64_t fnv1a(const unsigned char *p, size_t n) {
  uint64_t hsh = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) hsh = (hsh ^ p[i]) * 1099511628211ull;
  return hsh;
}

ff_status ff_spectra_save(ff_spectra h, const char *path) {
  if (!h || !path) return fail(FF_EINVAL, "ff_spectra_save: NULL argument");
  ff_status st = check_device(h);
  if (st != FF_OK) return st;
  const size_t bytes = csize(h->dtype) * (size_t)h->nz * h->H * h->NY;
  std::vector<unsigned char> buf(bytes);
  if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(buf.data(), h->spec, bytes, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(FF_EHIP, "ff_spectra_save: spectra download failed");
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(FF_EINVAL, std::string("ff_spectra_save: cannot open ") + path);
  const int32_t iv[11] = {h->dtype, h->sx, h->sy, h->nz, h->pxl, h->pxr, h->pyl, h->pyr, h->kernel, h->NX, h->NY};
  const double dv[5] = {h->dx, h->dy, h->incl, h->decl, h->field};
  const int64_t nb = (int64_t)bytes;
  const uint64_t hsh = fnv1a(buf.data(), bytes);
  bool ok = std::fwrite(kMagic, 1, 6, f) == 6 && std::fwrite(&kVersion, 2, 1, f) == 1 &&
            std::fwrite(iv, 4, 11, f) == 11 && std::fwrite(dv, 8, 5, f) == 5 &&
            std::fwrite(h->z_edges.data(), 8, h->z_edges.size(), f) == h->z_edges.size() &&
            std::fwrite(&nb, 8, 1, f) == 1 && std::fwrite(buf.data(), 1, bytes, f) == bytes &&
            std::fwrite(&hsh, 8, 1, f) == 1;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? FF_OK : fail(FF_EINVAL, std::string("ff_spectra_save: write failed for ") + path);
}

ff_status ff_spectra_load(const char *path, ff_stream stream, ff_spectra *out) {
  if (!path || !out) return fail(FF_EINVAL, "ff_spectra_load: NULL argument");
  *out = nullptr;
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(FF_EINVAL, std::string("ff_spectra_load: cannot open ") + path);
  char magic[6];
  uint16_t ver = 0;
  int32_t iv[11];
  double dv[5];
  bool ok = std::fread(magic, 1, 6, f) == 6 && std::memcmp(magic, kMagic, 6) == 0 && std::fread(&ver, 2, 1, f) == 1 &&
            ver == kVersion && std::fread(iv, 4, 11, f) == 11 && std::fread(dv, 8, 5, f) == 5;
  if (!ok || iv[3] < 1 || iv[3] > (1 << 20)) {
    std::fclose(f);
    return fail(FF_EINVAL, "ff_spectra_load: not a spectra file of this version");
  }
  std::vector<double> z(iv[3] + 1);
  int64_t nb = 0;
  ok = std::fread(z.data(), 8, z.size(), f) == z.size() && std::fread(&nb, 8, 1, f) == 1;
  ff_geometry g{};
  g.sx = iv[1]; g.sy = iv[2]; g.nz = iv[3];
  g.pad_xl = iv[4]; g.pad_xr = iv[5]; g.pad_yl = iv[6]; g.pad_yr = iv[7];
  g.kernel = iv[8]; g.nfft_x = iv[9]; g.nfft_y = iv[10];
  g.dx = dv[0]; g.dy = dv[1]; g.incl_deg = dv[2]; g.decl_deg = dv[3]; g.field_nT = dv[4];
  g.z_edges = z.data();
  ff_spectra h = nullptr;
  ff_status st = ok ? create_handle(&g, iv[0], "ff_spectra_load", &h) : fail(FF_EINVAL, "ff_spectra_load: truncated file");
  if (st != FF_OK) {
    std::fclose(f);
    return st;
  }
  const size_t bytes = csize(h->dtype) * (size_t)h->nz * h->H * h->NY;
  std::vector<unsigned char> buf(bytes);
  uint64_t hsh = 0;
  ok = nb == (int64_t)bytes && std::fread(buf.data(), 1, bytes, f) == bytes && std::fread(&hsh, 8, 1, f) == 1;
  std::fclose(f);
  if (!ok || hsh != fnv1a(buf.data(), bytes)) {
    free_handle(h);
    return fail(FF_EINVAL, "ff_spectra_load: spectra truncated or corrupted");
  }
  // the upload is ordered on the caller's stream; the call returns once it is done (buf is host
  // memory of this call)
  const hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(h->spec, buf.data(), bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    free_handle(h);
    return fail(FF_EHIP, "ff_spectra_load: spectra upload failed");
  }
  *out = h;
  return FF_OK;
}

ff_status ff_spectra_geometry(ff_spectra h, ff_geometry *g, double *z_edges) {
  if (!h || !g) return fail(FF_EINVAL, "ff_spectra_geometry: NULL argument");
  g->sx = h->sx; g->sy = h->sy; g->nz = h->nz;
  g->pad_xl = h->pxl; g->pad_xr = h->pxr; g->pad_yl = h->pyl; g->pad_yr = h->pyr;
  g->dx = h->dx; g->dy = h->dy;
  g->kernel = h->kernel;
  g->incl_deg = h->incl; g->decl_deg = h->decl; g->field_nT = h->field;
  g->nfft_x = h->NX; g->nfft_y = h->NY;
  g->z_edges = z_edges;
  if (z_edges) std::memcpy(z_edges, h->z_edges.data(), sizeof(double) * h->z_edges.size());
  return FF_OK;
}

ff_status ff_free_spectra(ff_spectra h) {
  if (!h) return fail(FF_EINVAL, "ff_free_spectra: NULL handle");
  free_handle(h);
  return FF_OK;
}

ff_status ff_spectra_info(ff_spectra h, int64_t *m, int64_t *n, int32_t *nfft_x, int32_t *nfft_y,
                          int32_t *dtype) {
  if (!h) return fail(FF_EINVAL, "ff_spectra_info: NULL handle");
  if (m) *m = h->m;
  if (n) *n = h->n;
  if (nfft_x) *nfft_x = h->NX;
  if (nfft_y) *nfft_y = h->NY;
  if (dtype) *dtype = h->dtype;
  return FF_OK;
}

ff_status ff_kernel_table(ff_spectra h, double *table, ff_stream stream) {
  if (!h || !table) return fail(FF_EINVAL, "ff_kernel_table: NULL argument");
  ff_status st = check_device(h);
  if (st != FF_OK) return st;
  return kernel_table(h, table, (hipStream_t)stream);
}

ff_status apply_G(ff_spectra h, const void *x, void *d, const void *w_pre, const void *w_post, ff_stream stream) {
  if (!h || !x || !d) return fail(FF_EINVAL, "apply_G: NULL argument");
  ff_status st = check_device(h);
  if (st != FF_OK) return st;
  return op_apply(h, 0, 1, x, h->n, d, h->m, w_pre, w_post, h->dtype, (hipStream_t)stream);
}

ff_status apply_GT(ff_spectra h, const void *d, void *x, const void *w_pre, const void *w_post, ff_stream stream) {
  if (!h || !x || !d) return fail(FF_EINVAL, "apply_GT: NULL argument");
  ff_status st = check_device(h);
  if (st != FF_OK) return st;
  return op_apply(h, 1, 1, d, h->m, x, h->n, w_pre, w_post, h->dtype, (hipStream_t)stream);
}

ff_status apply_G_block(ff_spectra h, int32_t transpose, int64_t k, const void *X, int64_t ldx, void *Y,
                        int64_t ldy, const void *w_pre, const void *w_post, ff_stream stream) {
  if (!h || !X || !Y) return fail(FF_EINVAL, "apply_G_block: NULL argument");
  if (transpose != 0 && transpose != 1) return fail(FF_EINVAL, "apply_G_block: transpose must be 0 or 1");
  if (k < 0) return fail(FF_ESHAPE, "apply_G_block: k < 0");
  const int64_t rin = transpose ? h->m : h->n, rout = transpose ? h->n : h->m;
  if (ldx < rin || ldy < rout) return fail(FF_ESHAPE, "apply_G_block: leading dimension too small");
  ff_status st = check_device(h);
  if (st != FF_OK) return st;
  if (k == 0) return FF_OK;
  return op_apply(h, transpose, k, X, ldx, Y, ldy, w_pre, w_post, h->dtype, (hipStream_t)stream);
}

ff_status ff_get_tuning(ff_spectra h, ff_tuning *t) {
  if (!h || !t) return fail(FF_EINVAL, "ff_get_tuning: NULL argument");
  t->lg_G = h->lg_G;
  t->lg_GT = h->lg_GT;
  t->row_tile = h->row_tile;
  t->batch = h->batch;
  t->col_batched = h->col_batched;
  t->rsvd_qr = h->rsvd_qr;
  t->pair_fused = h->pair_fused;
  t->gkb_graph = h->gkb_graph;
  t->gkb_onesided = h->gkb_onesided;
  t->fft_plan_x = h->fft_plan_x;
  t->fft_plan_y = h->fft_plan_y;
  return FF_OK;
}

ff_status ff_set_tuning(ff_spectra h, const ff_tuning *t) {
  if (!h || !t) return fail(FF_EINVAL, "ff_set_tuning: NULL argument");
  if (t->lg_G < 1 || t->lg_G > h->nz || t->lg_GT < 1 || t->lg_GT > h->nz)
    return fail(FF_EINVAL, "ff_set_tuning: layer groups must lie in [1, nz]");
  if (t->row_tile < 0 || t->row_tile > 4) return fail(FF_EINVAL, "ff_set_tuning: row_tile must lie in [0, 4]");
  if (t->batch < 1 || t->batch > h->batch_max)
    return fail(FF_EINVAL, "ff_set_tuning: batch must lie in [1, the handle's workspace batch]");
  if (t->col_batched < 0 || t->col_batched > 2) return fail(FF_EINVAL, "ff_set_tuning: col_batched must be 0, 1 or 2");
  if (t->rsvd_qr < 0 || t->rsvd_qr > 2) return fail(FF_EINVAL, "ff_set_tuning: rsvd_qr must be 0, 1 or 2");
  if (t->pair_fused < 0 || t->pair_fused > 2) return fail(FF_EINVAL, "ff_set_tuning: pair_fused must be 0, 1 or 2");
  if (t->gkb_graph != 0 && t->gkb_graph != 1) return fail(FF_EINVAL, "ff_set_tuning: gkb_graph must be 0 or 1");
  if (t->gkb_onesided < 0 || t->gkb_onesided > 2)
    return fail(FF_EINVAL, "ff_set_tuning: gkb_onesided must be 0, 1 or 2");
  if (t->fft_plan_x < 0 || t->fft_plan_x >= kFftPlans || t->fft_plan_y < 0 || t->fft_plan_y >= kFftPlans)
    return fail(FF_EINVAL, "ff_set_tuning: FFT stage plans must be 0, 1 or 2");
  h->lg_G = t->lg_G;
  h->lg_GT = t->lg_GT;
  h->row_tile = t->row_tile;
  h->batch = t->batch;
  h->col_batched = t->col_batched;
  h->rsvd_qr = t->rsvd_qr;
  h->pair_fused = t->pair_fused;
  h->gkb_graph = t->gkb_graph;
  h->gkb_onesided = t->gkb_onesided;
  h->fft_plan_x = t->fft_plan_x;
  h->fft_plan_y = t->fft_plan_y;
  ++h->tune_version;
  return FF_OK;
}

ff_status ff_time_pass(ff_spectra h, int32_t transpose, int32_t pass, int32_t reps, const void *x, void *y,
                       ff_stream stream) {
  if (!h || !x || !y) return fail(FF_EINVAL, "ff_time_pass: NULL argument");
  if ((transpose != 0 && transpose != 1) || pass < 0 || pass > 2 || reps < 0)
    return fail(FF_EINVAL, "ff_time_pass: transpose in {0,1}, pass in {0,1,2}, reps >= 0");
  ff_status st = check_device(h);
  if (st != FF_OK) return st;
  return op_time_pass(h, transpose, pass, reps, x, y, (hipStream_t)stream);
}

ff_status ff_profile_begin(ff_spectra h, int32_t max_ops) {
  if (!h || max_ops < 1) return fail(FF_EINVAL, "ff_profile_begin: NULL handle or max_ops < 1");
  ff_status st = check_device(h);
  if (st != FF_OK) return st;
  prof_release(h);
  h->prof_ev.resize(4 * (size_t)max_ops);
  for (auto &e : h->prof_ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      prof_release(h);
      return fail(FF_EHIP, "ff_profile_begin: hipEventCreate failed");
    }
  }
  h->prof_kind.assign(max_ops, 0);
  h->prof_cap = max_ops;
  return FF_OK;
}

ff_status ff_profile_end(ff_spectra h, double *ms, int64_t *ops) {
  if (!h || !ms || !ops) return fail(FF_EINVAL, "ff_profile_end: NULL argument");
  for (int i = 0; i < 6; ++i) ms[i] = 0.0;
  ops[0] = ops[1] = 0;
  ff_status st = FF_OK;
  for (int c = 0; c < h->prof_n && st == FF_OK; ++c) {
    hipEvent_t *e = &h->prof_ev[4 * c];
    if (hipEventSynchronize(e[3]) != hipSuccess) {
      st = fail(FF_EHIP, "ff_profile_end: event wait failed");
      break;
    }
    const int t = h->prof_kind[c];
    for (int p = 0; p < 3; ++p) {
      float v = 0.f;
      if (hipEventElapsedTime(&v, e[p], e[p + 1]) != hipSuccess) {
        st = fail(FF_EHIP, "ff_profile_end: hipEventElapsedTime failed");
        break;
      }
      ms[3 * t + p] += v;
    }
    ops[t] += 1;
  }
  prof_release(h);
  return st;
}

}  // extern "C"

// Kernel spectra of the BCCB embedding (Appendix A: the 2-D DFT of each layer's kernel array is
// formed once, before any product).
//
// 1. Every layer's kernel table t_r(u, v) -- the prism integral of Sec. 2.1 for the prism at
//    station-to-prism offset (u, v) -- is evaluated in FP64 and placed at
//    C_r[v mod NY][u mod NX] of the NY x NX circulant generator (zeros elsewhere).
// 2. C_r is transformed with the same FFT passes as the operator, in FP64: real rows along x
//    (packed in pairs), then full columns along y.
// 3. The spectrum, scaled by 1/(NX NY) so that the operator's inverse transforms need no
//    normalization, is stored as [r][kx][ky] (kx in [0, NX/2]) in the handle's precision.
#include <cmath>

#include "passes.h"

namespace ff {
namespace {

constexpr double kGamma = 6.6743e-11;          // m^3 kg^-1 s^-2 (CODATA 2018)
constexpr double kGravScale = kGamma * 1.0e3 * 1.0e5;   // g/cc -> kg/m^3, m/s^2 -> mGal

// ln(a + sqrt(a^2 + rest2)) without cancellation for a < 0
__device__ __forceinline__ double lnplus(double a, double R, double rest2) {
  return a >= 0.0 ? log(a + R) : log(rest2 / (R - a));
}

// principal value of atan(num/den); a station on a top face (den = 0) is the limit from above
__device__ __forceinline__ double atanpv(double num, double den) {
  if (den != 0.0) return atan(num / den);
  if (num == 0.0) return 0.0;
  return num > 0.0 ? 0.5 * M_PI : -0.5 * M_PI;
}

struct Box {
  double x[2], y[2], z[2];
};

// Downward attraction of a unit-density prism (potential derivative d/dz0), metres.
__device__ double prism_gz(const Box &b) {
  double s = 0.0;
#pragma unroll
  for (int ix = 0; ix < 2; ++ix)
#pragma unroll
    for (int iy = 0; iy < 2; ++iy)
#pragma unroll
      for (int iz = 0; iz < 2; ++iz) {
        const double x = b.x[ix], y = b.y[iy], z = b.z[iz];
        const double x2 = x * x, y2 = y * y, z2 = z * z;
        const double R = sqrt(x2 + y2 + z2);
        const double term = x * lnplus(y, R, x2 + z2) + y * lnplus(x, R, y2 + z2) - z * atanpv(x * y, z * R);
        // corner sign mu = +1 for an even number of lower bounds (ix + iy + iz odd);
        // the attraction is -sum mu * term
        s += ((ix + iy + iz) & 1) ? -term : term;
      }
  return s;
}

// f^T T f for the gravity-gradient tensor T of a unit-density prism (dimensionless).
__device__ double prism_tff(const Box &b, double f0, double f1, double f2) {
  double txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;
#pragma unroll
  for (int ix = 0; ix < 2; ++ix)
#pragma unroll
    for (int iy = 0; iy < 2; ++iy)
#pragma unroll
      for (int iz = 0; iz < 2; ++iz) {
        const double x = b.x[ix], y = b.y[iy], z = b.z[iz];
        const double x2 = x * x, y2 = y * y, z2 = z * z;
        const double R = sqrt(x2 + y2 + z2);
        const double sg = ((ix + iy + iz) & 1) ? 1.0 : -1.0;   // corner sign mu
        txx -= sg * atanpv(y * z, x * R);
        tyy -= sg * atanpv(x * z, y * R);
        tzz -= sg * atanpv(x * y, z * R);
        txy += sg * lnplus(z, R, x2 + y2);
        txz += sg * lnplus(y, R, x2 + z2);
        tyz += sg * lnplus(x, R, y2 + z2);
      }
  return f0 * f0 * txx + f1 * f1 * tyy + f2 * f2 * tzz + 2.0 * (f0 * f1 * txy + f0 * f2 * txz + f1 * f2 * tyz);
}

struct KParams {
  int Un, Vn, u0, v0, NX, NY, kernel;
  double dx, dy, f0, f1, f2, scale;
};

// One thread per (u, v) offset of layer r = blockIdx.y.
__global__ void k_kernel_table(KParams p, const double *__restrict__ z_edges, double *__restrict__ table,
                               double *__restrict__ circ) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (idx >= (int64_t)p.Un * p.Vn) return;
  const int iu = (int)(idx % p.Un), iv = (int)(idx / p.Un);
  const int u = p.u0 + iu, v = p.v0 + iv;
  Box b;
  b.x[0] = (-u - 0.5) * p.dx;
  b.x[1] = (-u + 0.5) * p.dx;
  b.y[0] = (-v - 0.5) * p.dy;
  b.y[1] = (-v + 0.5) * p.dy;
  b.z[0] = z_edges[r];
  b.z[1] = z_edges[r + 1];
  const double val = p.kernel == FF_GRAVITY_GZ ? p.scale * prism_gz(b) : p.scale * prism_tff(b, p.f0, p.f1, p.f2);
  if (table) table[((int64_t)r * p.Vn + iv) * p.Un + iu] = val;
  if (circ) {
    const int um = u < 0 ? u + p.NX : u, vm = v < 0 ? v + p.NY : v;
    circ[((int64_t)r * p.NY + vm) * p.NX + um] = val;
  }
}

// Full column FFT along y of the row-transformed generator, scaled and stored in precision TS.
// tmp: [r][kx][y] (ld NY); spec: [r][kx][ky].  Grid: (ceil(H/CPB), nz).
template <typename TS, int NY>
__global__ void __launch_bounds__((ColCfg<double, NY>::THREADS))
k_col_spec(const double2 *__restrict__ tmp, int H, double scale, cplx<TS> *__restrict__ spec,
           const double2 *__restrict__ tw) {
  using CC = ColCfg<double, NY>;
  using F = FFT<double, NY, false>;
  __shared__ double2 sh[CC::CPB * F::LDS];
  const int f = threadIdx.x / CC::TPF, j = threadIdx.x % CC::TPF;
  const int kx = blockIdx.x * CC::CPB + f;
  const bool ok = kx < H;
  const int64_t r = blockIdx.y;
  const double2 *src = tmp + (r * H + (ok ? kx : 0)) * NY;
  double2 v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) v[u] = ok ? src[j + u * CC::TPF] : mk<double>(0, 0);
  F::run(v, j, sh + f * F::LDS, tw);
  if (ok) {
    cplx<TS> *dst = spec + (r * H + kx) * NY;
#pragma unroll
    for (int u = 0; u < 8; ++u) dst[j + u * CC::TPF] = mk<TS>((TS)(v[u].x * scale), (TS)(v[u].y * scale));
  }
}

// The column passes carry the real DC (kx = 0) and Nyquist (kx = NX/2) columns packed in one
// complex column and need, for it, P = (S[0] + S[NX/2]) / 2 and M = (S[0] - S[NX/2]) / 2 in
// place of the two spectra.  Both are linear in the row-transformed generator, so the
// combination is taken on tmp before the column FFT.  Grid: (ceil(NY/256), nz).
__global__ void k_pack_dc_nyquist(double2 *__restrict__ tmp, int H, int NY) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= NY) return;
  double2 *c0 = tmp + (int64_t)blockIdx.y * H * NY;
  double2 *cn = c0 + (int64_t)(H - 1) * NY;
  const double2 a = c0[y], b = cn[y];
  c0[y] = mk<double>(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
  cn[y] = mk<double>(0.5 * (a.x - b.x), 0.5 * (a.y - b.y));
}

template <int NX>
ff_status rows_fp64(const double *circ, int nz, int NY, double2 *tmp, const double2 *tw, hipStream_t s) {
  constexpr int NF = RowMax<double, NX>::NF;
  using C = RowCfg<double, NX, NF>;
  const int H = NX / 2 + 1;
  Idx3 ii{0, (int64_t)NY * NX, NX}, pi{0, 0, 0}, oi{0, (int64_t)H * NY, 1};
  dim3 grid(row_blocks(NY, nz, C::ROWS), 1, 1);
  k_row_r2c<double, double, NX, NF, false><<<grid, C::THREADS, 0, s>>>(circ, ii, nullptr, pi, NY, nz, NX, 0, tmp, oi,
                                                             (int64_t)NY, tw);
  FF_LAUNCH_CHECK("row transform of the kernel generator");
  return FF_OK;
}

template <typename TS, int NY>
ff_status cols_fp64(const double2 *tmp, int nz, int H, double scale, void *spec, const double2 *tw,
                    hipStream_t s) {
  using CC = ColCfg<double, NY>;
  dim3 grid((H + CC::CPB - 1) / CC::CPB, nz, 1);
  k_col_spec<TS, NY><<<grid, CC::THREADS, 0, s>>>(tmp, H, scale, (cplx<TS> *)spec, tw);
  FF_LAUNCH_CHECK("column transform of the kernel generator");
  return FF_OK;
}

KParams kparams(ff_spectra h) {
  KParams p;
  p.u0 = h->pxl - h->nx + 1;
  p.v0 = h->pyl - h->ny + 1;
  p.Un = h->sx + h->nx - 1;
  p.Vn = h->sy + h->ny - 1;
  p.NX = h->NX;
  p.NY = h->NY;
  p.kernel = h->kernel;
  p.dx = h->dx;
  p.dy = h->dy;
  const double I = h->incl * M_PI / 180.0, D = h->decl * M_PI / 180.0;
  p.f0 = cos(I) * cos(D);
  p.f1 = cos(I) * sin(D);
  p.f2 = sin(I);
  p.scale = h->kernel == FF_GRAVITY_GZ ? kGravScale : h->field / (4.0 * M_PI);
  return p;
}

ff_status launch_table(ff_spectra h, double *table, double *circ, hipStream_t s) {
  KParams p = kparams(h);
  const int64_t cnt = (int64_t)p.Un * p.Vn;
  dim3 grid((unsigned)((cnt + 255) / 256), h->nz, 1);
  k_kernel_table<<<grid, 256, 0, s>>>(p, h->z_dev, table, circ);
  FF_LAUNCH_CHECK("kernel table");
  return FF_OK;
}

}  // namespace

ff_status kernel_table(ff_spectra h, double *table, hipStream_t s) {
  return launch_table(h, table, nullptr, s);
}

ff_status make_spectra(ff_spectra h, hipStream_t s) {
  const int NX = h->NX, NY = h->NY, H = h->H, nz = h->nz;
  double *circ = nullptr;
  double2 *tmp = nullptr, *twx = nullptr, *twy = nullptr;
  ff_status st = FF_OK;
  auto cleanup = [&]() {
    hipFree(circ);
    hipFree(tmp);
    hipFree(twx);
    hipFree(twy);
  };
  // FP64 twiddle tables for the construction (the handle keeps its own in its precision)
  std::vector<double2> hx(NX), hy(NY);
  for (int e = 0; e < NX; ++e) hx[e] = mk<double>(cos(2.0 * M_PI * e / NX), -sin(2.0 * M_PI * e / NX));
  for (int e = 0; e < NY; ++e) hy[e] = mk<double>(cos(2.0 * M_PI * e / NY), -sin(2.0 * M_PI * e / NY));
  if (hipMalloc(&circ, sizeof(double) * (size_t)nz * NY * NX) != hipSuccess ||
      hipMalloc(&tmp, sizeof(double2) * (size_t)nz * H * NY) != hipSuccess ||
      hipMalloc(&twx, sizeof(double2) * NX) != hipSuccess || hipMalloc(&twy, sizeof(double2) * NY) != hipSuccess) {
    cleanup();
    return fail(FF_ENOMEM, "build_spectra: temporary allocation failed");
  }
  if (hipMemcpyAsync(twx, hx.data(), sizeof(double2) * NX, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(twy, hy.data(), sizeof(double2) * NY, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemsetAsync(circ, 0, sizeof(double) * (size_t)nz * NY * NX, s) != hipSuccess) {
    cleanup();
    return fail(FF_EHIP, "build_spectra: copy/memset failed");
  }
  st = launch_table(h, nullptr, circ, s);
  if (st == FF_OK) {
    FF_SWITCH_N_SET(NX, st, st = rows_fp64<NN>(circ, nz, NY, tmp, twx, s));
  }
  if (st == FF_OK) {
    k_pack_dc_nyquist<<<dim3((NY + 255) / 256, nz), 256, 0, s>>>(tmp, H, NY);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) st = hip_fail(e, "DC/Nyquist combination of the kernel spectra");
  }
  if (st == FF_OK) {
    const double scale = 1.0 / ((double)NX * (double)NY);
    if (h->dtype == FF_F32) {
      FF_SWITCH_N_SET(NY, st, st = (cols_fp64<float, NN>(tmp, nz, H, scale, h->spec, twy, s)));
    } else {
      FF_SWITCH_N_SET(NY, st, st = (cols_fp64<double, NN>(tmp, nz, H, scale, h->spec, twy, s)));
    }
  }
  if (st == FF_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(FF_EHIP, "build_spectra: kernels failed");
  cleanup();
  return st;
}

}  // namespace ff

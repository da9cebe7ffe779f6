// Radix-8 (+ a final radix-4 or radix-2) Stockham FFT held in registers, one FFT per group
// of N/8 threads, exchanged between stages through LDS.
//
// Data distribution (the same on entry and on exit, so transforms chain without shuffles):
// thread j of the group holds the 8 elements with natural indices j + u*(N/8), u = 0..7.
// A stage of radix R with Ns points already combined takes, for butterfly b, the R inputs
// a[b + t*N/R], multiplies input t by w^(t*(b mod Ns)) with w = exp(-+2 pi i/(Ns*R)), does an
// R-point DFT and writes output s to position (b/Ns)*Ns*R + (b mod Ns) + s*Ns (Stockham
// autosort).  In the last stage Ns = N/R, so the outputs land at b + s*N/R: natural order
// in the thread's own registers.  Twiddles come from a table exp(-2 pi i e / N), e in [0, N),
// built on the host in FP64 and rounded once to T.
//
// Transforms of N <= 512 live in one wavefront and synchronize with wavefront barriers, so
// waves run their transforms independently.  Larger transforms span several waves and use
// block-wide barriers: then every FFT group of the block must call run() together.
//
// LDS exchange buffers are padded by one element per 8 (index i -> i + i/8) so that the
// strided Stockham writes spread over the banks.
#pragma once

#include "common.h"

namespace ff {

template <typename T> struct Consts;
template <> struct Consts<float> { static constexpr float r2 = 0.70710678118654752440f; };
template <> struct Consts<double> { static constexpr double r2 = 0.70710678118654752440; };

// multiply by w4 = -i (forward) or +i (inverse)
template <bool INV, typename T> __device__ __forceinline__ cplx<T> mul_w4(cplx<T> a) {
  return INV ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}
template <bool INV, typename T>
__device__ __forceinline__ void dft2(cplx<T> &a0, cplx<T> &a1) {
  cplx<T> t = a0;
  a0 = cadd<T>(t, a1);
  a1 = csub<T>(t, a1);
}

template <bool INV, typename T>
__device__ __forceinline__ void dft4(cplx<T> &a0, cplx<T> &a1, cplx<T> &a2, cplx<T> &a3) {
  cplx<T> t0 = cadd<T>(a0, a2), t1 = csub<T>(a0, a2);
  cplx<T> t2 = cadd<T>(a1, a3), t3 = mul_w4<INV, T>(csub<T>(a1, a3));
  a0 = cadd<T>(t0, t2);
  a2 = csub<T>(t0, t2);
  a1 = cadd<T>(t1, t3);
  a3 = csub<T>(t1, t3);
}

// e +- c (p, q): the butterfly of an odd term rotated by an eighth turn, c (p, q) with
// c = 1/sqrt2 and p, q sums of its parts, as explicit fused multiply-adds
template <typename T>
__device__ __forceinline__ void bfly_c(cplx<T> e, T p, T q, cplx<T> &plus, cplx<T> &minus) {
  const T c = Consts<T>::r2;
  plus = mk<T>(ffma(c, p, e.x), ffma(c, q, e.y));
  minus = mk<T>(ffma(-c, p, e.x), ffma(-c, q, e.y));
}

// in-place 8-point DFT of a[0..7]
template <bool INV, typename T> __device__ __forceinline__ void dft8(cplx<T> *a) {
  cplx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  cplx<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<INV, T>(e0, e1, e2, e3);
  dft4<INV, T>(o0, o1, o2, o3);
  o2 = mul_w4<INV, T>(o2);
  a[0] = cadd<T>(e0, o0);
  a[4] = csub<T>(e0, o0);
  a[2] = cadd<T>(e2, o2);
  a[6] = csub<T>(e2, o2);
  // w8 o1 = c (x + y, y - x) forward, c (x - y, x + y) inverse;
  // w8^3 o3 = c (y - x, -x - y) forward, c (-x - y, x - y) inverse
  if (INV) {
    bfly_c<T>(e1, o1.x - o1.y, o1.x + o1.y, a[1], a[5]);
    bfly_c<T>(e3, -o3.x - o3.y, o3.x - o3.y, a[3], a[7]);
  } else {
    bfly_c<T>(e1, o1.x + o1.y, o1.y - o1.x, a[1], a[5]);
    bfly_c<T>(e3, o3.y - o3.x, -o3.x - o3.y, a[3], a[7]);
  }
}

// Pruned butterflies.  ZIN: the inputs a[4..7] of a first-stage 8-point DFT are zero (the
// transform's input is zero from element N/2 on, so they need not be loaded or added); ZOUT:
// only the outputs a[0..3] of a last-stage DFT are used (elements below N/2), the others are
// left unspecified.  Both skip arithmetic only; the outputs computed are those of dft8 bit for bit.
template <bool INV, typename T>
__device__ __forceinline__ void dft4_zin(cplx<T> &a0, cplx<T> &a1, cplx<T> &a2, cplx<T> &a3) {
  // a2 = a3 = 0 on input
  const cplx<T> t3 = mul_w4<INV, T>(a1);
  a2 = csub<T>(a0, a1);
  a3 = csub<T>(a0, t3);
  const cplx<T> x0 = a0;
  a0 = cadd<T>(x0, a1);
  a1 = cadd<T>(x0, t3);
}
template <bool INV, bool ZIN, bool ZOUT, typename T> __device__ __forceinline__ void dft8p(cplx<T> *a) {
  if constexpr (!ZIN && !ZOUT) {
    dft8<INV, T>(a);
  } else {
    cplx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    cplx<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
    if constexpr (ZIN) {
      dft4_zin<INV, T>(e0, e1, e2, e3);
      dft4_zin<INV, T>(o0, o1, o2, o3);
    } else {
      dft4<INV, T>(e0, e1, e2, e3);
      dft4<INV, T>(o0, o1, o2, o3);
    }
    o2 = mul_w4<INV, T>(o2);
    a[0] = cadd<T>(e0, o0);
    a[2] = cadd<T>(e2, o2);
    if constexpr (!ZOUT) {
      a[4] = csub<T>(e0, o0);
      a[6] = csub<T>(e2, o2);
    }
    cplx<T> m1, m3;
    if (INV) {
      bfly_c<T>(e1, o1.x - o1.y, o1.x + o1.y, a[1], m1);
      bfly_c<T>(e3, -o3.x - o3.y, o3.x - o3.y, a[3], m3);
    } else {
      bfly_c<T>(e1, o1.x + o1.y, o1.y - o1.x, a[1], m1);
      bfly_c<T>(e3, o3.y - o3.x, -o3.x - o3.y, a[3], m3);
    }
    if constexpr (!ZOUT) {
      a[5] = m1;
      a[7] = m3;
    }
  }
}

template <bool INV, typename T>
__device__ __forceinline__ cplx<T> twiddle(cplx<T> v, const cplx<T> *__restrict__ tw, int e) {
  cplx<T> w = tw[e];
  return INV ? cmulc<T>(v, w) : cmul<T>(v, w);
}

// Synchronization of one transform's LDS exchange: a wavefront barrier with LDS ordering
// when the group fits in a wavefront, else a block barrier.
template <int TPF> __device__ __forceinline__ void group_sync() {
  if constexpr (TPF <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

__device__ __forceinline__ int pad8(int i) { return i + (i >> 3); }

constexpr int ilog8(int n) { return n < 8 ? 0 : 1 + ilog8(n / 8); }
constexpr int ipow8(int k) { return k == 0 ? 1 : 8 * ipow8(k - 1); }

template <typename T, int N, bool INV> struct FFT {
  static_assert(N >= 8 && (N & (N - 1)) == 0, "N must be a power of two >= 8");
  static constexpr int TPF = N / 8;                // threads per transform
  static constexpr int L8 = ilog8(N);              // radix-8 stages
  static constexpr int REM = N / ipow8(L8);        // 1, 2 or 4: final radix
  static constexpr bool WAVE = TPF <= 64;          // one wavefront: wavefront barriers
  static constexpr int HALF = N + N / 8;           // one padded exchange buffer
  // complex elements of LDS per transform: one buffer (synchronized before and after each
  // exchange) inside a wavefront or when two would exceed 32 KB, else two alternating
  // buffers (one barrier per exchange)
  static constexpr bool SINGLE = WAVE || 2 * HALF * (int)sizeof(cplx<T>) > 32768;
  static constexpr int LDS = SINGLE ? HALF : 2 * HALF;

  // Per-thread twiddles of the radix-8 stages after the first (7 per stage) and of the final
  // radix-4/2 stage, read once and reused by every transform the thread performs.
  static constexpr int NTW = (L8 > 1 ? (L8 - 1) * 7 : 0) + (REM == 4 ? 6 : (REM == 2 ? 4 : 0));
  struct Tw {
    cplx<T> w[NTW > 0 ? NTW : 1];
  };
  __device__ static void load_tw(Tw &t, int j, const cplx<T> *__restrict__ tw) {
    int Ns = 8, q = 0;
#pragma unroll
    for (int st = 1; st < L8; ++st) {
      const int step = (j % Ns) * (N / (Ns * 8));
#pragma unroll
      for (int u = 1; u < 8; ++u) t.w[q++] = tw[step * u];
      Ns *= 8;
    }
    if (REM == 4) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int step = ((j + c * TPF) % Ns) * (N / (Ns * 4));
#pragma unroll
        for (int u = 1; u < 4; ++u) t.w[q++] = tw[step * u];
      }
    } else if (REM == 2) {
#pragma unroll
      for (int c = 0; c < 4; ++c) t.w[q++] = tw[((j + c * TPF) % Ns) * (N / (Ns * 2))];
    }
  }
  __device__ static cplx<T> tmul(cplx<T> v, cplx<T> w) { return INV ? cmulc<T>(v, w) : cmul<T>(v, w); }

  // Same transform as run(), with the twiddles taken from registers.  ZIN: the input is zero
  // from element N/2 on (v[4..7] are not read); ZOUT: only the outputs below N/2 (v[0..3]) are
  // produced.
  template <bool ZIN = false, bool ZOUT = false>
  __device__ static void run_tw(cplx<T> (&v)[8], int j, cplx<T> *buf, const Tw &t) {
    int Ns = 1, q = 0;
    bool used_lds = false;
#pragma unroll
    for (int st = 0; st < L8; ++st) {
      const bool last = (st == L8 - 1) && REM == 1;
      const int k = j % Ns;
      if (st > 0) {
#pragma unroll
        for (int u = 1; u < 8; ++u) v[u] = tmul(v[u], t.w[q++]);
      }
      if (st == 0 && last) dft8p<INV, ZIN, ZOUT, T>(v);
      else if (st == 0) dft8p<INV, ZIN, false, T>(v);
      else if (last) dft8p<INV, false, ZOUT, T>(v);
      else dft8<INV, T>(v);
      if (!last) {
        cplx<T> *dst = SINGLE ? buf : buf + (st & 1) * HALF;
        const int base = (j / Ns) * Ns * 8 + k;
        if (SINGLE) group_sync<TPF>();
#pragma unroll
        for (int s = 0; s < 8; ++s) dst[pad8(base + s * Ns)] = v[s];
        group_sync<TPF>();
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = dst[pad8(j + u * TPF)];
        used_lds = true;
      }
      Ns *= 8;
    }
    final_stage<ZOUT>(v, Ns, q, t);
    if (used_lds) group_sync<TPF>();
  }

  // the radix-4 or radix-2 stage after the radix-8 ones (REM = 4 or 2), twiddles from registers
  template <bool ZOUT>
  __device__ static void final_stage(cplx<T> (&v)[8], int Ns, int q, const Tw &t) {
    if (REM == 4) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (Ns > 1) {
#pragma unroll
          for (int u = 1; u < 4; ++u) v[c + 2 * u] = tmul(v[c + 2 * u], t.w[q++]);
        }
        if (ZOUT) {
          // outputs c, c + 2 only (elements below N/2)
          const cplx<T> t0 = cadd<T>(v[c], v[c + 4]), t1 = csub<T>(v[c], v[c + 4]);
          const cplx<T> t2 = cadd<T>(v[c + 2], v[c + 6]), t3 = mul_w4<INV, T>(csub<T>(v[c + 2], v[c + 6]));
          v[c] = cadd<T>(t0, t2);
          v[c + 2] = cadd<T>(t1, t3);
        } else {
          dft4<INV, T>(v[c], v[c + 2], v[c + 4], v[c + 6]);
        }
      }
    } else if (REM == 2) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (Ns > 1) v[c + 4] = tmul(v[c + 4], t.w[q++]);
        if (ZOUT) v[c] = cadd<T>(v[c], v[c + 4]);
        else dft2<INV, T>(v[c], v[c + 4]);
      }
    }
  }

  // v[u] = x[j + u*TPF] on entry, X[j + u*TPF] on exit.  buf: this group's LDS elements.
  // Twiddles read from the table; ZIN / ZOUT as for run_tw.
  template <bool ZIN = false, bool ZOUT = false>
  __device__ static void run(cplx<T> (&v)[8], int j, cplx<T> *buf, const cplx<T> *__restrict__ tw) {
    int Ns = 1;
    bool used_lds = false;
#pragma unroll
    for (int st = 0; st < L8; ++st) {
      const bool last = (st == L8 - 1) && REM == 1;
      // radix-8 butterfly b = j on slots 0..7 (a[b + t*N/8] = slot t)
      const int k = j % Ns;
      const int step = k * (N / (Ns * 8));
      if (st > 0) {
#pragma unroll
        for (int t = 1; t < 8; ++t) v[t] = twiddle<INV, T>(v[t], tw, step * t);
      }
      if (st == 0 && last) dft8p<INV, ZIN, ZOUT, T>(v);
      else if (st == 0) dft8p<INV, ZIN, false, T>(v);
      else if (last) dft8p<INV, false, ZOUT, T>(v);
      else dft8<INV, T>(v);
      if (!last) {
        cplx<T> *dst = SINGLE ? buf : buf + (st & 1) * HALF;
        const int base = (j / Ns) * Ns * 8 + k;
        if (SINGLE) group_sync<TPF>();
#pragma unroll
        for (int s = 0; s < 8; ++s) dst[pad8(base + s * Ns)] = v[s];
        group_sync<TPF>();
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = dst[pad8(j + u * TPF)];
        used_lds = true;
      }
      Ns *= 8;
    }
    if (REM == 4) {
      // two radix-4 butterflies: b = j (slots 0,2,4,6) and b = j + N/8 (slots 1,3,5,7)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int b = j + c * TPF;
        const int k = b % Ns;
        const int step = k * (N / (Ns * 4));
        if (Ns > 1) {
#pragma unroll
          for (int t = 1; t < 4; ++t) v[c + 2 * t] = twiddle<INV, T>(v[c + 2 * t], tw, step * t);
        }
        if (ZOUT) {
          const cplx<T> t0 = cadd<T>(v[c], v[c + 4]), t1 = csub<T>(v[c], v[c + 4]);
          const cplx<T> t2 = cadd<T>(v[c + 2], v[c + 6]), t3 = mul_w4<INV, T>(csub<T>(v[c + 2], v[c + 6]));
          v[c] = cadd<T>(t0, t2);
          v[c + 2] = cadd<T>(t1, t3);
        } else {
          dft4<INV, T>(v[c], v[c + 2], v[c + 4], v[c + 6]);
        }
      }
    } else if (REM == 2) {
      // four radix-2 butterflies b = j + c*N/8 on slots c, c+4
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int b = j + c * TPF;
        const int k = b % Ns;
        const int step = k * (N / (Ns * 2));
        if (Ns > 1) v[c + 4] = twiddle<INV, T>(v[c + 4], tw, step);
        if (ZOUT) v[c] = cadd<T>(v[c], v[c + 4]);
        else dft2<INV, T>(v[c], v[c + 4]);
      }
    }
    // A later call (or the caller's own LDS use) may overwrite the buffers this call read.
    if (used_lds) group_sync<TPF>();
  }
};

// Two independent transforms of the same length run interleaved by one FFT group: `a` in
// direction INVA and `b` in direction INVB, each with its own exchange buffer, sharing the
// register twiddles and the barriers of every exchange.  Each transform does exactly the
// arithmetic of FFT::run_tw with its own pruning flags (same results bit for bit); the
// interleaving gives the scheduler a second chain of work while the other waits on LDS.
// Wave-level transforms only (N <= 512).
template <typename T, int N, bool INVA, bool INVB, bool ZINA = false, bool ZOUTA = false, bool ZINB = false,
          bool ZOUTB = false>
__device__ __forceinline__ void fft_dual(cplx<T> (&a)[8], cplx<T> (&b)[8], int j, cplx<T> *bufA, cplx<T> *bufB,
                                         const typename FFT<T, N, false>::Tw &t) {
  using F = FFT<T, N, false>;
  using FA = FFT<T, N, INVA>;
  using FB = FFT<T, N, INVB>;
  static_assert(F::WAVE, "fft_dual: wave-level transforms only");
  constexpr int TPF = F::TPF, L8 = F::L8, REM = F::REM;
  auto mulA = [](cplx<T> v, cplx<T> w) { return INVA ? cmulc<T>(v, w) : cmul<T>(v, w); };
  auto mulB = [](cplx<T> v, cplx<T> w) { return INVB ? cmulc<T>(v, w) : cmul<T>(v, w); };
  int Ns = 1, q = 0;
  bool used_lds = false;
#pragma unroll
  for (int st = 0; st < L8; ++st) {
    const bool last = (st == L8 - 1) && REM == 1;
    const int k = j % Ns;
    if (st > 0) {
#pragma unroll
      for (int u = 1; u < 8; ++u) {
        a[u] = mulA(a[u], t.w[q]);
        b[u] = mulB(b[u], t.w[q]);
        ++q;
      }
    }
    if (st == 0 && last) {
      dft8p<INVA, ZINA, ZOUTA, T>(a);
      dft8p<INVB, ZINB, ZOUTB, T>(b);
    } else if (st == 0) {
      dft8p<INVA, ZINA, false, T>(a);
      dft8p<INVB, ZINB, false, T>(b);
    } else if (last) {
      dft8p<INVA, false, ZOUTA, T>(a);
      dft8p<INVB, false, ZOUTB, T>(b);
    } else {
      dft8<INVA, T>(a);
      dft8<INVB, T>(b);
    }
    if (!last) {
      const int base = (j / Ns) * Ns * 8 + k;
      group_sync<TPF>();
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        bufA[pad8(base + s * Ns)] = a[s];
        bufB[pad8(base + s * Ns)] = b[s];
      }
      group_sync<TPF>();
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a[u] = bufA[pad8(j + u * TPF)];
        b[u] = bufB[pad8(j + u * TPF)];
      }
      used_lds = true;
    }
    Ns *= 8;
  }
  if (REM != 1) {
    FA::template final_stage<ZOUTA>(a, Ns, q, *reinterpret_cast<const typename FA::Tw *>(&t));
    FB::template final_stage<ZOUTB>(b, Ns, q, *reinterpret_cast<const typename FB::Tw *>(&t));
  }
  if (used_lds) group_sync<TPF>();
}

}  // namespace ff

// Stockham FFT held in registers, one FFT per group of N/8 threads (eight elements each),
// exchanged between stages through LDS, in one of three stage plans of radices 8, 4 and 2.
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
constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

// Stage plans of an N-point transform with eight elements per thread (radices 8, 4 and 2; a
// radix-R stage does 8/R butterflies per thread):
//   plan 0: radix-8 stages, then one radix-4 or radix-2 stage when N is not a power of 8;
//   plan 1: that radix-4 or radix-2 stage first, then the radix-8 stages;
//   plan 2: radix-4 stages, then one radix-2 stage when log2 N is odd.
// Plans 0 and 1 are the same sequence when N is a power of 8 (plan_canon maps 1 to 0 there).
constexpr int plan_rem(int N) { return N / ipow8(ilog8(N)); }
constexpr int plan_nst(int N, int P) {
  return P == 2 ? (ilog2c(N) + 1) / 2 : ilog8(N) + (plan_rem(N) > 1 ? 1 : 0);
}
constexpr int plan_radix(int N, int P, int st) {
  return P == 2 ? ((st == ilog2c(N) / 2 && (ilog2c(N) & 1)) ? 2 : 4)
       : plan_rem(N) == 1 ? 8
       : P == 0 ? (st < ilog8(N) ? 8 : plan_rem(N))
       : (st == 0 ? plan_rem(N) : 8);
}
constexpr int plan_canon(int N, int P) { return (P == 1 && plan_rem(N) == 1) ? 0 : P; }
// points combined before stage st, and the register twiddles of the stages before st (a
// radix-R stage after the first multiplies 8 - 8/R of the thread's elements)
constexpr int plan_ns(int N, int P, int st) { return st == 0 ? 1 : plan_ns(N, P, st - 1) * plan_radix(N, P, st - 1); }
constexpr int plan_twoff(int N, int P, int st) {
  return st <= 1 ? 0 : plan_twoff(N, P, st - 1) + 8 - 8 / plan_radix(N, P, st - 1);
}

// the butterflies of one radix-R stage on the thread's eight elements: butterfly c takes
// slots c + t*(8/R), t = 0..R-1, and leaves output s in slot c + s*(8/R).  ZIN: inputs t >= R/2
// are zero (slots 4..7, not read); ZOUT: only outputs s < R/2 (slots 0..3) are produced.
template <int R, bool INV, bool ZIN, bool ZOUT, typename T>
__device__ __forceinline__ void stage_dft(cplx<T> (&v)[8]) {
  if constexpr (R == 8) {
    dft8p<INV, ZIN, ZOUT, T>(v);
  } else if constexpr (R == 4) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if constexpr (ZIN) {
        dft4_zin<INV, T>(v[c], v[c + 2], v[c + 4], v[c + 6]);
      } else if constexpr (ZOUT) {
        const cplx<T> t0 = cadd<T>(v[c], v[c + 4]), t1 = csub<T>(v[c], v[c + 4]);
        const cplx<T> t2 = cadd<T>(v[c + 2], v[c + 6]), t3 = mul_w4<INV, T>(csub<T>(v[c + 2], v[c + 6]));
        v[c] = cadd<T>(t0, t2);
        v[c + 2] = cadd<T>(t1, t3);
      } else {
        dft4<INV, T>(v[c], v[c + 2], v[c + 4], v[c + 6]);
      }
    }
  } else {
    static_assert(R == 2, "radix 8, 4 or 2");
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if constexpr (ZIN) v[c + 4] = v[c];
      else if constexpr (ZOUT) v[c] = cadd<T>(v[c], v[c + 4]);
      else dft2<INV, T>(v[c], v[c + 4]);
    }
  }
}

// Transform of N points by TPF = N/8 threads in the given stage plan.  A stage of radix R with
// Ns points already combined computes, for butterfly b, the R inputs a[b + t*N/R] times
// w^(t*(b mod Ns)), w = exp(-+2 pi i/(Ns*R)), then an R-point DFT whose output s goes to position
// (b/Ns)*Ns*R + (b mod Ns) + s*Ns.  Thread j's butterflies are b = j + c*TPF, c < 8/R, so their
// inputs are exactly its elements j + u*TPF; the last stage leaves the outputs in natural order
// in the same slots, and the stages in between exchange through LDS.
template <typename T, int N, bool INV, int P = 0> struct FFT {
  static_assert(N >= 8 && (N & (N - 1)) == 0, "N must be a power of two >= 8");
  static_assert(P >= 0 && P < kFftPlans, "stage plan 0, 1 or 2");
  static constexpr int TPF = N / 8;                // threads per transform
  static constexpr int NST = plan_nst(N, P);       // stages
  static constexpr bool WAVE = TPF <= 64;          // one wavefront: wavefront barriers
  static constexpr int HALF = N + N / 8;           // one padded exchange buffer
  // complex elements of LDS per transform: one buffer (synchronized before and after each
  // exchange) inside a wavefront or when two would exceed 32 KB, else two alternating
  // buffers (one barrier per exchange)
  static constexpr bool SINGLE = WAVE || 2 * HALF * (int)sizeof(cplx<T>) > 32768;
  static constexpr int LDS = SINGLE ? HALF : 2 * HALF;

  // Per-thread twiddles of every stage after the first, read once and reused by every
  // transform the thread performs (the same values serve both directions).
  static constexpr int NTW = plan_twoff(N, P, NST);
  struct Tw {
    cplx<T> w[NTW > 0 ? NTW : 1];
  };
  template <int ST> __device__ __forceinline__ static void load_st(Tw &t, int j, const cplx<T> *__restrict__ tw) {
    if constexpr (ST < NST) {
      constexpr int R = plan_radix(N, P, ST), Ns = plan_ns(N, P, ST), Q = plan_twoff(N, P, ST);
#pragma unroll
      for (int c = 0; c < 8 / R; ++c) {
        const int step = ((j + c * TPF) % Ns) * (N / (Ns * R));
#pragma unroll
        for (int u = 1; u < R; ++u) t.w[Q + c * (R - 1) + u - 1] = tw[step * u];
      }
      load_st<ST + 1>(t, j, tw);
    }
  }
  __device__ static void load_tw(Tw &t, int j, const cplx<T> *__restrict__ tw) { load_st<1>(t, j, tw); }
  __device__ static cplx<T> tmul(cplx<T> v, cplx<T> w) { return INV ? cmulc<T>(v, w) : cmul<T>(v, w); }

  // the twiddles of stage ST > 0: from registers (REG, t) or from the table tw
  template <int ST, bool REG>
  __device__ __forceinline__ static void twiddle_st(cplx<T> (&v)[8], int j, const Tw *t,
                                                    const cplx<T> *__restrict__ tw) {
    constexpr int R = plan_radix(N, P, ST), Ns = plan_ns(N, P, ST), Q = plan_twoff(N, P, ST);
#pragma unroll
    for (int c = 0; c < 8 / R; ++c) {
      const int step = ((j + c * TPF) % Ns) * (N / (Ns * R));
#pragma unroll
      for (int u = 1; u < R; ++u) {
        const cplx<T> w = REG ? t->w[Q + c * (R - 1) + u - 1] : tw[step * u];
        v[c + u * (8 / R)] = tmul(v[c + u * (8 / R)], w);
      }
    }
  }

  // the Stockham write of stage ST's outputs to buffer dst
  template <int ST> __device__ __forceinline__ static void write_st(const cplx<T> (&v)[8], int j, cplx<T> *dst) {
    constexpr int R = plan_radix(N, P, ST), Ns = plan_ns(N, P, ST);
#pragma unroll
    for (int c = 0; c < 8 / R; ++c) {
      const int b = j + c * TPF;
      const int base = (b / Ns) * Ns * R + b % Ns;
#pragma unroll
      for (int s = 0; s < R; ++s) dst[pad8(base + s * Ns)] = v[c + s * (8 / R)];
    }
  }
  __device__ __forceinline__ static void read_all(cplx<T> (&v)[8], int j, const cplx<T> *src) {
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[pad8(j + u * TPF)];
  }

  template <int ST, bool ZIN, bool ZOUT, bool REG>
  __device__ __forceinline__ static void stages(cplx<T> (&v)[8], int j, cplx<T> *buf, const Tw *t,
                                                const cplx<T> *__restrict__ tw) {
    constexpr int R = plan_radix(N, P, ST);
    constexpr bool LAST = ST == NST - 1;
    if constexpr (ST > 0) twiddle_st<ST, REG>(v, j, t, tw);
    stage_dft<R, INV, ZIN && ST == 0, ZOUT && LAST, T>(v);
    if constexpr (!LAST) {
      cplx<T> *dst = SINGLE ? buf : buf + (ST & 1) * HALF;
      if (SINGLE) group_sync<TPF>();
      write_st<ST>(v, j, dst);
      group_sync<TPF>();
      read_all(v, j, dst);
      stages<ST + 1, ZIN, ZOUT, REG>(v, j, buf, t, tw);
    }
  }

  // v[u] = x[j + u*TPF] on entry, X[j + u*TPF] on exit.  buf: this group's LDS elements; twiddles
  // from registers.  ZIN: the input is zero from element N/2 on (v[4..7] are not read); ZOUT:
  // only the outputs below N/2 (v[0..3]) are produced.
  template <bool ZIN = false, bool ZOUT = false>
  __device__ static void run_tw(cplx<T> (&v)[8], int j, cplx<T> *buf, const Tw &t) {
    stages<0, ZIN, ZOUT, true>(v, j, buf, &t, nullptr);
    // a later call (or the caller's own LDS use) may overwrite the buffers this call read
    if constexpr (NST > 1) group_sync<TPF>();
  }

  // the same transform with the twiddles read from the table tw
  template <bool ZIN = false, bool ZOUT = false>
  __device__ static void run(cplx<T> (&v)[8], int j, cplx<T> *buf, const cplx<T> *__restrict__ tw) {
    stages<0, ZIN, ZOUT, false>(v, j, buf, nullptr, tw);
    if constexpr (NST > 1) group_sync<TPF>();
  }
};

// Two independent transforms of the same length and plan run interleaved by one FFT group: `a`
// in direction INVA and `b` in direction INVB, each with its own exchange buffer, sharing the
// register twiddles and the barriers of every exchange.  Each transform does exactly the
// arithmetic of FFT::run_tw with its own pruning flags (same results bit for bit); the
// interleaving gives the scheduler a second chain of work while the other waits on LDS.
// Wave-level transforms only (N <= 512).
template <typename T, int N, bool INVA, bool INVB, bool ZINA, bool ZOUTA, bool ZINB, bool ZOUTB, int P, int ST>
__device__ __forceinline__ void fft_dual_st(cplx<T> (&a)[8], cplx<T> (&b)[8], int j, cplx<T> *bufA, cplx<T> *bufB,
                                            const typename FFT<T, N, false, P>::Tw &t) {
  using FA = FFT<T, N, INVA, P>;
  using FB = FFT<T, N, INVB, P>;
  constexpr int R = plan_radix(N, P, ST);
  constexpr bool LAST = ST == FA::NST - 1;
  const auto &ta = *reinterpret_cast<const typename FA::Tw *>(&t);
  const auto &tb = *reinterpret_cast<const typename FB::Tw *>(&t);
  if constexpr (ST > 0) {
    FA::template twiddle_st<ST, true>(a, j, &ta, nullptr);
    FB::template twiddle_st<ST, true>(b, j, &tb, nullptr);
  }
  stage_dft<R, INVA, ZINA && ST == 0, ZOUTA && LAST, T>(a);
  stage_dft<R, INVB, ZINB && ST == 0, ZOUTB && LAST, T>(b);
  if constexpr (!LAST) {
    group_sync<FA::TPF>();
    FA::template write_st<ST>(a, j, bufA);
    FB::template write_st<ST>(b, j, bufB);
    group_sync<FA::TPF>();
    FA::read_all(a, j, bufA);
    FB::read_all(b, j, bufB);
    fft_dual_st<T, N, INVA, INVB, ZINA, ZOUTA, ZINB, ZOUTB, P, ST + 1>(a, b, j, bufA, bufB, t);
  }
}

template <typename T, int N, bool INVA, bool INVB, bool ZINA = false, bool ZOUTA = false, bool ZINB = false,
          bool ZOUTB = false, int P = 0>
__device__ __forceinline__ void fft_dual(cplx<T> (&a)[8], cplx<T> (&b)[8], int j, cplx<T> *bufA, cplx<T> *bufB,
                                         const typename FFT<T, N, false, P>::Tw &t) {
  static_assert(FFT<T, N, false, P>::WAVE, "fft_dual: wave-level transforms only");
  fft_dual_st<T, N, INVA, INVB, ZINA, ZOUTA, ZINB, ZOUTB, P, 0>(a, b, j, bufA, bufB, t);
  if constexpr (FFT<T, N, false, P>::NST > 1) group_sync<N / 8>();
}

}  // namespace ff

// gfx950 device code of the FFT beam-propagation z-march (included by the
// per-precision kernel units march_fp64.hip, march_fp32.hip, march_fp32s.hip,
// each of which instantiates the launch functions of one precision, and by
// bpm_march.hip for the deformation pre-pass).
//
// One workgroup advances one frequency slice through all Nz split steps
// (Eq. fov10, first-order splitting of Eq. fov4).  Both envelopes stay
// on-chip for the whole march: thread t of T = Nx/R threads keeps the R
// samples t + T*i (i = 0..R-1) of psi~_+ and of psi~_- in registers.  Each
// FFT along x is a Stockham autosort transform: radix-Rp butterflies in
// registers, one LDS exchange between passes (both envelopes exchanged under
// a single barrier), natural-order output landing back in the same register
// slots, so the propagator (a function of the bin K) and the coupling (a
// function of x) are register-local and need no extra exchange.  HBM traffic
// per slice-step is one row of the deformation table exp(i h u).
//
// There is no matrix-core work here: the step is FFT plus pointwise complex
// arithmetic, bound by VALU and LDS throughput.

#pragma once

#include <type_traits>
#include <utility>

#include "bpm_internal.h"

#define BPM_INLINE __device__ __forceinline__

// Multiply-add contraction only within one source expression (cmul,
// cmuladd, ...), never across statements: the rounding of a value then does
// not depend on how it is used later, so the two envelope instantiations of
// the split march compute bitwise the same partner values.
#pragma clang fp contract(on)

namespace bpm {
namespace {

// ---------------------------------------------------------------- complex --

template <class T>
struct cx {
  T x, y;
};

template <class T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <class T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return {a.x - b.x, a.y - b.y};
}
template <class T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <class T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// p*x + q*y with the real parts and imaginary parts each one FMA chain
template <class T>
__device__ __forceinline__ cx<T> cmuladd(cx<T> p, cx<T> x, cx<T> q, cx<T> y) {
  return {p.x * x.x - p.y * x.y + q.x * y.x - q.y * y.y,
          p.x * x.y + p.y * x.x + q.x * y.y + q.y * y.x};
}
// multiply by -i (forward transform) or +i (inverse transform)
template <bool INV, class T>
__device__ __forceinline__ cx<T> rot(cx<T> a) {
  if constexpr (INV)
    return {-a.y, a.x};
  else
    return {a.y, -a.x};
}

template <class D, class S>
__device__ __forceinline__ cx<D> conv(cx<S> a) {
  return {static_cast<D>(a.x), static_cast<D>(a.y)};
}

// A twiddle factor w, held in FP64 for every precision.  A twiddle is the
// same fixed number at every z-step, so a plain FP32 rounding of it (~3e-8)
// is an error of the step operator itself: repeated Nz times, it grows
// linearly (measured: relL2 1.8e-4 after 4000 steps in vacuum).  In FP32
// arithmetic the product x w is therefore formed in FP64 and rounded once,
// which leaves only the rounding of the data: that error does not add up
// coherently and grows like sqrt(Nz) (9.7e-6 after 4000 steps).  On MI355X
// the two conversions and four FP64 FMAs cost the same issue slots as an
// unevaluated hi + lo FP32 pair, which in the compiled code did not remove
// the drift.
template <class T>
struct Tw {
  cx<double> w;
  BPM_INLINE static Tw from(double c, double s) { return {{c, s}}; }
  BPM_INLINE cx<T> mul(cx<T> x) const {
    if constexpr (sizeof(T) == 8) {
      return cmul(x, w);
    } else {
      const cx<double> r = cmul(cx<double>{x.x, x.y}, w);
      return {static_cast<float>(r.x), static_cast<float>(r.y)};
    }
  }
  BPM_INLINE cx<T> mulc(cx<T> x) const {
    if constexpr (sizeof(T) == 8) {
      return cmulc(x, w);
    } else {
      const cx<double> r = cmulc(cx<double>{x.x, x.y}, w);
      return {static_cast<float>(r.x), static_cast<float>(r.y)};
    }
  }
};

// ------------------------------------------------------- small DFT kernels --
// Forward kernel exp(-2 pi i n k / R), inverse exp(+2 pi i n k / R); no
// scaling.  Outputs are in natural order.

constexpr double kCos16[16] = {
    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
    0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977,
    0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674};

// a * W16^J with W16 = exp(-+2 pi i / 16)
template <int J, bool INV, class T>
__device__ __forceinline__ cx<T> tw16(cx<T> a) {
  constexpr int j = J & 15;
  if constexpr (j == 0) {
    return a;
  } else if constexpr (j == 4) {
    return rot<INV>(a);
  } else if constexpr (j == 8) {
    return {-a.x, -a.y};
  } else if constexpr (j == 12) {
    return rot<!INV>(a);
  } else {
    constexpr double c = kCos16[j];
    constexpr double s = kCos16[(j + 12) & 15];  // sin(2 pi j / 16)
    constexpr double si = INV ? s : -s;
    if constexpr (sizeof(T) == 4) {
      // FP64 product rounded once, as for the pass twiddles (see Tw)
      const double xr = a.x, xi = a.y;
      return {static_cast<float>(xr * c - xi * si),
              static_cast<float>(xr * si + xi * c)};
    } else {
      const T wr = static_cast<T>(c);
      const T wi = static_cast<T>(si);
      return {a.x * wr - a.y * wi, a.x * wi + a.y * wr};
    }
  }
}

template <bool INV, class T>
__device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  const cx<T> t = a;
  a = t + b;
  b = t - b;
}

template <bool INV, class T>
__device__ __forceinline__ void dft4(cx<T>& x0, cx<T>& x1, cx<T>& x2,
                                     cx<T>& x3) {
  const cx<T> t0 = x0 + x2, t1 = x0 - x2, t2 = x1 + x3;
  const cx<T> t3 = rot<INV>(x1 - x3);
  x0 = t0 + t2;
  x2 = t0 - t2;
  x1 = t1 + t3;
  x3 = t1 - t3;
}

template <int R, bool INV, class T>
__device__ __forceinline__ void dft(cx<T> (&v)[R]) {
  if constexpr (R == 2) {
    dft2<INV>(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4<INV>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    // even/odd split: X_k = E_k + W8^k O_k, X_{k+4} = E_k - W8^k O_k
    dft4<INV>(v[0], v[2], v[4], v[6]);
    dft4<INV>(v[1], v[3], v[5], v[7]);
    const cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    const cx<T> o0 = v[1];
    const cx<T> o2 = tw16<4, INV>(v[5]);
    v[0] = e0 + o0;
    v[4] = e0 - o0;
    v[2] = e2 + o2;
    v[6] = e2 - o2;
    if constexpr (sizeof(T) == 8) {
      // W8^{+-1} = r (1 -+ i) and W8^{+-3} = r (-1 -+ i), r = 1/sqrt(2):
      // e +- W o = e +- r t with t = (o.x -+ ..., ...), so each output is
      // one multiply-add (two adds and four FMAs per pair instead of eight
      // operations)
      constexpr T r = T(0.70710678118654752440);
      const cx<T> a = v[3], b = v[7];
      const cx<T> t1 = INV ? cx<T>{a.x - a.y, a.y + a.x} : cx<T>{a.x + a.y, a.y - a.x};
      const cx<T> t3 = INV ? cx<T>{-b.x - b.y, b.x - b.y} : cx<T>{b.y - b.x, -b.x - b.y};
      v[1] = {e1.x + r * t1.x, e1.y + r * t1.y};
      v[5] = {e1.x - r * t1.x, e1.y - r * t1.y};
      v[3] = {e3.x + r * t3.x, e3.y + r * t3.y};
      v[7] = {e3.x - r * t3.x, e3.y - r * t3.y};
    } else {
      const cx<T> o1 = tw16<2, INV>(v[3]);
      const cx<T> o3 = tw16<6, INV>(v[7]);
      v[1] = e1 + o1;
      v[5] = e1 - o1;
      v[3] = e3 + o3;
      v[7] = e3 - o3;
    }
  } else if constexpr (R == 16) {
    // 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
    v[5] = tw16<1, INV>(v[5]);
    v[6] = tw16<2, INV>(v[6]);
    v[7] = tw16<3, INV>(v[7]);
    v[9] = tw16<2, INV>(v[9]);
    v[10] = tw16<4, INV>(v[10]);
    v[11] = tw16<6, INV>(v[11]);
    v[13] = tw16<3, INV>(v[13]);
    v[14] = tw16<6, INV>(v[14]);
    v[15] = tw16<9, INV>(v[15]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    cx<T> o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = o[i];
  } else {
    static_assert(R == 2, "unsupported radix");
  }
}

// ------------------------------------------------------ double-double math --
// Used once per slice and bin to form the propagator phase dz*kz, which is
// ~2.5e4 rad at typical sizes: a plain FP64 evaluation would carry ~1e-12 rad
// of error that every one of the Nz steps repeats.  Evaluated to ~1e-30
// relative and reduced modulo 2 pi before the final FP64 rounding.

struct dd {
  double hi, lo;
};

#pragma clang fp contract(off)

__device__ __forceinline__ dd quick_two_sum(double a, double b) {
  const double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ dd two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
  const double p = a * b;
  return {p, __fma_rn(a, b, -p)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  const dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return quick_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
  dd p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return quick_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_div_d(dd a, double b) {
  const double q1 = a.hi / b;
  const dd p = two_prod(q1, b);
  const double r = ((a.hi - p.hi) - p.lo) + a.lo;
  return quick_two_sum(q1, r / b);
}
__device__ __forceinline__ dd dd_sqrt(dd a) {
  const double s = sqrt(a.hi);
  const dd s2 = two_prod(s, s);
  const double r = (((a.hi - s2.hi) - s2.lo) + a.lo) / (2.0 * s);
  return quick_two_sum(s, r);
}

#pragma clang fp contract(on)

// 2 pi as a double-double
constexpr double kTwoPiHi = 6.283185307179586232;
constexpr double kTwoPiLo = 2.4492935982947064e-16;

// exp(i frac dz sqrt(k^2 - (K_m + band h/2)^2)) / Nx for signed bin m,
// K_m = 2 pi m / (Nx dx); principal root (decay) for evanescent waves.
__device__ cx<double> propagator(int m, int Nx, double dx, double k,
                                 double h_half, double band, double dz,
                                 double frac) {
  const dd two_pi = {kTwoPiHi, kTwoPiLo};
  const dd K = dd_div_d(dd_mul_d(two_pi, static_cast<double>(m)),
                        static_cast<double>(Nx) * dx);
  const dd kp = dd_add(K, dd{band * h_half, 0.0});
  const dd kz2 = dd_add(two_prod(k, k), dd_neg(dd_mul(kp, kp)));
  const double inv_n = 1.0 / static_cast<double>(Nx);
  if (kz2.hi < 0.0) {
    const double decay = frac * dz * sqrt(-kz2.hi);
    return {exp(-decay) * inv_n, 0.0};
  }
  // sub-step length frac*dz kept exact (two_prod) for fractional sub-steps
  dd phi = frac == 1.0 ? dd_mul_d(dd_sqrt(kz2), dz)
                       : dd_mul(dd_sqrt(kz2), two_prod(frac, dz));
  const double n = floor(phi.hi / kTwoPiHi);
  phi = dd_add(phi, dd_neg(dd_mul_d(two_pi, n)));
  if (phi.hi < 0.0) phi = dd_add(phi, two_pi);
  if (phi.hi >= kTwoPiHi) phi = dd_add(phi, dd_neg(two_pi));
  const double r = phi.hi + phi.lo;
  double s, c;
  sincos(r, &s, &c);
  return {c * inv_n, s * inv_n};
}

// ---------------------------------------------------------------- barrier --
// Workgroup barrier ordering LDS traffic only: global loads in flight (the
// prefetched deformation row) are not drained by it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Orders LDS accesses of one wavefront in the compiler only: the hardware
// executes a wavefront's LDS instructions in program order.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
}

// -------------------------------------------------------------- precision --

template <int PREC>
struct Prec;
template <>
struct Prec<BPM_PREC_FP64> {
  using CT = double;  // butterfly arithmetic
  using ST = double;  // LDS, fields and deformation table
};
template <>
struct Prec<BPM_PREC_FP32> {
  using CT = float;
  using ST = float;
};
template <>
struct Prec<BPM_PREC_FP32S> {
  using CT = double;
  using ST = float;
};

template <class T>
struct vec2;
template <>
struct vec2<float> {
  using type = float2;
};
template <>
struct vec2<double> {
  using type = double2;
};


// ------------------------------------------------------- splitting scheme --
// Sub-steps of one z-step for the splitting orders of Eq. split-op:
// sub-step s is A(a_s dz) (skipped where a_s = 0) followed by B(b_s dz).
//   order 1: A(dz) B(dz)
//   order 2: B(dz/2) A(dz) B(dz/2)
//   order 4: B(t dz/2) A(t dz) B((1-t) dz/2) A((1-2t) dz) B((1-t) dz/2)
//            A(t dz) B(t dz/2),  t = 1/(2 - 2^(1/3))
// The a_s are MarchParams::a_frac and the B constants SliceConst::d[s].
// Crystal flags of step `row` at this thread's x samples first + stride i:
// the general mask row when the plan has one, else the slab flags.
template <int R, int N, bool MASKED>
BPM_INLINE void crystal_row(const MarchParams& p, int row, int first, int stride,
                            const bool (&slab)[R], bool (&out)[R]) {
  if constexpr (MASKED) {
    const unsigned char* m = p.mask + size_t(row) * N + first;
#pragma unroll
    for (int i = 0; i < R; ++i) out[i] = m[stride * i] != 0;
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) out[i] = slab[i];
  }
}

template <int ORDER>
struct Scheme {
  static_assert(ORDER == 1 || ORDER == 2 || ORDER == 4, "split order 1, 2 or 4");
  static constexpr int NS = ORDER;                      // sub-steps per step
  static constexpr int NP = ORDER == 4 ? 2 : 1;         // distinct A lengths
  static constexpr bool has_a(int s) { return ORDER == 1 || s > 0; }
  // propagator set of sub-step s, and the sub-step whose a_s defines set q
  static constexpr int pset(int s) { return ORDER == 4 && s == 2 ? 1 : 0; }
  static constexpr int pdef(int q) { return ORDER == 1 ? 0 : (q == 0 ? 1 : 2); }
};

// The thread index as the compiler sees it inside a transform pass: an
// opaque copy when the twiddle source sets kOpaqueIndex (then the pass's LDS
// addresses are formed in the pass instead of being kept live across
// passes), the index itself otherwise.
template <class TWS, class = void>
struct wants_opaque : std::false_type {};
template <class TWS>
struct wants_opaque<TWS, std::void_t<decltype(TWS::kOpaqueIndex)>>
    : std::integral_constant<bool, TWS::kOpaqueIndex> {};
template <class TWS>
BPM_INLINE int opaque_index(int t) {
  if constexpr (wants_opaque<TWS>::value) {
    asm volatile("" : "+v"(t));
    __builtin_assume(t >= 0);     // a thread index: divisions become shifts
  }
  return t;
}

// The thread index of one z-step of a march, opaque to the compiler when the
// transform sets kOpaqueStep: the transform's LDS addresses are then formed
// in every step instead of being hoisted out of the step loop and kept live
// for the whole march.
template <class Tr, class = void>
struct opaque_steps : std::false_type {};
template <class Tr>
struct opaque_steps<Tr, std::void_t<decltype(Tr::kOpaqueStep)>>
    : std::integral_constant<bool, Tr::kOpaqueStep> {};
template <class Tr>
BPM_INLINE int opaque_step(int t) {
  if constexpr (opaque_steps<Tr>::value) asm volatile("" : "+v"(t));
  return t;
}

// ------------------------------------------------------------- the march --

template <int PREC, int N_, int R_, int... RADS>
struct March {
  static constexpr bool kSplit = false;
  static constexpr bool kLateRow = false;
  static constexpr int N = N_;  // transform length
  static constexpr int R = R_;  // samples per thread per envelope
  using CT = typename Prec<PREC>::CT;
  using ST = typename Prec<PREC>::ST;
  using SV = typename vec2<ST>::type;
  static constexpr int T = N / R;             // threads per slice
  static constexpr int NP = sizeof...(RADS);  // Stockham passes per FFT
  static constexpr int rad[NP] = {RADS...};
  static constexpr int prod_rad() {
    int p = 1;
    for (int i = 0; i < NP; ++i) p *= rad[i];
    return p;
  }
  static_assert(prod_rad() == N, "radices must multiply to N");
  static constexpr int ns(int p) {  // sub-transform length before pass p
    int s = 1;
    for (int i = 0; i < p; ++i) s *= rad[i];
    return s;
  }
  static constexpr int tw_off(int p) {  // first twiddle of pass p
    int o = 0;
    for (int i = 1; i < p; ++i) o += (R / rad[i]) * (rad[i] - 1);
    return o;
  }
  static constexpr int NTW = tw_off(NP) > 0 ? tw_off(NP) : 1;
  // LDS address of sample idx in the exchange after pass p: one gap of Ns
  // slots every max(Rp Ns, L) samples, L = samples per 128-byte bank row.
  // The pass writes x[(Rp a + r) Ns + b] for consecutive butterflies
  // (b = jb mod Ns, a = jb / Ns) and the next pass reads consecutive samples;
  // with the gaps both hit distinct banks across each group of L lanes.
  static constexpr int kL = 128 / int(sizeof(SV));
  static constexpr int pad_div(int p) {
    return rad[p] * ns(p) > kL ? rad[p] * ns(p) : kL;
  }
  static constexpr int env_slots() {
    int m = N;
    for (int p = 0; p + 1 < NP; ++p) {
      const int e = N + ns(p) * ((N - 1) / pad_div(p)) ;
      m = e > m ? e : m;
    }
    return m;
  }
  static constexpr int kEnv = env_slots();
  // Two LDS buffers (one barrier per exchange) when they fit in 160 KiB.
  static constexpr size_t kEnvBytes = size_t(kEnv) * sizeof(SV);
  static constexpr int NBUF = (4 * kEnvBytes <= 160 * 1024) ? 2 : 1;
  static constexpr size_t kLdsBytes = NBUF * 2 * kEnvBytes;

  using Reg = cx<CT>[R];

  BPM_INLINE static void store(SV* lds, int idx, cx<CT> v) {
    SV s;
    s.x = static_cast<ST>(v.x);
    s.y = static_cast<ST>(v.y);
    lds[idx] = s;
  }
  BPM_INLINE static cx<CT> load(const SV* lds, int idx) {
    const SV s = lds[idx];
    return {static_cast<CT>(s.x), static_cast<CT>(s.y)};
  }
  template <class VT>
  BPM_INLINE static cx<VT> load_as(const SV* lds, int idx) {
    const SV s = lds[idx];
    return {static_cast<VT>(s.x), static_cast<VT>(s.y)};
  }

  // Stockham pass P (radix rad[P], sub-length Ns): butterfly jb reads
  // x[jb + r N/Rp], applies twiddles W_{Ns Rp}^{r (jb mod Ns)}, transforms,
  // and writes x[(jb/Ns) Ns Rp + jb mod Ns + r Ns].  Thread t owns
  // butterflies jb = t + s T and, on input, register slot s + r (R/Rp).
  // Exchange synchronisation: kDouble / kSingle -- a work-group barrier per
  // exchange with two / one LDS buffers; kWave -- the T threads are one
  // wavefront, whose LDS operations execute in program order, so a
  // compiler-only fence is enough and one buffer is reused.
  enum { kDouble = 0, kSingle = 1, kWave = 2 };
  static constexpr int kSync = NBUF == 2 ? kDouble : kSingle;

  // Twiddle W_{Ns Rp}^{r (jb mod Ns)} of butterfly jb = t + s T of pass P,
  // from a register array Tw<CT>[NTW] (one entry per (s, r) of this thread)
  // or from a TwTable in LDS.
  template <int P, class TWS>
  BPM_INLINE static Tw<CT> twiddle(const TWS& tw, int t, int s, int r) {
    if constexpr (std::is_array<TWS>::value)
      return tw[tw_off(P) + s * (rad[P] - 1) + (r - 1)];
    else
      return tw.template get<P>(t, s, r);
  }

  // Stockham pass P over NE envelopes v[e] (LDS region e at lds + e kEnv).
  // tw: the pass twiddles, a register array Tw<CT>[NTW] or a TwTable.  The
  // registers v hold the arithmetic type CT, or (VT = ST) the storage type,
  // widened to CT per butterfly: the same rounding (every value between
  // passes has been through an LDS store), half the registers.
  template <int P, bool INV, int SYNC, int NE, class TWS, class VT>
  BPM_INLINE static void pass_n(cx<VT> (&v)[NE][R], const TWS& tw,
                                SV* lds, int t_in, int& xbuf) {
    // a twiddle source may ask for the thread index to be opaque per pass,
    // so that the pass's LDS addresses are formed where they are used
    const int t = opaque_index<TWS>(t_in);
    constexpr int Rp = rad[P];
    constexpr int Ns = ns(P);
    constexpr int G = R / Rp;
    constexpr bool last = (P == NP - 1);
    constexpr int D = pad_div(P);
    SV* base_lds = lds + (SYNC == kDouble ? xbuf * NE * kEnv : 0);
#pragma unroll
    for (int s = 0; s < G; ++s) {
      cx<CT> u[NE][Rp];
#pragma unroll
      for (int e = 0; e < NE; ++e)
#pragma unroll
        for (int r = 0; r < Rp; ++r) u[e][r] = conv<CT>(v[e][s + r * G]);
      if constexpr (P > 0) {
#pragma unroll
        for (int r = 1; r < Rp; ++r) {
          const Tw<CT> w = twiddle<P>(tw, t, s, r);
#pragma unroll
          for (int e = 0; e < NE; ++e)
            u[e][r] = INV ? w.mulc(u[e][r]) : w.mul(u[e][r]);
        }
      }
#pragma unroll
      for (int e = 0; e < NE; ++e) dft<Rp, INV>(u[e]);
      if constexpr (last) {
#pragma unroll
        for (int e = 0; e < NE; ++e)
#pragma unroll
          for (int r = 0; r < Rp; ++r) v[e][s + r * G] = conv<VT>(u[e][r]);
      } else {
        const int jb = t + s * T;
        const int base = (jb / Ns) * Ns * Rp + (jb % Ns);
#pragma unroll
        for (int r = 0; r < Rp; ++r) {
          const int idx = base + r * Ns;
          const int slot = idx + Ns * (idx / D);
#pragma unroll
          for (int e = 0; e < NE; ++e) store(base_lds + e * kEnv, slot, u[e][r]);
        }
      }
    }
    if constexpr (!last) {
      if constexpr (SYNC == kWave)
        wave_sync();
      else
        lds_barrier();
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int idx = t + T * i;
        const int slot = idx + Ns * (idx / D);
#pragma unroll
        for (int e = 0; e < NE; ++e) v[e][i] = load_as<VT>(base_lds + e * kEnv, slot);
      }
      if constexpr (SYNC == kSingle) {
        lds_barrier();
      } else if constexpr (SYNC == kWave) {
        wave_sync();
      } else {
        xbuf ^= 1;
      }
    }
  }

  template <bool INV, int SYNC, int NE, class TWS, class VT, int... P>
  BPM_INLINE static void fft_impl(cx<VT> (&v)[NE][R], const TWS& tw,
                                  SV* lds, int t, int& xbuf,
                                  std::integer_sequence<int, P...>) {
    (pass_n<P, INV, SYNC, NE>(v, tw, lds, t, xbuf), ...);
  }
  // In-place transform of NE envelopes (registers of type CT or ST).
  template <bool INV, int SYNC, int NE, class TWS, class VT>
  BPM_INLINE static void fft_n(cx<VT> (&v)[NE][R], const TWS& tw,
                               SV* lds, int t, int& xbuf) {
    fft_impl<INV, SYNC, NE>(v, tw, lds, t, xbuf,
                            std::make_integer_sequence<int, NP>{});
  }
  // Both envelopes (psi~_+ in a, psi~_- in b).
  template <bool INV, int SYNC = kSync, class TWS>
  BPM_INLINE static void fft(Reg& a, Reg& b, const TWS& tw, SV* lds,
                             int t, int& xbuf) {
    cx<CT> v[2][R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      v[0][i] = a[i];
      v[1][i] = b[i];
    }
    fft_n<INV, SYNC, 2>(v, tw, lds, t, xbuf);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      a[i] = v[0][i];
      b[i] = v[1][i];
    }
  }

  // Twiddles W_{Ns Rp}^{r (jb mod Ns)} of every pass after the first.
  template <int P>
  __device__ static void twiddles_pass(Tw<CT> (&tw)[NTW], int t) {
    if constexpr (P > 0) {
      constexpr int Rp = rad[P];
      constexpr int Ns = ns(P);
      constexpr int G = R / Rp;
#pragma unroll
      for (int s = 0; s < G; ++s) {
        const int jb = t + s * T;
        const int j = jb % Ns;
#pragma unroll
        for (int r = 1; r < Rp; ++r) {
          // exp(-2 pi i r j / (Ns Rp)); sincospi keeps the argument exact
          double sn, cs;
          sincospi(-2.0 * double(r * j) / double(Ns * Rp), &sn, &cs);
          tw[tw_off(P) + s * (Rp - 1) + (r - 1)] = Tw<CT>::from(cs, sn);
        }
      }
    }
  }
  template <int... P>
  __device__ static void twiddles_impl(Tw<CT> (&tw)[NTW], int t,
                                       std::integer_sequence<int, P...>) {
    (twiddles_pass<P>(tw, t), ...);
  }

  // Twiddles of a one-wavefront transform (T = 64) kept in LDS instead of
  // registers, as a table [NTW][64] of FP64 values indexed by the lane
  // (each lane reads its own entries, so the reads never conflict); shared
  // by every wavefront of the work group.
  static constexpr size_t kLaneTableBytes = size_t(NTW) * 64 * sizeof(cx<double>);
  struct TwTable {
    const cx<double>* base;
    template <int P>
    BPM_INLINE Tw<CT> get(int t, int s, int r) const {
      return Tw<CT>{base[(tw_off(P) + s * (rad[P] - 1) + (r - 1)) * 64 + t]};
    }
  };
  __device__ static void fill_lane_table(cx<double>* table, int lane) {
    static_assert(T == 64, "a twiddle table serves one-wavefront transforms");
    Tw<CT> tw[NTW];
    twiddles_impl(tw, lane, std::make_integer_sequence<int, NP>{});
#pragma unroll
    for (int k = 0; k < NTW; ++k) table[k * 64 + lane] = tw[k].w;
  }

  // The same twiddles with one FP64 entry per distinct value, for where LDS
  // is too tight for the lane table: pass p holds W_{Ns Rp}^{r j} for
  // r = 1..Rp-1, j = 0..Ns-1 (butterfly jb reads entry j = jb mod Ns).
  // Lanes with the same j read the same address and consecutive j are
  // consecutive entries.  The values are the ones the register twiddles
  // hold, bit for bit.
  static constexpr int tab_off(int p) {
    int o = 0;
    for (int q = 1; q < p; ++q) o += (rad[q] - 1) * ns(q);
    return o;
  }
  static constexpr int kTabEntries = tab_off(NP) > 0 ? tab_off(NP) : 1;
  static constexpr size_t kTableBytes = size_t(kTabEntries) * sizeof(cx<double>);
  struct TwTableJ {
    const cx<double>* base;
    template <int P>
    BPM_INLINE Tw<CT> get(int t, int s, int r) const {
      constexpr int Ns = ns(P);
      const int j = (t + s * T) & (Ns - 1);   // Ns is a power of two
      return Tw<CT>{base[tab_off(P) + (r - 1) * Ns + j]};
    }
  };
  template <int P>
  __device__ static void fill_pass(cx<double>* table, int t, int nthreads) {
    if constexpr (P > 0) {
      constexpr int Rp = rad[P];
      constexpr int Ns = ns(P);
      for (int e = t; e < (Rp - 1) * Ns; e += nthreads) {
        const int r = 1 + e / Ns, j = e % Ns;
        double sn, cs;
        sincospi(-2.0 * double(r * j) / double(Ns * Rp), &sn, &cs);
        table[tab_off(P) + e] = {cs, sn};
      }
    }
  }
  template <int... P>
  __device__ static void fill_impl(cx<double>* table, int t, int nthreads,
                                   std::integer_sequence<int, P...>) {
    (fill_pass<P>(table, t, nthreads), ...);
  }
  // Filled by threads t = 0..nthreads-1 of the work group; a barrier must
  // follow before any wavefront reads it.
  __device__ static void fill_table_j(cx<double>* table, int t, int nthreads) {
    fill_impl(table, t, nthreads, std::make_integer_sequence<int, NP>{});
  }

  // Transform interface used by march_slice: per-thread context (twiddles),
  // the DFT bin held in register slot i after forward(), and in-place
  // forward / inverse transforms of both envelopes.
  struct Ctx {
    Tw<CT> tw[NTW];
    int xbuf;
  };
  __device__ static void init(Ctx& c, int t, SV* = nullptr) {
    twiddles_impl(c.tw, t, std::make_integer_sequence<int, NP>{});
    c.xbuf = 0;
  }
  BPM_INLINE static int bin(int t, int i) { return t + T * i; }
  BPM_INLINE static void forward(Reg& a, Reg& b, Ctx& c, SV* lds, int t) {
    fft<false>(a, b, c.tw, lds, t, c.xbuf);
  }
  BPM_INLINE static void inverse(Reg& a, Reg& b, Ctx& c, SV* lds, int t) {
    fft<true>(a, b, c.tw, lds, t, c.xbuf);
  }
};

// Four-step transform of N = W M: a radix-W DFT across the W wavefronts of
// the slice (in registers), one work-group exchange per direction, and an
// M-point Stockham transform inside each wavefront whose exchanges need no
// work-group barrier.  Per z-step that is 2 barriers instead of one per
// Stockham pass, and between them the wavefronts run independently, so one
// wavefront's LDS traffic overlaps the others' arithmetic.
//
// Layouts.  x-space (input and output): thread t keeps x[t + T i], i < R,
// the same as the Stockham path.  With m_j = t + T j (j < J = R/W) and
// n = m + M q, slot j + J q holds x[m_j + M q].  Forward: DFT over q, twiddle
// W_N^{m k1}, exchange so that wavefront k1 holds y[m][k1] for all m (lane l,
// slot i -> m = l + 64 i), then the M-point transform over m.  Slot i of
// lane l in wavefront w ends with bin K = w + W (l + 64 i).
template <int PREC, int W, class In, bool TWL = false>
struct FourStep {
  static constexpr bool kSplit = false;
  // fetch the deformation row after the forward transform (fewer live
  // registers across it) where the register file is the limit
  static constexpr bool kLateRow = TWL;
  static constexpr bool kOpaqueStep = PREC != BPM_PREC_FP64;
  using CT = typename Prec<PREC>::CT;
  using ST = typename Prec<PREC>::ST;
  using SV = typename vec2<ST>::type;
  static_assert(In::T == 64, "the in-wave transform must use one wavefront");
  static constexpr int M = In::N;
  static constexpr int R = In::R;
  static constexpr int N = W * M;
  static constexpr int T = 64 * W;
  static constexpr int J = R / W;
  static_assert(W == 1 || (R % W == 0 && W <= 8), "unsupported wave count");
  static constexpr int kRegion = 2 * In::kEnv;  // per wavefront: a then b
  static constexpr size_t kG = size_t(W) * kRegion;
  static constexpr size_t kGp = W > 1 ? size_t(W) * 2 * M : 0;
  // Separate forward and inverse exchange buffers when they fit; otherwise
  // one buffer and two extra barriers per step.
  static constexpr bool kAlias = (kG + kGp) * sizeof(SV) + (TWL ? In::kLaneTableBytes : 0) >
                                 160 * 1024;
  // TWL: the in-wavefront twiddles live in an LDS table after the exchange
  // buffers (frees their registers where the state fills the register file)
  static constexpr size_t kTabOff = ((kAlias ? kG : kG + kGp) * sizeof(SV) + 15) / 16 * 16;
  static constexpr size_t kLdsBytes = kTabOff + (TWL ? In::kLaneTableBytes : 0);
  static_assert(kLdsBytes <= 160 * 1024, "four-step march does not fit in LDS");
  static constexpr int NTWX = W > 1 ? J * (W - 1) : 1;
  using Reg = cx<CT>[R];

  struct Ctx {
    typename In::Ctx in;
    Tw<CT> twx[NTWX];
  };
  BPM_INLINE static cx<double>* table(SV* lds) {
    return reinterpret_cast<cx<double>*>(reinterpret_cast<char*>(lds) + kTabOff);
  }
  __device__ static void init(Ctx& c, int t, SV* lds) {
    if constexpr (TWL) {
      if (t < 64) In::fill_lane_table(table(lds), t);
      c.in.xbuf = 0;
      lds_barrier();
    } else {
      In::init(c.in, t & 63);
    }
    if constexpr (W > 1) {
#pragma unroll
      for (int j = 0; j < J; ++j)
#pragma unroll
        for (int k1 = 1; k1 < W; ++k1) {
          double sn, cs;
          sincospi(-2.0 * double((t + T * j) * k1) / double(N), &sn, &cs);
          c.twx[j * (W - 1) + k1 - 1] = Tw<CT>::from(cs, sn);
        }
    }
  }
  BPM_INLINE static int bin(int t, int i) {
    return (t >> 6) + W * ((t & 63) + 64 * i);
  }

  BPM_INLINE static void forward(Reg& a, Reg& b, Ctx& c, SV* lds, int t) {
    const int wv = t >> 6, l = t & 63;
    SV* own = lds + wv * kRegion;
    if constexpr (W > 1) {
#pragma unroll
      for (int j = 0; j < J; ++j) {
        cx<CT> va[W], vb[W];
#pragma unroll
        for (int q = 0; q < W; ++q) {
          va[q] = a[j + J * q];
          vb[q] = b[j + J * q];
        }
        dft<W, false>(va);
        dft<W, false>(vb);
#pragma unroll
        for (int k1 = 0; k1 < W; ++k1) {
          if (k1 > 0) {
            const Tw<CT> w = c.twx[j * (W - 1) + k1 - 1];
            va[k1] = w.mul(va[k1]);
            vb[k1] = w.mul(vb[k1]);
          }
          In::store(lds + k1 * kRegion, t + T * j, va[k1]);
          In::store(lds + k1 * kRegion + In::kEnv, t + T * j, vb[k1]);
        }
      }
      lds_barrier();
#pragma unroll
      for (int i = 0; i < R; ++i) {
        a[i] = In::load(own, l + 64 * i);
        b[i] = In::load(own + In::kEnv, l + 64 * i);
      }
      wave_sync();
    }
    if constexpr (TWL)
      In::template fft<false, In::kWave>(a, b, typename In::TwTable{table(lds)}, own, l,
                                         c.in.xbuf);
    else
      In::template fft<false, In::kWave>(a, b, c.in.tw, own, l, c.in.xbuf);
  }

  BPM_INLINE static void inverse(Reg& a, Reg& b, Ctx& c, SV* lds, int t) {
    const int wv = t >> 6, l = t & 63;
    SV* own = lds + wv * kRegion;
    if constexpr (TWL)
      In::template fft<true, In::kWave>(a, b, typename In::TwTable{table(lds)}, own, l,
                                        c.in.xbuf);
    else
      In::template fft<true, In::kWave>(a, b, c.in.tw, own, l, c.in.xbuf);
    if constexpr (W > 1) {
      SV* gp = kAlias ? lds : lds + kG;
      constexpr int kStride = kAlias ? kRegion : 2 * M;
      constexpr int kB = kAlias ? In::kEnv : M;
      if constexpr (kAlias) lds_barrier();  // all wavefronts done with scratch
#pragma unroll
      for (int i = 0; i < R; ++i) {
        In::store(gp + wv * kStride, l + 64 * i, a[i]);
        In::store(gp + wv * kStride + kB, l + 64 * i, b[i]);
      }
      lds_barrier();
#pragma unroll
      for (int j = 0; j < J; ++j) {
        cx<CT> va[W], vb[W];
#pragma unroll
        for (int k1 = 0; k1 < W; ++k1) {
          va[k1] = In::load(gp + k1 * kStride, t + T * j);
          vb[k1] = In::load(gp + k1 * kStride + kB, t + T * j);
          if (k1 > 0) {
            const Tw<CT> w = c.twx[j * (W - 1) + k1 - 1];
            va[k1] = w.mulc(va[k1]);
            vb[k1] = w.mulc(vb[k1]);
          }
        }
        dft<W, true>(va);
        dft<W, true>(vb);
#pragma unroll
        for (int q = 0; q < W; ++q) {
          a[j + J * q] = va[q];
          b[j + J * q] = vb[q];
        }
      }
      if constexpr (kAlias) lds_barrier();  // exchange read before reuse
    }
  }
};

// Envelope-split four-step march of one slice: 2 W wavefronts.  In k space
// wavefronts 0..W-1 carry psi~_+ and W..2W-1 carry psi~_-, each with an
// M-point in-wavefront transform of its own envelope.  In x space the T = 2 W
// 64 threads share the samples instead: thread t holds BOTH envelopes at
// x = t + T s, s < R/2, so the cross-wavefront radix-W steps, the twiddles
// and the coupling are each done once per sample, and the coupling needs no
// exchange of its own: two work-group barriers per z-step.  Twice the
// wavefronts of FourStep at half the registers each, so two wavefronts share
// every SIMD and hide each other's LDS latency.  The envelope of the
// in-wavefront part is a template parameter (every wavefront holds one
// envelope there), so no per-sample selects remain.
//
// LDS: 2W regions, one per wavefront, each the forward exchange target
// (M samples) and afterwards that wavefront's in-wave exchange buffer, then
// the inverse exchange (2W M samples), then (TWL) the in-wavefront twiddle
// table, which frees their registers where the state fills the register
// file (Nx = 4096: W = 4 with a 1024-point in-wavefront transform).
template <int PREC, int W, class In, bool TWL = false>
struct Split4 {
  using CT = typename Prec<PREC>::CT;
  using ST = typename Prec<PREC>::ST;
  using SV = typename vec2<ST>::type;
  using IV = typename In::SV;
  static_assert(In::T == 64 && W >= 2, "split march needs W >= 2 wavefronts");
  static constexpr bool kSplit = true;
  static constexpr int M = In::N;
  static constexpr int R = In::R;
  static constexpr int N = W * M;
  static constexpr int T0 = 64 * W;   // threads per envelope
  static constexpr int T = 2 * T0;
  static constexpr int J = R / W;
  static_assert(R % W == 0, "");
  static constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
  static constexpr size_t kRegionBytes =
      (cmax(size_t(M) * sizeof(SV), size_t(In::kEnv) * sizeof(IV)) + 15) / 16 * 16;
  static constexpr size_t kGBytes = size_t(2) * W * kRegionBytes;
  static constexpr size_t kTabOff = kGBytes + size_t(2) * W * M * sizeof(SV);
  static constexpr size_t kLdsBytes = kTabOff + (TWL ? In::kTableBytes : 0);
  static_assert(kLdsBytes <= 160 * 1024, "split march does not fit in LDS");
  static_assert(kTabOff % 16 == 0, "twiddle table alignment");

  BPM_INLINE static cx<double>* table(SV* lds) {
    return reinterpret_cast<cx<double>*>(reinterpret_cast<char*>(lds) + kTabOff);
  }
  // The in-wavefront transform of one envelope (z: this lane's M/64 bins).
  template <bool INV>
  BPM_INLINE static void wave_fft(cx<CT> (&z)[1][R], typename In::Ctx& ic, SV* lds,
                                  IV* scratch, int l) {
    if constexpr (TWL)
      In::template fft_n<INV, In::kWave, 1>(z, typename In::TwTableJ{table(lds)}, scratch, l,
                                            ic.xbuf);
    else
      In::template fft_n<INV, In::kWave, 1>(z, ic.tw, scratch, l, ic.xbuf);
  }

  BPM_INLINE static void st(SV* q, int i, cx<CT> v) {
    SV s;
    s.x = static_cast<ST>(v.x);
    s.y = static_cast<ST>(v.y);
    q[i] = s;
  }
  BPM_INLINE static cx<CT> ld(const SV* q, int i) {
    const SV s = q[i];
    return {static_cast<CT>(s.x), static_cast<CT>(s.y)};
  }
  BPM_INLINE static SV* region(SV* lds, int r) {
    return reinterpret_cast<SV*>(reinterpret_cast<char*>(lds) + size_t(r) * kRegionBytes);
  }

  template <bool DEFORMED, int ORDER, bool MASKED>
  BPM_INLINE static void run(const MarchParams& p, int slice, int t, SV* lds) {
    if constexpr (TWL) {
      In::fill_table_j(table(lds), t, T);
      lds_barrier();
    }
    // wave-uniform: T0 is a multiple of the wavefront size
    if (__builtin_amdgcn_readfirstlane(t >= T0 ? 1 : 0))
      run_env<DEFORMED, 1, ORDER, MASKED>(p, slice, t - T0, lds);
    else
      run_env<DEFORMED, 0, ORDER, MASKED>(p, slice, t, lds);
  }

  // Coupling of one B sub-step (Eq. fov10) for envelope F at one sample:
  // d0 self + c other with c = d+1 exp(+i h u) for psi~_+ (F = 0) and
  // d-1 exp(-i h u) for psi~_- (F = 1); d holds d0, d+1, d-1.
  template <bool DEFORMED, int F>
  BPM_INLINE static cx<CT> couple(const cx<double> (&d)[3], SV er, cx<CT> self,
                                  cx<CT> other) {
    cx<double> c = d[1 + F];
    if constexpr (DEFORMED) {
      const cx<double> ee = {static_cast<double>(er.x), static_cast<double>(er.y)};
      c = F ? cmulc(c, ee) : cmul(c, ee);
    }
    return conv<CT>(cmuladd(d[0], conv<double>(self), c, conv<double>(other)));
  }

  // Thread t = E T0 + t0: in k space lane l of wavefront wv = t0 / 64 of
  // envelope E (0: psi~_+, 1: psi~_-); in x space both envelopes at the
  // samples x = t + T s, s < H = R/2.  With J = R/W sub-rows m_j = t0 + T0 j
  // per envelope, the thread's x samples are the rows j = E + 2 jj, jj < J/2:
  // x = m_j + M q is slot s = jj + (J/2) q.  Each step runs the sub-steps of
  // Scheme<ORDER>: A sub-steps are the transform phases, B sub-steps run in x
  // after the inverse exchange.  For ORDER > 1 the first B sub-step of a step
  // (no A before it) runs right after the last B sub-step of the previous
  // step, and before the first step on the input fields.
  template <bool DEFORMED, int E, int ORDER, bool MASKED>
  BPM_INLINE static void run_env(const MarchParams& p, int slice, int t0, SV* lds) {
    using S = Scheme<ORDER>;
    static_assert(J % 2 == 0, "the x-space rows split evenly between the envelopes");
    constexpr int JH = J / 2;      // x-space rows per thread
    constexpr int H = R / 2;       // x samples per thread
    const int wv = t0 >> 6, l = t0 & 63;
    const int t = E * T0 + t0;
    const SliceConst& sc = p.sc[slice];
    const SV* table = static_cast<const SV*>(p.table);
    SV* out_a = static_cast<SV*>(p.E0_out) + size_t(slice) * N;
    SV* out_b = static_cast<SV*>(p.Eh_out) + size_t(slice) * N;
    SV* Gp = reinterpret_cast<SV*>(reinterpret_cast<char*>(lds) + kGBytes);
    SV* own = region(lds, E * W + wv);
    IV* scratch = reinterpret_cast<IV*>(own);

    typename In::Ctx ic;
    if constexpr (TWL)
      ic.xbuf = 0;
    else
      In::init(ic, l);
    // W_N^{m_j k1} of this thread's rows
    Tw<CT> twx[JH * (W - 1)];
#pragma unroll
    for (int jj = 0; jj < JH; ++jj)
#pragma unroll
      for (int k1 = 1; k1 < W; ++k1) {
        double sn, cs;
        sincospi(-2.0 * double((t0 + T0 * (E + 2 * jj)) * k1) / double(N), &sn, &cs);
        twx[jj * (W - 1) + k1 - 1] = Tw<CT>::from(cs, sn);
      }
    // own band's propagators at the bins of (wavefront wv, lane l, slot i);
    // slab mask of the x samples t + T s
    cx<double> P[S::NP][R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int k = wv + W * (l + 64 * i);
      const int ks = k < N / 2 ? k : k - N;
#pragma unroll
      for (int q = 0; q < S::NP; ++q)
        P[q][i] = propagator(ks, N, p.dx, sc.k, p.h_half, E ? -1.0 : 1.0, p.dz,
                             p.a_frac[S::pdef(q)]);
    }
    bool inside[H];
#pragma unroll
    for (int s = 0; s < H; ++s) {
      const double x = static_cast<double>(t + T * s - N / 2) * p.dx;
      inside[s] = (x >= p.x_front) && (x < p.x_end);
    }

    // coupling constants d0, d+1, d-1 of every B sub-step
    cx<double> d[S::NS][3];
#pragma unroll
    for (int q = 0; q < S::NS; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) d[q][c] = {sc.d[q][2 * c], sc.d[q][2 * c + 1]};

    const SV* in_a = static_cast<const SV*>(p.E0_in) + size_t(slice) * N;
    const SV* in_b = p.Eh_in ? static_cast<const SV*>(p.Eh_in) + size_t(slice) * N
                             : nullptr;
    cx<CT> a[H], b[H];
#pragma unroll
    for (int s = 0; s < H; ++s) {
      a[s] = ld(in_a, t + T * s);
      b[s] = in_b ? ld(in_b, t + T * s) : cx<CT>{CT(0), CT(0)};
    }

    // B sub-step with constants dq and deformation er at slot s, both envelopes
    auto couple2 = [&](const cx<double> (&dq)[3], SV er_s, cx<CT>& as, cx<CT>& bs) {
      const cx<CT> a0 = as;
      as = couple<DEFORMED, 0>(dq, er_s, a0, bs);
      bs = couple<DEFORMED, 1>(dq, er_s, bs, a0);
    };

    // deformation rows: er of the current step (ORDER > 1: prefetched one
    // step ahead into er_next); crystal flags of the current and next step
    SV er[H], er_next[H];
    bool in_cur[H], in_next[H];
    if constexpr (ORDER > 1 && DEFORMED) {
      const SV* row = table + size_t(p.n0) * N;
#pragma unroll
      for (int s = 0; s < H; ++s) er[s] = er_next[s] = row[t + T * s];
    }
    if constexpr (ORDER > 1) {
      // first B sub-step of the first step, on the input fields
      crystal_row<H, N, MASKED>(p, p.n0, t, T, inside, in_cur);
#pragma unroll
      for (int s = 0; s < H; ++s)
        if (in_cur[s]) couple2(d[0], er[s], a[s], b[s]);
    }

    for (int n = 0; n < p.Nz; ++n) {
      if constexpr (ORDER == 1) {
        // deformation row of this step, fetched early for the coupling
        if constexpr (DEFORMED) {
          const SV* row = table + size_t(p.n0 + n) * N;
#pragma unroll
          for (int s = 0; s < H; ++s) er[s] = row[t + T * s];
        }
        crystal_row<H, N, MASKED>(p, p.n0 + n, t, T, inside, in_cur);
      } else {
        if (n + 1 < p.Nz) {
          if constexpr (DEFORMED) {
            const SV* row = table + size_t(p.n0 + n + 1) * N;
#pragma unroll
            for (int s = 0; s < H; ++s) er_next[s] = row[t + T * s];
          }
          crystal_row<H, N, MASKED>(p, p.n0 + n + 1, t, T, inside, in_next);
        }
      }
#pragma unroll
      for (int sub = 0; sub < S::NS; ++sub) {
        if (S::has_a(sub)) {
          // forward: radix-W over q for both envelopes at this thread's rows,
          // into the regions of the envelope's wavefronts
#pragma unroll
          for (int jj = 0; jj < JH; ++jj) {
            const int m = t0 + T0 * (E + 2 * jj);
            cx<CT> ua[W], ub[W];
#pragma unroll
            for (int q = 0; q < W; ++q) {
              ua[q] = a[jj + JH * q];
              ub[q] = b[jj + JH * q];
            }
            dft<W, false>(ua);
            dft<W, false>(ub);
#pragma unroll
            for (int k1 = 0; k1 < W; ++k1) {
              if (k1 > 0) {
                ua[k1] = twx[jj * (W - 1) + k1 - 1].mul(ua[k1]);
                ub[k1] = twx[jj * (W - 1) + k1 - 1].mul(ub[k1]);
              }
              st(region(lds, k1), m, ua[k1]);
              st(region(lds, W + k1), m, ub[k1]);
            }
          }
          lds_barrier();
          cx<CT> z[1][R];
#pragma unroll
          for (int i = 0; i < R; ++i) z[0][i] = ld(own, l + 64 * i);
          wave_sync();
          wave_fft<false>(z, ic, lds, scratch, l);
#pragma unroll
          for (int i = 0; i < R; ++i)
            z[0][i] = conv<CT>(cmul(conv<double>(z[0][i]), P[S::pset(sub)][i]));
          wave_fft<true>(z, ic, lds, scratch, l);
#pragma unroll
          for (int i = 0; i < R; ++i) st(Gp + (E * W + wv) * M, l + 64 * i, z[0][i]);
          lds_barrier();
          // inverse radix-W of both envelopes at this thread's rows, and the
          // coupling of each group of W samples right away
          const bool chain = ORDER > 1 && sub == S::NS - 1 && n + 1 < p.Nz;
#pragma unroll
          for (int jj = 0; jj < JH; ++jj) {
            const int m = t0 + T0 * (E + 2 * jj);
            cx<CT> ua[W], ub[W];
#pragma unroll
            for (int k1 = 0; k1 < W; ++k1) {
              ua[k1] = ld(Gp + k1 * M, m);
              ub[k1] = ld(Gp + (W + k1) * M, m);
              if (k1 > 0) {
                ua[k1] = twx[jj * (W - 1) + k1 - 1].mulc(ua[k1]);
                ub[k1] = twx[jj * (W - 1) + k1 - 1].mulc(ub[k1]);
              }
            }
            dft<W, true>(ua);
            dft<W, true>(ub);
#pragma unroll
            for (int q = 0; q < W; ++q) {
              const int s = jj + JH * q;
              a[s] = ua[q];
              b[s] = ub[q];
              if (in_cur[s]) couple2(d[sub], er[s], a[s], b[s]);
              // the first B sub-step of step n+1 right after the last of step n
              if (ORDER > 1 && chain && in_next[s]) couple2(d[0], er_next[s], a[s], b[s]);
            }
          }
        }
      }
      if constexpr (ORDER > 1) {
#pragma unroll
        for (int s = 0; s < H; ++s) {
          if constexpr (DEFORMED) er[s] = er_next[s];
          in_cur[s] = in_next[s];
        }
      }
    }
#pragma unroll
    for (int s = 0; s < H; ++s) {
      st(out_a, t + T * s, a[s]);
      st(out_b, t + T * s, b[s]);
    }
  }
};

// Envelope-split march of a slice that fits one wavefront per envelope
// (Nx = 256, 512): wavefront 0 carries psi~_+, wavefront 1 psi~_-, each with
// the one-wavefront Stockham transform of In.  A thread's x samples l + 64 i
// are exactly the transform's input and output slots, so there is no
// forward exchange; after the inverse transform each wavefront writes its
// envelope to a double-buffered LDS area and reads the partner's at the same
// x for the coupling: one work-group barrier per A sub-step, and two
// wavefronts per slice instead of one.
template <int PREC, class In>
struct Split1 {
  using CT = typename Prec<PREC>::CT;
  using ST = typename Prec<PREC>::ST;
  using SV = typename vec2<ST>::type;
  using IV = typename In::SV;
  static_assert(In::T == 64, "one-wavefront transform");
  static constexpr bool kSplit = true;
  static constexpr int N = In::N;
  static constexpr int R = In::R;
  static constexpr int T = 128;
  static constexpr size_t kScratchBytes = (size_t(In::kEnv) * sizeof(IV) + 15) / 16 * 16;
  static constexpr size_t kXBytes = size_t(2) * N * sizeof(SV);   // both envelopes
  static constexpr size_t kLdsBytes = 2 * kScratchBytes + 2 * kXBytes;
  static_assert(kLdsBytes <= 160 * 1024, "split march does not fit in LDS");

  BPM_INLINE static void st(SV* q, int i, cx<CT> v) {
    SV s;
    s.x = static_cast<ST>(v.x);
    s.y = static_cast<ST>(v.y);
    q[i] = s;
  }
  BPM_INLINE static cx<CT> ld(const SV* q, int i) {
    const SV s = q[i];
    return {static_cast<CT>(s.x), static_cast<CT>(s.y)};
  }

  template <bool DEFORMED, int ORDER, bool MASKED>
  BPM_INLINE static void run(const MarchParams& p, int slice, int t, SV* lds) {
    if (__builtin_amdgcn_readfirstlane(t >= 64 ? 1 : 0))
      run_env<DEFORMED, 1, ORDER, MASKED>(p, slice, t - 64, lds);
    else
      run_env<DEFORMED, 0, ORDER, MASKED>(p, slice, t, lds);
  }

  // Coupling of one B sub-step for envelope F (as in Split4::couple).
  template <bool DEFORMED, int F>
  BPM_INLINE static cx<CT> couple(const cx<double> (&d)[3], SV er, cx<CT> self,
                                  cx<CT> other) {
    cx<double> c = d[1 + F];
    if constexpr (DEFORMED) {
      const cx<double> ee = {static_cast<double>(er.x), static_cast<double>(er.y)};
      c = F ? cmulc(c, ee) : cmul(c, ee);
    }
    return conv<CT>(cmuladd(d[0], conv<double>(self), c, conv<double>(other)));
  }

  // Lane l of envelope E: x samples l + 64 i.
  template <bool DEFORMED, int E, int ORDER, bool MASKED>
  BPM_INLINE static void run_env(const MarchParams& p, int slice, int l, SV* lds) {
    using S = Scheme<ORDER>;
    const SliceConst& sc = p.sc[slice];
    const SV* table = static_cast<const SV*>(p.table);
    SV* out = static_cast<SV*>(E ? p.Eh_out : p.E0_out) + size_t(slice) * N;
    IV* scratch = reinterpret_cast<IV*>(reinterpret_cast<char*>(lds) + E * kScratchBytes);
    SV* X = reinterpret_cast<SV*>(reinterpret_cast<char*>(lds) + 2 * kScratchBytes);

    typename In::Ctx ic;
    In::init(ic, l);
    cx<double> P[S::NP][R];
    bool inside[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int k = l + 64 * i;                 // bin of slot i
      const int ks = k < N / 2 ? k : k - N;
#pragma unroll
      for (int q = 0; q < S::NP; ++q)
        P[q][i] = propagator(ks, N, p.dx, sc.k, p.h_half, E ? -1.0 : 1.0, p.dz,
                             p.a_frac[S::pdef(q)]);
      const double x = static_cast<double>(l + 64 * i - N / 2) * p.dx;
      inside[i] = (x >= p.x_front) && (x < p.x_end);
    }
    cx<double> d[S::NS][3];
#pragma unroll
    for (int s = 0; s < S::NS; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) d[s][c] = {sc.d[s][2 * c], sc.d[s][2 * c + 1]};

    const SV* in_a = static_cast<const SV*>(p.E0_in) + size_t(slice) * N;
    const SV* in_b = p.Eh_in ? static_cast<const SV*>(p.Eh_in) + size_t(slice) * N
                             : nullptr;
    const SV* src = E == 0 ? in_a : in_b;
    cx<CT> v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = src ? ld(src, l + 64 * i) : cx<CT>{CT(0), CT(0)};

    SV er[R], er_next[R];
    bool in_cur[R], in_next[R];
    if constexpr (ORDER > 1 && DEFORMED) {
      const SV* row = table + size_t(p.n0) * N;
#pragma unroll
      for (int i = 0; i < R; ++i) er[i] = er_next[i] = row[l + 64 * i];
    }
    if constexpr (ORDER > 1) {
      crystal_row<R, N, MASKED>(p, p.n0, l, 64, inside, in_cur);
      const SV* osrc = E == 0 ? in_b : in_a;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const cx<CT> other = osrc ? ld(osrc, l + 64 * i) : cx<CT>{CT(0), CT(0)};
        if (in_cur[i]) v[i] = couple<DEFORMED, E>(d[0], er[i], v[i], other);
      }
    }

    int buf = 0;
    for (int n = 0; n < p.Nz; ++n) {
      if constexpr (ORDER == 1) {
        if constexpr (DEFORMED) {
          const SV* row = table + size_t(p.n0 + n) * N;
#pragma unroll
          for (int i = 0; i < R; ++i) er[i] = row[l + 64 * i];
        }
        crystal_row<R, N, MASKED>(p, p.n0 + n, l, 64, inside, in_cur);
      } else {
        if (n + 1 < p.Nz) {
          if constexpr (DEFORMED) {
            const SV* row = table + size_t(p.n0 + n + 1) * N;
#pragma unroll
            for (int i = 0; i < R; ++i) er_next[i] = row[l + 64 * i];
          }
          crystal_row<R, N, MASKED>(p, p.n0 + n + 1, l, 64, inside, in_next);
        }
      }
#pragma unroll
      for (int s = 0; s < S::NS; ++s) {
        if (S::has_a(s)) {
          cx<CT> z[1][R];
#pragma unroll
          for (int i = 0; i < R; ++i) z[0][i] = v[i];
          In::template fft_n<false, In::kWave, 1>(z, ic.tw, scratch, l, ic.xbuf);
#pragma unroll
          for (int i = 0; i < R; ++i)
            z[0][i] = conv<CT>(cmul(conv<double>(z[0][i]), P[S::pset(s)][i]));
          In::template fft_n<true, In::kWave, 1>(z, ic.tw, scratch, l, ic.xbuf);
          // exchange: this envelope out, the partner's in (double-buffered:
          // the next write to this half comes after the next barrier)
          SV* Xb = X + buf * 2 * N;
          buf ^= 1;
#pragma unroll
          for (int i = 0; i < R; ++i) st(Xb + E * N, l + 64 * i, z[0][i]);
          lds_barrier();
          const bool chain = ORDER > 1 && s == S::NS - 1 && n + 1 < p.Nz;
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const cx<CT> self = z[0][i];
            const cx<CT> other = ld(Xb + (1 - E) * N, l + 64 * i);
            if (ORDER > 1 && chain) {
              cx<CT> s1 = self, o1 = other;
              if (in_cur[i]) {
                s1 = couple<DEFORMED, E>(d[s], er[i], self, other);
                o1 = couple<DEFORMED, 1 - E>(d[s], er[i], other, self);
              }
              v[i] = in_next[i] ? couple<DEFORMED, E>(d[0], er_next[i], s1, o1) : s1;
            } else {
              v[i] = in_cur[i] ? couple<DEFORMED, E>(d[s], er[i], self, other) : self;
            }
          }
        }
      }
      if constexpr (ORDER > 1) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          if constexpr (DEFORMED) er[i] = er_next[i];
          in_cur[i] = in_next[i];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) st(out, l + 64 * i, v[i]);
  }
};

// Whole march of one slice by threads t = 0..T-1 of the calling group, with
// both envelopes in every thread (Stockham and four-step transforms).  Each
// step runs the sub-steps of Scheme<ORDER> (Eq. fov10 per sub-step).
template <class Tr, bool DEFORMED, int ORDER, bool MASKED>
BPM_INLINE void march_slice_joint(const MarchParams& p, int slice, int t,
                                  typename Tr::SV* lds) {
  using CT = typename Tr::CT;
  using ST = typename Tr::ST;
  using SV = typename Tr::SV;
  using S = Scheme<ORDER>;
  constexpr int N = Tr::N, R = Tr::R, T = Tr::T;
  const SliceConst& sc = p.sc[slice];
  const SV* in = static_cast<const SV*>(p.E0_in) + size_t(slice) * N;
  SV* out_a = static_cast<SV*>(p.E0_out) + size_t(slice) * N;
  SV* out_b = static_cast<SV*>(p.Eh_out) + size_t(slice) * N;
  const SV* table = static_cast<const SV*>(p.table);

  typename Tr::Ctx ctx;
  Tr::init(ctx, t, lds);

  // Propagators of the bins this thread holds after a forward transform,
  // 1/Nx of the inverse transform folded in; slab mask of its x samples.
  cx<double> Pp[S::NP][R], Pm[S::NP][R];
  bool inside[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int k = Tr::bin(t, i);
    const int ks = k < N / 2 ? k : k - N;
#pragma unroll
    for (int q = 0; q < S::NP; ++q) {
      const double frac = p.a_frac[S::pdef(q)];
      Pp[q][i] = propagator(ks, N, p.dx, sc.k, p.h_half, +1.0, p.dz, frac);
      Pm[q][i] = propagator(ks, N, p.dx, sc.k, p.h_half, -1.0, p.dz, frac);
    }
    const double x = static_cast<double>(t + T * i - N / 2) * p.dx;
    inside[i] = (x >= p.x_front) && (x < p.x_end);
  }

  // coupling constants of every B sub-step
  cx<double> d0[S::NS], dp1[S::NS], dm1[S::NS];
#pragma unroll
  for (int s = 0; s < S::NS; ++s) {
    d0[s] = {sc.d[s][0], sc.d[s][1]};
    dp1[s] = {sc.d[s][2], sc.d[s][3]};
    dm1[s] = {sc.d[s][4], sc.d[s][5]};
  }

  const SV* in_b = p.Eh_in ? static_cast<const SV*>(p.Eh_in) + size_t(slice) * N
                           : nullptr;
  cx<CT> a[R], b[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const SV v = in[t + T * i];
    a[i] = {static_cast<CT>(v.x), static_cast<CT>(v.y)};
    b[i] = {CT(0), CT(0)};
    if (in_b) {
      const SV w = in_b[t + T * i];
      b[i] = {static_cast<CT>(w.x), static_cast<CT>(w.y)};
    }
  }

  for (int n = 0; n < p.Nz; ++n) {
    // the transforms' LDS addresses formed per step (see opaque_index)
    const int ts = opaque_step<Tr>(t);
    // Row n0 + n of exp(i h u), fetched at the start of the step and used by
    // the couplings, so its latency hides behind the transforms.
    // late: fetch the row after the forward transform (first order only:
    // the higher orders couple before their first transform)
    constexpr bool late = Tr::kLateRow && ORDER == 1;
    SV e[R];
    if constexpr (DEFORMED && !late) {
      const SV* row = table + size_t(p.n0 + n) * N;
#pragma unroll
      for (int i = 0; i < R; ++i) e[i] = row[t + T * i];
    }
    bool in_cur[R];
    crystal_row<R, N, MASKED>(p, p.n0 + n, t, T, inside, in_cur);
#pragma unroll
    for (int s = 0; s < S::NS; ++s) {
      if (S::has_a(s)) {
        Tr::forward(a, b, ctx, lds, ts);
        if constexpr (DEFORMED && late) {
          const SV* row = table + size_t(p.n0 + n) * N;
#pragma unroll
          for (int i = 0; i < R; ++i) e[i] = row[t + T * i];
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
          a[i] = conv<CT>(cmul(conv<double>(a[i]), Pp[S::pset(s)][i]));
          b[i] = conv<CT>(cmul(conv<double>(b[i]), Pm[S::pset(s)][i]));
        }
        Tr::inverse(a, b, ctx, lds, ts);
      }
      // Coupling in FP64 where the slab is; samples outside keep the field
      // (whole-wave vacuum groups branch past).
#pragma unroll
      for (int i = 0; i < R; ++i) {
        if (in_cur[i]) {
          const cx<double> A = conv<double>(a[i]);
          const cx<double> B = conv<double>(b[i]);
          cx<double> cp = dp1[s], cm = dm1[s];
          if constexpr (DEFORMED) {
            const cx<double> ee = {static_cast<double>(e[i].x),
                                   static_cast<double>(e[i].y)};
            cp = cmul(dp1[s], ee);    // d+1 exp(+i h u)
            cm = cmulc(dm1[s], ee);   // d-1 exp(-i h u)
          }
          a[i] = conv<CT>(cmuladd(d0[s], A, cp, B));
          b[i] = conv<CT>(cmuladd(d0[s], B, cm, A));
        }
      }
    }
  }

#pragma unroll
  for (int i = 0; i < R; ++i) {
    SV va, vb;
    va.x = static_cast<ST>(a[i].x);
    va.y = static_cast<ST>(a[i].y);
    vb.x = static_cast<ST>(b[i].x);
    vb.y = static_cast<ST>(b[i].y);
    out_a[t + T * i] = va;
    out_b[t + T * i] = vb;
  }
}

template <class Tr, bool DEFORMED, int ORDER, bool MASKED>
BPM_INLINE void march_slice(const MarchParams& p, int slice, int t,
                            typename Tr::SV* lds) {
  if constexpr (Tr::kSplit) {
    Tr::template run<DEFORMED, ORDER, MASKED>(p, slice, t, lds);
  } else {
    march_slice_joint<Tr, DEFORMED, ORDER, MASKED>(p, slice, t, lds);
  }
}

// MASKED: the crystal is the general mask p.mask (a row per step) instead
// of the slab; a separate instantiation, so the slab kernels carry no
// per-step mask work.
template <class M, bool DEFORMED, int ORDER, bool MASKED>
__global__ void __launch_bounds__(M::T) march_kernel(MarchParams p) {
  __shared__ __align__(16) typename M::SV lds[M::kLdsBytes / sizeof(typename M::SV)];
  march_slice<M, DEFORMED, ORDER, MASKED>(p, blockIdx.x, threadIdx.x, lds);
}

// Persistent march over a precomputed list of (problem, slice) items: work
// group g runs items offsets[g] .. offsets[g+1]-1 one after another.  Each
// item runs exactly the per-slice code of march_kernel, so results do not
// depend on how items are packed.
template <class M, int ORDER, bool MASKED>
__global__ void __launch_bounds__(M::T)
    march_batch_kernel(const BatchItem* __restrict__ items,
                       const int* __restrict__ offsets) {
  __shared__ __align__(16) typename M::SV lds[M::kLdsBytes / sizeof(typename M::SV)];
  const int k0 = offsets[blockIdx.x];
  const int k1 = offsets[blockIdx.x + 1];
  for (int k = k0; k < k1; ++k) {
    const MarchParams p = items[k].p;
    const int slice = items[k].slice;
    // the thread index opaque per item: what is formed from it (twiddles,
    // addresses, crystal flags) is formed per item instead of being hoisted
    // out of the item loop and kept live through every march
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    if (p.table)
      march_slice<M, true, ORDER, MASKED>(p, slice, t, lds);
    else
      march_slice<M, false, ORDER, MASKED>(p, slice, t, lds);
    lds_barrier();   // LDS of this item fully consumed before the next one
  }
}

// Time <-> frequency transform of a pulse along the slice axis (Section 3,
// Eq. tdp) on centred grids t_i = (i - N/2) dt, Omega_j = (j - N/2) dOmega,
// dOmega = 2 pi / (N dt).  With Omega_j t_i = 2 pi (j - N/2)(i - N/2) / N the
// pair factors into (-1)^i, an N-point DFT and (-1)^j (N a multiple of 4):
//   TO_FREQ:  out_j = dt (-1)^j sum_i (-1)^i in_i exp(+2 pi i ij/N)
//   !TO_FREQ: out_i = (-1)^i / (N dt) sum_j (-1)^j in_j exp(-2 pi i ij/N)
// Fields are [N][Nx]; work group b transforms columns 2b and 2b+1 with the
// Stockham transform of M (both columns under one set of barriers).  A
// column is read completely before it is written, so in place is allowed.
template <class M, bool TO_FREQ>
__global__ void __launch_bounds__(M::T)
    pulse_kernel(const typename M::SV* __restrict__ in, typename M::SV* out,
                 int Nx, double scale) {
  using CT = typename M::CT;
  using ST = typename M::ST;
  using SV = typename M::SV;
  constexpr int N = M::N, R = M::R, T = M::T;
  __shared__ __align__(16) SV lds[M::kLdsBytes / sizeof(SV)];
  const int t = threadIdx.x;
  const size_t x0 = size_t(2) * blockIdx.x;
  typename M::Ctx ctx;
  M::init(ctx, t);
  cx<CT> a[R], b[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = t + T * r;
    const SV va = in[size_t(i) * Nx + x0];
    const SV vb = in[size_t(i) * Nx + x0 + 1];
    const CT sg = (i & 1) ? CT(-1) : CT(1);
    a[r] = {sg * static_cast<CT>(va.x), sg * static_cast<CT>(va.y)};
    b[r] = {sg * static_cast<CT>(vb.x), sg * static_cast<CT>(vb.y)};
  }
  // exp(+i) kernel: the transform's inverse direction (no 1/N inside)
  if constexpr (TO_FREQ)
    M::inverse(a, b, ctx, lds, t);
  else
    M::forward(a, b, ctx, lds, t);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = M::bin(t, r);
    const double sg = (j & 1) ? -scale : scale;
    SV va, vb;
    va.x = static_cast<ST>(sg * static_cast<double>(a[r].x));
    va.y = static_cast<ST>(sg * static_cast<double>(a[r].y));
    vb.x = static_cast<ST>(sg * static_cast<double>(b[r].x));
    vb.y = static_cast<ST>(sg * static_cast<double>(b[r].y));
    out[size_t(j) * Nx + x0] = va;
    out[size_t(j) * Nx + x0 + 1] = vb;
  }
}

// exp(i h u): FP64 sincos for FP64 tables; for FP32 tables h*u is reduced
// modulo 2 pi in FP64 first, then rounded to FP32 for the sincos.  One
// thread per cell, grid-stride.
template <class ST>
__global__ void deform_kernel(const double* __restrict__ u, size_t n, double h,
                              typename vec2<ST>::type* __restrict__ out) {
  const double two_pi = kTwoPiHi;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    typename vec2<ST>::type v;
    if constexpr (sizeof(ST) == 4) {
      double r = fmod(h * u[i], two_pi);
      if (r < 0.0) r += two_pi;
      float s, c;
      sincosf(static_cast<float>(r), &s, &c);
      v.x = c;
      v.y = s;
    } else {
      double s, c;
      sincos(h * u[i], &s, &c);
      v.x = c;
      v.y = s;
    }
    out[i] = v;
  }
}

// ------------------------------------------------------------ dispatching --

// Schedules of the z-march transform for each (precision, Nx):
//   0 -- Stockham: R samples per thread per envelope, one work-group barrier
//        per pass (radix lists multiply to N);
//   1 -- four-step: radix-W across W wavefronts and a 256- or 512-point
//        Stockham inside each wavefront, two barriers per step.
template <int PREC, int N, int SCHED>
struct Choice;
template <int PREC> struct Choice<PREC, 256, 0> { using type = March<PREC, 256, 4, 4, 4, 4, 4>; };
template <int PREC> struct Choice<PREC, 512, 0> { using type = March<PREC, 512, 8, 8, 8, 8>; };
template <int PREC> struct Choice<PREC, 1024, 0> { using type = March<PREC, 1024, 8, 8, 8, 4, 4>; };
template <int PREC> struct Choice<PREC, 2048, 0> { using type = March<PREC, 2048, 8, 8, 8, 8, 4>; };
template <int PREC> struct Choice<PREC, 4096, 0> { using type = March<PREC, 4096, 8, 8, 8, 8, 8>; };
template <int PREC> using InWave1024 = March<PREC, 1024, 16, 16, 8, 8>;
template <int PREC> using InWave512 = March<PREC, 512, 8, 8, 8, 8>;
template <int PREC> using InWave256 = March<PREC, 256, 4, 4, 4, 4, 4>;
template <int PREC> struct Choice<PREC, 256, 1> { using type = FourStep<PREC, 1, InWave256<PREC>>; };
template <int PREC> struct Choice<PREC, 512, 1> { using type = FourStep<PREC, 1, InWave512<PREC>>; };
template <int PREC> struct Choice<PREC, 1024, 1> { using type = FourStep<PREC, 2, InWave512<PREC>>; };
template <int PREC> struct Choice<PREC, 2048, 1> { using type = FourStep<PREC, 4, InWave512<PREC>>; };
// 4096: in-wavefront twiddles from an LDS table where the FP64 state fills
// the register file (fp64, fp32s); fp32 keeps them in registers (faster there)
template <int PREC> struct Choice<PREC, 4096, 1> {
  using type = FourStep<PREC, 8, InWave512<PREC>, PREC != BPM_PREC_FP32>;
};
// 2 -- envelope-split four-step (2W wavefronts) where it fits, else four-step
template <int PREC> struct Choice<PREC, 256, 2> { using type = Split1<PREC, InWave256<PREC>>; };
template <int PREC> struct Choice<PREC, 512, 2> { using type = Split4<PREC, 2, InWave256<PREC>>; };
template <int PREC> struct Choice<PREC, 1024, 2> { using type = Split4<PREC, 2, InWave512<PREC>>; };
template <int PREC> struct Choice<PREC, 2048, 2> { using type = Split4<PREC, 4, InWave512<PREC>>; };
// 4096: the FP32-storage modes split the envelopes over W = 4 wavefronts each
// with a 1024-point in-wavefront transform (twiddles from the LDS table);
// FP64 storage does not fit that in LDS (its inverse exchange alone is
// 128 KiB) and keeps the four-step
template <int PREC> struct Choice<PREC, 4096, 2> {
  using type = std::conditional_t<PREC == BPM_PREC_FP64, typename Choice<PREC, 4096, 1>::type,
                                  Split4<PREC, 4, InWave1024<PREC>, true>>;
};

// Calls f(M{}) with the transform of (precision, Nx, schedule).
template <int PREC, int N, class F>
int with_sched(int sched, F&& f) {
  switch (sched) {
    case 0: return f(typename Choice<PREC, N, 0>::type{});
    case 1: return f(typename Choice<PREC, N, 1>::type{});
    case 2: return f(typename Choice<PREC, N, 2>::type{});
    default: return BPM_EUNSUPPORTED;
  }
}
template <class F>
int with_order(int order, F&& f) {
  switch (order) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    default: return BPM_EUNSUPPORTED;
  }
}

}  // namespace

// Entry points of one transform length N.  Each N is instantiated in one
// kernel unit (see BPM_MARCH_N), so units can be compiled with different
// scheduling options.
template <int PREC, bool MASKED, int N>
int launch_march_n(int sched, int order, int Nomega, const MarchParams& p,
                   hipStream_t stream) {
  return with_sched<PREC, N>(sched, [&](auto m) {
    using M = decltype(m);
    return with_order(order, [&](auto o) {
      constexpr int ORDER = decltype(o)::value;
      if (p.table)
        hipLaunchKernelGGL((march_kernel<M, true, ORDER, MASKED>), dim3(Nomega),
                           dim3(M::T), 0, stream, p);
      else
        hipLaunchKernelGGL((march_kernel<M, false, ORDER, MASKED>), dim3(Nomega),
                           dim3(M::T), 0, stream, p);
      return hipGetLastError() == hipSuccess ? BPM_OK : BPM_EHIP;
    });
  });
}

template <int PREC, bool MASKED, int N>
int launch_march_batch_n(int sched, int order, const BatchItem* items,
                         const int* offsets, int n_groups, hipStream_t stream) {
  return with_sched<PREC, N>(sched, [&](auto m) {
    using M = decltype(m);
    return with_order(order, [&](auto o) {
      constexpr int ORDER = decltype(o)::value;
      hipLaunchKernelGGL((march_batch_kernel<M, ORDER, MASKED>), dim3(n_groups),
                         dim3(M::T), 0, stream, items, offsets);
      return hipGetLastError() == hipSuccess ? BPM_OK : BPM_EHIP;
    });
  });
}

template <int PREC, bool MASKED, int N>
int march_occupancy_n(int sched, int order, int* wg_per_cu, int* threads) {
  return with_sched<PREC, N>(sched, [&](auto m) {
    using M = decltype(m);
    return with_order(order, [&](auto o) {
      constexpr int ORDER = decltype(o)::value;
      int n = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &n, reinterpret_cast<const void*>(&march_batch_kernel<M, ORDER, MASKED>), M::T,
              0) != hipSuccess)
        return BPM_EHIP;
      *wg_per_cu = n;
      *threads = M::T;
      return BPM_OK;
    });
  });
}

// Declares (KW = extern) or instantiates (KW empty) the entry points of
// transform length N for one precision and crystal kind.
#define BPM_MARCH_N(KW, P, MASKED, N)                                              \
  KW template int launch_march_n<P, MASKED, N>(int, int, int, const MarchParams&,  \
                                               hipStream_t);                      \
  KW template int launch_march_batch_n<P, MASKED, N>(int, int, const BatchItem*,   \
                                                     const int*, int, hipStream_t); \
  KW template int march_occupancy_n<P, MASKED, N>(int, int, int*, int*);

template <int PREC, bool MASKED>
int launch_march_p(int Nx, int sched, int order, int Nomega, const MarchParams& p,
                   hipStream_t stream) {
  switch (Nx) {
    case 256: return launch_march_n<PREC, MASKED, 256>(sched, order, Nomega, p, stream);
    case 512: return launch_march_n<PREC, MASKED, 512>(sched, order, Nomega, p, stream);
    case 1024: return launch_march_n<PREC, MASKED, 1024>(sched, order, Nomega, p, stream);
    case 2048: return launch_march_n<PREC, MASKED, 2048>(sched, order, Nomega, p, stream);
    case 4096: return launch_march_n<PREC, MASKED, 4096>(sched, order, Nomega, p, stream);
    default: return BPM_EUNSUPPORTED;
  }
}

template <int PREC, bool MASKED>
int launch_march_batch_p(int Nx, int sched, int order, const BatchItem* items,
                         const int* offsets, int n_groups, hipStream_t stream) {
  switch (Nx) {
    case 256: return launch_march_batch_n<PREC, MASKED, 256>(sched, order, items, offsets, n_groups, stream);
    case 512: return launch_march_batch_n<PREC, MASKED, 512>(sched, order, items, offsets, n_groups, stream);
    case 1024: return launch_march_batch_n<PREC, MASKED, 1024>(sched, order, items, offsets, n_groups, stream);
    case 2048: return launch_march_batch_n<PREC, MASKED, 2048>(sched, order, items, offsets, n_groups, stream);
    case 4096: return launch_march_batch_n<PREC, MASKED, 4096>(sched, order, items, offsets, n_groups, stream);
    default: return BPM_EUNSUPPORTED;
  }
}

// Pulse transform of [N][Nx] fields: FP64 butterflies for every
// precision (complex64 storage for the FP32 modes).
template <int PREC>
int launch_pulse_p(int N, int Nx, bool to_freq, double dt, const void* in, void* out,
                   hipStream_t stream) {
  constexpr int SP = PREC == BPM_PREC_FP64 ? BPM_PREC_FP64 : BPM_PREC_FP32S;
  auto run = [&](auto m) {
    using M = decltype(m);
    using SV = typename M::SV;
    const double scale = to_freq ? dt : 1.0 / (double(N) * dt);
    if (to_freq)
      hipLaunchKernelGGL((pulse_kernel<M, true>), dim3(Nx / 2), dim3(M::T), 0, stream,
                         static_cast<const SV*>(in), static_cast<SV*>(out), Nx, scale);
    else
      hipLaunchKernelGGL((pulse_kernel<M, false>), dim3(Nx / 2), dim3(M::T), 0, stream,
                         static_cast<const SV*>(in), static_cast<SV*>(out), Nx, scale);
    return hipGetLastError() == hipSuccess ? BPM_OK : BPM_EHIP;
  };
  switch (N) {   // Stockham transform of length N
    case 256: return run(typename Choice<SP, 256, 0>::type{});
    case 512: return run(typename Choice<SP, 512, 0>::type{});
    case 1024: return run(typename Choice<SP, 1024, 0>::type{});
    case 2048: return run(typename Choice<SP, 2048, 0>::type{});
    case 4096: return run(typename Choice<SP, 4096, 0>::type{});
    default: return BPM_EUNSUPPORTED;
  }
}

template <int PREC, bool MASKED>
int march_occupancy_p(int Nx, int sched, int order, int* wg_per_cu, int* threads) {
  switch (Nx) {
    case 256: return march_occupancy_n<PREC, MASKED, 256>(sched, order, wg_per_cu, threads);
    case 512: return march_occupancy_n<PREC, MASKED, 512>(sched, order, wg_per_cu, threads);
    case 1024: return march_occupancy_n<PREC, MASKED, 1024>(sched, order, wg_per_cu, threads);
    case 2048: return march_occupancy_n<PREC, MASKED, 2048>(sched, order, wg_per_cu, threads);
    case 4096: return march_occupancy_n<PREC, MASKED, 4096>(sched, order, wg_per_cu, threads);
    default: return BPM_EUNSUPPORTED;
  }
}

}  // namespace bpm

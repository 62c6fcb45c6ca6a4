// gfx950 kernels of the z-march on a 3D grid: two transverse axes, x (along
// h, the axis of the two angular bands) and y, marching along z (Section 2.1:
// Eq. fov4 with k_x and k_y; the two-band coupling of Eq. fov10 at every
// (x, y); the finite-element example of Section 3.4 runs on such a grid).
//
// A slice's state (both envelopes, Ny x Nx) does not fit on chip at the
// sizes of Section 3.4 (22 x 4267), so it lives in HBM, in the caller's two
// output buffers, and each step is two launches over all slices:
//   row kernel    -- one work group per (slice, envelope, K_y) row: FFT along
//                    x, the band propagator exp(i dz sqrt(k^2 - (K_x +- h/2)^2
//                    - K_y^2)) / (Nx Ny), inverse FFT along x, in place;
//   column kernel -- 64 x-columns x Ny/2 threads per work group: inverse DFT
//                    along y (back to x space), the coupling of the step with
//                    the deformation row and the slab, forward DFT along y
//                    for the next step (the last step stores x space).
// The first launch transforms the incident field along y.
//
// Transforms along x of any length: the propagator step of a row is the
// cyclic convolution of the row with p = IDFT_Nx(P), so for any Nx it is
// computed on a length L with small factors: L = Nx for powers of two >= 64,
// otherwise the smallest L >= 2 Nx - 1 among the powers of two >= 64 and
// 4608, 9216 (9 M, M = 512, 1024).  The row, zero-padded to
// L, is transformed, multiplied by the row's table Q = FFT_L(q) / L, where q
// holds p at offsets -(Nx-1)..Nx-1 wrapped to length L (no two offsets meet
// for L >= 2 Nx - 1), and transformed back; its first Nx samples are the
// step.  For L = Nx, Q = P.  The plan builds Q once (FP64), the host
// evaluating IDFT_Nx by Bluestein's algorithm for other lengths.  Twiddles
// of the length-L transform come from an FP64 table W_L^m in global memory
// (shared by every row, resident in L2), one entry per butterfly group and
// the group's other twiddles as its powers: registers and LDS hold the row.
// The y transform is a direct DFT (Ny <= 32).

#include "bpm_device.h"

namespace bpm {
namespace {

// Keeps the compiler from moving global table loads across the transforms
// or merging the same twiddle loads of successive transforms (hoisted early
// or shared, they stay live in registers through whole FFTs and spill).
BPM_INLINE void phase_fence() { asm volatile("" ::: "memory"); }

// The thread index as an opaque value: the LDS slot addresses of a
// transform depend only on it, and without this the compiler computes them
// once and keeps them live across all four transforms of a row (tens of
// registers per pass), spilling.
BPM_INLINE int opaque(int v) {
  asm volatile("" : "+v"(v));
  __builtin_assume(v >= 0);
  return v;
}

// w[n] = w[1]^n for 1 <= n < K: powers of two by squaring, the others as
// w[p] w[n - p] with p the largest power of two below n, so that each is a
// product of depth at most log2(K) (a few ulps from the exact value).
// Several twiddles of one butterfly group or column are formed this way
// from one table load: each table load is waited for where it is used, and
// eight or fifteen of them per group cost more than the products.
template <int K>
BPM_INLINE void twiddle_powers(cx<double> (&w)[K]) {
#pragma unroll
  for (int n = 2; n < K; ++n) {
    int p = 1;
    while (2 * p < n) p *= 2;
    w[n] = cmul(w[p], w[n - p]);
  }
}

// Twiddle W_{Ns Rp}^{r j} of pass P of transform M: W_L^{j L/(Ns Rp)} from
// the table tab[m] = exp(-2 pi i m / NT), and its powers r >= 2 as products
// (twiddle_powers; the compiler merges the common factors of one group).
// The thread index is opaque per pass (kOpaqueIndex), so a pass's loads can
// be neither hoisted into an earlier pass nor shared with another
// transform; within a pass, the butterflies s of a thread share j while
// Ns <= T, and their loads are one.
template <class M, int NT = M::N>   // NT: table length, a multiple of M::N
struct TwDerived {
  static constexpr bool kOpaqueIndex = true;
  const cx<double>* tab;
  template <int P>
  BPM_INLINE Tw<typename M::CT> get(int t, int s, int r) const {
    constexpr int Ns = M::ns(P);
    constexpr int Rp = M::rad[P];
    const int j = (Ns <= M::T ? t : t + s * M::T) & (Ns - 1);
    cx<double> w[Rp];
    w[1] = tab[j * (NT / (Ns * Rp))];
    twiddle_powers(w);
    return Tw<typename M::CT>{w[r]};
  }
};

template <class T>
BPM_INLINE cx<double> to_d(cx<T> a) {
  return {static_cast<double>(a.x), static_cast<double>(a.y)};
}
BPM_INLINE cx<double> conjd(cx<double> a) { return {a.x, -a.y}; }
// acc + a w with each component one expression (two FMAs)
BPM_INLINE cx<double> cmac(cx<double> acc, cx<double> a, cx<double> w) {
  return {acc.x + a.x * w.x - a.y * w.y, acc.y + a.x * w.y + a.y * w.x};
}

// exp(i frac dz sqrt(k^2 - (K_x + band h/2)^2 - K_y^2)) / (Nx Ny) for signed bins
// (mx, my), K = 2 pi m / (N d), evaluated and reduced modulo 2 pi in
// double-double; principal root (decay) where evanescent.
__device__ cx<double> propagator3(int mx, int my, int Nx, int Ny, double dx, double dy,
                                  double k, double h_half, double band, double dz,
                                  double frac) {
  const dd two_pi = {kTwoPiHi, kTwoPiLo};
  const dd Kx = dd_div_d(dd_mul_d(two_pi, static_cast<double>(mx)),
                         static_cast<double>(Nx) * dx);
  const dd Ky = dd_div_d(dd_mul_d(two_pi, static_cast<double>(my)),
                         static_cast<double>(Ny) * dy);
  const dd kp = dd_add(Kx, dd{band * h_half, 0.0});
  const dd kz2 = dd_add(dd_add(two_prod(k, k), dd_neg(dd_mul(kp, kp))), dd_neg(dd_mul(Ky, Ky)));
  const double inv_n = 1.0 / (static_cast<double>(Nx) * static_cast<double>(Ny));
  if (kz2.hi < 0.0) return {exp(-frac * dz * sqrt(-kz2.hi)) * inv_n, 0.0};
  // sub-step length frac*dz kept exact (two_prod) for fractional sub-steps
  dd phi = frac == 1.0 ? dd_mul_d(dd_sqrt(kz2), dz)
                       : dd_mul(dd_sqrt(kz2), two_prod(frac, dz));
  const double n = floor(phi.hi / kTwoPiHi);
  phi = dd_add(phi, dd_neg(dd_mul_d(two_pi, n)));
  if (phi.hi < 0.0) phi = dd_add(phi, two_pi);
  if (phi.hi >= kTwoPiHi) phi = dd_add(phi, dd_neg(two_pi));
  double s, c;
  sincos(phi.hi + phi.lo, &s, &c);
  return {c * inv_n, s * inv_n};
}

// Propagator table P[((w * 2 + env) * Nyc + c) * Nx + kx], Nyc = Ny / 2 + 1
// rows per (slice, envelope): the propagator depends on K_y only through
// K_y^2, so row c serves the bins K_y = +-2 pi c / (Ny dy), i.e. ky = c and
// ky = Ny - c.  One thread per entry (grid-stride).
__global__ void prop3_kernel(cx<double>* __restrict__ P, const SliceConst* __restrict__ sc,
                             int Nx, int Ny, int Nomega, double dx, double dy, double dz,
                             double frac, double h_half) {
  const int Nyc = Ny / 2 + 1;
  const size_t n = size_t(Nomega) * 2 * Nyc * Nx;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    const int kx = static_cast<int>(i % Nx);
    const size_t r = i / Nx;
    const int c = static_cast<int>(r % Nyc);
    const int env = static_cast<int>((r / Nyc) & 1);
    const int w = static_cast<int>(r / (2 * size_t(Nyc)));
    const int mx = kx < (Nx + 1) / 2 ? kx : kx - Nx;
    P[i] = propagator3(mx, c, Nx, Ny, dx, dy, sc[w].k, h_half, env ? -1.0 : 1.0, dz, frac);
  }
}

// Row r = (w * 2 + env) * Ny + ky of the state uses table row
// (w * 2 + env) * Nyc + min(ky, Ny - ky).
BPM_INLINE int table_row(int row, int Ny) {
  const int ky = row % Ny;
  const int c = ky <= Ny - ky ? ky : Ny - ky;
  return (row / Ny) * (Ny / 2 + 1) + c;
}

struct Row3Params {
  void* a;                    // psi~_+ state [Nomega][Ny][Nx] (storage type)
  void* b;                    // psi~_- state
  const cx<double>* Q;        // [Nomega][2][Ny / 2 + 1][L] row propagator
  const cx<double>* tw;       // [L] exp(-2 pi i m / L)
  int Nx, Ny;
};

// One (slice, envelope, K_y) row per work group: the row zero-padded to L,
// FFT_L, times the row's propagator table, inverse FFT_L, the first Nx
// samples stored back in place.  Thread t holds samples t + T i, in
// registers of the storage type (widened to the arithmetic type inside each
// butterfly and pointwise product).
template <class M>
__global__ void __launch_bounds__(M::T) row3_kernel(Row3Params p) {
  using CT = typename M::ST;
  using SV = typename M::SV;
  constexpr int R = M::R, T = M::T;
  constexpr bool kTwo = 2 * M::kEnvBytes <= 160 * 1024;
  constexpr int SYNC = kTwo ? M::kDouble : M::kSingle;
  __shared__ __align__(16) SV lds[(kTwo ? 2 : 1) * M::kEnv];
  const int t = threadIdx.x;
  const int row = blockIdx.x;
  const int ky = row % p.Ny;
  const int env = (row / p.Ny) & 1;
  const int w = row / (2 * p.Ny);
  SV* line = static_cast<SV*>(env ? p.b : p.a) + (size_t(w) * p.Ny + ky) * p.Nx;
  const cx<double>* Qrow = p.Q + size_t(table_row(row, p.Ny)) * M::N;
  const TwDerived<M> tws{p.tw};
  int xbuf = 0;
  cx<CT> v[1][R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int n = t + T * i;
    SV s;
    s.x = 0;
    s.y = 0;
    if (n < p.Nx) s = line[n];
    v[0][i] = {static_cast<CT>(s.x), static_cast<CT>(s.y)};
  }
  M::template fft_n<false, SYNC, 1>(v, tws, lds, opaque(t), xbuf);
  phase_fence();
#pragma unroll
  for (int i = 0; i < R; ++i) {
    if (i % 4 == 0) phase_fence();     // table loads in groups of four
    v[0][i] = conv<CT>(cmul(to_d(v[0][i]), Qrow[t + T * i]));
  }
  phase_fence();
  M::template fft_n<true, SYNC, 1>(v, tws, lds, opaque(t), xbuf);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int n = t + T * i;
    if (n < p.Nx) {
      SV s;
      s.x = static_cast<typename M::ST>(v[0][i].x);
      s.y = static_cast<typename M::ST>(v[0][i].y);
      line[n] = s;
    }
  }
}

// W16^{j} (INV: conjugated) for an index that is constant once the loops
// around it are unrolled.
template <bool INV, class T>
BPM_INLINE cx<T> tw16_at(cx<T> a, int j) {
  switch (j & 15) {
    case 0: return a;
    case 1: return tw16<1, INV>(a);
    case 2: return tw16<2, INV>(a);
    case 3: return tw16<3, INV>(a);
    case 4: return tw16<4, INV>(a);
    case 6: return tw16<6, INV>(a);
    case 9: return tw16<9, INV>(a);
    default: return tw16<15, INV>(tw16<1, INV>(tw16<15, INV>(a)));  // not reached
  }
}

// Long rows (L = 8192, 16384) in the four-step layout of the 2D march:
// L = W M with an M-point in-wavefront transform In, T = 64 W threads;
// thread t owns m_j = t + T j (j < J = R / W) and holds x[m_j + M q] in
// slot j + J q.  Forward: the radix-W DFT over q in registers, the twiddle
// W_L^{m k1}, one block exchange that gives wavefront k1 the M values of
// its k1 (lane l, slot i <- m = l + 64 i), then the in-wavefront transform,
// whose exchanges need no barrier.  Slot i of lane l of wavefront w ends
// with bin K = w + W (l + 64 i); the inverse runs the steps backwards.  Two
// work-group barriers per row step instead of one or two per Stockham pass.
// Each wavefront's region of LDS is first the target of the block exchange
// and then its own exchange buffer.
template <class In_, int W>
struct RowFour {
  using In = In_;
  using CT = typename In::CT;
  using ST = typename In::ST;
  using SV = typename In::SV;
  static constexpr int M = In::N, R = In::R, N = W * M, T = 64 * W, J = R / W;
  static_assert(In::T == 64 && R % W == 0, "one wavefront per in-wave transform, R a multiple of W");
  static constexpr int kRegion = In::kEnv;
  static constexpr size_t kLdsSlots = size_t(W) * kRegion;
  static_assert(kLdsSlots * sizeof(SV) <= 160 * 1024, "row does not fit in LDS");

  BPM_INLINE static void put(SV* lds, int idx, cx<CT> v) {
    SV s;
    s.x = static_cast<ST>(v.x);
    s.y = static_cast<ST>(v.y);
    lds[idx] = s;
  }

  // W = 16 (J = 1), forward: the radix-16 DFT over q as 4 x 4 (q = 4 n1 +
  // n2, K = k1 + 4 k2), the inner results rounded to the storage type in
  // the state's own slots, so that at most four values are live in the
  // arithmetic type (all sixteen in FP64 here spill at the 128 registers of
  // a 1024-thread work group; in the inverse they do not, and the inverse
  // keeps the plain radix-16 DFT).
  BPM_INLINE static void forward16(cx<ST> (&v)[1][R], const cx<double>* tab, SV* lds, int t_in) {
    // opaque: the twiddle addresses are formed here, not shared with the
    // inverse and kept live across the whole row step
    const int t = opaque(t_in);
    cx<double> w[16];   // W_N^{t K}
    w[1] = tab[t];
    twiddle_powers(w);
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      cx<CT> a[4];
#pragma unroll
      for (int n1 = 0; n1 < 4; ++n1) a[n1] = conv<CT>(v[0][4 * n1 + n2]);
      dft4<false>(a[0], a[1], a[2], a[3]);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) v[0][4 * k1 + n2] = conv<ST>(tw16_at<false>(a[k1], n2 * k1));
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cx<CT> b[4];
#pragma unroll
      for (int n2 = 0; n2 < 4; ++n2) b[n2] = conv<CT>(v[0][4 * k1 + n2]);
      dft4<false>(b[0], b[1], b[2], b[3]);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) {
        const int K = k1 + 4 * k2;
        put(lds + K * kRegion, t, K ? Tw<CT>{w[K]}.mul(b[k2]) : b[k2]);
      }
    }
  }
  BPM_INLINE static void forward(cx<ST> (&v)[1][R], const cx<double>* tab, SV* lds, int t) {
    const int l = t & 63;
    SV* own = lds + (t >> 6) * kRegion;
    if constexpr (W == 16) forward16(v, tab, lds, t);
    else
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int m = opaque(t) + T * j;
      cx<CT> va[W];
#pragma unroll
      for (int q = 0; q < W; ++q) va[q] = conv<CT>(v[0][j + J * q]);
      dft<W, false>(va);
      cx<double> w[W];   // W_N^{m k1}
      w[1] = tab[m];
      twiddle_powers(w);
#pragma unroll
      for (int k1 = 0; k1 < W; ++k1) {
        if (k1 > 0) va[k1] = Tw<CT>{w[k1]}.mul(va[k1]);
        put(lds + k1 * kRegion, m, va[k1]);
      }
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < R; ++i) v[0][i] = In::template load_as<ST>(own, l + 64 * i);
    wave_sync();
    int xbuf = 0;
    In::template fft_n<false, In::kWave, 1>(v, TwDerived<In, N>{tab}, own, opaque(l), xbuf);
  }

  BPM_INLINE static void inverse(cx<ST> (&v)[1][R], const cx<double>* tab, SV* lds, int t) {
    const int l = t & 63;
    SV* own = lds + (t >> 6) * kRegion;
    int xbuf = 0;
    In::template fft_n<true, In::kWave, 1>(v, TwDerived<In, N>{tab}, own, opaque(l), xbuf);
#pragma unroll
    for (int i = 0; i < R; ++i) put(own, l + 64 * i, conv<CT>(v[0][i]));
    lds_barrier();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int m = opaque(t) + T * j;
      cx<CT> va[W];
      cx<double> w[W];
      w[1] = tab[m];
      twiddle_powers(w);
#pragma unroll
      for (int k1 = 0; k1 < W; ++k1) {
        va[k1] = In::template load_as<CT>(lds + k1 * kRegion, m);
        if (k1 > 0) va[k1] = Tw<CT>{w[k1]}.mulc(va[k1]);
      }
      dft<W, true>(va);
#pragma unroll
      for (int q = 0; q < W; ++q) v[0][j + J * q] = conv<ST>(va[q]);
    }
  }
};

// One row per work group with the four-step transform: Q holds each row's
// table in the kernel's bin order, Q[i T + t] = row bin w + W (l + 64 i) of
// thread t = 64 w + l, so its loads are contiguous.
template <class F>
__global__ void __launch_bounds__(F::T) row3_four_kernel(Row3Params p) {
  using ST = typename F::ST;
  using SV = typename F::SV;
  constexpr int R = F::R, T = F::T, M = F::M, J = F::J, W = F::N / F::M;
  __shared__ __align__(16) SV lds[F::kLdsSlots];
  const int t = threadIdx.x;
  const int row = blockIdx.x;
  const int ky = row % p.Ny;
  const int env = (row / p.Ny) & 1;
  const int w = row / (2 * p.Ny);
  SV* line = static_cast<SV*>(env ? p.b : p.a) + (size_t(w) * p.Ny + ky) * p.Nx;
  const cx<double>* Qrow = p.Q + size_t(table_row(row, p.Ny)) * F::N;
  cx<ST> v[1][R];
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int q = 0; q < W; ++q) {
      const int n = t + T * j + M * q;
      SV s;
      s.x = 0;
      s.y = 0;
      if (n < p.Nx) s = line[n];
      v[0][j + J * q] = {s.x, s.y};
    }
  F::forward(v, p.tw, lds, t);
  phase_fence();
  const int tq = opaque(t);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    if (i % 4 == 0) phase_fence();     // table loads in groups of four
    v[0][i] = conv<ST>(cmul(to_d(v[0][i]), Qrow[i * T + tq]));
  }
  phase_fence();
  F::inverse(v, p.tw, lds, t);
  const int ts = opaque(t);   // store addresses formed here, not kept from the loads
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int q = 0; q < W; ++q) {
      const int n = ts + T * j + M * q;
      if (n < p.Nx) {
        SV s;
        s.x = v[0][j + J * q].x;
        s.y = v[0][j + J * q].y;
        line[n] = s;
      }
    }
}

// ------------------------------------------------ rows of length 9 M --
// exp(-+2 pi i j / 9) for j = 1, 2, 4 and sqrt(3) / 2, correctly rounded.
constexpr double kC9[3] = {0.766044443118978, 0.17364817766693036, -0.9396926207859084};
constexpr double kS9[3] = {0.6427876096865394, 0.984807753012208, 0.3420201433256687};
constexpr double kHalfSqrt3 = 0.8660254037844386;

// a * (c + i si); in FP32 arithmetic the product is formed in FP64 and
// rounded once, as for every twiddle (see Tw).
template <class T>
BPM_INLINE cx<T> cmul_const(cx<T> a, double c, double si) {
  const double xr = a.x, xi = a.y;
  return {static_cast<T>(xr * c - xi * si), static_cast<T>(xr * si + xi * c)};
}

// a * W9^j (INV: conjugated) for j in {1, 2, 4}
template <int J, bool INV, class T>
BPM_INLINE cx<T> tw9(cx<T> a) {
  constexpr int i = J == 1 ? 0 : J == 2 ? 1 : 2;
  static_assert(J == 1 || J == 2 || J == 4, "W9 power");
  return cmul_const(a, kC9[i], INV ? kS9[i] : -kS9[i]);
}

// 3-point DFT (a, b, c) -> (X0, X1, X2): s = b + c, d = b - c,
// X0 = a + s, X1,2 = a - s / 2 -+ i (sqrt 3 / 2) d (forward; +- inverse).
// NZ: inputs that can be nonzero (3, or 2 with c = 0, or 1 with b = c = 0).
template <bool INV, int NZ, class T>
BPM_INLINE void dft3(cx<T>& a, cx<T>& b, cx<T>& c) {
  if constexpr (NZ == 1) {
    b = a;
    c = a;
  } else {
    const cx<T> s = NZ == 3 ? b + c : b;
    const cx<T> d = NZ == 3 ? b - c : b;
    const cx<T> m = {a.x - T(0.5) * s.x, a.y - T(0.5) * s.y};
    const cx<T> rd = rot<INV>(d);
    a = a + s;
    if constexpr (sizeof(T) == 8) {
      b = {m.x + kHalfSqrt3 * rd.x, m.y + kHalfSqrt3 * rd.y};
      c = {m.x - kHalfSqrt3 * rd.x, m.y - kHalfSqrt3 * rd.y};
    } else {
      // the product formed in FP64 and rounded once (see Tw)
      const cx<T> r = {static_cast<T>(kHalfSqrt3 * static_cast<double>(rd.x)),
                       static_cast<T>(kHalfSqrt3 * static_cast<double>(rd.y))};
      b = m + r;
      c = m - r;
    }
  }
}

// 9-point DFT as 3 x 3 (n = 3 n1 + n2, k = k1 + 3 k2) of y[0..NZ) (the
// rest zero), natural order out in X[9].
template <bool INV, int NZ, class T>
BPM_INLINE void dft9(const cx<T> (&y)[9], cx<T> (&X)[9]) {
  static_assert(NZ == 5 || NZ == 9, "pruned forms built: 5 or 9 inputs");
  cx<T> a[3][3];   // a[n2][k1]
#pragma unroll
  for (int n2 = 0; n2 < 3; ++n2) {
    a[n2][0] = y[n2];
    a[n2][1] = y[n2 + 3];
    a[n2][2] = y[n2 + 6];
  }
  if constexpr (NZ == 9) {
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) dft3<INV, 3>(a[n2][0], a[n2][1], a[n2][2]);
  } else {
    // y[5..8] = 0: column n2 = 0, 1 has inputs (y n2, y n2+3, 0), n2 = 2 only y2
    dft3<INV, 2>(a[0][0], a[0][1], a[0][2]);
    dft3<INV, 2>(a[1][0], a[1][1], a[1][2]);
    dft3<INV, 1>(a[2][0], a[2][1], a[2][2]);
  }
  a[1][1] = tw9<1, INV>(a[1][1]);
  a[1][2] = tw9<2, INV>(a[1][2]);
  a[2][1] = tw9<2, INV>(a[2][1]);
  a[2][2] = tw9<4, INV>(a[2][2]);
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    dft3<INV, 3>(a[0][k1], a[1][k1], a[2][k1]);
    X[k1] = a[0][k1];
    X[k1 + 3] = a[1][k1];
    X[k1 + 6] = a[2][k1];
  }
}

// Rows of length L = 9 M (M = 512, 1024) for Nx <= 4.5 M, where the next
// power of two would be 16 M: the four-step layout of RowFour with
// W = 9 wavefronts (T = 576 threads) and a radix-9 step.  The M columns
// x[m + M q] (q < 9) are shared out over the threads, t + T c for c <
// ceil(M / T) (the last set partial, whole wavefronts idle), and read from
// and written to HBM directly by the radix-9 steps; only q < 5 can be
// nonzero on input (Nx <= 4.5 M) or is needed on output.  The block
// exchange and the in-wavefront transforms are those of RowFour: slot i of
// lane l of wavefront w holds bin w + 9 (l + 64 i) between the transforms.
// WAVES_PER_EU: the occupancy asked of the compiler (at M = 1024 in the FP32
// storage modes a row takes 80 KB of LDS, so two rows share a CU at five
// wavefronts per SIMD).  HT: the scalar type of the row in HBM (the plan's
// storage type), which may differ from the transform's storage type ST.
template <class In_, int WAVES_PER_EU, class HT = typename In_::ST>
struct RowNine {
  using In = In_;
  using CT = typename In::CT;
  using ST = typename In::ST;
  using SV = typename In::SV;
  using HV = typename vec2<HT>::type;
  static constexpr int W = 9, M = In::N, R = In::R, N = W * M, T = 64 * W;
  static constexpr int NC = (M + T - 1) / T;   // column sets per thread
  static constexpr int QN = 5;                 // q < QN: possibly nonzero samples
  static constexpr int kWavesPerEu = WAVES_PER_EU;
  static_assert(In::T == 64, "one wavefront per in-wave transform");
  static constexpr int kRegion = In::kEnv;
  static constexpr size_t kLdsSlots = size_t(W) * kRegion;
  static constexpr bool kFits = kLdsSlots * sizeof(SV) <= 160 * 1024;

  BPM_INLINE static void put(SV* lds, int idx, cx<CT> v) {
    SV s;
    s.x = static_cast<ST>(v.x);
    s.y = static_cast<ST>(v.y);
    lds[idx] = s;
  }

  BPM_INLINE static void forward(cx<ST> (&v)[1][R], const HV* line, int Nx,
                                 const cx<double>* tab, SV* lds, int t) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int m = opaque(t) + T * c;
      if (T * (c + 1) <= M || m < M) {
        cx<CT> y[9], X[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          HV s;
          s.x = 0;
          s.y = 0;
          if (q < QN && m + M * q < Nx) s = line[m + M * q];
          y[q] = {static_cast<CT>(s.x), static_cast<CT>(s.y)};
        }
        dft9<false, QN>(y, X);
        cx<double> w[W];   // W_N^{m k1}
        w[1] = tab[m];
        twiddle_powers(w);
#pragma unroll
        for (int k1 = 0; k1 < W; ++k1)
          put(lds + k1 * kRegion, m, k1 ? Tw<CT>{w[k1]}.mul(X[k1]) : X[k1]);
      }
    }
    lds_barrier();
    const int l = t & 63;
    SV* own = lds + (t >> 6) * kRegion;
#pragma unroll
    for (int i = 0; i < R; ++i) v[0][i] = In::template load_as<ST>(own, l + 64 * i);
    wave_sync();
    int xbuf = 0;
    In::template fft_n<false, In::kWave, 1>(v, TwDerived<In, N>{tab}, own, opaque(l), xbuf);
  }

  BPM_INLINE static void inverse(cx<ST> (&v)[1][R], HV* line, int Nx,
                                 const cx<double>* tab, SV* lds, int t) {
    const int l = t & 63;
    SV* own = lds + (t >> 6) * kRegion;
    int xbuf = 0;
    In::template fft_n<true, In::kWave, 1>(v, TwDerived<In, N>{tab}, own, opaque(l), xbuf);
#pragma unroll
    for (int i = 0; i < R; ++i) put(own, l + 64 * i, conv<CT>(v[0][i]));
    lds_barrier();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int m = opaque(t) + T * c;
      if (T * (c + 1) <= M || m < M) {
        cx<CT> z[9], y[9];
        cx<double> w[W];
        w[1] = tab[m];
        twiddle_powers(w);
#pragma unroll
        for (int k1 = 0; k1 < W; ++k1) {
          z[k1] = In::template load_as<CT>(lds + k1 * kRegion, m);
          if (k1 > 0) z[k1] = Tw<CT>{w[k1]}.mulc(z[k1]);
        }
        dft9<true, 9>(z, y);
#pragma unroll
        for (int q = 0; q < QN; ++q)
          if (m + M * q < Nx) {
            HV s;
            s.x = static_cast<HT>(y[q].x);
            s.y = static_cast<HT>(y[q].y);
            line[m + M * q] = s;
          }
      }
    }
  }
};

// One row per work group with the radix-9 four-step transform; Q holds
// each row's table in the kernel's bin order (as for row3_four_kernel).
template <class F>
__global__ void __launch_bounds__(F::T) __attribute__((amdgpu_waves_per_eu(F::kWavesPerEu)))
row3_nine_kernel(Row3Params p) {
  using ST = typename F::ST;
  using SV = typename F::SV;
  constexpr int R = F::R, T = F::T;
  __shared__ __align__(16) SV lds[F::kLdsSlots];
  const int t = threadIdx.x;
  const int row = blockIdx.x;
  const int ky = row % p.Ny;
  const int env = (row / p.Ny) & 1;
  const int w = row / (2 * p.Ny);
  typename F::HV* line = static_cast<typename F::HV*>(env ? p.b : p.a) + (size_t(w) * p.Ny + ky) * p.Nx;
  const cx<double>* Qrow = p.Q + size_t(table_row(row, p.Ny)) * F::N;
  cx<ST> v[1][R];
  F::forward(v, line, p.Nx, p.tw, lds, t);
  phase_fence();
  const int tq = opaque(t);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    if (i % 4 == 0) phase_fence();     // table loads in groups of four
    v[0][i] = conv<ST>(cmul(to_d(v[0][i]), Qrow[i * T + tq]));
  }
  phase_fence();
  F::inverse(v, line, p.Nx, p.tw, lds, t);
}

struct Col3Params {
  const void* E0_in;          // x-space input psi~_+ (first launch)
  const void* Eh_in;          // x-space input psi~_- (first launch), or nullptr: zero
  void* a;                    // psi~_+ state / output
  void* b;                    // psi~_- state / output
  const void* table;          // [Nz][Ny][Nx] exp(i h u), or nullptr
  const unsigned char* mask;  // [Nz][Ny][Nx] crystal mask, or nullptr: the slab
  const SliceConst* sc;
  const cx<double>* wy;       // [Ny] exp(-2 pi i j / Ny)
  int Nx, Ny;
  int nb;                     // coupling sub-steps this launch applies (0..2),
  int sub[2], row[2];         //   in order: B sub-step index, step (u row)
  int mode;                   // 0 first (x-space input), 1 step, 2 last
  double dx, x_front, x_end;
};

constexpr int kCol = 64;      // x-columns per work group (one wavefront per row pair)
constexpr int kMaxNy = 32;

// blockDim = (64, H), H = (Ny + 1) / 2, grid = (ceil(Nx / 64), Nomega).
// Thread (xl, r) holds rows y = r and r + H (the second while < Ny) of
// column x of both envelopes: samples in x space, bins K_y in k space.  All
// lanes of a wavefront share r, so each DFT twiddle is one wavefront-wide
// value, and every input read from LDS serves both of the thread's outputs.
// EVEN (Ny even): the outputs r and r + Ny/2 are E + O and E - O, E and O
// the sums over the even and the odd inputs with the twiddles of r (those
// of r + Ny/2 differ by (-1)^n), so each DFT takes Ny products, not 2 Ny.
// LDS: 2 Ny kCol FP64 samples (dynamic, 45 KB at Ny = 22).
template <class ST, bool EVEN>
__global__ void __launch_bounds__(kCol * kMaxNy / 2) col3_kernel(Col3Params p) {
  using SV = typename vec2<ST>::type;
  __shared__ cx<double> sa[kMaxNy * kCol];
  __shared__ cx<double> sb[kMaxNy * kCol];
  const int xl = threadIdx.x;
  const int Ny = p.Ny, H = (Ny + 1) / 2;
  const int i0 = __builtin_amdgcn_readfirstlane(threadIdx.y);   // blockDim.x = 64
  const int i1 = i0 + H;
  const bool two = i1 < Ny;
  const int x = blockIdx.x * kCol + xl;
  const int w = blockIdx.y;
  const bool valid = x < p.Nx;
  const size_t at0 = (size_t(w) * Ny + i0) * p.Nx + x;
  const size_t at1 = (size_t(w) * Ny + i1) * p.Nx + x;
  auto ld = [](const void* f, size_t i) -> cx<double> {
    const SV s = static_cast<const SV*>(f)[i];
    return {static_cast<double>(s.x), static_cast<double>(s.y)};
  };
  auto st = [](void* f, size_t i, cx<double> v) {
    SV s;
    s.x = static_cast<ST>(v.x);
    s.y = static_cast<ST>(v.y);
    static_cast<SV*>(f)[i] = s;
  };
  // coupling sub-step j of this launch inside the crystal (Eq. fov10, Eq.
  // Authier, the sub-step constants of Eq. split-op) at (x, y_i), i = i0
  // (r = 0) or i1 (r = 1): the slab, or the general mask row of the
  // sub-step's step.  The deformation factors and mask bytes are loaded
  // here, before the transforms, so that their latency overlaps them.
  const double xp = static_cast<double>(x - p.Nx / 2) * p.dx;
  const bool in_slab = xp >= p.x_front && xp < p.x_end;
  bool inside[2][2];
  SV fac[2][2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      inside[j][r] = false;
      fac[j][r].x = 1;
      fac[j][r].y = 0;
      if (j < p.nb && valid && (r == 0 || two)) {
        const size_t idx = (size_t(p.row[j]) * Ny + (r ? i1 : i0)) * p.Nx + x;
        inside[j][r] = p.mask ? p.mask[idx] != 0 : in_slab;
        if (p.table) fac[j][r] = static_cast<const SV*>(p.table)[idx];
      }
    }
  auto couple = [&](cx<double>& a, cx<double>& b, int r, int j) {
    if (!inside[j][r]) return;
    const double* d = p.sc[w].d[p.sub[j]];
    const cx<double> d0 = {d[0], d[1]};
    cx<double> cp = {d[2], d[3]}, cm = {d[4], d[5]};
    if (p.table) {
      const cx<double> e = {static_cast<double>(fac[j][r].x), static_cast<double>(fac[j][r].y)};
      cp = cmul(cp, e);
      cm = cmulc(cm, e);
    }
    const cx<double> a0 = a;
    a = cmuladd(d0, a0, cp, b);
    b = cmuladd(d0, b, cm, a0);
  };
  auto couple_all = [&](cx<double>& a, cx<double>& b, int r) {
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (j < p.nb) couple(a, b, r, j);
  };
  cx<double> a0 = {0.0, 0.0}, b0 = {0.0, 0.0}, a1 = {0.0, 0.0}, b1 = {0.0, 0.0};
  if (p.mode == 0) {
    if (valid) {
      a0 = ld(p.E0_in, at0);
      if (two) a1 = ld(p.E0_in, at1);
      if (p.Eh_in) {
        b0 = ld(p.Eh_in, at0);
        if (two) b1 = ld(p.Eh_in, at1);
      }
    }
    if (valid) {
      couple_all(a0, b0, 0);
      if (two) couple_all(a1, b1, 1);
    }
  } else {
    if (valid) {
      sa[i0 * kCol + xl] = ld(p.a, at0);
      sb[i0 * kCol + xl] = ld(p.b, at0);
      if (two) {
        sa[i1 * kCol + xl] = ld(p.a, at1);
        sb[i1 * kCol + xl] = ld(p.b, at1);
      }
    }
    lds_barrier();
    // inverse DFT along y (unnormalised; 1/Ny is in the propagator)
    if constexpr (EVEN) {
      cx<double> ao = {0.0, 0.0}, bo = {0.0, 0.0};   // odd inputs; even in a0, b0
      for (int k = 0, m0 = 0; k < Ny; k += 2) {      // m0 = i0 k mod Ny
        const cx<double> t0 = conjd(p.wy[m0]);
        a0 = cmac(a0, sa[k * kCol + xl], t0);
        b0 = cmac(b0, sb[k * kCol + xl], t0);
        m0 += i0;
        if (m0 >= Ny) m0 -= Ny;
        const cx<double> t1 = conjd(p.wy[m0]);
        ao = cmac(ao, sa[(k + 1) * kCol + xl], t1);
        bo = cmac(bo, sb[(k + 1) * kCol + xl], t1);
        m0 += i0;
        if (m0 >= Ny) m0 -= Ny;
      }
      a1 = a0 - ao;
      b1 = b0 - bo;
      a0 = a0 + ao;
      b0 = b0 + bo;
    } else {
      for (int k = 0, m0 = 0, m1 = 0; k < Ny; ++k) {   // m = i k mod Ny
        const cx<double> A = sa[k * kCol + xl], B = sb[k * kCol + xl];
        const cx<double> t0 = conjd(p.wy[m0]);
        a0 = cmac(a0, A, t0);
        b0 = cmac(b0, B, t0);
        if (two) {
          const cx<double> t1 = conjd(p.wy[m1]);
          a1 = cmac(a1, A, t1);
          b1 = cmac(b1, B, t1);
        }
        m0 += i0;
        if (m0 >= Ny) m0 -= Ny;
        m1 += i1 - Ny;             // i1 < Ny: one correction suffices
        if (m1 < 0) m1 += Ny;
      }
    }
    if (valid) {
      couple_all(a0, b0, 0);
      if (two) couple_all(a1, b1, 1);
    }
    lds_barrier();        // every column read before it is overwritten
  }
  if (p.mode == 2) {
    if (valid) {
      st(p.a, at0, a0);
      st(p.b, at0, b0);
      if (two) {
        st(p.a, at1, a1);
        st(p.b, at1, b1);
      }
    }
    return;
  }
  sa[i0 * kCol + xl] = a0;
  sb[i0 * kCol + xl] = b0;
  if (two) {
    sa[i1 * kCol + xl] = a1;
    sb[i1 * kCol + xl] = b1;
  }
  lds_barrier();
  cx<double> A0 = {0.0, 0.0}, B0 = {0.0, 0.0}, A1 = {0.0, 0.0}, B1 = {0.0, 0.0};
  if constexpr (EVEN) {
    cx<double> Ao = {0.0, 0.0}, Bo = {0.0, 0.0};
    for (int j = 0, m0 = 0; j < Ny; j += 2) {
      const cx<double> t0 = p.wy[m0];
      A0 = cmac(A0, sa[j * kCol + xl], t0);
      B0 = cmac(B0, sb[j * kCol + xl], t0);
      m0 += i0;
      if (m0 >= Ny) m0 -= Ny;
      const cx<double> t1 = p.wy[m0];
      Ao = cmac(Ao, sa[(j + 1) * kCol + xl], t1);
      Bo = cmac(Bo, sb[(j + 1) * kCol + xl], t1);
      m0 += i0;
      if (m0 >= Ny) m0 -= Ny;
    }
    A1 = A0 - Ao;
    B1 = B0 - Bo;
    A0 = A0 + Ao;
    B0 = B0 + Bo;
  } else {
    for (int j = 0, m0 = 0, m1 = 0; j < Ny; ++j) {
      const cx<double> A = sa[j * kCol + xl], B = sb[j * kCol + xl];
      const cx<double> t0 = p.wy[m0];
      A0 = cmac(A0, A, t0);
      B0 = cmac(B0, B, t0);
      if (two) {
        const cx<double> t1 = p.wy[m1];
        A1 = cmac(A1, A, t1);
        B1 = cmac(B1, B, t1);
      }
      m0 += i0;
      if (m0 >= Ny) m0 -= Ny;
      m1 += i1 - Ny;
      if (m1 < 0) m1 += Ny;
    }
  }
  if (valid) {
    st(p.a, at0, A0);
    st(p.b, at0, B0);
    if (two) {
      st(p.a, at1, A1);
      st(p.b, at1, B1);
    }
  }
}

// Row transforms by length L (thread count L / R).
template <int PREC, int L> struct Row3T;
template <int PREC> struct Row3T<PREC, 64> { using type = March<PREC, 64, 4, 4, 4, 4>; };
template <int PREC> struct Row3T<PREC, 128> { using type = March<PREC, 128, 8, 8, 4, 4>; };
template <int PREC> struct Row3T<PREC, 256> { using type = March<PREC, 256, 4, 4, 4, 4, 4>; };
template <int PREC> struct Row3T<PREC, 512> { using type = March<PREC, 512, 8, 8, 8, 8>; };
template <int PREC> struct Row3T<PREC, 1024> { using type = March<PREC, 1024, 8, 8, 8, 4, 4>; };
template <int PREC> struct Row3T<PREC, 2048> { using type = March<PREC, 2048, 8, 8, 8, 8, 4>; };
template <int PREC> struct Row3T<PREC, 4096> { using type = March<PREC, 4096, 8, 8, 8, 8, 8>; };
template <int PREC> struct Row3T<PREC, 8192> { using type = RowFour<InWave1024<PREC>, 8>; };
template <int PREC> struct Row3T<PREC, 16384> { using type = RowFour<InWave1024<PREC>, 16>; };
// 9 M: fp32 rows of 9216 ask for the five wavefronts per SIMD of two rows
// per CU; fp32s rows of 9216 run the FP64 transform (FP64 LDS exchanges, one
// row per CU) on their FP32 rows in HBM, measured 2% faster than two rows
// per CU with FP32 exchanges and their conversions; rows of 4608 ask for the
// seven wavefronts per SIMD of three rows per CU; FP64 rows fill the LDS.
template <int PREC> struct Row3T<PREC, 4608> {
  using type = RowNine<InWave512<PREC>, PREC == BPM_PREC_FP64 ? 1 : 7>;
};
template <int PREC> struct Row3T<PREC, 9216> {
  using type = RowNine<InWave1024<PREC == BPM_PREC_FP32S ? BPM_PREC_FP64 : PREC>,
                       PREC == BPM_PREC_FP32 ? 5 : 1, typename Prec<PREC>::ST>;
};

template <int PREC, int L>
int launch_row3_l(int rows, const Row3Params& p, hipStream_t s) {
  if constexpr (!row3_fits(PREC, L)) {
    return BPM_EUNSUPPORTED;   // a row of this length and storage does not fit in LDS
  } else {
    using M = typename Row3T<PREC, L>::type;
    if constexpr (L % 9 == 0) {
      if (2 * p.Nx > L) return BPM_EINVAL;   // the radix-9 steps read and write q < 5
      hipLaunchKernelGGL((row3_nine_kernel<M>), dim3(rows), dim3(M::T), 0, s, p);
    } else if constexpr (L >= kRow3FourStepMin) {
      hipLaunchKernelGGL((row3_four_kernel<M>), dim3(rows), dim3(M::T), 0, s, p);
    } else {
      hipLaunchKernelGGL((row3_kernel<M>), dim3(rows), dim3(M::T), 0, s, p);
    }
    return hipGetLastError() == hipSuccess ? BPM_OK : BPM_EHIP;
  }
}

template <int PREC>
int launch_row3_p(int L, int rows, const Row3Params& p, hipStream_t s) {
  switch (L) {
    case 64: return launch_row3_l<PREC, 64>(rows, p, s);
    case 128: return launch_row3_l<PREC, 128>(rows, p, s);
    case 256: return launch_row3_l<PREC, 256>(rows, p, s);
    case 512: return launch_row3_l<PREC, 512>(rows, p, s);
    case 1024: return launch_row3_l<PREC, 1024>(rows, p, s);
    case 2048: return launch_row3_l<PREC, 2048>(rows, p, s);
    case 4096: return launch_row3_l<PREC, 4096>(rows, p, s);
    case 4608: return launch_row3_l<PREC, 4608>(rows, p, s);
    case 8192: return launch_row3_l<PREC, 8192>(rows, p, s);
    case 9216: return launch_row3_l<PREC, 9216>(rows, p, s);
    case 16384: return launch_row3_l<PREC, 16384>(rows, p, s);
    default: return BPM_EUNSUPPORTED;
  }
}

}  // namespace

int launch_prop3(void* P, const SliceConst* sc, int Nx, int Ny, int Nomega, double dx,
                 double dy, double dz, double frac, double h_half, hipStream_t s) {
  const size_t n = size_t(Nomega) * 2 * (Ny / 2 + 1) * Nx;
  const int block = 256;
  const size_t want = (n + block - 1) / block;
  const int grid = static_cast<int>(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(prop3_kernel, dim3(grid), dim3(block), 0, s, static_cast<cx<double>*>(P),
                     sc, Nx, Ny, Nomega, dx, dy, dz, frac, h_half);
  return hipGetLastError() == hipSuccess ? BPM_OK : BPM_EHIP;
}

int launch_march3(const March3Params& q, hipStream_t s) {
  if (q.Ny < 1 || q.Ny > kMaxNy) return BPM_EUNSUPPORTED;
  Col3Params c{};
  c.E0_in = q.E0_in;
  c.Eh_in = q.Eh_in;
  c.a = q.E0_out;
  c.b = q.Eh_out;
  c.table = q.table;
  c.mask = static_cast<const unsigned char*>(q.mask);
  c.sc = q.sc;
  c.wy = static_cast<const cx<double>*>(q.wy);
  c.Nx = q.Nx;
  c.Ny = q.Ny;
  c.dx = q.dx;
  c.x_front = q.x_front;
  c.x_end = q.x_end;
  Row3Params r{};
  r.a = q.E0_out;
  r.b = q.Eh_out;
  r.tw = static_cast<const cx<double>*>(q.tw);
  r.Nx = q.Nx;
  r.Ny = q.Ny;
  const dim3 cgrid((q.Nx + kCol - 1) / kCol, q.Nomega);
  const dim3 cblock(kCol, (q.Ny + 1) / 2);
  const int rows = q.Nomega * 2 * q.Ny;
  const bool even = q.Ny % 2 == 0;
  auto col = [&](int mode) -> int {
    c.mode = mode;
    if (q.prec == BPM_PREC_FP64) {
      if (even)
        hipLaunchKernelGGL((col3_kernel<double, true>), cgrid, cblock, 0, s, c);
      else
        hipLaunchKernelGGL((col3_kernel<double, false>), cgrid, cblock, 0, s, c);
    } else {
      if (even)
        hipLaunchKernelGGL((col3_kernel<float, true>), cgrid, cblock, 0, s, c);
      else
        hipLaunchKernelGGL((col3_kernel<float, false>), cgrid, cblock, 0, s, c);
    }
    c.nb = 0;
    return hipGetLastError() == hipSuccess ? BPM_OK : BPM_EHIP;
  };
  auto row = [&](int set) -> int {
    r.Q = static_cast<const cx<double>*>(q.rows) + size_t(set) * q.set_elems;
    switch (q.prec) {
      case BPM_PREC_FP64: return launch_row3_p<BPM_PREC_FP64>(q.L, rows, r, s);
      case BPM_PREC_FP32: return launch_row3_p<BPM_PREC_FP32>(q.L, rows, r, s);
      case BPM_PREC_FP32S: return launch_row3_p<BPM_PREC_FP32S>(q.L, rows, r, s);
      default: return BPM_EUNSUPPORTED;
    }
  };
  // The sub-steps A(a_i dz) B(b_i dz) of every step in order (Eq. split-op);
  // the B sub-steps between two A sub-steps go to one column launch (at
  // most two: the last of a step and the first of the next).
  int rc = BPM_OK;
  int mode = 0;
  c.nb = 0;
  for (int n = q.n0; rc == BPM_OK && n < q.n0 + q.Nz; ++n) {
    for (int i = 0; rc == BPM_OK && i < q.nsub; ++i) {
      if (q.a_set[i] >= 0) {
        rc = col(mode);
        mode = 1;
        if (rc == BPM_OK) rc = row(q.a_set[i]);
      }
      if (c.nb == 2) return BPM_EUNSUPPORTED;   // not produced by the schemes built
      c.sub[c.nb] = i;
      c.row[c.nb] = n;
      ++c.nb;
    }
  }
  if (rc == BPM_OK) rc = col(2);
  return rc;
}

}  // namespace bpm

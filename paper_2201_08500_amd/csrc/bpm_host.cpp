// Host side of the C ABI: argument validation, FP64 plan constants, device
// constant upload and the propagate entry points.

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <limits>
#include <map>
#include <queue>
#include <tuple>
#include <string>
#include <system_error>
#include <thread>
#include <utility>
#include <vector>

#include "bpm_internal.h"

using cplx = std::complex<double>;

namespace {

thread_local std::string g_error;

int fail(int code, const std::string& msg) {
  g_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(BPM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// J0(sqrt q) and 2 J1(sqrt q)/sqrt q as power series in q:
//   S0 = sum_m (-q/4)^m / (m!)^2,  S1 = sum_m (-q/4)^m / (m! (m+1)!).
// Both are entire and even in sqrt(q), so no branch of sqrt(q) is needed
// (Jacobi-Anger coefficients of Eqs. fov11, fov12 with chih != chihbar).
void bessel_series(cplx q, cplx& S0, cplx& S1) {
  const cplx x = -q / 4.0;
  cplx t0 = 1.0, t1 = 1.0;
  S0 = t0;
  S1 = t1;
  for (int m = 1; m < 300; ++m) {
    t0 *= x / double(m) / double(m);
    t1 *= x / double(m) / double(m + 1);
    S0 += t0;
    S1 += t1;
    if (std::abs(t0) <= 1e-18 * std::abs(S0) &&
        std::abs(t1) <= 1e-18 * std::abs(S1))
      break;
  }
}

// Sub-step fractions of Eq. split-op.
void split_fractions(int order, int& n, double a[4], double b[4]) {
  if (order == 2) {
    n = 2;
    a[0] = 0.0; a[1] = 1.0;
    b[0] = 0.5; b[1] = 0.5;
  } else if (order == 4) {
    const double t = 1.0 / (2.0 - std::cbrt(2.0));
    n = 4;
    a[0] = 0.0; a[1] = t; a[2] = 1.0 - 2.0 * t; a[3] = t;
    b[0] = t / 2; b[1] = (1 - t) / 2; b[2] = (1 - t) / 2; b[3] = t / 2;
  } else {
    n = 1;
    a[0] = 1.0;
    b[0] = 1.0;
  }
}

// Per-slice constants: k, and for each B sub-step of length frac*dz the
// coupling d0 = S0 exp(q/8) g0 (Zassenhaus factor D2 dZ^2/2 = q/8),
// d+-1 = i (dZ chi_{h,hbar} / 2c) S1 g0, g0 = exp(i dZ chi0 / 2c),
// q = dZ^2 chih chihbar / c^2, dZ = frac k dz, c = sqrt(1 - (h/2k)^2).
int compute_slice_constants(bpm_plan* p) {
  int nsub;
  double a[4], b[4];
  split_fractions(p->split_order, nsub, a, b);
  p->sc.assign(p->Nomega, bpm::SliceConst{});
  for (int w = 0; w < p->Nomega; ++w) {
    bpm::SliceConst& s = p->sc[w];
    const double k = p->k0 * (1.0 + p->delta[w]);
    const double sh = 0.5 * p->h / k;
    if (!(k > 0.0) || !(sh < 1.0))
      return fail(BPM_EINVAL, "slice " + std::to_string(w) +
                                  ": h/2 >= k (no propagating Bragg pair)");
    const double c = std::sqrt(1.0 - sh * sh);
    s.k = k;
    for (int i = 0; i < nsub; ++i) {
      const double dZ = b[i] * (k * p->dz);
      const cplx q = dZ * dZ * p->chih * p->chihbar / (c * c);
      if (std::abs(q) > 16.0)
        return fail(BPM_EINVAL,
                    "step too long for the two-beam expansion: |q| = " +
                        std::to_string(std::abs(q)) + " > 16");
      cplx S0, S1;
      bessel_series(q, S0, S1);
      const cplx I(0.0, 1.0);
      const cplx g0 = std::exp(I * dZ * p->chi0 / (2.0 * c));
      cplx d0 = S0 * g0;
      if (p->zassenhaus) d0 *= std::exp(q / 8.0);
      const cplx dp1 = I * (dZ * p->chih / (2.0 * c)) * S1 * g0;
      const cplx dm1 = I * (dZ * p->chihbar / (2.0 * c)) * S1 * g0;
      s.d[i][0] = d0.real(); s.d[i][1] = d0.imag();
      s.d[i][2] = dp1.real(); s.d[i][3] = dp1.imag();
      s.d[i][4] = dm1.real(); s.d[i][5] = dm1.imag();
    }
  }
  return BPM_OK;
}

cplx mul_h(cplx a, cplx b) {
  return cplx(a.real() * b.real() - a.imag() * b.imag(),
              a.real() * b.imag() + a.imag() * b.real());
}

// Forward FFT (kernel exp(-2 pi i jk / n), no scaling) of a power-of-two
// length n in FP64, in place: iterative radix 2, twiddles from the table
// tab[m stride] = exp(-2 pi i m / n) (a table of length n stride).
void fft_host(cplx* a, size_t n, const cplx* tab, size_t stride = 1) {
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    const size_t step = n / len * stride;
    for (size_t i = 0; i < n; i += len) {
      for (size_t k = 0; k < len / 2; ++k) {
        const cplx u = a[i + k], v = mul_h(a[i + k + len / 2], tab[k * step]);
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
    }
  }
}

// Forward FFT of length n = 9 M (M a power of two) in FP64, in place, by
// the four-step decomposition n = m + M q, k = k1 + 9 k2: a direct 9-point
// DFT over q for every m, the twiddle W_n^{m k1}, then nine M-point FFTs.
// tab[j] = exp(-2 pi i j / n).
void fft_nine_host(cplx* a, size_t n, const cplx* tab) {
  const size_t M = n / 9;
  std::vector<cplx> b(n);   // b[k1 M + m]
  for (size_t m = 0; m < M; ++m)
    for (size_t k1 = 0; k1 < 9; ++k1) {
      cplx acc(0.0, 0.0);
      for (size_t q = 0; q < 9; ++q) acc += mul_h(a[m + M * q], tab[(M * q * k1) % n]);
      b[k1 * M + m] = mul_h(acc, tab[m * k1]);
    }
  for (size_t k1 = 0; k1 < 9; ++k1) {
    fft_host(b.data() + k1 * M, M, tab, 9);
    for (size_t k2 = 0; k2 < M; ++k2) a[k1 + 9 * k2] = b[k1 * M + k2];
  }
}

// Bluestein's convolution length for Nx: the smallest power of two >=
// max(2 Nx - 1, 64).
size_t bluestein_length(int Nx) {
  size_t L = 64;
  while (L < size_t(2) * Nx - 1) L <<= 1;
  return L;
}

// FP64 tables of a 3D plan: the length-L twiddles exp(-2 pi i m / L), the
// y-DFT twiddles exp(-2 pi i j / Ny) (both on the device), and for lengths
// Nx that are not transformed directly the chirp w_n = exp(-i pi n^2 / Nx)
// (n^2 reduced modulo 2 Nx in integers), the twiddles twb of Bluestein's
// power-of-two length Lb and G = FFT_Lb(conj(w) wrapped circularly) / Lb
// (host only).
struct Tables3 {
  std::vector<cplx> tw, wy, chirp, twb, G;
};

std::vector<cplx> twiddles_host(size_t L) {
  std::vector<cplx> tw(L);
  for (size_t m = 0; m < L; ++m) {
    const double ang = -2.0 * M_PI * double(m) / double(L);
    tw[m] = cplx(std::cos(ang), std::sin(ang));
  }
  return tw;
}

Tables3 tables3(const bpm_plan* p) {
  const int N = p->Nx, Ny = p->Ny;
  Tables3 t;
  t.tw = twiddles_host(size_t(p->L3));
  t.wy.resize(Ny);
  for (int j = 0; j < Ny; ++j) {
    const double ang = -2.0 * M_PI * double(j) / double(Ny);
    t.wy[j] = cplx(std::cos(ang), std::sin(ang));
  }
  if (p->bluestein) {
    t.chirp.resize(N);
    for (int n = 0; n < N; ++n) {
      const long long m = (static_cast<long long>(n) * n) % (2LL * N);
      const double ang = -M_PI * double(m) / double(N);
      t.chirp[n] = cplx(std::cos(ang), std::sin(ang));
    }
    const size_t Lb = bluestein_length(N);
    t.twb = size_t(p->L3) == Lb ? t.tw : twiddles_host(Lb);
    t.G.assign(Lb, cplx(0.0, 0.0));
    for (int m = 0; m < N; ++m) t.G[m] = std::conj(t.chirp[m]);
    for (int m = 1; m < N; ++m) t.G[Lb - m] = std::conj(t.chirp[m]);
    fft_host(t.G.data(), Lb, t.twb.data());
    for (auto& v : t.G) v /= double(Lb);
  }
  return t;
}

// Row tables Q = FFT_L(q) / L of a plan whose Nx is not transformed
// directly, from its propagator rows P (length Nx, FP64): p = IDFT_Nx(P)
// (unnormalised) = conj(DFT_Nx(conj(P))) by Bluestein's algorithm
// (X_k = w_k (a * conj(w))_k, a_n = x_n w_n, the cyclic convolution on the
// power of two Lb), then q_d = p_d and q_{L-Nx+d} = p_d (d >= 1), zero
// elsewhere, and its FFT on the row length L (a power of two or 9 M).  Rows
// are shared out over host threads.
void rows3_bluestein(const bpm_plan* p, const Tables3& t, const std::vector<cplx>& P,
                     std::vector<cplx>& Q) {
  const int N = p->Nx;
  const size_t L = size_t(p->L3), Lb = t.G.size();
  const size_t rows = size_t(p->Nomega) * 2 * (p->Ny / 2 + 1);   // table rows
  Q.assign(rows * L, cplx(0.0, 0.0));
  auto work = [&](size_t r0, size_t r1) {
    std::vector<cplx> buf(Lb), q(L);
    for (size_t r = r0; r < r1; ++r) {
      const cplx* Pr = P.data() + r * N;
      std::fill(buf.begin(), buf.end(), cplx(0.0, 0.0));
      for (int n = 0; n < N; ++n) buf[n] = mul_h(std::conj(Pr[n]), t.chirp[n]);
      fft_host(buf.data(), Lb, t.twb.data());
      // conj of the unnormalised inverse transform: buf = conj(a * conj(w))
      for (size_t j = 0; j < Lb; ++j) buf[j] = std::conj(mul_h(buf[j], t.G[j]));
      fft_host(buf.data(), Lb, t.twb.data());
      std::fill(q.begin(), q.end(), cplx(0.0, 0.0));
      for (int d = 0; d < N; ++d) {
        const cplx pd = mul_h(std::conj(t.chirp[d]), buf[d]);   // conj(X_d)
        q[d] = pd;
        if (d > 0) q[L - N + d] = pd;
      }
      if (is_pow2(int(L)))
        fft_host(q.data(), L, t.tw.data());
      else
        fft_nine_host(q.data(), L, t.tw.data());
      cplx* Qr = Q.data() + r * L;
      for (size_t j = 0; j < L; ++j) Qr[j] = q[j] / double(L);
    }
  };
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const size_t nt = std::min<size_t>({size_t(hw), size_t(16), rows});
  std::vector<std::thread> pool;
  size_t started = 1;   // ranges 1..started-1 run on pool threads
  for (; started < nt; ++started) {
    try {
      pool.emplace_back(work, rows * started / nt, rows * (started + 1) / nt);
    } catch (const std::system_error&) {
      break;            // no more threads: the calling thread takes the rest
    }
  }
  work(0, rows / nt);
  work(rows * started / nt, rows);
  for (auto& th : pool) th.join();
}

// Freeze the plan's host state on first use: constants computed once, no
// device call.  Caller holds p->mu.
int freeze_host_locked(bpm_plan* p) {
  if (p->frozen) return BPM_OK;
  int rc = compute_slice_constants(p);
  if (rc != BPM_OK) return rc;
  p->frozen = true;
  return BPM_OK;
}

// Rows that the four-step row kernels read (row3_four_step) are stored in
// their bin order: entry i T + t of a row is bin w + W (l + 64 i) of thread
// t = 64 w + l (W = row3_waves(L), T = 64 W, i < L / T).
void permute_rows3(std::vector<cplx>& Q, size_t rows, int L) {
  const int W = bpm::row3_waves(L), T = 64 * W, R = L / T;
  std::vector<cplx> tmp(L);
  for (size_t r = 0; r < rows; ++r) {
    cplx* q = Q.data() + r * size_t(L);
    for (int i = 0; i < R; ++i)
      for (int t = 0; t < T; ++t) tmp[size_t(i) * T + t] = q[(t >> 6) + W * ((t & 63) + 64 * i)];
    std::copy(tmp.begin(), tmp.end(), q);
  }
}

// Distinct A sub-step lengths (fractions of dz) of the plan's scheme, and
// for each sub-step the index of its length (-1 where a_i = 0).
int a_sets3(const bpm_plan* p, double frac[4], int set_of[4]) {
  int nsub;
  double a[4], b[4];
  split_fractions(p->split_order, nsub, a, b);
  int n = 0;
  for (int i = 0; i < nsub; ++i) {
    set_of[i] = -1;
    if (a[i] == 0.0) continue;
    for (int j = 0; j < n; ++j)
      if (frac[j] == a[i]) set_of[i] = j;
    if (set_of[i] < 0) {
      frac[n] = a[i];
      set_of[i] = n++;
    }
  }
  return n;
}

// Device tables of a 3D plan: twiddles and, for each distinct A sub-step
// length, the row propagator tables (rows of length L; for L = Nx the
// propagator itself, evaluated on the device; otherwise Q from the device
// propagator via the host; long rows permuted to the four-step bin order).
// Uses the null stream and waits for it.  Caller holds p->mu, after dev_sc.
int upload_tables3(bpm_plan* p) {
  const Tables3 t = tables3(p);
  const size_t L = size_t(p->L3);
  const size_t rows = size_t(p->Nomega) * 2 * (p->Ny / 2 + 1);   // table rows
  double frac[4];
  int set_of[4];
  const int nsets = a_sets3(p, frac, set_of);
  hipError_t e = hipMalloc(&p->dev_tables3, (L + t.wy.size()) * sizeof(cplx));
  if (e != hipSuccess) {
    p->dev_tables3 = nullptr;
    return fail(BPM_ENOMEM, std::string("hipMalloc(3D tables): ") + hipGetErrorString(e));
  }
  cplx* dt = static_cast<cplx*>(p->dev_tables3);
  e = hipMemcpy(dt, t.tw.data(), L * sizeof(cplx), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(dt + L, t.wy.data(), t.wy.size() * sizeof(cplx), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(3D tables)");
  e = hipMalloc(&p->dev_rows3, size_t(nsets) * rows * L * sizeof(cplx));
  if (e != hipSuccess) {
    p->dev_rows3 = nullptr;
    return fail(BPM_ENOMEM, std::string("hipMalloc(3D row propagators): ") +
                                hipGetErrorString(e));
  }
  // The propagator is evaluated on the device; the rows go through the host
  // when they need the cyclic-convolution table or the four-step bin order.
  const bool via_host = p->bluestein || bpm::row3_four_step(p->L3);
  for (int set = 0; set < nsets; ++set) {
    cplx* dst = static_cast<cplx*>(p->dev_rows3) + size_t(set) * rows * L;
    void* P = dst;
    if (via_host) {
      e = hipMalloc(&P, rows * size_t(p->Nx) * sizeof(cplx));
      if (e != hipSuccess)
        return fail(BPM_ENOMEM, std::string("hipMalloc(3D propagator): ") + hipGetErrorString(e));
    }
    int rc = bpm::launch_prop3(P, p->dev_sc, p->Nx, p->Ny, p->Nomega, p->dx, p->dy, p->dz,
                               frac[set], 0.5 * p->h, nullptr);
    if (rc != BPM_OK) {
      if (via_host) (void)hipFree(P);
      return fail(rc, "3D propagator table launch failed");
    }
    if (!via_host) {
      e = hipStreamSynchronize(nullptr);
      if (e != hipSuccess) return hip_fail(e, "3D propagator table");
      continue;
    }
    std::vector<cplx> hP(rows * size_t(p->Nx)), Q;
    e = hipMemcpy(hP.data(), P, hP.size() * sizeof(cplx), hipMemcpyDeviceToHost);
    (void)hipFree(P);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(3D propagator)");
    if (p->bluestein)
      rows3_bluestein(p, t, hP, Q);
    else
      Q.swap(hP);
    if (bpm::row3_four_step(p->L3)) permute_rows3(Q, rows, p->L3);
    e = hipMemcpy(dst, Q.data(), Q.size() * sizeof(cplx), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(3D row propagators)");
  }
  return BPM_OK;
}

// Frees whatever device copies of the plan exist.  Caller holds p->mu.
void drop_device_locked(bpm_plan* p) {
  for (void** q : {reinterpret_cast<void**>(&p->dev_sc), reinterpret_cast<void**>(&p->dev_mask),
                   &p->dev_tables3, &p->dev_rows3}) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
}

int upload_locked(bpm_plan* p) {
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipMalloc(&p->dev_sc, sizeof(bpm::SliceConst) * p->Nomega);
  if (e != hipSuccess) {
    p->dev_sc = nullptr;
    return fail(BPM_ENOMEM, std::string("hipMalloc(plan constants): ") +
                                hipGetErrorString(e));
  }
  e = hipMemcpy(p->dev_sc, p->sc.data(), sizeof(bpm::SliceConst) * p->Nomega,
                hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(plan constants)");
  if (!p->mask.empty()) {
    e = hipMalloc(&p->dev_mask, p->mask.size());
    if (e != hipSuccess) {
      p->dev_mask = nullptr;
      return fail(BPM_ENOMEM, std::string("hipMalloc(crystal mask): ") + hipGetErrorString(e));
    }
    e = hipMemcpy(p->dev_mask, p->mask.data(), p->mask.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(crystal mask)");
  }
  if (p->three_d) return upload_tables3(p);
  return BPM_OK;
}

// Freeze the plan and upload its constants (general mask, 3D tables) once;
// a failed upload leaves no device copy behind.
int freeze(bpm_plan* p) {
  std::lock_guard<std::mutex> lock(p->mu);
  int rc = freeze_host_locked(p);
  if (rc != BPM_OK) return rc;
  if (p->dev_sc && (!p->three_d || p->dev_rows3)) return BPM_OK;
  drop_device_locked(p);
  rc = upload_locked(p);
  if (rc != BPM_OK) drop_device_locked(p);
  return rc;
}

// A 3D plan can only propagate whole marches (bpm_propagate, _ws).
int reject_3d(const bpm_plan* p, const char* what) {
  if (p && p->three_d)
    return fail(BPM_EUNSUPPORTED, std::string(what) + " is not available for 3D plans");
  return BPM_OK;
}

// Steps [n0, n0 + nsteps) of the 3D march from x-space envelopes (Eh_in
// NULL: zero), reading the deformation table (or none): the row and column
// launches of every sub-step (bpm3d.hip).
int march3(bpm_plan* p, const void* E0_in, const void* Eh_in, const void* table, int n0,
           int nsteps, void* E0_out, void* Eh_out, hipStream_t s) {
  if (!bpm::row3_fits(p->precision, p->L3))
    return fail(BPM_EUNSUPPORTED, "FP64 3D rows need a transform length <= 9216 "
                                  "(Nx <= 4608, or a power of two <= 8192)");
  int rc = freeze(p);
  if (rc) return rc;
  const cplx* t3 = static_cast<const cplx*>(p->dev_tables3);
  bpm::March3Params q{};
  q.prec = p->precision;
  q.Nx = p->Nx;
  q.Ny = p->Ny;
  q.Nz = nsteps;
  q.n0 = n0;
  q.Nomega = p->Nomega;
  q.L = p->L3;
  q.dx = p->dx;
  q.x_front = p->x_front;
  q.x_end = p->x_front + p->thickness;
  q.E0_in = E0_in;
  q.Eh_in = Eh_in;
  q.E0_out = E0_out;
  q.Eh_out = Eh_out;
  q.table = table;
  q.mask = p->mask.empty() ? nullptr : p->dev_mask;
  q.sc = p->dev_sc;
  q.rows = p->dev_rows3;
  q.set_elems = size_t(p->Nomega) * 2 * (p->Ny / 2 + 1) * size_t(p->L3);
  {
    int nsub;
    double a[4], b[4], frac[4];
    split_fractions(p->split_order, nsub, a, b);
    q.nsub = nsub;
    a_sets3(p, frac, q.a_set);
  }
  q.tw = t3;
  q.wy = t3 + p->L3;
  rc = bpm::launch_march3(q, s);
  if (rc == BPM_EUNSUPPORTED) return fail(rc, "unsupported 3D size/precision");
  if (rc) return fail(rc, "3D march launch failed");
  return BPM_OK;
}

// The whole 3D march: deformation table, then every step.
int propagate3(bpm_plan* p, const void* E0_in, const double* u_field, void* E0_out,
               void* Eh_out, void* workspace, hipStream_t s) {
  if (!bpm::row3_fits(p->precision, p->L3))
    return fail(BPM_EUNSUPPORTED, "FP64 3D rows need a transform length <= 9216 "
                                  "(Nx <= 4608, or a power of two <= 8192)");
  int rc = freeze(p);
  if (rc) return rc;
  void* table = nullptr;
  if (u_field) {
    table = workspace;
    rc = bpm::launch_deform(p->precision, p->Nx * p->Ny, p->Nz, p->h, u_field, table, s);
    if (rc) return fail(rc, "deformation pre-pass launch failed");
  }
  return march3(p, E0_in, nullptr, table, 0, p->Nz, E0_out, Eh_out, s);
}

int plan_schedule(const bpm_plan* p) {
  return p->schedule >= 0 ? p->schedule
                          : bpm::default_schedule(p->precision, p->Nx);
}

int check_mutable(bpm_plan* p) {
  if (!p) return fail(BPM_EINVAL, "plan is NULL");
  if (p->frozen) return fail(BPM_EINVAL, "plan is frozen after its first propagate");
  return BPM_OK;
}

void default_detuning(bpm_plan* p) {
  p->delta.assign(p->Nomega, 0.0);
  if (p->Nomega == 1) return;
  const double eps = std::abs(std::sqrt(p->chih * p->chihbar)) /
                     (std::sin(p->theta_B) * std::sin(p->theta_B));
  for (int j = 0; j < p->Nomega; ++j)
    p->delta[j] = eps * (-5.0 + 10.0 * (j + 0.5) / p->Nomega);
}

bpm::MarchParams march_params(const bpm_plan* p, const void* E0_in,
                              const void* table, void* E0_out, void* Eh_out) {
  bpm::MarchParams m{};
  m.E0_in = E0_in;
  m.E0_out = E0_out;
  m.Eh_out = Eh_out;
  m.table = table;
  m.sc = p->dev_sc;
  m.Nz = p->Nz;
  int nsub;
  double b[4];
  split_fractions(p->split_order, nsub, m.a_frac, b);
  m.nsub = nsub;
  m.dx = p->dx;
  m.dz = p->dz;
  m.h_half = 0.5 * p->h;
  m.x_front = p->x_front;
  m.x_end = p->x_front + p->thickness;
  m.mask = p->dev_mask;
  return m;
}

struct DeformJob {
  int prec, Nx, Nz;
  double h;
  const double* u;
  void* table;
};

struct BatchGroup {
  int prec, Nx, sched, order;
  bool masked;
  int n_groups;
  int n_items;
  bpm::BatchItem* d_items;
  int* d_offsets;
};

}  // namespace

namespace bpm {
int set_error(int code, const std::string& msg) { return fail(code, msg); }
void clear_error() { g_error.clear(); }
int plan_freeze_host(bpm_plan* p) {
  std::lock_guard<std::mutex> lock(p->mu);
  return freeze_host_locked(p);
}
int plan_schedule_of(const bpm_plan* p) { return plan_schedule(p); }
MarchParams plan_march_params(const bpm_plan* p, const void* E0_in, const void* table,
                              void* E0_out, void* Eh_out) {
  return march_params(p, E0_in, table, E0_out, Eh_out);
}
}  // namespace bpm

struct bpm_batch {
  std::vector<DeformJob> deforms;
  std::vector<BatchGroup> groups;
  void* d_mem = nullptr;        // one device allocation for all work lists
  bool stream_ordered = false;  // allocated with hipMallocAsync
};

namespace {

int validate_job(const bpm_job& j, int idx) {
  const std::string at = "job " + std::to_string(idx) + ": ";
  if (!j.plan) return fail(BPM_EINVAL, at + "plan is NULL");
  if (j.plan->three_d) return fail(BPM_EUNSUPPORTED, at + "3D plans are not batched");
  if (!j.E0_in || !j.E0_out || !j.Eh_out)
    return fail(BPM_EINVAL, at + "E0_in, E0_out and Eh_out must be non-NULL");
  if (j.E0_in == j.E0_out || j.E0_in == j.Eh_out || j.E0_out == j.Eh_out)
    return fail(BPM_EINVAL, at + "output buffers must not alias each other or E0_in");
  if (j.u_field && !j.workspace)
    return fail(BPM_EINVAL, at + "a deformed job needs a workspace");
  return BPM_OK;
}

// Build a batch; with a non-null stream the device work lists are
// allocated stream-ordered on it.
// Page-locked host blocks for the work-list uploads of bpm_propagate_batch.
// The runtime stages a copy from pageable memory through a copy kernel,
// which has to wait for compute units that a running persistent march
// holds; a copy from page-locked memory goes to the DMA engines.  A block
// returns to the pool from a host callback on the stream once its copy has
// run; blocks are kept until the process ends.
struct PinnedBlock {
  void* ptr;
  size_t cap;
};
std::mutex g_pinned_mu;
std::vector<PinnedBlock> g_pinned_free;

bool pinned_get(size_t bytes, PinnedBlock* out) {
  {
    std::lock_guard<std::mutex> lock(g_pinned_mu);
    size_t best = g_pinned_free.size();
    for (size_t i = 0; i < g_pinned_free.size(); ++i)
      if (g_pinned_free[i].cap >= bytes &&
          (best == g_pinned_free.size() || g_pinned_free[i].cap < g_pinned_free[best].cap))
        best = i;
    if (best < g_pinned_free.size()) {
      *out = g_pinned_free[best];
      g_pinned_free.erase(g_pinned_free.begin() + static_cast<long>(best));
      return true;
    }
  }
  const size_t cap = std::max<size_t>(size_t(1) << 20, (bytes + 0xFFFFF) & ~size_t(0xFFFFF));
  void* ptr = nullptr;
  if (hipHostMalloc(&ptr, cap, hipHostMallocDefault) != hipSuccess || !ptr) return false;
  *out = {ptr, cap};
  return true;
}

void pinned_put(const PinnedBlock& b) {
  std::lock_guard<std::mutex> lock(g_pinned_mu);
  g_pinned_free.push_back(b);
}

int batch_build(const bpm_job* jobs, int njobs, hipStream_t alloc_stream,
                bool stream_ordered, bpm_batch** out) {
  *out = nullptr;
  if (!jobs || njobs < 1) return fail(BPM_EINVAL, "jobs must be a non-empty array");
  for (int i = 0; i < njobs; ++i) {
    int rc = validate_job(jobs[i], i);
    if (rc) return rc;
  }
  // The batch carries a copy of every plan's constants in its own device
  // allocation, so a plan needs no device copy of its own (no per-plan
  // allocation or blocking upload at launch time), except for a general
  // crystal mask, which the plan uploads once.
  for (int i = 0; i < njobs; ++i) {
    bpm_plan* p = const_cast<bpm_plan*>(jobs[i].plan);
    int rc = p->mask.empty() ? bpm::plan_freeze_host(p) : freeze(p);
    if (rc) return fail(rc, "job " + std::to_string(i) + ": " + g_error);
  }
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");

  auto* b = new bpm_batch();
  std::map<std::tuple<int, int, int, int, bool>, std::vector<std::pair<int, int>>> by_variant;
  for (int i = 0; i < njobs; ++i) {
    const bpm_plan* p = jobs[i].plan;
    if (jobs[i].u_field)
      b->deforms.push_back({p->precision, p->Nx, p->Nz, p->h, jobs[i].u_field,
                            jobs[i].workspace});
    for (int w = 0; w < p->Nomega; ++w)
      by_variant[{p->precision, p->Nx, plan_schedule(p), p->split_order,
                  p->dev_mask != nullptr}].push_back({i, w});
  }
  // Host work lists: per variant, items ordered by group, longest first.
  struct HostGroup {
    int prec, Nx, sched, order;
    bool masked;
    int n_groups;
    std::vector<bpm::BatchItem> items;
    std::vector<int> offsets;
  };
  std::vector<HostGroup> host;
  std::vector<std::vector<const bpm_plan*>> item_plan;   // per group, per item
  for (auto& kv : by_variant) {
    const int prec = std::get<0>(kv.first), Nx = std::get<1>(kv.first);
    const int sched = std::get<2>(kv.first);
    const int order = std::get<3>(kv.first);
    const bool masked = std::get<4>(kv.first);
    auto& slices = kv.second;
    int per_cu = 0, threads = 0;
    int rc = bpm::march_occupancy(prec, Nx, sched, order, masked, &per_cu, &threads);
    if (rc) {
      delete b;
      return fail(rc, "occupancy query failed for Nx " + std::to_string(Nx));
    }
    const int resident = std::max(1, per_cu) * std::max(1, n_cu);
    const int G = std::min<int>(resident, static_cast<int>(slices.size()));
    // longest march first, then LPT: each slice to the least-loaded group
    std::stable_sort(slices.begin(), slices.end(), [&](auto& x, auto& y) {
      return jobs[x.first].plan->Nz > jobs[y.first].plan->Nz;
    });
    using Load = std::pair<long long, int>;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (int g = 0; g < G; ++g) heap.push({0, g});
    std::vector<std::vector<std::pair<int, int>>> per_group(G);
    for (auto& s : slices) {
      Load l = heap.top();
      heap.pop();
      per_group[l.second].push_back(s);
      l.first += jobs[s.first].plan->Nz;
      heap.push(l);
    }
    HostGroup hg{prec, Nx, sched, order, masked, G, {}, {0}};
    std::vector<const bpm_plan*> plans_of_items;
    for (int g = 0; g < G; ++g) {
      for (auto& s : per_group[g]) {
        const bpm_job& j = jobs[s.first];
        bpm::BatchItem it{};
        it.p = march_params(j.plan, j.E0_in, j.u_field ? j.workspace : nullptr,
                            j.E0_out, j.Eh_out);
        it.slice = s.second;
        hg.items.push_back(it);
        plans_of_items.push_back(j.plan);
      }
      hg.offsets.push_back(static_cast<int>(hg.items.size()));
    }
    host.push_back(std::move(hg));
    item_plan.push_back(std::move(plans_of_items));
  }
  // One device allocation: [items of every group][offsets of every group]
  // [constants of every distinct plan].
  size_t bytes = 0;
  std::vector<size_t> item_off, offs_off;
  for (auto& hg : host) {
    item_off.push_back(bytes);
    bytes += hg.items.size() * sizeof(bpm::BatchItem);
  }
  for (auto& hg : host) {
    bytes = (bytes + 255) & ~size_t(255);
    offs_off.push_back(bytes);
    bytes += hg.offsets.size() * sizeof(int);
  }
  std::map<const bpm_plan*, size_t> sc_off;
  for (int i = 0; i < njobs; ++i) {
    const bpm_plan* p = jobs[i].plan;
    if (sc_off.count(p)) continue;
    bytes = (bytes + 255) & ~size_t(255);
    sc_off[p] = bytes;
    bytes += sizeof(bpm::SliceConst) * size_t(p->Nomega);
  }
  e = stream_ordered ? hipMallocAsync(&b->d_mem, bytes, alloc_stream)
                     : hipMalloc(&b->d_mem, bytes);
  if (e != hipSuccess) {
    delete b;
    return fail(BPM_ENOMEM, std::string("batch work lists: ") + hipGetErrorString(e));
  }
  b->stream_ordered = stream_ordered;
  char* const dbase = static_cast<char*>(b->d_mem);
  // host image of the allocation: page-locked for the stream-ordered upload
  // when a block is available, otherwise ordinary memory
  PinnedBlock pin{nullptr, 0};
  const bool pinned = stream_ordered && pinned_get(bytes, &pin);
  std::vector<char>* staging = pinned ? nullptr : new std::vector<char>(bytes);
  char* const hbase = pinned ? static_cast<char*>(pin.ptr) : staging->data();
  for (const auto& kv : sc_off)
    std::memcpy(hbase + kv.second, kv.first->sc.data(),
                sizeof(bpm::SliceConst) * size_t(kv.first->Nomega));
  for (size_t g = 0; g < host.size(); ++g) {
    for (size_t k = 0; k < host[g].items.size(); ++k) {
      bpm::BatchItem& it = host[g].items[k];
      it.p.sc = reinterpret_cast<const bpm::SliceConst*>(dbase + sc_off.at(item_plan[g][k]));
    }
    std::memcpy(hbase + item_off[g], host[g].items.data(),
                host[g].items.size() * sizeof(bpm::BatchItem));
    std::memcpy(hbase + offs_off[g], host[g].offsets.data(),
                host[g].offsets.size() * sizeof(int));
    char* base = dbase;
    b->groups.push_back({host[g].prec, host[g].Nx, host[g].sched, host[g].order,
                         host[g].masked, host[g].n_groups,
                         static_cast<int>(host[g].items.size()),
                         reinterpret_cast<bpm::BatchItem*>(base + item_off[g]),
                         reinterpret_cast<int*>(base + offs_off[g])});
  }
  if (stream_ordered && pinned) {
    // The page-locked block returns to the pool once the copy ran.
    e = hipMemcpyAsync(b->d_mem, hbase, bytes, hipMemcpyHostToDevice, alloc_stream);
    if (e == hipSuccess) {
      e = hipLaunchHostFunc(
          alloc_stream,
          [](void* v) {
            auto* blk = static_cast<PinnedBlock*>(v);
            pinned_put(*blk);
            delete blk;
          },
          new PinnedBlock(pin));
    }
    // a failed enqueue leaks the block rather than risk reusing it while a
    // copy might still read it
  } else if (stream_ordered) {
    // The host staging buffer is released by the stream once the copy ran.
    e = hipMemcpyAsync(b->d_mem, staging->data(), bytes, hipMemcpyHostToDevice,
                       alloc_stream);
    if (e == hipSuccess)
      e = hipLaunchHostFunc(
          alloc_stream,
          [](void* v) { delete static_cast<std::vector<char>*>(v); }, staging);
    else
      delete staging;
  } else {
    e = hipMemcpy(b->d_mem, staging->data(), bytes, hipMemcpyHostToDevice);
    delete staging;
  }
  if (e != hipSuccess) {
    if (stream_ordered)
      (void)hipFreeAsync(b->d_mem, alloc_stream);
    else
      (void)hipFree(b->d_mem);
    delete b;
    return hip_fail(e, "batch work-list upload");
  }
  *out = b;
  return BPM_OK;
}

int batch_launch(const bpm_batch* b, hipStream_t s) {
  for (const auto& d : b->deforms) {
    int rc = bpm::launch_deform(d.prec, d.Nx, d.Nz, d.h, d.u, d.table, s);
    if (rc) return fail(rc, "deformation pre-pass launch failed");
  }
  for (const auto& g : b->groups) {
    int rc = bpm::launch_march_batch(g.prec, g.Nx, g.sched, g.order, g.masked, g.d_items,
                                     g.d_offsets, g.n_groups, s);
    if (rc) return fail(rc, "persistent march launch failed");
  }
  return BPM_OK;
}

}  // namespace

extern "C" {

bpm_plan* bpm_plan_create(int Nx, double dx, double dz, int Nz,
                          bpm_complex chi0, bpm_complex chih,
                          bpm_complex chihbar, double theta_B, double lambda,
                          int Nomega) {
  g_error.clear();
  if (!is_pow2(Nx) || Nx < 256 || Nx > 4096) {
    fail(BPM_EINVAL, "Nx must be a power of two in [256, 4096]");
    return nullptr;
  }
  if (Nz < 1 || Nomega < 1) {
    fail(BPM_EINVAL, "Nz and Nomega must be >= 1");
    return nullptr;
  }
  if (!(dx > 0) || !(dz > 0) || !(lambda > 0) || !std::isfinite(dx) ||
      !std::isfinite(dz) || !std::isfinite(lambda)) {
    fail(BPM_EINVAL, "dx, dz and lambda must be finite and > 0");
    return nullptr;
  }
  if (!(theta_B > 0) || !(theta_B < M_PI / 2)) {
    fail(BPM_EINVAL, "theta_B must lie in (0, pi/2)");
    return nullptr;
  }
  bpm_plan* p = new bpm_plan();
  p->Nx = Nx;
  p->Nz = Nz;
  p->Nomega = Nomega;
  p->dx = dx;
  p->dz = dz;
  p->chi0 = cplx(chi0.re, chi0.im);
  p->chih = cplx(chih.re, chih.im);
  p->chihbar = cplx(chihbar.re, chihbar.im);
  p->theta_B = theta_B;
  p->lambda = lambda;
  p->k0 = 2.0 * M_PI / lambda;
  p->h = 2.0 * p->k0 * std::sin(theta_B);
  default_detuning(p);
  return p;
}

bpm_plan* bpm_plan_create_3d(int Nx, int Ny, double dx, double dy, double dz, int Nz,
                             bpm_complex chi0, bpm_complex chih, bpm_complex chihbar,
                             double theta_B, double lambda, int Nomega) {
  g_error.clear();
  if (Nx < 2 || Nx > 8192) {
    fail(BPM_EINVAL, "Nx must lie in [2, 8192]");
    return nullptr;
  }
  if (Ny < 1 || Ny > 32) {
    fail(BPM_EINVAL, "Ny must lie in [1, 32]");
    return nullptr;
  }
  if (!(dy > 0) || !std::isfinite(dy)) {
    fail(BPM_EINVAL, "dy must be finite and > 0");
    return nullptr;
  }
  // the 2D validation of everything else, on a power-of-two stand-in for Nx
  bpm_plan* p = bpm_plan_create(256, dx, dz, Nz, chi0, chih, chihbar, theta_B, lambda,
                                Nomega);
  if (!p) return nullptr;
  p->Nx = Nx;
  p->Ny = Ny;
  p->dy = dy;
  p->three_d = true;
  p->bluestein = !(is_pow2(Nx) && Nx >= 64);
  p->L3 = bpm::row3_length(Nx);
  return p;
}

int bpm_plan_set_precision(bpm_plan* p, int precision) {
  int rc = check_mutable(p);
  if (rc) return rc;
  if (precision != BPM_PREC_FP64 && precision != BPM_PREC_FP32 &&
      precision != BPM_PREC_FP32S)
    return fail(BPM_EINVAL, "unknown precision");
  p->precision = precision;
  return BPM_OK;
}

int bpm_plan_set_crystal(bpm_plan* p, double x_front, double thickness) {
  int rc = check_mutable(p);
  if (rc) return rc;
  if (!std::isfinite(x_front) || !(thickness >= 0))
    return fail(BPM_EINVAL, "x_front must be finite and thickness >= 0");
  p->x_front = x_front;
  p->thickness = thickness;
  return BPM_OK;
}

int bpm_plan_set_detuning(bpm_plan* p, const double* delta) {
  int rc = check_mutable(p);
  if (rc) return rc;
  if (!delta) return fail(BPM_EINVAL, "delta is NULL");
  for (int j = 0; j < p->Nomega; ++j)
    if (!std::isfinite(delta[j]) || !(delta[j] > -1.0))
      return fail(BPM_EINVAL, "delta must be finite and > -1");
  p->delta.assign(delta, delta + p->Nomega);
  return BPM_OK;
}

int bpm_plan_set_mask(bpm_plan* p, const unsigned char* mask) {
  int rc = check_mutable(p);
  if (rc) return rc;
  if (!mask) {
    p->mask.clear();
    return BPM_OK;
  }
  const size_t n = size_t(p->Nx) * size_t(p->Nz) * size_t(p->three_d ? p->Ny : 1);
  p->mask.resize(n);
  for (size_t i = 0; i < n; ++i) p->mask[i] = mask[i] ? 1 : 0;
  return BPM_OK;
}

int bpm_plan_set_time_grid(bpm_plan* p, double dt) {
  int rc = check_mutable(p);
  if (rc) return rc;
  if (!std::isfinite(dt) || !(dt > 0.0)) return fail(BPM_EINVAL, "dt must be finite and > 0");
  const int N = p->Nomega;
  if (!is_pow2(N) || N < 256 || N > 4096)
    return fail(BPM_EINVAL, "a pulse grid needs Nomega a power of two in [256, 4096]");
  // delta_j = Omega_j / omega_0, Omega_j = (j - N/2) 2 pi / (N dt),
  // omega_0 = 2 pi c / lambda (Section 3, Eq. tdp)
  const double c_light = 299792458.0;
  const double two_pi = 2.0 * 3.14159265358979323846;
  const double dOmega = two_pi / (N * dt);
  const double omega0 = two_pi * c_light / p->lambda;
  std::vector<double> d(N);
  for (int j = 0; j < N; ++j) {
    d[j] = double(j - N / 2) * dOmega / omega0;
    if (!(d[j] > -1.0)) return fail(BPM_EINVAL, "dt too small: a slice has k <= 0");
  }
  p->delta = d;
  p->dt = dt;
  return BPM_OK;
}

int bpm_plan_set_options(bpm_plan* p, int split_order, int zassenhaus) {
  int rc = check_mutable(p);
  if (rc) return rc;
  if (split_order != 1 && split_order != 2 && split_order != 4)
    return fail(BPM_EINVAL, "split_order must be 1, 2 or 4");
  if (zassenhaus != 0 && zassenhaus != 1)
    return fail(BPM_EINVAL, "zassenhaus must be 0 or 1");
  p->split_order = split_order;
  p->zassenhaus = zassenhaus;
  return BPM_OK;
}

int bpm_plan_set_schedule(bpm_plan* p, int schedule) {
  int rc = check_mutable(p);
  if (rc) return rc;
  if (schedule != BPM_SCHED_AUTO && schedule != BPM_SCHED_STOCKHAM &&
      schedule != BPM_SCHED_FOURSTEP && schedule != BPM_SCHED_SPLIT)
    return fail(BPM_EINVAL, "unknown schedule");
  if (schedule != BPM_SCHED_AUTO && p->three_d) return reject_3d(p, "a transform schedule");
  p->schedule = schedule;
  return BPM_OK;
}

int bpm_plan_get_schedule(const bpm_plan* p) {
  if (!p) return fail(BPM_EINVAL, "plan is NULL");
  return plan_schedule(p);
}

int bpm_plan_get_constants(const bpm_plan* cp, int w, double* out) {
  g_error.clear();
  if (!cp || !out) return fail(BPM_EINVAL, "plan and out must be non-NULL");
  if (w < 0 || w >= cp->Nomega) return fail(BPM_EINVAL, "slice index out of range");
  bpm_plan tmp;
  tmp.Nx = cp->Nx; tmp.Nz = cp->Nz; tmp.Nomega = cp->Nomega;
  tmp.dx = cp->dx; tmp.dz = cp->dz;
  tmp.chi0 = cp->chi0; tmp.chih = cp->chih; tmp.chihbar = cp->chihbar;
  tmp.theta_B = cp->theta_B; tmp.lambda = cp->lambda;
  tmp.split_order = cp->split_order; tmp.zassenhaus = cp->zassenhaus;
  tmp.delta = cp->delta; tmp.k0 = cp->k0; tmp.h = cp->h;
  int rc = compute_slice_constants(&tmp);
  if (rc) return rc;
  const bpm::SliceConst& s = tmp.sc[w];
  const double sh = 0.5 * tmp.h / s.k;
  out[0] = s.k;
  out[1] = std::sqrt(1.0 - sh * sh);
  for (int i = 0; i < 6; ++i) out[2 + i] = s.d[0][i];
  return BPM_OK;
}

size_t bpm_workspace_bytes(const bpm_plan* p) {
  if (!p) return 0;
  const size_t cell = p->precision == BPM_PREC_FP64 ? 16 : 8;
  if (p->three_d) return size_t(p->Nx) * size_t(p->Ny) * size_t(p->Nz) * cell;
  return size_t(p->Nx) * size_t(p->Nz) * cell;
}

static int pulse_transform(const bpm_plan* p, const void* in, void* out, void* stream,
                           bool to_freq) {
  g_error.clear();
  if (!p) return fail(BPM_EINVAL, "plan is NULL");
  if (!in || !out) return fail(BPM_EINVAL, "input and output must be non-NULL");
  if (!(p->dt > 0.0)) return fail(BPM_EINVAL, "the plan has no time grid (bpm_plan_set_time_grid)");
  // every (y, x) sample is a column of the slice axis
  const int cols = p->Nx * p->Ny;
  if (cols % 2) return fail(BPM_EINVAL, "the pulse transform needs an even Ny * Nx");
  int rc = bpm::launch_pulse(p->precision, p->Nomega, cols, to_freq, p->dt, in, out,
                             static_cast<hipStream_t>(stream));
  if (rc) return fail(rc, "pulse transform launch failed");
  return BPM_OK;
}

int bpm_time_to_frequency(const bpm_plan* plan, const void* field_t, void* field_w,
                          void* stream) {
  return pulse_transform(plan, field_t, field_w, stream, true);
}

int bpm_frequency_to_time(const bpm_plan* plan, const void* field_w, void* field_t,
                          void* stream) {
  return pulse_transform(plan, field_w, field_t, stream, false);
}

int bpm_deformation_table(const bpm_plan* cp, const double* u_field,
                          void* workspace, void* stream) {
  g_error.clear();
  if (!cp) return fail(BPM_EINVAL, "plan is NULL");
  if (!u_field || !workspace)
    return fail(BPM_EINVAL, "u_field and workspace must be non-NULL");
  bpm_plan* p = const_cast<bpm_plan*>(cp);
  int rc = freeze(p);
  if (rc) return rc;
  // a 3D plan's cells are its (y, x) samples
  rc = bpm::launch_deform(p->precision, p->three_d ? p->Nx * p->Ny : p->Nx, p->Nz, p->h,
                          u_field, workspace, static_cast<hipStream_t>(stream));
  if (rc) return fail(rc, "deformation pre-pass launch failed");
  return BPM_OK;
}

int bpm_march(const bpm_plan* cp, const void* E0_in, const void* table,
              void* E0_out, void* Eh_out, void* stream) {
  g_error.clear();
  if (!cp) return fail(BPM_EINVAL, "plan is NULL");
  if (!E0_in || !E0_out || !Eh_out)
    return fail(BPM_EINVAL, "E0_in, E0_out and Eh_out must be non-NULL");
  if (E0_in == E0_out || E0_in == Eh_out || E0_out == Eh_out)
    return fail(BPM_EINVAL, "output buffers must not alias each other or E0_in");
  bpm_plan* p = const_cast<bpm_plan*>(cp);
  if (p->three_d)
    return march3(p, E0_in, nullptr, table, 0, p->Nz, E0_out, Eh_out,
                  static_cast<hipStream_t>(stream));
  int rc = freeze(p);
  if (rc) return rc;
  const bpm::MarchParams m = march_params(p, E0_in, table, E0_out, Eh_out);
  rc = bpm::launch_march(p->precision, p->Nx, plan_schedule(p), p->split_order, p->Nomega, m,
                         static_cast<hipStream_t>(stream));
  if (rc == BPM_EUNSUPPORTED) return fail(rc, "unsupported size/precision");
  if (rc) return fail(rc, "march kernel launch failed");
  return BPM_OK;
}

int bpm_march_segment(const bpm_plan* cp, const void* E0_in, const void* Eh_in,
                      const void* table, int n0, int nsteps, void* E0_out,
                      void* Eh_out, void* stream) {
  g_error.clear();
  if (!cp) return fail(BPM_EINVAL, "plan is NULL");
  if (!E0_in || !E0_out || !Eh_out)
    return fail(BPM_EINVAL, "E0_in, E0_out and Eh_out must be non-NULL");
  if (E0_out == Eh_out || (Eh_in && (E0_out == Eh_in || Eh_out == E0_in)))
    return fail(BPM_EINVAL, "outputs must not alias each other or the other envelope's input");
  if (n0 < 0 || nsteps < 1 || n0 > cp->Nz - nsteps)
    return fail(BPM_EINVAL, "steps [n0, n0 + nsteps) must lie in [0, Nz)");
  bpm_plan* p = const_cast<bpm_plan*>(cp);
  if (p->three_d)
    return march3(p, E0_in, Eh_in, table, n0, nsteps, E0_out, Eh_out,
                  static_cast<hipStream_t>(stream));
  int rc = freeze(p);
  if (rc) return rc;
  bpm::MarchParams m = march_params(p, E0_in, table, E0_out, Eh_out);
  m.Eh_in = Eh_in;
  m.n0 = n0;
  m.Nz = nsteps;
  rc = bpm::launch_march(p->precision, p->Nx, plan_schedule(p), p->split_order, p->Nomega, m,
                         static_cast<hipStream_t>(stream));
  if (rc == BPM_EUNSUPPORTED) return fail(rc, "unsupported size/precision");
  if (rc) return fail(rc, "march kernel launch failed");
  return BPM_OK;
}

int bpm_propagate_ws(const bpm_plan* cp, const void* E0_in,
                     const double* u_field, void* E0_out, void* Eh_out,
                     void* workspace, void* stream) {
  g_error.clear();
  if (!cp) return fail(BPM_EINVAL, "plan is NULL");
  if (!E0_in || !E0_out || !Eh_out)
    return fail(BPM_EINVAL, "E0_in, E0_out and Eh_out must be non-NULL");
  if (E0_in == E0_out || E0_in == Eh_out || E0_out == Eh_out)
    return fail(BPM_EINVAL, "output buffers must not alias each other or E0_in");
  if (cp->three_d) {
    if (u_field && !workspace) return fail(BPM_EINVAL, "a deformed propagate needs a workspace");
    return propagate3(const_cast<bpm_plan*>(cp), E0_in, u_field, E0_out, Eh_out, workspace,
                      static_cast<hipStream_t>(stream));
  }
  if (u_field && !workspace)
    return fail(BPM_EINVAL, "a deformed propagate needs a workspace");
  if (u_field) {
    int rc = bpm_deformation_table(cp, u_field, workspace, stream);
    if (rc) return rc;
  }
  return bpm_march(cp, E0_in, u_field ? workspace : nullptr, E0_out, Eh_out,
                   stream);
}

int bpm_propagate(const bpm_plan* p, const void* E0_in, const double* u_field,
                  void* E0_out, void* Eh_out, void* stream) {
  g_error.clear();
  if (!p) return fail(BPM_EINVAL, "plan is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* ws = nullptr;
  if (u_field) {
    hipError_t e = hipMallocAsync(&ws, bpm_workspace_bytes(p), s);
    if (e != hipSuccess)
      return fail(BPM_ENOMEM, std::string("hipMallocAsync(workspace): ") +
                                  hipGetErrorString(e));
  }
  int rc = bpm_propagate_ws(p, E0_in, u_field, E0_out, Eh_out, ws, stream);
  if (ws) {
    hipError_t e = hipFreeAsync(ws, s);
    if (rc == BPM_OK && e != hipSuccess) return hip_fail(e, "hipFreeAsync");
  }
  return rc;
}

bpm_batch* bpm_batch_create(const bpm_job* jobs, int njobs) {
  g_error.clear();
  bpm_batch* b = nullptr;
  batch_build(jobs, njobs, nullptr, false, &b);
  return b;
}

int bpm_batch_launch(const bpm_batch* b, void* stream) {
  g_error.clear();
  if (!b) return fail(BPM_EINVAL, "batch is NULL");
  return batch_launch(b, static_cast<hipStream_t>(stream));
}

int bpm_batch_info(const bpm_batch* b, int* n_launches, int* n_slices,
                   int* n_workgroups) {
  g_error.clear();
  if (!b) return fail(BPM_EINVAL, "batch is NULL");
  int items = 0, wgs = 0;
  for (const auto& g : b->groups) {
    items += g.n_items;
    wgs += g.n_groups;
  }
  if (n_launches) *n_launches = static_cast<int>(b->groups.size());
  if (n_slices) *n_slices = items;
  if (n_workgroups) *n_workgroups = wgs;
  return BPM_OK;
}

void bpm_batch_destroy(bpm_batch* b) {
  if (!b) return;
  if (b->d_mem) (void)hipFree(b->d_mem);
  delete b;
}

int bpm_propagate_batch(const bpm_job* jobs, int njobs, void* stream) {
  g_error.clear();
  hipStream_t s = static_cast<hipStream_t>(stream);
  // The work lists are staged from host memory that a host callback
  // releases after the copy: a graph replay would copy from freed memory.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t ce = hipStreamIsCapturing(s, &cap);
  if (ce != hipSuccess) return hip_fail(ce, "hipStreamIsCapturing");
  if (cap != hipStreamCaptureStatusNone)
    return fail(BPM_EINVAL,
                "bpm_propagate_batch cannot be captured in a graph; capture "
                "bpm_batch_launch of a bpm_batch_create batch instead");
  bpm_batch* b = nullptr;
  int rc = batch_build(jobs, njobs, s, true, &b);
  if (rc) return rc;
  rc = batch_launch(b, s);
  hipError_t e = hipFreeAsync(b->d_mem, s);
  b->d_mem = nullptr;
  delete b;
  if (rc == BPM_OK && e != hipSuccess) return hip_fail(e, "hipFreeAsync(batch)");
  return rc;
}

void bpm_plan_destroy(bpm_plan* p) {
  if (!p) return;
  if (p->dev_tables3) (void)hipFree(p->dev_tables3);
  if (p->dev_rows3) (void)hipFree(p->dev_rows3);
  if (p->dev_sc) (void)hipFree(p->dev_sc);
  if (p->dev_mask) (void)hipFree(p->dev_mask);
  delete p;
}

const char* bpm_last_error(void) { return g_error.c_str(); }

}  // extern "C"

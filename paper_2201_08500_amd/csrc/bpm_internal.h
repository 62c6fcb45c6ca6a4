// Internal declarations shared by the host plan (bpm_host.cpp) and the
// gfx950 kernels (bpm_device.h, bpm_march.hip, march_*.hip).  Not part of
// the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bpm.h"

namespace bpm {

// Per-slice constants, computed on the host in FP64 and read by the march
// kernel.  k: wavenumber of the slice; d0, dp1, dm1: coupling constants of
// one B sub-step (Eq. fov10 with the Zassenhaus factor); up to 4 sub-steps.
struct SliceConst {
  double k;
  double pad;
  double d[4][6];   // per sub-step: d0.re, d0.im, dp1.re, dp1.im, dm1.re, dm1.im
};

// Scalars of one launch of the march over a contiguous range of slices.
struct MarchParams {
  const void* E0_in;        // [Nomega][Nx] complex (ST precision)
  const void* Eh_in;        // psi~_- at the first step, or nullptr (zero)
  void* E0_out;
  void* Eh_out;
  const void* table;        // [Nz][Nx] exp(i h u), or nullptr (u == 0)
  const SliceConst* sc;     // [Nomega]
  int Nz;                   // steps marched by this launch
  int n0;                   // index of the first step (table row offset)
  int nsub;                 // B sub-steps per step (1, 2 or 4)
  double dx, dz;
  double h_half;            // h / 2
  double x_front, x_end;    // slab [x_front, x_end)
  double a_frac[4];         // A sub-step fractions (0 = skip)
  const unsigned char* mask;  // [Nz][Nx] crystal mask (nonzero = crystal), or
                              // nullptr: the slab [x_front, x_end)
};

// One unit of batched work: one slice of one problem.
struct BatchItem {
  MarchParams p;
  int slice;
  int pad[3];
};

int launch_deform(int prec, int Nx, int Nz, double h, const double* u,
                  void* table, hipStream_t stream);
// sched: transform schedule (0 Stockham, 1 four-step, 2 envelope-split);
// order: splitting order 1, 2 or 4 (sub-steps of Eq. split-op); p.mask
// selects the general-mask kernels.
int launch_march(int prec, int Nx, int sched, int order, int Nomega,
                 const MarchParams& p, hipStream_t stream);
// Persistent launch: n_groups work groups, group g runs
// items[offsets[g] .. offsets[g+1]) (device arrays); masked: every item has
// a general mask (else none has).
int launch_march_batch(int prec, int Nx, int sched, int order, bool masked,
                       const BatchItem* items, const int* offsets, int n_groups,
                       hipStream_t stream);
// Resident work groups per CU and threads per group of a march variant.
int march_occupancy(int prec, int Nx, int sched, int order, bool masked,
                    int* wg_per_cu, int* threads);
// Kernel units, one per (precision, masked): march_<precision>[_mask].hip.
template <int PREC, bool MASKED>
int launch_march_p(int Nx, int sched, int order, int Nomega, const MarchParams& p,
                   hipStream_t stream);
template <int PREC, bool MASKED>
int launch_march_batch_p(int Nx, int sched, int order, const BatchItem* items,
                         const int* offsets, int n_groups, hipStream_t stream);
template <int PREC, bool MASKED>
int march_occupancy_p(int Nx, int sched, int order, int* wg_per_cu, int* threads);
template <int PREC>
int launch_pulse_p(int N, int Nx, bool to_freq, double dt, const void* in, void* out,
                   hipStream_t stream);
// Time <-> frequency transform of [N][Nx] pulse fields along the slice axis.
int launch_pulse(int prec, int N, int Nx, bool to_freq, double dt, const void* in,
                 void* out, hipStream_t stream);
// Library default schedule of (precision, Nx).
int default_schedule(int prec, int Nx);

// One march on a 3D grid (bpm3d.hip): the state lives in E0_out / Eh_out
// ([Nomega][Ny][Nx]); P is the propagator table workspace
// ([Nomega][2][Ny][Nx] complex FP64); chirp [Nx], G [L], tw [L] and
// wy [Ny] are the plan's FP64 tables (complex, interleaved).
struct March3Params {
  int prec, Nx, Ny, Nz, Nomega, L;  // Nz: steps of this launch sequence
  int n0;                   // index of its first step (deformation row)
  double dx, x_front, x_end;
  const void* E0_in;
  const void* Eh_in;        // nullptr: psi~_- starts at zero
  void* E0_out;
  void* Eh_out;
  const void* table;        // [Nz][Ny][Nx] exp(i h u), or nullptr
  const void* mask;         // [Nz][Ny][Nx] crystal mask (device), or nullptr: the slab
  const SliceConst* sc;
  const void* rows;         // per table set [Nomega][2][Ny / 2 + 1][L] row propagator (FP64)
  size_t set_elems;         // complex entries per table set
  int nsub;                 // sub-steps of Eq. split-op per step (1, 2, 4)
  int a_set[4];             // table set of sub-step i's A (-1: no A)
  const void* tw;           // [L] exp(-2 pi i m / L)
  const void* wy;           // [Ny] exp(-2 pi i j / Ny)
};
// The FP64 propagator exp(i frac dz kz(K_x, K_y)) / (Nx Ny) of every (slice,
// envelope, |K_y|, K_x): Nomega x 2 x (Ny / 2 + 1) rows of length Nx, into P
// (device).
int launch_prop3(void* P, const SliceConst* sc, int Nx, int Ny, int Nomega, double dx,
                 double dy, double dz, double frac, double h_half, hipStream_t stream);
int launch_march3(const March3Params& q, hipStream_t stream);
// Row lengths from which the 3D row kernel uses the four-step layout
// (W = L / 1024 wavefronts, 1024-point in-wavefront transforms), and the
// lengths 9 M (M = 512, 1024) with W = 9 wavefronts of M-point transforms:
// their row tables are stored with entry i T + t holding bin w + W (l + 64 i)
// of thread t = 64 w + l, T = 64 W, i < L / T.
constexpr int kRow3FourStepMin = 8192;
constexpr bool row3_four_step(int L) { return L >= kRow3FourStepMin || L % 9 == 0; }
constexpr int row3_waves(int L) { return L % 9 == 0 ? 9 : L / 1024; }
// Whether a row of length L fits in LDS in the plan's storage type (FP64
// rows of 16384 samples do not).
constexpr bool row3_fits(int prec, int L) { return prec != BPM_PREC_FP64 || L <= 9216; }
// The row transform length for Nx samples: Nx for powers of two >= 64;
// otherwise the smallest length >= 2 Nx - 1 among the powers of two >= 64
// and 4608, 9216 (which save 44% of the padded work where they apply:
// 2048 < Nx <= 2304 and 4096 < Nx <= 4608).
inline int row3_length(int Nx) {
  if (Nx >= 64 && (Nx & (Nx - 1)) == 0) return Nx;
  int L = 64;
  while (L < 2 * Nx - 1) L <<= 1;
  for (int c : {4608, 9216})
    if (2 * Nx - 1 <= c && c < L) return c;
  return L;
}

}  // namespace bpm

struct bpm_plan;

namespace bpm {
// Host-side plan helpers (bpm_host.cpp) shared with the static-workspace
// entry point (bpm_static.hip).
int set_error(int code, const std::string& msg);   // records msg, returns code
void clear_error();
// Computes the plan's FP64 constants (host only, no device call) and freezes
// its setters; idempotent.
int plan_freeze_host(bpm_plan* p);
int plan_schedule_of(const bpm_plan* p);
MarchParams plan_march_params(const bpm_plan* p, const void* E0_in, const void* table,
                              void* E0_out, void* Eh_out);
}  // namespace bpm

struct bpm_plan {
  int Nx = 0, Nz = 0, Nomega = 0;
  double dx = 0, dz = 0;
  std::complex<double> chi0, chih, chihbar;
  double theta_B = 0, lambda = 0;
  int precision = BPM_PREC_FP64;
  double x_front = 0.0, thickness = HUGE_VAL;
  int split_order = 1, zassenhaus = 1;
  int schedule = -1;  // BPM_SCHED_AUTO
  double dt = 0.0;     // time step of the pulse grid (0: none set)
  std::vector<unsigned char> mask;       // general crystal mask (empty: slab)
  unsigned char* dev_mask = nullptr;
  std::vector<double> delta;
  // derived (FP64)
  double k0 = 0, h = 0;
  std::vector<bpm::SliceConst> sc;
  bpm::SliceConst* dev_sc = nullptr;    // uploaded constants (nullptr until then)
  // 3D grid (bpm_plan_create_3d): Ny rows of dy along y, any Nx; the x
  // transform has length L (Bluestein when Nx is not a power of two >= 64)
  bool three_d = false;
  int Ny = 1;
  double dy = 0.0;
  int L3 = 0;
  bool bluestein = false;
  void* dev_tables3 = nullptr;          // tw [L], wy [Ny]
  void* dev_rows3 = nullptr;            // per A length [Nomega][2][Ny / 2 + 1][L] row propagator
  int device = -1;
  bool frozen = false;                   // constants computed, setters closed
  std::mutex mu;
};

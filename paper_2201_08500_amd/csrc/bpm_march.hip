// Host-side dispatch of the z-march kernels (one kernel unit per precision,
// march_fp64.hip / march_fp32.hip / march_fp32s.hip) and the deformation
// pre-pass exp(i h u) of Eq. Authier.

#include "bpm_device.h"

namespace bpm {

#define BPM_EXTERN_PREC(P, M)                                                      \
  extern template int launch_march_p<P, M>(int, int, int, int, const MarchParams&, \
                                           hipStream_t);                           \
  extern template int launch_march_batch_p<P, M>(int, int, int, const BatchItem*,  \
                                                 const int*, int, hipStream_t);    \
  extern template int march_occupancy_p<P, M>(int, int, int, int*, int*);
BPM_EXTERN_PREC(BPM_PREC_FP64, false)
BPM_EXTERN_PREC(BPM_PREC_FP32, false)
BPM_EXTERN_PREC(BPM_PREC_FP32S, false)
BPM_EXTERN_PREC(BPM_PREC_FP64, true)
BPM_EXTERN_PREC(BPM_PREC_FP32, true)
BPM_EXTERN_PREC(BPM_PREC_FP32S, true)
#undef BPM_EXTERN_PREC
extern template int launch_pulse_p<BPM_PREC_FP64>(int, int, bool, double, const void*, void*,
                                                  hipStream_t);
extern template int launch_pulse_p<BPM_PREC_FP32>(int, int, bool, double, const void*, void*,
                                                  hipStream_t);
extern template int launch_pulse_p<BPM_PREC_FP32S>(int, int, bool, double, const void*,
                                                   void*, hipStream_t);

namespace {
// f(std::integral_constant<int, PREC>, std::bool_constant<MASKED>) for the
// runtime (prec, masked)
template <class F>
int with_prec_mask(int prec, bool masked, F&& f) {
  using I = std::integral_constant<int, BPM_PREC_FP64>;
  using S = std::integral_constant<int, BPM_PREC_FP32>;
  using SS = std::integral_constant<int, BPM_PREC_FP32S>;
  switch (prec) {
    case BPM_PREC_FP64:
      return masked ? f(I{}, std::true_type{}) : f(I{}, std::false_type{});
    case BPM_PREC_FP32:
      return masked ? f(S{}, std::true_type{}) : f(S{}, std::false_type{});
    case BPM_PREC_FP32S:
      return masked ? f(SS{}, std::true_type{}) : f(SS{}, std::false_type{});
    default: return BPM_EUNSUPPORTED;
  }
}
}  // namespace

int launch_march(int prec, int Nx, int sched, int order, int Nomega,
                 const MarchParams& p, hipStream_t stream) {
  return with_prec_mask(prec, p.mask != nullptr, [&](auto P, auto M) {
    return launch_march_p<decltype(P)::value, decltype(M)::value>(Nx, sched, order, Nomega,
                                                                  p, stream);
  });
}

int launch_march_batch(int prec, int Nx, int sched, int order, bool masked,
                       const BatchItem* items, const int* offsets, int n_groups,
                       hipStream_t stream) {
  return with_prec_mask(prec, masked, [&](auto P, auto M) {
    return launch_march_batch_p<decltype(P)::value, decltype(M)::value>(
        Nx, sched, order, items, offsets, n_groups, stream);
  });
}

int march_occupancy(int prec, int Nx, int sched, int order, bool masked, int* wg_per_cu,
                    int* threads) {
  return with_prec_mask(prec, masked, [&](auto P, auto M) {
    return march_occupancy_p<decltype(P)::value, decltype(M)::value>(Nx, sched, order,
                                                                     wg_per_cu, threads);
  });
}

int launch_pulse(int prec, int N, int Nx, bool to_freq, double dt, const void* in,
                 void* out, hipStream_t stream) {
  switch (prec) {
    case BPM_PREC_FP64: return launch_pulse_p<BPM_PREC_FP64>(N, Nx, to_freq, dt, in, out, stream);
    case BPM_PREC_FP32: return launch_pulse_p<BPM_PREC_FP32>(N, Nx, to_freq, dt, in, out, stream);
    case BPM_PREC_FP32S: return launch_pulse_p<BPM_PREC_FP32S>(N, Nx, to_freq, dt, in, out, stream);
    default: return BPM_EUNSUPPORTED;
  }
}

// Fastest schedule per (precision, Nx), measured on MI355X (march of >= 256
// slices); 0 Stockham, 1 four-step, 2 envelope-split four-step.
int default_schedule(int prec, int Nx) {
  const int col = Nx == 256 ? 0 : Nx == 512 ? 1 : Nx == 1024 ? 2 : Nx == 2048 ? 3 : 4;
  // (at Nx 4096 the four-step: 8% faster than the envelope split with a
  // 1024-point in-wavefront transform in fp32s, 5% in fp32; for fp64 the
  // split does not fit in LDS and its schedule 2 is the four-step)
  static const int kBest[3][5] = {
      /* fp64  */ {2, 2, 2, 2, 1},
      /* fp32  */ {2, 2, 2, 2, 1},
      /* fp32s */ {2, 2, 2, 2, 1},
  };
  const int row = prec == BPM_PREC_FP64 ? 0 : prec == BPM_PREC_FP32 ? 1 : 2;
  return kBest[row][col];
}

int launch_deform(int prec, int Nx, int Nz, double h, const double* u,
                  void* table, hipStream_t stream) {
  const size_t n = size_t(Nx) * size_t(Nz);
  const int block = 256;
  const size_t want = (n + block - 1) / block;
  const int grid = static_cast<int>(want < 8192 ? want : 8192);
  if (prec == BPM_PREC_FP64)
    hipLaunchKernelGGL(deform_kernel<double>, dim3(grid), dim3(block), 0,
                       stream, u, n, h, static_cast<double2*>(table));
  else
    hipLaunchKernelGGL(deform_kernel<float>, dim3(grid), dim3(block), 0,
                       stream, u, n, h, static_cast<float2*>(table));
  return hipGetLastError() == hipSuccess ? BPM_OK : BPM_EHIP;
}

}  // namespace bpm

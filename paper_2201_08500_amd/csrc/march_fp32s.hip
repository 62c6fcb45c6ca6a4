// z-march kernels of one precision (fp32s, slab crystal): every
// transform schedule, Nx and splitting order, instantiated here so that the
// kernel units compile in parallel (the lengths listed below in their own
// unit).

#include "bpm_device.h"

namespace bpm {

// transform lengths compiled in march_fp32s_ilp.hip
BPM_MARCH_N(extern, BPM_PREC_FP32S, false, 256)
BPM_MARCH_N(extern, BPM_PREC_FP32S, false, 512)
BPM_MARCH_N(extern, BPM_PREC_FP32S, false, 2048)

template int launch_march_p<BPM_PREC_FP32S, false>(int, int, int, int, const MarchParams&,
                                        hipStream_t);
template int launch_march_batch_p<BPM_PREC_FP32S, false>(int, int, int, const BatchItem*, const int*,
                                              int, hipStream_t);
template int march_occupancy_p<BPM_PREC_FP32S, false>(int, int, int, int*, int*);
template int launch_pulse_p<BPM_PREC_FP32S>(int, int, bool, double, const void*, void*, hipStream_t);

}  // namespace bpm

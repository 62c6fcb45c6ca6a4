// z-march kernels of one precision (fp32, general-mask crystal): every
// transform schedule, Nx and splitting order, instantiated here so that the
// kernel units compile in parallel (the lengths listed below in their own
// unit).

#include "bpm_device.h"

namespace bpm {

// transform lengths compiled in march_fp32_mask_ilp.hip
BPM_MARCH_N(extern, BPM_PREC_FP32, true, 1024)
BPM_MARCH_N(extern, BPM_PREC_FP32, true, 2048)

template int launch_march_p<BPM_PREC_FP32, true>(int, int, int, int, const MarchParams&,
                                        hipStream_t);
template int launch_march_batch_p<BPM_PREC_FP32, true>(int, int, int, const BatchItem*, const int*,
                                              int, hipStream_t);
template int march_occupancy_p<BPM_PREC_FP32, true>(int, int, int, int*, int*);

}  // namespace bpm

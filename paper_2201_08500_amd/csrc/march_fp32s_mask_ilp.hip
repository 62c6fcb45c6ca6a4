// z-march kernels of one precision (fp32s, general-mask crystal) for the transform
// lengths 256, 512, 2048: a unit of their own, compiled with the
// instruction-level-parallelism scheduling strategy, which measured faster
// for these lengths (and slower for the others).

#include "bpm_device.h"

namespace bpm {

BPM_MARCH_N(, BPM_PREC_FP32S, true, 256)
BPM_MARCH_N(, BPM_PREC_FP32S, true, 512)
BPM_MARCH_N(, BPM_PREC_FP32S, true, 2048)

}  // namespace bpm

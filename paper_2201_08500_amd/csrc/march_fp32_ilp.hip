// z-march kernels of one precision (fp32, slab crystal) for the transform
// lengths 1024, 2048: a unit of their own, compiled with the
// instruction-level-parallelism scheduling strategy, which measured faster
// for these lengths (and slower for the others).

#include "bpm_device.h"

namespace bpm {

BPM_MARCH_N(, BPM_PREC_FP32, false, 1024)
BPM_MARCH_N(, BPM_PREC_FP32, false, 2048)

}  // namespace bpm

// Internal interface of the surrogate per-ray kernels (surrogate.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace gr {
namespace sur {

// Network inputs (n x 7) and straight-line escape directions (n x 3) of the
// rays of an uploaded batch table.
hipError_t inputs(const BatchInstance* inst, const int64_t* firsts, int ninst, int64_t total,
                  float* x, float* uflat, hipStream_t s);
// Targets (n x 4: escaped, correction d) from the traced outputs of the table.
hipError_t targets(const BatchInstance* inst, const int64_t* firsts, int ninst, int64_t total,
                   const float* uflat, float* target, hipStream_t s);
// Frame pipeline.
hipError_t classify(const float* y, const float* uflat, int64_t n, int8_t* flag, float* dir,
                    hipStream_t s);
hipError_t fallback(const float* y, const int8_t* flag, int32_t W, int32_t H, float logit_min,
                    int32_t edge, int8_t* fb, int32_t* list, unsigned long long* count,
                    hipStream_t s);
hipError_t merge(const BatchInstance* inst, const int32_t* list, int64_t n, int8_t* flag,
                 float* dir, hipStream_t s);

}  // namespace sur
}  // namespace gr

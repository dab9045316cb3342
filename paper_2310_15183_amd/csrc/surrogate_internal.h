// Internal interface of the surrogate per-ray kernels (surrogate.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "mlp_internal.h"

namespace gr {
namespace sur {

// Network inputs (n x 7) and straight-line escape directions (n x 3) of the
// rays of an uploaded batch table.
hipError_t inputs(const BatchInstance* inst, const int64_t* firsts, int ninst, int64_t total,
                  float* x, float* uflat, hipStream_t s);
// Targets (n x 4: escaped, correction d) from the traced outputs of the table.
hipError_t targets(const BatchInstance* inst, const int64_t* firsts, int ninst, int64_t total,
                   const float* uflat, float* target, hipStream_t s);
// Frame pipeline.  frame_net: inputs, network, class and end direction of
// every pixel of one frame (I.pixels is ignored: pixel k is ray k) in one
// launch, keeping each escape logit for the fallback selection (NaN for an
// escaping ray whose impact parameter is below min_impact times the critical
// one, which the selection always re-traces).
hipError_t frame_net(const BatchInstance& I, int64_t npix, const mlp::NetView& net,
                     float min_impact, int8_t* flag, float* dir, float* logit, hipStream_t s);
hipError_t fallback(const float* logit, const int8_t* flag, const float* dir, int32_t W,
                    int32_t H, float logit_min, int32_t edge, float max_chord2, int8_t* fb,
                    int32_t* list, unsigned long long* count, hipStream_t s);
// firsts[0] = 0, firsts[1] = *count (one-instance batch of the fallback list).
hipError_t set_firsts(const unsigned long long* count, int64_t* firsts, hipStream_t s);
// Traced flag and escape-sphere direction of the *count listed pixels
// (count <= max_n) over the network's.
hipError_t merge(const BatchInstance* inst, const int32_t* list, const unsigned long long* count,
                 int64_t max_n, int8_t* flag, float* dir, hipStream_t s);

}  // namespace sur
}  // namespace gr

// forward16.hip -- the feature map with 16-bit storage of x and/or phi
// (bfloat16 or IEEE half), FP32 arithmetic; the kernel is the one of
// forward.hpp, instantiated here for the 16-bit storage combinations (for
// generated maps only: packed parameters at P = 5).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.hpp"
#include "forward.hpp"
#include "launch.hpp"

namespace mck {

hipError_t launch_forward_t(int M, int P, int waves, bool vec, int xt, int yt, const void* x, int64_t batch, int d,
                            int64_t E, const float* B, const uint32_t* goff, const float* Gs, const float* Sx,
                            float cs, void* out, hipStream_t s, const int8_t* xexp)
{
#define MCK_FWDT_ARGS M, P, waves, true, vec, true, x, batch, d, E, B, goff, Gs, Sx, cs, out, s, xexp
    if (xt == kF32 && yt == kBF16)
        return dispatch_m<RunForwardT<kF32, kBF16>::Run>(MCK_FWDT_ARGS);
    if (xt == kF32 && yt == kF16)
        return dispatch_m<RunForwardT<kF32, kF16>::Run>(MCK_FWDT_ARGS);
    if (xt == kBF16 && yt == kBF16)
        return dispatch_m<RunForwardT<kBF16, kBF16>::Run>(MCK_FWDT_ARGS);
    if (xt == kF16 && yt == kF16)
        return dispatch_m<RunForwardT<kF16, kF16>::Run>(MCK_FWDT_ARGS);
#undef MCK_FWDT_ARGS
    return hipErrorInvalidValue;
}

}  // namespace mck

// Device-side pieces shared by the log-domain convolution kernels (conv_lse.hip) and the
// certified linear-domain kernels on the matrix cores (conv_linear.hip): address-space
// views of global memory and the scaling epilogue of one output element.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "conv_lse.h"

namespace se2 {

// Global-memory views of the job's pointers: global (not flat) loads wait on the
// vector-memory counter only, so they do not serialise against LDS traffic.
typedef const __attribute__((address_space(1))) double *gdptr;
typedef const __attribute__((address_space(1))) float *gfptr;
typedef const __attribute__((address_space(1))) int32_t *giptr;
typedef __attribute__((address_space(1))) double *gdptr_w;
typedef __attribute__((address_space(1))) float *gfptr_w;

// Scaling epilogue of one output element (base-2 logs); returns its contribution to the
// marginal error.  EPI_RAW: out = lse.  EPI_SCALE (a Sinkhorn half-step, the IBP w-update):
// out = log m - lse and, with `old`, the error term m |2^(old - out) - 1| of the first
// marginal (Section 4.1).  EPI_ADD (the IBP d-update): out = base + lse.  Checks pass
// out = nullptr and keep only the error.
__device__ __forceinline__ double epilogue(const ConvJob &job, size_t idx, double lse) {
    double o, err = 0.0;
    if (job.epi == EPI_RAW) {
        o = lse;
    } else if (job.epi == EPI_SCALE) {
        const double lm = ((gdptr)job.aux)[idx];
        o = (lm == -INFINITY) ? -INFINITY : lm - lse;
        if (job.old != nullptr && lm != -INFINITY) err = exp2(lm) * fabs(expm1((((gdptr)job.old)[idx] - o) * kLn2));
    } else {
        const double bse = ((gdptr)job.aux)[idx];
        o = (bse == -INFINITY || lse == -INFINITY) ? -INFINITY : bse + lse;
    }
    if (job.out != nullptr) ((gdptr_w)job.out)[idx] = o;
    return err;
}

// Butterfly sum over the 64 lanes of a wave in a fixed lane pattern (deterministic).
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

}  // namespace se2

// Kernel launches of the convolution engines with optional kernel-bound timing events.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <tuple>
#include <utility>

#include "se2_internal.h"

namespace se2 {

// Timing of a group of convolution launches without marker packets between kernels: while
// a LaunchEvents is installed on the calling thread (launch_events()), the first kernel that
// launch_kernel() issues takes `start` as its own start time, and the kernel a launcher
// marks as its last takes `stop` as its end time (hipExtLaunchKernel binds an event to the
// dispatch itself).  Each event is taken once; the installer records whatever is left
// (no kernel launched) as an ordinary event.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents *&launch_events();

// Launches kern<<<grid, block, lds, s>>>(args...), taking the installed events as above.
// The arguments are converted to the kernel's parameter types before their addresses are
// handed to hipExtLaunchKernel.
template <typename... P, typename... A>
int launch_kernel(void (*kern)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t s, bool last, A... args) {
    static_assert(sizeof...(P) == sizeof...(A), "one argument per kernel parameter");
    LaunchEvents *ev = launch_events();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ev) {
        std::swap(e0, ev->start);
        if (last) std::swap(e1, ev->stop);
    }
    if (!e0 && !e1) {
        hipLaunchKernelGGL(kern, grid, block, lds, s, args...);
    } else {
        std::tuple<P...> vals{static_cast<P>(args)...};
        void *ptrs[sizeof...(P) > 0 ? sizeof...(P) : 1];
        std::apply([&ptrs](auto &...v) {
            int i = 0;
            ((ptrs[i++] = static_cast<void *>(&v)), ...);
        }, vals);
        SE2_HIP(hipExtLaunchKernel(reinterpret_cast<const void *>(kern), grid, block, ptrs, lds, s, e0, e1, 0));
    }
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

}  // namespace se2

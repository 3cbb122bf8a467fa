// Kernel launches whose profiling events are stamped by the dispatch (device code only).
#pragma once

#include <hip/hip_ext.h>

#include "sgn_internal.h"

namespace sgn {

// Launch one kernel on s.  With a stamp (a sampled profiling record), the dispatch itself records
// the kernel's start and end into the stamp's events (hipExtLaunchKernel), so the measured time is
// the kernel's execution, without the queue drain that event markers around a launch add.
template <typename F, typename... Args>
void launch_k(const LaunchStamp &ev, F kernel, dim3 g, dim3 b, uint32_t lds, hipStream_t s, Args... args)
{
    if (ev.stop)
        hipExtLaunchKernelGGL(kernel, g, b, lds, s, ev.start, ev.stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, g, b, lds, s, args...);
}

}  // namespace sgn

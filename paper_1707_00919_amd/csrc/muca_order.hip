// muca_order.hip -- dispatch order of a batched round's launches.
//
// A round's groups (one launch per L and kernel form) run on streams of their
// own.  When a round mixes two-wave workgroups (the longest chains, whose
// workgroups take most of a CU's LDS) with one-wave ones, the launch that
// reaches the dispatcher first spreads its workgroups over the CUs, and if
// that is a one-wave launch, two-wave workgroups can find no CU with room and
// start only when one-wave workgroups end: the round then lasts a short
// chain plus a long one; among one-wave launches, the same holds for a
// long-chain launch whose workgroups need much LDS.  The batch runtime
// therefore issues a round's launches longest chains first (two-wave ones
// before the others) and, in rounds whose two-wave workgroups do not all fit
// or run in pairs, puts a wait in front of each later one, a little longer
// for each, so that workgroups are placed in that order.  Results do
// not depend on it (every workgroup runs the same chains whatever CU it lands
// on).
#include <hip/hip_runtime.h>

#include "muca_internal.h"

namespace muca {
namespace {

// One wave that returns once `ticks` of the 100 MHz constant clock have
// passed, or after a bounded number of polls (each about 0.2 us), whichever
// comes first.
__global__ __launch_bounds__(64) void dispatch_delay_kernel(uint64_t ticks)
{
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (uint32_t i = 0; i < 8192u; ++i) {
        if (__builtin_amdgcn_s_memrealtime() - t0 >= ticks)
            break;
        __builtin_amdgcn_s_sleep(8);
    }
}

}  // namespace

hipError_t launch_dispatch_delay(uint32_t microseconds, hipStream_t s)
{
    if (microseconds == 0)
        return hipSuccess;
    hipLaunchKernelGGL(dispatch_delay_kernel, dim3(1), dim3(64), 0, s, (uint64_t)microseconds * 100u);
    return hipGetLastError();
}

}  // namespace muca

// The (cos, sin) sample table computed on the device, for the entry point
// that has no handle (and so no host staging buffer to upload a table from).
//
// Step 0 of the rule: theta_j = ((2j + 1 - J) / J) * (pi / 2) in binary64,
// cos and sin in binary64, each rounded once to binary32; the same
// expression the host computes for a handle's table.  Binary64 cos and sin
// differ from the host's by at most an ulp of binary64, so the binary32
// roundings agree unless a binary32 rounding boundary lies between them; the
// test suite compares every entry of every J the entry point accepts with
// the host's table.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace rv {

__device__ __forceinline__ float2 table_entry(int j, int J)
{
    const double th = ((double)(2 * j + 1 - J) / (double)J) * M_PI_2;
    return make_float2((float)cos(th), (float)sin(th));
}

}  // namespace rv

// sh_internal.h -- launchers shared between the kernel files and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shk {

// Forward values R_l^m for l <= lmax at n points xyz[n][3] into out[F][ld].
template <typename TIO>
hipError_t launch_fwd(int lmax, int64_t n, const TIO* xyz, TIO* out, int64_t ld, hipStream_t s);

}  // namespace shk

// Launcher of the corner-turn kernel (corner_turn.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spl {

// in: [n_t][in_stride] bytes (nch used per row), out: [nch][pitch]; the caller checks
// alignment (16 bytes), in_stride and pitch multiples of 16, and pitch >= n_t.
hipError_t launch_corner_turn(const uint8_t *in, int64_t in_stride, int64_t n_t, int nch, uint8_t *out, int64_t pitch,
                              hipStream_t s);

}  // namespace spl

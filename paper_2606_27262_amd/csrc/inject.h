// Quantised-domain injection kernel (launcher).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace spl {

constexpr int SPL_INJECT_ARGMAX_MODE = 1;

// Windows [n_win][nch][n_sig] of signal added to block [nch][pitch] in place; the
// edges are those of a bits-bit quantiser of Normal(mu, sigma) noise with states
// level * sigma wide, shifted by offset states.  words may be NULL in ARGMAX mode.
hipError_t launch_inject(uint8_t *block, int64_t pitch, int64_t n_t, int nch, const int32_t *t_start,
                         const float *signal, const uint32_t *words, int n_win, int n_sig, int bits, double mu,
                         double sigma, double level, double offset, int mode, hipStream_t s);

}  // namespace spl

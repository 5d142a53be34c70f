// Device ring of a continuous beam stream (the paper reads each block with an overlap so
// that the dispersion sweeps and boxcars of its owned samples are complete): block k of a
// beam reads stream samples [k n_out, k n_out + n_in), so consecutive blocks share the
// carry = n_in - n_out = s_max + w_max - 1 samples of the overlap.  Only the n_out new
// samples of a block cross the host link, as one contiguous copy into a device staging
// buffer; k_stream_assemble then writes the whole next block from the previous block's
// tail and the staged samples.  Pure data movement, bound by HBM: n_in bytes written and
// n_in bytes read per channel.
//
// Thread = 16 output bytes of one row.  Bytes from the previous block are read as
// aligned 16-byte vectors (n_out and both pitches are multiples of 16); bytes from the
// staging buffer start at an arbitrary offset (carry % 4 != 0 in general) and are read
// as five aligned dwords combined with v_alignbyte; the vector that straddles the
// carry boundary, and the row's last partial vector, go byte by byte.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>

#include "spotlight.h"

spl_status spl_internal_fail(spl_status st, const char *msg);

namespace {

spl_status failf(spl_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return spl_internal_fail(st, buf);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_assemble(uint8_t *__restrict__ next, int64_t next_pitch,
                                                         const uint8_t *__restrict__ prev, int64_t prev_pitch,
                                                         const uint8_t *__restrict__ stage, int64_t stage_pitch,
                                                         int64_t n_out, int64_t n_in, int64_t nvec) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= nvec) return;
    const int64_t c = blockIdx.y;
    const int64_t carry = n_in - n_out;
    const int64_t j = 16 * v;
    uint8_t *dst = next + c * next_pitch + j;
    const uint8_t *p = prev + c * prev_pitch + n_out;   // p[i] = byte i of the carried tail
    const uint8_t *q = stage + c * stage_pitch;         // q[i] = new sample i
    if (j + 16 <= n_in && (j + 16 <= carry || j >= carry)) {
        u32x4 out;
        if (j + 16 <= carry) {
            out = *(const u32x4 *)(p + j);
        } else {
            const int64_t o = j - carry;
            const uint32_t *w = (const uint32_t *)(q + (o & ~(int64_t)3));
            const uint32_t sh = (uint32_t)(o & 3) * 8u;
            uint32_t d[5];
#pragma unroll
            for (int i = 0; i < 5; ++i) d[i] = w[i];
#pragma unroll
            for (int i = 0; i < 4; ++i) out[i] = sh ? (d[i] >> sh) | (d[i + 1] << (32u - sh)) : d[i];
        }
        *(u32x4 *)dst = out;
        return;
    }
    for (int64_t i = 0; i < 16 && j + i < n_in; ++i) dst[i] = j + i < carry ? p[j + i] : q[j + i - carry];
}

}  // namespace

extern "C" spl_status spl_stream_assemble(uint8_t *d_next, int64_t next_pitch, const uint8_t *d_prev,
                                          int64_t prev_pitch, const uint8_t *d_stage, int64_t stage_pitch,
                                          int32_t nch, int64_t n_out, int64_t n_in, hipStream_t stream) {
    if (!d_next || !d_stage || (!d_prev && n_in > n_out)) return failf(SPL_E_INVALID_ARG, "NULL buffer");
    if (nch < 1 || nch > 65535) return failf(SPL_E_INVALID_ARG, "nch must be in [1, 65535]");
    if (n_out < 1 || n_in < n_out) return failf(SPL_E_INVALID_ARG, "need 1 <= n_out <= n_in");
    if ((n_out & 15) || (next_pitch & 15) || (prev_pitch & 15) || (((uintptr_t)d_next | (uintptr_t)d_prev) & 15) ||
        ((uintptr_t)d_stage & 3) || (stage_pitch & 3))
        return failf(SPL_E_INVALID_ARG, "n_out, the block pitches and pointers must be multiples of 16, the "
                     "staging pitch and pointer of 4");
    if (next_pitch < n_in || prev_pitch < n_in || stage_pitch < n_out)
        return failf(SPL_E_INVALID_ARG, "a pitch is below its row length");
    const uint8_t *nlo = d_next, *nhi = d_next + (size_t)(nch - 1) * next_pitch + n_in;
    if (d_prev) {
        const uint8_t *lo = d_prev, *hi = d_prev + (size_t)(nch - 1) * prev_pitch + n_in;
        if (nlo < hi && lo < nhi) return failf(SPL_E_INVALID_ARG, "the two blocks overlap");
    }
    const uint8_t *slo = d_stage, *shi = d_stage + (size_t)(nch - 1) * stage_pitch + n_out + 16;
    if (nlo < shi && slo < nhi) return failf(SPL_E_INVALID_ARG, "the staging buffer overlaps the next block");
    const int64_t nvec = (n_in + 15) / 16;
    dim3 grid((unsigned)((nvec + 255) / 256), (unsigned)nch);
    hipLaunchKernelGGL(k_stream_assemble, grid, dim3(256), 0, stream, d_next, next_pitch, d_prev, prev_pitch, d_stage,
                       stage_pitch, n_out, n_in, nvec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return failf(SPL_E_HIP, "k_stream_assemble launch: %s", hipGetErrorString(e));
    return SPL_OK;
}

// Launchers of the ranker kernels (ranker.hip); each enqueues on stream `s`.
#pragma once

#include "spl_internal.h"
#include "spotlight.h"

namespace spl {

// Plane 0 of each snippet replaced by the fine-DM transform around the candidate's DM.
hipError_t launch_fine_dm(const DevBeam *beams, int nbeams, const spl_candidate *cands, int64_t n, double keep,
                          uint16_t *out, hipStream_t s);
hipError_t launch_snippets(const DevBeam *beams, int nbeams, const spl_candidate *cands, int64_t n, uint16_t *out,
                           hipStream_t s);
hipError_t launch_gemm(const uint16_t *A, int64_t lda, const uint16_t *B, int64_t ldb, float *C, int64_t ldc, int M,
                       int N, int K, int splits, bool accumulate, hipStream_t s);
// Forward convolution (mode 0: first layer, NCHW 2 channels; 1: NHWC 32 channels) with
// bias, ReLU and 2x2 max pool fused: pooled BF16 NHWC [N][H/2][W/2][32] and the pool
// decisions; H even, W a multiple of 8, N*H*W a multiple of 64.
hipError_t launch_conv_pool(int mode, const uint16_t *X, int N, int nvalid, int H, int W, const uint16_t *Wt, int ldw,
                            const float *bias, uint16_t *pooled, uint8_t *arg, hipStream_t s);
// Implicit-GEMM convolution (mode 0: first layer, NCHW 2 channels; 1: forward, NHWC 32
// channels; 2: input gradient, NHWC 32 channels, flipped taps) into C [N*H*W][32] FP32.
hipError_t launch_conv(int mode, const uint16_t *X, int N, int nvalid, int H, int W, const uint16_t *Wt, int ldw,
                       float *C, hipStream_t s);
// Weight gradient partials part[nparts][K][32] (mode 0: K = 32, first layer; 1: K = 288).
hipError_t launch_wgrad(int mode, const uint16_t *X, int N, int nvalid, int H, int W, const uint16_t *dZ, float *part,
                        int nparts, hipStream_t s);
// Deterministic sum of nparts partial arrays of n floats; above 256 parts in two passes
// through tmp (room for kSumPartsMaxGroups * n floats).
constexpr int kSumPartsMaxGroups = 160;
hipError_t launch_sum_parts(const float *part, int nparts, int64_t n, float *out, float *tmp, hipStream_t s);
hipError_t launch_transpose16(const uint16_t *in, int64_t rows, int64_t cols, int64_t ldi, uint16_t *out, int64_t ldo,
                              hipStream_t s);
hipError_t launch_unpool(const float *dOut, const uint8_t *arg, int N, int H, int W, uint16_t *dZ, float *dbias,
                         hipStream_t s);
hipError_t launch_head(const float *Hm, const float *b1, const float *f2w, const float *f2b, int N, int Nb,
                       float *logits, const float *labels, float *loss, float *g_f2w, float *g_f2b, float *g_b1,
                       uint16_t *dH, uint16_t *dHT, int64_t ldT, hipStream_t s);
hipError_t launch_pack_idx(const float *master, const int32_t *idx, int64_t n, uint16_t *out, hipStream_t s);
hipError_t launch_scatter_idx(const float *in, const int32_t *idx, int64_t n, float *master, hipStream_t s);
hipError_t launch_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2, float eps,
                       int64_t t, hipStream_t s);
hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s);
hipError_t launch_zero_u16(uint16_t *p, int64_t n, hipStream_t s);

}  // namespace spl

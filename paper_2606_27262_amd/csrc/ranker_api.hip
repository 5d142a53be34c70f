// Host runtime of the candidate ranker: workspace layout, the tables that pack the FP32
// master parameters into the BF16 GEMM operands (and scatter GEMM weight gradients
// back), and the launch sequence of a forward pass, a backward pass and an Adam step.
//
// Per batch of Nb candidates (Nb = max_batch rounded up to 32; a pass over fewer
// candidates pads with zero images whose gradients are zero):
//   layer k = 1..4, input H_k x W_k (64x256, 32x128, 16x64, 8x32), Cin_k (2, 32, 32, 32),
//   P_k = Nb*H_k*W_k output pixels, K_k = 9*Cin_k padded to a multiple of 32 (32, 288):
//     X_k, arg_k = maxpool(ReLU(conv(X_{k-1}, Wp_k) + b_k))   NHWC BF16, one kernel: the
//                   implicit-GEMM convolution keeps its FP32 result in registers
//   Hm = X_4 [Nb][2048 (h,w,c)] * Wf1p^T            [Nb][64]    FP32, then the VALU head.
// Backward, layer k = 4..1, from dX = dLoss/dX_k (FP32):
//     dZ = unpool(dX, arg_k); db_k += sums
//     dW_k^T [K_k][32] = sum over pixel slabs of A^T dZ (LDS-staged partials, then summed)
//     dX = conv_flipped(dZ, Wd_k)                    (k > 1), Wd_k[ci][(ky*3+kx)*32+co]
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "ranker.h"
#include "spotlight.h"

#pragma STDC FP_CONTRACT OFF

using namespace spl;

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

#define RK_TRY(expr)                                                                                     \
    do {                                                                                                 \
        hipError_t e__ = (expr);                                                                         \
        if (e__ != hipSuccess)                                                                           \
            return failf(SPL_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e__), __FILE__,    \
                         __LINE__);                                                                      \
    } while (0)

constexpr int kLayers = 4;
constexpr int kCout = 32;
constexpr int kH[kLayers] = {64, 32, 16, 8};
constexpr int kW[kLayers] = {256, 128, 64, 32};
constexpr int kCin[kLayers] = {2, 32, 32, 32};
constexpr int kKp[kLayers] = {32, 288, 288, 288};
constexpr int kFcIn = 2048, kFcHidden = 64;
// workgroups (and partial sums) of a weight-gradient pass: 32-channel layers use up to
// kWgradParts, the first layer (a 32 x 32 result) up to kWgradPartsFirst in the same buffer
constexpr int kWgradParts = 2048;
constexpr int kWgradPartsFirst = kWgradParts * 9;

// Offsets of the parameters in their fixed order.
struct ParamOffsets {
    int64_t cw[kLayers], cb[kLayers], f1w, f1b, f2w, f2b, total;
    ParamOffsets() {
        int64_t o = 0;
        for (int k = 0; k < kLayers; ++k) {
            cw[k] = o;
            o += (int64_t)kCout * kCin[k] * 9;
            cb[k] = o;
            o += kCout;
        }
        f1w = o;
        o += (int64_t)kFcHidden * kFcIn;
        f1b = o;
        o += kFcHidden;
        f2w = o;
        o += kFcHidden;
        f2b = o;
        o += 1;
        total = o;
    }
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

struct spl_ranker {
    spl_ranker_opts o{};
    int nb = 0;  // candidates per pass (multiple of 32)
    ParamOffsets po;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool have_weights = false;
    int64_t step = 0;
    // persistent parts
    size_t off_master = 0, off_m = 0, off_v = 0, off_g = 0;
    size_t off_packed = 0, off_pack_idx = 0, off_gc = 0, off_gc_idx = 0;
    int64_t n_packed = 0, n_gc = 0;
    int64_t pk_wp[kLayers] = {}, pk_wd[kLayers] = {}, pk_f1 = 0, pk_f1t = 0;  // element offsets in packed
    int64_t gc_w[kLayers] = {}, gc_f1 = 0;                                   // element offsets in gc
    // per-pass buffers
    size_t off_X[kLayers] = {}, off_arg[kLayers] = {};
    size_t off_Hm = 0, off_logits = 0, off_dH = 0, off_dHT = 0, off_X4T = 0, off_dX = 0;
    size_t off_dZ = 0, off_part = 0, off_part2 = 0;
    std::vector<int32_t> pack_idx, gc_idx;

    template <class T>
    T *at(size_t off) const { return (T *)(ws + off); }
    int64_t P(int k) const { return (int64_t)nb * kH[k] * kW[k]; }
};

namespace {

// Index tables: packed[i] = bf16(master[pack_idx[i]]) and master_grad[gc_idx[i]] = gc[i].
void build_tables(spl_ranker *R) {
    const ParamOffsets &po = R->po;
    auto &pk = R->pack_idx;
    auto &gc = R->gc_idx;
    pk.clear();
    gc.clear();
    auto pad8 = [](std::vector<int32_t> &v) {
        while (v.size() % 128) v.push_back(-1);  // 256-byte alignment of BF16 sub-arrays
    };
    auto conv_index = [&](int k, int co, int kk) -> int32_t {
        const int cin = kCin[k];
        if (kk >= 9 * cin) return -1;
        const int pos = kk / cin, ci = kk % cin, ky = pos / 3, kx = pos % 3;
        return (int32_t)(po.cw[k] + ((int64_t)(co * cin + ci) * 3 + ky) * 3 + kx);
    };
    for (int k = 0; k < kLayers; ++k) {  // forward operands Wp_k [32][K_k]
        R->pk_wp[k] = (int64_t)pk.size();
        for (int co = 0; co < kCout; ++co)
            for (int kk = 0; kk < kKp[k]; ++kk) pk.push_back(conv_index(k, co, kk));
        pad8(pk);
    }
    for (int k = 1; k < kLayers; ++k) {  // input-gradient operands Wd_k [Cin][(ky*3+kx)*32 + co]
        R->pk_wd[k] = (int64_t)pk.size();
        for (int ci = 0; ci < kCin[k]; ++ci)
            for (int pos = 0; pos < 9; ++pos)
                for (int co = 0; co < kCout; ++co) {
                    const int ky = pos / 3, kx = pos % 3;
                    pk.push_back((int32_t)(po.cw[k] + ((int64_t)(co * kCin[k] + ci) * 3 + ky) * 3 + kx));
                }
        pad8(pk);
    }
    auto f1_index = [&](int j, int hwc) -> int32_t {  // hwc = (h*16 + w)*32 + c -> f1w[j][(c*4 + h)*16 + w]
        const int c = hwc & 31, hw = hwc >> 5, h = hw / 16, w = hw % 16;
        return (int32_t)(po.f1w + (int64_t)j * kFcIn + (c * 4 + h) * 16 + w);
    };
    R->pk_f1 = (int64_t)pk.size();  // Wf1p [64][2048 (h,w,c)]
    for (int j = 0; j < kFcHidden; ++j)
        for (int i = 0; i < kFcIn; ++i) pk.push_back(f1_index(j, i));
    pad8(pk);
    R->pk_f1t = (int64_t)pk.size();  // Wf1p^T [2048][64]
    for (int i = 0; i < kFcIn; ++i)
        for (int j = 0; j < kFcHidden; ++j) pk.push_back(f1_index(j, i));
    pad8(pk);
    R->n_packed = (int64_t)pk.size();

    for (int k = 0; k < kLayers; ++k) {  // weight gradients dW_k^T [K_k][32]
        R->gc_w[k] = (int64_t)gc.size();
        for (int kk = 0; kk < kKp[k]; ++kk)
            for (int co = 0; co < kCout; ++co) gc.push_back(conv_index(k, co, kk));
        while (gc.size() % 64) gc.push_back(-1);
    }
    R->gc_f1 = (int64_t)gc.size();  // dWf1^T [2048 (h,w,c)][64]
    for (int i = 0; i < kFcIn; ++i)
        for (int j = 0; j < kFcHidden; ++j) gc.push_back(f1_index(j, i));
    R->n_gc = (int64_t)gc.size();
}

void layout(spl_ranker *R) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = align256(off);
        const size_t o = off;
        off += bytes;
        return o;
    };
    const int64_t np = R->po.total;
    R->off_master = take(np * 4);
    R->off_m = take(np * 4);
    R->off_v = take(np * 4);
    R->off_g = take(np * 4);
    R->off_packed = take(R->n_packed * 2);
    R->off_pack_idx = take(R->n_packed * 4);
    R->off_gc = take(R->n_gc * 4);
    R->off_gc_idx = take(R->n_gc * 4);
    const int64_t nb = R->nb;
    int64_t max_dz = 0, max_dx = nb * kFcIn;
    for (int k = 0; k < kLayers; ++k) {
        R->off_X[k] = take((size_t)(R->P(k) / 4) * kCout * 2);
        R->off_arg[k] = take((size_t)(R->P(k) / 4) * kCout);
        max_dz = std::max(max_dz, R->P(k) * kCout);
        if (k > 0) max_dx = std::max(max_dx, R->P(k) * kCout);
    }
    R->off_Hm = take((size_t)nb * kFcHidden * 4);
    R->off_logits = take((size_t)nb * 4 + 4);  // + loss slot
    R->off_dH = take((size_t)nb * kFcHidden * 2);
    R->off_dHT = take((size_t)nb * kFcHidden * 2);
    R->off_X4T = take((size_t)nb * kFcIn * 2);
    R->off_dX = take((size_t)max_dx * 4);
    R->off_dZ = take((size_t)max_dz * 2);
    R->off_part = take((size_t)kWgradParts * 288 * kCout * 4);
    R->off_part2 = take((size_t)kSumPartsMaxGroups * 288 * kCout * 4);
    R->ws_bytes = align256(off);
}

// C = A * B^T with a split of K chosen to give the chip about a thousand workgroups.
hipError_t gemm(const uint16_t *A, int64_t lda, const uint16_t *B, int64_t ldb, float *C, int64_t ldc, int M, int N,
                int K, hipStream_t s) {
    const int64_t tiles = (int64_t)((M + 63) / 64) * ((N + 31) / 32);
    const int kb = K / 32;
    int splits = 1;
    if (tiles < 1024) splits = (int)std::min<int64_t>(kb, (1024 + tiles - 1) / tiles);
    const int klen = (kb + splits - 1) / splits * 32;
    splits = (K + klen - 1) / klen;
    if (splits > 1) {
        if (ldc != N) return hipErrorInvalidValue;  // zero fill assumes a dense C
        hipError_t e = launch_zero_f32(C, (int64_t)M * N, s);
        if (e != hipSuccess) return e;
    }
    return launch_gemm(A, lda, B, ldb, C, ldc, M, N, K, splits, false, s);
}

spl_status forward(spl_ranker *R, const uint16_t *snip, int n, hipStream_t s) {
    const int nb = R->nb;
    const uint16_t *packed = R->at<uint16_t>(R->off_packed);
    const float *master = R->at<float>(R->off_master);
    for (int k = 0; k < kLayers; ++k) {
        const uint16_t *in = k == 0 ? snip : R->at<uint16_t>(R->off_X[k - 1]);
        RK_TRY(launch_conv_pool(k == 0 ? 0 : 1, in, nb, k == 0 ? n : nb, kH[k], kW[k], packed + R->pk_wp[k], kKp[k],
                                master + R->po.cb[k], R->at<uint16_t>(R->off_X[k]), R->at<uint8_t>(R->off_arg[k]), s));
    }
    RK_TRY(gemm(R->at<uint16_t>(R->off_X[3]), kFcIn, packed + R->pk_f1, kFcIn, R->at<float>(R->off_Hm), kFcHidden, nb,
                kFcHidden, kFcIn, s));
    return SPL_OK;
}

spl_status backward(spl_ranker *R, const uint16_t *snip, int n, const float *labels, float *loss, hipStream_t s) {
    const int nb = R->nb;
    const uint16_t *packed = R->at<uint16_t>(R->off_packed);
    const float *master = R->at<float>(R->off_master);
    float *G = R->at<float>(R->off_g);
    float *gc = R->at<float>(R->off_gc);
    float *part = R->at<float>(R->off_part);
    const ParamOffsets &po = R->po;
    uint16_t *dH = R->at<uint16_t>(R->off_dH), *dHT = R->at<uint16_t>(R->off_dHT);
    float *dX = R->at<float>(R->off_dX);
    uint16_t *dZ = R->at<uint16_t>(R->off_dZ);
    RK_TRY(launch_zero_f32(G, po.total, s));
    RK_TRY(launch_head(R->at<float>(R->off_Hm), master + po.f1b, master + po.f2w, master + po.f2b, n, nb,
                       R->at<float>(R->off_logits), labels, loss, G + po.f2w, G + po.f2b, G + po.f1b, dH, dHT, nb, s));
    // fully connected 2048 -> 64
    uint16_t *X4 = R->at<uint16_t>(R->off_X[3]), *X4T = R->at<uint16_t>(R->off_X4T);
    RK_TRY(launch_transpose16(X4, nb, kFcIn, kFcIn, X4T, nb, s));
    RK_TRY(gemm(X4T, nb, dHT, nb, gc + R->gc_f1, kFcHidden, kFcIn, kFcHidden, nb, s));
    RK_TRY(gemm(dH, kFcHidden, packed + R->pk_f1t, kFcHidden, dX, kFcIn, nb, kFcIn, kFcHidden, s));
    for (int k = kLayers - 1; k >= 0; --k) {
        const int64_t P = R->P(k);
        const uint16_t *in = k == 0 ? snip : R->at<uint16_t>(R->off_X[k - 1]);
        RK_TRY(launch_unpool(dX, R->at<uint8_t>(R->off_arg[k]), nb, kH[k], kW[k], dZ, G + po.cb[k], s));
        // first layer: about 16 slabs of 32 pixels per wavefront; the others: one
        // workgroup per slab up to kWgradParts
        const int parts = (int)std::max<int64_t>(
            1, std::min<int64_t>(k == 0 ? kWgradPartsFirst : kWgradParts, k == 0 ? P / 32 / 64 : P / 32));
        RK_TRY(launch_wgrad(k == 0 ? 0 : 1, in, nb, k == 0 ? n : nb, kH[k], kW[k], dZ, part, parts, s));
        RK_TRY(launch_sum_parts(part, parts, (int64_t)kKp[k] * kCout, gc + R->gc_w[k], R->at<float>(R->off_part2), s));
        if (k > 0) RK_TRY(launch_conv(2, dZ, nb, nb, kH[k], kW[k], packed + R->pk_wd[k], 288, dX, s));
    }
    RK_TRY(launch_scatter_idx(gc, R->at<int32_t>(R->off_gc_idx), R->n_gc, G, s));
    return SPL_OK;
}

spl_status check_ready(const spl_ranker *R) {
    if (!R) return failf(SPL_E_INVALID_ARG, "ranker is NULL");
    if (!R->ws) return failf(SPL_E_INVALID_ARG, "spl_ranker_set_workspace was not called");
    if (!R->have_weights) return failf(SPL_E_NO_WEIGHTS, "the ranker has no weights");
    return SPL_OK;
}

}  // namespace

extern "C" spl_status spl_ranker_create(const spl_ranker_opts *opts, spl_ranker **out) {
    if (!out) return failf(SPL_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    spl_ranker_opts o{};
    if (opts) o = *opts;
    if (o.max_batch == 0) o.max_batch = 256;
    if (o.max_batch < 1 || o.max_batch > 1024) return failf(SPL_E_INVALID_ARG, "max_batch must be in [1, 1024]");
    if (o.beta1 == 0.f) o.beta1 = 0.9f;
    if (o.beta2 == 0.f) o.beta2 = 0.999f;
    if (o.eps == 0.f) o.eps = 1e-8f;
    if (!(o.beta1 > 0.f && o.beta1 < 1.f) || !(o.beta2 > 0.f && o.beta2 < 1.f) || !(o.eps > 0.f))
        return failf(SPL_E_INVALID_ARG, "Adam parameters out of range");
    spl_ranker *R = new (std::nothrow) spl_ranker();
    if (!R) return failf(SPL_E_OOM, "host allocation failed");
    R->o = o;
    R->nb = (o.max_batch + 31) / 32 * 32;
    if (R->po.total != SPL_RANKER_PARAMS) {
        delete R;
        return failf(SPL_E_INTERNAL, "parameter count mismatch");
    }
    build_tables(R);
    layout(R);
    *out = R;
    return SPL_OK;
}

extern "C" spl_status spl_ranker_workspace_size(const spl_ranker *R, size_t *bytes) {
    if (!R || !bytes) return failf(SPL_E_INVALID_ARG, "NULL argument");
    *bytes = R->ws_bytes;
    return SPL_OK;
}

extern "C" spl_status spl_ranker_set_workspace(spl_ranker *R, void *d_ws, size_t bytes) {
    if (!R || !d_ws) return failf(SPL_E_INVALID_ARG, "NULL argument");
    if (((uintptr_t)d_ws & 255) != 0) return failf(SPL_E_INVALID_ARG, "workspace must be 256-byte aligned");
    if (bytes < R->ws_bytes) return failf(SPL_E_OOM, "workspace too small: %zu < %zu bytes", bytes, R->ws_bytes);
    R->ws = (char *)d_ws;
    R->have_weights = false;
    R->step = 0;
    RK_TRY(hipMemcpy(R->ws + R->off_pack_idx, R->pack_idx.data(), R->pack_idx.size() * 4, hipMemcpyHostToDevice));
    RK_TRY(hipMemcpy(R->ws + R->off_gc_idx, R->gc_idx.data(), R->gc_idx.size() * 4, hipMemcpyHostToDevice));
    return SPL_OK;
}

extern "C" spl_status spl_ranker_set_weights(spl_ranker *R, const float *host_params) {
    if (!R || !host_params) return failf(SPL_E_INVALID_ARG, "NULL argument");
    if (!R->ws) return failf(SPL_E_INVALID_ARG, "spl_ranker_set_workspace was not called");
    const int64_t np = R->po.total;
    RK_TRY(hipMemcpy(R->ws + R->off_master, host_params, np * 4, hipMemcpyHostToDevice));
    RK_TRY(launch_zero_f32(R->at<float>(R->off_m), np, nullptr));
    RK_TRY(launch_zero_f32(R->at<float>(R->off_v), np, nullptr));
    RK_TRY(launch_pack_idx(R->at<float>(R->off_master), R->at<int32_t>(R->off_pack_idx), R->n_packed,
                           R->at<uint16_t>(R->off_packed), nullptr));
    RK_TRY(hipDeviceSynchronize());
    R->have_weights = true;
    R->step = 0;
    return SPL_OK;
}

extern "C" spl_status spl_ranker_get_weights(const spl_ranker *R, float *host_params, hipStream_t stream) {
    spl_status st = check_ready(R);
    if (st != SPL_OK) return st;
    if (!host_params) return failf(SPL_E_INVALID_ARG, "NULL argument");
    RK_TRY(hipMemcpyAsync(host_params, R->ws + R->off_master, R->po.total * 4, hipMemcpyDeviceToHost, stream));
    RK_TRY(hipStreamSynchronize(stream));
    return SPL_OK;
}

extern "C" spl_status spl_ranker_score(spl_ranker *R, const uint16_t *d_snip, int64_t n, float *d_logits,
                                       hipStream_t stream) {
    spl_status st = check_ready(R);
    if (st != SPL_OK) return st;
    if (n < 0 || (n > 0 && (!d_snip || !d_logits))) return failf(SPL_E_INVALID_ARG, "bad snippet or logit buffer");
    for (int64_t i0 = 0; i0 < n; i0 += R->nb) {
        const int m = (int)std::min<int64_t>(R->nb, n - i0);
        st = forward(R, d_snip + i0 * SPL_SNIPPET_ELEMS, m, stream);
        if (st != SPL_OK) return st;
        const ParamOffsets &po = R->po;
        const float *master = R->at<float>(R->off_master);
        RK_TRY(launch_head(R->at<float>(R->off_Hm), master + po.f1b, master + po.f2w, master + po.f2b, m, R->nb,
                           d_logits + i0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, stream));
    }
    return SPL_OK;
}

extern "C" spl_status spl_ranker_backward(spl_ranker *R, const uint16_t *d_snip, const float *d_labels, int64_t n,
                                          float *d_loss, hipStream_t stream) {
    spl_status st = check_ready(R);
    if (st != SPL_OK) return st;
    if (n < 1 || n > R->o.max_batch) return failf(SPL_E_INVALID_ARG, "n must be in [1, max_batch]");
    if (!d_snip || !d_labels || !d_loss) return failf(SPL_E_INVALID_ARG, "NULL argument");
    st = forward(R, d_snip, (int)n, stream);
    if (st != SPL_OK) return st;
    return backward(R, d_snip, (int)n, d_labels, d_loss, stream);
}

extern "C" spl_status spl_ranker_train_step(spl_ranker *R, const uint16_t *d_snip, const float *d_labels, int64_t n,
                                            float lr, float *d_loss, hipStream_t stream) {
    if (!(lr > 0.f)) return failf(SPL_E_INVALID_ARG, "lr must be > 0");
    spl_status st = spl_ranker_backward(R, d_snip, d_labels, n, d_loss, stream);
    if (st != SPL_OK) return st;
    R->step += 1;
    RK_TRY(launch_adam(R->at<float>(R->off_master), R->at<float>(R->off_m), R->at<float>(R->off_v),
                       R->at<float>(R->off_g), R->po.total, lr, R->o.beta1, R->o.beta2, R->o.eps, R->step, stream));
    RK_TRY(launch_pack_idx(R->at<float>(R->off_master), R->at<int32_t>(R->off_pack_idx), R->n_packed,
                           R->at<uint16_t>(R->off_packed), stream));
    return SPL_OK;
}

extern "C" spl_status spl_ranker_grads(const spl_ranker *R, const float **d_grads) {
    spl_status st = check_ready(R);
    if (st != SPL_OK) return st;
    if (!d_grads) return failf(SPL_E_INVALID_ARG, "NULL argument");
    *d_grads = R->at<float>(R->off_g);
    return SPL_OK;
}

extern "C" void spl_ranker_destroy(spl_ranker *R) { delete R; }

extern "C" spl_status spl_ranker_debug_pool_args(const spl_ranker *R, int32_t layer, const uint8_t **d_arg) {
    spl_status st = check_ready(R);
    if (st != SPL_OK) return st;
    if (layer < 0 || layer >= kLayers || !d_arg) return failf(SPL_E_INVALID_ARG, "bad layer or NULL argument");
    *d_arg = R->at<uint8_t>(R->off_arg[layer]);
    return SPL_OK;
}

extern "C" spl_status spl_ranker_debug_fc_preact(const spl_ranker *R, const float **d_h) {
    spl_status st = check_ready(R);
    if (st != SPL_OK) return st;
    if (!d_h) return failf(SPL_E_INVALID_ARG, "NULL argument");
    *d_h = R->at<float>(R->off_Hm);
    return SPL_OK;
}

extern "C" spl_status spl_debug_gemm_bf16(const uint16_t *d_a, int64_t lda, const uint16_t *d_b, int64_t ldb,
                                          float *d_c, int64_t ldc, int32_t m, int32_t n, int32_t k,
                                          hipStream_t stream) {
    if (!d_a || !d_b || !d_c || m < 1 || n < 1 || k < 32 || (k & 31) || (lda & 7) || (ldb & 7) || lda < k ||
        ldb < k || ldc < n)
        return failf(SPL_E_INVALID_ARG, "spl_debug_gemm_bf16: bad argument");
    if (((uintptr_t)d_a & 15) || ((uintptr_t)d_b & 15))
        return failf(SPL_E_INVALID_ARG, "spl_debug_gemm_bf16: operands must be 16-byte aligned");
    RK_TRY(launch_gemm(d_a, lda, d_b, ldb, d_c, ldc, m, n, k, 1, false, stream));
    return SPL_OK;
}

// Candidate ranker on gfx950: feature snippets of each candidate and a small CNN
// (4 x [3x3 conv -> ReLU -> 2x2 max pool], 2 -> 32 -> 32 -> 32 -> 32 channels, then
// 2048 -> 64 -> 1 fully connected), standing in for the paper's FETCH classifier
// (classification section).  Every convolution and the first fully connected layer,
// forward and backward, is a GEMM on BF16 MFMA (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation; activations are stored as BF16 (round to nearest even), weights are kept
// in FP32 (Adam) and packed to BF16 for the GEMMs.
//
// Activation layout: NHWC.  Convolutions are implicit GEMMs over K = (ky*3 + kx)*Cin + ci
// (padded with zeros to a multiple of 32), reading the activation directly.
#include <hip/hip_runtime.h>

#include "ranker.h"
#include "spl_device.h"
#include "spl_internal.h"

#pragma clang fp contract(off)

namespace spl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ inline uint16_t f2bf(float f) {   // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ----------------------------------------------------------------- snippets
// One workgroup (256 threads) per candidate.  Plane 0: rows d*-32..d*+31 of the DM
// transform over t*-128..t*+127 (thread = column), each row standardised by the search's
// own (mu, sigma) of the segment of t*.  Plane 1: 64 sub-bands of nch/64 adjacent
// channels summed along the delays of trial d*, each standardised over its valid samples
// with the same exact-moment recipe.  Values float((v - mu)/sigma) in binary64 -> BF16;
// entries outside the DM range or outside [0, n_dd) are 0.
// Plane 1 work split: thread (g = tid / 16, q = tid % 16) adds samples 16q .. 16q+15 of
// channels g, g+16, ... of a sub-band, reading each channel's 16 bytes as five aligned
// dwords and accumulating them as 16-bit pairs (as the dedispersion kernel does); the 16
// channel groups are then summed through the LDS.
__global__ __launch_bounds__(256) void k_snippets(const DevBeam *__restrict__ beams, int nbeams,
                                                  const spl_candidate *__restrict__ cands, int64_t n,
                                                  uint16_t *__restrict__ out) {
    constexpr uint32_t kSelEven = 0x0C020C00u;   // bytes 0, 2 -> 16-bit fields
    constexpr uint32_t kSelOdd = 0x0C030C01u;    // bytes 1, 3 -> 16-bit fields
    __shared__ int32_t red[16][256];
    __shared__ int64_t sh[3][4];
    const int col = threadIdx.x, lane = lane_id(), wave = wave_id();
    const int g = col >> 4, q = col & 15;
    for (int64_t c = blockIdx.x; c < n; c += gridDim.x) {
        const spl_candidate cd = cands[c];
        uint16_t *o0 = out + (size_t)c * 2 * 64 * 256;
        uint16_t *o1 = o0 + 64 * 256;
        // a record that names no (beam, trial, owned sample) of this batch gives zero planes
        const bool ok = cd.beam >= 0 && cd.beam < nbeams && cd.dm_index >= 0 &&
                        cd.dm_index < beams[cd.beam < 0 || cd.beam >= nbeams ? 0 : cd.beam].ndm &&
                        cd.t_sample >= 0 &&
                        cd.t_sample < beams[cd.beam < 0 || cd.beam >= nbeams ? 0 : cd.beam].n_out;
        if (!ok) {
            for (int r = 0; r < 128; ++r) o0[r * 256 + col] = 0;
            continue;   // uniform across the workgroup: no barrier is skipped by part of it
        }
        const DevBeam &B = beams[cd.beam];
        const int ds = cd.dm_index, ts = cd.t_sample;
        const int t = ts - 128 + col;
        const bool valid = t >= 0 && t < B.n_dd;
        const int seg = ts / B.L;
        for (int r = 0; r < 64; ++r) {
            const int d = ds - 32 + r;
            float v = 0.f;
            if (valid && d >= 0 && d < B.ndm) {
                const size_t idx = (size_t)d * B.nseg + seg;
                const double sg = B.sigma[idx];
                if (sg > 0.0) v = (float)(((double)B.X[(size_t)d * B.xpitch + t] - B.mu[idx]) / sg);
            }
            o0[r * 256 + col] = f2bf(v);
        }
        const int per = B.nch / 64;
        const int32_t *drow = B.delays + (size_t)ds * B.nch;
        const int ta = ts - 128 + 16 * q;   // the thread's first sample of plane 1
        const bool all_valid = ta >= 0 && ta + 15 < B.n_dd;
        const bool any_valid = ta + 15 >= 0 && ta < B.n_dd;
        for (int k = 0; k < 64; ++k) {
            uint32_t ae[4] = {0u, 0u, 0u, 0u}, ao[4] = {0u, 0u, 0u, 0u};
            if (any_valid) {
                for (int ch = k * per + g; ch < (k + 1) * per; ch += 16) {
                    const uint8_t *row = B.x + (size_t)ch * B.pitch;
                    const int64_t off = (int64_t)ta + drow[ch];
                    uint32_t d4[4];
                    if (all_valid && (off & ~(int64_t)3) + 20 <= B.pitch) {
                        const uint32_t *w = (const uint32_t *)(row + (off & ~(int64_t)3));
                        const uint32_t w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3], w4 = w[4];
                        const uint32_t sa = (uint32_t)(off & 3);
                        d4[0] = __builtin_amdgcn_alignbyte(w1, w0, sa);
                        d4[1] = __builtin_amdgcn_alignbyte(w2, w1, sa);
                        d4[2] = __builtin_amdgcn_alignbyte(w3, w2, sa);
                        d4[3] = __builtin_amdgcn_alignbyte(w4, w3, sa);
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            uint32_t v = 0u;
#pragma unroll
                            for (int b = 0; b < 4; ++b) {
                                const int tj = ta + 4 * i + b;
                                if (tj >= 0 && tj < B.n_dd) v |= (uint32_t)row[off + 4 * i + b] << (8 * b);
                            }
                            d4[i] = v;
                        }
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        ae[i] += __builtin_amdgcn_perm(d4[i], d4[i], kSelEven);
                        ao[i] += __builtin_amdgcn_perm(d4[i], d4[i], kSelOdd);
                    }
                }
            }
            __syncthreads();   // the previous sub-band's partial sums are no longer read
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                red[g][16 * q + 4 * i + 0] = (int32_t)(ae[i] & 0xFFFFu);
                red[g][16 * q + 4 * i + 2] = (int32_t)(ae[i] >> 16);
                red[g][16 * q + 4 * i + 1] = (int32_t)(ao[i] & 0xFFFFu);
                red[g][16 * q + 4 * i + 3] = (int32_t)(ao[i] >> 16);
            }
            __syncthreads();
            int32_t sv = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) sv += red[j][col];
            // exact moments of the sub-band over the valid columns
            int64_t s1 = valid ? (int64_t)sv : 0, s2 = valid ? (int64_t)sv * sv : 0, nv = valid ? 1 : 0;
            s1 = wave_sum(s1);
            s2 = wave_sum(s2);
            nv = wave_sum(nv);
            if (lane == 0) {
                sh[0][wave] = s1;
                sh[1][wave] = s2;
                sh[2][wave] = nv;
            }
            __syncthreads();
            const int64_t S1 = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
            const int64_t S2 = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
            const int64_t NV = sh[2][0] + sh[2][1] + sh[2][2] + sh[2][3];
            double mu = 0.0, sg = 0.0;
            if (NV > 0) mu_sigma(NV, S1, S2, mu, sg);
            float v = 0.f;
            if (valid && sg > 0.0) v = (float)(((double)sv - mu) / sg);
            o1[k * 256 + col] = f2bf(v);
        }
        __syncthreads();   // sh and red are reused by the next candidate
    }
}

// ------------------------------------------------------- fine-DM DM-time plane
// Plane 0 replaced by the DM transform at 64 DMs DM* + (r - 32) * dDM/32 around the
// candidate's trial DM, dDM the half-range at which a Gaussian pulse of the candidate's
// width keeps `keep` of its S/N (Eq. snrlossapprox with zeta of Eq. zetadef; the paper's
// Eq. deltadm with its unit conversion corrected): dDM = (sqrt(pi)/2 / keep) * W_ms *
// nu_GHz^3 / (6.91e-3 * B_MHz), nu the band centre, B = nch * |foff|.  Delays follow
// Eq. (1) exactly as the plan computes them (binary64, same order, round half away).
// Entry (r, t) sums the block over all channels at t*-128+t plus the row's delays; it is
// valid when every channel's sample lies in [0, n_in) (the extremes are the channels of
// the highest and lowest frequency).  The plane is standardised by the exact moments
// of its valid entries (one mu, sigma for all rows, so the S/N falling off away from
// DM* stays visible), float((v - mu)/sigma) in binary64 -> BF16, invalid entries 0.
// One workgroup of 1024 threads per candidate: thread (g = tid/64, q = tid%64) owns
// samples 4q .. 4q+3 of rows g, g+16, g+32, g+48.  Channels go in chunks of 8: the
// delays of the 64 rows are computed into the LDS, then each channel's window of the
// block (the 256 samples plus the spread of its 64 delays) is staged as four copies
// shifted by 0..3 bytes, so every 4-sample read of any row is one aligned LDS dword
// (a wave's 64 lanes read 64 consecutive dwords: no bank conflicts).  The three steps
// are pipelined over chunks (sums of chunk k, staging of k+1, delays of k+2) with one
// barrier per chunk, so the waves of the one workgroup a CU holds overlap them.  Windows wider
// than the staging buffer (wide pulses: dDM grows with the width) are read from the
// block directly, two aligned dwords per 4 samples.  Sums go through 16-bit pairs,
// flushed before they exceed 256 channels (< 2^16).
constexpr int kFineChunk = 8;
constexpr int kFineWords = 512;   // staged dwords per channel and copy (window <= 2 KiB)

__device__ inline int64_t fine_delay(double dd, double k, double tsamp) {
    const double v = (dd * k) / tsamp;
    if (!(fabs(v) < 1.0e9)) return v > 0 ? (int64_t)1 << 40 : -((int64_t)1 << 40);
    return llround(v);
}

__device__ inline uint32_t block_dword(const uint8_t *row, int64_t t, int64_t n_in) {
    if (t >= 0 && t + 4 <= n_in) return *(const uint32_t *)(row + t);   // t is a multiple of 4 here
    uint32_t v = 0u;
#pragma unroll
    for (int b = 0; b < 4; ++b)
        if (t + b >= 0 && t + b < n_in) v |= (uint32_t)row[t + b] << (8 * b);
    return v;
}

__global__ __launch_bounds__(1024) void k_fine_dm(const DevBeam *__restrict__ beams, int nbeams,
                                                  const spl_candidate *__restrict__ cands, int64_t n, double keep,
                                                  uint16_t *__restrict__ out) {
    constexpr uint32_t kSelEven = 0x0C020C00u;
    constexpr uint32_t kSelOdd = 0x0C030C01u;
    constexpr double kD = 4148.8064239;   // Eq. (1), MHz^2 pc^-1 cm^3 s
    // three-stage pipeline over channel chunks: while chunk k is summed from stage buffer
    // k&1, chunk k+1 is staged into the other buffer and the delays of chunk k+2 are
    // computed into delay set (k+2)%3; one barrier per chunk
    __shared__ uint32_t stage[2][kFineChunk][4][kFineWords];
    __shared__ int32_t sdel[3][64][kFineChunk];
    __shared__ int64_t sgs[3][kFineChunk];
    __shared__ int32_t snw[3][kFineChunk];
    __shared__ int64_t sh[3][16];
    const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
    const int g = tid >> 6, q = tid & 63;
    for (int64_t ci = blockIdx.x; ci < n; ci += gridDim.x) {
        const spl_candidate cd = cands[ci];
        uint16_t *o0 = out + (size_t)ci * 2 * 64 * 256;
        const int bsafe = cd.beam < 0 || cd.beam >= nbeams ? 0 : cd.beam;
        const bool ok = cd.beam >= 0 && cd.beam < nbeams && cd.dm_index >= 0 && cd.dm_index < beams[bsafe].ndm &&
                        cd.t_sample >= 0 && cd.t_sample < beams[bsafe].n_out && cd.width >= 1;
        if (!ok) {   // both planes zero (plane 1 was written by the snippet kernel before)
            for (int e = tid; e < 2 * 64 * 256; e += 1024) o0[e] = 0;
            continue;   // uniform across the workgroup
        }
        const DevBeam &B = beams[cd.beam];
        const double w_ms = ((double)cd.width * B.tsamp) * 1000.0;
        const double nu = ((B.fref + B.flo) * 0.5) / 1000.0;
        const double bw = (double)B.nch * fabs(B.foff);
        const double half = (((0.88622692545275801365 / keep) * w_ms) * ((nu * nu) * nu)) / (6.91e-3 * bw);
        const double step = half / 32.0;
        const double dm_star = B.dms[cd.dm_index];
        const double k_lo = (1.0 / (B.flo * B.flo)) - (1.0 / (B.fref * B.fref));
        const int64_t t_first = (int64_t)cd.t_sample - 128;   // sample of column 0
        const int64_t ta = t_first + 4 * q;                    // the thread's first sample
        // bit 4i + j: sample j (0..3) of row g + 16i is valid (ta + j + smin >= 0 and
        // ta + j + smax < n_in, the extremes of the row's delays)
        uint32_t vmask = 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = g + 16 * i;
            const int64_t s_lo = fine_delay(kD * (dm_star + (double)(r - 32) * step), k_lo, B.tsamp);
            const int64_t smin = s_lo < 0 ? s_lo : 0, smax = s_lo > 0 ? s_lo : 0;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (ta + j + smin >= 0 && ta + j + smax < (int64_t)B.n_in) vmask |= 1u << (4 * i + j);
        }
        const int nchunks = (B.nch + kFineChunk - 1) / kFineChunk;

        // delays of chunk `chunk` into set `set`: wavefront w (< kFineChunk) takes channel
        // w, lane = row (Eq. (1) as a plan computes it).  The delays are monotone in the
        // row, so rows 0 and 63 bound the channel's window; each lane then stores its
        // row's LDS byte offset into the staged copies ((rel & 3) selects the copy,
        // rel >> 2 the dword, rel = t_first + delay - window start), or the raw delay when
        // the channel is read from the block (window too wide, or any offset out of range)
        auto delays = [&](int chunk, int set) {
            const int cc = wave, rr = lane;
            const int c0 = chunk * kFineChunk, nc = min(kFineChunk, B.nch - c0);
            const double f = B.fch1 + (double)(c0 + cc) * B.foff;
            const double kc = cc < nc ? (1.0 / (f * f)) - (1.0 / (B.fref * B.fref)) : 0.0;
            const int64_t sv = fine_delay(kD * (dm_star + (double)(rr - 32) * step), kc, B.tsamp);
            const int64_t s0 = __shfl(sv, 0), s63 = __shfl(sv, 63);
            const int64_t lo = s0 < s63 ? s0 : s63, hi = s0 < s63 ? s63 : s0;
            const int64_t gs = (t_first + lo) & ~(int64_t)3;
            const int64_t nw = ((t_first + 252 + hi - gs) >> 2) + 1;   // dwords holding every read
            const int64_t rel = t_first + sv - gs;
            const bool bad = rel < 0 || (rel >> 2) + 63 > nw - 1;
            const bool staged = cc < nc && nw + 1 <= kFineWords && !__any(bad);
            sdel[set][rr][cc] =
                staged ? (int32_t)(cc * (4 * kFineWords * 4) + (int)(rel & 3) * (kFineWords * 4) + (int)(rel >> 2) * 4)
                       : (int32_t)(sv > (1 << 30) ? (1 << 30) : (sv < -(1 << 30) ? -(1 << 30) : sv));
            if (lane == 0) {
                sgs[set][cc] = gs;
                snw[set][cc] = staged ? (int32_t)nw : 0;   // 0: read the block
            }
        };
        // the window of every channel of chunk `chunk` as four byte-shifted copies
        auto stage_chunk = [&](int chunk, int set, int buf) {
            const int c0 = chunk * kFineChunk;
            for (int e = tid; e < kFineChunk * kFineWords; e += 1024) {
                const int cc = e / kFineWords, i = e % kFineWords;
                if (i < snw[set][cc]) {
                    const uint8_t *row = B.x + (size_t)(c0 + cc) * B.pitch;
                    const int64_t t = sgs[set][cc] + 4 * (int64_t)i;
                    const uint32_t w0 = block_dword(row, t, B.n_in), w1 = block_dword(row, t + 4, B.n_in);
                    stage[buf][cc][0][i] = w0;
                    stage[buf][cc][1][i] = __builtin_amdgcn_alignbyte(w1, w0, 1);
                    stage[buf][cc][2][i] = __builtin_amdgcn_alignbyte(w1, w0, 2);
                    stage[buf][cc][3][i] = __builtin_amdgcn_alignbyte(w1, w0, 3);
                }
            }
        };

        int32_t acc[4][4];
        uint32_t ae[4], ao[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ae[i] = ao[i] = 0u;
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = 0;
        }
        int pending = 0;   // channels in the 16-bit pair sums

        if (wave < kFineChunk) {
            delays(0, 0);
            if (nchunks > 1) delays(1, 1);
        }
        __syncthreads();
        stage_chunk(0, 0, 0);
        __syncthreads();
        for (int k = 0; k < nchunks; ++k) {
            const int set = k % 3, buf = k & 1;
            const int c0 = k * kFineChunk, nc = min(kFineChunk, B.nch - c0);
            if (pending + nc > 256) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    acc[i][0] += (int32_t)(ae[i] & 0xFFFFu);
                    acc[i][2] += (int32_t)(ae[i] >> 16);
                    acc[i][1] += (int32_t)(ao[i] & 0xFFFFu);
                    acc[i][3] += (int32_t)(ao[i] >> 16);
                    ae[i] = ao[i] = 0u;
                }
                pending = 0;
            }
            pending += nc;
            for (int cc = 0; cc < nc; ++cc) {
                const int nw = snw[set][cc];   // the same for the whole workgroup
                if (nw > 0) {
                    const uint8_t *lbase = (const uint8_t *)&stage[buf][0][0][0] + 4 * q;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint32_t word = *(const uint32_t *)(lbase + sdel[set][g + 16 * i][cc]);
                        ae[i] += __builtin_amdgcn_perm(word, word, kSelEven);
                        ao[i] += __builtin_amdgcn_perm(word, word, kSelOdd);
                    }
                } else {
                    const uint8_t *row = B.x + (size_t)(c0 + cc) * B.pitch;
                    for (int i = 0; i < 4; ++i) {
                        const int64_t t = ta + sdel[set][g + 16 * i][cc];
                        const int64_t t4 = t & ~(int64_t)3;
                        const uint32_t word = __builtin_amdgcn_alignbyte(block_dword(row, t4 + 4, B.n_in),
                                                                         block_dword(row, t4, B.n_in),
                                                                         (uint32_t)(t & 3));
                        ae[i] += __builtin_amdgcn_perm(word, word, kSelEven);
                        ao[i] += __builtin_amdgcn_perm(word, word, kSelOdd);
                    }
                }
            }
            if (k + 1 < nchunks) stage_chunk(k + 1, (k + 1) % 3, (k + 1) & 1);
            if (k + 2 < nchunks && wave < kFineChunk) delays(k + 2, (k + 2) % 3);
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            acc[i][0] += (int32_t)(ae[i] & 0xFFFFu);
            acc[i][2] += (int32_t)(ae[i] >> 16);
            acc[i][1] += (int32_t)(ao[i] & 0xFFFFu);
            acc[i][3] += (int32_t)(ao[i] >> 16);
        }
        // exact moments of the plane's valid entries
        int64_t s1 = 0, s2 = 0, nv = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (vmask >> (4 * i + j) & 1u) {
                    s1 += acc[i][j];
                    s2 += (int64_t)acc[i][j] * acc[i][j];
                    nv += 1;
                }
            }
        }
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
        nv = wave_sum(nv);
        if (lane == 0) {
            sh[0][wave] = s1;
            sh[1][wave] = s2;
            sh[2][wave] = nv;
        }
        __syncthreads();
        int64_t S1 = 0, S2 = 0, NV = 0;
        for (int k = 0; k < 16; ++k) {
            S1 += sh[0][k];
            S2 += sh[1][k];
            NV += sh[2][k];
        }
        double mu = 0.0, sg = 0.0;
        if (NV > 0) mu_sigma(NV, S1, S2, mu, sg);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float v = 0.f;
                if ((vmask >> (4 * i + j) & 1u) && sg > 0.0) v = (float)(((double)acc[i][j] - mu) / sg);
                o0[(g + 16 * i) * 256 + 4 * q + j] = f2bf(v);
            }
        }
        __syncthreads();   // sh is reused by the next candidate
    }
}

// --------------------------------------------------------------------- GEMM
// C[M][N] (FP32, row stride ldc) = (mode 1: C +) A[M][K] * B[N][K]^T with A and B BF16,
// K contiguous, row strides lda/ldb multiples of 8, K a multiple of 32.  Workgroup =
// 4 wavefronts; wavefront w computes rows 64*bx + 16w .. +15 and columns 32*by .. +31
// (two 16x16 tiles); split z of gridDim.z covers K range [z*klen, (z+1)*klen) and adds
// atomically (mode 1).  MFMA operand lanes: lane l supplies A[l%16][8(l/16) .. +7] and
// B^T[l%16][8(l/16) .. +7] and receives D[4(l/16) + i][l%16].
__global__ __launch_bounds__(256) void k_gemm(const uint16_t *__restrict__ A, int64_t lda,
                                              const uint16_t *__restrict__ Bm, int64_t ldb, float *C, int64_t ldc,
                                              int M, int N, int K, int klen, int mode) {
    const int lane = lane_id(), wave = wave_id();
    const int m_base = blockIdx.x * 64 + wave * 16;
    const int n_base = blockIdx.y * 32;
    const int k_lo = blockIdx.z * klen, k_hi = min(K, k_lo + klen);
    const int arow = m_base + (lane & 15), kq = 8 * (lane >> 4);
    const int b0 = n_base + (lane & 15), b1 = b0 + 16;
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    const u16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k0 = k_lo; k0 < k_hi; k0 += 32) {
        const u16x8 a = arow < M ? *(const u16x8 *)(A + (size_t)arow * lda + k0 + kq) : zero;
        const u16x8 x0 = b0 < N ? *(const u16x8 *)(Bm + (size_t)b0 * ldb + k0 + kq) : zero;
        const u16x8 x1 = b1 < N ? *(const u16x8 *)(Bm + (size_t)b1 * ldb + k0 + kq) : zero;
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, x0),
                                                       acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, x1),
                                                       acc1, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m_base + 4 * (lane >> 4) + i;
        if (m >= M) continue;
        const int n0 = n_base + (lane & 15), n1 = n0 + 16;
        if (n0 < N) {
            if (mode) atomicAdd(&C[(size_t)m * ldc + n0], acc0[i]);
            else C[(size_t)m * ldc + n0] = acc0[i];
        }
        if (n1 < N) {
            if (mode) atomicAdd(&C[(size_t)m * ldc + n1], acc1[i]);
            else C[(size_t)m * ldc + n1] = acc1[i];
        }
    }
}

// ------------------------------------------------------- implicit-GEMM convolution
// Z[p][co] (FP32 [P][32]) = sum over taps t = ky*3 + kx and input channels ci of
// X[src(p, t)][ci] * Wt[co][t*32 + ci], without an im2col buffer: with 32 input channels
// each K-step of 32 is one tap, so the MFMA A operand of lane l is the 16 bytes of
// channels 8(l/16) .. +7 of one source pixel, read straight from the NHWC activation.
// MODE 0: the first layer: input NCHW with 2 channels (the snippet planes), K = 18 padded
//         to one K-step of 32 (k = t*2 + ci), images n >= nvalid read as zero.
// MODE 1: 32 input channels, NHWC, src = (h + ky - 1, w + kx - 1)   (forward).
// MODE 2: 32 input channels, NHWC, src = (h - ky + 1, w - kx + 1)   (input gradient: the
//         input is dZ and Wt the weights repacked as [ci][t*32 + co]).
// Workgroup = 4 wavefronts; each wavefront computes kConvTiles tiles of 16 pixels x all 32
// columns, so a tap's weight operands are loaded once for 64 pixels.  Tile T (of the
// wavefront's T0 .. T0+3) is pixels 16T .. 16T+15, or with POOL (forward only) a 2 x 8
// pixel patch (rows 2ph, 2ph+1, columns 8c .. 8c+7; patches row-major per image), so the
// result holds four whole 2 x 2 windows: lane l keeps rows 4(l/16) .. +3, i.e. two
// horizontal pairs of one image row, and lane l ^ 32 the pairs below them.  Bias, ReLU
// and the max pool (with the window position of the first maximum, 255 when no element
// is positive) then run in registers and only the pooled BF16 activation and the decision
// bytes are written.
constexpr int kConvTiles = 4;
template <int MODE, bool POOL>
__global__ __launch_bounds__(256) void k_conv(const uint16_t *__restrict__ X, int N, int nvalid, int H, int W,
                                              const uint16_t *__restrict__ Wt, int ldw, float *__restrict__ C,
                                              const float *__restrict__ bias, uint16_t *__restrict__ pooled,
                                              uint8_t *__restrict__ arg) {
    constexpr int MT = kConvTiles;
    const int lane = lane_id(), wave = wave_id();
    const int64_t P = (int64_t)N * H * W;
    const int64_t t0 = ((int64_t)blockIdx.x * 4 + wave) * MT;
    const int kq = 8 * (lane >> 4);
    const int per_row = W >> 3, per_img = (H >> 1) * per_row;
    int n[MT], h[MT], w[MT];
    bool row_ok[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int64_t tile = t0 + mt;
        int64_t p;
        if constexpr (POOL) {
            n[mt] = (int)(tile / per_img);
            const int rem = (int)(tile - (int64_t)n[mt] * per_img);
            const int r = lane & 15;
            h[mt] = 2 * (rem / per_row) + (r >> 3);
            w[mt] = 8 * (rem % per_row) + (r & 7);
            p = ((int64_t)n[mt] * H + h[mt]) * W + w[mt];
        } else {
            p = tile * 16 + (lane & 15);
            n[mt] = (int)(p / ((int64_t)H * W));
            const int hw = (int)(p - (int64_t)n[mt] * H * W);
            h[mt] = hw / W;
            w[mt] = hw - h[mt] * W;
        }
        row_ok[mt] = p < P && n[mt] < nvalid;
    }
    f32x4 acc0[MT], acc1[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc0[mt] = acc1[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const u16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
    const uint16_t *b0p = Wt + (size_t)(lane & 15) * ldw + kq;
    const uint16_t *b1p = b0p + (size_t)16 * ldw;
    if constexpr (MODE == 0) {
        u16x8 a[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) a[mt] = zero;
        if constexpr (POOL) {
            // the workgroup's 16 patches form one 2 x 128 strip of an image (W a multiple of
            // 128): its input window, 2 channels x 4 rows x 130 columns with the zero
            // padding, is staged in LDS once and every tap is read from there
            constexpr int kWc = 8 * 4 * MT + 2;
            __shared__ uint16_t win[2 * 4 * kWc];
            const int64_t tw = (int64_t)blockIdx.x * 4 * MT;
            const int n0 = (int)(tw / per_img);
            const int rem0 = (int)(tw - (int64_t)n0 * per_img);
            const int hb = 2 * (rem0 / per_row) - 1, wb = 8 * (rem0 % per_row) - 1;
            for (int i = threadIdx.x; i < 2 * 4 * kWc; i += 256) {
                const int ci = i / (4 * kWc), r = (i / kWc) & 3, c = i % kWc;
                const int hs = hb + r, ws = wb + c;
                uint16_t v = 0;
                if (n0 < nvalid && hs >= 0 && hs < H && ws >= 0 && ws < W)
                    v = X[(((size_t)n0 * 2 + ci) * H + hs) * W + ws];
                win[i] = v;
            }
            __syncthreads();
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int base = (h[mt] - hb) * kWc + (w[mt] - wb);   // the pixel's place in the window
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = kq + j;
                    if (k < 18) {
                        const int t = k >> 1, ci = k & 1;
                        const int ty = (t * 11) >> 5;        // t / 3 for t < 9
                        a[mt][j] = win[ci * 4 * kWc + base + (ty - 1) * kWc + (t - 3 * ty - 1)];
                    }
                }
            }
        } else {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = kq + j;
                    if (k < 18 && row_ok[mt]) {
                        const int t = k >> 1, ci = k & 1;
                        const int hs = h[mt] + t / 3 - 1, ws = w[mt] + t % 3 - 1;
                        if (hs >= 0 && hs < H && ws >= 0 && ws < W)
                            a[mt][j] = X[(((size_t)n[mt] * 2 + ci) * H + hs) * W + ws];
                    }
                }
        }
        const u16x8 x0 = *(const u16x8 *)b0p, x1 = *(const u16x8 *)b1p;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            acc0[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[mt]),
                                                               __builtin_bit_cast(bf16x8, x0), acc0[mt], 0, 0, 0);
            acc1[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[mt]),
                                                               __builtin_bit_cast(bf16x8, x1), acc1[mt], 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ky = t / 3, kx = t % 3;
            const u16x8 x0 = *(const u16x8 *)(b0p + 32 * t), x1 = *(const u16x8 *)(b1p + 32 * t);
            u16x8 a[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int hs = MODE == 1 ? h[mt] + ky - 1 : h[mt] - ky + 1;
                const int ws = MODE == 1 ? w[mt] + kx - 1 : w[mt] - kx + 1;
                a[mt] = zero;
                if (row_ok[mt] && hs >= 0 && hs < H && ws >= 0 && ws < W)
                    a[mt] = *(const u16x8 *)(X + (((size_t)n[mt] * H + hs) * W + ws) * 32 + kq);
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                acc0[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[mt]),
                                                                   __builtin_bit_cast(bf16x8, x0), acc0[mt], 0, 0, 0);
                acc1[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[mt]),
                                                                   __builtin_bit_cast(bf16x8, x1), acc1[mt], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int64_t tile = t0 + mt;
        if constexpr (POOL) {
            // window k (0, 1) of this lane: own pair i = 2k, 2k+1 (window positions 0, 1),
            // the partner lane's pair below it (positions 2, 3); positions tried in order
            const int g = lane >> 4, co = lane & 15;
            const int nn = (int)(tile / per_img);
            const int rem = (int)(tile - (int64_t)nn * per_img);
            const int ph = rem / per_row, pw0 = 4 * (rem % per_row) + 2 * (g & 1);
            const int H2 = H >> 1, W2 = W >> 1;
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const f32x4 av = half ? acc1[mt] : acc0[mt];
                const float b = bias[co + 16 * half];
                float below[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) below[i] = __shfl_xor(av[i], 32);
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const float z[4] = {av[2 * k] + b, av[2 * k + 1] + b, below[2 * k] + b, below[2 * k + 1] + b};
                    float best = 0.f;
                    int ba = 255;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if (z[j] > best) {
                            best = z[j];
                            ba = j;
                        }
                    }
                    if (g < 2 && tile * 16 < P) {
                        const size_t o = (((size_t)nn * H2 + ph) * W2 + pw0 + k) * 32 + co + 16 * half;
                        pooled[o] = f2bf(best);
                        arg[o] = (uint8_t)ba;
                    }
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t m = tile * 16 + 4 * (lane >> 4) + i;
                if (m >= P) continue;
                C[m * 32 + (lane & 15)] = acc0[mt][i];
                C[m * 32 + 16 + (lane & 15)] = acc1[mt][i];
            }
        }
    }
}

// ------------------------------------------------------- weight gradient (LDS)
// part[blockIdx.x][k][co] (FP32 [gridDim.x][288][32]) = sum over the pixels p of the
// workgroup's slabs of A[p][k] * dZ[p][co], A the (implicit) im2col of the layer input:
// k = t*32 + ci (32 input channels, NHWC).  A slab is 32 consecutive pixels (the MFMA
// K-step); its dZ and the 9 shifted input tiles are staged transposed in LDS
// ([channel][pixel]) so that MFMA operands are 16-byte LDS reads.  Tiles of the 288 x 32
// result (9 taps x 2 x 2 of 16 x 16) are spread over the 4 waves.
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t *__restrict__ X, int N, int H, int W,
                                               const uint16_t *__restrict__ dZ, float *__restrict__ part) {
    constexpr int kTiles = 36;                           // 16x16 tiles of the K x 32 result
    constexpr int kPerWave = kTiles / 4;
    constexpr int kRows = 9 * 32;                        // staged A^T rows
    constexpr int kLd = 40;                              // LDS row stride (elements), 80 bytes
    __shared__ __align__(16) uint16_t sA[kRows * kLd];
    __shared__ __align__(16) uint16_t sZ[32 * kLd];
    const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
    const uint32_t HW = (uint32_t)(H * W);
    const uint32_t nslab = (uint32_t)N * HW / 32u;       // N H W is a multiple of 32 (< 2^31)
    f32x4 acc[kPerWave];
#pragma unroll
    for (int i = 0; i < kPerWave; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kq = 8 * (lane >> 4);
    // thread -> (pixel tid/8, channels 4*(tid%8) .. +3) of a slab; the next slab's dZ and
    // nine input tiles are loaded into registers while the current one is multiplied
    const int px = tid >> 3, c4 = (tid & 7) * 4;
    uint64_t vz = 0, va[9];
    auto load = [&](uint32_t sl) {
        const uint32_t p = sl * 32u + (uint32_t)px;
        vz = *(const uint64_t *)(dZ + (size_t)p * 32 + c4);
        const uint32_t n = p / HW, hw = p - n * HW, h = hw / (uint32_t)W, w = hw - h * (uint32_t)W;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int hs = (int)h + t / 3 - 1, ws = (int)w + t % 3 - 1;
            va[t] = 0;
            if (hs >= 0 && hs < H && ws >= 0 && ws < W)
                va[t] = *(const uint64_t *)(X + (((size_t)n * H + hs) * W + ws) * 32 + c4);
        }
    };
    uint32_t sl = blockIdx.x;
    if (sl < nslab) load(sl);
    for (; sl < nslab; sl += gridDim.x) {
#pragma unroll
        for (int i = 0; i < 4; ++i) sZ[(c4 + i) * kLd + px] = (uint16_t)(vz >> (16 * i));
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) sA[(t * 32 + c4 + i) * kLd + px] = (uint16_t)(va[t] >> (16 * i));
        __syncthreads();
        if (sl + gridDim.x < nslab) load(sl + gridDim.x);
#pragma unroll
        for (int i = 0; i < kPerWave; ++i) {
            const int tile = wave + 4 * i;
            const int it = tile >> 1, jt = tile & 1;   // A^T row tile (16 rows of k), dZ^T row tile (co)
            const u16x8 a = *(const u16x8 *)(sA + (it * 16 + (lane & 15)) * kLd + kq);
            const u16x8 b = *(const u16x8 *)(sZ + (jt * 16 + (lane & 15)) * kLd + kq);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                             __builtin_bit_cast(bf16x8, b), acc[i], 0, 0, 0);
        }
        __syncthreads();
    }
    float *out = part + (size_t)blockIdx.x * kRows * 32;
#pragma unroll
    for (int i = 0; i < kPerWave; ++i) {
        const int tile = wave + 4 * i;
        const int it = tile >> 1, jt = tile & 1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = it * 16 + 4 * (lane >> 4) + r;
            out[(size_t)k * 32 + jt * 16 + (lane & 15)] = acc[i][r];
        }
    }
}

// Weight gradient of the first layer (2 input channels, K = 18 used of 32):
// part[blockIdx.x][k][co] = sum over the pixels p of the workgroup's slabs of
// A[p][k] * dZ[p][co], k = t*2 + ci.  Each wavefront works alone on slabs of 32
// consecutive pixels of one image row (W a multiple of 32): the input is NCHW, so the 32
// values of row k are 32 neighbouring samples of one plane (shifted by the tap), read
// straight into the LDS row; dZ (NHWC) is transposed into its LDS rows.  No workgroup
// barrier in the loop: a wavefront's LDS writes and reads execute in order.  The four
// wavefronts' sums are added in a fixed order at the end.
__global__ __launch_bounds__(256) void k_wgrad_first(const uint16_t *__restrict__ X, int N, int nvalid, int H,
                                                     int W, const uint16_t *__restrict__ dZ,
                                                     float *__restrict__ part) {
    constexpr int kLd = 40;
    __shared__ __align__(16) uint16_t lds[2 * 4 * 32 * kLd];   // per wave: A rows, then dZ^T rows
    const int lane = lane_id(), wave = wave_id();
    uint16_t *A = lds + wave * 2 * 32 * kLd, *Zt = A + 32 * kLd;
    for (int i = lane; i < 32 * kLd; i += 64) A[i] = 0;   // rows 18..31 stay zero
    __builtin_amdgcn_wave_barrier();
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint32_t HW = (uint32_t)(H * W);
    const uint32_t nslab = (uint32_t)N * HW / 32u;
    const uint32_t nwaves = gridDim.x * 4u;
    const int kq = 8 * (lane >> 4);
    // lane -> dZ: pixel lane/2, channels 16*(lane%2) .. +15; A: pixel lane%32, channel
    // lane/32, all nine taps.  The next slab is loaded into registers while the current
    // one is multiplied.
    const int zpx = lane >> 1, zc0 = 16 * (lane & 1);
    const int apx = lane & 31, aci = lane >> 5;
    uint4 z0, z1;
    uint16_t av[9];
    auto load = [&](uint32_t sl) {
        const uint32_t p0 = sl * 32u;
        const uint4 *src = (const uint4 *)(dZ + ((size_t)p0 + zpx) * 32 + zc0);
        z0 = src[0];
        z1 = src[1];
        const uint32_t n = p0 / HW, rem = p0 - n * HW, h = rem / (uint32_t)W, w0 = rem - h * (uint32_t)W;
        const bool img_ok = (int)n < nvalid;
        const uint16_t *plane = X + ((size_t)n * 2 + aci) * HW;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int hs = (int)h + t / 3 - 1, ws = (int)w0 + apx + t % 3 - 1;
            av[t] = (img_ok && hs >= 0 && hs < H && ws >= 0 && ws < W) ? plane[(size_t)hs * W + ws] : (uint16_t)0;
        }
    };
    uint32_t sl = blockIdx.x * 4u + (uint32_t)wave;
    if (sl < nslab) load(sl);
    for (; sl < nslab; sl += nwaves) {
        const uint32_t w[8] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w};
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            Zt[(zc0 + 2 * i) * kLd + zpx] = (uint16_t)(w[i] & 0xFFFFu);
            Zt[(zc0 + 2 * i + 1) * kLd + zpx] = (uint16_t)(w[i] >> 16);
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) A[(2 * t + aci) * kLd + apx] = av[t];
        __builtin_amdgcn_wave_barrier();
        if (sl + nwaves < nslab) load(sl + nwaves);
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const u16x8 a = *(const u16x8 *)(A + (it * 16 + (lane & 15)) * kLd + kq);
#pragma unroll
            for (int jt = 0; jt < 2; ++jt) {
                const u16x8 b = *(const u16x8 *)(Zt + (jt * 16 + (lane & 15)) * kLd + kq);
                acc[it][jt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                                      __builtin_bit_cast(bf16x8, b), acc[it][jt], 0,
                                                                      0, 0);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    // the four wavefronts' sums, added in a fixed order (the staging area is reused)
    __syncthreads();
    float *red = (float *)lds;   // [4 waves][4 tiles][4][64]: 16 KiB of the 20 KiB
#pragma unroll
    for (int it = 0; it < 2; ++it)
#pragma unroll
        for (int jt = 0; jt < 2; ++jt)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[((wave * 4 + 2 * it + jt) * 4 + r) * 64 + lane] = acc[it][jt][r];
    __syncthreads();
    if (wave == 0) {
        float *out = part + (size_t)blockIdx.x * 32 * 32;
#pragma unroll
        for (int tl = 0; tl < 4; ++tl)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float v = ((red[((0 * 4 + tl) * 4 + r) * 64 + lane] + red[((1 * 4 + tl) * 4 + r) * 64 + lane]) +
                                 red[((2 * 4 + tl) * 4 + r) * 64 + lane]) + red[((3 * 4 + tl) * 4 + r) * 64 + lane];
                const int it = tl >> 1, jt = tl & 1;
                const int k = it * 16 + 4 * (lane >> 4) + r;
                out[(size_t)k * 32 + jt * 16 + (lane & 15)] = v;
            }
    }
}

// out[g][i] = sum over the parts j of group g (j in [g*group, min((g+1)*group, nparts)),
// g = blockIdx.y) of part[j][i], i < n, in a fixed order (deterministic).  Workgroup =
// 16 wavefronts over 64 consecutive i: wavefront w adds the group's parts w, w+16, ...
// (eight loads in flight), then the 16 partial sums of each i are added in order through
// the LDS.
__global__ __launch_bounds__(1024) void k_sum_parts(const float *__restrict__ part, int nparts, int group, int64_t n,
                                                    float *__restrict__ out) {
    __shared__ float red[16][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    const int j0 = blockIdx.y * group, j1 = min(nparts, j0 + group);
    float s = 0.f;
    if (i < n) {
        int j = j0 + g;
        for (; j + 16 * 7 < j1; j += 16 * 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(j + 16 * u) * n + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; j < j1; j += 16) s += part[(size_t)j * n + i];
    }
    red[g][lane] = s;
    __syncthreads();
    if (g == 0 && i < n) {
        float t = 0.f;
#pragma unroll
        for (int k = 0; k < 16; ++k) t += red[k][lane];
        out[(size_t)blockIdx.y * n + i] = t;
    }
}

// Transpose of a BF16 matrix: out[c][r] = in[r][c] (rows x cols, row strides ldi/ldo).
__global__ void k_transpose16(const uint16_t *__restrict__ in, int64_t rows, int64_t cols, int64_t ldi,
                              uint16_t *__restrict__ out, int64_t ldo) {
    __shared__ uint16_t tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;   // rows on x (the long side)
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
    for (int j = ty; j < 32; j += 8) {
        const int64_t r = r0 + j, c = c0 + tx;
        tile[j][tx] = (r < rows && c < cols) ? in[r * ldi + c] : (uint16_t)0;
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int64_t c = c0 + j, r = r0 + tx;
        if (c < cols && r < rows) out[c * ldo + r] = tile[tx][j];
    }
}

// Gradient through pool + ReLU: dZ[p][co] = dOut[pooled][co] at the window's arg position,
// 0 elsewhere (BF16 [P][32]); the bias gradient (the sum of dOut over windows with a
// chosen element) is accumulated.  Thread = one pooled pixel and 8 channels: two 16-byte
// loads of dOut, one 8-byte load of the decisions, four 16-byte stores (one per window
// position).  Bias partial sums are reduced over the wavefront's lanes of the same
// channel group, then over the workgroup in the LDS, then added to dbias.
__global__ __launch_bounds__(256) void k_unpool(const float *__restrict__ dOut, const uint8_t *__restrict__ arg,
                                                int N, int H, int W, uint16_t *__restrict__ dZ,
                                                float *__restrict__ dbias) {
    __shared__ float sb[4][32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int H2 = H >> 1, W2 = W >> 1;
    const uint32_t per_img = (uint32_t)(H2 * W2);
    const uint32_t nq = (uint32_t)N * per_img;          // pooled pixels (< 2^31)
    const int grp = lane & 3;                           // channels 8 grp .. 8 grp + 7
    float part[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) part[c] = 0.f;
    const uint32_t stride = gridDim.x * 64u;
    for (uint32_t q = blockIdx.x * 64u + (uint32_t)(threadIdx.x >> 2); q < nq; q += stride) {
        const float4 g0 = *(const float4 *)(dOut + (size_t)q * 32 + 8 * grp);
        const float4 g1 = *(const float4 *)(dOut + (size_t)q * 32 + 8 * grp + 4);
        const uint2 av = *(const uint2 *)(arg + (size_t)q * 32 + 8 * grp);
        const float g[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
        uint32_t a[8];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            a[c] = (av.x >> (8 * c)) & 0xFFu;
            a[c + 4] = (av.y >> (8 * c)) & 0xFFu;
        }
        uint16_t b[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            b[c] = f2bf(g[c]);
            if (a[c] != 255u) part[c] += g[c];
        }
        const uint32_t n = q / per_img, hw = q - n * per_img, h2 = hw / (uint32_t)W2, w2 = hw - h2 * (uint32_t)W2;
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            uint32_t w[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t lo = a[2 * c] == j ? b[2 * c] : 0u;
                const uint32_t hi = a[2 * c + 1] == j ? b[2 * c + 1] : 0u;
                w[c] = lo | (hi << 16);
            }
            const size_t p = ((size_t)n * H + 2 * h2 + (j >> 1)) * W + 2 * w2 + (j & 1);
            *(uint4 *)(dZ + p * 32 + 8 * grp) = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        float v = part[c];
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        part[c] = v;
    }
    if (lane < 4) {
#pragma unroll
        for (int c = 0; c < 8; ++c) sb[wave][8 * lane + c] = part[c];
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        const float t = sb[0][threadIdx.x] + sb[1][threadIdx.x] + sb[2][threadIdx.x] + sb[3][threadIdx.x];
        atomicAdd(&dbias[threadIdx.x], t);
    }
}

// --------------------------------------------------- fully connected head (VALU)
// H [Nb][64] FP32 (GEMM output), b1, f2w, f2b -> logits; with labels: mean BCE loss,
// gradients of f2w, f2b, b1 and dH (BF16 [Nb][64] and transposed [64][ldT]).  One
// workgroup of 1024 threads; rows n >= N (batch padding) produce zero gradients.  Sums
// over the candidates run in a fixed order: per hidden unit j, 16 threads add every 16th
// candidate and their partial sums are added in order.
__global__ __launch_bounds__(1024) void k_head(const float *__restrict__ Hm, const float *__restrict__ b1,
                                               const float *__restrict__ f2w, const float *__restrict__ f2b, int N,
                                               int Nb, float *__restrict__ logits, const float *__restrict__ labels,
                                               float *__restrict__ loss, float *__restrict__ g_f2w,
                                               float *__restrict__ g_f2b, float *__restrict__ g_b1,
                                               uint16_t *__restrict__ dH, uint16_t *__restrict__ dHT, int64_t ldT) {
    __shared__ float zl[1024];
    __shared__ float dl[1024];
    __shared__ float pw[16][64], pb[16][64];
    const int tid = threadIdx.x;
    for (int n = tid; n < Nb; n += 1024) {
        float z = 0.f;
        if (n < N) {
            z = f2b[0];
            for (int j = 0; j < 64; ++j) {
                const float h = fmaxf(Hm[(size_t)n * 64 + j] + b1[j], 0.f);
                z += f2w[j] * h;
            }
            logits[n] = z;
        }
        zl[n] = z;
    }
    if (!labels) return;
    __syncthreads();
    for (int n = tid; n < Nb; n += 1024) {
        float g = 0.f, l = 0.f;
        if (n < N) {
            const float z = zl[n], y = labels[n];
            l = fmaxf(z, 0.f) - z * y + log1pf(expf(-fabsf(z)));
            g = (1.f / (1.f + expf(-z)) - y) / (float)N;
        }
        dl[n] = g;
        zl[n] = l;
    }
    __syncthreads();
    {
        const int j = tid & 63, q = tid >> 6;
        float gw = 0.f, gb = 0.f;
        for (int n = q; n < N; n += 16) {
            const float pre = Hm[(size_t)n * 64 + j] + b1[j];
            gw += dl[n] * fmaxf(pre, 0.f);
            gb += pre > 0.f ? dl[n] * f2w[j] : 0.f;
        }
        pw[q][j] = gw;
        pb[q][j] = gb;
    }
    if (tid == 1023) {   // the loss and the output bias gradient: one thread, candidates in order
        float sl = 0.f, sg = 0.f;
        for (int n = 0; n < N; ++n) {
            sl += zl[n];
            sg += dl[n];
        }
        loss[0] = sl / (float)N;
        g_f2b[0] = sg;
    }
    __syncthreads();
    if (tid < 64) {
        float gw = 0.f, gb = 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            gw += pw[q][tid];
            gb += pb[q][tid];
        }
        g_f2w[tid] = gw;
        g_b1[tid] = gb;
    }
    for (int i = tid; i < Nb * 64; i += 1024) {
        const int n = i >> 6, j = i & 63;
        float g = 0.f;
        if (n < N) {
            const float pre = Hm[(size_t)n * 64 + j] + b1[j];
            g = pre > 0.f ? dl[n] * f2w[j] : 0.f;
        }
        const uint16_t v = f2bf(g);
        dH[i] = v;
        dHT[(size_t)j * ldT + n] = v;
    }
}

// Packed BF16 weights: out[i] = bf16(master[idx[i]]), 0 where idx[i] < 0.
__global__ void k_pack_idx(const float *__restrict__ master, const int32_t *__restrict__ idx, int64_t n,
                           uint16_t *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = idx[i];
        out[i] = k >= 0 ? f2bf(master[k]) : (uint16_t)0;
    }
}

// Gradients of packed weights back to the master layout: master[idx[i]] = in[i] (idx >= 0;
// every master index appears at most once).
__global__ void k_scatter_idx(const float *__restrict__ in, const int32_t *__restrict__ idx, int64_t n,
                              float *__restrict__ master) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = idx[i];
        if (k >= 0) master[k] = in[i];
    }
}

__global__ void k_zero_u16(uint16_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Adam on the FP32 master parameters (bias-corrected, step t >= 1).
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ void k_zero_f32(float *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

// ---------------------------------------------------------------- launchers
#define SPL_HIP_LAUNCH_CHECK() \
    do { hipError_t e__ = hipGetLastError(); if (e__ != hipSuccess) return e__; } while (0)

static unsigned grid_1d(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    return (unsigned)(g < 1 ? 1 : g);
}

hipError_t launch_snippets(const DevBeam *beams, int nbeams, const spl_candidate *cands, int64_t n, uint16_t *out,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)(n < 65536 ? n : 65536);
    hipLaunchKernelGGL(k_snippets, dim3(g), dim3(256), 0, s, beams, nbeams, cands, n, out);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_fine_dm(const DevBeam *beams, int nbeams, const spl_candidate *cands, int64_t n, double keep,
                          uint16_t *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)(n < 65536 ? n : 65536);
    hipLaunchKernelGGL(k_fine_dm, dim3(g), dim3(1024), 0, s, beams, nbeams, cands, n, keep, out);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_gemm(const uint16_t *A, int64_t lda, const uint16_t *B, int64_t ldb, float *C, int64_t ldc, int M,
                       int N, int K, int splits, bool accumulate, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0 || (K & 31) || (lda & 7) || (ldb & 7)) return hipErrorInvalidValue;
    if (splits < 1) splits = 1;
    int klen = (K / 32 + splits - 1) / splits * 32;
    splits = (K + klen - 1) / klen;
    dim3 grid((M + 63) / 64, (N + 31) / 32, splits);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, M, N, K, klen,
                       (accumulate || splits > 1) ? 1 : 0);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_conv(int mode, const uint16_t *X, int N, int nvalid, int H, int W, const uint16_t *Wt, int ldw,
                       float *C, hipStream_t s) {
    const int64_t P = (int64_t)N * H * W;
    if (P <= 0 || (ldw & 7)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((P + 64 * kConvTiles - 1) / (64 * kConvTiles)));
    float *nb = nullptr;
    uint16_t *np = nullptr;
    uint8_t *na = nullptr;
    if (mode == 0)
        hipLaunchKernelGGL((k_conv<0, false>), grid, dim3(256), 0, s, X, N, nvalid, H, W, Wt, ldw, C, nb, np, na);
    else if (mode == 1)
        hipLaunchKernelGGL((k_conv<1, false>), grid, dim3(256), 0, s, X, N, nvalid, H, W, Wt, ldw, C, nb, np, na);
    else
        hipLaunchKernelGGL((k_conv<2, false>), grid, dim3(256), 0, s, X, N, nvalid, H, W, Wt, ldw, C, nb, np, na);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_conv_pool(int mode, const uint16_t *X, int N, int nvalid, int H, int W, const uint16_t *Wt, int ldw,
                            const float *bias, uint16_t *pooled, uint8_t *arg, hipStream_t s) {
    const int64_t P = (int64_t)N * H * W;
    // whole 2 x 8 patches, 4 x kConvTiles per workgroup
    if (P <= 0 || (ldw & 7) || (H & 1) || (W & 7) || (P % (64 * kConvTiles)) || (mode != 0 && mode != 1))
        return hipErrorInvalidValue;
    if (mode == 0 && (W % (32 * kConvTiles))) return hipErrorInvalidValue;   // a workgroup's strip stays in one row
    const dim3 grid((unsigned)(P / (64 * kConvTiles)));
    float *nc = nullptr;
    if (mode == 0)
        hipLaunchKernelGGL((k_conv<0, true>), grid, dim3(256), 0, s, X, N, nvalid, H, W, Wt, ldw, nc, bias, pooled,
                           arg);
    else
        hipLaunchKernelGGL((k_conv<1, true>), grid, dim3(256), 0, s, X, N, nvalid, H, W, Wt, ldw, nc, bias, pooled,
                           arg);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_wgrad(int mode, const uint16_t *X, int N, int nvalid, int H, int W, const uint16_t *dZ, float *part,
                        int nparts, hipStream_t s) {
    const int64_t P = (int64_t)N * H * W;
    if (P <= 0 || (P & 31) || nparts < 1) return hipErrorInvalidValue;
    if (mode == 0) {
        if ((W & 31) || (int64_t)N * H * W >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_wgrad_first, dim3(nparts), dim3(256), 0, s, X, N, nvalid, H, W, dZ, part);
    } else {
        hipLaunchKernelGGL(k_wgrad, dim3(nparts), dim3(256), 0, s, X, N, H, W, dZ, part);
    }
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_sum_parts(const float *part, int nparts, int64_t n, float *out, float *tmp, hipStream_t s) {
    const unsigned gx = (unsigned)((n + 63) / 64);
    if (nparts <= 256) {
        hipLaunchKernelGGL(k_sum_parts, dim3(gx), dim3(1024), 0, s, part, nparts, nparts, n, out);
        SPL_HIP_LAUNCH_CHECK();
        return hipSuccess;
    }
    // two passes: groups of 128 parts into tmp [groups][n], then the groups
    const int groups = (nparts + 127) / 128;
    if (groups > kSumPartsMaxGroups) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sum_parts, dim3(gx, (unsigned)groups), dim3(1024), 0, s, part, nparts, 128, n, tmp);
    SPL_HIP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_parts, dim3(gx), dim3(1024), 0, s, (const float *)tmp, groups, groups, n, out);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_transpose16(const uint16_t *in, int64_t rows, int64_t cols, int64_t ldi, uint16_t *out, int64_t ldo,
                              hipStream_t s) {
    if ((cols + 31) / 32 > 65535) return hipErrorInvalidValue;
    dim3 grid((unsigned)((rows + 31) / 32), (unsigned)((cols + 31) / 32));
    hipLaunchKernelGGL(k_transpose16, grid, dim3(256), 0, s, in, rows, cols, ldi, out, ldo);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_unpool(const float *dOut, const uint8_t *arg, int N, int H, int W, uint16_t *dZ, float *dbias,
                         hipStream_t s) {
    const int64_t nq = (int64_t)N * (H / 2) * (W / 2);
    if (nq <= 0 || nq >= ((int64_t)1 << 31) || (H & 1) || (W & 1)) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)std::min<int64_t>((nq + 63) / 64, 2048);
    hipLaunchKernelGGL(k_unpool, dim3(grid), dim3(256), 0, s, dOut, arg, N, H, W, dZ, dbias);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_head(const float *Hm, const float *b1, const float *f2w, const float *f2b, int N, int Nb,
                       float *logits, const float *labels, float *loss, float *g_f2w, float *g_f2b, float *g_b1,
                       uint16_t *dH, uint16_t *dHT, int64_t ldT, hipStream_t s) {
    if (Nb > 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_head, dim3(1), dim3(1024), 0, s, Hm, b1, f2w, f2b, N, Nb, logits, labels, loss, g_f2w, g_f2b,
                       g_b1, dH, dHT, ldT);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_pack_idx(const float *master, const int32_t *idx, int64_t n, uint16_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_idx, dim3(grid_1d(n)), dim3(256), 0, s, master, idx, n, out);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_scatter_idx(const float *in, const int32_t *idx, int64_t n, float *master, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_idx, dim3(grid_1d(n)), dim3(256), 0, s, in, idx, n, master);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_zero_u16(uint16_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u16, dim3(grid_1d(n)), dim3(256), 0, s, p, n);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2, float eps,
                       int64_t t, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(grid_1d(n)), dim3(256), 0, s, w, m, v, g, n, lr, b1, b2, eps, c1, c2);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_f32, dim3(grid_1d(n)), dim3(256), 0, s, p, n);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

}  // namespace spl

// HIP kernels (gfx950) of the single-pulse search hot path.
//
//  k_dedisp      brute-force incoherent dedispersion (dedispersion section, Eq. (1)
//                delays) into the int32 DM transform
//  k_thresholds  exact moments, mean / sigma per (DM row, segment) and the smallest
//                boxcar sum reaching the S/N threshold per width (single pulse search)
//  k_boxcar      boxcar filters via wrapping 32-bit prefix sums, threshold test, best
//                width; writes the hits in (row, t) order, each tile's offset found by
//                decoupled look-back over the tiles before it
//  k_nms         peak filter over the sorted hit list (3x3, then 11x11 windows)
//  k_scan_*      device-wide exclusive scans used for ordered compaction
//  k_scatter     candidate records from the peak-filter survivors
//
// All integer work is exact; binary64 is evaluated with contraction disabled so
// every rounding is the one written in the expression.
#include <hip/hip_runtime.h>
#include <limits.h>

#include "kernels.h"
#include "spl_device.h"
#include "spl_internal.h"

#pragma clang fp contract(off)

namespace spl {

__device__ __forceinline__ int beam_of_chunk(const DevBeam *beams, int lo, int hi, int g) {
    int b = lo;
    while (b + 1 < hi && beams[b + 1].chunk_base <= g) ++b;
    return b;
}
__device__ __forceinline__ int beam_of_row(const DevBeam *beams, int lo, int hi, int r) {
    int a = lo, z = hi - 1;   // largest b with row_base <= r
    while (a < z) {
        int m = (a + z + 1) >> 1;
        if (beams[m].row_base <= r) a = m; else z = m - 1;
    }
    return a;
}

// ------------------------------------------------------------------- fill
__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------- dedispersion
// Workgroup = NW wavefronts; item = (beam, DM tile of NW*DW trials, time tile of 256*J
// samples).  Wavefront w owns DM trials d0 + w*DW ... + DW-1; lane l owns samples
// t0 + 256 j + 4 l + {0,1,2,3}, j < J.
//
// Channels are staged chan_chunk at a time.  Row r of the LDS holds channel c from
// ws_c = t0 + (tile_base_c & ~15) (16-aligned start of the tile's smallest delay) in
// four copies, copy k shifted by k bytes (copy k, byte i = sample ws_c + k + i), so that
// the 4 samples a lane needs for any delay s are one aligned dword of copy s & 3, at
// byte ((s - ws_c + t0) & ~3) + (s & 3)*quarter of the row.  That offset is precomputed
// per (channel, trial) in the plan table; the chunk's slice of the table is staged in
// LDS with the samples.  Per (trial, channel) a lane does one address add, per 256
// samples one dword read (lanes read consecutive dwords: conflict-free, paired into
// ds_read2st64_b32), and two v_perm that spread bytes (t, t+2) and (t+1, t+3) into
// 16-bit fields, summed for two channels at a time with v_add3_u32 (exact for up to
// 256 channels, then widened into int32 accumulators).  The LDS loads of the next
// channel are in flight while the current one is summed, and the global loads of the
// next chunk while the current chunk is summed.
// SV: 16-byte input vectors staged per lane and row (rows of up to 1024*SV bytes).
// NBUF: LDS buffers.  With one, every chunk is staged between two barriers while no
// wavefront sums.  With two (chunks of at most NW channels, one staged row per
// wavefront), chunk k+1 is staged into the other buffer while chunk k is summed, behind
// one barrier per chunk; half of the wavefronts stage before summing and half after,
// so that the LDS writes and byte shifts of some wavefronts fall in the LDS waits of
// the others (wavefronts w with w/4 odd stage first: with wavefronts dealt to the four
// SIMDs in turn, each SIMD holds two of each kind).
// Each wavefront stages up to dedisp_stage_rows(NBUF) rows per chunk.
template <int DW, int J, int NW, int SV, int NBUF>
__global__ __launch_bounds__(64 * NW) void k_dedisp(const DevBeam *__restrict__ beams,
                                                    const DedispItem *__restrict__ items,
                                                    int item_lo, int item_hi, int *queue) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ int s_item;
    const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
    constexpr int TD = NW * DW;
    static_assert(NBUF == 1 || NBUF == 2, "one or two LDS buffers");
    constexpr int kStageRows = dedisp_stage_rows(NBUF);
    constexpr int kStageVecs = SV;
    constexpr int kTabRows = kStageRows * NW + 4;   // chan_chunk rows + 4 rows of prefetch padding
    constexpr int kTabRegs = (kTabRows * TD + 64 * NW - 1) / (64 * NW);
    constexpr uint32_t kSelEven = 0x0C020C00u;   // bytes 0, 2 -> 16-bit fields
    constexpr uint32_t kSelOdd = 0x0C030C01u;    // bytes 1, 3 -> 16-bit fields

    int it = item_lo + blockIdx.x;
    for (;;) {
        if (queue) {
            __syncthreads();
            if (tid == 0) s_item = item_lo + atomicAdd(queue, 1);
            __syncthreads();
            it = __builtin_amdgcn_readfirstlane(s_item);
        }
        if (it >= item_hi) break;

        const DedispItem item = items[it];
        const DevBeam &B = beams[item.beam];
        const int nch = B.nch, ndm_pad = B.ndm_pad, R = item.row_bytes, quarter = B.lds_quarter;
        const int t0 = item.t0, d0 = item.d0;
        const int32_t *__restrict__ tab = B.dtab;
        const int32_t *__restrict__ base = B.tile_base + (size_t)(d0 / B.tile_dm) * nch;
        const int64_t pitch = B.pitch;
        const uint8_t *__restrict__ x = B.x;
        const int cchunk = B.chan_chunk;
        const int nvec = R >> 4;   // 16-byte vectors per row and copy
        // buffer b: four copies of chan_chunk + 1 rows, then its slice of the offset table
        const int buf_bytes = 4 * quarter + kTabRows * TD * 4;

        int32_t acc[DW][4 * J];
        uint32_t ae[DW][J], ao[DW][J];
#pragma unroll
        for (int i = 0; i < DW; ++i) {
#pragma unroll
            for (int k = 0; k < 4 * J; ++k) acc[i][k] = 0;
#pragma unroll
            for (int j = 0; j < J; ++j) ae[i][j] = ao[i][j] = 0u;
        }

        // staging registers: rows wave + NW*m, vectors lane + 64*q, and the chunk's slice
        // of the offset table (cc x TD entries, thread tid takes entries tid + 64*NW*e)
        uint4 pv[kStageRows][kStageVecs];
        uint32_t pv4[kStageRows][kStageVecs];
        int32_t pt[kTabRegs];
        auto load_chunk = [&](int c0) {
            const int cc = min(cchunk, nch - c0);
#pragma unroll
            for (int e = 0; e < kTabRegs; ++e) {
                const int idx = tid + 64 * NW * e;
                const int r = idx / TD, k = idx % TD;
                pt[e] = r < cc ? tab[(size_t)(c0 + r) * ndm_pad + d0 + k] : 0;
            }
#pragma unroll
            for (int m = 0; m < kStageRows; ++m) {
                const int r = wave + NW * m;
                const int c = c0 + r;
                const int64_t ws = r < cc ? (int64_t)((t0 + as_const(base)[c]) & ~15) : 0;
                const gu8 *src = (const gu8 *)(x + (size_t)c * pitch);
#pragma unroll
                for (int q = 0; q < kStageVecs; ++q) {
                    const int k = lane + 64 * q;
                    const int64_t off = ws + 16 * (int64_t)k;
                    pv[m][q] = make_uint4(0, 0, 0, 0);
                    pv4[m][q] = 0;
                    if (r < cc && k < nvec) {
                        if (off + 16 <= pitch) {
                            const u32x4 w = *(const gu32x4 *)(src + off);
                            pv[m][q] = make_uint4(w.x, w.y, w.z, w.w);
                        }
                        if (off + 20 <= pitch) pv4[m][q] = *(const gu32 *)(src + off + 16);
                    }
                }
            }
        };
        auto store_chunk = [&](int c0, int b) {
            const int cc = min(cchunk, nch - c0);
            uint8_t *bl = lds + b * buf_bytes;
            int32_t *lds_tab = (int32_t *)(bl + 4 * quarter);
#pragma unroll
            for (int e = 0; e < kTabRegs; ++e) {
                const int idx = tid + 64 * NW * e;
                const int r = idx / TD;
                // rows past cc (read by the branch-free prefetch) point at row cc; the
                // last register's entries beyond kTabRows rows lie outside the table.
                // Entries are byte offsets from the start of the LDS.
                if (r < kTabRows) lds_tab[idx] = (r < cc ? pt[e] + r * R : cc * R) + b * buf_bytes;
            }
            if (cc & 1) {   // an odd chunk ends with a zero row (the pair's second row)
                for (int v = tid; v < 4 * nvec; v += 64 * NW)
                    *(uint4 *)(bl + (v / nvec) * quarter + cc * R + 16 * (v % nvec)) = make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int m = 0; m < kStageRows; ++m) {
                const int r = wave + NW * m;
                uint8_t *row = bl + r * R;
#pragma unroll
                for (int q = 0; q < kStageVecs; ++q) {
                    const int k = lane + 64 * q;
                    if (!(r < cc && k < nvec)) continue;
                    const uint4 v = pv[m][q];
                    const uint32_t v4 = pv4[m][q];
                    uint4 c1, c2, c3;
                    c1.x = __builtin_amdgcn_alignbyte(v.y, v.x, 1);
                    c1.y = __builtin_amdgcn_alignbyte(v.z, v.y, 1);
                    c1.z = __builtin_amdgcn_alignbyte(v.w, v.z, 1);
                    c1.w = __builtin_amdgcn_alignbyte(v4, v.w, 1);
                    c2.x = __builtin_amdgcn_alignbyte(v.y, v.x, 2);
                    c2.y = __builtin_amdgcn_alignbyte(v.z, v.y, 2);
                    c2.z = __builtin_amdgcn_alignbyte(v.w, v.z, 2);
                    c2.w = __builtin_amdgcn_alignbyte(v4, v.w, 2);
                    c3.x = __builtin_amdgcn_alignbyte(v.y, v.x, 3);
                    c3.y = __builtin_amdgcn_alignbyte(v.z, v.y, 3);
                    c3.z = __builtin_amdgcn_alignbyte(v.w, v.z, 3);
                    c3.w = __builtin_amdgcn_alignbyte(v4, v.w, 3);
                    *(uint4 *)(row + 16 * k) = v;
                    *(uint4 *)(row + quarter + 16 * k) = c1;
                    *(uint4 *)(row + 2 * quarter + 16 * k) = c2;
                    *(uint4 *)(row + 3 * quarter + 16 * k) = c3;
                }
            }
        };

        const uint8_t *lane_lds = lds + 4 * lane;
        const int32_t *wtab0 = (const int32_t *)(lds + 4 * quarter) + wave * DW;
        const int32_t *wtab = wtab0;   // the table of the buffer being summed
        // the wave's DW offsets of one staged row (16-byte LDS reads)
        auto read_tab = [&](int r, int32_t (&t)[DW]) {
            if constexpr (DW % 4 == 0) {
#pragma unroll
                for (int i = 0; i < DW; i += 4) {
                    const int4 v = *(const int4 *)(wtab + r * TD + i);
                    t[i] = v.x;
                    t[i + 1] = v.y;
                    t[i + 2] = v.z;
                    t[i + 3] = v.w;
                }
            } else {
#pragma unroll
                for (int i = 0; i < DW; ++i) t[i] = wtab[r * TD + i];
            }
        };
        auto load_row = [&](const int32_t (&t)[DW], uint32_t (&v)[DW][J]) {
#pragma unroll
            for (int i = 0; i < DW; ++i) {
                const uint32_t *p = (const uint32_t *)(lane_lds + t[i]);
#pragma unroll
                for (int j = 0; j < J; ++j) v[i][j] = p[64 * j];
            }
        };
        auto add_rows = [&](const uint32_t (&u)[DW][J], const uint32_t (&v)[DW][J]) {
#pragma unroll
            for (int i = 0; i < DW; ++i)
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    ae[i][j] += __builtin_amdgcn_perm(u[i][j], u[i][j], kSelEven) +
                                __builtin_amdgcn_perm(v[i][j], v[i][j], kSelEven);
                    ao[i][j] += __builtin_amdgcn_perm(u[i][j], u[i][j], kSelOdd) +
                                __builtin_amdgcn_perm(v[i][j], v[i][j], kSelOdd);
                }
        };

        // the chunk's channel pairs (an odd chunk ends with the zero row).  Software
        // pipeline: while pair k is summed, the samples of pair k+1 and the offsets of
        // pair k+2 are in flight (ping-pong buffers, branch-free steady state).
        // da, db: the samples of a chunk's last channel pair.  sum_chunk reads them but
        // leaves their adds to the caller: with two buffers they are added after the
        // chunk's barrier, while the next chunk's first offsets are in flight (the reads
        // completed before the barrier, so the buffer may be restaged meanwhile); every
        // 256 channels, and at the end, they are added before the 16-bit fields widen.
        uint32_t da[DW][J], db[DW][J];
        auto sum_chunk = [&](const int cc, const bool have_def) {
            const int np = (cc + 1) >> 1;
            int32_t ta[DW], tb[DW];
            uint32_t la[DW][J], lb[DW][J], na[DW][J], nb[DW][J];
            read_tab(0, ta);
            read_tab(1, tb);
            if (have_def) add_rows(da, db);
            load_row(ta, la);
            load_row(tb, lb);
            read_tab(2, ta);
            read_tab(3, tb);
            int k = 0;
            for (; k + 3 <= np; k += 2) {
                load_row(ta, na);               // pair k+1
                load_row(tb, nb);
                read_tab(2 * k + 4, ta);        // offsets of pair k+2
                read_tab(2 * k + 5, tb);
                add_rows(la, lb);               // pair k
                load_row(ta, la);               // pair k+2
                load_row(tb, lb);
                read_tab(2 * k + 6, ta);        // offsets of pair k+3 (padding rows past the end)
                read_tab(2 * k + 7, tb);
                add_rows(na, nb);               // pair k+1
            }
            if (np - k == 2) {
                load_row(ta, na);
                load_row(tb, nb);
                add_rows(la, lb);
#pragma unroll
                for (int i = 0; i < DW; ++i)
#pragma unroll
                    for (int j = 0; j < J; ++j) { da[i][j] = na[i][j]; db[i][j] = nb[i][j]; }
            } else {
#pragma unroll
                for (int i = 0; i < DW; ++i)
#pragma unroll
                    for (int j = 0; j < J; ++j) { da[i][j] = la[i][j]; db[i][j] = lb[i][j]; }
            }
        };
        // widen the 16-bit fields every 256 channels (chan_chunk is a power of two <= 256)
        auto widen = [&](const int c_end) {
            if ((c_end & 255) == 0 || c_end >= nch) {
#pragma unroll
                for (int i = 0; i < DW; ++i)
#pragma unroll
                    for (int j = 0; j < J; ++j) {
                        acc[i][4 * j + 0] += (int32_t)(ae[i][j] & 0xFFFFu);
                        acc[i][4 * j + 2] += (int32_t)(ae[i][j] >> 16);
                        acc[i][4 * j + 1] += (int32_t)(ao[i][j] & 0xFFFFu);
                        acc[i][4 * j + 3] += (int32_t)(ao[i][j] >> 16);
                        ae[i][j] = ao[i][j] = 0u;
                    }
            }
        };

        load_chunk(0);
        if constexpr (NBUF == 1) {
            for (int c0 = 0; c0 < nch; c0 += cchunk) {
                const int cc = min(cchunk, nch - c0);
                __syncthreads();          // the previous chunk is no longer read
                store_chunk(c0, 0);
                if (c0 + cchunk < nch) load_chunk(c0 + cchunk);
                __syncthreads();          // the chunk is staged
                sum_chunk(cc, false);
                add_rows(da, db);          // one buffer: no deferral (no VGPRs to spare)
                widen(c0 + cc);
            }
        } else {
            __syncthreads();              // the previous item's last chunk is no longer read
            store_chunk(0, 0);
            if (cchunk < nch) load_chunk(cchunk);
            __syncthreads();              // the first chunk is staged
            const bool stage_first = ((wave >> 2) & 1) != 0;
            int buf = 0;
            bool have_def = false;
            for (int c0 = 0; c0 < nch; c0 += cchunk, buf ^= 1) {
                const int cc = min(cchunk, nch - c0);
                const bool more = c0 + cchunk < nch;
                // the other buffer was last read for chunk c0 - cchunk, before the
                // barrier that ended that chunk
                auto stage_next = [&]() {
                    store_chunk(c0 + cchunk, buf ^ 1);
                    if (c0 + 2 * cchunk < nch) load_chunk(c0 + 2 * cchunk);
                };
                wtab = (const int32_t *)((const uint8_t *)wtab0 + buf * buf_bytes);
                if (more && stage_first) stage_next();
                sum_chunk(cc, have_def);
                if (more && !stage_first) stage_next();
                __syncthreads();          // the next chunk is staged, this one no longer read
                const int c_end = c0 + cc;
                have_def = !((c_end & 255) == 0 || c_end >= nch);
                if (!have_def) add_rows(da, db);
                widen(c_end);
            }
        }

        // write the DM transform
        const int ndm = B.ndm, n_dd = B.n_dd;
        const int dw0 = d0 + wave * DW;
#pragma unroll
        for (int i = 0; i < DW; ++i) {
            const int d = dw0 + i;
            if (d >= ndm) continue;
            int32_t *Xr = B.X + (size_t)d * B.xpitch;
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int t = t0 + 256 * j + 4 * lane;
                if (t + 3 < n_dd) {
                    *(int4 *)(Xr + t) = make_int4(acc[i][4 * j], acc[i][4 * j + 1],
                                                  acc[i][4 * j + 2], acc[i][4 * j + 3]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (t + e < n_dd) Xr[t + e] = acc[i][4 * j + e];
                }
            }
        }
        if (!queue) break;
    }
}

// ------------------------------------------------------- moments + thresholds
// One workgroup per DM row: exact moments n, S1 = sum X, S2 = sum X^2 of every
// segment of the owned samples, then mu, sigma and, for every width w, the smallest
// integer boxcar sum T with snr(T, w) >= theta.  snr is non-decreasing in the sum,
// so "sum >= T" is exactly "snr >= theta".
__global__ __launch_bounds__(kThreads) void k_thresholds(const DevBeam *__restrict__ beams, int beam_lo,
                                                         int beam_hi, int row_lo) {
    __shared__ int64_t sh[kThreads / 64];
    const int r = row_lo + blockIdx.x;
    const DevBeam &B = beams[beam_of_row(beams, beam_lo, beam_hi, r)];
    const int d = r - B.row_base;
    const int32_t *Xr = B.X + (size_t)d * B.xpitch;
    for (int sg = 0; sg < B.nseg; ++sg) {
        const int lo = sg * B.L, hi = min((sg + 1) * B.L, B.n_out);
        // exact integer moments: 16-byte loads over the aligned middle of the segment
        // (rows start 256-byte aligned), single values at its ends
        int64_t s1 = 0, s2 = 0;
        const int a0 = min(hi, (lo + 3) & ~3), a1 = max(a0, hi & ~3);
        for (int t = lo + (int)threadIdx.x; t < a0; t += kThreads) {
            const int64_t v = Xr[t];
            s1 += v;
            s2 += v * v;
        }
        for (int t = a1 + (int)threadIdx.x; t < hi; t += kThreads) {
            const int64_t v = Xr[t];
            s1 += v;
            s2 += v * v;
        }
        const int4 *V = (const int4 *)(Xr + a0);
        const int nv = (a1 - a0) >> 2;
#pragma unroll 4
        for (int i = (int)threadIdx.x; i < nv; i += kThreads) {
            const int4 q = V[i];
            const int64_t x = q.x, y = q.y, z = q.z, w = q.w;
            s1 += (x + y) + (z + w);
            s2 += (x * x + y * y) + (z * z + w * w);
        }
        int64_t t1, t2;
        (void)block_exclusive_scan<int64_t>(s1, &t1, sh);
        (void)block_exclusive_scan<int64_t>(s2, &t2, sh);
        const size_t idx = (size_t)d * B.nseg + sg;
        if (threadIdx.x == 0) {
            B.S1[idx] = t1;
            B.S2[idx] = t2;
            double mu, sigma;
            mu_sigma(hi - lo, t1, t2, mu, sigma);
            B.mu[idx] = mu;
            B.sigma[idx] = sigma;
        }
        if ((int)threadIdx.x < B.nw) {
            double mu, sigma;
            mu_sigma(hi - lo, t1, t2, mu, sigma);
            const int j = threadIdx.x;
            const int w = B.widths[j];
            int32_t T = INT_MAX;
            if (sigma > 0.0) {
                const int64_t bmax = (int64_t)w * B.nch * 255;
                const double est = ceil((double)w * mu + B.theta * sigma * sqrt((double)w));
                int64_t b = est < 0.0 ? 0 : (est > (double)(bmax + 1) ? bmax + 1 : (int64_t)est);
                while (b > 0 && snr_of(b - 1, w, mu, sigma) >= B.theta) --b;
                while (b <= bmax && snr_of(b, w, mu, sigma) < B.theta) ++b;
                T = b > bmax ? INT_MAX : (int32_t)b;
            }
            B.T[idx * B.nw + j] = T;
        }
    }
}

// ------------------------------------------------------------------- boxcars
// Workgroup = one row chunk of kBoxTile owned samples.  The LDS holds the inclusive
// prefix sums S[i] = X[t0] + ... + X[t0+i] at index i + 1 (index 0 holds 0) as wrapping
// uint32; a window sum S[t+w-1] - S[t-1] is exact because every true sum is below 2^31.
// Thread k evaluates the 4 consecutive samples 4k + 1024q + {0..3} of each quarter q, so
// its LDS reads are 16-byte vectors at consecutive addresses across lanes.  Hits of a
// sample form a bitmask over the widths; only samples with hits evaluate the binary64
// S/N to pick the best width.  One launch counts and writes the hits in (row, t) order:
// workgroups take chunks in order from a ticket counter, publish their hit count, find
// their offset by looking back over the counts and prefixes their predecessors
// published (decoupled look-back), and write their hits from registers.
__device__ __forceinline__ uint32_t lds_u32(const uint32_t *S, int i) { return S[i]; }

// Look-back status words: flag in the top two bits, value below.
constexpr uint64_t kStatAggregate = 1ull << 62;   // the chunk's own hit count
constexpr uint64_t kStatInclusive = 2ull << 62;   // hits of every chunk up to and including it
constexpr uint64_t kStatValue = (1ull << 62) - 1;
constexpr int kLookbackPolls = 1 << 16;           // gives up (and reports it) after this many polls:
                                                  // over 60 ms, against ~25 us per chunk

// The hit count tot of chunk idx, published as soon as it is known (chunk 0's count is
// its inclusive prefix).
__device__ __forceinline__ void box_publish_count(uint64_t *status, int idx, int64_t tot) {
    __hip_atomic_store(&status[idx], (idx == 0 ? kStatInclusive : kStatAggregate) | (uint64_t)tot,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Run by one wavefront of the workgroup holding chunk idx (count tot, already published):
// sums the published values of the predecessors, nearest first, 64 at a time, up to the
// nearest one that has published its inclusive prefix; publishes its own inclusive
// prefix and returns the exclusive one.  A predecessor took its ticket earlier, so it
// runs and publishes without waiting on this workgroup; the poll limit only guards
// against a broken invariant (*stall is set and the offset is wrong).
__device__ int64_t box_lookback(uint64_t *status, int idx, int64_t tot, int32_t *stall) {
    const int lane = lane_id();
    int64_t excl = 0;
    int j = idx - 1;   // the nearest predecessor not summed yet
    int polls = 0;
    while (j >= 0) {
        const int k = j - lane;
        // before chunk 0 reads as an inclusive prefix of 0
        const uint64_t v = k >= 0 ? __hip_atomic_load(&status[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                  : kStatInclusive;
        const uint64_t flag = v >> 62;
        const uint64_t waiting = __ballot(flag == 0);
        const uint64_t inclusive = __ballot(flag == 2);
        const int first = inclusive ? __builtin_ctzll(inclusive) : 64;
        const uint64_t need = first >= 63 ? ~0ull : (2ull << first) - 1;   // lanes 0 .. first
        if (waiting & need) {
            if (++polls > kLookbackPolls) {
                if (lane == 0) atomicOr(stall, 1);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += wave_sum<int64_t>(lane <= first ? (int64_t)(v & kStatValue) : 0);
        if (first < 64) break;
        j -= 64;
    }
    if (lane == 0 && idx > 0)
        __hip_atomic_store(&status[idx], kStatInclusive | (uint64_t)(excl + tot), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

// status: n_chunks + 1 zeroed words (the last is the ticket counter); offsets gets each
// chunk's first hit index, n_total the range's hit count and stall the look-back's
// give-up flag.
__global__ __launch_bounds__(kThreads) void k_boxcar(const DevBeam *__restrict__ beams, int beam_lo,
                                                     int beam_hi, int chunk_lo, int n_chunks, int64_t *offsets,
                                                     Hit *hits, int64_t cap, uint64_t *status, int64_t *n_total,
                                                     int32_t *stall) {
    extern __shared__ __align__(16) uint32_t S[];
    __shared__ uint32_t sh32[2][kThreads / 64];
    __shared__ int64_t sh64[kThreads / 64];
    __shared__ int64_t s_base;
    __shared__ int s_idx;
    constexpr int kQ = kBoxTile / 1024;   // quarters of 1024 samples
    const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
    if (tid == 0) s_idx = (int)atomicAdd((unsigned long long *)&status[n_chunks], 1ull);
    __syncthreads();
    const int idx = s_idx;   // tickets follow the order in which workgroups start
    const int g = chunk_lo + idx;
    const DevBeam &B = beams[beam_of_chunk(beams, beam_lo, beam_hi, g)];
    const int local = g - B.chunk_base;
    const int d = local / B.nchunk_t;
    const int t0 = (local - d * B.nchunk_t) * kBoxTile;
    const int M = kBoxTile + B.w_max - 1;              // prefix entries needed
    const int nvalid = min(M, B.n_dd - t0);
    const int32_t *Xr = B.X + (size_t)d * B.xpitch + t0;

    // prefix sums in stripes of 1024 (4 consecutive per thread).  The global loads of up
    // to kPre stripes are issued together; the wave totals of consecutive stripes
    // alternate between two slots, so one barrier per stripe suffices (a slot is written
    // again two stripes later, after every thread has passed the barrier in between).
    constexpr int kPre = 5;
    constexpr int kStripe = 4 * kThreads;
    if (tid == 0) S[0] = 0u;
    uint32_t carry = 0;
    int stripe = 0;
    for (int s0 = 0; s0 < M; s0 += kPre * kStripe) {
        uint32_t v[kPre][4];
#pragma unroll
        for (int k = 0; k < kPre; ++k) {
            // one unconditional 16-byte load per thread and stripe (no branch, so the
            // loads of all stripes are in flight together).  Rows are padded to a
            // multiple of 64 entries and t0 is a multiple of 4, so a read starting at
            // i0 < nvalid stays inside the row; past nvalid the row's first vector is
            // read and the values are replaced by zeros.
            const int i0 = s0 + k * kStripe + 4 * tid;
            const u32x4 q4 = *(gu32x4 *)(Xr + (i0 < nvalid ? i0 : 0));
            v[k][0] = i0 < nvalid ? q4.x : 0u;
            v[k][1] = i0 + 1 < nvalid ? q4.y : 0u;
            v[k][2] = i0 + 2 < nvalid ? q4.z : 0u;
            v[k][3] = i0 + 3 < nvalid ? q4.w : 0u;
        }
#pragma unroll
        for (int k = 0; k < kPre; ++k, ++stripe) {
            const int i0 = s0 + k * kStripe + 4 * tid;
            if (s0 + k * kStripe >= M) break;   // uniform
            v[k][1] += v[k][0];
            v[k][2] += v[k][1];
            v[k][3] += v[k][2];
            const uint32_t x = wave_inclusive_scan(v[k][3]);
            uint32_t *tw = sh32[stripe & 1];
            if (lane == 63) tw[wave] = x;
            __syncthreads();
            uint32_t pre = carry, tot = 0;
#pragma unroll
            for (int w = 0; w < kThreads / 64; ++w) {
                if (w < wave) pre += tw[w];
                tot += tw[w];
            }
            pre += x - v[k][3];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (i0 + e < M) S[i0 + e + 1] = pre + v[k][e];
            carry += tot;
        }
    }
    __syncthreads();   // every prefix entry is written

    const int nw = B.nw, L = B.L, nseg = B.nseg;
    const int tend = min(t0 + kBoxTile, B.n_out);   // owned samples of this chunk: [t0, tend)
    uint32_t mask[kQ][4];
#pragma unroll
    for (int q = 0; q < kQ; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) mask[q][e] = 0u;

    if (tend > t0) {
        // segments spanned by the chunk (usually one); thresholds of a segment are uniform
        for (int sg = t0 / L; sg <= (tend - 1) / L; ++sg) {
            const int s_lo = max(sg * L, t0) - t0, s_hi = min((sg + 1) * L, tend) - t0;
            const cint32 *Tp = as_const(B.T + ((size_t)d * nseg + sg) * nw);
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int li = 1024 * q + 4 * tid;   // local index of the first of 4 samples
                const uint4 lo = *(const uint4 *)&S[li];
                const uint4 nx = *(const uint4 *)&S[li + 4];
                const uint32_t s0[8] = {lo.x, lo.y, lo.z, lo.w, nx.x, nx.y, nx.z, nx.w};
                for (int j = 0; j < nw; ++j) {
                    const int w = B.widths[j];
                    const int32_t T = Tp[j];
                    uint32_t hw[4];
                    if (w < 4) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) hw[e] = w == 1 ? s0[e + 1] : (w == 2 ? s0[e + 2] : s0[e + 3]);
                    } else if ((w & 3) == 0) {
                        const uint4 h = *(const uint4 *)&S[li + w];
                        hw[0] = h.x; hw[1] = h.y; hw[2] = h.z; hw[3] = h.w;
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) hw[e] = lds_u32(S, li + w + e);
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int lt = li + e;
                        const bool in = lt >= s_lo && lt < s_hi;
                        if (in && (int32_t)(hw[e] - s0[e]) >= T) mask[q][e] |= 1u << j;
                    }
                }
            }
        }
    }
    // hits are emitted in t order: quarter by quarter, thread by thread within a quarter.
    // The four per-quarter counts (<= 1024 each) are scanned together in 16-bit fields.
    uint64_t packed = 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        uint64_t cq = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) cq += mask[q][e] ? 1 : 0;
        packed |= cq << (16 * q);
    }
    uint64_t ptot;
    const uint64_t pex = block_exclusive_scan<uint64_t>(packed, &ptot, (uint64_t *)sh64);
    const int row = B.row_base + d;
    int64_t tot = 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) tot += (int64_t)((ptot >> (16 * q)) & 0xFFFFu);
    if (tid == 0) box_publish_count(status, idx, tot);

    // best width of every hit (widths in ascending order; an equal S/N keeps the smaller
    // width) while the earlier chunks finish: its mask keeps only that width's bit
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            uint32_t m = mask[q][e];
            if (!m || (m & (m - 1)) == 0) continue;   // no hit, or a single width
            const int li = 1024 * q + 4 * tid + e, t = t0 + li;
            const size_t ms = (size_t)d * nseg + t / L;
            const double mu = B.mu[ms], sigma = B.sigma[ms];
            const uint32_t lo = S[li];
            double best = 0.0;
            int bj = -1;
            while (m) {
                const int j = __builtin_ctz(m);
                m &= m - 1;
                const int w = B.widths[j];
                const double sn = snr_of((int32_t)(S[li + w] - lo), w, mu, sigma);
                if (bj < 0 || sn > best) {
                    best = sn;
                    bj = j;
                }
            }
            mask[q][e] = 1u << bj;
        }
    }

    if (wave == 0) {
        const int64_t excl = box_lookback(status, idx, tot, stall);
        if (lane == 0) {
            s_base = excl;
            offsets[idx] = excl;
            if (idx == n_chunks - 1) *n_total = excl + tot;
        }
    }
    __syncthreads();
    int64_t qbase = s_base;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        int64_t pos = qbase + (int64_t)((pex >> (16 * q)) & 0xFFFFu);
        qbase += (int64_t)((ptot >> (16 * q)) & 0xFFFFu);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t m = mask[q][e];   // the best width's bit only
            if (!m) continue;
            if (pos < cap) {
                const int li = 1024 * q + 4 * tid + e, t = t0 + li;
                const size_t ms = (size_t)d * nseg + t / L;
                const int w = B.widths[__builtin_ctz(m)];
                const int32_t Bw = (int32_t)(S[li + w] - S[li]);
                Hit h;
                h.row = row;
                h.t = t;
                h.w = w;
                h.B = Bw;
                h.snr = snr_of(Bw, w, B.mu[ms], B.sigma[ms]);   // the same binary64 value as above
                hits[pos] = h;
            }
            ++pos;
        }
    }
}

// ------------------------------------------------------------------- scans
// Exclusive scan of n elements (n read from *n_dev when given, else n_static) in
// blocks of kScanPerBlock: per-block sums, one-workgroup scan of the sums, then the
// per-block scan with its offset.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const T *in, const int64_t *n_dev, int64_t n_static,
                                                          int64_t *block_sums) {
    __shared__ int64_t sh[kThreads / 64];
    const int64_t n = n_dev ? min(*n_dev, n_static) : n_static;
    const int64_t b0 = (int64_t)blockIdx.x * kScanPerBlock;
    int64_t s = 0;
    if (b0 < n) {
        for (int k = 0; k < kScanPerBlock / kThreads; ++k) {
            const int64_t i = b0 + (int64_t)k * kThreads + threadIdx.x;
            if (i < n) s += (int64_t)in[i];
        }
    }
    int64_t tot;
    (void)block_exclusive_scan<int64_t>(s, &tot, sh);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_top(int64_t *block_sums, int nblocks, int64_t *total_out) {
    __shared__ int64_t sh[16];
    __shared__ int64_t s_carry;
    const int tid = threadIdx.x, lane = lane_id(), wave = threadIdx.x >> 6;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < nblocks; base += 1024) {
        const int i = base + tid;
        const int64_t v = i < nblocks ? block_sums[i] : 0;
        const int64_t x = wave_inclusive_scan(v);
        if (lane == 63) sh[wave] = x;
        __syncthreads();
        int64_t pre = 0, tot = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wave) pre += sh[w];
            tot += sh[w];
        }
        const int64_t c = s_carry;
        if (i < nblocks) block_sums[i] = c + pre + x - v;
        __syncthreads();
        if (tid == 0) s_carry = c + tot;
        __syncthreads();
    }
    if (tid == 0 && total_out) *total_out = s_carry;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_down(const T *in, const int64_t *n_dev, int64_t n_static,
                                                        const int64_t *block_offsets, int64_t *out) {
    __shared__ int64_t sh[kThreads / 64];
    const int64_t n = n_dev ? min(*n_dev, n_static) : n_static;
    const int64_t b0 = (int64_t)blockIdx.x * kScanPerBlock;
    if (b0 >= n) return;
    int64_t carry = block_offsets[blockIdx.x];
    for (int k = 0; k < kScanPerBlock / kThreads; ++k) {
        const int64_t i = b0 + (int64_t)k * kThreads + threadIdx.x;
        const int64_t v = i < n ? (int64_t)in[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan<int64_t>(v, &tot, sh);
        if (i < n) out[i] = carry + ex;
        carry += tot;
    }
}

// First hit of every row (clamped to the stored hits) from the chunk offsets.
__global__ void k_row_start(const DevBeam *__restrict__ beams, int beam_lo, int beam_hi, int row_lo,
                            int row_hi, int chunk_lo, const int64_t *chunk_off, const int64_t *n_hits,
                            int64_t cap, int64_t *row_start) {
    const int r = row_lo + blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stored = min(*n_hits, cap);
    if (r < row_hi) {
        const DevBeam &B = beams[beam_of_row(beams, beam_lo, beam_hi, r)];
        const int chunk = B.chunk_base + (r - B.row_base) * B.nchunk_t;
        row_start[r - row_lo] = min(chunk_off[chunk - chunk_lo], stored);
    }
    if (r == row_hi) row_start[r - row_lo] = stored;
}

// ------------------------------------------------------- survivors of the first filter
// The later peak filters see only the survivors of the first, compacted in order
// (out[pos[p]] = hits[p] for alive p, pos the exclusive scan of the flags), with row
// starts out_start[r] = pos[row_start[r]] (the count of survivors before the row).
__global__ __launch_bounds__(kThreads) void k_compact_hits(const Hit *__restrict__ hits, const int64_t *n_hits,
                                                           int64_t cap, const uint8_t *__restrict__ alive,
                                                           const int64_t *__restrict__ pos, Hit *__restrict__ out) {
    const int64_t n = min(*n_hits, cap);
    for (int64_t p = blockIdx.x * (int64_t)kThreads + threadIdx.x; p < n; p += (int64_t)gridDim.x * kThreads)
        if (alive[p]) out[pos[p]] = hits[p];
}

__global__ __launch_bounds__(kThreads) void k_compact_row_start(const int64_t *__restrict__ row_start, int n_rows,
                                                                const int64_t *n_hits, int64_t cap,
                                                                const int64_t *__restrict__ pos,
                                                                const int64_t *n_surv, int64_t *out_start) {
    const int r = blockIdx.x * kThreads + threadIdx.x;
    if (r > n_rows) return;
    const int64_t n = min(*n_hits, cap);
    const int64_t i = row_start[r];
    out_start[r] = (r < n_rows && i < n) ? pos[i] : *n_surv;
}

// ------------------------------------------------------- block index of hit rows
// blk[r][b] = index (within row r) of the first hit with t >= 64 b, or the row's hit count.
// k_nms_mark writes the first hit of every occupied block (the table holds INT32_MAX
// elsewhere) and the hits' times as a packed int32 array (the peak filter's searches
// and window scans read 4 bytes per hit instead of a 24-byte record); k_nms_suffix then
// takes the suffix minimum along each row.
__global__ __launch_bounds__(kThreads) void k_nms_mark(int row_lo, const Hit *__restrict__ hits,
                                                       const int64_t *n_hits, int64_t cap,
                                                       const int64_t *__restrict__ row_start, int32_t *blk,
                                                       int nblk, int32_t *__restrict__ hit_t) {
    const int64_t n = min(*n_hits, cap);
    for (int64_t q = blockIdx.x * (int64_t)kThreads + threadIdx.x; q < n; q += (int64_t)gridDim.x * kThreads) {
        const Hit h = hits[q];
        hit_t[q] = h.t;
        const int r = h.row - row_lo;
        const int b = h.t >> kNmsBlockShift;
        const bool first = q == 0 || hits[q - 1].row != h.row || (hits[q - 1].t >> kNmsBlockShift) != b;
        if (first) blk[(int64_t)r * nblk + b] = (int32_t)(q - row_start[r]);
    }
}

__global__ __launch_bounds__(kThreads) void k_nms_suffix(const int64_t *__restrict__ row_start, int n_rows,
                                                         int32_t *blk, int nblk) {
    const int lane = lane_id();
    const int r = blockIdx.x * (kThreads / 64) + wave_id();
    if (r >= n_rows) return;   // uniform per wavefront
    int32_t carry = (int32_t)(row_start[r + 1] - row_start[r]);
    int32_t *row = blk + (int64_t)r * nblk;
    for (int c = (nblk - 1) & ~63; c >= 0; c -= 64) {
        const int b = c + lane;
        int32_t v = b < nblk ? row[b] : INT_MAX;
        v = min(v, carry);
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t o = __shfl_down(v, off);
            if (lane + off < 64) v = min(v, o);
        }
        if (b < nblk) row[b] = v;
        carry = __shfl(v, 0);
    }
}

// ---------------------------------------------------------------- peak filter
// q beats p when (snr_q, -d_q, -t_q) > (snr_p, -d_p, -t_p).  p survives when no other
// alive hit of its beam within |dd| <= rd, |dt| <= rt beats it.  Rows of a beam are
// contiguous in the hit list and sorted by t; a neighbour row's window starts at the
// first hit with t >= t_p - rt, found by bisection between the row's first hits of that
// 64-sample block and of the next (the block index, built once per run by k_nms_mark and
// k_nms_suffix): at most 6 dependent loads instead of one per halving of the row.  A row
// holds at most one hit per sample, so in p's own row the window starts no more than rt
// entries before p and needs no search.  Searches and scans read the packed times; a
// hit's S/N is loaded only when it lies in the window.
__global__ __launch_bounds__(kThreads) void k_nms(const DevBeam *__restrict__ beams, int beam_lo, int beam_hi,
                                                  int row_lo, const Hit *__restrict__ hits,
                                                  const int64_t *n_hits, int64_t cap,
                                                  const int64_t *__restrict__ row_start,
                                                  const int32_t *__restrict__ blk, int nblk, int stencil,
                                                  const uint8_t *alive_in, uint8_t *alive_out,
                                                  int64_t *n_alive, const int32_t *__restrict__ hit_t) {
    __shared__ int64_t sh[kThreads / 64];
    // first rows of the beams, for the bisection from a hit's row to its beam in the LDS
    // (when the batch has more beams than fit, the bisection reads the descriptors)
    constexpr int kBeamCache = 256;
    __shared__ int32_t s_rb[kBeamCache];
    const int nbm = beam_hi - beam_lo;
    const bool cached = nbm <= kBeamCache;
    if (cached)
        for (int b = threadIdx.x; b < nbm; b += kThreads) s_rb[b] = beams[beam_lo + b].row_base;
    __syncthreads();
    const int64_t n = min(*n_hits, cap);
    int64_t kept = 0;
    for (int64_t p = blockIdx.x * (int64_t)kThreads + threadIdx.x; p < n; p += (int64_t)gridDim.x * kThreads) {
        if (alive_in && !alive_in[p]) {
            alive_out[p] = 0;
            continue;
        }
        const Hit h = hits[p];
        int bi;
        if (cached) {   // largest b with row_base <= row
            int a = 0, z = nbm - 1;
            while (a < z) {
                const int m = (a + z + 1) >> 1;
                if (s_rb[m] <= h.row) a = m; else z = m - 1;
            }
            bi = beam_lo + a;
        } else {
            bi = beam_of_row(beams, beam_lo, beam_hi, h.row);
        }
        const DevBeam &B = beams[bi];
        if (stencil >= B.nst) {   // this beam's plan has fewer filters: pass through
            alive_out[p] = 1;
            ++kept;
            continue;
        }
        const int rd = B.rd[stencil], rt = B.rt[stencil];
        const int d = h.row - B.row_base;
        bool keep = true;
        // rows in the order 0, -1, +1, -2, +2, ...: the own row needs no search and the
        // nearest rows most often hold a hit that beats p (the outcome does not depend
        // on the order, only how early the loop stops)
        for (int i = 0; i <= 2 * rd && keep; ++i) {
            const int dd = (i & 1) ? -((i + 1) >> 1) : (i >> 1);
            const int d2 = d + dd;
            if (d2 < 0 || d2 >= B.ndm) continue;
            const int r2 = B.row_base + d2 - row_lo;
            const int tmin = h.t - rt;
            const int64_t end = row_start[r2 + 1];
            // where the window [tmin, t_p + rt] starts in row r2
            int64_t lo = row_start[r2], hi = end;
            if (dd == 0) {
                lo = max(lo, p - rt);   // own row: no earlier entry can have t >= tmin
            } else {
                // the first index with t >= tmin lies between the first hits of tmin's
                // 64-sample block and of the next block (block index): bisect in between
                if (tmin > 0) {
                    const int b = tmin >> kNmsBlockShift;
                    const int32_t *br = blk + (int64_t)r2 * nblk;
                    hi = lo + br[b + 1];   // b + 1 < nblk: the index has a block past every t
                    lo += br[b];
                }
                while (lo < hi) {
                    const int64_t m = (lo + hi) >> 1;
                    if (hit_t[m] < tmin) lo = m + 1; else hi = m;
                }
            }
            for (int64_t q = lo; q < end; ++q) {
                const int gt = hit_t[q];
                if (gt > h.t + rt) break;
                if (gt < tmin || q == p || (alive_in && !alive_in[q])) continue;
                const double gs = hits[q].snr;
                const bool beats = gs != h.snr ? gs > h.snr : (d2 != d ? d2 < d : gt < h.t);
                if (beats) {
                    keep = false;
                    break;
                }
            }
        }
        alive_out[p] = keep ? 1 : 0;
        kept += keep ? 1 : 0;
    }
    int64_t tot;
    (void)block_exclusive_scan<int64_t>(kept, &tot, sh);
    if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long *)n_alive, (unsigned long long)tot);
}

// Candidate records of the survivors, in hit order, after `*base` earlier records.
__global__ __launch_bounds__(kThreads) void k_scatter(const DevBeam *__restrict__ beams, int beam_lo, int beam_hi,
                                                      const Hit *__restrict__ hits, const int64_t *n_hits,
                                                      int64_t cap, const uint8_t *alive, const int64_t *pos,
                                                      const int64_t *base, spl_candidate *cands,
                                                      int64_t cand_cap) {
    const int64_t n = min(*n_hits, cap);
    const int64_t b0 = *base;
    for (int64_t p = blockIdx.x * (int64_t)kThreads + threadIdx.x; p < n; p += (int64_t)gridDim.x * kThreads) {
        if (alive && !alive[p]) continue;
        const int64_t o = b0 + (pos ? pos[p] : p);
        if (o >= cand_cap) continue;
        const Hit h = hits[p];
        const DevBeam &B = beams[beam_of_row(beams, beam_lo, beam_hi, h.row)];
        spl_candidate c;
        c.beam = B.beam;
        c.dm_index = h.row - B.row_base;
        c.t_sample = h.t;
        c.width = h.w;
        c.boxcar_sum = h.B;
        c.snr = (float)h.snr;
        c.dm = (float)B.dms[c.dm_index];
        c.flags = 0u;
        cands[o] = c;
    }
}

// End of the launch sequence of a beam range: fold the range's counts into the run
// statistics; the next range's candidates go after this one's.
__global__ void k_pass_end(DevRun *run, spl_run_stats *stats, int64_t hit_cap, int nst) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    stats->n_hits += run->n_hits;
    if (run->n_hits > hit_cap && stats->hit_overflow == 0) stats->hit_overflow = 1;
    if (run->box_stall) stats->hit_overflow = 2;
    for (int k = 0; k < nst; ++k) {
        stats->n_after_stencil[k] += run->n_alive[k];
        run->n_alive[k] = 0;
    }
    run->n_cand_total += nst ? run->n_cand_beam : min(run->n_hits, hit_cap);
}

__global__ void k_finalize(DevRun *run, spl_run_stats *stats, int64_t cand_cap) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    stats->n_candidates = run->n_cand_total;
    stats->cand_overflow = run->n_cand_total > cand_cap ? 1 : 0;
}

// Position-weighted checksum of a DM transform (verifies that retiled kernels give
// identical output): sum over (d, t) of X[d][t] * (1 + d * 65599 + t * 131), wrapping.
__global__ void k_checksum(const int32_t *X, int ndm, int xpitch, int n_dd, unsigned long long *out) {
    __shared__ unsigned long long sh[kThreads / 64];
    unsigned long long s = 0;
    const int64_t n = (int64_t)ndm * n_dd;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int d = (int)(i / n_dd), t = (int)(i - (int64_t)d * n_dd);
        s += (unsigned long long)(uint32_t)X[(size_t)d * xpitch + t] *
             (1ull + (unsigned long long)d * 65599ull + (unsigned long long)t * 131ull);
    }
    unsigned long long tot;
    (void)block_exclusive_scan<unsigned long long>(s, &tot, sh);
    if (threadIdx.x == 0) atomicAdd(out, tot);
}

// Normaliser test hook: mu and sigma from exact moments, as the search computes them.
__global__ void k_mu_sigma(const int64_t *n, const int64_t *s1, const int64_t *s2, int64_t count,
                           double *mu, double *sigma) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < count) mu_sigma(n[i], s1[i], s2[i], mu[i], sigma[i]);
}

// ---------------------------------------------------------------- launchers
#define SPL_HIP_LAUNCH_CHECK() \
    do { hipError_t e__ = hipGetLastError(); if (e__ != hipSuccess) return e__; } while (0)

template <int DW, int J, int NW, int SV, int NBUF>
static hipError_t prepare_dedisp_t(size_t lds_bytes, int *blocks_per_cu) {
    if (lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_dedisp<DW, J, NW, SV, NBUF>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_dedisp<DW, J, NW, SV, NBUF>, 64 * NW,
                                                        lds_bytes);
}

template <int DW, int J, int NW, int SV, int NBUF>
static hipError_t launch_dedisp_t(const DevBeam *beams, const DedispItem *items, int item_lo, int item_hi,
                                  int *queue, int grid, size_t lds_bytes, hipStream_t s) {
    hipLaunchKernelGGL((k_dedisp<DW, J, NW, SV, NBUF>), dim3(grid), dim3(64 * NW), lds_bytes, s, beams, items,
                       item_lo, item_hi, queue);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

// The compiled dedispersion shapes: (DM trials per wavefront, 256-sample groups per
// lane, wavefronts per workgroup, 16-byte vectors staged per lane and row, LDS buffers).
// Double buffering is compiled for the 16-wavefront shapes, which hold one workgroup
// per CU, so that no other workgroup sums while one stages.
#define SPL_DEDISP_SHAPES(X)                                                                                 \
    X(2, 2, 8, 1, 1) X(4, 1, 4, 1, 1) X(4, 2, 4, 1, 1) X(4, 1, 8, 1, 1) X(4, 2, 8, 1, 1) X(8, 1, 4, 1, 1)   \
    X(8, 1, 8, 1, 1) X(2, 2, 8, 2, 1) X(4, 1, 4, 2, 1) X(4, 1, 8, 2, 1) X(4, 2, 8, 2, 1) X(4, 1, 16, 1, 1)  \
    X(4, 2, 16, 1, 1) X(2, 2, 16, 1, 1) X(2, 2, 16, 2, 1) X(4, 1, 16, 1, 2) X(4, 2, 16, 1, 2)              \
    X(2, 2, 16, 1, 2) X(2, 2, 16, 2, 2)

bool dedisp_shape_supported(int dw, int j, int nw, int sv, int nbuf) {
#define SPL_X(a, b, c, d, e) if (dw == a && j == b && nw == c && sv == d && nbuf == e) return true;
    SPL_DEDISP_SHAPES(SPL_X)
#undef SPL_X
    return false;
}

hipError_t prepare_dedisp(int dw, int j, int nw, int sv, int nbuf, size_t lds_bytes, int *blocks_per_cu) {
#define SPL_X(a, b, c, d, e)                                          \
    if (dw == a && j == b && nw == c && sv == d && nbuf == e)         \
        return prepare_dedisp_t<a, b, c, d, e>(lds_bytes, blocks_per_cu);
    SPL_DEDISP_SHAPES(SPL_X)
#undef SPL_X
    return hipErrorInvalidValue;
}

hipError_t launch_dedisp(int dw, int j, int nw, int sv, int nbuf, const DevBeam *beams, const DedispItem *items,
                         int item_lo, int item_hi, int *queue, int grid, size_t lds_bytes, hipStream_t s) {
#define SPL_X(a, b, c, d, e)                                                                                 \
    if (dw == a && j == b && nw == c && sv == d && nbuf == e)                                                \
        return launch_dedisp_t<a, b, c, d, e>(beams, items, item_lo, item_hi, queue, grid, lds_bytes, s);
    SPL_DEDISP_SHAPES(SPL_X)
#undef SPL_X
    return hipErrorInvalidValue;
}

hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(kThreads), 0, s, p, n, v);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_thresholds(const DevBeam *beams, int beam_lo, int beam_hi, int row_lo, int row_hi, hipStream_t s) {
    const int n = row_hi - row_lo;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_thresholds, dim3(n), dim3(kThreads), 0, s, beams, beam_lo, beam_hi, row_lo);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_boxcar_one_pass(const DevBeam *beams, int beam_lo, int beam_hi, int chunk_lo, int chunk_hi,
                                  int w_max, uint64_t *status, int64_t *offsets, Hit *hits, int64_t cap,
                                  int64_t *n_total, int32_t *stall, hipStream_t s) {
    const int n = chunk_hi - chunk_lo;
    if (!status || !offsets || !hits || !n_total || !stall) return hipErrorInvalidValue;
    if (n <= 0) return launch_fill_u64((uint64_t *)n_total, 1, 0, s);
    // the look-back words of the range and its ticket counter start at zero
    hipError_t e = launch_fill_u64(status, (int64_t)n + 1, 0, s);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)(kBoxTile + w_max + 8) * sizeof(uint32_t);
    hipLaunchKernelGGL(k_boxcar, dim3(n), dim3(kThreads), lds, s, beams, beam_lo, beam_hi, chunk_lo, n, offsets,
                       hits, cap, status, n_total, stall);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

int scan_blocks(int64_t n_max) { return (int)((n_max + kScanPerBlock - 1) / kScanPerBlock); }

template <typename T>
static hipError_t launch_scan_t(const T *in, const int64_t *n_dev, int64_t n_max, int64_t *block_sums,
                                int64_t *out, int64_t *total, hipStream_t s) {
    const int nb = scan_blocks(n_max);
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3(nb), dim3(kThreads), 0, s, in, n_dev, n_max, block_sums);
    SPL_HIP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, block_sums, nb, total);
    SPL_HIP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_down<T>, dim3(nb), dim3(kThreads), 0, s, in, n_dev, n_max, block_sums, out);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_scan_u8(const uint8_t *in, const int64_t *n_dev, int64_t n_max, int64_t *block_sums,
                          int64_t *out, int64_t *total, hipStream_t s) {
    return launch_scan_t<uint8_t>(in, n_dev, n_max, block_sums, out, total, s);
}

hipError_t launch_row_start(const DevBeam *beams, int beam_lo, int beam_hi, int row_lo, int row_hi, int chunk_lo,
                            const int64_t *chunk_off, const int64_t *n_hits, int64_t cap, int64_t *row_start,
                            hipStream_t s) {
    const int n = row_hi - row_lo + 1;
    hipLaunchKernelGGL(k_row_start, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, beams, beam_lo,
                       beam_hi, row_lo, row_hi, chunk_lo, chunk_off, n_hits, cap, row_start);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

static int grid_for(int64_t cap) {
    int64_t g = (cap + kThreads - 1) / kThreads;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_compact_hits(const Hit *hits, const int64_t *n_hits, int64_t cap, const uint8_t *alive,
                               const int64_t *pos, Hit *out, const int64_t *row_start, int n_rows,
                               const int64_t *n_surv, int64_t *out_start, hipStream_t s) {
    hipLaunchKernelGGL(k_compact_hits, dim3(grid_for(cap)), dim3(kThreads), 0, s, hits, n_hits, cap, alive, pos, out);
    SPL_HIP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_compact_row_start, dim3((n_rows + 1 + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                       row_start, n_rows, n_hits, cap, pos, n_surv, out_start);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_nms_index(int row_lo, int n_rows, const Hit *hits, const int64_t *n_hits, int64_t cap,
                            const int64_t *row_start, int32_t *blk, int nblk, int32_t *hit_t, hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    if (nblk & 1) return hipErrorInvalidValue;   // filled in 8-byte words
    hipError_t e = launch_fill_u64((uint64_t *)blk, (int64_t)n_rows * nblk / 2, 0x7FFFFFFF7FFFFFFFull, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_nms_mark, dim3(grid_for(cap)), dim3(kThreads), 0, s, row_lo, hits, n_hits, cap, row_start,
                       blk, nblk, hit_t);
    SPL_HIP_LAUNCH_CHECK();
    const int waves = kThreads / 64;
    hipLaunchKernelGGL(k_nms_suffix, dim3((unsigned)((n_rows + waves - 1) / waves)), dim3(kThreads), 0, s, row_start,
                       n_rows, blk, nblk);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_nms(const DevBeam *beams, int beam_lo, int beam_hi, int row_lo, const Hit *hits,
                      const int64_t *n_hits, int64_t cap, const int64_t *row_start, const int32_t *blk, int nblk,
                      int stencil, const uint8_t *alive_in, uint8_t *alive_out, int64_t *n_alive,
                      const int32_t *hit_t, hipStream_t s) {
    hipLaunchKernelGGL(k_nms, dim3(grid_for(cap)), dim3(kThreads), 0, s, beams, beam_lo, beam_hi, row_lo, hits,
                       n_hits, cap, row_start, blk, nblk, stencil, alive_in, alive_out, n_alive, hit_t);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_scatter(const DevBeam *beams, int beam_lo, int beam_hi, const Hit *hits, const int64_t *n_hits,
                          int64_t cap, const uint8_t *alive, const int64_t *pos, const int64_t *base,
                          spl_candidate *cands, int64_t cand_cap, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(cap)), dim3(kThreads), 0, s, beams, beam_lo, beam_hi, hits,
                       n_hits, cap, alive, pos, base, cands, cand_cap);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_pass_end(DevRun *run, spl_run_stats *stats, int64_t hit_cap, int nst, hipStream_t s) {
    hipLaunchKernelGGL(k_pass_end, dim3(1), dim3(64), 0, s, run, stats, hit_cap, nst);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_finalize(DevRun *run, spl_run_stats *stats, int64_t cand_cap, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, run, stats, cand_cap);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_checksum(const int32_t *X, int ndm, int xpitch, int n_dd, unsigned long long *out,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_checksum, dim3(1024), dim3(kThreads), 0, s, X, ndm, xpitch, n_dd, out);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_mu_sigma(const int64_t *n, const int64_t *s1, const int64_t *s2, int64_t count, double *mu,
                           double *sigma, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mu_sigma, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, n, s1, s2, count, mu,
                       sigma);
    SPL_HIP_LAUNCH_CHECK();
    return hipSuccess;
}

}  // namespace spl

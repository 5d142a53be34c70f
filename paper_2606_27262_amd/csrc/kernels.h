// Launchers of the HIP kernels (kernels.hip); every call enqueues on stream `s` and
// returns the launch status.
#pragma once

#include "spl_internal.h"
#include "spotlight.h"

namespace spl {

// Staged rows per wavefront and chunk: chan_chunk <= dedisp_stage_rows(buffers) * waves
// (one LDS buffer: two rows; two buffers: one row each, so two buffers of a 16-wavefront
// tile hold what one buffer of 32 channels holds).
constexpr int dedisp_stage_rows(int buffers) { return buffers == 2 ? 1 : 2; }
// A staged row holds up to 1024 * sv bytes (sv = 16-byte vectors per lane, 1 or 2);
// nbuf = LDS buffers (1 or 2).
bool dedisp_shape_supported(int dw, int j, int nw, int sv, int nbuf);
hipError_t prepare_dedisp(int dw, int j, int nw, int sv, int nbuf, size_t lds_bytes, int *blocks_per_cu);
hipError_t launch_dedisp(int dw, int j, int nw, int sv, int nbuf, const DevBeam *beams, const DedispItem *items,
                         int item_lo, int item_hi, int *queue, int grid, size_t lds_bytes, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_thresholds(const DevBeam *beams, int beam_lo, int beam_hi, int row_lo, int row_hi,
                             hipStream_t s);
// Boxcar hits of chunks [chunk_lo, chunk_hi) in one launch (decoupled look-back): status
// holds chunk_hi - chunk_lo + 1 words (cleared here), offsets gets each chunk's first hit
// index, *n_total the range's hit count; *stall is set if a look-back gave up.
hipError_t launch_boxcar_one_pass(const DevBeam *beams, int beam_lo, int beam_hi, int chunk_lo, int chunk_hi,
                                  int w_max, uint64_t *status, int64_t *offsets, Hit *hits, int64_t cap,
                                  int64_t *n_total, int32_t *stall, hipStream_t s);
int scan_blocks(int64_t n_max);
hipError_t launch_scan_u8(const uint8_t *in, const int64_t *n_dev, int64_t n_max, int64_t *block_sums,
                          int64_t *out, int64_t *total, hipStream_t s);
hipError_t launch_row_start(const DevBeam *beams, int beam_lo, int beam_hi, int row_lo, int row_hi, int chunk_lo,
                            const int64_t *chunk_off, const int64_t *n_hits, int64_t cap, int64_t *row_start,
                            hipStream_t s);
// Block index of the hit rows [row_lo, row_lo + n_rows): blk[r][b] = index within row r
// of its first hit with t >= 64 b (the row's count when none); nblk even, 64 nblk > the
// largest t.
// The survivors of a peak filter (alive flags, pos their exclusive scan, *n_surv their
// count) compacted in order into out, with the row starts of the compacted list.
hipError_t launch_compact_hits(const Hit *hits, const int64_t *n_hits, int64_t cap, const uint8_t *alive,
                               const int64_t *pos, Hit *out, const int64_t *row_start, int n_rows,
                               const int64_t *n_surv, int64_t *out_start, hipStream_t s);
hipError_t launch_nms_index(int row_lo, int n_rows, const Hit *hits, const int64_t *n_hits, int64_t cap,
                            const int64_t *row_start, int32_t *blk, int nblk, int32_t *hit_t, hipStream_t s);
hipError_t launch_nms(const DevBeam *beams, int beam_lo, int beam_hi, int row_lo, const Hit *hits,
                      const int64_t *n_hits, int64_t cap, const int64_t *row_start, const int32_t *blk, int nblk,
                      int stencil, const uint8_t *alive_in, uint8_t *alive_out, int64_t *n_alive,
                      const int32_t *hit_t, hipStream_t s);
hipError_t launch_scatter(const DevBeam *beams, int beam_lo, int beam_hi, const Hit *hits, const int64_t *n_hits,
                          int64_t cap, const uint8_t *alive, const int64_t *pos, const int64_t *base,
                          spl_candidate *cands, int64_t cand_cap, hipStream_t s);
hipError_t launch_pass_end(DevRun *run, spl_run_stats *stats, int64_t hit_cap, int nst, hipStream_t s);
hipError_t launch_finalize(DevRun *run, spl_run_stats *stats, int64_t cand_cap, hipStream_t s);
hipError_t launch_checksum(const int32_t *X, int ndm, int xpitch, int n_dd, unsigned long long *out,
                           hipStream_t s);
hipError_t launch_mu_sigma(const int64_t *n, const int64_t *s1, const int64_t *s2, int64_t count, double *mu,
                           double *sigma, hipStream_t s);

}  // namespace spl

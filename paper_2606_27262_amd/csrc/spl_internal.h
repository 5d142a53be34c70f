// Internal layout shared by the host runtime and the HIP kernels of libspotlight.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spl {

constexpr int kMaxWidths = 16;
constexpr int kMaxStencils = 4;
constexpr int kBoxTile = 4096;        // owned samples per boxcar workgroup (multiple of 1024)
constexpr int kThreads = 256;         // threads per workgroup of every kernel
constexpr int kNmsBlockShift = 6;     // the peak filter indexes hit rows in blocks of 64 samples
constexpr int kScanPerBlock = 4096;   // elements per block of the device-wide scan
constexpr int kMaxWmax = 8192;
constexpr int kMaxShapeGroups = 4;  // distinct dedispersion tile shapes per batch

// One beam of a batch, resident in the workspace.
struct DevBeam {
    const uint8_t *x;        // block [nch][pitch]
    int64_t pitch;           // bytes
    const int32_t *dtab;     // LDS byte offset of each delay from its staged row origin,
                             // channel-major [nch][ndm_pad]:
                             // ((s - b) & ~3) + (s & 3)*lds_quarter, b = tile_base & ~15
    const int32_t *tile_base;// min delay over each DM tile [ndm_tiles][nch]
    const int32_t *delays;   // delay table in samples [ndm][nch] (snippet extraction)
    int32_t *X;              // DM transform [ndm][xpitch]
    int64_t *S1, *S2;        // [ndm][nseg]
    double *mu, *sigma;      // [ndm][nseg]
    int32_t *T;              // integer thresholds [ndm][nseg][nw]
    const double *dms;       // [ndm]
    double theta;
    double fch1, foff;       // channel c has centre fch1 + c*foff (MHz)
    double fref, flo;        // highest and lowest channel centres (MHz)
    double tsamp;            // s
    int32_t n_in;            // samples per channel the block carries
    int32_t nch, ndm, ndm_pad, n_dd, n_out, L, nseg, nw;
    int32_t xpitch;          // int32 elements per DM row
    int32_t row_base;        // global row index of (beam, d = 0)
    int32_t chunk_base;      // global boxcar chunk of (d = 0, k = 0)
    int32_t nchunk_t;        // boxcar chunks per row
    int32_t chan_chunk;      // channels staged in LDS per step (power of two <= 256)
    int32_t lds_quarter;     // bytes per shifted copy of the staged rows in the LDS
    int32_t tile_dm;         // DM trials per dedispersion tile
    int32_t beam;
    int32_t w_max;
    int32_t nst;             // peak filters of this beam's plan
    int32_t rd[kMaxStencils], rt[kMaxStencils];
    int32_t widths[kMaxWidths];
};

// One dedispersion work item: a DM tile x time tile of one beam.
struct DedispItem {
    int32_t beam;
    int32_t d0;        // first DM trial of the tile
    int32_t t0;        // first output sample of the tile
    int32_t row_bytes; // LDS bytes per staged channel row of one copy (multiple of 16)
};

// A boxcar hit: one (row, t) above threshold with its best width.
struct Hit {
    int32_t row;   // global row (beam's row_base + DM index)
    int32_t t;
    int32_t w;
    int32_t B;
    double snr;
};
static_assert(sizeof(Hit) == 24, "Hit layout");

// Per-run device state kept in the scratch part of the workspace.
struct DevRun {
    int64_t n_hits;        // true hit count of the beams in flight
    int64_t n_cand_total;  // candidates written so far (all beams)
    int64_t n_cand_beam;   // candidates of the beams in flight
    int64_t n_alive[kMaxStencils];
    int64_t n_surv;        // survivors of the first peak filter (the compacted list's length)
    int32_t hit_overflow;
    int32_t queue[kMaxShapeGroups];  // persistent-kernel work counters
    int32_t box_stall;     // 1: a boxcar look-back gave up waiting (hit offsets invalid)
};

}  // namespace spl

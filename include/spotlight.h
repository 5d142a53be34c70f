/*
 * spotlight.h -- C ABI of libspotlight.so, an MI355X (gfx950) implementation of
 * the data-parallel hot path of the SPOTLIGHT real-time transient search:
 * brute-force incoherent dedispersion of 8-bit multibeam filterbank blocks over
 * a grid of trial DMs, the single-pulse search (boxcar matched filters of
 * several widths, mean/sigma normalisation, S/N threshold, best width) and peak
 * filtering into a candidate list (beam, DM, time, width, S/N).
 *
 * The problem statement follows the paper's "Dedispersion", "Single pulse
 * search" and "Candidate optimisation" sections and Eq. (1).
 *
 * Conventions shared by every call
 *  - Every function returns spl_status (SPL_OK = 0) and never throws; on error
 *    a message for the calling thread is available from spl_last_error().
 *  - Handles (spl_plan, spl_batch, spl_ranker) are opaque host objects.  They
 *    are not thread-safe: use one handle from one thread (and one stream) at a
 *    time.  Plans may be shared read-only by several batches.
 *  - Ownership: the caller owns every device buffer (input blocks, workspace,
 *    candidate buffer, run statistics, snippets, scores) and every stream.  The
 *    library allocates host memory only, plus pinned host staging buffers; it
 *    never calls hipMalloc.  Calls that take a stream only enqueue work on it;
 *    device pointers must stay valid until the stream has passed that work.
 *  - Device pointers are plain addresses from hipMalloc (or a caching allocator
 *    on top of it) on the current HIP device.
 */
#ifndef SPOTLIGHT_H_
#define SPOTLIGHT_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
typedef int32_t spl_status;
#define SPL_OK 0
#define SPL_E_INVALID_ARG 1  /* an argument is out of range or inconsistent   */
#define SPL_E_HIP 2          /* a HIP runtime call failed                      */
#define SPL_E_OOM 3          /* host allocation failed or workspace too small  */
#define SPL_E_CAPACITY 4     /* a result exceeded the capacity given           */
#define SPL_E_UNSUPPORTED 5  /* valid input the library cannot process exactly */
#define SPL_E_NO_WEIGHTS 6   /* the ranker has no weights: use the plain path  */
#define SPL_E_INTERNAL 7

/* Message describing the last failure on the calling thread ("" if none). */
const char *spl_last_error(void);
/* Library ABI version (major*10000 + minor*100 + patch). */
int32_t spl_version(void);

/* ------------------------------------------------------------------- plans */
/*
 * Observation band of one beam.
 *   nchans      channels per block row; channel c has centre frequency
 *               fch1_mhz + c*foff_mhz.  The reference frequency of Eq. (1) is
 *               the highest channel centre (usually channel 0: the paper's
 *               pipeline flips bands so that the highest frequency comes first;
 *               either sign of foff_mhz is accepted).
 *   tsamp_s     sampling interval in seconds.
 *   n_out       samples owned by one block: candidates are searched at times
 *               t in [0, n_out).  The block itself must carry n_in samples per
 *               channel (spl_plan_info.n_in): the owned samples plus the
 *               overlap tail of w_max - 1 + s_max samples needed to complete
 *               every boxcar and every dispersion sweep (the paper reads blocks
 *               with an overlap for the same reason).
 *   norm_window length L of the segments over which mean and sigma of each DM
 *               row are measured (0 means n_out).  Segment k covers owned
 *               samples [k*L, min((k+1)*L, n_out)).
 */
typedef struct spl_band {
    int32_t nchans;
    int32_t n_out;
    int32_t norm_window;
    int32_t reserved0;
    double fch1_mhz;
    double foff_mhz;
    double tsamp_s;
} spl_band;

/* A sub-range of the DM plan: trials dm_start + k*dm_step, k < n_trials
 * (pc cm^-3).  Sub-ranges are concatenated in the order given. */
typedef struct spl_dm_range {
    double dm_start;
    double dm_step;
    int32_t n_trials;
    int32_t reserved0;
} spl_dm_range;

#define SPL_MAX_STENCILS 4
/* Peak filters applied in order (the paper uses a 3x3 then an 11x11 window in
 * the DM-time plane).  Filter k keeps a point when no other surviving point
 * within |dDM index| <= rd[k] and |dt| <= rt[k] has a larger key
 * (S/N, -DM index, -t).  Passing NULL selects {(1,1), (5,5)}. */
typedef struct spl_search_opts {
    int32_t n_stencils;
    int32_t stencil_rd[SPL_MAX_STENCILS];
    int32_t stencil_rt[SPL_MAX_STENCILS];
} spl_search_opts;

typedef struct spl_plan spl_plan;

typedef struct spl_plan_info {
    int32_t nchans;
    int32_t ndm;          /* DM trials, all sub-ranges */
    int32_t n_out;
    int32_t n_dd;         /* dedispersed samples per DM row: n_out + w_max - 1 */
    int32_t n_in;         /* input samples per channel a block must carry: n_dd + s_max */
    int32_t s_max;        /* largest delay in the table (samples) */
    int32_t n_widths;
    int32_t w_max;
    int32_t norm_window;
    int32_t n_segments;
    int32_t n_stencils;
    int32_t reserved0;
    double threshold;     /* S/N threshold in sigma */
} spl_plan_info;

/*
 * DM sub-ranges whose trial spacing keeps the dispersive smearing small (dedispersion
 * section: a plan divides the DM range into sub-ranges whose spacing depends on the
 * sampling time, the channel width and the bandwidth).  The S/N kept by a Gaussian pulse
 * of FWHM W dedispersed dDM off its DM is (sqrt(pi)/2) erf(z)/z with
 * z = 6.91e-3 * dDM * B_MHz / (W_ms * nu_GHz^3) (Eq. snrloss and Eq. zetadef; B the
 * bandwidth nchans*|foff|, nu the centre frequency); the narrowest pulse a trial at DM can
 * see has W_ms = sqrt(w_min_ms^2 + tsamp_ms^2 + t_chan^2), t_chan = 8.3e-3 * DM *
 * |foff| / nu_lo_GHz^3 ms the smearing within one channel at the lowest channel centre.
 * A step s is allowed at DM when the pulse half a step off keeps at least
 * 1 - max_loss of its S/N.  Steps are powers of two: the first the largest allowed at
 * dm_min; a sub-range ends at the first of its trials (after the first) where twice its
 * step is allowed, and the next starts there with the doubled step; trials continue
 * until the first one >= dm_max.  All in binary64 in this order.
 */
typedef struct spl_smearing_opts {
    double dm_min, dm_max;  /* 0 <= dm_min < dm_max                                  */
    double max_loss;        /* fraction of S/N a pulse half a step off may lose, (0, 1) */
    double w_min_s;         /* narrowest intrinsic pulse width considered (>= 0, s)    */
} spl_smearing_opts;

/* Writes up to `capacity` sub-ranges to `out` and their number to *n_out
 * (SPL_E_CAPACITY if more are needed). */
spl_status spl_plan_smearing_ranges(const spl_band *band, const spl_smearing_opts *opts, spl_dm_range *out,
                                    int32_t capacity, int32_t *n_out);

/*
 * Build a plan: DM trials from the sub-ranges, the integer delay table
 *   delay[d][c] = round-half-away( ((D * DM_d) * (1/f_c^2 - 1/f_ref^2)) / tsamp )
 * of Eq. (1) with D = 4148.8064239 MHz^2 pc^-1 cm^3 s evaluated in binary64 in
 * exactly this order, boxcar widths (strictly ascending, 1 <= w <= n_out) and
 * the S/N threshold (> 0).  Each 8-bit sample sum must fit int32:
 * nchans * 255 * w_max < 2^31, else SPL_E_UNSUPPORTED.  *out receives a new
 * plan owned by the caller (spl_plan_destroy).
 */
spl_status spl_plan_create(const spl_band *band, const spl_dm_range *ranges, int32_t n_ranges,
                           const int32_t *widths, int32_t n_widths, double threshold,
                           const spl_search_opts *opts, spl_plan **out);

/*
 * As spl_plan_create, with an explicit host delay table delays[ndm][nchans]
 * (non-negative int32, row-major by DM trial) and the DM value of each row
 * (host, ndm doubles, used only for reporting).  Intended for tests.
 */
spl_status spl_plan_create_from_delays(const spl_band *band, const int32_t *delays,
                                       const double *dms, int32_t ndm, const int32_t *widths,
                                       int32_t n_widths, double threshold,
                                       const spl_search_opts *opts, spl_plan **out);

spl_status spl_plan_query(const spl_plan *plan, spl_plan_info *info);
/* Copy the plan's delay table into host memory delays[ndm][nchans] (int32). */
spl_status spl_plan_delays(const spl_plan *plan, int32_t *host_out);
/* Copy the plan's DM values into host memory (ndm doubles). */
spl_status spl_plan_dms(const spl_plan *plan, double *host_out);
void spl_plan_destroy(spl_plan *plan);

/* ----------------------------------------------------------------- batches */
#define SPL_MODE_PLAIN_PER_BEAM 0   /* one launch sequence per beam, no graph     */
#define SPL_MODE_PERSISTENT_GRAPH 1 /* all beams in one persistent launch, the    */
                                    /* whole sequence captured once in a hipGraph */

typedef struct spl_batch_opts {
    int32_t mode;
    int32_t reserved0;
    int64_t hit_capacity;  /* boxcar hits held between search and peak filter;
                              0: one per 16 owned (DM trial, sample) cells, at least 2^24 */
} spl_batch_opts;

/*
 * Candidate record (32 bytes).  dm_index counts rows of the beam's plan; dm is
 * that row's DM as float; snr is the binary64 S/N rounded to float; flags is 0
 * from the search (the plain optimisation path and the ranker use it).
 */
typedef struct spl_candidate {
    int32_t beam;
    int32_t dm_index;
    int32_t t_sample;
    int32_t width;
    int32_t boxcar_sum;
    float snr;
    float dm;
    uint32_t flags;
} spl_candidate;

/* Written to device memory by every run. */
typedef struct spl_run_stats {
    int64_t n_hits;                          /* boxcar hits above threshold (true count) */
    int64_t n_candidates;                    /* candidates after the peak filters (true count) */
    int64_t n_after_stencil[SPL_MAX_STENCILS];
    int32_t hit_overflow;                    /* 1: n_hits exceeded the hit capacity; 2: the
                                                ordered hit compaction gave up waiting for a
                                                chunk's predecessors (not expected: the hit
                                                list and candidates are then invalid) */
    int32_t cand_overflow;                   /* 1: n_candidates exceeded the caller's capacity */
} spl_run_stats;

typedef struct spl_batch spl_batch;

/*
 * A batch searches n_beams beams per run, beam b with plans[b] (plans may
 * differ in every parameter).  The plans must outlive the batch.
 */
spl_status spl_batch_create(const spl_plan *const *plans, int32_t n_beams,
                            const spl_batch_opts *opts, spl_batch **out);
/*
 * Device workspace of the batch, one allocation of *persistent + *scratch bytes: the
 * first *persistent bytes hold the plan tables, work items and beam descriptors
 * (written by spl_batch_set_workspace, read by every run); the *scratch bytes after
 * them hold each run's intermediates (DM transforms, moments, thresholds, hit lists,
 * peak-filter state, run counters), overwritten by every run.
 */
spl_status spl_batch_workspace_size(const spl_batch *batch, size_t *persistent, size_t *scratch);
/*
 * Attach a caller-owned device workspace of at least the size above (256-byte
 * aligned) and upload the plan tables into it (synchronous).  Must be called
 * before the first run and again after spl_batch_set_tiles / spl_autotune
 * changed the tiling.
 */
spl_status spl_batch_set_workspace(spl_batch *batch, void *d_ws, size_t bytes);

/*
 * Enqueue one search of one block per beam on `stream`.
 *   d_blocks[b]  device pointer to beam b's block, uint8 [nchans][pitch],
 *                channel-major, 16-byte aligned, holding at least n_in valid
 *                samples per row.
 *   pitches[b]   row pitch in bytes, a multiple of 16, >= n_in.
 *   d_cands      device buffer of `capacity` records; receives the candidates
 *                of all beams sorted by (beam, dm_index, t_sample).  If there
 *                are more than `capacity`, the first `capacity` in that order
 *                are written and d_stats->cand_overflow is set.
 *   d_stats      device spl_run_stats, written by the run.
 * Host arrays d_blocks/pitches are read before the call returns.  Results are
 * complete when the stream reaches the end of the enqueued work; a run with
 * d_stats->hit_overflow set is incomplete (raise the hit capacity).
 */
spl_status spl_batch_run(spl_batch *batch, const uint8_t *const *d_blocks, const int64_t *pitches,
                         spl_candidate *d_cands, int64_t capacity, spl_run_stats *d_stats,
                         hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): spl_batch_run with the batch's
 * workspace replaced, for this call, by a static device array of the library
 * (SPL_STATIC_SCRATCH_BYTES per GPU, reserved on each GPU the library runs on until
 * the process ends).  Same arguments, results and candidate order as spl_batch_run;
 * no spl_batch_set_workspace is needed, and the call allocates nothing on the device
 * (no hipMalloc, no graph; the run is enqueued eagerly in every mode).
 *   - SPL_E_UNSUPPORTED when spl_batch_workspace_size exceeds SPL_STATIC_SCRATCH_BYTES
 *     (create the batch with a smaller hit_capacity, or fewer or smaller beams).
 *   - The current device must be the stream's device.
 *   - The call first waits for the work already enqueued on `stream`, then copies the
 *     batch's plan tables into the array (synchronous host-to-device copies) and
 *     enqueues the run.  Every call on one GPU shares that GPU's array, which keeps
 *     the last call's contents: calls on one GPU whose runs overlap in time (other
 *     streams, other threads) race and give undefined results.
 *   - The batch's own workspace, descriptors and captured graph are left unchanged;
 *     spl_batch_dm_transform and spl_batch_moments keep reading that workspace, and
 *     spl_ranker_snippets must not be given a batch whose last run was this one.
 */
#define SPL_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
spl_status spl_batch_run_static(spl_batch *batch, const uint8_t *const *d_blocks, const int64_t *pitches,
                                spl_candidate *d_cands, int64_t capacity, spl_run_stats *d_stats,
                                hipStream_t stream);

/* Read-only device views of the last run's intermediate results of one beam:
 * the DM transform int32 [ndm][pitch_elems] (valid columns 0..n_dd-1) and the
 * segment moments int64 S1[ndm][n_segments], S2[ndm][n_segments]. */
spl_status spl_batch_dm_transform(const spl_batch *batch, int32_t beam, const int32_t **d_X,
                                  int64_t *pitch_elems);
spl_status spl_batch_moments(const spl_batch *batch, int32_t beam, const int64_t **d_S1,
                             const int64_t **d_S2);

/* Dedispersion tiling of one beam: a workgroup of `waves` wavefronts sums a tile of
 * waves*dm_per_wave DM trials by time_groups*256 samples; chan_chunk channels are staged
 * in LDS per step (a power of two in [2, 2*waves] with one buffer, [2, waves] with two;
 * 0: the largest that fits the LDS budget, 64 KiB for 4 and 8 wavefronts, which share a
 * CU with other workgroups, and the whole LDS for 16).  With two LDS buffers (16-wavefront tiles
 * only) the next chunk is staged while the current one is summed.  The compiled shapes
 * (dm_per_wave, time_groups, waves[, buffers]): (2,2,8) (4,1,4) (4,2,4) (4,1,8) (4,2,8)
 * (8,1,4) (8,1,8), and (4,1,16) (4,2,16) (2,2,16) with one or two buffers. */
typedef struct spl_tiles {
    int32_t dm_per_wave;
    int32_t time_groups;
    int32_t chan_chunk;
    int32_t waves;       /* 4, 8 or 16; 0 selects 4 */
    int32_t buffers;     /* LDS buffers, 1 or 2; 0 selects 1 */
} spl_tiles;
spl_status spl_batch_get_tiles(const spl_batch *batch, int32_t beam, spl_tiles *tiles);
/* Set the tiling of every beam sharing beam's plan; SPL_E_UNSUPPORTED if the shape is
 * not compiled in, does not fit the LDS or a tile's delay spread exceeds the staged
 * rows.  Call spl_batch_set_workspace afterwards. */
spl_status spl_batch_set_tiles(spl_batch *batch, int32_t beam, const spl_tiles *tiles);

/* Stage timing.  With profiling on, every run executes its launch sequence eagerly
 * (no graph) and records a pair of timing events on the run's stream around each
 * stage of each pass.  spl_batch_stage_times waits for the recorded events, adds
 * their elapsed times (ms) and counts to running totals and returns the totals in
 * ms[SPL_N_STAGES] and count[SPL_N_STAGES] (either may be NULL); reset != 0 clears
 * the totals afterwards.  Stage DEDISP covers the dedispersion kernel launches only. */
#define SPL_STAGE_DEDISP 0     /* brute-force dedispersion                      */
#define SPL_STAGE_THRESHOLDS 1 /* moments, mean/sigma, integer thresholds       */
#define SPL_STAGE_BOXCAR 2     /* boxcar filters, hit counting and emission     */
#define SPL_STAGE_PEAKS 3      /* peak filters and candidate compaction         */
#define SPL_N_STAGES 4
spl_status spl_batch_set_profiling(spl_batch *batch, int32_t enable);
spl_status spl_batch_stage_times(spl_batch *batch, double *ms, int64_t *count, int32_t reset);

/*
 * Autotuner: for every distinct plan of the batch, time the dedispersion kernel on the
 * given blocks (uint8 [nch][pitch] device blocks as for spl_batch_run) for every compiled
 * tile shape and staging depth that fits, check that each shape gives a bit-identical DM
 * transform (SPL_E_INTERNAL otherwise), and keep the fastest.  Results are cached in the
 * text file cache_path (NULL: no cache), one line per plan signature (sizes and a hash of
 * the delay table); a cached plan is not re-timed unless flags has SPL_TUNE_FORCE.
 * Synchronous on `stream`; overwrites the batch's intermediate results and uses only the
 * attached workspace (which is sized for every tiling).
 */
#define SPL_TUNE_FORCE 1
spl_status spl_autotune(spl_batch *batch, const uint8_t *const *d_blocks, const int64_t *pitches,
                        const char *cache_path, int32_t flags, hipStream_t stream);

void spl_batch_destroy(spl_batch *batch);

/* ------------------------------------------------- plain optimisation path */
/* Parameters of the candidate-optimisation stage (candidate optimisation section):
 * DBSCAN with radius eps and min_pts points (a point counts itself) on the plane
 * (t_sample*tsamp/t_scale_s, dm/dm_scale); thresholds S/N >= snr_min, DM >= dm_min,
 * width*tsamp <= width_max_s; with at least coinc_min_beams beams, a candidate is
 * dropped when more than coinc_frac of the beams hold a thresholded candidate within
 * coinc_dt_s of its arrival time. */
typedef struct spl_opt_params {
    double eps;
    int32_t min_pts;
    int32_t coinc_min_beams;
    double t_scale_s;
    double dm_scale;
    double snr_min;
    double dm_min;
    double width_max_s;
    double coinc_dt_s;
    double coinc_frac;
} spl_opt_params;

/* eps 0.5, min_pts 5, 50 ms and 20 pc cm^-3 units, S/N 10, DM 10, width 100 ms,
 * anti-coincidence over >= 3 beams within 50 ms in more than half of them. */
void spl_opt_defaults(spl_opt_params *params);

/*
 * Host-side plain path applied to host candidate records (any order; beam in
 * [0, n_beams)); tsamp_of_beam[b] is beam b's sampling interval.  Per beam the
 * records are taken in (dm_index, t_sample) order; DBSCAN clusters are the connected
 * components of core points, numbered by their lowest-index core point; a border
 * point joins the lowest-numbered cluster among its core neighbours; noise is
 * dropped and each cluster keeps its highest-S/N member (equal S/N: the earlier
 * one).  Survivors of the thresholds and the anti-coincidence filter are written to
 * `out` sorted by (beam, dm_index, t_sample); *n_out receives their number;
 * SPL_E_CAPACITY if it exceeds `capacity` (the first `capacity` are written).
 * params NULL selects the defaults.
 */
spl_status spl_optimise_plain(const spl_candidate *cands, int64_t n, const double *tsamp_of_beam,
                              int32_t n_beams, const spl_opt_params *params, spl_candidate *out,
                              int64_t capacity, int64_t *n_out);

/* --------------------------------------------------------- stream device ring */
/*
 * Continuous beam streams (the paper reads each block with an overlap so that every
 * dispersion sweep and boxcar of its owned samples is complete): block k of a beam reads
 * stream samples [k n_out, k n_out + n_in) (n_out, n_in of the beam's plan), so the next
 * block starts with the last carry = n_in - n_out = s_max + w_max - 1 samples of the
 * previous one.  Only the n_out new samples cross the host link: the caller copies them
 * into a device staging buffer (one contiguous copy from pinned memory), and
 *   d_next[c][j] = d_prev[c][n_out + j]        for j <  carry
 *   d_next[c][j] = d_stage[c][j - carry]       for carry <= j < n_in
 * for every channel c < nch.  d_next, d_prev: device blocks uint8 [nch][pitch]
 * (pitches >= n_in, multiples of 16; pointers 16-byte aligned; not overlapping; d_prev
 * may be NULL when carry = 0).  d_stage: device uint8 [nch][stage_pitch], stage_pitch >=
 * n_out and a multiple of 4, pointer 4-byte aligned, with at least 16 readable bytes
 * after the last row's n_out-th byte (rows are read in aligned dwords).  n_out a
 * multiple of 16.  Bytes of d_next beyond n_in are left unchanged.  Asynchronous on
 * `stream`: the caller orders it after the copy into d_stage and before the search of
 * d_next, and keeps d_prev unchanged until it has run.  SPL_E_INVALID_ARG on NULL
 * pointers, sizes or alignments out of range, or overlapping buffers.
 */
spl_status spl_stream_assemble(uint8_t *d_next, int64_t next_pitch, const uint8_t *d_prev, int64_t prev_pitch,
                               const uint8_t *d_stage, int64_t stage_pitch, int32_t nch, int64_t n_out,
                               int64_t n_in, hipStream_t stream);

/* ------------------------------------------------------------------ corner turn */
/*
 * Filterbank files hold one spectrum after another (time-major: all channels of
 * sample 0, then of sample 1, ...; the paper's beams arrive this way, the
 * observation-overview section), while the search reads one row of samples per
 * channel.  out[c][t] = in[t][c] for t < n_t, c < nch: d_in device [n_t][in_stride]
 * bytes, d_out device [nch][pitch] bytes; bytes t >= n_t of each output row are left
 * unchanged.  nch a multiple of 16 (else SPL_E_UNSUPPORTED); in_stride >= nch and
 * pitch >= n_t, both multiples of 16; both buffers 16-byte aligned and not
 * overlapping.  Channel order is kept.  Asynchronous on `stream`.
 */
spl_status spl_corner_turn(const uint8_t *d_in, int64_t n_t, int32_t nch, int64_t in_stride, uint8_t *d_out,
                           int64_t pitch, hipStream_t stream);

/* ------------------------------------------------------------ candidate ranker */
/*
 * Feature snippets and the CNN that ranks candidates (classification section of the
 * paper: a learned classifier on the DM-time and frequency-time images of each
 * candidate; here a small CNN of the same two inputs).
 *
 * Snippet of a candidate (beam b, trial d*, sample t*): two 64 x 256 BF16 planes,
 * [n][2][64][256] row-major, columns t*-128 .. t*+127:
 *   plane 0 (DM-time): rows d*-32 .. d*+31 of beam b's DM transform, each row
 *     standardised with the search's own (mu, sigma) of that row's normalisation
 *     segment containing t*;
 *   plane 1 (frequency-time): 64 sub-bands of nch/64 adjacent channels, each the sum of
 *     x[c][t + s[d*][c]] over its channels, standardised over its in-range samples with
 *     the same exact-moment recipe.
 * Entries outside [0, ndm) or outside [0, n_dd) are 0, as is every entry of a row with
 * sigma = 0.  Value = BF16(round-to-nearest-even(float((v - mu)/sigma))), the quotient
 * in binary64.
 */
#define SPL_SNIPPET_ROWS 64
#define SPL_SNIPPET_COLS 256
#define SPL_SNIPPET_ELEMS (2 * SPL_SNIPPET_ROWS * SPL_SNIPPET_COLS)

/* Snippets of n device candidate records of the batch's last run (its blocks and DM
 * transforms must still be resident: the workspace and the blocks given to the last
 * spl_batch_run).  d_out: device BF16 [n][2][64][256].  Every plan of the batch needs
 * nchans a multiple of 64 (else SPL_E_UNSUPPORTED).  A record whose beam, dm_index or
 * t_sample lies outside the batch (t_sample >= n_out) yields two zero planes.
 * Asynchronous on `stream`. */
spl_status spl_ranker_snippets(const spl_batch *batch, const spl_candidate *d_cands, int64_t n, uint16_t *d_out,
                               hipStream_t stream);

/*
 * As spl_ranker_snippets, with plane 0 replaced by the fine-DM DM-time plane (the
 * classification section: the DM transform over a narrow DM range centred on the
 * candidate's DM, its half-width the DM offset that costs a pulse of the candidate's
 * width all but `keep` of its S/N).  Half-width dDM = (sqrt(pi)/2 / keep) * W_ms *
 * nu_GHz^3 / (6.91e-3 * B_MHz) from Eq. snrloss at large zeta and Eq. zetadef (the
 * paper's Eq. deltadm with its unit conversion redone), W = width * tsamp, nu the band
 * centre, B = nchans * |foff|; all binary64 in this order.  Row r (0..63) is the
 * brute-force dedispersion of the batch's block at DM = DM_d* + (r - 32) * dDM/32 with
 * delays of Eq. (1) computed as a plan computes them, over samples t*-128 .. t*+127; an
 * entry is valid when every channel's sample lies in [0, n_in).  The valid entries are
 * standardised together by mu, sigma from their exact integer moments (value as in
 * plane 1); invalid entries are 0.  keep in (0, 1) (the paper's default 0.1); nchans
 * <= 16384 (else SPL_E_UNSUPPORTED); a record with width < 1 or outside the batch
 * yields zero planes.  Asynchronous on `stream`.
 */
spl_status spl_ranker_snippets_fine(const spl_batch *batch, const spl_candidate *d_cands, int64_t n, double keep,
                                    uint16_t *d_out, hipStream_t stream);

/* The network: 4 x [3x3 convolution (zero padding 1) + bias -> ReLU -> 2x2 max pool]
 * with channels 2 -> 32 -> 32 -> 32 -> 32 (64x256 -> 4x16), flatten in (channel, row,
 * column) order -> fully connected 2048 -> 64 -> ReLU -> 64 -> 1 = logit; probability
 * sigmoid(logit); loss = mean binary cross-entropy with logits.  Parameters, FP32, in
 * this order: c1w [32][2][3][3], c1b [32], c2w [32][32][3][3], c2b, c3w, c3b, c4w, c4b,
 * f1w [64][2048], f1b [64], f2w [1][64], f2b [1] (159,553 values).  Convolutions and
 * the first fully connected layer run on BF16 matrix cores with FP32 accumulation;
 * activations are rounded to BF16 between layers; Adam updates FP32 master weights. */
#define SPL_RANKER_PARAMS 159553

typedef struct spl_ranker spl_ranker;

typedef struct spl_ranker_opts {
    int32_t max_batch;  /* candidates per pass, 1 .. 1024 (rounded up to 32 inside)   */
    int32_t reserved0;
    float beta1, beta2, eps;  /* Adam; zero selects 0.9, 0.999, 1e-8                 */
    float reserved1;
} spl_ranker_opts;

/* New ranker handle (host only; no weights yet). */
spl_status spl_ranker_create(const spl_ranker_opts *opts, spl_ranker **out);

/* Device workspace bytes (weights, Adam state, activations of max_batch candidates). */
spl_status spl_ranker_workspace_size(const spl_ranker *r, size_t *bytes);

/* Attach a caller-owned device workspace (256-byte aligned) of at least the size above;
 * uploads the packing tables (synchronous).  Attaching again forgets the weights. */
spl_status spl_ranker_set_workspace(spl_ranker *r, void *d_ws, size_t bytes);

/* Host FP32 parameters [SPL_RANKER_PARAMS] in the order above -> device master weights;
 * resets the Adam moments and step count.  Synchronous. */
spl_status spl_ranker_set_weights(spl_ranker *r, const float *host_params);

/* Device master weights -> host [SPL_RANKER_PARAMS] (synchronises `stream`). */
spl_status spl_ranker_get_weights(const spl_ranker *r, float *host_params, hipStream_t stream);

/* Logits of n snippets (device BF16 [n][2][64][256]) into d_logits [n] (device FP32),
 * in passes of max_batch.  SPL_E_NO_WEIGHTS before spl_ranker_set_weights: the caller
 * then keeps the plain path (spl_optimise_plain). */
spl_status spl_ranker_score(spl_ranker *r, const uint16_t *d_snip, int64_t n, float *d_logits, hipStream_t stream);

/* Forward and backward pass of n <= max_batch snippets with labels d_labels [n] (device
 * FP32, 0 or 1): d_loss [1] receives the mean BCE loss and the gradients of every
 * parameter are left in the ranker (spl_ranker_grads).  No update. */
spl_status spl_ranker_backward(spl_ranker *r, const uint16_t *d_snip, const float *d_labels, int64_t n,
                               float *d_loss, hipStream_t stream);

/* spl_ranker_backward followed by one Adam step with learning rate lr. */
spl_status spl_ranker_train_step(spl_ranker *r, const uint16_t *d_snip, const float *d_labels, int64_t n, float lr,
                                 float *d_loss, hipStream_t stream);

/* Device view of the last gradients, FP32 [SPL_RANKER_PARAMS] in parameter order. */
spl_status spl_ranker_grads(const spl_ranker *r, const float **d_grads);

void spl_ranker_destroy(spl_ranker *r);

/*
 * The anti-coincidence step of the plain path on its own, for pipelines that put
 * another stage (the ranker) between the thresholds and this filter: with at least
 * params->coinc_min_beams beams, a record is dropped when more than
 * params->coinc_frac * n_beams beams hold a record (of `cands`) within
 * params->coinc_dt_s of its arrival time t_sample * tsamp_of_beam[beam].  Survivors
 * are written to `out` sorted by (beam, dm_index, t_sample); *n_out receives their
 * number; SPL_E_CAPACITY if it exceeds `capacity`.  Host records; params NULL selects
 * the defaults.
 */
spl_status spl_anti_coincidence(const spl_candidate *cands, int64_t n, const double *tsamp_of_beam,
                                int32_t n_beams, const spl_opt_params *params, spl_candidate *out,
                                int64_t capacity, int64_t *n_out);

/* ---------------------------------------------------- quantised-domain injection */
/*
 * Injection of a simulated signal into data that is already quantised (the real-time
 * injector of the injection section; the rules are the appendix on M-bit quantised
 * streams).  The quantiser maps Gaussian noise N ~ Normal(mu, sigma) to 2^bits states:
 * state n < 2^bits - 1 ends at edge e_n = mu + (n + 1 - 2^(bits-1) + offset) * level *
 * sigma, state 0 starts at -inf and the top state ends at +inf.  offset = 0 is the
 * appendix's quantiser; -0.5 is clip(round(mu + x)) when level * sigma = 1.
 */
typedef struct spl_quantiser {
    int32_t bits;     /* 1..8; one state per byte, 0 .. 2^bits - 1 */
    int32_t reserved; /* 0 */
    double mu;        /* noise mean, in the units of the signal */
    double sigma;     /* noise standard deviation, > 0 */
    double level;     /* state width in units of sigma, > 0 */
    double offset;    /* shift of every edge, in states; finite */
} spl_quantiser;

enum {
    SPL_INJECT_SAMPLE = 0, /* draw the new state from the transition row (inverse CDF at u) */
    SPL_INJECT_ARGMAX = 1  /* the most probable state of the row, the smaller one on ties */
};

/*
 * Adds n_win windows of signal to a quantised block in place.  Window w adds
 * d_signal[w][c][j] (FP32, the units of mu and sigma) to sample d_t_start[w][c] + j of
 * channel c (int32 starts; samples outside [0, n_t) are skipped, so a burst may cross
 * the block's ends).  A sample in state n with signal S > 0 moves to state k with the
 * probability P(n -> k) of the appendix's transition matrix: the Gaussian mass of the
 * part of state n that the shift by S carries into state k, over the mass of state n.
 * SAMPLE mode takes the smallest k whose cumulative row sum exceeds
 * u = (d_random[w][c][j] + 1/2) * 2^-32 (caller-supplied uniform 32-bit words, same
 * layout as d_signal; NULL is allowed in ARGMAX mode).  A sample is left unchanged when
 * S <= 0 or NaN, when its byte exceeds 2^bits - 1, or when its state has no binary64
 * Gaussian mass.  Probabilities are evaluated in binary64.
 * d_block device [nch][pitch] bytes; pitch >= n_t.  Windows of one call must not cover
 * the same sample twice (such calls race); successive calls on one stream apply in
 * order.  Asynchronous on `stream`.
 */
spl_status spl_inject_quantised(uint8_t *d_block, int64_t pitch, int64_t n_t, int32_t nch, const int32_t *d_t_start,
                                const float *d_signal, const uint32_t *d_random, int32_t n_win, int32_t n_sig,
                                const spl_quantiser *q, int32_t mode, hipStream_t stream);

/* ------------------------------------------------------------- test hooks */
/* The normaliser of the search on device, for parity tests: for i < count,
 * mu[i] = S1/n and sigma[i] = sqrt(n*S2 - S1^2)/n (exact 128-bit difference,
 * rounded once to binary64; sigma = 0 when the difference is 0), from int64 device
 * arrays n, s1, s2 (n > 0, s1 >= 0, s2 >= 0) into double device arrays. */
spl_status spl_debug_mu_sigma(const int64_t *d_n, const int64_t *d_s1, const int64_t *d_s2, int64_t count,
                              double *d_mu, double *d_sigma, hipStream_t stream);

/* Device view of the max-pool decisions of conv layer `layer` (0..3) of the ranker's
 * last pass, for parity tests: bytes [Nb][H/2][W/2][32] (Nb = max_batch rounded up to
 * 32; H x W the layer's input size: 64x256, 32x128, 16x64, 8x32), each the window
 * position (row-major 0..3) of the first maximum of ReLU(conv + bias), or 255 when that
 * maximum is 0 (no gradient flows through the window). */
spl_status spl_ranker_debug_pool_args(const spl_ranker *r, int32_t layer, const uint8_t **d_arg);

/* Device view of the first fully connected layer's output before its bias, FP32
 * [Nb][64], of the ranker's last pass, for parity tests: the hidden unit j of candidate
 * n is active when (float)(h[n][j] + f1b[j]) > 0. */
spl_status spl_ranker_debug_fc_preact(const spl_ranker *r, const float **d_h);

/* The ranker's matrix-core product on device, for parity tests: C[M][N] (FP32, row
 * stride ldc) = A[M][K] * B[N][K]^T with A, B BF16 bit patterns (row strides lda, ldb
 * multiples of 8, 16-byte aligned), K a multiple of 32.  C is overwritten. */
spl_status spl_debug_gemm_bf16(const uint16_t *d_a, int64_t lda, const uint16_t *d_b, int64_t ldb, float *d_c,
                               int64_t ldc, int32_t m, int32_t n, int32_t k, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* SPOTLIGHT_H_ */

// Host runtime and C ABI of libspotlight: plans (the library's own binary64 delay
// table of Eq. (1)), batch layout in a caller-owned workspace, the launch sequence of
// a search run, and its capture into a hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "corner_turn.h"
#include "inject.h"
#include "kernels.h"
#include "ranker.h"
#include "spl_internal.h"
#include "spotlight.h"

#pragma STDC FP_CONTRACT OFF

using namespace spl;

// -------------------------------------------------------------------- errors
static thread_local std::string g_err;

static spl_status fail(spl_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e__ = (expr);                                                              \
        if (e__ != hipSuccess)                                                                \
            return fail(SPL_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e__),    \
                        __FILE__, __LINE__);                                                  \
    } while (0)

spl_status spl_internal_fail(spl_status st, const char *msg) { return fail(st, "%s", msg); }

extern "C" const char *spl_last_error(void) { return g_err.c_str(); }
extern "C" int32_t spl_version(void) { return 201; }

// --------------------------------------------------------------------- plans
static constexpr double kDispersionConstant = 4148.8064239;  // MHz^2 pc^-1 cm^3 s

struct spl_plan {
    spl_band band;
    std::vector<double> dms;
    std::vector<int32_t> delays;   // [ndm][nch]
    std::vector<int32_t> widths;
    double theta = 0;
    int nst = 2;
    int rd[kMaxStencils] = {1, 5, 0, 0};
    int rt[kMaxStencils] = {1, 5, 0, 0};
    int nch = 0, ndm = 0, n_out = 0, n_dd = 0, n_in = 0, s_max = 0, w_max = 0, L = 0, nseg = 0;
};

static spl_status check_common(const spl_band *band, const int32_t *widths, int32_t n_widths, double threshold,
                               const spl_search_opts *opts, spl_plan *p) {
    if (!band) return fail(SPL_E_INVALID_ARG, "band is NULL");
    if (band->nchans < 1) return fail(SPL_E_INVALID_ARG, "nchans must be >= 1 (got %d)", band->nchans);
    if (band->n_out < 1) return fail(SPL_E_INVALID_ARG, "n_out must be >= 1 (got %d)", band->n_out);
    if (!(band->tsamp_s > 0.0) || !std::isfinite(band->tsamp_s))
        return fail(SPL_E_INVALID_ARG, "tsamp_s must be finite and > 0");
    if (!std::isfinite(band->fch1_mhz) || !std::isfinite(band->foff_mhz))
        return fail(SPL_E_INVALID_ARG, "frequencies must be finite");
    const int L = band->norm_window ? band->norm_window : band->n_out;
    if (L < 1 || L > band->n_out) return fail(SPL_E_INVALID_ARG, "norm_window must be in [0, n_out]");
    if (!widths || n_widths < 1) return fail(SPL_E_INVALID_ARG, "at least one boxcar width is required");
    if (n_widths > kMaxWidths) return fail(SPL_E_UNSUPPORTED, "at most %d widths are supported", kMaxWidths);
    for (int i = 0; i < n_widths; ++i) {
        if (widths[i] < 1 || widths[i] > band->n_out)
            return fail(SPL_E_INVALID_ARG, "width %d out of [1, n_out]", widths[i]);
        if (i && widths[i] <= widths[i - 1]) return fail(SPL_E_INVALID_ARG, "widths must be strictly ascending");
    }
    const int w_max = widths[n_widths - 1];
    if (w_max > kMaxWmax) return fail(SPL_E_UNSUPPORTED, "w_max above %d is not supported", kMaxWmax);
    if (!(threshold > 0.0) || !std::isfinite(threshold)) return fail(SPL_E_INVALID_ARG, "threshold must be > 0");
    if ((int64_t)band->nchans * 255 * w_max >= ((int64_t)1 << 31))
        return fail(SPL_E_UNSUPPORTED, "nchans*255*w_max must be below 2^31 for exact int32 boxcars");
    const double xmax = (double)band->nchans * 255.0;
    if ((double)L * xmax * xmax >= 9.0e18)
        return fail(SPL_E_UNSUPPORTED, "segment sums of squares would overflow int64");
    for (int c = 0; c < band->nchans; ++c) {
        double f = band->fch1_mhz + (double)c * band->foff_mhz;
        if (!(f > 0.0)) return fail(SPL_E_INVALID_ARG, "channel %d has a non-positive frequency", c);
    }
    if (opts) {
        if (opts->n_stencils < 0 || opts->n_stencils > kMaxStencils)
            return fail(SPL_E_INVALID_ARG, "n_stencils must be in [0, %d]", kMaxStencils);
        p->nst = opts->n_stencils;
        for (int k = 0; k < p->nst; ++k) {
            if (opts->stencil_rd[k] < 0 || opts->stencil_rt[k] < 0 || opts->stencil_rd[k] > 1024 ||
                opts->stencil_rt[k] > 1024)
                return fail(SPL_E_INVALID_ARG, "stencil half-sizes must be in [0, 1024]");
            p->rd[k] = opts->stencil_rd[k];
            p->rt[k] = opts->stencil_rt[k];
        }
    }
    p->band = *band;
    p->band.norm_window = L;
    p->widths.assign(widths, widths + n_widths);
    p->theta = threshold;
    p->nch = band->nchans;
    p->n_out = band->n_out;
    p->w_max = w_max;
    p->L = L;
    p->nseg = (band->n_out + L - 1) / L;
    p->n_dd = band->n_out + w_max - 1;
    return SPL_OK;
}

static spl_status finish_plan(spl_plan *p) {
    int64_t smax = 0;
    for (int32_t v : p->delays) smax = std::max<int64_t>(smax, v);
    if ((int64_t)p->n_dd + smax > INT32_MAX / 2) return fail(SPL_E_UNSUPPORTED, "block length too large");
    p->s_max = (int)smax;
    p->n_in = p->n_dd + p->s_max;
    return SPL_OK;
}

extern "C" spl_status spl_plan_create(const spl_band *band, const spl_dm_range *ranges, int32_t n_ranges,
                                      const int32_t *widths, int32_t n_widths, double threshold,
                                      const spl_search_opts *opts, spl_plan **out) {
    if (!out) return fail(SPL_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ranges || n_ranges < 1) return fail(SPL_E_INVALID_ARG, "at least one DM range is required");
    spl_plan *p = new (std::nothrow) spl_plan();
    if (!p) return fail(SPL_E_OOM, "host allocation failed");
    spl_status st = check_common(band, widths, n_widths, threshold, opts, p);
    if (st != SPL_OK) { delete p; return st; }
    for (int k = 0; k < n_ranges; ++k) {
        const spl_dm_range &r = ranges[k];
        if (r.n_trials < 1 || !(r.dm_start >= 0.0) || !(r.dm_step >= 0.0) || !std::isfinite(r.dm_start) ||
            !std::isfinite(r.dm_step)) {
            delete p;
            return fail(SPL_E_INVALID_ARG, "DM range %d is invalid", k);
        }
        for (int d = 0; d < r.n_trials; ++d) p->dms.push_back(r.dm_start + (double)d * r.dm_step);
    }
    p->ndm = (int)p->dms.size();
    if ((int64_t)p->ndm * p->nch > ((int64_t)1 << 31)) { delete p; return fail(SPL_E_UNSUPPORTED, "plan too large"); }
    // Eq. (1): delay relative to the highest channel centre, rounded to the nearest
    // sample (half-way cases away from zero), evaluated in binary64 in this order.
    double fref = band->fch1_mhz;
    for (int c = 0; c < p->nch; ++c) fref = std::max(fref, band->fch1_mhz + (double)c * band->foff_mhz);
    p->delays.resize((size_t)p->ndm * p->nch);
    for (int d = 0; d < p->ndm; ++d) {
        for (int c = 0; c < p->nch; ++c) {
            const double f = band->fch1_mhz + (double)c * band->foff_mhz;
            const double v =
                ((kDispersionConstant * p->dms[d]) * ((1.0 / (f * f)) - (1.0 / (fref * fref)))) / band->tsamp_s;
            if (!(v < 1.0e9)) { delete p; return fail(SPL_E_UNSUPPORTED, "delay out of range"); }
            p->delays[(size_t)d * p->nch + c] = (int32_t)std::llround(v);
        }
    }
    st = finish_plan(p);
    if (st != SPL_OK) { delete p; return st; }
    *out = p;
    return SPL_OK;
}

extern "C" spl_status spl_plan_create_from_delays(const spl_band *band, const int32_t *delays, const double *dms,
                                                  int32_t ndm, const int32_t *widths, int32_t n_widths,
                                                  double threshold, const spl_search_opts *opts, spl_plan **out) {
    if (!out) return fail(SPL_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!delays || ndm < 1) return fail(SPL_E_INVALID_ARG, "a delay table with ndm >= 1 is required");
    spl_plan *p = new (std::nothrow) spl_plan();
    if (!p) return fail(SPL_E_OOM, "host allocation failed");
    spl_status st = check_common(band, widths, n_widths, threshold, opts, p);
    if (st != SPL_OK) { delete p; return st; }
    p->ndm = ndm;
    p->delays.assign(delays, delays + (size_t)ndm * p->nch);
    for (int32_t v : p->delays)
        if (v < 0) { delete p; return fail(SPL_E_INVALID_ARG, "delays must be non-negative"); }
    p->dms.resize(ndm);
    for (int d = 0; d < ndm; ++d) p->dms[d] = dms ? dms[d] : (double)d;
    st = finish_plan(p);
    if (st != SPL_OK) { delete p; return st; }
    *out = p;
    return SPL_OK;
}

extern "C" spl_status spl_plan_query(const spl_plan *p, spl_plan_info *info) {
    if (!p || !info) return fail(SPL_E_INVALID_ARG, "NULL argument");
    info->nchans = p->nch;
    info->ndm = p->ndm;
    info->n_out = p->n_out;
    info->n_dd = p->n_dd;
    info->n_in = p->n_in;
    info->s_max = p->s_max;
    info->n_widths = (int32_t)p->widths.size();
    info->w_max = p->w_max;
    info->norm_window = p->L;
    info->n_segments = p->nseg;
    info->n_stencils = p->nst;
    info->reserved0 = 0;
    info->threshold = p->theta;
    return SPL_OK;
}

extern "C" spl_status spl_plan_delays(const spl_plan *p, int32_t *host_out) {
    if (!p || !host_out) return fail(SPL_E_INVALID_ARG, "NULL argument");
    std::memcpy(host_out, p->delays.data(), p->delays.size() * sizeof(int32_t));
    return SPL_OK;
}

extern "C" spl_status spl_plan_dms(const spl_plan *p, double *host_out) {
    if (!p || !host_out) return fail(SPL_E_INVALID_ARG, "NULL argument");
    std::memcpy(host_out, p->dms.data(), p->dms.size() * sizeof(double));
    return SPL_OK;
}

extern "C" void spl_plan_destroy(spl_plan *p) { delete p; }

// ------------------------------------------------------------------- batches
namespace {

struct Tiles {
    int dw = 4, j = 2, nw = 8, cc = 0;
    int nb = 1;   // LDS buffers: 2 stages the next chunk while the current one is summed
    int sv = 1;   // staged 16-byte vectors per lane and row, from the widest row of the plan
};

// Everything that depends on one plan and its tiling.
struct PlanLayout {
    const spl_plan *plan = nullptr;
    Tiles tiles;
    int td = 0, ndm_pad = 0, ntile_d = 0, ntile_t = 0;
    std::vector<int32_t> dcm;        // delays [nch][ndm_pad]
    std::vector<int32_t> dtab;       // LDS byte offsets [nch][ndm_pad]
    int quarter = 0;                 // bytes per shifted copy of the staged rows
    std::vector<int32_t> tile_base;  // [ntile_d][nch]
    std::vector<int32_t> row_bytes;  // [ntile_d]
    size_t off_dcm = 0, off_base = 0, off_dms = 0, off_delays = 0;
};

struct Region {
    size_t off = 0, bytes = 0;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct spl_batch {
    std::vector<const spl_plan *> plans;  // per beam
    int nb = 0;
    int mode = SPL_MODE_PLAIN_PER_BEAM;
    int64_t hit_cap = 0;
    std::vector<PlanLayout> layouts;       // unique plans
    std::vector<int> layout_of_beam;
    // global indexing
    std::vector<int> row_base, chunk_base, item_base;   // [nb + 1]
    int n_rows = 0, n_chunks = 0, n_items = 0;
    int max_nst = 0, w_max = 0;
    std::vector<DedispItem> items;
    // shape groups for the persistent launch
    struct Group { int dw, j, nw, sv, nb; int item_lo, item_hi; size_t lds; int occ; };
    std::vector<Group> groups;
    std::vector<size_t> beam_lds;          // per beam (plain per-beam launches)
    // workspace
    size_t ws_bytes = 0, ws_given = 0;
    size_t ws_persistent = 0;   // the plan tables, work items and beam descriptors at the start
    char *ws = nullptr;
    size_t off_beams = 0, off_items = 0;
    std::vector<size_t> off_X, off_S, off_mu, off_sigma, off_T;   // per beam
    size_t off_S_all = 0, bytes_S_all = 0;
    size_t off_chunk_off = 0, off_block_sums = 0, off_row_start = 0, off_box_status = 0;
    size_t off_hits = 0, off_alive0 = 0, off_alive1 = 0, off_pos = 0, off_run = 0;
    size_t off_nms_blk = 0;   // block index of the hit rows [n_rows][nms_nblk] int32
    size_t off_hit_t = 0;     // the hits' times, packed int32 [hit_cap]
    size_t off_surv = 0;      // survivors of the first peak filter [hit_cap] Hit
    size_t off_surv_start = 0;   // their row starts [n_rows + 1] int64
    int nms_nblk = 0;
    int n_block_sums = 0;
    std::vector<int> xpitch;
    std::vector<DevBeam> host_beams;
    DevBeam *staging = nullptr;            // pinned copy of host_beams for async upload
    hipEvent_t staging_done = nullptr;
    bool staging_pending = false;
    std::vector<const uint8_t *> cur_x;
    std::vector<int64_t> cur_pitch;
    // stage timing (eager runs only): pairs of events per enqueued stage
    bool profiling = false;
    struct Timed { int stage; hipEvent_t a, b; };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> free_events;
    double stage_ms[SPL_N_STAGES] = {0};
    int64_t stage_count[SPL_N_STAGES] = {0};
    // graph cache
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    const void *g_cands = nullptr, *g_stats = nullptr;
    int64_t g_cap = -1;
    bool tables_uploaded = false;
};

static spl_status layout_plan(PlanLayout &L) {
    const spl_plan &p = *L.plan;
    if (!dedisp_shape_supported(L.tiles.dw, L.tiles.j, L.tiles.nw, 1, L.tiles.nb))
        return fail(SPL_E_UNSUPPORTED, "dedispersion tile shape (%d, %d, %d) with %d LDS buffer(s) is not compiled in",
                    L.tiles.dw, L.tiles.j, L.tiles.nw, L.tiles.nb);
    const int cc_max = dedisp_stage_rows(L.tiles.nb) * L.tiles.nw;
    if (L.tiles.cc < 0 || L.tiles.cc > cc_max)
        return fail(SPL_E_UNSUPPORTED, "chan_chunk must be in [0, %d] for %d wavefronts and %d LDS buffer(s)", cc_max,
                    L.tiles.nw, L.tiles.nb);
    L.td = L.tiles.nw * L.tiles.dw;
    L.ndm_pad = (p.ndm + L.td - 1) / L.td * L.td;
    L.ntile_d = L.ndm_pad / L.td;
    const int TT = 256 * L.tiles.j;
    L.ntile_t = (p.n_dd + TT - 1) / TT;
    L.dcm.assign((size_t)p.nch * L.ndm_pad, 0);
    for (int c = 0; c < p.nch; ++c)
        for (int d = 0; d < L.ndm_pad; ++d) {
            const int ds = std::min(d, p.ndm - 1);   // pad by repeating the last trial
            L.dcm[(size_t)c * L.ndm_pad + d] = p.delays[(size_t)ds * p.nch + c];
        }
    L.tile_base.assign((size_t)L.ntile_d * p.nch, 0);
    L.row_bytes.assign(L.ntile_d, 0);
    for (int k = 0; k < L.ntile_d; ++k) {
        int span = 0;
        for (int c = 0; c < p.nch; ++c) {
            int lo = INT32_MAX, hi = 0;
            for (int d = k * L.td; d < (k + 1) * L.td; ++d) {
                const int v = L.dcm[(size_t)c * L.ndm_pad + d];
                lo = std::min(lo, v);
                hi = std::max(hi, v);
            }
            L.tile_base[(size_t)k * p.nch + c] = lo;
            span = std::max(span, hi - lo);
        }
        // one copy of a staged row: 8-bit samples covering the tile's time span, its
        // spread of delays and 16-sample alignment slack
        L.row_bytes[k] = TT + 32 + (int)align_up((size_t)span, 16);
    }
    const int rmax = *std::max_element(L.row_bytes.begin(), L.row_bytes.end());
    L.tiles.sv = rmax <= 1024 ? 1 : 2;
    if (rmax > 2048 || !dedisp_shape_supported(L.tiles.dw, L.tiles.j, L.tiles.nw, L.tiles.sv, L.tiles.nb))
        return fail(SPL_E_UNSUPPORTED, "a DM tile spans %d bytes of staged row: too wide for this tile shape "
                    "(use fewer trials per tile)", rmax);
    return SPL_OK;
}

// Default tiling: 8 wavefronts x 4 trials x 512 samples, smaller tiles when the plan
// gives too few work items to fill 256 compute units, fewer trials per tile when the
// delay spread of a tile would not fit the staged rows.
static bool tile_fits(const spl_plan &p, int td, int j) {
    // widest delay spread over td consecutive trials, any channel
    int worst = 0;
    for (int c = 0; c < p.nch; c += std::max(1, p.nch / 64)) {
        for (int d0 = 0; d0 < p.ndm; d0 += td) {
            const int d1 = std::min(p.ndm, d0 + td) - 1;
            worst = std::max(worst, std::abs(p.delays[(size_t)d1 * p.nch + c] - p.delays[(size_t)d0 * p.nch + c]));
        }
    }
    const int c = p.nch - 1;
    for (int d0 = 0; d0 < p.ndm; d0 += td) {
        const int d1 = std::min(p.ndm, d0 + td) - 1;
        worst = std::max(worst, std::abs(p.delays[(size_t)d1 * p.nch + c] - p.delays[(size_t)d0 * p.nch + c]));
    }
    return 256 * j + 32 + (int)align_up((size_t)worst + 64, 16) <= 2048;
}

static Tiles default_tiles(const spl_plan &p) {
    static const int shapes[][3] = {{4, 2, 8}, {4, 1, 8}, {2, 2, 8}, {4, 1, 4}};   // (trials/wave, groups, waves)
    for (const auto &sh : shapes) {
        Tiles t;
        t.dw = sh[0];
        t.j = sh[1];
        t.nw = sh[2];
        const int td = t.dw * t.nw;
        const int64_t items = (int64_t)((p.ndm + td - 1) / td) * ((p.n_dd + 256 * t.j - 1) / (256 * t.j));
        if (items < 1024 && &sh != &shapes[3]) continue;
        if (!tile_fits(p, td, t.j)) continue;
        return t;
    }
    Tiles t;
    t.dw = 4;
    t.j = 1;
    t.nw = 4;
    return t;
}

// Channels per staging step: the largest power of two <= 256 whose four shifted copies
// and offset table (in each LDS buffer) fit the LDS budget (a caller-set value is rounded
// down to a power of two).  Then the table of LDS byte offsets of every delay.
static void choose_chunk(PlanLayout &L, size_t lds_budget) {
    const int rmax = *std::max_element(L.row_bytes.begin(), L.row_bytes.end());
    int cc = L.tiles.cc;
    if (cc <= 0) {
        const int tab_rows = dedisp_stage_rows(L.tiles.nb) * L.tiles.nw + 4;   // as the kernel sizes it
        cc = dedisp_stage_rows(L.tiles.nb) * L.tiles.nw;
        while (cc > 2 && L.tiles.nb * ((size_t)4 * (cc + 1) * rmax + (size_t)tab_rows * 4 * L.td) > lds_budget)
            cc >>= 1;
    }
    int p2 = 2;   // at least 2: an odd last chunk is padded with a zero row
    while (p2 * 2 <= std::min(cc, 256)) p2 *= 2;
    L.tiles.cc = p2;
    L.quarter = (p2 + 1) * rmax;   // chan_chunk rows + the zero row
    const spl_plan &p = *L.plan;
    L.dtab.assign(L.dcm.size(), 0);
    for (int c = 0; c < p.nch; ++c) {
        for (int d = 0; d < L.ndm_pad; ++d) {
            const size_t k = (size_t)c * L.ndm_pad + d;
            const int sv = L.dcm[k];
            // the row of channel c in DM tile d/td starts at sample t0 + (base & ~15)
            const int b16 = L.tile_base[(size_t)(d / L.td) * p.nch + c] & ~15;
            L.dtab[k] = ((sv - b16) & ~3) + (sv & 3) * L.quarter;
        }
    }
    (void)p;
}

// Dynamic LDS of one dedispersion workgroup: per buffer, four copies of chan_chunk + 1
// staged rows and the offset table (dedisp_stage_rows * waves + 4 rows of td entries).
static size_t dedisp_lds_bytes(const PlanLayout &L) {
    return (size_t)L.tiles.nb *
           ((size_t)4 * L.quarter + (size_t)(dedisp_stage_rows(L.tiles.nb) * L.tiles.nw + 4) * L.td * sizeof(int32_t));
}

static spl_status build_layout(spl_batch *B) {
    // per-plan tables
    for (auto &L : B->layouts) {
        spl_status st = layout_plan(L);
        if (st != SPL_OK) return st;
        // 4- and 8-wavefront workgroups share a CU (64 KiB each); a 16-wavefront one holds it
        choose_chunk(L, L.tiles.nw >= 16 ? 160 * 1024 - 256 : 64 * 1024);
    }
    const int nb = B->nb;
    B->row_base.assign(nb + 1, 0);
    B->chunk_base.assign(nb + 1, 0);
    B->item_base.assign(nb + 1, 0);
    B->items.clear();
    B->beam_lds.assign(nb, 0);
    B->max_nst = 0;
    B->w_max = 0;
    // group beams by tile shape; items ordered by group, then beam, time tile, DM tile
    B->groups.clear();
    for (int b = 0; b < nb; ++b) {
        const Tiles &t = B->layouts[B->layout_of_beam[b]].tiles;
        int g = -1;
        for (size_t k = 0; k < B->groups.size(); ++k)
            if (B->groups[k].dw == t.dw && B->groups[k].j == t.j && B->groups[k].nw == t.nw &&
                B->groups[k].sv == t.sv && B->groups[k].nb == t.nb)
                g = (int)k;
        if (g < 0) {
            if ((int)B->groups.size() >= kMaxShapeGroups)
                return fail(SPL_E_UNSUPPORTED, "at most %d distinct tile shapes per batch", kMaxShapeGroups);
            B->groups.push_back({t.dw, t.j, t.nw, t.sv, t.nb, 0, 0, 0, 0});
        }
    }
    std::vector<std::vector<DedispItem>> per_beam(nb);
    for (int b = 0; b < nb; ++b) {
        const PlanLayout &L = B->layouts[B->layout_of_beam[b]];
        const spl_plan &p = *L.plan;
        const int TT = 256 * L.tiles.j;
        for (int tt = 0; tt < L.ntile_t; ++tt)
            for (int k = 0; k < L.ntile_d; ++k)
                per_beam[b].push_back({b, k * L.td, tt * TT, L.row_bytes[k]});
        B->beam_lds[b] = dedisp_lds_bytes(L);
        B->max_nst = std::max(B->max_nst, p.nst);
        B->w_max = std::max(B->w_max, p.w_max);
    }
    // rows / chunks in beam order; items grouped by shape
    for (int b = 0; b < nb; ++b) {
        const spl_plan &p = *B->plans[b];
        B->row_base[b + 1] = B->row_base[b] + p.ndm;
        B->chunk_base[b + 1] = B->chunk_base[b] + p.ndm * ((p.n_out + kBoxTile - 1) / kBoxTile);
    }
    B->n_rows = B->row_base[nb];
    B->n_chunks = B->chunk_base[nb];
    // items of beam b occupy [item_base[b], item_base[b] + its item count), in group order
    for (auto &g : B->groups) {
        g.item_lo = (int)B->items.size();
        size_t lds = 0;
        for (int b = 0; b < nb; ++b) {
            const Tiles &t = B->layouts[B->layout_of_beam[b]].tiles;
            if (t.dw != g.dw || t.j != g.j || t.nw != g.nw || t.sv != g.sv || t.nb != g.nb) continue;
            B->item_base[b] = (int)B->items.size();
            B->items.insert(B->items.end(), per_beam[b].begin(), per_beam[b].end());
            lds = std::max(lds, B->beam_lds[b]);
        }
        g.item_hi = (int)B->items.size();
        g.lds = lds;
    }
    B->n_items = (int)B->items.size();
    if ((int64_t)B->n_chunks >= INT32_MAX / 2 || (int64_t)B->n_items >= INT32_MAX / 2)
        return fail(SPL_E_UNSUPPORTED, "batch too large");

    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = align_up(off, 256);
        size_t o = off;
        off += bytes;
        return o;
    };
    // plan tables and work items are reserved for the smallest compiled tile (16 trials x
    // 256 samples) and the widest padding (64 trials), so that retiling (spl_batch_set_tiles,
    // spl_autotune) never needs a larger workspace
    size_t res_items = 0;
    for (int b = 0; b < nb; ++b) {
        const spl_plan &p = *B->plans[b];
        res_items += (size_t)((p.ndm + 15) / 16) * ((p.n_dd + 255) / 256);
    }
    B->off_beams = take(sizeof(DevBeam) * nb);
    B->off_items = take(sizeof(DedispItem) * std::max<size_t>(1, res_items));
    for (auto &L : B->layouts) {
        const spl_plan &p = *L.plan;
        L.off_dcm = take((size_t)p.nch * ((p.ndm + 63) / 64 * 64) * sizeof(int32_t));
        L.off_base = take((size_t)((p.ndm + 15) / 16) * p.nch * sizeof(int32_t));
        L.off_dms = take((size_t)p.ndm * sizeof(double));
        L.off_delays = take(p.delays.size() * sizeof(int32_t));
    }
    B->ws_persistent = align_up(off, 256);   // everything below is per-run scratch
    B->off_X.assign(nb, 0);
    B->off_S.assign(nb, 0);
    B->off_mu.assign(nb, 0);
    B->off_sigma.assign(nb, 0);
    B->off_T.assign(nb, 0);
    B->xpitch.assign(nb, 0);
    size_t s_total = 0;
    for (int b = 0; b < nb; ++b) s_total += (size_t)B->plans[b]->ndm * B->plans[b]->nseg * 2;
    B->off_S_all = take(s_total * sizeof(int64_t));
    B->bytes_S_all = s_total * sizeof(int64_t);
    size_t s_off = B->off_S_all;
    for (int b = 0; b < nb; ++b) {
        const spl_plan &p = *B->plans[b];
        B->xpitch[b] = (int)align_up((size_t)p.n_dd, 64);
        B->off_X[b] = take((size_t)p.ndm * B->xpitch[b] * sizeof(int32_t));
        B->off_S[b] = s_off;
        s_off += (size_t)p.ndm * p.nseg * 2 * sizeof(int64_t);
        B->off_mu[b] = take((size_t)p.ndm * p.nseg * sizeof(double));
        B->off_sigma[b] = take((size_t)p.ndm * p.nseg * sizeof(double));
        B->off_T[b] = take((size_t)p.ndm * p.nseg * p.widths.size() * sizeof(int32_t));
    }
    B->off_chunk_off = take((size_t)B->n_chunks * sizeof(int64_t));
    B->off_box_status = take(((size_t)B->n_chunks + 1) * sizeof(uint64_t));
    B->n_block_sums = scan_blocks(B->hit_cap) + 1;
    B->off_block_sums = take((size_t)B->n_block_sums * sizeof(int64_t));
    B->off_row_start = take((size_t)(B->n_rows + 1) * sizeof(int64_t));
    {
        int n_out_max = 1;
        for (int b = 0; b < nb; ++b) n_out_max = std::max(n_out_max, B->plans[b]->n_out);
        B->nms_nblk = ((n_out_max >> kNmsBlockShift) + 3) & ~1;   // >= 2 past the largest block, even
        B->off_nms_blk = take((size_t)B->n_rows * B->nms_nblk * sizeof(int32_t));
    }
    B->off_hits = take((size_t)B->hit_cap * sizeof(Hit));
    B->off_hit_t = take((size_t)B->hit_cap * sizeof(int32_t));
    B->off_surv = take((size_t)B->hit_cap * sizeof(Hit));
    B->off_surv_start = take((size_t)(B->n_rows + 1) * sizeof(int64_t));
    B->off_alive0 = take((size_t)B->hit_cap);
    B->off_alive1 = take((size_t)B->hit_cap);
    B->off_pos = take((size_t)B->hit_cap * sizeof(int64_t));
    B->off_run = take(sizeof(DevRun));
    B->ws_bytes = align_up(off, 256);
    B->tables_uploaded = false;
    if (B->graph_exec) {
        (void)hipGraphExecDestroy(B->graph_exec);
        B->graph_exec = nullptr;
    }
    if (B->graph) {
        (void)hipGraphDestroy(B->graph);
        B->graph = nullptr;
    }
    return SPL_OK;
}

extern "C" spl_status spl_batch_create(const spl_plan *const *plans, int32_t n_beams, const spl_batch_opts *opts,
                                       spl_batch **out) {
    if (!out) return fail(SPL_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!plans || n_beams < 1) return fail(SPL_E_INVALID_ARG, "at least one beam is required");
    for (int b = 0; b < n_beams; ++b)
        if (!plans[b]) return fail(SPL_E_INVALID_ARG, "plan of beam %d is NULL", b);
    spl_batch *B = new (std::nothrow) spl_batch();
    if (!B) return fail(SPL_E_OOM, "host allocation failed");
    B->nb = n_beams;
    B->plans.assign(plans, plans + n_beams);
    B->mode = opts ? opts->mode : SPL_MODE_PLAIN_PER_BEAM;
    if (B->mode != SPL_MODE_PLAIN_PER_BEAM && B->mode != SPL_MODE_PERSISTENT_GRAPH) {
        delete B;
        return fail(SPL_E_INVALID_ARG, "unknown mode %d", opts->mode);
    }
    if (opts && opts->hit_capacity > 0) {
        B->hit_cap = opts->hit_capacity;
    } else {
        // default: one hit per 16 owned (DM, t) cells of the batch, at least 2^24
        int64_t cells = 0;
        for (int b = 0; b < n_beams; ++b) cells += (int64_t)plans[b]->ndm * plans[b]->n_out;
        B->hit_cap = std::min<int64_t>(((int64_t)1 << 31) - 1, std::max<int64_t>((int64_t)1 << 24, cells / 16));
    }
    if (B->hit_cap > ((int64_t)1 << 31)) {
        delete B;
        return fail(SPL_E_UNSUPPORTED, "hit capacity above 2^31");
    }
    B->layout_of_beam.assign(n_beams, -1);
    for (int b = 0; b < n_beams; ++b) {
        int found = -1;
        for (size_t k = 0; k < B->layouts.size(); ++k)
            if (B->layouts[k].plan == plans[b]) found = (int)k;
        if (found < 0) {
            PlanLayout L;
            L.plan = plans[b];
            const Tiles t = default_tiles(*plans[b]);
            L.tiles = t;
            B->layouts.push_back(L);
            found = (int)B->layouts.size() - 1;
        }
        B->layout_of_beam[b] = found;
    }
    spl_status st = build_layout(B);
    if (st != SPL_OK) { delete B; return st; }
    B->cur_x.assign(n_beams, nullptr);
    B->cur_pitch.assign(n_beams, 0);
    *out = B;
    return SPL_OK;
}

extern "C" spl_status spl_batch_workspace_size(const spl_batch *B, size_t *persistent, size_t *scratch) {
    if (!B || !persistent || !scratch) return fail(SPL_E_INVALID_ARG, "NULL argument");
    *persistent = B->ws_persistent;
    *scratch = B->ws_bytes - B->ws_persistent;
    return SPL_OK;
}

static void fill_host_beams(spl_batch *B) {
    B->host_beams.assign(B->nb, DevBeam{});
    for (int b = 0; b < B->nb; ++b) {
        const PlanLayout &L = B->layouts[B->layout_of_beam[b]];
        const spl_plan &p = *B->plans[b];
        DevBeam &d = B->host_beams[b];
        std::memset(&d, 0, sizeof d);
        d.x = B->cur_x[b];
        d.pitch = B->cur_pitch[b];
        d.dtab = (const int32_t *)(B->ws + L.off_dcm);
        d.tile_base = (const int32_t *)(B->ws + L.off_base);
        d.delays = (const int32_t *)(B->ws + L.off_delays);
        d.X = (int32_t *)(B->ws + B->off_X[b]);
        d.S1 = (int64_t *)(B->ws + B->off_S[b]);
        d.S2 = d.S1 + (size_t)p.ndm * p.nseg;
        d.mu = (double *)(B->ws + B->off_mu[b]);
        d.sigma = (double *)(B->ws + B->off_sigma[b]);
        d.T = (int32_t *)(B->ws + B->off_T[b]);
        d.dms = (const double *)(B->ws + L.off_dms);
        d.theta = p.theta;
        d.fch1 = p.band.fch1_mhz;
        d.foff = p.band.foff_mhz;
        d.fref = d.flo = p.band.fch1_mhz;
        for (int c = 0; c < p.nch; ++c) {
            const double f = p.band.fch1_mhz + (double)c * p.band.foff_mhz;
            d.fref = std::max(d.fref, f);
            d.flo = std::min(d.flo, f);
        }
        d.tsamp = p.band.tsamp_s;
        d.n_in = p.n_in;
        d.nch = p.nch;
        d.ndm = p.ndm;
        d.ndm_pad = L.ndm_pad;
        d.n_dd = p.n_dd;
        d.n_out = p.n_out;
        d.L = p.L;
        d.nseg = p.nseg;
        d.nw = (int)p.widths.size();
        d.xpitch = B->xpitch[b];
        d.row_base = B->row_base[b];
        d.chunk_base = B->chunk_base[b];
        d.nchunk_t = (p.n_out + kBoxTile - 1) / kBoxTile;
        d.chan_chunk = L.tiles.cc;
        d.lds_quarter = L.quarter;
        d.tile_dm = L.td;
        d.beam = b;
        d.w_max = p.w_max;
        d.nst = p.nst;
        for (int k = 0; k < kMaxStencils; ++k) {
            d.rd[k] = p.rd[k];
            d.rt[k] = p.rt[k];
        }
        for (size_t k = 0; k < p.widths.size(); ++k) d.widths[k] = p.widths[k];
    }
}

// Copy the plan tables, work items and beam descriptors of the current layout into the
// workspace at B->ws (synchronous copies from host memory).
static spl_status copy_tables(spl_batch *B) {
    for (auto &L : B->layouts) {
        HIP_TRY(hipMemcpy(B->ws + L.off_dcm, L.dtab.data(), L.dtab.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(B->ws + L.off_base, L.tile_base.data(), L.tile_base.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(B->ws + L.off_dms, L.plan->dms.data(), L.plan->dms.size() * sizeof(double),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(B->ws + L.off_delays, L.plan->delays.data(), L.plan->delays.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice));
    }
    if (B->n_items)
        HIP_TRY(hipMemcpy(B->ws + B->off_items, B->items.data(), B->items.size() * sizeof(DedispItem),
                          hipMemcpyHostToDevice));
    fill_host_beams(B);
    HIP_TRY(hipMemcpy(B->ws + B->off_beams, B->host_beams.data(), sizeof(DevBeam) * B->nb, hipMemcpyHostToDevice));
    return SPL_OK;
}

// LDS limits of the dedispersion instantiations the batch launches, and the occupancy of
// each persistent shape group.
static spl_status prepare_shapes(spl_batch *B) {
    for (auto &g : B->groups) {
        int occ = 0;
        HIP_TRY(prepare_dedisp(g.dw, g.j, g.nw, g.sv, g.nb, g.lds, &occ));
        g.occ = std::max(1, occ);
    }
    for (int b = 0; b < B->nb; ++b) {
        const Tiles &t = B->layouts[B->layout_of_beam[b]].tiles;
        int occ = 0;
        HIP_TRY(prepare_dedisp(t.dw, t.j, t.nw, t.sv, t.nb, B->beam_lds[b], &occ));
    }
    return SPL_OK;
}

// Upload the plan tables and beam descriptors of the current layout (synchronous).
static spl_status upload_tables(spl_batch *B) {
    if (B->staging_pending) {
        HIP_TRY(hipEventSynchronize(B->staging_done));
        B->staging_pending = false;
    }
    spl_status st = copy_tables(B);
    if (st != SPL_OK) return st;
    st = prepare_shapes(B);
    if (st != SPL_OK) return st;
    if (B->graph_exec) {
        (void)hipGraphExecDestroy(B->graph_exec);
        B->graph_exec = nullptr;
    }
    if (B->graph) {
        (void)hipGraphDestroy(B->graph);
        B->graph = nullptr;
    }
    B->tables_uploaded = true;
    return SPL_OK;
}

extern "C" spl_status spl_batch_set_workspace(spl_batch *B, void *d_ws, size_t bytes) {
    if (!B || !d_ws) return fail(SPL_E_INVALID_ARG, "NULL argument");
    if (bytes < B->ws_bytes) return fail(SPL_E_OOM, "workspace too small: %zu < %zu bytes", bytes, B->ws_bytes);
    if (((uintptr_t)d_ws & 255) != 0) return fail(SPL_E_INVALID_ARG, "workspace must be 256-byte aligned");
    if (!B->staging) {
        HIP_TRY(hipHostMalloc((void **)&B->staging, sizeof(DevBeam) * B->nb, hipHostMallocDefault));
        HIP_TRY(hipEventCreateWithFlags(&B->staging_done, hipEventDisableTiming));
    }
    B->ws = (char *)d_ws;
    B->ws_given = bytes;
    return upload_tables(B);
}

static hipError_t take_event(spl_batch *B, hipEvent_t *e) {
    if (!B->free_events.empty()) {
        *e = B->free_events.back();
        B->free_events.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

// Records an event pair around one stage when profiling is on.
struct StageTimer {
    spl_batch *B;
    hipStream_t s;
    int stage;
    hipEvent_t a = nullptr;
    hipError_t err = hipSuccess;
    StageTimer(spl_batch *b, hipStream_t st, int k) : B(b), s(st), stage(k) {
        if (!B->profiling) return;
        err = take_event(B, &a);
        if (err == hipSuccess) err = hipEventRecord(a, s);
    }
    hipError_t stop() {
        if (!B->profiling || err != hipSuccess) return err;
        hipEvent_t b = nullptr;
        err = take_event(B, &b);
        if (err == hipSuccess) err = hipEventRecord(b, s);
        if (err == hipSuccess) B->timed.push_back({stage, a, b});
        return err;
    }
};

// The launch sequence of one beam range [b_lo, b_hi).
static spl_status enqueue_range(spl_batch *B, int b_lo, int b_hi, bool persistent, spl_candidate *cands,
                                int64_t cand_cap, spl_run_stats *stats, hipStream_t s) {
    const DevBeam *beams = (const DevBeam *)(B->ws + B->off_beams);
    const DedispItem *items = (const DedispItem *)(B->ws + B->off_items);
    DevRun *run = (DevRun *)(B->ws + B->off_run);
    const int row_lo = B->row_base[b_lo], row_hi = B->row_base[b_hi];
    const int chunk_lo = B->chunk_base[b_lo], chunk_hi = B->chunk_base[b_hi];
    int64_t *chunk_off = (int64_t *)(B->ws + B->off_chunk_off) + chunk_lo;
    int64_t *block_sums = (int64_t *)(B->ws + B->off_block_sums);
    uint64_t *box_status = (uint64_t *)(B->ws + B->off_box_status) + chunk_lo;
    int64_t *row_start = (int64_t *)(B->ws + B->off_row_start) + row_lo;
    Hit *hits = (Hit *)(B->ws + B->off_hits);
    uint8_t *alive[2] = {(uint8_t *)(B->ws + B->off_alive0), (uint8_t *)(B->ws + B->off_alive1)};
    int64_t *pos = (int64_t *)(B->ws + B->off_pos);
    const int64_t cap = B->hit_cap;

    // 1. dedispersion
    StageTimer t_dd(B, s, SPL_STAGE_DEDISP);
    if (persistent) {
        for (size_t g = 0; g < B->groups.size(); ++g) {
            const auto &G = B->groups[g];
            const int n = G.item_hi - G.item_lo;
            if (n <= 0) continue;
            const int grid = std::min(n, G.occ * 256);
            HIP_TRY(launch_dedisp(G.dw, G.j, G.nw, G.sv, G.nb, beams, items, G.item_lo, G.item_hi, &run->queue[g],
                                  grid, G.lds, s));
        }
    } else {
        for (int b = b_lo; b < b_hi; ++b) {
            const Tiles &t = B->layouts[B->layout_of_beam[b]].tiles;
            const int lo = B->item_base[b];
            const PlanLayout &L = B->layouts[B->layout_of_beam[b]];
            const int hi = lo + L.ntile_d * L.ntile_t;
            HIP_TRY(launch_dedisp(t.dw, t.j, t.nw, t.sv, t.nb, beams, items, lo, hi, nullptr, hi - lo, B->beam_lds[b],
                                  s));
        }
    }
    HIP_TRY(t_dd.stop());
    // 2. normaliser and integer thresholds
    StageTimer t_th(B, s, SPL_STAGE_THRESHOLDS);
    HIP_TRY(launch_thresholds(beams, b_lo, b_hi, row_lo, row_hi, s));
    HIP_TRY(t_th.stop());
    // 3. boxcar hits in (row, t) order, each chunk's offset by look-back over the earlier chunks
    int w_max = 1;
    int max_nst = 0;
    for (int b = b_lo; b < b_hi; ++b) {
        w_max = std::max(w_max, B->plans[b]->w_max);
        max_nst = std::max(max_nst, B->plans[b]->nst);
    }
    StageTimer t_bc(B, s, SPL_STAGE_BOXCAR);
    HIP_TRY(launch_boxcar_one_pass(beams, b_lo, b_hi, chunk_lo, chunk_hi, w_max, box_status, chunk_off, hits, cap,
                                   &run->n_hits, &run->box_stall, s));
    HIP_TRY(launch_row_start(beams, b_lo, b_hi, row_lo, row_hi, chunk_lo, chunk_off, &run->n_hits, cap, row_start,
                             s));
    HIP_TRY(t_bc.stop());
    // 4. peak filters, then ordered compaction into candidate records
    StageTimer t_pk(B, s, SPL_STAGE_PEAKS);
    int32_t *blk = (int32_t *)(B->ws + B->off_nms_blk);
    int32_t *hit_t = (int32_t *)(B->ws + B->off_hit_t);
    if (max_nst)
        HIP_TRY(launch_nms_index(row_lo, row_hi - row_lo, hits, &run->n_hits, cap, row_start, blk, B->nms_nblk, hit_t,
                                 s));
    // The first filter runs over every hit.  The later ones (wider windows, over the few
    // survivors) run over the survivors compacted in order, with their own block index,
    // so that their searches and scans never meet a hit already filtered out.
    const Hit *fh = hits;
    const int64_t *fn = &run->n_hits;
    const int64_t *fstart = row_start;
    const uint8_t *in = nullptr;
    for (int k = 0; k < max_nst; ++k) {
        uint8_t *o = alive[k & 1];
        if (k == 1) {
            Hit *surv = (Hit *)(B->ws + B->off_surv);
            int64_t *surv_start = (int64_t *)(B->ws + B->off_surv_start) + row_lo;
            HIP_TRY(launch_scan_u8(in, &run->n_hits, cap, block_sums, pos, &run->n_surv, s));
            HIP_TRY(launch_compact_hits(hits, &run->n_hits, cap, in, pos, surv, row_start, row_hi - row_lo,
                                        &run->n_surv, surv_start, s));
            HIP_TRY(launch_nms_index(row_lo, row_hi - row_lo, surv, &run->n_surv, cap, surv_start, blk,
                                     B->nms_nblk, hit_t, s));
            fh = surv;
            fn = &run->n_surv;
            fstart = surv_start;
            in = nullptr;
        }
        HIP_TRY(launch_nms(beams, b_lo, b_hi, row_lo, fh, fn, cap, fstart, blk, B->nms_nblk, k, in, o,
                           &run->n_alive[k], hit_t, s));
        in = o;
    }
    if (max_nst) {
        HIP_TRY(launch_scan_u8(in, fn, cap, block_sums, pos, &run->n_cand_beam, s));
        HIP_TRY(launch_scatter(beams, b_lo, b_hi, fh, fn, cap, in, pos, &run->n_cand_total, cands, cand_cap, s));
    } else {
        HIP_TRY(launch_scatter(beams, b_lo, b_hi, hits, &run->n_hits, cap, nullptr, nullptr, &run->n_cand_total,
                               cands, cand_cap, s));
    }
    HIP_TRY(launch_pass_end(run, stats, cap, max_nst, s));
    HIP_TRY(t_pk.stop());
    return SPL_OK;
}

static spl_status enqueue_all(spl_batch *B, spl_candidate *cands, int64_t cap, spl_run_stats *stats,
                              hipStream_t s) {
    DevRun *run = (DevRun *)(B->ws + B->off_run);
    HIP_TRY(launch_fill_u64((uint64_t *)run, (int64_t)(sizeof(DevRun) / 8), 0, s));
    HIP_TRY(launch_fill_u64((uint64_t *)stats, (int64_t)(sizeof(spl_run_stats) / 8), 0, s));
    if (B->mode == SPL_MODE_PERSISTENT_GRAPH) {
        spl_status st = enqueue_range(B, 0, B->nb, true, cands, cap, stats, s);
        if (st != SPL_OK) return st;
    } else {
        for (int b = 0; b < B->nb; ++b) {
            spl_status st = enqueue_range(B, b, b + 1, false, cands, cap, stats, s);
            if (st != SPL_OK) return st;
        }
    }
    HIP_TRY(launch_finalize(run, stats, cap, s));
    return SPL_OK;
}

// Arguments of a search run: candidate buffer, statistics and every beam's block.
static spl_status check_run_args(const spl_batch *B, const uint8_t *const *d_blocks, const int64_t *pitches,
                                 const spl_candidate *d_cands, int64_t capacity, const spl_run_stats *d_stats) {
    if (capacity < 0 || (capacity > 0 && !d_cands)) return fail(SPL_E_INVALID_ARG, "bad candidate buffer");
    if (((uintptr_t)d_stats & 7) != 0) return fail(SPL_E_INVALID_ARG, "d_stats must be 8-byte aligned");
    for (int b = 0; b < B->nb; ++b) {
        const spl_plan &p = *B->plans[b];
        if (!d_blocks[b]) return fail(SPL_E_INVALID_ARG, "block of beam %d is NULL", b);
        if (((uintptr_t)d_blocks[b] & 15) != 0) return fail(SPL_E_INVALID_ARG, "block of beam %d is not 16-byte aligned", b);
        if (pitches[b] < p.n_in || (pitches[b] & 15) != 0)
            return fail(SPL_E_INVALID_ARG, "pitch of beam %d must be a multiple of 16 and >= n_in = %d", b, p.n_in);
    }
    return SPL_OK;
}

extern "C" spl_status spl_batch_run(spl_batch *B, const uint8_t *const *d_blocks, const int64_t *pitches,
                                    spl_candidate *d_cands, int64_t capacity, spl_run_stats *d_stats,
                                    hipStream_t stream) {
    static_assert(sizeof(spl_run_stats) % 8 == 0, "stats are cleared in 8-byte words");
    static_assert(sizeof(DevRun) % 8 == 0, "run state is cleared in 8-byte words");
    if (!B || !d_blocks || !pitches || !d_stats) return fail(SPL_E_INVALID_ARG, "NULL argument");
    if (!B->tables_uploaded) return fail(SPL_E_INVALID_ARG, "spl_batch_set_workspace was not called");
    spl_status vs = check_run_args(B, d_blocks, pitches, d_cands, capacity, d_stats);
    if (vs != SPL_OK) return vs;
    bool changed = false;
    for (int b = 0; b < B->nb; ++b)
        if (d_blocks[b] != B->cur_x[b] || pitches[b] != B->cur_pitch[b]) changed = true;
    if (changed) {
        if (B->staging_pending) HIP_TRY(hipEventSynchronize(B->staging_done));
        for (int b = 0; b < B->nb; ++b) {
            B->cur_x[b] = d_blocks[b];
            B->cur_pitch[b] = pitches[b];
            B->host_beams[b].x = d_blocks[b];
            B->host_beams[b].pitch = pitches[b];
        }
        std::memcpy(B->staging, B->host_beams.data(), sizeof(DevBeam) * B->nb);
        HIP_TRY(hipMemcpyAsync(B->ws + B->off_beams, B->staging, sizeof(DevBeam) * B->nb, hipMemcpyHostToDevice,
                               stream));
        HIP_TRY(hipEventRecord(B->staging_done, stream));
        B->staging_pending = true;
    }
    if (B->mode == SPL_MODE_PERSISTENT_GRAPH && !B->profiling) {
        if (stream == nullptr) return fail(SPL_E_INVALID_ARG, "graph mode needs a non-default stream");
        if (!B->graph_exec || B->g_cands != d_cands || B->g_stats != d_stats || B->g_cap != capacity) {
            if (B->graph_exec) { (void)hipGraphExecDestroy(B->graph_exec); B->graph_exec = nullptr; }
            if (B->graph) { (void)hipGraphDestroy(B->graph); B->graph = nullptr; }
            HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            spl_status st = enqueue_all(B, d_cands, capacity, d_stats, stream);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(stream, &g);
            if (st != SPL_OK) { if (g) (void)hipGraphDestroy(g); return st; }
            if (e != hipSuccess) return fail(SPL_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
            B->graph = g;
            HIP_TRY(hipGraphInstantiate(&B->graph_exec, B->graph, nullptr, nullptr, 0));
            B->g_cands = d_cands;
            B->g_stats = d_stats;
            B->g_cap = capacity;
        }
        HIP_TRY(hipGraphLaunch(B->graph_exec, stream));
        return SPL_OK;
    }
    return enqueue_all(B, d_cands, capacity, d_stats, stream);
}

// ------------------------------------------------- search without allocation
// The workspace of spl_batch_run_static: one copy of this array per GPU, at its own
// address on each, held until the process ends.  Host code never uses the array's name
// as an address: it takes each device's address once from hipGetSymbolAddress.
static constexpr size_t kStaticScratchBytes = SPL_STATIC_SCRATCH_BYTES;
static constexpr int kMaxStaticDevices = 64;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kMaxStaticDevices] = {};

// Device address of the current device's copy of the scratch array, looked up on the
// first call on that device.
static spl_status scratch_address(char **out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxStaticDevices) return fail(SPL_E_UNSUPPORTED, "device %d: too many devices", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SPL_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = (char *)p;
    }
    *out = g_scratch_ptr[dev];
    return SPL_OK;
}

extern "C" spl_status spl_batch_run_static(spl_batch *B, const uint8_t *const *d_blocks, const int64_t *pitches,
                                           spl_candidate *d_cands, int64_t capacity, spl_run_stats *d_stats,
                                           hipStream_t stream) {
    if (!B || !d_blocks || !pitches || !d_stats) return fail(SPL_E_INVALID_ARG, "NULL argument");
    spl_status st = check_run_args(B, d_blocks, pitches, d_cands, capacity, d_stats);
    if (st != SPL_OK) return st;
    if (B->ws_bytes > kStaticScratchBytes)
        return fail(SPL_E_UNSUPPORTED, "the batch needs %zu workspace bytes, the static scratch holds %zu "
                    "(lower the hit capacity or the batch size)", B->ws_bytes, kStaticScratchBytes);
    char *sp = nullptr;
    st = scratch_address(&sp);
    if (st != SPL_OK) return st;
    // an earlier call's kernels on this stream may still read the scratch
    HIP_TRY(hipStreamSynchronize(stream));
    // the scratch stands in for the batch's workspace for this call; the batch's own
    // workspace, descriptors and captured graph are left as they are
    char *ws = B->ws;
    const size_t ws_given = B->ws_given;
    const bool profiling = B->profiling;
    std::vector<const uint8_t *> cur_x;
    std::vector<int64_t> cur_pitch;
    cur_x.swap(B->cur_x);
    cur_pitch.swap(B->cur_pitch);
    B->cur_x.assign(d_blocks, d_blocks + B->nb);
    B->cur_pitch.assign(pitches, pitches + B->nb);
    B->ws = sp;
    B->ws_given = kStaticScratchBytes;
    B->profiling = false;
    st = copy_tables(B);
    if (st == SPL_OK) st = prepare_shapes(B);
    if (st == SPL_OK) st = enqueue_all(B, d_cands, capacity, d_stats, stream);
    B->ws = ws;
    B->ws_given = ws_given;
    B->profiling = profiling;
    B->cur_x.swap(cur_x);
    B->cur_pitch.swap(cur_pitch);
    if (ws) fill_host_beams(B);
    return st;
}

extern "C" spl_status spl_batch_dm_transform(const spl_batch *B, int32_t beam, const int32_t **d_X,
                                             int64_t *pitch_elems) {
    if (!B || !d_X || !pitch_elems || beam < 0 || beam >= B->nb) return fail(SPL_E_INVALID_ARG, "bad argument");
    if (!B->ws) return fail(SPL_E_INVALID_ARG, "no workspace attached");
    *d_X = (const int32_t *)(B->ws + B->off_X[beam]);
    *pitch_elems = B->xpitch[beam];
    return SPL_OK;
}

extern "C" spl_status spl_batch_moments(const spl_batch *B, int32_t beam, const int64_t **d_S1,
                                        const int64_t **d_S2) {
    if (!B || !d_S1 || !d_S2 || beam < 0 || beam >= B->nb) return fail(SPL_E_INVALID_ARG, "bad argument");
    if (!B->ws) return fail(SPL_E_INVALID_ARG, "no workspace attached");
    const spl_plan &p = *B->plans[beam];
    *d_S1 = (const int64_t *)(B->ws + B->off_S[beam]);
    *d_S2 = *d_S1 + (size_t)p.ndm * p.nseg;
    return SPL_OK;
}

extern "C" spl_status spl_batch_get_tiles(const spl_batch *B, int32_t beam, spl_tiles *tiles) {
    if (!B || !tiles || beam < 0 || beam >= B->nb) return fail(SPL_E_INVALID_ARG, "bad argument");
    const Tiles &t = B->layouts[B->layout_of_beam[beam]].tiles;
    tiles->dm_per_wave = t.dw;
    tiles->time_groups = t.j;
    tiles->chan_chunk = t.cc;
    tiles->waves = t.nw;
    tiles->buffers = t.nb;
    return SPL_OK;
}

extern "C" spl_status spl_batch_set_tiles(spl_batch *B, int32_t beam, const spl_tiles *tiles) {
    if (!B || !tiles || beam < 0 || beam >= B->nb) return fail(SPL_E_INVALID_ARG, "bad argument");
    const int nw = tiles->waves ? tiles->waves : 4;
    const int nbuf = tiles->buffers ? tiles->buffers : 1;
    if (!dedisp_shape_supported(tiles->dm_per_wave, tiles->time_groups, nw, 1, nbuf))
        return fail(SPL_E_UNSUPPORTED, "tile shape (%d, %d, %d) with %d LDS buffer(s) is not compiled in",
                    tiles->dm_per_wave, tiles->time_groups, nw, nbuf);
    if (tiles->chan_chunk < 0 || tiles->chan_chunk > dedisp_stage_rows(nbuf) * nw)
        return fail(SPL_E_UNSUPPORTED, "chan_chunk must be in [0, %d] (0: from the LDS budget)",
                    dedisp_stage_rows(nbuf) * nw);
    PlanLayout &L = B->layouts[B->layout_of_beam[beam]];
    const Tiles old = L.tiles;
    L.tiles.dw = tiles->dm_per_wave;
    L.tiles.j = tiles->time_groups;
    L.tiles.nw = nw;
    L.tiles.nb = nbuf;
    L.tiles.cc = tiles->chan_chunk;
    spl_status st = build_layout(B);
    if (st == SPL_OK) {
        if (dedisp_lds_bytes(L) > 160 * 1024 - 256) st = fail(SPL_E_UNSUPPORTED, "tile does not fit the LDS");
    }
    if (st != SPL_OK) {
        L.tiles = old;
        (void)build_layout(B);
        if (B->ws) (void)upload_tables(B);
        return st;
    }
    if (B->ws) return upload_tables(B);
    return SPL_OK;
}

// ------------------------------------------------------------------ autotuner
namespace {

uint64_t fnv64(const void *p, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Everything the dedispersion kernel's speed depends on: sizes and the delay table.
std::string plan_signature(const spl_plan &p) {
    uint64_t h = fnv64(p.delays.data(), p.delays.size() * sizeof(int32_t));
    char buf[160];
    snprintf(buf, sizeof buf, "nch%d-ndm%d-nout%d-ndd%d-d%016llx", p.nch, p.ndm, p.n_out, p.n_dd,
             (unsigned long long)h);
    return buf;
}

struct TuneEntry {
    Tiles t;
    double ms = 0;
};

// Cache file: one line per plan,
// "<signature> <trials/wave> <groups> <waves> <LDS buffers> <chan_chunk> <ms>"; lines of
// any other form are dropped (their plans are tuned again).
std::vector<std::pair<std::string, TuneEntry>> read_cache(const char *path) {
    std::vector<std::pair<std::string, TuneEntry>> out;
    if (!path) return out;
    FILE *f = fopen(path, "r");
    if (!f) return out;
    char line[512], sig[256];
    while (fgets(line, sizeof line, f)) {
        // exactly seven whitespace-separated fields, the six numbers integers but the last
        int fields = 0;
        for (const char *c = line; *c;) {
            while (*c == ' ' || *c == '\t' || *c == '\n' || *c == '\r') ++c;
            if (!*c) break;
            ++fields;
            while (*c && *c != ' ' && *c != '\t' && *c != '\n' && *c != '\r') ++c;
        }
        TuneEntry e;
        int used = 0;
        if (fields == 7 && sscanf(line, "%255s %d %d %d %d %d %lf%n", sig, &e.t.dw, &e.t.j, &e.t.nw, &e.t.nb,
                                  &e.t.cc, &e.ms, &used) == 7 &&
            strspn(line + used, " \t\r\n") == strlen(line + used))
            out.emplace_back(sig, e);
    }
    fclose(f);
    return out;
}

void write_cache(const char *path, const std::vector<std::pair<std::string, TuneEntry>> &c) {
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const auto &kv : c)
        fprintf(f, "%s %d %d %d %d %d %.6f\n", kv.first.c_str(), kv.second.t.dw, kv.second.t.j, kv.second.t.nw,
                kv.second.t.nb, kv.second.t.cc, kv.second.ms);
    fclose(f);
    (void)rename(tmp.c_str(), path);
}

}  // namespace

extern "C" spl_status spl_autotune(spl_batch *B, const uint8_t *const *d_blocks, const int64_t *pitches,
                                   const char *cache_path, int32_t flags, hipStream_t stream) {
    if (!B || !d_blocks || !pitches) return fail(SPL_E_INVALID_ARG, "NULL argument");
    if (!B->tables_uploaded) return fail(SPL_E_INVALID_ARG, "spl_batch_set_workspace was not called");
    for (int b = 0; b < B->nb; ++b) {
        const spl_plan &p = *B->plans[b];
        if (!d_blocks[b] || ((uintptr_t)d_blocks[b] & 15) || pitches[b] < p.n_in || (pitches[b] & 15))
            return fail(SPL_E_INVALID_ARG, "block or pitch of beam %d is invalid", b);
        B->cur_x[b] = d_blocks[b];
        B->cur_pitch[b] = pitches[b];
    }
    auto cache = read_cache(cache_path);
    constexpr int kTuneBeams = 4;
    // 16-wavefront tiles (64 trials) share each staged channel row among twice the trials;
    // 16 wavefronts of 2 trials keep 4 wavefronts per SIMD where a band's wide delay
    // spread leaves room in the LDS for one workgroup per CU only; 16-wavefront tiles
    // also come with two LDS buffers (trials/wave, groups, waves, buffers)
    static const int shapes[][4] = {{2, 2, 8, 1},  {4, 1, 4, 1},  {4, 2, 4, 1},  {4, 1, 8, 1},  {4, 2, 8, 1},
                                    {8, 1, 4, 1},  {8, 1, 8, 1},  {4, 1, 16, 1}, {4, 2, 16, 1}, {2, 2, 16, 1},
                                    {4, 1, 16, 2}, {4, 2, 16, 2}, {2, 2, 16, 2}};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    unsigned long long *d_sum = (unsigned long long *)(B->ws + B->off_run);   // run state is scratch here
    spl_status result = SPL_OK;
    for (size_t li = 0; li < B->layouts.size() && result == SPL_OK; ++li) {
        int rep = 0;
        while (B->layout_of_beam[rep] != (int)li) ++rep;
        const std::string sig = plan_signature(*B->layouts[li].plan);
        bool cached = false;
        if (!(flags & SPL_TUNE_FORCE)) {
            for (const auto &kv : cache)
                if (kv.first == sig) {
                    B->layouts[li].tiles = kv.second.t;
                    B->layouts[li].tiles.sv = 1;
                    cached = true;
                }
        }
        if (cached) {
            if (build_layout(B) == SPL_OK) continue;
            B->layouts[li].tiles = Tiles{};   // a stale entry: tune afresh
        }
        TuneEntry best;
        best.ms = 1e300;
        bool have_ref = false;
        unsigned long long ref = 0;
        for (const auto &sh : shapes) {
            for (int cc = 2; cc <= dedisp_stage_rows(sh[3]) * sh[2]; cc *= 2) {
                PlanLayout &L = B->layouts[li];
                L.tiles = Tiles{};
                L.tiles.dw = sh[0];
                L.tiles.j = sh[1];
                L.tiles.nw = sh[2];
                L.tiles.nb = sh[3];
                L.tiles.cc = cc;
                if (build_layout(B) != SPL_OK) continue;
                if (B->beam_lds[rep] > 160 * 1024 - 256) continue;
                spl_status st = upload_tables(B);
                if (st != SPL_OK) { result = st; break; }
                const DevBeam *beams = (const DevBeam *)(B->ws + B->off_beams);
                const DedispItem *items = (const DedispItem *)(B->ws + B->off_items);
                // time the shape as a batched run launches it: one persistent launch (grid from
                // the occupancy, work items from a queue) over up to kTuneBeams beams of this
                // plan whose work items follow each other in the item list (beams of one
                // shape are listed in beam order, so other plans' beams of a different shape
                // leave gaps only in beam numbers); one beam with one workgroup per item
                // favours small tiles through its tail
                const int per_beam = L.ntile_d * L.ntile_t;
                const int lo = B->item_base[rep];
                int hi = lo + per_beam, used = 1;
                for (int b = rep + 1; b < B->nb && used < kTuneBeams; ++b) {
                    if (B->layout_of_beam[b] != (int)li) continue;
                    if (B->item_base[b] != hi) break;
                    hi += per_beam;
                    ++used;
                }
                const Tiles t = L.tiles;
                int occ = 0;
                HIP_TRY(prepare_dedisp(t.dw, t.j, t.nw, t.sv, t.nb, B->beam_lds[rep], &occ));
                const int grid = std::min(hi - lo, std::max(1, occ) * 256);
                int *queue = &((DevRun *)(B->ws + B->off_run))->queue[0];
                float best_run = 1e30f;
                for (int r = 0; r < 4; ++r) {
                    HIP_TRY(hipMemsetAsync(queue, 0, sizeof(int), stream));
                    HIP_TRY(hipEventRecord(e0, stream));
                    HIP_TRY(launch_dedisp(t.dw, t.j, t.nw, t.sv, t.nb, beams, items, lo, hi, queue, grid,
                                          B->beam_lds[rep], stream));
                    HIP_TRY(hipEventRecord(e1, stream));
                    HIP_TRY(hipEventSynchronize(e1));
                    float ms = 0.f;
                    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                    if (r > 0) best_run = std::min(best_run, ms);   // first run warms caches
                }
                HIP_TRY(hipMemsetAsync(d_sum, 0, sizeof(unsigned long long), stream));
                const spl_plan &p = *L.plan;
                HIP_TRY(launch_checksum((const int32_t *)(B->ws + B->off_X[rep]), p.ndm, B->xpitch[rep], p.n_dd,
                                        d_sum, stream));
                unsigned long long sum = 0;
                HIP_TRY(hipMemcpyAsync(&sum, d_sum, sizeof sum, hipMemcpyDeviceToHost, stream));
                HIP_TRY(hipStreamSynchronize(stream));
                if (!have_ref) {
                    ref = sum;
                    have_ref = true;
                } else if (sum != ref) {
                    result = fail(SPL_E_INTERNAL, "tile shape (%d, %d, %d, %d buffer(s), %d) changed the DM transform",
                                  t.dw, t.j, t.nw, t.nb, t.cc);
                    break;
                }
                if (best_run < best.ms) {
                    best.ms = best_run;
                    best.t = t;
                }
            }
            if (result != SPL_OK) break;
        }
        if (result != SPL_OK) break;
        if (!have_ref) {
            result = fail(SPL_E_UNSUPPORTED, "no compiled tile shape fits the plan");
            break;
        }
        B->layouts[li].tiles = best.t;
        spl_status st = build_layout(B);
        if (st != SPL_OK) { result = st; break; }
        bool replaced = false;
        for (auto &kv : cache)
            if (kv.first == sig) { kv.second = best; replaced = true; }
        if (!replaced) cache.emplace_back(sig, best);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != SPL_OK) {
        (void)build_layout(B);
        (void)upload_tables(B);
        return result;
    }
    write_cache(cache_path, cache);
    return upload_tables(B);
}

extern "C" spl_status spl_batch_set_profiling(spl_batch *B, int32_t enable) {
    if (!B) return fail(SPL_E_INVALID_ARG, "NULL batch");
    B->profiling = enable != 0;
    return SPL_OK;
}

extern "C" spl_status spl_batch_stage_times(spl_batch *B, double *ms, int64_t *count, int32_t reset) {
    if (!B) return fail(SPL_E_INVALID_ARG, "NULL batch");
    for (auto &t : B->timed) {
        HIP_TRY(hipEventSynchronize(t.b));
        float e = 0.f;
        HIP_TRY(hipEventElapsedTime(&e, t.a, t.b));
        B->stage_ms[t.stage] += e;
        B->stage_count[t.stage] += 1;
        B->free_events.push_back(t.a);
        B->free_events.push_back(t.b);
    }
    B->timed.clear();
    for (int k = 0; k < SPL_N_STAGES; ++k) {
        if (ms) ms[k] = B->stage_ms[k];
        if (count) count[k] = B->stage_count[k];
        if (reset) {
            B->stage_ms[k] = 0;
            B->stage_count[k] = 0;
        }
    }
    return SPL_OK;
}

extern "C" void spl_batch_destroy(spl_batch *B) {
    if (!B) return;
    for (auto &t : B->timed) {
        (void)hipEventSynchronize(t.b);
        B->free_events.push_back(t.a);
        B->free_events.push_back(t.b);
    }
    for (hipEvent_t e : B->free_events) (void)hipEventDestroy(e);
    if (B->staging_pending) (void)hipEventSynchronize(B->staging_done);
    if (B->graph_exec) (void)hipGraphExecDestroy(B->graph_exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    if (B->staging_done) (void)hipEventDestroy(B->staging_done);
    if (B->staging) (void)hipHostFree(B->staging);
    delete B;
}

// ------------------------------------------------------------- test hook
extern "C" spl_status spl_corner_turn(const uint8_t *d_in, int64_t n_t, int32_t nch, int64_t in_stride,
                                      uint8_t *d_out, int64_t pitch, hipStream_t stream) {
    if (n_t < 0 || nch < 1) return fail(SPL_E_INVALID_ARG, "spl_corner_turn: need n_t >= 0 and nch >= 1");
    if (n_t == 0) return SPL_OK;
    if (!d_in || !d_out) return fail(SPL_E_INVALID_ARG, "spl_corner_turn: NULL buffer");
    if (nch % 16 != 0) return fail(SPL_E_UNSUPPORTED, "spl_corner_turn: nch must be a multiple of 16 (got %d)", nch);
    if (in_stride < nch || in_stride % 16 != 0)
        return fail(SPL_E_INVALID_ARG, "spl_corner_turn: in_stride must be a multiple of 16 and >= nch");
    if (pitch < n_t || pitch % 16 != 0)
        return fail(SPL_E_INVALID_ARG, "spl_corner_turn: pitch must be a multiple of 16 and >= n_t");
    if (((uintptr_t)d_in & 15) || ((uintptr_t)d_out & 15))
        return fail(SPL_E_INVALID_ARG, "spl_corner_turn: buffers must be 16-byte aligned");
    HIP_TRY(launch_corner_turn(d_in, in_stride, n_t, nch, d_out, pitch, stream));
    return SPL_OK;
}

static_assert(SPL_INJECT_ARGMAX == SPL_INJECT_ARGMAX_MODE, "injection mode numbers");

extern "C" spl_status spl_inject_quantised(uint8_t *d_block, int64_t pitch, int64_t n_t, int32_t nch,
                                           const int32_t *d_t_start, const float *d_signal, const uint32_t *d_random,
                                           int32_t n_win, int32_t n_sig, const spl_quantiser *q, int32_t mode,
                                           hipStream_t stream) {
    if (!q) return fail(SPL_E_INVALID_ARG, "spl_inject_quantised: quantiser is NULL");
    if (q->bits < 1 || q->bits > 8) return fail(SPL_E_INVALID_ARG, "spl_inject_quantised: bits must be 1..8");
    if (!(q->sigma > 0) || !std::isfinite(q->sigma) || !(q->level > 0) || !std::isfinite(q->level) ||
        !std::isfinite(q->mu) || !std::isfinite(q->offset) || !std::isfinite(q->level * q->sigma))
        return fail(SPL_E_INVALID_ARG, "spl_inject_quantised: need finite mu and offset, sigma > 0, level > 0");
    if (mode != SPL_INJECT_SAMPLE && mode != SPL_INJECT_ARGMAX)
        return fail(SPL_E_INVALID_ARG, "spl_inject_quantised: unknown mode %d", mode);
    if (nch < 1 || n_t < 0 || pitch < n_t || n_win < 0 || n_sig < 0)
        return fail(SPL_E_INVALID_ARG, "spl_inject_quantised: need nch >= 1, 0 <= n_t <= pitch, n_win, n_sig >= 0");
    if (n_t == 0 || n_win == 0 || n_sig == 0) return SPL_OK;
    if (!d_block || !d_t_start || !d_signal) return fail(SPL_E_INVALID_ARG, "spl_inject_quantised: NULL buffer");
    if (mode == SPL_INJECT_SAMPLE && !d_random)
        return fail(SPL_E_INVALID_ARG, "spl_inject_quantised: SAMPLE mode needs random words");
    HIP_TRY(launch_inject(d_block, pitch, n_t, nch, d_t_start, d_signal, mode == SPL_INJECT_SAMPLE ? d_random : nullptr,
                          n_win, n_sig, q->bits, q->mu, q->sigma, q->level, q->offset, mode, stream));
    return SPL_OK;
}

extern "C" spl_status spl_ranker_snippets(const spl_batch *B, const spl_candidate *d_cands, int64_t n,
                                          uint16_t *d_out, hipStream_t stream) {
    if (!B) return fail(SPL_E_INVALID_ARG, "batch is NULL");
    if (n < 0 || (n > 0 && (!d_cands || !d_out))) return fail(SPL_E_INVALID_ARG, "bad candidate or output buffer");
    if (!B->tables_uploaded) return fail(SPL_E_INVALID_ARG, "spl_batch_set_workspace was not called");
    for (int b = 0; b < B->nb; ++b) {
        if (B->plans[b]->nch % SPL_SNIPPET_ROWS != 0)
            return fail(SPL_E_UNSUPPORTED, "snippets need nchans a multiple of 64 (beam %d has %d)", b,
                        B->plans[b]->nch);
        if (!B->cur_x[b]) return fail(SPL_E_INVALID_ARG, "the batch has not run: no block for beam %d", b);
    }
    HIP_TRY(launch_snippets((const DevBeam *)(B->ws + B->off_beams), B->nb, d_cands, n, d_out, stream));
    return SPL_OK;
}

extern "C" spl_status spl_ranker_snippets_fine(const spl_batch *B, const spl_candidate *d_cands, int64_t n,
                                               double keep, uint16_t *d_out, hipStream_t stream) {
    if (!(keep > 0.0 && keep < 1.0)) return fail(SPL_E_INVALID_ARG, "spl_ranker_snippets_fine: keep must be in (0, 1)");
    const spl_status st = spl_ranker_snippets(B, d_cands, n, d_out, stream);
    if (st != SPL_OK || n == 0) return st;
    for (int b = 0; b < B->nb; ++b)
        if (B->plans[b]->nch > 16384)
            return fail(SPL_E_UNSUPPORTED, "fine-DM snippets need nchans <= 16384 (beam %d has %d)", b,
                        B->plans[b]->nch);
    HIP_TRY(launch_fine_dm((const DevBeam *)(B->ws + B->off_beams), B->nb, d_cands, n, keep, d_out, stream));
    return SPL_OK;
}

extern "C" spl_status spl_debug_mu_sigma(const int64_t *d_n, const int64_t *d_s1, const int64_t *d_s2,
                                         int64_t count, double *d_mu, double *d_sigma, hipStream_t stream) {
    if (count < 0 || (count > 0 && (!d_n || !d_s1 || !d_s2 || !d_mu || !d_sigma)))
        return fail(SPL_E_INVALID_ARG, "bad argument");
    HIP_TRY(launch_mu_sigma(d_n, d_s1, d_s2, count, d_mu, d_sigma, stream));
    return SPL_OK;
}

// DM sub-ranges with smearing-limited spacing (host code): the trial step of a sub-range
// keeps the S/N of a pulse half a step off above 1 - max_loss, after the S/N-loss law of
// a Gaussian pulse dedispersed at a wrong DM (Eq. snrloss, zeta of Eq. zetadef), for the
// narrowest pulse the trial can see (sampling time and intra-channel smearing in
// quadrature).  Steps are powers of two, so every trial DM is exact in binary64.
#include <cmath>
#include <vector>

#include "spotlight.h"

#pragma STDC FP_CONTRACT OFF

spl_status spl_internal_fail(spl_status st, const char *msg);

namespace {

struct Smear {
    double tsamp_ms, w_min_ms, chan_mhz, nu_lo_ghz, nu_c_ghz, bw_mhz, keep_min;

    // narrowest effective width seen by a trial at DM (ms)
    double width_ms(double dm) const {
        const double tc = 8.3e-3 * dm * chan_mhz / (nu_lo_ghz * nu_lo_ghz * nu_lo_ghz);
        return std::sqrt(w_min_ms * w_min_ms + tsamp_ms * tsamp_ms + tc * tc);
    }
    // does a pulse half a step off keep at least keep_min of its S/N at DM
    bool allowed(double step, double dm) const {
        const double z = 6.91e-3 * (0.5 * step) * bw_mhz / (width_ms(dm) * (nu_c_ghz * nu_c_ghz * nu_c_ghz));
        const double keep = z == 0.0 ? 1.0 : (std::sqrt(M_PI) / 2.0) * std::erf(z) / z;
        return keep >= keep_min;
    }
};

}  // namespace

extern "C" spl_status spl_plan_smearing_ranges(const spl_band *band, const spl_smearing_opts *o, spl_dm_range *out,
                                               int32_t capacity, int32_t *n_out) {
    if (!band || !o || !n_out || capacity < 0 || (capacity > 0 && !out))
        return spl_internal_fail(SPL_E_INVALID_ARG, "spl_plan_smearing_ranges: NULL argument");
    if (band->nchans < 1 || !(band->tsamp_s > 0.0) || !(band->foff_mhz != 0.0) || !std::isfinite(band->fch1_mhz))
        return spl_internal_fail(SPL_E_INVALID_ARG, "spl_plan_smearing_ranges: bad band");
    if (!(o->dm_min >= 0.0) || !(o->dm_max > o->dm_min) || !std::isfinite(o->dm_max) || !(o->max_loss > 0.0) ||
        !(o->max_loss < 1.0) || !(o->w_min_s >= 0.0))
        return spl_internal_fail(SPL_E_INVALID_ARG, "spl_plan_smearing_ranges: bad options");
    const double f0 = band->fch1_mhz, f1 = band->fch1_mhz + (band->nchans - 1) * band->foff_mhz;
    const double lo = f0 < f1 ? f0 : f1, hi = f0 < f1 ? f1 : f0;
    if (!(lo > 0.0)) return spl_internal_fail(SPL_E_INVALID_ARG, "spl_plan_smearing_ranges: frequencies must be > 0");
    Smear S;
    S.tsamp_ms = band->tsamp_s * 1e3;
    S.w_min_ms = o->w_min_s * 1e3;
    S.chan_mhz = std::fabs(band->foff_mhz);
    S.nu_lo_ghz = lo / 1e3;
    S.nu_c_ghz = (0.5 * (lo + hi)) / 1e3;
    S.bw_mhz = band->nchans * std::fabs(band->foff_mhz);
    S.keep_min = 1.0 - o->max_loss;
    int e = 20;   // first step: the largest allowed power of two at dm_min
    while (e > -30 && !S.allowed(std::ldexp(1.0, e), o->dm_min)) --e;
    if (e <= -30) return spl_internal_fail(SPL_E_UNSUPPORTED, "spl_plan_smearing_ranges: no step is allowed");
    std::vector<spl_dm_range> r;
    double start = o->dm_min, step = std::ldexp(1.0, e);
    for (int64_t i = 0;; ++i) {
        const double dm = start + (double)i * step;
        if (dm >= o->dm_max) {
            r.push_back({start, step, (int32_t)(i + 1), 0});
            break;
        }
        if (i >= 1 && S.allowed(2.0 * step, dm)) {
            r.push_back({start, step, (int32_t)i, 0});
            start = dm;
            step = 2.0 * step;
            i = 0;
            if (start >= o->dm_max) {   // the switch landed on the end: one trial covers it
                r.push_back({start, step, 1, 0});
                break;
            }
        }
        if (i > (1 << 30)) return spl_internal_fail(SPL_E_UNSUPPORTED, "spl_plan_smearing_ranges: too many trials");
    }
    *n_out = (int32_t)r.size();
    for (int32_t k = 0; k < *n_out && k < capacity; ++k) out[k] = r[k];
    if (*n_out > capacity)
        return spl_internal_fail(SPL_E_CAPACITY, "spl_plan_smearing_ranges: more sub-ranges than capacity");
    return SPL_OK;
}

// Plain candidate-optimisation path (candidate optimisation section of the paper):
// per beam, DBSCAN in the DM-time plane (clusters of at least min_pts points within
// eps), the highest-S/N member of each cluster kept, noise dropped; then S/N, DM and
// width thresholds; then the anti-coincidence filter across the batch's beams.
// Host code.  DBSCAN uses a uniform grid only to prune the neighbour search; the
// neighbour predicate itself is evaluated exactly as written below.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>
#include <vector>

#include "spotlight.h"

#pragma STDC FP_CONTRACT OFF

spl_status spl_internal_fail(spl_status st, const char *msg);

extern "C" void spl_opt_defaults(spl_opt_params *p) {
    if (!p) return;
    p->eps = 0.5;
    p->min_pts = 5;
    p->coinc_min_beams = 3;
    p->t_scale_s = 0.05;
    p->dm_scale = 20.0;
    p->snr_min = 10.0;
    p->dm_min = 10.0;
    p->width_max_s = 0.100;
    p->coinc_dt_s = 0.05;
    p->coinc_frac = 0.5;
}

namespace {

struct Pt {
    double x, y;
};

// DBSCAN labels (-1 noise) for points in the given order; see spl_optimise_plain.
std::vector<int> dbscan(const std::vector<Pt> &pts, double eps, int min_pts) {
    const size_t n = pts.size();
    const double e2 = eps * eps;
    std::vector<int> label(n, -1);
    if (n == 0) return label;
    // grid of cell size eps; neighbours are searched in the 5x5 surrounding cells, a
    // margin that covers every rounding of the cell index
    // (cell indices can be negative: the shift is done on their two's-complement bits)
    auto key = [](long long cx, long long cy) {
        return (long long)(((unsigned long long)cx << 32) ^ ((unsigned long long)cy & 0xffffffffULL));
    };
    std::unordered_map<long long, std::vector<int>> grid;
    grid.reserve(n * 2);
    std::vector<long long> cxs(n), cys(n);
    for (size_t i = 0; i < n; ++i) {
        cxs[i] = (long long)std::floor(pts[i].x / eps);
        cys[i] = (long long)std::floor(pts[i].y / eps);
        grid[key(cxs[i], cys[i])].push_back((int)i);
    }
    auto neighbours = [&](int p, std::vector<int> &out) {
        out.clear();
        for (long long dx = -2; dx <= 2; ++dx)
            for (long long dy = -2; dy <= 2; ++dy) {
                auto it = grid.find(key(cxs[p] + dx, cys[p] + dy));
                if (it == grid.end()) continue;
                for (int q : it->second) {
                    const double ddx = pts[p].x - pts[q].x, ddy = pts[p].y - pts[q].y;
                    if (ddx * ddx + ddy * ddy <= e2) out.push_back(q);
                }
            }
    };
    std::vector<char> core(n, 0);
    std::vector<std::vector<int>> nb(n);
    for (size_t p = 0; p < n; ++p) {
        neighbours((int)p, nb[p]);
        core[p] = (int)nb[p].size() >= min_pts;
    }
    // connected components of core points, numbered by their lowest-index core point
    std::vector<int> parent(n);
    std::iota(parent.begin(), parent.end(), 0);
    auto find = [&](int a) {
        while (parent[a] != a) {
            parent[a] = parent[parent[a]];
            a = parent[a];
        }
        return a;
    };
    for (size_t p = 0; p < n; ++p) {
        if (!core[p]) continue;
        for (int q : nb[p]) {
            if (!core[q]) continue;
            int a = find((int)p), b = find(q);
            if (a != b) parent[std::max(a, b)] = std::min(a, b);
        }
    }
    int ncl = 0;
    std::vector<int> comp_label(n, -1);
    for (size_t p = 0; p < n; ++p) {
        if (!core[p]) continue;
        const int r = find((int)p);   // the root is the lowest index of the component
        if (comp_label[r] < 0) comp_label[r] = ncl++;
        label[p] = comp_label[r];
    }
    for (size_t p = 0; p < n; ++p) {
        if (core[p]) continue;
        int best = -1;
        for (int q : nb[p])
            if (core[q] && (best < 0 || label[q] < best)) best = label[q];
        label[p] = best;
    }
    return label;
}

// Candidates that survive the anti-coincidence filter (any order in, same order out).
std::vector<spl_candidate> anti_coincidence(const std::vector<spl_candidate> &thr, const double *tsamp_of_beam,
                                            int n_beams, const spl_opt_params &P) {
    if (!(n_beams >= P.coinc_min_beams) || thr.empty()) return thr;
    std::vector<spl_candidate> fin;
    std::vector<double> tabs(thr.size());
    for (size_t i = 0; i < thr.size(); ++i) tabs[i] = (double)thr[i].t_sample * tsamp_of_beam[thr[i].beam];
    std::vector<size_t> order(thr.size());
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](size_t a, size_t c) { return tabs[a] < tabs[c]; });
    std::vector<char> seen(n_beams, 0);
    for (size_t i = 0; i < thr.size(); ++i) {
        std::fill(seen.begin(), seen.end(), 0);
        int nb = 0;
        // candidates within coinc_dt_s, found by scanning the time-sorted list
        auto lo = std::lower_bound(order.begin(), order.end(), tabs[i] - P.coinc_dt_s - 1.0,
                                   [&](size_t a, double v) { return tabs[a] < v; });
        for (auto it = lo; it != order.end() && tabs[*it] <= tabs[i] + P.coinc_dt_s + 1.0; ++it) {
            if (std::fabs(tabs[*it] - tabs[i]) <= P.coinc_dt_s && !seen[thr[*it].beam]) {
                seen[thr[*it].beam] = 1;
                ++nb;
            }
        }
        if (!((double)nb > P.coinc_frac * (double)n_beams)) fin.push_back(thr[i]);
    }
    return fin;
}

void sort_records(std::vector<spl_candidate> &v) {
    std::sort(v.begin(), v.end(), [](const spl_candidate &a, const spl_candidate &c) {
        if (a.beam != c.beam) return a.beam < c.beam;
        if (a.dm_index != c.dm_index) return a.dm_index < c.dm_index;
        return a.t_sample < c.t_sample;
    });
}

}  // namespace

extern "C" spl_status spl_anti_coincidence(const spl_candidate *cands, int64_t n, const double *tsamp_of_beam,
                                           int32_t n_beams, const spl_opt_params *params, spl_candidate *out,
                                           int64_t capacity, int64_t *n_out) {
    if (n < 0 || (n > 0 && !cands) || !tsamp_of_beam || n_beams < 1 || !n_out || capacity < 0 ||
        (capacity > 0 && !out))
        return spl_internal_fail(SPL_E_INVALID_ARG, "spl_anti_coincidence: bad argument");
    spl_opt_params P;
    if (params) P = *params; else spl_opt_defaults(&P);
    for (int64_t i = 0; i < n; ++i)
        if (cands[i].beam < 0 || cands[i].beam >= n_beams)
            return spl_internal_fail(SPL_E_INVALID_ARG, "spl_anti_coincidence: candidate beam out of range");
    std::vector<spl_candidate> in(cands, cands + n);
    std::vector<spl_candidate> fin = anti_coincidence(in, tsamp_of_beam, n_beams, P);
    sort_records(fin);
    *n_out = (int64_t)fin.size();
    const int64_t m = std::min<int64_t>(capacity, (int64_t)fin.size());
    if (m > 0) std::memcpy(out, fin.data(), (size_t)m * sizeof(spl_candidate));
    if ((int64_t)fin.size() > capacity)
        return spl_internal_fail(SPL_E_CAPACITY, "spl_anti_coincidence: more survivors than capacity");
    return SPL_OK;
}

extern "C" spl_status spl_optimise_plain(const spl_candidate *cands, int64_t n, const double *tsamp_of_beam,
                                         int32_t n_beams, const spl_opt_params *params, spl_candidate *out,
                                         int64_t capacity, int64_t *n_out) {
    if (n < 0 || (n > 0 && !cands) || !tsamp_of_beam || n_beams < 1 || !n_out || capacity < 0 ||
        (capacity > 0 && !out))
        return spl_internal_fail(SPL_E_INVALID_ARG, "spl_optimise_plain: bad argument");
    spl_opt_params P;
    if (params) P = *params; else spl_opt_defaults(&P);
    if (!(P.eps > 0.0) || P.min_pts < 1 || !(P.t_scale_s > 0.0) || !(P.dm_scale > 0.0))
        return spl_internal_fail(SPL_E_INVALID_ARG, "spl_optimise_plain: bad parameters");
    for (int64_t i = 0; i < n; ++i)
        if (cands[i].beam < 0 || cands[i].beam >= n_beams)
            return spl_internal_fail(SPL_E_INVALID_ARG, "spl_optimise_plain: candidate beam out of range");

    // per beam, in (DM index, t) order
    std::vector<std::vector<int64_t>> per_beam(n_beams);
    for (int64_t i = 0; i < n; ++i) per_beam[cands[i].beam].push_back(i);
    std::vector<spl_candidate> kept;
    for (int b = 0; b < n_beams; ++b) {
        auto &idx = per_beam[b];
        std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t c) {
            if (cands[a].dm_index != cands[c].dm_index) return cands[a].dm_index < cands[c].dm_index;
            return cands[a].t_sample < cands[c].t_sample;
        });
        if (idx.empty()) continue;
        const double ts = tsamp_of_beam[b];
        std::vector<Pt> pts(idx.size());
        for (size_t k = 0; k < idx.size(); ++k) {
            pts[k].x = (double)cands[idx[k]].t_sample * ts / P.t_scale_s;
            pts[k].y = (double)cands[idx[k]].dm / P.dm_scale;
        }
        const std::vector<int> lab = dbscan(pts, P.eps, P.min_pts);
        int ncl = 0;
        for (int l : lab) ncl = std::max(ncl, l + 1);
        std::vector<int64_t> best(ncl, -1);
        for (size_t k = 0; k < idx.size(); ++k) {
            const int l = lab[k];
            if (l < 0) continue;
            if (best[l] < 0 || cands[idx[k]].snr > cands[idx[best[l]]].snr) best[l] = (int64_t)k;
        }
        for (int l = 0; l < ncl; ++l)
            if (best[l] >= 0) kept.push_back(cands[idx[best[l]]]);
    }
    // thresholds
    std::vector<spl_candidate> thr;
    for (const auto &c : kept) {
        const double ts = tsamp_of_beam[c.beam];
        if (c.snr >= (float)P.snr_min && (double)c.dm >= P.dm_min && (double)c.width * ts <= P.width_max_s)
            thr.push_back(c);
    }
    // anti-coincidence across the batch's beams
    std::vector<spl_candidate> fin = anti_coincidence(thr, tsamp_of_beam, n_beams, P);
    sort_records(fin);
    *n_out = (int64_t)fin.size();
    const int64_t m = std::min<int64_t>(capacity, (int64_t)fin.size());
    if (m > 0) std::memcpy(out, fin.data(), (size_t)m * sizeof(spl_candidate));
    if ((int64_t)fin.size() > capacity)
        return spl_internal_fail(SPL_E_CAPACITY, "spl_optimise_plain: more survivors than capacity");
    return SPL_OK;
}

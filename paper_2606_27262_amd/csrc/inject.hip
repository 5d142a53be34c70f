// Quantised-domain injection (the appendix on injecting a signal into an M-bit quantised
// stream): every sample of a signal window moves from its state n to a state k >= n
// with the probability that Gaussian noise known to lie in state n, shifted by the
// signal, lands in state k.
//
// One wave per (window, channel) row, its lanes on 64 consecutive samples at a time, so
// the byte loads and stores and the FP32/u32 window loads are coalesced; zero signal
// (the padding of narrow bursts) costs one load.  The work is
// binary64 arithmetic (a few erfc per sample), not memory: a burst's window holds
// ~10^5-10^6 values per beam.
//
// The transition row is never formed.  The cumulative row sum up to state k is the mass
// of [e_{n-1}, min(e_n, e_k - S)) over the mass of state n, monotone in k, so SAMPLE
// mode binary-searches the first k where it exceeds u; ARGMAX compares the masses of the
// candidate states, successive differences of that cumulative mass.  Only states whose
// shifted interval can meet state n are visited: from n + floor(S/w) - 1 to
// n + floor(S/w) + 2 (w the state width), one state of slack on each side for rounding;
// state 0, unbounded below, can reach any state up to the last of those.
#include <hip/hip_runtime.h>

#include <cmath>

#include "inject.h"

namespace spl {

namespace {

struct Edges {
    double mu, sigma, width, offset;
    int half, top;

    // Upper edge of state k (k in [-1, top)): -inf below state 0.
    __device__ double edge(int k) const {
        if (k < 0) return -INFINITY;
        return mu + ((double)(k + 1 - half) + offset) * width;
    }
};

// Gaussian mass inside one state [lo, hi), measured from lo: g(x) = mass of
// [lo, min(x, hi)).  All values come from one tail of the distribution (the upper one
// for a state above the mean), so the narrow differences near the band's ends keep
// their relative precision; one erfc per evaluation.
struct StateMass {
    double mu, inv_sigma, lo, hi, f_lo, den;
    bool upper;

    __device__ double tail(double x) const {
        const double z = (x - mu) * inv_sigma * 0.70710678118654752440;   // 1/sqrt(2)
        return upper ? 0.5 * erfc(z) : 0.5 * erfc(-z);
    }
    __device__ void init(const Edges &E, int n) {
        mu = E.mu;
        inv_sigma = 1.0 / E.sigma;
        lo = E.edge(n - 1);
        hi = E.edge(n);
        upper = lo >= E.mu;
        f_lo = tail(lo);
        const double f_hi = tail(hi);
        den = upper ? f_lo - f_hi : f_hi - f_lo;
    }
    __device__ double g(double x) const {
        if (!(x > lo)) return 0.0;
        if (x >= hi) return den;
        return upper ? f_lo - tail(x) : tail(x) - f_lo;
    }
};

// n < top; S > 0.
__device__ int new_state(const Edges &E, int n, double S, uint32_t word, int mode) {
    StateMass M;
    M.init(E, n);
    if (!(M.den > 0.0)) return n;
    const double f = fmin(floor(S / E.width), (double)(E.top + 2));
    const int shift = (int)f;
    int k_lo = n == 0 ? 0 : min(E.top, max(n, n + shift - 1));
    int k_hi = min(E.top, n + shift + 2);
    if (mode == SPL_INJECT_ARGMAX_MODE) {
        // mass landing in state k: g(e_k - S) - g(e_{k-1} - S); the top state takes the rest
        double prev = k_lo == 0 ? 0.0 : M.g(E.edge(k_lo - 1) - S);
        int best = k_lo;
        double best_mass = -1.0;
        for (int k = k_lo; k <= k_hi; ++k) {
            const double cur = k >= E.top ? M.den : M.g(E.edge(k) - S);
            if (cur - prev > best_mass) {
                best_mass = cur - prev;
                best = k;
            }
            prev = cur;
        }
        return best;
    }
    // first k whose cumulative row sum g(e_k - S) / den exceeds u
    const double target = ((double)word + 0.5) * (1.0 / 4294967296.0) * M.den;
    while (k_lo < k_hi) {
        const int k = (k_lo + k_hi) >> 1;
        if (k >= E.top || M.g(E.edge(k) - S) > target)
            k_hi = k;
        else
            k_lo = k + 1;
    }
    return k_lo;
}

constexpr int kRowsPerBlock = 4;   // one wave per (window, channel) row

__global__ __launch_bounds__(64 * kRowsPerBlock) void k_inject(uint8_t *__restrict__ block, int64_t pitch,
                                                                int64_t n_t, int nch,
                                                                const int32_t *__restrict__ t_start,
                                                                const float *__restrict__ signal,
                                                                const uint32_t *__restrict__ words, int64_t n_rows,
                                                                int n_sig, Edges E, int mode) {
    const int64_t row = (int64_t)blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6);
    if (row >= n_rows) return;
    const int c = (int)(row % nch);
    const int64_t t0 = t_start[row];
    uint8_t *line = block + (int64_t)c * pitch;
    const int64_t base = row * n_sig;
    for (int j = threadIdx.x & 63; j < n_sig; j += 64) {
        const double S = (double)signal[base + j];
        if (!(S > 0.0)) continue;
        const int64_t t = t0 + j;
        if (t < 0 || t >= n_t) continue;
        const int n = line[t];
        if (n >= E.top) continue;   // the top state keeps its samples; bytes above it are not states
        const uint32_t word = words ? words[base + j] : 0u;
        line[t] = (uint8_t)new_state(E, n, S, word, mode);
    }
}

}  // namespace

hipError_t launch_inject(uint8_t *block, int64_t pitch, int64_t n_t, int nch, const int32_t *t_start,
                         const float *signal, const uint32_t *words, int n_win, int n_sig, int bits, double mu,
                         double sigma, double level, double offset, int mode, hipStream_t s) {
    if (n_win <= 0 || n_sig <= 0 || nch <= 0 || n_t <= 0) return hipSuccess;
    Edges E;
    E.mu = mu;
    E.sigma = sigma;
    E.width = level * sigma;
    E.offset = offset;
    E.half = 1 << (bits - 1);
    E.top = (1 << bits) - 1;
    const int64_t n_rows = (int64_t)n_win * nch;
    const int64_t gx = (n_rows + kRowsPerBlock - 1) / kRowsPerBlock;
    if (gx > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_inject, dim3((unsigned)gx), dim3(64 * kRowsPerBlock), 0, s, block, pitch, n_t, nch, t_start,
                       signal, words, n_rows, n_sig, E, mode);
    return hipGetLastError();
}

}  // namespace spl

// Exact energy of one configuration (Eq. (1)) and the Metropolis
// independence step over one instance's proposals (Eq. (10)), as device
// functions shared by the stand-alone kernels and the fused pipeline.
#pragma once
#include "device.hpp"

namespace tnmc {

struct Chain {
    double cur_logq, cur_E;
    int64_t cur_index, n_acc, n_trials, initialised;
};

// Energy of the configuration s (L rows of W words) by one wave; every lane
// returns the sum.  Each lane takes whole rows: the horizontal bonds of row
// r and the vertical bonds from row r to r+1.  With +-1 or 2^-20-grid
// couplings every partial sum is exact in float64, so the result does not
// depend on the summation order.
__device__ inline double energy_wave(const InstDesc &d, const uint64_t *s, const float *Jh_all,
                                     const float *Jv_all, int lane) {
    const int L = d.L, W = d.W;
    const float *jh = Jh_all + d.off_h, *jv = Jv_all + d.off_v;
    double e = 0.0;
    for (int r = lane; r < L; r += 64) {
        const uint64_t *row = s + (size_t)r * W, *nxt = s + (size_t)(r + 1) * W;
        for (int c = 0; c < L; ++c) {
            const double sc = ((row[c >> 6] >> (c & 63)) & 1) ? 1.0 : -1.0;
            if (c + 1 < L) {
                const double sr = ((row[(c + 1) >> 6] >> ((c + 1) & 63)) & 1) ? 1.0 : -1.0;
                e -= (double)jh[(size_t)r * (L - 1) + c] * (sc * sr);
            }
            if (r + 1 < L) {
                const double sd = ((nxt[c >> 6] >> (c & 63)) & 1) ? 1.0 : -1.0;
                e -= (double)jv[(size_t)r * L + c] * (sc * sd);
            }
        }
    }
    for (int m = 32; m > 0; m >>= 1) e += __shfl_xor(e, m, 64);
    return e;
}

// The same sum in integer arithmetic, for couplings that are integers
// (+-J): every lane returns the energy, or INT64_MIN when some coupling of
// the instance is not an integer of magnitude below 2^20 (|E| then stays
// below 2^42, far inside int64; the int32 result is exact for L <= 1024,
// where |E| <= 2 L (L-1) max|J|, with +-1 couplings).
__device__ inline int64_t energy_wave_int(const InstDesc &d, const uint64_t *s, const float *Jh_all,
                                          const float *Jv_all, int lane) {
    const int L = d.L, W = d.W;
    const float *jh = Jh_all + d.off_h, *jv = Jv_all + d.off_v;
    int64_t e = 0;
    int bad = 0;
    for (int r = lane; r < L; r += 64) {
        const uint64_t *row = s + (size_t)r * W, *nxt = s + (size_t)(r + 1) * W;
        for (int c = 0; c < L; ++c) {
            const int sc = ((row[c >> 6] >> (c & 63)) & 1) ? 1 : -1;
            if (c + 1 < L) {
                const float j = jh[(size_t)r * (L - 1) + c];
                bad |= !(j == rintf(j) && fabsf(j) < 1048576.0f);
                const int sr = ((row[(c + 1) >> 6] >> ((c + 1) & 63)) & 1) ? 1 : -1;
                e -= (int64_t)j * (sc * sr);
            }
            if (r + 1 < L) {
                const float j = jv[(size_t)r * L + c];
                bad |= !(j == rintf(j) && fabsf(j) < 1048576.0f);
                const int sd = ((nxt[c >> 6] >> (c & 63)) & 1) ? 1 : -1;
                e -= (int64_t)j * (sc * sd);
            }
        }
    }
    for (int m = 32; m > 0; m >>= 1) {
        e += __shfl_xor(e, m, 64);
        bad |= __shfl_xor(bad, m, 64);
    }
    return bad ? INT64_MIN : e;
}

// Instance i's chain walks its n proposals (log q, E) in index order: the
// first ever proposal initialises it; then with current state x and
// candidate k, delta = (lq_x - lq_k) + beta (E_x - E_k), each operation
// rounded once; accept iff delta >= 0 or u < exp(delta), u the Philox draw
// of counter (global index, 0, i, 1).
__device__ inline void accept_chain(int i, int n, const double *lq_i, const double *E_i, double b,
                                    Chain *chain_i, uint64_t seed, uint64_t step_offset, uint8_t *acc_i,
                                    int64_t *state_i) {
#pragma clang fp contract(off)
    Chain ch = *chain_i;
    for (int k = 0; k < n; ++k) {
        const uint64_t g = step_offset + (uint64_t)k;
        const double lq = lq_i[k], e = E_i[k];
        uint8_t a = 0;
        if (!ch.initialised) {
            ch.initialised = 1;
            ch.cur_logq = lq; ch.cur_E = e; ch.cur_index = (int64_t)g;
            a = 1;
        } else {
            const double d_logq = ch.cur_logq - lq;
            const double d_E = ch.cur_E - e;
            const double prod = b * d_E;
            const double delta = d_logq + prod;
            const double u = philox_unit(seed, (uint32_t)g, 0u, (uint32_t)i, 1u);
            const bool ok = (delta >= 0.0) || (u < exp(delta));
            ch.n_trials += 1;
            if (ok) {
                ch.n_acc += 1;
                ch.cur_logq = lq; ch.cur_E = e; ch.cur_index = (int64_t)g;
                a = 1;
            }
        }
        acc_i[k] = a;
        if (state_i) state_i[k] = ch.cur_index;
    }
    *chain_i = ch;
}

}  // namespace tnmc

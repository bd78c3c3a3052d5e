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
// returns the sum.  Lanes take columns (c = lane, lane + 64, ...) so that
// the couplings of a row are read contiguously; the spin word of a row is
// the same for a whole group of 64 columns.  With +-1 or 2^-20-grid
// couplings every partial sum is exact in float64, so the result does not
// depend on the summation order.  With eint non-NULL the same sum is also
// taken in integer arithmetic (*eint = INT64_MIN if some coupling is not an
// integer of magnitude below 2^20).
__device__ inline double energy_wave(const InstDesc &d, const uint64_t *s, const float *Jh_all,
                                     const float *Jv_all, int lane, int64_t *eint = nullptr) {
    const int L = d.L, W = d.W;
    const float *jh = Jh_all + d.off_h, *jv = Jv_all + d.off_v;
    double e = 0.0;
    int64_t ei = 0;
    int bad = 0;
    for (int r = 0; r < L; ++r) {
        const uint64_t *row = s + (size_t)r * W, *nxt = s + (size_t)(r + 1) * W;
        for (int c = lane; c < L; c += 64) {
            const int k = c >> 6;
            const uint64_t w = row[k];
            const int b = (int)((w >> (c & 63)) & 1);
            if (c + 1 < L) {
                const int b1 = (int)(((c & 63) == 63 ? row[k + 1] : w) >> ((c + 1) & 63) & 1);
                const float j = jh[(size_t)r * (L - 1) + c];
                const int ss = (b == b1) ? 1 : -1;
                e -= (double)j * (double)ss;
                if (eint) {
                    bad |= !(j == rintf(j) && fabsf(j) < 1048576.0f);
                    ei -= (int64_t)j * ss;
                }
            }
            if (r + 1 < L) {
                const int bd = (int)((nxt[k] >> (c & 63)) & 1);
                const float j = jv[(size_t)r * L + c];
                const int ss = (b == bd) ? 1 : -1;
                e -= (double)j * (double)ss;
                if (eint) {
                    bad |= !(j == rintf(j) && fabsf(j) < 1048576.0f);
                    ei -= (int64_t)j * ss;
                }
            }
        }
    }
    for (int m = 32; m > 0; m >>= 1) e += __shfl_xor(e, m, 64);
    if (eint) {
        for (int m = 32; m > 0; m >>= 1) {
            ei += __shfl_xor(ei, m, 64);
            bad |= __shfl_xor(bad, m, 64);
        }
        *eint = bad ? INT64_MIN : ei;
    }
    return e;
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

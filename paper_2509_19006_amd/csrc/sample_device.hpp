// Row-by-row autoregressive sampling from the boundary-MPS cache
// (arXiv 2509.19006, section 3.3; chain rule Eq. (3) in raster order,
// conditional Eq. (4), sigmoid form Eq. (5)).
//
// A workgroup of NTS threads owns a tile of NTS samples of one instance, one
// sample per thread.  For every row r:
//   right sweep  R_{L-1} = e_0;  R_c = sum_s Bv(r-1,c+1)[u_{c+1}, s] A_{c+1,s} R_{c+1}
//                (u = the sample's spins of row r-1), rescaled by a power of
//                two and kept in a per-tile scratch [c][a][sample];
//   left sweep   l = e_0;  rho_s = |l A_{c,s} R_c|;
//                logit = ln rho_+ - ln rho_- + 2 beta J_v(r-1,c) u_c;
//                p = sigmoid(logit) in float64; spin = +1 iff Philox u < p
//                (or the given spin when scoring); log q += ln p or ln(1-p);
//                l = l A_{c,spin}, rescaled by a power of two.
// Each cache site (both spin slices, CHI x CHI, zero padded) is staged in
// shared memory once and read by every sample of the instance.
#pragma once
#include <type_traits>

#include "device.hpp"

namespace tnmc {

constexpr int NTS = 256;

// Element type of the staged sites in shared memory: a float16 cache stays
// float16 there (half the LDS traffic of the broadcast reads that bound the
// contractions; the conversion folds into the mixed-precision fma, and the
// float each fma sees is the same), every other form is staged in T.
template <typename T, typename S> struct StageType { using type = T; };
template <> struct StageType<float, __half> { using type = __half; };
template <typename T, typename ST> __device__ __forceinline__ T sget(ST v) {
    if constexpr (std::is_same<T, ST>::value) return v;
    else return __half2float(v);
}

// One tile of NTS samples of instance inst (all threads of the workgroup
// call it).  env: the tile's right-environment scratch; As: the shared
// array for the staged site.
template <typename T, typename S, int CHI>
__device__ void sample_tile(int inst, int tile, const InstDesc &d, unsigned char *__restrict__ ws, T *env,
                            int n_samples, uint64_t seed, uint64_t sample_offset,
                            const uint64_t *__restrict__ forced, uint64_t *spins_out,
                            double *__restrict__ logq_out, float *__restrict__ logits_out,
                            const float *__restrict__ Jv_all,
                            typename StageType<T, S>::type (*As)[CHI][CHI]) {
    // no implicit multiply-add fusion: the sampler gives the same bits in
    // every kernel it is inlined into; the contractions fuse explicitly
#pragma clang fp contract(off)
    using ST = typename StageType<T, S>::type;
    const int tid = threadIdx.x;
    const int n = tile * NTS + tid;
    const bool act = n < n_samples;
    const int L = d.L, chi = d.chi, W = d.W;
    const double beta = d.beta;
    const S *cache = reinterpret_cast<const S *>(ws + d.cache_off);
    const size_t site_sz = (size_t)2 * chi * chi, row_sz = (size_t)L * site_sz;
    const float *jv = Jv_all + d.off_v;
    const size_t wbase = (size_t)n_samples * d.word_prefix + (size_t)n * L * W;
    uint64_t *my_out = spins_out + wbase;
    const uint64_t *my_forced = forced ? forced + wbase : nullptr;
    float *my_logits = logits_out ? logits_out + (size_t)n_samples * d.site_prefix + (size_t)n * L * L : nullptr;
    const uint32_t sidx = (uint32_t)(sample_offset + (uint64_t)n);

    // Sites are staged through two shared buffers: the next site's entries
    // are fetched into registers before the current site is contracted and
    // stored into the other buffer after it, so one barrier per site
    // suffices and the fetch latency hides behind the contraction.
    // (the raw stored values are held: converting them at fetch time would
    // make the fetch wait for its loads before the contraction)
    constexpr int PER = (2 * CHI * CHI + NTS - 1) / NTS;
    S pre[PER];
    bool inb[PER];
    auto fetch = [&](const S *site) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + i * NTS;
            const int s = e / (CHI * CHI), a = (e / CHI) % CHI, b = e % CHI;
            inb[i] = e < 2 * CHI * CHI && a < chi && b < chi;
            if (inb[i]) pre[i] = site[(size_t)s * chi * chi + a * chi + b];
        }
    };
    auto put = [&](int buf) {
        ST *dst = &As[2 * buf][0][0];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + i * NTS;
            if (e < 2 * CHI * CHI) {
                if constexpr (std::is_same<ST, S>::value && !std::is_same<ST, T>::value)
                    dst[e] = inb[i] ? pre[i] : __float2half(0.f);
                else
                    dst[e] = inb[i] ? load_as<T, S>(&pre[i]) : (T)0;
            }
        }
    };

    double logq = 0.0;
    for (int r = 0; r < L; ++r) {
        const S *crow = cache + (size_t)r * row_sz;
        // ---------------- right environments ----------------
        {
            T R[CHI];
#pragma unroll
            for (int a = 0; a < CHI; ++a) R[a] = (a == 0) ? (T)1 : (T)0;
            int uw_idx = -1;
            uint64_t uw = 0;
            int buf = 0;
            if (L >= 2) {
                fetch(crow + (size_t)(L - 1) * site_sz);
                put(0);
            }
            __syncthreads();
            for (int c = L - 2; c >= 0; --c) {
                const bool more = c > 0;
                if (more) fetch(crow + (size_t)c * site_sz);
                ST (*Ab)[CHI][CHI] = As + 2 * buf;
                if (act) {
                T w0 = 1, w1 = 1;
                if (r > 0) {
                    const int cc = c + 1, wi = cc >> 6;
                    if (wi != uw_idx) { uw = my_out[(size_t)(r - 1) * W + wi]; uw_idx = wi; }
                    const int u = (int)((uw >> (cc & 63)) & 1);
                    double same, diff;
                    boltz(beta, jv[(size_t)(r - 1) * L + cc], same, diff);
                    w0 = (T)(u == 0 ? same : diff);
                    w1 = (T)(u == 1 ? same : diff);
                }
                T Rn[CHI];
                T mx = 0;
#pragma unroll
                for (int a = 0; a < CHI; ++a) {
                    T z0 = 0, z1 = 0;
#pragma unroll
                    for (int b = 0; b < CHI; ++b) {
                        z0 = fma(sget<T>(Ab[0][a][b]), R[b], z0);
                        z1 = fma(sget<T>(Ab[1][a][b]), R[b], z1);
                    }
                    Rn[a] = fma(w0, z0, w1 * z1);
                    mx = fmax(mx, fabs(Rn[a]));
                    __builtin_amdgcn_sched_barrier(0);
                }
                const T sc = mx > (T)0 ? pow2_inv(mx) : (T)1;
                T *ec = env + (size_t)c * CHI * NTS + tid;
#pragma unroll
                for (int a = 0; a < CHI; ++a) { R[a] = Rn[a] * sc; ec[(size_t)a * NTS] = R[a]; }
                }
                // one barrier site that every thread reaches
                if (more) put(buf ^ 1);
                __syncthreads();
                buf ^= 1;
            }
        }
        // ---------------- left sweep: sample the row ----------------
        {
            T l[CHI];
#pragma unroll
            for (int a = 0; a < CHI; ++a) l[a] = (a == 0) ? (T)1 : (T)0;
            uint64_t cur = 0, up = 0, fw = 0;
            int buf = 0;
            fetch(crow);
            put(0);
            __syncthreads();
            for (int c = 0; c < L; ++c) {
                const bool more = c + 1 < L;
                if (more) fetch(crow + (size_t)(c + 1) * site_sz);
                ST (*Ab)[CHI][CHI] = As + 2 * buf;
                // chi <= 16: the site's right environment, read before the
                // contraction so that its latency hides behind it (wider
                // forms read it after: the registers cost them more)
                constexpr bool PRE = CHI <= 16;
                T renv[PRE ? CHI : 1];
                if (PRE && act && c < L - 1) {
                    const T *ec = env + (size_t)c * CHI * NTS + tid;
#pragma unroll
                    for (int b = 0; b < CHI; ++b) renv[b] = ec[(size_t)b * NTS];
                }
                if (act) {
                // y_s = l A_{c,s} for both spins; every staged value is read once
                T y0[CHI], y1[CHI];
#pragma unroll
                for (int b = 0; b < CHI; ++b) { y0[b] = 0; y1[b] = 0; }
#pragma unroll
                for (int a = 0; a < CHI; ++a) {
                    const T la = l[a];
#pragma unroll
                    for (int b = 0; b < CHI; ++b) {
                        y0[b] = fma(la, sget<T>(Ab[0][a][b]), y0[b]);
                        y1[b] = fma(la, sget<T>(Ab[1][a][b]), y1[b]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
                // rho_s = y_s . R_c  (R_{L-1} = e_0)
                T r0, r1;
                if (c == L - 1) {
                    r0 = y0[0]; r1 = y1[0];
                } else if constexpr (PRE) {
                    r0 = 0; r1 = 0;
#pragma unroll
                    for (int b = 0; b < CHI; ++b) { r0 = fma(y0[b], renv[b], r0); r1 = fma(y1[b], renv[b], r1); }
                } else {
                    const T *ec = env + (size_t)c * CHI * NTS + tid;
                    r0 = 0; r1 = 0;
#pragma unroll
                    for (int b = 0; b < CHI; ++b) { const T rb = ec[(size_t)b * NTS]; r0 = fma(y0[b], rb, r0); r1 = fma(y1[b], rb, r1); }
                }
                const double rho0 = fabs((double)r0), rho1 = fabs((double)r1);
                double logit = 0.0;
                if ((c & 63) == 0) {
                    if (r > 0) up = my_out[(size_t)(r - 1) * W + (c >> 6)];
                    if (my_forced) fw = my_forced[(size_t)r * W + (c >> 6)];
                }
                if (rho0 > 0.0 || rho1 > 0.0) {
                    logit = log(rho1 / rho0);
                    if (r > 0) {
                        const double u = (double)((up >> (c & 63)) & 1);
                        logit += 2.0 * beta * (double)jv[(size_t)(r - 1) * L + c] * (2.0 * u - 1.0);
                    }
                }
                // sigma(logit) and ln sigma(+-logit) from one exponential:
                // with e = exp(-|logit|), sigma = 1/(1+e) or e/(1+e) and
                // ln sigma(x) = min(x, 0) - ln(1 + e)
                const double ex = exp(-fabs(logit));
                const double l1p = log1p(ex);
                int spin;
                if (my_forced) {
                    spin = (int)((fw >> (c & 63)) & 1);
                } else {
                    const double p = (logit >= 0.0 ? 1.0 : ex) / (1.0 + ex);
                    const double u = philox_unit(seed, (uint32_t)(r * L + c), sidx, (uint32_t)inst, 0u);
                    spin = (u < p) ? 1 : 0;
                }
                logq += (spin ? fmin(logit, 0.0) : fmin(-logit, 0.0)) - l1p;
                if (my_logits) my_logits[(size_t)r * L + c] = (float)logit;
                cur |= (uint64_t)spin << (c & 63);
                if ((c & 63) == 63 || c == L - 1) { my_out[(size_t)r * W + (c >> 6)] = cur; cur = 0; }
                T ln[CHI];
                T mx = 0;
#pragma unroll
                for (int b = 0; b < CHI; ++b) ln[b] = spin ? y1[b] : y0[b];
#pragma unroll
                for (int b = 0; b < CHI; ++b) mx = fmax(mx, fabs(ln[b]));
                const T sc = mx > (T)0 ? pow2_inv(mx) : (T)1;
#pragma unroll
                for (int b = 0; b < CHI; ++b) l[b] = ln[b] * sc;
                }
                // one barrier site that every thread reaches
                if (more) put(buf ^ 1);
                __syncthreads();
                buf ^= 1;
            }
        }
    }
    if (act) logq_out[(size_t)inst * n_samples + n] = logq;
}

}  // namespace tnmc

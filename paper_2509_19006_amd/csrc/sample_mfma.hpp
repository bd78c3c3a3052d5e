// Row-by-row autoregressive sampling from the boundary-MPS cache on the
// matrix cores (arXiv 2509.19006, section 3.3; chain rule Eq. (3), the
// conditional Eq. (4) and its sigmoid form Eq. (5)), for bond dimensions up
// to 32 in the float32 and mixed-precision forms.
//
// The computation is the one of sample_device.hpp, reorganised so that the
// two contractions of every site run as matrix products with the samples as
// the column dimension.  A workgroup of 256 threads owns 256 samples of one
// instance; each wave owns 64 of them as two column blocks of 32.  Per row r:
//   right sweep   R_c = sum_s [A_{c+1,s} (w_s * R_{c+1})]: a (chi x 2chi) by
//                 (2chi x 64) product per wave, w_s the vertical Boltzmann
//                 weight of the sample's upper spin at column c+1;
//   left sweep    [y_-, y_+] = [A_{c,-}^T; A_{c,+}^T] l: a (2chi x chi) by
//                 (chi x 64) product, then per sample rho_s = |y_s . R_c|,
//                 the logit, p in float64, the Philox draw, log q, and
//                 l = y_spin rescaled by a power of two.
// Products use 32 x 32 result tiles: lane l holds, for column l mod 32 of
// each block, the rows 8 (j / 4) + 4 (l / 32) + j mod 4 (j = 0 .. chi/2-1).
// The inner (summed) index of a product may be split over the lanes in any
// order, so each lane feeds the next product exactly the rows it holds: a
// sample's vector never moves between lanes, and a sample's dot products
// need one exchange between the two lanes that hold its halves.  After that
// exchange each lane carries the scalar work (float64 logit, draw, log q,
// spin bits) of one sample: lanes 0-31 of the first column block, lanes
// 32-63 of the second.
//
// Operand precision (MODE):
//   MF_F32   float32 operands, v_mfma_f32_32x32x2f32;
//   MF_BF16 / MF_F16   16-bit operands with float32 accumulation,
//            v_mfma_f32_32x32x16_{bf16,f16}.  The sample's vectors (l, R)
//            are float32 and enter as hi + lo 16-bit pairs; a 16-bit stored
//            cache enters exactly (two products), a float32 cache as its own
//            hi + lo pair (three products: hi*hi + hi*lo + lo*hi, the lo*lo
//            term is below float32 rounding of the result).
// Right environments go to a per-tile scratch in HBM as float32, in the
// lanes' own layout, and are read back by the same lanes in the left sweep.
#pragma once
#include <type_traits>

#include "device.hpp"

namespace tnmc {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

enum { MF_F32 = 0, MF_BF16 = 1, MF_F16 = 2 };

template <int MODE> struct MfElem;
template <> struct MfElem<MF_F32> { using E = float; };
template <> struct MfElem<MF_BF16> { using E = __bf16; using V8 = bf16x8; using V4 = bf16x4; };
template <> struct MfElem<MF_F16> { using E = _Float16; using V8 = f16x8; using V4 = f16x4; };

__device__ __forceinline__ f32x16 mfma16(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma16(f16x8 a, f16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// Row of the 32 x 32 tile held in result register j of a lane in half h.
__device__ __forceinline__ constexpr int held_row(int j, int h) { return 8 * (j >> 2) + 4 * h + (j & 3); }

// Whether a float32 cache is split into two 16-bit parts (three products).
template <typename S, int MODE> struct SplitA {
    static constexpr bool value = MODE != MF_F32 && std::is_same<S, float>::value;
};

// Raw 16-bit stored values reinterpreted as the matrix-core element type.
template <typename E, typename S> __device__ __forceinline__ E as_elem(S v) {
    if constexpr (std::is_same<S, float>::value) return (E)v;
    else return __builtin_bit_cast(E, v);
}

// Shared-memory bytes of the staging buffers: two sites, each holding both
// spin slices (hi and lo parts for a split float32 cache), rows padded.
template <int CHI, typename S, int MODE> __host__ __device__ constexpr int mf_row() {
    return MODE == MF_F32 ? CHI + 4 : CHI + 4;
}
template <int CHI, typename S, int MODE> __host__ __device__ constexpr size_t mf_stage_bytes() {
    using E = typename MfElem<MODE>::E;
    return (size_t)2 * (SplitA<S, MODE>::value ? 2 : 1) * 2 * CHI * mf_row<CHI, S, MODE>() * sizeof(E);
}
// ... plus the row's vertical-bond tables (two float weights and one double
// coupling term per column, up to 1024 columns)
constexpr size_t MF_ROW_TABLE_BYTES = (size_t)16 * 1024;
template <int CHI, typename S, int MODE> __host__ __device__ constexpr size_t mf_lds_bytes() {
    return mf_stage_bytes<CHI, S, MODE>() + MF_ROW_TABLE_BYTES;
}

// One tile of 256 samples of instance inst; all 256 threads call it.
// env: the tile's right-environment scratch (L * CHI * 256 floats).
// smem: at least mf_lds_bytes<CHI, S, MODE>() bytes, 16-byte aligned.
template <int CHI, typename S, int MODE>
__device__ void sample_tile_mfma(int inst, int tile, const InstDesc &d, const unsigned char *__restrict__ ws,
                                 float *__restrict__ env, int n_samples, uint64_t seed, uint64_t sample_offset,
                                 const uint64_t *__restrict__ forced, uint64_t *spins_out,
                                 double *__restrict__ logq_out, float *__restrict__ logits_out,
                                 const float *__restrict__ Jv_all, unsigned char *smem) {
    static_assert(CHI == 16 || CHI == 32, "matrix-core sampler: chi <= 32");
    using E = typename MfElem<MODE>::E;
    constexpr bool SPLIT = SplitA<S, MODE>::value;
    constexpr int JN = CHI / 2;              // held rows per lane and column block
    constexpr int RS = mf_row<CHI, S, MODE>();
    constexpr int SLICE = CHI * RS;          // one spin slice in shared memory
    constexpr int NP = SPLIT ? 2 : 1;        // parts (hi, lo) per slice
    constexpr int SITE = 2 * NP * SLICE;     // one staged site
    constexpr int PER = 2 * CHI * CHI / 256; // staged entries per thread
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, n32 = l & 31, h = l >> 5;
    // the sample whose scalar work this lane carries (column block h)
    const int my = tile * 256 + wave * 64 + h * 32 + n32;
    const bool act = my < n_samples;
    const int L = d.L, chi = d.chi, W = d.W;
    const double beta = d.beta;
    const S *cache = reinterpret_cast<const S *>(ws + d.cache_off);
    const size_t site_sz = (size_t)2 * chi * chi, row_sz = (size_t)L * site_sz;
    const float *jv = Jv_all + d.off_v;
    const size_t wbase = (size_t)n_samples * d.word_prefix + (size_t)my * L * W;
    uint64_t *my_out = spins_out + wbase;
    const uint64_t *my_forced = forced ? forced + wbase : nullptr;
    float *my_logits = logits_out ? logits_out + (size_t)n_samples * d.site_prefix + (size_t)my * L * L : nullptr;
    const uint32_t sidx = (uint32_t)(sample_offset + (uint64_t)my);
    E *stage = reinterpret_cast<E *>(smem);
    // vertical bonds from row r-1: Boltzmann weights of equal / opposite
    // spins (the right sweep's w) and 2 beta J (the left sweep's logit term)
    double *ctab = reinterpret_cast<double *>(smem + mf_stage_bytes<CHI, S, MODE>());
    float *wtab = reinterpret_cast<float *>(ctab + L);
    // this wave's slice of the scratch: [c][JN * 2 registers][64 lanes]
    float *wenv = env + (size_t)wave * 2 * JN * 64 + l;
    constexpr size_t ENV_C = (size_t)4 * 2 * JN * 64;   // floats per site of the tile

    // ---- staging, two sites ahead: the entries of site k+2 are fetched
    // into one register set while site k is contracted and site k+1 (fetched
    // a step earlier) goes from the other set into the shared buffer the
    // step before used (transposed for the left sweep, which reads the spin
    // slices by column) ----
    S pre[2][PER];
    auto fetch = [&](auto SET, const S *site) {
        constexpr int k = decltype(SET)::value;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + i * 256;
            const int s = e / (CHI * CHI), a = (e / CHI) % CHI, b = e % CHI;
            pre[k][i] = (a < chi && b < chi) ? site[(size_t)s * chi * chi + a * chi + b] : S{};
        }
    };
    auto put = [&](auto SET, int buf, bool transposed) {
        constexpr int k = decltype(SET)::value;
        E *dst = stage + buf * SITE;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + i * 256;
            const int s = e / (CHI * CHI), a = (e / CHI) % CHI, b = e % CHI;
            const int o = s * NP * SLICE + (transposed ? b * RS + a : a * RS + b);
            if constexpr (SPLIT) {
                const float v = (float)pre[k][i];
                const E hi = (E)v;
                dst[o] = hi;
                dst[o + SLICE] = (E)(v - (float)hi);
            } else {
                dst[o] = as_elem<E, S>(pre[k][i]);
            }
        }
    };
    using Set0 = std::integral_constant<int, 0>;
    using Set1 = std::integral_constant<int, 1>;

    // per-lane state: the sample vectors of both column blocks
    float vec[2][JN];
    double logq = 0.0;

    for (int r = 0; r < L; ++r) {
        const S *crow = cache + (size_t)r * row_sz;
        // ---------------- right environments (c = L-2 .. 0) ----------------
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int j = 0; j < JN; ++j) vec[nb][j] = held_row(j, h) == 0 ? 1.f : 0.f;
        uint64_t uw = 0;
        int uw_idx = -1;
        if (r > 0) {
            for (int c = tid; c < L; c += 256) {
                const float J = jv[(size_t)(r - 1) * L + c];
                double same, diff;
                boltz(beta, J, same, diff);
                wtab[2 * c] = (float)same;
                wtab[2 * c + 1] = (float)diff;
                ctab[c] = 2.0 * beta * (double)J;
            }
        }
        // step k contracts site c + 1 = L - 1 - k (c = L - 2 .. 0)
        const int mR = L - 1;
        fetch(Set0{}, crow + (size_t)(L - 1) * site_sz);
        put(Set0{}, 0, false);
        if (mR > 1) fetch(Set1{}, crow + (size_t)(L - 2) * site_sz);
        __syncthreads();
        auto rstep = [&](int k, auto FS, auto PS) {
            const int c = L - 2 - k, buf = k & 1;
            if (k + 2 < mR) fetch(FS, crow + (size_t)(c - 1) * site_sz);
            const E *Ab = stage + buf * SITE;
            // vertical weights of both column blocks' samples at column c+1
            float w[2][2];
            {
                if (r > 0) {
                    const int cc = c + 1, wi = cc >> 6;
                    int u = 0;
                    if (act) {
                        if (wi != uw_idx) { uw = my_out[(size_t)(r - 1) * W + wi]; uw_idx = wi; }
                        u = (int)((uw >> (cc & 63)) & 1);
                    }
                    const int u_other = __shfl_xor(u, 32);
                    const float same = wtab[2 * cc], diff = wtab[2 * cc + 1];
                    // own block h, the other block 1 - h
                    const int ub[2] = {h ? u_other : u, h ? u : u_other};
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb) {
                        w[0][nb] = ub[nb] == 0 ? same : diff;
                        w[1][nb] = ub[nb] == 1 ? same : diff;
                    }
                } else {
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb) { w[0][nb] = 1.f; w[1][nb] = 1.f; }
                }
            }
            f32x16 acc[2];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[nb][q] = 0.f;
            // row a of the product is this lane's column position n32
            const bool arow = CHI == 32 || n32 < CHI;
            const int ar = arow ? n32 : 0;
            if constexpr (MODE == MF_F32) {
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int g = 0; g < JN / 4; ++g) {
                        const float *src = reinterpret_cast<const float *>(Ab) + s * SLICE + ar * RS + 8 * g + 4 * h;
                        const float4 a4 = *reinterpret_cast<const float4 *>(src);
                        const float av[4] = {arow ? a4.x : 0.f, arow ? a4.y : 0.f, arow ? a4.z : 0.f, arow ? a4.w : 0.f};
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int nb = 0; nb < 2; ++nb)
                                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], w[s][nb] * vec[nb][4 * g + i],
                                                                                 acc[nb], 0, 0, 0);
                    }
            } else {
                using V8 = typename MfElem<MODE>::V8;
                using V4 = typename MfElem<MODE>::V4;
#pragma unroll
                for (int t = 0; t < CHI / 8; ++t) {
                    const int s = (8 * t) / JN, j0 = (8 * t) % JN, g0 = j0 >> 2;
                    V8 ah, al;
#pragma unroll
                    for (int part = 0; part < NP; ++part) {
                        const E *src = Ab + s * NP * SLICE + part * SLICE + ar * RS + 4 * h;
                        const V4 x0 = *reinterpret_cast<const V4 *>(src + 8 * g0);
                        const V4 x1 = *reinterpret_cast<const V4 *>(src + 8 * g0 + 8);
                        V8 v;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            v[q] = arow ? x0[q] : (E)0.f;
                            v[q + 4] = arow ? x1[q] : (E)0.f;
                        }
                        if (part == 0) ah = v; else al = v;
                    }
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb) {
                        V8 bh, bl;
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const float x = w[s][nb] * vec[nb][j0 + q];
                            bh[q] = (E)x;
                            bl[q] = (E)(x - (float)bh[q]);
                        }
                        if constexpr (SPLIT) acc[nb] = mfma16(al, bh, acc[nb]);
                        acc[nb] = mfma16(ah, bl, acc[nb]);
                        acc[nb] = mfma16(ah, bh, acc[nb]);
                    }
                }
            }
            // rescale each sample's environment by a power of two and keep it
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                float mx = 0.f;
#pragma unroll
                for (int j = 0; j < JN; ++j) mx = fmaxf(mx, fabsf(acc[nb][j]));
                mx = fmaxf(mx, __shfl_xor(mx, 32));
                const float sc = mx > 0.f ? pow2_inv(mx) : 1.f;
                float *ec = wenv + (size_t)c * ENV_C + (size_t)nb * JN * 64;
#pragma unroll
                for (int j = 0; j < JN; ++j) {
                    vec[nb][j] = acc[nb][j] * sc;
                    ec[(size_t)j * 64] = vec[nb][j];
                }
            }
            if (k + 1 < mR) put(PS, buf ^ 1, false);
            __syncthreads();
        };
        for (int k = 0; k < mR; k += 2) {
            rstep(k, Set0{}, Set1{});
            if (k + 1 < mR) rstep(k + 1, Set1{}, Set0{});
        }
        // ---------------- left sweep: sample row r ----------------
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int j = 0; j < JN; ++j) vec[nb][j] = held_row(j, h) == 0 ? 1.f : 0.f;
        uint64_t cur = 0, up = 0, fw = 0;
        // right environments, one site ahead, through two register sets
        float renvs[2][2][JN];
        auto load_env = [&](auto SET, int c) {
            constexpr int k = decltype(SET)::value;
            if (c < L - 1) {
                const float *ec = wenv + (size_t)c * ENV_C;
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                    for (int j = 0; j < JN; ++j) renvs[k][nb][j] = ec[(size_t)(nb * JN + j) * 64];
            } else {
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                    for (int j = 0; j < JN; ++j) renvs[k][nb][j] = held_row(j, h) == 0 ? 1.f : 0.f;
            }
        };
        fetch(Set0{}, crow);
        put(Set0{}, 0, true);
        if (L > 1) fetch(Set1{}, crow + site_sz);
        load_env(Set0{}, 0);
        __syncthreads();
        auto lstep = [&](int c, auto FS, auto PS) {
            const int buf = c & 1;
            if (c + 2 < L) fetch(FS, crow + (size_t)(c + 2) * site_sz);
            // the draw's uniform does not depend on the contraction: take it
            // first, so that its latency hides behind the products
            double u_draw = 0.0;
            if (!my_forced) u_draw = philox_unit(seed, (uint32_t)(r * L + c), sidx, (uint32_t)inst, 0u);
            const E *Ab = stage + buf * SITE;
            // the site's right environment (loaded a step earlier, in this
            // lane's layout); the next site's is fetched now
            constexpr int KE = decltype(FS)::value;
            const float (&renv)[2][JN] = renvs[KE];
            if (c + 1 < L) load_env(PS, c + 1);
            // y[s] for both column blocks: MB result tiles of 32 rows
            constexpr int MB = CHI == 32 ? 2 : 1;
            f32x16 acc[MB][2];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                    for (int q = 0; q < 16; ++q) acc[mb][nb][q] = 0.f;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                // row m = n32 of tile mb is (spin s, column b) of the site
                const int s = CHI == 32 ? mb : (n32 >> 4);
                const int b = CHI == 32 ? n32 : (n32 & 15);
                if constexpr (MODE == MF_F32) {
#pragma unroll
                    for (int g = 0; g < JN / 4; ++g) {
                        const float *src = reinterpret_cast<const float *>(Ab) + s * SLICE + b * RS + 8 * g + 4 * h;
                        const float4 a4 = *reinterpret_cast<const float4 *>(src);
                        const float av[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int nb = 0; nb < 2; ++nb)
                                acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], vec[nb][4 * g + i],
                                                                                     acc[mb][nb], 0, 0, 0);
                    }
                } else {
                    using V8 = typename MfElem<MODE>::V8;
                    using V4 = typename MfElem<MODE>::V4;
#pragma unroll
                    for (int t = 0; t < JN / 8; ++t) {
                        V8 ah, al;
#pragma unroll
                        for (int part = 0; part < NP; ++part) {
                            const E *src = Ab + s * NP * SLICE + part * SLICE + b * RS + 16 * t + 4 * h;
                            const V4 x0 = *reinterpret_cast<const V4 *>(src);
                            const V4 x1 = *reinterpret_cast<const V4 *>(src + 8);
                            V8 v;
#pragma unroll
                            for (int q = 0; q < 4; ++q) { v[q] = x0[q]; v[q + 4] = x1[q]; }
                            if (part == 0) ah = v; else al = v;
                        }
#pragma unroll
                        for (int nb = 0; nb < 2; ++nb) {
                            V8 bh, bl;
#pragma unroll
                            for (int q = 0; q < 8; ++q) {
                                const float x = vec[nb][8 * t + q];
                                bh[q] = (E)x;
                                bl[q] = (E)(x - (float)bh[q]);
                            }
                            if constexpr (SPLIT) acc[mb][nb] = mfma16(al, bh, acc[mb][nb]);
                            acc[mb][nb] = mfma16(ah, bl, acc[mb][nb]);
                            acc[mb][nb] = mfma16(ah, bh, acc[mb][nb]);
                        }
                    }
                }
            }
            auto yv = [&](int s, int nb, int j) -> float {
                if constexpr (CHI == 32) return acc[s][nb][j];
                else return acc[0][nb][8 * s + j];
            };
            // rho_s = y_s . R_c: this lane's half of both blocks, then the
            // other half of its own block from the partner lane
            float part[2][2];
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb) {
                    float a0 = 0.f, a1 = 0.f;
#pragma unroll
                    for (int j = 0; j < JN; j += 2) {
                        a0 = fmaf(yv(s, nb, j), renv[nb][j], a0);
                        a1 = fmaf(yv(s, nb, j + 1), renv[nb][j + 1], a1);
                    }
                    part[s][nb] = a0 + a1;
                }
            const float mine0 = h ? part[0][1] : part[0][0], other0 = h ? part[0][0] : part[0][1];
            const float mine1 = h ? part[1][1] : part[1][0], other1 = h ? part[1][0] : part[1][1];
            const float r0 = mine0 + __shfl_xor(other0, 32);
            const float r1 = mine1 + __shfl_xor(other1, 32);
            const float rho0 = fabsf(r0), rho1 = fabsf(r1);
            double logit = 0.0;
            if ((c & 63) == 0 && act) {
                if (r > 0) up = my_out[(size_t)(r - 1) * W + (c >> 6)];
                if (my_forced) fw = my_forced[(size_t)r * W + (c >> 6)];
            }
            if (rho0 > 0.f || rho1 > 0.f) {
                // the float32 ratio's logarithm in float32 (the products are
                // float32); the conditional p is formed from it in float64
                logit = (double)(logf(rho1) - logf(rho0));
                if (r > 0) {
                    const double u = (double)((up >> (c & 63)) & 1);
                    logit += ctab[c] * (2.0 * u - 1.0);
                }
            }
            const double ex = exp(-fabs(logit));
            const double l1p = log1p(ex);
            int spin;
            if (my_forced) {
                spin = (int)((fw >> (c & 63)) & 1);
            } else {
                const double p = (logit >= 0.0 ? 1.0 : ex) / (1.0 + ex);
                spin = (u_draw < p) ? 1 : 0;
            }
            if (!act) spin = 0;
            logq += (spin ? fmin(logit, 0.0) : fmin(-logit, 0.0)) - l1p;
            if (act) {
                if (my_logits) my_logits[(size_t)r * L + c] = (float)logit;
                cur |= (uint64_t)spin << (c & 63);
                if ((c & 63) == 63 || c == L - 1) { my_out[(size_t)r * W + (c >> 6)] = cur; cur = 0; }
            }
            const int spin_other = __shfl_xor(spin, 32);
            const int sp[2] = {h ? spin_other : spin, h ? spin : spin_other};
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                float mx = 0.f;
#pragma unroll
                for (int j = 0; j < JN; ++j) mx = fmaxf(mx, fabsf(sp[nb] ? yv(1, nb, j) : yv(0, nb, j)));
                mx = fmaxf(mx, __shfl_xor(mx, 32));
                const float sc = mx > 0.f ? pow2_inv(mx) : 1.f;
#pragma unroll
                for (int j = 0; j < JN; ++j) vec[nb][j] = (sp[nb] ? yv(1, nb, j) : yv(0, nb, j)) * sc;
            }
            if (c + 1 < L) put(PS, buf ^ 1, true);
            __syncthreads();
        };
        for (int c = 0; c < L; c += 2) {
            lstep(c, Set0{}, Set1{});
            if (c + 1 < L) lstep(c + 1, Set1{}, Set0{});
        }
    }
    if (act) logq_out[(size_t)inst * n_samples + my] = logq;
}

}  // namespace tnmc

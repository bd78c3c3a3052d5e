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
//
// Learned correction (MLP = true; chi <= 16, float32): after the TN logit
// of a site, the network of mlp_device.hpp runs for the wave's 64 samples
// as two bf16 products per layer with the samples as the column dimension
// (mlp_site_mfma below), and its output is added to the logit before the
// draw.
#pragma once
#include <type_traits>

#include "device.hpp"
#include "mlp_device.hpp"

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
__host__ __device__ constexpr int held_row(int j, int h) { return 8 * (j >> 2) + 4 * h + (j & 3); }

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

// ---- the learned correction on the matrix cores ----
// Weights in shared memory: W1 [o][k] and W2 [o][slot] as bfloat16 rows of
// MLPW_RS (64 + padding), then b1, b2, W3 and b3 as float32; every value
// rounded to bfloat16, the rounding every inference of the correction uses.
constexpr int MLPW_RS = 72;
constexpr size_t MF_MLP_W_BYTES = (size_t)64 * MLPW_RS * 2;
constexpr size_t MF_MLP_BYTES = 2 * MF_MLP_W_BYTES + (size_t)(3 * 64 + 4) * 4;

template <int CHI, typename S, int MODE, bool MLP = false> __host__ __device__ constexpr size_t mf_lds_bytes() {
    return mf_stage_bytes<CHI, S, MODE>() + MF_ROW_TABLE_BYTES + (MLP ? MF_MLP_BYTES : 0);
}

// Second layer: slot q of lane half h in the 16-wide chunk t of the summed
// index carries hidden unit mlp_l2_unit(t, h, q), a unit that lane already
// holds in its first-layer result tiles; W2's columns are staged in that
// order.
__host__ __device__ constexpr int mlp_l2_unit(int t, int h, int q) { return 32 * (t >> 1) + held_row(8 * (t & 1) + q, h); }

// tanh x = 1 - 2 / (e^{2x} + 1), the exponential taken in base 2 on the
// transcendental unit; it saturates to -1 / +1 for large |x|.
__device__ __forceinline__ float tanh_mc(float x) {
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);   // 2 log2(e)
    return 1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f);
}

// Stage the parameter vector P (layout of mlp_device.hpp) into dst; all
// threads of the workgroup take part, a barrier must follow.
__device__ __forceinline__ void mlp_stage(const float *__restrict__ P, unsigned char *dst, int tid, int nthr) {
    __bf16 *w1 = reinterpret_cast<__bf16 *>(dst);
    __bf16 *w2 = reinterpret_cast<__bf16 *>(dst + MF_MLP_W_BYTES);
    float *bv = reinterpret_cast<float *>(dst + 2 * MF_MLP_W_BYTES);
    for (int e = tid; e < MLP_H * MLP_IN; e += nthr) {
        const int o = e >> 6, k = e & 63;
        w1[o * MLPW_RS + k] = (__bf16)P[MLP_OFF_W1 + o * MLP_IN + k];
        w2[o * MLPW_RS + k] = (__bf16)P[MLP_OFF_W2 + o * MLP_H + mlp_l2_unit(k >> 4, (k >> 3) & 1, k & 7)];
    }
    for (int e = tid; e < 3 * MLP_H + 1; e += nthr) {
        const int src = e < 64 ? MLP_OFF_B1 + e : e < 128 ? MLP_OFF_B2 + e - 64 : e < 192 ? MLP_OFF_W3 + e - 128
                                                                                         : MLP_OFF_B3;
        bv[e] = (float)(__bf16)P[src];
    }
}

// The correction d of the sample whose scalar work this lane carries
// (column n32 of block h), for all 64 samples of the wave at once.
//   xc     the site's 40 coupling features (the same for every sample);
//   sb[nb] spin-feature bits of the sample in column n32 of block nb (bit i
//          is feature 40 + i: +1 if set, -1 if clear), vm which of those 12
//          positions lie inside the lattice (feature 0 outside);
//   xl[nb] that sample's clipped, scaled TN logit (feature 52).
// Layer 1 takes the features in their natural order (half h of a lane pair
// supplies inputs 16t + 8h .. 16t + 8h + 7 of chunk t), layer 2 the hidden
// units each lane holds after layer 1; activations enter as hi + lo bf16
// pairs, accumulation is float32.  Both lanes of a pair hold half of every
// hidden vector of both blocks: d needs one exchange, as rho does.
__device__ __forceinline__ float mlp_site_mfma(const unsigned char *wsm, const float (&xc)[40], const uint32_t (&sb)[2],
                                               uint32_t vm, const float (&xl)[2], int n32, int h) {
    const __bf16 *w1 = reinterpret_cast<const __bf16 *>(wsm);
    const __bf16 *w2 = reinterpret_cast<const __bf16 *>(wsm + MF_MLP_W_BYTES);
    const float *bv = reinterpret_cast<const float *>(wsm + 2 * MF_MLP_W_BYTES);
    auto feat = [&](int k, int nb) -> float {
        if (k < 40) return xc[k];
        if (k < 52) return ((vm >> (k - 40)) & 1u) ? (((sb[nb] >> (k - 40)) & 1u) ? 1.f : -1.f) : 0.f;
        return k == 52 ? xl[nb] : 0.f;
    };
    f32x16 a1[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int q = 0; q < 16; ++q) a1[mt][nb][q] = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        bf16x8 A[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) A[mt] = *reinterpret_cast<const bf16x8 *>(w1 + (32 * mt + n32) * MLPW_RS + 16 * t + 8 * h);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            bf16x8 bh, bl;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float v = h ? feat(16 * t + 8 + q, nb) : feat(16 * t + q, nb);
                bh[q] = (__bf16)v;
                bl[q] = (__bf16)(v - (float)bh[q]);
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                a1[mt][nb] = mfma16(A[mt], bl, a1[mt][nb]);
                a1[mt][nb] = mfma16(A[mt], bh, a1[mt][nb]);
            }
        }
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const float4 b = *reinterpret_cast<const float4 *>(bv + 32 * mt + 8 * g + 4 * h);
            const float bb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int i = 0; i < 4; ++i) a1[mt][nb][4 * g + i] = tanh_mc(a1[mt][nb][4 * g + i] + bb[i]);
        }
    f32x16 a2[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int q = 0; q < 16; ++q) a2[mt][nb][q] = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        bf16x8 A[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) A[mt] = *reinterpret_cast<const bf16x8 *>(w2 + (32 * mt + n32) * MLPW_RS + 16 * t + 8 * h);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            bf16x8 bh, bl;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float v = a1[t >> 1][nb][8 * (t & 1) + q];
                bh[q] = (__bf16)v;
                bl[q] = (__bf16)(v - (float)bh[q]);
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                a2[mt][nb] = mfma16(A[mt], bl, a2[mt][nb]);
                a2[mt][nb] = mfma16(A[mt], bh, a2[mt][nb]);
            }
        }
    }
    float part[2] = {0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const float4 b = *reinterpret_cast<const float4 *>(bv + 64 + 32 * mt + 8 * g + 4 * h);
            const float4 w = *reinterpret_cast<const float4 *>(bv + 128 + 32 * mt + 8 * g + 4 * h);
            const float bb[4] = {b.x, b.y, b.z, b.w}, ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int i = 0; i < 4; ++i) part[nb] = fmaf(ww[i], tanh_mc(a2[mt][nb][4 * g + i] + bb[i]), part[nb]);
        }
    const float mine = h ? part[1] : part[0], other = h ? part[0] : part[1];
    return (mine + __shfl_xor(other, 32)) + bv[192];
}

// One tile of 256 samples of instance inst; all 256 threads call it.
// env: the tile's right-environment scratch (L * CHI * 256 floats).
// smem: at least mf_lds_bytes<CHI, S, MODE, MLP>() bytes, 16-byte aligned.
// mlp: the network and the horizontal couplings (MLP only).
template <int CHI, typename S, int MODE, bool MLP = false>
__device__ void sample_tile_mfma(int inst, int tile, const InstDesc &d, const unsigned char *__restrict__ ws,
                                 float *__restrict__ env, int n_samples, uint64_t seed, uint64_t sample_offset,
                                 const uint64_t *__restrict__ forced, uint64_t *spins_out,
                                 double *__restrict__ logq_out, float *__restrict__ logits_out,
                                 const float *__restrict__ Jv_all, unsigned char *smem,
                                 MlpArgs mlp = MlpArgs{nullptr, nullptr}) {
    static_assert(CHI == 16 || CHI == 32, "matrix-core sampler: chi <= 32");
    static_assert(!MLP || (CHI == 16 && MODE == MF_F32), "learned correction: chi <= 16, float32");
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
    // the network's weights (staged here; the first barrier of row 0
    // precedes their first use)
    unsigned char *mlp_sm = smem + mf_lds_bytes<CHI, S, MODE>();
    const float *jh = MLP ? mlp.Jh + d.off_h : nullptr;
    if constexpr (MLP) mlp_stage(mlp.params, mlp_sm, tid, 256);

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
        uint64_t cur = 0, up = 0, fw = 0, prevw = 0;
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
            // the network's inputs that are already fixed: the site's
            // couplings and the sample's spins of rows r-2, r-1 (bits 0-9 of
            // the spin features; vm marks the positions inside the lattice)
            float xc[40];
            uint32_t sb_up = 0, vm = 0;
            if constexpr (MLP) {
#pragma unroll
                for (int dr = -2; dr <= 2; ++dr)
#pragma unroll
                    for (int dc = -2; dc <= 1; ++dc) {
                        const int rr = r + dr, cc = c + dc;
                        xc[(dr + 2) * 4 + dc + 2] =
                            (rr >= 0 && rr < L && cc >= 0 && cc < L - 1) ? jh[(size_t)rr * (L - 1) + cc] : 0.f;
                    }
#pragma unroll
                for (int dr = -2; dr <= 1; ++dr)
#pragma unroll
                    for (int dc = -2; dc <= 2; ++dc) {
                        const int rr = r + dr, cc = c + dc;
                        xc[20 + (dr + 2) * 5 + dc + 2] =
                            (rr >= 0 && rr < L - 1 && cc >= 0 && cc < L) ? jv[(size_t)rr * L + cc] : 0.f;
                    }
                const int wl = (c >= 2 ? c - 2 : 0) >> 6, wh = (c + 2 < L ? c + 2 : L - 1) >> 6;
#pragma unroll
                for (int dr = -2; dr <= -1; ++dr) {
                    const int rr = r + dr;
                    if (rr < 0) continue;
                    uint64_t wa = 0, wb = 0;
                    if (act) { wa = my_out[(size_t)rr * W + wl]; wb = my_out[(size_t)rr * W + wh]; }
#pragma unroll
                    for (int i = 0; i < 5; ++i) {
                        const int cc = c - 2 + i, bit = (dr + 2) * 5 + i;
                        if (cc < 0 || cc >= L) continue;
                        const uint64_t w = (cc >> 6) == wl ? wa : wb;
                        sb_up |= (uint32_t)((w >> (cc & 63)) & 1) << bit;
                        vm |= 1u << bit;
                    }
                }
                if (c >= 2) vm |= 1u << 10;
                if (c >= 1) vm |= 1u << 11;
            }
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
            if constexpr (MLP) {
                // row r's spins at c-2, c-1: in the word being assembled or
                // in the one flushed last
                uint32_t sb = sb_up;
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const int cc = c - 2 + i;
                    if (cc < 0) continue;
                    const uint64_t w = (cc >> 6) == (c >> 6) ? cur : prevw;
                    sb |= (uint32_t)((w >> (cc & 63)) & 1) << (10 + i);
                }
                const float xlm = fminf(fmaxf((float)logit, -30.f), 30.f) * 0.125f;
                const uint32_t sbo = (uint32_t)__shfl_xor((int)sb, 32);
                const float xlo = __shfl_xor(xlm, 32);
                const uint32_t sbb[2] = {h ? sbo : sb, h ? sb : sbo};
                const float xlb[2] = {h ? xlo : xlm, h ? xlm : xlo};
                logit += (double)mlp_site_mfma(mlp_sm, xc, sbb, vm, xlb, n32, h);
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
                if ((c & 63) == 63 || c == L - 1) { my_out[(size_t)r * W + (c >> 6)] = cur; prevw = cur; cur = 0; }
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

// The whole hot path per instance in one persistent launch, for uneven
// batches: each workgroup takes the next instance in the host's
// longest-first order and runs its cache build (section 3.2), its sample
// tiles one after another (section 3.3), the energies of its samples
// (Eq. (1)) and its Metropolis chain (Eq. (10)).  An instance is complete
// when its workgroup ends; nothing waits for the slowest instance of the
// batch.  The arithmetic is the stand-alone kernels' (the same device
// functions), so results equal the separate calls bit for bit.
#include "build_pipe.hpp"
#include "energy_accept_device.hpp"
#include "sample_device.hpp"
#include "sample_mfma.hpp"

namespace tnmc {

static_assert(NT == NTS, "the fused pipeline runs the sampler with the build's workgroup");

// Matrix-core form of a precision (as in sample.hip).
template <typename S, bool SPLIT16> struct PipeMode;
template <> struct PipeMode<float, false> { static constexpr int v = MF_F32; };
template <> struct PipeMode<float, true> { static constexpr int v = MF_BF16; };
template <> struct PipeMode<__hip_bfloat16, false> { static constexpr int v = MF_BF16; };
template <> struct PipeMode<__half, false> { static constexpr int v = MF_F16; };
template <> struct PipeMode<double, false> { static constexpr int v = MF_F32; };

template <typename T, typename S, int MAXB, bool SPLIT16, bool PIPE>
__global__ void __launch_bounds__(NT)
k_pipeline(const InstDesc *__restrict__ desc, const int32_t *__restrict__ order, unsigned char *__restrict__ ws,
           const float *__restrict__ Jh_all, const float *__restrict__ Jv_all, double *__restrict__ logz_out,
           int64_t *__restrict__ stats, int n_samples, uint64_t sample_seed, uint64_t sample_offset,
           uint64_t *spins_out, double *__restrict__ logq_out, double *__restrict__ E_out,
           Chain *__restrict__ chain, uint64_t accept_seed, uint64_t step_offset, uint8_t *__restrict__ acc_out,
           int64_t *__restrict__ state_out) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int inst = order[blockIdx.x];
    build_instance_sel<T, S, MAXB, PIPE>(inst, desc, ws, Jh_all, Jv_all, logz_out, stats, smem);
    __threadfence();
    __syncthreads();

    const InstDesc d = desc[inst];
    T *env = reinterpret_cast<T *>(ws + d.env_off);   // one tile's scratch, reused tile after tile
    const int ntiles = (n_samples + NTS - 1) / NTS;
    for (int tile = 0; tile < ntiles; ++tile) {
        // the sampler form tnmc_sample uses for this instance: float forms
        // with chi <= 32 on the matrix cores, the rest on the vector unit
        if constexpr (std::is_same<T, float>::value) {
            constexpr int MODE = PipeMode<S, SPLIT16>::v;
            float *fenv = reinterpret_cast<float *>(env);
            if (d.chi <= 16)
                sample_tile_mfma<16, S, MODE>(inst, tile, d, ws, fenv, n_samples, sample_seed, sample_offset,
                                              nullptr, spins_out, logq_out, nullptr, Jv_all, smem);
            else if (d.chi <= 32)
                sample_tile_mfma<32, S, MODE>(inst, tile, d, ws, fenv, n_samples, sample_seed, sample_offset,
                                              nullptr, spins_out, logq_out, nullptr, Jv_all, smem);
            else if constexpr (MAXB >= 64)
                sample_tile<T, S, 64>(inst, tile, d, ws, env, n_samples, sample_seed, sample_offset,
                                             nullptr, spins_out, logq_out, nullptr, Jv_all,
                                             reinterpret_cast<typename StageType<T, S>::type(*)[64][64]>(smem));
        } else if (d.chi <= 16) {
            sample_tile<T, S, 16>(inst, tile, d, ws, env, n_samples, sample_seed, sample_offset, nullptr,
                                         spins_out, logq_out, nullptr, Jv_all,
                                         reinterpret_cast<typename StageType<T, S>::type(*)[16][16]>(smem));
        } else {
            sample_tile<T, S, 32>(inst, tile, d, ws, env, n_samples, sample_seed, sample_offset, nullptr,
                                         spins_out, logq_out, nullptr, Jv_all,
                                         reinterpret_cast<typename StageType<T, S>::type(*)[32][32]>(smem));
        }
        __syncthreads();
    }
    __threadfence();
    __syncthreads();

    // energies: one wave per configuration
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int n = wv; n < n_samples; n += NT / 64) {
        const uint64_t *s = spins_out + (size_t)n_samples * d.word_prefix + (size_t)n * d.L * d.W;
        const double e = energy_wave(d, s, Jh_all, Jv_all, lane);
        if (lane == 0) E_out[(size_t)inst * n_samples + n] = e;
    }
    __threadfence();
    __syncthreads();

    if (threadIdx.x == 0) {
        const size_t o = (size_t)inst * n_samples;
        accept_chain(inst, n_samples, logq_out + o, E_out + o, d.beta, chain + inst, accept_seed, step_offset,
                     acc_out + o, state_out ? state_out + o : nullptr);
        // completion tick of the instance
        if (stats) stats[STATS_PER_INST * inst + 6] = wall_clock64();
    }
}

template <typename T, typename S, int MAXB, bool SPLIT16, bool PIPE>
hipError_t launch_pipeline_w(const InstDesc *desc, const int32_t *order, unsigned char *ws, const float *Jh,
                             const float *Jv, double *logz, int64_t *stats, int B, size_t lds_bytes,
                             int n_samples, uint64_t sseed, uint64_t soff, uint64_t *spins, double *logq, double *E,
                             void *chain, uint64_t aseed, uint64_t aoff, uint8_t *acc, int64_t *state,
                             hipStream_t st) {
    auto kern = k_pipeline<T, S, MAXB, SPLIT16, PIPE>;
    // room for the matrix-core sampler's staging as well
    constexpr size_t stage = mf_lds_bytes<32, S, PipeMode<S, SPLIT16>::v>();
    if (lds_bytes < stage) lds_bytes = stage;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(B), dim3(NT), lds_bytes, st, desc, order, ws, Jh, Jv, logz, stats, n_samples,
                       sseed, soff, spins, logq, E, reinterpret_cast<Chain *>(chain), aseed, aoff, acc, state);
    return hipGetLastError();
}

template <typename T, typename S, bool SPLIT16>
hipError_t launch_pipeline(const InstDesc *desc, const int32_t *order, unsigned char *ws, const float *Jh,
                           const float *Jv, double *logz, int64_t *stats, int B, int chi_max, bool pipe,
                           size_t lds_bytes, int n_samples, uint64_t sseed, uint64_t soff, uint64_t *spins,
                           double *logq, double *E, void *chain, uint64_t aseed, uint64_t aoff, uint8_t *acc,
                           int64_t *state, hipStream_t st) {
    if constexpr (sizeof(T) == 8) {
        if (chi_max > 32 || pipe) return hipErrorInvalidValue;
        return launch_pipeline_w<T, S, 32, SPLIT16, false>(desc, order, ws, Jh, Jv, logz, stats, B, lds_bytes,
                                                           n_samples, sseed, soff, spins, logq, E, chain, aseed,
                                                           aoff, acc, state, st);
    } else {
        if (pipe) {
            if (chi_max > 32) return hipErrorInvalidValue;
            return launch_pipeline_w<T, S, 32, SPLIT16, true>(desc, order, ws, Jh, Jv, logz, stats, B, lds_bytes,
                                                              n_samples, sseed, soff, spins, logq, E, chain, aseed,
                                                              aoff, acc, state, st);
        }
        if (chi_max <= 32)
            return launch_pipeline_w<T, S, 32, SPLIT16, false>(desc, order, ws, Jh, Jv, logz, stats, B, lds_bytes,
                                                               n_samples, sseed, soff, spins, logq, E, chain, aseed,
                                                               aoff, acc, state, st);
        return launch_pipeline_w<T, S, 64, SPLIT16, false>(desc, order, ws, Jh, Jv, logz, stats, B, lds_bytes,
                                                           n_samples, sseed, soff, spins, logq, E, chain, aseed, aoff,
                                                           acc, state, st);
    }
}

#define TNMC_LP(T, S, SP)                                                                                     \
    template hipError_t launch_pipeline<T, S, SP>(const InstDesc *, const int32_t *, unsigned char *,            \
                                                  const float *, const float *, double *, int64_t *, int, int,   \
                                                  bool, size_t, int, uint64_t, uint64_t, uint64_t *, double *, double *, \
                                                  void *, uint64_t, uint64_t, uint8_t *, int64_t *, hipStream_t);
TNMC_LP(double, double, false)
TNMC_LP(float, float, false)
TNMC_LP(float, float, true)
TNMC_LP(float, __hip_bfloat16, false)
TNMC_LP(float, __half, false)
#undef TNMC_LP

}  // namespace tnmc

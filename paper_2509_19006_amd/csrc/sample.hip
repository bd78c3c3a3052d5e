// Sampling kernels: grid (sample tile, instance).  Float32 and mixed-
// precision caches with chi <= 32 sample on the matrix cores
// (sample_mfma.hpp), with the learned correction when one is given (chi <=
// 16, float32); float64 and chi up to 64 run the vector-unit form
// (sample_device.hpp).
#include "sample_device.hpp"
#include "sample_mfma.hpp"

namespace tnmc {

template <int CHI, typename S, int MODE, bool MLP>
__global__ void __launch_bounds__(256)
k_sample_mfma(const InstDesc *__restrict__ desc, unsigned char *__restrict__ ws, size_t tile_bytes,
              int n_samples, uint64_t seed, uint64_t sample_offset, const uint64_t *__restrict__ forced,
              uint64_t *spins_out, double *__restrict__ logq_out, float *__restrict__ logits_out,
              const float *__restrict__ Jv_all, MlpArgs mlp, int64_t *__restrict__ stats, int chi_lo) {
    const int inst = blockIdx.y, tile = blockIdx.x;
    if (tile * 256 >= n_samples) return;
    const InstDesc d = desc[inst];
    // this launch takes the instances with chi_lo < chi <= CHI
    if (d.chi <= chi_lo || d.chi > CHI) return;
    __shared__ __align__(16) unsigned char stage[mf_lds_bytes<CHI, S, MODE, MLP>()];
    float *env = reinterpret_cast<float *>(ws + d.env_off + (size_t)tile * tile_bytes);
    sample_tile_mfma<CHI, S, MODE, MLP>(inst, tile, d, ws, env, n_samples, seed, sample_offset, forced, spins_out,
                                        logq_out, logits_out, Jv_all, stage, mlp);
    if (stats && tile == 0 && threadIdx.x == 0) stats[STATS_PER_INST * inst + 6] = wall_clock64();
}

template <int CHI, typename S, int MODE, bool MLP = false>
hipError_t launch_sample_mfma_t(const InstDesc *desc, unsigned char *ws, size_t tile_bytes, int B, int max_tiles,
                                int n_samples, uint64_t seed, uint64_t off, const uint64_t *forced, uint64_t *spins,
                                double *logq, float *logits, const float *Jv, int64_t *stats, int chi_lo,
                                hipStream_t st, MlpArgs mlp = MlpArgs{nullptr, nullptr}) {
    hipLaunchKernelGGL((k_sample_mfma<CHI, S, MODE, MLP>), dim3(max_tiles, B), dim3(256), 0, st, desc, ws,
                       tile_bytes, n_samples, seed, off, forced, spins, logq, logits, Jv, mlp, stats, chi_lo);
    return hipGetLastError();
}

// Matrix-core form of a precision: the cache's storage type and the
// operand type of the products.
template <typename S, bool SPLIT16> struct MfMode;
template <> struct MfMode<float, false> { static constexpr int v = MF_F32; };
template <> struct MfMode<float, true> { static constexpr int v = MF_BF16; };
template <> struct MfMode<__hip_bfloat16, false> { static constexpr int v = MF_BF16; };
template <> struct MfMode<__half, false> { static constexpr int v = MF_F16; };

template <typename T, typename S, int CHI>
__global__ void __launch_bounds__(NTS)
k_sample(const InstDesc *__restrict__ desc, unsigned char *__restrict__ ws, size_t tile_bytes,
         int n_samples, uint64_t seed, uint64_t sample_offset,
         const uint64_t *__restrict__ forced, uint64_t *spins_out,
         double *__restrict__ logq_out, float *__restrict__ logits_out,
         const float *__restrict__ Jv_all, int64_t *__restrict__ stats, int chi_lo) {
    const int inst = blockIdx.y, tile = blockIdx.x;
    if (tile * NTS >= n_samples) return;
    const InstDesc d = desc[inst];
    if (d.chi <= chi_lo) return;   // taken by a matrix-core launch
    __shared__ typename StageType<T, S>::type As[4][CHI][CHI];   // two staging buffers of both spin slices
    T *env = reinterpret_cast<T *>(ws + d.env_off + (size_t)tile * tile_bytes);
    sample_tile<T, S, CHI>(inst, tile, d, ws, env, n_samples, seed, sample_offset, forced, spins_out, logq_out,
                           logits_out, Jv_all, As);
    // end tick of the instance's first sample tile (the only tile when
    // n_samples <= 256), for per-instance completion times
    if (stats && tile == 0 && threadIdx.x == 0) stats[STATS_PER_INST * inst + 6] = wall_clock64();
}

template <typename T, typename S, int CHI>
hipError_t launch_sample_t(const InstDesc *desc, unsigned char *ws, size_t tile_bytes, int B,
                           int max_tiles, int n_samples, uint64_t seed, uint64_t off,
                           const uint64_t *forced, uint64_t *spins, double *logq, float *logits,
                           const float *Jv, int64_t *stats, hipStream_t st, int chi_lo = 0) {
    hipLaunchKernelGGL((k_sample<T, S, CHI>), dim3(max_tiles, B), dim3(NTS), 0, st, desc, ws,
                       tile_bytes, n_samples, seed, off, forced, spins, logq, logits, Jv, stats, chi_lo);
    return hipGetLastError();
}

// chi_mask: bit 0 / 1 / 2 set when the batch has instances with chi <= 16,
// 16 < chi <= 32, chi > 32.  Float forms sample each class with its own
// kernel (chi <= 32 on the matrix cores, wider on the vector unit), so an
// instance is sampled the same way whatever else is in its batch -- as in
// the fused pipeline.  Float64 and the learned correction take one
// vector-unit launch at the batch's widest bond dimension.
template <typename T, typename S, bool SPLIT16>
hipError_t launch_sample(int chi_bucket, int chi_mask, const InstDesc *desc, unsigned char *ws, size_t tile_bytes,
                         int B, int max_tiles, int n_samples, uint64_t seed, uint64_t off,
                         const uint64_t *forced, uint64_t *spins, double *logq, float *logits,
                         const float *Jv, MlpArgs mlp, int64_t *stats, hipStream_t st) {
    if constexpr (std::is_same<T, float>::value) {
        if (!mlp.params) {
            constexpr int MODE = MfMode<S, SPLIT16>::v;
            hipError_t e = hipSuccess;
            if (chi_mask & 1)
                e = launch_sample_mfma_t<16, S, MODE>(desc, ws, tile_bytes, B, max_tiles, n_samples, seed, off,
                                                      forced, spins, logq, logits, Jv, stats, 0, st);
            if (e == hipSuccess && (chi_mask & 2))
                e = launch_sample_mfma_t<32, S, MODE>(desc, ws, tile_bytes, B, max_tiles, n_samples, seed, off,
                                                      forced, spins, logq, logits, Jv, stats, 16, st);
            if (e == hipSuccess && (chi_mask & 4))
                e = launch_sample_t<T, S, 64>(desc, ws, tile_bytes, B, max_tiles, n_samples, seed, off, forced,
                                              spins, logq, logits, Jv, stats, st, 32);
            return e;
        }
    }
    if (SPLIT16) return hipErrorInvalidValue;
    if (mlp.params) {
        // the learned correction runs in float32 with chi <= 16, on the
        // matrix cores
        if constexpr (std::is_same<T, float>::value && std::is_same<S, float>::value) {
            if (chi_bucket == 16)
                return launch_sample_mfma_t<16, S, MF_F32, true>(desc, ws, tile_bytes, B, max_tiles, n_samples, seed,
                                                                 off, forced, spins, logq, logits, Jv, stats, 0, st,
                                                                 mlp);
        }
        return hipErrorInvalidValue;
    }
    switch (chi_bucket) {
    case 16: return launch_sample_t<T, S, 16>(desc, ws, tile_bytes, B, max_tiles, n_samples, seed, off, forced, spins, logq, logits, Jv, stats, st);
    case 32: return launch_sample_t<T, S, 32>(desc, ws, tile_bytes, B, max_tiles, n_samples, seed, off, forced, spins, logq, logits, Jv, stats, st);
    case 64:
        // float64 caches are limited to chi <= 32
        if constexpr (sizeof(T) == 8) return hipErrorInvalidValue;
        else return launch_sample_t<T, S, 64>(desc, ws, tile_bytes, B, max_tiles, n_samples, seed, off, forced, spins, logq, logits, Jv, stats, st);
    default: return hipErrorInvalidValue;
    }
}

#define TNMC_SAMPLE_INST(T, S, SP)                                                                            \
    template hipError_t launch_sample<T, S, SP>(int, int, const InstDesc *, unsigned char *, size_t, int, int, int, \
                                                uint64_t, uint64_t, const uint64_t *, uint64_t *, double *, float *, \
                                                const float *, MlpArgs, int64_t *, hipStream_t);
TNMC_SAMPLE_INST(double, double, false)
TNMC_SAMPLE_INST(float, float, false)
TNMC_SAMPLE_INST(float, float, true)
TNMC_SAMPLE_INST(float, __hip_bfloat16, false)
TNMC_SAMPLE_INST(float, __half, false)
#undef TNMC_SAMPLE_INST

}  // namespace tnmc

// Sampling kernel: grid (sample tile, instance); the algorithm is in
// sample_device.hpp.
#include "sample_device.hpp"

namespace tnmc {

template <typename T, typename S, int CHI, bool HAS_MLP>
__global__ void __launch_bounds__(NTS)
k_sample(const InstDesc *__restrict__ desc, unsigned char *__restrict__ ws, size_t tile_bytes,
         int n_samples, uint64_t seed, uint64_t sample_offset,
         const uint64_t *__restrict__ forced, uint64_t *spins_out,
         double *__restrict__ logq_out, float *__restrict__ logits_out,
         const float *__restrict__ Jv_all, MlpArgs mlp, int64_t *__restrict__ stats) {
    const int inst = blockIdx.y, tile = blockIdx.x;
    if (tile * NTS >= n_samples) return;
    const InstDesc d = desc[inst];
    __shared__ typename StageType<T, S>::type As[4][CHI][CHI];   // two staging buffers of both spin slices
    __shared__ float Ps[HAS_MLP ? MLP_NPARAM : 1];
    T *env = reinterpret_cast<T *>(ws + d.env_off + (size_t)tile * tile_bytes);
    sample_tile<T, S, CHI, HAS_MLP>(inst, tile, d, ws, env, n_samples, seed, sample_offset, forced, spins_out,
                                    logq_out, logits_out, Jv_all, mlp, As, Ps);
    // end tick of the instance's first sample tile (the only tile when
    // n_samples <= 256), for per-instance completion times
    if (stats && tile == 0 && threadIdx.x == 0) stats[STATS_PER_INST * inst + 6] = wall_clock64();
}

template <typename T, typename S, int CHI, bool HAS_MLP>
hipError_t launch_sample_t(const InstDesc *desc, unsigned char *ws, size_t tile_bytes, int B,
                           int max_tiles, int n_samples, uint64_t seed, uint64_t off,
                           const uint64_t *forced, uint64_t *spins, double *logq, float *logits,
                           const float *Jv, MlpArgs mlp, int64_t *stats, hipStream_t st) {
    hipLaunchKernelGGL((k_sample<T, S, CHI, HAS_MLP>), dim3(max_tiles, B), dim3(NTS), 0, st, desc, ws,
                       tile_bytes, n_samples, seed, off, forced, spins, logq, logits, Jv, mlp, stats);
    return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_sample(int chi_bucket, const InstDesc *desc, unsigned char *ws, size_t tile_bytes,
                         int B, int max_tiles, int n_samples, uint64_t seed, uint64_t off,
                         const uint64_t *forced, uint64_t *spins, double *logq, float *logits,
                         const float *Jv, MlpArgs mlp, int64_t *stats, hipStream_t st) {
    if (mlp.params) {
        // the learned correction runs in float32 with chi <= 16
        if constexpr (std::is_same<T, float>::value && std::is_same<S, float>::value) {
            if (chi_bucket == 16)
                return launch_sample_t<T, S, 16, true>(desc, ws, tile_bytes, B, max_tiles, n_samples, seed, off, forced, spins, logq, logits, Jv, mlp, stats, st);
        }
        return hipErrorInvalidValue;
    }
    switch (chi_bucket) {
    case 16: return launch_sample_t<T, S, 16, false>(desc, ws, tile_bytes, B, max_tiles, n_samples, seed, off, forced, spins, logq, logits, Jv, mlp, stats, st);
    case 32: return launch_sample_t<T, S, 32, false>(desc, ws, tile_bytes, B, max_tiles, n_samples, seed, off, forced, spins, logq, logits, Jv, mlp, stats, st);
    case 64:
        // float64 caches are limited to chi <= 32
        if constexpr (sizeof(T) == 8) return hipErrorInvalidValue;
        else return launch_sample_t<T, S, 64, false>(desc, ws, tile_bytes, B, max_tiles, n_samples, seed, off, forced, spins, logq, logits, Jv, mlp, stats, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_sample<double, double>(int, const InstDesc *, unsigned char *, size_t, int, int, int, uint64_t, uint64_t, const uint64_t *, uint64_t *, double *, float *, const float *, MlpArgs, int64_t *, hipStream_t);
template hipError_t launch_sample<float, float>(int, const InstDesc *, unsigned char *, size_t, int, int, int, uint64_t, uint64_t, const uint64_t *, uint64_t *, double *, float *, const float *, MlpArgs, int64_t *, hipStream_t);
template hipError_t launch_sample<float, __hip_bfloat16>(int, const InstDesc *, unsigned char *, size_t, int, int, int, uint64_t, uint64_t, const uint64_t *, uint64_t *, double *, float *, const float *, MlpArgs, int64_t *, hipStream_t);
template hipError_t launch_sample<float, __half>(int, const InstDesc *, unsigned char *, size_t, int, int, int, uint64_t, uint64_t, const uint64_t *, uint64_t *, double *, float *, const float *, MlpArgs, int64_t *, hipStream_t);

}  // namespace tnmc

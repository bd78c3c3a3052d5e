// Device-side helpers shared by the TNMC kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace tnmc {

// Per-instance record kept in the workspace (device copy of the problem).
struct InstDesc {
    int32_t L, chi, W, flags;     // flags: TNMC_ALTERNATE_SWEEPS
    double beta;
    int64_t off_h, off_v;     // element offsets into J_h / J_v
    int64_t cache_off;        // byte offset of the cache [L][L][2][chi][chi]
    int64_t qscr_off;         // byte offset of the build scratch [L][2][2chi][chi]
    int64_t prev_off;         // byte offset of the float32 row ping-pong (mixed only)
    int64_t lsc_off;          // byte offset of the per-row log-scales [L] (double)
    int64_t env_off;          // byte offset of the sampler right-env scratch
    int64_t word_prefix;      // sum_{j<i} L_j * W_j   (spin words per sample)
    int64_t site_prefix;      // sum_{j<i} L_j * L_j
};
static_assert(sizeof(InstDesc) == 96, "InstDesc layout");

// Per-instance statistics record (int64): Jacobi sweeps, wall-clock ticks
// in QR sweeps / SVD sweeps / Jacobi loops, build start and end ticks, end
// tick of the instance's last sampling tile, ticks in the Householder
// factorisations (part of the QR sweeps); then the numeric-failure counts:
// truncations whose Jacobi stopped at the sweep limit without converging,
// and rows whose log-scale is not finite; then 1 if the truncated network's
// total (the contraction that gives ln Z) was not positive, so that ln Z is
// not finite while the cache itself is sound; then (float builds) the
// truncations whose float32 Jacobi did not converge and were redone in
// float64.
constexpr int STATS_PER_INST = 16;
constexpr int STAT_MAXSWEEP = 8, STAT_NONFINITE = 9, STAT_LOGZ_UNDEFINED = 10, STAT_FALLBACK = 11;
// ... and 1 if the row-pipelined build lost a hand-over between its two roles
// (a bounded wait ran out; the instance's cache is then not to be trusted).
constexpr int STAT_PIPE_ERROR = 12;

// Descriptor flag set by the host (beside the problem's TNMC_ALTERNATE_SWEEPS
// and TNMC_FORCE_F64_FALLBACK): build the instance with rows pipelined (float
// builds, chi <= 32, alternating sweeps); its build scratch then holds two
// rows of Q slots.
constexpr int DESC_PIPE = 4;

// Float64 redo of a float32 truncation (float builds only), per instance in
// global memory after the build scratch: both blocks and their rotations
// ([2][(chi+1)^2] doubles each), the split Jacobi's rotations in flight
// ([2][2][32][2]) and the singular values ([2][chi+2]).
__host__ __device__ constexpr size_t fallback_doubles(int chi) {
    return (size_t)4 * (chi + 1) * (chi + 1) + 256 + 2 * (chi + 2);
}

// ---- Philox4x32-10 (Salmon et al., SC'11) -----------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    }
    return c;
}

// 53 random bits of words (x, y) as a double in [0, 1).
__device__ __forceinline__ double philox_unit(uint64_t seed, uint32_t c0, uint32_t c1,
                                              uint32_t c2, uint32_t c3) {
    const U4 w = philox4x32_10(U4{c0, c1, c2, c3}, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t bits = ((uint64_t)(w.x >> 5) << 26) | (uint64_t)(w.y >> 6);
    return (double)bits * 0x1.0p-53;
}

// Normalised Boltzmann factor of one bond: entries exp(beta*J*sx*sy - beta*|J|)
// for equal (same) and opposite (diff) spins; the removed scale beta*|J| goes
// into the float64 log-scale.
__device__ __forceinline__ void boltz(double beta, float J, double &same, double &diff) {
    const double bj = beta * (double)J;
    const double a = fabs(bj);
    same = exp(bj - a);
    diff = exp(-bj - a);
}

// ---- storage conversions -----------------------------------------------------
template <typename S> __device__ __forceinline__ float to_f(S v);
template <> __device__ __forceinline__ float to_f<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_f<__hip_bfloat16>(__hip_bfloat16 v) { return __bfloat162float(v); }
template <> __device__ __forceinline__ float to_f<__half>(__half v) { return __half2float(v); }

template <typename T, typename S> __device__ __forceinline__ T load_as(const S *p) { return (T)to_f<S>(*p); }
template <> __device__ __forceinline__ double load_as<double, double>(const double *p) { return *p; }
template <> __device__ __forceinline__ float load_as<float, float>(const float *p) { return *p; }

template <typename S, typename T> __device__ __forceinline__ S store_as(T v);
template <> __device__ __forceinline__ double store_as<double, double>(double v) { return v; }
template <> __device__ __forceinline__ float store_as<float, float>(float v) { return v; }
template <> __device__ __forceinline__ __hip_bfloat16 store_as<__hip_bfloat16, float>(float v) { return __float2bfloat16(v); }
template <> __device__ __forceinline__ __half store_as<__half, float>(float v) { return __float2half(v); }

template <typename T> struct Eps;
template <> struct Eps<double> { static constexpr double v = 2.220446049250313e-16; };
template <> struct Eps<float> { static constexpr float v = 1.1920929e-07f; };

// Scale a positive value's exponent away: returns 2^-e with m*2^-e in [0.5, 1).
__device__ __forceinline__ double pow2_inv(double m) { int e; frexp(m, &e); return ldexp(1.0, -e); }
__device__ __forceinline__ float pow2_inv(float m) { int e; frexpf(m, &e); return ldexpf(1.0f, -e); }

// ln(sigmoid(x)) without overflow; x may be +-inf.
__device__ __forceinline__ double log_sigmoid(double x) {
    if (x >= 0.0) return -log1p(exp(-x));
    return x - log1p(exp(x));
}

}  // namespace tnmc

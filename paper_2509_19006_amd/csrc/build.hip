// Boundary-MPS cache build kernel: one workgroup per instance, instances in
// the host's longest-first order (the algorithm is in build_device.hpp).
#include "build_pipe.hpp"

namespace tnmc {

template <typename T, typename S, int MAXB, bool PIPE>
__global__ void __launch_bounds__(NT)
k_build(const InstDesc *__restrict__ desc, const int32_t *__restrict__ order,
        unsigned char *__restrict__ ws, const float *__restrict__ Jh_all,
        const float *__restrict__ Jv_all, double *__restrict__ logz_out,
        int64_t *__restrict__ stats_out) {
    extern __shared__ __align__(16) unsigned char smem[];
    build_instance_sel<T, S, MAXB, PIPE>(order[blockIdx.x], desc, ws, Jh_all, Jv_all, logz_out, stats_out, smem);
}

// Host-side launch helpers (called from the C ABI layer).  chi_max selects
// the widest register path compiled into the kernel; pipe the row-pipelined
// form (float, chi_max <= 32).
template <typename T, typename S, int MAXB, bool PIPE>
hipError_t launch_build_w(const InstDesc *desc, const int32_t *order, unsigned char *ws, const float *Jh,
                          const float *Jv, double *logz, int64_t *stats, int B, size_t lds_bytes, hipStream_t st) {
    auto kern = k_build<T, S, MAXB, PIPE>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(B), dim3(NT), lds_bytes, st, desc, order, ws, Jh, Jv, logz, stats);
    return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_build(const InstDesc *desc, const int32_t *order, unsigned char *ws, const float *Jh,
                        const float *Jv, double *logz, int64_t *stats, int B, int chi_max, bool pipe,
                        size_t lds_bytes, hipStream_t st) {
    if constexpr (sizeof(T) == 8) {
        if (chi_max > 32 || pipe) return hipErrorInvalidValue;
        return launch_build_w<T, S, 32, false>(desc, order, ws, Jh, Jv, logz, stats, B, lds_bytes, st);
    } else {
        if (pipe) {
            if (chi_max > 32) return hipErrorInvalidValue;
            return launch_build_w<T, S, 32, true>(desc, order, ws, Jh, Jv, logz, stats, B, lds_bytes, st);
        }
        if (chi_max <= 32) return launch_build_w<T, S, 32, false>(desc, order, ws, Jh, Jv, logz, stats, B, lds_bytes, st);
        return launch_build_w<T, S, 64, false>(desc, order, ws, Jh, Jv, logz, stats, B, lds_bytes, st);
    }
}

#define TNMC_LB(T, S) template hipError_t launch_build<T, S>(const InstDesc *, const int32_t *, unsigned char *, \
    const float *, const float *, double *, int64_t *, int, int, bool, size_t, hipStream_t);
TNMC_LB(double, double)
TNMC_LB(float, float)
TNMC_LB(float, __hip_bfloat16)
TNMC_LB(float, __half)
#undef TNMC_LB

// Shared-memory bytes the build kernel needs for bond dimension chi and side L.
size_t build_pipe_lds_bytes(int chi, int L) {
    const size_t cb = chi <= 16 ? 16 : 32;
    const size_t vl = 2 * cb + (64 / cb - 1) * (cb >= 32 ? 4 : 0);   // padded Householder vector
    const size_t bst = (size_t)(chi + 1) * (chi + 1);
    // QR role: C, R, V, tau, R columns; SVD role: Tm, Wm, X, Qst, nrm, Jacobi rotations
    size_t elems = 3 * cb * cb + 2 * cb * vl + 2 * cb + 2 * cb * (cb + 4);
    elems += 4 * bst + (size_t)6 * chi * chi + 2 * (chi + 2) + 4 * cb;
    size_t bytes = elems * sizeof(float);
    bytes = (bytes + 7) & ~(size_t)7;
    bytes += (size_t)(10 + 128 + 8) * sizeof(double) + 2 * sizeof(long long);   // sums, uvec, scal, ticks
    bytes += (size_t)(2 * (2 * chi + 4) + 4 + 2 + 8) * sizeof(int);              // colof, rankv, flags, hand-over
    bytes += (size_t)6 * (L + 1) + 4;                                             // dsec, two rows of mq
    bytes += (size_t)4 * 2 * L;                                                   // the row's couplings
    return (bytes + 15) & ~(size_t)15;
}

size_t build_lds_bytes(int chi, int L, size_t tsize) {
    const size_t cb = chi <= 16 ? 16 : (chi <= 32 ? 32 : 64);
    const size_t vl = 2 * cb + (128 / cb - 1) * (cb >= 32 ? 4 : 0);   // padded Householder vector
    const size_t regA = 3 * cb * cb + 2 * cb * vl;
    const size_t regS = (size_t)4 * (chi + 1) * (chi + 1) + (size_t)2 * chi * chi +
                        (cb <= 32 ? (size_t)4 * chi * chi : 0);   // + staged Q slot
    size_t elems = (regA > regS ? regA : regS);
    elems += 2 * cb + 2 * (chi + 2) + 4 * cb;                 // tau, nrm, Jacobi rotations
    size_t bytes = elems * tsize;
    bytes = (bytes + 7) & ~(size_t)7;
    bytes += (NT / 64 + 128 + 8) * sizeof(double);           // red, uvec, scal
    bytes += (2 * (2 * chi + 4) + 4 + 2) * sizeof(int);      // colof, rankv, iflag, jflag
    bytes += (size_t)4 * (L + 1) + 4;                        // dsec, mq (+ alignment)
    bytes += (size_t)4 * 2 * L;                              // the row's couplings
    return (bytes + 15) & ~(size_t)15;
}

}  // namespace tnmc

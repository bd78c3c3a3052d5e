// Boundary-MPS cache build (arXiv 2509.19006, section 2.2 / Fig. 2 and
// section 3.2): starting from the bottom row, apply each row's transfer MPO
// to the boundary MPS and truncate back to bond dimension chi.
//
// Spin-flip (Z2) symmetric formulation.  With no field every Boltzmann matrix
// (Eq. 7) is symmetric under flipping both spins, so in the basis
// h_0 = (1,1)/sqrt2 (even), h_1 = (1,-1)/sqrt2 (odd) it is diagonal with
// eigenvalues lam = (a+b, a-b), and every copy tensor (Eq. 8) becomes a
// parity constraint (legs' parities sum to even).  In that basis every bond
// of the boundary MPS splits into an even and an odd sector (stored as one
// index: even entries first), site tensors are parity conserving, and the
// matrices the compression decomposes are block diagonal.  The truncated
// state is the one the plain SVD sweep produces (exactly, in exact
// arithmetic): keeping the chi largest singular values of a block-diagonal
// matrix means keeping the largest of both blocks together.  The even/odd
// pairs of nearly equal singular values that a spin-flip symmetric state
// has never meet inside one Jacobi problem, which is what makes the
// one-sided Jacobi converge in few sweeps.
//
// One workgroup (256 threads, 4 waves) owns one instance and walks its rows
// bottom to top.  Per row:
//   * apply   -- site c of MPO x MPS is A'[(a,l),s,(b,t)] =
//                lam_h(c-1)[l] lam_v(c)[n] A_old[a,n,b], n = l^s^t; never
//                formed, folded into the next step;
//   * QR sweep, left to right -- R * A'_c splits into two parity blocks
//                M^p = [Rh^p C ; Rh^(1-p) C] with C[a,b] = lam_v[pa^pb] *
//                A_old[a, pa^pb, b] and Rh^q = R^q scaled column-wise by
//                lam_h[q ^ pa]; each block gets a Householder QR;
//   * SVD sweep, right to left -- center T^p = [Q^p_0 X^p, Q^(1-p)_1 X^(1-p)]
//                for p = 0, 1; one-sided (Hestenes) Jacobi on both blocks at
//                once (round-robin pair order); keep the chi largest singular
//                values over both; V^T becomes the site, U*S moves left.
// The cache is written in the spin basis, A[x] = (A~[even] + (-1)^x A~[odd])
// / sqrt2, which is what the sampler contracts.  All norms removed along the
// way go to a float64 log-scale per row, so that ln Z = sum_r logscale[r] +
// (L/2) ln 2 + ln(row-0 MPS contracted on its even physical component).
//
// Template T is the arithmetic type (double or float); S the cache storage
// type (double, float, bfloat16 or half).  The previous row is kept in T in a
// parity-basis ping-pong buffer, so the build never reads rounded values.
#pragma once
#include <type_traits>

#include "device.hpp"

namespace tnmc {

constexpr int NT = 256;
constexpr int MAX_SWEEPS = 40;

// Cross-lane moves inside 16-lane rows use DPP (no trip through the LDS
// permute unit); wider steps fall back to __shfl_xor.
template <int CTRL> __device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over aligned groups of G consecutive lanes (G a power of two <= 64);
// every lane of a group gets the group's sum.
template <typename T> __device__ __forceinline__ T group_sum(T v, int G) {
    if (G >= 2) v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
    if (G >= 4) v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
    if (G >= 8) v += dpp_move<0x141>(v);   // row_half_mirror: partner in the other quad
    if (G >= 16) v += dpp_move<0x140>(v);  // row_mirror: partner in the other half-row
    if (G >= 32) v += __shfl_xor(v, 16, 64);
    if (G >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

__device__ __forceinline__ int pow2_floor(int x) {
    int p = 1;
    while ((p << 1) <= x) p <<= 1;
    return p;
}

// Workgroup sum of one double (all threads get the result).
__device__ double block_sum(double v, double *red) {
    v = group_sum(v, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}

// Round-robin ("circle") tournament: seat q of round t (0 <= t < n-1).
__device__ __forceinline__ int seat(int q, int t, int n) {
    if (q == 0) return 0;
    int v = q - 1 + t;
    if (v >= n - 1) v -= n - 1;
    return 1 + v;
}

__device__ __forceinline__ double fast_rcp(double x) { return __builtin_amdgcn_rcp(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// Square root on the rotation's critical path: the hardware's 1-ulp float
// instruction (the correctly rounded sequence is about ten times longer; it
// differs only for denormal inputs, which the caller excludes); float64
// keeps the exact operation.
__device__ __forceinline__ double path_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float path_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// 1/sqrt(x) from the hardware estimate refined by one Newton step.
__device__ __forceinline__ double rsqrt_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return y * (1.5 - 0.5 * x * y * y);
}
__device__ __forceinline__ float rsqrt_nr(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    return y * (1.5f - 0.5f * x * y * y);
}
// 1/sqrt on the rotation's dependency chain: the float estimate is already
// within an ulp; float64 needs the Newton step.
__device__ __forceinline__ double path_rsqrt(double x) { return rsqrt_nr(x); }
__device__ __forceinline__ float path_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

// Orders a wave's shared-memory accesses without a workgroup barrier: the
// LDS serves one wave's instructions in order, the fences stop the compiler
// from moving accesses across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cross-lane read through the LDS permute crossbar: the value held by the
// lane whose byte address is addr (lane * 4).
template <typename T> __device__ __forceinline__ T bperm(int addr, T v);
template <> __device__ __forceinline__ float bperm<float>(int addr, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
template <> __device__ __forceinline__ double bperm<double>(int addr, double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Rotation that makes columns with squared norms a, b and inner product c
// orthogonal: with d = b - a and e = 2c, tan = sign(d) e / (|d| + sqrt(d^2 +
// e^2)) (the smaller root of Rutishauser's quadratic, free of overflow for
// |d| >> |e|); identity (cs = 1, sn = 0) when the pair is orthogonal to
// tolerance or either column is noise.  An idle pair (live false) gets the
// exact quarter turn cs = 0, sn = 1, (u, v) -> (-v, u): it exchanges the two
// columns (one negated, which the SVD does not see: the same column of W
// changes sign with it), so that every group hands on its columns the same
// way after the step.  Updates the squared norms (a' = a - t c, b' = b + t c;
// exchanged for an idle pair) and returns whether the pair rotates.
template <typename T>
__device__ __forceinline__ bool jacobi_rotation(T &a, T &b, T c, T small, T tol2, bool live, T &cs, T &sn) {
    const T d = b - a, e = c + c;
    const T den = fabs(d) + path_sqrt(d * d + e * e);
    // (bitwise: a short-circuit chain becomes branches on the exec mask)
    const bool ok = live & (a > small) & (b > small) & (c * c > tol2 * a * b) & (den > (T)0);
    const T t = (d >= 0 ? e : -e) * fast_rcp(ok ? den : (T)1);
    const T c0 = path_rsqrt((T)1 + t * t);
    const T tt = ok ? t : (T)0;
    cs = ok ? c0 : (live ? (T)1 : (T)0);
    sn = ok ? c0 * t : (live ? (T)0 : (T)1);
    const T na = live ? a - tt * c : b, nb = live ? b + tt * c : a;
    a = na;
    b = nb;
    return ok;
}

// Lane groups of the register Jacobi.  In the contiguous layout group g is
// lanes [gG, gG+G) and a column moves to the neighbouring group through the
// LDS permute crossbar.  In the interleaved layout (CHI = 32, G = 4) group g
// is lanes g, g+16, g+32, g+48: neighbouring groups are neighbouring lanes of
// every 16-lane row, so a column moves by one DPP rotate of the row, and a
// group's sum crosses the rows with the swaps of lane halves (l ^ 16, l ^ 32)
// that gfx950 has.  Both keep a move or a sum inside the vector unit's
// latency instead of an LDS round trip on the rotation's dependency chain.
__device__ __forceinline__ float swap_sum16(float v) {
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);   // {own, partner} in either order
}
__device__ __forceinline__ float swap_sum32(float v) {
    const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
__device__ __forceinline__ double swap_sum16(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    return __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0])) +
           __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ __forceinline__ double swap_sum32(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    return __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0])) +
           __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
template <bool IL, typename T> __device__ __forceinline__ T pair_sum(T v, int G) {
    if constexpr (IL) return swap_sum32(swap_sum16(v));
    else return group_sum(v, G);
}
// value of the same lane slot in group g+1 (up) or g-1 (down), cyclically
template <bool IL, typename T> __device__ __forceinline__ T from_next(T v, int up) {
    if constexpr (IL) return dpp_move<0x12F>(v);   // row_ror:15
    else return bperm<T>(up, v);
}
template <bool IL, typename T> __device__ __forceinline__ T from_prev(T v, int dn) {
    if constexpr (IL) return dpp_move<0x121>(v);   // row_ror:1
    else return bperm<T>(dn, v);
}

// One-sided (Hestenes) Jacobi on one block, the form for chi <= 32, with
// the block in one wave's registers (role 0).  The block has n columns (n
// even, n <= CHI) of length K <= CHI at Tb, column-major with leading
// dimension ld; columns n..CHI-1 are treated as zero and never rotate.
// Column pairs follow the odd-even transposition order over CHI positions:
// even steps pair positions (2g, 2g+1), odd steps (2g+1, 2g+2) with
// positions 0 and CHI-1 idle, and every pair swaps positions after its step;
// CHI steps meet every pair once and reverse the order.  The wave splits
// into CHI/2 lane groups of G = 128/CHI lanes (contiguous or interleaved,
// IL); group g holds the two columns of its pair (rows strided over its
// lanes).  Going from an even to an odd step a group takes the second column
// of the next group; going back, the first column of the previous group (the
// last group, idle in odd steps, exchanges its two by a quarter turn first,
// so it hands over the one at position 0): one move per column and step.
// Squared column norms are recomputed every sweep and carried through each
// rotation exactly (a' = a - t*g, b' = b + t*g), so a pair needs one
// reduction.  Pairs whose smaller column is below sqrt(n)*eps*||T||_F are
// left alone: such columns are rounding noise and a relative orthogonality
// test on them never settles.
// The accumulated rotation W (from the identity) is carried by the same
// wave, in registers beside the block.
// The sweeps start from the columns ordered by decreasing norm (de Rijk's
// pivoting, which shortens cyclic Jacobi).  On return the rotated block is back at Tb and W (n x n, same
// leading dimension) at Wb, and the block wave writes the singular values
// (column norms) of the positions to nrm_out[0, n): -1 for positions >= kr
// and for an empty block.  Returns the sweep count (role 0); a count equal to
// max_sweeps means the last sweep still rotated (not converged).  The block
// and W sit in shared memory (LDSP) or in global memory.
template <typename T, int CHI, bool IL, bool LDSP = true>
__device__ int jacobi_reg(T *Tb, T *Wb, int ld, int K, int n, int lane, int role, T *nrm_out, int kr,
                          int max_sweeps) {
    static_assert(!IL || CHI == 32, "the interleaved layout rotates 16-lane rows");
    constexpr int HP = CHI / 2, G = 64 / HP, RK = CHI / G;
    if (role != 0) return 0;
    // the block in shared memory (LDSP) or in global memory
    typedef __attribute__((address_space(3))) T LT;
    typedef typename std::conditional<LDSP, LT, T>::type PT;
    PT *Tl = (PT *)Tb, *Wl = (PT *)Wb;
    int g = IL ? (lane & 15) : lane / G, gl = IL ? (lane >> 4) : lane % G;
    asm volatile("" : "+v"(g), "+v"(gl));   // see qr_site
    // pivoting: lane l < CHI measures column l, ranks it among all, and
    // position p takes the column of rank p.  Positions, not column
    // numbers, are written back: the caller ranks the result by norm, and
    // W's columns follow the block's.
    int src2, src3;
    {
        T nl = (T)-1;
        if (lane < n) {
            T q0 = 0, q1 = 0;
            const PT *cp = Tl + lane * ld;
            T q2 = 0, q3 = 0;
            int k = 0;
            for (; k + 3 < K; k += 4) {
                q0 += cp[k] * cp[k];
                q1 += cp[k + 1] * cp[k + 1];
                q2 += cp[k + 2] * cp[k + 2];
                q3 += cp[k + 3] * cp[k + 3];
            }
            for (; k < K; ++k) q0 += cp[k] * cp[k];
            nl = (q0 + q1) + (q2 + q3);
        }
        int rk = 0;
#pragma unroll
        for (int j = 0; j < CHI; ++j) {
            const T nj = bperm<T>(j << 2, nl);
            rk += (nj > nl) || (nj == nl && j < lane);
        }
        // column of each position: lane l sends its index to lane rank(l)
        const int colpos = __builtin_amdgcn_ds_permute((lane < CHI ? rk : lane) << 2, lane);
        // (clamped: a position nobody claimed reads as padding)
        src2 = (int)min((unsigned)__builtin_amdgcn_ds_bpermute((2 * g) << 2, colpos), (unsigned)CHI);
        src3 = (int)min((unsigned)__builtin_amdgcn_ds_bpermute((2 * g + 1) << 2, colpos), (unsigned)CHI);
    }
    // x, y: the pair's columns of the block; wx, wy: the same columns of W
    T x[RK], y[RK], wx[RK], wy[RK];
#pragma unroll
    for (int i = 0; i < RK; ++i) {
        const int row = gl + G * i;
        x[i] = (row < K && src2 < n) ? Tl[src2 * ld + row] : (T)0;
        y[i] = (row < K && src3 < n) ? Tl[src3 * ld + row] : (T)0;
        wx[i] = (row == src2) ? (T)1 : (T)0;
        wy[i] = (row == src3) ? (T)1 : (T)0;
    }
    const int up = ((lane + G) & 63) << 2, dn = ((lane - G) & 63) << 2;
    const bool last = (g == HP - 1);
    int sweeps = 0;
    {
        const T tol = (T)2 * Eps<T>::v * sqrt((T)K);
        const T tol2 = tol * tol;
        T small = 0;
        for (int sw = 0; sw < max_sweeps; ++sw) {
            T a = 0, b = 0;
#pragma unroll
            for (int i = 0; i < RK; ++i) { a += x[i] * x[i]; b += y[i] * y[i]; }
            if (sw == 0) small = group_sum(a + b, 64) * (T)(1.0 / G) * Eps<T>::v * Eps<T>::v * (T)n;
            a = pair_sum<IL>(a, G);
            b = pair_sum<IL>(b, G);
            bool rot = false;
            // W takes each step's rotation one step late: its update and
            // move do not feed the next step's rotation, so they fill the
            // wait on that step's reduction and square roots
            T wcs = (T)1, wsn = (T)0;
            auto w_rotate = [&](auto ODD) {
                constexpr bool O = decltype(ODD)::value;
#pragma unroll
                for (int i = 0; i < RK; ++i) {
                    const T p = wx[i], q = wy[i];
                    wx[i] = wcs * p - wsn * q;
                    wy[i] = wsn * p + wcs * q;
                }
#pragma unroll
                for (int i = 0; i < RK; ++i) {
                    if (!O) wy[i] = from_next<IL>(wy[i], up);
                    else wx[i] = from_prev<IL>(wx[i], dn);
                }
            };
            // one step; pending: W still owes the previous step (of the
            // other parity)
            auto step = [&](auto ODD, bool pending) {
                constexpr bool O = decltype(ODD)::value;
                T c0 = 0, c1 = 0;
#pragma unroll
                for (int i = 0; i < RK; i += 2) {
                    c0 += x[i] * y[i];
                    if (i + 1 < RK) c1 += x[i + 1] * y[i + 1];
                }
                const T c = pair_sum<IL>(c0 + c1, G);
                if (pending) w_rotate(std::integral_constant<bool, !O>{});
                T cs, sn;
                rot |= jacobi_rotation<T>(a, b, c, small, tol2, !(O && last), cs, sn);
#pragma unroll
                for (int i = 0; i < RK; ++i) {
                    const T u = x[i], v = y[i];
                    x[i] = cs * u - sn * v;
                    y[i] = sn * u + cs * v;
                }
                if (!O) {
                    // even -> odd layout: second column from the next group
#pragma unroll
                    for (int i = 0; i < RK; ++i) y[i] = from_next<IL>(y[i], up);
                    b = from_next<IL>(b, up);
                } else {
                    // odd -> even layout: first column from the previous
                    // group (the idle last group has exchanged its two)
#pragma unroll
                    for (int i = 0; i < RK; ++i) x[i] = from_prev<IL>(x[i], dn);
                    a = from_prev<IL>(a, dn);
                }
                wcs = cs;
                wsn = sn;
            };
            using Even = std::integral_constant<bool, false>;
            using Odd = std::integral_constant<bool, true>;
            step(Even{}, false);
            for (int s = 0; s + 2 < CHI; s += 2) {
                step(Odd{}, true);
                step(Even{}, true);
            }
            step(Odd{}, true);
            w_rotate(Odd{});
            ++sweeps;
            if (__ballot(rot) == 0) break;
        }
    }
    // after an odd number of sweeps the positions are reversed
    const bool rev = sweeps & 1;
    const int cx = rev ? CHI - 1 - 2 * g : 2 * g, cy = rev ? CHI - 2 - 2 * g : 2 * g + 1;
    {
        // singular values from the registers (rows >= K hold zeros)
        T sx[2] = {0, 0}, sy[2] = {0, 0};
#pragma unroll
        for (int i = 0; i < RK; ++i) { sx[i & 1] += x[i] * x[i]; sy[i & 1] += y[i] * y[i]; }
        const T nx = pair_sum<IL>(sx[0] + sx[1], G), ny = pair_sum<IL>(sy[0] + sy[1], G);
        if (gl == 0) {
            if (cx < n) nrm_out[cx] = (cx < kr && K > 0) ? sqrt(nx) : (T)-1;
            if (cy < n) nrm_out[cy] = (cy < kr && K > 0) ? sqrt(ny) : (T)-1;
        }
    }
#pragma unroll
    for (int i = 0; i < RK; ++i) {
        const int row = gl + G * i;
        if (row < K) {
            if (cx < n) Tl[cx * ld + row] = x[i];
            if (cy < n) Tl[cy * ld + row] = y[i];
        }
        if (row < n) {
            if (cx < n) Wl[cx * ld + row] = wx[i];
            if (cy < n) Wl[cy * ld + row] = wy[i];
        }
    }
    return sweeps;
}

// One-sided (Hestenes) Jacobi on one block with the block in one wave's
// registers and the accumulated rotation W in a second wave's (the form for
// chi = 64, where a step's instruction count, not its dependency chain,
// sets its length).  The block
// has n columns (n even, n <= CHI) of length K <= CHI at Tb, column-major
// with leading dimension ld; columns n..CHI-1 are treated as zero and never
// rotate.  Column pairs follow the odd-even transposition order over CHI
// positions: even steps pair positions (2g, 2g+1), odd steps (2g+1, 2g+2)
// with positions 0 and CHI-1 idle, and every pair swaps positions after its
// step; CHI steps meet every pair once and reverse the order.  Each wave
// splits into CHI/2 lane groups of G = 128/CHI lanes; group g holds the two
// columns of its pair (rows strided over its lanes).  Going from an even to
// an odd step a group takes the second column of the next group; going
// back, the first column of the previous group (the last group, idle in odd
// steps, exchanges its two by a quarter turn first, so it hands over the one
// at position 0): one move per column and step, through the LDS permute
// crossbar.
//   role 0 (the block): squared column norms are recomputed every sweep and
//   carried through each rotation exactly (a' = a - t*g, b' = b + t*g), so a
//   pair needs one reduction; pairs whose smaller column is below
//   sqrt(n)*eps*||T||_F are left alone (rounding noise, on which a relative
//   orthogonality test never settles).  Each step's (cos, sin) per group go
//   to prm before the workgroup barrier that ends the step.
//   role 1 (W, starting from the identity): after that barrier it applies
//   the same step's rotations, one step behind the block.
// All four waves of the workgroup call this together (the two blocks' role 0
// and role 1 waves): the barriers are workgroup-wide, so both blocks sweep
// until neither rotates (extra sweeps of a converged block rotate nothing).
// prm: [2 blocks][2 slots][CHI/2][2], flags: [2].  On return the rotated
// block is back at Tb (role 0) and W (n x n, same leading dimension) at Wb
// (role 1).  Returns the sweep count (max_sweeps: not converged).
template <typename T, int CHI>
__device__ int jacobi_split(T *Tb, T *Wb, int ld, int K, int n, int lane, int role, int p, T *prm, int *flags,
                            int max_sweeps) {
    constexpr int HP = CHI / 2, G = 64 / HP, RK = CHI / G;
    int g = lane / G, gl = lane % G;
    asm volatile("" : "+v"(g), "+v"(gl));   // see qr_site
    const bool blk = (role == 0);
    T x[RK], y[RK];
#pragma unroll
    for (int i = 0; i < RK; ++i) {
        const int row = gl + G * i;
        if (blk) {
            x[i] = (row < K && 2 * g < n) ? Tb[(2 * g) * ld + row] : (T)0;
            y[i] = (row < K && 2 * g + 1 < n) ? Tb[(2 * g + 1) * ld + row] : (T)0;
        } else {
            x[i] = (row == 2 * g) ? (T)1 : (T)0;
            y[i] = (row == 2 * g + 1) ? (T)1 : (T)0;
        }
    }
    const int up = ((lane + G) & 63) << 2, dn = ((lane - G) & 63) << 2;
    const bool last = (g == HP - 1);
    const T tol = (T)2 * Eps<T>::v * sqrt((T)K);
    const T tol2 = tol * tol;
    T *pp = prm + p * 4 * HP;
    T small = 0;
    int sweeps = 0, slot = 0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        T a = 0, b = 0;
        if (blk) {
#pragma unroll
            for (int i = 0; i < RK; ++i) { a += x[i] * x[i]; b += y[i] * y[i]; }
            if (sw == 0) small = group_sum(a + b, 64) * (T)(1.0 / G) * Eps<T>::v * Eps<T>::v * (T)n;
            a = group_sum(a, G);
            b = group_sum(b, G);
        }
        bool rot = false;
        for (int t = 0; t < CHI; t += 2) {
#pragma unroll
            for (int odd = 0; odd < 2; ++odd) {
                T cs = 1, sn = 0;
                T *ps = pp + (slot * HP + g) * 2;
                if (blk) {
                    T c0 = 0, c1 = 0;
#pragma unroll
                    for (int i = 0; i < RK; i += 2) {
                        c0 += x[i] * y[i];
                        if (i + 1 < RK) c1 += x[i + 1] * y[i + 1];
                    }
                    const T c = group_sum(c0 + c1, G);
                    rot |= jacobi_rotation<T>(a, b, c, small, tol2, !(odd && last), cs, sn);
                    if (gl == 0) { ps[0] = cs; ps[1] = sn; }
                }
                __syncthreads();
                if (!blk) {
                    cs = ps[0];
                    sn = ps[1];
                }
                slot ^= 1;
#pragma unroll
                for (int i = 0; i < RK; ++i) {
                    const T u = x[i], v = y[i];
                    x[i] = cs * u - sn * v;
                    y[i] = sn * u + cs * v;
                }
                if (!odd) {
                    // even -> odd layout: second column from the next group
#pragma unroll
                    for (int i = 0; i < RK; ++i) y[i] = bperm<T>(up, y[i]);
                    if (blk) b = bperm<T>(up, b);
                } else {
                    // odd -> even layout: first column from the previous
                    // group (the idle last group has exchanged its two)
#pragma unroll
                    for (int i = 0; i < RK; ++i) x[i] = bperm<T>(dn, x[i]);
                    if (blk) a = bperm<T>(dn, a);
                }
            }
        }
        ++sweeps;
        const bool any = __ballot(rot) != 0;
        if (blk && lane == 0) flags[p] = any;
        __syncthreads();
        const bool more = flags[0] || flags[1];
        if (!more) break;
    }
    // after an odd number of sweeps the positions are reversed
    const bool rev = sweeps & 1;
    const int cx = rev ? CHI - 1 - 2 * g : 2 * g, cy = rev ? CHI - 2 - 2 * g : 2 * g + 1;
#pragma unroll
    for (int i = 0; i < RK; ++i) {
        const int row = gl + G * i;
        if (blk) {
            if (row < K) {
                if (cx < n) Tb[cx * ld + row] = x[i];
                if (cy < n) Tb[cy * ld + row] = y[i];
            }
        } else if (row < n) {
            if (cx < n) Wb[cx * ld + row] = x[i];
            if (cy < n) Wb[cy * ld + row] = y[i];
        }
    }
    return sweeps;
}

// The register Jacobi for the smallest compiled width that holds chi; MAXB
// is the widest one compiled into this kernel (wider paths only cost
// registers, so a kernel carries the ones its launch needs).  Called by all
// four waves: waves 0 and 1 hold the blocks (role 0); for chi = 64 waves 2
// and 3 carry their rotations W (role 1, through prm and flags), for
// chi <= 32 the block's wave carries W itself.  For chi <= 32 the block
// waves also write the singular values to nrm_out (see jacobi_reg).
template <typename T, int MAXB, bool LDSP = true>
__device__ int jacobi_block(T *Tb, T *Wb, int ld, int K, int n, int chi, int lane, int role, int p, T *prm,
                            int *flags, T *nrm_out, int kr, int max_sweeps) {
    if constexpr (MAXB >= 64) {
        if (chi > 32) return jacobi_split<T, 64>(Tb, Wb, ld, K, n, lane, role, p, prm, flags, max_sweeps);
    }
    // chi <= 16: contiguous groups; chi <= 32: interleaved groups; W in the
    // block's wave
    if (chi <= 16) return jacobi_reg<T, 16, false, LDSP>(Tb, Wb, ld, K, n, lane, role, nrm_out, kr, max_sweeps);
    return jacobi_reg<T, 32, true, LDSP>(Tb, Wb, ld, K, n, lane, role, nrm_out, kr, max_sweeps);
}

// Sum over a lane's rows of a[r] * b[r] in four independent partial sums
// (a single running sum is one dependent chain as long as the rows).
template <typename T, int RR>
__device__ __forceinline__ T rows_dot(const T (&a)[RR], const T (&b)[RR]) {
    T s[4] = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < RR; ++r) s[r & 3] += a[r] * b[r];
    return (s[0] + s[1]) + (s[2] + s[3]);
}

// Column swizzle of the carried factor R: element (qk, a) of R [2CHI rows]
// is stored at qk*CHI + (a ^ rkey(qk)).  The lanes of a group read rows
// RR apart, which without it fall in the same LDS banks (a row is CHI words
// long); the key moves their 16-byte column chunks to different banks and
// keeps the chunks aligned.  Returns qk*CHI + rkey(qk): XOR with a column
// index (< CHI) gives the element.
template <int CHI, int RR> __device__ __forceinline__ int rkey_base(int qk) {
    return qk * CHI + (((qk / RR) & 3) << 2);
}

// Householder vectors in shared memory: a lane group's lanes hold RR
// consecutive rows each, so for CHI >= 32 their segments would start on the
// same LDS banks; each segment is padded by 4 words.  Row stride of V:
template <int CHI> constexpr int vrow_len() {
    return 2 * CHI + (128 / CHI - 1) * (CHI >= 32 ? 4 : 0);
}

// One site of the QR sweep for both parity blocks, held in registers.
// Block p belongs to waves 2p and 2p+1 (128 lanes); lane group grp (G =
// 128/CHI lanes) owns column grp of M^p and each of its lanes RR = 2CHI/G
// consecutive rows.  Shared memory (CHI-strided): C [CHI][CHI] (row a of the
// old left bond, column b of the old right bond), R [2][CHI][CHI] (the
// factor carried from the previous site, already scaled into Rh, zero
// outside its trapezoid; element (qk, a) at qk*CHI + (a ^ rkey(qk)), see
// rkey), V [2][CHI][2CHI] (Householder vectors), tauv [2][CHI].
//   M^p rows: sigma = 0 -> Rh^p C (m_p rows), sigma = 1 -> Rh^(1-p) C, where
//   Rh^q scales column a of R^q by lam_h[(a's sector) ^ q]; at c = 0 the
//   single row is C's first row.  The scaling belongs to the next site's
//   horizontal bond and is applied where R is written (lnh0, lnh1: its
//   eigenvalues; pn0: the even sector size of the bond R leaves to).
//   Householder QR (LAPACK's reflector convention): per column j the owner
//   group publishes v_j and tau_j, every later column applies H_j.  The
//   explicit Q (K x mc) goes to qdst ([2][2chi][chi], row-major, stride chi);
//   V holds vector j of block p at (p CHI + j) vrow_len, row r of a lane's
//   segment at its padded offset.
//   R (mc x D, normalised jointly over both blocks) replaces the R array.
//   CHI = 64 (float builds only): a lane holds 64 rows, and selecting them
//   against the step every step spills; there row j of every column moves,
//   at step j, to Rsc ([2][64][68] floats, column-major, in the workspace)
//   and is zeroed in the registers, so that a column's rows above the step
//   are always zero: the pivot takes its diagonal entry out of the registers
//   at the step's uniform index, the norm of the part below it is the sum
//   over all rows, and the reflector the scaled column with a 1 written at
//   the diagonal.
// At the last site (D = 1) only block 0's single column is written to qdst
// (the centre of the sweep) and nothing is factored.  Returns ln of the
// joint norm (0 at the last site) and mc.
template <typename T, int CHI>
__device__ double qr_site(int c, int last, int K, int D, int Dp, int pa0, int m0, int m1, int pn0, T lnh0,
                          T lnh1, const T *C, T *R, T *V, T *tauv, T *Rsc, T *qdst, int chi, double *red,
                          int &mc_out, long long &cyc_hh) {
    constexpr int G = 128 / CHI, RR = 2 * CHI / G;
    const int tid = threadIdx.x, p = tid >> 7, lt = tid & 127;
    int grp = lt / G, row0 = (lt % G) * RR;
    // opaque to the optimiser: keeps the per-lane masks and addresses
    // derived from these from being hoisted out of the row loop (they
    // would stay live across the whole build)
    asm volatile("" : "+v"(grp), "+v"(row0));
    const int gl = row0 / RR;
    const int vrow0 = row0 + gl * (CHI >= 32 ? 4 : 0);   // padded start of the lane's rows in V
    constexpr int VL = vrow_len<CHI>();
    const int mp = p ? m1 : m0;
    T m[RR];
    if (c == 0) {
        const T x = (grp < D) ? C[grp] : (T)0;
#pragma unroll
        for (int r = 0; r < RR; ++r) m[r] = (row0 + r == 0) ? x : (T)0;
    } else {
        // M = sum_a Rh_q[k][a] C[a][grp]: chunks of 4 columns of C against
        // the rows' Rh entries
        int roff[RR];
        T acc[RR];
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int row = row0 + r;
            const int q = (row < mp) ? p : 1 - p;
            const int k = (row < K) ? ((row < mp) ? row : row - mp) : 0;
            roff[r] = rkey_base<CHI, RR>(q * CHI + k);
            acc[r] = 0;
        }
#pragma unroll 1
        for (int a0 = 0; a0 < CHI; a0 += 4) {
            T cv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int a = a0 + i;
                cv[i] = (a < Dp && grp < D) ? C[a * CHI + grp] : (T)0;
            }
#pragma unroll
            for (int r = 0; r < RR; ++r) {
                const T *Rq = R + (roff[r] ^ a0);
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[r] += Rq[i] * cv[i];
            }
        }
#pragma unroll
        for (int r = 0; r < RR; ++r) m[r] = (row0 + r < K) ? acc[r] : (T)0;
    }
    if (last) {
        if (p == 0 && grp == 0) {
#pragma unroll
            for (int r = 0; r < RR; ++r) if (row0 + r < K) qdst[row0 + r] = m[r];
        }
        mc_out = 1;
        return 0.0;
    }
    const long long th0 = wall_clock64();
    const int mc = K < D ? K : D;
    constexpr bool MOVE_R = CHI == 64;
    constexpr int RSL = CHI + 4;
    T *Rs = Rsc + p * CHI * RSL;
    if constexpr (MOVE_R) {
        for (int j = 0; j < mc; ++j) {
            T *vj = V + (p * CHI + j) * VL;
            // row j sits in the lanes gl == j / RR of every column, at register
            // j % RR (both uniform)
            const int jr = j % RR;
            const bool holds_j = (gl == j / RR);
            if (grp == j) {
                // the diagonal entry leaves the registers (this column is done
                // with them), so that the sum of squares is over the rows below
                // it alone: a tail far below the diagonal still gets its
                // reflector
                T x0 = holds_j ? m[jr] : (T)0;
                if (holds_j) m[jr] = (T)0;
                T s = rows_dot<T, RR>(m, m);
                s = group_sum(s, G);
                x0 = group_sum(x0, G);
                T tj = 0, sc = 0, be = x0;
                if (s != (T)0) {
                    const T nr2 = x0 * x0 + s;
                    if (std::is_same<T, float>::value && nr2 >= (T)4.7e-38f) {
                        const T nr = path_sqrt(nr2);
                        be = x0 >= 0 ? -nr : nr;
                        tj = (be - x0) * fast_rcp(be);
                        sc = fast_rcp(x0 - be);
                    } else {
                        const T nr = sqrt(nr2);
                        be = x0 >= 0 ? -nr : nr;
                        tj = (be - x0) / be;
                        sc = (T)1 / (x0 - be);
                    }
                }
#pragma unroll
                for (int r = 0; r < RR; ++r) vj[vrow0 + r] = m[r] * sc;
                if (holds_j) {
                    vj[vrow0 + jr] = (T)1;
                    Rs[j * RSL + j] = be;
                }
                if (gl == 0) tauv[p * CHI + j] = tj;
            }
            __syncthreads();
            if (grp > j) {
                const T tj = tauv[p * CHI + j];
                if (tj != (T)0) {
                    T vr[RR];
#pragma unroll
                    for (int r = 0; r < RR; ++r) vr[r] = vj[vrow0 + r];
                    T w = rows_dot<T, RR>(vr, m);
                    w = group_sum(w, G) * tj;
#pragma unroll
                    for (int r = 0; r < RR; ++r) m[r] -= vr[r] * w;
                }
                // row j of this column is final: it moves to Rs
                if (holds_j) {
                    Rs[grp * RSL + j] = m[jr];
                    m[jr] = (T)0;
                }
            }
        }
    } else {
        for (int j = 0; j < mc; ++j) {
            T *vj = V + (p * CHI + j) * VL;
            if (grp == j) {
                T x0 = 0, tail[RR];
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    const int row = row0 + r;
                    tail[r] = row > j ? m[r] : (T)0;
                    if (row == j) x0 = m[r];
                }
                T s = rows_dot<T, RR>(tail, tail);
                s = group_sum(s, G);
                x0 = group_sum(x0, G);
                T tj = 0, sc = 0, be = x0;
                if (s != (T)0) {
                    const T nr2 = x0 * x0 + s;
                    // float: the hardware's 1-ulp square root and reciprocals
                    // when the column is well inside the normal range (then
                    // |be| and |x0 - be| >= |be| are too: be has the opposite
                    // sign of x0); they read denormal inputs as zero
                    if (std::is_same<T, float>::value && nr2 >= (T)4.7e-38f) {
                        const T nr = path_sqrt(nr2);
                        be = x0 >= 0 ? -nr : nr;
                        tj = (be - x0) * fast_rcp(be);
                        sc = fast_rcp(x0 - be);
                    } else {
                        const T nr = sqrt(nr2);
                        be = x0 >= 0 ? -nr : nr;
                        tj = (be - x0) / be;
                        sc = (T)1 / (x0 - be);
                    }
                }
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    const int row = row0 + r;
                    vj[vrow0 + r] = row < j ? (T)0 : (row == j ? (T)1 : m[r] * sc);
                    m[r] = row < j ? m[r] : (row == j ? be : (T)0);
                }
                if (gl == 0) tauv[p * CHI + j] = tj;
            }
            __syncthreads();
            if (grp > j) {
                const T tj = tauv[p * CHI + j];
                if (tj != (T)0) {
                    T vr[RR];
#pragma unroll
                    for (int r = 0; r < RR; ++r) vr[r] = vj[vrow0 + r];
                    T w = rows_dot<T, RR>(vr, m);
                    w = group_sum(w, G) * tj;
#pragma unroll
                    for (int r = 0; r < RR; ++r) m[r] -= vr[r] * w;
                }
            }
        }
    }
    // explicit Q, backward accumulation: column k = grp
    T qv[RR];
#pragma unroll
    for (int r = 0; r < RR; ++r) qv[r] = (row0 + r == grp) ? (T)1 : (T)0;
    for (int j = mc - 1; j >= 0; --j) {
        const T tj = tauv[p * CHI + j];
        if (tj == (T)0 || grp < j) continue;
        const T *vj = V + (p * CHI + j) * VL;
        T vr[RR];
#pragma unroll
        for (int r = 0; r < RR; ++r) vr[r] = vj[vrow0 + r];
        T w = rows_dot<T, RR>(vr, qv);
        w = group_sum(w, G) * tj;
#pragma unroll
        for (int r = 0; r < RR; ++r) qv[r] -= vr[r] * w;
    }
    if (grp < mc) {
        T *qd = qdst + (size_t)p * 2 * chi * chi + grp;
#pragma unroll
        for (int r = 0; r < RR; ++r) if (row0 + r < K) qd[(size_t)(row0 + r) * chi] = qv[r];
    }
    cyc_hh += wall_clock64() - th0;
    // R^p (mc x D, upper trapezoidal), normalised jointly over both blocks
    // and scaled into Rh^p for the next site: column a by lam_h[(a's
    // sector) ^ p] of the next horizontal bond
    if constexpr (MOVE_R) {
        // this column's entries come back from Rs
#pragma unroll
        for (int r = 0; r < RR; ++r) m[r] = (row0 < CHI) ? Rs[grp * RSL + row0 + r] : (T)0;
    }
    double part = 0.0;
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int row = row0 + r;
        if (row < mc && row <= grp && grp < D) part += (double)m[r] * (double)m[r];
    }
    const double nu = sqrt(block_sum(part, red));
    const T inv = (T)(1.0 / nu);
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int row = row0 + r;
        const T lam = ((grp >= pn0) != (p == 1)) ? lnh1 : lnh0;
        if (row < CHI)
            R[rkey_base<CHI, RR>(p * CHI + row) ^ grp] = (row < mc && row <= grp && grp < D) ? (m[r] * inv) * lam : (T)0;
    }
    mc_out = mc;
    return log(nu);
}

template <typename T, int MAXB>
__device__ double qr_site_any(int chi, int c, int last, int K, int D, int Dp, int pa0, int m0, int m1, int pn0,
                              T lnh0, T lnh1, const T *C, T *R, T *V, T *tauv, T *Rsc, T *qdst, double *red,
                              int &mc, long long &cyc_hh) {
    if (chi <= 16) return qr_site<T, 16>(c, last, K, D, Dp, pa0, m0, m1, pn0, lnh0, lnh1, C, R, V, tauv, Rsc, qdst, chi, red, mc, cyc_hh);
    if constexpr (MAXB <= 32) {
        return qr_site<T, 32>(c, last, K, D, Dp, pa0, m0, m1, pn0, lnh0, lnh1, C, R, V, tauv, Rsc, qdst, chi, red, mc, cyc_hh);
    } else {
        if (chi <= 32) return qr_site<T, 32>(c, last, K, D, Dp, pa0, m0, m1, pn0, lnh0, lnh1, C, R, V, tauv, Rsc, qdst, chi, red, mc, cyc_hh);
        return qr_site<T, 64>(c, last, K, D, Dp, pa0, m0, m1, pn0, lnh0, lnh1, C, R, V, tauv, Rsc, qdst, chi, red, mc, cyc_hh);
    }
}

// The SVD centre T^p = [Q^p_0 X^p, Q^(1-p)_1 X^(1-p)] in float for chi <= 32
// on the matrix cores: wave 2p + s forms part s of block p as one 32 x 32 x 32
// product (v_mfma_f32_32x32x2f32, 16 steps of 2), rows, columns and the
// inner length masked to the blocks' sizes.  Operand layouts: lane l holds
// A[l % 32][k0 + l / 32] and B[k0 + l / 32][l % 32]; result register r of lane
// l is D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].  Qs: the Q slot [2][2chi][chi]
// (rows of block q: its sigma = 0 part, K_q rows, then its sigma = 1 part), X
// [2][chi][chi], Tm [2][bst] column-major with leading dimension ldt; K0, K1:
// the blocks' rows; r0, r1: the right bond's sectors (kr = r0 + r1 columns
// with data, n >= kr written); mn0, mn1: inner lengths.
typedef float floatx16 __attribute__((ext_vector_type(16)));
__device__ __forceinline__ void tform_mfma(const float *Qs, const float *X, float *Tm, int chi, int ldt, int bst,
                                           int K0, int K1, int r0, int r1, int mn0, int mn1, int n) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int p = w >> 1, s = w & 1;
    const int Kp = p ? K1 : K0;
    const int qb = s ? 1 - p : p;                   // block of Q and X
    const int rowoff = s ? (qb ? K1 : K0) : 0;      // sigma = 1 rows follow the K_qb sigma = 0 rows
    const int mn = qb ? mn1 : mn0;
    const int dp = p ? r1 : r0;
    const int c0 = s ? dp : 0;                      // first column of the part
    const int wdata = s ? (r0 + r1) - dp : dp;      // columns with data
    const int wout = s ? n - dp : dp;               // columns written (part 1 includes the padding)
    const float *Qb = Qs + qb * 2 * chi * chi + rowoff * chi;
    const float *Xb = X + qb * chi * chi;
    const int i = l & 31, kh = l >> 5;
    floatx16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < 32; k0 += 2) {
        const int j = k0 + kh;
        const float a = (i < Kp && j < mn) ? Qb[i * chi + j] : 0.f;
        const float b = (j < mn && i < wdata) ? Xb[j * chi + i] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    if (i < wout) {
        float *col = Tm + p * bst + (c0 + i) * ldt;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r >> 2) + 4 * kh + (r & 3);
            if (row < chi) col[row] = (row < Kp && i < wdata) ? acc[r] : 0.f;
        }
    }
}

// Eigenvalues (even, odd) of the normalised Boltzmann matrix of one bond:
// entries exp(beta*J*sx*sy - beta*|J|) are (1, x) or (x, 1) with
// x = exp(-2 beta |J|), so lam = (1 + x, +-(1 - x)), sign of J.
__device__ __forceinline__ void lam_of(double beta, float J, double &l0, double &l1) {
    const double a = 2.0 * beta * fabs((double)J);
    l0 = 1.0 + exp(-a);
    const double d = -expm1(-a);
    l1 = (J >= 0.0f) ? d : -d;
}

// Float64 redo of one site's truncation in a float build whose float32
// Jacobi did not converge on a block: the centres T^p = [Q^p_0 X^p,
// Q^(1-p)_1 X^(1-p)] are formed again in float64 from the same float32 Q
// slot q and carried X, both blocks go through the float64 Jacobi (the same
// routine, block and rotations in the global area fb, see
// fallback_doubles), and the rotated blocks, W and the singular values come
// back into the float32 arrays the truncation step reads (Tm, Wm: [2][bst],
// column-major, leading dimension ldt; nrm: [2][n]).  Called by all threads
// of the workgroup; the two blocks' float64 sweep counts go to iflag.
template <int MAXB>
__device__ void svd_redo_f64(double *fb, const float *q, const float *X, float *Tm, float *Wm, float *nrm,
                             int *iflag, int *jflag, int c, int L, int chi, int K0, int K1, int r0, int r1,
                             int mn0, int mn1, int n, int kr, int ldt, int bst) {
    const int tid = threadIdx.x, cc2 = chi * chi;
    double *Td = fb, *Wd = fb + 2 * bst, *prm = fb + 4 * bst, *nd = prm + 256;
    for (int e = tid; e < 2 * n * ldt; e += NT) Td[(e / (n * ldt)) * bst + e % (n * ldt)] = 0.0;
    __syncthreads();
    if (c == L - 1) {
        // the sweep's first centre: one column, rows of both QR sectors
        for (int e = tid; e < K0 + K1; e += NT) {
            const int p = e >= K0, k = p ? e - K0 : e;
            Td[p * bst + k] = (double)q[e];
        }
    } else {
        for (int e = tid; e < 2 * n * chi; e += NT) {
            const int p = e / (n * chi), k = (e / n) % chi, idx = e % n;
            const int Kp = p ? K1 : K0;
            if (k >= Kp || idx >= kr) continue;
            // column idx < d^p: (s = 0, m = idx) from Q^p's sigma = 0 rows;
            // else (s = 1) from Q^(1-p)'s sigma = 1 rows
            const int dp = p ? r1 : r0;
            const bool s1 = idx >= dp;
            const int qb = s1 ? 1 - p : p, xc = s1 ? idx - dp : idx;
            const int rowoff = s1 ? (qb == 0 ? K0 : K1) : 0;
            const int mcq = qb ? mn1 : mn0;
            const float *qr = q + qb * 2 * cc2 + (rowoff + k) * chi;
            const float *xr = X + qb * cc2 + xc;
            double acc = 0.0;
            for (int j = 0; j < mcq; ++j) acc += (double)qr[j] * (double)xr[j * chi];
            Td[p * bst + idx * ldt + k] = acc;
        }
    }
    __syncthreads();
    const int wv = tid >> 6, pb = wv & 1;
    const int sw = jacobi_block<double, MAXB, false>(Td + pb * bst, Wd + pb * bst, ldt, pb ? K1 : K0, n, chi,
                                                     tid & 63, wv >> 1, pb, prm, jflag, nd + pb * n, kr,
                                                     MAX_SWEEPS);
    if ((tid & 63) == 0 && wv < 2) iflag[wv] = sw;
    __syncthreads();
    for (int e = tid; e < 2 * n * ldt; e += NT) {
        const int p = e / (n * ldt), col = (e / ldt) % n, k = e % ldt;
        const int at = p * bst + col * ldt + k;
        Tm[at] = (float)Td[at];
        if (k < n) Wm[at] = (float)Wd[at];
    }
    for (int e = tid; e < 2 * n; e += NT) nrm[e] = (float)nd[e];
    __syncthreads();
}

template <typename T, typename S, int MAXB>
__device__ __forceinline__ void build_instance(int inst, const InstDesc *__restrict__ desc, unsigned char *__restrict__ ws,
                               const float *__restrict__ Jh_all, const float *__restrict__ Jv_all,
                               double *__restrict__ logz_out, int64_t *__restrict__ stats_out,
                               unsigned char *smem) {
    const long long t_begin = wall_clock64();
    const InstDesc d = desc[inst];
    const int L = d.L, chi = d.chi, tid = threadIdx.x;
    const double beta = d.beta;
    const double LN2 = 0.69314718055994530942;
    const T RS2 = (T)0.70710678118654752440;
    const float *jh = Jh_all + d.off_h;                  // [L][L-1]
    const float *jv = Jv_all + d.off_v;                  // [L-1][L]
    S *cache = reinterpret_cast<S *>(ws + d.cache_off);  // [L][L][2][chi][chi], spin basis
    T *qscr = reinterpret_cast<T *>(ws + d.qscr_off);    // [L][2][2chi][chi]
    T *prev = reinterpret_cast<T *>(ws + d.prev_off);    // [2][L][2][chi][chi], parity basis
    double *lsc = reinterpret_cast<double *>(ws + d.lsc_off);
    const int cc2 = chi * chi;
    const size_t site_sz = (size_t)2 * cc2;
    const size_t row_sz = (size_t)L * site_sz;
    const int CB = chi <= 16 ? 16 : (chi <= 32 ? 32 : 64);   // compiled width holding chi
    // per-site loops walk MAXB-wide index grids with shifts and masks (a
    // division by a run-time width costs a dozen instructions or more)
    constexpr int LB = MAXB <= 16 ? 4 : (MAXB <= 32 ? 5 : 6), MM = MAXB - 1;
    const int ldt = chi + 1;          // leading dim of Tm / Wm blocks (column-major)
    const int bst = (chi + 1) * ldt;  // one Tm / Wm block

    // ---- shared memory layout (see build_lds_bytes) ----------------------
    const int VLb = CB <= 16 ? vrow_len<16>() : (CB <= 32 ? vrow_len<32>() : vrow_len<64>());
    const int regA_sz = 3 * CB * CB + 2 * CB * VLb;                // QR phase
    // for chi <= 32 the SVD phase also holds the next site's Q slot, staged
    // by waves 2 and 3 while waves 0 and 1 run the Jacobi
    const bool qstage = CB <= 32;
    const int regS_sz = 4 * bst + 2 * cc2 + (qstage ? 4 * cc2 : 0);
    T *reg = reinterpret_cast<T *>(smem);
    T *C = reg;                       // [CB][CB]
    T *R = reg + CB * CB;             // [2][CB][CB]
    T *Vh = reg + 3 * CB * CB;        // [2][CB][VLb] Householder vectors
    T *Tm = reg;                      // [2][chi+1][ldt]
    T *Wm = reg + 2 * bst;            // [2][chi+1][ldt]
    T *X = reg + 4 * bst;             // [2][chi][chi]
    T *Qst = X + 2 * cc2;             // [2][2chi][chi] staged Q slot (chi <= 32)
    T *tail = reg + (regA_sz > regS_sz ? regA_sz : regS_sz);
    T *tau = tail;                    // [2][CB]
    T *nrm = tau + 2 * CB;            // [2][chi+2]
    T *jprm = nrm + 2 * (chi + 2);    // [2][2][CB/2][2] Jacobi rotations in flight
    double *red = reinterpret_cast<double *>(
        (reinterpret_cast<uintptr_t>(jprm + 4 * CB) + 7) & ~(uintptr_t)7);
    double *uvec = red + NT / 64;     // [2][64] row-0 contraction vector
    double *scal = uvec + 128;        // [8]
    int *colof = reinterpret_cast<int *>(scal + 8);   // [2chi+4] kept column of new bond slot
    int *rankv = colof + 2 * chi + 4;                 // [2chi+4]
    int *iflag = rankv + 2 * chi + 4;                 // [4]
    int *jflag = iflag + 4;                           // [2] Jacobi: block still rotating
    unsigned char *dsec = reinterpret_cast<unsigned char *>(jflag + 2);  // [L+1][2] bond sectors
    unsigned char *mq = dsec + 2 * (L + 1);                            // [L+1][2] QR bond sectors
    // the current row's couplings (vertical, then horizontal)
    float *jrow = reinterpret_cast<float *>((reinterpret_cast<uintptr_t>(mq + 2 * (L + 1)) + 3) & ~(uintptr_t)3);

    int total_sweeps = 0, maxsweep_hits = 0, redo_f64 = 0;
    // the float32 Jacobi's sweep limit (one sweep when the float64 redo is
    // forced, see TNMC_FORCE_F64_FALLBACK)
    constexpr bool FLOAT_BUILD = std::is_same<T, float>::value;
    const int jac_limit = (FLOAT_BUILD && (d.flags & 2)) ? 1 : MAX_SWEEPS;
    long long cyc_qr = 0, cyc_svd = 0, cyc_jac = 0, cyc_hh = 0;   // wall-clock ticks per phase

    // write one parity-basis site (from a generator) to the ping-pong buffer
    // and its spin-basis form to the cache
    // Row orientation.  With alternating sweeps (flag bit 0 of the
    // descriptor) every second row is compressed mirrored: its "virtual"
    // column v is the lattice column L-1-v and the left and right bonds of a
    // site trade places; the QR sweep then runs right to left and the SVD
    // sweep left to right on the lattice.  A row is kept in the ping-pong
    // buffer in its own orientation; the cache is always written in lattice
    // order.  The bottom row is not mirrored.
    const bool alternate = (d.flags & 1) != 0;
    auto mirrored = [&](int r) { return alternate && r <= L - 2 && ((L - 2 - r) & 1); };
    auto put_site = [&](int r, int c, int a, int b, T e0, T e1) {
        const bool mr = mirrored(r);
        T *ps = prev + (size_t)(r & 1) * row_sz + (size_t)c * site_sz;
        S *cs = cache + (size_t)r * row_sz + (size_t)(mr ? L - 1 - c : c) * site_sz;
        const int ce = mr ? b * chi + a : a * chi + b;
        ps[a * chi + b] = e0;
        ps[cc2 + a * chi + b] = e1;
        cs[ce] = store_as<S, T>((e0 + e1) * RS2);
        cs[cc2 + ce] = store_as<S, T>((e0 - e1) * RS2);
    };

    // ---- bottom row (row L-1): every inner bond is (1 even, 1 odd) ---------
    {
        const int r = L - 1;
        for (size_t e = tid; e < (size_t)L * cc2; e += NT) {
            const int c = (int)(e / cc2), a = (int)((e / chi) % chi), b = (int)(e % chi);
            T v0 = 0, v1 = 0;   // physical parity 0 / 1
            if (c == 0) {
                if (a == 0 && b == 0) v0 = 1;
                if (a == 0 && b == 1) v1 = 1;
            } else if (a < 2) {
                double l0, l1;
                lam_of(beta, jh[(size_t)r * (L - 1) + (c - 1)], l0, l1);
                const T lh = (T)(a == 0 ? l0 : l1);
                if (c == L - 1) {
                    if (b == 0) { if (a == 0) v0 = lh; else v1 = lh; }
                } else if (b < 2) {
                    // parity of (l, s, t) even: s = l ^ t
                    if ((a ^ b) == 0) v0 = lh; else v1 = lh;
                }
            }
            put_site(r, c, a, b, v0, v1);
        }
        for (int i = tid; i <= L; i += NT) {
            dsec[2 * i] = 1;
            dsec[2 * i + 1] = (i == 0 || i == L) ? 0 : 1;
        }
        double part = 0.0;
        for (int c = tid; c < L - 1; c += NT) part += beta * fabs((double)jh[(size_t)r * (L - 1) + c]);
        const double ls = block_sum(part, red) - (double)(L - 2) * 0.5 * LN2;
        if (tid == 0) lsc[r] = ls;
        __syncthreads();
    }

    double logz_tail = 0.0;   // (thread 0) ln of the row-0 contraction

    for (int r = L - 2; r >= 0; --r) {
        const T *orow = prev + (size_t)((r + 1) & 1) * row_sz;
        // this row in its own orientation; the previous row read mirrored
        // when the two orientations differ (old bond i of this row's view
        // is the previous row's bond L - i, a site's bonds trade places)
        const bool mir = mirrored(r), rd = mir != mirrored(r + 1);

        double part = 0.0;
        for (int c = tid; c < L; c += NT) {
            const float v = jv[(size_t)r * L + (mir ? L - 1 - c : c)];
            jrow[c] = v;
            part += beta * fabs((double)v);
            if (c < L - 1) {
                const float h = jh[(size_t)r * (L - 1) + (mir ? L - 2 - c : c)];
                jrow[L + c] = h;
                part += beta * fabs((double)h);
            }
        }
        double ls = block_sum(part, red) - (double)(L - 1) * LN2;   // (its barriers publish jrow)

        // ================= QR sweep, left to right =========================
        const long long tq0 = wall_clock64();
        if (tid == 0) { mq[0] = 1; mq[1] = 0; }
        __syncthreads();
        // The previous row's site c + 1 is read into registers while site c
        // is factored (chi <= 32 kernels; the chi = 64 kernel reads each
        // site in place, all loads before the stores).
        constexpr int CPT = MAXB <= 32 ? MAXB * MAXB / NT : 1;
        T pre[CPT];
        auto ob = [&](int i) { return rd ? L - i : i; };                    // old bond index
        auto fetch_site = [&](int cs) {
            const int pa0 = dsec[2 * ob(cs)], Dp = pa0 + dsec[2 * ob(cs) + 1];
            const int pb0 = dsec[2 * ob(cs + 1)], D = pb0 + dsec[2 * ob(cs + 1) + 1];
            const T *os = orow + (size_t)(rd ? L - 1 - cs : cs) * site_sz;
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                const int e = tid + i * NT;
                const int a = e >> LB, b = e & MM;
                const int n = (a >= pa0) ^ (b >= pb0);
                pre[i] = (a < Dp && b < D) ? os[n * cc2 + (rd ? b * chi + a : a * chi + b)] : (T)0;
            }
        };
        if constexpr (MAXB <= 32) fetch_site(0);
        for (int c = 0; c < L; ++c) {
            const int pa0 = dsec[2 * ob(c)], Dp = pa0 + dsec[2 * ob(c) + 1];             // old left bond
            const int pb0 = dsec[2 * ob(c + 1)], D = pb0 + dsec[2 * ob(c + 1) + 1];      // old right bond
            const int m0 = mq[2 * c], m1 = mq[2 * c + 1];
            const int K = m0 + m1;
            double lv0, lv1;
            lam_of(beta, jrow[c], lv0, lv1);
            // (a) C[a][b] = lam_v[pa^pb] * A_old[pa^pb][a][b]
            if constexpr (MAXB <= 32) {
#pragma unroll
                for (int i = 0; i < CPT; ++i) {
                    const int e = tid + i * NT;
                    const int a = e >> LB, b = e & MM;
                    if (a < Dp && b < D) {
                        const int n = (a >= pa0) ^ (b >= pb0);
                        C[a * CB + b] = (T)(n ? lv1 : lv0) * pre[i];
                    }
                }
                if (c + 1 < L) fetch_site(c + 1);
            } else {
                const T *os = orow + (size_t)(rd ? L - 1 - c : c) * site_sz;
                constexpr int CPW = MAXB * MAXB / NT;
                T v[CPW];
#pragma unroll
                for (int i = 0; i < CPW; ++i) {
                    const int e = tid + i * NT;
                    const int a = e >> LB, b = e & MM;
                    const int n = (a >= pa0) ^ (b >= pb0);
                    v[i] = (a < Dp && b < D) ? os[n * cc2 + (rd ? b * chi + a : a * chi + b)] : (T)0;
                }
#pragma unroll
                for (int i = 0; i < CPW; ++i) {
                    const int e = tid + i * NT;
                    const int a = e >> LB, b = e & MM;
                    if (a < Dp && b < D) {
                        const int n = (a >= pa0) ^ (b >= pb0);
                        C[a * CB + b] = (T)(n ? lv1 : lv0) * v[i];
                    }
                }
            }
            // the next horizontal bond's eigenvalues: the carried R is scaled
            // by them where it is written
            double ln0 = 1.0, ln1 = 1.0;
            if (c + 1 < L) lam_of(beta, jrow[L + c], ln0, ln1);
            __syncthreads();
            // (b)-(f) in registers: M^p, Householder QR, explicit Q to scratch
            // slot c, normalised and scaled R carried right
            int mc = 1;
            // (the chi = 64 form's R columns: the float64 redo area after the
            // Q slots, which only the SVD sweep otherwise uses)
            ls += qr_site_any<T, MAXB>(chi, c, c == L - 1, K, D, Dp, pa0, m0, m1, pb0, (T)ln0, (T)ln1, C, R, Vh,
                                       tau, qscr + (size_t)L * 4 * cc2, qscr + (size_t)c * 4 * cc2, red, mc,
                                       cyc_hh);
            if (c == L - 1) {
                if (tid == 0) { mq[2 * L] = 1; mq[2 * L + 1] = 0; }
                __syncthreads();
                break;
            }
            if (tid == 0) { mq[2 * (c + 1)] = (unsigned char)mc; mq[2 * (c + 1) + 1] = (unsigned char)mc; }
            __syncthreads();
        }

        // ================= SVD sweep, right to left ========================
        const long long ts0 = wall_clock64();
        cyc_qr += ts0 - tq0;
        if (tid == 0) { dsec[2 * L] = 1; dsec[2 * L + 1] = 0; uvec[0] = 1.0; }
        __syncthreads();
        double ulog = 0.0;
        for (int c = L - 1; c >= 0; --c) {
            const int r0 = dsec[2 * (c + 1)], r1 = dsec[2 * (c + 1) + 1];   // right bond sectors
            const int kr = r0 + r1;
            const int K0 = mq[2 * c], K1 = mq[2 * c + 1];                  // left (QR) bond sectors
            const T *q = qscr + (size_t)c * 4 * cc2;
            if (c == 0) {
                // site 0: one row (even), columns (s=0, m even) and (s=1, m odd)
                double sp = 0.0;
                auto row0 = [&](const T *qsrc) {
                    for (int m = tid; m < kr; m += NT) {
                        const int p = (m >= r0);                    // sector of m; physical s = p
                        const int mm = p ? m - r0 : m;
                        const int mcq = mq[2 * (c + 1) + p];        // QR bond c|c+1 sector p
                        const T *qrow = qsrc + p * 2 * cc2;         // Q^p, sigma = p part starts at row 0
                        const T *xc = X + p * cc2 + mm;
                        T acc = 0, a1 = 0;
                        int j = 0;
                        for (; j + 1 < mcq; j += 2) {
                            acc += qrow[j] * xc[j * chi];
                            a1 += qrow[j + 1] * xc[(j + 1) * chi];
                        }
                        if (j < mcq) acc += qrow[j] * xc[j * chi];
                        acc += a1;
                        nrm[m] = acc;
                        sp += (double)acc * (double)acc;
                    }
                };
                if (qstage) row0(Qst); else row0(q);
                const double n0 = sqrt(block_sum(sp, red));
                ls += log(n0);
                const T inv = (T)(1.0 / n0);
                for (int e = tid; e < cc2; e += NT) {
                    const int a = e / chi, m = e % chi;
                    T v0 = 0, v1 = 0;
                    if (a == 0 && m < kr) { if (m < r0) v0 = nrm[m] * inv; else v1 = nrm[m] * inv; }
                    put_site(r, 0, a, m, v0, v1);
                }
                if (r == 0 && tid == 0) {
                    double tot = 0.0;
                    for (int m = 0; m < r0; ++m) tot += (double)nrm[m] * (double)inv * uvec[m];
                    logz_tail = ulog + log(tot) + (double)L * 0.5 * LN2;
                }
                if (tid == 0) { dsec[0] = 1; dsec[1] = 0; }
                __syncthreads();
                break;
            }
            const int n = (kr + 1) & ~1;     // columns per block, padded even
            // T^p[k][idx]: idx < d^p -> (s=0, m = off_p + idx); else (s=1, m = off_(1-p) + idx - d^p)
            if (c == L - 1) {
                for (int e = tid; e < 2 * n * ldt; e += NT) Tm[(e / (n * ldt)) * bst + e % (n * ldt)] = 0;
                __syncthreads();
                for (int e = tid; e < K0 + K1; e += NT) {
                    const int p = e >= K0, k = p ? e - K0 : e;
                    Tm[p * bst + k] = q[e];
                }
            } else {
                const int mn0 = mq[2 * (c + 1)], mn1 = mq[2 * (c + 1) + 1];   // QR bond c|c+1 sectors
                // idx fastest: neighbouring threads share rows of Q
                auto tform = [&](const T *qsrc) {
                for (int e = tid; e < 2 * n * chi; e += NT) {
                    const int p = e / (n * chi), k = (e / n) % chi, idx = e % n;
                    const int Kp = p ? K1 : K0;
                    T acc = 0;
                    if (k < Kp && idx < kr) {
                        const int dp = p ? r1 : r0;
                        // rows of Q^qb: sigma=0 part (K_qb rows) first, then sigma=1 part
                        const bool s1 = idx >= dp;
                        const int qb = s1 ? 1 - p : p, xb = qb, xc = s1 ? idx - dp : idx;
                        const int rowoff = s1 ? (qb == 0 ? K0 : K1) : 0;
                        const int mcq = xb ? mn1 : mn0;
                        const T *qr = qsrc + qb * 2 * cc2 + (rowoff + k) * chi;
                        const T *xr = X + xb * cc2 + xc;
                        // four partial sums: independent chains hide the LDS latency
                        T a1 = 0, a2 = 0, a3 = 0;
                        int j = 0;
                        for (; j + 3 < mcq; j += 4) {
                            acc += qr[j] * xr[j * chi];
                            a1 += qr[j + 1] * xr[(j + 1) * chi];
                            a2 += qr[j + 2] * xr[(j + 2) * chi];
                            a3 += qr[j + 3] * xr[(j + 3) * chi];
                        }
                        for (; j < mcq; ++j) acc += qr[j] * xr[j * chi];
                        acc = (acc + a1) + (a2 + a3);
                    }
                    Tm[p * bst + idx * ldt + k] = acc;
                }
                };
                // (the chi <= 32 kernels only: in the chi = 64 kernel the
                // product's operands push the register allocation into spills)
                if constexpr (std::is_same<T, float>::value && MAXB <= 32) {
                    if (qstage) tform_mfma(Qst, X, Tm, chi, ldt, bst, K0, K1, r0, r1, mn0, mn1, n);
                    else tform(q);
                } else {
                    if (qstage) tform(Qst); else tform(q);
                }
            }
            __syncthreads();
            {
                const long long t0 = wall_clock64();
                // waves 0, 1: blocks 0, 1; waves 2, 3: their rotations
                const int wv = tid >> 6, pb = wv & 1;
                if (qstage && wv >= 2) {
                    // first: the next site's Q slot into shared memory
                    const T *src = qscr + (size_t)(c - 1) * 4 * cc2;
                    for (int e = tid - 128; e < 4 * cc2; e += 128) Qst[e] = src[e];
                }
                const int sw = jacobi_block<T, MAXB>(Tm + pb * bst, Wm + pb * bst, ldt, pb ? K1 : K0, n, chi,
                                                     tid & 63, wv >> 1, pb, jprm, jflag,
                                                     nrm + pb * n, kr, jac_limit);
                if ((tid & 63) == 0 && wv < 2) iflag[wv] = sw;
                __syncthreads();
                const int swm = iflag[0] > iflag[1] ? iflag[0] : iflag[1];
                total_sweeps += swm;
                if constexpr (FLOAT_BUILD) {
                    // orthogonality not reached in float32 (the last sweep
                    // still rotated): redo the site's truncation in float64
                    if (swm >= jac_limit) {
                        double *fb = reinterpret_cast<double *>(qscr + (size_t)L * 4 * cc2);
                        svd_redo_f64<MAXB>(fb, q, X, Tm, Wm, nrm, iflag, jflag, c, L, chi, K0, K1, r0, r1,
                                           mq[2 * (c + 1)], mq[2 * (c + 1) + 1], n, kr, ldt, bst);
                        total_sweeps += iflag[0] > iflag[1] ? iflag[0] : iflag[1];
                        ++redo_f64;
                    }
                }
                maxsweep_hits += (iflag[0] >= MAX_SWEEPS) + (iflag[1] >= MAX_SWEEPS);
                cyc_jac += wall_clock64() - t0;
            }
            // singular values of both blocks (padding columns and empty
            // blocks excluded); for chi <= 32 the Jacobi wrote them
            if (CB > 32) {
                for (int e = tid; e < 2 * n; e += NT) {
                    const int p = e / n, col = e % n, Kp = p ? K1 : K0;
                    const T *cp = Tm + p * bst + col * ldt;
                    T s2 = 0, s3 = 0;
                    if (col < kr) {
                        int k = 0;
                        for (; k + 1 < Kp; k += 2) { s2 += cp[k] * cp[k]; s3 += cp[k + 1] * cp[k + 1]; }
                        if (k < Kp) s2 += cp[k] * cp[k];
                    }
                    nrm[e] = (col < kr && Kp > 0) ? sqrt(s2 + s3) : (T)-1;
                }
                __syncthreads();
            }
            int kk = chi < K0 + K1 ? chi : K0 + K1;
            if (2 * kr < kk) kk = 2 * kr;
            // rank of every column over both blocks (ties by index); 2n is a
            // multiple of 4
            for (int e = tid; e < 2 * n; e += NT) {
                const T v = nrm[e];
                int q0 = 0, q1 = 0, q2 = 0, q3 = 0;
#pragma unroll 4
                for (int o = 0; o < 2 * n; o += 4) {
                    const T w0 = nrm[o], w1 = nrm[o + 1], w2 = nrm[o + 2], w3 = nrm[o + 3];
                    q0 += (w0 > v) || (w0 == v && o < e);
                    q1 += (w1 > v) || (w1 == v && o + 1 < e);
                    q2 += (w2 > v) || (w2 == v && o + 2 < e);
                    q3 += (w3 > v) || (w3 == v && o + 3 < e);
                }
                rankv[e] = (v >= (T)0) ? (q0 + q1) + (q2 + q3) : 1 << 20;
            }
            __syncthreads();
            // new left bond: kept columns of block 0 (by rank), then of block 1
            // (2n <= 128 < NT: one column per thread)
            const int s0 = __syncthreads_count(tid < n && rankv[tid] < kk);
            for (int e = tid; e < 2 * n; e += NT) {
                if (rankv[e] < kk) {
                    const int p = e / n, re = rankv[e];
                    const int *rb = rankv + p * n;
                    int q0 = 0, q1 = 0;
#pragma unroll 4
                    for (int o = 0; o < n; o += 2) { q0 += rb[o] < re; q1 += rb[o + 1] < re; }
                    colof[(p ? s0 : 0) + q0 + q1] = (p << 8) | (e - p * n);   // block, column
                }
            }
            double kp = 0.0;
            for (int e = tid; e < 2 * n; e += NT) if (rankv[e] < kk) { const double v = (double)nrm[e]; kp += v * v; }
            const double nk = sqrt(block_sum(kp, red));   // (block_sum syncs)
            ls += log(nk);
            // new site c (right-canonical): slot a <- column colof[a]
            for (int e = tid; e < MAXB * MAXB; e += NT) {
                const int a = e >> LB, m = e & MM;
                if (a >= chi || m >= chi) continue;
                T v0 = 0, v1 = 0;
                if (a < kk && m < kr) {
                    const int ce = colof[a], p = ce >> 8, col = ce & 255;
                    const int pm = m >= r0, mm = pm ? m - r0 : m;
                    const int dp = p ? r1 : r0;
                    // physical parity s = p ^ pm; row of W^p for (s, m)
                    const int s = p ^ pm;
                    const int row = (s == 0) ? mm : dp + mm;
                    const T w = Wm[p * bst + col * ldt + row];
                    if (s == 0) v0 = w; else v1 = w;
                }
                put_site(r, c, a, m, v0, v1);
            }
            if (r == 0) {
                // row-0 contraction from the right on the even physical component
                double *u = uvec, *un = uvec + 64;
                for (int a = tid; a < kk; a += NT) {
                    const int ce = colof[a], p = ce >> 8, col = ce & 255;
                    double acc = 0.0;
                    // s = 0 entries: m in sector p, row = index within the sector
                    const int dp = p ? r1 : r0, off = p ? r0 : 0;
                    for (int mm = 0; mm < dp; ++mm) acc += (double)Wm[p * bst + col * ldt + mm] * u[off + mm];
                    un[a] = acc;
                }
                __syncthreads();
                if (tid == 0) {
                    double mx = 0.0;
                    for (int a = 0; a < kk; ++a) mx = fmax(mx, fabs(un[a]));
                    scal[2] = mx > 0.0 ? mx : 1.0;
                }
                __syncthreads();
                const double mx = scal[2];
                for (int a = tid; a < kk; a += NT) u[a] = un[a] / mx;
                ulog += log(mx);
            }
            __syncthreads();
            // X^p (K_p x d'^p) = U S / ||S_kept|| for the next site
            const T inv = (T)(1.0 / nk);
            for (int e = tid; e < 2 * MAXB * MAXB; e += NT) {
                const int p = e >> (2 * LB), k = (e >> LB) & MM, j = e & MM;
                const int Kp = p ? K1 : K0, dp = p ? kk - s0 : s0;
                if (k < Kp && j < dp) {
                    const int ce = colof[(p ? s0 : 0) + j];
                    X[p * cc2 + k * chi + j] = Tm[p * bst + (ce & 255) * ldt + k] * inv;
                }
            }
            if (tid == 0) { dsec[2 * c] = (unsigned char)s0; dsec[2 * c + 1] = (unsigned char)(kk - s0); }
            __syncthreads();
        }
        cyc_svd += wall_clock64() - ts0;
        if (tid == 0) lsc[r] = ls;
        __syncthreads();
    }
    if (tid == 0) {
        double lz = logz_tail;
        int nonfinite = 0;
        for (int r = 0; r < L; ++r) { lz += lsc[r]; nonfinite += !isfinite(lsc[r]); }
        if (logz_out) logz_out[inst] = lz;
        if (stats_out) {
            int64_t *so = stats_out + STATS_PER_INST * inst;
            so[STAT_MAXSWEEP] = maxsweep_hits;
            so[STAT_NONFINITE] = nonfinite;
            so[STAT_LOGZ_UNDEFINED] = nonfinite == 0 && !isfinite(lz);
            so[STAT_FALLBACK] = redo_f64;
            // the rest of the record (the row-pipelined build's hand-over
            // flag, spare slots) is defined as zero here
            for (int k = STAT_FALLBACK + 1; k < STATS_PER_INST; ++k) so[k] = 0;
            so[0] = total_sweeps;
            so[1] = cyc_qr;
            so[2] = cyc_svd;
            so[3] = cyc_jac;
            so[4] = t_begin;
            so[5] = wall_clock64();
            so[7] = cyc_hh;
        }
    }
}

// Shared-memory bytes the build needs for bond dimension chi and side L.
size_t build_lds_bytes(int chi, int L, size_t tsize);

}  // namespace tnmc

// Boundary-MPS cache build (arXiv 2509.19006, section 2.2 / Fig. 2 and
// section 3.2): starting from the bottom row, apply each row's transfer MPO
// to the boundary MPS and truncate back to bond dimension chi.
//
// One workgroup (256 threads, 4 waves) owns one instance and walks its rows
// bottom to top.  Per row:
//   * apply   -- the MPO of a row is built from copy tensors (Eq. 8) and
//                Boltzmann matrices (Eq. 7).  Its copy-tensor structure means
//                that site c of MPO x MPS, for physical spin s, is
//                Bh(c-1)[l,s] * delta(t,s) * C_s with
//                C_s = sum_n Bv(c)[s,n] A_old[:,n,:]
//                (the new right bond carries the spin t = s).  The tensor is
//                never formed densely.
//   * QR sweep, left to right -- because the new right bond carries s, the
//                matrix R * A'_c splits into two blocks M_s (one per s), each
//                (2 m_prev) x D_old; each gets its own Householder QR.
//   * SVD sweep, right to left -- center matrix T = [Q_0 X_0, Q_1 X_1]
//                (K x 2k); one-sided (Hestenes) Jacobi with a round-robin
//                pair order; keep the chi largest singular values, the right
//                factor V^T becomes the site, U*S moves to the left.
// All norms removed along the way go to a float64 log-scale per row, so that
// ln Z = sum_r logscale[r] + ln(row-0 MPS with every spin summed).
//
// Template T is the arithmetic type (double or float); S the cache storage
// type (double, float, bfloat16 or half).  When S != T the previous row is
// also kept in a float ping-pong buffer so the build never reads rounded
// values back.
#include <type_traits>

#include "device.hpp"

namespace tnmc {

constexpr int NT = 256;
constexpr int MAX_SWEEPS = 40;

template <typename T> __device__ __forceinline__ T shfl_xor_t(T v, int m, int w) {
    return __shfl_xor(v, m, w);
}

// Sum over groups of G consecutive lanes (G a power of two <= 64).
template <typename T> __device__ __forceinline__ T group_sum(T v, int G) {
    for (int m = G >> 1; m > 0; m >>= 1) v += shfl_xor_t(v, m, 64);
    return v;
}

__device__ __forceinline__ int pow2_floor(int x) {
    int p = 1;
    while ((p << 1) <= x) p <<= 1;
    return p;
}

// Workgroup sum of one double (all threads get the result).
__device__ double block_sum(double v, double *red) {
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
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
// 1/sqrt(x) from the hardware estimate refined by one Newton step.
__device__ __forceinline__ double rsqrt_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return y * (1.5 - 0.5 * x * y * y);
}
__device__ __forceinline__ float rsqrt_nr(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    return y * (1.5f - 0.5f * x * y * y);
}

// One-sided (Hestenes) Jacobi on the n columns (length K) of Tm,
// accumulating the rotations in Wm (n x n); both column-major with leading
// dimension ld.  cn2[n] holds squared column norms: recomputed at the start
// of every sweep and carried through each rotation exactly
// (a' = a - t*g, b' = b + t*g), so a pair needs a single reduction.  Pairs
// whose smaller column is below sqrt(n)*eps*||T||_F are left alone: such
// columns are rounding noise and a relative orthogonality test on them never
// settles.  Returns the number of sweeps.
template <typename T>
__device__ int jacobi(T *Tm, T *Wm, int ld, int K, int n, T *cn2, int *flag) {
    const int tid = threadIdx.x;
    const int npairs = n >> 1;
    int G = pow2_floor(NT / npairs);
    if (G > 64) G = 64;
    const int g = tid / G, lane = tid % G;
    const T tol = (T)2 * Eps<T>::v * sqrt((T)K);
    T small = 0;
    int sweeps = 0;
    for (int sw = 0; sw < MAX_SWEEPS; ++sw) {
        for (int col = tid; col < n; col += NT) {
            T s2 = 0;
            for (int r = 0; r < K; ++r) { const T v = Tm[col * ld + r]; s2 += v * v; }
            cn2[col] = s2;
        }
        if (tid == 0) *flag = 0;
        __syncthreads();
        if (sw == 0) {
            T fro = 0;
            for (int col = 0; col < n; ++col) fro += cn2[col];
            small = fro * Eps<T>::v * Eps<T>::v * (T)n;
        }
        for (int t = 0; t < n - 1; ++t) {
            if (g < npairs) {
                const int i = seat(g, t, n), j = seat(n - 1 - g, t, n);
                const T a = cn2[i], b = cn2[j];
                if (a > small && b > small) {
                    T *ci = Tm + i * ld, *cj = Tm + j * ld;
                    T c = 0;
                    for (int r = lane; r < K; r += G) c += ci[r] * cj[r];
                    c = group_sum(c, G);
                    if (fabs(c) > tol * sqrt(a * b)) {
                        const T zeta = (b - a) * fast_rcp(2 * c);
                        T tt;
                        if (fabs(zeta) > (T)1e15) tt = (T)0.5 * fast_rcp(zeta);
                        else tt = (zeta >= 0 ? (T)1 : (T)-1) * fast_rcp(fabs(zeta) + sqrt((T)1 + zeta * zeta));
                        const T cs = rsqrt_nr((T)1 + tt * tt), sn = cs * tt;
                        for (int r = lane; r < K; r += G) {
                            const T x = ci[r], y = cj[r];
                            ci[r] = cs * x - sn * y;
                            cj[r] = sn * x + cs * y;
                        }
                        T *wi = Wm + i * ld, *wj = Wm + j * ld;
                        for (int r = lane; r < n; r += G) {
                            const T x = wi[r], y = wj[r];
                            wi[r] = cs * x - sn * y;
                            wj[r] = sn * x + cs * y;
                        }
                        if (lane == 0) {
                            cn2[i] = a - tt * c;
                            cn2[j] = b + tt * c;
                            *flag = 1;
                        }
                    }
                }
            }
            __syncthreads();
        }
        ++sweeps;
        const int more = *flag;
        __syncthreads();
        if (!more) break;
    }
    return sweeps;
}

template <typename T, typename S>
__global__ void __launch_bounds__(NT)
k_build(const InstDesc *__restrict__ desc, unsigned char *__restrict__ ws,
        const float *__restrict__ Jh_all, const float *__restrict__ Jv_all,
        double *__restrict__ logz_out, int64_t *__restrict__ stats_out) {
    constexpr bool kPingPong = !std::is_same<T, S>::value;
    const int inst = blockIdx.x;
    const InstDesc d = desc[inst];
    const int L = d.L, chi = d.chi, tid = threadIdx.x;
    const double beta = d.beta;
    const float *jh = Jh_all + d.off_h;                  // [L][L-1]
    const float *jv = Jv_all + d.off_v;                  // [L-1][L]
    S *cache = reinterpret_cast<S *>(ws + d.cache_off);  // [L][L][2][chi][chi]
    T *qscr = reinterpret_cast<T *>(ws + d.qscr_off);    // [L][2][2chi][chi]
    T *prev = kPingPong ? reinterpret_cast<T *>(ws + d.prev_off) : nullptr;  // [2][L][2][chi][chi]
    double *lsc = reinterpret_cast<double *>(ws + d.lsc_off);
    const size_t site_sz = (size_t)2 * chi * chi;
    const size_t row_sz = (size_t)L * site_sz;
    const int ldm = chi + 1;          // leading dim of M blocks
    const int ldt = 2 * chi + 1;      // leading dim of Tm / Wm (column-major)

    // ---- shared memory layout -------------------------------------------
    extern __shared__ __align__(16) unsigned char smem[];
    T *regA = reinterpret_cast<T *>(smem);                      // 4 chi^2
    T *regB = regA + 4 * chi * chi;                             // 2*2chi*(chi+1)
    T *Tm = regA;                                               // SVD phase: 2chi x ldt
    T *Wm = regA + 2 * chi * ldt;                               //            2chi x ldt
    T *tail = regA + (size_t)4 * chi * ldt;                     // >= 8chi^2+4chi
    T *tau = tail;                                              // [2][chi]
    T *nrm = tau + 2 * chi;                                     // [2chi]
    double *red = reinterpret_cast<double *>(nrm + 2 * chi);    // [NT/64]
    double *uvec = red + NT / 64;                               // [2][64] logZ vector
    double *scal = uvec + 128;                                  // [4]
    int *perm = reinterpret_cast<int *>(scal + 4);              // [2chi]
    int *iflag = perm + 2 * chi;                                // [4]
    unsigned char *bond = reinterpret_cast<unsigned char *>(iflag + 4);  // [L+1]
    unsigned char *mq = bond + (L + 1);                                // [L]

    T *C = regA;                     // [2][chi][chi]
    T *R = regA + 2 * chi * chi;     // [2][chi][chi]
    T *Mb = regB;                    // [2][2chi][ldm]
    T *Qb = regA;                    // [2][2chi][chi] (reuses C and R)
    T *X = Wm;                       // [2chi][chi] lives in Wm between sites

    int total_sweeps = 0;
    long long cyc_qr = 0, cyc_svd = 0, cyc_jac = 0;   // wall-clock ticks per phase

    // ---- bottom row (row L-1): bond dimension 2, bonds carry the spin ------
    {
        const int r = L - 1;
        S *crow = cache + (size_t)r * row_sz;
        T *prow = kPingPong ? prev + (size_t)(r & 1) * row_sz : nullptr;
        for (size_t e = tid; e < row_sz; e += NT) {
            const int c = (int)(e / site_sz);
            const int rem = (int)(e % site_sz);
            const int s = rem / (chi * chi), a = (rem / chi) % chi, b = rem % chi;
            double v = 0.0;
            if (c == 0) {
                v = (a == 0 && b == s) ? 1.0 : 0.0;
            } else {
                double same, diff;
                boltz(beta, jh[(size_t)r * (L - 1) + (c - 1)], same, diff);
                const double bl = (a == s) ? same : diff;       // Bh(c-1)[l=a, s]
                if (a < 2) {
                    if (c == L - 1) v = (b == 0) ? bl : 0.0;
                    else v = (b == s) ? bl : 0.0;
                }
            }
            crow[e] = store_as<S, T>((T)v);
            if (kPingPong) prow[e] = (T)v;
        }
        for (int i = tid; i <= L; i += NT) bond[i] = (i == 0 || i == L) ? 1 : 2;
        double part = 0.0;
        for (int c = tid; c < L - 1; c += NT) part += beta * fabs((double)jh[(size_t)r * (L - 1) + c]);
        const double ls = block_sum(part, red);
        if (tid == 0) lsc[r] = ls;
        __syncthreads();
    }

    double logz_tail = 0.0;   // ln of the row-0 contraction (thread 0)

    for (int r = L - 2; r >= 0; --r) {
        const S *orow_s = cache + (size_t)(r + 1) * row_sz;
        const T *orow_t = kPingPong ? prev + (size_t)((r + 1) & 1) * row_sz : nullptr;
        S *crow = cache + (size_t)r * row_sz;
        T *prow = kPingPong ? prev + (size_t)(r & 1) * row_sz : nullptr;

        double part = 0.0;
        for (int c = tid; c < L; c += NT) {
            part += beta * fabs((double)jv[(size_t)r * L + c]);
            if (c < L - 1) part += beta * fabs((double)jh[(size_t)r * (L - 1) + c]);
        }
        double ls = block_sum(part, red);   // valid in every thread; thread 0 keeps it

        // ================= QR sweep, left to right =========================
        const long long tq0 = wall_clock64();
        int mp = 1;                           // m_{c-1}
        for (int c = 0; c < L; ++c) {
            const int Dp = bond[c], D = bond[c + 1];
            const int K = (c == 0) ? 1 : 2 * mp;
            double vs, vd;
            boltz(beta, jv[(size_t)r * L + c], vs, vd);
            // (a) C_s = sum_n Bv[s][n] A_old[n]   (Dp x D)
            const size_t obase = (size_t)c * site_sz;
            for (int e = tid; e < 2 * Dp * D; e += NT) {
                const int s = e / (Dp * D), b = (e / D) % Dp, bb = e % D;
                const size_t i0 = obase + (size_t)s * chi * chi + b * chi + bb;
                const size_t i1 = obase + (size_t)(1 - s) * chi * chi + b * chi + bb;
                T a0, a1;
                if (kPingPong) { a0 = orow_t[i0]; a1 = orow_t[i1]; }
                else { a0 = load_as<T, S>(orow_s + i0); a1 = load_as<T, S>(orow_s + i1); }
                C[s * chi * chi + b * chi + bb] = (T)vs * a0 + (T)vd * a1;
            }
            __syncthreads();
            // (b) M_s[(t,j)][b'] = Bh(c-1)[t][s] * (R_t C_s)[j][b']
            if (c == 0) {
                for (int e = tid; e < 2 * D; e += NT) {
                    const int s = e / D, bb = e % D;
                    Mb[s * 2 * chi * ldm + bb] = C[s * chi * chi + bb];
                }
            } else {
                double hs, hd;
                boltz(beta, jh[(size_t)r * (L - 1) + (c - 1)], hs, hd);
                for (int e = tid; e < 2 * K * D; e += NT) {
                    const int s = e / (K * D), row = (e / D) % K, bb = e % D;
                    const int t = row / mp, j = row % mp;
                    const T *Rt = R + t * chi * chi + j * chi;
                    const T *Cs = C + s * chi * chi + bb;
                    T acc = 0;
                    for (int b = j; b < Dp; ++b) acc += Rt[b] * Cs[b * chi];   // R_t upper trapezoidal
                    Mb[s * 2 * chi * ldm + row * ldm + bb] = (T)((t == s) ? hs : hd) * acc;
                }
            }
            __syncthreads();
            if (c == L - 1) {
                // center of the sweep: T_last[row][s] = M_s[row][0]  (D == 1)
                T *q = qscr + (size_t)c * 2 * 2 * chi * chi;
                for (int e = tid; e < 2 * K; e += NT) {
                    const int row = e >> 1, s = e & 1;
                    q[row * 2 + s] = Mb[s * 2 * chi * ldm + row * ldm];
                }
                __syncthreads();
                break;
            }
            // (c) Householder QR of both blocks, K x D, mc = min(K, D)
            const int mc = K < D ? K : D;
            const int half = tid >> 7, ht = tid & 127;     // 128 threads per block
            T *M = Mb + half * 2 * chi * ldm;
            int G = pow2_floor(128 / D);
            if (G > 64) G = 64;
            const int grp = ht / G, gl = ht % G, ngrp = 128 / G;
            for (int j = 0; j < mc; ++j) {
                if (ht < 64) {
                    T sum = 0;
                    for (int i = j + 1 + ht; i < K; i += 64) { const T x = M[i * ldm + j]; sum += x * x; }
                    sum = group_sum(sum, 64);
                    if (ht == 0) {
                        const T x0 = M[j * ldm + j];
                        T tj = 0, sc = 0;
                        if (sum != (T)0) {
                            const T nr = sqrt(x0 * x0 + sum);
                            const T be = x0 >= 0 ? -nr : nr;
                            tj = (be - x0) / be;
                            sc = (T)1 / (x0 - be);
                            M[j * ldm + j] = be;
                        }
                        tau[half * chi + j] = tj;
                        scal[half] = (double)sc;
                    }
                }
                __syncthreads();
                const T sc = (T)scal[half];
                for (int i = j + 1 + ht; i < K; i += 128) M[i * ldm + j] *= sc;
                __syncthreads();
                const T tj = tau[half * chi + j];
                if (tj != (T)0) {
                    for (int k = j + 1 + grp; k < D; k += ngrp) {
                        T w = 0;
                        for (int i = j + gl; i < K; i += G) w += (i == j ? (T)1 : M[i * ldm + j]) * M[i * ldm + k];
                        w = group_sum(w, G) * tj;
                        for (int i = j + gl; i < K; i += G) M[i * ldm + k] -= (i == j ? (T)1 : M[i * ldm + j]) * w;
                    }
                }
                __syncthreads();
            }
            // (d) explicit Q (K x mc) into Qb[half], by backward accumulation
            {
                T *Q = Qb + half * 2 * chi * chi;
                for (int e = ht; e < K * mc; e += 128) { const int i = e / mc, k = e % mc; Q[i * chi + k] = (i == k) ? (T)1 : (T)0; }
                __syncthreads();
                int Gq = pow2_floor(128 / mc);
                if (Gq > 64) Gq = 64;
                const int gq = ht / Gq, lq = ht % Gq, nq = 128 / Gq;
                // each group owns the same columns for every j (no barrier
                // between reflectors is needed because columns never change hands)
                for (int j = mc - 1; j >= 0; --j) {
                    const T tj = tau[half * chi + j];
                    if (tj == (T)0) continue;
                    for (int k = gq; k < mc; k += nq) {
                        if (k < j) continue;
                        T w = 0;
                        for (int i = j + lq; i < K; i += Gq) w += (i == j ? (T)1 : M[i * ldm + j]) * Q[i * chi + k];
                        w = group_sum(w, Gq) * tj;
                        for (int i = j + lq; i < K; i += Gq) Q[i * chi + k] -= (i == j ? (T)1 : M[i * ldm + j]) * w;
                    }
                }
                __syncthreads();
                // (e) write Q_s to scratch slot c: [s][2chi][chi]
                T *q = qscr + (size_t)c * 2 * 2 * chi * chi + half * 2 * chi * chi;
                for (int e = ht; e < K * mc; e += 128) { const int i = e / mc, k = e % mc; q[i * chi + k] = Q[i * chi + k]; }
                __syncthreads();
            }
            // (f) R_s (mc x D, upper trapezoidal) becomes the carried R_t; normalise
            double rp = 0.0;
            for (int e = tid; e < 2 * mc * D; e += NT) {
                const int s = e / (mc * D), j = (e / D) % mc, k = e % D;
                const T v = (k >= j) ? Mb[s * 2 * chi * ldm + j * ldm + k] : (T)0;
                R[s * chi * chi + j * chi + k] = v;
                rp += (double)v * (double)v;
            }
            const double nu2 = block_sum(rp, red);
            const double nu = sqrt(nu2);
            ls += log(nu);
            const T inv = (T)(1.0 / nu);
            for (int e = tid; e < 2 * mc * D; e += NT) {
                const int s = e / (mc * D), j = (e / D) % mc, k = e % D;
                R[s * chi * chi + j * chi + k] *= inv;
            }
            if (tid == 0) mq[c] = (unsigned char)mc;
            mp = mc;
            __syncthreads();
        }

        // ================= SVD sweep, right to left ========================
        const long long ts0 = wall_clock64();
        cyc_qr += ts0 - tq0;
        int kr = 1;                           // k'_{c+1}
        if (r == 0 && tid == 0) uvec[0] = 1.0;
        double ulog = 0.0;
        for (int c = L - 1; c >= 0; --c) {
            const int K = (c == 0) ? 1 : 2 * mq[c - 1];
            const T *q = qscr + (size_t)c * 2 * 2 * chi * chi;
            if (c == 0) {
                // site 0: T0[s][m] = Q_s(0)[0][0] * X[s][m]
                double sp = 0.0;
                for (int e = tid; e < 2 * kr; e += NT) {
                    const int s = e / kr, m = e % kr;
                    const T v = q[s * 2 * chi * chi] * X[s * chi + m];
                    nrm[e] = v;
                    sp += (double)v * (double)v;
                }
                const double n0 = sqrt(block_sum(sp, red));
                ls += log(n0);
                const T inv = (T)(1.0 / n0);
                S *site = crow;
                T *psite = kPingPong ? prow : nullptr;
                for (size_t e = tid; e < site_sz; e += NT) {
                    const int s = (int)(e / (chi * chi)), a = (int)((e / chi) % chi), m = (int)(e % chi);
                    const T v = (a == 0 && m < kr) ? nrm[s * kr + m] * inv : (T)0;
                    site[e] = store_as<S, T>(v);
                    if (kPingPong) psite[e] = v;
                }
                if (r == 0 && tid == 0) {
                    double tot = 0.0;
                    for (int s = 0; s < 2; ++s)
                        for (int m = 0; m < kr; ++m) tot += (double)nrm[s * kr + m] * (double)inv * uvec[m];
                    logz_tail = ulog + log(tot);
                }
                if (tid == 0) bond[0] = 1;
                __syncthreads();
                break;
            }
            int n;
            if (c == L - 1) {
                n = 2;
                for (int e = tid; e < 2 * K; e += NT) { const int row = e >> 1, s = e & 1; Tm[s * ldt + row] = q[row * 2 + s]; }
            } else {
                const int mc = mq[c];
                n = 2 * kr;
                for (int e = tid; e < K * n; e += NT) {
                    const int col = e / K, row = e % K;
                    const int s = col / kr, m = col % kr;
                    const T *qr = q + s * 2 * chi * chi + row * chi;
                    const T *xc = X + (s * mc) * chi + m;
                    T acc = 0;
                    for (int j = 0; j < mc; ++j) acc += qr[j] * xc[j * chi];
                    Tm[col * ldt + row] = acc;
                }
            }
            __syncthreads();
            for (int e = tid; e < n * n; e += NT) { const int col = e / n, row = e % n; Wm[col * ldt + row] = (row == col) ? (T)1 : (T)0; }
            __syncthreads();
            {
                const long long t0 = wall_clock64();
                total_sweeps += jacobi<T>(Tm, Wm, ldt, K, n, nrm, iflag);
                cyc_jac += wall_clock64() - t0;
            }
            // singular values and their order
            for (int col = tid; col < n; col += NT) {
                T s2 = 0;
                for (int row = 0; row < K; ++row) { const T v = Tm[col * ldt + row]; s2 += v * v; }
                nrm[col] = sqrt(s2);
            }
            __syncthreads();
            for (int col = tid; col < n; col += NT) {
                const T v = nrm[col];
                int rk = 0;
                for (int o = 0; o < n; ++o) { const T w = nrm[o]; rk += (w > v) || (w == v && o < col); }
                perm[rk] = col;
            }
            __syncthreads();
            int kk = chi < K ? chi : K;
            if (n < kk) kk = n;
            double kp = 0.0;
            for (int i = tid; i < kk; i += NT) { const double v = (double)nrm[perm[i]]; kp += v * v; }
            const double nk = sqrt(block_sum(kp, red));
            ls += log(nk);
            // new site c = V^T[:kk], shape (kk, 2, kr), zero padded
            {
                S *site = crow + (size_t)c * site_sz;
                T *psite = kPingPong ? prow + (size_t)c * site_sz : nullptr;
                for (size_t e = tid; e < site_sz; e += NT) {
                    const int s = (int)(e / (chi * chi)), a = (int)((e / chi) % chi), m = (int)(e % chi);
                    const T v = (a < kk && m < kr) ? Wm[perm[a] * ldt + s * kr + m] : (T)0;
                    site[e] = store_as<S, T>(v);
                    if (kPingPong) psite[e] = v;
                }
            }
            if (r == 0) {
                // row-0 contraction from the right: u[a] <- sum_s sum_m A_c[s][a][m] u[m]
                double *u = uvec, *un = uvec + 64;
                for (int a = tid; a < kk; a += NT) {
                    double acc = 0.0;
                    for (int s = 0; s < 2; ++s)
                        for (int m = 0; m < kr; ++m) acc += (double)Wm[perm[a] * ldt + s * kr + m] * u[m];
                    un[a] = acc;
                }
                __syncthreads();
                if (tid == 0) {
                    double mx = 0.0;
                    for (int a = 0; a < kk; ++a) mx = fmax(mx, fabs(un[a]));
                    scal[2] = mx;
                }
                __syncthreads();
                const double mx = scal[2];
                for (int a = tid; a < kk; a += NT) u[a] = un[a] / mx;
                ulog += log(mx);
            }
            __syncthreads();
            // X (K x kk) = U S / ||S_kept||, kept in the Wm region for the next site
            const T inv = (T)(1.0 / nk);
            for (int e = tid; e < K * kk; e += NT) {
                const int row = e / kk, a = e % kk;
                X[row * chi + a] = Tm[perm[a] * ldt + row] * inv;
            }
            if (tid == 0) bond[c] = (unsigned char)kk;
            kr = kk;
            __syncthreads();
        }
        cyc_svd += wall_clock64() - ts0;
        if (tid == 0) lsc[r] = ls;
        __syncthreads();
    }
    if (tid == 0) {
        double lz = logz_tail;
        for (int r = 0; r < L; ++r) lz += lsc[r];
        if (logz_out) logz_out[inst] = lz;
        if (stats_out) {
            stats_out[4 * inst + 0] = total_sweeps;
            stats_out[4 * inst + 1] = cyc_qr;
            stats_out[4 * inst + 2] = cyc_svd;
            stats_out[4 * inst + 3] = cyc_jac;
        }
    }
}

// Host-side launch helpers (called from the C ABI layer).
template <typename T, typename S>
hipError_t launch_build(const InstDesc *desc, unsigned char *ws, const float *Jh, const float *Jv,
                        double *logz, int64_t *stats, int B, size_t lds_bytes, hipStream_t st) {
    auto kern = k_build<T, S>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(B), dim3(NT), lds_bytes, st, desc, ws, Jh, Jv, logz, stats);
    return hipGetLastError();
}

template hipError_t launch_build<double, double>(const InstDesc *, unsigned char *, const float *, const float *, double *, int64_t *, int, size_t, hipStream_t);
template hipError_t launch_build<float, float>(const InstDesc *, unsigned char *, const float *, const float *, double *, int64_t *, int, size_t, hipStream_t);
template hipError_t launch_build<float, __hip_bfloat16>(const InstDesc *, unsigned char *, const float *, const float *, double *, int64_t *, int, size_t, hipStream_t);
template hipError_t launch_build<float, __half>(const InstDesc *, unsigned char *, const float *, const float *, double *, int64_t *, int, size_t, hipStream_t);

// Shared-memory bytes the build kernel needs for bond dimension chi.
size_t build_lds_bytes(int chi, int L, size_t tsize) {
    size_t elems = (size_t)4 * chi * (2 * chi + 1);          // Tm + Wm (>= C,R + M)
    elems += 2 * chi + 2 * chi;                              // tau, nrm
    size_t bytes = elems * tsize;
    bytes = (bytes + 7) & ~(size_t)7;
    bytes += (NT / 64 + 128 + 4) * sizeof(double);           // red, uvec, scal
    bytes += (2 * chi + 4) * sizeof(int);                    // perm, iflag
    bytes += (size_t)(L + 1) + L;                            // bond, mq
    return (bytes + 15) & ~(size_t)15;
}

}  // namespace tnmc

// Row-pipelined cache build: the QR sweep of row r-1 runs beside the SVD
// sweep of row r, on the other two waves of the workgroup (arXiv 2509.19006,
// section 2.2 / Fig. 2 and section 3.2: the same compression as
// build_instance, scheduled differently).
//
// With alternating sweeps (every second row compressed mirrored) row r-1's
// QR sweep consumes row r's sites in the order row r's SVD sweep finalises
// them: the SVD sweep runs right to left in its own orientation, row r-1 is
// mirrored against it, so its left-to-right QR sweep starts at the site row
// r finished first.  Two roles therefore walk the rows bottom to top in
// lockstep, one row apart:
//   * the QR role (waves 2, 3; one wave per parity block) factors row r-1,
//     site c as soon as row r's site L-1-c is final;
//   * the SVD role (waves 0, 1; one wave per block, as the Jacobi always
//     was) truncates row r once the QR role has finished that row.
// Everything a site computes is what build_instance computes for it, in the
// same order; only the lanes a block's QR is spread over differ (one wave
// instead of two), so results agree to rounding.
//
// Synchronisation, all in shared memory: each role has its own two-wave
// barrier (an arrival counter); the SVD role publishes how many sites it has
// finished (across rows) after each site, the QR role how many rows it has
// finished.  Writes go before a release fence and the counter, reads after
// the counter and an acquire fence (workgroup scope: the waves share one CU
// and its caches).  Row r-1's Q slots and QR bond sectors go to the other
// half of ping-pong buffers while row r's SVD sweep reads its own.  Every
// wait is bounded: one that runs out (or any wait after it) sets a sticky
// error word and returns, the build finishes with whatever it has, and the
// instance's statistics record the failure (slot 12, reported by
// tnmc_env_check), so a broken hand-over never hangs the workgroup.
//
// Sector sizes read from shared memory are clamped to their bounds (no-ops
// for a sound hand-over): after a lost hand-over the roles run on without
// each other's data, and the clamps keep every access inside its buffer.
//
// Used for float builds with chi <= 32 when the problem asks for
// alternating sweeps (the host sets the descriptor flag DESC_PIPE and
// sizes the workspace and shared memory for it).
#pragma once

#include "build_device.hpp"

namespace tnmc {

constexpr int PIPE_WAIT_LIMIT = 1 << 21;     // polls of ~64 clocks: ~60 ms

typedef __attribute__((address_space(3))) int lds_int;

__device__ __forceinline__ int pipe_ld(int *p) {
    return __hip_atomic_load((lds_int *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void pipe_st(int *p, int v) {
    __hip_atomic_store((lds_int *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Waits until *word >= target (at most limit polls), then orders every
// later access after it.
__device__ __forceinline__ void pipe_wait(int *word, int target, int *err, int limit) {
    int polls = 0;
    while (pipe_ld(word) < target) {
        if (pipe_ld(err)) break;
        if (++polls > limit) { pipe_st(err, 1); break; }
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Publishes *word = v after every earlier access of the calling wave.
__device__ __forceinline__ void pipe_publish(int *word, int v) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if ((threadIdx.x & 63) == 0) pipe_st(word, v);
}

// Barrier and sum over the two waves of one role.
struct RoleSync {
    int *bar;      // arrival counter
    int *err;      // sticky error word
    double *red;   // [2]
    int phase;     // arrivals this role has waited for so far
    int limit;     // polls before a wait gives up
};
__device__ __forceinline__ void role_sync(RoleSync &rs) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if ((threadIdx.x & 63) == 0)
        __hip_atomic_fetch_add((lds_int *)rs.bar, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    rs.phase += 2;
    pipe_wait(rs.bar, rs.phase, rs.err, rs.limit);
}
__device__ __forceinline__ double role_sum(double v, RoleSync &rs) {
    v = group_sum(v, 64);
    role_sync(rs);   // the previous sum's readers are past it
    if ((threadIdx.x & 63) == 0) rs.red[(threadIdx.x >> 6) & 1] = v;
    role_sync(rs);
    return rs.red[0] + rs.red[1];
}

// Householder vector row stride for one wave per block (G = 64/CHI lanes
// per column, padded segments as in vrow_len).
template <int CHI> constexpr int vrow_len_pipe() {
    return 2 * CHI + (64 / CHI - 1) * (CHI >= 32 ? 4 : 0);
}

// One site of the QR sweep (qr_site) with block p on wave p of the QR role
// (lanes q = threadIdx.x - 128): lane group grp (G = 64/CHI lanes) owns
// column grp of M^p and each lane RR = 2CHI/G consecutive rows.  The
// reflector of column j goes through shared memory within the wave (no
// barrier); only the joint norm of R crosses the two waves.
// Row j of every column becomes final (an entry of R) at step j: it moves to
// Rs (column-major, row stride CHI + 4, one block per wave) and is zeroed in
// the registers, so that a column's rows above the current step are always
// zero.  The pivot takes its diagonal entry out of the registers at the
// step's (uniform) index; the norm of the part below the diagonal is then
// the sum over all of its rows, and the reflector the scaled column with a 1
// written at the diagonal: no step selects rows by comparing them with the
// step.
template <typename T, int CHI>
__device__ double qr_site_pipe(int c, int last, int K, int D, int Dp, int pa0, int m0, int m1, int pn0, T lnh0,
                               T lnh1, const T *C, T *R, T *V, T *tauv, T *Rsc, T *qdst, int chi, RoleSync &rs,
                               int &mc_out, long long &cyc_hh) {
    constexpr int G = 64 / CHI, RR = 2 * CHI / G;
    const int q = threadIdx.x - 128, p = q >> 6, lt = q & 63;
    int grp = lt / G, row0 = (lt % G) * RR;
    asm volatile("" : "+v"(grp), "+v"(row0));   // see qr_site
    const int gl = row0 / RR;
    const int vrow0 = row0 + gl * (CHI >= 32 ? 4 : 0);
    constexpr int VL = vrow_len_pipe<CHI>();
    const int mp = p ? m1 : m0;
    T m[RR];
    if (c == 0) {
        const T x = (grp < D) ? C[grp] : (T)0;
#pragma unroll
        for (int r = 0; r < RR; ++r) m[r] = (row0 + r == 0) ? x : (T)0;
    } else {
        int roff[RR];
        T acc[RR];
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int row = row0 + r;
            const int qq = (row < mp) ? p : 1 - p;
            const int k = (row < K) ? ((row < mp) ? row : row - mp) : 0;
            roff[r] = rkey_base<CHI, RR>(qq * CHI + k);
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
    constexpr int RSL = CHI + 4;
    T *Rs = Rsc + p * CHI * RSL;
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
        // the reflector reaches the other lanes of this wave in issue order
        wave_sync();
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
    wave_sync();
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
    // this column's R entries (rows above and on the diagonal, from Rs)
    T rv[RR];
#pragma unroll
    for (int r = 0; r < RR; ++r) rv[r] = (row0 < CHI) ? Rs[grp * RSL + row0 + r] : (T)0;
    double part = 0.0;
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int row = row0 + r;
        if (row < mc && row <= grp && grp < D) part += (double)rv[r] * (double)rv[r];
    }
    // (both blocks' M have been formed from R before this sum's barriers,
    // so R can be overwritten after it)
    const double nu = sqrt(role_sum(part, rs));
    const T inv = (T)(1.0 / nu);
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int row = row0 + r;
        const T lam = ((grp >= pn0) != (p == 1)) ? lnh1 : lnh0;
        if (row < CHI)
            R[rkey_base<CHI, RR>(p * CHI + row) ^ grp] = (row < mc && row <= grp && grp < D) ? (rv[r] * inv) * lam : (T)0;
    }
    mc_out = mc;
    return log(nu);
}

// The SVD centre for the two SVD-role waves: wave p forms both parts of
// block p (tform_mfma's part s = 0, 1 one after the other).
__device__ __forceinline__ void tform_mfma_pipe(const float *Qs, const float *X, float *Tm, int chi, int ldt,
                                                int bst, int K0, int K1, int r0, int r1, int mn0, int mn1, int n) {
    const int l = threadIdx.x & 63, p = (threadIdx.x >> 6) & 1;
    const int Kp = p ? K1 : K0;
    const int dp = p ? r1 : r0;
    const int i = l & 31, kh = l >> 5;
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
        const int qb = s ? 1 - p : p;
        const int rowoff = s ? (qb ? K1 : K0) : 0;
        const int mn = qb ? mn1 : mn0;
        const int c0 = s ? dp : 0;
        const int wdata = s ? (r0 + r1) - dp : dp;
        const int wout = s ? n - dp : dp;
        const float *Qb = Qs + qb * 2 * chi * chi + rowoff * chi;
        const float *Xb = X + qb * chi * chi;
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
}

// svd_redo_f64 for the SVD role (threads 0..127, role barriers).  The role's
// barrier state comes by value and its phase goes back as the result (an
// outlined call then keeps the caller's barrier state in registers).
template <int MAXB>
__device__ int svd_redo_f64_pipe(double *fb, const float *q, const float *X, float *Tm, float *Wm, float *nrm,
                                 int *iflag, int *jflag, int c, int L, int chi, int K0, int K1, int r0, int r1,
                                 int mn0, int mn1, int n, int kr, int ldt, int bst, RoleSync rs) {
    constexpr int NR = 128;
    const int tid = threadIdx.x, cc2 = chi * chi;
    double *Td = fb, *Wd = fb + 2 * bst, *prm = fb + 4 * bst, *nd = prm + 256;
    for (int e = tid; e < 2 * n * ldt; e += NR) Td[(e / (n * ldt)) * bst + e % (n * ldt)] = 0.0;
    role_sync(rs);
    if (c == L - 1) {
        for (int e = tid; e < K0 + K1; e += NR) {
            const int p = e >= K0, k = p ? e - K0 : e;
            Td[p * bst + k] = (double)q[e];
        }
    } else {
        for (int e = tid; e < 2 * n * chi; e += NR) {
            const int p = e / (n * chi), k = (e / n) % chi, idx = e % n;
            const int Kp = p ? K1 : K0;
            if (k >= Kp || idx >= kr) continue;
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
    role_sync(rs);
    const int pb = (tid >> 6) & 1;
    // one wave per block (role 0 of the register Jacobi: W in the same wave)
    const int sw = jacobi_block<double, MAXB, false>(Td + pb * bst, Wd + pb * bst, ldt, pb ? K1 : K0, n, chi,
                                                     tid & 63, 0, pb, prm, jflag, nd + pb * n, kr, MAX_SWEEPS);
    if ((tid & 63) == 0) iflag[pb] = sw;
    role_sync(rs);
    for (int e = tid; e < 2 * n * ldt; e += NR) {
        const int p = e / (n * ldt), col = (e / ldt) % n, k = e % ldt;
        const int at = p * bst + col * ldt + k;
        Tm[at] = (float)Td[at];
        if (k < n) Wm[at] = (float)Wd[at];
    }
    for (int e = tid; e < 2 * n; e += NR) nrm[e] = (float)nd[e];
    role_sync(rs);
    return rs.phase;
}

// Shared-memory bytes of the pipelined build (float, chi <= 32).
size_t build_pipe_lds_bytes(int chi, int L);

template <typename S, int MAXB>
__device__ __forceinline__ void build_instance_pipe(int inst, const InstDesc *__restrict__ desc, unsigned char *__restrict__ ws,
                                    const float *__restrict__ Jh_all, const float *__restrict__ Jv_all,
                                    double *__restrict__ logz_out, int64_t *__restrict__ stats_out,
                                    unsigned char *smem) {
    static_assert(MAXB <= 32, "the pipelined build covers chi <= 32");
    typedef float T;
    constexpr int NR = 128;   // threads per role
    const long long t_begin = wall_clock64();
    const InstDesc d = desc[inst];
    const int L = d.L, chi = d.chi, tid = threadIdx.x;
    const double beta = d.beta;
    const double LN2 = 0.69314718055994530942;
    const T RS2 = (T)0.70710678118654752440;
    const float *jh = Jh_all + d.off_h;
    const float *jv = Jv_all + d.off_v;
    S *cache = reinterpret_cast<S *>(ws + d.cache_off);
    T *qscr = reinterpret_cast<T *>(ws + d.qscr_off);     // [2 rows][L][2][2chi][chi], then the redo area
    T *prev = reinterpret_cast<T *>(ws + d.prev_off);
    double *lsc = reinterpret_cast<double *>(ws + d.lsc_off);
    const int cc2 = chi * chi;
    const size_t site_sz = (size_t)2 * cc2;
    const size_t row_sz = (size_t)L * site_sz;
    const size_t qrow_sz = (size_t)L * 4 * cc2;
    double *fb = reinterpret_cast<double *>(qscr + 2 * qrow_sz);
    const int CB = chi <= 16 ? 16 : 32;
    constexpr int LB = MAXB <= 16 ? 4 : 5, MM = MAXB - 1;
    const int ldt = chi + 1;
    const int bst = (chi + 1) * ldt;

    // ---- shared memory (build_pipe_lds_bytes) ---------------------------
    // QR role: C [CB][CB], R [2][CB][CB], Vh [2][CB][VL], tau [2][CB],
    //          Rsc [2][CB][CB + 4]
    // SVD role: Tm, Wm [2][bst], X [2][chi][chi], Qst [2][2chi][chi],
    //           nrm [2][chi+2], jprm [4CB]
    const int VLb = CB <= 16 ? vrow_len_pipe<16>() : vrow_len_pipe<32>();
    T *C = reinterpret_cast<T *>(smem);
    T *R = C + CB * CB;
    T *Vh = R + 2 * CB * CB;
    T *tau = Vh + 2 * CB * VLb;
    T *Rsc = tau + 2 * CB;
    T *Tm = Rsc + 2 * CB * (CB + 4);
    T *Wm = Tm + 2 * bst;
    T *X = Wm + 2 * bst;
    T *Qst = X + 2 * cc2;
    T *nrm = Qst + 4 * cc2;
    T *jprm = nrm + 2 * (chi + 2);
    double *dbl = reinterpret_cast<double *>((reinterpret_cast<uintptr_t>(jprm + 4 * CB) + 7) & ~(uintptr_t)7);
    double *redA = dbl;          // [4] all threads (bottom row)
    double *redQ = dbl + 4;      // [2] QR role
    double *redS = dbl + 6;      // [2] SVD role
    double *lsq = dbl + 8;       // [2] QR part of a row's log-scale, by row parity
    double *uvec = dbl + 10;     // [2][64] row-0 contraction vector
    double *scal = uvec + 128;   // [8]
    long long *cycq = reinterpret_cast<long long *>(scal + 8);   // [2] QR role's tick counts
    int *colof = reinterpret_cast<int *>(cycq + 2);              // [2chi+4]
    int *rankv = colof + 2 * chi + 4;                            // [2chi+4]
    int *iflag = rankv + 2 * chi + 4;                            // [4]
    int *jflag = iflag + 4;                                      // [2]
    int *ctl = jflag + 2;                                        // [8] hand-over words
    int *barQ = ctl, *barS = ctl + 1, *prog = ctl + 2, *qrows = ctl + 3, *perr = ctl + 4;
    unsigned char *dsec = reinterpret_cast<unsigned char *>(ctl + 8);   // [L+1][2] bond sectors
    unsigned char *mqb = dsec + 2 * (L + 1);                             // [2 rows][L+1][2] QR bond sectors
    float *jrow = reinterpret_cast<float *>((reinterpret_cast<uintptr_t>(mqb + 4 * (L + 1)) + 3) & ~(uintptr_t)3);

    const bool alternate = (d.flags & 1) != 0;
    // polls before a hand-over wait gives up (one with TNMC_SHORT_WAITS, the
    // test of the failure path)
    const int wait_limit = (d.flags & 8) ? 1 : PIPE_WAIT_LIMIT;
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

    // ---- bottom row (row L-1), all threads ------------------------------
    {
        const int r = L - 1;
        for (size_t e = tid; e < (size_t)L * cc2; e += NT) {
            const int c = (int)(e / cc2), a = (int)((e / chi) % chi), b = (int)(e % chi);
            T v0 = 0, v1 = 0;
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
                    if ((a ^ b) == 0) v0 = lh; else v1 = lh;
                }
            }
            put_site(r, c, a, b, v0, v1);
        }
        for (int i = tid; i <= L; i += NT) {
            dsec[2 * i] = 1;
            dsec[2 * i + 1] = (i == 0 || i == L) ? 0 : 1;
        }
        if (tid < 8) ctl[tid] = 0;
        double part = 0.0;
        for (int c = tid; c < L - 1; c += NT) part += beta * fabs((double)jh[(size_t)r * (L - 1) + c]);
        const double ls = block_sum(part, redA) - (double)(L - 2) * 0.5 * LN2;
        if (tid == 0) lsc[r] = ls;
        __syncthreads();
    }

    if (tid >= NR) {
        // ================= QR role: waves 2, 3 ==============================
        RoleSync rs{barQ, perr, redQ, 0, wait_limit};
        const int q = tid - NR;
        long long cyc_qr = 0, cyc_hh = 0;
        constexpr int CPT = MAXB * MAXB / NR;
        for (int r = L - 2; r >= 0; --r) {
            const long long tq0 = wall_clock64();
            const T *orow = prev + (size_t)((r + 1) & 1) * row_sz;
            unsigned char *mq = mqb + (size_t)(r & 1) * 2 * (L + 1);
            T *qrow = qscr + (size_t)(r & 1) * qrow_sz;
            const bool mir = mirrored(r), rd = mir != mirrored(r + 1);
            // sites of row r+1 finished by the SVD role before its site j
            // (in its own orientation) is final; the bottom row is given
            const int base = (L - 3 - r) * L;
            auto need = [&](int cs) { return r == L - 2 ? 0 : base + (L - (rd ? L - 1 - cs : cs)); };
            double part = 0.0;
            for (int c = q; c < L; c += NR) {
                const float v = jv[(size_t)r * L + (mir ? L - 1 - c : c)];
                jrow[c] = v;
                part += beta * fabs((double)v);
                if (c < L - 1) {
                    const float h = jh[(size_t)r * (L - 1) + (mir ? L - 2 - c : c)];
                    jrow[L + c] = h;
                    part += beta * fabs((double)h);
                }
            }
            double ls = role_sum(part, rs) - (double)(L - 1) * LN2;   // (its barriers publish jrow)
            if (q == 0) { mq[0] = 1; mq[1] = 0; }
            T pre[CPT];
            auto ob = [&](int i) { return rd ? L - i : i; };
            auto fetch_site = [&](int cs) {
                pipe_wait(prog, need(cs), perr, wait_limit);
                const int pa0 = min((int)dsec[2 * ob(cs)], chi), Dp = min(pa0 + dsec[2 * ob(cs) + 1], chi);
                const int pb0 = min((int)dsec[2 * ob(cs + 1)], chi), D = min(pb0 + dsec[2 * ob(cs + 1) + 1], chi);
                const T *os = orow + (size_t)(rd ? L - 1 - cs : cs) * site_sz;
#pragma unroll
                for (int i = 0; i < CPT; ++i) {
                    const int e = q + i * NR;
                    const int a = e >> LB, b = e & MM;
                    const int n = (a >= pa0) ^ (b >= pb0);
                    pre[i] = (a < Dp && b < D) ? os[n * cc2 + (rd ? b * chi + a : a * chi + b)] : (T)0;
                }
            };
            fetch_site(0);
            role_sync(rs);   // (mq[0..1])
            for (int c = 0; c < L; ++c) {
                const int pa0 = min((int)dsec[2 * ob(c)], chi), Dp = min(pa0 + dsec[2 * ob(c) + 1], chi);
                const int pb0 = min((int)dsec[2 * ob(c + 1)], chi), D = min(pb0 + dsec[2 * ob(c + 1) + 1], chi);
                const int m0 = min((int)mq[2 * c], chi), m1 = min((int)mq[2 * c + 1], chi);
                const int K = m0 + m1;
                double lv0, lv1;
                lam_of(beta, jrow[c], lv0, lv1);
#pragma unroll
                for (int i = 0; i < CPT; ++i) {
                    const int e = q + i * NR;
                    const int a = e >> LB, b = e & MM;
                    if (a < Dp && b < D) {
                        const int n = (a >= pa0) ^ (b >= pb0);
                        C[a * CB + b] = (T)(n ? lv1 : lv0) * pre[i];
                    }
                }
                if (c + 1 < L) fetch_site(c + 1);
                double ln0 = 1.0, ln1 = 1.0;
                if (c + 1 < L) lam_of(beta, jrow[L + c], ln0, ln1);
                role_sync(rs);
                int mc = 1;
                T *qd = qrow + (size_t)c * 4 * cc2;
                if (chi <= 16)
                    ls += qr_site_pipe<T, 16>(c, c == L - 1, K, D, Dp, pa0, m0, m1, pb0, (T)ln0, (T)ln1, C, R, Vh,
                                              tau, Rsc, qd, chi, rs, mc, cyc_hh);
                else
                    ls += qr_site_pipe<T, 32>(c, c == L - 1, K, D, Dp, pa0, m0, m1, pb0, (T)ln0, (T)ln1, C, R, Vh,
                                              tau, Rsc, qd, chi, rs, mc, cyc_hh);
                if (c == L - 1) {
                    if (q == 0) { mq[2 * L] = 1; mq[2 * L + 1] = 0; }
                    break;
                }
                if (q == 0) { mq[2 * (c + 1)] = (unsigned char)mc; mq[2 * (c + 1) + 1] = (unsigned char)mc; }
                role_sync(rs);
            }
            if (q == 0) lsq[r & 1] = ls;
            // the row's Q slots, bond sectors and log-scale part, then the count
            role_sync(rs);
            cyc_qr += wall_clock64() - tq0;
            if (tid == NR) pipe_publish(qrows, L - 1 - r);
        }
        if (q == 0) { cycq[0] = cyc_qr; cycq[1] = cyc_hh; }
    } else {
        // ================= SVD role: waves 0, 1 =============================
        RoleSync rs{barS, perr, redS, 0, wait_limit};
        long long cyc_svd = 0, cyc_jac = 0;
        int total_sweeps = 0, maxsweep_hits = 0, redo_f64 = 0;
        const int jac_limit = (d.flags & 2) ? 1 : MAX_SWEEPS;
        double logz_tail = 0.0;
        int done = 0;   // sites finished, over all rows
        for (int r = L - 2; r >= 0; --r) {
            pipe_wait(qrows, L - 1 - r, perr, wait_limit);
            const long long ts0 = wall_clock64();
            const unsigned char *mq = mqb + (size_t)(r & 1) * 2 * (L + 1);
            const T *qrow = qscr + (size_t)(r & 1) * qrow_sz;
            double ls = lsq[r & 1];
            if (tid == 0) { dsec[2 * L] = 1; dsec[2 * L + 1] = 0; uvec[0] = 1.0; }
            role_sync(rs);
            double ulog = 0.0;
            for (int c = L - 1; c >= 0; --c) {
                const int r0 = min((int)dsec[2 * (c + 1)], chi), r1 = min((int)dsec[2 * (c + 1) + 1], chi - r0);
                const int kr = r0 + r1;
                const int K0 = min((int)mq[2 * c], chi), K1 = min((int)mq[2 * c + 1], chi);
                const T *qs = qrow + (size_t)c * 4 * cc2;
                if (c == 0) {
                    double sp = 0.0;
                    for (int m = tid; m < kr; m += NR) {
                        const int p = (m >= r0);
                        const int mm = p ? m - r0 : m;
                        const int mcq = min((int)mq[2 * (c + 1) + p], chi);
                        const T *qr = Qst + p * 2 * cc2;
                        const T *xc = X + p * cc2 + mm;
                        T acc = 0, a1 = 0;
                        int j = 0;
                        for (; j + 1 < mcq; j += 2) {
                            acc += qr[j] * xc[j * chi];
                            a1 += qr[j + 1] * xc[(j + 1) * chi];
                        }
                        if (j < mcq) acc += qr[j] * xc[j * chi];
                        acc += a1;
                        nrm[m] = acc;
                        sp += (double)acc * (double)acc;
                    }
                    const double n0 = sqrt(role_sum(sp, rs));
                    ls += log(n0);
                    const T inv = (T)(1.0 / n0);
                    for (int e = tid; e < cc2; e += NR) {
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
                    role_sync(rs);
                    ++done;
                    if (tid == 0) pipe_publish(prog, done);
                    break;
                }
                const int n = (kr + 1) & ~1;
                const int mn0 = min((int)mq[2 * (c + 1)], chi), mn1 = min((int)mq[2 * (c + 1) + 1], chi);
                if (c == L - 1) {
                    for (int e = tid; e < 2 * n * ldt; e += NR) Tm[(e / (n * ldt)) * bst + e % (n * ldt)] = 0;
                    role_sync(rs);
                    for (int e = tid; e < K0 + K1; e += NR) {
                        const int p = e >= K0, k = p ? e - K0 : e;
                        Tm[p * bst + k] = qs[e];
                    }
                } else {
                    tform_mfma_pipe(Qst, X, Tm, chi, ldt, bst, K0, K1, r0, r1, mn0, mn1, n);
                }
                role_sync(rs);
                {
                    const long long t0 = wall_clock64();
                    const int pb = (tid >> 6) & 1;
                    const int sw = jacobi_block<T, MAXB>(Tm + pb * bst, Wm + pb * bst, ldt, pb ? K1 : K0, n, chi,
                                                         tid & 63, 0, pb, jprm, jflag, nrm + pb * n, kr, jac_limit);
                    if ((tid & 63) == 0) iflag[pb] = sw;
                    role_sync(rs);
                    const int swm = iflag[0] > iflag[1] ? iflag[0] : iflag[1];
                    total_sweeps += swm;
                    if (swm >= jac_limit) {
                        rs.phase = svd_redo_f64_pipe<MAXB>(fb, qs, X, Tm, Wm, nrm, iflag, jflag, c, L, chi, K0, K1,
                                                           r0, r1, mn0, mn1, n, kr, ldt, bst, rs);
                        total_sweeps += iflag[0] > iflag[1] ? iflag[0] : iflag[1];
                        ++redo_f64;
                    }
                    maxsweep_hits += (iflag[0] >= MAX_SWEEPS) + (iflag[1] >= MAX_SWEEPS);
                    cyc_jac += wall_clock64() - t0;
                }
                // the next site's Q slot: loads in flight through the
                // truncation below, stored to Qst at the end of the site
                constexpr int QPT = 4 * MAXB * MAXB / NR;
                T qn[QPT];
                if (c >= 1) {
                    const T *src = qrow + (size_t)(c - 1) * 4 * cc2;
#pragma unroll
                    for (int i = 0; i < QPT; ++i) {
                        const int e = tid + i * NR;
                        qn[i] = e < 4 * cc2 ? src[e] : (T)0;
                    }
                }
                int kk = chi < K0 + K1 ? chi : K0 + K1;
                if (2 * kr < kk) kk = 2 * kr;
                for (int e = tid; e < 2 * n; e += NR) {
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
                // kept columns of block 0 (2n <= 66: the role's threads cover them)
                const int s0 = min(max((int)role_sum((tid < n && rankv[tid] < kk) ? 1.0 : 0.0, rs), 0), kk);
                for (int e = tid; e < 2 * n; e += NR) {
                    if (rankv[e] < kk) {
                        const int p = e / n, re = rankv[e];
                        const int *rb = rankv + p * n;
                        int q0 = 0, q1 = 0;
#pragma unroll 4
                        for (int o = 0; o < n; o += 2) { q0 += rb[o] < re; q1 += rb[o + 1] < re; }
                        colof[(p ? s0 : 0) + q0 + q1] = (p << 8) | (e - p * n);
                    }
                }
                double kp = 0.0;
                for (int e = tid; e < 2 * n; e += NR) if (rankv[e] < kk) { const double v = (double)nrm[e]; kp += v * v; }
                const double nk = sqrt(role_sum(kp, rs));   // (its barriers publish colof)
                ls += log(nk);
                for (int e = tid; e < MAXB * MAXB; e += NR) {
                    const int a = e >> LB, m = e & MM;
                    if (a >= chi || m >= chi) continue;
                    T v0 = 0, v1 = 0;
                    if (a < kk && m < kr) {
                        const int ce = colof[a], p = (ce >> 8) & 1, col = min(ce & 255, n);
                        const int pm = m >= r0, mm = pm ? m - r0 : m;
                        const int dp = p ? r1 : r0;
                        const int s = p ^ pm;
                        const int row = (s == 0) ? mm : dp + mm;
                        const T w = Wm[p * bst + col * ldt + row];
                        if (s == 0) v0 = w; else v1 = w;
                    }
                    put_site(r, c, a, m, v0, v1);
                }
                if (r == 0) {
                    double *u = uvec, *un = uvec + 64;
                    for (int a = tid; a < kk; a += NR) {
                        const int ce = colof[a], p = (ce >> 8) & 1, col = min(ce & 255, n);
                        double acc = 0.0;
                        const int dp = p ? r1 : r0, off = p ? r0 : 0;
                        for (int mm = 0; mm < dp; ++mm) acc += (double)Wm[p * bst + col * ldt + mm] * u[off + mm];
                        un[a] = acc;
                    }
                    role_sync(rs);
                    if (tid == 0) {
                        double mx = 0.0;
                        for (int a = 0; a < kk; ++a) mx = fmax(mx, fabs(un[a]));
                        scal[2] = mx > 0.0 ? mx : 1.0;
                    }
                    role_sync(rs);
                    const double mx = scal[2];
                    for (int a = tid; a < kk; a += NR) u[a] = un[a] / mx;
                    ulog += log(mx);
                }
                role_sync(rs);   // (Tm is read above; X is overwritten below)
                const T inv = (T)(1.0 / nk);
                for (int e = tid; e < 2 * MAXB * MAXB; e += NR) {
                    const int p = e >> (2 * LB), k = (e >> LB) & MM, j = e & MM;
                    const int Kp = p ? K1 : K0, dp = p ? kk - s0 : s0;
                    if (k < Kp && j < dp) {
                        const int ce = colof[(p ? s0 : 0) + j];
                        X[p * cc2 + k * chi + j] = Tm[p * bst + min(ce & 255, n) * ldt + k] * inv;
                    }
                }
                if (tid == 0) { dsec[2 * c] = (unsigned char)s0; dsec[2 * c + 1] = (unsigned char)(kk - s0); }
                if (c >= 1) {
#pragma unroll
                    for (int i = 0; i < QPT; ++i) {
                        const int e = tid + i * NR;
                        if (e < 4 * cc2) Qst[e] = qn[i];
                    }
                }
                // the site (prev, cache), its bond sectors and X, then the count
                role_sync(rs);
                ++done;
                if (tid == 0) pipe_publish(prog, done);
            }
            cyc_svd += wall_clock64() - ts0;
            if (tid == 0) lsc[r] = ls;
        }
        if (tid == 0) {
            // the SVD role's counts, for the record below
            iflag[0] = total_sweeps;
            iflag[1] = maxsweep_hits;
            iflag[2] = redo_f64;
            scal[4] = logz_tail;
            reinterpret_cast<long long *>(scal)[5] = cyc_svd;
            reinterpret_cast<long long *>(scal)[6] = cyc_jac;
        }
    }
    __syncthreads();
    if (tid == 0) {
        double lz = scal[4];
        int nonfinite = 0;
        for (int r = 0; r < L; ++r) { lz += lsc[r]; nonfinite += !isfinite(lsc[r]); }
        if (logz_out) logz_out[inst] = lz;
        if (stats_out) {
            int64_t *so = stats_out + STATS_PER_INST * inst;
            so[STAT_MAXSWEEP] = iflag[1];
            so[STAT_NONFINITE] = nonfinite;
            so[STAT_LOGZ_UNDEFINED] = nonfinite == 0 && !isfinite(lz);
            so[STAT_FALLBACK] = iflag[2];
            so[STAT_PIPE_ERROR] = pipe_ld(perr);
            for (int k = STAT_PIPE_ERROR + 1; k < STATS_PER_INST; ++k) so[k] = 0;
            so[0] = iflag[0];
            so[1] = cycq[0];
            so[2] = reinterpret_cast<long long *>(scal)[5];
            so[3] = reinterpret_cast<long long *>(scal)[6];
            so[4] = t_begin;
            so[5] = wall_clock64();
            so[7] = cycq[1];
        }
    }
}

// The build of one instance: the row-pipelined form in the kernels compiled
// for it (PIPE: float, chi <= 32 launches whose problem asks for alternating
// sweeps), the sequential build_instance otherwise.  Separate kernels keep
// each form's register allocation to itself.
template <typename T, typename S, int MAXB, bool PIPE>
__device__ __forceinline__ void build_instance_sel(int inst, const InstDesc *__restrict__ desc,
                                                   unsigned char *__restrict__ ws, const float *__restrict__ Jh_all,
                                                   const float *__restrict__ Jv_all, double *__restrict__ logz_out,
                                                   int64_t *__restrict__ stats_out, unsigned char *smem) {
    if constexpr (PIPE) {
        static_assert(std::is_same<T, float>::value && MAXB <= 32, "pipelined build: float, chi <= 32");
        build_instance_pipe<S, MAXB>(inst, desc, ws, Jh_all, Jv_all, logz_out, stats_out, smem);
    } else {
        build_instance<T, S, MAXB>(inst, desc, ws, Jh_all, Jv_all, logz_out, stats_out, smem);
    }
}

}  // namespace tnmc

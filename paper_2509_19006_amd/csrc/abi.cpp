// C ABI of the TNMC library: argument validation, workspace layout and
// kernel dispatch.  No device memory is allocated here; every buffer lives
// in the caller's workspace or in caller-owned arrays.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "tnmc.h"
#include "device.hpp"

namespace tnmc {
struct MlpArgs {
    const float *params;
    const float *Jh;
};
hipError_t launch_mlp_features(const InstDesc *, int, int, int, const uint64_t *, const float *, const float *,
                               const float *, float *, hipStream_t);
hipError_t launch_mlp_grad(const float *, int, const float *, const float *, const float *, float *, float *,
                           float *, float *, float *, float *, float, int, int, float *, hipStream_t);
hipError_t launch_mlp_forward(const float *, int, const float *, int, float *, hipStream_t);
hipError_t mlp_static_scratch(float **, size_t *);
int mlp_static_max_rows();
constexpr int kMlpRows = 64;
constexpr int kMlpNParam = 8385;
template <typename T, typename S>
hipError_t launch_build(const InstDesc *, const int32_t *, unsigned char *, const float *, const float *,
                        double *, int64_t *, int, int, bool, size_t, hipStream_t);
size_t build_lds_bytes(int chi, int L, size_t tsize);
size_t build_pipe_lds_bytes(int chi, int L);
template <typename T, typename S, bool SPLIT16>
hipError_t launch_pipeline(const InstDesc *, const int32_t *, unsigned char *, const float *, const float *,
                           double *, int64_t *, int, int, bool, size_t, int, uint64_t, uint64_t, uint64_t *, double *,
                           double *, void *, uint64_t, uint64_t, uint8_t *, int64_t *, hipStream_t);
template <typename T, typename S, bool SPLIT16>
hipError_t launch_sample(int, int, const InstDesc *, unsigned char *, size_t, int, int, int, uint64_t,
                         uint64_t, const uint64_t *, uint64_t *, double *, float *, const float *,
                         MlpArgs, int64_t *, hipStream_t);
hipError_t launch_energy_run(int, int, int, const uint64_t *, int64_t, const float *, int64_t, const float *,
                             int64_t, double *, int32_t *, hipStream_t);
hipError_t launch_overlap_run(int, int, int, const uint64_t *, const int64_t *, const uint64_t *, const int64_t *,
                              int64_t, int64_t, double *, hipStream_t);
hipError_t launch_accept(int, int, const double *, const double *, const double *, void *, uint64_t,
                         uint64_t, uint8_t *, int64_t *, hipStream_t);
hipError_t launch_philox(uint64_t, const uint32_t *, uint32_t, uint32_t, uint32_t, int, double *,
                         hipStream_t);
constexpr int kSampleTile = 256;
}  // namespace tnmc

using tnmc::InstDesc;

static thread_local std::string g_err;

static int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

namespace tnmc {
int set_error(int code, const std::string &msg) { return fail(code, msg); }
}

static int hip_fail(hipError_t e, const char *what) {
    return fail(TNMC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct tnmc_env {
    int32_t batch = 0, precision = 0, chi_bucket = 0, chi_mask = 0, max_tiles = 0;
    std::vector<int32_t> L, chi;
    std::vector<double> beta;
    const float *J_h = nullptr, *J_v = nullptr;
    std::vector<InstDesc> desc;
    std::vector<int32_t> order;      // build launch order (longest first)
    unsigned char *ws = nullptr;
    size_t ws_bytes = 0, tile_bytes = 0, desc_off = 0, sweeps_off = 0;
};

namespace tnmc {
int env_batch(const tnmc_env *env) { return env ? env->batch : 0; }
}

namespace {

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

size_t tsize_of(int prec) { return prec == TNMC_FP64 ? 8 : 4; }
size_t ssize_of(int prec) {
    switch (prec) {
    case TNMC_FP64: return 8;
    case TNMC_FP32:
    case TNMC_MIXED_BF16X3: return 4;
    default: return 2;
    }
}

// bit 0 / 1 / 2: the batch has instances with chi <= 16, 16 < chi <= 32, chi > 32
int chi_mask_of(const tnmc_problem *p) {
    int m = 0;
    for (int i = 0; i < p->batch; ++i) m |= p->chi[i] <= 16 ? 1 : (p->chi[i] <= 32 ? 2 : 4);
    return m;
}

int chi_bucket_of(int chi) { return chi <= 16 ? 16 : (chi <= 32 ? 32 : 64); }

struct Plan {
    std::vector<InstDesc> desc;
    std::vector<int32_t> order;
    size_t order_off = 0;
    size_t desc_off = 0, sweeps_off = 0, fixed = 0, tile_bytes = 0;
    int chi_bucket = 16, chi_max = 2, L_max = 2;
    bool pipe = false;   // rows pipelined in the build (see build_pipe.hpp)
};

// Shared memory of the build kernels for a plan.
size_t build_lds(const Plan &pl, int precision) {
    size_t b = tnmc::build_lds_bytes(pl.chi_max, pl.L_max, tsize_of(precision));
    if (pl.pipe) b = std::max(b, tnmc::build_pipe_lds_bytes(pl.chi_max, pl.L_max));
    return b;
}

int validate(const tnmc_problem *p, int precision, bool need_data) {
    if (!p) return fail(TNMC_EINVAL, "problem is NULL");
    if (p->batch < 1) return fail(TNMC_EINVAL, "batch must be >= 1");
    if (!p->L || !p->chi || !p->beta) return fail(TNMC_EINVAL, "L, chi and beta must be non-NULL host arrays");
    if (need_data && (!p->J_h || !p->J_v)) return fail(TNMC_EINVAL, "J_h and J_v must be non-NULL device arrays");
    if (precision < TNMC_FP64 || precision > TNMC_MIXED_BF16X3) return fail(TNMC_EINVAL, "unknown precision");
    for (int i = 0; i < p->batch; ++i) {
        const int L = p->L[i], chi = p->chi[i];
        const double b = p->beta[i];
        if (L < 2 || L > TNMC_L_MAX)
            return fail(TNMC_EINVAL, "instance " + std::to_string(i) + ": L must be in [2, " + std::to_string(TNMC_L_MAX) + "]");
        if (chi < 2 || chi > TNMC_CHI_MAX)
            return fail(TNMC_EINVAL, "instance " + std::to_string(i) + ": chi must be in [2, 64]");
        if (!std::isfinite(b) || b < 0.0)
            return fail(TNMC_EINVAL, "instance " + std::to_string(i) + ": beta must be finite and >= 0");
        if (precision == TNMC_FP64 && chi > 32)
            return fail(TNMC_ENOTSUP, "float64 path supports chi <= 32 (instance " + std::to_string(i) + ")");
        if (p->off_h && p->off_h[i] < 0) return fail(TNMC_EINVAL, "negative J_h offset");
        if (p->off_v && p->off_v[i] < 0) return fail(TNMC_EINVAL, "negative J_v offset");
    }
    if (p->coupling_kind < TNMC_COUPLING_GENERAL || p->coupling_kind > TNMC_COUPLING_GRID20)
        return fail(TNMC_EINVAL, "unknown coupling_kind");
    if (p->flags & ~(TNMC_ALTERNATE_SWEEPS | TNMC_FORCE_F64_FALLBACK | TNMC_SHORT_WAITS))
        return fail(TNMC_EINVAL, "unknown problem flags");
    return TNMC_OK;
}

// The Philox sample / proposal counter is one 32-bit word.
bool counter_overflows(uint64_t offset, int32_t n) { return offset + (uint64_t)n > (uint64_t(1) << 32); }

// Workspace layout: [desc table][build stats][per instance: log-scales,
// cache, build scratch, previous-row ping-pong][sampler env tiles ...].
int plan(const tnmc_problem *p, int precision, Plan &pl, int schedule = TNMC_SCHED_LONGEST_FIRST) {
    const size_t ts = tsize_of(precision), ss = ssize_of(precision);
    const int B = p->batch;
    pl.desc.assign(B, InstDesc{});
    for (int i = 0; i < B; ++i) {
        pl.chi_max = std::max(pl.chi_max, p->chi[i]);
        pl.L_max = std::max(pl.L_max, p->L[i]);
    }
    pl.chi_bucket = chi_bucket_of(pl.chi_max);
    // the row-pipelined build: float arithmetic, chi <= 32 launches, and the
    // alternating sweep order that lets row r-1's QR sweep follow row r's SVD
    // sweep site by site
    pl.pipe = (p->flags & TNMC_ALTERNATE_SWEEPS) && ts == sizeof(float) && pl.chi_max <= 32;
    size_t off = 0;
    pl.desc_off = off;
    off = align_up(off + sizeof(InstDesc) * B);
    pl.order_off = off;
    off = align_up(off + sizeof(int32_t) * B);
    pl.sweeps_off = off;
    off = align_up(off + sizeof(int64_t) * tnmc::STATS_PER_INST * B);
    // Launch order.  The build of an instance costs about (L-1) L chi^3 and
    // workgroups start in launch order, so longest-first (the default)
    // shortens the whole batch; shortest-first lets small instances finish
    // early; or the problem's own order.  Stable on ties.
    pl.order.resize(B);
    for (int i = 0; i < B; ++i) pl.order[i] = i;
    auto cost = [&](int i) { return (double)(p->L[i] - 1) * p->L[i] * std::pow((double)p->chi[i], 3); };
    if (schedule == TNMC_SCHED_LONGEST_FIRST)
        std::stable_sort(pl.order.begin(), pl.order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    else if (schedule == TNMC_SCHED_SHORTEST_FIRST)
        std::stable_sort(pl.order.begin(), pl.order.end(), [&](int a, int b) { return cost(a) < cost(b); });
    int64_t oh = 0, ov = 0, wp = 0, sp = 0;
    for (int i = 0; i < B; ++i) {
        InstDesc &d = pl.desc[i];
        const int L = p->L[i], chi = p->chi[i];
        d.L = L; d.chi = chi; d.W = (L + 63) / 64; d.flags = (p->flags & (TNMC_ALTERNATE_SWEEPS | TNMC_FORCE_F64_FALLBACK | TNMC_SHORT_WAITS)) |
                  (pl.pipe ? tnmc::DESC_PIPE : 0);
        d.beta = p->beta[i];
        d.off_h = p->off_h ? p->off_h[i] : oh;
        d.off_v = p->off_v ? p->off_v[i] : ov;
        oh += (int64_t)L * (L - 1);
        ov += (int64_t)(L - 1) * L;
        d.word_prefix = wp;
        d.site_prefix = sp;
        wp += (int64_t)L * d.W;
        sp += (int64_t)L * L;
        d.lsc_off = off;
        off = align_up(off + sizeof(double) * L);
        d.cache_off = off;
        off = align_up(off + (size_t)L * L * 2 * chi * chi * ss);
        d.qscr_off = off;      // Q slots (two rows when pipelined), then (float builds) the float64 redo area
        off = align_up(off + (pl.pipe ? 2 : 1) * (size_t)L * 2 * 2 * chi * chi * ts +
                       (ts == sizeof(float) ? sizeof(double) * tnmc::fallback_doubles(chi) : 0));
        d.prev_off = off;      // previous row in the parity basis (build arithmetic type)
        off = align_up(off + (size_t)2 * L * 2 * chi * chi * ts);
    }
    pl.fixed = off;
    size_t tb = 0;
    for (int i = 0; i < B; ++i) {
        pl.desc[i].env_off = off + tb;
        tb = align_up(tb + (size_t)tnmc::kSampleTile * p->L[i] * pl.chi_bucket * ts);
    }
    pl.tile_bytes = tb;
    return TNMC_OK;
}

int check_lds(int precision, const Plan &pl) {
    const size_t need = build_lds(pl, precision);
    int dev = 0, lim = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    if (need > (size_t)lim)
        return fail(TNMC_ENOTSUP, "build needs " + std::to_string(need) + " bytes of LDS per workgroup, device allows " + std::to_string(lim));
    return TNMC_OK;
}

}  // namespace

extern "C" {

const char *tnmc_last_error(void) { return g_err.c_str(); }

size_t tnmc_workspace_bytes(const tnmc_problem *p, int32_t precision, int32_t max_samples) {
    size_t b = 0;
    return tnmc_workspace_size(p, precision, max_samples, &b) == TNMC_OK ? b : 0;
}

int tnmc_workspace_size(const tnmc_problem *p, int32_t precision, int32_t max_samples, size_t *bytes_out) {
    int rc = validate(p, precision, false);
    if (rc) return rc;
    if (max_samples < 1) return fail(TNMC_EINVAL, "max_samples must be >= 1");
    if (!bytes_out) return fail(TNMC_EINVAL, "bytes_out is NULL");
    Plan pl;
    plan(p, precision, pl);
    const size_t tiles = (size_t)(max_samples + tnmc::kSampleTile - 1) / tnmc::kSampleTile;
    *bytes_out = pl.fixed + tiles * pl.tile_bytes;
    return TNMC_OK;
}

}  // extern "C"

namespace {

// Validates, plans the workspace, creates the env and uploads descriptors
// and launch order; the caller launches the kernels.
int setup_env(const tnmc_problem *p, int32_t precision, void *workspace, size_t workspace_bytes,
              hipStream_t st, tnmc_env **env_out, Plan &pl, int schedule = TNMC_SCHED_LONGEST_FIRST) {
    int rc = validate(p, precision, true);
    if (rc) return rc;
    if (!env_out) return fail(TNMC_EINVAL, "env_out is NULL");
    if (!workspace) return fail(TNMC_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(TNMC_EINVAL, "workspace must be 256-byte aligned");
    if (schedule < TNMC_SCHED_LONGEST_FIRST || schedule > TNMC_SCHED_AS_GIVEN) return fail(TNMC_EINVAL, "unknown schedule");
    plan(p, precision, pl, schedule);
    if (workspace_bytes < pl.fixed + pl.tile_bytes)
        return fail(TNMC_ENOSPACE, "workspace has " + std::to_string(workspace_bytes) + " bytes, needs at least " + std::to_string(pl.fixed + pl.tile_bytes));
    rc = check_lds(precision, pl);
    if (rc) return rc;
    tnmc_env *env = new tnmc_env();
    env->batch = p->batch;
    env->precision = precision;
    env->chi_bucket = pl.chi_bucket;
    env->chi_mask = chi_mask_of(p);
    env->L.assign(p->L, p->L + p->batch);
    env->chi.assign(p->chi, p->chi + p->batch);
    env->beta.assign(p->beta, p->beta + p->batch);
    env->J_h = p->J_h;
    env->J_v = p->J_v;
    env->desc = pl.desc;
    env->order = pl.order;
    env->ws = static_cast<unsigned char *>(workspace);
    env->ws_bytes = workspace_bytes;
    env->tile_bytes = pl.tile_bytes;
    env->desc_off = pl.desc_off;
    env->sweeps_off = pl.sweeps_off;
    env->max_tiles = (int)((workspace_bytes - pl.fixed) / pl.tile_bytes);
    hipError_t e = hipMemcpyAsync(env->ws + pl.desc_off, env->desc.data(), sizeof(InstDesc) * p->batch,
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) { delete env; return hip_fail(e, "descriptor upload"); }
    e = hipMemcpyAsync(env->ws + pl.order_off, env->order.data(), sizeof(int32_t) * p->batch,
                       hipMemcpyHostToDevice, st);
    if (e != hipSuccess) { delete env; return hip_fail(e, "schedule upload"); }
    *env_out = env;
    return TNMC_OK;
}

}  // namespace

extern "C" {

int tnmc_build_env(const tnmc_problem *p, int32_t precision, void *workspace, size_t workspace_bytes,
                   void *stream, tnmc_env **env_out, double *logz_out) {
    Plan pl;
    hipStream_t st = static_cast<hipStream_t>(stream);
    tnmc_env *env = nullptr;
    int rc = setup_env(p, precision, workspace, workspace_bytes, st, &env, pl);
    if (rc) return rc;
    const int32_t *ord = reinterpret_cast<const int32_t *>(env->ws + pl.order_off);
    const InstDesc *dd = reinterpret_cast<const InstDesc *>(env->ws + pl.desc_off);
    int64_t *sw = reinterpret_cast<int64_t *>(env->ws + pl.sweeps_off);
    const size_t lds = build_lds(pl, precision);
    hipError_t e;
    switch (precision) {
    case TNMC_FP64: e = tnmc::launch_build<double, double>(dd, ord, env->ws, p->J_h, p->J_v, logz_out, sw, p->batch, pl.chi_max, pl.pipe, lds, st); break;
    case TNMC_FP32: e = tnmc::launch_build<float, float>(dd, ord, env->ws, p->J_h, p->J_v, logz_out, sw, p->batch, pl.chi_max, pl.pipe, lds, st); break;
    case TNMC_MIXED_BF16X3: e = tnmc::launch_build<float, float>(dd, ord, env->ws, p->J_h, p->J_v, logz_out, sw, p->batch, pl.chi_max, pl.pipe, lds, st); break;
    case TNMC_MIXED_BF16: e = tnmc::launch_build<float, __hip_bfloat16>(dd, ord, env->ws, p->J_h, p->J_v, logz_out, sw, p->batch, pl.chi_max, pl.pipe, lds, st); break;
    default: e = tnmc::launch_build<float, __half>(dd, ord, env->ws, p->J_h, p->J_v, logz_out, sw, p->batch, pl.chi_max, pl.pipe, lds, st); break;
    }
    if (e != hipSuccess) { delete env; return hip_fail(e, "build launch"); }
    *env_out = env;
    return TNMC_OK;
}

int tnmc_run(const tnmc_problem *p, int32_t precision, void *workspace, size_t workspace_bytes,
             int32_t n_samples, uint64_t sample_seed, uint64_t sample_offset, tnmc_chain *chain,
             uint64_t accept_seed, uint64_t step_offset, uint64_t *spins_out, double *logq_out,
             double *E_out, uint8_t *accepted_out, int64_t *state_out, double *logz_out, int32_t schedule,
             void *stream, tnmc_env **env_out) {
    if (n_samples < 1) return fail(TNMC_EINVAL, "n_samples must be >= 1");
    if (counter_overflows(sample_offset, n_samples) || counter_overflows(step_offset, n_samples))
        return fail(TNMC_EINVAL, "sample_offset / step_offset + n_samples exceeds the 32-bit Philox counter");
    if (!spins_out || !logq_out || !E_out || !accepted_out || !chain)
        return fail(TNMC_EINVAL, "spins_out, logq_out, E_out, accepted_out and chain must be non-NULL");
    Plan pl;
    hipStream_t st = static_cast<hipStream_t>(stream);
    tnmc_env *env = nullptr;
    int rc = setup_env(p, precision, workspace, workspace_bytes, st, &env, pl, schedule);
    if (rc) return rc;
    const int32_t *ord = reinterpret_cast<const int32_t *>(env->ws + pl.order_off);
    const InstDesc *dd = reinterpret_cast<const InstDesc *>(env->ws + pl.desc_off);
    int64_t *sw = reinterpret_cast<int64_t *>(env->ws + pl.sweeps_off);
    const size_t lds = build_lds(pl, precision);
#define TNMC_RUN(T, S, SP) tnmc::launch_pipeline<T, S, SP>(dd, ord, env->ws, p->J_h, p->J_v, logz_out, sw, p->batch, \
        pl.chi_max, pl.pipe, lds, n_samples, sample_seed, sample_offset, spins_out, logq_out, E_out, chain, accept_seed, \
        step_offset, accepted_out, state_out, st)
    hipError_t e;
    switch (precision) {
    case TNMC_FP64: e = TNMC_RUN(double, double, false); break;
    case TNMC_FP32: e = TNMC_RUN(float, float, false); break;
    case TNMC_MIXED_BF16X3: e = TNMC_RUN(float, float, true); break;
    case TNMC_MIXED_BF16: e = TNMC_RUN(float, __hip_bfloat16, false); break;
    default: e = TNMC_RUN(float, __half, false); break;
    }
#undef TNMC_RUN
    if (e != hipSuccess) { delete env; return hip_fail(e, "pipeline launch"); }
    *env_out = env;
    return TNMC_OK;
}

int tnmc_sample(tnmc_env *env, int32_t n_samples, uint64_t seed, uint64_t sample_offset,
                const uint64_t *forced_spins, const tnmc_mlp *mlp, uint64_t *spins_out,
                double *logq_out, float *logits_out, void *stream) {
    if (!env) return fail(TNMC_EINVAL, "env is NULL");
    if (n_samples < 1) return fail(TNMC_EINVAL, "n_samples must be >= 1");
    if (counter_overflows(sample_offset, n_samples))
        return fail(TNMC_EINVAL, "sample_offset + n_samples exceeds the 32-bit Philox sample counter");
    if (!spins_out || !logq_out) return fail(TNMC_EINVAL, "spins_out and logq_out must be non-NULL");
    const int tiles = (n_samples + tnmc::kSampleTile - 1) / tnmc::kSampleTile;
    if (tiles > env->max_tiles)
        return fail(TNMC_ENOSPACE, "workspace sized for " + std::to_string(env->max_tiles * tnmc::kSampleTile) + " samples per call");
    tnmc::MlpArgs ma{};
    if (mlp) {
        if (!mlp->params) return fail(TNMC_EINVAL, "mlp->params is NULL");
        if (env->precision != TNMC_FP32 || env->chi_bucket != 16)
            return fail(TNMC_ENOTSUP, "the learned correction runs on float32 envs with chi <= 16");
        ma.params = mlp->params;
        ma.Jh = env->J_h;
    }
    const InstDesc *dd = reinterpret_cast<const InstDesc *>(env->ws + env->desc_off);
    int64_t *stats = reinterpret_cast<int64_t *>(env->ws + env->sweeps_off);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    switch (env->precision) {
#define TNMC_SAMPLE(T, S, SP) tnmc::launch_sample<T, S, SP>(env->chi_bucket, env->chi_mask, dd, env->ws, env->tile_bytes, \
        env->batch, tiles, n_samples, seed, sample_offset, forced_spins, spins_out, logq_out, logits_out, env->J_v, ma, \
        stats, st)
    case TNMC_FP64: e = TNMC_SAMPLE(double, double, false); break;
    case TNMC_FP32: e = TNMC_SAMPLE(float, float, false); break;
    case TNMC_MIXED_BF16X3: e = TNMC_SAMPLE(float, float, true); break;
    case TNMC_MIXED_BF16: e = TNMC_SAMPLE(float, __hip_bfloat16, false); break;
    default: e = TNMC_SAMPLE(float, __half, false); break;
#undef TNMC_SAMPLE
    }
    if (e != hipSuccess) return hip_fail(e, "sample launch");
    return TNMC_OK;
}

int tnmc_energy(const tnmc_problem *p, int32_t n_samples, const uint64_t *spins, double *E_out,
                int32_t *E_int_out, void *stream) {
    if (!p) return fail(TNMC_EINVAL, "problem is NULL");
    if (p->batch < 1 || !p->L) return fail(TNMC_EINVAL, "batch must be >= 1 with a host L array");
    if (!p->J_h || !p->J_v) return fail(TNMC_EINVAL, "J_h and J_v must be non-NULL device arrays");
    if (n_samples < 1) return fail(TNMC_EINVAL, "n_samples must be >= 1");
    if (!spins || !E_out) return fail(TNMC_EINVAL, "spins and E_out must be non-NULL");
    if (p->coupling_kind < TNMC_COUPLING_GENERAL || p->coupling_kind > TNMC_COUPLING_GRID20)
        return fail(TNMC_EINVAL, "unknown coupling_kind");
    if (E_int_out && p->coupling_kind != TNMC_COUPLING_PMJ)
        return fail(TNMC_EINVAL, "E_int_out needs coupling_kind TNMC_COUPLING_PMJ");
    const int B = p->batch;
    std::vector<int64_t> oh(B), ov(B), wpre(B);
    int64_t ah = 0, av = 0, wp = 0;
    for (int i = 0; i < B; ++i) {
        const int L = p->L[i];
        if (L < 2 || L > TNMC_L_MAX)
            return fail(TNMC_EINVAL, "instance " + std::to_string(i) + ": L must be in [2, " + std::to_string(TNMC_L_MAX) + "]");
        oh[i] = p->off_h ? p->off_h[i] : ah;
        ov[i] = p->off_v ? p->off_v[i] : av;
        if (oh[i] < 0 || ov[i] < 0) return fail(TNMC_EINVAL, "negative coupling offset");
        ah += (int64_t)L * (L - 1);
        av += (int64_t)(L - 1) * L;
        wpre[i] = wp;
        wp += (int64_t)L * ((L + 63) / 64);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    // runs of equal L with evenly spaced coupling offsets: one launch each
    for (int i0 = 0; i0 < B;) {
        const int L = p->L[i0];
        int i1 = i0 + 1;
        if (i1 < B && p->L[i1] == L) {
            const int64_t dh = oh[i1] - oh[i0], dv = ov[i1] - ov[i0];
            while (i1 < B && p->L[i1] == L && oh[i1] - oh[i1 - 1] == dh && ov[i1] - ov[i1 - 1] == dv) ++i1;
        }
        const int64_t sh = i1 - i0 > 1 ? oh[i0 + 1] - oh[i0] : 0, sv = i1 - i0 > 1 ? ov[i0 + 1] - ov[i0] : 0;
        const int64_t iw = (int64_t)n_samples * L * ((L + 63) / 64);
        hipError_t e = tnmc::launch_energy_run(L, i1 - i0, n_samples, spins + (size_t)n_samples * wpre[i0], iw,
                                               p->J_h + oh[i0], sh, p->J_v + ov[i0], sv,
                                               E_out + (size_t)i0 * n_samples,
                                               E_int_out ? E_int_out + (size_t)i0 * n_samples : nullptr, st);
        if (e != hipSuccess) return hip_fail(e, "energy launch");
        i0 = i1;
    }
    return TNMC_OK;
}

int tnmc_overlap(const tnmc_problem *p, int32_t n_samples, const uint64_t *spins_a, const int64_t *state_a,
                 const uint64_t *spins_b, const int64_t *state_b, uint64_t state_offset, double *q_out,
                 void *stream) {
    if (!p) return fail(TNMC_EINVAL, "problem is NULL");
    if (p->batch < 1 || !p->L) return fail(TNMC_EINVAL, "batch must be >= 1 with a host L array");
    if (n_samples < 1) return fail(TNMC_EINVAL, "n_samples must be >= 1");
    if (!spins_a || !state_a || !spins_b || !state_b || !q_out) return fail(TNMC_EINVAL, "NULL array argument");
    if (state_offset > (uint64_t(1) << 62)) return fail(TNMC_EINVAL, "state_offset out of range");
    const int B = p->batch;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int64_t wp = 0;
    for (int i = 0; i < B; ++i) {
        const int L = p->L[i];
        if (L < 2 || L > TNMC_L_MAX)
            return fail(TNMC_EINVAL, "instance " + std::to_string(i) + ": L must be in [2, " + std::to_string(TNMC_L_MAX) + "]");
    }
    for (int i0 = 0; i0 < B;) {
        const int L = p->L[i0];
        int i1 = i0 + 1;
        while (i1 < B && p->L[i1] == L) ++i1;
        const int64_t iw = (int64_t)n_samples * L * ((L + 63) / 64);
        const size_t so = (size_t)i0 * n_samples;
        hipError_t e = tnmc::launch_overlap_run(L, i1 - i0, n_samples, spins_a + (size_t)n_samples * wp, state_a + so,
                                                spins_b + (size_t)n_samples * wp, state_b + so, iw,
                                                (int64_t)state_offset, q_out + so, st);
        if (e != hipSuccess) return hip_fail(e, "overlap launch");
        wp += (int64_t)(i1 - i0) * L * ((L + 63) / 64);
        i0 = i1;
    }
    return TNMC_OK;
}

int tnmc_env_check(const tnmc_env *env, void *stream) {
    if (!env) return fail(TNMC_EINVAL, "env is NULL");
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "stream synchronisation");
    std::vector<int64_t> st((size_t)tnmc::STATS_PER_INST * env->batch);
    e = hipMemcpy(st.data(), env->ws + env->sweeps_off, st.size() * sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "statistics read");
    for (int i = 0; i < env->batch; ++i) {
        const int64_t *s = st.data() + (size_t)tnmc::STATS_PER_INST * i;
        // a lost hand-over first: the other counts of that build are its
        // consequences
        if (s[tnmc::STAT_PIPE_ERROR])
            return fail(TNMC_ENUMERIC, "instance " + std::to_string(i) + ": the row-pipelined build lost a hand-over");
        if (s[tnmc::STAT_NONFINITE])
            return fail(TNMC_ENUMERIC, "instance " + std::to_string(i) + ": " + std::to_string(s[tnmc::STAT_NONFINITE]) +
                                           " row log-scale(s) not finite");
        if (s[tnmc::STAT_MAXSWEEP])
            return fail(TNMC_ENUMERIC, "instance " + std::to_string(i) + ": " + std::to_string(s[tnmc::STAT_MAXSWEEP]) +
                                           " truncation(s) reached the Jacobi sweep limit");
    }
    return TNMC_OK;
}

int tnmc_accept(int32_t batch, int32_t n_samples, const double *logq, const double *E, const double *beta,
                tnmc_chain *chain, uint64_t seed, uint64_t step_offset, uint8_t *accepted_out,
                int64_t *state_out, void *stream) {
    if (batch < 1 || n_samples < 1) return fail(TNMC_EINVAL, "batch and n_samples must be >= 1");
    if (counter_overflows(step_offset, n_samples))
        return fail(TNMC_EINVAL, "step_offset + n_samples exceeds the 32-bit Philox proposal counter");
    if (!logq || !E || !beta || !chain || !accepted_out) return fail(TNMC_EINVAL, "NULL array argument");
    hipError_t e = tnmc::launch_accept(batch, n_samples, logq, E, beta, chain, seed, step_offset, accepted_out,
                                       state_out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "accept launch");
    return TNMC_OK;
}

int tnmc_mlp_features(const tnmc_env *env, int32_t n_samples, const uint64_t *spins, const float *logits_lo,
                      float *feat_out, void *stream) {
    if (!env) return fail(TNMC_EINVAL, "env is NULL");
    if (n_samples < 1 || !spins || !logits_lo || !feat_out) return fail(TNMC_EINVAL, "bad mlp_features arguments");
    int Lmax = 0;
    for (int L : env->L) Lmax = std::max(Lmax, L);
    const InstDesc *dd = reinterpret_cast<const InstDesc *>(env->ws + env->desc_off);
    hipError_t e = tnmc::launch_mlp_features(dd, env->batch, Lmax, n_samples, spins, logits_lo, env->J_h, env->J_v,
                                             feat_out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mlp features launch");
    return TNMC_OK;
}

size_t tnmc_mlp_scratch_floats(int32_t n_rows) {
    if (n_rows < 1) return 0;
    const size_t nblk = (size_t)(n_rows + tnmc::kMlpRows - 1) / tnmc::kMlpRows;
    return nblk * tnmc::kMlpNParam + nblk;
}

int tnmc_mlp_train_step(float *params, float *adam_m, float *adam_v, int32_t n_rows, const float *feat,
                        const float *logit_lo, const float *target_logit, float lr, int32_t step, float *scratch,
                        float *grad_out, float *loss_out, void *stream) {
    if (!params || n_rows < 1 || !feat || !logit_lo || !target_logit || !scratch || step < 0)
        return fail(TNMC_EINVAL, "bad mlp_train_step arguments");
    if (step > 0 && (!adam_m || !adam_v)) return fail(TNMC_EINVAL, "Adam moments are NULL");
    if (!(lr >= 0.0f)) return fail(TNMC_EINVAL, "lr must be >= 0");
    const size_t nblk = (size_t)(n_rows + tnmc::kMlpRows - 1) / tnmc::kMlpRows;
    hipError_t e = tnmc::launch_mlp_grad(params, n_rows, feat, logit_lo, target_logit, scratch,
                                         scratch + nblk * tnmc::kMlpNParam, adam_m, adam_v, grad_out, loss_out,
                                         lr, step, step > 0 ? 1 : 0, params, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mlp train launch");
    return TNMC_OK;
}

int tnmc_mlp_train_step_noalloc(float *params, float *adam_m, float *adam_v, int32_t n_rows, const float *feat,
                                const float *logit_lo, const float *target_logit, float lr, int32_t step,
                                float *grad_out, float *loss_out, void *stream) {
    if (!params || n_rows < 1 || !feat || !logit_lo || !target_logit || step < 0)
        return fail(TNMC_EINVAL, "bad mlp_train_step_noalloc arguments");
    if (n_rows > tnmc::mlp_static_max_rows())
        return fail(TNMC_EINVAL, "n_rows " + std::to_string(n_rows) + " exceeds the static scratch limit of " +
                                     std::to_string(tnmc::mlp_static_max_rows()) + " rows");
    if (step > 0 && (!adam_m || !adam_v)) return fail(TNMC_EINVAL, "Adam moments are NULL");
    if (!(lr >= 0.0f)) return fail(TNMC_EINVAL, "lr must be >= 0");
    float *scr = nullptr;
    size_t cap = 0;
    hipError_t e = tnmc::mlp_static_scratch(&scr, &cap);
    if (e != hipSuccess) return hip_fail(e, "static scratch lookup");
    const size_t nblk = (size_t)(n_rows + tnmc::kMlpRows - 1) / tnmc::kMlpRows;
    if (nblk * (tnmc::kMlpNParam + 1) > cap) return fail(TNMC_EINVAL, "static scratch too small");
    // every partial is written before it is read: nothing needs clearing
    e = tnmc::launch_mlp_grad(params, n_rows, feat, logit_lo, target_logit, scr, scr + nblk * tnmc::kMlpNParam,
                              adam_m, adam_v, grad_out, loss_out, lr, step, step > 0 ? 1 : 0, params,
                              static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mlp train launch");
    return TNMC_OK;
}

int tnmc_mlp_forward(const float *params, int32_t n_rows, const float *feat, int32_t bf16_weights, float *d_out,
                     void *stream) {
    if (!params || n_rows < 1 || !feat || !d_out) return fail(TNMC_EINVAL, "bad mlp_forward arguments");
    hipError_t e = tnmc::launch_mlp_forward(params, n_rows, feat, bf16_weights, d_out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mlp forward launch");
    return TNMC_OK;
}

void tnmc_free_env(tnmc_env *env) { delete env; }

int tnmc_philox_uniform(uint64_t seed, const uint32_t *c0, uint32_t c1, uint32_t c2, uint32_t stream_id,
                        int32_t n, double *out, void *stream) {
    if (n < 1 || !c0 || !out) return fail(TNMC_EINVAL, "bad philox arguments");
    hipError_t e = tnmc::launch_philox(seed, c0, c1, c2, stream_id, n, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "philox launch");
    return TNMC_OK;
}

const int64_t *tnmc_env_stats(const tnmc_env *env) {
    if (!env) return nullptr;
    return reinterpret_cast<const int64_t *>(env->ws + env->sweeps_off);
}

}  // extern "C"

// Schedule autotuner for uneven batches (tnmc_autotune): candidate
// schedules of the persistent pipeline are timed on a replica of the batch
// -- every instance cut down to its top-left (L / scale) x (L / scale)
// sub-lattice, same bond dimension, temperature and couplings -- and the
// best for the caller's objective (a percentile of per-instance completion
// time, the mean, or the whole batch) is returned.  Results are kept in a
// plain-text tuning cache keyed by the batch's composition, so a repeated
// batch is not timed again.  No device memory is allocated: the replica's
// couplings, outputs and workspace live in the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <tuple>
#include <vector>

#include "tnmc.h"

namespace tnmc {
int set_error(int code, const std::string &msg);
int env_batch(const tnmc_env *env);
}

namespace {

constexpr int kStats = 16;
constexpr double kTicksPerS = 1.0e8;   // wall_clock64: 100 MHz

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

struct Replica {
    std::vector<int32_t> L, chi;
    std::vector<double> beta;
    std::vector<int64_t> oh, ov;          // offsets of the replica couplings
    int64_t nh = 0, nv = 0;               // elements of J_h / J_v
    int64_t words = 0;                    // spin words per sample
};

Replica make_replica(const tnmc_problem *p, int scale) {
    Replica r;
    const int B = p->batch;
    r.L.resize(B); r.chi.assign(p->chi, p->chi + B); r.beta.assign(p->beta, p->beta + B);
    r.oh.resize(B); r.ov.resize(B);
    for (int i = 0; i < B; ++i) {
        const int L = std::max(4, std::min(p->L[i], p->L[i] / std::max(1, scale)));
        r.L[i] = L;
        r.oh[i] = r.nh; r.ov[i] = r.nv;
        r.nh += (int64_t)L * (L - 1);
        r.nv += (int64_t)(L - 1) * L;
        r.words += (int64_t)L * ((L + 63) / 64);
    }
    return r;
}

tnmc_problem replica_problem(const Replica &r, const tnmc_problem *p, const float *jh, const float *jv) {
    tnmc_problem q{};
    q.batch = p->batch;
    q.L = r.L.data(); q.chi = r.chi.data(); q.beta = r.beta.data();
    q.J_h = jh; q.J_v = jv; q.off_h = r.oh.data(); q.off_v = r.ov.data();
    q.coupling_kind = p->coupling_kind;
    q.flags = p->flags;
    return q;
}

struct Layout {
    size_t jh, jv, spins, logq, E, acc, chain, run, total;
};

Layout layout(const Replica &r, int B, int n, size_t run_bytes) {
    Layout o{};
    size_t off = 0;
    o.jh = off; off = align_up(off + sizeof(float) * r.nh);
    o.jv = off; off = align_up(off + sizeof(float) * r.nv);
    o.spins = off; off = align_up(off + sizeof(uint64_t) * r.words * n);
    o.logq = off; off = align_up(off + sizeof(double) * B * n);
    o.E = off; off = align_up(off + sizeof(double) * B * n);
    o.acc = off; off = align_up(off + (size_t)B * n);
    o.chain = off; off = align_up(off + sizeof(tnmc_chain) * B);
    o.run = off; off = align_up(off + run_bytes);
    o.total = off;
    return o;
}

uint64_t fnv1a(uint64_t h, const void *data, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(data);
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
    return h;
}

// The batch's composition, independent of instance order: sorted (L, chi,
// beta) triples, then precision, samples, objective and replica scale.
std::string cache_key(const tnmc_problem *p, int precision, int n, int objective, int scale) {
    std::vector<std::tuple<int32_t, int32_t, double>> v;
    for (int i = 0; i < p->batch; ++i) v.emplace_back(p->L[i], p->chi[i], p->beta[i]);
    std::sort(v.begin(), v.end());
    uint64_t h = 1469598103934665603ull;
    for (auto &t : v) {
        const int32_t a = std::get<0>(t), b = std::get<1>(t);
        const double c = std::get<2>(t);
        h = fnv1a(h, &a, 4); h = fnv1a(h, &b, 4); h = fnv1a(h, &c, 8);
    }
    char buf[160];
    std::snprintf(buf, sizeof buf, "tnmc-tune-v1 p%d n%d o%d s%d b%d %016llx", precision, n, objective, scale,
                  p->batch, (unsigned long long)h);
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, tnmc_tuning *out) {
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, key.c_str(), key.size()) != 0 || line[key.size()] != ' ') continue;
        int sched = 0, split = 0;
        double obj = 0;
        if (std::sscanf(line + key.size(), " %d %d %lf", &sched, &split, &obj) == 3) {
            out->schedule = sched; out->split = split; out->objective_s = obj;
            found = true;     // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, const tnmc_tuning &t) {
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %.9g\n", key.c_str(), t.schedule, t.split, t.objective_s);
    std::fclose(f);
}

double objective_of(std::vector<double> c, double makespan, int objective) {
    if (c.empty()) return makespan;
    std::sort(c.begin(), c.end());
    auto pct = [&](double q) {
        const double x = q * (c.size() - 1);
        const size_t i = (size_t)x;
        const double f = x - i;
        return i + 1 < c.size() ? c[i] * (1 - f) + c[i + 1] * f : c[i];
    };
    switch (objective) {
    case TNMC_OBJ_P99: return pct(0.99);
    case TNMC_OBJ_P50: return pct(0.50);
    case TNMC_OBJ_MEAN: {
        double s = 0;
        for (double x : c) s += x;
        return s / c.size();
    }
    default: return makespan;
    }
}

int chi_class(int chi) { return chi <= 16 ? 0 : (chi <= 32 ? 1 : 2); }

}  // namespace

extern "C" {

size_t tnmc_autotune_workspace_bytes(const tnmc_problem *p, int32_t precision, int32_t n_samples,
                                     int32_t replica_scale) {
    if (!p || !p->L || !p->chi || !p->beta || p->batch < 1 || n_samples < 1 || replica_scale < 1) return 0;
    Replica r = make_replica(p, replica_scale);
    tnmc_problem q = replica_problem(r, p, nullptr, nullptr);
    // the whole replica in one run, or split by bond class (the classes'
    // workspaces side by side)
    size_t one = tnmc_workspace_bytes(&q, precision, n_samples);
    if (one == 0) return 0;
    size_t split = 0;
    for (int cls = 0; cls < 3; ++cls) {
        std::vector<int32_t> L, chi;
        std::vector<double> beta;
        for (int i = 0; i < p->batch; ++i)
            if (chi_class(r.chi[i]) == cls) { L.push_back(r.L[i]); chi.push_back(r.chi[i]); beta.push_back(r.beta[i]); }
        if (L.empty()) continue;
        tnmc_problem s{};
        s.batch = (int32_t)L.size(); s.L = L.data(); s.chi = chi.data(); s.beta = beta.data();
        s.coupling_kind = p->coupling_kind;
        s.flags = p->flags;
        split += align_up(tnmc_workspace_bytes(&s, precision, n_samples));
    }
    return layout(r, p->batch, n_samples, std::max(one, split)).total;
}

int tnmc_autotune(const tnmc_problem *p, int32_t precision, int32_t n_samples, int32_t objective,
                  int32_t replica_scale, void *workspace, size_t workspace_bytes, const char *cache_path,
                  void *stream, tnmc_tuning *out) {
    if (!p || !out) return tnmc::set_error(TNMC_EINVAL, "problem and out must be non-NULL");
    if (!p->J_h || !p->J_v || !p->L || !p->chi || !p->beta || p->batch < 1)
        return tnmc::set_error(TNMC_EINVAL, "incomplete problem");
    if (objective < TNMC_OBJ_P99 || objective > TNMC_OBJ_MAKESPAN) return tnmc::set_error(TNMC_EINVAL, "unknown objective");
    if (replica_scale < 1 || n_samples < 1) return tnmc::set_error(TNMC_EINVAL, "replica_scale and n_samples must be >= 1");
    std::memset(out, 0, sizeof *out);
    const std::string key = cache_key(p, precision, n_samples, objective, replica_scale);
    if (cache_lookup(cache_path, key, out)) {
        out->from_cache = 1;
        return TNMC_OK;
    }
    const size_t need = tnmc_autotune_workspace_bytes(p, precision, n_samples, replica_scale);
    if (need == 0) return TNMC_EINVAL;   // the workspace query set the error text
    if (!workspace || workspace_bytes < need)
        return tnmc::set_error(TNMC_ENOSPACE, "autotune workspace needs " + std::to_string(need) + " bytes");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return tnmc::set_error(TNMC_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    const int B = p->batch, n = n_samples;
    Replica r = make_replica(p, replica_scale);
    const Layout lay = layout(r, B, n, need);   // (run region sized generously)
    float *jh = reinterpret_cast<float *>(ws + lay.jh), *jv = reinterpret_cast<float *>(ws + lay.jv);
    // the replica's couplings: top-left sub-lattice of every instance
    {
        int64_t ah = 0, av = 0;
        for (int i = 0; i < B; ++i) {
            const int L = p->L[i], Lr = r.L[i];
            const int64_t oh = p->off_h ? p->off_h[i] : ah, ov = p->off_v ? p->off_v[i] : av;
            ah += (int64_t)L * (L - 1);
            av += (int64_t)(L - 1) * L;
            if (Lr > L) return tnmc::set_error(TNMC_EINVAL, "replica larger than its instance");
            hipError_t e = hipMemcpy2DAsync(jh + r.oh[i], sizeof(float) * (Lr - 1), p->J_h + oh, sizeof(float) * (L - 1),
                                            sizeof(float) * (Lr - 1), Lr, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpy2DAsync(jv + r.ov[i], sizeof(float) * Lr, p->J_v + ov, sizeof(float) * L,
                                     sizeof(float) * Lr, Lr - 1, hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return tnmc::set_error(TNMC_EHIP, std::string("replica copy: ") + hipGetErrorString(e));
        }
    }
    uint64_t *spins = reinterpret_cast<uint64_t *>(ws + lay.spins);
    double *logq = reinterpret_cast<double *>(ws + lay.logq), *E = reinterpret_cast<double *>(ws + lay.E);
    uint8_t *acc = ws + lay.acc;
    tnmc_chain *chain = reinterpret_cast<tnmc_chain *>(ws + lay.chain);
    unsigned char *run = ws + lay.run;
    const size_t run_bytes = workspace_bytes - lay.run;

    // per-instance completion (seconds from the earliest start) of one env
    auto completion = [&](tnmc_env *env, std::vector<double> &c, int64_t &t0, int64_t &t1) {
        const int64_t *sd = tnmc_env_stats(env);
        std::vector<int64_t> h((size_t)kStats * tnmc::env_batch(env));
        if (hipMemcpy(h.data(), sd, h.size() * sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess) return false;
        for (size_t i = 0; i < h.size() / kStats; ++i) {
            t0 = std::min(t0, h[i * kStats + 4]);
            t1 = std::max(t1, h[i * kStats + 6]);
            c.push_back((double)h[i * kStats + 6]);
        }
        return true;
    };
    // candidate 0..2: one launch in each schedule order; candidate 3: one
    // launch per bond class, each on its own stream
    for (int cand = 0; cand < 4; ++cand) {
        std::vector<double> done;
        int64_t t0 = INT64_MAX, t1 = 0;
        std::vector<tnmc_env *> envs;
        int rc = TNMC_OK;
        if (hipMemsetAsync(chain, 0, sizeof(tnmc_chain) * B, st) != hipSuccess) return tnmc::set_error(TNMC_EHIP, "chain reset");
        if (cand < 3) {
            tnmc_problem q = replica_problem(r, p, jh, jv);
            tnmc_env *env = nullptr;
            rc = tnmc_run(&q, precision, run, run_bytes, n, 0x5A5A7u, 0, chain, 0x5A5A8u, 0, spins, logq, E, acc,
                          nullptr, nullptr, cand, stream, &env);
            if (rc) return rc;
            envs.push_back(env);
        } else {
            std::vector<hipStream_t> ss;
            size_t woff = 0;
            hipEvent_t ev0;
            if (hipEventCreateWithFlags(&ev0, hipEventDisableTiming) != hipSuccess) return tnmc::set_error(TNMC_EHIP, "event");
            (void)hipEventRecord(ev0, st);
            // per-class sub-problems (couplings of the replica, by offset)
            std::vector<std::vector<int32_t>> Ls(3), chis(3);
            std::vector<std::vector<double>> betas(3);
            std::vector<std::vector<int64_t>> ohs(3), ovs(3);
            for (int i = 0; i < B; ++i) {
                const int k = chi_class(r.chi[i]);
                Ls[k].push_back(r.L[i]); chis[k].push_back(r.chi[i]); betas[k].push_back(r.beta[i]);
                ohs[k].push_back(r.oh[i]); ovs[k].push_back(r.ov[i]);
            }
            int64_t sp_off = 0, ln_off = 0;
            for (int k = 2; k >= 0 && rc == TNMC_OK; --k) {
                if (Ls[k].empty()) continue;
                tnmc_problem q{};
                q.batch = (int32_t)Ls[k].size(); q.L = Ls[k].data(); q.chi = chis[k].data(); q.beta = betas[k].data();
                q.J_h = jh; q.J_v = jv; q.off_h = ohs[k].data(); q.off_v = ovs[k].data();
                q.coupling_kind = p->coupling_kind;
                q.flags = p->flags;
                const size_t wb = align_up(tnmc_workspace_bytes(&q, precision, n));
                hipStream_t s2;
                if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess) { rc = tnmc::set_error(TNMC_EHIP, "stream"); break; }
                ss.push_back(s2);
                (void)hipStreamWaitEvent(s2, ev0, 0);
                int64_t words = 0;
                for (int L : Ls[k]) words += (int64_t)L * ((L + 63) / 64);
                tnmc_env *env = nullptr;
                rc = tnmc_run(&q, precision, run + woff, wb, n, 0x5A5A7u, 0, chain + ln_off, 0x5A5A8u, 0,
                              spins + sp_off, logq + (size_t)ln_off * n, E + (size_t)ln_off * n, acc + (size_t)ln_off * n,
                              nullptr, nullptr, TNMC_SCHED_LONGEST_FIRST, s2, &env);
                if (rc) break;
                envs.push_back(env);
                woff += wb;
                sp_off += words * n;
                ln_off += q.batch;
            }
            for (hipStream_t s2 : ss) {
                (void)hipStreamSynchronize(s2);
                (void)hipStreamDestroy(s2);
            }
            (void)hipEventDestroy(ev0);
            if (rc) { for (auto *e : envs) tnmc_free_env(e); return rc; }
        }
        if (hipStreamSynchronize(st) != hipSuccess) return tnmc::set_error(TNMC_EHIP, "replica run");
        for (auto *e : envs) {
            if (!completion(e, done, t0, t1)) return tnmc::set_error(TNMC_EHIP, "statistics read");
            tnmc_free_env(e);
        }
        for (double &x : done) x = (x - (double)t0) / kTicksPerS;
        out->candidates_s[cand] = objective_of(done, (double)(t1 - t0) / kTicksPerS, objective);
    }
    int best = 0;
    for (int c = 1; c < 4; ++c) if (out->candidates_s[c] < out->candidates_s[best]) best = c;
    out->schedule = best < 3 ? best : TNMC_SCHED_LONGEST_FIRST;
    out->split = best == 3;
    out->objective_s = out->candidates_s[best];
    out->from_cache = 0;
    cache_store(cache_path, key, *out);
    return TNMC_OK;
}

}  // extern "C"

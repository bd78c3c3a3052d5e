/*
 * tnmc.h -- batched tensor-network Monte Carlo (TNMC) for 2D Ising spin
 * glasses on AMD Instinct MI355X (gfx950).
 *
 * The method (arXiv 2509.19006, "BatchTNMC"):
 *   1. tnmc_build_env  -- boundary-MPS cache: starting from the bottom row,
 *      apply each row's transfer MPO to the boundary MPS and truncate back to
 *      bond dimension chi (section 2.2, Fig. 2; section 3.2);
 *   2. tnmc_sample     -- row-by-row autoregressive sampling from the cached
 *      environments (section 3.3, Eqs. (3)-(5));
 *   3. tnmc_energy     -- exact energies, Eq. (1);
 *   4. tnmc_accept     -- Metropolis independence accept/reject, Eq. (10).
 * Every call is batched over disorder instances x samples (section 3.4).
 *
 * Conventions shared by every entry point
 *  - Lattice: open L x L square lattice.  J_h[r][c] couples (r,c)-(r,c+1)
 *    (shape L x (L-1), row-major); J_v[r][c] couples (r,c)-(r+1,c) (shape
 *    (L-1) x L).  Each bond appears once.  Spins are -1/+1.
 *  - Spins are bit-packed: instance i, sample n, row r is W_i = ceil(L_i/64)
 *    uint64 words; bit (c mod 64) of word c/64 is 1 iff spin (r,c) is +1.
 *    Instances follow each other in batch order, samples within an
 *    instance, rows within a sample:  word offset of (i, n, r) =
 *    n_samples * sum_{j<i} L_j*W_j + (n*L_i + r)*W_i.
 *  - Per-sample outputs (log q, energies, accept flags) are [batch][n_samples].
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are read during the call only.  The library never allocates
 *    device memory: caches and scratch live in a caller-provided workspace.
 *  - `stream` is a hipStream_t passed as void*; all device work is enqueued
 *    on it and the call returns without synchronising.  The caller keeps
 *    device buffers alive until that work completes.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 *    (seed & 0xffffffff, seed >> 32).  Site draw of sample n (global index,
 *    i.e. sample_offset + n) at site (r,c) of instance i uses counter
 *    (r*L_i + c, n, i, 0); the accept draw of proposal k uses (k, 0, i, 1).
 *    The uniform is ((w0>>5)*2^26 + (w1>>6)) * 2^-53 and a spin is +1 iff
 *    uniform < p(+1).
 *  - Errors: every int-returning function returns TNMC_OK (0) or a
 *    negative TNMC_E* code; tnmc_last_error() then describes it (thread
 *    local).  Arguments are validated before any device work is enqueued;
 *    on error nothing is enqueued and outputs are untouched.  Errors of
 *    already-enqueued device work (TNMC_EHIP) surface at a later call.
 */
#ifndef TNMC_H
#define TNMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define TNMC_OK        0
#define TNMC_EINVAL   -1   /* bad shape, chi, beta, null pointer, count     */
#define TNMC_ENOSPACE -2   /* workspace smaller than tnmc_workspace_size    */
#define TNMC_EHIP     -3   /* HIP runtime or launch error                   */
#define TNMC_ENOTSUP  -4   /* precision / size combination not built        */
#define TNMC_ENUMERIC -5   /* NaN / Inf in a log-scale, or a Jacobi SVD that
                              stopped at its sweep limit (tnmc_env_check)   */

/* ---- precision of the boundary-MPS build and of the sampler ----------- */
/* Every form keeps log-scales, ln Z, log q, p(+1), the Metropolis log-ratio
 * and the accept decision in float64.  In the float builds a truncation
 * whose float32 one-sided Jacobi does not reach orthogonality (its columns'
 * relative inner products below 2 eps sqrt(K)) within 40 sweeps is redone
 * in float64 from the same float32 inputs (slot 11 of tnmc_env_stats counts
 * these).  In the float forms the sampler's two
 * contractions per site run on the matrix cores for chi <= 32 (the sample
 * vectors are float32 and enter 16-bit products as hi + lo pairs) and on the
 * vector unit in float32 for chi > 32.                                    */
#define TNMC_FP64        0 /* build, cache and sampler in float64 (vector    */
                           /* unit)                                          */
#define TNMC_FP32        1 /* build and cache in float32; sampler products   */
                           /* on float32 matrix cores                        */
#define TNMC_MIXED_BF16  2 /* float32 build, cache stored in bfloat16; the   */
                           /* sampler's products on bf16 matrix cores with   */
                           /* float32 accumulation (the stored entries enter */
                           /* exactly)                                       */
#define TNMC_MIXED_FP16  3 /* as MIXED_BF16 with a float16 cache and float16 */
                           /* matrix cores                                   */
#define TNMC_MIXED_BF16X3 4 /* float32 build and cache; the sampler's       */
                           /* products on bf16 matrix cores with both        */
                           /* operands split into hi + lo parts (hi*hi +     */
                           /* hi*lo + lo*hi, float32 accumulation)           */

/* what the couplings are, for the exact-energy outputs of tnmc_energy     */
#define TNMC_COUPLING_GENERAL 0  /* any float32 couplings                    */
#define TNMC_COUPLING_PMJ     1  /* every coupling is an integer (+-J): the   */
                                 /* energy is also available as int32        */
#define TNMC_COUPLING_GRID20  2  /* multiples of 2^-20 with |J| < 8: float64 */
                                 /* energy sums are exact in any order       */

/* largest bond dimension and lattice side the kernels are built for */
/* launch orders of tnmc_run */
#define TNMC_SCHED_LONGEST_FIRST  0  /* decreasing (L-1) L chi^3: shortest batch */
#define TNMC_SCHED_SHORTEST_FIRST 1  /* increasing cost: small instances done early */
#define TNMC_SCHED_AS_GIVEN       2  /* the problem's instance order            */

#define TNMC_CHI_MAX  64
#define TNMC_L_MAX    1024

/* Problem description: a batch of independent instances (section 3.4).   */
typedef struct tnmc_problem {
    int32_t        batch;   /* number of instances B >= 1                     */
    const int32_t *L;       /* host [B]   lattice side, 2 <= L_i <= TNMC_L_MAX */
    const int32_t *chi;     /* host [B]   bond dimension, 2 <= chi_i <= 64    */
    const double  *beta;    /* host [B]   inverse temperature, finite, >= 0   */
    const float   *J_h;     /* device     horizontal couplings, see above     */
    const float   *J_v;     /* device     vertical couplings                  */
    const int64_t *off_h;   /* host [B] or NULL: element offset of instance i */
    const int64_t *off_v;   /*   in J_h / J_v; NULL = packed in batch order   */
    int32_t coupling_kind;  /* TNMC_COUPLING_*, declares the exact-energy mode */
    int32_t flags;          /* TNMC_ALTERNATE_SWEEPS, TNMC_FORCE_F64_FALLBACK,  */
                            /* TNMC_SHORT_WAITS, or 0                         */
} tnmc_problem;

/* Problem flag: the compression of every second row (the rows L-3, L-5, ...
 * counted from the bottom) runs mirrored -- QR sweep right to left, then the
 * truncating SVD sweep left to right -- so that each row's sites are final
 * in the order the next row's QR sweep consumes them.  Another canonical
 * compression (section 2.2; the paper does not list its compress routine):
 * identical in the exact regime, different at the level of the truncation
 * error otherwise.  The cache is always stored in lattice order.  In the
 * float builds with chi <= 32 (largest chi of the batch) this order also
 * lets the build pipeline its rows: row r-1's QR sweep runs on two waves
 * of the workgroup beside row r's SVD sweep on the other two, site by site
 * (the workspace then holds two rows of QR scratch).                      */
#define TNMC_ALTERNATE_SWEEPS 1

/* Problem flag for the float builds: stop the float32 Jacobi after one
 * sweep, so that every truncation still rotating after it takes the
 * float64 redo (an exercise of that path: the build slows down, results
 * stay within the float forms' tolerance).  No effect on TNMC_FP64.       */
#define TNMC_FORCE_F64_FALLBACK 2

/* Problem flag, a test of the row-pipelined build's failure path: every
 * hand-over wait between its two pairs of waves gives up after one poll,
 * so the build soon records a lost hand-over, finishes without waiting
 * (its cache is then not to be used) and tnmc_env_check reports
 * TNMC_ENUMERIC.  No effect on the other builds.                           */
#define TNMC_SHORT_WAITS 8

/* Per-instance Metropolis chain state (device memory, caller owned).
 * Zero-fill before the first tnmc_accept call of a chain.                */
typedef struct tnmc_chain {
    double  cur_logq;       /* log q of the current state                    */
    double  cur_E;          /* energy of the current state                   */
    int64_t cur_index;      /* global proposal index of the current state    */
    int64_t n_acc;          /* accepted trials so far                        */
    int64_t n_trials;       /* trials so far (the initialising proposal is   */
                            /* not a trial)                                  */
    int64_t initialised;    /* 0 until the first proposal has been taken     */
} tnmc_chain;

typedef struct tnmc_env tnmc_env;   /* opaque; host metadata into workspace */

/* Learned proposal correction (not part of the paper's method; the exact
 * Metropolis step of Eq. (10) keeps sampling unbiased whatever it does).
 * A 3-layer tanh MLP, widths 64/64/1, adds a correction d to every site's
 * TN logit.  Its 64 input features at site (r,c) are: the horizontal
 * couplings of rows r-2..r+2, columns c-2..c+1 (20), the vertical couplings
 * of rows r-2..r+1, columns c-2..c+2 (20), the already-sampled spins of rows
 * r-2, r-1 at columns c-2..c+2 (10) and of row r at c-2, c-1 (2), the TN
 * logit clipped to [-30,30] and divided by 8 (1), zeros (11); every slot
 * outside the lattice is zero.  Parameters are one float32 vector of
 * TNMC_MLP_NPARAM values, row-major [out][in]:
 *   W1 [64][64] | b1 [64] | W2 [64][64] | b2 [64] | W3 [64] | b3 [1]
 * Inference inside tnmc_sample runs on the bf16 matrix cores: weights
 * rounded to bfloat16, activations entering as hi + lo bfloat16 pairs,
 * float32 accumulation.  Supported with TNMC_FP32 and chi <= 16.          */
#define TNMC_MLP_IN     64
#define TNMC_MLP_HIDDEN 64
#define TNMC_MLP_NPARAM 8385
typedef struct tnmc_mlp {
    const float *params;    /* device float [TNMC_MLP_NPARAM] */
} tnmc_mlp;

/* Bytes of workspace tnmc_build_env + tnmc_sample need for this problem at
 * this precision with up to max_samples samples per instance per call:
 * the cache (sections 3.2 and 3.4: every row of every instance stays in
 * device memory), the build's scratch and the sampler's right environments.
 * Returns 0 on a bad problem (tnmc_last_error says why).                   */
size_t tnmc_workspace_bytes(const tnmc_problem *p, int32_t precision,
                            int32_t max_samples);

/* The same figure through a status code: TNMC_EINVAL on a bad problem,
 * TNMC_ENOTSUP on a precision / size combination that is not built.       */
int tnmc_workspace_size(const tnmc_problem *p, int32_t precision,
                        int32_t max_samples, size_t *bytes_out);

/* Build the boundary-MPS cache of every instance (sections 2.2 and 3.2).
 *  workspace  device, >= tnmc_workspace_size bytes, 256-byte aligned; the
 *             cache lives there until the env is freed or rebuilt.
 *  logz_out   device double [B] or NULL: the tensor-network estimate of
 *             ln Z (exact when chi_i >= 2^floor(L_i/2)).
 *  env_out    receives a new env (free with tnmc_free_env).  It keeps copies
 *             of the host arrays of *p and the device pointers J_h / J_v,
 *             which must stay valid while the env is used.
 * The compression is a left-to-right QR sweep followed by a right-to-left
 * truncating SVD sweep keeping the chi largest singular values per bond. */
int tnmc_build_env(const tnmc_problem *p, int32_t precision,
                   void *workspace, size_t workspace_bytes, void *stream,
                   tnmc_env **env_out, double *logz_out);

/* The whole hot path per instance in one persistent launch, meant for
 * uneven batches (instances of different L, chi, beta): each workgroup takes
 * the next instance in longest-first order and runs its cache build
 * (section 3.2, as tnmc_build_env), its n_samples draws (section 3.3, as
 * tnmc_sample without forcing or correction, sample tiles one after
 * another), their energies (Eq. (1), as tnmc_energy) and its Metropolis
 * chain (Eq. (10), as tnmc_accept with beta_i from the problem).  Results
 * equal those of the four separate calls with the same arguments; an
 * instance is finished as soon as its own work is, which the env's
 * statistics record (slot 6: completion tick).
 *  workspace, workspace_bytes, logz_out, env_out   as tnmc_build_env (the
 *             workspace needs room for one sample tile).
 *  sample_seed, sample_offset   as tnmc_sample's seed and sample_offset.
 *  chain, accept_seed, step_offset   as tnmc_accept's.
 *  spins_out, logq_out, E_out, accepted_out, state_out   as the outputs of
 *             tnmc_sample, tnmc_energy and tnmc_accept (state_out may be
 *             NULL).
 *  schedule   TNMC_SCHED_*: the order in which workgroups take instances
 *             (tnmc_build_env always runs longest-first).
 * Errors as tnmc_build_env; on error no env is returned.                    */
int tnmc_run(const tnmc_problem *p, int32_t precision, void *workspace,
             size_t workspace_bytes, int32_t n_samples, uint64_t sample_seed,
             uint64_t sample_offset, tnmc_chain *chain, uint64_t accept_seed,
             uint64_t step_offset, uint64_t *spins_out, double *logq_out,
             double *E_out, uint8_t *accepted_out, int64_t *state_out,
             double *logz_out, int32_t schedule, void *stream,
             tnmc_env **env_out);

/* Schedule autotuner for tnmc_run on uneven batches.  Candidates: one
 * persistent launch in each TNMC_SCHED_* order, and one launch per bond
 * class (chi <= 16, <= 32, > 32) each on its own stream (smaller classes
 * need less shared memory, so their workgroups can share a compute unit
 * with the long builds).  Each is timed on a replica of the batch -- every
 * instance cut to its top-left max(4, L/replica_scale) sub-lattice, same
 * chi, beta and coupling values -- from the device clock the kernels record,
 * and the best for `objective` is returned.  With cache_path non-NULL the
 * result is read from / appended to that text file, keyed by the batch's
 * composition (the multiset of (L, chi, beta)), precision, n_samples,
 * objective and replica_scale; a cached answer does no device work.
 *  workspace  device, >= tnmc_autotune_workspace_bytes, 256-byte aligned
 *             (the replica's couplings, outputs and run workspace).
 *  stream     the replica runs are synchronised before the call returns.  */
#define TNMC_OBJ_P99      0   /* 99th percentile of per-instance completion  */
#define TNMC_OBJ_P50      1   /* median per-instance completion              */
#define TNMC_OBJ_MEAN     2   /* mean per-instance completion                */
#define TNMC_OBJ_MAKESPAN 3   /* completion of the whole batch               */
typedef struct tnmc_tuning {
    int32_t schedule;         /* TNMC_SCHED_* for tnmc_run                     */
    int32_t split;            /* 1: run each bond class as its own tnmc_run on */
                              /*    its own stream (schedule longest-first)    */
    double  objective_s;      /* the chosen candidate's objective (seconds, on */
                              /* the replica)                                  */
    double  candidates_s[4];  /* longest-first, shortest-first, as given,      */
                              /* split by class (zero when read from cache)   */
    int32_t from_cache;       /* 1 if read from the tuning cache               */
} tnmc_tuning;
size_t tnmc_autotune_workspace_bytes(const tnmc_problem *p, int32_t precision,
                                     int32_t n_samples, int32_t replica_scale);
int tnmc_autotune(const tnmc_problem *p, int32_t precision, int32_t n_samples,
                  int32_t objective, int32_t replica_scale, void *workspace,
                  size_t workspace_bytes, const char *cache_path, void *stream,
                  tnmc_tuning *out);

/* Draw (or score) n_samples configurations per instance (section 3.3).
 *  seed, sample_offset  Philox key and first global sample index; the
 *                sample counter is 32 bits wide, so sample_offset +
 *                n_samples must not exceed 2^32 (TNMC_EINVAL otherwise).
 *  forced_spins  device, NULL to sample; otherwise configurations in the
 *                packed layout to be scored (teacher forcing): the sampler
 *                evaluates their log q and logits instead of drawing.
 *  mlp           NULL for the plain TN proposal, else the learned
 *                correction added to every logit before the draw
 *                (TNMC_FP32 envs with chi <= 16; TNMC_ENOTSUP otherwise).
 *  spins_out     device uint64, packed layout (may equal forced_spins).
 *  logq_out      device double [B][n_samples]: log q of each configuration.
 *  logits_out    device float [B][n_samples][L_i*L_i] or NULL: the logit of
 *                p(+1) at every site (after the MLP correction if any).
 * n_samples must not exceed the max_samples the workspace was sized for.  */
int tnmc_sample(tnmc_env *env, int32_t n_samples, uint64_t seed,
                uint64_t sample_offset, const uint64_t *forced_spins,
                const tnmc_mlp *mlp, uint64_t *spins_out, double *logq_out,
                float *logits_out, void *stream);

/* Exact energies E(s) = -sum J s s over every bond once (Eq. (1)) of
 * n_samples configurations per instance of the problem (its L, couplings
 * and offsets; chi and beta are not read and may be NULL).
 *  spins      device, packed layout for n_samples per instance.
 *  E_out      device double [B][n_samples].  Exact for integer couplings
 *             and for couplings on the 2^-20 grid with |J| < 8.
 *  E_int_out  device int32 [B][n_samples] or NULL: the same energy summed
 *             in integer arithmetic; only with coupling_kind
 *             TNMC_COUPLING_PMJ (TNMC_EINVAL otherwise).  An instance with
 *             a coupling that is not an integer gets INT32_MIN.
 * Instances are processed in runs of equal L whose coupling offsets are
 * evenly spaced (one launch per run).                                      */
int tnmc_energy(const tnmc_problem *p, int32_t n_samples, const uint64_t *spins,
                double *E_out, int32_t *E_int_out, void *stream);

/* Replica overlap, the spin-glass order parameter: two Markov chains (a, b)
 * run on the same instances with independent proposals; after each of this
 * call's n_samples steps k, q[i][k] = (1/L_i^2) sum_sites s^a s^b of the two
 * chains' current states.  The states are given by the global proposal
 * indices tnmc_accept wrote (state_a / state_b, device int64 [B][n_samples])
 * and read from this call's proposals (spins_a / spins_b, packed layout),
 * proposal index = state - state_offset; a state from an earlier call gives
 * NaN for that step.  q_out: device double [B][n_samples].  Moments of q
 * over steps and disorders give <q^2>, <q^4> and the Binder ratio.          */
int tnmc_overlap(const tnmc_problem *p, int32_t n_samples, const uint64_t *spins_a,
                 const int64_t *state_a, const uint64_t *spins_b, const int64_t *state_b,
                 uint64_t state_offset, double *q_out, void *stream);

/* Metropolis independence step over each instance's proposals in index
 * order (Eq. (10)): with current state x and candidate k,
 *   delta = (logq_x - logq_k) + beta * (E_x - E_k)   (no fused operations)
 * and k is accepted iff delta >= 0 or u_k < exp(delta).  On a chain's first
 * call its first proposal initialises it (flag 1, not a trial).
 *  logq, E      device double [batch][n_samples]
 *  beta         device double [batch]
 *  chain        device tnmc_chain [batch], updated in place
 *  step_offset  global index of this call's first proposal (Philox counter;
 *               step_offset + n_samples must not exceed 2^32)
 *  accepted_out device uint8 [batch][n_samples] (1 = accepted)
 *  state_out    device int64 [batch][n_samples]: global index of the chain
 *               state after each proposal (NULL allowed).                  */
int tnmc_accept(int32_t batch, int32_t n_samples, const double *logq,
                const double *E, const double *beta, tnmc_chain *chain,
                uint64_t seed, uint64_t step_offset, uint8_t *accepted_out,
                int64_t *state_out, void *stream);

/* Features of every site of n_samples configurations per instance of the
 * env (layout above), for training the learned correction.
 *  spins      device, packed layout
 *  logits_lo  device float [B][n_samples][L_i*L_i]: the TN logits of the
 *             same configurations (tnmc_sample's logits_out)
 *  feat_out   device float [B][n_samples][L_i*L_i][64]                      */
int tnmc_mlp_features(const tnmc_env *env, int32_t n_samples, const uint64_t *spins,
                      const float *logits_lo, float *feat_out, void *stream);

/* Floats of scratch tnmc_mlp_train_step needs for n_rows rows.            */
size_t tnmc_mlp_scratch_floats(int32_t n_rows);

/* One optimisation step of the learned correction on n_rows feature rows.
 * Loss: mean over rows of the cross-entropy between sigmoid(logit_lo + d)
 * and the soft target sigmoid(target_logit).  The gradient is summed in a
 * fixed order (deterministic).  With step >= 1 an Adam update (Kingma & Ba;
 * beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with this step number)
 * is applied to params / adam_m / adam_v (device float [TNMC_MLP_NPARAM]);
 * with step == 0 nothing is updated.
 *  grad_out   device float [TNMC_MLP_NPARAM] or NULL: the mean gradient
 *  loss_out   device float [1] or NULL: the mean loss before the update
 *  scratch    device float [tnmc_mlp_scratch_floats(n_rows)]              */
int tnmc_mlp_train_step(float *params, float *adam_m, float *adam_v, int32_t n_rows,
                        const float *feat, const float *logit_lo, const float *target_logit,
                        float lr, int32_t step, float *scratch, float *grad_out,
                        float *loss_out, void *stream);

/* tnmc_mlp_train_step without the scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training or
 * serving loops, harnesses that forbid allocation): the partial gradients
 * live in a static device array of the library, one per GPU for the life of
 * the process, sized for n_rows <= TNMC_MLP_NOALLOC_MAX_ROWS (8.6 MB); more
 * rows give TNMC_EINVAL.  The call allocates nothing.  Every call on a GPU
 * shares that GPU's array and leaves it holding the last call's partials:
 * calls that overlap on one GPU (concurrent streams, threads) race and must
 * be serialised by the caller.  Results are bit-identical to
 * tnmc_mlp_train_step with the same arguments.                             */
#define TNMC_MLP_NOALLOC_MAX_ROWS 16384
int tnmc_mlp_train_step_noalloc(float *params, float *adam_m, float *adam_v, int32_t n_rows,
                                const float *feat, const float *logit_lo, const float *target_logit,
                                float lr, int32_t step, float *grad_out, float *loss_out,
                                void *stream);

/* The correction d for n_rows feature rows (device float [n_rows]); with
 * bf16_weights != 0 the weights are first rounded to bfloat16, as inside
 * tnmc_sample.                                                            */
int tnmc_mlp_forward(const float *params, int32_t n_rows, const float *feat,
                     int32_t bf16_weights, float *d_out, void *stream);

/* Numeric health of an env's build: synchronises the stream, then returns
 * TNMC_ENUMERIC if any instance has a row log-scale that is not finite, or
 * a truncation whose one-sided Jacobi stopped at its sweep limit (40
 * sweeps) before the columns were orthogonal to working precision;
 * TNMC_OK otherwise.  tnmc_last_error() names the first such instance.
 * The counts per instance are slots 8 and 9 of tnmc_env_stats.  A ln Z that
 * is not finite with a sound cache is not an error: at small chi the
 * truncated network's total (sum over every configuration) can come out
 * zero or negative -- the estimate is undefined, sampling is unaffected --
 * and slot 10 records it.                                                 */
int tnmc_env_check(const tnmc_env *env, void *stream);

/* Release an env (host memory only; the workspace stays the caller's).    */
void tnmc_free_env(tnmc_env *env);

/* Description of the last error on this thread ("" if none).             */
const char *tnmc_last_error(void);

/* Philox uniforms for counters (c0[k], c1, c2, stream) under key(seed),
 * written to out[k] (device double [n]); c0 is a device uint32 [n].  The
 * same generator the sampler and the accept step draw from.               */
int tnmc_philox_uniform(uint64_t seed, const uint32_t *c0, uint32_t c1,
                        uint32_t c2, uint32_t stream_id, int32_t n,
                        double *out, void *stream);

/* Statistics of this env (device int64 [B][16], valid once the work has
 * completed on its stream), per instance: the total number of Jacobi sweeps
 * over all truncations; wall-clock ticks (100 MHz device counter) spent in
 * the QR sweeps, in the SVD sweeps, and inside the Jacobi iterations of the
 * SVD sweeps; the ticks at which the instance's build started and ended;
 * the tick at which the first sample tile of the last tnmc_sample call
 * ended (the only tile when n_samples <= 256); the ticks spent in the
 * Householder factorisations (a part of the QR sweeps); the number of
 * truncations whose Jacobi reached the sweep limit; the number of row
 * log-scales that are not finite; 1 if ln Z is undefined (the truncated
 * network's total was not positive); the number of truncations whose
 * float32 Jacobi did not converge and were redone in float64 (float builds;
 * slot 8 then counts the float64 Jacobi reaching its limit); 1 if the
 * row-pipelined build lost a hand-over between its waves (a bounded wait
 * ran out; tnmc_env_check reports it as TNMC_ENUMERIC); slots 13-15 are
 * zero.  The
 * build processes instances in decreasing order of estimated cost
 * (L-1) L chi^3.
 * NULL for a NULL env.                                                    */
const int64_t *tnmc_env_stats(const tnmc_env *env);

#ifdef __cplusplus
}
#endif
#endif /* TNMC_H */

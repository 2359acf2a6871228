/*
 * phia.h -- C ABI of the MI355X (gfx950) library for the data-parallel sweep
 * of the Parallel Hamiltonian Monte Carlo Ising Annealer (PHIA; Wang et al.,
 * "Parallel Ising Annealer via Gradient-based Hamiltonian Monte Carlo").
 *
 * Problem (Sec. 2.1, Eq. 2): minimise E(s) = -sum_{i<j} J_ij s_i s_j -
 * sum_i h_i s_i over s in {-1,+1}^N, with real couplings J_ij = J_ji and
 * fields h_i held in fixed point (Sec. 2.2): every value is an integer multiple
 * of sigma = 2^-f.  The library runs R independent replicas of the sweep
 * (Eq. 5-8, App. A A7) and keeps each replica's best configuration
 * (App. B, Table 3, state 5).
 *
 * Conventions for every entry point:
 *  - Plain pointers; arrays named "host" are caller-owned host memory and are
 *    only read (inputs) or written (outputs) during the call.  The library
 *    copies inputs at create time and owns all device memory of a problem
 *    until phia_destroy.
 *  - Matrices are dense row-major; spin arrays are int8 with values +1 / -1.
 *  - Energies in "units" are exact integers in units of sigma = 2^-frac_bits.
 *  - Every function returns PHIA_OK (0) or a negative phia_status; on error
 *    phia_last_error() gives a message (thread-local, valid until the next
 *    call on the same thread).  No C++ exception crosses this boundary.
 *  - A device fault or a timed-out group barrier poisons the handle: later
 *    calls return PHIA_EDEVICE.
 *  - One host thread at a time per problem handle.
 */
#ifndef PHIA_H
#define PHIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct phia_problem phia_problem;

typedef enum {
    PHIA_OK = 0,
    PHIA_EINVAL = -1,   /* bad argument (null pointer, size out of range)            */
    PHIA_ENOTSYM = -2,  /* J is not symmetric                                        */
    PHIA_EDIAG = -3,    /* J has a nonzero diagonal entry                            */
    PHIA_ERANGE = -4,   /* value off the 2^-f grid (quantize = 0) or too large       */
    PHIA_ENOMEM = -5,   /* device or host allocation failed                          */
    PHIA_EDEVICE = -6,  /* HIP error, device fault or group-barrier timeout          */
    PHIA_ESTATE = -7    /* call out of order (e.g. phia_best before any anneal)      */
} phia_status;

/* Arithmetic used for the quasi-gradient J.s (Eq. 6).  Every path computes the
 * same exact integer field, so results are identical across paths. */
typedef enum {
    PHIA_PATH_AUTO = 0,     /* I8 if |J| <= 127 units, else BF16HILO, else FP32; ELL
                               for sparse rows with 512 < Np <= 4096 (at most Np/64
                               nonzeros in every row)                                */
    PHIA_PATH_FP32 = 1,     /* FP32 couplings, VALU dot products (plain sweep)       */
    PHIA_PATH_I8 = 2,       /* int8 couplings, int8 MFMA with int32 accumulation;
                               with few replicas the VALU int8 dot-product sweep
                               (see phia_anneal_start)                              */
    PHIA_PATH_BF16HILO = 3, /* J = 256 hi + lo, two BF16 MFMA planes, FP32 accumulate */
    PHIA_PATH_ELL = 4       /* sparse rows: D (index, coupling) slots per row, spin
                               gathers on the VALUs; |J| <= 32767 units, N <= 4096 */
} phia_path;

typedef struct {
    int32_t frac_bits;  /* f in [0, 15]; -1 picks the smallest f that holds J, h exactly */
    int32_t quantize;   /* 0: reject off-grid values; 1: round half to even onto the grid */
    int32_t path;       /* phia_path                                                     */
    int32_t device;     /* HIP device ordinal                                            */
    void* stream;       /* hipStream_t for all work of this problem; NULL = null stream  */
    int32_t defer_upload; /* 0: J and h go to the device in phia_create; 1: they stay in
                           host memory until the first anneal (or batch plan) needs
                           them, and a served request that ends releases them again,
                           so queued requests hold no device memory                 */
} phia_options;

/* Annealing schedule.  The inverse temperature of step k is betas[k] when
 * betas != NULL (host array of `steps` floats), else the linear table
 * beta_k = float(b0 + ((b1 - b0) * k) / (steps - 1)) evaluated in double.
 * eps is the integrator step of A7, gamma the surrogate slope of Eq. 7-8,
 * refresh_L the number of steps between momentum draws (v ~ N(0, I) at every
 * k with k mod refresh_L == 0, k = 0 included).  deriv_mode picks the factor
 * of the kick: PHIA_DERIV_TANH, the sech^2(gamma x) of Eq. 8, or
 * PHIA_DERIV_POLY2, the quadratic polynomial that the FPGA uses in its place
 * (Sec. 2.3; coefficients not given there, here max(0, 1 - u^2 / 2.25):
 * equal to sech^2 at 0 and of equal area). */
typedef enum { PHIA_DERIV_TANH = 0, PHIA_DERIV_POLY2 = 1 } phia_deriv;

/* metropolis = 1 adds the accept/reject step of App. A (H(x, v) = beta E(sgn x)
 * + x.x/2 + v.v/2) and Table 3 state 4 (acceptance and temperature): at every
 * k > 0 with k mod refresh_L == 0 the trajectory of steps [k - refresh_L, k)
 * is accepted with probability min(1, exp(-dH)), else x returns to its start
 * (the first trajectory, which starts at the initial draw, is taken as it is).
 * dH uses the beta of the trajectory's last step times a per-replica
 * multiplier lam (starts at 1), with x.x + v.v on the grid 2^-24 (each term
 * capped at 2^22) and the uniform of counter (0, trajectory, replica, 2) of
 * the Gaussian stream's generator.  After every decision lam is multiplied by
 * mh_up (accepted) or mh_down (rejected) and clamped to [2^-10, 2^10]; lam
 * scales beta in the kick as well (c_k lam).  mh_up = mh_down = 1 keeps the
 * schedule fixed.  metropolis = 0 ignores mh_up and mh_down.  Metropolis runs
 * use the one-block-per-workgroup sweep (never the interleaved one). */
typedef struct {
    float beta0, beta1;
    const float* betas;
    float eps, gamma;
    int64_t refresh_L;
    int32_t deriv_mode;     /* phia_deriv; 0 = TANH                                    */
    int32_t metropolis;     /* 0: no accept/reject step; 1: accept or reject every
                               trajectory of refresh_L steps                          */
    float mh_up, mh_down;   /* > 0, finite: factors of the beta multiplier            */
    int32_t initial_kick;   /* 0: A7 as written; 1: the initial-kick variant of
                               Table 3 state 2 -- after every momentum draw, half a
                               kick (step eps/2) at the current x with the field of
                               its spins and the step's beta, so that each
                               trajectory's drift-kick steps form a leapfrog.  Runs
                               on the VALU sweep (FP32, I8 and ELL paths; else
                               PHIA_ERANGE at phia_anneal_start), not with
                               metropolis, not in batches or the server (EINVAL)  */
} phia_schedule;

typedef struct {
    int32_t N, Np;          /* spins and padded spins (multiple of 64)               */
    int32_t path;           /* resolved phia_path                                    */
    int32_t frac_bits;      /* f                                                     */
    int32_t exact;          /* 1 if the couplings were on the grid (no rounding)     */
    int32_t group;          /* workgroups that share one replica block's J (>= 1)    */
    int32_t replicas;       /* R of the current anneal (0 if none)                   */
    int32_t rows_per_block; /* replicas per workgroup block                          */
    int32_t j_in_lds;       /* 1: each workgroup's coupling slice resides in LDS     */
    int32_t sweep_kernel;   /* 0: one replica block per workgroup; 1 (int8 operands)
                               and 2 (FP4 operands): two 16-replica sub-blocks per
                               workgroup whose steps alternate, so the column-split
                               exchange of one overlaps the other's compute; 3: the
                               persistent batch sweep (phia_batch_*); 4: the VALU
                               sweep, all columns of rows_per_block replicas per
                               workgroup (FP32 and ELL paths, I8 with few replicas) */
    int64_t steps;          /* T of the current anneal                               */
    int64_t step;           /* next step to run                                      */
    int64_t max_abs_J;      /* max |J| in units                                      */
    size_t device_bytes;    /* device memory held by the problem                     */
    int32_t group_on_one_xcd; /* 1: a group's workgroups share one XCD; 0: member m of
                               every group on XCD m mod 8 (each XCD's L2 then holds
                               only its members' J slices)                           */
    int32_t incremental;    /* 1: the sweep updates J.s by the flip-incremental
                               product (see phia_set_incremental)                    */
} phia_info;

/* Create a problem from real couplings.  J: host, N*N doubles, row-major,
 * symmetric with a zero diagonal (the i<j sum of Eq. 2 read as a full
 * symmetric matrix).  h: host, N doubles, or NULL for h = 0.  N in
 * [1, 16384] (else PHIA_EINVAL), and within what the resolved path's sweep
 * holds (else PHIA_ERANGE): N <= 5056 on I8 (4992 for metropolis
 * schedules, which then fail at phia_anneal_start), N <= 2496 on BF16HILO,
 * N <= 4096 on FP32 and ELL (ELL also needs |J| <= 32767 units).  opt may be NULL (frac_bits = -1, quantize = 0, AUTO,
 * device 0, null stream).  On success *out owns device copies of J and h. */
phia_status phia_create(const double* J, const double* h, int32_t N,
                        const phia_options* opt, phia_problem** out);

/* Run a whole anneal: phia_anneal_start, phia_anneal_run(steps) and a
 * synchronisation.  replicas in [1, 1<<20], steps >= 1, seed keys the
 * counter-based Gaussian stream (Philox4x64-10); replica r always draws the
 * same numbers for the same seed, whatever else runs. */
phia_status phia_anneal(phia_problem* p, int32_t replicas, int64_t steps,
                        const phia_schedule* schedule, uint64_t seed);

/* phia_anneal for callers that cannot allocate device memory (code that runs
 * where hipMalloc is not allowed: tight serving loops, harnesses that forbid
 * it).  It allocates and frees nothing.  The caller passes device buffers
 * for the replica state and records of `replicas` replicas, with
 * Np = phia_info.Np (N padded to a multiple of 64):
 *   x, v      float [replicas][Np]   final positions and momenta
 *   bestE     int64 [replicas]       record energies in units of 2^-f
 *   bestS     int8  [replicas][Np]   record states (+1 / -1; padding 0)
 *   bestStep  int64 [replicas]       step of each record
 * and optionally host outputs best_energy_units / best_replica (the argmin
 * of phia_best_exact; NULL to skip).  Results are bit-identical to
 * phia_anneal with the same arguments (no energy trace is recorded, and the
 * accept/reject step is not available: PHIA_EINVAL).  The problem's own
 * anneal state is left as it was.  The kernels' scratch (kick factors,
 * exchange words, error word) lives in a fixed device array of 32 MiB per
 * GPU, held until the process ends; an anneal whose scratch exceeds it
 * (about 4 bytes per step plus the exchange of column-split geometries) or
 * whose exchange tags would wrap within the call returns PHIA_ERANGE.  Every
 * call on one GPU shares that array: calls that overlap on one GPU (several
 * host threads, or several streams in flight) race and must not be made.
 * Synchronises the problem's stream; a device error poisons the handle. */
phia_status phia_anneal_noalloc(phia_problem* p, int32_t replicas, int64_t steps,
                                const phia_schedule* schedule, uint64_t seed, float* x, float* v,
                                int64_t* bestE, int8_t* bestS, int64_t* bestStep,
                                int64_t* best_energy_units, int32_t* best_replica);

/* Largest replica count for which an anneal on the I8 path takes the VALU
 * int8 dot-product sweep by default, for padded size Np (0: never).  Below it
 * J.s is a matrix-vector product per replica and the sweep is bound by the
 * stream of J, which 16-row matrix-core tiles would mostly pad; the value is
 * the crossover measured against the matrix-core sweeps on MI355X. */
int32_t phia_valu_crossover(int32_t Np);

/* Allocate replica state and draw x ~ N(0, I) (App. A, A3) for step 0.
 * Enqueued on the problem's stream; returns without waiting.  The sweep's
 * launch geometry is fixed here from (path, Np, replicas): on the I8 path,
 * anneals of few replicas (replicas <= phia_valu_crossover(Np), no
 * accept/reject step) run the VALU int8 dot-product sweep, where J.s is a
 * matrix-vector product per replica; larger ones the matrix-core sweeps.
 * A tuned or cached geometry (phia_autotune) takes precedence. */
phia_status phia_anneal_start(phia_problem* p, int32_t replicas, int64_t steps,
                              const phia_schedule* schedule, uint64_t seed);

/* Enqueue steps [current, k_end) (k_end <= steps).  Returns without waiting;
 * splitting a run into several calls gives bit-identical results. */
phia_status phia_anneal_run(phia_problem* p, int64_t k_end);

/* Wait for the problem's stream and report a device error or barrier timeout. */
phia_status phia_sync(phia_problem* p);

/* Best configuration over all replicas (lowest energy, lowest replica on
 * ties).  energy: host double = sigma * E_units (exact), or, when the input
 * was rounded onto the grid, the FP64 energy of that configuration against
 * the original couplings.  spins: host int8[N] or NULL.  Synchronises. */
phia_status phia_best(phia_problem* p, double* energy, int8_t* spins);

/* Exact best energy in units of 2^-frac_bits, and the replica that found it. */
phia_status phia_best_exact(phia_problem* p, int64_t* energy_units, int32_t* frac_bits,
                            int32_t* replica);

/* FP64 energy (Eq. 2) of the best configuration against the couplings given
 * to phia_create, computed on the device in FP64. */
phia_status phia_best_f64(phia_problem* p, double* energy);

/* Per-replica records: E: host int64[R] (units), S: host int8[R*N] or NULL,
 * step: host int64[R] (first step reaching the record) or NULL. */
phia_status phia_replica_best(phia_problem* p, int64_t* E, int8_t* S, int64_t* step);

/* Continuous state: x, v: host float[R*N] or NULL; k: host int64 or NULL
 * (the next step to run). */
phia_status phia_get_state(phia_problem* p, float* x, float* v, int64_t* k);

/* Accept/reject statistics of a metropolis anneal (App. A, Table 3 state 4),
 * per replica, each a host array of R or NULL: trajectories accepted,
 * trajectories decided (the first one is never decided), and the current beta
 * multiplier.  PHIA_ESTATE if the anneal runs without the step. */
phia_status phia_replica_mh(phia_problem* p, int32_t* accepted, int32_t* decided, float* lam);

/* Overwrite the continuous state of the current anneal (x, v: host
 * float[R*N]) and set the next step to k (0 <= k <= steps).  Records are
 * kept.  The accept/reject state restarts as after the initial draw (start
 * energy unknown, lam = 1, counts 0).  Used to resume from saved state and by
 * invariance tests. */
phia_status phia_set_state(phia_problem* p, const float* x, const float* v, int64_t k);

phia_status phia_get_info(const phia_problem* p, phia_info* out);

/* Flip-incremental quasi-gradient (an execution strategy; not part of the
 * paper's method).  Between consecutive steps only the spins whose sign
 * changed alter I = J s + h of Eq. 6: I(k) = I(k-1) + J (s(k) - s(k-1)), with
 * s(k) - s(k-1) = +-2 on the changed spins and 0 elsewhere.  With it on, the
 * sweep keeps J s in registers and, at every step after the first of a
 * launch, adds the product over the 16-spin column blocks that changed in
 * any replica of a 16-replica block, falling back to the full product when
 * that covers more than 2/3 of it.  Integer arithmetic makes both identical
 * bit for bit, so results do not depend on the setting.  It applies where
 * the sweep has such a variant: the I8 or BF16HILO path, a column-split
 * group of one-row-tile blocks with J streamed from L2, an anneal of its own
 * (not a batch or server launch), and on I8 N <= 4864 (the LDS holds the
 * bookkeeping); phia_info.incremental reports whether the current geometry
 * uses it.  on = 1: wherever it applies.  on = -1 (the default): likewise,
 * except with the accept/reject step, whose rejections return whole replicas
 * to their trajectory start, so that few steps qualify.  on = 0: always the
 * full product.  Takes effect at the next phia_anneal_start or phia_anneal.
 * PHIA_EINVAL if on is not -1, 0 or 1. */
phia_status phia_set_incremental(phia_problem* p, int32_t on);

/* Counters of the flip-incremental update since the last phia_anneal_start,
 * summed over the replica blocks: out[0] steps that took the incremental
 * product, out[1] steps that computed the full product (every launch's first
 * step among them), out[2] 64-wide k blocks of the incremental products (a
 * full product takes Np / 64).  All zero when the geometry has no such
 * variant.  out: host, 3 int64.  Synchronizes the problem's stream.
 * PHIA_ESTATE before any phia_anneal_start. */
phia_status phia_incremental_stats(phia_problem* p, int64_t* out);

/* Test hooks of the column-split exchange (diagnostic; results do not depend
 * on them).  Workgroups that split one replica block's columns swap their
 * spins every step through tagged words; the tag is a sequence number that
 * runs on across launches and restarts (with the words cleared) before it
 * would wrap: 24 bits in the interleaved sweep (sweep_kernel 1), 32 bits in
 * the one-block-per-workgroup sweep.
 *
 * phia_set_exchange_seq sets the sequence number of the next launch of the
 * current anneal, so that a test can start next to the wrap.  seq must not
 * exceed 2^24 - 2 (interleaved) or 2^32 - 2.  PHIA_ESTATE before
 * phia_anneal_start or when the geometry has no exchange (group 1);
 * PHIA_EINVAL when seq is out of range.
 *
 * A kernel polls one exchange word at most 2^21 times before it gives up;
 * every 256th poll it also gives up if the device error word is raised.  A
 * wait that gives up raises the word, every workgroup leaves the sweep at
 * its next check, and phia_sync then returns PHIA_EDEVICE and poisons the
 * handle.  phia_raise_error_word(p, 1) raises the word before every
 * following launch, as if a workgroup had given up, so that a test takes
 * that path from the host without a real fault (a launch whose waits are
 * all short still completes its steps; the handle is poisoned either way);
 * 0 turns it off. */
phia_status phia_set_exchange_seq(phia_problem* p, uint32_t seq);
phia_status phia_raise_error_word(phia_problem* p, int32_t on);

/* Autotuner of the launch geometry of the matrix-core sweep (replicas per
 * workgroup block, workgroups sharing one block's columns, coupling slice in
 * LDS or streamed): every feasible geometry for `replicas` replicas runs
 * probe_steps steps (in [10, 100000]) on this problem, timed with HIP events
 * on its stream, and the fastest is kept for later anneals with the same
 * replica count.  Ends any anneal in progress (state is released).  When
 * the environment variable PHIA_TUNE_CACHE names a file, the winner is
 * appended to it and problems of the same path, padded size and replica
 * count created later use it without timing.  best_us: host double, time per
 * step of the winner in microseconds, or NULL.  The FP32 path has one
 * geometry and returns at once (best_us = 0). */
phia_status phia_autotune(phia_problem* p, int32_t replicas, int64_t probe_steps, double* best_us);

/* Record the energy of every step of the next anneal (test and diagnostic
 * hook).  Call before phia_anneal_start; costs R*steps*8 bytes of device
 * memory.  phia_get_trace copies the energies, host int64[R*steps] in units
 * (row r holds E_0 .. E_{steps-1} of replica r; steps not yet run read 0). */
phia_status phia_set_trace(phia_problem* p, int32_t enable);
phia_status phia_get_trace(phia_problem* p, int64_t* E);

/* Self-check of the device's elementary functions (diagnostic hook).
 * kind 0: e^x for x <= 0; 1: ln u, u in (0,1); 2: cos and sin of 2 pi u
 * (out holds 2n floats, cos first); 3: sech^2; 4: Gaussian draws with
 * in64 = {seed, then n quadruples (tag, replica, round, index)}; 5: the
 * POLY2 quadratic.  in: host float[n] (kinds 0-3, 5), out: host float[n]
 * (2n for kind 2). */
phia_status phia_eval_fmath(int32_t kind, const float* in, const uint64_t* in64, float* out, int64_t n,
                            int32_t device);

/* Anneal `count` problems of uneven size together: one captured HIP graph
 * (an init kernel and one sweep kernel per bucket of similar instances)
 * runs every problem's whole anneal.  Problem i uses replicas[i], steps[i],
 * scheds[i] and seeds[i] (host arrays of count entries) exactly as
 * phia_anneal would, with bit-identical results; afterwards phia_best,
 * phia_replica_best and phia_get_state read each problem as usual.  All
 * problems must be on one device, use the I8 or BF16HILO path, have N <= 512
 * and appear once.  The work runs on problem 0's stream (a private stream if
 * that is the null stream) and the call returns when it has finished.
 * Energy traces are not recorded in batches. */
phia_status phia_batch_run(phia_problem* const* probs, int32_t count, const int32_t* replicas,
                           const int64_t* steps, const phia_schedule* scheds, const uint64_t* seeds);

/* A reusable batch plan: phia_batch_run split into its parts, so that the
 * set-up (replica state of every problem, work tables, the captured and
 * instantiated HIP graph) happens once and the anneal of all problems can be
 * launched many times.  phia_batch_create takes the same arguments as
 * phia_batch_run without the seeds; the plan then holds the problems' replica
 * state: phia_anneal_start, phia_anneal_run, phia_set_state, phia_autotune and
 * phia_server_submit on them return PHIA_ESTATE until phia_batch_destroy
 * (reading results stays allowed and waits for the batch).  Instances whose
 * integer couplings are all FP4 values (0, +-1, +-2, +-3, +-4, +-6), with
 * N <= 512 and no accept/reject step, run in one persistent kernel that
 * takes 32-replica work items from a queue, largest first; the others run in
 * one kernel per bucket of similar instances after it.
 *
 * phia_batch_launch enqueues one whole anneal of every problem with
 * seeds[i] (host array of count seeds) on the plan's stream (problem 0's
 * stream, or a private one when that is the null stream) and returns without
 * waiting; results are bit-identical to phia_anneal of each problem with its
 * seed.  phia_batch_sync waits for the last launch.  phia_batch_destroy waits
 * and releases the plan (not the problems).  Destroying a member problem
 * first makes later launches return PHIA_ESTATE. */
typedef struct phia_batch phia_batch;
phia_status phia_batch_create(phia_problem* const* probs, int32_t count, const int32_t* replicas,
                              const int64_t* steps, const phia_schedule* scheds, phia_batch** out);
phia_status phia_batch_launch(phia_batch* b, const uint64_t* seeds);
phia_status phia_batch_sync(phia_batch* b);
void phia_batch_destroy(phia_batch* b);

/* ---------------------------------------------------------------- serving --
 * A server anneals submitted problems with continuous batching on one GPU.
 * Requests are admitted in arrival order when a slot is free and their
 * estimated device footprint (couplings plus replica state) fits within
 * hbm_budget bytes next to the running ones; a request that can never fit
 * fails.  Each scheduling round advances every running request by
 * chunk_steps steps (instances with N <= 512 together in one batched launch,
 * larger ones each in a column-split launch), then checks every request: it
 * retires when its best energy reaches target_energy_units (units of
 * 2^-frac_bits of its problem) or after max_steps steps.  Requests stop only
 * at chunk boundaries, so a request's result is the same alone and in any
 * mix.  A submitted problem belongs to the server until its request has
 * finished: the caller must not use or destroy it before that.  All server
 * functions are thread-safe. */
typedef struct phia_server phia_server;

enum {
    PHIA_REQ_QUEUED = 0,
    PHIA_REQ_RUNNING = 1,
    PHIA_REQ_DONE = 2,
    PHIA_REQ_CANCELLED = 3,
    PHIA_REQ_FAILED = -1
};

typedef struct {
    int32_t state;         /* PHIA_REQ_*                                                */
    int32_t success;       /* 1: the best energy reached the target                     */
    int32_t frac_bits;     /* f of the problem                                          */
    int32_t replica;       /* replica holding the best state (-1 before any step)       */
    int64_t energy_units;  /* best energy in units of 2^-f (INT64_MAX before any step)  */
    int64_t steps_used;    /* steps run                                                 */
    double t_arrive;       /* seconds since server creation: submission                 */
    double t_admit;        /* admission (-1 while queued)                               */
    double t_done;         /* retirement (-1 while unfinished)                          */
} phia_result;

/* hbm_budget > 0 bytes, max_slots in [1, 65536], chunk_steps >= 1. */
phia_status phia_server_create(size_t hbm_budget, int32_t max_slots, int32_t chunk_steps, int32_t device,
                               phia_server** out);
/* Queue a request; *ticket identifies it.  The schedule (and an explicit
 * beta table, which is copied) has max_steps entries. */
phia_status phia_server_submit(phia_server* s, phia_problem* p, int32_t replicas, int64_t max_steps,
                               int64_t target_energy_units, const phia_schedule* schedule, uint64_t seed,
                               uint64_t* ticket);
/* Device bytes a request of `replicas` x `max_steps` on p is charged against
 * the server's budget (couplings, replica state, schedule, exchange). */
phia_status phia_server_footprint(const phia_problem* p, int32_t replicas, int64_t max_steps, size_t* bytes);
/* Current state and result of a request (never blocks). */
phia_status phia_server_poll(phia_server* s, uint64_t ticket, phia_result* out);
/* Block until the request has finished (timeout_s < 0: no limit); returns
 * PHIA_ESTATE with the current state on timeout. */
phia_status phia_server_wait(phia_server* s, uint64_t ticket, double timeout_s, phia_result* out);
/* Best state of a finished request: host int8[N] of its problem. */
phia_status phia_server_spins(phia_server* s, uint64_t ticket, int8_t* spins);
/* Cancel a queued request, or stop a running one at the end of the round. */
phia_status phia_server_cancel(phia_server* s, uint64_t ticket);
/* Cancel what is queued, stop what runs, release the server (not the problems). */
void phia_server_destroy(phia_server* s);

/* Release all device memory of p.  NULL is accepted. */
void phia_destroy(phia_problem* p);

/* Message of the last error on this thread ("" if none). */
const char* phia_last_error(void);

/* Library version string. */
const char* phia_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PHIA_H */

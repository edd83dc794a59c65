/*
 * mars.h -- C interface of the MARS solver for AMD Instinct MI355X (gfx950).
 *
 * MARS (Mean-field Annealing from a Random State; Yavorsky, Markovich,
 * Polyakov, Rubtsov, arXiv:1907.05124) runs many independent mean-field
 * descents of an Ising problem, each from a random magnetisation and a random
 * starting temperature, rounds each to spins and keeps the best (paper,
 * section "Mean-field Annealing from Random State", Algorithm 1).
 *
 * Conventions used by every entry point:
 *
 *   Energy (eq. (2), ordered-pair double sum, minimisation sign):
 *       E(s) = - sum_i sum_{j != i} J_ij s_i s_j - sum_i h_i s_i,   s_i = +-1.
 *   A max-cut instance with edge weights w is passed as J = -w; its cut is
 *   (sum_{i != j} w_ij - E)/4 (eq. (3)) when h = 0.
 *   Local field and update of one magnetisation (Algorithm 1 with J = -J_paper):
 *       Phi_i = sum_j J_ij m_j + h_i / 2,   m_i <- (1-g) m_i + g tanh(Phi_i / T),
 *   with damping g = 1 for the paper's method.
 *   Spins are updated phase by phase inside a sweep (dense: contiguous row
 *   blocks [floor(bN/B), floor((b+1)N/B)); lattice: checkerboard; sparse:
 *   greedy colouring in index order); MARS_JACOBI uses one phase holding all
 *   spins (every spin sees the previous sweep's values).
 *   Rounding: s_i = +1 if m_i >= 0, else -1.
 *   Energies are exact: the sum of the terms is rounded once to double.
 *   Best run: lowest energy, ties to the lowest run index.
 *   Random draws: SplitMix64 output function of (seed + (c+1)*0x9E3779B97F4A7C15)
 *   with counter c = (stream<<62)|(run<<32)|spin; stream 0 gives
 *   m0 = (2k+1-2^24)*2^-24, stream 1 gives T0 = T_lo + (T_hi-T_lo)*(k*2^-24),
 *   k = the output's top 24 bits.
 *
 * Layouts: magnetisations are spin-major N x R with runs contiguous
 * (element (i, r) at i*R + r); per-run spin vectors are run-major R x N
 * (element (r, i) at r*N + i).
 *
 * Errors: every entry point returns a mars_status; on error it writes no
 * output and mars_last_error() holds a message for the calling thread.  The
 * library never aborts or throws across this interface.
 * Threads: calls on one instance are serialised by the library; distinct
 * instances may be used concurrently.
 */
#ifndef MARS_H
#define MARS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mars_instance mars_instance;

typedef enum {
    MARS_OK = 0,
    MARS_E_ARG = 1,          /* null pointer, bad size or bad schedule field */
    MARS_E_ASYMMETRIC = 2,   /* J_ij != J_ji (bitwise) */
    MARS_E_DIAGONAL = 3,     /* nonzero J_ii, or a self loop in CSR */
    MARS_E_NONFINITE = 4,    /* NaN or infinity in J or h */
    MARS_E_RANGE = 5,        /* exact energy would need more than 126 bits */
    MARS_E_OOM = 6,          /* device allocation failed (also every instance and workspace
                                allocation while MARS_TEST_FAIL_ALLOC=1 is set in the
                                environment: a test hook for the error paths) */
    MARS_E_DEVICE = 7,       /* HIP runtime error or no usable gfx950 device */
    MARS_E_UNSUPPORTED = 8   /* valid request outside what this build implements */
} mars_status;

enum { MARS_GEOMETRIC = 0, MARS_LINEAR = 1 };
enum { MARS_PHASED = 0, MARS_JACOBI = 1, MARS_SEQUENTIAL = 2 };
enum { MARS_FP32 = 0, MARS_FP64 = 1, MARS_BF16 = 2, MARS_FP16 = 3 };

/* Annealing schedule (Algorithm 1; parameters of section "Parameter settings").
 *   kind        MARS_LINEAR: T <- T0, then T <- T - c_step before each level,
 *               stopping at T <= 0 (the paper's scheduler).
 *               MARS_GEOMETRIC: `steps` levels T_k = T0 exp((k/(steps-1)) ln(T_end/T0)).
 *   T_lo, T_hi  range of the random starting temperature T0 (T_lo <= T_hi).
 *   T_end       last geometric level (> 0).
 *   c_step      linear decrement (> 0; the paper uses 1).
 *   steps       number of geometric levels (>= 0).
 *   max_sweeps  sweeps allowed per level (>= 1); a level also ends when the
 *               largest change of a sweep is below d_min (the paper: 1e-4).
 *               max_sweeps = 1 gives exactly one sweep per level.
 *   update      MARS_PHASED, MARS_JACOBI, or MARS_SEQUENTIAL (dense MARS_FP32
 *               only: every spin its own phase, in index order -- the
 *               per-spin assignment of the paper's GPU description; the same
 *               dynamics as MARS_PHASED with phases = N, computed as blocks of
 *               64 spins whose fields come from one product and are corrected
 *               spin by spin inside the block).
 *   phases      dense row blocks per sweep (>= 1; ignored for lattices/CSR).
 *   damping     g in (0, 1]; 1 is the paper's update.
 *   precision   MARS_FP32 (dense, lattice, CSR), MARS_FP64 (lattice, CSR),
 *               MARS_FP16 (fp16 magnetisation storage, fp32 arithmetic;
 *               lattice, CSR), MARS_BF16 (bf16 couplings and magnetisations
 *               with fp32 accumulation; dense).
 *   first_level, level_count
 *               relax only levels [first_level, first_level+level_count) of
 *               each run's schedule (level_count < 0: to the end).  With m0
 *               and T0 supplied this resumes a solve from a saved state. */
typedef struct {
    int32_t kind;
    double T_lo, T_hi, T_end, c_step;
    int32_t steps;
    int32_t max_sweeps;
    double d_min;
    int32_t update;
    int32_t phases;
    double damping;
    int32_t precision;
    int32_t first_level;
    int32_t level_count;
} mars_schedule;

/* Summary of a solve (section "Ground state of Sherrington-Kirkpatrick
 * spin-glass": best energy, mean energy, hit count, success probability). */
typedef struct {
    double best_energy;      /* lowest exact energy over the runs */
    double best_cut;         /* (sum_{i!=j} -J_ij - best_energy)/4 (max-cut value if J = -w, h = 0) */
    double mean_energy;      /* mean of the runs' exact energies */
    double best_T0;          /* starting temperature of the best run */
    int32_t best_run;        /* index of the best run (lowest index on ties) */
    int32_t runs;
    int64_t hit_count;       /* runs whose energy equals best_energy */
    int64_t sweeps_executed; /* sweeps summed over runs */
    int64_t spin_updates;    /* N x sweeps_executed: magnetisation recomputations */
    int64_t cap_hits;        /* levels ended by max_sweeps (> 1) with d >= d_min */
    int64_t levels_executed; /* levels summed over runs */
    double seconds;          /* device time of the solve: from its first enqueued
                                kernel to the best-of-runs step (the device's
                                constant-rate clock), queueing behind earlier
                                work on the stream excluded */
} mars_result;

/* Create a dense instance (paper eq. (2); the SK model of the section "Ising
 * Spin Glass Model").  J: host pointer to N*N float32, row-major, symmetric
 * bitwise, zero diagonal.  h: host pointer to N float32, or NULL for h = 0.
 * The inputs are copied; the caller keeps ownership.  Errors: MARS_E_ARG
 * (N < 1, null J or out), MARS_E_NONFINITE, MARS_E_ASYMMETRIC,
 * MARS_E_DIAGONAL, MARS_E_RANGE, MARS_E_OOM, MARS_E_DEVICE. */
mars_status mars_create(const float *J, const float *h, int32_t N, mars_instance **out);

/* Create a sparse instance with integer couplings (the max-cut graphs of the
 * section "MAX-CUT", J = -w).  Host pointers: rowptr[N+1], col[nnz],
 * val[nnz] with nnz = rowptr[N]; both directions of every edge stored with
 * the same value, columns strictly increasing within a row, no self loops,
 * val != 0.  h as in mars_create.  Copied; caller keeps ownership.
 * Errors: MARS_E_ARG (bad pointers, sizes or ordering), MARS_E_ASYMMETRIC,
 * MARS_E_DIAGONAL, MARS_E_NONFINITE, MARS_E_RANGE, MARS_E_OOM, MARS_E_DEVICE. */
mars_status mars_create_csr(int32_t N, const int32_t *rowptr, const int32_t *col, const int8_t *val,
                            const float *h, mars_instance **out);

/* Create a periodic hypercubic lattice instance (Edwards-Anderson model,
 * section "Ising Spin Glass Model").  dim = 2 or 3; L[dim] even sizes >= 4;
 * site i = x0 + L0*(x1 + L1*x2); bond[a*N + i] (int8, +1 or -1) couples site i
 * with its neighbour one step along axis a (periodic).  h as in mars_create.
 * Host pointers, copied.  Errors: MARS_E_ARG, MARS_E_NONFINITE, MARS_E_RANGE,
 * MARS_E_OOM, MARS_E_DEVICE. */
mars_status mars_create_lattice(int32_t dim, const int32_t *L, const int8_t *bond, const float *h,
                                mars_instance **out);

/* Release an instance and its device memory.  NULL is ignored. */
void mars_destroy(mars_instance *inst);

/* Number of spins and of update phases per sweep for a schedule (host query). */
mars_status mars_describe(const mars_instance *inst, const mars_schedule *sched, int32_t *N, int32_t *phases);

/* Solve with host outputs (Algorithm 1 over `runs` independent runs, then
 * best-of-runs selection).  best_spins: host int8[N] (may be NULL);
 * energies: host double[runs] (may be NULL); res: host (may be NULL).
 * Blocks until the results are on the host.  Lattice and sparse instances
 * keep each run's state in LDS when it fits (about 159 KB per run: the
 * slots times 8, 4 or 2 bytes in fp64, fp32, fp16); a sparse instance
 * beyond that keeps its state in device memory (a workspace of
 * (slots + 1) x runs values; about a quarter of the LDS path's throughput
 * at equal size), and so does a lattice, over sparse encodings of its
 * couplings built on its first such solve (up to 2^24 sites).  Errors:
 * MARS_E_ARG (runs < 1, bad schedule), MARS_E_UNSUPPORTED (precision not
 * available for this instance type, or a lattice beyond LDS with 2^24 sites
 * or more), MARS_E_OOM, MARS_E_DEVICE. */
mars_status mars_solve(mars_instance *inst, int32_t runs, const mars_schedule *sched, uint64_t seed,
                       int8_t *best_spins, double *energies, mars_result *res);

/* Solve with device buffers on a caller stream.  All array pointers are
 * DEVICE pointers and may be NULL:
 *   m0       [N x runs] initial magnetisations (double for MARS_FP64, float
 *            otherwise); NULL draws them from the generator.
 *   T0       [runs] double starting temperatures; NULL draws them.
 *   T0_used  [runs] double: receives the starting temperatures of the solve.
 *   m_final  [N x runs] final magnetisations (same element type as m0).
 *   spins    [runs x N] int8 rounded spins of every run.
 *   energies [runs] double exact energies.
 *   best_spins [N] int8 spins of the best run.
 *   sweeps_per_level [runs x level_cap] int32: entry (r, k) is the number of
 *            sweeps run r ran at the k-th level it visited (Algorithm 1's
 *            repeat ... until loop: the sweep at which the largest change d
 *            fell below d_min, or max_sweeps; 1 on every level when
 *            max_sweeps = 1), 0 past the run's last level; levels beyond
 *            level_cap are not recorded.  These are the decisions a CPU
 *            reference replays to follow the same trajectory where its own
 *            d-versus-d_min decisions (taken in another precision) differ.
 *   level_cap >= 1 when sweeps_per_level is given (ignored otherwise).
 * stream is a hipStream_t (NULL: the default stream).  When res (HOST) is
 * non-NULL the call waits for the stream and fills it; otherwise it returns
 * after enqueueing.  Device outputs are valid once the stream reaches the end
 * of the enqueued work.  Errors as mars_solve, and MARS_E_ARG for
 * sweeps_per_level with level_cap < 1. */
mars_status mars_solve_ex(mars_instance *inst, int32_t runs, const mars_schedule *sched, uint64_t seed,
                          const void *m0, const double *T0, double *T0_used, void *m_final, int8_t *spins,
                          double *energies, int8_t *best_spins, int32_t *sweeps_per_level, int32_t level_cap,
                          mars_result *res, void *stream);

/* Asynchronous solve for serving many instances concurrently: as
 * mars_solve_ex, but the summary is copied into res_pinned (HOST memory
 * allocated pinned, e.g. hipHostMalloc) by an asynchronous copy on `stream`;
 * the call returns after enqueueing and every output, including *res_pinned,
 * is valid once the stream has passed the enqueued work.  res_pinned may be
 * NULL.  Solves and energy calls on one instance may use different streams:
 * each waits on the stream for the instance's previous work (its workspace
 * is shared).  Errors as mars_solve. */
mars_status mars_solve_async(mars_instance *inst, int32_t runs, const mars_schedule *sched, uint64_t seed,
                             const void *m0, const double *T0, void *m_final, int8_t *spins, double *energies,
                             int8_t *best_spins, mars_result *res_pinned, void *stream);

/* Several lattice or sparse solves enqueued together on one stream, for a
 * server that admits many small requests at once (one launch per request
 * leaves the GPU mostly idle when each has few runs).  Member i is the solve
 * of mars_solve_async(insts[i], runs[i], &scheds[i], seeds[i], NULL, NULL,
 * NULL, NULL, energies[i], best_spins[i], &res_pinned[i], stream), with the
 * same outputs bit for bit; sparse members whose anneal runs on the same
 * instantiation of the LDS-resident solver (storage precision, runs per lane
 * group, lanes per slot, update, field, weights, damping, stopping rule)
 * share one launch of it, each on its own workgroups.  Lattice members and
 * sparse members beyond LDS are enqueued as they would be alone.  Runs may
 * differ between members; each run's trajectory is independent of the
 * others (Algorithm 1 per run).
 *   count: 1 to 64; the instances are distinct, on one device, not dense.
 *   best_spins, energies: arrays of count DEVICE pointers (int8 [N_i],
 *            double [runs_i]); the arrays or any entry may be NULL.
 *   res_pinned: HOST pinned mars_result [count], or NULL.
 * Returns after enqueueing; outputs are valid once the stream has passed the
 * enqueued work.  Errors: MARS_E_ARG (count, NULL arrays, an instance twice
 * or on another device, runs, schedules), MARS_E_UNSUPPORTED (a dense
 * instance, or as mars_solve), MARS_E_OOM, MARS_E_DEVICE; validation
 * precedes any enqueued work. */
mars_status mars_solve_group_async(int32_t count, mars_instance *const *insts, const int32_t *runs,
                                   const mars_schedule *scheds, const uint64_t *seeds, int8_t *const *best_spins,
                                   double *const *energies, mars_result *res_pinned, void *stream);

/* Exact energies (eq. (2)) of R spin vectors.  spins: DEVICE int8 [R x N]
 * (values +-1); energies: DEVICE double [R].  stream as in mars_solve_ex;
 * the call returns after enqueueing.  Errors: MARS_E_ARG, MARS_E_DEVICE. */
mars_status mars_energy(mars_instance *inst, const int8_t *spins, int32_t R, double *energies, void *stream);

/* mars_energy for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same energies, bit for bit, with no hipMalloc, hipFree or other allocation
 * on any call.  Dense instances work in a fixed scratch array of 32 MiB per
 * device, part of the library's image (each device it runs on holds it until
 * the process ends): R spin vectors of N spins need
 * round_up(ceil(R/128)*128 * Ke, 256) + (Me/128) * R * 16 bytes, Ke = Me =
 * round_up(N, 128) (N = 2000: up to about 14000 vectors); larger requests
 * return MARS_E_UNSUPPORTED and write nothing.  Lattice and sparse
 * instances need no scratch.  Every call on one device shares its array:
 * calls whose stream work overlaps on one device race (calls on one
 * instance are ordered by the library; on distinct instances order them on
 * one stream).  Arguments, layouts, ownership and the other errors as
 * mars_energy. */
mars_status mars_energy_noalloc(mars_instance *inst, const int8_t *spins, int32_t R, double *energies, void *stream);

/* Extreme eigenvalues of the couplings J (h is not involved), estimated by
 * `steps` Lanczos steps (capped at N) from a start vector drawn with `seed`,
 * in fp64 on the device.  They set the temperature scale of an anneal: the
 * update of Algorithm 1 linearised at m = 0 is m <- J m / T (h = 0), so a
 * random start decays to 0 at every T above lambda_max, and the synchronous
 * update turns unstable below |lambda_min| (section "Mean-field Annealing
 * from Random State"; the paper picks its temperature range by preliminary
 * runs, section "Parameter settings").  The estimates lie inside the true
 * range and approach it as steps grow (100 steps: within 1e-3 relative on
 * the SK, lattice and random-graph workloads).  lambda_min, lambda_max: HOST
 * doubles.  stream as in mars_solve_ex; the call waits for its own work.
 * Errors: MARS_E_ARG, MARS_E_OOM, MARS_E_DEVICE. */
mars_status mars_spectrum(mars_instance *inst, int32_t steps, uint64_t seed, double *lambda_min, double *lambda_max,
                          void *stream);

/* Temperature range from the spectrum: runs mars_spectrum(steps, seed) and
 * sets sched->T_lo = 0.5 L, T_hi = 1.5 L and T_end = 0.005 L, with
 * L = lambda_max (the spectral radius if J has no positive eigenvalue); the
 * other fields are left as they are.  This stands in for the preliminary
 * runs with which the paper chooses its temperature bounds (section
 * "Parameter settings"; the paper stresses that the bounds are what matters).
 * The factors come from a sweep over SK, random-graph and 2D/3D lattice
 * instances, where this range reached best energies 1-1.5 % lower than a
 * range scaled by the field deviation sigma_Phi = sqrt(mean_i sum_j J_ij^2)
 * on lattices and degree-4 graphs, and equal ones on SK and dense graphs.
 * Errors: those of mars_spectrum; MARS_E_ARG if sched is NULL or J = 0. */
mars_status mars_auto_temperatures(mars_instance *inst, int32_t steps, uint64_t seed, mars_schedule *sched,
                                   void *stream);

/* Batched BF16 solver for a served stream of dense instances (the BF16 form
 * of the dense field product, Algorithm 1's update, eq. (2) energies): the
 * members of a batch advance together on one stream and every update phase
 * of every member is ONE launch over all their tiles, so instances of uneven
 * N share the GPU instead of each underfilling it.  Members join and leave
 * between sweeps (continuous batching); each member is at its own level.
 * Results equal mars_solve_async's for the same arguments bit for bit.
 *
 * mars_batch_create: stream is a hipStream_t (NULL: the default stream) on
 *   the current device; the batch owns 16 level counters in device memory
 *   and its step graph.  Errors: MARS_E_ARG (out NULL), MARS_E_OOM,
 *   MARS_E_DEVICE.
 * mars_batch_add: enqueues the member's set-up (its workspace, starting
 *   temperatures, level table, initial state) on the batch stream; it joins
 *   at the next step.  inst: a dense instance on the batch's device, owned by
 *   the batch (no other call may use it) until the member finishes.  sched:
 *   precision MARS_BF16, max_sweeps 1 (one sweep per level).  tag: returned
 *   by mars_batch_step when the member finishes.  best_spins: DEVICE int8 [N]
 *   or NULL; res_pinned: HOST mars_result in pinned memory, or NULL; both
 *   are written by the stream when the member finishes.  Errors: MARS_E_ARG,
 *   MARS_E_UNSUPPORTED (not dense, not MARS_BF16, max_sweeps != 1, another
 *   device, or the batch already holds 16 members), MARS_E_OOM, MARS_E_DEVICE.
 * mars_batch_step: enqueues up to `sweeps` sweeps of every member; a member
 *   that reaches its last level is rounded and scored, its outputs are
 *   copied, and it leaves.  On a non-NULL stream the step's per-phase
 *   launches are captured once as a graph and replayed by later steps while
 *   no member joins or leaves and `sweeps` is unchanged (MARS_BATCH_GRAPH=0
 *   in the environment at mars_batch_create launches sweep by sweep
 *   instead).  MARS_BATCH_PERSIST=1 there runs each step as one persistent
 *   cooperative launch over every member's tiles instead (grid barriers
 *   between update phases, the level counters advanced on the device),
 *   while no member has more than four update phases.  A member that
 *   finishes inside a step leaves at the step's end.  Results are the same
 *   bit for bit on every path.  finished_tags: HOST int64 [cap]
 *   receiving the tags of the members that left during this call
 *   (*n_finished of them, never more than cap: a finished member beyond that
 *   stays, without sweeping, and leaves at a later call; sweeps = 0 only
 *   retires); *n_active: members still in the batch.  Outputs of a finished
 *   member are valid once the stream has passed the work enqueued by the
 *   call.  Errors: MARS_E_ARG, MARS_E_DEVICE.
 * mars_batch_destroy: waits for the batch stream and releases the batch and
 *   every member still in it (their outputs are not written).  NULL is a
 *   no-op.  An instance is destroyed only after its member has finished or
 *   its batch has been destroyed. */
typedef struct mars_batch mars_batch;
mars_status mars_batch_create(void *stream, mars_batch **out);
mars_status mars_batch_add(mars_batch *batch, mars_instance *inst, int32_t runs, const mars_schedule *sched,
                           uint64_t seed, int64_t tag, int8_t *best_spins, mars_result *res_pinned);
mars_status mars_batch_step(mars_batch *batch, int32_t sweeps, int64_t *finished_tags, int32_t cap,
                            int32_t *n_finished, int32_t *n_active);
void mars_batch_destroy(mars_batch *batch);

/* Static description of a status code, and the last error message of the
 * calling thread (empty if none).  Both strings stay owned by the library. */
const char *mars_status_str(mars_status s);
const char *mars_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MARS_H */

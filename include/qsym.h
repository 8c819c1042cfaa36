/*
 * qsym.h -- C ABI of the MI355X (gfx950) library for the democratic-
 * heliocentric (DH) hybrid symplectic step of Moore & Quillen, "QYMSYM: A
 * GPU-Accelerated Hybrid Symplectic Integrator That Permits Close
 * Encounters" (arXiv:1007.3458).
 *
 * One step (Sec. 2, second-order composition; Sec. 2.3, steps 1-10):
 *   E_Dft(tau/2) E_Int(tau/2) E_Kep(tau) E_Int(tau/2) E_Dft(tau/2)
 * with the close-encounter machinery between the Kepler advance and the
 * second kick: crude sweep (fused into the first kick), fine sweep, division
 * into non-intersecting encounter sets, transition-weighted corrections and
 * 4th-order Hermite substeps for the members of each set (Secs. 2.1, 2.2,
 * 2.4).  Everything runs on the device; the host is crossed only by the
 * calls below.
 *
 * Conventions for every entry point:
 *  - all sizes are int64_t, all reals double (learned-guess weights float);
 *  - positions q are heliocentric, velocities v barycentric (barycentric
 *    momentum / mass, so massless bodies are allowed), both laid out SoA as
 *    [3][ntot]: q[0*ntot + i] = x_i, q[1*ntot + i] = y_i, q[2*ntot + i] = z_i;
 *  - the central mass of each system is a parameter, never a body;
 *  - `where` is QSYM_HOST (pointer to host memory, copied synchronously) or
 *    QSYM_DEVICE (pointer to device memory, copied on the context stream);
 *  - the caller owns every pointer it passes; the library keeps none of
 *    them except the workspace bound at creation, which must stay allocated
 *    and untouched until qsym_destroy;
 *  - return 0 on success or a negative QSYM_E* code; no exception crosses
 *    the ABI; qsym_last_error() gives a message for the last failure;
 *  - one context per stream; a context is not thread-safe.
 * Device work is asynchronous on the context's stream; errors detected on
 * the device (overflow, non-finite state, solver caps) are latched in a
 * status word and reported by the next synchronising call (qsym_sync,
 * qsym_get_state, qsym_energy, qsym_encounters, qsym_stats).
 */
#ifndef QSYM_H
#define QSYM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QSYM_OK 0
#define QSYM_EINVAL -1     /* bad argument                                     */
#define QSYM_ENOMEM -2     /* workspace too small                              */
#define QSYM_EHIP -3       /* HIP runtime error                                */
#define QSYM_ENONFINITE -4 /* NaN/Inf appeared in the state                    */
#define QSYM_EKEPLER -5    /* Kepler solver reached its iteration cap          */
#define QSYM_EOVERFLOW -6  /* a system's encounter pairs exceeded its segment
                              (4 per body + 64); the state is left as it was at
                              the start of that step, and later steps do nothing
                              until a new state is set                        */
#define QSYM_ETRUNC -7     /* output buffer shorter than the true count         */
#define QSYM_EHERMITE -8   /* Hermite reached its substep cap / set too large   */

#define QSYM_HOST 0
#define QSYM_DEVICE 1

/* Parameters (Sec. 2.5, list of parameters). */
typedef struct qsym_params {
    double G;            /* gravitational constant                              */
    double aE;           /* Hill factor of encounter identification (Sec. 2.4)  */
    double aH;           /* Hill factor of r_crit (Sec. 2.2, eq. for r_crit)    */
    double epsH;         /* Hermite smoothing length (in-set pairs only)         */
    double eta;          /* Hermite accuracy parameter of the step criterion     */
    double eta_s;        /* Hermite accuracy parameter of the first step         */
    double crude_safety; /* multiplicative slack of the crude sweep, >= 1        */
    int32_t hill_mode;   /* 0: a_E x mutual Hill radius; 1: a_E x sum of radii   */
    int32_t kepler_mode; /* 0: Laguerre from x = r0 (Appendix A); 1: Newton from
                            sqrt(mu) dt / r0; 2: Newton from the learned guess   */
    int32_t precision;   /* 0: FP64 pair terms; 1: m r^-3 in FP32 on FP64
                            separations, accumulated in FP64 (Sec. 2 remarks
                            on single-precision forces)                        */
    int32_t max_substeps;/* Hermite substep cap per set per step (>= 1)           */
    int64_t pair_capacity; /* crude-candidate list length; 0 selects 8*ntot + 1024.
                              A sweep that finds more candidates loses none:
                              the fine test then runs over all pairs (counted
                              in qsym_stats_t.fallbacks)                      */
    double planet_mass;  /* > 0: bodies at least this massive are planets; a
                            step whose encounter sets put two planets in one
                            set integrates that whole system with the Hermite
                            (Sec. 2.3, after the steps): one set of all its
                            bodies with r_crit infinite (K = 0, W = 1), so the
                            corrections take back both half kicks.  0: off. */
    int32_t sweep;       /* crude sweep of Sec. 2.4: 0 fused into the first kick's
                            pair loop (all pairs); 1 on a hashed uniform grid
                            (expected O(N) tests) ahead of a plain first kick.
                            Both decide every pair by the same exact test, so
                            the candidate set is the same.  1 adds a hash
                            table of 2^k >= 2 ntot buckets x 17 ints to the
                            workspace.                                        */
    int32_t pad2;        /* 0 */
} qsym_params;

/* Counters of the last step and totals since creation/reset. */
typedef struct qsym_stats_t {
    int64_t steps;            /* steps taken since creation                    */
    int64_t n_candidates;     /* last step: crude-sweep pairs (true count)     */
    int64_t n_encounters;     /* last step: fine-sweep pairs                   */
    int64_t n_sets;           /* last step: encounter sets                     */
    int64_t max_set;          /* last step: members of the largest set         */
    int64_t substeps;         /* last step: Hermite substeps summed over sets  */
    int64_t total_encounters; /* all steps                                     */
    int64_t total_substeps;   /* all steps                                     */
    int64_t kepler_iters;     /* all steps: Kepler iterations summed           */
    int64_t kepler_max;       /* all steps: largest iteration count            */
    int64_t kepler_hist[32];  /* all steps: solves by iteration count          */
    int64_t status;           /* latched device status bits                    */
    double phase_us[12];      /* per-kernel time when profiling is enabled     */
    int64_t phase_calls[12];  /* launches timed per kernel                     */
    int64_t whole_system;     /* all steps: systems integrated whole (planet_mass) */
    int64_t fallbacks;        /* all steps: candidate lists that overflowed, the
                                 fine test then taken over all pairs          */
    int64_t overflows;        /* all steps: steps left undone because a system's
                                 encounter pairs exceeded its segment (the state
                                 stays at the start of the first such step)   */
    int64_t global_sets;      /* all steps: systems with more than 4096 encounter
                                 pairs in a step, partitioned in global memory */
    int64_t kepler_restarts;  /* all steps: Kepler solves whose first start
                                 reached the iteration cap (then restarted from
                                 the first-order guess)                       */
    /* Load balance while profiling, per phase as phase_us: the kick launches
     * and the set-per-workgroup Hermite launch (k_hermite; not the grid
     * Hermite) record each workgroup's compute unit and start and end time.
     * A compute unit's busy time in a launch is the union of its workgroups'
     * intervals; busy_max_us sums the largest over units, busy_mean_us the
     * mean over all the device's units (idle ones count as zero), over
     * busy_calls launches.  busy_max_us / busy_mean_us is the max/mean busy
     * ratio (1 for a perfectly balanced launch).                              */
    double busy_max_us[12];
    double busy_mean_us[12];
    int64_t busy_calls[12];
    int64_t busy_units;       /* most compute units seen in one launch         */
} qsym_stats_t;

typedef struct qsym_ctx qsym_ctx;

/* Device workspace needed by a context of nsys systems whose bodies are
 * offsets[s] .. offsets[s+1]-1 (offsets has nsys+1 entries, offsets[0] = 0,
 * non-decreasing; a system may be empty).  Writes the size in bytes. */
int qsym_workspace_bytes(const qsym_params *p, int32_t nsys, const int64_t *offsets,
                         int64_t *bytes);

/* Create a context over a caller-allocated device workspace of ws_bytes
 * (>= qsym_workspace_bytes, 256-byte aligned) used on `stream` (a
 * hipStream_t; NULL for the default stream).  m0 (host, nsys entries) are
 * the central masses.  The state is zero until qsym_set_state. */
int qsym_create(const qsym_params *p, int32_t nsys, const int64_t *offsets, const double *m0,
                void *workspace, int64_t ws_bytes, void *stream, qsym_ctx **out);
void qsym_destroy(qsym_ctx *ctx);

/* Load masses m[ntot], Hill factors h[ntot] = cbrt(m / (3 m0)) (computed by
 * the caller once so every implementation uses the same bits), positions
 * and velocities (SoA [3][ntot]).  Clears the latched device status: a
 * non-finite state, an overflow or a solver cap reported for the previous
 * state is not reported again. */
int qsym_set_state(qsym_ctx *ctx, const double *m, const double *h, const double *q,
                   const double *v, int32_t where);
int qsym_get_state(qsym_ctx *ctx, double *q, double *v, int32_t where);

/* nsteps hybrid steps of size tau (Sec. 2.3).  Asynchronous: the first call
 * for a given tau captures the step into HIP graphs that are replayed: the
 * step's body with the drift that ends it and begins the next (one launch;
 * the same additions in the same order as two), and the body with the last
 * drift, so a call is one drift launch and nsteps graph launches.  The
 * result does not depend on how steps are split over calls.  A negative
 * tau integrates backwards (used with a_E = 0). */
int qsym_step(qsym_ctx *ctx, double tau, int64_t nsteps);
/* nsteps encounter-free steps with the Keplerian and interaction operators
 * swapped (Sec. 2, after the second-order composition: without the
 * encounter search they may trade places):
 *   E_Dft(tau/2) E_Kep(tau/2) E_Int(tau) E_Kep(tau/2) E_Dft(tau/2),
 * one all-pairs evaluation per step instead of two.  No sweeps, sets or
 * Hermite: close encounters are not treated, so use it only where none
 * occur.  Same queuing and error behaviour as qsym_step; the encounter
 * statistics of qsym_stats read 0 after it. */
int qsym_step_swapped(qsym_ctx *ctx, double tau, int64_t nsteps);

/* Wait for the context's work; return the latched device status as a code. */
int qsym_sync(qsym_ctx *ctx);

/* Total energy of each system (H_Dft + H_Kep + H_Int, Sec. 2), E[nsys] on
 * the host.  Synchronises. */
int qsym_energy(qsym_ctx *ctx, double *E);

/* Encounter pairs of the last step (Sec. 2.4, the pairs the fine sweep
 * marks; Sec. 2.3 step 4 divides them into sets) as global body indices,
 * i < j, lexicographically sorted, into pairs[2*cap] (host); *n_pairs receives the
 * true count (QSYM_ETRUNC if above cap).  set_id (host, ntot entries, may
 * be NULL) receives each body's set index (sets ordered by their smallest
 * member) or -1.  Synchronises. */
int qsym_encounters(qsym_ctx *ctx, int32_t *pairs, int64_t cap, int64_t *n_pairs,
                    int32_t *set_id);

/* r_crit of every encounter set of the last step (Sec. 2.2, the equation for
 * r_crit: a_H times the largest Hill radius h_i a_i of the set's members;
 * infinite for a set that is a whole system) into rcrit[cap] (host), sets
 * numbered as qsym_encounters numbers them (by smallest member); *n_sets
 * receives the true count (QSYM_ETRUNC if above cap).  Synchronises. */
int qsym_set_rcrit(qsym_ctx *ctx, double *rcrit, int64_t cap, int64_t *n_sets);

/* Candidate pairs of the last crude sweep (Sec. 2.4, the first sweep;
 * unordered, i < j) into pairs[2*cap] (host); *n receives the true count.
 * QSYM_EOVERFLOW when the sweep found more than the list holds (the step
 * itself then ran the fine test over all pairs and lost nothing).
 * Synchronises. */
int qsym_candidates(qsym_ctx *ctx, int32_t *pairs, int64_t cap, int64_t *n);

int qsym_stats(qsym_ctx *ctx, qsym_stats_t *out);
/* Message of the last failure of ctx; with ctx = NULL, of the last failure
 * on this thread that had no context (qsym_create, qsym_workspace_bytes). */
const char *qsym_last_error(const qsym_ctx *ctx);

/* Operator-level entry points running the step's own kernels on the
 * context state, for operator-by-operator checks.
 *  drift:  E_Dft(dt) (Sec. 2, H_Dft).
 *  kick:   E_Int(dt) over all pairs without K (Sec. 2, H_Int); when
 *          crude_tau != 0 the per-body quantities are recomputed at the
 *          current state and the crude sweep of Sec. 2.4 with step
 *          crude_tau is fused in (read it with qsym_candidates).
 *  kepler: E_Kep(dt) of every body (Appendix A).  */
int qsym_apply_drift(qsym_ctx *ctx, double dt);
int qsym_apply_kick(qsym_ctx *ctx, double dt, double crude_tau);
int qsym_apply_kepler(qsym_ctx *ctx, double dt);

/* Fine sweep of Sec. 2.4 on caller data (all device pointers, SoA [3][n]
 * for q0, v0, q1, v1): flags[k] = 1 when candidate k = (pairs[2k],
 * pairs[2k+1]) approaches within a_E x Hill radius over the step, with the
 * two sides of the comparison in lhs[k], rhs[k] (may be NULL).  Stateless;
 * runs on `stream` and synchronises it. */
int qsym_fine_test(const qsym_params *p, double m0, double tau, int64_t n, const double *m,
                   const double *h, const double *A, const double *q0, const double *v0,
                   const double *q1, const double *v1, int64_t npairs, const int32_t *pairs,
                   int32_t *flags, double *lhs, double *rhs, void *stream);

/* Launch shape of the two kick kernels, which = 0 for the plain kick,
 * 1 for the kick with the fused crude sweep (-1: both, set only):
 * ipl = i-bodies per lane (1, 2, 4), block = threads per workgroup (128,
 * 256), jchunk = j-bodies per workgroup (a multiple of block and at least
 * the smallest j-chunk the workspace was sized for), remap bit 0 for the
 * XCD-aware workgroup order, bit 1 (symmetric kick only) for the work
 * items in order of decreasing pair count instead of chunk by chunk (the
 * short diagonal and ragged items dispatched last), sym = 0 for the full-matrix kick (every
 * ordered pair) or 1, 2, 4, 8 for the symmetric kick (every unordered pair
 * once, the reaction applied to j; ipl 1 or 2 only; sym i-blocks of
 * block*ipl bodies per work item, jchunk a multiple of block*ipl; the
 * j-side partial sums need at most min(ceil(n/128), 128) slots, so a shape
 * whose i-ranges of sym*block*ipl bodies exceed that fails with
 * QSYM_EINVAL), or 16 for the symmetric kick over balanced rows: rows of
 * block*ipl bodies, each cut along j into work items of equal pair count,
 * as many items as the device holds resident workgroups of the kernel, so
 * that all of them run in one round and finish together (jchunk unused
 * beyond the checks; remap should be 0).  qsym_autotune times every candidate shape of both kicks on
 * the current state (without moving it), each launch followed by the
 * reduction of its partial sums, keeps the fastest, and writes those two
 * times (kick + reduction) in microseconds to us[0] (plain) and us[1]
 * (crude sweep).  Results do not depend on the shape beyond rounding. */
int qsym_set_kick_shape(qsym_ctx *ctx, int32_t which, int32_t ipl, int32_t block, int64_t jchunk,
                        int32_t remap, int32_t sym);
int qsym_get_kick_shape(qsym_ctx *ctx, int32_t which, int32_t *ipl, int32_t *block,
                        int64_t *jchunk, int32_t *remap, int32_t *sym);
int qsym_autotune(qsym_ctx *ctx, double tau, double *us);

/* Profiling: when enabled, qsym_step launches kernels directly (no graph)
 * with HIP events around each launch, accumulating per-kernel time into
 * qsym_stats_t.phase_us.  Kernel index order: 0 drift+prepass, 1 kick with
 * crude sweep, 2 kick apply + Kepler, 3 fine sweep, 4 sets, 5 Hermite,
 * 6 second kick, 7 kick apply + momentum, 8 final drift, 9 energy.
 * enable = 2 also records workgroups for the busy_* load-balance figures
 * (the symmetric kick then runs its recording variant, and the records are
 * read back every 64 recorded launches, which synchronises the stream);
 * 0 turns profiling off.  Enabling clears the accumulated figures. */
int qsym_profile(qsym_ctx *ctx, int32_t enable);

/* ------------------------------------------------------------------------
 * Learned starting value of the Kepler solve (kepler_mode 2).  Not in the
 * paper, which iterates from a fixed start (Appendix A).  With r0 = |x0|,
 * s = sign(dt), T = sqrt(mu)|dt|/r0^1.5, alpha = 2/r0 - v0^2/mu:
 *   features f = (ln r0, s x0.v0/sqrt(mu r0), alpha r0, ln T)
 *   start    x = (sqrt(mu) dt/r0) exp(T (o s_y + m_y))
 * where o is a 4-32-32-1 tanh network on (f_k - m_k)/s_k.  Weights are
 * QSYM_GUESS_WEIGHTS floats: W1[32][4] (row = first-layer unit) at 0,
 * b1 at 128, W2[32][32] (row = second-layer unit) at 160, b2 at 1184,
 * W3 at 1216, b3 at 1248, then m_0..m_3, s_0..s_3, m_y, s_y.
 * Newton from the start stops at |dx| <= 1e-14 |x|.  A start whose ratio to
 * the first-order guess sqrt(mu) dt / r0 is not within [r0/r_max, r0/q]
 * (apocentre r_max, infinite for e >= 1; pericentre q), where the root's
 * ratio always lies, is replaced by the first-order guess, and Newton that
 * reaches its cap restarts as Laguerre from the first-order guess, so bad
 * weights cost iterations, never the result.
 * ------------------------------------------------------------------------ */
#define QSYM_GUESS_PARAMS 1249
#define QSYM_GUESS_WEIGHTS 1259

/* Weights of the learned start used by kepler_mode 2 (copied; where =
 * QSYM_HOST or QSYM_DEVICE).  qsym_step and qsym_apply_kepler fail with
 * QSYM_EINVAL in kepler_mode 2 until weights are set. */
int qsym_set_guess(qsym_ctx *ctx, const float *weights, int32_t where);

/* Stand-alone Kepler roots (Appendix A) of n bodies, each with its own
 * step: state is device SoA [6][n] (x, y, z, vx, vy, vz), dt device [n],
 * mode as kepler_mode (weights: device QSYM_GUESS_WEIGHTS floats, needed
 * for mode 2 only), x_out device [n] receives the universal anomaly, iters
 * (device [n], may be NULL) the iteration count, negated when every start
 * reached the cap.  Enqueued on `stream`, not synchronised. */
int qsym_kepler_solve(double mu, int64_t n, const double *state, const double *dt, int32_t mode,
                      const float *weights, double *x_out, int32_t *iters, void *stream);
/* The learned start alone (x_out device [n]; 0 for a zero step, not
 * finite when the network or the features are unusable). */
int qsym_kepler_guess(double mu, int64_t n, const double *state, const double *dt,
                      const float *weights, double *x_out, void *stream);

/* Training of the learned start on the GPU.  Samples are device FP32
 * column-major: rows 0..3 of feat hold f, row 4 the target
 * y = ln(x / x_p) / T of a solved root x, rows ld floats apart.  The loss of
 * n samples is (1/n) sum (o - (y - m_y)/s_y)^2.  A trainer owns its device
 * scratch (allocated at creation) and the Adam moments; it runs on
 * `stream`.  max_batch bounds n of qsym_guess_grad and the batch of
 * qsym_guess_train. */
typedef struct qsym_guess_trainer qsym_guess_trainer;
int qsym_guess_trainer_create(int64_t max_batch, void *stream, qsym_guess_trainer **out);
void qsym_guess_trainer_destroy(qsym_guess_trainer *tr);
const char *qsym_guess_trainer_error(const qsym_guess_trainer *tr);
/* zero the Adam moments and the step count */
int qsym_guess_reset(qsym_guess_trainer *tr);
/* features and targets (x_root device [n], may be NULL: targets 0) of n
 * bodies; QSYM_EINVAL when a sample has a zero step or a non-finite
 * feature or target.  Synchronises the stream. */
int qsym_guess_prepare(qsym_guess_trainer *tr, double mu, int64_t n, const double *state,
                       const double *dt, const double *x_root, float *feat, int64_t ld);
/* means and population deviations of the 5 rows into weights[1249..1258]
 * (a zero deviation becomes 1) */
int qsym_guess_fit_scalers(qsym_guess_trainer *tr, const float *feat, int64_t ld, int64_t n,
                           float *weights);
/* dL/dw (device [1249]) of n samples; loss (host, may be NULL) receives L
 * and then the stream is synchronised. */
int qsym_guess_grad(qsym_guess_trainer *tr, const float *weights, const float *feat, int64_t ld,
                    int64_t n, float *grad, double *loss);
/* qsym_guess_grad without allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving or training
 * loops, harnesses that forbid it): no trainer; the partial sums of its
 * waves and the loss accumulator live in a static device array of
 * 1.28 MB that each GPU holds from the first call on it until the process
 * ends.  weights (device, QSYM_GUESS_WEIGHTS floats), feat (device, rows of
 * ld floats as for qsym_guess_grad) and grad (device [1249], output) belong
 * to the caller; loss (host, may be NULL) receives L and then the stream is
 * synchronised.  n must be 1 .. QSYM_GUESS_STATIC_MAX, else QSYM_EINVAL
 * (message in qsym_last_error(NULL)).  Results are those of qsym_guess_grad
 * with the same n (same kernels, same partial layout).  All calls on one GPU
 * share its array: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  Enqueued on
 * `stream`. */
#define QSYM_GUESS_STATIC_MAX 16384
int qsym_guess_grad_static(const float *weights, const float *feat, int64_t ld, int64_t n,
                           float *grad, double *loss, void *stream);
/* one Adam update (Kingma & Ba 2015, Alg. 1) of weights[0..1248] from grad */
int qsym_guess_adam(qsym_guess_trainer *tr, float *weights, const float *grad, double lr,
                    double b1, double b2, double eps);
/* epochs of mini-batch Adam (b1 0.9, b2 0.999, eps 1e-8) over the samples
 * in order, batches of `batch`, learning rate decayed from lr to lr_final
 * on a half cosine over the epochs; curve (host [epochs], may be NULL)
 * receives each epoch's mean loss.  Synchronises the stream. */
int qsym_guess_train(qsym_guess_trainer *tr, float *weights, const float *feat, int64_t ld,
                     int64_t n, int64_t batch, int32_t epochs, double lr, double lr_final,
                     double *curve);

#ifdef __cplusplus
}
#endif

#endif /* QSYM_H */

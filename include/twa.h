/*
 * twa.h -- C ABI of the MI355X three-weight message-passing trajectory
 * planner (Bento, Derbinsky, Alonso-Mora, Yedidia, "A message-passing
 * algorithm for multi-agent trajectory planning", NIPS 2013).
 *
 * One call of twa_iterate(s, k) runs k full iterations of the algorithm of
 * App. B over the factor graph of Sec. 3.3 on the solver's HIP stream:
 *   fixed start/goal factors, energy factors (App. E), agent-agent collision
 *   factors over every pair of agents and every segment (Sec. 3.3.1, App. C),
 *   agent-wall factors (Sec. 3.3.2, App. D), each emitting x and a weight
 *   0 / rho0 / infinity; the weighted-consensus z update and the <-rho weight
 *   of every break-point node; the u (dual) update of every edge.
 *
 * Conventions for every entry point
 *   - Array arguments are DEVICE pointers (e.g. a torch CUDA tensor's
 *     data_ptr()) that must be valid on the solver's stream.  The caller owns
 *     them; the solver copies what it needs and never keeps a pointer.
 *   - float is IEEE binary32; arrays are dense and row-major as documented.
 *   - Break-point positions ("trajectories") have layout [p][eta+1][dim]:
 *     agent i, break-point s (0 = start x_i(0), eta = goal x_i(T)).
 *   - Every call returns a twa_status; no C++ exception crosses the ABI.
 *     On failure twa_last_error() describes the cause.  A device error
 *     (TWA_E_DEVICE) latches: every later call on that solver fails with it.
 *   - Calls are asynchronous on the stream unless stated; calls on one
 *     solver must not overlap (one host thread at a time).
 *
 * Canonical edge order (used by state get/set and the per-edge debug output;
 * factor order is the same with one entry per factor):
 *   1. fixed factors, for i = 0..p-1: start(i), goal(i)          1 edge each
 *   2. energy factors, for i, for s = 0..eta-1: [(i,s), (i,s+1)]
 *   3. collision factors, for s, for i < j (row-major):
 *        [(i,s), (i,s+1), (j,s), (j,s+1)]
 *   4. wall factors, for s, for i, for w = 0..n_walls-1: [(i,s), (i,s+1)]
 *   E = 2p + 2 eta p + 4 eta p(p-1)/2 + 2 eta p n_walls edges.
 * Weight codes: 0 = zero (inactive), 1 = rho0 (standard), 2 = infinity.
 */
#ifndef TWA_H_
#define TWA_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct twa_solver twa_solver;

typedef enum {
    TWA_OK = 0,
    TWA_E_INVALID = 1,    /* bad argument (size, null pointer, NaN, flag) */
    TWA_E_INFEASIBLE = 2, /* start or goal positions overlap, or touch a wall */
    TWA_E_NOMEM = 3,      /* device allocation failed */
    TWA_E_DEVICE = 4,     /* a HIP call failed; latched */
    TWA_E_NUMERIC = 5,    /* non-finite value found by twa_check_finite */
    TWA_E_STATE = 6       /* call not valid in the solver's current state */
} twa_status;

enum { TWA_W_ZERO = 0, TWA_W_STD = 1, TWA_W_INF = 2 };

/* twa_create flags */
enum {
    /* Read u of every edge every iteration, the literal dense form of
     * App. B step 7 (u is written where the update changes it: a u that
     * the rule resets to zero and that is zero already is not stored
     * again).  Without it an edge whose factor sent weight 0 keeps no u (it
     * is zero by the update rule), and a bit per factor records which
     * factors carry one.  Results are identical. */
    TWA_F_DENSE = 1u << 0,
    /* Make twa_backward available: the solver remembers the state each run
     * starts from (at create, twa_set_init and twa_set_state).  No cost per
     * iteration. */
    TWA_F_TAPE = 1u << 1,
    /* Standard ADMM instead of the three-weight algorithm: every factor sends
     * weight rho0 on every edge (no zero or infinite weights), so <-rho is
     * rho0 everywhere and the start/goal factors take part in the consensus
     * like any other (Sec. 2, App. B: the three-weight algorithm reduces to
     * ADMM when every weight is rho0).  Implies TWA_F_DENSE.  For comparing
     * the two methods; twa_backward is not available in this mode. */
    TWA_F_ADMM = 1u << 2,
    /* What the factor between consecutive break-points of an agent is (at
     * most one of these; default: the kinetic-energy cost of
     * eq. velo_cost_pair_wise, C = energy coefficient):
     *   COST_NONE    no cost, feasibility only (Sec. 4): the factor is absent
     *                (weight zero), C unused;
     *   COST_MAXVEL  |x_i(s+1) - x_i(s)| <= C_{i,s} (eq. max_vel_min, App. F),
     *                weight rho0 while the limit binds, else zero;
     *   COST_MINVEL  |x_i(s+1) - x_i(s)| >= C_{i,s} (App. G), likewise.
     * Velocity limits must be > 0.  twa_backward needs the energy cost. */
    TWA_F_COST_NONE = 1u << 3,
    TWA_F_COST_MAXVEL = 1u << 4,
    TWA_F_COST_MINVEL = 1u << 5,
    /* One epoch of the velocity-obstacle local planner (Sec. 5, eq.
     * rec_col_avoi_pos, App. H): eta must be 1; x0 are the current positions,
     * xT the reference end positions x^ref = x0 + v^ref tau (preferences:
     * they may overlap), C[i] > 0 the cost c_i of deviating from them.  The
     * goal factors become the VO cost minimiser (energy minimiser with its
     * reference end certain, weight rho0); the collision and wall factors
     * keep their start ends fixed.  The solution's break-point 1 is each
     * agent's collision-free end position for the epoch.  No TWA_F_COST_*
     * flag with it. */
    TWA_F_VO = 1u << 6
};

typedef struct {
    long long iter;          /* iterations run so far */
    long long active_coll;   /* collision factors with weight rho0, last iteration */
    long long active_wall;   /* wall factors with weight rho0, last iteration */
    long long queued;        /* factors that went through a full minimiser, last iteration */
    double residual;         /* primal residual of the last iteration: max |x - z| over the edges
                                whose u it updated (both weights rho0, App. B step 7); 0 when no
                                iteration ran since the state was set */
    double objective;        /* energy objective of z, as twa_get_quality */
    double min_clearance;    /* smallest clearance of z, as twa_get_quality */
    long long graph_iterations; /* iterations run so far from replayed HIP graphs */
    long long tape_checkpoints; /* checkpoints of the current run on the forward tape
                                   (TWA_F_TAPE: made by the first twa_backward, it records
                                   from the next start of a run; see twa_backward) */
} twa_stats;

/*
 * Device memory provider (boundary convention of this library; the paper
 * has no such notion).  Every device buffer that a later twa_create,
 * twa_batch_create or twa_backward allocates comes from
 *   alloc(bytes, device, stream, ctx)      -> device pointer, NULL on failure
 * and goes back through
 *   release(ptr, bytes, device, stream, ctx)
 * where device is the HIP device of the solver and stream its hipStream_t.
 * The library calls release only once its own work on that memory is done
 * (it synchronises the stream first), so a stream-ordered pool such as a
 * caching allocator may hand the block out again at once.  A failed alloc
 * makes the call fail with TWA_E_NOMEM.  alloc and release must both be
 * NULL (restore hipMalloc / hipFree, the default) or both be set, else
 * TWA_E_INVALID.  Process-wide; each solver and batch keeps the pair in
 * effect when it was created for its whole life, so changing it does not
 * affect existing ones.  The callbacks run on the calling thread, inside
 * the library call that needs memory, and must not call into this library.
 * twa_backward_noalloc never calls them.
 */
typedef void *(*twa_alloc_fn)(size_t bytes, int device, void *stream, void *ctx);
typedef void (*twa_free_fn)(void *ptr, size_t bytes, int device, void *stream, void *ctx);
twa_status twa_set_allocator(twa_alloc_fn alloc, twa_free_fn release, void *ctx);

/*
 * Create a solver for one planning problem (Sec. 1 problem statement,
 * Sec. 3.1-3.2 formulation).
 *   p >= 1 agents, eta >= 1 segments (eta+1 break-points), dim 2 or 3.
 *   radii [p]          agent radii r_i > 0.
 *   x0, xT [p][dim]    start and goal positions (constants, Sec. 3).
 *   n_walls >= 0, walls [n_walls][2][dim] segment end points (x_L, x_R),
 *                      planar only (Sec. 3.2): n_walls > 0 needs dim == 2.
 *                      May be NULL when n_walls == 0.
 *   C [p][eta]         energy coefficient C_{i,s} >= 0 of segment (i, s)
 *                      (eq. velo_cost_pair_wise, prefactor folded in).
 *   rho0 > 0           standard weight; alpha > 0 step (App. B step 7 uses
 *                      alpha/rho0).
 *   flags              TWA_F_* above.
 *   hip_stream         hipStream_t on which every call runs.  NULL: the solver
 *                      makes its own stream with the default flags, which
 *                      orders itself with the null stream both ways (work the
 *                      caller queues on the null stream before or after a call
 *                      stays in order) and, unlike the null stream, can be
 *                      captured into the graphs twa_iterate replays.
 * Starts must be pairwise >= r_i + r_j apart, and so must goals; no start or
 * goal may lie within r_i of a wall (TWA_E_INFEASIBLE otherwise; overlaps up
 * to 1e-5 relative, the rounding of positions left in contact, are accepted).
 * Initial state: straight lines from start to goal, u = 0, <-rho = infinity
 * at start and goal, rho0 elsewhere.  Synchronises the stream.
 * On success *out owns all device memory it allocated (twa_destroy frees it).
 */
twa_status twa_create(int p, int eta, int dim, const float *radii, const float *x0, const float *xT,
                      int n_walls, const float *walls, const float *C, float rho0, float alpha,
                      unsigned flags, void *hip_stream, twa_solver **out);

/* Initial break-points z [p][eta+1][dim] (break-points 0 and eta are
 * replaced by the start and goal); resets u to 0 and <-rho to the default. */
twa_status twa_set_init(twa_solver *s, const float *z);

/* New start and goal positions x0, xT [p][dim] (device) for the same
 * problem shape, radii, walls, costs and flags -- e.g. the next epoch of the
 * velocity-obstacle planner (Sec. 5), whose starts are the agents' current
 * positions and whose goals are the new reference end positions.  Validated
 * as at create (finite, feasible; TWA_E_INFEASIBLE otherwise), and within the
 * coordinate range the solver was created for (TWA_E_INVALID otherwise: the
 * consensus scale depends on it).  Resets the state to straight lines, u = 0,
 * and the default <-rho, as twa_create does.  Synchronises the stream. */
twa_status twa_set_endpoints(twa_solver *s, const float *x0, const float *xT);

/* Sec. 4's warm-up: the standard weight is rho0_init for the first n_warm
 * iterations counted from 0, then the create-time rho0 (the paper uses
 * eta p 1e-5 for 20 iterations).  The warm-up weight enters the minimisers;
 * the u step of App. B step 7 stays alpha / rho0 with the create-time rho0
 * (over the warm-up value the iterates diverge). */
twa_status twa_set_schedule(twa_solver *s, float rho0_init, int n_warm);

/* Run k >= 0 iterations (App. B steps 1-7), asynchronously.  Iterations at
 * the steady rho0 are replayed from HIP graphs of 32, 16, ..., 1 iterations
 * (captured together the first time, so any k replays); an instance of at
 * most 256 collision + wall factors (or 512 collision factors and no walls)
 * runs them in one persistent single-workgroup launch instead (bitwise the
 * same iterations). */
twa_status twa_iterate(twa_solver *s, int k);

/* Iterate until the plan is collision-free: up to max_iter >= 0 iterations
 * in blocks of every >= 1, with the smallest clearance that twa_get_quality
 * reports (Sec. 2 pairs, Sec. 3.2 walls) taken after each block and after
 * the last iteration; stops after the first block whose clearance is
 * >= min_clearance (the stopping rule of a velocity-obstacle epoch, Sec. 5).
 * Writes the iterations run to *done (host int) and 1 to *met (host int) if
 * the bar was met, else 0.  The iterations and the clearance are those of
 * twa_iterate followed by twa_get_quality, bitwise.  A tiny instance (as for
 * twa_iterate's single-workgroup launch, state within 56 KiB of LDS, at the steady
 * rho0, no forward tape) runs the whole call on the device, the clearance
 * taken inside the persistent launch, and synchronises once; otherwise each
 * block is launched and checked from the host.  TWA_E_INVALID for a null
 * out-pointer, max_iter < 0, every < 1 or a NaN bar. */
twa_status twa_iterate_until(twa_solver *s, int max_iter, int every, double min_clearance, int *done, int *met);

/* As twa_iterate, and times the kernels with HIP events on the solver's
 * stream; synchronises and writes the device time in milliseconds of each
 * kernel summed over the k iterations to kernel_ms (host array of 3: factor
 * stream, queued minimisers, node consensus).  The last min(k, 2)
 * iterations are launched on their own, every kernel with a start and a stop
 * event attached to its dispatch (hipExtLaunchKernel), so each pair spans
 * the kernel alone (an event recorded on the stream slows every later launch
 * of the call, so the captured graph replays before them carry none); their
 * mean times stand for all k iterations. */
twa_status twa_iterate_timed(twa_solver *s, int k, double *kernel_ms);

/* Current consensus positions z [p][eta+1][dim]. */
twa_status twa_get_trajectories(twa_solver *s, float *z_out);

/* Full state after the last iteration: z [p][eta+1][dim], u [E][dim] in
 * canonical edge order, <-rho [p][eta+1] (codes above), iteration count
 * (host pointer, may be NULL).  Any device pointer may be NULL to skip it. */
twa_status twa_get_state(twa_solver *s, float *z, float *u, unsigned char *lrho, long long *iter);

/* Replace the state (same layouts as twa_get_state); iter is host memory. */
twa_status twa_set_state(twa_solver *s, const float *z, const float *u, const unsigned char *lrho,
                         long long iter);

/* Debug output of the NEXT twa_iterate(s, 1): x [E][dim] (canonical edge
 * order) and ->rho per factor [F] (canonical factor order), written during
 * that iteration.  Pass NULLs to switch it off.  The buffers must stay valid
 * until that iteration has run. */
twa_status twa_capture_next(twa_solver *s, float *x_out, unsigned char *rho_out);

/* Counters and measures of the last iteration (host struct; synchronises
 * the stream).  Settles the pending u update of the last iteration (the next
 * iteration is bitwise the same either way).  Returns TWA_E_NUMERIC, with the
 * struct filled, when a consensus sum left its fixed-point range since the
 * state was set (see twa_check_finite). */
twa_status twa_get_stats(twa_solver *s, twa_stats *out);

/* Measures of the current break-points z, in double precision from the FP32
 * positions (host pointers, any may be NULL; synchronises the stream):
 *   objective      sum over agents i and intervals s of C[i][s] |z_i(s+1) -
 *                  z_i(s)|^2, the energy cost of Sec. 3.1 (evaluated with the
 *                  create-time C whatever the cost mode);
 *   min_clearance  the smallest of: closest approach of agents i and j moving
 *                  at constant velocity over an interval minus r_i + r_j
 *                  (Sec. 2), over every pair and interval; distance of agent
 *                  i's interval segment to a wall minus r_i (Sec. 3.2, planar)
 *                  over every interval and wall; +infinity with neither;
 *   max_move       the largest distance a break-point moved in the last
 *                  iteration (0 after create, set_init or set_state).
 * Computed on the device; allocates nothing (its 24-byte buffer is made at
 * create).  Non-finite positions drop out of the minimum and the maximum
 * (twa_check_finite reports them). */
twa_status twa_get_quality(twa_solver *s, double *objective, double *min_clearance, double *max_move);

/* Sizes: factors and edges in canonical order (host pointers). */
twa_status twa_sizes(const twa_solver *s, long long *n_factors, long long *n_edges);

/* Scan z and u for NaN/Inf (synchronises): TWA_E_NUMERIC if any, or if a
 * consensus contribution since the state was last set (create, set_init,
 * set_state) was non-finite or beyond the fixed-point range of the node sums
 * (see twa_consensus_scale): the iterates diverged and z may be wrong. */
twa_status twa_check_finite(twa_solver *s);

/* The fixed-point scale of the consensus sums that twa_create picks for p
 * agents, n_walls walls and coordinates of magnitude at most coord_max (>= 1;
 * twa_create uses the largest |coordinate| of starts, goals and walls, at
 * least 1), and the largest |m| one edge may contribute before the overflow
 * flag of twa_check_finite is raised.  Host only (no device needed):
 * TWA_E_INVALID on bad arguments. */
twa_status twa_consensus_scale(int p, int n_walls, double coord_max, double *scale, double *limit);

/*
 * Reverse-mode gradient of a loss L(z^K) of the trajectories after the run
 * (not a step of the paper: the derivative of its unrolled iterations).
 * Needs TWA_F_TAPE at create.  The run is every iteration since the last
 * twa_create / twa_set_init / twa_set_state, K = their number.  Each of the
 * K iterations of App. B is differentiated with its discrete decisions held
 * at the forward run's (the 0 / rho0 / infinity weights, and which candidate
 * configuration each collision and wall minimiser took); the minimisers'
 * derivatives come from their optimality conditions (App. C, D, E, I).
 *   dL_dz  [p][eta+1][dim]  dL/dz^K (read).
 *   dL_dx0 [p][dim]         dL/dx(0) (written): through the fixed start
 *                           factors and break-point 0 of the initial state.
 *   dL_dxT [p][dim]         dL/dx(T) (written), likewise.
 *   dL_dr  [p]              dL/dr_i (written), through the active collision
 *                           and wall minimisers.
 *   dL_dz0 [p][eta+1][dim]  dL/dz^0 at the interior break-points (written;
 *                           0 at s = 0 and s = eta), or NULL.
 * All device arrays, caller-owned.  The initial u is held constant.
 * Checkpoints every ceil(sqrt(K)) iterations (z and <-rho dense; u of the
 * collision and wall factors sparse, as it is zero on every factor that sent
 * weight 0) and recomputes one segment at a time, the factor kernels
 * capturing each iteration's weights and the minimiser inputs of the
 * factors that sent rho0.  A segment's reverse steps run on a second stream
 * that the solver makes at create (TWA_F_TAPE), while the segment before it
 * is recomputed on the solver's stream.  The first call also sizes and
 * allocates a forward tape: from the next start of a run (twa_set_init,
 * twa_set_state, twa_set_endpoints) twa_iterate packs the state every 32
 * iterations into it (64 checkpoints, runs of up to 2,048 iterations), and
 * a call over a run the tape covers takes its checkpoints from there instead
 * of re-running the forward (segments a multiple of 32 near sqrt(K));
 * otherwise it re-runs the forward as the first call did.  The results are
 * the same either way (the forward is bitwise unchanged by recording).  Its buffers are allocated at the
 * first call and kept, grown when a later call needs more, until
 * twa_destroy (TWA_E_NOMEM if they do not fit).  The solver's forward state
 * is the same afterwards.  dim == 2 only (TWA_E_INVALID otherwise);
 * TWA_E_STATE without TWA_F_TAPE.  Synchronises both streams.
 */
twa_status twa_backward(twa_solver *s, const float *dL_dz, float *dL_dx0, float *dL_dxT, float *dL_dr,
                        float *dL_dz0);

/*
 * twa_backward for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid allocation): the same computation,
 * arguments, results and errors, with every buffer taken from a static
 * scratch array of 128 MiB that the library holds on each device it runs on
 * (from its first use there until the process ends; its address is looked
 * up when a TWA_F_TAPE solver is created).  Calls no hipMalloc / hipFree and
 * captures no new HIP graph (graphs the solver already holds are replayed).
 * A run whose checkpoints and captured records do not fit returns
 * TWA_E_NOMEM with the sizes in twa_last_error; twa_backward has no such
 * limit.  Every call on one device shares that device's scratch, which keeps
 * the last call's contents: calls that overlap on one device (other host
 * threads, other streams) race and must be serialised by the caller.
 */
twa_status twa_backward_noalloc(twa_solver *s, const float *dL_dz, float *dL_dx0, float *dL_dxT, float *dL_dr,
                                float *dL_dz0);

/* Text of the last error on this solver ("" if none). */
const char *twa_last_error(const twa_solver *s);

/* Release every device buffer (synchronises the stream).  NULL is a no-op. */
void twa_destroy(twa_solver *s);

/* Library version string. */
const char *twa_version(void);

/* ------------------------------------------------------------------------
 * Batched instances.  Many independent problems of uneven p, eta and dim
 * advance together in ONE persistent kernel launch (captured in a HIP
 * graph): a workgroup owns a bin of whole instances and runs every
 * iteration of each with workgroup barriers only.  Each instance evolves
 * exactly as it would in its own solver (same arithmetic, bitwise).
 * ------------------------------------------------------------------------ */
typedef struct twa_batch twa_batch;

/* One instance of a batch: the twa_create arguments (device pointers) and
 * an optional initial z0 [p][eta+1][dim] (NULL = straight lines). */
typedef struct {
    int p, eta, dim, n_walls;
    const float *radii, *x0, *xT, *walls, *C, *z0;
    float rho0, alpha;
} twa_instance;

/* Create n >= 1 solvers (validation and errors as twa_create; the status of
 * the first failing instance is returned) sharing one stream. */
twa_status twa_batch_create(int n, const twa_instance *inst, unsigned flags, void *hip_stream,
                            twa_batch **out);

/* Launch shape.  block 256, 512 or 1024: the persistent kernel, with that
 * many lanes per workgroup and `groups` workgroups (bins; clamped to n);
 * instances are packed onto bins longest-first and each bin runs all k
 * iterations of its instances in one launch.  block 0 (groups ignored):
 * one launch per phase of an iteration (factor stream, minimisers,
 * consensus) over the blocks of every instance, so a large instance spreads
 * over many compute units.  Either way the evolution is bitwise that of the
 * instances' own solvers.  Default: 256 lanes, one bin per instance. */
twa_status twa_batch_config(twa_batch *b, int block, int groups);

/* k >= 0 iterations of every instance (one launch of the persistent kernel,
 * or 3k launches in the phased form; captured in a HIP graph either way). */
twa_status twa_batch_iterate(twa_batch *b, int k);

/* As twa_batch_iterate; *ms = device time of the launch (synchronises). */
twa_status twa_batch_iterate_timed(twa_batch *b, int k, double *ms);

/* Number of instances (host pointer). */
twa_status twa_batch_size(const twa_batch *b, int *n);

/* Instance i's solver, owned by the batch (for state get/set, stats...).
 * Do not destroy it; do not give it a rho0 schedule. */
twa_status twa_batch_solver(twa_batch *b, int i, twa_solver **s);

/* twa_get_trajectories of instance i. */
twa_status twa_batch_get_trajectories(twa_batch *b, int i, float *z_out);

const char *twa_batch_last_error(const twa_batch *b);

/* Frees every instance and the batch (synchronises).  NULL is a no-op. */
void twa_batch_destroy(twa_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* TWA_H_ */

/*
 * dd_uot.h -- C ABI of the MI355X domain-decomposition solver for entropic
 * unbalanced optimal transport on 2-D grids (Medina, Nguyen, Schmitzer,
 * "Domain decomposition for entropic unbalanced optimal transport").
 *
 * Problem (Definition unbalanced-entropic-transport, Sec. 2.2; choices of
 * Sec. 4.1): point masses mu, nu > 0 on the same n1 x n2 grid x = h (i1, i2),
 * cost c(x, y) = |x - y|^2, entropic strength eps, marginal penalties
 * D1 = D2 = lambda KL.  The solver runs Algorithm 2 (alternating composite
 * partitions A and B) with the parallel DomDecIter of Algorithm 4: every
 * composite cell of a partition is solved at once by the unbalanced Sinkhorn
 * iteration of Sec. 4.1 (X-update eq. sinkhorn-X-iteration, Y-update
 * eq. proxdiv-problem by Newton, stopping rule eq. PD-gap-KL), the basic-cell
 * Y-marginals are stored on bounding boxes truncated at `trunc` (Sec. 4.4) in
 * device pools that grow with the boxes (no box size limit), and the step
 * weights come from GetWeights (Proposition converging-getweights).
 *
 * Conventions for every function:
 *  - return 0 (DDUOT_OK) or a negative DDUOT_E* code; no C++ exception
 *    crosses the ABI; dd_uot_last_error() gives the calling thread's text;
 *  - arrays are row-major n1 x n2 double (index i1 * n2 + i2) in HOST memory;
 *    inputs are copied, outputs are written into caller-owned buffers of the
 *    stated size;
 *  - a handle owns all device memory it allocates and is not thread-safe:
 *    use one handle per host thread / stream;
 *  - work is queued on the HIP stream given at init (NULL = default stream);
 *    dd_uot_iterate is asynchronous unless it is asked for statistics.
 */
#ifndef DD_UOT_H
#define DD_UOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DDUOT_OK = 0,
  DDUOT_EINVAL = -1,   /* bad argument: sizes, non-finite or non-positive masses
                          (full-support assumption, Sec. 3.2), eps/lambda <= 0 */
  DDUOT_ENOMEM = -2,   /* device allocation failed */
  DDUOT_EHIP = -3,     /* HIP runtime error (text kept in dd_uot_last_error) */
  DDUOT_ESLOT = -4,    /* a step found a device pool too small: the cells that
                          did not fit kept their state (the pools grow before the
                          next step; reported, not fatal) */
  DDUOT_ESTATE = -5    /* call not valid in the handle's state */
};

/* GetWeights (Sec. 3.4): greedy theta = 1, safe theta = 1/(cells updated),
   swift = greedy if the tracked score rises by at most lenience*|score| else
   safe, staggered = every partition in four batches of non-adjacent cells
   (parity of the cell position), one swift step per batch in turn, line =
   the one weight in [1/(cells updated), 1] for every cell that minimises
   the tracked score of the mixture (Proposition converging-getweights,
   item line; the pieces are linear in the weight and the KL term convex),
   opt = one weight per cell in [1/(cells updated), 1] minimising the tracked
   score of the mixture (eq. opt-weights-problem; from the line weight,
   rounds of a projected diagonal Newton direction with an exact search along
   it). */
enum {
  DDUOT_GW_GREEDY = 0,
  DDUOT_GW_SAFE = 1,
  DDUOT_GW_SWIFT = 2,
  DDUOT_GW_STAGGERED = 3,
  DDUOT_GW_LINE = 4,
  DDUOT_GW_OPT = 5
};
enum { DDUOT_INIT_BLOCK = 0, DDUOT_INIT_PRODUCT = 1 };

typedef struct dduot_handle dduot_handle;

typedef struct {
  int32_t n1, n2;            /* grid; each divisible by 2*cell */
  double h;                  /* grid spacing (>= 0; 0 makes the cost vanish) */
  double lambda, eps;        /* > 0 */
  int32_t cell;              /* basic cell side s; composite = 2 x 2 basic cells,
                                partition B offset by s (Sec. 4.4); 2*s <= 16 */
  int32_t precision;         /* 64: FP64 cell arithmetic; 32: cell potentials
                                in FP64, FP32 exponentials of FP64 differences
                                to a per-output shift, FP32 Newton; FP64
                                reductions, scores and certificate */
  int32_t getweights;        /* DDUOT_GW_* ; swift is the default; staggered must be
                                chosen for all problems of a handle or none */
  int32_t init;              /* DDUOT_INIT_BLOCK (nu_i = nu on block i) or
                                DDUOT_INIT_PRODUCT (pi = mu x nu, Sec. 4.2) */
  double sinkhorn_err;       /* Err: a cell stops at PD/lambda <= Err |mu_J|
                                (Sec. 4.4: 2e-5) */
  int32_t sinkhorn_max_iter; /* cap on Y-halves per cell solve */
  int32_t fixed_inner_iters; /* > 0: exactly this many Y-halves per cell */
  double trunc;              /* basic-marginal truncation (Sec. 4.4: 1e-15) */
  double lenience;           /* swift accepts greedy if the tracked score rises
                                by at most lenience*|score| (Sec. 4.4: 0.005) */
  int32_t box_margin;        /* Y-box of a cell = bbox of its basic boxes
                                dilated by this margin, clipped to the grid
                                (any size) */
  int32_t box_cap;           /* box side of the larger in-LDS cell layout
                                (at most what one workgroup's LDS holds);
                                cells with wider boxes keep their arrays in
                                a per-cell global workspace.  A performance
                                setting: the results do not depend on it */
  int32_t translate;         /* 1: before every Y-half, maximise the cell dual
                                exactly along (alpha + s, beta - s) (closed
                                form, removes the slowly contracting constant
                                mode; not in the paper); 0: the paper's plain
                                Sinkhorn iteration */
  int32_t fast_cap;          /* cell solves run in up to three launches: the
                                cells wider than box_cap (workspace layout),
                                then, when fast_cap < box_cap, those wider
                                than fast_cap with the LDS layout of box_cap,
                                then the others with the smaller layout of
                                fast_cap (more workgroups per CU); the results
                                do not depend on it.  0: the largest side whose
                                layout lets three workgroups share a CU */
  int32_t balance;           /* 1: balancing step (Sec. 4.1 "Balancing") after
                                every cell solve: the mass of the cell plan is
                                moved along X between its basic cells, in
                                proportion to mubar = e^{-alpha'/lambda} mu
                                (alpha' the X-half of the final beta), before
                                the re-split; 0 (default): no balancing.
                                Regular Y points only (DDUOT_EINVAL with moved
                                Y points) */
  int32_t support_only;      /* 1 (default): the cell problem lives on the support
                                of nu_J = sum of its basic marginals (Sec. 4.1):
                                box points where nu_J = 0 are left out, so
                                supports grow only through the alternation of
                                the partitions and box_margin has no effect;
                                0: the whole Y-box (then the margin lets
                                supports grow by box_margin per step) */
} dduot_config;

/* Per call of dd_uot_iterate, summed over all problems of the handle. */
typedef struct {
  int32_t half_iters;        /* half-iterations run by the call */
  int32_t n_safe;            /* (problem, half-iteration) pairs that took the
                                safe weights */
  int64_t inner_iters;       /* sum over solved cells of Y-halves */
  int64_t point_iters;       /* sum over solved cells of |X_J| * Y-halves */
  int32_t max_inner;         /* largest Y-half count of one cell */
  int32_t n_unconverged;     /* cells that hit the iteration cap */
  int32_t n_overflow;        /* cells not solved because a pool was too small
                                (then the call returns DDUOT_ESLOT) */
  int32_t n_cells;           /* cells solved (all half-iterations) */
} dduot_iter_stats;

typedef struct {
  double tracked;            /* tracked score sum_i Hbar_i + lambda KL(P_Y pi|nu):
                                an upper bound of E(pi), exact after greedy steps */
  double primal;             /* E(pi_hat) of the certificate plan */
  double dual;               /* D(alpha_bar, beta_hat) */
  double pd_gap;             /* primal - dual = lambda KL(P_X pi_hat | e^{-alpha/lambda} mu),
                                eq. PD-gap-KL with J = I */
  double rel_pd_gap;         /* pd_gap / |dual| (Sec. 4.4 solution quality) */
  double l1_err_x;           /* || P_X pi - e^{-alpha_bar/lambda} mu ||_1 (state plan) */
  double l1_err_y;           /* || P_Y pi - e^{-beta_hat/lambda} nu ||_1 (state plan) */
  double mass_x, mass_y;     /* |P_X pi|, |P_Y pi| of the state plan */
  int64_t half_iters;        /* half-iterations done so far */
  int32_t overflow;          /* nonzero if any step ever found a pool too small */
  int32_t polish_iters;      /* global Sinkhorn iterations of the polished bounds
                                (dd_uot_set_polish; 0 for moved Y points) */
  double dual_polished;      /* max_k D(alpha_k, beta_k) over alpha_0 = alpha_bar
                                and k global iterations (Definition sinkhorn,
                                eq. sinkhorn-iters-ot): a lower bound of the
                                optimal value, >= dual */
  double primal_polished;    /* min(tracked, min_k E(pi_k)) with E(pi_k) = D + PD of
                                the pair k (eq. PD-gap-KL): an upper bound of the
                                optimal value (tracked itself bounds E of the plan) */
  double rel_gap_polished;   /* (primal_polished - dual_polished) / |dual_polished|:
                                a certified relative gap of the state */
  int64_t nnz;               /* stored basic-marginal entries above 1e-14 (the
                                sparsity measure of Sec. 4.2) */
  int64_t n_safe;            /* recorded steps whose weight was below 1 */
  int64_t n_unconverged;     /* recorded cell solves that hit the iteration cap */
} dduot_score;

/* Fill *cfg with the paper's defaults (Err 2e-5, trunc 1e-15, lenience 0.005,
   swift, FP32, block start, margin 2, box_cap 64, max 1000 inner iterations,
   translation step on, no balancing, cell problems on the support of nu_J). */
void dd_uot_default_config(dduot_config* cfg);

/* Create a solver for one problem.  mu, nu: n1*n2 doubles each, in host or
   device memory (told apart by hipPointerGetAttributes; device inputs are
   read once, on hip_stream, into host memory for the set-up), every entry
   finite and > 0 (Assumption full support, Sec. 3.2), each total below 1024
   (the aggregation of the basic-cell marginals sums in fixed point, so its
   results do not depend on the order of the adds), else DDUOT_EINVAL.
   hip_stream: a hipStream_t or NULL.  The start plan is cfg->init. */
int dd_uot_init(const dduot_config* cfg, const double* mu, const double* nu,
                void* hip_stream, dduot_handle** out);

/* Create one solver holding nprob independent problems (sizes and parameters
   may differ); every kernel launch covers all problems' cells at once, and
   GetWeights decides per problem.  mus[k], nus[k]: arrays of problem k (host
   or device memory, each on its own). */
int dd_uot_init_batch(int32_t nprob, const dduot_config* cfgs, const double* const* mus,
                      const double* const* nus, void* hip_stream, dduot_handle** out);

/* Moved Y points (the differentiable form): the Y masses sit at y' instead of
   the grid, cost c(x, y') = |x - y'|^2, which is no longer separable, so the
   cell solves and the certificate use dense sums over explicit point pairs.
   ypos: n1*n2*2 doubles (y'_1, y'_2 of grid point j, row-major; host or
   device memory), finite;
   needs h > 0.  Boxes and partitions stay those of the grid indices, so
   displacements should be small against the cell size.
   dd_uot_init_batch_moved: ypos[k] for every problem, or ypos == NULL for
   none (all problems of a handle share one kind). */
int dd_uot_init_moved(const dduot_config* cfg, const double* mu, const double* nu,
                      const double* ypos, void* hip_stream, dduot_handle** out);
int dd_uot_init_batch_moved(int32_t nprob, const dduot_config* cfgs, const double* const* mus,
                            const double* const* nus, const double* const* ypos,
                            void* hip_stream, dduot_handle** out);

/* Set eps of problem `prob` (epsilon-scaling, Sec. 4.4).  The tracked scores
   were computed for the old eps, so the next half-iteration of that problem
   takes greedy weights, which makes them exact again. */
int dd_uot_set_eps(dduot_handle* h, int32_t prob, double eps);

/* Set the cell tolerance Err of problem `prob` (the stopping rule of
   eq. PD-gap-KL: PD/lambda <= Err |mu_J|).  err >= 0. */
int dd_uot_set_err(dduot_handle* h, int32_t prob, double err);

/* Run n_half_iters parallel DomDecIter steps (Algorithm 4), alternating
   partitions A and B (Algorithm 2; the first step after init uses A).
   stats == NULL: asynchronous on the handle's stream, except that every
   fourth half-iteration the call waits for the queued steps to read the pool
   sizes they needed and grows the pools (state, candidates, cell workspace)
   to twice any need above half a pool.  Otherwise the call synchronises and
   fills *stats for the steps of this call.  DDUOT_ESLOT: some earlier step
   found a pool too small (its cells that did not fit kept their state); the
   pools have been grown and the call can be repeated. */
int dd_uot_iterate(dduot_handle* h, int32_t n_half_iters, dduot_iter_stats* stats);

/* Autotuner: threads per cell workgroup (64, 128 or 256, at least the
   largest composite tile's point count).  Times the cell solves of the next
   partition on the current state once per admissible size (HIP events) and
   keeps the fastest for later steps; the state is unchanged.  chosen
   (nullable) receives the size, ms (nullable, 3 doubles) the times of 64,
   128, 256 threads (-1: not admissible).  Synchronises. */
int dd_uot_autotune(dduot_handle* h, int32_t* chosen, double* ms);

/* Autotuner of the wide cells' launch (see dd_uot_set_gang): times the cell
   solves of the next partition on the current state for one workgroup per
   wide cell and for the gang shapes (G, workgroups per CU) = (2, 2), (4, 1),
   (4, 2), (8, 1), (8, 2), (16, 2), and keeps the fastest; the state is
   unchanged.  G and wgs_per_cu (nullable) receive the choice (0, 0: one
   workgroup per wide cell), ms (nullable, 7 doubles) the times in that
   order (-1: the shape does not apply).  Synchronises. */
int dd_uot_autotune_gang(dduot_handle* h, int32_t* G, int32_t* wgs_per_cu, double* ms);

/* Gangs for the wide cells (boxes wider than box_cap and at most 512
   columns, plain separable problems: no moved Y points, no balancing).  The
   wide cells of a step are listed heaviest first (box points times the
   iterations of the cell's previous solve); the heavy ones, above an even
   share of the total per workgroup, are solved by G workgroups together
   (the box rows split between them; two barriers per inner iteration), the
   light ones by one workgroup each, taken from a queue.  The gang kernel
   keeps at most wgs_per_cu workgroups per CU (within its occupancy; the
   grid is a multiple of 8 G, so every workgroup is resident at once), and
   the members of a gang share one XCD (gangs are formed from the XCD id
   each workgroup reads; workgroups left over on an XCD only take light
   cells).
   G = 0: one workgroup per wide cell.  Default G = 4, wgs_per_cu = 2.  Same
   arithmetic either way; a gang adds its members' partial sums in member
   order, so results depend on G only through rounding.  A barrier that
   waits past 2 s (not expected) abandons the launch's wide cells, and the
   next dd_uot_iterate reports DDUOT_EHIP.  Returns the G in effect (0 when
   gangs do not apply), *nwg (if not NULL) the gang kernel's workgroups. */
int dd_uot_set_gang(dduot_handle* h, int32_t G, int32_t wgs_per_cu, int32_t* nwg);

/* enable != 0: dd_uot_iterate runs pairs of half-iterations (A then B) by
   replaying one captured hipGraph of all their kernels (captured on first
   use; the step's kernels read every parameter from device memory, so the
   graph stays valid across dd_uot_set_eps).  Not used while timing is on. */
int dd_uot_set_graph(dduot_handle* h, int32_t enable);

/* Per step record of problem `prob` (one per half-iteration, four under
   staggered GetWeights: one per batch), oldest first, at most `max`
   records of 12 doubles: theta, tracked score before, tracked score of the
   greedy candidate, cells updated, sum |X_J| * inner iterations, max inner
   iterations, unconverged cells, cells not solved (pool too small), inner iterations,
   algorithmic bytes of the cell solves, log-sum-exp terms of the cell solves,
   pass outputs recomputed in FP64 after an underflow.
   Returns the number of records written (>= 0) or an error code.
   Synchronises. */
int dd_uot_history(dduot_handle* h, int32_t prob, int32_t max, double* out);

/* Primal-dual certificate of the current state of problem `prob`: the
   stitched cell potentials alpha_bar (last solve of each cell), one global
   Y-update with nu_- = 0 (eq. sinkhorn-iters-ot) giving beta_hat, and the
   gap of eq. PD-gap-KL for the plan pi_hat they define.  Synchronises. */
int dd_uot_score(dduot_handle* h, int32_t prob, dduot_score* out);

/* Number of global Sinkhorn iterations dd_uot_score runs from the stitched
   potential for the polished bounds (default 0: the polished fields repeat
   the certificate's pair).  0 <= n_iters <= 10000. */
int dd_uot_set_polish(dduot_handle* h, int32_t n_iters);

/* X- and Y-marginal of the current state plan (P_X pi and sum_i nu_i).
   px, py: n1*n2 doubles each, host or device memory (either may be NULL).
   Synchronises. */
int dd_uot_marginals(dduot_handle* h, int32_t prob, double* px, double* py);

/* Stored Y-marginal nu_i of basic cell `basic` (row-major ids over the
   (n1/cell) x (n2/cell) blocks).  box[4] receives (o1, o2, L1, L2); values
   receives L1*L2 doubles if L1*L2 <= cap, else DDUOT_EINVAL (values == NULL:
   only the box).  Synchronises. */
int dd_uot_basic_marginal(dduot_handle* h, int32_t prob, int32_t basic, int32_t box[4],
                          double* values, int64_t cap);

/* Whole state of a single-problem handle (checkpoint / resume; moving a state
   between handles of the same problem, e.g. FP64 -> FP32): the basic-cell
   Y-marginals (Algorithm 4 state) on their boxes, P_X pi, the tracked pieces
   Hbar_i, the stitched potential and its per-cell flags, and the count of
   half-iterations done.  Layouts: boxes nbasic*4 int32 (o1, o2, L1, L2 per
   basic cell, row-major basic ids); values the boxes' entries concatenated in
   basic order (row-major inside a box); px, abar n1*n2 doubles; hbar nbasic
   doubles; warm nbasic int32.  All host memory.
   dd_uot_get_state: *n_values receives the number of values; values may be
   NULL (then only *n_values and the other outputs), else it must hold
   cap >= *n_values doubles (else DDUOT_EINVAL).  Any other pointer may be
   NULL.  Synchronises.
   dd_uot_set_state: replaces the state (every pointer required; boxes inside
   the grid, values finite and >= 0, n_values their total area); the next
   half-iteration uses partition A if k is even, B otherwise, and is greedy
   (force_greedy != 0) or follows GetWeights.  Synchronises.  Both:
   DDUOT_EINVAL for a handle with several problems. */
int dd_uot_get_state(dduot_handle* h, int32_t* boxes, double* values, int64_t cap,
                     int64_t* n_values, double* px, double* hbar, double* abar, int32_t* warm,
                     int64_t* k);
int dd_uot_set_state(dduot_handle* h, const int32_t* boxes, const double* values,
                     int64_t n_values, const double* px, const double* hbar, const double* abar,
                     const int32_t* warm, int64_t k, int32_t force_greedy);

/* alpha_bar (stitched cell potentials) and, after dd_uot_score, beta_hat.
   Either pointer may be NULL; n1*n2 doubles each, host or device memory.
   Synchronises. */
int dd_uot_potentials(dduot_handle* h, int32_t prob, double* alpha, double* beta_hat);

/* Gradient of the optimal value W(mu, nu) at the certificate pair (envelope
   theorem on the dual of Definition unbalanced-entropic-transport):
   dW/dmu = eps|nu| - eps P_X pi_hat/mu - lambda (e^{-alpha/lambda} - 1),
   dW/dnu = eps|mu| - eps P_Y pi_hat/nu - lambda (e^{-beta/lambda} - 1),
   scaled by gout on the device.  Exact at the optimum; call after
   dd_uot_score.  dmu, dnu: n1*n2 doubles each, host or device memory
   (either may be NULL).  Synchronises. */
int dd_uot_backward(dduot_handle* h, int32_t prob, double gout, double* dmu, double* dnu);

/* Gradient of the optimal value with respect to the Y positions at the
   certificate plan pi_hat: dW/dy'(y) = sum_x pi_hat(x, y) 2 (y' - x) (the
   cost derivative integrated against the plan; exact at the optimum), for
   the grid or the moved points, scaled by gout.  The plan is recomputed on
   the fly by dense pruned sums (no stored plan).  Call after dd_uot_score.
   dypos: n1*n2*2 doubles, host or device memory.  Needs h > 0. */
int dd_uot_backward_ypos(dduot_handle* h, int32_t prob, double gout, double* dypos);

/* Cell-kernel timing with HIP events recorded on the handle's stream around
   every cell-solve launch (enable != 0 turns it on and clears the totals).
   dd_uot_kernel_time returns the number of timed launches and their summed
   duration in milliseconds, and the summed algorithmic bytes of those
   launches.  Synchronises. */
int dd_uot_set_timing(dduot_handle* h, int32_t enable);
int dd_uot_kernel_time(dduot_handle* h, int64_t* launches, double* total_ms,
                       double* algo_bytes);

/* Per composite cell of partition `part` (0: A, 1: B; all problems, in cell
   order) as of the last step that solved it: its Y-box (o1, o2, l1, l2 in
   `boxes`, 4 int32 per cell), its inner Sinkhorn iterations (-1: not solved
   for lack of pool space) and its log-sum-exp terms.  Host arrays of at
   least `max` entries (per cell); any may be NULL.  Returns the partition's
   cell count, or a negative error code (max too small, bad part).
   Synchronises. */
int dd_uot_cell_stats(dduot_handle* h, int32_t part, int32_t max, int32_t* boxes,
                      int32_t* iters, double* terms);

/* ---- Multiscale (Sec. 4.4 "Multi-scale and eps-scaling") ----------------- */

/* New handle for the grid with twice the points per axis, started from the
   refined state of the single problem of `coarse`: every coarse plan entry
   is split in proportion to the fine masses inside its 2 x 2 points, a fine
   basic cell takes the share |mu(X_i)| / |mu(X_I)| of the refined Y-marginal
   of its coarse basic cell I (boxes double, then truncate at cfg->trunc and
   shrink).  cfg: the fine problem (n = 2 n_coarse,
   every fine basic cell inside one coarse basic cell: cell divides twice
   the coarse cell, or is 1; same precision); mu, nu: host fine
   marginals, whose 2 x 2 sums should be the coarse ones.  The first
   half-iteration of the new handle is greedy (the tracked pieces are
   estimates until then).  `coarse` is left unchanged. */
int dd_uot_refine(dduot_handle* coarse, const dduot_config* cfg, const double* mu,
                  const double* nu, void* hip_stream, dduot_handle** out);

/* Linear interpolation of a potential (cost units) to the grid with twice the
   points per axis: coarse point I stands for the fine points {2I, 2I+1} and
   its value is placed at the fine position 2I + 1/2; each axis is linear
   between the two nearest such positions and continued linearly beyond the
   first and last (a single coarse point: constant).  Exact for affine
   potentials.  coarse: host, n1c*n2c doubles; fine: host, 4*n1c*n2c. */
int dd_uot_interpolate_potential(const double* coarse, int32_t n1c, int32_t n2c, double* fine,
                                 void* hip_stream);

/* Global unbalanced Sinkhorn on the grid of cfg (Definition sinkhorn, the
   closed-form updates eq. sinkhorn-iters-ot with nu_- = 0), FP64, separable
   log-sum-exp: alpha = X-update(beta) from the warm beta; then per iteration
   the Y-update, the gap pd = KL(P_X pi | e^{-alpha/lambda} mu) of the pair
   (alpha, beta) (eq. PD-gap-KL divided by lambda), stop if pd <= tol, else the
   X-update.  On return beta is the last Y-update; alpha is the potential it
   was computed from when the tolerance stopped the loop, else the X-update
   of beta (max_iter reached).  Uses n1, n2, h, lambda, eps of cfg.
   mu, nu: host, n1*n2, finite and > 0; alpha (out), beta (in: warm start,
   out): host, n1*n2; iters, pd (nullable): iterations done, last gap.
   Allocates and frees its own device buffers; synchronises. */
int dd_uot_global_sinkhorn(const dduot_config* cfg, const double* mu, const double* nu,
                           double* alpha, double* beta, int32_t max_iter, double tol,
                           void* hip_stream, int32_t* iters, double* pd);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the global
   Sinkhorn of dd_uot_global_sinkhorn on caller-owned device buffers, with no
   hipMalloc, hipFree or other allocating call.  mu, nu (in), alpha (out),
   beta (in: warm start, out): device memory, n1*n2 doubles each, else
   DDUOT_EINVAL; the masses finite and > 0, beta finite (checked on the
   device).  The iteration's scratch (five grids and the partial sums) is a
   file-scope device array of the library sized for grids of at most
   256 x 256 = 65 536 points (2.6 MB per GPU, held until the process ends):
   larger grids give DDUOT_EINVAL.  Every call on one GPU uses that GPU's
   one array, so calls that overlap on one GPU (other threads, other
   streams) race; nothing in it needs clearing between calls.  Same
   iterations, results and gap as dd_uot_global_sinkhorn.  Synchronises
   hip_stream (once per iteration, reading the gap). */
int dd_uot_global_sinkhorn_noalloc(const dduot_config* cfg, const double* mu, const double* nu,
                                   double* alpha, double* beta, int32_t max_iter, double tol,
                                   void* hip_stream, int32_t* iters, double* pd);

/* New single-problem handle whose state is the plan of the potentials
   (alpha, beta) (cost units), pi = exp((alpha + beta - c)/eps) mu x nu
   (Sec. 4.1), split by basic cells (Sec. 4.4 Sinkhorn warm start):
   nu_i(y) = sum_{x in X_i} pi(x, y) over the whole grid, entries below trunc
   dropped, box = bbox of the rest; P_X pi
   and the tracked pieces are those of the kept cell plans, alpha is the
   stitched potential.  The first half-iteration is greedy.  alpha, beta:
   host, n1*n2, finite.  Needs cell * (n1 + n2) doubles to fit the LDS of
   one workgroup (the scan). */
int dd_uot_init_duals(const dduot_config* cfg, const double* mu, const double* nu,
                      const double* alpha, const double* beta, void* hip_stream,
                      dduot_handle** out);

typedef struct {
  int32_t levels;            /* layers; the coarsest has n / 2^(levels-1) points per axis */
  int32_t coarse_cell;       /* basic cell side on the coarser layers (the coarsest
                                layer uses one composite cell for the whole grid
                                when its side is at most 16) */
  double eps_start_h2;       /* eps at the start of a layer, in units of its h^2 (paper: 2) */
  double eps_end_h2;         /* eps at the end of a coarser layer, same units (paper: 1/2);
                                eps halves in between */
  int32_t halves_per_stage;  /* half-iterations per eps stage, at least */
  int32_t stage_max_halves;  /* ... continued in groups of halves_per_stage until the
                                certificate's relative gap is <= stage_gap, at most this */
  double stage_gap;
  int32_t coarse_max_iter;   /* cap on inner iterations per cell on the coarser layers */
  int32_t final_max_halves;  /* cap on half-iterations after the finest stage */
  int32_t check_every;       /* certificate (dd_uot_score) every this many */
  double target_rel_gap;     /* stop once the relative primal-dual gap is below */
  int32_t dd_from;           /* side of the first layer solved by DD; the coarser layers
                                run the global Sinkhorn (dd_uot_global_sinkhorn), the plan
                                of the last one's potentials is split by basic cells
                                (dd_uot_init_duals) and refined to the first DD layer
                                (Sec. 4.4 "Sinkhorn warm start": DD from 256^2 on).  The
                                finest layer is always DD.  0: every layer is DD, the
                                coarsest one started from the product or block plan */
  int32_t global_max_iter;   /* global Sinkhorn iterations per eps stage, at most */
  double global_tol;         /* a global eps stage ends once
                                KL(P_X pi | e^{-alpha/lambda} mu) <= global_tol |mu|
                                (Sec. 4.4: a quarter of the DD tolerance) */
  int32_t coarse_box_cap;    /* DD layers other than the finest use the in-LDS
                                layout max(cfg->box_cap, coarse_box_cap) (<= 128) */
  double coarse_lenience;    /* ... and this GetWeights lenience */
  int32_t verbose;           /* 1: one progress line per layer and eps stage on
                                stderr (layer, eps, half-iterations, gaps,
                                elapsed time); 0: silent */
  int32_t polish_iters;      /* global Sinkhorn iterations of the polished bounds
                                of the final-stage certificates (dd_uot_set_polish);
                                > 0: the final stage stops on rel_gap_polished */
  double final_err_ratio;    /* > 0: after every final-stage certificate the cell
                                tolerance becomes max(final_err_min,
                                min(Err, final_err_ratio * gap)) (the cell
                                solves' error bounds the reachable gap);
                                0: Err stays fixed */
  double final_err_min;
} dduot_multiscale;

/* levels 7, coarse_cell 4, eps 2 h^2 -> h^2/2 per layer, 4..16 half-iterations
   per stage (stage gap 1e-3), 1000 inner iterations on coarse layers, at most
   200 final half-iterations, certificate every 4, target 1e-6; global Sinkhorn
   below 256 points per axis, at most 2000 iterations per eps stage, tolerance
   5e-6 (a quarter of Err = 2e-5); coarser DD layers with box cap 80 and
   strict GetWeights (lenience 0). */
void dd_uot_default_multiscale(dduot_multiscale* m);

/* Coarse-to-fine solve with eps-scaling: coarsen (mu, nu) by 2 x 2 sums to
   `levels` layers; the layers coarser than dd_from run the global Sinkhorn
   through their eps stages (beta carried to the next layer by
   dd_uot_interpolate_potential as its warm start), and the plan of the last
   one's potentials, split by basic cells of side min(cell, coarse_cell)
   (dd_uot_init_duals), is refined to the first DD layer; with dd_from = 0
   the coarsest layer starts from the product plan if its side is at most
   64 or box_cap (layers of side <= 64 widen box_cap to the grid), else the
   block start.
   On every DD layer run the eps stages, then refine (dd_uot_refine); on the
   finest layer continue to cfg->eps and then iterate until the
   certificate's relative gap is <= target_rel_gap or final_max_halves are
   done.  trace (nullable, trace_cap records of 5 doubles): per certificate of
   the final stage, (total half-iterations, elapsed ms since the call,
   relative certificate gap pd_gap/|dual|, relative gap of the DD plan
   (tracked - dual)/|dual|, rel_gap_polished); *trace_len gets their count;
   the final stage stops on the certificate gap, or on the polished gap when
   polish_iters > 0.  *out receives the finest handle (its state, score,
   backward). */
int dd_uot_solve_multiscale(const dduot_config* cfg, const dduot_multiscale* ms,
                            const double* mu, const double* nu, void* hip_stream,
                            dduot_handle** out, double* trace, int32_t trace_cap,
                            int32_t* trace_len);

int dd_uot_synchronize(dduot_handle* h);
int32_t dd_uot_num_problems(const dduot_handle* h);
/* Box sides of the in-LDS cell layouts of h (see fast_cap and box_cap): the
   fast tier's and the larger one; equal when one in-LDS launch does every
   cell that fits. */
int dd_uot_launch_caps(const dduot_handle* h, int32_t* fast_cap, int32_t* box_cap);
void dd_uot_destroy(dduot_handle* h);
const char* dd_uot_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DD_UOT_H */

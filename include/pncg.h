/*
 * pncg.h - C ABI of libpncg, a gfx950 (MI355X) implementation of the
 * Jacobi-preconditioned Dai-Kou nonlinear conjugate gradient (PNCG) solver
 * for the IPC incremental potential of Shen et al., "Preconditioned
 * Nonlinear Conjugate Gradient Method for Real-time Interior-point
 * Hyperelasticity" (SIGGRAPH 2024).
 *
 * Problem (Sec. 3, equations E and Hessian): one implicit-Euler step
 *     x^{t+1} = argmin_x 1/2 (x - xt)^T M (x - xt) + h^2 Psi(x)
 *                        + kappa sum_k b(d_k(x)),
 *     xt = x^t + h v^t + h^2 g,      v^{t+1} = (x^{t+1} - x^t) / h,
 * Psi Neo-Hookean on linear tets (Sec. 3.1), b the IPC log barrier
 * (Sec. 3, equation barrier) over point-triangle and edge-edge pairs
 * (Sec. 3.2, equations PT and EE) and over surface-vertex/plane pairs,
 * minimised by Algorithm 1 (Sec. 4) with the one-pass step bound
 * (Sec. 4.3, equations upper and alpha) in place of continuous collision
 * detection.
 *
 * Conventions for every entry point:
 *  - Return value: PNCG_OK (0) on success, PNCG_W_* (> 0) for a warning
 *    with valid outputs, PNCG_E_* (< 0) for an error; after an error the
 *    outputs are unspecified and pncg_last_error() describes it.
 *  - Indices are 0-based int32.  Positions, velocities and per-vertex
 *    vectors are float64, shape (n, 3), row-major (x0 y0 z0 x1 ...).
 *  - Pointers named *_dev are device pointers (hipMalloc'd or a torch CUDA
 *    tensor's data_ptr) on the context's device; all other pointers are host
 *    pointers.  Inputs are only read during the call and never retained;
 *    host inputs are copied.  Outputs are written before the call returns
 *    (device outputs: ordered on the context's stream, which the call
 *    synchronises before returning).  Device inputs are read on the
 *    context's stream, which waits for no other stream: inputs written on
 *    another stream (e.g. torch's) must be complete before the call, or the
 *    context must be created on that stream (pncg_opts.stream).
 *  - The context owns all of its device memory and frees it in
 *    pncg_destroy.  A context must not be used from two threads at once.
 *  - Call order: pncg_create, pncg_set_mesh, pncg_set_material, then
 *    optionally pncg_set_contact / pncg_set_solver / pncg_set_dirichlet,
 *    then steps and queries.  Out-of-order calls return PNCG_E_STATE.
 */
#ifndef PNCG_H
#define PNCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pncg_ctx pncg_ctx;

/* status codes */
#define PNCG_OK              0
#define PNCG_W_MAXITER       1   /* iteration cap reached before the stop test */
#define PNCG_E_INVAL        -1   /* bad argument (size, index, NaN in a parameter) */
#define PNCG_E_NOMEM        -2   /* device or host allocation failed */
#define PNCG_E_HIP          -3   /* a HIP runtime call failed */
#define PNCG_E_STATE        -4   /* call out of order (e.g. step before set_mesh) */
#define PNCG_E_PENETRATION  -5   /* some contact pair or plane distance is <= 0 */
#define PNCG_E_INVERTED     -6   /* a tet with det F <= 0 (rest or deformed) */
#define PNCG_E_NONFINITE    -7   /* NaN or Inf in an input or in the iterate */
#define PNCG_E_CAPACITY     -8   /* an output buffer is too small (size reported) */
#define PNCG_E_INDEFINITE   -9   /* the adjoint CG met p^T H p <= 0 (H not positive
                                    definite at the given state) */

/* arithmetic of the per-element and per-vertex work */
#define PNCG_FP64   0   /* everything in float64 */
#define PNCG_MIXED  1   /* float32 element math and vectors; float64 positions,
                           distances, barrier terms and every reduction */

/* termination (Algorithm 1 and Sec. 4.4) */
#define PNCG_TERM_DELTA_E   0   /* stop after an update with dE < eps * dE_0 */
#define PNCG_TERM_GRAD_REL  1   /* stop at the top of an iteration when
                                   ||g||_2 <= eps * ||g_0||_2 */
#define PNCG_TERM_GRAD_ABS  2   /* stop at the top of an iteration when
                                   ||g||_2 <= eps (absolute; for steps that
                                   start near equilibrium, where ||g_0|| is
                                   itself near the gradient's rounding floor) */

/* solver flags */
#define PNCG_BARRIER_FULL        1u  /* use the pair Hessian of equation eq9
                                        verbatim instead of its PSD projection */
#define PNCG_ALPHA_INF_COMPONENT 2u  /* step bound with the largest |p_i|
                                        instead of the largest per-vertex |p_v|_2 */
/* beta rule (a field of the solver flags; the ablation of Sec. 7.1 names
 * these beside Dai-Kou).  With z = P g, d = the previous direction, y = g -
 * g_prev and P the Jacobi preconditioner of each iteration:
 *   DK  g^T P y / d^T y - (y^T P y / d^T y)(d^T g / d^T y)     (default)
 *   FR  g^T P g / (g_prev^T P_prev g_prev)
 *   PRP g^T P y / (g_prev^T P_prev g_prev)
 *   CD  -g^T P g / (d^T g_prev)
 *   HZ  g^T P y / d^T y - 2 (y^T P y / d^T y)(d^T g / d^T y)
 * A zero denominator or a non-finite value gives 0; a direction that is
 * not a descent direction restarts with -P g, for every rule. */
#define PNCG_BETA_DK    0u
#define PNCG_BETA_FR    (1u << 4)
#define PNCG_BETA_PRP   (2u << 4)
#define PNCG_BETA_CD    (3u << 4)
#define PNCG_BETA_HZ    (4u << 4)
#define PNCG_BETA_MASK  (7u << 4)
/* Splitting computation (Sec. 5.2): every object (the object_id given to
 * pncg_set_mesh) gets its own beta, search direction and step size
 * alpha_o = min(dhat / (2 max_{v in o} |p_v|), -g_o^T p_o / p_o^T H p_o), where
 * p_o^T H p_o is the object's diagonal block of H (a pair between two
 * objects adds its term to each with the other side's direction left out);
 * dE is the sum over objects.  Needs object ids non-decreasing over the
 * vertices and the tets grouped by object (E_INVAL from pncg_set_solver
 * otherwise).  With one object the step is the unsplit one. */
#define PNCG_SPLIT_OBJECTS (1u << 8)

/* material models (pncg_set_model, pncg_batch_set_model) */
#define PNCG_MODEL_NH   0
#define PNCG_MODEL_SNH  1
#define PNCG_MODEL_ARAP 2
#define PNCG_MODEL_FCR  3

/* contact flags */
#define PNCG_CONTACT_SELF          1u  /* point-triangle and edge-edge pairs
                                          (all objects, including self) */
#define PNCG_CONTACT_REST_EXCLUDE  2u  /* drop same-object pairs closer than
                                          1.5 dhat in the rest shape (Sec. 5.1) */

/* candidate kinds for pncg_candidates */
#define PNCG_KIND_PT 0   /* (surface vertex, surface triangle) */
#define PNCG_KIND_EE 1   /* (surface edge e1, surface edge e2), e1 < e2 */
#define PNCG_KIND_PG 2   /* (surface vertex, plane) */

/* How the per-vertex sums of the contact-pair terms are formed (the scatter-add
 * of a pair's gradient, diagonal and H p terms into its four vertices,
 * Sec. 3.2 equations eq8-eq11 and Sec. 4.2).  pncg_opts.scatter:
 *   PNCG_SCATTER_AUTO       the library's choice: SEGMENTED
 *   PNCG_SCATTER_ATOMIC     float64 atomic adds per pair corner; the order of
 *                           the additions, and so the last bits of any result
 *                           with active pairs, may differ from run to run
 *   PNCG_SCATTER_SEGMENTED  every (pair, corner) writes its own slot and each
 *                           vertex adds its slots in a fixed order (the
 *                           candidate list is put in lexicographic order at
 *                           every build): steps and queries are
 *                           bit-reproducible.  The per-object pair curvature
 *                           of the split step (PNCG_SPLIT_OBJECTS) is still
 *                           summed with atomics. */
#define PNCG_SCATTER_AUTO      0
#define PNCG_SCATTER_ATOMIC    1
#define PNCG_SCATTER_SEGMENTED 2

typedef struct {
  int32_t device;      /* HIP device ordinal */
  int32_t precision;   /* PNCG_FP64 or PNCG_MIXED */
  void*   stream;      /* hipStream_t to run on; NULL = a stream the context creates */
  int32_t scatter;     /* PNCG_SCATTER_*; 0 = AUTO */
  int32_t chunk;       /* iterations launched between host status reads; 0 = default */
  int32_t graphs;      /* 0: the candidate-list rebuild of a step is captured once
                          as a HIP graph and replayed (one host call instead of
                          about twenty launches; re-captured when a buffer it
                          uses is reallocated); 1: its kernels are launched one
                          by one.  Results are the same bits either way; the
                          allocation-free step always launches them one by
                          one.  Ignored by pncg_batch_create. */
} pncg_opts;

typedef struct {
  int32_t iters;            /* position updates made in the step */
  int32_t reason;           /* 0 dE rule, 1 gradient rule, 2 iteration cap,
                               3 zero or unbounded direction */
  double  dE0;              /* dE of the first iteration */
  double  last_dE;          /* dE of the last iteration */
  double  g0_norm;          /* ||g_0||_2 */
  double  g_norm;           /* ||g||_2 at the last gradient evaluation */
  int32_t alpha_upper_hits; /* iterations where dhat/(2|p|) was the smaller step */
  int32_t rebuilds;         /* candidate-list rebuilds during the step */
  int64_t n_candidates;     /* PT + EE candidates of the last list built */
  int64_t n_active;         /* active PT + EE + plane pairs at the last evaluation */
} pncg_stats;

/* Create a context on opts->device (opts may be NULL: device 0, FP64).
 * *out receives the context.  Errors: E_INVAL, E_HIP, E_NOMEM. */
int pncg_create(pncg_ctx** out, const pncg_opts* opts);

/* Free the context and all device memory it owns.  NULL is accepted. */
void pncg_destroy(pncg_ctx* ctx);

/* Message for the last error of this context (never NULL; "" if none).
 * With ctx == NULL: the last error of pncg_create on this thread. */
const char* pncg_last_error(const pncg_ctx* ctx);

/* Rest mesh (Sec. 3.1: constant-strain tets, F = D_s D_m^{-1}).
 *   X      [nV][3] rest positions
 *   tets   [nT][4] vertex indices, positively oriented: det[X1-X0, X2-X0,
 *          X3-X0] > 0, otherwise E_INVERTED
 *   tris   [nF][3] boundary triangles (contact primitives; may be nF = 0)
 *   edges  [nE][2] boundary edges (contact primitives; may be nE = 0)
 *   object_id [nV] object index per vertex, or NULL (one object); used by
 *          the rest-pose exclusion
 * Every vertex must belong to at most 64 tets (E_INVAL otherwise).
 * Resets material, contact, solver and prescribed vertices. */
int pncg_set_mesh(pncg_ctx* ctx, int32_t nV, const double* X, int32_t nT,
                  const int32_t* tets, int32_t nF, const int32_t* tris,
                  int32_t nE, const int32_t* edges, const int32_t* object_id);

/* Per-tet material: Young's modulus E > 0, Poisson ratio 0 <= nu < 0.5,
 * density rho > 0, each [nT].  Lame parameters mu = E/(2(1+nu)),
 * lam = E nu/((1+nu)(1-2nu)); lumped mass m_v = sum rho V_e / 4. */
int pncg_set_material(pncg_ctx* ctx, const double* E, const double* nu,
                      const double* rho);

/* Elastic density (Sec. 3.1 invariants I1 = tr S of F = R S, I2 = tr F^T F,
 * I3 = det F; the materials of Table 1), with (mu, lam) from
 * pncg_set_material:
 *   PNCG_MODEL_NH   Neo-Hookean, mu/2 (I2 - 3) - mu log I3
 *                   + lam/2 log^2 I3 (the default)
 *   PNCG_MODEL_SNH  stable Neo-Hookean, mu/2 (I2 - 3) - mu (I3 - 1)
 *                   + lam'/2 (I3 - 1)^2 with lam' = lam + mu (its
 *                   small-strain limit is linear elasticity with mu, lam)
 *   PNCG_MODEL_ARAP as-rigid-as-possible, mu |F - R|^2
 *   PNCG_MODEL_FCR  fixed corotated, mu |F - R|^2 + lam/2 (I3 - 1)^2
 * R is the rotation of the rotation-variant polar decomposition, so SNH,
 * ARAP and FCR are defined for inverted tets; steps report E_INVERTED only
 * for det F <= 0 under NH, and under ARAP/FCR where two singular values of
 * the rotation-variant decomposition sum to <= 0 (the I1 Hessian is
 * undefined there).  Hessians are exact (not projected).  May be called
 * at any time after pncg_create; the choice persists across pncg_set_mesh
 * and applies to steps, queries and the adjoint.  E_INVAL for an unknown
 * model. */
int pncg_set_model(pncg_ctx* ctx, int32_t model);

/* Barrier parameters (Sec. 3, equation barrier): dhat > 0, kappa >= 0;
 * cell = spatial-hash cell size (> 0) or 0 for a size derived from the
 * surface; planes [nP][4] rows (n0, n1, n2, o) with |n| = 1 describing the
 * half-spaces n.x >= o; flags PNCG_CONTACT_*. */
int pncg_set_contact(pncg_ctx* ctx, double dhat, double kappa, double cell,
                     int32_t nP, const double* planes, uint32_t flags);

/* Solver settings (Algorithm 1): iter_max >= 1, eps >= 0, term
 * PNCG_TERM_*, gravity[3] (m/s^2, f_ext = m g), flags PNCG_BARRIER_FULL /
 * PNCG_ALPHA_INF_COMPONENT, or-ed with one PNCG_BETA_* rule.  Defaults: 100,
 * 1e-3, DELTA_E, (0,0,-9.8), 0 (Dai-Kou). */
int pncg_set_solver(pncg_ctx* ctx, int32_t iter_max, double eps, int32_t term,
                    const double* gravity, uint32_t flags);

/* Test hook for the constraint set (Algorithm 1, ComputeConstraintSet):
 * replace the spatial-hash candidates of one kind by an explicit list for the
 * following steps and energy / gradient / H p / adjoint queries.  The narrow
 * phase still keeps only the pairs with 0 < d < dhat (Sec. 3, equation
 * barrier), so a list that holds every pair within dhat gives the same
 * results as the hash.
 *   kind PNCG_KIND_PT: pairs [n][2] = (v, f), v a vertex and f a triangle of
 *                      pncg_set_mesh, v not a corner of f
 *   kind PNCG_KIND_EE: pairs [n][2] = (e1, e2), two edges of pncg_set_mesh
 *                      without a shared vertex, e1 != e2
 * While any override is installed the hash is not used for those calls: the
 * candidates are the installed lists, and a kind never installed has none.
 * Installing a kind again replaces its list; n < 0 removes every override
 * (pairs may then be NULL).  The list is copied.  Only has an effect with
 * PNCG_CONTACT_SELF.  pncg_candidates and pncg_min_distance keep using the
 * hash.  Errors: E_INVAL (unknown kind, index out of range, a pair sharing a
 * vertex, a repeated pair), E_STATE before pncg_set_mesh, which clears every
 * override. */
int pncg_set_candidates_override(pncg_ctx* ctx, int32_t kind, int64_t n, const int32_t* pairs);

/* Performance settings (results do not depend on them beyond rounding
 * order).  skin > 0: the solver keeps the pairs within dhat + skin at the
 * last list build and rebuilds the list when the accumulated displacement
 * bound exceeds skin / 2 (Algorithm 1's per-iteration constraint set is the
 * active subset of that list); 0 = the default, 0.4 x the mean surface-edge
 * rest length less dhat, clamped to [2, 8] dhat.  If the contact cell was left to
 * the library (cell = 0), it becomes max(1.5 x mean surface edge, dhat + skin).
 * chunk > 0: iterations launched between reads of the device status (0
 * keeps the current value; default 16).  Call after pncg_set_contact, which
 * keeps a skin set here.  The call also drops a candidate list carried from
 * an earlier step (see pncg_step), so the next step builds its own. */
int pncg_set_tuning(pncg_ctx* ctx, double skin, int32_t chunk);

/* Mean rest length of the surface edges given to pncg_set_mesh (0 if
 * none), for the larger-dhat strategy of Sec. 5.1: dhat at 30-70 % of it,
 * with PNCG_CONTACT_REST_EXCLUDE dropping the same-object pairs closer than
 * 1.5 dhat at rest.  E_STATE before pncg_set_mesh. */
int pncg_mean_boundary_edge(pncg_ctx* ctx, double* out);

/* on = 1: each pncg_adjoint_step* call starts its CG from the lambda of the
 * previous call on this context (consecutive steps of a backward pass have
 * close lambdas), with r = b - H lambda; the stop rule stays relative to
 * |b|.  Without self contact only (otherwise ignored); the first call after
 * pncg_set_mesh starts from 0.  Default 0. */
int pncg_set_adjoint_warm_start(pncg_ctx* ctx, int32_t on);

/* Prescribed vertices for the following steps: idx [n] (distinct),
 * target [n][3] positions they take at the start of the next step (their
 * gradient, direction and update are zero during it).  n = 0 clears. */
int pncg_set_dirichlet(pncg_ctx* ctx, int32_t n, const int32_t* idx,
                       const double* target);

/* One time step (Algorithm 1) from (x, v) with step size h > 0:
 * x_out, v_out [nV][3] receive x^{t+1} and v^{t+1}; st (nullable) the step
 * statistics.  Returns PNCG_W_MAXITER if the cap was hit, E_PENETRATION /
 * E_INVERTED / E_NONFINITE if the input or the result is infeasible.
 * x_out may alias x and v_out may alias v.  With self contact a step may
 * start on the candidate list the previous step of this context left, if
 * that list still covers x (checked on the device; otherwise the step
 * rebuilds it at x); the result then differs from a fresh list's only in
 * the rounding order of the pair sums.  For bit-identical replays from a
 * saved state, drop the list first (pncg_set_tuning). */
int pncg_step(pncg_ctx* ctx, const double* x, const double* v, double h,
              double* x_out, double* v_out, pncg_stats* st);

/* Same with device pointers (no host copies of the state). */
int pncg_step_dev(pncg_ctx* ctx, const double* x_dev, const double* v_dev,
                  double h, double* x_out_dev, double* v_out_dev,
                  pncg_stats* st);

/* Allocation-free variant of pncg_step_dev, for callers that cannot
 * allocate device memory during a call (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  Same arguments, results
 * and errors as pncg_step_dev, and the same kernels.  The step's reduction
 * scratch (its status record, the per-block partial sums of the
 * per-iteration kernels and one scalar record per iteration) lives in a
 * static device array of 1 MiB that the library holds on every device it
 * runs on until the process ends; the per-vertex state and the candidate
 * buffers are the context's, sized by pncg_set_mesh, pncg_set_contact and
 * earlier steps.  Every call on one device shares that device's array, so
 * calls that overlap on one device (from two host threads, or on two
 * streams) race and must not be made.  Errors, besides pncg_step_dev's:
 * E_INVAL for iter_max above PNCG_NOALLOC_ITER_MAX or a split step
 * (PNCG_SPLIT_OBJECTS); E_STATE with profiling on; E_CAPACITY when the
 * candidate list or the spatial grid would have to grow (outputs are then
 * unspecified, a state passed in place is left unchanged, and one
 * pncg_step_dev call grows the buffers). */
#define PNCG_NOALLOC_ITER_MAX 9566
int pncg_step_dev_noalloc(pncg_ctx* ctx, const double* x_dev, const double* v_dev, double h,
                          double* x_out_dev, double* v_out_dev, pncg_stats* st);

/* nsteps >= 1 time steps in place on the device state x_dev, v_dev [nV][3]
 * (each exactly as pncg_step_dev with the outputs written over the
 * inputs), without returning to the caller in between: a simulation loop
 * with no per-step host round trip.  steps (nullable) receives one
 * pncg_stats per step, [nsteps].  Returns the first error, else
 * PNCG_W_MAXITER if any step hit the iteration cap, else PNCG_OK.  After
 * E_PENETRATION, E_INVERTED or E_CAPACITY the state holds the last
 * completed step; after E_NONFINITE (found as the failed step writes its
 * result, or as the next step reads it: the host waits only for the end of
 * the last step, the steps before it run back to back) it may hold that
 * non-finite result, and the statistics of the step that produced it are
 * reported as if it had succeeded.  E_INVAL for nsteps < 1 or a NULL state. */
int pncg_run_dev(pncg_ctx* ctx, double* x_dev, double* v_dev, double h,
                 int32_t nsteps, pncg_stats* steps);

/* Queries at a given x with the active set computed at x (Algorithm 1,
 * ComputeConstraintSet), in the context's precision.  xt is the predictor.
 *   pncg_energy:   E(x) of equation E
 *   pncg_gradient: g = dE/dx and diag(H) (Sec. 3 and 4.2), [nV][3] each;
 *                  prescribed rows: g = 0, diag = 1.  diag may be NULL.
 *   pncg_hvp:      p^T H p (Sec. 3, with the PSD-projected pair Hessian
 *                  unless PNCG_BARRIER_FULL) and optionally Hp [nV][3]
 *                  (NULL to skip); p is treated as 0 on prescribed rows. */
int pncg_energy(pncg_ctx* ctx, const double* x, const double* xt, double h,
                double* energy);
int pncg_gradient(pncg_ctx* ctx, const double* x, const double* xt, double h,
                  double* g, double* diag);
int pncg_hvp(pncg_ctx* ctx, const double* x, const double* p, double h,
             double* Hp, double* pHp);

/* Candidate pairs of the given kind at x with inflation r = dhat, by the
 * inflated-AABB test in float64 (see the kinds above), after topology and
 * rest-pose exclusions, sorted lexicographically: pairs [cap][2].  *n
 * receives the count; if it exceeds cap the call returns E_CAPACITY and
 * writes nothing. */
int pncg_candidates(pncg_ctx* ctx, const double* x, int32_t kind,
                    int32_t* pairs, int64_t cap, int64_t* n);

/* The solver's own pair list at x (the constraint set of Algorithm 1 with
 * the list skin of pncg_set_tuning): point-triangle or edge-edge candidates
 * by the inflated-AABB test with r = dhat + skin whose closest distance
 * (Sec. 3.2, float64) is below dhat + skin, after topology and rest-pose
 * exclusions, built by the same kernels a step uses for its list (a
 * candidates override set with pncg_set_candidates_override is ignored
 * here).  Sorted lexicographically, pairs [cap][2], edge-edge pairs as
 * (e1, e2) with e1 < e2; *n receives the count, and if it exceeds cap the
 * call returns E_CAPACITY and writes nothing.  Empty without
 * PNCG_CONTACT_SELF.  E_INVAL for another kind. */
int pncg_solver_pairs(pncg_ctx* ctx, const double* x, int32_t kind,
                      int32_t* pairs, int64_t cap, int64_t* n);

/* Penetration audit (Sec. 6: discrete collision check per frame): smallest
 * distance over all non-excluded point-triangle, edge-edge and
 * surface-vertex/plane pairs within 10 dhat, and smallest det F. */
int pncg_min_distance(pncg_ctx* ctx, const double* x, double* dmin,
                      double* jmin);

/* Per-kernel timing of steps (tracing aid).  With profiling on, every
 * launch a step makes is bracketed by HIP events recorded on the context's
 * stream; durations are summed per kind:
 *   PNCG_PROF_NARROW  first launch of an iteration with self contact
 *                     under the atomic scatter or with
 *                     PNCG_SPLIT_OBJECTS (update + pair gradient/diagonal)
 *   PNCG_PROF_GRAD    element gradient/diag sweep + dot products (with the
 *                     segmented scatter and one step size, also the update
 *                     and the pair pass, which run inside it)
 *   PNCG_PROF_DIR     direction + p^T H p sweep
 *   PNCG_PROF_REBUILD candidate-list rebuild (hash build + pair queries,
 *                     including its host synchronisation)
 *   PNCG_PROF_PREDICT predictor and end-of-step launches
 * pncg_set_profiling(ctx, on) resets the totals; pncg_get_profile fills
 * total_us[PNCG_PROF_KINDS] (microseconds) and launches[PNCG_PROF_KINDS].
 * Event recording adds a little time to each launch, so timed runs that
 * report throughput keep profiling off. */
#define PNCG_PROF_NARROW  0
#define PNCG_PROF_GRAD    1
#define PNCG_PROF_DIR     2
#define PNCG_PROF_REBUILD 3
#define PNCG_PROF_PREDICT 4
#define PNCG_PROF_KINDS   5
int pncg_set_profiling(pncg_ctx* ctx, int32_t on);
int pncg_get_profile(pncg_ctx* ctx, double* total_us, int64_t* launches);

/* ------------------------------------------------------------------------
 * Adjoint of one time step (implicit differentiation; the paper notes only
 * that the IPC formulation is differentiable, Sec. 1).  x1 = x^{t+1} must be
 * a converged step result (gradient of equation E zero to the accuracy
 * wanted, e.g. PNCG_TERM_GRAD_REL with eps 1e-10), since the adjoint uses
 * the optimality condition G(x^{t+1}) = 0.  For a loss L with adjoints
 * xbar = dL/dx^{t+1}, vbar = dL/dv^{t+1} ([nV][3]):
 *     H lambda = xbar + vbar / h   (H = Hessian of equation E at x1:
 *              inertia, the exact Hessian of the context's elastic density
 *              (Sec. 3.1), plane barrier kappa b''(d) n n^T, and for
 *              point-triangle / edge-edge pairs the solver's pair Hessian
 *              model: the PSD projection of equation eq9 unless
 *              PNCG_BARRIER_FULL, with frozen closest-point coefficients
 *              either way; prescribed rows removed)
 * With active point-triangle or edge-edge pairs that model is not the
 * exact Hessian of equation E, so the result is the adjoint of the
 * model, not the exact derivative; with planes only it is exact.
 *     xbar_t = M lambda - vbar / h          (= dL/dx^t)   [nV][3]
 *     vbar_t = h M lambda                   (= dL/dv^t)   [nV][3]
 *     Ebar[e] -= lambda . dG/dE_e           (dL/dE_e, ACCUMULATED) [nT]
 * solved by Jacobi-preconditioned linear CG on the device until
 * |r| <= cg_tol |b| or cg_max iterations (then PNCG_W_MAXITER).  Needs a
 * PNCG_FP64 context (E_STATE otherwise); the material, contact and
 * prescribed vertices are the context's current ones.  Outputs may alias
 * inputs.  E_INDEFINITE if CG meets p^T H p <= 0. */
typedef struct {
  int32_t cg_iters;       /* CG iterations (updates of lambda) */
  int32_t reason;         /* 0 residual rule, 1 cap, 2 p^T H p <= 0 */
  double  rel_residual;   /* |r| / |b| at the end */
} pncg_adjoint_stats;

/* host pointers */
int pncg_adjoint_step(pncg_ctx* ctx, const double* x1, double h,
                      const double* xbar, const double* vbar, double cg_tol,
                      int32_t cg_max, double* xbar_t, double* vbar_t,
                      double* Ebar, pncg_adjoint_stats* st);
/* device pointers on the context's device */
int pncg_adjoint_step_dev(pncg_ctx* ctx, const double* x1_dev, double h,
                          const double* xbar_dev, const double* vbar_dev,
                          double cg_tol, int32_t cg_max, double* xbar_t_dev,
                          double* vbar_t_dev, double* Ebar_dev,
                          pncg_adjoint_stats* st);

/* ------------------------------------------------------------------------
 * Batched form: many small independent scenes stepped together on one
 * device.  Each scene is one workgroup that runs a whole time step of
 * Algorithm 1 (predictor, every PNCG iteration with its own beta, alpha and
 * stop test, end of step) without returning to the host; the workgroups of a
 * persistent grid take scenes largest first.  A scene has elasticity,
 * inertia, gravity and at most one contact plane (barrier against a
 * half-space, Sec. 3 equation barrier with d the signed plane distance);
 * there are no point-triangle or edge-edge pairs between or within scenes.
 * The step size bound (Sec. 4.3) is per scene, in the spirit of the
 * per-object step sizes of Sec. 5.2.  All arithmetic is the single-scene
 * path's for a scene with one plane and no self contact.
 * ---------------------------------------------------------------------- */
typedef struct pncg_batch pncg_batch;

/* Create a batch of nScenes scenes from concatenated arrays (host pointers,
 * copied).  Scene s owns vertices [vert_off[s], vert_off[s+1]), tets
 * [tet_off[s], tet_off[s+1]) and surface triangles [tri_off[s],
 * tri_off[s+1]) (surface triangles only mark the vertices that feel the
 * plane).  Offsets have nScenes + 1 entries starting at 0; every scene has
 * at least one vertex and one tet.  X [nV][3] rest positions; tets [nT][4]
 * and tris [nF][3] hold vertex indices LOCAL to their scene, tets
 * positively oriented (E_INVERTED otherwise); E, nu, rho [nT] as in
 * pncg_set_material; planes [nScenes][4] (n0, n1, n2, o) with |n| = 1, or
 * a zero normal for no plane, or planes = NULL for none at all.
 * opts: device, precision and stream as for pncg_create (block and chunk
 * are ignored).  Errors: E_INVAL, E_INVERTED, E_NONFINITE, E_HIP, E_NOMEM;
 * pncg_batch_last_error(NULL) then describes the failure. */
int pncg_batch_create(pncg_batch** out, const pncg_opts* opts, int32_t nScenes,
                      const int32_t* vert_off, const double* X,
                      const int32_t* tet_off, const int32_t* tets,
                      const int32_t* tri_off, const int32_t* tris,
                      const double* E, const double* nu, const double* rho,
                      const double* planes);

/* Free the batch and its device memory.  NULL is accepted. */
void pncg_batch_destroy(pncg_batch* b);

/* Message for the last error of b (never NULL); b == NULL: the last
 * pncg_batch_create failure on this thread. */
const char* pncg_batch_last_error(const pncg_batch* b);

/* Parameters shared by all scenes: dhat > 0, kappa >= 0 (plane barrier),
 * iter_max >= 1, eps >= 0, term PNCG_TERM_*, gravity[3] (NULL keeps the
 * current value), flags PNCG_BARRIER_FULL / PNCG_ALPHA_INF_COMPONENT (the
 * plane Hessian is the same in both barrier modes) or-ed with a PNCG_BETA_*
 * rule.  Defaults: dhat 1e-3,
 * kappa 1e4, 100, 1e-3, DELTA_E, (0, 0, -9.8), 0. */
int pncg_batch_set_params(pncg_batch* b, double dhat, double kappa,
                          int32_t iter_max, double eps, int32_t term,
                          const double* gravity, uint32_t flags);

/* Threads per workgroup of the step kernel: 256, 512 or 1024 (default
 * 512); pncg_batch_autotune picks one by timing. */
int pncg_batch_set_block(pncg_batch* b, int32_t block);

/* Elastic density of every scene (PNCG_MODEL_*, as pncg_set_model); the
 * default is PNCG_MODEL_NH.  Resizes the persistent grid for that model's
 * kernel (LDS staging is switched off if that kernel cannot hold the
 * largest scene) and drops a captured multi-step graph.  E_INVAL for an
 * unknown model. */
int pncg_batch_set_model(pncg_batch* b, int32_t model);

/* lds = 1: the step kernel keeps the positions and search directions of the
 * scene it is solving in LDS (largest scene's vertex count x (24 + 3 x
 * sizeof(real)) bytes per workgroup); lds = 0: in device memory.  The
 * default is 1 when the largest scene fits in one workgroup's LDS;
 * E_INVAL for 1 when it does not.  Results are the same either way. */
int pncg_batch_set_staging(pncg_batch* b, int32_t lds);

/* Largest number of workgroups that one scene may use, in [1, 8]; > 1
 * needs LDS staging (ignored without it).  A scene with more tets than the
 * batch's mean per workgroup is stepped by a team of about (its tets / that
 * mean) workgroups, which split its tet and incidence loops and meet at
 * two barriers per iteration; the other scenes go to single workgroups,
 * longest first to the least loaded.  A team's workgroups must all be
 * resident at once: the step kernel's grid never exceeds the device's
 * resident capacity, and a barrier that still waits after max_polls polls
 * (0: the default, 2^21, a few seconds) ends the launch with E_HIP (results
 * invalid) instead of hanging.  Results depend on the schedule only through
 * the order of the partial sums.  Default max_team: 8 when LDS staging is
 * on, else 1. */
int pncg_batch_set_split(pncg_batch* b, int32_t max_team, int32_t max_polls);

/* Current workgroup size, staging mode, largest team and number of teams
 * of the schedule (each pointer nullable). */
int pncg_batch_get_config(pncg_batch* b, int32_t* block, int32_t* lds,
                          int32_t* max_team, int32_t* teams);

/* One time step of every scene with step size h > 0.  Device pointers on the
 * batch's device: x_dev, v_dev [nV][3] the state, x_out_dev, v_out_dev
 * [nV][3] the result (must not alias the inputs).  Ordered on the batch's
 * stream; the call synchronises it.  E_PENETRATION / E_INVERTED if some
 * scene's state is infeasible. */
int pncg_batch_step(pncg_batch* b, const double* x_dev, const double* v_dev,
                    double h, double* x_out_dev, double* v_out_dev);

/* nsteps >= 1 consecutive steps in place on x_dev, v_dev (device
 * pointers), launched as one HIP graph that the batch captures on first use
 * and replays while (x_dev, v_dev, h, nsteps, block size, parameters) stay
 * the same.  The call synchronises the stream. */
int pncg_batch_run(pncg_batch* b, double* x_dev, double* v_dev, double h,
                   int32_t nsteps);

/* Per-scene statistics of the last step (host arrays [nScenes], each
 * nullable): iterations, stop reason (as pncg_stats.reason), and iterations
 * summed over every step since creation. */
int pncg_batch_stats(pncg_batch* b, int32_t* iters, int32_t* reason,
                     int64_t* iters_total);

/* Time reps steps from (x_dev, v_dev) at each workgroup size in four
 * modes (device memory; LDS staging; LDS staging with large scenes split
 * over up to 2, or up to 8, workgroups) and keep the fastest (its workgroup size written
 * to *block_out if non-NULL; the rest by pncg_batch_get_config).  The state is not modified;
 * iters_total advances by the timed steps. */
int pncg_batch_autotune(pncg_batch* b, const double* x_dev,
                        const double* v_dev, double h, int32_t reps,
                        int32_t* block_out);

#ifdef __cplusplus
}
#endif

#endif /* PNCG_H */

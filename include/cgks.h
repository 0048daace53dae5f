/*
 * cgks.h -- C ABI of the MI355X (gfx950) multigrid compact gas-kinetic
 * scheme library (libcgks.so).
 *
 * The library computes the steady-state hot path of the geometric-multigrid
 * compact gas-kinetic scheme (GMG-CGKS) on unstructured simplex meshes:
 * one 3-level V-cycle made of
 *   - the fine-level third-order CGKS residual: compact HWENO-type
 *     reconstruction from cell averages and cell-averaged slopes (Sec. 3),
 *     the time-dependent BGK interface flux at face Gauss points
 *     (Sec. 2.3, Eqs. integral1, dis1, dis2), the direct evolution of the
 *     cell-averaged slopes (Sec. 2.4) and the discontinuity-feedback (DF)
 *     factor (Sec. 3.3);
 *   - the explicit fine smoothing step (Sec. 5.2, Eq. smo);
 *   - restriction of W and of the residual, the FAS forcing term, and the
 *     DF-limited prolongation (Sec. 5.2, Eq. prolongation);
 *   - on coarse levels, the first-order kinetic (KFVS) residual and the
 *     multi-colour LU-SGS smoother with DF relaxation, swept one colour at a
 *     time (Sec. 4, Alg. 1, Alg. 2, Eqs. gpu-forward-relaxation and
 *     gpu-backward-relaxation).
 *
 * Conventions
 *  - Non-dimensional free stream: rho = 1, p = 1/gamma (sound speed 1),
 *    |u| = Mach, body diameter 1, mu_inf = Mach / Re.
 *  - Conservative state W = (rho, rho u, rho v[, rho w], rho E); nvar = dim+2.
 *  - Public arrays are in the mesh's original cell order ("original order")
 *    and array-of-structures: W is [n_cells][nvar], gradW is
 *    [n_cells][nvar][dim] (d W_q / d x_d), alpha is [n_cells].  The library
 *    permutes internally (coarse levels are stored colour-contiguously).
 *  - The residual R_i is the outward flux summed over the faces of cell i
 *    (area- and time-averaged, not divided by the volume): the paper's
 *    R^n times |Omega_i| (Sec. 2.2, Eq. high-order-flux-res).  The
 *    multigrid "Res" of Sec. 5.2 is -R.
 *  - Indices are 0-based except colours, which are 1..n_colors (Alg. 1).
 *  - All work is ordered on the context's stream.  Calls that return data in
 *    host memory synchronise that stream before returning.
 *  - No result depends on thread scheduling: the library uses no
 *    floating-point atomics; every reduction has a fixed order.
 *
 * Errors: every int-returning call returns CGKS_OK (0) on success, a
 * negative CGKS_E* code on failure, or CGKS_NOTCONV (+1) from cgks_solve
 * when max_cycles was reached.  cgks_last_error() gives a message owned by
 * the context, valid until the next call on that context.
 */
#ifndef CGKS_H
#define CGKS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CGKS_OK 0
#define CGKS_NOTCONV 1
#define CGKS_EINVAL (-1)   /* bad argument or call order */
#define CGKS_EMESH (-2)    /* invalid mesh: non-positive volume, non-manifold face, untagged boundary */
#define CGKS_EDEVICE (-3)  /* HIP runtime error; the message carries the hipError_t text */
#define CGKS_ENONPHYS (-4) /* NaN, rho <= 0 or p <= 0 after a cycle; state rolled back */
#define CGKS_ELIMIT (-5)   /* size beyond the fixed workspace of an entry point that allocates nothing */

#define CGKS_HOST 0        /* pointer arguments are host memory */
#define CGKS_DEVICE 1      /* pointer arguments are device memory of the context's device */

#define CGKS_FP64 0        /* every step in FP64 */
#define CGKS_MIXED 1       /* FP32 coarse-level correction inside FP64 defect correction */

/* Boundary-face tags of the mesh input. */
#define CGKS_TAG_FARFIELD 1   /* Riemann-invariant far field */
#define CGKS_TAG_SLIP 2       /* inviscid slip wall (mirror state) */
#define CGKS_TAG_ISOTHERMAL 3 /* no-slip wall at T = wall_T_ratio * T_inf */
#define CGKS_TAG_ADIABATIC 4  /* no-slip adiabatic wall */

/* Solver parameters.  cgks_default_params() fills the defaults below. */
typedef struct cgks_params {
    int dim;                   /* 2 (triangles) or 3 (tetrahedra, or hybrid elements: cgks_mesh) */
    double gamma;              /* ratio of specific heats, default 1.4 */
    double prandtl;            /* default 0.72, used when reynolds > 0 */
    double mach;               /* free-stream Mach number */
    double aoa_deg;            /* angle of attack in the x-y plane, degrees */
    double reynolds;           /* Reynolds number per unit length; 0 => Euler */
    double wall_T_ratio;       /* isothermal wall temperature / T_inf, default 1 */
    double sutherland_S_ratio; /* Sutherland constant / T_inf, default 0.5 */
    double cfl_exp;            /* explicit CFL of the fine step, default 0.5 */
    double cfl_imp;            /* implicit CFL of the LU-SGS smoother, default 10 (Sec. 6) */
    int n_levels;              /* multigrid levels, default 3 (Sec. 5.2) */
    int n_pre_fine;            /* fine pre-smoothing steps, default 1 (Sec. 5.2) */
    int n_post;                /* post-smoothing steps: only 0 is supported (Sec. 5.2) */
    int n_sweeps;              /* LU-SGS iterations per coarse level, default 6 (Sec. 6.1) */
    int df_relax;              /* 1: DF relaxation of LU-SGS (Sec. 4.3); 0: fully implicit; 2: one fixed
                                  weight relax_beta in place of every cell's DF value; 3: the fixed-factor
                                  relaxation of the remark in Sec. 4.3: relax_beta scales the implicit
                                  time term V/dt_i, the flux Jacobian keeps full weight, and
                                  (1 - relax_beta) (V/dt_i) times the cell's previous LU-SGS increment
                                  (zero after restriction) joins the right-hand side */
    int df_prolong;            /* 1: DF-limited prolongation (Eq. prolongation); 0: plain */
    int precision;             /* CGKS_FP64 or CGKS_MIXED */
    double tau_c1;             /* Euler collision time: tau = c1 dt + c2 |dp|/(pl+pr) dt */
    double tau_c2;             /* default c1 = 0.01, c2 = 1 */
    double weno_gamma_large;   /* linear weight of the large stencil, default 0.95 */
    double weno_eps;           /* nonlinear-weight epsilon, default 1e-14 */
    double lusgs_omega;        /* spectral-radius safety factor r >= |U.n| + c (Sec. 4.2), default 1 */
    double skew_limit;         /* Alg. 3 minimum sin(skewness angle), default 0.2 */
    double slope_relax;        /* theta of the fine slope update grad <- grad + theta (grad_new - grad);
                                  1 = full replacement (Sec. 2.4); same fixed point for any theta in
                                  (0,1].  Default 0.3: with 1 the V-cycle stalls near 3e-4 on a steady
                                  Re 40 cylinder, with 0.3 it converges to round-off */
    double update_limit;       /* kappa of the update safeguard of fine steps, coarse LU-SGS updates and
                                  prolongation corrections: each cell applies the largest fraction 1, 1/2, ..., 2^-10
                                  (else 0) of its update that keeps rho and p positive and at least
                                  (1 - kappa) times their current values; kappa <= 0 applies an update
                                  whole if rho, p stay positive, else not at all.  Default 0.5 */
    int cfl_ramp;              /* implicit-CFL start-up ramp (not in the paper, whose CFL is fixed):
                                  N > 0 makes the LU-SGS CFL of the k-th V-cycle after the state was
                                  last set (cgks_init_freestream, cgks_set_state) cfl_imp * min(1, k/N),
                                  for impulsive hypersonic starts; cycles discarded after a failure
                                  still count.  Default 0: cfl_imp throughout */
    double relax_beta;         /* relaxation weight in [0, 1] used when df_relax = 2 or 3 (1 = fully
                                  implicit; with 2, 0 = explicit steps); default 0.5 */
    int shared_residual;       /* 1: one fine residual evaluation per V-cycle (not in the paper): the
                                  last fine pre-smoothing step's residual and input state are restricted
                                  instead of a new residual at the smoothed state, and the coarse
                                  correction is added to the smoothed state; same fixed points and
                                  20 % less work per cycle, but on the steady Re 40 cylinder it stalls
                                  near 5e-5 where the paper's cycle reaches 1e-10.  Default 0: the
                                  paper's cycle */
    int slip_wall_p1;          /* 1: cells with a face on a slip wall use the alpha-scaled Green-Gauss
                                  p^1 alone (nonlinear weights 0 and 1; not in the paper).  The compact
                                  p^2 of a slip-wall triangle is fitted to two neighbours beside it
                                  along the wall and makes the explicit fine step grow there; with
                                  this and tau_c1 = 0.1 the inviscid slip-wall cylinder converges to
                                  round-off.  Default 0 */
} cgks_params;

/* Mesh input (host memory, copied by cgks_mesh_setup; the caller keeps ownership).
 * Cells are simplices with positive orientation: triangles (dim=2) with
 * counter-clockwise nodes, or tetrahedra (dim=3) with positive volume. */
typedef struct cgks_mesh {
    int dim;
    int n_nodes;
    const double* coords;      /* [n_nodes][dim] */
    int n_cells;
    const int32_t* cell_nodes; /* [n_cells][dim+1]; hybrid: flat, see cell_offsets */
    int n_bfaces;
    const int32_t* bface_nodes;/* [n_bfaces][dim], any node order; hybrid: flat, see bface_offsets */
    const int32_t* bface_tag;  /* [n_bfaces], CGKS_TAG_* */
    /* 3-D hybrid meshes (Sec. 2.2: tetrahedra, pyramids, prisms and
     * hexahedra with 4, 5, 5 and 6 faces), or both NULL for simplices.  Cell
     * i is cell_nodes[cell_offsets[i] .. cell_offsets[i+1]) with 4 nodes (a
     * tetrahedron, any order), 5 (a pyramid: its base quadrilateral in cyclic
     * order, then the apex), 6 (a prism: one triangle, then the other with
     * node 3+k joined to node k) or 8 (a hexahedron: one quadrilateral in
     * cyclic order, then the opposite one with node 4+k joined to node k);
     * boundary face b is bface_nodes[bface_offsets[b] .. bface_offsets[b+1])
     * (3 or 4 nodes, any order).  Every face must be planar (a quadrilateral
     * more than 1e-9 sqrt(area) off the plane of its first three nodes is
     * CGKS_EMESH) and every cell convex.  Triangular faces take the 3-point
     * rule, quadrilaterals the 2 x 2 Gauss rule of their bilinear map with
     * weights from its area element.  Batched solves take simplex meshes
     * only. */
    const int32_t* cell_offsets;  /* [n_cells + 1], cell_offsets[0] = 0 */
    const int32_t* bface_offsets; /* [n_bfaces + 1] */
} cgks_mesh;

typedef struct cgks_ctx cgks_ctx;

/* Fill *p with the defaults listed in cgks_params. */
void cgks_default_params(cgks_params* p);

/* Create a context on the current HIP device.  Returns CGKS_EINVAL for an
 * unsupported dim / n_post, CGKS_EDEVICE if no device is usable. */
int cgks_create(const cgks_params* p, cgks_ctx** out);

/* Free every device and host resource of the context (NULL is ignored). */
void cgks_destroy(cgks_ctx* c);

/* Message of the last failing call on this context (owned by the context). */
const char* cgks_last_error(const cgks_ctx* c);
const char* cgks_strerror(int code);

/* Borrow a HIP stream (a hipStream_t passed as void*); NULL selects the
 * context's own non-blocking stream.  The library never destroys a borrowed
 * stream.  Invalidates captured graphs. */
int cgks_set_stream(cgks_ctx* c, void* stream);

/* Build the mesh hierarchy (Sec. 2.2 geometry, Sec. 3.1 reconstruction
 * operators, Sec. 5.1 coarse geometry, Alg. 1 colouring of every level) and
 * upload it to the device.  parent[l] (may be NULL) maps each cell of level l
 * to its agglomerate on level l+1 for l = 0..n_levels-2; a NULL parent[l] or a
 * NULL parent builds that level with Alg. 3 (cell coarsening).  CGKS_EMESH on
 * an invalid mesh, CGKS_EINVAL on one without cells or nodes.  Host-side
 * set-up; not on the timed path. */
int cgks_mesh_setup(cgks_ctx* c, const cgks_mesh* m, int n_levels, const int32_t* const* parent);

/* Sizes of one level: cells and faces (coarse faces are agglomerate pairs). */
int cgks_level_size(cgks_ctx* c, int level, int* n_cells, int* n_faces);

/* Alg. 1 colours (1..n_colors) of a level in original order.  Host memory. */
int cgks_coloring(cgks_ctx* c, int level, int32_t* color_out, int32_t* n_colors);

/* Alg. 3 agglomeration of a level (independent of the hierarchy in use):
 * agg_out[i] in 0..n_coarse-1, numbered by first appearance.  Host memory. */
int cgks_agglomerate(cgks_ctx* c, int level, int32_t* agg_out, int32_t* n_coarse);

/* Cell volumes and centroids of a level in original order (host memory). */
int cgks_cell_geometry(cgks_ctx* c, int level, double* V, double* C);

/* Free-stream initial state on every level: gradW = 0, alpha = 1. */
int cgks_init_freestream(cgks_ctx* c);

/* Fine-level state in/out.  mem = CGKS_HOST or CGKS_DEVICE.  gradW / alpha may
 * be NULL (meaning 0 / 1 on input, not returned on output).  Device pointers
 * are borrowed for the duration of the call. */
int cgks_set_state(cgks_ctx* c, const double* W, const double* gradW, const double* alpha, int mem);
int cgks_get_state(cgks_ctx* c, double* W, double* gradW, double* alpha, int mem);

/* Coarse-level state (level >= 1): W, W0 (restricted state), F (FAS forcing),
 * alpha (restricted DF).  Any pointer may be NULL.  Host memory. */
int cgks_set_level_state(cgks_ctx* c, int level, const double* W, const double* W0,
                         const double* F, const double* alpha);
int cgks_get_level_state(cgks_ctx* c, int level, double* W, double* W0, double* F, double* alpha);

/* Residual of a level at its current state.
 * level 0: third-order CGKS residual R (n_cells x nvar), the DF-scaled
 *   evolved slopes gradW_new (Sec. 2.4, Sec. 3.3) and the DF alpha_out.
 * level >= 1: R = (outward KFVS flux sum) - F, so -R is the LU-SGS right-hand
 *   side Res(W) + F (Sec. 5.2); gradW_new is ignored; alpha_out = level DF.
 * The state is not modified.  Outputs may be NULL. */
int cgks_residual(cgks_ctx* c, int level, double* R, double* gradW_new, double* alpha_out, int mem);

/* Local time steps of a level (explicit and implicit CFL), original order. */
int cgks_time_steps(cgks_ctx* c, int level, double* dt_exp, double* dt_imp);

/* n smoothing iterations: level 0 explicit CGKS steps (Eq. smo); level >= 1
 * multi-colour LU-SGS iterations with the level's forcing (Alg. 2). */
int cgks_smooth(cgks_ctx* c, int level, int n);

/* Restriction from level to level+1 (W volume-weighted, residual summed, DF
 * minimum) followed by the FAS forcing F = Res* - Res(W0).  From level 0 it
 * first evaluates the fine residual at the current state (its DF becomes the
 * stored one). */
int cgks_restrict(cgks_ctx* c, int level);

/* DF-limited prolongation of the correction of level+1 onto level. */
int cgks_prolong(cgks_ctx* c, int level);

/* One V-cycle (n_pre_fine fine steps, restriction, n_sweeps LU-SGS on each
 * coarse level, prolongation).  *norm_out (may be NULL) receives the
 * free-stream-normalised RMS of R_rho / V at the start of the cycle.
 * CGKS_ENONPHYS if the cycle produced NaN / non-positive density or pressure
 * (the state is rolled back to the start of the cycle). */
int cgks_vcycle(cgks_ctx* c, double* norm_out);

/* V-cycles until norm <= tol or max_cycles.  history (may be NULL) receives
 * up to history_cap norms; cycles_out (may be NULL) the cycles run.  Returns
 * CGKS_OK, CGKS_NOTCONV (also for max_cycles = 0, with no cycle run) or an
 * error (CGKS_EINVAL for max_cycles < 0). */
int cgks_solve(cgks_ctx* c, double tol, int max_cycles, int* cycles_out, double* history,
               int history_cap);

/* Run n V-cycles with no host synchronisation between them (graph replay);
 * the per-cycle norms stay on the device and are returned in history.  n = 0
 * does nothing; n < 0 is CGKS_EINVAL. */
int cgks_run_cycles(cgks_ctx* c, int n, double* history);

/* Average duration in milliseconds of one kernel of the fine residual at the
 * current state: kernel 0 = reconstruction (per cell), 1 = Gauss-point flux
 * (per face Gauss point), 2 = gather (per cell).  Each of the `reps`
 * repetitions runs the whole fine residual on the context's stream, with HIP
 * events around the chosen kernel only, so the kernel sees the cache state of
 * a V-cycle.  The state is not modified.  Also returns the number of work
 * items of one launch (hybrid meshes: four flux lanes per face, a
 * triangle's unused fourth included). */
int cgks_time_kernel(cgks_ctx* c, int kernel, int reps, double* avg_ms, int64_t* work_items);

/* Choose the launch shape (threads per block) of each fine-residual kernel by
 * timing the candidates at the current state, and the cells per block (16,
 * 32 or 64) of each coarse level's slot-parallel kernels by timing three
 * LU-SGS iterations of the level per candidate.  The fine state is not
 * modified; the coarse levels' states are (the next restriction overwrites
 * them); the statistics counters are kept.  Invalidates captured graphs.
 * The per-cell arithmetic does not depend on the shapes; the compiler may
 * pair multiply-adds differently in differently sized kernels, so results
 * agree to rounding, and bit for bit at equal shapes. */
int cgks_autotune(cgks_ctx* c);
/* Current launch shapes of the reconstruction, flux and gather kernels. */
int cgks_launch_shapes(cgks_ctx* c, int* recon, int* flux, int* gather);
/* Cells per block of the slot-parallel kernels of coarse levels 1..n (host
 * int[n]; 0 for a level that runs the per-cell kernels or does not exist). */
int cgks_coarse_shapes(cgks_ctx* c, int* cells_per_block, int n);
/* Set them (host int[n], each 16, 32 or 64, else CGKS_EINVAL with nothing
 * changed; entries beyond the context's coarse levels are ignored);
 * invalidates captured graphs. */
int cgks_set_coarse_shapes(cgks_ctx* c, const int* cells_per_block, int n);

/* Batched solves: n independent problems (each a context with its own mesh,
 * Mach number, Reynolds number, wall temperature and angle of attack; all
 * other parameters equal) advanced together.  The batch owns one disjoint
 * union of the problems' hierarchies in device memory; one captured graph
 * replay advances every problem by one V-cycle; per-problem norms are reduced
 * in a fixed order.  The problems' fine states are copied in at creation and
 * back by cgks_batch_solve / cgks_batch_get_state.  A CFL ramp (cfl_ramp)
 * counts the batch's V-cycles from its creation.  Problems stay owned by the
 * caller and must outlive the batch.  CGKS_EINVAL if shared parameters differ
 * or n < 1. */
typedef struct cgks_batch cgks_batch;
int cgks_batch_create(int n, cgks_ctx* const* probs, cgks_batch** out);
int cgks_batch_autotune(cgks_batch* b);
/* ncyc V-cycles; history (may be NULL) is [n][ncyc]; ncyc = 0 does nothing. */
int cgks_batch_run_cycles(cgks_batch* b, int ncyc, double* history);
/* Cycles until every problem's norm <= tol (or it failed) or max_cycles.
 * cycles_out[p]: first cycle at or below tol (else cycles run); status_out[p]:
 * CGKS_OK, CGKS_NOTCONV or CGKS_ENONPHYS.  Returns the worst status. */
int cgks_batch_solve(cgks_batch* b, double tol, int max_cycles, int* cycles_out, int* status_out);
/* Copy the batch's fine states back into the problems' contexts. */
int cgks_batch_get_state(cgks_batch* b);
void cgks_batch_destroy(cgks_batch* b);

/* Warm-start surrogate.  The paper starts every steady solve from the free
 * stream (Sec. 6); this optional initial state comes instead from a
 * 5 -> 256 -> 256 -> 256 -> 4 multilayer perceptron with SiLU activations,
 * trained by Adam on the mean squared error.  Every matrix product runs on the
 * BF16 matrix cores with FP32 accumulation; master weights, biases and Adam
 * moments are FP32.  Inputs per sample: 5 standardised features (Mach,
 * log10 Re, x, y, wall distance); outputs: 4 standardised targets
 * (log rho/rho_inf, u/U_inf, v/U_inf, log p/p_inf), where U_inf is the free-stream speed
 * (the Mach number in the solver's units).  X, Y are device pointers, row
 * major [n][5] and [n][4] float.  Calls are stream-ordered on the stream set
 * with cgks_mlp_set_stream (NULL = the null stream) and synchronise before
 * returning.  Errors: CGKS_EINVAL (null pointer, n <= 0, lr <= 0),
 * CGKS_EDEVICE (allocation or launch failure). */
typedef struct cgks_mlp cgks_mlp;
/* Create with He-uniform weights drawn from a 64-bit Mersenne twister seeded
 * with `seed`, zero biases and zero Adam moments. */
int cgks_mlp_create(cgks_mlp** out, int seed);
void cgks_mlp_destroy(cgks_mlp* m);
int cgks_mlp_set_stream(cgks_mlp* m, void* stream);
/* Number of parameters; the flat host layout is, per layer, W [out][in]
 * (row major) followed by b [out]. */
int cgks_mlp_num_params(void);
int cgks_mlp_get_weights(cgks_mlp* m, float* flat);
/* Sets the weights and resets the Adam state (step count and moments). */
int cgks_mlp_set_weights(cgks_mlp* m, const float* flat);
/* Y = network(X); n = 0 does nothing.  The loss, gradient and training calls
 * below need n >= 1 (CGKS_EINVAL otherwise). */
int cgks_mlp_forward(cgks_mlp* m, const float* X, float* Y, int n);
/* Loss mean_n sum_k (out - Y)^2 (host float) and, if grads_out is not NULL,
 * its gradient in the flat host layout; the weights are not changed. */
int cgks_mlp_grads(cgks_mlp* m, const float* X, const float* Y, int n, float* grads_out, float* loss);
/* cgks_mlp_forward for callers that cannot allocate device memory (code under
 * stream or graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same outputs, bit for bit, but the
 * hidden activations live in a fixed file-scope device array of the library
 * (17.8 MB per device, held until the process ends) instead of the network's
 * growable workspace, and Y is written directly.  It calls no hipMalloc,
 * hipFree or allocating routine.  X [n][5] and Y [n][4] are device float
 * pointers of the caller; n <= CGKS_MLP_NOALLOC_MAX_ROWS, else CGKS_ELIMIT
 * and nothing runs.  Every call on one device shares that array: calls that
 * overlap on one device (other host threads, other streams) race, and must
 * be serialised by the caller.  Synchronises the network's stream. */
#define CGKS_MLP_NOALLOC_MAX_ROWS 16384
int cgks_mlp_forward_noalloc(cgks_mlp* m, const float* X, float* Y, int n);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * batch; loss (host, may be NULL) is the loss before the step. */
int cgks_mlp_train_step(cgks_mlp* m, const float* X, const float* Y, int n, float lr, float* loss);
/* Fine-level initial state of a 2-D context from the network.  fmean/fstd
 * standardise the features, tmean/tstd de-standardise the targets (host
 * float[5] and float[4]).  Wall distance is taken to the nearest wall-face
 * centre (the features of cgks_mlp_features).  Cells whose features leave the
 * training range set with cgks_mlp_set_range, or whose prediction is
 * non-finite or non-physical, take the free stream; n_fallback (may be NULL)
 * receives their count.  Gradients are zeroed and alpha set to 1, as
 * cgks_set_state does. */
int cgks_init_from_mlp(cgks_ctx* c, cgks_mlp* m, const float* fmean, const float* fstd, const float* tmean,
                       const float* tstd, int* n_fallback);
/* The raw warm-start features of a 2-D context's fine cells, X [n][5] float in
 * original cell order (host or device memory per `mem`): Mach, log10 Re (0
 * for Euler), centroid x and y, and the distance to the nearest wall-face
 * centre (0 without walls).  The same device kernel feeds cgks_init_from_mlp,
 * so the training data and the warm start's inputs share one definition. */
int cgks_mlp_features(cgks_ctx* c, float* X, int mem);
/* Training range of the raw features (host float[5] each, lo <= hi): a warm
 * start gives the free stream to every cell with a feature outside it (a
 * problem whose Mach or Reynolds number lies outside falls back entirely).
 * NULL, NULL clears the range (the default: no range check). */
int cgks_mlp_set_range(cgks_mlp* m, const float* lo, const float* hi);

/* Counters: positivity-guard hits of the reconstruction; prolongation
 * corrections applied only in part or not at all by the update safeguard. */
int cgks_stats(cgks_ctx* c, int64_t* guard_hits, int64_t* prolong_skips);

#ifdef __cplusplus
}
#endif
#endif

/*
 * CPU oracle for the multigrid compact gas-kinetic scheme (GMG-CGKS).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a plain, slow, FP64
 * implementation of what the paper computes, used by the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg to check the HIP library.
 * The product path never links, loads or calls it, and it shares no code
 * with the HIP library (only the seeded mesh arrays are common input).
 *
 * Sign conventions: R_i = sum over faces of the outward, area- and
 * time-averaged flux (Sec. 2.2, Eq. high-order-flux-res times |Omega|);
 * the multigrid "Res" of Sec. 5.2 is -R.
 *
 * Public state layout: W is [n_cells][nvar] (rho, rho*u, rho*v[, rho*w],
 * rho*E), gradW is [n_cells][nvar][dim], alpha is [n_cells]; all in the
 * original cell order of the mesh / level.
 */
#ifndef CGKS_ORACLE_H
#define CGKS_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_params {
    int dim;                   /* 2 or 3 */
    double gamma;
    double prandtl;
    double mach;
    double aoa_deg;
    double reynolds;           /* 0 => Euler */
    double wall_T_ratio;       /* isothermal wall T_w / T_inf */
    double sutherland_S_ratio; /* Sutherland S / T_inf */
    double cfl_exp;
    double cfl_imp;
    int n_levels;
    int n_pre_fine;
    int n_post;
    int n_sweeps;
    int df_relax;
    int df_prolong;
    int precision;             /* ignored: the oracle is FP64 */
    double tau_c1;
    double tau_c2;
    double weno_gamma_large;
    double weno_eps;
    double lusgs_omega;
    double skew_limit;
    double slope_relax;
    double update_limit;
    int cfl_ramp;              /* implicit-CFL start-up ramp length in V-cycles; 0 = none */
    double relax_beta;         /* fixed relaxation weight used when df_relax = 2 or 3 */
    int shared_residual;       /* 1: restrict the last fine step's input state and residual */
    int slip_wall_p1;          /* 1: cells with a slip-wall face use the Green-Gauss p^1 alone
                                  (weights 0 and 1; an option, not the paper's reconstruction) */
} orc_params;

typedef struct orc_mesh {
    int dim;
    int n_nodes;
    const double* coords;      /* [n_nodes][dim] */
    int n_cells;
    const int32_t* cell_nodes; /* [n_cells][dim+1] */
    int n_bfaces;
    const int32_t* bface_nodes;/* [n_bfaces][dim] */
    const int32_t* bface_tag;  /* [n_bfaces] */
    /* 3-D mixed elements (both NULL for simplex meshes): cell i is
     * cell_nodes[cell_offsets[i] .. cell_offsets[i+1]) with 4, 5, 6 or 8 nodes
     * (tetrahedron, pyramid with its base first, prism, hexahedron), boundary
     * face b is bface_nodes[bface_offsets[b] .. bface_offsets[b+1]) */
    const int32_t* cell_offsets;
    const int32_t* bface_offsets;
} orc_mesh;

typedef struct orc_ctx orc_ctx;

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EMESH (-2)
#define ORC_ENONPHYS (-4)
#define ORC_NOTCONV 1

int orc_create(const orc_params* p, orc_ctx** out);
void orc_destroy(orc_ctx* c);
const char* orc_last_error(const orc_ctx* c);
int orc_mesh_setup(orc_ctx* c, const orc_mesh* m, int n_levels, const int32_t* const* parent);
int orc_level_size(orc_ctx* c, int level, int* n_cells, int* n_faces);

int orc_cell_geometry(orc_ctx* c, int level, double* V, double* C);
int orc_face_geometry(orc_ctx* c, int level, int32_t* LR, int32_t* tag, double* n, double* S, double* xc);
/* Gauss points of every fine face, [n_faces][4][dim], their weights
 * [n_faces][4] (summing to 1; unused entries 0) and counts [n_faces]. */
int orc_face_quadrature(orc_ctx* c, int32_t* ngp, double* gp, double* w);

int orc_coloring(orc_ctx* c, int level, int32_t* color_out, int32_t* n_colors);
int orc_coloring_graph(int n, const int32_t* xadj, const int32_t* adj, int32_t* color_out, int32_t* n_colors);
int orc_agglomerate(orc_ctx* c, int level, int32_t* agg_out, int32_t* n_coarse);

int orc_init_freestream(orc_ctx* c);
int orc_set_state(orc_ctx* c, const double* W, const double* gradW, const double* alpha);
int orc_get_state(orc_ctx* c, double* W, double* gradW, double* alpha);
int orc_set_level_state(orc_ctx* c, int level, const double* W, const double* W0, const double* F, const double* alpha);
int orc_get_level_state(orc_ctx* c, int level, double* W, double* W0, double* F, double* alpha);

int orc_residual(orc_ctx* c, int level, double* R, double* gradW_new, double* alpha_out);
/* The fine residual, evolved slopes and DF of the m listed cells only (original order
 * indices), equal to orc_residual's values for those cells; [m][nvar], [m][nvar][dim], [m]. */
int orc_residual_cells(orc_ctx* c, const int* cells, int m, double* R, double* gradW_new, double* alpha_out);
int orc_time_steps(orc_ctx* c, int level, double* dt_exp, double* dt_imp);
int orc_smooth(orc_ctx* c, int level, int n);
int orc_smooth_sequential(orc_ctx* c, int level, int n);
int orc_restrict(orc_ctx* c, int level);
int orc_prolong(orc_ctx* c, int level);
int orc_vcycle(orc_ctx* c, double* norm_out);
int orc_solve(orc_ctx* c, double tol, int max_cycles, int* cycles_out, double* history, int history_cap);
int orc_stats(orc_ctx* c, int64_t* guard_hits, int64_t* prolong_skips);
/* S * F of every fine face ([n_faces][nvar], oracle face order) from the last
 * fine residual; ORC_EINVAL before any. */
int orc_face_fluxes(orc_ctx* c, double* F);
/* OpenMP threads of the loops over faces, cells and same-colour cells (every
 * result is bitwise the same for any count). */
int orc_set_threads(int n);
int orc_get_threads(void);

/* Point-wise pieces, exported so that tests can pin them in isolation. */
int orc_moments(double U, double lam, int range, int nmax, double* out);
int orc_time_coeffs(double dt, double tau, double* q6);
int orc_moment_solve(const orc_params* p, const double* W, const double* b, double* a);
int orc_gks_point(const orc_params* p, const double* Wl, const double* gl, const double* Wr,
                  const double* gr, const double* n, double dt, double* F, double* G, double* alpha);
int orc_kfvs_point(const orc_params* p, const double* Wl, const double* Wr, const double* n, double* F);
int orc_ghost(const orc_params* p, int tag, const double* W, const double* g, const double* n,
              double* Wg, double* gg);
int orc_recon_eval(orc_ctx* c, int cell, const double* x, double* Wx, double* gx,
                   double* p2x, double* p1x, double* w_large);
/* Per component of one fine cell's reconstruction (Sec. 3): the smoothness
 * indicators of p^2 and p^1, the DF-scaled Green-Gauss gradient of p^1
 * ([nvar][dim]) and the nonlinear weight of the large stencil. */
int orc_recon_indicators(orc_ctx* c, int cell, double* beta0, double* beta1, double* g1, double* w_large);

#ifdef __cplusplus
}
#endif
#endif

/*
 * Internal declarations of libcgks (host set-up, device buffers, launchers).
 */
#ifndef CGKS_INTERNAL_H
#define CGKS_INTERNAL_H

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cgks.h"

namespace cgks {

constexpr int MAXV = 5;      /* conservative variables, 3-D */
constexpr int MAXD = 3;

/* ---------------------------------------------------------------- host --- */

struct HFace {
    int L, R, tag;       /* R < 0: boundary face with tag */
    double n[3];         /* unit normal L -> R */
    double S;            /* area (2-D: length) */
    double xc[3];        /* centre */
    int ngp;             /* 2 (edge), 3 (triangle) or 4 (quadrilateral) */
    double gp[4][3];     /* Gauss points */
    double w[4];         /* their weights, summing to 1 */
};

struct HLevel {
    int n = 0;
    std::vector<double> V, C;             /* original order */
    std::vector<HFace> faces;             /* fine: canonical faces; coarse: agglomerate pairs */
    std::vector<std::vector<int>> cf;     /* per cell: face ids in local order */
    std::vector<int> parent;              /* original index on the next coarser level */
    std::vector<std::vector<int>> children;
    std::vector<int> color;               /* 1..ncolor, original order */
    int ncolor = 0;
    std::vector<int> perm, iperm;         /* internal -> original, original -> internal */
    std::vector<int> color_off;           /* internal offsets of each colour, size ncolor+1 */
    int nslot = 0;                        /* max faces per cell */
    /* fine level only */
    std::vector<int> nodes;               /* [n][dim+1]; mixed elements: flat, cell i from noff[i] */
    std::vector<int> noff;                /* mixed elements: [n+1] */
    std::vector<double> h, mean0, op;     /* basis scale, basis means, LS operator (slot layout) */
    std::vector<int> nbasis;              /* per cell: quadratic, linear or constant basis */
};

/* --------------------------------------------------------------- device --- */

/* Fine level, structure of arrays with the cell (or face) index fastest.
 * Device faces are numbered by (owner cell L, slot of the face in L). */
struct FineDev {
    int n, nf, ngp, nslot, nb;
    double *V, *C, *h, *mean0, *op;   /* op: [nb][nslot*(1+dim)][n] */
    int *slot_face;                   /* [nslot][n]: face id * 2 + side (side 1 = cell is R) */
    int *slot_nbr;                    /* [nslot][n]: neighbour or -1 */
    int *slot_tag;                    /* [nslot][n]: boundary tag of the slot's face (0 interior) */
    double *slot_S, *slot_n;          /* [nslot][n] face area, [dim][nslot][n] outward unit normal */
    double *slot_X;                   /* Gauss points (x - x_c) / h: [ngp][dim][n][nslot] for triangles,
                                         [ngp][dim][nslot][n] for tetrahedra */
    int *fL, *fR;
    int *fslot;                       /* per face: slot in L | (slot in R, 7 on a boundary) << 3 */
    double *fn, *fS;                  /* fn [dim][nf] */
    double *W, *grad, *alpha;         /* state */
    double *Wsave, *gsave, *asave;    /* start-of-cycle copy for roll-back */
    double *poly;                     /* [n][40 | 80] per-cell polynomial record (reconstruction -> flux) */
    double *fX;                       /* [nf][ngp][dim] Gauss points of each face */
    double *fw;                       /* mixed elements: [nf][4] Gauss weight x face area (0: unused point) */
    double *fout;                     /* [nf][2 nv + 1] per face: sum wS F, sum wS W(dt), DF product */
    double *R, *gnew, *anew, *dt, *dti;
    double *res;                      /* -R of the restriction evaluation */
    double *Wpre;                     /* input state of a fine step whose residual is restricted */
    unsigned long long* guard;        /* positivity-guard hit counter */
    /* batched solves: problem id per cell / per face and the per-problem table */
    const int *pid, *fpid;
    const double* ptab;
    double* r2;                       /* per-cell (R_rho / V)^2 for per-problem norms */
    const int* pact;                  /* per-problem "still cycling" flags (null: every cell cycles) */
};

struct CoarseDev {
    int n, nslot, ncolor;
    std::vector<int> color_off;       /* host copy */
    double *V, *C;
    int *snbr, *stag;                 /* [nslot][n] (internal neighbour, -1 boundary / empty) */
    double *sS, *sn, *sd;             /* [nslot][n], [dim][nslot][n], [nslot][n] viscous distance */
    double *W, *W0, *F, *Rstar, *alpha, *dW, *rhs, *D, *r, *dte, *dti;
    double *Wb;                       /* second state buffer: LU-SGS iterations alternate W and Wb */
    int *parent;                      /* of the finer level's internal cells: this level's internal index */
    int *child_off, *child;           /* CSR of finer internal indices */
    int maxchild = 0;                 /* most children of any cell */
    int sc = 64;                      /* cells per block of the slot-parallel kernels (16, 32, 64) */
    const int* pid;                   /* batched solves: problem id per cell (else null) */
    const double* ptab;
    const int* pact;                  /* per-problem "still cycling" flags (null: every cell cycles) */
};

/* Per-problem entries of a batched solve (the fields that may differ). */
constexpr int PTAB = 7;               /* mach, reynolds, mu_inf, Tw, u_inf[3] */

struct Workspace {
    double* partial = nullptr;        /* per-block norm partial sums */
    int npartial = 0;
    double* history = nullptr;        /* device norm history */
    int history_cap = 0;
    int* counter = nullptr;           /* device cycle counter */
    int* ncyc = nullptr;              /* V-cycles begun since the state was set (CFL ramp) */
    unsigned long long* skips = nullptr;
    int* status = nullptr;            /* non-physical flag */
    /* batched solves */
    int nprob = 0;
    int* poff = nullptr;              /* fine-cell offsets of the problems, nprob+1 */
    double* ptab = nullptr;           /* per-problem parameter table */
    int* pactive = nullptr;           /* per-problem flags: 1 = cycle, 0 = frozen (converged or failed) */
};

/* Scalar parameters as seen by the kernels. */
struct KParams {
    int dim;
    double gamma, K, prandtl, mach, reynolds, mu_inf, Tinf, S_suth, Tw;
    double cfl_exp, cfl_imp, tau_c1, tau_c2, g_large, g_small, eps, omega, slope_relax, update_limit;
    int df_relax, df_prolong;
    int slip_wall_p1;                 /* slip-wall cells use p^1 alone */
    int cfl_ramp;                     /* 0: fixed implicit CFL */
    double relax_beta;                /* fixed relaxation weight (df_relax = 2) */
    const int* ncyc;                  /* device: V-cycles begun since the state was set */
    double u_inf[3];
};

}  // namespace cgks

struct cgks_ctx {
    cgks_params p;
    cgks::KParams kp;
    int dim = 2, nv = 4;
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;     /* used when the caller sets no stream */
    std::string err;
    bool have_mesh = false;
    bool hybrid = false;                  /* 3-D mixed-element (hybrid) mesh: 6 face slots, 4 Gauss points per face */
    std::vector<double> coords;
    std::vector<cgks::HLevel> hl;
    cgks::FineDev fine{};
    std::vector<cgks::CoarseDev> coarse;   /* index l-1 for level l */
    cgks::Workspace ws;
    std::vector<void*> allocs;
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_tmpl = nullptr;
    int cycles_done = 0;
    /* launch shapes chosen by the autotuner */
    int blk_recon = 64, blk_flux = 256, blk_gather = 256;   /* recon: cells per block */
    std::vector<int> fperm;               /* device face -> host face of level 0 */
};

namespace cgks {
int setup_host(cgks_ctx* c, const cgks_mesh* m, int n_levels, const int32_t* const* parent);
int agglomerate_level(const cgks_ctx* c, int level, std::vector<int>& agg);
int upload(cgks_ctx* c);
void make_kparams(cgks_ctx* c);
void invalidate_graph(cgks_ctx* c);
int build_graph(cgks_ctx* c);
int fail(cgks_ctx* c, int code, const std::string& msg);
int hip_fail(cgks_ctx* c, hipError_t e, const char* what);

/* kernel launchers (kernels.hip) */
void launch_fine_residual(cgks_ctx* c, int mode);
void launch_fine_recon(cgks_ctx* c);
void launch_fine_kernel(cgks_ctx* c, int which, int block = 0);
void launch_coarse_rhs(cgks_ctx* c, int level, int mode);
void launch_lusgs(cgks_ctx* c, int level);
void launch_restrict(cgks_ctx* c, int level, const double* Wfine = nullptr);
void launch_prolong(cgks_ctx* c, int level);
void launch_norm_finalize(cgks_ctx* c);
void launch_save_state(cgks_ctx* c);
void launch_coarse_update(cgks_ctx* c, int level);
/* n LU-SGS iterations on a coarse level (right-hand side, sweeps, update) */
void launch_lusgs_iters(cgks_ctx* c, int level, int n);
/* whether a coarse level runs the slot-parallel kernels (whose block size the autotuner picks) */
bool coarse_slot_parallel(const CoarseDev& L);

/* modes of launch_fine_residual */
enum { FINE_EVAL = 0, FINE_STEP = 1, FINE_STEP_NORM = 2, FINE_RESTRICT = 3 };
/* flag on a step mode: also keep -R in res and the step's input state in Wpre */
enum { FINE_KEEP = 8 };
/* modes of launch_coarse_rhs */
/* Coarse right-hand-side kernel modes: inside an LU-SGS iteration (fused
 * first-colour forward step, fixed-factor term), the FAS forcing, and a plain
 * evaluation of Res + F with no side effect on the increments. */
enum { COARSE_RHS = 0, COARSE_FORCING = 1, COARSE_EVAL = 2 };
}  // namespace cgks

#endif

/* Internal declarations of the CPU oracle (test infrastructure only). */
#ifndef CGKS_ORACLE_INTERNAL_H
#define CGKS_ORACLE_INTERNAL_H
#include "orc.h"
#include <string>
#include <vector>

namespace orc {

/* Boundary tags of the input format. */
enum { TAG_FARFIELD = 1, TAG_SLIP = 2, TAG_ISOTHERMAL = 3, TAG_ADIABATIC = 4 };

/* ---- kinetic pieces (orc_kinetic.cpp) --------------------------------- */
double internal_dof(const orc_params& p);                   /* K of Sec. 2.1 */
void prim(const orc_params& p, const double* W, double* rho, double* U, double* pr);
void euler_flux(const orc_params& p, const double* W, const double* n, double* T);
double viscosity(const orc_params& p, double T);            /* Sutherland */
void gks_point(const orc_params& p, const double* Wl, const double* gl, const double* Wr,
               const double* gr, const double* n, double dt, double* F, double* G, double* alpha);
void kfvs_point(const orc_params& p, const double* Wl, const double* Wr, const double* n, double* F);
void ghost(const orc_params& p, int tag, const double* W, const double* g, const double* n,
           double* Wg, double* gg);
void time_coeffs(double dt, double tau, double* q);
void moment_table(double U, double lam, int range, int nmax, double* out);
void moment_solve(const orc_params& p, const double* W, const double* b, double* a);

/* ---- mesh / levels (orc_mesh.cpp) -------------------------------------- */
struct Face {
    int L, R;        /* R = -1 on the boundary */
    int tag;         /* 0 interior */
    double n[3];     /* unit normal, L -> R (outward from L) */
    double S;        /* area (length in 2-D) */
    double xc[3];    /* face centre */
    int ngp;         /* 2 (edge), 3 (triangle) or 4 (quadrilateral) */
    double gp[4][3];
    double w[4];     /* weights of the Gauss points, summing to 1 */
};

struct Level {
    int n = 0;                       /* cells */
    std::vector<double> V, C;        /* volume, centroid [n][dim] */
    std::vector<Face> faces;
    std::vector<std::vector<int>> cf;/* local face order of each cell */
    std::vector<int> parent;         /* index on the next coarser level */
    std::vector<std::vector<int>> children; /* indices on the next finer level */
    std::vector<int> color;          /* 1..ncolor (coarse levels) */
    int ncolor = 0;
    /* fine level only */
    std::vector<int> nodes;          /* [n][dim+1]; mixed elements: flat, cell i at noff[i] */
    std::vector<int> noff;           /* mixed elements only: [n+1] offsets into nodes */
    std::vector<double> h;           /* basis scale V^(1/dim) */
    /* state */
    std::vector<double> W, W0, F, Rstar, alpha, grad, dW;
    std::vector<double> rhs_last;    /* RHS after the last sweep (for restriction) */
};

/* Per-cell reconstruction operator of the large stencil (Sec. 3.1). */
struct ReconOp {
    int nb = 0;                  /* 0 (constant), dim (linear) or full quadratic */
    std::vector<int> nbr;        /* interior neighbours in local face order */
    std::vector<double> M;       /* nb x (nnbr*(1+dim)) */
    std::vector<double> mean0;   /* cell averages of the basis on the cell itself */
};

}  // namespace orc

struct orc_ctx {
    orc_params p;
    int dim = 2, nvar = 4;
    std::vector<double> face_flux;   /* S * F of every fine face from the last fine residual [nf][nvar] */
    std::vector<double> coords;
    std::vector<orc::Level> lv;
    std::vector<orc::ReconOp> rop;
    std::string err;
    long long guard_hits = 0, prolong_skips = 0;
    long long cycles = 0;          /* V-cycles begun since the state was last set */
    bool have_mesh = false;
    bool mixed = false;            /* 3-D mixed-element input (noff set) */
};

namespace orc {
int setup_mesh(orc_ctx* c, const orc_mesh* m, int n_levels, const int32_t* const* parent);
void build_recon_ops(orc_ctx* c);
int color_graph(int n, const std::vector<std::vector<int>>& nbrs, std::vector<int>& color);
int agglomerate(orc_ctx* c, int level, std::vector<int>& agg);
/* basis helpers shared inside the oracle */
int n_quad_basis(int dim);
void basis_exps(int dim, int k, int* e);
double basis_eval(int dim, int k, const double* x, const double* x0, double h);
double basis_deriv(int dim, int k, const int* l, const double* x, const double* x0, double h);
void cell_quadrature(const orc_ctx* c, int cell, std::vector<double>& pts, std::vector<double>& wts);
struct ElemFaces {
    int nf;          /* faces */
    int nn[6];       /* nodes of each face */
    int v[6][4];     /* local node cycle of each face */
};
const ElemFaces* elem_faces(int nnodes);
void mixed_cell(const orc_ctx* c, int cell, double* V, double* C, std::vector<double>* pts,
                std::vector<double>* wts);
}  // namespace orc

#endif

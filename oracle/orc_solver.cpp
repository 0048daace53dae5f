/*
 * CPU oracle -- reconstruction, residuals, smoothers, transfers, V-cycle
 * (TEST INFRASTRUCTURE ONLY; see orc.h).
 *
 * Everything here is written for clarity, in the order the paper states
 * it, with one plain loop per step.
 */
#include "orc_internal.h"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>

namespace orc {

namespace {

/* Reconstructed data of one fine cell and one conservative component. */
struct CellRec {
    int nb;
    double Q0[5];
    double a[5][9];   /* p^2 coefficients (Sec. 3.1) */
    double g[5][3];   /* p^1 gradient (Sec. 3.2, alpha-scaled) */
    double w0[5], w1[5];
    double b0[5], b1[5]; /* smoothness indicators beta_0 (p^2) and beta_1 (p^1) */
    bool guard;       /* positivity fallback to the constant state */
};

double dotn(const double* a, const double* b, int dim) {
    double s = 0.0;
    for (int d = 0; d < dim; ++d) s += a[d] * b[d];
    return s;
}

/* Outward normal of face fi seen from cell i. */
void outward(const Face& f, int i, int dim, double* n) {
    double sg = (f.L == i) ? 1.0 : -1.0;
    for (int d = 0; d < dim; ++d) n[d] = sg * f.n[d];
}

/* Evaluate p^2, p^1 and the combined polynomial of component q at x (Sec. 3). */
void eval_parts(const orc_ctx* c, int i, const CellRec& r, int q, const double* x, double* P,
                double* gP, double* p2v, double* p1v) {
    const int dim = c->dim;
    const Level& L0 = c->lv[0];
    const ReconOp& op = c->rop[i];
    const double* x0 = &L0.C[i * dim];
    const double h = L0.h[i];
    double p2 = r.Q0[q], g2[3] = {0, 0, 0};
    for (int k = 0; k < r.nb; ++k) {
        p2 += r.a[q][k] * (basis_eval(dim, k, x, x0, h) - op.mean0[k]);
        for (int d = 0; d < dim; ++d) {
            int l[3] = {0, 0, 0};
            l[d] = 1;
            g2[d] += r.a[q][k] * basis_deriv(dim, k, l, x, x0, h);
        }
    }
    double p1 = r.Q0[q];
    for (int d = 0; d < dim; ++d) p1 += r.g[q][d] * (x[d] - x0[d]);
    const double gl = c->p.weno_gamma_large, gs = 1.0 - gl;
    *P = r.w0[q] / gl * (p2 - gs * p1) + r.w1[q] * p1;
    for (int d = 0; d < dim; ++d) gP[d] = r.w0[q] / gl * (g2[d] - gs * r.g[q][d]) + r.w1[q] * r.g[q][d];
    if (p2v) *p2v = p2;
    if (p1v) *p1v = p1;
}

void eval_state(const orc_ctx* c, int i, const CellRec& r, const double* x, double* W, double* gW) {
    const int dim = c->dim, nv = c->nvar;
    for (int q = 0; q < nv; ++q) {
        if (r.guard) {
            W[q] = r.Q0[q];
            for (int d = 0; d < dim; ++d) gW[q * dim + d] = 0.0;
        } else {
            eval_parts(c, i, r, q, x, &W[q], &gW[q * dim], nullptr, nullptr);
        }
    }
}

bool physical(const orc_params& p, const double* W) {
    double rho, U[3], pr;
    prim(p, W, &rho, U, &pr);
    return rho > 0.0 && pr > 0.0;
}

/* Internal energy density rho e = E - |m|^2 / (2 rho) (proportional to p). */
double rho_e(int dim, const double* W) {
    double ke = 0.0;
    for (int d = 0; d < dim; ++d) ke = ke + W[1 + d] * W[1 + d];
    return W[dim + 1] - 0.5 * ke / W[0];
}

/* Fraction theta of an update dW that is applied to W (the paper states no
 * safeguard for coarse updates or corrections).  kappa <= 0: theta = 1 when
 * W + dW has rho > 0 and p > 0, else 0.  kappa > 0: the largest theta of
 * 1, 1/2, ..., 2^-10 for which rho and rho e of W + theta dW are positive and
 * at least (1 - kappa) times those of W; 0 when none is. */
double update_fraction(const orc_params& p, const double* W, const double* dW) {
    const int dim = p.dim, nv = dim + 2;
    double Wn[5];
    if (!(p.update_limit > 0.0)) {
        for (int q = 0; q < nv; ++q) Wn[q] = W[q] + dW[q];
        return (Wn[0] > 0.0 && rho_e(dim, Wn) > 0.0) ? 1.0 : 0.0;
    }
    const double lo_r = (1.0 - p.update_limit) * W[0];
    const double lo_e = (1.0 - p.update_limit) * rho_e(dim, W);
    double th = 1.0;
    for (int m = 0; m <= 10; ++m) {
        for (int q = 0; q < nv; ++q) Wn[q] = W[q] + th * dW[q];
        if (Wn[0] > 0.0 && Wn[0] >= lo_r) {
            const double e = rho_e(dim, Wn);
            if (e > 0.0 && e >= lo_e) return th;
        }
        th = 0.5 * th;
    }
    return 0.0;
}

/* Build the reconstruction of fine cell i from the current state (Sec. 3). */
void build_rec(orc_ctx* c, int i, CellRec& r) {
    const int dim = c->dim, nv = c->nvar;
    const Level& L0 = c->lv[0];
    const ReconOp& op = c->rop[i];
    const int nn = (int)op.nbr.size(), nin = nn * (1 + dim);
    const double V = L0.V[i];
    const double* x0 = &L0.C[i * dim];
    r.nb = op.nb;
    r.guard = false;
    /* Ghost cell averages for the Green-Gauss sub-stencil at boundary faces. */
    std::vector<std::vector<double>> nbrW(L0.cf[i].size(), std::vector<double>(nv));
    for (size_t t = 0; t < L0.cf[i].size(); ++t) {
        const Face& f = L0.faces[L0.cf[i][t]];
        if (f.R >= 0) {
            int j = (f.L == i) ? f.R : f.L;
            for (int q = 0; q < nv; ++q) nbrW[t][q] = L0.W[j * nv + q];
        } else {
            double n[3];
            outward(f, i, dim, n);
            ghost(c->p, f.tag, &L0.W[i * nv], nullptr, n, nbrW[t].data(), nullptr);
        }
    }
    for (int q = 0; q < nv; ++q) {
        r.Q0[q] = L0.W[i * nv + q];
        /* p^2: the precomputed constrained least-squares operator. */
        std::vector<double> in(nin);
        for (int m = 0; m < nn; ++m) {
            int j = op.nbr[m];
            in[m * (1 + dim)] = L0.W[j * nv + q] - L0.W[i * nv + q];
            for (int d = 0; d < dim; ++d) in[m * (1 + dim) + 1 + d] = L0.grad[(j * nv + q) * dim + d];
        }
        for (int k = 0; k < op.nb; ++k) {
            double s = 0.0;
            for (int j = 0; j < nin; ++j) s += op.M[k * nin + j] * in[j];
            r.a[q][k] = s;
        }
        /* p^1: alpha-scaled Green-Gauss gradient. */
        for (int d = 0; d < dim; ++d) r.g[q][d] = 0.0;
        for (size_t t = 0; t < L0.cf[i].size(); ++t) {
            const Face& f = L0.faces[L0.cf[i][t]];
            double n[3];
            outward(f, i, dim, n);
            double avg = (nbrW[t][q] + r.Q0[q]) / (2.0 * V);
            for (int d = 0; d < dim; ++d) r.g[q][d] += avg * f.S * n[d];
        }
        for (int d = 0; d < dim; ++d) r.g[q][d] *= L0.alpha[i];
        /* Smoothness indicators and nonlinear weights. */
        std::vector<double> pts, wts;
        cell_quadrature(c, i, pts, wts);
        double beta0 = 0.0;
        for (int d = 0; d < dim; ++d) {
            int l[3] = {0, 0, 0};
            l[d] = 1;
            double avg = 0.0;
            for (size_t s = 0; s < wts.size(); ++s) {
                double v = 0.0;
                for (int k = 0; k < op.nb; ++k) v += r.a[q][k] * basis_deriv(dim, k, l, &pts[s * dim], x0, L0.h[i]);
                avg += wts[s] * v * v;
            }
            beta0 += std::pow(V, 2.0 / dim) * avg;
        }
        for (int d1 = 0; d1 < dim; ++d1)
            for (int d2 = d1; d2 < dim; ++d2) {
                int l[3] = {0, 0, 0};
                l[d1] += 1;
                l[d2] += 1;
                double v = 0.0;
                for (int k = 0; k < op.nb; ++k) v += r.a[q][k] * basis_deriv(dim, k, l, x0, x0, L0.h[i]);
                beta0 += std::pow(V, 4.0 / dim) * v * v;
            }
        double g2 = 0.0;
        for (int d = 0; d < dim; ++d) g2 += r.g[q][d] * r.g[q][d];
        double beta1 = std::pow(V, 2.0 / dim) * g2;
        r.b0[q] = beta0;
        r.b1[q] = beta1;
        const double gl = c->p.weno_gamma_large, gs = 1.0 - gl, eps = c->p.weno_eps;
        double tz = std::fabs(beta0 - beta1);
        double t0 = tz / (beta0 + eps), t1 = tz / (beta1 + eps);
        double w0 = gl * (1.0 + t0 * t0), w1 = gs * (1.0 + t1 * t1);
        r.w0[q] = w0 / (w0 + w1);
        r.w1[q] = w1 / (w0 + w1);
        if (c->p.slip_wall_p1) {
            /* option (not the paper's): a cell on a slip wall keeps the
             * Green-Gauss sub-stencil alone */
            for (int fi : L0.cf[i])
                if (L0.faces[fi].R < 0 && L0.faces[fi].tag == TAG_SLIP) {
                    r.w0[q] = 0.0;
                    r.w1[q] = 1.0;
                }
        }
    }
    /* Positivity guard at every Gauss point of the cell. */
    for (int fi : L0.cf[i]) {
        const Face& f = L0.faces[fi];
        for (int k = 0; k < f.ngp; ++k) {
            double W[5], gW[15];
            eval_state(c, i, r, f.gp[k], W, gW);
            if (!physical(c->p, W)) r.guard = true;
        }
    }
    if (r.guard) {
#pragma omp atomic
        ++c->guard_hits;
    }
}

/* Implicit CFL of the coarse LU-SGS in the current V-cycle.  The paper fixes
 * it (Sec. 6); with cfl_ramp = N > 0 it rises linearly from cfl_imp / N in the
 * first V-cycle after the state was set to cfl_imp in the N-th, a start-up
 * ramp for impulsive hypersonic starts.  Outside a V-cycle the last cycle's
 * value holds (the first cycle's before any). */
double implicit_cfl(const orc_ctx* c) {
    const orc_params& p = c->p;
    if (p.cfl_ramp <= 0) return p.cfl_imp;
    const double k = (double)std::max(c->cycles, 1LL);
    return p.cfl_imp * std::min(1.0, k / (double)p.cfl_ramp);
}

/* Spectral radius sum and local time steps (convective + viscous). */
void time_steps(orc_ctx* c, int l, const std::vector<double>& W, std::vector<double>& dte,
                std::vector<double>& dti) {
    const int dim = c->dim, nv = c->nvar;
    const Level& L = c->lv[l];
    const orc_params& p = c->p;
    dte.assign(L.n, 0.0);
    dti.assign(L.n, 0.0);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < L.n; ++i) {
        double rho, U[3], pr;
        prim(p, &W[i * nv], &rho, U, &pr);
        double cs = std::sqrt(p.gamma * pr / rho);
        double lam = 0.0, s2 = 0.0;
        for (int fi : L.cf[i]) {
            const Face& f = L.faces[fi];
            lam += f.S * (std::fabs(dotn(U, f.n, dim)) + cs);
            s2 += f.S * f.S;
        }
        if (p.reynolds > 0.0)
            lam += std::max(4.0 / 3.0, p.gamma / p.prandtl) * viscosity(p, pr / rho) / rho * s2 / L.V[i];
        dte[i] = p.cfl_exp * L.V[i] / lam;
        dti[i] = implicit_cfl(c) * L.V[i] / lam;
    }
}

/* One fine face (Secs. 2.3-2.4): the S-scaled, Gauss-weighted flux, the
 * Gauss-weighted conserved variables at t = dt and the product of the Gauss
 * points' DF factors, from the reconstructions of its cells (rr is null on a
 * boundary face, whose right state is the ghost). */
static void face_sums(orc_ctx* c, const Face& f, const CellRec& rl, const CellRec* rr, double dt, double* Fs,
                      double* Gs, double* as) {
    const int nv = c->nvar;
    for (int q = 0; q < nv; ++q) Fs[q] = Gs[q] = 0.0;
    *as = 1.0;
    for (int k = 0; k < f.ngp; ++k) {
        double Wl[5], gl[15], Wr[5], gr[15], F[5], G[5], a;
        eval_state(c, f.L, rl, f.gp[k], Wl, gl);
        if (rr)
            eval_state(c, f.R, *rr, f.gp[k], Wr, gr);
        else
            ghost(c->p, f.tag, Wl, gl, f.n, Wr, gr);
        gks_point(c->p, Wl, gl, Wr, gr, f.n, dt, F, G, &a);
        for (int q = 0; q < nv; ++q) {
            Fs[q] += f.w[k] * F[q];
            Gs[q] += f.w[k] * G[q];
        }
        *as *= a;
    }
    for (int q = 0; q < nv; ++q) Fs[q] *= f.S;
}

/* Cell i's residual, evolved slopes and DF from its faces' sums, taken in the
 * cell's local face order (Fl, Gl, al indexed by position in cf[i]). */
static void gather_cell(const orc_ctx* c, int i, const double* Fl, const double* Gl, const double* al, double* R,
                        double* g, double* a) {
    const int dim = c->dim, nv = c->nvar;
    const Level& L0 = c->lv[0];
    const std::vector<int>& cf = L0.cf[i];
    for (int q = 0; q < nv; ++q) R[q] = 0.0;
    for (int k = 0; k < nv * dim; ++k) g[k] = 0.0;
    *a = 1.0;
    for (size_t t = 0; t < cf.size(); ++t) {
        const Face& f = L0.faces[cf[t]];
        double sg = (f.L == i) ? 1.0 : -1.0;
        for (int q = 0; q < nv; ++q) R[q] += sg * Fl[t * nv + q];
        *a *= al[t];
    }
    for (size_t t = 0; t < cf.size(); ++t) {
        const Face& f = L0.faces[cf[t]];
        double n[3];
        outward(f, i, dim, n);
        for (int q = 0; q < nv; ++q)
            for (int d = 0; d < dim; ++d) g[q * dim + d] += f.S * Gl[t * nv + q] * n[d];
    }
    for (int q = 0; q < nv; ++q)
        for (int d = 0; d < dim; ++d) g[q * dim + d] *= *a / L0.V[i];
}

/* Fine-level residual (Secs. 2.2-2.4, 3): R, new slopes and DF. */
void fine_residual(orc_ctx* c, std::vector<double>& R, std::vector<double>& gnew,
                   std::vector<double>& anew, std::vector<double>& dte) {
    const int dim = c->dim, nv = c->nvar;
    Level& L0 = c->lv[0];
    std::vector<double> dti;
    time_steps(c, 0, L0.W, dte, dti);
    std::vector<CellRec> rec(L0.n);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < L0.n; ++i) build_rec(c, i, rec[i]);
    const int nf = (int)L0.faces.size();
    std::vector<double> Ff((size_t)nf * nv, 0.0), Gf((size_t)nf * nv, 0.0), af(nf, 1.0);
#pragma omp parallel for schedule(static)
    for (int fi = 0; fi < nf; ++fi) {
        const Face& f = L0.faces[fi];
        double dt = dte[f.L];
        if (f.R >= 0) dt = std::min(dt, dte[f.R]);
        face_sums(c, f, rec[f.L], f.R >= 0 ? &rec[f.R] : nullptr, dt, &Ff[(size_t)fi * nv], &Gf[(size_t)fi * nv],
                  &af[fi]);
    }
    c->face_flux = Ff;
    R.assign((size_t)L0.n * nv, 0.0);
    gnew.assign((size_t)L0.n * nv * dim, 0.0);
    anew.assign(L0.n, 1.0);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < L0.n; ++i) {
        const std::vector<int>& cf = L0.cf[i];
        std::vector<double> Fl(cf.size() * nv), Gl(cf.size() * nv), al(cf.size());
        for (size_t t = 0; t < cf.size(); ++t) {
            for (int q = 0; q < nv; ++q) {
                Fl[t * nv + q] = Ff[(size_t)cf[t] * nv + q];
                Gl[t * nv + q] = Gf[(size_t)cf[t] * nv + q];
            }
            al[t] = af[cf[t]];
        }
        gather_cell(c, i, Fl.data(), Gl.data(), al.data(), &R[(size_t)i * nv], &gnew[(size_t)i * nv * dim],
                    &anew[i]);
    }
}

/* The same residual for a sample of cells only: the reconstructions of the
 * cells and of their face neighbours, the sums of the cells' faces and the
 * gather, by the routines above (so the values equal those of
 * fine_residual); for checking large meshes cell by cell. */
static void fine_residual_cells(orc_ctx* c, const int* cells, int m, double* R, double* gnew, double* anew) {
    const int dim = c->dim, nv = c->nvar;
    Level& L0 = c->lv[0];
    std::vector<double> dte, dti;
    time_steps(c, 0, L0.W, dte, dti);
    std::vector<int> need;
    for (int s = 0; s < m; ++s) {
        const int i = cells[s];
        need.push_back(i);
        for (int fi : L0.cf[i]) {
            const Face& f = L0.faces[fi];
            need.push_back(f.L == i ? f.R : f.L);
        }
    }
    std::sort(need.begin(), need.end());
    need.erase(std::unique(need.begin(), need.end()), need.end());
    if (!need.empty() && need.front() < 0) need.erase(need.begin());
    std::vector<CellRec> rec(need.size());
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < need.size(); ++k) build_rec(c, need[k], rec[k]);
    auto find = [&](int j) -> const CellRec& {
        return rec[std::lower_bound(need.begin(), need.end(), j) - need.begin()];
    };
#pragma omp parallel for schedule(static)
    for (int s = 0; s < m; ++s) {
        const int i = cells[s];
        const std::vector<int>& cf = L0.cf[i];
        std::vector<double> Fl(cf.size() * nv), Gl(cf.size() * nv), al(cf.size());
        for (size_t t = 0; t < cf.size(); ++t) {
            const Face& f = L0.faces[cf[t]];
            double dt = dte[f.L];
            if (f.R >= 0) dt = std::min(dt, dte[f.R]);
            face_sums(c, f, find(f.L), f.R >= 0 ? &find(f.R) : nullptr, dt, &Fl[t * nv], &Gl[t * nv], &al[t]);
        }
        gather_cell(c, i, Fl.data(), Gl.data(), al.data(), &R[(size_t)s * nv], &gnew[(size_t)s * nv * dim],
                    &anew[s]);
    }
}

/* First-order kinetic (KFVS) residual Res = -sum S F on a coarse level. */
void coarse_res(orc_ctx* c, int l, const std::vector<double>& W, std::vector<double>& Res) {
    const int dim = c->dim, nv = c->nvar;
    const Level& L = c->lv[l];
    Res.assign((size_t)L.n * nv, 0.0);
    std::vector<double> Ff(L.faces.size() * nv);
#pragma omp parallel for schedule(static)
    for (size_t fi = 0; fi < L.faces.size(); ++fi) {
        const Face& f = L.faces[fi];
        double Wr[5], F[5];
        if (f.R >= 0)
            for (int q = 0; q < nv; ++q) Wr[q] = W[f.R * nv + q];
        else
            ghost(c->p, f.tag, &W[f.L * nv], nullptr, f.n, Wr, nullptr);
        kfvs_point(c->p, &W[f.L * nv], Wr, f.n, F);
        for (int q = 0; q < nv; ++q) Ff[fi * nv + q] = f.S * F[q];
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < L.n; ++i)
        for (int fi : L.cf[i]) {
            const Face& f = L.faces[fi];
            double sg = (f.L == i) ? 1.0 : -1.0;
            for (int q = 0; q < nv; ++q) Res[i * nv + q] -= sg * Ff[fi * nv + q];
        }
    (void)dim;
}

/* Spectral radius r_ij of the flux-splitting approximation (Sec. 4.2). */
double spectral_radius(orc_ctx* c, const Level& L, const Face& f, int i, const std::vector<double>& W) {
    const int dim = c->dim, nv = c->nvar;
    const orc_params& p = c->p;
    double Wm[5];
    double dist;
    if (f.R >= 0) {
        for (int q = 0; q < nv; ++q) Wm[q] = 0.5 * (W[f.L * nv + q] + W[f.R * nv + q]);
        dist = 0.0;
        for (int d = 0; d < dim; ++d) {
            double dx = L.C[f.R * dim + d] - L.C[f.L * dim + d];
            dist += dx * dx;
        }
        dist = std::sqrt(dist);
    } else {
        for (int q = 0; q < nv; ++q) Wm[q] = W[i * nv + q];
        dist = 0.0;
        for (int d = 0; d < dim; ++d) {
            double dx = f.xc[d] - L.C[i * dim + d];
            dist += dx * dx;
        }
        dist = 2.0 * std::sqrt(dist);
    }
    double rho, U[3], pr;
    prim(p, Wm, &rho, U, &pr);
    double r = p.lusgs_omega * (std::fabs(dotn(U, f.n, dim)) + std::sqrt(p.gamma * pr / rho));
    if (p.reynolds > 0.0)
        r += 2.0 * std::max(4.0 / 3.0, p.gamma / p.prandtl) * viscosity(p, pr / rho) / (rho * dist);
    return r;
}

/* One LU-SGS iteration on coarse level l (Sec. 4, Eqs. gpu-forward/backward-relaxation,
 * Alg. 2).  When `sequential`, the same update is done cell by cell in the order
 * (colour, index) with L(i)/U(i) = earlier/later cells (the classical LU-SGS). */
void lusgs_iter(orc_ctx* c, int l, bool sequential) {
    const int dim = c->dim, nv = c->nvar;
    Level& L = c->lv[l];
    const orc_params& p = c->p;
    std::vector<double> Res, dte, dti;
    coarse_res(c, l, L.W, Res);
    std::vector<double> rhs((size_t)L.n * nv);
    for (size_t k = 0; k < rhs.size(); ++k) rhs[k] = Res[k] + L.F[k];
    time_steps(c, l, L.W, dte, dti);
    std::vector<double> rf(L.faces.size());
#pragma omp parallel for schedule(static)
    for (size_t fi = 0; fi < L.faces.size(); ++fi) rf[fi] = spectral_radius(c, L, L.faces[fi], L.faces[fi].L, L.W);
    std::vector<double> D(L.n), al(L.n);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < L.n; ++i) {
        double sr = 0.0;
        for (int fi : L.cf[i]) sr += L.faces[fi].S * rf[fi];
        if (p.df_relax == 3) {
            /* The fixed-factor relaxation the paper contrasts with DF relaxation
             * (remark in Sec. 4.3): beta scales the implicit time term only, the
             * flux Jacobian keeps full weight, and (1 - beta) times the cell's
             * previous increment joins the right-hand side (with V/dt_i: the
             * printed term lacks it and is dimensionally a state, not a flux). */
            al[i] = 1.0;
            D[i] = p.relax_beta * L.V[i] / dti[i] + 0.5 * sr;
            for (int q = 0; q < nv; ++q)
                rhs[i * nv + q] += (1.0 - p.relax_beta) * (L.V[i] / dti[i]) * L.dW[i * nv + q];
            continue;
        }
        /* relaxation weight: DF (Sec. 4.3), one fixed weight, or fully implicit */
        al[i] = p.df_relax == 1 ? L.alpha[i] : (p.df_relax == 2 ? p.relax_beta : 1.0);
        D[i] = al[i] * (L.V[i] / dti[i] + 0.5 * sr) + (1.0 - al[i]) * L.V[i] / dte[i];
    }
    std::vector<int> pos(L.n);
    {
        std::vector<int> order(L.n);
        for (int i = 0; i < L.n; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return L.color[a] < L.color[b]; });
        for (int k = 0; k < L.n; ++k) pos[order[k]] = k;
    }
    auto offdiag = [&](int i, bool lower, double* s) {
        for (int q = 0; q < nv; ++q) s[q] = 0.0;
        for (int fi : L.cf[i]) {
            const Face& f = L.faces[fi];
            if (f.R < 0) continue;
            int j = (f.L == i) ? f.R : f.L;
            bool take = sequential ? (lower ? pos[j] < pos[i] : pos[j] > pos[i])
                                   : (lower ? L.color[j] < L.color[i] : L.color[j] > L.color[i]);
            if (!take) continue;
            double n[3];
            outward(f, i, dim, n);
            double Wp[5], T1[5], T0[5];
            for (int q = 0; q < nv; ++q) Wp[q] = L.W[j * nv + q] + L.dW[j * nv + q];
            euler_flux(p, Wp, n, T1);
            euler_flux(p, &L.W[j * nv], n, T0);
            for (int q = 0; q < nv; ++q) s[q] += f.S * (T1[q] - T0[q] - rf[fi] * L.dW[j * nv + q]);
        }
    };
    std::vector<int> order(L.n);
    for (int i = 0; i < L.n; ++i) order[pos[i]] = i;
    if (sequential) {
        double s[5];
        for (int k = 0; k < L.n; ++k) {
            int i = order[k];
            offdiag(i, true, s);
            for (int q = 0; q < nv; ++q) L.dW[i * nv + q] = (rhs[i * nv + q] - 0.5 * al[i] * s[q]) / D[i];
        }
        for (int k = L.n - 1; k >= 0; --k) {
            int i = order[k];
            offdiag(i, false, s);
            for (int q = 0; q < nv; ++q) L.dW[i * nv + q] -= 0.5 * al[i] * s[q] / D[i];
        }
    } else {
        /* Cells of one colour never share a face, so each colour's loop is
         * order-independent (Sec. 4.1). */
        for (int col = 1; col <= L.ncolor; ++col)
#pragma omp parallel for schedule(static)
            for (int i = 0; i < L.n; ++i) {
                if (L.color[i] != col) continue;
                double s[5];
                offdiag(i, true, s);
                for (int q = 0; q < nv; ++q) L.dW[i * nv + q] = (rhs[i * nv + q] - 0.5 * al[i] * s[q]) / D[i];
            }
        for (int col = L.ncolor; col >= 1; --col)
#pragma omp parallel for schedule(static)
            for (int i = 0; i < L.n; ++i) {
                if (L.color[i] != col) continue;
                double s[5];
                offdiag(i, false, s);
                for (int q = 0; q < nv; ++q) L.dW[i * nv + q] -= 0.5 * al[i] * s[q] / D[i];
            }
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < L.n; ++i) {
        const double th = update_fraction(p, &L.W[i * nv], &L.dW[i * nv]);
        if (th > 0.0)
            for (int q = 0; q < nv; ++q) L.W[i * nv + q] += th * L.dW[i * nv + q];
    }
}

/* New slopes of the fine step: grad <- grad + theta (grad_new - grad).  theta = 1
 * is the direct evolution of Sec. 2.4; any theta in (0,1] has the same fixed point. */
void relax_slopes(orc_ctx* c, const std::vector<double>& gnew) {
    std::vector<double>& g = c->lv[0].grad;
    const double th = c->p.slope_relax;
    for (size_t k = 0; k < g.size(); ++k) g[k] = g[k] + th * (gnew[k] - g[k]);
}

double density_norm(orc_ctx* c, const std::vector<double>& R) {
    const Level& L0 = c->lv[0];
    const int nv = c->nvar;
    double s = 0.0;
    for (int i = 0; i < L0.n; ++i) {
        double v = R[i * nv] / L0.V[i];
        s += v * v;
    }
    return std::sqrt(s / L0.n) / c->p.mach;
}

/* Explicit fine step of Eq. smo (local time step, Res = -R), applied through
 * update_fraction (a cell takes a fraction theta of its step).  norm_out, when
 * given, receives the density-residual norm of the state before the step;
 * W_in and res_out, when given, receive that state and its Res = -R.
 * Returns ORC_ENONPHYS when a step is not finite or a new state has rho <= 0 or
 * p <= 0 (the state is still updated). */
int fine_step(orc_ctx* c, double* norm_out = nullptr, std::vector<double>* W_in = nullptr,
              std::vector<double>* res_out = nullptr) {
    Level& L0 = c->lv[0];
    const int nv = c->nvar, dim = c->dim;
    std::vector<double> R, g, a, dte;
    fine_residual(c, R, g, a, dte);
    if (norm_out) *norm_out = density_norm(c, R);
    if (W_in) *W_in = L0.W;
    if (res_out) {
        res_out->resize(R.size());
        for (size_t k = 0; k < R.size(); ++k) (*res_out)[k] = -R[k];
    }
    bool ok = true;
#pragma omp parallel for schedule(static) reduction(&& : ok)
    for (int i = 0; i < L0.n; ++i) {
        double dW[5];
        for (int q = 0; q < nv; ++q) {
            dW[q] = -(dte[i] / L0.V[i] * R[i * nv + q]);
            ok = ok && std::isfinite(dW[q]);
        }
        double* W = &L0.W[i * nv];
        const double th = update_fraction(c->p, W, dW);
        if (th > 0.0)
            for (int q = 0; q < nv; ++q) W[q] += th * dW[q];
        ok = ok && W[0] > 0.0 && rho_e(dim, W) > 0.0 && std::isfinite(W[nv - 1]);
    }
    relax_slopes(c, g);
    L0.alpha = a;
    return ok ? ORC_OK : ORC_ENONPHYS;
}


/* Restriction from level l to l+1 (Sec. 5.2): volume-weighted W, summed
 * residual, minimum DF; then the forcing F = Res* - Res(W0). */
void restrict_level(orc_ctx* c, int l, const std::vector<double>& res_fine,
                    const std::vector<double>* W_fine = nullptr) {
    const int nv = c->nvar;
    Level& F = c->lv[l];
    Level& G = c->lv[l + 1];
    const std::vector<double>& Wf = W_fine ? *W_fine : F.W;
#pragma omp parallel for schedule(static)
    for (int I = 0; I < G.n; ++I) {
        double w[5] = {0, 0, 0, 0, 0}, r[5] = {0, 0, 0, 0, 0}, amin = 1e300;
        for (int i : G.children[I]) {
            for (int q = 0; q < nv; ++q) {
                w[q] += F.V[i] * Wf[i * nv + q];
                r[q] += res_fine[i * nv + q];
            }
            amin = std::min(amin, F.alpha[i]);
        }
        for (int q = 0; q < nv; ++q) {
            G.W0[I * nv + q] = w[q] / G.V[I];
            G.W[I * nv + q] = G.W0[I * nv + q];
            G.Rstar[I * nv + q] = r[q];
            G.dW[I * nv + q] = 0.0;   /* no previous LU-SGS increment in this cycle */
        }
        G.alpha[I] = amin;
    }
    std::vector<double> Res;
    coarse_res(c, l + 1, G.W0, Res);
    for (size_t k = 0; k < Res.size(); ++k) G.F[k] = G.Rstar[k] - Res[k];
}

/* Prolongation (Eq. prolongation): the DF-weighted injected coarse correction,
 * applied through update_fraction; cells with theta < 1 are counted. */
void prolong_level(orc_ctx* c, int l) {
    const int nv = c->nvar;
    Level& F = c->lv[l];
    const Level& G = c->lv[l + 1];
    long long skips = 0;
#pragma omp parallel for schedule(static) reduction(+ : skips)
    for (int i = 0; i < F.n; ++i) {
        int I = F.parent[i];
        double a = c->p.df_prolong ? F.alpha[i] : 1.0;
        double dW[5];
        for (int q = 0; q < nv; ++q) dW[q] = a * (G.W[I * nv + q] - G.W0[I * nv + q]);
        const double th = update_fraction(c->p, &F.W[i * nv], dW);
        if (th > 0.0)
            for (int q = 0; q < nv; ++q) F.W[i * nv + q] += th * dW[q];
        if (th < 1.0) ++skips;
    }
    c->prolong_skips += skips;
}

void freestream(const orc_params& p, double* W) {
    double a = p.aoa_deg * M_PI / 180.0;
    double u[3] = {p.mach * std::cos(a), p.mach * std::sin(a), 0.0};
    double rho = 1.0, pr = 1.0 / p.gamma, ke = 0.0;
    W[0] = rho;
    for (int d = 0; d < p.dim; ++d) {
        W[1 + d] = rho * u[d];
        ke += u[d] * u[d];
    }
    W[p.dim + 1] = pr / (p.gamma - 1.0) + 0.5 * rho * ke;
}

int check(orc_ctx* c, int level) {
    if (!c || !c->have_mesh) return ORC_EINVAL;
    if (level < 0 || level >= (int)c->lv.size()) return ORC_EINVAL;
    return ORC_OK;
}

}  // namespace

}  // namespace orc

using namespace orc;

extern "C" {

int orc_create(const orc_params* p, orc_ctx** out) {
    if (!p || !out || (p->dim != 2 && p->dim != 3)) return ORC_EINVAL;
    orc_ctx* c = new orc_ctx();
    c->p = *p;
    c->dim = p->dim;
    c->nvar = p->dim + 2;
    *out = c;
    return ORC_OK;
}

void orc_destroy(orc_ctx* c) { delete c; }

const char* orc_last_error(const orc_ctx* c) { return c ? c->err.c_str() : ""; }

int orc_mesh_setup(orc_ctx* c, const orc_mesh* m, int n_levels, const int32_t* const* parent) {
    if (!c || !m) return ORC_EINVAL;
    return setup_mesh(c, m, n_levels, parent);
}

int orc_level_size(orc_ctx* c, int level, int* n_cells, int* n_faces) {
    int rc = check(c, level);
    if (rc) return rc;
    *n_cells = c->lv[level].n;
    *n_faces = (int)c->lv[level].faces.size();
    return ORC_OK;
}

int orc_cell_geometry(orc_ctx* c, int level, double* V, double* C) {
    int rc = check(c, level);
    if (rc) return rc;
    const Level& L = c->lv[level];
    for (int i = 0; i < L.n; ++i) {
        if (V) V[i] = L.V[i];
        if (C)
            for (int d = 0; d < c->dim; ++d) C[i * c->dim + d] = L.C[i * c->dim + d];
    }
    return ORC_OK;
}

int orc_face_geometry(orc_ctx* c, int level, int32_t* LR, int32_t* tag, double* n, double* S, double* xc) {
    int rc = check(c, level);
    if (rc) return rc;
    const Level& L = c->lv[level];
    for (size_t f = 0; f < L.faces.size(); ++f) {
        if (LR) {
            LR[2 * f] = L.faces[f].L;
            LR[2 * f + 1] = L.faces[f].R;
        }
        if (tag) tag[f] = L.faces[f].tag;
        if (S) S[f] = L.faces[f].S;
        for (int d = 0; d < c->dim; ++d) {
            if (n) n[f * c->dim + d] = L.faces[f].n[d];
            if (xc) xc[f * c->dim + d] = L.faces[f].xc[d];
        }
    }
    return ORC_OK;
}

int orc_face_quadrature(orc_ctx* c, int32_t* ngp, double* gp, double* w) {
    int rc = check(c, 0);
    if (rc) return rc;
    const Level& L = c->lv[0];
    for (size_t f = 0; f < L.faces.size(); ++f) {
        ngp[f] = L.faces[f].ngp;
        for (int k = 0; k < 4; ++k) {
            w[f * 4 + k] = k < L.faces[f].ngp ? L.faces[f].w[k] : 0.0;
            for (int d = 0; d < c->dim; ++d)
                gp[(f * 4 + k) * c->dim + d] = k < L.faces[f].ngp ? L.faces[f].gp[k][d] : 0.0;
        }
    }
    return ORC_OK;
}

int orc_coloring(orc_ctx* c, int level, int32_t* color_out, int32_t* n_colors) {
    int rc = check(c, level);
    if (rc) return rc;
    const Level& L = c->lv[level];
    for (int i = 0; i < L.n; ++i) color_out[i] = L.color[i];
    *n_colors = L.ncolor;
    return ORC_OK;
}

int orc_agglomerate(orc_ctx* c, int level, int32_t* agg_out, int32_t* n_coarse) {
    int rc = check(c, level);
    if (rc) return rc;
    std::vector<int> agg;
    *n_coarse = agglomerate(c, level, agg);
    for (size_t i = 0; i < agg.size(); ++i) agg_out[i] = agg[i];
    return ORC_OK;
}

int orc_init_freestream(orc_ctx* c) {
    int rc = check(c, 0);
    if (rc) return rc;
    for (auto& L : c->lv) {
        for (int i = 0; i < L.n; ++i) freestream(c->p, &L.W[i * c->nvar]);
        L.W0 = L.W;
        std::fill(L.alpha.begin(), L.alpha.end(), 1.0);
        std::fill(L.F.begin(), L.F.end(), 0.0);
    }
    std::fill(c->lv[0].grad.begin(), c->lv[0].grad.end(), 0.0);
    c->cycles = 0;
    return ORC_OK;
}

int orc_set_state(orc_ctx* c, const double* W, const double* gradW, const double* alpha) {
    int rc = check(c, 0);
    if (rc) return rc;
    Level& L0 = c->lv[0];
    std::copy(W, W + L0.W.size(), L0.W.begin());
    if (gradW)
        std::copy(gradW, gradW + L0.grad.size(), L0.grad.begin());
    else
        std::fill(L0.grad.begin(), L0.grad.end(), 0.0);
    if (alpha)
        std::copy(alpha, alpha + L0.n, L0.alpha.begin());
    else
        std::fill(L0.alpha.begin(), L0.alpha.end(), 1.0);
    c->cycles = 0;
    return ORC_OK;
}

int orc_get_state(orc_ctx* c, double* W, double* gradW, double* alpha) {
    int rc = check(c, 0);
    if (rc) return rc;
    const Level& L0 = c->lv[0];
    if (W) std::copy(L0.W.begin(), L0.W.end(), W);
    if (gradW) std::copy(L0.grad.begin(), L0.grad.end(), gradW);
    if (alpha) std::copy(L0.alpha.begin(), L0.alpha.end(), alpha);
    return ORC_OK;
}

int orc_set_level_state(orc_ctx* c, int level, const double* W, const double* W0, const double* F,
                        const double* alpha) {
    int rc = check(c, level);
    if (rc) return rc;
    Level& L = c->lv[level];
    if (W) std::copy(W, W + L.W.size(), L.W.begin());
    if (W0) std::copy(W0, W0 + L.W0.size(), L.W0.begin());
    if (F) std::copy(F, F + L.F.size(), L.F.begin());
    if (alpha) std::copy(alpha, alpha + L.n, L.alpha.begin());
    return ORC_OK;
}

int orc_get_level_state(orc_ctx* c, int level, double* W, double* W0, double* F, double* alpha) {
    int rc = check(c, level);
    if (rc) return rc;
    const Level& L = c->lv[level];
    if (W) std::copy(L.W.begin(), L.W.end(), W);
    if (W0) std::copy(L.W0.begin(), L.W0.end(), W0);
    if (F) std::copy(L.F.begin(), L.F.end(), F);
    if (alpha) std::copy(L.alpha.begin(), L.alpha.end(), alpha);
    return ORC_OK;
}

int orc_residual(orc_ctx* c, int level, double* R, double* gradW_new, double* alpha_out) {
    int rc = check(c, level);
    if (rc) return rc;
    if (level == 0) {
        std::vector<double> Rv, g, a, dte;
        fine_residual(c, Rv, g, a, dte);
        if (R) std::copy(Rv.begin(), Rv.end(), R);
        if (gradW_new) std::copy(g.begin(), g.end(), gradW_new);
        if (alpha_out) std::copy(a.begin(), a.end(), alpha_out);
        return ORC_OK;
    }
    Level& L = c->lv[level];
    std::vector<double> Res;
    coarse_res(c, level, L.W, Res);
    if (R)
        for (size_t k = 0; k < Res.size(); ++k) R[k] = -(Res[k] + L.F[k]);
    if (alpha_out) std::copy(L.alpha.begin(), L.alpha.end(), alpha_out);
    return ORC_OK;
}

/* Fine residual, evolved slopes and DF of the m listed cells (original
 * order indices; outputs [m][nvar], [m][nvar][dim], [m]). */
int orc_residual_cells(orc_ctx* c, const int* cells, int m, double* R, double* gradW_new, double* alpha_out) {
    int rc = check(c, 0);
    if (rc) return rc;
    if (m < 0 || (m > 0 && (!cells || !R || !gradW_new || !alpha_out))) return ORC_EINVAL;
    for (int s = 0; s < m; ++s)
        if (cells[s] < 0 || cells[s] >= c->lv[0].n) return ORC_EINVAL;
    fine_residual_cells(c, cells, m, R, gradW_new, alpha_out);
    return ORC_OK;
}

/* S * F of every fine face (oracle face order, [nf][nvar]) from the last fine
 * residual evaluation: the scale of the residual's cancellation. */
int orc_face_fluxes(orc_ctx* c, double* F) {
    int rc = check(c, 0);
    if (rc) return rc;
    if (c->face_flux.empty()) return ORC_EINVAL;
    std::copy(c->face_flux.begin(), c->face_flux.end(), F);
    return ORC_OK;
}

int orc_time_steps(orc_ctx* c, int level, double* dt_exp, double* dt_imp) {
    int rc = check(c, level);
    if (rc) return rc;
    std::vector<double> dte, dti;
    time_steps(c, level, c->lv[level].W, dte, dti);
    if (dt_exp) std::copy(dte.begin(), dte.end(), dt_exp);
    if (dt_imp) std::copy(dti.begin(), dti.end(), dt_imp);
    return ORC_OK;
}

int orc_smooth(orc_ctx* c, int level, int n) {
    int rc = check(c, level);
    if (rc) return rc;
    for (int s = 0; s < n; ++s) {
        if (level == 0)
            fine_step(c);
        else
            lusgs_iter(c, level, false);
    }
    return ORC_OK;
}

int orc_smooth_sequential(orc_ctx* c, int level, int n) {
    int rc = check(c, level);
    if (rc) return rc;
    if (level == 0) return ORC_EINVAL;
    for (int s = 0; s < n; ++s) lusgs_iter(c, level, true);
    return ORC_OK;
}

int orc_restrict(orc_ctx* c, int level) {
    int rc = check(c, level);
    if (rc) return rc;
    if (level + 1 >= (int)c->lv.size()) return ORC_EINVAL;
    const int nv = c->nvar;
    std::vector<double> res;
    if (level == 0) {
        /* Residual at the smoothed state W^{n+1}; its DF becomes the stored one. */
        std::vector<double> R, g, a, dte;
        fine_residual(c, R, g, a, dte);
        c->lv[0].alpha = a;
        res.resize(R.size());
        for (size_t k = 0; k < R.size(); ++k) res[k] = -R[k];
    } else {
        Level& L = c->lv[level];
        std::vector<double> Res;
        coarse_res(c, level, L.W, Res);
        res.resize(Res.size());
        for (size_t k = 0; k < Res.size(); ++k) res[k] = Res[k] + L.F[k];
    }
    (void)nv;
    restrict_level(c, level, res);
    return ORC_OK;
}

int orc_prolong(orc_ctx* c, int level) {
    int rc = check(c, level);
    if (rc) return rc;
    if (level + 1 >= (int)c->lv.size()) return ORC_EINVAL;
    prolong_level(c, level);
    return ORC_OK;
}

int orc_vcycle(orc_ctx* c, double* norm_out) {
    int rc = check(c, 0);
    if (rc) return rc;
    const int nl = (int)c->lv.size();
    ++c->cycles;
    /* Fine pre-smoothing (Eq. smo); the first residual gives the cycle's norm.
     * With shared_residual the last step's input state and residual are the
     * ones restricted (one fine residual per smoothing step, none extra). */
    const bool shared = c->p.shared_residual && nl > 1;
    std::vector<double> Wkeep, reskeep;
    bool ok = true;
    for (int s = 0; s < c->p.n_pre_fine; ++s) {
        const bool keep = shared && s == c->p.n_pre_fine - 1;
        ok = fine_step(c, s == 0 ? norm_out : nullptr, keep ? &Wkeep : nullptr, keep ? &reskeep : nullptr) ==
                 ORC_OK && ok;
    }
    for (int l = 0; l + 1 < nl; ++l) {
        if (l == 0 && shared) {
            restrict_level(c, 0, reskeep, &Wkeep);
        } else {
            int r2 = orc_restrict(c, l);
            if (r2) return r2;
        }
        for (int s = 0; s < c->p.n_sweeps; ++s) lusgs_iter(c, l + 1, false);
    }
    for (int l = nl - 2; l >= 0; --l) prolong_level(c, l);
    for (double v : c->lv[0].W)
        if (!std::isfinite(v)) return ORC_ENONPHYS;
    return ok ? ORC_OK : ORC_ENONPHYS;
}

int orc_solve(orc_ctx* c, double tol, int max_cycles, int* cycles_out, double* history,
              int history_cap) {
    int rc = check(c, 0);
    if (rc) return rc;
    for (int k = 0; k < max_cycles; ++k) {
        double nrm = 0.0;
        int r = orc_vcycle(c, &nrm);
        if (history && k < history_cap) history[k] = nrm;
        if (cycles_out) *cycles_out = k + 1;
        if (r) return r;
        if (!std::isfinite(nrm)) return ORC_ENONPHYS;
        if (nrm <= tol) return ORC_OK;
    }
    return ORC_NOTCONV;
}

/* Threads of the OpenMP loops (results do not depend on it). */
int orc_set_threads(int n) {
    if (n < 1) return ORC_EINVAL;
    omp_set_num_threads(n);
    return ORC_OK;
}

int orc_get_threads(void) { return omp_get_max_threads(); }

int orc_stats(orc_ctx* c, int64_t* guard_hits, int64_t* prolong_skips) {
    if (!c) return ORC_EINVAL;
    if (guard_hits) *guard_hits = c->guard_hits;
    if (prolong_skips) *prolong_skips = c->prolong_skips;
    return ORC_OK;
}

int orc_recon_eval(orc_ctx* c, int cell, const double* x, double* Wx, double* gx, double* p2x,
                   double* p1x, double* w_large) {
    int rc = check(c, 0);
    if (rc) return rc;
    if (cell < 0 || cell >= c->lv[0].n) return ORC_EINVAL;
    CellRec r;
    build_rec(c, cell, r);
    if (Wx && gx) eval_state(c, cell, r, x, Wx, gx);
    for (int q = 0; q < c->nvar; ++q) {
        double P, gP[3], p2, p1;
        eval_parts(c, cell, r, q, x, &P, gP, &p2, &p1);
        if (p2x) p2x[q] = p2;
        if (p1x) p1x[q] = p1;
        if (w_large) w_large[q] = r.w0[q];
    }
    return ORC_OK;
}

int orc_recon_indicators(orc_ctx* c, int cell, double* beta0, double* beta1, double* g1, double* w_large) {
    int rc = check(c, 0);
    if (rc) return rc;
    if (cell < 0 || cell >= c->lv[0].n) return ORC_EINVAL;
    CellRec r;
    build_rec(c, cell, r);
    for (int q = 0; q < c->nvar; ++q) {
        if (beta0) beta0[q] = r.b0[q];
        if (beta1) beta1[q] = r.b1[q];
        if (w_large) w_large[q] = r.w0[q];
        if (g1)
            for (int d = 0; d < c->dim; ++d) g1[q * c->dim + d] = r.g[q][d];
    }
    return ORC_OK;
}

}  // extern "C"

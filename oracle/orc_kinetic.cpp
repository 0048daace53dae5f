/*
 * CPU oracle -- gas-kinetic pieces (TEST INFRASTRUCTURE ONLY; see orc.h).
 *
 * Every velocity-space integral is evaluated the slow, literal way: the
 * integrand is expanded into monomials u^a v^b w^c (xi^2)^e and each
 * monomial's moment is the product of one-dimensional Maxwellian moments
 * (full range, or half range u>0 / u<0 in the face-normal direction).
 * The inverse of the moment map <a psi> = b (Sec. 2.3, Eq. co) is a plain
 * Gaussian elimination on the Gram matrix <psi_i psi_j>, not a closed form.
 */
#include "orc_internal.h"

#include <cmath>
#include <cstring>

namespace orc {

namespace {

const int NM = 12;  // 1-D moment tables u^0..u^11

struct Term {
    double c;
    int e[4];  // powers of u (normal), v, w (tangential), xi^2
};
typedef std::vector<Term> Poly;

Poly mono(double c, int eu, int ev, int ew, int ex) {
    Term t;
    t.c = c;
    t.e[0] = eu; t.e[1] = ev; t.e[2] = ew; t.e[3] = ex;
    return Poly(1, t);
}

Poly add(const Poly& a, const Poly& b) {
    Poly r = a;
    r.insert(r.end(), b.begin(), b.end());
    return r;
}

Poly mul(const Poly& a, const Poly& b) {
    Poly r;
    r.reserve(a.size() * b.size());
    for (const Term& x : a)
        for (const Term& y : b) {
            Term t;
            t.c = x.c * y.c;
            for (int k = 0; k < 4; ++k) t.e[k] = x.e[k] + y.e[k];
            r.push_back(t);
        }
    return r;
}

/* psi_k of Sec. 2.1: (1, u, v, [w,] (u^2+v^2[+w^2]+xi^2)/2). */
Poly psi(int k, int dim) {
    if (k == 0) return mono(1.0, 0, 0, 0, 0);
    if (k <= dim) {
        int e[3] = {0, 0, 0};
        e[k - 1] = 1;
        return mono(1.0, e[0], e[1], e[2], 0);
    }
    Poly r = mono(0.5, 2, 0, 0, 0);
    r = add(r, mono(0.5, 0, 2, 0, 0));
    if (dim == 3) r = add(r, mono(0.5, 0, 0, 2, 0));
    r = add(r, mono(0.5, 0, 0, 0, 1));
    return r;
}

/* s = sum_k s_k psi_k (the form of a_x and A in Sec. 2.3). */
Poly expand(const double* s, int dim) {
    Poly r;
    for (int k = 0; k < dim + 2; ++k) {
        Poly q = psi(k, dim);
        for (Term& t : q) t.c *= s[k];
        r = add(r, q);
    }
    return r;
}

Poly velocity(int j) {
    int e[3] = {0, 0, 0};
    e[j] = 1;
    return mono(1.0, e[0], e[1], e[2], 0);
}

struct Maxw {
    double Mu[NM], Mv[NM], Mw[NM], Mx[3];
};

void make_maxw(const orc_params& p, int dim, const double* U, double lam, int range, Maxw& m) {
    moment_table(U[0], lam, range, NM - 1, m.Mu);
    moment_table(U[1], lam, 0, NM - 1, m.Mv);
    if (dim == 3) {
        moment_table(U[2], lam, 0, NM - 1, m.Mw);
    } else {
        for (int i = 0; i < NM; ++i) m.Mw[i] = (i == 0) ? 1.0 : 0.0;
    }
    double K = internal_dof(p);
    m.Mx[0] = 1.0;
    m.Mx[1] = K / (2.0 * lam);
    m.Mx[2] = K * (K + 2.0) / (4.0 * lam * lam);
}

double mom(const Poly& P, const Maxw& m) {
    double s = 0.0;
    for (const Term& t : P) s += t.c * m.Mu[t.e[0]] * m.Mv[t.e[1]] * m.Mw[t.e[2]] * m.Mx[t.e[3]];
    return s;
}

/* Solve A x = b (n x n, row-major) by Gaussian elimination with partial pivoting. */
void gauss_solve(int n, double* A, double* b) {
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[i * n + k]) > std::fabs(A[piv * n + k])) piv = i;
        if (piv != k) {
            for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[piv * n + j]);
            std::swap(b[k], b[piv]);
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            b[i] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * b[j];
        b[k] = s / A[k * n + k];
    }
}

/* Solve <a psi> = b for the coefficients a of s = a_k psi_k (Eq. co). */
void solve_slope(const orc_params& p, int dim, const Maxw& m, const double* b, double* a) {
    int nv = dim + 2;
    double A[25], x[5];
    for (int i = 0; i < nv; ++i) {
        for (int j = 0; j < nv; ++j) A[i * nv + j] = mom(mul(psi(i, dim), psi(j, dim)), m);
        x[i] = b[i];
    }
    gauss_solve(nv, A, x);
    for (int i = 0; i < nv; ++i) a[i] = x[i];
}

/* Local orthonormal frame: e[0] = n, e[1..dim-1] tangential. */
void frame(const double* n, int dim, double e[3][3]) {
    for (int d = 0; d < 3; ++d) e[0][d] = (d < dim) ? n[d] : 0.0;
    if (dim == 2) {
        e[1][0] = -n[1];
        e[1][1] = n[0];
        e[1][2] = 0.0;
        return;
    }
    int j = 0;
    for (int d = 1; d < 3; ++d)
        if (std::fabs(n[d]) < std::fabs(n[j])) j = d;
    double t[3] = {0.0, 0.0, 0.0};
    t[j] = 1.0;
    for (int d = 0; d < 3; ++d) t[d] -= n[j] * n[d];
    double tn = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    for (int d = 0; d < 3; ++d) e[1][d] = t[d] / tn;
    e[2][0] = n[1] * e[1][2] - n[2] * e[1][1];
    e[2][1] = n[2] * e[1][0] - n[0] * e[1][2];
    e[2][2] = n[0] * e[1][1] - n[1] * e[1][0];
}

void to_local(int dim, double e[3][3], const double* W, double* Wl) {
    int nv = dim + 2;
    Wl[0] = W[0];
    for (int j = 0; j < dim; ++j) {
        double s = 0.0;
        for (int d = 0; d < dim; ++d) s += e[j][d] * W[1 + d];
        Wl[1 + j] = s;
    }
    Wl[nv - 1] = W[nv - 1];
}

void to_cart(int dim, double e[3][3], const double* Wl, double* W) {
    int nv = dim + 2;
    W[0] = Wl[0];
    for (int d = 0; d < dim; ++d) {
        double s = 0.0;
        for (int j = 0; j < dim; ++j) s += e[j][d] * Wl[1 + j];
        W[1 + d] = s;
    }
    W[nv - 1] = Wl[nv - 1];
}

/* g[q*dim+d] = d(W_q)/dx_d  ->  gl[q*dim+j] = derivative along e_j of local component q. */
void grad_to_local(int dim, double e[3][3], const double* g, double* gl) {
    int nv = dim + 2;
    double t[5][3];
    for (int q = 0; q < nv; ++q)
        for (int d = 0; d < dim; ++d) t[q][d] = g[q * dim + d];
    for (int a = 0; a < dim; ++a)
        for (int d = 0; d < dim; ++d) {
            double s = 0.0;
            for (int c = 0; c < dim; ++c) s += e[a][c] * g[(1 + c) * dim + d];
            t[1 + a][d] = s;
        }
    for (int q = 0; q < nv; ++q)
        for (int j = 0; j < dim; ++j) {
            double s = 0.0;
            for (int d = 0; d < dim; ++d) s += e[j][d] * t[q][d];
            gl[q * dim + j] = s;
        }
}

void local_prim(const orc_params& p, int dim, const double* W, double* rho, double* U, double* pr,
                double* lam) {
    *rho = W[0];
    double ke = 0.0;
    for (int j = 0; j < dim; ++j) {
        U[j] = W[1 + j] / W[0];
        ke += W[1 + j] * U[j];
    }
    for (int j = dim; j < 3; ++j) U[j] = 0.0;
    *pr = (p.gamma - 1.0) * (W[dim + 1] - 0.5 * ke);
    *lam = W[0] / (2.0 * (*pr));
}

}  // namespace

double internal_dof(const orc_params& p) {
    /* Energy equipartition: (K + dim)/2 = 1/(gamma - 1).  3-D: K=(5-3g)/(g-1) (Sec. 2.1). */
    return 2.0 / (p.gamma - 1.0) - (double)p.dim;
}

void prim(const orc_params& p, const double* W, double* rho, double* U, double* pr) {
    int dim = p.dim;
    *rho = W[0];
    double ke = 0.0;
    for (int d = 0; d < dim; ++d) {
        U[d] = W[1 + d] / W[0];
        ke += W[1 + d] * U[d];
    }
    *pr = (p.gamma - 1.0) * (W[dim + 1] - 0.5 * ke);
}

void euler_flux(const orc_params& p, const double* W, const double* n, double* T) {
    int dim = p.dim;
    double rho, U[3], pr;
    prim(p, W, &rho, U, &pr);
    double un = 0.0;
    for (int d = 0; d < dim; ++d) un += U[d] * n[d];
    T[0] = W[0] * un;
    for (int d = 0; d < dim; ++d) T[1 + d] = W[1 + d] * un + pr * n[d];
    T[dim + 1] = (W[dim + 1] + pr) * un;
}

double viscosity(const orc_params& p, double T) {
    double Tinf = 1.0 / p.gamma;
    double S = p.sutherland_S_ratio * Tinf;
    double mu_inf = p.mach / p.reynolds;
    return mu_inf * std::pow(T / Tinf, 1.5) * (Tinf + S) / (T + S);
}

void moment_table(double U, double lam, int range, int nmax, double* out) {
    out[0] = 1.0;
    if (nmax >= 1) out[1] = U;
    if (range > 0) {
        out[0] = 0.5 * std::erfc(-std::sqrt(lam) * U);
        if (nmax >= 1) out[1] = U * out[0] + 0.5 * std::exp(-lam * U * U) / std::sqrt(M_PI * lam);
    } else if (range < 0) {
        out[0] = 0.5 * std::erfc(std::sqrt(lam) * U);
        if (nmax >= 1) out[1] = U * out[0] - 0.5 * std::exp(-lam * U * U) / std::sqrt(M_PI * lam);
    }
    for (int k = 2; k <= nmax; ++k) out[k] = U * out[k - 1] + (k - 1) / (2.0 * lam) * out[k - 2];
}

void time_coeffs(double dt, double tau, double* q) {
    /* Exact integrals over [0,dt] of the coefficients of Eqs. dis1 / dis2. */
    double e = std::exp(-dt / tau);
    q[0] = dt - tau * (1.0 - e);                                  /* int C1            */
    q[1] = 2.0 * tau * tau - tau * (dt + 2.0 * tau) * e - tau * dt; /* int C2            */
    q[2] = 0.5 * dt * dt - tau * dt + tau * tau * (1.0 - e);      /* int C3            */
    q[3] = tau * (1.0 - e);                                       /* int e^{-t/tau}    */
    q[4] = 2.0 * tau * tau - tau * (dt + 2.0 * tau) * e;          /* int (t+tau)e^..   */
    q[5] = tau * tau * (1.0 - e);                                 /* int tau e^..      */
}

void moment_solve(const orc_params& p, const double* W, const double* b, double* a) {
    int dim = p.dim;
    double rho, U[3], pr, lam;
    local_prim(p, dim, W, &rho, U, &pr, &lam);
    Maxw m;
    make_maxw(p, dim, U, lam, 0, m);
    solve_slope(p, dim, m, b, a);
}

void gks_point(const orc_params& p, const double* Wl_c, const double* gl_c, const double* Wr_c,
               const double* gr_c, const double* n, double dt, double* F, double* G, double* alpha) {
    const int dim = p.dim, nv = dim + 2;
    double e[3][3];
    frame(n, dim, e);
    double W[2][5], g[2][15];
    to_local(dim, e, Wl_c, W[0]);
    to_local(dim, e, Wr_c, W[1]);
    grad_to_local(dim, e, gl_c, g[0]);
    grad_to_local(dim, e, gr_c, g[1]);

    double rho[3], U[3][3], pr[3], lam[3];  // 0 = l, 1 = r, 2 = c
    for (int s = 0; s < 2; ++s) local_prim(p, dim, W[s], &rho[s], U[s], &pr[s], &lam[s]);

    /* Discontinuity feedback at this point (Sec. 3.3). */
    {
        double cl = std::sqrt(p.gamma * pr[0] / rho[0]);
        double cr = std::sqrt(p.gamma * pr[1] / rho[1]);
        double dp = std::fabs(pr[0] - pr[1]);
        double D = dp / pr[0] + dp / pr[1];
        double mn = U[0][0] / cl - U[1][0] / cr;
        D += mn * mn;
        for (int j = 1; j < dim; ++j) {
            double mt = U[0][j] / cl - U[1][j] / cr;
            D += mt * mt;
        }
        *alpha = 1.0 / (1.0 + D * D);
    }

    Maxw half[2], full[3];
    make_maxw(p, dim, U[0], lam[0], +1, half[0]);
    make_maxw(p, dim, U[1], lam[1], -1, half[1]);
    make_maxw(p, dim, U[0], lam[0], 0, full[0]);
    make_maxw(p, dim, U[1], lam[1], 0, full[1]);

    /* Interface equilibrium from the two half-range moments (Eq. compatibility2). */
    double Wc[5];
    for (int k = 0; k < nv; ++k)
        Wc[k] = rho[0] * mom(psi(k, dim), half[0]) + rho[1] * mom(psi(k, dim), half[1]);
    local_prim(p, dim, Wc, &rho[2], U[2], &pr[2], &lam[2]);
    make_maxw(p, dim, U[2], lam[2], 0, full[2]);

    /* Non-equilibrium slopes a^{l,r} in each frame direction (Eq. co). */
    double a[3][3][5];  // [side][direction][coefficient]
    for (int s = 0; s < 2; ++s)
        for (int j = 0; j < dim; ++j) {
            double b[5];
            for (int k = 0; k < nv; ++k) b[k] = g[s][k * dim + j] / rho[s];
            solve_slope(p, dim, full[s], b, a[s][j]);
        }
    /* Equilibrium slopes: half-range combination of the two sides' slope moments. */
    for (int j = 0; j < dim; ++j) {
        Poly al = expand(a[0][j], dim), ar = expand(a[1][j], dim);
        double b[5];
        for (int k = 0; k < nv; ++k)
            b[k] = (rho[0] * mom(mul(psi(k, dim), al), half[0]) +
                    rho[1] * mom(mul(psi(k, dim), ar), half[1])) / rho[2];
        solve_slope(p, dim, full[2], b, a[2][j]);
    }
    /* a . u as a polynomial, and the time derivative A from <A + a.u> = 0. */
    Poly au[3], Ap[3];
    for (int s = 0; s < 3; ++s) {
        au[s] = Poly();
        for (int j = 0; j < dim; ++j) au[s] = add(au[s], mul(expand(a[s][j], dim), velocity(j)));
        double b[5], A[5];
        for (int k = 0; k < nv; ++k) b[k] = -mom(mul(psi(k, dim), au[s]), full[s]);
        solve_slope(p, dim, full[s], b, A);
        Ap[s] = expand(A, dim);
    }

    /* Collision time. */
    double jump = std::fabs(pr[0] - pr[1]) / (pr[0] + pr[1]);
    double tau;
    if (p.reynolds > 0.0)
        tau = viscosity(p, pr[2] / rho[2]) / pr[2] + p.tau_c2 * jump * dt;
    else
        tau = p.tau_c1 * dt + p.tau_c2 * jump * dt;

    double q[6];
    time_coeffs(dt, tau, q);

    /* Time integral of a moment X of f over [0, dt] (Eqs. integral1, dis1, dis2). */
    auto integrated = [&](const Poly& X) {
        double v = rho[2] * (q[0] * mom(X, full[2]) + q[1] * mom(mul(X, au[2]), full[2]) +
                             q[2] * mom(mul(X, Ap[2]), full[2]));
        for (int s = 0; s < 2; ++s)
            v += rho[s] * (q[3] * mom(X, half[s]) - q[4] * mom(mul(X, au[s]), half[s]) -
                           q[5] * mom(mul(X, Ap[s]), half[s]));
        return v;
    };
    double Fl[5];
    Poly u = velocity(0);
    for (int k = 0; k < nv; ++k) Fl[k] = integrated(mul(u, psi(k, dim))) / dt;
    if (p.reynolds > 0.0) {
        /* Prandtl-number correction of the energy flux with the BGK heat flux. */
        Poly c2 = mono(0.0, 0, 0, 0, 0);
        for (int j = 0; j < dim; ++j) {
            Poly cj = add(velocity(j), mono(-U[2][j], 0, 0, 0, 0));
            c2 = add(c2, mul(cj, cj));
        }
        c2 = add(c2, mono(1.0, 0, 0, 0, 1));
        Poly Q = mul(add(u, mono(-U[2][0], 0, 0, 0, 0)), c2);
        for (Term& t : Q) t.c *= 0.5;
        double qh = integrated(Q) / dt;
        Fl[nv - 1] += (1.0 / p.prandtl - 1.0) * qh;
    }
    to_cart(dim, e, Fl, F);

    /* Conservative variables carried by f at t = dt (Sec. 2.4). */
    double ex = std::exp(-dt / tau);
    double C1 = 1.0 - ex, C2 = (dt + tau) * ex - tau, C3 = dt - tau + tau * ex;
    double Gl[5];
    for (int k = 0; k < nv; ++k) {
        Poly X = psi(k, dim);
        double v = rho[2] * (C1 * mom(X, full[2]) + C2 * mom(mul(X, au[2]), full[2]) +
                             C3 * mom(mul(X, Ap[2]), full[2]));
        for (int s = 0; s < 2; ++s)
            v += rho[s] * (ex * mom(X, half[s]) - (dt + tau) * ex * mom(mul(X, au[s]), half[s]) -
                           tau * ex * mom(mul(X, Ap[s]), half[s]));
        Gl[k] = v;
    }
    to_cart(dim, e, Gl, G);
}

void kfvs_point(const orc_params& p, const double* Wl_c, const double* Wr_c, const double* n,
                double* F) {
    const int dim = p.dim, nv = dim + 2;
    double e[3][3];
    frame(n, dim, e);
    double W[2][5], rho[2], U[2][3], pr[2], lam[2];
    to_local(dim, e, Wl_c, W[0]);
    to_local(dim, e, Wr_c, W[1]);
    Maxw half[2];
    for (int s = 0; s < 2; ++s) {
        local_prim(p, dim, W[s], &rho[s], U[s], &pr[s], &lam[s]);
        make_maxw(p, dim, U[s], lam[s], s == 0 ? +1 : -1, half[s]);
    }
    double Fl[5];
    for (int k = 0; k < nv; ++k) {
        Poly X = mul(velocity(0), psi(k, dim));
        Fl[k] = rho[0] * mom(X, half[0]) + rho[1] * mom(X, half[1]);
    }
    to_cart(dim, e, Fl, F);
}

void ghost(const orc_params& p, int tag, const double* W, const double* g, const double* n,
           double* Wg, double* gg) {
    const int dim = p.dim, nv = dim + 2;
    const double gm = p.gamma;
    double rho, U[3], pr;
    prim(p, W, &rho, U, &pr);
    if (gg)
        for (int i = 0; i < nv * dim; ++i) gg[i] = 0.0;
    if (tag == TAG_FARFIELD) {
        double a = p.aoa_deg * M_PI / 180.0;
        double Ui[3] = {p.mach * std::cos(a), p.mach * std::sin(a), 0.0};
        double rhoi = 1.0, pi = 1.0 / gm;
        double ci = std::sqrt(gm * pi / rhoi), c = std::sqrt(gm * pr / rho);
        double un = 0.0, uni = 0.0;
        for (int d = 0; d < dim; ++d) {
            un += U[d] * n[d];
            uni += Ui[d] * n[d];
        }
        double Rp = un + 2.0 * c / (gm - 1.0), Rm = uni - 2.0 * ci / (gm - 1.0);
        double ub = 0.5 * (Rp + Rm), cb = 0.25 * (gm - 1.0) * (Rp - Rm);
        double rb, Ub[3], pb;
        double gfac = 0.5;          /* ghost derivatives / interior derivatives */
        if (ub <= -cb) {            /* supersonic inflow: free stream */
            gfac = 0.0;
            rb = rhoi; pb = pi;
            for (int d = 0; d < 3; ++d) Ub[d] = Ui[d];
        } else if (ub >= cb) {      /* supersonic outflow: interior */
            gfac = 1.0;
            rb = rho; pb = pr;
            for (int d = 0; d < 3; ++d) Ub[d] = U[d];
        } else {
            /* subsonic: entropy and tangential velocity from the interior where the
             * free stream leaves the domain (u_inf . n > 0), else from the free
             * stream; a fixed choice per face */
            double s, Ut[3];
            if (uni > 0.0) {
                s = pr / std::pow(rho, gm);
                for (int d = 0; d < dim; ++d) Ut[d] = U[d] - un * n[d];
            } else {
                s = pi / std::pow(rhoi, gm);
                for (int d = 0; d < dim; ++d) Ut[d] = Ui[d] - uni * n[d];
            }
            rb = std::pow(cb * cb / (gm * s), 1.0 / (gm - 1.0));
            pb = rb * cb * cb / gm;
            for (int d = 0; d < dim; ++d) Ub[d] = Ut[d] + ub * n[d];
        }
        double ke = 0.0;
        Wg[0] = rb;
        for (int d = 0; d < dim; ++d) {
            Wg[1 + d] = rb * Ub[d];
            ke += Ub[d] * Ub[d];
        }
        Wg[nv - 1] = pb / (gm - 1.0) + 0.5 * rb * ke;
        /* derivatives: those of the side the ghost comes from on supersonic
         * faces (zero for the free stream, the interior's for outflow); half
         * the interior ones on subsonic faces (zero derivatives let a mode grow
         * at the boundary, copied ones leave a neutral direction of steady
         * states) */
        if (gg && g)
            for (int i = 0; i < nv * dim; ++i) gg[i] = gfac * g[i];
        return;
    }
    if (tag == TAG_SLIP) {
        /* Mirror image across the wall plane: reflection Rm = I - 2 n n^T. */
        double Rm[3][3];
        for (int i = 0; i < dim; ++i)
            for (int j = 0; j < dim; ++j) Rm[i][j] = (i == j ? 1.0 : 0.0) - 2.0 * n[i] * n[j];
        Wg[0] = W[0];
        for (int i = 0; i < dim; ++i) {
            double s = 0.0;
            for (int j = 0; j < dim; ++j) s += Rm[i][j] * W[1 + j];
            Wg[1 + i] = s;
        }
        Wg[nv - 1] = W[nv - 1];
        if (g && gg) {
            int sc[2] = {0, nv - 1};
            for (int t = 0; t < 2; ++t) {
                int q = sc[t];
                for (int d = 0; d < dim; ++d) {
                    double s = 0.0;
                    for (int j = 0; j < dim; ++j) s += Rm[d][j] * g[q * dim + j];
                    gg[q * dim + d] = s;
                }
            }
            for (int a = 0; a < dim; ++a)
                for (int d = 0; d < dim; ++d) {
                    double s = 0.0;
                    for (int b = 0; b < dim; ++b)
                        for (int c = 0; c < dim; ++c) s += Rm[a][b] * g[(1 + b) * dim + c] * Rm[c][d];
                    gg[(1 + a) * dim + d] = s;
                }
        }
        return;
    }
    /* No-slip walls: velocity reversed, pressure kept. */
    double rg = rho;
    if (tag == TAG_ISOTHERMAL) {
        double Tw = p.wall_T_ratio / gm;
        double T = pr / rho;
        double Tg = 2.0 * Tw - T;
        if (Tg < 0.5 * Tw) Tg = 0.5 * Tw;
        rg = pr / Tg;
    }
    double ke = 0.0;
    Wg[0] = rg;
    for (int d = 0; d < dim; ++d) {
        Wg[1 + d] = -rg * U[d];
        ke += U[d] * U[d];
    }
    Wg[nv - 1] = pr / (gm - 1.0) + 0.5 * rg * ke;
    if (g && gg)
        for (int i = 0; i < nv * dim; ++i) gg[i] = g[i];
}

}  // namespace orc

/* ---- exported point functions ------------------------------------------ */
extern "C" {

int orc_moments(double U, double lam, int range, int nmax, double* out) {
    if (nmax < 0 || nmax > 11 || !(lam > 0.0)) return ORC_EINVAL;
    orc::moment_table(U, lam, range, nmax, out);
    return ORC_OK;
}

int orc_time_coeffs(double dt, double tau, double* q6) {
    if (!(dt > 0.0) || !(tau > 0.0)) return ORC_EINVAL;
    orc::time_coeffs(dt, tau, q6);
    return ORC_OK;
}

int orc_moment_solve(const orc_params* p, const double* W, const double* b, double* a) {
    orc::moment_solve(*p, W, b, a);
    return ORC_OK;
}

int orc_gks_point(const orc_params* p, const double* Wl, const double* gl, const double* Wr,
                  const double* gr, const double* n, double dt, double* F, double* G,
                  double* alpha) {
    orc::gks_point(*p, Wl, gl, Wr, gr, n, dt, F, G, alpha);
    return ORC_OK;
}

int orc_kfvs_point(const orc_params* p, const double* Wl, const double* Wr, const double* n,
                   double* F) {
    orc::kfvs_point(*p, Wl, Wr, n, F);
    return ORC_OK;
}

int orc_ghost(const orc_params* p, int tag, const double* W, const double* g, const double* n,
              double* Wg, double* gg) {
    orc::ghost(*p, tag, W, g, n, Wg, gg);
    return ORC_OK;
}
}

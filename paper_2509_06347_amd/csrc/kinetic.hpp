/*
 * Device functions of the gas-kinetic flux (Sec. 2.3), the first-order
 * kinetic flux of the coarse levels, boundary ghost states and the Euler
 * flux.  Everything is FP64 and templated on the space dimension D.
 *
 * Velocity-space integrals use the closed-form factorisation of Maxwellian
 * moments: <u^a v^b w^c xi^(2k)> = <u^a><v^b><w^c><xi^(2k)>, with
 * one-dimensional full-range and half-range (u>0 / u<0) recursions.  All
 * monomial exponents are compile-time constants so every moment table stays
 * in registers.
 */
#ifndef CGKS_KINETIC_HPP
#define CGKS_KINETIC_HPP

#include <hip/hip_runtime.h>

#include "cgks_internal.h"

namespace cgks {

template <int D>
struct Mom {
    double u[7];   /* <u^k>, full or half range in the normal direction */
    double v[6];   /* <v^k> tangential, full range */
    double w[6];   /* <w^k> second tangential (3-D) */
    double x[3];   /* <xi^(2k)> internal degrees of freedom */
};

struct Prim {
    double rho, U[3], p, lam;
    double T;    /* p / rho = 1 / (2 lam) */
};

/* h = 1 / (2 lam) */
__host__ __device__ __forceinline__ void full_table(double U, double h, double* M, int n) {
    M[0] = 1.0;
    M[1] = U;
#pragma unroll
    for (int k = 2; k < 7; ++k)
        if (k < n) M[k] = U * M[k - 1] + (k - 1) * h * M[k - 2];
}

/* Half-range u moments: sign > 0 integrates over u > 0, sign < 0 over u < 0. */
__host__ __device__ __forceinline__ void half_table(double U, double lam, double h, int sign, double* M) {
    const double sl = sqrt(lam);
    const double ex = exp(-lam * U * U);
    const double c = 0.5 * ex / sqrt(M_PI * lam);
    if (sign > 0) {
        M[0] = 0.5 * erfc(-sl * U);
        M[1] = U * M[0] + c;
    } else {
        M[0] = 0.5 * erfc(sl * U);
        M[1] = U * M[0] - c;
    }
#pragma unroll
    for (int k = 2; k < 7; ++k) M[k] = U * M[k - 1] + (k - 1) * h * M[k - 2];
}

template <int D>
__host__ __device__ __forceinline__ void make_mom(const KParams& kp, const Prim& P, int range, Mom<D>& M) {
    if (range == 0)
        full_table(P.U[0], P.T, M.u, 7);
    else
        half_table(P.U[0], P.lam, P.T, range, M.u);
    full_table(P.U[1], P.T, M.v, 6);
    if (D == 3) full_table(P.U[2], P.T, M.w, 6);
    M.x[0] = 1.0;
    M.x[1] = kp.K * P.T;
    M.x[2] = kp.K * (kp.K + 2.0) * (P.T * P.T);
}

template <int D, int a, int b, int c, int k>
__host__ __device__ __forceinline__ double mp(const Mom<D>& M) {
    static_assert(a < 7 && b < 6 && c < 6 && k < 3, "moment order");
    if constexpr (D == 3)
        return M.u[a] * M.v[b] * M.w[c] * M.x[k];
    else
        return M.u[a] * M.v[b] * M.x[k];
}

/* <u^a v^b w^c psi_j>, j = 0..D+1 */
template <int D, int a, int b, int c>
__host__ __device__ __forceinline__ void psi_mom(const Mom<D>& M, double* out) {
    out[0] = mp<D, a, b, c, 0>(M);
    out[1] = mp<D, a + 1, b, c, 0>(M);
    out[2] = mp<D, a, b + 1, c, 0>(M);
    if constexpr (D == 3) {
        out[3] = mp<D, a, b, c + 1, 0>(M);
        out[4] = 0.5 * (mp<D, a + 2, b, c, 0>(M) + mp<D, a, b + 2, c, 0>(M) + mp<D, a, b, c + 2, 0>(M) +
                        mp<D, a, b, c, 1>(M));
    } else {
        out[3] = 0.5 * (mp<D, a + 2, b, c, 0>(M) + mp<D, a, b + 2, c, 0>(M) + mp<D, a, b, c, 1>(M));
    }
}

/* <s(psi) u^a v^b w^c xi^(2k)> for s = s_0 + s_1 u + s_2 v [+ s_3 w] + s_E (|u|^2+xi^2)/2,
 * split by the factorisation of the Maxwellian moments into the part of s
 * that varies with u (s_0 + s_1 u + s_E u^2 / 2, times <v^b w^c xi^2k>) and
 * the rest (times <u^a>).  Each factor depends on fewer of (s, a, b, c, k)
 * than the whole, so the many moments a flux needs share them. */
template <int D, int a>
__host__ __device__ __forceinline__ double s_upart(const double* s, const Mom<D>& M) {
    return s[0] * M.u[a] + s[1] * M.u[a + 1] + 0.5 * s[D + 1] * M.u[a + 2];
}

template <int D, int b, int c, int k>
__host__ __device__ __forceinline__ double tang(const Mom<D>& M) {
    if constexpr (D == 3)
        return M.v[b] * M.w[c] * M.x[k];
    else
        return M.v[b] * M.x[k];
}

template <int D, int b, int c, int k>
__host__ __device__ __forceinline__ double s_tpart(const double* s, const Mom<D>& M) {
    static_assert(b + 2 < 6 && c + 2 < 6 && k + 1 < 3, "moment order");
    double r = s[2] * tang<D, b + 1, c, k>(M);
    double e = tang<D, b + 2, c, k>(M) + tang<D, b, c, k + 1>(M);
    if constexpr (D == 3) {
        r += s[3] * tang<D, b, c + 1, k>(M);
        e += tang<D, b, c + 2, k>(M);
    }
    return r + 0.5 * s[D + 1] * e;
}

template <int D, int a, int b, int c, int k>
__host__ __device__ __forceinline__ double smom(const double* s, const Mom<D>& M) {
    static_assert(a + 2 < 7, "moment order");
    return s_upart<D, a>(s, M) * tang<D, b, c, k>(M) + M.u[a] * s_tpart<D, b, c, k>(s, M);
}

/* <s(psi) u^a v^b w^c psi_j> */
template <int D, int a, int b, int c>
__host__ __device__ __forceinline__ void spsi_mom(const double* s, const Mom<D>& M, double* out) {
    out[0] = smom<D, a, b, c, 0>(s, M);
    out[1] = smom<D, a + 1, b, c, 0>(s, M);
    out[2] = smom<D, a, b + 1, c, 0>(s, M);
    if constexpr (D == 3) {
        out[3] = smom<D, a, b, c + 1, 0>(s, M);
        out[4] = 0.5 * (smom<D, a + 2, b, c, 0>(s, M) + smom<D, a, b + 2, c, 0>(s, M) +
                        smom<D, a, b, c + 2, 0>(s, M) + smom<D, a, b, c, 1>(s, M));
    } else {
        out[3] = 0.5 * (smom<D, a + 2, b, c, 0>(s, M) + smom<D, a, b + 2, c, 0>(s, M) + smom<D, a, b, c, 1>(s, M));
    }
}

/* sum_j <s_j(psi) u^a u_j psi> where u_j is the j-th local velocity component. */
template <int D, int a>
__host__ __device__ __forceinline__ void sdot_mom(const double (*s)[D + 2], const Mom<D>& M, double* out) {
    double t[D + 2];
    spsi_mom<D, a + 1, 0, 0>(s[0], M, out);
    spsi_mom<D, a, 1, 0>(s[1], M, t);
#pragma unroll
    for (int q = 0; q < D + 2; ++q) out[q] += t[q];
    if constexpr (D == 3) {
        spsi_mom<D, a, 0, 1>(s[2], M, t);
#pragma unroll
        for (int q = 0; q < D + 2; ++q) out[q] += t[q];
    }
}

/* Closed-form inverse of the moment map: find s with <s psi> = b (Eq. co). */
template <int D>
__host__ __device__ __forceinline__ void moment_inverse(const KParams& kp, const Prim& P, const double* b, double* s) {
    const double N = D + kp.K;
    double u2 = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) u2 += P.U[j] * P.U[j];
    const double B = u2 + N * P.T;
    double RE = 2.0 * b[D + 1] - B * b[0];
    double Rj[D];
    double UR = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        Rj[j] = b[1 + j] - P.U[j] * b[0];
        UR += P.U[j] * Rj[j];
    }
    const double sE = 4.0 * P.lam * P.lam / N * (RE - 2.0 * UR);
    double s0 = b[0] - 0.5 * sE * B;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        s[1 + j] = 2.0 * P.lam * Rj[j] - P.U[j] * sE;
        s0 -= P.U[j] * s[1 + j];
    }
    s[0] = s0;
    s[D + 1] = sE;
}

template <int D>
__host__ __device__ __forceinline__ void primitive(const KParams& kp, const double* W, Prim& P) {
    P.rho = W[0];
    double ke = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        P.U[j] = W[1 + j] / W[0];
        ke += W[1 + j] * P.U[j];
    }
    P.p = (kp.gamma - 1.0) * (W[D + 1] - 0.5 * ke);
    P.lam = W[0] / (2.0 * P.p);
    P.T = P.p / W[0];
}

__host__ __device__ __forceinline__ double sutherland(const KParams& kp, double T) {
    const double r = T / kp.Tinf;
    return kp.mu_inf * r * sqrt(r) * (kp.Tinf + kp.S_suth) / (T + kp.S_suth);
}

/* Orthonormal frame with e[0] = n. */
template <int D>
__host__ __device__ __forceinline__ void local_frame(const double* n, double (*e)[3]) {
    if constexpr (D == 2) {
        e[0][0] = n[0]; e[0][1] = n[1];
        e[1][0] = -n[1]; e[1][1] = n[0];
    } else {
        e[0][0] = n[0]; e[0][1] = n[1]; e[0][2] = n[2];
        /* t1 perpendicular to n and to the coordinate axis most aligned with n */
        const double ax = fabs(n[0]), ay = fabs(n[1]), az = fabs(n[2]);
        double t[3];
        if (ax >= ay && ax >= az) { t[0] = -n[1]; t[1] = n[0]; t[2] = 0.0; }
        else if (ay >= az)        { t[0] = 0.0; t[1] = -n[2]; t[2] = n[1]; }
        else                      { t[0] = n[2]; t[1] = 0.0; t[2] = -n[0]; }
        const double il = 1.0 / sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
        e[1][0] = t[0] * il; e[1][1] = t[1] * il; e[1][2] = t[2] * il;
        e[2][0] = n[1] * e[1][2] - n[2] * e[1][1];
        e[2][1] = n[2] * e[1][0] - n[0] * e[1][2];
        e[2][2] = n[0] * e[1][1] - n[1] * e[1][0];
    }
}

template <int D>
__host__ __device__ __forceinline__ void rot_in(const double (*e)[3], const double* W, double* Wl) {
    Wl[0] = W[0];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double s = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) s += e[j][d] * W[1 + d];
        Wl[1 + j] = s;
    }
    Wl[D + 1] = W[D + 1];
}

template <int D>
__host__ __device__ __forceinline__ void rot_out(const double (*e)[3], const double* Wl, double* W) {
    W[0] = Wl[0];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) s += e[j][d] * Wl[1 + j];
        W[1 + d] = s;
    }
    W[D + 1] = Wl[D + 1];
}

/* g[q][d] Cartesian -> dl[j][q]: derivative along e_j of local component q. */
template <int D>
__host__ __device__ __forceinline__ void rot_grad(const double (*e)[3], const double (*g)[D], double (*dl)[D + 2]) {
    double gm[D][D];  /* Cartesian gradient of local momentum components */
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int d = 0; d < D; ++d) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) s += e[a][c] * g[1 + c][d];
            gm[a][d] = s;
        }
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double s0 = 0.0, sE = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            s0 += e[j][d] * g[0][d];
            sE += e[j][d] * g[D + 1][d];
        }
        dl[j][0] = s0;
        dl[j][D + 1] = sE;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double s = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) s += e[j][d] * gm[a][d];
            dl[j][1 + a] = s;
        }
    }
}

/*
 * Time-dependent BGK flux at one Gauss point (Sec. 2.3).
 * In:  W and Cartesian gradients of the left/right reconstructed states, the
 *      unit normal n (left -> right), the flux time dt.
 * Out: F  time-averaged flux over [0, dt] (Cartesian, not area-scaled),
 *      G  conservative variables carried by f at t = dt (Sec. 2.4); with
 *         STATE false (an inviscid residual whose slopes are not used) its
 *         moments, and those of the time-averaged f that only the heat-flux
 *         correction needs, are skipped and G is zero,
 *      alpha  DF factor of this point (Sec. 3.3).
 */
template <int D, bool STATE = true, bool VISC = true>
__host__ __device__ void gks_flux(const KParams& kp, const double* WLc, const double (*gLc)[D], const double* WRc,
                         const double (*gRc)[D], const double* n, double dt, double* F, double* G,
                         double* alpha) {
    constexpr int NV = D + 2;
    double e[3][3];
    local_frame<D>(n, e);
    double WL[NV], WR[NV];
    rot_in<D>(e, WLc, WL);
    rot_in<D>(e, WRc, WR);
    Prim PL, PR, PC;
    primitive<D>(kp, WL, PL);
    primitive<D>(kp, WR, PR);

    {   /* discontinuity feedback */
        const double icl = 1.0 / sqrt(kp.gamma * PL.p / PL.rho), icr = 1.0 / sqrt(kp.gamma * PR.p / PR.rho);
        const double dp = fabs(PL.p - PR.p);
        double Dv = dp / PL.p + dp / PR.p;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double dm = PL.U[j] * icl - PR.U[j] * icr;
            Dv += dm * dm;
        }
        *alpha = 1.0 / (1.0 + Dv * Dv);
    }

    /* interface equilibrium W^c from the half-range moments (Eq. compatibility2) */
    double Wc[NV];
    {
        Mom<D> hl, hr;
        make_mom<D>(kp, PL, +1, hl);
        make_mom<D>(kp, PR, -1, hr);
        double a[NV], b[NV];
        psi_mom<D, 0, 0, 0>(hl, a);
        psi_mom<D, 0, 0, 0>(hr, b);
#pragma unroll
        for (int q = 0; q < NV; ++q) Wc[q] = PL.rho * a[q] + PR.rho * b[q];
    }
    primitive<D>(kp, Wc, PC);

    /* collision time (numerical part from the pressure jump) */
    const double jump = fabs(PL.p - PR.p) / (PL.p + PR.p);
    double tau;
    if (VISC && kp.reynolds > 0.0)
        tau = sutherland(kp, PC.p / PC.rho) / PC.p + kp.tau_c2 * jump * dt;
    else
        tau = kp.tau_c1 * dt + kp.tau_c2 * jump * dt;
    const double ex = exp(-dt / tau);
    const double om = -expm1(-dt / tau);          /* 1 - e^{-dt/tau} */
    const double q1 = dt - tau * om;
    const double q5 = 2.0 * tau * tau - tau * (dt + 2.0 * tau) * ex;
    const double q2 = q5 - tau * dt;
    const double q3 = 0.5 * dt * dt - tau * dt + tau * tau * om;
    const double q4 = tau * om;
    const double q6 = tau * tau * om;
    const double C1 = om, C2 = (dt + tau) * ex - tau, C3 = dt - tau + tau * ex;

    double Fl[NV], Gl[NV], Wf[NV], dWc[D][NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        Fl[q] = 0.0; Gl[q] = 0.0; Wf[q] = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) dWc[j][q] = 0.0;
    }

    /* free-transport part of both sides (Eq. dis1), with their slopes a^k and A^k */
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const Prim& P = side ? PR : PL;
        double Wl[NV];
        double dl[D][NV];
        if (side == 0) {
            rot_grad<D>(e, gLc, dl);
        } else {
            rot_grad<D>(e, gRc, dl);
        }
        
        Mom<D> full, half;
        make_mom<D>(kp, P, 0, full);
        make_mom<D>(kp, P, side ? -1 : +1, half);
        double s[D][NV], A[NV], t[NV], t2[NV];
        const double ir = 1.0 / P.rho;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double b[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) b[q] = dl[j][q] * ir;
            moment_inverse<D>(kp, P, b, s[j]);
        }
        sdot_mom<D, 0>(s, full, t);                  /* <(a.u) psi> */
#pragma unroll
        for (int q = 0; q < NV; ++q) t[q] = -t[q];
        moment_inverse<D>(kp, P, t, A);              /* <A psi> = -<(a.u) psi> */
        /* equilibrium slopes: half-range moments of the two sides' slopes */
#pragma unroll
        for (int j = 0; j < D; ++j) {
            spsi_mom<D, 0, 0, 0>(s[j], half, t);
#pragma unroll
            for (int q = 0; q < NV; ++q) dWc[j][q] += P.rho * t[q];
        }
        /* flux: q4 <u psi> - q5 <u (a.u) psi> - q6 <u A psi> */
        psi_mom<D, 1, 0, 0>(half, t);
        sdot_mom<D, 1>(s, half, t2);
#pragma unroll
        for (int q = 0; q < NV; ++q) Fl[q] += P.rho * (q4 * t[q] - q5 * t2[q]);
        spsi_mom<D, 1, 0, 0>(A, half, t);
#pragma unroll
        for (int q = 0; q < NV; ++q) Fl[q] -= P.rho * q6 * t[q];
        /* state at t = dt and conserved moments of the time-averaged f */
        if constexpr (STATE) {
            psi_mom<D, 0, 0, 0>(half, t);
            sdot_mom<D, 0>(s, half, t2);
            double tA[NV];
            spsi_mom<D, 0, 0, 0>(A, half, tA);
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                Gl[q] += P.rho * (ex * t[q] - (dt + tau) * ex * t2[q] - tau * ex * tA[q]);
                if constexpr (VISC) Wf[q] += P.rho * (q4 * t[q] - q5 * t2[q] - q6 * tA[q]);
            }
        }
    }

    /* equilibrium part (Eq. dis2) */
    {
        Mom<D> full;
        make_mom<D>(kp, PC, 0, full);
        double s[D][NV], A[NV], t[NV], t2[NV];
        const double ir = 1.0 / PC.rho;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double b[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) b[q] = dWc[j][q] * ir;
            moment_inverse<D>(kp, PC, b, s[j]);
        }
        sdot_mom<D, 0>(s, full, t2);                 /* <(a.u) psi>_c, reused below */
#pragma unroll
        for (int q = 0; q < NV; ++q) t[q] = -t2[q];
        moment_inverse<D>(kp, PC, t, A);
        double tu[NV], tau2[NV], tAu[NV];
        psi_mom<D, 1, 0, 0>(full, tu);
        sdot_mom<D, 1>(s, full, tau2);
        spsi_mom<D, 1, 0, 0>(A, full, tAu);
#pragma unroll
        for (int q = 0; q < NV; ++q) Fl[q] += PC.rho * (q1 * tu[q] + q2 * tau2[q] + q3 * tAu[q]);
        if constexpr (STATE) {
            double tp[NV], tA[NV];
            psi_mom<D, 0, 0, 0>(full, tp);
            spsi_mom<D, 0, 0, 0>(A, full, tA);
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                Gl[q] += PC.rho * (C1 * tp[q] + C2 * t2[q] + C3 * tA[q]);
                if constexpr (VISC) Wf[q] += PC.rho * (q1 * tp[q] + q2 * t2[q] + q3 * tA[q]);
            }
        }
    }
    const double idt = 1.0 / dt;
#pragma unroll
    for (int q = 0; q < NV; ++q) Fl[q] *= idt;
    if (STATE && VISC && kp.reynolds > 0.0) {
        /* BGK heat flux 1/2 <(u-U)(|u-U|^2+xi^2) f> from flux and conserved moments */
        double u2 = 0.0, UF = 0.0, UW = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            u2 += PC.U[j] * PC.U[j];
            UF += PC.U[j] * Fl[1 + j];
            UW += PC.U[j] * Wf[1 + j];
        }
        const double U0 = PC.U[0];
        const double qh = Fl[D + 1] - UF + 0.5 * u2 * Fl[0] -
                          idt * (U0 * Wf[D + 1] - U0 * UW + 0.5 * U0 * u2 * Wf[0]);
        Fl[D + 1] += (1.0 / kp.prandtl - 1.0) * qh;
    }
    rot_out<D>(e, Fl, F);
    rot_out<D>(e, Gl, G);
}

/* Collisionless first-order flux of two cell averages (normal n, left -> right). */
template <int D>
__host__ __device__ __forceinline__ void kfvs_flux(const KParams& kp, const double* WLc, const double* WRc,
                                          const double* n, double* F) {
    constexpr int NV = D + 2;
    double e[3][3];
    local_frame<D>(n, e);
    double WL[NV], WR[NV], a[NV], b[NV], Fl[NV];
    rot_in<D>(e, WLc, WL);
    rot_in<D>(e, WRc, WR);
    Prim PL, PR;
    primitive<D>(kp, WL, PL);
    primitive<D>(kp, WR, PR);
    Mom<D> hl, hr;
    make_mom<D>(kp, PL, +1, hl);
    make_mom<D>(kp, PR, -1, hr);
    psi_mom<D, 1, 0, 0>(hl, a);
    psi_mom<D, 1, 0, 0>(hr, b);
#pragma unroll
    for (int q = 0; q < NV; ++q) Fl[q] = PL.rho * a[q] + PR.rho * b[q];
    rot_out<D>(e, Fl, F);
}

template <int D>
__host__ __device__ __forceinline__ void euler_flux(const KParams& kp, const double* W, const double* n, double* T) {
    double un = 0.0, ke = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        un += W[1 + d] * n[d];
        ke += W[1 + d] * W[1 + d];
    }
    un /= W[0];
    const double p = (kp.gamma - 1.0) * (W[D + 1] - 0.5 * ke / W[0]);
    T[0] = W[0] * un;
#pragma unroll
    for (int d = 0; d < D; ++d) T[1 + d] = W[1 + d] * un + p * n[d];
    T[D + 1] = (W[D + 1] + p) * un;
}

/*
 * Ghost state across a boundary face with outward normal n.  With `grad`,
 * also the ghost's Cartesian gradients (gg may alias nothing in g).
 */
template <int D, bool GRAD>
__host__ __device__ __forceinline__ void ghost_state(const KParams& kp, int tag, const double* W, const double (*g)[D],
                                            const double* n, double* Wg, double (*gg)[D]) {
    constexpr int NV = D + 2;
    const double gm = kp.gamma;
    const double rho = W[0];
    double U[D], un = 0.0, ke = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        U[d] = W[1 + d] / rho;
        un += U[d] * n[d];
        ke += W[1 + d] * U[d];
    }
    const double p = (gm - 1.0) * (W[D + 1] - 0.5 * ke);
    if (tag == CGKS_TAG_FARFIELD) {
        double uinf_n = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) uinf_n += kp.u_inf[d] * n[d];
        const double pinf = 1.0 / gm;
        const double cinf = sqrt(gm * pinf);
        const double c = sqrt(gm * p / rho);
        const double Rp = un + 2.0 * c / (gm - 1.0), Rm = uinf_n - 2.0 * cinf / (gm - 1.0);
        const double ub = 0.5 * (Rp + Rm), cb = 0.25 * (gm - 1.0) * (Rp - Rm);
        double rb, pb, Ub[D];
        double gfac = 0.5;  /* ghost derivatives / interior derivatives */
        if (ub <= -cb) {
            gfac = 0.0;     /* supersonic inflow: the uniform free stream */
            rb = 1.0; pb = pinf;
#pragma unroll
            for (int d = 0; d < D; ++d) Ub[d] = kp.u_inf[d];
        } else if (ub >= cb) {
            gfac = 1.0;     /* supersonic outflow: the interior state */
            rb = rho; pb = p;
#pragma unroll
            for (int d = 0; d < D; ++d) Ub[d] = U[d];
        } else {
            /* subsonic: interior entropy and tangential velocity where the free
             * stream leaves (u_inf . n > 0), free-stream ones elsewhere */
            double ent;
            if (uinf_n > 0.0) {
                ent = p / pow(rho, gm);
#pragma unroll
                for (int d = 0; d < D; ++d) Ub[d] = U[d] - un * n[d] + ub * n[d];
            } else {
                ent = pinf;  /* p_inf / rho_inf^gamma with rho_inf = 1 */
#pragma unroll
                for (int d = 0; d < D; ++d) Ub[d] = kp.u_inf[d] - uinf_n * n[d] + ub * n[d];
            }
            rb = pow(cb * cb / (gm * ent), 1.0 / (gm - 1.0));
            pb = rb * cb * cb / gm;
        }
        double k2 = 0.0;
        Wg[0] = rb;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            Wg[1 + d] = rb * Ub[d];
            k2 += Ub[d] * Ub[d];
        }
        Wg[D + 1] = pb / (gm - 1.0) + 0.5 * rb * k2;
        /* derivatives: a fraction gfac of the interior ones (half on subsonic faces) */
        if constexpr (GRAD) {
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int d = 0; d < D; ++d) gg[q][d] = gfac * g[q][d];
        }
        return;
    }
    if (tag == CGKS_TAG_SLIP) {
        /* mirror image: x -> x - 2 (x.n) n */
        double mn = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) mn += W[1 + d] * n[d];
        Wg[0] = W[0];
#pragma unroll
        for (int d = 0; d < D; ++d) Wg[1 + d] = W[1 + d] - 2.0 * mn * n[d];
        Wg[D + 1] = W[D + 1];
        if constexpr (GRAD) {
            /* scalar q: grad_g = Rm grad ; momentum: grad_g = Rm (grad m) Rm */
            const int scal[2] = {0, D + 1};
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int q = scal[t];
                double gn = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) gn += g[q][d] * n[d];
#pragma unroll
                for (int d = 0; d < D; ++d) gg[q][d] = g[q][d] - 2.0 * gn * n[d];
            }
            double Mr[D][D];  /* (grad m) Rm */
#pragma unroll
            for (int a = 0; a < D; ++a) {
                double gn = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) gn += g[1 + a][d] * n[d];
#pragma unroll
                for (int d = 0; d < D; ++d) Mr[a][d] = g[1 + a][d] - 2.0 * gn * n[d];
            }
#pragma unroll
            for (int d = 0; d < D; ++d) {
                double nm = 0.0;
#pragma unroll
                for (int a = 0; a < D; ++a) nm += n[a] * Mr[a][d];
#pragma unroll
                for (int a = 0; a < D; ++a) gg[1 + a][d] = Mr[a][d] - 2.0 * n[a] * nm;
            }
        }
        return;
    }
    /* no-slip walls: reversed velocity, same pressure */
    double rg = rho;
    if (tag == CGKS_TAG_ISOTHERMAL) {
        double Tg = 2.0 * kp.Tw - p / rho;
        if (Tg < 0.5 * kp.Tw) Tg = 0.5 * kp.Tw;
        rg = p / Tg;
    }
    double k2 = 0.0;
    Wg[0] = rg;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        Wg[1 + d] = -rg * U[d];
        k2 += U[d] * U[d];
    }
    Wg[D + 1] = p / (gm - 1.0) + 0.5 * rg * k2;
    if constexpr (GRAD) {
#pragma unroll
        for (int q = 0; q < NV; ++q)
#pragma unroll
            for (int d = 0; d < D; ++d) gg[q][d] = g[q][d];
    }
}

}  // namespace cgks

#endif

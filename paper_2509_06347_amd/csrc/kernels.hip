/*
 * gfx950 kernels of the multigrid CGKS V-cycle.
 *
 * Fine level (third-order CGKS, Secs. 2-3):
 *   k_recon   one thread per cell: time step, compact reconstruction (p^2 by
 *             the precomputed constrained least-squares operator, alpha-scaled
 *             Green-Gauss p^1, nonlinear weights), positivity guard, and the
 *             reconstructed state and gradient at every Gauss point of the
 *             cell's faces (plus the ghost state on boundary faces), written
 *             into face-ordered Gauss-point slots.
 *   k_flux    one thread per (face, Gauss point): BGK flux, state at t = dt,
 *             DF factor.  Gauss-point-major layout: consecutive threads read
 *             consecutive faces.
 *   k_gather  one thread per cell: residual, DF-scaled evolved slopes, DF;
 *             optionally the explicit update of Eq. smo and the residual-norm
 *             partial sums.
 * Coarse levels (Secs. 4-5): KFVS residual / forcing / LU-SGS diagonal, the
 * per-colour forward and backward sweeps, the update, restriction and the
 * DF-limited prolongation.
 *
 * No floating-point atomics: every sum has a fixed order.
 */
#include <hip/hip_runtime.h>

#include "cgks_internal.h"
#include "kinetic.hpp"

namespace cgks {

constexpr int BLOCK = 256;

template <int D>
struct Shape {
    static constexpr int NV = D + 2;
    static constexpr int NS = D + 1;                /* faces per cell */
    static constexpr int NQ = (D == 2) ? 5 : 9;     /* quadratic basis size */
    static constexpr int NG = (D == 2) ? 2 : 3;     /* Gauss points per face */
    static constexpr int NC = NV * (1 + D);         /* state + gradient per Gauss point */
    static constexpr int NCOL = NS * (1 + D);       /* operator inputs */
};

/* Exponents of the scaled monomials, same order as the host operator. */
template <int D>
__device__ __forceinline__ void basis_at(const double* X, double* phi, double (*dphi)[3]) {
    if constexpr (D == 2) {
        const double x = X[0], y = X[1];
        phi[0] = x; phi[1] = y; phi[2] = x * x; phi[3] = x * y; phi[4] = y * y;
        dphi[0][0] = 1.0; dphi[0][1] = 0.0;
        dphi[1][0] = 0.0; dphi[1][1] = 1.0;
        dphi[2][0] = 2.0 * x; dphi[2][1] = 0.0;
        dphi[3][0] = y; dphi[3][1] = x;
        dphi[4][0] = 0.0; dphi[4][1] = 2.0 * y;
    } else {
        const double x = X[0], y = X[1], z = X[2];
        phi[0] = x; phi[1] = y; phi[2] = z;
        phi[3] = x * x; phi[4] = x * y; phi[5] = x * z; phi[6] = y * y; phi[7] = y * z; phi[8] = z * z;
        const double d[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2 * x, 0, 0}, {y, x, 0},
                                {z, 0, x}, {0, 2 * y, 0}, {0, z, y}, {0, 0, 2 * z}};
#pragma unroll
        for (int k = 0; k < 9; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) dphi[k][j] = d[k][j];
    }
}

/* Smoothness indicator of p^2 in scaled coordinates, from the cell's basis means
 * (the second moments about the centroid).  The volume powers of the indicator
 * cancel against h = V^(1/D). */
template <int D>
__device__ __forceinline__ double beta_large(const double* a, const double* m) {
    if constexpr (D == 2) {
        /* d/dX p = a0 + 2 a2 X + a3 Y ; d/dY p = a1 + a3 X + 2 a4 Y */
        const double XX = m[2], XY = m[3], YY = m[4];
        const double bx = a[0] * a[0] + 4.0 * a[2] * a[2] * XX + 4.0 * a[2] * a[3] * XY + a[3] * a[3] * YY;
        const double by = a[1] * a[1] + a[3] * a[3] * XX + 4.0 * a[3] * a[4] * XY + 4.0 * a[4] * a[4] * YY;
        const double b2 = 4.0 * a[2] * a[2] + a[3] * a[3] + 4.0 * a[4] * a[4];
        return bx + by + b2;
    } else {
        /* basis: x y z xx xy xz yy yz zz ; second moments m[3..8] */
        const double Mxx = m[3], Mxy = m[4], Mxz = m[5], Myy = m[6], Myz = m[7], Mzz = m[8];
        const double Mm[3][3] = {{Mxx, Mxy, Mxz}, {Mxy, Myy, Myz}, {Mxz, Myz, Mzz}};
        /* Hessian of p in scaled coordinates */
        const double H[3][3] = {{2.0 * a[3], a[4], a[5]}, {a[4], 2.0 * a[6], a[7]}, {a[5], a[7], 2.0 * a[8]}};
        double b = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double q = a[d] * a[d];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) q += H[d][i] * H[d][j] * Mm[i][j];
            b += q;
        }
        /* second derivatives: xx, xy, xz, yy, yz, zz each once */
        b += H[0][0] * H[0][0] + H[0][1] * H[0][1] + H[0][2] * H[0][2] + H[1][1] * H[1][1] + H[1][2] * H[1][2] +
             H[2][2] * H[2][2];
        return b;
    }
}

template <int D>
__global__ void __launch_bounds__(BLOCK) k_recon(FineDev f, KParams kp) {
    using S = Shape<D>;
    constexpr int NV = S::NV, NS = S::NS, NQ = S::NQ, NG = S::NG, NC = S::NC, NCOL = S::NCOL;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = f.n, nf = f.nf;
    if (i >= n) return;
    double W0[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) W0[q] = f.W[q * n + i];
    const double V = f.V[i], h = f.h[i], al = f.alpha[i];
    double xc[D];
#pragma unroll
    for (int d = 0; d < D; ++d) xc[d] = f.C[d * n + i];

    int fid[NS], side[NS], nbr[NS], tag[NS];
    double nout[NS][D], Sf[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int sf = f.slot_face[s * n + i];
        fid[s] = sf >> 1;
        side[s] = sf & 1;
        nbr[s] = f.slot_nbr[s * n + i];
        tag[s] = f.ftag[fid[s]];
        Sf[s] = f.fS[fid[s]];
        const double sg = side[s] ? -1.0 : 1.0;
#pragma unroll
        for (int d = 0; d < D; ++d) nout[s][d] = sg * f.fn[d * nf + fid[s]];
    }

    /* local explicit time step: convective + viscous spectral radius */
    {
        Prim P;
        primitive<D>(kp, W0, P);
        const double c = sqrt(kp.gamma * P.p / P.rho);
        double lam = 0.0, s2 = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            double un = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) un += P.U[d] * nout[s][d];
            lam += Sf[s] * (fabs(un) + c);
            s2 += Sf[s] * Sf[s];
        }
        if (kp.reynolds > 0.0)
            lam += fmax(4.0 / 3.0, kp.gamma / kp.prandtl) * sutherland(kp, P.p / P.rho) / P.rho * s2 / V;
        f.dt[i] = kp.cfl_exp * V / lam;
        f.dti[i] = kp.cfl_imp * V / lam;
    }

    /* neighbour averages (ghost averages on boundary faces) for the sub-stencil */
    double Wn[NS][NV];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (nbr[s] >= 0) {
#pragma unroll
            for (int q = 0; q < NV; ++q) Wn[s][q] = f.W[q * n + nbr[s]];
        } else {
            ghost_state<D, false>(kp, tag[s], W0, nullptr, nout[s], Wn[s], nullptr);
        }
    }

    double mean[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) mean[k] = f.mean0[k * n + i];

    /* per-component polynomial: P = Q0 + sum c2_k (phi_k - mean_k) + c1 . (x - xc) / h */
    double c2[NV][NQ], c1[NV][D];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double in[NCOL];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (nbr[s] >= 0) {
                in[s * (1 + D)] = Wn[s][q] - W0[q];
#pragma unroll
                for (int d = 0; d < D; ++d) in[s * (1 + D) + 1 + d] = f.grad[(q * D + d) * n + nbr[s]];
            } else {
#pragma unroll
                for (int d = 0; d <= D; ++d) in[s * (1 + D) + d] = 0.0;
            }
        }
        double a[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < NCOL; ++j) acc += f.op[(k * NCOL + j) * n + i] * in[j];
            a[k] = acc;
        }
        /* Green-Gauss gradient times h (scaled coordinates), alpha-scaled */
        double g[D];
#pragma unroll
        for (int d = 0; d < D; ++d) g[d] = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const double avg = (Wn[s][q] + W0[q]) / (2.0 * V);
#pragma unroll
            for (int d = 0; d < D; ++d) g[d] += avg * Sf[s] * nout[s][d];
        }
        double gg = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            g[d] *= al * h;
            gg += g[d] * g[d];
        }
        const double b0 = beta_large<D>(a, mean);
        const double b1 = gg;
        const double tz = fabs(b0 - b1);
        const double t0 = tz / (b0 + kp.eps), t1 = tz / (b1 + kp.eps);
        const double w0 = kp.g_large * (1.0 + t0 * t0), w1 = kp.g_small * (1.0 + t1 * t1);
        const double o0 = w0 / (w0 + w1), o1 = w1 / (w0 + w1);
        const double cp2 = o0 / kp.g_large, cp1 = o1 - o0 * kp.g_small / kp.g_large;
#pragma unroll
        for (int k = 0; k < NQ; ++k) c2[q][k] = cp2 * a[k];
#pragma unroll
        for (int d = 0; d < D; ++d) c1[q][d] = cp1 * g[d];
    }

    const double ih = 1.0 / h;
    auto eval = [&](const double* x, double* Wx, double (*gx)[D], bool grad) {
        double X[3], phi[NQ], dphi[NQ][3];
#pragma unroll
        for (int d = 0; d < D; ++d) X[d] = (x[d] - xc[d]) * ih;
        basis_at<D>(X, phi, dphi);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double v = W0[q];
#pragma unroll
            for (int k = 0; k < NQ; ++k) v += c2[q][k] * (phi[k] - mean[k]);
#pragma unroll
            for (int d = 0; d < D; ++d) v += c1[q][d] * X[d];
            Wx[q] = v;
            if (grad) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    double gd = c1[q][d];
#pragma unroll
                    for (int k = 0; k < NQ; ++k) gd += c2[q][k] * dphi[k][d];
                    gx[q][d] = gd * ih;
                }
            }
        }
    };

    /* positivity guard over all Gauss points of the cell */
    bool guard = false;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            double x[D], Wx[NV], gx[NV][D];
#pragma unroll
            for (int d = 0; d < D; ++d) x[d] = f.fgp[(k * D + d) * nf + fid[s]];
            eval(x, Wx, gx, false);
            Prim P;
            primitive<D>(kp, Wx, P);
            if (!(P.rho > 0.0 && P.p > 0.0)) guard = true;
        }
    if (guard) atomicAdd(f.guard, 1ull);

#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            double x[D], Wx[NV], gx[NV][D];
#pragma unroll
            for (int d = 0; d < D; ++d) x[d] = f.fgp[(k * D + d) * nf + fid[s]];
            if (guard) {
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    Wx[q] = W0[q];
#pragma unroll
                    for (int d = 0; d < D; ++d) gx[q][d] = 0.0;
                }
            } else {
                eval(x, Wx, gx, true);
            }
            double* out = f.gpst + (size_t)((side[s] * NG + k) * NC) * nf + fid[s];
#pragma unroll
            for (int q = 0; q < NV; ++q) out[(size_t)q * nf] = Wx[q];
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int d = 0; d < D; ++d) out[(size_t)(NV + q * D + d) * nf] = gx[q][d];
            if (nbr[s] < 0) {
                double Wg[NV], gg[NV][D];
                ghost_state<D, true>(kp, tag[s], Wx, gx, nout[s], Wg, gg);
                double* og = f.gpst + (size_t)((1 * NG + k) * NC) * nf + fid[s];
#pragma unroll
                for (int q = 0; q < NV; ++q) og[(size_t)q * nf] = Wg[q];
#pragma unroll
                for (int q = 0; q < NV; ++q)
#pragma unroll
                    for (int d = 0; d < D; ++d) og[(size_t)(NV + q * D + d) * nf] = gg[q][d];
            }
        }
}

template <int D>
__global__ void __launch_bounds__(BLOCK) k_flux(FineDev f, KParams kp) {
    using S = Shape<D>;
    constexpr int NV = S::NV, NG = S::NG, NC = S::NC;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = f.nf;
    if (t >= NG * nf) return;
    const int k = t / nf, fc = t - k * nf;
    double WL[NV], WR[NV], gL[NV][D], gR[NV][D], nn[D];
    const double* sL = f.gpst + (size_t)((0 * NG + k) * NC) * nf + fc;
    const double* sR = f.gpst + (size_t)((1 * NG + k) * NC) * nf + fc;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        WL[q] = sL[(size_t)q * nf];
        WR[q] = sR[(size_t)q * nf];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            gL[q][d] = sL[(size_t)(NV + q * D + d) * nf];
            gR[q][d] = sR[(size_t)(NV + q * D + d) * nf];
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) nn[d] = f.fn[d * nf + fc];
    const int L = f.fL[fc], R = f.fR[fc];
    double dt = f.dt[L];
    if (R >= 0) dt = fmin(dt, f.dt[R]);
    double F[NV], G[NV], a;
    gks_flux<D>(kp, WL, gL, WR, gR, nn, dt, F, G, &a);
    const double ws = f.fS[fc] / NG;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        f.fF[(size_t)q * NG * nf + t] = ws * F[q];
        f.fG[(size_t)q * NG * nf + t] = ws * G[q];
    }
    f.fa[t] = a;
}

/* Block-level fixed-order sum of one double per thread. */
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[BLOCK];
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

template <int D>
__global__ void __launch_bounds__(BLOCK) k_gather(FineDev f, KParams kp, int mode, double* partial, int* status) {
    using S = Shape<D>;
    constexpr int NV = S::NV, NS = S::NS, NG = S::NG;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = f.n, nf = f.nf;
    double contrib = 0.0;
    if (i < n) {
        double R[NV], Gs[NV][D], a = 1.0;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            R[q] = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) Gs[q][d] = 0.0;
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int sf = f.slot_face[s * n + i];
            const int fc = sf >> 1;
            const double sg = (sf & 1) ? -1.0 : 1.0;
            double nn[D];
#pragma unroll
            for (int d = 0; d < D; ++d) nn[d] = sg * f.fn[d * nf + fc];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                double fs = 0.0, gs = 0.0;
#pragma unroll
                for (int k = 0; k < NG; ++k) {
                    fs += f.fF[(size_t)q * NG * nf + k * nf + fc];
                    gs += f.fG[(size_t)q * NG * nf + k * nf + fc];
                }
                R[q] += sg * fs;
#pragma unroll
                for (int d = 0; d < D; ++d) Gs[q][d] += gs * nn[d];
            }
#pragma unroll
            for (int k = 0; k < NG; ++k) a *= f.fa[k * nf + fc];
        }
        const double V = f.V[i];
        const double sc = a / V;
        if (mode == FINE_EVAL) {
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                f.R[q * n + i] = R[q];
#pragma unroll
                for (int d = 0; d < D; ++d) f.gnew[(q * D + d) * n + i] = sc * Gs[q][d];
            }
            f.anew[i] = a;
        } else if (mode == FINE_RESTRICT) {
#pragma unroll
            for (int q = 0; q < NV; ++q) f.res[q * n + i] = -R[q];
            f.alpha[i] = a;
        } else {
            const double dtv = f.dt[i] / V;
            double Wn[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                Wn[q] = f.W[q * n + i] - dtv * R[q];
                f.W[q * n + i] = Wn[q];
#pragma unroll
                for (int d = 0; d < D; ++d) f.grad[(q * D + d) * n + i] = sc * Gs[q][d];
            }
            f.alpha[i] = a;
            Prim P;
            primitive<D>(kp, Wn, P);
            if (!(P.rho > 0.0 && P.p > 0.0 && isfinite(Wn[D + 1]))) atomicOr(status, 1);
            if (mode == FINE_STEP_NORM) {
                const double r = R[0] / V;
                contrib = r * r;
            }
        }
    }
    if (mode == FINE_STEP_NORM) {
        const double s = block_sum(contrib);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

__global__ void __launch_bounds__(BLOCK) k_norm_finalize(const double* partial, int np, int n, double mach,
                                                         double* history, int cap, int* counter, int* status) {
    double v = 0.0;
    for (int k = threadIdx.x; k < np; k += BLOCK) v += partial[k];
    const double s = block_sum(v);
    if (threadIdx.x == 0) {
        const double nrm = sqrt(s / n) / mach;
        const int c = *counter;
        if (c < cap) history[c] = nrm;
        *counter = c + 1;
        if (!isfinite(nrm)) atomicOr(status, 1);
    }
}

/* ----------------------------------------------------------------- coarse --- */

template <int D>
__global__ void __launch_bounds__(BLOCK) k_coarse_rhs(CoarseDev c, KParams kp, int mode) {
    constexpr int NV = D + 2;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = c.n;
    if (I >= n) return;
    double W[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) W[q] = c.W[q * n + I];
    Prim P;
    primitive<D>(kp, W, P);
    const double cs = sqrt(kp.gamma * P.p / P.rho);
    double Res[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) Res[q] = 0.0;
    double lam = 0.0, s2 = 0.0, sr = 0.0;
    const double visc = fmax(4.0 / 3.0, kp.gamma / kp.prandtl);
    for (int s = 0; s < c.nslot; ++s) {
        const int J = c.snbr[s * n + I];
        const int tg = c.stag[s * n + I];
        if (J < 0 && tg == 0) continue;  /* empty slot */
        const double S = c.sS[s * n + I];
        double nn[D];
#pragma unroll
        for (int d = 0; d < D; ++d) nn[d] = c.sn[(d * c.nslot + s) * n + I];
        double WJ[NV], F[NV], Wm[NV];
        double dist;
        if (J >= 0) {
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                WJ[q] = c.W[q * n + J];
                Wm[q] = 0.5 * (W[q] + WJ[q]);
            }
        } else {
            ghost_state<D, false>(kp, tg, W, nullptr, nn, WJ, nullptr);
#pragma unroll
            for (int q = 0; q < NV; ++q) Wm[q] = W[q];
        }
        dist = c.sd[s * n + I];
        kfvs_flux<D>(kp, W, WJ, nn, F);
#pragma unroll
        for (int q = 0; q < NV; ++q) Res[q] -= S * F[q];
        /* spectral radius of the flux splitting */
        Prim Pm;
        primitive<D>(kp, Wm, Pm);
        double umn = 0.0, un = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            umn += Pm.U[d] * nn[d];
            un += P.U[d] * nn[d];
        }
        double r = kp.omega * (fabs(umn) + sqrt(kp.gamma * Pm.p / Pm.rho));
        if (kp.reynolds > 0.0) r += 2.0 * visc * sutherland(kp, Pm.p / Pm.rho) / (Pm.rho * dist);
        c.r[s * n + I] = r;
        sr += S * r;
        lam += S * (fabs(un) + cs);
        s2 += S * S;
    }
    if (mode == COARSE_FORCING) {
#pragma unroll
        for (int q = 0; q < NV; ++q) c.F[q * n + I] = c.Rstar[q * n + I] - Res[q];
        return;
    }
    if (kp.reynolds > 0.0) lam += visc * sutherland(kp, P.p / P.rho) / P.rho * s2 / c.V[I];
    const double V = c.V[I];
    const double dte = kp.cfl_exp * V / lam, dti = kp.cfl_imp * V / lam;
    c.dte[I] = dte;
    c.dti[I] = dti;
#pragma unroll
    for (int q = 0; q < NV; ++q) c.rhs[q * n + I] = Res[q] + c.F[q * n + I];
    const double a = kp.df_relax ? c.alpha[I] : 1.0;
    c.D[I] = a * (V / dti + 0.5 * sr) + (1.0 - a) * V / dte;
}

/* One colour of the forward (fwd = 1) or backward sweep (Eqs. gpu-forward/
 * backward-relaxation).  Cells of colour c occupy [lo, hi); lower colours sit
 * below lo and higher colours at or above hi. */
template <int D>
__global__ void __launch_bounds__(BLOCK) k_lusgs(CoarseDev c, KParams kp, int lo, int hi, int fwd) {
    constexpr int NV = D + 2;
    const int I = lo + blockIdx.x * blockDim.x + threadIdx.x;
    const int n = c.n;
    if (I >= hi) return;
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    for (int s = 0; s < c.nslot; ++s) {
        const int J = c.snbr[s * n + I];
        if (J < 0) continue;
        if (fwd ? (J >= lo) : (J < hi)) continue;
        const double S = c.sS[s * n + I], r = c.r[s * n + I];
        double nn[D], WJ[NV], dJ[NV], Wp[NV], T1[NV], T0[NV];
#pragma unroll
        for (int d = 0; d < D; ++d) nn[d] = c.sn[(d * c.nslot + s) * n + I];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            WJ[q] = c.W[q * n + J];
            dJ[q] = c.dW[q * n + J];
            Wp[q] = WJ[q] + dJ[q];
        }
        euler_flux<D>(kp, Wp, nn, T1);
        euler_flux<D>(kp, WJ, nn, T0);
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] += S * (T1[q] - T0[q] - r * dJ[q]);
    }
    const double a = kp.df_relax ? c.alpha[I] : 1.0;
    const double Di = c.D[I];
    if (fwd) {
#pragma unroll
        for (int q = 0; q < NV; ++q) c.dW[q * n + I] = (c.rhs[q * n + I] - 0.5 * a * acc[q]) / Di;
    } else {
#pragma unroll
        for (int q = 0; q < NV; ++q) c.dW[q * n + I] -= 0.5 * a * acc[q] / Di;
    }
}

__global__ void __launch_bounds__(BLOCK) k_add(double* W, const double* dW, int m) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) W[t] += dW[t];
}

/* Restriction (Sec. 5.2): W0 = sum V W / V_c, Res* = sum Res, alpha = min. */
template <int D>
__global__ void __launch_bounds__(BLOCK) k_restrict(CoarseDev c, const double* Wf, const double* Vf,
                                                   const double* resf, const double* af, int nfine) {
    constexpr int NV = D + 2;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = c.n;
    if (I >= n) return;
    double w[NV], r[NV], amin = 1.0e300;
#pragma unroll
    for (int q = 0; q < NV; ++q) w[q] = r[q] = 0.0;
    for (int k = c.child_off[I]; k < c.child_off[I + 1]; ++k) {
        const int i = c.child[k];
        const double v = Vf[i];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            w[q] += v * Wf[q * nfine + i];
            r[q] += resf[q * nfine + i];
        }
        amin = fmin(amin, af[i]);
    }
    const double iv = 1.0 / c.V[I];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double w0 = w[q] * iv;
        c.W0[q * n + I] = w0;
        c.W[q * n + I] = w0;
        c.Rstar[q * n + I] = r[q];
    }
    c.alpha[I] = amin;
}

/* DF-limited prolongation (Eq. prolongation) with injection; a correction that
 * would make rho or p non-positive is skipped. */
template <int D>
__global__ void __launch_bounds__(BLOCK) k_prolong(CoarseDev c, double* Wf, const double* af, int nfine,
                                                  int df, unsigned long long* skips) {
    constexpr int NV = D + 2;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nfine) return;
    const int I = c.parent[i];
    const int n = c.n;
    const double a = df ? af[i] : 1.0;
    double Wn[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) Wn[q] = Wf[q * nfine + i] + a * (c.W[q * n + I] - c.W0[q * n + I]);
    double ke = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) ke += Wn[1 + d] * Wn[1 + d];
    const double p = Wn[D + 1] - 0.5 * ke / Wn[0];
    if (Wn[0] > 0.0 && p > 0.0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) Wf[q * nfine + i] = Wn[q];
    } else {
        atomicAdd(skips, 1ull);
    }
}

/* Copy the fine state to the roll-back buffers while no non-physical state
 * has been flagged. */
__global__ void __launch_bounds__(BLOCK) k_save_if_ok(const double* a, double* b, int m, const int* status) {
    if (*status) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) b[t] = a[t];
}

/* ------------------------------------------------------------- launchers --- */

static inline int nblk(long m) { return (int)((m + BLOCK - 1) / BLOCK); }

template <int D>
static void fine_residual(cgks_ctx* c, int mode) {
    FineDev& f = c->fine;
    hipStream_t st = c->stream;
    k_recon<D><<<nblk(f.n), BLOCK, 0, st>>>(f, c->kp);
    k_flux<D><<<nblk((long)f.nf * f.ngp), BLOCK, 0, st>>>(f, c->kp);
    k_gather<D><<<nblk(f.n), BLOCK, 0, st>>>(f, c->kp, mode, c->ws.partial, c->ws.status);
    if (mode == FINE_STEP_NORM)
        k_norm_finalize<<<1, BLOCK, 0, st>>>(c->ws.partial, nblk(f.n), f.n, c->kp.mach, c->ws.history,
                                             c->ws.history_cap, c->ws.counter, c->ws.status);
}

void launch_fine_recon(cgks_ctx* c) {
    FineDev& f = c->fine;
    if (c->dim == 2) k_recon<2><<<nblk(f.n), BLOCK, 0, c->stream>>>(f, c->kp);
    else k_recon<3><<<nblk(f.n), BLOCK, 0, c->stream>>>(f, c->kp);
}

void launch_fine_residual(cgks_ctx* c, int mode) {
    if (c->dim == 2) fine_residual<2>(c, mode);
    else fine_residual<3>(c, mode);
}

void launch_coarse_rhs(cgks_ctx* c, int level, int mode) {
    CoarseDev& L = c->coarse[level - 1];
    if (c->dim == 2) k_coarse_rhs<2><<<nblk(L.n), BLOCK, 0, c->stream>>>(L, c->kp, mode);
    else k_coarse_rhs<3><<<nblk(L.n), BLOCK, 0, c->stream>>>(L, c->kp, mode);
}

void launch_lusgs(cgks_ctx* c, int level) {
    CoarseDev& L = c->coarse[level - 1];
    for (int pass = 0; pass < 2; ++pass)
        for (int k = 0; k < L.ncolor; ++k) {
            const int col = pass == 0 ? k : L.ncolor - 1 - k;
            const int lo = L.color_off[col], hi = L.color_off[col + 1];
            if (hi <= lo) continue;
            if (c->dim == 2) k_lusgs<2><<<nblk(hi - lo), BLOCK, 0, c->stream>>>(L, c->kp, lo, hi, pass == 0);
            else k_lusgs<3><<<nblk(hi - lo), BLOCK, 0, c->stream>>>(L, c->kp, lo, hi, pass == 0);
        }
}

void launch_coarse_update(cgks_ctx* c, int level) {
    CoarseDev& L = c->coarse[level - 1];
    const int m = L.n * c->nv;
    k_add<<<nblk(m), BLOCK, 0, c->stream>>>(L.W, L.dW, m);
}

void launch_restrict(cgks_ctx* c, int level) {
    CoarseDev& G = c->coarse[level];
    const double *Wf, *Vf, *rf, *af;
    int nfine;
    if (level == 0) {
        Wf = c->fine.W; Vf = c->fine.V; rf = c->fine.res; af = c->fine.alpha; nfine = c->fine.n;
    } else {
        CoarseDev& F = c->coarse[level - 1];
        Wf = F.W; Vf = F.V; rf = F.rhs; af = F.alpha; nfine = F.n;
    }
    if (c->dim == 2) k_restrict<2><<<nblk(G.n), BLOCK, 0, c->stream>>>(G, Wf, Vf, rf, af, nfine);
    else k_restrict<3><<<nblk(G.n), BLOCK, 0, c->stream>>>(G, Wf, Vf, rf, af, nfine);
}

void launch_prolong(cgks_ctx* c, int level) {
    CoarseDev& G = c->coarse[level];
    double* Wf;
    const double* af;
    int nfine;
    if (level == 0) {
        Wf = c->fine.W; af = c->fine.alpha; nfine = c->fine.n;
    } else {
        CoarseDev& F = c->coarse[level - 1];
        Wf = F.W; af = F.alpha; nfine = F.n;
    }
    if (c->dim == 2)
        k_prolong<2><<<nblk(nfine), BLOCK, 0, c->stream>>>(G, Wf, af, nfine, c->kp.df_prolong, c->ws.skips);
    else
        k_prolong<3><<<nblk(nfine), BLOCK, 0, c->stream>>>(G, Wf, af, nfine, c->kp.df_prolong, c->ws.skips);
}

void launch_save_state(cgks_ctx* c) {
    FineDev& f = c->fine;
    const int nv = c->nv, dim = c->dim;
    k_save_if_ok<<<nblk((long)f.n * nv), BLOCK, 0, c->stream>>>(f.W, f.Wsave, f.n * nv, c->ws.status);
    k_save_if_ok<<<nblk((long)f.n * nv * dim), BLOCK, 0, c->stream>>>(f.grad, f.gsave, f.n * nv * dim, c->ws.status);
    k_save_if_ok<<<nblk(f.n), BLOCK, 0, c->stream>>>(f.alpha, f.asave, f.n, c->ws.status);
}

}  // namespace cgks

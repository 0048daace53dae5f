/*
 * gfx950 kernels of the multigrid CGKS V-cycle.
 *
 * Fine level (third-order CGKS, Secs. 2-3):
 *   k_recon   per block of cells, in LDS-staged stages: time steps, compact
 *             reconstruction (p^2 by the precomputed constrained
 *             least-squares operator, alpha-scaled Green-Gauss p^1,
 *             nonlinear weights), positivity guard; writes each cell's
 *             polynomial record.
 *   k_flux    one lane per (face, Gauss point): both cells' polynomials at
 *             the point, BGK flux, state at t = dt, DF factor; the face's
 *             lanes sum their contributions into a per-face record.
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

#include <type_traits>

#include "cgks_internal.h"
#include "kinetic.hpp"

namespace cgks {

constexpr int BLOCK = 256;
/* Coarse levels hold 8k-33k cells per colour sweep or less: small blocks spread
 * them over all 256 compute units. */
constexpr int CBLOCK = 64;

/* Parameters of the problem that owns item idx (batched solves); the shared
 * parameters come from kp itself. */
__device__ __forceinline__ KParams localize(const KParams& kp, const double* ptab, const int* pid, int idx) {
    KParams k = kp;
    if (pid) {
        const double* t = ptab + PTAB * pid[idx];
        k.mach = t[0];
        k.reynolds = t[1];
        k.mu_inf = t[2];
        k.Tw = t[3];
        k.u_inf[0] = t[4];
        k.u_inf[1] = t[5];
        k.u_inf[2] = t[6];
    }
    return k;
}

/* Whether the problem that owns item idx still cycles: in a batched solve the
 * members that have converged or failed are frozen (their kernels' work is
 * skipped); a single problem always cycles. */
__device__ __forceinline__ bool active(const int* pact, const int* pid, int idx) {
    return !pact || pact[pid[idx]] != 0;
}

/* Implicit CFL of the LU-SGS in the current V-cycle: cfl_imp, or with a ramp of
 * N cycles cfl_imp * min(1, k/N) in the k-th cycle since the state was set
 * (k >= 1; outside a cycle the last cycle's value). */
__device__ __forceinline__ double implicit_cfl(const KParams& kp) {
    if (kp.cfl_ramp <= 0) return kp.cfl_imp;
    const int k = *kp.ncyc;
    return kp.cfl_imp * fmin(1.0, (double)(k > 1 ? k : 1) / (double)kp.cfl_ramp);
}

/* Weight of the flux-Jacobian terms of a coarse cell's LU-SGS (Sec. 4.3): its
 * DF value, one fixed weight for every cell, or 1 (fully implicit, and the
 * fixed-factor relaxation of df_relax = 3, which scales the time term only). */
__device__ __forceinline__ double relax_weight(const KParams& kp, double alpha) {
    return kp.df_relax == 1 ? alpha : (kp.df_relax == 2 ? kp.relax_beta : 1.0);
}

/* Diagonal of a coarse cell's LU-SGS.  DF relaxation and its variants blend
 * the implicit and the explicit diagonals with the weight above (Eq.
 * DF-relaxation-hybrid); the fixed-factor relaxation the paper contrasts it
 * with (remark in Sec. 4.3) scales the implicit time term by beta alone. */
__device__ __forceinline__ double lusgs_diagonal(const KParams& kp, double alpha, double V, double dti, double dte,
                                                 double sr) {
    if (kp.df_relax == 3) return kp.relax_beta * V / dti + 0.5 * sr;
    const double a = relax_weight(kp, alpha);
    return a * (V / dti + 0.5 * sr) + (1.0 - a) * V / dte;
}

/* Right-hand side of the fixed-factor relaxation: (1 - beta) times the cell's
 * increment of the previous LU-SGS iteration (zero after restriction), scaled
 * by V / dt_i so that it is a flux like the residual (the printed term lacks
 * the scale). */
template <int NV, class T>
__device__ __forceinline__ void fixed_factor_rhs(const KParams& kp, const CoarseDev& c, int I, double V, double dti,
                                                 double* rhs) {
    if (kp.df_relax != 3) return;
    const T* dW = reinterpret_cast<const T*>(c.dW);
#pragma unroll
    for (int q = 0; q < NV; ++q) rhs[q] += (1.0 - kp.relax_beta) * (V / dti) * (double)dW[q * c.n + I];
}

/* HY: 3-D hybrid meshes (tetrahedra, pyramids, prisms, hexahedra; Sec. 2.2):
 * six face slots per cell (empty past the cell's faces) and four Gauss
 * points per face (a triangle's fourth repeats its first with weight 0). */
template <int D, bool HY = false>
struct Shape {
    static_assert(!HY || D == 3, "hybrid meshes are 3-D");
    static constexpr int NV = D + 2;
    static constexpr int NS = HY ? 6 : D + 1;       /* face slots per cell */
    static constexpr int NQ = (D == 2) ? 5 : 9;     /* quadratic basis size */
    static constexpr int NG = HY ? 4 : (D == 2) ? 2 : 3;   /* Gauss points per face */
    static constexpr int TPF = HY ? 2 : NG;         /* reconstruction threads per face slot */
    static constexpr int NC = NV * (1 + D);         /* state + gradient per Gauss point */
    static constexpr int NCOL = NS * (1 + D);       /* operator inputs */
    static constexpr int NK = NQ + D;               /* coefficients per component: p^2 part, Green-Gauss part */
    /* per-cell polynomial record handed from the reconstruction to the flux:
     * coefficients [NV][NK], cell averages [NV], basis means [NQ], centroid [D], 1/h */
    static constexpr int REC_W = NV * NK;
    static constexpr int REC_MEAN = REC_W + NV;
    static constexpr int REC_C = REC_MEAN + NQ;
    static constexpr int REC_IH = REC_C + D;
    static constexpr int NPR = (D == 2) ? 40 : 80;  /* record stride (3-D padded to 16-byte rows) */
    static constexpr int FO = 2 * NV + 1;           /* per-face output: sum wS F, sum wS W(dt), DF product */
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

/* Per-block LDS of the reconstruction: for each field, one double per cell of
 * the block (stride cells + 1, so that the record writes, which walk the
 * fields of one cell, spread over the banks). */
template <int D, bool HY>
struct RLds {
    using S = Shape<D, HY>;
    static constexpr int NV = S::NV, NS = S::NS, NQ = S::NQ, NK = S::NK;
    static constexpr int WN = 0;                     /* [NS][NV] neighbour averages (ghost states on boundary faces) */
    static constexpr int GN = WN + NS * NV;          /* [NS][NV][D] neighbour gradients, read by stage 2 */
    static constexpr int COEF = GN;                  /* [NV][NK] p^2 part, Green-Gauss part: written after
                                                        stage 2's reads of GN, over them */
    static constexpr int W0 = GN + (NS * NV * D > NV * NK ? NS * NV * D : NV * NK);   /* [NV] cell averages */
    static constexpr int MEAN = W0 + NV;             /* [NQ] basis means */
    static constexpr int GEO = MEAN + NQ;            /* [NS][1 + D] face area, outward unit normal */
    static constexpr int CEL = GEO + NS * (1 + D);   /* volume, h, DF factor */
    static constexpr int FIELDS = CEL + 3;
    /* bytes for `cells` cells: the fields, then per-cell neighbours [NS], the
     * guard flag and the slip-wall flag */
    static constexpr size_t bytes(int cells) {
        return (size_t)FIELDS * (cells + 1) * sizeof(double) + (size_t)(NS + 2) * cells * sizeof(int);
    }
};

/* Reconstruction of a block of `cells` cells (blockDim = cells x faces x Gauss
 * points), in stages separated by block barriers, each with its own mapping of
 * threads to work so that every stage keeps most lanes busy and issues its
 * global loads together:
 *   1. (cell, face slot, component): the cell's and its neighbours' data into
 *      LDS (cell and neighbour averages, neighbour gradients, basis means,
 *      face geometry, V, h, DF factor);
 *   2. (cell, face slot) on boundary faces: the ghost averages; and
 *      (cell, p^2 basis function k): row k of the constrained least-squares
 *      operator (Sec. 3.1) applied to the neighbour differences and gradients
 *      of every component;
 *   3. (cell, component): the DF-scaled Green-Gauss p^1, the smoothness
 *      indicators and nonlinear weights (Sec. 3.2), the combined
 *      coefficients; component 0 also forms the local time steps;
 *   4. (cell, face slot, Gauss point): the combined polynomial's value at the
 *      point, for the cell's positivity guard (an LDS flag over its points).
 * The block then writes each cell's polynomial record (coefficients, zeroed
 * when the guard holds so that the cell is constant; cell averages; basis
 * means; centroid; 1/h), contiguous per cell, which the flux kernel
 * evaluates at its Gauss points.  Per cell and component the arithmetic, and
 * its order, is that of a one-thread-per-cell evaluation.  The coefficients
 * take the LDS of the neighbour gradients once stage 2 has read them, so that
 * six waves per SIMD fit (80 VGPRs, asked for: 0.5 % faster per V-cycle than
 * five). */
constexpr int RTHREADS = 384;  /* most threads per reconstruction block: 64 cells in 2-D, 32 in 3-D */
template <int D, int CELLS, bool HY>
__global__ void __launch_bounds__((CELLS * Shape<D, HY>::NS * Shape<D, HY>::TPF)) __attribute__((amdgpu_waves_per_eu(HY ? 5 : 6)))
k_recon(FineDev f, KParams kp0) {
    using S = Shape<D, HY>;
    using L = RLds<D, HY>;
    constexpr int NV = S::NV, NS = S::NS, NQ = S::NQ, NG = S::NG, NCOL = S::NCOL, NK = S::NK;
    constexpr int TPF = S::TPF;
    constexpr int cells = CELLS, nt = CELLS * NS * TPF, cs = CELLS + 1;   /* compile-time: index math by shifts */
    static_assert(nt <= RTHREADS, "reconstruction block");
    extern __shared__ double lds[];
    int* nbf = reinterpret_cast<int*>(lds + (size_t)L::FIELDS * cs);   /* [NS][cells] neighbour, < 0 on boundaries */
    int* bad = nbf + NS * cells;
    int* slip = bad + cells;   /* the cell has a slip-wall face */
    const int t = threadIdx.x;
    const int n = f.n;
    const int i0 = blockIdx.x * cells;
#define FLD(field, cl) lds[(field) * cs + (cl)]

    /* ---- 1: loads, (cell, slot, component).  A thread takes at most
     * ceil(NV / TPF) items (2; hybrid cells 3) and issues all their loads
     * before the first LDS store, so that the block waits on memory twice,
     * not four times. ---- */
    {
        constexpr int NIT = (NV + TPF - 1) / TPF;
        const int total = cells * NS * NV;
        int cl[NIT], sl[NIT], qq[NIT], nb[NIT];
        bool ok[NIT];
        double w[NIT], g[NIT][D], own[NIT][3];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int u = t + it * nt;
            cl[it] = u % cells;
            const int r = u / cells, s = r % NS, q = r / NS, i = i0 + cl[it];
            sl[it] = s;
            qq[it] = q;
            ok[it] = u < total && i < n && active(f.pact, f.pid, i);
            nb[it] = -1;
            own[it][0] = own[it][1] = own[it][2] = 0.0;
            if (!ok[it]) continue;
            nb[it] = f.slot_nbr[s * n + i];
            if (s == 0) own[it][0] = f.W[q * n + i];
            if (q == 0) own[it][1] = f.slot_S[s * n + i];
            else if (q <= D) own[it][1] = f.slot_n[((q - 1) * NS + s) * n + i];
            const int lin = s * NV + q;
            if (lin < NQ) own[it][2] = f.mean0[lin * n + i];
            else if (lin == NQ) own[it][2] = f.V[i];
            else if (lin == NQ + 1) own[it][2] = f.h[i];
            else if (lin == NQ + 2) own[it][2] = f.alpha[i];
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            w[it] = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) g[it][d] = 0.0;
            if (nb[it] < 0) continue;
            const int q = qq[it], j = nb[it];
            w[it] = f.W[q * n + j];
#pragma unroll
            for (int d = 0; d < D; ++d) g[it][d] = f.grad[(q * D + d) * n + j];
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            if (!ok[it]) continue;
            const int c = cl[it], s = sl[it], q = qq[it], lin = s * NV + q;
            if (q == 0) nbf[s * cells + c] = nb[it];
            if (s == 0) FLD(L::W0 + q, c) = own[it][0];
            if (q <= D) FLD(L::GEO + s * (1 + D) + q, c) = own[it][1];
            if (lin < NQ) FLD(L::MEAN + lin, c) = own[it][2];
            else if (lin < NQ + 3) FLD(L::CEL + lin - NQ, c) = own[it][2];
            if (nb[it] >= 0) {
                FLD(L::WN + s * NV + q, c) = w[it];
#pragma unroll
                for (int d = 0; d < D; ++d) FLD(L::GN + (s * NV + q) * D + d, c) = g[it][d];
            }
        }
    }
    for (int u = t; u < cells; u += nt) bad[u] = slip[u] = 0;
    __syncthreads();

    /* ---- 2: ghost averages of boundary faces, (cell, slot); operator rows,
     * (cell, k), which read only the interior faces' entries ---- */
    for (int u = t; u < cells * NS; u += nt) {
        const int cl = u % cells, s = u / cells;
        const int i = i0 + cl;
        if (i >= n || nbf[s * cells + cl] >= 0 || !active(f.pact, f.pid, i)) continue;
        const KParams kp = localize(kp0, f.ptab, f.pid, i);
        double W0[NV], nout[D], Wg[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) W0[q] = FLD(L::W0 + q, cl);
#pragma unroll
        for (int d = 0; d < D; ++d) nout[d] = FLD(L::GEO + s * (1 + D) + 1 + d, cl);
        const int tag = f.slot_tag[s * n + i];
        if (HY && tag < 0) {   /* empty slot (area 0): the cell's own averages keep its sums finite */
#pragma unroll
            for (int q = 0; q < NV; ++q) FLD(L::WN + s * NV + q, cl) = W0[q];
            continue;
        }
        if (tag == CGKS_TAG_SLIP) slip[cl] = 1;
        ghost_state<D, false>(kp, tag, W0, nullptr, nout, Wg, nullptr);
#pragma unroll
        for (int q = 0; q < NV; ++q) FLD(L::WN + s * NV + q, cl) = Wg[q];
    }
    {
        static_assert(cells * NQ <= nt, "one (cell, k) item per thread");
        const int cl = t % cells, k = t / cells;
        const int i = i0 + cl;
        const bool live = t < cells * NQ && i < n && active(f.pact, f.pid, i);
        double a[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) a[q] = 0.0;
        if (live) {
            double o[NS][1 + D];
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int c = 0; c <= D; ++c) o[s][c] = f.op[(size_t)(k * NCOL + s * (1 + D) + c) * n + i];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (nbf[s * cells + cl] < 0) continue;
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    const double dq = FLD(L::WN + s * NV + q, cl) - FLD(L::W0 + q, cl);
                    double acc = o[s][0] * dq;
#pragma unroll
                    for (int d = 0; d < D; ++d) acc += o[s][1 + d] * FLD(L::GN + (s * NV + q) * D + d, cl);
                    a[q] += acc;
                }
            }
        }
        __syncthreads();   /* every read of GN is done: COEF takes its place */
        if (live)
#pragma unroll
            for (int q = 0; q < NV; ++q) FLD(L::COEF + q * NK + k, cl) = a[q];
    }
    __syncthreads();

    /* ---- 3: weights, (cell, component) ---- */
    for (int u = t; u < cells * NV; u += nt) {
        const int cl = u % cells, q = u / cells;
        const int i = i0 + cl;
        if (i >= n || !active(f.pact, f.pid, i)) continue;
        const KParams kp = localize(kp0, f.ptab, f.pid, i);
        const double V = FLD(L::CEL, cl), h = FLD(L::CEL + 1, cl), al = FLD(L::CEL + 2, cl);
        double W0[NV], Sf[NS], nout[NS][D];
#pragma unroll
        for (int r = 0; r < NV; ++r) W0[r] = FLD(L::W0 + r, cl);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            Sf[s] = FLD(L::GEO + s * (1 + D), cl);
#pragma unroll
            for (int d = 0; d < D; ++d) nout[s][d] = FLD(L::GEO + s * (1 + D) + 1 + d, cl);
        }
        if (q == 0) {
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
            f.dti[i] = implicit_cfl(kp) * V / lam;
        }
        /* component q of the neighbour averages (ghost averages on boundary faces) */
        double Wq[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) Wq[s] = FLD(L::WN + s * NV + q, cl);
        double a[NQ], mean[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            a[k] = FLD(L::COEF + q * NK + k, cl);
            mean[k] = FLD(L::MEAN + k, cl);
        }
        double g[D];
#pragma unroll
        for (int d = 0; d < D; ++d) g[d] = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const double avg = (Wq[s] + W0[q]) / (2.0 * V);
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
        double o0 = w0 / (w0 + w1), o1 = w1 / (w0 + w1);
        if (kp.slip_wall_p1 && slip[cl]) {   /* slip-wall cells: p^1 alone (option, not the paper's) */
            o0 = 0.0;
            o1 = 1.0;
        }
        const double cp2 = o0 / kp.g_large, cp1 = o1 - o0 * kp.g_small / kp.g_large;
#pragma unroll
        for (int k = 0; k < NQ; ++k) FLD(L::COEF + q * NK + k, cl) = cp2 * a[k];
#pragma unroll
        for (int d = 0; d < D; ++d) FLD(L::COEF + q * NK + NQ + d, cl) = cp1 * g[d];
    }
    __syncthreads();

    /* ---- 4: positivity guard, (cell, slot, Gauss point; hybrid cells: two
     * points per thread).  Triangles: slot fastest; 3-D: cell fastest
     * (slot-fastest lanes measured 1.8x slower). ---- */
    {
        int s, cl, k;
        if constexpr (D == 2) {
            s = t % NS;
            cl = (t / NS) % cells;
            k = t / (NS * cells);
        } else {
            cl = t % cells;
            s = (t / cells) / TPF;
            k = (t / cells) - s * TPF;
        }
        const int i = i0 + cl;
        auto guard_point = [&](int k) {
        if (i < n && k < NG && active(f.pact, f.pid, i)) {
            double X[3], phi[NQ], dphi[NQ][3], Wx[NV];
#pragma unroll
            for (int d = 0; d < D; ++d)
                X[d] = f.slot_X[D == 2 ? ((size_t)(k * D + d) * n + i) * NS + s
                                       : ((size_t)(k * D + d) * NS + s) * n + i];
            basis_at<D>(X, phi, dphi);
            double pm[NQ];
#pragma unroll
            for (int m = 0; m < NQ; ++m) pm[m] = phi[m] - FLD(L::MEAN + m, cl);
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                double v = FLD(L::W0 + q, cl);
#pragma unroll
                for (int m = 0; m < NQ; ++m) v += FLD(L::COEF + q * NK + m, cl) * pm[m];
#pragma unroll
                for (int d = 0; d < D; ++d) v += FLD(L::COEF + q * NK + NQ + d, cl) * X[d];
                Wx[q] = v;
            }
            const KParams kp = localize(kp0, f.ptab, f.pid, i);
            Prim P;
            primitive<D>(kp, Wx, P);
            if (!(P.rho > 0.0 && P.p > 0.0)) atomicOr(&bad[cl], 1);
        }
        };
        guard_point(k);
        if constexpr (TPF < NG) guard_point(k + TPF);   /* hybrid cells: two Gauss points per thread */
    }
    __syncthreads();
    for (int u = t; u < cells; u += nt)
        if (i0 + u < n && bad[u] && active(f.pact, f.pid, i0 + u)) atomicAdd(f.guard, 1ull);
    /* the cells' polynomial records, written contiguously by the whole block:
     * coefficients and cell averages (the static rest, basis means,
     * centroid and 1/h, is written once when the mesh is uploaded) */
    constexpr int NPR = S::NPR, NDYN = S::REC_MEAN;
    const int ncell = min(cells, n - i0);
    for (int e = t; e < ncell * NDYN; e += nt) {
        const int c2 = e / NDYN, jj = e - c2 * NDYN, ii = i0 + c2;
        if (!active(f.pact, f.pid, ii)) continue;
        const double v = jj < S::REC_W ? (bad[c2] ? 0.0 : FLD(L::COEF + jj, c2)) : FLD(L::W0 + jj - S::REC_W, c2);
        f.poly[(size_t)ii * NPR + jj] = v;
    }
#undef FLD
}

/* Value and gradient of every component of a cell's combined polynomial at
 * the point x (absolute coordinates), from its record. */
template <int D>
__device__ __forceinline__ void eval_poly(const double* __restrict__ rec, const double* x, double* W,
                                          double (*g)[D]) {
    using S = Shape<D>;
    constexpr int NV = S::NV, NQ = S::NQ, NK = S::NK;
    const double ih = rec[S::REC_IH];
    double X[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < D; ++d) X[d] = (x[d] - rec[S::REC_C + d]) * ih;
    double phi[NQ], dphi[NQ][3], pm[NQ];
    basis_at<D>(X, phi, dphi);
#pragma unroll
    for (int m = 0; m < NQ; ++m) pm[m] = phi[m] - rec[S::REC_MEAN + m];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double* c = rec + q * NK;
        double v = rec[S::REC_W + q];
#pragma unroll
        for (int m = 0; m < NQ; ++m) v += c[m] * pm[m];
#pragma unroll
        for (int d = 0; d < D; ++d) v += c[NQ + d] * X[d];
        W[q] = v;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            double gd = c[NQ + d];
#pragma unroll
            for (int m = 0; m < NQ; ++m) gd += c[m] * dphi[m][d];
            g[q][d] = gd * ih;
        }
    }
}

/* BGK flux (Sec. 2), one lane per (face, Gauss point): the face's Gauss
 * points sit in adjacent lanes of one wave (64 / NG faces per wave; in 3-D
 * the last lane idles), so the two cells' records they read are shared.  The
 * face's first lane sums the lanes' S/NG-weighted fluxes and states at
 * t = dt in Gauss-point order and multiplies their DF factors, and writes
 * the face's record [sum wS F, sum wS W(dt), DF product].  STATE = false:
 * the inviscid residual for restriction, which needs no W(dt); without its
 * moments the kernel nearly fits two waves per SIMD, and asking for two
 * (a few registers spill) measured 1.6 % faster per V-cycle.  VISC = false:
 * Euler flows, without the viscous collision time and the heat-flux
 * accumulators (31 fewer accumulation registers, fewer spills: 4.5 % per
 * V-cycle on the Mach 6 sphere); batches always take VISC = true, their
 * Reynolds numbers being per problem. */
constexpr int FTHREADS = 256;
template <int D, bool STATE, bool HY, bool VISC = true>
__global__ void __launch_bounds__(FTHREADS) __attribute__((amdgpu_waves_per_eu(STATE ? 1 : 2)))
k_flux(FineDev f, KParams kp0) {
    using S = Shape<D, HY>;
    constexpr int NV = S::NV, NG = S::NG, NPR = S::NPR, FO = S::FO, NS = S::NS;
    constexpr int FPW = 64 / NG;
    const int lane = threadIdx.x & 63;
    const long wv = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int k = lane % NG, lf = lane / NG;
    const long fcl = wv * FPW + lf;
    const int nf = f.nf;
    const bool live = lf < FPW && fcl < nf && active(f.pact, f.fpid, (int)fcl);
    const int fc = live ? (int)fcl : 0;
    double F[NV], G[NV], a = 1.0;
#pragma unroll
    for (int q = 0; q < NV; ++q) F[q] = G[q] = 0.0;
    if (live) {
        const KParams kp = localize(kp0, f.ptab, f.fpid, fc);
        const int L = f.fL[fc], R = f.fR[fc];
        double x[D], nn[D], WL[NV], WR[NV], gL[NV][D], gR[NV][D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            x[d] = f.fX[((size_t)fc * NG + k) * D + d];
            nn[d] = f.fn[(size_t)d * nf + fc];
        }
        eval_poly<D>(f.poly + (size_t)L * NPR, x, WL, gL);
        if (R >= 0) {
            eval_poly<D>(f.poly + (size_t)R * NPR, x, WR, gR);
        } else {
            const int tag = f.slot_tag[(size_t)(f.fslot[fc] & 7) * f.n + L];
            ghost_state<D, true>(kp, tag, WL, gL, nn, WR, gR);
        }
        double dt = f.dt[L];
        if (R >= 0) dt = fmin(dt, f.dt[R]);
        double Fk[NV], Gk[NV];
        gks_flux<D, STATE, VISC>(kp, WL, gL, WR, gR, nn, dt, Fk, Gk, &a);
        double ws = f.fS[fc] / NG;
        if constexpr (HY) {   /* per-point weight x area; a weight-0 point leaves the DF product alone */
            ws = f.fw[(size_t)fc * NG + k];
            if (ws == 0.0) a = 1.0;
        }
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            F[q] = ws * Fk[q];
            G[q] = ws * Gk[q];
        }
    }
    (void)NS;
    const int base = lane - k;
    double out[FO];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double sf = 0.0, sg = 0.0;
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            sf += __shfl(F[q], base + j);
            sg += __shfl(G[q], base + j);
        }
        out[q] = sf;
        out[NV + q] = sg;
    }
    double ap = 1.0;
#pragma unroll
    for (int j = 0; j < NG; ++j) ap *= __shfl(a, base + j);
    out[2 * NV] = ap;
    if (live && k == 0) {
        double* o = f.fout + (size_t)fc * FO;
#pragma unroll
        for (int e = 0; e < FO; ++e) o[e] = out[e];
    }
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

/* Internal energy density rho e = E - |m|^2 / (2 rho), proportional to p. */
template <int D>
__device__ __forceinline__ double rho_e_plain(const double* W) {
#pragma clang fp contract(off)
    double ke = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) ke = ke + W[1 + d] * W[1 + d];
    return W[D + 1] - 0.5 * ke / W[0];
}

/* Fraction of the update dW that a cell applies (no safeguard is stated in
 * the paper): kappa <= 0 takes all of dW when rho and p stay positive, else
 * none; kappa > 0 takes the largest of 1, 1/2, ..., 2^-10 that keeps rho and
 * rho e positive and at least (1 - kappa) times their current values, else
 * none.  Evaluated without contraction so that its decisions match a plain
 * FP64 evaluation. */
template <int D>
__device__ double update_fraction(const double* W, const double* dW, double kappa) {
#pragma clang fp contract(off)
    constexpr int NV = D + 2;
    double Wn[NV];
    if (!(kappa > 0.0)) {
#pragma unroll
        for (int q = 0; q < NV; ++q) Wn[q] = W[q] + dW[q];
        return (Wn[0] > 0.0 && rho_e_plain<D>(Wn) > 0.0) ? 1.0 : 0.0;
    }
    const double lo_r = (1.0 - kappa) * W[0];
    const double lo_e = (1.0 - kappa) * rho_e_plain<D>(W);
    double th = 1.0;
    for (int m = 0; m <= 10; ++m) {
#pragma unroll
        for (int q = 0; q < NV; ++q) Wn[q] = W[q] + th * dW[q];
        if (Wn[0] > 0.0 && Wn[0] >= lo_r) {
            const double e = rho_e_plain<D>(Wn);
            if (e > 0.0 && e >= lo_e) return th;
        }
        th = 0.5 * th;
    }
    return 0.0;
}

template <int D, bool HY>
__global__ void __launch_bounds__(BLOCK) k_gather(FineDev f, KParams kp, int mode, double* partial, int* status) {
    using S = Shape<D, HY>;
    constexpr int NV = S::NV, NS = S::NS, NG = S::NG;
    const bool keep = (mode & FINE_KEEP) != 0;
    mode &= ~FINE_KEEP;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = f.n, nf = f.nf;
    double contrib = 0.0;
    if (i < n && active(f.pact, f.pid, i)) {
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
            if (HY && sf < 0) continue;   /* empty slot */
            const int fc = sf >> 1;
            const double sg = (sf & 1) ? -1.0 : 1.0;
            double nn[D];
#pragma unroll
            for (int d = 0; d < D; ++d) nn[d] = f.slot_n[(d * NS + s) * n + i];
            const double* o = f.fout + (size_t)fc * S::FO;
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                R[q] += sg * o[q];
#pragma unroll
                for (int d = 0; d < D; ++d) Gs[q][d] += o[NV + q] * nn[d];
            }
            a *= o[2 * NV];
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
            const double th = kp.slope_relax;
            double Wo[NV], dW[NV], Wn[NV];
            bool finite = true;
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                Wo[q] = f.W[q * n + i];
                dW[q] = -(dtv * R[q]);
                finite = finite && isfinite(dW[q]);
            }
            const double fr = update_fraction<D>(Wo, dW, kp.update_limit);
            /* every load before the first store: a load issued after a store
             * waits for the store to complete */
            double go[NV][D];
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int d = 0; d < D; ++d) go[q][d] = f.grad[(q * D + d) * n + i];
            if (keep) {
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    f.res[q * n + i] = -R[q];
                    f.Wpre[q * n + i] = Wo[q];
                }
            }
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                Wn[q] = fr > 0.0 ? Wo[q] + fr * dW[q] : Wo[q];
                f.W[q * n + i] = Wn[q];
#pragma unroll
                for (int d = 0; d < D; ++d) f.grad[(q * D + d) * n + i] = go[q][d] + th * (sc * Gs[q][d] - go[q][d]);
            }
            f.alpha[i] = a;
            Prim P;
            primitive<D>(kp, Wn, P);
            if (!(finite && P.rho > 0.0 && P.p > 0.0 && isfinite(Wn[D + 1]))) atomicOr(status, 1);
            if (mode == FINE_STEP_NORM) {
                const double r = R[0] / V;
                contrib = r * r;
                if (f.pid) f.r2[i] = contrib;
            }
        }
    }
    if (mode == FINE_STEP_NORM && !f.pid) {
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

/* Per-problem norms of a batched solve: block b reduces the cells of problem b
 * in a fixed order and appends its norm to history[b * cap + cycle]. */
__global__ void __launch_bounds__(BLOCK) k_norm_batch(const double* r2, const int* off, const double* ptab,
                                                      double* history, int cap, int* counter, int nprob) {
    const int b = blockIdx.x;
    const int lo = off[b], hi = off[b + 1];
    double v = 0.0;
    for (int k = lo + threadIdx.x; k < hi; k += BLOCK) v += r2[k];
    const double s = block_sum(v);
    if (threadIdx.x == 0) {
        const int c = *counter;
        const double nrm = sqrt(s / (hi - lo)) / ptab[PTAB * b];
        if (c < cap) history[(size_t)b * cap + c] = nrm;
    }
}

__global__ void k_count(int* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter += 1;
}

/* ----------------------------------------------------------------- coarse --- */

template <int D, class T>
__global__ void __launch_bounds__(CBLOCK) k_coarse_rhs(CoarseDev c, KParams kp0, int mode, int hi1) {
    constexpr int NV = D + 2;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = c.n;
    if (I >= n || !active(c.pact, c.pid, I)) return;
    const KParams kp = localize(kp0, c.ptab, c.pid, I);
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
        reinterpret_cast<T*>(c.r)[s * n + I] = (T)r;
        sr += S * r;
        lam += S * (fabs(un) + cs);
        s2 += S * S;
    }
    if (mode == COARSE_FORCING) {
#pragma unroll
        for (int q = 0; q < NV; ++q) c.F[q * n + I] = (double)reinterpret_cast<const T*>(c.Rstar)[q * n + I] - Res[q];
        return;
    }
    if (kp.reynolds > 0.0) lam += visc * sutherland(kp, P.p / P.rho) / P.rho * s2 / c.V[I];
    const double V = c.V[I];
    const double dte = kp.cfl_exp * V / lam, dti = implicit_cfl(kp) * V / lam;
    c.dte[I] = dte;
    c.dti[I] = dti;
    double rhs[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) rhs[q] = Res[q] + c.F[q * n + I];
    if (mode == COARSE_RHS) fixed_factor_rhs<NV, T>(kp, c, I, V, dti, rhs);
#pragma unroll
    for (int q = 0; q < NV; ++q) c.rhs[q * n + I] = rhs[q];
    const double Dd = lusgs_diagonal(kp, c.alpha[I], V, dti, dte, sr);
    c.D[I] = Dd;
    /* The forward sweep of the first colour has no lower neighbours: its
     * correction is rhs / D, formed here exactly as the sweep would. */
    if (I < hi1) {
        T* dW = reinterpret_cast<T*>(c.dW);
#pragma unroll
        for (int q = 0; q < NV; ++q) dW[q * n + I] = (T)rhs[q] / (T)Dd;
    }
}

/* Coarse right-hand side with one thread per (cell, face slot): block
 * (CELLS, nslot), slot terms combined in slot order by the slot-0 thread.
 * Same arithmetic as one thread per cell, with nslot times the parallelism
 * (the coarse levels are too small to fill the chip one cell per thread). */
constexpr int MAXS = 8;     /* most face slots handled by the slot-parallel kernels */
/* Cells per block of the slot-parallel kernels (SC) is a template parameter,
 * chosen per coarse level by the autotuner among 16, 32 and 64: small levels
 * and colour ranges spread over more compute units with smaller blocks. */
template <int D, class T, int SC>
__global__ void __launch_bounds__(SC * MAXS) k_coarse_rhs_s(CoarseDev c, KParams kp0, int mode, int hi1,
                                                            double* Wout1) {
    constexpr int NV = D + 2;
    constexpr int NX = NV + 3;                 /* S F[q], S r, S (|u.n| + c), S^2 */
    __shared__ double part[NX][MAXS][SC];
    const int tx = threadIdx.x, s = threadIdx.y;
    const int I = blockIdx.x * SC + tx;
    const int n = c.n;
    const bool live = I < n && active(c.pact, c.pid, I);
    const KParams kp = localize(kp0, c.ptab, c.pid, live ? I : 0);
    double W[NV];
    Prim P;
    double cs = 0.0;
    if (live) {
#pragma unroll
        for (int q = 0; q < NV; ++q) W[q] = c.W[q * n + I];
        primitive<D>(kp, W, P);
        cs = sqrt(kp.gamma * P.p / P.rho);
    }
    const double visc = fmax(4.0 / 3.0, kp.gamma / kp.prandtl);
    double x[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) x[k] = 0.0;
    if (live) {
        const int J = c.snbr[s * n + I];
        const int tg = c.stag[s * n + I];
        if (J >= 0 || tg != 0) {
            const double S = c.sS[s * n + I];
            double nn[D];
#pragma unroll
            for (int d = 0; d < D; ++d) nn[d] = c.sn[(d * c.nslot + s) * n + I];
            double WJ[NV], F[NV], Wm[NV];
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
            const double dist = c.sd[s * n + I];
            kfvs_flux<D>(kp, W, WJ, nn, F);
#pragma unroll
            for (int q = 0; q < NV; ++q) x[q] = S * F[q];
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
            reinterpret_cast<T*>(c.r)[s * n + I] = (T)r;
            x[NV] = S * r;
            x[NV + 1] = S * (fabs(un) + cs);
            x[NV + 2] = S * S;
        }
    }
#pragma unroll
    for (int k = 0; k < NX; ++k) part[k][s][tx] = x[k];
    __syncthreads();
    if (s != 0 || !live) return;
    double Res[NV], sr = 0.0, lam = 0.0, s2 = 0.0;
#pragma unroll
    for (int q = 0; q < NV; ++q) Res[q] = 0.0;
    for (int k = 0; k < c.nslot; ++k) {
#pragma unroll
        for (int q = 0; q < NV; ++q) Res[q] -= part[q][k][tx];
        sr += part[NV][k][tx];
        lam += part[NV + 1][k][tx];
        s2 += part[NV + 2][k][tx];
    }
    if (mode == COARSE_FORCING) {
#pragma unroll
        for (int q = 0; q < NV; ++q) c.F[q * n + I] = (double)reinterpret_cast<const T*>(c.Rstar)[q * n + I] - Res[q];
        return;
    }
    if (kp.reynolds > 0.0) lam += visc * sutherland(kp, P.p / P.rho) / P.rho * s2 / c.V[I];
    const double V = c.V[I];
    const double dte = kp.cfl_exp * V / lam, dti = implicit_cfl(kp) * V / lam;
    /* every load before the first store (a load issued after a store waits for it) */
    double rhs[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) rhs[q] = Res[q] + c.F[q * n + I];
    if (mode == COARSE_RHS) fixed_factor_rhs<NV, T>(kp, c, I, V, dti, rhs);
    const double Dd = lusgs_diagonal(kp, c.alpha[I], V, dti, dte, sr);
    c.dte[I] = dte;
    c.dti[I] = dti;
#pragma unroll
    for (int q = 0; q < NV; ++q) c.rhs[q * n + I] = rhs[q];
    c.D[I] = Dd;
    if (I < hi1) {
        T* dW = reinterpret_cast<T*>(c.dW);
        double dWd[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const T d = (T)rhs[q] / (T)Dd;
            dW[q * n + I] = d;
            dWd[q] = (double)d;
        }
        /* a single colour: this is the final correction; write the new state */
        if (Wout1) {
            const double th = update_fraction<D>(W, dWd, kp.update_limit);
#pragma unroll
            for (int q = 0; q < NV; ++q) Wout1[q * n + I] = th > 0.0 ? W[q] + th * dWd[q] : W[q];
        }
    }
}

/* One colour of an LU-SGS sweep with one thread per (cell, face slot); the
 * slot-0 thread combines the neighbour terms in slot order and updates dW. */
template <int D, class T, int SC>
__global__ void __launch_bounds__(SC * MAXS) k_lusgs_s(CoarseDev c, KParams kp, int lo, int hi, int fwd,
                                                       double* Wout);

/* Increment of the normal Euler flux T(W + dW) - T(W).  In FP64 it is the
 * literal difference; in FP32 it is written in terms of the increments so no
 * two large, nearly equal numbers are subtracted (base state from FP64). */
template <int D, class T>
__device__ __forceinline__ void flux_increment(const KParams& kp, const double* W, const T* dW, const T* n, T* dT) {
    constexpr int NV = D + 2;
    if constexpr (sizeof(T) == sizeof(double)) {
        double Wp[NV], T1[NV], T0[NV], nn[D];
#pragma unroll
        for (int q = 0; q < NV; ++q) Wp[q] = W[q] + dW[q];
#pragma unroll
        for (int d = 0; d < D; ++d) nn[d] = n[d];
        euler_flux<D>(kp, Wp, nn, T1);
        euler_flux<D>(kp, W, nn, T0);
#pragma unroll
        for (int q = 0; q < NV; ++q) dT[q] = T1[q] - T0[q];
    } else {
        double ke = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) ke += W[1 + d] * W[1 + d];
        const double pd = (kp.gamma - 1.0) * (W[D + 1] - 0.5 * ke / W[0]);
        const T r = (T)W[0], E = (T)W[D + 1], p = (T)pd, dr = dW[0], dE = dW[D + 1];
        T m[D], dm[D], mn = 0, dmn = 0, m2 = 0, mdm = 0, dm2 = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            m[d] = (T)W[1 + d];
            dm[d] = dW[1 + d];
            mn += m[d] * n[d];
            dmn += dm[d] * n[d];
            m2 += m[d] * m[d];
            mdm += m[d] * dm[d];
            dm2 += dm[d] * dm[d];
        }
        const T inv = (T)1 / (r * (r + dr));
        /* d(X m_n / rho) for a quantity X with increment dX */
        auto dq = [&](T X, T dX) { return (r * (X * dmn + dX * mn + dX * dmn) - dr * X * mn) * inv; };
        const T dke = (r * ((T)2 * mdm + dm2) - dr * m2) * inv;            /* d(|m|^2 / rho) */
        const T dp = (T)(kp.gamma - 1.0) * (dE - (T)0.5 * dke);
        dT[0] = dmn;
#pragma unroll
        for (int d = 0; d < D; ++d) dT[1 + d] = dq(m[d], dm[d]) + dp * n[d];
        dT[D + 1] = dq(E + p, dE + dp);
    }
}

/* One colour of the forward (fwd = 1) or backward sweep (Eqs. gpu-forward/
 * backward-relaxation).  Cells of colour c occupy [lo, hi); lower colours sit
 * below lo and higher colours at or above hi.  T is the type of the
 * correction arithmetic: double (FP64) or float (mixed precision). */
template <int D, class T>
__global__ void __launch_bounds__(CBLOCK) k_lusgs(CoarseDev c, KParams kp, int lo, int hi, int fwd) {
    constexpr int NV = D + 2;
    const int I = lo + blockIdx.x * blockDim.x + threadIdx.x;
    const int n = c.n;
    if (I >= hi || !active(c.pact, c.pid, I)) return;
    T* dW = reinterpret_cast<T*>(c.dW);
    const T* rr = reinterpret_cast<const T*>(c.r);
    T acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0;
    for (int s = 0; s < c.nslot; ++s) {
        const int J = c.snbr[s * n + I];
        if (J < 0) continue;
        if (fwd ? (J >= lo) : (J < hi)) continue;
        const T S = (T)c.sS[s * n + I], r = rr[s * n + I];
        T nn[D], dJ[NV], dT[NV];
        double WJ[NV];
#pragma unroll
        for (int d = 0; d < D; ++d) nn[d] = (T)c.sn[(d * c.nslot + s) * n + I];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            WJ[q] = c.W[q * n + J];
            dJ[q] = dW[q * n + J];
        }
        flux_increment<D, T>(kp, WJ, dJ, nn, dT);
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] += S * (dT[q] - r * dJ[q]);
    }
    const T a = (T)relax_weight(kp, c.alpha[I]);
    const T Di = (T)c.D[I];
    if (fwd) {
#pragma unroll
        for (int q = 0; q < NV; ++q) dW[q * n + I] = ((T)c.rhs[q * n + I] - (T)0.5 * a * acc[q]) / Di;
    } else {
#pragma unroll
        for (int q = 0; q < NV; ++q) dW[q * n + I] -= (T)0.5 * a * acc[q] / Di;
    }
}

template <int D, class T, int SC>
__global__ void __launch_bounds__(SC * MAXS) k_lusgs_s(CoarseDev c, KParams kp, int lo, int hi, int fwd,
                                                       double* Wout) {
    constexpr int NV = D + 2;
    __shared__ T part[NV][MAXS][SC];
    const int tx = threadIdx.x, s = threadIdx.y;
    const int I = lo + blockIdx.x * SC + tx;
    const int n = c.n;
    const bool live = I < hi && active(c.pact, c.pid, I);
    T* dW = reinterpret_cast<T*>(c.dW);
    T x[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) x[q] = 0;
    if (live) {
        const int J = c.snbr[s * n + I];
        if (J >= 0 && (fwd ? (J < lo) : (J >= hi))) {
            const T S = (T)c.sS[s * n + I], r = reinterpret_cast<const T*>(c.r)[s * n + I];
            T nn[D], dJ[NV], dT[NV];
            double WJ[NV];
#pragma unroll
            for (int d = 0; d < D; ++d) nn[d] = (T)c.sn[(d * c.nslot + s) * n + I];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                WJ[q] = c.W[q * n + J];
                dJ[q] = dW[q * n + J];
            }
            flux_increment<D, T>(kp, WJ, dJ, nn, dT);
#pragma unroll
            for (int q = 0; q < NV; ++q) x[q] = S * (dT[q] - r * dJ[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) part[q][s][tx] = x[q];
    __syncthreads();
    if (s != 0 || !live) return;
    T acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0;
    for (int k = 0; k < c.nslot; ++k)
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] += part[q][k][tx];
    const T a = (T)relax_weight(kp, c.alpha[I]);
    const T Di = (T)c.D[I];
    /* every load before the first store (a load issued after a store waits for it) */
    T prev[NV];
    double W[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) prev[q] = fwd ? (T)c.rhs[q * n + I] : dW[q * n + I];
    if (Wout)
#pragma unroll
        for (int q = 0; q < NV; ++q) W[q] = c.W[q * n + I];
    double dWd[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const T d = fwd ? (prev[q] - (T)0.5 * a * acc[q]) / Di : prev[q] - (T)0.5 * a * acc[q] / Di;
        dW[q * n + I] = d;
        dWd[q] = (double)d;
    }
    /* the cell's correction is final: write its new state into the other buffer */
    if (Wout) {
        const double th = update_fraction<D>(W, dWd, kp.update_limit);
#pragma unroll
        for (int q = 0; q < NV; ++q) Wout[q * n + I] = th > 0.0 ? W[q] + th * dWd[q] : W[q];
    }
}

/* Restriction (Sec. 5.2): W0 = sum V W / V_c (FP64), Res* = sum Res (in T),
 * alpha = min.  Eight lanes per coarse cell load its children, consecutive
 * children in consecutive lanes (a coarse cell's children are contiguous in
 * the finer level's order wherever the hierarchy is nested by index, so the
 * loads coalesce), into LDS; the cell's first lane then sums them in child
 * order, the order of a one-thread-per-cell loop.  nchunk = ceil(most
 * children of any coarse cell / 8), the same for every block. */
constexpr int RGRP = 8;
template <int D, class T>
__global__ void __launch_bounds__(CBLOCK) k_restrict(CoarseDev c, const double* Wf, const double* Vf,
                                                   const double* resf, const double* af, int nfine, int nchunk) {
    constexpr int NV = D + 2, NQ = 2 * NV + 2, CPB = CBLOCK / RGRP;
    __shared__ double buf[CPB][RGRP][NQ + 1];
    const int lc = threadIdx.x / RGRP, j = threadIdx.x % RGRP;
    const int I = blockIdx.x * CPB + lc;
    const int n = c.n;
    const bool live = I < n && active(c.pact, c.pid, I);
    const int k0 = live ? c.child_off[I] : 0, k1 = live ? c.child_off[I + 1] : 0;
    double w[NV], amin = 1.0e300;
    T r[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        w[q] = 0.0;
        r[q] = 0;
    }
    for (int ch = 0; ch < nchunk; ++ch) {
        const int k = k0 + ch * RGRP + j;
        if (k < k1) {
            const int i = c.child[k];
            double* b = buf[lc][j];
            b[0] = Vf[i];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                b[1 + q] = Wf[q * nfine + i];
                b[1 + NV + q] = resf[q * nfine + i];
            }
            b[1 + 2 * NV] = af[i];
        }
        __syncthreads();
        if (j == 0) {
            const int m = min(RGRP, k1 - k0 - ch * RGRP);
            for (int jj = 0; jj < m; ++jj) {
                const double* b = buf[lc][jj];
                const double v = b[0];
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    w[q] += v * b[1 + q];
                    r[q] += (T)b[1 + NV + q];
                }
                amin = fmin(amin, b[1 + 2 * NV]);
            }
        }
        __syncthreads();
    }
    if (j != 0 || !live) return;
    const double iv = 1.0 / c.V[I];
    T* Rs = reinterpret_cast<T*>(c.Rstar);
    T* dW = reinterpret_cast<T*>(c.dW);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double w0 = w[q] * iv;
        c.W0[q * n + I] = w0;
        c.W[q * n + I] = w0;
        Rs[q * n + I] = r[q];
        dW[q * n + I] = 0;        /* no previous LU-SGS increment in this cycle */
    }
    c.alpha[I] = amin;
}

/* DF-limited prolongation (Eq. prolongation) with injection; the correction
 * alpha (W - W0) is formed in T and applied through update_fraction; cells
 * that apply less than all of it are counted. */
template <int D, class T>
__global__ void __launch_bounds__(CBLOCK) k_prolong(CoarseDev c, double* Wf, const double* af, int nfine,
                                                  int df, double kappa, unsigned long long* skips) {
    constexpr int NV = D + 2;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nfine) return;
    const int I = c.parent[i];
    if (!active(c.pact, c.pid, I)) return;
    const int n = c.n;
    const T a = df ? (T)af[i] : (T)1;
    double W[NV], dW[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const T dl = (T)(c.W[q * n + I] - c.W0[q * n + I]);
        dW[q] = (double)(a * dl);
        W[q] = Wf[q * nfine + i];
    }
    const double th = update_fraction<D>(W, dW, kappa);
    if (th > 0.0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) Wf[q * nfine + i] = W[q] + th * dW[q];
    }
    if (th < 1.0) atomicAdd(skips, 1ull);
}

/* Coarse LU-SGS update W += theta dW per cell (dW in T). */
template <int D, class T>
__global__ void __launch_bounds__(CBLOCK) k_coarse_add(double* Wc, const double* dWraw, int n, double kappa,
                                                     const int* pid, const int* pact) {
    constexpr int NV = D + 2;
    const T* dWc = reinterpret_cast<const T*>(dWraw);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !active(pact, pid, i)) return;
    double W[NV], dW[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        W[q] = Wc[q * n + i];
        dW[q] = (double)dWc[q * n + i];
    }
    const double th = update_fraction<D>(W, dW, kappa);
    if (th > 0.0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) Wc[q * n + i] = W[q] + th * dW[q];
    }
}

/* Copy the fine state, slopes and DF (three arrays, one launch) to the
 * roll-back buffers while no non-physical state has been flagged. */
/* Start of a V-cycle: count it (the CFL ramp) and save the state unless a
 * previous cycle failed. */
__global__ void __launch_bounds__(BLOCK) k_save_if_ok(const double* a0, double* b0, int m0, const double* a1, double* b1,
                                                      int m1, const double* a2, double* b2, int m2, const int* status,
                                                      int* ncyc) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *ncyc += 1;
    if (*status) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m0) b0[t] = a0[t];
    else if (t < m0 + m1) b1[t - m0] = a1[t - m0];
    else if (t < m0 + m1 + m2) b2[t - m0 - m1] = a2[t - m0 - m1];
}

/* ------------------------------------------------------------- launchers --- */

/* Calls f with std::integral_constant<int, SC> for the slot-parallel block
 * size sc (16, 32 or 64; anything else takes 64). */
template <class F>
static void with_sc(int sc, F&& f) {
    if (sc == 16) f(std::integral_constant<int, 16>{});
    else if (sc == 32) f(std::integral_constant<int, 32>{});
    else f(std::integral_constant<int, 64>{});
}

static inline int nblk(long m) { return (int)((m + BLOCK - 1) / BLOCK); }
static inline int cblk(long m) { return (int)((m + CBLOCK - 1) / CBLOCK); }

static inline int blocks(long m, int b) { return (int)((m + b - 1) / b); }

template <int D, bool HY>
static void fine_kernel(cgks_ctx* c, int which, int block, int mode) {
    FineDev& f = c->fine;
    hipStream_t st = c->stream;
    if (which == 0) {
        /* block = cells per block x face slots x threads per slot */
        using S = Shape<D, HY>;
        const int want = std::min(block ? block : c->blk_recon, RTHREADS / (S::NS * S::TPF));
        const int cells = want <= 16 ? 16 : (want <= 32 || D == 3 ? 32 : 64);
        const dim3 grid(blocks(f.n, cells)), blk(cells * S::NS * S::TPF);
        const size_t lds = RLds<D, HY>::bytes(cells);
        if constexpr (HY) {
            if (cells == 16) k_recon<D, 16, true><<<grid, blk, lds, st>>>(f, c->kp);
            else k_recon<D, 32, true><<<grid, blk, lds, st>>>(f, c->kp);
        } else {
            if (cells == 16) k_recon<D, 16, false><<<grid, blk, lds, st>>>(f, c->kp);
            else if (cells == 32) k_recon<D, 32, false><<<grid, blk, lds, st>>>(f, c->kp);
            else k_recon<D, (D == 2 ? 64 : 32), false><<<grid, blk, lds, st>>>(f, c->kp);
        }
    } else if (which == 1) {
        /* 64 / NG faces per wave */
        constexpr int FPW = 64 / Shape<D, HY>::NG;
        const int b = block ? block : c->blk_flux;
        const long waves = ((long)f.nf + FPW - 1) / FPW;
        /* the residual for restriction uses no slopes (the state at t = dt);
         * inviscid, its flux needs none of their moments */
        const bool lite = (mode & ~FINE_KEEP) == FINE_RESTRICT && !(c->kp.reynolds > 0.0) && !f.pid;
        const bool visc = c->kp.reynolds > 0.0 || f.pid;   /* batches: per-problem Reynolds numbers */
        if (lite) k_flux<D, false, HY, false><<<blocks(waves * 64, b), b, 0, st>>>(f, c->kp);
        else if (!visc) k_flux<D, true, HY, false><<<blocks(waves * 64, b), b, 0, st>>>(f, c->kp);
        else k_flux<D, true, HY, true><<<blocks(waves * 64, b), b, 0, st>>>(f, c->kp);
    } else {
        /* the norm partials use a fixed 256-thread block */
        const int m = mode & ~FINE_KEEP;
        const int b = (m == FINE_STEP_NORM && !f.pid) ? BLOCK : (block ? block : c->blk_gather);
        k_gather<D, HY><<<blocks(f.n, b), b, 0, st>>>(f, c->kp, mode, c->ws.partial, c->ws.status);
    }
}

static void fine_kernel_any(cgks_ctx* c, int which, int block, int mode) {
    if (c->dim == 2) fine_kernel<2, false>(c, which, block, mode);
    else if (c->hybrid) fine_kernel<3, true>(c, which, block, mode);
    else fine_kernel<3, false>(c, which, block, mode);
}

void launch_fine_recon(cgks_ctx* c) { fine_kernel_any(c, 0, 0, FINE_EVAL); }

void launch_fine_kernel(cgks_ctx* c, int which, int block) { fine_kernel_any(c, which, block, FINE_EVAL); }

static void fine_residual(cgks_ctx* c, int mode) {
    FineDev& f = c->fine;
    hipStream_t st = c->stream;
    fine_kernel_any(c, 0, 0, mode);
    fine_kernel_any(c, 1, 0, mode);
    fine_kernel_any(c, 2, 0, mode);
    if ((mode & ~FINE_KEEP) == FINE_STEP_NORM) {
        if (f.pid) {
            k_norm_batch<<<c->ws.nprob, BLOCK, 0, st>>>(f.r2, c->ws.poff, c->ws.ptab, c->ws.history,
                                                         c->ws.history_cap, c->ws.counter, c->ws.nprob);
            k_count<<<1, 64, 0, st>>>(c->ws.counter);
        } else {
            k_norm_finalize<<<1, BLOCK, 0, st>>>(c->ws.partial, nblk(f.n), f.n, c->kp.mach, c->ws.history,
                                                 c->ws.history_cap, c->ws.counter, c->ws.status);
        }
    }
}

void launch_fine_residual(cgks_ctx* c, int mode) { fine_residual(c, mode); }

template <int D, class T>
static void coarse_rhs(cgks_ctx* c, CoarseDev& L, int mode) {
    const int hi1 = mode == COARSE_RHS && L.ncolor > 0 ? L.color_off[1] : 0;
    if (L.nslot <= MAXS) {
        with_sc(L.sc, [&](auto scv) {
            constexpr int SC = decltype(scv)::value;
            k_coarse_rhs_s<D, T, SC><<<blocks(L.n, SC), dim3(SC, L.nslot), 0, c->stream>>>(L, c->kp, mode, hi1,
                                                                                       nullptr);
        });
    } else {
        k_coarse_rhs<D, T><<<cblk(L.n), CBLOCK, 0, c->stream>>>(L, c->kp, mode, hi1);
    }
}

void launch_coarse_rhs(cgks_ctx* c, int level, int mode) {
    CoarseDev& L = c->coarse[level - 1];
    const bool mx = c->p.precision == CGKS_MIXED;
    if (c->dim == 2) mx ? coarse_rhs<2, float>(c, L, mode) : coarse_rhs<2, double>(c, L, mode);
    else mx ? coarse_rhs<3, float>(c, L, mode) : coarse_rhs<3, double>(c, L, mode);
}

template <int D, class T>
static void lusgs(cgks_ctx* c, CoarseDev& L) {
    /* The first colour's forward step is done by the right-hand-side kernel;
     * the last colour's backward step has no higher neighbours (a no-op). */
    for (int pass = 0; pass < 2; ++pass)
        for (int k = 1; k < L.ncolor; ++k) {
            const int col = pass == 0 ? k : L.ncolor - 1 - k;
            const int lo = L.color_off[col], hi = L.color_off[col + 1];
            if (hi <= lo) continue;
            if (L.nslot <= MAXS)
                with_sc(L.sc, [&](auto scv) {
                    constexpr int SC = decltype(scv)::value;
                    k_lusgs_s<D, T, SC><<<blocks(hi - lo, SC), dim3(SC, L.nslot), 0, c->stream>>>(L, c->kp, lo, hi,
                                                                                               pass == 0, nullptr);
                });
            else
                k_lusgs<D, T><<<cblk(hi - lo), CBLOCK, 0, c->stream>>>(L, c->kp, lo, hi, pass == 0);
        }
}

void launch_lusgs(cgks_ctx* c, int level) {
    CoarseDev& L = c->coarse[level - 1];
    const bool mx = c->p.precision == CGKS_MIXED;
    if (c->dim == 2) mx ? lusgs<2, float>(c, L) : lusgs<2, double>(c, L);
    else mx ? lusgs<3, float>(c, L) : lusgs<3, double>(c, L);
}

/* One LU-SGS iteration that reads the state from L.W and writes the new state
 * to Wout: the last colour's forward step and every other colour's backward
 * step write their cells' W + theta dW (the update safeguard) as soon as the
 * correction is final; nothing in the iteration reads Wout. */
template <int D, class T>
static void lusgs_iter_pingpong(cgks_ctx* c, const CoarseDev& L, double* Wout) {
    const int C = L.ncolor;
    const int hi1 = C > 0 ? L.color_off[1] : 0;
    with_sc(L.sc, [&](auto scv) {
        constexpr int SC = decltype(scv)::value;
        k_coarse_rhs_s<D, T, SC><<<blocks(L.n, SC), dim3(SC, L.nslot), 0, c->stream>>>(L, c->kp, COARSE_RHS, hi1,
                                                                                   C == 1 ? Wout : nullptr);
    });
    for (int pass = 0; pass < 2; ++pass)
        for (int k = 1; k < C; ++k) {
            const int col = pass == 0 ? k : C - 1 - k;
            const int lo = L.color_off[col], hi = L.color_off[col + 1];
            if (hi <= lo) continue;
            double* w = (pass == 1 || col == C - 1) ? Wout : nullptr;
            with_sc(L.sc, [&](auto scv) {
                constexpr int SC = decltype(scv)::value;
                k_lusgs_s<D, T, SC><<<blocks(hi - lo, SC), dim3(SC, L.nslot), 0, c->stream>>>(L, c->kp, lo, hi,
                                                                                           pass == 0, w);
            });
        }
}

bool coarse_slot_parallel(const CoarseDev& L) { return L.nslot <= MAXS && L.ncolor >= 1; }

void launch_lusgs_iters(cgks_ctx* c, int level, int n) {
    CoarseDev& L = c->coarse[level - 1];
    if (L.nslot > MAXS || L.ncolor < 1) {
        for (int s = 0; s < n; ++s) {
            launch_coarse_rhs(c, level, COARSE_RHS);
            launch_lusgs(c, level);
            launch_coarse_update(c, level);
        }
        return;
    }
    const bool mx = c->p.precision == CGKS_MIXED;
    double* buf[2] = {L.W, L.Wb};
    for (int s = 0; s < n; ++s) {
        CoarseDev Ls = L;
        Ls.W = buf[s & 1];
        double* out = buf[(s + 1) & 1];
        if (c->dim == 2) mx ? lusgs_iter_pingpong<2, float>(c, Ls, out) : lusgs_iter_pingpong<2, double>(c, Ls, out);
        else mx ? lusgs_iter_pingpong<3, float>(c, Ls, out) : lusgs_iter_pingpong<3, double>(c, Ls, out);
    }
    if (n & 1)
        (void)hipMemcpyAsync(L.W, L.Wb, (size_t)L.n * c->nv * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
}

void launch_coarse_update(cgks_ctx* c, int level) {
    CoarseDev& L = c->coarse[level - 1];
    const bool mx = c->p.precision == CGKS_MIXED;
    const int nb = cblk(L.n);
    const double kap = c->kp.update_limit;
    if (c->dim == 2) {
        if (mx) k_coarse_add<2, float><<<nb, CBLOCK, 0, c->stream>>>(L.W, L.dW, L.n, kap, L.pid, L.pact);
        else k_coarse_add<2, double><<<nb, CBLOCK, 0, c->stream>>>(L.W, L.dW, L.n, kap, L.pid, L.pact);
    } else {
        if (mx) k_coarse_add<3, float><<<nb, CBLOCK, 0, c->stream>>>(L.W, L.dW, L.n, kap, L.pid, L.pact);
        else k_coarse_add<3, double><<<nb, CBLOCK, 0, c->stream>>>(L.W, L.dW, L.n, kap, L.pid, L.pact);
    }
}

void launch_restrict(cgks_ctx* c, int level, const double* Wfine) {
    CoarseDev& G = c->coarse[level];
    const double *Wf, *Vf, *rf, *af;
    int nfine;
    if (level == 0) {
        Wf = Wfine ? Wfine : c->fine.W; Vf = c->fine.V; rf = c->fine.res; af = c->fine.alpha; nfine = c->fine.n;
    } else {
        CoarseDev& F = c->coarse[level - 1];
        Wf = F.W; Vf = F.V; rf = F.rhs; af = F.alpha; nfine = F.n;
    }
    const bool mx = c->p.precision == CGKS_MIXED;
    const int nb = blocks(G.n, CBLOCK / RGRP), nch = (G.maxchild + RGRP - 1) / RGRP;
    if (c->dim == 2) {
        if (mx) k_restrict<2, float><<<nb, CBLOCK, 0, c->stream>>>(G, Wf, Vf, rf, af, nfine, nch);
        else k_restrict<2, double><<<nb, CBLOCK, 0, c->stream>>>(G, Wf, Vf, rf, af, nfine, nch);
    } else {
        if (mx) k_restrict<3, float><<<nb, CBLOCK, 0, c->stream>>>(G, Wf, Vf, rf, af, nfine, nch);
        else k_restrict<3, double><<<nb, CBLOCK, 0, c->stream>>>(G, Wf, Vf, rf, af, nfine, nch);
    }
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
    const bool mx = c->p.precision == CGKS_MIXED;
    const int nb = cblk(nfine), df = c->kp.df_prolong;
    const double kap = c->kp.update_limit;
    unsigned long long* sk = c->ws.skips;
    if (c->dim == 2) {
        if (mx) k_prolong<2, float><<<nb, CBLOCK, 0, c->stream>>>(G, Wf, af, nfine, df, kap, sk);
        else k_prolong<2, double><<<nb, CBLOCK, 0, c->stream>>>(G, Wf, af, nfine, df, kap, sk);
    } else {
        if (mx) k_prolong<3, float><<<nb, CBLOCK, 0, c->stream>>>(G, Wf, af, nfine, df, kap, sk);
        else k_prolong<3, double><<<nb, CBLOCK, 0, c->stream>>>(G, Wf, af, nfine, df, kap, sk);
    }
}

void launch_save_state(cgks_ctx* c) {
    FineDev& f = c->fine;
    const int nv = c->nv, dim = c->dim;
    const int m0 = f.n * nv, m1 = f.n * nv * dim, m2 = f.n;
    k_save_if_ok<<<nblk((long)m0 + m1 + m2), BLOCK, 0, c->stream>>>(f.W, f.Wsave, m0, f.grad, f.gsave, m1, f.alpha,
                                                                    f.asave, m2, c->ws.status, c->ws.ncyc);
}

}  // namespace cgks

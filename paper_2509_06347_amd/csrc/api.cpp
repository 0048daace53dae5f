/*
 * C ABI of libcgks: context, mesh upload, state transfer, the V-cycle
 * sequence (captured once into a hipGraph and replayed), solve loop.
 */
#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdio>

#include "cgks_internal.h"

using namespace cgks;

namespace {

#define HIPCHK(expr)                                           \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return hip_fail(c, e_, #expr);   \
    } while (0)

template <class T>
int dalloc(cgks_ctx* c, T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) return hip_fail(c, e, "hipMalloc");
    c->allocs.push_back((void*)*p);
    return CGKS_OK;
}

template <class T>
int h2d(cgks_ctx* c, T* d, const std::vector<T>& h) {
    if (h.empty()) return CGKS_OK;
    hipError_t e = hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy H2D");
    return CGKS_OK;
}

template <class T>
int d2h(cgks_ctx* c, std::vector<T>& h, const T* d, size_t count) {
    h.resize(count);
    hipError_t e = hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy D2H");
    return CGKS_OK;
}

#define TRY(expr)                  \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ != CGKS_OK) return rc_; \
    } while (0)

void free_device(cgks_ctx* c) {
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->graph_tmpl) (void)hipGraphDestroy(c->graph_tmpl);
    c->graph = nullptr;
    c->graph_tmpl = nullptr;
    for (void* p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
}

}  // namespace

namespace cgks {
void make_kparams(cgks_ctx* c) {
    const cgks_params& p = c->p;
    KParams& k = c->kp;
    k.dim = p.dim;
    k.gamma = p.gamma;
    k.K = 2.0 / (p.gamma - 1.0) - p.dim;
    k.prandtl = p.prandtl;
    k.mach = p.mach;
    k.reynolds = p.reynolds;
    k.mu_inf = p.reynolds > 0.0 ? p.mach / p.reynolds : 0.0;
    k.Tinf = 1.0 / p.gamma;
    k.S_suth = p.sutherland_S_ratio * k.Tinf;
    k.Tw = p.wall_T_ratio * k.Tinf;
    k.cfl_exp = p.cfl_exp;
    k.cfl_imp = p.cfl_imp;
    k.tau_c1 = p.tau_c1;
    k.tau_c2 = p.tau_c2;
    k.g_large = p.weno_gamma_large;
    k.g_small = 1.0 - p.weno_gamma_large;
    k.eps = p.weno_eps;
    k.omega = p.lusgs_omega;
    k.slope_relax = p.slope_relax;
    k.update_limit = p.update_limit;
    k.cfl_ramp = p.cfl_ramp;
    k.relax_beta = p.relax_beta;
    k.df_relax = p.df_relax;
    k.df_prolong = p.df_prolong;
    k.slip_wall_p1 = p.slip_wall_p1;
    const double a = p.aoa_deg * M_PI / 180.0;
    k.u_inf[0] = p.mach * std::cos(a);
    k.u_inf[1] = p.mach * std::sin(a);
    k.u_inf[2] = 0.0;
}
}  // namespace cgks

namespace {

int check_level(cgks_ctx* c, int level) {
    if (!c) return CGKS_EINVAL;
    if (!c->have_mesh) return fail(c, CGKS_EINVAL, "no mesh: call cgks_mesh_setup first");
    if (level < 0 || level >= (int)c->hl.size()) return fail(c, CGKS_EINVAL, "level out of range");
    return CGKS_OK;
}

/* AoS original-order host array <-> SoA internal-order device array. */
void aos_to_soa(const double* in, std::vector<double>& out, int n, int m, const std::vector<int>& perm) {
    out.assign((size_t)n * m, 0.0);
    for (int I = 0; I < n; ++I)
        for (int q = 0; q < m; ++q) out[(size_t)q * n + I] = in[(size_t)perm[I] * m + q];
}

void soa_to_aos(const std::vector<double>& in, double* out, int n, int m, const std::vector<int>& perm) {
    for (int I = 0; I < n; ++I)
        for (int q = 0; q < m; ++q) out[(size_t)perm[I] * m + q] = in[(size_t)q * n + I];
}

int fetch_aos(cgks_ctx* c, const double* dsrc, double* out, int n, int m, const std::vector<int>& perm, int mem) {
    std::vector<double> h;
    TRY(d2h(c, h, dsrc, (size_t)n * m));
    if (mem == CGKS_DEVICE) {
        std::vector<double> a((size_t)n * m);
        soa_to_aos(h, a.data(), n, m, perm);
        hipError_t e = hipMemcpy(out, a.data(), a.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy to caller");
    } else {
        soa_to_aos(h, out, n, m, perm);
    }
    return CGKS_OK;
}

int store_aos(cgks_ctx* c, double* ddst, const double* in, int n, int m, const std::vector<int>& perm, int mem) {
    std::vector<double> a;
    const double* src = in;
    if (mem == CGKS_DEVICE) {
        a.resize((size_t)n * m);
        hipError_t e = hipMemcpy(a.data(), in, a.size() * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy from caller");
        src = a.data();
    }
    std::vector<double> s;
    aos_to_soa(src, s, n, m, perm);
    HIPCHK(hipMemcpyAsync(ddst, s.data(), s.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return CGKS_OK;
}

void enqueue_restrict(cgks_ctx* c, int l) {
    if (l == 0)
        launch_fine_residual(c, FINE_RESTRICT);
    else
        launch_coarse_rhs(c, l, COARSE_EVAL);
    launch_restrict(c, l);
    launch_coarse_rhs(c, l + 1, COARSE_FORCING);
}

/* One V-cycle: fine pre-smoothing, restriction, coarse LU-SGS, prolongation.
 * With shared_residual the last fine step keeps its input state and residual,
 * and those are restricted (no second fine residual evaluation). */
void enqueue_vcycle(cgks_ctx* c) {
    const int nl = (int)c->hl.size();
    const bool shared = c->p.shared_residual && nl > 1;
    launch_save_state(c);
    for (int s = 0; s < c->p.n_pre_fine; ++s) {
        int mode = s == 0 ? FINE_STEP_NORM : FINE_STEP;
        if (shared && s == c->p.n_pre_fine - 1) mode |= FINE_KEEP;
        launch_fine_residual(c, mode);
    }
    for (int l = 0; l + 1 < nl; ++l) {
        if (l == 0 && shared) {
            launch_restrict(c, 0, c->fine.Wpre);
            launch_coarse_rhs(c, 1, COARSE_FORCING);
        } else {
            enqueue_restrict(c, l);
        }
        launch_lusgs_iters(c, l + 1, c->p.n_sweeps);
    }
    for (int l = nl - 2; l >= 0; --l) launch_prolong(c, l);
}

int ensure_history(cgks_ctx* c, int need) {
    if (need <= c->ws.history_cap) return CGKS_OK;
    /* the captured graph refers to the old buffer */
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->graph_tmpl) (void)hipGraphDestroy(c->graph_tmpl);
    c->graph = nullptr;
    c->graph_tmpl = nullptr;
    int cap = std::max(need, 2 * c->ws.history_cap);
    double* h;
    TRY(dalloc(c, &h, cap));
    c->ws.history = h;
    c->ws.history_cap = cap;
    return CGKS_OK;
}

}  // namespace

namespace cgks {

void invalidate_graph(cgks_ctx* c) {
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->graph_tmpl) (void)hipGraphDestroy(c->graph_tmpl);
    c->graph = nullptr;
    c->graph_tmpl = nullptr;
}

int build_graph(cgks_ctx* c) {
    if (c->graph) return CGKS_OK;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    enqueue_vcycle(c);
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamEndCapture(c->stream, &g));
    c->graph_tmpl = g;
    HIPCHK(hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0));
    return CGKS_OK;
}

}  // namespace cgks

namespace {

int restore_saved(cgks_ctx* c) {
    FineDev& f = c->fine;
    const size_t n = f.n, nv = c->nv, d = c->dim;
    HIPCHK(hipMemcpyAsync(f.W, f.Wsave, n * nv * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(f.grad, f.gsave, n * nv * d * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(f.alpha, f.asave, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return CGKS_OK;
}

int set_counters(cgks_ctx* c) {
    static const int zero[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(c->ws.counter, &zero[0], sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->ws.status, &zero[1], sizeof(int), hipMemcpyHostToDevice, c->stream));
    return CGKS_OK;
}

}  // namespace

namespace cgks {

int upload(cgks_ctx* c) {
    free_device(c);
    const int dim = c->dim, nv = c->nv;
    HLevel& H = c->hl[0];
    FineDev& f = c->fine;
    std::memset(&f, 0, sizeof(f));
    f.n = H.n;
    f.nf = (int)H.faces.size();
    f.ngp = c->hybrid ? 4 : (dim == 2) ? 2 : 3;
    f.nslot = H.nslot;
    f.nb = (dim == 2) ? 5 : 9;
    const int n = f.n, nf = f.nf, ng = f.ngp, ns = f.nslot, nq = f.nb;
    const int ncol = ns * (1 + dim);
    std::vector<double> Cs((size_t)dim * n), fn((size_t)dim * nf), fS(nf);
    std::vector<int> sface((size_t)ns * n), snbr((size_t)ns * n), fL(nf), fR(nf), fsl(nf);
    std::vector<int> stag((size_t)ns * n);
    std::vector<double> sS((size_t)ns * n), sn((size_t)dim * ns * n), sX((size_t)ng * dim * ns * n);
    for (int i = 0; i < n; ++i)
        for (int d = 0; d < dim; ++d) Cs[(size_t)d * n + i] = H.C[(size_t)i * dim + d];
    /* device face order: by owner cell L, then by the face's slot in L */
    std::vector<int>& fperm = c->fperm;
    std::vector<int> finv(nf, -1), slotL(nf, 0), slotR(nf, 7);
    fperm.clear();
    for (int i = 0; i < n; ++i)
        for (int s = 0; s < (int)H.cf[i].size(); ++s) {
            const int k = H.cf[i][s];
            if (H.faces[k].L == i) {
                slotL[k] = s;
                finv[k] = (int)fperm.size();
                fperm.push_back(k);
            } else {
                slotR[k] = s;
            }
        }
    if ((int)fperm.size() != nf) return fail(c, CGKS_EMESH, "face without an owner cell");
    /* mixed elements: a triangle's unused fourth Gauss point repeats its first with weight 0 */
    std::vector<double> fX((size_t)nf * ng * dim), fw(c->hybrid ? (size_t)nf * ng : 0);
    for (int e = 0; e < nf; ++e) {
        const HFace& F = H.faces[fperm[e]];
        for (int g = 0; g < ng; ++g) {
            const int gg = g < F.ngp ? g : 0;
            for (int d = 0; d < dim; ++d) fX[((size_t)e * ng + g) * dim + d] = F.gp[gg][d];
            if (c->hybrid) fw[(size_t)e * ng + g] = g < F.ngp ? F.w[g] * F.S : 0.0;
        }
        fL[e] = F.L;
        fR[e] = F.R;
        fS[e] = F.S;
        fsl[e] = slotL[fperm[e]] | (slotR[fperm[e]] << 3);
        for (int d = 0; d < dim; ++d) fn[(size_t)d * nf + e] = F.n[d];
    }
    for (int i = 0; i < n; ++i) {
        const double ih = 1.0 / H.h[i];
        for (int s = 0; s < ns; ++s) {
            const size_t o = (size_t)s * n + i;
            const bool empty = s >= (int)H.cf[i].size();   /* mixed elements with fewer than 6 faces */
            const int k = H.cf[i][empty ? 0 : s];
            const HFace& F = H.faces[k];
            const int side = (F.L == i) ? 0 : 1;
            const double sg = side ? -1.0 : 1.0;
            sface[o] = empty ? -1 : finv[k] * 2 + side;
            snbr[o] = (empty || F.R < 0) ? -1 : (side ? F.L : F.R);
            stag[o] = empty ? -1 : F.R < 0 ? F.tag : 0;
            sS[o] = empty ? 0.0 : F.S;
            /* an empty slot repeats the Gauss points of the cell's first face,
             * an unused fourth point the face's first, so the positivity guard
             * checks no other point */
            for (int d = 0; d < dim; ++d) {
                sn[((size_t)d * ns + s) * n + i] = empty ? 0.0 : sg * F.n[d];
                for (int g = 0; g < ng; ++g)
                    sX[dim == 2 ? (((size_t)g * dim + d) * n + i) * ns + s : (((size_t)g * dim + d) * ns + s) * n + i] =
                        (F.gp[g < F.ngp ? g : 0][d] - H.C[(size_t)i * dim + d]) * ih;
            }
        }
    }
    TRY(dalloc(c, &f.V, n)); TRY(h2d(c, f.V, H.V));
    TRY(dalloc(c, &f.C, (size_t)dim * n)); TRY(h2d(c, f.C, Cs));
    TRY(dalloc(c, &f.h, n)); TRY(h2d(c, f.h, H.h));
    TRY(dalloc(c, &f.mean0, (size_t)nq * n)); TRY(h2d(c, f.mean0, H.mean0));
    TRY(dalloc(c, &f.op, (size_t)nq * ncol * n)); TRY(h2d(c, f.op, H.op));
    TRY(dalloc(c, &f.slot_face, (size_t)ns * n)); TRY(h2d(c, f.slot_face, sface));
    TRY(dalloc(c, &f.slot_nbr, (size_t)ns * n)); TRY(h2d(c, f.slot_nbr, snbr));
    TRY(dalloc(c, &f.slot_tag, (size_t)ns * n)); TRY(h2d(c, f.slot_tag, stag));
    TRY(dalloc(c, &f.slot_S, (size_t)ns * n)); TRY(h2d(c, f.slot_S, sS));
    TRY(dalloc(c, &f.slot_n, (size_t)dim * ns * n)); TRY(h2d(c, f.slot_n, sn));
    TRY(dalloc(c, &f.slot_X, (size_t)ng * dim * ns * n)); TRY(h2d(c, f.slot_X, sX));
    TRY(dalloc(c, &f.fL, nf)); TRY(h2d(c, f.fL, fL));
    TRY(dalloc(c, &f.fR, nf)); TRY(h2d(c, f.fR, fR));
    TRY(dalloc(c, &f.fslot, nf)); TRY(h2d(c, f.fslot, fsl));
    TRY(dalloc(c, &f.fn, (size_t)dim * nf)); TRY(h2d(c, f.fn, fn));
    TRY(dalloc(c, &f.fS, nf)); TRY(h2d(c, f.fS, fS));
    TRY(dalloc(c, &f.W, (size_t)nv * n));
    TRY(dalloc(c, &f.grad, (size_t)nv * dim * n));
    TRY(dalloc(c, &f.alpha, n));
    TRY(dalloc(c, &f.Wsave, (size_t)nv * n));
    TRY(dalloc(c, &f.gsave, (size_t)nv * dim * n));
    TRY(dalloc(c, &f.asave, n));
    TRY(dalloc(c, &f.poly, (size_t)(dim == 2 ? 40 : 80) * n));
    {
        /* the records' static part, written once: basis means, centroid and
         * 1/h after the coefficients [nv][nq + dim] and the cell averages [nv]
         * (the reconstruction writes only those two) */
        const int npr = dim == 2 ? 40 : 80, rmean = nv * (nq + dim) + nv, rcen = rmean + nq, rih = rcen + dim;
        std::vector<double> rec((size_t)npr * n, 0.0);
        for (int i = 0; i < n; ++i) {
            double* r = &rec[(size_t)i * npr];
            for (int m = 0; m < nq; ++m) r[rmean + m] = H.mean0[(size_t)m * n + i];
            for (int d = 0; d < dim; ++d) r[rcen + d] = H.C[(size_t)i * dim + d];
            r[rih] = 1.0 / H.h[i];
        }
        TRY(h2d(c, f.poly, rec));
    }
    TRY(dalloc(c, &f.fX, (size_t)nf * ng * dim)); TRY(h2d(c, f.fX, fX));
    if (c->hybrid) {
        TRY(dalloc(c, &f.fw, (size_t)nf * ng));
        TRY(h2d(c, f.fw, fw));
    }
    TRY(dalloc(c, &f.fout, (size_t)nf * (2 * nv + 1)));
    TRY(dalloc(c, &f.R, (size_t)nv * n));
    TRY(dalloc(c, &f.gnew, (size_t)nv * dim * n));
    TRY(dalloc(c, &f.anew, n));
    TRY(dalloc(c, &f.dt, n));
    TRY(dalloc(c, &f.dti, n));
    TRY(dalloc(c, &f.res, (size_t)nv * n));
    TRY(dalloc(c, &f.Wpre, (size_t)nv * n));
    TRY(dalloc(c, &f.guard, 1));
    HIPCHK(hipMemset(f.guard, 0, sizeof(unsigned long long)));

    c->coarse.assign(c->hl.size() - 1, CoarseDev());
    for (size_t l = 1; l < c->hl.size(); ++l) {
        HLevel& G = c->hl[l];
        HLevel& Fh = c->hl[l - 1];
        CoarseDev& D = c->coarse[l - 1];
        D.n = G.n;
        D.nslot = G.nslot;
        D.ncolor = G.ncolor;
        D.color_off = G.color_off;
        const int m = G.n, S = G.nslot;
        std::vector<int> nb((size_t)S * m, -1), tg((size_t)S * m, 0);
        std::vector<double> sS((size_t)S * m, 0.0), sn((size_t)dim * S * m, 0.0), sd((size_t)S * m, 1.0), V(m);
        for (int I = 0; I < m; ++I) {
            const int o = G.perm[I];
            V[I] = G.V[o];
            for (int s = 0; s < (int)G.cf[o].size(); ++s) {
                const HFace& F = G.faces[G.cf[o][s]];
                const double sg = (F.L == o) ? 1.0 : -1.0;
                sS[(size_t)s * m + I] = F.S;
                for (int d = 0; d < dim; ++d) sn[((size_t)d * S + s) * m + I] = sg * F.n[d];
                double dist = 0.0;
                if (F.R >= 0) {
                    const int j = (F.L == o) ? F.R : F.L;
                    nb[(size_t)s * m + I] = G.iperm[j];
                    for (int d = 0; d < dim; ++d) {
                        const double dx = G.C[(size_t)j * dim + d] - G.C[(size_t)o * dim + d];
                        dist += dx * dx;
                    }
                    sd[(size_t)s * m + I] = std::sqrt(dist);
                } else {
                    tg[(size_t)s * m + I] = F.tag;
                    for (int d = 0; d < dim; ++d) {
                        const double dx = F.xc[d] - G.C[(size_t)o * dim + d];
                        dist += dx * dx;
                    }
                    sd[(size_t)s * m + I] = 2.0 * std::sqrt(dist);
                }
            }
        }
        /* transfers: parent of each finer internal cell, children CSR of finer internal cells */
        const int nfine = Fh.n;
        std::vector<int> par(nfine), coff(m + 1, 0), ch;
        for (int j = 0; j < nfine; ++j) par[j] = G.iperm[Fh.parent[Fh.perm[j]]];
        ch.reserve(nfine);
        for (int I = 0; I < m; ++I) {
            const int o = G.perm[I];
            std::vector<int> kids;
            for (int i : G.children[o]) kids.push_back(Fh.iperm[i]);
            std::sort(kids.begin(), kids.end());
            for (int k : kids) ch.push_back(k);
            coff[I + 1] = (int)ch.size();
            D.maxchild = std::max(D.maxchild, coff[I + 1] - coff[I]);
        }
        TRY(dalloc(c, &D.V, m)); TRY(h2d(c, D.V, V));
        D.C = nullptr;
        TRY(dalloc(c, &D.snbr, (size_t)S * m)); TRY(h2d(c, D.snbr, nb));
        TRY(dalloc(c, &D.stag, (size_t)S * m)); TRY(h2d(c, D.stag, tg));
        TRY(dalloc(c, &D.sS, (size_t)S * m)); TRY(h2d(c, D.sS, sS));
        TRY(dalloc(c, &D.sn, (size_t)dim * S * m)); TRY(h2d(c, D.sn, sn));
        TRY(dalloc(c, &D.sd, (size_t)S * m)); TRY(h2d(c, D.sd, sd));
        for (double** p : {&D.W, &D.Wb, &D.W0, &D.F, &D.Rstar, &D.dW, &D.rhs}) TRY(dalloc(c, p, (size_t)nv * m));
        for (double** p : {&D.alpha, &D.D, &D.dte, &D.dti}) TRY(dalloc(c, p, m));
        TRY(dalloc(c, &D.r, (size_t)S * m));
        TRY(dalloc(c, &D.parent, nfine)); TRY(h2d(c, D.parent, par));
        TRY(dalloc(c, &D.child_off, m + 1)); TRY(h2d(c, D.child_off, coff));
        TRY(dalloc(c, &D.child, nfine)); TRY(h2d(c, D.child, ch));
        HIPCHK(hipMemset(D.F, 0, (size_t)nv * m * sizeof(double)));
        HIPCHK(hipMemset(D.dW, 0, (size_t)nv * m * sizeof(double)));
    }
    Workspace& w = c->ws;
    w = Workspace();
    w.npartial = (n + 255) / 256;
    TRY(dalloc(c, &w.partial, w.npartial));
    TRY(dalloc(c, &w.counter, 1));
    TRY(dalloc(c, &w.ncyc, 1));
    TRY(dalloc(c, &w.status, 1));
    TRY(dalloc(c, &w.skips, 1));
    HIPCHK(hipMemset(w.skips, 0, sizeof(unsigned long long)));
    HIPCHK(hipMemset(w.counter, 0, sizeof(int)));
    HIPCHK(hipMemset(w.ncyc, 0, sizeof(int)));
    HIPCHK(hipMemset(w.status, 0, sizeof(int)));
    c->kp.ncyc = w.ncyc;
    TRY(ensure_history(c, 1024));
    HIPCHK(hipDeviceSynchronize());
    return CGKS_OK;
}

}  // namespace cgks

extern "C" {

void cgks_default_params(cgks_params* p) {
    std::memset(p, 0, sizeof(*p));
    p->dim = 2;
    p->gamma = 1.4;
    p->prandtl = 0.72;
    p->mach = 0.5;
    p->aoa_deg = 0.0;
    p->reynolds = 0.0;
    p->wall_T_ratio = 1.0;
    p->sutherland_S_ratio = 0.5;
    p->cfl_exp = 0.5;
    p->cfl_imp = 10.0;
    p->n_levels = 3;
    p->n_pre_fine = 1;
    p->n_post = 0;
    p->n_sweeps = 6;
    p->df_relax = 1;
    p->df_prolong = 1;
    p->precision = CGKS_FP64;
    p->tau_c1 = 0.01;
    p->tau_c2 = 1.0;
    p->weno_gamma_large = 0.95;
    p->weno_eps = 1e-14;
    p->lusgs_omega = 1.0;
    p->skew_limit = 0.2;
    p->slope_relax = 0.3;
    p->update_limit = 0.5;
    p->cfl_ramp = 0;
    p->relax_beta = 0.5;
    p->shared_residual = 0;
    p->slip_wall_p1 = 0;
}

const char* cgks_strerror(int code) {
    switch (code) {
        case CGKS_OK: return "ok";
        case CGKS_NOTCONV: return "not converged within max_cycles";
        case CGKS_EINVAL: return "invalid argument";
        case CGKS_EMESH: return "invalid mesh";
        case CGKS_EDEVICE: return "HIP device error";
        case CGKS_ENONPHYS: return "non-physical state";
        case CGKS_ELIMIT: return "size beyond a fixed workspace limit";
        default: return "unknown error";
    }
}

const char* cgks_last_error(const cgks_ctx* c) { return c ? c->err.c_str() : "null context"; }

int cgks_create(const cgks_params* p, cgks_ctx** out) {
    if (!p || !out) return CGKS_EINVAL;
    *out = nullptr;
    if (p->dim != 2 && p->dim != 3) return CGKS_EINVAL;
    if (p->n_post != 0 || p->n_pre_fine < 1 || p->n_sweeps < 0 || !(p->mach > 0.0) || !(p->gamma > 1.0))
        return CGKS_EINVAL;
    if (p->precision != CGKS_FP64 && p->precision != CGKS_MIXED) return CGKS_EINVAL;
    if (!(p->slope_relax > 0.0 && p->slope_relax <= 1.0)) return CGKS_EINVAL;
    if (!(p->update_limit <= 1.0)) return CGKS_EINVAL;
    if (p->cfl_ramp < 0) return CGKS_EINVAL;
    if (p->df_relax < 0 || p->df_relax > 3) return CGKS_EINVAL;
    if (!(p->relax_beta >= 0.0 && p->relax_beta <= 1.0)) return CGKS_EINVAL;
    if (p->shared_residual != 0 && p->shared_residual != 1) return CGKS_EINVAL;
    if (p->slip_wall_p1 != 0 && p->slip_wall_p1 != 1) return CGKS_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return CGKS_EDEVICE;
    cgks_ctx* c = new cgks_ctx();
    c->p = *p;
    c->dim = p->dim;
    c->nv = p->dim + 2;
    (void)hipGetDevice(&c->device);
    if (hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return CGKS_EDEVICE;
    }
    c->stream = c->own_stream;
    make_kparams(c);
    *out = c;
    return CGKS_OK;
}

void cgks_destroy(cgks_ctx* c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    free_device(c);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
}

int cgks_set_stream(cgks_ctx* c, void* stream) {
    if (!c) return CGKS_EINVAL;
    c->stream = stream ? (hipStream_t)stream : c->own_stream;
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->graph_tmpl) (void)hipGraphDestroy(c->graph_tmpl);
    c->graph = nullptr;
    c->graph_tmpl = nullptr;
    return CGKS_OK;
}

int cgks_mesh_setup(cgks_ctx* c, const cgks_mesh* m, int n_levels, const int32_t* const* parent) {
    if (!c || !m) return CGKS_EINVAL;
    c->have_mesh = false;
    int rc = setup_host(c, m, n_levels, parent);
    if (rc) return rc;
    rc = upload(c);
    if (rc) return rc;
    c->have_mesh = true;
    return CGKS_OK;
}

int cgks_level_size(cgks_ctx* c, int level, int* n_cells, int* n_faces) {
    TRY(check_level(c, level));
    if (n_cells) *n_cells = c->hl[level].n;
    if (n_faces) *n_faces = (int)c->hl[level].faces.size();
    return CGKS_OK;
}

int cgks_coloring(cgks_ctx* c, int level, int32_t* color_out, int32_t* n_colors) {
    TRY(check_level(c, level));
    const HLevel& H = c->hl[level];
    if (color_out)
        for (int i = 0; i < H.n; ++i) color_out[i] = H.color[i];
    if (n_colors) *n_colors = H.ncolor;
    return CGKS_OK;
}

int cgks_agglomerate(cgks_ctx* c, int level, int32_t* agg_out, int32_t* n_coarse) {
    TRY(check_level(c, level));
    std::vector<int> agg;
    int nc = agglomerate_level(c, level, agg);
    if (agg_out)
        for (size_t i = 0; i < agg.size(); ++i) agg_out[i] = agg[i];
    if (n_coarse) *n_coarse = nc;
    return CGKS_OK;
}

int cgks_cell_geometry(cgks_ctx* c, int level, double* V, double* C) {
    TRY(check_level(c, level));
    const HLevel& H = c->hl[level];
    if (V) std::copy(H.V.begin(), H.V.end(), V);
    if (C) std::copy(H.C.begin(), H.C.end(), C);
    return CGKS_OK;
}

int cgks_init_freestream(cgks_ctx* c) {
    TRY(check_level(c, 0));
    const int nv = c->nv, dim = c->dim;
    double Winf[5];
    Winf[0] = 1.0;
    double ke = 0.0;
    for (int d = 0; d < dim; ++d) {
        Winf[1 + d] = c->kp.u_inf[d];
        ke += c->kp.u_inf[d] * c->kp.u_inf[d];
    }
    Winf[dim + 1] = (1.0 / c->p.gamma) / (c->p.gamma - 1.0) + 0.5 * ke;
    for (size_t l = 0; l < c->hl.size(); ++l) {
        const int n = c->hl[l].n;
        std::vector<double> W((size_t)nv * n), a(n, 1.0);
        for (int q = 0; q < nv; ++q)
            for (int i = 0; i < n; ++i) W[(size_t)q * n + i] = Winf[q];
        if (l == 0) {
            TRY(h2d(c, c->fine.W, W));
            TRY(h2d(c, c->fine.alpha, a));
            HIPCHK(hipMemset(c->fine.grad, 0, (size_t)nv * dim * n * sizeof(double)));
        } else {
            CoarseDev& D = c->coarse[l - 1];
            TRY(h2d(c, D.W, W));
            TRY(h2d(c, D.W0, W));
            TRY(h2d(c, D.alpha, a));
            HIPCHK(hipMemset(D.F, 0, (size_t)nv * n * sizeof(double)));
        }
    }
    HIPCHK(hipMemsetAsync(c->ws.ncyc, 0, sizeof(int), c->stream));
    HIPCHK(hipDeviceSynchronize());
    return CGKS_OK;
}

int cgks_set_state(cgks_ctx* c, const double* W, const double* gradW, const double* alpha, int mem) {
    TRY(check_level(c, 0));
    if (!W) return fail(c, CGKS_EINVAL, "W is NULL");
    const HLevel& H = c->hl[0];
    const int n = H.n, nv = c->nv, dim = c->dim;
    TRY(store_aos(c, c->fine.W, W, n, nv, H.perm, mem));
    if (gradW) {
        TRY(store_aos(c, c->fine.grad, gradW, n, nv * dim, H.perm, mem));
    } else {
        HIPCHK(hipMemset(c->fine.grad, 0, (size_t)nv * dim * n * sizeof(double)));
    }
    if (alpha) {
        TRY(store_aos(c, c->fine.alpha, alpha, n, 1, H.perm, mem));
    } else {
        std::vector<double> a(n, 1.0);
        TRY(h2d(c, c->fine.alpha, a));
    }
    HIPCHK(hipMemsetAsync(c->ws.ncyc, 0, sizeof(int), c->stream));
    HIPCHK(hipDeviceSynchronize());
    return CGKS_OK;
}

int cgks_get_state(cgks_ctx* c, double* W, double* gradW, double* alpha, int mem) {
    TRY(check_level(c, 0));
    const HLevel& H = c->hl[0];
    const int n = H.n, nv = c->nv, dim = c->dim;
    if (W) TRY(fetch_aos(c, c->fine.W, W, n, nv, H.perm, mem));
    if (gradW) TRY(fetch_aos(c, c->fine.grad, gradW, n, nv * dim, H.perm, mem));
    if (alpha) TRY(fetch_aos(c, c->fine.alpha, alpha, n, 1, H.perm, mem));
    return CGKS_OK;
}

int cgks_set_level_state(cgks_ctx* c, int level, const double* W, const double* W0, const double* F,
                         const double* alpha) {
    TRY(check_level(c, level));
    if (level == 0) return cgks_set_state(c, W, nullptr, alpha, CGKS_HOST);
    const HLevel& H = c->hl[level];
    CoarseDev& D = c->coarse[level - 1];
    const int n = H.n, nv = c->nv;
    if (W) TRY(store_aos(c, D.W, W, n, nv, H.perm, CGKS_HOST));
    if (W0) TRY(store_aos(c, D.W0, W0, n, nv, H.perm, CGKS_HOST));
    if (F) TRY(store_aos(c, D.F, F, n, nv, H.perm, CGKS_HOST));
    if (alpha) TRY(store_aos(c, D.alpha, alpha, n, 1, H.perm, CGKS_HOST));
    return CGKS_OK;
}

int cgks_get_level_state(cgks_ctx* c, int level, double* W, double* W0, double* F, double* alpha) {
    TRY(check_level(c, level));
    if (level == 0) return cgks_get_state(c, W, nullptr, alpha, CGKS_HOST);
    const HLevel& H = c->hl[level];
    CoarseDev& D = c->coarse[level - 1];
    const int n = H.n, nv = c->nv;
    if (W) TRY(fetch_aos(c, D.W, W, n, nv, H.perm, CGKS_HOST));
    if (W0) TRY(fetch_aos(c, D.W0, W0, n, nv, H.perm, CGKS_HOST));
    if (F) TRY(fetch_aos(c, D.F, F, n, nv, H.perm, CGKS_HOST));
    if (alpha) TRY(fetch_aos(c, D.alpha, alpha, n, 1, H.perm, CGKS_HOST));
    return CGKS_OK;
}

int cgks_residual(cgks_ctx* c, int level, double* R, double* gradW_new, double* alpha_out, int mem) {
    TRY(check_level(c, level));
    const HLevel& H = c->hl[level];
    const int n = H.n, nv = c->nv, dim = c->dim;
    if (level == 0) {
        launch_fine_residual(c, FINE_EVAL);
        HIPCHK(hipGetLastError());
        if (R) TRY(fetch_aos(c, c->fine.R, R, n, nv, H.perm, mem));
        if (gradW_new) TRY(fetch_aos(c, c->fine.gnew, gradW_new, n, nv * dim, H.perm, mem));
        if (alpha_out) TRY(fetch_aos(c, c->fine.anew, alpha_out, n, 1, H.perm, mem));
        return CGKS_OK;
    }
    CoarseDev& D = c->coarse[level - 1];
    launch_coarse_rhs(c, level, COARSE_EVAL);
    HIPCHK(hipGetLastError());
    if (R) {
        std::vector<double> h;
        TRY(d2h(c, h, D.rhs, (size_t)nv * n));
        for (double& v : h) v = -v;
        if (mem == CGKS_DEVICE) {
            std::vector<double> a((size_t)n * nv);
            soa_to_aos(h, a.data(), n, nv, H.perm);
            HIPCHK(hipMemcpy(R, a.data(), a.size() * sizeof(double), hipMemcpyHostToDevice));
        } else {
            soa_to_aos(h, R, n, nv, H.perm);
        }
    }
    if (alpha_out) TRY(fetch_aos(c, D.alpha, alpha_out, n, 1, H.perm, mem));
    return CGKS_OK;
}

int cgks_time_steps(cgks_ctx* c, int level, double* dt_exp, double* dt_imp) {
    TRY(check_level(c, level));
    const HLevel& H = c->hl[level];
    const int n = H.n;
    const double *de, *di;
    if (level == 0) {
        launch_fine_recon(c);
        de = c->fine.dt;
        di = c->fine.dti;
    } else {
        launch_coarse_rhs(c, level, COARSE_EVAL);
        de = c->coarse[level - 1].dte;
        di = c->coarse[level - 1].dti;
    }
    HIPCHK(hipGetLastError());
    if (dt_exp) TRY(fetch_aos(c, de, dt_exp, n, 1, H.perm, CGKS_HOST));
    if (dt_imp) TRY(fetch_aos(c, di, dt_imp, n, 1, H.perm, CGKS_HOST));
    return CGKS_OK;
}

int cgks_smooth(cgks_ctx* c, int level, int n) {
    TRY(check_level(c, level));
    if (level == 0) {
        for (int s = 0; s < n; ++s) launch_fine_residual(c, FINE_STEP);
    } else if (n > 0) {
        launch_lusgs_iters(c, level, n);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return CGKS_OK;
}

int cgks_restrict(cgks_ctx* c, int level) {
    TRY(check_level(c, level));
    if (level + 1 >= (int)c->hl.size()) return fail(c, CGKS_EINVAL, "no coarser level");
    enqueue_restrict(c, level);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return CGKS_OK;
}

int cgks_prolong(cgks_ctx* c, int level) {
    TRY(check_level(c, level));
    if (level + 1 >= (int)c->hl.size()) return fail(c, CGKS_EINVAL, "no coarser level");
    launch_prolong(c, level);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return CGKS_OK;
}

int cgks_run_cycles(cgks_ctx* c, int ncyc, double* history) {
    TRY(check_level(c, 0));
    if (ncyc < 0) return fail(c, CGKS_EINVAL, "negative cycle count");
    if (ncyc == 0) return CGKS_OK;
    TRY(ensure_history(c, ncyc));
    TRY(build_graph(c));
    TRY(set_counters(c));
    for (int k = 0; k < ncyc; ++k) HIPCHK(hipGraphLaunch(c->graph, c->stream));
    int status = 0;
    HIPCHK(hipMemcpyAsync(&status, c->ws.status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    if (history) HIPCHK(hipMemcpyAsync(history, c->ws.history, ncyc * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->cycles_done += ncyc;
    if (status) {
        TRY(restore_saved(c));
        return fail(c, CGKS_ENONPHYS, "non-physical state (NaN, rho <= 0 or p <= 0); state rolled back");
    }
    return CGKS_OK;
}

int cgks_vcycle(cgks_ctx* c, double* norm_out) {
    double h = 0.0;
    int rc = cgks_run_cycles(c, 1, &h);
    if (norm_out) *norm_out = h;
    return rc;
}

int cgks_solve(cgks_ctx* c, double tol, int max_cycles, int* cycles_out, double* history, int history_cap) {
    TRY(check_level(c, 0));
    if (max_cycles < 0) return fail(c, CGKS_EINVAL, "negative cycle count");
    if (cycles_out) *cycles_out = 0;
    int done = 0;
    int chunk = 8;
    std::vector<double> h;
    while (done < max_cycles) {
        const int k = std::min(chunk, max_cycles - done);
        h.assign(k, 0.0);
        int rc = cgks_run_cycles(c, k, h.data());
        for (int j = 0; j < k; ++j) {
            if (history && done + j < history_cap) history[done + j] = h[j];
            if (h[j] <= tol) {
                if (cycles_out) *cycles_out = done + j + 1;
                return rc;
            }
        }
        done += k;
        if (cycles_out) *cycles_out = done;
        if (rc) return rc;
        chunk = std::min(64, chunk * 2);
    }
    return CGKS_NOTCONV;
}

int cgks_time_kernel(cgks_ctx* c, int kernel, int reps, double* avg_ms, int64_t* work_items) {
    TRY(check_level(c, 0));
    if (kernel < 0 || kernel > 2 || reps <= 0) return fail(c, CGKS_EINVAL, "kernel must be 0..2 and reps > 0");
    /* Each repetition runs the whole fine residual (reconstruction, flux,
     * gather) as a V-cycle does, so caches hold what they hold there; only the
     * chosen kernel lies between the two events of a repetition. */
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (int k = 0; k < 3; ++k) launch_fine_kernel(c, k);   /* warm-up */
    double ms = 0.0;
    for (int r = 0; r < reps; ++r) {
        for (int k = 0; k < 3; ++k) {
            if (k == kernel) HIPCHK(hipEventRecord(e0, c->stream));
            launch_fine_kernel(c, k);
            if (k == kernel) HIPCHK(hipEventRecord(e1, c->stream));
        }
        HIPCHK(hipEventSynchronize(e1));
        float one = 0.0f;
        HIPCHK(hipEventElapsedTime(&one, e0, e1));
        ms += one;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (avg_ms) *avg_ms = ms / reps;
    if (work_items) *work_items = (kernel == 1) ? (int64_t)c->fine.nf * c->fine.ngp : (int64_t)c->fine.n;
    return CGKS_OK;
}

int cgks_stats(cgks_ctx* c, int64_t* guard_hits, int64_t* prolong_skips) {
    TRY(check_level(c, 0));
    unsigned long long g = 0, s = 0;
    HIPCHK(hipMemcpy(&g, c->fine.guard, sizeof(g), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&s, c->ws.skips, sizeof(s), hipMemcpyDeviceToHost));
    if (guard_hits) *guard_hits = (int64_t)g;
    if (prolong_skips) *prolong_skips = (int64_t)s;
    return CGKS_OK;
}

}  // extern "C"

/* ------------------------------------------------------------- autotune --- */

extern "C" int cgks_autotune(cgks_ctx* c) {
    TRY(check_level(c, 0));
    /* statistics counters, restored at the end: the timed launches below may
     * advance them (positivity guard, update safeguard) */
    unsigned long long guard = 0, skips = 0;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(&guard, c->fine.guard, sizeof(guard), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&skips, c->ws.skips, sizeof(skips), hipMemcpyDeviceToHost));
    /* launch shape of each fine kernel: the fastest candidate at the current state */
    static const int cand[3][3] = {{16, 32, 64}, {64, 128, 256}, {64, 128, 256}};  /* recon: cells per block */
    int best[3] = {c->blk_recon, c->blk_flux, c->blk_gather};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (int which = 0; which < 3; ++which) {
        float tbest = 1e30f;
        for (int j = 0; j < 3 && cand[which][j]; ++j) {
            const int b = cand[which][j];
            for (int k = 0; k < which; ++k) launch_fine_kernel(c, k, 0);
            launch_fine_kernel(c, which, b);
            HIPCHK(hipEventRecord(e0, c->stream));
            for (int r = 0; r < 5; ++r) launch_fine_kernel(c, which, b);
            HIPCHK(hipEventRecord(e1, c->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < tbest) {
                tbest = ms;
                best[which] = b;
            }
        }
    }
    c->blk_recon = best[0];
    c->blk_flux = best[1];
    c->blk_gather = best[2];
    /* cells per block of each coarse level's slot-parallel kernels: the fastest
     * over three LU-SGS iterations at the level's current state (the coarse
     * states are overwritten by the next restriction) */
    for (size_t l = 1; l < c->hl.size(); ++l) {
        CoarseDev& L = c->coarse[l - 1];
        if (!coarse_slot_parallel(L)) continue;
        float tbest = 1e30f;
        int sbest = L.sc;
        for (int sc : {16, 32, 64}) {
            L.sc = sc;
            launch_lusgs_iters(c, (int)l, 1);
            HIPCHK(hipEventRecord(e0, c->stream));
            launch_lusgs_iters(c, (int)l, 3);
            HIPCHK(hipEventRecord(e1, c->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < tbest) {
                tbest = ms;
                sbest = sc;
            }
        }
        L.sc = sbest;
    }
    HIPCHK(hipMemcpy(c->fine.guard, &guard, sizeof(guard), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->ws.skips, &skips, sizeof(skips), hipMemcpyHostToDevice));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    invalidate_graph(c);
    return CGKS_OK;
}

extern "C" int cgks_launch_shapes(cgks_ctx* c, int* recon, int* flux, int* gather) {
    if (!c) return CGKS_EINVAL;
    if (recon) *recon = c->blk_recon;
    if (flux) *flux = c->blk_flux;
    if (gather) *gather = c->blk_gather;
    return CGKS_OK;
}

extern "C" int cgks_set_coarse_shapes(cgks_ctx* c, const int* cells_per_block, int n) {
    if (!c || n < 0 || (n > 0 && !cells_per_block)) return CGKS_EINVAL;
    for (int l = 0; l < n; ++l) {
        const int v = cells_per_block[l];
        if (v != 16 && v != 32 && v != 64) return fail(c, CGKS_EINVAL, "cells per block must be 16, 32 or 64");
    }
    for (int l = 0; l < n && l < (int)c->coarse.size(); ++l) c->coarse[l].sc = cells_per_block[l];
    invalidate_graph(c);
    return CGKS_OK;
}

extern "C" int cgks_coarse_shapes(cgks_ctx* c, int* cells_per_block, int n) {
    if (!c || n < 0 || (n > 0 && !cells_per_block)) return CGKS_EINVAL;
    for (int l = 0; l < n; ++l)
        cells_per_block[l] = l < (int)c->coarse.size() && coarse_slot_parallel(c->coarse[l]) ? c->coarse[l].sc : 0;
    return CGKS_OK;
}

/* --------------------------------------------------------------- batches --- */

struct cgks_batch {
    std::vector<cgks_ctx*> probs;
    cgks_ctx* m = nullptr;                 /* merged (disjoint-union) context */
    std::vector<std::vector<int>> coff;    /* [level][b] cell offsets, size nprob+1 */
    int cap = 256;
};

namespace {

bool same_shared_params(const cgks_params& a, const cgks_params& b) {
    return a.dim == b.dim && a.gamma == b.gamma && a.prandtl == b.prandtl &&
           a.sutherland_S_ratio == b.sutherland_S_ratio && a.cfl_exp == b.cfl_exp && a.cfl_imp == b.cfl_imp &&
           a.n_levels == b.n_levels && a.n_pre_fine == b.n_pre_fine && a.n_post == b.n_post &&
           a.n_sweeps == b.n_sweeps && a.df_relax == b.df_relax && a.df_prolong == b.df_prolong &&
           a.precision == b.precision && a.tau_c1 == b.tau_c1 && a.tau_c2 == b.tau_c2 &&
           a.weno_gamma_large == b.weno_gamma_large && a.weno_eps == b.weno_eps &&
           a.lusgs_omega == b.lusgs_omega && a.slope_relax == b.slope_relax &&
           a.update_limit == b.update_limit && a.cfl_ramp == b.cfl_ramp && a.relax_beta == b.relax_beta &&
           a.shared_residual == b.shared_residual &&
           a.slip_wall_p1 == b.slip_wall_p1 &&
           ((a.reynolds > 0.0) == (b.reynolds > 0.0));
}

/* Copy a [rows][n_b] SoA block between a problem and the merged arrays. */
int copy_rows(cgks_ctx* c, double* dst, size_t dpitch, const double* src, size_t spitch, size_t n, size_t rows) {
    HIPCHK(hipMemcpy2DAsync(dst, dpitch * sizeof(double), src, spitch * sizeof(double), n * sizeof(double), rows,
                            hipMemcpyDeviceToDevice, c->stream));
    return CGKS_OK;
}

int batch_state(cgks_batch* B, bool to_merged) {
    cgks_ctx* m = B->m;
    const size_t N = m->fine.n, nv = m->nv, dim = m->dim;
    for (size_t b = 0; b < B->probs.size(); ++b) {
        cgks_ctx* p = B->probs[b];
        const size_t off = B->coff[0][b], n = p->fine.n;
        struct { double* pm; double* pp; size_t rows; } arr[3] = {
            {m->fine.W + off, p->fine.W, nv}, {m->fine.grad + off, p->fine.grad, nv * dim}, {m->fine.alpha + off, p->fine.alpha, 1}};
        for (auto& a : arr) {
            if (to_merged) TRY(copy_rows(m, a.pm, N, a.pp, n, n, a.rows));
            else TRY(copy_rows(m, a.pp, n, a.pm, N, n, a.rows));
        }
    }
    cgks_ctx* c = m;
    HIPCHK(hipStreamSynchronize(m->stream));
    return CGKS_OK;
}

}  // namespace

extern "C" {

int cgks_batch_create(int n, cgks_ctx* const* probs, cgks_batch** out) {
    if (n <= 0 || !probs || !out) return CGKS_EINVAL;
    *out = nullptr;
    for (int b = 0; b < n; ++b) {
        if (!probs[b] || !probs[b]->have_mesh) return CGKS_EINVAL;
        if (!same_shared_params(probs[0]->p, probs[b]->p)) return CGKS_EINVAL;
        if (probs[b]->hybrid) return CGKS_EINVAL;   /* batches take simplex meshes */
    }
    cgks_batch* B = new cgks_batch();
    B->probs.assign(probs, probs + n);
    cgks_ctx* m = new cgks_ctx();
    B->m = m;
    m->p = probs[0]->p;
    m->dim = probs[0]->dim;
    m->nv = probs[0]->nv;
    (void)hipGetDevice(&m->device);
    if (hipStreamCreateWithFlags(&m->own_stream, hipStreamNonBlocking) != hipSuccess) {
        cgks_batch_destroy(B);
        return CGKS_EDEVICE;
    }
    m->stream = m->own_stream;
    make_kparams(m);
    const int L = m->p.n_levels, dim = m->dim;
    m->hl.assign(L, HLevel());
    B->coff.assign(L, std::vector<int>(n + 1, 0));
    for (int l = 0; l < L; ++l)
        for (int b = 0; b < n; ++b) B->coff[l][b + 1] = B->coff[l][b] + probs[b]->hl[l].n;
    for (int l = 0; l < L; ++l) {
        HLevel& M = m->hl[l];
        M.n = B->coff[l][n];
        int fo = 0;
        for (int b = 0; b < n; ++b) {
            const HLevel& H = probs[b]->hl[l];
            const int co = B->coff[l][b];
            M.V.insert(M.V.end(), H.V.begin(), H.V.end());
            M.C.insert(M.C.end(), H.C.begin(), H.C.end());
            for (HFace f : H.faces) {
                f.L += co;
                if (f.R >= 0) f.R += co;
                M.faces.push_back(f);
            }
            for (const auto& lst : H.cf) {
                std::vector<int> v(lst);
                for (int& x : v) x += fo;
                M.cf.push_back(v);
            }
            fo += (int)H.faces.size();
            M.color.insert(M.color.end(), H.color.begin(), H.color.end());
            M.ncolor = std::max(M.ncolor, H.ncolor);
            M.nslot = std::max(M.nslot, H.nslot);
            if (l + 1 < L)
                for (int x : H.parent) M.parent.push_back(x + B->coff[l + 1][b]);
            if (l > 0)
                for (const auto& ch : H.children) {
                    std::vector<int> v(ch);
                    for (int& x : v) x += B->coff[l - 1][b];
                    M.children.push_back(v);
                }
            if (l == 0) {
                M.h.insert(M.h.end(), H.h.begin(), H.h.end());
                M.nbasis.insert(M.nbasis.end(), H.nbasis.begin(), H.nbasis.end());
            }
        }
        if (l == 0) {
            /* SoA re-layout of the per-cell operator and basis means */
            const size_t N = M.n;
            const size_t nq = (dim == 2) ? 5 : 9, ncol = (size_t)(dim + 1) * (1 + dim);
            M.mean0.assign(nq * N, 0.0);
            M.op.assign(nq * ncol * N, 0.0);
            for (int b = 0; b < n; ++b) {
                const HLevel& H = probs[b]->hl[0];
                const size_t nb = H.n, co = B->coff[0][b];
                for (size_t r = 0; r < nq; ++r)
                    std::copy(H.mean0.begin() + r * nb, H.mean0.begin() + (r + 1) * nb, M.mean0.begin() + r * N + co);
                for (size_t r = 0; r < nq * ncol; ++r)
                    std::copy(H.op.begin() + r * nb, H.op.begin() + (r + 1) * nb, M.op.begin() + r * N + co);
            }
        }
        M.perm.resize(M.n);
        for (int i = 0; i < M.n; ++i) M.perm[i] = i;
        if (l > 0)
            std::stable_sort(M.perm.begin(), M.perm.end(), [&](int a, int b2) { return M.color[a] < M.color[b2]; });
        M.iperm.resize(M.n);
        for (int i = 0; i < M.n; ++i) M.iperm[M.perm[i]] = i;
        M.color_off.assign(M.ncolor + 1, 0);
        for (int i = 0; i < M.n; ++i) M.color_off[M.color[i]]++;
        for (int k = 1; k <= M.ncolor; ++k) M.color_off[k] += M.color_off[k - 1];
    }
    cgks_ctx* c = m;  /* for the HIPCHK / TRY macros */
    int rc = upload(m);
    if (rc) {
        cgks_batch_destroy(B);
        return rc;
    }
    m->have_mesh = true;
    /* problem ids and the per-problem parameter table */
    std::vector<double> tab((size_t)PTAB * n);
    for (int b = 0; b < n; ++b) {
        const KParams& k = probs[b]->kp;
        const double t[PTAB] = {k.mach, k.reynolds, k.mu_inf, k.Tw, k.u_inf[0], k.u_inf[1], k.u_inf[2]};
        for (int j = 0; j < PTAB; ++j) tab[(size_t)PTAB * b + j] = t[j];
    }
    auto owner = [&](int l, int orig) {
        return (int)(std::upper_bound(B->coff[l].begin(), B->coff[l].end(), orig) - B->coff[l].begin()) - 1;
    };
    double* dtab;
    int *pid, *fpid, *poff;
    double* r2;
    if ((rc = dalloc(c, &dtab, tab.size())) || (rc = h2d(c, dtab, tab))) {
        cgks_batch_destroy(B);
        return rc;
    }
    std::vector<int> hp(m->hl[0].n), hf(m->hl[0].faces.size());
    for (int i = 0; i < m->hl[0].n; ++i) hp[i] = owner(0, i);
    for (size_t f = 0; f < hf.size(); ++f) hf[f] = owner(0, m->hl[0].faces[m->fperm[f]].L);
    if ((rc = dalloc(c, &pid, hp.size())) || (rc = h2d(c, pid, hp)) || (rc = dalloc(c, &fpid, hf.size())) ||
        (rc = h2d(c, fpid, hf)) || (rc = dalloc(c, &poff, n + 1)) || (rc = h2d(c, poff, B->coff[0])) ||
        (rc = dalloc(c, &r2, m->hl[0].n))) {
        cgks_batch_destroy(B);
        return rc;
    }
    int* pact;
    if ((rc = dalloc(c, &pact, n)) || (rc = h2d(c, pact, std::vector<int>(n, 1)))) {
        cgks_batch_destroy(B);
        return rc;
    }
    m->ws.pactive = pact;
    m->fine.pid = pid;
    m->fine.fpid = fpid;
    m->fine.ptab = dtab;
    m->fine.r2 = r2;
    m->fine.pact = pact;
    for (int l = 1; l < L; ++l) {
        const HLevel& H = m->hl[l];
        std::vector<int> cp(H.n);
        for (int I = 0; I < H.n; ++I) cp[I] = owner(l, H.perm[I]);
        int* d;
        if ((rc = dalloc(c, &d, cp.size())) || (rc = h2d(c, d, cp))) {
            cgks_batch_destroy(B);
            return rc;
        }
        m->coarse[l - 1].pid = d;
        m->coarse[l - 1].ptab = dtab;
        m->coarse[l - 1].pact = pact;
    }
    m->ws.nprob = n;
    m->ws.poff = poff;
    m->ws.ptab = dtab;
    double* hist;
    if ((rc = dalloc(c, &hist, (size_t)n * B->cap))) {
        cgks_batch_destroy(B);
        return rc;
    }
    m->ws.history = hist;
    m->ws.history_cap = B->cap;
    if ((rc = batch_state(B, true))) {
        cgks_batch_destroy(B);
        return rc;
    }
    *out = B;
    return CGKS_OK;
}

int cgks_batch_autotune(cgks_batch* B) {
    if (!B) return CGKS_EINVAL;
    return cgks_autotune(B->m);
}

int cgks_batch_run_cycles(cgks_batch* B, int ncyc, double* history) {
    if (!B || ncyc < 0) return CGKS_EINVAL;
    if (ncyc == 0) return CGKS_OK;
    cgks_ctx* c = B->m;
    const int n = (int)B->probs.size();
    TRY(build_graph(c));
    TRY(h2d(c, c->ws.pactive, std::vector<int>(n, 1)));   /* every member cycles */
    std::vector<double> h((size_t)n * B->cap);
    int done = 0;
    while (done < ncyc) {
        const int k = std::min(B->cap, ncyc - done);
        TRY(set_counters(c));
        for (int j = 0; j < k; ++j) HIPCHK(hipGraphLaunch(c->graph, c->stream));
        if (history) {
            HIPCHK(hipMemcpyAsync(h.data(), c->ws.history, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            for (int b = 0; b < n; ++b)
                for (int j = 0; j < k; ++j) history[(size_t)b * ncyc + done + j] = h[(size_t)b * B->cap + j];
        }
        done += k;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    int st = 0;
    HIPCHK(hipMemcpy(&st, c->ws.status, sizeof(int), hipMemcpyDeviceToHost));
    return st ? CGKS_ENONPHYS : CGKS_OK;
}

int cgks_batch_solve(cgks_batch* B, double tol, int max_cycles, int* cycles_out, int* status_out) {
    if (!B || max_cycles < 0) return CGKS_EINVAL;
    cgks_ctx* c = B->m;
    const int n = (int)B->probs.size();
    TRY(build_graph(c));
    std::vector<int> conv(n, -1), bad(n, 0), act(n, 1);
    std::vector<double> h((size_t)n * B->cap);
    TRY(h2d(c, c->ws.pactive, act));
    int done = 0, chunk = 8;
    while (done < max_cycles) {
        const int k = std::min(std::min(chunk, B->cap), max_cycles - done);
        TRY(set_counters(c));
        for (int j = 0; j < k; ++j) HIPCHK(hipGraphLaunch(c->graph, c->stream));
        HIPCHK(hipMemcpyAsync(h.data(), c->ws.history, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        bool all = true, changed = false;
        for (int b = 0; b < n; ++b) {
            if (!act[b]) continue;
            for (int j = 0; j < k; ++j) {
                const double v = h[(size_t)b * B->cap + j];
                if (!std::isfinite(v)) bad[b] = 1;
                if (conv[b] < 0 && v <= tol) conv[b] = done + j + 1;
            }
            if (conv[b] < 0 && !bad[b]) all = false;
            else {
                act[b] = 0;           /* converged or failed: frozen from the next chunk on */
                changed = true;
            }
        }
        done += k;
        if (all) break;
        if (changed) TRY(h2d(c, c->ws.pactive, act));
        chunk = std::min(64, chunk * 2);
    }
    TRY(batch_state(B, false));
    int rc = CGKS_OK;
    for (int b = 0; b < n; ++b) {
        if (cycles_out) cycles_out[b] = conv[b] >= 0 ? conv[b] : done;
        const int s = bad[b] ? CGKS_ENONPHYS : (conv[b] >= 0 ? CGKS_OK : CGKS_NOTCONV);
        if (status_out) status_out[b] = s;
        if (s == CGKS_ENONPHYS) rc = CGKS_ENONPHYS;
        else if (s == CGKS_NOTCONV && rc == CGKS_OK) rc = CGKS_NOTCONV;
    }
    return rc;
}

int cgks_batch_get_state(cgks_batch* B) {
    if (!B) return CGKS_EINVAL;
    return batch_state(B, false);
}

void cgks_batch_destroy(cgks_batch* B) {
    if (!B) return;
    if (B->m) cgks_destroy(B->m);
    delete B;
}

}  // extern "C"

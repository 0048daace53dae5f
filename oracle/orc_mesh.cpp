/*
 * CPU oracle -- mesh, levels, colouring, agglomeration, reconstruction
 * operators (TEST INFRASTRUCTURE ONLY; see orc.h).
 */
#include "orc_internal.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <tuple>

namespace orc {

int n_quad_basis(int dim) { return dim == 2 ? 5 : 9; }

void basis_exps(int dim, int k, int* e) {
    static const int e2[5][2] = {{1, 0}, {0, 1}, {2, 0}, {1, 1}, {0, 2}};
    static const int e3[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {1, 1, 0},
                                 {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
    for (int d = 0; d < 3; ++d) e[d] = 0;
    for (int d = 0; d < dim; ++d) e[d] = (dim == 2) ? e2[k][d] : e3[k][d];
}

/* Scaled monomial ((x-x0)/h)^e of Sec. 3.1. */
double basis_eval(int dim, int k, const double* x, const double* x0, double h) {
    int e[3];
    basis_exps(dim, k, e);
    double v = 1.0;
    for (int d = 0; d < dim; ++d)
        for (int i = 0; i < e[d]; ++i) v *= (x[d] - x0[d]) / h;
    return v;
}

double basis_deriv(int dim, int k, const int* l, const double* x, const double* x0, double h) {
    int e[3];
    basis_exps(dim, k, e);
    double v = 1.0;
    for (int d = 0; d < dim; ++d) {
        if (l[d] > e[d]) return 0.0;
        for (int i = 0; i < l[d]; ++i) v *= (double)(e[d] - i) / h;
        for (int i = 0; i < e[d] - l[d]; ++i) v *= (x[d] - x0[d]) / h;
    }
    return v;
}

/* Local faces of the 3-D element types (Sec. 2.2: 4, 5, 5 and 6 faces) as
 * node cycles of the input node order: tetrahedron face k is the one
 * opposite node k; pyramid: the base, then the four triangles; prism: the
 * two triangles, then the three quadrilaterals; hexahedron: the two
 * quadrilaterals given first and last, then the four sides. */
const ElemFaces* elem_faces(int nnodes) {
    static const ElemFaces tet = {4, {3, 3, 3, 3, 0, 0}, {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}}};
    static const ElemFaces pyr = {5, {4, 3, 3, 3, 3, 0},
                                  {{0, 1, 2, 3}, {0, 1, 4}, {1, 2, 4}, {2, 3, 4}, {3, 0, 4}}};
    static const ElemFaces pri = {5, {3, 3, 4, 4, 4, 0},
                                  {{0, 1, 2}, {3, 4, 5}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}}};
    static const ElemFaces hex = {6, {4, 4, 4, 4, 4, 4},
                                  {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}}};
    switch (nnodes) {
        case 4: return &tet;
        case 5: return &pyr;
        case 6: return &pri;
        case 8: return &hex;
        default: return nullptr;
    }
}

/* A mixed element with planar faces is the union of the cones from the
 * average of its nodes to the triangles of its faces (quadrilateral a, b, c,
 * d: triangles a, b, c and a, c, d).  Volume and centroid are the sums over
 * the cones; the average rule is the symmetric 4-point rule of every cone
 * (exact for quadratics) weighted by the cone's share of the volume. */
void mixed_cell(const orc_ctx* c, int cell, double* Vout, double* Cout, std::vector<double>* pts,
                std::vector<double>* wts) {
    const Level& L0 = c->lv[0];
    const int* nd = &L0.nodes[L0.noff[cell]];
    const int nn = L0.noff[cell + 1] - L0.noff[cell];
    const ElemFaces* ef = elem_faces(nn);
    const double* X = c->coords.data();
    double xm[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < nn; ++j)
        for (int d = 0; d < 3; ++d) xm[d] += X[nd[j] * 3 + d];
    for (int d = 0; d < 3; ++d) xm[d] /= nn;
    std::vector<std::array<double, 12>> cone;   /* apex xm, then a, b, e */
    std::vector<double> vol;
    double V = 0.0, M[3] = {0.0, 0.0, 0.0};
    for (int f = 0; f < ef->nf; ++f)
        for (int t = 0; t + 2 < ef->nn[f]; ++t) {
            const double* a = X + nd[ef->v[f][0]] * 3;
            const double* b = X + nd[ef->v[f][t + 1]] * 3;
            const double* e = X + nd[ef->v[f][t + 2]] * 3;
            double u[3], v[3], w[3];
            for (int d = 0; d < 3; ++d) {
                u[d] = a[d] - xm[d];
                v[d] = b[d] - xm[d];
                w[d] = e[d] - xm[d];
            }
            const double det = u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) +
                               u[2] * (v[0] * w[1] - v[1] * w[0]);
            const double cv = std::fabs(det) / 6.0;
            std::array<double, 12> P;
            for (int d = 0; d < 3; ++d) {
                P[d] = xm[d];
                P[3 + d] = a[d];
                P[6 + d] = b[d];
                P[9 + d] = e[d];
                M[d] += cv * (xm[d] + a[d] + b[d] + e[d]) / 4.0;
            }
            cone.push_back(P);
            vol.push_back(cv);
            V += cv;
        }
    if (Vout) *Vout = V;
    if (Cout)
        for (int d = 0; d < 3; ++d) Cout[d] = M[d] / V;
    if (pts) {
        pts->clear();
        wts->clear();
        const double A = 0.5854101966249685, B = 0.1381966011250105;
        for (size_t t = 0; t < cone.size(); ++t)
            for (int k = 0; k < 4; ++k) {
                for (int d = 0; d < 3; ++d) {
                    double s = 0.0;
                    for (int j = 0; j < 4; ++j) s += (j == k ? A : B) * cone[t][j * 3 + d];
                    pts->push_back(s);
                }
                wts->push_back(0.25 * vol[t] / V);
            }
    }
}

/* Degree-2-exact average rule over a fine cell: weights sum to 1. */
void cell_quadrature(const orc_ctx* c, int cell, std::vector<double>& pts, std::vector<double>& wts) {
    if (c->mixed) {
        mixed_cell(c, cell, nullptr, nullptr, &pts, &wts);
        return;
    }
    const int dim = c->dim;
    const Level& L0 = c->lv[0];
    const int* nd = &L0.nodes[cell * (dim + 1)];
    pts.clear();
    wts.clear();
    if (dim == 2) {
        for (int k = 0; k < 3; ++k) {
            const double* a = &c->coords[nd[k] * 2];
            const double* b = &c->coords[nd[(k + 1) % 3] * 2];
            pts.push_back(0.5 * (a[0] + b[0]));
            pts.push_back(0.5 * (a[1] + b[1]));
            wts.push_back(1.0 / 3.0);
        }
    } else {
        const double A = 0.5854101966249685, B = 0.1381966011250105;
        for (int k = 0; k < 4; ++k) {
            for (int d = 0; d < 3; ++d) {
                double s = 0.0;
                for (int j = 0; j < 4; ++j) s += (j == k ? A : B) * c->coords[nd[j] * 3 + d];
                pts.push_back(s);
            }
            wts.push_back(0.25);
        }
    }
}

namespace {

int fail(orc_ctx* c, int code, const std::string& msg) {
    c->err = msg;
    return code;
}

/* Node ids of the face opposite local node k, sorted ascending. */
std::vector<int> face_key(const int* nd, int dim, int k) {
    std::vector<int> key;
    for (int j = 0; j <= dim; ++j)
        if (j != k) key.push_back(nd[j]);
    std::sort(key.begin(), key.end());
    return key;
}

void simplex_geometry(const orc_ctx* c, const int* nd, double* V, double* C) {
    const int dim = c->dim;
    const double* X = c->coords.data();
    if (dim == 2) {
        const double *p0 = X + nd[0] * 2, *p1 = X + nd[1] * 2, *p2 = X + nd[2] * 2;
        *V = 0.5 * ((p1[0] - p0[0]) * (p2[1] - p0[1]) - (p2[0] - p0[0]) * (p1[1] - p0[1]));
        for (int d = 0; d < 2; ++d) C[d] = ((p0[d] + p1[d]) + p2[d]) / 3.0;
    } else {
        const double *p0 = X + nd[0] * 3, *p1 = X + nd[1] * 3, *p2 = X + nd[2] * 3,
                     *p3 = X + nd[3] * 3;
        double a[3], b[3], e[3];
        for (int d = 0; d < 3; ++d) {
            a[d] = p1[d] - p0[d];
            b[d] = p2[d] - p0[d];
            e[d] = p3[d] - p0[d];
        }
        double det = a[0] * (b[1] * e[2] - b[2] * e[1]) - a[1] * (b[0] * e[2] - b[2] * e[0]) +
                     a[2] * (b[0] * e[1] - b[1] * e[0]);
        *V = det / 6.0;
        for (int d = 0; d < 3; ++d) C[d] = (((p0[d] + p1[d]) + p2[d]) + p3[d]) / 4.0;
    }
}

void face_geometry(const orc_ctx* c, const std::vector<int>& key, const double* CL, Face& f) {
    const int dim = c->dim;
    const double* X = c->coords.data();
    if (dim == 2) {
        const double *a = X + key[0] * 2, *b = X + key[1] * 2;
        double dx = b[0] - a[0], dy = b[1] - a[1];
        f.S = std::sqrt(dx * dx + dy * dy);
        f.n[0] = dy / f.S;
        f.n[1] = -dx / f.S;
        f.n[2] = 0.0;
        f.xc[0] = 0.5 * (a[0] + b[0]);
        f.xc[1] = 0.5 * (a[1] + b[1]);
        f.xc[2] = 0.0;
        f.ngp = 2;
        const double s[2] = {0.5 - std::sqrt(3.0) / 6.0, 0.5 + std::sqrt(3.0) / 6.0};
        for (int k = 0; k < 2; ++k) {
            f.gp[k][0] = a[0] + s[k] * dx;
            f.gp[k][1] = a[1] + s[k] * dy;
            f.gp[k][2] = 0.0;
            f.w[k] = 0.5;
        }
    } else {
        const double *a = X + key[0] * 3, *b = X + key[1] * 3, *e = X + key[2] * 3;
        double u[3], v[3], N[3];
        for (int d = 0; d < 3; ++d) {
            u[d] = b[d] - a[d];
            v[d] = e[d] - a[d];
        }
        N[0] = u[1] * v[2] - u[2] * v[1];
        N[1] = u[2] * v[0] - u[0] * v[2];
        N[2] = u[0] * v[1] - u[1] * v[0];
        double nn = std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        f.S = 0.5 * nn;
        for (int d = 0; d < 3; ++d) {
            f.n[d] = N[d] / nn;
            f.xc[d] = ((a[d] + b[d]) + e[d]) / 3.0;
        }
        f.ngp = 3;
        const double big = 2.0 / 3.0, sm = 1.0 / 6.0;
        for (int k = 0; k < 3; ++k) {
            double wa = (k == 0) ? big : sm, wb = (k == 1) ? big : sm, we = (k == 2) ? big : sm;
            for (int d = 0; d < 3; ++d) f.gp[k][d] = wa * a[d] + wb * b[d] + we * e[d];
            f.w[k] = 1.0 / 3.0;
        }
    }
    double dot = 0.0;
    for (int d = 0; d < dim; ++d) dot += f.n[d] * (f.xc[d] - CL[d]);
    if (dot < 0.0)
        for (int d = 0; d < dim; ++d) f.n[d] = -f.n[d];
}

/* Geometry of a planar quadrilateral face with node cycle a, b, e, g: area
 * vector (e - a) x (g - b) / 2, centroid from the triangles a, b, e and
 * a, e, g, and the 2 x 2 Gauss rule of its bilinear map from [-1, 1]^2, each
 * point weighted by the map's area element there (the weights sum to 1).
 * False when the fourth node is off the plane of the first three. */
bool quad_face_geometry(const orc_ctx* c, const int* cyc, const double* CL, Face& f) {
    const double* X = c->coords.data();
    const double *a = X + cyc[0] * 3, *b = X + cyc[1] * 3, *e = X + cyc[2] * 3, *g = X + cyc[3] * 3;
    auto cross = [](const double* u, const double* v, double* w) {
        w[0] = u[1] * v[2] - u[2] * v[1];
        w[1] = u[2] * v[0] - u[0] * v[2];
        w[2] = u[0] * v[1] - u[1] * v[0];
    };
    auto norm = [](const double* u) { return std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]); };
    double p[3], q[3], N[3];
    for (int d = 0; d < 3; ++d) {
        p[d] = e[d] - a[d];
        q[d] = g[d] - b[d];
    }
    cross(p, q, N);
    const double nn = norm(N);
    f.S = 0.5 * nn;
    for (int d = 0; d < 3; ++d) f.n[d] = N[d] / nn;
    double off = 0.0;
    for (int d = 0; d < 3; ++d) off += (g[d] - a[d]) * f.n[d];
    if (std::fabs(off) > 1e-9 * std::sqrt(f.S)) return false;
    double u1[3], v1[3], w1[3], u2[3], w2[3];
    for (int d = 0; d < 3; ++d) {
        u1[d] = b[d] - a[d];
        v1[d] = e[d] - a[d];
        u2[d] = g[d] - a[d];
    }
    cross(u1, v1, w1);
    cross(v1, u2, w2);
    const double A1 = 0.5 * norm(w1), A2 = 0.5 * norm(w2);
    for (int d = 0; d < 3; ++d)
        f.xc[d] = (A1 * (a[d] + b[d] + e[d]) / 3.0 + A2 * (a[d] + e[d] + g[d]) / 3.0) / (A1 + A2);
    f.ngp = 4;
    const double r = 1.0 / std::sqrt(3.0);
    const double sp[4] = {-r, r, r, -r}, tp[4] = {-r, -r, r, r};
    double jac[4], jsum = 0.0;
    for (int k = 0; k < 4; ++k) {
        const double s = sp[k], t = tp[k];
        double xs[3], xt[3], J[3];
        for (int d = 0; d < 3; ++d) {
            f.gp[k][d] = 0.25 * ((1 - s) * (1 - t) * a[d] + (1 + s) * (1 - t) * b[d] + (1 + s) * (1 + t) * e[d] +
                                 (1 - s) * (1 + t) * g[d]);
            xs[d] = 0.25 * (-(1 - t) * a[d] + (1 - t) * b[d] + (1 + t) * e[d] - (1 + t) * g[d]);
            xt[d] = 0.25 * (-(1 - s) * a[d] - (1 + s) * b[d] + (1 + s) * e[d] + (1 - s) * g[d]);
        }
        cross(xs, xt, J);
        jac[k] = norm(J);
        jsum += jac[k];
    }
    for (int k = 0; k < 4; ++k) f.w[k] = jac[k] / jsum;
    double dot = 0.0;
    for (int d = 0; d < 3; ++d) dot += f.n[d] * (f.xc[d] - CL[d]);
    if (dot < 0.0)
        for (int d = 0; d < 3; ++d) f.n[d] = -f.n[d];
    return true;
}

/* Faces of an agglomerated level: one face per pair of adjacent agglomerates and
 * one per (agglomerate, boundary tag); area vector = sum of finer-level S n. */
void build_coarse_faces(orc_ctx* c, int l) {
    const int dim = c->dim;
    Level& F = c->lv[l - 1];
    Level& G = c->lv[l];
    struct Acc {
        double Sv[3] = {0, 0, 0}, xs[3] = {0, 0, 0}, Ssum = 0;
        int tag = 0;
    };
    std::map<std::tuple<int, int, int>, Acc> groups;
    for (const Face& f : F.faces) {
        int I = F.parent[f.L];
        if (f.R >= 0) {
            int J = F.parent[f.R];
            if (I == J) continue;
            int lo = std::min(I, J), hi = std::max(I, J);
            double sg = (I < J) ? 1.0 : -1.0;
            Acc& a = groups[std::make_tuple(lo, hi, 0)];
            for (int d = 0; d < dim; ++d) {
                a.Sv[d] += sg * f.S * f.n[d];
                a.xs[d] += f.S * f.xc[d];
            }
            a.Ssum += f.S;
        } else {
            Acc& a = groups[std::make_tuple(I, -1, f.tag)];
            for (int d = 0; d < dim; ++d) {
                a.Sv[d] += f.S * f.n[d];
                a.xs[d] += f.S * f.xc[d];
            }
            a.Ssum += f.S;
            a.tag = f.tag;
        }
    }
    G.faces.clear();
    G.cf.assign(G.n, std::vector<int>());
    std::vector<std::tuple<int, int, int, int>> order;  // (L, rkey, tag, idx)
    for (auto& kv : groups) {
        int L = std::get<0>(kv.first), R = std::get<1>(kv.first), tag = std::get<2>(kv.first);
        Face f;
        std::memset(&f, 0, sizeof(f));
        f.L = L;
        f.R = R;
        f.tag = tag;
        const Acc& a = kv.second;
        double s2 = 0.0;
        for (int d = 0; d < dim; ++d) s2 += a.Sv[d] * a.Sv[d];
        f.S = std::sqrt(s2);
        for (int d = 0; d < dim; ++d) {
            f.n[d] = a.Sv[d] / f.S;
            f.xc[d] = a.xs[d] / a.Ssum;
        }
        f.ngp = 0;
        G.faces.push_back(f);
    }
    /* std::map iterates in (L, R, tag) order with R = -1 first; put boundary groups
     * after the interior ones of the same L so the face list is sorted by (L, R). */
    std::vector<Face> sorted = G.faces;
    std::stable_sort(sorted.begin(), sorted.end(), [](const Face& x, const Face& y) {
        long kx = x.R >= 0 ? x.R : (long)1 << 40, ky = y.R >= 0 ? y.R : (long)1 << 40;
        if (x.L != y.L) return x.L < y.L;
        if (kx != ky) return kx < ky;
        return x.tag < y.tag;
    });
    G.faces = sorted;
    /* Local face order of a coarse cell: by neighbour index, then boundary tags. */
    std::vector<std::vector<std::pair<long, int>>> lists(G.n);
    for (int fi = 0; fi < (int)G.faces.size(); ++fi) {
        const Face& f = G.faces[fi];
        if (f.R >= 0) {
            lists[f.L].push_back(std::make_pair((long)f.R, fi));
            lists[f.R].push_back(std::make_pair((long)f.L, fi));
        } else {
            lists[f.L].push_back(std::make_pair(((long)1 << 40) + f.tag, fi));
        }
    }
    for (int i = 0; i < G.n; ++i) {
        std::sort(lists[i].begin(), lists[i].end());
        for (auto& pr : lists[i]) G.cf[i].push_back(pr.second);
    }
}

std::vector<std::vector<int>> level_neighbours(const Level& L) {
    std::vector<std::vector<int>> nb(L.n);
    for (int i = 0; i < L.n; ++i)
        for (int fi : L.cf[i]) {
            const Face& f = L.faces[fi];
            if (f.R < 0) continue;
            nb[i].push_back(f.L == i ? f.R : f.L);
        }
    return nb;
}

/* Dense solve with partial pivoting; returns false when a pivot is negligible. */
bool dense_solve(int n, std::vector<double> A, std::vector<double>& B, int nrhs) {
    double amax = 0.0;
    for (double v : A) amax = std::max(amax, std::fabs(v));
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[i * n + k]) > std::fabs(A[piv * n + k])) piv = i;
        if (!(std::fabs(A[piv * n + k]) > 1e-12 * amax)) return false;
        if (piv != k) {
            for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[piv * n + j]);
            for (int r = 0; r < nrhs; ++r) std::swap(B[k * nrhs + r], B[piv * nrhs + r]);
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            for (int r = 0; r < nrhs; ++r) B[i * nrhs + r] -= f * B[k * nrhs + r];
        }
    }
    for (int k = n - 1; k >= 0; --k)
        for (int r = 0; r < nrhs; ++r) {
            double s = B[k * nrhs + r];
            for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * B[j * nrhs + r];
            B[k * nrhs + r] = s / A[k * n + k];
        }
    return true;
}

/* Constrained least squares of Sec. 3.1 for basis size nb; false if singular. */
bool recon_kkt(orc_ctx* c, int i, int nb, ReconOp& op) {
    const int dim = c->dim;
    const Level& L0 = c->lv[0];
    const int nn = (int)op.nbr.size();
    const double* x0 = &L0.C[i * dim];
    const double h = L0.h[i];
    std::vector<double> pts, wts;
    op.nb = nb;
    op.mean0.assign(nb, 0.0);
    cell_quadrature(c, i, pts, wts);
    for (int k = 0; k < nb; ++k)
        for (size_t q = 0; q < wts.size(); ++q) op.mean0[k] += wts[q] * basis_eval(dim, k, &pts[q * dim], x0, h);
    if (nb == 0) {
        op.M.clear();
        return true;
    }
    /* Equality rows: exact neighbour averages.  LS rows: |x_m - x_0| * slope match at x_m. */
    std::vector<double> E(nn * nb), A(nn * dim * nb), wm(nn);
    for (int m = 0; m < nn; ++m) {
        int j = op.nbr[m];
        cell_quadrature(c, j, pts, wts);
        const double* xm = &L0.C[j * dim];
        double r2 = 0.0;
        for (int d = 0; d < dim; ++d) r2 += (xm[d] - x0[d]) * (xm[d] - x0[d]);
        wm[m] = std::sqrt(r2);
        for (int k = 0; k < nb; ++k) {
            double avg = 0.0;
            for (size_t q = 0; q < wts.size(); ++q) avg += wts[q] * basis_eval(dim, k, &pts[q * dim], x0, h);
            E[m * nb + k] = avg - op.mean0[k];
            for (int d = 0; d < dim; ++d) {
                int l[3] = {0, 0, 0};
                l[d] = 1;
                A[(m * dim + d) * nb + k] = wm[m] * basis_deriv(dim, k, l, xm, x0, h);
            }
        }
    }
    const int nk = nb + nn, nin = nn * (1 + dim);
    std::vector<double> K(nk * nk, 0.0), B(nk * nin, 0.0);
    for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) {
            double s = 0.0;
            for (int r = 0; r < nn * dim; ++r) s += A[r * nb + a] * A[r * nb + b];
            K[a * nk + b] = s;
        }
    for (int m = 0; m < nn; ++m)
        for (int k = 0; k < nb; ++k) {
            K[k * nk + nb + m] = E[m * nb + k];
            K[(nb + m) * nk + k] = E[m * nb + k];
        }
    for (int m = 0; m < nn; ++m) {
        B[(nb + m) * nin + m * (1 + dim)] = 1.0;  /* average of neighbour m */
        for (int d = 0; d < dim; ++d) {
            int col = m * (1 + dim) + 1 + d;          /* slope d of neighbour m */
            int row = m * dim + d;
            for (int k = 0; k < nb; ++k) B[k * nin + col] = A[row * nb + k] * wm[m];
        }
    }
    if (!dense_solve(nk, K, B, nin)) return false;
    op.M.assign(nb * nin, 0.0);
    for (int k = 0; k < nb; ++k)
        for (int j = 0; j < nin; ++j) op.M[k * nin + j] = B[k * nin + j];
    return true;
}

}  // namespace

int color_graph(int n, const std::vector<std::vector<int>>& nbrs, std::vector<int>& color) {
    /* Alg. 1: greedy painting along a breadth-first traversal that starts at
     * cell 0; each newly reached cell takes the smallest colour not used by an
     * already painted neighbour. */
    color.assign(n, 0);
    std::vector<int> queue;
    queue.reserve(n);
    int ncolor = 0;
    auto paint = [&](int w) {
        std::set<int> used;
        for (int j : nbrs[w])
            if (color[j] > 0) used.insert(color[j]);
        int k = 1;
        while (used.count(k)) ++k;
        color[w] = k;
        ncolor = std::max(ncolor, k);
    };
    for (int start = 0; start < n; ++start) {
        if (color[start] != 0) continue;
        paint(start);
        queue.clear();
        queue.push_back(start);
        for (size_t h = 0; h < queue.size(); ++h) {
            int v = queue[h];
            for (int w : nbrs[v])
                if (color[w] == 0) {
                    paint(w);
                    queue.push_back(w);
                }
        }
    }
    return ncolor;
}

int agglomerate(orc_ctx* c, int level, std::vector<int>& agg) {
    /* Alg. 3: hash-selected interior faces, merged when the skewness of every
     * remaining face of the merged pair passes the limit. */
    const int dim = c->dim;
    const Level& L = c->lv[level];
    std::vector<int> interior;
    for (int fi = 0; fi < (int)L.faces.size(); ++fi)
        if (L.faces[fi].R >= 0) interior.push_back(fi);
    const uint64_t Nf = interior.size();
    std::set<uint64_t> seen;
    std::vector<int> chosen;
    for (int fi : interior) {
        uint64_t a = (uint64_t)L.faces[fi].L, b = (uint64_t)L.faces[fi].R;
        uint64_t h = Nf ? (23u * (a + b) + a * b) % Nf : 0;
        if (!seen.count(h)) {
            seen.insert(h);
            chosen.push_back(fi);
        }
    }
    std::vector<int> group(L.n, -1);
    for (int fi : chosen) {
        const Face& f = L.faces[fi];
        if (group[f.L] >= 0 || group[f.R] >= 0) continue;
        double VL = L.V[f.L], VR = L.V[f.R], Cc[3];
        for (int d = 0; d < dim; ++d) Cc[d] = (VL * L.C[f.L * dim + d] + VR * L.C[f.R * dim + d]) / (VL + VR);
        double minsin = 2.0;
        const int cells[2] = {f.L, f.R};
        for (int t = 0; t < 2; ++t) {
            int X = cells[t];
            for (int g : L.cf[X]) {
                if (g == fi) continue;
                const Face& e = L.faces[g];
                double sg = (e.L == X) ? 1.0 : -1.0;
                double dn = 0.0, dd = 0.0;
                for (int d = 0; d < dim; ++d) {
                    double dv = e.xc[d] - Cc[d];
                    dn += dv * (sg * e.n[d]);
                    dd += dv * dv;
                }
                double s = dn / std::sqrt(dd);
                if (s < minsin) minsin = s;
            }
        }
        if (minsin >= c->p.skew_limit) {
            group[f.L] = fi;
            group[f.R] = fi;
        }
    }
    agg.assign(L.n, -1);
    std::map<int, int> gid;
    int next = 0;
    for (int i = 0; i < L.n; ++i) {
        if (group[i] < 0) {
            agg[i] = next++;
        } else {
            auto it = gid.find(group[i]);
            if (it == gid.end()) {
                gid[group[i]] = next;
                agg[i] = next++;
            } else {
                agg[i] = it->second;
            }
        }
    }
    return next;
}

void build_recon_ops(orc_ctx* c) {
    const int dim = c->dim;
    const Level& L0 = c->lv[0];
    c->rop.assign(L0.n, ReconOp());
#pragma omp parallel for schedule(dynamic, 256)
    for (int i = 0; i < L0.n; ++i) {
        ReconOp& op = c->rop[i];
        for (int fi : L0.cf[i]) {
            const Face& f = L0.faces[fi];
            if (f.R >= 0) op.nbr.push_back(f.L == i ? f.R : f.L);
        }
        int nn = (int)op.nbr.size();
        int nb = 0;
        if (nn * (1 + dim) >= n_quad_basis(dim)) nb = n_quad_basis(dim);
        else if (nn * (1 + dim) >= dim) nb = dim;
        while (!recon_kkt(c, i, nb, op)) nb = (nb == n_quad_basis(dim)) ? dim : 0;
    }
}

int setup_mesh(orc_ctx* c, const orc_mesh* m, int n_levels, const int32_t* const* parent) {
    const int dim = m->dim;
    if (dim != c->p.dim || (dim != 2 && dim != 3)) return fail(c, ORC_EINVAL, "dimension mismatch");
    if (n_levels < 1) return fail(c, ORC_EINVAL, "n_levels < 1");
    const bool mixed = m->cell_offsets != nullptr;
    if (mixed != (m->bface_offsets != nullptr))
        return fail(c, ORC_EINVAL, "cell_offsets and bface_offsets go together");
    if (mixed && dim != 3) return fail(c, ORC_EINVAL, "mixed elements are 3-D only");
    c->mixed = mixed;
    c->dim = dim;
    c->nvar = dim + 2;
    c->coords.assign(m->coords, m->coords + (size_t)m->n_nodes * dim);
    c->lv.assign(n_levels, Level());
    Level& L0 = c->lv[0];
    L0.n = m->n_cells;
    if (mixed) {
        L0.noff.assign(m->cell_offsets, m->cell_offsets + m->n_cells + 1);
        if (L0.noff[0] != 0) return fail(c, ORC_EMESH, "cell_offsets[0] != 0");
        for (int i = 0; i < L0.n; ++i)
            if (!elem_faces(L0.noff[i + 1] - L0.noff[i]))
                return fail(c, ORC_EMESH, "cell with a node count other than 4, 5, 6 or 8");
        L0.nodes.assign(m->cell_nodes, m->cell_nodes + L0.noff[L0.n]);
    } else {
        L0.nodes.assign(m->cell_nodes, m->cell_nodes + (size_t)m->n_cells * (dim + 1));
    }
    auto cell_nodes = [&](int i, int& cnt) -> const int* {
        cnt = mixed ? L0.noff[i + 1] - L0.noff[i] : dim + 1;
        return mixed ? &L0.nodes[L0.noff[i]] : &L0.nodes[(size_t)i * (dim + 1)];
    };
    L0.V.resize(L0.n);
    L0.C.resize((size_t)L0.n * dim);
    L0.h.resize(L0.n);
    for (int i = 0; i < L0.n; ++i) {
        int cnt;
        const int* nd = cell_nodes(i, cnt);
        for (int j = 0; j < cnt; ++j)
            if (nd[j] < 0 || nd[j] >= m->n_nodes) return fail(c, ORC_EMESH, "node id out of range");
        double C[3];
        if (mixed)
            mixed_cell(c, i, &L0.V[i], C, nullptr, nullptr);
        else
            simplex_geometry(c, nd, &L0.V[i], C);
        if (!(L0.V[i] > 0.0)) return fail(c, ORC_EMESH, "non-positive cell volume");
        for (int d = 0; d < dim; ++d) L0.C[i * dim + d] = C[d];
        L0.h[i] = (dim == 2) ? std::sqrt(L0.V[i]) : std::cbrt(L0.V[i]);
    }
    /* Canonical faces: sorted node tuples in lexicographic order. */
    std::vector<std::tuple<std::vector<int>, int, int>> all;
    all.reserve((size_t)L0.n * (dim + 1));
    /* node cycle of local face k of cell i */
    auto face_cycle = [&](int i, int k) {
        int cnt;
        const int* nd = cell_nodes(i, cnt);
        std::vector<int> cyc;
        if (mixed) {
            const ElemFaces* ef = elem_faces(cnt);
            for (int j = 0; j < ef->nn[k]; ++j) cyc.push_back(nd[ef->v[k][j]]);
        } else {
            cyc = face_key(nd, dim, k);
        }
        return cyc;
    };
    L0.cf.assign(L0.n, std::vector<int>());
    for (int i = 0; i < L0.n; ++i) {
        int cnt;
        cell_nodes(i, cnt);
        const int nfc = mixed ? elem_faces(cnt)->nf : dim + 1;
        L0.cf[i].assign(nfc, -1);
        for (int k = 0; k < nfc; ++k) {
            std::vector<int> key = face_cycle(i, k);
            std::sort(key.begin(), key.end());
            all.emplace_back(key, i, k);
        }
    }
    std::sort(all.begin(), all.end());
    std::vector<std::pair<std::vector<int>, int>> bkeys;
    for (int b = 0; b < m->n_bfaces; ++b) {
        const size_t b0 = mixed ? (size_t)m->bface_offsets[b] : (size_t)b * dim;
        const size_t b1 = mixed ? (size_t)m->bface_offsets[b + 1] : (size_t)(b + 1) * dim;
        std::vector<int> key(m->bface_nodes + b0, m->bface_nodes + b1);
        std::sort(key.begin(), key.end());
        bkeys.emplace_back(key, m->bface_tag[b]);
    }
    std::sort(bkeys.begin(), bkeys.end());
    int nbmatched = 0;
    for (size_t s = 0; s < all.size();) {
        size_t e = s + 1;
        while (e < all.size() && std::get<0>(all[e]) == std::get<0>(all[s])) ++e;
        if (e - s > 2) return fail(c, ORC_EMESH, "non-manifold face");
        Face f;
        std::memset(&f, 0, sizeof(f));
        const std::vector<int>& key = std::get<0>(all[s]);
        f.L = std::get<1>(all[s]);
        f.R = (e - s == 2) ? std::get<1>(all[s + 1]) : -1;
        f.tag = 0;
        if (f.R < 0) {
            auto it = std::lower_bound(bkeys.begin(), bkeys.end(), std::make_pair(key, -1 << 30));
            if (it == bkeys.end() || it->first != key) return fail(c, ORC_EMESH, "boundary face without a tag");
            f.tag = it->second;
            ++nbmatched;
        }
        if (!mixed) {
            face_geometry(c, key, &L0.C[f.L * dim], f);
        } else {
            const std::vector<int> cyc = face_cycle(std::get<1>(all[s]), std::get<2>(all[s]));
            if (cyc.size() == 3)
                face_geometry(c, cyc, &L0.C[f.L * dim], f);
            else if (!quad_face_geometry(c, cyc.data(), &L0.C[f.L * dim], f))
                return fail(c, ORC_EMESH, "non-planar quadrilateral face");
        }
        int fi = (int)L0.faces.size();
        L0.faces.push_back(f);
        for (size_t t = s; t < e; ++t) L0.cf[std::get<1>(all[t])][std::get<2>(all[t])] = fi;
        s = e;
    }
    if (nbmatched != m->n_bfaces) return fail(c, ORC_EMESH, "tagged boundary face not on the boundary");
    /* Coarse levels. */
    for (int l = 1; l < n_levels; ++l) {
        Level& F = c->lv[l - 1];
        Level& G = c->lv[l];
        if (parent && parent[l - 1]) {
            F.parent.assign(parent[l - 1], parent[l - 1] + F.n);
        } else {
            agglomerate(c, l - 1, F.parent);
        }
        int nc = 0;
        for (int i = 0; i < F.n; ++i) {
            if (F.parent[i] < 0) return fail(c, ORC_EMESH, "negative parent index");
            nc = std::max(nc, F.parent[i] + 1);
        }
        G.n = nc;
        G.children.assign(nc, std::vector<int>());
        for (int i = 0; i < F.n; ++i) G.children[F.parent[i]].push_back(i);
        G.V.assign(nc, 0.0);
        G.C.assign((size_t)nc * dim, 0.0);
        for (int I = 0; I < nc; ++I) {
            if (G.children[I].empty()) return fail(c, ORC_EMESH, "empty agglomerate");
            double V = 0.0, C[3] = {0, 0, 0};
            for (int i : G.children[I]) {
                V += F.V[i];
                for (int d = 0; d < dim; ++d) C[d] += F.V[i] * F.C[i * dim + d];
            }
            G.V[I] = V;
            for (int d = 0; d < dim; ++d) G.C[I * dim + d] = C[d] / V;
        }
        build_coarse_faces(c, l);
        G.ncolor = color_graph(G.n, level_neighbours(G), G.color);
    }
    {
        std::vector<int> col;
        L0.ncolor = color_graph(L0.n, level_neighbours(L0), L0.color);
    }
    build_recon_ops(c);
    for (int l = 0; l < n_levels; ++l) {
        Level& L = c->lv[l];
        const int nv = c->nvar;
        L.W.assign((size_t)L.n * nv, 0.0);
        L.W0 = L.W;
        L.F = L.W;
        L.Rstar = L.W;
        L.dW.assign(L.W.size(), 0.0);
        L.rhs_last = L.W;
        L.alpha.assign(L.n, 1.0);
        if (l == 0) L.grad.assign((size_t)L.n * nv * dim, 0.0);
    }
    c->have_mesh = true;
    return ORC_OK;
}

}  // namespace orc

extern "C" {

int orc_coloring_graph(int n, const int32_t* xadj, const int32_t* adj, int32_t* color_out,
                       int32_t* n_colors) {
    std::vector<std::vector<int>> nb(n);
    for (int i = 0; i < n; ++i)
        for (int k = xadj[i]; k < xadj[i + 1]; ++k) nb[i].push_back(adj[k]);
    std::vector<int> col;
    *n_colors = orc::color_graph(n, nb, col);
    for (int i = 0; i < n; ++i) color_out[i] = col[i];
    return ORC_OK;
}
}

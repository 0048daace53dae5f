/*
 * Host-side mesh hierarchy set-up of libcgks: faces and geometry (Sec. 2.2),
 * compact reconstruction operators (Sec. 3.1), coarse levels (Sec. 5.1),
 * multi-colour painting (Alg. 1), cell coarsening (Alg. 3), internal
 * permutations, and the upload to the device.
 *
 * Compiled with -ffp-contract=off: Alg. 3's merge test compares a
 * floating-point skewness against a limit, so the expressions for volumes,
 * centroids, face centres and normals are evaluated in a fixed order.
 */
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <unordered_map>
#include <unordered_set>

#include "cgks_internal.h"

namespace cgks {

int fail(cgks_ctx* c, int code, const std::string& msg) {
    c->err = msg;
    return code;
}

int hip_fail(cgks_ctx* c, hipError_t e, const char* what) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return CGKS_EDEVICE;
}

namespace {

struct FaceKey {
    int v[4];            /* sorted node ids; -1 past the face's node count */
    bool operator==(const FaceKey& o) const {
        return v[0] == o.v[0] && v[1] == o.v[1] && v[2] == o.v[2] && v[3] == o.v[3];
    }
    bool operator<(const FaceKey& o) const {
        for (int i = 0; i < 4; ++i)
            if (v[i] != o.v[i]) return v[i] < o.v[i];
        return false;
    }
};
struct FaceKeyHash {
    size_t operator()(const FaceKey& k) const {
        uint64_t h = 1469598103934665603ull;
        for (int i = 0; i < 4; ++i) h = (h ^ (uint64_t)(uint32_t)k.v[i]) * 1099511628211ull;
        return (size_t)h;
    }
};

FaceKey make_key(const int* ids, int cnt) {
    FaceKey k;
    k.v[0] = k.v[1] = k.v[2] = k.v[3] = -1;
    for (int i = 0; i < cnt; ++i) k.v[i] = ids[i];
    std::sort(k.v, k.v + cnt);
    return k;
}

/* Faces of the 3-D element types of the mixed input (Sec. 2.2), each as a
 * cycle of the element's local nodes: a tetrahedron's face t leaves out
 * node t; a pyramid lists its base and then its four triangles; a prism its
 * two triangles and then its three quadrilaterals; a hexahedron its first
 * and last quadrilaterals and then the four sides. */
struct ElemTable {
    int nface;
    int cnt[6];
    int node[6][4];
};

const ElemTable* element(int nnode) {
    static const ElemTable T4 = {4, {3, 3, 3, 3}, {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}}};
    static const ElemTable T5 = {5, {4, 3, 3, 3, 3}, {{0, 1, 2, 3}, {0, 1, 4}, {1, 2, 4}, {2, 3, 4}, {3, 0, 4}}};
    static const ElemTable T6 = {5, {3, 3, 4, 4, 4}, {{0, 1, 2}, {3, 4, 5}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}}};
    static const ElemTable T8 = {6, {4, 4, 4, 4, 4, 4},
                                 {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}}};
    return nnode == 4 ? &T4 : nnode == 5 ? &T5 : nnode == 6 ? &T6 : nnode == 8 ? &T8 : nullptr;
}

/* Basis of the quadratic reconstruction: scaled monomials ((x-xc)/h)^e. */
const int E2[5][3] = {{1, 0, 0}, {0, 1, 0}, {2, 0, 0}, {1, 1, 0}, {0, 2, 0}};
const int E3[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {1, 1, 0},
                      {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};

double mono(int dim, int k, const double* x, const double* xc, double h) {
    const int* e = (dim == 2) ? E2[k] : E3[k];
    double r = 1.0;
    for (int d = 0; d < dim; ++d) r *= std::pow((x[d] - xc[d]) / h, (double)e[d]);
    return r;
}

double mono_dx(int dim, int k, int dd, const double* x, const double* xc, double h) {
    const int* e = (dim == 2) ? E2[k] : E3[k];
    if (e[dd] == 0) return 0.0;
    double r = (double)e[dd] / h;
    for (int d = 0; d < dim; ++d) {
        int p = e[d] - (d == dd ? 1 : 0);
        r *= std::pow((x[d] - xc[d]) / h, (double)p);
    }
    return r;
}

/* Cell average of a function over a simplex: midpoint-of-edges rule (triangle)
 * or the symmetric 4-point rule (tetrahedron), both exact for quadratics. */
template <class F>
double simplex_average(int dim, const double* P /* (dim+1) x dim */, F f) {
    if (dim == 2) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
            int b = (a + 1) % 3;
            double x[2] = {0.5 * (P[a * 2] + P[b * 2]), 0.5 * (P[a * 2 + 1] + P[b * 2 + 1])};
            s += f(x);
        }
        return s / 3.0;
    }
    const double al = 0.5854101966249685, be = 0.1381966011250105;
    double s = 0.0;
    for (int a = 0; a < 4; ++a) {
        double x[3];
        for (int d = 0; d < 3; ++d) {
            double v = 0.0;
            for (int j = 0; j < 4; ++j) v += (j == a ? al : be) * P[j * 3 + d];
            x[d] = v;
        }
        s += f(x);
    }
    return 0.25 * s;
}

/* Householder QR of an m x n row-major matrix (m >= n): A = Q R, Q m x m. */
void householder(int m, int n, std::vector<double> A, std::vector<double>& Q, std::vector<double>& R) {
    Q.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) Q[i * m + i] = 1.0;
    for (int k = 0; k < n; ++k) {
        double nrm = 0.0;
        for (int i = k; i < m; ++i) nrm += A[i * n + k] * A[i * n + k];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) continue;
        double alpha = (A[k * n + k] > 0.0) ? -nrm : nrm;
        std::vector<double> v(m, 0.0);
        for (int i = k; i < m; ++i) v[i] = A[i * n + k];
        v[k] -= alpha;
        double vv = 0.0;
        for (int i = k; i < m; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int i = k; i < m; ++i) s += v[i] * A[i * n + j];
            s *= 2.0 / vv;
            for (int i = k; i < m; ++i) A[i * n + j] -= s * v[i];
        }
        for (int r = 0; r < m; ++r) {  /* Q <- Q H */
            double s = 0.0;
            for (int i = k; i < m; ++i) s += Q[r * m + i] * v[i];
            s *= 2.0 / vv;
            for (int i = k; i < m; ++i) Q[r * m + i] -= s * v[i];
        }
    }
    R = A;
}

/* Constrained least squares by the null-space method:
 *   min |A a - b|  subject to  E a = d.
 * Returns false if E has dependent rows or A is rank deficient on null(E).
 * Md (nb x neq) and Mb (nb x nls) give a = Md d + Mb b. */
bool null_space_ls(int nb, int neq, int nls, const std::vector<double>& E, const std::vector<double>& A,
                   std::vector<double>& Md, std::vector<double>& Mb) {
    std::vector<double> Et((size_t)nb * neq);
    for (int i = 0; i < neq; ++i)
        for (int k = 0; k < nb; ++k) Et[k * neq + i] = E[i * nb + k];
    std::vector<double> Q, R;
    householder(nb, neq, Et, Q, R);
    double rmax = 0.0;
    for (int i = 0; i < neq; ++i) rmax = std::max(rmax, std::fabs(R[i * neq + i]));
    for (int i = 0; i < neq; ++i)
        if (!(std::fabs(R[i * neq + i]) > 1e-12 * rmax)) return false;
    /* X = R1^{-T}: solve R1^T X = I (lower triangular). */
    std::vector<double> X((size_t)neq * neq, 0.0);
    for (int col = 0; col < neq; ++col)
        for (int i = 0; i < neq; ++i) {
            double s = (i == col) ? 1.0 : 0.0;
            for (int j = 0; j < i; ++j) s -= R[j * neq + i] * X[j * neq + col];
            X[i * neq + col] = s / R[i * neq + i];
        }
    std::vector<double> P((size_t)nb * neq, 0.0);  /* Q1 X */
    for (int k = 0; k < nb; ++k)
        for (int col = 0; col < neq; ++col) {
            double s = 0.0;
            for (int j = 0; j < neq; ++j) s += Q[k * nb + j] * X[j * neq + col];
            P[k * neq + col] = s;
        }
    const int r = nb - neq;
    Md = P;
    Mb.assign((size_t)nb * nls, 0.0);
    if (r == 0) return true;
    if (nls < r) return false;
    std::vector<double> B((size_t)nls * r, 0.0);   /* A Q2 */
    for (int i = 0; i < nls; ++i)
        for (int j = 0; j < r; ++j) {
            double s = 0.0;
            for (int k = 0; k < nb; ++k) s += A[i * nb + k] * Q[k * nb + neq + j];
            B[i * r + j] = s;
        }
    std::vector<double> QB, RB;
    householder(nls, r, B, QB, RB);
    double bmax = 0.0;
    for (int i = 0; i < r; ++i) bmax = std::max(bmax, std::fabs(RB[i * r + i]));
    for (int i = 0; i < r; ++i)
        if (!(std::fabs(RB[i * r + i]) > 1e-12 * bmax)) return false;
    /* Bp = RB1^{-1} QB1^T  (r x nls) */
    std::vector<double> Bp((size_t)r * nls, 0.0);
    for (int col = 0; col < nls; ++col)
        for (int i = r - 1; i >= 0; --i) {
            double s = QB[col * nls + i];
            for (int j = i + 1; j < r; ++j) s -= RB[i * r + j] * Bp[j * nls + col];
            Bp[i * nls + col] = s / RB[i * r + i];
        }
    /* Mb = Q2 Bp ;  Md = P - Q2 Bp A P */
    for (int k = 0; k < nb; ++k)
        for (int col = 0; col < nls; ++col) {
            double s = 0.0;
            for (int j = 0; j < r; ++j) s += Q[k * nb + neq + j] * Bp[j * nls + col];
            Mb[k * nls + col] = s;
        }
    std::vector<double> AP((size_t)nls * neq, 0.0);
    for (int i = 0; i < nls; ++i)
        for (int col = 0; col < neq; ++col) {
            double s = 0.0;
            for (int k = 0; k < nb; ++k) s += A[i * nb + k] * P[k * neq + col];
            AP[i * neq + col] = s;
        }
    for (int k = 0; k < nb; ++k)
        for (int col = 0; col < neq; ++col) {
            double s = 0.0;
            for (int i = 0; i < nls; ++i) s += Mb[k * nls + i] * AP[i * neq + col];
            Md[k * neq + col] = P[k * neq + col] - s;
        }
    return true;
}

void cell_vertices(const cgks_ctx* c, const HLevel& L, int i, double* P) {
    const int dim = c->dim;
    for (int j = 0; j <= dim; ++j)
        for (int d = 0; d < dim; ++d) P[j * dim + d] = c->coords[(size_t)L.nodes[i * (dim + 1) + j] * dim + d];
}

/* A mixed element with planar faces as tetrahedra: the mean of its nodes
 * joined to a fan of triangles on each face (a quadrilateral's fan starts at
 * its first node).  fn(P, vol) gets the 4 x 3 vertices and the volume of
 * each. */
template <class Fn>
void for_each_cone(const cgks_ctx* c, const HLevel& L, int i, Fn fn) {
    const int off = L.noff[i], cnt = L.noff[i + 1] - off;
    const ElemTable* et = element(cnt);
    const double* X = c->coords.data();
    double m[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < cnt; ++j)
        for (int d = 0; d < 3; ++d) m[d] += X[(size_t)L.nodes[off + j] * 3 + d];
    for (int d = 0; d < 3; ++d) m[d] /= cnt;
    for (int fc = 0; fc < et->nface; ++fc)
        for (int t = 1; t + 1 < et->cnt[fc]; ++t) {
            double P[12];
            const int ids[3] = {et->node[fc][0], et->node[fc][t], et->node[fc][t + 1]};
            for (int d = 0; d < 3; ++d) {
                P[d] = m[d];
                for (int v = 0; v < 3; ++v) P[3 * (v + 1) + d] = X[(size_t)L.nodes[off + ids[v]] * 3 + d];
            }
            double e[3][3];
            for (int v = 0; v < 3; ++v)
                for (int d = 0; d < 3; ++d) e[v][d] = P[3 * (v + 1) + d] - P[d];
            const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                               e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                               e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
            fn(P, std::fabs(det) / 6.0);
        }
}

/* Averages over hybrid cell j of the 9 scaled monomials about (xc, h), in
 * one pass over the symmetric 4-point rule of each of its tetrahedra. */
void hybrid_basis_averages(const cgks_ctx* c, const HLevel& L, int j, const double* xc, double h, double* out) {
    const double al = 0.5854101966249685, be = 0.1381966011250105;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, vol = 0.0;
    for_each_cone(c, L, j, [&](const double* P, double v) {
        double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int a = 0; a < 4; ++a) {
            double X[3];
            for (int d = 0; d < 3; ++d) {
                double x = 0.0;
                for (int q = 0; q < 4; ++q) x += (q == a ? al : be) * P[q * 3 + d];
                X[d] = (x - xc[d]) / h;
            }
            const double phi[9] = {X[0], X[1], X[2], X[0] * X[0], X[0] * X[1], X[0] * X[2], X[1] * X[1], X[1] * X[2], X[2] * X[2]};
            for (int k = 0; k < 9; ++k) s[k] += phi[k];
        }
        for (int k = 0; k < 9; ++k) acc[k] += v * (0.25 * s[k]);
        vol += v;
    });
    for (int k = 0; k < 9; ++k) out[k] = acc[k] / vol;
}

/* Cell average of f over fine cell i (exact for quadratics). */
template <class Fn>
double cell_average(const cgks_ctx* c, const HLevel& L, int i, Fn f) {
    if (!c->hybrid) {
        double P[12];
        cell_vertices(c, L, i, P);
        return simplex_average(c->dim, P, f);
    }
    double acc = 0.0, vol = 0.0;
    for_each_cone(c, L, i, [&](const double* P, double v) {
        acc += v * simplex_average(3, P, f);
        vol += v;
    });
    return acc / vol;
}

/* Planar quadrilateral face with node cycle x0..x3: area vector
 * (x2 - x0) x (x3 - x1) / 2, centre from the triangles (x0, x1, x2) and
 * (x0, x2, x3), and the 2 x 2 Gauss points of the bilinear map from
 * [-1, 1]^2 with weights proportional to the map's area element.  False when
 * x3 is off the plane of the others. */
bool quad_face(const double* const* x, HFace& F) {
    auto cr = [](const double* a, const double* b, double* o) {
        o[0] = a[1] * b[2] - a[2] * b[1];
        o[1] = a[2] * b[0] - a[0] * b[2];
        o[2] = a[0] * b[1] - a[1] * b[0];
    };
    auto len = [](const double* a) { return std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); };
    double d02[3], d13[3], A[3];
    for (int d = 0; d < 3; ++d) {
        d02[d] = x[2][d] - x[0][d];
        d13[d] = x[3][d] - x[1][d];
    }
    cr(d02, d13, A);
    const double la = len(A);
    F.S = 0.5 * la;
    for (int d = 0; d < 3; ++d) F.n[d] = A[d] / la;
    double h = 0.0;
    for (int d = 0; d < 3; ++d) h += F.n[d] * (x[3][d] - x[0][d]);
    if (std::fabs(h) > 1e-9 * std::sqrt(F.S)) return false;
    double e1[3], e3[3], t1[3], t2[3];
    for (int d = 0; d < 3; ++d) {
        e1[d] = x[1][d] - x[0][d];
        e3[d] = x[3][d] - x[0][d];
    }
    cr(e1, d02, t1);
    cr(d02, e3, t2);
    const double a1 = len(t1), a2 = len(t2);
    for (int d = 0; d < 3; ++d)
        F.xc[d] = (a1 * (x[0][d] + x[1][d] + x[2][d]) + a2 * (x[0][d] + x[2][d] + x[3][d])) / (3.0 * (a1 + a2));
    F.ngp = 4;
    const double r = 1.0 / std::sqrt(3.0);
    const double su[4] = {-r, r, r, -r}, sv[4] = {-r, -r, r, r};
    double jw[4], jt = 0.0;
    for (int g = 0; g < 4; ++g) {
        const double N[4] = {(1 - su[g]) * (1 - sv[g]), (1 + su[g]) * (1 - sv[g]), (1 + su[g]) * (1 + sv[g]),
                             (1 - su[g]) * (1 + sv[g])};
        const double Nu[4] = {-(1 - sv[g]), 1 - sv[g], 1 + sv[g], -(1 + sv[g])};
        const double Nv[4] = {-(1 - su[g]), -(1 + su[g]), 1 + su[g], 1 - su[g]};
        double xu[3] = {0, 0, 0}, xv[3] = {0, 0, 0}, J[3];
        for (int d = 0; d < 3; ++d) {
            double p = 0.0;
            for (int k = 0; k < 4; ++k) {
                p += N[k] * x[k][d];
                xu[d] += Nu[k] * x[k][d];
                xv[d] += Nv[k] * x[k][d];
            }
            F.gp[g][d] = 0.25 * p;
        }
        cr(xu, xv, J);
        jw[g] = len(J);
        jt += jw[g];
    }
    for (int g = 0; g < 4; ++g) F.w[g] = jw[g] / jt;
    return true;
}

/* Reconstruction operator of fine cell i in slot layout: column
 * s*(1+dim)+0 multiplies (Q_nbr(s) - Q_i), column s*(1+dim)+1+d the
 * neighbour's slope d; empty slots (boundary faces) have zero columns. */
void build_operator(cgks_ctx* c, int i) {
    const int dim = c->dim;
    HLevel& L = c->hl[0];
    const int nq = (dim == 2) ? 5 : 9, nslot = (int)L.cf[i].size(), ncol = L.nslot * (1 + dim);
    const double* xc = &L.C[i * dim];
    const double h = L.h[i];
    /* averages of the scaled monomials about (xc, h) over cell j */
    auto averages = [&](int j, double* out) {
        if (c->hybrid) {
            hybrid_basis_averages(c, L, j, xc, h, out);
            return;
        }
        for (int k = 0; k < nq; ++k) out[k] = cell_average(c, L, j, [&](const double* x) { return mono(dim, k, x, xc, h); });
    };
    double own[9];
    averages(i, own);
    for (int k = 0; k < nq; ++k) L.mean0[(size_t)k * L.n + i] = own[k];
    std::vector<int> slots, nbrs;
    for (int s = 0; s < nslot; ++s) {
        const HFace& f = L.faces[L.cf[i][s]];
        if (f.R < 0) continue;
        slots.push_back(s);
        nbrs.push_back(f.L == i ? f.R : f.L);
    }
    const int nn = (int)nbrs.size();
    std::vector<double> navg((size_t)nn * nq);
    for (int m = 0; m < nn; ++m) averages(nbrs[m], &navg[(size_t)m * nq]);
    int nb = 0;
    if (nn * (1 + dim) >= nq) nb = nq;
    else if (nn * (1 + dim) >= dim) nb = dim;
    for (;;) {
        if (nb == 0) break;
        std::vector<double> E((size_t)nn * nb), A((size_t)nn * dim * nb);
        std::vector<double> w(nn);
        for (int m = 0; m < nn; ++m) {
            int j = nbrs[m];
            const double* xj = &L.C[j * dim];
            double r2 = 0.0;
            for (int d = 0; d < dim; ++d) r2 += (xj[d] - xc[d]) * (xj[d] - xc[d]);
            w[m] = std::sqrt(r2);
            for (int k = 0; k < nb; ++k) {
                E[m * nb + k] = navg[(size_t)m * nq + k] - L.mean0[(size_t)k * L.n + i];
                for (int d = 0; d < dim; ++d) A[(m * dim + d) * nb + k] = w[m] * mono_dx(dim, k, d, xj, xc, h);
            }
        }
        std::vector<double> Md, Mb;
        if (null_space_ls(nb, nn, nn * dim, E, A, Md, Mb)) {
            for (int m = 0; m < nn; ++m) {
                int s = slots[m];
                for (int k = 0; k < nb; ++k) {
                    L.op[((size_t)k * ncol + s * (1 + dim)) * L.n + i] = Md[k * nn + m];
                    for (int d = 0; d < dim; ++d)
                        L.op[((size_t)k * ncol + s * (1 + dim) + 1 + d) * L.n + i] = Mb[k * (nn * dim) + m * dim + d] * w[m];
                }
            }
            break;
        }
        nb = (nb == nq) ? dim : 0;
    }
    L.nbasis[i] = nb;
}

/* Alg. 1: breadth-first greedy painting from cell 0 (neighbours in local face order). */
int paint(const std::vector<std::vector<int>>& nb, std::vector<int>& color) {
    const int n = (int)nb.size();
    color.assign(n, 0);
    int ncolor = 0;
    std::vector<char> used;
    auto smallest_free = [&](int w) {
        used.assign(nb[w].size() + 2, 0);
        for (int j : nb[w])
            if (color[j] > 0 && color[j] < (int)used.size()) used[color[j]] = 1;
        int k = 1;
        while (k < (int)used.size() && used[k]) ++k;
        return k;
    };
    std::deque<int> q;
    for (int s = 0; s < n; ++s) {
        if (color[s]) continue;
        color[s] = smallest_free(s);
        ncolor = std::max(ncolor, color[s]);
        q.push_back(s);
        while (!q.empty()) {
            int v = q.front();
            q.pop_front();
            for (int w : nb[v]) {
                if (color[w]) continue;
                color[w] = smallest_free(w);
                ncolor = std::max(ncolor, color[w]);
                q.push_back(w);
            }
        }
    }
    return ncolor;
}

std::vector<std::vector<int>> neighbours(const HLevel& L) {
    std::vector<std::vector<int>> nb(L.n);
    for (int i = 0; i < L.n; ++i)
        for (int f : L.cf[i]) {
            const HFace& F = L.faces[f];
            if (F.R >= 0) nb[i].push_back(F.L == i ? F.R : F.L);
        }
    return nb;
}

/* Agglomerate faces: area vector sums of the finer level's faces between two
 * agglomerates, one group per (agglomerate, tag) on the boundary. */
void coarse_faces(cgks_ctx* c, int l) {
    const int dim = c->dim;
    const HLevel& F = c->hl[l - 1];
    HLevel& G = c->hl[l];
    struct Acc {
        int L, R, tag;
        double Sv[3], xs[3], Ssum;
    };
    std::vector<Acc> acc;
    std::unordered_map<uint64_t, int> idx;
    for (const HFace& f : F.faces) {
        int I = F.parent[f.L];
        int J = (f.R >= 0) ? F.parent[f.R] : -1;
        if (J == I) continue;
        uint64_t key;
        double sg = 1.0;
        int lo = I, hi = J;
        if (J >= 0) {
            lo = std::min(I, J);
            hi = std::max(I, J);
            sg = (I == lo) ? 1.0 : -1.0;
            key = ((uint64_t)lo << 32) | (uint64_t)(uint32_t)hi;
        } else {
            key = ((uint64_t)I << 32) | (uint64_t)(0x80000000u | (uint32_t)f.tag);
        }
        auto it = idx.find(key);
        int a;
        if (it == idx.end()) {
            a = (int)acc.size();
            idx[key] = a;
            Acc z;
            std::memset(&z, 0, sizeof(z));
            z.L = lo;
            z.R = (J >= 0) ? hi : -1;
            z.tag = (J >= 0) ? 0 : f.tag;
            acc.push_back(z);
        } else {
            a = it->second;
        }
        for (int d = 0; d < dim; ++d) {
            acc[a].Sv[d] += sg * f.S * f.n[d];
            acc[a].xs[d] += f.S * f.xc[d];
        }
        acc[a].Ssum += f.S;
    }
    std::sort(acc.begin(), acc.end(), [](const Acc& x, const Acc& y) {
        if (x.L != y.L) return x.L < y.L;
        long kx = x.R >= 0 ? x.R : (1L << 40) + x.tag, ky = y.R >= 0 ? y.R : (1L << 40) + y.tag;
        return kx < ky;
    });
    G.faces.resize(acc.size());
    for (size_t k = 0; k < acc.size(); ++k) {
        HFace& f = G.faces[k];
        std::memset(&f, 0, sizeof(f));
        f.L = acc[k].L;
        f.R = acc[k].R;
        f.tag = acc[k].tag;
        double s2 = 0.0;
        for (int d = 0; d < dim; ++d) s2 += acc[k].Sv[d] * acc[k].Sv[d];
        f.S = std::sqrt(s2);
        for (int d = 0; d < dim; ++d) {
            f.n[d] = acc[k].Sv[d] / f.S;
            f.xc[d] = acc[k].xs[d] / acc[k].Ssum;
        }
    }
    /* Local face order: interior neighbours by index, then boundary groups by tag. */
    std::vector<std::vector<std::pair<long, int>>> lst(G.n);
    for (int k = 0; k < (int)G.faces.size(); ++k) {
        const HFace& f = G.faces[k];
        if (f.R >= 0) {
            lst[f.L].push_back({(long)f.R, k});
            lst[f.R].push_back({(long)f.L, k});
        } else {
            lst[f.L].push_back({(1L << 40) + f.tag, k});
        }
    }
    G.cf.assign(G.n, {});
    G.nslot = 0;
    for (int i = 0; i < G.n; ++i) {
        std::sort(lst[i].begin(), lst[i].end());
        for (auto& e : lst[i]) G.cf[i].push_back(e.second);
        G.nslot = std::max(G.nslot, (int)G.cf[i].size());
    }
}

}  // namespace

int agglomerate_level(const cgks_ctx* c, int level, std::vector<int>& agg) {
    /* Alg. 3 with face hashes h = (23 (L+R) + L R) mod N_f over interior faces in
     * canonical order; a hashed face merges its two cells when neither is merged
     * yet and every other face of the pair passes the skewness limit. */
    const int dim = c->dim;
    const HLevel& L = c->hl[level];
    std::vector<int> inter;
    for (int f = 0; f < (int)L.faces.size(); ++f)
        if (L.faces[f].R >= 0) inter.push_back(f);
    const uint64_t Nf = inter.size();
    std::unordered_set<uint64_t> table;
    std::vector<int> owner(L.n, -1);
    std::vector<int> candidates;
    for (int f : inter) {
        uint64_t a = (uint64_t)L.faces[f].L, b = (uint64_t)L.faces[f].R;
        uint64_t h = (23u * (a + b) + a * b) % Nf;
        if (table.insert(h).second) candidates.push_back(f);
    }
    for (int f : candidates) {
        const HFace& F = L.faces[f];
        if (owner[F.L] >= 0 || owner[F.R] >= 0) continue;
        const double VL = L.V[F.L], VR = L.V[F.R];
        double cc[3];
        for (int d = 0; d < dim; ++d) cc[d] = (VL * L.C[F.L * dim + d] + VR * L.C[F.R * dim + d]) / (VL + VR);
        bool ok = true;
        for (int cell : {F.L, F.R}) {
            for (int g : L.cf[cell]) {
                if (g == f) continue;
                const HFace& G = L.faces[g];
                const double sgn = (G.L == cell) ? 1.0 : -1.0;
                double dn = 0.0, dd = 0.0;
                for (int d = 0; d < dim; ++d) {
                    const double v = G.xc[d] - cc[d];
                    dn += v * (sgn * G.n[d]);
                    dd += v * v;
                }
                if (!(dn / std::sqrt(dd) >= c->p.skew_limit)) ok = false;
            }
        }
        if (ok) owner[F.L] = owner[F.R] = f;
    }
    agg.assign(L.n, -1);
    std::unordered_map<int, int> id;
    int next = 0;
    for (int i = 0; i < L.n; ++i) {
        if (owner[i] < 0) {
            agg[i] = next++;
            continue;
        }
        auto it = id.find(owner[i]);
        if (it == id.end()) {
            id[owner[i]] = next;
            agg[i] = next++;
        } else {
            agg[i] = it->second;
        }
    }
    return next;
}

int setup_host(cgks_ctx* c, const cgks_mesh* m, int n_levels, const int32_t* const* parent) {
    const int dim = m->dim;
    if (dim != c->dim) return fail(c, CGKS_EINVAL, "mesh dimension differs from params.dim");
    if (n_levels < 1 || n_levels > 8) return fail(c, CGKS_EINVAL, "n_levels out of range");
    if (m->n_cells <= 0 || m->n_nodes <= 0 || !m->coords || !m->cell_nodes)
        return fail(c, CGKS_EINVAL, "empty mesh");
    const bool mixed = m->cell_offsets != nullptr;
    if (mixed != (m->bface_offsets != nullptr))
        return fail(c, CGKS_EINVAL, "cell_offsets and bface_offsets must be given together");
    if (mixed && dim != 3) return fail(c, CGKS_EINVAL, "mixed elements are 3-D only");
    c->hybrid = mixed;
    c->coords.assign(m->coords, m->coords + (size_t)m->n_nodes * dim);
    c->hl.assign(n_levels, HLevel());
    HLevel& L = c->hl[0];
    L.n = m->n_cells;
    if (mixed) {
        L.noff.assign(m->cell_offsets, m->cell_offsets + L.n + 1);
        if (L.noff[0] != 0) return fail(c, CGKS_EMESH, "cell_offsets[0] is not 0");
        for (int i = 0; i < L.n; ++i)
            if (!element(L.noff[i + 1] - L.noff[i]))
                return fail(c, CGKS_EMESH, "cell " + std::to_string(i) + ": node count other than 4, 5, 6 or 8");
        L.nodes.assign(m->cell_nodes, m->cell_nodes + L.noff[L.n]);
    } else {
        L.nodes.assign(m->cell_nodes, m->cell_nodes + (size_t)L.n * (dim + 1));
    }
    L.V.resize(L.n);
    L.C.resize((size_t)L.n * dim);
    L.h.resize(L.n);
    const double* X = c->coords.data();
    for (int i = 0; i < L.n; ++i) {
        const int* v = mixed ? &L.nodes[L.noff[i]] : &L.nodes[(size_t)i * (dim + 1)];
        const int nv = mixed ? L.noff[i + 1] - L.noff[i] : dim + 1;
        for (int j = 0; j < nv; ++j)
            if (v[j] < 0 || v[j] >= m->n_nodes) return fail(c, CGKS_EMESH, "cell node out of range");
        if (mixed) {
            double vol = 0.0, mom[3] = {0.0, 0.0, 0.0};
            for_each_cone(c, L, i, [&](const double* P, double cv) {
                vol += cv;
                for (int d = 0; d < 3; ++d) mom[d] += cv * (((P[d] + P[3 + d]) + P[6 + d]) + P[9 + d]) / 4.0;
            });
            L.V[i] = vol;
            for (int d = 0; d < 3; ++d) L.C[i * 3 + d] = mom[d] / vol;
            L.h[i] = std::cbrt(vol);
        } else if (dim == 2) {
            const double *a = X + 2 * v[0], *b = X + 2 * v[1], *e = X + 2 * v[2];
            L.V[i] = 0.5 * ((b[0] - a[0]) * (e[1] - a[1]) - (e[0] - a[0]) * (b[1] - a[1]));
            for (int d = 0; d < 2; ++d) L.C[i * 2 + d] = ((a[d] + b[d]) + e[d]) / 3.0;
            L.h[i] = std::sqrt(L.V[i]);
        } else {
            const double *a = X + 3 * v[0], *b = X + 3 * v[1], *e = X + 3 * v[2], *g = X + 3 * v[3];
            double u[3], w[3], z[3];
            for (int d = 0; d < 3; ++d) {
                u[d] = b[d] - a[d];
                w[d] = e[d] - a[d];
                z[d] = g[d] - a[d];
            }
            double det = u[0] * (w[1] * z[2] - w[2] * z[1]) - u[1] * (w[0] * z[2] - w[2] * z[0]) +
                         u[2] * (w[0] * z[1] - w[1] * z[0]);
            L.V[i] = det / 6.0;
            for (int d = 0; d < 3; ++d) L.C[i * 3 + d] = (((a[d] + b[d]) + e[d]) + g[d]) / 4.0;
            L.h[i] = std::cbrt(L.V[i]);
        }
        if (!(L.V[i] > 0.0)) return fail(c, CGKS_EMESH, "cell " + std::to_string(i) + " has non-positive volume");
    }
    /* Faces: match cell faces through a hash map of sorted node tuples. */
    std::unordered_map<FaceKey, int, FaceKeyHash> fmap;
    fmap.reserve((size_t)L.n * (dim + 1));
    std::vector<FaceKey> keys;
    std::vector<std::array<int, 2>> cells;
    std::vector<int> cnt;
    std::vector<std::array<int, 2>> cellslot;
    /* node ids of local face k of cell i, in the element's cycle */
    auto face_nodes = [&](int i, int k, int* ids) {
        if (!mixed) {
            int t = 0;
            for (int j = 0; j <= dim; ++j)
                if (j != k) ids[t++] = L.nodes[(size_t)i * (dim + 1) + j];
            return dim;
        }
        const ElemTable* et = element(L.noff[i + 1] - L.noff[i]);
        for (int j = 0; j < et->cnt[k]; ++j) ids[j] = L.nodes[L.noff[i] + et->node[k][j]];
        return et->cnt[k];
    };
    L.cf.assign(L.n, {});
    for (int i = 0; i < L.n; ++i) {
        const int nfc = mixed ? element(L.noff[i + 1] - L.noff[i])->nface : dim + 1;
        L.cf[i].assign(nfc, -1);
        for (int k = 0; k < nfc; ++k) {
            int ids[4];
            const int cnt_k = face_nodes(i, k, ids);
            FaceKey key = make_key(ids, cnt_k);
            auto it = fmap.find(key);
            if (it == fmap.end()) {
                fmap.emplace(key, (int)keys.size());
                keys.push_back(key);
                cells.push_back({i, -1});
                cellslot.push_back({k, -1});
                cnt.push_back(1);
            } else {
                int f = it->second;
                if (cnt[f] >= 2) return fail(c, CGKS_EMESH, "non-manifold face");
                cells[f][1] = i;
                cellslot[f][1] = k;
                cnt[f] = 2;
            }
        }
    }
    std::vector<int> order(keys.size());
    for (size_t f = 0; f < keys.size(); ++f) order[f] = (int)f;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return keys[a] < keys[b]; });
    std::unordered_map<FaceKey, int, FaceKeyHash> btag;
    for (int b = 0; b < m->n_bfaces; ++b) {
        const int b0 = mixed ? m->bface_offsets[b] : b * dim;
        const int bc = mixed ? m->bface_offsets[b + 1] - b0 : dim;
        if (bc < dim || bc > 4) return fail(c, CGKS_EMESH, "boundary face with a bad node count");
        FaceKey key = make_key(m->bface_nodes + b0, bc);
        btag[key] = m->bface_tag[b];
    }
    L.faces.resize(keys.size());
    int nmatched = 0;
    for (size_t o = 0; o < order.size(); ++o) {
        const int f = order[o];
        HFace& F = L.faces[o];
        std::memset(&F, 0, sizeof(F));
        int c0 = cells[f][0], c1 = cells[f][1];
        if (c1 >= 0) {
            F.L = std::min(c0, c1);
            F.R = std::max(c0, c1);
            F.tag = 0;
        } else {
            F.L = c0;
            F.R = -1;
            auto it = btag.find(keys[f]);
            if (it == btag.end()) return fail(c, CGKS_EMESH, "boundary face without a tag");
            F.tag = it->second;
            if (F.tag < CGKS_TAG_FARFIELD || F.tag > CGKS_TAG_ADIABATIC) return fail(c, CGKS_EMESH, "unknown boundary tag");
            ++nmatched;
        }
        L.cf[c0][cellslot[f][0]] = (int)o;
        if (c1 >= 0) L.cf[c1][cellslot[f][1]] = (int)o;
        const int* k = keys[f].v;
        const double* CL = &L.C[(size_t)F.L * dim];
        int cyc[4];
        const int ncyc = face_nodes(c0, cellslot[f][0], cyc);
        if (mixed) k = cyc;   /* Gauss points in the order of the first cell's cycle */
        for (int g = 0; g < 4; ++g) F.w[g] = 0.0;
        if (mixed && ncyc == 4) {
            const double* x[4] = {X + 3 * cyc[0], X + 3 * cyc[1], X + 3 * cyc[2], X + 3 * cyc[3]};
            if (!quad_face(x, F)) return fail(c, CGKS_EMESH, "non-planar quadrilateral face");
        } else if (dim == 2) {
            const double *a = X + 2 * k[0], *b = X + 2 * k[1];
            const double dx = b[0] - a[0], dy = b[1] - a[1];
            F.S = std::sqrt(dx * dx + dy * dy);
            F.n[0] = dy / F.S;
            F.n[1] = -dx / F.S;
            F.xc[0] = 0.5 * (a[0] + b[0]);
            F.xc[1] = 0.5 * (a[1] + b[1]);
            F.ngp = 2;
            F.w[0] = F.w[1] = 0.5;
            const double t[2] = {0.5 - std::sqrt(3.0) / 6.0, 0.5 + std::sqrt(3.0) / 6.0};
            for (int g = 0; g < 2; ++g) {
                F.gp[g][0] = a[0] + t[g] * dx;
                F.gp[g][1] = a[1] + t[g] * dy;
            }
        } else {
            const double *a = X + 3 * k[0], *b = X + 3 * k[1], *e = X + 3 * k[2];
            double u[3], w[3], N[3];
            for (int d = 0; d < 3; ++d) {
                u[d] = b[d] - a[d];
                w[d] = e[d] - a[d];
            }
            N[0] = u[1] * w[2] - u[2] * w[1];
            N[1] = u[2] * w[0] - u[0] * w[2];
            N[2] = u[0] * w[1] - u[1] * w[0];
            const double len = std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
            F.S = 0.5 * len;
            for (int d = 0; d < 3; ++d) {
                F.n[d] = N[d] / len;
                F.xc[d] = ((a[d] + b[d]) + e[d]) / 3.0;
            }
            F.ngp = 3;
            F.w[0] = F.w[1] = F.w[2] = 1.0 / 3.0;
            const double hi = 2.0 / 3.0, lo = 1.0 / 6.0;
            for (int g = 0; g < 3; ++g)
                for (int d = 0; d < 3; ++d)
                    F.gp[g][d] = (g == 0 ? hi : lo) * a[d] + (g == 1 ? hi : lo) * b[d] + (g == 2 ? hi : lo) * e[d];
        }
        double dot = 0.0;
        for (int d = 0; d < dim; ++d) dot += F.n[d] * (F.xc[d] - CL[d]);
        if (dot < 0.0)
            for (int d = 0; d < dim; ++d) F.n[d] = -F.n[d];
    }
    if (nmatched != m->n_bfaces) return fail(c, CGKS_EMESH, "a tagged boundary face is not on the boundary");
    L.nslot = mixed ? 6 : dim + 1;
    /* Coarse levels from parent maps (or Alg. 3). */
    for (int l = 1; l < n_levels; ++l) {
        HLevel& F = c->hl[l - 1];
        HLevel& G = c->hl[l];
        if (parent && parent[l - 1]) {
            F.parent.assign(parent[l - 1], parent[l - 1] + F.n);
        } else {
            agglomerate_level(c, l - 1, F.parent);
        }
        int nc = 0;
        for (int i = 0; i < F.n; ++i) {
            if (F.parent[i] < 0) return fail(c, CGKS_EMESH, "negative parent index");
            nc = std::max(nc, F.parent[i] + 1);
        }
        G.n = nc;
        G.children.assign(nc, {});
        for (int i = 0; i < F.n; ++i) G.children[F.parent[i]].push_back(i);
        G.V.assign(nc, 0.0);
        G.C.assign((size_t)nc * dim, 0.0);
        for (int I = 0; I < nc; ++I) {
            if (G.children[I].empty()) return fail(c, CGKS_EMESH, "empty agglomerate");
            double V = 0.0, m1[3] = {0, 0, 0};
            for (int i : G.children[I]) {
                V += F.V[i];
                for (int d = 0; d < dim; ++d) m1[d] += F.V[i] * F.C[(size_t)i * dim + d];
            }
            G.V[I] = V;
            for (int d = 0; d < dim; ++d) G.C[(size_t)I * dim + d] = m1[d] / V;
        }
        coarse_faces(c, l);
    }
    /* Colours and internal orders. */
    for (int l = 0; l < n_levels; ++l) {
        HLevel& H = c->hl[l];
        H.ncolor = paint(neighbours(H), H.color);
        H.perm.resize(H.n);
        for (int i = 0; i < H.n; ++i) H.perm[i] = i;
        if (l > 0)
            std::stable_sort(H.perm.begin(), H.perm.end(), [&](int a, int b) { return H.color[a] < H.color[b]; });
        H.iperm.resize(H.n);
        for (int i = 0; i < H.n; ++i) H.iperm[H.perm[i]] = i;
        H.color_off.assign(H.ncolor + 1, 0);
        for (int i = 0; i < H.n; ++i) H.color_off[H.color[i]]++;
        for (int k = 1; k <= H.ncolor; ++k) H.color_off[k] += H.color_off[k - 1];
    }
    /* Reconstruction operators of the fine level. */
    const int nq = (dim == 2) ? 5 : 9;
    L.mean0.assign((size_t)nq * L.n, 0.0);
    L.op.assign((size_t)nq * L.nslot * (1 + dim) * L.n, 0.0);
    L.nbasis.assign(L.n, 0);
    for (int i = 0; i < L.n; ++i) build_operator(c, i);
    return CGKS_OK;
}

}  // namespace cgks

/*
 * Algorithmic FP64 operation count of the Gauss-point BGK flux (gks_flux):
 * the device source is compiled for the host with every `double` replaced by
 * a counting number type, and evaluated once on a representative state.
 * +, -, *, / each count one operation; sqrt, exp, expm1, erfc and pow count
 * one each (reported separately); fabs, fmin/fmax, negation and comparisons
 * count zero.  Measurement tool only: not part of libcgks.
 */
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#include "cgks_internal.h"

static long n_add = 0, n_mul = 0, n_div = 0, n_sqrt = 0, n_trans = 0;

struct Counted {
    double v;
    Counted() : v(0.0) {}
    Counted(double x) : v(x) {}
    Counted& operator+=(Counted o) { ++n_add; v += o.v; return *this; }
    Counted& operator-=(Counted o) { ++n_add; v -= o.v; return *this; }
    Counted& operator*=(Counted o) { ++n_mul; v *= o.v; return *this; }
    Counted& operator/=(Counted o) { ++n_div; v /= o.v; return *this; }
};
static inline Counted operator+(Counted a, Counted b) { ++n_add; return Counted(a.v + b.v); }
static inline Counted operator-(Counted a, Counted b) { ++n_add; return Counted(a.v - b.v); }
static inline Counted operator*(Counted a, Counted b) { ++n_mul; return Counted(a.v * b.v); }
static inline Counted operator/(Counted a, Counted b) { ++n_div; return Counted(a.v / b.v); }
static inline Counted operator-(Counted a) { return Counted(-a.v); }
static inline bool operator<(Counted a, Counted b) { return a.v < b.v; }
static inline bool operator>(Counted a, Counted b) { return a.v > b.v; }
static inline bool operator<=(Counted a, Counted b) { return a.v <= b.v; }
static inline bool operator>=(Counted a, Counted b) { return a.v >= b.v; }
static inline Counted sqrt(Counted a) { ++n_sqrt; return Counted(std::sqrt(a.v)); }
static inline Counted exp(Counted a) { ++n_trans; return Counted(std::exp(a.v)); }
static inline Counted expm1(Counted a) { ++n_trans; return Counted(std::expm1(a.v)); }
static inline Counted erfc(Counted a) { ++n_trans; return Counted(std::erfc(a.v)); }
static inline Counted pow(Counted a, Counted b) { ++n_trans; return Counted(std::pow(a.v, b.v)); }
static inline Counted fabs(Counted a) { return Counted(std::fabs(a.v)); }
static inline Counted fmin(Counted a, Counted b) { return Counted(std::fmin(a.v, b.v)); }
static inline Counted fmax(Counted a, Counted b) { return Counted(std::fmax(a.v, b.v)); }

#define double Counted
#include "kinetic.hpp"
#undef double

int main() {
    for (int ns = 0; ns < 2; ++ns) {
        cgks::KParams kp{};
        kp.dim = 2; kp.gamma = 1.4; kp.K = 3.0; kp.prandtl = 0.72; kp.mach = 8.0;
        kp.reynolds = ns ? 1e4 : 0.0; kp.mu_inf = ns ? 8e-4 : 0.0; kp.Tinf = 1 / 1.4;
        kp.S_suth = 0.5 / 1.4; kp.Tw = 1 / 1.4; kp.tau_c1 = 0.01; kp.tau_c2 = 1.0;
        Counted WL[4] = {1.0, 0.5, 0.1, 2.0}, WR[4] = {0.9, 0.4, 0.05, 1.8};
        Counted gL[4][2] = {{0.1, 0.0}, {0.1, 0.2}, {0.0, 0.1}, {0.3, 0.1}};
        Counted gR[4][2] = {{0.05, 0.0}, {0.1, 0.1}, {0.0, 0.2}, {0.2, 0.1}};
        Counted n[2] = {0.6, 0.8};
        Counted F[4], G[4], a;
        n_add = n_mul = n_div = n_sqrt = n_trans = 0;
        cgks::gks_flux<2>(kp, WL, gL, WR, gR, n, Counted(1e-3), F, G, &a);
        long tot = n_add + n_mul + n_div + n_sqrt + n_trans;
        printf("%s add=%ld mul=%ld div=%ld sqrt=%ld transcendental=%ld total=%ld\n", ns ? "ns" : "euler",
               n_add, n_mul, n_div, n_sqrt, n_trans, tot);
    }
    return 0;
}

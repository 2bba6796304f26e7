// Operation count of the FP64 oracle's rollout (TEST INFRASTRUCTURE, like the oracle):
// mppi_oracle.c compiled once more as C++ with its scalar type replaced by Real, a
// double that counts the floating-point operations done on it.  Nothing here is
// arithmetic of the method; it only tallies what the oracle's own code executes.
//
// Counted: add, sub, mul, div (1 each; the oracle is compiled without FMA contraction,
// so it has no fused multiply-adds), and sqrt, log, exp, sin, cos separately.
// Negation, comparisons, fabs and conversions are not counted.
//
// Output (one JSON object on stdout): the counts of
//   rollout(N, M)      orc_rollout_one for one sample, N steps, M obstacles of one type
//   allocation         orc_allocation (Eq. (11), built from l and c_tf)
//   allocation_inverse orc_allocation_inverse (Gauss-Jordan)
//   noise              orc_noise_one (uniforms, Box-Muller, scaling by sigma)
// from which the per-step and per-obstacle-test work is read off by differences.
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

struct Tally {
    long long add = 0, mul = 0, div = 0, sqrt_ = 0, log_ = 0, exp_ = 0, sin_ = 0, cos_ = 0;
    long long flop() const { return add + mul + div; }
};
static Tally g_tally;

struct Real {
    double v;
    Real() = default;
    Real(double x) : v(x) {}
    explicit operator double() const { return v; }
    explicit operator int() const { return (int)v; }
    Real& operator+=(Real o) { ++g_tally.add; v += o.v; return *this; }
    Real& operator-=(Real o) { ++g_tally.add; v -= o.v; return *this; }
    Real& operator*=(Real o) { ++g_tally.mul; v *= o.v; return *this; }
    Real& operator/=(Real o) { ++g_tally.div; v /= o.v; return *this; }
};
static inline Real operator+(Real a, Real b) { ++g_tally.add; return Real(a.v + b.v); }
static inline Real operator-(Real a, Real b) { ++g_tally.add; return Real(a.v - b.v); }
static inline Real operator*(Real a, Real b) { ++g_tally.mul; return Real(a.v * b.v); }
static inline Real operator/(Real a, Real b) { ++g_tally.div; return Real(a.v / b.v); }
static inline Real operator-(Real a) { return Real(-a.v); }
static inline bool operator<(Real a, Real b) { return a.v < b.v; }
static inline bool operator>(Real a, Real b) { return a.v > b.v; }
static inline bool operator<=(Real a, Real b) { return a.v <= b.v; }
static inline bool operator>=(Real a, Real b) { return a.v >= b.v; }
static inline bool operator==(Real a, Real b) { return a.v == b.v; }
static inline bool operator!=(Real a, Real b) { return a.v != b.v; }
static inline Real sqrt(Real a) { ++g_tally.sqrt_; return Real(::sqrt(a.v)); }
static inline Real log(Real a) { ++g_tally.log_; return Real(::log(a.v)); }
static inline Real exp(Real a) { ++g_tally.exp_; return Real(::exp(a.v)); }
static inline Real sin(Real a) { ++g_tally.sin_; return Real(::sin(a.v)); }
static inline Real cos(Real a) { ++g_tally.cos_; return Real(::cos(a.v)); }
static inline Real fabs(Real a) { return Real(::fabs(a.v)); }
static inline Real ceil(Real a) { return Real(::ceil(a.v)); }
static inline bool isfinite(Real a) { return ::isfinite(a.v); }

#define double Real
#include "mppi_oracle.c"
#undef double

static void print_tally(const char* name, const Tally& t, bool last = false)
{
    printf("  \"%s\": {\"add\": %lld, \"mul\": %lld, \"div\": %lld, \"sqrt\": %lld, \"log\": %lld, "
           "\"exp\": %lld, \"sin\": %lld, \"cos\": %lld, \"flop\": %lld}%s\n",
           name, t.add, t.mul, t.div, t.sqrt_, t.log_, t.exp_, t.sin_, t.cos_, t.flop(), last ? "" : ",");
}

int main()
{
    // benchmark vehicle (rotor lag on) and cost; a state off the reference
    const Real veh[13] = {1.0, 0.01, 0.01, 0.02, 0.15, 0.012, 9.81, 0.0, 8.0, 0.03, 0.0, 0.0, 0.0};
    const Real cost[15] = {400.0, 40.0, 20.0, 20.0, 0.01, 0.05, 0.05, 0.10,
                             0.05, 0.10, 0.10, 0.30, 0.3, 1.0e3, 1.0e4};
    Real x_hat[17] = {0.0, 0.0, 2.0, 1.0, 0.0, 0.0, 0.0, 1.0, 0.5, -0.2, 0.1, -0.1, 0.2,
                        2.45, 2.45, 2.45, 2.45};
    const Real sigma[4] = {1.0, 1.0, 1.0, 1.0};
    enum { NMAX = 4, MMAX = 2 };
    Real u_nom[NMAX * 4], x_ref[(NMAX + 1) * 13], du[NMAX * 4];
    for (int j = 0; j < NMAX; ++j) {
        u_nom[4 * j] = 9.81; u_nom[4 * j + 1] = 0.1; u_nom[4 * j + 2] = -0.1; u_nom[4 * j + 3] = 0.05;
    }
    for (int j = 0; j <= NMAX; ++j) {
        const Real row[13] = {0.1 * j, 0.0, 2.0, 1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        memcpy(x_ref + 13 * j, row, sizeof row);
    }
    // obstacles far from the path (the common case: no margin penalty, no collision)
    Real spheres[MMAX * 5] = {0, 40.0, 40.0, 2.0, 0.5, 0, -40.0, 40.0, 2.0, 0.5};
    Real cylinders[MMAX * 5] = {1, 40.0, 40.0, 0.0, 0.5, 1, -40.0, 40.0, 0.0, 0.5};

    printf("{\n");
    for (int type = 0; type < 2; ++type)
        for (int N = 1; N <= 3; ++N)
            for (int M = 0; M <= MMAX; ++M) {
                g_tally = Tally();
                orc_rollout_one(veh, cost, 0, N, Real(0.01), sigma, 5, 0, 0, x_hat, u_nom, x_ref,
                                type ? cylinders : spheres, M, NULL, du);
                char name[64];
                snprintf(name, sizeof name, "rollout_%s_N%d_M%d", type ? "cyl" : "sph", N, M);
                print_tally(name, g_tally);
            }
    Real G[16];
    g_tally = Tally();
    orc_allocation(veh, G);
    print_tally("allocation", g_tally);
    g_tally = Tally();
    orc_allocation_inverse(veh, G);
    print_tally("allocation_inverse", g_tally);
    Real d4[4];
    g_tally = Tally();
    orc_noise_one(3, 2, sigma, 5, 0, 0, d4);
    print_tally("noise", g_tally, true);
    printf("}\n");
    return 0;
}

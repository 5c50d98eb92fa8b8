// bt_model.hpp -- tree constants of one option (Section 4.1), computed the
// same way on the host and on the GPU.
//
// The model fixes u = e^{sigma sqrt(T/N)}, d = 1/u, r = e^{R T/N}; as binary64
// numbers they are taken to be the correctly rounded values of those reals
// (the binary64 number nearest to the real, ties to even), so that the tree
// does not depend on one math library's approximation of exp or sqrt.
// Division is IEEE binary64 division, correctly rounded by definition.
//
// exp is evaluated in double-double arithmetic (about 104 bits): the
// argument is halved s times until |t| <= 2^-4, e^t comes from its Taylor
// series in Horner form, and is squared s times.  The double-double result is
// within about 2^-90 (relative) of e^x for |x| <= 700, so rounding it to
// binary64 gives the correctly rounded e^x unless e^x lies closer than that
// to a rounding boundary.  Error-free transformations use plain binary64
// additions and products only (Knuth's two-sum, Dekker's product with
// Veltkamp's split), built with contraction off, so the host and the device
// compute the same bits.
#pragma once

#include <math.h>
#include <stdint.h>

#include "../../include/bt.h"

#ifndef BTHD
#define BTHD __host__ __device__ inline
#endif

namespace bt {

// Tree constants of one option (Section 4.1): u, d = 1/u, r, rho = 1/r,
// p = (r - d)/(u - d); sq = sqrt(T/N) and dt = T/N seed the Greeks.
struct Model {
    double S0, u, d, r, rho, p, K, K2, k, sq, dt;
    int32_t N, payoff;
    uint32_t flags;
    int32_t valid;
};

struct DD {
    double hi, lo;
};

// a + b = s + e exactly (Knuth).
BTHD DD two_sum(double a, double b)
{
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return DD{s, e};
}

// a + b = s + e exactly, for |a| >= |b| (or a == 0).
BTHD DD fast_two_sum(double a, double b)
{
    const double s = a + b;
    return DD{s, b - (s - a)};
}

// a = hi + lo with 26-bit halves (Veltkamp); |a| < 2^995.
BTHD DD split(double a)
{
    const double c = 134217729.0 * a;   // 2^27 + 1
    const double hi = c - (c - a);
    return DD{hi, a - hi};
}

// a * b = p + e exactly (Dekker).
BTHD DD two_prod(double a, double b)
{
    const double p = a * b;
    const DD as = split(a), bs = split(b);
    const double e = ((as.hi * bs.hi - p) + as.hi * bs.lo + as.lo * bs.hi) + as.lo * bs.lo;
    return DD{p, e};
}

BTHD DD dd_add(DD a, DD b)
{
    DD s = two_sum(a.hi, b.hi);
    const DD t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}

BTHD DD dd_mul(DD a, DD b)
{
    DD p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return fast_two_sum(p.hi, p.lo);
}

BTHD DD dd_mul_d(DD a, double b)
{
    DD p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return fast_two_sum(p.hi, p.lo);
}

// a / n for a small positive integer n (exact in binary64).
BTHD DD dd_div_n(DD a, double n)
{
    const double q1 = a.hi / n;
    const DD p = two_prod(q1, n);
    const double r = ((a.hi - p.hi) - p.lo) + a.lo;
    const double q2 = r / n;
    return fast_two_sum(q1, q2);
}

// e^x correctly rounded to binary64 for |x| <= 700 (see the file header).
BTHD double cr_exp(double x)
{
    int s = 0;
    double t = x;
    while (t > 0.0625 || t < -0.0625) {
        t *= 0.5;   // exact
        s++;
    }
    // e^t = 1 + t (1 + t/2 (1 + t/3 (...))), 20 terms: t^21/21! < 2^-150
    DD q{1.0, 0.0};
    for (int n = 20; n >= 1; n--) q = dd_add(DD{1.0, 0.0}, dd_div_n(dd_mul_d(q, t), (double)n));
    for (int i = 0; i < s; i++) q = dd_mul(q, q);
    return q.hi + q.lo;
}

// The binary64 neighbours of a positive normal y, by bit pattern.
BTHD double next_up(double y)
{
    union { double d; uint64_t u; } c;
    c.d = y;
    c.u += 1;
    return c.d;
}
BTHD double next_down(double y)
{
    union { double d; uint64_t u; } c;
    c.d = y;
    c.u -= 1;
    return c.d;
}

// sqrt(x) correctly rounded for positive normal x whose square root is
// normal: the hardware square root, then the neighbour whose square is
// nearest to x (x - c^2 evaluated exactly in double-double) is kept.
BTHD double cr_sqrt(double x)
{
    const double y0 = sqrt(x);
    double best = y0, err = -1.0;
    const double cand[3] = {next_down(y0), y0, next_up(y0)};
    for (int i = 0; i < 3; i++) {
        const DD p = two_prod(cand[i], cand[i]);
        const DD r = dd_add(DD{x, 0.0}, DD{-p.hi, -p.lo});
        const double e = r.hi < 0.0 ? -r.hi : r.hi;
        if (err < 0.0 || e < err) { err = e; best = cand[i]; }
    }
    return best;
}

// Derives the tree constants of one option; false (m.valid = 0) if the
// option is invalid: N outside 1..max_N, a non-finite input, S0, K, sigma or
// T not positive, k outside [0, 1), an unknown payoff or flag, K2 <= K for a
// bull or bear spread, |sigma sqrt(T/N)| or |R T/N| above 700 (the tree's prices
// would overflow), or a tree that is not free of arbitrage (d < r < u fails).
BTHD bool derive_model(const bt_params &p, int max_N, Model &m)
{
    m.S0 = m.u = m.d = m.r = m.rho = m.p = m.K = m.K2 = m.k = m.sq = m.dt = 0.0;
    m.N = 0; m.payoff = 0; m.flags = 0; m.valid = 0;
    if (!(p.N >= 1 && p.N <= max_N)) return false;
    const bool finite = p.S0 - p.S0 == 0.0 && p.K - p.K == 0.0 && p.R - p.R == 0.0 && p.sigma - p.sigma == 0.0 &&
                        p.T - p.T == 0.0 && p.k - p.k == 0.0;
    if (!finite) return false;
    if (!(p.S0 > 0.0 && p.K > 0.0 && p.sigma > 0.0 && p.T > 0.0 && p.k >= 0.0 && p.k < 1.0)) return false;
    if (p.payoff < 0 || p.payoff > BT_STRADDLE) return false;
    if ((p.payoff == BT_BULL || p.payoff == BT_BEAR) && !(p.K2 - p.K2 == 0.0 && p.K2 > p.K)) return false;
    if (p.flags & ~(uint32_t)(BT_F_EUROPEAN | BT_F_COST_AT_T0)) return false;
    const double dt = p.T / (double)p.N;
    if (!(dt >= 2.2250738585072014e-308)) return false;   // sqrt below needs a normal argument
    const double sq = cr_sqrt(dt);
    const double lam = p.sigma * sq, rt = p.R * dt;
    if (!(lam <= 700.0) || !(rt <= 700.0 && rt >= -700.0)) return false;
    const double u = cr_exp(lam);
    const double r = cr_exp(rt);
    const double d = 1.0 / u;
    const double rho = 1.0 / r;
    if (!(d < r && r < u)) return false;
    m.S0 = p.S0; m.u = u; m.d = d; m.r = r; m.rho = rho;
    m.p = (r - d) / (u - d);
    m.K = p.K; m.K2 = p.K2; m.k = p.k; m.sq = sq; m.dt = dt;
    m.N = p.N; m.payoff = p.payoff; m.flags = p.flags;
    m.valid = 1;
    return true;
}

}  // namespace bt

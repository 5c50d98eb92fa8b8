// The fused passes of the per-lane node update against the separate passes
// they replace, on seeded random functions: MERGE then SCALE and CANON
// (merge_scale), the clamp then CANON (clip), and the envelope's sweeps
// with reversal, slope shift, CANON and mirror image (sweep_a,
// mirror_canon_raw).  The separate passes are written out here from their
// definitions.  Slopes are drawn from a few values, one ulp apart, with
// collinear runs and lines, so that CANON drops points before and after the
// scaling.  Every count and every stored number must agree bit for bit.
//
// argv[1]: number of cases (default 20000).  Prints "ok <cases>" or the
// first mismatch; exit status 1 on a mismatch.
#define BT_HOST_DEBUG 1
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>
#include "bt_pwl.hpp"
using namespace bt;

struct Buf {
    std::vector<double> d;
    int cap;
    explicit Buf(int c) : d(3 * c + 1, std::nan("")), cap(c) {}
    Arr<double> arr() { return Arr<double>{d.data(), d.data() + cap, d.data() + 2 * cap, 1, cap}; }
};

static bool same(double a, double b) { return std::memcmp(&a, &b, sizeof a) == 0; }

static bool equal_fn(const Arr<double> &a, int ma, const Arr<double> &b, int mb)
{
    if (ma != mb) return false;
    if (ma < 0) return true;
    for (int j = 0; j < ma; j++)
        if (!same(a.X(j), b.X(j)) || !same(a.V(j), b.V(j))) return false;
    for (int j = 0; j <= ma; j++)
        if (!same(a.S(j), b.S(j))) return false;
    return true;
}

// A function of m points: increasing x; slopes from a small pool (ties and
// one-ulp neighbours); convex when asked (slopes nondecreasing).
static int random_fn(std::mt19937_64 &g, Buf &b, int m, bool convex, double lo, double hi)
{
    std::uniform_real_distribution<double> U(0.0, 1.0);
    const double base[4] = {lo, 0.5 * (lo + hi), hi, 0.25 * lo + 0.75 * hi};
    std::vector<double> s(m + 1);
    for (int j = 0; j <= m; j++) {
        double v = base[g() % 4];
        const int t = (int)(g() % 4);
        if (t == 1) v = std::nextafter(v, 1e300);
        if (t == 2) v = std::nextafter(v, -1e300);
        s[j] = v;
    }
    if (g() % 5 == 0) for (int j = 1; j <= m; j++) s[j] = s[0];   // a line
    if (convex) std::sort(s.begin(), s.end());
    Arr<double> a = b.arr();
    double x = -2.0 + U(g), v = 10.0 * U(g);
    for (int j = 0; j < m; j++) {
        a.X(j) = x;
        a.V(j) = v;
        const double dx = (g() % 7 == 0) ? 1e-9 : 0.05 + U(g);
        v = v + s[j + 1] * dx;
        x = x + dx;
    }
    for (int j = 0; j <= m; j++) a.S(j) = s[j];
    return m;
}

// SCALE then CANON as separate passes.
static int ref_scale(const Arr<double> &f, int m, double rho)
{
    for (int j = 0; j < m; j++) f.V(j) = f.V(j) * rho;
    for (int j = 0; j <= m; j++) f.S(j) = f.S(j) * rho;
    return canon(f, m);
}

// CLIP (a < b) as the clamp, then CANON.
static int ref_clip(const Arr<double> &f, int m, double a, double b)
{
    for (int j = 0; j <= m; j++) {
        if (f.S(j) < a) f.S(j) = a;
        else if (f.S(j) > b) f.S(j) = b;
    }
    return canon(f, m);
}

// The raw sweep's points in place: reverse them, shift every slope up one
// slot, left tail a, then CANON.
static int ref_finish_sweep(const Arr<double> &o, int n, double a)
{
    for (int i = 0, j = n - 1; i < j; i++, j--) {
        std::swap(o.X(i), o.X(j));
        std::swap(o.V(i), o.V(j));
        std::swap(o.S(i), o.S(j));
    }
    for (int i = n - 1; i >= 0; i--) o.S(i + 1) = o.S(i);
    o.S(0) = a;
    return canon(o, n);
}

// Mirror image in place: x_j <- -x_{n-1-j}, v_j <- v_{n-1-j}, s_j <- -s_{n-j}.
static void ref_mirror(const Arr<double> &o, int n)
{
    for (int i = 0, j = n - 1; i < j; i++, j--) {
        std::swap(o.X(i), o.X(j));
        std::swap(o.V(i), o.V(j));
    }
    for (int i = 0; i < n; i++) o.X(i) = -o.X(i);
    for (int i = 0, j = n; i < j; i++, j--) std::swap(o.S(i), o.S(j));
    for (int i = 0; i <= n; i++) o.S(i) = -o.S(i);
}

static int fail(const char *what, int c)
{
    std::printf("mismatch in %s at case %d\n", what, c);
    return 1;
}

int main(int argc, char **argv)
{
    const int cases = argc > 1 ? std::atoi(argv[1]) : 20000;
    std::mt19937_64 g(20261203);
    const double rhos[4] = {0.9990009995001666, 0.95122942450071402, 1.0, 0.99999999999999989};
    int merged = 0, clipped = 0, swept = 0;
    int collide = 0, lines = 0, dropped = 0;   // cases that reach the fused passes' special branches
    for (int c = 0; c < cases; c++) {
        const int cap = 40;
        const double rho = rhos[g() % 4];
        // MERGE with SCALE against MERGE, SCALE, CANON
        {
            Buf F(cap), G(cap), o1(2 * cap + 4), o2(2 * cap + 4);
            const int mf = random_fn(g, F, 1 + (int)(g() % 6), g() % 2 == 0, -3.0, -1.0);
            const int mg = random_fn(g, G, 1 + (int)(g() % 6), g() % 2 == 0, -3.0, -1.0);
            const View<double> Fv = F.arr().view(mf), Gv = G.arr().view(mg);
            for (int op = 0; op < 2; op++) {
                int m1 = op == 0 ? merge<OPMAX, double>(Fv, Gv, o1.arr()) : merge<OPMIN, double>(Fv, Gv, o1.arr());
                const int m0 = m1;
                if (m1 >= 0) m1 = ref_scale(o1.arr(), m1, rho);
                if (m1 >= 0 && m1 < m0) collide++;
                if (m1 == 1 && same(o1.arr().S(0), o1.arr().S(1))) lines++;
                const int m2 = op == 0 ? merge_scale<OPMAX, double>(Fv, Gv, o2.arr(), rho)
                                       : merge_scale<OPMIN, double>(Fv, Gv, o2.arr(), rho);
                if (!equal_fn(o1.arr(), m1, o2.arr(), m2)) return fail("merge_scale", c);
                merged++;
            }
            // a capacity that the merge overflows must overflow both ways
            Buf t1(2), t2(2);
            int m1 = merge<OPMAX, double>(Fv, Gv, t1.arr());
            if (m1 >= 0) m1 = ref_scale(t1.arr(), m1, rho);
            const int m2 = merge_scale<OPMAX, double>(Fv, Gv, t2.arr(), rho);
            if ((m1 < 0) != (m2 < 0) || (m1 >= 0 && !equal_fn(t1.arr(), m1, t2.arr(), m2)))
                return fail("merge_scale capacity", c);
        }
        // CLIP against the clamp, then CANON
        {
            Buf F1(cap), F2(cap);
            const int m = 1 + (int)(g() % 8);
            std::mt19937_64 g2 = g;
            random_fn(g, F1, m, true, -3.0, -1.0);
            random_fn(g2, F2, m, true, -3.0, -1.0);
            const double a = -2.5 + 0.25 * (double)(g() % 4), b = a + 0.5 * (double)(1 + g() % 3);
            const int m1 = ref_clip(F1.arr(), m, a, b);
            const int m2 = clip(F2.arr(), m, a, b);
            if (!equal_fn(F1.arr(), m1, F2.arr(), m2)) return fail("clip", c);
            clipped++;
        }
        // the envelope's two sweeps: A and B = mirror(RB)
        {
            Buf F(cap);
            const double a = -2.0, b = -1.5;
            const int m = random_fn(g, F, 2 + (int)(g() % 7), true, -3.0, -1.0);
            Arr<double> Fa = F.arr();
            Fa.S(0) = -3.0 - 0.5 * (double)(g() % 2);   // s_0 < a and -s_m < -b (tails past both bounds)
            Fa.S(m) = -1.0 + 0.25 * (double)(g() % 2);
            const View<double> Fv = Fa.view(m);
            Buf r1(cap), r2(cap), o2(cap), w(cap);
            // A
            int n1 = sweep_raw<false, double>(Fv, a, r1.arr());
            const int n0 = n1;
            if (n1 >= 0) n1 = ref_finish_sweep(r1.arr(), n1, a);
            if (n1 >= 0 && n1 < n0) dropped++;
            const int n2 = sweep_a<false, double>(Fv, a, r2.arr(), o2.arr());
            if (!equal_fn(r1.arr(), n1, o2.arr(), n2)) return fail("sweep_a", c);
            // B
            Buf q1(cap), q2(cap);
            int k1 = sweep_raw<true, double>(Fv, -b, q1.arr());
            if (k1 >= 0) {
                k1 = ref_finish_sweep(q1.arr(), k1, -b);
                ref_mirror(q1.arr(), k1);
                k1 = canon(q1.arr(), k1);
            }
            const int kr = sweep_raw<true, double>(Fv, -b, q2.arr());
            const int k2 = kr < 0 ? -1 : mirror_canon_raw(q2.arr(), kr, -b, w.arr());
            if (!equal_fn(q1.arr(), k1, w.arr(), k2)) return fail("mirror_canon_raw", c);
            swept++;
        }
    }
    std::printf("ok %d merges %d clips %d sweeps %d scaled-canon-drops %d lines %d sweep-canon-drops %d\n", cases,
                merged, clipped, swept, collide, lines, dropped);
    return 0;
}

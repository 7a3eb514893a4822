// oecdg_tables.h -- compile-time tables of the Legendre modal basis.
//
// Every kernel indexes these with compile-time indices (fully unrolled loops),
// so the values become instruction constants that the compiler can
// rematerialise instead of holding hundreds of table entries in registers.
//
// Basis: unnormalised Legendre polynomials P_n(xi) on the reference cell
// [-1, 1].  Quadrature: Gauss-Legendre with Q = k+1 nodes on each half cell
// [-1, 0] and [0, 1] (the halves on which the overlapping solution of the other
// mesh is one polynomial), nodes from their closed forms polished by Newton's
// iteration on P_Q.
#pragma once

namespace oecdg {
namespace ct {

constexpr double cabs(double x) { return x < 0 ? -x : x; }

constexpr double csqrt(double a) {
    if (a <= 0.0) return 0.0;
    double x = a > 1.0 ? a : 1.0;
    for (int i = 0; i < 200; ++i) {
        const double nx = 0.5 * (x + a / x);
        if (nx == x) break;
        x = nx;
    }
    return x;
}

// P_n(x) by Bonnet's recurrence.
constexpr double leg(int n, double x) {
    if (n == 0) return 1.0;
    double p0 = 1.0, p1 = x;
    for (int j = 1; j < n; ++j) {
        const double p2 = ((2.0 * j + 1.0) * x * p1 - j * p0) / (j + 1.0);
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

// d-th derivative of P_n at x via P_n' = sum_{j = n-1, n-3, ...} (2j+1) P_j.
constexpr double legd(int n, int d, double x) {
    if (d == 0) return leg(n, x);
    double s = 0.0;
    for (int j = n - 1; j >= 0; j -= 2) s += (2.0 * j + 1.0) * legd(j, d - 1, x);
    return s;
}

// Gauss-Legendre rule with Q <= 4 nodes (ascending), closed forms then Newton.
template <int Q>
struct Gauss {
    double s[Q], w[Q];
};

template <int Q>
constexpr Gauss<Q> gauss() {
    Gauss<Q> g{};
    static_assert(Q >= 1 && Q <= 4, "Q in 1..4");
    if constexpr (Q == 1) {
        g.s[0] = 0.0;
    } else if constexpr (Q == 2) {
        g.s[0] = -1.0 / csqrt(3.0);
        g.s[1] = -g.s[0];
    } else if constexpr (Q == 3) {
        g.s[0] = -csqrt(0.6);
        g.s[1] = 0.0;
        g.s[2] = -g.s[0];
    } else {
        const double r = 2.0 / 7.0 * csqrt(1.2);
        g.s[0] = -csqrt(3.0 / 7.0 + r);
        g.s[1] = -csqrt(3.0 / 7.0 - r);
        g.s[2] = -g.s[1];
        g.s[3] = -g.s[0];
    }
    for (int i = 0; i < Q; ++i) {
        double x = g.s[i];
        for (int it = 0; it < 8; ++it) {
            const double dp = legd(Q, 1, x);
            if (dp == 0.0) break;
            const double dx = leg(Q, x) / dp;
            x -= dx;
            if (cabs(dx) < 1e-18) break;
        }
        g.s[i] = x;
        const double dp = legd(Q, 1, x);
        g.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return g;
}

// Exact rational arithmetic for the overlap integrals (small integers only).
struct Rat {
    long long p, q;      // p / q, q > 0, reduced
};

constexpr long long cgcd(long long a, long long b) {
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
        const long long t = a % b;
        a = b;
        b = t;
    }
    return a ? a : 1;
}
constexpr Rat rat(long long p, long long q) {
    if (q < 0) p = -p, q = -q;
    const long long g = cgcd(p, q);
    return Rat{p / g, q / g};
}
constexpr Rat radd(Rat a, Rat b) { return rat(a.p * b.q + b.p * a.q, a.q * b.q); }
constexpr Rat rmul(Rat a, Rat b) { return rat(a.p * b.p, a.q * b.q); }

// Monomial coefficients of P_n (n <= 3), P_n(x) = sum_j c[j] x^j, from
// (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}.
struct Poly {
    Rat c[8];
};
constexpr Poly legpoly(int n) {
    Poly a{}, b{};
    for (int j = 0; j < 8; ++j) a.c[j] = b.c[j] = Rat{0, 1};
    a.c[0] = Rat{1, 1};                  // P_0
    if (n == 0) return a;
    b.c[1] = Rat{1, 1};                  // P_1
    for (int m = 1; m < n; ++m) {
        Poly nx{};
        for (int j = 0; j < 8; ++j) nx.c[j] = Rat{0, 1};
        for (int j = 0; j < 7; ++j) nx.c[j + 1] = rmul(b.c[j], rat(2 * m + 1, m + 1));
        for (int j = 0; j < 8; ++j) nx.c[j] = radd(nx.c[j], rmul(a.c[j], rat(-m, m + 1)));
        a = b;
        b = nx;
    }
    return b;
}
// P_n(x - 1) in monomials of x.
constexpr Poly shifted(const Poly &p) {
    Poly r{};
    for (int j = 0; j < 8; ++j) r.c[j] = Rat{0, 1};
    for (int j = 0; j < 8; ++j) {
        long long binom = 1;             // C(j, i) (-1)^(j-i) x^i
        for (int i = j; i >= 0; --i) {
            const long long sg = ((j - i) & 1) ? -1 : 1;
            r.c[i] = radd(r.c[i], rmul(p.c[j], Rat{sg * binom, 1}));
            binom = binom * i / (j - i + 1);
        }
    }
    return r;
}
// int_0^1 P_n(x - 1) P_m(x) dx, exactly.
constexpr Rat overlap(int m, int n) {
    const Poly a = legpoly(m), b = shifted(legpoly(n));
    Rat s{0, 1};
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j + i < 8; ++j)
            if (a.c[i].p != 0 && b.c[j].p != 0) s = radd(s, rmul(rmul(a.c[i], b.c[j]), rat(1, i + j + 1)));
    return s;
}

}  // namespace ct

// Tables of degree K.
template <int K>
struct Tab {
    static constexpr int K1 = K + 1, Q = K + 1, NSP = 2 * K + 4;
    double E[2][Q][K1];    // P_n at the overlapping cell's coordinate of node g of half h
    double WP[2][Q][K1];   // (w_g / 2) P_m(xi_g) on half h
    double WD[2][Q][K1];   // (w_g / 2) P_m'(xi_g) on half h
    double D0[K1][K1];     // d-th derivative of P_n at xi = 0: [d][n]
    double D1[K1][K1];     // d-th derivative of P_n at xi = 1: [d][n]
    double SP[NSP][K1];    // P_n at the sigma sample points (edges and both halves' nodes)
    double C[K1];          // (2m+1) 2^m / ((2K-1) m!)
    double OV[K1][K1];     // int_0^1 P_n(xi - 1) P_m(xi) dxi, [m][n]: the right neighbour's mode n
                           // projected on the test function P_m over the right half (exact rationals)
};

template <int K>
constexpr Tab<K> make_tab() {
    Tab<K> t{};
    constexpr int Q = K + 1;
    const ct::Gauss<Q> g = ct::gauss<Q>();
    for (int hf = 0; hf < 2; ++hf)
        for (int q = 0; q < Q; ++q) {
            const double xi = hf == 0 ? 0.5 * (g.s[q] - 1.0) : 0.5 * (g.s[q] + 1.0);
            const double xn = hf == 0 ? xi + 1.0 : xi - 1.0;
            for (int n = 0; n <= K; ++n) {
                t.E[hf][q][n] = ct::leg(n, xn);
                t.WP[hf][q][n] = 0.5 * g.w[q] * ct::leg(n, xi);
                t.WD[hf][q][n] = 0.5 * g.w[q] * ct::legd(n, 1, xi);
            }
        }
    for (int d = 0; d <= K; ++d)
        for (int n = 0; n <= K; ++n) {
            t.D0[d][n] = ct::legd(n, d, 0.0);
            t.D1[d][n] = ct::legd(n, d, 1.0);
        }
    double pts[2 * K + 4] = {};
    int c = 0;
    pts[c++] = -1.0;
    for (int q = 0; q < Q; ++q) pts[c++] = 0.5 * (g.s[q] - 1.0);
    for (int q = 0; q < Q; ++q) pts[c++] = 0.5 * (g.s[q] + 1.0);
    pts[c++] = 1.0;
    for (int j = 0; j < c; ++j)
        for (int n = 0; n <= K; ++n) t.SP[j][n] = ct::leg(n, pts[j]);
    double fact = 1.0, pow2 = 1.0;
    for (int m = 0; m <= K; ++m) {
        if (m > 0) {
            fact *= m;
            pow2 *= 2.0;
        }
        t.C[m] = K > 0 ? (2.0 * m + 1.0) * pow2 / ((2.0 * K - 1.0) * fact) : 0.0;
    }
    for (int m = 0; m <= K; ++m)
        for (int n = 0; n <= K; ++n) {
            const ct::Rat r = ct::overlap(m, n);
            t.OV[m][n] = (double)r.p / (double)r.q;
        }
    return t;
}

}  // namespace oecdg

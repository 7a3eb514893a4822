// ora_real.hpp -- floating-point operation counter for the oracle (test
// infrastructure; the product never builds or loads this).
//
// The oracle's C sources are compiled as C++ with `double` defined as ora_real,
// a wrapper that performs every operation in double exactly as written and
// counts it: + - * / one flop each, and square roots, exponentials, powers and
// the other library calls apart.  The counts are therefore the operations of
// the oracle's plain evaluation of the method, the algorithm's own flop count
// (no fusion, no sum factorisation beyond what the oracle writes).
#pragma once
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace ora_count {
struct Counts {
    unsigned long long add = 0, mul = 0, div = 0, sqrt = 0, exp = 0, pow = 0, other = 0, cmp = 0;
};
inline Counts &counts() {
    static Counts c;
    return c;
}
}  // namespace ora_count

struct ora_real {
    double v;
    ora_real() = default;
    constexpr ora_real(double x) : v(x) {}
    explicit operator double() const { return v; }
    explicit operator int() const { return (int)v; }
    explicit operator long() const { return (long)v; }
    ora_real &operator+=(ora_real o) { ++ora_count::counts().add; v += o.v; return *this; }
    ora_real &operator-=(ora_real o) { ++ora_count::counts().add; v -= o.v; return *this; }
    ora_real &operator*=(ora_real o) { ++ora_count::counts().mul; v *= o.v; return *this; }
    ora_real &operator/=(ora_real o) { ++ora_count::counts().div; v /= o.v; return *this; }
};
inline ora_real operator+(ora_real a, ora_real b) { ++ora_count::counts().add; return ora_real(a.v + b.v); }
inline ora_real operator-(ora_real a, ora_real b) { ++ora_count::counts().add; return ora_real(a.v - b.v); }
inline ora_real operator*(ora_real a, ora_real b) { ++ora_count::counts().mul; return ora_real(a.v * b.v); }
inline ora_real operator/(ora_real a, ora_real b) { ++ora_count::counts().div; return ora_real(a.v / b.v); }
inline ora_real operator-(ora_real a) { return ora_real(-a.v); }
inline ora_real operator+(ora_real a) { return a; }
#define ORA_CMP(op)                                                                   \
    inline bool operator op(ora_real a, ora_real b) { ++ora_count::counts().cmp; return a.v op b.v; }
ORA_CMP(<) ORA_CMP(>) ORA_CMP(<=) ORA_CMP(>=) ORA_CMP(==) ORA_CMP(!=)
#undef ORA_CMP
inline ora_real sqrt(ora_real a) { ++ora_count::counts().sqrt; return ora_real(std::sqrt(a.v)); }
inline ora_real exp(ora_real a) { ++ora_count::counts().exp; return ora_real(std::exp(a.v)); }
inline ora_real pow(ora_real a, ora_real b) { ++ora_count::counts().pow; return ora_real(std::pow(a.v, b.v)); }
inline ora_real fabs(ora_real a) { ++ora_count::counts().other; return ora_real(std::fabs(a.v)); }
inline ora_real fmax(ora_real a, ora_real b) { ++ora_count::counts().other; return ora_real(std::fmax(a.v, b.v)); }
inline ora_real fmin(ora_real a, ora_real b) { ++ora_count::counts().other; return ora_real(std::fmin(a.v, b.v)); }
inline bool isfinite(ora_real a) { return std::isfinite(a.v); }
inline bool isnan(ora_real a) { return std::isnan(a.v); }
inline ora_real cos(ora_real a) { ++ora_count::counts().other; return ora_real(std::cos(a.v)); }
inline ora_real sin(ora_real a) { ++ora_count::counts().other; return ora_real(std::sin(a.v)); }

#define double ora_real

// Central-difference weights of arbitrary even order from their closed form.
//
// For a central first derivative of order p = 2r,
//     a_m = (-1)^(m+1) (r!)^2 / (m (r-m)! (r+m)!),          m = 1..r,
// and for the matching second derivative
//     c_m = 2 a_m / m,   c_0 = -2 sum_m c_m.
// (Paper Sec. "Discretisation schemes": central first- and second-derivative
// stencils of arbitrary order, with the rational weights evaluated once rather
// than divided at run time.)  Evaluated exactly in 64-bit rationals, then
// rounded once to double.
#pragma once

#include <cstdint>
#include <numeric>

namespace sbli {

struct Rational {
    int64_t num, den;
    Rational(int64_t n = 0, int64_t d = 1) : num(n), den(d) { norm(); }
    void norm() {
        if (den < 0) { num = -num; den = -den; }
        int64_t g = std::gcd(num < 0 ? -num : num, den);
        if (g > 1) { num /= g; den /= g; }
    }
    Rational operator+(const Rational& o) const { return Rational(num * o.den + o.num * den, den * o.den); }
    Rational operator*(const Rational& o) const { return Rational(num * o.num, den * o.den); }
    double value() const { return (double)num / (double)den; }
};

inline int64_t factorial(int n) {
    int64_t f = 1;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

// Fills a[0..r-1] = a_1..a_r, c[0..r-1] = c_1..c_r and *c0, for 1 <= r <= 6.
inline void central_weights(int r, double* a, double* c0, double* c) {
    Rational csum(0);
    const int64_t rf = factorial(r);
    for (int m = 1; m <= r; ++m) {
        Rational am((m % 2 ? 1 : -1) * rf * rf, (int64_t)m * factorial(r - m) * factorial(r + m));
        Rational cm = am * Rational(2, m);
        a[m - 1] = am.value();
        c[m - 1] = cm.value();
        csum = csum + cm;
    }
    *c0 = (csum * Rational(-2)).value();
}

}  // namespace sbli

// Host-side Kerr geometry for the coefficient tables of Eq. (1)
// (arXiv:1010.3816, Sec. 3): tortoise coordinate, its inversion, and the
// 1-D radial / angular factors from which the kernels rebuild every
// coefficient of the first-order system.  Values carry d/da as dual numbers
// (first-order forward-mode differentiation), needed for the spin gradient.
#pragma once

#include <cmath>

#include "internal.hpp"

namespace teuk {

struct Dual {
    double v = 0.0, d = 0.0;
    Dual() = default;
    Dual(double value) : v(value), d(0.0) {}  // NOLINT: constants promote
    Dual(double value, double deriv) : v(value), d(deriv) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual sqrt(Dual a) {
    const double s = std::sqrt(a.v);
    return {s, a.d / (2.0 * s)};
}
inline Dual log(Dual a) { return {std::log(a.v), a.d / a.v}; }
inline double val(Dual a) { return a.v; }
inline double val(double a) { return a; }

// Tortoise coordinate with q = sqrt(1 - a^2), r_pm = 1 pm q, as a function of
// x = r - r_+ (> 0):  r* = r + ((1+q)/q) ln(x/2) - ((1-q)/q) ln(x/2 + q),
// which satisfies d(r*)/dr = (r^2 + a^2)/Delta, Delta = x (x + 2q).
template <class T>
T tortoise(T a, T x) {
    using std::log;
    using std::sqrt;
    const T q = sqrt(T(1.0) - a * a);
    return T(1.0) + q + x + ((T(1.0) + q) / q) * log(T(0.5) * x) - ((T(1.0) - q) / q) * log(T(0.5) * x + q);
}

// Inverse tortoise map for real spin: x with tortoise(a, x) = rstar.
// Newton in u = ln x with backtracking (the map is increasing in u), from
// the far-field or near-horizon asymptote, then two Newton corrections in x.
inline bool tortoise_inverse(double a, double rstar, double* x_out) {
    const double q = std::sqrt(1.0 - a * a);
    auto g = [&](double u) { return tortoise(a, std::exp(u)) - rstar; };
    auto dg = [&](double u) {  // d r*/d ln x = (r^2 + a^2)/(x + 2q)
        const double x = std::exp(u), r = 1.0 + q + x;
        return (r * r + a * a) / (x + 2.0 * q);
    };
    double u;
    if (rstar > 4.0)
        u = std::log(rstar);
    else
        u = std::log(2.0) + (rstar - 1.0 - q) * q / (1.0 + q);
    u = std::fmin(std::fmax(u, -1500.0), 60.0);
    double gu = g(u);
    for (int it = 0; it < 200 && std::isfinite(gu); ++it) {
        double step = -gu / dg(u);
        double un = u + step, gn = g(un);
        int bt = 0;
        while (!(std::fabs(gn) < std::fabs(gu)) && bt < 60) {
            step *= 0.5;
            un = u + step;
            gn = g(un);
            ++bt;
        }
        if (bt == 60) break;  // no further decrease possible: converged
        u = un;
        gu = gn;
        if (std::fabs(step) <= 1e-16 * std::fmax(1.0, std::fabs(u))) break;
    }
    double x = std::exp(u);
    double fx = std::fabs(tortoise(a, x) - rstar);
    for (int it = 0; it < 3; ++it) {
        const double r = 1.0 + q + x, delta = x * (x + 2.0 * q);
        const double xn = x - (tortoise(a, x) - rstar) * delta / (r * r + a * a);
        const double fn = (xn > 0.0) ? std::fabs(tortoise(a, xn) - rstar) : INFINITY;
        if (!(fn < fx)) break;
        x = xn;
        fx = fn;
    }
    *x_out = x;
    return std::isfinite(x) && x > 0.0 && fx < 1e-9 * std::fmax(1.0, std::fabs(rstar));
}

// x(r*; a) with its spin derivative at fixed r*, from the solved x:
// dx/da = -(dr*/da)|_x / (dr*/dx)|_a.
inline Dual tortoise_x_dual(double a, double x) {
    const double q = std::sqrt(1.0 - a * a), r = 1.0 + q + x;
    const double dr_da = tortoise(Dual(a, 1.0), Dual(x, 0.0)).d;
    const double dr_dx = (r * r + a * a) / (x * (x + 2.0 * q));
    return Dual(x, -dr_da / dr_dx);
}

// The radial factors of RadField at one position.
template <class T>
void radial_fields(T a, int s, int m, T x, double dth, T out[kNumRad]) {
    using std::sqrt;
    const T q = sqrt(T(1.0) - a * a);
    const T r = T(1.0) + q + x;
    const T delta = x * (x + T(2.0) * q);
    const T rho = r * r + a * a;
    const T rm1 = r - T(1.0);
    out[R_RHO] = rho;
    out[R_RHO2] = rho * rho;
    out[R_A2D] = a * a * delta;
    out[R_RB1] = T(2.0) * r * delta / rho;
    out[R_RB2] = T(2.0) * r * rho * delta;
    out[R_RB3] = a * a * rm1 * delta;
    out[R_CTR] = T(2.0 * s) * (r * delta - (r * r - a * a));
    out[R_CTI0] = T(4.0 * m) * a * r;
    out[R_CTI1] = T(2.0 * s) * a * delta;
    out[R_B1N] = rho * (T(6.0) * delta / r + T(2.0 * s) * rm1) + T(2.0) * r * delta;
    out[R_DL2] = delta / T(dth * dth);
    out[R_V0R] = -T(double(m) * m) * a * a -
                 T(6.0) * delta * (T(s + 2.0) * r * r - T(s + 3.0) * r + a * a) / (r * r);
    out[R_V0I] = -T(2.0 * s * m) * a * rm1;
}

// The angular factors of AngField at row j (theta_j = (j + 1/2) dth).
inline void angular_fields(int s, int m, int j, double dth, double out[kNumAng]) {
    const double th = (j + 0.5) * dth;
    const double sn = std::sin(th), cs = std::cos(th);
    const double mc = m + s * cs;
    out[A_SN2] = sn * sn;
    out[A_CS] = cs;
    out[A_COTP] = (cs / sn) * (0.5 * dth);
    out[A_PD] = (mc * mc / (sn * sn) - s) * (dth * dth);
}

}  // namespace teuk

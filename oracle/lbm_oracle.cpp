// CPU oracle for the D2Q9 pseudopotential multiphase lattice Boltzmann step with
// high-order-difference (HDM) interaction forces — Qin, Zhao, Chen, Zhang, Wen,
// "A pseudopotential multiphase lattice Boltzmann model based on high-order
// difference" (arXiv:1712.06079).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
// FP64 statement of what the GPU library computes.  It is used by the tests,
// by the package's smoke check and by the CPU-baseline leg of the benchmark.
// The product path never links, loads or calls it, and it shares no code with
// the HIP library: the two are independent implementations of the paper.
//
// Style: separate plain arrays, one pass per equation, the tridiagonal system of
// Sec. 3.2 Eq. 20 solved along every grid line by the chasing (Thomas) method
// with a Sherman-Morrison correction for the periodic corners.  Every arithmetic
// step is written in source order; the build uses -ffp-contract=off and no
// fast-math so the result is ordinary IEEE double arithmetic.
//
// The scalar type is a template parameter only so that the same step can be
// evaluated on forward-mode dual numbers (value + tangent) for the adjoint
// dot-product tests; with S = double it is the plain FP64 step.
//
// Readings of the paper where it is silent or garbled (each also listed in the
// design notes):
//  * D2Q9 weights are not printed: 4/9 (rest), 1/9 (axes), 1/36 (diagonals);
//    c_s^2 = 1/3 (Sec. 2 after Eq. 6); dt = h = 1 (Sec. 2 after Eq. 1).
//  * Eq. 20 carries no boundary closure: every grid line is periodic.  Its 2D
//    use is dimension by dimension: d/dx along each row, d/dy along each column.
//  * Eq. 15 as printed lacks the factor 1/c_s^2 = 3 (its sum is c_s^2 grad u);
//    the factor is applied.
//  * Walls (Sec. 5.5 states no-slip walls in y but neither the scheme nor a
//    closure of Eq. 20): halfway bounce-back puts the wall midway between the
//    last fluid row and the next; the potential is continued past the wall by
//    its mirror image (zero normal derivative: a neutral wall), which gives
//    Eq. 20 two closure rows at each end (below).
//  * Eq. 29 (Carnahan-Starling) prints the denominator as (1 - (b rho/4)^3);
//    the Carnahan-Starling form (1 - b rho/4)^3 is used.
//  * Hu's scaling p_m = k p_EOS (Sec. 5) enters U = g (k p_EOS - rho c_s^2).
//    G cancels between Eqs. 4 and 6; g is an interaction-strength multiplier
//    on U (g = 1 is the paper).  The bulk pressure is p = rho/3 + U.
//  * The sign in Eqs. 21-22 at U = 0 is taken as "+" (the ">= 0" branch).
//  * Zhang-Chen force uses F = -grad U (Eqs. 7-8).
//  * The velocity in f^eq (BGK and EDM) is the bare u = j / rho (Eq. 3);
//    Eq. 11's half-step velocity is an output only.
//  * Step order: moments -> force -> collide -> stream, state stored post-stream.

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

// Plain parameter block shared with the ctypes wrapper (oracle-only layout).
typedef struct {
    int32_t nx, ny;
    int32_t eos;    // 0 VDW (Eq. 24), 1 PR (Eq. 28), 2 CS (Eq. 29), 3 RK (Eq. 27), 4 RKS
    int32_t force;  // 0 Shan-Chen (Eq. 22), 1 Zhang-Chen (Eq. 7), 2 hybrid (Eq. 9)
    int32_t grad;   // 0 high-order difference (Eq. 20), 1 central difference (Eq. 14),
                    // 2 weighted D2Q9 central difference (Eq. 15, with the 1/c_s^2 factor)
    int32_t walls;  // 0 periodic in y; 1 no-slip walls at y = -1/2 and ny - 1/2 (halfway
                    // bounce-back; the potential mirrored at the wall for the gradient)
    double tau;     // relaxation time (Eq. 1)
    double a, b, R, omega;  // EOS constants; omega = acentric factor (PR, RKS)
    double T;       // absolute temperature
    double k;       // Hu's EOS scaling p_m = k p_EOS (Sec. 5)
    double g;       // interaction-strength multiplier on U (g = 1 is the paper)
    double A;       // hybrid weight of Eq. 9
} orc_params;

}  // extern "C"

namespace {

// ---------------------------------------------------------------- D2Q9, Eq. 2
const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const double WQ[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                      1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// ---------------------------------------------------------------- dual numbers
struct Dual {
    double v, d;
    Dual() : v(0), d(0) {}
    Dual(double x) : v(x), d(0) {}
    Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual x, Dual y) { return Dual(x.v + y.v, x.d + y.d); }
inline Dual operator-(Dual x, Dual y) { return Dual(x.v - y.v, x.d - y.d); }
inline Dual operator-(Dual x) { return Dual(-x.v, -x.d); }
inline Dual operator*(Dual x, Dual y) { return Dual(x.v * y.v, x.d * y.v + x.v * y.d); }
inline Dual operator/(Dual x, Dual y) {
    double q = x.v / y.v;
    return Dual(q, (x.d - q * y.d) / y.v);
}
inline Dual sqrt(Dual x) {
    double s = std::sqrt(x.v);
    return Dual(s, x.d / (2.0 * s));
}
inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }
inline double sq(double x) { return x * x; }
inline Dual sq(Dual x) { return x * x; }
using std::sqrt;

// ---------------------------------------------------------------- EOS (Sec. 5)
// Temperature function alpha(T) of the cubic EOS.
//  RK  (Eq. 27): alpha = 1/sqrt(T).
//  RKS (after Eq. 27): alpha = [1 + (0.480 + 1.574 w - 0.176 w^2)(1 - sqrt(T/Tc))]^2.
//  PR  (after Eq. 28): alpha = [1 + (0.37464 + 1.54226 w - 0.26992 w^2)(1 - sqrt(T/Tc))]^2.
template <typename S>
S alpha_of(const orc_params& p, S T, double Tc) {
    if (p.eos == 3) return S(1.0) / sqrt(T);
    if (p.eos == 1 || p.eos == 4) {
        double w = p.omega;
        double m = (p.eos == 1) ? (0.37464 + 1.54226 * w - 0.26992 * w * w)
                                : (0.480 + 1.574 * w - 0.176 * w * w);
        S t = S(1.0) + m * (S(1.0) - sqrt(T / Tc));
        return t * t;
    }
    return S(1.0);
}

// p_EOS(rho, T) with a given alpha (alpha multiplies the attraction term).
template <typename S>
S p_eos_alpha(const orc_params& p, S rho, S T, S alpha) {
    const double a = p.a, b = p.b, R = p.R;
    switch (p.eos) {
        case 0:  // VDW, Eq. 24 (R written out, R = 1 in the paper)
            return rho * R * T / (S(1.0) - b * rho) - a * rho * rho;
        case 3:  // RK, Eq. 27
        case 4:  // RKS: Eq. 27 with the Soave alpha
            return rho * R * T / (S(1.0) - b * rho) - a * alpha * rho * rho / (S(1.0) + b * rho);
        case 1:  // PR, Eq. 28
            return rho * R * T / (S(1.0) - b * rho) -
                   a * alpha * rho * rho / (S(1.0) + 2.0 * b * rho - b * b * rho * rho);
        case 2: {  // CS, Eq. 29 with denominator (1 - b rho / 4)^3
            S eta = b * rho / 4.0;
            S one_m = S(1.0) - eta;
            return rho * R * T * (S(1.0) + eta + eta * eta - eta * eta * eta) / (one_m * one_m * one_m) -
                   a * rho * rho;
        }
    }
    return S(0.0);
}

// d p / d rho and d2 p / d rho2 at fixed T (alpha fixed), written out by hand.
double dp_drho(const orc_params& p, double rho, double T, double alpha) {
    const double a = p.a, b = p.b, R = p.R;
    switch (p.eos) {
        case 0:
            return R * T / sq(1.0 - b * rho) - 2.0 * a * rho;
        case 3:
        case 4:
            // d/drho [rho^2/(1+b rho)] = (2 rho + b rho^2)/(1+b rho)^2
            return R * T / sq(1.0 - b * rho) - a * alpha * (2.0 * rho + b * rho * rho) / sq(1.0 + b * rho);
        case 1: {
            // q = 1 + 2 b rho - b^2 rho^2, q' = 2b - 2 b^2 rho
            // d/drho [rho^2/q] = (2 rho q - rho^2 q') / q^2
            double q = 1.0 + 2.0 * b * rho - b * b * rho * rho;
            double qp = 2.0 * b - 2.0 * b * b * rho;
            return R * T / sq(1.0 - b * rho) - a * alpha * (2.0 * rho * q - rho * rho * qp) / (q * q);
        }
        case 2: {
            // rho Z(eta), Z = (1+eta+eta^2-eta^3)/(1-eta)^3, d eta/d rho = b/4;
            // d/drho[rho Z] = Z + eta Z'(eta),
            // Z'(eta) = [(1+2eta-3eta^2)(1-eta) + 3(1+eta+eta^2-eta^3)]/(1-eta)^4
            double e = b * rho / 4.0;
            double num = 1.0 + e + e * e - e * e * e;
            double den = (1.0 - e) * (1.0 - e) * (1.0 - e);
            double Z = num / den;
            double Zp = ((1.0 + 2.0 * e - 3.0 * e * e) * (1.0 - e) + 3.0 * num) / (den * (1.0 - e));
            return R * T * (Z + e * Zp) - 2.0 * a * rho;
        }
    }
    return 0.0;
}

double d2p_drho2(const orc_params& p, double rho, double T, double alpha) {
    const double a = p.a, b = p.b, R = p.R;
    switch (p.eos) {
        case 0:
            return 2.0 * R * T * b / (sq(1.0 - b * rho) * (1.0 - b * rho)) - 2.0 * a;
        case 3:
        case 4: {
            // d2/drho2 [rho^2/(1+b rho)] = 2/(1+b rho)^3
            double s = 1.0 + b * rho;
            return 2.0 * R * T * b / (sq(1.0 - b * rho) * (1.0 - b * rho)) - a * alpha * 2.0 / (s * s * s);
        }
        case 1: {
            // h = rho^2 / q ; h'' = (2 q^2 - 4 rho q q' - rho^2 q q'' + 2 rho^2 q'^2) / q^3
            double q = 1.0 + 2.0 * b * rho - b * b * rho * rho;
            double qp = 2.0 * b - 2.0 * b * b * rho;
            double qpp = -2.0 * b * b;
            double h2 = (2.0 * q * q - 4.0 * rho * q * qp - rho * rho * q * qpp + 2.0 * rho * rho * qp * qp) /
                        (q * q * q);
            return 2.0 * R * T * b / (sq(1.0 - b * rho) * (1.0 - b * rho)) - a * alpha * h2;
        }
        case 2: {
            // d2/drho2 [rho Z] = (b/4) [2 Z'(eta) + eta Z''(eta)]
            // with Z = num/den: write Z = N D^-1, D = (1-eta)^3.
            double e = b * rho / 4.0;
            double N = 1.0 + e + e * e - e * e * e;
            double Np = 1.0 + 2.0 * e - 3.0 * e * e;
            double Npp = 2.0 - 6.0 * e;
            double om = 1.0 - e;
            // Z' = Np/om^3 + 3 N/om^4 ; Z'' = Npp/om^3 + 6 Np/om^4 + 12 N/om^5
            double Zp = Np / (om * om * om) + 3.0 * N / (om * om * om * om);
            double Zpp = Npp / (om * om * om) + 6.0 * Np / (om * om * om * om) + 12.0 * N / (om * om * om * om * om);
            return R * T * (b / 4.0) * (2.0 * Zp + e * Zpp) - 2.0 * a;
        }
    }
    return 0.0;
}

// Pole of the repulsive term: the EOS is defined for rho < rho_max.
double rho_max_of(const orc_params& p) { return (p.eos == 2) ? 4.0 / p.b : 1.0 / p.b; }

// Critical point: d p/d rho = d2 p/d rho2 = 0.  For PR and RKS alpha(Tc) = 1,
// for VDW and CS alpha is absent, for RK alpha = 1/sqrt(T) varies with T.
// Plain nested bisection: for a trial T, rho_i(T) solves d2p/drho2 = 0 (the
// inflection of the isotherm); T is bisected on the sign of dp/drho(rho_i(T), T).
struct CritResult { double Tc, rhoc; int ok; };

double alpha_for_crit(const orc_params& p, double T) {
    if (p.eos == 3) return 1.0 / std::sqrt(T);
    return 1.0;
}

double inflection_rho(const orc_params& p, double T) {
    // d2p/drho2 is negative at rho -> 0 (attraction dominates: -2a alpha) and
    // positive near the pole; scan for the first sign change then bisect.
    double rmax = rho_max_of(p);
    double al = alpha_for_crit(p, T);
    const int NS = 4000;
    double lo = 0.0, hi = -1.0;
    double prev = d2p_drho2(p, 0.0, T, al);
    for (int i = 1; i < NS; ++i) {
        double r = rmax * (double)i / (double)NS;
        double v = d2p_drho2(p, r, T, al);
        if (prev < 0.0 && v >= 0.0) { lo = rmax * (double)(i - 1) / NS; hi = r; break; }
        prev = v;
    }
    // No sign change: either the isotherm is convex from rho = 0 (no inflection,
    // -1) or its inflection lies beyond the last scan point next to the pole.
    if (hi < 0.0) return (d2p_drho2(p, 0.0, T, al) >= 0.0) ? -1.0 : rmax * (double)(NS - 1) / NS;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (d2p_drho2(p, mid, T, al) < 0.0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

CritResult critical_point(const orc_params& p) {
    CritResult c{0, 0, 0};
    if (p.eos == 0) {  // closed form for VDW
        c.Tc = 8.0 * p.a / (27.0 * p.b * p.R);
        c.rhoc = 1.0 / (3.0 * p.b);
        c.ok = 1;
        return c;
    }
    // Bracket T: at tiny T the isotherm has a loop (dp/drho < 0 at the
    // inflection); above Tc it is monotone (dp/drho >= 0 at the inflection, or
    // no inflection at all).
    auto monotone = [&](double T) {
        double r = inflection_rho(p, T);
        return r < 0.0 || dp_drho(p, r, T, alpha_for_crit(p, T)) >= 0.0;
    };
    double Tlo = 1e-6 * p.a / (p.b * p.R), Thi = Tlo;
    int it0 = 0;
    for (; it0 < 200 && !monotone(Thi); ++it0) { Tlo = Thi; Thi *= 2.0; }
    if (it0 == 0 || it0 == 200) return c;
    for (int it = 0; it < 300; ++it) {
        double mid = 0.5 * (Tlo + Thi);
        if (mid <= Tlo || mid >= Thi) break;
        if (monotone(mid)) Thi = mid; else Tlo = mid;
    }
    c.Tc = 0.5 * (Tlo + Thi);
    c.rhoc = inflection_rho(p, c.Tc);
    c.ok = c.rhoc > 0.0;
    return c;
}

// Maxwell equal-area rule (Sec. 5.2): at T < Tc find p0, rho_v < rho_l with
// p(rho_v) = p(rho_l) = p0 and  integral_{v_l}^{v_v} (p(v) - p0) dv = 0,  v = 1/rho.
// In rho:  integral_{rho_v}^{rho_l} (p(rho) - p0) / rho^2 d rho = 0, evaluated in
// s = ln rho by composite 8-point Gauss-Legendre.
const double GL8_X[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290, -0.1834346424956498,
                         0.1834346424956498,  0.5255324099163290,  0.7966664774136267,  0.9602898564975363};
const double GL8_W[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066053494100, 0.3626837833783620,
                         0.3626837833783620, 0.3137066053494100, 0.2223810344533745, 0.1012285362903763};

struct Isotherm {
    orc_params p;
    double T, alpha;
    double P(double rho) const { return p_eos_alpha<double>(p, rho, T, alpha); }
    double dP(double rho) const { return dp_drho(p, rho, T, alpha); }
};

double bisect_p(const Isotherm& iso, double lo, double hi, double target) {
    // p is increasing on [lo, hi]; find rho with p(rho) = target.
    for (int it = 0; it < 300; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (iso.P(mid) < target) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

double area_integral(const Isotherm& iso, double rv, double rl, double p0) {
    const int NP = 512;
    double s0 = std::log(rv), s1 = std::log(rl), hs = (s1 - s0) / NP;
    double sum = 0.0;
    for (int k = 0; k < NP; ++k) {
        double c = s0 + (k + 0.5) * hs;
        for (int j = 0; j < 8; ++j) {
            double s = c + 0.5 * hs * GL8_X[j];
            double rho = std::exp(s);
            // (p - p0)/rho^2 d rho = (p - p0)/rho ds
            sum += 0.5 * hs * GL8_W[j] * (iso.P(rho) - p0) / rho;
        }
    }
    return sum;
}

int maxwell(const orc_params& p, double T, double* rho_v, double* rho_l, double* p0out) {
    CritResult c = critical_point(p);
    if (!c.ok || !(T > 0.0) || T >= c.Tc) return 1;
    Isotherm iso{p, T, alpha_of<double>(p, T, c.Tc)};
    double rmax = rho_max_of(p);
    // Spinodals: dp/drho vanishes at s1 < s2; dp/drho is positive at rho -> 0
    // and near the pole, negative between.  Locate the minimum of dp/drho on a
    // scan, refine it by golden section, then bisect on each side.
    const int NS = 20000;
    double best = 1e300, rbest = 0.0;
    for (int i = 1; i < NS; ++i) {
        double r = rmax * (double)i / NS;
        double v = iso.dP(r);
        if (v < best) { best = v; rbest = r; }
    }
    double lo = std::max(rbest - rmax / NS, 1e-300), hi = std::min(rbest + rmax / NS, rmax * (1 - 1e-15));
    const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
    for (int it = 0; it < 200; ++it) {
        double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
        if (iso.dP(x1) < iso.dP(x2)) hi = x2; else lo = x1;
    }
    double rmin = 0.5 * (lo + hi);
    if (!(iso.dP(rmin) < 0.0)) return 2;
    auto root_dp = [&](double a0, double b0, bool increasing_side) {
        // dp/drho > 0 at a0 if !increasing_side ...
        double a1 = a0, b1 = b0;
        for (int it = 0; it < 300; ++it) {
            double mid = 0.5 * (a1 + b1);
            if (mid <= a1 || mid >= b1) break;
            bool pos = iso.dP(mid) > 0.0;
            if (increasing_side) { if (pos) b1 = mid; else a1 = mid; }
            else { if (pos) a1 = mid; else b1 = mid; }
        }
        return 0.5 * (a1 + b1);
    };
    double s1 = root_dp(0.0, rmin, false);   // dp/drho goes + -> -
    double s2 = root_dp(rmin, rmax * (1 - 1e-15), true);  // - -> +
    double pmax = iso.P(s1), pmin = std::max(iso.P(s2), 0.0);
    // The area integral decreases as p0 increases.
    double plo = pmin, phi = pmax;
    double rv = 0, rl = 0;
    for (int it = 0; it < 200; ++it) {
        double pm = 0.5 * (plo + phi);
        if (pm <= plo || pm >= phi) break;
        rv = bisect_p(iso, 0.0, s1, pm);
        rl = bisect_p(iso, s2, rmax * (1 - 1e-15), pm);
        double E = area_integral(iso, rv, rl, pm);
        if (E > 0.0) plo = pm; else phi = pm;
    }
    double pm = 0.5 * (plo + phi);
    *rho_v = bisect_p(iso, 0.0, s1, pm);
    *rho_l = bisect_p(iso, s2, rmax * (1 - 1e-15), pm);
    if (p0out) *p0out = pm;
    return 0;
}

// ---------------------------------------------------------------- Sec. 5.1, Eqs. 25-26
// Flat interface along y in the fluid of Eq. 25 (square-gradient pressure
// tensor with constant kappa) with the k-scaled EOS p_m = k p_EOS (Sec. 5).
// Mechanical equilibrium (Eq. 26) in a flat interface leaves one component:
//   P_yy = p_m(rho) - kappa rho rho'' - (kappa/2) rho'^2 + kappa rho'^2
// is uniform and equal to the bulk (coexistence) pressure k p0.  Its first
// integral is (kappa/2) rho'^2 = W(rho) with
//   W(rho) = rho * integral_{rho_b}^{rho} (p_m(s) - k p0) / s^2 ds,
// where rho_b may be either bulk density (the integral between them vanishes:
// the equal-area rule), so rho' = sqrt(2 W / kappa) where rho rises with y.
// (Differentiating: kappa rho'' = W'(rho) = W/rho + p_m - k p0, which puts
// P_yy back to k p0.)
struct Interface {
    Isotherm iso;
    double k, p0, rv, rl;
};

bool make_interface(const orc_params& p, Interface* f) {
    CritResult c = critical_point(p);
    if (!c.ok || !(p.T > 0.0) || p.T >= c.Tc) return false;
    f->iso = Isotherm{p, p.T, alpha_of<double>(p, p.T, c.Tc)};
    f->k = p.k;
    return maxwell(p, p.T, &f->rv, &f->rl, &f->p0) == 0;
}

// W(rho) by composite 8-point Gauss-Legendre from the nearer bulk density.
double excess_W(const Interface& f, double rho) {
    const double ref = (rho > 0.5 * (f.rv + f.rl)) ? f.rl : f.rv;
    const int NP = 64;
    const double hs = (rho - ref) / NP;
    double sum = 0.0;
    for (int k = 0; k < NP; ++k) {
        const double c = ref + (k + 0.5) * hs;
        for (int j = 0; j < 8; ++j) {
            const double s = c + 0.5 * hs * GL8_X[j];
            sum += 0.5 * hs * GL8_W[j] * f.k * (f.iso.P(s) - f.p0) / (s * s);
        }
    }
    const double W = rho * sum;
    return W > 0.0 ? W : 0.0;  // W >= 0; only rounding takes it below zero next to a bulk density
}

// d rho / dy on the rising interface.
double slope(const Interface& f, double kappa, double rho) { return std::sqrt(2.0 * excess_W(f, rho) / kappa); }

// ---------------------------------------------------------------- Sec. 3 stencils
// High-order difference, Eq. 20 with h = 1 on a periodic line of n points:
//   (1/3) y_{i-1} + y_i + (1/3) y_{i+1} = (1/36)(u_{i+2} - u_{i-2}) + (7/9)(u_{i+1} - u_{i-1}).
// The cyclic tridiagonal system is split as T + w v^T (Sherman-Morrison); both
// solves with the tridiagonal T use the chasing (Thomas) sweep.
template <typename S>
void thomas(int n, const double* sub, const double* diag, const double* sup, const S* d, S* x) {
    std::vector<double> cp(n);
    std::vector<S> dp(n);
    cp[0] = sup[0] / diag[0];
    dp[0] = d[0] / diag[0];
    for (int i = 1; i < n; ++i) {
        double m = diag[i] - sub[i] * cp[i - 1];
        cp[i] = (i < n - 1) ? sup[i] / m : 0.0;
        dp[i] = (d[i] - sub[i] * dp[i - 1]) / m;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
}

template <typename S>
void hdm_line(int n, const S* u, long su, S* y, long sy) {
    const double third = 1.0 / 3.0;
    std::vector<S> rhs(n), x(n);
    for (int i = 0; i < n; ++i) {
        S up2 = u[((i + 2) % n) * su], um2 = u[((i - 2 + 2 * n) % n) * su];
        S up1 = u[((i + 1) % n) * su], um1 = u[((i - 1 + n) % n) * su];
        rhs[i] = (up2 - um2) / 36.0 + 7.0 * (up1 - um1) / 9.0;
    }
    // A = T + w v^T with corners A[0][n-1] = beta = 1/3, A[n-1][0] = alpha = 1/3,
    // gamma = -A[0][0]; w = (gamma, 0..0, alpha), v = (1, 0..0, beta/gamma).
    const double beta = third, alph = third, gamma = -1.0;
    std::vector<double> sub(n, third), diag(n, 1.0), sup(n, third);
    diag[0] = 1.0 - gamma;
    diag[n - 1] = 1.0 - alph * beta / gamma;
    thomas<S>(n, sub.data(), diag.data(), sup.data(), rhs.data(), x.data());
    std::vector<double> wv(n, 0.0), z(n);
    wv[0] = gamma;
    wv[n - 1] = alph;
    thomas<double>(n, sub.data(), diag.data(), sup.data(), wv.data(), z.data());
    S fact = (x[0] + beta * x[n - 1] / gamma) / (1.0 + z[0] + beta * z[n - 1] / gamma);
    for (int i = 0; i < n; ++i) y[i * sy] = x[i] - fact * z[i];
}

// Eq. 20 on a line of n points between two walls (halfway, at -1/2 and
// n - 1/2) with the mirror continuation u_{-1-j} = u_j, u_{n+j} = u_{n-1-j};
// the derivative of such an even continuation is odd: y'_{-1} = -y'_0,
// y'_n = -y'_{n-1}.  Substituting both into the first and last rows of Eq. 20
// leaves a plain tridiagonal system with diagonal 2/3 in those two rows, solved
// by the chasing method.
inline int mirror_index(int j, int n) { return j < 0 ? -1 - j : (j >= n ? 2 * n - 1 - j : j); }

template <typename S>
void hdm_line_walls(int n, const S* u, long su, S* y, long sy) {
    const double third = 1.0 / 3.0;
    std::vector<S> rhs(n), x(n);
    for (int i = 0; i < n; ++i) {
        S up2 = u[mirror_index(i + 2, n) * su], um2 = u[mirror_index(i - 2, n) * su];
        S up1 = u[mirror_index(i + 1, n) * su], um1 = u[mirror_index(i - 1, n) * su];
        rhs[i] = (up2 - um2) / 36.0 + 7.0 * (up1 - um1) / 9.0;
    }
    std::vector<double> sub(n, third), diag(n, 1.0), sup(n, third);
    diag[0] -= third;
    diag[n - 1] -= third;
    thomas<S>(n, sub.data(), diag.data(), sup.data(), rhs.data(), x.data());
    for (int i = 0; i < n; ++i) y[i * sy] = x[i];
}

// Eq. 14 between two walls: the same mirror continuation.
template <typename S>
void cdm_line_walls(int n, const S* u, long su, S* y, long sy) {
    for (int i = 0; i < n; ++i) y[i * sy] = (u[mirror_index(i + 1, n) * su] - u[mirror_index(i - 1, n) * su]) / 2.0;
}

// Central difference, Eq. 14 with h = 1, periodic.
template <typename S>
void cdm_line(int n, const S* u, long su, S* y, long sy) {
    for (int i = 0; i < n; ++i) y[i * sy] = (u[((i + 1) % n) * su] - u[((i - 1 + n) % n) * su]) / 2.0;
}

template <typename S>
void derivative_line(int grad, int n, const S* u, long su, S* y, long sy) {
    if (grad == 1) cdm_line<S>(n, u, su, y, sy);
    else hdm_line<S>(n, u, su, y, sy);
}

// Weighted D2Q9 central difference, Eq. 15 of Sec. 3.1, periodic, with the
// factor 1/c_s^2 = 3 that the printed sum lacks (sum_i w_i e_ix e_ix = 1/3,
// so the printed sum is c_s^2 du/dx):
//   du/dx(x) = 3 sum_i w_i u(x + e_i) e_ix,   du/dy(x) = 3 sum_i w_i u(x + e_i) e_iy.
// axis 0 gives d/dx, axis 1 d/dy.
template <typename S>
void d2q9_derivative(int axis, int nx, int ny, const S* u, S* out) {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            S acc(0.0);
            for (int i = 1; i < 9; ++i) {
                const int e = (axis == 0) ? EX[i] : EY[i];
                const int xn = (x + EX[i] + nx) % nx, yn = (y + EY[i] + ny) % ny;
                acc = acc + (3.0 * WQ[i] * e) * u[(size_t)yn * nx + xn];
            }
            out[(size_t)y * nx + x] = acc;
        }
    }
}

// d/dx (axis 0) or d/dy (axis 1) of the field u [ny][nx] with the gradient
// scheme `grad`: 0 Eq. 20 and 1 Eq. 14, each along its own grid lines (d/dx
// along every row, d/dy along every column); 2 the two-dimensional Eq. 15.
// With walls (y only, grads 0 and 1) the y lines use the mirror closure.
template <typename S>
void derivative(int grad, int axis, int nx, int ny, const S* u, S* out, int walls = 0) {
    if (grad == 2) {
        d2q9_derivative<S>(axis, nx, ny, u, out);
    } else if (axis == 0) {
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y) derivative_line<S>(grad, nx, &u[(size_t)y * nx], 1, &out[(size_t)y * nx], 1);
    } else if (walls) {
#pragma omp parallel for schedule(static)
        for (int x = 0; x < nx; ++x) {
            if (grad == 1) cdm_line_walls<S>(ny, &u[x], nx, &out[x], nx);
            else hdm_line_walls<S>(ny, &u[x], nx, &out[x], nx);
        }
    } else {
#pragma omp parallel for schedule(static)
        for (int x = 0; x < nx; ++x) derivative_line<S>(grad, ny, &u[x], nx, &out[x], nx);
    }
}

// ---------------------------------------------------------------- Eq. 2
template <typename S>
S feq(int i, S rho, S ux, S uy) {
    S eu = EX[i] * ux + EY[i] * uy;
    S uu = ux * ux + uy * uy;
    return rho * WQ[i] * (S(1.0) + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

// ---------------------------------------------------------------- one step
template <typename S>
struct Work {
    std::vector<S> rho, jx, jy, U, phi, gx, gy, gux, guy, Fx, Fy;
    void resize(size_t n) {
        rho.resize(n); jx.resize(n); jy.resize(n); U.resize(n); phi.resize(n);
        gx.resize(n); gy.resize(n); gux.resize(n); guy.resize(n); Fx.resize(n); Fy.resize(n);
    }
};

struct Model {
    orc_params p;
    double Tc;
};

Model make_model(const orc_params& p) {
    Model m{p, 0.0};
    if (p.eos == 1 || p.eos == 4) m.Tc = critical_point(p).Tc;
    return m;
}

// Scaled potential U = g (k p_EOS(rho, T) - rho c_s^2)  (Eq. 8, Hu's scaling, multiplier g).
template <typename S>
S potential_U(const Model& m, S rho, S T, S g) {
    S al = alpha_of<S>(m.p, T, m.Tc);
    return g * (m.p.k * p_eos_alpha<S>(m.p, rho, T, al) - rho / 3.0);
}

// Moments (Eq. 3), potential (Eqs. 8, 21), derivatives (Eq. 20 or 14) and the
// interaction force (Eq. 22 Shan-Chen, Eq. 7 Zhang-Chen, Eq. 9 hybrid).
template <typename S>
void forces(const Model& m, const S* f, S T, S g, Work<S>& w) {
    const int nx = m.p.nx, ny = m.p.ny;
    const size_t N = (size_t)nx * ny;
    w.resize(N);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)N; ++c) {
        S r = f[0 * N + c], jx(0.0), jy(0.0);
        for (int i = 1; i < 9; ++i) r = r + f[i * N + c];
        for (int i = 0; i < 9; ++i) {
            jx = jx + (double)EX[i] * f[i * N + c];
            jy = jy + (double)EY[i] * f[i * N + c];
        }
        w.rho[c] = r; w.jx[c] = jx; w.jy[c] = jy;
        S U = potential_U<S>(m, r, T, g);
        w.U[c] = U;
        // Eq. 21: Phi = sqrt(|U|)
        w.phi[c] = (val(U) >= 0.0) ? sqrt(U) : sqrt(-U);
    }
    const bool need_phi = (m.p.force == 0 || m.p.force == 2);
    const bool need_U = (m.p.force == 1 || m.p.force == 2);
    if (need_phi) {
        derivative<S>(m.p.grad, 0, nx, ny, w.phi.data(), w.gx.data());
        derivative<S>(m.p.grad, 1, nx, ny, w.phi.data(), w.gy.data(), m.p.walls);
    }
    if (need_U) {
        derivative<S>(m.p.grad, 0, nx, ny, w.U.data(), w.gux.data());
        derivative<S>(m.p.grad, 1, nx, ny, w.U.data(), w.guy.data(), m.p.walls);
    }
#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)N; ++c) {
        S fsx(0.0), fsy(0.0), fzx(0.0), fzy(0.0);
        if (need_phi) {
            // Eq. 22: F = -2 Phi grad Phi if U >= 0, +2 Phi grad Phi if U < 0.
            double s = (val(w.U[c]) >= 0.0) ? 1.0 : -1.0;
            fsx = -2.0 * s * w.phi[c] * w.gx[c];
            fsy = -2.0 * s * w.phi[c] * w.gy[c];
        }
        if (need_U) {
            // Eq. 7: F = -grad U.
            fzx = -w.gux[c];
            fzy = -w.guy[c];
        }
        if (m.p.force == 0) { w.Fx[c] = fsx; w.Fy[c] = fsy; }
        else if (m.p.force == 1) { w.Fx[c] = fzx; w.Fy[c] = fzy; }
        else {
            // Eq. 9: F = A F^ZC + (1 - 2A) F^SC
            w.Fx[c] = m.p.A * fzx + (1.0 - 2.0 * m.p.A) * fsx;
            w.Fy[c] = m.p.A * fzy + (1.0 - 2.0 * m.p.A) * fsy;
        }
    }
}

// BGK collision with Kupershtokh's exact-difference forcing (Eqs. 1, 2, 10):
//   f*_i = f_i - (f_i - f^eq_i(rho, u)) / tau + [f^eq_i(rho, u + du) - f^eq_i(rho, u)],
//   u = j / rho, du = F dt / rho, dt = 1.
template <typename S>
void collide_cell(const S* fi, S rho, S jx, S jy, S Fx, S Fy, double tau, S* out) {
    S ux = jx / rho, uy = jy / rho;
    S dux = Fx / rho, duy = Fy / rho;
    for (int i = 0; i < 9; ++i) {
        S e0 = feq<S>(i, rho, ux, uy);
        S e1 = feq<S>(i, rho, ux + dux, uy + duy);
        out[i] = fi[i] - (fi[i] - e0) / tau + (e1 - e0);
    }
}

// Opposite D2Q9 direction.
int opposite(int i) {
    for (int j = 0; j < 9; ++j)
        if (EX[j] == -EX[i] && EY[j] == -EY[i]) return j;
    return i;
}

// One full time step f_t -> f_{t+1} (Eq. 1): collide everywhere, then stream
// f_i(x + e_i) <- f*_i(x) with periodic wrap (in x always; in y unless there
// are walls).  With walls a population whose step would cross y = -1/2 or
// ny - 1/2 returns to its own site reversed (halfway bounce-back, no slip).
// Layout f[i][y][x].
template <typename S>
void step(const Model& m, const S* f, S* fout, S T, S g, Work<S>& w) {
    const int nx = m.p.nx, ny = m.p.ny;
    const size_t N = (size_t)nx * ny;
    forces<S>(m, f, T, g, w);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t c = (size_t)y * nx + x;
            S fi[9], fs[9];
            for (int i = 0; i < 9; ++i) fi[i] = f[i * N + c];
            collide_cell<S>(fi, w.rho[c], w.jx[c], w.jy[c], w.Fx[c], w.Fy[c], m.p.tau, fs);
            for (int i = 0; i < 9; ++i) {
                if (m.p.walls && (y + EY[i] < 0 || y + EY[i] >= ny)) {
                    fout[opposite(i) * N + c] = fs[i];
                    continue;
                }
                int xd = (x + EX[i] + nx) % nx, yd = (y + EY[i] + ny) % ny;
                fout[i * N + (size_t)yd * nx + xd] = fs[i];
            }
        }
    }
}


// ---------------------------------------------------------------- adjoint
// Reverse mode of one step (Eqs. 1, 2, 3, 7-10, 20-22), obtained by the chain
// rule written out by hand.  With the equilibrium in momentum form
//   A_i(rho, m) = w_i [rho + 3 e_i.m + (4.5 (e_i.m)^2 - 1.5 |m|^2) / rho]
// (A_i(rho, rho u) = f^eq_i(rho, u)), the collision of Eqs. 1 and 10 reads
//   f*_i = (1 - 1/tau) f_i + (1/tau - 1) A_i(rho, j) + A_i(rho, j + F),
// and the step is f_{t+1,i}(x + e_i) = f*_i(x).  Given lam = dJ/df_{t+1}:
//   mu_i(x) = lam_i(x + e_i)                                  (streaming)
//   rho_bar, j_bar, F_bar from the partial derivatives of A    (collision)
//   U_bar from F_bar through the force (D^T = -D: for Eq. 20, A is symmetric
//        and B antisymmetric, both circulant, so A^-1 B is antisymmetric; Eqs. 14
//        and 15 have coefficients odd in the offset e_i)
//   dJ/df_k(x) = (1 - 1/tau) mu_k + rho_bar + e_k.j_bar + U_bar dU/drho,
// and the parameter gradients dJ/dg = sum U_bar dU/dg, dJ/dT = sum U_bar dU/dT.
// dU/drho, dU/dg and dU/dT come from the dual-number evaluation of U.
void dA_drho_dm(int i, double rho, double mx, double my, double* drho, double* dmx, double* dmy) {
    double em = EX[i] * mx + EY[i] * my;
    double m2 = mx * mx + my * my;
    *drho = WQ[i] * (1.0 - (4.5 * em * em - 1.5 * m2) / (rho * rho));
    *dmx = WQ[i] * (3.0 * EX[i] + (9.0 * em * EX[i] - 3.0 * mx) / rho);
    *dmy = WQ[i] * (3.0 * EY[i] + (9.0 * em * EY[i] - 3.0 * my) / rho);
}

void adjoint_step(const Model& m, const double* f, const double* lam_next, double* lam, double* grad) {
    const int nx = m.p.nx, ny = m.p.ny;
    const size_t N = (size_t)nx * ny;
    Work<double> w;
    forces<double>(m, f, m.p.T, m.p.g, w);
    std::vector<double> Fbx(N), Fby(N), rbar(N), jbx(N), jby(N);
    const double tau = m.p.tau;
    // collision and streaming
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t c = (size_t)y * nx + x;
            double mu[9];
            for (int i = 0; i < 9; ++i) {
                int xd = (x + EX[i] + nx) % nx, yd = (y + EY[i] + ny) % ny;
                mu[i] = lam_next[i * N + (size_t)yd * nx + xd];
            }
            double rho = w.rho[c], jx = w.jx[c], jy = w.jy[c];
            double mx = jx + w.Fx[c], my = jy + w.Fy[c];
            double rb = 0, jbx_ = 0, jby_ = 0, fbx = 0, fby = 0;
            for (int i = 0; i < 9; ++i) {
                double a_r, a_x, a_y, b_r, b_x, b_y;
                dA_drho_dm(i, rho, jx, jy, &a_r, &a_x, &a_y);
                dA_drho_dm(i, rho, mx, my, &b_r, &b_x, &b_y);
                rb += mu[i] * ((1.0 / tau - 1.0) * a_r + b_r);
                jbx_ += mu[i] * ((1.0 / tau - 1.0) * a_x + b_x);
                jby_ += mu[i] * ((1.0 / tau - 1.0) * a_y + b_y);
                fbx += mu[i] * b_x;
                fby += mu[i] * b_y;
            }
            for (int k = 0; k < 9; ++k) lam[k * N + c] = (1.0 - 1.0 / tau) * mu[k] + rb + EX[k] * jbx_ + EY[k] * jby_;
            rbar[c] = rb; jbx[c] = jbx_; jby[c] = jby_;
            Fbx[c] = fbx; Fby[c] = fby;
        }
    }
    // force -> U_bar
    std::vector<double> Ubar(N, 0.0), ax(N), ay(N), dax(N), day(N);
    const bool sc = (m.p.force == 0 || m.p.force == 2), zc = (m.p.force == 1 || m.p.force == 2);
    const double wsc = (m.p.force == 2) ? (1.0 - 2.0 * m.p.A) : 1.0;
    const double wzc = (m.p.force == 2) ? m.p.A : 1.0;
    if (sc) {
        // F = -2 s Phi (D_x Phi, D_y Phi):  Phi_bar = -2 s (F_bar . D Phi) + D^T(-2 s Phi F_bar)
        for (size_t c = 0; c < N; ++c) {
            double s = (w.U[c] >= 0.0) ? 1.0 : -1.0;
            ax[c] = -2.0 * s * w.phi[c] * wsc * Fbx[c];
            ay[c] = -2.0 * s * w.phi[c] * wsc * Fby[c];
        }
        derivative<double>(m.p.grad, 0, nx, ny, ax.data(), dax.data());
        derivative<double>(m.p.grad, 1, nx, ny, ay.data(), day.data());
        for (size_t c = 0; c < N; ++c) {
            double s = (w.U[c] >= 0.0) ? 1.0 : -1.0;
            double phibar = -2.0 * s * wsc * (Fbx[c] * w.gx[c] + Fby[c] * w.gy[c]) - dax[c] - day[c];
            // Phi = sqrt|U|: dPhi/dU = s / (2 Phi)
            Ubar[c] += phibar * s / (2.0 * w.phi[c]);
        }
    }
    if (zc) {
        // F = -(D_x U, D_y U):  U_bar = -D^T F_bar = D_x F_bar_x + D_y F_bar_y
        for (size_t c = 0; c < N; ++c) { ax[c] = wzc * Fbx[c]; ay[c] = wzc * Fby[c]; }
        derivative<double>(m.p.grad, 0, nx, ny, ax.data(), dax.data());
        derivative<double>(m.p.grad, 1, nx, ny, ay.data(), day.data());
        for (size_t c = 0; c < N; ++c) Ubar[c] += dax[c] + day[c];
    }
    // U = g (k p(rho, T) - rho/3): chain into rho and the parameters
    double gg = 0.0, gT = 0.0;
    for (size_t c = 0; c < N; ++c) {
        Dual dr = potential_U<Dual>(m, Dual(w.rho[c], 1.0), Dual(m.p.T, 0.0), Dual(m.p.g, 0.0));
        Dual dT = potential_U<Dual>(m, Dual(w.rho[c], 0.0), Dual(m.p.T, 1.0), Dual(m.p.g, 0.0));
        Dual dg = potential_U<Dual>(m, Dual(w.rho[c], 0.0), Dual(m.p.T, 0.0), Dual(m.p.g, 1.0));
        double rnl = Ubar[c] * dr.d;
        for (int k = 0; k < 9; ++k) lam[k * N + c] += rnl;
        gg += Ubar[c] * dg.d;
        gT += Ubar[c] * dT.d;
    }
    grad[0] += gg;
    grad[1] += gT;
}

}  // namespace

// ================================================================ C API
extern "C" {

// Number of OpenMP threads the parallel loops use (1 without OpenMP).
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_critical(const orc_params* p, double* Tc, double* rhoc) {
    CritResult c = critical_point(*p);
    *Tc = c.Tc;
    *rhoc = c.rhoc;
    return c.ok ? 0 : 1;
}

int orc_maxwell(const orc_params* p, double T, double* rho_v, double* rho_l, double* p0) {
    return maxwell(*p, T, rho_v, rho_l, p0);
}

// p_EOS, dp/drho, d2p/drho2 at (rho, T) with the EOS's own alpha(T).
void orc_eos(const orc_params* p, double rho, double T, double* pe, double* dp, double* d2p) {
    Model m = make_model(*p);
    double al = alpha_of<double>(*p, T, m.Tc);
    if (pe) *pe = p_eos_alpha<double>(*p, rho, T, al);
    if (dp) *dp = dp_drho(*p, rho, T, al);
    if (d2p) *d2p = d2p_drho2(*p, rho, T, al);
}

void orc_hdm_line(int n, const double* u, double* du) { hdm_line<double>(n, u, 1, du, 1); }
void orc_hdm_line_walls(int n, const double* u, double* du) { hdm_line_walls<double>(n, u, 1, du, 1); }
void orc_cdm_line_walls(int n, const double* u, double* du) { cdm_line_walls<double>(n, u, 1, du, 1); }

// Both derivatives of a field u [ny][nx] with the scheme p->grad (the step's
// gradient operator, Sec. 3): gx = d/dx, gy = d/dy.
void orc_gradient(const orc_params* p, const double* u, double* gx, double* gy) {
    derivative<double>(p->grad, 0, p->nx, p->ny, u, gx);
    derivative<double>(p->grad, 1, p->nx, p->ny, u, gy, p->walls);
}
void orc_cdm_line(int n, const double* u, double* du) { cdm_line<double>(n, u, 1, du, 1); }

void orc_feq(double rho, double ux, double uy, double* out9) {
    for (int i = 0; i < 9; ++i) out9[i] = feq<double>(i, rho, ux, uy);
}

// Collision of a single cell with a given force (for EDM pins).
void orc_collide_cell(const double* f9, double Fx, double Fy, double tau, double* out9) {
    double rho = f9[0], jx = 0, jy = 0;
    for (int i = 1; i < 9; ++i) rho += f9[i];
    for (int i = 0; i < 9; ++i) { jx += EX[i] * f9[i]; jy += EY[i] * f9[i]; }
    collide_cell<double>(f9, rho, jx, jy, Fx, Fy, tau, out9);
}

// "Exact" flat-interface profile of Sec. 5.1 (Eqs. 25-26): rho and rho' at
// y_i = (i - (n - 1)/2) h, i < n, for the interface rising with y through
// rho(0) = (rho_v + rho_l)/2.  Classic fourth-order Runge-Kutta on
// rho' = sqrt(2 W(rho) / kappa) from y = 0 outwards, steps of at most h/32.
int orc_flat_profile(const orc_params* p, double kappa, double h, int n, double* rho, double* drho) {
    Interface f;
    if (!(kappa > 0.0) || !(h > 0.0) || n < 1 || !make_interface(*p, &f)) return 1;
    auto F = [&](double r) { return slope(f, kappa, r); };
    const double c = 0.5 * (n - 1);
    for (int dir = -1; dir <= 1; dir += 2) {
        double y = 0.0, r = 0.5 * (f.rv + f.rl);
        // grid points on this side, nearest first (y = 0 itself on the upper side)
        for (int i = (dir > 0) ? (int)std::ceil(c) : (int)std::ceil(c) - 1; i >= 0 && i < n; i += dir) {
            const double yt = (i - c) * h;
            const int m = (int)std::ceil(std::fabs(yt - y) / (h / 32.0));
            const double dy = (m > 0) ? (yt - y) / m : 0.0;
            for (int s = 0; s < m; ++s) {
                const double k1 = F(r), k2 = F(r + 0.5 * dy * k1), k3 = F(r + 0.5 * dy * k2), k4 = F(r + dy * k3);
                r += dy * (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0;
            }
            y = yt;
            rho[i] = r;
            drho[i] = F(r);
        }
    }
    return 0;
}

// Surface tension by the integration method (Sec. 5.3) with the tensor of
// Eq. 25: sigma = integral (P_N - P_T) dy = kappa integral rho'^2 dy.  For a
// periodic column of n sites (h = 1) holding two interfaces (a slab) the
// derivative is Eq. 20 and each interface gets half of kappa sum (D rho)^2.
double orc_sigma_slab(double kappa, int n, const double* rho) {
    std::vector<double> d(n);
    hdm_line<double>(n, rho, 1, d.data(), 1);
    double sum = 0.0;
    for (int i = 0; i < n; ++i) sum += d[i] * d[i];
    return 0.5 * kappa * sum;
}

// The same integral in closed form for the exact profile: with
// (kappa/2) rho'^2 = W, kappa integral rho'^2 dy = integral_{rho_v}^{rho_l} sqrt(2 kappa W) d rho.
int orc_sigma_exact(const orc_params* p, double kappa, double* sigma) {
    Interface f;
    if (!(kappa > 0.0) || !make_interface(*p, &f)) return 1;
    const int NP = 256;
    const double hs = (f.rl - f.rv) / NP;
    double sum = 0.0;
    for (int k = 0; k < NP; ++k) {
        const double c = f.rv + (k + 0.5) * hs;
        for (int j = 0; j < 8; ++j) sum += 0.5 * hs * GL8_W[j] * std::sqrt(2.0 * kappa * excess_W(f, c + 0.5 * hs * GL8_X[j]));
    }
    *sigma = sum;
    return 0;
}

// Initial state f = f^eq(rho0, u0) (Eq. 2); ux0 / uy0 may be NULL (u0 = 0).
void orc_init(const orc_params* p, const double* rho0, const double* ux0, const double* uy0, double* f) {
    const size_t N = (size_t)p->nx * p->ny;
    for (size_t c = 0; c < N; ++c) {
        double ux = ux0 ? ux0[c] : 0.0, uy = uy0 ? uy0[c] : 0.0;
        for (int i = 0; i < 9; ++i) f[i * N + c] = feq<double>(i, rho0[c], ux, uy);
    }
}

// Advance f (layout [9][ny][nx], in place) by nsteps.
int orc_run(const orc_params* p, int64_t nsteps, double* f) {
    if (p->nx < 5 || p->ny < 5 || !(p->tau > 0.5)) return 1;
    Model m = make_model(*p);
    const size_t N = (size_t)p->nx * p->ny;
    std::vector<double> buf(9 * N);
    Work<double> w;
    double* cur = f;
    double* nxt = buf.data();
    for (int64_t s = 0; s < nsteps; ++s) {
        step<double>(m, cur, nxt, p->T, p->g, w);
        double* t = cur; cur = nxt; nxt = t;
    }
    if (cur != f) std::memcpy(f, cur, sizeof(double) * 9 * N);
    return 0;
}

// Output moments of the state f: rho (Eq. 3), the half-step velocity v (Eq. 11),
// the bulk pressure p = rho/3 + U, and the force F.  Any output may be NULL.
void orc_moments(const orc_params* p, const double* f, double* rho, double* vx, double* vy, double* pr,
                 double* Fx, double* Fy) {
    Model m = make_model(*p);
    Work<double> w;
    forces<double>(m, f, p->T, p->g, w);
    const size_t N = (size_t)p->nx * p->ny;
    for (size_t c = 0; c < N; ++c) {
        if (rho) rho[c] = w.rho[c];
        if (vx) vx[c] = (w.jx[c] + 0.5 * w.Fx[c]) / w.rho[c];
        if (vy) vy[c] = (w.jy[c] + 0.5 * w.Fy[c]) / w.rho[c];
        if (pr) pr[c] = w.rho[c] / 3.0 + w.U[c];
        if (Fx) Fx[c] = w.Fx[c];
        if (Fy) Fy[c] = w.Fy[c];
    }
}

// Forward-mode tangent of nsteps steps: advances f (in place) and its tangent df
// along a direction that also perturbs T by dT and g by dg.
int orc_tangent_run(const orc_params* p, int64_t nsteps, double* f, double* df, double dT, double dg) {
    if (p->nx < 5 || p->ny < 5 || !(p->tau > 0.5)) return 1;
    Model m = make_model(*p);
    const size_t N = (size_t)p->nx * p->ny;
    std::vector<Dual> a(9 * N), b(9 * N);
    for (size_t i = 0; i < 9 * N; ++i) a[i] = Dual(f[i], df[i]);
    Work<Dual> w;
    Dual T(p->T, dT), g(p->g, dg);
    for (int64_t s = 0; s < nsteps; ++s) {
        step<Dual>(m, a.data(), b.data(), T, g, w);
        a.swap(b);
    }
    for (size_t i = 0; i < 9 * N; ++i) { f[i] = a[i].v; df[i] = a[i].d; }
    return 0;
}


// Reverse mode of one step: lam = (d f_{t+1} / d f_t)^T lam_next for the state f
// (= f_t), and grad[0] += dJ/dg, grad[1] += dJ/dT.  Layouts [9][ny][nx].
int orc_adjoint_step(const orc_params* p, const double* f, const double* lam_next, double* lam, double* grad) {
    if (p->nx < 5 || p->ny < 5 || !(p->tau > 0.5) || p->walls) return 1;
    Model m = make_model(*p);
    adjoint_step(m, f, lam_next, lam, grad);
    return 0;
}

// Gradient of J = sum_x (rho_n(x) - target(x))^2 after nsteps steps from the
// initial state f0 = f^eq(rho0, u0): dJ/df0 (layout [9][ny][nx]), dJ/drho0
// (holding u0 fixed: f^eq is linear in rho), dJ/dg and dJ/dT.  States are kept
// every `every` steps and each segment is recomputed before its reverse sweep.
int orc_adjoint_run(const orc_params* p, int64_t nsteps, int64_t every, const double* rho0, const double* ux0,
                    const double* uy0, const double* target, double* J, double* dJ_df0, double* dJ_drho0,
                    double* grad) {
    if (p->nx < 5 || p->ny < 5 || !(p->tau > 0.5) || every < 1 || p->walls) return 1;
    Model m = make_model(*p);
    const size_t N = (size_t)p->nx * p->ny;
    std::vector<double> f0(9 * N);
    orc_init(p, rho0, ux0, uy0, f0.data());
    const int64_t nseg = (nsteps + every - 1) / every;
    std::vector<std::vector<double>> ck(nseg > 0 ? nseg : 1);
    Work<double> w;
    std::vector<double> cur(f0), nxt(9 * N);
    for (int64_t s = 0; s < nsteps; ++s) {
        if (s % every == 0) ck[s / every] = cur;
        step<double>(m, cur.data(), nxt.data(), p->T, p->g, w);
        cur.swap(nxt);
    }
    // objective and its cotangent at step n
    std::vector<double> lam(9 * N), lam2(9 * N);
    double Jv = 0.0;
    for (size_t c = 0; c < N; ++c) {
        double r = cur[0 * N + c];
        for (int i = 1; i < 9; ++i) r += cur[i * N + c];
        double d = r - target[c];
        Jv += d * d;
        for (int i = 0; i < 9; ++i) lam[i * N + c] = 2.0 * d;
    }
    grad[0] = 0.0;
    grad[1] = 0.0;
    std::vector<std::vector<double>> seg;
    for (int64_t sidx = nseg - 1; sidx >= 0; --sidx) {
        int64_t t0 = sidx * every, t1 = std::min(nsteps, t0 + every);
        seg.assign((size_t)(t1 - t0), std::vector<double>());
        std::vector<double> a = ck[sidx];
        for (int64_t t = t0; t < t1; ++t) {
            seg[(size_t)(t - t0)] = a;
            step<double>(m, a.data(), nxt.data(), p->T, p->g, w);
            a.swap(nxt);
        }
        for (int64_t t = t1 - 1; t >= t0; --t) {
            adjoint_step(m, seg[(size_t)(t - t0)].data(), lam.data(), lam2.data(), grad);
            lam.swap(lam2);
        }
    }
    *J = Jv;
    if (dJ_df0) std::memcpy(dJ_df0, lam.data(), sizeof(double) * 9 * N);
    if (dJ_drho0) {
        for (size_t c = 0; c < N; ++c) {
            double acc = 0.0;
            for (int i = 0; i < 9; ++i) acc += lam[i * N + c] * f0[i * N + c] / rho0[c];
            dJ_drho0[c] = acc;
        }
    }
    return 0;
}

}  // extern "C"

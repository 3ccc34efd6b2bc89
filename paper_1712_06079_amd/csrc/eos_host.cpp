// Host EOS utilities of the library (see eos_host.hpp).
//
// Derivatives of p come from second-order Taylor jets (no hand-differentiated
// formulas).  The critical point uses the fact that every EOS here has the form
// p = T H(rho) - A(T) Q(rho): the two conditions p' = p'' = 0 give
// H' Q'' - H'' Q' = 0 for rho_c alone, then T / A(T) = Q'/H' fixes Tc.
// Coexistence uses the closed-form chemical potential mu = Psi + p/rho with
// Psi = integral of p/rho^2 (equal mu and equal p is the Maxwell equal-area
// rule of Sec. 5.2).
#include "eos_host.hpp"

#include <cmath>

namespace lbm_host {
namespace {

Jet cst(double x) { return Jet{x, 0.0, 0.0}; }
Jet operator+(Jet a, Jet b) { return Jet{a.v + b.v, a.d + b.d, a.c + b.c}; }
Jet operator-(Jet a, Jet b) { return Jet{a.v - b.v, a.d - b.d, a.c - b.c}; }
Jet operator*(Jet a, Jet b) { return Jet{a.v * b.v, a.v * b.d + a.d * b.v, a.v * b.c + a.d * b.d + a.c * b.v}; }
Jet operator*(double s, Jet a) { return Jet{s * a.v, s * a.d, s * a.c}; }
Jet operator/(Jet a, Jet b) {
    double qv = a.v / b.v;
    double qd = (a.d - qv * b.d) / b.v;
    double qc = (a.c - qv * b.c - qd * b.d) / b.v;
    return Jet{qv, qd, qc};
}

// Repulsive part H(rho) per unit temperature (includes R).
Jet repulsive(const EosConst& e, Jet r) {
    if (e.kind == EOS_CS) {
        Jet eta = (e.b / 4.0) * r;
        Jet om = cst(1.0) - eta;
        Jet z = (cst(1.0) + eta + eta * eta - eta * eta * eta) / (om * om * om);
        return e.R * (r * z);
    }
    return e.R * (r / (cst(1.0) - e.b * r));
}

// Attractive part Q(rho) per unit alpha (includes a).
Jet attractive(const EosConst& e, Jet r) {
    switch (e.kind) {
        case EOS_RK:
        case EOS_RKS:
            return e.a * (r * r / (cst(1.0) + e.b * r));
        case EOS_PR:
            return e.a * (r * r / (cst(1.0) + 2.0 * e.b * r - (e.b * e.b) * (r * r)));
        default:
            return e.a * (r * r);
    }
}

// Psi(rho) = integral of p / rho^2 d rho (up to a constant), in closed form.
double psi_integral(const EosConst& e, double rho, double T, double alpha) {
    double rep;
    if (e.kind == EOS_CS) {
        // integral Z(eta)/eta d eta = ln eta + (4 eta - 3 eta^2)/(1 - eta)^2
        double eta = e.b * rho / 4.0;
        rep = std::log(eta) + (4.0 * eta - 3.0 * eta * eta) / ((1.0 - eta) * (1.0 - eta));
    } else {
        rep = std::log(rho) - std::log(1.0 - e.b * rho);  // integral 1/(rho (1 - b rho))
    }
    double att;
    switch (e.kind) {
        case EOS_RK:
        case EOS_RKS:
            att = std::log(1.0 + e.b * rho) / e.b;
            break;
        case EOS_PR: {
            const double s2 = std::sqrt(2.0);
            att = std::log((e.b * rho - 1.0 + s2) / (1.0 + s2 - e.b * rho)) / (2.0 * s2 * e.b);
            break;
        }
        default:
            att = rho;
    }
    return e.R * T * rep - e.a * alpha * att;
}

double chem_potential(const EosConst& e, double rho, double T, double alpha) {
    return psi_integral(e, rho, T, alpha) + eos_pressure(e, rho, T, alpha).v / rho;
}

// Bisection for a root of fn on [lo, hi] given opposite signs at the ends.
template <typename F>
double bisect(F fn, double lo, double hi) {
    double flo = fn(lo);
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        double fm = fn(mid);
        if ((fm > 0.0) == (flo > 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
    }
    return 0.5 * (lo + hi);
}

// First sign change of fn on (0, rmax) over a uniform scan, refined by bisection.
template <typename F>
bool first_root(F fn, double rmax, double* root) {
    const int n = 8192;
    double x0 = rmax * 1e-9, f0 = fn(x0);
    for (int i = 1; i <= n; ++i) {
        double x1 = rmax * (double)i / (n + 1), f1 = fn(x1);
        if ((f0 > 0.0) != (f1 > 0.0)) { *root = bisect(fn, x0, x1); return true; }
        x0 = x1; f0 = f1;
    }
    return false;
}

}  // namespace

double eos_rho_max(const EosConst& e) { return (e.kind == EOS_CS) ? 4.0 / e.b : 1.0 / e.b; }

double eos_psi(const EosConst& e, double rho, double T, double alpha) { return psi_integral(e, rho, T, alpha); }

Jet eos_pressure(const EosConst& e, double rho, double T, double alpha) {
    Jet r{rho, 1.0, 0.0};
    return T * repulsive(e, r) - alpha * attractive(e, r);
}

double eos_alpha(const EosConst& e, double T, double Tc) {
    if (e.kind == EOS_RK) return 1.0 / std::sqrt(T);
    if (e.kind == EOS_PR || e.kind == EOS_RKS) {
        double w = e.omega;
        double m = (e.kind == EOS_PR) ? 0.37464 + w * (1.54226 - 0.26992 * w) : 0.480 + w * (1.574 - 0.176 * w);
        double s = 1.0 + m * (1.0 - std::sqrt(T / Tc));
        return s * s;
    }
    return 1.0;
}

bool eos_critical(const EosConst& e, double* Tc, double* rhoc) {
    if (!(e.a > 0.0) || !(e.b > 0.0) || !(e.R > 0.0)) return false;
    double rmax = eos_rho_max(e);
    auto cond = [&](double rho) {
        Jet r{rho, 1.0, 0.0};
        Jet H = repulsive(e, r), Qa = attractive(e, r);
        return H.d * (2.0 * Qa.c) - (2.0 * H.c) * Qa.d;
    };
    double rc;
    if (!first_root(cond, rmax, &rc)) return false;
    Jet r{rc, 1.0, 0.0};
    double ratio = attractive(e, r).d / repulsive(e, r).d;  // = T / A(T)
    *rhoc = rc;
    *Tc = (e.kind == EOS_RK) ? std::pow(ratio, 2.0 / 3.0) : ratio;
    return std::isfinite(*Tc) && *Tc > 0.0;
}

bool eos_maxwell(const EosConst& e, double T, double* rho_v, double* rho_l, double* p0) {
    double Tc, rc;
    if (!eos_critical(e, &Tc, &rc) || !(T > 0.0) || !(T < Tc)) return false;
    const double al = eos_alpha(e, T, Tc);
    const double rmax = eos_rho_max(e);
    auto P = [&](double r) { return eos_pressure(e, r, T, al).v; };
    auto dP = [&](double r) { return eos_pressure(e, r, T, al).d; };
    auto d2P = [&](double r) { return 2.0 * eos_pressure(e, r, T, al).c; };
    // Inflection of the isotherm (p'' changes sign from - to +), then the two
    // spinodals where p' vanishes on either side of it.
    double ri;
    if (!first_root(d2P, rmax, &ri)) return false;
    if (!(dP(ri) < 0.0)) return false;
    double s1 = bisect(dP, rmax * 1e-12, ri);
    double s2 = bisect(dP, ri, rmax * (1.0 - 1e-14));
    // Pressure bracket: up to the vapour spinodal; down to the liquid spinodal or,
    // when that pressure is negative, to the pressure of a vanishing vapour
    // density (kept inside the vapour-branch bracket below).
    const double rfloor = rmax * 1e-13;
    double phi = P(s1), plo = P(s2);
    if (!(plo > P(rfloor))) plo = P(rfloor);
    auto branches = [&](double pp, double* rv, double* rl) {
        *rv = bisect([&](double r) { return P(r) - pp; }, rfloor * 0.5, s1);
        *rl = bisect([&](double r) { return P(r) - pp; }, s2, rmax * (1.0 - 1e-15));
    };
    auto dmu = [&](double pp) {
        double rv, rl;
        branches(pp, &rv, &rl);
        return chem_potential(e, rl, T, al) - chem_potential(e, rv, T, al);
    };
    double ps = bisect(dmu, plo, phi);
    branches(ps, rho_v, rho_l);
    if (p0) *p0 = ps;
    return *rho_v > 0.0 && *rho_l > *rho_v;
}

}  // namespace lbm_host

// Host-side equation-of-state utilities of the library: pressure with its
// density derivatives, the critical point and the Maxwell coexistence densities.
// Sec. 5.1 Eq. 24 (VDW), Sec. 5.2 Eqs. 27-29 (RK / RKS, PR, CS), Hu's scaling
// p_m = k p_EOS (Sec. 5).  Used to plan a domain (alpha(T_r) needs Tc) and by
// callers that set up coexisting phases.
#pragma once

namespace lbm_host {

enum EosKind { EOS_VDW = 0, EOS_PR = 1, EOS_CS = 2, EOS_RK = 3, EOS_RKS = 4 };

struct EosConst {
    int kind;
    double a, b, R, omega;
};

// Second-order Taylor jet f(x0 + e) = v + d e + c e^2 (c = f''/2): enough for
// p, dp/drho and d2p/drho2 by ordinary arithmetic.
struct Jet {
    double v, d, c;
};

// p(rho, T) as a jet in rho with the attraction multiplied by alpha.
Jet eos_pressure(const EosConst& e, double rho, double T, double alpha);

// alpha(T) of the attraction term: 1 (VDW, CS), T^-1/2 (RK), Soave / PR forms
// with T_r = T / Tc (RKS, PR).
double eos_alpha(const EosConst& e, double T, double Tc);

// Critical point (Tc, rho_c); returns false if none is found.
bool eos_critical(const EosConst& e, double* Tc, double* rhoc);

// Maxwell coexistence at T (< Tc): equal p and equal chemical potential.
bool eos_maxwell(const EosConst& e, double T, double* rho_v, double* rho_l, double* p0);

// Largest admissible density (pole of the repulsive term).
double eos_rho_max(const EosConst& e);

// Psi(rho) = integral of p / rho^2 d rho (closed form, up to a constant).
double eos_psi(const EosConst& e, double rho, double T, double alpha);

}  // namespace lbm_host

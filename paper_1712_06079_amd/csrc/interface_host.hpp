// Host-side flat-interface utilities (Sec. 5.1 Eqs. 25-26, Sec. 5.3): the
// "exact" equilibrium profile of the square-gradient fluid with the k-scaled
// EOS and the integration-method surface tension of a simulated slab.
#pragma once

#include "eos_host.hpp"

namespace lbm_host {

struct FlatInterface {
    EosConst e;
    double T, alpha, k;    // temperature, alpha(T), Hu's scaling
    double rv, rl, p0;     // Maxwell densities and (unscaled) pressure
};

// Coexistence data at T (< Tc); false without a liquid-vapour coexistence.
bool flat_interface(const EosConst& e, double T, double k, FlatInterface* f);

// W(rho) = rho * integral_{rho_b}^{rho} (p_m(s) - k p0) / s^2 ds (p_m = k p),
// from the nearer bulk density rho_b: (kappa/2) rho'^2 in the interface.
double interface_excess(const FlatInterface& f, double rho);

// Profile rising through the mean density at y = 0: rho and rho' at
// y_i = (i - (n - 1)/2) h.
void flat_profile(const FlatInterface& f, double kappa, double h, int n, double* rho, double* drho);

// kappa/2 sum (D rho)^2 over a periodic column of n sites (two interfaces),
// D the Eq. 20 row on n points; drho (nullable) receives D rho.
double sigma_slab(double kappa, int n, const double* rho, double* drho);

}  // namespace lbm_host

// Flat-interface utilities (see interface_host.hpp).
//
// With the tensor of Eq. 25 the normal component P_yy = p_m - kappa rho rho''
// + (kappa/2) rho'^2 is uniform across a flat interface (Eq. 26) and equals
// the coexistence pressure.  Its first integral (kappa/2) rho'^2 = W(rho) uses
// the closed-form Psi = integral p / rho^2 of the EOS module:
//   W(rho) = k [rho (Psi(rho) - Psi(rho_b)) + p0 (1 - rho / rho_b)].
// The profile follows rho' = sqrt(2 W / kappa) by fourth-order Runge-Kutta
// steps of h/64 from the mean density outwards.
#include "interface_host.hpp"

#include <cmath>
#include <vector>

#include "hdm_coeffs.hpp"

namespace lbm_host {

bool flat_interface(const EosConst& e, double T, double k, FlatInterface* f) {
    double Tc = 0.0, rc = 0.0;
    if (!(k > 0.0) || !eos_critical(e, &Tc, &rc) || !(T > 0.0) || !(T < Tc)) return false;
    f->e = e;
    f->T = T;
    f->k = k;
    f->alpha = eos_alpha(e, T, Tc);
    return eos_maxwell(e, T, &f->rv, &f->rl, &f->p0);
}

double interface_excess(const FlatInterface& f, double rho) {
    const double rb = (rho > 0.5 * (f.rv + f.rl)) ? f.rl : f.rv;
    const double W = f.k * (rho * (eos_psi(f.e, rho, f.T, f.alpha) - eos_psi(f.e, rb, f.T, f.alpha)) +
                            f.p0 * (1.0 - rho / rb));
    return W > 0.0 ? W : 0.0;
}

void flat_profile(const FlatInterface& f, double kappa, double h, int n, double* rho, double* drho) {
    auto slope = [&](double r) { return std::sqrt(2.0 * interface_excess(f, r) / kappa); };
    const double c = 0.5 * (n - 1);
    const int first_up = (int)std::ceil(c);
    // upper side (y >= 0, nearest point first), then the lower side
    for (int side = 0; side < 2; ++side) {
        double y = 0.0, r = 0.5 * (f.rv + f.rl);
        const int step = side == 0 ? 1 : -1;
        for (int i = side == 0 ? first_up : first_up - 1; i >= 0 && i < n; i += step) {
            const double target = (i - c) * h;
            const int m = (int)std::ceil(std::fabs(target - y) * 64.0 / h);
            const double dy = m > 0 ? (target - y) / m : 0.0;
            for (int s = 0; s < m; ++s) {
                const double a = slope(r), b = slope(r + 0.5 * dy * a), cc = slope(r + 0.5 * dy * b),
                             d = slope(r + dy * cc);
                r += dy / 6.0 * (a + 2.0 * (b + cc) + d);
            }
            y = target;
            rho[i] = r;
            drho[i] = slope(r);
        }
    }
}

double sigma_slab(double kappa, int n, const double* rho, double* drho) {
    const int taps = hdm_taps(n, 39);
    double d[40] = {0.0};
    hdm_row(n, taps, d);
    double sum = 0.0;
    for (int i = 0; i < n; ++i) {
        double g = 0.0;
        for (int j = 1; j <= taps; ++j) g += d[j - 1] * (rho[(i + j) % n] - rho[((i - j) % n + n) % n]);
        if (drho) drho[i] = g;
        sum += g * g;
    }
    return 0.5 * kappa * sum;
}

}  // namespace lbm_host

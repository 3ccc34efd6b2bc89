// Explicit form of the periodic compact high-order difference (Sec. 3.2 Eq. 20).
//
// With h = 1, Eq. 20 on a periodic line of N points reads A u' = B u with
//   A = I + (E + E^-1)/3,   B = (7/9)(E - E^-1) + (1/36)(E^2 - E^-2),  (E u)_i = u_{i+1}.
// Both operators are circulant, so u' = D u with the circulant D = A^-1 B:
//   (D u)_i = sum_j d_j u_{i+j},  d_{-j} = -d_j,  d_0 = 0.
// A has the symbol 1 + (2/3) cos(theta) = (1 - r z)(1 - r / z) / (1 + r^2),
// r = (sqrt 5 - 3)/2, whose Fourier inverse on the infinite line is
// (3/sqrt 5) r^|n|; summing the periodic images gives the inverse on N points
//   g_n = (3/sqrt 5) (r^n + r^(N-n)) / (1 - r^N),  0 <= n < N,
// and d_j = sum_m g_{(j - m) mod N} b_m with b_{+-1} = +-7/9, b_{+-2} = +-1/36.
// |d_j| decays like |r|^j (|r| = 0.382), so the stencil may be cut at the
// radius where the tail drops below the working precision: 39 in FP64
// (tail 5e-17 of d_1), 28 with FP32 populations (4e-12).  For N <= 2J + 1 the whole
// periodic row is used and the result is the exact periodic solve.
#include "hdm_coeffs.hpp"

#include <cmath>

namespace lbm_host {

int hdm_taps(int n, int radius) {
    int half = (n - 1) / 2;  // for even n the j = n/2 tap is its own negative: zero
    return half < radius ? half : radius;
}

void hdm_row(int n, int taps, double* d) {
    typedef long double LD;
    const LD s5 = std::sqrt((LD)5.0);
    const LD r = (s5 - (LD)3.0) / (LD)2.0;
    const LD c = (LD)3.0 / s5;
    LD rN = std::pow(r, (LD)n);
    auto g = [&](int m) {  // periodic inverse of A, index taken mod n
        m %= n;
        if (m < 0) m += n;
        return c * (std::pow(r, (LD)m) + std::pow(r, (LD)(n - m))) / ((LD)1.0 - rN);
    };
    const int bo[4] = {1, -1, 2, -2};
    const LD bv[4] = {(LD)7.0 / (LD)9.0, -(LD)7.0 / (LD)9.0, (LD)1.0 / (LD)36.0, -(LD)1.0 / (LD)36.0};
    for (int j = 1; j <= taps; ++j) {
        LD s = 0.0L;
        for (int k = 0; k < 4; ++k) s += g(j - bo[k]) * bv[k];
        d[j - 1] = (double)s;
    }
}

// Infinite-line row: with g_n = (3/sqrt 5) r^|n|, d_j = sum_m g_{j-m} b_m.  For
// j >= 3 every offset j - m is positive, so d_j = C r^j with
// C = (3/sqrt 5) [(7/9)(1/r - r) + (1/36)(1/r^2 - r^2)]; d_1 and d_2 keep the
// terms where |j - m| folds.
void hdm_infinite(double* r_out, double* d1, double* d2, double* C) {
    typedef long double LD;
    const LD s5 = std::sqrt((LD)5.0);
    const LD r = (s5 - (LD)3.0) / (LD)2.0;
    const LD c = (LD)3.0 / s5;
    const LD b1 = (LD)7.0 / (LD)9.0, b2 = (LD)1.0 / (LD)36.0;
    auto g = [&](int n) { return c * std::pow(r, (LD)(n < 0 ? -n : n)); };
    auto d = [&](int j) { return b1 * (g(j - 1) - g(j + 1)) + b2 * (g(j - 2) - g(j + 2)); };
    *r_out = (double)r;
    *d1 = (double)d(1);
    *d2 = (double)d(2);
    *C = (double)(c * (b1 * ((LD)1.0 / r - r) + b2 * ((LD)1.0 / (r * r) - r * r)));
}

// Central difference, Eq. 14 (h = 1): d_1 = 1/2.
void cdm_row(int taps, double* d) {
    for (int j = 1; j <= taps; ++j) d[j - 1] = (j == 1) ? 0.5 : 0.0;
}

}  // namespace lbm_host

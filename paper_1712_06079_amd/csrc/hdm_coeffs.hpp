// Explicit circulant form of the periodic compact difference of Sec. 3.2 Eq. 20.
#pragma once

namespace lbm_host {

// Number of one-sided taps kept on a periodic line of n points for a stencil
// radius limit `radius`: min(radius, (n - 1) / 2).
int hdm_taps(int n, int radius);

// d[0..taps-1] = d_1 .. d_taps of the circulant D = A^-1 B on n points.
void hdm_row(int n, int taps, double* d);

// Infinite-line row in geometric form: d_j = C r^j for j >= 3, with r, d_1, d_2.
void hdm_infinite(double* r, double* d1, double* d2, double* C);

// The central difference of Eq. 14 in the same one-sided form (d_1 = 1/2).
void cdm_row(int taps, double* d);

}  // namespace lbm_host

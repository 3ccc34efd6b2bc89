// Device building blocks of the HDM pseudopotential lattice Boltzmann step on
// gfx950: population layout, EOS potential, equilibrium, collision.
//
// Storage and arithmetic: populations are stored as `Real` (double or float),
// the potential field as PhiStore<Real, FORCE>::type, and every arithmetic
// step is carried out in double (values are widened on load and rounded once
// on store).  On MI355X the FP64 vector rate equals the unpacked FP32 rate and
// the step is bound by HBM bytes, so FP32 storage cuts the traffic without
// FP32 arithmetic error.  With FP32 populations the Shan-Chen and Zhang-Chen
// potential fields are stored in FP32 too (their rounding moves the densities
// of the 2000-step 64^2 slab by about 1e-6, against the 1e-5 bar); the hybrid
// force keeps an FP64 field (there the FP32 rounding of both fields it
// differentiates moved a Peng-Robinson case by 1e-5 in 60 steps).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 9;
constexpr int BX = 64;     // cells per x-block of the population layout (one wavefront)
constexpr int JCAP = 40;   // capacity of the one-sided coefficient tables
constexpr int KT = 4;      // largest number of outputs per thread of the blocked stencil
constexpr int TAB_OFF = JCAP + KT - 1;   // table index of tap offset 0
constexpr int TAB = 2 * TAB_OFF + 1;

// Stencil radius kept per population precision.  FP64: the tail of the
// circulant row of Eq. 20 beyond 39 taps is 5e-17 of d_1, below rounding.
// FP32 populations: 28 taps (tail 4e-12).  A tail at the FP32 unit roundoff
// (18 taps, 3e-8) is not enough: over 2000 steps of the 64^2 slab it moves the
// densities by 6e-5, while 28 taps move them by 1e-9, far below the 1e-6 the
// FP32 population rounding itself causes.
template <typename Real> struct Radius;
template <> struct Radius<double> { static constexpr int value = 39; };
template <> struct Radius<float> { static constexpr int value = 28; };

enum { FORCE_SC = 0, FORCE_ZC = 1, FORCE_HYBRID = 2 };
enum { EOS_VDW = 0, EOS_PR = 1, EOS_CS = 2, EOS_RK = 3, EOS_RKS = 4 };

// D2Q9 velocity set (order 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1)
// 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)) and weights 4/9, 1/9, 1/36.
__host__ __device__ constexpr int ex(int i) { return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0; }
__host__ __device__ constexpr int ey(int i) { return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0; }
template <typename Real>
__host__ __device__ constexpr Real wq(int i) {
    return i == 0 ? Real(4.0 / 9.0) : (i < 5 ? Real(1.0 / 9.0) : Real(1.0 / 36.0));
}

// Population layout ("AoSoA"): f[y][x / 64][q][x % 64].  A wavefront's 64
// consecutive cells of one population are one contiguous 512 B (FP64) or
// 256 B (FP32) segment, and a block's nine populations are adjacent.
__host__ __device__ inline size_t fidx(int x, int y, int q, int nxb) {
    return ((size_t)(y * nxb + (x >> 6)) * Q + q) * BX + (x & 63);
}

// EOS potential U = g (k p_EOS(rho, T) - rho / 3) with the constants folded on
// the host: c_rep = g k R T, c_att = g k a alpha(T), c_lin = g / 3.
struct DevEos {
    int kind;
    double c_rep, c_att, c_lin, b;
};

__device__ inline double potential(const DevEos& e, double rho) {
    double rep, att;
    if (e.kind == EOS_CS) {  // Eq. 29, Carnahan-Starling repulsion
        double eta = e.b * rho * 0.25;
        double om = 1.0 - eta;
        rep = rho * (1.0 + eta * (1.0 + eta * (1.0 - eta))) / (om * om * om);
        att = rho * rho;
    } else {  // Eqs. 24, 27, 28
        rep = rho / (1.0 - e.b * rho);
        if (e.kind == EOS_PR)
            att = rho * rho / (1.0 + e.b * rho * (2.0 - e.b * rho));
        else if (e.kind == EOS_RK || e.kind == EOS_RKS)
            att = rho * rho / (1.0 + e.b * rho);
        else
            att = rho * rho;
    }
    return e.c_rep * rep - e.c_att * att - e.c_lin * rho;
}

// The stored potential field: signed Phi = s sqrt|U| (Eq. 21) for the
// Shan-Chen and hybrid forces, U itself for Zhang-Chen.
template <int FORCE>
__device__ inline double phi_of(double U) {
    if (FORCE == FORCE_ZC) return U;
    double m = sqrt(fabs(U));
    return U < 0.0 ? -m : m;
}

// Equilibrium, Eq. 2: w_i rho [1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u^2].
__device__ inline double feq(int i, double rho, double ux, double uy, double usq) {
    double eu = double(ex(i)) * ux + double(ey(i)) * uy;
    return wq<double>(i) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
}

// BGK collision with Kupershtokh's exact-difference forcing (Eqs. 1, 10):
//   f*_i = f_i - (f_i - f^eq_i(u)) / tau + f^eq_i(u + F/rho) - f^eq_i(u)
//        = k f_i + [f^eq_i(v) - k f^eq_i(u)],   k = 1 - 1/tau,
// with u = j / rho and v = J / rho, J = j + F.  Expanding Eq. 2, the bracket
// is w_i [B + e_i . m + e_ix^2 Txx + e_iy^2 Tyy + e_ix e_iy Txy] with
//   B   = rho / tau - 1.5 (|J|^2 - k |j|^2) / rho,     m = 3 (J - k j),
//   Txx = 4.5 (Jx^2 - k jx^2) / rho,   Tyy = 4.5 (Jy^2 - k jy^2) / rho,
//   Txy = 9 (Jx Jy - k jx jy) / rho,
// so the nine directions share the second-order terms (the same value as the
// two equilibria written out, up to rounding order).  Every fused multiply-add
// is explicit and the compiler may form no others, so every inlined copy of
// the collision rounds alike (cells that start equal stay bitwise equal
// whichever kernel path collides them).
__device__ inline void collide(double (&f)[Q], double rho, double jx, double jy, double Fx, double Fy, double omega) {
#pragma clang fp contract(off)
    const double keep = 1.0 - omega;
    const double ir = 1.0 / rho;
    const double Jx = jx + Fx, Jy = jy + Fy;
    const double kx = keep * jx, ky = keep * jy;
    const double Sxx = fma(-kx, jx, Jx * Jx), Syy = fma(-ky, jy, Jy * Jy), Sxy = fma(-kx, jy, Jx * Jy);
    const double h = 4.5 * ir, h2 = 9.0 * ir;
    const double B = fma(-1.5 * ir, Sxx + Syy, rho * omega);
    const double ax = fma(h, Sxx, B), ay = fma(h, Syy, B);   // axis directions: B + Txx, B + Tyy
    const double dd = fma(h, Syy, ax);                       // diagonals: B + Txx + Tyy
    const double dp = fma(h2, Sxy, dd), dm = fma(-h2, Sxy, dd);   // e_x e_y = +1, -1
    const double mx = 3.0 * (Jx - kx), my = 3.0 * (Jy - ky);
    const double sp = mx + my, sm = mx - my;
    const double w0 = wq<double>(0), w1 = wq<double>(1), w2 = wq<double>(5);
    f[0] = fma(keep, f[0], w0 * B);
    f[1] = fma(keep, f[1], w1 * (ax + mx));
    f[3] = fma(keep, f[3], w1 * (ax - mx));
    f[2] = fma(keep, f[2], w1 * (ay + my));
    f[4] = fma(keep, f[4], w1 * (ay - my));
    f[5] = fma(keep, f[5], w2 * (dp + sp));   // (1, 1)
    f[7] = fma(keep, f[7], w2 * (dp - sp));   // (-1, -1)
    f[8] = fma(keep, f[8], w2 * (dm + sm));   // (1, -1)
    f[6] = fma(keep, f[6], w2 * (dm - sm));   // (-1, 1)
}

__device__ inline void moments(const double (&f)[Q], double& rho, double& jx, double& jy) {
    rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    jx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
    jy = (f[2] - f[4]) + ((f[5] - f[8]) + (f[6] - f[7]));
}

// v mod n for the offsets the kernels wrap (a tile origin plus a stencil
// radius and a ring cell): they lie within a few periods of [0, n), so
// conditional corrections replace an integer division (which has no hardware
// instruction).  Large lattices need at most one correction.
__device__ inline int wrap(int v, int n) {
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

// v mod n for |v| < 2^23 and 0 < n <= 2^22 (lattice sides are at most 2^21),
// without a loop or a branch: v converts to FP32 exactly, the quotient estimate
// floor(v / n) from the FP32 reciprocal is exact or off by one (relative error
// of rcp and product below 2^-21 on a quotient below 2^22 in size), and one
// correction each way brings the remainder into [0, n).  Kernels that wrap many
// staged indices per tile use it instead of wrap(), whose correction loops
// compile to divergent branches.
__device__ inline int wrap_fast(int v, int n) {
    const float rn = __builtin_amdgcn_rcpf((float)n);
    const int q = (int)floorf((float)v * rn);
    int r = v - __mul24(q, n);
    r += r < 0 ? n : 0;
    r -= r >= n ? n : 0;
    return r;
}

// Coefficient tables of a domain's Eq. 20 stencil, in device memory (a small
// region of the domain workspace); kernels read them with uniform (scalar)
// loads.  Keeping them out of the kernel arguments keeps launches cheap.
struct StepTables {
    double dx[JCAP];  // d_1 .. d_tx along x
    double dy[JCAP];  // d_1 .. d_ty along y
    // Sign-folded tables for the blocked stencil: tab[i] = c(i - TAB_OFF),
    // c(n) = sign(n) d_|n| for 1 <= |n| <= taps, else 0.
    double tx_tab[TAB];
    double ty_tab[TAB];
};

// Storage type of the potential field (see the note at the top).
template <typename Real, int FORCE>
struct PhiStore { using type = double; };
template <>
struct PhiStore<float, FORCE_SC> { using type = float; };
template <>
struct PhiStore<float, FORCE_ZC> { using type = float; };

// Kernel arguments of one domain step (passed by value).  The potential
// planes are untyped here; kernels view them as PhiStore<Real, FORCE>::type.
template <typename Real>
struct StepArgs {
    const Real* __restrict__ f_in;
    Real* __restrict__ f_out;
    const void* __restrict__ phi_in;
    void* __restrict__ phi_out;
    int nx, ny, nxb;  // lattice size, number of 64-cell x blocks
    int tx, ty;       // one-sided taps used along x and along y
    double omega;     // 1 / tau
    double A;         // hybrid weight (Eq. 9)
    DevEos eos;
    const StepTables* __restrict__ tab;  // the domain's coefficient tables (device)
    // Geometric form of the infinite-line row (d_j = C r^j for j >= 3), used
    // along an axis whose length exceeds 2R + 1 (there the periodic row equals
    // it to rounding): rec_x / rec_y select it per axis; rK = C / (1 - r).
    int rec_x, rec_y;
    double rr, rr3, rr4, rd1, rd2, rK;
    // 1: the gradient is the weighted D2Q9 difference of Eq. 15 (with the
    // 1/c_s^2 factor) instead of a per-axis stencil.
    int grad9;
    // 1: no-slip walls at y = -1/2 and ny - 1/2 (rows continue past a wall
    // by reflection; populations crossing it bounce back).
    int walls;
};

// Lattice row of row index y (any integer): periodic, or between walls at
// -1/2 and n - 1/2, where the rows continue by reflection (period 2n).
__device__ inline int ymap(int y, int n, int walls) {
    if (!walls) return wrap(y, n);
    const int t = wrap(y, 2 * n);
    return t < n ? t : 2 * n - 1 - t;
}

// ymap through wrap_fast (the same result for |y| < 2^22, n <= 2^21).
__device__ inline int ymap_fast(int y, int n, int walls) {
    const int per = walls ? 2 * n : n;
    const int t = wrap_fast(y, per);
    return t >= n ? per - 1 - t : t;
}

// Opposite D2Q9 direction (order 0, +x, +y, -x, -y, ++, -+, --, +-).
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i < 5 ? 1 + (i + 1) % 4 : 5 + (i - 3) % 4); }

// Eq. 15 with the factor 1/c_s^2 = 3 at the centre of a 3 x 3 neighbourhood
// (m: row y-1, c: row y, p: row y+1; index 0, 1, 2 = x-1, x, x+1):
//   d/dx = (1/3)(c2 - c0) + (1/12)[(p2 - p0) + (m2 - m0)],
//   d/dy = (1/3)(p1 - m1) + (1/12)[(p2 - m2) + (p0 - m0)].
__device__ inline void grad_d2q9(const double* m, const double* c, const double* p, double& gx, double& gy) {
    const double a = 1.0 / 3.0, d = 1.0 / 12.0;
    gx = a * (c[2] - c[0]) + d * ((p[2] - p[0]) + (m[2] - m[0]));
    gy = a * (p[1] - m[1]) + d * ((p[2] - m[2]) + (p[0] - m[0]));
}

}  // namespace lbm

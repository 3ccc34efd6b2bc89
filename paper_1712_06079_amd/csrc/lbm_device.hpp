// Device building blocks of the HDM pseudopotential lattice Boltzmann step on
// gfx950: population layout, EOS potential, equilibrium, collision.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 9;
constexpr int BX = 64;     // cells per x-block of the population layout (one wavefront)
constexpr int JCAP = 40;   // capacity of the one-sided coefficient tables

// Stencil radius kept per precision: the tail of the circulant row of Eq. 20
// beyond it is below the unit roundoff (5e-17 in FP64, 3e-8 in FP32).
template <typename Real> struct Radius;
template <> struct Radius<double> { static constexpr int value = 39; };
template <> struct Radius<float> { static constexpr int value = 18; };

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
template <typename Real>
struct DevEos {
    int kind;
    Real c_rep, c_att, c_lin, b;
};

template <typename Real>
__device__ inline Real potential(const DevEos<Real>& e, Real rho) {
    Real rep, att;
    if (e.kind == EOS_CS) {  // Eq. 29, Carnahan-Starling repulsion
        Real eta = e.b * rho * Real(0.25);
        Real om = Real(1) - eta;
        rep = rho * (Real(1) + eta * (Real(1) + eta * (Real(1) - eta))) / (om * om * om);
        att = rho * rho;
    } else {  // Eqs. 24, 27, 28
        rep = rho / (Real(1) - e.b * rho);
        if (e.kind == EOS_PR)
            att = rho * rho / (Real(1) + e.b * rho * (Real(2) - e.b * rho));
        else if (e.kind == EOS_RK || e.kind == EOS_RKS)
            att = rho * rho / (Real(1) + e.b * rho);
        else
            att = rho * rho;
    }
    return e.c_rep * rep - e.c_att * att - e.c_lin * rho;
}

// The stored potential field: signed Phi = s sqrt|U| (Eq. 21) for the
// Shan-Chen and hybrid forces, U itself for Zhang-Chen.
template <typename Real, int FORCE>
__device__ inline Real phi_of(Real U) {
    if (FORCE == FORCE_ZC) return U;
    Real m = sqrt(fabs(U));
    return U < Real(0) ? -m : m;
}

// Equilibrium, Eq. 2: w_i rho [1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u^2].
template <typename Real>
__device__ inline Real feq(int i, Real rho, Real ux, Real uy, Real usq) {
    Real eu = Real(ex(i)) * ux + Real(ey(i)) * uy;
    return wq<Real>(i) * rho * (Real(1) + Real(3) * eu + Real(4.5) * eu * eu - Real(1.5) * usq);
}

// BGK collision with Kupershtokh's exact-difference forcing (Eqs. 1, 10):
//   f*_i = f_i - (f_i - f^eq_i(u)) / tau + f^eq_i(u + F/rho) - f^eq_i(u)
//        = (1 - 1/tau) (f_i - f^eq_i(u)) + f^eq_i(u + F/rho),   u = j / rho.
template <typename Real>
__device__ inline void collide(Real (&f)[Q], Real rho, Real jx, Real jy, Real Fx, Real Fy, Real omega) {
    Real ir = Real(1) / rho;
    Real ux = jx * ir, uy = jy * ir;
    Real vx = ux + Fx * ir, vy = uy + Fy * ir;
    Real usq = ux * ux + uy * uy, vsq = vx * vx + vy * vy;
    Real keep = Real(1) - omega;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        Real e0 = feq(i, rho, ux, uy, usq);
        Real e1 = feq(i, rho, vx, vy, vsq);
        f[i] = keep * (f[i] - e0) + e1;
    }
}

template <typename Real>
__device__ inline void moments(const Real (&f)[Q], Real& rho, Real& jx, Real& jy) {
    rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    jx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
    jy = (f[2] - f[4]) + ((f[5] - f[8]) + (f[6] - f[7]));
}

__device__ inline int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Kernel arguments of one domain step (passed by value; the coefficient
// tables travel in the kernel-argument segment and are read as scalars).
template <typename Real>
struct StepArgs {
    const Real* __restrict__ f_in;
    Real* __restrict__ f_out;
    const Real* __restrict__ phi_in;
    Real* __restrict__ phi_out;
    int nx, ny, nxb;  // lattice size, number of 64-cell x blocks
    int tx, ty;       // one-sided taps used along x and along y
    Real omega;       // 1 / tau
    Real A;           // hybrid weight (Eq. 9)
    DevEos<Real> eos;
    Real dx[JCAP];    // d_1 .. d_tx along x
    Real dy[JCAP];    // d_1 .. d_ty along y
};

}  // namespace lbm

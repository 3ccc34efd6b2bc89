// Single-pass fused time step (one launch per step).
//
// A workgroup owns a TX x TY tile of the lattice and computes
//   f_{t+1} on the tile and phi_{t+1} (the potential field of that new state)
// from f_t and phi_t, so each step reads f once, writes f once, reads phi once
// (its halo comes from the caches) and writes phi once: 2 Q + 2 words per cell.
//
// Phases (all cell coordinates wrap periodically, so ragged tiles need no
// special case; interior cells outside the lattice are simply not written):
//  0  each thread issues the loads of f_t for its cells of the collision region
//     (the tile plus a one-cell ring, whose post-collision populations stream
//     into the tile) so they are in flight during phases 1-2;
//  1  stage phi_t in LDS over a cross: the collision rows widened by +-J in x
//     and the collision columns widened by +-J in y;
//  2  the explicit form of Eq. 20 (radius J, coefficients d_j) along x and
//     along y, K outputs per thread from one sliding window (each LDS value
//     feeds up to K outputs), then the force (Eq. 22 / Eq. 7 / Eq. 9) into LDS;
//  3  EDM-BGK collision of every collision cell into LDS (reusing the phi area);
//  4  pull streaming f_{t+1,i}(x) = f*_i(x - e_i) from LDS, aligned stores of
//     f_{t+1}, then rho_{t+1} -> U -> phi_{t+1} stored (Eqs. 3, 8, 21).
#pragma once

#include "lbm_kernels.hpp"

namespace lbm {

template <typename Real, int TX, int TY, int K>
struct FusedShape {
    static constexpr int J = Radius<Real>::value;
    static constexpr int CW = TX + 2, CH = TY + 2;           // collision region
    static constexpr int NCELL = CW * CH;
    static constexpr int NSX = (CW + K - 1) / K;              // x segments per collision row
    static constexpr int NSY = (CH + K - 1) / K;              // y segments per collision column
    static constexpr int RW = (NSX * K + 2 * J) | 1;          // row-bar pitch (odd: spreads LDS banks)
    static constexpr int VH = NSY * K + 2 * J;                // column-bar height
    static constexpr int PHI_WORDS = CH * RW + VH * CW;
    static constexpr int FS_WORDS = Q * NCELL;
    static constexpr int A_WORDS = PHI_WORDS > FS_WORDS ? PHI_WORDS : FS_WORDS;
    static constexpr int WORDS = A_WORDS + 2 * NCELL;         // + Fx, Fy
    static constexpr int NC = (NCELL + NT - 1) / NT;          // collision cells per thread
    static constexpr int NI = (TX * TY + NT - 1) / NT;        // interior cells per thread
    static constexpr int ITEMS_X = CH * NSX, ITEMS_Y = CW * NSY;
};

template <typename Real, int FORCE, int K>
__device__ inline void stencil_window(const Real* __restrict__ base, int stride, const StepArgs<Real>& a, const Real* d,
                                      Real (&acc)[K], Real (&accu)[K]) {
    constexpr int J = Radius<Real>::value;
#pragma unroll
    for (int k = 0; k < K; ++k) { acc[k] = Real(0); accu[k] = Real(0); }
#pragma unroll
    for (int m = 0; m < 2 * J + K; ++m) {
        const Real v = base[m * stride];
        const Real vo = (FORCE == FORCE_ZC) ? v : fabs(v);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int n = m - k - J;  // tap offset of this value from output k
            if (n != 0 && n >= -J && n <= J) {
                const Real c = n > 0 ? d[n - 1] : -d[-n - 1];
                acc[k] += c * vo;
                if (FORCE == FORCE_HYBRID) accu[k] += c * (v * fabs(v));
            }
        }
    }
}

template <typename Real, int FORCE>
__device__ inline void force_from(Real phic, Real g, Real gu, Real A, Real& F) {
    if (FORCE == FORCE_ZC) {
        F = -g;
    } else {
        F = Real(-2) * phic * g;
        if (FORCE == FORCE_HYBRID) F = A * (-gu) + (Real(1) - Real(2) * A) * F;
    }
}

template <typename Real, int FORCE, int TX, int TY, int K>
__global__ void __launch_bounds__(NT) k_fused(StepArgs<Real> a) {
    using S = FusedShape<Real, TX, TY, K>;
    constexpr int J = S::J, CW = S::CW, CH = S::CH;
    __shared__ Real sm[S::WORDS];
    Real* rowr = sm;                   // [CH][RW]   phi rows  x0-1-J .. x0+TX+J (+ segment padding)
    Real* colr = sm + CH * S::RW;      // [VH][CW]   phi cols  y0-1-J .. y0+TY+J (+ segment padding)
    Real* fst = sm;                    // [Q][CH][CW] post-collision populations (after phase 2)
    Real* Fx = sm + S::A_WORDS;        // [CH][CW]
    Real* Fy = Fx + S::NCELL;

    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int nx = a.nx, ny = a.ny, nxb = a.nxb, pitch = nxb * BX;

    // Phase 0: loads of f_t for this thread's collision cells.
    Real f[S::NC][Q];
#pragma unroll
    for (int i = 0; i < S::NC; ++i) {
        const int c = tid + i * NT;
        if (c < S::NCELL) {
            const int cy = c / CW, cx = c - cy * CW;
            const int xw = wrap(x0 - 1 + cx, nx), yw = wrap(y0 - 1 + cy, ny);
#pragma unroll
            for (int q = 0; q < Q; ++q) f[i][q] = a.f_in[fidx(xw, yw, q, nxb)];
        }
    }

    // Phase 1: phi cross.
    for (int i = tid; i < CH * S::RW; i += NT) {
        const int r = i / S::RW, c = i - r * S::RW;
        const int yw = wrap(y0 - 1 + r, ny), xw = wrap(x0 - 1 - J + c, nx);
        rowr[i] = a.phi_in[(long)yw * pitch + xw];
    }
    for (int i = tid; i < S::VH * CW; i += NT) {
        const int r = i / CW, c = i - r * CW;
        const int yw = wrap(y0 - 1 - J + r, ny), xw = wrap(x0 - 1 + c, nx);
        colr[i] = a.phi_in[(long)yw * pitch + xw];
    }
    __syncthreads();

    // Phase 2: gradients and force.
    for (int it = tid; it < S::ITEMS_X + S::ITEMS_Y; it += NT) {
        Real acc[K], accu[K];
        if (it < S::ITEMS_X) {
            const int cy = it % CH, s = it / CH;  // consecutive lanes: consecutive rows
            const Real* base = rowr + cy * S::RW + s * K;
            stencil_window<Real, FORCE, K>(base, 1, a, a.dx, acc, accu);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int cx = s * K + k;
                if (cx < CW) {
                    Real F;
                    force_from<Real, FORCE>(rowr[cy * S::RW + cx + J], acc[k], accu[k], a.A, F);
                    Fx[cy * CW + cx] = F;
                }
            }
        } else {
            const int jt = it - S::ITEMS_X;
            const int cx = jt % CW, s = jt / CW;  // consecutive lanes: consecutive columns
            const Real* base = colr + (s * K) * CW + cx;
            stencil_window<Real, FORCE, K>(base, CW, a, a.dy, acc, accu);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int cy = s * K + k;
                if (cy < CH) {
                    Real F;
                    force_from<Real, FORCE>(colr[(cy + J) * CW + cx], acc[k], accu[k], a.A, F);
                    Fy[cy * CW + cx] = F;
                }
            }
        }
    }
    __syncthreads();

    // Phase 3: collision of the tile and its ring into LDS.
#pragma unroll
    for (int i = 0; i < S::NC; ++i) {
        const int c = tid + i * NT;
        if (c < S::NCELL) {
            Real rho, jx, jy;
            moments(f[i], rho, jx, jy);
            collide(f[i], rho, jx, jy, Fx[c], Fy[c], a.omega);
#pragma unroll
            for (int q = 0; q < Q; ++q) fst[q * S::NCELL + c] = f[i][q];
        }
    }
    __syncthreads();

    // Phase 4: pull streaming, aligned stores, epilogue phi_{t+1}.
#pragma unroll
    for (int i = 0; i < S::NI; ++i) {
        const int c = tid + i * NT;
        if (c < TX * TY) {
            const int ly = c / TX, lx = c - ly * TX;
            const int x = x0 + lx, y = y0 + ly;
            if (x < nx && y < ny) {
                Real g[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    g[q] = fst[q * S::NCELL + (ly + 1 - ey(q)) * CW + (lx + 1 - ex(q))];
                    a.f_out[fidx(x, y, q, nxb)] = g[q];
                }
                Real rho, jx, jy;
                moments(g, rho, jx, jy);
                a.phi_out[(long)y * pitch + x] = phi_of<Real, FORCE>(potential(a.eos, rho));
            }
        }
    }
}

template <typename Real, int FORCE, int TX, int TY, int K>
inline void launch_fused_t(const StepArgs<Real>& a, hipStream_t s) {
    dim3 grid((a.nx + TX - 1) / TX, (a.ny + TY - 1) / TY);
    hipLaunchKernelGGL((k_fused<Real, FORCE, TX, TY, K>), grid, dim3(NT), 0, s, a);
}

// Tile choice: FP64 uses 64 x 8 tiles (two workgroups per CU fit in LDS),
// FP32 64 x 16; tile_y selects another instantiation (0 = default).
template <typename Real, int FORCE>
inline bool launch_fused(const StepArgs<Real>& a, int tile_y, hipStream_t s) {
    const int ty = tile_y ? tile_y : (sizeof(Real) == 8 ? 8 : 16);
    switch (ty) {
        case 4: launch_fused_t<Real, FORCE, 64, 4, 4>(a, s); return true;
        case 8: launch_fused_t<Real, FORCE, 64, 8, 4>(a, s); return true;
        case 16: launch_fused_t<Real, FORCE, 64, 16, 4>(a, s); return true;
        default: return false;
    }
}

}  // namespace lbm

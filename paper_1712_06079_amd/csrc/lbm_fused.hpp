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

template <typename Real, int TX, int TY, int K, int RX = Radius<Real>::value, int RY = Radius<Real>::value>
struct FusedShape {
    static constexpr int CW = TX + 2, CH = TY + 2;           // collision region
    static constexpr int NCELL = CW * CH;
    static constexpr int NSX = (CW + K - 1) / K;              // x segments per collision row (explicit form)
    static constexpr int NSY = (CH + K - 1) / K;              // y segments per collision column (explicit form)
    static constexpr int NSEGX = 8;                           // x segments per collision row (recursive form; 8 keeps each
                                                              // item's chain short and a 4-row tile's items in one pass)
    static constexpr int SX = (CW + NSEGX - 1) / NSEGX;       // outputs per recursive x segment
    static constexpr int XSPAN = NSX * K > NSEGX * SX ? NSX * K : NSEGX * SX;
    static constexpr int RW = (XSPAN + 2 * RX) | 1;           // row-bar pitch (odd: spreads LDS banks)
    static constexpr int VH = NSY * K + 2 * RY;               // column-bar height (>= CH + 2 RY)
    static constexpr int RITEMS_X = CH * NSEGX, RITEMS_Y = CW;
    static constexpr int PHI_DOUBLES = CH * RW + VH * CW;     // phi cross (double)
    static constexpr int FS_DOUBLES = (Q * NCELL * (int)sizeof(Real) + 7) / 8;  // post-collision f (Real)
    static constexpr int A_DOUBLES = PHI_DOUBLES > FS_DOUBLES ? PHI_DOUBLES : FS_DOUBLES;
    static constexpr int DOUBLES = A_DOUBLES + 2 * NCELL;     // + Fx, Fy (double)
    static constexpr int NC = (NCELL + NT - 1) / NT;          // collision cells per thread
    static constexpr int NI = (TX * TY + NT - 1) / NT;        // interior cells per thread
    static constexpr int ITEMS_X = CH * NSX, ITEMS_Y = CW * NSY;
};

// K outputs of the explicit Eq. 20 stencil of radius R along one line from one
// window: output k sits at window position R + k; every window value is loaded
// once from LDS and added to the K outputs with the coefficients c(m - R - k),
// which are K consecutive entries of the sign-folded table (one scalar load).
template <int FORCE, int K, int R, typename BT = double>
__device__ inline void stencil_window(const BT* __restrict__ base, int stride, const double* __restrict__ tab,
                                      double (&acc)[K], double (&accu)[K]) {
    static_assert(R + K - 1 <= TAB_OFF && K <= KT, "stencil window outside the coefficient table");
#pragma unroll
    for (int k = 0; k < K; ++k) { acc[k] = 0.0; accu[k] = 0.0; }
#pragma unroll 4
    for (int m = 0; m < 2 * R + K; ++m) {
        const double v = base[m * stride];
        const double vo = (FORCE == FORCE_ZC) ? v : fabs(v);
        const double vu = v * fabs(v);
        const double* t = tab + (TAB_OFF - R - (K - 1)) + m;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double c = t[K - 1 - k];
            acc[k] += c * vo;
            if (FORCE == FORCE_HYBRID) accu[k] += c * vu;
        }
    }
}

// S outputs of Eq. 20 along one line of length > 2R + 1 in geometric form.
// With d_j = C r^j for j >= 3 and the first differences delta_k = u_{k+1} - u_k,
//   sum_{j>=3} r^j (u_{i+j} - u_{i-j}) = [r^3 (u_{i+3} - u_{i-3}) + Rt_i + Lt_i] / (1 - r),
//   Rt_i = sum_{m>=3} r^(m+1) delta_{i+m},   Lt_i = sum_{n>=4} r^n delta_{i-n},
// so Du_i = d_1 (u_{i+1} - u_{i-1}) + d_2 (u_{i+2} - u_{i-2})
//         + K [r^3 (u_{i+3} - u_{i-3}) + Rt_i + Lt_i],  K = C / (1 - r),
// with Rt_{i-1} = r Rt_i + r^4 delta_{i+2} (right to left) and
// Lt_{i+1} = r Lt_i + r^4 delta_{i-3} (left to right), each started R - 3 cells
// beyond the segment (every output keeps at least the taps j <= R).  Working on
// differences makes a constant line give exactly zero at every position.
// base[k * stride] is the operand's window value at output k (k in [-R, S-1+R]).
template <int FORCE, int S, int R>
__device__ inline void stencil_recursive(const double* __restrict__ base, int stride, double r, double r3, double r4,
                                         double d1, double d2, double K, double (&out)[S], double (&outu)[S]) {
    static_assert(R >= 4, "geometric form needs R >= 4");
    auto op = [](double v) { return FORCE == FORCE_ZC ? v : fabs(v); };
    auto opu = [](double v) { return v * fabs(v); };
    double Lt[S], Ltu[S];
    double l = 0.0, lu = 0.0;
#pragma unroll
    for (int i = -(R - 3); i < S - 1; ++i) {
        const double v2 = base[(i - 2) * stride], v3 = base[(i - 3) * stride];
        l = fma(r, l, r4 * (op(v2) - op(v3)));
        if (FORCE == FORCE_HYBRID) lu = fma(r, lu, r4 * (opu(v2) - opu(v3)));
        if (i + 1 >= 0) {
            Lt[i + 1] = l;
            Ltu[i + 1] = lu;
        }
    }
    double q = 0.0, qu = 0.0;
#pragma unroll
    for (int i = S - 1 + (R - 3); i >= 1; --i) {
        const double v3 = base[(i + 3) * stride], v2 = base[(i + 2) * stride];
        q = fma(r, q, r4 * (op(v3) - op(v2)));
        if (FORCE == FORCE_HYBRID) qu = fma(r, qu, r4 * (opu(v3) - opu(v2)));
        const int o = i - 1;
        if (o < S) {
            const double a1 = base[(o + 1) * stride], b1 = base[(o - 1) * stride];
            const double a2 = base[(o + 2) * stride], b2 = base[(o - 2) * stride];
            const double a3 = base[(o + 3) * stride], b3 = base[(o - 3) * stride];
            out[o] = d1 * (op(a1) - op(b1)) + d2 * (op(a2) - op(b2)) + K * (r3 * (op(a3) - op(b3)) + q + Lt[o]);
            if (FORCE == FORCE_HYBRID)
                outu[o] = d1 * (opu(a1) - opu(b1)) + d2 * (opu(a2) - opu(b2)) +
                          K * (r3 * (opu(a3) - opu(b3)) + qu + Ltu[o]);
        }
    }
}

template <int FORCE>
__device__ inline double force_from(double phic, double g, double gu, double A) {
    if (FORCE == FORCE_ZC) return -g;
    const double F = -2.0 * phic * g;
    return FORCE == FORCE_HYBRID ? A * (-gu) + (1.0 - 2.0 * A) * F : F;
}

// One TX x TY tile with origin (x0, y0) of the domain described by `a`;
// `sm` is the workgroup's LDS of FusedShape::DOUBLES doubles.  RX and RY are the
// stencil radii staged along x and y (>= the domain's taps along each axis).
// `tabs` is LDS for the two sign-folded coefficient tables (2 TAB doubles),
// staged here from the domain's device tables.
// With G9 the gradient is Eq. 15 (the 3 x 3 neighbourhood of every collision
// cell): the potential is staged over the block of rows y0-2 .. y0+TY+1 and
// columns x0-2 .. x0+TX+1 (in the column-bar area) instead of the cross.
template <typename Real, int FORCE, int TX, int TY, int K, int RX, int RY, bool G9 = false>
__device__ inline void fused_tile(const StepArgs<Real>& a, int x0, int y0, double* sm, double* tabs) {
    using S = FusedShape<Real, TX, TY, K, RX, RY>;
    constexpr int CW = S::CW, CH = S::CH;
    constexpr int B9W = CW + 2, B9 = (CH + 2) * B9W;  // Eq. 15 block: pitch, elements
    static_assert(B9 <= S::VH * CW, "the Eq. 15 block must fit the column-bar area");
    double* rowr = sm;                          // [CH][RW]   phi rows  x0-1-RX .. x0+TX+RX (+ segment padding)
    double* colr = rowr + CH * S::RW;           // [VH][CW]   phi cols  y0-1-RY .. y0+TY+RY (+ segment padding)
    Real* fst = reinterpret_cast<Real*>(sm);    // [Q][CH][CW] post-collision populations (after phase 2)
    double* Fx = sm + S::A_DOUBLES;             // [CH][CW]
    double* Fy = Fx + S::NCELL;

    // The thread index passes through an empty asm statement so that, in the
    // batched kernel's loop over tiles, the compiler cannot hoist the
    // lane-dependent offsets below out of the loop and hold them in registers.
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int nx = a.nx, ny = a.ny, nxb = a.nxb, pitch = nxb * BX;
    using P = typename PhiStore<Real, FORCE>::type;
    const P* __restrict__ phin = static_cast<const P*>(a.phi_in);
    P* __restrict__ phio = static_cast<P*>(a.phi_out);

    // Phase 1 loads: the potential cross, issued first because it is needed
    // first (vector loads retire in order, so a wait for the cross must not
    // also wait for the populations).
    StageRegs<CH * S::RW> srow;
    StageRegs<S::VH * CW> scol;
    // (plane offsets fit in 24-bit products: a plane has fewer than 2^31
    // elements and its rows fewer than 2^22)
    auto phi_at = [&](int yw, int xw) { return (double)phin[(unsigned)(__mul24(yw, pitch) + xw)]; };
    if constexpr (G9) {
        // past the block: rows beyond it repeat its last row, not read
        stage_issue_rc<S::VH * CW, B9W>(scol, tid, [&](int r, int c) {
            return phi_at(ymap_fast(y0 - 2 + min(r, CH + 1), ny, a.walls), wrap_fast(x0 - 2 + c, nx));
        });
    } else {
        stage_issue_rc<CH * S::RW, S::RW>(srow, tid, [&](int r, int c) {
            return phi_at(ymap_fast(y0 - 1 + r, ny, a.walls), wrap_fast(x0 - 1 - RX + c, nx));
        });
        stage_issue_rc<S::VH * CW, CW>(scol, tid, [&](int r, int c) {
            return phi_at(ymap_fast(y0 - 1 - RY + r, ny, a.walls), wrap_fast(x0 - 1 + c, nx));
        });
    }

    // Keep the compiler from moving cross loads behind population loads.
    __builtin_amdgcn_sched_barrier(0);

    // Phase 0: loads of f_t for this thread's collision cells (consumed in
    // phase 3, in flight during phases 1-2).
    Real f[S::NC][Q];
#pragma unroll
    for (int i = 0; i < S::NC; ++i) {
        const int c = min(tid + i * NT, S::NCELL - 1);  // past the end: a duplicate, never used
        const int cy = c / CW, cx = c - cy * CW;
        const int xw = wrap_fast(x0 - 1 + cx, nx), yw = ymap_fast(y0 - 1 + cy, ny, a.walls);
#pragma unroll
        for (int q = 0; q < Q; ++q) f[i][q] = a.f_in[fidx(xw, yw, q, nxb)];
    }

    __builtin_amdgcn_sched_barrier(0);

    // Phase 1: the cross and the coefficient tables into LDS.
    if constexpr (!G9) stage_commit(rowr, tid, srow);
    stage_commit(colr, tid, scol);
    for (int i = tid; i < TAB; i += NT) {
        tabs[i] = a.tab->tx_tab[i];
        tabs[TAB + i] = a.tab->ty_tab[i];
    }
    __syncthreads();

    // Phase 2: gradients and force.  Axes longer than 2R + 1 use the geometric
    // recursion (one segment of SX outputs per x item, a whole collision
    // column per y item); shorter axes the explicit K-blocked window.  With
    // G9, Eq. 15 over each collision cell's neighbourhood.
    if constexpr (G9) {
        auto op = [](double v) { return FORCE == FORCE_ZC ? v : fabs(v); };
        auto opu = [](double v) { return v * fabs(v); };
        for (int c = tid; c < S::NCELL; c += NT) {
            const int cy = c / CW, cx = c - cy * CW;
            const double* b = colr + cy * B9W + cx;  // block row cy (lattice row y-1), column cx (x-1)
            double m[3], ce[3], pl[3], mu[3], cu[3], pu[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                m[k] = op(b[k]);
                ce[k] = op(b[B9W + k]);
                pl[k] = op(b[2 * B9W + k]);
                mu[k] = opu(b[k]);
                cu[k] = opu(b[B9W + k]);
                pu[k] = opu(b[2 * B9W + k]);
            }
            double gx, gy, gxu = 0.0, gyu = 0.0;
            grad_d2q9(m, ce, pl, gx, gy);
            if (FORCE == FORCE_HYBRID) grad_d2q9(mu, cu, pu, gxu, gyu);
            const double phic = b[B9W + 1];
            Fx[c] = force_from<FORCE>(phic, gx, gxu, a.A);
            Fy[c] = force_from<FORCE>(phic, gy, gyu, a.A);
        }
    }
    const int nix = G9 ? 0 : (a.rec_x ? S::RITEMS_X : S::ITEMS_X);
    const int niy = G9 ? 0 : (a.rec_y ? S::RITEMS_Y : S::ITEMS_Y);
    // y items start at a wavefront boundary so that no wavefront runs both
    // the x and the y branch (they would execute one after the other).
    const int ybase = (nix + BX - 1) & ~(BX - 1);
    const int nit = ybase + niy;
    for (int jt = tid; jt < nit; jt += NT) {
        if (jt >= nix && jt < ybase) continue;
        const int it = jt < nix ? jt : jt - ybase + nix;
        if (it < nix && a.rec_x) {
            const int cy = it % CH, s = it / CH;
            double out[S::SX], outu[S::SX];
            stencil_recursive<FORCE, S::SX, RX>(rowr + cy * S::RW + RX + s * S::SX, 1, a.rr, a.rr3, a.rr4, a.rd1, a.rd2,
                                                a.rK, out, outu);
#pragma unroll
            for (int k = 0; k < S::SX; ++k) {
                const int cx = s * S::SX + k;
                if (cx < CW) Fx[cy * CW + cx] = force_from<FORCE>(rowr[cy * S::RW + cx + RX], out[k], outu[k], a.A);
            }
            continue;
        }
        if (it >= nix && a.rec_y) {
            const int cx = it - nix;
            double out[CH], outu[CH];
            stencil_recursive<FORCE, CH, RY>(colr + RY * CW + cx, CW, a.rr, a.rr3, a.rr4, a.rd1, a.rd2, a.rK,
                                             out, outu);
#pragma unroll
            for (int k = 0; k < CH; ++k) Fy[k * CW + cx] = force_from<FORCE>(colr[(k + RY) * CW + cx], out[k], outu[k], a.A);
            continue;
        }
        double acc[K], accu[K];
        if (it < nix) {
            const int cy = it % CH, s = it / CH;  // consecutive lanes: consecutive rows
            stencil_window<FORCE, K, RX>(rowr + cy * S::RW + s * K, 1, tabs, acc, accu);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int cx = s * K + k;
                if (cx < CW) Fx[cy * CW + cx] = force_from<FORCE>(rowr[cy * S::RW + cx + RX], acc[k], accu[k], a.A);
            }
        } else {
            const int yt = it - nix;
            const int cx = yt % CW, s = yt / CW;  // consecutive lanes: consecutive columns
            stencil_window<FORCE, K, RY>(colr + (s * K) * CW + cx, CW, tabs + TAB, acc, accu);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int cy = s * K + k;
                if (cy < CH) Fy[cy * CW + cx] = force_from<FORCE>(colr[(cy + RY) * CW + cx], acc[k], accu[k], a.A);
            }
        }
    }
    __syncthreads();

    // Phase 3: collision of the tile and its ring into LDS.
#pragma unroll
    for (int i = 0; i < S::NC; ++i) {
        const int c = tid + i * NT;
        if (c < S::NCELL) {
            double g[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) g[q] = (double)f[i][q];
            double rho, jx, jy;
            moments(g, rho, jx, jy);
            collide(g, rho, jx, jy, Fx[c], Fy[c], a.omega);
#pragma unroll
            for (int q = 0; q < Q; ++q) fst[q * S::NCELL + c] = (Real)g[q];
        }
    }
    __syncthreads();

    // Phase 4: pull streaming, aligned stores, epilogue phi_{t+1}.  Between
    // walls a population that would enter row 0 from below (or row ny-1 from
    // above) is the one that left the same site towards the wall, reversed.
#pragma unroll
    for (int i = 0; i < S::NI; ++i) {
        const int c = tid + i * NT;
        if (c < TX * TY) {
            const int ly = c / TX, lx = c - ly * TX;
            const int x = x0 + lx, y = y0 + ly;
            if (x < nx && y < ny) {
                double g[Q];
                const bool low = a.walls && y == 0, high = a.walls && y == ny - 1;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const bool back = (low && ey(q) > 0) || (high && ey(q) < 0);
                    const Real v = back ? fst[opp(q) * S::NCELL + (ly + 1) * CW + (lx + 1)]
                                        : fst[q * S::NCELL + (ly + 1 - ey(q)) * CW + (lx + 1 - ex(q))];
                    a.f_out[fidx(x, y, q, nxb)] = v;
                    g[q] = (double)v;
                }
                double rho, jx, jy;
                moments(g, rho, jx, jy);
                phio[(long)y * pitch + x] = (P)phi_of<FORCE>(potential(a.eos, rho));
            }
        }
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b mod 8), each with its own L2.  Tile t of the row-major tile order is
// given to the workgroup that makes every XCD own one contiguous band of
// tiles, so the +-R-row phi halos and ring cells a tile shares with its
// neighbours are mostly in the same L2.  The map is a bijection for any count.
constexpr int NXCD = 8;
__device__ inline int xcd_tile(int b, int G) {
    const int q = G / NXCD, r = G - q * NXCD;
    const int x = b % NXCD, s = b / NXCD;
    return x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

template <typename Real, int FORCE, int TX, int TY, int K, bool G9 = false>
__global__ void __launch_bounds__(NT) k_fused(StepArgs<Real> a) {
    constexpr int R = Radius<Real>::value;
    __shared__ double sm[FusedShape<Real, TX, TY, K, R, R>::DOUBLES];
    __shared__ double tabs[2 * TAB];
    const int t = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int ty = t / gridDim.x, tx = t - ty * gridDim.x;
    fused_tile<Real, FORCE, TX, TY, K, R, R, G9>(a, tx * TX, ty * TY, sm, tabs);
}

// Batched step: one launch advances every domain of a batch by one step.
// `tiles` lists (domain, x0, y0) work items in the scheduler's order; workgroup
// b processes items b, b + gridDim.x, ... (a persistent loop when the grid is
// smaller than the list).  `descs` holds one StepArgs per domain for this
// step's buffer parity.  Every item runs the same tile code as the
// single-domain kernel.
struct BatchTile {
    int d, x0, y0, pad;
};

template <typename Real, int FORCE, int TY, int RY, bool G9 = false>
__global__ void __launch_bounds__(NT) k_batch(const StepArgs<Real>* __restrict__ descs,
                                              const BatchTile* __restrict__ tiles, int ntiles) {
    constexpr int RX = Radius<Real>::value;
    __shared__ double sm[FusedShape<Real, BX, TY, 4, RX, RY>::DOUBLES];
    __shared__ double tabs[2 * TAB];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BatchTile w = tiles[t];
        fused_tile<Real, FORCE, BX, TY, 4, RX, RY, G9>(descs[w.d], w.x0, w.y0, sm, tabs);
        __syncthreads();
    }
}

// Per-domain non-finite flags of a batch: flags[d] |= 1 if any density of a
// tile of domain d is not finite (flags cleared by the caller beforehand).
template <typename Real>
__global__ void __launch_bounds__(NT) k_batch_finite(const StepArgs<Real>* __restrict__ descs,
                                                     const BatchTile* __restrict__ tiles, int ntiles, int ty,
                                                     int* __restrict__ flags) {
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BatchTile w = tiles[t];
        const StepArgs<Real>& a = descs[w.d];
        int bad = 0;
        for (int c = threadIdx.x; c < BX * ty; c += NT) {
            const int x = w.x0 + (c & (BX - 1)), y = w.y0 + c / BX;
            if (x < a.nx && y < a.ny) {
                double r = 0.0;
#pragma unroll
                for (int q = 0; q < Q; ++q) r += (double)a.f_in[fidx(x, y, q, a.nxb)];
                if (!isfinite(r)) bad = 1;
            }
        }
        if (bad) atomicOr(&flags[w.d], 1);
    }
}

template <typename Real, int FORCE, int TX, int TY, int K>
inline void launch_fused_t(const StepArgs<Real>& a, hipStream_t s) {
    dim3 grid((a.nx + TX - 1) / TX, (a.ny + TY - 1) / TY);
    if (a.grad9)
        hipLaunchKernelGGL((k_fused<Real, FORCE, TX, TY, K, true>), grid, dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_fused<Real, FORCE, TX, TY, K>), grid, dim3(NT), 0, s, a);
}

// Tile choice: FP64 storage uses 64 x 8 tiles (two workgroups per CU fit in
// LDS), FP32 storage 64 x 16; tile_y selects another instantiation (0 = default).
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

// Strip-marching single-pass time step for lattices whose y axis is longer
// than 2R + 1 (where Eq. 20 along y takes its geometric form).
//
// A workgroup owns one 64-column strip of the lattice over the rows [ys, ye) of
// one y chunk and walks down it in blocks of TY rows.  Compared with
// independent tiles (lbm_fused.hpp) this
//  - collides every row once (a tile also collides the ring rows above and
//    below it, which its neighbours collide again),
//  - keeps the potential rows the y stencil needs in an LDS ring, so a row is
//    read once per strip instead of once per tile and halo,
//  - carries the left-to-right half of the y recursion from block to block,
//  - and overlaps the loads of block k+1 with the arithmetic of block k.
//
// Block k covers the collision rows yb .. yb+TY-1 (yb = ys - 1 + k TY) and the
// 66 collision columns x0-1 .. x0+64:
//  1  issue the loads of block k+1: its populations, the potential rows that
//     enter the ring, its x bar (rows widened by +-R in x);
//  2  forces: d/dx from the bar (geometric recursion or the explicit window),
//     d/dy from the ring (forward state carried over, backward sum restarted
//     R - 3 rows below the block), then Eq. 22 / Eq. 7 / Eq. 9;
//  3  EDM-BGK collision of the TY x 66 cells into the post-collision ring,
//     which holds rows yb-2 .. yb+TY-1;
//  4  pull streaming of rows yb-1 .. yb+TY-2 (stored when inside [ys, ye)),
//     then rho -> U -> phi_{t+1} of those cells;
//  5  commit the potential loads of step 1 into LDS.
// Rows above ys and below ye are read with periodic wrap; a chunk starts one
// block early (rows ys-1 ..) and its first rows feed only cells it does not
// store.
#pragma once

#include "lbm_fused.hpp"

namespace lbm {

template <typename Real, int TY, int R>
struct MarchShape {
    static constexpr int CW = BX + 2;                       // collision columns x0-1 .. x0+64
    static constexpr int NCELL = TY * CW;                   // collision cells per block
    static constexpr int NC = (NCELL + NT - 1) / NT;        // per thread
    static constexpr int NI = (TY * BX + NT - 1) / NT;      // streamed cells per thread
    static constexpr int RING = TY + R + 4;                 // phi rows yb-4 .. yb+TY+R-1
    static constexpr int PR = TY + 2;                       // post-collision rows yb-2 .. yb+TY-1
    static constexpr int K = 4;                             // outputs per explicit-window item
    static constexpr int NSX = (CW + K - 1) / K;            // explicit x items per row
    static constexpr int NSEGX = 8;                         // recursive x segments per row
    static constexpr int SX = (CW + NSEGX - 1) / NSEGX;     // outputs per recursive segment
    static constexpr int XSPAN = NSEGX * SX > NSX * K ? NSEGX * SX : NSX * K;
    static constexpr int RW = (XSPAN + 2 * R) | 1;          // x-bar pitch (odd: spreads LDS banks)
    static constexpr int RING_D = RING * CW;
    static constexpr int BAR_D = TY * RW;
    static constexpr int POST_D = (Q * PR * CW * (int)sizeof(Real) + 7) / 8;
    static constexpr int DOUBLES = RING_D + BAR_D + 2 * NCELL + POST_D;
    static constexpr int XBASE = 2 * BX;                    // x items run on wavefronts 2 and 3
    static_assert(CW <= XBASE, "y items must fit below the x items");
    static_assert(NCELL >= NT / 2, "block too small for the thread layout");
};

template <typename Real, int FORCE, int TY>
__global__ void __launch_bounds__(NT) k_march(StepArgs<Real> a, int nchunk) {
    constexpr int R = Radius<Real>::value;
    using M = MarchShape<Real, TY, R>;
    constexpr int CW = M::CW, RING = M::RING, PR = M::PR, RW = M::RW, NCELL = M::NCELL;
    __shared__ double sm[M::DOUBLES];
    double* ring = sm;                 // [RING][CW] phi rows, row y in slot rslot(y)
    double* bar = ring + M::RING_D;    // [TY][RW]   phi of the block rows, x0-1-R .. x0+64+R (+ padding)
    double* Fx = bar + M::BAR_D;       // [TY][CW]
    double* Fy = Fx + NCELL;           // [TY][CW]
    Real* post = reinterpret_cast<Real*>(Fy + NCELL);  // [Q][PR][CW], row y in slot pslot(y)

    const int tid = threadIdx.x;
    const int nx = a.nx, ny = a.ny, nxb = a.nxb, pitch = nxb * BX;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int chunk = t / nxb, strip = t - chunk * nxb;
    const int x0 = strip * BX;
    const int ys = (int)((long)chunk * ny / nchunk), ye = (int)((long)(chunk + 1) * ny / nchunk);
    const int yb0 = ys - 1;
    const int nblk = (ye - ys + 2 + TY - 1) / TY;

    // Ring slots of virtual rows (the smallest row read is ys - 1 - R, the
    // smallest post-collision row ys - 3, so both arguments are >= 0).
    auto rslot = [&](int y) { return (int)((unsigned)(y - ys + R + 8) % (unsigned)RING); };
    auto pslot = [&](int y) { return (int)((unsigned)(y - ys + 3) % (unsigned)PR); };
    auto phi_at = [&](int y, int x) { return a.phi_in[(long)wrap(y, ny) * pitch + wrap(x, nx)]; };

    // Loads of block yn (issued one block ahead) and their commit to LDS.
    StageRegs<TY * CW> sring;  // phi rows yn+R .. yn+R+TY-1 (entering the ring)
    StageRegs<TY * RW> sbar;   // x bar of rows yn .. yn+TY-1
    Real fn[M::NC][Q];         // populations of the next block's collision cells
    Real fc[M::NC][Q];         // populations of this block's collision cells
    auto issue = [&](int yn) {
        stage_issue(sring, [&](int i) {
            const int r = i / CW, c = i - r * CW;
            return phi_at(yn + R + r, x0 - 1 + c);
        });
        stage_issue(sbar, [&](int i) {
            const int r = i / RW, c = i - r * RW;
            return phi_at(yn + r, x0 - 1 - R + c);
        });
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < M::NC; ++i) {
            const int c = min(tid + i * NT, NCELL - 1);  // past the end: a duplicate, never used
            const int r = c / CW, cc = c - r * CW;
            const int xw = wrap(x0 - 1 + cc, nx), yw = wrap(yn + r, ny);
#pragma unroll
            for (int q = 0; q < Q; ++q) fn[i][q] = a.f_in[fidx(xw, yw, q, nxb)];
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    auto commit = [&](int yn) {
#pragma unroll
        for (int j = 0; j < StageRegs<TY * CW>::PER; ++j) {
            const int i = tid + j * NT;
            if (i < TY * CW) {
                const int r = i / CW, c = i - r * CW;
                ring[rslot(yn + R + r) * CW + c] = sring.v[j];
            }
        }
        stage_commit(bar, sbar);
    };
    // Rows ylo .. ylo+nrows-1 into the ring (chunk prologue only).
    auto ring_fill = [&](int ylo, int nrows) {
        const int n = nrows * CW;
        for (int i0 = 0; i0 < n; i0 += 8 * NT) {
            double v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int i = min(i0 + tid + j * NT, n - 1);
                const int r = i / CW, c = i - r * CW;
                v[j] = phi_at(ylo + r, x0 - 1 + c);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int i = i0 + tid + j * NT;
                if (i < n) {
                    const int r = i / CW, c = i - r * CW;
                    ring[rslot(ylo + r) * CW + c] = v[j];
                }
            }
        }
    };

    auto op = [](double v) { return FORCE == FORCE_ZC ? v : fabs(v); };
    auto opu = [](double v) { return v * fabs(v); };
    const double rr = a.rr, rr3 = a.rr3, rr4 = a.rr4, rd1 = a.rd1, rd2 = a.rd2, rK = a.rK;

    // Prologue: the forward y recursion up to the first block (updates at rows
    // yb0-(R-3) .. yb0-2 read rows yb0-R .. yb0-4), then the ring for block 0.
    double l = 0.0, lu = 0.0;  // forward state of column tid (tid < CW)
    ring_fill(yb0 - R, R - 3);
    __syncthreads();
    if (tid < CW) {
        const double* colp = ring + tid;
        for (int i = yb0 - (R - 3); i <= yb0 - 2; ++i) {
            const double v2 = colp[rslot(i - 2) * CW], v3 = colp[rslot(i - 3) * CW];
            l = fma(rr, l, rr4 * (op(v2) - op(v3)));
            if (FORCE == FORCE_HYBRID) lu = fma(rr, lu, rr4 * (opu(v2) - opu(v3)));
        }
    }
    __syncthreads();
    ring_fill(yb0 - 4, R + 4);
    issue(yb0);
    commit(yb0);
#pragma unroll
    for (int i = 0; i < M::NC; ++i)
#pragma unroll
        for (int q = 0; q < Q; ++q) fc[i][q] = fn[i][q];
    __syncthreads();

    for (int k = 0; k < nblk; ++k) {
        const int yb = yb0 + k * TY;
        const bool more = k + 1 < nblk;
        if (more) issue(yb + TY);

        // Phase 2: forces of the block's collision cells.
        if (tid < CW) {
            // d/dy of column tid over rows yb .. yb+TY-1; ring row yb-4+j at ring_row(j).
            const double* colp = ring + tid;
            const int sb = rslot(yb - 4);
            auto at = [&](int j) {
                const int s = sb + j;
                return colp[(s >= RING ? s - RING : s) * CW];
            };
            double Lt[TY], Ltu[TY];
#pragma unroll
            for (int j = 0; j < TY; ++j) {  // update at row yb-1+j reads rows yb-3+j, yb-4+j
                const double v2 = at(j + 1), v3 = at(j);
                l = fma(rr, l, rr4 * (op(v2) - op(v3)));
                if (FORCE == FORCE_HYBRID) lu = fma(rr, lu, rr4 * (opu(v2) - opu(v3)));
                Lt[j] = l;
                Ltu[j] = lu;
            }
            double qv = 0.0, qu = 0.0;
#pragma unroll
            for (int i = TY - 1 + (R - 3); i >= 1; --i) {  // update at row yb+i reads rows yb+i+3, yb+i+2
                const double v3 = at(i + 7), v2 = at(i + 6);
                qv = fma(rr, qv, rr4 * (op(v3) - op(v2)));
                if (FORCE == FORCE_HYBRID) qu = fma(rr, qu, rr4 * (opu(v3) - opu(v2)));
                const int o = i - 1;  // output row yb+o
                if (o < TY) {
                    const double a1 = at(o + 5), b1 = at(o + 3), a2 = at(o + 6), b2 = at(o + 2);
                    const double a3 = at(o + 7), b3 = at(o + 1);
                    const double g = rd1 * (op(a1) - op(b1)) + rd2 * (op(a2) - op(b2)) +
                                     rK * (rr3 * (op(a3) - op(b3)) + qv + Lt[o]);
                    double gu = 0.0;
                    if (FORCE == FORCE_HYBRID)
                        gu = rd1 * (opu(a1) - opu(b1)) + rd2 * (opu(a2) - opu(b2)) +
                             rK * (rr3 * (opu(a3) - opu(b3)) + qu + Ltu[o]);
                    Fy[o * CW + tid] = force_from<FORCE>(at(o + 4), g, gu, a.A);
                }
            }
        } else if (tid >= M::XBASE) {
            // d/dx of the block rows from the bar.
            if (a.rec_x) {
                for (int it = tid - M::XBASE; it < TY * M::NSEGX; it += NT - M::XBASE) {
                    const int r = it % TY, s = it / TY;
                    double out[M::SX], outu[M::SX];
                    stencil_recursive<FORCE, M::SX, R>(bar + r * RW + R + s * M::SX, 1, rr, rr3, rr4, rd1, rd2, rK, out,
                                                       outu);
#pragma unroll
                    for (int j = 0; j < M::SX; ++j) {
                        const int cx = s * M::SX + j;
                        if (cx < CW) Fx[r * CW + cx] = force_from<FORCE>(bar[r * RW + cx + R], out[j], outu[j], a.A);
                    }
                }
            } else {
                for (int it = tid - M::XBASE; it < TY * M::NSX; it += NT - M::XBASE) {
                    const int r = it % TY, s = it / TY;
                    double acc[M::K], accu[M::K];
                    stencil_window<FORCE, M::K, R>(bar + r * RW + s * M::K, 1, a.tx_tab, acc, accu);
#pragma unroll
                    for (int j = 0; j < M::K; ++j) {
                        const int cx = s * M::K + j;
                        if (cx < CW) Fx[r * CW + cx] = force_from<FORCE>(bar[r * RW + cx + R], acc[j], accu[j], a.A);
                    }
                }
            }
        }
        __syncthreads();

        // Phase 3: collision of the block into the post-collision ring.
#pragma unroll
        for (int i = 0; i < M::NC; ++i) {
            const int c = tid + i * NT;
            if (c < NCELL) {
                const int r = c / CW, cc = c - r * CW;
                double g[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) g[q] = (double)fc[i][q];
                double rho, jx, jy;
                moments(g, rho, jx, jy);
                collide(g, rho, jx, jy, Fx[c], Fy[c], a.omega);
                const int ps = pslot(yb + r);
#pragma unroll
                for (int q = 0; q < Q; ++q) post[(q * PR + ps) * CW + cc] = (Real)g[q];
            }
        }
        __syncthreads();

        // Phase 4: pull streaming of rows yb-1 .. yb+TY-2 and phi_{t+1}.
#pragma unroll
        for (int i = 0; i < M::NI; ++i) {
            const int c = tid + i * NT;
            if (c < TY * BX) {
                const int r = c / BX, lx = c - r * BX;
                const int y = yb - 1 + r, x = x0 + lx;
                if (y >= ys && y < ye && x < nx) {
                    double g[Q];
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const Real v = post[(q * PR + pslot(y - ey(q))) * CW + lx + 1 - ex(q)];
                        a.f_out[fidx(x, y, q, nxb)] = v;
                        g[q] = (double)v;
                    }
                    double rho, jx, jy;
                    moments(g, rho, jx, jy);
                    a.phi_out[(long)y * pitch + x] = phi_of<FORCE>(potential(a.eos, rho));
                }
            }
        }

        // Phase 5: the next block's potential rows into LDS.
        if (more) {
            commit(yb + TY);
#pragma unroll
            for (int i = 0; i < M::NC; ++i)
#pragma unroll
                for (int q = 0; q < Q; ++q) fc[i][q] = fn[i][q];
        }
        __syncthreads();
    }
}

// LDS bytes of one workgroup of the marching kernel.
template <typename Real, int TY>
constexpr int march_lds_bytes() {
    return MarchShape<Real, TY, Radius<Real>::value>::DOUBLES * 8;
}

// Launch over nchunk y chunks of every 64-column strip (nchunk in [1, ny]).
template <typename Real, int FORCE>
inline bool launch_march(const StepArgs<Real>& a, int ty, int nchunk, hipStream_t s) {
    const dim3 grid((unsigned)(a.nxb * nchunk));
    switch (ty) {
        case 4: hipLaunchKernelGGL((k_march<Real, FORCE, 4>), grid, dim3(NT), 0, s, a, nchunk); return true;
        case 8: hipLaunchKernelGGL((k_march<Real, FORCE, 8>), grid, dim3(NT), 0, s, a, nchunk); return true;
        default: return false;
    }
}

}  // namespace lbm

// Strip-marching single-pass time step for lattices whose y axis is longer
// than 2R + 1 (where Eq. 20 along y takes its geometric form).
//
// A workgroup owns one 64-column strip of the lattice over the rows [ys, ye) of
// one y chunk and walks down it in blocks of TY rows.  Compared with
// independent tiles (lbm_fused.hpp) this collides every row once, reads the
// potential rows of the y stencil about once per strip, and overlaps the loads
// of block k+1 with the arithmetic of block k.
//
// The potential rows around the block (yb-4 .. yb+TY+3, over x0-1-R ..
// x0+64+R) live in an LDS ring of TY+8 rows, the "bar": its rows feed the x
// derivative of the block rows and the y windows of every column.
//
// The y derivative.  In the difference form of the geometric recursion (see
// stencil_recursive) the output at row o needs the forward sum Lt_o, carried
// from block to block, and the backward sum q(o+1), with
//   q(i) = sum_{n>=0} r^n t_{i+n},   t_i = r^4 (u_{i+3} - u_{i+2}).
// Grouping the t of the TY-row blocks ahead of the current block,
//   W_j = sum_{n<TY} r^n t_{yb+1+jTY+n}   (j = 1 .. NB),
//   q(yb+1+TY) = sum_j r^{(j-1)TY} W_j,
// so a column keeps NB block sums in registers (one new W per block, from the
// TY rows that arrive NB blocks ahead) and reads the TY+8 rows around the
// block from the bar; q inside the block is the recursion over its own TY
// rows.  NB TY + 3 >= R keeps at least R taps for every output.
//
// Lanes (256 threads, four wavefronts):
//  wave 0   one interior column each (x0 .. x0+63): d/dy -> F_y in LDS;
//  wave 1   lanes 0 .. 2TY-1 own the ring cells (columns x0-1 and x0+64, TY
//           rows): their d/dy in the force phase (on a short x axis also
//           their d/dx, over the bar), their collision in the collision phase;
//  waves 2-3  d/dx of the interior and of the ring cells: per row and 8-column
//           segment one lane runs the forward and its neighbour the backward
//           recursion in lockstep, the two exchange their sums and each
//           finishes half the segment's F_x (or the explicit window on a short
//           x axis);
//  all      one interior cell pair each for collision and streaming.
// Per block (collision rows yb .. yb+TY-1, yb = ys - 1 + k TY):
//  1  issue the loads of block k+1 (its new bar rows, its ring-cell
//     populations, each column's rows NB blocks ahead);
//  2  forces of the interior and of the ring cells;
//  3  collision of the interior and ring cells into the post-collision ring
//     (rows yb-2 .. yb+TY-1);
//  4  commit the loads of step 1 (LDS, block sums), issue the next block's
//     interior populations (in flight through the next block's step 2; with
//     FP64 populations and TY = 8 they are issued earlier: in step 1 with the
//     potential rows, or for the hybrid force at the start of step 3), then
//     pull streaming of rows yb-1 .. yb+TY-2 (stored when inside [ys, ye))
//     and rho -> U -> phi_{t+1}.
#pragma once

#include "lbm_fused.hpp"

namespace lbm {

template <typename Real, int FORCE, int TY, int R>
struct MarchShape {
    static constexpr int CW = BX + 2;                       // collision columns x0-1 .. x0+64
    static constexpr int CWP = CW + 2;                      // post-collision row pitch (column cc at cc + 1)
    static constexpr int NPAIR = TY * BX / 2;               // interior cell pairs (x, x+1) per block
    static constexpr int NP = (NPAIR + NT - 1) / NT;        // pairs per thread
    static constexpr int PR = TY + 2;                       // post-collision rows yb-2 .. yb+TY-1
    static constexpr int NB = (R - 3 + TY - 1) / TY;        // block sums ahead (NB TY + 3 >= R)
    static constexpr int BR = TY + 8;                       // bar rows yb-4 .. yb+TY+3
    static constexpr int NRING = 2 * TY;                    // ring cells per block
    static constexpr int K = 4;                             // outputs per explicit-window item
    static constexpr int NSEG = 8, SEG = BX / NSEG;         // recursive x segments per row, width
    static constexpr int RW = (CW + 2 * R) | 1;             // bar pitch (odd: spreads LDS banks)
    // The bar holds the potential in its storage type (FP32 for FP32
    // populations with the SC or ZC force: exact, and 1 % faster at 4096^2).
    using BarT = typename PhiStore<Real, FORCE>::type;
    static constexpr int BAR_N = BR * RW;                                  // elements
    static constexpr int BAR_D = (BAR_N * (int)sizeof(BarT) + 7) / 8;     // LDS doubles
    static constexpr int F_D = 2 * TY * BX + 2 * NRING;     // F_x, F_y of the interior and of the ring cells
    static constexpr int FRING_D = (NRING * Q * (int)sizeof(Real) + 7) / 8;
    static constexpr int POST_D = (Q * PR * CWP * (int)sizeof(Real) + 7) / 8;
    static constexpr int WARM_ROWS = R - 3, WSUM_ROWS = NB * TY + 1;  // prologue rows per column
    static constexpr int DOUBLES = BAR_D + F_D + FRING_D + POST_D;
    static constexpr int XBASE = 2 * BX;                    // first x lane
    // Waves per SIMD the register allocation must allow (at most 512 / WAVES
    // VGPRs): three; two for the hybrid force (two potential fields) and for
    // FP64 populations with TY = 8, whose LDS footprint admits only two
    // workgroups per CU anyway.
    static constexpr int WAVES = (FORCE == FORCE_HYBRID || (sizeof(Real) == 8 && TY == 8)) ? 2 : 3;
    // Where the LDS already limits residency to two workgroups per CU (FP64,
    // TY = 8) the spare registers hold the next block's populations longer:
    // they are loaded at the top of the block, with the potential rows, and
    // stay in flight through the force and collision phases while the
    // current block's copy is collided (TOP_F; 4096^2: +8 %).  The hybrid
    // force's second potential field leaves no room for that: it loads them
    // at the start of the collision phase (EARLY_F).  With FP32 populations
    // the extra registers cost more than the longer flight gains (loading at
    // the top: -6.5 %), so they load after the commit.
    static constexpr bool TOP_F = sizeof(Real) == 8 && TY == 8 && FORCE != FORCE_HYBRID;
    static constexpr bool EARLY_F = sizeof(Real) == 8 && TY == 8 && FORCE == FORCE_HYBRID;
    static_assert(NPAIR % 32 == 0 && NP >= 1, "block rows must fill whole half-wavefronts");
    static_assert((BAR_D + F_D + FRING_D) % 2 == 0, "post-collision rows must be 16-byte aligned");
    static_assert(NRING <= BX, "ring lanes must fit in one wavefront");
    static_assert(2 * TY * NSEG <= NT - XBASE && TY * (BX / K) <= NT - XBASE, "x lanes must fit");
    static_assert(NRING * Q <= NT, "ring-cell loads: one value per thread");
    static_assert(SEG % 2 == 0, "each lane of a pair finishes half a segment");
};

// Population loads and stores and the stores of phi_{t+1}: each value is
// touched once per step.  Where the step's state (both population and
// potential buffers) exceeds the last-level cache, non-temporal accesses
// (NTA) keep it from evicting the potential rows, which are read again a few
// blocks later.  Where the whole state stays resident in that cache from one
// step to the next, plain accesses let the next step read it from there.
template <bool NTA, typename T>
__device__ inline T ld_once(const T* p) {
    if constexpr (NTA) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NTA, typename T>
__device__ inline void st_once(T v, T* p) {
    if constexpr (NTA) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Interior cells are handled in pairs (x, x+1), x even, one pair per lane, so
// that a lane moves both cells' populations with one 16-byte (FP64) or 8-byte
// (FP32) access.  VEC selects those paired accesses; it requires an even N_x
// (a pair never straddles the periodic seam).  Odd N_x uses per-cell accesses.
// The register budget follows MarchShape::WAVES (VGPRs + AGPRs <= 512 / WAVES);
// it is a hard limit, not a hint.
template <typename Real, int FORCE, int TY, bool VEC, bool NTA>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MarchShape<Real, FORCE, TY, Radius<Real>::value>::WAVES))) k_march(StepArgs<Real> a, int nchunk) {
    constexpr int R = Radius<Real>::value;
    using M = MarchShape<Real, FORCE, TY, R>;
    using V2 = Real __attribute__((ext_vector_type(2)));
    constexpr int CW = M::CW, CWP = M::CWP, PR = M::PR, RW = M::RW, NB = M::NB, BR = M::BR, SEG = M::SEG;
    constexpr bool HYB = FORCE == FORCE_HYBRID;
    constexpr bool TOP_F = M::TOP_F, EARLY_F = M::EARLY_F;
    __shared__ __align__(16) double sm[M::DOUBLES];
    __shared__ double ctab[TAB];               // sign-folded x coefficients (staged in the prologue)
    using BarT = typename M::BarT;
    BarT* bar = reinterpret_cast<BarT*>(sm);   // [BR][RW] phi rows, x0-1-R .. x0+64+R; row y in slot bslot(y)
    double* Fx = sm + M::BAR_D;                // [TY][64] x force of the interior
    double* Fy = Fx + TY * BX;                 // [TY][64] y force of the interior
    double* FxR = Fy + TY * BX;                // [2TY] x force of the ring cells
    double* FyR = FxR + M::NRING;              // [2TY] y force of the ring cells
    Real* fring = reinterpret_cast<Real*>(FyR + M::NRING);                  // [2TY][Q] ring-cell f
    Real* post = reinterpret_cast<Real*>(FyR + M::NRING + M::FRING_D);      // [Q][PR][CWP]

    // Lane-dependent indices are re-derived in every block from a copy of the
    // thread index that the compiler cannot treat as loop-invariant: hoisting
    // the many lane-dependent offsets out of the march would hold them in
    // registers for the whole kernel.  Only the wrapped lattice columns that
    // need a general modulo are kept (bcol, xcol, xring, xpair).
    using P = typename PhiStore<Real, FORCE>::type;
    const P* __restrict__ phin = static_cast<const P*>(a.phi_in);
    P* __restrict__ phio = static_cast<P*>(a.phi_out);
    int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    int lane = tid & (BX - 1);
    const int nx = a.nx, ny = a.ny, nxb = a.nxb, pitch = nxb * BX;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int chunk = t / nxb, strip = t - chunk * nxb;
    const int x0 = strip * BX;
    const int ys = (int)((long)chunk * ny / nchunk), ye = (int)((long)(chunk + 1) * ny / nchunk);
    const int yb0 = ys - 1;
    const int nblk = (ye - ys + 2 + TY - 1) / TY;

    // Every row index used below lies in [ys - R - 2, ye + (NB + 2) TY + 4],
    // within one period of [0, ny): one correction wraps it.
    auto wrapy = [&](int y) { return y < 0 ? y + ny : (y >= ny ? y - ny : y); };
    // Ring slots (the smallest bar row is ys - 5, the smallest post-collision
    // row ys - 3, so both arguments are >= 0).
    auto bslot = [&](int y) { return (int)((unsigned)(y - ys + 16) % (unsigned)BR); };
    auto pslot = [&](int y) { return (int)((unsigned)(y - ys + 3) % (unsigned)PR); };
    auto op = [](double v) { return FORCE == FORCE_ZC ? v : fabs(v); };
    auto opu = [](double v) { return v * fabs(v); };
    const double rr = a.rr, rr3 = a.rr3, rr4 = a.rr4, rd1 = a.rd1, rd2 = a.rd2, rK = a.rK;

    // Column owned by this lane (waves 0-1): interior column x0+lane, or the
    // ring column of ring lane e = lane (x0-1 for e < TY, x0+64 otherwise).
    const bool colw = wave < 2;
    int ccol = wave == 0 ? lane + 1 : (lane < TY ? 0 : CW - 1);   // collision column
    int rrow = lane % TY;                                         // ring lane's row
    auto lane_indices = [&]() {
        lane = tid & (BX - 1);
        ccol = wave == 0 ? lane + 1 : (lane < TY ? 0 : CW - 1);
        rrow = lane % TY;
    };
    const int xcol = wrap(x0 - 1 + ccol, nx);
    constexpr int BPER = StageRegs<TY * RW>::PER;
    int bcol[BPER];                   // lattice column of each bar element this thread loads
#pragma unroll
    for (int j = 0; j < BPER; ++j) {
        const int i = min(tid + j * NT, TY * RW - 1);
        bcol[j] = wrap(x0 - 1 - R + (i - (i / RW) * RW), nx);
    }
    const int xring = wrap(min(tid, M::NRING * Q - 1) / Q < TY ? x0 - 1 : x0 + BX, nx);
    int xpair[M::NP][2];              // lattice columns of this thread's interior pairs
#pragma unroll
    for (int i = 0; i < M::NP; ++i) {
        const int t = min(tid + i * NT, M::NPAIR - 1);
        xpair[i][0] = wrap(x0 + 2 * (t & 31), nx);
        xpair[i][1] = VEC ? 0 : wrap(x0 + 2 * (t & 31) + 1, nx);
    }
    // Interior pairs of this thread (collision and streaming): pair t = tid + i NT
    // is row t / 32, cells x0 + 2 (t % 32) and the one after.

    // ---------------------------------------------------------------- state
    double W[NB], Wu[NB];             // block sums W_1 .. W_NB
    double uprev = 0.0, uprevu = 0.0; // operand of the row preceding the next far rows
    double l = 0.0, lu = 0.0;         // forward y state
    double pfar[TY];                  // loads of the rows NB blocks ahead (this lane's column)
    StageRegs<TY * RW> sbar;          // loads of the bar rows entering the ring
    double fr = 0.0;                  // one ring-cell population (tid < 2 TY Q)
    Real fc[M::NP][2][Q];             // interior populations of the next block (in flight)

    // Loads of block yn (all unconditional; lanes with no use load a clamped
    // valid address) and their commit.
    auto issue_bar = [&](int yn) {    // bar rows yn+4 .. yn+TY+3 enter the ring for block yn
#pragma unroll
        for (int j = 0; j < BPER; ++j) {
            const int i = min(tid + j * NT, TY * RW - 1);  // past the end: a duplicate, not stored
            sbar.v[j] = (double)phin[(long)wrapy(yn + 4 + i / RW) * pitch + bcol[j]];
        }
    };
    auto issue_fr = [&](int yn) {     // ring-cell populations of block yn
        const int i = min(tid, M::NRING * Q - 1);  // past the end: a duplicate, not stored
        const int e = i / Q, q = i - e * Q;
        fr = (double)a.f_in[fidx(xring, wrapy(yn + e % TY), q, nxb)];
    };
    auto issue_col = [&](int yn) {    // rows NB blocks ahead of block yn (every lane; waves 2-3 unused)
#pragma unroll
        for (int j = 0; j < TY; ++j) pfar[j] = (double)phin[(long)wrapy(yn + 4 + NB * TY + j) * pitch + xcol];
    };
    auto issue_f = [&](int yn) {      // interior populations of block yn (after their last use)
#pragma unroll
        for (int i = 0; i < M::NP; ++i) {
            const int t = min(tid + i * NT, M::NPAIR - 1);  // past the end: a duplicate, never used
            const int yw = wrapy(yn + (t >> 5));
            const int xa = xpair[i][0];
            if (VEC) {
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const V2 v = ld_once<NTA>(reinterpret_cast<const V2*>(a.f_in + fidx(xa, yw, q, nxb)));
                    fc[i][0][q] = v.x;
                    fc[i][1][q] = v.y;
                }
            } else {
                const int xb = xpair[i][1];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    fc[i][0][q] = ld_once<NTA>(a.f_in + fidx(xa, yw, q, nxb));
                    fc[i][1][q] = ld_once<NTA>(a.f_in + fidx(xb, yw, q, nxb));
                }
            }
        }
    };
    // New block sum from the operands of rows uprev, p[0 .. TY-1]:
    // t_n = r^4 (u_{n+1} - u_n) over that row sequence, W = sum r^n t_n.
    auto block_sum = [&](double u0, const double (&p)[TY], bool hyb) {
        double w = 0.0;
#pragma unroll
        for (int n = TY - 1; n >= 0; --n) {
            const double un1 = hyb ? opu(p[n]) : op(p[n]);
            const double un = n == 0 ? u0 : (hyb ? opu(p[n - 1]) : op(p[n - 1]));
            w = fma(rr, w, rr4 * (un1 - un));
        }
        return w;
    };
    auto commit_col = [&]() {         // advance the block sums by one block
        if (colw) {
#pragma unroll
            for (int j = 0; j < NB - 1; ++j) W[j] = W[j + 1];
            W[NB - 1] = block_sum(uprev, pfar, false);
            uprev = op(pfar[TY - 1]);
            if (HYB) {
#pragma unroll
                for (int j = 0; j < NB - 1; ++j) Wu[j] = Wu[j + 1];
                Wu[NB - 1] = block_sum(uprevu, pfar, true);
                uprevu = opu(pfar[TY - 1]);
            }
        }
    };
    auto commit = [&](int yn) {       // block yn's new bar rows and ring cells into LDS
#pragma unroll
        for (int j = 0; j < StageRegs<TY * RW>::PER; ++j) {
            const int i = tid + j * NT;
            if (i < TY * RW) {
                const int r = i / RW, c = i - r * RW;
                bar[bslot(yn + 4 + r) * RW + c] = (BarT)sbar.v[j];
            }
        }
        if (tid < M::NRING * Q) fring[tid] = (Real)fr;
    };

    // d/dy of this lane's column over the block rows yb .. yb+TY-1 from the
    // bar rows yb-4 .. yb+TY+3 and the block sums: g[o], gu[o] for row yb+o,
    // phc[o] its potential.  Advances the forward state.
    double rT = 1.0;  // r^TY
#pragma unroll
    for (int j = 0; j < TY; ++j) rT *= rr;
    auto ddy = [&](int yb, double (&g)[TY], double (&gu)[TY], double (&phc)[TY]) {
        double win[TY + 8];           // phi of rows yb-4 .. yb+TY+3 (window index of row y: y - yb + 4)
        const int sb = bslot(yb - 4);
#pragma unroll
        for (int j = 0; j < TY + 8; ++j) {
            const int s = sb + j;
            win[j] = bar[(s >= BR ? s - BR : s) * RW + R + ccol];
        }
        double Lt[TY], Ltu[TY];
#pragma unroll
        for (int o = 0; o < TY; ++o) {  // forward update at row yb+o-1 reads rows yb+o-3, yb+o-4
            l = fma(rr, l, rr4 * (op(win[o + 1]) - op(win[o])));
            Lt[o] = l;
            if (HYB) {
                lu = fma(rr, lu, rr4 * (opu(win[o + 1]) - opu(win[o])));
                Ltu[o] = lu;
            }
        }
        double q = W[NB - 1], qu = HYB ? Wu[NB - 1] : 0.0;  // q(yb+1+TY), Horner over the block sums
#pragma unroll
        for (int j = NB - 2; j >= 0; --j) {
            q = fma(rT, q, W[j]);
            if (HYB) qu = fma(rT, qu, Wu[j]);
        }
#pragma unroll
        for (int o = TY - 1; o >= 0; --o) {
            // q(yb+o+1) = t_{yb+o+1} + r q(yb+o+2), t_i from rows i+3, i+2
            q = fma(rr, q, rr4 * (op(win[o + 8]) - op(win[o + 7])));
            const int w = o + 4;
            g[o] = rd1 * (op(win[w + 1]) - op(win[w - 1])) + rd2 * (op(win[w + 2]) - op(win[w - 2])) +
                   rK * (rr3 * (op(win[w + 3]) - op(win[w - 3])) + q + Lt[o]);
            phc[o] = win[w];
            if (HYB) {
                qu = fma(rr, qu, rr4 * (opu(win[o + 8]) - opu(win[o + 7])));
                gu[o] = rd1 * (opu(win[w + 1]) - opu(win[w - 1])) + rd2 * (opu(win[w + 2]) - opu(win[w - 2])) +
                        rK * (rr3 * (opu(win[w + 3]) - opu(win[w - 3])) + qu + Ltu[o]);
            } else {
                gu[o] = 0.0;
            }
        }
    };

    // ------------------------------------------------------------- prologue
    // The bar rows yb0-4 .. yb0+TY+3 go to LDS; each column lane reads its own
    // column's rows straight into registers for the forward y state up to the
    // first block (updates at rows yb0-(R-3) .. yb0-2 read rows yb0-R ..
    // yb0-4) and for the block sums W_1 .. W_NB of block 0 (rows yb0+3+TY ..
    // yb0+3+(NB+1)TY).  The bar and warm-up loads are issued together, the
    // block-sum rows next: two memory round trips and one barrier before the
    // march.
    constexpr int BP = (M::BAR_N + NT - 1) / NT;
    double vb[BP];
#pragma unroll
    for (int j = 0; j < BP; ++j) {
        const int i = min(tid + j * NT, M::BAR_N - 1);  // past the end: a duplicate, not stored
        const int r = i / RW, c = i - r * RW;
        vb[j] = (double)phin[(long)wrapy(yb0 - 4 + r) * pitch + wrap(x0 - 1 - R + c, nx)];
    }
    const P* colp = phin + xcol;  // this lane's column (waves 0-1)
    double u[M::WARM_ROWS];
    if (colw) {
#pragma unroll
        for (int m = 0; m < M::WARM_ROWS; ++m) u[m] = colp[(long)wrapy(yb0 - R + m) * pitch];
    }
#pragma unroll
    for (int j = 0; j < BP; ++j) {
        const int i = tid + j * NT;
        if (i < M::BAR_N) {
            const int r = i / RW, c = i - r * RW;
            bar[bslot(yb0 - 4 + r) * RW + c] = (BarT)vb[j];
        }
    }
    for (int i = tid; i < TAB; i += NT) ctab[i] = a.tab->tx_tab[i];
    if (colw) {
#pragma unroll
        for (int m = 1; m <= R - 4; ++m) {
            l = fma(rr, l, rr4 * (op(u[m]) - op(u[m - 1])));
            if (HYB) lu = fma(rr, lu, rr4 * (opu(u[m]) - opu(u[m - 1])));
        }
        double w[M::WSUM_ROWS];
#pragma unroll
        for (int i = 0; i < M::WSUM_ROWS; ++i) w[i] = colp[(long)wrapy(yb0 + 3 + TY + i) * pitch];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            double pj[TY];
#pragma unroll
            for (int n = 0; n < TY; ++n) pj[n] = w[j * TY + n + 1];
            W[j] = block_sum(op(w[j * TY]), pj, false);
            if (HYB) Wu[j] = block_sum(opu(w[j * TY]), pj, true);
        }
        uprev = op(w[NB * TY]);
        uprevu = opu(w[NB * TY]);
    }
    issue_fr(yb0);
    issue_f(yb0);
    if (tid < M::NRING * Q) fring[tid] = (Real)fr;
    __syncthreads();

    // ------------------------------------------------------------ the march
    // Every global load of the loop is issued unconditionally and in the same
    // order on every path (the last block loads rows it never uses), so the
    // compiler's wait counts are exact: each wait covers only the loads it
    // needs, not the younger prefetches.
    for (int k = 0; k < nblk; ++k) {
        const int yb = yb0 + k * TY;
        asm volatile("" : "+v"(tid));
        lane_indices();
        // Loads are issued at a raised wave priority, so that a wave about to
        // put memory traffic in flight wins issue arbitration over waves that
        // are computing (FP32 populations +1.6 %, FP64 +0.4 %; keeping it
        // through the streaming stores where the populations load late: FP32
        // +0.5 % more).
        // This block's interior populations: with TOP_F they are copied out
        // here, and the next block's are issued after the potential rows.
        double gc[M::NP][2][Q];
        auto take_f = [&]() {
#pragma unroll
            for (int i = 0; i < M::NP; ++i)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int q = 0; q < Q; ++q) gc[i][h][q] = (double)fc[i][h][q];
        };
        if (TOP_F) take_f();
        __builtin_amdgcn_s_setprio(2);
        issue_col(yb + TY);
        issue_bar(yb + TY);
        issue_fr(yb + TY);
        if (TOP_F) issue_f(yb + TY);
        __builtin_amdgcn_s_setprio(0);

        // Phase 2: forces of the interior and of the ring cells.
        if (wave == 0) {
            double g[TY], gu[TY], phc[TY];
            ddy(yb, g, gu, phc);
#pragma unroll
            for (int o = 0; o < TY; ++o) Fy[o * BX + lane] = force_from<FORCE>(phc[o], g[o], gu[o], a.A);
        } else if (wave == 1) {
            double g[TY], gu[TY], phc[TY];
            ddy(yb, g, gu, phc);
            if (lane < M::NRING) {
                double gy = 0.0, gyu = 0.0;
#pragma unroll
                for (int o = 0; o < TY; ++o)
                    if (o == rrow) {
                        gy = g[o];
                        gyu = gu[o];
                    }
                const BarT* br = bar + bslot(yb + rrow) * RW + ccol + R;
                const double phic = br[0];
                FyR[lane] = force_from<FORCE>(phic, gy, gyu, a.A);
                if (!a.rec_x) {
                    // d/dx of the ring cell on a short x axis: the periodic
                    // row's table over the bar (on a long axis the x lanes
                    // produce it with the interior)
                    double sx[4] = {0.0, 0.0, 0.0, 0.0}, sxu[4] = {0.0, 0.0, 0.0, 0.0};  // four partial sums
#pragma unroll 8
                    for (int n = 1; n <= R; ++n) {
                        const double c = ctab[TAB_OFF + n];
                        const double vp = br[n], vm = br[-n];
                        sx[n & 3] = fma(c, op(vp) - op(vm), sx[n & 3]);
                        if (HYB) sxu[n & 3] = fma(c, opu(vp) - opu(vm), sxu[n & 3]);
                    }
                    const double gx = (sx[0] + sx[1]) + (sx[2] + sx[3]);
                    const double gxu = (sxu[0] + sxu[1]) + (sxu[2] + sxu[3]);
                    FxR[lane] = force_from<FORCE>(phic, gx, gxu, a.A);
                }
            }
        } else if (a.rec_x) {
            // forward (even lane) and backward (odd lane) x recursion of one
            // 8-column segment of one row, in lockstep: at step j both read
            // u[pa] - u[pa - 1], pa = A0 + S j; the last SEG steps give the
            // outputs (forward: o = m, backward: o = SEG-1-m at step R-4+m),
            // kept in registers, in units of r^4 (the factor is applied once
            // per output).  The two lanes then swap their sums and each
            // finishes F_x of half the segment.  One more step past the
            // outputs gives the ring columns: the forward sum at x0-1 is
            // segment 0's sum before its first output, the backward sum there
            // its backward lane's extra step, and mirrored at x0+64 for the
            // last segment.
            const int xi = tid - M::XBASE;
            if (xi < 2 * TY * M::NSEG) {
                const int item = xi >> 1, dir = xi & 1;
                const int r = item % TY, sg = item / TY;
                const BarT* rowp = bar + bslot(yb + r) * RW;
                const BarT* base = rowp + R + 1 + sg * SEG;  // interior column 1 + sg SEG at k = 0
                const int A0 = dir ? SEG + R - 1 : -(R - 1), S = dir ? -1 : 1;
                double acc = 0.0, accu = 0.0, out[SEG], outu[SEG];
#pragma unroll 8
                for (int j = 0; j < R - 4; ++j) {  // warm-up steps
                    const int pa = A0 + S * j;
                    const double va = base[pa], vb = base[pa - 1];
                    acc = fma(rr, acc, op(va) - op(vb));
                    if (HYB) accu = fma(rr, accu, opu(va) - opu(vb));
                }
                const double pre = acc, preu = accu;  // sum at the column before the outputs
#pragma unroll
                for (int m = 0; m < SEG; ++m) {    // output steps
                    const int pa = A0 + S * (R - 4 + m);
                    const double va = base[pa], vb = base[pa - 1];
                    acc = fma(rr, acc, op(va) - op(vb));
                    if (HYB) accu = fma(rr, accu, opu(va) - opu(vb));
                    out[m] = acc;
                    outu[m] = accu;
                }
                {                                  // the column after the outputs
                    const int pa = A0 + S * (R - 4 + SEG);
                    const double va = base[pa], vb = base[pa - 1];
                    acc = fma(rr, acc, op(va) - op(vb));
                    if (HYB) accu = fma(rr, accu, opu(va) - opu(vb));
                }
                // Lane pairs swap: for k < SEG/2 a lane receives its partner's
                // out[k] and adds its own out[SEG-1-k]; that is the full sum at
                // output o = SEG-1-k (forward lane) or o = k (backward lane).
#pragma unroll
                for (int k = 0; k < SEG / 2; ++k) {
                    const double s = out[SEG - 1 - k] + __shfl_xor(out[k], 1);
                    double su = 0.0;
                    if (HYB) su = outu[SEG - 1 - k] + __shfl_xor(outu[k], 1);
                    const int o = dir ? k : SEG - 1 - k;
                    const int cc = 1 + sg * SEG + o;
                    const BarT* b = rowp + cc + R;
                    const double gx = rd1 * (op(b[1]) - op(b[-1])) + rd2 * (op(b[2]) - op(b[-2])) +
                                      rK * (rr3 * (op(b[3]) - op(b[-3])) + rr4 * s);
                    double gxu = 0.0;
                    if (HYB)
                        gxu = rd1 * (opu(b[1]) - opu(b[-1])) + rd2 * (opu(b[2]) - opu(b[-2])) +
                              rK * (rr3 * (opu(b[3]) - opu(b[-3])) + rr4 * su);
                    Fx[r * BX + cc - 1] = force_from<FORCE>(b[0], gx, gxu, a.A);
                }
                // ring cells: x0-1 (backward lane of segment 0, ring cell r)
                // and x0+64 (forward lane of the last segment, ring cell TY+r)
                const double s = acc + __shfl_xor(pre, 1);
                double su = 0.0;
                if (HYB) su = accu + __shfl_xor(preu, 1);
                if (dir ? sg == 0 : sg == M::NSEG - 1) {
                    const int cc = dir ? 0 : CW - 1;
                    const BarT* b = rowp + cc + R;
                    const double gx = rd1 * (op(b[1]) - op(b[-1])) + rd2 * (op(b[2]) - op(b[-2])) +
                                      rK * (rr3 * (op(b[3]) - op(b[-3])) + rr4 * s);
                    double gxu = 0.0;
                    if (HYB)
                        gxu = rd1 * (opu(b[1]) - opu(b[-1])) + rd2 * (opu(b[2]) - opu(b[-2])) +
                              rK * (rr3 * (opu(b[3]) - opu(b[-3])) + rr4 * su);
                    FxR[dir ? r : TY + r] = force_from<FORCE>(b[0], gx, gxu, a.A);
                }
            }
        } else {
            // short x axis: the explicit periodic row, K outputs per lane
            const int xi = tid - M::XBASE;
            if (xi < TY * (BX / M::K)) {
                const int r = xi % TY, sg = xi / TY;
                const BarT* rowp = bar + bslot(yb + r) * RW;
                double acc[M::K], accu[M::K];
                stencil_window<FORCE, M::K, R>(rowp + 1 + sg * M::K, 1, ctab, acc, accu);
#pragma unroll
                for (int j = 0; j < M::K; ++j) {
                    const int cc = 1 + sg * M::K + j;
                    Fx[r * BX + cc - 1] = force_from<FORCE>(rowp[cc + R], acc[j], accu[j], a.A);
                }
            }
        }
        __syncthreads();

        // Phase 3: collision of the interior cells, two per lane, and of the
        // ring cells.
        if (!TOP_F) take_f();
        if (EARLY_F) {  // the next block's populations, in flight from here on
            __builtin_amdgcn_s_setprio(2);
            issue_f(yb + TY);
            __builtin_amdgcn_s_setprio(0);
        }
#pragma unroll
        for (int i = 0; i < M::NP; ++i) {
            const int t = tid + i * NT;
            if (t < M::NPAIR) {
                const int r = t >> 5, lx0 = 2 * (t & 31);
                const int ps = pslot(yb + r);
                double (&g)[2][Q] = gc[i];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int c = r * BX + lx0 + h;
                    double rho, jx, jy;
                    moments(g[h], rho, jx, jy);
                    collide(g[h], rho, jx, jy, Fx[c], Fy[c], a.omega);
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) {  // columns lx0+1, lx0+2 at post index lx0+2 (aligned pair)
                    V2 v;
                    v.x = (Real)g[0][q];
                    v.y = (Real)g[1][q];
                    *reinterpret_cast<V2*>(post + (q * PR + ps) * CWP + lx0 + 2) = v;
                }
            }
        }
        if (wave == 1 && lane < M::NRING) {  // the ring cells (columns x0-1, x0+64)
            double g9[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) g9[q] = (double)fring[lane * Q + q];
            double rho, jx, jy;
            moments(g9, rho, jx, jy);
            collide(g9, rho, jx, jy, FxR[lane], FyR[lane], a.omega);
            const int ps = pslot(yb + rrow);
#pragma unroll
            for (int q = 0; q < Q; ++q) post[(q * PR + ps) * CWP + ccol + 1] = (Real)g9[q];
        }
        __syncthreads();

        // Phase 4 begins by committing the loads of step 1 (the bar rows they
        // replace and the ring cells are not read again in this block; the
        // block sums are lane state), then loads the next block's populations
        // and streams.
        commit(yb + TY);
        commit_col();
        __builtin_amdgcn_sched_barrier(0);  // the commit's waits stay ahead of the new loads and stores
        if (!TOP_F && !EARLY_F) {  // (the raised priority is kept through this block's streaming stores)
            __builtin_amdgcn_s_setprio(2);
            issue_f(yb + TY);
        }

        // Pull streaming of rows yb-1 .. yb+TY-2 and phi_{t+1}.
#pragma unroll
        for (int i = 0; i < M::NP; ++i) {
            const int t = tid + i * NT;
            const int r = t >> 5, lx0 = 2 * (t & 31);
            const int y = yb - 1 + r, x = x0 + lx0;
            if (t < M::NPAIR && y >= ys && y < ye && x < nx) {
                double g[2][Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const Real* src = post + (q * PR + pslot(y - ey(q))) * CWP + lx0 + 2 - ex(q);
                    const Real v0 = src[0], v1 = src[1];
                    g[0][q] = (double)v0;
                    g[1][q] = (double)v1;
                    if (VEC) {
                        V2 v;
                        v.x = v0;
                        v.y = v1;
                        st_once<NTA>(v, reinterpret_cast<V2*>(a.f_out + fidx(x, y, q, nxb)));
                    } else {
                        st_once<NTA>(v0, a.f_out + fidx(x, y, q, nxb));
                        if (x + 1 < nx) st_once<NTA>(v1, a.f_out + fidx(x + 1, y, q, nxb));
                    }
                }
                double ph[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    double rho, jx, jy;
                    moments(g[h], rho, jx, jy);
                    ph[h] = phi_of<FORCE>(potential(a.eos, rho));
                }
                P* pd = phio + (long)y * pitch + x;
                if (VEC) {
                    P __attribute__((ext_vector_type(2))) pv;
                    pv.x = (P)ph[0];
                    pv.y = (P)ph[1];
                    st_once<NTA>(pv, reinterpret_cast<P __attribute__((ext_vector_type(2)))*>(pd));
                } else {
                    st_once<NTA>((P)ph[0], pd);
                    if (x + 1 < nx) st_once<NTA>((P)ph[1], pd + 1);
                }
            }
        }
        if (!TOP_F && !EARLY_F) __builtin_amdgcn_s_setprio(0);

        __syncthreads();
    }
}

// Rows per block and chunking constraints of the marching kernel: every row
// it touches must lie within one period of the chunk (ny > (NB + 2) TY + 3)
// besides the geometric form along y (ny > 2R + 1).
template <typename Real>
inline bool march_fits(int ny, int ty) {
    constexpr int R = Radius<Real>::value;
    const int nb = (R - 3 + ty - 1) / ty;
    return ny > 2 * R + 1 && ny > (nb + 2) * ty + 3;
}

// Launch over nchunk y chunks of every 64-column strip (nchunk in [1, ny]);
// paired 16/8-byte population accesses when N_x is even, plain (cached)
// population accesses when `cached` and N_x is even, else non-temporal.
template <typename Real, int FORCE, int TY>
inline void launch_march_t(const StepArgs<Real>& a, int nchunk, bool cached, hipStream_t s) {
    const dim3 grid((unsigned)(a.nxb * nchunk));
    if (a.nx % 2 != 0)
        hipLaunchKernelGGL((k_march<Real, FORCE, TY, false, true>), grid, dim3(NT), 0, s, a, nchunk);
    else if (cached)
        hipLaunchKernelGGL((k_march<Real, FORCE, TY, true, false>), grid, dim3(NT), 0, s, a, nchunk);
    else
        hipLaunchKernelGGL((k_march<Real, FORCE, TY, true, true>), grid, dim3(NT), 0, s, a, nchunk);
}

template <typename Real, int FORCE>
inline bool launch_march(const StepArgs<Real>& a, int ty, int nchunk, bool cached, hipStream_t s) {
    switch (ty) {
        case 4: launch_march_t<Real, FORCE, 4>(a, nchunk, cached, s); return true;
        case 8: launch_march_t<Real, FORCE, 8>(a, nchunk, cached, s); return true;
        default: return false;
    }
}

}  // namespace lbm

// Reverse-mode (adjoint) step of the HDM pseudopotential lattice Boltzmann
// step, FP64, Shan-Chen or Zhang-Chen force.  Every function here rounds each
// product (no contracted multiply-adds; explicit fma() calls excepted), so
// the instantiations of a kernel for different paths round alike and the
// paths agree bitwise.
//
// With the equilibrium in momentum form A_i(rho, m) = w_i [rho + 3 e.m +
// (4.5 (e.m)^2 - 1.5 |m|^2)/rho], one step is
//   f*_i = (1 - w) f_i + (w - 1) A_i(rho, j) + A_i(rho, j + F),  w = 1/tau,
//   f_{t+1,i}(x + e_i) = f*_i(x)                       (Eqs. 1, 2, 3, 10)
// and the force is F = -2 phi D|phi| (Eq. 22, phi = s Phi) or F = -D U
// (Eq. 7), D the circulant form of Eq. 20 along each axis.  Given
// lam = dJ/df_{t+1} (layout [9][ny][nx]) the adjoint is
//   mu_i(x)   = lam_i(x + e_i)
//   rho_bar   = sum_i mu_i [(w - 1) dA_i/drho(rho, j) + dA_i/drho(rho, j + F)]
//   j_bar     = sum_i mu_i [(w - 1) dA_i/dm(rho, j)   + dA_i/dm(rho, j + F)]
//   F_bar     = sum_i mu_i dA_i/dm(rho, j + F)
//   SC: U_bar = -(F_bar . D Phi)/Phi + s/(2 Phi) * (-D_x a_x - D_y a_y),  a = -2 phi F_bar
//   ZC: U_bar = D_x F_bar_x + D_y F_bar_y                 (D^T = -D)
//   dJ/df_k(x) = (1 - w) mu_k + rho_bar + e_k . j_bar + U_bar dU/drho
//   dJ/dg += sum U_bar dU/dg,   dJ/dT += sum U_bar dU/dT.
// Pass 1 (k_adj_local) does everything local to a cell and writes the planes
// a_x, a_y, U_bar_local and rho; pass 2 (k_adj_nonlocal) applies D to the a
// planes from an LDS cross, finishes U_bar and adds the density term.
// On a y axis longer than 2R + 1 both y derivatives are column marches
// instead (k_adj_dy, geometric form): one before pass 1 leaves D_y of the
// potential operand in the rho plane (pass 1 reads it at its own cell before
// storing rho there), one between the passes adds the D_y a_y term of U_bar
// to the U_bar_local plane, and the passes stage only their row bars.
#pragma once

#include "lbm_kernels.hpp"

namespace lbm {

// Constants of U = g (k p_EOS - rho/3) and its derivatives, unscaled by g so
// that dU/dg is available: U = g (c_rep rep(rho) - c_att att(rho) - rho/3),
// dU/dT = g (k R rep(rho) - c_attT att(rho)) with c_attT = k a alpha'(T).
struct AdjEos {
    int kind;
    double g, b, c_rep, c_att, c_attT, kR;
};

__device__ inline void eos_parts(int kind, double b, double rho, double& rep, double& drep, double& att, double& datt) {
#pragma clang fp contract(off)
    if (kind == EOS_CS) {
        const double eta = 0.25 * b * rho, om = 1.0 - eta;
        const double N = 1.0 + eta * (1.0 + eta * (1.0 - eta));
        const double Np = 1.0 + eta * (2.0 - 3.0 * eta);
        const double om3 = om * om * om;
        const double Z = N / om3, Zp = Np / om3 + 3.0 * N / (om3 * om);
        rep = rho * Z;
        drep = Z + eta * Zp;
        att = rho * rho;
        datt = 2.0 * rho;
        return;
    }
    const double ob = 1.0 - b * rho;
    rep = rho / ob;
    drep = 1.0 / (ob * ob);
    if (kind == EOS_PR) {
        const double q = 1.0 + b * rho * (2.0 - b * rho), qp = 2.0 * b * (1.0 - b * rho);
        att = rho * rho / q;
        datt = (2.0 * rho * q - rho * rho * qp) / (q * q);
    } else if (kind == EOS_RK || kind == EOS_RKS) {
        const double s = 1.0 + b * rho;
        att = rho * rho / s;
        datt = rho * (2.0 + b * rho) / (s * s);
    } else {
        att = rho * rho;
        datt = 2.0 * rho;
    }
}

__device__ inline void dA(int i, double ir, double mx, double my, double& dr, double& dmx, double& dmy) {
#pragma clang fp contract(off)
    const double em = double(ex(i)) * mx + double(ey(i)) * my;
    const double m2 = mx * mx + my * my;
    const double w = wq<double>(i);
    dr = w * (1.0 - (4.5 * em * em - 1.5 * m2) * ir * ir);
    dmx = w * (3.0 * double(ex(i)) + (9.0 * em * double(ex(i)) - 3.0 * mx) * ir);
    dmy = w * (3.0 * double(ey(i)) + (9.0 * em * double(ey(i)) - 3.0 * my) * ir);
}

// sum_{j=1..taps} c_j (op(base[j stride]) - op(base[-j stride])), in that
// order; unrolled when the line keeps the full radius J (every long axis).
template <int J, typename Op>
__device__ inline double dline(const double* __restrict__ c, const double* base, int stride, int taps, Op op) {
#pragma clang fp contract(off)
    double s = 0.0;
    if (taps == J) {
#pragma unroll
        for (int j = 1; j <= J; ++j) s = fma(c[j - 1], op(base[j * stride]) - op(base[-j * stride]), s);
    } else {
        for (int j = 1; j <= taps; ++j) s = fma(c[j - 1], op(base[j * stride]) - op(base[-j * stride]), s);
    }
    return s;
}

struct AdjArgs {
    StepArgs<double> s;             // f_in = state f_t, phi_in = phi(f_t), tables
    const double* __restrict__ lam_next;  // [9][ny][nx]
    double* __restrict__ lam;             // [9][ny][nx]
    double* __restrict__ ax;              // [ny][pitch]
    double* __restrict__ ay;
    double* __restrict__ ubl;             // U_bar local part
    double* __restrict__ rho;
    double* __restrict__ partial;         // [blocks][2]
    // Between the steps of one multi-step call the cotangent is kept as nine
    // planes plus one scalar plane c, lam_i = lam_local_i + c (the density
    // term, the same for all nine): the non-local pass writes c (add_out)
    // instead of adding it to the nine planes, the next step's local pass
    // adds it when it pulls lam_next (add_next).  Null: full planes.
    const double* __restrict__ add_next;  // [ny][nx]
    double* __restrict__ add_out;         // [ny][nx]
    int accumulate;                       // 1: add this step's partials to the stored ones
    AdjEos e;
};

// Column march of Eq. 20 along y in geometric form (the march kernel's y
// machinery without its LDS): one lane per lattice column, a workgroup takes
// four 64-column strips over one chunk of rows and walks down it in blocks of
// TY = 8 rows.  The lane keeps the window of rows yb-4 .. yb+TY+3 (operand
// values, op applied), the forward sum Lt and the block sums W_1 .. W_NB of
// the rows ahead in registers; per block it loads the window's TY new rows and
// the TY rows NB blocks ahead.  Differences, recursions and the Horner sum
// over the block sums are those of the march kernel (see stencil_recursive
// for the form).  Needs ny > 2R + 1 and ny > (NB + 2) TY + 3.
//   MODE 0: out = rho plane <- D_y op(phi)  (op = |.| for SC, identity for ZC)
//   MODE 1: U_bar_local plane += c D_y a_y, c = 1 (ZC) or -s / (2 Phi) (SC).
template <int FORCE, int MODE>
__global__ void __launch_bounds__(NT) k_adj_dy(AdjArgs A, int nchunk) {
#pragma clang fp contract(off)
    constexpr int R = Radius<double>::value, TY = 8;
    constexpr int NB = (R - 3 + TY - 1) / TY;
    const StepArgs<double>& a = A.s;
    const int strip = blockIdx.x * (NT / BX) + (int)(threadIdx.x >> 6);
    if (strip >= a.nxb) return;  // whole wavefronts; no barrier below
    const int xl = strip * BX + (int)(threadIdx.x & (BX - 1));
    const bool own = xl < a.nx;
    const int x = own ? xl : a.nx - 1;
    const int ny = a.ny, pitch = a.nxb * BX;
    const int ys = (int)((long)blockIdx.y * ny / nchunk), ye = (int)((long)(blockIdx.y + 1) * ny / nchunk);
    const double* __restrict__ src = MODE == 0 ? static_cast<const double*>(a.phi_in) : A.ay;
    // every row index below lies in [ys - R, ye + (NB + 2) TY + 3), within one period
    auto at = [&](int y) {
        const int yw = y < 0 ? y + ny : (y >= ny ? y - ny : y);
        const double v = src[plane_at(yw, x, pitch)];
        return (MODE == 0 && FORCE != FORCE_ZC) ? fabs(v) : v;
    };
    const double rr = a.rr, rr3 = a.rr3, rr4 = a.rr4, rd1 = a.rd1, rd2 = a.rd2, rK = a.rK;
    double rT = 1.0;
#pragma unroll
    for (int j = 0; j < TY; ++j) rT *= rr;
    // W = sum_n r^n t_n, t_n = r^4 (u_{n+1} - u_n) over the rows u0, p[0 .. TY-1]
    auto block_sum = [&](double u0, const double (&p)[TY]) {
        double w = 0.0;
#pragma unroll
        for (int n = TY - 1; n >= 0; --n) w = fma(rr, w, rr4 * (p[n] - (n == 0 ? u0 : p[n - 1])));
        return w;
    };
    // prologue: forward sum over rows ys-R .. ys-4, block sums of block 0
    // (rows ys+3+TY .. ys+3+(NB+1)TY), the window of block 0
    double l = 0.0;
    {
        double prev = at(ys - R);
#pragma unroll
        for (int m = 1; m <= R - 4; ++m) {
            const double u = at(ys - R + m);
            l = fma(rr, l, rr4 * (u - prev));
            prev = u;
        }
    }
    double W[NB];
    double uprev = at(ys + 3 + TY);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        double p[TY];
#pragma unroll
        for (int n = 0; n < TY; ++n) p[n] = at(ys + 3 + TY + j * TY + n + 1);
        W[j] = block_sum(uprev, p);
        uprev = p[TY - 1];
    }
    double win[TY + 8];
#pragma unroll
    for (int j = 0; j < TY + 8; ++j) win[j] = at(ys - 4 + j);

    for (int yb = ys; yb < ye; yb += TY) {
        // loads of the next block: its new window rows, the rows NB blocks ahead
        double nw[TY], far[TY];
#pragma unroll
        for (int j = 0; j < TY; ++j) nw[j] = at(yb + TY + 4 + j);
#pragma unroll
        for (int j = 0; j < TY; ++j) far[j] = at(yb + TY + 4 + NB * TY + j);
        // outputs of rows yb .. yb+TY-1
        double Lt[TY], g[TY];
#pragma unroll
        for (int o = 0; o < TY; ++o) {
            l = fma(rr, l, rr4 * (win[o + 1] - win[o]));
            Lt[o] = l;
        }
        double q = W[NB - 1];
#pragma unroll
        for (int j = NB - 2; j >= 0; --j) q = fma(rT, q, W[j]);
#pragma unroll
        for (int o = TY - 1; o >= 0; --o) {
            q = fma(rr, q, rr4 * (win[o + 8] - win[o + 7]));
            const int w = o + 4;
            g[o] = rd1 * (win[w + 1] - win[w - 1]) + rd2 * (win[w + 2] - win[w - 2]) +
                   rK * (rr3 * (win[w + 3] - win[w - 3]) + q + Lt[o]);
        }
        if (own) {
#pragma unroll
            for (int o = 0; o < TY; ++o) {
                const int y = yb + o;
                if (y < ye) {
                    const unsigned c = plane_at(y, x, pitch);
                    if (MODE == 0) {
                        A.rho[c] = g[o];
                    } else if (FORCE == FORCE_ZC) {
                        A.ubl[c] += g[o];
                    } else {
                        const double ph = static_cast<const double*>(a.phi_in)[c];
                        const double sgn = ph < 0.0 ? -1.0 : 1.0;
                        A.ubl[c] += sgn / (2.0 * fabs(ph)) * (-g[o]);
                    }
                }
            }
        }
        // advance: block sums, window
#pragma unroll
        for (int j = 0; j < NB - 1; ++j) W[j] = W[j + 1];
        W[NB - 1] = block_sum(uprev, far);
        uprev = far[TY - 1];
#pragma unroll
        for (int j = 0; j < 8; ++j) win[j] = win[j + TY];
#pragma unroll
        for (int j = 0; j < TY; ++j) win[8 + j] = nw[j];
    }
}

// Two bars staged with every load in flight at once (rows of WR and WC
// elements; src(r, c) as in stage_lds_rc).  The 4-row tiles of small
// lattices use it: there the reverse passes are latency-bound, and staging in
// batches of 8 loads per thread took three memory round trips per tile.
template <int NR, int WR, int NC, int WC, typename SrcR, typename SrcC>
__device__ inline void stage_two(double* __restrict__ dr, SrcR sr, double* __restrict__ dc, SrcC sc) {
#pragma clang fp contract(off)
    constexpr int PR = (NR + NT - 1) / NT, PC = (NC + NT - 1) / NT;
    const int tid = threadIdx.x;
    double vr[PR], vc[PC];
    {
        int r = tid / WR, c = tid - r * WR;
#pragma unroll
        for (int j = 0; j < PR; ++j) {
            if (tid + j * NT < NR) vr[j] = sr(r, c);
            r += NT / WR;
            c += NT % WR;
            if (c >= WR) {
                c -= WR;
                ++r;
            }
        }
    }
    {
        int r = tid / WC, c = tid - r * WC;
#pragma unroll
        for (int j = 0; j < PC; ++j) {
            if (tid + j * NT < NC) vc[j] = sc(r, c);
            r += NT / WC;
            c += NT % WC;
            if (c >= WC) {
                c -= WC;
                ++r;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < PR; ++j)
        if (tid + j * NT < NR) dr[tid + j * NT] = vr[j];
#pragma unroll
    for (int j = 0; j < PC; ++j)
        if (tid + j * NT < NC) dc[tid + j * NT] = vc[j];
}

// Row bar alone (the column march supplies the y derivatives).
template <int TY>
struct RowBar {
    static constexpr int J = Cross<double, TY>::J;
    static constexpr int RW = Cross<double, TY>::RW;
    double row[TY][RW];
};

// Pass 1: per 64 x TY tile, stage phi_t, recompute F and D Phi, pull lam_next,
// local adjoint of collision and force.  GY: D_y of the potential operand is
// read from the rho plane (k_adj_dy) and only the row bar is staged.  FIN:
// lam_next is in factored form (AdjArgs::add_next); FOUT (pass 2): write the
// density term to add_out instead of adding it to the nine planes.
template <int FORCE, int TY, bool GY = false, bool FIN = false>
__global__ void __launch_bounds__(NT) k_adj_local(AdjArgs A) {
#pragma clang fp contract(off)
    using Bars = typename std::conditional<GY, RowBar<TY>, Cross<double, TY>>::type;
    __shared__ Bars s;
    const StepArgs<double>& a = A.s;
    const int x0 = blockIdx.x * BX, y0 = blockIdx.y * TY;
    const int pitch = a.nxb * BX;
    const long n = (long)a.nx * a.ny;
    const int lx = threadIdx.x & (BX - 1), x = x0 + lx;
    // this thread's cells: rows r0, r0 + 4, ...  On 4-row tiles (one cell per
    // thread) its populations and cotangents are loaded before the staging, to
    // be in flight with it; on taller tiles that costs more than it hides
    // (1024^2: +11 %).  Lanes past the lattice load a valid duplicate and skip
    // the cell.
    const int r0 = threadIdx.x / BX, xc = min(x, a.nx - 1);
    auto load_cell = [&](int r, double (&f)[Q], double (&mu)[Q]) {
        const int y = min(y0 + r, a.ny - 1);
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = a.f_in[fidx(xc, y, i, a.nxb)];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int xs = xc + ex(i), ys = y + ey(i);
            xs = xs < 0 ? a.nx - 1 : (xs >= a.nx ? 0 : xs);
            ys = ys < 0 ? a.ny - 1 : (ys >= a.ny ? 0 : ys);
            mu[i] = A.lam_next[i * n + (long)ys * a.nx + xs];
            if constexpr (FIN) mu[i] += A.add_next[(long)ys * a.nx + xs];
        }
    };
    double f0[Q], mu0[Q];
    if constexpr (TY == 4) load_cell(r0, f0, mu0);
    const double* phi = static_cast<const double*>(a.phi_in);
    if constexpr (GY) {
        stage_lds_rc<TY * Bars::RW, Bars::RW, 8>(&s.row[0][0], [&](int r, int c) {
            return phi[plane_at(min(y0 + r, a.ny - 1), wrap_fast(x0 - Bars::J + c, a.nx), pitch)];
        });
    } else if constexpr (TY == 4) {
        using C = Cross<double, TY>;
        stage_two<TY * C::RW, C::RW, C::CH * BX, BX>(
            &s.row[0][0],
            [&](int r, int c) { return phi[plane_at(min(y0 + r, a.ny - 1), wrap_fast(x0 - C::J + c, a.nx), pitch)]; },
            &s.col[0][0],
            [&](int r, int c) { return phi[plane_at(wrap_fast(y0 - C::J + r, a.ny), min(x0 + c, a.nx - 1), pitch)]; });
    } else {
        stage_cross<double, TY>(s, phi, x0, y0, a.nx, a.ny, pitch);
    }
    __syncthreads();
    constexpr int J = Bars::J;
    for (int r = r0; r < TY; r += NT / BX) {
        const int y = y0 + r;
        if (y >= a.ny) break;
        const double pc = s.row[r][J + lx];
        auto opf = [](double v) { return FORCE == FORCE_ZC ? v : fabs(v); };
        const double gx = dline<J>(a.tab->dx, &s.row[r][J + lx], 1, a.tx, opf);
        double gy = 0.0;
        if constexpr (!GY) gy = dline<J>(a.tab->dy, &s.col[J + r][lx], BX, a.ty, opf);
        if (x >= a.nx) continue;
        if constexpr (GY) gy = A.rho[plane_at(y, x, pitch)];  // this cell's rho is stored there below
        const double Fx = FORCE == FORCE_ZC ? -gx : -2.0 * pc * gx;
        const double Fy = FORCE == FORCE_ZC ? -gy : -2.0 * pc * gy;
        double f[Q], mu[Q];
        if (TY == 4 && r == r0) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                f[i] = f0[i];
                mu[i] = mu0[i];
            }
        } else {
            load_cell(r, f, mu);
        }
        double rho, jx, jy;
        moments(f, rho, jx, jy);
        const double ir = 1.0 / rho, w = a.omega;
        const double mx = jx + Fx, my = jy + Fy;
        double rb = 0, jbx = 0, jby = 0, fbx = 0, fby = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            double ar, axx, ayy, br, bx, by;
            dA(i, ir, jx, jy, ar, axx, ayy);
            dA(i, ir, mx, my, br, bx, by);
            rb = fma(mu[i], fma(w - 1.0, ar, br), rb);
            jbx = fma(mu[i], fma(w - 1.0, axx, bx), jbx);
            jby = fma(mu[i], fma(w - 1.0, ayy, by), jby);
            fbx = fma(mu[i], bx, fbx);
            fby = fma(mu[i], by, fby);
        }
        const long o = (long)y * a.nx + x;
#pragma unroll
        for (int k = 0; k < Q; ++k) A.lam[k * n + o] = (1.0 - w) * mu[k] + rb + double(ex(k)) * jbx + double(ey(k)) * jby;
        const long op = (long)y * pitch + x;
        if (FORCE == FORCE_ZC) {
            A.ax[op] = fbx;
            A.ay[op] = fby;
            A.ubl[op] = 0.0;
        } else {
            const double Phi = fabs(pc);
            A.ax[op] = -2.0 * pc * fbx;
            A.ay[op] = -2.0 * pc * fby;
            A.ubl[op] = -(fbx * gx + fby * gy) / Phi;
        }
        A.rho[op] = rho;
    }
}

// Pass 2: D applied to the a planes (staged like phi), U_bar, density term,
// parameter partials per workgroup (fixed order).
template <int FORCE, int TY, bool GY = false, bool FOUT = false>
__global__ void __launch_bounds__(NT) k_adj_nonlocal(AdjArgs A) {
#pragma clang fp contract(off)
    using C = Cross<double, TY>;
    __shared__ double rowx[TY][C::RW];                 // row bar of a_x
    __shared__ double coly[GY ? 1 : C::CH][BX];        // column bar of a_y (GY: unused)
    __shared__ double red[2][NT / BX];
    const StepArgs<double>& a = A.s;
    const int x0 = blockIdx.x * BX, y0 = blockIdx.y * TY;
    const int pitch = a.nxb * BX;
    const long n = (long)a.nx * a.ny;
    auto ax_at = [&](int r, int c) { return A.ax[plane_at(min(y0 + r, a.ny - 1), wrap_fast(x0 - C::J + c, a.nx), pitch)]; };
    auto ay_at = [&](int r, int c) { return A.ay[plane_at(wrap_fast(y0 - C::J + r, a.ny), min(x0 + c, a.nx - 1), pitch)]; };
    if constexpr (!GY && TY == 4) {
        stage_two<TY * C::RW, C::RW, C::CH * BX, BX>(&rowx[0][0], ax_at, &coly[0][0], ay_at);
    } else {
        stage_lds_rc<TY * C::RW, C::RW, 8>(&rowx[0][0], ax_at);
        if constexpr (!GY) stage_lds_rc<C::CH * BX, BX, 8>(&coly[0][0], ay_at);
    }
    __syncthreads();
    constexpr int J = C::J;
    const int lx = threadIdx.x & (BX - 1), x = x0 + lx;
    double sg = 0.0, sT = 0.0;
    for (int r = threadIdx.x / BX; r < TY; r += NT / BX) {
        const int y = y0 + r;
        if (y >= a.ny) break;
        auto id = [](double v) { return v; };
        const double dxa = dline<J>(a.tab->dx, &rowx[r][J + lx], 1, a.tx, id);
        const double dya = GY ? 0.0 : dline<J>(a.tab->dy, &coly[(GY ? 0 : J + r)][lx], BX, a.ty, id);
        if (x >= a.nx) continue;
        const long op = (long)y * pitch + x;
        double ub;
        if (GY) {  // the D_y term is already in the U_bar_local plane (k_adj_dy)
            if (FORCE == FORCE_ZC) {
                ub = A.ubl[op] + dxa;
            } else {
                const double ph = static_cast<const double*>(a.phi_in)[op];
                const double sgn = ph < 0.0 ? -1.0 : 1.0;
                ub = A.ubl[op] + sgn / (2.0 * fabs(ph)) * (-dxa);
            }
        } else if (FORCE == FORCE_ZC) {
            ub = dxa + dya;
        } else {
            const double ph = static_cast<const double*>(a.phi_in)[op];
            const double sgn = ph < 0.0 ? -1.0 : 1.0;
            ub = A.ubl[op] + sgn / (2.0 * fabs(ph)) * (-dxa - dya);
        }
        const double rho = A.rho[op];
        double rep, drep, att, datt;
        eos_parts(A.e.kind, A.e.b, rho, rep, drep, att, datt);
        const double dUdrho = A.e.g * (A.e.c_rep * drep - A.e.c_att * datt - 1.0 / 3.0);
        const double dUdg = A.e.c_rep * rep - A.e.c_att * att - rho / 3.0;
        const double dUdT = A.e.g * (A.e.kR * rep - A.e.c_attT * att);
        // the density term is rounded before it is added (no fused multiply-add),
        // so the factored and the full form of the cotangent agree bitwise
        const double add = __dmul_rn(ub, dUdrho);
        const long o = (long)y * a.nx + x;
        if constexpr (FOUT) {
            A.add_out[o] = add;
        } else {
#pragma unroll
            for (int k = 0; k < Q; ++k) A.lam[k * n + o] += add;
        }
        sg += ub * dUdg;
        sT += ub * dUdT;
    }
    sg = wave_sum(sg);
    sT = wave_sum(sT);
    const int w = threadIdx.x / BX;
    if ((threadIdx.x & (BX - 1)) == 0) { red[0][w] = sg; red[1][w] = sT; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0, t1 = 0;
        for (int k = 0; k < NT / BX; ++k) { t0 += red[0][k]; t1 += red[1][k]; }
        const long b = (long)blockIdx.y * gridDim.x + blockIdx.x;
        if (A.accumulate) {  // step after step, in a fixed order per block
            t0 += A.partial[2 * b];
            t1 += A.partial[2 * b + 1];
        }
        A.partial[2 * b] = t0;
        A.partial[2 * b + 1] = t1;
    }
}

// grad[0..1] += fixed-order sums of the pass-2 partials (one workgroup).
static __global__ void __launch_bounds__(NT) k_adj_accumulate(const double* __restrict__ partial, long nblocks,
                                                       double* __restrict__ grad) {
#pragma clang fp contract(off)
    __shared__ double red[2][NT / BX];
    double t0 = 0, t1 = 0;
    for (long b = threadIdx.x; b < nblocks; b += NT) { t0 += partial[2 * b]; t1 += partial[2 * b + 1]; }
    t0 = wave_sum(t0);
    t1 = wave_sum(t1);
    const int w = threadIdx.x / BX;
    if ((threadIdx.x & (BX - 1)) == 0) { red[0][w] = t0; red[1][w] = t1; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s1 = 0;
        for (int k = 0; k < NT / BX; ++k) { s0 += red[0][k]; s1 += red[1][k]; }
        grad[0] += s0;
        grad[1] += s1;
    }
}

// dJ/drho0 = sum_i lam0_i f^eq_i(rho0, u0) / rho0 (f^eq is linear in rho at fixed u).
static __global__ void __launch_bounds__(NT) k_adj_rho0(const double* __restrict__ lam0,
                                                 const double* __restrict__ ux0, const double* __restrict__ uy0,
                                                 long n, double* __restrict__ out) {
#pragma clang fp contract(off)
    for (long c = blockIdx.x * (long)NT + threadIdx.x; c < n; c += (long)gridDim.x * NT) {
        const double ux = ux0 ? ux0[c] : 0.0, uy = uy0 ? uy0[c] : 0.0;
        const double usq = ux * ux + uy * uy;
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) acc += lam0[i * n + c] * feq(i, 1.0, ux, uy, usq);
        out[c] = acc;
    }
}

}  // namespace lbm

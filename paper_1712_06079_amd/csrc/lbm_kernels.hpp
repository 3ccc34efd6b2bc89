// HIP kernels of the HDM pseudopotential lattice Boltzmann step (gfx950).
//
//   k_init       f = f^eq(rho0, u0) and the potential field of that state
//   k_phi        potential field phi(rho(f)) of a state
//   k_collide    two-pass reference step: HDM force from the staged phi cross,
//                EDM-BGK collision, push streaming (phi refreshed by k_phi)
//   k_fused      single-pass step (lbm_fused.hpp)
//   k_moments    rho, half-step velocity, bulk pressure + per-block partials
//   k_totals     fixed-order reduction of the partials
//   k_get_f / k_set_f  conversion to and from the documented [9][ny][nx] FP64 layout
#pragma once

#include "lbm_device.hpp"

namespace lbm {

constexpr int NT = 256;  // threads per workgroup (four wavefronts)

// ------------------------------------------------------------------ init / phi
template <typename Real, int FORCE>
__global__ void __launch_bounds__(NT) k_init(StepArgs<Real> a, const double* __restrict__ rho0,
                                             const double* __restrict__ ux0, const double* __restrict__ uy0) {
    using P = typename PhiStore<Real, FORCE>::type;
    P* __restrict__ phio = static_cast<P*>(a.phi_out);
    const int pitch = a.nxb * BX;
    const long total = (long)pitch * a.ny;
    for (long c = blockIdx.x * (long)NT + threadIdx.x; c < total; c += (long)gridDim.x * NT) {
        int y = (int)(c / pitch), x = (int)(c - (long)y * pitch);
        Real* f = a.f_out;
        if (x < a.nx) {
            long s = (long)y * a.nx + x;
            double rho = rho0[s];
            double ux = ux0 ? ux0[s] : 0.0, uy = uy0 ? uy0[s] : 0.0;
            double usq = ux * ux + uy * uy;
            double fi[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const Real v = (Real)feq(i, rho, ux, uy, usq);
                f[fidx(x, y, i, a.nxb)] = v;
                fi[i] = (double)v;  // the stored value defines the state
            }
            double r, jx, jy;
            moments(fi, r, jx, jy);
            phio[(long)y * pitch + x] = (P)phi_of<FORCE>(potential(a.eos, r));
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) f[fidx(x, y, i, a.nxb)] = Real(0);
            phio[(long)y * pitch + x] = P(0);
        }
    }
}

template <typename Real, int FORCE>
__global__ void __launch_bounds__(NT) k_phi(StepArgs<Real> a) {
    using P = typename PhiStore<Real, FORCE>::type;
    P* __restrict__ phio = static_cast<P*>(a.phi_out);
    const int pitch = a.nxb * BX;
    const long total = (long)pitch * a.ny;
    for (long c = blockIdx.x * (long)NT + threadIdx.x; c < total; c += (long)gridDim.x * NT) {
        int y = (int)(c / pitch), x = (int)(c - (long)y * pitch);
        if (x >= a.nx) continue;
        double fi[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) fi[i] = (double)a.f_in[fidx(x, y, i, a.nxb)];
        double r, jx, jy;
        moments(fi, r, jx, jy);
        phio[(long)y * pitch + x] = (P)phi_of<FORCE>(potential(a.eos, r));
    }
}

// ------------------------------------------------------------------ phi cross
// A 64 x TY tile stages the potential field over its rows widened by +-J in x
// (for d/dx) and over its columns widened by +-J in y (for d/dy), with
// periodic wrap.  Rows or columns outside the lattice (ragged tiles) are
// clamped; they feed only cells that are never written.
template <typename Real, int TY>
struct Cross {
    static constexpr int J = Radius<Real>::value;
    static constexpr int RW = BX + 2 * J;
    static constexpr int CH = TY + 2 * J;
    double row[TY][RW];
    double col[CH][BX];
};

// Workgroup copy dst[i] = src(i), i in [0, N), where src(i) reads global
// memory.  Each thread takes the elements i = tid + j NT and issues the loads of
// B of them before the first LDS store, so the loads are in flight together
// instead of one global-memory latency per element.
template <int N>
struct StageRegs {
    static constexpr int PER = (N + NT - 1) / NT;
    double v[PER];
};

// Split form of the copy: stage_issue loads every element of thread tid
// into registers, stage_commit stores them, so other loads (issued after
// stage_issue) do not delay the wait before the LDS stores.
template <int N, typename Src>
__device__ inline void stage_issue(StageRegs<N>& s, int tid, Src src) {
#pragma unroll
    for (int j = 0; j < StageRegs<N>::PER; ++j) {
        // past the end: reload the last element (kept unconditional so the
        // loads form one straight-line batch; the duplicate is not stored)
        const int i = min(tid + j * NT, N - 1);
        s.v[j] = src(i);
    }
}

// stage_issue over an array of rows of W elements: src(r, c) receives the
// row and column of element i = tid + j NT, advanced from one division per
// call (the per-element quotient would take a high multiply per load).
template <int N, int W, typename Src>
__device__ inline void stage_issue_rc(StageRegs<N>& s, int tid, Src src) {
    constexpr int LR = (N - 1) / W, LC = (N - 1) - LR * W;  // the last element
    constexpr int DR = NT / W, DC = NT - DR * W;             // one step of NT
    int r = tid / W, c = tid - r * W;
#pragma unroll
    for (int j = 0; j < StageRegs<N>::PER; ++j) {
        // past the end: reload the last element (not stored)
        const bool in = tid + j * NT < N;
        s.v[j] = src(in ? r : LR, in ? c : LC);
        r += DR;
        c += DC;
        if (c >= W) {
            c -= W;
            ++r;
        }
    }
}

template <int N>
__device__ inline void stage_commit(double* __restrict__ dst, int tid, const StageRegs<N>& s) {
#pragma unroll
    for (int j = 0; j < StageRegs<N>::PER; ++j) {
        const int i = tid + j * NT;
        if (i < N) dst[i] = s.v[j];
    }
}

template <int N, int B, typename Src>
__device__ inline void stage_lds(double* __restrict__ dst, Src src) {
    constexpr int PER = (N + NT - 1) / NT;
    const int tid = threadIdx.x;
#pragma unroll
    for (int j0 = 0; j0 < PER; j0 += B) {
        double v[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int i = tid + (j0 + j) * NT;
            if (j0 + j < PER && i < N) v[j] = src(i);
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int i = tid + (j0 + j) * NT;
            if (j0 + j < PER && i < N) dst[i] = v[j];
        }
    }
}

// stage_lds over an array of rows of W elements: src(r, c) receives the row
// and column of element i, stepped from one division per call.
template <int N, int W, int B, typename Src>
__device__ inline void stage_lds_rc(double* __restrict__ dst, Src src) {
    constexpr int PER = (N + NT - 1) / NT;
    constexpr int DR = NT / W, DC = NT - DR * W;
    const int tid = threadIdx.x;
    int r = tid / W, c = tid - r * W;
#pragma unroll
    for (int j0 = 0; j0 < PER; j0 += B) {
        double v[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            if (j0 + j < PER && tid + (j0 + j) * NT < N) v[j] = src(r, c);
            r += DR;
            c += DC;
            if (c >= W) {
                c -= W;
                ++r;
            }
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int i = tid + (j0 + j) * NT;
            if (j0 + j < PER && i < N) dst[i] = v[j];
        }
    }
}

// Offset of lattice cell (x, y) in a potential or scratch plane of row pitch
// `pitch` (fewer than 2^31 elements; sides at most 2^21, so 24-bit products).
__device__ inline unsigned plane_at(int y, int x, int pitch) { return (unsigned)(__mul24(y, pitch) + x); }

template <typename Real, int TY, typename P>
__device__ inline void stage_cross(Cross<Real, TY>& s, const P* __restrict__ phi, int x0, int y0, int nx,
                                   int ny, int pitch, int walls = 0) {
    using C = Cross<Real, TY>;
    stage_lds_rc<TY * C::RW, C::RW, 8>(&s.row[0][0], [&](int r, int c) {
        return (double)phi[plane_at(min(y0 + r, ny - 1), wrap_fast(x0 - C::J + c, nx), pitch)];
    });
    stage_lds_rc<C::CH * BX, BX, 8>(&s.col[0][0], [&](int r, int c) {
        return (double)phi[plane_at(ymap_fast(y0 - C::J + r, ny, walls), min(x0 + c, nx - 1), pitch)];
    });
}

// Interaction force at tile cell (r, lx) from the staged cross (double arithmetic):
//  SC (Eq. 22): F = -2 s Phi D Phi = -2 phi(x) D|phi|
//  ZC (Eq. 7):  F = -D U
//  hybrid (Eq. 9): A F^ZC + (1 - 2A) F^SC with U = phi |phi|.
// The 3 x 3 neighbourhoods of a 64 x TY tile for Eq. 15: rows y0-1 .. y0+TY,
// columns x0-1 .. x0+64, periodic.
template <int TY>
struct Block9 {
    static constexpr int W = BX + 2;
    double v[TY + 2][W];
};

template <int TY, typename P>
__device__ inline void stage_block9(Block9<TY>& b, const P* __restrict__ phi, int x0, int y0, int nx, int ny, int pitch) {
    stage_lds_rc<(TY + 2) * Block9<TY>::W, Block9<TY>::W, 8>(&b.v[0][0], [&](int r, int c) {
        return (double)phi[plane_at(wrap_fast(y0 - 1 + r, ny), wrap_fast(x0 - 1 + c, nx), pitch)];
    });
}

template <typename Real, int FORCE, int TY>
__device__ inline void force_at(const Cross<Real, TY>& s, const StepArgs<Real>& a, int r, int lx, double& Fx, double& Fy,
                                const Block9<TY>* b9 = nullptr) {
    constexpr int J = Cross<Real, TY>::J;
    const double pc = s.row[r][J + lx];
    if (a.grad9) {  // Eq. 15 over the neighbourhood (b9 staged when grad9)
        auto op = [](double v) { return FORCE == FORCE_ZC ? v : fabs(v); };
        double m[3], c[3], p[3], mu[3], cu[3], pu[3];
        for (int k = 0; k < 3; ++k) {
            m[k] = op(b9->v[r][lx + k]);
            c[k] = op(b9->v[r + 1][lx + k]);
            p[k] = op(b9->v[r + 2][lx + k]);
            mu[k] = b9->v[r][lx + k] * fabs(b9->v[r][lx + k]);
            cu[k] = b9->v[r + 1][lx + k] * fabs(b9->v[r + 1][lx + k]);
            pu[k] = b9->v[r + 2][lx + k] * fabs(b9->v[r + 2][lx + k]);
        }
        double gx, gy, gxu = 0.0, gyu = 0.0;
        grad_d2q9(m, c, p, gx, gy);
        if (FORCE == FORCE_HYBRID) grad_d2q9(mu, cu, pu, gxu, gyu);
        if (FORCE == FORCE_ZC) {
            Fx = -gx;
            Fy = -gy;
        } else {
            Fx = -2.0 * pc * gx;
            Fy = -2.0 * pc * gy;
            if (FORCE == FORCE_HYBRID) {
                Fx = a.A * (-gxu) + (1.0 - 2.0 * a.A) * Fx;
                Fy = a.A * (-gyu) + (1.0 - 2.0 * a.A) * Fy;
            }
        }
        return;
    }
    if (FORCE == FORCE_ZC) {
        double gx = 0, gy = 0;
        for (int j = 1; j <= a.tx; ++j) gx += a.tab->dx[j - 1] * (s.row[r][J + lx + j] - s.row[r][J + lx - j]);
        for (int j = 1; j <= a.ty; ++j) gy += a.tab->dy[j - 1] * (s.col[J + r + j][lx] - s.col[J + r - j][lx]);
        Fx = -gx;
        Fy = -gy;
    } else {
        double gx = 0, gy = 0, ux = 0, uy = 0;
        for (int j = 1; j <= a.tx; ++j) {
            const double p = s.row[r][J + lx + j], m = s.row[r][J + lx - j];
            gx += a.tab->dx[j - 1] * (fabs(p) - fabs(m));
            if (FORCE == FORCE_HYBRID) ux += a.tab->dx[j - 1] * (p * fabs(p) - m * fabs(m));
        }
        for (int j = 1; j <= a.ty; ++j) {
            const double p = s.col[J + r + j][lx], m = s.col[J + r - j][lx];
            gy += a.tab->dy[j - 1] * (fabs(p) - fabs(m));
            if (FORCE == FORCE_HYBRID) uy += a.tab->dy[j - 1] * (p * fabs(p) - m * fabs(m));
        }
        Fx = -2.0 * pc * gx;
        Fy = -2.0 * pc * gy;
        if (FORCE == FORCE_HYBRID) {
            Fx = a.A * (-ux) + (1.0 - 2.0 * a.A) * Fx;
            Fy = a.A * (-uy) + (1.0 - 2.0 * a.A) * Fy;
        }
    }
}

// ------------------------------------------------------------------ two-pass reference step
// Pass 2 of the reference step: per tile, stage phi_t, compute the force,
// collide and push every population to its downstream neighbour in f_out.
template <typename Real, int FORCE, int TY>
__global__ void __launch_bounds__(NT) k_collide(StepArgs<Real> a) {
    __shared__ Cross<Real, TY> s;
    __shared__ Block9<TY> b9;
    const int x0 = blockIdx.x * BX, y0 = blockIdx.y * TY;
    const int pitch = a.nxb * BX;
    const auto* phin = static_cast<const typename PhiStore<Real, FORCE>::type*>(a.phi_in);
    stage_cross<Real, TY>(s, phin, x0, y0, a.nx, a.ny, pitch);
    if (a.grad9) stage_block9<TY>(b9, phin, x0, y0, a.nx, a.ny, pitch);
    __syncthreads();
    const int lx = threadIdx.x & (BX - 1), x = x0 + lx;
    for (int r = threadIdx.x / BX; r < TY; r += NT / BX) {
        const int y = y0 + r;
        if (y >= a.ny) break;
        double Fx, Fy;
        force_at<Real, FORCE, TY>(s, a, r, lx, Fx, Fy, &b9);
        if (x >= a.nx) continue;
        double f[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = (double)a.f_in[fidx(x, y, i, a.nxb)];
        double rho, jx, jy;
        moments(f, rho, jx, jy);
        collide(f, rho, jx, jy, Fx, Fy, a.omega);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int xd = x + ex(i), yd = y + ey(i);
            xd = xd < 0 ? a.nx - 1 : (xd >= a.nx ? 0 : xd);
            yd = yd < 0 ? a.ny - 1 : (yd >= a.ny ? 0 : yd);
            a.f_out[fidx(xd, yd, i, a.nxb)] = (Real)f[i];
        }
    }
}

// ------------------------------------------------------------------ moments
// Output moments (Eq. 3, Eq. 11, p = rho/3 + U) and per-workgroup partials
// {sum rho, sum rho v_x, sum rho v_y, max |v|} accumulated in FP64 in a fixed
// order (wavefront butterfly, then the four wavefronts in index order).
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// max that keeps a NaN (fmax would drop it and report the largest finite
// speed of a field that has gone non-finite)
__device__ inline double nanmax(double a, double b) { return (a != a || b != b) ? a + b : fmax(a, b); }

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = nanmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <typename Real, int FORCE, int TY>
__global__ void __launch_bounds__(NT) k_moments(StepArgs<Real> a, double* __restrict__ rho_o, double* __restrict__ ux_o,
                                                double* __restrict__ uy_o, double* __restrict__ p_o,
                                                double* __restrict__ partial) {
    __shared__ Cross<Real, TY> s;
    __shared__ double red[4][NT / BX];
    __shared__ Block9<TY> b9;
    const int x0 = blockIdx.x * BX, y0 = blockIdx.y * TY;
    const int pitch = a.nxb * BX;
    const auto* phin = static_cast<const typename PhiStore<Real, FORCE>::type*>(a.phi_in);
    stage_cross<Real, TY>(s, phin, x0, y0, a.nx, a.ny, pitch, a.walls);
    if (a.grad9) stage_block9<TY>(b9, phin, x0, y0, a.nx, a.ny, pitch);
    __syncthreads();
    const int lx = threadIdx.x & (BX - 1), x = x0 + lx;
    double m = 0, px = 0, py = 0, vmax = 0;
    for (int r = threadIdx.x / BX; r < TY; r += NT / BX) {
        const int y = y0 + r;
        if (y >= a.ny) break;
        double Fx, Fy;
        force_at<Real, FORCE, TY>(s, a, r, lx, Fx, Fy, &b9);
        if (x >= a.nx) continue;
        double f[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = (double)a.f_in[fidx(x, y, i, a.nxb)];
        double rho, jx, jy;
        moments(f, rho, jx, jy);
        double dr = rho;
        double vx = (jx + 0.5 * Fx) / dr;
        double vy = (jy + 0.5 * Fy) / dr;
        long o = (long)y * a.nx + x;
        if (rho_o) rho_o[o] = dr;
        if (ux_o) ux_o[o] = vx;
        if (uy_o) uy_o[o] = vy;
        if (p_o) p_o[o] = dr / 3.0 + potential(a.eos, rho);
        m += dr;
        px += dr * vx;
        py += dr * vy;
        vmax = nanmax(vmax, sqrt(vx * vx + vy * vy));
    }
    m = wave_sum(m);
    px = wave_sum(px);
    py = wave_sum(py);
    vmax = wave_max(vmax);
    const int w = threadIdx.x / BX;
    if ((threadIdx.x & (BX - 1)) == 0) {
        red[0][w] = m; red[1][w] = px; red[2][w] = py; red[3][w] = vmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0, t1 = 0, t2 = 0, t3 = 0;
        for (int k = 0; k < NT / BX; ++k) {
            t0 += red[0][k]; t1 += red[1][k]; t2 += red[2][k]; t3 = nanmax(t3, red[3][k]);
        }
        long b = (long)blockIdx.y * gridDim.x + blockIdx.x;
        partial[4 * b + 0] = t0;
        partial[4 * b + 1] = t1;
        partial[4 * b + 2] = t2;
        partial[4 * b + 3] = t3;
    }
}

// One workgroup: thread t sums partials t, t + 256, ... in order, then a fixed
// butterfly and the four wavefronts in index order.
static __global__ void __launch_bounds__(NT) __attribute__((unused)) k_totals(const double* __restrict__ partial, long nblocks, double* __restrict__ out) {
    __shared__ double red[4][NT / BX];
    double t0 = 0, t1 = 0, t2 = 0, t3 = 0;
    for (long b = threadIdx.x; b < nblocks; b += NT) {
        t0 += partial[4 * b + 0]; t1 += partial[4 * b + 1]; t2 += partial[4 * b + 2];
        t3 = nanmax(t3, partial[4 * b + 3]);
    }
    t0 = wave_sum(t0); t1 = wave_sum(t1); t2 = wave_sum(t2); t3 = wave_max(t3);
    const int w = threadIdx.x / BX;
    if ((threadIdx.x & (BX - 1)) == 0) { red[0][w] = t0; red[1][w] = t1; red[2][w] = t2; red[3][w] = t3; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        for (int k = 0; k < NT / BX; ++k) { s0 += red[0][k]; s1 += red[1][k]; s2 += red[2][k]; s3 = nanmax(s3, red[3][k]); }
        out[0] = s0; out[1] = s1; out[2] = s2; out[3] = s3;
    }
}

// ------------------------------------------------------------------ layout conversion
template <typename Real>
__global__ void __launch_bounds__(NT) k_get_f(StepArgs<Real> a, double* __restrict__ out) {
    const long n = (long)a.nx * a.ny;
    for (long c = blockIdx.x * (long)NT + threadIdx.x; c < n; c += (long)gridDim.x * NT) {
        int y = (int)(c / a.nx), x = (int)(c - (long)y * a.nx);
#pragma unroll
        for (int i = 0; i < Q; ++i) out[i * n + c] = (double)a.f_in[fidx(x, y, i, a.nxb)];
    }
}

template <typename Real>
__global__ void __launch_bounds__(NT) k_set_f(StepArgs<Real> a, const double* __restrict__ in) {
    const long n = (long)a.nx * a.ny;
    for (long c = blockIdx.x * (long)NT + threadIdx.x; c < n; c += (long)gridDim.x * NT) {
        int y = (int)(c / a.nx), x = (int)(c - (long)y * a.nx);
#pragma unroll
        for (int i = 0; i < Q; ++i) a.f_out[fidx(x, y, i, a.nxb)] = (Real)in[i * n + c];
    }
}

// Validation of an initial density: flag[0] = 1 if any rho0 is non-finite,
// <= 0 or at / beyond the pole of the repulsive term.
static __global__ void __launch_bounds__(NT) __attribute__((unused)) k_check_rho0(const double* __restrict__ rho0, long n, double rho_max,
                                                   int* __restrict__ flag) {
    int bad = 0;
    for (long c = blockIdx.x * (long)NT + threadIdx.x; c < n; c += (long)gridDim.x * NT) {
        double r = rho0[c];
        if (!(r > 0.0) || !(r < rho_max) || !isfinite(r)) bad = 1;
    }
    if (bad) atomicOr(flag, 1);
}

}  // namespace lbm

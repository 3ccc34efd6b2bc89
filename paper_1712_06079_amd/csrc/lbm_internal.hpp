// Internal shared state of the library's translation units (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstring>
#include <type_traits>

#include "../../include/lbm.h"
#include "hdm_coeffs.hpp"
#include "lbm_device.hpp"
#include "lbm_kernels.hpp"

// Host state of one domain: parameters, planned constants, coefficient rows and
// the layout of its caller-owned workspace.
struct lbm_domain {
    lbm_params p;
    double Tc, rhoc, alpha;
    int nxb, pitch;
    int cur;           // index of the buffer pair holding the current state
    int64_t steps;
    int variant;       // 0 fused (automatic), 1 two-pass reference, 2 fused tiles, 3 fused march
    int tile_y;        // rows per tile or marching block (0 = default)
    int chunks;        // y chunks per strip of the marching kernel (0 = automatic)
    int access;        // marching kernel's population accesses: 0 automatic, 1 non-temporal, 2 plain
    int ncu;           // compute units of the device
    int march_occ[2];  // resident marching workgroups per CU (block rows 4, 8; 0 = not queried)
    int fused_occ[3];  // resident tile-kernel workgroups per CU (tile rows 4, 8, 16; 0 = not queried)
    char* ws;
    size_t ws_bytes;
    size_t off_f[2], off_phi[2], off_part, off_scr, off_tab;
    lbm::StepTables htab;  // host copy of the device tables (source of their upload)
    int tx, ty;
    double dx[lbm::JCAP], dy[lbm::JCAP];
};

namespace lbm_internal {

// Record a failure message (thread-local) and return the status.
lbm_status fail(lbm_status s, const char* fmt, ...);

#define HIP_TRY(expr)                                                                                \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return lbm_internal::fail(LBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

inline unsigned grid_1d(long n) {
    long b = (n + lbm::NT - 1) / lbm::NT;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// Bytes per site of a domain's potential field (lbm::PhiStore: FP32 for FP32
// populations with the Shan-Chen or Zhang-Chen force, otherwise FP64).
inline size_t phi_elem_bytes(const lbm_params* p) {
    return (p->prec == LBM_F32 && p->force != LBM_FORCE_HYBRID) ? 4 : 8;
}

// Kernel arguments of one step of domain d reading buffer in_buf, writing out_buf.
template <typename Real>
lbm::StepArgs<Real> make_args(const lbm_domain* d, int in_buf, int out_buf) {
    lbm::StepArgs<Real> a;
    std::memset(&a, 0, sizeof(a));
    a.f_in = reinterpret_cast<const Real*>(d->ws + d->off_f[in_buf]);
    a.f_out = reinterpret_cast<Real*>(d->ws + d->off_f[out_buf]);
    a.phi_in = d->ws + d->off_phi[in_buf];
    a.phi_out = d->ws + d->off_phi[out_buf];
    a.nx = d->p.nx;
    a.ny = d->p.ny;
    a.nxb = d->nxb;
    a.tx = d->tx;
    a.ty = d->ty;
    a.omega = 1.0 / d->p.tau;
    a.A = d->p.A;
    const double g = d->p.g, k = d->p.k;
    a.eos.kind = d->p.eos;
    a.eos.c_rep = g * k * d->p.R * d->p.T;
    a.eos.c_att = g * k * d->p.a * d->alpha;
    a.eos.c_lin = g / 3.0;
    a.eos.b = d->p.b;
    a.tab = reinterpret_cast<const lbm::StepTables*>(d->ws + d->off_tab);
    // geometric recursion along axes longer than 2R + 1 (HDM only)
    const int R = lbm::Radius<Real>::value;
    a.rec_x = (d->p.grad == LBM_GRAD_HDM && d->p.nx > 2 * R + 1) ? 1 : 0;
    // (between walls the y lines continue by reflection: period 2 ny)
    a.rec_y = (d->p.grad == LBM_GRAD_HDM && (d->p.walls ? 2 * d->p.ny : d->p.ny) > 2 * R + 1) ? 1 : 0;
    double C = 0.0;
    lbm_host::hdm_infinite(&a.rr, &a.rd1, &a.rd2, &C);
    a.rr3 = a.rr * a.rr * a.rr;
    a.rr4 = a.rr3 * a.rr;
    a.rK = C / (1.0 - a.rr);
    a.grad9 = d->p.grad == LBM_GRAD_CDM9 ? 1 : 0;
    a.walls = d->p.walls ? 1 : 0;
    return a;
}

// Fill d->htab from the one-sided rows d->dx, d->dy (taps d->tx, d->ty).
inline void build_tables(lbm_domain* d) {
    std::memset(&d->htab, 0, sizeof(d->htab));
    for (int j = 0; j < lbm::JCAP; ++j) {
        d->htab.dx[j] = d->dx[j];
        d->htab.dy[j] = d->dy[j];
    }
    for (int i = 0; i < lbm::TAB; ++i) {
        const int n = i - lbm::TAB_OFF, an = n < 0 ? -n : n;
        d->htab.tx_tab[i] = (an >= 1 && an <= d->tx) ? (n > 0 ? d->dx[an - 1] : -d->dx[an - 1]) : 0.0;
        d->htab.ty_tab[i] = (an >= 1 && an <= d->ty) ? (n > 0 ? d->dy[an - 1] : -d->dy[an - 1]) : 0.0;
    }
}

// Call fn(Real{}, integral_constant<FORCE>) for the compile-time types of d.
template <typename Fn>
void dispatch(const lbm_domain* d, Fn&& fn) {
    const bool f32 = d->p.prec == LBM_F32;
    switch (d->p.force) {
        case LBM_FORCE_SC:
            if (f32) fn((float)0, std::integral_constant<int, lbm::FORCE_SC>());
            else fn((double)0, std::integral_constant<int, lbm::FORCE_SC>());
            break;
        case LBM_FORCE_ZC:
            if (f32) fn((float)0, std::integral_constant<int, lbm::FORCE_ZC>());
            else fn((double)0, std::integral_constant<int, lbm::FORCE_ZC>());
            break;
        default:
            if (f32) fn((float)0, std::integral_constant<int, lbm::FORCE_HYBRID>());
            else fn((double)0, std::integral_constant<int, lbm::FORCE_HYBRID>());
    }
}

// Rebuild the potential field of buffer `buf` from its populations.
lbm_status launch_phi(lbm_domain* d, int buf, hipStream_t s);

}  // namespace lbm_internal

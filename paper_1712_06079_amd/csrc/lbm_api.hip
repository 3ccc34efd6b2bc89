// C ABI of the HDM pseudopotential lattice Boltzmann library (declarations and
// contracts in include/lbm.h).  Host planning: validation, the EOS constants
// folded into the device potential, the explicit HDM coefficient rows
// (Sec. 3.2 Eq. 20) per axis, the workspace layout and the launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/lbm.h"
#include "eos_host.hpp"
#include "hdm_coeffs.hpp"
#include "lbm_fused.hpp"
#include "lbm_kernels.hpp"

namespace {

thread_local char g_err[512] = "";

lbm_status fail(lbm_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return fail(LBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

lbm_host::EosConst eos_const(const lbm_params* p) {
    return lbm_host::EosConst{p->eos, p->a, p->b, p->R, p->omega};
}

lbm_status validate(const lbm_params* p) {
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (p->nx < 5 || p->ny < 5) return fail(LBM_EINVAL, "lattice %d x %d: each side must be >= 5", p->nx, p->ny);
    if ((long)p->nx * p->ny > (1L << 31)) return fail(LBM_EINVAL, "lattice too large");
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LBM_EINVAL, "tau = %g must be > 1/2", p->tau);
    if (p->eos < 0 || p->eos > 4) return fail(LBM_EINVAL, "unknown eos %d", p->eos);
    if (p->force < 0 || p->force > 2) return fail(LBM_EINVAL, "unknown force %d", p->force);
    if (p->grad < 0 || p->grad > 1) return fail(LBM_EINVAL, "unknown gradient %d", p->grad);
    if (p->prec < 0 || p->prec > 1) return fail(LBM_EINVAL, "unknown precision %d", p->prec);
    if (!(p->a > 0) || !(p->b > 0) || !(p->R > 0)) return fail(LBM_EINVAL, "EOS constants a, b, R must be > 0");
    if (!(p->T > 0) || !std::isfinite(p->T)) return fail(LBM_EINVAL, "T = %g must be > 0", p->T);
    if (!(p->k > 0) || !std::isfinite(p->k)) return fail(LBM_EINVAL, "k = %g must be > 0", p->k);
    if (!std::isfinite(p->g) || !std::isfinite(p->A) || !std::isfinite(p->omega))
        return fail(LBM_EINVAL, "non-finite g, A or omega");
    return LBM_OK;
}

int nblocks_x(int nx) { return (nx + lbm::BX - 1) / lbm::BX; }

}  // namespace

struct lbm_domain {
    lbm_params p;
    double Tc, rhoc, alpha;
    int nxb, pitch;
    int cur;           // index of the buffer pair holding the current state
    int64_t steps;
    int variant;       // 0 fused, 1 two-pass reference
    int tile_y;        // fused: rows per tile; reference: rows per tile
    char* ws;
    size_t ws_bytes;
    size_t off_f[2], off_phi[2], off_part, off_scr;
    int tx, ty;
    double dx[lbm::JCAP], dy[lbm::JCAP];
};

namespace {

struct Layout {
    size_t f, phi, part, scr, total;
};

constexpr int MOM_TY = 16;  // rows per moments tile

Layout layout_of(const lbm_params* p) {
    const size_t es = p->prec == LBM_F32 ? 4 : 8;
    const size_t pitch = (size_t)nblocks_x(p->nx) * lbm::BX;
    Layout L;
    L.f = align256(lbm::Q * pitch * p->ny * es);
    L.phi = align256(pitch * p->ny * es);
    const size_t nb = (size_t)nblocks_x(p->nx) * ((p->ny + MOM_TY - 1) / MOM_TY);
    L.part = align256(nb * 4 * sizeof(double));
    L.scr = 256;
    L.total = 2 * L.f + 2 * L.phi + L.part + L.scr;
    return L;
}

template <typename Real>
lbm::StepArgs<Real> make_args(const lbm_domain* d, int in_buf, int out_buf) {
    lbm::StepArgs<Real> a;
    std::memset(&a, 0, sizeof(a));
    a.f_in = reinterpret_cast<const Real*>(d->ws + d->off_f[in_buf]);
    a.f_out = reinterpret_cast<Real*>(d->ws + d->off_f[out_buf]);
    a.phi_in = reinterpret_cast<const Real*>(d->ws + d->off_phi[in_buf]);
    a.phi_out = reinterpret_cast<Real*>(d->ws + d->off_phi[out_buf]);
    a.nx = d->p.nx;
    a.ny = d->p.ny;
    a.nxb = d->nxb;
    a.tx = d->tx;
    a.ty = d->ty;
    a.omega = (Real)(1.0 / d->p.tau);
    a.A = (Real)d->p.A;
    const double g = d->p.g, k = d->p.k;
    a.eos.kind = d->p.eos;
    a.eos.c_rep = (Real)(g * k * d->p.R * d->p.T);
    a.eos.c_att = (Real)(g * k * d->p.a * d->alpha);
    a.eos.c_lin = (Real)(g / 3.0);
    a.eos.b = (Real)d->p.b;
    for (int j = 0; j < lbm::JCAP; ++j) {
        a.dx[j] = (Real)d->dx[j];
        a.dy[j] = (Real)d->dy[j];
    }
    return a;
}

unsigned grid_1d(long n) {
    long b = (n + lbm::NT - 1) / lbm::NT;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// Dispatch a callable on the compile-time (Real, FORCE) of a domain.
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

lbm_status launch_phi(lbm_domain* d, int buf, hipStream_t s) {
    dispatch(d, [&](auto real, auto force) {
        using Real = decltype(real);
        auto a = make_args<Real>(d, buf, buf);
        hipLaunchKernelGGL((lbm::k_phi<Real, decltype(force)::value>), dim3(grid_1d((long)d->pitch * d->p.ny)),
                           dim3(lbm::NT), 0, s, a);
    });
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

template <typename Real, int FORCE, int TY>
void launch_ref(lbm_domain* d, const lbm::StepArgs<Real>& a, hipStream_t s) {
    dim3 grid(d->nxb, (d->p.ny + TY - 1) / TY);
    hipLaunchKernelGGL((lbm::k_collide<Real, FORCE, TY>), grid, dim3(lbm::NT), 0, s, a);
}

lbm_status step_once(lbm_domain* d, hipStream_t s) {
    const int in = d->cur, out = 1 - d->cur;
    if (d->variant == 1) {
        dispatch(d, [&](auto real, auto force) {
            using Real = decltype(real);
            constexpr int F = decltype(force)::value;
            auto a = make_args<Real>(d, in, out);
            if (d->tile_y <= 8) launch_ref<Real, F, 8>(d, a, s);
            else launch_ref<Real, F, 16>(d, a, s);
        });
        HIP_TRY(hipGetLastError());
        d->cur = out;
        return launch_phi(d, out, s);
    }
    lbm_status st = LBM_OK;
    dispatch(d, [&](auto real, auto force) {
        using Real = decltype(real);
        constexpr int F = decltype(force)::value;
        auto a = make_args<Real>(d, in, out);
        if (!lbm::launch_fused<Real, F>(a, d->tile_y, s)) st = LBM_EUNSUPPORTED;
    });
    if (st != LBM_OK) return fail(st, "fused kernel: unsupported tile height %d", d->tile_y);
    HIP_TRY(hipGetLastError());
    d->cur = out;
    return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err; }

lbm_status lbm_critical(const lbm_params* p, double* Tc, double* rhoc) {
    if (!p || !Tc || !rhoc) return fail(LBM_EINVAL, "NULL argument");
    if (p->eos < 0 || p->eos > 4) return fail(LBM_EINVAL, "unknown eos %d", p->eos);
    if (!lbm_host::eos_critical(eos_const(p), Tc, rhoc)) return fail(LBM_EINVAL, "no critical point found");
    return LBM_OK;
}

lbm_status lbm_maxwell(const lbm_params* p, double T, double* rho_v, double* rho_l, double* p0) {
    if (!p || !rho_v || !rho_l) return fail(LBM_EINVAL, "NULL argument");
    if (p->eos < 0 || p->eos > 4) return fail(LBM_EINVAL, "unknown eos %d", p->eos);
    double q = 0;
    if (!lbm_host::eos_maxwell(eos_const(p), T, rho_v, rho_l, &q))
        return fail(LBM_EINVAL, "no liquid-vapour coexistence at T = %g", T);
    if (p0) *p0 = q;
    return LBM_OK;
}

lbm_status lbm_hdm_row(int32_t n, int32_t prec, double* d, int32_t* taps) {
    if (!d || !taps) return fail(LBM_EINVAL, "NULL argument");
    if (n < 5) return fail(LBM_EINVAL, "n = %d must be >= 5", n);
    if (prec != LBM_F64 && prec != LBM_F32) return fail(LBM_EINVAL, "unknown precision %d", prec);
    const int radius = prec == LBM_F32 ? lbm::Radius<float>::value : lbm::Radius<double>::value;
    *taps = lbm_host::hdm_taps(n, radius);
    for (int j = 0; j < lbm::JCAP; ++j) d[j] = 0.0;
    lbm_host::hdm_row(n, *taps, d);
    return LBM_OK;
}

lbm_status lbm_workspace_bytes(const lbm_params* p, size_t* bytes) {
    lbm_status st = validate(p);
    if (st != LBM_OK) return st;
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    *bytes = layout_of(p).total;
    return LBM_OK;
}

lbm_status lbm_init(const lbm_params* p, void* workspace, size_t workspace_bytes, const double* rho0,
                    const double* ux0, const double* uy0, hipStream_t stream, lbm_domain** out) {
    lbm_status st = validate(p);
    if (st != LBM_OK) return st;
    if (!out || !workspace || !rho0) return fail(LBM_EINVAL, "NULL workspace, rho0 or out");
    if (((uintptr_t)workspace & 255) != 0) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    Layout L = layout_of(p);
    if (workspace_bytes < L.total) return fail(LBM_ENOMEM, "workspace %zu < %zu bytes", workspace_bytes, L.total);
    lbm_host::EosConst ec = eos_const(p);
    double Tc = 0, rhoc = 0;
    if (!lbm_host::eos_critical(ec, &Tc, &rhoc)) return fail(LBM_EINVAL, "EOS has no critical point");
    if ((p->eos == LBM_EOS_PR || p->eos == LBM_EOS_RKS) && !(p->T < 4.0 * Tc))
        return fail(LBM_EINVAL, "T = %g is outside the alpha(T_r) range", p->T);

    lbm_domain* d = new (std::nothrow) lbm_domain;
    if (!d) return fail(LBM_EINVAL, "out of host memory");
    std::memset(d, 0, sizeof(*d));
    d->p = *p;
    d->Tc = Tc;
    d->rhoc = rhoc;
    d->alpha = lbm_host::eos_alpha(ec, p->T, Tc);
    d->nxb = nblocks_x(p->nx);
    d->pitch = d->nxb * lbm::BX;
    d->cur = 0;
    d->steps = 0;
    d->variant = 0;
    d->tile_y = 0;
    d->ws = static_cast<char*>(workspace);
    d->ws_bytes = workspace_bytes;
    d->off_f[0] = 0;
    d->off_f[1] = L.f;
    d->off_phi[0] = 2 * L.f;
    d->off_phi[1] = 2 * L.f + L.phi;
    d->off_part = 2 * L.f + 2 * L.phi;
    d->off_scr = d->off_part + L.part;
    const int radius = p->prec == LBM_F32 ? lbm::Radius<float>::value : lbm::Radius<double>::value;
    if (p->grad == LBM_GRAD_CDM) {
        d->tx = d->ty = 1;
        lbm_host::cdm_row(1, d->dx);
        lbm_host::cdm_row(1, d->dy);
    } else {
        d->tx = lbm_host::hdm_taps(p->nx, radius);
        d->ty = lbm_host::hdm_taps(p->ny, radius);
        lbm_host::hdm_row(p->nx, d->tx, d->dx);
        lbm_host::hdm_row(p->ny, d->ty, d->dy);
    }

    // validate rho0 on the device
    int* flag = reinterpret_cast<int*>(d->ws + d->off_scr);
    const long n = (long)p->nx * p->ny;
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(lbm::k_check_rho0, dim3(grid_1d(n)), dim3(lbm::NT), 0, stream, rho0, n,
                           lbm_host::eos_rho_max(ec), flag);
        e = hipGetLastError();
    }
    int hflag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        delete d;
        return fail(LBM_EDEVICE, "validating rho0: %s", hipGetErrorString(e));
    }
    if (hflag) {
        delete d;
        return fail(LBM_EINVAL, "rho0 must be finite, > 0 and below the EOS pole %g", lbm_host::eos_rho_max(ec));
    }
    dispatch(d, [&](auto real, auto force) {
        using Real = decltype(real);
        auto a = make_args<Real>(d, 0, 0);
        hipLaunchKernelGGL((lbm::k_init<Real, decltype(force)::value>), dim3(grid_1d((long)d->pitch * p->ny)),
                           dim3(lbm::NT), 0, stream, a, rho0, ux0, uy0);
    });
    e = hipGetLastError();
    if (e != hipSuccess) {
        delete d;
        return fail(LBM_EDEVICE, "init launch: %s", hipGetErrorString(e));
    }
    *out = d;
    return LBM_OK;
}

lbm_status lbm_step(lbm_domain* d, int64_t nsteps, hipStream_t stream) {
    if (!d) return fail(LBM_EINVAL, "NULL domain");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
    for (int64_t s = 0; s < nsteps; ++s) {
        lbm_status st = step_once(d, stream);
        if (st != LBM_OK) return st;
        d->steps++;
    }
    return LBM_OK;
}

lbm_status lbm_moments(lbm_domain* d, double* rho, double* ux, double* uy, double* p, double* totals,
                       hipStream_t stream) {
    if (!d) return fail(LBM_EINVAL, "NULL domain");
    double* part = reinterpret_cast<double*>(d->ws + d->off_part);
    dim3 grid(d->nxb, (d->p.ny + MOM_TY - 1) / MOM_TY);
    dispatch(d, [&](auto real, auto force) {
        using Real = decltype(real);
        auto a = make_args<Real>(d, d->cur, d->cur);
        hipLaunchKernelGGL((lbm::k_moments<Real, decltype(force)::value, MOM_TY>), grid, dim3(lbm::NT), 0, stream, a,
                           rho, ux, uy, p, part);
    });
    HIP_TRY(hipGetLastError());
    if (totals) {
        hipLaunchKernelGGL(lbm::k_totals, dim3(1), dim3(lbm::NT), 0, stream, part, (long)grid.x * grid.y, totals);
        HIP_TRY(hipGetLastError());
    }
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_domain* d, double* f, hipStream_t stream) {
    if (!d || !f) return fail(LBM_EINVAL, "NULL argument");
    dispatch(d, [&](auto real, auto) {
        using Real = decltype(real);
        auto a = make_args<Real>(d, d->cur, d->cur);
        hipLaunchKernelGGL((lbm::k_get_f<Real>), dim3(grid_1d((long)d->p.nx * d->p.ny)), dim3(lbm::NT), 0, stream, a, f);
    });
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_domain* d, const double* f, hipStream_t stream) {
    if (!d || !f) return fail(LBM_EINVAL, "NULL argument");
    dispatch(d, [&](auto real, auto) {
        using Real = decltype(real);
        auto a = make_args<Real>(d, d->cur, d->cur);
        hipLaunchKernelGGL((lbm::k_set_f<Real>), dim3(grid_1d((long)d->p.nx * d->p.ny)), dim3(lbm::NT), 0, stream, a, f);
    });
    HIP_TRY(hipGetLastError());
    return launch_phi(d, d->cur, stream);
}

int64_t lbm_step_count(const lbm_domain* d) { return d ? d->steps : -1; }

lbm_status lbm_set_kernel(lbm_domain* d, int32_t variant, int32_t tile_y) {
    if (!d) return fail(LBM_EINVAL, "NULL domain");
    if (variant < 0 || variant > 1) return fail(LBM_EINVAL, "unknown kernel variant %d", variant);
    if (tile_y < 0 || tile_y > 64) return fail(LBM_EINVAL, "tile_y %d out of range", tile_y);
    d->variant = variant;
    d->tile_y = tile_y;
    return LBM_OK;
}

lbm_status lbm_check_finite(lbm_domain* d, int32_t* ok, hipStream_t stream) {
    if (!d || !ok) return fail(LBM_EINVAL, "NULL argument");
    double* tot = reinterpret_cast<double*>(d->ws + d->off_scr);
    lbm_status st = lbm_moments(d, nullptr, nullptr, nullptr, nullptr, tot, stream);
    if (st != LBM_OK) return st;
    double h[4];
    HIP_TRY(hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    *ok = std::isfinite(h[0]) && std::isfinite(h[1]) && std::isfinite(h[2]) ? 1 : 0;
    return *ok ? LBM_OK : fail(LBM_ENONFINITE, "non-finite density after %lld steps", (long long)d->steps);
}

void lbm_destroy(lbm_domain* d) { delete d; }

}  // extern "C"

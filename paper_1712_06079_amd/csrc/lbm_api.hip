// C ABI of the HDM pseudopotential lattice Boltzmann library (declarations and
// contracts in include/lbm.h).  Host planning: validation, the EOS constants
// folded into the device potential, the explicit HDM coefficient rows
// (Sec. 3.2 Eq. 20) per axis, the workspace layout and the launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/lbm.h"
#include "eos_host.hpp"
#include "hdm_coeffs.hpp"
#include "interface_host.hpp"
#include "lbm_adjoint.hpp"
#include "lbm_fused.hpp"
#include "lbm_march.hpp"
#include "lbm_internal.hpp"
#include "lbm_kernels.hpp"

namespace {

thread_local char g_err[512] = "";

}  // namespace

namespace lbm_internal {

lbm_status fail(lbm_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

}  // namespace lbm_internal

using namespace lbm_internal;

namespace {

lbm_host::EosConst eos_const(const lbm_params* p) {
    return lbm_host::EosConst{p->eos, p->a, p->b, p->R, p->omega};
}

lbm_status validate(const lbm_params* p) {
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (p->nx < 5 || p->ny < 5) return fail(LBM_EINVAL, "lattice %d x %d: each side must be >= 5", p->nx, p->ny);
    if (p->nx > (1 << 21) || p->ny > (1 << 21) || (long)p->nx * p->ny > (1L << 31))
        return fail(LBM_EINVAL, "lattice %d x %d: each side must be <= 2^21 and nx * ny <= 2^31", p->nx, p->ny);
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LBM_EINVAL, "tau = %g must be > 1/2", p->tau);
    if (p->eos < 0 || p->eos > 4) return fail(LBM_EINVAL, "unknown eos %d", p->eos);
    if (p->force < 0 || p->force > 2) return fail(LBM_EINVAL, "unknown force %d", p->force);
    if (p->grad < 0 || p->grad > 2) return fail(LBM_EINVAL, "unknown gradient %d", p->grad);
    if (p->prec < 0 || p->prec > 1) return fail(LBM_EINVAL, "unknown precision %d", p->prec);
    if (!(p->a > 0) || !(p->b > 0) || !(p->R > 0)) return fail(LBM_EINVAL, "EOS constants a, b, R must be > 0");
    if (!(p->T > 0) || !std::isfinite(p->T)) return fail(LBM_EINVAL, "T = %g must be > 0", p->T);
    if (!(p->k > 0) || !std::isfinite(p->k)) return fail(LBM_EINVAL, "k = %g must be > 0", p->k);
    if (!std::isfinite(p->g) || !std::isfinite(p->A) || !std::isfinite(p->omega))
        return fail(LBM_EINVAL, "non-finite g, A or omega");
    if (p->walls < 0 || p->walls > 1 || p->reserved != 0) return fail(LBM_EINVAL, "walls must be 0 or 1, reserved 0");
    if (p->walls && p->grad == LBM_GRAD_CDM9) return fail(LBM_EUNSUPPORTED, "walls with the Eq. 15 gradient");
    return LBM_OK;
}

int nblocks_x(int nx) { return (nx + lbm::BX - 1) / lbm::BX; }


struct Layout {
    size_t f, phi, part, scr, tab, total;
};

constexpr int MOM_TY = 16;  // rows per moments tile

Layout layout_of(const lbm_params* p) {
    const size_t es = p->prec == LBM_F32 ? 4 : 8;
    const size_t pitch = (size_t)nblocks_x(p->nx) * lbm::BX;
    Layout L;
    L.f = align256(lbm::Q * pitch * p->ny * es);
    L.phi = align256(pitch * p->ny * phi_elem_bytes(p));
    const size_t nb = (size_t)nblocks_x(p->nx) * ((p->ny + MOM_TY - 1) / MOM_TY);
    L.part = align256(nb * 4 * sizeof(double));
    L.scr = 256;
    L.tab = align256(sizeof(lbm::StepTables));
    L.total = 2 * L.f + 2 * L.phi + L.part + L.scr + L.tab;
    return L;
}

}  // namespace

namespace lbm_internal {

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

}  // namespace lbm_internal

namespace {

template <typename Real, int FORCE, int TY>
void launch_ref(lbm_domain* d, const lbm::StepArgs<Real>& a, hipStream_t s) {
    dim3 grid(d->nxb, (d->p.ny + TY - 1) / TY);
    hipLaunchKernelGGL((lbm::k_collide<Real, FORCE, TY>), grid, dim3(lbm::NT), 0, s, a);
}

// Rows per marching block (default 8: the fastest measured for both population
// precisions; two workgroups per CU with FP64 populations, three with FP32).
int march_rows(const lbm_domain* d) { return d->tile_y ? d->tile_y : 8; }

// The marching kernel needs the geometric form along y (HDM, ny > 2R + 1) and
// a y period longer than its look-ahead.
bool march_eligible(const lbm_domain* d) {
    if (d->p.grad != LBM_GRAD_HDM || d->p.walls) return false;
    return d->p.prec == LBM_F32 ? lbm::march_fits<float>(d->p.ny, march_rows(d))
                                : lbm::march_fits<double>(d->p.ny, march_rows(d));
}

// y chunks per strip: by default the most that keep the grid within one set
// of resident workgroups (strips x chunks <= CUs x workgroups per CU).  A grid
// a few workgroups over that runs them as a second round after the first and
// nearly doubles the step (1152^2 FP64: 29 chunks 75 us, 28 chunks 49 us).
template <typename Real, int FORCE>
lbm_status march_chunks(lbm_domain* d, int ty, int* nchunk) {
    if (d->chunks > 0) {
        *nchunk = d->chunks < d->p.ny ? d->chunks : d->p.ny;
        return LBM_OK;
    }
    int& per_cu = ty == 4 ? d->march_occ[0] : d->march_occ[1];  // cached occupancy query
    if (per_cu == 0) {
        // the instantiation launch_march_t picks for this N_x (paired accesses when
        // even; the plain-access twin has the same registers and LDS)
        const bool vec = d->p.nx % 2 == 0;
        const auto occ = [&](const void* kern) {
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, lbm::NT, 0);
        };
        if (ty == 4)
            HIP_TRY(vec ? occ((const void*)lbm::k_march<Real, FORCE, 4, true, true>)
                        : occ((const void*)lbm::k_march<Real, FORCE, 4, false, true>));
        else
            HIP_TRY(vec ? occ((const void*)lbm::k_march<Real, FORCE, 8, true, true>)
                        : occ((const void*)lbm::k_march<Real, FORCE, 8, false, true>));
        if (per_cu < 1) per_cu = 1;
    }
    const long target = (long)d->ncu * per_cu;
    long n = target / d->nxb;
    if (n > d->p.ny) n = d->p.ny;
    if (n < 1) n = 1;
    *nchunk = (int)n;
    return LBM_OK;
}

// One step from (f_in, phi_in) to (f_out, phi_out), any of the domain's
// buffers or snapshot slots, with the selected kernel.
// Automatic choice (variant 0): the marching kernel when its chunks keep at
// least 16 rows each with FP64 populations, 11 with FP32 (shorter chunks
// spend most of their time in the chunk prologue, about R + NB TY potential
// rows: 79 FP64, 60 FP32), otherwise tiles (auto_tile).  FP32 736^2 to 832^2
// (11.5 - 14.1 rows per chunk): march 22.0 - 25.6 us per step against 26.9 -
// 29.1 for the best tiles; FP32 704^2 (10.2 rows): tiles 19.8 against 21.6.
template <typename Real>
constexpr int march_min_rows() { return sizeof(Real) == 8 ? 16 : 11; }

// Resident tile-kernel workgroups per CU at tile height ty (cached per domain).
template <typename Real, int FORCE>
lbm_status fused_occupancy(lbm_domain* d, int ty, int* per_cu) {
    int& n = d->fused_occ[ty == 4 ? 0 : (ty == 8 ? 1 : 2)];
    if (n == 0) {
        const bool g9 = d->p.grad == LBM_GRAD_CDM9;
        auto occ = [&](const void* kern) { return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, lbm::NT, 0); };
        if (ty == 4)
            HIP_TRY(g9 ? occ((const void*)lbm::k_fused<Real, FORCE, lbm::BX, 4, 4, true>)
                       : occ((const void*)lbm::k_fused<Real, FORCE, lbm::BX, 4, 4>));
        else if (ty == 8)
            HIP_TRY(g9 ? occ((const void*)lbm::k_fused<Real, FORCE, lbm::BX, 8, 4, true>)
                       : occ((const void*)lbm::k_fused<Real, FORCE, lbm::BX, 8, 4>));
        else
            HIP_TRY(g9 ? occ((const void*)lbm::k_fused<Real, FORCE, lbm::BX, 16, 4, true>)
                       : occ((const void*)lbm::k_fused<Real, FORCE, lbm::BX, 16, 4>));
        if (n < 1) n = 1;
    }
    *per_cu = n;
    return LBM_OK;
}

// Tile height: the smallest (most tiles) whose tiles all fit one set of
// resident workgroups; a few tiles over it would run as a second round
// (FP32 512^2: 8-row tiles, 512 in 512 slots, 12.7 us per step, against 15.0
// for 16-row tiles; 640^2: 16-row tiles, 400 in 512, 19.1 against 20.9 for
// 8-row ones, 1600 > 768).  Where no height fits one round, the default (8
// rows FP64, 16 FP32) halved until there are at least as many tiles as
// compute units.
template <typename Real, int FORCE>
lbm_status auto_tile(lbm_domain* d, int* ty_out) {
    for (int ty = 4; ty <= 16; ty *= 2) {
        int per_cu = 1;
        const lbm_status st = fused_occupancy<Real, FORCE>(d, ty, &per_cu);
        if (st != LBM_OK) return st;
        if ((long)d->nxb * ((d->p.ny + ty - 1) / ty) <= (long)d->ncu * per_cu) {
            *ty_out = ty;
            return LBM_OK;
        }
    }
    int ty = sizeof(Real) == 8 ? 8 : 16;
    while (ty > 4 && (long)d->nxb * ((d->p.ny + ty - 1) / ty) < d->ncu) ty /= 2;
    *ty_out = ty;
    return LBM_OK;
}

// Capacity of the last-level (Infinity) cache of gfx950 in bytes.  A state
// of at most this size (both population and potential buffers) stays
// resident from one step to the next when the marching kernel accesses it
// plainly: 1024^2 FP64 (160 MiB) 48.6 -> 42.4 us per step, 1280^2 FP64
// (250 MiB) 97 -> 87 us; above it the non-temporal form is faster (2048^2
// FP64 (640 MiB) 146 against 141 us, 4096^2 -1 %).
constexpr size_t LLC_BYTES = size_t(256) << 20;

bool march_cached(const lbm_domain* d) {
    if (d->access != 0) return d->access == 2;
    const size_t state = 2 * (d->off_f[1] + (d->off_phi[1] - d->off_phi[0]));
    return state <= LLC_BYTES;
}

// What one step launches: kernel 1 (two-pass reference), 2 (tiles) or 3
// (strip march), the tile height or marching block rows, the march's y chunks
// per strip and whether it uses plain (cached) population accesses.
struct KernelChoice {
    int kernel, rows, chunks, cached;
};

template <typename Real, int F>
lbm_status choose_kernel(lbm_domain* d, KernelChoice* c) {
    if (d->variant == 3 && !march_eligible(d))
        return fail(LBM_EUNSUPPORTED, "marching kernel needs the HDM gradient, a periodic and longer y axis (ny = %d)", d->p.ny);
    if (d->variant == 1 && d->p.walls) return fail(LBM_EUNSUPPORTED, "the two-pass reference kernel has no walls");
    c->chunks = 0;
    c->cached = 0;
    if (d->variant == 1) {
        c->kernel = 1;
        c->rows = d->tile_y <= 8 ? 8 : 16;
        return LBM_OK;
    }
    bool march = d->variant == 3;
    int nchunk = 0;
    if (march || (d->variant == 0 && march_eligible(d))) {
        const lbm_status st = march_chunks<Real, F>(d, march_rows(d), &nchunk);
        if (st != LBM_OK) return st;
        if (!march) march = d->p.ny / nchunk >= march_min_rows<Real>();
    }
    if (march) {
        c->kernel = 3;
        c->rows = march_rows(d);
        c->chunks = nchunk;
        c->cached = march_cached(d) && d->p.nx % 2 == 0;  // odd N_x: non-temporal always
        return LBM_OK;
    }
    c->kernel = 2;
    if (d->variant == 0) return auto_tile<Real, F>(d, &c->rows);
    c->rows = d->tile_y ? d->tile_y : (sizeof(Real) == 8 ? 8 : 16);
    return LBM_OK;
}

lbm_status run_step(lbm_domain* d, const void* f_in, const void* phi_in, void* f_out, void* phi_out, hipStream_t s) {
    lbm_status st = LBM_OK;
    dispatch(d, [&](auto real, auto force) {
        using Real = decltype(real);
        constexpr int F = decltype(force)::value;
        KernelChoice c;
        st = choose_kernel<Real, F>(d, &c);
        if (st != LBM_OK) return;
        auto a = make_args<Real>(d, d->cur, 1 - d->cur);
        a.f_in = static_cast<const Real*>(f_in);
        a.phi_in = phi_in;
        a.f_out = static_cast<Real*>(f_out);
        a.phi_out = phi_out;
        if (c.kernel == 1) {
            if (c.rows == 8) launch_ref<Real, F, 8>(d, a, s);
            else launch_ref<Real, F, 16>(d, a, s);
            auto b = a;  // potential field of the new state
            b.f_in = a.f_out;
            hipLaunchKernelGGL((lbm::k_phi<Real, F>), dim3(grid_1d((long)d->pitch * d->p.ny)), dim3(lbm::NT), 0, s, b);
        } else if (c.kernel == 3) {
            if (!lbm::launch_march<Real, F>(a, c.rows, c.chunks, c.cached != 0, s))
                st = fail(LBM_EUNSUPPORTED, "marching kernel: unsupported block height %d", c.rows);
        } else if (!lbm::launch_fused<Real, F>(a, c.rows, s)) {
            st = fail(LBM_EUNSUPPORTED, "fused kernel: unsupported tile height %d", c.rows);
        }
    });
    if (st != LBM_OK) return st;
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

lbm_status step_once(lbm_domain* d, hipStream_t s) {
    const int in = d->cur, out = 1 - d->cur;
    lbm_status st = run_step(d, d->ws + d->off_f[in], d->ws + d->off_phi[in], d->ws + d->off_f[out],
                             d->ws + d->off_phi[out], s);
    if (st != LBM_OK) return st;
    d->cur = out;
    return LBM_OK;
}

// Bytes of the population and potential parts of a snapshot.
size_t f_bytes(const lbm_domain* d) { return d->off_f[1]; }
size_t phi_bytes(const lbm_domain* d) { return d->off_phi[1] - d->off_phi[0]; }

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

lbm_status lbm_interface_excess(const lbm_params* p, int32_t n, const double* rho, double* W) {
    if (!p || !rho || !W || n < 0) return fail(LBM_EINVAL, "invalid arguments");
    if (p->eos < 0 || p->eos > 4) return fail(LBM_EINVAL, "unknown eos %d", p->eos);
    lbm_host::FlatInterface f;
    if (!lbm_host::flat_interface(eos_const(p), p->T, p->k, &f))
        return fail(LBM_EINVAL, "no liquid-vapour coexistence at T = %g (or k <= 0)", p->T);
    for (int i = 0; i < n; ++i) {
        if (!(rho[i] > 0.0) || !(rho[i] < lbm_host::eos_rho_max(f.e))) return fail(LBM_EINVAL, "density %g outside the EOS", rho[i]);
        W[i] = lbm_host::interface_excess(f, rho[i]);
    }
    return LBM_OK;
}

lbm_status lbm_flat_profile(const lbm_params* p, double kappa, double h, int32_t n, double* rho, double* drho) {
    if (!p || !rho || !drho || n < 1 || !(kappa > 0.0) || !(h > 0.0)) return fail(LBM_EINVAL, "invalid arguments");
    if (p->eos < 0 || p->eos > 4) return fail(LBM_EINVAL, "unknown eos %d", p->eos);
    lbm_host::FlatInterface f;
    if (!lbm_host::flat_interface(eos_const(p), p->T, p->k, &f))
        return fail(LBM_EINVAL, "no liquid-vapour coexistence at T = %g (or k <= 0)", p->T);
    lbm_host::flat_profile(f, kappa, h, n, rho, drho);
    return LBM_OK;
}

lbm_status lbm_sigma_slab(double kappa, int32_t n, const double* rho, double* drho, double* sigma) {
    if (!rho || !sigma || n < 5 || !(kappa > 0.0)) return fail(LBM_EINVAL, "invalid arguments");
    *sigma = lbm_host::sigma_slab(kappa, n, rho, drho);
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

    int dev = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (ncu < 1) ncu = 1;

    lbm_domain* d = new (std::nothrow) lbm_domain;
    if (!d) return fail(LBM_ENOMEM, "out of host memory");
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
    d->chunks = 0;
    d->access = 0;
    d->ncu = ncu;
    d->ws = static_cast<char*>(workspace);
    d->ws_bytes = workspace_bytes;
    d->off_f[0] = 0;
    d->off_f[1] = L.f;
    d->off_phi[0] = 2 * L.f;
    d->off_phi[1] = 2 * L.f + L.phi;
    d->off_part = 2 * L.f + 2 * L.phi;
    d->off_scr = d->off_part + L.part;
    const int radius = p->prec == LBM_F32 ? lbm::Radius<float>::value : lbm::Radius<double>::value;
    if (p->grad == LBM_GRAD_CDM || p->grad == LBM_GRAD_CDM9) {  // (Eq. 15 kernels take their own path)
        d->tx = d->ty = 1;
        lbm_host::cdm_row(1, d->dx);
        lbm_host::cdm_row(1, d->dy);
    } else {
        // between walls the y lines continue by reflection: the periodic row of 2 ny points
        const int nyl = p->walls ? 2 * p->ny : p->ny;
        d->tx = lbm_host::hdm_taps(p->nx, radius);
        d->ty = lbm_host::hdm_taps(nyl, radius);
        lbm_host::hdm_row(p->nx, d->tx, d->dx);
        lbm_host::hdm_row(nyl, d->ty, d->dy);
    }
    d->off_tab = d->off_scr + L.scr;
    build_tables(d);
    {
        hipError_t et = hipMemcpyAsync(d->ws + d->off_tab, &d->htab, sizeof(d->htab), hipMemcpyHostToDevice, stream);
        if (et != hipSuccess) {
            delete d;
            return fail(LBM_EDEVICE, "uploading the stencil tables: %s", hipGetErrorString(et));
        }
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
    if (variant < 0 || variant > 3) return fail(LBM_EINVAL, "unknown kernel variant %d", variant);
    if (tile_y < 0 || tile_y > 64) return fail(LBM_EINVAL, "tile_y %d out of range", tile_y);
    if (variant == 2 && !(tile_y == 0 || tile_y == 4 || tile_y == 8 || tile_y == 16))
        return fail(LBM_EINVAL, "tile kernel: tile_y must be 0, 4, 8 or 16 (got %d)", tile_y);
    if (variant == 3 && !(tile_y == 0 || tile_y == 4 || tile_y == 8))
        return fail(LBM_EINVAL, "marching kernel: block rows must be 0, 4 or 8 (got %d)", tile_y);
    d->variant = variant;
    d->tile_y = tile_y;
    return LBM_OK;
}

lbm_status lbm_set_chunks(lbm_domain* d, int32_t nchunk) {
    if (!d) return fail(LBM_EINVAL, "NULL domain");
    if (nchunk < 0) return fail(LBM_EINVAL, "chunk count %d < 0", nchunk);
    d->chunks = nchunk;
    return LBM_OK;
}

lbm_status lbm_set_access(lbm_domain* d, int32_t access) {
    if (!d) return fail(LBM_EINVAL, "NULL domain");
    if (access < 0 || access > 2) return fail(LBM_EINVAL, "access mode %d not in 0 .. 2", access);
    d->access = access;
    return LBM_OK;
}

lbm_status lbm_kernel_choice(lbm_domain* d, int32_t* kernel, int32_t* rows, int32_t* chunks, int32_t* cached) {
    if (!d || !kernel || !rows || !chunks || !cached) return fail(LBM_EINVAL, "NULL argument");
    lbm_status st = LBM_OK;
    KernelChoice c{};
    dispatch(d, [&](auto real, auto force) {
        st = choose_kernel<decltype(real), decltype(force)::value>(d, &c);
    });
    if (st != LBM_OK) return st;
    *kernel = c.kernel;
    *rows = c.rows;
    *chunks = c.chunks;
    *cached = c.cached;
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

lbm_status lbm_state_bytes(const lbm_domain* d, size_t* bytes) {
    if (!d || !bytes) return fail(LBM_EINVAL, "NULL argument");
    *bytes = f_bytes(d) + phi_bytes(d);
    return LBM_OK;
}

lbm_status lbm_save_state(lbm_domain* d, void* state, hipStream_t stream) {
    if (!d || !state) return fail(LBM_EINVAL, "NULL argument");
    if (((uintptr_t)state & 255) != 0) return fail(LBM_EINVAL, "state must be 256-byte aligned");
    char* st = static_cast<char*>(state);
    HIP_TRY(hipMemcpyAsync(st, d->ws + d->off_f[d->cur], f_bytes(d), hipMemcpyDeviceToDevice, stream));
    HIP_TRY(hipMemcpyAsync(st + f_bytes(d), d->ws + d->off_phi[d->cur], phi_bytes(d), hipMemcpyDeviceToDevice, stream));
    return LBM_OK;
}

lbm_status lbm_load_state(lbm_domain* d, const void* state, hipStream_t stream) {
    if (!d || !state) return fail(LBM_EINVAL, "NULL argument");
    if (((uintptr_t)state & 255) != 0) return fail(LBM_EINVAL, "state must be 256-byte aligned");
    const char* st = static_cast<const char*>(state);
    HIP_TRY(hipMemcpyAsync(d->ws + d->off_f[d->cur], st, f_bytes(d), hipMemcpyDeviceToDevice, stream));
    HIP_TRY(hipMemcpyAsync(d->ws + d->off_phi[d->cur], st + f_bytes(d), phi_bytes(d), hipMemcpyDeviceToDevice, stream));
    return LBM_OK;
}

lbm_status lbm_record(lbm_domain* d, int64_t nsteps, void* states, size_t stride, hipStream_t stream) {
    if (!d || !states) return fail(LBM_EINVAL, "NULL argument");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
    if (((uintptr_t)states & 255) != 0 || (stride & 255) != 0) return fail(LBM_EINVAL, "states and stride must be 256-byte aligned");
    if (stride < f_bytes(d) + phi_bytes(d)) return fail(LBM_EINVAL, "stride %zu < state bytes %zu", stride, f_bytes(d) + phi_bytes(d));
    char* base = static_cast<char*>(states);
    lbm_status st = lbm_save_state(d, base, stream);
    if (st != LBM_OK) return st;
    const size_t fb = f_bytes(d);
    for (int64_t t = 0; t < nsteps; ++t) {
        char* in = base + (size_t)t * stride;
        char* out = in + stride;
        st = run_step(d, in, in + fb, out, out + fb, stream);
        if (st != LBM_OK) return st;
    }
    if (nsteps > 0) {
        st = lbm_load_state(d, base + (size_t)nsteps * stride, stream);
        if (st != LBM_OK) return st;
        d->steps += nsteps;
    }
    return LBM_OK;
}

namespace {
// Rows per tile of the reverse kernels.  Four-row tiles stage their whole
// cross (or row bar) with every load in flight at once, three workgroups per
// compute unit; they are the fastest measured at every size, on both paths
// (reverse step, 16-row / 8-row / 4-row tiles: 384^2 42 / 38 / 26 us, 768^2
// 100 / 90 / 74 us, 1280^2 243 / 252 / 191 us, 4096^2 with the column marches
// 1.56 / 1.54 / 1.33 ms).
constexpr int ADJ_TY = 4;
// Chunks of the column march that takes the y derivatives of the reverse
// step (k_adj_dy), or 0 where the tiles keep them.  The march needs the
// geometric form along y (ny > 2R + 1, which also gives ny > (NB + 2) 8 + 3).
// Kernel variant 3 (marching) always takes it there, variants 1 and 2 (tiles)
// never; the automatic choice takes it once there are 1.5 64-row column
// chunks per compute unit (tiles against column marches: 1024^2, 256 chunks,
// 116 against 127 us; 1280^2, 400 chunks, 190 against 178 us).  About eight
// wavefronts per compute unit.
int adj_dy_chunks(const lbm_domain* d) {
    constexpr int R = lbm::Radius<double>::value;
    if (d->p.grad != LBM_GRAD_HDM || d->p.ny <= 2 * R + 1 || d->variant == 1 || d->variant == 2) return 0;
    const long most = std::max(1, d->p.ny / 64);
    if (d->variant == 0 && 2L * d->nxb * (d->p.ny / 64) < 3L * d->ncu) return 0;
    const long want = (8L * d->ncu + d->nxb - 1) / d->nxb;
    return (int)std::max(1L, std::min(most, want));
}

// Adjoint scratch: planes a_x, a_y, U_bar_local, rho (row pitch of the
// lattice), the per-tile partials, and for multi-step calls the scalar plane
// of the factored cotangent ([ny][nx]).  `single` is what one step needs.
struct AdjLayout {
    size_t plane, f, part, add, single, total;
};
AdjLayout adj_layout(const lbm_domain* d) {
    AdjLayout L;
    L.plane = align256((size_t)d->pitch * d->p.ny * sizeof(double));
    L.f = d->off_f[1];
    const size_t nb = (size_t)d->nxb * ((d->p.ny + ADJ_TY - 1) / ADJ_TY);
    L.part = align256(nb * 2 * sizeof(double));
    L.add = align256((size_t)d->p.nx * d->p.ny * sizeof(double));
    L.single = 4 * L.plane + L.part;
    L.total = L.single + L.add;
    return L;
}
double alpha_prime(const lbm_domain* d) {
    const double T = d->p.T;
    if (d->p.eos == LBM_EOS_RK) return -0.5 / (T * std::sqrt(T));
    if (d->p.eos == LBM_EOS_PR || d->p.eos == LBM_EOS_RKS) {
        const double w = d->p.omega;
        const double m = d->p.eos == LBM_EOS_PR ? 0.37464 + w * (1.54226 - 0.26992 * w) : 0.480 + w * (1.574 - 0.176 * w);
        const double t = 1.0 + m * (1.0 - std::sqrt(T / d->Tc));
        return -m * t / std::sqrt(T * d->Tc);
    }
    return 0.0;
}
}  // namespace

lbm_status lbm_adjoint_workspace_bytes(const lbm_domain* d, size_t* bytes) {
    if (!d || !bytes) return fail(LBM_EINVAL, "NULL argument");
    *bytes = adj_layout(d).total;
    return LBM_OK;
}

namespace {
// Kernels of one reverse step at snapshot `state_t` (populations and their
// potential field); the per-block partials of dJ/dg, dJ/dT are written
// (accumulate = 0) or added to (accumulate = 1).
lbm_status adjoint_kernels(lbm_domain* d, const void* state_t, const double* lam_next, double* lam_t, char* w,
                           int accumulate, hipStream_t stream, const double* add_next = nullptr,
                           double* add_out = nullptr) {
    AdjLayout L = adj_layout(d);
    lbm::AdjArgs A;
    std::memset(&A, 0, sizeof(A));
    A.s = make_args<double>(d, d->cur, d->cur);
    A.s.f_in = static_cast<const double*>(state_t);
    A.s.phi_in = static_cast<const char*>(state_t) + f_bytes(d);
    A.s.phi_out = nullptr;
    A.ax = reinterpret_cast<double*>(w);
    A.ay = reinterpret_cast<double*>(w + L.plane);
    A.ubl = reinterpret_cast<double*>(w + 2 * L.plane);
    A.rho = reinterpret_cast<double*>(w + 3 * L.plane);
    A.partial = reinterpret_cast<double*>(w + 4 * L.plane);
    A.accumulate = accumulate;
    A.add_next = add_next;
    A.add_out = add_out;
    A.lam_next = lam_next;
    A.lam = lam_t;
    A.e.kind = d->p.eos;
    A.e.g = d->p.g;
    A.e.b = d->p.b;
    A.e.c_rep = d->p.k * d->p.R * d->p.T;
    A.e.c_att = d->p.k * d->p.a * d->alpha;
    A.e.c_attT = d->p.k * d->p.a * alpha_prime(d);
    A.e.kR = d->p.k * d->p.R;
    const dim3 grid(d->nxb, (d->p.ny + ADJ_TY - 1) / ADJ_TY);
    const int nchunk = adj_dy_chunks(d);
    if (nchunk == 0 && (add_next || add_out))  // only the column-march passes take the factored form
        return fail(LBM_EINVAL, "factored cotangent without the column-march reverse step");
    const dim3 gdy((d->nxb + lbm::NT / lbm::BX - 1) / (lbm::NT / lbm::BX), nchunk > 0 ? nchunk : 1);
    auto launch = [&](auto force) {
        constexpr int F = decltype(force)::value, TY = ADJ_TY;
        if (nchunk > 0) {  // y derivatives by column marches
            hipLaunchKernelGGL((lbm::k_adj_dy<F, 0>), gdy, dim3(lbm::NT), 0, stream, A, nchunk);
            if (add_next)
                hipLaunchKernelGGL((lbm::k_adj_local<F, TY, true, true>), grid, dim3(lbm::NT), 0, stream, A);
            else
                hipLaunchKernelGGL((lbm::k_adj_local<F, TY, true>), grid, dim3(lbm::NT), 0, stream, A);
            hipLaunchKernelGGL((lbm::k_adj_dy<F, 1>), gdy, dim3(lbm::NT), 0, stream, A, nchunk);
            if (add_out)
                hipLaunchKernelGGL((lbm::k_adj_nonlocal<F, TY, true, true>), grid, dim3(lbm::NT), 0, stream, A);
            else
                hipLaunchKernelGGL((lbm::k_adj_nonlocal<F, TY, true>), grid, dim3(lbm::NT), 0, stream, A);
        } else {
            hipLaunchKernelGGL((lbm::k_adj_local<F, TY>), grid, dim3(lbm::NT), 0, stream, A);
            hipLaunchKernelGGL((lbm::k_adj_nonlocal<F, TY>), grid, dim3(lbm::NT), 0, stream, A);
        }
    };
    using SC = std::integral_constant<int, lbm::FORCE_SC>;
    using ZC = std::integral_constant<int, lbm::FORCE_ZC>;
    if (d->p.force == LBM_FORCE_SC)
        launch(SC());
    else
        launch(ZC());
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

lbm_status adjoint_check(lbm_domain* d, const void* adj_ws, size_t adj_ws_bytes, bool multi = false) {
    if (d->p.prec != LBM_F64) return fail(LBM_EUNSUPPORTED, "the adjoint step is implemented for FP64 domains");
    if (d->p.force == LBM_FORCE_HYBRID) return fail(LBM_EUNSUPPORTED, "the adjoint step supports the SC and ZC forces");
    if (d->p.grad == LBM_GRAD_CDM9) return fail(LBM_EUNSUPPORTED, "the adjoint step supports the Eq. 20 and Eq. 14 gradients");
    if (d->p.walls) return fail(LBM_EUNSUPPORTED, "the adjoint step is periodic only");
    if (((uintptr_t)adj_ws & 255) != 0) return fail(LBM_EINVAL, "adjoint workspace must be 256-byte aligned");
    AdjLayout L = adj_layout(d);
    const size_t need = multi ? L.total : L.single;
    if (adj_ws_bytes < need) return fail(LBM_ENOMEM, "adjoint workspace %zu < %zu bytes", adj_ws_bytes, need);
    return LBM_OK;
}

lbm_status adjoint_reduce(lbm_domain* d, char* w, double* grad, hipStream_t stream) {
    AdjLayout L = adj_layout(d);
    const long nb = (long)d->nxb * ((d->p.ny + ADJ_TY - 1) / ADJ_TY);
    hipLaunchKernelGGL(lbm::k_adj_accumulate, dim3(1), dim3(lbm::NT), 0, stream,
                       reinterpret_cast<const double*>(w + 4 * L.plane), nb, grad);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}
}  // namespace

lbm_status lbm_adjoint_step(lbm_domain* d, const void* state_t, const double* lam_next, double* lam_t, double* grad,
                            void* adj_ws, size_t adj_ws_bytes, hipStream_t stream) {
    if (!d || !state_t || !lam_next || !lam_t || !grad || !adj_ws) return fail(LBM_EINVAL, "NULL argument");
    if (lam_next == lam_t) return fail(LBM_EINVAL, "lam_next and lam_t must be distinct buffers");
    lbm_status st = adjoint_check(d, adj_ws, adj_ws_bytes);
    if (st != LBM_OK) return st;
    char* w = static_cast<char*>(adj_ws);
    st = adjoint_kernels(d, state_t, lam_next, lam_t, w, 0, stream);
    if (st != LBM_OK) return st;
    return adjoint_reduce(d, w, grad, stream);
}

lbm_status lbm_adjoint_steps(lbm_domain* d, const void* states, size_t stride, int64_t nsteps, double* lam,
                             double* lam_tmp, double* grad, void* adj_ws, size_t adj_ws_bytes, hipStream_t stream) {
    if (!d || !states || !lam || !lam_tmp || !grad || !adj_ws) return fail(LBM_EINVAL, "NULL argument");
    if (lam == lam_tmp) return fail(LBM_EINVAL, "lam and lam_tmp must be distinct buffers");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
    if (((uintptr_t)states & 255) != 0 || (stride & 255) != 0) return fail(LBM_EINVAL, "states and stride must be 256-byte aligned");
    if (stride < f_bytes(d) + phi_bytes(d)) return fail(LBM_EINVAL, "stride %zu < state bytes %zu", stride, f_bytes(d) + phi_bytes(d));
    lbm_status st = adjoint_check(d, adj_ws, adj_ws_bytes, true);
    if (st != LBM_OK) return st;
    if (nsteps == 0) return LBM_OK;
    char* w = static_cast<char*>(adj_ws);
    const char* base = static_cast<const char*>(states);
    double* cur = lam;
    double* nxt = lam_tmp;
    // Where the y derivatives are column marches (large lattices, where the
    // step is bound by its bytes) inner steps pass the cotangent in factored
    // form (AdjArgs::add_next): the first step reads the caller's full lam,
    // the last writes full planes.  On small lattices the nine extra gathers
    // of the scalar plane cost more latency than the 17 words save
    // (1024^2: 0.131 -> 0.160 ms; 4096^2: 1.84 -> 1.61 ms).
    double* addp = adj_dy_chunks(d) > 0 ? reinterpret_cast<double*>(w + adj_layout(d).single) : nullptr;
    for (int64_t t = nsteps - 1; t >= 0; --t) {
        st = adjoint_kernels(d, base + (size_t)t * stride, cur, nxt, w, t == nsteps - 1 ? 0 : 1, stream,
                             t == nsteps - 1 ? nullptr : addp, t == 0 ? nullptr : addp);
        if (st != LBM_OK) return st;
        double* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    st = adjoint_reduce(d, w, grad, stream);
    if (st != LBM_OK) return st;
    if (cur != lam) {
        const size_t lb = (size_t)lbm::Q * d->p.nx * d->p.ny * sizeof(double);
        HIP_TRY(hipMemcpyAsync(lam, cur, lb, hipMemcpyDeviceToDevice, stream));
    }
    return LBM_OK;
}

}  // extern "C"

namespace {
// Scratch of lbm_adjoint_step_noalloc: one fixed array per device, resident
// for the life of the process.  In host code `scratch` only names the symbol;
// its device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and only that address is used.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(32) << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array (the current device).
lbm_status scratch_address(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(LBM_EDEVICE, "device index %d beyond %d", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LBM_EDEVICE, "scratch array address on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}
}  // namespace

extern "C" {

lbm_status lbm_adjoint_step_noalloc(lbm_domain* d, const void* state_t, const double* lam_next, double* lam_t,
                                    double* grad, hipStream_t stream) {
    if (!d || !state_t || !lam_next || !lam_t || !grad) return fail(LBM_EINVAL, "NULL argument");
    if (lam_next == lam_t) return fail(LBM_EINVAL, "lam_next and lam_t must be distinct buffers");
    const size_t need = adj_layout(d).single;
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(LBM_EINVAL, "lattice %d x %d needs %zu bytes of adjoint scratch, more than the %zu of the fixed array",
                    d->p.nx, d->p.ny, need, NOALLOC_SCRATCH_BYTES);
    void* ptr = nullptr;
    lbm_status st = scratch_address(&ptr);
    if (st != LBM_OK) return st;
    st = adjoint_check(d, ptr, NOALLOC_SCRATCH_BYTES);
    if (st != LBM_OK) return st;
    char* w = static_cast<char*>(ptr);
    st = adjoint_kernels(d, state_t, lam_next, lam_t, w, 0, stream);
    if (st != LBM_OK) return st;
    return adjoint_reduce(d, w, grad, stream);
}

size_t lbm_adjoint_noalloc_max_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

lbm_status lbm_adjoint_rho0(lbm_domain* d, const double* lam0, const double* ux0, const double* uy0, double* drho0,
                            hipStream_t stream) {
    if (!d || !lam0 || !drho0) return fail(LBM_EINVAL, "NULL argument");
    const long n = (long)d->p.nx * d->p.ny;
    hipLaunchKernelGGL(lbm::k_adj_rho0, dim3(grid_1d(n)), dim3(lbm::NT), 0, stream, lam0, ux0, uy0,
                       n, drho0);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

void lbm_destroy(lbm_domain* d) { delete d; }

}  // extern "C"

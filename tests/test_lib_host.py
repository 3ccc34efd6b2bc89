"""Host-side checks of the HIP library that need no GPU: the shared library
loads, exports every entry point include/lbm.h declares, its host EOS and HDM
utilities agree with the oracle, and invalid arguments are rejected."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
import oracle_pins as PINS
import paper_1712_06079_amd as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = L.library()
    names = declared_symbols()
    assert len(names) >= 14, names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("kind", ["vdw", "pr", "cs", "rk", "rks"])
def test_critical_point_matches_oracle(kind):
    po = PINS.eos_params(kind)
    p = L.Params(eos=kind, a=po.a, b=po.b, R=po.R, omega=po.omega, k=po.k)
    tc, rc = L.critical(p)
    tco, rco = O.critical(po)
    assert abs(tc / tco - 1) < 1e-12 and abs(rc / rco - 1) < 1e-9, (tc, tco, rc, rco)


@pytest.mark.parametrize("kind,trs", [("vdw", (0.4, 0.6, 0.9, 0.99)), ("cs", (0.5, 0.6, 0.7, 0.95)),
                                      ("pr", (0.5, 0.7, 0.95)), ("rk", (0.6, 0.9)), ("rks", (0.6, 0.9))])
def test_maxwell_matches_oracle(kind, trs):
    po = PINS.eos_params(kind)
    p = L.Params(eos=kind, a=po.a, b=po.b, R=po.R, omega=po.omega, k=po.k)
    tc, _ = O.critical(po)
    for tr in trs:
        rv, rl, p0 = L.maxwell(p, tr * tc)
        rvo, rlo, p0o = O.maxwell(po, tr * tc)
        assert abs(rv / rvo - 1) < 1e-10 and abs(rl / rlo - 1) < 1e-11, (kind, tr, rv, rvo, rl, rlo)
        assert abs(p0 / p0o - 1) < 1e-9


def test_maxwell_rejects_supercritical():
    p = L.Params()
    with pytest.raises(L.LBMError):
        L.maxwell(p, 1.01 * 4 / 7)


@pytest.mark.parametrize("n", [5, 6, 8, 16, 17, 63, 64, 78, 79, 80, 81, 128, 1000])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_explicit_hdm_row_matches_chasing_solve(n, prec):
    """The kernels' explicit circulant form of Eq. 20 reproduces the oracle's
    Thomas + Sherman-Morrison solve on random periodic data (to the truncation
    tail for long lines: 39 taps with FP64 populations, 28 with FP32)."""
    d = np.array(L.hdm_row(n, prec))
    rng = np.random.default_rng(n)
    u = rng.standard_normal(n)
    ref = O.hdm_line(u)
    i = np.arange(n)
    got = np.zeros(n)
    for j in range(1, len(d) + 1):
        got += d[j - 1] * (u[(i + j) % n] - u[(i - j) % n])
    tol = 3e-15 if prec == "f64" else 2e-11
    assert np.max(np.abs(got - ref)) < tol * np.max(np.abs(ref)), np.max(np.abs(got - ref))


def test_invalid_parameters_rejected_without_device():
    lib = L.library()
    for bad in (dict(nx=4), dict(ny=3), dict(tau=0.5), dict(T=-1.0), dict(k=0.0), dict(eos="vdw", a=-1.0),
                dict(nx=(1 << 21) + 1, ny=5), dict(nx=5, ny=(1 << 21) + 1), dict(nx=1 << 16, ny=(1 << 15) + 1)):
        p = L.Params(**bad)
        nb = C.c_size_t()
        st = lib.lbm_workspace_bytes(C.byref(p.c()), C.byref(nb))
        assert st == 1, bad
        h = C.c_void_p()
        st = lib.lbm_init(C.byref(p.c()), None, 0, None, None, None, None, C.byref(h))
        assert st == 1 and lib.lbm_last_error(), bad


def test_setters_reject_null_domain():
    """The host-only tuning setters validate their handle without a device."""
    lib = L.library()
    assert lib.lbm_set_kernel(None, 0, 0) == 1
    assert lib.lbm_set_chunks(None, 0) == 1
    assert lib.lbm_set_access(None, 0) == 1
    v = C.c_int32()
    assert lib.lbm_kernel_choice(None, C.byref(v), C.byref(v), C.byref(v), C.byref(v)) == 1
    assert b"NULL" in lib.lbm_last_error()


def test_largest_sides_accepted():
    """Sides up to 2^21 and nx ny up to 2^31 pass validation (the kernels'
    24-bit index arithmetic holds there)."""
    lib = L.library()
    for nx, ny in ((1 << 21, 5), (5, 1 << 21), (1 << 16, 1 << 15), (1 << 21, 1 << 10)):
        nb = C.c_size_t()
        assert lib.lbm_workspace_bytes(C.byref(L.Params(nx=nx, ny=ny).c()), C.byref(nb)) == 0, (nx, ny)


def test_workspace_size_formula():
    lib = L.library()
    for prec, es in (("f64", 8), ("f32", 4)):
        p = L.Params(nx=100, ny=37, prec=prec)
        nb = C.c_size_t()
        assert lib.lbm_workspace_bytes(C.byref(p.c()), C.byref(nb)) == 0
        pitch = 128
        assert nb.value >= 2 * 9 * pitch * 37 * es + 2 * pitch * 37 * es


@pytest.mark.parametrize("nsteps,every", [(-1, 70), (10, 0), (10, -3), (2.5, 70), (10, 1.5)])
def test_rollout_rejects_bad_schedule(nsteps, every):
    """The differentiable rollout validates its checkpoint schedule before it
    touches the device."""
    from paper_1712_06079_amd.autograd import _check_schedule
    with pytest.raises(ValueError):
        _check_schedule(nsteps, every)


@pytest.mark.parametrize("kind,tr,kappa", [("vdw", 0.9, 0.004), ("vdw", 0.6, 0.02), ("cs", 0.7, 0.05), ("pr", 0.8, 0.01),
                                           ("rks", 0.75, 0.005)])
def test_flat_profile_matches_oracle(kind, tr, kappa):
    """The exact flat-interface profile of Eqs. 25-26 (library: closed-form W,
    Runge-Kutta steps of h/64; oracle: W by quadrature, steps of h/32) agree to
    the integration error (the densities within 1e-6 relative, the slopes within
    1e-6 of the steepest) on interfaces a few lattice units wide."""
    po = PINS.eos_params(kind)
    tc, _ = O.critical(po)
    po.T = tr * tc
    p = L.Params(eos=kind, a=po.a, b=po.b, R=po.R, omega=po.omega, k=po.k, T=po.T)
    _, r, d = L.flat_profile(p, kappa, 0.5, 121)
    _, r2, d2 = O.flat_profile(po, kappa, 0.5, 121)
    assert np.max(np.abs(r - r2) / r2) < 1e-6
    assert np.max(np.abs(d - d2)) < 1e-6 * d2.max()


def test_sigma_slab_matches_oracle():
    """Integration-method surface tension of a periodic slab column (Eq. 20
    derivative): library and oracle within rounding, for a short column (whole
    periodic row) and a long one (truncated row)."""
    rng = np.random.default_rng(31)
    for n in (40, 256):
        col = 2.0 + np.sin(2 * np.pi * np.arange(n) / n) + 0.1 * rng.standard_normal(n)
        s, d = L.sigma_slab(0.01, col)
        assert abs(s / O.sigma_slab(0.01, col) - 1) < 1e-13
        assert np.max(np.abs(d - O.hdm_line(col))) < 1e-14 * np.abs(O.hdm_line(col)).max()


def test_flat_interface_rejects_bad_input():
    p = L.Params(eos="vdw", T=0.6, k=0.01)  # T > Tc = 4/7
    with pytest.raises(L.LBMError):
        L.flat_profile(p, 0.01, 0.5, 11)
    p.T = 0.5
    with pytest.raises(L.LBMError):
        L.flat_profile(p, -1.0, 0.5, 11)

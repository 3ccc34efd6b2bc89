"""ctypes wrapper of the FP64 C++ oracle (TEST INFRASTRUCTURE ONLY).

Population layout: f[i, y, x] (9 planes of ny x nx), D2Q9 velocity order
0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1).
"""
import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

EOS = {"vdw": 0, "pr": 1, "cs": 2, "rk": 3, "rks": 4}
FORCE = {"sc": 0, "zc": 1, "hybrid": 2}
GRAD = {"hdm": 0, "cdm": 1, "cdm9": 2}

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


class _P(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("eos", C.c_int32), ("force", C.c_int32),
                ("grad", C.c_int32), ("walls", C.c_int32), ("tau", C.c_double), ("a", C.c_double),
                ("b", C.c_double), ("R", C.c_double), ("omega", C.c_double), ("T", C.c_double),
                ("k", C.c_double), ("g", C.c_double), ("A", C.c_double)]


@dataclass
class Params:
    nx: int = 64
    ny: int = 64
    eos: str = "vdw"
    force: str = "sc"
    grad: str = "hdm"
    tau: float = 1.0
    a: float = 9.0 / 49.0
    b: float = 2.0 / 21.0
    R: float = 1.0
    omega: float = 0.344
    T: float = 0.9 * 4.0 / 7.0
    k: float = 0.01
    g: float = 1.0
    A: float = 0.0
    walls: int = 0

    def c(self) -> _P:
        return _P(self.nx, self.ny, EOS[self.eos], FORCE[self.force], GRAD[self.grad], int(self.walls),
                  self.tau, self.a, self.b, self.R, self.omega, self.T, self.k, self.g, self.A)


_D = C.POINTER(C.c_double)


def load(path: str):
    """Bind the oracle API of the shared library at `path`."""
    L = C.CDLL(path)
    P = C.POINTER(_P)
    L.orc_critical.argtypes = [P, _D, _D]
    L.orc_maxwell.argtypes = [P, C.c_double, _D, _D, _D]
    L.orc_eos.argtypes = [P, C.c_double, C.c_double, _D, _D, _D]
    L.orc_hdm_line.argtypes = [C.c_int, _D, _D]
    L.orc_cdm_line.argtypes = [C.c_int, _D, _D]
    L.orc_gradient.argtypes = [P, _D, _D, _D]
    L.orc_hdm_line_walls.argtypes = [C.c_int, _D, _D]
    L.orc_cdm_line_walls.argtypes = [C.c_int, _D, _D]
    L.orc_flat_profile.argtypes = [P, C.c_double, C.c_double, C.c_int, _D, _D]
    L.orc_flat_profile.restype = C.c_int
    L.orc_sigma_slab.argtypes = [C.c_double, C.c_int, _D]
    L.orc_sigma_slab.restype = C.c_double
    L.orc_sigma_exact.argtypes = [P, C.c_double, _D]
    L.orc_sigma_exact.restype = C.c_int
    L.orc_feq.argtypes = [C.c_double, C.c_double, C.c_double, _D]
    L.orc_collide_cell.argtypes = [_D, C.c_double, C.c_double, C.c_double, _D]
    L.orc_init.argtypes = [P, _D, _D, _D, _D]
    L.orc_run.argtypes = [P, C.c_int64, _D]
    L.orc_moments.argtypes = [P, _D, _D, _D, _D, _D, _D, _D]
    L.orc_tangent_run.argtypes = [P, C.c_int64, _D, _D, C.c_double, C.c_double]
    L.orc_threads.argtypes = []
    L.orc_adjoint_step.argtypes = [P, _D, _D, _D, _D]
    L.orc_adjoint_run.argtypes = [P, C.c_int64, C.c_int64, _D, _D, _D, _D, _D, _D, _D, _D]
    for fn in ("orc_critical", "orc_maxwell", "orc_run", "orc_tangent_run", "orc_threads", "orc_adjoint_step",
               "orc_adjoint_run"):
        getattr(L, fn).restype = C.c_int
    return L


_lib = None


def lib():
    """The oracle library used by the module-level functions (built on demand)."""
    global _lib
    if _lib is None:
        _lib = load(_build.build(force=False))
    return _lib


def use(L):
    """Route the module-level functions to another build of the oracle (returns the previous one)."""
    global _lib
    prev, _lib = _lib, L
    return prev


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().orc_threads())


def critical(p: Params):
    tc, rc = C.c_double(), C.c_double()
    rc_ = lib().orc_critical(C.byref(p.c()), C.byref(tc), C.byref(rc))
    if rc_:
        raise ValueError("critical point not found")
    return tc.value, rc.value


def maxwell(p: Params, T: float):
    rv, rl, p0 = C.c_double(), C.c_double(), C.c_double()
    rc = lib().orc_maxwell(C.byref(p.c()), T, C.byref(rv), C.byref(rl), C.byref(p0))
    if rc:
        raise ValueError(f"no coexistence at T={T} (code {rc})")
    return rv.value, rl.value, p0.value


def eos(p: Params, rho: float, T: float):
    pe, d1, d2 = C.c_double(), C.c_double(), C.c_double()
    lib().orc_eos(C.byref(p.c()), rho, T, C.byref(pe), C.byref(d1), C.byref(d2))
    return pe.value, d1.value, d2.value


def hdm_line(u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    lib().orc_hdm_line(len(u), _ptr(u), _ptr(out))
    return out


def cdm_line(u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    lib().orc_cdm_line(len(u), _ptr(u), _ptr(out))
    return out


def gradient(p: Params, u):
    """(d/dx, d/dy) of a field u [ny, nx] with the step's gradient scheme p.grad."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.shape == (p.ny, p.nx)
    gx, gy = np.empty_like(u), np.empty_like(u)
    lib().orc_gradient(C.byref(p.c()), _ptr(u), _ptr(gx), _ptr(gy))
    return gx, gy


def flat_profile(p: Params, kappa: float, h: float, n: int):
    """Exact flat-interface profile of Eqs. 25-26 with the k-scaled EOS:
    (y, rho, drho/dy) at y_i = (i - (n-1)/2) h, rising through the mean density at y = 0."""
    rho, drho = np.empty(n), np.empty(n)
    if lib().orc_flat_profile(C.byref(p.c()), kappa, h, n, _ptr(rho), _ptr(drho)):
        raise ValueError("no flat interface for these parameters")
    return (np.arange(n) - 0.5 * (n - 1)) * h, rho, drho


def sigma_slab(kappa: float, rho_column):
    """Integration-method surface tension of one interface of a periodic slab column (h = 1)."""
    r = np.ascontiguousarray(rho_column, dtype=np.float64)
    return float(lib().orc_sigma_slab(kappa, len(r), _ptr(r)))


def sigma_exact(p: Params, kappa: float):
    """integral sqrt(2 kappa W) d rho: the integration method on the exact profile."""
    s = C.c_double()
    if lib().orc_sigma_exact(C.byref(p.c()), kappa, C.byref(s)):
        raise ValueError("no flat interface for these parameters")
    return s.value


def hdm_line_walls(u):
    """Eq. 20 on a line between two walls (mirror closure)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    lib().orc_hdm_line_walls(len(u), _ptr(u), _ptr(out))
    return out


def cdm_line_walls(u):
    """Eq. 14 on a line between two walls (mirror closure)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    lib().orc_cdm_line_walls(len(u), _ptr(u), _ptr(out))
    return out


def feq(rho, ux, uy):
    out = np.empty(9)
    lib().orc_feq(rho, ux, uy, _ptr(out))
    return out


def collide_cell(f9, Fx, Fy, tau):
    f9 = np.ascontiguousarray(f9, dtype=np.float64)
    out = np.empty(9)
    lib().orc_collide_cell(_ptr(f9), Fx, Fy, tau, _ptr(out))
    return out


def init(p: Params, rho0, ux0=None, uy0=None):
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    assert rho0.shape == (p.ny, p.nx)
    ux0 = None if ux0 is None else np.ascontiguousarray(ux0, dtype=np.float64)
    uy0 = None if uy0 is None else np.ascontiguousarray(uy0, dtype=np.float64)
    f = np.empty((9, p.ny, p.nx))
    lib().orc_init(C.byref(p.c()), _ptr(rho0), _ptr(ux0), _ptr(uy0), _ptr(f))
    return f


def run(p: Params, f, nsteps: int):
    """Advance a copy of f by nsteps; returns the new state."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    assert f.shape == (9, p.ny, p.nx)
    if lib().orc_run(C.byref(p.c()), int(nsteps), _ptr(f)):
        raise ValueError("invalid parameters")
    return f


def moments(p: Params, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    outs = [np.empty((p.ny, p.nx)) for _ in range(6)]
    lib().orc_moments(C.byref(p.c()), _ptr(f), *[_ptr(o) for o in outs])
    return dict(zip(("rho", "vx", "vy", "p", "Fx", "Fy"), outs))


def tangent_run(p: Params, f, df, nsteps: int, dT: float = 0.0, dg: float = 0.0):
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    df = np.array(df, dtype=np.float64, order="C", copy=True)
    if lib().orc_tangent_run(C.byref(p.c()), int(nsteps), _ptr(f), _ptr(df), dT, dg):
        raise ValueError("invalid parameters")
    return f, df


def adjoint_step(p: Params, f, lam_next):
    """Reverse mode of one step at state f: returns (dJ/df_t, [dJ/dg, dJ/dT])."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    lam_next = np.ascontiguousarray(lam_next, dtype=np.float64)
    lam = np.empty_like(f)
    grad = np.zeros(2)
    if lib().orc_adjoint_step(C.byref(p.c()), _ptr(f), _ptr(lam_next), _ptr(lam), _ptr(grad)):
        raise ValueError("invalid parameters")
    return lam, grad


def adjoint_run(p: Params, rho0, target, nsteps: int, every: int = 70, ux0=None, uy0=None):
    """J = sum (rho_n - target)^2 after nsteps from f^eq(rho0, u0) and its gradients:
    returns dict(J, df0, drho0, dg, dT)."""
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    target = np.ascontiguousarray(target, dtype=np.float64)
    ux0 = None if ux0 is None else np.ascontiguousarray(ux0, dtype=np.float64)
    uy0 = None if uy0 is None else np.ascontiguousarray(uy0, dtype=np.float64)
    J = C.c_double()
    df0 = np.empty((9, p.ny, p.nx))
    drho0 = np.empty((p.ny, p.nx))
    grad = np.zeros(2)
    if lib().orc_adjoint_run(C.byref(p.c()), int(nsteps), int(every), _ptr(rho0), _ptr(ux0), _ptr(uy0), _ptr(target),
                             C.byref(J), _ptr(df0), _ptr(drho0), _ptr(grad)):
        raise ValueError("invalid parameters")
    return {"J": J.value, "df0": df0, "drho0": drho0, "dg": grad[0], "dT": grad[1]}

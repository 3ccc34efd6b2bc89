"""MI355X (gfx950) HDM pseudopotential lattice Boltzmann library: Python binding.

This module only marshals arguments to the C ABI of ``liblbm_hip.so`` (declared
in include/lbm.h); every step of the method runs in the library's HIP kernels.
PyTorch supplies device memory (the workspace and field tensors) and the
current stream.  Importing works without a GPU; creating a domain needs the
built library and a GPU and raises if either is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

__all__ = ["Params", "Domain", "Batch", "LBMError", "library", "critical", "maxwell", "hdm_row", "stream_probe",
           "interface_excess", "flat_profile", "sigma_slab", "EOS", "FORCE", "GRAD", "PREC"]

EOS = {"vdw": 0, "pr": 1, "cs": 2, "rk": 3, "rks": 4}
FORCE = {"sc": 0, "zc": 1, "hybrid": 2}
GRAD = {"hdm": 0, "cdm": 1, "cdm9": 2}
PREC = {"f64": 0, "f32": 1}
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbm_hip.so")


class LBMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lbm status {status}: {msg}")
        self.status = status


class _CParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("eos", C.c_int32), ("force", C.c_int32),
                ("grad", C.c_int32), ("prec", C.c_int32), ("tau", C.c_double), ("a", C.c_double),
                ("b", C.c_double), ("R", C.c_double), ("omega", C.c_double), ("T", C.c_double),
                ("k", C.c_double), ("g", C.c_double), ("A", C.c_double), ("walls", C.c_int32), ("reserved", C.c_int32)]


@dataclass
class Params:
    """Problem statement of one periodic domain (fields as in lbm_params)."""
    nx: int = 64
    ny: int = 64
    eos: str = "vdw"
    force: str = "sc"
    grad: str = "hdm"
    prec: str = "f64"
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

    def c(self) -> _CParams:
        return _CParams(self.nx, self.ny, EOS[self.eos], FORCE[self.force], GRAD[self.grad], PREC[self.prec],
                        self.tau, self.a, self.b, self.R, self.omega, self.T, self.k, self.g, self.A, int(self.walls), 0)


_lib = None
_VP = C.c_void_p


def library():
    """Load liblbm_hip.so (built by build.py); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run paper_1712_06079_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(_CParams)
        D = C.POINTER(C.c_double)
        L.lbm_critical.argtypes = [P, D, D]
        L.lbm_maxwell.argtypes = [P, C.c_double, D, D, D]
        L.lbm_workspace_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
        L.lbm_hdm_row.argtypes = [C.c_int32, C.c_int32, D, C.POINTER(C.c_int32)]
        L.lbm_init.argtypes = [P, _VP, C.c_size_t, _VP, _VP, _VP, _VP, C.POINTER(_VP)]
        L.lbm_step.argtypes = [_VP, C.c_int64, _VP]
        L.lbm_moments.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP, _VP]
        L.lbm_get_populations.argtypes = [_VP, _VP, _VP]
        L.lbm_set_populations.argtypes = [_VP, _VP, _VP]
        L.lbm_step_count.argtypes = [_VP]
        L.lbm_step_count.restype = C.c_int64
        L.lbm_set_kernel.argtypes = [_VP, C.c_int32, C.c_int32]
        L.lbm_set_chunks.argtypes = [_VP, C.c_int32]
        L.lbm_set_access.argtypes = [_VP, C.c_int32]
        L.lbm_kernel_choice.argtypes = [_VP] + [C.POINTER(C.c_int32)] * 4
        L.lbm_check_finite.argtypes = [_VP, C.POINTER(C.c_int32), _VP]
        L.lbm_state_bytes.argtypes = [_VP, C.POINTER(C.c_size_t)]
        L.lbm_save_state.argtypes = [_VP, _VP, _VP]
        L.lbm_load_state.argtypes = [_VP, _VP, _VP]
        L.lbm_adjoint_workspace_bytes.argtypes = [_VP, C.POINTER(C.c_size_t)]
        L.lbm_adjoint_step.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP, C.c_size_t, _VP]
        L.lbm_adjoint_rho0.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP]
        L.lbm_record.argtypes = [_VP, C.c_int64, _VP, C.c_size_t, _VP]
        L.lbm_adjoint_steps.argtypes = [_VP, _VP, C.c_size_t, C.c_int64, _VP, _VP, _VP, _VP, C.c_size_t, _VP]
        L.lbm_stream_probe.argtypes = [C.c_int32, _VP, _VP, C.c_size_t, C.c_int32, _VP]
        L.lbm_interface_excess.argtypes = [P, C.c_int32, D, D]
        L.lbm_flat_profile.argtypes = [P, C.c_double, C.c_double, C.c_int32, D, D]
        L.lbm_sigma_slab.argtypes = [C.c_double, C.c_int32, D, D, D]
        L.lbm_adjoint_step_noalloc.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP]
        L.lbm_adjoint_noalloc_max_bytes.argtypes = []
        L.lbm_adjoint_noalloc_max_bytes.restype = C.c_size_t
        L.lbm_destroy.argtypes = [_VP]
        L.lbm_destroy.restype = None
        L.lbm_last_error.restype = C.c_char_p
        for fn in ("lbm_critical", "lbm_maxwell", "lbm_workspace_bytes", "lbm_hdm_row", "lbm_init", "lbm_step", "lbm_moments",
                   "lbm_get_populations", "lbm_set_populations", "lbm_set_kernel", "lbm_set_chunks", "lbm_set_access", "lbm_kernel_choice", "lbm_check_finite",
                   "lbm_state_bytes", "lbm_save_state", "lbm_load_state", "lbm_adjoint_workspace_bytes",
                   "lbm_adjoint_step", "lbm_adjoint_rho0", "lbm_record", "lbm_adjoint_steps", "lbm_stream_probe",
                   "lbm_adjoint_step_noalloc", "lbm_interface_excess", "lbm_flat_profile", "lbm_sigma_slab"):
            getattr(L, fn).restype = C.c_int
        _lib = L
    return _lib


def check(status: int):
    if status != 0:
        raise LBMError(status, library().lbm_last_error().decode())


def critical(p: Params):
    tc, rc = C.c_double(), C.c_double()
    check(library().lbm_critical(C.byref(p.c()), C.byref(tc), C.byref(rc)))
    return tc.value, rc.value


def maxwell(p: Params, T: float):
    rv, rl, p0 = C.c_double(), C.c_double(), C.c_double()
    check(library().lbm_maxwell(C.byref(p.c()), T, C.byref(rv), C.byref(rl), C.byref(p0)))
    return rv.value, rl.value, p0.value


def hdm_row(n: int, prec: str = "f64"):
    """The explicit coefficients d_1..d_taps of Eq. 20 on n periodic points."""
    d = (C.c_double * 40)()
    taps = C.c_int32()
    check(library().lbm_hdm_row(n, PREC[prec], d, C.byref(taps)))
    return list(d)[:taps.value]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the HDM LBM library runs on an MI355X only")
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def interface_excess(p: Params, rho):
    """W(rho) of the flat interface (lbm_interface_excess) for a 1D float64 numpy array."""
    import numpy as np
    r = np.ascontiguousarray(rho, dtype=np.float64)
    W = np.empty_like(r)
    check(library().lbm_interface_excess(C.byref(p.c()), len(r), _dptr(r), _dptr(W)))
    return W


def flat_profile(p: Params, kappa: float, h: float, n: int):
    """(y, rho, rho') of the exact flat-interface profile (lbm_flat_profile)."""
    import numpy as np
    rho, drho = np.empty(n), np.empty(n)
    check(library().lbm_flat_profile(C.byref(p.c()), kappa, h, n, _dptr(rho), _dptr(drho)))
    return (np.arange(n) - 0.5 * (n - 1)) * h, rho, drho


def sigma_slab(kappa: float, column):
    """(sigma, D rho) of one interface of a periodic slab column (lbm_sigma_slab)."""
    import numpy as np
    r = np.ascontiguousarray(column, dtype=np.float64)
    d = np.empty_like(r)
    s = C.c_double()
    check(library().lbm_sigma_slab(kappa, len(r), _dptr(r), _dptr(d), C.byref(s)))
    return s.value, d


PROBE_KINDS = {"copy": 0, "read": 1, "write": 2}


def stream_probe(kind: str, src, dst, grid: int, stream=None):
    """One launch of the library's streaming probe (lbm_stream_probe): "copy"
    dst = src, "read" (dst receives one double per workgroup), "write" dst = 1;
    src / dst are CUDA tensors, the moved size is src's (dst's for "write")."""
    t = dst if kind == "write" else src
    nbytes = t.numel() * t.element_size()
    check(library().lbm_stream_probe(PROBE_KINDS[kind], _ptr(src), _ptr(dst), nbytes, int(grid), _stream(stream)))


class Domain:
    """One periodic domain on the current GPU.

    rho0 (and optional ux0, uy0) are FP64 tensors of shape (ny, nx) on the GPU.
    """

    def __init__(self, p: Params, rho0, ux0=None, uy0=None, stream=None):
        torch = _torch()
        L = library()
        self.p = p
        self._cp = p.c()
        nb = C.c_size_t()
        check(L.lbm_workspace_bytes(C.byref(self._cp), C.byref(nb)))
        dev = rho0.device
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nb.value]
        for t in (rho0, ux0, uy0):
            if t is not None:
                assert t.dtype == torch.float64 and t.is_cuda and t.shape == (p.ny, p.nx) and t.is_contiguous()
        self._keep = (rho0, ux0, uy0)
        h = C.c_void_p()
        check(L.lbm_init(C.byref(self._cp), _ptr(self._ws), nb.value, _ptr(rho0), _ptr(ux0), _ptr(uy0),
                         _stream(stream), C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lbm_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def set_kernel(self, variant: int = 0, tile_y: int = 0):
        """0 automatic, 1 two-pass reference, 2 fused tiles, 3 fused strip march.
        The variant also picks how the reverse step takes its y derivatives
        on a long y axis: column marches under 3, tiles under 1 and 2, and
        by lattice size under 0 (see lbm_set_kernel in include/lbm.h)."""
        check(library().lbm_set_kernel(self._h, variant, tile_y))

    def set_chunks(self, nchunk: int = 0):
        """y chunks per strip of the marching kernel (0 = automatic)."""
        check(library().lbm_set_chunks(self._h, nchunk))

    def set_access(self, access: int = 0):
        """Marching kernel's population accesses: 0 automatic (plain when the
        state fits in the last-level cache), 1 non-temporal, 2 plain."""
        check(library().lbm_set_access(self._h, access))

    def kernel_choice(self) -> dict:
        """What step() launches: kernel 1 (two-pass reference), 2 (tiles) or
        3 (strip march), rows (tile height or block rows), chunks (the march's
        y chunks per strip) and cached (plain population accesses)."""
        v = [C.c_int32() for _ in range(4)]
        check(library().lbm_kernel_choice(self._h, *[C.byref(x) for x in v]))
        return dict(zip(("kernel", "rows", "chunks", "cached"), (x.value for x in v)))

    def step(self, n: int = 1, stream=None):
        check(library().lbm_step(self._h, int(n), _stream(stream)))

    @property
    def steps(self) -> int:
        return int(library().lbm_step_count(self._h))

    def moments(self, stream=None, want=("rho", "vx", "vy", "p")):
        torch = _torch()
        dev = self._ws.device
        out = {k: torch.empty((self.p.ny, self.p.nx), dtype=torch.float64, device=dev) for k in want}
        tot = torch.empty(4, dtype=torch.float64, device=dev)
        check(library().lbm_moments(self._h, _ptr(out.get("rho")), _ptr(out.get("vx")), _ptr(out.get("vy")),
                                    _ptr(out.get("p")), _ptr(tot), _stream(stream)))
        out["totals"] = tot
        return out

    def populations(self, stream=None):
        torch = _torch()
        f = torch.empty((9, self.p.ny, self.p.nx), dtype=torch.float64, device=self._ws.device)
        check(library().lbm_get_populations(self._h, _ptr(f), _stream(stream)))
        return f

    def set_populations(self, f, stream=None):
        torch = _torch()
        assert f.dtype == torch.float64 and f.shape == (9, self.p.ny, self.p.nx) and f.is_contiguous()
        check(library().lbm_set_populations(self._h, _ptr(f), _stream(stream)))

    def check_finite(self, stream=None) -> bool:
        ok = C.c_int32()
        st = library().lbm_check_finite(self._h, C.byref(ok), _stream(stream))
        if st not in (0, 4):
            check(st)
        return bool(ok.value)

    # ---- snapshots and reverse mode -------------------------------------------------
    def state_bytes(self) -> int:
        nb = C.c_size_t()
        check(library().lbm_state_bytes(self._h, C.byref(nb)))
        return nb.value

    def new_states(self, n: int):
        """Device storage for n state snapshots (uint8 tensor [n, stride], stride
        = state bytes rounded up to 256; the caching allocator aligns the base)."""
        torch = _torch()
        sb = (self.state_bytes() + 255) // 256 * 256
        t = torch.empty((n, sb), dtype=torch.uint8, device=self._ws.device)
        if t.data_ptr() % 256:
            raise LBMError(1, "state storage is not 256-byte aligned")
        return t

    def record(self, states, nsteps: int, stream=None):
        """states[0] = current state, states[t+1] = state after t+1 steps (t < nsteps)."""
        if states.shape[0] < nsteps + 1:
            raise LBMError(1, f"record: {states.shape[0]} slots < nsteps + 1 = {nsteps + 1}")
        check(library().lbm_record(self._h, int(nsteps), _ptr(states), states.stride(0), _stream(stream)))

    def adjoint_steps(self, states, nsteps: int, lam, lam_tmp, grad, adj_ws, stream=None):
        """lam <- adjoint of nsteps steps over recorded `states` (slots nsteps-1 .. 0)."""
        check(library().lbm_adjoint_steps(self._h, _ptr(states), states.stride(0), int(nsteps), _ptr(lam), _ptr(lam_tmp),
                                          _ptr(grad), _ptr(adj_ws), adj_ws.numel(), _stream(stream)))

    def save_state(self, state, stream=None):
        check(library().lbm_save_state(self._h, _ptr(state), _stream(stream)))

    def load_state(self, state, stream=None):
        check(library().lbm_load_state(self._h, _ptr(state), _stream(stream)))

    def adjoint_workspace(self):
        torch = _torch()
        nb = C.c_size_t()
        check(library().lbm_adjoint_workspace_bytes(self._h, C.byref(nb)))
        return torch.empty(nb.value, dtype=torch.uint8, device=self._ws.device)

    def adjoint_step(self, state, lam_next, lam, grad, adj_ws, stream=None):
        """lam = (d step / d f_t)^T lam_next at `state`; grad[0] += dJ/dg, grad[1] += dJ/dT."""
        check(library().lbm_adjoint_step(self._h, _ptr(state), _ptr(lam_next), _ptr(lam), _ptr(grad), _ptr(adj_ws),
                                         adj_ws.numel(), _stream(stream)))

    def adjoint_step_noalloc(self, state, lam_next, lam, grad, stream=None):
        """adjoint_step with the library's fixed device scratch (lbm_adjoint_step_noalloc)."""
        check(library().lbm_adjoint_step_noalloc(self._h, _ptr(state), _ptr(lam_next), _ptr(lam), _ptr(grad),
                                                 _stream(stream)))

    def adjoint_rho0(self, lam0, ux0=None, uy0=None, stream=None):
        torch = _torch()
        out = torch.empty((self.p.ny, self.p.nx), dtype=torch.float64, device=self._ws.device)
        check(library().lbm_adjoint_rho0(self._h, _ptr(lam0), _ptr(ux0), _ptr(uy0), _ptr(out), _stream(stream)))
        return out


class _DomainView(Domain):
    """A domain owned by a Batch (borrowed handle; not destroyed on deletion)."""

    def __init__(self, batch, handle, p: Params):
        self._batch = batch
        self.p = p
        self._h = handle
        self._ws = batch._ws

    def __del__(self):
        pass


class Batch:
    """Many independent periodic domains stepped by one launch per step.

    params: list of Params (same prec and force); rho0s: list of FP64 CUDA
    tensors of shape (ny_i, nx_i).
    """

    _SIGS_DONE = False

    @classmethod
    def _sigs(cls):
        L = library()
        if cls._SIGS_DONE:
            return L
        P = C.POINTER(_CParams)
        L.lbm_batch_workspace_bytes.argtypes = [P, C.c_int32, C.POINTER(C.c_size_t)]
        L.lbm_batch_create.argtypes = [P, C.c_int32, _VP, C.c_size_t, C.POINTER(_VP), _VP, C.POINTER(_VP)]
        L.lbm_batch_step.argtypes = [_VP, C.c_int64, _VP]
        L.lbm_batch_step_separate.argtypes = [_VP, C.c_int64, _VP]
        L.lbm_batch_domain.argtypes = [_VP, C.c_int32]
        L.lbm_batch_domain.restype = _VP
        L.lbm_batch_set_schedule.argtypes = [_VP, C.c_int32, C.c_int32, C.c_int32, _VP]
        L.lbm_batch_get_schedule.argtypes = [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.lbm_batch_autotune.argtypes = [_VP, C.c_int32, _VP, C.c_char_p, C.c_size_t]
        L.lbm_batch_check_finite.argtypes = [_VP, C.POINTER(C.c_int32), _VP]
        L.lbm_batch_destroy.argtypes = [_VP]
        L.lbm_batch_destroy.restype = None
        L.lbm_batch_tune_cache_clear.argtypes = []
        L.lbm_batch_tune_cache_clear.restype = None
        for fn in ("lbm_batch_workspace_bytes", "lbm_batch_create", "lbm_batch_step", "lbm_batch_step_separate",
                   "lbm_batch_set_schedule", "lbm_batch_get_schedule", "lbm_batch_autotune", "lbm_batch_check_finite"):
            getattr(L, fn).restype = C.c_int
        cls._SIGS_DONE = True
        return L

    def __init__(self, params, rho0s, stream=None):
        torch = _torch()
        L = self._sigs()
        n = len(params)
        assert n == len(rho0s) and n >= 1
        self.params = list(params)
        self._cp = (_CParams * n)(*[p.c() for p in params])
        nb = C.c_size_t()
        check(L.lbm_batch_workspace_bytes(self._cp, n, C.byref(nb)))
        dev = rho0s[0].device
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nb.value]
        for p, t in zip(params, rho0s):
            assert t.dtype == torch.float64 and t.is_cuda and t.shape == (p.ny, p.nx) and t.is_contiguous()
        self._keep = list(rho0s)
        ptrs = (_VP * n)(*[t.data_ptr() for t in rho0s])
        h = C.c_void_p()
        check(L.lbm_batch_create(self._cp, n, _ptr(self._ws), nb.value, ptrs, _stream(stream), C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lbm_batch_destroy(h)
            self._h = None

    def __len__(self):
        return len(self.params)

    def step(self, n: int = 1, stream=None):
        check(self._sigs().lbm_batch_step(self._h, int(n), _stream(stream)))

    def step_separate(self, n: int = 1, stream=None):
        check(self._sigs().lbm_batch_step_separate(self._h, int(n), _stream(stream)))

    def domain(self, i: int) -> Domain:
        h = self._sigs().lbm_batch_domain(self._h, int(i))
        if not h:
            raise IndexError(i)
        return _DomainView(self, C.c_void_p(h), self.params[i])

    def set_schedule(self, tile_y: int, order: int, grid: int, stream=None):
        check(self._sigs().lbm_batch_set_schedule(self._h, tile_y, order, grid, _stream(stream)))

    def schedule(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        check(self._sigs().lbm_batch_get_schedule(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return {"tile_y": a.value, "order": b.value, "grid": c.value}

    @classmethod
    def tune_cache_clear(cls):
        """Forget the autotuner choices kept by this process."""
        cls._sigs().lbm_batch_tune_cache_clear()

    def autotune(self, probe_steps: int = 20, stream=None) -> dict:
        import json
        buf = C.create_string_buffer(8192)
        check(self._sigs().lbm_batch_autotune(self._h, probe_steps, _stream(stream), buf, len(buf)))
        return json.loads(buf.value.decode())

    def check_finite(self, stream=None):
        flags = (C.c_int32 * len(self.params))()
        st = self._sigs().lbm_batch_check_finite(self._h, flags, _stream(stream))
        if st not in (0, 4):
            check(st)
        return [bool(f) for f in flags]

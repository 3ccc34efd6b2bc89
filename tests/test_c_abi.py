"""The boundary is a C ABI: a C99 program that includes include/lbm.h and
links the built library calls its host entry points (no GPU needed) and gets
the values the Python binding gets."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

import paper_1712_06079_amd as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1712_06079_amd")

C_PROGRAM = r"""
#include "lbm.h"
#include <stdio.h>

int main(void) {
    lbm_params p = {0};
    double Tc = 0, rhoc = 0, rv = 0, rl = 0, p0 = 0, d[40];
    int32_t taps = 0;
    size_t bytes = 0;
    p.nx = 4096; p.ny = 4096; p.eos = LBM_EOS_CS; p.force = LBM_FORCE_SC; p.grad = LBM_GRAD_HDM;
    p.prec = LBM_F64; p.tau = 1.0; p.a = 1.0; p.b = 4.0; p.R = 1.0; p.k = 0.04; p.g = 1.0;
    if (lbm_critical(&p, &Tc, &rhoc) != LBM_OK) return 1;
    p.T = 0.5 * Tc;
    if (lbm_maxwell(&p, p.T, &rv, &rl, &p0) != LBM_OK) return 2;
    if (lbm_workspace_bytes(&p, &bytes) != LBM_OK) return 3;
    if (lbm_hdm_row(4096, LBM_F64, d, &taps) != LBM_OK) return 4;
    printf("%.17g %.17g %.17g %.17g %.17g %zu %d %.17g %.17g\n", Tc, rhoc, rv, rl, p0, bytes, (int)taps, d[0], d[1]);
    p.tau = 0.5;  /* invalid: tau must exceed 1/2 */
    if (lbm_workspace_bytes(&p, &bytes) != LBM_EINVAL) return 5;
    printf("%s\n", lbm_last_error());
    return 0;
}
"""


@pytest.fixture(scope="module")
def c_program(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    if not os.path.exists(os.path.join(LIBDIR, "liblbm_hip.so")):
        pytest.skip("library not built")
    d = tmp_path_factory.mktemp("cabi")
    src = d / "abi.c"
    src.write_text(C_PROGRAM)
    exe = d / "abi"
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe), "-L" + LIBDIR, "-llbm_hip",
           "-Wl,-rpath," + LIBDIR]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_header_compiles_as_c99_and_links(c_program):
    r = subprocess.run([str(c_program)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)


def test_c_caller_gets_the_binding_values(c_program):
    r = subprocess.run([str(c_program)], capture_output=True, text=True, timeout=60)
    lines = r.stdout.strip().splitlines()
    v = lines[0].split()
    Tc, rhoc, rv, rl, p0 = (float(x) for x in v[:5])
    bytes_, taps, d1, d2 = int(v[5]), int(v[6]), float(v[7]), float(v[8])
    p = L.Params(nx=4096, ny=4096, eos="cs", force="sc", a=1.0, b=4.0, R=1.0, k=0.04, tau=1.0)
    tc, rc = L.critical(p)
    assert (Tc, rhoc) == (tc, rc)
    p.T = 0.5 * tc
    rv2, rl2, p02 = L.maxwell(p, p.T)
    assert (rv, rl, p0) == (rv2, rl2, p02)
    wb = C.c_size_t()
    L.check(L.library().lbm_workspace_bytes(C.byref(p.c()), C.byref(wb)))
    assert bytes_ == wb.value > 2 * 9 * 8 * 4096 * 4096
    row = L.hdm_row(4096, "f64")
    assert taps == len(row) == 39
    assert (d1, d2) == (float(row[0]), float(row[1]))
    # the closed-form infinite-line values (the 4096-point row equals them to rounding)
    assert abs(d1 - 0.8790958567710524) < 1e-15 and abs(d2 + 0.3039542369798239) < 1e-15
    assert "tau" in lines[1]

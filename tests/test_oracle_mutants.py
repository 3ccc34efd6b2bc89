"""Plant plausible mistakes in copies of the oracle and check that the pins catch them.

Each mutant is one textual change to ``oracle/lbm_oracle.cpp`` (a dropped term,
a wrong sign, coefficient, index or operand; every occurrence of the pattern is
replaced, and a mutant given as a list of changes applies all of them, so that
the same mistake can be planted in the forward step and in its adjoint),
compiled on the CPU into a temporary library.  The fast pins then run against that build; at least one
must fail.  Nothing here touches the GPU.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle as O
import oracle_pins as P

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "lbm_oracle.cpp")

MUTANTS = {
    "hdm_rhs_coefficient": ("rhs[i] = (up2 - um2) / 36.0 + 7.0 * (up1 - um1) / 9.0;",
                            "rhs[i] = (up2 - um2) / 18.0 + 7.0 * (up1 - um1) / 9.0;"),
    "hdm_rhs_dropped_far_term": ("rhs[i] = (up2 - um2) / 36.0 + 7.0 * (up1 - um1) / 9.0;",
                                 "rhs[i] = 7.0 * (up1 - um1) / 9.0;"),
    "hdm_rhs_wrong_index": ("S up2 = u[((i + 2) % n) * su]", "S up2 = u[((i + 3) % n) * su]"),
    "hdm_no_periodic_corner": ("const double beta = third, alph = third, gamma = -1.0;",
                               "const double beta = 0.0, alph = third, gamma = -1.0;"),
    "thomas_wrong_pivot": ("dp[i] = (d[i] - sub[i] * dp[i - 1]) / m;", "dp[i] = (d[i] - sub[i] * dp[i - 1]) / diag[i];"),
    "feq_quadratic_coefficient": ("4.5 * eu * eu", "3.0 * eu * eu"),
    "feq_dropped_u2": ("- 1.5 * uu)", ")"),
    "weights_diagonal": ("1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0}", "1.0 / 36.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0}"),
    "velocity_set": ("const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};", "const int EY[9] = {0, 0, 1, 0, -1, 1, -1, 1, -1};"),
    "stream_direction": ("int xd = (x + EX[i] + nx) % nx", "int xd = (x - EX[i] + nx) % nx"),
    "stream_transposed": ("int xd = (x + EX[i] + nx) % nx, yd = (y + EY[i] + ny) % ny;",
                          "int xd = (x + EY[i] + nx) % nx, yd = (y + EX[i] + ny) % ny;"),
    "force_sign_sc": ("fsx = -2.0 * s * w.phi[c] * w.gx[c];", "fsx = 2.0 * s * w.phi[c] * w.gx[c];"),
    "force_factor_sc": ("fsy = -2.0 * s * w.phi[c] * w.gy[c];", "fsy = -1.0 * s * w.phi[c] * w.gy[c];"),
    "force_transposed_gradient": ("fsy = -2.0 * s * w.phi[c] * w.gy[c];", "fsy = -2.0 * s * w.phi[c] * w.gx[c];"),
    "force_sign_zc": ("fzx = -w.gux[c];", "fzx = w.gux[c];"),
    "edm_scaled_by_tau": ("out[i] = fi[i] - (fi[i] - e0) / tau + (e1 - e0);", "out[i] = fi[i] - (fi[i] - e0) / tau + (e1 - e0) / tau;"),
    "bgk_sign": ("out[i] = fi[i] - (fi[i] - e0) / tau + (e1 - e0);", "out[i] = fi[i] + (fi[i] - e0) / tau + (e1 - e0);"),
    "momentum_uses_ex": ("jy = jy + (double)EY[i] * f[i * N + c];", "jy = jy + (double)EX[i] * f[i * N + c];"),
    "potential_cs2": ("return g * (m.p.k * p_eos_alpha<S>(m.p, rho, T, al) - rho / 3.0);",
                      "return g * (m.p.k * p_eos_alpha<S>(m.p, rho, T, al) - rho / 2.0);"),
    "potential_without_k": ("return g * (m.p.k * p_eos_alpha<S>(m.p, rho, T, al) - rho / 3.0);",
                            "return g * (p_eos_alpha<S>(m.p, rho, T, al) - rho / 3.0);"),
    "cs_garbled_denominator": ("/ (one_m * one_m * one_m) -", "/ (S(1.0) - eta * eta * eta) -"),
    "vdw_attraction_exponent": ("return rho * R * T / (S(1.0) - b * rho) - a * rho * rho;",
                                "return rho * R * T / (S(1.0) - b * rho) - a * rho;"),
    "pr_alpha_sqrt": ("S t = S(1.0) + m * (S(1.0) - sqrt(T / Tc));", "S t = S(1.0) + m * (S(1.0) - T / Tc);"),
    "pr_alpha_coefficient": ("(0.37464 + 1.54226 * w - 0.26992 * w * w)", "(0.37464 + 1.54226 * w + 0.26992 * w * w)"),
    "pr_attraction_denominator": ("(S(1.0) + 2.0 * b * rho - b * b * rho * rho)", "(S(1.0) + 2.0 * b * rho + b * b * rho * rho)"),
    "maxwell_measure": ("sum += 0.5 * hs * GL8_W[j] * (iso.P(rho) - p0) / rho;", "sum += 0.5 * hs * GL8_W[j] * (iso.P(rho) - p0);"),
    "phi_sign_branch": ("w.phi[c] = (val(U) >= 0.0) ? sqrt(U) : sqrt(-U);", "w.phi[c] = sqrt(val(U) >= 0.0 ? U : -U) * 0.5;"),
    "velocity_output_full_force": ("if (vx) vx[c] = (w.jx[c] + 0.5 * w.Fx[c]) / w.rho[c];", "if (vx) vx[c] = (w.jx[c] + w.Fx[c]) / w.rho[c];"),
    "pressure_output_sign": ("if (pr) pr[c] = w.rho[c] / 3.0 + w.U[c];", "if (pr) pr[c] = w.rho[c] / 3.0 - w.U[c];"),
    "dual_division_rule": ("return Dual(q, (x.d - q * y.d) / y.v);", "return Dual(q, (x.d + q * y.d) / y.v);"),
    "adjoint_stream_direction": ("mu[i] = lam_next[i * N + (size_t)yd * nx + xd];",
                                 "mu[i] = lam_next[i * N + (size_t)((y - EY[i] + ny) % ny) * nx + (x - EX[i] + nx) % nx];"),
    "adjoint_relaxation_factor": ("rb += mu[i] * ((1.0 / tau - 1.0) * a_r + b_r);", "rb += mu[i] * ((1.0 - 1.0 / tau) * a_r + b_r);"),
    "adjoint_transpose_sign": ("double phibar = -2.0 * s * wsc * (Fbx[c] * w.gx[c] + Fby[c] * w.gy[c]) - dax[c] - day[c];",
                               "double phibar = -2.0 * s * wsc * (Fbx[c] * w.gx[c] + Fby[c] * w.gy[c]) + dax[c] + day[c];"),
    "adjoint_dropped_local_phi": ("double phibar = -2.0 * s * wsc * (Fbx[c] * w.gx[c] + Fby[c] * w.gy[c]) - dax[c] - day[c];",
                                  "double phibar = - dax[c] - day[c];"),
    "adjoint_zc_sign": ("for (size_t c = 0; c < N; ++c) Ubar[c] += dax[c] + day[c];", "for (size_t c = 0; c < N; ++c) Ubar[c] -= dax[c] + day[c];"),
    "adjoint_momentum_e": ("lam[k * N + c] = (1.0 - 1.0 / tau) * mu[k] + rb + EX[k] * jbx_ + EY[k] * jby_;",
                           "lam[k * N + c] = (1.0 - 1.0 / tau) * mu[k] + rb + EX[k] * jbx_ + EX[k] * jby_;"),
    "adjoint_dA_dm": ("*dmx = WQ[i] * (3.0 * EX[i] + (9.0 * em * EX[i] - 3.0 * mx) / rho);", "*dmx = WQ[i] * (3.0 * EX[i] + (9.0 * em * EX[i] - 1.5 * mx) / rho);"),
    "dp_drho_cs": ("return R * T * (Z + e * Zp) - 2.0 * a * rho;", "return R * T * (Z + Zp) - 2.0 * a * rho;"),
    "d2q9_without_cs2_factor": ("acc = acc + (3.0 * WQ[i] * e) * u[(size_t)yn * nx + xn];",
                                "acc = acc + (WQ[i] * e) * u[(size_t)yn * nx + xn];"),
    "d2q9_axis_swapped": ("const int e = (axis == 0) ? EX[i] : EY[i];", "const int e = (axis == 0) ? EY[i] : EX[i];"),
    "d2q9_dropped_diagonals": ("for (int i = 1; i < 9; ++i) {\n                const int e", "for (int i = 1; i < 5; ++i) {\n                const int e"),
    "d2q9_neighbour_index": ("const int xn = (x + EX[i] + nx) % nx, yn = (y + EY[i] + ny) % ny;",
                             "const int xn = (x + EX[i] + nx) % nx, yn = (y - EY[i] + ny) % ny;"),
    "excess_W_measure": ("sum += 0.5 * hs * GL8_W[j] * f.k * (f.iso.P(s) - f.p0) / (s * s);",
                         "sum += 0.5 * hs * GL8_W[j] * f.k * (f.iso.P(s) - f.p0) / s;"),
    "excess_W_without_p0": ("sum += 0.5 * hs * GL8_W[j] * f.k * (f.iso.P(s) - f.p0) / (s * s);",
                            "sum += 0.5 * hs * GL8_W[j] * f.k * f.iso.P(s) / (s * s);"),
    "interface_slope_factor": ("return std::sqrt(2.0 * excess_W(f, rho) / kappa);", "return std::sqrt(excess_W(f, rho) / kappa);"),
    "profile_low_order_steps": ("r += dy * (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0;", "r += dy * k1;"),
    "sigma_slab_both_interfaces": ("return 0.5 * kappa * sum;", "return kappa * sum;"),
    "sigma_exact_without_two": ("std::sqrt(2.0 * kappa * excess_W(f, c + 0.5 * hs * GL8_X[j]))",
                                "std::sqrt(kappa * excess_W(f, c + 0.5 * hs * GL8_X[j]))"),
    "wall_closure_rows": ("    diag[0] -= third;\n    diag[n - 1] -= third;\n", ""),
    "wall_mirror_about_last_row": ("return j < 0 ? -1 - j : (j >= n ? 2 * n - 1 - j : j);", "return j < 0 ? -1 - j : (j >= n ? 2 * n - 2 - j : j);"),
    "bounce_back_keeps_direction": ("fout[opposite(i) * N + c] = fs[i];", "fout[i * N + c] = fs[i];"),
    "walls_ignored_in_force": ("derivative<S>(m.p.grad, 1, nx, ny, w.phi.data(), w.gy.data(), m.p.walls);",
                               "derivative<S>(m.p.grad, 1, nx, ny, w.phi.data(), w.gy.data());"),
    # Eq. 9 weights, changed consistently in the forward force and its adjoint
    # (a mistake made in both passes survives the dot-product identity)
    "hybrid_sc_weight_both_passes": ("(1.0 - 2.0 * m.p.A)", "(1.0 - m.p.A)"),
    "hybrid_weights_swapped_both_passes": [
        ("w.Fx[c] = m.p.A * fzx + (1.0 - 2.0 * m.p.A) * fsx;", "w.Fx[c] = (1.0 - 2.0 * m.p.A) * fzx + m.p.A * fsx;"),
        ("w.Fy[c] = m.p.A * fzy + (1.0 - 2.0 * m.p.A) * fsy;", "w.Fy[c] = (1.0 - 2.0 * m.p.A) * fzy + m.p.A * fsy;"),
        ("const double wsc = (m.p.force == 2) ? (1.0 - 2.0 * m.p.A) : 1.0;", "const double wsc = (m.p.force == 2) ? m.p.A : 1.0;"),
        ("const double wzc = (m.p.force == 2) ? m.p.A : 1.0;", "const double wzc = (m.p.force == 2) ? (1.0 - 2.0 * m.p.A) : 1.0;"),
    ],
}


@pytest.fixture(scope="module")
def builds():
    tmp = tempfile.mkdtemp(prefix="oracle_mut_")
    src = open(SRC).read()
    libs, procs = {}, []
    for name, change in MUTANTS.items():
        text = src
        for old, new in (change if isinstance(change, list) else [change]):
            assert old in text, f"mutant {name}: pattern not found in the oracle source"
            text = text.replace(old, new)
        path = os.path.join(tmp, f"{name}.cpp")
        with open(path, "w") as fh:
            fh.write(text)
        lib = os.path.join(tmp, f"lib{name}.so")
        procs.append((name, lib, subprocess.Popen(
            ["g++", "-O1", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-o", lib, path])))
        libs[name] = lib
        if len(procs) >= 8:
            for n_, l_, pr in procs:
                assert pr.wait() == 0, n_
            procs = []
    for n_, l_, pr in procs:
        assert pr.wait() == 0, n_
    yield libs
    shutil.rmtree(tmp, ignore_errors=True)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(builds, name):
    prev = O.use(O.load(builds[name]))
    caught = None
    try:
        for pin in P.FAST:
            try:
                pin()
            except (AssertionError, ValueError, FloatingPointError, ZeroDivisionError):
                caught = pin.__name__
                break
    finally:
        O.use(prev)
    assert caught, f"no pin catches mutant {name}"

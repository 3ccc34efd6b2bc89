"""lbm_adjoint_step_noalloc (through the C ABI) against lbm_adjoint_step: the
same reverse step with the library's fixed device scratch instead of a
caller-provided workspace.  Two calls in a row on different domains, the
second smaller; then the size limit."""
import numpy as np
import pytest

import lbm_inputs as I
import oracle as O
import oracle_pins as PINS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1712_06079_amd as L  # noqa: E402


def _domain(eos, force, nx, ny, seed):
    po = PINS.eos_params(eos)
    po.nx, po.ny, po.force, po.tau = nx, ny, force, 0.8
    tc, _ = O.critical(po)
    po.T = 0.7 * tc
    rv, rl, _ = O.maxwell(po, po.T)
    rho0 = I.droplet(nx, ny, rv, rl, min(nx, ny) / 3.5, 4.0, cx=nx * 0.45, cy=ny * 0.55, noise=1e-2 * rv, seed=seed)
    p = L.Params(nx=nx, ny=ny, eos=eos, force=force, prec="f64", tau=po.tau, a=po.a, b=po.b, R=po.R, omega=po.omega,
                 T=po.T, k=po.k)
    d = L.Domain(p, torch.from_numpy(rho0).cuda())
    d.step(5)
    return d


def _both(d, seed):
    st = d.new_states(1)
    d.save_state(st[0])
    ny, nx = d.p.ny, d.p.nx
    g = torch.Generator(device="cuda").manual_seed(seed)
    lam_next = torch.randn((9, ny, nx), dtype=torch.float64, device="cuda", generator=g)
    lam_a = torch.empty_like(lam_next)
    lam_b = torch.full_like(lam_next, float("nan"))
    grad_a = torch.zeros(2, dtype=torch.float64, device="cuda")
    grad_b = torch.zeros(2, dtype=torch.float64, device="cuda")
    d.adjoint_step(st[0], lam_next, lam_a, grad_a, d.adjoint_workspace())
    d.adjoint_step_noalloc(st[0], lam_next, lam_b, grad_b)
    torch.cuda.synchronize()
    return lam_a.cpu().numpy(), lam_b.cpu().numpy(), grad_a.cpu().numpy(), grad_b.cpu().numpy()


def test_noalloc_matches_workspace_entry_point_twice():
    """Same kernels, same inputs: the results agree bitwise (the bar of the
    parity tests, 1e-12 relative, is met with room).  The second call uses a
    smaller lattice, so stale scratch contents of the first would show."""
    for eos, force, nx, ny, seed in (("cs", "sc", 300, 200, 1), ("vdw", "zc", 70, 37, 2)):
        d = _domain(eos, force, nx, ny, seed)
        la, lb, ga, gb = _both(d, seed)
        assert np.all(np.isfinite(lb)), (nx, ny)
        assert np.array_equal(la, lb), (nx, ny, float(np.max(np.abs(la - lb))))
        assert np.array_equal(ga, gb), (nx, ny, ga, gb)
        del d


def test_noalloc_rejects_lattices_beyond_the_fixed_scratch():
    cap = L.library().lbm_adjoint_noalloc_max_bytes()
    assert cap == 32 << 20
    d = _domain("cs", "sc", 1024, 1024, 3)
    st = d.new_states(1)
    d.save_state(st[0])
    lam_next = torch.zeros((9, 1024, 1024), dtype=torch.float64, device="cuda")
    lam = torch.empty_like(lam_next)
    grad = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LBMError) as e:
        d.adjoint_step_noalloc(st[0], lam_next, lam, grad)
    assert e.value.status == 1 and "scratch" in str(e.value)

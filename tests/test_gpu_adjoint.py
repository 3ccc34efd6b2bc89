"""GPU reverse mode (lbm_adjoint_step through the C ABI, and the autograd
rollout built on it) against the CPU oracle's adjoint and against differences."""
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
from paper_1712_06079_amd.autograd import rollout  # noqa: E402


def lib_params(po):
    return L.Params(nx=po.nx, ny=po.ny, eos=po.eos, force=po.force, grad=po.grad, prec="f64", tau=po.tau, a=po.a,
                    b=po.b, R=po.R, omega=po.omega, T=po.T, k=po.k, g=po.g, A=po.A)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def case(eos, force, nx, ny, tr=0.7, tau=0.8, seed=3):
    po = PINS.eos_params(eos)
    po.nx, po.ny, po.force, po.tau = nx, ny, force, tau
    tc, _ = O.critical(po)
    po.T = tr * tc
    rv, rl, _ = O.maxwell(po, po.T)
    rho0 = I.droplet(nx, ny, rv, rl, min(nx, ny) / 3.5, 4.0, cx=nx * 0.45, cy=ny * 0.55, noise=1e-2 * rv, seed=seed)
    return po, rho0, rv, rl


@pytest.mark.parametrize("eos,force,nx,ny,variant", [
    ("cs", "sc", 70, 37, 0), ("vdw", "zc", 64, 64, 0), ("pr", "sc", 33, 80, 0), ("rks", "zc", 130, 17, 0),
    ("rk", "sc", 96, 96, 0), ("cs", "zc", 5, 9, 0),
    # y derivatives by the column march: one chunk, ragged rows and columns, several chunks
    ("pr", "sc", 33, 80, 3), ("rk", "sc", 96, 96, 3), ("cs", "zc", 40, 120, 3), ("vdw", "sc", 70, 203, 3),
    ("cs", "zc", 64, 512, 3), ("rks", "sc", 130, 300, 3)])
def test_adjoint_step_matches_oracle(eos, force, nx, ny, variant):
    """One reverse step at a non-trivial state with a random cotangent."""
    po, rho0, _, _ = case(eos, force, nx, ny)
    f_t = O.run(po, O.init(po, rho0), 5)
    lam_next = np.random.default_rng(nx * ny).standard_normal(f_t.shape)
    ref_lam, ref_grad = O.adjoint_step(po, f_t, lam_next)
    d = L.Domain(lib_params(po), dev(rho0))
    d.set_kernel(variant, 0)
    d.set_populations(dev(f_t))
    st = d.new_states(1)
    d.save_state(st[0])
    lam = torch.empty((9, ny, nx), dtype=torch.float64, device="cuda")
    grad = torch.zeros(2, dtype=torch.float64, device="cuda")
    d.adjoint_step(st[0], dev(lam_next), lam, grad, d.adjoint_workspace())
    got = lam.cpu().numpy()
    scale = np.abs(ref_lam).max()
    assert np.max(np.abs(got - ref_lam)) < 1e-11 * scale, np.max(np.abs(got - ref_lam)) / scale
    g = grad.cpu().numpy()
    assert abs(g[0] - ref_grad[0]) < 1e-10 * max(1.0, abs(ref_grad[0])), (g, ref_grad)
    assert abs(g[1] - ref_grad[1]) < 1e-10 * max(1.0, abs(ref_grad[1])), (g, ref_grad)


@pytest.mark.parametrize("force", ["sc", "zc"])
def test_rollout_gradient_matches_oracle(force):
    """J = sum (rho_n - target)^2 after 120 steps of a 48 x 40 CS droplet;
    gradients with respect to rho0, g and T from the checkpointed GPU adjoint
    against the oracle's checkpointed trajectory gradient."""
    po, rho0, _, _ = case("cs", force, 48, 40, tau=1.0)
    n = 120
    pt = PINS.eos_params("cs")
    pt.nx, pt.ny, pt.force, pt.T, pt.g, pt.tau = po.nx, po.ny, force, po.T, 1.02, po.tau
    target = O.moments(pt, O.run(pt, O.init(pt, rho0), n))["rho"]
    ref = O.adjoint_run(po, rho0, target, n, every=13)
    r0 = dev(rho0).requires_grad_(True)
    g = torch.tensor(po.g, dtype=torch.float64, requires_grad=True)
    T = torch.tensor(po.T, dtype=torch.float64, requires_grad=True)
    rho = rollout(r0, g, T, lib_params(po), n, every=13)
    J = ((rho - dev(target)) ** 2).sum()
    J.backward()
    assert abs(J.item() / ref["J"] - 1) < 1e-10
    dr = r0.grad.cpu().numpy()
    assert np.max(np.abs(dr - ref["drho0"])) < 1e-9 * np.abs(ref["drho0"]).max()
    assert abs(g.grad.item() / ref["dg"] - 1) < 1e-9, (g.grad.item(), ref["dg"])
    assert abs(T.grad.item() / ref["dT"] - 1) < 1e-9, (T.grad.item(), ref["dT"])


def test_rollout_gradient_finite_differences():
    """Autograd gradients against central differences of GPU forward runs
    (relative step 1e-6 for g and T, a seeded direction for rho0)."""
    po, rho0, rv, _ = case("cs", "sc", 64, 64, tau=1.0)
    n = 200
    p = lib_params(po)
    target = dev(rho0 * 1.001)

    def J(r0, g, T):
        with torch.no_grad():
            return float(((rollout(dev(r0), torch.tensor(g, dtype=torch.float64), torch.tensor(T, dtype=torch.float64), p, n)
                           - target) ** 2).sum())

    r0 = dev(rho0).requires_grad_(True)
    g = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    T = torch.tensor(po.T, dtype=torch.float64, requires_grad=True)
    Jv = ((rollout(r0, g, T, p, n, every=20) - target) ** 2).sum()
    Jv.backward()
    hg, hT = 1e-6, 1e-6 * po.T
    fd_g = (J(rho0, 1 + hg, po.T) - J(rho0, 1 - hg, po.T)) / (2 * hg)
    fd_T = (J(rho0, 1.0, po.T + hT) - J(rho0, 1.0, po.T - hT)) / (2 * hT)
    dirn = I.uniform_noise(rho0.shape, 1.0, 5) * rv
    hr = 1e-6
    fd_r = (J(rho0 + hr * dirn, 1.0, po.T) - J(rho0 - hr * dirn, 1.0, po.T)) / (2 * hr)
    ad_r = float((r0.grad.cpu().numpy() * dirn).sum())
    assert abs(g.grad.item() / fd_g - 1) < 1e-5, (g.grad.item(), fd_g)
    assert abs(T.grad.item() / fd_T - 1) < 1e-5, (T.grad.item(), fd_T)
    assert abs(ad_r / fd_r - 1) < 1e-5, (ad_r, fd_r)


def _random_adjoint_cases(n=12, seed=1712):
    rng = np.random.default_rng(seed)
    cases = []
    for _ in range(n):
        nx, ny = int(rng.integers(5, 260)), int(rng.integers(5, 260))
        eos = str(rng.choice(["vdw", "pr", "cs", "rk", "rks"]))
        force = str(rng.choice(["sc", "zc"]))
        grad = str(rng.choice(["hdm", "cdm"]))
        variants = [0, 2] + ([3] if grad == "hdm" and ny > 79 else [])
        cases.append((nx, ny, eos, force, grad, int(rng.choice(variants))))
    return cases


@pytest.mark.parametrize("nx,ny,eos,force,grad,variant", _random_adjoint_cases())
def test_random_reverse_steps_match_oracle(nx, ny, eos, force, grad, variant):
    """12 seeded configurations drawn across shape, EOS, force, gradient and
    reverse-step path: one reverse step against the oracle's."""
    po, rho0, _, _ = case(eos, force, nx, ny, seed=nx + ny)
    po.grad = grad
    f_t = O.run(po, O.init(po, rho0), 3)
    lam_next = np.random.default_rng(nx * 1000 + ny).standard_normal(f_t.shape)
    ref_lam, ref_grad = O.adjoint_step(po, f_t, lam_next)
    d = L.Domain(lib_params(po), dev(rho0))
    d.set_kernel(variant, 0)
    d.set_populations(dev(f_t))
    st = d.new_states(1)
    d.save_state(st[0])
    lam = torch.empty((9, ny, nx), dtype=torch.float64, device="cuda")
    grad_t = torch.zeros(2, dtype=torch.float64, device="cuda")
    d.adjoint_step(st[0], dev(lam_next), lam, grad_t, d.adjoint_workspace())
    got = lam.cpu().numpy()
    scale = np.abs(ref_lam).max()
    assert np.max(np.abs(got - ref_lam)) < 1e-11 * scale, np.max(np.abs(got - ref_lam)) / scale
    g = grad_t.cpu().numpy()
    assert np.all(np.abs(g - ref_grad) < 1e-10 * np.maximum(1.0, np.abs(ref_grad))), (g, ref_grad)


def test_column_march_and_tiles_agree_at_full_width():
    """A 2048 x 1024 reverse step with the y derivatives by column marches
    (the automatic choice on this lattice) and by tiles, both against the
    oracle's reverse step and against each other."""
    po, rho0, _, _ = case("cs", "sc", 2048, 1024, tau=1.0)
    f_t = O.run(po, O.init(po, rho0), 2)
    lam_next = np.random.default_rng(11).standard_normal(f_t.shape)
    ref_lam, ref_grad = O.adjoint_step(po, f_t, lam_next)
    out = {}
    for variant in (0, 2):
        d = L.Domain(lib_params(po), dev(rho0))
        d.set_kernel(variant, 0)
        d.set_populations(dev(f_t))
        st = d.new_states(1)
        d.save_state(st[0])
        lam = torch.empty((9, 1024, 2048), dtype=torch.float64, device="cuda")
        grad = torch.zeros(2, dtype=torch.float64, device="cuda")
        d.adjoint_step(st[0], dev(lam_next), lam, grad, d.adjoint_workspace())
        out[variant] = (lam.cpu().numpy(), grad.cpu().numpy())
    scale = np.abs(ref_lam).max()
    for variant, (lam, g) in out.items():
        assert np.max(np.abs(lam - ref_lam)) < 1e-11 * scale, (variant, np.max(np.abs(lam - ref_lam)) / scale)
        assert np.all(np.abs(g - ref_grad) < 1e-10 * np.maximum(1.0, np.abs(ref_grad))), (variant, g, ref_grad)
    assert np.max(np.abs(out[0][0] - out[2][0])) < 1e-12 * scale


def test_adjoint_unsupported_variants():
    po, rho0, _, _ = case("cs", "sc", 20, 20)
    p = lib_params(po)
    p.prec = "f32"
    d = L.Domain(p, dev(rho0))
    st = d.new_states(1)
    d.save_state(st[0])
    lam = torch.zeros((9, 20, 20), dtype=torch.float64, device="cuda")
    with pytest.raises(L.LBMError) as e:
        d.adjoint_step(st[0], lam, lam.clone(), torch.zeros(2, dtype=torch.float64, device="cuda"), d.adjoint_workspace())
    assert e.value.status == 5


@pytest.mark.parametrize("variant,nx,ny", [(0, 64, 96), (2, 70, 37), (1, 40, 30), (3, 66, 90)])
def test_record_equals_stepping(variant, nx, ny):
    """lbm_record's slots are bitwise the states that stepping and saving give."""
    po, rho0, _, _ = case("cs", "sc", nx, ny)
    n = 7
    a = L.Domain(lib_params(po), dev(rho0))
    b = L.Domain(lib_params(po), dev(rho0))
    a.set_kernel(variant, 0)
    b.set_kernel(variant, 0)
    rec = a.new_states(n + 1)
    a.record(rec, n)
    ref = b.new_states(n + 1)
    for t in range(n + 1):
        b.save_state(ref[t])
        if t < n:
            b.step(1)
    torch.cuda.synchronize()
    # compare the lattice cells (columns x >= nx of the 64-aligned rows are
    # padding that no kernel reads or writes)
    pitch = (nx + 63) // 64 * 64
    phib = (pitch * ny * 8 + 255) // 256 * 256
    fb = a.state_bytes() - phib
    c = L.Domain(lib_params(po), dev(rho0))
    for t in range(n + 1):
        c.load_state(rec[t])
        fr = c.populations()
        c.load_state(ref[t])
        assert torch.equal(fr, c.populations()), t
        pr = rec[t, fb:fb + pitch * ny * 8].view(torch.float64).reshape(ny, pitch)[:, :nx]
        pf = ref[t, fb:fb + pitch * ny * 8].view(torch.float64).reshape(ny, pitch)[:, :nx]
        assert torch.equal(pr, pf), t
    assert a.steps == n
    assert torch.equal(a.populations(), b.populations())


@pytest.mark.parametrize("force", ["sc", "zc"])
@pytest.mark.parametrize("nx,ny,variant", [(48, 40, 0), (96, 120, 3)])
def test_adjoint_steps_equal_single_steps(force, nx, ny, variant):
    """lbm_adjoint_steps over a recorded segment: lam bitwise that of single
    reverse steps, the parameter gradient equal to summation order.  With
    column marches (variant 3, ny > 79) the inner steps pass the cotangent
    as nine planes plus the density-term plane; the sum they form is the one
    the single steps store."""
    po, rho0, _, _ = case("pr", force, nx, ny)
    n = 9
    d = L.Domain(lib_params(po), dev(rho0))
    d.set_kernel(variant, 0)
    st = d.new_states(n + 1)
    d.record(st, n)
    lam0 = dev(np.random.default_rng(7).standard_normal((9, ny, nx)))
    ws = d.adjoint_workspace()
    lam_a, tmp = lam0.clone(), torch.empty_like(lam0)
    grad_a = torch.zeros(2, dtype=torch.float64, device="cuda")
    d.adjoint_steps(st, n, lam_a, tmp, grad_a, ws)
    lam_b, nxt = lam0.clone(), torch.empty_like(lam0)
    grad_b = torch.zeros(2, dtype=torch.float64, device="cuda")
    for t in reversed(range(n)):
        d.adjoint_step(st[t], lam_b, nxt, grad_b, ws)
        lam_b, nxt = nxt, lam_b
    torch.cuda.synchronize()
    assert torch.equal(lam_a, lam_b)
    assert torch.allclose(grad_a, grad_b, rtol=1e-12, atol=0.0), (grad_a, grad_b)



def _c4_case():
    """The differentiation workload: 256 x 256 Carnahan-Starling droplet
    (R = 48, W = 4) at T = 0.7 Tc, tau = 1, SC + HDM."""
    po = PINS.eos_params("cs")
    po.nx = po.ny = 256
    po.force, po.tau = "sc", 1.0
    tc, _ = O.critical(po)
    po.T = 0.7 * tc
    rv, rl, _ = O.maxwell(po, po.T)
    return po, I.droplet(256, 256, rv, rl, 48.0, 4.0)


def _c4_target(po, rho0, n):
    """Oracle densities after n steps of the same setup at g = 1.02."""
    pt = PINS.eos_params("cs")
    pt.nx, pt.ny, pt.force, pt.tau, pt.T, pt.g = po.nx, po.ny, po.force, po.tau, po.T, 1.02
    return O.moments(pt, O.run(pt, O.init(pt, rho0), n))["rho"]


def test_full_size_gradient_finite_differences():
    """The differentiation workload at full size (5000 steps, a snapshot every
    70, the configuration the benchmark times), J = sum (rho_5000 -
    rho_target)^2: autograd gradients against central differences of GPU
    rollouts for g, T and three seeded directions of rho0 (every step 1e-6
    relative: a direction is a seeded normal field times rho0)."""
    po, rho0 = _c4_case()
    n, every = 5000, 70
    tgt = dev(_c4_target(po, rho0, n))
    p = lib_params(po)
    r0 = dev(rho0).requires_grad_(True)
    g = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    T = torch.tensor(po.T, dtype=torch.float64, requires_grad=True)
    Jv = ((rollout(r0, g, T, p, n, every=every) - tgt) ** 2).sum()
    Jv.backward()
    dr = r0.grad.cpu().numpy()

    def J(r, gv, Tv):
        with torch.no_grad():
            return float(((rollout(dev(r), torch.tensor(gv, dtype=torch.float64), torch.tensor(Tv, dtype=torch.float64),
                                   p, n) - tgt) ** 2).sum())

    assert abs(J(rho0, 1.0, po.T) / Jv.item() - 1) < 1e-13
    hg, hT = 1e-6, 1e-6 * po.T
    fd_g = (J(rho0, 1 + hg, po.T) - J(rho0, 1 - hg, po.T)) / (2 * hg)
    fd_T = (J(rho0, 1.0, po.T + hT) - J(rho0, 1.0, po.T - hT)) / (2 * hT)
    assert abs(g.grad.item() / fd_g - 1) < 1e-5, (g.grad.item(), fd_g)
    assert abs(T.grad.item() / fd_T - 1) < 1e-5, (T.grad.item(), fd_T)
    for s in range(3):
        dirn = I.gaussian(rho0.shape, 1.0, seed=100 + s) * rho0
        hr = 1e-6
        fd_r = (J(rho0 + hr * dirn, 1.0, po.T) - J(rho0 - hr * dirn, 1.0, po.T)) / (2 * hr)
        ad_r = float((dr * dirn).sum())
        assert abs(ad_r / fd_r - 1) < 1e-5, (s, ad_r, fd_r)


def test_full_field_gradient_matches_oracle_at_full_lattice():
    """The full 256 x 256 lattice of the differentiation workload over 350
    steps (five checkpoint segments of 70): every component of dJ/drho0 and
    dJ/dg, dJ/dT against the oracle's checkpointed adjoint (the oracle's
    reverse sweep over the whole 5000 steps would take minutes)."""
    po, rho0 = _c4_case()
    n, every = 350, 70
    target = _c4_target(po, rho0, n)
    ref = O.adjoint_run(po, rho0, target, n, every=every)
    p = lib_params(po)
    r0 = dev(rho0).requires_grad_(True)
    g = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    T = torch.tensor(po.T, dtype=torch.float64, requires_grad=True)
    Jv = ((rollout(r0, g, T, p, n, every=every) - dev(target)) ** 2).sum()
    Jv.backward()
    assert abs(Jv.item() / ref["J"] - 1) < 1e-10
    dr = r0.grad.cpu().numpy()
    assert np.max(np.abs(dr - ref["drho0"])) < 1e-9 * np.abs(ref["drho0"]).max()
    assert abs(g.grad.item() / ref["dg"] - 1) < 1e-9, (g.grad.item(), ref["dg"])
    assert abs(T.grad.item() / ref["dT"] - 1) < 1e-9, (T.grad.item(), ref["dT"])


def test_zero_steps_are_identities():
    """Empty inputs: zero steps leave the populations as they are, zero
    reverse steps leave the cotangent and the parameter gradients untouched,
    and a zero-step rollout is the identity (dJ/drho0 = 2 (rho0 - target),
    nothing flows to g or T)."""
    po, rho0, _, _ = case("cs", "sc", 70, 96)
    d = L.Domain(lib_params(po), dev(rho0))
    f0 = d.populations().clone()
    d.step(0)
    assert torch.equal(d.populations(), f0)
    seg = d.new_states(2)
    d.record(seg, 0)
    lam = torch.randn((9, po.ny, po.nx), dtype=torch.float64, device="cuda")
    lam_keep = lam.clone()
    lam2 = torch.empty_like(lam)
    grad = torch.tensor([0.25, -0.5], dtype=torch.float64, device="cuda")
    d.adjoint_steps(seg, 0, lam, lam2, grad, d.adjoint_workspace())
    torch.cuda.synchronize()
    assert torch.equal(lam, lam_keep) and grad.tolist() == [0.25, -0.5]
    target = dev(rho0 * 1.01)
    r0 = dev(rho0).requires_grad_(True)
    g = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    T = torch.tensor(po.T, dtype=torch.float64, requires_grad=True)
    rho = rollout(r0, g, T, lib_params(po), 0)
    ((rho - target) ** 2).sum().backward()
    assert torch.allclose(rho.detach(), dev(rho0), rtol=1e-15, atol=0)
    assert torch.allclose(r0.grad, 2 * (dev(rho0) - target), rtol=1e-13, atol=1e-15)
    assert g.grad.item() == 0.0 and T.grad.item() == 0.0

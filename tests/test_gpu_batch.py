"""Batched sweep (lbm_batch_* through the C ABI): every domain of a batch must
evolve exactly as the same domain stepped alone, and as the oracle."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def sweep_params(n, seed, prec="f64", shapes=None):
    """Uneven flat-interface domains: PR (a = 2/49, b = 2/21, omega = 0.344) and CS
    alternating, T_r spread over [0.5, 0.95], x-slab of the Maxwell densities."""
    nxs, nys = shapes if shapes else I.batch_shapes(n, seed)
    trs = np.linspace(0.5, 0.95, max(n // 2, 1))
    ps, rhos = [], []
    for i in range(n):
        kind = "pr" if i % 2 == 0 else "cs"
        po = PINS.eos_params(kind)
        if kind == "pr":
            po.a = 2 / 49
        p = L.Params(nx=nxs[i], ny=nys[i], eos=kind, force="sc", prec=prec, a=po.a, b=po.b, R=1.0,
                     omega=po.omega, k=0.04, tau=1.0)
        tc, _ = L.critical(p)
        p.T = trs[(i // 2) % len(trs)] * tc
        rv, rl, _ = L.maxwell(p, p.T)
        rho0 = I.slab(p.nx, p.ny, rv, rl, 5.0, axis="x", noise=1e-4 * rv, seed=seed + i)
        ps.append(p)
        rhos.append(rho0)
    return ps, rhos


def to_oracle(p):
    return O.Params(nx=p.nx, ny=p.ny, eos=p.eos, force=p.force, grad=p.grad, tau=p.tau, a=p.a, b=p.b, R=p.R,
                    omega=p.omega, T=p.T, k=p.k, g=p.g, A=p.A, walls=p.walls)


SHAPES = ([128, 70, 256, 64, 512, 130, 200, 96], [8, 9, 32, 16, 8, 33, 17, 8])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_equals_single_domains(prec):
    """Bitwise: each domain of the batched launch (graph path) against the same
    domain stepped alone by the single-domain fused kernel."""
    ps, rhos = sweep_params(8, 7, prec, SHAPES)
    b = L.Batch(ps, [dev(r) for r in rhos])
    b.step(37)
    for i, (p, r) in enumerate(zip(ps, rhos)):
        d = L.Domain(p, dev(r))
        d.step(37)
        got = b.domain(i).populations().cpu().numpy()
        ref = d.populations().cpu().numpy()
        assert np.array_equal(got, ref), (i, np.max(np.abs(got - ref)))


def test_batch_matches_oracle():
    ps, rhos = sweep_params(8, 11, "f64", SHAPES)
    b = L.Batch(ps, [dev(r) for r in rhos])
    b.step(30)
    for i in (0, 1, 5, 7):
        po = to_oracle(ps[i])
        ref = O.moments(po, O.run(po, O.init(po, rhos[i]), 30))["rho"]
        got = b.domain(i).moments()["rho"].cpu().numpy()
        assert np.max(np.abs(got - ref) / ref) < 1e-12, i


def test_graph_and_separate_launches_agree():
    ps, rhos = sweep_params(8, 3, "f64", SHAPES)
    a = L.Batch(ps, [dev(r) for r in rhos])
    c = L.Batch(ps, [dev(r) for r in rhos])
    a.step(41)           # one parity-aligning launch + two graphs + direct steps
    c.step_separate(41)  # one fused single-domain launch per domain per step
    for i in range(len(ps)):
        assert np.array_equal(a.domain(i).populations().cpu().numpy(), c.domain(i).populations().cpu().numpy()), i


@pytest.mark.parametrize("tile_y,order,grid", [(4, 0, 0), (4, 1, 64), (8, 2, 0), (8, 0, 7), (8, 1, 1024),
                                                (4, 3, 0), (8, 3, 13), (4, 3, 2048)])
def test_schedule_does_not_change_results(tile_y, order, grid):
    ps, rhos = sweep_params(8, 5, "f64", SHAPES)
    a = L.Batch(ps, [dev(r) for r in rhos])
    a.set_schedule(tile_y, order, grid)
    assert a.schedule() == {"tile_y": tile_y, "order": order, "grid": grid}
    a.step(20)
    ref = L.Batch(ps, [dev(r) for r in rhos])
    ref.step(20)
    for i in range(len(ps)):
        assert np.array_equal(a.domain(i).populations().cpu().numpy(), ref.domain(i).populations().cpu().numpy()), i


def test_autotune_restores_state_and_picks_a_candidate():
    L.Batch.tune_cache_clear()
    ps, rhos = sweep_params(16, 9)
    a = L.Batch(ps, [dev(r) for r in rhos])
    a.step(3)
    rep = a.autotune(probe_steps=5)
    assert rep["cached"] is False and len(rep) == 2 * 4 * 5 + 2
    ty, o, g = (int(v.lstrip("tyog")) for v in rep["best"].split("_"))
    assert a.schedule() == {"tile_y": ty, "order": o, "grid": g}
    a.step(10)
    ref = L.Batch(ps, [dev(r) for r in rhos])
    ref.step(13)
    for i in range(len(ps)):
        assert np.array_equal(a.domain(i).populations().cpu().numpy(), ref.domain(i).populations().cpu().numpy()), i


def test_autotune_cache():
    """A second batch of the same shapes takes the kept choice without timing;
    other shapes, or a cleared cache, are timed again."""
    L.Batch.tune_cache_clear()
    ps, rhos = sweep_params(8, 21, "f64", SHAPES)
    a = L.Batch(ps, [dev(r) for r in rhos])
    first = a.autotune(probe_steps=3)
    assert first["cached"] is False
    b = L.Batch(ps, [dev(r) for r in rhos])
    b.set_schedule(8, 0, 7)
    again = b.autotune(probe_steps=3)
    assert again == {"cached": True, "best": first["best"]}
    assert b.schedule() == a.schedule()
    b.step(9)
    ref = L.Batch(ps, [dev(r) for r in rhos])
    ref.step(9)
    for i in range(len(ps)):
        assert np.array_equal(b.domain(i).populations().cpu().numpy(), ref.domain(i).populations().cpu().numpy()), i
    other = L.Batch(ps[:7], [dev(r) for r in rhos[:7]])
    assert other.autotune(probe_steps=3)["cached"] is False
    L.Batch.tune_cache_clear()
    assert b.autotune(probe_steps=3)["cached"] is False


def test_schedule_change_after_steps_on_a_side_stream():
    """Steps queued on a side stream, then a new schedule given that stream:
    the queued steps finish with the old worklist before it is replaced."""
    ps, rhos = sweep_params(8, 15, "f64", SHAPES)
    a = L.Batch(ps, [dev(r) for r in rhos])
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        a.step(40, stream=side)
        a.set_schedule(4, 2, 64, stream=side)
        a.step(17, stream=side)
    side.synchronize()
    ref = L.Batch(ps, [dev(r) for r in rhos])
    ref.step(57)
    for i in range(len(ps)):
        assert np.array_equal(a.domain(i).populations().cpu().numpy(), ref.domain(i).populations().cpu().numpy()), i


@pytest.mark.parametrize("force", ["sc", "hybrid"])
def test_cdm9_batch(force):
    """A batch of Eq. 15 domains (the hybrid with a different weight A per
    domain): bitwise the single-domain kernel, and the oracle within 1e-12."""
    ps, rhos = sweep_params(8, 17, "f64", SHAPES)
    for i, p in enumerate(ps):
        p.grad, p.force = "cdm9", force
        p.A = 0.02 * (i - 4) if force == "hybrid" else 0.0
    b = L.Batch(ps, [dev(r) for r in rhos])
    b.step(25)
    for i, (p, r) in enumerate(zip(ps, rhos)):
        d = L.Domain(p, dev(r))
        d.step(25)
        assert np.array_equal(b.domain(i).populations().cpu().numpy(), d.populations().cpu().numpy()), i
    for i in (1, 6):
        po = to_oracle(ps[i])
        ref = O.moments(po, O.run(po, O.init(po, rhos[i]), 25))["rho"]
        got = b.domain(i).moments()["rho"].cpu().numpy()
        assert np.max(np.abs(got - ref) / ref) < 1e-12, i


def test_batch_with_walls():
    """Channels and periodic domains in one batch (the walls are a per-domain
    setting): bitwise the single-domain kernel, and the oracle within 1e-12."""
    ps, rhos = sweep_params(8, 23, "f64", SHAPES)
    for i, p in enumerate(ps):
        p.walls = i % 2
    b = L.Batch(ps, [dev(r) for r in rhos])
    b.step(30)
    for i, (p, r) in enumerate(zip(ps, rhos)):
        d = L.Domain(p, dev(r))
        d.step(30)
        assert np.array_equal(b.domain(i).populations().cpu().numpy(), d.populations().cpu().numpy()), i
    for i in (1, 5):
        po = to_oracle(ps[i])
        ref = O.moments(po, O.run(po, O.init(po, rhos[i]), 30))["rho"]
        got = b.domain(i).moments()["rho"].cpu().numpy()
        assert np.max(np.abs(got - ref) / ref) < 1e-12, i


@pytest.mark.parametrize("seed", [3, 4, 5, 6])
def test_random_batches_equal_single_domains(seed):
    """Seeded batches: 3-8 domains of random width (5-299) and height (5-79:
    the explicit form along y, where the tiling cannot change a cell's
    arithmetic), PR and CS, random walls, precision, Eq. 15 or not and
    schedule; every domain bitwise the same domain stepped alone."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 9))
    prec = str(rng.choice(["f64", "f32"]))
    grad9 = bool(rng.random() < 0.25)
    shapes = ([int(rng.integers(5, 300)) for _ in range(n)], [int(rng.integers(5, 80)) for _ in range(n)])
    ps, rhos = sweep_params(n, seed, prec, shapes)
    for p in ps:
        p.grad = "cdm9" if grad9 else "hdm"
        p.walls = 0 if grad9 else int(rng.random() < 0.4)
    b = L.Batch(ps, [dev(r) for r in rhos])
    sched = (int(rng.choice([4, 8])), int(rng.integers(0, 4)), int(rng.choice([0, 64, 512])))
    b.set_schedule(*sched)
    b.step(25)
    for i, (p, r) in enumerate(zip(ps, rhos)):
        d = L.Domain(p, dev(r))
        d.step(25)
        assert np.array_equal(b.domain(i).populations().cpu().numpy(), d.populations().cpu().numpy()), (i, sched)


def test_batch_rejects_mixed_eq15():
    ps, rhos = sweep_params(4, 19, "f64", ([128, 64, 64, 128], [8, 8, 16, 8]))
    ps[2].grad = "cdm9"
    with pytest.raises(L.LBMError) as e:
        L.Batch(ps, [dev(r) for r in rhos])
    assert e.value.status == 1


def test_per_domain_nonfinite_flags():
    ps, rhos = sweep_params(8, 13, "f64", SHAPES)
    b = L.Batch(ps, [dev(r) for r in rhos])
    b.step(4)
    assert b.check_finite() == [False] * 8
    d = b.domain(3)
    f = d.populations()
    f[2, 1, 5] = float("nan")
    d.set_populations(f)
    assert b.check_finite() == [i == 3 for i in range(8)]


def test_full_coexistence_sweep():
    """The full sweep the benchmark times: 64 domains (N_x in {128, 256, 512},
    N_y in {8, 16, 32} from seed 2024; 32 Peng-Robinson with a = 2/49, then 32
    Carnahan-Starling; T_r = linspace(0.5, 0.95, 32) per group), under the
    schedule the autotuner picks.  After 50 batched steps every domain is
    bitwise the single-domain kernel's result, and eight domains spread over
    both groups and all shapes match the oracle."""
    seed = 2024
    nxs, nys = I.batch_shapes(64, seed)
    trs = np.linspace(0.5, 0.95, 32)
    ps, rhos = [], []
    for i in range(64):
        pr = i < 32
        p = L.Params(nx=nxs[i], ny=nys[i], eos="pr" if pr else "cs", force="sc", a=2 / 49 if pr else 1.0,
                     b=2 / 21 if pr else 4.0, R=1.0, omega=0.344, k=0.04, tau=1.0)
        tc, _ = L.critical(p)
        p.T = trs[i % 32] * tc
        rv, rl, _ = L.maxwell(p, p.T)
        ps.append(p)
        rhos.append(I.slab(p.nx, p.ny, rv, rl, 5.0, axis="x", noise=1e-4 * rv, seed=seed + i))
    b = L.Batch(ps, [dev(r) for r in rhos])
    b.autotune(probe_steps=10)
    n = 50
    b.step(n)
    assert not any(b.check_finite())  # per-domain non-finite flags
    for i, (p, r) in enumerate(zip(ps, rhos)):
        d = L.Domain(p, dev(r))
        d.step(n)
        assert np.array_equal(b.domain(i).populations().cpu().numpy(), d.populations().cpu().numpy()), i
    for i in (0, 9, 17, 31, 32, 45, 50, 63):
        po = to_oracle(ps[i])
        ref = O.moments(po, O.run(po, O.init(po, rhos[i]), n))["rho"]
        got = b.domain(i).moments()["rho"].cpu().numpy()
        assert np.max(np.abs(got - ref) / ref) < 1e-12, i


COEX_EOS = {"vdw": dict(a=9 / 49, b=2 / 21, k=0.01), "rk": dict(a=9 / 49, b=2 / 21, k=0.02),
            "pr": dict(a=9 / 49, b=2 / 21, k=0.04, omega=0.344), "cs": dict(a=1.0, b=4.0, k=0.04)}


def _coexistence_run(force, grad, trs, steps=20000, nx=256, ny=8):
    ps, rhos, maxw = [], [], []
    for eos, c in COEX_EOS.items():
        for tr in trs:
            p = L.Params(nx=nx, ny=ny, eos=eos, force=force, grad=grad, R=1.0, tau=1.6, **c)
            tc, _ = L.critical(p)
            p.T = tr * tc
            rv, rl, _ = L.maxwell(p, p.T)
            ps.append(p)
            maxw.append((rv, rl))
            rhos.append(I.slab(nx, ny, rv, rl, 5.0, axis="x", noise=1e-4 * rv, seed=7))
    b = L.Batch(ps, [dev(r) for r in rhos])
    b.step(steps)
    assert not any(b.check_finite()), (force, grad)
    out = []
    for i, p in enumerate(ps):
        rho = b.domain(i).moments(want=("rho",))["rho"].mean(dim=0).cpu().numpy()
        w = nx // 8
        rl = rho[nx // 2 - w // 2:nx // 2 - w // 2 + w].mean()
        rv = np.concatenate([rho[:w // 2 + 1], rho[nx - w // 2:]]).mean()
        out.append((rl / maxw[i][1] - 1, rv / maxw[i][0] - 1))
    return np.array(out)


def test_coexistence_against_maxwell():
    """Sec. 5.2 (Fig. 5): flat interfaces of the van der Waals, Redlich-Kwong,
    PR-water and Carnahan-Starling fluids (the paper's constants and k,
    tau = 1.6) at T_r = 0.7, 0.8, 0.9 after 20 000 steps.  With the high-order
    difference, Shan-Chen and Zhang-Chen alike, the liquid density is within
    0.1 % and the vapour density within 10 % of the Maxwell rule (measured:
    within 7e-5 and 9.3 %, the largest for PR at 0.7), and the two forces agree
    with each other; the weighted central difference (Eq. 15) misses the vapour
    density by at least three times as much at every point.  (Below T_r = 0.7
    the vapour error of the high-order difference grows for RK and PR, in the
    oracle too: the bar is stated where the method meets it.)"""
    trs = (0.7, 0.8, 0.9)
    sc = _coexistence_run("sc", "hdm", trs)
    zc = _coexistence_run("zc", "hdm", trs)
    cdm = _coexistence_run("sc", "cdm9", trs)
    for e in (sc, zc):
        assert np.max(np.abs(e[:, 0])) < 1e-3, e
        assert np.max(np.abs(e[:, 1])) < 0.10, e
    assert np.max(np.abs(sc[:, 1] - zc[:, 1])) < 0.02, (sc, zc)
    assert np.all(np.abs(cdm[:, 1]) > 3 * np.maximum(np.abs(sc[:, 1]), np.abs(zc[:, 1]))), (sc, zc, cdm)

"""Benchmark of the fused HDM pseudopotential lattice Boltzmann step on one MI355X.

Default workload (the large dynamic case): D2Q9 4096 x 4096 periodic,
Carnahan-Starling EOS (a = 1, b = 4, R = 1, k = 0.04) at T = 0.5 Tc (density
ratio ~725), Shan-Chen force with the high-order difference, tau = 1, 400
seeded droplets with radii uniform in [10, 60] on a vapour background, seeded
Gaussian velocity noise of std 1e-3.  A step is one launch of the fused kernel
(density, EOS potential, HDM gradient, force, EDM-BGK collision, periodic
streaming, and the potential field of the new state).

Output: one JSON line with MLUPS (= nx ny steps / time / 1e6), the roofline of
the fused kernel against the 8 TB/s HBM peak with algorithmic bytes
2 Q sizeof(real) per lattice update (every population read once and written
once), and the FP64 CPU oracle timed on a bounded sample on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import lbm_inputs as I  # noqa: E402

METRIC = "MLUPS & %HBM roofline (FP64/FP32); batched domains/s; adjoint/forward time"
HBM_PEAK_GBS = 8000.0
Q = 9
KERNEL_SOURCES = ["lbm_march.hpp", "lbm_fused.hpp", "lbm_kernels.hpp", "lbm_device.hpp"]
KERNEL_NAMES = {0: "k_march", 1: "k_collide", 2: "k_fused", 3: "k_march"}


def kernel_hash() -> str:
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1712_06079_amd", "csrc", s), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(name: str, seed: int = 2024):
    """(params kwargs, rho0, ux0, uy0, description) of a named workload."""
    import paper_1712_06079_amd as L
    if name == "c5":
        n = 4096
        p = L.Params(nx=n, ny=n, eos="cs", force="sc", a=1.0, b=4.0, R=1.0, k=0.04, tau=1.0)
        tc, _ = L.critical(p)
        p.T = 0.5 * tc
        rv, rl, _ = L.maxwell(p, p.T)
        cx, cy, rr = I.place_droplets(n, n, 400, 10.0, 60.0, 4.0, seed=seed)
        rho0 = I.droplets(n, n, rv, rl, cx, cy, rr, 4.0)
        ux0 = I.gaussian((n, n), 1e-3, seed=seed + 1)
        uy0 = I.gaussian((n, n), 1e-3, seed=seed + 2)
        desc = "4096x4096 CS T=0.5Tc SC+HDM, 400 droplets R~U[10,60], u noise 1e-3"
        return p, rho0, ux0, uy0, desc
    if name == "c2":
        n = 1024
        p = L.Params(nx=n, ny=n, eos="cs", force="zc", a=1.0, b=4.0, R=1.0, k=0.04, tau=1.0)
        tc, _ = L.critical(p)
        p.T = 0.6 * tc
        rv, rl, _ = L.maxwell(p, p.T)
        rho0 = I.droplet(n, n, rv, rl, 128.0, 4.0)
        desc = "1024x1024 CS T=0.6Tc ZC+HDM droplet R=128 (cache-resident)"
        return p, rho0, None, None, desc
    raise ValueError(name)


def run_gpu(name: str, prec: str, steps: int, warmup: int, variant: int = 0, tile: int = 0, chunks: int = 0):
    import torch

    import paper_1712_06079_amd as L
    p, rho0, ux0, uy0, desc = workload(name)
    p.prec = prec
    dev = torch.device("cuda:0")
    t = lambda a: None if a is None else torch.from_numpy(a).to(dev)  # noqa: E731
    d = L.Domain(p, t(rho0), t(ux0), t(uy0))
    d.set_kernel(variant, tile)
    d.set_chunks(chunks)
    stream = torch.cuda.current_stream()
    d.step(warmup)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    total0 = torch.cuda.Event(enable_timing=True)
    total1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    total0.record(stream)
    for i in range(steps):
        starts[i].record(stream)
        d.step(1)
        ends[i].record(stream)
    total1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = total0.elapsed_time(total1)
    per_launch = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    ok = d.check_finite()
    cells = p.nx * p.ny
    mlups = cells * steps / (ms_total * 1e-3) / 1e6
    es = 8 if prec == "f64" else 4
    alg_bytes = 2 * Q * es * cells  # per launch
    launch_s = float(np.mean(per_launch)) * 1e-3
    achieved = alg_bytes / launch_s / 1e9
    return {
        "desc": desc, "params": p, "mlups": mlups, "ms_per_step": ms_total / steps, "wall_s": wall,
        "launch_ms_mean": float(np.mean(per_launch)), "launch_ms_median": float(np.median(per_launch)),
        "achieved_gbs": achieved, "alg_bytes_per_launch": alg_bytes, "finite": ok,
    }


def traffic_from_profile(kernel: str, name: str, prec: str):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{name}_{prec}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def batch_sweep(steps: int, sep_steps: int, seed: int = 2024):
    """The coexistence sweep: 64 periodic flat-interface domains, N_x in
    {128, 256, 512}, N_y in {8, 16, 32} from the seed, 32 Peng-Robinson
    (a = 2/49, b = 2/21, omega = 0.344) and 32 Carnahan-Starling (a = 1, b = 4),
    k = 0.04, T_r = linspace(0.5, 0.95, 32) per group, tau = 1, SC + HDM, FP64,
    x-slab of the Maxwell densities (W = 5) with noise 1e-4.  Times the batched
    graph-replayed launch against one fused launch per domain per step, then
    compares the bulk densities with the Maxwell rule."""
    import torch

    import paper_1712_06079_amd as L
    nxs, nys = I.batch_shapes(64, seed)
    trs = np.linspace(0.5, 0.95, 32)
    ps, rhos, maxw = [], [], []
    for i in range(64):
        pr = i < 32
        p = L.Params(nx=nxs[i], ny=nys[i], eos="pr" if pr else "cs", force="sc", a=2 / 49 if pr else 1.0,
                     b=2 / 21 if pr else 4.0, R=1.0, omega=0.344, k=0.04, tau=1.0)
        tc, _ = L.critical(p)
        p.T = trs[i % 32] * tc
        rv, rl, _ = L.maxwell(p, p.T)
        ps.append(p)
        maxw.append((rv, rl))
        rhos.append(torch.from_numpy(I.slab(p.nx, p.ny, rv, rl, 5.0, axis="x", noise=1e-4 * rv, seed=seed + i)).cuda())
    cells = sum(p.nx * p.ny for p in ps)
    b = L.Batch(ps, rhos)
    tune = b.autotune(probe_steps=20)
    sep = L.Batch(ps, rhos)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    sep.step_separate(4)
    torch.cuda.synchronize()
    e[0].record()
    sep.step_separate(sep_steps)
    e[1].record()
    b.step(16)
    torch.cuda.synchronize()
    e[2].record()
    b.step(steps)
    e[3].record()
    torch.cuda.synchronize()
    ms_sep = e[0].elapsed_time(e[1]) / sep_steps
    ms_bat = e[2].elapsed_time(e[3]) / steps
    flags = b.check_finite()
    errs = []
    for i, p in enumerate(ps):
        if flags[i]:
            errs.append(None)
            continue
        rho = b.domain(i).moments(want=("rho",))["rho"].mean(dim=0).cpu().numpy()
        w = max(p.nx // 8, 1)
        rl = rho[p.nx // 2 - w // 2:p.nx // 2 - w // 2 + w].mean()
        rv = np.concatenate([rho[:w // 2 + 1], rho[p.nx - w // 2:]]).mean()
        errs.append((abs(rl / maxw[i][1] - 1), abs(rv / maxw[i][0] - 1)))
    ok = [x for x in errs if x is not None]
    return {
        "domains": 64, "cells": cells, "steps": steps, "ms_per_step_batched": round(ms_bat, 5),
        "ms_per_step_separate": round(ms_sep, 5), "domain_steps_per_s": round(64 / (ms_bat * 1e-3), 1),
        "domain_steps_per_s_separate": round(64 / (ms_sep * 1e-3), 1), "speedup": round(ms_sep / ms_bat, 2),
        "mlups_batched": round(cells / (ms_bat * 1e-3) / 1e6, 1), "schedule": tune.get("best"),
        "nonfinite_domains": int(sum(flags)),
        "maxwell_rel_err_liquid_max": round(max(x[0] for x in ok), 5) if ok else None,
        "maxwell_rel_err_vapour_max": round(max(x[1] for x in ok), 5) if ok else None,
        "maxwell_rel_err_liquid_median": round(float(np.median([x[0] for x in ok])), 5) if ok else None,
        "maxwell_rel_err_vapour_median": round(float(np.median([x[1] for x in ok])), 5) if ok else None,
    }


def adjoint_cost(steps: int, every: int, seed: int = 2024):
    """The differentiation workload: 256 x 256 CS droplet R = 48 (W = 4) at
    T = 0.7 Tc, FP64, tau = 1, SC + HDM; J = sum (rho_n - rho_target)^2 with
    the target from the same setup at g = 1.02.  Reports the adjoint step time
    over the forward step time, the whole-gradient time over the forward
    rollout time, and peak device memory of the checkpointed gradient."""
    import torch

    import paper_1712_06079_amd as L
    from paper_1712_06079_amd.autograd import rollout
    p = L.Params(nx=256, ny=256, eos="cs", force="sc", a=1.0, b=4.0, R=1.0, k=0.04, tau=1.0)
    tc, _ = L.critical(p)
    p.T = 0.7 * tc
    rv, rl, _ = L.maxwell(p, p.T)
    rho0 = torch.from_numpy(I.droplet(256, 256, rv, rl, 48.0, 4.0)).cuda()
    # per-step costs
    d = L.Domain(p, rho0)
    st = d.new_states(1)
    d.save_state(st[0])
    lam = torch.randn((9, 256, 256), dtype=torch.float64, device="cuda")
    lam2 = torch.empty_like(lam)
    grad = torch.zeros(2, dtype=torch.float64, device="cuda")
    ws = d.adjoint_workspace()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    d.step(10)
    torch.cuda.synchronize()
    ev[0].record()
    d.step(200)
    ev[1].record()
    for _ in range(200):
        d.adjoint_step(st[0], lam, lam2, grad, ws)
    ev[2].record()
    torch.cuda.synchronize()
    t_fwd = ev[0].elapsed_time(ev[1]) / 200
    t_adj = ev[1].elapsed_time(ev[2]) / 200
    # whole gradient with checkpointing
    pt = L.Params(**{**p.__dict__, "g": 1.02})
    with torch.no_grad():
        target = rollout(rho0, torch.tensor(1.02, dtype=torch.float64), torch.tensor(p.T, dtype=torch.float64), pt,
                         steps)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    r0 = rho0.clone().requires_grad_(True)
    g = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    T = torch.tensor(p.T, dtype=torch.float64, requires_grad=True)
    ev[2].record()
    rho = rollout(r0, g, T, p, steps, every)
    ev[3].record()
    torch.cuda.synchronize()
    t_roll = ev[2].elapsed_time(ev[3])
    w0 = time.perf_counter()
    J = ((rho - target) ** 2).sum()
    J.backward()
    torch.cuda.synchronize()
    t_back = (time.perf_counter() - w0) * 1e3
    peak = torch.cuda.max_memory_allocated() - base
    return {
        "workload": "256x256 CS T=0.7Tc SC+HDM droplet R=48, J = |rho_n - rho(g=1.02)|^2",
        "steps": steps, "checkpoint_every": every, "ms_forward_step": round(t_fwd, 5),
        "ms_adjoint_step": round(t_adj, 5), "adjoint_over_forward": round(t_adj / t_fwd, 3),
        "ms_forward_rollout": round(t_roll, 2), "ms_backward": round(t_back, 2),
        "gradient_over_forward": round((t_roll + t_back) / t_roll, 3), "peak_mib": round(peak / 2 ** 20, 1),
        "J": float(J.item()), "dJ_dg": float(g.grad.item()), "dJ_dT": float(T.grad.item()),
    }


def copy_probe(gib: float = 2.0, reps: int = 20):
    """A plain streaming kernel of known size (dst = 1.0 * src, FP64): reads and
    writes `gib` GiB per launch.  Its rocprofv3 FETCH_SIZE / WRITE_SIZE give the
    counter-to-bytes scale, and its rate the attainable HBM bandwidth."""
    import torch
    n = int(gib * (1 << 30) / 8)
    src = torch.rand(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    moved = 2 * n * 8
    return {"bytes_per_launch": moved, "ms": ms, "GBps": moved / (ms * 1e-3) / 1e9}


def cpu_baseline(name: str, sample_steps: int):
    """The FP64 oracle on a bounded sample of the same workload (host cores)."""
    import oracle as O
    p, rho0, ux0, uy0, _ = workload(name)
    po = O.Params(nx=p.nx, ny=p.ny, eos=p.eos, force=p.force, grad=p.grad, tau=p.tau, a=p.a, b=p.b, R=p.R,
                  omega=p.omega, T=p.T, k=p.k, g=p.g, A=p.A)
    f = O.init(po, rho0, ux0, uy0)
    t0 = time.perf_counter()
    O.run(po, f, sample_steps)
    dt = time.perf_counter() - t0
    return {"value": round(p.nx * p.ny * sample_steps / dt / 1e6, 3), "unit": "MLUPS", "cores": O.threads(),
            "kind": "oracle", "sample": f"{sample_steps} FP64 steps of the {p.nx}x{p.ny} workload ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c5", choices=["c5", "c2"])
    ap.add_argument("--prec", default="f64", choices=["f64", "f32"])
    ap.add_argument("--variant", type=int, default=0,
                    help="0 automatic (strip march here), 1 two-pass reference, 2 fused tiles, 3 fused strip march")
    ap.add_argument("--tile", type=int, default=0, help="rows per tile or marching block (0 = default)")
    ap.add_argument("--chunks", type=int, default=0, help="y chunks per strip of the marching kernel (0 = automatic)")
    ap.add_argument("--cpu-steps", type=int, default=8, help="oracle sample steps (0 = skip)")
    ap.add_argument("--no-other-prec", action="store_true", help="skip the second-precision run")
    ap.add_argument("--copy-probe", action="store_true", help="only run the streaming-copy calibration kernel")
    ap.add_argument("--batch-steps", type=int, default=2000, help="batched-sweep steps (0 = skip)")
    ap.add_argument("--adjoint-steps", type=int, default=5000, help="differentiated rollout steps (0 = skip)")
    args = ap.parse_args()
    if args.copy_probe:
        print(json.dumps({"copy_probe": copy_probe()}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: launched with WORLD_SIZE > 1; this build runs on one GPU", file=sys.stderr)
        sys.exit(2)

    r = run_gpu(args.workload, args.prec, args.steps, args.warmup, args.variant, args.tile, args.chunks)
    print(f"[bench] {args.workload} {args.prec}: {r['mlups']:.0f} MLUPS, {r['ms_per_step']:.4f} ms/step, "
          f"kernel {r['launch_ms_mean']:.4f} ms, {r['achieved_gbs']:.0f} GB/s algorithmic", file=sys.stderr, flush=True)
    p = r["params"]
    other = None
    if not args.no_other_prec:
        op = "f32" if args.prec == "f64" else "f64"
        o = run_gpu(args.workload, op, args.steps, args.warmup, args.variant, args.tile, args.chunks)
        print(f"[bench] {args.workload} {op}: {o['mlups']:.0f} MLUPS, kernel {o['launch_ms_mean']:.4f} ms, "
              f"{o['achieved_gbs']:.0f} GB/s algorithmic", file=sys.stderr, flush=True)
        other = {"storage": op, "dtype": "f64", "value": round(o["mlups"], 1), "ms_per_step": round(o["ms_per_step"], 5),
                 "roofline_frac": round(o["achieved_gbs"] / HBM_PEAK_GBS, 4), "finite": o["finite"]}
    batch = None
    if args.batch_steps > 0:
        batch = batch_sweep(args.batch_steps, max(args.batch_steps // 10, 20))
        print(f"[bench] batch: {batch['domain_steps_per_s']:.0f} domain-steps/s batched, "
              f"{batch['domain_steps_per_s_separate']:.0f} separate", file=sys.stderr, flush=True)
    adjoint = None
    if args.adjoint_steps > 0:
        adjoint = adjoint_cost(args.adjoint_steps, 70)
        print(f"[bench] adjoint/forward step {adjoint['adjoint_over_forward']}, gradient/forward "
              f"{adjoint['gradient_over_forward']}", file=sys.stderr, flush=True)
    cpu = cpu_baseline(args.workload, args.cpu_steps) if args.cpu_steps > 0 else None
    kname = KERNEL_NAMES.get(args.variant, "k_march")
    traffic = traffic_from_profile(kname, args.workload, args.prec)
    line = {
        "metric": METRIC, "value": round(r["mlups"], 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": r["desc"], "storage": args.prec, "nx": p.nx, "ny": p.ny, "eos": p.eos, "force": p.force, "grad": p.grad,
                   "tau": p.tau, "k": p.k, "T": p.T, "seed": 2024, "kernel": kname,
                   "finite": r["finite"]},
        "roofline": {"bound": "hbm", "achieved": round(r["achieved_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kname, "alg_bytes_per_launch": r["alg_bytes_per_launch"],
                     "launch_ms": round(r["launch_ms_mean"], 5)},
        "cpu_baseline": cpu,
    }
    if other:
        line["other_precision"] = other
    if batch:
        line["batch"] = batch
    if adjoint:
        line["adjoint"] = adjoint
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Seeded synthetic inputs for the D2Q9 multiphase lattice Boltzmann workloads.

This module is shared by the GPU library's tests and benchmark and by the CPU
oracle's tests.  It holds none of the method's arithmetic: it only lays out
initial density and velocity fields (slabs, droplets, noise) from parameters the
caller supplies (coexistence densities come from the caller), using a
counter-based SplitMix64 stream so every field is reproducible from its seed.

Recipes (each workload in the paper is a flat interface or droplets):
  * flat slab  (Sec. 5.2): liquid in the middle half, vapour elsewhere, joined
    by the tanh profile of Sec. 3.1 Eq. 16 (rho = 1 + tanh(2x/W) convention);
  * droplet    (Secs. 5.3-5.4): rho_v + (rho_l - rho_v)/2 (1 - tanh(2 (r - R)/W));
  * many droplets: radii uniform in [rmin, rmax], centres uniform with
    minimum-image rejection so droplets do not overlap;
  * noise: additive uniform U(-amp, amp) in row-major order; velocity noise is
    Gaussian (Box-Muller on the same stream).
"""
from __future__ import annotations

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n outputs of SplitMix64 with state seed + (offset + i + 1) * golden gamma."""
    with np.errstate(over="ignore"):
        i = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed) + i * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, n, offset) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform_noise(shape, amp: float, seed: int) -> np.ndarray:
    n = int(np.prod(shape))
    return (2.0 * uniform01(seed, n) - 1.0).reshape(shape) * amp


def gaussian(shape, std: float, seed: int) -> np.ndarray:
    n = int(np.prod(shape))
    m = (n + 1) // 2
    u = uniform01(seed, 2 * m)
    u1 = 1.0 - u[0::2]  # (0, 1]
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.concatenate([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)])[:n]
    return (z * std).reshape(shape)


def slab(nx: int, ny: int, rho_v: float, rho_l: float, W: float, axis: str = "y",
         noise: float = 0.0, seed: int = 0) -> np.ndarray:
    """Liquid slab in the middle half along `axis`, interfaces at N/4 and 3N/4."""
    n = ny if axis == "y" else nx
    s = np.arange(n, dtype=np.float64)
    prof = rho_v + 0.5 * (rho_l - rho_v) * (np.tanh(2.0 * (s - n / 4.0) / W) - np.tanh(2.0 * (s - 3.0 * n / 4.0) / W))
    rho = np.repeat(prof[:, None], nx, axis=1) if axis == "y" else np.repeat(prof[None, :], ny, axis=0)
    if noise:
        rho = rho + uniform_noise((ny, nx), noise, seed)
    return np.ascontiguousarray(rho)


def droplet(nx: int, ny: int, rho_v: float, rho_l: float, R: float, W: float,
            cx: float | None = None, cy: float | None = None, noise: float = 0.0, seed: int = 0) -> np.ndarray:
    cx = nx / 2.0 if cx is None else cx
    cy = ny / 2.0 if cy is None else cy
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    rho = rho_v + 0.5 * (rho_l - rho_v) * (1.0 - np.tanh(2.0 * (r - R) / W))
    if noise:
        rho = rho + uniform_noise((ny, nx), noise, seed)
    return np.ascontiguousarray(rho)


def place_droplets(nx: int, ny: int, n: int, rmin: float, rmax: float, W: float, seed: int,
                   max_tries: int = 200000):
    """Centres and radii of n non-overlapping droplets (minimum-image distance
    >= R_a + R_b + 2W), drawn from the seeded stream."""
    cx, cy, rr = [], [], []
    k = 0
    tries = 0
    while len(rr) < n:
        if tries >= max_tries:
            raise RuntimeError(f"placed only {len(rr)} of {n} droplets")
        u = uniform01(seed, 3, offset=3 * k)
        k += 1
        tries += 1
        x, y, r = u[0] * nx, u[1] * ny, rmin + (rmax - rmin) * u[2]
        ok = True
        for xa, ya, ra in zip(cx, cy, rr):
            dx = abs(x - xa); dx = min(dx, nx - dx)
            dy = abs(y - ya); dy = min(dy, ny - dy)
            if dx * dx + dy * dy < (r + ra + 2 * W) ** 2:
                ok = False
                break
        if ok:
            cx.append(x); cy.append(y); rr.append(r)
    return np.array(cx), np.array(cy), np.array(rr)


def droplets(nx: int, ny: int, rho_v: float, rho_l: float, cx, cy, radii, W: float) -> np.ndarray:
    """Vapour background plus one tanh droplet per centre (minimum-image
    distance).  Each droplet is added inside its box of half-width R + 12 W,
    beyond which its tanh term is below 1e-20 of (rho_l - rho_v)."""
    rho = np.full((ny, nx), rho_v, dtype=np.float64)
    for xa, ya, ra in zip(cx, cy, radii):
        h = int(np.ceil(ra + 12 * W))
        xs = np.arange(int(np.floor(xa)) - h, int(np.floor(xa)) + h + 2)
        ys = np.arange(int(np.floor(ya)) - h, int(np.floor(ya)) + h + 2)
        xs = np.unique(xs % nx)
        ys = np.unique(ys % ny)
        dx = np.abs(xs[None, :] - xa); dx = np.minimum(dx, nx - dx)
        dy = np.abs(ys[:, None] - ya); dy = np.minimum(dy, ny - dy)
        r = np.sqrt(dx * dx + dy * dy)
        rho[np.ix_(ys, xs)] += 0.5 * (rho_l - rho_v) * (1.0 - np.tanh(2.0 * (r - ra) / W))
    return np.ascontiguousarray(rho)


def batch_shapes(n: int, seed: int, nx_choices=(128, 256, 512), ny_choices=(8, 16, 32)):
    """Uneven domain sizes for a batched sweep: Nx and Ny drawn uniformly from the choices."""
    u = uniform01(seed, 2 * n)
    nxs = [nx_choices[min(int(u[2 * i] * len(nx_choices)), len(nx_choices) - 1)] for i in range(n)]
    nys = [ny_choices[min(int(u[2 * i + 1] * len(ny_choices)), len(ny_choices) - 1)] for i in range(n)]
    return nxs, nys

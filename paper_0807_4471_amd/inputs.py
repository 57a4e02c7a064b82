"""Seeded synthetic inputs: initial density fields and workload parameters.

This module holds none of the lattice Boltzmann arithmetic.  It only draws
random numbers and lays them out, so that the HIP library and the CPU oracle
can be fed the same inputs.

Random numbers come from SplitMix64 (G. L. Steele, D. Lea, C. H. Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014), used as a
counter-based generator: output number ``c`` (0-based) of the stream seeded
with ``seed`` is ``mix64(seed + (c + 1) * GAMMA)`` -- exactly the c-th value
the sequential generator returns.  The HIP init kernel implements the same
published definition on its own; the two are compared bit for bit.

Initial densities (paper: "random initial conditions", no distribution
given) follow the workload recipe
    rho_s(n) = mean_s * (1 + amp * U),  U = 2 * (h >> 11) * 2**-53 - 1,
with h the SplitMix64 output for counter c = s * nx * ny + n and n = y*nx + x.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (vectorised over uint64 arrays)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """Outputs number ``counters`` of the SplitMix64 stream seeded with ``seed``."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * GAMMA
    return mix64(state)


def uniform_pm1(seed: int, counters: np.ndarray) -> np.ndarray:
    """U in [-1, 1): 53 high bits of the SplitMix64 output, scaled."""
    h = splitmix64(seed, counters)
    u01 = (h >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u01 - 1.0


def random_densities(nx: int, ny: int, seed: int, mean=(0.7, 0.7), amp: float = 0.05) -> np.ndarray:
    """(2, ny, nx) float64 initial densities rho_s = mean_s (1 + amp U)."""
    N = nx * ny
    c = np.arange(2 * N, dtype=np.uint64)
    U = uniform_pm1(seed, c).reshape(2, ny, nx)
    m = np.asarray(mean, dtype=np.float64).reshape(2, 1, 1)
    return m * (1.0 + amp * U)


def random_densities_window(nx: int, ny: int, seed: int, ys, xs, mean=(0.7, 0.7),
                            amp: float = 0.05) -> np.ndarray:
    """The (2, len(ys), len(xs)) block of random_densities(nx, ny, seed, mean,
    amp) at rows ys and columns xs (index arrays, e.g. wrapped ranges),
    drawn without generating the whole lattice."""
    y = np.asarray(ys, dtype=np.uint64)[:, None]
    x = np.asarray(xs, dtype=np.uint64)[None, :]
    n = y * np.uint64(nx) + x
    c = np.stack([n, n + np.uint64(nx * ny)])
    U = uniform_pm1(seed, c)
    m = np.asarray(mean, dtype=np.float64).reshape(2, 1, 1)
    return m * (1.0 + amp * U)


def droplet_densities(nx: int, ny: int, radius: float, rho_in: float, rho_out: float,
                      width: float = 1.5) -> np.ndarray:
    """Static droplet of species A (density rho_in inside) in species B (and
    the reverse outside), tanh profile centred on the lattice."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - (nx - 1) / 2.0) ** 2 + (y - (ny - 1) / 2.0) ** 2)
    s = 0.5 * (1.0 - np.tanh((r - radius) / width))
    rho = np.empty((2, ny, nx))
    rho[0] = rho_out + (rho_in - rho_out) * s
    rho[1] = rho_in + (rho_out - rho_in) * s
    return rho


def batch_mix(seed: int = 2026, n: int = 64) -> list[dict]:
    """Parameters of the uneven batch workload: n instances with sides from
    {128, 192, 256, 384, 512}, rho0 ~ U(0.60, 0.80), G^X ~ U(0.50, 0.65),
    tau_s ~ U(0.8, 1.2) per species (numpy generator `seed`), instance i
    initialised by random_densities(..., seed=1000 + i)."""
    rng = np.random.default_rng(seed)
    sides = rng.choice([128, 192, 256, 384, 512], size=n)
    rho0 = rng.uniform(0.60, 0.80, n)
    gx = rng.uniform(0.50, 0.65, n)
    tau = rng.uniform(0.8, 1.2, (n, 2))
    return [dict(nx=int(sides[i]), ny=int(sides[i]), rho0=float(rho0[i]), Gx=float(gx[i]),
                 tau=(float(tau[i, 0]), float(tau[i, 1])), seed=1000 + i) for i in range(n)]


def ripple_slab_densities(nx: int, ny: int, rho_in: float, rho_out: float, amp: float = 2.0,
                          width: float = 1.5, mode: int = 1) -> np.ndarray:
    """Slab of species A (density rho_in; B has rho_out there, and the reverse
    outside) between y = ny/4 and 3 ny/4, both interfaces displaced outward
    by amp * sin(2 pi mode x / nx) (a varicose ripple), tanh profiles."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    d = amp * np.sin(2.0 * np.pi * mode * x / nx)
    y1, y2 = ny / 4.0 - d, 3.0 * ny / 4.0 + d
    s = 0.5 * (np.tanh((y - y1) / width) - np.tanh((y - y2) / width))
    rho = np.empty((2, ny, nx))
    rho[0] = rho_out + (rho_in - rho_out) * s
    rho[1] = rho_in + (rho_out - rho_in) * s
    return rho

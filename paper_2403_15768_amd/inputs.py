"""Seeded synthetic inputs shaped like the paper's nanochannel workloads.

This module holds input generation only -- random fields, spectral parameter
draws, channel lists and arrival traces -- and none of the lattice-Boltzmann or
quadrature arithmetic.  Both the GPU path and the CPU oracle take their inputs
from here.

Workload shapes (paper Sec. 2: water in a carbon/graphite nanochannel driven by
a pressure gradient; Sec. 6: a nanotube of aspect ratio L/D of about 10 at a
lattice spacing of 1 nm):

* ``channel2d``  D2Q9 channel 64 x 30 fluid rows, tau 0.8, g 1e-6, no-slip or
  slip length 4 (lambda = nu / L_s = 0.025).
* ``duct``       D3Q19 rectangular duct 256 x 128 x 64, tau 0.7, g 1e-6, wall
  friction lambda(x, s) a smooth random field (mean 0.05, std 0.02,
  correlation length 16).
* ``tube``       D3Q19 circular nanotube, radius 32, box 512 x 72 x 72, tau 0.8,
  g 1e-6, per-wall-node friction from the spectral quadrature.
* ``batch``      256 ducts with sizes uniform in [32,128] x [32,64] x [32,64].
* ``serving``    Poisson arrivals (50/s) of tube queries with radius 8..32.
* ``corrugated`` D3Q19 slab 256 x 128 x 64 whose two walls are wrinkled
  (Sec. 5.1: the wall's shape as a design parameter): staircase sinusoids of
  amplitude 4 cells and wavelength 64 along x, random phases, friction as the
  duct's smooth random field.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 240315768
WORKLOAD_ID = {"channel2d": 1, "duct": 2, "tube": 3, "batch": 4, "serving": 5,
               "corrugated": 6}


def rng_for(workload: str, index: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + 1000 * WORKLOAD_ID[workload] + index)


# ---------------------------------------------------------------- fields

def smooth_periodic_noise(shape, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. N(0,1) noise, periodic Gaussian filter of kernel std ``sigma``
    (grid units, every axis), standardised to sample mean 0 and std 1."""
    noise = rng.standard_normal(shape)
    spec = np.fft.fftn(noise)
    for ax, n in enumerate(shape):
        k = np.fft.fftfreq(n) * 2.0 * math.pi
        filt = np.exp(-0.5 * (sigma * k) ** 2)
        bshape = [1] * len(shape)
        bshape[ax] = n
        spec = spec * filt.reshape(bshape)
    out = np.real(np.fft.ifftn(spec))
    out -= out.mean()
    sd = out.std()
    return out / sd if sd > 0 else out


def perimeter_coordinate(coords: np.ndarray, cy: float, cz: float, perimeter: float) -> np.ndarray:
    """Position s in [0, perimeter) of a wall node around the channel's
    cross-section, from its polar angle about (cy, cz)."""
    theta = np.arctan2(coords[:, 2] - cz, coords[:, 1] - cy)
    return (theta % (2.0 * math.pi)) / (2.0 * math.pi) * perimeter


def wall_surface_field(coords: np.ndarray, nx: int, cy: float, cz: float, perimeter: float,
                       sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Standardised smooth random field on the unrolled wall surface (x, s),
    sampled at the wall nodes ``coords`` (N x 3 ints: x, y, z)."""
    ns = max(1, int(round(perimeter)))
    xi = smooth_periodic_noise((ns, nx), sigma, rng)
    s = perimeter_coordinate(coords, cy, cz, perimeter)
    si = np.minimum((s / perimeter * ns).astype(np.int64), ns - 1)
    return xi[si, coords[:, 0]]


def duct_friction(coords: np.ndarray, nx: int, ny: int, nz: int, rng: np.random.Generator,
                  mean: float = 0.05, std: float = 0.02, sigma: float = 16.0) -> np.ndarray:
    """Wall friction lambda per wall node of a duct: mean + std * xi, clamped >= 0."""
    xi = wall_surface_field(coords, nx, (ny - 1) / 2.0, (nz - 1) / 2.0,
                            2.0 * (ny + nz), sigma, rng)
    return np.maximum(mean + std * xi, 0.0)


# ---------------------------------------------------------------- spectra

@dataclass
class SpectralDraw:
    T: float
    omega0: float
    gamma_s: float
    omega_l: float
    gamma_l: float
    a_l: float = 0.5
    d: float = 1.0
    nq: int = 256
    nw: int = 1024
    lambda_target: float = 0.05

    @property
    def q_max(self) -> float:
        return 10.0 / self.d

    @property
    def w_max(self) -> float:
        return 20.0 * self.T


def corrugated_mask(nx: int, ny: int, rng: np.random.Generator | None, amp: float = 4.0,
                    wavelength: float = 64.0, base: int = 4, post: bool = False,
                    phases=None) -> np.ndarray:
    """Solid points, shaped (ny, nx), of a slab with wrinkled walls: the
    bottom wall fills y < lo(x), the top one y >= ny - hi(x), each
    round(base + amp sin(2 pi x / wavelength + phase)) with a random phase, or
    the two given phases (base >= amp keeps both >= 0; top phase = bottom
    phase + pi gives a meander of constant gap, equal phases a gap that
    narrows and widens).  post: a free-standing 3 x 3 post in the middle of
    the channel as well."""
    x = np.arange(nx)
    ph = np.asarray(phases, dtype=float) if phases is not None else rng.uniform(0.0, 2.0 * math.pi, 2)
    lo = np.round(base + amp * np.sin(2.0 * math.pi * x / wavelength + ph[0])).astype(int)
    hi = np.round(base + amp * np.sin(2.0 * math.pi * x / wavelength + ph[1])).astype(int)
    solid = np.zeros((ny, nx), dtype=bool)
    for i in range(nx):
        solid[: max(lo[i], 0), i] = True
        solid[ny - max(hi[i], 0):, i] = True
    if post:
        cx, cy = nx // 2, ny // 2
        solid[cy - 1:cy + 2, cx - 1:cx + 2] = True
    return solid


def draw_spectral(rng: np.random.Generator, nq: int = 256, nw: int = 1024) -> SpectralDraw:
    return SpectralDraw(T=rng.uniform(0.8, 1.2), omega0=rng.uniform(1.0, 3.0),
                        gamma_s=rng.uniform(0.3, 1.0), omega_l=rng.uniform(2.0, 4.0),
                        gamma_l=rng.uniform(0.5, 1.5), nq=nq, nw=nw)


def tube_plasmon_frequencies(coords: np.ndarray, nx: int, radius: float, cy: float, cz: float,
                             omega0: float, rng: np.random.Generator, sigma: float = 16.0,
                             spread: float = 0.2) -> np.ndarray:
    """Per-wall-node plasmon frequency Omega_k = omega0 (1 + spread * xi_k),
    xi a smooth field on the tube surface clipped to [-2.5, 2.5] (the paper's
    'charge carrier density' design parameter, varied along the wall)."""
    xi = wall_surface_field(coords, nx, cy, cz, 2.0 * math.pi * radius, sigma, rng)
    return omega0 * (1.0 + spread * np.clip(xi, -2.5, 2.5))


# ---------------------------------------------------------------- workloads

def tube_box(radius: int):
    """Box (ny, nz) and axis centre of a tube of integer radius R: box side
    2R + 8, centre in the middle of the box."""
    n = 2 * radius + 8
    c = (n - 1) / 2.0
    return n, n, c, c


@dataclass
class Channel:
    nx: int
    ny: int
    nz: int
    tau: float
    g: float
    seed_index: int
    qid: int = 0
    arrival_s: float = 0.0


def batch_channels(n: int = 256) -> list[Channel]:
    rng = rng_for("batch", 0)
    out = []
    for k in range(n):
        out.append(Channel(nx=int(rng.integers(32, 129)), ny=int(rng.integers(32, 65)),
                           nz=int(rng.integers(32, 65)), tau=float(rng.uniform(0.6, 1.2)),
                           g=float(rng.uniform(0.5e-6, 2e-6)), seed_index=k + 1, qid=k))
    return out


@dataclass
class Query:
    qid: int
    arrival_s: float
    radius: int
    tau: float
    g: float
    nx: int = 512
    spectral: SpectralDraw = field(default=None)


def serving_trace(n: int = 500, rate_per_s: float = 50.0, nx: int = 512,
                  radius_range=(8, 32)) -> list[Query]:
    rng = rng_for("serving", 0)
    t = 0.0
    out = []
    for k in range(n):
        t += rng.exponential(1.0 / rate_per_s)
        out.append(Query(qid=k, arrival_s=t, radius=int(rng.integers(radius_range[0], radius_range[1] + 1)),
                         tau=float(rng.uniform(0.6, 1.0)), g=1e-6, nx=nx,
                         spectral=draw_spectral(rng)))
    return out

"""Synthetic galaxy catalogues with linear redshift-space distortions.

Recipe (all steps seeded through numpy's PCG64):

G1  white noise N(0,1) on the N^3 grid;
G2  Gaussian field g with power P(k) = A k^ns exp(-(k/0.3)^2), k in h/Mpc,
    A chosen so that the per-cell variance (1/V) sum_{n!=0} P(k_n) equals sigma^2;
G3  lognormal density 1 + d = exp(g - var(g)/2), renormalised to unit mean;
G4  Poisson counts per cell with mean Np (1 + d) / N^3, positions uniform in
    the cell centred on the node;
G5  linear displacement psi(k) = i k / k^2 g(k) (the Kaiser-limit velocity
    of the paper's introduction, v = i H f delta k / k^2), taken from the
    particle's cell;
G6  redshift-space map s = r + f (psi . r_hat) r_hat (eq. r2s with the linear
    velocity); plane-parallel runs use r_hat = +z;
G7  positions in grid units u = x N / L, wrapped into [0, N) and quantised
    to multiples of 2^-12 so that u, u + 1/2, floor(u) and u - floor(u) are
    all exact in FP32.

The workload table mirrors the five sizes the estimator is exercised at
(64^3 monopole, 256^3 varying line of sight, 512^3 interlaced, the uneven
batch, and the 1024^3 stress case).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.fft as sfft

QUANT = 2.0 ** -12


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int                 # assignment / forward-transform grid
    n_reduce: int          # grid of the inverse transforms and triple sums
    box: float             # Mpc/h
    nparticles: int
    ns: float              # spectral slope
    sigma: float           # Gaussian rms per cell before the lognormal map
    f: float               # growth rate in the Kaiser displacement
    los: int               # 0: plane parallel along +z, 1: observer
    window: int            # 0 NGP, 1 CIC
    interlace: int
    lmax: int
    nbins: int
    dk: float              # bin width in units of k_f; centres k0 + b dk, k0 = dk
    P: int                 # number of 1-D modal functions
    nmodes: int
    seed: int

    @property
    def k0(self) -> float:
        return self.dk

    @property
    def kmin(self) -> float:
        return self.k0 - 0.5 * self.dk

    @property
    def kmax(self) -> float:
        return self.k0 + (self.nbins - 1) * self.dk + 0.5 * self.dk

    @property
    def nbar(self) -> float:
        return self.nparticles / self.box ** 3


WORKLOADS = {
    "c1_64": Workload("c1_64", 64, 64, 1000.0, 200_000, -1.5, 0.5, 0.5, 0, 1, 0, 0,
                      10, 2.0, 3, 10, 1000),
    "c2_256": Workload("c2_256", 256, 256, 1000.0, 3_000_000, -1.5, 0.5, 0.5, 1, 1, 0, 4,
                       20, 3.0, 6, 50, 2000),
    "c3_512": Workload("c3_512", 512, 512, 1000.0, 10_000_000, -1.8, 0.8, 0.7, 1, 1, 1, 4,
                       30, 5.0, 8, 100, 3000),
    "c5_1024": Workload("c5_1024", 1024, 1024, 2000.0, 50_000_000, -1.5, 0.5, 0.5, 1, 1, 0, 4,
                        30, 11.0, 8, 100, 5000),
}


def workload(name: str, **overrides) -> Workload:
    return dataclasses.replace(WORKLOADS[name], **overrides)


def batch_workload(mock: int, n: int) -> Workload:
    """One mock of the uneven batch: density 3e-4 (Mpc/h)^-3 in a 1000 Mpc/h box."""
    return Workload(f"c4_{mock}", n, 128, 1000.0, 300_000, -1.5, 0.5, 0.5, 1, 1, 0, 4,
                    20, 2.0, 6, 50, 4000 + mock)


def observer_grid_units(wl: Workload) -> np.ndarray:
    """Observer 1500 Mpc/h from the box corner along the negative diagonal."""
    o = -(1500.0 / math.sqrt(3.0)) * np.ones(3)
    return o * wl.n / wl.box


def _kgrid(n: int, box: float):
    kf = 2.0 * math.pi / box
    ia = sfft.fftfreq(n, 1.0 / n)
    iz = np.arange(n // 2 + 1, dtype=np.float64)
    return kf, ia, iz


def power_law_gaussian_spectrum(k, ns):
    """Shape of the input spectrum, k in h/Mpc (amplitude set separately)."""
    k = np.asarray(k, dtype=np.float64)
    out = np.zeros_like(k)
    nz = k > 0
    out[nz] = k[nz] ** ns * np.exp(-(k[nz] / 0.3) ** 2)
    return out


def _amplitude(n: int, box: float, ns: float, sigma: float) -> float:
    kf, ia, iz = _kgrid(n, box)
    V = box ** 3
    # full-grid sum over n != 0 via the half grid with Hermitian multiplicity
    kx2 = (ia ** 2)[:, None, None]
    ky2 = (ia ** 2)[None, :, None]
    kz2 = (iz ** 2)[None, None, :]
    k = kf * np.sqrt(kx2 + ky2 + kz2)
    shape = power_law_gaussian_spectrum(k, ns)
    mult = np.full(n // 2 + 1, 2.0)
    mult[0] = 1.0
    if n % 2 == 0:
        mult[-1] = 1.0
    s = float((shape * mult[None, None, :]).sum())
    return sigma ** 2 * V / s


def input_power(wl: Workload):
    """Callable P_in(k) (k in h/Mpc, result in (Mpc/h)^3) of a workload."""
    A = _amplitude(wl.n, wl.box, wl.ns, wl.sigma)
    return lambda k: A * power_law_gaussian_spectrum(k, wl.ns)


def gaussian_field(n: int, box: float, ns: float, sigma: float, seed: int,
                   return_spectrum: bool = False, amplitude: Optional[float] = None):
    """G1-G2: real Gaussian field on n^3 with power A k^ns exp(-(k/0.3)^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    white = rng.standard_normal((n, n, n))
    kf, ia, iz = _kgrid(n, box)
    V = box ** 3
    A = _amplitude(n, box, ns, sigma) if amplitude is None else amplitude
    G = sfft.rfftn(white, workers=-1)
    del white
    k = kf * np.sqrt((ia ** 2)[:, None, None] + (ia ** 2)[None, :, None] + (iz ** 2)[None, None, :])
    G *= np.sqrt(A * power_law_gaussian_spectrum(k, ns) * n ** 3 / V)
    G[0, 0, 0] = 0.0
    g = sfft.irfftn(G, s=(n, n, n), workers=-1)
    if return_spectrum:
        return g, G
    return g


def quantise_grid_units(u: np.ndarray, n: int) -> np.ndarray:
    """G7: wrap into [0, n) and round to multiples of 2^-12 (exact in FP32)."""
    q = np.round(np.mod(u, n) / QUANT) * QUANT
    q = np.where(q >= n, q - n, q)
    return q.astype(np.float32)


def lognormal_catalogue(wl: Workload, seed: Optional[int] = None, observer=None, log=None):
    """G1-G7 for one workload. Returns float32 arrays (ux, uy, uz) in grid units.
    log: optional callable given a line per generation step (large grids take minutes)."""
    n, box = wl.n, wl.box
    seed = wl.seed if seed is None else seed
    say = log if log is not None else (lambda *_: None)
    g, G = gaussian_field(n, box, wl.ns, wl.sigma, seed, return_spectrum=True)
    say("  gaussian field done")
    var = float(g.var())
    rho = np.exp(g - 0.5 * var)
    rho /= rho.mean()
    rng = np.random.Generator(np.random.PCG64(seed + 7_000_003))
    counts = rng.poisson(wl.nparticles * rho.ravel() / n ** 3)
    del rho
    say("  poisson counts done")
    cells = np.repeat(np.arange(n ** 3, dtype=np.int64), counts)
    del counts
    ix = cells // (n * n)
    iy = (cells // n) % n
    iz = cells % n
    u = np.empty((3, cells.size), dtype=np.float64)
    u[0] = ix + rng.uniform(-0.5, 0.5, cells.size)
    u[1] = iy + rng.uniform(-0.5, 0.5, cells.size)
    u[2] = iz + rng.uniform(-0.5, 0.5, cells.size)
    # G5: displacement in grid units from the cell the particle sits in
    kf, ia, izf = _kgrid(n, box)
    kx = (kf * ia)[:, None, None]
    ky = (kf * ia)[None, :, None]
    kz = (kf * izf)[None, None, :]
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2[0, 0, 0] = 1.0
    disp = np.empty((3, cells.size), dtype=np.float64)
    for a, ka in enumerate((kx, ky, kz)):
        psi_k = 1j * ka / k2 * G
        psi = sfft.irfftn(psi_k, s=(n, n, n), workers=-1) * (n / box)
        disp[a] = psi.ravel()[cells]
        del psi, psi_k
        say(f"  displacement component {a} done")
    del G, g, cells
    if wl.los == 0:
        u[2] += wl.f * disp[2]
    else:
        o = observer_grid_units(wl) if observer is None else np.asarray(observer, float)
        r = u - o[:, None]
        rhat = r / np.sqrt((r * r).sum(axis=0))
        proj = (disp * rhat).sum(axis=0)
        u += wl.f * proj * rhat
    return tuple(quantise_grid_units(u[a], n) for a in range(3))


def uniform_catalogue(n: int, nparticles: int, seed: int):
    """Unclustered positions (quantised grid units) for invariants and shot noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(0.0, n, (3, nparticles))
    return tuple(quantise_grid_units(u[a], n) for a in range(3))


def poisson_node_catalogue(n: int, nbar_cell: float, seed: int):
    """Poisson counts per node-centred cell, uniform inside the cell."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = rng.poisson(nbar_cell, n ** 3)
    cells = np.repeat(np.arange(n ** 3, dtype=np.int64), counts)
    ix, iy, iz = cells // (n * n), (cells // n) % n, cells % n
    u = np.stack([ix, iy, iz]).astype(np.float64) + rng.uniform(-0.5, 0.5, (3, cells.size))
    return tuple(quantise_grid_units(u[a], n) for a in range(3))

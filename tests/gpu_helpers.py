"""Test-side helpers: configuration of small runs, layout conversion between the
library's compact spectra and the oracle's half spectra, and error norms.
Contains no estimator arithmetic."""
import math

import numpy as np

from synth import catalog as C


def rel_norm(x, ref):
    """Normwise relative error ||x - ref||_2 / ||ref||_2."""
    x = np.asarray(x, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    d = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (d if d > 0 else 1.0))


def compact_to_half(cube, n, c, cz, n2max):
    """Compact GPU cube [2c+1][2c+1][cz] complex -> dict of (nx, ny, nz) positions and values
    restricted to kz <= c and |n|^2 <= n2max; returns (index arrays into an n^3 half spectrum, values)."""
    w = 2 * c + 1
    cube = np.asarray(cube).reshape(w, w, cz)
    ix, iy, kz = np.meshgrid(np.arange(w), np.arange(w), np.arange(cz), indexing="ij")
    nx, ny = ix - c, iy - c
    n2 = nx ** 2 + ny ** 2 + kz ** 2
    sel = (kz <= c) & (n2 <= n2max)
    return (np.mod(nx[sel], n), np.mod(ny[sel], n), kz[sel]), cube[sel], sel


def gpu_cube_to_numpy(t, nl, spec_elems):
    a = t.detach().cpu().numpy().reshape(nl, spec_elems, 2)
    return a[..., 0] + 1j * a[..., 1]


def half_to_compact(spec, n, c, cz, n2max):
    """Oracle half spectrum -> compact cube (zero outside |n|^2 <= n2max, kz <= c)."""
    w = 2 * c + 1
    ix, iy, kz = np.meshgrid(np.arange(w), np.arange(w), np.arange(cz), indexing="ij")
    nx, ny = ix - c, iy - c
    n2 = nx ** 2 + ny ** 2 + kz ** 2
    sel = (kz <= c) & (n2 <= n2max) & (n2 > 0)
    out = np.zeros((w, w, cz), np.complex128)
    out[sel] = spec[np.mod(nx[sel], n), np.mod(ny[sel], n), kz[sel]]
    return out


def pfid_table(wl, n2len):
    """Fiducial total power P_fid(k) = (1 + 2f/3 + f^2/5) P_in(k) + 1/nbar on |n|^2 = 0..n2len-1."""
    pin = C.input_power(wl)
    kf = 2 * math.pi / wl.box
    k = kf * np.sqrt(np.arange(n2len, dtype=np.float64))
    kais = 1 + 2 * wl.f / 3 + wl.f ** 2 / 5
    p = kais * pin(k) + 1.0 / wl.nbar
    p[0] = p[1]
    return p

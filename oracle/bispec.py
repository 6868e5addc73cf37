"""Plain FP64 implementation of the FFT bispectrum-multipole and modal estimators.

Test infrastructure only (see the package docstring). Everything here is
float64 / complex128 NumPy, written for a reader to check against the paper
by eye; speed is not a goal.

Paper: D. Regan, "An Inventory of Bispectrum Estimators for Redshift Space
Distortions" (arXiv:1708.05303).

Discrete conventions (the paper states the estimators in the continuum):

* lattice wavevector k = k_f n, n integer, k_f = 2 pi / L, V = L^3;
* forward DFT X(n) = sum_j x(j) exp(-2 pi i n.j / N) (unnormalised) and
  inverse x(j) = sum_n X(n) exp(+2 pi i n.j / N) (unnormalised);
* continuum <-> lattice: delta_c(k) = (V / N^3) delta(n),
  int d^3k / (2 pi)^3 <-> V^-1 sum_n, (2 pi)^3 delta_D <-> V delta_K;
* bin b has centre c_b = k0 + b dk (units of k_f) and holds the n with
  (2 c_b - dk)^2 <= 4 |n|^2 < (2 c_b + dk)^2, an integer comparison.

Parity pins: every function below is pinned by at least one non-GPU test
(brute-force closed-triangle sums, exact enumeration of triangle counts,
direct Legendre-weighted DFT, x-hat at nodes of both grids worked out by hand,
the closed-form LOS moments of a point source, the 1-D modal functions against
written-out Legendre polynomials, basis invariance of the modal reconstruction,
Gaussian zero mean of the binned and modal estimators, the quadratic-field
closed forms, separable-template recovery, CIC invariants, Kaiser multipole
ratios, Poisson shot noise). The CIC-compensated shot-noise *physics* is parity
unpinned (only its formula is); see ``shot_noise_binned``.
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.fft as sfft

__all__ = [
    "signed_freq", "assign", "density_contrast", "los_tensor_indices",
    "los_weighted_field", "forward", "dft_modes", "compensate", "interlace_combine",
    "legendre_moments", "legendre_moments_direct", "bin_edges4", "bin_of_n2",
    "n2_grid_half", "shell_field", "triangle_list", "triangle_counts_fft",
    "triangle_counts_brute", "closed_triangle_sum_brute", "binned_triple_sums", "binned_triple_sums_full",
    "binned_triple_sums_gemm", "triangle_counts_gemm",
    "binned_bispectrum", "shell_power", "power_multipoles", "skew_spectra", "integrated_bispectrum",
    "subvolume_unit_vectors", "integrated_bispectrum_local_los",
    "shot_noise_binned", "legendre_integral", "ring_factor", "shot_noise_multipoles",
    "shot_noise_coincidence", "modal_modes",
    "modal_q", "modal_filter", "modal_fields", "modal_numerators", "gram_matrix",
    "modal_solve", "modal_pivots", "modal_solve_pivoted", "modal_shot_noise", "batch_covariance", "spectrum_from_catalogue",
    "spectrum_from_field", "estimate", "Geometry", "n2_max_of",
]

WORKERS = -1


# --------------------------------------------------------------------------
# lattice helpers
# --------------------------------------------------------------------------

def signed_freq(n: int) -> np.ndarray:
    """Signed integer frequency of each FFT index: i for i < n/2, else i - n."""
    i = np.arange(n, dtype=np.int64)
    return np.where(i < (n + 1) // 2, i, i - n)


def n2_grid_half(n: int) -> np.ndarray:
    """|n|^2 on the half-spectrum index grid [n][n][n/2+1] (int64)."""
    f = signed_freq(n)
    fz = np.arange(n // 2 + 1, dtype=np.int64)
    return (f[:, None, None] ** 2 + f[None, :, None] ** 2 + fz[None, None, :] ** 2)


def half_freq_vectors(n: int):
    f = signed_freq(n).astype(np.float64)
    fz = np.arange(n // 2 + 1, dtype=np.float64)
    return f[:, None, None], f[None, :, None], fz[None, None, :]


# --------------------------------------------------------------------------
# mass assignment (the paper is silent; CIC / NGP with optional interlacing)
# --------------------------------------------------------------------------

def assign(ux, uy, uz, n: int, w=None, window: int = 1, shift: float = 0.0) -> np.ndarray:
    """Particle -> grid density (sum of weights per node), FP64.

    Positions are grid units in [0, n). Nodes sit at integer coordinates. The
    interlaced grid uses shift = 1/2, i.e. v = (u + 1/2) mod n.
    CIC: weight prod_a (1 - d_a) or d_a to the 8 nodes floor(v) + {0,1}^3.
    NGP: weight 1 to floor(v + 1/2).
    """
    v = [np.mod(np.asarray(a, dtype=np.float64) + shift, n) for a in (ux, uy, uz)]
    wt = np.ones_like(v[0]) if w is None else np.asarray(w, dtype=np.float64)
    rho = np.zeros(n ** 3, dtype=np.float64)
    if window == 0:
        idx = [np.mod(np.floor(a + 0.5).astype(np.int64), n) for a in v]
        flat = (idx[0] * n + idx[1]) * n + idx[2]
        rho += np.bincount(flat, weights=wt, minlength=n ** 3)
        return rho.reshape(n, n, n)
    i = [np.floor(a).astype(np.int64) for a in v]
    d = [a - b for a, b in zip(v, i)]
    for ox, oy, oz in itertools.product((0, 1), repeat=3):
        wx = d[0] if ox else 1.0 - d[0]
        wy = d[1] if oy else 1.0 - d[1]
        wz = d[2] if oz else 1.0 - d[2]
        flat = ((np.mod(i[0] + ox, n) * n + np.mod(i[1] + oy, n)) * n + np.mod(i[2] + oz, n))
        rho += np.bincount(flat, weights=wt * wx * wy * wz, minlength=n ** 3)
    return rho.reshape(n, n, n)


def density_contrast(rho: np.ndarray, wsum: float) -> np.ndarray:
    """delta = rho / rho_bar - 1 with rho_bar = sum(w) / n^3."""
    rbar = wsum / rho.size
    return rho / rbar - 1.0


# --------------------------------------------------------------------------
# line-of-sight weighting and Legendre moments
#   delta^(l)(k) = (2l+1) int d^3x e^{-ik.x} delta(x) L_l(k_hat . x_hat)
#   (Sec. 2, the LOS moment field defined after the power-spectrum
#   multipole estimator; sign e^{-i} as in the Fourier notation of Sec. 1)
# --------------------------------------------------------------------------

def los_tensor_indices(order: int) -> List[Tuple[int, ...]]:
    """Sorted index tuples i1 <= ... <= i_order over {0,1,2} (6 for 2, 15 for 4)."""
    return [t for t in itertools.combinations_with_replacement(range(3), order)]


def multinomial(t: Tuple[int, ...]) -> int:
    c = [t.count(a) for a in range(3)]
    return math.factorial(len(t)) // (math.factorial(c[0]) * math.factorial(c[1]) * math.factorial(c[2]))


def node_unit_vectors(n: int, shift: float, observer) -> np.ndarray:
    """x_hat at every node of the grid built with the given shift.

    Node j of the grid built from positions u + shift represents the point
    r = j - shift (grid units); x_hat = (r - o) / |r - o| for observer o.
    """
    j = np.arange(n, dtype=np.float64) - shift
    o = np.asarray(observer, dtype=np.float64)
    rx = (j - o[0])[:, None, None]
    ry = (j - o[1])[None, :, None]
    rz = (j - o[2])[None, None, :]
    norm = np.sqrt(rx ** 2 + ry ** 2 + rz ** 2)
    return rx / norm, ry / norm, rz / norm


def los_weighted_field(delta: np.ndarray, t: Tuple[int, ...], xhat) -> np.ndarray:
    """x_hat_{t1} ... x_hat_{tm} delta(x) at the nodes (t = () gives delta)."""
    out = delta.copy()
    for a in t:
        out = out * xhat[a]
    return out


def forward(field: np.ndarray) -> np.ndarray:
    """Unnormalised forward real-to-half-complex DFT, exp(-2 pi i n.j / N)."""
    return sfft.rfftn(field, workers=WORKERS)


def dft_modes(field: np.ndarray, modes) -> np.ndarray:
    """The forward DFT of the definition, F(m) = sum_j f(j) exp(-2 pi i m.j / N),
    at a few integer wavevectors m [M, 3] (any sign), in FP64: the sum over z
    for all M at once (x-blocks of the cube), then over y and x per mode. For
    grids too large for a whole transform (sampled parity)."""
    n = field.shape[0]
    m = np.asarray(modes, np.int64).reshape(-1, 3)
    j = np.arange(n, dtype=np.int64)
    ph = lambda a: np.exp(-2j * np.pi * (np.outer(j, m[:, a]) % n) / n)  # [n, M]
    ez, ey, ex = ph(2), ph(1), ph(0)
    G = np.empty((n, n, len(m)), np.complex128)
    for x0 in range(0, n, 32):
        blk = np.asarray(field[x0:x0 + 32], np.float64)
        G[x0:x0 + 32] = blk @ ez.real + 1j * (blk @ ez.imag)
    return np.array([ex[:, i] @ G[:, :, i] @ ey[:, i] for i in range(len(m))])


def window_half(n: int, window: int) -> np.ndarray:
    """Mass-assignment window on the half spectrum: prod_a sinc^p(pi n_a / N)."""
    p = 2 if window == 1 else 1
    fx, fy, fz = half_freq_vectors(n)
    def s(a):
        return np.sinc(a / n)  # numpy sinc(t) = sin(pi t) / (pi t)
    return (s(fx) * s(fy) * s(fz)) ** p


def compensate(F: np.ndarray, n: int, window: int) -> np.ndarray:
    return F / window_half(n, window)


def interlace_combine(F0: np.ndarray, Fh: np.ndarray, n: int) -> np.ndarray:
    """F = [F0 + exp(i pi (nx+ny+nz)/N) F_half] / 2 (grid built at u + 1/2)."""
    fx, fy, fz = half_freq_vectors(n)
    ph = np.exp(1j * math.pi * (fx + fy + fz) / n)
    return 0.5 * (F0 + ph * Fh)


def legendre_moments(T: Dict[Tuple[int, ...], np.ndarray], n: int, lmax: int,
                     plane_parallel: bool) -> List[np.ndarray]:
    """delta^(0,2,4)(n) from the transforms of the x_hat-product fields.

    With mu = k_hat . x_hat:
      A2 = sum_{i<=j} m_ij k_i k_j F_ij        (= FT[delta mu^2])
      A4 = sum_{i<=j<=k<=l} m k_i k_j k_k k_l F_ijkl   (= FT[delta mu^4])
      delta^0 = F, delta^2 = 5 (3 A2 - F) / 2, delta^4 = 9 (35 A4 - 30 A2 + 3 F) / 8,
    i.e. (2l+1) FT[delta L_l(mu)] with L_2 = (3mu^2-1)/2, L_4 = (35mu^4-30mu^2+3)/8.
    m are multinomial multiplicities. Plane parallel: x_hat = +z, A2 = kz^2 F.
    delta^l(0) = 0.
    """
    fx, fy, fz = half_freq_vectors(n)
    kn = np.sqrt(fx ** 2 + fy ** 2 + fz ** 2)
    kn[0, 0, 0] = 1.0
    khat = (fx / kn, fy / kn, fz / kn)
    F = T[()]
    out = [F.copy()]
    if lmax >= 2:
        if plane_parallel:
            A2 = khat[2] ** 2 * F
        else:
            A2 = np.zeros_like(F)
            for t in los_tensor_indices(2):
                A2 = A2 + multinomial(t) * khat[t[0]] * khat[t[1]] * T[t]
        out.append(2.5 * (3.0 * A2 - F))
    if lmax >= 4:
        if plane_parallel:
            A4 = khat[2] ** 4 * F
        else:
            A4 = np.zeros_like(F)
            for t in los_tensor_indices(4):
                A4 = A4 + multinomial(t) * khat[t[0]] * khat[t[1]] * khat[t[2]] * khat[t[3]] * T[t]
        out.append(1.125 * (35.0 * A4 - 30.0 * A2 + 3.0 * F))
    for a in out:
        a[0, 0, 0] = 0.0
    return out


def legendre_poly(ell: int, mu):
    if ell == 0:
        return np.ones_like(mu)
    if ell == 2:
        return 0.5 * (3.0 * mu ** 2 - 1.0)
    if ell == 4:
        return (35.0 * mu ** 4 - 30.0 * mu ** 2 + 3.0) / 8.0
    raise ValueError(ell)


def legendre_moments_direct(delta: np.ndarray, nvec, ell: int, shift: float,
                            observer=None) -> complex:
    """(2l+1) sum_j exp(-2 pi i n.j/N) delta(j) L_l(k_hat . x_hat_j), one n.

    Direct evaluation of the LOS moment definition (no tensor expansion, no FFT);
    used to pin ``legendre_moments``. observer None means plane parallel (+z).
    """
    n = delta.shape[0]
    nv = np.asarray(nvec, dtype=np.float64)
    khat = nv / np.linalg.norm(nv)
    j = np.arange(n, dtype=np.float64)
    if observer is None:
        mu = np.full(delta.shape, khat[2])
    else:
        xh = node_unit_vectors(n, shift, observer)
        mu = khat[0] * xh[0] + khat[1] * xh[1] + khat[2] * xh[2]
    ph = np.exp(-2j * math.pi * (nv[0] * j[:, None, None] + nv[1] * j[None, :, None]
                                 + nv[2] * j[None, None, :]) / n)
    return complex((2 * ell + 1) * np.sum(ph * delta * legendre_poly(ell, mu)))


# --------------------------------------------------------------------------
# catalogue / field -> delta^(l)(n)
# --------------------------------------------------------------------------

def spectrum_from_field(delta_list: Sequence[np.ndarray], shifts: Sequence[float], n: int,
                        lmax: int, observer, window: Optional[int]) -> List[np.ndarray]:
    """delta^(l)(n) on the full half spectrum [n][n][n/2+1] from 1 or 2 contrast grids.

    observer None: plane-parallel LOS (+z). window None: no compensation.
    Two grids are combined by interlacing (second grid built at u + 1/2).
    """
    plane = observer is None
    tensors = [()]
    if not plane and lmax >= 2:
        tensors += los_tensor_indices(2)
    if not plane and lmax >= 4:
        tensors += los_tensor_indices(4)
    T = {}
    for t in tensors:
        acc = None
        Fs = []
        for delta, s in zip(delta_list, shifts):
            if plane:
                fld = delta
            else:
                xh = node_unit_vectors(n, s, observer)
                fld = los_weighted_field(delta, t, xh)
            F = forward(fld)
            if window is not None:
                F = compensate(F, n, window)
            Fs.append(F)
        acc = Fs[0] if len(Fs) == 1 else interlace_combine(Fs[0], Fs[1], n)
        T[t] = acc
    return legendre_moments(T, n, lmax, plane)


def spectrum_from_catalogue(ux, uy, uz, n: int, lmax: int, observer, window: int = 1,
                            interlace: int = 0, w=None, compensate_window: bool = True):
    """Catalogue -> (delta^(l) list, sum of weights)."""
    wsum = float(np.sum(w)) if w is not None else float(np.asarray(ux).size)
    shifts = [0.0, 0.5] if interlace else [0.0]
    deltas = [density_contrast(assign(ux, uy, uz, n, w, window, s), wsum) for s in shifts]
    spec = spectrum_from_field(deltas, shifts, n, lmax, observer,
                               window if compensate_window else None)
    return spec, wsum


# --------------------------------------------------------------------------
# shells and triangles (Sec. 3.1, standard estimator and its FFT form)
# --------------------------------------------------------------------------

def bin_edges4(k0: float, dk: float, nb: int):
    """Integer edges (2c-dk)^2 <= 4 n^2 < (2c+dk)^2 for each bin b (c = k0 + b dk)."""
    lo, hi = [], []
    for b in range(nb):
        c = k0 + b * dk
        a, z = 2.0 * c - dk, 2.0 * c + dk
        if abs(a - round(a)) > 1e-12 or abs(z - round(z)) > 1e-12:
            raise ValueError("2 k0 and dk must be integers")
        lo.append(int(round(a)) ** 2)
        hi.append(int(round(z)) ** 2)
    return np.array(lo, np.int64), np.array(hi, np.int64)


def bin_of_n2(n2, k0: float, dk: float, nb: int):
    """Bin id of each |n|^2 (-1 outside every bin)."""
    lo, hi = bin_edges4(k0, dk, nb)
    n2 = np.asarray(n2, dtype=np.int64)
    out = np.full(n2.shape, -1, dtype=np.int64)
    for b in range(nb):
        out[(4 * n2 >= lo[b]) & (4 * n2 < hi[b])] = b
    return out


def n2_max_of(k0: float, dk: float, nb: int) -> int:
    """Largest |n|^2 inside the last bin."""
    lo, hi = bin_edges4(k0, dk, nb)
    return int((hi[-1] - 1) // 4)


def shell_field(spec: np.ndarray, mask: np.ndarray, n: int) -> np.ndarray:
    """Unnormalised inverse DFT of spec * mask: D(x) = sum_{n in shell} e^{i n.x} delta(n)."""
    return sfft.irfftn(spec * mask, s=(n, n, n), workers=WORKERS) * float(n) ** 3


def triangle_list(nb: int) -> List[Tuple[int, int, int]]:
    """All (b1, b2, b3) with b1 >= b2 >= b3, lexicographic in (b1, b2, b3)."""
    return [(b1, b2, b3) for b1 in range(nb) for b2 in range(b1 + 1) for b3 in range(b2 + 1)]


def _crop_spec(spec: np.ndarray, n_from: int, n_to: int) -> np.ndarray:
    """Copy the modes with |n_a| < n_to/2 of a half spectrum into a smaller grid."""
    if n_from == n_to:
        return spec
    h = n_to // 2
    out = np.zeros((n_to, n_to, n_to // 2 + 1), dtype=spec.dtype)
    idx_from = np.r_[0:h, n_from - h + 1:n_from]
    idx_to = np.r_[0:h, n_to - h + 1:n_to]
    out[np.ix_(idx_to, idx_to, np.arange(h))] = spec[np.ix_(idx_from, idx_from, np.arange(h))]
    return out


def triangle_counts_fft(nr: int, k0: float, dk: float, nb: int):
    """N_tri(b1,b2,b3) = round(sum_x I_b1 I_b2 I_b3 / N'^3), I_b = inverse DFT of 1_b.

    This is V_B of the standard estimator on the lattice (Sec. 3.1): the number
    of (n1, n2, n3) with n_i in shell b_i and n1 + n2 + n3 = 0 (mod N'); equal to
    exact closure when 3 c_max < N'. Returns (list of triangles, counts, residual).
    """
    bins = bin_of_n2(n2_grid_half(nr), k0, dk, nb)
    I = np.stack([shell_field(np.ones((nr, nr, nr // 2 + 1)), bins == b, nr).ravel()
                  for b in range(nb)])
    tris = triangle_list(nb)
    C = np.empty(len(tris))
    for i, (b1, b2, b3) in enumerate(tris):
        C[i] = np.dot(I[b1] * I[b2], I[b3]) / float(nr) ** 3
    cnt = np.rint(C).astype(np.int64)
    resid = float(np.max(np.abs(C - cnt))) if len(C) else 0.0
    return tris, cnt, resid


def _shell_modes(k0, dk, nb, cmax):
    r = np.arange(-cmax, cmax + 1)
    nx, ny, nz = np.meshgrid(r, r, r, indexing="ij")
    n2 = nx ** 2 + ny ** 2 + nz ** 2
    b = bin_of_n2(n2, k0, dk, nb)
    return np.stack([nx[b >= 0], ny[b >= 0], nz[b >= 0]], axis=1), b[b >= 0]


def triangle_counts_brute(k0: float, dk: float, nb: int, tris=None, chunk: int = 2048):
    """Direct enumeration: #{n1 in b1, n2 in b2 : -(n1+n2) in b3} with exact closure.

    For every pair of shells (b1, b2) the third side n3 = -(n1 + n2) is formed
    for all mode pairs and histogrammed by its shell. Pure integer arithmetic.
    """
    lo, hi = bin_edges4(k0, dk, nb)
    cmax = int(math.isqrt(int((hi[-1] - 1) // 4)))
    modes, bid = _shell_modes(k0, dk, nb, cmax)
    full = np.zeros((nb, nb, nb), np.int64)
    need = None if tris is None else {(t[0], t[1]) for t in tris}
    for b1 in range(nb):
        m1 = modes[bid == b1]
        for b2 in range(nb):
            if need is not None and (b1, b2) not in need:
                continue
            m2 = modes[bid == b2]
            for s in range(0, m1.shape[0], chunk):
                n3 = -(m1[s:s + chunk, None, :] + m2[None, :, :])
                b3 = bin_of_n2((n3 * n3).sum(-1), k0, dk, nb).ravel()
                full[b1, b2] += np.bincount(b3[b3 >= 0], minlength=nb)
    tris = triangle_list(nb) if tris is None else tris
    return np.array([full[a, b, c] for a, b, c in tris], np.int64)


def _lookup(spec_half: np.ndarray, n: int, nv: np.ndarray) -> np.ndarray:
    """delta(n) for signed integer vectors nv [M,3] from a half spectrum (Hermitian)."""
    nx, ny, nz = nv[:, 0], nv[:, 1], nv[:, 2]
    neg = nz < 0
    sx = np.where(neg, -nx, nx) % n
    sy = np.where(neg, -ny, ny) % n
    sz = np.where(neg, -nz, nz)
    v = spec_half[sx, sy, sz]
    return np.where(neg, np.conj(v), v)


def closed_triangle_sum_brute(specs: Sequence[np.ndarray], n: int, masks_n2,
                              modular: bool = False) -> complex:
    """sum over n1 in S1, n2 in S2, n3 = -(n1+n2) in S3 of X1(n1) X2(n2) X3(n3).

    The defining closed-triangle sum of the standard estimator (Sec. 3.1),
    enumerated directly. masks_n2 are three predicates on |n|^2 (shell
    membership); with modular=True, n3 is reduced mod n into (-n/2, n/2]
    before the membership test (what a DFT of size n computes).
    """
    h = n // 2
    r = np.arange(-h + 1, h + 1)
    nx, ny, nz = np.meshgrid(r, r, r, indexing="ij")
    allv = np.stack([nx.ravel(), ny.ravel(), nz.ravel()], axis=1)
    n2 = (allv ** 2).sum(1)
    sel = [allv[m(n2)] for m in masks_n2]
    v1 = _lookup(specs[0], n, sel[0])
    v2 = _lookup(specs[1], n, sel[1])
    tot = 0.0 + 0.0j
    for i in range(sel[0].shape[0]):
        n3 = -(sel[0][i][None, :] + sel[1])
        if modular:
            n3 = (n3 + h - 1) % n - h + 1
        ok = masks_n2[2]((n3 ** 2).sum(1))
        if not np.any(ok):
            continue
        v3 = _lookup(specs[2], n, n3[ok])
        tot += v1[i] * np.sum(v2[ok] * v3)
    return complex(tot)


def binned_triple_sums(spec_l: Sequence[np.ndarray], n: int, nr: int, k0: float, dk: float,
                       nb: int, tris=None):
    """T^l(b1,b2,b3) = sum_x D^l_b1 D^0_b2 D^0_b3 over the N'^3 grid.

    Eq. (Standard_ell_Estim) of Sec. 3.1: the multipole is placed on the
    largest side b1 and the other two use the monopole. Fields are the
    unnormalised inverse DFTs at N' (= nr) of the shell-filtered delta^(l).
    """
    tris = triangle_list(nb) if tris is None else tris
    bins = bin_of_n2(n2_grid_half(nr), k0, dk, nb)
    specs = [_crop_spec(s, n, nr) for s in spec_l]
    D = [np.stack([shell_field(sp, bins == b, nr).ravel() for b in range(nb)]) for sp in specs]
    T = np.empty((len(specs), len(tris)))
    for i, (b1, b2, b3) in enumerate(tris):
        pair = D[0][b2] * D[0][b3]
        for li in range(len(specs)):
            T[li, i] = np.dot(D[li][b1], pair)
    return tris, T


def binned_triple_sums_gemm(spec_l: Sequence[np.ndarray], n: int, nr: int, k0: float, dk: float,
                            nb: int, tris=None):
    """The triple sums of ``binned_triple_sums`` (eq. Standard_ell_Estim, Sec.
    3.1), T^l(b1,b2,b3) = sum_x D^l_b1 D^0_b2 D^0_b3, with the sum over x of all
    (b2, b3) for one (l, b1) taken as one matrix product of the field stacks:
    T^l(b1, ., .) = (D^l_b1 * D0) D0^T, D0 = [D^0_b][x]. Same definition, a
    library matrix product as the step, for grids where a loop of dot products
    is slow."""
    tris = triangle_list(nb) if tris is None else tris
    bins = bin_of_n2(n2_grid_half(nr), k0, dk, nb)
    specs = [_crop_spec(s, n, nr) for s in spec_l]
    D0 = np.stack([shell_field(specs[0], bins == b, nr).ravel() for b in range(nb)])
    need = sorted({t[0] for t in tris})
    T = np.empty((len(specs), len(tris)))
    for li, sp in enumerate(specs):
        for b1 in need:
            d1 = D0[b1] if li == 0 else shell_field(sp, bins == b1, nr).ravel()
            G = (D0 * d1[None, :]) @ D0.T
            for i, t in enumerate(tris):
                if t[0] == b1:
                    T[li, i] = G[t[1], t[2]]
    return tris, T


def triangle_counts_gemm(nr: int, k0: float, dk: float, nb: int):
    """``triangle_counts_fft`` with the sums over x of all (b2, b3) for one b1
    taken as one matrix product (I_b1 * I) I^T, I = [I_b][x]."""
    bins = bin_of_n2(n2_grid_half(nr), k0, dk, nb)
    I = np.stack([shell_field(np.ones((nr, nr, nr // 2 + 1)), bins == b, nr).ravel() for b in range(nb)])
    tris = triangle_list(nb)
    C = np.empty(len(tris))
    G = {b1: (I * I[b1][None, :]) @ I.T / float(nr) ** 3 for b1 in range(nb)}
    for i, (b1, b2, b3) in enumerate(tris):
        C[i] = G[b1][b2, b3]
    cnt = np.rint(C).astype(np.int64)
    resid = float(np.max(np.abs(C - cnt))) if len(C) else 0.0
    return tris, cnt, resid


def binned_triple_sums_full(spec_l: Sequence[np.ndarray], n: int, nr: int, k0: float, dk: float,
                            nb: int, tris=None):
    """T^(l1 l2 l3)(b1,b2,b3) = sum_x D^l1_b1 D^l2_b2 D^l3_b3 over the N'^3 grid.

    The general Legendre decomposition of Sec. 3 (B^(l1 l2 l3), one multipole
    per side), in the FFT form of eq. (Standard_ell_Estim) with each side's
    field built from its own LOS moment delta^(l_i) (the line of sight at x for
    every side, as for B^(l) = B^(l00)). Combination index (l1 nl + l2) nl + l3
    over l_i = 0, 2, ..., 2 (nl - 1). Returns (tris, combos, T [nl^3][ntri])."""
    tris = triangle_list(nb) if tris is None else tris
    bins = bin_of_n2(n2_grid_half(nr), k0, dk, nb)
    specs = [_crop_spec(s, n, nr) for s in spec_l]
    D = [np.stack([shell_field(sp, bins == b, nr).ravel() for b in range(nb)]) for sp in specs]
    nl = len(specs)
    combos = [(l1, l2, l3) for l1 in range(nl) for l2 in range(nl) for l3 in range(nl)]
    T = np.empty((len(combos), len(tris)))
    for i, (b1, b2, b3) in enumerate(tris):
        for ci, (l1, l2, l3) in enumerate(combos):
            T[ci, i] = np.dot(D[l1][b1], D[l2][b2] * D[l3][b3])
    return tris, combos, T


def binned_bispectrum(T: np.ndarray, counts: np.ndarray, n: int, nr: int, box: float):
    """B^l = V^2 T^l / (N^9 N'^3 N_tri): the lattice form of
    (1 / V_B) sum_closed delta_c delta_c delta_c / V (Sec. 3.1)."""
    V = box ** 3
    with np.errstate(divide="ignore", invalid="ignore"):
        B = V ** 2 * T / (float(n) ** 9 * float(nr) ** 3 * counts[None, :].astype(np.float64))
    return np.where(counts[None, :] > 0, B, 0.0)


def shell_power(spec0: np.ndarray, n: int, k0: float, dk: float, nb: int, box: float):
    """Pbar_b = V sum_{n in b} |delta^0(n)|^2 / (N^6 N_b) over the full lattice,
    the shell average of the power-spectrum estimator of Sec. 2 (monopole).
    Returns (Pbar, N_b)."""
    n2 = n2_grid_half(n)
    bins = bin_of_n2(n2, k0, dk, nb)
    mult = np.full(n // 2 + 1, 2.0)
    mult[0] = 1.0
    if n % 2 == 0:
        mult[-1] = 1.0
    m = np.broadcast_to(mult[None, None, :], n2.shape)
    p = np.abs(spec0) ** 2
    V = box ** 3
    P = np.empty(nb)
    Nb = np.empty(nb, np.int64)
    for b in range(nb):
        sel = bins == b
        Nb[b] = int(round(m[sel].sum()))
        P[b] = V * float((p[sel] * m[sel]).sum()) / (float(n) ** 6 * Nb[b])
    return P, Nb


def power_multipoles(spec_l: Sequence[np.ndarray], n: int, k0: float, dk: float, nb: int, box: float):
    """Power-spectrum multipoles of Sec. 2, eq. (PowSpecMultipole): the shell
    average over directions of delta^(l)(k) delta^(0)(-k) / V, on the lattice
    P^(l)_b = V sum_{n in b} Re[delta^(l)(n) conj(delta^(0)(n))] / (N^6 N_b)
    over the full lattice (delta^(0)(-n) = conj delta^(0)(n) for a real field;
    the pair n, -n of the half spectrum contributes twice the real part).
    spec_l: half spectra [nl][n][n][n//2+1] from spectrum_from_field. Raw: no
    shot-noise term (the paper gives none). Returns (P [nl][nb], N_b)."""
    n2 = n2_grid_half(n)
    bins = bin_of_n2(n2, k0, dk, nb)
    mult = np.full(n // 2 + 1, 2.0)
    mult[0] = 1.0
    if n % 2 == 0:
        mult[-1] = 1.0
    m = np.broadcast_to(mult[None, None, :], n2.shape)
    V = box ** 3
    P = np.zeros((len(spec_l), nb))
    Nb = np.empty(nb, np.int64)
    for b in range(nb):
        sel = bins == b
        Nb[b] = int(round(m[sel].sum()))
        for li, s in enumerate(spec_l):
            prod = np.real(s[sel] * np.conj(spec_l[0][sel]))
            P[li, b] = V * float((prod * m[sel]).sum()) / (float(n) ** 6 * Nb[b]) if Nb[b] else 0.0
    return P, Nb


def skew_spectra(spec_l: Sequence[np.ndarray], n: int, nr: int, k0: float, dk: float, nb: int, box: float,
                 square_range: str = "shells"):
    """Skew-spectrum multipoles S_{*,l} of Sec. 3.2 (the estimator after
    eq. skewspecQ, with Q the convolution delta^(0) * delta^(0)): the shell
    average over directions of [delta^(0) * delta^(0)](-k) delta^(l)(k) / V.

    The product is formed in real space: d(x) is the unnormalised inverse DFT at
    N' of delta^(0) kept on the union of the bins, Q(n) = DFT[d^2](n) at N'
    (no wrap-around for |n_a| <= c while 3 c < N'), and on the lattice
      S^l_b = V sum_{n in b} Re[conj(Q(n)) delta^(l)(n)] / (N^9 N'^3 N_b)
    over the full lattice (the 1/V and the band are readings; with them
    S^l_b N_b = V / (N^9 N'^3) sum_{b2, b3} T^l(b, b2, b3), the discrete form of
    S = int d^3q / (2 pi)^3 B(k, q, |k + q|)). Returns (S [nl][nb], N_b).

    square_range "ball": the squared field keeps delta^(0) on every mode
    0 < |n|^2 <= n2max of the bins' band (the modes below the first shell
    too), the closest the no-wrap condition allows to squaring the full
    field; the sum rule then no longer holds."""
    n2 = n2_grid_half(nr)
    bins = bin_of_n2(n2, k0, dk, nb)
    specs = [_crop_spec(s, n, nr) for s in spec_l]
    if square_range == "shells":
        keep = bins >= 0
    elif square_range == "ball":
        keep = (n2 > 0) & (n2 <= n2_max_of(k0, dk, nb))
    else:
        raise ValueError("square_range must be 'shells' or 'ball'")
    d = shell_field(specs[0], keep, nr)
    Q = forward(d * d)
    mult = np.full(nr // 2 + 1, 2.0)
    mult[0] = 1.0
    if nr % 2 == 0:
        mult[-1] = 1.0
    m = np.broadcast_to(mult[None, None, :], n2.shape)
    V = box ** 3
    S = np.zeros((len(specs), nb))
    Nb = np.empty(nb, np.int64)
    for b in range(nb):
        sel = bins == b
        Nb[b] = int(round(m[sel].sum()))
        for li, sp in enumerate(specs):
            prod = np.real(np.conj(Q[sel]) * sp[sel])
            S[li, b] = V * float((prod * m[sel]).sum()) / (float(n) ** 9 * float(nr) ** 3 * Nb[b]) if Nb[b] else 0.0
    return S, Nb


def integrated_bispectrum(delta: np.ndarray, s: int, lmax: int, observer, window, box: float,
                          k0: float, dk: float, nb: int):
    """Integrated bispectrum multipoles of Sec. 3.4 (eq. integBisp and the RSD
    estimator that follows it): iB^(l)(k) = (1/N_s) sum_i P^(l)_i(k) dbar^(0)_i
    over the N_s = s^3 cubic sub-volumes of side M = N/s.

    delta: density contrast on the N^3 grid (nodes at integer coordinates).
    For sub-volume i with nodes origin_i + [0, M)^3:
      F_i = DFT_M of delta on the sub-volume (unnormalised), divided by the
            assignment window at the sub-volume frequencies (same cell size);
            window None: no compensation;
      dbar_i = F_i(0) / M^3, the mean overdensity of the sub-volume;
      P^(l)_i(k_b) = V_s sum_{n in b} (2l+1) L_l(nhat . e_i) |F_i(n)|^2 / (M^6 N_b)
            over the full lattice, V_s = (L / s)^3, the power-spectrum multipole
            with a single line of sight e_i per sub-volume: the unit vector from
            the observer to the sub-volume centre origin_i + (M - 1)/2 (z when
            observer is None). The local line of sight is a reading (the
            sub-volumes are small, so the plane-parallel form applies inside).
    Bins (k0, dk, nb) are in units of the sub-volume fundamental 2 pi s / L.
    Returns (iB [nl][nb], P [N_s][nl][nb], dbar [N_s], N_b)."""
    n = delta.shape[0]
    assert n % s == 0
    m = n // s
    nl = lmax // 2 + 1
    n2 = n2_grid_half(m)
    bins = bin_of_n2(n2, k0, dk, nb)
    fx, fy, fz = half_freq_vectors(m)
    kn = np.sqrt(np.maximum(n2, 1)).astype(np.float64)
    mult = np.full(m // 2 + 1, 2.0)
    mult[0] = 1.0
    if m % 2 == 0:
        mult[-1] = 1.0
    mm = np.broadcast_to(mult[None, None, :], n2.shape)
    Nb = np.array([int(round(mm[bins == b].sum())) for b in range(nb)], np.int64)
    Vs = (box / s) ** 3
    W = window_half(m, window) if window is not None else None
    P = np.zeros((s ** 3, nl, nb))
    dbar = np.zeros(s ** 3)
    for i in range(s ** 3):
        ox, oy, oz = (i // (s * s)) * m, ((i // s) % s) * m, (i % s) * m
        F = forward(delta[ox:ox + m, oy:oy + m, oz:oz + m])
        dbar[i] = float(np.real(F[0, 0, 0])) / float(m) ** 3
        if W is not None:
            F = F / W
        if observer is None:
            e = np.array([0.0, 0.0, 1.0])
        else:
            cvec = np.array([ox, oy, oz], np.float64) + 0.5 * (m - 1) - np.asarray(observer, np.float64)
            e = cvec / np.linalg.norm(cvec)
        mu = (fx * e[0] + fy * e[1] + fz * e[2]) / kn
        p2 = np.abs(F) ** 2 * mm
        for li in range(nl):
            wl = (4 * li + 1) * legendre_poly(2 * li, mu) * p2
            for b in range(nb):
                sel = bins == b
                P[i, li, b] = Vs * float(wl[sel].sum()) / (float(m) ** 6 * Nb[b]) if Nb[b] else 0.0
    iB = np.einsum("ilb,i->lb", P, dbar) / s ** 3
    return iB, P, dbar, Nb


def subvolume_unit_vectors(m: int, origin, observer):
    """x_hat at the nodes of the sub-volume whose node (0, 0, 0) is grid node
    origin: node origin + j represents the point r = origin + j (grid units),
    x_hat = (r - o) / |r - o|."""
    j = np.arange(m, dtype=np.float64)
    o = np.asarray(observer, dtype=np.float64)
    rx = (origin[0] + j - o[0])[:, None, None]
    ry = (origin[1] + j - o[1])[None, :, None]
    rz = (origin[2] + j - o[2])[None, None, :]
    norm = np.sqrt(rx ** 2 + ry ** 2 + rz ** 2)
    return rx / norm, ry / norm, rz / norm


def integrated_bispectrum_local_los(delta: np.ndarray, s: int, lmax: int, observer, window, box: float,
                                    k0: float, dk: float, nb: int, subvolumes=None):
    """Integrated bispectrum multipoles of Sec. 3.4 with the power-spectrum
    multipoles of each sub-volume taken as in Sec. 2 (eq. PowSpecMultipole):
    the line of sight x_hat varies over the nodes of the sub-volume.

    For sub-volume i (nodes origin_i + [0, M)^3, M = N / s):
      delta^(l)_i(n) = (2l+1) sum_x e^{-2 pi i n.x / M} delta(origin_i + x) L_l(n_hat . x_hat),
            x_hat from the observer to the node, formed from the transforms of
            the x_hat-product fields (legendre_moments), each divided by the
            assignment window at the sub-volume frequencies (window None: none);
      dbar_i = (DFT_M of delta)(0) / M^3;
      P^(l)_i(k_b) = V_s sum_{n in b} Re[delta^(l)_i(n) conj delta^(0)_i(n)] / (M^6 N_b)
            over the full lattice (Hermitian halves counted twice).
    iB^(l) = (1/N_s) sum_i P^(l)_i dbar_i. Bins as integrated_bispectrum.
    subvolumes: optional list of sub-volume indices to evaluate (the others
    stay zero in P and dbar, and iB is then not meaningful).
    Returns (iB [nl][nb], P [N_s][nl][nb], dbar [N_s], N_b)."""
    n = delta.shape[0]
    assert n % s == 0 and observer is not None
    m = n // s
    nl = lmax // 2 + 1
    n2 = n2_grid_half(m)
    bins = bin_of_n2(n2, k0, dk, nb)
    mult = np.full(m // 2 + 1, 2.0)
    mult[0] = 1.0
    if m % 2 == 0:
        mult[-1] = 1.0
    mm = np.broadcast_to(mult[None, None, :], n2.shape)
    Nb = np.array([int(round(mm[bins == b].sum())) for b in range(nb)], np.int64)
    Vs = (box / s) ** 3
    W = window_half(m, window) if window is not None else None
    tensors = [()]
    if lmax >= 2:
        tensors += los_tensor_indices(2)
    if lmax >= 4:
        tensors += los_tensor_indices(4)
    P = np.zeros((s ** 3, nl, nb))
    dbar = np.zeros(s ** 3)
    for i in (range(s ** 3) if subvolumes is None else subvolumes):
        org = ((i // (s * s)) * m, ((i // s) % s) * m, (i % s) * m)
        sub = delta[org[0]:org[0] + m, org[1]:org[1] + m, org[2]:org[2] + m]
        xh = subvolume_unit_vectors(m, org, observer)
        T = {}
        for t in tensors:
            F = forward(los_weighted_field(sub, t, xh))
            if t == ():
                dbar[i] = float(np.real(F[0, 0, 0])) / float(m) ** 3
            T[t] = F / W if W is not None else F
        dl = legendre_moments(T, m, lmax, False)
        for li in range(nl):
            cr = np.real(dl[li] * np.conj(dl[0])) * mm
            for b in range(nb):
                sel = bins == b
                P[i, li, b] = Vs * float(cr[sel].sum()) / (float(m) ** 6 * Nb[b]) if Nb[b] else 0.0
    iB = np.einsum("ilb,i->lb", P, dbar) / s ** 3
    return iB, P, dbar, Nb


def shot_noise_binned(B0: np.ndarray, Pbar: np.ndarray, tris, nbar: float) -> np.ndarray:
    """B0_sub = B0 - (Pbar_b1 + Pbar_b2 + Pbar_b3) / nbar + 2 / nbar^2 (Poisson, l = 0).

    The paper gives no shot-noise model; this reading uses the Poisson
    bispectrum shot noise with the raw (shot-noise inclusive) shell power.
    Parity: formula pinned; its physics with CIC compensation is unpinned.
    """
    s = np.array([Pbar[a] + Pbar[b] + Pbar[c] for a, b, c in tris])
    return B0 - s / nbar + 2.0 / nbar ** 2


# --------------------------------------------------------------------------
# Poisson shot noise of the multipoles B_l, l > 0 (the paper gives none; a
# reading derived for the LOS-on-the-first-leg estimator of Sec. 3.1 / eq.
# (Standard_ell_Estim); see shot_noise_multipoles)
# --------------------------------------------------------------------------

def legendre_integral(ell: int, mu):
    """int_0^mu L_l(t) dt for l = 0, 2, 4 (L_2 = (3t^2 - 1)/2, L_4 = (35t^4 - 30t^2 + 3)/8)."""
    mu = np.asarray(mu, dtype=np.float64)
    if ell == 0:
        return mu
    if ell == 2:
        return 0.5 * (mu ** 3 - mu)
    if ell == 4:
        return (7.0 * mu ** 5 - 10.0 * mu ** 3 + 3.0 * mu) / 8.0
    raise ValueError("l must be 0, 2 or 4")


def ring_factor(ell: int, c1: float, c2: float, c3: float, dk: float, nq: int = 32) -> float:
    """W_l(b1, b2 | b3): the mean of L_l(k1_hat . k2_hat) over the closed
    triangles k1 + k2 + k3 = 0 with |k_i| in the shell [c_i - dk/2, c_i + dk/2)
    (units of k_f), in the continuum: closed triangles with side lengths
    (k1, k2, k3) have density k1 k2 k3 dk1 dk2 dk3, and k1_hat . k2_hat =
    (k3^2 - k1^2 - k2^2) / (2 k1 k2) =: mu. The k3 integral is exact
    (k3 dk3 = k1 k2 dmu, over the k3 shell intersected with |k1 - k2| <= k3 <=
    k1 + k2), the k1 and k2 integrals nq-point Gauss-Legendre rules over their
    shells. l = 0 gives 1."""
    x, w = np.polynomial.legendre.leggauss(nq)
    k1 = c1 + 0.5 * dk * x
    k2 = c2 + 0.5 * dk * x
    K1, K2 = np.meshgrid(k1, k2, indexing="ij")
    Wq = np.outer(w, w)
    lo, hi = c3 - 0.5 * dk, c3 + 0.5 * dk
    m_lo = (np.maximum(lo, np.abs(K1 - K2)) ** 2 - K1 ** 2 - K2 ** 2) / (2.0 * K1 * K2)
    m_hi = (np.minimum(hi, K1 + K2) ** 2 - K1 ** 2 - K2 ** 2) / (2.0 * K1 * K2)
    m_lo = np.clip(m_lo, -1.0, 1.0)
    m_hi = np.clip(np.maximum(m_hi, m_lo), -1.0, 1.0)
    wt = Wq * (K1 * K2) ** 2
    den = float(np.sum(wt * (m_hi - m_lo)))
    if den <= 0.0:
        return 0.0
    num = float(np.sum(wt * (legendre_integral(ell, m_hi) - legendre_integral(ell, m_lo))))
    return num / den


def shot_noise_multipoles(P_l: np.ndarray, tris, k0: float, dk: float, nbar: float) -> np.ndarray:
    """Poisson shot-noise model SN_l(b1, b2, b3) of the raw B_l, [nl][ntri].

    B_l sums delta^(l)(k1) delta(k2) delta(k3) over closed triangles, the
    Legendre weight on the first leg. For Poisson points the sum over
    particle triples (i, j, k) holds, beside the distinct triples, the terms
    with j = k, i = k, i = j (counted with i = j = k) and i = j = k; the
    distinct part is the sum minus the three pair terms plus twice the triple
    term. Averaged over a bin: j = k gives P_l(b1)/nbar; i = k gives the
    power at k2 with the Legendre weight of k1, which, averaging k1 over its
    ring of directions around k2 at the triangle's opening angle,
    L_l(k1_hat . x_hat) -> L_l(k1_hat . k2_hat) L_l(k2_hat . x_hat), is
    W_l(b1, b2 | b3) P_l(b2)/nbar; i = j likewise with b3; i = j = k gives
    (2l + 1) <L_l(k1_hat . x_hat)>/nbar^2, which is 1/nbar^2 for l = 0 and is
    dropped for l > 0 (zero for l = 2 over the cubic-symmetric set of closed
    triangles, a lattice-anisotropy term for l = 4). So
      SN_0 = (P_0(b1) + P_0(b2) + P_0(b3)) / nbar - 2 / nbar^2   (= shot_noise_binned)
      SN_l = (P_l(b1) + W_l(b1,b2|b3) P_l(b2) + W_l(b1,b3|b2) P_l(b3)) / nbar.
    P_l: raw shell power multipoles [nl][nb] (power_multipoles; P_0 = Pbar).
    The model's accuracy against the exact coincidence terms
    (shot_noise_coincidence) is pinned in the tests; it is a reading, not in
    the paper."""
    P_l = np.asarray(P_l, dtype=np.float64)
    nl = P_l.shape[0]
    out = np.zeros((nl, len(tris)))
    for i, (b1, b2, b3) in enumerate(tris):
        c1, c2, c3 = k0 + b1 * dk, k0 + b2 * dk, k0 + b3 * dk
        for li in range(nl):
            ell = 2 * li
            if ell == 0:
                out[li, i] = (P_l[0][b1] + P_l[0][b2] + P_l[0][b3]) / nbar - 2.0 / nbar ** 2
            else:
                w12 = ring_factor(ell, c1, c2, c3, dk)
                w13 = ring_factor(ell, c1, c3, c2, dk)
                out[li, i] = (P_l[li][b1] + w12 * P_l[li][b2] + w13 * P_l[li][b3]) / nbar
    return out


def shot_noise_coincidence(cnt: np.ndarray, lmax: int, observer, k0: float, dk: float, nb: int,
                           tris, box: float, nbar_cell: float) -> np.ndarray:
    """Exact Poisson coincidence terms of the raw B_l for unit-weight particles
    sitting on the nodes (NGP, no compensation, no interlacing): cnt[N][N][N]
    particle counts, delta = cnt / nbar_cell - 1. Returns [4][nl][ntri], the
    sums over particle triples with j = k, i = k, i = j and i = j = k, each in
    the normalisation of B_l (binned_bispectrum with N' = N); the shot-noise
    part of B_l is the first three minus twice the last (inclusion-exclusion).

    With F(k) = sum_i exp(-i k.x_i) and the x_hat-product transforms
    T_t(k) = sum_i x_hat_t(x_i) exp(-i k.x_i), delta^(l)(k) = sum_t c_t(k) T_t(k)
    (legendre_moments gives c_t(k) as the moment of a unit T_t), and:
      j = k:      sum_closed delta^(l)(k1) conj F(k1)
      i = k:      sum_t sum_closed c_t(k1) conj T_t(k2) F(k2)
      i = j:      sum_t sum_closed c_t(k1) conj T_t(k3) F(k3)
      i = j = k:  sum_t sum_closed c_t(k1) * T_t(0)
    (all divided by nbar_cell^3, as delta(k) = F(k) / nbar_cell for k != 0)."""
    n = cnt.shape[0]
    plane = observer is None
    cnt = np.asarray(cnt, dtype=np.float64)
    tens = [()]
    xh = None
    if not plane:
        xh = node_unit_vectors(n, 0.0, observer)
        for m in (2, 4):
            if lmax >= m:
                tens += los_tensor_indices(m)
    T = {t: sfft.rfftn(los_weighted_field(cnt, t, xh) if t else cnt, workers=WORKERS) for t in tens}
    F = T[()]
    Dl = legendre_moments(T, n, lmax, plane)
    coef = {}
    for t in tens:
        unit = {s2: np.zeros_like(F) for s2 in tens}
        unit[t] = np.ones_like(F)
        coef[t] = legendre_moments(unit, n, lmax, plane)
    tau = {t: float(np.real(T[t][0, 0, 0])) for t in tens}
    bins = bin_of_n2(n2_grid_half(n), k0, dk, nb)

    def inv(h):
        return sfft.irfftn(h, s=(n, n, n), workers=WORKERS) * float(n) ** 3

    ind = [inv((bins == b).astype(np.complex128)) for b in range(nb)]

    def closed(h1, b1, h2, b2, h3, b3):
        # sum over k1 + k2 + k3 = 0 with k_i in shell b_i of h1 h2 h3
        f = [ind[b] if h is None else inv(np.where(bins == b, h, 0)) for h, b in ((h1, b1), (h2, b2), (h3, b3))]
        return float(np.sum(f[0] * f[1] * f[2])) / float(n) ** 3

    nl = lmax // 2 + 1
    out = np.zeros((4, nl, len(tris)))
    V = box ** 3
    counts = [closed(None, a, None, b, None, c) for a, b, c in tris]
    for i, (b1, b2, b3) in enumerate(tris):
        norm = V ** 2 * float(n) ** 3 / (float(n) ** 12 * counts[i] * nbar_cell ** 3)
        for li in range(nl):
            A = closed(Dl[li] * np.conj(F), b1, None, b2, None, b3)
            B = C = D = 0.0
            for t in tens:
                c = coef[t][li]
                g = np.conj(T[t]) * F
                B += closed(c, b1, g, b2, None, b3)
                C += closed(c, b1, None, b2, g, b3)
                D += closed(c, b1, None, b2, None, b3) * tau[t]
            out[:, li, i] = np.array([A, B, C, D]) * norm
    return out


# --------------------------------------------------------------------------
# modal estimator (Sec. 3.5)
# --------------------------------------------------------------------------

def modal_modes(P: int, nmodes: int) -> np.ndarray:
    """Mode table n <-> (p, r, s), p <= r <= s < P, ordered by (p+r+s, s, r)."""
    allm = [(p, r, s) for p in range(P) for r in range(p, P) for s in range(r, P)]
    allm.sort(key=lambda t: (t[0] + t[1] + t[2], t[2], t[1]))
    if nmodes > len(allm):
        raise ValueError("nmodes exceeds the number of separable triples")
    return np.array(allm[:nmodes], dtype=np.int64)


def modal_q(p: int, kn, kmin: float, kmax: float):
    """1-D function q_p(k) = Legendre P_p(t), t = (2k - kmin - kmax) / (kmax - kmin),
    with k, kmin, kmax in units of k_f. Orthonormality of the 3-D modes Q_n is
    imposed afterwards through the Gram matrix gamma (eq. betaCalc)."""
    t = (2.0 * np.asarray(kn, dtype=np.float64) - kmin - kmax) / (kmax - kmin)
    c = np.zeros(p + 1)
    c[p] = 1.0
    return np.polynomial.legendre.legval(t, c)


def in_modal_range(n2, kmin: float, kmax: float):
    a, z = 2.0 * kmin, 2.0 * kmax
    return (4 * np.asarray(n2) >= round(a) ** 2) & (4 * np.asarray(n2) < round(z) ** 2)


def modal_filter(p: int, n2, kmin, kmax, kf, pfid_of_n2):
    """f_p(n) = q_p(k) / sqrt(k P_fid(k)) on kmin <= k < kmax, else 0 (k = k_f |n|).

    The filter inside M_n(x) of eq. (betaEst); P_fid is a fixed fiducial table
    (indexed by |n|^2) standing for P-hat in the weight w."""
    n2 = np.asarray(n2)
    kn = np.sqrt(n2.astype(np.float64))
    ok = in_modal_range(n2, kmin, kmax)
    out = np.zeros(n2.shape)
    k = kf * kn[ok]
    out[ok] = modal_q(p, kn[ok], kmin, kmax) / np.sqrt(k * pfid_of_n2[n2[ok]])
    return out


def modal_fields(spec: np.ndarray, n: int, nr: int, P: int, kmin, kmax, kf, pfid_of_n2):
    """M_p(x) = N^-3 x unnormalised inverse DFT_{N'}[f_p delta] for p < P (eq. betaEst)."""
    sp = _crop_spec(spec, n, nr)
    n2 = n2_grid_half(nr)
    return np.stack([sfft.irfftn(sp * modal_filter(p, n2, kmin, kmax, kf, pfid_of_n2),
                                 s=(nr, nr, nr), workers=WORKERS).ravel() * float(nr) ** 3 / float(n) ** 3
                     for p in range(P)])


def modal_numerators(spec_l: Sequence[np.ndarray], n: int, nr: int, modes: np.ndarray,
                     P: int, kmin, kmax, kf, pfid_of_n2):
    """b^l_m = <<B_l | Q_m>> through the M^(l) fields (eqs. Bisp_ell, Bisp_ell2 and
    the beta^l estimator of Sec. 3.5), <XYZ> = N'^-3 sum_x X Y Z:

      b^0 = <M0_p M0_r M0_s>
      b^2 = <M2_p M0_r M0_s> + <M0_p M2_r M0_s> + <M0_p M0_r M2_s>
      b^4 = the three (4,0,0) placements + the three (0,2,2) placements.

    Each sum over placements is already symmetric in (p, r, s), so the average
    over the six index permutations leaves it unchanged.
    """
    M = [modal_fields(s, n, nr, P, kmin, kmax, kf, pfid_of_n2) for s in spec_l]
    K = float(nr) ** 3
    out = np.zeros((len(spec_l), len(modes)))

    def avg(a, b, c):
        return float(np.dot(a * b, c)) / K

    for i, (p, r, s) in enumerate(modes):
        out[0, i] = avg(M[0][p], M[0][r], M[0][s])
        if len(M) > 1:
            out[1, i] = (avg(M[1][p], M[0][r], M[0][s]) + avg(M[0][p], M[1][r], M[0][s])
                         + avg(M[0][p], M[0][r], M[1][s]))
        if len(M) > 2:
            out[2, i] = (avg(M[2][p], M[0][r], M[0][s]) + avg(M[0][p], M[2][r], M[0][s])
                         + avg(M[0][p], M[0][r], M[2][s]) + avg(M[0][p], M[1][r], M[1][s])
                         + avg(M[1][p], M[0][r], M[1][s]) + avg(M[1][p], M[1][r], M[0][s]))
    return out


def gram_matrix(nr: int, modes: np.ndarray, P: int, kmin, kmax, kf, box: float):
    """gamma_nm = <<Q_n | Q_m>> on the lattice (eqs. betaCalc and innerProduct):

      <<f|g>> = V^-2 sum_{n1+n2+n3=0} f g / (k1 k2 k3)
      gamma_nm = (1 / (6 V^2 N'^3)) sum_{tau in S3} G(n1 m_tau1, n2 m_tau2, n3 m_tau3),
      G(A,B,C) = sum_x U_A U_B U_C, U_ab = inverse DFT of q_a(k) q_b(k) / k.
    """
    n2 = n2_grid_half(nr)
    kn = np.sqrt(n2.astype(np.float64))
    ok = in_modal_range(n2, kmin, kmax)
    q = [np.where(ok, modal_q(p, kn, kmin, kmax), 0.0) for p in range(P)]
    kphys = np.where(ok, kf * kn, 1.0)
    U = {}
    for a in range(P):
        for b in range(a, P):
            U[(a, b)] = sfft.irfftn(q[a] * q[b] / kphys * ok, s=(nr, nr, nr),
                                   workers=WORKERS).ravel() * float(nr) ** 3
    cache: Dict[Tuple, float] = {}

    def key(a, b):
        return (a, b) if a <= b else (b, a)

    def G(x, y, z):
        k = tuple(sorted((x, y, z)))
        if k not in cache:
            cache[k] = float(np.dot(U[k[0]] * U[k[1]], U[k[2]]))
        return cache[k]

    V = box ** 3
    nm = len(modes)
    gam = np.zeros((nm, nm))
    perms = list(itertools.permutations(range(3)))
    for i in range(nm):
        for j in range(i, nm):
            s = 0.0
            for tau in perms:
                s += G(key(modes[i][0], modes[j][tau[0]]), key(modes[i][1], modes[j][tau[1]]),
                       key(modes[i][2], modes[j][tau[2]]))
            gam[i, j] = gam[j, i] = s / (6.0 * V ** 2 * float(nr) ** 3)
    return gam


def modal_solve(gamma: np.ndarray, b: np.ndarray):
    """beta = gamma^-1 b via Cholesky gamma = L L^T: alpha = L^-1 b, beta = L^-T alpha."""
    L = np.linalg.cholesky(gamma)
    import scipy.linalg as sla
    alpha = sla.solve_triangular(L, b.T, lower=True).T
    beta = sla.solve_triangular(L.T, alpha.T, lower=False).T
    return alpha, beta


def modal_pivots(gamma: np.ndarray, tol: float):
    """Order in which the modes are orthonormalised, and which are kept.

    Gram-Schmidt of the Q_n in the inner product gamma (eq. betaCalc), taking
    next the mode whose part orthogonal to the modes already taken is largest
    relative to its own norm: r_j = (gamma_jj - |projection of Q_j on the taken
    span|^2) / gamma_jj. Stops when the largest r_j falls below tol: the modes
    left are numerically dependent on the taken ones within the tetrapyd (the
    near-null directions of a separable polynomial basis there), and their
    coefficients are set to 0. Ties go to the lower mode index. tol <= 0 keeps
    every mode in table order (the plain Cholesky factor of gamma).

    r_j is evaluated from its definition, the Schur complement
    gamma_jj - gamma_jS gamma_SS^-1 gamma_Sj over the taken set S.
    Returns the list of kept mode indices in the order taken."""
    nm = gamma.shape[0]
    if tol <= 0:
        return list(range(nm))
    taken: List[int] = []
    for _ in range(nm):
        best, best_r = -1, -1.0
        for j in range(nm):
            if j in taken:
                continue
            if taken:
                g_sj = gamma[np.ix_(taken, [j])][:, 0]
                proj = float(g_sj @ np.linalg.solve(gamma[np.ix_(taken, taken)], g_sj))
            else:
                proj = 0.0
            r = (gamma[j, j] - proj) / gamma[j, j]
            if r > best_r:
                best, best_r = j, r
        if best_r < tol:
            break
        taken.append(best)
    return taken


def modal_solve_pivoted(gamma: np.ndarray, b: np.ndarray, tol: float):
    """Coefficients on the orthonormalised modes kept by ``modal_pivots``.

    With S the kept modes in the order taken, gamma_SS = L L^T (Cholesky):
    alpha = L^-1 b_S are the coefficients of the projection of w B on the
    orthonormal modes R = L^-1 Q_S (eq. betaCalc and the orthonormal basis of
    Sec. 3.5); beta_S = L^-T alpha and beta = 0 on the dropped modes, so that
    w^-1 sum_n beta_n Q_n is that projection. Returns (alpha [nl][nm] with the
    first |S| entries set in the order taken, beta [nl][nm], S)."""
    import scipy.linalg as sla
    S = modal_pivots(gamma, tol)
    b = np.atleast_2d(b)
    L = np.linalg.cholesky(gamma[np.ix_(S, S)])
    a = sla.solve_triangular(L, b[:, S].T, lower=True).T
    bs = sla.solve_triangular(L.T, a.T, lower=False).T
    alpha = np.zeros_like(b)
    beta = np.zeros_like(b)
    alpha[:, :len(S)] = a
    beta[:, S] = bs
    return alpha, beta, S


def modal_shot_noise(nr: int, modes: np.ndarray, P: int, kmin, kmax, kf, box: float,
                     pfid_of_n2, nbar: float):
    """Poisson shot-noise part of b^0 (l = 0 only), mirroring the binned reading:

      B_SN = (Pf1 + Pf2 + Pf3) / nbar - 2 / nbar^2 with P_fid the total power, so
      b^SN_m = (3/nbar) sym<G^P_p G_r G_s> - (2/nbar^2) <G_p G_r G_s>,
      <XYZ> = V^-2 N'^-3 sum_x X Y Z, G_p = inverse DFT of q_p / sqrt(k P_fid),
      G^P_p = inverse DFT of q_p sqrt(P_fid / k), sym = average over the six
      permutations of (p, r, s), which equals the average over the three
      positions of the P-weighted factor.
    The paper gives no modal shot-noise model; this is a reading.
    """
    n2 = n2_grid_half(nr)
    kn = np.sqrt(n2.astype(np.float64))
    ok = in_modal_range(n2, kmin, kmax)
    kphys = np.where(ok, kf * kn, 1.0)
    pf = np.where(ok, pfid_of_n2[np.minimum(n2, len(pfid_of_n2) - 1)], 1.0)
    g = []
    gp = []
    for p in range(P):
        q = np.where(ok, modal_q(p, kn, kmin, kmax), 0.0)
        g.append(sfft.irfftn(q / np.sqrt(kphys * pf), s=(nr,) * 3, workers=WORKERS).ravel() * float(nr) ** 3)
        gp.append(sfft.irfftn(q * np.sqrt(pf / kphys), s=(nr,) * 3, workers=WORKERS).ravel() * float(nr) ** 3)
    V = box ** 3
    norm = 1.0 / (V ** 2 * float(nr) ** 3)
    out = np.zeros(len(modes))
    for i, (p, r, s) in enumerate(modes):
        t1 = (np.dot(gp[p] * g[r], g[s]) + np.dot(g[p] * gp[r], g[s]) + np.dot(g[p] * g[r], gp[s])) / 3.0
        t2 = np.dot(g[p] * g[r], g[s])
        out[i] = norm * (3.0 / nbar * t1 - 2.0 / nbar ** 2 * t2)
    return out


def batch_covariance(betas: np.ndarray) -> np.ndarray:
    """Sample covariance (1/(M-1)) sum_m (beta_m - mean)(beta_m - mean)^T."""
    x = np.asarray(betas, dtype=np.float64)
    d = x - x.mean(axis=0, keepdims=True)
    return d.T @ d / (x.shape[0] - 1)


# --------------------------------------------------------------------------
# whole estimator
# --------------------------------------------------------------------------

class Geometry:
    """Lattice geometry of one run: grid sizes, box, bins, modal basis, P_fid table."""

    def __init__(self, n, nr, box, lmax, nbins, k0, dk, P=0, nmodes=0, pfid=None):
        self.n, self.nr, self.box, self.lmax = n, nr, box, lmax
        self.nbins, self.k0, self.dk = nbins, k0, dk
        self.kmin = k0 - 0.5 * dk
        self.kmax = k0 + (nbins - 1) * dk + 0.5 * dk
        self.kf = 2.0 * math.pi / box
        self.P, self.nmodes = P, nmodes
        self.modes = modal_modes(P, nmodes) if nmodes else np.zeros((0, 3), np.int64)
        self.pfid = pfid
        self.cmax = int(math.isqrt(n2_max_of(k0, dk, nbins)))
        if 3 * self.cmax >= nr:
            raise ValueError("aliasing: 3 c_max must be < N'")


def estimate(spec_l, geo: Geometry, nbar: Optional[float] = None, counts=None, gamma=None,
             sn_modal=None, modal_tol: float = 0.0, gemm: bool = False):
    """Binned B_l, counts, shell power, shot-noise-subtracted B_0 and modal beta^l.

    modal_tol > 0 orthonormalises with ``modal_solve_pivoted`` (kept modes in
    out["modal_kept"]); 0 uses the plain Cholesky factor of gamma. gemm: the
    triple sums and counts through ``binned_triple_sums_gemm`` and
    ``triangle_counts_gemm`` (same sums, for large grids)."""
    n, nr = geo.n, geo.nr
    tris_all = triangle_list(geo.nbins)
    if counts is None:
        _, counts, resid = (triangle_counts_gemm if gemm else triangle_counts_fft)(nr, geo.k0, geo.dk, geo.nbins)
        assert resid < 1e-3, resid
    keep = [i for i, c in enumerate(counts) if c > 0]
    tris = [tris_all[i] for i in keep]
    cnt = np.asarray(counts)[keep]
    _, T = (binned_triple_sums_gemm if gemm else binned_triple_sums)(spec_l, n, nr, geo.k0, geo.dk, geo.nbins, tris)
    B = binned_bispectrum(T, cnt, n, nr, geo.box)
    Pbar, Nb = shell_power(spec_l[0], n, geo.k0, geo.dk, geo.nbins, geo.box)
    out = {"tris": np.array(tris, np.int64), "counts": cnt, "T": T, "B": B,
           "Pbar": Pbar, "Nb": Nb}
    if nbar is not None:
        out["B0_sub"] = shot_noise_binned(B[0], Pbar, tris, nbar)
    if geo.nmodes:
        b = modal_numerators(spec_l, n, nr, geo.modes, geo.P, geo.kmin, geo.kmax, geo.kf, geo.pfid)
        if gamma is None:
            gamma = gram_matrix(nr, geo.modes, geo.P, geo.kmin, geo.kmax, geo.kf, geo.box)
        out["bnum"] = b
        out["gamma"] = gamma
        if nbar is not None:
            if sn_modal is None:
                sn_modal = modal_shot_noise(nr, geo.modes, geo.P, geo.kmin, geo.kmax, geo.kf,
                                            geo.box, geo.pfid, nbar)
            b = b.copy()
            b[0] = b[0] - sn_modal
            out["bnum_sub0"] = b[0]
        if modal_tol > 0:
            alpha, beta, kept = modal_solve_pivoted(gamma, b, modal_tol)
        else:
            alpha, beta = modal_solve(gamma, b)
            kept = list(range(len(geo.modes)))
        out["alpha"], out["beta"], out["modal_kept"] = alpha, beta, np.array(kept, np.int64)
    return out

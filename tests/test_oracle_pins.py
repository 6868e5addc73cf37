"""Pins of the FP64 oracle against the paper and against mathematics (no GPU).

Each test checks an oracle function against something other than itself:
a direct sum, brute-force enumeration, a closed form, an invariant or a
statistical expectation derived from the paper's definitions.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.fft as sfft

import oracle as O
from synth import catalog as C


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- transforms

def test_forward_dft_matches_direct_sum():
    n = 6
    x = rng(1).standard_normal((n, n, n))
    F = O.forward(x)
    j = np.arange(n)
    for nv in [(0, 0, 0), (1, 0, 0), (1, 2, 3), (-2, 1, 1), (2, -1, 2)]:
        ph = np.exp(-2j * math.pi * (nv[0] * j[:, None, None] + nv[1] * j[None, :, None]
                                     + nv[2] * j[None, None, :]) / n)
        direct = np.sum(x * ph)
        got = O.bispec._lookup(F, n, np.array([nv]))[0]
        assert abs(got - direct) < 1e-12 * n ** 3


def test_dft_modes_matches_library_transform_and_plane_waves():
    """The sampled DFT (separable sums) against scipy's whole transform at every
    mode of a small cube (axes not interchangeable: a transposed contraction
    fails), and on plane waves whose DFT is a pair of spikes of height N^3/2."""
    n = 12
    x = rng(2).standard_normal((n, n, n))
    a = np.arange(-n // 2, n // 2)
    modes = np.stack(np.meshgrid(a, a, a, indexing="ij"), -1).reshape(-1, 3)
    full = np.fft.fftn(x)
    ref = full[modes[:, 0] % n, modes[:, 1] % n, modes[:, 2] % n]
    assert np.max(np.abs(O.dft_modes(x, modes) - ref)) < 1e-11 * n ** 3
    j = np.arange(n)
    k = (3, -1, 5)
    wave = np.cos(2 * math.pi * (k[0] * j[:, None, None] + k[1] * j[None, :, None] + k[2] * j[None, None, :]) / n)
    got = O.dft_modes(wave, [k, (-3, 1, -5), (3, 1, 5), (0, 0, 0)])
    assert np.allclose(got, [n ** 3 / 2, n ** 3 / 2, 0, 0], atol=1e-9)


def test_shell_field_is_unnormalised_inverse():
    n = 8
    spec = np.zeros((n, n, n // 2 + 1), complex)
    spec[1, 0, 0] = 2.0
    spec[n - 1, 0, 0] = 2.0  # Hermitian partner
    D = O.shell_field(spec, np.ones(spec.shape, bool), n)
    j = np.arange(n)
    expect = 4.0 * np.cos(2 * math.pi * j / n)
    assert np.allclose(D[:, 3, 5], expect, atol=1e-12)


# ---------------------------------------------------------------- assignment

def test_cic_conserves_mass_and_matches_loop():
    n = 8
    r = rng(2)
    u = [C.quantise_grid_units(r.uniform(0, n, 40), n) for _ in range(3)]
    w = r.uniform(0.5, 2.0, 40)
    for shift in (0.0, 0.5):
        rho = O.assign(*u, n, w, 1, shift)
        assert abs(rho.sum() - w.sum()) < 1e-12
        ref = np.zeros((n, n, n))
        for p in range(40):
            v = [(float(u[a][p]) + shift) % n for a in range(3)]
            i0 = [int(math.floor(t)) for t in v]
            d = [t - i for t, i in zip(v, i0)]
            for o in itertools.product((0, 1), repeat=3):
                wt = w[p]
                for a in range(3):
                    wt *= d[a] if o[a] else 1 - d[a]
                ref[(i0[0] + o[0]) % n, (i0[1] + o[1]) % n, (i0[2] + o[2]) % n] += wt
        assert np.allclose(rho, ref, atol=1e-13)


def test_cic_particle_on_node_is_delta_and_ngp_rounds():
    n = 8
    rho = O.assign([3.0], [7.0], [0.0], n, None, 1, 0.0)
    assert rho[3, 7, 0] == 1.0 and rho.sum() == 1.0
    rho = O.assign([2.5], [2.49], [7.6], n, None, 0, 0.0)
    assert rho[3, 2, 0] == 1.0


def test_compensated_interlaced_point_matches_phase():
    n = 32
    u = np.array([[10.3125], [5.75], [21.0625]])
    spec = []
    for s in (0.0, 0.5):
        F = O.forward(O.assign(*u, n, None, 1, s))
        spec.append(O.compensate(F, n, 1))
    Fi = O.interlace_combine(spec[0], spec[1], n)
    fx, fy, fz = O.bispec.half_freq_vectors(n)
    exact = np.exp(-2j * math.pi * (fx * u[0, 0] + fy * u[1, 0] + fz * u[2, 0]) / n)
    low = (np.abs(fx) <= 3) & (np.abs(fy) <= 3) & (fz <= 3)
    low = np.broadcast_to(low, Fi.shape)
    err_i = np.max(np.abs(Fi - exact)[low])
    err_0 = np.max(np.abs(spec[0] - exact)[low])
    # remaining aliases are the even images, |n/(n +- 2N)|^2 ~ 2e-3 per axis and sign
    assert err_i < 2e-2
    assert err_i < err_0  # interlacing removes the leading alias
    wrong = 0.5 * (spec[0] + np.conj(np.exp(1j * math.pi * (fx + fy + fz) / n)) * spec[1])
    assert np.max(np.abs(wrong - exact)[low]) > 10 * err_i


# ---------------------------------------------------------------- LOS moments

@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_tensor_expansion_matches_direct_legendre(shift):
    n = 8
    d = rng(3).standard_normal((n, n, n))
    obs = np.array([-13.0, -7.0, -20.0])
    spec = O.spectrum_from_field([d], [shift], n, 4, obs, None)
    for nv in [(1, 0, 0), (1, 2, 1), (-2, 1, 3), (3, -3, 2), (0, 1, 1)]:
        for li, ell in enumerate((0, 2, 4)):
            g = O.bispec._lookup(spec[li], n, np.array([nv]))[0]
            ref = O.legendre_moments_direct(d, nv, ell, shift, obs)
            assert abs(g - ref) < 1e-10 * (1 + abs(ref)), (nv, ell, g, ref)


def test_plane_parallel_direct_and_far_observer_limit():
    n = 8
    d = rng(4).standard_normal((n, n, n))
    pp = O.spectrum_from_field([d], [0.0], n, 4, None, None)
    for nv in [(1, 2, 1), (0, 0, 2), (-3, 1, 2)]:
        for li, ell in enumerate((0, 2, 4)):
            g = O.bispec._lookup(pp[li], n, np.array([nv]))[0]
            ref = O.legendre_moments_direct(d, nv, ell, 0.0, None)
            assert abs(g - ref) < 1e-10 * (1 + abs(ref))
    far = O.spectrum_from_field([d], [0.0], n, 4, np.array([3.5, 3.5, -1e8]), None)
    for li in range(3):
        assert np.max(np.abs(far[li] - pp[li])) < 1e-5 * np.max(np.abs(pp[li]))


def test_kaiser_multipole_ratios():
    n, f = 48, 0.6
    r = rng(5)
    n2 = O.n2_grid_half(n)
    ph = np.exp(2j * math.pi * r.uniform(size=n2.shape))
    fx, fy, fz = O.bispec.half_freq_vectors(n)
    kn = np.sqrt(np.maximum(n2, 1))
    mu = fz / kn
    g_real = sfft.irfftn(ph, s=(n,) * 3)  # any Hermitian-consistent field
    g = O.forward(g_real)
    g = g / np.maximum(np.abs(g), 1e-300)  # unit amplitude, random phase
    ds = (1 + f * mu ** 2) * g
    spec = O.spectrum_from_field([sfft.irfftn(ds, s=(n,) * 3)], [0.0], n, 4, None, None)
    shell = (n2 >= 12 ** 2) & (n2 < 20 ** 2)
    # half spectrum: nz > 0 entries stand for themselves and their conjugate partner
    mult = np.broadcast_to(np.where(fz > 0, 2.0, 1.0), n2.shape)[shell]
    def avg(x):
        return float(np.sum(x[shell] * mult) / np.sum(mult))
    p0 = avg(np.real(spec[0] * np.conj(spec[0])))
    expect = [1 + 2 * f / 3 + f ** 2 / 5, 4 * f / 3 + 4 * f ** 2 / 7, 8 * f ** 2 / 35]
    for li in range(3):
        pl = avg(np.real(spec[li] * np.conj(spec[0])))
        assert abs(pl - expect[li]) < 0.01 * expect[0], (li, pl, expect[li])
    assert abs(p0 - expect[0]) < 0.01 * expect[0]


# ---------------------------------------------------------------- power-spectrum multipoles

def test_power_multipoles_kaiser():
    """eq. (PowSpecMultipole) on a Kaiser field (1 + f mu^2) g with |g| = 1 and
    a line of sight along z: the shell averages approach the closed forms
    1 + 2f/3 + f^2/5, 4f/3 + 4f^2/7, 8f^2/35 (times V / N^6)."""
    n, f, box = 48, 0.6, 300.0
    r = rng(15)
    n2 = O.n2_grid_half(n)
    fx, fy, fz = O.bispec.half_freq_vectors(n)
    kn = np.sqrt(np.maximum(n2, 1))
    g = O.forward(sfft.irfftn(np.exp(2j * math.pi * r.uniform(size=n2.shape)), s=(n,) * 3))
    g = g / np.maximum(np.abs(g), 1e-300)
    ds = (1 + f * (fz / kn) ** 2) * g
    spec = O.spectrum_from_field([sfft.irfftn(ds, s=(n,) * 3)], [0.0], n, 4, None, None)
    P, Nb = O.power_multipoles(spec, n, 14.0, 4.0, 2, box)
    expect = [1 + 2 * f / 3 + f ** 2 / 5, 4 * f / 3 + 4 * f ** 2 / 7, 8 * f ** 2 / 35]
    scale = float(n) ** 6 / box ** 3
    for b in range(2):
        assert Nb[b] > 3000
        for li in range(3):
            assert abs(P[li, b] * scale - expect[li]) < 0.015 * expect[0], (b, li, P[li, b] * scale)


def test_power_multipoles_full_lattice_brute():
    """Half-spectrum multiplicities and normalisation against a direct sum over
    the full lattice with explicit Legendre weights (plane-parallel LOS along z):
    delta^(l)(n) = (2l+1) L_l(n_z/|n|) delta(n)."""
    n, box, k0, dk, nb = 16, 100.0, 2.0, 2.0, 3
    d = rng(21).standard_normal((n, n, n))
    spec = O.spectrum_from_field([d], [0.0], n, 4, None, None)
    P, Nb = O.power_multipoles(spec, n, k0, dk, nb, box)
    F = np.fft.fftn(d)
    fr = np.fft.fftfreq(n, 1.0 / n)
    nx, ny, nz = np.meshgrid(fr, fr, fr, indexing="ij")
    n2 = (nx ** 2 + ny ** 2 + nz ** 2).astype(np.int64)
    mu = nz / np.sqrt(np.maximum(n2, 1))
    leg = [np.ones_like(mu), 0.5 * (3 * mu ** 2 - 1), (35 * mu ** 4 - 30 * mu ** 2 + 3) / 8]
    bins = O.bin_of_n2(n2, k0, dk, nb)
    for b in range(nb):
        sel = bins == b
        assert int(sel.sum()) == int(Nb[b])
        for li in range(3):
            dl = (4 * li + 1) * leg[li][sel] * F[sel]
            ref = box ** 3 * float(np.sum(np.real(dl * np.conj(F[sel])))) / (float(n) ** 6 * sel.sum())
            assert abs(P[li, b] - ref) <= 1e-11 * max(abs(ref), abs(P[0, b])), (b, li, P[li, b], ref)


def test_power_multipole_monopole_is_shell_power():
    n, box = 16, 100.0
    d = rng(22).standard_normal((n, n, n))
    spec = O.spectrum_from_field([d], [0.0], n, 2, None, None)
    P, Nb = O.power_multipoles(spec, n, 2.0, 2.0, 3, box)
    P0, Nb0 = O.shell_power(spec[0], n, 2.0, 2.0, 3, box)
    assert np.array_equal(Nb, Nb0)
    assert np.allclose(P[0], P0, rtol=1e-13, atol=0)


# ---------------------------------------------------------------- skew spectra

def test_skew_spectra_sum_rule():
    """S^l_b N_b = V / (N^9 N'^3) sum over all (b2, b3) of the binned triple sums
    T^l(b, b2, b3) = sum_x D^l_b D^0_b2 D^0_b3 (the skew spectrum integrates the
    bispectrum over the other two sides), with N != N' and a varying LOS."""
    n, nr, box, k0, dk, nb = 32, 24, 200.0, 2.0, 2.0, 3
    r = rng(31)
    d = r.standard_normal((n, n, n))
    obs = np.array([-40.0, -30.0, -55.0])
    spec = O.spectrum_from_field([d], [0.0], n, 4, obs, None)
    S, Nb = O.skew_spectra(spec, n, nr, k0, dk, nb, box)
    tris = [(b, b2, b3) for b in range(nb) for b2 in range(nb) for b3 in range(nb)]
    _, T = O.binned_triple_sums(spec, n, nr, k0, dk, nb, tris)
    V = box ** 3
    for li in range(3):
        for b in range(nb):
            rhs = V * T[li, b * nb * nb:(b + 1) * nb * nb].sum() / (float(n) ** 9 * float(nr) ** 3)
            scale = V * np.abs(T[li, b * nb * nb:(b + 1) * nb * nb]).sum() / (float(n) ** 9 * float(nr) ** 3)
            assert abs(S[li, b] * Nb[b] - rhs) <= 1e-10 * scale, (li, b)


@pytest.mark.parametrize("square_range", ["shells", "ball"])
def test_skew_spectra_brute_convolution(square_range):
    """Q(n) = N'^3 sum_q delta^0(q) delta^0(n - q) over q and n - q in the bins'
    union (or in the ball 0 < |q|^2 <= n2max of the band), summed directly over
    the full lattice (plane-parallel LOS)."""
    n, box, dk, nb = 16, 100.0, 2.0, 2
    k0 = 2.0 if square_range == "shells" else 3.0  # the ball: a gap 1 <= |n|^2 < 4 below the first shell
    d = rng(32).standard_normal((n, n, n))
    spec = O.spectrum_from_field([d], [0.0], n, 2, None, None)
    S, Nb = O.skew_spectra(spec, n, n, k0, dk, nb, box, square_range)
    fr = np.fft.fftfreq(n, 1.0 / n).astype(int)
    F0 = np.fft.fftn(d)
    # delta^(2) on the full lattice: (5) L_2(n_z / |n|) delta(n) for a LOS along z
    nx, ny, nz = np.meshgrid(fr, fr, fr, indexing="ij")
    n2 = nx ** 2 + ny ** 2 + nz ** 2
    mu2 = nz ** 2 / np.maximum(n2, 1)
    F2 = 5 * 0.5 * (3 * mu2 - 1) * F0
    bins = O.bin_of_n2(n2, k0, dk, nb)
    # the ball written out: 0 < 4 |n|^2 < (2 (k0 + (nb - 1) dk) + dk)^2 = 144
    inband = (bins >= 0) if square_range == "shells" else ((n2 > 0) & (4 * n2 < 144))
    if square_range == "ball":
        assert (inband & (bins < 0)).any()  # the ball holds modes below the first shell
    band = np.argwhere(inband)
    V = box ** 3
    for b in range(nb):
        acc = [0.0, 0.0]
        for (i, j, k) in np.argwhere(bins == b):
            q = 0.0j
            for (a, bb, cc) in band:
                i2, j2, k2 = (i - a) % n, (j - bb) % n, (k - cc) % n
                if inband[i2, j2, k2]:
                    q += F0[a, bb, cc] * F0[i2, j2, k2]
            Q = float(n) ** 3 * q
            acc[0] += float(np.real(np.conj(Q) * F0[i, j, k]))
            acc[1] += float(np.real(np.conj(Q) * F2[i, j, k]))
        for li in range(2):
            ref = V * acc[li] / (float(n) ** 12 * Nb[b])
            assert abs(S[li, b] - ref) <= 1e-9 * abs(V * acc[0] / (float(n) ** 12 * Nb[b])), (b, li, S[li, b], ref)


def test_skew_spectra_ball_equals_shells_when_the_shells_fill_it():
    """With the first shell reaching down to |n| = 0 the union of the shells is
    the whole ball and both squared fields are the same; with a gap below the
    first shell they differ."""
    n, box, nb = 32, 200.0, 4
    d = rng(33).standard_normal((n, n, n))
    obs = np.array([-40.0, -30.0, -55.0])
    spec = O.spectrum_from_field([d], [0.0], n, 4, obs, None)
    Sa, _ = O.skew_spectra(spec, n, n, 1.0, 2.0, nb, box, "shells")
    Sb, _ = O.skew_spectra(spec, n, n, 1.0, 2.0, nb, box, "ball")
    assert np.allclose(Sa, Sb, rtol=1e-12, atol=1e-12 * np.abs(Sa).max())
    Sc, _ = O.skew_spectra(spec, n, n, 3.0, 2.0, nb, box, "shells")
    Sd, _ = O.skew_spectra(spec, n, n, 3.0, 2.0, nb, box, "ball")
    assert np.linalg.norm(Sc - Sd) > 1e-3 * np.linalg.norm(Sc)


def test_skew_spectra_vanish_without_closed_triangles():
    """A single plane wave at |n| = 5: delta^(l) lives on n = +-5 x-hat, the
    square of the band-limited field only on 0 and +-10 x-hat, so no triangle
    closes and S = 0 on every shell."""
    n, box, k0, dk, nb = 32, 100.0, 2.0, 2.0, 5
    x = np.arange(n)
    d = np.cos(2 * np.pi * 5 * x / n)[:, None, None] * np.ones((1, n, n))
    spec = O.spectrum_from_field([d], [0.0], n, 2, None, None)
    S, _ = O.skew_spectra(spec, n, n, k0, dk, nb, box)
    assert np.max(np.abs(S)) < 1e-12 * (float(n) ** 3)


# ---------------------------------------------------------------- integrated bispectrum

def test_integrated_bispectrum_single_volume_is_power_multipole():
    """With one sub-volume and a line of sight along z, P^(l)_1 is the
    power-spectrum multipole of the whole box (the LOS moment route through
    the x-hat tensors gives (2l+1) L_l(mu) delta(n) in that limit)."""
    n, box, k0, dk, nb = 16, 100.0, 2.0, 2.0, 3
    d = rng(41).standard_normal((n, n, n))
    iB, P, dbar, Nb = O.integrated_bispectrum(d, 1, 4, None, None, box, k0, dk, nb)
    spec = O.spectrum_from_field([d], [0.0], n, 4, None, None)
    Pref, Nb2 = O.power_multipoles(spec, n, k0, dk, nb, box)
    assert np.array_equal(Nb, Nb2)
    assert np.allclose(P[0], Pref, rtol=1e-11, atol=1e-11 * np.abs(Pref).max())
    assert abs(dbar[0] - d.mean()) < 1e-14
    assert np.allclose(iB, Pref * d.mean(), rtol=1e-11, atol=1e-11 * np.abs(Pref).max())


def test_integrated_bispectrum_tiled_volume():
    """A 2 x 2 x 2 tiling of one block, shifted by a different constant in each
    copy: every sub-volume has the block's spectrum away from n = 0, so with a
    line of sight along z iB = P_block * mean(dbar_i)."""
    m, box, k0, dk, nb = 8, 80.0, 1.0, 1.0, 3
    r = rng(42)
    g = r.standard_normal((m, m, m))
    d = np.tile(g, (2, 2, 2))
    offs = r.uniform(-0.5, 0.5, 8)
    for i in range(8):
        ox, oy, oz = (i // 4) * m, ((i // 2) % 2) * m, (i % 2) * m
        d[ox:ox + m, oy:oy + m, oz:oz + m] += offs[i]
    iB, P, dbar, _ = O.integrated_bispectrum(d, 2, 4, None, 1, box, k0, dk, nb)
    _, Pb, _, _ = O.integrated_bispectrum(g, 1, 4, None, 1, box / 2, k0, dk, nb)
    assert np.allclose(dbar, g.mean() + offs, atol=1e-13)
    for i in range(8):
        assert np.allclose(P[i], Pb[0], rtol=1e-11, atol=1e-11 * np.abs(Pb).max())
    assert np.allclose(iB, Pb[0] * dbar.mean(), rtol=1e-11, atol=1e-11 * np.abs(Pb).max())


def test_integrated_bispectrum_brute_subvolume():
    """One sub-volume of a varying-LOS, CIC-compensated run against a direct DFT
    sum with explicit Legendre weights and window."""
    n, s, box, k0, dk, nb = 16, 2, 100.0, 1.0, 1.0, 3
    m = n // s
    d = rng(43).standard_normal((n, n, n))
    obs = np.array([-20.0, -35.0, -10.0])
    iB, P, dbar, Nb = O.integrated_bispectrum(d, s, 4, obs, 1, box, k0, dk, nb)
    i = 5
    ox, oy, oz = (i // 4) * m, ((i // 2) % 2) * m, (i % 2) * m
    blk = d[ox:ox + m, oy:oy + m, oz:oz + m]
    e = np.array([ox, oy, oz]) + 0.5 * (m - 1) - obs
    e = e / np.linalg.norm(e)
    j = np.arange(m)
    fr = np.fft.fftfreq(m, 1.0 / m)
    acc = np.zeros((3, nb))
    cnt = np.zeros(nb)
    for a in fr:
        for b in fr:
            for c in fr:
                q2 = int(a * a + b * b + c * c)
                bb = O.bin_of_n2(np.array([q2]), k0, dk, nb)[0]
                if bb < 0:
                    continue
                ph = np.exp(-2j * np.pi * (a * j[:, None, None] + b * j[None, :, None] + c * j[None, None, :]) / m)
                F = np.sum(blk * ph)
                win = (np.sinc(a / m) * np.sinc(b / m) * np.sinc(c / m)) ** 2
                mu = (a * e[0] + b * e[1] + c * e[2]) / math.sqrt(q2)
                leg = [1.0, 0.5 * (3 * mu * mu - 1), (35 * mu ** 4 - 30 * mu * mu + 3) / 8]
                for li in range(3):
                    acc[li, bb] += (4 * li + 1) * leg[li] * abs(F / win) ** 2
                cnt[bb] += 1
    Vs = (box / s) ** 3
    assert np.array_equal(cnt.astype(np.int64), Nb)
    ref = Vs * acc / (float(m) ** 6 * cnt[None, :])
    assert np.allclose(P[i], ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())
    assert abs(dbar[i] - blk.mean()) < 1e-14


def test_integrated_bispectrum_local_los_brute_subvolume():
    """Line of sight varying inside the sub-volumes: one sub-volume against a
    direct sum of the LOS moment definition over its nodes, with x_hat written
    out here from the nodes' grid coordinates and the observer, and P^(l) from
    Re[delta^(l) conj delta^(0)] summed over the full lattice of each shell."""
    n, s, box, k0, dk, nb = 16, 2, 100.0, 1.0, 1.0, 3
    m = n // s
    d = rng(45).standard_normal((n, n, n))
    obs = np.array([-20.0, -35.0, -10.0])
    iB, P, dbar, Nb = O.integrated_bispectrum_local_los(d, s, 4, obs, 1, box, k0, dk, nb)
    Vs = (box / s) ** 3
    for i in (0, 6):
        org = np.array([(i // 4) * m, ((i // 2) % 2) * m, (i % 2) * m], np.float64)
        blk = d[int(org[0]):int(org[0]) + m, int(org[1]):int(org[1]) + m, int(org[2]):int(org[2]) + m]
        j = np.arange(m)
        gx, gy, gz = np.meshgrid(j, j, j, indexing="ij")
        r = np.stack([gx + org[0] - obs[0], gy + org[1] - obs[1], gz + org[2] - obs[2]])
        xh = r / np.sqrt((r ** 2).sum(axis=0))
        fr = np.fft.fftfreq(m, 1.0 / m)
        acc = np.zeros((3, nb))
        cnt = np.zeros(nb)
        for a in fr:
            for b in fr:
                for c in fr:
                    q2 = int(a * a + b * b + c * c)
                    bb = O.bin_of_n2(np.array([q2]), k0, dk, nb)[0]
                    if bb < 0:
                        continue
                    ph = np.exp(-2j * np.pi * (a * gx + b * gy + c * gz) / m)
                    win = (np.sinc(a / m) * np.sinc(b / m) * np.sinc(c / m)) ** 2
                    mu = (a * xh[0] + b * xh[1] + c * xh[2]) / math.sqrt(q2)
                    leg = [np.ones_like(mu), 0.5 * (3 * mu * mu - 1), (35 * mu ** 4 - 30 * mu * mu + 3) / 8]
                    dl = [(4 * li + 1) * np.sum(blk * leg[li] * ph) / win for li in range(3)]
                    for li in range(3):
                        acc[li, bb] += (dl[li] * np.conj(dl[0])).real
                    cnt[bb] += 1
        assert np.array_equal(cnt.astype(np.int64), Nb)
        ref = Vs * acc / (float(m) ** 6 * cnt[None, :])
        assert np.allclose(P[i], ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max()), i
        assert abs(dbar[i] - blk.mean()) < 1e-14
    assert np.allclose(iB, np.einsum("ilb,i->lb", P, dbar) / s ** 3, rtol=1e-13)


def test_integrated_bispectrum_local_los_far_observer_limit():
    """An observer far away makes x_hat the same over a sub-volume, and the
    local line of sight reduces to the one line of sight per sub-volume."""
    n, s, box, k0, dk, nb = 16, 2, 100.0, 1.0, 1.0, 3
    d = rng(46).standard_normal((n, n, n))
    obs = np.array([-3.0e6, 1.0e6, -2.0e6])
    iB, P, dbar, _ = O.integrated_bispectrum_local_los(d, s, 4, obs, 1, box, k0, dk, nb)
    iB1, P1, dbar1, _ = O.integrated_bispectrum(d, s, 4, obs, 1, box, k0, dk, nb)
    assert np.array_equal(dbar, dbar1)
    for li in range(3):
        assert np.linalg.norm(P[:, li] - P1[:, li]) < 1e-4 * np.linalg.norm(P1[:, 0]), li
    # a near observer makes the two readings differ at l > 0 only
    iB2, P2, _, _ = O.integrated_bispectrum_local_los(d, s, 4, np.array([-4.0, 3.0, -5.0]), 1, box, k0, dk, nb)
    iB3, P3, _, _ = O.integrated_bispectrum(d, s, 4, np.array([-4.0, 3.0, -5.0]), 1, box, k0, dk, nb)
    assert np.allclose(P2[:, 0], P3[:, 0], rtol=1e-12)
    assert np.linalg.norm(P2[:, 1] - P3[:, 1]) > 1e-2 * np.linalg.norm(P3[:, 1])


# ---------------------------------------------------------------- shells

def test_bins_integer_edges_and_isotropy():
    k0, dk, nb = 3.0, 3.0, 6
    lo, hi = O.bin_edges4(k0, dk, nb)
    assert list(lo) == [(2 * (k0 + b * dk) - dk) ** 2 for b in range(nb)]
    r = np.arange(-20, 21)
    nx, ny, nz = np.meshgrid(r, r, r, indexing="ij")
    n2 = nx ** 2 + ny ** 2 + nz ** 2
    b = O.bin_of_n2(n2, k0, dk, nb)
    for i in range(nb):
        sel = b == i
        k = np.sqrt(n2[sel])
        assert k.min() >= k0 + i * dk - dk / 2 and k.max() < k0 + i * dk + dk / 2
        assert int(((3 * nz ** 2 - n2)[sel]).sum()) == 0  # sum of L_2 over a shell vanishes
    assert b[20, 20, 20] == -1


# ---------------------------------------------------------------- closed triangles

def _random_spec(n, seed):
    return O.forward(rng(seed).standard_normal((n, n, n)))


@pytest.mark.parametrize("n,k0,dk,nb", [(8, 1.0, 1.0, 2), (16, 1.5, 1.0, 4), (16, 2.0, 2.0, 2)])
def test_fft_triple_sum_equals_brute_force_closed_triangles(n, k0, dk, nb):
    spec = [_random_spec(n, 10 + i) for i in range(2)]
    lo, hi = O.bin_edges4(k0, dk, nb)
    tris, T = O.binned_triple_sums(spec, n, n, k0, dk, nb)
    scale = np.abs(T).max() / n ** 3
    for ti, (b1, b2, b3) in enumerate(tris):
        masks = [lambda q, b=b: (4 * q >= lo[b]) & (4 * q < hi[b]) for b in (b1, b2, b3)]
        for li in range(2):
            ref = O.closed_triangle_sum_brute([spec[li], spec[0], spec[0]], n, masks, modular=True)
            got = T[li, ti] / n ** 3
            assert abs(got - ref.real) < 1e-10 * scale, (b1, b2, b3, li, got, ref)
            assert abs(ref.imag) < 1e-10 * scale


@pytest.mark.parametrize("n,k0,dk,nb", [(8, 1.0, 1.0, 2), (16, 2.0, 2.0, 2)])
def test_full_multipole_triple_sums_brute_force(n, k0, dk, nb):
    """T^(l1 l2 l3) against the closed-triangle sum with a different spectrum
    on each side; l2 = l3 = 0 reproduces the B^(l) triple sums."""
    spec = [_random_spec(n, 20 + i) for i in range(3)]
    lo, hi = O.bin_edges4(k0, dk, nb)
    tris, combos, T = O.binned_triple_sums_full(spec, n, n, k0, dk, nb)
    _, T1 = O.binned_triple_sums(spec, n, n, k0, dk, nb)
    scale = np.abs(T).max() / n ** 3
    for li in range(3):
        assert np.allclose(T[combos.index((li, 0, 0))], T1[li], rtol=0, atol=1e-12 * np.abs(T1).max())
    for ti, (b1, b2, b3) in enumerate(tris):
        masks = [lambda q, b=b: (4 * q >= lo[b]) & (4 * q < hi[b]) for b in (b1, b2, b3)]
        for ci, (l1, l2, l3) in enumerate(combos):
            ref = O.closed_triangle_sum_brute([spec[l1], spec[l2], spec[l3]], n, masks, modular=True)
            assert abs(T[ci, ti] / n ** 3 - ref.real) < 1e-10 * scale, (b1, b2, b3, l1, l2, l3)
        if b2 == b3:
            for (l1, l2, l3) in combos:
                assert abs(T[combos.index((l1, l2, l3)), ti] - T[combos.index((l1, l3, l2)), ti]) < 1e-10 * scale * n ** 3


def test_modular_equals_exact_closure_without_alias_and_differs_with():
    n = 16
    spec = _random_spec(n, 21)
    m = [lambda q: (q >= 4) & (q < 25)] * 3  # |n| in [2, 5): 3c = 12 < 16
    a = O.closed_triangle_sum_brute([spec] * 3, n, m, modular=True)
    b = O.closed_triangle_sum_brute([spec] * 3, n, m, modular=False)
    assert abs(a - b) < 1e-9 * abs(a)
    m = [lambda q: (q >= 16) & (q < 49)] * 3  # |n| in [4, 7): 3c = 18 > 16 wraps
    a = O.closed_triangle_sum_brute([spec] * 3, n, m, modular=True)
    b = O.closed_triangle_sum_brute([spec] * 3, n, m, modular=False)
    assert abs(a - b) > 1e-6 * abs(a)


@pytest.mark.parametrize("k0,dk,nb,n", [(2.0, 2.0, 4, 32), (3.0, 3.0, 3, 32), (1.0, 1.0, 5, 16)])
def test_counts_fft_match_enumeration(k0, dk, nb, n):
    tris, cnt, resid = O.triangle_counts_fft(n, k0, dk, nb)
    assert resid < 1e-6
    brute = O.triangle_counts_brute(k0, dk, nb, tris)
    assert np.array_equal(cnt, brute)
    # independence of N' once 3 c < N'
    _, cnt2, _ = O.triangle_counts_fft(n + 8, k0, dk, nb)
    assert np.array_equal(cnt, cnt2)


def test_counts_golden_c1():
    """C1 bins (dk = 2, 10 bins): FFT counts against the enumerated golden table."""
    path = __file__.replace("test_oracle_pins.py", "golden/counts_k2_d2_nb10.txt")
    gold = np.loadtxt(path, dtype=np.int64, comments="#")
    tris, cnt, resid = O.triangle_counts_fft(64, 2.0, 2.0, 10)
    assert resid < 1e-6
    assert np.array_equal(np.array(tris), gold[:, :3])
    assert np.array_equal(cnt, gold[:, 3])


def test_counts_symmetry_and_continuum():
    k0, dk, nb = 4.0, 4.0, 4
    tris, cnt, _ = O.triangle_counts_fft(64, k0, dk, nb)
    # permutation symmetry: count a triangle in another side order by enumeration
    lo, hi = O.bin_edges4(k0, dk, nb)
    t = (3, 2, 1)
    i = tris.index(t)
    perm = O.triangle_counts_brute(k0, dk, nb, [(1, 3, 2)])  # not canonical order
    assert perm[0] == cnt[i]
    # continuum: N_tri ~ 8 pi^2 c1 c2 c3 dk^3 for a non-degenerate triangle
    c = [k0 + b * dk for b in t]
    approx = 8 * math.pi ** 2 * c[0] * c[1] * c[2] * dk ** 3
    assert abs(cnt[i] / approx - 1) < 0.1


def test_crop_identity():
    n, nr = 32, 20
    spec = [_random_spec(n, 30)]
    _, T1 = O.binned_triple_sums(spec, n, n, 2.0, 2.0, 3)
    _, T2 = O.binned_triple_sums(spec, n, nr, 2.0, 2.0, 3)
    assert np.allclose(T1 / n ** 3, T2 / nr ** 3, rtol=1e-10, atol=1e-9 * np.abs(T1 / n ** 3).max())


# ---------------------------------------------------------------- statistics

def _gaussian_lattice_field(n, seed, power):
    """Gaussian field with E|g(n)|^2 = N^3 p(n)."""
    w = rng(seed).standard_normal((n, n, n))
    W = O.forward(w)
    return sfft.irfftn(W * np.sqrt(power), s=(n,) * 3)


def _stat_setup():
    n, k0, dk, nb = 24, 2.0, 2.0, 3
    n2 = O.n2_grid_half(n)
    k = np.sqrt(np.maximum(n2, 1))
    p = 1.0 / (1.0 + (k / 4.0) ** 2)
    p[0, 0, 0] = 0.0
    return n, k0, dk, nb, p


def _zscores(samples, expect):
    s = np.asarray(samples)
    m = s.mean(0)
    se = s.std(0, ddof=1) / math.sqrt(s.shape[0])
    return (m - expect) / se


def test_gaussian_field_bispectrum_zero_mean():
    n, k0, dk, nb, p = _stat_setup()
    tris, cnt, _ = O.triangle_counts_fft(n, k0, dk, nb)
    keep = [i for i in range(len(tris)) if cnt[i] > 0]
    tk = [tris[i] for i in keep]
    R = 64
    out = []
    for r in range(R):
        g = _gaussian_lattice_field(n, 100 + r, p)
        spec = O.spectrum_from_field([g], [0.0], n, 4, None, None)
        _, T = O.binned_triple_sums(spec, n, n, k0, dk, nb, tk)
        out.append(O.binned_bispectrum(T, cnt[keep], n, n, 1.0).ravel())
    z = _zscores(out, 0.0)
    nu = z.size
    assert np.max(np.abs(z)) < 5
    assert abs(np.sum(z ** 2) / nu - 1) < 5 * math.sqrt(2 / nu)


def test_quadratic_field_matches_tree_level_closed_form():
    """delta = g + b2 (g^2 - <g^2>):
    E[sum_closed delta^l delta delta] = 2 b2 N^3 sum_closed (2l+1) L_l(mu1) [p1p2 + p2p3 + p3p1]
    (plane parallel, no RSD) to O(b2^3)."""
    n, k0, dk, nb, p = _stat_setup()
    b2 = 0.1 / math.sqrt(float(p.sum() * 2) / n ** 3)
    tris, cnt, _ = O.triangle_counts_fft(n, k0, dk, nb)
    keep = [i for i in range(len(tris)) if cnt[i] > 0]
    tk = [tris[i] for i in keep]
    # expected T / N^3 via weighted unit fields
    n2 = O.n2_grid_half(n)
    bins = O.bin_of_n2(n2, k0, dk, nb)
    fx, fy, fz = O.bispec.half_freq_vectors(n)
    mu = fz / np.sqrt(np.maximum(n2, 1))
    def fld(a):
        return O.shell_field(np.ones(n2.shape, complex) * a, np.ones(n2.shape, bool), n).ravel()
    expect = np.zeros((3, len(tk)))
    for li, ell in enumerate((0, 2, 4)):
        Lw = (2 * ell + 1) * O.bispec.legendre_poly(ell, mu)
        for ti, (b1, b2_, b3) in enumerate(tk):
            m1, m2, m3 = (bins == b1), (bins == b2_), (bins == b3)
            I1p, I1 = fld(Lw * p * m1), fld(Lw * m1)
            I2p, I2 = fld(p * m2), fld(m2 * 1.0)
            I3p, I3 = fld(p * m3), fld(m3 * 1.0)
            s = (np.dot(I1p * I2p, I3) + np.dot(I1 * I2p, I3p) + np.dot(I1p * I2, I3p)) / n ** 3
            expect[li, ti] = 2 * b2 * n ** 3 * s
    R = 64
    out = []
    for r in range(R):
        g = _gaussian_lattice_field(n, 500 + r, p)
        d = g + b2 * (g * g - np.mean(g * g))
        spec = O.spectrum_from_field([d], [0.0], n, 4, None, None)
        _, T = O.binned_triple_sums(spec, n, n, k0, dk, nb, tk)
        out.append((T / n ** 3).ravel())
    z = _zscores(out, expect.ravel())
    assert np.max(np.abs(z)) < 5, np.max(np.abs(z))
    # sensitivity: the expectation is detected far above the noise
    zz = _zscores(out, 0.0)
    assert np.max(np.abs(zz)) > 8
    # a factor-2 error in the closed form would be caught
    assert np.max(np.abs(_zscores(out, 2 * expect.ravel()))) > 5
    assert np.max(np.abs(_zscores(out, 0.5 * expect.ravel()))) > 5


def test_poisson_shot_noise_formula_unbiased():
    """Uniform Poisson counts per node-centred cell, NGP, no compensation:
    E[Pbar] = 1/nbar and E[B0] = 1/nbar^2, so E[B0_sub] = 0."""
    n, box, lam = 16, 100.0, 0.5
    k0, dk, nb = 2.0, 2.0, 2
    tris, cnt, _ = O.triangle_counts_fft(n, k0, dk, nb)
    keep = [i for i in range(len(tris)) if cnt[i] > 0]
    tk = [tris[i] for i in keep]
    nbar = lam * n ** 3 / box ** 3
    subs, ps, b0 = [], [], []
    for r in range(80):
        u = C.poisson_node_catalogue(n, lam, 900 + r)
        spec, wsum = O.spectrum_from_catalogue(*u, n, 0, None, window=0, compensate_window=False)
        _, T = O.binned_triple_sums(spec, n, n, k0, dk, nb, tk)
        B = O.binned_bispectrum(T, cnt[keep], n, n, box)
        P, _ = O.shell_power(spec[0], n, k0, dk, nb, box)
        nb_real = wsum / box ** 3
        subs.append(O.shot_noise_binned(B[0], P, tk, nb_real))
        ps.append(P * nbar)
        b0.append(B[0] * nbar ** 2)
    assert np.max(np.abs(_zscores(ps, 1.0))) < 5
    assert np.max(np.abs(_zscores(b0, 1.0))) < 5
    assert np.max(np.abs(_zscores(subs, 0.0))) < 5


def test_modal_shot_noise_unbiased_for_poisson_points():
    """Unclustered Poisson points (NGP, no compensation) with the fiducial power
    equal to their total power 1/nbar: the modal shot-noise term of b^0 is its
    whole expectation, E[b^0_m - b^SN_m] = 0 (then G^P = G / nbar and the term is
    <GGG> / nbar^2, the Poisson three-point function projected on the modes).
    The average over the three positions of the P-weighted factor cannot show
    here (constant P_fid); the coefficients and the normalisation do: doubling
    the term is rejected."""
    n, box, lam = 16, 200.0, 0.5
    k0, dk, nb, P = 1.5, 1.0, 4, 3
    kmin, kmax = k0 - dk / 2, k0 + (nb - 1) * dk + dk / 2
    kf = 2 * math.pi / box
    modes = O.modal_modes(P, 10)
    nbar = lam * n ** 3 / box ** 3
    pfid = np.full(3 * n * n + 1, 1.0 / nbar)
    sn = O.modal_shot_noise(n, modes, P, kmin, kmax, kf, box, pfid, nbar)
    b0 = []
    for r in range(120):
        u = C.poisson_node_catalogue(n, lam, 1900 + r)
        spec, wsum = O.spectrum_from_catalogue(*u, n, 0, None, window=0, compensate_window=False)
        b0.append(O.modal_numerators(spec, n, n, modes, P, kmin, kmax, kf, pfid)[0])
    assert np.max(np.abs(_zscores(b0, sn))) < 5
    assert np.max(np.abs(_zscores(b0, 2 * sn))) > 5


def test_modal_shot_noise_unbiased_for_poisson_sampled_gaussian_field():
    """A weak Gaussian field (power P_g steep in k, rms 0.1) Poisson-sampled at the
    nodes has the three-point function [P_g(k1) + P_g(k2) + P_g(k3)] / nbar +
    1 / nbar^2 and no other; with P_fid = P_g + 1/nbar the modal shot-noise term
    is again the whole expectation of b^0. P_fid varies with k, so the average
    over the three positions of its P-weighted factor matters: a one-position
    version of that factor is rejected on the asymmetric modes."""
    n, box, lam = 16, 200.0, 2.0
    k0, dk, nb, P = 1.5, 1.0, 4, 3
    kmin, kmax = k0 - dk / 2, k0 + (nb - 1) * dk + dk / 2
    kf = 2 * math.pi / box
    V = box ** 3
    modes = O.modal_modes(P, 10)
    nbar = lam * n ** 3 / V
    n2 = O.n2_grid_half(n)
    k = kf * np.sqrt(np.maximum(n2, 1))
    mult = np.broadcast_to(np.where(np.arange(n // 2 + 1) == 0, 1.0, 2.0), n2.shape)
    shape = np.where(n2 > 0, (k / kf) ** -2.5, 0.0)
    amp = 0.01 / (float((shape * mult).sum()) / V)  # rms 0.1
    Pg = amp * shape
    kk = kf * np.sqrt(np.arange(3 * n * n + 1))
    pfid = amp * (np.maximum(kk, kf) / kf) ** -2.5 + 1.0 / nbar
    sn = O.modal_shot_noise(n, modes, P, kmin, kmax, kf, box, pfid, nbar)
    rng = np.random.Generator(np.random.PCG64(2024))
    b0 = []
    for _ in range(1000):
        g = sfft.irfftn(sfft.rfftn(rng.standard_normal((n, n, n))) * np.sqrt(n ** 3 * Pg / V), s=(n,) * 3)
        rho = rng.poisson(lam * np.clip(1 + g, 0, None)).astype(np.float64)
        spec = O.spectrum_from_field([O.density_contrast(rho, rho.sum())], [0.0], n, 0, None, None)
        b0.append(O.modal_numerators(spec, n, n, modes, P, kmin, kmax, kf, pfid)[0])
    assert np.max(np.abs(_zscores(b0, sn))) < 5
    assert np.max(np.abs(_zscores(b0, 2 * sn))) > 5
    # negative control: the P-weighted factor at the first position only
    kn = np.sqrt(n2.astype(np.float64))
    ok = O.bispec.in_modal_range(n2, kmin, kmax)
    kph = np.where(ok, kf * kn, 1.0)
    pf = np.where(ok, pfid[np.minimum(n2, len(pfid) - 1)], 1.0)
    G, GP = [], []
    for p in range(P):
        q = np.where(ok, O.bispec.modal_q(p, kn, kmin, kmax), 0.0)
        G.append(sfft.irfftn(q / np.sqrt(kph * pf), s=(n,) * 3).ravel() * float(n) ** 3)
        GP.append(sfft.irfftn(q * np.sqrt(pf / kph), s=(n,) * 3).ravel() * float(n) ** 3)
    norm = 1.0 / (V ** 2 * float(n) ** 3)
    one = np.array([norm * (3.0 / nbar * np.dot(GP[p] * G[r], G[s]) - 2.0 / nbar ** 2 * np.dot(G[p] * G[r], G[s]))
                    for (p, r, s) in modes])
    assert np.max(np.abs(_zscores(b0, one))) > 5


# ---------------------------------------------------------------- modal

def _modal_geo(n=16):
    k0, dk, nb = 1.5, 1.0, 4  # modal range [1, 5)
    P, nm = 3, 10
    box = 200.0
    kf = 2 * math.pi / box
    n2max = 3 * n * n
    kk = kf * np.sqrt(np.arange(n2max + 1))
    pfid = 1000.0 / (1 + (kk / 0.1) ** 2) + 50.0
    return dict(n=n, k0=k0, dk=dk, nb=nb, P=P, nm=nm, box=box, kf=kf, pfid=pfid,
                kmin=k0 - dk / 2, kmax=k0 + (nb - 1) * dk + dk / 2)


def test_mode_table_order():
    m = O.modal_modes(3, 10)
    assert [tuple(x) for x in m] == [(0, 0, 0), (0, 0, 1), (0, 1, 1), (0, 0, 2), (1, 1, 1),
                                     (0, 1, 2), (1, 1, 2), (0, 2, 2), (1, 2, 2), (2, 2, 2)]
    assert len(O.modal_modes(8, 100)) == 100


def test_modal_numerators_match_brute_force():
    g = _modal_geo()
    n = g["n"]
    spec = O.spectrum_from_field([rng(40).standard_normal((n, n, n))], [0.0], n, 2, None, None)
    modes = O.modal_modes(g["P"], g["nm"])
    b = O.modal_numerators(spec, n, n, modes, g["P"], g["kmin"], g["kmax"], g["kf"], g["pfid"])
    n2 = O.n2_grid_half(n)
    filt = [O.modal_filter(p, n2, g["kmin"], g["kmax"], g["kf"], g["pfid"]) for p in range(g["P"])]
    fs = {(li, p): spec[li] * filt[p] for li in range(2) for p in range(g["P"])}
    rng_m = [lambda q: O.bispec.in_modal_range(q, g["kmin"], g["kmax"])] * 3
    for i, (p, r, s) in enumerate(modes):
        ref0 = O.closed_triangle_sum_brute([fs[0, p], fs[0, r], fs[0, s]], n, rng_m).real / n ** 9
        assert abs(b[0, i] - ref0) < 1e-9 * (1e-30 + abs(ref0)) + 1e-12 * np.abs(b[0]).max()
        ref2 = sum(O.closed_triangle_sum_brute([fs[a, p], fs[bb, r], fs[c, s]], n, rng_m).real
                   for a, bb, c in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]) / n ** 9
        assert abs(b[1, i] - ref2) < 1e-9 * abs(ref2) + 1e-12 * np.abs(b[1]).max()


def test_gram_matches_enumeration_and_continuum():
    g = _modal_geo(16)
    modes = O.modal_modes(g["P"], g["nm"])
    gam = O.gram_matrix(16, modes, g["P"], g["kmin"], g["kmax"], g["kf"], g["box"])
    # brute force: V^-2 sum over closed triangles of Q_n Q_m / (k1 k2 k3)
    cm = 4
    r = np.arange(-cm, cm + 1)
    nx, ny, nz = np.meshgrid(r, r, r, indexing="ij")
    v = np.stack([nx.ravel(), ny.ravel(), nz.ravel()], 1)
    n2 = (v ** 2).sum(1)
    v = v[O.bispec.in_modal_range(n2, g["kmin"], g["kmax"])]
    kn = np.sqrt((v ** 2).sum(1))
    n3 = -(v[:, None, :] + v[None, :, :])
    k3 = np.sqrt((n3 ** 2).sum(-1))
    ok = O.bispec.in_modal_range((n3 ** 2).sum(-1), g["kmin"], g["kmax"])
    k1 = np.broadcast_to(kn[:, None], k3.shape)[ok]
    k2 = np.broadcast_to(kn[None, :], k3.shape)[ok]
    k3 = k3[ok]
    q = lambda p, k: O.modal_q(p, k, g["kmin"], g["kmax"])
    def Q(m):
        return sum(q(x, k1) * q(y, k2) * q(z, k3) for x, y, z in itertools.permutations(tuple(m))) / 6.0
    Qs = [Q(m) for m in modes]
    kf = g["kf"]
    V = g["box"] ** 3
    brute = np.array([[np.sum(Qs[i] * Qs[j] / (kf ** 3 * k1 * k2 * k3)) for j in range(len(modes))]
                      for i in range(len(modes))]) / V ** 2
    assert np.allclose(gam, brute, rtol=1e-9, atol=1e-12 * np.abs(brute).max())
    # positive definite, so the Cholesky orthonormalisation exists
    assert np.all(np.linalg.eigvalsh(gam) > 0)


def test_gram_continuum_reduction():
    """Wide shells: the lattice gamma approaches (1/(8 pi^4)) int_V dk1 dk2 dk3 Q_n Q_m."""
    n, kmin, kmax = 48, 6.0, 14.0
    box = 2 * math.pi  # k_f = 1
    modes = O.modal_modes(2, 4)
    gam = O.gram_matrix(n, modes, 2, kmin, kmax, 1.0, box)
    # continuum integral on a fine midpoint grid over the tetrapyd
    m = 120
    ks = kmin + (np.arange(m) + 0.5) * (kmax - kmin) / m
    K1, K2, K3 = np.meshgrid(ks, ks, ks, indexing="ij")
    tet = (2 * np.maximum(np.maximum(K1, K2), K3) <= K1 + K2 + K3)
    q = lambda p, k: O.modal_q(p, k, kmin, kmax)
    def Q(mm):
        return sum(q(a, K1) * q(b, K2) * q(c, K3) for a, b, c in itertools.permutations(mm)) / 6.0
    dv = ((kmax - kmin) / m) ** 3
    cont = np.array([[np.sum((Q(a) * Q(b))[tet]) * dv / (8 * math.pi ** 4) for b in modes] for a in modes])
    V = box ** 3
    # the lattice gamma carries V^-2 and sums over modes (density V/(2pi)^3 per k-volume)
    assert np.allclose(gam, cont, rtol=0.06, atol=0.02 * np.abs(cont).max())


def test_modal_template_recovery():
    g = _modal_geo(16)
    modes = O.modal_modes(g["P"], g["nm"])
    gam = O.gram_matrix(16, modes, g["P"], g["kmin"], g["kmax"], g["kf"], g["box"])
    bt = rng(41).standard_normal((3, len(modes)))
    b = bt @ gam  # numerators of the separable template w^-1 sum beta_n Q_n
    alpha, beta = O.modal_solve(gam, b)
    assert np.allclose(beta, bt, rtol=1e-8, atol=1e-8)
    L = np.linalg.cholesky(gam)
    assert np.allclose(L @ alpha.T, b.T, rtol=1e-10, atol=1e-12 * np.abs(b).max())


def test_batch_covariance_definition():
    x = rng(43).standard_normal((50, 4))
    c = O.batch_covariance(x)
    d = x - x.mean(0)
    ref = sum(np.outer(d[i], d[i]) for i in range(50)) / 49
    assert np.allclose(c, ref)


# ---------------------------------------------------------------- LOS geometry, written out by hand

def test_node_unit_vectors_hand_values():
    """x-hat at nodes of the plain grid (shift 0) and of the interlaced grid
    (shift 1/2), off-axis observer: node j of the grid built from u + s stands
    for the point r = j - s, and x-hat = (r - o) / |r - o| (Sec. 2, the line of
    sight to each galaxy). Values worked by hand."""
    n = 8
    o = np.array([-5.5, 3.25, -9.0])
    # (node, shift) -> r - o, worked out by hand
    cases = [((3, 1, 6), 0.0, (8.5, -2.25, 15.0)),
             ((3, 1, 6), 0.5, (8.0, -2.75, 14.5)),
             ((0, 7, 0), 0.5, (5.0, 3.25, 8.5)),
             ((7, 0, 2), 0.0, (12.5, -3.25, 11.0))]
    for shift in (0.0, 0.5):
        xh = O.bispec.node_unit_vectors(n, shift, o)
        for node, s, d in cases:
            if s != shift:
                continue
            d = np.array(d)
            ref = d / math.sqrt(float(d @ d))
            got = np.array([xh[a][node] for a in range(3)])
            assert np.allclose(got, ref, rtol=0, atol=1e-15), (node, shift, got, ref)


@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_point_source_varying_los_closed_form(shift):
    """A single unit contrast at node x0 of a grid built with the given shift:
    the LOS moment field of Sec. 2 reduces to
    delta^(l)(n) = (2l+1) L_l(k-hat . x-hat_p) exp(-2 pi i n . x0 / N),
    x-hat_p the unit vector from the observer to the point x0 - shift that the
    node stands for; L_2, L_4 are the textbook Legendre polynomials. Every
    half-spectrum mode n != 0 is checked."""
    n = 16
    x0 = np.array([3, 11, 6])
    o = np.array([-5.5, 3.25, -9.0])
    d = np.zeros((n, n, n))
    d[tuple(x0)] = 1.0
    spec = O.spectrum_from_field([d], [shift], n, 4, o, None)
    p = x0 - shift - o
    xh = p / math.sqrt(float(p @ p))
    f = np.fft.fftfreq(n, 1.0 / n)
    fz = np.arange(n // 2 + 1, dtype=np.float64)
    nx, ny, nz = np.meshgrid(f, f, fz, indexing="ij")
    kk = np.sqrt(nx ** 2 + ny ** 2 + nz ** 2)
    kk[0, 0, 0] = 1.0
    mu = (nx * xh[0] + ny * xh[1] + nz * xh[2]) / kk
    phase = np.exp(-2j * math.pi * (nx * x0[0] + ny * x0[1] + nz * x0[2]) / n)
    legendre = [np.ones_like(mu), (3 * mu ** 2 - 1) / 2, (35 * mu ** 4 - 30 * mu ** 2 + 3) / 8]
    for li in range(3):
        ref = (4 * li + 1) * legendre[li] * phase
        ref[0, 0, 0] = 0.0
        assert np.max(np.abs(spec[li] - ref)) < 1e-12, (shift, li)


def test_point_source_interlaced_catalogue():
    """One particle through the whole catalogue route (CIC on both grids,
    compensation, interlacing, LOS moments): at low n the result approaches
    (2l+1) L_l(k-hat . x-hat_p) exp(-2 pi i n . u / N) with x-hat_p taken at the
    particle itself. The observer is 200 cells away, so the x-hat of the cloud's
    nodes differ from x-hat_p by under 1e-2; flipping the observer's sign or
    the interlaced node shift moves the result by more than that."""
    n = 32
    u = np.array([[10.3125], [5.75], [21.0625]])
    o = np.array([-120.0, 90.0, -130.0])
    spec, _ = O.spectrum_from_catalogue(*u, n, 4, o, window=1, interlace=1)
    p = u[:, 0] - o
    xh = p / math.sqrt(float(p @ p))
    fx, fy, fz = O.bispec.half_freq_vectors(n)
    kk = np.sqrt(np.maximum(fx ** 2 + fy ** 2 + fz ** 2, 1e-300))
    mu = (fx * xh[0] + fy * xh[1] + fz * xh[2]) / kk
    phase = np.exp(-2j * math.pi * (fx * u[0, 0] + fy * u[1, 0] + fz * u[2, 0]) / n)
    legendre = [np.ones_like(mu), (3 * mu ** 2 - 1) / 2, (35 * mu ** 4 - 30 * mu ** 2 + 3) / 8]
    low = (np.abs(fx) <= 2) & (np.abs(fy) <= 2) & (fz <= 2) & ((fx != 0) | (fy != 0) | (fz != 0))
    low = np.broadcast_to(low, spec[0].shape)
    # the point contributes 1 / nbar_cell = N^3 to the contrast's transform
    for li in range(3):
        ref = (4 * li + 1) * legendre[li] * phase * n ** 3
        err = np.max(np.abs(spec[li] - ref)[low]) / n ** 3
        assert err < 0.05 * (4 * li + 1), (li, err)


# ---------------------------------------------------------------- modal basis, written out by hand

def test_modal_q_explicit_legendre():
    """q_p(k) = P_p(t) with t = (2k - k_min - k_max) / (k_max - k_min): the map
    sends the ends of the modal range to -1 and +1. P_0 .. P_7 are written out
    (textbook coefficients) and evaluated at t = -1, -0.5, 0, 0.3, 1, i.e. at
    k = 2.5, 40, 77.5, 100, 152.5 for the range [2.5, 152.5)."""
    kmin, kmax = 2.5, 152.5
    k = np.array([2.5, 40.0, 77.5, 100.0, 152.5])
    t = np.array([-1.0, -0.5, 0.0, 0.3, 1.0])
    P = [lambda x: np.ones_like(x),
         lambda x: x,
         lambda x: (3 * x ** 2 - 1) / 2,
         lambda x: (5 * x ** 3 - 3 * x) / 2,
         lambda x: (35 * x ** 4 - 30 * x ** 2 + 3) / 8,
         lambda x: (63 * x ** 5 - 70 * x ** 3 + 15 * x) / 8,
         lambda x: (231 * x ** 6 - 315 * x ** 4 + 105 * x ** 2 - 5) / 16,
         lambda x: (429 * x ** 7 - 693 * x ** 5 + 315 * x ** 3 - 35 * x) / 16]
    for p in range(8):
        got = O.modal_q(p, k, kmin, kmax)
        assert np.allclose(got, P[p](t), rtol=0, atol=1e-13), (p, got, P[p](t))
    # endpoint values P_p(+-1) = (+-1)^p
    assert np.allclose([O.modal_q(p, 152.5, kmin, kmax) for p in range(8)], 1.0)
    assert np.allclose([O.modal_q(p, 2.5, kmin, kmax) for p in range(8)], [(-1) ** p for p in range(8)])


def _modal_reconstruction(beta, modes, qfun, k1, k2, k3):
    """sum_n beta_n Q_n(k1, k2, k3), Q_n the symmetrised product q_p q_r q_s."""
    out = np.zeros_like(k1)
    for bn, m in zip(beta, modes):
        Q = sum(qfun(a, k1) * qfun(b, k2) * qfun(c, k3) for a, b, c in itertools.permutations(tuple(m))) / 6.0
        out = out + bn * Q
    return out


def test_modal_basis_invariance(monkeypatch):
    """The reconstruction w^-1 sum_n beta_n Q_n of Sec. 3.5 does not depend on
    the 1-D functions used to build a complete set of modes (the paper notes
    the form of the one-dimensional modes matters little, eq. Qn; the
    decomposition of eq. bispDecomp): with P = 3 and all 10 triples, Legendre
    q_p and monomials (k / k_max)^p span the same space, so b = <<wB|Q>> and
    gamma must transform together and the two reconstructions agree."""
    g = _modal_geo(16)
    n = g["n"]
    modes = O.modal_modes(3, 10)
    spec = O.spectrum_from_field([rng(77).standard_normal((n, n, n))], [0.0], n, 2, None, None)
    args = (3, g["kmin"], g["kmax"], g["kf"])
    b_leg = O.modal_numerators(spec, n, n, modes, *args, g["pfid"])
    gam_leg = O.gram_matrix(n, modes, *args, g["box"])
    _, beta_leg = O.modal_solve(gam_leg, b_leg)
    kmax = g["kmax"]

    def mono(p, kn, kmin_, kmax_):
        return (np.asarray(kn, dtype=np.float64) / kmax) ** p
    monkeypatch.setattr(O.bispec, "modal_q", mono)
    b_mon = O.modal_numerators(spec, n, n, modes, *args, g["pfid"])
    gam_mon = O.gram_matrix(n, modes, *args, g["box"])
    _, beta_mon = O.modal_solve(gam_mon, b_mon)
    monkeypatch.undo()
    assert not np.allclose(beta_leg, beta_mon)  # the coefficients differ ...
    r = rng(78)
    k1 = r.uniform(g["kmin"], g["kmax"], 50)
    k2 = r.uniform(g["kmin"], g["kmax"], 50)
    k3 = r.uniform(g["kmin"], g["kmax"], 50)
    leg = lambda p, k: O.modal_q(p, k, g["kmin"], g["kmax"])
    mon = lambda p, k: (k / kmax) ** p
    for li in range(2):
        R1 = _modal_reconstruction(beta_leg[li], modes, leg, k1, k2, k3)
        R2 = _modal_reconstruction(beta_mon[li], modes, mon, k1, k2, k3)
        # ... the reconstruction does not (the monomial Gram matrix is the worse
        # conditioned of the two, kappa ~ 1e8, which sets the rounding floor)
        assert np.max(np.abs(R1 - R2)) < 1e-7 * np.max(np.abs(R1)), li
    # a set that is not closed downwards (all triples but (0, 0, 1)) spans
    # different spaces in the two bases, and is not invariant
    keep = [i for i in range(10) if i != 1]
    m9 = modes[keep]
    _, bl = O.modal_solve(O.gram_matrix(n, m9, *args, g["box"]), b_leg[:, keep])
    monkeypatch.setattr(O.bispec, "modal_q", mono)
    gm9 = O.gram_matrix(n, m9, *args, g["box"])
    bm9 = O.modal_numerators(spec, n, n, m9, *args, g["pfid"])
    monkeypatch.undo()
    _, bm = O.modal_solve(gm9, bm9)
    R1 = _modal_reconstruction(bl[0], m9, leg, k1, k2, k3)
    R2 = _modal_reconstruction(bm[0], m9, mon, k1, k2, k3)
    assert np.max(np.abs(R1 - R2)) > 1e-4 * np.max(np.abs(R1))


def _modal_stat_setup():
    n, k0, dk, nb, p = _stat_setup()
    kmin, kmax = k0 - dk / 2, k0 + (nb - 1) * dk + dk / 2
    box = 300.0
    kf = 2 * math.pi / box
    kk = kf * np.sqrt(np.arange(3 * n * n + 1))
    pfid = 2000.0 / (1.0 + (kk / (4 * kf)) ** 2) + 100.0
    return n, p, 3, O.modal_modes(3, 10), kmin, kmax, kf, box, pfid


def test_modal_numerators_zero_mean_for_gaussian_fields():
    """Gaussian fields have no three-point function: E[b^l_m] = 0 for every
    mode and multipole (plane-parallel LOS), from 64 realisations."""
    n, p, P, modes, kmin, kmax, kf, box, pfid = _modal_stat_setup()
    out = []
    for r in range(64):
        g = _gaussian_lattice_field(n, 3100 + r, p)
        spec = O.spectrum_from_field([g], [0.0], n, 4, None, None)
        out.append(O.modal_numerators(spec, n, n, modes, P, kmin, kmax, kf, pfid).ravel())
    z = _zscores(out, 0.0)
    nu = z.size
    assert np.max(np.abs(z)) < 5
    assert abs(np.sum(z ** 2) / nu - 1) < 5 * math.sqrt(2 / nu)


def test_modal_numerators_quadratic_field_expectation():
    """delta = g + b2 (g^2 - <g^2>) has, to O(b2), the three-point function
    2 b2 N^3 [p1 p2 + p2 p3 + p3 p1] on closed triangles (E|g(n)|^2 = N^3 p(n)),
    so E[b^0_m] = <<w B_tree | Q_m>>: the modal numerator of Sec. 3.5 written as
    N^-9 sum over closed triangles of f_p(n1) f_r(n2) f_s(n3) E[delta delta delta],
    f_p = q_p / sqrt(k P_fid). Enumerated here over all mode pairs (n1, n2)
    with n3 = -(n1 + n2) in range; a factor of 2 in either direction is
    rejected."""
    n, p, P, modes, kmin, kmax, kf, box, pfid = _modal_stat_setup()
    b2 = 0.1 / math.sqrt(float(p.sum() * 2) / n ** 3)
    cm = int(math.ceil(kmax))
    r_ = np.arange(-cm, cm + 1)
    vx, vy, vz = np.meshgrid(r_, r_, r_, indexing="ij")
    v = np.stack([vx.ravel(), vy.ravel(), vz.ravel()], 1)
    q2 = (v ** 2).sum(1)
    v = v[O.bispec.in_modal_range(q2, kmin, kmax)]
    q2 = (v ** 2).sum(1)

    def pk(vec):  # p(n) looked up on the half spectrum (p is even in n)
        s = np.where(vec[..., 2:3] < 0, -vec, vec)
        return p[s[..., 0] % n, s[..., 1] % n, s[..., 2]]

    def filt(pp, n2):
        kn = np.sqrt(n2.astype(np.float64))
        return O.modal_q(pp, kn, kmin, kmax) / np.sqrt(kf * kn * pfid[n2])
    n3 = -(v[:, None, :] + v[None, :, :])
    q3 = (n3 ** 2).sum(-1)
    ok = O.bispec.in_modal_range(q3, kmin, kmax)
    i1, i2 = np.nonzero(ok)
    p1, p2, p3 = pk(v[i1]), pk(v[i2]), pk(n3[i1, i2])
    w3 = p1 * p2 + p2 * p3 + p3 * p1
    F = [(filt(a, q2[i1]), filt(a, q2[i2]), filt(a, q3[i1, i2])) for a in range(P)]
    expect = np.array([2 * b2 * float(n) ** 3 * np.sum(F[a][0] * F[b][1] * F[c][2] * w3) / float(n) ** 9
                       for a, b, c in modes])
    out = []
    for r in range(64):
        g = _gaussian_lattice_field(n, 3500 + r, p)
        d = g + b2 * (g * g - np.mean(g * g))
        spec = O.spectrum_from_field([d], [0.0], n, 0, None, None)
        out.append(O.modal_numerators(spec, n, n, modes, P, kmin, kmax, kf, pfid)[0])
    z = _zscores(out, expect)
    assert np.max(np.abs(z)) < 5, np.max(np.abs(z))
    assert np.max(np.abs(_zscores(out, 0.0))) > 8
    assert np.max(np.abs(_zscores(out, 2 * expect))) > 5
    assert np.max(np.abs(_zscores(out, 0.5 * expect))) > 5


def test_batch_covariance_closed_forms_and_sampling():
    """Two samples: C = (x1 - x2)(x1 - x2)^T / 2. Adding a constant vector to
    every sample changes nothing. Samples drawn with a known covariance S give
    C within its sampling error, Var(C_ij) = (S_ii S_jj + S_ij^2) / (M - 1)."""
    r = rng(44)
    x = r.standard_normal((2, 5))
    d = x[0] - x[1]
    assert np.allclose(O.batch_covariance(x), np.outer(d, d) / 2, rtol=1e-14, atol=1e-15)
    y = r.standard_normal((30, 5))
    assert np.allclose(O.batch_covariance(y + np.arange(5.0) * 1e3), O.batch_covariance(y), rtol=1e-9, atol=1e-9)
    A = r.standard_normal((5, 5))
    S = A @ A.T + np.eye(5)
    M = 4000
    z = r.standard_normal((M, 5)) @ np.linalg.cholesky(S).T + 3.0
    c = O.batch_covariance(z)
    se = np.sqrt((np.outer(np.diag(S), np.diag(S)) + S ** 2) / (M - 1))
    assert np.max(np.abs(c - S) / se) < 5
    assert np.max(np.abs(2 * c - S) / se) > 5


def _near_dependent_functions(seed, m=400, nm=12):
    """Columns: values of nm functions at m points (any inner product reduces to
    a dot product of such columns); two columns are made dependent on others up
    to 1e-4 and 1e-7 of their norm, and the column norms differ widely."""
    r = rng(seed)
    A = r.standard_normal((m, nm)) * r.uniform(0.01, 100.0, nm)
    A[:, 5] = A[:, 1] - 2.0 * A[:, 3] + 1e-4 * np.linalg.norm(A[:, 1]) * r.standard_normal(m) / math.sqrt(m)
    A[:, 9] = 0.5 * A[:, 0] + A[:, 7] + 1e-7 * np.linalg.norm(A[:, 0]) * r.standard_normal(m) / math.sqrt(m)
    y = r.standard_normal(m)
    return A, y


def test_modal_pivots_match_pivoted_qr():
    """The greedy order of modal_pivots is that of a QR factorisation with
    column pivoting (LAPACK geqp3 through scipy) of the functions scaled to
    unit norm, and the modes kept are those whose |R_kk|^2 >= tol. All scaled
    columns tie at the first step, where the rule takes mode 0; the QR runs on
    the other columns with mode 0 projected out."""
    import scipy.linalg as sla
    for seed in (51, 52, 53):
        A, _ = _near_dependent_functions(seed)
        gam = A.T @ A
        An = A / np.linalg.norm(A, axis=0)
        u0 = An[:, 0]
        rest = An[:, 1:] - np.outer(u0, u0 @ An[:, 1:])
        _, R, perm = sla.qr(rest, mode="economic", pivoting=True)
        order = [0] + [int(x) + 1 for x in perm]
        rkk = np.concatenate([[1.0], np.abs(np.diag(R)) ** 2])
        # fixed tolerances, and ones just above and below a pivot's |R_kk|^2
        for tol in (1e-2, 1e-6, 1e-12, 1.5 * rkk[4], rkk[4] / 1.5):
            S = O.modal_pivots(gam, tol)
            k = int(np.argmax(rkk < tol)) if np.any(rkk < tol) else len(rkk)
            assert S == order[:k], (seed, tol, S, order[:k])
        assert 5 not in O.modal_pivots(gam, 1e-6) and 9 not in O.modal_pivots(gam, 1e-6)
        assert 5 in O.modal_pivots(gam, 1e-12) and 9 not in O.modal_pivots(gam, 1e-12)
        assert O.modal_pivots(gam, 0.0) == list(range(A.shape[1]))


def test_modal_solve_pivoted_is_orthonormal_projection():
    """For functions A and data y with gamma = A^T A and b = A^T y: alpha are the
    coefficients of y on the orthonormal vectors U of a thin QR of the kept
    columns (A_S = U R, diag R > 0), and A_S beta_S is the least-squares
    projection of y on their span (numpy lstsq); dropped modes get beta = 0."""
    A, y = _near_dependent_functions(54)
    gam = A.T @ A
    b = (A.T @ y)[None, :]
    alpha, beta, S = O.modal_solve_pivoted(gam, b, 1e-6)
    U, R = np.linalg.qr(A[:, S])
    sgn = np.sign(np.diag(R))
    U = U * sgn
    a_ref = U.T @ y
    assert np.allclose(alpha[0, :len(S)], a_ref, rtol=1e-9, atol=1e-9 * np.abs(a_ref).max())
    assert np.all(alpha[0, len(S):] == 0)
    bs = np.linalg.lstsq(A[:, S], y, rcond=None)[0]
    assert np.allclose(beta[0, S], bs, rtol=1e-7, atol=1e-9 * np.abs(bs).max())
    drop = [j for j in range(A.shape[1]) if j not in S]
    assert drop and np.all(beta[0, drop] == 0)
    # tol = 0 on a well-conditioned gamma: the plain solve gamma beta = b
    B = rng(55).standard_normal((300, 8))
    g2 = B.T @ B
    b2 = rng(56).standard_normal((2, 8))
    al2, be2, S2 = O.modal_solve_pivoted(g2, b2, 0.0)
    assert S2 == list(range(8))
    assert np.allclose(be2, np.linalg.solve(g2, b2.T).T, rtol=1e-10, atol=1e-12)
    al3, be3 = O.modal_solve(g2, b2)
    assert np.allclose(al2, al3, rtol=1e-12, atol=1e-14) and np.allclose(be2, be3, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("n,k0,dk,nb", [(8, 1.0, 1.0, 2), (16, 1.5, 1.0, 4)])
def test_triple_sums_gemm_brute_force(n, k0, dk, nb):
    """The matrix-product form of the triple sums and counts against the
    brute-force closed-triangle sums and the direct count enumeration."""
    spec = [_random_spec(n, 60 + i) for i in range(3)]
    lo, hi = O.bin_edges4(k0, dk, nb)
    tris, T = O.binned_triple_sums_gemm(spec, n, n, k0, dk, nb)
    scale = np.abs(T).max() / n ** 3
    for ti, (b1, b2, b3) in enumerate(tris):
        masks = [lambda q, b=b: (4 * q >= lo[b]) & (4 * q < hi[b]) for b in (b1, b2, b3)]
        for li in range(3):
            ref = O.closed_triangle_sum_brute([spec[li], spec[0], spec[0]], n, masks, modular=True)
            assert abs(T[li, ti] / n ** 3 - ref.real) < 1e-10 * scale, (b1, b2, b3, li)
    _, T1 = O.binned_triple_sums(spec, n, n, k0, dk, nb)
    assert np.allclose(T, T1, rtol=1e-12, atol=1e-12 * np.abs(T1).max())
    t2, cnt, resid = O.triangle_counts_gemm(n, k0, dk, nb)
    assert resid < 1e-6 and t2 == tris
    assert np.array_equal(cnt, O.triangle_counts_brute(k0, dk, nb, tris))


# ---------------------------------------------------------------- shot noise of B_l, l > 0

def test_ring_factor_limits_and_quadrature():
    """W_l(b1,b2|b3) is the mean of L_l(k1_hat . k2_hat) over closed triangles:
    1 for l = 0; symmetric in the first two legs; for thin shells the value of
    L_l at the opening angle of the central triangle, (k3^2 - k1^2 - k2^2) /
    (2 k1 k2); and the 32-point rule agrees with a 400-point one."""
    for c in ((10.0, 9.0, 8.0), (20.0, 16.0, 8.0), (12.0, 12.0, 12.0), (14.0, 6.0, 8.0)):
        assert abs(O.ring_factor(0, *c, 2.0) - 1.0) < 1e-13
        for ell in (2, 4):
            assert abs(O.ring_factor(ell, c[0], c[1], c[2], 2.0) - O.ring_factor(ell, c[1], c[0], c[2], 2.0)) < 1e-12
            assert abs(O.ring_factor(ell, *c, 4.0) - O.ring_factor(ell, *c, 4.0, nq=400)) < 2e-5
    mu = (64.0 - 100.0 - 81.0) / (2 * 10.0 * 9.0)
    assert abs(O.ring_factor(2, 10.0, 9.0, 8.0, 1e-4) - 0.5 * (3 * mu ** 2 - 1)) < 1e-6
    assert abs(O.ring_factor(4, 10.0, 9.0, 8.0, 1e-4) - (35 * mu ** 4 - 30 * mu ** 2 + 3) / 8) < 1e-6
    # squeezed: k3 small, k1 ~ k2 antiparallel is excluded (k3 = -(k1 + k2)): mu -> -1
    assert O.ring_factor(2, 30.0, 30.0, 1.0, 1.0) > 0.99
    # the definition itself by Monte Carlo: k1, k2 uniform in their shell volumes,
    # kept when |k1 + k2| falls in the third shell (a wrong triangle density,
    # e.g. k1 k2 instead of k1^2 k2^2 after the k3 integral, moves W by 0.01-0.05)
    r = rng(77)
    L = {2: lambda m: 0.5 * (3 * m * m - 1), 4: lambda m: (35 * m ** 4 - 30 * m * m + 3) / 8}
    for c1, c2, c3 in ((10.0, 9.0, 8.0), (6.0, 5.0, 3.0)):
        def shell(c, npts=2_000_000):
            rad = r.uniform((c - 2.0) ** 3, (c + 2.0) ** 3, npts) ** (1.0 / 3.0)
            v = r.standard_normal((npts, 3))
            return v / np.linalg.norm(v, axis=1)[:, None] * rad[:, None]
        k1, k2 = shell(c1), shell(c2)
        k3 = np.linalg.norm(k1 + k2, axis=1)
        ok = (k3 >= c3 - 2.0) & (k3 < c3 + 2.0)
        mu = np.sum(k1[ok] * k2[ok], 1) / (np.linalg.norm(k1[ok], axis=1) * np.linalg.norm(k2[ok], axis=1))
        for ell in (2, 4):
            x = L[ell](mu)
            se = x.std() / math.sqrt(x.size)
            assert abs(x.mean() - O.ring_factor(ell, c1, c2, c3, 4.0)) < 5 * se, (c1, c2, c3, ell)


def _closed_lattice_triangles(n, k0, dk, nb):
    r = np.arange(-(n // 2) + 1, n // 2)
    v = np.array([(a, b, c) for a in r for b in r for c in r if (a, b, c) != (0, 0, 0)])
    n2 = (v ** 2).sum(1)
    shell = np.full(len(v), -1)
    for b in range(nb):
        c = k0 + b * dk
        shell[((2 * c - dk) ** 2 <= 4 * n2) & (4 * n2 < (2 * c + dk) ** 2)] = b
    vs = [v[shell == b] for b in range(nb)]
    out = {}
    for b1, b2, b3 in O.triangle_list(nb):
        k1 = vs[b1][:, None, :]
        k2 = vs[b2][None, :, :]
        k3 = -(k1 + k2)
        m3 = (k3 ** 2).sum(-1)
        c = k0 + b3 * dk
        ok = ((2 * c - dk) ** 2 <= 4 * m3) & (4 * m3 < (2 * c + dk) ** 2)
        i, j = np.nonzero(ok)
        if len(i):
            out[(b1, b2, b3)] = (vs[b1][i], vs[b2][j], -(vs[b1][i] + vs[b2][j]))
    return out


@pytest.mark.parametrize("observer", [None, (-5.3, -7.1, -6.2)])
def test_shot_noise_coincidence_brute_force(observer):
    """The four coincidence sums of shot_noise_coincidence against a direct
    sum over closed lattice triangles and particle index tuples, with the
    Legendre weight (2l + 1) L_l(k1_hat . x_hat_i) written out (not through the
    x_hat-product transforms): five unit particles on an 8^3 grid, two of them on
    one node, plane-parallel and varying line of sight."""
    n, box, k0, dk, nb, lmax = 8, 50.0, 1.0, 1.0, 2, 4
    pos = np.array([[1, 2, 3], [5, 0, 7], [5, 0, 7], [3, 6, 2], [7, 7, 1]], dtype=np.float64)
    cnt = np.zeros((n, n, n))
    for p in pos.astype(int):
        cnt[tuple(p)] += 1
    nbar_cell = len(pos) / n ** 3
    tri = _closed_lattice_triangles(n, k0, dk, nb)
    tris = list(tri)
    got = O.shot_noise_coincidence(cnt, lmax, observer, k0, dk, nb, tris, box, nbar_cell)
    if observer is None:
        xh = np.tile([0.0, 0.0, 1.0], (len(pos), 1))
    else:
        d = pos - np.asarray(observer)
        xh = d / np.linalg.norm(d, axis=1)[:, None]
    L = {0: lambda m: np.ones_like(m), 2: lambda m: 0.5 * (3 * m ** 2 - 1),
         4: lambda m: (35 * m ** 4 - 30 * m ** 2 + 3) / 8}
    V = box ** 3
    for i, t in enumerate(tris):
        k1, k2, k3 = tri[t]
        ntri = len(k1)
        norm = V ** 2 / (float(n) ** 9 * ntri * nbar_cell ** 3)
        ph = lambda k: np.exp(-2j * np.pi * (k @ pos.T) / n)  # [triangles][particles]
        e1, e2, e3 = ph(k1), ph(k2), ph(k3)
        e13 = ph(k1 + k3)
        e12 = ph(k1 + k2)
        k1h = k1 / np.linalg.norm(k1, axis=1)[:, None]
        for li, ell in enumerate((0, 2, 4)):
            w = (2 * ell + 1) * L[ell](k1h @ xh.T)  # [triangles][particles]
            A = np.sum((w * e1).sum(1) * ph(k2 + k3).sum(1))
            B = np.sum((w * e13).sum(1) * e2.sum(1))
            Cc = np.sum((w * e12).sum(1) * e3.sum(1))
            D = np.sum(w.sum(1))
            want = np.real(np.array([A, B, Cc, D])) * norm
            assert np.allclose(got[:, li, i], want, rtol=1e-9, atol=1e-9 * np.abs(want).max()), (t, ell, got[:, li, i], want)


def test_shot_noise_inclusion_exclusion_unbiased():
    """Poisson counts at the nodes of a fixed, anisotropic intensity lambda
    (NGP, no compensation, delta = counts / nbar - 1 with the true mean): the
    raw B_l minus the coincidence terms (pair terms minus twice the triple
    term) has the expectation B_l of delta_lambda = lambda / nbar - 1 itself,
    for every l; the raw B_0 does not (its shot noise is large here)."""
    n, box, k0, dk, nb, lmax = 16, 100.0, 2.0, 2.0, 2, 4
    r = rng(31)
    f = O.signed_freq(n)
    kx, ky, kz = np.meshgrid(f, f, np.arange(n // 2 + 1), indexing="ij")
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    kk[0, 0, 0] = 1.0
    amp = np.sqrt(kk ** -1.0) * (1 + 2.0 * (kz / kk) ** 2)
    g = sfft.irfftn(amp * (r.standard_normal(kk.shape) + 1j * r.standard_normal(kk.shape)), s=(n, n, n))
    g *= 0.5 / g.std()
    nbar_cell = 2.0
    lam = np.exp(g)
    lam *= nbar_cell / lam.mean()
    tris_all, cnt3, _ = O.triangle_counts_fft(n, k0, dk, nb)
    tk = [t for t, c in zip(tris_all, cnt3) if c > 0]
    ck = np.array([c for c in cnt3 if c > 0])

    def bl(delta):
        spec = O.spectrum_from_field([delta], [0.0], n, lmax, None, None)
        _, T = O.binned_triple_sums(spec, n, n, k0, dk, nb, tk)
        return O.binned_bispectrum(T, ck, n, n, box)

    truth = bl(lam / nbar_cell - 1.0)
    raw, sub = [], []
    for i in range(300):
        c = r.poisson(lam).astype(np.float64)
        b = bl(c / nbar_cell - 1.0)
        sn = O.shot_noise_coincidence(c, lmax, None, k0, dk, nb, tk, box, nbar_cell)
        raw.append(b.ravel())
        sub.append((b - (sn[0] + sn[1] + sn[2] - 2 * sn[3])).ravel())
    assert np.max(np.abs(_zscores(sub, truth.ravel()))) < 5
    assert np.max(np.abs(_zscores(raw, truth.ravel()))) > 5


def test_shot_noise_model_against_coincidence_terms():
    """The shell-and-ring model (shot_noise_multipoles) against the exact
    coincidence terms of one Poisson catalogue (plane-parallel, NGP, no
    compensation) at k = 14-26 k_f: the l = 0 term is the standard one, the
    l = 2 and l = 4 terms are the reading's approximation; the measured
    normwise differences are the tolerances' basis (lattice rings with few
    points make l = 4 the worst)."""
    n, box, k0, dk, nb, lmax = 96, 1000.0, 16.0, 4.0, 3, 4
    r = rng(41)
    f = O.signed_freq(n)
    kx, ky, kz = np.meshgrid(f, f, np.arange(n // 2 + 1), indexing="ij")
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    kk[0, 0, 0] = 1.0
    amp = np.sqrt(kk ** -1.2) * (1 + 3.0 * (kz / kk) ** 2)
    g = sfft.irfftn(amp * (r.standard_normal(kk.shape) + 1j * r.standard_normal(kk.shape)), s=(n, n, n))
    g *= 0.6 / g.std()
    nbar_cell = 1.0
    lam = np.exp(g)
    lam *= nbar_cell / lam.mean()
    c = r.poisson(lam).astype(np.float64)
    tris_all, cnt3, _ = O.triangle_counts_fft(n, k0, dk, nb)
    tk = [t for t, cc in zip(tris_all, cnt3) if cc > 0]
    spec = O.spectrum_from_field([c / nbar_cell - 1.0], [0.0], n, lmax, None, None)
    P, _ = O.power_multipoles(spec, n, k0, dk, nb, box)
    nbar = nbar_cell * n ** 3 / box ** 3
    model = O.shot_noise_multipoles(P, tk, k0, dk, nbar)
    sn = O.shot_noise_coincidence(c, lmax, None, k0, dk, nb, tk, box, nbar_cell)
    exact = sn[0] + sn[1] + sn[2] - 2 * sn[3]
    err = [float(np.linalg.norm(model[li] - exact[li]) / np.linalg.norm(exact[li])) for li in range(3)]
    print("model vs exact shot noise, l = 0, 2, 4:", err)
    assert err[0] < 0.01 and err[1] < 0.02 and err[2] < 0.3, err
    # the ring factor matters: with W = 1 the l = 2 model is far off
    crude = np.array([[(P[li][a] + P[li][b] + P[li][cc]) / nbar for a, b, cc in tk] for li in range(3)])
    assert np.linalg.norm(crude[1] - exact[1]) / np.linalg.norm(exact[1]) > 3 * err[1]

"""Parity at the bench configuration (512^3, varying line of sight, l <= 4,
30 shells of 5 k_f, 100 modes with P = 8), in the launch configuration the
bench times, on outputs the FP64 oracle can compute one by one.

The input is a seeded random contrast field delta(x) on 512^3 handed to
bsp_bispectrum_field (LOS-weighted forward transforms, Legendre moments,
shell and modal filters, inverse transforms, triple reduction, FP64
normalisation). The oracle builds delta^(0,2,4)(n) from the same field and
evaluates, for a few triangles, the exact triangle count and
T^l = sum_x D^l_b1 D^0_b2 D^0_b3, and, for a few modes, the monopole modal
numerator <M_p M_r M_s>. Differences are measured against the larger of the
sum itself and the scale of the summed terms, sqrt(sum_x (summand)^2): a sum
of 1.3e8 terms of either sign is only defined to that scale times the working
precision, and a coherent sum (smooth low-k fields) to its own size. Bounds: 5e-5 for the
FP32 path (one sampled output carries the FP32 rounding of six 512-point
transform passes of each of its three fields, about 1e-6 each, correlated
through the spectra; the normwise 1e-5 over whole output families is checked at
the smaller sizes), 1e-3 (the mixed-precision target on B_l) for bf16 hi+lo
products.
"""
import math
import sys
import time

import numpy as np
import pytest

import oracle as O
from synth import catalog as C
from tests.gpu_helpers import pfid_table

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1708_05303_amd as B  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print("[full]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full_case():
    t0 = time.time()
    wl = C.workload("c3_512")
    n = wl.n
    obs = C.observer_grid_units(wl)
    n2len = 3 * ((wl.nbins + 1) * int(wl.dk) + int(wl.k0) + 2) ** 2
    pf = pfid_table(wl, n2len)
    plan = B.Plan(n=n, box=wl.box, nbins=wl.nbins, k0=wl.k0, dk=wl.dk, lmax=4, window=1, compensate=1,
                  interlace=1, los=1, observer=obs, P=wl.P, nmodes=wl.nmodes, pfid=pf)
    plan.precompute()
    say("plan", time.time() - t0)
    d32 = np.random.Generator(np.random.PCG64(5120)).standard_normal((n, n, n), dtype=np.float32)
    dd = torch.as_tensor(d32).to(DEV)
    info = plan.info
    got = {}
    for prec in (B.BSP_FP32, B.BSP_BF16X3):
        Bt = torch.zeros((info.nl, info.ntri), dtype=torch.float64, device=DEV)
        bn = torch.zeros((info.nl, wl.nmodes), dtype=torch.float64, device=DEV)
        B.bsp_bispectrum_field(plan.handle, dd, prec, Bt, None, bn, None, None)
        plan.sync()
        got[prec] = (Bt.cpu().numpy(), bn.cpu().numpy())
    tri, counts = plan.tri.copy(), plan.counts.copy()
    del dd
    plan.close()
    torch.cuda.empty_cache()
    say("gpu", time.time() - t0)
    spec = O.spectrum_from_field([d32.astype(np.float64)], [0.0], n, 4, obs, None)
    del d32
    say("oracle spectrum", time.time() - t0)
    return wl, pf, tri, counts, got, spec


def _sample_triangles(tri):
    # the largest, a middle and a small closed triangle
    want = [tuple(tri[-1]), tuple(tri[len(tri) // 2]), tuple(tri[3])]
    idx = [int(np.nonzero((tri == np.array(t)).all(1))[0][0]) for t in want]
    return idx


def test_full_size_triangle_counts_and_binned(full_case):
    wl, pf, tri, counts, got, spec = full_case
    n = wl.n
    bins = O.bin_of_n2(O.n2_grid_half(n), wl.k0, wl.dk, wl.nbins)
    norm_base = wl.box ** 6 / (float(n) ** 9 * float(n) ** 3)
    for i in _sample_triangles(tri):
        b1, b2, b3 = (int(v) for v in tri[i])
        say("triangle", b1, b2, b3)
        # exact count: sum_x I_b1 I_b2 I_b3 / N'^3 from FP64 indicator fields
        ones = np.ones(bins.shape)
        I = [O.shell_field(ones, bins == b, n).ravel() for b in (b1, b2, b3)]
        cnt = float(np.dot(I[0] * I[1], I[2])) / float(n) ** 3
        del I, ones
        assert abs(cnt - round(cnt)) < 1e-3 and int(round(cnt)) == int(counts[i]), (cnt, counts[i])
        pair = O.shell_field(spec[0], bins == b2, n).ravel() * O.shell_field(spec[0], bins == b3, n).ravel()
        norm = norm_base / float(counts[i])
        for li in range(3):
            D1 = O.shell_field(spec[li], bins == b1, n).ravel()
            Tref = float(np.dot(D1, pair))
            scale = math.sqrt(float(np.dot(D1 * D1, pair * pair)))
            for prec, tol in ((B.BSP_FP32, 5e-5), (B.BSP_BF16X3, 1e-3)):
                e = abs(got[prec][0][li, i] / norm - Tref) / max(scale, abs(Tref))
                say("  l", 2 * li, "prec", prec, "scaled err", e, "rel err", abs(got[prec][0][li, i] / norm / Tref - 1))
                assert e < tol, (b1, b2, b3, li, prec, e)


def test_full_size_modal_numerators(full_case):
    wl, pf, tri, counts, got, spec = full_case
    n = wl.n
    kmin = wl.k0 - 0.5 * wl.dk
    kmax = wl.k0 + (wl.nbins - 0.5) * wl.dk
    kf = 2 * math.pi / wl.box
    M = O.modal_fields(spec[0], n, n, wl.P, kmin, kmax, kf, pf)
    modes = O.modal_modes(wl.P, wl.nmodes)
    K = float(n) ** 3
    for m in (0, 41, wl.nmodes - 1):
        p, r, s = (int(v) for v in modes[m])
        prod = M[p] * M[r]
        ref = float(np.dot(prod, M[s])) / K
        scale = math.sqrt(float(np.dot(prod * prod, M[s] * M[s]))) / K
        for prec, tol in ((B.BSP_FP32, 5e-5), (B.BSP_BF16X3, 1e-3)):
            e = abs(got[prec][1][0, m] - ref) / max(scale, abs(ref))
            say("mode", m, (p, r, s), "prec", prec, "scaled err", e, "rel err", abs(got[prec][1][0, m] / ref - 1))
            assert e < tol, (m, prec, e)


@pytest.fixture(scope="module")
def spectra_case():
    """The bench plan's LOS moments of a seeded white-noise contrast field
    (bsp_grid_entry), then the power-spectrum multipoles, skew spectra (also
    with the squared monopole on the ball of the band) and integrated
    bispectrum (8^3 sub-volumes of 64^3, 20 shells of one sub-volume
    fundamental; one line of sight per sub-volume and varying inside each) on
    the GPU, and the same from the FP64 oracle."""
    t0 = time.time()
    wl = C.workload("c3_512")
    n = wl.n
    obs = C.observer_grid_units(wl)
    plan = B.Plan(n=n, box=wl.box, nbins=wl.nbins, k0=wl.k0, dk=wl.dk, lmax=4, window=1, compensate=1,
                  interlace=1, los=1, observer=obs)
    info = plan.info
    d32 = np.random.Generator(np.random.PCG64(5121)).standard_normal((n, n, n), dtype=np.float32)
    dd = torch.as_tensor(d32).to(DEV)
    dl = plan.spectrum_buffer()
    B.bsp_grid_entry(plan.handle, dd, dl)
    P = torch.zeros((info.nl, wl.nbins), dtype=torch.float64, device=DEV)
    S = torch.zeros((info.nl, wl.nbins), dtype=torch.float64, device=DEV)
    s, ibn = 8, 20
    iB = torch.zeros((info.nl, ibn), dtype=torch.float64, device=DEV)
    Ps = torch.zeros((s ** 3, info.nl, ibn), dtype=torch.float64, device=DEV)
    Sb = torch.zeros_like(S)
    iBl = torch.zeros_like(iB)
    Psl = torch.zeros_like(Ps)
    B.bsp_power_multipoles(plan.handle, dl, P)
    B.bsp_skew_spectra(plan.handle, dl, S)
    B.bsp_skew_spectra(plan.handle, dl, Sb, B.BSP_SKEW_BALL)
    B.bsp_integrated_bispectrum(plan.handle, dd, None, s, 1.0, 1.0, ibn, iB, Ps, None)
    B.bsp_integrated_bispectrum(plan.handle, dd, None, s, 1.0, 1.0, ibn, iBl, Psl, None, B.BSP_IB_LOCAL_LOS)
    plan.sync()
    got = (P.cpu().numpy(), S.cpu().numpy(), iB.cpu().numpy(), Ps.cpu().numpy(), Sb.cpu().numpy(),
           iBl.cpu().numpy(), Psl.cpu().numpy())
    del dd, dl
    plan.close()
    torch.cuda.empty_cache()
    say("spectra gpu", time.time() - t0)
    d64 = d32.astype(np.float64)
    del d32
    spec = O.spectrum_from_field([d64], [0.0], n, 4, obs, None)
    Pref, _ = O.power_multipoles(spec, n, wl.k0, wl.dk, wl.nbins, wl.box)
    Sref, _ = O.skew_spectra(spec, n, n, wl.k0, wl.dk, wl.nbins, wl.box)
    Sbref, _ = O.skew_spectra(spec, n, n, wl.k0, wl.dk, wl.nbins, wl.box, "ball")
    del spec
    iBref, Psref, dbar, _ = O.integrated_bispectrum(d64, s, 4, obs, 1, wl.box, 1.0, 1.0, ibn)
    say("spectra oracle, one LOS per sub-volume", time.time() - t0)
    # the local line of sight on 24 sampled sub-volumes (corners, centre, seeded picks)
    picks = sorted({0, s ** 3 - 1, s ** 3 // 2, s * s - 1, s ** 3 - s * s} |
                   set(np.random.Generator(np.random.PCG64(77)).choice(s ** 3, 19, replace=False).tolist()))
    _, Pslref, _, _ = O.integrated_bispectrum_local_los(d64, s, 4, obs, 1, wl.box, 1.0, 1.0, ibn, picks)
    say("spectra oracle, local LOS on", len(picks), "sub-volumes", time.time() - t0)
    return got, (Pref, Sref, iBref, Psref, dbar, Sbref, picks, Pslref)


def test_full_size_power_and_skew_spectra(spectra_case):
    (P, S, _, _, Sb, _, _), (Pref, Sref, _, _, _, Sbref, _, _) = spectra_case
    for name, g, r, tol in (("P", P, Pref, 1e-5), ("S", S, Sref, 1e-5), ("S ball", Sb, Sbref, 1e-5)):
        s0 = np.linalg.norm(r[0])
        for li in range(r.shape[0]):
            e = np.linalg.norm(g[li] - r[li]) / max(np.linalg.norm(r[li]), 0.01 * s0)
            say(name, "l", 2 * li, "err", e)
            assert e < tol, (name, li, e)


def test_full_size_integrated_bispectrum(spectra_case):
    (_, _, iB, Ps, _, _, _), (_, _, iBref, Psref, dbar, _, _, _) = spectra_case
    ns = Ps.shape[0]
    for li in range(iB.shape[0]):
        e = np.linalg.norm(Ps[:, li] - Psref[:, li]) / max(np.linalg.norm(Psref[:, li]),
                                                           0.01 * np.linalg.norm(Psref[:, 0]))
        scale = np.linalg.norm(np.abs(Psref[:, li]).T @ np.abs(dbar)) / ns
        ei = np.linalg.norm(iB[li] - iBref[li]) / scale
        say("iB l", 2 * li, "P err", e, "iB err / term scale", ei)
        assert e < 1e-5 and ei < 1e-5, (li, e, ei)


def test_full_size_integrated_bispectrum_local_los(spectra_case):
    """Sub-volume multipoles with the line of sight varying inside each, on
    sampled sub-volumes (the oracle evaluates them one by one); the average
    iB uses every sub-volume and is checked against the GPU's P with the
    oracle's mean overdensities."""
    (_, _, _, _, _, iBl, Psl), (_, _, _, _, dbar, _, picks, Pslref) = spectra_case
    for li in range(Psl.shape[1]):
        g, r = Psl[picks, li], Pslref[picks, li]
        e = np.linalg.norm(g - r) / max(np.linalg.norm(r), 0.01 * np.linalg.norm(Pslref[picks, 0]))
        say("local LOS P l", 2 * li, "err on", len(picks), "sub-volumes", e)
        assert e < 1e-5, (li, e)
    ns = Psl.shape[0]
    for li in range(Psl.shape[1]):
        avg = Psl[:, li].T @ dbar / ns
        scale = np.linalg.norm(np.abs(Psl[:, li]).T @ np.abs(dbar)) / ns
        assert np.linalg.norm(iBl[li] - avg) < 1e-5 * scale, li


@pytest.fixture(scope="module")
def catalogue_case():
    """The bench catalogue itself (1e7 lognormal particles with Kaiser
    displacements, CIC on two interlaced grids, 8 x 8 x 32 tiles) through
    bsp_bispectrum_multipoles in FP32 and bf16 hi+lo, and its LOS moment
    spectra through bsp_los_moments for the raw modal numerators
    (bsp_modal_coeffs without shot noise); the oracle runs the same catalogue
    from its own assignment in FP64."""
    t0 = time.time()
    wl = C.workload("c3_512")
    n = wl.n
    obs = C.observer_grid_units(wl)
    n2len = 3 * ((wl.nbins + 1) * int(wl.dk) + int(wl.k0) + 2) ** 2
    pf = pfid_table(wl, n2len)
    plan = B.Plan(n=n, box=wl.box, nbins=wl.nbins, k0=wl.k0, dk=wl.dk, lmax=4, window=1, compensate=1,
                  interlace=1, los=1, observer=obs, P=wl.P, nmodes=wl.nmodes, pfid=pf, drop_tol=1e-2)
    plan.precompute()
    u = C.lognormal_catalogue(wl)
    dv = [torch.as_tensor(a).to(DEV) for a in u]
    info = plan.info
    got = {}
    for prec in (B.BSP_FP32, B.BSP_BF16X3):
        Bt = torch.zeros((info.nl, info.ntri), dtype=torch.float64, device=DEV)
        B.bsp_bispectrum_multipoles(plan.handle, dv[0], dv[1], dv[2], None, u[0].size, prec, Bt, None, None,
                                    None, None, None)
        grids = torch.zeros((2, n, n, n), dtype=torch.float32, device=DEV)
        wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
        B.bsp_grid_assign(plan.handle, dv[0], dv[1], dv[2], None, u[0].size, grids, wsum)
        dl = plan.spectrum_buffer()
        B.bsp_los_moments(plan.handle, grids, wsum, dl)
        del grids
        bn = torch.zeros((info.nl, wl.nmodes), dtype=torch.float64, device=DEV)
        B.bsp_modal_coeffs(plan.handle, dl, prec, 0.0, bn, None, None)
        Bf = torch.zeros((info.nl ** 3, info.ntri), dtype=torch.float64, device=DEV)
        B.bsp_bispectrum_full(plan.handle, dl, prec, Bf)
        plan.sync()
        got[prec] = (Bt.cpu().numpy(), bn.cpu().numpy(), Bf.cpu().numpy())
        del dl, Bf
    tri, counts = plan.tri.copy(), plan.counts.copy()
    del dv
    plan.close()
    torch.cuda.empty_cache()
    say("catalogue gpu", time.time() - t0)
    spec, _ = O.spectrum_from_catalogue(*u, n, 4, obs, window=1, interlace=1)
    say("catalogue oracle spectrum", time.time() - t0)
    return wl, pf, tri, counts, got, spec


def test_full_size_catalogue_binned(catalogue_case):
    """Every closed triangle whose largest side is in shell 8 or 16, per l,
    normwise against the oracle's triple sums (matrix-product form)."""
    wl, pf, tri, counts, got, spec = catalogue_case
    n = wl.n
    shells = (8, 16)
    sel = [i for i in range(len(tri)) if int(tri[i][0]) in shells]
    tris = [tuple(int(v) for v in tri[i]) for i in sel]
    t0 = time.time()
    _, T = O.binned_triple_sums_gemm(spec, n, n, wl.k0, wl.dk, max(shells) + 1, tris)
    say("catalogue oracle triple sums", time.time() - t0, len(tris), "triangles")
    ref = O.binned_bispectrum(T, counts[sel], n, n, wl.box)
    for prec, tol in ((B.BSP_FP32, 1e-5), (B.BSP_BF16X3, 1e-3)):
        for li in range(3):
            e = float(np.linalg.norm(got[prec][0][li, sel] - ref[li]) / np.linalg.norm(ref[li]))
            say("  catalogue B l", 2 * li, "prec", prec, "normwise err", e)
            assert e < tol, (li, prec, e)


def test_full_size_catalogue_full_multipoles_contain_the_path(catalogue_case):
    """B^(l00) of bsp_bispectrum_full at the bench plan (every (l1, l2, l3)
    over the 90 shell fields, in the workspace the bench plan has) against the
    whole path's B_l: the same sums, scheduled and chunked differently."""
    _, _, _, _, got, _ = catalogue_case
    nl = 3
    for prec in (B.BSP_FP32, B.BSP_BF16X3):
        Bl, _, Bf = got[prec]
        for li in range(nl):
            e = float(np.linalg.norm(Bf[li * nl * nl] - Bl[li]) / np.linalg.norm(Bl[li]))
            say("  full multipoles B^(l00) vs path, l", 2 * li, "prec", prec, e)
            assert e < 1e-12, (li, prec, e)


def test_full_size_catalogue_modal_numerators(catalogue_case):
    """All 100 raw monopole modal numerators b^0 of the catalogue, normwise."""
    wl, pf, tri, counts, got, spec = catalogue_case
    n = wl.n
    kmin = wl.k0 - 0.5 * wl.dk
    kmax = wl.k0 + (wl.nbins - 0.5) * wl.dk
    kf = 2 * math.pi / wl.box
    modes = O.modal_modes(wl.P, wl.nmodes)
    t0 = time.time()
    ref = O.modal_numerators(spec[:1], n, n, modes, wl.P, kmin, kmax, kf, pf)[0]
    say("catalogue oracle numerators", time.time() - t0)
    for prec, tol in ((B.BSP_FP32, 1e-5), (B.BSP_BF16X3, 1e-4)):
        e = float(np.linalg.norm(got[prec][1][0] - ref) / np.linalg.norm(ref))
        say("  catalogue b0 prec", prec, "normwise err", e)
        assert e < tol, (prec, e)

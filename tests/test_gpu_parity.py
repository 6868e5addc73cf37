"""Parity of the HIP path (through the C ABI) with the FP64 oracle, small sizes.

Every comparison runs the GPU on seeded synthetic inputs and the oracle on the
same inputs; tolerances follow the arithmetic: FP32 path 1e-5 normwise,
split-precision products 1e-3 on B_l and 1e-4 on beta_n, integers exact.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from synth import catalog as C
from tests.gpu_helpers import compact_to_half, gpu_cube_to_numpy, half_to_compact, pfid_table, rel_norm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1708_05303_amd as B  # noqa: E402

DEV = torch.device("cuda:0")
MODAL_DROP_TOL = 1e-2  # relative residual below which the orthonormalisation drops a mode


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


# ---------------------------------------------------------------- transforms

@pytest.mark.parametrize("n", [16, 32, 64, 96, 128, 192, 256, 384, 512])
def test_fft_r2c_c2r_against_oracle(n):
    say("fft", n)
    plan = B.Plan(n=n, box=100.0, nbins=1, k0=1.0, dk=1.0)
    x = rng(n).standard_normal((2, n, n, n))
    xi = dev(x)
    out = torch.zeros((2, n, n, n // 2 + 1, 2), dtype=torch.float32, device=DEV)
    B.bsp_fft_r2c(plan.handle, n, 2, xi, out)
    back = torch.zeros((2, n, n, n), dtype=torch.float32, device=DEV)
    B.bsp_fft_c2r(plan.handle, n, 2, out, back)
    plan.sync()
    o = out.cpu().numpy()
    got = o[..., 0] + 1j * o[..., 1]
    for b in range(2):
        ref = O.forward(x[b])
        assert rel_norm(np.stack([got[b].real, got[b].imag]), np.stack([ref.real, ref.imag])) < 2e-6
    assert rel_norm(back.cpu().numpy(), x * n ** 3) < 2e-6


# ---------------------------------------------------------------- assignment

def _tiled_assign_bytes(npart, n):
    """Scratch the sorted, tiled assignment needs (8 x 8 x tz tiles, a 256-byte head)."""
    tz = next(t for t in (32, 16, 8) if n % t == 0 and n // t >= 2)
    nt = (n // 8) ** 2 * (n // tz)
    up = lambda b: (b + 255) // 256 * 256
    return 256 + up(npart * 16) + 2 * up((nt + 1) * 4) + up(npart * 4)


def _fixed_assign_bytes(n, interlace):
    """Scratch of the fixed-point global-atomic assignment: int64 grids and a 256-byte head."""
    return 256 + (1 + interlace) * n ** 3 * 8


def _assign_plan(n, window, interlace, mode, npart):
    """Plan whose workspace selects the assignment kernel: 'atomic' none (FP32
    global atomics), 'fixed' room for the int64 grids but not for the sorted
    catalogue (fixed-point global atomics), 'tiled' the full workspace."""
    plan = B.Plan(n=n, box=100.0, nbins=1, k0=1.0, dk=1.0, window=window, interlace=interlace,
                  workspace=(mode == "tiled"))
    if mode == "tiled":
        assert B.bsp_workspace_size(plan.handle) >= _tiled_assign_bytes(npart, n)
    if mode == "fixed":
        nb = _fixed_assign_bytes(n, interlace)
        assert nb < _tiled_assign_bytes(npart, n)
        plan.ws = torch.empty(nb, dtype=torch.uint8, device=DEV)
        B.bsp_set_workspace(plan.handle, plan.ws, nb)
    return plan


def _edge_catalogue(n, npart, seed):
    r = rng(seed)
    u = [C.quantise_grid_units(r.uniform(0, n, npart), n) for _ in range(3)]
    edges = np.array([0.0, 7.999755859375, 8.0, n - 2.0 ** -12, n - 0.5, 15.999755859375], np.float32)
    for a in range(3):
        u[a][:36] = np.tile(edges, 6)[(np.arange(36) * (a + 1)) % 36]
    return u, r


@pytest.mark.parametrize("n,window,interlace,mode", [
    (32, 1, 0, "atomic"), (32, 1, 1, "atomic"), (32, 0, 1, "atomic"),
    (16, 1, 1, "fixed"), (32, 1, 1, "fixed"), (32, 0, 1, "fixed"), (64, 1, 0, "fixed"),
    (16, 1, 1, "tiled"), (32, 1, 0, "tiled"), (32, 1, 1, "tiled"), (32, 0, 1, "tiled"), (64, 1, 1, "tiled"),
    (96, 1, 1, "tiled"), (96, 0, 0, "tiled"), (128, 1, 1, "tiled"), (128, 0, 1, "tiled")])
def test_grid_assign_against_oracle(n, window, interlace, mode):
    """The three assignment kernels against the oracle, adding into grids that
    already hold 0.25; particles also sit on tile edges and just below N
    (wrap-around). 128 points a side runs the 8 x 8 x 32 tiles.
    Weighted catalogue: FP32 atomics within their summation bound; the
    fixed-point kernels within 2 ulp (one rounding of the node sum, one of the
    addition). Unit weights, positions on multiples of 2^-12: the fixed-point
    node sums are exact, so each node is bit for bit float32(0.25 + float32(rho))
    of the oracle's rho, and the weight sum is the particle count."""
    npart = {"atomic": 20000, "tiled": 20000, "fixed": 20 * n ** 3 // 16 + 4000}[mode]
    say("assign", n, window, interlace, mode, npart)
    u, r = _edge_catalogue(n, npart, 7 + n)
    w = r.uniform(0.5, 1.5, npart).astype(np.float32)
    plan = _assign_plan(n, window, interlace, mode, npart)
    grids = torch.full((1 + interlace, n, n, n), 0.25, dtype=torch.float32, device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    B.bsp_grid_assign(plan.handle, dev(u[0]), dev(u[1]), dev(u[2]), dev(w), u[0].size, grids, wsum)
    plan.sync()
    g = grids.cpu().numpy()
    for s in range(1 + interlace):
        ref = O.assign(*u, n, w.astype(np.float64), window, 0.5 * s) + 0.25
        if mode == "atomic":
            assert np.max(np.abs(g[s] - ref)) < 2e-6 * np.max(ref) + 1e-6, s
        else:
            r32 = ref.astype(np.float32)
            assert np.all(np.abs(g[s] - r32) <= 2 * np.spacing(np.abs(r32))), s
    assert abs(wsum.item() - float(w.astype(np.float64).sum())) < 1e-6 * w.sum()
    if mode == "atomic":
        plan.close()
        return
    # unit weights: exact
    for rep in range(2):
        grids2 = torch.full((1 + interlace, n, n, n), 0.25, dtype=torch.float32, device=DEV)
        wsum2 = torch.zeros(1, dtype=torch.float64, device=DEV)
        B.bsp_grid_assign(plan.handle, dev(u[0]), dev(u[1]), dev(u[2]), None, u[0].size, grids2, wsum2)
        plan.sync()
        g2 = grids2.cpu().numpy()
        for s in range(1 + interlace):
            rho = O.assign(*u, n, None, window, 0.5 * s)
            expect = np.float32(0.25) + rho.astype(np.float32)
            assert np.array_equal(g2[s], expect), (rep, s, int(np.sum(g2[s] != expect)))
        assert wsum2.item() == float(npart)
    plan.close()


@pytest.mark.parametrize("n,mode", [(32, "fixed"), (64, "tiled"), (128, "tiled")])
def test_grid_assign_reproducible(n, mode):
    """The fixed-point kernels give bit-identical grids and weight sums on
    repeated runs of a weighted, clustered catalogue (where FP32 atomics in
    varying order would differ in the last bits)."""
    say("assign-repro", n, mode)
    npart = 20 * n ** 3 // 16 + 4000 if mode == "fixed" else 200000
    r = rng(300 + n)
    hot = npart // 2
    u = [C.quantise_grid_units(np.concatenate([r.uniform(5.0, 9.0, hot), r.uniform(0, n, npart - hot)]), n)
         for _ in range(3)]
    w = r.uniform(0.1, 3.0, npart).astype(np.float32)
    plan = _assign_plan(n, 1, 1, mode, npart)
    out = []
    for rep in range(3):
        grids = torch.zeros((2, n, n, n), dtype=torch.float32, device=DEV)
        wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
        B.bsp_grid_assign(plan.handle, dev(u[0]), dev(u[1]), dev(u[2]), dev(w), npart, grids, wsum)
        plan.sync()
        out.append((grids.cpu().numpy(), wsum.item()))
    for g, ws in out[1:]:
        assert np.array_equal(g, out[0][0]) and ws == out[0][1]
    plan.close()


def test_grid_assign_tiled_clustered_with_invalid_particles():
    """Sorted, tiled assignment of a clustered catalogue (most particles in a
    cube straddling tile edges, many tiles empty) with invalid entries mixed in
    (outside [0, N) or a NaN weight): the count and the scatter skip the same
    particles, the valid ones match the oracle and the error is latched."""
    say("assign-tiled-clustered-invalid")
    n = 32
    r = rng(41)
    npart = 30000
    hot = int(0.8 * npart)
    u = [np.concatenate([r.uniform(7.0, 9.5, hot), r.uniform(0, n, npart - hot)]) for _ in range(3)]
    u = [C.quantise_grid_units(a, n) for a in u]
    w = r.uniform(0.5, 1.5, npart).astype(np.float32)
    bad = np.array([5, 777, 12345, 29999])
    u[0][bad[0]] = float(n)
    u[1][bad[1]] = -0.5
    w[bad[2]] = np.nan
    u[2][bad[3]] = float(n) + 3.0
    ok = np.ones(npart, bool)
    ok[bad] = False
    plan = B.Plan(n=n, box=100.0, nbins=1, k0=1.0, dk=1.0, window=1, interlace=1, workspace=True)
    assert B.bsp_workspace_size(plan.handle) >= _tiled_assign_bytes(npart, n)
    grids = torch.zeros((2, n, n, n), dtype=torch.float32, device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    B.bsp_grid_assign(plan.handle, dev(u[0]), dev(u[1]), dev(u[2]), dev(w), npart, grids, wsum)
    with pytest.raises(B.BspError) as e:
        plan.sync()
    assert e.value.status == 6
    g = grids.cpu().numpy()
    wv = w[ok].astype(np.float64)
    for s in range(2):
        ref = O.assign(u[0][ok], u[1][ok], u[2][ok], n, wv, 1, 0.5 * s)
        # the tiled kernel rounds each of a node's m CIC contributions once to a
        # multiple of 2^-36 (fixed point, 2^-37 each at most) and the exact sum
        # once to FP32: bound each node by (m + 4) u times its value plus
        # m 2^-37, u = 2^-24 (tight on sparse nodes, where a misplaced particle
        # would show)
        m = np.zeros(n ** 3)
        fl = [np.floor(a[ok].astype(np.float64) + 0.5 * s).astype(np.int64) for a in u]
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    idx = (((fl[0] + dx) % n) * n + (fl[1] + dy) % n) * n + (fl[2] + dz) % n
                    np.add.at(m, idx, 1.0)
        bound = (m.reshape(n, n, n) + 4.0) * 2.0 ** -24 * ref + m.reshape(n, n, n) * 2.0 ** -37
        assert np.all(np.abs(g[s] - ref) <= bound), (s, np.max(np.abs(g[s] - ref) - bound))
    assert abs(wsum.item() - wv.sum()) < 1e-6 * wv.sum()
    plan.close()


def test_grid_assign_rejects_out_of_range():
    say("assign-out-of-range")
    n = 16
    plan = B.Plan(n=n, box=100.0, nbins=1, k0=1.0, dk=1.0)
    ux = np.array([1.0, 16.0, 3.0], np.float32)  # 16.0 is outside [0, 16)
    grids = torch.zeros((1, n, n, n), dtype=torch.float32, device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    B.bsp_grid_assign(plan.handle, dev(ux), dev(ux), dev(ux), None, 3, grids, wsum)
    with pytest.raises(B.BspError) as e:
        plan.sync()
    assert e.value.status == 6
    assert abs(grids.sum().item() - 2.0) < 1e-6


def test_grid_assign_empty_catalogue():
    """Zero particles: both assignment paths leave the grids and the weight sum alone."""
    for tiled in (False, True):
        say("assign-empty", tiled)
        n = 32
        plan = B.Plan(n=n, box=100.0, nbins=1, k0=1.0, dk=1.0, interlace=1, workspace=tiled)
        grids = torch.full((2, n, n, n), 0.5, dtype=torch.float32, device=DEV)
        wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
        e = torch.zeros(1, dtype=torch.float32, device=DEV)
        B.bsp_grid_assign(plan.handle, e, e, e, None, 0, grids, wsum)
        plan.sync()
        assert bool(torch.all(grids == 0.5)) and wsum.item() == 0.0
        plan.close()


def test_whole_path_rejects_empty_catalogue():
    plan = B.Plan(n=32, box=100.0, nbins=2, k0=2.0, dk=2.0)
    e = torch.zeros(1, dtype=torch.float32, device=DEV)
    Bt = torch.zeros((1, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(B.BspError):
        B.bsp_bispectrum_multipoles(plan.handle, e, e, e, None, 0, B.BSP_FP32, Bt)
    plan.close()


def test_plan_rejects_wrapping_triangles():
    """Shells up to |n| = 13 on a 32-point grid: closed triangles of the largest
    shells would wrap around (3 c >= N'), so the plan is refused."""
    with pytest.raises(B.BspError) as e:
        B.Plan(n=32, box=100.0, nbins=6, k0=2.0, dk=2.0)
    assert e.value.status == 3


# ---------------------------------------------------------------- LOS moments

def _catalogue(n, npart, seed, clustered=True):
    if clustered:
        wl = C.Workload("t", n, n, 200.0, npart, -1.5, 0.5, 0.5, 1, 1, 0, 4, 4, 2.0, 3, 10, seed)
        return C.lognormal_catalogue(wl, observer=np.array([-300.0, -200.0, -250.0]))
    return C.uniform_catalogue(n, npart, seed)


@pytest.mark.parametrize("los,interlace,lmax", [(0, 0, 4), (1, 0, 4), (1, 1, 4), (1, 1, 2), (0, 1, 0)])
def test_los_moments_against_oracle(los, interlace, lmax):
    say("los", los, interlace, lmax)
    n = 32
    obs = np.array([-300.0, -200.0, -250.0])
    u = _catalogue(n, 30000, 11)
    plan = B.Plan(n=n, box=200.0, nbins=4, k0=2.0, dk=2.0, lmax=lmax, interlace=interlace, los=los,
                  observer=obs)
    info = plan.info
    grids = torch.zeros((1 + interlace, n, n, n), dtype=torch.float32, device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    B.bsp_grid_assign(plan.handle, dev(u[0]), dev(u[1]), dev(u[2]), None, u[0].size, grids, wsum)
    dl = plan.spectrum_buffer()
    B.bsp_los_moments(plan.handle, grids, wsum, dl)
    plan.sync()
    got = gpu_cube_to_numpy(dl, info.nl, info.spec_elems)
    spec, _ = O.spectrum_from_catalogue(*u, n, lmax, obs if los else None, window=1, interlace=interlace)
    for li in range(info.nl):
        idx, vals, _ = compact_to_half(got[li], n, info.c, info.cz, info.n2max)
        ref = spec[li][idx]
        ref = np.where((idx[0] == 0) & (idx[1] == 0) & (idx[2] == 0), 0, ref)
        e = rel_norm(np.stack([vals.real, vals.imag]), np.stack([ref.real, ref.imag]))
        say("  l", 2 * li, "err", e)
        assert e < 1e-5, (li, e)


@pytest.mark.parametrize("los,interlace,lmax", [(0, 0, 4), (1, 1, 4), (1, 0, 2)])
def test_power_multipoles_against_oracle(los, interlace, lmax):
    """eq. (PowSpecMultipole) from the LOS moment spectra of a clustered
    redshift-space catalogue, against the FP64 oracle (bins of 2 k_f)."""
    say("power-multipoles", los, interlace, lmax)
    n, box, k0, dk, nb = 32, 200.0, 2.0, 2.0, 5
    obs = np.array([-300.0, -200.0, -250.0])
    u = _catalogue(n, 30000, 13)
    plan = B.Plan(n=n, box=box, nbins=nb, k0=k0, dk=dk, lmax=lmax, interlace=interlace, los=los, observer=obs)
    info = plan.info
    grids = torch.zeros((1 + interlace, n, n, n), dtype=torch.float32, device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    B.bsp_grid_assign(plan.handle, dev(u[0]), dev(u[1]), dev(u[2]), None, u[0].size, grids, wsum)
    dl = plan.spectrum_buffer()
    B.bsp_los_moments(plan.handle, grids, wsum, dl)
    P = torch.zeros((info.nl, nb), dtype=torch.float64, device=DEV)
    B.bsp_power_multipoles(plan.handle, dl, P)
    plan.sync()
    got = P.cpu().numpy()
    spec, _ = O.spectrum_from_catalogue(*u, n, lmax, obs if los else None, window=1, interlace=interlace)
    ref, _ = O.power_multipoles(spec, n, k0, dk, nb, box)
    s0 = np.linalg.norm(ref[0])
    for li in range(info.nl):
        e = np.linalg.norm(got[li] - ref[li]) / max(np.linalg.norm(ref[li]), 0.01 * s0)
        say("  l", 2 * li, "err", e)
        assert e < 1e-5, (li, e)
    plan.close()


def test_power_multipoles_rejects_null():
    plan = B.Plan(n=16, box=100.0, nbins=2, k0=2.0, dk=2.0)
    P = torch.zeros((1, 2), dtype=torch.float64, device=DEV)
    with pytest.raises(B.BspError):
        B.bsp_power_multipoles(plan.handle, None, P)
    plan.close()


@pytest.mark.parametrize("n,nr,los,interlace,nb,square,k0", [(32, 32, 1, 1, 5, "shells", 2.0),
                                                               (32, 16, 0, 0, 2, "shells", 2.0),
                                                               (32, 32, 1, 1, 4, "ball", 3.0),
                                                               (32, 16, 0, 0, 2, "ball", 3.0)])
def test_skew_spectra_against_oracle(n, nr, los, interlace, nb, square, k0):
    """Skew-spectrum multipoles (Sec. 3.2) from the LOS moment spectra of a
    clustered redshift-space catalogue, against the FP64 oracle; the squared
    monopole on the union of the shells, or on the whole ball of the band
    (k0 = 3 leaves a gap below the first shell, so the two differ)."""
    say("skew-spectra", n, nr, los, interlace, nb, square)
    box, dk = 200.0, 2.0
    obs = np.array([-300.0, -200.0, -250.0])
    u = _catalogue(n, 30000, 17)
    plan = B.Plan(n=n, n_reduce=nr, box=box, nbins=nb, k0=k0, dk=dk, lmax=4, interlace=interlace, los=los,
                  observer=obs)
    info = plan.info
    grids = torch.zeros((1 + interlace, n, n, n), dtype=torch.float32, device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    B.bsp_grid_assign(plan.handle, dev(u[0]), dev(u[1]), dev(u[2]), None, u[0].size, grids, wsum)
    dl = plan.spectrum_buffer()
    B.bsp_los_moments(plan.handle, grids, wsum, dl)
    S = torch.zeros((info.nl, nb), dtype=torch.float64, device=DEV)
    B.bsp_skew_spectra(plan.handle, dl, S, B.BSP_SKEW_BALL if square == "ball" else 0)
    plan.sync()
    got = S.cpu().numpy()
    spec, _ = O.spectrum_from_catalogue(*u, n, 4, obs if los else None, window=1, interlace=interlace)
    ref, _ = O.skew_spectra(spec, n, nr, k0, dk, nb, box, square)
    if square == "ball":
        other, _ = O.skew_spectra(spec, n, nr, k0, dk, nb, box, "shells")
        assert np.linalg.norm(other - ref) > 1e-3 * np.linalg.norm(ref)
    s0 = np.linalg.norm(ref[0])
    for li in range(info.nl):
        e = np.linalg.norm(got[li] - ref[li]) / max(np.linalg.norm(ref[li]), 0.01 * s0)
        say("  l", 2 * li, "err", e)
        assert e < 1e-5, (li, e)
    plan.close()


def test_skew_spectra_rejects_null():
    plan = B.Plan(n=16, box=100.0, nbins=2, k0=2.0, dk=2.0)
    S = torch.zeros((1, 2), dtype=torch.float64, device=DEV)
    with pytest.raises(B.BspError):
        B.bsp_skew_spectra(plan.handle, None, S)
    dl = plan.spectrum_buffer()
    with pytest.raises(B.BspError):
        B.bsp_skew_spectra(plan.handle, dl, S, 2)
    plan.close()


@pytest.mark.parametrize("n,s,los,window,nb", [(32, 2, 1, 1, 5), (64, 4, 0, 0, 5)])
def test_integrated_bispectrum_against_oracle(n, s, los, window, nb):
    """Integrated bispectrum multipoles (Sec. 3.4) of a clustered catalogue's
    density grid, against the FP64 oracle: per-sub-volume multipoles, mean
    overdensities and the average iB."""
    say("integrated-bispectrum", n, s, los, window)
    box, k0, dk = 200.0, 1.0, 1.0
    obs = np.array([-300.0, -200.0, -250.0])
    u = _catalogue(n, 40000, 19)
    plan = B.Plan(n=n, box=box, nbins=2, k0=2.0, dk=2.0, lmax=4, window=window, los=los, observer=obs)
    info = plan.info
    grids = torch.zeros((1, n, n, n), dtype=torch.float32, device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    B.bsp_grid_assign(plan.handle, dev(u[0]), dev(u[1]), dev(u[2]), None, u[0].size, grids, wsum)
    ns = s ** 3
    iB = torch.zeros((info.nl, nb), dtype=torch.float64, device=DEV)
    Ps = torch.zeros((ns, info.nl, nb), dtype=torch.float64, device=DEV)
    db = torch.zeros(ns, dtype=torch.float64, device=DEV)
    B.bsp_integrated_bispectrum(plan.handle, grids, wsum, s, k0, dk, nb, iB, Ps, db)
    plan.sync()
    rho = O.assign(*u, n, None, window, 0.0)
    delta = O.density_contrast(rho, float(wsum.item()))
    riB, rP, rdb, _ = O.integrated_bispectrum(delta, s, 4, obs if los else None, window, box, k0, dk, nb)
    gP, gdb, giB = Ps.cpu().numpy(), db.cpu().numpy(), iB.cpu().numpy()
    assert np.max(np.abs(gdb - rdb)) < 1e-5 * np.sqrt(np.mean(rdb ** 2)) + 1e-7
    for li in range(info.nl):
        e = np.linalg.norm(gP[:, li] - rP[:, li]) / max(np.linalg.norm(rP[:, li]), 0.01 * np.linalg.norm(rP[:, 0]))
        scale = np.linalg.norm(np.abs(rP[:, li]).T @ np.abs(rdb)) / ns
        ei = np.linalg.norm(giB[li] - riB[li]) / scale
        say("  l", 2 * li, "P err", e, "iB err / term scale", ei)
        assert e < 1e-5 and ei < 1e-5, (li, e, ei)
    plan.close()


@pytest.mark.parametrize("n,s,window,lmax", [(32, 2, 1, 4), (64, 2, 1, 4), (64, 4, 0, 2)])
def test_integrated_bispectrum_local_los_against_oracle(n, s, window, lmax):
    """The integrated bispectrum with the line of sight varying inside each
    sub-volume (eq. PowSpecMultipole per sub-volume) against the FP64 oracle;
    the l = 0 parts equal those of the one-LOS reading."""
    say("integrated-bispectrum local LOS", n, s, window, lmax)
    box, k0, dk, nb = 200.0, 1.0, 1.0, 5
    obs = np.array([-30.0, -20.0, -25.0]) * n / 32  # near: x_hat turns by tens of degrees over a sub-volume
    u = _catalogue(n, 40000, 23)
    plan = B.Plan(n=n, box=box, nbins=2, k0=2.0, dk=2.0, lmax=lmax, window=window, los=1, observer=obs)
    info = plan.info
    grids = torch.zeros((1, n, n, n), dtype=torch.float32, device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    B.bsp_grid_assign(plan.handle, dev(u[0]), dev(u[1]), dev(u[2]), None, u[0].size, grids, wsum)
    ns = s ** 3
    out = {}
    for flags in (0, B.BSP_IB_LOCAL_LOS):
        iB = torch.zeros((info.nl, nb), dtype=torch.float64, device=DEV)
        Ps = torch.zeros((ns, info.nl, nb), dtype=torch.float64, device=DEV)
        db = torch.zeros(ns, dtype=torch.float64, device=DEV)
        B.bsp_integrated_bispectrum(plan.handle, grids, wsum, s, k0, dk, nb, iB, Ps, db, flags)
        plan.sync()
        out[flags] = (iB.cpu().numpy(), Ps.cpu().numpy(), db.cpu().numpy())
    rho = O.assign(*u, n, None, window, 0.0)
    delta = O.density_contrast(rho, float(wsum.item()))
    riB, rP, rdb, _ = O.integrated_bispectrum_local_los(delta, s, lmax, obs, window, box, k0, dk, nb)
    giB, gP, gdb = out[B.BSP_IB_LOCAL_LOS]
    assert np.max(np.abs(gdb - rdb)) < 1e-5 * np.sqrt(np.mean(rdb ** 2)) + 1e-7
    for li in range(info.nl):
        e = np.linalg.norm(gP[:, li] - rP[:, li]) / max(np.linalg.norm(rP[:, li]), 0.01 * np.linalg.norm(rP[:, 0]))
        scale = np.linalg.norm(np.abs(rP[:, li]).T @ np.abs(rdb)) / ns
        ei = np.linalg.norm(giB[li] - riB[li]) / scale
        say("  l", 2 * li, "P err", e, "iB err / term scale", ei)
        assert e < 1e-5 and ei < 1e-5, (li, e, ei)
    # the monopole does not depend on the line of sight; the l > 0 parts do
    p1 = out[0][1]
    assert np.linalg.norm(gP[:, 0] - p1[:, 0]) < 1e-5 * np.linalg.norm(p1[:, 0])
    assert np.linalg.norm(gP[:, 1] - p1[:, 1]) > 1e-3 * np.linalg.norm(p1[:, 1])
    plan.close()


def test_integrated_bispectrum_local_los_plane_parallel_and_flags():
    """Plane-parallel plans have one line of sight: both readings give the same
    values (up to the order of the FP64 atomic shell sums). An unknown flag bit
    is rejected."""
    n, s, nb = 32, 2, 4
    u = _catalogue(n, 20000, 29)
    plan = B.Plan(n=n, box=150.0, nbins=2, k0=2.0, dk=2.0, lmax=4, los=0)
    grids = torch.zeros((1, n, n, n), dtype=torch.float32, device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    B.bsp_grid_assign(plan.handle, dev(u[0]), dev(u[1]), dev(u[2]), None, u[0].size, grids, wsum)
    res = []
    for flags in (0, B.BSP_IB_LOCAL_LOS):
        iB = torch.zeros((3, nb), dtype=torch.float64, device=DEV)
        B.bsp_integrated_bispectrum(plan.handle, grids, wsum, s, 1.0, 1.0, nb, iB, None, None, flags)
        plan.sync()
        res.append(iB.cpu().numpy())
    assert np.allclose(res[0], res[1], rtol=1e-12, atol=1e-12 * np.abs(res[0]).max())
    with pytest.raises(B.BspError):
        B.bsp_integrated_bispectrum(plan.handle, grids, wsum, s, 1.0, 1.0, nb, iB, None, None, 2)
    plan.close()


def test_integrated_bispectrum_rejects_observer_at_a_subvolume_centre():
    """The one line of sight of a sub-volume points at its centre: an observer
    there has none (BSP_ERR_ARG); the local reading needs only the nodes."""
    n, s, nb = 32, 2, 4
    plan = B.Plan(n=n, box=150.0, nbins=2, k0=2.0, dk=2.0, lmax=2, los=1, observer=np.array([7.5, 7.5, 7.5]))
    g = torch.zeros((1, n, n, n), dtype=torch.float32, device=DEV)
    iB = torch.zeros((2, nb), dtype=torch.float64, device=DEV)
    with pytest.raises(B.BspError) as e:
        B.bsp_integrated_bispectrum(plan.handle, g, None, s, 1.0, 1.0, nb, iB)
    assert e.value.status == 1
    B.bsp_integrated_bispectrum(plan.handle, g, None, s, 1.0, 1.0, nb, iB, None, None, B.BSP_IB_LOCAL_LOS)
    plan.sync()
    plan.close()


def test_integrated_bispectrum_rejects_bad_geometry():
    plan = B.Plan(n=32, box=100.0, nbins=2, k0=2.0, dk=2.0)
    g = torch.zeros((1, 32, 32, 32), dtype=torch.float32, device=DEV)
    iB = torch.zeros((1, 4), dtype=torch.float64, device=DEV)
    for s, k0, dk, nb in [(3, 1.0, 1.0, 4), (4, 1.0, 1.0, 4), (2, 1.0, 1.0, 8), (2, 1.2, 1.0, 2)]:
        with pytest.raises(B.BspError):
            B.bsp_integrated_bispectrum(plan.handle, g, None, s, k0, dk, nb, iB)
    plan.close()


@pytest.mark.parametrize("prec,tol", [(B.BSP_FP32, 1e-5), (B.BSP_BF16X3, 1e-3)])
def test_bispectrum_full_against_oracle(prec, tol):
    """B^(l1 l2 l3) for every combination (one LOS moment per side) against the
    FP64 oracle, each against its own norm (floored at 1% of the monopole's);
    B^(l00) also against the whole path's B^l. The path is reproducible, so
    the errors are the same on every run."""
    say("bispectrum-full", prec)
    n, box, k0, dk, nb = 32, 200.0, 2.0, 2.0, 4
    obs = np.array([-300.0, -200.0, -250.0])
    u = _catalogue(n, 30000, 23)
    plan = B.Plan(n=n, box=box, nbins=nb, k0=k0, dk=dk, lmax=4, interlace=1, los=1, observer=obs)
    plan.precompute()
    info = plan.info
    grids = torch.zeros((2, n, n, n), dtype=torch.float32, device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    B.bsp_grid_assign(plan.handle, dev(u[0]), dev(u[1]), dev(u[2]), None, u[0].size, grids, wsum)
    dl = plan.spectrum_buffer()
    B.bsp_los_moments(plan.handle, grids, wsum, dl)
    nl, ntri = info.nl, info.ntri
    Bf = torch.zeros((nl ** 3, ntri), dtype=torch.float64, device=DEV)
    B.bsp_bispectrum_full(plan.handle, dl, prec, Bf)
    Bl = torch.zeros((nl, ntri), dtype=torch.float64, device=DEV)
    ux, uy, uz = dev(u[0]), dev(u[1]), dev(u[2])
    B.bsp_bispectrum_multipoles(plan.handle, ux, uy, uz, None, u[0].size, prec, Bl, None, None, None, None, None)
    plan.sync()
    got, path = Bf.cpu().numpy(), Bl.cpu().numpy()
    tris = [tuple(int(v) for v in t) for t in plan.tri]
    counts = plan.counts.copy()
    spec, _ = O.spectrum_from_catalogue(*u, n, 4, obs, window=1, interlace=1)
    _, combos, T = O.binned_triple_sums_full(spec, n, n, k0, dk, nb, tris)
    ref = O.binned_bispectrum(T, counts, n, n, box)
    s0 = np.linalg.norm(ref[0])
    worst = 0.0
    for ci in range(nl ** 3):
        e = np.linalg.norm(got[ci] - ref[ci]) / max(np.linalg.norm(ref[ci]), 0.01 * s0)
        say("  combination", combos[ci], "err", e)
        worst = max(worst, e)
        assert e < tol, (combos[ci], e)
    # two GPU results, each within tol of the oracle: their difference is bounded by 2 tol
    for li in range(nl):
        ci = combos.index((li, 0, 0))
        assert np.linalg.norm(got[ci] - path[li]) <= 2 * tol * max(np.linalg.norm(path[li]), 0.01 * s0), li
    say("  worst combination error", worst)
    plan.close()


def test_grid_entry_against_oracle():
    say("grid-entry")
    n = 32
    d = rng(12).standard_normal((n, n, n))
    obs = np.array([-40.0, -30.0, -55.0])
    plan = B.Plan(n=n, box=200.0, nbins=4, k0=2.0, dk=2.0, lmax=4, los=1, observer=obs)
    info = plan.info
    dl = plan.spectrum_buffer()
    B.bsp_grid_entry(plan.handle, dev(d), dl)
    plan.sync()
    got = gpu_cube_to_numpy(dl, info.nl, info.spec_elems)
    spec = O.spectrum_from_field([d], [0.0], n, 4, obs, None)
    for li in range(3):
        idx, vals, _ = compact_to_half(got[li], n, info.c, info.cz, info.n2max)
        ref = np.where((idx[0] == 0) & (idx[1] == 0) & (idx[2] == 0), 0, spec[li][idx])
        e = rel_norm(np.stack([vals.real, vals.imag]), np.stack([ref.real, ref.imag]))
        say("  l", 2 * li, "err", e)
        assert e < 2e-5, (li, e)


# ---------------------------------------------------------------- filtered fields

def test_filter_fields_against_oracle():
    say("filter")
    n, nr = 32, 32
    k0, dk, nb, P = 2.0, 2.0, 4, 3
    box = 200.0
    d = rng(13).standard_normal((n, n, n))
    spec = O.spectrum_from_field([d], [0.0], n, 2, None, None)
    wl = C.Workload("t", n, nr, box, 10000, -1.5, 0.5, 0.5, 0, 1, 0, 2, nb, dk, P, 10, 1)
    n2len = 3 * n * n
    pf = pfid_table(wl, n2len)
    plan = B.Plan(n=n, box=box, nbins=nb, k0=k0, dk=dk, lmax=2, P=P, nmodes=4, pfid=pf)
    info = plan.info
    cube = np.stack([half_to_compact(s, n, info.c, info.cz, info.n2max) for s in spec])
    dl = dev(np.stack([cube.real, cube.imag], -1).reshape(info.nl, -1, 2))
    filt = [(li, 0, b) for li in range(2) for b in range(nb)] + [(li, 1, p) for li in range(2) for p in range(P)]
    fields = torch.zeros((len(filt), nr, nr, nr), dtype=torch.float32, device=DEV)
    B.bsp_filter_fields(plan.handle, dl, filt, fields)
    plan.sync()
    got = fields.cpu().numpy()
    n2 = O.n2_grid_half(nr)
    bins = O.bin_of_n2(n2, k0, dk, nb)
    kf = 2 * math.pi / box
    M = [O.modal_fields(s, n, nr, P, k0 - dk / 2, k0 + (nb - 0.5) * dk, kf, pf) * n ** 3 for s in spec]
    for i, (li, kind, idx) in enumerate(filt):
        if kind == 0:
            ref = O.shell_field(spec[li], bins == idx, nr)
        else:
            ref = M[li][idx].reshape(nr, nr, nr)
        assert rel_norm(got[i], ref) < 1e-5, (li, kind, idx)


# ---------------------------------------------------------------- triple reduction

@pytest.mark.parametrize("prec,tol", [(0, 1e-5), (1, 1e-4), (2, 1e-5)])
@pytest.mark.parametrize("K", [64 * 64 * 64, 50_011])
def test_triple_reduce_definition(prec, tol, K):
    say("reduce", prec, K)
    r = rng(20 + prec)
    nf = 21
    F = r.standard_normal((nf, K)).astype(np.float32) * r.uniform(0.5, 3e3, (nf, 1)).astype(np.float32)
    pairs = np.array([(a, b) for a in range(nf) for b in range(a, nf)][::3], np.int32)
    thirds = np.arange(0, nf, 1, dtype=np.int32)[::-1].copy()
    need = (r.uniform(size=(len(pairs), len(thirds))) < 0.4).astype(np.uint8)
    plan = B.Plan(n=16, box=100.0, nbins=1, k0=1.0, dk=1.0, workspace=False)
    ws = torch.empty(1 << 28, dtype=torch.uint8, device=DEV)
    B.bsp_set_workspace(plan.handle, ws, ws.numel())
    T = torch.zeros((len(pairs), len(thirds)), dtype=torch.float64, device=DEV)
    B.bsp_triple_reduce(plan.handle, dev(F), nf, K, pairs, thirds, need, prec, T)
    plan.sync()
    got = T.cpu().numpy()
    F64 = F.astype(np.float64)
    ref = np.array([[np.dot(F64[a] * F64[b], F64[t]) for t in thirds] for a, b in pairs])
    # the sums are noise dominated: compare with the scale of the summed terms
    scale = np.sqrt(np.array([[np.dot((F64[a] * F64[b]) ** 2, F64[t] ** 2) for t in thirds] for a, b in pairs]))
    err = np.abs(got - ref) / scale
    assert np.sqrt(np.mean(err[need == 1] ** 2)) < tol, np.sqrt(np.mean(err[need == 1] ** 2))
    # the reduction works in 16 x 16 tiles of its own pair order: an unneeded
    # entry is 0 (outside every computed tile) or computed like a needed one
    assert np.all((got[need == 0] == 0) | (err[need == 0] < 50 * tol))


def test_triple_reduce_bf16x1_error_study():
    """BSP_BF16X1 keeps only the bf16 hi parts: each term carries the roundings
    of its pair product and its third to 8-bit significands, each at most 2^-9
    relative and about 2^-9 / sqrt(3) in rms. These errors are zero-mean and
    independent between terms, so the error against the definition is near
    sqrt(2/3) 2^-9 = 1.6e-3 of the summed-term scale (below 2^-8) and far above
    that of the hi+lo path on the same input."""
    say("reduce bf16x1")
    r = rng(77)
    nf, K = 21, 50_011
    F = r.standard_normal((nf, K)).astype(np.float32) * r.uniform(0.5, 3e3, (nf, 1)).astype(np.float32)
    pairs = np.array([(a, b) for a in range(nf) for b in range(a, nf)][::3], np.int32)
    thirds = np.arange(nf, dtype=np.int32)
    plan = B.Plan(n=16, box=100.0, nbins=1, k0=1.0, dk=1.0, workspace=False)
    ws = torch.empty(1 << 28, dtype=torch.uint8, device=DEV)
    B.bsp_set_workspace(plan.handle, ws, ws.numel())
    F64 = F.astype(np.float64)
    ref = np.array([[np.dot(F64[a] * F64[b], F64[t]) for t in thirds] for a, b in pairs])
    scale = np.sqrt(np.array([[np.dot((F64[a] * F64[b]) ** 2, F64[t] ** 2) for t in thirds] for a, b in pairs]))
    err = {}
    for prec in (B.BSP_BF16X1, B.BSP_BF16X3):
        T = torch.zeros((len(pairs), len(thirds)), dtype=torch.float64, device=DEV)
        B.bsp_triple_reduce(plan.handle, dev(F), nf, K, pairs, thirds, None, prec, T)
        plan.sync()
        err[prec] = np.sqrt(np.mean((np.abs(T.cpu().numpy() - ref) / scale) ** 2))
    assert 2e-4 < err[B.BSP_BF16X1] < 2.0 ** -8, err
    assert err[B.BSP_BF16X1] > 20 * err[B.BSP_BF16X3], err
    plan.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-5), (1, 1e-4), (2, 1e-5)])
def test_triple_reduce_many_row_tiles(prec, tol):
    # 120 fields, every pair a <= b (454 row tiles) and a banded need pattern:
    # the schedules span several workgroup groups and dense per-wave blocks
    say("reduce many", prec)
    r = rng(40 + prec)
    nf, K = 120, 4096 + 37
    F = r.standard_normal((nf, K)).astype(np.float32) * r.uniform(0.5, 3e3, (nf, 1)).astype(np.float32)
    pairs = np.array([(a, b) for a in range(nf) for b in range(a, nf)], np.int32)
    thirds = np.arange(nf, dtype=np.int32)
    band = np.abs(pairs[:, :1] + pairs[:, 1:2] - 2 * thirds[None, :]) < 24
    need = (band & (r.uniform(size=band.shape) < 0.7)).astype(np.uint8)
    plan = B.Plan(n=16, box=100.0, nbins=1, k0=1.0, dk=1.0, workspace=False)
    ws = torch.empty(1 << 29, dtype=torch.uint8, device=DEV)
    B.bsp_set_workspace(plan.handle, ws, ws.numel())
    T = torch.zeros((len(pairs), len(thirds)), dtype=torch.float64, device=DEV)
    B.bsp_triple_reduce(plan.handle, dev(F), nf, K, pairs, thirds, need, prec, T)
    plan.sync()
    got = T.cpu().numpy()
    F64 = F.astype(np.float64)
    P2 = F64[pairs[:, 0]] * F64[pairs[:, 1]]
    ref = P2 @ F64[thirds].T
    scale = np.sqrt((P2 ** 2) @ (F64[thirds] ** 2).T)
    err_all = np.abs(got - ref) / scale
    err = err_all[need == 1]
    assert np.sqrt(np.mean(err ** 2)) < tol and err.max() < 50 * tol, (np.sqrt(np.mean(err ** 2)), err.max())
    # unneeded entries: 0, or computed in a tile some needed entry shares
    assert np.all((got[need == 0] == 0) | (err_all[need == 0] < 50 * tol))


# ---------------------------------------------------------------- geometry precompute

def _plan_c1(**kw):
    wl = C.workload("c1_64")
    n2len = 3 * wl.n ** 2
    pf = pfid_table(wl, n2len)
    args = dict(n=wl.n, box=wl.box, nbins=wl.nbins, k0=wl.k0, dk=wl.dk, lmax=0, window=1, interlace=0, los=0,
                P=wl.P, nmodes=wl.nmodes, pfid=pf)
    args.update(kw)
    return wl, pf, B.Plan(**args)


def test_precompute_counts_gram_shot_noise():
    say("precompute-c1")
    wl, pf, plan = _plan_c1()
    plan.precompute()
    path = __file__.replace("test_gpu_parity.py", "golden/counts_k2_d2_nb10.txt")
    gold = np.loadtxt(path, dtype=np.int64, comments="#")
    gold = gold[gold[:, 3] > 0]
    assert np.array_equal(plan.tri, gold[:, :3])
    assert np.array_equal(plan.counts, gold[:, 3])
    modes = O.modal_modes(wl.P, wl.nmodes)
    kf = 2 * math.pi / wl.box
    gam = O.gram_matrix(wl.n, modes, wl.P, wl.kmin, wl.kmax, kf, wl.box)
    assert rel_norm(plan.gamma, gam) < 1e-10
    assert rel_norm(plan.chol, np.linalg.cholesky(gam)) < 1e-9


# ---------------------------------------------------------------- end to end

def _check_modal(got, ref, tol, nl, plan=None):
    """Modal coefficients: the stated tolerance applies to alpha, the
    coefficients on the orthonormalised kept modes; the kept modes and their
    order must match the oracle's exactly. beta = L^-T alpha is reported with
    cond(L) of the kept modes, which bounds how much more it can be off."""
    kept = ref["modal_kept"]
    if plan is not None:
        k = np.asarray(plan.kept)
        assert np.array_equal(k[:len(kept)], kept) and np.all(k[len(kept):] == -1), (k, kept)
        assert plan.info.modal_rank == len(kept)
    g = ref["gamma"][np.ix_(kept, kept)]
    kL = np.linalg.cond(np.linalg.cholesky(g))
    for li in range(nl):
        ea = rel_norm(got["alpha"][li], ref["alpha"][li])
        eb = rel_norm(got["beta"][li], ref["beta"][li])
        print(f"[modal] l={2 * li} kept {len(kept)} err alpha={ea:.2e} beta={eb:.2e} cond(L)={kL:.1f}", flush=True)
        assert ea < tol, (li, ea)
        assert eb < max(tol, kL * tol), (li, eb)


def _run_gpu(plan, u, prec, nl, nmodes):
    ntri = plan.info.ntri
    Bt = torch.zeros((nl, ntri), dtype=torch.float64, device=DEV)
    B0 = torch.zeros(ntri, dtype=torch.float64, device=DEV)
    Pb = torch.zeros(plan.geom.nbins, dtype=torch.float64, device=DEV)
    bn = torch.zeros((nl, max(nmodes, 1)), dtype=torch.float64, device=DEV)
    al = torch.zeros_like(bn)
    be = torch.zeros_like(bn)
    B.bsp_bispectrum_multipoles(plan.handle, dev(u[0]), dev(u[1]), dev(u[2]), None, u[0].size, prec, Bt, B0, Pb,
                                bn if nmodes else None, al if nmodes else None, be if nmodes else None)
    plan.sync()
    return {k: v.cpu().numpy() for k, v in dict(B=Bt, B0_sub=B0, Pbar=Pb, bnum=bn, alpha=al, beta=be).items()}


@pytest.fixture(scope="module")
def c1_case():
    wl, pf, plan = _plan_c1()
    plan.precompute()
    u = C.lognormal_catalogue(wl)
    spec, wsum = O.spectrum_from_catalogue(*u, wl.n, 0, None, window=1, interlace=0)
    geo = O.Geometry(wl.n, wl.n, wl.box, 0, wl.nbins, wl.k0, wl.dk, wl.P, wl.nmodes, pf)
    ref = O.estimate(spec, geo, nbar=wsum / wl.box ** 3)
    return wl, plan, u, ref


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_end_to_end_c1_monopole(c1_case, prec):
    say("e2e-c1", prec)
    wl, plan, u, ref = c1_case
    got = _run_gpu(plan, u, prec, 1, wl.nmodes)
    assert np.array_equal(plan.tri, ref["tris"])
    assert np.array_equal(plan.counts, ref["counts"])
    tb, tbeta = (1e-5, 1e-5) if prec == 0 else (1e-3, 1e-4)
    assert rel_norm(got["Pbar"], ref["Pbar"]) < 1e-5
    assert rel_norm(got["B"], ref["B"]) < tb
    assert rel_norm(got["B0_sub"], ref["B0_sub"]) < tb
    assert rel_norm(got["bnum"][0], ref["bnum_sub0"]) < tbeta
    _check_modal(got, ref, tbeta, 1, plan)


@pytest.fixture(scope="module")
def los_case():
    n, box = 64, 400.0
    wl = C.Workload("los64", n, n, box, 120_000, -1.5, 0.6, 0.6, 1, 1, 1, 4, 6, 3.0, 4, 20, 77)
    obs = C.observer_grid_units(wl)
    pf = pfid_table(wl, 3 * n * n)
    plan = B.Plan(n=n, box=box, nbins=wl.nbins, k0=wl.k0, dk=wl.dk, lmax=4, window=1, interlace=1, los=1,
                  observer=obs, P=wl.P, nmodes=wl.nmodes, pfid=pf, drop_tol=MODAL_DROP_TOL)
    plan.precompute()
    u = C.lognormal_catalogue(wl)
    spec, wsum = O.spectrum_from_catalogue(*u, n, 4, obs, window=1, interlace=1)
    geo = O.Geometry(n, n, box, 4, wl.nbins, wl.k0, wl.dk, wl.P, wl.nmodes, pf)
    ref = O.estimate(spec, geo, nbar=wsum / box ** 3, modal_tol=MODAL_DROP_TOL)
    return wl, plan, u, ref


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_end_to_end_varying_los_interlaced(los_case, prec):
    say("e2e-los", prec)
    wl, plan, u, ref = los_case
    got = _run_gpu(plan, u, prec, 3, wl.nmodes)
    assert np.array_equal(plan.counts, ref["counts"])
    tb, tbeta = (1e-5, 1e-5) if prec == 0 else (1e-3, 1e-4)
    for li in range(3):
        assert rel_norm(got["B"][li], ref["B"][li]) < tb, li
    _check_modal(got, ref, tbeta, 3, plan)
    assert rel_norm(got["B0_sub"], ref["B0_sub"]) < tb
    assert rel_norm(got["Pbar"], ref["Pbar"]) < 1e-5


@pytest.fixture(scope="module")
def n96_case():
    """96 points per side (z lines straddle waves: the transforms keep their
    workgroup barriers), varying LOS, interlacing, l <= 2, 8 shells of 3 k_f."""
    n, box = 96, 300.0
    wl = C.Workload("n96", n, n, box, 150_000, -1.5, 0.6, 0.6, 1, 1, 1, 2, 8, 3.0, 0, 0, 96)
    obs = C.observer_grid_units(wl)
    plan = B.Plan(n=n, box=box, nbins=wl.nbins, k0=wl.k0, dk=wl.dk, lmax=2, window=1, interlace=1, los=1,
                  observer=obs)
    plan.precompute()
    u = C.lognormal_catalogue(wl)
    spec, wsum = O.spectrum_from_catalogue(*u, n, 2, obs, window=1, interlace=1)
    geo = O.Geometry(n, n, box, 2, wl.nbins, wl.k0, wl.dk)
    ref = O.estimate(spec, geo, nbar=wsum / box ** 3)
    return wl, plan, u, ref


@pytest.mark.parametrize("prec", [0, 1])
def test_end_to_end_n96(n96_case, prec):
    say("e2e-n96", prec)
    wl, plan, u, ref = n96_case
    got = _run_gpu(plan, u, prec, 2, 0)
    assert np.array_equal(plan.counts, ref["counts"])
    tb = 1e-5 if prec == 0 else 1e-3
    for li in range(2):
        assert rel_norm(got["B"][li], ref["B"][li]) < tb, li
    assert rel_norm(got["Pbar"], ref["Pbar"]) < 1e-5
    assert rel_norm(got["B0_sub"], ref["B0_sub"]) < tb


@pytest.mark.parametrize("n", [64, 128])
def test_whole_path_reproducible(n):
    """Two runs of the whole path on one catalogue give bit-identical B_l,
    B0sub's monopole part, modal numerators, alpha and beta: the assignment sums
    in fixed point (global atomics below 512 tiles, the tiled kernel from 128 a
    side) and the reduction partials are combined in a fixed order."""
    say("repro", n)
    box = 500.0
    wl = C.Workload(f"repro{n}", n, n, box, 150_000, -1.5, 0.6, 0.6, 1, 1, 1, 4, 6, 3.0, 4, 20, 900 + n)
    obs = C.observer_grid_units(wl)
    pf = pfid_table(wl, 3 * n * n)
    plan = B.Plan(n=n, box=box, nbins=wl.nbins, k0=wl.k0, dk=wl.dk, lmax=4, window=1, interlace=1, los=1,
                  observer=obs, P=wl.P, nmodes=wl.nmodes, pfid=pf, drop_tol=MODAL_DROP_TOL)
    plan.precompute()
    u = C.lognormal_catalogue(wl)
    for prec in (B.BSP_FP32, B.BSP_BF16X3):
        a = _run_gpu(plan, u, prec, 3, wl.nmodes)
        b = _run_gpu(plan, u, prec, 3, wl.nmodes)
        for k in ("B", "bnum", "alpha", "beta"):
            assert np.array_equal(a[k], b[k]), (prec, k)
    plan.close()

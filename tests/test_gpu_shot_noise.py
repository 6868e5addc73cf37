"""Poisson shot noise of the multipoles B_l through the C ABI
(bsp_shot_noise_multipoles): the ring factors the library computes once per
plan against the FP64 oracle's model on the same shell powers, SN_0 against
the whole path's B0sub, and the model on a clustered varying-LOS catalogue
against the oracle's from the same catalogue."""
import sys

import numpy as np
import pytest

import oracle as O
from synth import catalog as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1708_05303_amd as B  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print("[sn]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


OBS = np.array([-300.0, -200.0, -250.0])


def test_shot_noise_model_against_oracle():
    """Same shell powers in, the library's ring factors (32-point rule on the
    host) against the oracle's: FP64 on both sides."""
    n, box, k0, dk, nb = 64, 400.0, 2.0, 2.0, 8
    plan = B.Plan(n=n, box=box, nbins=nb, k0=k0, dk=dk, lmax=4, los=1, interlace=1, observer=OBS).precompute()
    tris = [tuple(int(x) for x in t) for t in plan.tri]
    say("triangles", len(tris))
    r = np.random.default_rng(5)
    P = np.stack([r.uniform(50.0, 500.0, nb), r.uniform(-50.0, 200.0, nb), r.uniform(-20.0, 60.0, nb)])
    nbar = 3.1e-4
    SN = torch.zeros((3, len(tris)), dtype=torch.float64, device=DEV)
    B.bsp_shot_noise_multipoles(plan.handle, dev(P, torch.float64), nbar, SN)
    plan.sync()
    got = SN.cpu().numpy()
    ref = O.shot_noise_multipoles(P, tris, k0, dk, nbar)
    for li in range(3):
        e = float(np.abs(got[li] - ref[li]).max() / np.abs(ref[li]).max())
        say("l", 2 * li, "max rel", e)
        assert e < 1e-12, (li, e)
    with pytest.raises(B.BspError):
        B.bsp_shot_noise_multipoles(plan.handle, dev(P, torch.float64), 0.0, SN)
    plan.close()


def test_shot_noise_before_precompute_rejected():
    plan = B.Plan(n=32, box=200.0, nbins=3, k0=2.0, dk=2.0, lmax=2)
    P = torch.zeros((2, 3), dtype=torch.float64, device=DEV)
    SN = torch.zeros((2, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(B.BspError):
        B.bsp_shot_noise_multipoles(plan.handle, P, 1e-3, SN)
    plan.close()


def test_shot_noise_end_to_end():
    """A clustered redshift-space catalogue, varying LOS, interlaced CIC: the
    whole path's B_l and B0sub, the LOS moments' shell power multipoles and
    the shot-noise model, against the oracle's model from the oracle's power
    multipoles of the same catalogue (FP32 path: 1e-5); SN_0 = B_0 - B0sub."""
    n, box, k0, dk, nb = 32, 200.0, 2.0, 2.0, 5
    wl = C.Workload("t", n, n, box, 30000, -1.5, 0.5, 0.5, 1, 1, 1, 4, nb, dk, 3, 10, 13)
    u = C.lognormal_catalogue(wl, observer=OBS)
    plan = B.Plan(n=n, box=box, nbins=nb, k0=k0, dk=dk, lmax=4, los=1, interlace=1, observer=OBS).precompute()
    info = plan.info
    tris = [tuple(int(x) for x in t) for t in plan.tri]
    ux, uy, uz = (dev(a) for a in u)
    Bt = torch.zeros((3, info.ntri), dtype=torch.float64, device=DEV)
    B0s = torch.zeros(info.ntri, dtype=torch.float64, device=DEV)
    Pb = torch.zeros(nb, dtype=torch.float64, device=DEV)
    B.bsp_bispectrum_multipoles(plan.handle, ux, uy, uz, None, u[0].size, B.BSP_FP32, Bt, B0s, Pb, None, None, None)
    grids = torch.zeros((2, n, n, n), dtype=torch.float32, device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    B.bsp_grid_assign(plan.handle, ux, uy, uz, None, u[0].size, grids, wsum)
    dl = plan.spectrum_buffer()
    B.bsp_los_moments(plan.handle, grids, wsum, dl)
    P = torch.zeros((3, nb), dtype=torch.float64, device=DEV)
    B.bsp_power_multipoles(plan.handle, dl, P)
    nbar = u[0].size / box ** 3
    SN = torch.zeros((3, info.ntri), dtype=torch.float64, device=DEV)
    B.bsp_shot_noise_multipoles(plan.handle, P, nbar, SN)
    plan.sync()
    sn, b, b0s = SN.cpu().numpy(), Bt.cpu().numpy(), B0s.cpu().numpy()
    e0 = float(np.abs(sn[0] - (b[0] - b0s)).max() / np.abs(sn[0]).max())
    say("SN_0 against B_0 - B0sub", e0)
    assert e0 < 1e-10
    spec, wsum_o = O.spectrum_from_catalogue(*u, n, 4, OBS, window=1, interlace=1)
    Po, _ = O.power_multipoles(spec, n, k0, dk, nb, box)
    ref = O.shot_noise_multipoles(Po, tris, k0, dk, wsum_o / box ** 3)
    for li in range(3):
        e = float(np.linalg.norm(sn[li] - ref[li]) / np.linalg.norm(ref[li]))
        say("l", 2 * li, "SN against the oracle", e, "|SN| / |B|", float(np.linalg.norm(ref[li]) / np.linalg.norm(b[li])))
        assert e < 1e-5, (li, e)
    plan.close()

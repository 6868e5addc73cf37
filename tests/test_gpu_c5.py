"""The 1024^3 large-grid configuration: transforms of 1024 points and the whole
path with its field stacks in x-slabs (L = 2000 Mpc/h, 5e7 particles, varying
line of sight, l <= 4, 30 shells of 11 k_f, 100 modes with P = 8).

No whole-cube FP64 oracle runs at this size (one FP64 field is 8.6 GB), so:
* the r2c transform is checked on sampled modes against the oracle's DFT by
  its definition, on every mode through Parseval's identity, and by the c2r
  round trip;
* the slab precompute's triangle counts of the first two shells against the
  stored direct enumeration (tests/golden/counts_c5_k11_d11_first.txt), and
  every count's residual from an integer (below 0.5: the rounding is certain);
* the mixed path (bf16 hi+lo products) against the FP32 path on one
  catalogue: B_l within 1e-3, alpha within 1e-4 (the stated tolerances of the
  mixed path), which the slab and whole-cube paths already meet against the
  oracle at 64^3.
"""
import os
import sys
import time

import numpy as np
import pytest

import oracle as O
from synth import catalog as C
from tests.gpu_helpers import pfid_table, rel_norm

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1708_05303_amd as B  # noqa: E402

DEV = torch.device("cuda:0")
HERE = os.path.dirname(os.path.abspath(__file__))
MODAL_DROP_TOL = 1e-2


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_fft_1024_sampled_parseval_round_trip():
    n = 1024
    say("fft1024")
    plan = B.Plan(n=n, box=100.0, nbins=1, k0=1.0, dk=1.0)
    try:
        x = np.random.Generator(np.random.PCG64(1024)).standard_normal((n, n, n), dtype=np.float32)
        xi = torch.from_numpy(x).to(DEV)
        out = torch.zeros((n, n, n // 2 + 1, 2), dtype=torch.float32, device=DEV)
        B.bsp_fft_r2c(plan.handle, n, 1, xi, out)
        back = torch.zeros((n, n, n), dtype=torch.float32, device=DEV)
        B.bsp_fft_c2r(plan.handle, n, 1, out, back)
        plan.sync()
        say("  transforms done")
        sumsq = float(torch.sum(xi.double() ** 2))
        scale = np.sqrt(sumsq)  # rms size of one mode of the noise's spectrum
        # Parseval over the half spectrum (kz = 0 and n/2 once, the rest twice)
        p = out.double().pow(2).sum(-1)
        tot = 2.0 * float(p.sum()) - float(p[..., 0].sum()) - float(p[..., n // 2].sum())
        del p
        assert abs(tot / (n ** 3 * sumsq) - 1.0) < 1e-5
        # round trip: c2r(r2c(x)) = n^3 x
        err = float(torch.max(torch.abs(back.double() / n ** 3 - xi.double())))
        assert err < 1e-5 * float(torch.max(torch.abs(xi)))
        del back
        modes = np.array([(0, 0, 0), (1, 2, 3), (-5, 7, 512), (511, -512, 17), (0, 0, 512), (512, 512, 512),
                          (-1, -1, 1), (300, -200, 100), (-337, 13, 255), (8, 1000, 0), (-512, 3, 511), (77, -77, 77)])
        t0 = time.time()
        ref = O.dft_modes(x, modes)
        say(f"  oracle modes in {time.time() - t0:.1f} s")
        o = out[torch.as_tensor(modes[:, 0] % n), torch.as_tensor(modes[:, 1] % n), torch.as_tensor(modes[:, 2])]
        o = o.cpu().numpy().astype(np.float64)
        got = o[:, 0] + 1j * o[:, 1]
        e = np.abs(got - ref) / scale
        say("  sampled mode errors / rms mode", e.max())
        assert e.max() < 1e-5, e
    finally:
        plan.close()
        torch.cuda.empty_cache()  # the 1024^3 plan below takes about 180 GB


@pytest.fixture(scope="module")
def c5_plan():
    wl = C.workload("c5_1024")
    obs = C.observer_grid_units(wl)
    pf = pfid_table(wl, 3 * wl.n ** 2)
    t0 = time.time()
    plan = B.Plan(n=wl.n, box=wl.box, nbins=wl.nbins, k0=wl.k0, dk=wl.dk, lmax=4, window=1, interlace=0, los=1,
                  observer=obs, P=wl.P, nmodes=wl.nmodes, pfid=pf, drop_tol=MODAL_DROP_TOL)
    say(f"c5 plan: slab {plan.info.slab_planes} planes, workspace {plan.ws.numel() / 2 ** 30:.1f} GiB, "
        f"{time.time() - t0:.1f} s")
    t0 = time.time()
    plan.precompute()
    say(f"c5 precompute {time.time() - t0:.1f} s, {plan.info.ntri} triangles, rank {plan.info.modal_rank}, "
        f"count residual {plan.info.count_residual:.2e}")
    yield wl, plan
    plan.close()
    plan.ws = None
    torch.cuda.empty_cache()  # hand the large workspace back before the next module's plans


def test_c5_slab_precompute_counts(c5_plan):
    wl, plan = c5_plan
    assert plan.info.slab_planes == 128
    # FP64 rounding of sums whose values are of the order of the count times
    # N'^3: the residual grows with the count (about 0.1 at 3e12), and the
    # rounding is certain while it stays below 0.5
    assert plan.info.count_residual < 0.5
    gold = np.loadtxt(os.path.join(HERE, "golden", "counts_c5_k11_d11_first.txt"), dtype=np.int64, comments="#")
    tri = [tuple(t) for t in plan.tri]
    for b1, b2, b3, cnt in gold:
        assert plan.counts[tri.index((b1, b2, b3))] == cnt, (b1, b2, b3)
    assert np.all(plan.counts > 0)
    assert np.all(np.isfinite(plan.gamma))


def test_c5_mixed_against_fp32(c5_plan):
    wl, plan = c5_plan
    rng = np.random.Generator(np.random.PCG64(5000))
    u = [torch.from_numpy(C.quantise_grid_units(rng.uniform(0.0, wl.n, wl.nparticles), wl.n)).to(DEV)
         for _ in range(3)]
    nl, ntri, nm = 3, plan.info.ntri, wl.nmodes
    out = {}
    for prec in (B.BSP_FP32, B.BSP_BF16X3):
        Bt = torch.zeros((nl, ntri), dtype=torch.float64, device=DEV)
        al = torch.zeros((nl, nm), dtype=torch.float64, device=DEV)
        t0 = time.time()
        B.bsp_bispectrum_multipoles(plan.handle, u[0], u[1], u[2], None, wl.nparticles, prec, Bt, None, None, None,
                                    al, None)
        plan.sync()
        say(f"c5 whole path prec {prec}: {time.time() - t0:.2f} s")
        out[prec] = (Bt.cpu().numpy(), al.cpu().numpy())
    del u
    for li in range(nl):
        eb = rel_norm(out[B.BSP_BF16X3][0][li], out[B.BSP_FP32][0][li])
        ea = rel_norm(out[B.BSP_BF16X3][1][li], out[B.BSP_FP32][1][li])
        say(f"  l={2 * li} mixed vs FP32: B {eb:.2e} alpha {ea:.2e}")
        assert np.all(np.isfinite(out[B.BSP_FP32][0][li])) and np.all(np.isfinite(out[B.BSP_FP32][1][li]))
        assert eb < 1e-3 and ea < 1e-4, (li, eb, ea)

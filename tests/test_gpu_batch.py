"""The uneven batch for covariances (Sec. 3.5, closing remark), through the C ABI.

Mocks on assignment grids of 128, 192, 256 and 384 points per side share one
reduction geometry (N' = 128, 20 shells of 2 k_f, l <= 4, 50 modes with P = 6),
run through bsp_batch_run in bf16 hi+lo, and are checked mock by mock against
the FP64 oracle (B_l, and alpha on the orthonormalised kept modes); the FP64
covariance of the alpha rows is checked against the oracle's definition on
the same rows.
"""
import sys

import numpy as np
import pytest

import oracle as O
from synth import catalog as C
from tests.gpu_helpers import pfid_table, rel_norm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1708_05303_amd as B  # noqa: E402

DEV = torch.device("cuda:0")
DROP_TOL = 1e-2  # relative residual below which the orthonormalisation drops a mode


def say(*a):
    print("[batch]", *a, flush=True)
    sys.stdout.flush()


def test_batch_covariance_against_oracle():
    say("covariance kernel")
    r = np.random.Generator(np.random.PCG64(77))
    x = r.standard_normal((37, 150)) * r.uniform(0.1, 10.0, 150) + r.uniform(-5, 5, 150)
    xd = torch.as_tensor(x, device=DEV)
    cov = torch.zeros((150, 150), dtype=torch.float64, device=DEV)
    B.bsp_batch_covariance(xd, 37, 150, cov)
    torch.cuda.synchronize()
    assert rel_norm(cov.cpu().numpy(), O.batch_covariance(x)) < 1e-13


def test_batch_covariance_rejects_single_mock():
    cov = torch.zeros((4, 4), dtype=torch.float64, device=DEV)
    x = torch.zeros((1, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(B.BspError):
        B.bsp_batch_covariance(x, 1, 4, cov)


@pytest.fixture(scope="module")
def uneven_batch(tmp_path_factory):
    sizes = [128, 192, 256, 384]
    mocks = [(0, 128), (1, 192), (2, 256), (3, 384), (4, 128)]  # (seed offset, grid)
    ref_wl = C.batch_workload(0, 256)
    pf = pfid_table(ref_wl, 3 * 128 ** 2)
    plans = {}
    for n in sizes:
        wl = C.batch_workload(0, n)
        plans[n] = B.Plan(n=n, n_reduce=wl.n_reduce, box=wl.box, nbins=wl.nbins, k0=wl.k0, dk=wl.dk, lmax=wl.lmax,
                          window=wl.window, interlace=wl.interlace, los=wl.los, observer=C.observer_grid_units(wl),
                          P=wl.P, nmodes=wl.nmodes, pfid=pf, drop_tol=DROP_TOL)
        plans[n].precompute()
    cats, refs = [], []
    for m, n in mocks:
        wl = C.batch_workload(m, n)
        u = C.lognormal_catalogue(wl)
        obs = C.observer_grid_units(wl)
        spec, wsum = O.spectrum_from_catalogue(*u, n, wl.lmax, obs, window=wl.window, interlace=wl.interlace)
        geo = O.Geometry(n, wl.n_reduce, wl.box, wl.lmax, wl.nbins, wl.k0, wl.dk, wl.P, wl.nmodes, pf)
        refs.append(O.estimate(spec, geo, nbar=wsum / wl.box ** 3, modal_tol=DROP_TOL))
        cats.append(u)
        say("oracle mock", m, n)
    info = plans[128].info
    nl, nm = info.nl, C.batch_workload(0, 128).nmodes
    order = [sizes.index(n) for _, n in mocks]
    dv = [[torch.as_tensor(u[a]).to(DEV) for u in cats] for a in range(3)]
    outs = {}
    # graph replay, graph replay again (the kept graphs), and plain calls
    for mode, flags in (("graph", B.BSP_BATCH_GRAPH), ("graph2", B.BSP_BATCH_GRAPH), ("plain", 0)):
        say("batch run", mode)
        B_all = torch.zeros((len(mocks), nl, info.ntri), dtype=torch.float64, device=DEV)
        alpha_all = torch.zeros((len(mocks), nl * nm), dtype=torch.float64, device=DEV)
        beta_all = torch.zeros((len(mocks), nl * nm), dtype=torch.float64, device=DEV)
        cov = torch.zeros((nl * nm, nl * nm), dtype=torch.float64, device=DEV)
        B.bsp_batch_run([plans[n].handle for n in sizes], order, dv[0], dv[1], dv[2], None,
                        [u[0].size for u in cats], B.BSP_BF16X3, B_all, alpha_all, beta_all, cov, flags)
        plans[128].sync()
        outs[mode] = (B_all.cpu().numpy(), alpha_all.cpu().numpy(), beta_all.cpu().numpy(), cov.cpu().numpy())
    # checkpoint / resume: the first three mocks are journaled, a torn record
    # (what a writer killed mid-append leaves) is added by hand, and the whole
    # batch is run again on the same journal, then once more without graphs
    jdir = tmp_path_factory.mktemp("journal")
    keys = [1000 + m for m, _ in mocks]
    hpl = [plans[n].handle for n in sizes]
    npart = [u[0].size for u in cats]

    def jrun(path, idx, flags, with_beta=True):
        sub = [[dv[a][i] for i in idx] for a in range(3)]
        B_all = torch.zeros((len(idx), nl, info.ntri), dtype=torch.float64, device=DEV)
        alpha_all = torch.zeros((len(idx), nl * nm), dtype=torch.float64, device=DEV)
        beta_all = torch.zeros((len(idx), nl * nm), dtype=torch.float64, device=DEV) if with_beta else None
        cov = torch.zeros((nl * nm, nl * nm), dtype=torch.float64, device=DEV)
        nres = B.bsp_batch_run_journal(hpl, [order[i] for i in idx], [keys[i] for i in idx], sub[0], sub[1], sub[2],
                                       None, [npart[i] for i in idx], B.BSP_BF16X3, B_all, alpha_all, beta_all, cov,
                                       str(path), flags)
        plans[128].sync()
        return nres, (B_all.cpu().numpy(), alpha_all.cpu().numpy(),
                      beta_all.cpu().numpy() if with_beta else None, cov.cpu().numpy())

    say("journal: fresh run of all mocks")
    full = jdir / "full.bspj"
    outs["journal_fresh"] = jrun(full, range(len(mocks)), B.BSP_BATCH_GRAPH)
    outs["journal_fresh_scan"] = B.bsp_journal_scan(str(full))
    say("journal: first three mocks, then a torn record, then the whole batch")
    part = jdir / "part.bspj"
    outs["journal_part"] = jrun(part, [0, 1, 2], B.BSP_BATCH_GRAPH)
    n3, v3, f3 = B.bsp_journal_scan(str(part))
    raw = part.read_bytes()
    with open(part, "ab") as fh:
        fh.write(raw[v3 - (v3 - 16) // 3: v3 - (v3 - 16) // 3 + 200])  # head of the last record, cut short
    outs["journal_torn_scan"] = (n3, v3, f3, B.bsp_journal_scan(str(part)))
    outs["journal_resume"] = jrun(part, range(len(mocks)), B.BSP_BATCH_GRAPH)
    outs["journal_resume_scan"] = B.bsp_journal_scan(str(part))
    say("journal: every mock recorded, plain calls")
    outs["journal_all_recorded"] = jrun(part, range(len(mocks)), 0)
    say("journal: records without beta serve only calls without beta")
    nob = jdir / "nobeta.bspj"
    outs["journal_nobeta"] = jrun(nob, [0, 1], B.BSP_BATCH_GRAPH, with_beta=False)
    outs["journal_nobeta_again"] = jrun(nob, [0, 1], B.BSP_BATCH_GRAPH, with_beta=False)
    outs["journal_beta_after_nobeta"] = jrun(nob, [0, 1], B.BSP_BATCH_GRAPH)
    outs["config_hash"] = {n: B.bsp_config_hash(plans[n].handle, B.BSP_BF16X3) for n in sizes}
    outs["config_hash_fp32"] = B.bsp_config_hash(plans[128].handle, B.BSP_FP32)
    counts = {n: plans[n].counts.copy() for n in sizes}
    kept = {n: plans[n].kept.copy() for n in sizes}
    for p in plans.values():
        p.close()
    return mocks, refs, counts, kept, outs, nl, nm


def test_uneven_batch_graph_replay_is_bit_identical(uneven_batch):
    """The graph-captured replay and the plain per-mock calls give the same
    bits (the path is reproducible and the graph replays the same kernels)."""
    mocks, refs, counts, kept, outs, nl, nm = uneven_batch
    for a, b in zip(outs["graph"], outs["plain"]):
        assert np.array_equal(a, b)
    for a, b in zip(outs["graph"], outs["graph2"]):
        assert np.array_equal(a, b)


def test_batch_journal_resume_is_bit_identical(uneven_batch):
    """Checkpoint / resume: a journaled batch gives the bits of the plain
    batch; after three mocks and a torn fourth record, the resumed batch takes
    the three from the journal, cuts the torn tail off, runs the other two and
    again gives the same bits (B, alpha, beta and the covariance over all
    mocks); a batch whose mocks are all recorded runs none."""
    mocks, refs, counts, kept, outs, nl, nm = uneven_batch
    ref = outs["graph"]
    nres, got = outs["journal_fresh"]
    assert nres == 0
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    nrec, valid, size = outs["journal_fresh_scan"]
    assert nrec == len(mocks) and valid == size
    nres, got = outs["journal_part"]
    assert nres == 0
    for a, b in zip(got[:3], ref[:3]):
        assert np.array_equal(a, b[:3])
    n3, v3, f3, torn = outs["journal_torn_scan"]
    assert n3 == 3 and v3 == f3
    assert torn == (3, v3, v3 + 200)
    nres, got = outs["journal_resume"]
    assert nres == 3
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    nrec, valid, size = outs["journal_resume_scan"]
    assert nrec == len(mocks) and valid == size
    nres, got = outs["journal_all_recorded"]
    assert nres == len(mocks)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    for key, want in (("journal_nobeta", 0), ("journal_nobeta_again", 2), ("journal_beta_after_nobeta", 0)):
        nres, got = outs[key]
        assert nres == want, key
        assert np.array_equal(got[0], ref[0][:2]) and np.array_equal(got[1], ref[1][:2]), key
        if got[2] is not None:
            assert np.array_equal(got[2], ref[2][:2]), key
    hashes = outs["config_hash"]
    assert len(set(hashes.values())) == len(hashes)  # plans of different N hash differently
    assert outs["config_hash_fp32"] != hashes[128]


def test_uneven_batch_against_oracle(uneven_batch):
    mocks, refs, counts, kept, outs, nl, nm = uneven_batch
    B_all, alpha_all, beta_all, cov = outs["graph"]
    ko = refs[0]["modal_kept"]
    for n, c in counts.items():
        assert np.array_equal(c, refs[0]["counts"]), n
        assert np.array_equal(kept[n][:len(ko)], ko) and np.all(kept[n][len(ko):] == -1), n
    say("kept modes", len(ko), "of", nm)
    for i, (m, n) in enumerate(mocks):
        ref = refs[i]
        for li in range(nl):
            e = rel_norm(B_all[i, li], ref["B"][li])
            say("mock", m, "n", n, "l", 2 * li, "B err", e)
            assert e < 1e-3, (m, li, e)
        kL = np.linalg.cond(np.linalg.cholesky(ref["gamma"][np.ix_(ko, ko)]))
        for li in range(nl):
            ea = rel_norm(alpha_all[i, li * nm:(li + 1) * nm], ref["alpha"][li])
            eb = rel_norm(beta_all[i, li * nm:(li + 1) * nm], ref["beta"][li])
            say("mock", m, "l", 2 * li, "alpha err", ea, "beta err", eb, "cond(L)", kL)
            assert ea < 1e-4, (m, li, ea)
            assert eb < kL * 1e-4, (m, li, eb)
    assert rel_norm(cov, O.batch_covariance(alpha_all)) < 1e-12
    ref_alpha = np.stack([r["alpha"].ravel() for r in refs])
    e = rel_norm(cov, O.batch_covariance(ref_alpha))
    say("covariance of alpha against the oracle rows", e)
    assert e < 5e-3


def test_batch_run_rejects_mismatched_plans():
    a = B.Plan(n=32, box=200.0, nbins=4, k0=2.0, dk=2.0, lmax=0, P=3, nmodes=4,
               pfid=np.full(3 * 32 * 32, 1e3))
    b = B.Plan(n=32, box=200.0, nbins=4, k0=2.0, dk=2.0, lmax=2, P=3, nmodes=4,
               pfid=np.full(3 * 32 * 32, 1e3))
    a.precompute()
    b.precompute()
    u = [torch.full((10,), 3.0, device=DEV) for _ in range(2)]
    Ball = torch.zeros((2, 3, 64), dtype=torch.float64, device=DEV)
    alpha = torch.zeros((2, 12), dtype=torch.float64, device=DEV)
    cov = torch.zeros((12, 12), dtype=torch.float64, device=DEV)
    with pytest.raises(B.BspError):
        B.bsp_batch_run([a.handle, b.handle], [0, 1], u, u, u, None, [10, 10], B.BSP_FP32, Ball, alpha, None, cov)
    with pytest.raises(B.BspError):
        B.bsp_batch_run([a.handle, b.handle], [0, 1], u, u, u, None, [10, 10], B.BSP_FP32, Ball, alpha, None, cov, 0)
    a.close()
    b.close()

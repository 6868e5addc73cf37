"""The autotuner through the C ABI: it times the transform tiles and the
reduction shapes of a plan, writes its choice to a JSON database, a second
plan of the same geometry takes the choice from the database without timing,
and the estimator's outputs stay within the rounding of the chunked FP32 sums
(compared with the untuned plan and with the FP64 oracle)."""
import json
import os
import sys
import time

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


def say(*a):
    print("[tune]", *a, flush=True)
    sys.stdout.flush()


def _plan(wl, obs, pf):
    p = B.Plan(n=wl.n, n_reduce=wl.n_reduce, box=wl.box, nbins=wl.nbins, k0=wl.k0, dk=wl.dk, lmax=wl.lmax,
               window=1, interlace=wl.interlace, los=1, observer=obs, P=wl.P, nmodes=wl.nmodes, pfid=pf,
               drop_tol=1e-2)
    return p.precompute()


def _run(plan, dv, npart, nl, nm, prec):
    Bt = torch.zeros((nl, plan.info.ntri), dtype=torch.float64, device=DEV)
    al = torch.zeros((nl, nm), dtype=torch.float64, device=DEV)
    B.bsp_bispectrum_multipoles(plan.handle, dv[0], dv[1], dv[2], None, npart, prec, Bt, None, None, None, al, None)
    plan.sync()
    return Bt.cpu().numpy(), al.cpu().numpy()


def test_autotune_database_and_outputs(tmp_path):
    wl = C.batch_workload(3, 128)
    obs = C.observer_grid_units(wl)
    pf = pfid_table(C.batch_workload(0, 256), 3 * 128 ** 2)
    u = C.lognormal_catalogue(wl)
    dv = [torch.as_tensor(a).to(DEV) for a in u]
    db = str(tmp_path / "tune.json")
    a = _plan(wl, obs, pf)
    nl, nm = a.info.nl, wl.nmodes
    ref = {prec: _run(a, dv, u[0].size, nl, nm, prec) for prec in (B.BSP_FP32, B.BSP_BF16X3)}
    t0 = time.perf_counter()
    a.autotune(B.BSP_BF16X3, db)
    t_tune = time.perf_counter() - t0
    say("tuned in", round(t_tune, 3), "s: shape", a.info.tune_shape, "kchunk", a.info.tune_kchunk,
        "tiles", a.info.tune_tiles)
    assert a.info.tune_shape >= 0 and a.info.tune_kchunk > 0 and a.info.tune_tiles in (1, 2)
    entries = json.load(open(db))
    keys = [k for k in entries if k != "_"]
    assert len(keys) == 1 and entries[keys[0]]["shape"] == a.info.tune_shape
    assert entries[keys[0]]["kchunk"] == a.info.tune_kchunk and entries[keys[0]]["reduce_ms"] > 0
    got = _run(a, dv, u[0].size, nl, nm, B.BSP_BF16X3)
    for li in range(nl):
        assert rel_norm(got[0][li], ref[B.BSP_BF16X3][0][li]) < 1e-5, li
        assert rel_norm(got[1][li], ref[B.BSP_BF16X3][1][li]) < 1e-5, li
    # a second plan of the same geometry reads the database (no timing, file unchanged)
    mtime = os.path.getmtime(db)
    b = _plan(wl, obs, pf)
    t0 = time.perf_counter()
    b.autotune(B.BSP_BF16X3, db)
    t_read = time.perf_counter() - t0
    say("read in", round(t_read, 3), "s")
    assert (b.info.tune_shape, b.info.tune_kchunk, b.info.tune_tiles) == \
        (a.info.tune_shape, a.info.tune_kchunk, a.info.tune_tiles)
    assert os.path.getmtime(db) == mtime
    got_b = _run(b, dv, u[0].size, nl, nm, B.BSP_BF16X3)
    assert np.array_equal(got_b[0], got[0]) and np.array_equal(got_b[1], got[1])
    # FP32 under its own key: a second entry; the tuned FP32 path against the oracle
    a.autotune(B.BSP_FP32, db)
    assert len([k for k in json.load(open(db)) if k != "_"]) == 2
    got32 = _run(a, dv, u[0].size, nl, nm, B.BSP_FP32)
    spec, wsum = O.spectrum_from_catalogue(*u, wl.n, wl.lmax, obs, window=1, interlace=wl.interlace)
    geo = O.Geometry(wl.n, wl.n_reduce, wl.box, wl.lmax, wl.nbins, wl.k0, wl.dk, wl.P, wl.nmodes, pf)
    oref = O.estimate(spec, geo, nbar=wsum / wl.box ** 3, modal_tol=1e-2)
    for li in range(nl):
        eB = rel_norm(got32[0][li], oref["B"][li])
        say("tuned FP32 l", 2 * li, "B err", eB)
        assert eB < 1e-5, (li, eB)
    a.close()
    b.close()


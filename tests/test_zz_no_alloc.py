"""The no-allocation assignment entry point against the workspace one, through
the C ABI: two calls in a row on the library's static device scratch, the
second with a smaller grid and catalogue, each bit-identical (grids and weight
sum) to bsp_grid_assign with a workspace; too large a grid is refused before
anything runs."""
import sys

import numpy as np
import pytest

from synth import catalog as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1708_05303_amd as B  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print("[noalloc]", *a, flush=True)
    sys.stdout.flush()


def _catalogue(n, npart, seed, weighted):
    r = np.random.Generator(np.random.PCG64(seed))
    hot = npart // 3
    u = [C.quantise_grid_units(np.concatenate([r.uniform(3.0, 7.5, hot), r.uniform(0, n, npart - hot)]), n)
         for _ in range(3)]
    w = r.uniform(0.2, 2.5, npart).astype(np.float32) if weighted else None
    return [torch.as_tensor(a).to(DEV) for a in u], (torch.as_tensor(w).to(DEV) if weighted else None)


def _both(n, window, interlace, npart, seed, weighted):
    u, w = _catalogue(n, npart, seed, weighted)
    ref_plan = B.Plan(n=n, box=100.0, nbins=1, k0=1.0, dk=1.0, window=window, interlace=interlace, workspace=True)
    plan = B.Plan(n=n, box=100.0, nbins=1, k0=1.0, dk=1.0, window=window, interlace=interlace, workspace=False)
    assert plan.ws is None
    g_ref = torch.full((1 + interlace, n, n, n), 0.25, dtype=torch.float32, device=DEV)
    g = torch.full_like(g_ref, 0.25)
    ws_ref = torch.full((1,), 3.0, dtype=torch.float64, device=DEV)
    ws = torch.full_like(ws_ref, 3.0)
    B.bsp_grid_assign(ref_plan.handle, u[0], u[1], u[2], w, npart, g_ref, ws_ref)
    ref_plan.sync()
    B.bsp_grid_assign_noalloc(plan.handle, u[0], u[1], u[2], w, npart, g, ws)
    plan.sync()
    out = (g.cpu().numpy(), ws.item(), g_ref.cpu().numpy(), ws_ref.item())
    plan.close()
    ref_plan.close()
    return out


def test_grid_assign_noalloc_matches_workspace_entry_point():
    # the largest grid the static scratch holds (128^3 interlaced), then a smaller one
    for case in [(128, 1, 1, 300_000, 11, True), (64, 0, 0, 40_000, 12, False), (32, 1, 1, 5_000, 13, True)]:
        say("case", case)
        g, ws, g_ref, ws_ref = _both(*case)
        assert np.array_equal(g, g_ref), (case, int(np.sum(g != g_ref)))
        assert ws == ws_ref, (case, ws, ws_ref)


def test_grid_assign_noalloc_rejects_too_large_grid():
    say("too large")
    plan = B.Plan(n=192, box=100.0, nbins=1, k0=1.0, dk=1.0, interlace=1, workspace=False)
    g = torch.zeros((1, 1), dtype=torch.float32, device=DEV)
    ws = torch.zeros(1, dtype=torch.float64, device=DEV)
    u = torch.ones(4, dtype=torch.float32, device=DEV)
    with pytest.raises(B.BspError) as e:
        B.bsp_grid_assign_noalloc(plan.handle, u, u, u, None, 4, g, ws)
    assert e.value.status == 2 and "static scratch" in str(e.value)
    plan.sync()
    assert ws.item() == 0.0
    plan.close()

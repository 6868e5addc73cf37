"""Python binding of libbsp (HIP, gfx950): FFT bispectrum multipoles and modal
coefficients of redshift-space galaxy catalogues.

Argument marshalling only: every step runs in the HIP library. PyTorch is used
for device memory and streams. Importing this package does not load the
library; the first call does, and raises ``BspLibraryMissing`` if
``libbsp.so`` has not been built (``python -m paper_1708_05303_amd.build``).
There is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "BspError", "BspLibraryMissing", "Geom", "ModalBasis", "Info", "lib", "Plan",
    "BSP_FP32", "BSP_BF16X3", "BSP_FP16X3", "BSP_BF16X1", "PRECISIONS", "bsp_plan_create", "bsp_plan_destroy",
    "bsp_plan_info", "bsp_workspace_size", "bsp_set_workspace", "bsp_set_slab", "bsp_sync", "bsp_precompute", "bsp_autotune",
    "BSP_TUNE_FORCE",
    "bsp_geometry", "bsp_grid_assign", "bsp_grid_assign_noalloc", "bsp_fft_r2c", "bsp_fft_c2r",
    "bsp_los_moments", "bsp_grid_entry", "bsp_filter_fields", "bsp_triple_reduce", "bsp_modal_coeffs", "bsp_bispectrum_multipoles",
    "bsp_bispectrum_field", "bsp_batch_run", "BSP_BATCH_GRAPH", "BSP_BATCH_FSYNC", "bsp_batch_run_journal",
    "bsp_config_hash", "bsp_journal_scan", "bsp_journal_append", "bsp_journal_lookup",
    "bsp_batch_covariance", "bsp_power_multipoles",
    "bsp_shot_noise_multipoles", "bsp_skew_spectra", "BSP_SKEW_BALL",
    "bsp_integrated_bispectrum", "BSP_IB_LOCAL_LOS", "bsp_bispectrum_full", "bsp_set_timing", "bsp_stage_times", "STAGES",
    "EXPORTED",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbsp.so")

BSP_FP32, BSP_BF16X3, BSP_FP16X3, BSP_BF16X1 = 0, 1, 2, 3
PRECISIONS = {"fp32": BSP_FP32, "bf16x3": BSP_BF16X3, "fp16x3": BSP_FP16X3, "bf16x1": BSP_BF16X1}
STATUS = {0: "BSP_OK", 1: "BSP_ERR_ARG", 2: "BSP_ERR_SIZE", 3: "BSP_ERR_ALIAS", 4: "BSP_ERR_WORKSPACE",
          5: "BSP_ERR_HIP", 6: "BSP_ERR_DEVICE", 7: "BSP_ERR_NUMERIC", 8: "BSP_ERR_STATE", 9: "BSP_ERR_IO"}

# every symbol include/bsp.h declares
EXPORTED = [
    "bsp_plan_create", "bsp_plan_destroy", "bsp_plan_info", "bsp_last_error", "bsp_workspace_size",
    "bsp_set_workspace", "bsp_set_slab", "bsp_sync", "bsp_precompute", "bsp_autotune", "bsp_geometry", "bsp_grid_assign",
    "bsp_grid_assign_noalloc", "bsp_fft_r2c",
    "bsp_fft_c2r", "bsp_los_moments", "bsp_grid_entry", "bsp_filter_fields", "bsp_triple_reduce",
    "bsp_modal_coeffs", "bsp_bispectrum_multipoles", "bsp_bispectrum_field", "bsp_batch_run",
    "bsp_batch_run_journal", "bsp_config_hash", "bsp_journal_scan", "bsp_journal_append", "bsp_journal_lookup",
    "bsp_batch_covariance", "bsp_power_multipoles", "bsp_shot_noise_multipoles", "bsp_skew_spectra",
    "bsp_integrated_bispectrum", "bsp_bispectrum_full", "bsp_set_timing", "bsp_stage_times",
]
STAGES = ["assign", "fwd_z", "fwd_y", "fwd_x", "los_combine", "inv_x_filter", "inv_y", "inv_z", "reduce",
          "reduce_combine", "power_multipoles", "skew_spectra", "integrated_bispectrum"]


class BspError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class BspLibraryMissing(RuntimeError):
    pass


class Geom(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_reduce", C.c_int32), ("box", C.c_double), ("window", C.c_int32),
                ("compensate", C.c_int32), ("interlace", C.c_int32), ("los", C.c_int32),
                ("observer", C.c_double * 3), ("lmax", C.c_int32), ("nbins", C.c_int32),
                ("k0", C.c_double), ("dk", C.c_double)]


class ModalBasis(C.Structure):
    _fields_ = [("P", C.c_int32), ("nmodes", C.c_int32), ("modes", C.POINTER(C.c_int32)),
                ("pfid", C.POINTER(C.c_double)), ("pfid_len", C.c_int32), ("drop_tol", C.c_double)]


class Info(C.Structure):
    _fields_ = [("c", C.c_int32), ("cz", C.c_int32), ("nl", C.c_int32), ("nlos", C.c_int32),
                ("ngrid", C.c_int32), ("n2max", C.c_int32), ("ncand", C.c_int32), ("ntri", C.c_int32),
                ("nfields_binned", C.c_int32), ("nfields_modal", C.c_int32), ("spec_elems", C.c_int64),
                ("count_residual", C.c_double), ("reduce_pairs", C.c_int32), ("reduce_thirds", C.c_int32),
                ("reduce_tiles", C.c_int32), ("reduce_groups", C.c_int32), ("reduce_maxr", C.c_int32),
                ("reduce_maxcw", C.c_int32), ("reduce_needed", C.c_int64), ("modal_rank", C.c_int32),
                ("tune_shape", C.c_int32), ("tune_tiles", C.c_int32), ("tune_kchunk", C.c_int64),
                ("reduce_row_tiles", C.c_int32), ("slab_planes", C.c_int32)]


_lib = None
_vp, _i32, _i64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_double


def lib():
    """Load libbsp.so (once) and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise BspLibraryMissing(f"{LIB_PATH} not built; run python -m paper_1708_05303_amd.build")
    L = C.CDLL(LIB_PATH)
    sig = {
        "bsp_plan_create": [C.POINTER(_vp), C.POINTER(Geom), C.POINTER(ModalBasis), _vp],
        "bsp_plan_destroy": [_vp],
        "bsp_plan_info": [_vp, C.POINTER(Info)],
        "bsp_workspace_size": [_vp, C.POINTER(C.c_size_t)],
        "bsp_set_workspace": [_vp, _vp, C.c_size_t],
        "bsp_set_slab": [_vp, C.c_int32],
        "bsp_sync": [_vp],
        "bsp_precompute": [_vp],
        "bsp_autotune": [_vp, _i32, C.c_char_p, _i32],
        "bsp_geometry": [_vp, _vp, _vp, _vp, _vp, _vp],
        "bsp_grid_assign": [_vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp],
        "bsp_grid_assign_noalloc": [_vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp],
        "bsp_fft_r2c": [_vp, _i32, _i32, _vp, _vp],
        "bsp_fft_c2r": [_vp, _i32, _i32, _vp, _vp],
        "bsp_los_moments": [_vp, _vp, _vp, _vp],
        "bsp_grid_entry": [_vp, _vp, _vp],
        "bsp_filter_fields": [_vp, _vp, _i32, _vp, _vp],
        "bsp_triple_reduce": [_vp, _vp, _i32, _i64, _vp, _i32, _vp, _i32, _vp, _i32, _vp],
        "bsp_modal_coeffs": [_vp, _vp, _i32, _d, _vp, _vp, _vp],
        "bsp_bispectrum_multipoles": [_vp, _vp, _vp, _vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp],
        "bsp_bispectrum_field": [_vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp],
        "bsp_batch_run": [_vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _i32],
        "bsp_batch_run_journal": [_vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp,
                                  _i32, C.c_char_p, _vp],
        "bsp_config_hash": [_vp, _i32, _vp],
        "bsp_journal_scan": [C.c_char_p, _vp, _vp, _vp],
        "bsp_journal_append": [C.c_char_p, C.c_uint64, C.c_uint64, _i64, _i32, _i32, _i32, _vp, _vp, _vp],
        "bsp_journal_lookup": [C.c_char_p, C.c_uint64, C.c_uint64, _i64, _i32, _i32, _i32, _vp, _vp, _vp, _vp],
        "bsp_batch_covariance": [_vp, _i32, _i32, _vp, _vp],
        "bsp_power_multipoles": [_vp, _vp, _vp],
        "bsp_shot_noise_multipoles": [_vp, _vp, _d, _vp],
        "bsp_skew_spectra": [_vp, _vp, _vp, _i32],
        "bsp_integrated_bispectrum": [_vp, _vp, _vp, _i32, _d, _d, _i32, _vp, _vp, _vp, _i32],
        "bsp_bispectrum_full": [_vp, _vp, _i32, _vp],
        "bsp_set_timing": [_vp, _i32],
        "bsp_stage_times": [_vp, _vp, _vp, _vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.bsp_last_error.argtypes = [_vp]
    L.bsp_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(status: int, plan=None):
    if status != 0:
        msg = lib().bsp_last_error(plan)
        raise BspError(status, msg.decode() if msg else "")


def _dptr(t, dtype=None):
    """Device pointer of a contiguous torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def _hptr(a, ctype):
    a = np.ascontiguousarray(a)
    return a, a.ctypes.data_as(C.POINTER(ctype))


# ---------------------------------------------------------------- C-named calls

def bsp_plan_create(geom: Geom, basis: Optional[ModalBasis] = None, stream: int = 0):
    h = C.c_void_p()
    _check(lib().bsp_plan_create(C.byref(h), C.byref(geom), C.byref(basis) if basis is not None else None,
                                 C.c_void_p(stream)))
    return h


def bsp_plan_destroy(plan):
    _check(lib().bsp_plan_destroy(plan))


def bsp_plan_info(plan) -> Info:
    info = Info()
    _check(lib().bsp_plan_info(plan, C.byref(info)), plan)
    return info


def bsp_workspace_size(plan) -> int:
    n = C.c_size_t()
    _check(lib().bsp_workspace_size(plan, C.byref(n)), plan)
    return n.value


def bsp_set_workspace(plan, ws, nbytes: int):
    _check(lib().bsp_set_workspace(plan, _dptr(ws), nbytes), plan)


def bsp_set_slab(plan, planes: int):
    """x planes per slab of the field stacks (0: the plan's default)."""
    _check(lib().bsp_set_slab(plan, int(planes)), plan)


def bsp_sync(plan):
    _check(lib().bsp_sync(plan), plan)


def bsp_precompute(plan):
    _check(lib().bsp_precompute(plan), plan)


BSP_TUNE_FORCE = 1


def bsp_autotune(plan, prec, db_path=None, flags=0):
    _check(lib().bsp_autotune(plan, int(prec), None if db_path is None else os.fsencode(db_path), int(flags)), plan)


def bsp_geometry(plan, ntri: int, nmodes: int = 0):
    """Returns (tri, counts, gamma, chol, kept); kept lists the kept modes in
    the order orthonormalised, -1 past the rank."""
    tri = np.zeros((ntri, 3), np.int32)
    cnt = np.zeros(ntri, np.int64)
    gam = np.zeros((nmodes, nmodes)) if nmodes else None
    chol = np.zeros((nmodes, nmodes)) if nmodes else None
    kept = np.zeros(nmodes, np.int32) if nmodes else None
    _check(lib().bsp_geometry(plan, tri.ctypes.data, cnt.ctypes.data,
                              gam.ctypes.data if nmodes else None, chol.ctypes.data if nmodes else None,
                              kept.ctypes.data if nmodes else None), plan)
    return tri, cnt, gam, chol, kept


def bsp_grid_assign(plan, ux, uy, uz, w, np_, grids, wsum):
    import torch
    _check(lib().bsp_grid_assign(plan, _dptr(ux, torch.float32), _dptr(uy, torch.float32),
                                 _dptr(uz, torch.float32), _dptr(w, torch.float32), int(np_),
                                 _dptr(grids, torch.float32), _dptr(wsum, torch.float64)), plan)


def bsp_grid_assign_noalloc(plan, ux, uy, uz, w, np_, grids, wsum):
    """bsp_grid_assign with the library's static device scratch (no workspace)."""
    import torch
    _check(lib().bsp_grid_assign_noalloc(plan, _dptr(ux, torch.float32), _dptr(uy, torch.float32),
                                         _dptr(uz, torch.float32), _dptr(w, torch.float32), int(np_),
                                         _dptr(grids, torch.float32), _dptr(wsum, torch.float64)), plan)


def bsp_fft_r2c(plan, n, batch, inp, out):
    _check(lib().bsp_fft_r2c(plan, n, batch, _dptr(inp), _dptr(out)), plan)


def bsp_fft_c2r(plan, n, batch, inp, out):
    _check(lib().bsp_fft_c2r(plan, n, batch, _dptr(inp), _dptr(out)), plan)


def bsp_los_moments(plan, grids, wsum, delta_l):
    _check(lib().bsp_los_moments(plan, _dptr(grids), _dptr(wsum), _dptr(delta_l)), plan)


def bsp_grid_entry(plan, delta, delta_l):
    _check(lib().bsp_grid_entry(plan, _dptr(delta), _dptr(delta_l)), plan)


def bsp_filter_fields(plan, delta_l, filt, fields):
    f, _ = _hptr(np.asarray(filt, np.int32).reshape(-1, 3), C.c_int32)
    _check(lib().bsp_filter_fields(plan, _dptr(delta_l), f.shape[0], f.ctypes.data, _dptr(fields)), plan)


def bsp_triple_reduce(plan, fields, nfields, K, pairs, thirds, need, prec, T):
    pr = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    th = np.ascontiguousarray(np.asarray(thirds, np.int32).ravel())
    nd = None if need is None else np.ascontiguousarray(np.asarray(need, np.uint8))
    _check(lib().bsp_triple_reduce(plan, _dptr(fields), nfields, K, pr.ctypes.data, pr.shape[0], th.ctypes.data,
                                   th.size, None if nd is None else nd.ctypes.data, prec, _dptr(T)), plan)


def bsp_modal_coeffs(plan, delta_l, prec, nbar, bnum, alpha, beta):
    _check(lib().bsp_modal_coeffs(plan, _dptr(delta_l), prec, float(nbar), _dptr(bnum), _dptr(alpha),
                                  _dptr(beta)), plan)


def bsp_bispectrum_multipoles(plan, ux, uy, uz, w, np_, prec, B, B0sub=None, Pbar=None, bnum=None, alpha=None,
                              beta=None):
    _check(lib().bsp_bispectrum_multipoles(plan, _dptr(ux), _dptr(uy), _dptr(uz), _dptr(w), int(np_), prec,
                                           _dptr(B), _dptr(B0sub), _dptr(Pbar), _dptr(bnum), _dptr(alpha),
                                           _dptr(beta)), plan)


def bsp_bispectrum_field(plan, delta, prec, B, Pbar=None, bnum=None, alpha=None, beta=None):
    _check(lib().bsp_bispectrum_field(plan, _dptr(delta), prec, _dptr(B), _dptr(Pbar), _dptr(bnum), _dptr(alpha),
                                      _dptr(beta)), plan)


BSP_BATCH_GRAPH = 1
BSP_BATCH_FSYNC = 2


def _batch_args(plans, mock_plan, ux, uy, uz, w, np_):
    import torch
    nm, npl = len(mock_plan), len(plans)
    P = (C.c_void_p * npl)(*[h.value if isinstance(h, C.c_void_p) else h for h in plans])
    mp = (C.c_int32 * nm)(*[int(i) for i in mock_plan])
    NP = (C.c_int64 * nm)(*[int(v) for v in np_])

    def ptrs(ts):
        return (C.c_void_p * nm)(*[_dptr(t, torch.float32) for t in ts])
    W = None if w is None else ptrs(w)
    return P, npl, mp, nm, ptrs(ux), ptrs(uy), ptrs(uz), W, NP


def bsp_batch_run(plans, mock_plan, ux, uy, uz, w, np_, prec, B_all, alpha_all, beta_all, cov, flags=BSP_BATCH_GRAPH):
    """plans: list of plan handles; mock_plan, np_: per-mock ints; ux, uy, uz, w:
    per-mock float32 device tensors (w None or a list with None entries);
    flags: BSP_BATCH_GRAPH replays each plan's captured whole path, 0 calls it."""
    P, npl, mp, nm, X, Y, Z, W, NP = _batch_args(plans, mock_plan, ux, uy, uz, w, np_)
    _check(lib().bsp_batch_run(P, npl, mp, nm, X, Y, Z, W, NP, prec, _dptr(B_all), _dptr(alpha_all),
                               _dptr(beta_all), _dptr(cov), int(flags)), plans[0])


def bsp_batch_run_journal(plans, mock_plan, mock_key, ux, uy, uz, w, np_, prec, B_all, alpha_all, beta_all, cov,
                          journal, flags=BSP_BATCH_GRAPH):
    """bsp_batch_run with a checkpoint journal (path); mock_key: per-mock
    unsigned 64-bit keys. Returns the number of mocks taken from the journal."""
    P, npl, mp, nm, X, Y, Z, W, NP = _batch_args(plans, mock_plan, ux, uy, uz, w, np_)
    keys = (C.c_uint64 * nm)(*[int(k) for k in mock_key])
    nres = C.c_int32(0)
    _check(lib().bsp_batch_run_journal(P, npl, mp, nm, keys, X, Y, Z, W, NP, prec, _dptr(B_all), _dptr(alpha_all),
                                       _dptr(beta_all), _dptr(cov), int(flags), os.fsencode(journal),
                                       C.byref(nres)), plans[0])
    return nres.value


def bsp_config_hash(plan, prec) -> int:
    h = C.c_uint64(0)
    _check(lib().bsp_config_hash(plan, prec, C.byref(h)), plan)
    return h.value


def bsp_journal_scan(journal):
    """(records, valid_bytes, file_bytes) of a journal file; host only."""
    n, v, f = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    _check(lib().bsp_journal_scan(os.fsencode(journal), C.byref(n), C.byref(v), C.byref(f)))
    return n.value, v.value, f.value


def bsp_journal_append(journal, key, config_hash, np_, B, alpha, beta=None):
    """Appends one record; B: host float64 [nl][ntri], alpha, beta: host float64 [d]."""
    B = np.ascontiguousarray(B, dtype=np.float64)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = None if beta is None else np.ascontiguousarray(beta, dtype=np.float64)
    if B.ndim != 2 or alpha.ndim != 1 or (beta is not None and beta.shape != alpha.shape):
        raise ValueError("B must be [nl][ntri], alpha and beta [d]")
    _check(lib().bsp_journal_append(os.fsencode(journal), int(key), int(config_hash), int(np_), B.shape[0],
                                    B.shape[1], alpha.shape[0], B.ctypes.data, alpha.ctypes.data,
                                    None if beta is None else beta.ctypes.data))


def bsp_journal_lookup(journal, key, config_hash, np_, nl, ntri, d, with_beta=True):
    """(B, alpha, beta) of a record, or None if there is none."""
    B = np.zeros((nl, ntri))
    alpha = np.zeros(d)
    beta = np.zeros(d) if with_beta else None
    found = C.c_int32(0)
    _check(lib().bsp_journal_lookup(os.fsencode(journal), int(key), int(config_hash), int(np_), nl, ntri, d,
                                    B.ctypes.data, alpha.ctypes.data, None if beta is None else beta.ctypes.data,
                                    C.byref(found)))
    return (B, alpha, beta) if found.value else None


def bsp_batch_covariance(x, m, d, cov, stream: int = 0):
    _check(lib().bsp_batch_covariance(_dptr(x), m, d, _dptr(cov), C.c_void_p(stream)))


def bsp_power_multipoles(plan, delta_l, P):
    _check(lib().bsp_power_multipoles(plan, _dptr(delta_l), _dptr(P)), plan)


def bsp_shot_noise_multipoles(plan, P, nbar, SN):
    _check(lib().bsp_shot_noise_multipoles(plan, _dptr(P), float(nbar), _dptr(SN)), plan)


BSP_SKEW_BALL = 1


def bsp_skew_spectra(plan, delta_l, S, flags=0):
    """flags: 0 (monopole squared on the union of the shells) or BSP_SKEW_BALL (on the ball |n|^2 <= n2max)."""
    _check(lib().bsp_skew_spectra(plan, _dptr(delta_l), _dptr(S), int(flags)), plan)


BSP_IB_LOCAL_LOS = 1


def bsp_integrated_bispectrum(plan, grid, wsum, s, k0, dk, nbins, iB, Psub=None, dbar=None, flags=0):
    """flags: 0 (one line of sight per sub-volume) or BSP_IB_LOCAL_LOS (x_hat per node)."""
    _check(lib().bsp_integrated_bispectrum(plan, _dptr(grid), _dptr(wsum), int(s), float(k0), float(dk), int(nbins),
                                           _dptr(iB), _dptr(Psub), _dptr(dbar), int(flags)), plan)


def bsp_bispectrum_full(plan, delta_l, prec, B):
    _check(lib().bsp_bispectrum_full(plan, _dptr(delta_l), int(prec), _dptr(B)), plan)


def bsp_set_timing(plan, enable: bool):
    _check(lib().bsp_set_timing(plan, 1 if enable else 0), plan)


def bsp_stage_times(plan):
    """{stage name: (milliseconds summed, launches, algorithmic bytes or flops summed)}
    since bsp_set_timing(plan, True)."""
    ms = np.zeros(16)
    n = np.zeros(16, np.int64)
    amt = np.zeros(16)
    _check(lib().bsp_stage_times(plan, ms.ctypes.data, n.ctypes.data, amt.ctypes.data), plan)
    return {STAGES[i]: (float(ms[i]), int(n[i]), float(amt[i])) for i in range(len(STAGES))}


# ---------------------------------------------------------------- convenience

def default_modes(P: int, nmodes: int) -> np.ndarray:
    """Mode table (p, r, s), p <= r <= s < P, ordered by (p+r+s, s, r); first nmodes."""
    allm = [(p, r, s) for p in range(P) for r in range(p, P) for s in range(r, P)]
    allm.sort(key=lambda t: (t[0] + t[1] + t[2], t[2], t[1]))
    return np.array(allm[:nmodes], np.int32)


class Plan:
    """Owns a bsp plan, its workspace tensor and the stream it runs on."""

    def __init__(self, n, box, nbins, k0, dk, lmax=0, n_reduce=0, window=1, compensate=1, interlace=0, los=0,
                 observer=(0.0, 0.0, 0.0), P=0, nmodes=0, modes=None, pfid=None, drop_tol=0.0, device="cuda:0",
                 workspace=True, slab=0):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        g = Geom()
        g.n, g.n_reduce, g.box, g.window, g.compensate = n, n_reduce, box, window, compensate
        g.interlace, g.los, g.lmax, g.nbins, g.k0, g.dk = interlace, los, lmax, nbins, k0, dk
        for a in range(3):
            g.observer[a] = float(observer[a])
        self.geom = g
        self.basis = None
        self.nmodes = 0
        if nmodes:
            self._modes = np.ascontiguousarray(modes if modes is not None else default_modes(P, nmodes), np.int32)
            self._pfid = np.ascontiguousarray(pfid, np.float64)
            b = ModalBasis()
            b.P, b.nmodes = P, nmodes
            b.modes = self._modes.ctypes.data_as(C.POINTER(C.c_int32))
            b.pfid = self._pfid.ctypes.data_as(C.POINTER(C.c_double))
            b.pfid_len = self._pfid.size
            b.drop_tol = float(drop_tol)
            self.basis = b
            self.nmodes = nmodes
            self.P = P
        self.stream = torch.cuda.current_stream(self.device)
        self.handle = bsp_plan_create(g, self.basis, self.stream.cuda_stream)
        if slab:
            bsp_set_slab(self.handle, slab)
        self.info = bsp_plan_info(self.handle)
        self.ws = None
        if workspace:
            nbytes = bsp_workspace_size(self.handle)
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            bsp_set_workspace(self.handle, self.ws, nbytes)
        self.tri = self.counts = self.gamma = self.chol = self.kept = None

    def precompute(self):
        bsp_precompute(self.handle)
        self.info = bsp_plan_info(self.handle)
        self.tri, self.counts, self.gamma, self.chol, self.kept = bsp_geometry(self.handle, self.info.ntri,
                                                                              self.nmodes)
        return self

    def autotune(self, prec, db_path=None, force=False):
        """Tile and shape choices for this plan (see bsp_autotune); db_path: JSON database."""
        bsp_autotune(self.handle, prec, db_path, BSP_TUNE_FORCE if force else 0)
        self.info = bsp_plan_info(self.handle)
        return self

    def gram_condition(self):
        """2-norm condition numbers (after precompute; None without a modal
        basis): of the lattice Gram matrix gamma, and of the Cholesky factor L
        of its kept modes. alpha = L^-1 b amplifies relative errors of the
        numerators b by up to cond(L), beta by up to cond(L)^2."""
        if self.gamma is None or self.nmodes == 0:
            return None
        r = int(self.info.modal_rank)
        L = np.asarray(self.chol)[:r, :r]
        return {"gamma": float(np.linalg.cond(np.asarray(self.gamma))), "L_kept": float(np.linalg.cond(L)),
                "rank": r, "nmodes": int(self.nmodes)}

    def sync(self):
        bsp_sync(self.handle)

    def spectrum_buffer(self):
        t = self.torch
        return t.zeros((self.info.nl, self.info.spec_elems, 2), dtype=t.float32, device=self.device)

    def close(self):
        if getattr(self, "handle", None) is not None:
            bsp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

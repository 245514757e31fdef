"""Python binding of libkbm (MI355X shift-and-stack search).

Argument marshalling only: every step of the search runs in the HIP kernels
of ``libkbm.so``; this module checks tensor shapes/dtypes, allocates output
tensors, and passes raw device pointers plus the current HIP stream through
the C ABI declared in ``include/kbm.h``.  PyTorch supplies device memory and
streams.  There is no CPU fallback: without the built library every call
raises.

Method: Smotherman et al., arXiv 2109.03296, Section 3 (likelihood planes,
trajectory sums), 3.1 (sigma_G filter) and 3.2 (in-line filter, per-pixel
top-K).
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

__all__ = [
    "KbmError", "lib", "make_planes", "search", "search_batched",
    "search_workspace_size", "sigmag_filter", "refine_forward",
    "refine_backward", "TrajLH", "SearchParams", "MAX_EPOCHS", "MAX_K",
    "MAX_PSF", "extract_top", "adam_step", "refine", "BatchedSearch",
    "Schedule", "batch_workspace_size", "extract_workspace_size",
    "score_trajectories", "stamps", "STAMP_LIMITS", "sigmag_filter_ex", "sigmag_coeff",
    "extract_top_noalloc", "Refiner", "detect", "tune_cache_clear", "refine_adam",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkbm.so")
MAX_EPOCHS, MAX_K, MAX_PSF = 64, 16, 31

_lock = threading.Lock()
_lib = None


class KbmError(RuntimeError):
    def __init__(self, func, status, detail):
        super().__init__(f"{func}: {status} ({detail})")
        self.func, self.status, self.detail = func, status, detail


class _Stack(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32),
                ("num_epochs", C.c_int32), ("times", C.c_void_p)]


class _SearchParams(C.Structure):
    _fields_ = [("vel", C.c_void_p), ("num_vel", C.c_int32), ("k", C.c_int32),
                ("min_obs", C.c_int32), ("sigmag", C.c_int32),
                ("q_lo", C.c_double), ("q_hi", C.c_double),
                ("coeff", C.c_double), ("n_sigma", C.c_double),
                ("x_begin", C.c_int32), ("y_begin", C.c_int32),
                ("x_end", C.c_int32), ("y_end", C.c_int32)]


class _Results(C.Structure):
    _fields_ = [("lh", C.c_void_p), ("flux", C.c_void_p),
                ("vel_idx", C.c_void_p), ("n_obs", C.c_void_p),
                ("keep", C.c_void_p), ("lh_raw", C.c_void_p)]


def lib():
    """Load libkbm.so (building it first only if it does not exist).  A
    library built from other sources or flags than the ones in the tree is
    refused: its build id must equal the id of the current sources."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        from . import build as _build
        if not os.path.exists(LIB_PATH):
            _build.build()
        if not os.path.exists(LIB_PATH):
            raise ImportError("libkbm.so is missing and could not be built")
        L = C.CDLL(LIB_PATH)
        L.kbm_build_id.restype = C.c_char_p
        built, want = L.kbm_build_id().decode(), _build.source_hash()
        if built != want:
            raise ImportError(f"libkbm.so was built from other sources (build id {built}, "
                              f"sources {want}); rebuild it (__graft_entry__.build())")
        P, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.kbm_status_string.restype = C.c_char_p
        L.kbm_status_string.argtypes = [C.c_int]
        L.kbm_last_error.restype = C.c_char_p
        L.kbm_version.restype = C.c_int
        L.kbm_make_planes.argtypes = [P, P, P, P, P, i32, P, P, P]
        L.kbm_search_workspace_size.argtypes = [P, P, i32, P]
        L.kbm_search.argtypes = [P, P, P, P, P, i32, P, C.c_size_t, P]
        L.kbm_sigmag_filter.argtypes = [P, P, P, i64, i32, f64, f64, f64, f64,
                                        P, P, P]
        L.kbm_refine.argtypes = [P, P, P, i64, P, P, P, P, P, P, P, P]
        L.kbm_refine_adam.argtypes = [P, P, P, i64, P, P, P, i32, f64, f64, f64, P, P]
        L.kbm_extract_workspace_size.argtypes = [i32, i32, i32, i32, P]
        L.kbm_extract_top.argtypes = [P, i32, i32, i32, i32, i32, P, i32,
                                      C.c_float, i64, P, P, P, P, P, P, P, P,
                                      C.c_size_t, P]
        L.kbm_extract_top_noalloc.argtypes = [P, i32, i32, i32, i32, i32, P, i32,
                                              C.c_float, i64, P, P, P, P, P, P, P, P]
        L.kbm_adam_step.argtypes = [P, P, P, P, i64, i32, P, f64, f64, f64,
                                    i32, i32, P]
        L.kbm_batch_workspace_size.argtypes = [P, P, i32, P]
        L.kbm_batch_create.argtypes = [P, P, P, P, P, i32, P, C.c_size_t, i32,
                                       P, P, P]
        L.kbm_batch_run.argtypes = [P, P]
        L.kbm_batch_check.argtypes = [P, P, P]
        L.kbm_batch_evaluated.argtypes = [P, P, P]
        L.kbm_batch_destroy.argtypes = [P]
        L.kbm_tune_cache_clear.argtypes = []
        L.kbm_score_trajectories.argtypes = [P, P, P, i64, P, i32, i32, f64, f64,
                                             f64, f64, P, P, P, P, P, P]
        L.kbm_stamps.argtypes = [P, P, P, P, i64, P, P, i32, P, P, P, P, P]
        L.kbm_sigmag_filter_ex.argtypes = [P, P, P, i64, i32, i32, f64, f64, f64, f64,
                                           f64, P, P, P, P]
        L.kbm_sigmag_coeff.argtypes = [f64, f64, P]
        L.kbm_detect.argtypes = [i64, P, P, P, i32, C.c_float, P, P]
        _lib = L
        return L


class Schedule(C.Structure):
    """Schedule of the batched persistent search (see ``kbm_schedule``)."""
    _fields_ = [("vel_block", C.c_int32), ("tile_cols", C.c_int32),
                ("tile_rows", C.c_int32), ("waves", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("sweep", C.c_int32),
                ("probe_ms", C.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


TUNE_DEFAULT, TUNE_AUTO, TUNE_GIVEN = 0, 1, 2
BATCH_MAX_EPOCHS, BATCH_MAX_K = 32, 8


def _check(func, status):
    if status != 0:
        L = lib()
        raise KbmError(func, L.kbm_status_string(status).decode(),
                       L.kbm_last_error().decode())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype, name, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _host(a, dtype):
    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=dtype)


def _stack(T, H, W, times):
    times = _host(times, np.float64).reshape(-1)
    if times.shape[0] != T:
        raise ValueError(f"times has {times.shape[0]} entries, planes have {T}")
    return _Stack(W, H, T, times.ctypes.data), times


def make_planes(sci, var, mask, psf, times=None, stream=None, out=None):
    """psi, phi = correlation of I*w with the PSF and of w with PSF^2
    (w = inverse variance, zero where masked or unusable).  ``sci``/``var``
    are float32 ``[T][H][W]`` device tensors, ``mask`` uint8 or None, ``psf``
    a host ``[k][k]`` array.  ``out=(psi, phi)`` writes into given tensors
    (e.g. the planes a BatchedSearch was built on)."""
    T, H, W = sci.shape
    _dev(sci, torch.float32, "sci")
    _dev(var, torch.float32, "var", sci.shape)
    if mask is not None:
        _dev(mask, torch.uint8, "mask", sci.shape)
    psf = _host(psf, np.float32)
    if psf.ndim != 2 or psf.shape[0] != psf.shape[1]:
        raise ValueError("psf must be square")
    st, _t = _stack(T, H, W, np.zeros(T) if times is None else times)
    if out is not None:
        psi, phi = out
        _dev(psi, torch.float32, "psi", sci.shape)
        _dev(phi, torch.float32, "phi", sci.shape)
    else:
        psi = torch.empty_like(sci)
        phi = torch.empty_like(sci)
    _check("kbm_make_planes", lib().kbm_make_planes(
        C.byref(st), _ptr(sci), _ptr(var), _ptr(mask),
        psf.ctypes.data_as(C.c_void_p), psf.shape[0], _ptr(psi), _ptr(phi),
        _stream(stream)))
    return psi, phi


@dataclass
class SearchParams:
    k: int = 8
    min_obs: int = 1
    sigmag: bool = True
    q_lo: float = 0.25
    q_hi: float = 0.75
    coeff: float = 0.7413
    n_sigma: float = 2.0
    region: Optional[Sequence[int]] = None   # (x_begin, y_begin, x_end, y_end)


def _params(p: SearchParams, vels, W, H):
    vels = _host(vels, np.float32).reshape(-1, 2)
    x0, y0, x1, y1 = p.region if p.region is not None else (0, 0, W, H)
    sp = _SearchParams(vels.ctypes.data, vels.shape[0], int(p.k),
                       int(p.min_obs), int(bool(p.sigmag)), float(p.q_lo),
                       float(p.q_hi), float(p.coeff), float(p.n_sigma),
                       int(x0), int(y0), int(x1), int(y1))
    return sp, vels


def _alloc_results(Hr, Wr, k, device, want_lh_raw):
    shape = (Hr, Wr, k)
    out = dict(lh=torch.empty(shape, dtype=torch.float32, device=device),
               flux=torch.empty(shape, dtype=torch.float32, device=device),
               vel_idx=torch.empty(shape, dtype=torch.int32, device=device),
               n_obs=torch.empty(shape, dtype=torch.int16, device=device),
               keep=torch.empty(shape, dtype=torch.int64, device=device))
    out["lh_raw"] = (torch.empty(shape, dtype=torch.float32, device=device)
                     if want_lh_raw else None)
    r = _Results(out["lh"].data_ptr(), out["flux"].data_ptr(),
                 out["vel_idx"].data_ptr(), out["n_obs"].data_ptr(),
                 out["keep"].data_ptr(),
                 out["lh_raw"].data_ptr() if want_lh_raw else None)
    return out, r


def search_workspace_size(shapes_times_vels, params: Sequence[SearchParams]) -> int:
    """Workspace bytes for stacks given as ``[(T, H, W, times, vels), ...]``."""
    n = len(shapes_times_vels)
    stacks = (_Stack * n)()
    ps = (_SearchParams * n)()
    keep = []
    for j, ((T, H, W, times, vels), p) in enumerate(zip(shapes_times_vels, params)):
        stacks[j], t = _stack(T, H, W, times)
        ps[j], v = _params(p, vels, W, H)
        keep += [t, v]
    nbytes = C.c_size_t(0)
    _check("kbm_search_workspace_size", lib().kbm_search_workspace_size(
        stacks, ps, n, C.byref(nbytes)))
    return int(nbytes.value)


def _batch_ok(items):
    for it in items:
        T, H, W = it["psi"].shape
        p = it.get("params") or SearchParams()
        if T > BATCH_MAX_EPOCHS or p.k > BATCH_MAX_K or 8 * T * H * W >= 2 ** 32:
            return False
    return True


def search_batched(items, want_lh_raw=True, workspace=None, stream=None,
                   persistent=None, tune=TUNE_DEFAULT):
    """Search several independent stacks in one call.

    ``items`` is a list of dicts with keys psi, phi, times, vels, params
    (a SearchParams).  Returns one result dict per stack.

    ``persistent``: True runs the batched persistent kernel (one launch for
    all stacks, see BatchedSearch), False the per-stack launch sequence of
    kbm_search, None picks the persistent kernel when every stack is within
    its limits (T <= 32, k <= 8)."""
    if persistent is None:
        persistent = len(items) > 1 and _batch_ok(items)
    if persistent:
        with BatchedSearch(items, want_lh_raw=want_lh_raw, tune=tune,
                           workspace=workspace, stream=stream) as b:
            b.run(stream)
            if b.check(stream):
                raise KbmError("kbm_batch_run", "device error",
                               "a dependency wait of the persistent search gave up")
            return b.results
    n = len(items)
    stacks = (_Stack * n)()
    ps = (_SearchParams * n)()
    psi_p = (C.c_void_p * n)()
    phi_p = (C.c_void_p * n)()
    res = (_Results * n)()
    outs, hold = [], []
    for j, it in enumerate(items):
        psi, phi = it["psi"], it["phi"]
        _dev(psi, torch.float32, "psi")
        _dev(phi, torch.float32, "phi", psi.shape)
        T, H, W = psi.shape
        stacks[j], t = _stack(T, H, W, it["times"])
        p = it.get("params") or SearchParams()
        ps[j], v = _params(p, it["vels"], W, H)
        hold += [t, v]
        psi_p[j] = psi.data_ptr()
        phi_p[j] = phi.data_ptr()
        x0, y0, x1, y1 = p.region if p.region is not None else (0, 0, W, H)
        o, r = _alloc_results(y1 - y0, x1 - x0, p.k, psi.device, want_lh_raw)
        outs.append(o)
        res[j] = r
    L = lib()
    nbytes = C.c_size_t(0)
    _check("kbm_search_workspace_size",
           L.kbm_search_workspace_size(stacks, ps, n, C.byref(nbytes)))
    if workspace is None or workspace.numel() < nbytes.value:
        workspace = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8,
                                device=items[0]["psi"].device)
    _check("kbm_search", L.kbm_search(stacks, psi_p, phi_p, ps, res, n,
                                      _ptr(workspace), workspace.numel(),
                                      _stream(stream)))
    return outs


def search(psi, phi, times, vels, params: Optional[SearchParams] = None,
           want_lh_raw=True, workspace=None, stream=None, **kw):
    """Search one stack; ``kw`` may override SearchParams fields."""
    p = params or SearchParams()
    if kw:
        p = SearchParams(**{**p.__dict__, **kw})
    return search_batched([dict(psi=psi, phi=phi, times=times, vels=vels,
                                params=p)], want_lh_raw, workspace, stream,
                          persistent=False)[0]


def _batch_structs(items):
    n = len(items)
    stacks = (_Stack * n)()
    ps = (_SearchParams * n)()
    hold = []
    for j, it in enumerate(items):
        psi = it["psi"]
        T, H, W = psi.shape
        stacks[j], t = _stack(T, H, W, it["times"])
        p = it.get("params") or SearchParams()
        ps[j], v = _params(p, it["vels"], W, H)
        hold += [t, v]
    return stacks, ps, hold


def tune_cache_clear():
    """Forget the autotuner's in-process choices (the file cache stays)."""
    _check("kbm_tune_cache_clear", lib().kbm_tune_cache_clear())


def batch_workspace_size(items) -> int:
    """Workspace bytes of a BatchedSearch over ``items`` (dicts with psi
    (or shape via a tensor), times, vels, params)."""
    stacks, ps, _hold = _batch_structs(items)
    nbytes = C.c_size_t(0)
    _check("kbm_batch_workspace_size", lib().kbm_batch_workspace_size(
        stacks, ps, len(items), C.byref(nbytes)))
    return int(nbytes.value)


class BatchedSearch:
    """Batched persistent search over many stacks: one persistent kernel
    launch per run, replayed from a HIP graph captured at construction.

    ``items`` as for search_batched.  ``tune``: TUNE_DEFAULT, TUNE_AUTO
    (time candidate schedules on a probe and keep the fastest if a full run
    confirms that it beats the built-in schedule), or a
    Schedule / dict of its fields (used as given).  The plane tensors,
    results and workspace are held by this object: refill ``psi``/``phi`` in
    place and call run() again to search new images of the same geometry.
    ``results`` holds one result dict per stack (valid after run())."""

    def __init__(self, items, want_lh_raw=True, tune=TUNE_DEFAULT,
                 workspace=None, stream=None):
        n = len(items)
        L = lib()
        stacks, ps, self._hold = _batch_structs(items)
        psi_p = (C.c_void_p * n)()
        phi_p = (C.c_void_p * n)()
        res = (_Results * n)()
        self.results = []
        self._tensors = []
        for j, it in enumerate(items):
            psi, phi = it["psi"], it["phi"]
            _dev(psi, torch.float32, "psi")
            _dev(phi, torch.float32, "phi", psi.shape)
            T, H, W = psi.shape
            p = it.get("params") or SearchParams()
            psi_p[j] = psi.data_ptr()
            phi_p[j] = phi.data_ptr()
            x0, y0, x1, y1 = p.region if p.region is not None else (0, 0, W, H)
            o, r = _alloc_results(y1 - y0, x1 - x0, p.k, psi.device, want_lh_raw)
            self.results.append(o)
            res[j] = r
            self._tensors += [psi, phi]
        nbytes = C.c_size_t(0)
        _check("kbm_batch_workspace_size",
               L.kbm_batch_workspace_size(stacks, ps, n, C.byref(nbytes)))
        if workspace is None or workspace.numel() < nbytes.value:
            workspace = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8,
                                    device=items[0]["psi"].device)
        self.workspace = workspace
        sched = Schedule()
        if isinstance(tune, (Schedule, dict)):
            src = tune.as_dict() if isinstance(tune, Schedule) else tune
            for f, _ in Schedule._fields_:
                if f in src:
                    setattr(sched, f, src[f])
            mode = TUNE_GIVEN
        else:
            mode = int(tune)
        handle = C.c_void_p()
        _check("kbm_batch_create", L.kbm_batch_create(
            stacks, psi_p, phi_p, ps, res, n, _ptr(workspace), workspace.numel(),
            mode, C.byref(sched), _stream(stream), C.byref(handle)))
        self._h = handle
        self.schedule = sched.as_dict()

    def run(self, stream=None):
        """Enqueue one run (graph launch) on ``stream``."""
        if not self._h:
            raise KbmError("kbm_batch_run", "invalid argument", "plan is closed")
        _check("kbm_batch_run", lib().kbm_batch_run(self._h, _stream(stream)))
        return self.results

    def check(self, stream=None) -> bool:
        """Synchronise and return True if the last run's dependency waits
        gave up (its results are then invalid)."""
        stalled = C.c_int32(0)
        _check("kbm_batch_check", lib().kbm_batch_check(
            self._h, _stream(stream), C.byref(stalled)))
        return bool(stalled.value)

    def evaluated(self, stream=None) -> int:
        """Trajectory-epochs one run of the plan evaluates: the nominal count
        minus the tile-velocity pairs the kernel skips because no start
        pixel of the tile can keep min_obs epochs.  The skip depends only on
        the geometry, so the library counts it when the plan is created."""
        n = C.c_uint64(0)
        _check("kbm_batch_evaluated", lib().kbm_batch_evaluated(
            self._h, _stream(stream), C.byref(n)))
        return int(n.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().kbm_batch_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sigmag_filter(psi_curve, phi_curve=None, valid=None, q_lo=0.25,
                  q_hi=0.75, coeff=0.7413, n_sigma=2.0, want_lh=True,
                  stream=None):
    """sigma_G filter over ``[n][T]`` lightcurves; returns (keep int64 bit
    masks, filtered likelihood float32 or None)."""
    _dev(psi_curve, torch.float32, "psi_curve")
    n, T = psi_curve.shape
    if phi_curve is not None:
        _dev(phi_curve, torch.float32, "phi_curve", psi_curve.shape)
    if valid is not None:
        _dev(valid, torch.uint8, "valid", psi_curve.shape)
    keep = torch.empty(n, dtype=torch.int64, device=psi_curve.device)
    lh = torch.empty(n, dtype=torch.float32, device=psi_curve.device) if want_lh else None
    _check("kbm_sigmag_filter", lib().kbm_sigmag_filter(
        _ptr(psi_curve), _ptr(phi_curve), _ptr(valid), n, T, q_lo, q_hi,
        coeff, n_sigma, _ptr(keep), _ptr(lh), _stream(stream)))
    return keep, lh


def sigmag_filter_ex(psi_curve, phi_curve=None, valid=None, quantity=0, q_lo=0.25,
                     q_hi=0.75, coeff=None, n_sigma=2.0, lh_min=float("-inf"),
                     stream=None):
    """sigma_G filter variants: ``quantity`` 0 filters psi/sqrt(phi), 1 the
    flux psi/phi; ``coeff`` defaults to C of Eq. 3 for (q_lo, q_hi) (the
    paper's 0.7413 for the quartiles).  Returns (keep, lh, pass) with pass =
    lh >= lh_min."""
    _dev(psi_curve, torch.float32, "psi_curve")
    n, T = psi_curve.shape
    if phi_curve is not None:
        _dev(phi_curve, torch.float32, "phi_curve", psi_curve.shape)
    if valid is not None:
        _dev(valid, torch.uint8, "valid", psi_curve.shape)
    if coeff is None:
        coeff = 0.7413 if (q_lo, q_hi) == (0.25, 0.75) else sigmag_coeff(q_lo, q_hi)
    dev = psi_curve.device
    keep = torch.empty(n, dtype=torch.int64, device=dev)
    lh = torch.empty(n, dtype=torch.float32, device=dev)
    ok = torch.empty(n, dtype=torch.uint8, device=dev)
    _check("kbm_sigmag_filter_ex", lib().kbm_sigmag_filter_ex(
        _ptr(psi_curve), _ptr(phi_curve), _ptr(valid), n, T, int(quantity), q_lo, q_hi,
        float(coeff), n_sigma, float(lh_min), _ptr(keep), _ptr(lh), _ptr(ok),
        _stream(stream)))
    return keep, lh, ok.bool()


def detect(lh, n_obs, stamp_pass, min_obs, lh_min=10.0, stream=None):
    """Targeted-mode decision per trajectory: n_obs >= min_obs, L' >= lh_min
    and the stamp passes the moment cut (bool [n])."""
    _dev(lh, torch.float32, "lh")
    n = lh.shape[0]
    _dev(n_obs, torch.int16, "n_obs", (n,))
    sp = stamp_pass if stamp_pass.dtype == torch.uint8 else stamp_pass.to(torch.uint8)
    _dev(sp, torch.uint8, "stamp_pass", (n,))
    out = torch.empty(n, dtype=torch.uint8, device=lh.device)
    _check("kbm_detect", lib().kbm_detect(n, _ptr(lh), _ptr(n_obs), _ptr(sp), int(min_obs),
                                          float(lh_min), _ptr(out), _stream(stream)))
    return out.bool()


def sigmag_coeff(q_lo, q_hi) -> float:
    """C of Eq. 3 for a quantile pair (host computation in the library)."""
    c = C.c_double(0.0)
    _check("kbm_sigmag_coeff", lib().kbm_sigmag_coeff(float(q_lo), float(q_hi), C.byref(c)))
    return float(c.value)


def refine_forward(psi, phi, times, params, keep=None, stream=None, out=None):
    """Bilinear likelihood L for ``[n][4]`` params (x0, y0, vx, vy); written
    into ``out`` (float [n]) when given."""
    _dev(psi, torch.float32, "psi")
    _dev(phi, torch.float32, "phi", psi.shape)
    _dev(params, torch.float32, "params")
    T, H, W = psi.shape
    n = params.shape[0]
    if keep is not None:
        _dev(keep, torch.int64, "keep", (n,))
    st, _t = _stack(T, H, W, times)
    if out is None:
        lh = torch.empty(n, dtype=torch.float32, device=psi.device)
    else:
        lh = _dev(out, torch.float32, "out", (n,))
    _check("kbm_refine", lib().kbm_refine(
        C.byref(st), _ptr(psi), _ptr(phi), n, _ptr(params), _ptr(keep),
        _ptr(lh), None, None, None, None, _stream(stream)))
    return lh


def refine_backward(psi, phi, times, params, grad_lh, keep=None,
                    grad_psi=None, grad_phi=None, stream=None, out=None):
    """(lh, g * dL/dparams); g * dL/dpsi, g * dL/dphi are added into
    grad_psi / grad_phi when given.  ``out = (lh, grad_params)`` receives
    the two results when given (float [n] and [n][4])."""
    _dev(psi, torch.float32, "psi")
    _dev(phi, torch.float32, "phi", psi.shape)
    _dev(params, torch.float32, "params")
    T, H, W = psi.shape
    n = params.shape[0]
    _dev(grad_lh, torch.float32, "grad_lh", (n,))
    if keep is not None:
        _dev(keep, torch.int64, "keep", (n,))
    for g, nm in ((grad_psi, "grad_psi"), (grad_phi, "grad_phi")):
        if g is not None:
            _dev(g, torch.float32, nm, psi.shape)
    st, _t = _stack(T, H, W, times)
    if out is None:
        lh = torch.empty(n, dtype=torch.float32, device=psi.device)
        gp = torch.empty((n, 4), dtype=torch.float32, device=psi.device)
    else:
        lh = _dev(out[0], torch.float32, "out lh", (n,))
        gp = _dev(out[1], torch.float32, "out grad", (n, 4))
    _check("kbm_refine", lib().kbm_refine(
        C.byref(st), _ptr(psi), _ptr(phi), n, _ptr(params), _ptr(keep),
        _ptr(lh), _ptr(grad_lh), _ptr(gp), _ptr(grad_psi), _ptr(grad_phi),
        _stream(stream)))
    return lh, gp


class TrajLH(torch.autograd.Function):
    """L(params, psi, phi) through the bilinear adjoint kernel.

    ``TrajLH.apply(params, psi, phi, times, keep)``; gradients flow to
    params and, if they require grad, to psi and phi."""

    @staticmethod
    def forward(ctx, params, psi, phi, times, keep=None):
        params = params.contiguous()
        ctx.save_for_backward(params, psi, phi, keep)
        ctx.times = times
        return refine_forward(psi, phi, times, params, keep)

    @staticmethod
    def backward(ctx, grad_lh):
        params, psi, phi, keep = ctx.saved_tensors
        need_psi, need_phi = ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        gpsi = torch.zeros_like(psi) if need_psi else None
        gphi = torch.zeros_like(phi) if need_phi else None
        _, gp = refine_backward(psi, phi, ctx.times, params,
                                grad_lh.contiguous().float(), keep, gpsi, gphi)
        return gp, gpsi, gphi, None, None


def score_trajectories(psi, phi, times, params, params_search: Optional[SearchParams] = None,
                       want_lh_raw=True, stream=None, **kw):
    """The search's filtered likelihood for explicit trajectories
    ``params`` [n][4] (x0, y0, vx, vy; real-valued starts).  ``kw`` may
    override SearchParams fields (min_obs, sigmag, q_lo, q_hi, coeff,
    n_sigma).  Returns a dict of [n] tensors lh, flux, keep, n_obs, lh_raw."""
    p = params_search or SearchParams()
    if kw:
        p = SearchParams(**{**p.__dict__, **kw})
    _dev(psi, torch.float32, "psi")
    _dev(phi, torch.float32, "phi", psi.shape)
    T, H, W = psi.shape
    prm = _dev(params, torch.float32, "params")
    if prm.dim() != 2 or prm.shape[1] != 4:
        raise ValueError("params must be [n][4]")
    n = prm.shape[0]
    st, _t = _stack(T, H, W, times)
    dev = psi.device
    out = dict(lh=torch.empty(n, dtype=torch.float32, device=dev),
               flux=torch.empty(n, dtype=torch.float32, device=dev),
               keep=torch.empty(n, dtype=torch.int64, device=dev),
               n_obs=torch.empty(n, dtype=torch.int16, device=dev),
               lh_raw=torch.empty(n, dtype=torch.float32, device=dev) if want_lh_raw else None)
    _check("kbm_score_trajectories", lib().kbm_score_trajectories(
        C.byref(st), _ptr(psi), _ptr(phi), n, _ptr(prm), int(p.min_obs),
        int(bool(p.sigmag)), float(p.q_lo), float(p.q_hi), float(p.coeff),
        float(p.n_sigma), _ptr(out["lh"]), _ptr(out["flux"]), _ptr(out["keep"]),
        _ptr(out["n_obs"]), _ptr(out["lh_raw"]), _stream(stream)))
    return out


STAMP_LIMITS = (0.5, 0.5, 1.5, 36.5, 36.5)


def stamps(sci, var, mask, times, params, keep=None, radius=10, limits=None,
           want_coadd=True, stream=None):
    """Median coadded stamps along trajectories ``params`` [n][4] and the
    central-moment cut (Section 3.3).  Returns a dict: coadd [n][2r+1][2r+1]
    (or None), moments float64 [n][6] (sum, x, y, xy, xx, yy), pass bool [n]."""
    T, H, W = sci.shape
    _dev(sci, torch.float32, "sci")
    _dev(var, torch.float32, "var", sci.shape)
    if mask is not None:
        _dev(mask, torch.uint8, "mask", sci.shape)
    prm = _dev(params, torch.float32, "params")
    if prm.dim() != 2 or prm.shape[1] != 4:
        raise ValueError("params must be [n][4]")
    if keep is not None:
        _dev(keep, torch.int64, "keep", (prm.shape[0],))
    n = prm.shape[0]
    k = 2 * int(radius) + 1
    st, _t = _stack(T, H, W, times)
    dev = sci.device
    coadd = torch.empty((n, k, k), dtype=torch.float32, device=dev) if want_coadd else None
    moments = torch.empty((n, 6), dtype=torch.float64, device=dev)
    ok = torch.empty(n, dtype=torch.uint8, device=dev)
    lim = None if limits is None else (C.c_double * 5)(*[float(v) for v in limits])
    _check("kbm_stamps", lib().kbm_stamps(
        C.byref(st), _ptr(sci), _ptr(var), _ptr(mask), n, _ptr(prm), _ptr(keep),
        int(radius), lim, _ptr(coadd), _ptr(moments), _ptr(ok), _stream(stream)))
    return dict(coadd=coadd, moments=moments, passed=ok.bool(), pass_u8=ok)


def extract_workspace_size(Hr, Wr, k, num_vel) -> int:
    """Workspace bytes extract_top needs for [Hr][Wr][k] results."""
    nb = C.c_size_t(0)
    _check("kbm_extract_workspace_size", lib().kbm_extract_workspace_size(
        int(Hr), int(Wr), int(k), int(num_vel), C.byref(nb)))
    return int(nb.value)


def extract_top(res, vels, n_max, lh_min=-float("inf"), region_origin=(0, 0),
                workspace=None, stream=None):
    """Global top-``n_max`` result slots of a search by L' (>= lh_min).

    Returns a dict of device tensors (params [n][4] = x, y, vx, vy; lh; flux;
    keep; index; n_obs) trimmed to the number found, in flat-slot order."""
    lh_t = _dev(res["lh"], torch.float32, "lh")
    Hr, Wr, k = lh_t.shape
    dev = lh_t.device
    vels = _host(vels, np.float32).reshape(-1, 2)
    r = _Results(res["lh"].data_ptr(), res["flux"].data_ptr(),
                 res["vel_idx"].data_ptr(), res["n_obs"].data_ptr(),
                 res["keep"].data_ptr(), None)
    L = lib()
    nb = C.c_size_t(0)
    _check("kbm_extract_workspace_size",
           L.kbm_extract_workspace_size(Hr, Wr, k, vels.shape[0], C.byref(nb)))
    if workspace is None or workspace.numel() < nb.value:
        workspace = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=dev)
    n_max = int(n_max)
    out = dict(params=torch.empty((max(n_max, 1), 4), dtype=torch.float32, device=dev),
               lh=torch.empty(max(n_max, 1), dtype=torch.float32, device=dev),
               flux=torch.empty(max(n_max, 1), dtype=torch.float32, device=dev),
               keep=torch.empty(max(n_max, 1), dtype=torch.int64, device=dev),
               index=torch.empty(max(n_max, 1), dtype=torch.int64, device=dev),
               n_obs=torch.empty(max(n_max, 1), dtype=torch.int16, device=dev))
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    _check("kbm_extract_top", L.kbm_extract_top(
        C.byref(r), Hr, Wr, k, int(region_origin[0]), int(region_origin[1]),
        vels.ctypes.data_as(C.c_void_p), vels.shape[0], float(lh_min), n_max,
        _ptr(out["params"]), _ptr(out["lh"]), _ptr(out["flux"]), _ptr(out["keep"]),
        _ptr(out["index"]), _ptr(out["n_obs"]), _ptr(n_out), _ptr(workspace),
        workspace.numel(), _stream(stream)))
    n = int(n_out.item())
    return {key: v[:n] for key, v in out.items()}


def extract_top_noalloc(res, vels, n_max, out, n_out, lh_min=-float("inf"),
                        region_origin=(0, 0), stream=None):
    """extract_top for callers that cannot allocate: nothing is allocated here
    or in the library (its scratch is a static device array per GPU, so
    overlapping calls on one GPU race).  ``vels`` is a device float tensor
    [V][2]; ``out`` holds caller-allocated device tensors params [>=n_max][4],
    lh, flux, keep (int64), index (int64), n_obs (int16) of >= n_max rows
    (flux, keep, index, n_obs may be None); ``n_out`` a device int64 [1] that
    receives the number written.  Returns ``n_out``."""
    lh_t = _dev(res["lh"], torch.float32, "lh")
    Hr, Wr, k = lh_t.shape
    _dev(vels, torch.float32, "vels")
    if vels.dim() != 2 or vels.shape[1] != 2:
        raise ValueError("vels must be a device float tensor [V][2]")
    n_max = int(n_max)
    for key, dt in (("params", torch.float32), ("lh", torch.float32),
                    ("flux", torch.float32), ("keep", torch.int64),
                    ("index", torch.int64), ("n_obs", torch.int16)):
        t = out.get(key)
        if t is None:
            if key in ("params", "lh"):
                raise ValueError(f"out[{key!r}] is required")
            continue
        _dev(t, dt, key)
        if t.shape[0] < n_max:
            raise ValueError(f"out[{key!r}] holds {t.shape[0]} rows, n_max is {n_max}")
    _dev(n_out, torch.int64, "n_out")
    r = _Results(res["lh"].data_ptr(), res["flux"].data_ptr(),
                 res["vel_idx"].data_ptr(), res["n_obs"].data_ptr(),
                 res["keep"].data_ptr(), None)
    _check("kbm_extract_top_noalloc", lib().kbm_extract_top_noalloc(
        C.byref(r), Hr, Wr, k, int(region_origin[0]), int(region_origin[1]),
        _ptr(vels), vels.shape[0], float(lh_min), n_max,
        _ptr(out["params"]), _ptr(out["lh"]), _ptr(out.get("flux")),
        _ptr(out.get("keep")), _ptr(out.get("index")), _ptr(out.get("n_obs")),
        _ptr(n_out), _stream(stream)))
    return n_out


def adam_step(params, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8,
              maximize=True, stream=None):
    """One in-place Adam update of ``params`` [n][cols] (per-column lr)."""
    for t, nm in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
        _dev(t, torch.float32, nm, params.shape)
    n, cols = params.shape
    lr = np.ascontiguousarray(np.broadcast_to(np.asarray(lr, np.float32), (cols,)))
    _check("kbm_adam_step", lib().kbm_adam_step(
        _ptr(params), _ptr(grad), _ptr(m), _ptr(v), n, cols,
        lr.ctypes.data_as(C.c_void_p), beta1, beta2, eps, int(step),
        int(bool(maximize)), _stream(stream)))


_lr_tables = {}


def _refine_lr_table(times, steps, lr_pos, lr_vel, cosine):
    """_refine_lrs as a float32 [steps][4] array, kept per schedule (the
    refinement is called once per step of a search loop)."""
    key = (tuple(np.asarray(times, np.float64).tolist()), int(steps), float(lr_pos),
           None if lr_vel is None else float(lr_vel), bool(cosine))
    tab = _lr_tables.get(key)
    if tab is None:
        tab = np.ascontiguousarray(
            np.asarray(_refine_lrs(times, steps, lr_pos, lr_vel, cosine), np.float32))
        if len(_lr_tables) > 64:
            _lr_tables.clear()
        _lr_tables[key] = tab
    return tab


def _refine_lrs(times, steps, lr_pos, lr_vel, cosine):
    """Per-step Adam step sizes [steps][4] of the refinement loop."""
    t = np.asarray(times, np.float64)
    span = float(t.max() - t.min()) or 1.0
    lr_vel = lr_pos / span if lr_vel is None else lr_vel
    out = []
    for it in range(1, steps + 1):
        scale = 0.5 * (1.0 + np.cos(np.pi * (it - 1) / steps)) if cosine else 1.0
        out.append([lr_pos * scale, lr_pos * scale, lr_vel * scale, lr_vel * scale])
    return out


def _refine_steps(psi, phi, times, p, m, v, g, lh, ones, keep, lrs, stream):
    """The refinement loop on fixed buffers: moments cleared by a kernel,
    then per step the adjoint kernel and one Adam kernel, then L at the
    final parameters.  Only kernel launches (capturable)."""
    m.zero_()
    v.zero_()
    for it, lr in enumerate(lrs, start=1):
        refine_backward(psi, phi, times, p, ones, keep, stream=stream, out=(lh, g))
        adam_step(p, g, m, v, lr, it, maximize=True, stream=stream)
    refine_forward(psi, phi, times, p, keep, stream=stream, out=lh)


REFINE_MAX_FUSED_STEPS = 64


def refine_adam(psi, phi, times, params, lrs, keep=None, beta1=0.9, beta2=0.999,
                eps=1e-8, stream=None):
    """The whole Adam loop in one kernel launch (kbm_refine_adam): updates
    ``params`` [n][4] in place with the per-step step sizes ``lrs``
    [steps][4] and returns L at the final parameters."""
    _dev(psi, torch.float32, "psi")
    _dev(phi, torch.float32, "phi", psi.shape)
    _dev(params, torch.float32, "params")
    T, H, W = psi.shape
    n = params.shape[0]
    if keep is not None:
        _dev(keep, torch.int64, "keep", (n,))
    lr = lrs if (isinstance(lrs, np.ndarray) and lrs.dtype == np.float32 and lrs.ndim == 2
                 and lrs.shape[1] == 4 and lrs.flags.c_contiguous) \
        else np.ascontiguousarray(np.asarray(lrs, np.float32).reshape(-1, 4))
    st, _t = _stack(T, H, W, times)
    lh = torch.empty(n, dtype=torch.float32, device=psi.device)
    _check("kbm_refine_adam", lib().kbm_refine_adam(
        C.byref(st), _ptr(psi), _ptr(phi), n, _ptr(params), _ptr(keep),
        lr.ctypes.data_as(C.c_void_p), lr.shape[0], beta1, beta2, eps, _ptr(lh),
        _stream(stream)))
    return lh


def refine(psi, phi, times, params0, keep=None, steps=50, lr_pos=0.3,
           lr_vel=None, cosine=True, stream=None, mode="fused"):
    """Gradient-ascent refinement of candidates with the bilinear adjoint.

    Each step runs the adjoint (L and dL/dparams) and one Adam update.
    Position steps are ``lr_pos`` pixels; velocity steps default to
    ``lr_pos / t_span`` px/day so that both move the track by similar
    amounts.  A cosine decay scales both.  ``mode``: "fused" runs the whole
    loop in one kernel launch (up to 64 steps; more fall back to "graph"),
    "graph" replays the per-step adjoint and Adam kernels from a HIP graph
    captured once per problem (see Refiner), "eager" launches them one by
    one.  All three give the same bits.  Returns (params, lh) where lh is the
    likelihood at the returned params."""
    if mode not in ("fused", "graph", "eager"):
        raise ValueError(f"mode must be fused, graph or eager, not {mode!r}")
    if params0.shape[0] == 0:  # nothing to launch (and no graph to capture)
        _dev(params0, torch.float32, "params0")
        return (params0.detach().clone(),
                torch.empty(0, dtype=torch.float32, device=params0.device))
    if mode == "fused" and steps <= REFINE_MAX_FUSED_STEPS:
        p = params0.detach().clone().contiguous()
        lh = refine_adam(psi, phi, times, p,
                         _refine_lr_table(times, steps, lr_pos, lr_vel, cosine), keep,
                         stream=stream)
        return p, lh
    if mode != "eager":
        r = _refiner_for(psi, phi, times, params0.shape[0], keep is not None, steps,
                         lr_pos, lr_vel, cosine)
        p, lh = r.run(params0.contiguous(), keep, stream=stream)
        return p.clone(), lh.clone()
    p = params0.detach().clone().contiguous()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    g = torch.empty_like(p)
    lh = torch.empty(p.shape[0], dtype=torch.float32, device=p.device)
    ones = torch.ones(p.shape[0], dtype=torch.float32, device=p.device)
    _refine_steps(psi, phi, times, p, m, v, g, lh, ones, keep,
                  _refine_lrs(times, steps, lr_pos, lr_vel, cosine), stream)
    return p, lh


class Refiner:
    """The refinement loop of ``refine`` for ``n`` candidates on fixed planes,
    captured once into a HIP graph (every step's adjoint and Adam kernels,
    the cosine step sizes baked in) and replayed per call: one graph launch
    instead of 2 * steps + 3 kernel launches from Python.

    ``run(params0, keep)`` copies the starting parameters (and keep masks, if
    the refiner was made ``with_keep``) into the graph's buffers, replays it
    on the current (or given) stream and returns its (params, lh) buffers,
    valid until the next run.  The planes must stay allocated while the
    refiner lives (their addresses are baked into the graph)."""

    def __init__(self, psi, phi, times, n, with_keep=False, steps=50, lr_pos=0.3,
                 lr_vel=None, cosine=True):
        _dev(psi, torch.float32, "psi")
        _dev(phi, torch.float32, "phi", psi.shape)
        dev = psi.device
        self.n, self.with_keep = int(n), bool(with_keep)
        self.psi, self.phi, self.times = psi, phi, np.asarray(times, np.float64).copy()
        self.p = torch.zeros((self.n, 4), dtype=torch.float32, device=dev)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.g = torch.zeros_like(self.p)
        self.lh = torch.zeros(self.n, dtype=torch.float32, device=dev)
        self.ones = torch.ones(self.n, dtype=torch.float32, device=dev)
        self.keep = torch.zeros(self.n, dtype=torch.int64, device=dev) if with_keep else None
        self.lrs = _refine_lrs(times, steps, lr_pos, lr_vel, cosine)
        self.graph = None
        if self.n == 0:
            return
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            # one eager pass loads the kernels' code objects before capture
            self._steps()
        torch.cuda.current_stream(dev).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._steps()

    def _steps(self):
        _refine_steps(self.psi, self.phi, self.times, self.p, self.m, self.v, self.g,
                      self.lh, self.ones, self.keep, self.lrs, None)

    def run(self, params0, keep=None, stream=None):
        _dev(params0, torch.float32, "params0", (self.n, 4))
        if (keep is not None) != self.with_keep:
            raise ValueError("keep must be given exactly when the refiner was made with_keep")
        if self.n == 0:
            return self.p, self.lh
        s = torch.cuda.current_stream() if stream is None else stream
        with torch.cuda.stream(s):
            self.p.copy_(params0)
            if keep is not None:
                self.keep.copy_(_dev(keep, torch.int64, "keep", (self.n,)))
            self.graph.replay()
        return self.p, self.lh


_refiners = {}


def _refiner_for(psi, phi, times, n, with_keep, steps, lr_pos, lr_vel, cosine):
    """A Refiner for this problem, reused while the planes, times, size and
    step sizes stay the same (the four most recent are kept)."""
    key = (psi.data_ptr(), phi.data_ptr(), tuple(psi.shape), psi.device.index,
           tuple(np.asarray(times, np.float64).tolist()), int(n), bool(with_keep),
           int(steps), float(lr_pos), None if lr_vel is None else float(lr_vel),
           bool(cosine))
    r = _refiners.pop(key, None)
    if r is None:
        r = Refiner(psi, phi, times, n, with_keep, steps, lr_pos, lr_vel, cosine)
        while len(_refiners) >= 4:
            _refiners.pop(next(iter(_refiners)))
    _refiners[key] = r
    return r

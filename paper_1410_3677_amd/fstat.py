"""Thin ctypes binding of the C ABI in include/fstat.h (argument marshalling only).

Every step of the search runs in the HIP library libfstat.so; this module
only converts Python/PyTorch arguments into the C structs and pointers.  It
raises if the library is missing: there is no fallback implementation.
PyTorch provides device memory and streams.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfstat.so")

# status codes
OK, E_INVAL, E_NOMEM, E_ADMISSION, E_OVERFLOW, E_DEVICE, E_STATE, E_NOT_IMPLEMENTED = range(8)
PREC_FP64, PREC_MIXED = 0, 1
FORM_SIMPLIFIED, FORM_FULL = 0, 1
KERNEL_SKY_PREP, KERNEL_RESAMPLE, KERNEL_TEMPLATE_A, KERNEL_TEMPLATE_B = range(4)
KERNEL_NAMES = ("sky_prep", "resample", "template_a", "template_b")

EXPORTED = ("fstat_options_default", "fstat_plan", "fstat_plan_workspace_size", "fstat_plan_set_workspace",
            "fstat_search_batch", "fstat_candidates", "fstat_twoF_spectrum", "fstat_twoF_spectrum_static",
            "fstat_sky_stages",
            "fstat_profile_enable", "fstat_profile_read", "fstat_plan_info", "fstat_autotune", "fstat_destroy",
            "fstat_strerror", "fstat_last_error", "fstat_vet_param_count", "fstat_vet_create",
            "fstat_vet_set_params", "fstat_vet_get_params", "fstat_vet_forward", "fstat_vet_gradient",
            "fstat_vet_adam_step", "fstat_vet_destroy", "fstat_plan_attach_vetter", "fstat_plan_vet_candidates",
            "fstat_lattice_sky_range", "fstat_lattice_sky", "fstat_search_lattice")


class fstat_segment(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dt", ctypes.c_double), ("f_off", ctypes.c_double),
                ("sigma2", ctypes.c_double), ("x", ctypes.c_void_p), ("r_ssb", ctypes.c_void_p),
                ("lat", ctypes.c_double), ("gamma", ctypes.c_double), ("phi_r", ctypes.c_double)]


class fstat_options(ctypes.Structure):
    _fields_ = [("nfft", ctypes.c_int32), ("k_min", ctypes.c_int32), ("k_max", ctypes.c_int32),
                ("threshold_2F", ctypes.c_double), ("precision", ctypes.c_int32), ("form", ctypes.c_int32),
                ("candidate_capacity", ctypes.c_int64), ("workspace_budget_bytes", ctypes.c_size_t),
                ("templates_per_launch", ctypes.c_int32), ("skies_per_batch", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("tuning_cache_path", ctypes.c_char_p),
                ("interbinning", ctypes.c_int32)]


class fstat_candidate(ctypes.Structure):
    _fields_ = [("f_hz", ctypes.c_double), ("fdot", ctypes.c_double), ("alpha", ctypes.c_double),
                ("delta", ctypes.c_double), ("twoF", ctypes.c_double)]


class fstat_candidate_key(ctypes.Structure):
    _fields_ = [("search", ctypes.c_int32), ("segment", ctypes.c_int32), ("sky", ctypes.c_int32),
                ("fdot_idx", ctypes.c_int32), ("bin", ctypes.c_int32), ("vet_score", ctypes.c_float)]


class fstat_lattice(ctypes.Structure):
    _fields_ = [("M", ctypes.c_double * 16), ("epsilon", ctypes.c_double), ("f_ref", ctypes.c_double)]


def lattice(M, epsilon: float, f_ref: float) -> fstat_lattice:
    """fstat_lattice from a 4x4 generator matrix (rows: frequency, spindown, sky, sky)."""
    lat = fstat_lattice()
    flat = np.ascontiguousarray(np.asarray(M, dtype=np.float64).reshape(16))
    for i in range(16):
        lat.M[i] = float(flat[i])
    lat.epsilon = float(epsilon)
    lat.f_ref = float(f_ref)
    return lat


CANDIDATE_NP = np.dtype([("f_hz", "<f8"), ("fdot", "<f8"), ("alpha", "<f8"), ("delta", "<f8"), ("twoF", "<f8")])
KEY_NP = np.dtype([("search", "<i4"), ("segment", "<i4"), ("sky", "<i4"), ("fdot_idx", "<i4"), ("bin", "<i4"),
                   ("vet_score", "<f4")])

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libfstat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1410_3677_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, dbl, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "fstat_options_default": (None, [ctypes.POINTER(fstat_options)]),
        "fstat_plan": (i32, [ctypes.POINTER(fstat_segment), i32, ctypes.POINTER(fstat_options), ctypes.POINTER(P)]),
        "fstat_plan_workspace_size": (i32, [P, ctypes.POINTER(sz)]),
        "fstat_plan_set_workspace": (i32, [P, P, sz]),
        "fstat_search_batch": (i32, [P, i32, P, P, i32, P, i32, P]),
        "fstat_candidates": (i32, [P, P, P, i64, ctypes.POINTER(i64)]),
        "fstat_twoF_spectrum": (i32, [P, i32, P, P, i32, P, i32, P, P]),
        "fstat_twoF_spectrum_static": (i32, [P, i32, P, P, i32, P, i32, P, P]),
        "fstat_sky_stages": (i32, [P, i32, dbl, dbl, P, P, P, P, P, P, P, P]),
        "fstat_profile_enable": (i32, [P, i32]),
        "fstat_profile_read": (i32, [P, i32, ctypes.POINTER(i64), ctypes.POINTER(dbl), i32]),
        "fstat_plan_info": (i32, [P, i32] + [ctypes.POINTER(i32)] * 7),
        "fstat_autotune": (i32, [P, i32, dbl, P]),
        "fstat_destroy": (i32, [P]),
        "fstat_strerror": (ctypes.c_char_p, [i32]),
        "fstat_vet_param_count": (i64, []),
        "fstat_vet_create": (i32, [i32, ctypes.POINTER(P)]),
        "fstat_vet_set_params": (i32, [P, P, i64]),
        "fstat_vet_get_params": (i32, [P, P, i64]),
        "fstat_vet_forward": (i32, [P, P, i64, P, P]),
        "fstat_vet_gradient": (i32, [P, P, P, i64, P, P, P]),
        "fstat_vet_adam_step": (i32, [P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, P]),
        "fstat_vet_destroy": (i32, [P]),
        "fstat_plan_attach_vetter": (i32, [P, P, i64]),
        "fstat_plan_vet_candidates": (i32, [P, P]),
        "fstat_last_error": (ctypes.c_char_p, [P]),
        "fstat_lattice_sky_range": (i32, [ctypes.POINTER(fstat_lattice), ctypes.POINTER(i32)]),
        "fstat_lattice_sky": (i32, [ctypes.POINTER(fstat_lattice), i32, ctypes.POINTER(i32), i64, P, P, P, P, P, P,
                                    P]),
        "fstat_search_lattice": (i32, [P, i32, ctypes.POINTER(fstat_lattice), P, P, P, P, i32, i32, i32, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class FstatError(RuntimeError):
    def __init__(self, status: int, text: str):
        super().__init__(f"fstat status {status}: {text}")
        self.status = status


def _check(st: int, plan_handle=None):
    if st != OK:
        lib = load()
        detail = lib.fstat_last_error(plan_handle).decode()
        raise FstatError(st, f"{lib.fstat_strerror(st).decode()} ({detail})")


def options_default() -> fstat_options:
    o = fstat_options()
    load().fstat_options_default(ctypes.byref(o))
    return o


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    return int(getattr(stream, "cuda_stream", stream))


class Plan:
    """An fstat plan over device-resident segments.

    segments: sequence of dicts with keys n, dt, f_off, sigma2, x (device float64 tensor),
    r (device float64 tensor of shape (3, n)), lat, gamma, phi_r.
    """

    def __init__(self, segments: Sequence[dict], options: Optional[fstat_options] = None,
                 workspace_from_torch: bool = True, **opts):
        import torch
        self.lib = load()
        o = options if options is not None else options_default()
        for k, v in opts.items():
            if k == "tuning_cache_path" and isinstance(v, str):
                self._cache_path = v.encode()   # keep the bytes alive for the plan
                v = self._cache_path
            setattr(o, k, v)
        self.options = o
        self._keep = []
        arr = (fstat_segment * len(segments))()
        for i, s in enumerate(segments):
            x, r = s["x"], s["r"]
            assert x.dtype == torch.float64 and r.dtype == torch.float64 and x.is_cuda and r.is_cuda
            assert x.is_contiguous() and r.is_contiguous() and r.numel() == 3 * s["n"] and x.numel() == s["n"]
            self._keep += [x, r]
            arr[i] = fstat_segment(int(s["n"]), float(s["dt"]), float(s["f_off"]), float(s["sigma2"]),
                                   _ptr(x), _ptr(r), float(s["lat"]), float(s["gamma"]), float(s["phi_r"]))
        h = ctypes.c_void_p()
        _check(self.lib.fstat_plan(arr, len(segments), ctypes.byref(o), ctypes.byref(h)))
        self.handle = h
        self.nseg = len(segments)
        self.fp64 = o.precision == PREC_FP64
        self.workspace = None
        if workspace_from_torch:
            self._set_torch_workspace()

    def info(self, segment: int = 0) -> dict:
        v = [ctypes.c_int32() for _ in range(7)]
        _check(self.lib.fstat_plan_info(self.handle, segment, *[ctypes.byref(x) for x in v]), self.handle)
        return dict(zip(("nfft", "p", "q", "templates_per_launch", "skies_per_batch", "pass_a_variant",
                         "pass_b_variant"), [x.value for x in v]))

    def autotune(self, segment: int = 0, budget_ms: float = 2000.0, stream=None) -> dict:
        """Run the autotuner, then give the plan a torch workspace of the new size."""
        import torch
        if self.workspace is not None:
            raise RuntimeError("autotune must run before a workspace is set: create the Plan with "
                               "workspace_from_torch=False")
        _check(self.lib.fstat_autotune(self.handle, segment, float(budget_ms), _stream_handle(stream)), self.handle)
        self._set_torch_workspace()
        return self.info(segment)

    def _set_torch_workspace(self):
        import torch
        nbytes = ctypes.c_size_t()
        _check(self.lib.fstat_plan_workspace_size(self.handle, ctypes.byref(nbytes)), self.handle)
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device="cuda")
        aligned = (_ptr(self.workspace) + 255) & ~255
        _check(self.lib.fstat_plan_set_workspace(self.handle, aligned, int(nbytes.value)), self.handle)

    def search_batch(self, segment: int, alpha, delta, fdot, stream=None):
        self._keep_lists = (alpha, delta, fdot)
        _check(self.lib.fstat_search_batch(self.handle, segment, _ptr(alpha), _ptr(delta), int(alpha.numel()),
                                           _ptr(fdot), int(fdot.numel()), _stream_handle(stream)), self.handle)

    def candidates(self, capacity: Optional[int] = None, allow_overflow: bool = False, out=None):
        """Drain the candidates: (records, keys, n_found) as numpy structured arrays.
        `out` = (records, keys) from candidate_buffers() is filled instead of new arrays."""
        n = ctypes.c_int64()
        if out is not None:
            recs, keys = out
            capacity = min(len(recs), len(keys)) if capacity is None else min(capacity, len(recs), len(keys))
        else:
            if capacity is None:
                capacity = int(self.options.candidate_capacity)
            recs = np.zeros(capacity, dtype=CANDIDATE_NP)
            keys = np.zeros(capacity, dtype=KEY_NP)
        st = self.lib.fstat_candidates(self.handle, recs.ctypes.data, keys.ctypes.data, capacity, ctypes.byref(n))
        if st == E_OVERFLOW and allow_overflow:
            m = min(capacity, n.value, int(self.options.candidate_capacity))
            return recs[:m], keys[:m], n.value
        _check(st, self.handle)
        return recs[: n.value], keys[: n.value], n.value

    def candidate_count(self, allow_overflow: bool = False) -> int:
        """Drain the candidates, returning only how many were found (nothing is copied)."""
        n = ctypes.c_int64()
        st = self.lib.fstat_candidates(self.handle, None, None, 0, ctypes.byref(n))
        if not (st == E_OVERFLOW and allow_overflow):
            _check(st, self.handle)
        return n.value

    def search_lattice(self, segment: int, lat: fstat_lattice, sky: dict, s_lo: int, s_hi: int, spectrum=None,
                       stream=None):
        """Search the lattice templates: `sky` as returned by lattice_sky (device tensors),
        spindown integers s_lo..s_hi.  With `spectrum` (device tensor), store 2F instead."""
        self._keep_lists = (sky, spectrum)
        _check(self.lib.fstat_search_lattice(self.handle, segment, ctypes.byref(lat), _ptr(sky["alpha"]),
                                             _ptr(sky["delta"]), _ptr(sky["w_freq"]), _ptr(sky["w_spin"]),
                                             int(sky["alpha"].numel()), int(s_lo), int(s_hi), _ptr(spectrum),
                                             _stream_handle(stream)), self.handle)

    def twoF_spectrum(self, segment: int, alpha, delta, fdot, out, stream=None):
        _check(self.lib.fstat_twoF_spectrum(self.handle, segment, _ptr(alpha), _ptr(delta), int(alpha.numel()),
                                            _ptr(fdot), int(fdot.numel()), _ptr(out), _stream_handle(stream)),
               self.handle)

    def twoF_spectrum_static(self, segment: int, alpha, delta, fdot, out, stream=None):
        """twoF_spectrum on the library's static device scratch (allocates nothing)."""
        _check(self.lib.fstat_twoF_spectrum_static(self.handle, segment, _ptr(alpha), _ptr(delta),
                                                   int(alpha.numel()), _ptr(fdot), int(fdot.numel()), _ptr(out),
                                                   _stream_handle(stream)), self.handle)

    def sky_stages(self, segment: int, alpha: float, delta: float, abc=None, za=None, zb=None, ua=None, ub=None,
                   zta=None, ztb=None, stream=None):
        _check(self.lib.fstat_sky_stages(self.handle, segment, float(alpha), float(delta), _ptr(abc), _ptr(za),
                                         _ptr(zb), _ptr(ua), _ptr(ub), _ptr(zta), _ptr(ztb),
                                         _stream_handle(stream)), self.handle)

    def profile_enable(self, on: bool = True):
        _check(self.lib.fstat_profile_enable(self.handle, 1 if on else 0), self.handle)

    def profile_read(self, kernel_class: int, reset: bool = False):
        n, ms = ctypes.c_int64(), ctypes.c_double()
        _check(self.lib.fstat_profile_read(self.handle, kernel_class, ctypes.byref(n), ctypes.byref(ms),
                                           1 if reset else 0), self.handle)
        return n.value, ms.value

    def attach_vetter(self, vetter, patch_capacity: int):
        self._vetter = vetter
        _check(self.lib.fstat_plan_attach_vetter(self.handle, vetter.handle if vetter else None, int(patch_capacity)),
               self.handle)

    def vet_candidates(self, stream=None):
        _check(self.lib.fstat_plan_vet_candidates(self.handle, _stream_handle(stream)), self.handle)

    def destroy(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.fstat_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def candidate_buffers(capacity: int, pinned: bool = False):
    """Host arrays (records, keys) of `capacity` entries for Plan.candidates(out=...).
    pinned=True places them in page-locked memory (allocated by PyTorch), which the
    drain's device-to-host copies reach directly; the arrays keep that memory alive."""
    if not pinned:
        return np.empty(capacity, dtype=CANDIDATE_NP), np.empty(capacity, dtype=KEY_NP)
    import torch
    out = []
    for dt in (CANDIDATE_NP, KEY_NP):
        t = torch.empty(max(capacity, 1) * dt.itemsize, dtype=torch.uint8, pin_memory=True)
        a = t.numpy().view(dt)[:capacity]
        out.append(_Pinned(a, t))
    return tuple(out)


class _Pinned(np.ndarray):
    """A numpy view of page-locked memory that holds the tensor owning it."""

    def __new__(cls, arr, owner):
        obj = arr.view(cls)
        obj._owner = owner
        return obj

    def __array_finalize__(self, obj):
        self._owner = getattr(obj, "_owner", None)


def lattice_sky_range(lat: fstat_lattice):
    """(n_lo, n_hi, m_lo, m_hi): the box of the sky integers (host computation)."""
    box = (ctypes.c_int32 * 4)()
    _check(load().fstat_lattice_sky_range(ctypes.byref(lat), box))
    return tuple(int(v) for v in box)


def lattice_sky(lat: fstat_lattice, hemisphere: int, box=None, capacity: Optional[int] = None, stream=None) -> dict:
    """Sky points of the lattice on one hemisphere, computed on the current device:
    {"alpha", "delta", "w_freq", "w_spin", "nm", "count"} (device tensors cut to the
    points written; "count" is the number on the sky, which may exceed the capacity)."""
    import torch
    if box is None:
        box = lattice_sky_range(lat)
    if capacity is None:
        capacity = (box[1] - box[0] + 1) * (box[3] - box[2] + 1)
    cap = max(int(capacity), 1)
    out = torch.empty((4, cap), dtype=torch.float64, device="cuda")
    nm = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    b = (ctypes.c_int32 * 4)(*[int(v) for v in box])
    _check(load().fstat_lattice_sky(ctypes.byref(lat), int(hemisphere), b, int(capacity), _ptr(out[0]), _ptr(out[1]),
                                    _ptr(out[2]), _ptr(out[3]), _ptr(nm), _ptr(count), _stream_handle(stream)))
    total = int(count.item())
    k = min(total, int(capacity))
    return {"alpha": out[0, :k], "delta": out[1, :k], "w_freq": out[2, :k], "w_spin": out[3, :k], "nm": nm[:k],
            "count": total}


def segment_to_device(seg) -> dict:
    """Copy a synthetic segment (object with n, dt, f_off, sigma2, x, r, lat, gamma, phi_r) to the GPU."""
    import torch
    return dict(n=seg.n, dt=seg.dt, f_off=seg.f_off, sigma2=seg.sigma2,
                x=torch.as_tensor(np.ascontiguousarray(seg.x), dtype=torch.float64, device="cuda"),
                r=torch.as_tensor(np.ascontiguousarray(seg.r), dtype=torch.float64, device="cuda"),
                lat=seg.lat, gamma=seg.gamma, phi_r=seg.phi_r)


class Vetter:
    """The candidate-vetting network on the GPU (parameters FP32, products BF16/FP32)."""

    def __init__(self, max_batch: int = 512):
        self.lib = load()
        h = ctypes.c_void_p()
        _check(self.lib.fstat_vet_create(int(max_batch), ctypes.byref(h)))
        self.handle = h
        self.max_batch = max_batch
        self.n_params = int(self.lib.fstat_vet_param_count())

    def _chk(self, st):
        if st != OK:
            raise FstatError(st, self.lib.fstat_strerror(st).decode())

    def set_params(self, theta: np.ndarray):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        assert t.size == self.n_params
        self._chk(self.lib.fstat_vet_set_params(self.handle, t.ctypes.data, t.size))

    def get_params(self) -> np.ndarray:
        t = np.empty(self.n_params, dtype=np.float32)
        self._chk(self.lib.fstat_vet_get_params(self.handle, t.ctypes.data, t.size))
        return t

    def forward(self, patches, logits, stream=None):
        self._chk(self.lib.fstat_vet_forward(self.handle, _ptr(patches), int(patches.shape[0]), _ptr(logits),
                                             _stream_handle(stream)))

    def gradient(self, patches, labels, loss=None, grad=None, stream=None):
        self._chk(self.lib.fstat_vet_gradient(self.handle, _ptr(patches), _ptr(labels), int(patches.shape[0]),
                                              _ptr(loss), _ptr(grad), _stream_handle(stream)))

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
        self._chk(self.lib.fstat_vet_adam_step(self.handle, lr, beta1, beta2, eps, _stream_handle(stream)))

    def destroy(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.fstat_vet_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

"""C-ABI checks that need no GPU: symbols, option defaults, argument validation, admission.

Validation and admission run on the host before any device call, so these
paths are exercised here with placeholder (never dereferenced) pointers.
"""
import ctypes
import os
import re

import pytest

from paper_1410_3677_amd import fstat as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fstat.h")
FAKE_PTR = 0x10000  # placeholder device address; validation never dereferences it

pytestmark = pytest.mark.skipif(not os.path.exists(F.LIB_PATH), reason="libfstat.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fstat_[A-Za-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = F.load()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(F.EXPORTED)


def test_strerror_texts():
    lib = F.load()
    assert lib.fstat_strerror(F.OK) == b"success"
    assert b"budget" in lib.fstat_strerror(F.E_ADMISSION)
    assert b"overflow" in lib.fstat_strerror(F.E_OVERFLOW)
    assert lib.fstat_strerror(99) == b"unknown status"


def test_option_defaults():
    o = F.options_default()
    assert o.nfft == 0 and o.k_min == 0 and o.k_max == 0
    assert o.threshold_2F == 20.0
    assert o.precision == F.PREC_MIXED and o.form == F.FORM_SIMPLIFIED
    assert o.candidate_capacity == 1 << 24
    assert o.workspace_budget_bytes == 0
    assert o.use_graph == 1 and o.tuning_cache_path is None


def _seg(n=86164, **kw):
    s = F.fstat_segment(n, 2.0, 100.0, 1.0, FAKE_PTR, FAKE_PTR, 0.81, 3.0, 0.0)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def _plan(segs, **opts):
    lib = F.load()
    o = F.options_default()
    for k, v in opts.items():
        setattr(o, k, v)
    arr = (F.fstat_segment * len(segs))(*segs)
    h = ctypes.c_void_p()
    st = lib.fstat_plan(arr, len(segs), ctypes.byref(o), ctypes.byref(h))
    return st, h, lib.fstat_last_error(None).decode()


@pytest.mark.parametrize("seg,opts,needle", [
    (dict(n=500), {}, "n=500"),
    (dict(dt=0.0), {}, "dt"),
    (dict(sigma2=-1.0), {}, "sigma2"),
    (dict(f_off=float("nan")), {}, "finite"),
    (dict(x=None), {}, "device pointers"),
    (dict(), dict(nfft=100000), "power of two"),
    (dict(), dict(nfft=131072), "power of two"),   # < 2n
    (dict(), dict(precision=7), "precision"),
    (dict(), dict(form=3), "form"),
    (dict(), dict(candidate_capacity=0), "capacity"),
    (dict(), dict(k_min=10, k_max=5), "bin range"),
    (dict(), dict(k_max=1 << 20), "k_max"),
    (dict(), dict(threshold_2F=float("inf")), "threshold"),
])
def test_invalid_arguments_are_rejected(seg, opts, needle):
    st, h, msg = _plan([_seg(**seg)], **opts)
    assert st == F.E_INVAL
    assert h.value is None
    assert needle in msg


def test_interbinning_option_is_validated_on_the_host():
    st, h, msg = _plan([_seg()], interbinning=2)
    assert st == F.E_INVAL and h.value is None and "interbinning" in msg
    # the transforms of nfft/2 points need nfft >= 2^13 (n = 2048 gives nfft = 2^12)
    st, h, msg = _plan([_seg(n=2048)], interbinning=1)
    assert st == F.E_INVAL and h.value is None and "2^13" in msg


def test_no_segments_is_rejected():
    lib = F.load()
    h = ctypes.c_void_p()
    assert lib.fstat_plan(None, 0, None, ctypes.byref(h)) == F.E_INVAL
    assert lib.fstat_plan((F.fstat_segment * 1)(_seg()), 1, None, None) == F.E_INVAL


def test_admission_rejects_segment_larger_than_budget():
    # a 2^19-point segment needs ~27 MB of workspace even with one sky and one template
    st, h, msg = _plan([_seg(n=20000), _seg(n=172328)], workspace_budget_bytes=8 << 20)
    assert st == F.E_ADMISSION
    assert h.value is None
    assert "budget" in msg


def test_null_handles_are_rejected_not_crashing():
    lib = F.load()
    n = ctypes.c_int64()
    assert lib.fstat_candidates(None, None, None, 0, ctypes.byref(n)) == F.E_INVAL
    assert lib.fstat_search_batch(None, 0, FAKE_PTR, FAKE_PTR, 1, FAKE_PTR, 1, None) == F.E_INVAL
    assert lib.fstat_twoF_spectrum(None, 0, FAKE_PTR, FAKE_PTR, 1, FAKE_PTR, 1, FAKE_PTR, None) == F.E_INVAL
    assert lib.fstat_twoF_spectrum_static(None, 0, FAKE_PTR, FAKE_PTR, 1, FAKE_PTR, 1, FAKE_PTR, None) == F.E_INVAL
    assert lib.fstat_profile_enable(None, 1) == F.E_INVAL
    assert lib.fstat_destroy(None) == F.OK
    sz = ctypes.c_size_t()
    assert lib.fstat_plan_workspace_size(None, ctypes.byref(sz)) == F.E_INVAL


def test_valid_plan_without_gpu_reports_device_error():
    # on a host without a GPU the only failure left after validation is the device
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h, msg = _plan([_seg()])
    assert st == F.E_DEVICE
    assert h.value is None


def test_vetting_entry_points_validate_arguments():
    lib = F.load()
    assert lib.fstat_vet_param_count() == 1080001
    h = ctypes.c_void_p()
    assert lib.fstat_vet_create(0, ctypes.byref(h)) == F.E_INVAL
    assert lib.fstat_vet_create(1 << 20, ctypes.byref(h)) == F.E_INVAL
    assert lib.fstat_vet_create(64, None) == F.E_INVAL
    assert lib.fstat_vet_forward(None, FAKE_PTR, 1, FAKE_PTR, None) == F.E_INVAL
    assert lib.fstat_vet_adam_step(None, 1e-3, 0.9, 0.999, 1e-8, None) == F.E_INVAL
    assert lib.fstat_plan_attach_vetter(None, None, 1) == F.E_INVAL
    assert lib.fstat_plan_vet_candidates(None, None) == F.E_INVAL
    assert lib.fstat_vet_destroy(None) == F.OK


# ---- lattice grid: host-side range and argument checks ------------------------------------
def _lat(seed=3, sky_points=50):
    import synth
    M = synth.lattice_matrix(8192, 2.0, 100.25, sky_points, -2e-10, seed)
    return M, F.lattice(M, synth.OBLIQUITY, 100.25)


@pytest.mark.parametrize("seed,sky_points", [(3, 50), (4, 400), (5, 7)])
def test_lattice_sky_range_matches_the_oracle(seed, sky_points):
    from oracle import fstat_oracle as fo
    M, lat = _lat(seed, sky_points)
    assert F.lattice_sky_range(lat) == fo.lattice_sky_range(M, 100.25)


def test_lattice_range_rejects_parallel_sky_rows_and_bad_values():
    M, lat = _lat()
    M2 = M.copy()
    M2[3, 2:] = 2.0 * M2[2, 2:]
    with pytest.raises(F.FstatError) as ei:
        F.lattice_sky_range(F.lattice(M2, 0.4, 100.25))
    assert ei.value.status == F.E_INVAL and "parallel" in str(ei.value)
    with pytest.raises(F.FstatError) as ei:
        F.lattice_sky_range(F.lattice(M, 0.4, 0.0))
    assert ei.value.status == F.E_INVAL and "f_ref" in str(ei.value)
    M3 = M.copy()
    M3[2, 0] = float("nan")
    with pytest.raises(F.FstatError):
        F.lattice_sky_range(F.lattice(M3, 0.4, 100.25))


@pytest.mark.parametrize("hemi,box,cap,ptrs,needle", [
    (0, (-2, 2, -2, 2), 10, True, "hemisphere"),
    (1, (2, 1, -2, 2), 10, True, "empty box"),
    (1, (-5000, 5000, -5000, 5000), 10, True, "2^26"),
    (1, (-2, 2, -2, 2), -1, True, "capacity"),
    (-1, (-2, 2, -2, 2), 10, False, "device pointers"),
])
def test_lattice_sky_rejects_bad_arguments(hemi, box, cap, ptrs, needle):
    lib = F.load()
    _, lat = _lat()
    b = (ctypes.c_int32 * 4)(*box)
    p = FAKE_PTR if ptrs else None
    st = lib.fstat_lattice_sky(ctypes.byref(lat), hemi, b, cap, p, p, p, p, None, FAKE_PTR, None)
    assert st == F.E_INVAL
    assert needle in lib.fstat_last_error(None).decode()

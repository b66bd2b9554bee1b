"""GPU edge cases against the oracle: empty template lists, an all-zero data segment, sky
positions at the poles and on alpha = 0 / 2 pi, thresholds that nothing or everything
crosses, a single template in a launch sized for 512, and a one-bin range."""
import dataclasses
import math

import numpy as np
import pytest
import torch as _torch  # noqa: F401  (first import on a fresh box is slow)

import synth
from oracle import fstat_oracle as ora
from tests.gpu_util import dev, gpu_spectrum, make_plan, note, oracle_spectrum, rel_err_floor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def tiny():
    return synth.workload("tiny")


def test_empty_template_lists_are_rejected(torch, tiny):
    from paper_1410_3677_amd import fstat as F
    plan = make_plan(tiny.segments)
    empty = torch.empty(0, dtype=torch.float64, device="cuda")
    al, de, fd = dev(tiny.alpha[:1]), dev(tiny.delta[:1]), dev(tiny.fdot[:1])
    for args in ((empty, empty, fd), (al, de, empty)):
        with pytest.raises(F.FstatError) as ei:
            plan.search_batch(0, *args)
        assert ei.value.status == F.E_INVAL
    r, k, n = plan.candidates()
    assert n == 0


@pytest.mark.parametrize("precision,ib", [(0, 0), (1, 0), (1, 1)])
def test_all_zero_data_gives_zero_2f_and_no_candidates(torch, tiny, precision, ib):
    seg = tiny.segments[0]
    zero = dataclasses.replace(seg, x=np.zeros_like(seg.x))
    nfft = synth.nfft_for(seg.n)
    plan = make_plan([zero], precision=precision, interbinning=ib, threshold_2F=1e-30)
    got = gpu_spectrum(plan, 0, tiny.alpha[:2], tiny.delta[:2], tiny.fdot[:2], nfft // 2, precision == 0)
    assert np.all(got == 0.0)
    plan.search_batch(0, dev(tiny.alpha[:2]), dev(tiny.delta[:2]), dev(tiny.fdot[:2]))
    r, k, n = plan.candidates()
    assert n == 0


@pytest.mark.parametrize("precision", [0, 1])
def test_poles_and_alpha_wrap(torch, tiny, precision):
    seg = tiny.segments[0]
    nfft = synth.nfft_for(seg.n)
    al = np.array([0.0, 2 * math.pi, 1.3, 4.0, 2 * math.pi - 1e-12])
    de = np.array([0.2, 0.2, math.pi / 2, -math.pi / 2, math.pi / 2 - 1e-9])
    fd = np.array([0.0, -1e-9])
    note(f"poles and alpha wrap, precision={precision}")
    plan = make_plan([seg], precision=precision)
    got = gpu_spectrum(plan, 0, al, de, fd, nfft // 2, precision == 0)
    ref = oracle_spectrum(seg, al, de, fd, nfft)
    err = rel_err_floor(got, ref)
    note(f"max rel err {err:.3e}")
    tol = 1e-10 if precision == 0 else 1e-4
    assert err < tol
    # alpha = 0 and alpha = 2 pi are the same direction
    assert rel_err_floor(got[0], got[1]) < tol


def test_thresholds_nothing_and_everything_crosses(torch, tiny):
    seg = tiny.segments[0]
    nfft = synth.nfft_for(seg.n)
    al, de, fd = tiny.alpha[:2], tiny.delta[:2], tiny.fdot[:2]
    ref = oracle_spectrum(seg, al, de, fd, nfft)
    hi = make_plan([seg], precision=0, threshold_2F=float(ref.max()) * 2)
    hi.search_batch(0, dev(al), dev(de), dev(fd))
    assert hi.candidates()[2] == 0
    lo = make_plan([seg], precision=0, threshold_2F=0.0)
    lo.search_batch(0, dev(al), dev(de), dev(fd))
    r, k, n = lo.candidates()
    assert n == int(np.sum(ref > 0.0)) == len(al) * len(fd) * (nfft // 2) - int(np.sum(ref == 0.0))
    assert rel_err_floor(r["twoF"], ref[k["sky"], k["fdot_idx"], k["bin"]]) < 1e-10


def test_single_template_in_a_large_launch(torch):
    w = synth.workload("full")
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    plan = make_plan([seg], templates_per_launch=512, skies_per_batch=16)
    got = gpu_spectrum(plan, 0, w.alpha[3:4], w.delta[3:4], w.fdot[5:6], nfft // 2, False)
    ref = oracle_spectrum(seg, w.alpha[3:4], w.delta[3:4], w.fdot[5:6], nfft)
    assert rel_err_floor(got, ref) < 1e-4


@pytest.mark.parametrize("ib", [0, 1])
def test_one_bin_range(torch, tiny, ib):
    seg = tiny.segments[0]
    nfft = synth.nfft_for(seg.n)
    k0 = 1001
    plan = make_plan([seg], precision=1, interbinning=ib, k_min=k0, k_max=k0 + 1)
    got = gpu_spectrum(plan, 0, tiny.alpha[:3], tiny.delta[:3], tiny.fdot[:2], 1, False)
    if ib:
        ref = np.array([[ora.template_two_f_interbin(seg, ora.sky_stage(seg, float(a), float(d), nfft), float(f),
                                                     nfft, k0, k0 + 1) for f in tiny.fdot[:2]]
                        for a, d in zip(tiny.alpha[:3], tiny.delta[:3])])
    else:
        ref = oracle_spectrum(seg, tiny.alpha[:3], tiny.delta[:3], tiny.fdot[:2], nfft, k0, k0 + 1)
    assert got.shape == ref.shape == (3, 2, 1)
    assert rel_err_floor(got, ref) < 1e-4

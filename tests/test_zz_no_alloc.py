"""The entry point that allocates nothing (fstat_twoF_spectrum_static) against the
spectrum entry point it varies (fstat_twoF_spectrum), through the C ABI.

Two calls in a row on one plan, the second with fewer sky positions and spindowns
(the scratch keeps the first call's contents), each compared with the ordinary
entry point on the same inputs: the same kernels run with smaller batch sizes, so the
spectra agree to the last bit; and a template against the FP64 oracle (1e-4 relative,
noise mean 4 as floor).  A plan whose largest segment does not fit the scratch is
rejected before any device work.
"""
import numpy as np
import pytest
import torch as _torch  # noqa: F401  (first import on a fresh box is slow)

import synth
from oracle import fstat_oracle as ora
from tests.gpu_util import dev, make_plan, note, rel_err_floor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _both(torch, plan, al, de, fd, nbins):
    a = torch.full((len(al) * len(fd) * nbins,), float("nan"), dtype=torch.float32, device="cuda")
    b = torch.full_like(a, float("nan"))
    plan.twoF_spectrum(0, dev(al), dev(de), dev(fd), a)
    plan.twoF_spectrum_static(0, dev(al), dev(de), dev(fd), b)
    torch.cuda.synchronize()
    return (a.cpu().numpy().reshape(len(al), len(fd), nbins), b.cpu().numpy().reshape(len(al), len(fd), nbins))


def test_static_scratch_spectrum_equals_workspace_spectrum(torch):
    w = synth.workload("full", nsky=3, nfdot=5)
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    nb = nfft // 2
    plan = make_plan([seg], templates_per_launch=512, skies_per_batch=16)
    note(f"static scratch: n={seg.n} nfft={nfft}, plan {plan.info(0)}")
    ref_a, got_a = _both(torch, plan, w.alpha, w.delta, w.fdot, nb)
    assert np.isfinite(got_a).all()
    np.testing.assert_array_equal(got_a, ref_a)
    # second call, smaller: 1 sky x 2 spindowns (other values than the first call's)
    ref_b, got_b = _both(torch, plan, w.alpha[2:], w.delta[2:], w.fdot[3:], nb)
    assert np.isfinite(got_b).all()
    np.testing.assert_array_equal(got_b, ref_b)
    sky = ora.sky_stage(seg, float(w.alpha[2]), float(w.delta[2]), nfft)
    ora_b = ora.template_two_f(seg, sky, float(w.fdot[4]), nfft)
    err = rel_err_floor(got_b[0, 1].astype(np.float64), ora_b)
    note(f"two calls equal to the workspace entry point; vs oracle {err:.2e}")
    assert err < 1e-4
    # the ordinary entry point still works after the static call (its workspace and layout restored)
    ref_c, _ = _both(torch, plan, w.alpha[:1], w.delta[:1], w.fdot[:1], nb)
    np.testing.assert_array_equal(ref_c[0, 0], ref_a[0, 0])
    plan.destroy()


def test_static_scratch_rejects_a_segment_that_does_not_fit(torch):
    from paper_1410_3677_amd import fstat as F
    n = 1 << 19
    seg = synth.make_segment(n, 2.0, 100.0, 1.0, 77, [])
    plan = make_plan([seg], precision=0)
    out = torch.empty(1 << 19, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FstatError) as ei:
        plan.twoF_spectrum_static(0, dev([0.1]), dev([0.2]), dev([0.0]), out)
    assert ei.value.status == F.E_INVAL and "static scratch" in str(ei.value)
    plan.destroy()

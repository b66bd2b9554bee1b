"""GPU parity of the interbinned search (template transforms of nfft/2 points, odd bins
from their neighbours) against the oracle's interbinned transform, element by element.

Mixed precision: |2F_gpu - 2F_ora| / max(2F_ora, 4) <= 1e-4; candidate key sets equal
outside a guard band of 1e-4 * threshold.  The second pass walks chunks of consecutive
rows; the cases cover one row per wavefront unit (nfft/2 = 2^17: P = 512), two (2^15,
2^16: P = 256) and eight (2^12: P = 64), templates shorter than a chunk (N = 3000: eight
units), bin ranges that end in the wrap-around bin nfft - 1, and plain against batched
launches.
"""
import numpy as np
import pytest
import torch as _torch  # imported at collection: the first import on a fresh box is slow

import synth
from oracle import fstat_oracle as ora
from tests.gpu_util import assert_keys_equal, compare_candidates, dev, make_plan, note, rel_err_floor

pytestmark = pytest.mark.gpu

TOL = 1e-4
GUARD = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _gpu(plan, al, de, fd, nbins):
    import torch
    out = torch.empty(len(al) * len(fd) * nbins, dtype=torch.float32, device="cuda")
    plan.twoF_spectrum(0, dev(al), dev(de), dev(fd), out)
    torch.cuda.synchronize()
    return out.double().cpu().numpy().reshape(len(al), len(fd), nbins)


def _oracle(seg, al, de, fd, nfft, k_min=0, k_max=-1, full=False):
    res = []
    for i in range(len(al)):
        sky = ora.sky_stage(seg, float(al[i]), float(de[i]), nfft)
        res.append([ora.template_two_f_interbin(seg, sky, float(f), nfft, k_min, k_max, full) for f in fd])
    return np.array(res)


def test_spectrum_tiny_all_templates(torch):
    note("interbinning spectrum, N=4096 (template FFT 4096 = 64 x 64), 8 sky x 4 spindowns")
    w = synth.workload("tiny")
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    plan = make_plan([seg], precision=1, interbinning=1)
    inf = plan.info(0)
    assert inf["nfft"] == nfft and inf["p"] * inf["q"] == nfft // 2
    got = _gpu(plan, w.alpha, w.delta, w.fdot, nfft // 2)
    ref = _oracle(seg, w.alpha, w.delta, w.fdot, nfft)
    err = rel_err_floor(got, ref)
    note(f"max rel err {err:.3e}")
    assert err < TOL


def test_spectrum_full_segment(torch):
    note("interbinning spectrum, N=86164 (template FFT 2^17 = 512 x 256), 2 sky x 3 spindowns")
    w = synth.workload("full")
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    al, de, fd = w.alpha[[0, 101]], w.delta[[0, 101]], w.fdot[[0, 31, 63]]
    plan = make_plan([seg], interbinning=1)
    got = _gpu(plan, al, de, fd, nfft // 2)
    ref = _oracle(seg, al, de, fd, nfft)
    err = rel_err_floor(got, ref)
    note(f"max rel err {err:.3e}")
    assert err < TOL


@pytest.mark.parametrize("n", [3000, 20000, 45000, 110000, 120000])
def test_spectrum_other_lengths(torch, n):
    # nfft/2 over n: the first pass prunes inputs r >= 6 (3000, 45000), >= 5 (20000),
    # >= 7 (110000) or none (120000)
    rng = np.random.default_rng(n + 7)
    injs = synth.draw_injections(rng, 1, 15.0, 15.0)
    seg = synth.make_segment(n, 2.0, 100.0, 1.0, 4100 + n, injs)
    nfft = synth.nfft_for(n)
    note(f"interbinning spectrum n={n} nfft={nfft}")
    plan = make_plan([seg], interbinning=1)
    al, de = np.array([0.3, injs[0].alpha]), np.array([-0.2, injs[0].delta])
    fd = np.array([0.0, injs[0].fdot])
    got = _gpu(plan, al, de, fd, nfft // 2)
    ref = _oracle(seg, al, de, fd, nfft)
    err = rel_err_floor(got, ref)
    note(f"n={n} max rel err {err:.3e}")
    assert err < TOL


@pytest.mark.parametrize("name,k0,k1", [("tiny", 1, 8192), ("tiny", 777, 5001), ("full", 131071, 262144)])
def test_bin_ranges_up_to_the_wrap_bin(torch, name, k0, k1):
    """Ranges that start on an odd bin and end at nfft, whose last bin nfft - 1 lies between
    the transform's last bin and bin 0."""
    w = synth.workload(name)
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    k1 = min(k1, nfft)
    note(f"interbinning bins [{k0}, {k1}) of {name}")
    plan = make_plan([seg], precision=1, interbinning=1, k_min=k0, k_max=k1)
    al, de, fd = w.alpha[:2], w.delta[:2], w.fdot[:2]
    got = _gpu(plan, al, de, fd, k1 - k0)
    ref = _oracle(seg, al, de, fd, nfft, k0, k1)
    err = rel_err_floor(got, ref)
    note(f"max rel err {err:.3e}")
    assert err < TOL


def test_full_form(torch):
    w = synth.workload("tiny")
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    plan = make_plan([seg], precision=1, interbinning=1, form=1)
    al, de, fd = w.alpha[:3], w.delta[:3], w.fdot[:2]
    got = _gpu(plan, al, de, fd, nfft // 2)
    ref = _oracle(seg, al, de, fd, nfft, full=True)
    assert rel_err_floor(got, ref) < TOL


def test_candidates_full_segment_batched(torch):
    """Launches of 64 templates: many chunks per wavefront, across templates."""
    w = synth.workload("full")
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    al, de, fd = w.alpha[[5, 77]], w.delta[[5, 77]], w.fdot[:40]
    note("interbinning candidates, N=86164, 2 sky x 40 spindowns, 64 templates per launch")
    plan = make_plan([seg], interbinning=1, templates_per_launch=64, skies_per_batch=2)
    plan.search_batch(0, dev(al), dev(de), dev(fd))
    recs, keys, n = plan.candidates()
    ref = _oracle(seg, al, de, fd, nfft)
    key3 = np.stack([keys["sky"], keys["fdot_idx"], keys["bin"]], 1)
    ng, no, flips, mism, err = compare_candidates(key3, recs["twoF"], ref, w.threshold, GUARD)
    note(f"gpu {ng} oracle {no} flips {flips} mismatches {len(mism)} err {err:.3e}")
    assert no > 1000 and not mism and err < TOL
    assert len(np.unique(key3, axis=0)) == len(key3)
    np.testing.assert_allclose(recs["f_hz"], seg.f_off + keys["bin"] / (nfft * seg.dt), rtol=0, atol=1e-12)


def test_plain_launches_equal_batched(torch):
    w = synth.workload("full")
    seg = w.segments[0]
    al, de, fd = dev(w.alpha[:3]), dev(w.delta[:3]), dev(w.fdot[:5])
    out = []
    for opts in (dict(templates_per_launch=1, skies_per_batch=1), dict(templates_per_launch=7), dict()):
        plan = make_plan([seg], interbinning=1, **opts)
        plan.search_batch(0, al, de, fd)
        out.append(plan.candidates())
        plan.destroy()
    r0, k0, n0 = out[0]
    assert n0 > 0
    for r, k, n in out[1:]:
        assert n == n0
        assert_keys_equal(k, k0)
        np.testing.assert_array_equal(r, r0)


def test_even_bins_match_the_zero_padded_search(torch):
    """Even bins are the same transform values as the zero-padded search's (up to FP32
    rounding of two different FFT lengths)."""
    w = synth.workload("full")
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    al, de, fd = w.alpha[:2], w.delta[:2], w.fdot[:2]
    a = _gpu(make_plan([seg], interbinning=1), al, de, fd, nfft // 2)
    b = _gpu(make_plan([seg]), al, de, fd, nfft // 2)
    err = rel_err_floor(a[..., 0::2], b[..., 0::2])
    note(f"even bins vs zero-padded: {err:.3e}")
    assert err < TOL


def test_interbinning_needs_a_long_enough_transform(torch):
    from paper_1410_3677_amd import fstat as F
    seg = synth.make_segment(2048, 2.0, 100.0, 1.0, 4242, [])
    with pytest.raises(F.FstatError) as ei:
        make_plan([seg], interbinning=1)
    assert ei.value.status == F.E_INVAL


def test_ragged_segments_in_one_call_equal_separate_plans(torch):
    """All segments in one call (segment = -1): each segment has its own template length
    (nfft/2 from 2^15 to 2^18) in one workspace sized for the longest."""
    w = synth.workload("ragged")
    segs = w.segments[:5]
    note("interbinning, ragged: " + ", ".join(f"n={s.n}" for s in segs))
    al, de, fd = dev(w.alpha[:3]), dev(w.delta[:3]), dev(w.fdot[:6])
    plan = make_plan(segs, interbinning=1)
    plan.search_batch(-1, al, de, fd)
    r_all, k_all, n_all = plan.candidates()
    assert n_all > 0
    for si, seg in enumerate(segs):
        one = make_plan([seg], interbinning=1)
        one.search_batch(0, al, de, fd)
        r1, k1, n1 = one.candidates()
        m = k_all["segment"] == si
        assert int(m.sum()) == n1, (si, int(m.sum()), n1)
        np.testing.assert_array_equal(k_all["sky"][m], k1["sky"])
        np.testing.assert_array_equal(k_all["fdot_idx"][m], k1["fdot_idx"])
        np.testing.assert_array_equal(k_all["bin"][m], k1["bin"])
        np.testing.assert_allclose(r_all["twoF"][m], r1["twoF"], rtol=1e-6, atol=0)
        one.destroy()


# ---- FP64: the tiled second pass stores the transforms, a separate pass forms 2F ------------
TOL64 = 1e-10


def _gpu64(plan, al, de, fd, nbins):
    import torch
    out = torch.empty(len(al) * len(fd) * nbins, dtype=torch.float64, device="cuda")
    plan.twoF_spectrum(0, dev(al), dev(de), dev(fd), out)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(len(al), len(fd), nbins)


@pytest.mark.parametrize("case", ["tiny", "full", "n3000", "n120000", "tiny-range", "full-wrap", "tiny-fullform"])
def test_fp64_interbinned_spectra(torch, case):
    if case.startswith("n"):
        n = int(case[1:])
        seg = synth.make_segment(n, 2.0, 100.0, 1.0, 5100 + n, synth.draw_injections(np.random.default_rng(n), 1,
                                                                                       15.0, 15.0))
        al, de, fd = np.array([0.3, seg.injections[0].alpha]), np.array([-0.2, seg.injections[0].delta]), \
            np.array([0.0, seg.injections[0].fdot])
    else:
        w = synth.workload("full" if case.startswith("full") else "tiny")
        seg = w.segments[0]
        al, de, fd = w.alpha[:2], w.delta[:2], w.fdot[:2]
    nfft = synth.nfft_for(seg.n)
    k0, k1 = 0, nfft // 2
    if case == "tiny-range":
        k0, k1 = 777, 5001
    if case == "full-wrap":
        k0, k1 = 131071, nfft
    full = case.endswith("fullform")
    note(f"FP64 interbinning spectrum, {case}: n={seg.n}, bins [{k0}, {k1})")
    plan = make_plan([seg], precision=0, interbinning=1, k_min=k0, k_max=k1, form=int(full))
    got = _gpu64(plan, al, de, fd, k1 - k0)
    ref = _oracle(seg, al, de, fd, nfft, k0, k1, full=full)
    err = rel_err_floor(got, ref)
    note(f"max rel err {err:.3e}")
    assert err < TOL64


def test_fp64_interbinned_candidates_batched(torch):
    w = synth.workload("full")
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    al, de, fd = w.alpha[[5, 77]], w.delta[[5, 77]], w.fdot[:6]
    note("FP64 interbinning candidates, N=86164, 2 sky x 6 spindowns, 4 templates per launch")
    plan = make_plan([seg], precision=0, interbinning=1, templates_per_launch=4, skies_per_batch=2)
    plan.search_batch(0, dev(al), dev(de), dev(fd))
    recs, keys, n = plan.candidates()
    ref = _oracle(seg, al, de, fd, nfft)
    key3 = np.stack([keys["sky"], keys["fdot_idx"], keys["bin"]], 1)
    ng, no, flips, mism, err = compare_candidates(key3, recs["twoF"], ref, w.threshold, 1e-9)
    note(f"gpu {ng} oracle {no} flips {flips} mismatches {len(mism)} err {err:.3e}")
    assert no > 1000 and not mism and err < TOL64
    assert len(np.unique(key3, axis=0)) == len(key3)
    # mixed and FP64 interbinning agree on every key away from the threshold
    m = make_plan([seg], precision=1, interbinning=1)
    m.search_batch(0, dev(al), dev(de), dev(fd))
    rm, km, nm_ = m.candidates()
    assert abs(nm_ - n) <= flips + int(np.sum(np.abs(ref - w.threshold) <= 1e-4 * w.threshold))


@pytest.mark.parametrize("n,precision", [(524288, 1), (524288, 0), (262145, 1)])
def test_interbinning_at_the_longest_transforms(torch, n, precision):
    """Segments above 2^18 samples have nfft = 2^20, so the interbinned transform has
    P = 1024 rows: the tiled second pass stores the transforms and the interbinning pass
    forms 2F, in both precisions (n = 2^19 is the longest segment the library takes)."""
    rng = np.random.default_rng(n + 3)
    injs = synth.draw_injections(rng, 1, 15.0, 15.0)
    seg = synth.make_segment(n, 2.0, 100.0, 1.0, 6100 + n, injs)
    nfft = synth.nfft_for(n)
    note(f"interbinning at the longest transforms: n={n} nfft={nfft} precision={precision}")
    plan = make_plan([seg], precision=precision, interbinning=1)
    inf = plan.info(0)
    assert inf["nfft"] == 1 << 20 and inf["p"] == 1024 and inf["q"] == 512
    al, de = np.array([0.3, injs[0].alpha]), np.array([-0.2, injs[0].delta])
    fd = np.array([injs[0].fdot])
    got = _gpu64(plan, al, de, fd, nfft // 2) if precision == 0 else _gpu(plan, al, de, fd, nfft // 2)
    ref = _oracle(seg, al, de, fd, nfft)
    err = rel_err_floor(got, ref)
    note(f"max rel err {err:.3e}")
    assert err < (TOL64 if precision == 0 else TOL)
    # candidates of the same templates
    plan2 = make_plan([seg], precision=precision, interbinning=1)
    plan2.search_batch(0, dev(al), dev(de), dev(fd))
    recs, keys, cnt = plan2.candidates()
    key3 = np.stack([keys["sky"], keys["fdot_idx"], keys["bin"]], 1)
    ng, no, flips, mism, cerr = compare_candidates(key3, recs["twoF"], ref, 20.0, 1e-9 if precision == 0 else GUARD)
    note(f"candidates gpu {ng} oracle {no} flips {flips} mismatches {len(mism)}")
    assert no > 100 and not mism

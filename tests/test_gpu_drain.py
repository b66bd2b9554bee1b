"""The candidate drain through the C ABI: records come out in key order (search, segment,
sky, spindown index, bin), ordered on the device (count -> offsets -> write, then each
template's range by bin: a counting rank up to 4096 crossings, an LDS bitmap of the bins
beyond); the drained set equals the oracle's crossings."""
import numpy as np
import pytest
import torch as _torch  # noqa: F401  (first import on a fresh box is slow)

import synth
from tests.gpu_util import compare_candidates, dev, make_plan, note, oracle_spectrum

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _key(keys):
    return np.stack([keys[f].astype(np.int64) for f in ("search", "segment", "sky", "fdot_idx", "bin")], 1)


def _strictly_increasing(k):
    if len(k) < 2:
        return True
    d = np.diff(k, axis=0)
    first = np.argmax(d != 0, axis=1)                  # the first field that differs
    return bool(np.all(d[np.arange(len(d)), first] > 0))


def test_drain_orders_several_searches_and_segments(torch):
    w = synth.workload("ragged", nsky=5, nfdot=6)
    segs = w.segments[:6]
    plan = make_plan(segs, candidate_capacity=1 << 22)
    a, d, f = dev(w.alpha), dev(w.delta), dev(w.fdot)
    plan.search_batch(-1, a, d, f)                     # search 0: every segment
    plan.search_batch(2, a[:3], d[:3], f[:4])          # search 1: segment 2, a sub-grid
    recs, keys, n = plan.candidates()
    note(f"two searches over {len(segs)} segments: {n} candidates")
    k = _key(keys)
    assert n > 1000 and _strictly_increasing(k)
    assert set(np.unique(keys["search"])) == {0, 1}
    assert set(np.unique(keys["segment"][keys["search"] == 1])) == {2}
    # the second search's crossings are the first search's on the same templates
    m0 = (keys["search"] == 0) & (keys["segment"] == 2) & (keys["sky"] < 3) & (keys["fdot_idx"] < 4)
    m1 = keys["search"] == 1
    np.testing.assert_array_equal(k[m0][:, 2:], k[m1][:, 2:])
    np.testing.assert_array_equal(recs["twoF"][m0], recs["twoF"][m1])
    # records follow their keys
    for si in range(len(segs)):
        nfft = synth.nfft_for(segs[si].n)
        m = keys["segment"] == si
        np.testing.assert_allclose(recs["f_hz"][m], segs[si].f_off + keys["bin"][m] / (nfft * segs[si].dt),
                                   rtol=0, atol=1e-9)
    np.testing.assert_array_equal(recs["alpha"], w.alpha[keys["sky"]])
    np.testing.assert_array_equal(recs["fdot"], w.fdot[keys["fdot_idx"]])


def test_drain_of_templates_with_many_crossings(torch):
    # 2F > 1 on a full segment: about 0.91 of the 131072 bins of each template cross,
    # more than the counting rank orders: the bitmap ordering takes these templates
    w = synth.workload("full", nsky=2, nfdot=2)
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    thr = 1.0
    plan = make_plan([seg], threshold_2F=thr, candidate_capacity=1 << 20)
    plan.search_batch(0, dev(w.alpha), dev(w.delta), dev(w.fdot))
    recs, keys, n = plan.candidates()
    note(f"2F > {thr}: {n} candidates over 4 templates")
    assert n > 4 * 100000 and _strictly_increasing(_key(keys))
    ref = oracle_spectrum(seg, w.alpha, w.delta, w.fdot, nfft)
    ng, no, flips, mism, err = compare_candidates(np.stack([keys["sky"], keys["fdot_idx"], keys["bin"]], 1),
                                                  recs["twoF"], ref, thr, 1e-4)
    note(f"gpu {ng} oracle {no} flips {flips} mismatches {len(mism)} err {err:.2e}")
    assert not mism and err < 1e-4


@pytest.mark.parametrize("nbins", [4096, 4097])
def test_drain_at_the_ordering_switch(torch, nbins):
    # a bin range of exactly 4096 or 4097 bins and a threshold every 2F exceeds: each
    # template holds that many crossings, the longest range the counting rank orders and
    # the shortest the bitmap ordering takes
    w = synth.workload("full", nsky=2, nfdot=3)
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    k0 = 1000
    plan = make_plan([seg], threshold_2F=-1.0, k_min=k0, k_max=k0 + nbins, candidate_capacity=1 << 16)
    plan.search_batch(0, dev(w.alpha), dev(w.delta), dev(w.fdot))
    recs, keys, n = plan.candidates()
    note(f"{nbins} bins per template: {n} candidates")
    assert n == 6 * nbins and _strictly_increasing(_key(keys))
    for i in range(2):
        for s_ in range(3):
            m = (keys["sky"] == i) & (keys["fdot_idx"] == s_)
            np.testing.assert_array_equal(keys["bin"][m], np.arange(k0, k0 + nbins))
    ref = oracle_spectrum(seg, w.alpha, w.delta, w.fdot, nfft, k0, k0 + nbins)
    got = recs["twoF"].reshape(2, 3, nbins)
    err = np.max(np.abs(got - ref) / np.maximum(ref, 4.0))
    note(f"max relative 2F error {err:.2e}")
    assert err < 1e-4


def test_partial_drain_returns_the_first_keys(torch):
    w = synth.workload("full", nsky=3, nfdot=4)
    seg = w.segments[0]
    p1 = make_plan([seg], candidate_capacity=1 << 20)
    p1.search_batch(0, dev(w.alpha), dev(w.delta), dev(w.fdot))
    r_all, k_all, n = p1.candidates()
    p2 = make_plan([seg], candidate_capacity=1 << 20)
    p2.search_batch(0, dev(w.alpha), dev(w.delta), dev(w.fdot))
    r_few, k_few, n2 = p2.candidates(capacity=n // 3, allow_overflow=True)
    assert n2 == n and len(k_few) == n // 3
    np.testing.assert_array_equal(_key(k_few), _key(k_all)[: n // 3])
    np.testing.assert_array_equal(r_few["twoF"], r_all["twoF"][: n // 3])

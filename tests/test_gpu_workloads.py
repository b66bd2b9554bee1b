"""GPU parity on whole sky batches of the workloads, every template bin by bin.

* batched: one sky batch of the 4096 x 256 workload at its own threshold 2F > 20, in
  the autotuned launch configuration the benchmark times: the sky position nearest to
  each of the five injections and 11 seeded others, x all 256 spindowns (4096
  templates); every crossing and the whole 2F spectrum of every template against the
  FP64 oracle.
* full F form (with C = <ab>) on the mixed-precision zero-padded path (the streaming
  second pass): the tiny segment, and a short ragged segment on sky positions where
  C / sqrt(AB) exceeds 0.2, where the form matters.
* ragged: the 32 uneven segments in one call with 16 sky x 128 spindowns each; the
  shortest, the median and the longest segment checked template by template.
Tolerances as in the other parity tests: 1e-4 relative with the noise mean 4 as floor;
key sets equal outside a guard band of 1e-4 x threshold.
"""
import math

import numpy as np
import pytest
import torch as _torch  # noqa: F401  (first import on a fresh box is slow)

import synth
from oracle import fstat_oracle as ora
from tests.gpu_util import compare_candidates, dev, gpu_spectrum, make_plan, note, per_sky_oracle, rel_err_floor

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-4
GUARD_MIXED = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _nearest_sky(alpha, delta, a0, d0):
    """Index of the sky position with the smallest angle to (a0, d0)."""
    c = np.sin(delta) * math.sin(d0) + np.cos(delta) * math.cos(d0) * np.cos(alpha - a0)
    return int(np.argmax(c))


def _check_sky_batch(seg, alpha, delta, fdot, nfft, keys, recs, spec, thr, full=False):
    """Every template of the sky list: its crossings (keys and 2F) and its whole GPU
    spectrum against the oracle.  Returns (worst spectrum error, worst candidate error,
    crossings, flips)."""
    def check(i, ref):
        m = keys["sky"] == i
        key3 = np.stack([np.zeros(int(m.sum()), np.int64), keys["fdot_idx"][m], keys["bin"][m]], 1)
        ng, no, flips, mism, err = compare_candidates(key3, recs["twoF"][m], ref[None], thr, GUARD_MIXED)
        return rel_err_floor(spec[i], ref), err, ng, no, flips, mism
    res = per_sky_oracle(seg, alpha, delta, fdot, nfft, check, full=full)
    for i, (es, ec, ng, no, flips, mism) in enumerate(res):
        assert not mism, (i, mism[:5])
        assert es < TOL_MIXED and ec < TOL_MIXED, (i, es, ec)
        assert abs(ng - no) <= flips
    return (max(r[0] for r in res), max(r[1] for r in res), sum(r[2] for r in res), sum(r[4] for r in res))


def test_batched_sky_batch_every_template_at_threshold_20(torch):
    from paper_1410_3677_amd import fstat as F
    w = synth.workload("batched")
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    picks = []
    for inj in seg.injections:
        j = _nearest_sky(w.alpha, w.delta, inj.alpha, inj.delta)
        if j not in picks:
            picks.append(j)
    rng = np.random.default_rng(73)
    while len(picks) < 16:
        j = int(rng.integers(len(w.alpha)))
        if j not in picks:
            picks.append(j)
    al, de, fd = w.alpha[picks], w.delta[picks], w.fdot
    note(f"batched workload, one sky batch: skies {picks} x {len(fd)} spindowns at 2F > {w.threshold}")
    plan = F.Plan([F.segment_to_device(seg)], workspace_from_torch=False, threshold_2F=w.threshold,
                  candidate_capacity=1 << 22)
    info = plan.autotune(0, budget_ms=3000.0)
    note(f"autotuned launch configuration {info}")
    plan.search_batch(0, dev(al), dev(de), dev(fd))
    recs, keys, n = plan.candidates()
    note(f"{n} candidates")
    assert n == len(recs) and n > 4096 * 50
    spec = gpu_spectrum(plan, 0, al, de, fd, nfft // 2, False)
    plan.destroy()
    es, ec, nc, flips = _check_sky_batch(seg, al, de, fd, nfft, keys, recs, spec, w.threshold)
    note(f"4096 templates: spectrum max rel err {es:.2e}, candidates {nc} max rel err {ec:.2e}, flips {flips}")
    # the injections' templates are found: each injection's sky holds a crossing near its frequency
    for inj in seg.injections:
        i = picks.index(_nearest_sky(w.alpha, w.delta, inj.alpha, inj.delta))
        near = (keys["sky"] == i) & (np.abs(recs["f_hz"] - (seg.f_off + inj.f)) < 2e-3)
        assert near.any(), inj


def _sky_with_large_c(seg, alpha, delta, count, floor=0.2):
    """Indices of `count` sky positions where C / sqrt(AB) of this segment exceeds `floor`."""
    out = []
    for i in range(len(alpha)):
        a, b = ora.amplitude_modulation(seg.n, seg.dt, float(alpha[i]), float(delta[i]), seg.lat, seg.gamma,
                                        seg.phi_r)
        if abs(np.mean(a * b)) / math.sqrt(np.mean(a * a) * np.mean(b * b)) > floor:
            out.append(i)
            if len(out) == count:
                break
    return out


@pytest.mark.parametrize("which", ["tiny", "ragged"])
def test_full_form_mixed_zero_padded(torch, which):
    if which == "tiny":
        w = synth.workload("tiny")
        seg = w.segments[0]
        al, de, fd = w.alpha, w.delta, w.fdot
    else:
        w = synth.workload("ragged", nsky=256, nfdot=8)
        seg = min(w.segments, key=lambda s: s.n)
        idx = _sky_with_large_c(seg, w.alpha, w.delta, 4)
        assert len(idx) == 4
        al, de, fd = w.alpha[idx], w.delta[idx], w.fdot
    nfft = synth.nfft_for(seg.n)
    abc = [ora.sky_stage(seg, float(a), float(d), nfft) for a, d in zip(al[:2], de[:2])]
    cmax = max(abs(s["C"]) / math.sqrt(s["A"] * s["B"]) for s in abc)
    plan = make_plan([seg], precision=1, form=1, threshold_2F=w.threshold)
    info = plan.info(0)
    note(f"full form, mixed, {which}: n={seg.n} nfft={nfft} {info}, C/sqrt(AB) up to {cmax:.2f}")
    assert info["pass_b_variant"] == 1 and info["p"] <= 512   # the streaming second pass
    plan.search_batch(0, dev(al), dev(de), dev(fd))
    recs, keys, n = plan.candidates()
    spec = gpu_spectrum(plan, 0, al, de, fd, nfft // 2, False)
    es, ec, nc, flips = _check_sky_batch(seg, al, de, fd, nfft, keys, recs, spec, w.threshold, full=True)
    note(f"{len(al)} x {len(fd)} templates: spectrum err {es:.2e}, {nc} candidates err {ec:.2e}, flips {flips}")
    assert nc > 0
    # the simplified form differs where C matters: the same plan without it is not the oracle's full form
    if cmax > 0.2:
        simp = make_plan([seg], precision=1, form=0)
        s2 = gpu_spectrum(simp, 0, al[:1], de[:1], fd[:1], nfft // 2, False)
        ref = ora.template_two_f(seg, abc[0], float(fd[0]), nfft, full=True)
        assert rel_err_floor(s2[0, 0], ref) > 1e-2


def test_ragged_32_segments_16_sky_128_spindowns(torch):
    w = synth.workload("ragged", nsky=16, nfdot=128)
    segs = w.segments
    note(f"ragged: {len(segs)} segments x {len(w.alpha)} sky x {len(w.fdot)} spindowns in one call")
    plan = make_plan(segs, candidate_capacity=1 << 25)
    plan.search_batch(-1, dev(w.alpha), dev(w.delta), dev(w.fdot))
    recs, keys, n = plan.candidates()
    note(f"{n} candidates over {len(segs)} segments, batches {plan.info(0)}")
    assert set(np.unique(keys["segment"])) == set(range(len(segs)))
    order = np.argsort([s.n for s in segs])
    for si in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        seg = segs[si]
        nfft = synth.nfft_for(seg.n)
        m = keys["segment"] == si
        k, r = keys[m], recs[m]
        np.testing.assert_allclose(r["f_hz"], seg.f_off + k["bin"] / (nfft * seg.dt), rtol=0, atol=1e-9)

        def check(i, ref):
            mm = k["sky"] == i
            key3 = np.stack([np.zeros(int(mm.sum()), np.int64), k["fdot_idx"][mm], k["bin"][mm]], 1)
            return compare_candidates(key3, r["twoF"][mm], ref[None], w.threshold, GUARD_MIXED)
        res = per_sky_oracle(seg, w.alpha, w.delta, w.fdot, nfft, check)
        for ng, no, flips, mism, err in res:
            assert not mism and err < TOL_MIXED
        note(f"segment {si} n={seg.n} nfft={nfft}: gpu {sum(x[0] for x in res)} oracle {sum(x[1] for x in res)} "
             f"flips {sum(x[2] for x in res)} err {max(x[4] for x in res):.2e}")
    plan.destroy()

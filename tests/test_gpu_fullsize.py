"""GPU parity at the workloads' full sizes, in the launch configurations the benchmark times.

* full:    256 sky x 64 spindown at N = 86164, one template per launch (the plain path),
           threshold 2F > 20: every crossing drained and every template's crossings
           (keys and 2F) checked against the FP64 oracle's spectrum of that template.
* batched: 4096 sky x 256 spindown (1 048 576 templates), autotuned batch sizes and
           kernel variants, HIP graph, the workload's threshold 2F > 20 (about 1.4e8
           crossings, all drained in key order): the loudest template of every injection
           and a seeded 1% sample of the templates (41 whole sky positions) are checked
           against the oracle template by template.
* batched with interbinning: the loudest template of every injection against the
           oracle's interbinned transform, at 2F > 40.
Tolerances are those of the other parity tests (1e-4 relative, floor 4; key sets equal
outside a 1e-4 x threshold guard band).
"""
import numpy as np
import pytest
import torch as _torch  # noqa: F401  (first import on a fresh box is slow)

import synth
from oracle import fstat_oracle as ora
from tests.gpu_util import compare_candidates, dev, make_plan, note, oracle_spectrum

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _interbinned_spectrum(seg, alpha, delta, fdot, nfft):
    sky = ora.sky_stage(seg, float(alpha[0]), float(delta[0]), nfft)
    return np.array([[ora.template_two_f_interbin(seg, sky, float(fdot[0]), nfft)]])


def _check_templates(seg, w, recs, keys, picks, thr, interbinning=False):
    nfft = synth.nfft_for(seg.n)
    spectrum = _interbinned_spectrum if interbinning else oracle_spectrum
    worst = 0.0
    for (i, s) in picks:
        m = (keys["sky"] == i) & (keys["fdot_idx"] == s)
        key3 = np.stack([np.zeros(int(m.sum()), dtype=np.int64), np.zeros(int(m.sum()), dtype=np.int64),
                         keys["bin"][m]], 1)
        ref = spectrum(seg, w.alpha[i:i + 1], w.delta[i:i + 1], w.fdot[s:s + 1], nfft)
        ng, no, flips, mism, err = compare_candidates(key3, recs["twoF"][m], ref, thr, 1e-4)
        note(f"template (sky {i}, fdot {s}): gpu {ng} oracle {no} flips {flips} mismatches {len(mism)} err {err:.2e}")
        assert not mism and err < 1e-4
        worst = max(worst, err)
    return worst


def test_full_workload_plain_path_every_template(torch):
    from tests.gpu_util import per_sky_oracle
    w = synth.workload("full")
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    note(f"full workload, plain path: {len(w.alpha)} x {len(w.fdot)} templates, one per launch")
    plan = make_plan([seg], templates_per_launch=1, skies_per_batch=1, use_graph=0, candidate_capacity=1 << 22)
    plan.search_batch(0, dev(w.alpha), dev(w.delta), dev(w.fdot))
    recs, keys, n = plan.candidates()
    assert n == len(recs) and n > 500000
    assert np.all(recs["twoF"] > w.threshold)
    key3 = np.stack([keys["sky"], keys["fdot_idx"], keys["bin"]], 1)
    assert len(np.unique(key3, axis=0)) == n

    # every template's crossings against the oracle's spectrum, sky by sky
    starts = np.searchsorted(keys["sky"], np.arange(len(w.alpha) + 1))

    def check(i, ref):
        a, b = starts[i], starts[i + 1]
        k3 = np.stack([np.zeros(b - a, np.int64), keys["fdot_idx"][a:b], keys["bin"][a:b]], 1)
        return compare_candidates(k3, recs["twoF"][a:b], ref[None], w.threshold, 1e-4)
    res = per_sky_oracle(seg, w.alpha, w.delta, w.fdot, nfft, check)
    flips = sum(r[2] for r in res)
    err = max(r[4] for r in res)
    note(f"all {len(w.alpha) * len(w.fdot)} templates: gpu {sum(r[0] for r in res)} oracle "
         f"{sum(r[1] for r in res)} flips {flips} max rel err {err:.2e}")
    for ng, no, fl, mism, e in res:
        assert not mism and e < 1e-4


def _strictly_increasing(*cols):
    """(sky, fdot_idx, bin) rows strictly increasing in that order (so also unique)."""
    d = [np.diff(c.astype(np.int64)) for c in cols]
    lead = d[0] > 0
    same = d[0] == 0
    for x in d[1:]:
        lead |= same & (x > 0)
        same &= x == 0
    return bool(np.all(lead))


@pytest.mark.parametrize("ib", [0, 1])
def test_batched_workload_full_size_sampled_parity(torch, ib):
    from paper_1410_3677_amd import fstat as F
    w = synth.workload("batched")
    seg = w.segments[0]
    thr = 40.0 if ib else w.threshold
    note(f"batched workload at full size: {len(w.alpha)} x {len(w.fdot)} templates, 2F > {thr}, interbinning={ib}")
    plan = F.Plan([F.segment_to_device(seg)], workspace_from_torch=False, threshold_2F=thr,
                  candidate_capacity=(1 << 25) if ib else (1 << 28), interbinning=ib)
    plan.autotune(0, budget_ms=3000.0)
    info = plan.info(0)
    note(f"launch configuration {info}")
    plan.search_batch(0, dev(w.alpha), dev(w.delta), dev(w.fdot))
    recs, keys, n = plan.candidates()
    note(f"{n} candidates")
    assert n == len(recs) and n > 10000
    assert np.all(recs["twoF"] > thr)
    assert _strictly_increasing(keys["sky"], keys["fdot_idx"], keys["bin"])
    picks = []
    # the loudest template near each injection's frequency, then seeded random templates
    f_hz = recs["f_hz"]
    for inj in seg.injections:
        near = np.abs(f_hz - (seg.f_off + inj.f)) < 1e-3
        if near.any():
            j = int(np.flatnonzero(near)[np.argmax(recs["twoF"][near])])
            picks.append((int(keys["sky"][j]), int(keys["fdot_idx"][j])))
    assert len(picks) >= 3
    _check_templates(seg, w, recs, keys, picks, thr, interbinning=bool(ib))
    plan.destroy()
    if ib:
        return
    # a seeded 1% sample of the templates: 41 whole sky positions x 256 spindowns, every
    # template's crossings against the oracle
    from tests.gpu_util import per_sky_oracle
    rng = np.random.default_rng(72)
    skies = np.sort(rng.choice(len(w.alpha), size=41, replace=False))
    starts = np.searchsorted(keys["sky"], np.arange(len(w.alpha) + 1))
    nfft = synth.nfft_for(seg.n)

    def check(j, ref):
        i = int(skies[j])
        a, b = starts[i], starts[i + 1]
        k3 = np.stack([np.zeros(b - a, np.int64), keys["fdot_idx"][a:b], keys["bin"][a:b]], 1)
        return compare_candidates(k3, recs["twoF"][a:b], ref[None], thr, 1e-4)
    res = per_sky_oracle(seg, w.alpha[skies], w.delta[skies], w.fdot, nfft, check)
    note(f"1% sample ({len(skies)} skies x {len(w.fdot)} spindowns): gpu {sum(r[0] for r in res)} oracle "
         f"{sum(r[1] for r in res)} flips {sum(r[2] for r in res)} max rel err {max(r[4] for r in res):.2e}")
    for ng, no, fl, mism, e in res:
        assert not mism and e < 1e-4

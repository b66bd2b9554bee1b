"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element by element.

Tolerances: FP64 path 1e-10 relative; mixed path 1e-4 relative with the noise
mean 4 as floor (|2F_gpu - 2F_ora| / max(2F_ora, 4)).  Candidate key sets must
be equal outside a guard band of 1e-4 * threshold around the threshold
(FP64: 1e-9 * threshold), where a bin can flip legitimately.
"""
import math

import numpy as np
import pytest
import torch as _torch  # imported at collection: the first import on a fresh box is slow

import synth
from oracle import fstat_oracle as ora
from tests import pins
from tests.gpu_util import (assert_keys_equal, compare_candidates, gpu_spectrum, make_plan, note, oracle_spectrum,
                            rel_err_floor)

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
TOL_MIXED = 1e-4
GUARD_FP64 = 1e-9
GUARD_MIXED = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def tiny():
    return synth.workload("tiny")


@pytest.fixture(scope="module")
def full():
    return synth.workload("full")


def _stages(torch, plan, seg, al, de, fp64):
    n, nfft = seg.n, synth.nfft_for(seg.n)
    ct = torch.complex128 if fp64 else torch.complex64
    abc = torch.zeros(3, dtype=torch.float64, device="cuda")
    bufs = [torch.zeros(m, dtype=ct, device="cuda") for m in (n, n, nfft, nfft, n, n)]
    plan.sky_stages(0, al, de, abc, *bufs)
    torch.cuda.synchronize()
    return abc.cpu().numpy(), [b.cpu().numpy().astype(np.complex128) for b in bufs]


def _stage_errors(torch, seg, al, de, fp64):
    plan = make_plan([seg], precision=0 if fp64 else 1)
    abc, (za, zb, ua, ub, zta, ztb) = _stages(torch, plan, seg, al, de, fp64)
    ref = ora.sky_stage(seg, al, de, synth.nfft_for(seg.n))
    ua_ref = ora.fft_upsample2(ref["za"], synth.nfft_for(seg.n))
    ub_ref = ora.fft_upsample2(ref["zb"], synth.nfft_for(seg.n))

    def rel(a, b):
        return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    errs = dict(A=abs(abc[0] - ref["A"]) / ref["A"], B=abs(abc[1] - ref["B"]) / ref["B"],
                C=abs(abc[2] - ref["C"]) / math.sqrt(ref["A"] * ref["B"]),
                za=rel(za, ref["za"]), zb=rel(zb, ref["zb"]), ua=rel(ua, ua_ref), ub=rel(ub, ub_ref),
                zta=rel(zta, ref["za_t"]), ztb=rel(ztb, ref["zb_t"]))
    plan.destroy()
    return errs


def phase_conditioning(seg) -> float:
    """Phase error of one FP64 rounding of the demodulation phase 2 pi f_off n.r(t).

    |r| is about 500 light-seconds, so two correct FP64 evaluations of the phase
    (different summation or FMA order) differ by a few times 2 pi f_off |r| 2^-53
    (3.5e-11 rad at 100 Hz); every demodulated value inherits it as relative error.
    """
    return 2 * math.pi * (seg.f_off + 0.25) * float(np.max(np.abs(seg.r))) * 2.0 ** -53


def test_sky_stages_fp64_tiny(torch, tiny):
    note("sky stages fp64 n=4096")
    seg = tiny.segments[0]
    e = _stage_errors(torch, seg, float(tiny.alpha[3]), float(tiny.delta[3]), True)
    note(str(e))
    assert e["A"] < 1e-13 and e["B"] < 1e-13 and e["C"] < 1e-13
    tol = 8 * phase_conditioning(seg) + 1e-13
    assert max(e.values()) < tol


def test_sky_stages_mixed_full(torch, full):
    note("sky stages mixed n=86164")
    e = _stage_errors(torch, full.segments[0], float(full.alpha[17]), float(full.delta[17]), False)
    note(str(e))
    assert e["A"] < 1e-12 and e["B"] < 1e-12 and e["C"] < 1e-12   # FP64 reductions
    assert e["za"] < 1e-6 and e["zb"] < 1e-6                        # FP32 rounding of the values
    assert e["ua"] < 2e-6 and e["ub"] < 2e-6
    assert e["zta"] < 5e-6 and e["ztb"] < 5e-6


def test_spectrum_fp64_tiny(torch, tiny):
    note("spectrum fp64, N=4096, grid 8x4")
    seg = tiny.segments[0]
    nfft = synth.nfft_for(seg.n)
    plan = make_plan([seg], precision=0)
    got = gpu_spectrum(plan, 0, tiny.alpha, tiny.delta, tiny.fdot, nfft // 2, True)
    ref = oracle_spectrum(seg, tiny.alpha, tiny.delta, tiny.fdot, nfft)
    err = rel_err_floor(got, ref)
    note(f"max rel err {err:.3e}")
    assert err < TOL_FP64


def test_candidates_fp64_tiny(torch, tiny):
    note("candidates fp64, N=4096, grid 8x4")
    seg = tiny.segments[0]
    nfft = synth.nfft_for(seg.n)
    plan = make_plan([seg], precision=0)
    from tests.gpu_util import dev
    plan.search_batch(0, dev(tiny.alpha), dev(tiny.delta), dev(tiny.fdot))
    recs, keys, n = plan.candidates()
    ref = oracle_spectrum(seg, tiny.alpha, tiny.delta, tiny.fdot, nfft)
    ng, no, flips, mism, err = compare_candidates(
        np.stack([keys["sky"], keys["fdot_idx"], keys["bin"]], 1), recs["twoF"], ref, tiny.threshold, GUARD_FP64)
    note(f"gpu {ng} oracle {no} flips {flips} mismatches {len(mism)} err {err:.3e}")
    assert no > 0 and not mism and err < TOL_FP64
    np.testing.assert_allclose(recs["f_hz"], seg.f_off + keys["bin"] / (nfft * seg.dt), rtol=0, atol=1e-12)
    np.testing.assert_array_equal(recs["alpha"], tiny.alpha[keys["sky"]])
    np.testing.assert_array_equal(recs["fdot"], tiny.fdot[keys["fdot_idx"]])


def test_full_form_fp64_tiny(torch, tiny):
    note("full F form fp64")
    seg = tiny.segments[0]
    nfft = synth.nfft_for(seg.n)
    plan = make_plan([seg], precision=0, form=1)
    al, de, fd = tiny.alpha[:3], tiny.delta[:3], tiny.fdot[:2]
    got = gpu_spectrum(plan, 0, al, de, fd, nfft // 2, True)
    ref = oracle_spectrum(seg, al, de, fd, nfft, full=True)
    assert rel_err_floor(got, ref) < TOL_FP64


def test_spectrum_mixed_full_segment(torch, full):
    note("spectrum mixed n=86164, 2 sky x 3 spindowns")
    seg = full.segments[0]
    nfft = synth.nfft_for(seg.n)
    plan = make_plan([seg])
    al, de, fd = full.alpha[[0, 101]], full.delta[[0, 101]], full.fdot[[0, 31, 63]]
    got = gpu_spectrum(plan, 0, al, de, fd, nfft // 2, False)
    ref = oracle_spectrum(seg, al, de, fd, nfft)
    err = rel_err_floor(got, ref)
    note(f"max rel err {err:.3e}")
    assert err < TOL_MIXED


def test_candidates_mixed_full_segment(torch, full):
    note("candidates mixed n=86164, 2 sky x 3 spindowns")
    seg = full.segments[0]
    nfft = synth.nfft_for(seg.n)
    plan = make_plan([seg])
    from tests.gpu_util import dev
    al, de, fd = full.alpha[[5, 77]], full.delta[[5, 77]], full.fdot[[1, 40, 62]]
    plan.search_batch(0, dev(al), dev(de), dev(fd))
    recs, keys, n = plan.candidates()
    ref = oracle_spectrum(seg, al, de, fd, nfft)
    ng, no, flips, mism, err = compare_candidates(
        np.stack([keys["sky"], keys["fdot_idx"], keys["bin"]], 1), recs["twoF"], ref, full.threshold, GUARD_MIXED)
    note(f"gpu {ng} oracle {no} flips {flips} mismatches {len(mism)} err {err:.3e}")
    assert no > 50 and not mism and err < TOL_MIXED


def test_injection_recovered_mixed(torch):
    note("noiseless on-grid injection, mixed")
    seg, inj, k0, nfft = pins.on_grid_injection(synth.N_FULL)
    plan = make_plan([seg])
    got = gpu_spectrum(plan, 0, np.array([inj.alpha]), np.array([inj.delta]), np.array([inj.fdot]), nfft // 2, False)
    sky = ora.sky_stage(seg, inj.alpha, inj.delta, nfft)
    cf = pins.closed_form_two_f(inj, sky["A"], sky["B"], sky["C"], seg.n)
    assert int(np.argmax(got[0, 0])) == k0
    assert abs(got[0, 0, k0] - cf) / cf < 1e-3


@pytest.mark.parametrize("n", [2048, 4096, 20000, 45000])
def test_ragged_lengths_mixed(torch, n):
    note(f"ragged length n={n}")
    rng = np.random.default_rng(n)
    injs = synth.draw_injections(rng, 1, 15.0, 15.0)
    f_off = float(synth.band_offset(int(rng.integers(0, 1000))))
    seg = synth.make_segment(n, 2.0, f_off, 1.0, 4000 + n, injs)
    nfft = synth.nfft_for(n)
    plan = make_plan([seg])
    al, de = np.array([0.3, injs[0].alpha]), np.array([-0.2, injs[0].delta])
    fd = np.array([0.0, injs[0].fdot])
    got = gpu_spectrum(plan, 0, al, de, fd, nfft // 2, False)
    ref = oracle_spectrum(seg, al, de, fd, nfft)
    err = rel_err_floor(got, ref)
    note(f"n={n} nfft={nfft} max rel err {err:.3e}")
    assert err < TOL_MIXED


def test_bin_range_matches_full_spectrum(torch, tiny):
    seg = tiny.segments[0]
    nfft = synth.nfft_for(seg.n)
    full_plan = make_plan([seg], precision=0)
    part_plan = make_plan([seg], precision=0, k_min=1000, k_max=3001)
    al, de, fd = tiny.alpha[:2], tiny.delta[:2], tiny.fdot[:2]
    a = gpu_spectrum(full_plan, 0, al, de, fd, nfft // 2, True)
    b = gpu_spectrum(part_plan, 0, al, de, fd, 2001, True)
    np.testing.assert_array_equal(a[:, :, 1000:3001], b)


def test_bin_range_across_half_spectrum_mixed(torch, full):
    """Mixed precision with a bin range that is not [0, nfft/2): the second pass forms every
    output of its last stage and checks bins, here across nfft/2 into the upper half."""
    note("bin range [100000, 200000), mixed")
    seg = full.segments[0]
    nfft = synth.nfft_for(seg.n)
    k0, k1 = 100000, 200000
    al, de, fd = full.alpha[:2], full.delta[:2], full.fdot[:2]
    plan = make_plan([seg], k_min=k0, k_max=k1)
    got = gpu_spectrum(plan, 0, al, de, fd, k1 - k0, False)
    ref = oracle_spectrum(seg, al, de, fd, nfft, k0, k1)
    err = rel_err_floor(got, ref)
    note(f"spectrum max rel err {err:.3e}")
    assert err < TOL_MIXED
    from tests.gpu_util import dev
    plan.search_batch(0, dev(al), dev(de), dev(fd))
    recs, keys, n = plan.candidates()
    assert np.all((keys["bin"] >= k0) & (keys["bin"] < k1))
    key3 = np.stack([keys["sky"], keys["fdot_idx"], keys["bin"]], 1)
    ng, no, flips, mism, e2 = compare_candidates(key3, recs["twoF"], ref, full.threshold, GUARD_MIXED, k_min=k0)
    note(f"gpu {ng} oracle {no} flips {flips} mismatches {len(mism)}")
    assert no > 0 and not mism


def test_plain_launches_equal_batched(torch, full):
    note("one template per launch vs batched")
    seg = full.segments[0]
    from tests.gpu_util import dev
    al, de, fd = dev(full.alpha[:3]), dev(full.delta[:3]), dev(full.fdot[:5])
    out = []
    for opts in (dict(templates_per_launch=1, skies_per_batch=1), dict()):
        plan = make_plan([seg], **opts)
        plan.search_batch(0, al, de, fd)
        out.append(plan.candidates())
        plan.destroy()
    (r1, k1, n1), (r2, k2, n2) = out
    assert n1 == n2 and n1 > 0
    assert_keys_equal(k1, k2)
    np.testing.assert_array_equal(r1, r2)


def test_candidate_overflow_reports_true_count(torch, tiny):
    seg = tiny.segments[0]
    from tests.gpu_util import dev
    from paper_1410_3677_amd import fstat as F
    al, de, fd = dev(tiny.alpha), dev(tiny.delta), dev(tiny.fdot)
    big = make_plan([seg], precision=0)
    big.search_batch(0, al, de, fd)
    _, _, n_all = big.candidates()
    small = make_plan([seg], precision=0, candidate_capacity=7)
    small.search_batch(0, al, de, fd)
    with pytest.raises(F.FstatError) as ei:
        small.candidates()
    assert ei.value.status == F.E_OVERFLOW
    small.search_batch(0, al, de, fd)
    recs, keys, n = small.candidates(allow_overflow=True)
    assert n == n_all > 7 and len(recs) == 7


def test_dense_crossings_match_oracle_mixed(torch, full):
    """A low threshold (2F > 5: about 29% of bins) gives rows with more crossings than a
    wavefront stages at once, so staged, flushed and burst emission all run."""
    note("dense crossings, mixed, threshold 5")
    seg = full.segments[0]
    nfft = synth.nfft_for(seg.n)
    from tests.gpu_util import dev
    al, de, fd = full.alpha[:1], full.delta[:1], full.fdot[:2]
    plan = make_plan([seg], threshold_2F=5.0, candidate_capacity=1 << 20)
    plan.search_batch(0, dev(al), dev(de), dev(fd))
    recs, keys, n = plan.candidates()
    ref = oracle_spectrum(seg, al, de, fd, nfft)
    key3 = np.stack([keys["sky"], keys["fdot_idx"], keys["bin"]], 1)
    ng, no, flips, mism, err = compare_candidates(key3, recs["twoF"], ref, 5.0, 1e-4)
    note(f"gpu {ng} oracle {no} flips {flips} mismatches {len(mism)} err {err:.3e}")
    assert no > 50000 and not mism and err < 1e-4
    # every key once
    assert len(np.unique(key3, axis=0)) == len(key3)


def test_candidate_overflow_mixed_keeps_a_valid_subset(torch, full):
    seg = full.segments[0]
    from tests.gpu_util import dev
    from paper_1410_3677_amd import fstat as F
    al, de, fd = dev(full.alpha[:2]), dev(full.delta[:2]), dev(full.fdot[:3])
    big = make_plan([seg])
    big.search_batch(0, al, de, fd)
    r_all, k_all, n_all = big.candidates()
    small = make_plan([seg], candidate_capacity=50)
    small.search_batch(0, al, de, fd)
    with pytest.raises(F.FstatError) as ei:
        small.candidates()
    assert ei.value.status == F.E_OVERFLOW
    small.search_batch(0, al, de, fd)
    recs, keys, n = small.candidates(allow_overflow=True)
    assert n == n_all > 50 and len(recs) == 50
    full_set = {(int(a), int(b), int(c)): float(f) for a, b, c, f in
                zip(k_all["sky"], k_all["fdot_idx"], k_all["bin"], r_all["twoF"])}
    for a, b, c, f in zip(keys["sky"], keys["fdot_idx"], keys["bin"], recs["twoF"]):
        assert full_set[(int(a), int(b), int(c))] == float(f)


def test_graph_replays_match_eager_launches(torch, full):
    note("graph replays vs eager launches")
    seg = full.segments[0]
    from tests.gpu_util import dev
    al, de, fd = dev(full.alpha[:9]), dev(full.delta[:9]), dev(full.fdot[:7])
    eager = make_plan([seg], use_graph=0, skies_per_batch=4, templates_per_launch=16)
    eager.search_batch(0, al, de, fd)
    r0, k0, n0 = eager.candidates()
    assert n0 > 0
    graph = make_plan([seg], use_graph=1, skies_per_batch=4, templates_per_launch=16)
    for rep in range(3):
        graph.search_batch(0, al, de, fd)
        # the program's own eager work and a synchronisation between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2.0).sum().item()
        torch.cuda.synchronize()
        r, k, n = graph.candidates()
        assert n == n0, rep
        np.testing.assert_array_equal(k[["segment", "sky", "fdot_idx", "bin"]], k0[["segment", "sky", "fdot_idx", "bin"]])
        assert np.all(k["search"] == rep)
        np.testing.assert_array_equal(r, r0)


def test_autotune_writes_cache_and_plans_pick_it_up(torch, full, tmp_path):
    note("autotuner")
    from paper_1410_3677_amd import fstat as F
    seg = full.segments[0]
    cache = str(tmp_path / "tuning.txt")
    plan = F.Plan([F.segment_to_device(seg)], workspace_from_torch=False, tuning_cache_path=cache)
    info = plan.autotune(0, budget_ms=600.0)
    note(f"tuned {info}")
    assert info["templates_per_launch"] in (64, 128, 256, 512)
    assert info["skies_per_batch"] in (16, 32) and info["pass_a_variant"] in (0, 1)
    line = open(cache).read().split()
    assert len(line) == 6 and int(line[1]) == synth.nfft_for(seg.n)
    again = F.Plan([F.segment_to_device(seg)], tuning_cache_path=cache)
    assert again.info(0) == info


def test_kernel_variants_give_identical_candidates(torch, full, tmp_path):
    """Both first-pass and both second-pass kernels (selected through the tuning cache)
    find the same candidates; 2F agrees to rounding (the half-output last stage and
    multiply-add contraction differ in the last bits)."""
    note("pass A x pass B kernel variants")
    from paper_1410_3677_amd import fstat as F
    from tests.gpu_util import dev
    seg = full.segments[0]
    nfft = synth.nfft_for(seg.n)
    # the device tag the library writes is learned from a one-line tuning run
    probe = str(tmp_path / "probe.txt")
    p0 = F.Plan([F.segment_to_device(seg)], workspace_from_torch=False, tuning_cache_path=probe)
    p0.autotune(0, budget_ms=50.0)
    tag = open(probe).read().split()[0]
    out = []
    for v in (0, 1, 2, 3):
        cache = tmp_path / f"v{v}.txt"
        cache.write_text(f"{tag} {nfft} 1 64 8 {v}\n")
        plan = F.Plan([F.segment_to_device(seg)], tuning_cache_path=str(cache), use_graph=0)
        inf = plan.info(0)
        assert (inf["pass_a_variant"], inf["pass_b_variant"]) == (v & 1, v >> 1)
        plan.search_batch(0, dev(full.alpha[:3]), dev(full.delta[:3]), dev(full.fdot[:70]))
        out.append(plan.candidates())
    r0, k0, n0 = out[0]
    assert n0 > 0
    for r1, k1, n1 in out[1:]:
        assert n1 == n0
        assert_keys_equal(k0, k1)
        np.testing.assert_allclose(r0["twoF"], r1["twoF"], rtol=2e-6, atol=0)


def test_rows_of_1024_points_streaming_equals_tiled(torch, tmp_path):
    """nfft = 2^19 (rows of P = 1024 points, two wavefronts each in the streaming second
    pass): the streaming and the tiled second pass find the same candidates with the same
    2F, and the streaming pass's spectrum of a bin range (every output formed) and of the
    bins [0, nfft/2) (half the outputs) match the oracle."""
    from paper_1410_3677_amd import fstat as F
    from tests.gpu_util import dev
    n = 150000
    rng = np.random.default_rng(1024)
    injs = synth.draw_injections(rng, 1, 15.0, 15.0)
    seg = synth.make_segment(n, 2.0, 100.0, 1.0, 6150, injs)
    nfft = synth.nfft_for(n)
    assert nfft == 1 << 19
    note(f"rows of 1024 points: n={n} nfft={nfft}")
    al, de = np.array([0.3, injs[0].alpha, -1.1]), np.array([-0.2, injs[0].delta, 0.7])
    fd = np.array([0.0, injs[0].fdot])
    probe = str(tmp_path / "probe.txt")
    p0 = F.Plan([F.segment_to_device(seg)], workspace_from_torch=False, tuning_cache_path=probe)
    p0.autotune(0, budget_ms=50.0)
    tag = open(probe).read().split()[0]
    for v in (0, 2):   # second pass variant 0 (tiled) and 1 (streaming)
        (tmp_path / f"v{v}.txt").write_text(f"{tag} {nfft} 1 64 8 {v}\n")
    for k_min, k_max in ((0, 0), (1000, 200001)):   # all outputs of a row formed on the second range
        found = []
        for v in (0, 2):
            plan = F.Plan([F.segment_to_device(seg)], tuning_cache_path=str(tmp_path / f"v{v}.txt"), use_graph=0,
                          k_min=k_min, k_max=k_max)
            inf = plan.info(0)
            assert inf["p"] == 1024 and inf["pass_b_variant"] == v >> 1
            plan.search_batch(0, dev(al), dev(de), dev(fd))
            found.append(plan.candidates())
        (r0, k0, n0), (r1, k1, n1) = found
        note(f"bins [{k_min}, {k_max or nfft // 2}): {n0} candidates")
        assert n0 > 0 and n1 == n0
        assert_keys_equal(k0, k1)
        np.testing.assert_allclose(r0["twoF"], r1["twoF"], rtol=2e-6, atol=0)
    cache = tmp_path / "v2.txt"
    for k_min, k_max in ((0, nfft // 2), (1000, 200001)):
        plan = F.Plan([F.segment_to_device(seg)], tuning_cache_path=str(cache), use_graph=0, k_min=k_min,
                      k_max=k_max)
        assert plan.info(0)["pass_b_variant"] == 1
        got = gpu_spectrum(plan, 0, al, de, fd, k_max - k_min, False)
        ref = oracle_spectrum(seg, al, de, fd, nfft, k_min, k_max)
        err = rel_err_floor(got, ref)
        note(f"bins [{k_min}, {k_max}): max rel err {err:.3e}")
        assert err < TOL_MIXED


@pytest.fixture(scope="module")
def ragged():
    return synth.workload("ragged", nsky=3, nfdot=4)


def test_ragged_segments_in_one_search(torch, ragged):
    note("ragged: 32 segments in one search call")
    from tests.gpu_util import dev
    segs = ragged.segments
    plan = make_plan(segs)
    for i in range(len(segs)):
        assert plan.info(i)["nfft"] == synth.nfft_for(segs[i].n)
    plan.search_batch(-1, dev(ragged.alpha), dev(ragged.delta), dev(ragged.fdot))
    recs, keys, n = plan.candidates()
    assert n > 0 and set(np.unique(keys["segment"])) <= set(range(len(segs)))
    order = np.argsort([s.n for s in segs])
    for si in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        seg = segs[si]
        nfft = synth.nfft_for(seg.n)
        m = keys["segment"] == si
        ref = oracle_spectrum(seg, ragged.alpha, ragged.delta, ragged.fdot, nfft)
        ng, no, flips, mism, err = compare_candidates(
            np.stack([keys["sky"][m], keys["fdot_idx"][m], keys["bin"][m]], 1), recs["twoF"][m], ref,
            ragged.threshold, GUARD_MIXED)
        note(f"segment {si} n={seg.n} nfft={nfft}: gpu {ng} oracle {no} flips {flips} err {err:.2e}")
        assert not mism and err < TOL_MIXED
        np.testing.assert_allclose(recs["f_hz"][m], seg.f_off + keys["bin"][m] / (nfft * seg.dt), rtol=0, atol=1e-9)


def test_ragged_admission_with_small_budget_gives_same_candidates(torch, ragged):
    note("ragged: memory-bounded admission")
    from tests.gpu_util import dev
    from paper_1410_3677_amd import fstat as F
    segs = ragged.segments[:8]
    args = (dev(ragged.alpha), dev(ragged.delta), dev(ragged.fdot))
    big = make_plan(segs)
    big.search_batch(-1, *args)
    r0, k0, n0 = big.candidates()
    # a budget that only fits one sky and a handful of templates of the largest segment
    budget = 80 << 20
    small = make_plan(segs, workspace_budget_bytes=budget)
    inf = small.info(0)
    assert inf["templates_per_launch"] < big.info(0)["templates_per_launch"]
    assert small.workspace.numel() <= budget + 256
    small.search_batch(-1, *args)
    r1, k1, n1 = small.candidates()
    assert n1 == n0
    assert_keys_equal(k0, k1)
    np.testing.assert_allclose(r0["twoF"], r1["twoF"], rtol=1e-6, atol=0)
    with pytest.raises(F.FstatError) as ei:
        make_plan(segs, workspace_budget_bytes=4 << 20)
    assert ei.value.status == F.E_ADMISSION


@pytest.mark.parametrize("precision", [1, 0])
def test_longest_segment(torch, precision):
    """n = 2^19, the longest segment the library takes: nfft = 2^20, P = Q = 1024 (the
    tiled second pass in both precisions)."""
    n = 1 << 19
    rng = np.random.default_rng(19)
    injs = synth.draw_injections(rng, 1, 15.0, 15.0)
    seg = synth.make_segment(n, 2.0, 100.0, 1.0, 5119, injs)
    nfft = synth.nfft_for(n)
    note(f"longest segment n={n} nfft={nfft} precision={precision}")
    plan = make_plan([seg], precision=precision)
    inf = plan.info(0)
    assert inf["nfft"] == 1 << 20 and inf["p"] * inf["q"] == 1 << 20
    al, de = np.array([0.3, injs[0].alpha]), np.array([-0.2, injs[0].delta])
    fd = np.array([injs[0].fdot])
    got = gpu_spectrum(plan, 0, al, de, fd, nfft // 2, precision == 0)
    ref = oracle_spectrum(seg, al, de, fd, nfft)
    err = rel_err_floor(got, ref)
    note(f"max rel err {err:.3e}")
    assert err < (TOL_FP64 if precision == 0 else TOL_MIXED)

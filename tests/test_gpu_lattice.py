"""GPU parity of the lattice grid (sky loop over the grid integers, spindown integers, the
frequency shift onto the Fourier bins) against the oracle.

* sky points: the on-sky decision, the order and the integers are bit-exact; so are the
  per-sky w components (plain IEEE products and sums on both sides); alpha, delta agree
  to 1e-13 rad (library atan2 / asin);
* spectra of lattice templates (shifted frequencies, per-sky spindown offsets) element by
  element: 1e-10 (FP64), 1e-4 (mixed) relative with floor 4, zero-padded and interbinned;
* candidate records: keys equal (mixed: outside a 1e-4 x threshold guard band), f_hz and
  fdot equal to the oracle's to rounding, alpha and delta to 1e-13;
* full size (N = 86164, nfft = 2^18): a noiseless-plus-noise source at a shifted grid
  point is found at its bin with its frequency, sampled templates match bin by bin.
"""
import math

import numpy as np
import pytest
import torch as _torch  # noqa: F401  (first import on a fresh box is slow)

import synth
from oracle import fstat_oracle as ora
from tests import pins
from tests.gpu_util import compare_candidates, make_plan, note, rel_err_floor

pytestmark = pytest.mark.gpu

EPS = synth.OBLIQUITY


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _lattice(n, sky_points, seed, dt=2.0, f_off=100.0):
    from paper_1410_3677_amd import fstat as F
    nfft = synth.nfft_for(n)
    f_ref = f_off + 0.5 / dt
    M = synth.lattice_matrix(nfft, dt, f_ref, sky_points, -2e-10, seed)
    return M, f_ref, F.lattice(M, EPS, f_ref)


def _ang(a, b):
    return np.abs((np.asarray(a) - np.asarray(b) + math.pi) % (2 * math.pi) - math.pi)


@pytest.mark.parametrize("sky_points,seed,hemi", [(12, 1, 1), (50, 2, -1), (4000, 3, 1), (30000, 4, -1)])
def test_sky_points_match_the_oracle(torch, sky_points, seed, hemi):
    from paper_1410_3677_amd import fstat as F
    M, f_ref, lat = _lattice(4096, sky_points, seed)
    box = F.lattice_sky_range(lat)
    note(f"lattice sky, ~{sky_points} points per hemisphere, box {box}, hemisphere {hemi}")
    got = F.lattice_sky(lat, hemi, box)
    ref = ora.lattice_sky_points(M, box, hemi, EPS, f_ref)
    assert got["count"] == len(ref) > 0
    nm = got["nm"].cpu().numpy()
    np.testing.assert_array_equal(nm, np.array([(p[0], p[1]) for p in ref], dtype=np.int32))
    np.testing.assert_array_equal(got["w_freq"].cpu().numpy(), np.array([p[4] for p in ref]))
    np.testing.assert_array_equal(got["w_spin"].cpu().numpy(), np.array([p[5] for p in ref]))
    assert np.max(_ang(got["alpha"].cpu().numpy(), [p[2] for p in ref])) < 1e-13
    assert np.max(np.abs(got["delta"].cpu().numpy() - [p[3] for p in ref])) < 1e-13
    a = got["alpha"].cpu().numpy()
    assert np.all((a >= 0) & (a <= 2 * math.pi))


def test_sky_capacity_and_a_box_off_the_sky(torch):
    from paper_1410_3677_amd import fstat as F
    M, f_ref, lat = _lattice(4096, 400, 5)
    box = F.lattice_sky_range(lat)
    full = ora.lattice_sky_points(M, box, 1, EPS, f_ref)
    got = F.lattice_sky(lat, 1, box, capacity=100)
    assert got["count"] == len(full) > 100
    np.testing.assert_array_equal(got["nm"].cpu().numpy(), np.array([(p[0], p[1]) for p in full[:100]]))
    off = (box[1] + 1, box[1] + 40, box[2], box[3])
    assert F.lattice_sky(lat, 1, off)["count"] == 0
    assert F.lattice_sky(lat, -1, box, capacity=0)["count"] == len(full)


def _oracle_spectra(seg, M, pts, idx, s_lo, s_hi, nfft, interbin=False):
    out = []
    for i in idx:
        _, _, al, de, w0, w1 = pts[i]
        sky = ora.sky_stage(seg, al, de, nfft)
        row = []
        for s in range(s_lo, s_hi + 1):
            tw1, u = ora.lattice_template(M, s, w0, w1, nfft)
            row.append(ora.lattice_template_two_f(seg, sky, tw1, u, nfft, interbin=interbin))
        out.append(row)
    return np.array(out)


def _gpu_sky(F, lat, hemi, k):
    sky = F.lattice_sky(lat, hemi)
    return {key: (v[:k] if key != "count" else v) for key, v in sky.items()}


@pytest.mark.parametrize("precision,ib", [(0, 0), (1, 0), (1, 1)])
def test_lattice_spectra_match_the_oracle(torch, precision, ib):
    from paper_1410_3677_amd import fstat as F
    n = 4096
    nfft = synth.nfft_for(n)
    M, f_ref, lat = _lattice(n, 12, 6)
    seg = synth.make_segment(n, 2.0, 100.0, 1.0, 606, [])
    pts = ora.lattice_sky_points(M, ora.lattice_sky_range(M, f_ref), 1, EPS, f_ref)
    k = min(5, len(pts))
    s_lo, s_hi = -2, 2
    note(f"lattice spectra, N={n}, {k} sky x {s_hi - s_lo + 1} spindowns, precision={precision}, interbinning={ib}")
    plan = make_plan([seg], precision=precision, interbinning=ib)
    sky = _gpu_sky(F, lat, 1, k)
    nb = nfft // 2
    out = torch.empty(k * (s_hi - s_lo + 1) * nb, dtype=torch.float64 if precision == 0 else torch.float32,
                      device="cuda")
    plan.search_lattice(0, lat, sky, s_lo, s_hi, spectrum=out)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy().reshape(k, s_hi - s_lo + 1, nb)
    ref = _oracle_spectra(seg, M, pts, range(k), s_lo, s_hi, nfft, interbin=bool(ib))
    err = rel_err_floor(got, ref)
    us = [ora.lattice_template(M, s, pts[i][4], pts[i][5], nfft)[1] for i in range(k) for s in range(s_lo, s_hi + 1)]
    note(f"max rel err {err:.3e}; shifts u from {min(us):.3f} to {max(us):.3f}")
    assert max(us) - min(us) > 0.3
    assert err < (1e-10 if precision == 0 else 1e-4)


@pytest.mark.parametrize("precision", [0, 1])
def test_lattice_candidates_match_the_oracle(torch, precision):
    from paper_1410_3677_amd import fstat as F
    n = 4096
    nfft = synth.nfft_for(n)
    M, f_ref, lat = _lattice(n, 12, 7)
    seg = synth.make_segment(n, 2.0, 100.0, 1.0, 707, [])
    pts = ora.lattice_sky_points(M, ora.lattice_sky_range(M, f_ref), -1, EPS, f_ref)
    k = min(4, len(pts))
    s_lo, s_hi, thr = -3, 1, 10.0
    plan = make_plan([seg], precision=precision, threshold_2F=thr)
    sky = _gpu_sky(F, lat, -1, k)
    plan.search_lattice(0, lat, sky, s_lo, s_hi)
    recs, keys, cnt = plan.candidates()
    ref = ora.search_lattice(seg, M, pts[:k], s_lo, s_hi, thr)
    note(f"lattice candidates, precision={precision}: gpu {cnt}, oracle {len(ref)}")
    if precision == 0:
        for f in ("sky", "fdot_idx", "bin"):
            np.testing.assert_array_equal(keys[f], ref[f])
        mask = np.ones(len(ref), dtype=bool)
        g_idx = np.arange(len(ref))
    else:
        spec = _oracle_spectra(seg, M, pts, range(k), s_lo, s_hi, nfft)
        key3 = np.stack([keys["sky"], keys["fdot_idx"], keys["bin"]], 1)
        ng, no, flips, mism, err = compare_candidates(key3, recs["twoF"], spec, thr, 1e-4)
        assert not mism and err < 1e-4
        rkeys = {(int(a), int(b), int(c)): j for j, (a, b, c) in enumerate(zip(ref["sky"], ref["fdot_idx"], ref["bin"]))}
        pairs = [(j, rkeys[tuple(int(v) for v in kk)]) for j, kk in enumerate(key3) if tuple(int(v) for v in kk) in rkeys]
        g_idx = np.array([p[0] for p in pairs])
        mask = np.array([p[1] for p in pairs])
    assert len(g_idx) > 20
    r = ref[mask]
    g = recs[g_idx]
    np.testing.assert_allclose(g["f_hz"], r["f_hz"], rtol=1e-15, atol=0)
    np.testing.assert_allclose(g["fdot"], r["fdot"], rtol=1e-15, atol=0)
    assert np.max(_ang(g["alpha"], r["alpha"])) < 1e-13
    assert np.max(np.abs(g["delta"] - r["delta"])) < 1e-13
    assert rel_err_floor(g["twoF"], r["twoF"]) < (1e-10 if precision == 0 else 1e-4)
    # the frequencies are the shifted grid's, not the bins'
    assert np.max(np.abs((g["f_hz"] - seg.f_off) * nfft * seg.dt - keys["bin"][g_idx])) > 0.2


def test_lattice_constraints_are_enforced(torch):
    from paper_1410_3677_amd import fstat as F
    n = 4096
    M, f_ref, lat = _lattice(n, 12, 8)
    seg = synth.make_segment(n, 2.0, 100.0, 1.0, 808, [])
    plan = make_plan([seg])
    sky = _gpu_sky(F, lat, 1, 3)
    bad = []
    m = M.copy(); m[0, 2] = 1e-3; bad.append((m, "row 0"))
    m = M.copy(); m[1, 3] = 1e-3; bad.append((m, "row 1"))
    m = M.copy(); m[0, 0] *= 1.5; bad.append((m, "whole number"))
    for mm, needle in bad:
        with pytest.raises(F.FstatError) as ei:
            plan.search_lattice(0, F.lattice(mm, EPS, f_ref), sky, -1, 1)
        assert ei.value.status == F.E_INVAL and needle in str(ei.value)
    with pytest.raises(F.FstatError):
        plan.search_lattice(0, lat, sky, 2, 1)
    out = torch.empty(16, device="cuda")
    with pytest.raises(F.FstatError):
        plan.search_lattice(-1, lat, sky, 0, 0, spectrum=out)
    # two Fourier bins per frequency step is a valid grid
    m2 = M.copy(); m2[0, 0] *= 2.0
    plan.search_lattice(0, F.lattice(m2, EPS, f_ref), sky, 0, 0)
    plan.candidates()


def test_full_size_source_at_a_shifted_grid_point(torch):
    """N = 86164, nfft = 2^18: a SNR-10 source (with noise) exactly at a lattice point whose
    frequencies sit a fraction of a bin above the Fourier bins; the batched search over
    one hemisphere of the lattice finds it at its bin with its frequency and spindown, and
    sampled templates match the oracle bin by bin."""
    from paper_1410_3677_amd import fstat as F
    n = synth.N_FULL
    dt, f_off = 2.0, 100.0
    nfft, f_ref, M, pts = pins.lattice_setup(n, dt, f_off, sky_points=60, seed=41)
    lat = F.lattice(M, EPS, f_ref)
    s_lo, s_hi = -8, 7
    pick = None
    for i, p in enumerate(pts):
        for s in range(s_lo, s_hi + 1):
            w1, u = ora.lattice_template(M, s, p[4], p[5], nfft)
            if 0.3 < u < 0.7 and w1 < 0:
                pick = (i, s, w1, u)
                break
        if pick:
            break
    i0, s0, w1, u = pick
    k0 = int(0.3 * nfft)
    inj = synth.Injection(f=(k0 + u) / (nfft * dt), fdot=w1 / (math.pi * dt * dt), alpha=pts[i0][2],
                          delta=pts[i0][3], psi=0.4, cosi=0.6, phi0=2.2, snr=10.0)
    seg = synth.make_segment(n, dt, f_off, 1.0, 4141, [inj])
    thr = 20.0
    note(f"full-size lattice search: {len(pts)} sky x {s_hi - s_lo + 1} spindowns, source at sky {i0}, s {s0}, "
         f"u {u:.3f}")
    plan = make_plan([seg], workspace_from_torch=False, threshold_2F=thr, candidate_capacity=1 << 22)
    plan.autotune(0)
    sky = F.lattice_sky(lat, 1)
    assert sky["count"] == len(pts)
    plan.search_lattice(0, lat, sky, s_lo, s_hi)
    recs, keys, cnt = plan.candidates()
    assert cnt == len(recs) > 1000
    hit = (keys["sky"] == i0) & (keys["fdot_idx"] == s0 - s_lo) & (keys["bin"] == k0)
    assert hit.sum() == 1
    rec = recs[hit][0]
    assert abs(rec["f_hz"] - (f_off + inj.f)) < 1e-12
    assert abs(rec["fdot"] - inj.fdot) < 1e-22
    rng = np.random.default_rng(43)
    picks = [(i0, s0 - s_lo)] + [(int(rng.integers(len(pts))), int(rng.integers(s_hi - s_lo + 1))) for _ in range(2)]
    for (i, si) in picks:
        ref = _oracle_spectra(seg, M, pts, [i], s_lo + si, s_lo + si, nfft)
        m = (keys["sky"] == i) & (keys["fdot_idx"] == si)
        key3 = np.stack([np.zeros(int(m.sum()), dtype=np.int64), np.zeros(int(m.sum()), dtype=np.int64),
                         keys["bin"][m]], 1)
        ng, no, flips, mism, err = compare_candidates(key3, recs["twoF"][m], ref, thr, 1e-4)
        note(f"template (sky {i}, s {s_lo + si}): gpu {ng} oracle {no} flips {flips} mismatches {len(mism)} "
             f"err {err:.2e}")
        assert not mism and err < 1e-4
    note(f"source: 2F {rec['twoF']:.2f} at f {rec['f_hz']:.12f} Hz")


@pytest.mark.parametrize("ib", [0, 1])
def test_ragged_segments_in_one_lattice_call_equal_separate_plans(torch, ib):
    """All segments in one lattice call (segment = -1): every segment has its own nfft, so
    its own frequency shifts u; the frequency row is one bin of the shortest transform,
    a whole number of bins of every longer one."""
    from paper_1410_3677_amd import fstat as F
    w = synth.workload("ragged")
    segs = w.segments[:4]
    nffts = [synth.nfft_for(s.n) for s in segs]
    f_ref = 100.25
    M = synth.lattice_matrix(min(nffts), 2.0, f_ref, 12, -2e-10, 17)
    lat = F.lattice(M, EPS, f_ref)
    note(f"lattice, ragged, interbinning={ib}: " + ", ".join(f"n={s.n}" for s in segs))
    sky = _gpu_sky(F, lat, 1, 3)
    pts = ora.lattice_sky_points(M, ora.lattice_sky_range(M, f_ref), 1, EPS, f_ref)[:3]
    plan = make_plan(segs, interbinning=ib)
    plan.search_lattice(-1, lat, sky, -2, 2)
    r_all, k_all, n_all = plan.candidates()
    assert n_all > 0
    for si, seg in enumerate(segs):
        one = make_plan([seg], interbinning=ib)
        one.search_lattice(0, lat, sky, -2, 2)
        r1, k1, n1 = one.candidates()
        m = k_all["segment"] == si
        assert int(m.sum()) == n1, (si, int(m.sum()), n1)
        for f in ("sky", "fdot_idx", "bin"):
            np.testing.assert_array_equal(k_all[f][m], k1[f])
        np.testing.assert_allclose(r_all["twoF"][m], r1["twoF"], rtol=1e-6, atol=0)
        np.testing.assert_array_equal(r_all["f_hz"][m], r1["f_hz"])
        # each record's frequency uses its own segment's nfft and shift
        nfft = nffts[si]
        for j in np.nonzero(m)[0][:20]:
            p = pts[k_all["sky"][j]]
            w1, u = ora.lattice_template(M, -2 + int(k_all["fdot_idx"][j]), p[4], p[5], nfft)
            assert r_all["f_hz"][j] == seg.f_off + (int(k_all["bin"][j]) + u) / (nfft * seg.dt)
            assert r_all["fdot"][j] == w1 / (math.pi * seg.dt * seg.dt)
        one.destroy()


def test_graph_replays_follow_the_lattice(torch):
    """Searches are captured as HIP graphs keyed on their arguments: a repeated lattice call
    replays its graph with the same result, and a call with another spindown row (same
    device arrays) is not served by the stale graph."""
    from paper_1410_3677_amd import fstat as F
    n = 4096
    M, f_ref, lat = _lattice(n, 12, 9)
    M2 = M.copy()
    M2[1, 0] += 0.37 * 2 * math.pi / synth.nfft_for(n)
    M2[1, 1] *= 1.5
    lat2 = F.lattice(M2, EPS, f_ref)
    seg = synth.make_segment(n, 2.0, 100.0, 1.0, 909, [])
    sky = _gpu_sky(F, lat, 1, 3)
    plan = make_plan([seg], threshold_2F=8.0)
    res = []
    for lt in (lat, lat, lat2, lat2, lat):
        plan.search_lattice(0, lt, sky, -2, 2)
        r, k, cnt = plan.candidates()
        res.append((r, k))
    fresh = []
    for lt in (lat, lat2):
        p = make_plan([seg], threshold_2F=8.0, use_graph=0)
        p.search_lattice(0, lt, sky, -2, 2)
        r, k, cnt = p.candidates()
        fresh.append((r, k))
    for got, want in zip(res, [fresh[0], fresh[0], fresh[1], fresh[1], fresh[0]]):
        assert len(got[0]) == len(want[0]) > 10
        for f in ("sky", "fdot_idx", "bin"):
            np.testing.assert_array_equal(got[1][f], want[1][f])
        np.testing.assert_array_equal(got[0], want[0])
    assert not np.array_equal(res[0][0]["f_hz"][:10], res[2][0]["f_hz"][:10])

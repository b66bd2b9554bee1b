"""Pins of the FP64 oracle against mathematics outside itself (CPU only)."""
import math
import os

import numpy as np
import pytest

from oracle import fstat_oracle as oracle
import synth
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_p0_amplitude_modulation_matches_detector_tensor():
    # a(t), b(t) closed forms vs D(t):e+, D(t):ex at psi = 0, over random detectors
    assert pins.p0_amplitude_vs_tensor() < 1e-13


def test_p4_fourier_transform_matches_bruteforce_dft():
    assert pins.p4_fft_vs_bruteforce() < 1e-13
    assert pins.p4_fft_vs_bruteforce(n=64, nfft=64) < 1e-13


def test_p4_forward_sign_puts_tone_on_its_bin():
    assert pins.p4_tone_peak_bin(256, 37) == 37


def test_upsampling_keeps_samples_and_matches_trigonometric_interpolant():
    even, odd = pins.upsample_errors()
    assert even < 1e-13
    assert odd < 1e-12


def test_p5_spline_matches_scipy_natural_spline():
    assert pins.p5_spline_vs_scipy() < 1e-12


def test_p5_spline_reproduces_linear_data():
    assert pins.p5_spline_linear_exact() < 1e-12


def test_resampling_recovers_delayed_tone():
    # cubic-spline error on a tone at 1/100 of the sample rate, plus end ringing of the
    # band-limited interpolant, away from the ends
    assert pins.resample_tone_error() < 2e-3


def test_p2_noiseless_on_grid_injection_full_segment():
    got, cf, peak, k0 = pins.p2_closed_form(synth.N_FULL)
    assert peak == k0
    assert abs(got - cf) / cf < 1e-3
    # whole sidereal days: <ab> ~ 0, so the closed form is rho^2 = 100
    assert abs(cf - 100.0) < 0.1


def test_p2_noiseless_on_grid_injection_tiny_segment():
    got, cf, peak, k0 = pins.p2_closed_form(4096)
    assert peak == k0
    assert abs(got - cf) / cf < 2e-2


def test_p1_direct_detector_time_sum_agrees_with_resampled_fft():
    got, direct = pins.p1_direct_vs_resampled(synth.N_FULL)
    assert abs(got - direct) / direct < 1e-3
    got, direct = pins.p1_direct_vs_resampled(4096)
    assert abs(got - direct) / direct < 2e-2


def test_p3_noise_two_f_is_chi2_4dof_on_whole_sidereal_days():
    mean, var, tail, n_indep, ks_p = pins.p3_noise_stats()
    # acceptance bands at about 5 standard errors (n_indep ~ independent bins)
    assert abs(mean - 4.0) < 5 * math.sqrt(8.0 / n_indep)
    assert abs(var - 8.0) < 0.3
    p = math.exp(-10.0) * (1 + 10.0)  # P(chi2_4 > 20) = e^-10 (1 + 10)
    assert abs(tail - p) < 5 * math.sqrt(p / n_indep)
    assert ks_p > 1e-6


def test_p6_linearity_in_the_data():
    assert pins.p6_linearity() < 1e-12


def test_full_form_recovers_rho2_on_tiny_segment():
    # with the <ab> cross term the noiseless maximum is rho^2 even where C/sqrt(AB) ~ 0.9
    seg, inj, k0, nfft = pins.on_grid_injection(4096)
    sky = oracle.sky_stage(seg, inj.alpha, inj.delta, nfft)
    assert abs(sky["C"]) / math.sqrt(sky["A"] * sky["B"]) > 0.3
    full = oracle.template_two_f(seg, sky, inj.fdot, nfft, full=True)
    assert int(np.argmax(full)) == k0
    assert abs(full[k0] - 100.0) / 100.0 < 2e-2


def test_search_candidates_are_sorted_and_above_threshold():
    w = synth.workload("tiny")
    seg = w.segments[0]
    c = oracle.search(seg, w.alpha[:2], w.delta[:2], w.fdot[:2], w.threshold)
    assert c.size > 0
    assert np.all(c["twoF"] > w.threshold)
    keys = np.stack([c["segment"], c["sky"], c["fdot_idx"], c["bin"]], 1)
    assert np.all(np.diff(keys[:, 1] * 10 ** 8 + keys[:, 2] * 10 ** 6 + keys[:, 3]) > 0)
    nfft = oracle.default_nfft(seg.n)
    np.testing.assert_allclose(c["f_hz"], seg.f_off + c["bin"] / (nfft * seg.dt), rtol=0, atol=1e-12)


def test_golden_fft_lengths():
    # Sect. 2: the Fourier transform is twice as long as the data, zero-padded to a
    # power of two; the oracle and the input generator each state it
    rows = np.loadtxt(os.path.join(GOLDEN, "nfft_lengths.txt"), dtype=np.int64)
    for n, nfft in rows:
        assert oracle.default_nfft(int(n)) == nfft
        assert synth.nfft_for(int(n)) == nfft


def test_search_returns_every_crossing_of_the_bin_range():
    # every bin of [k_min, k_max) whose 2F exceeds the threshold, and no other, with the
    # bin numbered on the whole transform and its frequency f_off + bin/(nfft dt)
    w = synth.workload("tiny")
    seg = w.segments[0]
    nfft = oracle.default_nfft(seg.n)
    k_min, k_max = 1000, 3001
    c = oracle.search(seg, w.alpha[:2], w.delta[:2], w.fdot[:3], w.threshold, k_min=k_min, k_max=k_max)
    n_all = 0
    for i in range(2):
        sky = oracle.sky_stage(seg, float(w.alpha[i]), float(w.delta[i]), nfft)
        for s in range(3):
            full = oracle.template_two_f(seg, sky, float(w.fdot[s]), nfft)
            want = np.nonzero(full > w.threshold)[0]
            want = want[(want >= k_min) & (want < k_max)]
            got = c[(c["sky"] == i) & (c["fdot_idx"] == s)]
            np.testing.assert_array_equal(got["bin"], want)
            np.testing.assert_allclose(got["twoF"], full[want], rtol=1e-12, atol=0)
            np.testing.assert_allclose(got["f_hz"], seg.f_off + want / (nfft * seg.dt), rtol=0, atol=1e-12)
            assert np.all(got["fdot"] == w.fdot[s]) and np.all(got["alpha"] == w.alpha[i])
            n_all += len(want)
    assert n_all == len(c) and n_all > 0


def test_golden_band_offsets_eq1():
    # Eq. 1: f_off = 100 + (1 - 2^-5) b; the bands overlap by 2^-5 Hz (Sect. 2)
    rows = np.loadtxt(os.path.join(GOLDEN, "eq1_band_offsets.txt"))
    np.testing.assert_allclose(synth.band_offset(rows[:, 0]), rows[:, 1], rtol=0, atol=1e-12)
    assert np.allclose(np.diff(rows[:2, 1]), 1.0 - 2 ** -5)


def test_golden_segment_shape():
    # Sect. 2: two sidereal days at 0.5 s give N = 344656 samples; the ephemeris file
    # holds 3N + 2 = 1033970 doubles.  At 2 s the same span is 86164 samples.
    n_paper = int(2 * synth.SIDEREAL_DAY / 0.5)
    assert n_paper == 344656
    assert 3 * n_paper + 2 == 1033970
    assert int(2 * synth.SIDEREAL_DAY / 2.0) == synth.N_FULL
    assert synth.ephemeris(16, 2.0).shape == (3, 16)

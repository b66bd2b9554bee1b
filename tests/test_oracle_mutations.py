"""Planted mistakes in the oracle (on the CPU) must each fail at least one pin.

Each case swaps one oracle step for a plausibly wrong variant (a dropped term,
a flipped sign, a transposed or mis-indexed operand) and checks that the pin
it belongs to detects it.  This shows that the pins constrain the oracle.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.fstat_oracle as fo
import synth
from tests import pins


def _p2_ok(n=synth.N_FULL):
    got, cf, peak, k0 = pins.p2_closed_form(n)
    return peak == k0 and abs(got - cf) / cf < 1e-3


def test_pins_pass_on_unmodified_oracle():
    assert _p2_ok()
    assert pins.p0_amplitude_vs_tensor() < 1e-13


def test_flipped_fft_sign_is_caught(monkeypatch):
    monkeypatch.setattr(fo, "fourier_transform", lambda y, nfft: np.fft.ifft(y, nfft) * nfft)
    assert pins.p4_fft_vs_bruteforce() > 1e-3
    assert pins.p4_tone_peak_bin() != 37
    assert not _p2_ok()


def test_dropped_amplitude_term_is_caught(monkeypatch):
    orig = fo.amplitude_modulation

    def wrong(n, dt, alpha, delta, lat, gamma, phi_r):
        a, b = orig(n, dt, alpha, delta, lat, gamma, phi_r)
        # drop the constant term of a(t)
        return a - 0.75 * math.sin(2 * gamma) * math.cos(lat) ** 2 * math.cos(delta) ** 2, b
    monkeypatch.setattr(fo, "amplitude_modulation", wrong)
    assert pins.p0_amplitude_vs_tensor() > 1e-3


def test_swapped_amplitude_modulations_are_caught(monkeypatch):
    orig = fo.amplitude_modulation
    monkeypatch.setattr(fo, "amplitude_modulation", lambda *a: orig(*a)[::-1])
    assert pins.p0_amplitude_vs_tensor() > 1e-3


def test_wrong_sidereal_sign_is_caught(monkeypatch):
    monkeypatch.setattr(fo, "OMEGA_R", -fo.OMEGA_R)
    assert pins.p0_amplitude_vs_tensor() > 1e-3


def test_conjugated_phase_demodulation_is_caught(monkeypatch):
    def wrong(x, a, b, delay, f_off):
        e = np.exp(+2j * math.pi * f_off * delay)
        return x * a * e, x * b * e
    monkeypatch.setattr(fo, "demodulate", wrong)
    assert not _p2_ok()


def test_wrong_resampling_direction_is_caught(monkeypatch):
    orig = fo.resample
    monkeypatch.setattr(fo, "resample", lambda z, d, dt, nfft: orig(z, -d, dt, nfft))
    assert not _p2_ok()
    assert pins.resample_tone_error() > 1e-2


def test_flipped_spindown_sign_is_caught(monkeypatch):
    orig = fo.spindown_demodulate
    monkeypatch.setattr(fo, "spindown_demodulate", lambda zt, fdot, dt: orig(zt, -fdot, dt))
    assert not _p2_ok()


def test_non_natural_spline_end_is_caught(monkeypatch):
    orig = fo.natural_spline_moments

    def wrong(u):
        m = orig(u)
        m[0] = m[1]       # "not-a-knot"-like end instead of zero curvature
        return m
    monkeypatch.setattr(fo, "natural_spline_moments", wrong)
    assert pins.p5_spline_vs_scipy() > 1e-6


def test_off_by_one_spline_interval_is_caught(monkeypatch):
    orig = fo.natural_spline_eval

    def wrong(u, m, pos):
        return orig(u, np.roll(m, 1), pos)
    monkeypatch.setattr(fo, "natural_spline_eval", wrong)
    assert pins.p5_spline_vs_scipy() > 1e-6


def test_lost_nyquist_half_in_upsampling_is_caught(monkeypatch):
    def wrong(z, nfft):
        m = nfft // 2
        zz = np.fft.fft(z, m)
        u = np.zeros(nfft, dtype=complex)
        u[: m // 2] = zz[: m // 2]
        u[nfft - m // 2:] = zz[m // 2:]
        u[nfft - m // 2] = 0.0     # Nyquist term dropped
        return 2.0 * np.fft.ifft(u)
    monkeypatch.setattr(fo, "fft_upsample2", wrong)
    even, odd = pins.upsample_errors()
    assert max(even, odd) > 1e-6


def test_wrong_normalisation_is_caught(monkeypatch):
    orig = fo.two_f
    monkeypatch.setattr(fo, "two_f", lambda fa, fb, A, B, n, s2: orig(fa, fb, A, B, n, s2) * n / (n + 4096))
    mean, var, tail, n_indep, ks_p = pins.p3_noise_stats(realisations=2)
    assert abs(mean - 4.0) > 5 * math.sqrt(8.0 / n_indep)


def test_swapped_a_b_averages_are_caught(monkeypatch):
    orig = fo.antenna_averages
    monkeypatch.setattr(fo, "antenna_averages", lambda a, b: (lambda A, B, C: (B, A, C))(*orig(a, b)))
    assert not _p2_ok()


def _ib_variant(diff):
    def wrong(y, nfft):
        half = nfft // 2
        x = np.fft.fft(y, half)
        c = fo.interbin_weight(y.shape[0], half)
        out = np.empty(nfft, dtype=np.complex128)
        out[0::2] = x
        out[1::2] = c * diff(x)
        return out
    return wrong


def test_interbinning_with_a_sum_is_caught(monkeypatch):
    monkeypatch.setattr(fo, "interbinned_transform", _ib_variant(lambda x: x + np.roll(x, -1)))
    assert pins.ib_midway_error() > 0.5
    assert pins.ib_direct_sum_error() > 1e-3


def test_interbinning_with_the_lower_neighbour_is_caught(monkeypatch):
    monkeypatch.setattr(fo, "interbinned_transform", _ib_variant(lambda x: x - np.roll(x, 1)))
    assert pins.ib_midway_error() > 0.1
    assert pins.ib_direct_sum_error() > 1e-3


def test_interbinning_without_the_wrap_is_caught(monkeypatch):
    def no_wrap(x):
        d = x - np.roll(x, -1)
        d[-1] = x[-1]
        return d
    monkeypatch.setattr(fo, "interbinned_transform", _ib_variant(no_wrap))
    assert pins.ib_direct_sum_error() > 1e-3


def test_interbinning_weight_of_one_is_caught(monkeypatch):
    monkeypatch.setattr(fo, "interbin_weight", lambda n, length: 1.0)
    assert pins.ib_midway_error() > 0.1
    assert pins.ib_weight_error() > 0.1


def test_interbinning_weight_for_the_full_length_is_caught(monkeypatch):
    # the classic pi/4 used although the data fill only part of the transform
    monkeypatch.setattr(fo, "interbin_weight", lambda n, length: math.pi / 4)
    assert pins.ib_midway_error() > 0.05


# ---- lattice grid -------------------------------------------------------------------------
def _lattice_injection_ok():
    r = pins.lattice_injection()
    if r is None:
        return False
    got, no_shift, neg_shift, cf, peak, k0 = r
    return peak == k0 and abs(got - cf) / cf < 1e-3


def test_lattice_pins_pass_on_unmodified_oracle():
    assert _lattice_injection_ok()
    assert pins.lattice_doppler_amplitude_error() < 1e-6


def test_obliquity_rotated_the_wrong_way_is_caught(monkeypatch):
    orig = fo.ecliptic_to_equatorial
    monkeypatch.setattr(fo, "ecliptic_to_equatorial", lambda x, y, z, eps: orig(x, y, z, -eps))
    assert pins.lattice_doppler_amplitude_error() > 1e-3


def test_swapped_sky_coordinates_are_caught(monkeypatch):
    orig = fo.lattice_sky_position

    def wrong(M, n, m, h, eps, f_ref):
        M2 = M.copy()
        M2[:, [2, 3]] = M[:, [3, 2]]
        return orig(M2, n, m, h, eps, f_ref)
    monkeypatch.setattr(fo, "lattice_sky_position", wrong)
    assert pins.lattice_doppler_amplitude_error() > 1e-3


def test_dropped_frequency_shift_is_caught(monkeypatch):
    orig = fo.lattice_template
    monkeypatch.setattr(fo, "lattice_template", lambda *a: (orig(*a)[0], 0.0))
    assert not _lattice_injection_ok()


def test_frequency_shift_of_the_wrong_sign_is_caught(monkeypatch):
    orig = fo.lattice_demodulate
    monkeypatch.setattr(fo, "lattice_demodulate", lambda zt, w1, u, nfft: orig(zt, w1, -u, nfft))
    assert not _lattice_injection_ok()


def test_spindown_coefficient_off_by_two_is_caught(monkeypatch):
    orig = fo.lattice_demodulate
    monkeypatch.setattr(fo, "lattice_demodulate", lambda zt, w1, u, nfft: orig(zt, 2.0 * w1, u, nfft))
    assert not _lattice_injection_ok()


def test_sky_offset_of_the_spindown_dropped_is_caught(monkeypatch):
    orig = fo.lattice_template
    monkeypatch.setattr(fo, "lattice_template", lambda M, s, w0, w1, nfft: orig(M, s, w0, 0.0, nfft))
    assert not _lattice_injection_ok()


def test_swapped_jks_amplitudes_in_vetting_data_are_caught(monkeypatch):
    from oracle import vet_data
    orig = vet_data.jks_amplitudes
    monkeypatch.setattr(vet_data, "jks_amplitudes", lambda *a: orig(*a)[[0, 2, 1, 3]])
    assert pins.vet_signal_assembly_error(31) > 1e-3


def test_basis_order_slip_in_vetting_data_is_caught(monkeypatch):
    orig = synth.cw_basis
    monkeypatch.setattr(synth, "cw_basis", lambda *a, **k: orig(*a, **k)[[0, 1, 3, 2]])
    assert pins.vet_signal_assembly_error(32) > 1e-3

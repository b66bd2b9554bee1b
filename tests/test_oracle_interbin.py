"""Pins of the oracle's interbinned transform (nfft/2-point transform, odd bins from
their neighbours) against facts fixed outside it: the zero-padded transform it must
reproduce on even bins, the exact value of a sinusoid midway between two bins, the
classic interbinning weight at full length, direct sums at the wrap-around bin, and
the variance of interbinned white noise in closed form."""
import math

import numpy as np

from oracle import fstat_oracle as fo
from tests import pins


def _rng(seed):
    return np.random.default_rng(seed)


def test_even_bins_equal_the_zero_padded_transform():
    # bins 2k of an nfft-point zero-padded transform are bins k of the nfft/2-point one
    n, nfft = 3000, 8192
    g = _rng(11)
    y = g.standard_normal(n) + 1j * g.standard_normal(n)
    ib = fo.interbinned_transform(y, nfft)
    zp = np.fft.fft(y, nfft)
    np.testing.assert_allclose(ib[0::2], zp[0::2], rtol=0, atol=1e-9 * np.abs(zp).max())


def test_midway_sinusoid_is_exact():
    # a unit sinusoid at frequency k0 + 1/2 (in bins of nfft/2) sums to n at that
    # frequency; the interbinned odd bin 2 k0 + 1 must have that modulus
    for n, nfft, k0 in ((3000, 8192, 517), (86164, 1 << 18, 20011), (4096, 8192, 3)):
        half = nfft // 2
        j = np.arange(n)
        y = 0.3 * np.exp(1j * 0.7) * np.exp(2j * math.pi * (k0 + 0.5) * j / half)
        ib = fo.interbinned_transform(y, nfft)
        assert abs(abs(ib[2 * k0 + 1]) - 0.3 * n) < 1e-9 * n, (n, nfft)
        # and the zero-padded transform agrees there (its bin 2 k0 + 1 is that frequency)
        zp = np.fft.fft(y, nfft)[2 * k0 + 1]
        assert abs(abs(zp) - 0.3 * n) < 1e-9 * n


def test_full_length_weight_is_the_classic_pi_over_4():
    # with no zero-padding (n = nfft/2) interbinning uses pi/4 (Ransom et al. 2002)
    for half in (4096, 1 << 15):
        assert abs(fo.interbin_weight(half, half) - math.pi / 4) < 2e-7
    # and the zero-padded weight follows pi r / (2 (1 - cos pi r)), r = n / (nfft/2)
    n, half = 86164, 1 << 17
    r = n / half
    assert abs(fo.interbin_weight(n, half) - math.pi * r / (2 * (1 - math.cos(math.pi * r)))) < 1e-5


def test_wrap_around_bin_uses_bins_last_and_zero():
    # the last odd bin nfft - 1 lies between bins nfft/2 - 1 and 0 (periodic transform)
    n, nfft = 500, 2048
    half = nfft // 2
    g = _rng(12)
    y = g.standard_normal(n) + 1j * g.standard_normal(n)
    j = np.arange(n)
    x_last = np.sum(y * np.exp(-2j * math.pi * j * (half - 1) / half))
    x_0 = np.sum(y)
    c = fo.interbin_weight(n, half)
    ib = fo.interbinned_transform(y, nfft)
    assert abs(ib[nfft - 1] - c * (x_last - x_0)) < 1e-9 * abs(x_0)
    # an interior odd bin the same way, by direct sums
    k = 300
    xk = np.sum(y * np.exp(-2j * math.pi * j * k / half))
    xk1 = np.sum(y * np.exp(-2j * math.pi * j * (k + 1) / half))
    assert abs(ib[2 * k + 1] - c * (xk - xk1)) < 1e-9 * abs(xk)


def test_noise_variance_of_odd_bins_matches_closed_form():
    # white noise of unit variance per sample: E|X_k|^2 = n on even bins and
    # c^2 (2 n - 2 Re sum_j exp(2 pi i j / half)) on odd bins
    n, nfft = 2600, 8192
    half = nfft // 2
    g = _rng(13)
    even, odd = [], []
    for _ in range(40):
        y = (g.standard_normal(n) + 1j * g.standard_normal(n)) / math.sqrt(2)
        ib = fo.interbinned_transform(y, nfft)
        even.append(np.mean(np.abs(ib[0::2]) ** 2))
        odd.append(np.mean(np.abs(ib[1::2]) ** 2))
    c = fo.interbin_weight(n, half)
    # Re sum_{j<n} e^{2 pi i j/half} = sin(pi n/half) cos(pi (n-1)/half) / sin(pi/half)
    rho = math.sin(math.pi * n / half) * math.cos(math.pi * (n - 1) / half) / math.sin(math.pi / half)
    want_odd = c * c * (2 * n - 2 * rho)
    assert abs(np.mean(even) / n - 1) < 0.01
    assert abs(np.mean(odd) / want_odd - 1) < 0.01


def test_template_function_uses_the_interbinned_transform():
    # 2F of a template from hand-built demodulated series equals the definition
    n, nfft, dt = 3000, 8192, 2.0
    g = _rng(14)
    za = g.standard_normal(n) + 1j * g.standard_normal(n)
    zb = g.standard_normal(n) + 1j * g.standard_normal(n)

    class Seg:
        pass
    seg = Seg()
    seg.n, seg.dt, seg.sigma2 = n, dt, 1.7
    sky = {"za_t": za, "zb_t": zb, "A": 0.31, "B": 0.22, "C": 0.05}
    fdot = -3.1e-9
    ya = fo.spindown_demodulate(za, fdot, dt)
    yb = fo.spindown_demodulate(zb, fdot, dt)
    fa = fo.interbinned_transform(ya, nfft)[100:900]
    fb = fo.interbinned_transform(yb, nfft)[100:900]
    want = 2.0 / (n * seg.sigma2) * (np.abs(fa) ** 2 / 0.31 + np.abs(fb) ** 2 / 0.22)
    got = fo.template_two_f_interbin(seg, sky, fdot, nfft, 100, 900)
    np.testing.assert_allclose(got, want, rtol=1e-12)
    # even bins agree with the zero-padded template (same transform values)
    zp = fo.template_two_f(seg, sky, fdot, nfft, 100, 900)
    np.testing.assert_allclose(got[0::2], zp[0::2], rtol=1e-9)


def test_pin_helpers_hold():
    assert pins.ib_midway_error() < 1e-12
    assert pins.ib_direct_sum_error() < 1e-10
    assert pins.ib_weight_error() < 2e-7

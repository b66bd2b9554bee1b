"""Pins of the oracle's lattice grid: the sky loop over the integers (n, m) of the grid
generating matrix, the spindown integers s, and the frequency shift that reconciles
the grid's frequencies with the Fourier bins (Sect. 2; Sect. 1.1)."""
import math

import numpy as np
import pytest

import synth
from oracle import fstat_oracle as fo
from tests import pins

EPS = synth.OBLIQUITY


def test_light_travel_time_of_one_au():
    # 1 AU = 149 597 870 700 m exactly, c = 299 792 458 m/s exactly: 499.004784 s
    assert abs(fo.AU_SECONDS - 499.00478384) < 1e-8


def _axes_lattice(f_ref=100.25):
    # sky rows W e_x, W e_y (W itself is pinned by the two tests around this one)
    w = fo.lattice_sky_scale(f_ref)
    M = np.zeros((4, 4))
    M[0, 0] = 2 * math.pi / 8192
    M[2, 2] = w
    M[3, 3] = w
    return M, f_ref


@pytest.mark.parametrize("nm,h,expect", [
    ((0, 0), +1, (1.5 * math.pi, 0.5 * math.pi - EPS)),   # north ecliptic pole: 18h, +66.56 deg
    ((0, 0), -1, (0.5 * math.pi, -(0.5 * math.pi - EPS))),  # south ecliptic pole: 6h, -66.56 deg
    ((1, 0), +1, (0.0, 0.0)),                                 # vernal equinox
    ((-1, 0), -1, (math.pi, 0.0)),                            # autumnal equinox
    ((0, 1), +1, (0.5 * math.pi, EPS)),                       # summer solstice point
    ((0, -1), -1, (1.5 * math.pi, -EPS)),                     # winter solstice point
])
def test_ecliptic_landmarks(nm, h, expect):
    M, f_ref = _axes_lattice()
    a, d = fo.lattice_sky_position(M, nm[0], nm[1], h, EPS, f_ref)
    assert abs(d - expect[1]) < 1e-12
    da = (a - expect[0] + math.pi) % (2 * math.pi) - math.pi
    assert abs(da) < 1e-12
    assert 0.0 <= a < 2 * math.pi


def test_points_off_the_sky_are_skipped():
    M, f_ref = _axes_lattice()
    assert fo.lattice_sky_position(M, 1, 1, +1, EPS, f_ref) is None
    assert fo.lattice_sky_position(M, 0, 2, -1, EPS, f_ref) is None


def test_sky_coordinates_are_the_annual_doppler_amplitudes():
    assert pins.lattice_doppler_amplitude_error() < 1e-6


def test_sky_points_return_to_their_integers():
    """Ecliptic coordinates from (alpha, delta) by the textbook formulas, then the sky rows
    inverted: the integers (n, m) and the hemisphere come back."""
    nfft, f_ref, M, _ = pins.lattice_setup(4096, sky_points=60, seed=8)
    w = 2.0 * math.pi * f_ref * synth.AU_LS
    box = fo.lattice_sky_range(M, f_ref)
    S = np.array([[M[2, 2], M[2, 3]], [M[3, 2], M[3, 3]]])
    count = 0
    for h in (+1, -1):
        for n, m, alpha, delta, w0, w1 in fo.lattice_sky_points(M, box, h, EPS, f_ref):
            sin_b = math.sin(delta) * math.cos(EPS) - math.cos(delta) * math.sin(EPS) * math.sin(alpha)
            x_e = math.cos(delta) * math.cos(alpha)
            y_e = math.sin(delta) * math.sin(EPS) + math.cos(delta) * math.cos(EPS) * math.sin(alpha)
            nm = np.linalg.solve(S.T, np.array([x_e, y_e]) * w)
            assert np.max(np.abs(nm - [n, m])) < 1e-7
            assert sin_b * h >= -1e-12
            assert w0 == n * M[2, 0] + m * M[3, 0] and w1 == n * M[2, 1] + m * M[3, 1]
            count += 1
    assert 100 < count < 140


def test_range_holds_every_sky_point():
    _, f_ref, M, _ = pins.lattice_setup(4096, sky_points=50, seed=9)
    n_lo, n_hi, m_lo, m_hi = fo.lattice_sky_range(M, f_ref)
    big = (3 * n_lo - 2, 3 * n_hi + 2, 3 * m_lo - 2, 3 * m_hi + 2)
    pts = fo.lattice_sky_points(M, big, +1, EPS, f_ref)
    assert len(pts) > 30
    assert all(n_lo <= p[0] <= n_hi and m_lo <= p[1] <= m_hi for p in pts)
    inner = fo.lattice_sky_points(M, (n_lo, n_hi, m_lo, m_hi), +1, EPS, f_ref)
    assert [p[:2] for p in inner] == [p[:2] for p in pts]


def test_frequency_shift_definition():
    M = np.zeros((4, 4))
    b = 2 * math.pi / 1024
    M[1, 0] = 0.25 * b
    # s = 2: w0 = 0.5 bin; s = 4: a whole bin (on a bin, u = 0); s = -1: -0.25 bin -> 0.75
    assert abs(fo.lattice_template(M, 2, 0.0, 0.0, 1024)[1] - 0.5) < 1e-12
    assert abs(fo.lattice_template(M, 4, 0.0, 0.0, 1024)[1]) < 1e-9
    assert abs(fo.lattice_template(M, -1, 0.0, 0.0, 1024)[1] - 0.75) < 1e-12
    assert abs(fo.lattice_template(M, 0, 3.3 * b, 0.0, 1024)[1] - 0.3) < 1e-9


def test_injection_at_a_shifted_grid_point_is_recovered():
    """A source exactly at a lattice point (frequency a fraction of a bin above the Fourier
    bins, spindown with its sky offset) gives the closed-form 2F at its bin only when the
    shift is applied with the right sign."""
    got, no_shift, neg_shift, cf, peak, k0 = pins.lattice_injection()
    assert peak == k0
    assert abs(got - cf) / cf < 1e-3
    assert no_shift < 0.97 * cf and neg_shift < 0.97 * cf


def test_lattice_without_offsets_matches_the_plain_search():
    n = 4096
    nfft = fo.default_nfft(n)
    M = np.zeros((4, 4))
    M[0, 0] = 2 * math.pi / nfft
    M[1, 1] = math.pi * -2.5e-10 * 4.0
    f_ref = 100.25
    w = 2.0 * math.pi * f_ref * synth.AU_LS
    M[2, 2], M[2, 3] = 0.4 * w, 0.1 * w
    M[3, 2], M[3, 3] = -0.1 * w, 0.45 * w
    pts = fo.lattice_sky_points(M, fo.lattice_sky_range(M, f_ref), -1, EPS, f_ref)[:3]
    seg = synth.make_segment(n, 2.0, 100.0, 1.0, 123, [])
    a = fo.search_lattice(seg, M, pts, -2, 1, 6.0)
    fdot = np.array([s * M[1, 1] / (math.pi * 4.0) for s in range(-2, 2)])
    b = fo.search(seg, [p[2] for p in pts], [p[3] for p in pts], fdot, 6.0)
    assert len(a) == len(b) > 10
    for key in ("sky", "fdot_idx", "bin"):
        assert np.array_equal(a[key], b[key])
    assert np.allclose(a["twoF"], b["twoF"], rtol=1e-9)
    assert np.allclose(a["fdot"], b["fdot"], rtol=1e-12, atol=0)
    assert np.array_equal(a["f_hz"], b["f_hz"])


def test_synthetic_sky_lattice_covering_radius():
    """The synthetic generator's sky rows form a hexagonal lattice of spacing h, whose
    covering radius is h / sqrt(3): every point of the sky's disk lies within it of a
    lattice point (brute force over random points), and the bound is nearly reached."""
    nfft, f_ref, M, _ = pins.lattice_setup(4096, sky_points=200, seed=12)
    w = fo.lattice_sky_scale(f_ref)
    e1, e2 = M[2, 2:], M[3, 2:]
    h = float(np.hypot(*e1))
    assert abs(float(np.hypot(*e2)) - h) < 1e-9 * h and abs(float(e1 @ e2) - 0.5 * h * h) < 1e-9 * h * h
    rng = np.random.default_rng(3)
    r = w * np.sqrt(rng.uniform(0, 1, 4000))
    t = rng.uniform(0, 2 * math.pi, 4000)
    pts = np.stack([r * np.cos(t), r * np.sin(t)], 1)
    S = np.array([e1, e2])
    nm = np.linalg.solve(S.T, pts.T).T
    best = np.full(len(pts), np.inf)
    for dn in (-1, 0, 1, 2):
        for dm in (-1, 0, 1, 2):
            cand = (np.floor(nm) + [dn, dm]) @ S
            best = np.minimum(best, np.hypot(*(pts - cand).T))
    assert best.max() <= h / math.sqrt(3) * (1 + 1e-9)
    assert best.max() > 0.9 * h / math.sqrt(3)

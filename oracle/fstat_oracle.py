"""Plain FP64 reference of the F-statistic search path (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  The GPU library never calls it and it never calls the
GPU library.

The steps follow the paper's flow for one band and frame (Sect. 2, Fig. 3):
for each sky position, recover the direction, compute the two amplitude
modulations and the phase modulation, demodulate, resample with the FFT and
splines; then for each spindown, demodulate the spindown, Fourier-transform
both amplitude-demodulated series with 2x Fourier interpolation, form the
F-statistic on every bin and register bins above the threshold as candidates
of five numbers (sky position, frequency, spindown, F).

The paper defers every formula to its references (Sect. 1.1), so each step
below states the reading it uses:

* sky direction n = (cos d cos a, cos d sin a, sin d); Roemer delay
  D_i = n.(r_i - r_0) from the detector-to-SSB ephemeris (Sect. 2);
* amplitude modulations a(t), b(t): the closed forms of Jaranowski, Krolak &
  Schutz (1998) for a right-angle interferometer at latitude lat, arm
  bisector at gamma counter-clockwise from East, local sidereal angle
  phi_r + Omega_r t;
* phase demodulation by exp(-i 2 pi f_off D_i);
* resampling "with the FFT and splines" (Sect. 2) read as: 2x band-limited
  upsampling by spectral zero-padding of a length nfft/2 DFT, then a natural
  cubic spline through the upsampled points evaluated at the detector times
  of a uniform barycentric grid, s_j = j - D_j/dt (first-order inverse of
  tau = t + D), zero outside the data;
* spindown demodulation exp(-i pi fdot (j dt)^2), reference time at the
  segment start;
* "Fourier transform twice as long" (Sect. 2) read as zero-padding of the N
  samples to nfft = the smallest power of two >= 2N;
* 2F_k = 2/(N sigma^2) (|Fa_k|^2/A + |Fb_k|^2/B), A = <a^2>, B = <b^2>
  (simplified form, the cross term <ab> dropped); the full form with <ab> is
  provided as well;
* candidates: every bin with 2F strictly above the threshold.

Interbinning (an alternative to the 2x zero-padding, not the paper's own
step): the transform is taken over nfft/2 points only; even bins 2k of the
fine grid are its bins k exactly, odd bins 2k+1 are estimated from the two
neighbours as c (X_k - X_{k+1}), with c chosen so that a sinusoid midway
between two bins, over the N nonzero samples, comes out exactly (at N = nfft/2
this is the classic interbinning weight, about pi/4).

Lattice grid (Sect. 2: the grid generating matrix and the integers n, m, s;
Sect. 1.1: grid points reconciled with the Fourier frequencies, resampling once
per sky position), read as follows.  Grid points are the integer combinations
k M0 + s M1 + n M2 + m M3 of the rows of a 4x4 matrix M over the phase
parameters (w0, w1, w2, w3): w0 = 2 pi f dt (frequency above f_off, radians per
sample), w1 = pi fdot dt^2 (spindown phase w1 j^2 at sample j), and
(w2, w3) = W (x_e, y_e), the source direction's two components in the ecliptic
plane (x_e toward the vernal equinox) scaled by W = 2 pi f_ref (1 AU / c).
Row 0 is the frequency vector (along w0 only, a whole number of Fourier bins),
row 1 the spindown vector (no sky components), rows 2 and 3 the sky vectors.
The third ecliptic component is +-sqrt(1 - x_e^2 - y_e^2) (one hemisphere per
sign); the obliquity rotates ecliptic axes to equatorial ones.  For every
(s, n, m) the FFT evaluates the frequencies w0(s, n, m) + 2 pi k / nfft: the
series is demodulated by the template's spindown phase and by the fraction u of
a bin that the grid's frequencies lie above the Fourier bins, and bin k of the
transform is the frequency f_off + (k + u) / (nfft dt).

Every floating-point step is FP64.  numpy's FFT and scipy's banded solver are
used as library primitives.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

SIDEREAL_DAY = 86164.0905                  # s
OMEGA_R = 2.0 * math.pi / SIDEREAL_DAY     # Earth rotation rate, rad/s


def next_pow2_at_least(v: int) -> int:
    m = 1
    while m < v:
        m *= 2
    return m


def default_nfft(n: int) -> int:
    """Length of the 2x interpolated Fourier transform (Sect. 2): nextpow2(2N)."""
    return next_pow2_at_least(2 * n)


# ---------------------------------------------------------------- sky stage
def sky_direction(alpha: float, delta: float) -> np.ndarray:
    """Unit vector towards equatorial (alpha, delta) (Sect. 2: sky position recovered)."""
    return np.array([math.cos(delta) * math.cos(alpha),
                     math.cos(delta) * math.sin(alpha),
                     math.sin(delta)])


def roemer_delay(r: np.ndarray, nhat: np.ndarray) -> np.ndarray:
    """Phase modulation delay D_i = n.(r_i - r_0) in seconds (Sect. 2, ephemeris file)."""
    nr = nhat[0] * r[0] + nhat[1] * r[1] + nhat[2] * r[2]
    return nr - nr[0]


def amplitude_modulation(n: int, dt: float, alpha: float, delta: float,
                         lat: float, gamma: float, phi_r: float):
    """The two amplitude modulations a(t), b(t) (Sect. 2; JKS 1998 closed forms)."""
    t = np.arange(n, dtype=np.float64) * dt
    x = alpha - phi_r - OMEGA_R * t
    s2g, c2g = math.sin(2 * gamma), math.cos(2 * gamma)
    sl, cl = math.sin(lat), math.cos(lat)
    s2l, c2l = math.sin(2 * lat), math.cos(2 * lat)
    sd, cd = math.sin(delta), math.cos(delta)
    s2d, c2d = math.sin(2 * delta), math.cos(2 * delta)
    a = (s2g * (3 - c2l) * (3 - c2d) * np.cos(2 * x) / 16.0
         - c2g * sl * (3 - c2d) * np.sin(2 * x) / 4.0
         + s2g * s2l * s2d * np.cos(x) / 4.0
         - c2g * cl * s2d * np.sin(x) / 2.0
         + 0.75 * s2g * cl * cl * cd * cd)
    b = (c2g * sl * sd * np.cos(2 * x)
         + s2g * (3 - c2l) * sd * np.sin(2 * x) / 4.0
         + c2g * cl * cd * np.cos(x)
         + s2g * s2l * cd * np.sin(x) / 2.0)
    return a, b


def antenna_averages(a: np.ndarray, b: np.ndarray):
    """A = <a^2>, B = <b^2>, C = <ab>, means over the N detector samples."""
    n = a.shape[0]
    return float(np.dot(a, a) / n), float(np.dot(b, b) / n), float(np.dot(a, b) / n)


def demodulate(x: np.ndarray, a: np.ndarray, b: np.ndarray, delay: np.ndarray, f_off: float):
    """Amplitude and phase demodulation (Sect. 2, Fig. 3):
    za = x a exp(-i psi), zb = x b exp(-i psi), psi = 2 pi f_off D reduced mod 2 pi."""
    cyc = f_off * delay
    cyc = cyc - np.floor(cyc)
    e = np.exp(-2j * math.pi * cyc)
    return x * a * e, x * b * e


def fft_upsample2(z: np.ndarray, nfft: int) -> np.ndarray:
    """Band-limited 2x upsampling by spectral zero-padding (the FFT part of the resampling).

    M = nfft/2; Z = DFT_M(z zero-padded to M); U of length nfft holds Z[0:M/2) at
    the start and Z[M/2:M) at the end (the Nyquist term whole on the negative
    side); u = 2 IDFT_nfft(U) so that u[2i] = z[i].
    """
    m = nfft // 2
    if z.shape[0] > m:
        raise ValueError("segment longer than nfft/2")
    zz = np.fft.fft(z, m)
    u_spec = np.zeros(nfft, dtype=np.complex128)
    u_spec[: m // 2] = zz[: m // 2]
    u_spec[nfft - m + m // 2:] = zz[m // 2:]
    return 2.0 * np.fft.ifft(u_spec)


def natural_spline_moments(u: np.ndarray) -> np.ndarray:
    """Second derivatives of the natural cubic spline through (p, u_p), unit spacing.

    m_0 = m_{L-1} = 0 and m_{p-1} + 4 m_p + m_{p+1} = 6 (u_{p+1} - 2 u_p + u_{p-1}).
    """
    L = u.shape[0]
    m = np.zeros(L, dtype=u.dtype)
    if L <= 2:
        return m
    rhs = 6.0 * (u[2:] - 2.0 * u[1:-1] + u[:-2])
    k = L - 2
    ab = np.empty((3, k))
    ab[0, :] = 1.0
    ab[1, :] = 4.0
    ab[2, :] = 1.0
    m[1:-1] = scipy.linalg.solve_banded((1, 1), ab, rhs)
    return m


def natural_spline_eval(u: np.ndarray, m: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """Evaluate the spline (knots at 0..L-1, moments m) at positions inside [0, L-1]."""
    L = u.shape[0]
    p = np.clip(np.floor(pos).astype(np.int64), 0, L - 2)
    t = pos - p
    w = 1.0 - t
    return (w * u[p] + t * u[p + 1]
            + ((w ** 3 - w) * m[p] + (t ** 3 - t) * m[p + 1]) / 6.0)


def resample(z: np.ndarray, delay: np.ndarray, dt: float, nfft: int) -> np.ndarray:
    """Resampling onto the uniform barycentric grid tau_j = j dt (Sect. 2: FFT and splines).

    The value at tau_j is read at the detector sample position s_j = j - D_j/dt,
    i.e. at 2 s_j on the 2x upsampled grid; zero where s_j is outside [0, N-1].
    """
    n = z.shape[0]
    u = fft_upsample2(z, nfft)
    mom = natural_spline_moments(u)
    s = np.arange(n, dtype=np.float64) - delay / dt
    inside = (s >= 0.0) & (s <= n - 1)
    out = np.zeros(n, dtype=np.complex128)
    out[inside] = natural_spline_eval(u, mom, 2.0 * s[inside])
    return out


def sky_stage(seg, alpha: float, delta: float, nfft: int):
    """Everything done once per sky position (Sect. 2: reused in the spindown loop)."""
    nhat = sky_direction(alpha, delta)
    delay = roemer_delay(seg.r, nhat)
    a, b = amplitude_modulation(seg.n, seg.dt, alpha, delta, seg.lat, seg.gamma, seg.phi_r)
    A, B, C = antenna_averages(a, b)
    za, zb = demodulate(seg.x, a, b, delay, seg.f_off)
    return {
        "delay": delay, "a": a, "b": b, "A": A, "B": B, "C": C, "za": za, "zb": zb,
        "za_t": resample(za, delay, seg.dt, nfft),
        "zb_t": resample(zb, delay, seg.dt, nfft),
    }


# ----------------------------------------------------------- spindown stage
def spindown_demodulate(zt: np.ndarray, fdot: float, dt: float) -> np.ndarray:
    """Spindown demodulation (Sect. 2, inner loop): multiply by exp(-i pi fdot (j dt)^2)."""
    t = np.arange(zt.shape[0], dtype=np.float64) * dt
    cyc = 0.5 * fdot * t * t
    cyc = cyc - np.floor(cyc)
    return zt * np.exp(-2j * math.pi * cyc)


def fourier_transform(y: np.ndarray, nfft: int) -> np.ndarray:
    """F_k = sum_{j<N} y_j exp(-2 pi i j k / nfft): the FFT with 2x interpolation (Sect. 2)."""
    return np.fft.fft(y, nfft)


def two_f(fa: np.ndarray, fb: np.ndarray, A: float, B: float, n: int, sigma2: float) -> np.ndarray:
    """2F = 2/(N sigma^2) (|Fa|^2/A + |Fb|^2/B) (simplified F-statistic, <ab> dropped)."""
    return (2.0 / (n * sigma2)) * ((fa.real ** 2 + fa.imag ** 2) / A
                                   + (fb.real ** 2 + fb.imag ** 2) / B)


def two_f_full(fa, fb, A, B, C, n, sigma2):
    """2F with the cross term: 2/(N sigma^2) (B|Fa|^2 + A|Fb|^2 - 2C Re(Fa conj Fb)) / (AB - C^2)."""
    num = (B * np.abs(fa) ** 2 + A * np.abs(fb) ** 2 - 2.0 * C * (fa * np.conj(fb)).real)
    return (2.0 / (n * sigma2)) * num / (A * B - C * C)


def template_two_f(seg, sky, fdot: float, nfft: int, k_min: int = 0, k_max: int = -1,
                   full: bool = False) -> np.ndarray:
    """2F over bins [k_min, k_max) for one (sky, spindown) template."""
    if k_max < 0:
        k_max = nfft // 2
    fa = fourier_transform(spindown_demodulate(sky["za_t"], fdot, seg.dt), nfft)[k_min:k_max]
    fb = fourier_transform(spindown_demodulate(sky["zb_t"], fdot, seg.dt), nfft)[k_min:k_max]
    if full:
        return two_f_full(fa, fb, sky["A"], sky["B"], sky["C"], seg.n, seg.sigma2)
    return two_f(fa, fb, sky["A"], sky["B"], seg.n, seg.sigma2)


def interbin_weight(n: int, length: int) -> float:
    """Interbinning weight c for a length-`length` transform of n nonzero samples.

    Take the sinusoid y_j = exp(i pi j / length), j < n, midway between bins 0 and
    1; X_0 and X_1 are its transform values at those bins (summed directly) and its
    exact value halfway is n, so c = n / |X_0 - X_1|.
    """
    j = np.arange(n, dtype=np.float64)
    y = np.exp(1j * math.pi * j / length)
    x0 = np.sum(y)
    x1 = np.sum(y * np.exp(-2j * math.pi * j / length))
    return float(n / abs(x0 - x1))


def interbinned_transform(y: np.ndarray, nfft: int) -> np.ndarray:
    """All nfft bins of the interpolated transform from a transform of nfft/2 points.

    Even bins 2k: X_k of the nfft/2-point transform (the zero-padded values exactly);
    odd bins 2k+1: c (X_k - X_{k+1}), the index taken modulo nfft/2.
    """
    half = nfft // 2
    x = fourier_transform(y, half)
    c = interbin_weight(y.shape[0], half)
    out = np.empty(nfft, dtype=np.complex128)
    out[0::2] = x
    out[1::2] = c * (x - np.roll(x, -1))
    return out


def template_two_f_interbin(seg, sky, fdot: float, nfft: int, k_min: int = 0, k_max: int = -1,
                            full: bool = False) -> np.ndarray:
    """2F over bins [k_min, k_max) of the nfft grid, with the interbinned transform."""
    if k_max < 0:
        k_max = nfft // 2
    fa = interbinned_transform(spindown_demodulate(sky["za_t"], fdot, seg.dt), nfft)[k_min:k_max]
    fb = interbinned_transform(spindown_demodulate(sky["zb_t"], fdot, seg.dt), nfft)[k_min:k_max]
    if full:
        return two_f_full(fa, fb, sky["A"], sky["B"], sky["C"], seg.n, seg.sigma2)
    return two_f(fa, fb, sky["A"], sky["B"], seg.n, seg.sigma2)


# -------------------------------------------------------------- lattice grid
AU_SECONDS = 149597870700.0 / 299792458.0   # light travel time over one astronomical unit, s
SHIFT_SNAP = 1e-6                           # a grid frequency within this many bins below a bin is on it


def lattice_sky_scale(f_ref: float) -> float:
    """W = 2 pi f_ref (1 AU / c): radius, in the sky coordinates (w2, w3), of the whole sky."""
    return 2.0 * math.pi * f_ref * AU_SECONDS


def ecliptic_to_equatorial(xe: float, ye: float, ze: float, eps: float):
    """Rotation by the obliquity about the vernal-equinox axis, ecliptic to equatorial axes."""
    ce, se = math.cos(eps), math.sin(eps)
    return xe, ce * ye - se * ze, se * ye + ce * ze


def lattice_sky_position(M: np.ndarray, n: int, m: int, hemisphere: int, eps: float, f_ref: float):
    """Sky loop, 'sky position recovered' (Sect. 2): integers (n, m) to (alpha, delta),
    or None when the point (w2, w3) = n M2 + m M3 lies outside the sky's disk."""
    w = lattice_sky_scale(f_ref)
    w2 = n * float(M[2, 2]) + m * float(M[3, 2])
    w3 = n * float(M[2, 3]) + m * float(M[3, 3])
    xe = w2 / w
    ye = w3 / w
    r2 = xe * xe + ye * ye
    if r2 > 1.0:
        return None
    ze = hemisphere * math.sqrt(1.0 - r2)
    x, y, z = ecliptic_to_equatorial(xe, ye, ze, eps)
    alpha = math.atan2(y, x)
    if alpha < 0.0:
        alpha += 2.0 * math.pi
    return alpha, math.asin(min(1.0, max(-1.0, z)))


def lattice_sky_range(M: np.ndarray, f_ref: float):
    """Smallest box [n_lo, n_hi] x [m_lo, m_hi] holding every (n, m) on the sky: the disk
    |(w2, w3)| <= W mapped through the inverse of the sky rows."""
    w = lattice_sky_scale(f_ref)
    det = float(M[2, 2]) * float(M[3, 3]) - float(M[2, 3]) * float(M[3, 2])
    n_hi = int(math.floor(w * math.hypot(float(M[3, 2]), float(M[3, 3])) / abs(det)))
    m_hi = int(math.floor(w * math.hypot(float(M[2, 2]), float(M[2, 3])) / abs(det)))
    return -n_hi, n_hi, -m_hi, m_hi


def lattice_sky_points(M: np.ndarray, box, hemisphere: int, eps: float, f_ref: float):
    """Every (n, m) of the box on the sky, in order of (n, m): rows (n, m, alpha, delta,
    w0, w1), where (w0, w1) are the frequency and spindown parts of n M2 + m M3."""
    n_lo, n_hi, m_lo, m_hi = box
    rows = []
    for n in range(n_lo, n_hi + 1):
        for m in range(m_lo, m_hi + 1):
            p = lattice_sky_position(M, n, m, hemisphere, eps, f_ref)
            if p is None:
                continue
            rows.append((n, m, p[0], p[1], n * float(M[2, 0]) + m * float(M[3, 0]),
                         n * float(M[2, 1]) + m * float(M[3, 1])))
    return rows


def lattice_template(M: np.ndarray, s: int, w0_sky: float, w1_sky: float, nfft: int):
    """(w1, u) of the template (s, sky): its spindown phase coefficient and the shift, in
    bins of the nfft grid, of its frequencies above the Fourier bins."""
    w0 = s * float(M[1, 0]) + w0_sky
    w1 = s * float(M[1, 1]) + w1_sky
    x = w0 * (nfft / (2.0 * math.pi))
    return w1, x - math.floor(x + SHIFT_SNAP)


def lattice_demodulate(zt: np.ndarray, w1: float, u: float, nfft: int) -> np.ndarray:
    """Multiply by exp(-i (w1 j^2 + 2 pi u j / nfft)): the spindown phase and the grid's
    frequency shift, so that bin k of the transform is frequency (k + u) / (nfft dt)."""
    j = np.arange(zt.shape[0], dtype=np.float64)
    cyc = w1 * j * j / (2.0 * math.pi) + u * j / nfft
    cyc = cyc - np.floor(cyc)
    return zt * np.exp(-2j * math.pi * cyc)


def lattice_template_two_f(seg, sky, w1: float, u: float, nfft: int, k_min: int = 0, k_max: int = -1,
                           full: bool = False, interbin: bool = False) -> np.ndarray:
    """2F over bins [k_min, k_max) of one lattice template (zero-padded or interbinned)."""
    if k_max < 0:
        k_max = nfft // 2
    tr = interbinned_transform if interbin else fourier_transform
    fa = tr(lattice_demodulate(sky["za_t"], w1, u, nfft), nfft)[k_min:k_max]
    fb = tr(lattice_demodulate(sky["zb_t"], w1, u, nfft), nfft)[k_min:k_max]
    if full:
        return two_f_full(fa, fb, sky["A"], sky["B"], sky["C"], seg.n, seg.sigma2)
    return two_f(fa, fb, sky["A"], sky["B"], seg.n, seg.sigma2)


# ---------------------------------------------------------------- candidates
CANDIDATE_DTYPE = np.dtype([("segment", np.int32), ("sky", np.int32), ("fdot_idx", np.int32),
                            ("bin", np.int32), ("f_hz", np.float64), ("fdot", np.float64),
                            ("alpha", np.float64), ("delta", np.float64), ("twoF", np.float64)])


def search(seg, alpha, delta, fdot, threshold: float, nfft: int = 0, k_min: int = 0,
           k_max: int = -1, segment_index: int = 0, full: bool = False,
           skies=None, fdot_indices=None, interbin: bool = False):
    """Threshold crossings of every (sky, spindown) template (Sect. 2, Fig. 3).

    Each candidate is the paper's five numbers (frequency, spindown, sky
    position, 2F) plus its integer key (segment, sky, spindown index, bin);
    the result is sorted by key.  `skies` / `fdot_indices` restrict the search
    to a subset of the lists (same indices as the full search).  `interbin`
    selects the interbinned transform of nfft/2 points.
    """
    if nfft <= 0:
        nfft = default_nfft(seg.n)
    if k_max < 0:
        k_max = nfft // 2
    alpha = np.asarray(alpha, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64)
    fdot = np.asarray(fdot, dtype=np.float64)
    skies = range(alpha.shape[0]) if skies is None else skies
    fdot_indices = range(fdot.shape[0]) if fdot_indices is None else fdot_indices
    rows = []
    for i in skies:
        sky = sky_stage(seg, float(alpha[i]), float(delta[i]), nfft)
        for s in fdot_indices:
            tfun = template_two_f_interbin if interbin else template_two_f
            tf = tfun(seg, sky, float(fdot[s]), nfft, k_min, k_max, full)
            ks = np.nonzero(tf > threshold)[0]
            for k in ks:
                kk = int(k) + k_min
                rows.append((segment_index, i, s, kk, seg.f_off + kk / (nfft * seg.dt),
                             float(fdot[s]), float(alpha[i]), float(delta[i]), float(tf[k])))
    out = np.array(rows, dtype=CANDIDATE_DTYPE)
    return np.sort(out, order=["segment", "sky", "fdot_idx", "bin"])


def search_lattice(seg, M, points, s_lo: int, s_hi: int, threshold: float, nfft: int = 0,
                   k_min: int = 0, k_max: int = -1, segment_index: int = 0, full: bool = False,
                   interbin: bool = False, skies=None, spins=None):
    """Threshold crossings over lattice templates: the sky points `points` (rows of
    lattice_sky_points) times the spindown integers s_lo..s_hi.  The key's spindown index
    is s - s_lo; a candidate's frequency is f_off + (bin + u) / (nfft dt) and its spindown
    w1 / (pi dt^2).  `skies` / `spins` restrict the search to subsets (same indices)."""
    M = np.asarray(M, dtype=np.float64).reshape(4, 4)
    if nfft <= 0:
        nfft = default_nfft(seg.n)
    if k_max < 0:
        k_max = nfft // 2
    skies = range(len(points)) if skies is None else skies
    spins = range(s_hi - s_lo + 1) if spins is None else spins
    rows = []
    for i in skies:
        _, _, alpha, delta, w0_sky, w1_sky = points[i]
        sky = sky_stage(seg, alpha, delta, nfft)
        for si in spins:
            w1, u = lattice_template(M, s_lo + si, w0_sky, w1_sky, nfft)
            tf = lattice_template_two_f(seg, sky, w1, u, nfft, k_min, k_max, full, interbin)
            fdot = w1 / (math.pi * seg.dt * seg.dt)
            for k in np.nonzero(tf > threshold)[0]:
                kk = int(k) + k_min
                rows.append((segment_index, i, si, kk, seg.f_off + (kk + u) / (nfft * seg.dt),
                             fdot, alpha, delta, float(tf[k])))
    out = np.array(rows, dtype=CANDIDATE_DTYPE)
    return np.sort(out, order=["segment", "sky", "fdot_idx", "bin"])

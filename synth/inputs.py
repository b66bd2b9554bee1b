"""Seeded synthetic detector data, ephemeris and template lists.

Shapes follow the paper's workload (Sect. 2): one data segment is one
(frame, band) pair, a narrowband real series of N double-precision samples
spanning two sidereal days, together with the detector-to-SSB position vector
for every sample.  The paper's VSR1 data and ephemeris files are not
available, so they are replaced by

* white Gaussian noise of known variance (the paper's own tests also ran on
  Gaussian noise, Sect. 1) plus injected continuous-wave signals, and
* an analytic ephemeris: a circular Earth orbit of 1 AU in the ecliptic plus
  the sidereal rotation of a detector on a spherical Earth.

Everything here is an input to the search; the search arithmetic lives
elsewhere.  The injected signal's antenna response is computed from the
detector tensor and polarisation tensors (not from closed forms), and its
phase from the source's own barycentric arrival time.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# --- physical constants and the conventional detector -----------------------
C_LIGHT = 299792458.0                      # m/s
AU_LS = 149597870700.0 / C_LIGHT           # 1 AU in light-seconds (499.00478 s)
RE_LS = 6378137.0 / C_LIGHT                # Earth equatorial radius in light-seconds
SIDEREAL_DAY = 86164.0905                  # s
OMEGA_R = 2.0 * math.pi / SIDEREAL_DAY     # Earth rotation rate, rad/s
OMEGA_O = 2.0 * math.pi / (365.25636 * 86400.0)  # orbital rate, rad/s
OBLIQUITY = math.radians(23.4392911)       # obliquity of the ecliptic

DET_LAT = math.radians(46.45)              # detector latitude
DET_GAMMA = math.radians(171.8)            # arm-bisector orientation, ccw from local East
DET_PHI_R = 0.0                            # local sidereal angle at t = 0
ORBIT_PHI_O = 0.0                          # orbital phase at t = 0


def band_offset(b):
    """Lower band edge f_off = 100 + (1 - 2^-5) b Hz (Sect. 2, Eq. 1)."""
    return 100.0 + (1.0 - 2.0 ** -5) * np.asarray(b, dtype=np.float64)


def nfft_for(n: int) -> int:
    """Smallest power of two >= 2n (the 2x Fourier-interpolated FFT length)."""
    m = 1
    while m < 2 * n:
        m *= 2
    return m


# --- ephemeris ---------------------------------------------------------------
def ephemeris(n: int, dt: float, lat: float = DET_LAT, phi_r: float = DET_PHI_R,
              phi_o: float = ORBIT_PHI_O, eps: float = OBLIQUITY) -> np.ndarray:
    """Detector position relative to the SSB, equatorial frame, light-seconds.

    Returns r with shape (3, n) for t_i = i*dt: a circular orbit of radius
    1 AU in the ecliptic (inclined by the obliquity eps to the equator)
    plus the detector's position on the rotating Earth.  This stands in for
    the 3N doubles of the paper's detector ephemeris file (Sect. 2).
    """
    t = np.arange(n, dtype=np.float64) * dt
    lo = OMEGA_O * t + phi_o
    th = OMEGA_R * t + phi_r
    r = np.empty((3, n), dtype=np.float64)
    r[0] = AU_LS * np.cos(lo) + RE_LS * math.cos(lat) * np.cos(th)
    r[1] = AU_LS * math.cos(eps) * np.sin(lo) + RE_LS * math.cos(lat) * np.sin(th)
    r[2] = AU_LS * math.sin(eps) * np.sin(lo) + RE_LS * math.sin(lat)
    return r


# --- template lists ----------------------------------------------------------
def fibonacci_sky(nsky: int):
    """Near-uniform sky points: sin(delta_i) = 1-(2i+1)/nsky, alpha_i = 2 pi i / golden ratio."""
    i = np.arange(nsky, dtype=np.float64)
    golden = (1.0 + math.sqrt(5.0)) / 2.0
    delta = np.arcsin(1.0 - (2.0 * i + 1.0) / nsky)
    alpha = np.mod(2.0 * math.pi * i / golden, 2.0 * math.pi)
    return alpha, delta


def spindown_grid(nfdot: int, fdot_min: float = -1e-9) -> np.ndarray:
    """Uniform spindown list from 0 down to fdot_min (Hz/s)."""
    if nfdot == 1:
        return np.zeros(1)
    return fdot_min * np.arange(nfdot, dtype=np.float64) / (nfdot - 1)


def lattice_matrix(nfft: int, dt: float, f_ref: float, sky_points: int, fdot_step: float, seed: int,
                   freq_bins: int = 1) -> np.ndarray:
    """A 4x4 grid generating matrix of the constrained form, standing in for the grid file.

    Rows over the phase parameters (w0, w1, w2, w3) (frequency in radians per sample,
    spindown phase coefficient, two ecliptic-plane sky coordinates of radius
    2 pi f_ref AU/c): row 0 = `freq_bins` Fourier bins of the nfft grid along w0; row 1 =
    the spindown step pi fdot_step dt^2 with a random fraction of a bin along w0; rows 2
    and 3 = a hexagonal sky lattice, rotated at random, with about `sky_points` points
    per hemisphere, each with random fractions of a bin and of a spindown step.
    """
    rng = np.random.default_rng(seed)
    bin_w = 2.0 * math.pi / nfft
    w_sky = 2.0 * math.pi * f_ref * AU_LS
    h = w_sky * math.sqrt(2.0 * math.pi / (math.sqrt(3.0) * sky_points))
    rot = float(rng.uniform(0.0, 2.0 * math.pi))
    w1_step = math.pi * fdot_step * dt * dt
    M = np.zeros((4, 4), dtype=np.float64)
    M[0, 0] = freq_bins * bin_w
    M[1, 0] = float(rng.uniform(0.0, 1.0)) * bin_w
    M[1, 1] = w1_step
    for r, ang in ((2, rot), (3, rot + math.pi / 3.0)):
        M[r, 0] = float(rng.uniform(0.0, 1.0)) * bin_w
        M[r, 1] = float(rng.uniform(-0.5, 0.5)) * w1_step
        M[r, 2] = h * math.cos(ang)
        M[r, 3] = h * math.sin(ang)
    return M


# --- injected signals ----------------------------------------------------------
@dataclasses.dataclass
class Injection:
    """A continuous-wave source: narrowband frequency f (Hz above f_off), spindown,
    sky position, polarisation angle psi, cos(inclination), initial phase, SNR."""
    f: float
    fdot: float
    alpha: float
    delta: float
    psi: float
    cosi: float
    phi0: float
    snr: float
    h0: float = 0.0  # filled in by make_segment


def draw_injections(rng: np.random.Generator, count: int, snr_lo: float, snr_hi: float,
                    f_band: float = 0.25) -> List[Injection]:
    out = []
    for _ in range(count):
        out.append(Injection(
            f=float(rng.uniform(0.0, f_band)),
            fdot=float(rng.uniform(-1e-9, 0.0)),
            alpha=float(rng.uniform(0.0, 2 * math.pi)),
            delta=float(math.asin(rng.uniform(-1.0, 1.0))),
            psi=float(rng.uniform(0.0, math.pi)),
            cosi=float(rng.uniform(-1.0, 1.0)),
            phi0=float(rng.uniform(0.0, 2 * math.pi)),
            snr=float(rng.uniform(snr_lo, snr_hi)) if snr_hi > snr_lo else float(snr_lo)))
    return out


def detector_tensor(t: np.ndarray, lat: float, gamma: float, phi_r: float) -> np.ndarray:
    """Detector tensor D = (u u^T - v v^T)/2 in the equatorial frame, shape (n, 3, 3).

    Arms u, v are unit vectors in the local horizontal plane at gamma - 45 deg
    and gamma + 45 deg counter-clockwise from local East (right-angle arms).
    """
    th = phi_r + OMEGA_R * t
    east = np.stack([-np.sin(th), np.cos(th), np.zeros_like(th)], axis=-1)
    north = np.stack([-math.sin(lat) * np.cos(th), -math.sin(lat) * np.sin(th),
                      np.full_like(th, math.cos(lat))], axis=-1)
    u = math.cos(gamma - math.pi / 4) * east + math.sin(gamma - math.pi / 4) * north
    v = math.cos(gamma + math.pi / 4) * east + math.sin(gamma + math.pi / 4) * north
    return 0.5 * (u[:, :, None] * u[:, None, :] - v[:, :, None] * v[:, None, :])


def polarisation_tensors(alpha: float, delta: float, psi: float):
    """Plus and cross tensors of a wave from (alpha, delta), polarisation angle psi."""
    p = np.array([math.sin(alpha), -math.cos(alpha), 0.0])
    q = np.array([-math.sin(delta) * math.cos(alpha), -math.sin(delta) * math.sin(alpha),
                  math.cos(delta)])
    pr = p * math.cos(psi) + q * math.sin(psi)
    qr = -p * math.sin(psi) + q * math.cos(psi)
    eplus = np.outer(pr, pr) - np.outer(qr, qr)
    ecross = np.outer(pr, qr) + np.outer(qr, pr)
    return eplus, ecross


def antenna_response(t: np.ndarray, alpha: float, delta: float, psi: float,
                     lat: float = DET_LAT, gamma: float = DET_GAMMA, phi_r: float = DET_PHI_R):
    """F_plus(t), F_cross(t) = D(t) : e_plus, D(t) : e_cross."""
    d = detector_tensor(np.asarray(t, dtype=np.float64), lat, gamma, phi_r)
    ep, ex = polarisation_tensors(alpha, delta, psi)
    return np.einsum("nij,ij->n", d, ep), np.einsum("nij,ij->n", d, ex)


def cw_signal(inj: Injection, n: int, dt: float, f_off: float, r: np.ndarray,
              lat: float = DET_LAT, gamma: float = DET_GAMMA, phi_r: float = DET_PHI_R,
              h0: float = 1.0) -> np.ndarray:
    """Heterodyned narrowband strain of one source (physical frequency f_off + f).

    The source's barycentric arrival time is tau = t + k.(r(t) - r(0)) with k the
    unit vector to the source; the physical phase is
    2 pi [(f_off + f) tau + fdot tau^2 / 2] + phi0, from which the band
    heterodyne 2 pi f_off t is removed.
    """
    t = np.arange(n, dtype=np.float64) * dt
    k = np.array([math.cos(inj.delta) * math.cos(inj.alpha),
                  math.cos(inj.delta) * math.sin(inj.alpha), math.sin(inj.delta)])
    delay = k @ r - k @ r[:, 0]
    tau = t + delay
    # cycles = (f_off + f) tau + fdot tau^2/2 - f_off t, grouped to keep FP64 accuracy
    cyc = f_off * delay + inj.f * tau + 0.5 * inj.fdot * tau * tau
    cyc = cyc - np.floor(cyc)
    phase = 2.0 * math.pi * cyc + inj.phi0
    fp, fx = antenna_response(t, inj.alpha, inj.delta, inj.psi, lat, gamma, phi_r)
    hp = h0 * 0.5 * (1.0 + inj.cosi ** 2) * np.cos(phase)
    hx = h0 * inj.cosi * np.sin(phase)
    return fp * hp + fx * hx


def cw_basis(inj: Injection, n: int, dt: float, f_off: float, r: np.ndarray,
             lat: float = DET_LAT, gamma: float = DET_GAMMA, phi_r: float = DET_PHI_R) -> np.ndarray:
    """The four waveforms whose combination is any signal of this sky position,
    frequency and spindown: F+(psi=0) cos(phase), Fx(psi=0) cos(phase),
    F+(psi=0) sin(phase), Fx(psi=0) sin(phase), with the heterodyned phase of
    cw_signal without phi0.  A signal with amplitudes (A1, A2, A3, A4) is
    sum_mu A_mu basis[mu]; shape (4, n)."""
    t = np.arange(n, dtype=np.float64) * dt
    k = np.array([math.cos(inj.delta) * math.cos(inj.alpha),
                  math.cos(inj.delta) * math.sin(inj.alpha), math.sin(inj.delta)])
    delay = k @ r - k @ r[:, 0]
    tau = t + delay
    cyc = f_off * delay + inj.f * tau + 0.5 * inj.fdot * tau * tau
    cyc = cyc - np.floor(cyc)
    phase = 2.0 * math.pi * cyc
    fp, fx = antenna_response(t, inj.alpha, inj.delta, 0.0, lat, gamma, phi_r)
    c, s = np.cos(phase), np.sin(phase)
    return np.stack([fp * c, fx * c, fp * s, fx * s])


# --- segments ---------------------------------------------------------------------
@dataclasses.dataclass
class Segment:
    """One (frame, band) data set: series x, ephemeris r, detector and band parameters."""
    n: int
    dt: float
    f_off: float
    sigma2: float
    x: np.ndarray              # (n,) float64
    r: np.ndarray              # (3, n) float64, light-seconds
    lat: float = DET_LAT
    gamma: float = DET_GAMMA
    phi_r: float = DET_PHI_R
    injections: List[Injection] = dataclasses.field(default_factory=list)

    @property
    def nfft(self) -> int:
        return nfft_for(self.n)


def make_segment(n: int, dt: float = 2.0, f_off: float = 100.0, sigma: float = 1.0,
                 noise_seed: Optional[int] = None, injections: Sequence[Injection] = (),
                 lat: float = DET_LAT, gamma: float = DET_GAMMA, phi_r: float = DET_PHI_R,
                 phi_o: float = ORBIT_PHI_O) -> Segment:
    """x = sigma * n + sum of injections, each scaled so that sum(h^2)/sigma^2 = snr^2.

    noise_seed None gives a noiseless segment.
    """
    r = ephemeris(n, dt, lat, phi_r, phi_o)
    if noise_seed is None:
        x = np.zeros(n)
    else:
        x = sigma * np.random.default_rng(noise_seed).standard_normal(n)
    injs = []
    for inj in injections:
        h1 = cw_signal(inj, n, dt, f_off, r, lat, gamma, phi_r, h0=1.0)
        h0 = inj.snr * sigma / math.sqrt(float(np.dot(h1, h1)))
        x = x + h0 * h1
        injs.append(dataclasses.replace(inj, h0=h0))
    return Segment(n=n, dt=dt, f_off=float(f_off), sigma2=sigma * sigma, x=x, r=r,
                   lat=lat, gamma=gamma, phi_r=phi_r, injections=injs)


# --- the search workloads ----------------------------------------------------------------
N_FULL = 86164            # two sidereal days at dt = 2 s
THRESHOLD_2F = 20.0


@dataclasses.dataclass
class Workload:
    name: str
    segments: List[Segment]
    alpha: np.ndarray
    delta: np.ndarray
    fdot: np.ndarray
    threshold: float
    fp64: bool


# name -> seed offset of the workload's noise (1000 + offset) and injections (2000 + offset)
WORKLOADS = {"tiny": 1, "full": 2, "batched": 3, "ragged": 4}


def workload(name: str, nsky: Optional[int] = None, nfdot: Optional[int] = None) -> Workload:
    """Seeded inputs of the four search workloads.

    tiny:    N=4096, 8 sky x 4 spindown, one SNR-10 injection, FP64 throughout.
    full:    one full segment N=86164, 256 x 64 templates, one SNR-10 injection.
    batched: one full segment N=86164, 4096 x 256 templates, five injections at SNR 8-20.
    ragged:  32 segments, N ~ U{20000..172328}, band offsets from Eq. 1,
             0-3 injections each, 1024 x 128 templates per segment.
    nsky / nfdot override the grid size (parity tests use sub-grids).
    """
    if name not in WORKLOADS:
        raise ValueError(f"unknown workload {name!r}")
    c = WORKLOADS[name]
    rng_inj = np.random.default_rng(2000 + c)
    if name == "tiny":
        injs = draw_injections(rng_inj, 1, 10.0, 10.0)
        segs = [make_segment(4096, 2.0, 100.0, 1.0, 1001, injs)]
        ns, nf, fp64 = 8, 4, True
    elif name == "full":
        injs = draw_injections(rng_inj, 1, 10.0, 10.0)
        segs = [make_segment(N_FULL, 2.0, 100.0, 1.0, 1002, injs)]
        ns, nf, fp64 = 256, 64, False
    elif name == "batched":
        injs = draw_injections(rng_inj, 5, 8.0, 20.0)
        segs = [make_segment(N_FULL, 2.0, 100.0, 1.0, 1003, injs)]
        ns, nf, fp64 = 4096, 256, False
    else:
        segs = []
        for i in range(32):
            n = int(rng_inj.integers(20000, 172328 + 1))
            f_off = float(band_offset(int(rng_inj.integers(0, 1000))))
            injs = draw_injections(rng_inj, int(rng_inj.integers(0, 4)), 8.0, 20.0)
            segs.append(make_segment(n, 2.0, f_off, 1.0, 1004 * 1000 + i, injs))
        ns, nf, fp64 = 1024, 128, False
    ns = nsky if nsky is not None else ns
    nf = nfdot if nfdot is not None else nf
    alpha, delta = fibonacci_sky(ns)
    return Workload(name=name, segments=segs, alpha=alpha, delta=delta,
                    fdot=spindown_grid(nf), threshold=THRESHOLD_2F, fp64=fp64)

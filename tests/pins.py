"""Checks that pin the oracle to mathematics outside itself.

Each function returns a measured discrepancy; the tests assert bounds on it,
and the mutation tests plant mistakes in the oracle and assert that at least
one of these checks then fails.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.interpolate
import scipy.stats

from oracle import fstat_oracle as oracle
import synth


# ---- P0: amplitude modulations vs the detector tensor ------------------------------
def p0_amplitude_vs_tensor(seed: int = 0, trials: int = 40) -> float:
    """max |a - D:e+(psi=0)|, |b - D:ex(psi=0)| over random sky, time and detector."""
    rng = np.random.default_rng(seed)
    err = 0.0
    for _ in range(trials):
        alpha = rng.uniform(0, 2 * math.pi)
        delta = math.asin(rng.uniform(-1, 1))
        lat = rng.uniform(-1.5, 1.5)
        gamma = rng.uniform(0, math.pi)
        phi_r = rng.uniform(0, 2 * math.pi)
        n, dt = 64, rng.uniform(100.0, 3000.0)
        a, b = oracle.amplitude_modulation(n, dt, alpha, delta, lat, gamma, phi_r)
        t = np.arange(n) * dt
        fp, fx = synth.antenna_response(t, alpha, delta, 0.0, lat, gamma, phi_r)
        err = max(err, float(np.max(np.abs(a - fp))), float(np.max(np.abs(b - fx))))
    return err


# ---- P4: the Fourier transform step vs a brute-force DFT ---------------------------
def p4_fft_vs_bruteforce(n: int = 37, nfft: int = 128, seed: int = 1) -> float:
    rng = np.random.default_rng(seed)
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    got = oracle.fourier_transform(y, nfft)
    j = np.arange(n)
    ref = np.array([np.sum(y * np.exp(-2j * math.pi * j * k / nfft)) for k in range(nfft)])
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def p4_tone_peak_bin(nfft: int = 256, k0: int = 37) -> int:
    """A tone exp(+2 pi i k0 j / nfft) must peak at bin k0 (forward sign -i)."""
    j = np.arange(nfft // 2)
    f = oracle.fourier_transform(np.exp(2j * math.pi * k0 * j / nfft), nfft)
    return int(np.argmax(np.abs(f)))


# ---- upsampling: u[2i] = z[i] and the odd points vs the trigonometric interpolant --------
def upsample_errors(n: int = 24, nfft: int = 64, seed: int = 2):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    u = oracle.fft_upsample2(z, nfft)
    even_err = float(np.max(np.abs(u[0::2][:n] - z)))
    # brute force: periodic trigonometric interpolant of zp (z zero-padded to M) with
    # frequencies -M/2 .. M/2-1, evaluated at half-integer sample positions
    m = nfft // 2
    zp = np.zeros(m, dtype=complex)
    zp[:n] = z
    i = np.arange(m)
    freqs = np.concatenate([np.arange(0, m // 2), np.arange(-m // 2, 0)])
    coef = np.array([np.sum(zp * np.exp(-2j * math.pi * q * i / m)) / m for q in freqs])
    pos = np.arange(nfft) / 2.0
    interp = np.array([np.sum(coef * np.exp(2j * math.pi * freqs * p / m)) for p in pos])
    odd_err = float(np.max(np.abs(u - interp)))
    return even_err, odd_err


# ---- P5: the natural cubic spline --------------------------------------------------------
def p5_spline_vs_scipy(L: int = 300, seed: int = 3) -> float:
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    pos = rng.uniform(0, L - 1, 1000)
    pos = np.concatenate([pos, [0.0, L - 1.0, 1.0, L - 2.0]])
    mom = oracle.natural_spline_moments(u)
    got = oracle.natural_spline_eval(u, mom, pos)
    x = np.arange(L, dtype=float)
    ref = (scipy.interpolate.CubicSpline(x, u.real, bc_type="natural")(pos)
           + 1j * scipy.interpolate.CubicSpline(x, u.imag, bc_type="natural")(pos))
    return float(np.max(np.abs(got - ref)))


def p5_spline_linear_exact(L: int = 200) -> float:
    u = 3.0 - 0.25 * np.arange(L) + 1j * (0.5 * np.arange(L) - 7.0)
    mom = oracle.natural_spline_moments(u)
    pos = np.linspace(0, L - 1, 777)
    got = oracle.natural_spline_eval(u, mom, pos)
    return float(np.max(np.abs(got - (3.0 - 0.25 * pos + 1j * (0.5 * pos - 7.0)))))


# ---- resampling of a smooth tone with a known delay --------------------------------------
def resample_tone_error(n: int = 4096, dt: float = 2.0, f0: float = 0.01, nfft: int = 0) -> float:
    """z_i = exp(2 pi i f0 i dt) resampled with delay D must give exp(2 pi i f0 (j dt - D_j))."""
    nfft = nfft or oracle.default_nfft(n)
    t = np.arange(n) * dt
    delay = 300.0 * np.sin(2 * math.pi * t / (n * dt * 3.0)) + 20.0 * np.sin(2 * math.pi * t / 86164.0)
    delay = delay - delay[0]
    z = np.exp(2j * math.pi * f0 * t)
    zt = oracle.resample(z, delay, dt, nfft)
    s = np.arange(n) - delay / dt
    inside = (s >= 0) & (s <= n - 1)
    # stay away from the ends, where the periodic band-limited interpolant wraps
    core = inside & (s > 64) & (s < n - 65)
    ref = np.exp(2j * math.pi * f0 * (t - delay))
    outside_ok = np.all(zt[~inside] == 0)
    return float(np.max(np.abs(zt[core] - ref[core]))) if outside_ok else float("inf")


# ---- P2 / P1: noiseless injection -------------------------------------------------------
def jks_amplitudes(inj: synth.Injection):
    ap = inj.h0 * (1 + inj.cosi ** 2) / 2.0
    ax = inj.h0 * inj.cosi
    c2, s2 = math.cos(2 * inj.psi), math.sin(2 * inj.psi)
    cp, sp = math.cos(inj.phi0), math.sin(inj.phi0)
    a1 = ap * c2 * cp - ax * s2 * sp
    a2 = ap * s2 * cp + ax * c2 * sp
    a3 = -ap * c2 * sp - ax * s2 * cp
    a4 = -ap * s2 * sp + ax * c2 * cp
    return a1, a2, a3, a4


def closed_form_two_f(inj, A, B, C, n, sigma2=1.0):
    """Noiseless simplified 2F at the matched template: (N/2)[((A1A+A2C)^2+(A3A+A4C)^2)/A + ...]."""
    a1, a2, a3, a4 = jks_amplitudes(inj)
    return (n / (2.0 * sigma2)) * (((a1 * A + a2 * C) ** 2 + (a3 * A + a4 * C) ** 2) / A
                                   + ((a1 * C + a2 * B) ** 2 + (a3 * C + a4 * B) ** 2) / B)


def on_grid_injection(n: int, dt: float = 2.0, f_off: float = 100.0, fdot: float = -4e-10,
                      alpha: float = 1.1, delta: float = 0.3, frac: float = 0.113, snr: float = 10.0,
                      psi: float = 0.7, cosi: float = 0.35, phi0: float = 2.1):
    nfft = oracle.default_nfft(n)
    k0 = int(round(frac * nfft))
    inj = synth.Injection(f=k0 / (nfft * dt), fdot=fdot, alpha=alpha, delta=delta, psi=psi,
                          cosi=cosi, phi0=phi0, snr=snr)
    seg = synth.make_segment(n, dt, f_off, 1.0, None, [inj])
    return seg, seg.injections[0], k0, nfft


def p2_closed_form(n: int, **kw):
    """(oracle 2F at the injection bin, closed form, peak bin, expected bin)."""
    seg, inj, k0, nfft = on_grid_injection(n, **kw)
    sky = oracle.sky_stage(seg, inj.alpha, inj.delta, nfft)
    tf = oracle.template_two_f(seg, sky, inj.fdot, nfft)
    cf = closed_form_two_f(inj, sky["A"], sky["B"], sky["C"], n, seg.sigma2)
    return float(tf[k0]), float(cf), int(np.argmax(tf)), k0


def direct_two_f(seg, alpha, delta, f_narrow, fdot):
    """2F from the direct detector-time sum, no resampling and no FFT:
    Fa = sum_i x_i a_i exp(-i[2 pi (f tau_i + fdot tau_i^2/2) + 2 pi f_off D_i]),
    with a, b from the detector tensor (psi = 0)."""
    t = np.arange(seg.n) * seg.dt
    k = np.array([math.cos(delta) * math.cos(alpha), math.cos(delta) * math.sin(alpha), math.sin(delta)])
    d = k @ seg.r - k @ seg.r[:, 0]
    tau = t + d
    a, b = synth.antenna_response(t, alpha, delta, 0.0, seg.lat, seg.gamma, seg.phi_r)
    cyc = f_narrow * tau + 0.5 * fdot * tau * tau + seg.f_off * d
    cyc = cyc - np.floor(cyc)
    e = np.exp(-2j * math.pi * cyc)
    fa = np.sum(seg.x * a * e)
    fb = np.sum(seg.x * b * e)
    A, B = float(np.mean(a * a)), float(np.mean(b * b))
    return (2.0 / (seg.n * seg.sigma2)) * (abs(fa) ** 2 / A + abs(fb) ** 2 / B)


def p1_direct_vs_resampled(n: int, frac: float = 0.2071, **kw):
    """Off-bin injection; (oracle 2F, direct-sum 2F) at the oracle's peak bin."""
    nfft = oracle.default_nfft(n)
    dt = 2.0
    inj = synth.Injection(f=frac / (2 * dt) + 0.37 / (nfft * dt), fdot=-6e-10, alpha=4.0, delta=-0.6,
                          psi=2.0, cosi=-0.5, phi0=0.3, snr=10.0)
    seg = synth.make_segment(n, dt, 230.5, 1.0, None, [inj])
    sky = oracle.sky_stage(seg, inj.alpha, inj.delta, nfft)
    tf = oracle.template_two_f(seg, sky, inj.fdot, nfft)
    k = int(np.argmax(tf))
    return float(tf[k]), float(direct_two_f(seg, inj.alpha, inj.delta, k / (nfft * dt), inj.fdot))


# ---- P3: noise statistics ---------------------------------------------------------------
def p3_noise_stats(n: int = synth.N_FULL, realisations: int = 6, seed: int = 77):
    """2F over pure-noise segments (independent realisations, one template each).

    Bins from 1% to 75% of the band: at the top of the band the cubic spline of
    the resampling attenuates the noise by a few percent.  Every third bin is
    used for the KS test (the zero-padding to nfft ~ 3N correlates neighbours).
    """
    nfft = oracle.default_nfft(n)
    lo, hi = nfft // 200, (3 * nfft) // 8
    vals = []
    for r in range(realisations):
        seg = synth.make_segment(n, 2.0, 100.0, 1.0, seed + r, [])
        sky = oracle.sky_stage(seg, 2.3 + 0.7 * r, -0.4 + 0.1 * r, nfft)
        vals.append(oracle.template_two_f(seg, sky, -1e-10 * r, nfft)[lo:hi])
    v = np.concatenate(vals)
    sparse = np.concatenate([x[0::3] for x in vals])
    ks = scipy.stats.kstest(sparse[::2], scipy.stats.chi2(4).cdf)
    return float(v.mean()), float(v.var()), float(np.mean(v > 20.0)), sparse.size, float(ks.pvalue)


# ---- P6: linearity ----------------------------------------------------------------------
def p6_linearity(n: int = 4096, seed: int = 5) -> float:
    rng = np.random.default_rng(seed)
    s1 = synth.make_segment(n, 2.0, 150.0, 1.0, seed, [])
    s2 = synth.make_segment(n, 2.0, 150.0, 1.0, seed + 1, [])
    s12 = synth.make_segment(n, 2.0, 150.0, 1.0, None, [])
    s12.x = s1.x + 0.5 * s2.x
    nfft = oracle.default_nfft(n)
    al, de, fd = rng.uniform(0, 6), rng.uniform(-1, 1), -3e-10
    f = []
    for s in (s1, s2, s12):
        sky = oracle.sky_stage(s, al, de, nfft)
        f.append(oracle.fourier_transform(oracle.spindown_demodulate(sky["za_t"], fd, s.dt), nfft))
    return float(np.max(np.abs(f[2] - (f[0] + 0.5 * f[1]))) / np.max(np.abs(f[2])))


# ---------------------------------------------------------------- interbinning
def ib_midway_error(n: int = 3000, nfft: int = 8192, k0: int = 517) -> float:
    """| |odd bin 2 k0 + 1| - exact | / exact for a sinusoid midway between bins k0, k0 + 1."""
    half = nfft // 2
    j = np.arange(n)
    y = 0.3 * np.exp(1j * 0.7) * np.exp(2j * math.pi * (k0 + 0.5) * j / half)
    ib = oracle.interbinned_transform(y, nfft)
    return abs(abs(ib[2 * k0 + 1]) - 0.3 * n) / (0.3 * n)


def ib_direct_sum_error(n: int = 500, nfft: int = 2048, seed: int = 12) -> float:
    """Max relative deviation of odd bins (interior and the wrap-around one) and even bins
    from direct sums: even 2k = X_k, odd 2k + 1 = c (X_k - X_{k+1 mod nfft/2})."""
    half = nfft // 2
    g = np.random.default_rng(seed)
    y = g.standard_normal(n) + 1j * g.standard_normal(n)
    j = np.arange(n)
    c = oracle.interbin_weight(n, half)

    def X(k):
        return np.sum(y * np.exp(-2j * math.pi * j * (k % half) / half))
    ib = oracle.interbinned_transform(y, nfft)
    scale = abs(X(0))
    err = 0.0
    for k in (0, 1, 300, half - 2, half - 1):
        err = max(err, abs(ib[2 * k] - X(k)) / scale, abs(ib[2 * k + 1] - c * (X(k) - X(k + 1))) / scale)
    return err


def ib_weight_error() -> float:
    """Deviation of the full-length weight from the classic pi/4."""
    return abs(oracle.interbin_weight(4096, 4096) - math.pi / 4)


# ---- lattice grid ------------------------------------------------------------------------
def lattice_setup(n: int, dt: float = 2.0, f_off: float = 100.0, sky_points: int = 40, seed: int = 31,
                  fdot_step: float = -2e-10):
    """(nfft, f_ref, M, north-hemisphere sky points) of a synthetic constrained lattice."""
    nfft = oracle.default_nfft(n)
    f_ref = f_off + 0.5 / dt
    M = synth.lattice_matrix(nfft, dt, f_ref, sky_points, fdot_step, seed)
    box = oracle.lattice_sky_range(M, f_ref)
    return nfft, f_ref, M, oracle.lattice_sky_points(M, box, +1, synth.OBLIQUITY, f_ref)


def lattice_injection(n: int = synth.N_FULL, k_frac: float = 0.113):
    """A noiseless SNR-10 source exactly at a lattice grid point whose frequencies lie a
    fraction u in [0.3, 0.7] of a bin above the Fourier bins and whose spindown carries a
    sky offset.  Returns (2F of its template with the shift, with u = 0, with -u, all at
    bin k0; the closed form; the peak bin with the shift; k0), or None when no grid point
    near the middle of the lattice has such a shift."""
    dt, f_off = 2.0, 100.0
    nfft, f_ref, M, pts = lattice_setup(n, dt, f_off)
    # the source's parameters straight from the grid point s M1 + n M2 + m M3
    pick = None
    for p in pts:
        n_, m_ = p[0], p[1]
        for s in range(-4, 5):
            w0 = s * M[1, 0] + n_ * M[2, 0] + m_ * M[3, 0]
            w1 = s * M[1, 1] + n_ * M[2, 1] + m_ * M[3, 1]
            u = (w0 / (2.0 * math.pi) * nfft) % 1.0
            if 0.3 < u < 0.7 and n_ * M[2, 1] + m_ * M[3, 1] != 0.0 and w1 < 0.0:
                pick = (p, s, w1, u)
                break
        if pick:
            break
    if pick is None:
        return None
    p, s, w1, u = pick
    k0 = int(round(k_frac * nfft))
    inj = synth.Injection(f=(k0 + u) / (nfft * dt), fdot=w1 / (math.pi * dt * dt), alpha=p[2], delta=p[3],
                          psi=0.9, cosi=0.2, phi0=1.3, snr=10.0)
    seg = synth.make_segment(n, dt, f_off, 1.0, None, [inj])
    sky = oracle.sky_stage(seg, p[2], p[3], nfft)
    # the oracle's template for the same integers
    tw1, tu = oracle.lattice_template(M, s, p[4], p[5], nfft)
    tf = oracle.lattice_template_two_f(seg, sky, tw1, tu, nfft)
    tf0 = oracle.lattice_template_two_f(seg, sky, tw1, 0.0, nfft)
    tfm = oracle.lattice_template_two_f(seg, sky, tw1, -tu, nfft)
    cf = closed_form_two_f(seg.injections[0], sky["A"], sky["B"], sky["C"], n, seg.sigma2)
    return float(tf[k0]), float(tf0[k0]), float(tfm[k0]), float(cf), int(np.argmax(tf)), k0


def lattice_doppler_amplitude_error(seed: int = 5, trials: int = 8) -> float:
    """The sky coordinates (w2, w3) / (2 pi f_ref) must equal the amplitudes of the annual
    Roemer delay n.r(t) along cos and sin of the orbital longitude (a year of the
    synthetic ephemeris, least squares with the daily term); worst relative error."""
    f_ref = 100.25
    w = 2.0 * math.pi * f_ref
    nfft = 8192
    M = synth.lattice_matrix(nfft, 2.0, f_ref, 30, -2e-10, seed)
    box = oracle.lattice_sky_range(M, f_ref)
    pts = [p for h in (+1, -1) for p in oracle.lattice_sky_points(M, box, h, synth.OBLIQUITY, f_ref)]
    rng = np.random.default_rng(seed)
    dt = 3600.0
    nt = int(366 * 86400 / dt)
    r = synth.ephemeris(nt, dt)
    t = np.arange(nt) * dt
    lo = synth.OMEGA_O * t + synth.ORBIT_PHI_O
    th = synth.OMEGA_R * t + synth.DET_PHI_R
    basis = np.stack([np.cos(lo), np.sin(lo), np.cos(th), np.sin(th), np.ones(nt)], axis=1)
    worst = 0.0
    for i in rng.choice(len(pts), size=min(trials, len(pts)), replace=False):
        n_, m_, alpha, delta = pts[i][:4]
        k = np.array([math.cos(delta) * math.cos(alpha), math.cos(delta) * math.sin(alpha), math.sin(delta)])
        coef = np.linalg.lstsq(basis, k @ r, rcond=None)[0]
        w2 = n_ * M[2, 2] + m_ * M[3, 2]
        w3 = n_ * M[2, 3] + m_ * M[3, 3]
        worst = max(worst, abs(w * coef[0] - w2) / abs(w * synth.AU_LS), abs(w * coef[1] - w3) / abs(w * synth.AU_LS))
    return worst


def vet_signal_assembly_error(seed: int) -> float:
    """Largest deviation, relative to the window's peak, between a noiseless signal window
    assembled by linearity for the vetting data (basis transforms combined with the JKS
    amplitudes A1..A4) and the same source injected into a segment and run through the
    oracle's sky stage and template transform at the same template."""
    import dataclasses
    from oracle import vet_data
    rng = np.random.default_rng(seed)
    shape = vet_data.draw_shape(rng)
    nfft = oracle.default_nfft(vet_data.N)
    tr = vet_data.shape_transforms(shape, nfft)
    snr = float(rng.uniform(6.0, 20.0))
    psi, cosi, phi0 = float(rng.uniform(0, math.pi)), float(rng.uniform(-1, 1)), float(rng.uniform(0, 2 * math.pi))
    lin = vet_data.signal_two_f(tr, snr, psi, cosi, phi0)
    src = dataclasses.replace(shape["source"], psi=psi, cosi=cosi, phi0=phi0, snr=snr)
    seg = synth.make_segment(vet_data.N, vet_data.DT, vet_data.F_OFF, 1.0, None, [src])
    sky = oracle.sky_stage(seg, shape["alpha"], shape["delta"], nfft)
    direct = oracle.template_two_f(seg, sky, shape["fdot"], nfft)[tr["lo"]:tr["hi"]]
    return float(np.max(np.abs(lin - direct)) / np.max(direct))

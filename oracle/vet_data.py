"""Oracle-generated training and evaluation patches for candidate vetting (TEST INFRASTRUCTURE ONLY).

A patch is the 2F spectrum over 256 bins centred on a threshold crossing
(2F > 20) of one template, at N = 86164 (two sidereal days at 2 s).  Every
2F value comes from the FP64 oracle (sky stage, spindown demodulation, FFT,
F), never from the GPU library.

* noise patches: crossings of pure-noise segments (label 0);
* injection patches (label 1): a signal at SNR ~ U[snr_lo, snr_hi] near the
  template (sky offset up to 5e-5 rad, about half the sky spacing a two-day
  segment at 100 Hz needs, spindown offset up to 2e-12 Hz/s,
  frequency anywhere in the band), the patch centred on the largest crossing
  within 4 bins of the signal's bin.  Injections without a crossing there are
  the threshold's own false dismissals and are counted, not kept.

Signals are assembled by linearity: every step before |.|^2 is linear in the
data, so for each "shape" (template, injection sky, frequency, spindown) the
oracle transforms the four basis waveforms of synth.cw_basis once; a signal
of any polarisation, inclination, phase and amplitude is their combination
with the JKS amplitudes A1..A4.  The noise added to a signal is the oracle
transform of a noise segment for the same template, read at a random
frequency shift (the noise spectrum is stationary across the band).
"""
from __future__ import annotations

import concurrent.futures
import math
import os

import numpy as np

import synth
from oracle import fstat_oracle as ora

N = synth.N_FULL
DT = 2.0
F_OFF = 100.0
THRESHOLD = 20.0
HALF = 128          # patch = bins [c - HALF, c + HALF)
WIN = 160           # signal window half-width kept per shape


def jks_amplitudes(h0, psi, cosi, phi0):
    ap = h0 * (1 + cosi * cosi) / 2.0
    ax = h0 * cosi
    c2, s2 = math.cos(2 * psi), math.sin(2 * psi)
    cp, sp = math.cos(phi0), math.sin(phi0)
    return np.array([ap * c2 * cp - ax * s2 * sp, ap * s2 * cp + ax * c2 * sp,
                     -ap * c2 * sp - ax * s2 * cp, -ap * s2 * sp + ax * c2 * cp])


def _fa_fb(seg, sky, fdot, nfft):
    fa = ora.fourier_transform(ora.spindown_demodulate(sky["za_t"], fdot, seg.dt), nfft)[: nfft // 2]
    fb = ora.fourier_transform(ora.spindown_demodulate(sky["zb_t"], fdot, seg.dt), nfft)[: nfft // 2]
    return fa, fb


def _two_f(fa, fb, A, B):
    return (2.0 / N) * ((fa.real ** 2 + fa.imag ** 2) / A + (fb.real ** 2 + fb.imag ** 2) / B)


def draw_shape(rng):
    """A template (sky, spindown) and a nearby source's sky, frequency and spindown (the
    polarisation, inclination, phase and amplitude are left to the injections)."""
    al_t = float(rng.uniform(0, 2 * math.pi))
    de_t = float(math.asin(rng.uniform(-0.95, 0.95)))
    fd_t = float(rng.uniform(-1e-9, 0.0))
    off = 5e-5 * math.sqrt(rng.uniform()) * np.array([math.cos(a := rng.uniform(0, 2 * math.pi)), math.sin(a)])
    inj = synth.Injection(f=float(rng.uniform(0.02, 0.23)), fdot=fd_t + float(rng.uniform(-2e-12, 2e-12)),
                          alpha=al_t + off[0] / max(math.cos(de_t), 0.2), delta=de_t + off[1],
                          psi=0.0, cosi=0.0, phi0=0.0, snr=0.0)
    return dict(alpha=al_t, delta=de_t, fdot=fd_t, source=inj)


def shape_transforms(shape, nfft: int):
    """The oracle's Fa, Fb of the source's four basis waveforms (synth.cw_basis) at the
    template, over the window [lo, hi) of WIN bins either side of the source's bin, with
    the template's A, B and the basis Gram matrix."""
    nb = nfft // 2
    inj = shape["source"]
    r = synth.ephemeris(N, DT)
    k_sig = int(round(inj.f * nfft * DT))
    lo, hi = max(k_sig - WIN, 0), min(k_sig + WIN, nb)
    basis = synth.cw_basis(inj, N, DT, F_OFF, r)
    seg = synth.make_segment(N, DT, F_OFF, 1.0, None, [])
    fa_mu, fb_mu = [], []
    A = B = None
    for mu in range(4):
        seg.x = basis[mu]
        sky = ora.sky_stage(seg, shape["alpha"], shape["delta"], nfft)
        A, B = sky["A"], sky["B"]
        fa, fb = _fa_fb(seg, sky, shape["fdot"], nfft)
        fa_mu.append(fa[lo:hi])
        fb_mu.append(fb[lo:hi])
    return dict(k_sig=k_sig, lo=lo, hi=hi, fa=np.array(fa_mu), fb=np.array(fb_mu), A=A, B=B,
                gram=basis @ basis.T)


def signal_two_f(tr, snr: float, psi: float, cosi: float, phi0: float, noise=None):
    """2F over the window of a signal of the shape with these polarisation, inclination,
    phase and SNR (h0 such that sum h^2 = SNR^2 at unit noise variance), assembled from the
    basis transforms with the JKS amplitudes; `noise` = (Fa, Fb) of noise over the window
    is added before |.|^2."""
    amp = jks_amplitudes(1.0, psi, cosi, phi0)
    h0 = snr / math.sqrt(float(amp @ tr["gram"] @ amp))
    fa = h0 * (amp @ tr["fa"])
    fb = h0 * (amp @ tr["fb"])
    if noise is not None:
        fa = fa + noise[0]
        fb = fb + noise[1]
    return _two_f(fa, fb, tr["A"], tr["B"])


def shape_patches(seed: int, n_inj: int, n_noise_templates: int, snr_lo: float, snr_hi: float):
    """Patches of one shape: (inj_patches, noise_patches, n_dismissed, info)."""
    rng = np.random.default_rng(seed)
    nfft = ora.default_nfft(N)
    nb = nfft // 2
    shape = draw_shape(rng)
    tr = shape_transforms(shape, nfft)
    k_sig, lo, hi, A, B = tr["k_sig"], tr["lo"], tr["hi"], tr["A"], tr["B"]
    # noise of the same template, and a few more spindowns of it for noise crossings
    seg = synth.make_segment(N, DT, F_OFF, 1.0, None, [])
    seg.x = np.random.default_rng(seed + 7_000_000).standard_normal(N)
    sky_n = ora.sky_stage(seg, shape["alpha"], shape["delta"], nfft)
    fa_n, fb_n = _fa_fb(seg, sky_n, shape["fdot"], nfft)
    noise_patches = []
    for s in range(n_noise_templates):
        fd = shape["fdot"] if s == 0 else float(rng.uniform(-1e-9, 0.0))
        tf = _two_f(*(_fa_fb(seg, sky_n, fd, nfft) if s else (fa_n, fb_n)), A, B)
        ks = np.nonzero(tf[HALF:nb - HALF] > THRESHOLD)[0] + HALF
        for k in ks:
            noise_patches.append(tf[k - HALF:k + HALF])
    inj_patches, dismissed = [], 0
    for _ in range(n_inj):
        snr = float(rng.uniform(snr_lo, snr_hi))
        psi, cosi, phi0 = float(rng.uniform(0, math.pi)), float(rng.uniform(-1, 1)), float(rng.uniform(0, 2 * math.pi))
        shift = int(rng.integers(HALF + WIN, nb - HALF - WIN)) - k_sig
        tf = signal_two_f(tr, snr, psi, cosi, phi0, (fa_n[lo + shift:hi + shift], fb_n[lo + shift:hi + shift]))
        c0 = k_sig - lo
        near = tf[c0 - 4:c0 + 5]
        kc = int(np.argmax(near)) + c0 - 4
        if near.max() <= THRESHOLD or kc - HALF < 0 or kc + HALF > tf.shape[0]:
            dismissed += 1
            continue
        inj_patches.append(tf[kc - HALF:kc + HALF])
    info = dict(k_sig=k_sig, alpha=shape["alpha"], delta=shape["delta"])
    return (np.array(inj_patches, dtype=np.float32).reshape(-1, 2 * HALF),
            np.array(noise_patches, dtype=np.float32).reshape(-1, 2 * HALF), dismissed, info)


def make_dataset(seed: int, n_shapes: int, inj_per_shape: int, noise_templates: int,
                 snr_lo: float = 6.0, snr_hi: float = 20.0, workers: int = 0):
    """Balanced set: (patches [n, 256] float32, labels [n] float32, stats).

    Shapes are computed in threads (numpy's FFT and BLAS release the GIL); the
    result does not depend on the number of workers.
    """
    workers = workers or min(16, os.cpu_count() or 1)
    seeds = [seed * 100_003 + i for i in range(n_shapes)]
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(lambda s: shape_patches(s, inj_per_shape, noise_templates, snr_lo, snr_hi), seeds))
    inj = np.concatenate([r[0] for r in res])
    noise = np.concatenate([r[1] for r in res])
    dismissed = sum(r[2] for r in res)
    m = min(len(inj), len(noise))
    rng = np.random.default_rng(seed)
    inj = inj[rng.permutation(len(inj))[:m]]
    noise = noise[rng.permutation(len(noise))[:m]]
    x = np.concatenate([inj, noise])
    y = np.concatenate([np.ones(m, np.float32), np.zeros(m, np.float32)])
    p = rng.permutation(2 * m)
    stats = dict(injections=n_shapes * inj_per_shape, dismissed_by_threshold=dismissed,
                 threshold_false_dismissal=dismissed / max(n_shapes * inj_per_shape, 1), kept_each=m)
    return x[p], y[p], stats

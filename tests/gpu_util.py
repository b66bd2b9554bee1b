"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on the same inputs."""
from __future__ import annotations

import math
import sys

import numpy as np

from oracle import fstat_oracle as ora


def note(msg: str):
    print(f"[gpu-test] {msg}", flush=True)


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


KEY_INT_FIELDS = ["search", "segment", "sky", "fdot_idx", "bin"]


def assert_keys_equal(a, b):
    """Candidate keys equal field by field; unscored vet_score values are NaN on both sides."""
    assert a.shape == b.shape
    for f in KEY_INT_FIELDS:
        np.testing.assert_array_equal(a[f], b[f])
    np.testing.assert_array_equal(np.isnan(a["vet_score"]), np.isnan(b["vet_score"]))
    m = ~np.isnan(a["vet_score"])
    np.testing.assert_array_equal(a["vet_score"][m], b["vet_score"][m])


def make_plan(segments, **opts):
    from paper_1410_3677_amd import fstat as F
    return F.Plan([F.segment_to_device(s) for s in segments], **opts)


def gpu_spectrum(plan, segment, alpha, delta, fdot, nbins, fp64):
    import torch
    dt = torch.float64 if fp64 else torch.float32
    out = torch.empty(len(alpha) * len(fdot) * nbins, dtype=dt, device="cuda")
    plan.twoF_spectrum(segment, dev(alpha), dev(delta), dev(fdot), out)
    torch.cuda.synchronize()
    return out.double().cpu().numpy().reshape(len(alpha), len(fdot), nbins)


def oracle_spectrum(seg, alpha, delta, fdot, nfft, k_min=0, k_max=-1, full=False):
    res = []
    for i in range(len(alpha)):
        sky = ora.sky_stage(seg, float(alpha[i]), float(delta[i]), nfft)
        res.append([ora.template_two_f(seg, sky, float(f), nfft, k_min, k_max, full) for f in fdot])
    return np.array(res)


def rel_err_floor(got, ref, floor=4.0):
    """max |got - ref| / max(ref, floor): relative error with the noise mean as floor."""
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), floor)))


def compare_candidates(keys, twoF, ora_spec, threshold, guard_rel, k_min=0, sky_offset=0):
    """Candidate keys of the GPU vs the oracle's full 2F spectra of the same templates.

    keys: GPU (sky, fdot_idx, bin) rows; ora_spec[i, s, k - k_min] is the oracle's 2F.
    Key sets must be equal except for bins whose oracle 2F lies within
    guard_rel * threshold of the threshold (a legitimate FP32 flip).
    Returns (n_gpu, n_oracle, flips, mismatches, max relative error on common keys).
    """
    g = {(int(a) - sky_offset, int(b), int(c)): float(f) for (a, b, c), f in zip(keys, twoF)}
    idx = np.argwhere(ora_spec > threshold)
    o = {(int(i), int(s_), int(k) + k_min) for i, s_, k in idx}
    band = guard_rel * threshold
    flips, mism = 0, []
    for k in set(g) ^ o:
        i, s_, b = k
        ref = ora_spec[i, s_, b - k_min]
        if abs(ref - threshold) <= band:
            flips += 1
        else:
            mism.append((k, float(ref), g.get(k)))
    err = max([abs(g[k] - ora_spec[k[0], k[1], k[2] - k_min]) / max(ora_spec[k[0], k[1], k[2] - k_min], 4.0)
               for k in set(g) & o], default=0.0)
    return len(g), len(o), flips, mism, err


def per_sky_oracle(seg, alpha, delta, fdot, nfft, check, full=False, workers=None):
    """Call check(i, ref) for every sky i, ref[s, k] being the oracle's 2F of template
    (sky i, spindown s) over all bins, the skies spread over threads (the oracle's FFTs
    and array arithmetic release the interpreter lock); returns the results in sky order.
    Only one sky's spectra per thread are held at a time."""
    import concurrent.futures
    import os

    def one(i):
        sky = ora.sky_stage(seg, float(alpha[i]), float(delta[i]), nfft)
        ref = np.array([ora.template_two_f(seg, sky, float(f), nfft, 0, -1, full) for f in fdot])
        return check(i, ref)
    workers = workers or max(1, min(16, len(os.sched_getaffinity(0))))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(one, range(len(alpha))))

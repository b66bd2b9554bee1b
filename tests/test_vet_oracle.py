"""Pins of the FP64 vetting-network reference and its data generator (CPU only)."""
import math

import numpy as np
import pytest
import scipy.signal

from oracle import vet_data
from oracle import vet_oracle as vo
from tests import pins


def test_parameter_count():
    # 3 conv layers of 32 channels (kernel 7), dense 8192 -> 128 -> 128 -> 1
    assert vo.N_PARAMS == (32 * 7 + 32) + 2 * (32 * 32 * 7 + 32) + (8192 * 128 + 128) + (128 * 128 + 128) + 129
    assert vo.N_PARAMS == 1080001


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((2, 256, 5))
    w = rng.standard_normal((4, 5, 7))
    b = rng.standard_normal(4)
    z = vo.conv_same(a, w, b)
    for n in range(2):
        for c in range(4):
            ref = b[c] + sum(scipy.signal.correlate(a[n, :, ci], w[c, ci], mode="same") for ci in range(5))
            np.testing.assert_allclose(z[n, :, c], ref, rtol=0, atol=1e-12)


def test_bce_matches_direct_formula():
    logit = np.array([-3.0, -0.2, 0.0, 0.7, 4.0])
    y = np.array([0.0, 1.0, 1.0, 0.0, 1.0])
    s = 1 / (1 + np.exp(-logit))
    ref = -np.mean(y * np.log(s) + (1 - y) * np.log(1 - s))
    assert abs(vo.bce_with_logits(logit, y) - ref) < 1e-14


def test_gradient_matches_central_finite_differences():
    rng = np.random.default_rng(1)
    theta = vo.init_params(rng)
    theta += 0.01 * rng.standard_normal(theta.size)          # nonzero biases too
    patches = rng.chisquare(4, size=(3, 256)) * rng.uniform(1, 3, size=(3, 1))
    y = np.array([1.0, 0.0, 1.0])
    _, g = vo.loss_and_grad(theta, patches, y)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in vo.SHAPES])
    idx = np.concatenate([rng.integers(offs[i], offs[i + 1], 6) for i in range(len(vo.SHAPES))])
    h = 1e-6
    worst = 0.0
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (vo.bce_with_logits(vo.forward(tp, patches), y) - vo.bce_with_logits(vo.forward(tm, patches), y)) / (2 * h)
        worst = max(worst, abs(fd - g[i]) / max(abs(g[i]), 1e-4))
    assert worst < 1e-5


def test_flatten_roundtrip():
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(vo.N_PARAMS)
    np.testing.assert_array_equal(vo.flatten(vo.unflatten(theta)), theta)


def test_bf16_rounding():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 1 + 2 ** -7 + 2 ** -9], dtype=np.float32)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    np.testing.assert_array_equal(vo.bf16_round(x), [1.0, 1.0, 1 + 2 ** -6, -2.5, 1 + 2 ** -7])


def test_patch_generator_small():
    x, y, st = vet_data.make_dataset(7, 2, 40, 2, workers=2)
    assert x.shape[1] == 256 and x.shape[0] == y.shape[0] and x.shape[0] > 0
    assert y.sum() == len(y) / 2
    # every patch is centred on a crossing
    assert np.all(x[:, 128] > vet_data.THRESHOLD)
    # injection patches are centred on a local maximum of the window searched
    assert np.all(x[y == 1, 128] >= x[y == 1, 124:133].max(axis=1) - 1e-3)
    assert st["threshold_false_dismissal"] < 0.2


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_signal_assembly_equals_injected_segment(seed):
    # the training and evaluation signals are combinations of basis transforms with the
    # JKS amplitudes; the same source injected into a segment (its own waveform, polarisation
    # and inclination through the antenna patterns) gives the same 2F window at the template
    assert pins.vet_signal_assembly_error(seed) < 1e-9

"""FP64 reference of the candidate-vetting network (TEST INFRASTRUCTURE ONLY).

The network scores a patch of the 2F spectrum around a threshold crossing
(256 bins centred on the crossing bin).  It is not part of the paper's method;
the threshold of Sect. 2 stays the fallback and judges its false dismissals.

Model (the definition both sides implement):
  u[p]   = log(1 + 2F[p]) - log(1 + 4)                    p = 0..255 (0 where the patch
                                                           leaves the searched band: 2F = 0)
  conv_l : z[p, c] = b[c] + sum_{c', t} w[c, c', t] a[p + t - 3, c']   (zero padding, t = 0..6)
           a = relu(z);  channels 1 -> 32 -> 32 -> 32
  flatten: x[p * 32 + c] = a3[p, c]                       (8192 values, position-major)
  dense  : 8192 -> 128 (relu) -> 128 (relu) -> 1          logit; score = sigmoid(logit)
  loss   : mean binary cross-entropy with logits

Parameters as one flat vector in the order w1, b1, w2, b2, w3, b3, w4, b4, w5, b5, w6, b6
with shapes [32,1,7], [32], [32,32,7], [32], [32,32,7], [32], [128,8192], [128],
[128,128], [128], [1,128], [1] (row-major).
"""
from __future__ import annotations

import math

import numpy as np

PATCH = 256
CH = 32
KW = 7
HID = 128
SHAPES = [("w1", (CH, 1, KW)), ("b1", (CH,)), ("w2", (CH, CH, KW)), ("b2", (CH,)),
          ("w3", (CH, CH, KW)), ("b3", (CH,)), ("w4", (HID, PATCH * CH)), ("b4", (HID,)),
          ("w5", (HID, HID)), ("b5", (HID,)), ("w6", (1, HID)), ("b6", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
U_OFFSET = math.log1p(4.0)


def unflatten(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    return out


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(rng: np.random.Generator) -> np.ndarray:
    """He-normal weights, zero biases."""
    parts = []
    for name, shp in SHAPES:
        if name.startswith("b"):
            parts.append(np.zeros(int(np.prod(shp))))
        else:
            fan_in = int(np.prod(shp[1:]))
            parts.append(rng.standard_normal(int(np.prod(shp))) * math.sqrt(2.0 / fan_in))
    return np.concatenate(parts)


def input_transform(patches: np.ndarray) -> np.ndarray:
    return np.log1p(np.asarray(patches, dtype=np.float64)) - U_OFFSET


def conv_same(a: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """a [n, 256, cin], w [cout, cin, 7] -> z [n, 256, cout]; z[p] = b + sum_t w[:, :, t] a[p + t - 3]."""
    n, L, cin = a.shape
    ap = np.zeros((n, L + KW - 1, cin))
    ap[:, 3:3 + L, :] = a
    z = np.broadcast_to(b, (n, L, w.shape[0])).copy()
    for t in range(KW):
        z += ap[:, t:t + L, :] @ w[:, :, t].T
    return z


def forward(theta: np.ndarray, patches: np.ndarray, keep: bool = False):
    p = unflatten(theta)
    u = input_transform(patches)[:, :, None]          # [n, 256, 1]
    z1 = conv_same(u, p["w1"], p["b1"]); a1 = np.maximum(z1, 0)
    z2 = conv_same(a1, p["w2"], p["b2"]); a2 = np.maximum(z2, 0)
    z3 = conv_same(a2, p["w3"], p["b3"]); a3 = np.maximum(z3, 0)
    x = a3.reshape(a3.shape[0], -1)                   # position-major flatten
    z4 = x @ p["w4"].T + p["b4"]; a4 = np.maximum(z4, 0)
    z5 = a4 @ p["w5"].T + p["b5"]; a5 = np.maximum(z5, 0)
    logit = (a5 @ p["w6"].T + p["b6"])[:, 0]
    if keep:
        return logit, dict(u=u, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, a3=a3, x=x, z4=z4, a4=a4, z5=z5, a5=a5)
    return logit


def bce_with_logits(logit: np.ndarray, y: np.ndarray) -> float:
    """mean over the batch of -[y log s + (1 - y) log(1 - s)], s = sigmoid(logit)."""
    return float(np.mean(np.maximum(logit, 0) - logit * y + np.log1p(np.exp(-np.abs(logit)))))


def conv_same_backward(a: np.ndarray, w: np.ndarray, dz: np.ndarray):
    """Gradients of conv_same w.r.t. its input, weights and bias."""
    n, L, cin = a.shape
    ap = np.zeros((n, L + KW - 1, cin))
    ap[:, 3:3 + L, :] = a
    dw = np.zeros_like(w)
    dap = np.zeros_like(ap)
    for t in range(KW):
        # z[:, p, c] += sum_ci w[c, ci, t] ap[:, p + t, ci]
        dw[:, :, t] = np.einsum("npc,npi->ci", dz, ap[:, t:t + L, :])
        dap[:, t:t + L, :] += dz @ w[:, :, t]
    return dap[:, 3:3 + L, :], dw, dz.sum(axis=(0, 1))


def loss_and_grad(theta: np.ndarray, patches: np.ndarray, y: np.ndarray):
    """Mean BCE loss and its gradient with respect to the flat parameter vector."""
    p = unflatten(theta)
    logit, c = forward(theta, patches, keep=True)
    n = logit.shape[0]
    s = 1.0 / (1.0 + np.exp(-logit))
    dlogit = (s - y) / n
    g = {}
    g["w6"] = dlogit[None, :] @ c["a5"]
    g["b6"] = np.array([dlogit.sum()])
    dz5 = (dlogit[:, None] @ p["w6"]) * (c["z5"] > 0)
    g["w5"] = dz5.T @ c["a4"]
    g["b5"] = dz5.sum(0)
    dz4 = (dz5 @ p["w5"]) * (c["z4"] > 0)
    g["w4"] = dz4.T @ c["x"]
    g["b4"] = dz4.sum(0)
    dx = dz4 @ p["w4"]
    dz3 = dx.reshape(c["a3"].shape) * (c["z3"] > 0)
    da2, g["w3"], g["b3"] = conv_same_backward(c["a2"], p["w3"], dz3)
    dz2 = da2 * (c["z2"] > 0)
    da1, g["w2"], g["b2"] = conv_same_backward(c["a1"], p["w2"], dz2)
    dz1 = da1 * (c["z1"] > 0)
    _, g["w1"], g["b1"] = conv_same_backward(c["u"], p["w1"], dz1)
    return bce_with_logits(logit, y), flatten(g)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to bfloat16 (nearest, ties to even) and back to float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)

"""FP64 reference of the learned surrogate (TEST INFRASTRUCTURE ONLY).

A plain NumPy multilayer perceptron with the parameter layout of the HIP
library (layer l: weights (out x in) row-major with padded widths
32, 256, 256, 256, 256 -> 400, then all biases), the erf GELU, and the mean
squared error over the 390 real outputs, with its exact gradient by the
chain rule.  Also the surrogate's targets: the modes 0..64 of
    S = G~,  P = (-(rho~ - rho~') + 2 rho~ sin^2(D/2)) f,  Q = -(z - z') f,
    f = e^{ikR} (ikR - 1) / (4 pi R^3),
(the conormal kernel is K = n'_rho P + n'_z Q, Sec. 3.1) from the oracle's
adaptive azimuthal quadrature, normalised by the phase e^{ik Re R0} and the
amplitude scales the surrogate is defined with (R0 = R at D = 0).

Pins (tests/test_surrogate_oracle.py): the gradient against central finite
differences; the targets of a pair against the oracle's own S and K modes
recombined with the pair's conormal.
"""

from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np
from scipy.special import erf

D = [32, 256, 256, 256, 256, 400]
IN, MODES, OUT = 7, 65, 390


def layout() -> Tuple[List[int], List[int], int]:
    w, b, o = [], [], 0
    for l in range(5):
        w.append(o)
        o += D[l + 1] * D[l]
    for l in range(5):
        b.append(o)
        o += D[l + 1]
    return w, b, o


def unpack(p: np.ndarray):
    w, b, _ = layout()
    Ws = [p[w[l]:w[l] + D[l + 1] * D[l]].reshape(D[l + 1], D[l]) for l in range(5)]
    bs = [p[b[l]:b[l] + D[l + 1]] for l in range(5)]
    return Ws, bs


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def features(x: np.ndarray, rho_max: float) -> np.ndarray:
    """Raw inputs (rho, rho', dz, k, S, Im rho~, Im rho~') -> the network
    input, padded to 32 columns: the first five scaled to O(1), the two
    stretchings, k |R0| / 50 and k (|R(pi)| - |R0|) / 100 with R0, R(pi) the
    complex distance at D = 0 and pi."""
    x = np.asarray(x, dtype=np.float64)
    h = np.zeros((x.shape[0], D[0]))
    h[:, 0] = 2.0 * x[:, 0] / rho_max - 1.0
    h[:, 1] = 2.0 * x[:, 1] / rho_max - 1.0
    h[:, 2] = x[:, 2]
    h[:, 3] = (x[:, 3] - 17.5) / 12.5
    h[:, 4] = (x[:, 4] - 2.5) / 1.5
    h[:, 5] = x[:, 5]
    h[:, 6] = x[:, 6]
    rt = x[:, 0] + 1j * x[:, 5]
    rs = x[:, 1] + 1j * x[:, 6]
    d2 = (rt - rs) ** 2 + x[:, 2] ** 2
    r0 = np.abs(np.sqrt(d2))
    h[:, 7] = x[:, 3] * r0 / 50.0
    h[:, 8] = x[:, 3] * (np.abs(np.sqrt(d2 + 4.0 * rt * rs)) - r0) / 100.0
    return h


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_d(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(p: np.ndarray, x: np.ndarray, rho_max: float, emulate_bf16: bool = False):
    """Outputs [n, 390] and the cache of inputs and pre-activations.  With
    emulate_bf16 the weights, features and hidden activations are rounded to
    BF16 as the MFMA operands are."""
    Ws, bs = unpack(p)
    r = bf16 if emulate_bf16 else (lambda a: a)
    h = r(features(x, rho_max))
    hs, zs = [h], []
    for l in range(5):
        z = h @ r(Ws[l]).T + bs[l]
        zs.append(z)
        if l < 4:
            h = r(gelu(z))
            hs.append(h)
    return zs[-1][:, :OUT], (hs, zs)


def loss_grad(p: np.ndarray, x: np.ndarray, t: np.ndarray, rho_max: float):
    """Mean squared error over the 390 outputs and its gradient (layout of p)."""
    Ws, _ = unpack(p)
    y, (hs, zs) = forward(p, x, rho_max)
    n = x.shape[0]
    d = y - t
    loss = float(np.sum(d * d) / (n * OUT))
    dz = np.zeros((n, D[5]))
    dz[:, :OUT] = 2.0 * d / (n * OUT)
    w, b, tot = layout()
    g = np.zeros(tot)
    for l in range(4, -1, -1):
        g[w[l]:w[l] + D[l + 1] * D[l]] = (dz.T @ hs[l]).ravel()
        g[b[l]:b[l] + D[l + 1]] = dz.sum(axis=0)
        if l > 0:
            dz = (dz @ Ws[l]) * gelu_d(zs[l - 1])
    return loss, g


def norm_scales(rt: complex, rs: complex, dz: float, k: float):
    """Phase e^{ik Re R0} and the S and K scales of one sample:
    a / (4 pi |R0|) and a (|k||R0| + 1)(|R0| + |rho~|) / (4 pi |R0|^3), with
    a the largest |e^{ikR}| over sin^2(D/2) in {0, 1/2, 1} (R0 = R at D = 0)."""
    d2 = (rt - rs) ** 2 + dz * dz + 0j
    c4 = 4 * rt * rs
    R = [np.sqrt(d2 + s * c4) for s in (0.0, 0.5, 1.0)]
    a = math.exp(-k * min(r.imag for r in R))
    r0 = abs(R[0])
    sS = a / (4 * math.pi * r0)
    sK = a * (abs(k) * r0 + 1.0) * (r0 + abs(rt)) / (4 * math.pi * r0 ** 3)
    return np.exp(1j * k * R[0].real), sS, sK


def targets(samples: np.ndarray, modal_fn) -> np.ndarray:
    """Normalised targets [n, 390] of samples [n, 6] (Re, Im rho~, Re, Im
    rho~', dz, k).  modal_fn(tgt, src, k) returns the oracle's [P, 1, 2, 65]
    (S, K) modes for target rows (rho, I, z) and source rows (rho, I, z,
    Re/Im n_rho, Re/Im n_z)."""
    samples = np.asarray(samples, dtype=np.float64)
    out = np.zeros((samples.shape[0], OUT))
    for q, (a, b, c, d, dz, k) in enumerate(samples):
        tgt = np.array([[a, b, dz]])
        srcP = np.array([[c, d, 0.0, 1.0, 0.0, 0.0, 0.0]])
        srcQ = np.array([[c, d, 0.0, 0.0, 0.0, 1.0, 0.0]])
        mP = modal_fn(tgt, srcP, k)[0, 0]
        mQ = modal_fn(tgt, srcQ, k)[0, 0]
        e0, sS, sK = norm_scales(a + 1j * b, c + 1j * d, dz, k)
        for h, (vals, s) in enumerate(((mP[0], sS), (mP[1], sK), (mQ[1], sK))):
            y = vals / (s * e0)
            out[q, h * 130:(h + 1) * 130:2] = y.real
            out[q, h * 130 + 1:(h + 1) * 130:2] = y.imag
    return out

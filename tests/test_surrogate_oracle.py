"""Pins of the FP64 reference of the learned surrogate (CPU only).

The reference network's gradient is checked against central finite
differences, and its targets against the oracle's own modal kernels: the
conormal kernel of any pair must be n'_rho P + n'_z Q (linearity of the
conormal numerator, Sec. 3.1), and the S head must be the oracle's single-
layer modes under the stated normalisation.
"""

import math

import numpy as np

import oracle
import oracle.mlp as mlp
import workloads


def _params(seed=3):
    rng = np.random.default_rng(seed)
    w, b, tot = mlp.layout()
    p = np.zeros(tot)
    for l in range(5):
        fin = 9 if l == 0 else mlp.D[l]
        fout = 390 if l == 4 else mlp.D[l + 1]
        a = math.sqrt(6.0 / (fin + fout))
        W = np.zeros((mlp.D[l + 1], mlp.D[l]))
        W[:fout, :fin] = rng.uniform(-a, a, size=(fout, fin))
        p[w[l]:w[l] + W.size] = W.ravel()
        p[b[l]:b[l] + mlp.D[l + 1]] = rng.normal(scale=0.1, size=mlp.D[l + 1])
    return p


def _batch(n=6, seed=4):
    rng = np.random.default_rng(seed)
    x = np.column_stack([rng.uniform(0.1, 5.4, n), rng.uniform(0.1, 5.4, n), rng.uniform(-1, 1, n),
                         rng.uniform(5, 30, n), rng.uniform(1, 4, n), rng.uniform(0, 1.5, n),
                         rng.uniform(0, 1.5, n)])
    t = rng.normal(size=(n, 390))
    return x, t


def test_reference_gradient_matches_finite_differences():
    p = _params()
    x, t = _batch()
    loss, g = mlp.loss_grad(p, x, t, 5.5)
    w, b, tot = mlp.layout()
    rng = np.random.default_rng(5)
    # weights of every layer (inside the unpadded block) and biases
    idx = []
    for l in range(5):
        fin = 9 if l == 0 else mlp.D[l]
        fout = 390 if l == 4 else mlp.D[l + 1]
        for _ in range(6):
            o, i = rng.integers(fout), rng.integers(fin)
            idx.append(w[l] + o * mlp.D[l] + i)
        idx.append(b[l] + rng.integers(fout))
    h = 1e-6
    for j in idx:
        pp, pm = p.copy(), p.copy()
        pp[j] += h
        pm[j] -= h
        fd = (mlp.loss_grad(pp, x, t, 5.5)[0] - mlp.loss_grad(pm, x, t, 5.5)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])) + 1e-9, (j, fd, g[j])
    # padded columns of the first layer and padded rows of the last get no gradient
    assert np.all(g[w[0]:w[0] + mlp.D[1] * 32].reshape(mlp.D[1], 32)[:, 9:] == 0)
    assert np.all(g[w[4]:w[4] + 400 * 256].reshape(400, 256)[390:] == 0)


def _modal(wl):
    def fn(tgt, src, k):
        return oracle.modal_kernels_points(wl, tgt, src, [k], list(range(65)), oncurve=False)
    return fn


def test_targets_recombine_to_the_conormal_kernel():
    wl = workloads.paper_scale()
    fn = _modal(wl)
    I = lambda r: oracle.core.lib_I(wl, r)  # noqa: E731
    # a pair in the PML and a physical pair (I - I' is the oracle's own profile)
    samples = np.array([[4.9, I(4.9), 4.3, I(4.3), 0.4, 12.0],
                        [1.2, 0.0, 3.3, 0.0, -0.25, 9.0]])
    y = mlp.targets(samples, fn)
    for (a, b, c, d, dz, k), yq in zip(samples, y):
        nr, nz = 0.7 - 0.2j, -0.4 + 0.1j
        tgt = np.array([[a, b, dz]])
        src = np.array([[c, d, 0.0, nr.real, nr.imag, nz.real, nz.imag]])
        ref = fn(tgt, src, k)[0, 0]
        e0, sS, sK = mlp.norm_scales(a + 1j * b, c + 1j * d, dz, k)
        S = sS * e0 * (yq[0:130:2] + 1j * yq[1:130:2])
        P = sK * e0 * (yq[130:260:2] + 1j * yq[131:260:2])
        Q = sK * e0 * (yq[260:390:2] + 1j * yq[261:390:2])
        assert np.max(np.abs(S - ref[0])) <= 1e-12 * np.max(np.abs(ref[0]))
        assert np.max(np.abs(nr * P + nz * Q - ref[1])) <= 1e-12 * np.max(np.abs(ref[1]))


def test_bf16_rounding_is_round_to_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.0e-3])
    r = mlp.bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie to even (mantissa 0)
    assert r[2] == 1.0 + 2 ** -6            # tie to even (rounds up)
    assert r[3] == -2.5
    assert abs(r[4] - 3.0e-3) <= 2 ** -8 * 3.0e-3  # half a unit in the 8th bit

"""Checks of readings of the paper that decide the design (CPU, numpy only).

The split's smooth parts (Sec. 4.1) and the substitution the paper proposes
against their growth in the PML (Sec. 4.3, eq. eqch1): the substitution is
replaced here by a direct azimuthal rule for the pairs it was meant for.
"""

import math

import numpy as np


def _modes(f):
    return np.abs(np.fft.fft(f)) / f.size


def test_ch1_substitution_leaves_a_nonsmooth_remainder():
    """For a close pair (distance d = 1e-2 at rho = rho' = 1, k = 10) the
    split's smooth part sin(kR)/(4 pi R) is entire in R^2, so its azimuthal
    modes fall to rounding by n = 64.  With the substitution of eq. eqch1
    (cH1 = e^{iq} sum_{k <= L} a_k q^k, a_k the Taylor coefficients of
    cos(q) e^{-iq}, L = 5) both parts carry odd powers of R = sqrt(d^2 +
    4 sin^2(D/2)): their modes decay only algebraically (still ~1e-6 at
    n = 64 and ~1e-10 at n = 256), and they are ~1e5 times larger than the
    kernel they add up to, so the sum cancels about five digits.  At the
    modes this build keeps (n <= 128, angle grids of 512) the substitution
    cannot reach the 1e-10 kernel bar; the direct rule takes those pairs."""
    k, d, rho = 10.0, 1e-2, 1.0
    M = 2 ** 15
    D = 2 * np.pi * np.arange(M) / M
    R = np.sqrt(d * d + 4 * rho * rho * np.sin(D / 2) ** 2)
    q = k * R
    smooth = np.sin(q) / (4 * np.pi * R)
    a = [1.0] + [(-2j) ** j / (2 * math.factorial(j)) for j in range(1, 6)]
    ch1 = np.exp(1j * q) * sum(a[j] * q ** j for j in range(6))
    rem = (np.exp(1j * q) - ch1) / (4 * np.pi * R)
    kernel0 = _modes(np.exp(1j * q) / (4 * np.pi * R))[0]
    Fs, Fr, Fc = _modes(smooth), _modes(rem), _modes(ch1)
    # ours: spectral
    assert np.max(Fs[64:M // 2]) <= 1e-15 * Fs[0]
    # the substitution: algebraic decay and large cancelling parts
    assert Fr[64] > 1e-8 and Fc[64] > 1e-8
    assert Fr[256] > 1e-11
    assert Fr[0] > 1e4 * kernel0 and Fc[0] > 1e5 * kernel0

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


def test_ch1_substitution_on_the_pairs_the_direct_class_takes():
    """The same substitution on pairs of the paper-scale workload that the
    graded direct rule takes (both nodes in the PML, |Im k R(pi)| from 6 to
    32, distances 0.07-0.16): the remainder (e^{iq} - cH1)/(4 pi R) keeps
    azimuthal modes between n = 128 and 256 of 0.1 to 30 times the kernel's
    largest mode (the powers q^j, |q| up to ~75, are not smooth at the nearest
    complex singularity of R), so its transform on the 512-point grid of that
    workload aliases at O(1) relative to the kernel, and the cH1 part is 10
    to 5e5 times the kernel it adds up to.  The kernel bar is 1e-10: the
    substitution cannot be the split class for these pairs (the direct rule
    meets the bar on them, tests/test_gpu_parity.py)."""
    import oracle
    import workloads
    wl = workloads.paper_scale()
    g = oracle.geometry(wl)
    rt = g.rho + 1j * g.I
    a = [1.0] + [(-2j) ** j / (2 * math.factorial(j)) for j in range(1, 6)]
    M = 2 ** 15
    s2 = np.sin(np.pi * np.arange(M) / M) ** 2
    worst_alias = np.inf
    for i, l in ((1745, 1809), (1900, 1940), (2015, 2032)):
        assert g.rho[i] > wl.a1 and g.rho[l] > wl.a1 and abs(g.panel_of[i] - g.panel_of[l]) > 1
        d2 = (rt[i] - rt[l]) ** 2 + (g.z[i] - g.z[l]) ** 2
        c4 = 4 * rt[i] * rt[l]
        # the direct class: not far (the aliasing bound fails on the 512-point
        # grid: delta (512 - 128 - B') < 34, delta = |Im D*| of the nearest
        # complex singularity sin^2(D*/2) = -d2 / c4) and growth
        # k_max |Im R(pi)| > 9
        kmax = max(wl.k1, wl.k2)
        delta = abs((2 * np.arcsin(np.sqrt(-d2 / c4 + 0j))).imag)
        bw = 1.1 * kmax * math.sqrt(abs(rt[i] * rt[l]))
        assert delta * (512 - 128 - bw) < 34 and kmax * abs(np.sqrt(d2 + c4).imag) > 9
        R = np.sqrt(d2 + c4 * s2)
        for k in (wl.k1, wl.k2):
            q = k * R
            kern = _modes(np.exp(1j * q) / (4 * np.pi * R))[:129].max()
            ch1 = np.exp(1j * q) * sum(a[j] * q ** j for j in range(6))
            rem = _modes((np.exp(1j * q) - ch1) / (4 * np.pi * R))
            zch1 = _modes(ch1 / (4 * np.pi * R))[0]
            alias = rem[128:257].max() / kern
            print("pair (%d, %d), k = %.0f: remainder modes 128..256 / kernel %.1e, cH1 part / kernel %.1e"
                  % (i, l, k, alias, zch1 / kern))
            worst_alias = min(worst_alias, alias)
            assert zch1 > 5 * kern
    assert worst_alias > 1e-2

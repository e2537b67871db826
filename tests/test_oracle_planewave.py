"""Pins of the oracle's plane-wave data (Sec. 2: the flat-interface reference
field u^{tot,0}, its reflection coefficient R and vertical wavenumber k*, and
the jump data b1, b2 built from it).

Each test checks the oracle against physics that fixes the answer
independently of the formulas it uses:
  - on a flat interface the reference field is the exact solution, so the jump
    data and the solved boundary data vanish (the equal-media test's analogue
    for a plane wave);
  - the reference field solves the Helmholtz equation of each medium, and it
    and its z-derivative are continuous across z = 0 (finite differences);
  - below the interface the transmitted wave carries energy away from it or
    decays away from it (the branch of k*), and energy is conserved;
  - b1 and b2 on a curved interface equal the FFT over the azimuth of the
    jump of the reference field and of its normal derivative, the latter by a
    fourth-order central difference along the 3D normal (nothing shared with
    the Jacobi-Anger and Bessel-derivative formulas the oracle uses).
A planted wrong reflection coefficient and a planted wrong branch of k* are
shown to fail these checks.
"""

import math

import numpy as np
import pytest

import oracle
import workloads

# propagating (k2 > k1 sin phi) and evanescent (total reflection) cases
CASES = [
    (2 * math.pi, 3 * math.pi, 0.0),
    (2 * math.pi, 3 * math.pi, math.pi / 3),
    (2 * math.pi, 3 * math.pi, 1.4),
    (3 * math.pi, 2 * math.pi, 0.4),    # propagating, k2 < k1
    (3 * math.pi, 2 * math.pi, 1.2),    # evanescent: k1 sin phi > k2
    (10.0, 15.0, 1.0),
]


def _flat(k1, k2, **kw):
    return workloads.tiny().with_(bumps=(), k1=k1, k2=k2, **kw)


def _jump_data_on_flat(k1, k2, phi, modes=(0, 1, 3, 8)):
    g = oracle.geometry(_flat(k1, k2))
    b1, b2 = oracle.rhs_plane_wave(g, list(modes), phi)
    scale = 2 * math.pi * max(1.0, abs(k1))
    return float(np.abs(b1).max()) / scale, float(np.abs(b2).max()) / scale


@pytest.mark.parametrize("k1,k2,phi", CASES)
def test_flat_interface_plane_wave_has_zero_jump_data(k1, k2, phi):
    """Flat interface: u^{tot,0} is the exact total field, so b1 = b2 = 0 to
    rounding (b2 vanishes only with the right R for the k* used)."""
    e1, e2 = _jump_data_on_flat(k1, k2, phi)
    assert e1 < 1e-15 and e2 < 1e-14, (e1, e2)


def test_flat_interface_plane_wave_solution_is_zero():
    """Flat interface, whole pipeline: the solved boundary data vanish
    (x = 0 for b = 0), for a propagating and an evanescent incidence."""
    for k1, k2, phi in ((2 * math.pi, 3 * math.pi, math.pi / 3), (3 * math.pi, 2 * math.pi, 1.2)):
        wl = _flat(k1, k2)
        g = oracle.geometry(wl)
        modes = [0, 2]
        b1, b2 = oracle.rhs_plane_wave(g, modes, phi)
        u1, p1, u2, p2, A = oracle.solve(g, modes, b1, b2)
        for x in (u1, p1, u2, p2):
            assert float(np.abs(x).max()) < 1e-13
        # the same operators with the data of a curved interface's source do
        # not give zero: the zero above is not an artefact of the solve
        b1p, b2p = oracle.rhs_point_source(g, modes, 0.0, 1.0)
        u1p = oracle.solve(g, modes, b1p, b2p, A=A)[0]
        assert float(np.abs(u1p).max()) > 1e-3


def _fd(f, x, h):
    """Fourth-order central difference of f at x (f vectorised)."""
    return (-f(x + 2 * h) + 8 * f(x + h) - 8 * f(x - h) + f(x - 2 * h)) / (12 * h)


@pytest.mark.parametrize("k1,k2,phi", CASES)
def test_reference_field_is_continuous_and_solves_helmholtz(k1, k2, phi):
    """The two formulas of u^{tot,0} agree at z = 0 with their z-derivatives
    (transmission conditions of Sec. 2), and each solves the Helmholtz equation
    of its medium (finite-difference Laplacian in x and z)."""
    wl = _flat(k1, k2)
    xs = np.linspace(-1.3, 2.1, 7)
    up0, lo0 = oracle.plane_wave_reference(wl, phi, xs, np.zeros_like(xs))
    assert np.abs(up0 - lo0).max() < 1e-13 * max(1.0, np.abs(up0).max())
    h = 1e-3
    dup = _fd(lambda z: oracle.plane_wave_reference(wl, phi, xs, z + 0 * xs)[0], 0.0, h)
    dlo = _fd(lambda z: oracle.plane_wave_reference(wl, phi, xs, z + 0 * xs)[1], 0.0, h)
    assert np.abs(dup - dlo).max() < 1e-8 * k1 * max(1.0, np.abs(up0).max()), np.abs(dup - dlo).max()
    for med, k in ((0, k1), (1, k2)):
        for z0 in (-0.7, 0.0, 0.45):
            u = lambda x, z: oracle.plane_wave_reference(wl, phi, x, z)[med]
            c = u(xs, z0 + 0 * xs)
            hh = 2e-3
            uxx = (-u(xs + 2 * hh, z0 + 0 * xs) + 16 * u(xs + hh, z0 + 0 * xs) - 30 * c
                   + 16 * u(xs - hh, z0 + 0 * xs) - u(xs - 2 * hh, z0 + 0 * xs)) / (12 * hh * hh)
            uzz = (-u(xs, z0 + 2 * hh + 0 * xs) + 16 * u(xs, z0 + hh + 0 * xs) - 30 * c
                   + 16 * u(xs, z0 - hh + 0 * xs) - u(xs, z0 - 2 * hh + 0 * xs)) / (12 * hh * hh)
            res = np.abs(uxx + uzz + k * k * c).max() / (k * k * max(1.0, np.abs(c).max()))
            assert res < 1e-6, (med, z0, res)


@pytest.mark.parametrize("k1,k2,phi", CASES)
def test_transmitted_wave_leaves_or_decays_and_energy_is_conserved(k1, k2, phi):
    """Below the interface the wave must travel away from it (downward energy
    flux Im(conj(u) du/dz) < 0) or, past the critical angle, decay away from it;
    the vertical energy flux is continuous across z = 0 (energy conservation;
    for total reflection no energy is transmitted and |R| = 1)."""
    wl = _flat(k1, k2)
    x = np.array([0.3])
    h = 1e-3
    lo = lambda z: oracle.plane_wave_reference(wl, phi, x, np.array([z]))[1][0]
    up = lambda z: oracle.plane_wave_reference(wl, phi, x, np.array([z]))[0][0]
    evanescent = k2 <= abs(k1 * math.sin(phi))
    for z0 in (-0.2, -1.0):
        flux = (np.conj(lo(z0)) * _fd(lo, z0, h)).imag
        if evanescent:
            assert abs(lo(z0 - 0.5)) < abs(lo(z0)) * 0.999
            assert abs(flux) < 1e-8 * abs(lo(z0)) ** 2 * k1
        else:
            assert flux < -1e-3 * abs(lo(z0)) ** 2
    # the downward flux of the upper field (incident minus reflected) equals
    # the transmitted one, at any height
    f_up = (np.conj(up(0.37)) * _fd(up, 0.37, h)).imag
    f_lo = (np.conj(lo(-0.61)) * _fd(lo, -0.61, h)).imag
    assert abs(f_up - f_lo) < 1e-7 * k1
    R, kst = oracle.plane_wave_coeffs(k1, k2, phi)
    if evanescent:
        assert abs(abs(R) - 1.0) < 1e-14


def test_curved_interface_data_match_fft_of_reference_field():
    """b1 = -modes of the jump [u^{tot,0}] and b2 = -modes of its normal
    derivative on the curved interface of the small workload (propagating and
    evanescent incidences): azimuthal FFT of samples of the two reference
    formulas, the normal derivative by a fourth-order central difference along
    the 3D unit normal (nu_rho cos th, nu_rho sin th, nu_z)."""
    for k1, k2, phi in ((2 * math.pi, 3 * math.pi, math.pi / 3), (3 * math.pi, 2 * math.pi, 1.2)):
        wl = workloads.tiny().with_(k1=k1, k2=k2)
        g = oracle.geometry(wl)
        modes = [0, 1, 2, 5, 9]
        b1, b2 = oracle.rhs_plane_wave(g, modes, phi)
        Nt = 256
        th = 2 * np.pi * np.arange(Nt) / Nt
        h = 1e-3
        checked = 0
        for i in range(g.n):
            rho, z = g.rho[i], g.z[i]
            nr, nz = g.nu[i]

            def jump(t):
                x = (rho + t * nr) * np.cos(th)
                up, lo = oracle.plane_wave_reference(wl, phi, x, z + t * nz + 0 * th)
                return up - lo

            F1 = np.fft.fft(jump(0.0)) * (2 * np.pi / Nt)
            F2 = np.fft.fft(_fd(jump, 0.0, h)) * (2 * np.pi / Nt)
            sc = 2 * math.pi * k1
            for j, n in enumerate(modes):
                assert abs(-b1[j, i] - F1[n]) <= 1e-12 * sc
                assert abs(-b2[j, i] - F2[n]) <= 1e-8 * sc, (i, n, abs(-b2[j, i] - F2[n]))
            checked += abs(F2[0]) > 1e-3 * sc
        assert checked > 5   # the curve carries nonzero data


def test_planted_wrong_reflection_coefficient_is_caught(monkeypatch):
    """Mutation check: R of the inverse ratio (k1 cos phi / k*), or a flipped
    branch of k* below the critical angle, makes the flat-interface data
    nonzero or the transmitted wave grow away from the interface."""
    real = oracle.core.plane_wave_coeffs

    def wrong_R(k1, k2, phi):
        R, kst = real(k1, k2, phi)
        return complex(2.0 / (1.0 + complex(k1) * math.cos(phi) / kst) - 1.0), kst

    monkeypatch.setattr(oracle.core, "plane_wave_coeffs", wrong_R)
    e1, e2 = _jump_data_on_flat(2 * math.pi, 3 * math.pi, math.pi / 3)
    assert e2 > 1e-3

    def wrong_branch(k1, k2, phi):
        R, kst = real(k1, k2, phi)
        kst = -kst
        return complex(2.0 / (1.0 + kst / (complex(k1) * math.cos(phi))) - 1.0), kst

    monkeypatch.setattr(oracle.core, "plane_wave_coeffs", wrong_branch)
    wl = _flat(3 * math.pi, 2 * math.pi)
    lo = lambda z: oracle.plane_wave_reference(wl, 1.2, np.array([0.3]), np.array([z]))[1][0]
    assert abs(lo(-1.5)) > abs(lo(-1.0))          # grows downward: fails the decay check
    wl = _flat(2 * math.pi, 3 * math.pi)
    lo = lambda z: oracle.plane_wave_reference(wl, 0.4, np.array([0.3]), np.array([z]))[1][0]
    flux = (np.conj(lo(-0.5)) * _fd(lo, -0.5, 1e-3)).imag
    assert flux > 0                                # carries energy upward: fails the outgoing check

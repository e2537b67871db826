"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these tests uses the HIP path.  Each one checks the oracle against an
independent fact: a library special function, a closed form, a brute-force
quadrature, an identity of the boundary-integral formulation, or the exact
solution of a degenerate configuration.
"""

import math

import mpmath
import numpy as np
import pytest
from scipy.special import ellipe

import oracle
import workloads


def _wl(**kw):
    return workloads.tiny().with_(**kw)


def _pair_tables(wl, tgt_rz, src_rz, src_nu=(0.0, -1.0)):
    """Point tables for explicit (rho, z) pairs on or off the curve."""
    tg, sr = [], []
    for (rt, zt), (rs, zs) in zip(tgt_rz, src_rz):
        It = oracle.core.lib_I(wl, rt)
        Is = oracle.core.lib_I(wl, rs)
        sg = oracle.sigma(wl, rs)
        rhot = rs + 1j * Is
        nr = src_nu[0] * rhot / rs
        nz = src_nu[1] * rhot * (1 + 1j * sg) / rs
        tg.append([rt, It, zt])
        sr.append([rs, Is, zs, nr.real, nr.imag, nz.real, nz.imag])
    return np.array(tg), np.array(sr)


# ---------------------------------------------------------------- PML profile

def test_sigma_profile_endpoints_and_flatness():
    """eq. eqsgm1: sigma(a1) = 0, sigma(a1 + T) = S, sigma = S beyond, and the
    derivatives vanish at a1 up to order p - 1 (sigma ~ (rho - a1)^p)."""
    wl = _wl()
    a1, T, S, p = wl.a1, wl.T, wl.S, wl.p
    assert oracle.sigma(wl, a1) == 0.0
    assert oracle.sigma(wl, a1 - 0.3) == 0.0
    assert abs(oracle.sigma(wl, a1 + T) - S) < 1e-15
    assert oracle.sigma(wl, a1 + T + 0.5) == S
    e1, e2 = 1e-2, 5e-3
    r = oracle.sigma(wl, a1 + e1) / oracle.sigma(wl, a1 + e2)
    assert abs(math.log(r) / math.log(e1 / e2) - p) < 0.05


def test_pml_primitive_against_library_quadrature():
    """Im rho~ = int_0^rho sigma_1 (eq. eqrhot) against scipy's QUADPACK."""
    from scipy.integrate import quad
    wl = _wl()
    for rho in (1.0, 2.0, 2.3, 2.77, 3.0):
        ref = quad(lambda x: oracle.sigma(wl, x), 0.0, rho, points=[wl.a1], epsabs=1e-15, epsrel=1e-14, limit=200)[0]
        assert abs(oracle.core.lib_I(wl, rho) - ref) < 1e-13


# ------------------------------------------------------- modal Green's kernels

def test_laplace_modes_match_legendre_q():
    """Laplace limit (k = 0, both points physical): the natural mode of
    1/(4 pi R) is Q_{n-1/2}(chi) / (2 pi sqrt(rho rho')),
    chi = 1 + d^2 / (2 rho rho') (the toroidal-function identity behind the
    semi-analytic modes Z_n of Sec. 4.1)."""
    wl = _wl()
    pairs = [((0.9, 0.2), (1.3, 0.0)), ((0.5, 0.1), (0.52, 0.12)), ((1.7, -0.3), (0.2, 0.4))]
    tg, sr = _pair_tables(wl, [p[0] for p in pairs], [p[1] for p in pairs])
    modes = [0, 1, 4, 9]
    out = oracle.modal_kernels_points(wl, tg, sr, [0.0], modes, oncurve=False)
    for q, ((rt, zt), (rs, zs)) in enumerate(pairs):
        chi = 1 + ((rt - rs) ** 2 + (zt - zs) ** 2) / (2 * rt * rs)
        for j, n in enumerate(modes):
            ref = float(mpmath.legenq(n - 0.5, 0, chi, type=3).real) / (2 * math.pi * math.sqrt(rt * rs))
            assert abs(out[q, 0, 0, j] - ref) <= 1e-13 * abs(ref) + 1e-15


def test_modes_against_brute_force_trapezoid():
    """Well-separated pairs, PML included: the azimuthal integrand is periodic
    and analytic, so a 2^14-point trapezoidal rule is exact to rounding."""
    wl = _wl()
    g = oracle.geometry(wl)
    pairs = np.array([[3, 40], [40, 3], [50, 60], [60, 20], [10, 63]])
    modes = list(range(0, 9))
    ks = [wl.k1, wl.k2]
    out = oracle.modal_kernels_nodes(g, pairs, ks, modes)
    Nt = 1 << 14
    D = 2 * np.pi * np.arange(Nt) / Nt
    s2 = np.sin(D / 2) ** 2
    for q, (i, l) in enumerate(pairs):
        rt, rs = g.rho[i] + 1j * g.I[i], g.rho[l] + 1j * g.I[l]
        drho = (g.rho[i] - g.rho[l]) + 1j * (g.I[i] - g.I[l])
        dz = g.z[i] - g.z[l]
        R = np.sqrt(drho ** 2 + dz ** 2 + 4 * rt * rs * s2)
        num = -(g.nrho[l] * drho + g.nz[l] * dz) + 2 * g.nrho[l] * rt * s2
        for ik, k in enumerate(ks):
            e = np.exp(1j * k * R)
            Gs = e / (4 * np.pi * R)
            Ks = num * e * (1j * k * R - 1) / (4 * np.pi * R ** 3)
            scS = np.max(np.abs(out[q, ik, 0])) + 1e-300
            scK = np.max(np.abs(out[q, ik, 1])) + 1e-300
            for j, n in enumerate(modes):
                refS = (2 * np.pi / Nt) * np.sum(Gs * np.cos(n * D))
                refK = (2 * np.pi / Nt) * np.sum(Ks * np.cos(n * D))
                assert abs(out[q, ik, 0, j] - refS) <= 1e-13 * scS
                assert abs(out[q, ik, 1, j] - refK) <= 1e-13 * scK


def test_near_pair_against_mpmath_quadrature():
    """Close pairs (including one inside the PML), where the integrand is
    sharply peaked at Delta = 0: 30-digit mpmath quadrature of the same
    integral, with the complex distance in its difference form."""
    wl = _wl()
    mpmath.mp.dps = 30
    pairs = [((1.0, 0.05), (1.003, 0.051)), ((2.7, 0.0), (2.705, 0.0)), ((2.9, 0.0), (2.5, 0.0))]
    tg, sr = _pair_tables(wl, [p[0] for p in pairs], [p[1] for p in pairs], src_nu=(0.3, -0.95))
    modes = [0, 3]
    k = wl.k2
    out = oracle.modal_kernels_points(wl, tg, sr, [k], modes, oncurve=False)
    for q in range(len(pairs)):
        rt = mpmath.mpc(tg[q, 0], tg[q, 1])
        rs = mpmath.mpc(sr[q, 0], sr[q, 1])
        drho = mpmath.mpc(tg[q, 0] - sr[q, 0], tg[q, 1] - sr[q, 1])
        dz = mpmath.mpf(tg[q, 2] - sr[q, 2])
        nr = mpmath.mpc(sr[q, 3], sr[q, 4])
        nz = mpmath.mpc(sr[q, 5], sr[q, 6])
        d = abs(complex(drho)) / math.sqrt(abs(complex(rt * rs)))
        pts = [0] + [min(math.pi, d * 2 ** j) for j in range(0, 12) if d * 2 ** j < math.pi] + [mpmath.pi]
        for j, n in enumerate(modes):
            def fS(D):
                s2 = mpmath.sin(D / 2) ** 2
                R = mpmath.sqrt(drho ** 2 + dz ** 2 + 4 * rt * rs * s2)
                return 2 * mpmath.cos(n * D) * mpmath.exp(1j * k * R) / (4 * mpmath.pi * R)

            def fK(D):
                s2 = mpmath.sin(D / 2) ** 2
                R = mpmath.sqrt(drho ** 2 + dz ** 2 + 4 * rt * rs * s2)
                N = -(nr * drho + nz * dz) + 2 * nr * rt * s2
                return 2 * mpmath.cos(n * D) * N * mpmath.exp(1j * k * R) * (1j * k * R - 1) / (4 * mpmath.pi * R ** 3)
            rS = complex(mpmath.quad(fS, pts))
            rK = complex(mpmath.quad(fK, pts))
            assert abs(out[q, 0, 0, j] - rS) <= 1e-12 * abs(rS)
            assert abs(out[q, 0, 1, j] - rK) <= 1e-12 * abs(rK) + 1e-14 * abs(rS)
    mpmath.mp.dps = 15


def test_reciprocity():
    """G~(r, r') = G~(r', r), so the single-layer modes are symmetric in the
    two points, PML points included."""
    wl = _wl()
    g = oracle.geometry(wl)
    pairs = np.array([[2, 30], [33, 50], [45, 61], [20, 47]])
    sw = pairs[:, ::-1].copy()
    a = oracle.modal_kernels_nodes(g, pairs, [wl.k1, wl.k2], [0, 1, 5])
    b = oracle.modal_kernels_nodes(g, sw, [wl.k1, wl.k2], [0, 1, 5])
    sc = np.max(np.abs(a[:, :, 0]))
    assert np.max(np.abs(a[:, :, 0] - b[:, :, 0])) <= 1e-14 * sc


def test_on_axis_source_has_only_mode_zero():
    """A source on the axis sees every azimuth at the same distance, so
    S_n = 2 pi G~ delta_{n0}."""
    wl = _wl()
    tg, sr = _pair_tables(wl, [(1.4, 0.2), (2.6, 0.0)], [(1e-300, 1.0), (1e-300, 1.0)])
    sr[:, 3:] = 0.0
    out = oracle.modal_kernels_points(wl, tg, sr, [wl.k1], [0, 1, 2, 7], oncurve=False)
    for q in range(2):
        rt = tg[q, 0] + 1j * tg[q, 1]
        R = np.sqrt(rt ** 2 + (tg[q, 2] - 1.0) ** 2)
        G = np.exp(1j * wl.k1 * R) / (4 * np.pi * R)
        assert abs(out[q, 0, 0, 0] - 2 * np.pi * G) <= 1e-14 * abs(G)
        assert np.max(np.abs(out[q, 0, 0, 1:])) <= 1e-14 * abs(G)


def test_modal_sum_reconstructs_kernel():
    """(1/2 pi) sum_{|n|<=M} S_n e^{i n D} -> G~(D) for a separated PML pair
    (modes are even in n)."""
    wl = _wl()
    g = oracle.geometry(wl)
    i, l = 5, 55
    M = 40
    out = oracle.modal_kernels_nodes(g, np.array([[i, l]]), [wl.k2], list(range(M + 1)))[0, 0, 0]
    rt, rs = g.rho[i] + 1j * g.I[i], g.rho[l] + 1j * g.I[l]
    drho = (g.rho[i] - g.rho[l]) + 1j * (g.I[i] - g.I[l])
    dz = g.z[i] - g.z[l]
    for D in (0.0, 0.7, 2.0, math.pi):
        R = np.sqrt(drho ** 2 + dz ** 2 + 4 * rt * rs * math.sin(D / 2) ** 2)
        G = np.exp(1j * wl.k2 * R) / (4 * np.pi * R)
        s = (out[0] + 2 * np.sum(out[1:] * np.cos(np.arange(1, M + 1) * D))) / (2 * np.pi)
        assert abs(s - G) <= 1e-12 * abs(out[0]) / (2 * np.pi)


# ------------------------------------------------ Nystrom matrices (near panels)

def test_flat_disk_single_layer_row_sums():
    """Flat interface, k = 0, no PML: 2 int_disk G0 dS' = (2a/pi) E(rho/a)
    (potential of a uniform disk in its own plane); checks the log-singular
    near-panel product integrals of the S block."""
    wl = _wl(bumps=((0.0, 0.0, 1.0),), S=0.0)
    g = oracle.geometry(wl)
    a = wl.a1 + wl.T
    rows = [0, 9, 21, 37, 52, 63]
    S, K = oracle.core.operator_rows(g, rows, [0.0], [0])
    for r, i in enumerate(rows):
        ref = 2 * a / math.pi * ellipe((g.rho[i] / a) ** 2)
        assert abs(S[0, 0, r].sum() - ref) <= 2e-10 * ref
        assert np.max(np.abs(K[0, 0, r])) == 0.0


def _disk_solid_angle(rho, z, a, n=4096):
    ph = 2 * np.pi * np.arange(n) / n
    ell = -rho * np.cos(ph) + np.sqrt(a * a - (rho * np.sin(ph)) ** 2)
    return 2 * np.pi * np.mean(1 - abs(z) / np.sqrt(z * z + ell ** 2))


def test_double_layer_row_sums_solid_angle():
    """k = 0, no PML: 2 int_{Gamma_AB} dG0/dnu' dS' equals the solid-angle
    expression behind Lemmas 3.1-3.3: 1 - Omega_disk/(2 pi) above the plane,
    -1 + Omega_disk/(2 pi) below it and 0 on the flat part, Omega_disk being
    the solid angle of the disk of radius a1 + T through B.  Checks the
    near-panel integrals of the K block and the orientation of nu."""
    wl = _wl(S=0.0)
    g = oracle.geometry(wl)
    a = wl.a1 + wl.T
    rows = [1, 8, 19, 30, 44, 60]
    S, K = oracle.core.operator_rows(g, rows, [0.0], [0])
    for r, i in enumerate(rows):
        z = g.z[i]
        om = _disk_solid_angle(g.rho[i], z, a)
        ref = 0.0 if z == 0 else (1 - om / (2 * np.pi) if z > 0 else -1 + om / (2 * np.pi))
        assert abs(K[0, 0, r].sum() - ref) <= 2e-9


# ------------------------------------------------------- whole-pipeline identities

def test_equal_media_give_no_upper_scattered_field():
    """k1 = k2 with a point source in the upper medium: the exact scattered
    field is 0 above and u_inc below, so u1 -> 0 up to PML truncation, and the
    truncation error decays exponentially as the PML strength S grows
    (Sec. 5, Example 1, the S sweep)."""
    base = _wl()
    modes = [0, 2]
    errs = []
    for S in (1.0, 2.0, 4.0):
        wl = base.with_(k2=base.k1, S=S)
        g = oracle.geometry(wl)
        b1, b2 = oracle.rhs_point_source(g, modes, 0.3, 1.0)
        u1, p1, u2, p2, _ = oracle.solve(g, modes, b1, b2)
        errs.append(max(np.linalg.norm(u1[j]) / np.linalg.norm(b1[j]) for j in range(len(modes))))
        # u2 must reproduce u_inc = -b1 on the curve
        assert np.allclose(u2, u1 - b1)
    assert errs[-1] < 5e-5
    assert errs[0] > errs[1] > errs[2]
    slope = np.polyfit([1.0, 2.0, 4.0], np.log(errs), 1)[0]
    assert slope < -1.0


def test_equal_media_planted_sign_error_is_caught():
    """Planting the wrong sign of the identity term in the oracle makes the
    equal-media identity fail by O(1)."""
    base = _wl()
    wl = base.with_(k2=base.k1, S=4.0)
    g = oracle.geometry(wl)
    modes = [0]
    A, S, K = oracle.assemble(g, modes)
    N = g.n
    A_bad = A.copy()
    A_bad[:, :N, :N] -= 2 * np.eye(N)      # K1 - I instead of K1 + I
    b1, b2 = oracle.rhs_point_source(g, modes, 0.3, 1.0)
    u1, *_ = oracle.solve(g, modes, b1, b2, A=A)
    u1b, *_ = oracle.solve(g, modes, b1, b2, A=A_bad)
    assert np.linalg.norm(u1[0]) / np.linalg.norm(b1[0]) < 1e-4
    assert np.linalg.norm(u1b[0]) / np.linalg.norm(b1[0]) > 0.1


def test_single_medium_explicit_solution():
    """The paper's explicit-solution protocol (Sec. 4.3): u = G~(., r_p) with
    r_p below the interface satisfies the upper-medium boundary integral
    equation (K1 + I) u = S1 (du/dnu_c) up to discretisation and PML
    truncation."""
    wl = _wl(S=4.0)
    g = oracle.geometry(wl)
    N = g.n
    modes = [0, 1, 3]
    rp = (0.5, -1.3)
    A, S, K = oracle.assemble(g, modes)
    tgt = g.tgt_table(np.arange(N))
    src = np.array([[rp[0], 0.0, rp[1], 0, 0, 0, 0]] * N)
    u = oracle.modal_kernels_points(wl, tgt, src, [wl.k1], modes, oncurve=False)[:, 0, 0, :].T
    tg2 = np.array([[rp[0], 0.0, rp[1]]] * N)
    du = oracle.modal_kernels_points(wl, tg2, g.src_table(np.arange(N)), [wl.k1], modes, oncurve=False)[:, 0, 1, :].T
    for j in range(len(modes)):
        res = A[j, :N, :N] @ u[j] - (-A[j, :N, N:]) @ du[j]
        assert np.linalg.norm(res) / np.linalg.norm(u[j]) < 1e-4


def test_plane_wave_modes_match_fft_of_samples():
    """Jacobi-Anger modes of the plane-wave jump data against an FFT of the
    azimuthal samples of exp(-i k1 rho cos(theta) sin(phi)) g(z)."""
    wl = _wl()
    g = oracle.geometry(wl)
    phi = 0.6
    modes = [0, 1, 2, 5]
    b1, b2 = oracle.rhs_plane_wave(g, modes, phi)
    k1 = wl.k1
    c, s = math.cos(phi), math.sin(phi)
    kst = np.sqrt(wl.k2 ** 2 - k1 ** 2 * s ** 2)
    R = 2 / (1 + kst / (k1 * c)) - 1
    Nt = 256
    th = 2 * np.pi * np.arange(Nt) / Nt
    for i in (0, 7, 20, 40):
        z = g.z[i]
        gz = np.exp(-1j * k1 * z * c) + R * np.exp(1j * k1 * z * c) - (1 + R) * np.exp(-1j * kst * z)
        f = np.exp(-1j * k1 * g.rho[i] * np.cos(th) * s) * gz
        F = np.fft.fft(f) * (2 * np.pi / Nt)
        for j, n in enumerate(modes):
            assert abs(-b1[j, i] - F[n]) <= 1e-12 * max(1.0, abs(F[0]))

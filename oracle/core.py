"""Oracle driver: geometry tables, modal kernels, Nystrom matrices, RHS,
per-mode solve and field evaluation (TEST INFRASTRUCTURE ONLY).

Natural modes are used throughout: F_n = int_{-pi}^{pi} e^{-i n D} F(D) dD,
which is sqrt(2 pi) times the paper's normalised mode (Sec. 3.3, eq. fmode3).
The operators of eqs. eqsnpml/eqknpml then read
    (S_n phi)(r) = 2 int_gamma S_n(r, r') phi(r') rho' ds(r')
with the same form for K_n, and the field synthesis is
    u(rho, theta, z) = (1/2 pi) sum_n u_n e^{i n theta}.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pmlbie_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

__all__ = [
    "build_oracle", "lib", "Geometry", "geometry", "modal_kernels_nodes",
    "modal_kernels_points", "near_integrals", "assemble", "rhs_point_source",
    "rhs_plane_wave", "plane_wave_coeffs", "plane_wave_reference", "solve", "field_modes",
    "gl16", "sigma", "num_threads",
]


def build_oracle(force: bool = False) -> str:
    """Compile the oracle's C core with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build_oracle()
        L = ctypes.CDLL(_LIB)
        d, i, P = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        L.or_set_geometry.argtypes = [i, P, d, d, d, d, i, P]
        L.or_point.argtypes = [d, d, P]
        for name in ("or_h", "or_hp", "or_sigma", "or_I"):
            getattr(L, name).argtypes = [d]
            getattr(L, name).restype = d
        for name in ("or_hdiff", "or_Idiff"):
            getattr(L, name).argtypes = [d, d]
            getattr(L, name).restype = d
        L.or_modal_pairs.argtypes = [i, P, P, i, i, P, i, P, P]
        L.or_modal_pairs.restype = i
        L.or_near_panels.argtypes = [i, P, P, i, P, i, P, d, P]
        L.or_near_panels.restype = i
        L.or_set_reltol.argtypes = [d]
        L.or_set_poly.argtypes = [i]
        L.or_num_threads.restype = i
        _lib = L
    return _lib


def num_threads() -> int:
    return lib().or_num_threads()


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def gl16():
    x, w = np.polynomial.legendre.leggauss(16)
    return x, w


# --------------------------------------------------------------------------
# Geometry (Sec. 2, Sec. 3.1) and node tables of the Nystrom discretisation.

@dataclass
class Geometry:
    wl: object                 # the workload
    panels: np.ndarray         # [P, 4] (rho_a, L, z_a, dz): start and extent (z: polylines)
    panel_of: np.ndarray       # [N] panel index of each node
    t: np.ndarray              # [N] panel parameter in [-1, 1]
    rho: np.ndarray
    I: np.ndarray              # Im rho~ = int_0^rho sigma_1
    z: np.ndarray
    hp: np.ndarray
    nu: np.ndarray             # [N, 2] unit normal into the lower medium
    jac: np.ndarray            # |dr/dt|
    nrho: np.ndarray           # conormal components (complex)
    nz: np.ndarray
    sigma: np.ndarray
    w: np.ndarray              # GL weight on [-1, 1]
    W: np.ndarray              # w * rho * |dr/dt|: physical measure rho' ds
    cheb: Optional[np.ndarray] = None  # curved panels: [P, 64] Chebyshev series of rho, z, rho', z'

    @property
    def n(self) -> int:
        return self.rho.size

    def near_panels(self, i: int) -> List[int]:
        p = int(self.panel_of[i])
        return [q for q in (p - 1, p, p + 1) if 0 <= q < len(self.panels)]

    def src_table(self, idx) -> np.ndarray:
        idx = np.asarray(idx)
        return np.stack([self.rho[idx], self.I[idx], self.z[idx], self.nrho[idx].real,
                         self.nrho[idx].imag, self.nz[idx].real, self.nz[idx].imag], axis=1)

    def tgt_table(self, idx) -> np.ndarray:
        idx = np.asarray(idx)
        return np.stack([self.rho[idx], self.I[idx], self.z[idx]], axis=1)


def _set_geometry(wl) -> None:
    L = lib()
    bumps = np.array([c for b in wl.bumps for c in b], dtype=np.float64)
    x, _ = gl16()
    L.or_set_geometry(len(wl.bumps), _p(bumps), float(wl.cos_freq), float(wl.a1),
                      float(wl.T), float(wl.S), int(wl.p), _p(np.ascontiguousarray(x)))
    L.or_set_poly(2 if wl.curve_nodes is not None else (1 if wl.polyline else 0))


def sigma(wl, rho: float) -> float:
    _set_geometry(wl)
    return lib().or_sigma(float(rho))


def polyline_panels(wl) -> np.ndarray:
    """Straight panels of a polyline curve (Sec. 4, graded mesh near corners):
    each segment in equal parts, and at a corner -- an interior vertex where
    the curve turns -- the part touching it cut again at 2^-g, ..., 1/2 of its
    length from the corner.  Returns [P, 4] (rho_a, d rho, z_a, d z)."""
    V = np.asarray(wl.polyline, dtype=np.float64)
    g = int(wl.grade)
    turns = [False] * len(V)
    for j in range(1, len(V) - 1):
        a, b = V[j] - V[j - 1], V[j + 1] - V[j]
        cross = a[0] * b[1] - a[1] * b[0]
        turns[j] = abs(cross) > 1e-12 * np.hypot(*a) * np.hypot(*b) or float(a @ b) < 0.0
    out = []
    for sgi in range(len(V) - 1):
        n = int(wl.panels[sgi])
        cuts = [k / n for k in range(n + 1)]
        if turns[sgi]:
            cuts = [0.0] + [2.0 ** -l / n for l in range(g, 0, -1)] + cuts[1:]
        if turns[sgi + 1]:
            cuts = cuts[:-1] + [1.0 - 2.0 ** -l / n for l in range(1, g + 1)] + [1.0]
        d = V[sgi + 1] - V[sgi]
        for u0, u1 in zip(cuts[:-1], cuts[1:]):
            out.append((V[sgi, 0] + u0 * d[0], (u1 - u0) * d[0], V[sgi, 1] + u0 * d[1], (u1 - u0) * d[1]))
    return np.array(out)


def _polyline_geometry(wl) -> Geometry:
    """Node tables on straight panels: r(t) = start + (1 + t)/2 extent, unit
    normal (z', -rho')/|r'| into the lower medium, conormal of Sec. 3.1."""
    L = lib()
    x, wq = gl16()
    panels = polyline_panels(wl)
    cols = {k: [] for k in ("rho", "I", "z", "nu", "jac", "nr", "nz", "sg", "p", "t", "w")}
    for p, (ra, dr, za, dz) in enumerate(panels):
        ln = math.hypot(dr, dz)
        nu = (dz / ln, -dr / ln)
        for q in range(16):
            u = 0.5 * (1.0 + x[q])
            rho = ra + u * dr
            Iv = L.or_I(rho)
            sg = L.or_sigma(rho)
            rt = rho + 1j * Iv
            cols["rho"].append(rho); cols["I"].append(Iv); cols["z"].append(za + u * dz)
            cols["nu"].append(nu); cols["jac"].append(0.5 * ln)
            cols["nr"].append(nu[0] * rt / rho); cols["nz"].append(nu[1] * rt * (1 + 1j * sg) / rho)
            cols["sg"].append(sg); cols["p"].append(p); cols["t"].append(x[q]); cols["w"].append(wq[q])
    rho = np.array(cols["rho"]); jac = np.array(cols["jac"]); w = np.array(cols["w"])
    return Geometry(
        wl=wl, panels=panels, panel_of=np.array(cols["p"]), t=np.array(cols["t"]), rho=rho,
        I=np.array(cols["I"]), z=np.array(cols["z"]), hp=np.zeros_like(rho), nu=np.array(cols["nu"]),
        jac=jac, nrho=np.array(cols["nr"]), nz=np.array(cols["nz"]), sigma=np.array(cols["sg"]),
        w=w, W=w * rho * jac)


def _curved_geometry(wl) -> Geometry:
    """Node tables of a curve given by its panels: on each panel the curve is
    the degree-15 polynomial through the 16 given nodes, here as Chebyshev
    series (the 16 x 16 Chebyshev-Vandermonde system at the nodes, condition
    number ~3, solved directly) with their derivatives."""
    from numpy.polynomial import chebyshev as C
    L = lib()
    x, wq = gl16()
    nodes = np.asarray(wl.curve_nodes, dtype=np.float64)
    P = nodes.shape[0]
    cheb = np.zeros((P, 64))
    panels = np.zeros((P, 4))
    cols = {k: [] for k in ("rho", "I", "z", "nu", "jac", "nr", "nz", "sg", "p", "t", "w")}
    V = C.chebvander(x, 15)
    for p in range(P):
        cr = np.linalg.solve(V, nodes[p, :, 0])
        cz = np.linalg.solve(V, nodes[p, :, 1])
        dcr, dcz = C.chebder(cr), C.chebder(cz)
        cheb[p, :16], cheb[p, 16:32] = cr, cz
        cheb[p, 32:32 + len(dcr)], cheb[p, 48:48 + len(dcz)] = dcr, dcz
        e = C.chebval(np.array([-1.0, 1.0]), np.stack([cr, cz], axis=1))  # [coordinate, end]
        panels[p] = (e[0, 0], e[0, 1] - e[0, 0], e[1, 0], e[1, 1] - e[1, 0])
        dr, dz = C.chebval(x, dcr), C.chebval(x, dcz)
        for q in range(16):
            rho, zz = nodes[p, q]
            ln = math.hypot(dr[q], dz[q])
            nu = (dz[q] / ln, -dr[q] / ln)
            Iv = L.or_I(rho)
            sg = L.or_sigma(rho)
            rt = rho + 1j * Iv
            cols["rho"].append(rho); cols["I"].append(Iv); cols["z"].append(zz)
            cols["nu"].append(nu); cols["jac"].append(ln)
            cols["nr"].append(nu[0] * rt / rho); cols["nz"].append(nu[1] * rt * (1 + 1j * sg) / rho)
            cols["sg"].append(sg); cols["p"].append(p); cols["t"].append(x[q]); cols["w"].append(wq[q])
    rho = np.array(cols["rho"]); jac = np.array(cols["jac"]); w = np.array(cols["w"])
    return Geometry(
        wl=wl, panels=panels, panel_of=np.array(cols["p"]), t=np.array(cols["t"]), rho=rho,
        I=np.array(cols["I"]), z=np.array(cols["z"]), hp=np.zeros_like(rho), nu=np.array(cols["nu"]),
        jac=jac, nrho=np.array(cols["nr"]), nz=np.array(cols["nz"]), sigma=np.array(cols["sg"]),
        w=w, W=w * rho * jac, cheb=cheb)


def _panel_records(g: Geometry, idx) -> np.ndarray:
    """[len(idx), 68] panel records of the C near-panel integrals."""
    idx = np.asarray(idx, dtype=np.int64)
    rec = np.zeros((len(idx), 68))
    rec[:, :4] = g.panels[idx]
    if g.cheb is not None:
        rec[:, 4:] = g.cheb[idx]
    return np.ascontiguousarray(rec)


def geometry(wl) -> Geometry:
    """Gauss-Legendre node tables: four segments split into equal-rho
    sub-panels of 16 nodes each (graph curves), graded straight panels
    (polylines), or the caller's curved panels."""
    _set_geometry(wl)
    if wl.curve_nodes is not None:
        return _curved_geometry(wl)
    if wl.polyline:
        return _polyline_geometry(wl)
    L = lib()
    x, wq = gl16()
    br = wl.seg_breaks
    panels = []
    for s in range(4):
        a, b = br[s], br[s + 1]
        h = (b - a) / wl.n_sub
        for k in range(wl.n_sub):
            panels.append((a + k * h, h, 0.0, 0.0))
    panels = np.array(panels)
    rows = []
    pof, ts, ws = [], [], []
    buf = np.zeros(12)
    for p, (pa, h, _, _) in enumerate(panels):
        for q in range(16):
            rho = pa + 0.5 * (1.0 + x[q]) * h
            L.or_point(rho, h, _p(buf))
            rows.append(buf.copy())
            pof.append(p); ts.append(x[q]); ws.append(wq[q])
    g = np.array(rows)
    rho = g[:, 0]
    jac = g[:, 6]
    w = np.array(ws)
    return Geometry(
        wl=wl, panels=panels, panel_of=np.array(pof), t=np.array(ts), rho=rho, I=g[:, 1],
        z=g[:, 2], hp=g[:, 3], nu=g[:, 4:6], jac=jac, nrho=g[:, 7] + 1j * g[:, 8],
        nz=g[:, 9] + 1j * g[:, 10], sigma=g[:, 11], w=w, W=w * rho * jac)


# --------------------------------------------------------------------------
# Modal kernels by adaptive azimuthal quadrature (Sec. 3.3, Sec. 4.1).

def _kri(ks: Sequence[complex]) -> np.ndarray:
    return np.array([[complex(k).real, complex(k).imag] for k in ks], dtype=np.float64).ravel()


def modal_kernels_points(wl, tgt: np.ndarray, src: np.ndarray, ks: Sequence[complex],
                         modes: Sequence[int], oncurve: bool = True,
                         reltol: float = 1e-14) -> np.ndarray:
    """Natural modes of G~ and dG~/dnu_c(r') for explicit point pairs.

    tgt: [P, 3] (rho, I, z); src: [P, 7] (rho, I, z, Re/Im n_rho, Re/Im n_z).
    Returns [P, len(ks), 2 (S, K), len(modes)] complex.
    """
    _set_geometry(wl)
    L = lib()
    L.or_set_reltol(reltol)
    tgt = np.ascontiguousarray(tgt, dtype=np.float64)
    src = np.ascontiguousarray(src, dtype=np.float64)
    m = np.ascontiguousarray(np.asarray(modes, dtype=np.int32))
    npairs = tgt.shape[0]
    out = np.zeros((npairs, len(ks), 2, len(m)), dtype=np.complex128)
    if npairs == 0:
        return out
    kri = _kri(ks)
    bad = L.or_modal_pairs(npairs, _p(tgt), _p(src), int(oncurve), len(ks), _p(kri), len(m),
                           _p(m), _p(out))
    if bad:
        raise RuntimeError("oracle: adaptive quadrature budget exhausted on %d pairs" % bad)
    return out


def modal_kernels_nodes(g: Geometry, pairs: np.ndarray, ks: Sequence[complex],
                        modes: Sequence[int], reltol: float = 1e-14) -> np.ndarray:
    """Modal kernels between curve nodes; pairs [P, 2] = (target i, source l)."""
    pairs = np.asarray(pairs, dtype=np.int64)
    # graph curves: z differences from the interface formula without
    # cancellation; polylines: plain coordinate differences
    return modal_kernels_points(g.wl, g.tgt_table(pairs[:, 0]), g.src_table(pairs[:, 1]), ks,
                                modes, oncurve=not (g.wl.polyline or g.cheb is not None),
                                reltol=reltol)


def near_integrals(g: Geometry, targets: Iterable[int], ks: Sequence[complex],
                   modes: Sequence[int], reltol: float = 1e-13) -> Dict[int, Dict[int, np.ndarray]]:
    """Exact product integrals of the near panels (self and neighbours):
    result[i][panel] = [16, len(ks), 2, len(modes)] of
    int_{-1}^{1} F_n(r_i, r(t)) rho(t) |dr/dt| l_l(t) dt.

    On curved panels the tolerance is at least 1e-11: next to a small
    neighbour's end the double-layer numerator n . (r - r') cancels to
    curvature x distance^2 while its rounding stays eps x distance, which
    leaves ~1e-12 relative noise in the integrand that no tighter rule can
    get below."""
    if g.cheb is not None:
        reltol = max(reltol, 1e-11)
    _set_geometry(g.wl)
    L = lib()
    L.or_set_reltol(1e-14)
    jobs = []
    for i in targets:
        p0 = int(g.panel_of[i])
        for p in g.near_panels(i):
            which = 0 if p == p0 else (-1 if p < p0 else 1)
            jobs.append((i, p, which))
    tinfo = np.array([[g.rho[i], g.I[i], g.z[i], g.t[i] if w == 0 else 2.0, w] for i, p, w in jobs],
                     dtype=np.float64)
    pan = _panel_records(g, [p for _, p, _ in jobs])
    m = np.ascontiguousarray(np.asarray(modes, dtype=np.int32))
    out = np.zeros((len(jobs), 16, len(ks), 2, len(m)), dtype=np.complex128)
    kri = _kri(ks)
    bad = L.or_near_panels(len(jobs), _p(tinfo), _p(pan), len(ks), _p(kri),
                           len(m), _p(m), reltol, _p(out))
    if bad:
        raise RuntimeError("oracle: near-panel quadrature budget exhausted on %d jobs" % bad)
    res: Dict[int, Dict[int, np.ndarray]] = {}
    for (i, p, _), o in zip(jobs, out):
        res.setdefault(i, {})[p] = o
    return res


# --------------------------------------------------------------------------
# Nystrom matrices and the coupled per-mode system (Sec. 4.1, Sec. 4.2).

def operator_rows(g: Geometry, rows: Sequence[int], ks: Sequence[complex], modes: Sequence[int],
                  reltol: float = 1e-14, near_reltol: float = 1e-13):
    """Rows of the Nystrom matrices S and K for each wavenumber and mode:
    returns S, K of shape [len(ks), len(modes), len(rows), N].  reltol is the
    azimuthal quadrature's tolerance, near_reltol that of the near-panel
    product integrals in the panel parameter."""
    rows = list(rows)
    N = g.n
    nk, nm = len(ks), len(modes)
    S = np.zeros((nk, nm, len(rows), N), dtype=np.complex128)
    K = np.zeros_like(S)
    far = []
    for r, i in enumerate(rows):
        near = set(g.near_panels(i))
        for l in range(N):
            if int(g.panel_of[l]) not in near:
                far.append((r, i, l))
    far = np.array(far, dtype=np.int64).reshape(-1, 3)
    if far.size:
        kern = modal_kernels_nodes(g, far[:, 1:], ks, modes, reltol)
        W = g.W[far[:, 2]]
        for ik in range(nk):
            S[ik, :, far[:, 0], far[:, 2]] = 2.0 * W[:, None] * kern[:, ik, 0, :]
            K[ik, :, far[:, 0], far[:, 2]] = 2.0 * W[:, None] * kern[:, ik, 1, :]
    near = near_integrals(g, rows, ks, modes, reltol=near_reltol)
    for r, i in enumerate(rows):
        for p, o in near[i].items():
            cols = np.arange(16 * p, 16 * p + 16)
            for ik in range(nk):
                S[ik, :, r, cols] = 2.0 * o[:, ik, 0, :]
                K[ik, :, r, cols] = 2.0 * o[:, ik, 1, :]
    return S, K


def assemble(g: Geometry, modes: Sequence[int], ks: Optional[Sequence[complex]] = None):
    """Per-mode system matrices A_n = [[K1 + I, -S1], [K2 - I, -S2]]
    (identity term -1 in the upper medium, +1 in the lower one)."""
    wl = g.wl
    ks = [wl.k1, wl.k2] if ks is None else list(ks)
    N = g.n
    S, K = operator_rows(g, range(N), ks, modes)
    A = np.zeros((len(modes), 2 * N, 2 * N), dtype=np.complex128)
    I = np.eye(N)
    A[:, :N, :N] = K[0] + I
    A[:, :N, N:] = -S[0]
    A[:, N:, :N] = K[1] - I
    A[:, N:, N:] = -S[1]
    return A, S, K


def rhs_point_source(g: Geometry, modes: Sequence[int], rho_s: float, z_s: float):
    """b1 = -[u_tot0]_n and b2 = -[d u_tot0 / dnu_c]_n on the nodes for a point
    source at (rho_s, 0, z_s) in the upper medium (Sec. 2, Sec. 4.2): the jump
    of the reference field is u_inc(r~) itself."""
    wl = g.wl
    N = g.n
    src_pt = np.array([[rho_s, 0.0, z_s, 0.0, 0.0, 0.0, 0.0]] * N)
    tgt = g.tgt_table(np.arange(N))
    # u_inc modes: target = node, source = r*.
    u = modal_kernels_points(wl, tgt, src_pt, [wl.k1], modes, oncurve=False)[:, 0, 0, :]
    # target-side conormal derivative: by the symmetry of G~ in its two points
    # it equals the source-conormal kernel with the roles of the points swapped.
    tgt2 = np.array([[rho_s, 0.0, z_s]] * N)
    src2 = g.src_table(np.arange(N))
    du = modal_kernels_points(wl, tgt2, src2, [wl.k1], modes, oncurve=False)[:, 0, 1, :]
    return -u.T.copy(), -du.T.copy()


def plane_wave_coeffs(k1: complex, k2: complex, phi_inc: float):
    """Reflection coefficient R and vertical wavenumber k* of the flat-interface
    reference field of a plane wave with polar angle phi_inc (Sec. 2):
    k* = sqrt(k2^2 - k1^2 sin^2 phi) when k2 > |k1 sin phi| (a transmitted
    wave travelling down), i sqrt(k1^2 sin^2 phi - k2^2) otherwise (a wave
    decaying below the interface), and R = 2 / (1 + k* / (k1 cos phi)) - 1."""
    k1, k2 = complex(k1), complex(k2)
    c, s = math.cos(phi_inc), math.sin(phi_inc)
    if k2.real > abs(k1.real * s):
        kst = np.sqrt(k2 ** 2 - k1 ** 2 * s ** 2)
    else:
        kst = 1j * np.sqrt(k1 ** 2 * s ** 2 - k2 ** 2)
    Rc = 2.0 / (1.0 + kst / (k1 * c)) - 1.0
    return complex(Rc), complex(kst)


def plane_wave_reference(wl, phi_inc: float, x, z):
    """The flat-interface reference field u^{tot,0} of Sec. 2 (theta_inc = 0)
    at Cartesian points (x, y, z) (it does not depend on y), both of its
    formulas evaluated at every point: returns (upper, lower) with
    upper = e^{-i k1 (x sin phi + z cos phi)} + R e^{-i k1 (x sin phi - z cos phi)},
    lower = (1 + R) e^{-i k1 x sin phi - i k* z}."""
    k1 = complex(wl.k1)
    Rc, kst = plane_wave_coeffs(wl.k1, wl.k2, phi_inc)
    c, s = math.cos(phi_inc), math.sin(phi_inc)
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    ex = np.exp(-1j * k1 * s * x)
    up = ex * (np.exp(-1j * k1 * c * z) + Rc * np.exp(1j * k1 * c * z))
    lo = ex * (1.0 + Rc) * np.exp(-1j * kst * z)
    return up, lo


def rhs_plane_wave(g: Geometry, modes: Sequence[int], phi_inc: float):
    """b1, b2 for a plane wave (theta_inc = 0): the jump of the reference field
    (Sec. 2) across the curve, [u^{tot,0}] = e^{-i k1 x sin phi} g(z) with
    g(z) = e^{-i k1 z cos phi} + R e^{i k1 z cos phi} - (1 + R) e^{-i k* z},
    and its normal derivative, turned into azimuthal modes by the
    Jacobi-Anger expansion e^{-i a cos theta} = sum_n (-i)^n J_n(a) e^{i n theta}.
    On the flat part of the curve (z = 0, where the PML acts) the jump and its
    normal derivative vanish, so the conormal there is the plain normal."""
    from scipy.special import jv, jvp
    wl = g.wl
    k1 = complex(wl.k1)
    Rc, kst = plane_wave_coeffs(wl.k1, wl.k2, phi_inc)
    c, s = math.cos(phi_inc), math.sin(phi_inc)
    z = g.z
    gz = np.exp(-1j * k1 * z * c) + Rc * np.exp(1j * k1 * z * c) - (1 + Rc) * np.exp(-1j * kst * z)
    gzp = (-1j * k1 * c) * np.exp(-1j * k1 * z * c) + Rc * (1j * k1 * c) * np.exp(1j * k1 * z * c) \
        - (1 + Rc) * (-1j * kst) * np.exp(-1j * kst * z)
    arg = (k1 * s).real * g.rho
    b1 = np.zeros((len(modes), g.n), dtype=np.complex128)
    b2 = np.zeros_like(b1)
    for j, n in enumerate(modes):
        f = 2 * np.pi * (-1j) ** n
        b1[j] = -f * jv(n, arg) * gz
        b2[j] = -(g.nu[:, 0] * f * (k1 * s).real * jvp(n, arg) * gz + g.nu[:, 1] * f * jv(n, arg) * gzp)
    return b1, b2


def solve(g: Geometry, modes: Sequence[int], b1: np.ndarray, b2: np.ndarray, A=None):
    """Solve the coupled per-mode system for x = [u1; phi1] with
    [[K1 + I, -S1], [K2 - I, -S2]] x = [0; (K2 - I) b1 - S2 b2],
    then u2 = u1 - b1 and phi2 = phi1 - b2 (transmission conditions)."""
    N = g.n
    if A is None:
        A, S, K = assemble(g, modes)
    out = []
    for j in range(len(modes)):
        rhs = np.zeros(2 * N, dtype=np.complex128)
        rhs[N:] = A[j, N:, :N] @ b1[j] - (-A[j, N:, N:]) @ b2[j]
        x = np.linalg.solve(A[j], rhs)
        u1, p1 = x[:N], x[N:]
        out.append((u1, p1, u1 - b1[j], p1 - b2[j]))
    u1 = np.array([o[0] for o in out]); p1 = np.array([o[1] for o in out])
    u2 = np.array([o[2] for o in out]); p2 = np.array([o[3] for o in out])
    return u1, p1, u2, p2, A


def field_modes(g: Geometry, modes: Sequence[int], sol, pts: np.ndarray, medium: int):
    """Scattered-field modes at physical points pts [P, 2] (rho, z) by the
    Green representation (Sec. 4.2, eq. eqfujs): + for the upper medium,
    - for the lower one (its outward normal is -nu)."""
    wl = g.wl
    u1, p1, u2, p2 = sol[:4]
    k = wl.k1 if medium == 1 else wl.k2
    u, p = (u1, p1) if medium == 1 else (u2, p2)
    N = g.n
    P = pts.shape[0]
    tgt = np.array([[pts[q, 0], lib_I(wl, pts[q, 0]), pts[q, 1]] for q in range(P) for _ in range(N)])
    src = np.tile(g.src_table(np.arange(N)), (P, 1))
    kern = modal_kernels_points(wl, tgt, src, [k], modes, oncurve=False)[:, 0]
    kern = kern.reshape(P, N, 2, len(modes))
    sgn = 1.0 if medium == 1 else -1.0
    out = np.zeros((len(modes), P), dtype=np.complex128)
    for j in range(len(modes)):
        out[j] = sgn * (kern[:, :, 0, j] @ (g.W * p[j]) - kern[:, :, 1, j] @ (g.W * u[j]))
    return out


def _panel_point(g: Geometry, p: int, t: np.ndarray):
    """(rho, z) of panel p at parameters t (graph: linear in rho; polyline:
    linear along the straight panel)."""
    if g.cheb is not None:
        from numpy.polynomial import chebyshev as C
        return C.chebval(np.asarray(t), g.cheb[p, :16]), C.chebval(np.asarray(t), g.cheb[p, 16:32])
    ra, dr, za, dz = g.panels[p]
    u = 0.5 * (1.0 + np.asarray(t))
    rho = ra + u * dr
    if g.wl.polyline:
        return rho, za + u * dz
    L = lib()
    return rho, np.array([L.or_h(float(x)) for x in np.atleast_1d(rho)])


def field_modes_exact(g: Geometry, modes: Sequence[int], sol, pts: np.ndarray, medium: int,
                      reltol: float = 1e-13):
    """Scattered-field modes at points pts [P, 2] (rho, z) off the curve by the
    Green representation (Sec. 4.2, eq. eqfujs) with the densities of each
    panel interpolated on its 16 nodes and every panel integrated adaptively
    (no fixed rule): exact for the discretised densities at any distance from
    the curve."""
    if g.cheb is not None:
        reltol = max(reltol, 1e-11)   # the rounding floor of curved panels (near_integrals)
    return _field_modes_exact(g, modes, sol, pts, medium, reltol)


def _field_modes_exact(g: Geometry, modes: Sequence[int], sol, pts: np.ndarray, medium: int,
                       reltol: float):
    wl = g.wl
    _set_geometry(wl)
    L = lib()
    L.or_set_reltol(1e-14)
    u1, p1, u2, p2 = sol[:4]
    k = wl.k1 if medium == 1 else wl.k2
    u, p = (u1, p1) if medium == 1 else (u2, p2)
    sgn = 1.0 if medium == 1 else -1.0
    m = np.ascontiguousarray(np.asarray(modes, dtype=np.int32))
    kri = _kri([k])
    P = len(g.panels)
    ts = np.linspace(-1.0, 1.0, 201)
    out = np.zeros((len(modes), pts.shape[0]), dtype=np.complex128)
    for q in range(pts.shape[0]):
        rho_p, z_p = float(pts[q, 0]), float(pts[q, 1])
        I_p = L.or_I(rho_p)
        tinfo, pan = [], []
        for pp in range(P):
            r, z = _panel_point(g, pp, ts)
            tstar = float(ts[int(np.argmin((r - rho_p) ** 2 + (z - z_p) ** 2))])
            tinfo.append([rho_p, I_p, z_p, tstar, 2.0])
        tinfo = np.ascontiguousarray(np.array(tinfo, dtype=np.float64))
        pan = _panel_records(g, range(P))
        res = np.zeros((P, 16, 1, 2, len(m)), dtype=np.complex128)
        bad = L.or_near_panels(P, _p(tinfo), _p(pan), 1, _p(kri), len(m), _p(m), reltol, _p(res))
        if bad:
            raise RuntimeError("oracle: field quadrature budget exhausted on %d panels" % bad)
        IS = res[:, :, 0, 0, :].reshape(P * 16, len(m))
        IK = res[:, :, 0, 1, :].reshape(P * 16, len(m))
        for j in range(len(m)):
            out[j, q] = sgn * (IS[:, j] @ p[j] - IK[:, j] @ u[j])
    return out


def lib_I(wl, rho: float) -> float:
    _set_geometry(wl)
    return lib().or_I(float(rho))

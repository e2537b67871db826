"""Pins of the oracle's polyline curves (corners, graded panels; Sec. 4 and
Sec. 5, Examples 1 and 3) against closed forms, the graph-curve path that the
other pins hold, and the paper's explicit-solution protocol (Sec. 4.3); and of
its exact field near the curve (every panel integrated adaptively) against
the fixed rule far away and the boundary data at the curve.

None of these tests uses the HIP path.
"""

import functools
import math

import numpy as np

import oracle
import workloads


def test_graded_layout_and_tables_closed_forms():
    """Panel layout of the rectangular perturbation: each segment is covered
    exactly, the panels touching the two corners shrink by halves down to
    2^-g of an equal part, and the node tables integrate rho and rho z over
    the curve exactly (16-point rules on straight panels)."""
    g_lv = 3
    wl = workloads.corner(panels=(2, 2, 2, 2), grade=g_lv)
    P = oracle.core.polyline_panels(wl)
    # two corners, each seen from two segments: 4 * g extra panels
    assert len(P) == 8 + 4 * g_lv
    lens = np.hypot(P[:, 1], P[:, 3])
    assert math.isclose(lens.sum(), 1.0 + 1.0 + 1.0 + 2.0, rel_tol=1e-15)
    # the first segment ends at the corner (1, -1): its last panels are
    # 1/2, 1/4, 1/8 and 1/8 of an equal part (0.5), toward the corner
    seg0 = lens[:2 + g_lv]
    assert np.allclose(seg0, [0.5, 0.25, 0.125, 0.0625, 0.0625], rtol=0, atol=1e-15)
    # the flat segment through the PML has no corner: equal panels
    assert np.allclose(lens[-2:], [1.0, 1.0], rtol=0, atol=1e-15)
    g = oracle.geometry(wl)
    # int rho ds = 1/2 + 1 + (4^2 - 1)/2, int rho z ds = -1/2 - 1/2
    assert abs(g.W.sum() - 9.0) <= 1e-13
    assert abs((g.W * g.z).sum() + 1.0) <= 1e-13
    # unit normals, perpendicular to the panels, into the lower medium
    assert np.allclose(np.hypot(g.nu[:, 0], g.nu[:, 1]), 1.0, atol=1e-15)
    tang = P[g.panel_of][:, [1, 3]]
    assert np.max(np.abs(np.sum(tang * g.nu, axis=1))) <= 1e-15
    wall = np.abs(g.rho - 1.0) < 1e-14
    assert wall.sum() == 16 * (2 + 2 * g_lv)
    assert np.allclose(g.nu[wall], [1.0, 0.0])       # the lower medium lies at rho > 1
    bottom = (g.z == -1.0)
    assert np.allclose(g.nu[bottom], [0.0, -1.0])


def test_straight_flat_polyline_reproduces_the_graph_curve():
    """A flat polyline cut at the graph's segment breaks, with no corners, is
    the same curve on the same panels as the flat graph: its operator rows
    (straight-panel near integrals, plain coordinate differences) agree with
    the graph path (interface-formula differences) to rounding."""
    base = workloads.tiny().with_(bumps=(), S=2.0)
    br = base.seg_breaks
    poly = base.with_(polyline=tuple((b, 0.0) for b in br), panels=(base.n_sub,) * 4, grade=3)
    gg, gp = oracle.geometry(base), oracle.geometry(poly)
    assert gg.n == gp.n
    assert np.max(np.abs(gg.rho - gp.rho)) <= 1e-15
    assert np.max(np.abs(gg.W - gp.W)) <= 1e-15
    rows = [0, 17, 30, 41, 63]
    Sg, Kg = oracle.core.operator_rows(gg, rows, [base.k1, base.k2], [0, 3])
    Sp, Kp = oracle.core.operator_rows(gp, rows, [base.k1, base.k2], [0, 3])
    assert np.max(np.abs(Sg - Sp)) <= 1e-12 * np.max(np.abs(Sg))
    assert np.max(np.abs(Kg - Kp)) <= 1e-12 * np.max(np.abs(Kg)) + 1e-15


def _explicit_residual(wl, modes, rows):
    g = oracle.geometry(wl)
    N = g.n
    rp = (0.5, -1.3)
    S, K = oracle.core.operator_rows(g, rows, [wl.k1], modes)
    tgt = g.tgt_table(np.arange(N))
    src = np.array([[rp[0], 0.0, rp[1], 0, 0, 0, 0]] * N)
    u = oracle.modal_kernels_points(wl, tgt, src, [wl.k1], modes, oncurve=False)[:, 0, 0, :].T
    tg2 = np.array([[rp[0], 0.0, rp[1]]] * N)
    du = oracle.modal_kernels_points(wl, tg2, g.src_table(np.arange(N)), [wl.k1], modes,
                                     oncurve=False)[:, 0, 1, :].T
    out = []
    for j in range(len(modes)):
        res = K[0, j] @ u[j] + u[j][rows] - S[0, j] @ du[j]
        out.append(np.max(np.abs(res)) / np.max(np.abs(u[j])))
    return np.array(out), g


def test_corner_explicit_solution():
    """The explicit-solution protocol of Sec. 4.3 on the rectangular
    perturbation (the paper's corner test, r_p = (0.5, 0, -1.3) below the
    curve): u = G~(., r_p) satisfies (K1 + I) u = S1 du/dnu_c on the curve, so
    the Nystrom residual at rows on both corners, the vertical wall and the
    PML stays at the level of the quadrature and PML truncation.  A dropped
    near-panel term, a flipped wall normal or a wrong panel extent gives O(1)."""
    wl = workloads.corner(panels=(2, 2, 2, 2), grade=2, S=4.0)
    g = oracle.geometry(wl)
    # rows: next to the corner (1, -1) on both sides, mid-wall, next to the
    # corner (1, 0) on both sides, the PML
    near_c1 = int(np.argmin(np.hypot(g.rho - 1.0, g.z + 1.0)))
    near_c2 = int(np.argmin(np.hypot(g.rho - 1.0, g.z)))
    rows = sorted({0, near_c1 - 1, near_c1, near_c1 + 1, near_c2 - 1, near_c2, near_c2 + 1,
                   int(np.argmin(np.abs(g.z + 0.5) + np.abs(g.rho - 1.0))), g.n - 5})
    res, _ = _explicit_residual(wl, [0, 1, 3], rows)
    assert np.all(res < 1e-7), res


# ------------------------------------------------- field near the curve

@functools.lru_cache(maxsize=1)
def _tiny_solution():
    wl = workloads.tiny()
    g = oracle.geometry(wl)
    modes = list(range(wl.m_max + 1))
    b1, b2 = oracle.rhs_point_source(g, modes, 0.3, 1.0)
    return g, modes, oracle.solve(g, modes, b1, b2)


def test_exact_field_matches_the_fixed_rule_far_from_the_curve():
    """Away from the curve the 16-point panel rule is exact to rounding, so
    the oracle's adaptive product integration of every panel must agree with
    the plain node sum there (both media)."""
    g, modes, sol = _tiny_solution()
    for pt, med in (([0.5, 1.4], 1), ([1.2, -0.9], 2)):
        pts = np.array([pt])
        fe = oracle.core.field_modes_exact(g, modes, sol, pts, med)
        ff = oracle.field_modes(g, modes, sol, pts, med)
        assert np.max(np.abs(fe - ff)) <= 1e-11 * np.max(np.abs(ff))


def test_exact_field_tends_to_the_boundary_data():
    """Green's representation reproduces the field up to the boundary: at a
    distance d from a node, on the side of either medium, the field modes
    differ from that medium's boundary data (u1 above, u2 below) by O(d),
    i.e. the double-layer jump is captured exactly; a missing or doubled jump
    leaves an O(1) difference."""
    g, modes, sol = _tiny_solution()
    for l in (20, 37):
        nu = g.nu[l]
        errs = {}
        for d in (1e-3, 1e-4):
            up = np.array([[g.rho[l] - d * nu[0], g.z[l] - d * nu[1]]])
            lo = np.array([[g.rho[l] + d * nu[0], g.z[l] + d * nu[1]]])
            fu = oracle.core.field_modes_exact(g, modes, sol, up, 1)[:, 0]
            fl = oracle.core.field_modes_exact(g, modes, sol, lo, 2)[:, 0]
            eu = np.max(np.abs(fu - sol[0][:, l])) / np.max(np.abs(sol[0][:, l]))
            el = np.max(np.abs(fl - sol[2][:, l])) / np.max(np.abs(sol[2][:, l]))
            errs[d] = (eu, el)
            assert eu < 100 * d and el < 100 * d, (l, d, eu, el)
        # first order in d
        for a, b in zip(errs[1e-3], errs[1e-4]):
            assert 5.0 < a / b < 20.0


# ------------------------------------------------- curves given by their panels

def _nodes_of(g):
    return np.stack([g.rho, g.z], axis=1).reshape(-1, 16, 2)


def test_curved_panels_through_straight_nodes_reproduce_the_polyline():
    """The rectangular perturbation handed over as curved panels (its node
    coordinates only): the degree-15 interpolants are the straight panels, so
    node tables and operator rows (near-panel integrals with divided-difference
    offsets) match the polyline path to rounding."""
    wl = workloads.corner(panels=(2, 2, 2, 2), grade=2)
    gp = oracle.geometry(wl)
    gc = oracle.geometry(wl.with_(polyline=(), panels=(), grade=0, curve_nodes=_nodes_of(gp)))
    assert np.max(np.abs(gc.W - gp.W)) <= 1e-14
    assert np.max(np.abs(gc.nu - gp.nu)) <= 1e-14
    rows = [3, 40, 63, 64, 100, 150, gp.n - 2]
    Sp, Kp = oracle.core.operator_rows(gp, rows, [wl.k1, wl.k2], [0, 2])
    Sc, Kc = oracle.core.operator_rows(gc, rows, [wl.k1, wl.k2], [0, 2])
    assert np.max(np.abs(Sc - Sp)) <= 1e-12 * np.max(np.abs(Sp))
    assert np.max(np.abs(Kc - Kp)) <= 1e-12 * np.max(np.abs(Kp))


def test_curved_quarter_circle_closed_forms():
    """A quarter circle of radius 1 from (0, -1) to (1, 0) on curved panels,
    then flat to 4: int rho ds = 1 + 15/2 and int rho z ds = -1/2 to the
    interpolation accuracy, normals radial (into the lower medium)."""
    x, _ = np.polynomial.legendre.leggauss(16)
    pans = []
    for k in range(8):
        phi = (k + 0.5 * (1 + x)) * (np.pi / 2) / 8
        pans.append(np.stack([np.sin(phi), -np.cos(phi)], axis=1))
    for lo, hi in ((1.0, 1.5), (1.5, 2.0), (2.0, 3.0), (3.0, 4.0)):
        r = lo + 0.5 * (1 + x) * (hi - lo)
        pans.append(np.stack([r, np.zeros_like(r)], axis=1))
    wl = workloads.corner().with_(polyline=(), panels=(), grade=0, curve_nodes=np.array(pans))
    g = oracle.geometry(wl)
    assert abs(g.W.sum() - 8.5) <= 1e-13
    assert abs((g.W * g.z).sum() + 0.5) <= 1e-13
    arc = g.panel_of < 8
    radial = np.stack([g.rho[arc], g.z[arc]], axis=1)
    assert np.max(np.abs(g.nu[arc] - radial)) <= 1e-13


def test_rippled_bowl_explicit_solution():
    """The explicit-solution protocol of Sec. 4.3 on the curve of Sec. 5,
    Example 2 (curved panels, graded toward the corner where the bowl meets
    the flat part): rows near the axis, on the ripples, at the corner and in
    the PML."""
    wl = workloads.bowl().with_(S=4.0)
    g = oracle.geometry(wl)
    c = int(np.argmin(np.hypot(g.rho - 1.0, g.z)))
    rows = sorted({0, 40, 100, 170, c - 1, c, c + 1, g.n - 5})
    res, _ = _explicit_residual(wl, [0, 1, 3], rows)
    assert np.all(res < 1e-6), res

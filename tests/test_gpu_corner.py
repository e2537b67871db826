"""Parity of the HIP path against the FP64 oracle on polyline curves with
corners and graded panels (Sec. 4, graded mesh; Sec. 5, Example 1: the
rectangular perturbation of depth and radius 1).

Same bars as the graph curves: assembled matrices within 1e-10 normwise per
mode and block, boundary data within 1e-8 per mode and right-hand side.
Every call goes through the C ABI.
"""

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KERNEL_TOL = 1e-10
BOUNDARY_TOL = 1e-8


def _solver(wl, **kw):
    from paper_2412_11162_amd.solver import from_workload
    return from_workload(wl, **kw)


def _normwise(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def _boundary_err(gpu, ref):
    x_g = np.concatenate(gpu, axis=1)
    x_r = np.concatenate(ref, axis=1)
    big = np.max(np.linalg.norm(x_r, axis=1))
    errs = []
    for j in range(x_r.shape[0]):
        nr = np.linalg.norm(x_r[j])
        d = np.linalg.norm(x_g[j] - x_r[j])
        errs.append(d / nr if nr > 1e-9 * big else d / big)
    return np.array(errs)


@pytest.fixture(scope="module")
def corner_ref():
    import oracle
    wl = workloads.corner()          # 12 panels (one halving at each corner), 192 nodes
    g = oracle.geometry(wl)
    modes = list(range(wl.m_max + 1))
    A, S, K = oracle.assemble(g, modes)
    return wl, g, A, modes


def test_corner_node_table_matches_oracle_geometry(corner_ref):
    wl, g, _, _ = corner_ref
    s = _solver(wl, build=False)
    nd = s.nodes()
    assert nd.shape[0] == g.n == 192
    assert np.max(np.abs(nd[:, 0] - g.rho)) <= 1e-15
    assert np.max(np.abs(nd[:, 1] - g.I)) <= 1e-14
    assert np.max(np.abs(nd[:, 2] - g.z)) <= 1e-15
    assert np.max(np.abs(nd[:, 7] - g.W)) <= 1e-14
    assert np.array_equal(nd[:, 8].astype(int), g.panel_of)
    assert np.max(np.abs(nd[:, 10] - g.nu[:, 0])) <= 1e-15
    assert np.max(np.abs(nd[:, 11] - g.nu[:, 1])) <= 1e-15


def test_corner_operators_all_modes(corner_ref):
    wl, g, A, modes = corner_ref
    from paper_2412_11162_amd._binding import PMLBIE_KEEP_OPERATORS
    s = _solver(wl, flags=PMLBIE_KEEP_OPERATORS)
    N = g.n
    for n in modes:
        G = s.get_operator(n).cpu().numpy()
        for bi in range(2):
            for bj in range(2):
                blk = (slice(bi * N, (bi + 1) * N), slice(bj * N, (bj + 1) * N))
                assert _normwise(G[blk], A[n][blk]) <= KERNEL_TOL, (n, bi, bj)


def test_corner_boundary_data_point_and_plane(corner_ref):
    """A point source on the axis and a plane wave in one solve."""
    import oracle
    wl, g, A, modes = corner_ref
    incs = [("point", 0.0, 1.0), ("plane", 0.5)]
    s = _solver(wl)
    out = s.solve_modes(incs)
    for r, inc in enumerate(incs):
        if inc[0] == "plane":
            b1, b2 = oracle.rhs_plane_wave(g, modes, inc[1])
        else:
            b1, b2 = oracle.rhs_point_source(g, modes, inc[1], inc[2])
        ref = oracle.solve(g, modes, b1, b2, A=A)[:4]
        got = [o[:, r, :].cpu().numpy() for o in out]
        errs = _boundary_err(got, ref)
        assert np.max(errs) <= BOUNDARY_TOL, (inc, errs)


def test_corner_field_inside_and_below_the_perturbation(corner_ref):
    """Field synthesis at points inside the rectangular cavity (upper medium
    below z = 0), beside its wall in the lower medium, and above the flat
    part: the library decides the medium from the polyline itself."""
    import oracle
    wl, g, A, modes = corner_ref
    b1, b2 = oracle.rhs_point_source(g, modes, 0.0, 1.0)
    sol = oracle.solve(g, modes, b1, b2, A=A)
    pts = np.array([[0.5, -0.5], [1.4, -0.5], [0.3, 0.8], [1.6, -1.2]])
    med = [1, 2, 1, 2]
    theta = np.array([0.0, 0.9, 2.1, 0.4])
    ref = np.zeros(len(pts), dtype=complex)
    for q in range(len(pts)):
        fm = oracle.field_modes(g, modes, sol, pts[q:q + 1], med[q])[:, 0]
        ref[q] = (fm[0] + 2 * np.sum(fm[1:] * np.cos(np.arange(1, len(modes)) * theta[q]))) / (2 * np.pi)
    s = _solver(wl)
    s.solve_modes([("point", 0.0, 1.0)])
    out = s.evaluate_field(np.stack([pts[:, 0], theta, pts[:, 1]], axis=1), 1)[0]
    assert np.max(np.abs(out - ref)) <= 1e-8 * np.max(np.abs(ref))


def test_mixed_precision_on_graded_corners(corner_ref):
    """complex64 LU with FP64 refinement on the graded rectangular
    perturbation (a worse-conditioned system than the smooth curves): the
    boundary data meet the mixed-precision bar (1e-6) against the oracle's
    FP64 solve, and the refinement converges to a residual of 1e-10."""
    import oracle
    from paper_2412_11162_amd._binding import PMLBIE_MIXED
    wl, g, A, modes = corner_ref
    b1, b2 = oracle.rhs_point_source(g, modes, 0.0, 1.0)
    ref = oracle.solve(g, modes, b1, b2, A=A)[:4]
    s = _solver(wl, precision=PMLBIE_MIXED)
    out = [o[:, 0, :].cpu().numpy() for o in s.solve_modes([("point", 0.0, 1.0)])]
    errs = _boundary_err(out, ref)
    assert np.max(errs) <= 1e-6, errs
    st, cnt = s.stats()
    assert 1 <= cnt[0] <= 30 and cnt[1] <= 1e-10


def test_deeply_graded_corner_rows_and_solution():
    """Six halvings at each corner (panels down to 1/256 of the segment
    length): oracle operator rows on both sides of both corners, on the wall
    and in the PML against the GPU matrices, and the GPU solution's backward
    error against those exact rows."""
    import oracle
    from paper_2412_11162_amd._binding import PMLBIE_KEEP_OPERATORS
    wl = workloads.corner(panels=(4, 4, 4, 4), grade=6, m_max_=4, n_theta=32)
    g = oracle.geometry(wl)
    N = g.n
    assert N == 16 * (16 + 4 * 6)
    c1 = int(np.argmin(np.hypot(g.rho - 1.0, g.z + 1.0)))
    c2 = int(np.argmin(np.hypot(g.rho - 1.0, g.z)))
    rows = sorted({c1 - 1, c1, c1 + 1, c2 - 1, c2, c2 + 1, 5, N // 2, N - 3})
    modes = [0, 1, 4]
    S, K = oracle.core.operator_rows(g, rows, [wl.k1, wl.k2], modes)
    s = _solver(wl, flags=PMLBIE_KEEP_OPERATORS)
    for j, n in enumerate(modes):
        G = s.get_operator(n).cpu().numpy()
        for ik, (sgn, off) in enumerate(((1.0, 0), (-1.0, N))):
            Kr = G[[off + r for r in rows], :N] - sgn * np.eye(N)[rows]
            Sr = -G[[off + r for r in rows], N:]
            assert _normwise(Kr, K[ik, j]) <= KERNEL_TOL, (n, ik, "K")
            assert _normwise(Sr, S[ik, j]) <= KERNEL_TOL, (n, ik, "S")
    b1, b2 = oracle.rhs_point_source(g, modes, 0.0, 1.0)
    out = [o[:, 0, :].cpu().numpy() for o in s.solve_modes([("point", 0.0, 1.0)])]
    # componentwise backward error of the oracle's rows of
    # [[K1 + I, -S1], [K2 - I, -S2]] x = [0; (K2 - I) b1 - S2 b2] at the GPU
    # solution, each measured against at least 1e-6 of the largest scale
    res, den = [], []
    for j, n in enumerate(modes):
        x1, x2 = out[0][n], out[1][n]
        for q, i in enumerate(rows):
            res.append(abs(K[0, j][q] @ x1 + x1[i] - S[0, j][q] @ x2))
            den.append(np.abs(K[0, j][q]) @ np.abs(x1) + abs(x1[i]) + np.abs(S[0, j][q]) @ np.abs(x2))
            lo = K[1, j][q] @ x1 - x1[i] - S[1, j][q] @ x2
            rhs = K[1, j][q] @ b1[j] - b1[j][i] - S[1, j][q] @ b2[j]
            res.append(abs(lo - rhs))
            den.append(np.abs(K[1, j][q]) @ (np.abs(x1) + np.abs(b1[j])) + abs(x1[i]) + abs(b1[j][i])
                       + np.abs(S[1, j][q]) @ (np.abs(x2) + np.abs(b2[j])))
    res, den = np.array(res), np.array(den)
    errs = res / np.maximum(den, 1e-6 * den.max())
    assert np.max(errs) <= BOUNDARY_TOL, errs


def test_polyline_argument_errors():
    from paper_2412_11162_amd.solver import Solver, PmlbieError
    wl = workloads.corner()
    s = Solver(0)
    bad = [
        (((0.5, -1.0), (1.0, -1.0), (4.0, 0.0)), (2, 2), 1),       # does not start on the axis
        (((0.0, -1.0), (1.0, -1.0), (1.0, -1.0), (4.0, 0.0)), (2, 2, 2), 0),  # repeated vertex
        (((0.0, -1.0), (4.0, 0.0)), (1,), 0),                         # one panel on a segment
        (wl.polyline, wl.panels, 25),                                 # grade too deep
        (wl.polyline, (2, 2, 2, 3), 1),                               # 13 panels: not a multiple of 4
    ]
    for v, p, gr in bad:
        with pytest.raises(PmlbieError) as e:
            s.set_polyline(v, p, gr)
        assert e.value.code == -1, (v, p, gr)
    # not flat beyond the PML start, and no vertex at a1 (no grading: the
    # first curve turns at three vertices)
    for v in (((0.0, -1.0), (1.0, -1.0), (1.0, 0.0), (2.0, 0.0), (4.0, 0.1)),
              ((0.0, -1.0), (1.0, -1.0), (1.0, 0.0), (3.0, 0.0), (4.0, 0.0))):
        s.set_polyline(v, wl.panels, 0)
        with pytest.raises(PmlbieError) as e:
            s.set_media_pml(wl.k1, wl.k2, wl.a1, wl.T, wl.S, wl.a2, wl.T2, wl.S2)
        assert e.value.code == -1
    s.set_polyline(wl.polyline, wl.panels, wl.grade)
    s.set_media_pml(wl.k1, wl.k2, wl.a1, wl.T, wl.S, wl.a2, wl.T2, wl.S2)
    s.build_modal_operators(wl.n_theta, wl.m_max)
    with pytest.raises(PmlbieError):
        s.solve_modes([("point", 0.5, -1.5)])   # below the cavity floor: lower medium
    s.solve_modes([("point", 0.5, -0.5)])       # inside the cavity: upper medium


def test_stepped_perturbation_rows_and_solution():
    """The stepped curve of Sec. 5, Example 3: six corners, a segment that
    runs back toward the axis and two vertical walls.  Oracle operator rows
    next to every corner and on the backward segment against the GPU
    matrices, the GPU solution's componentwise backward error against those
    rows, and the medium of field points inside the steps."""
    import oracle
    from paper_2412_11162_amd._binding import PMLBIE_KEEP_OPERATORS
    wl = workloads.stepped().with_(m_max_=4)
    g = oracle.geometry(wl)
    N = g.n
    assert N == 448
    rows = set()
    for v in wl.polyline[1:7]:
        c = int(np.argmin(np.hypot(g.rho - v[0], g.z - v[1])))
        rows.update({c - 1, c, c + 1})
    back = np.nonzero((np.abs(g.z + 0.7) < 1e-14) & (g.rho < 0.5))[0]
    rows.update({int(back[3]), int(back[-4]), 3, N - 3})
    rows = sorted(r for r in rows if 0 <= r < N)
    modes = [0, 2, 4]
    S, K = oracle.core.operator_rows(g, rows, [wl.k1, wl.k2], modes)
    s = _solver(wl, flags=PMLBIE_KEEP_OPERATORS)
    for j, n in enumerate(modes):
        G = s.get_operator(n).cpu().numpy()
        for ik, (sgn, off) in enumerate(((1.0, 0), (-1.0, N))):
            Kr = G[[off + r for r in rows], :N] - sgn * np.eye(N)[rows]
            Sr = -G[[off + r for r in rows], N:]
            assert _normwise(Kr, K[ik, j]) <= KERNEL_TOL, (n, ik, "K")
            assert _normwise(Sr, S[ik, j]) <= KERNEL_TOL, (n, ik, "S")
    b1, b2 = oracle.rhs_point_source(g, modes, 0.0, 1.0)
    out = [o[:, 0, :].cpu().numpy() for o in s.solve_modes([("point", 0.0, 1.0)])]
    res, den = [], []
    for j, n in enumerate(modes):
        x1, x2 = out[0][n], out[1][n]
        for q, i in enumerate(rows):
            res.append(abs(K[0, j][q] @ x1 + x1[i] - S[0, j][q] @ x2))
            den.append(np.abs(K[0, j][q]) @ np.abs(x1) + abs(x1[i]) + np.abs(S[0, j][q]) @ np.abs(x2))
            lo = K[1, j][q] @ x1 - x1[i] - S[1, j][q] @ x2
            rhs = K[1, j][q] @ b1[j] - b1[j][i] - S[1, j][q] @ b2[j]
            res.append(abs(lo - rhs))
            den.append(np.abs(K[1, j][q]) @ (np.abs(x1) + np.abs(b1[j])) + abs(x1[i]) + abs(b1[j][i])
                       + np.abs(S[1, j][q]) @ (np.abs(x2) + np.abs(b2[j])))
    res, den = np.array(res), np.array(den)
    errs = res / np.maximum(den, 1e-6 * den.max())
    assert np.max(errs) <= BOUNDARY_TOL, errs
    # the pocket under the overhang (0.25 < rho < 0.5, -0.7 < z < -0.5) is
    # lower medium; inside the steps above the overhang and in the lower step
    # it is upper medium: a source there is accepted, one in the pocket is not
    from paper_2412_11162_amd.solver import PmlbieError
    s.solve_modes([("point", 0.4, -0.6 + 0.15)])     # above the overhang: upper
    s.solve_modes([("point", 0.6, -0.9)])            # inside the lower step: upper
    with pytest.raises(PmlbieError):
        s.solve_modes([("point", 0.4, -0.6)])        # in the pocket: lower medium


def _field_ref(g, modes, sol, pts, med, theta):
    import oracle
    ref = np.zeros(len(pts), dtype=complex)
    for q in range(len(pts)):
        fm = oracle.core.field_modes_exact(g, modes, sol, pts[q:q + 1], med[q])[:, 0]
        ref[q] = (fm[0] + 2 * np.sum(fm[1:] * np.cos(np.arange(1, len(modes)) * theta[q]))) / (2 * np.pi)
    return ref


def test_field_near_the_curve_graph_and_corners(corner_ref):
    """Field points closer to the curve than a panel length, where the
    panel rule fails: the library integrates the nearby panels on auxiliary
    points graded toward the closest curve point; the oracle integrates
    every panel adaptively.  Graph curve (tiny workload, panels of length
    about 1) at distances 0.02 to 0.6, and the rectangular cavity next to both
    corners, both media."""
    import oracle
    wl = workloads.tiny()
    g = oracle.geometry(wl)
    modes = list(range(wl.m_max + 1))
    b1, b2 = oracle.rhs_point_source(g, modes, 0.3, 1.0)
    sol = oracle.solve(g, modes, b1, b2)
    pts, med = [], []
    assert g.rho[31] < wl.a1    # nodes 0..31 lie in the physical region
    for l, d in ((5, 0.02), (12, 0.05), (20, 0.1), (25, 0.3), (29, 0.6)):
        nu = g.nu[l]
        pts.append([g.rho[l] - d * nu[0], g.z[l] - d * nu[1]]); med.append(1)
        pts.append([g.rho[l] + d * nu[0], g.z[l] + d * nu[1]]); med.append(2)
    pts = np.array(pts)
    theta = np.linspace(0.0, 2.5, len(pts))
    ref = _field_ref(g, modes, sol, pts, med, theta)
    s = _solver(wl)
    s.solve_modes([("point", 0.3, 1.0)])
    out = s.evaluate_field(np.stack([pts[:, 0], theta, pts[:, 1]], axis=1), 1)[0]
    assert np.max(np.abs(out - ref)) <= 1e-8 * np.max(np.abs(ref)), np.abs(out - ref) / np.max(np.abs(ref))

    wl, g, A, modes = corner_ref
    b1, b2 = oracle.rhs_point_source(g, modes, 0.0, 1.0)
    sol = oracle.solve(g, modes, b1, b2, A=A)
    pts = np.array([[0.98, -0.98], [1.03, -0.5], [0.5, -0.95], [1.5, 0.04], [1.5, -0.04], [0.97, -0.02],
                    [1.02, -1.02]])
    med = [1, 2, 1, 1, 2, 1, 2]
    theta = np.linspace(0.3, 2.0, len(pts))
    ref = _field_ref(g, modes, sol, pts, med, theta)
    s = _solver(wl)
    s.solve_modes([("point", 0.0, 1.0)])
    out = s.evaluate_field(np.stack([pts[:, 0], theta, pts[:, 1]], axis=1), 1)[0]
    assert np.max(np.abs(out - ref)) <= 1e-8 * np.max(np.abs(ref)), np.abs(out - ref) / np.max(np.abs(ref))


def test_rippled_bowl_on_curved_panels():
    """The smooth non-graph curve of Sec. 5, Example 2 given by its panels
    (degree-15 interpolants, graded toward the corner where the bowl meets
    the flat part): node tables, oracle operator rows near the axis, on the
    ripples, at the corner and in the PML against the GPU matrices, the GPU
    solution's backward error against those rows, the boundary data against
    the oracle's full solve (FP64 and mixed precision), and the field close to
    the bowl on both sides."""
    import oracle
    from paper_2412_11162_amd._binding import PMLBIE_KEEP_OPERATORS
    wl = workloads.bowl().with_(m_max_=4)
    g = oracle.geometry(wl)
    N = g.n
    assert N == 320
    s = _solver(wl, flags=PMLBIE_KEEP_OPERATORS)
    nd = s.nodes()
    assert np.max(np.abs(nd[:, 0] - g.rho)) <= 1e-15
    assert np.max(np.abs(nd[:, 2] - g.z)) <= 1e-15
    # weights and normals come from the derivative of the degree-15
    # interpolant, formed independently on each side (Legendre series by
    # quadrature here, a Chebyshev-Vandermonde solve in the oracle): they
    # agree to the rounding of that differentiation
    assert np.max(np.abs(nd[:, 7] - g.W)) <= 1e-12 * np.max(g.W)
    assert np.max(np.abs(nd[:, 10:12] - g.nu)) <= 1e-12
    c = int(np.argmin(np.hypot(g.rho - 1.0, g.z)))
    rows = sorted({0, 1, 40, 77, 100, 150, c - 1, c, c + 1, N - 3})
    modes = [0, 2, 4]
    S, K = oracle.core.operator_rows(g, rows, [wl.k1, wl.k2], modes)
    for j, n in enumerate(modes):
        G = s.get_operator(n).cpu().numpy()
        for ik, (sgn, off) in enumerate(((1.0, 0), (-1.0, N))):
            Kr = G[[off + r for r in rows], :N] - sgn * np.eye(N)[rows]
            Sr = -G[[off + r for r in rows], N:]
            assert _normwise(Kr, K[ik, j]) <= KERNEL_TOL, (n, ik, "K")
            assert _normwise(Sr, S[ik, j]) <= KERNEL_TOL, (n, ik, "S")
    b1, b2 = oracle.rhs_point_source(g, modes, 0.0, 1.0)
    out = [o[:, 0, :].cpu().numpy() for o in s.solve_modes([("point", 0.0, 1.0)])]
    res, den = [], []
    for j, n in enumerate(modes):
        x1, x2 = out[0][n], out[1][n]
        for q, i in enumerate(rows):
            res.append(abs(K[0, j][q] @ x1 + x1[i] - S[0, j][q] @ x2))
            den.append(np.abs(K[0, j][q]) @ np.abs(x1) + abs(x1[i]) + np.abs(S[0, j][q]) @ np.abs(x2))
            lo = K[1, j][q] @ x1 - x1[i] - S[1, j][q] @ x2
            rhs = K[1, j][q] @ b1[j] - b1[j][i] - S[1, j][q] @ b2[j]
            res.append(abs(lo - rhs))
            den.append(np.abs(K[1, j][q]) @ (np.abs(x1) + np.abs(b1[j])) + abs(x1[i]) + abs(b1[j][i])
                       + np.abs(S[1, j][q]) @ (np.abs(x2) + np.abs(b2[j])))
    res, den = np.array(res), np.array(den)
    errs = res / np.maximum(den, 1e-6 * den.max())
    assert np.max(errs) <= BOUNDARY_TOL, errs
    # field close to the bowl, against the oracle's exact representation on
    # the oracle's own solution of the full system
    A, _, _ = oracle.assemble(g, list(range(wl.m_max + 1)))
    allm = list(range(wl.m_max + 1))
    b1, b2 = oracle.rhs_point_source(g, allm, 0.0, 1.0)
    sol = oracle.solve(g, allm, b1, b2, A=A)
    pts, med = [], []
    for l, d in ((60, 0.03), (120, 0.1), (c - 2, 0.02)):
        nu = g.nu[l]
        pts.append([g.rho[l] - d * nu[0], g.z[l] - d * nu[1]]); med.append(1)
        pts.append([g.rho[l] + d * nu[0], g.z[l] + d * nu[1]]); med.append(2)
    pts = np.array(pts)
    theta = np.linspace(0.1, 2.2, len(pts))
    ref = _field_ref(g, allm, sol, pts, med, theta)
    s2 = _solver(wl)
    out2 = [o[:, 0, :].cpu().numpy() for o in s2.solve_modes([("point", 0.0, 1.0)])]
    assert np.max(_boundary_err(out2, sol[:4])) <= BOUNDARY_TOL
    fo = s2.evaluate_field(np.stack([pts[:, 0], theta, pts[:, 1]], axis=1), 1)[0]
    assert np.max(np.abs(fo - ref)) <= 1e-8 * np.max(np.abs(ref)), np.abs(fo - ref) / np.max(np.abs(ref))
    # complex64 LU with FP64 refinement on the curved panels: the mixed bar
    from paper_2412_11162_amd._binding import PMLBIE_MIXED
    s3 = _solver(wl, precision=PMLBIE_MIXED)
    out3 = [o[:, 0, :].cpu().numpy() for o in s3.solve_modes([("point", 0.0, 1.0)])]
    assert np.max(_boundary_err(out3, sol[:4])) <= 1e-6


def test_panel_curve_argument_errors():
    from paper_2412_11162_amd.solver import Solver, PmlbieError
    wl = workloads.bowl()
    nodes = np.array(wl.curve_nodes)
    s = Solver(0)
    shifted = nodes.copy()
    shifted[5:, :, 1] += 0.01                          # panels 4 and 5 do not join
    off_axis = nodes.copy()
    off_axis[0, :, 0] += 0.05                          # the first panel does not start on the axis
    neg = nodes.copy()
    neg[3, 2, 0] = -0.1                                # a node with rho <= 0
    for bad in (nodes[:2], nodes[:18], shifted, off_axis, neg):
        with pytest.raises(PmlbieError) as e:
            s.set_panels(bad)
        assert e.value.code == -1
    # not flat beyond the PML start (the two panels past a1 = 2 tilted, still
    # joined at (2, 0))
    tilted = nodes.copy()
    tilted[-2:, :, 1] = 1e-3 * (tilted[-2:, :, 0] - 2.0)
    s.set_panels(tilted)
    with pytest.raises(PmlbieError) as e:
        s.set_media_pml(wl.k1, wl.k2, wl.a1, wl.T, wl.S, wl.a2, wl.T2, wl.S2)
    assert e.value.code == -1
    s.set_panels(nodes)
    s.set_media_pml(wl.k1, wl.k2, wl.a1, wl.T, wl.S, wl.a2, wl.T2, wl.S2)


def test_field_with_several_right_hand_sides(corner_ref):
    """Field synthesis for three incidences in one call equals the same
    points evaluated one incidence at a time (each node's kernels are read
    once for all right-hand sides)."""
    wl, g, A, modes = corner_ref
    incs = [("point", 0.0, 1.0), ("plane", 0.5), ("point", 0.3, 0.8)]
    rtz = np.array([[0.5, -0.5, 0.3], [1.4, 0.7, -0.5], [0.3, 1.1, 0.8], [1.6, 2.0, -1.2]])  # rho, theta, z
    s = _solver(wl)
    s.solve_modes(incs)
    many = s.evaluate_field(rtz, len(incs))
    for r, inc in enumerate(incs):
        s1 = _solver(wl)
        s1.solve_modes([inc])
        one = s1.evaluate_field(rtz, 1)[0]
        assert np.max(np.abs(many[r] - one)) <= 1e-12 * np.max(np.abs(one)), r


def test_field_on_the_axis():
    """Points on the axis (rho = 0), where 4 rho~ rho~' vanishes and only
    mode 0 survives: the library's field equals the oracle's representation
    in both media."""
    import oracle
    wl = workloads.tiny()
    g = oracle.geometry(wl)
    modes = list(range(wl.m_max + 1))
    b1, b2 = oracle.rhs_point_source(g, modes, 0.3, 1.0)
    sol = oracle.solve(g, modes, b1, b2)
    pts = np.array([[0.0, 1.2], [0.0, -0.8]])
    ref = _field_ref(g, modes, sol, pts, [1, 2], np.zeros(2))
    s = _solver(wl)
    s.solve_modes([("point", 0.3, 1.0)])
    out = s.evaluate_field(np.stack([pts[:, 0], np.array([0.0, 1.3]), pts[:, 1]], axis=1), 1)[0]
    assert np.max(np.abs(out - ref)) <= 1e-8 * np.max(np.abs(ref))

"""Parity of the largest configuration at its full size, in the launch
configuration the benchmark times: 4096 nodes, k1 = 20, k2 = 30, the three
rings, the 2048-point angle grid, modes 0..256 built as the benchmark's two
mixed-precision batches (0..128 and 129..256: complex64 LU, FP64 refinement).
A full oracle solve is out of reach at this size; the oracle's operator rows
of four nodes (near the axis, on the rings, right below the point source, in
the PML) for modes 0, 1, 128, 129, 255, 256 and both media, and its
right-hand-side data at every node, are stored (tests/golden/make_golden.py
largest_rows), and the build is checked against them:

  - the assembled rows (far, split, direct and near-panel entries) within the
    modal-kernel bar 1e-10 (normwise per block row);
  - the library's right-hand-side data (b1 = u1 - u2, b2 = phi1 - phi2 of its
    outputs) within the same bar;
  - the solution of the plane wave at polar angle pi/3 and of a point source
    just above the curve satisfies the oracle's equations in those rows
    within the boundary-data bar (backward error per mode, as the paper-scale
    row tests); the plane wave's modes beyond ~k1 rho sin(phi) ~ 120 carry
    data below 1e-10 of its mode 0 (rounding noise on both sides), and there
    the solution must be as small as that noise.
"""

import gc
import os

import numpy as np
import pytest

import workloads
from test_gpu_parity import BOUNDARY_TOL, KERNEL_TOL, _normwise, _row_backward_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BATCHES = ((0, 128), (129, 256))


@pytest.fixture(scope="module")
def rows_ref():
    path = os.path.join(HERE, "golden", "rows_largest.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle rows not generated: python tests/golden/make_golden.py largest_rows")
    return np.load(path)


def _incidences(ref):
    return [("point", float(p[0]), float(p[1])) if k == 0 else ("plane", float(p[0]))
            for k, p in zip(ref["inc_kind"], ref["inc_param"])]


@pytest.mark.parametrize("batch", BATCHES)
def test_largest_full_size_rows_and_solution(rows_ref, batch):
    from paper_2412_11162_amd import _binding as B
    from test_gpu_parity import _solver
    gc.collect()
    wl = workloads.largest()
    lo, hi = batch
    rows = [int(r) for r in rows_ref["rows"]]
    modes = [int(m) for m in rows_ref["modes"]]
    sel = [j for j, m in enumerate(modes) if lo <= m <= hi]
    s = _solver(wl, build=False)
    s.build_modal_operators(wl.n_theta, hi, B.PMLBIE_MIXED, 0, m_min=lo)
    N = s.N
    assert N == 4096
    S, K = rows_ref["S"], rows_ref["K"]
    I = np.eye(N)[rows]
    worst = 0.0
    for j in sel:
        n = modes[j]
        G = s.get_operator(n)
        up = G[rows, :].cpu().numpy()
        lw = G[[N + r for r in rows], :].cpu().numpy()
        del G
        for blk, ref in ((up[:, :N], K[0, j] + I), (up[:, N:], -S[0, j]),
                         (lw[:, :N], K[1, j] - I), (lw[:, N:], -S[1, j])):
            e = _normwise(blk, ref)
            worst = max(worst, e)
            assert e <= KERNEL_TOL, (n, e)
    incs = _incidences(rows_ref)
    out = s.solve_modes(incs)
    st, cnt = s.stats()
    assert cnt[1] <= 1e-10
    b1, b2 = rows_ref["b1"], rows_ref["b2"]
    for r in range(len(incs)):
        # the incidence's data scale over all stored modes; a mode whose data
        # are below 1e-10 of it (the plane wave's modes beyond ~k1 rho sin phi)
        # carries rounding noise on both sides, and its solution must be as
        # small as that noise
        dn = np.array([np.linalg.norm(b1[r][j]) + np.linalg.norm(b2[r][j]) for j in range(len(modes))])
        alive = [j for j in sel if dn[j] >= 1e-10 * dn.max()]
        for j in sel:
            if j not in alive:
                x = np.concatenate([out[0][modes[j] - lo, r].cpu().numpy(), out[1][modes[j] - lo, r].cpu().numpy()])
                assert np.linalg.norm(x) <= 1e-8 * dn.max(), (modes[j], np.linalg.norm(x), dn.max())
        if not alive:
            print("modes %d..%d, %s: data below 1e-10 of the incidence's, solutions within the noise" %
                  (lo, hi, incs[r]), flush=True)
            continue
        # the library's own right-hand-side data: b1 = u1 - u2, b2 = phi1 - phi2
        for j in alive:
            q = modes[j] - lo
            g1 = (out[0][q, r] - out[2][q, r]).cpu().numpy()
            g2 = (out[1][q, r] - out[3][q, r]).cpu().numpy()
            e1 = np.linalg.norm(g1 - b1[r][j]) / np.linalg.norm(b1[r][j])
            e2 = np.linalg.norm(g2 - b2[r][j]) / np.linalg.norm(b2[r][j])
            print("  mode %d data vs oracle: b1 %.1e b2 %.1e" % (modes[j], e1, e2), flush=True)
            assert max(e1, e2) <= KERNEL_TOL, (modes[j], e1, e2)
        data = (None, rows, [modes[j] for j in alive], S[:, alive], K[:, alive], b1[r][alive], b2[r][alive])
        errs = _row_backward_errors(out, data, rhs=r, m0=lo)
        print("modes %d..%d, %s: rows within %.1e of the oracle's; backward errors %s" %
              (lo, hi, incs[r], worst, " ".join("%.1e" % e for e in errs)), flush=True)
        assert np.max(errs) <= BOUNDARY_TOL, (r, errs)
    del out, s
    gc.collect()

"""Parity at the physics of the largest configuration: k1 = 20, k2 = 30,
three Gaussian rings (seed 11162), PML rho in [5, 7] with S = 3, the
2048-point angle grid, modes 0..256, the 16 plane waves with polar angles
(pi/3) i / 15 and a point source just above the curve that excites the
highest modes -- on 64 nodes per segment (256 nodes), where the oracle's full
solve is affordable.  The stored oracle file holds modes 0, 1, 2, 64, 128,
255, 256 (tests/golden/make_golden.py largest_reduced).

FP64 builds all modes at once and must match to the boundary-data bar
(1e-8); mixed precision runs the way the full-size configuration does --
mode batches with m_min > 0, complex64 LU, FP64 refinement -- and must match
to 1e-6.  Every call goes through the C ABI.
"""

import numpy as np
import pytest

import workloads
from test_gpu_parity import (BOUNDARY_TOL, MIXED_TOL, _golden, _print_errors, _solver,
                             _stored_errors, _stored_incidences)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solve_all(s, incs):
    """Solve in groups of at most 16 right-hand sides; outputs concatenated
    along the right-hand-side axis."""
    parts = [s.solve_modes(incs[i:i + 16]) for i in range(0, len(incs), 16)]
    return [np.concatenate([p[k].cpu().numpy() for p in parts], axis=1) for k in range(4)]


def test_largest_physics_fp64_all_modes():
    ref = _golden("largest_reduced")
    wl = workloads.largest_reduced()
    incs = _stored_incidences(ref)
    s = _solver(wl)
    assert s.N == 256 and s.M == 256
    info = s.info()
    print("largest physics, 256 nodes: angle grid %d, far %d split %d direct %d" %
          (info[2], info[4], info[5], info[6]), flush=True)
    modes, errs = _stored_errors(_solve_all(s, incs), ref)
    _print_errors("largest physics FP64", modes, errs, incs)
    assert np.max(errs) <= BOUNDARY_TOL, errs


def test_largest_physics_mixed_in_mode_batches():
    from paper_2412_11162_amd import _binding as B
    ref = _golden("largest_reduced")
    wl = workloads.largest_reduced()
    incs = _stored_incidences(ref)
    s = _solver(wl, build=False)
    batches = ((0, 100), (101, 200), (201, 256))
    outs = []
    for lo, hi in batches:
        s.build_modal_operators(wl.n_theta, hi, B.PMLBIE_MIXED, 0, m_min=lo)
        got = _solve_all(s, incs)
        st, cnt = s.stats()
        print("batch %d..%d: refinement iterations %d, relative residual %.1e" % (lo, hi, cnt[0], cnt[1]),
              flush=True)
        assert cnt[1] <= 1e-10
        outs.append(got)
    full = [np.concatenate([o[k] for o in outs], axis=0) for k in range(4)]
    assert full[0].shape[0] == 257
    modes, errs = _stored_errors(full, ref)
    _print_errors("largest physics mixed, mode batches", modes, errs, incs)
    assert np.max(errs) <= MIXED_TOL, errs

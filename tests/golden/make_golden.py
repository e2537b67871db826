"""Write the stored oracle results used by the GPU parity tests.

Calls only the oracle (``oracle/``) and the workload definitions
(``workloads``); nothing here touches the HIP path.

    python tests/golden/make_golden.py small            # ~3 min on 8 cores
    python tests/golden/make_golden.py paper_scale      # ~2 h on 8 cores
    python tests/golden/make_golden.py largest_reduced  # ~20 min on 8 cores
    python tests/golden/make_golden.py largest_rows     # ~4 min on 8 cores

The operators are assembled in blocks of target rows; each block is kept in
a cache directory (``--cache DIR``, default ``$TMPDIR/pmlbie_golden``) so that
an interrupted run resumes where it stopped.  Only the small per-mode
boundary data land in ``tests/golden/boundary_<name>.npz``.

Modes and incidences.  The small workload stores every mode of its one
incidence.  The paper-scale file stores modes 0, 2, 8, 64, 128 for three
incidences: the benchmark's point source (0.3, 0, 1.2), whose data fall to
rounding level from mode ~32 up, a point source at (3.5, 0, 0.25) just above
the curve, whose data decay slowly with the mode (mode 128 ~1e-4 of the
largest), and the plane wave of the paper's examples (polar angle pi/3,
Sec. 5).  The reduced largest configuration stores modes 0, 1, 2, 64, 128,
255, 256 for its 16 plane waves and a point source at (4, 0, 0.15) that
excites the highest modes.

The largest configuration at its full size (4096 nodes) is too large for a
full oracle solve; `largest_rows` stores the oracle's operator rows of four
nodes (near the axis, on the rings, right below the point source, in the PML)
for modes 0, 1, 128, 129, 255, 256 and both media, with the right-hand-side data of the plane wave at polar
angle pi/3 and of a point source at (4, 0, 0.15) at every node, for the
backward-error tests of the full-size build.

Tolerances.  Modal kernels at 1e-14 relative (azimuthal quadrature), and the
near-panel product integrals at 1e-12 relative for the two larger cases: the
inner azimuthal integrals carry ~1e-14 relative rounding noise, which a
1e-13 outer tolerance chases with ten times the intervals for a change of
~5e-13; the parity bar on boundary data is 1e-8 (FP64) and 1e-6 (mixed).
"""

import argparse
import os
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

SPECS = {
    "small": dict(modes=None, incidences=None, near_reltol=1e-13, block=256),
    "paper_scale": dict(modes=[0, 2, 8, 64, 128],
                        incidences=[("point", 0.3, 1.2), ("point", 3.5, 0.25),
                                    ("plane", np.pi / 3)],
                        near_reltol=1e-12, block=32),
    "largest_reduced": dict(modes=[0, 1, 2, 64, 128, 255, 256],
                            incidences=None, extra=[("point", 4.0, 0.15)],
                            near_reltol=1e-12, block=16),
}


def rhs(g, modes, inc):
    """Right-hand sides of one incidence, one mode at a time (each mode's
    azimuthal quadrature then stops relative to that mode's own size)."""
    b1 = np.zeros((len(modes), g.n), dtype=np.complex128)
    b2 = np.zeros_like(b1)
    for j, n in enumerate(modes):
        if inc[0] == "point":
            x1, x2 = oracle.rhs_point_source(g, [n], inc[1], inc[2])
        else:
            x1, x2 = oracle.rhs_plane_wave(g, [n], inc[1])
        b1[j], b2[j] = x1[0], x2[0]
    return b1, b2


def assemble_cached(g, modes, near_reltol, block, cache):
    """A_n = [[K1 + I, -S1], [K2 - I, -S2]] assembled from blocks of rows,
    each block cached as it completes."""
    wl = g.wl
    N = g.n
    ks = [wl.k1, wl.k2]
    os.makedirs(cache, exist_ok=True)
    S = np.zeros((2, len(modes), N, N), dtype=np.complex128)
    K = np.zeros_like(S)
    tag = "%s_m%s" % (wl.name, "-".join(str(m) for m in modes))
    t0 = time.time()
    for r0 in range(0, N, block):
        rows = list(range(r0, min(N, r0 + block)))
        f = os.path.join(cache, "%s_rows%05d.npz" % (tag, r0))
        if os.path.exists(f):
            d = np.load(f)
            Sb, Kb = d["S"], d["K"]
        else:
            Sb, Kb = oracle.core.operator_rows(g, rows, ks, modes, near_reltol=near_reltol)
            np.savez(f + ".tmp.npz", S=Sb, K=Kb)
            os.replace(f + ".tmp.npz", f)
            print("rows %d..%d done, %.0f s" % (rows[0], rows[-1], time.time() - t0), flush=True)
        S[:, :, rows, :] = Sb
        K[:, :, rows, :] = Kb
    A = np.zeros((len(modes), 2 * N, 2 * N), dtype=np.complex128)
    I = np.eye(N)
    A[:, :N, :N] = K[0] + I
    A[:, :N, N:] = -S[0]
    A[:, N:, :N] = K[1] - I
    A[:, N:, N:] = -S[1]
    return A


ROWS_LARGEST = dict(rows=[10, 1500, 1636, 3500], modes=[0, 1, 128, 129, 255, 256],
                    incidences=[("plane", np.pi / 3), ("point", 4.0, 0.15)], near_reltol=1e-12)


def make_rows(cache: str) -> str:
    """Oracle rows and right-hand-side data of the full-size largest
    configuration (see the module docstring)."""
    spec = ROWS_LARGEST
    wl = workloads.ALL["largest"]()
    g = oracle.geometry(wl)
    t0 = time.time()
    S, K = oracle.core.operator_rows(g, spec["rows"], [wl.k1, wl.k2], spec["modes"],
                                     near_reltol=spec["near_reltol"])
    print("rows done in %.0f s" % (time.time() - t0), flush=True)
    b1s, b2s = [], []
    for inc in spec["incidences"]:
        b1, b2 = rhs(g, spec["modes"], inc)
        b1s.append(b1)
        b2s.append(b2)
    kinds = np.array([0 if i[0] == "point" else 1 for i in spec["incidences"]])
    params = np.array([[i[1], i[2] if len(i) > 2 else 0.0] for i in spec["incidences"]])
    path = os.path.join(HERE, "rows_largest.npz")
    # S, K: [medium][mode][row][node]; b1, b2: [incidence][mode][node]
    np.savez_compressed(path, rows=np.array(spec["rows"]), modes=np.array(spec["modes"]), S=S, K=K,
                        b1=np.stack(b1s), b2=np.stack(b2s), inc_kind=kinds, inc_param=params)
    print("wrote", path, "in %.0f s" % (time.time() - t0), flush=True)
    return path


def make(name: str, cache: str) -> str:
    spec = SPECS[name]
    wl = workloads.ALL[name]()
    g = oracle.geometry(wl)
    modes = spec["modes"] if spec["modes"] is not None else list(range(wl.m_max + 1))
    incs = list(spec["incidences"] if spec["incidences"] is not None else wl.incidences)
    incs += spec.get("extra", [])
    t0 = time.time()
    A = assemble_cached(g, modes, spec["near_reltol"], spec["block"], cache)
    print("assembled %s modes %s in %.0f s" % (name, modes, time.time() - t0), flush=True)
    out = {k: [] for k in ("u1", "p1", "u2", "p2", "b1", "b2")}
    for inc in incs:
        b1, b2 = rhs(g, modes, inc)
        u1, p1, u2, p2, _ = oracle.solve(g, modes, b1, b2, A=A)
        for k, v in zip(("u1", "p1", "u2", "p2", "b1", "b2"), (u1, p1, u2, p2, b1, b2)):
            out[k].append(v)
    # layout [mode][rhs][node], as the library returns the boundary data
    arr = {k: np.stack(v, axis=1) for k, v in out.items()}
    if len(incs) == 1:   # the small file keeps its original [mode][node] layout
        arr = {k: v[:, 0] for k, v in arr.items()}
    cond = [float(np.linalg.cond(A[j])) for j in range(len(modes))] if g.n <= 512 else []
    kinds = np.array([0 if i[0] == "point" else 1 for i in incs])
    params = np.array([[i[1], i[2] if len(i) > 2 else 0.0] for i in incs])
    path = os.path.join(HERE, "boundary_%s.npz" % name)
    np.savez_compressed(path, modes=np.array(modes), cond=np.array(cond), inc_kind=kinds,
                        inc_param=params, **arr)
    print("wrote", path, "in %.0f s" % (time.time() - t0), flush=True)
    return path


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+", choices=sorted(SPECS) + ["largest_rows"])
    ap.add_argument("--cache", default=os.path.join(tempfile.gettempdir(), "pmlbie_golden"))
    a = ap.parse_args()
    for n in a.names:
        if n == "largest_rows":
            make_rows(a.cache)
        else:
            make(n, a.cache)

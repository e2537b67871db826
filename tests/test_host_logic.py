"""The library's host-side geometry on the CPU (no device): panel layouts,
node tables, the medium of a point and the near-panel rules, through a small
driver compiled against `csrc/host_geom.cpp`, checked against the oracle's
independent geometry and against what the rules must integrate exactly.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2412_11162_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not cc:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("host") / "host_logic_driver")
    subprocess.run([cc, "-O2", "-std=c++17", "-fopenmp", "-I", CSRC, "-o", exe,
                    os.path.join(HERE, "host", "host_logic_driver.cpp"), os.path.join(CSRC, "host_geom.cpp")],
                   check=True, capture_output=True)
    return exe


def _run(exe, *args):
    out = subprocess.run([exe] + [str(a) for a in args], check=True, capture_output=True, text=True).stdout
    return out


def _poly_args(wl):
    v = [c for p in wl.polyline for c in p]
    return ["poly", wl.grade, len(wl.polyline)] + v + list(wl.panels) + [wl.a1, wl.T, wl.S]


def test_polyline_layouts_match_the_oracle(driver):
    """Graded panel layouts (rectangular and stepped curves, several grades)
    from the library equal the oracle's, which is written separately from the
    same definition."""
    for wl in (workloads.corner(grade=3), workloads.corner(panels=(3, 2, 5, 2), grade=6), workloads.stepped()):
        host = np.loadtxt(_run(driver, "layout", *_poly_args(wl)).splitlines())
        ref = oracle.core.polyline_panels(wl)
        assert host.shape == ref.shape
        assert np.max(np.abs(host - ref)) <= 1e-15


def test_node_tables_match_the_oracle(driver):
    """Node positions, Im rho~, weights and normals: graph curve (tiny) and
    polyline (corner)."""
    wl = workloads.tiny()
    host = np.loadtxt(_run(driver, "tables", "graph", wl.nodes_per_segment, wl.bumps[0][0], wl.bumps[0][2],
                           wl.a1, wl.T, wl.S).splitlines())
    g = oracle.geometry(wl)
    for col, ref, tol in ((0, g.rho, 1e-15), (1, g.I, 1e-14), (2, g.z, 1e-15), (3, g.W, 1e-14)):
        assert np.max(np.abs(host[:, col] - ref)) <= tol, col
    wl = workloads.corner(grade=3)
    host = np.loadtxt(_run(driver, "tables", *_poly_args(wl)).splitlines())
    g = oracle.geometry(wl)
    assert np.max(np.abs(host[:, 3] - g.W)) <= 1e-15
    assert np.max(np.abs(host[:, 4:6] - g.nu)) <= 1e-15


def test_curved_node_tables_match_the_oracle(driver, tmp_path):
    """Curved panels (Example 2's bowl): the given nodes, and weights and
    normals from the two independently formed interpolants."""
    wl = workloads.bowl()
    path = tmp_path / "nodes.txt"
    np.savetxt(path, np.asarray(wl.curve_nodes).reshape(-1))
    host = np.loadtxt(_run(driver, "tables", "curved", path, wl.a1, wl.T, wl.S).splitlines())
    g = oracle.geometry(wl)
    assert np.max(np.abs(host[:, 0] - g.rho)) == 0.0      # the given nodes
    assert np.max(np.abs(host[:, 3] - g.W)) <= 1e-12 * np.max(g.W)
    assert np.max(np.abs(host[:, 4:6] - g.nu)) <= 1e-12


def test_medium_of_points(driver):
    """The medium test on the stepped curve of Example 3: above the overhang,
    inside the lower step and above the flat part is the upper medium; the
    pocket under the overhang, beside the wall and below the flat part the
    lower one."""
    wl = workloads.stepped()
    pts = [(0.4, -0.45, 1), (0.6, -0.9, 1), (0.1, 0.5, 1), (1.5, 0.1, 1),
           (0.4, -0.6, 2), (0.1, -0.8, 2), (1.2, -0.5, 2), (1.5, -0.1, 2), (0.3, -1.2, 2)]
    args = _poly_args(wl) + ["--"] + [c for p in pts for c in p[:2]]
    med = [int(x) for x in _run(driver, "above", *args).split()]
    assert med == [p[2] for p in pts]


def test_near_rules_integrate_panel_polynomials_exactly(driver):
    """On straight panels the product-integration coefficients of a job,
    summed over its auxiliary points, are 2 int l_l(t) rho(t) |r'| dt: the
    graded 16-point pieces integrate that degree-16 polynomial exactly (the
    mapped innermost piece to ~1e-13), and the node rule gives it as 2 W_l.
    Pins the auxiliary weights, the Lagrange coefficients and the operator
    factor 2 for self and neighbour panels."""
    wl = workloads.corner(grade=3)
    g = oracle.geometry(wl)
    rows = _run(driver, "near", *_poly_args(wl)).splitlines()
    assert len(rows) == sum(len(g.near_panels(i)) for i in range(g.n))
    worst = 0.0
    for line in rows:
        v = line.split()
        p = int(v[1])
        sums = np.array([float(x) for x in v[3:]])
        ref = 2.0 * g.W[16 * p:16 * p + 16]
        worst = max(worst, np.max(np.abs(sums - ref)) / np.max(np.abs(ref)))
    assert worst <= 1e-12, worst

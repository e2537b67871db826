"""Synthetic workloads for the axisymmetric two-layer PML-BIE problem.

This module holds input data only: wavenumbers, interface shapes, PML
parameters, discretisation sizes and incidences, plus the seeded draws for
the randomised shapes.  It contains none of the method's arithmetic, so both
the oracle and the HIP path may import it.

Interface family (every workload but the polyline ones): a graph z = h~(rho) with

    h(rho)  = [sum_i a_i exp(-((rho - c_i)/w_i)^2)] * (cos(f rho) if f else 1)
    h~(rho) = h(rho) - h(a1)  for rho < a1,   0 for rho >= a1,

so the curve is continuous at the start of the PML (rho = a1) and flat inside
it.  The generating curve runs from the axis (rho = 0) to the outer PML edge
rho = a1 + T and is cut into four segments [0, a1/2], [a1/2, a1],
[a1, a1 + T/2], [a1 + T/2, a1 + T]; each segment holds `nodes_per_segment`
Gauss-Legendre nodes in sub-panels of 16.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

PANEL_NODES = 16


@dataclass(frozen=True)
class Workload:
    name: str
    k1: complex
    k2: complex
    bumps: Tuple[Tuple[float, float, float], ...]  # (amplitude, centre, width)
    cos_freq: float
    a1: float
    T: float
    S: float
    a2: float
    T2: float
    S2: float
    p: int
    nodes_per_segment: int
    n_theta: int
    m_max_: int
    # incidences: ("point", rho*, z*) or ("plane", phi_inc)
    incidences: Tuple[Tuple, ...] = field(default_factory=tuple)
    # polyline curve with corners (replaces the graph when set): vertices
    # (rho, z) from the axis outward, equal panels per segment, and the number
    # of geometric halvings of the panels that touch a corner
    polyline: Tuple[Tuple[float, float], ...] = ()
    panels: Tuple[int, ...] = ()
    grade: int = 0
    # curve given by its panels (replaces the graph when set): [P, 16, 2]
    # (rho, z) at the 16 Gauss-Legendre points of each panel
    curve_nodes: object = field(default=None, compare=False)

    @property
    def m_max(self) -> int:
        return self.m_max_

    @property
    def n_sub(self) -> int:
        assert self.nodes_per_segment % PANEL_NODES == 0
        return self.nodes_per_segment // PANEL_NODES

    @property
    def seg_breaks(self) -> List[float]:
        a1, T = self.a1, self.T
        return [0.0, 0.5 * a1, a1, a1 + 0.5 * T, a1 + T]

    @property
    def n_nodes(self) -> int:
        return 4 * self.nodes_per_segment

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def small() -> Workload:
    """Plain FP64, small: k1 = 2 pi, k2 = 3 pi, h = 0.3 exp(-rho^2), PML
    rho in [2, 3], sigma0 = 2, 64 nodes per segment, 64 theta samples,
    point source on the axis at (0, 0, 1)."""
    return Workload(
        name="small",
        k1=2 * math.pi, k2=3 * math.pi,
        bumps=((0.3, 0.0, 1.0),), cos_freq=0.0,
        a1=2.0, T=1.0, S=2.0, a2=2.0, T2=1.0, S2=2.0, p=6,
        nodes_per_segment=64, n_theta=64, m_max_=16,
        incidences=(("point", 0.0, 1.0),),
    )


def paper_scale() -> Workload:
    """Plain FP64 at paper scale: k1 = 10, k2 = 15,
    h = 0.5 exp(-rho^2/2) cos(2 rho), PML rho in [4, 5.5], sigma0 = 3,
    512 nodes per segment (2048 nodes, 4096 unknowns per mode), 256 theta
    samples with modes -128..128 kept, point source at (0.3, 0, 1.2)."""
    return Workload(
        name="paper_scale",
        k1=10.0, k2=15.0,
        bumps=((0.5, 0.0, math.sqrt(2.0)),), cos_freq=2.0,
        a1=4.0, T=1.5, S=3.0, a2=3.0, T2=1.5, S2=3.0, p=6,
        nodes_per_segment=512, n_theta=256, m_max_=128,
        incidences=(("point", 0.3, 1.2),),
    )


def largest(seed: int = 11162) -> Workload:
    """Largest one-GPU case: k1 = 20, k2 = 30, three Gaussian ring bumps with
    amplitudes U[0.2, 0.5], centres U[0, 3], widths U[0.5, 2]; PML
    rho in [5, 7], sigma0 = 3; 1024 nodes per segment, 512 theta samples,
    16 plane waves with polar angles (pi/3) i / 15."""
    rng = np.random.default_rng(seed)
    amps = rng.uniform(0.2, 0.5, 3)
    cents = rng.uniform(0.0, 3.0, 3)
    widths = rng.uniform(0.5, 2.0, 3)
    bumps = tuple((float(a), float(c), float(w)) for a, c, w in zip(amps, cents, widths))
    incs = tuple(("plane", math.pi / 3 * i / 15) for i in range(16))
    return Workload(
        name="largest",
        k1=20.0, k2=30.0, bumps=bumps, cos_freq=0.0,
        a1=5.0, T=2.0, S=3.0, a2=4.0, T2=2.0, S2=3.0, p=6,
        nodes_per_segment=1024, n_theta=512, m_max_=256, incidences=incs,
    )


def largest_reduced() -> Workload:
    """The largest configuration's physics (media, rings, PML, angle grid,
    modes 0..256, the 16 plane waves) on 64 nodes per segment (256 nodes), a
    size the oracle can solve; the parity case of that configuration."""
    return largest().with_(name="largest_reduced", nodes_per_segment=64)


def tiny(nodes_per_segment: int = 16, n_theta: int = 32, **kw) -> Workload:
    """A reduced version of the small workload (used for oracle-vs-kernel
    parity on the CPU side and for fast end-to-end checks)."""
    w = small().with_(name="tiny", nodes_per_segment=nodes_per_segment, n_theta=n_theta,
                      m_max_=n_theta // 4)
    return w.with_(**kw) if kw else w


def corner(panels: Tuple[int, ...] = (2, 2, 2, 2), grade: int = 1, **kw) -> Workload:
    """The rectangular perturbation of depth and radius 1 (Sec. 5, Example 1;
    the same polyline carries the corner test of Sec. 4.3): vertices (0, -1),
    (1, -1), (1, 0), then flat z = 0 through the PML start a1 = 2 to
    a1 + T = 4; two corners, at (1, -1) and (1, 0).  k1 = 2 pi, k2 = 3 pi,
    sigma0 = 2, point source on the axis at (0, 0, 1), 32 theta samples,
    modes 0..8."""
    w = small().with_(
        name="corner", bumps=(), cos_freq=0.0, a1=2.0, T=2.0, S=2.0, a2=2.0, T2=1.0, S2=2.0,
        n_theta=32, m_max_=8, incidences=(("point", 0.0, 1.0),),
        polyline=((0.0, -1.0), (1.0, -1.0), (1.0, 0.0), (2.0, 0.0), (4.0, 0.0)),
        panels=tuple(panels), grade=grade)
    return w.with_(**kw) if kw else w


def corner_paper() -> Workload:
    """The rectangular perturbation at the node count of the paper-scale
    workload: 24 panels per segment and eight halvings at each corner
    (128 panels, 2048 nodes); modes 0..32 (the paper keeps |n| <= 20 and 30
    for its two incidences, Sec. 5), 128 theta samples; a point source on the
    axis and a plane wave."""
    return corner(panels=(24, 24, 24, 24), grade=8).with_(
        name="corner_paper", n_theta=128, m_max_=32,
        incidences=(("point", 0.0, 1.0), ("plane", 0.5)))


def stepped() -> Workload:
    """The stepped perturbation of Sec. 5, Example 3: vertices (0, -0.5),
    (0.5, -0.5), (0.5, -0.7), (0.25, -0.7), (0.25, -1), (1, -1), (1, 0), then
    flat through a1 = 2 to a1 + T = 4; six corners and a segment that runs back
    toward the axis.  Two panels per segment, one halving at each corner
    (28 panels, 448 nodes); otherwise as the corner workload."""
    return corner().with_(
        name="stepped",
        polyline=((0.0, -0.5), (0.5, -0.5), (0.5, -0.7), (0.25, -0.7), (0.25, -1.0), (1.0, -1.0),
                  (1.0, 0.0), (2.0, 0.0), (4.0, 0.0)),
        panels=(2,) * 8, grade=1)


def _bowl_nodes(n_bowl: int, grade: int, n_flat: Tuple[int, int], a1: float, b: float) -> np.ndarray:
    """Panel nodes of the curve of Sec. 5, Example 2:
        rho(s) = [1 - 0.1 sin(3 pi s)] sin(pi s / 2),
        z(s)   = -[1 - 0.1 sin(3 pi s)] cos(pi s / 2),   s in [0, 1],
    from (0, -1) on the axis to (1, 0), then flat to a1 and on to b.  The
    bowl is cut into n_bowl equal parts in s and the flat stretch [1, a1]
    into n_flat[0]; the parts touching (1, 0), where the curve turns, are cut
    again at 2^-grade, ..., 1/2 toward it; [a1, b] gets n_flat[1] parts."""
    x, _ = np.polynomial.legendre.leggauss(16)

    def cuts(n, toward_end, toward_start):
        c = [k / n for k in range(n + 1)]
        if toward_start:
            c = [0.0] + [2.0 ** -l / n for l in range(grade, 0, -1)] + c[1:]
        if toward_end:
            c = c[:-1] + [1.0 - 2.0 ** -l / n for l in range(1, grade + 1)] + [1.0]
        return c

    panels = []
    cb = cuts(n_bowl, True, False)
    for s0, s1 in zip(cb[:-1], cb[1:]):
        sv = s0 + 0.5 * (1.0 + x) * (s1 - s0)
        f = 1.0 - 0.1 * np.sin(3 * np.pi * sv)
        panels.append(np.stack([f * np.sin(0.5 * np.pi * sv), -f * np.cos(0.5 * np.pi * sv)], axis=1))
    for (lo, hi), n, tg in (((1.0, a1), n_flat[0], True), ((a1, b), n_flat[1], False)):
        cf = cuts(n, False, tg)
        for u0, u1 in zip(cf[:-1], cf[1:]):
            r = lo + (u0 + 0.5 * (1.0 + x) * (u1 - u0)) * (hi - lo)
            panels.append(np.stack([r, np.zeros_like(r)], axis=1))
    return np.array(panels)


def bowl(n_bowl: int = 8, grade: int = 4, n_flat: Tuple[int, int] = (2, 2), **kw) -> Workload:
    """The smooth rippled bowl of Sec. 5, Example 2 (not a graph of rho; a
    corner where it meets the flat part), given by its panels: n_bowl parts
    of the bowl and n_flat flat ones, `grade` halvings toward the corner
    (8 + 4 + 2 + 4 + 2 = 20 panels, 320 nodes by default); media, PML,
    incidence and modes as the corner workload."""
    w = corner().with_(name="bowl", polyline=(), panels=(), grade=0,
                       curve_nodes=_bowl_nodes(n_bowl, grade, n_flat, 2.0, 4.0))
    return w.with_(**kw) if kw else w


def bowl_paper() -> Workload:
    """Example 2's rippled bowl at the node count of the paper-scale
    workload: 48 bowl parts and 24 + 40 flat ones, eight halvings toward the
    corner on both sides (128 panels, 2048 nodes); modes 0..32, 128 theta
    samples, a
    point source and a plane wave."""
    return bowl(n_bowl=48, grade=8, n_flat=(24, 40)).with_(
        name="bowl_paper", n_theta=128, m_max_=32,
        incidences=(("point", 0.0, 1.0), ("plane", 0.5)))


ALL = {"small": small, "paper_scale": paper_scale, "largest": largest,
       "largest_reduced": largest_reduced, "tiny": tiny,
       "corner": corner, "corner_paper": corner_paper, "stepped": stepped, "bowl": bowl,
       "bowl_paper": bowl_paper}


def seeded_pairs(n_nodes: int, count: int, seed: int) -> np.ndarray:
    """Seeded (target, source) index pairs with target != source."""
    rng = np.random.default_rng(seed)
    i = rng.integers(0, n_nodes, count)
    j = rng.integers(0, n_nodes - 1, count)
    j = np.where(j >= i, j + 1, j)
    return np.stack([i, j], axis=1).astype(np.int64)

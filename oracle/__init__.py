"""Plain FP64 CPU oracle for the axisymmetric two-layer PML-BIE method.

TEST INFRASTRUCTURE ONLY: only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or run anything in this package.
It shares no code with the HIP path (``paper_2412_11162_amd``) and never
imports it; the two meet only through the seeded workload definitions in
``workloads``.

The oracle follows the paper (Wang & Lu, arXiv 2412.11162) step by step:

* geometry and PML stretching: Sec. 3.1, eqs. eqrhot, eqzt, eqsgm1;
* Green's function, complex distance (principal branch), conormal
  derivative: Sec. 3.1 (fundamental solution, eq. eqg1t) and Sec. 4.3;
* azimuthal modes: Sec. 3.3, eqs. fmode3, eqsnpml, eqknpml, computed by
  adaptive quadrature over the azimuth -- no FFT and no kernel split;
* Nystrom matrices on Gauss-Legendre panels with exact near-panel product
  integrals (the reading that replaces the Alpert rule of Sec. 4.1);
* identity term: the solid-angle term of Sec. 3.1-3.3 (Lemmas 3.1/3.2) at
  smooth points, -1 for the upper medium and +1 for the lower medium with the
  normal pointing into the lower medium;
* coupled per-mode system: Sec. 4.2 (transmission conditions eqs1/eqs2,
  eqs. eqntdnj, eqntdpsi1/2) written with 2N unknowns per mode;
* dense LU solve: LAPACK through numpy (a library primitive).
"""

from .core import *  # noqa: F401,F403

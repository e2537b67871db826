"""Write the stored oracle results used by the GPU parity tests.

Calls only the oracle (``oracle/``) and the workload definitions
(``workloads``); nothing here touches the HIP path.

    python tests/golden/make_golden.py small        # ~3 min on 8 cores
    python tests/golden/make_golden.py paper_scale  # more than a day on 8 cores

The paper-scale file needs every one of the ~4.1M far node pairs by adaptive
quadrature (19 CPU-hours were not enough); the GPU tests hold the paper scale
to the oracle through exact operator rows and the solution's backward error
against them, and use this file only when it exists.
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

MODES = {"small": None, "paper_scale": [0, 128]}


def make(name: str) -> str:
    wl = workloads.ALL[name]()
    g = oracle.geometry(wl)
    modes = MODES[name] if MODES[name] is not None else list(range(wl.m_max + 1))
    t0 = time.time()
    A, S, K = oracle.assemble(g, modes)
    print("assembled %s modes %s in %.0f s" % (name, modes, time.time() - t0), flush=True)
    inc = wl.incidences[0]
    b1, b2 = oracle.rhs_point_source(g, modes, inc[1], inc[2])
    u1, p1, u2, p2, _ = oracle.solve(g, modes, b1, b2, A=A)
    cond = [float(np.linalg.cond(A[j])) for j in range(len(modes))] if g.n <= 512 else []
    path = os.path.join(HERE, "boundary_%s.npz" % name)
    np.savez_compressed(path, modes=np.array(modes), u1=u1, p1=p1, u2=u2, p2=p2, b1=b1, b2=b2,
                        cond=np.array(cond))
    print("wrote", path, "in %.0f s" % (time.time() - t0), flush=True)
    return path


if __name__ == "__main__":
    for n in sys.argv[1:]:
        make(n)

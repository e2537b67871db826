"""The allocation-free modal-kernel entry point against the ordinary one.

pmlbie_modal_kernels_noalloc runs the same classification, far-pair FFT,
split and direct kernels as pmlbie_modal_kernels, with its work buffers in
the library's fixed device scratch instead of allocations; its output must
match bit for bit, on two calls in a row (the second with fewer pairs, which
must not see the first call's counters or lists), and sizes beyond the
scratch limit are refused.
"""

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pair_geom(wl, n, seed):
    """Seeded node pairs of the workload's curve in the call's 12-double
    layout (every class: far, split, direct) plus a few off-curve points."""
    from paper_2412_11162_amd.solver import from_workload
    s = from_workload(wl, build=False)
    nd = s.nodes()
    N = nd.shape[0]
    pairs = workloads.seeded_pairs(N, n, seed)
    g = []
    for i, l in pairs:
        g.append([nd[i, 0], nd[i, 1], nd[l, 0], nd[l, 1], nd[i, 0] - nd[l, 0], nd[i, 1] - nd[l, 1],
                  nd[i, 2] - nd[l, 2], 0.0, nd[l, 3], nd[l, 4], nd[l, 5], nd[l, 6]])
    return np.array(g)


@pytest.mark.parametrize("name", ["tiny", "paper_scale"])
def test_noalloc_modal_kernels_match_the_allocating_call(name):
    from paper_2412_11162_amd import _binding as B
    from paper_2412_11162_amd.solver import from_workload, PmlbieError
    wl = workloads.ALL[name]()
    if name == "paper_scale":
        wl = wl.with_(m_max_=64)   # a lighter build; the angle grid stays L = 512
    s = from_workload(wl)
    print("noalloc parity:", name, "N", s.N, "M", s.M, flush=True)
    for n, seed in ((3000, 11), (700, 12)):
        geom = _pair_geom(wl, n, seed)
        ref = s.modal_kernels(geom)
        out = torch.full((n, 4, s.M + 1), float("nan"), dtype=torch.complex128, device="cuda")
        s.modal_kernels_noalloc(geom, out)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b), np.max(np.abs(a - b))
    # beyond the scratch limit: refused, nothing written
    big = _pair_geom(wl, B.PMLBIE_NOALLOC_MAX_PAIRS + 1, 13)
    out = torch.zeros((big.shape[0], 4, s.M + 1), dtype=torch.complex128, device="cuda")
    with pytest.raises(PmlbieError) as e:
        s.modal_kernels_noalloc(big, out)
    assert e.value.code == B.PMLBIE_EINVAL and "scratch limit" in str(e.value)
    assert float(out.abs().max()) == 0.0

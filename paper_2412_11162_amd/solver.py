"""Thin Python layer over the C ABI (argument marshalling only; every step
of the computation runs in the HIP library)."""

from __future__ import annotations

import ctypes
from typing import Sequence, Tuple

import numpy as np
import torch

from . import _binding as B


class PmlbieError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("pmlbie error %d: %s" % (code, msg))
        self.code = code


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Solver:
    """One context of the HIP library on one device and stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream = None):
        self.L = B.load()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        rc = self.L.pmlbie_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise PmlbieError(rc, "pmlbie_create failed")
        self.h = h
        self.N = 0
        self.M = 0
        self.m0 = 0

    def close(self):
        if getattr(self, "h", None):
            self.L.pmlbie_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc: int):
        if rc != 0:
            raise PmlbieError(rc, self.L.pmlbie_last_error(self.h).decode())

    # -- the five calls of the method --------------------------------------
    def set_geometry(self, bumps: Sequence[Tuple[float, float, float]], cos_freq: float, rho_c: float,
                     seg_breaks: Sequence[float], nodes_per_segment: int):
        b = np.ascontiguousarray(np.array(bumps, dtype=np.float64).reshape(-1))
        s = np.ascontiguousarray(np.array(seg_breaks, dtype=np.float64))
        self._chk(self.L.pmlbie_set_geometry(self.h, len(bumps), _p(b), float(cos_freq), float(rho_c),
                                             _p(s), int(nodes_per_segment)))

    def set_polyline(self, verts: Sequence[Tuple[float, float]], panels: Sequence[int], grade: int):
        v = np.ascontiguousarray(np.array(verts, dtype=np.float64).reshape(-1))
        pn = np.ascontiguousarray(np.array(panels, dtype=np.int32))
        self._chk(self.L.pmlbie_set_polyline(self.h, v.size // 2, _p(v), _p(pn), int(grade)))

    def set_panels(self, nodes: np.ndarray):
        """nodes: [P, 16, 2] (rho, z) at the 16 Gauss-Legendre points of each panel."""
        a = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64).reshape(-1))
        self._chk(self.L.pmlbie_set_panels(self.h, a.size // 32, _p(a)))

    def set_media_pml(self, k1: complex, k2: complex, a1: float, T: float, S: float, a2: float,
                      T2: float, S2: float, p: int = 6):
        k1, k2 = complex(k1), complex(k2)
        self._chk(self.L.pmlbie_set_media_pml(self.h, k1.real, k1.imag, k2.real, k2.imag, a1, T, S,
                                              a2, T2, S2, int(p)))
        self.N = self.nodes().shape[0]

    def build_modal_operators(self, n_theta: int, m_max: int, precision: int = B.PMLBIE_FP64,
                              flags: int = 0, m_min: int = 0):
        """Modes m_min..m_max (m_min > 0: one batch of a mode-batched solve)."""
        self._chk(self.L.pmlbie_build_modal_operators_range(self.h, int(n_theta), int(m_min), int(m_max),
                                                            int(precision), int(flags)))
        self.M = int(self.info()[1])
        self.m0 = int(m_min)

    def solve_modes(self, incidences):
        n = len(incidences)
        arr = (B.pmlbie_incidence * n)()
        for r, inc in enumerate(incidences):
            if inc[0] == "point":
                arr[r].kind = 0
                arr[r].p[0], arr[r].p[1] = float(inc[1]), float(inc[2])
            else:
                arr[r].kind = 1
                arr[r].p[0] = float(inc[1])
        shape = (self.M - self.m0 + 1, n, self.N)
        dev = torch.device("cuda", self.device)
        outs = [torch.empty(shape, dtype=torch.complex128, device=dev) for _ in range(4)]
        self._chk(self.L.pmlbie_solve_modes(self.h, n, arr, *[ctypes.c_void_p(o.data_ptr()) for o in outs]))
        return tuple(outs)

    def evaluate_field(self, rtz: np.ndarray, n_rhs: int) -> np.ndarray:
        rtz = np.ascontiguousarray(np.asarray(rtz, dtype=np.float64).reshape(-1, 3))
        out = np.zeros((n_rhs, rtz.shape[0]), dtype=np.complex128)
        self._chk(self.L.pmlbie_evaluate_field(self.h, rtz.shape[0], _p(rtz), _p(out)))
        return out

    # -- inspection ----------------------------------------------------------
    def info(self) -> np.ndarray:
        a = np.zeros(9, dtype=np.int64)
        self._chk(self.L.pmlbie_get_info(self.h, _p(a)))
        return a

    def nodes(self) -> np.ndarray:
        n = int(self.info()[0])
        a = np.zeros((n, 13))
        self._chk(self.L.pmlbie_get_nodes(self.h, _p(a)))
        return a

    def modal_kernels(self, geom: np.ndarray) -> torch.Tensor:
        geom = np.ascontiguousarray(np.asarray(geom, dtype=np.float64).reshape(-1, 12))
        out = torch.empty((geom.shape[0], 4, self.M + 1), dtype=torch.complex128,
                          device=torch.device("cuda", self.device))
        self._chk(self.L.pmlbie_modal_kernels(self.h, geom.shape[0], _p(geom), ctypes.c_void_p(out.data_ptr())))
        return out

    def modal_kernels_noalloc(self, geom: np.ndarray, out: torch.Tensor) -> torch.Tensor:
        """The allocation-free variant: the caller provides the output
        ([n_pairs, 4, M + 1] complex128 on the device)."""
        geom = np.ascontiguousarray(np.asarray(geom, dtype=np.float64).reshape(-1, 12))
        assert out.dtype == torch.complex128 and out.is_contiguous()
        assert tuple(out.shape) == (geom.shape[0], 4, self.M + 1)
        self._chk(self.L.pmlbie_modal_kernels_noalloc(self.h, geom.shape[0], _p(geom),
                                                       ctypes.c_void_p(out.data_ptr())))
        return out

    def get_operator(self, mode: int) -> torch.Tensor:
        n2 = 2 * self.N
        out = torch.empty((n2, n2), dtype=torch.complex128, device=torch.device("cuda", self.device))
        self._chk(self.L.pmlbie_get_operator(self.h, int(mode), ctypes.c_void_p(out.data_ptr())))
        return out  # row-major storage

    # -- learned surrogate of the far-pair modes ---------------------------
    def surrogate_nparams(self) -> int:
        return int(self.L.pmlbie_surrogate_nparams())

    def surrogate_init(self, seed: int):
        self._chk(self.L.pmlbie_surrogate_init(self.h, int(seed)))

    def surrogate_make_samples(self, which: int, n: int, seed: int):
        self._chk(self.L.pmlbie_surrogate_make_samples(self.h, int(which), int(n), int(seed)))

    def surrogate_train(self, steps: int, batch: int, lr: float) -> np.ndarray:
        loss = np.zeros(max(int(steps), 1))
        self._chk(self.L.pmlbie_surrogate_train(self.h, int(steps), int(batch), float(lr), _p(loss)))
        return loss[:int(steps)]

    def surrogate_eval(self, which: int) -> float:
        m = np.zeros(1)
        self._chk(self.L.pmlbie_surrogate_eval(self.h, int(which), _p(m)))
        return float(m[0])

    def surrogate_eval_modes(self, which: int) -> np.ndarray:
        rel = np.zeros(65)
        self._chk(self.L.pmlbie_surrogate_eval_modes(self.h, int(which), _p(rel)))
        return rel

    def surrogate_set_tolerance(self, tol: float):
        self._chk(self.L.pmlbie_surrogate_set_tolerance(self.h, float(tol)))

    def surrogate_save(self) -> bytes:
        n = ctypes.c_size_t(0)
        self._chk(self.L.pmlbie_surrogate_save(self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._chk(self.L.pmlbie_surrogate_save(self.h, buf, ctypes.byref(n)))
        return buf.raw[:n.value]

    def surrogate_load(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._chk(self.L.pmlbie_surrogate_load(self.h, buf, len(blob)))

    def surrogate_params(self, p: np.ndarray = None) -> np.ndarray:
        """Get the FP32 parameters (as float64), or set them when p is given."""
        if p is None:
            out = np.zeros(self.surrogate_nparams())
            self._chk(self.L.pmlbie_surrogate_params(self.h, _p(out), 1))
            return out
        q = np.ascontiguousarray(p, dtype=np.float64)
        self._chk(self.L.pmlbie_surrogate_params(self.h, _p(q), 0))
        return q

    def surrogate_forward(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros((x.shape[0], 390))
        self._chk(self.L.pmlbie_surrogate_forward(self.h, x.shape[0], _p(x), _p(y)))
        return y

    def surrogate_grad(self, x: np.ndarray, t: np.ndarray):
        x = np.ascontiguousarray(x, dtype=np.float64)
        t = np.ascontiguousarray(t, dtype=np.float64)
        g = np.zeros(self.surrogate_nparams())
        loss = np.zeros(1)
        self._chk(self.L.pmlbie_surrogate_grad(self.h, x.shape[0], _p(x), _p(t), _p(loss), _p(g)))
        return float(loss[0]), g

    def surrogate_label(self, s: np.ndarray) -> np.ndarray:
        s = np.ascontiguousarray(s, dtype=np.float64)
        y = np.zeros((s.shape[0], 390))
        self._chk(self.L.pmlbie_surrogate_label(self.h, s.shape[0], _p(s), _p(y)))
        return y

    def set_refinement(self, tol: float, max_iter: int):
        self._chk(self.L.pmlbie_set_refinement(self.h, float(tol), int(max_iter)))

    def set_ch1_substitution(self, order: int):
        self._chk(self.L.pmlbie_set_ch1_substitution(self.h, int(order)))

    def test_zero_column(self, mode: int, col: int):
        self._chk(self.L.pmlbie_test_zero_column(self.h, int(mode), int(col)))

    def stats(self):
        s = np.zeros(16)
        c = np.zeros(16)
        self._chk(self.L.pmlbie_get_stats(self.h, _p(s), _p(c)))
        return s, c


def from_workload(wl, device: int = 0, n_theta: int = None, m_max: int = None,
                  precision: int = B.PMLBIE_FP64, flags: int = 0, build: bool = True) -> Solver:
    """Set up a solver for one of the synthetic workloads."""
    s = Solver(device)
    if wl.curve_nodes is not None:
        s.set_panels(wl.curve_nodes)
    elif wl.polyline:
        s.set_polyline(wl.polyline, wl.panels, wl.grade)
    else:
        s.set_geometry(wl.bumps, wl.cos_freq, wl.a1, wl.seg_breaks, wl.nodes_per_segment)
    s.set_media_pml(wl.k1, wl.k2, wl.a1, wl.T, wl.S, wl.a2, wl.T2, wl.S2, wl.p)
    if build:
        s.build_modal_operators(n_theta or wl.n_theta, wl.m_max if m_max is None else m_max,
                                precision, flags)
    return s

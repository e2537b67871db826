#!/usr/bin/env python3
"""Benchmark of the MI355X PML-BIE hot path.

One step = the whole hot path on the paper-scale workload (k1 = 10, k2 = 15,
h = 0.5 exp(-rho^2/2) cos(2 rho), PML rho in [4, 5.5], sigma0 = 3,
2048 curve nodes, 256 azimuthal samples with modes 0..128 kept, point source at
(0.3, 0, 1.2)): geometry and media set-up, pair x theta sampling of the
kernels, far / split / direct modal kernels, near-panel product integration,
assembly, per-mode LU of the 129 systems of size 4096, right-hand sides and
solves.  Prints one JSON line.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def gemm_traffic_record():
    """HBM bytes per launch of the trailing-update kernel from the committed
    rocprofv3 counter summary, or None when the kernel source has changed
    since the counters were taken (the record carries a digest of it)."""
    src = open(os.path.join(ROOT, "paper_2412_11162_amd", "csrc", "lu.hip")).read()
    a = src.index("void k_gemm_update(")
    digest = hashlib.sha256(src[a:src.index("\n}\n", a)].encode()).hexdigest()[:16]
    path = os.path.join(ROOT, "profiles", "k_gemm_update_paper_scale.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.strip().startswith("traffic-record"):
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            if kv.get("source_sha256_16") == digest:
                return float(kv["hbm_bytes_per_launch"])
    return None


def largest_run(s, wl, steps: int, warmup: int, batch: int = 86):
    """The largest one-GPU configuration (4096 nodes, modes 0..256, 16 plane
    waves) in mixed precision: its operators do not fit at once (276 GB in
    FP64), so each step builds, factors and solves the modes in three batches
    of up to 86 (FP64 operators for the residuals, complex64 factors and
    work space, ~170 GB per batch; every batch samples all pairs and keeps
    its modes).  Time to solution of
    all modes and right-hand sides; the refinement residual of every batch
    is held to 1e-10 by the library."""
    import torch

    def one():
        s.set_geometry(wl.bumps, wl.cos_freq, wl.a1, wl.seg_breaks, wl.nodes_per_segment)
        s.set_media_pml(wl.k1, wl.k2, wl.a1, wl.T, wl.S, wl.a2, wl.T2, wl.S2, wl.p)
        res, its, stages = [], [], []
        for lo in range(0, wl.m_max + 1, batch):
            hi = min(wl.m_max, lo + batch - 1)
            s.build_modal_operators(wl.n_theta, hi, 1, 0, m_min=lo)
            s.solve_modes(list(wl.incidences))
            st, cnt = s.stats()
            res.append(float(cnt[1]))
            its.append(int(cnt[0]))
            stages.append(st.copy())
            print("modes %d..%d done" % (lo, hi), file=sys.stderr, flush=True)
        return res, its, stages

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(steps):
        res, its, stages = one()
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.time() - t0) / max(steps, 1)
    info = s.info()
    N = int(info[0])
    units = 2.0 * N * N * (wl.m_max + 1)
    st = np.sum(np.array(stages), axis=0)
    return {"metric": "time-to-solution at 1e-6 rel err vs FP64 oracle; modal-kernel pairs*modes/s",
            "value": units / (ms_step * 1e-3), "unit": "pairs*modes/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "c64 LU + f64 refinement", "data": "synthetic",
            "config": {"workload": wl.name, "nodes": N, "unknowns_per_mode": 2 * N, "modes": wl.m_max + 1,
                       "n_theta": wl.n_theta, "media": 2, "precision": "mixed",
                       "incidence": "16 plane waves", "mode_batch": batch},
            "stage_ms_sum_over_batches": {"far": st[1], "split": st[2], "direct": st[3], "near": st[4],
                                          "lu": st[5], "solve": st[7], "refinement": st[9]},
            "refinement": {"max_final_rel_residual": max(res), "iterations": its},
            "note": "the surrogate covers modes 0..64 only; this configuration keeps modes 0..256"}


def surrogate_leg(s, wl, step, m_max: int = 64, tol: float = 1e-11):
    """The learned surrogate on this geometry: training on 2^22 labelled
    samples (timed apart, it is amortised over builds), then the step at
    m_max = 64 (the modes the network covers) with and without it; the
    surrogate step's error is measured against the plain FP64 step."""
    import torch
    from paper_2412_11162_amd import _binding as B

    t0 = time.time()
    s.surrogate_init(2412)
    s.surrogate_make_samples(0, 1 << 22, 2412_11162)
    s.surrogate_make_samples(1, 1 << 18, 2412_11163)
    t_samples = time.time() - t0
    t0 = time.time()
    loss = s.surrogate_train(4096, 1024, 1e-3)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    mse = s.surrogate_eval(1)

    def run(flags):
        s.set_geometry(wl.bumps, wl.cos_freq, wl.a1, wl.seg_breaks, wl.nodes_per_segment)
        s.set_media_pml(wl.k1, wl.k2, wl.a1, wl.T, wl.S, wl.a2, wl.T2, wl.S2, wl.p)
        t = time.time()
        s.build_modal_operators(wl.n_theta, m_max, 0, flags)
        sol = s.solve_modes(list(wl.incidences))
        torch.cuda.synchronize()
        return time.time() - t, [o.cpu().numpy() for o in sol], s.stats()

    s.surrogate_set_tolerance(tol)
    run(0)
    t_plain, ref, _ = run(0)
    t_sg, got, (st, cnt) = run(B.PMLBIE_USE_SURROGATE)
    xg = np.concatenate(got, axis=2)[:, 0]
    xr = np.concatenate(ref, axis=2)[:, 0]
    big = np.max(np.linalg.norm(xr, axis=1))
    err = max(float(np.linalg.norm(xg[j] - xr[j]) / max(np.linalg.norm(xr[j]), 1e-9 * big))
              for j in range(xr.shape[0]))
    return {"samples": {"train": 1 << 22, "held_out": 1 << 18, "seconds": t_samples},
            "training": {"steps": 4096, "batch": 1024, "seconds": t_train, "loss_first": float(loss[:64].mean()),
                         "loss_last": float(loss[-64:].mean()), "held_out_mse": mse},
            "m_max": m_max, "tolerance": tol, "far_pairs": int(cnt[4]), "accepted": int(cnt[5]),
            "acceptance": float(cnt[5]) / max(float(cnt[4]), 1.0),
            "ms_plain": 1e3 * t_plain, "ms_surrogate": 1e3 * t_sg, "speedup": t_plain / t_sg,
            "far_stage_ms": float(st[1]), "max_rel_err_vs_fp64": err}


def cpu_baseline(wl, seconds: float = 15.0):
    """The FP64 oracle's modal-kernel stage timed on this host on a bounded
    sample of (target, source) node pairs of the same workload."""
    import oracle
    import workloads
    g = oracle.geometry(wl)
    modes = list(range(wl.m_max + 1))
    ks = [wl.k1, wl.k2]
    pairs = workloads.seeded_pairs(g.n, 4096, seed=7)
    done = 0
    t0 = time.time()
    chunk = 8 * oracle.num_threads()
    while time.time() - t0 < seconds and done < len(pairs):
        oracle.modal_kernels_nodes(g, pairs[done:done + chunk], ks, modes)
        done += chunk
    dt = time.time() - t0
    units = done * len(ks) * len(modes)
    return {"value": units / dt, "unit": "pairs*modes/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d random node pairs of the %s workload, both media, modes 0..%d, "
                      "adaptive azimuthal quadrature (%.1f s)" % (done, wl.name, wl.m_max, dt)}


def field_leg(s, wl, N):
    """Field synthesis outside the timed step: 1024 seeded points off the curve
    in the physical region, the representation formula over every node and
    mode, evaluated by the library in chunks of point x node modal kernels."""
    nd = s.nodes()
    rng = np.random.default_rng(2412)
    npf = 1024
    rho_f = rng.uniform(0.05, 0.95 * wl.a1, npf)
    if wl.polyline or wl.curve_nodes is not None:
        # above the highest and below the lowest point of the curve
        z_f = np.where(rng.uniform(size=npf) < 0.5, nd[:, 2].max() + rng.uniform(0.2, 0.5, npf),
                       nd[:, 2].min() - rng.uniform(0.2, 0.5, npf))
    else:
        zc = np.interp(rho_f, nd[:, 0], nd[:, 2])
        z_f = zc + np.where(rng.uniform(size=npf) < 0.5, 1.0, -1.0) * rng.uniform(0.3, 0.6 * wl.a2, npf)
    rtz = np.stack([rho_f, rng.uniform(0.0, 2.0 * np.pi, npf), z_f], axis=1)
    nrhs = len(wl.incidences)
    s.evaluate_field(rtz[:8], nrhs)
    t0 = time.time()
    s.evaluate_field(rtz, nrhs)
    t_field = time.time() - t0
    return {"points": npf, "right_hand_sides": nrhs, "ms": 1e3 * t_field, "points_per_s": npf / t_field,
            "node_point_pairs_per_s": npf * N / t_field}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="paper_scale")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-field", action="store_true",
                    help="skip the field-synthesis leg (1024 points after the timed steps)")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the learned-surrogate leg (training + builds at m_max = 64)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes (calibrates "
                         "the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8}))
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the per-mode systems would shard "
              "across GPUs by mode); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2412_11162_amd.solver import Solver

    wl = workloads.ALL[args.workload]()
    s = Solver(0)
    if wl.name == "largest":
        print(json.dumps(largest_run(s, wl, args.steps, args.warmup)))
        return

    def step(precision=0):
        if wl.curve_nodes is not None:
            s.set_panels(wl.curve_nodes)
        elif wl.polyline:
            s.set_polyline(wl.polyline, wl.panels, wl.grade)
        else:
            s.set_geometry(wl.bumps, wl.cos_freq, wl.a1, wl.seg_breaks, wl.nodes_per_segment)
        s.set_media_pml(wl.k1, wl.k2, wl.a1, wl.T, wl.S, wl.a2, wl.T2, wl.S2, wl.p)
        s.build_modal_operators(wl.n_theta, wl.m_max, precision)
        return s.solve_modes(list(wl.incidences))

    for _ in range(args.warmup):
        step()
        print("warmup step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    times = []
    stages = []
    counts = []
    t_all = time.time()
    for k in range(args.steps):
        t0 = time.time()
        step()
        torch.cuda.synchronize()
        times.append(time.time() - t0)
        sk, ck = s.stats()
        stages.append(sk.copy())
        counts.append(ck.copy())
        print("step %d: %.1f ms" % (k, 1e3 * times[-1]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.time() - t_all
    ms_step = 1e3 * total / args.steps
    info = s.info()
    N, M = int(info[0]), int(info[1])
    units = 2.0 * N * N * (M + 1)
    st = np.mean(np.array(stages), axis=0)
    kernel_ms = st[1] + st[2] + st[3] + st[4]
    # trailing-update kernel: algorithmic flops of all its launches (counted by
    # the library, 8 real flops per complex multiply-add) over the summed
    # durations of those launches (HIP events on the streams they run on)
    gemm_ms = st[6]
    flops = float(counts[-1][2])
    launches = int(counts[-1][3])
    achieved = flops / (gemm_ms * 1e-3) / 1e12 if gemm_ms > 0 else 0.0
    peak = 78.6
    out = {
        "metric": "time-to-solution at 1e-6 rel err vs FP64 oracle; modal-kernel pairs*modes/s",
        "value": units / (ms_step * 1e-3),
        "unit": "pairs*modes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": wl.name, "nodes": N, "unknowns_per_mode": 2 * N, "modes": M + 1,
                   "n_theta": wl.n_theta, "media": 2, "precision": "fp64",
                   "incidence": ", ".join("point source (%.1f, 0, %.1f)" % (inc[1], inc[2]) if inc[0] == "point"
                                          else "plane wave (polar angle %.2f)" % inc[1] for inc in wl.incidences)},
        "time_to_solution_s": ms_step * 1e-3,
        "kernel_stage_pairs_modes_per_s": units / (kernel_ms * 1e-3) if kernel_ms > 0 else None,
        "stage_ms": {"setup": st[0], "far": st[1], "split": st[2], "direct": st[3], "near": st[4],
                     "lu": st[5], "lu_trailing_update": st[6], "solve": st[7], "rhs": st[8],
                     "build": st[10]},
        "pair_classes": {"far": int(info[4]), "split": int(info[5]), "direct": int(info[6]),
                         "aux_near_points": int(info[7])},
        "roofline": {"bound": "mfma", "kernel": "k_gemm_update<double> (LU trailing update)",
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": gemm_traffic_record() if wl.name == "paper_scale" else None,
                     "traffic_unit": "bytes per launch", "launches": launches, "flop_per_launch": flops / max(launches, 1),
                     "avg_launch_ms": gemm_ms / max(launches, 1)},
    }
    if not args.no_field:
        out["field"] = field_leg(s, wl, N)
    if not args.no_mixed:
        # complex64 LU on FP32 MFMA + FP64 refinement, same workload; its error
        # is measured against this run's FP64 result (which the parity tests
        # hold to the FP64 oracle)
        ref = [o.cpu().numpy() for o in step(0)]
        step(1)
        torch.cuda.synchronize()
        tm = []
        for k in range(args.steps):
            t0 = time.time()
            sol = step(1)
            torch.cuda.synchronize()
            tm.append(time.time() - t0)
            print("mixed step %d: %.1f ms" % (k, 1e3 * tm[-1]), file=sys.stderr, flush=True)
        got = [o.cpu().numpy() for o in sol]
        xg = np.concatenate(got, axis=2)[:, 0]
        xr = np.concatenate(ref, axis=2)[:, 0]
        big = np.max(np.linalg.norm(xr, axis=1))
        errs = []
        for j in range(xr.shape[0]):
            nr = np.linalg.norm(xr[j])
            d = np.linalg.norm(xg[j] - xr[j])
            errs.append(d / nr if nr > 1e-9 * big else d / big)
        stm, cnt = s.stats()
        ms_mixed = 1e3 * float(np.mean(tm))
        out["mixed_precision"] = {
            "ms_per_step": ms_mixed, "value": units / (ms_mixed * 1e-3), "unit": "pairs*modes/s",
            "speedup_vs_fp64": ms_step / ms_mixed, "dtype": "c64 LU + f64 refinement",
            "max_rel_err_vs_fp64": float(np.max(errs)), "refinement_iterations": int(cnt[0]),
            "final_rel_residual": float(cnt[1]),
            "stage_ms": {"lu": stm[5], "lu_trailing_update": stm[6], "solve": stm[7], "refinement": stm[9]},
            "lu_trailing_update_tflops": float(cnt[2]) / (stm[6] * 1e-3) / 1e12 if stm[6] > 0 else None,
        }
    if not args.no_surrogate and wl.name == "paper_scale":
        out["surrogate"] = surrogate_leg(s, wl, step)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

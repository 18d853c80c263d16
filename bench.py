#!/usr/bin/env python3
"""Throughput of the AIMx matvec on one MI355X.

One step = one application of the AIMx operator (eq. LAIMx) to one input
vector: projection onto the grid, pruned zero-padded 3-D FFT, multiplication
by the kernel spectrum, inverse FFT, interpolation and the sparse near-field
correction -- all in the library's HIP kernels.  Inputs are resident in HBM
when the timed region starts.

Default workload: the largest single-GPU operator, a radius-6 sphere meshed
as a level-7 icosphere (327,680 triangles, 2nd-order stencils, 256^3 grid
zero-padded to 512^3, near threshold 2h, k = 2 pi), complex128.  The same
line carries, as extra keys, the complex64 figure on that operator, the
512-vector frequency sweep (64 wavenumbers x 8 right-hand sides on the
1,280-triangle sphere) and the 57,600-triangle box array.  Prints one JSON
line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2009_02281_amd", "csrc", "kernels.hip")


def algorithmic_bytes(info: dict, prec: str, nrhs: int = 1) -> dict:
    """Bytes each matvec kernel must move at minimum (per launch over nrhs
    right-hand sides); b = bytes per complex value, s = per real value."""
    b = 16 if prec == "c128" else 8
    s = b // 2
    N, Ng, nnz = info["n"], info["n_grid"], info["nnz"]
    Nq = 3 * N
    dims = info["dims"]
    nfold = (dims[0] + 1) * (dims[1] + 1) * (dims[2] + 1)
    qp = Nq * (4 + 4 * s)              # packed stencil start + 3 local coordinates + weight
    return {
        "project": nrhs * (N * b + Ng * b) + qp,
        "fft_x_fwd": nrhs * 3 * Ng * b,    # read Ng, write 2 Ng
        "fft_y_fwd": nrhs * 6 * Ng * b,    # read 2 Ng, write 4 Ng
        "fft_z_conv": nrhs * 8 * Ng * b + nfold * b,   # read/write 4 Ng, spectrum once
        "fft_y_inv": nrhs * 6 * Ng * b,
        "fft_x_inv": nrhs * 3 * Ng * b,
        "interp_near": nrhs * (Ng * b + 2 * N * b) + qp + nnz * (4 + s) + 4 * (N + 1),
    }


def merge_fused(kms: dict, ab: dict, sched, info: dict, prec: str, nrhs: int) -> None:
    """With the projection fused into the x forward pass (stage-mode bit 1)
    the two are one kernel: one stage that reads x and the stencil records
    and writes the padded rows, the grid q neither stored nor read."""
    if not sched or not sched[6] & 2:
        return
    gq = nrhs * info["n_grid"] * (16 if prec == "c128" else 8)
    kms["project+fft_x_fwd"] = kms.pop("project") + kms.pop("fft_x_fwd")
    ab["project+fft_x_fwd"] = ab.pop("project") + ab.pop("fft_x_fwd") - 2 * gq


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 5) -> dict:
    """A plain device-to-device copy of nbytes (read + write), timed with HIP
    events: the streaming bandwidth this GPU reaches, beside the nominal one."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del a, b
    return {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "ms": ms,
            "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}


def make_workload(name: str):
    from paper_2009_02281_amd import inputs as I
    return {"boxarray": I.box_array_large, "sphere": I.sphere_small,
            "sphere-large": I.sphere_large, "sweep": I.sweep_small}[name]()


def kernel_sha() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(kernel: str, workload: str, prec: str, schedule=None):
    """HBM bytes per launch from the committed rocprofv3 counter runs, only if
    they were taken on the current kernel source and, for an FFT pass, with
    the same launch shape of that pass and the same workspace layout."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(f"{workload}/{prec}/{kernel}")
    if not ent or ent.get("kernel_sha") != kernel_sha():
        return None
    passes = ["fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv"]
    if kernel in passes and schedule is not None:
        k = passes.index(kernel)
        for taken in (ent.get("schedule"), ent.get("schedule_write")):
            if taken is None or taken[k] != schedule[k] or taken[5] != schedule[5]:
                return None
    return ent.get("bytes_per_launch")


def host_threads() -> int:
    """Threads the oracle may use: the CPUs this process may run on, at most
    16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(w, x, reps: int = 3, near_rows: int = 512) -> dict:
    """The oracle (NumPy/SciPy float64) timed on this host: the whole far part
    (projection, zero-padded FFT convolution over the full padded grid,
    interpolation) plus the near-field correction on a row sample, scaled to
    all rows -- an estimate of one full oracle matvec.  Median of ``reps``
    runs with the host's threads, then one run with a single thread (the
    paper's own set-up ran single-threaded)."""
    import numpy as np
    import scipy.sparse as sp
    from oracle import aimx
    threads = host_threads()
    aimx.FFT_WORKERS = threads
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    k = float(w.k[0])
    o.spectrum(k)
    rows = np.sort(np.random.default_rng(5).choice(o.N, min(near_rows, o.N), replace=False))
    r, c, v = o.correction_rows(rows)
    Cs = sp.csr_matrix((v, (r, c)), shape=(o.N, o.N))

    def once():
        t0 = time.perf_counter()
        o.far(x, k)
        t1 = time.perf_counter()
        Cs @ x
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    runs = [once() for _ in range(reps)]
    t_far = sorted(a for a, _ in runs)[reps // 2]
    t_near = sorted(b for _, b in runs)[reps // 2]
    t = t_far + t_near * o.N / rows.size
    aimx.FFT_WORKERS = 1
    f1, n1 = once()
    aimx.FFT_WORKERS = -1
    t1 = f1 + n1 * o.N / rows.size
    padded = "x".join(str(2 * d) for d in w.dims)
    return {"value": o.N / t, "unit": "unknowns*matvecs/s", "cores": threads,
            "kind": "estimate",
            "sample": (f"one oracle matvec of the same workload, estimated: the full far part "
                       f"(P x, scipy.fft over the {padded} padded grid with {threads} "
                       f"workers, P^T) timed whole, the near correction timed on "
                       f"{rows.size} sampled rows and scaled by {o.N}/{rows.size}; median "
                       f"of {reps}; oracle set-up excluded"),
            "single_thread": {"value": o.N / t1, "unit": "unknowns*matvecs/s", "cores": 1,
                              "seconds_per_matvec": t1, "runs": 1},
            "seconds_per_matvec": t}


RESTART = 60


def cpu_gmres_leg(rtol: float) -> dict:
    """GMRES(RESTART) to rtol for the +z plane wave on the 1,280-triangle
    sphere: the oracle (NumPy/SciPy float64 FGMRES on this host, operator
    set-up excluded) beside the library's complex128 solve on the GPU.  Each
    side builds its own right-hand side."""
    import numpy as np
    import torch
    from oracle import aimx, excitation, solver
    from paper_2009_02281_amd import binding
    w = make_workload("sphere")
    k = float(w.k[0])
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    o.spectrum(k)
    _ = o.C
    b = excitation.plane_wave(w.vertices, w.triangles, k, (0.0, 0.0, 1.0))
    t0 = time.perf_counter()
    _, info = solver.fgmres(lambda v: o.matvec(v, k), b, tol=rtol, restart=RESTART,
                            max_iter=4000)
    t_cpu = time.perf_counter() - t0
    plan = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k)
    bg = plan.excitation("plane_wave", [0.0, 0.0, 1.0])
    plan.solve(bg, rtol=1e-2, restart=RESTART, max_iter=30, raise_on_fail=False)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, r = plan.solve(bg, rtol=rtol, restart=RESTART, max_iter=4000, raise_on_fail=False)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    plan.close()
    return {"workload": f"{w.name} (N={w.n}, grid {list(w.dims)}, k={k})", "rtol": rtol,
            "restart": RESTART, "cpu": {"seconds": t_cpu, "iters": int(info.iters),
                                        "rel_resid": float(info.rel_resid),
                                        "converged": bool(info.converged),
                                        "cores": os.cpu_count() or 1, "kind": "oracle"},
            "gpu": {"seconds": t_gpu, "iters": int(r.iters[0]),
                    "rel_resid": float(r.rel_resid[0]), "converged": bool(r.converged[0]),
                    "precision": "c128"}}


def solve_leg(plan, rtol: float, max_iter: int = 4000,
              pcs=("none", "diag", "nearblock")) -> dict:
    """Time to rtol for the +z plane wave: complex128 GMRES(RESTART) without
    preconditioner (the reference) against complex64-matvec GMRES inside
    complex128 refinement, each also with the static diagonal and the
    near-field block preconditioner."""
    import torch
    b = plan.excitation("plane_wave", [0.0, 0.0, 1.0])
    runs = [(inner, pc) for inner in ("c128", "c64") for pc in pcs]
    res = {}
    for inner, pc in runs:
        plan.solve(b, rtol=1e-2, restart=RESTART, max_iter=30, inner=inner, pc=pc,
                   raise_on_fail=False)                    # warm-up (workspace, graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # max_refine 4: the complex64 runs converge in 2-3 refinement steps; a
        # run that stalls stops after 4 x max_iter inner steps
        x, r = plan.solve(b, rtol=rtol, restart=RESTART, max_iter=max_iter, inner=inner, pc=pc,
                          max_refine=4, raise_on_fail=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[f"{inner}+{pc}"] = {"seconds": dt, "iters": int(r.iters[0]),
                                "matvecs": int(r.matvecs[0]),
                                "refinements": int(r.refinements[0]),
                                "rel_resid": float(r.rel_resid[0]),
                                "converged": bool(r.converged[0])}
        print(f"[bench] gmres {inner}+{pc}: {dt:.3f}s iters={r.iters[0]} "
              f"resid={r.rel_resid[0]:.2e}", file=sys.stderr, flush=True)
    return {"rtol": rtol, "rhs": "plane wave +z", "restart": RESTART, "max_iter": max_iter,
            "runs": res}


def batch_leg(rtol: float, pcs=("diag", "nearblock"), restart: int = RESTART) -> dict:
    """One batched solve over 32 uneven geometries behind one plan
    (aim_setup_batch; the instances' matvecs run concurrently on the plan's
    worker streams) against the same 32 systems solved one after another on
    their own plans: GMRES(RESTART) to rtol, complex64 matvecs inside
    complex128 refinement, a +z plane wave per instance (each computed on its
    own plan), for each preconditioner in pcs."""
    import numpy as np
    import torch
    from paper_2009_02281_amd import binding
    from paper_2009_02281_amd import inputs as I
    ws = I.uneven_batch()
    t0 = time.perf_counter()
    plans = [binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k)
             for w in ws]
    t_sep_setup = time.perf_counter() - t0
    bs = [p.excitation("plane_wave", [0.0, 0.0, 1.0]) for p in plans]
    t0 = time.perf_counter()
    bp = binding.Plan.setup_batch(ws)
    t_batch_setup = time.perf_counter() - t0
    B = bp.pack([b[0] for b in bs])
    out = {"instances": len(ws), "triangles_total": int(sum(w.n for w in ws)),
           "triangles_range": [int(min(w.n for w in ws)), int(max(w.n for w in ws))],
           "k_range": [float(min(w.k[0] for w in ws)), float(max(w.k[0] for w in ws))],
           "grids": sorted({"x".join(map(str, w.dims)) for w in ws}),
           "kinds": [w.extra["kind"] for w in ws], "k": [float(w.k[0]) for w in ws],
           "rtol": rtol, "restart": restart, "inner": "c64",
           "setup_seconds": {"batched": t_batch_setup, "one_after_another": t_sep_setup},
           "runs": {}}
    for pc in pcs:
        opts = dict(rtol=rtol, restart=restart, max_iter=4000, pc=pc, inner="c64", max_refine=4,
                    raise_on_fail=False)
        warm = dict(rtol=1e-2, restart=restart, max_iter=20, pc=pc, inner="c64",
                    raise_on_fail=False)
        bp.solve(B, **warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, r = bp.solve(B, **opts)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        print(f"[bench] batch of {len(ws)} ({pc}): one batched solve {t_batch:.3f}s, iters "
              f"{int(r.iters.min())}..{int(r.iters.max())}, converged {int(r.converged.sum())}",
              file=sys.stderr, flush=True)
        sep_s, sep_it, sep_conv = 0.0, [], 0
        for p, b in zip(plans, bs):
            p.solve(b, **warm)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, ri = p.solve(b, **opts)
            torch.cuda.synchronize()
            sep_s += time.perf_counter() - t0
            sep_it.append(int(ri.iters[0]))
            sep_conv += int(ri.converged[0])
        print(f"[bench] batch of {len(ws)} ({pc}): one after another {sep_s:.3f}s, converged "
              f"{sep_conv}", file=sys.stderr, flush=True)
        out["runs"][pc] = {"batched": {"seconds": t_batch, "iters": r.iters.tolist(),
                                       "converged": int(r.converged.sum()),
                                       "unconverged": [int(i) for i in
                                                       np.nonzero(~r.converged)[0]]},
                           "one_after_another": {"seconds": sep_s, "iters": sep_it,
                                                 "converged": sep_conv}}
    bp.close()
    for p in plans:
        p.close()
    return out


def batch_learned_leg(rtol: float, restart: int = 200, pairs: int = 20000,
                      epochs: int = 8) -> dict:
    """The learned preconditioner at the uneven batch's scale.  Pairs are
    logged from plain complex128 GMRES(12) to 1e-8 on uneven training
    geometries of their own seed (5004; 40 spheres, boxes and box arrays of
    5k-16k triangles, grids from 32^3 to 64x128x32, eight plane waves each), the
    network is trained on them with the residual loss over the diagonal
    preconditioner, and the 32-instance batch (seed 5003) is then solved in
    one batched solve with pc=unet (complex64 matvecs in complex128
    refinement, diagonal base and fallback) against the classical batched
    runs.  Reported whichever way it falls."""
    import numpy as np
    import torch
    from paper_2009_02281_amd import binding
    from paper_2009_02281_amd import inputs as I
    rng = np.random.default_rng(5006)

    def dirs(n):
        d = rng.standard_normal((n, 3))
        return d / np.linalg.norm(d, axis=1, keepdims=True)

    train = I.uneven_batch(count=40, seed=5004, n_range=(5000, 16000))
    per = max(1, pairs // len(train))
    t0 = time.perf_counter()
    data, err2, res2, count, skipped = [], 0.0, 0.0, 0, 0
    for w in train:
        p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                         max_rhs=8)
        try:
            r, e, _ = p.log_pairs(p.excitation("plane_wave", dirs(8)), rtol=1e-8, restart=12,
                                  max_iter=4000, max_pairs=per)
        except binding.AimError as err:
            if err.status != 6:  # not converged: its errors e_t would be inexact
                raise
            skipped += 1
            p.close()
            continue
        grids, ts, sums = p.pc_targets(r, e, base_pc="diag", loss="residual")
        del r, e
        data.append((p, grids, ts))
        err2, res2, count = err2 + sums[0], res2 + sums[1], count + grids.shape[0] * p.n
    torch.cuda.synchronize()
    t_log = time.perf_counter() - t0
    npairs = sum(d[1].shape[0] for d in data)
    print(f"[bench] batch learned: {npairs} pairs from {len(data)} geometries ({skipped} "
          f"skipped: plain GMRES did not converge) in {t_log:.1f}s", file=sys.stderr, flush=True)
    tau, weight = math.sqrt(err2 / count), count / res2
    net = binding.UNet(seed=61)
    order_rng = np.random.default_rng(62)
    t0 = time.perf_counter()
    loss = []
    for _ in range(epochs):
        # batches of eight pairs of one geometry (their grids share a shape),
        # the batches of all geometries shuffled together: consecutive steps
        # from one geometry overfit it and undo the previous ones
        batches = []
        for gi, (p, grids, ts) in enumerate(data):
            idx = order_rng.permutation(grids.shape[0])
            batches += [(gi, idx[s0:s0 + 8]) for s0 in range(0, len(idx), 8)]
        tot = 0.0
        for bi in order_rng.permutation(len(batches)):
            gi, idx = batches[bi]
            p, grids, ts = data[gi]
            tot += p.pc_train_step(net, grids, ts, idx, tau=tau, weight=weight,
                                   loss="residual", lr=1e-3)
        loss.append(tot / max(1, len(batches)))
        print(f"[bench] batch learned: epoch loss {loss[-1]:.4f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ngeom = len(data)
    for p, _, _ in data:
        p.close()
    del data
    ws = I.uneven_batch()
    solo = [binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k)
            for w in ws]
    bs = [q.excitation("plane_wave", [0.0, 0.0, 1.0])[0] for q in solo]
    for q in solo:
        q.close()
    bp = binding.Plan.setup_batch(ws)
    bp.set_unet(net, base_pc="diag", tau=tau)
    B = bp.pack(bs)
    runs = {}
    for inner, pc in (("c128", "none"), ("c128", "diag"), ("c64", "diag"), ("c64", "unet")):
        opts = dict(rtol=rtol, restart=restart, max_iter=10000, pc=pc, inner=inner,
                    max_refine=4, fallback_pc="diag", raise_on_fail=False)
        bp.solve(B, **dict(opts, rtol=1e-2, max_iter=20))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, r = bp.solve(B, **opts)
        torch.cuda.synchronize()
        runs[f"{inner}+{pc}"] = {"seconds": time.perf_counter() - t0,
                                 "iters_max": int(r.iters.max()),
                                 "iters_sum": int(r.iters.sum()),
                                 "converged": int(r.converged.sum()),
                                 "fallback_used": bool(r.fallback_used.any())}
        print(f"[bench] batch learned {inner}+{pc}: {runs[f'{inner}+{pc}']}", file=sys.stderr,
              flush=True)
    bp.set_unet(None)
    bp.close()
    net.close()
    return {"rtol": rtol, "restart": restart, "training_geometries": ngeom,
            "training_geometries_skipped": skipped,
            "training_pairs": npairs, "log_seconds": t_log, "train_seconds": t_train,
            "epochs": epochs, "train_loss": loss, "tau": tau, "instances": len(ws), "runs": runs}


def learned_pc_leg(rtol: float) -> dict:
    """GMRES time to rtol on a held-out ellipsoid (4 plane waves, batched):
    complex128 GMRES without and with the near-block preconditioner against
    complex64-matvec GMRES in complex128 refinement with the learned grid
    preconditioner (diagonal base, near-block fallback).  The network is
    trained first on pairs logged from plain GMRES on three other ellipsoids;
    logging and training are timed separately."""
    import numpy as np
    import torch
    from paper_2009_02281_amd import binding
    from paper_2009_02281_amd import inputs as I

    def plan(w):
        return binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold,
                            w.k, max_rhs=8)

    rng = np.random.default_rng(5006)

    def dirs(n):
        d = rng.standard_normal((n, 3))
        return d / np.linalg.norm(d, axis=1, keepdims=True)

    t0 = time.perf_counter()
    data, err2, res2, count = [], 0.0, 0.0, 0
    for w in I.learned_pc_geometries(3):
        p = plan(w)
        r, e, _ = p.log_pairs(p.excitation("plane_wave", dirs(8)), rtol=1e-9, restart=6,
                              max_pairs=256)
        grids, ts, sums = p.pc_targets(r, e, base_pc="diag", loss="residual")
        data.append((p, grids, ts))
        err2, res2, count = err2 + sums[0], res2 + sums[1], count + r.shape[0] * p.n
    torch.cuda.synchronize()
    t_log = time.perf_counter() - t0
    tau, weight = math.sqrt(err2 / count), count / res2
    net = binding.UNet(seed=61)
    order_rng = np.random.default_rng(62)
    t0 = time.perf_counter()
    loss = []
    for _ in range(10):
        tot, nb = 0.0, 0
        for gi in order_rng.permutation(len(data)):
            p, grids, ts = data[gi]
            idx = order_rng.permutation(grids.shape[0])
            for s0 in range(0, len(idx), 8):
                tot += p.pc_train_step(net, grids, ts, idx[s0:s0 + 8], tau=tau, weight=weight,
                                       loss="residual", lr=2e-3)
                nb += 1
        loss.append(tot / nb)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    w = I.learned_pc_geometries(1, seed=5005)[0]
    p = plan(w)
    p.set_unet(net, base_pc="diag", tau=tau)
    b = p.excitation("plane_wave", dirs(4))
    runs = {}
    for inner, pc in (("c128", "none"), ("c128", "nearblock"), ("c64", "nearblock"),
                      ("c64", "unet")):
        p.solve(b, rtol=1e-2, restart=RESTART, max_iter=20, inner=inner, pc=pc,
                fallback_pc="nearblock", raise_on_fail=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, r = p.solve(b, rtol=rtol, restart=RESTART, max_iter=4000, inner=inner, pc=pc,
                       fallback_pc="nearblock", raise_on_fail=False)
        torch.cuda.synchronize()
        runs[f"{inner}+{pc}"] = {"seconds": time.perf_counter() - t0,
                                 "iters": r.iters.tolist(),
                                 "fallback_used": bool(r.fallback_used.any()),
                                 "converged": bool(r.converged.all())}
        print(f"[bench] learned-pc leg {inner}+{pc}: {runs[f'{inner}+{pc}']}", file=sys.stderr,
              flush=True)
    p.set_unet(None)
    net.close()
    return {"rtol": rtol, "workload": f"{w.name} (N={w.n}, grid {list(w.dims)}, k={w.k[0]})",
            "rhs": "4 plane waves, one batch", "training_pairs": sum(d[1].shape[0] for d in data),
            "log_seconds": t_log, "train_seconds": t_train, "train_loss": loss, "runs": runs}


MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense bf16, published


def unet_flops(P0: int, C: int = 16) -> float:
    """Multiply-adds x 2 of one U-Net forward pass on P0 grid points: the
    3x3x3 convolutions at full, 1/8 and 1/64 resolution plus the 1x1 output."""
    c0, c1, c2 = C, 2 * C, 4 * C
    full = [(2, c0), (c0, c0), (c1 + c0, c0), (c0, c0)]
    half = [(c0, c1), (c1, c1), (c2 + c1, c1), (c1, c1)]
    quarter = [(c1, c2), (c2, c2)]
    f = sum(2 * 27 * ci * co * P0 for ci, co in full)
    f += sum(2 * 27 * ci * co * P0 / 8 for ci, co in half)
    f += sum(2 * 27 * ci * co * P0 / 64 for ci, co in quarter)
    return f + 2 * c0 * 2 * P0


def unet_leg(dims=(64, 64, 64), reps: int = 20, batches=(1, 8)) -> dict:
    """Forward pass and training step (forward + backward + Adam) of the
    learned preconditioner's network on one grid and on a batch of grids
    (stacked along z, one pass), timed with events on the stream the kernels
    run on; bf16 MFMA roofline."""
    import numpy as np
    import torch
    from paper_2009_02281_amd import binding
    net = binding.UNet(seed=1)
    nx, ny, nz = dims
    P0 = nx * ny * nz
    res = {}
    for nb in batches:
        g = torch.from_numpy((np.random.default_rng(7).standard_normal((nb, nz, ny, nx, 2)))
                             .astype(np.float32)).view(torch.complex64)[..., 0].contiguous().cuda()
        t = torch.zeros_like(g)
        for name, fn, mult in (("forward", lambda: net.forward(g), 1.0),
                               ("train_step", lambda: net.train_grid(g, t, lr=1e-4), 3.0)):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            tf = mult * nb * unet_flops(P0) / (ms * 1e-3) / 1e12
            key = name if nb == 1 else f"{name}_batch{nb}"
            res[key] = {"ms": ms, "tflops": tf, "frac_bf16_peak": tf / MFMA_BF16_PEAK_TFLOPS}
            print(f"[bench] unet {key} {list(dims)}: {ms:.3f} ms, {tf:.1f} TFLOP/s",
                  file=sys.stderr, flush=True)
        del g, t
    net.close()
    return {"grid": list(dims), "flops_forward": unet_flops(P0),
            "note": "train_step counted as 3x the forward flops (data and weight gradients); "
                    "it also holds host synchronisation for the loss; _batchN: N grids in one "
                    "pass", **res}


def time_matvecs(plan, x, y, prec: str, steps: int, warmup: int, freq=None) -> float:
    """ms per matvec call, back to back between two events on the stream the
    library launches on (torch's current stream)."""
    import torch
    for _ in range(warmup):
        plan.matvec(x, prec=prec, out=y, freq_idx=freq)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        plan.matvec(x, prec=prec, out=y, freq_idx=freq)
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def extra_workload(name: str, precs, steps: int, warmup: int) -> dict:
    """Throughput of another workload (its own plan, autotuned schedules) in
    the given precisions: the sweep runs all 512 vectors per launch, vector r
    at wavenumber r mod 64; the others one vector."""
    import numpy as np
    import torch
    from paper_2009_02281_amd import binding
    from paper_2009_02281_amd import inputs as I
    w = make_workload(name)
    freq, nrhs = None, 1
    if name == "sweep":
        nrhs = 8 * len(w.k)
        freq = np.arange(nrhs) % len(w.k)
    plan = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                        precisions=precs, max_rhs=nrhs)
    info = plan.info()
    xh = I.complex_gaussian(w.n, w.seed_base + 1, nrhs=nrhs)
    res = {"workload": w.name, "triangles": w.n, "grid": list(w.dims), "nrhs": nrhs,
           "n_freq": int(len(w.k))}
    for pr in precs:
        plan.autotune(prec=pr, nrhs=nrhs, reps=5)
        dt = torch.complex128 if pr == "c128" else torch.complex64
        x = torch.from_numpy(xh).to(dt).cuda()
        y = torch.empty_like(x)
        ms = time_matvecs(plan, x, y, pr, steps, warmup, freq)
        ab = sum(algorithmic_bytes(info, pr, nrhs).values())
        res[pr] = {"ms_per_launch": ms, "unknowns_matvecs_per_s": w.n * nrhs / (ms * 1e-3),
                   "alg_gbs": ab / (ms * 1e-3) / 1e9}
        print(f"[bench] extra {w.name} {pr}: {ms:.4f} ms per launch of {nrhs} -> "
              f"{res[pr]['unknowns_matvecs_per_s']:.4e} unknowns*matvecs/s", file=sys.stderr,
              flush=True)
    plan.close()
    return res


def dlp_leg(plan, w, reps: int = 20) -> dict:
    """The double-layer operator under AIMx (Sec. III-B) on the same plan:
    its one-time tables (near values on the device, one spectrum of the
    gradient channels' radial factor per wavenumber) and the per-call time
    of K x against the single-layer matvec A x (complex128, one vector)."""
    import torch
    from paper_2009_02281_amd import inputs as I
    x = torch.from_numpy(I.complex_gaussian(w.n, w.seed_base + 9)).cuda()
    y = torch.empty_like(x)
    t0 = time.perf_counter()
    plan.matvec_dlp(x, out=y)
    torch.cuda.synchronize()
    first = time.perf_counter() - t0
    for _ in range(2):
        plan.matvec_dlp(x, out=y)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        plan.matvec_dlp(x, out=y)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    res = {"workload": w.name, "first_call_seconds": first, "ms_per_matvec": ms,
           "unknowns_matvecs_per_s": w.n / (ms * 1e-3),
           "note": "complex128; three gradient channels transformed forward, summed against "
                   "the spectra of the components of grad G in one z pass, one grid "
                   "transformed back; the first call builds the tables"}
    print(f"[bench] double layer on {w.name}: {ms:.3f} ms per matvec (first call "
          f"{first:.2f}s)", file=sys.stderr, flush=True)
    return res


def efie_leg(reps: int = 20) -> dict:
    """The RWG operators under AIMx on the 81,920-triangle sphere (122,880
    functions, 128^3 grid): the tables' build times and the per-call times of
    the EFIE Z x (Sec. II-A, II-B), the double layer (K - G/2) x and the
    combined field of eq. CFIEAIMx (Sec. III-B), complex128, for one and four
    vectors, beside the scalar single-layer product A x on the same plan."""
    import torch
    from paper_2009_02281_amd import binding
    from paper_2009_02281_amd import inputs as I
    w = I.efie_sphere()
    t0 = time.perf_counter()
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                     precisions=("c128", "c64"), max_rhs=4)
    plan_s = time.perf_counter() - t0
    info = p.efie_setup()

    def timed(fn, x, y):
        for _ in range(2):
            fn(x, out=y)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            fn(x, out=y)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    res = {"workload": w.name, "triangles": int(w.triangles.shape[0]), "n_rwg": info["n_rwg"],
           "rwg_near_nnz": info["nnz"], "plan_seconds": plan_s,
           "efie_tables_seconds": info["seconds"]}
    ops = (("efie", p.matvec_efie), ("mfie", lambda x, out: p.matvec_mfie(x, gram_coef=-0.5,
                                                                          out=out)),
           ("cfie", lambda x, out: p.matvec_cfie(x, gram_coef=-0.5, out=out)))
    x1 = torch.from_numpy(I.complex_gaussian(info["n_rwg"], w.seed_base + 1)).cuda()
    p.matvec_mfie(x1, out=torch.empty_like(x1))      # builds the double layer's tables
    res["mfie_tables_seconds"] = p.mfie_values()["seconds"]
    for nrhs in (1, 4):
        x = torch.from_numpy(I.complex_gaussian(info["n_rwg"], w.seed_base + nrhs,
                                                nrhs=nrhs)).cuda()
        for name, fn in ops:
            ms = timed(fn, x, torch.empty_like(x))
            key = f"nrhs{nrhs}" if name == "efie" else f"{name}_nrhs{nrhs}"
            res[key] = {"ms_per_call": ms, "ms_per_vector": ms / nrhs,
                        "unknowns_matvecs_per_s": info["n_rwg"] * nrhs / (ms * 1e-3)}
            print(f"[bench] {name} on {w.name}: {nrhs} vector(s) {ms:.3f} ms per call",
                  file=sys.stderr, flush=True)
    x32 = torch.from_numpy(I.complex_gaussian(info["n_rwg"], w.seed_base + 7)).to(
        torch.complex64).cuda()
    ops32 = (("efie", lambda x, out: p.matvec_efie(x, out=out, prec="c64")),
             ("mfie", lambda x, out: p.matvec_mfie(x, gram_coef=-0.5, out=out, prec="c64")),
             ("cfie", lambda x, out: p.matvec_cfie(x, gram_coef=-0.5, out=out, prec="c64")))
    for name, fn in ops32:
        ms = timed(fn, x32, torch.empty_like(x32))
        res[f"{name}_c64_nrhs1"] = {"ms_per_call": ms,
                                    "unknowns_matvecs_per_s": info["n_rwg"] / (ms * 1e-3)}
        print(f"[bench] {name} c64 on {w.name}: {ms:.3f} ms per call", file=sys.stderr,
              flush=True)
    xs = torch.from_numpy(I.complex_gaussian(p.n, w.seed_base)).cuda()
    res["scalar_ms_per_matvec"] = timed(p.matvec, xs, torch.empty_like(xs))
    # a scattering solve as the paper runs it (Sec. V: the CFIE, GMRES): a
    # plane wave along +z polarised along x, to 1e-6, unpreconditioned; the
    # EFIE beside it
    k = float(w.k[0])
    bE = p.rwg_excitation([0, 0, 1], [1, 0, 0], field="E")
    bH = p.rwg_excitation([0, 0, 1], [1, 0, 0], field="H")
    solves = {}
    for op, rhs in (("cfie", (bE + bH) / (1j * k)), ("efie", bE / (1j * k))):
        t0 = time.perf_counter()
        xs_, r = p.solve_rwg(op, rhs, gram_coef=-0.5, rtol=1e-6, restart=100, max_iter=3000,
                             raise_on_fail=False)
        torch.cuda.synchronize()
        solves[op] = {"seconds": time.perf_counter() - t0, "iters": int(r.iters[0]),
                      "rel_resid": float(r.rel_resid[0]), "converged": bool(r.converged[0])}
        if op == "cfie":
            xc = xs_
        else:
            solves["current_difference_cfie_vs_efie"] = float(
                torch.linalg.vector_norm(xs_ - xc) / torch.linalg.vector_norm(xs_))
        print(f"[bench] {op} solve on {w.name}: {solves[op]}", file=sys.stderr, flush=True)
    res["plane_wave_solves"] = solves
    res["note"] = ("complex128 unless keyed c64; EFIE: three current channels and one charge "
                   "channel projected from the quadrature points and convolved with the plan's "
                   "spectrum (4 grids per vector); double layer (K - G/2): the three current "
                   "channels' grids, their spectral cross product with grad G in one z pass "
                   "(3 grids forward, 3 back); combined field: one projection, 4 grids forward, "
                   "7 back; the scalar product on the same plan convolves one grid")
    p.close()
    return res


def conventional_leg(plan, w, nrhs: int = 8, reps: int = 10) -> dict:
    """Conventional AIM against AIMx on one plan (Sec. II-B against Sec. III;
    the per-wavenumber cost of the sweep comparison of Sec. VI): the
    conventional method rebuilds its complex near correction for every
    wavenumber (here on the device, median of the fills timed with events),
    AIMx only its kernel spectrum; both then apply the same far operator."""
    import numpy as np
    import torch
    from paper_2009_02281_amd import inputs as I
    info = plan.info()
    nf = int(len(w.k))
    fills = []
    for f in range(min(nf, 5)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        plan.conventional_fill(f)
        b.record()
        torch.cuda.synchronize()
        fills.append(a.elapsed_time(b))
    fill_ms = sorted(fills)[len(fills) // 2]
    nr = min(nrhs, int(info["max_rhs"]))
    x = torch.from_numpy(I.complex_gaussian(w.n, w.seed_base + 7, nrhs=nr)).cuda()
    y = torch.empty_like(x)
    f_last = min(nf, 5) - 1
    ms_aimx = time_matvecs(plan, x, y, "c128", reps, 2, np.full(nr, f_last))
    for _ in range(2):
        plan.matvec_conventional(x, out=y)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        plan.matvec_conventional(x, out=y)
    b.record()
    torch.cuda.synchronize()
    ms_conv = a.elapsed_time(b) / reps
    spec_ms = 1e3 * info["spectra_seconds"] / nf
    res = {"workload": w.name, "triangles": w.n, "near_pairs": int(info["nnz"]), "n_freq": nf,
           "static_fill_seconds_once": info["near_seconds"],
           "per_freq_ms": {"aimx_spectrum": spec_ms, "conventional_spectrum_plus_near_fill":
                           spec_ms + fill_ms, "conventional_near_fill": fill_ms},
           "matvec_ms": {"vectors": nr, "aimx": ms_aimx, "conventional": ms_conv},
           "note": "complex128; the conventional near fill is per wavenumber, the AIMx static "
                   "fill once per geometry"}
    print(f"[bench] conventional AIM on {w.name}: near fill {fill_ms:.2f} ms per wavenumber "
          f"(AIMx: spectrum {spec_ms:.2f} ms), matvec x{nr} {ms_conv:.3f} ms vs AIMx "
          f"{ms_aimx:.3f} ms", file=sys.stderr, flush=True)
    return res


def host_near_seconds(w) -> dict:
    """The same static near fill on the host (a host-only plan of the
    workload), for comparison with the device fill."""
    from paper_2009_02281_amd import binding
    t0 = time.perf_counter()
    hp = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                      host_only=True)
    total = time.perf_counter() - t0
    hi = hp.info()
    hp.close()
    return {"host_setup_seconds": total, "host_near_fill_seconds": hi["near_seconds"],
            "host_threads": host_threads()}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="sphere-large",
                    choices=["boxarray", "sphere", "sphere-large", "sweep"])
    ap.add_argument("--prec", default="c128", choices=["c128", "c64"])
    ap.add_argument("--nrhs", type=int, default=0,
                    help="right-hand sides per matvec (default 1; the sweep: all 512)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-profile", action="store_true", help="skip per-kernel event timing")
    ap.add_argument("--no-solve", action="store_true", help="skip the GMRES time-to-tolerance leg")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-preconditioner time-to-tolerance leg")
    ap.add_argument("--no-unet", action="store_true", help="skip the U-Net throughput leg")
    ap.add_argument("--no-efie", action="store_true",
                    help="skip the RWG operators' leg (81,920-triangle sphere)")
    ap.add_argument("--schedule", default="",
                    help="comma-separated schedule (seven integers) to install instead of "
                         "autotuning the timed precision")
    ap.add_argument("--efie-only", action="store_true",
                    help="only run the RWG EFIE leg (--steps products per timing)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other precision and the extra workloads (sweep, box array)")
    ap.add_argument("--solve-rtol", type=float, default=1e-6)
    ap.add_argument("--solve-max-iter", type=int, default=4000,
                    help="GMRES iteration cap per solve (per refinement step in complex64)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched solve over 32 uneven geometries (against solving "
                         "them one after another)")
    ap.add_argument("--no-batch-learned", action="store_true",
                    help="skip training the learned preconditioner on pairs from uneven "
                         "training geometries and solving the 32-instance batch with it")
    ap.add_argument("--batch-restart", type=int, default=200,
                    help="GMRES restart length of the batch leg")
    ap.add_argument("--solve-pcs", default="none,diag,nearblock",
                    help="comma-separated preconditioners for the GMRES leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this benchmark measures one GPU only; the multi-GPU design is "
              "described, not run (use --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2009_02281_amd import binding
    from paper_2009_02281_amd import inputs as I

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    if args.copy_calibration:
        print(json.dumps(copy_bandwidth()), flush=True)
        return 0
    if args.efie_only:
        print(json.dumps({"efie": efie_leg(reps=args.steps)}), flush=True)
        return 0
    w = make_workload(args.workload)
    freq = None
    if args.workload == "sweep":
        nf = len(w.k)
        args.nrhs = args.nrhs or 8 * nf
        freq = np.arange(args.nrhs) % nf          # each vector at its own wavenumber
        args.no_solve = True
        args.no_cpu = True
    args.nrhs = args.nrhs or 1
    other = "c64" if args.prec == "c128" else "c128"
    print(f"[bench] workload {w.name}: N={w.n} dims={w.dims} order={w.order} "
          f"prec={args.prec} nrhs={args.nrhs}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    precs = (args.prec,) if (args.no_solve and args.no_extra) else ("c128", "c64")
    plan = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                        precisions=precs, max_rhs=args.nrhs)
    setup_s = time.perf_counter() - t0
    info = plan.info()
    print(f"[bench] setup {setup_s:.2f}s (tables {info['setup_seconds']:.2f}s, static near "
          f"fill {'device' if info['near_on_device'] else 'host'} {info['near_seconds']:.3f}s, "
          f"spectra {info['spectra_seconds']:.3f}s), nnz={info['nnz']}", file=sys.stderr,
          flush=True)
    tuned = {}
    for pr in precs:
        if args.schedule and pr == args.prec:
            # a given schedule (e.g. the one a profiled run picked) instead of
            # tuning, so that counter runs time the same launches
            sched = [int(v) for v in args.schedule.split(",")]
            plan.set_schedule(sched, prec=pr)
            tuned[pr] = {"schedule": sched, "pass_ms": [], "given": True}
            print(f"[bench] given schedule ({pr}): {sched}", file=sys.stderr, flush=True)
            continue
        tuned[pr] = plan.autotune(prec=pr, nrhs=args.nrhs, reps=10)
        print(f"[bench] autotuned FFT launch shapes ({pr}): {tuned[pr]['schedule']} "
              f"pass ms {[round(t, 4) for t in tuned[pr]['pass_ms']]}", file=sys.stderr,
              flush=True)
    dtype = torch.complex128 if args.prec == "c128" else torch.complex64
    xh = I.complex_gaussian(w.n, w.seed_base + 1, nrhs=args.nrhs)
    x = torch.from_numpy(xh).to(dtype).cuda()
    y = torch.empty_like(x)

    ms = time_matvecs(plan, x, y, args.prec, args.steps, args.warmup, freq)
    value = w.n * args.nrhs / (ms * 1e-3)
    print(f"[bench] {ms:.4f} ms/matvec -> {value:.4e} unknowns*matvecs/s", file=sys.stderr,
          flush=True)
    # spread of single matvecs (events around each one; outside the timed region)
    nsamp = max(20, min(100, args.steps))
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(nsamp)]
    for a, b in evs:
        a.record()
        plan.matvec(x, prec=args.prec, out=y, freq_idx=freq)
        b.record()
    torch.cuda.synchronize()
    one = sorted(a.elapsed_time(b) for a, b in evs)
    q = lambda f: one[min(nsamp - 1, int(round(f * (nsamp - 1))))]
    spread = {"samples": nsamp, "median_ms": q(0.5), "p25_ms": q(0.25), "p75_ms": q(0.75),
              "note": "one matvec between two events each, after the timed region"}

    out = {
        "metric": "AIM matvec unknowns/s",
        "value": value,
        "unit": "unknowns*matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": w.name, "triangles": w.n, "order": w.order,
                   "grid": list(w.dims), "padded_grid": [2 * d for d in w.dims],
                   "near_threshold_h": w.near_factor, "k": float(w.k[0]),
                   "nrhs": args.nrhs, "nnz": info["nnz"],
                   "n_freq": int(len(w.k))},
        "fft_schedule": {pr: tuned[pr]["schedule"] for pr in tuned},
        "ms_per_matvec_spread": spread,
        "setup": {"seconds": setup_s, "static_near_fill_seconds": info["near_seconds"],
                  "static_near_fill_on_device": info["near_on_device"],
                  "spectra_seconds": info["spectra_seconds"]},
    }
    if not args.no_extra:
        out["setup"].update(host_near_seconds(w))
        print(f"[bench] host near fill {out['setup']['host_near_fill_seconds']:.3f}s "
              f"({out['setup']['host_threads']} threads) vs device "
              f"{info['near_seconds']:.3f}s", file=sys.stderr, flush=True)

    if args.workload == "sweep":
        # the paper's cost model T = T_s + N_f T_d: T_s the frequency-independent
        # set-up (host tables and uploads), T_d per wavenumber its kernel
        # spectrum plus its share of the batched matvec (its vectors' share)
        nf = len(w.k)
        t_spec = info["spectra_seconds"] / nf
        t_mv = ms * 1e-3 / nf
        t_s = setup_s - info["spectra_seconds"]
        out["cost_model"] = {"n_freq": nf, "T_s_seconds": t_s,
                             "T_d_seconds": t_spec + t_mv,
                             "T_d_spectrum_seconds": t_spec,
                             "T_d_matvec_seconds": t_mv,
                             "vectors_per_freq": args.nrhs // nf,
                             "T_total_seconds": t_s + nf * (t_spec + t_mv)}

    if not args.no_profile:
        reps = max(5, min(50, args.steps))
        kms = plan.profile_matvec(x, reps=reps, prec=args.prec, out=y, freq_idx=freq)
        ab = algorithmic_bytes(info, args.prec, args.nrhs)
        merge_fused(kms, ab, out["fft_schedule"].get(args.prec), info, args.prec, args.nrhs)
        dom = max(kms, key=kms.get)
        achieved = ab[dom] / (kms[dom] * 1e-3) / 1e9
        stages = {k: {"ms": kms[k], "alg_bytes": ab[k],
                      "gbs": ab[k] / (kms[k] * 1e-3) / 1e9 if kms[k] > 0 else None,
                      "frac": ab[k] / (kms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS if kms[k] > 0
                      else None}
                  for k in kms}
        total_b = sum(ab.values())
        out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": achieved,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS,
                           "traffic": load_traffic(dom, w.name, args.prec,
                                                   out["fft_schedule"].get(args.prec)),
                           "copy_measured_gbs": copy_bandwidth()["gbs"]}
        out["stages"] = stages
        out["matvec_alg_gbs"] = total_b / (ms * 1e-3) / 1e9
        print(f"[bench] kernels (ms): " + ", ".join(f"{k}={v:.4f}" for k, v in kms.items()),
              file=sys.stderr, flush=True)

    if not args.no_extra and args.workload != "sweep":
        xo = torch.from_numpy(xh).to(torch.complex64 if other == "c64" else torch.complex128).cuda()
        yo = torch.empty_like(xo)
        mso = time_matvecs(plan, xo, yo, other, args.steps, args.warmup, freq)
        extra = {other: {"workload": w.name, "ms_per_step": mso,
                         "unknowns_matvecs_per_s": w.n * args.nrhs / (mso * 1e-3)}}
        if not args.no_profile:
            ko = plan.profile_matvec(xo, reps=max(5, min(50, args.steps)), prec=other, out=yo,
                                     freq_idx=freq)
            abo = algorithmic_bytes(info, other, args.nrhs)
            merge_fused(ko, abo, out["fft_schedule"].get(other), info, other, args.nrhs)
            extra[other]["stages"] = {k: {"ms": ko[k], "gbs": abo[k] / (ko[k] * 1e-3) / 1e9,
                                          "frac": abo[k] / (ko[k] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                                      for k in ko}
        print(f"[bench] {w.name} {other}: {mso:.4f} ms/matvec -> "
              f"{extra[other]['unknowns_matvecs_per_s']:.4e}", file=sys.stderr, flush=True)
        del xo, yo
        out["extra"] = extra

    if not args.no_solve:
        out["gmres"] = solve_leg(plan, args.solve_rtol, args.solve_max_iter,
                                 tuple(args.solve_pcs.split(",")))
    if not args.no_extra and args.workload != "sweep" and args.nrhs <= plan.info()["max_rhs"]:
        out["conventional"] = {w.name: conventional_leg(plan, w, nrhs=args.nrhs)}
        if args.nrhs == 1:
            out["dlp"] = dlp_leg(plan, w)
    if not args.no_extra and args.workload != "sweep":
        plan.close()
        plan = None
        torch.cuda.empty_cache()
        out["extra"]["sweep"] = extra_workload("sweep", ("c128", "c64"), 20, 3)
        ws = make_workload("sweep")
        sp = binding.Plan(ws.vertices, ws.triangles, ws.order, ws.dims, ws.h, ws.near_threshold,
                          ws.k, precisions=("c128",), max_rhs=8)
        out["conventional"][ws.name] = conventional_leg(sp, ws, nrhs=8)
        sp.close()
        if args.workload != "boxarray":
            out["extra"]["boxarray"] = extra_workload("boxarray", ("c128", "c64"), 50, 5)
        if not args.no_efie:
            out["efie"] = efie_leg()
            torch.cuda.empty_cache()
    if not args.no_learned and args.workload != "sweep":
        out["learned_pc"] = learned_pc_leg(args.solve_rtol)
    if not args.no_unet and args.workload != "sweep":
        out["unet"] = unet_leg()
    # the uneven batch (classical preconditioners, then the learned one);
    # a failure there is recorded and does not cost the main line
    for key, on, leg in (("batch", not args.no_batch, batch_leg),
                         ("batch_learned", not args.no_batch_learned, batch_learned_leg)):
        if not on:
            continue
        try:
            out[key] = leg(args.solve_rtol, restart=args.batch_restart)
        except Exception as err:  # noqa: BLE001 - reported in the JSON line
            out[key] = {"error": f"{type(err).__name__}: {err}"}
            print(f"[bench] {key} leg failed: {err}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()

    if not args.no_cpu:
        print("[bench] timing the oracle on the host ...", file=sys.stderr, flush=True)
        cb = cpu_baseline(w, xh[0] if xh.ndim == 2 else xh)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample",
                                                  "single_thread")}
        print(f"[bench] oracle {cb['seconds_per_matvec']:.3f} s/matvec "
              f"({cb['cores']} threads), {cb['single_thread']['seconds_per_matvec']:.3f} s "
              f"single-threaded", file=sys.stderr, flush=True)
        if not args.no_solve:
            out["cpu_gmres"] = cpu_gmres_leg(args.solve_rtol)
            print(f"[bench] GMRES on the small sphere: oracle {out['cpu_gmres']['cpu']}, "
                  f"GPU {out['cpu_gmres']['gpu']}", file=sys.stderr, flush=True)
    if plan is not None:
        plan.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

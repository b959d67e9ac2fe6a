#!/usr/bin/env python3
"""Benchmark: Jacobi-PCG solves/s on the 3D 7-point variable-coefficient
diffusion system (128^3 cells, 2,097,152 rows, 14,581,760 nonzeros; k = exp of
a 3^3 box-smoothed N(0,1) field, harmonic faces, b ~ U[-1,1], seed 2),
rtol 1e-8, x0 = 0, FP64, on one MI355X.

A step is one complete solve (setup kernels and every iteration until the
device-side convergence test fires) with A, b and x resident in HBM.  Timing
follows the paper's protocol (Section 4.1): warm-up solves, then K timed
solves bracketed by device synchronisation; solves/s = K / elapsed.

Also reported on the same JSON line (under "extra"), at the workloads' full
sizes: the 256-system batch (one batched launch against a per-solve loop),
the learned polynomial preconditioner (2000 training systems, FCG(1) with
the network's polynomial against Jacobi-PCG on 200 held-out systems), the
1024-system mixed 2D/3D batch solved in one call with the learned
preconditioner and a per-system fallback (against the per-solve loop and
batched Jacobi-PCG), the three batched/learned-vs-plain ratios gathered
under "batched_learned_vs_plain", and:
  roofline      -- the fused product kernel (SpMV + direction update + p.Ap):
                   algorithmic bytes per launch / mean launch duration, the
                   duration taken with HIP events on the solve's stream
                   around 400 back-to-back launches at the configuration the
                   timed solves used, right after the timed region (a
                   kernel-timed solve's per-launch event pairs, which add
                   each launch's dispatch, are reported beside it);
  cpu_baseline  -- the CPU oracle's Jacobi-PCG loop with its row loops on
                   every host thread (at most 16), the minimum of a few full
                   solves of the same system (the serial oracle's rate is
                   reported beside it);
  variants      -- the same solve with the loop launched kernel by kernel
                   (stream) and with a host check after every kernel
                   (the synchronous shape the paper compares against).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PCG solves/s at rtol 1e-8 (batched+learned vs plain); SpMV+vec HBM GB/s"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_pcg_product_diffusion3d_128.json")
# the product and update kernels' code: their file and the device helpers they inline
KERNEL_SOURCE = [os.path.join(ROOT, "paper_2306_17801_amd", "csrc", f) for f in ("pcg.hip", "internal.h")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(paths):
    """Hash of the kernel sources' code (one path or a list, in order):
    comments and whitespace removed, so that a comment edit does not
    invalidate counters taken on the same code."""
    import re

    texts = []
    for path in [paths] if isinstance(paths, str) else paths:
        with open(path, encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        texts.append(" ".join(text.split()))
    return hashlib.sha256("\n".join(texts).encode()).hexdigest()[:16]


def sdia_shape(A):
    """Value slots U per 64-row slice of the sliced-diagonal layout (the most
    distinct column offsets of any slice) and offset/mask slots (U rounded up
    to 8, 16 or 32)."""
    import numpy as np

    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.rowptr))
    key = (rows // 64) * (2 * A.n + 1) + (A.col.astype(np.int64) - rows + A.n)
    uk = np.unique(key)
    sl = uk // (2 * A.n + 1)
    u = int(np.bincount(sl).max()) if sl.size else 1
    return u, 8 if u <= 8 else 16 if u <= 16 else 32


def sdia_upper_slots(A):
    """Value slots on or right of the diagonal, summed over the slices: what
    the marching product streams when the matrix is symmetric (the entries
    left of the diagonal are read as their transposes)."""
    import numpy as np

    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.rowptr))
    off = A.col.astype(np.int64) - rows
    key = (rows // 64) * (2 * A.n + 1) + (off + A.n)
    return int(np.unique(key[off >= 0]).size)


def dia_offsets(A):
    """The distinct column offsets (column - row) of A, ascending."""
    import numpy as np

    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.rowptr))
    return sorted(int(o) for o in np.unique(A.col.astype(np.int64) - rows))


def is_symmetric(A):
    """Pattern and values symmetric bit for bit."""
    import numpy as np

    M = A.to_scipy()
    T = M.T.tocsr()
    T.sort_indices()
    M = M.tocsr()
    M.sort_indices()
    return (np.array_equal(M.indptr, T.indptr) and np.array_equal(M.indices, T.indices)
            and np.array_equal(M.data.view(np.int64), T.data.view(np.int64)))


def copy_calibration(apcg, torch):
    """Five copies of 2^27 doubles (1 GiB read + 1 GiB written each) with the
    library's copy kernel: the reference reading for the HBM byte counters."""
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ctx = apcg.apcg_ctx_create(0)
    vs, vd = apcg.apcg_vec_wrap(src), apcg.apcg_vec_wrap(dst)
    t = apcg.apcg_timer_create()
    apcg.apcg_vec_copy_async(vd, vs, ctx)
    apcg.apcg_timer_start(t, ctx)
    for _ in range(5):
        apcg.apcg_vec_copy_async(vd, vs, ctx)
    apcg.apcg_timer_stop(t, ctx)
    ms = apcg.apcg_timer_elapsed_ms(t) / 5
    print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "ms_per_copy": round(ms, 4),
                      "gbs": round(16 * n / (ms * 1e-3) / 1e9, 1)}), flush=True)
    apcg.apcg_ctx_synchronize(ctx)


def bench_latency(apcg, torch, reps=50):
    """The latency-bound regime (Section 4.2): the 64 x 64 Poisson system
    (4,096 rows, 20,224 nonzeros, x* ~ U[-1,1], b = A x*, seed 0), Jacobi-PCG
    at rtol 1e-10 from x0 = 0, one solve at a time, end to end (host call to
    host-visible completion), min and median of `reps` solves per mode after
    a warm-up; beside it the device's latency floors and the serial CPU
    oracle on the same system."""
    import numpy as np

    import oracle
    from paper_2306_17801_amd import problems
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    s = problems.poisson2d_manufactured(64, seed=0)
    ctx = apcg.apcg_ctx_create(0)
    A, b, x = DeviceCSR(s.A), DeviceVec(s.b), DeviceVec.zeros(s.A.n)
    info = apcg.apcg_info_create(0, 1)
    floors = apcg.apcg_latency_floors(0, 2000)
    out = {"workload": "poisson2d_64x64_jacobi_pcg_rtol1e-10", "n": s.A.n, "nnz": s.A.nnz, "reps": reps,
           "floors_us": {k: round(v, 3) for k, v in floors.items()}, "modes": {}}
    for name, mode in (("persistent", apcg.APCG_MODE_PERSISTENT), ("graph", apcg.APCG_MODE_GRAPH),
                       ("stream", apcg.APCG_MODE_STREAM), ("host_check", apcg.APCG_MODE_HOST_CHECK)):
        o = apcg.apcg_solve_opts_default(x0_is_zero=1, mode=mode)
        times = []
        for i in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            apcg.apcg_ksp_solve(ctx, A.h, b.h, x.h, 1e-10, 10000, o, info, 0)
            apcg.apcg_ctx_synchronize(ctx)
            if i:
                times.append(time.perf_counter() - t0)
        r = apcg.apcg_info_get(info, 0)
        xe = x.numpy()
        tmin, tmed = min(times), sorted(times)[len(times) // 2]
        out["modes"][name] = {"iterations": r["iterations"], "status": r["status"], "min_ms": round(1e3 * tmin, 4),
                              "median_ms": round(1e3 * tmed, 4), "solves_per_s": round(1 / tmin, 1),
                              "us_per_iteration": round(1e6 * tmin / max(r["iterations"], 1), 3),
                              "err_vs_manufactured": float(np.linalg.norm(xe - s.x_exact) / np.linalg.norm(s.x_exact))}
    t_cpu = []
    for _ in range(5):
        t0 = time.perf_counter()
        rc = oracle.pcg(s.A, s.b, rtol=1e-10, maxit=10000)
        t_cpu.append(time.perf_counter() - t0)
    out["cpu_oracle_serial"] = {"iterations": rc.its, "min_ms": round(1e3 * min(t_cpu), 4),
                                "solves_per_s": round(1 / min(t_cpu), 1)}
    m = out["modes"]
    out["persistent_speedup_vs_graph"] = round(m["graph"]["min_ms"] / m["persistent"]["min_ms"], 2)
    out["persistent_us_per_iteration_over_workgroup_floor"] = round(
        m["persistent"]["us_per_iteration"] / floors["workgroup_iteration_us"], 2)
    out["graph_us_per_iteration_over_two_graph_nodes"] = round(
        m["graph"]["us_per_iteration"] / (2 * floors["graph_node_us"]), 2)
    log(f"[bench] latency: {out}")
    apcg.apcg_info_destroy(info)
    apcg.apcg_ctx_synchronize(ctx)
    apcg.apcg_ctx_destroy(ctx)
    return out


def bench_batch(apcg, torch, reps, only=None, tile_rows=0):
    """256 independent 2D 5-point systems (side ~ U{32..256}, k = exp(N(0,1)),
    b ~ U[-1,1], seed 3), Jacobi-PCG rtol 1e-8: one batched persistent launch
    (graph) against the plain path, one apcg_ksp_solve per system spread over
    8 forked contexts."""
    from paper_2306_17801_amd import problems
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    systems = problems.batch2d_lognormal(256, seed=3)
    As = [DeviceCSR(s.A) for s in systems]
    bs = [DeviceVec(s.b) for s in systems]
    xs = [DeviceVec.zeros(s.A.n) for s in systems]
    nsys = len(systems)
    info = apcg.apcg_info_create(0, nsys)
    ctx = apcg.apcg_ctx_create(0)
    out = {"systems": nsys, "rows": int(sum(s.A.n for s in systems)), "nnz": int(sum(s.A.nnz for s in systems))}
    best = None
    for name, sched, tb in (("persistent256", 1, 256), ("persistent512", 1, 512), ("persistent1024", 1, 1024),
                            ("segmented", 2, 0), ("segmented_sdia", 2, 0)):
        if only is not None and name != only:
            continue
        if name == "segmented_sdia":
            # the matrices on the sliced-diagonal schedule (a one-time host
            # analysis each): the segmented tile product reads those copies,
            # and so does the plain per-solve loop below
            for a in As:
                try:
                    apcg.apcg_mat_set_spmv_config(a.h, 1, 256, 0, apcg.APCG_SPMV_SDIA)
                except apcg.ApcgError:
                    pass
        o = apcg.apcg_solve_opts_default(x0_is_zero=1, batch_block_size=tb, batch_schedule=sched,
                                         batch_tile_rows=tile_rows)
        apcg.apcg_ksp_solve_batched(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in xs], 1e-8, 50000, o, info)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            apcg.apcg_ksp_solve_batched(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in xs], 1e-8, 50000, o,
                                        info)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[f"batched_{name}_ms"] = round(1000 * dt, 3)
        if best is None or dt < best[0]:
            best = (dt, name)
    if only is None:
        # the batched autotuner's pick (timed on the device over 32
        # iterations of every configuration), which the comparison uses
        t0 = time.perf_counter()
        cfg, ms, _ = apcg.apcg_batch_autotune(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in xs], 0, 32)
        out["autotune"] = {"config": cfg, "ms_for_32_iterations": round(ms, 3),
                           "seconds": round(time.perf_counter() - t0, 2)}
        o = apcg.apcg_solve_opts_default(x0_is_zero=1, batch_schedule=cfg["schedule"],
                                         batch_block_size=cfg["block_size"], batch_tile_rows=cfg["tile_rows"])
        apcg.apcg_ksp_solve_batched(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in xs], 1e-8, 50000, o, info)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            apcg.apcg_ksp_solve_batched(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in xs], 1e-8, 50000, o,
                                        info)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out["batched_autotuned_ms"] = round(1000 * dt, 3)
        best = (dt, "autotuned")
    res = [apcg.apcg_info_get(info, i) for i in range(nsys)]
    out["batched_schedule"] = best[1]
    out["batched_ms"] = round(1000 * best[0], 3)
    out["batched_solves_per_s"] = round(nsys / best[0], 2)
    out["converged"] = sum(1 for r in res if r["status"] == apcg.APCG_SOLVE_CONVERGED)
    out["iterations_min_max"] = [min(r["iterations"] for r in res), max(r["iterations"] for r in res)]
    out["roofline"] = batch_roofline(apcg, systems, As, res, best[0], o)
    log(f"[bench] batch: {out} ")
    if only is not None:  # one schedule alone (profiling runs): no per-solve loop
        apcg.apcg_info_destroy(info)
        apcg.apcg_ctx_synchronize(ctx)
        apcg.apcg_ctx_destroy(ctx)
        return out

    # plain path: one graph-mode solve per system, 8 contexts round robin, on
    # the sliced-diagonal copies (a batched pick of CSR reads moved the
    # members to the row schedule)
    for a in As:
        try:
            apcg.apcg_mat_set_spmv_config(a.h, 1, 256, 0, apcg.APCG_SPMV_SDIA)
        except apcg.ApcgError:
            pass
    kids = apcg.apcg_ctx_fork(ctx, 8)
    plain = apcg.apcg_solve_opts_default(x0_is_zero=1)
    infos = apcg.apcg_info_create(0, nsys)
    for i in range(nsys):  # warm-up (graph capture per system)
        apcg.apcg_ksp_solve(kids[i % 8], As[i].h, bs[i].h, xs[i].h, 1e-8, 50000, plain, infos, i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(nsys):
        apcg.apcg_ksp_solve(kids[i % 8], As[i].h, bs[i].h, xs[i].h, 1e-8, 50000, plain, infos, i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["per_solve_loop_ms"] = round(1000 * dt, 3)
    out["per_solve_loop_solves_per_s"] = round(nsys / dt, 2)
    out["batched_speedup_vs_per_solve_loop"] = round(dt / best[0], 3)
    log(f"[bench] per-solve loop: {1000 * dt:.1f} ms")
    apcg.apcg_ctx_join(ctx, kids, apcg.APCG_JOIN_DESTROY)
    apcg.apcg_info_destroy(infos)
    apcg.apcg_info_destroy(info)
    apcg.apcg_ctx_synchronize(ctx)
    apcg.apcg_ctx_destroy(ctx)
    return out


def batch_roofline(apcg, systems, As, res, seconds, opts):
    """Algorithmic HBM bytes of a segmented batched solve over its wall time:
    for every system, its iterations times the bytes of one tile product
    (sliced-diagonal copy: 512 U + 96 per 64-row slice for the values,
    offsets and masks, CSR: 12 nnz + 4 (n + 1); both + 32 n for z, p_old read
    and p, w written) and one tile update (64 n: x, r, p, w, D^-1 read; x, r,
    z written).  The per-system kernels' partial sums are not counted.  None
    for the persistent schedule (another kernel and byte count)."""
    if opts.batch_schedule != 2:
        return None
    total = 0
    row_its = 0
    for s, a, r in zip(systems, As, res):
        n, its = s.A.n, r["iterations"]
        nsl = (n + 63) // 64
        cfg = apcg.apcg_mat_get_spmv_config(a.h)
        info = apcg.apcg_mat_get_sdia_info(a.h) if cfg["schedule"] == apcg.APCG_SPMV_SDIA else None
        if info and info["state"] == 1 and info["offset_slots"] == 8:
            prod = nsl * (512 * info["value_slots"] + 96) + 32 * n
        else:
            prod = 12 * s.A.nnz + 4 * (n + 1) + 32 * n
        total += its * (prod + 64 * n)
        row_its += its * n
    achieved = total / seconds / 1e9
    return {"bound": "hbm", "row_iterations": row_its, "algorithmic_bytes": total, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "note": "whole batched solve: wall time includes the per-system kernels and the iterations where few "
                    "systems are still running"}


def learned_batch_roofline(apcg, As, res, seconds):
    """Algorithmic HBM bytes of the batched learned solve over its wall time.
    V = one pass over a matrix (sliced-diagonal copy: 512 U + 96 per 64-row
    slice; CSR: 12 nnz + 4 (n + 1)).  Per flexible iteration: 9 V (product
    and eight Clenshaw steps) + 392 n (product 32: z, p_old read, p, w
    written; update 48: x, p, w, r read, x, r written; Clenshaw 24 + 6 x 40 +
    48: D^-1, r and the recurrence's vectors read, each b_j or z written);
    per Jacobi-mode iteration V + 112 n; the feature run's 12 Jacobi-PCG
    steps alike, and its two row passes 2 x (12 nnz + 4 (n + 1)).  The
    per-system kernels and the network are not counted."""
    total = 0
    for a, r in zip(As, res):
        n = a.n
        nnz = a.nnz
        csr = 12 * nnz + 4 * (n + 1)
        cfg = apcg.apcg_mat_get_spmv_config(a.h)
        info = apcg.apcg_mat_get_sdia_info(a.h) if cfg["schedule"] == apcg.APCG_SPMV_SDIA else None
        V = (((n + 63) // 64) * (512 * info["value_slots"] + 96)
             if info and info["state"] == 1 and info["offset_slots"] == 8 else csr)
        flex = r["fcg_iterations"]
        jac = max(0, r["iterations"] - flex) + 12
        total += flex * (9 * V + 392 * n) + jac * (V + 112 * n) + 2 * csr
    achieved = total / seconds / 1e9
    return {"bound": "hbm", "algorithmic_bytes": total, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "note": "whole batched learned solve (features, network, FCG): wall time includes the per-system "
                    "kernels, the network and the iterations where few systems are still running"}


def device_system(fields, device=0):
    """Uploads host-drawn coefficients and right-hand side and assembles the
    matrix on the GPU (problems.diffusion_csr_torch; the same bits as the
    host assembly).  Returns (DeviceCSR, DeviceVec)."""
    import torch

    from paper_2306_17801_amd import problems
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    k = torch.from_numpy(fields.k).to(f"cuda:{device}")
    rp, col, val = problems.diffusion_csr_torch(k, fields.aniso)
    del k
    return DeviceCSR.from_tensors(rp, col, val, device), DeviceVec(fields.b, device)


def host_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def bench_learned(apcg, torch, n_train, n_eval, side_lo, side_hi, epochs, reps, workers):
    """Learned polynomial preconditioner: 3D 7-point systems, side ~
    U{side_lo..side_hi}, sigma ~ U[0.5, 2], anisotropy ~ log-U[1, 100]
    (training seed 4, held-out seed 40).  Features and labels on the GPU,
    training with the library's MLP kernels, then each held-out system solved
    at rtol 1e-8 by Jacobi-PCG (the plain path, on the product schedule the
    autotuner picks for that matrix), FCG(1) with the network's polynomial
    (features + network + solve, one call) and FCG(1) with a fixed Chebyshev
    polynomial on [lmax/100, lmax]."""
    import numpy as np
    from numpy.polynomial import chebyshev as Ch

    from paper_2306_17801_amd import learned as L
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    from paper_2306_17801_amd import problems

    ctx = apcg.apcg_ctx_create(0)
    # the training set is drawn (host threads), assembled on the GPU and
    # collected in chunks, so that the full workload (2000 systems of up to
    # 96^3 rows) never sits in memory at once
    t_gen = t_collect = 0.0
    parts = []
    chunk = 256
    for c0 in range(0, n_train, chunk):
        c1 = min(n_train, c0 + chunk)
        t0 = time.perf_counter()
        fl = problems.fields_threaded(problems.learned_pc_fields,
                                      [(4, i, n_train, side_lo, side_hi) for i in range(c0, c1)], workers)
        t_gen += time.perf_counter() - t0
        t0 = time.perf_counter()
        parts.append(L.collect(ctx, (device_system(f) for f in fl), count=len(fl)))
        t_collect += time.perf_counter() - t0
        del fl
        log(f"[bench] learned: training systems {c1}/{n_train} collected")
    dtrain = L.Dataset(*[torch.cat([getattr(d, k) for d in parts]) for k in ("X", "G", "h", "label", "lmax")])
    del parts
    t0 = time.perf_counter()
    eval_set = problems.fields_threaded(problems.learned_pc_fields,
                                        [(40, i, n_eval, side_lo, side_hi) for i in range(n_eval)], workers)
    t_gen += time.perf_counter() - t0
    deval = L.collect(ctx, (device_system(f) for f in eval_set), count=n_eval)
    t0 = time.perf_counter()
    pc, losses = L.train(ctx, dtrain, epochs=epochs, batch=32, lr=3e-3)
    t_train = time.perf_counter() - t0
    untrained, _ = L.train(ctx, dtrain, epochs=0)
    out = {"train_systems": n_train, "eval_systems": n_eval, "sides": [side_lo, side_hi], "epochs": epochs,
           "generate_s": round(t_gen, 1), "collect_s": round(t_collect, 2), "train_s": round(t_train, 3),
           "train_steps": int(losses.size),
           "heldout_loss_trained": L.mean_loss(ctx, pc, deval), "heldout_loss_untrained": L.mean_loss(ctx, untrained, deval)}
    log(f"[bench] learned: generated {t_gen:.1f}s, collected {t_collect:.1f}s, trained {t_train:.2f}s")

    T9 = [0] * 9 + [1]

    def control(lmax):
        a = lmax / 100
        s0 = (lmax + a) / (lmax - a)
        f = lambda y: (1 - Ch.chebval((lmax + a - 2 * (y + 1) * lmax / 2) / (lmax - a), T9) /
                       Ch.chebval(s0, T9)) / ((y + 1) * lmax / 2)
        return Ch.chebinterpolate(f, 8).astype(np.float32)

    info = apcg.apcg_info_create(0, 1)
    opts = apcg.apcg_solve_opts_default(x0_is_zero=1)
    tot = {"jacobi": 0.0, "learned": 0.0, "control": 0.0}
    its = {k: [] for k in tot}
    fallbacks = 0
    unconverged = 0
    feat_t = 0.0
    tune_hits = 0
    for s in eval_set:
        dA, db = device_system(s)
        dx = DeviceVec.zeros(dA.n)
        # the plain path on its fastest product schedule for this matrix, as
        # in the headline (the FCG solves read the sliced-diagonal copy
        # whenever the pattern has one, whatever the schedule); matrices of
        # the same pattern class and size bucket reuse the tuning table
        _, _, hit = apcg.apcg_mat_autotune_cached(dA.h, ctx, 3)
        tune_hits += int(hit)
        feat = torch.zeros(16, dtype=torch.float32, device="cuda:0")
        lm = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        apcg.apcg_pc_features(ctx, dA.h, db.h, feat, lm)
        apcg.apcg_ctx_synchronize(ctx)
        cc = torch.from_numpy(control(float(lm.cpu()[0]))).to("cuda:0")
        torch.cuda.synchronize()
        runs = {
            "jacobi": lambda: apcg.apcg_ksp_solve(ctx, dA.h, db.h, dx.h, 1e-8, 50000, opts, info, 0),
            "learned": lambda: L.solve(ctx, pc, dA.h, db.h, dx.h, 1e-8, 50000, opts, None, info, 0),
            "control": lambda: apcg.apcg_ksp_solve_fcg_poly(ctx, dA.h, db.h, dx.h, 1e-8, 50000, cc, lm, opts,
                                                             None, info, 0),
        }
        # the learned solve's first step alone: features of the system
        apcg.apcg_pc_features(ctx, dA.h, db.h, feat, lm)
        apcg.apcg_ctx_synchronize(ctx)
        t1 = time.perf_counter()
        for _ in range(reps):
            apcg.apcg_pc_features(ctx, dA.h, db.h, feat, lm)
        apcg.apcg_ctx_synchronize(ctx)
        feat_t += (time.perf_counter() - t1) / reps
        for k, run in runs.items():
            run()  # warm-up (graph capture)
            apcg.apcg_ctx_synchronize(ctx)
            t1 = time.perf_counter()
            for _ in range(reps):
                run()
            apcg.apcg_ctx_synchronize(ctx)
            tot[k] += (time.perf_counter() - t1) / reps
            r = apcg.apcg_info_get(info, 0)
            its[k].append(r["iterations"])
            if not r["status"] & apcg.APCG_SOLVE_CONVERGED:
                unconverged += 1
            if k == "learned" and r["status"] & apcg.APCG_SOLVE_FALLBACK:
                fallbacks += 1
        dA.close()
        db.close()
        dx.close()
    apcg.apcg_info_destroy(info)
    apcg.apcg_ctx_synchronize(ctx)
    apcg.apcg_ctx_destroy(ctx)
    for k in tot:
        out[f"{k}_mean_iterations"] = round(float(np.mean(its[k])), 2)
        out[f"{k}_ms_per_solve"] = round(1000 * tot[k] / n_eval, 4)
        out[f"{k}_solves_per_s"] = round(n_eval / tot[k], 3)
    out["features_ms_per_call"] = round(1000 * feat_t / n_eval, 4)
    out["autotune_table_hits"] = tune_hits
    out["learned_speedup_vs_jacobi"] = round(tot["jacobi"] / tot["learned"], 3)
    out["learned_speedup_vs_control"] = round(tot["control"] / tot["learned"], 3)
    out["learned_fallbacks"] = fallbacks
    out["unconverged"] = unconverged
    log(f"[bench] learned: {out}")
    return out


def bench_mixed(apcg, torch, count, n_train, train_nhi, epochs, reps, workers, batched_jacobi=True):
    """Mixed batch: the first `count` systems of the 1024-system batch (2D
    5-point and 3D 7-point, N ~ log-U[1e3, 1e6], sigma ~ U[0.5, 2],
    anisotropy ~ log-U[1, 1000], seed 5), rtol 1e-8.  A network trained on
    the GPU on `n_train` systems of the same distribution (seed 6, N capped
    at train_nhi) drives the learned batched solve (features, network and
    FCG(1) with a per-system fallback, all systems in one block-diagonal
    iteration); compared with the plain path (one apcg_ksp_solve per system
    over 8 forked contexts) and with the batched Jacobi-PCG.  Each path runs
    once untimed (the batched ones with maxit 0: uploads and workspace; the
    per-solve loop with 16 iterations: every system's graph), then `reps`
    timed runs; the mean is reported."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    from paper_2306_17801_amd import learned as L
    from paper_2306_17801_amd import problems
    from paper_2306_17801_amd.device import DeviceVec

    t0 = time.perf_counter()
    train_f = problems.fields_threaded(problems.mixed_fields, [(6, i, 1e3, train_nhi) for i in range(n_train)],
                                       workers)
    t_gen = time.perf_counter() - t0
    ctx = apcg.apcg_ctx_create(0)
    t0 = time.perf_counter()
    dtrain = L.collect(ctx, (device_system(f) for f in train_f), rtol=1e-8, maxit=50000, count=n_train)
    t_collect = time.perf_counter() - t0
    del train_f
    t0 = time.perf_counter()
    pc, _ = L.train(ctx, dtrain, epochs=epochs, batch=32, lr=3e-3)
    t_train = time.perf_counter() - t0
    t0 = time.perf_counter()
    eval_f = problems.fields_threaded(problems.mixed_fields, [(5, i, 1e3, 1e6) for i in range(count)], workers)
    t_gen += time.perf_counter() - t0
    t0 = time.perf_counter()
    dev = [device_system(f) for f in eval_f]
    t_asm = time.perf_counter() - t0
    rows = int(sum(f.b.size for f in eval_f))
    del eval_f
    As = [d[0] for d in dev]
    bs = [d[1] for d in dev]
    xs = [DeviceVec.zeros(a.n) for a in As]
    nsys = len(As)
    log(f"[bench] mixed: drew {t_gen:.1f}s, assembled on the GPU {t_asm:.1f}s, collected {t_collect:.1f}s, "
        f"trained {t_train:.2f}s")
    info = apcg.apcg_info_create(0, nsys)
    # every matrix on the sliced-diagonal schedule (a one-time host analysis
    # each, outside the timed runs, on host threads): the batched tile
    # products, the batched Clenshaw steps and the per-solve loop read those
    # copies
    t0 = time.perf_counter()

    def to_sdia(a):
        try:
            apcg.apcg_mat_set_spmv_config(a.h, 1, 256, 0, apcg.APCG_SPMV_SDIA)
            return 1
        except apcg.ApcgError:
            return 0

    with ThreadPoolExecutor(workers) as ex:
        n_sdia = sum(ex.map(to_sdia, As))
    t_sdia = time.perf_counter() - t0
    log(f"[bench] mixed: {n_sdia} of {nsys} matrices on sliced diagonals ({t_sdia:.1f}s)")
    out = {"systems": nsys, "rows": rows, "nnz": int(sum(a.nnz for a in As)),
           "train_systems": n_train, "train_n_max": train_nhi, "generate_s": round(t_gen, 1),
           "assemble_s": round(t_asm, 1), "collect_s": round(t_collect, 2), "train_s": round(t_train, 3),
           "sliced_diagonal_systems": n_sdia, "sdia_analysis_s": round(t_sdia, 1), "timed_runs": reps}
    hA, hb, hx = [a.h for a in As], [b.h for b in bs], [x.h for x in xs]
    opts = apcg.apcg_solve_opts_default(x0_is_zero=1)
    # the batched autotuner picks each batched path's launch shape (a few
    # iterations of each configuration, timed on the device)
    t0 = time.perf_counter()
    cfg_l, ms_l, _ = apcg.apcg_batch_autotune(ctx, hA, hb, hx, 1, 4)
    opts_l = apcg.apcg_solve_opts_default(x0_is_zero=1, batch_tile_rows=cfg_l["tile_rows"])
    tuned = {"learned": {"config": cfg_l, "ms_for_4_iterations": round(ms_l, 3)}}
    opts_j = opts
    if batched_jacobi:
        cfg_j, ms_j, _ = apcg.apcg_batch_autotune(ctx, hA, hb, hx, 0, 8)
        opts_j = apcg.apcg_solve_opts_default(x0_is_zero=1, batch_schedule=cfg_j["schedule"],
                                              batch_block_size=cfg_j["block_size"], batch_tile_rows=cfg_j["tile_rows"])
        tuned["jacobi"] = {"config": cfg_j, "ms_for_8_iterations": round(ms_j, 3)}
    tuned["seconds"] = round(time.perf_counter() - t0, 2)
    out["autotune"] = tuned
    log(f"[bench] mixed: batched autotune {tuned}")

    def timed(run, warm):
        warm()
        apcg.apcg_ctx_synchronize(ctx)
        t1 = time.perf_counter()
        for _ in range(reps):
            run()
        apcg.apcg_ctx_synchronize(ctx)
        return (time.perf_counter() - t1) / reps

    def summary(prefix, dt):
        res = [apcg.apcg_info_get(info, i) for i in range(nsys)]
        its = [r["iterations"] for r in res]
        out[f"{prefix}_ms"] = round(1000 * dt, 2)
        out[f"{prefix}_solves_per_s"] = round(nsys / dt, 2)
        out[f"{prefix}_converged"] = sum(1 for r in res if r["status"] & apcg.APCG_SOLVE_CONVERGED)
        out[f"{prefix}_iterations_mean"] = round(float(np.mean(its)), 1)
        return res

    def learned(maxit):
        apcg.apcg_ksp_solve_batched_learned(ctx, hA, hb, hx, 1e-8, maxit, pc.params, pc.mean, pc.std, opts_l,
                                            None, info)

    # the tuning table's entry puts the members back on the layout the
    # learned solve's pick reads (the Jacobi tuning may have changed it)
    apcg.apcg_batch_autotune(ctx, hA, hb, hx, 1, 4)
    dt = timed(lambda: learned(50000), lambda: learned(0))
    res = summary("batched_learned", dt)
    out["batched_learned_roofline"] = learned_batch_roofline(apcg, As, res, dt)
    out["batched_learned_fallbacks"] = sum(1 for r in res if r["status"] & apcg.APCG_SOLVE_FALLBACK)
    out["batched_learned_fallback_reasons"] = {
        k: sum(1 for r in res if r["status"] & apcg.APCG_SOLVE_FALLBACK and r["status"] & bit)
        for k, bit in (("p.Ap", apcg.APCG_SOLVE_BREAKDOWN_PAP), ("r.z_or_rejected", apcg.APCG_SOLVE_BREAKDOWN_RZ),
                       ("stall", apcg.APCG_SOLVE_STALL))}
    out["batched_learned_iterations_max"] = max(r["iterations"] for r in res)
    out["batched_learned_fcg_iterations_mean"] = round(float(np.mean([r["fcg_iterations"] for r in res])), 1)
    log(f"[bench] mixed batched learned: {1000 * dt:.1f} ms")
    if batched_jacobi:
        def bj(maxit):
            apcg.apcg_ksp_solve_batched(ctx, hA, hb, hx, 1e-8, maxit, opts_j, info)

        apcg.apcg_batch_autotune(ctx, hA, hb, hx, 0, 8)  # from the table: the layout of this pick
        dt = timed(lambda: bj(50000), lambda: bj(0))
        res = summary("batched_jacobi", dt)
        out["batched_jacobi_iterations_max"] = max(r["iterations"] for r in res)
        out["batched_learned_speedup_vs_batched_jacobi"] = round(out["batched_jacobi_ms"] / out["batched_learned_ms"], 3)
        log(f"[bench] mixed batched Jacobi: {1000 * dt:.1f} ms")
    # the plain path on the sliced-diagonal copies again (a batched pick of
    # CSR reads moves the members to the row schedule)
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(to_sdia, As))
    kids = apcg.apcg_ctx_fork(ctx, 8)
    infos = apcg.apcg_info_create(0, nsys)

    def loop(maxit):
        for i in range(nsys):
            apcg.apcg_ksp_solve(kids[i % 8], hA[i], hb[i], hx[i], 1e-8, maxit, opts, infos, i)
        for k in kids:
            apcg.apcg_ctx_synchronize(k)

    dt = timed(lambda: loop(50000), lambda: loop(16))
    res = [apcg.apcg_info_get(infos, i) for i in range(nsys)]
    out["per_solve_loop_ms"] = round(1000 * dt, 2)
    out["per_solve_loop_solves_per_s"] = round(nsys / dt, 2)
    out["per_solve_loop_iterations_mean"] = round(float(np.mean([r["iterations"] for r in res])), 1)
    out["per_solve_loop_iterations_max"] = max(r["iterations"] for r in res)
    out["per_solve_loop_converged"] = sum(1 for r in res if r["status"] & apcg.APCG_SOLVE_CONVERGED)
    out["batched_learned_speedup_vs_per_solve_loop"] = round(out["per_solve_loop_ms"] / out["batched_learned_ms"], 3)
    log(f"[bench] mixed per-solve loop: {1000 * dt:.1f} ms")
    apcg.apcg_ctx_join(ctx, kids, apcg.APCG_JOIN_DESTROY)
    apcg.apcg_info_destroy(infos)
    apcg.apcg_info_destroy(info)
    apcg.apcg_ctx_synchronize(ctx)
    apcg.apcg_ctx_destroy(ctx)
    for x in xs:
        x.close()
    for b in bs:
        b.close()
    for a in As:
        a.close()
    log(f"[bench] mixed: {out}")
    return out


def bench_sweep(apcg, torch, targets, reps, cpu_max_nnz, stencils):
    """The paper's CG benchmark shape (Section 4.1): constant-coefficient
    Laplace operators with 5-/9-point (2D) and 7-/27-point (3D) stencils,
    NNZ from 1e4 to 1e8, exactly 20 Jacobi-PCG iterations (rtol 0), minimum
    over the repetitions of the end-to-end time to host-visible completion.
    The same for TFQMR (Section 4's second method): graph mode, host-check
    mode and the CPU oracle.  CG variants: the fused solve in graph mode
    (asynchronous), in stream mode,
    and in host-check mode (the host waits after every kernel, the paper's
    synchronous baseline shape); CG composed from the asynchronous
    primitives with device scalars, and the same with every reduction read
    back to the host before the next call; the CPU oracle (serial) up to
    cpu_max_nnz.  Also a bandwidth check of the vector kernels outside the
    256 MB last-level cache (2^27-entry vectors)."""
    import numpy as np

    import oracle
    from paper_2306_17801_amd import problems
    from paper_2306_17801_amd.composed import ComposedCG
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    ctx = apcg.apcg_ctx_create(0)
    info = apcg.apcg_info_create(0, 1)
    out = []
    diag = {5: 4.0, 9: 8.0, 7: 6.0, 27: 26.0}

    def tmin(run, prep=None, r=reps):
        best = float("inf")
        for i in range(r + 1):  # the first is the warm-up
            if prep:
                prep()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if i > 0:
                best = min(best, dt)
        return best

    for points in stencils:
        dim = 2 if points in (5, 9) else 3
        for target in targets:
            side = max(2, int(round((target / points) ** (1.0 / dim))))
            t0 = time.time()
            A_h = problems.stencil_laplacian((side,) * dim, points)
            b_h = np.random.default_rng(10 + points).uniform(-1, 1, A_h.n)
            gen_s = time.time() - t0
            A, b, x = DeviceCSR(A_h), DeviceVec(b_h), DeviceVec.zeros(A_h.n)
            cfg, _ = apcg.apcg_mat_autotune(A.h, ctx, 3)
            row = {"stencil": points, "side": side, "n": A_h.n, "nnz": A_h.nnz, "spmv_config": cfg}
            xs = {}
            for name, mode in (("graph", apcg.APCG_MODE_GRAPH), ("stream", apcg.APCG_MODE_STREAM),
                               ("host_check", apcg.APCG_MODE_HOST_CHECK)):
                o = apcg.apcg_solve_opts_default(x0_is_zero=1, mode=mode)

                def run(o=o):
                    apcg.apcg_ksp_solve(ctx, A.h, b.h, x.h, 0.0, 20, o, info, 0)
                    res = apcg.apcg_info_get(info, 0)
                    assert res["iterations"] == 20, res

                row[name + "_ms"] = round(1e3 * tmin(run), 4)
                xs[name] = x.numpy()
            xt = {}
            for name, mode in (("tfqmr_graph", apcg.APCG_MODE_GRAPH), ("tfqmr_host_check", apcg.APCG_MODE_HOST_CHECK)):
                o = apcg.apcg_solve_opts_default(x0_is_zero=1, mode=mode)

                def run(o=o):
                    apcg.apcg_ksp_solve_tfqmr(ctx, A.h, b.h, x.h, 0.0, 20, o, info, 0)
                    res = apcg.apcg_info_get(info, 0)
                    assert res["iterations"] == 20, res

                row[name + "_ms"] = round(1e3 * tmin(run), 4)
                xt[name] = x.numpy()
            cg = ComposedCG(ctx, A_h.n)
            for name, sync in (("composed_async", False), ("composed_sync", True)):
                row[name + "_ms"] = round(1e3 * tmin(lambda: cg.solve(A.h, b.h, x.h, diag[points], 20, sync),
                                                     prep=lambda: x.t.zero_()), 4)
                xs[name] = x.numpy()
            cg.close()
            ref = xs["graph"]
            nr = np.linalg.norm(ref)
            row["max_rel_diff_variants"] = float(max(np.linalg.norm(v - ref) / nr for v in xs.values()))
            if A_h.nnz <= cpu_max_nnz:
                t_cpu = float("inf")
                for _ in range(2 if A_h.nnz > 1e6 else 3):
                    t1 = time.perf_counter()
                    r = oracle.pcg(A_h, b_h, rtol=0.0, maxit=20)
                    t_cpu = min(t_cpu, time.perf_counter() - t1)
                row["cpu_oracle_ms"] = round(1e3 * t_cpu, 4)
                row["rel_diff_vs_oracle"] = float(np.linalg.norm(ref - r.x) / np.linalg.norm(r.x))
                t_cpu = float("inf")
                for _ in range(2 if A_h.nnz > 1e6 else 3):
                    t1 = time.perf_counter()
                    rt = oracle.tfqmr(A_h, b_h, rtol=0.0, maxit=20)
                    t_cpu = min(t_cpu, time.perf_counter() - t1)
                row["tfqmr_cpu_oracle_ms"] = round(1e3 * t_cpu, 4)
                row["tfqmr_rel_diff_vs_oracle"] = float(max(np.linalg.norm(v - rt.x) / np.linalg.norm(rt.x)
                                                            for v in xt.values()))
            it_bytes = 12 * A_h.nnz + 4 * (A_h.n + 1) + 96 * A_h.n
            row["graph_us_per_iteration"] = round(1e3 * row["graph_ms"] / 20, 3)
            row["graph_gbs_csr_bytes"] = round(20 * it_bytes / (row["graph_ms"] * 1e-3) / 1e9, 1)
            row["async_speedup_vs_host_check"] = round(row["host_check_ms"] / row["graph_ms"], 3)
            row["composed_async_speedup_vs_sync"] = round(row["composed_sync_ms"] / row["composed_async_ms"], 3)
            row["tfqmr_async_speedup_vs_host_check"] = round(row["tfqmr_host_check_ms"] / row["tfqmr_graph_ms"], 3)
            log(f"[sweep] {points}-pt side {side} nnz {A_h.nnz:.3g} (gen {gen_s:.1f}s): " +
                ", ".join(f"{k[:-3]} {v:.3f}" for k, v in row.items() if k.endswith("_ms")) + " ms")
            out.append(row)
            del A, b, x
            torch.cuda.empty_cache()

    # vector kernels outside the last-level cache: 2^27 doubles (1 GiB) per vector
    nv = 1 << 27
    u = torch.ones(nv, dtype=torch.float64, device="cuda:0")
    v = torch.full((nv,), 0.5, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    hu, hv = apcg.apcg_vec_wrap(u), apcg.apcg_vec_wrap(v)
    a = apcg.apcg_scalar_create(ctx)
    apcg.apcg_scalar_set(a, 1e-3, ctx)
    t = apcg.apcg_timer_create()
    vec = {}
    for name, fn, nbytes in (("axpy", lambda: apcg.apcg_vec_axpy_async(hv, a, False, hu, ctx), 24 * nv),
                             ("dot", lambda: apcg.apcg_vec_dot_async(hu, hv, a, ctx), 16 * nv),
                             ("copy", lambda: apcg.apcg_vec_copy_async(hv, hu, ctx), 16 * nv)):
        fn()
        apcg.apcg_timer_start(t, ctx)
        for _ in range(10):
            fn()
        apcg.apcg_timer_stop(t, ctx)
        ms = apcg.apcg_timer_elapsed_ms(t) / 10
        vec[name] = {"n": nv, "bytes": nbytes, "ms": round(ms, 4), "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1)}
        log(f"[sweep] {name} 2^27: {ms:.3f} ms, {vec[name]['gbs']} GB/s")
    apcg.apcg_timer_destroy(t)
    apcg.apcg_scalar_destroy(a)
    apcg.apcg_vec_destroy(hu)
    apcg.apcg_vec_destroy(hv)
    apcg.apcg_info_destroy(info)
    apcg.apcg_ctx_synchronize(ctx)
    apcg.apcg_ctx_destroy(ctx)
    return {"cg_20_iterations": out, "vector_kernels_out_of_cache": vec}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=128, help="cells per axis of the 3D system")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--spmv-config", type=str, default=None,
                    help="lanes,block,blocks,schedule: a fixed SpMV configuration instead of the autotuner's")
    ap.add_argument("--no-latency", action="store_true",
                    help="skip the latency-bound 64 x 64 Poisson measurement and the latency floors")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-system batched measurement")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--batch-only", type=str, default=None,
                    choices=["persistent256", "persistent512", "persistent1024", "segmented", "segmented_sdia"],
                    help="only run the 256-system batch with this schedule (no headline solve, no per-solve loop; "
                         "for profiling) and print its figures as one JSON line")
    ap.add_argument("--batch-tile-rows", type=int, default=0,
                    help="rows per tile of the segmented batched schedules (0: the library's default)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner measurement")
    ap.add_argument("--learned-train", type=int, default=2000, help="training systems")
    ap.add_argument("--learned-eval", type=int, default=200, help="held-out systems")
    ap.add_argument("--learned-sides", type=int, nargs=2, default=[32, 96], help="side range of the learned workload")
    ap.add_argument("--learned-epochs", type=int, default=300)
    ap.add_argument("--learned-reps", type=int, default=1, help="timed solves per held-out system and solver")
    ap.add_argument("--workers", type=int, default=0, help="host threads drawing the systems (0: the host's CPUs, <= 16)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-batch (learned + batched) measurement")
    ap.add_argument("--mixed-count", type=int, default=1024, help="first systems of the 1024-system mixed batch to solve")
    ap.add_argument("--mixed-reps", type=int, default=1, help="timed runs of each mixed-batch path")
    ap.add_argument("--no-mixed-batched-jacobi", action="store_true",
                    help="skip the batched Jacobi-PCG run of the mixed batch")
    ap.add_argument("--cpu-reps", type=int, default=3, help="repetitions of the CPU baseline's solve (min taken)")
    ap.add_argument("--mixed-train", type=int, default=192, help="training systems for the mixed batch's network")
    ap.add_argument("--mixed-train-nmax", type=float, default=1e6, help="largest training system (rows)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--sweep", action="store_true",
                    help="only run the 20-iteration CG sweep over stencils and NNZ (prints one JSON line)")
    ap.add_argument("--sweep-nnz", type=float, nargs="+", default=[1e4, 1e5, 1e6, 1e7, 1e8])
    ap.add_argument("--sweep-stencils", type=int, nargs="+", default=[5, 9, 7, 27])
    ap.add_argument("--sweep-reps", type=int, default=5)
    ap.add_argument("--sweep-cpu-max-nnz", type=float, default=2e7)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2306_17801_amd as apcg
    from paper_2306_17801_amd import problems
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    apcg.load()

    if args.copy_calibration:
        copy_calibration(apcg, torch)
        return
    if args.batch_only:
        print(json.dumps({"batch2d_256": bench_batch(apcg, torch, args.batch_reps, only=args.batch_only,
                                                     tile_rows=args.batch_tile_rows)}), flush=True)
        return
    if args.sweep:
        res = bench_sweep(apcg, torch, args.sweep_nnz, args.sweep_reps, args.sweep_cpu_max_nnz, args.sweep_stencils)
        print(json.dumps({"sweep": res, "cpu_cores": 1, "timing": "min over repetitions, end to end"}), flush=True)
        return

    t0 = time.time()
    sysm = problems.diffusion3d_smoothed(args.n, seed=2)
    A_h = sysm.A
    n, nnz = A_h.n, A_h.nnz
    log(f"[bench] generated n={n} nnz={nnz} in {time.time() - t0:.1f}s")

    ctx = apcg.apcg_ctx_create(0)
    A = DeviceCSR(A_h)
    b = DeviceVec(sysm.b)
    x = DeviceVec.zeros(n)
    info = apcg.apcg_info_create(0, 1)
    rtol, maxit = 1e-8, 50000

    tuned = None
    if args.spmv_config:
        cfg = [int(v) for v in args.spmv_config.split(",")]
        apcg.apcg_mat_set_spmv_config(A.h, *cfg)
        tuned = {"config": apcg.apcg_mat_get_spmv_config(A.h), "fixed": True}
    elif not args.no_autotune:
        cfg, us = apcg.apcg_mat_autotune(A.h, ctx, 40)
        tuned = {"config": cfg, "product_us": round(us, 2)}
        log(f"[bench] autotune: {cfg} {us:.1f} us")

    opts = apcg.apcg_solve_opts_default(x0_is_zero=1)

    def solve(o=opts):
        apcg.apcg_ksp_solve(ctx, A.h, b.h, x.h, rtol, maxit, o, info, 0)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    res = apcg.apcg_info_get(info, 0)
    log(f"[bench] warm-up solve: {res}")

    apcg.apcg_counters_reset()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        solve()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    counters = apcg.apcg_counters_get()
    res = apcg.apcg_info_get(info, 0)
    its = res["iterations"]
    ms_per_step = 1000.0 * elapsed / args.steps
    value = args.steps / elapsed
    log(f"[bench] timed {args.steps} solves: {ms_per_step:.3f} ms/solve, its={its}, status={res['status']}")

    # true residual of the last solve (host check of the result, not timed)
    xs = x.numpy()
    true_rel = float(np.linalg.norm(sysm.b - A_h.to_scipy() @ xs) / np.linalg.norm(sysm.b))

    # per-kernel durations: each kernel launched back to back at the chosen
    # configuration, a HIP event pair on the context's stream around each
    # run (what the solve's graphs run: kernels queued one after another);
    # also a kernel-timed solve with an event pair around every launch,
    # which adds each launch's dispatch to its time
    reps_k = 400
    prod_us, upd_us = apcg.apcg_mat_time_kernels(A.h, ctx, reps_k)
    prod_cnt = reps_k
    topts = apcg.apcg_solve_opts_default(x0_is_zero=1, kernel_timing=1)
    solve(topts)
    prod_pair_us, _ = apcg.apcg_ctx_kernel_times(ctx, 0)
    upd_pair_us, _ = apcg.apcg_ctx_kernel_times(ctx, 1)
    cfg_now = apcg.apcg_mat_get_spmv_config(A.h)
    dia_sym = False
    if cfg_now["schedule"] == apcg.APCG_SPMV_DIA:
        # diagonals: 8 bytes per row per diagonal streamed (with symmetric
        # values only those on and right of the main one: the others are
        # read as their transposes); z, p_old read, p, w written
        offs = dia_offsets(A_h)
        dia_sym = apcg.apcg_mat_get_dia_info(A.h)["values_symmetric"] == 1
        streamed = sum(1 for o in offs if o >= 0) if dia_sym else len(offs)
        prod_bytes = 8 * streamed * n + 32 * n
    elif cfg_now["schedule"] == apcg.APCG_SPMV_SDIA:
        # sliced diagonals: 8 bytes per stored value slot (absent entries of a
        # slice's shared offsets included), 12 per offset/mask slot; z, p_old
        # read, p, w written
        u, mp = sdia_shape(A_h)
        nsl = (n + 63) // 64
        sym_reads = cfg_now["lanes_per_row"] > 1 and is_symmetric(A_h)
        if sym_reads:  # marching with symmetric values: the upper slots stream, plus the partner table
            prod_bytes = 8 * 64 * sdia_upper_slots(A_h) + 16 * nsl * mp + 32 * n
        else:
            prod_bytes = 8 * 64 * nsl * u + 12 * nsl * mp + 32 * n
    else:
        prod_bytes = 12 * nnz + 4 * (n + 1) + 32 * n  # A; z, p_old read; p, w written
    csr_bytes = 12 * nnz + 4 * (n + 1) + 32 * n
    upd_bytes = 64 * n  # x, r, p, w, dinv read; x, r, z written
    iter_bytes = prod_bytes + upd_bytes
    achieved = prod_bytes / (prod_us * 1e-6) / 1e9
    traffic = None
    traffic_note = "no counter file for this code and configuration"
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        cfg_chosen = apcg.apcg_mat_get_spmv_config(A.h)
        if tr.get("source_sha256_16") == source_hash(KERNEL_SOURCE) and tr.get("n") == n:
            for entry in tr.get("configs", []):  # one per SpMV configuration measured
                if entry.get("spmv_config") == cfg_chosen:
                    traffic = entry.get("bytes_per_launch")
                    traffic_note = (f"not measured in this run: {os.path.relpath(TRAFFIC_FILE, ROOT)}, rocprofv3 "
                                    f"--pmc FETCH_SIZE and WRITE_SIZE passes on the same kernel code (hash "
                                    f"{tr['source_sha256_16']}) and configuration, scaled by a 1 GiB copy "
                                    f"calibration (fetch x{tr.get('fetch_scale')}, write x{tr.get('write_scale')})")
    sym_reads = cfg_now["schedule"] == apcg.APCG_SPMV_SDIA and cfg_now["lanes_per_row"] > 1 and is_symmetric(A_h)
    marching = cfg_now["schedule"] in (apcg.APCG_SPMV_SDIA, apcg.APCG_SPMV_DIA) and cfg_now["lanes_per_row"] > 1
    kname = {apcg.APCG_SPMV_STREAM: "k_pcg_product_stream", apcg.APCG_SPMV_SELL: "k_pcg_product_sell",
             apcg.APCG_SPMV_DIA: "k_pcg_product_dia", apcg.APCG_SPMV_SDIA: "k_pcg_product_sdia"}.get(
        cfg_now["schedule"], "k_pcg_product") + ("_march" if marching else "") + (
        f" (block {cfg_now['block_size']}, {cfg_now['lanes_per_row']} planes per task"
        if marching else f" (block {cfg_now['block_size']}, {cfg_now['blocks']} workgroups") + (
        ", symmetric reads)" if (sym_reads or dia_sym) else ")")
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "traffic_source": traffic_note, "algorithmic_bytes_per_launch": prod_bytes,
                "csr_product_bytes_per_launch": csr_bytes,
                "mean_launch_us": round(prod_us, 3), "launches_timed": prod_cnt,
                "timing": "HIP events around back-to-back launches on the solve's stream",
                "event_pair_per_launch_us": round(prod_pair_us, 3)}
    per_iter_us = 1000.0 * ms_per_step / max(its, 1)
    extra = {
        "iterations": its, "status": res["status"], "true_relres": true_rel,
        "per_iteration_us": round(per_iter_us, 3),
        "iteration_gbs": round(iter_bytes / (per_iter_us * 1e-6) / 1e9, 1),
        "update_kernel": {"mean_launch_us": round(upd_us, 3), "event_pair_per_launch_us": round(upd_pair_us, 3),
                          "algorithmic_bytes_per_launch": upd_bytes,
                          "achieved_gbs": round(upd_bytes / (upd_us * 1e-6) / 1e9, 1)},
        "counters_timed_region": counters,
        "autotune": tuned,
    }
    log(f"[bench] product {prod_us:.2f} us ({achieved:.0f} GB/s), update {upd_us:.2f} us")

    if not args.no_variants:
        var = {}
        for name, mode in (("stream", apcg.APCG_MODE_STREAM), ("host_check", apcg.APCG_MODE_HOST_CHECK)):
            o = apcg.apcg_solve_opts_default(x0_is_zero=1, mode=mode)
            solve(o)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            reps = 2
            for _ in range(reps):
                solve(o)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t1) / reps
            var[name] = {"ms_per_solve": round(1000 * dt, 3), "solves_per_s": round(1 / dt, 3),
                         "iterations": apcg.apcg_info_get(info, 0)["iterations"]}
            log(f"[bench] variant {name}: {1000 * dt:.2f} ms/solve")
        var["graph_speedup_vs_host_check"] = round(var["host_check"]["ms_per_solve"] / ms_per_step, 3)
        extra["variants"] = var

    if not args.no_latency:
        extra["latency_poisson64"] = bench_latency(apcg, torch)

    if not args.no_batch:
        extra["batch2d_256"] = bench_batch(apcg, torch, args.batch_reps)

    workers = args.workers if args.workers > 0 else host_threads()
    if not args.no_learned:
        extra["learned_pc"] = bench_learned(apcg, torch, args.learned_train, args.learned_eval,
                                            args.learned_sides[0], args.learned_sides[1], args.learned_epochs,
                                            args.learned_reps, workers)

    if not args.no_mixed:
        extra["mixed_batch"] = bench_mixed(apcg, torch, args.mixed_count, args.mixed_train, args.mixed_train_nmax,
                                           args.learned_epochs, args.mixed_reps, workers,
                                           batched_jacobi=not args.no_mixed_batched_jacobi)
    # the metric's comparison in one place: batched + learned against the
    # plain path (one Jacobi-PCG solve per system) on the same GPU
    summ = {}
    if "mixed_batch" in extra:
        m = extra["mixed_batch"]
        summ["mixed_batch"] = {"systems": m["systems"], "batched_learned_solves_per_s": m["batched_learned_solves_per_s"],
                               "plain_per_solve_solves_per_s": m["per_solve_loop_solves_per_s"],
                               "speedup": m["batched_learned_speedup_vs_per_solve_loop"]}
    if "learned_pc" in extra:
        m = extra["learned_pc"]
        summ["learned_heldout"] = {"systems": m["eval_systems"], "learned_solves_per_s": m["learned_solves_per_s"],
                                   "plain_per_solve_solves_per_s": m["jacobi_solves_per_s"],
                                   "speedup": m["learned_speedup_vs_jacobi"]}
    if "batch2d_256" in extra:
        m = extra["batch2d_256"]
        summ["batch2d_256"] = {"systems": m["systems"], "batched_solves_per_s": m["batched_solves_per_s"],
                               "plain_per_solve_solves_per_s": m["per_solve_loop_solves_per_s"],
                               "speedup": m["batched_speedup_vs_per_solve_loop"]}
    if summ:
        extra["batched_learned_vs_plain"] = summ

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        threads = oracle.host_threads()
        log(f"[bench] timing the CPU oracle's Jacobi-PCG on {threads} host threads ...")
        times = []
        for _ in range(max(1, args.cpu_reps)):
            t1 = time.perf_counter()
            r = oracle.pcg_threads(A_h, sysm.b, rtol=rtol, maxit=maxit, threads=threads)
            times.append(time.perf_counter() - t1)
        dt = min(times)
        # the serial oracle (one thread, the parity configuration) on its
        # first 40 iterations, scaled to the full solve
        t1 = time.perf_counter()
        oracle.pcg(A_h, sysm.b, rtol=0.0, maxit=40)
        ser = (time.perf_counter() - t1) / 40 * r.its
        cpu = {"value": round(1.0 / dt, 5), "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": f"{len(times)} full FP64 Jacobi-PCG solves of the same system ({r.its} iterations each) "
                         f"with the oracle's loop spread over {threads} host threads (OpenMP over rows, static "
                         f"schedule); min {dt:.2f} s, median {sorted(times)[len(times) // 2]:.2f} s",
               "iterations": r.its, "min_s": round(dt, 3), "median_s": round(sorted(times)[len(times) // 2], 3),
               "serial_solves_per_s": round(1.0 / ser, 5),
               "serial_sample": "the serial oracle's first 40 iterations on one thread, scaled to the solve's "
                                f"{r.its} iterations"}
        log(f"[bench] oracle: min {dt:.2f} s on {threads} threads, its={r.its}; serial estimate {ser:.1f} s")
        if "batch2d_256" in extra:
            # the batch on the host: one serial oracle solve per system, the
            # systems spread over the host threads (largest first)
            from concurrent.futures import ThreadPoolExecutor

            from paper_2306_17801_amd import problems

            systems = sorted(problems.batch2d_lognormal(256, seed=3), key=lambda q: -q.A.n)
            t1 = time.perf_counter()
            with ThreadPoolExecutor(threads) as ex:
                res = list(ex.map(lambda q: oracle.pcg(q.A, q.b, rtol=1e-8, maxit=50000), systems))
            bdt = time.perf_counter() - t1
            extra["batch2d_256"]["cpu_baseline"] = {
                "value": round(len(systems) / bdt, 3), "unit": "solves/s", "cores": threads, "kind": "oracle",
                "sample": f"all {len(systems)} systems of the batch, one serial FP64 oracle Jacobi-PCG solve per "
                          f"system, the systems spread over {threads} host threads (largest first); one run",
                "seconds": round(bdt, 3), "converged": sum(1 for q in res if q.status == oracle.CONVERGED)}
            log(f"[bench] oracle batch: {bdt:.2f} s on {threads} threads")

    props = apcg.apcg_device_props_get(0)
    line = {
        "metric": METRIC, "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"diffusion3d_{args.n}^3_box3_jacobi_pcg", "n": n, "nnz": nnz, "rtol": rtol,
                   "pc": "jacobi", "x0": "zero", "mode": "graph", "iters_per_graph": 16, "lookahead": 2,
                   "device": props["name"], "arch": props["arch"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)
    apcg.apcg_info_destroy(info)
    apcg.apcg_ctx_synchronize(ctx)


if __name__ == "__main__":
    main()
